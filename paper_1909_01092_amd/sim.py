"""Simulation: a thin Python handle on the C ABI (include/lbm.h).

PyTorch supplies the device workspace (one uint8 tensor) and the HIP stream;
every step of the method runs in the library's HIP kernels.  The names follow
the C calls: step, particle_state, observables, populations, fields,
u_series, checkpoint / restore.
"""
import ctypes as C

import numpy as np

from . import _capi
from .workloads import entries, full


def _fill(p: _capi.LbmParams, q: dict):
    for name, ctype in _capi.LbmParams._fields_:
        v = q[name]
        if hasattr(ctype, "_length_"):
            setattr(p, name, ctype(*[float(x) for x in v]))
        elif ctype in (C.c_double,):
            setattr(p, name, float(v))
        else:
            setattr(p, name, int(v))


def make_params(replicas) -> C.Array:
    """ctypes array of lbm_params entries from one dict or a list of dicts
    (a dict's "spheres" become entries sharing its fluid)."""
    ents = entries(replicas)
    arr = (_capi.LbmParams * len(ents))()
    for k, q in enumerate(ents):
        _fill(arr[k], full(q))
    return arr


def workspace_bytes(replicas, precision="fp64") -> int:
    arr = make_params(replicas)
    n = C.c_size_t()
    _capi.check(_capi.lib().lbm_workspace_bytes(arr, len(arr), _capi.PRECISIONS[precision],
                                                C.byref(n)))
    return n.value


class Simulation:
    """One or more replicas advanced together on one GPU."""

    def __init__(self, replicas, precision: str = "fp64", device="cuda:0", stream=None,
                 fill=None):
        """fill: a byte value written over the whole workspace before
        lbm_init (0xff is a NaN in FP64, FP32 and FP16), so that a read of
        memory no kernel wrote shows up in the results."""
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("Simulation needs a ROCm GPU (torch.cuda.is_available() is False)")
        # one per lbm_init entry: a replica's extra spheres ("spheres") follow it
        self.replicas = entries(replicas)
        self.precision = precision
        self.device = torch.device(device)
        self._lib = _capi.lib()
        self._params = make_params(self.replicas)
        nbytes = workspace_bytes(self.replicas, precision)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        if fill is not None:
            self.workspace.fill_(int(fill))
            torch.cuda.synchronize(self.device)
        base = self.workspace.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        self._ws_bytes = nbytes
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        ctx = C.c_void_p()
        rc = self._lib.lbm_init(self._params, len(self._params), _capi.PRECISIONS[precision],
                                C.c_void_p(self._ws_ptr), nbytes, C.c_void_p(self.stream.cuda_stream),
                                C.byref(ctx))
        _capi.check(rc, None)
        self._ctx = ctx

    # -- lifetime
    def close(self):
        if getattr(self, "_ctx", None):
            self._lib.lbm_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        return _capi.check(rc, self._ctx)

    # -- stepping
    def step(self, n: int = 1):
        self._check(self._lib.lbm_step(self._ctx, int(n)))

    def step_noalloc(self, n: int = 1):
        """The same steps with the library's static step scratch instead of
        the workspace's (lbm_step_noalloc)."""
        self._check(self._lib.lbm_step_noalloc(self._ctx, int(n)))

    def sync(self):
        self._check(self._lib.lbm_sync(self._ctx))

    def set_launch(self, block: int = 256, zchunk: int = 0):
        """Main-kernel launch shape; zchunk 0 picks the default chunk."""
        self._check(self._lib.lbm_set_launch(self._ctx, int(block), int(zchunk)))

    def autotune(self, steps_per_trial: int = 10, preserve: bool = True):
        """Time every admissible (block, z-chunk) of the main kernel and keep the
        fastest (lbm_autotune).  preserve=True checkpoints and restores the
        state so the run is left where it was.  Returns (block, zchunk, ms)."""
        import torch
        buf = None
        if preserve:
            n = C.c_size_t()
            self._check(self._lib.lbm_checkpoint_bytes(self._ctx, C.byref(n)))
            buf = torch.empty(n.value, dtype=torch.uint8, device=self.device)
        b, z, ms = C.c_int32(), C.c_int32(), C.c_double()
        self._check(self._lib.lbm_autotune(self._ctx, int(steps_per_trial),
                                           C.c_void_p(buf.data_ptr()) if buf is not None else None,
                                           C.byref(b), C.byref(z), C.byref(ms)))
        return b.value, z.value, ms.value

    def get_launch(self):
        b, z = C.c_int32(), C.c_int32()
        self._check(self._lib.lbm_get_launch(self._ctx, C.byref(b), C.byref(z)))
        return b.value, z.value

    def set_graph(self, steps_per_graph: int):
        self._check(self._lib.lbm_set_graph(self._ctx, int(steps_per_graph)))

    def timing(self, every):
        """Main-kernel timing: False / 0 off, True / 1 every plain step, k:
        every k-th plain step (lbm_timing)."""
        self._check(self._lib.lbm_timing(self._ctx, int(every)))

    def timing_read(self):
        ms, n = C.c_double(), C.c_int64()
        self._check(self._lib.lbm_timing_read(self._ctx, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def step_bytes(self) -> float:
        b = C.c_double()
        self._check(self._lib.lbm_step_bytes(self._ctx, C.byref(b)))
        return b.value

    # -- queries
    def particle_state(self, replica: int = 0, allow_unstable: bool = False) -> dict:
        """State of entry `replica`'s sphere.  allow_unstable: return it even
        when the sticky flags are set ("unstable", "contact" say which)."""
        P = _capi.LbmParticle()
        rc = self._lib.lbm_particle_state(self._ctx, int(replica), C.byref(P))
        if not (allow_unstable and rc in (_capi.LBM_EUNSTABLE, _capi.LBM_ECONTACT)):
            self._check(rc)
        out = {}
        for name, ctype in _capi.LbmParticle._fields_:
            v = getattr(P, name)
            out[name] = np.array(list(v)) if hasattr(ctype, "_length_") else v
        out["unstable"] = rc == _capi.LBM_EUNSTABLE
        out["contact"] = rc == _capi.LBM_ECONTACT
        return out

    def _dims(self, r):
        q = self.replicas[r]
        return q["nx"], q["ny"], q["nz"]

    def populations(self, replica: int = 0) -> np.ndarray:
        nx, ny, nz = self._dims(replica)
        f = np.empty((2, 19, nz, ny, nx), dtype=np.float64)
        self._check(self._lib.lbm_populations(self._ctx, int(replica),
                                              f.ctypes.data_as(C.POINTER(C.c_double))))
        return f

    def fields(self, replica: int = 0):
        nx, ny, nz = self._dims(replica)
        rho = np.empty((2, nz, ny, nx))
        u = np.empty((3, nz, ny, nx))
        self._check(self._lib.lbm_fields(self._ctx, int(replica),
                                         rho.ctypes.data_as(C.POINTER(C.c_double)),
                                         u.ctypes.data_as(C.POINTER(C.c_double))))
        return rho, u

    def observables(self, replica: int = 0, profile: bool = False) -> dict:
        nx, ny, nz = self._dims(replica)
        o = _capi.LbmObs()
        prof = np.zeros((ny, nx)) if profile else None
        o.uz_profile = prof.ctypes.data_as(C.POINTER(C.c_double)) if profile else None
        self._check(self._lib.lbm_observables(self._ctx, int(replica), C.byref(o)))
        out = dict(mass=np.array(list(o.mass)), momentum=np.array(list(o.momentum)),
                   u2_mean=o.u2_mean, uz_mean=o.uz_mean, n_fluid=o.n_fluid)
        if profile:
            out["uz_profile"] = prof
        return out

    def u_series(self, replica: int = 0) -> np.ndarray:
        cap = int(self.replicas[replica]["series_cap"])
        buf = np.empty((cap, 3))
        n = C.c_int64()
        self._check(self._lib.lbm_u_series(self._ctx, int(replica),
                                           buf.ctypes.data_as(C.POINTER(C.c_double)), cap,
                                           C.byref(n)))
        return buf[: n.value].copy()

    # -- adjoint form
    def adjoint(self, nsteps: int, segment: int = 0):
        """Advance nsteps (as step() would) and return (J, grad): J = mean of
        U_z^{n+1/2} over those steps, grad = dJ/d(g_x, g_y, g_z, G, Delta rho)
        (lbm_adjoint; segment = checkpoint interval, 0 = 50 steps)."""
        import torch
        n = C.c_size_t()
        self._check(self._lib.lbm_adjoint_bytes(self._ctx, int(nsteps), int(segment), C.byref(n)))
        buf = torch.empty(n.value + 256, dtype=torch.uint8, device=self.device)
        ptr = (buf.data_ptr() + 255) // 256 * 256
        grad = np.empty(5)
        J = C.c_double()
        self._check(self._lib.lbm_adjoint(self._ctx, int(nsteps), int(segment), C.c_void_p(ptr), n.value,
                                          grad.ctypes.data_as(C.POINTER(C.c_double)), C.byref(J)))
        return J.value, grad

    def adjoint_forward(self, nsteps: int, segment: int = 0) -> float:
        """Forward sweep of the adjoint form alone (lbm_adjoint_forward):
        advance nsteps with checkpoints and return J; the tape stays in a
        buffer this object holds until adjoint_backward."""
        import torch
        n = C.c_size_t()
        self._check(self._lib.lbm_adjoint_bytes(self._ctx, int(nsteps), int(segment), C.byref(n)))
        self._tape = torch.empty(n.value + 256, dtype=torch.uint8, device=self.device)
        ptr = (self._tape.data_ptr() + 255) // 256 * 256
        J = C.c_double()
        self._check(self._lib.lbm_adjoint_forward(self._ctx, int(nsteps), int(segment), C.c_void_p(ptr),
                                                  n.value, C.byref(J)))
        return J.value

    def adjoint_backward(self) -> np.ndarray:
        """Reverse sweep over the tape of the last adjoint_forward
        (lbm_adjoint_backward): dJ/d(g_x, g_y, g_z, G, Delta rho)."""
        grad = np.empty(5)
        try:
            self._check(self._lib.lbm_adjoint_backward(self._ctx, grad.ctypes.data_as(C.POINTER(C.c_double))))
        finally:
            self._tape = None
        return grad

    # -- checkpoints (device tensors)
    def checkpoint(self):
        import torch
        n = C.c_size_t()
        self._check(self._lib.lbm_checkpoint_bytes(self._ctx, C.byref(n)))
        t = torch.empty(n.value, dtype=torch.uint8, device=self.device)
        self._check(self._lib.lbm_checkpoint(self._ctx, C.c_void_p(t.data_ptr())))
        return t

    def restore(self, t):
        self._check(self._lib.lbm_restore(self._ctx, C.c_void_p(t.data_ptr())))
