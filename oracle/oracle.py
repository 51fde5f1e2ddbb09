"""ctypes wrapper of the FP64 CPU oracle (test infrastructure only).

Only tests/, the smoke check in __graft_entry__ and the CPU-baseline leg of
bench.py import this module.  It imports nothing from the HIP package: it is
driven by a plain dict of run parameters.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm_oracle.so")
Q = 19


MAX_EXTRA = 7


class OrcSphere(C.Structure):
    _fields_ = [("radius", C.c_double), ("rho_p", C.c_double), ("wet_drho", C.c_double),
                ("X0", C.c_double * 3), ("U0", C.c_double * 3), ("W0", C.c_double * 3)]


class OrcParams(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("walls", C.c_uint32),
        ("rho0", C.c_double * 2), ("init_amp", C.c_double), ("G", C.c_double),
        ("tau_shear", C.c_double), ("tau_bulk", C.c_double), ("tau_mom", C.c_double),
        ("tau_ghost", C.c_double), ("kT", C.c_double), ("seed", C.c_uint64),
        ("replica", C.c_int32), ("g", C.c_double * 3), ("force_mode", C.c_int32),
        ("radius", C.c_double), ("rho_p", C.c_double), ("wet_drho", C.c_double),
        ("X0", C.c_double * 3), ("U0", C.c_double * 3), ("W0", C.c_double * 3),
        ("noise_diffusive", C.c_int32), ("fixed_velocity", C.c_int32),
        ("init_split", C.c_int32), ("n_extra", C.c_int32), ("extra", OrcSphere * MAX_EXTRA),
    ]


class OrcParticle(C.Structure):
    _fields_ = [
        ("X", C.c_double * 3), ("U", C.c_double * 3), ("W", C.c_double * 3),
        ("F", C.c_double * 3), ("T", C.c_double * 3), ("Pev", C.c_double * 3),
        ("Lev", C.c_double * 3), ("delta", C.c_double * 2), ("n_fluid", C.c_double),
        ("step", C.c_int64), ("n_covered", C.c_int64), ("n_uncovered", C.c_int64),
        ("n_links", C.c_int64),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from .build import build
            build()
        _lib = C.CDLL(LIB_PATH)
        d = C.POINTER(C.c_double)
        _lib.orc_create.restype = C.c_void_p
        _lib.orc_create.argtypes = [C.POINTER(OrcParams)]
        _lib.orc_destroy.argtypes = [C.c_void_p]
        _lib.orc_step.argtypes = [C.c_void_p, C.c_int32]
        _lib.orc_get_populations.argtypes = [C.c_void_p, d]
        _lib.orc_set_populations.argtypes = [C.c_void_p, d]
        _lib.orc_get_particle.argtypes = [C.c_void_p, C.POINTER(OrcParticle)]
        _lib.orc_set_particle.argtypes = [C.c_void_p, C.POINTER(OrcParticle)]
        _lib.orc_get_fields.argtypes = [C.c_void_p, d, d]
        _lib.orc_observables.argtypes = [C.c_void_p, d, d]
        _lib.orc_u_series.restype = C.c_int64
        _lib.orc_u_series.argtypes = [C.c_void_p, d, C.c_int64]
        _lib.orc_philox4x32_10.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32),
                                           C.POINTER(C.c_uint32)]
        _lib.orc_normals.argtypes = [C.c_void_p, C.c_int64, C.c_int64, d]
        _lib.orc_basis.argtypes = [d, d, d, C.POINTER(C.c_int32)]
        _lib.orc_collide_node.argtypes = [C.c_void_p, d, d, d, d]
        _lib.orc_forces.argtypes = [C.c_void_p, d]
        _lib.orc_adjoint.restype = C.c_int
        _lib.orc_adjoint.argtypes = [C.c_void_p, C.c_int32, d, d]
        _lib.orc_set_threads.restype = C.c_int
        _lib.orc_set_threads.argtypes = [C.c_int32]
        _lib.orc_n_spheres.restype = C.c_int32
        _lib.orc_n_spheres.argtypes = [C.c_void_p]
        _lib.orc_get_sphere.argtypes = [C.c_void_p, C.c_int32, C.POINTER(OrcParticle)]
        _lib.orc_set_sphere.argtypes = [C.c_void_p, C.c_int32, C.POINTER(OrcParticle)]
        _lib.orc_u_series_sphere.restype = C.c_int64
        _lib.orc_u_series_sphere.argtypes = [C.c_void_p, C.c_int32, d, C.c_int64]
    return _lib


def set_threads(n: int = 0) -> int:
    """Threads of the oracle's per-node loops (n <= 0: leave as is); returns
    the count in effect.  Results are bitwise independent of it."""
    return int(lib().orc_set_threads(int(n)))


DEFAULTS = dict(nx=8, ny=8, nz=8, walls=0, rho0=(0.95, 0.05), init_amp=0.0, G=0.0,
                tau_shear=1.0, tau_bulk=1.0, tau_mom=1.0, tau_ghost=1.0, kT=0.0, seed=0,
                replica=0, g=(0.0, 0.0, 0.0), force_mode=0, radius=0.0, rho_p=2.0,
                wet_drho=0.0, X0=None, U0=(0.0, 0.0, 0.0), W0=(0.0, 0.0, 0.0),
                noise_diffusive=1, fixed_velocity=0, init_split=0)


def make_params(d: dict) -> OrcParams:
    """Run parameters; d["spheres"] (optional) lists further spheres as dicts
    with radius, rho_p, wet_drho, X0, U0, W0."""
    q = dict(DEFAULTS)
    q.update(d)
    if q["X0"] is None:
        q["X0"] = ((q["nx"] - 1) / 2.0, (q["ny"] - 1) / 2.0, (q["nz"] - 1) / 2.0)
    p = OrcParams()
    extra = list(q.get("spheres", []))
    if len(extra) > MAX_EXTRA:
        raise ValueError(f"at most {MAX_EXTRA} further spheres")
    p.n_extra = len(extra)
    for k, e in enumerate(extra):
        sp = p.extra[k]
        sp.radius, sp.rho_p, sp.wet_drho = float(e["radius"]), float(e.get("rho_p", q["rho_p"])), \
            float(e.get("wet_drho", 0.0))
        for name in ("X0", "U0", "W0"):
            setattr(sp, name, (C.c_double * 3)(*[float(x) for x in e.get(name, (0.0, 0.0, 0.0))]))
    for name, ctype in OrcParams._fields_:
        if name in ("n_extra", "extra"):
            continue
        v = q[name]
        if hasattr(ctype, "_length_"):
            setattr(p, name, ctype(*[float(x) for x in v]))
        else:
            setattr(p, name, v)
    return p


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class OracleSim:
    """One replica of the method advanced by the FP64 CPU oracle."""

    def __init__(self, params: dict):
        self.params = dict(params)
        self._p = make_params(params)
        self.nx, self.ny, self.nz = self._p.nx, self._p.ny, self._p.nz
        self.N = self.nx * self.ny * self.nz
        self._h = lib().orc_create(C.byref(self._p))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_destroy(h)
            self._h = None

    def step(self, n: int = 1):
        lib().orc_step(self._h, int(n))

    def populations(self) -> np.ndarray:
        f = np.empty((2, Q, self.nz, self.ny, self.nx), dtype=np.float64)
        lib().orc_get_populations(self._h, _dp(f))
        return f

    def set_populations(self, f: np.ndarray):
        f = np.ascontiguousarray(f, dtype=np.float64)
        lib().orc_set_populations(self._h, _dp(f))

    def particle(self) -> dict:
        P = OrcParticle()
        lib().orc_get_particle(self._h, C.byref(P))
        out = {}
        for name, ctype in OrcParticle._fields_:
            v = getattr(P, name)
            out[name] = np.array(list(v)) if hasattr(ctype, "_length_") else v
        return out

    def set_particle(self, d: dict):
        P = OrcParticle()
        lib().orc_get_particle(self._h, C.byref(P))
        for k, v in d.items():
            cur = getattr(P, k)
            if hasattr(cur, "_length_"):
                for i, x in enumerate(v):
                    cur[i] = float(x)
            else:
                setattr(P, k, v)
        lib().orc_set_particle(self._h, C.byref(P))

    def n_spheres(self) -> int:
        return int(lib().orc_n_spheres(self._h))

    def sphere(self, k: int) -> dict:
        """State of sphere k (0: the first; the global fields are shared)."""
        P = OrcParticle()
        lib().orc_get_sphere(self._h, int(k), C.byref(P))
        out = {}
        for name, ctype in OrcParticle._fields_:
            v = getattr(P, name)
            out[name] = np.array(list(v)) if hasattr(ctype, "_length_") else v
        return out

    def set_sphere(self, k: int, d: dict):
        P = OrcParticle()
        lib().orc_get_sphere(self._h, int(k), C.byref(P))
        for key, v in d.items():
            cur = getattr(P, key)
            if hasattr(cur, "_length_"):
                for i, x in enumerate(v):
                    cur[i] = float(x)
            else:
                setattr(P, key, v)
        lib().orc_set_sphere(self._h, int(k), C.byref(P))

    def sphere_u_series(self, k: int) -> np.ndarray:
        n = self.particle()["step"]
        out = np.empty((max(int(n), 1), 3))
        m = lib().orc_u_series_sphere(self._h, int(k), _dp(out), out.shape[0])
        return out[:m]

    def fields(self):
        rho = np.empty((2, self.nz, self.ny, self.nx))
        u = np.empty((3, self.nz, self.ny, self.nx))
        lib().orc_get_fields(self._h, _dp(rho), _dp(u))
        return rho, u

    def forces(self) -> np.ndarray:
        F = np.empty((2, 3, self.nz, self.ny, self.nx))
        lib().orc_forces(self._h, _dp(F))
        return F

    def observables(self):
        m = np.empty(2)
        j = np.empty(3)
        lib().orc_observables(self._h, _dp(m), _dp(j))
        return m, j

    def u_series(self) -> np.ndarray:
        n = self.particle()["step"]
        out = np.empty((max(int(n), 1), 3))
        k = lib().orc_u_series(self._h, _dp(out), out.shape[0])
        return out[:k]

    def adjoint(self, nsteps: int):
        """Advance nsteps and return (J, grad): J = mean of U_z^{n+1/2} over
        those steps, grad = dJ/d(g_x, g_y, g_z, G, Delta rho)."""
        grad = np.empty(5)
        J = np.empty(1)
        rc = lib().orc_adjoint(self._h, int(nsteps), _dp(grad), _dp(J))
        if rc != 0:
            raise ValueError(f"oracle adjoint: unsupported configuration or no memory ({rc})")
        return float(J[0]), grad

    def normals(self, node: int, step: int) -> np.ndarray:
        z = np.empty(36)
        lib().orc_normals(self._h, int(node), int(step), _dp(z))
        return z

    def collide_node(self, fin, F, noise):
        fin = np.ascontiguousarray(fin, dtype=np.float64)
        F = np.ascontiguousarray(F, dtype=np.float64)
        noise = np.ascontiguousarray(noise, dtype=np.float64)
        out = np.empty((2, Q))
        lib().orc_collide_node(self._h, _dp(fin), _dp(F), _dp(noise), _dp(out))
        return out


def philox(ctr, key):
    c = (C.c_uint32 * 4)(*[int(x) & 0xffffffff for x in ctr])
    k = (C.c_uint32 * 2)(*[int(x) & 0xffffffff for x in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return [int(x) for x in o]


def basis():
    e = np.empty((Q, Q))
    w = np.empty(Q)
    b = np.empty(Q)
    c = (C.c_int32 * (Q * 3))()
    lib().orc_basis(_dp(e), _dp(w), _dp(b), c)
    return e, w, b, np.array(list(c), dtype=np.int64).reshape(Q, 3)
