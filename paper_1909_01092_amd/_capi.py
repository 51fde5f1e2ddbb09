"""ctypes declarations of the C ABI in include/lbm.h (argument marshalling only).

Every step of the method runs in the HIP kernels of liblbm.so; this module
only loads the library and describes its structs and signatures.  It fails
loudly when the library has not been built.
"""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm.so")

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EDEVICE, LBM_EUNSTABLE, LBM_ESTATE, LBM_ECONTACT = \
    0, -1, -2, -3, -4, -5, -6
PRECISIONS = {"fp64": 0, "fp32": 1, "fp16": 2}


class LbmParams(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("walls", C.c_uint32),
        ("rho0", C.c_double * 2), ("init_amp", C.c_double), ("G", C.c_double),
        ("tau_shear", C.c_double), ("tau_bulk", C.c_double), ("tau_mom", C.c_double),
        ("tau_ghost", C.c_double), ("kT", C.c_double), ("seed", C.c_uint64),
        ("replica", C.c_int32), ("g", C.c_double * 3), ("force_mode", C.c_int32),
        ("radius", C.c_double), ("rho_p", C.c_double), ("wet_drho", C.c_double),
        ("X0", C.c_double * 3), ("U0", C.c_double * 3), ("W0", C.c_double * 3),
        ("noise_diffusive", C.c_int32), ("fixed_velocity", C.c_int32),
        ("series_cap", C.c_int32), ("init_split", C.c_int32), ("shared_fluid", C.c_int32),
    ]


class LbmParticle(C.Structure):
    _fields_ = [
        ("X", C.c_double * 3), ("U", C.c_double * 3), ("W", C.c_double * 3),
        ("F", C.c_double * 3), ("T", C.c_double * 3), ("Pev", C.c_double * 3),
        ("Lev", C.c_double * 3), ("delta", C.c_double * 2), ("n_fluid", C.c_double),
        ("step", C.c_int64), ("n_covered", C.c_int64), ("n_uncovered", C.c_int64),
        ("n_links", C.c_int64),
    ]


class LbmObs(C.Structure):
    _fields_ = [
        ("mass", C.c_double * 2), ("momentum", C.c_double * 3), ("u2_mean", C.c_double),
        ("uz_mean", C.c_double), ("n_fluid", C.c_double), ("uz_profile", C.POINTER(C.c_double)),
    ]


# name -> (restype, argtypes); the exported set equals the header's declarations
_D = C.POINTER(C.c_double)
_V = C.c_void_p
SIGNATURES = {
    "lbm_workspace_bytes": (C.c_int, [C.POINTER(LbmParams), C.c_int32, C.c_int32, C.POINTER(C.c_size_t)]),
    "lbm_init": (C.c_int, [C.POINTER(LbmParams), C.c_int32, C.c_int32, _V, C.c_size_t, _V,
                           C.POINTER(_V)]),
    "lbm_step": (C.c_int, [_V, C.c_int32]),
    "lbm_step_noalloc": (C.c_int, [_V, C.c_int32]),
    "lbm_sync": (C.c_int, [_V]),
    "lbm_autotune": (C.c_int, [_V, C.c_int32, _V, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                               C.POINTER(C.c_double)]),
    "lbm_particle_state": (C.c_int, [_V, C.c_int32, C.POINTER(LbmParticle)]),
    "lbm_observables": (C.c_int, [_V, C.c_int32, C.POINTER(LbmObs)]),
    "lbm_populations": (C.c_int, [_V, C.c_int32, _D]),
    "lbm_fields": (C.c_int, [_V, C.c_int32, _D, _D]),
    "lbm_u_series": (C.c_int, [_V, C.c_int32, _D, C.c_int64, C.POINTER(C.c_int64)]),
    "lbm_checkpoint_bytes": (C.c_int, [_V, C.POINTER(C.c_size_t)]),
    "lbm_checkpoint": (C.c_int, [_V, _V]),
    "lbm_restore": (C.c_int, [_V, _V]),
    "lbm_set_launch": (C.c_int, [_V, C.c_int32, C.c_int32]),
    "lbm_get_launch": (C.c_int, [_V, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "lbm_set_graph": (C.c_int, [_V, C.c_int32]),
    "lbm_timing": (C.c_int, [_V, C.c_int32]),
    "lbm_timing_read": (C.c_int, [_V, _D, C.POINTER(C.c_int64)]),
    "lbm_step_bytes": (C.c_int, [_V, _D]),
    "lbm_adjoint_bytes": (C.c_int, [_V, C.c_int32, C.c_int32, C.POINTER(C.c_size_t)]),
    "lbm_adjoint": (C.c_int, [_V, C.c_int32, C.c_int32, _V, C.c_size_t, _D, _D]),
    "lbm_adjoint_forward": (C.c_int, [_V, C.c_int32, C.c_int32, _V, C.c_size_t, _D]),
    "lbm_adjoint_backward": (C.c_int, [_V, _D]),
    "lbm_destroy": (None, [_V]),
    "lbm_last_error": (C.c_char_p, [_V]),
}

_lib = None


class LbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"lbm error {code}: {msg}")
        self.code = code


def lib():
    """The loaded HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library {LIB_PATH} is missing: build it with "
                               "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(rc, ctx=None):
    if rc != LBM_OK:
        msg = lib().lbm_last_error(ctx)
        raise LbmError(rc, msg.decode() if msg else "")
    return rc
