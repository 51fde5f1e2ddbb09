"""Property test of the C ABI's parameter validation, without a GPU:
lbm_workspace_bytes on random parameter sets (sizes from degenerate to huge,
non-finite and out-of-range values, random several-sphere groupings and
precision codes) returns LBM_OK with a positive size or LBM_EINVAL with a
message, never anything else, and accepts only sets that satisfy the
documented requirements (include/lbm.h)."""
import ctypes as C
import math
import os

import pytest
from hypothesis import HealthCheck, given, settings, strategies as st

from paper_1909_01092_amd import _capi, workloads

pytestmark = pytest.mark.filterwarnings("ignore")

FLOATS = st.one_of(st.floats(allow_nan=True, allow_infinity=True, width=64),
                   st.floats(min_value=-2.0, max_value=2.0), st.sampled_from([0.0, 0.5, 1.0, 1e-5, 0.95, 0.05]))
SIZES = st.one_of(st.integers(min_value=-3, max_value=40), st.integers(min_value=200, max_value=300),
                  st.sampled_from([2, 3, 1 << 20, (1 << 31) - 1]))


@st.composite
def entry(draw):
    q = dict(workloads.channel(16, 24, kT=1e-5, radius=3.0, seed=1))
    for name in draw(st.lists(st.sampled_from(
            ["nx", "ny", "nz", "walls", "rho0", "init_amp", "G", "tau_shear", "tau_bulk", "tau_mom",
             "tau_ghost", "kT", "g", "force_mode", "radius", "rho_p", "wet_drho", "X0", "U0", "W0",
             "series_cap", "init_split", "shared_fluid"]), max_size=4)):
        if name in ("nx", "ny", "nz", "series_cap", "init_split"):
            q[name] = draw(SIZES)
        elif name == "walls":
            q[name] = draw(st.integers(min_value=0, max_value=12))
        elif name in ("force_mode", "shared_fluid"):
            q[name] = draw(st.integers(min_value=-1, max_value=2))
        elif name in ("rho0",):
            q[name] = (draw(FLOATS), draw(FLOATS))
        elif name in ("g", "X0", "U0", "W0"):
            q[name] = (draw(FLOATS), draw(FLOATS), draw(FLOATS))
        else:
            q[name] = draw(FLOATS)
    return q


def _arr(entries):
    arr = (_capi.LbmParams * len(entries))()
    for k, q in enumerate(entries):
        p = arr[k]
        for name, ctype in _capi.LbmParams._fields_:
            v = q[name]
            if hasattr(ctype, "_length_"):
                setattr(p, name, ctype(*[float(x) for x in v]))
            elif ctype is C.c_double:
                setattr(p, name, float(v))
            elif ctype is C.c_uint32 or ctype is C.c_uint64:
                setattr(p, name, int(v) & (0xFFFFFFFF if ctype is C.c_uint32 else 0xFFFFFFFFFFFFFFFF))
            else:
                setattr(p, name, max(min(int(v), 2**31 - 1), -2**31))
    return arr


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_capi.LIB_PATH):
        from paper_1909_01092_amd import build
        build.build()
    return _capi.lib()


@settings(max_examples=400, deadline=None, suppress_health_check=[HealthCheck.function_scoped_fixture])
@given(entries=st.lists(entry(), min_size=1, max_size=4), prec=st.sampled_from([0, 1, 2, 0, 1, 2, -1, 3]))
def test_workspace_bytes_accepts_or_rejects_cleanly(lib, entries, prec):
    arr = _arr([workloads.full(q) for q in entries])
    nbytes = C.c_size_t(0)
    rc = lib.lbm_workspace_bytes(arr, len(arr), prec, C.byref(nbytes))
    assert rc in (_capi.LBM_OK, _capi.LBM_EINVAL), rc
    if rc == _capi.LBM_EINVAL:
        msg = lib.lbm_last_error(None)
        assert msg and len(msg) > 0
        return
    assert nbytes.value > 0
    # what was accepted meets the documented requirements
    assert prec in (0, 1, 2)
    assert arr[0].shared_fluid == 0
    for p in arr:
        assert p.shared_fluid in (0, 1)
        for v in (*p.X0, *p.U0, *p.W0):
            assert math.isfinite(v)
        if p.radius > 0:
            assert p.rho_p > 0 and all(abs(u) < 0.5 for u in p.U0)
        if p.shared_fluid:
            # its fluid fields are not read: the fluid is its group's first entry's
            assert p.radius > 0
            continue
        assert 2 <= p.nx <= 256 and p.ny >= 2 and p.nz >= 2
        assert p.walls <= 7
        assert p.rho0[0] > 0 and p.rho0[1] > 0
        for t in (p.tau_shear, p.tau_bulk, p.tau_mom, p.tau_ghost):
            assert t > 0.5 and math.isfinite(t)
        assert p.kT >= 0 and math.isfinite(p.kT) and math.isfinite(p.G)
        assert p.force_mode in (0, 1) and p.series_cap >= 1 and 0 <= p.init_split < p.nz
        for v in p.g:
            assert math.isfinite(v)
