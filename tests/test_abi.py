"""C ABI of the HIP library, checked without a GPU: the library loads, exports
exactly the entry points include/lbm.h declares, and rejects invalid
configurations before any device work."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm.h")


@pytest.fixture(scope="module")
def capi():
    from paper_1909_01092_amd import _capi
    if not os.path.exists(_capi.LIB_PATH):
        from paper_1909_01092_amd import build
        build.build()
    return _capi


def header_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_0-9]+)\s*\(", txt)))


def test_exports_match_header(capi):
    out = subprocess.run(["nm", "-D", "--defined-only", capi.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = sorted(l.split()[-1] for l in out.splitlines() if " T " in l)
    assert exported == header_functions()
    assert sorted(capi.SIGNATURES) == header_functions()
    capi.lib()  # every symbol resolves with its declared signature


def test_struct_sizes_match_header(capi, tmp_path):
    src = tmp_path / "sz.c"
    src.write_text('#include "lbm.h"\n#include <stdio.h>\nint main(void){printf("%zu %zu %zu\\n",'
                   ' sizeof(lbm_params), sizeof(lbm_particle), sizeof(lbm_obs));return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I" + os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    sizes = list(map(int, subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()))
    assert sizes == [C.sizeof(capi.LbmParams), C.sizeof(capi.LbmParticle), C.sizeof(capi.LbmObs)]


def _bytes(capi, params, prec="fp32"):
    from paper_1909_01092_amd.sim import workspace_bytes
    return workspace_bytes(params, prec)


def test_workspace_sizes(capi):
    from paper_1909_01092_amd import workloads as w
    one = _bytes(capi, w.SINGLE_RUN, "fp32")
    assert one >= 2 * 38 * 64 * 64 * 256 * 4
    assert _bytes(capi, w.SINGLE_RUN, "fp16") < one < _bytes(capi, w.SINGLE_RUN, "fp64")
    two = _bytes(capi, [w.SINGLE_RUN, w.SINGLE_RUN], "fp32")
    assert two >= 2 * 38 * 2 * 64 * 64 * 256 * 4


@pytest.mark.parametrize("bad", [
    dict(nx=1), dict(nx=300), dict(tau_shear=0.5), dict(kT=-1.0), dict(rho0=(1.0, 0.0)),
    dict(force_mode=3), dict(series_cap=0), dict(walls=9), dict(init_amp=0.2),
    dict(nx=16, ny=16, nz=16, walls=3, radius=7.5),           # sphere touches a wall
    dict(nx=12, ny=12, nz=12, radius=3.5),                    # periodic box too short for the bbox
    dict(nx=16, ny=16, nz=32, walls=3, radius=3.0, U0=(0.0, 0.0, 0.6)),
    dict(init_split=-1), dict(init_split=16),                 # split plane outside the lattice
])
def test_invalid_parameters_rejected(capi, bad):
    from paper_1909_01092_amd.sim import workspace_bytes
    q = dict(nx=16, ny=16, nz=16)
    q.update(bad)
    with pytest.raises(capi.LbmError) as e:
        workspace_bytes(q, "fp32")
    assert e.value.code == capi.LBM_EINVAL


def test_init_rejects_bad_workspace_before_device_work(capi):
    from paper_1909_01092_amd.sim import make_params, workspace_bytes
    q = dict(nx=16, ny=16, nz=16)
    arr = make_params(q)
    need = workspace_bytes(q, "fp32")
    ctx = C.c_void_p()
    L = capi.lib()
    assert L.lbm_init(arr, 1, 1, C.c_void_p(4096 + 8), need, None, C.byref(ctx)) == capi.LBM_ENOMEM
    assert b"aligned" in L.lbm_last_error(None)
    assert L.lbm_init(arr, 1, 1, C.c_void_p(4096), need - 1, None, C.byref(ctx)) == capi.LBM_ENOMEM
    assert L.lbm_init(arr, 1, 7, C.c_void_p(4096), need, None, C.byref(ctx)) == capi.LBM_EINVAL
    assert not ctx.value


def test_lattice_size_limit_depends_on_precision(capi):
    """Byte offsets within one component block are 32-bit: a lattice of about
    36M padded nodes fits FP32 and FP16 storage but not FP64."""
    from paper_1909_01092_amd.sim import workspace_bytes
    q = dict(nx=190, ny=190, nz=1000, walls=3)
    assert workspace_bytes(q, "fp32") > 0
    assert workspace_bytes(q, "fp16") > 0
    with pytest.raises(capi.LbmError) as e:
        workspace_bytes(q, "fp64")
    assert e.value.code == capi.LBM_EINVAL and b"too large" in str(e.value).encode()
    with pytest.raises(capi.LbmError):
        workspace_bytes(dict(nx=200, ny=200, nz=1500, walls=3), "fp32")


def test_empty_replica_list_rejected(capi):
    from paper_1909_01092_amd.sim import make_params
    arr = make_params(dict(nx=16, ny=16, nz=16))
    n = C.c_size_t()
    L = capi.lib()
    assert L.lbm_workspace_bytes(arr, 0, 1, C.byref(n)) == capi.LBM_EINVAL
    assert L.lbm_workspace_bytes(arr, -3, 1, C.byref(n)) == capi.LBM_EINVAL
    assert b"n_replicas" in L.lbm_last_error(None)


def _group(**kw):
    q = dict(nx=16, ny=16, nz=48, walls=3, radius=2.5, X0=(7.5, 7.5, 8.0),
             spheres=[dict(radius=2.5, X0=(7.5, 7.5, 30.0))])
    q.update(kw)
    return q


def test_sphere_group_workspace(capi):
    """A second sphere in the same fluid adds its box, partials and U series,
    not a second population block."""
    one = _bytes(capi, _group(spheres=[]), "fp32")
    two = _bytes(capi, _group(), "fp32")
    rep2 = _bytes(capi, [_group(spheres=[]), _group(spheres=[])], "fp32")
    assert one < two < one + (rep2 - one) // 4


@pytest.mark.parametrize("bad", [
    dict(spheres=[dict(radius=2.5, X0=(7.5, 7.5, 17.0))]),    # initial boxes share nodes
    dict(spheres=[dict(radius=2.5, X0=(7.5, 7.5, 46.0))]),    # ... across the periodic face
    dict(spheres=[dict(radius=0.0, X0=(7.5, 7.5, 30.0))]),    # a shared entry without a sphere
    dict(radius=0.0),                                         # a fluid without its own sphere
    dict(spheres=[dict(radius=2.5, X0=(7.5, 7.5, 30.0), U0=(0.0, 0.0, 0.7))]),
    dict(spheres=[dict(radius=2.5, X0=(14.0, 7.5, 30.0))]),   # second sphere touches a wall
])
def test_invalid_sphere_groups_rejected(capi, bad):
    with pytest.raises(capi.LbmError) as e:
        _bytes(capi, _group(**bad), "fp32")
    assert e.value.code == capi.LBM_EINVAL


def test_group_limits_rejected(capi):
    from paper_1909_01092_amd.sim import make_params
    L = capi.lib()
    n = C.c_size_t()
    arr = make_params(dict(nx=16, ny=16, nz=16))
    arr[0].shared_fluid = 1                  # nothing before the first entry
    assert L.lbm_workspace_bytes(arr, 1, 1, C.byref(n)) == capi.LBM_EINVAL
    arr = make_params(_group())
    arr[1].shared_fluid = 2
    assert L.lbm_workspace_bytes(arr, 2, 1, C.byref(n)) == capi.LBM_EINVAL
    # 16 spheres per fluid at most: 17 spheres spaced 12 apart in a long duct
    many = dict(nx=16, ny=16, nz=12 * 17, walls=3, radius=2.5, X0=(7.5, 7.5, 6.0),
                spheres=[dict(radius=2.5, X0=(7.5, 7.5, 6.0 + 12 * k)) for k in range(1, 17)])
    with pytest.raises(capi.LbmError) as e:
        _bytes(capi, many, "fp32")
    assert e.value.code == capi.LBM_EINVAL and b"more than 16" in str(e.value).encode()
    many["spheres"] = many["spheres"][:15]
    assert _bytes(capi, many, "fp32") > 0
