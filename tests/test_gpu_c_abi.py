"""The C ABI from a plain C program: `tests/c_abi_driver.c`, built with gcc
against `include/lbm.h`, `liblbm.so` and the HIP runtime, with device memory
from hipMalloc, no Python and no torch.  It runs lbm_init, lbm_step and
lbm_step_noalloc on parameter sets the binding lays out; its sphere state and
populations must equal, bit for bit, those of the same steps driven through
the Python binding.
"""
import ctypes as C
import pathlib
import shutil
import subprocess

import numpy as np
import pytest

from paper_1909_01092_amd import _capi, workloads

pytestmark = pytest.mark.gpu

ROOT = pathlib.Path(__file__).resolve().parents[1]
PKG = ROOT / "paper_1909_01092_amd"
ROCM = pathlib.Path("/opt/rocm")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no gcc")
    exe = tmp_path_factory.mktemp("cabi") / "c_abi_driver"
    cmd = [gcc, "-std=c99", "-O2", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
           f"-I{ROCM / 'include'}", f"-I{ROOT / 'include'}", str(ROOT / "tests" / "c_abi_driver.c"),
           f"-L{PKG}", "-llbm", f"-L{ROCM / 'lib'}", "-lamdhip64",
           f"-Wl,-rpath,{PKG}", f"-Wl,-rpath,{ROCM / 'lib'}", "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16"])
def test_c_program_equals_the_binding(driver, tmp_path, prec):
    from paper_1909_01092_amd.sim import Simulation, make_params
    steps = 20
    p = workloads.channel(16, 24, kT=1e-5, radius=3.3, wet_drho=0.2, seed=8, U0=(0.02, -0.01, 0.08))
    arr = make_params(p)
    (tmp_path / "params.bin").write_bytes(bytes(arr))
    out = tmp_path / "out.bin"
    print(f"C driver: 16x16x24 {prec}, {steps} + {steps} steps", flush=True)
    r = subprocess.run([str(driver), str(tmp_path / "params.bin"), str(len(arr)),
                        str(_capi.PRECISIONS[prec]), str(steps), str(out)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    data = out.read_bytes()
    n = C.sizeof(_capi.LbmParticle)
    pc = _capi.LbmParticle.from_buffer_copy(data[:n])
    fc = np.frombuffer(data[n:], dtype=np.float64).reshape(2, 19, p["nz"], p["ny"], p["nx"])

    sim = Simulation(p, prec)
    sim.step(steps)
    sim.step_noalloc(steps)
    assert np.array_equal(fc, sim.populations())
    ps = sim.particle_state()
    for name in ("X", "U", "W", "F", "T", "Pev", "Lev", "delta"):
        assert np.array_equal(np.array(list(getattr(pc, name))), ps[name]), name
    assert (pc.step, pc.n_covered, pc.n_uncovered) == (ps["step"], ps["n_covered"], ps["n_uncovered"])
    assert pc.step == 2 * steps
