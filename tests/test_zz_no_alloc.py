"""lbm_step_noalloc (steps whose per-step scratch is the library's static
device array instead of the context workspace) against lbm_step, through the
C ABI: bitwise the same populations, sphere state and velocity series, on two
calls in a row (the second with a smaller lattice and box), when the two
entry points alternate on one context, and the rejection of a context whose
step scratch does not fit the array.
"""
import numpy as np
import pytest

from paper_1909_01092_amd import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def Sim():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1909_01092_amd.sim import Simulation
    return Simulation


def _same(a, b, what):
    fa, fb = a.populations(), b.populations()
    assert np.array_equal(fa, fb), what
    pa, pb = a.particle_state(), b.particle_state()
    for k in ("X", "U", "W", "F", "T", "Pev", "Lev", "delta"):
        assert np.array_equal(pa[k], pb[k]), (what, k)
    assert (pa["n_covered"], pa["n_uncovered"], pa["step"]) == (pb["n_covered"], pb["n_uncovered"], pb["step"])
    assert np.array_equal(a.u_series(), b.u_series()), what
    return pa


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_noalloc_steps_equal_plain_steps_two_calls(Sim, prec):
    import torch
    big = workloads.channel(24, 48, kT=1e-5, radius=4.0, wet_drho=0.1, g=(0.0, 0.0, 1e-4), seed=31,
                            U0=(0.01, 0.0, 0.06), series_cap=64)
    small = workloads.channel(16, 24, kT=1e-5, radius=3.3, wet_drho=0.2, fixed_velocity=1,
                              U0=(0.01, -0.02, 0.07), seed=5, series_cap=64)
    for p, what in ((big, "first call, 24x24x48"), (small, "second call, smaller 16x16x24")):
        a = Sim(p, prec, stream=torch.cuda.Stream())
        b = Sim(p, prec, stream=torch.cuda.Stream())
        a.step_noalloc(37)
        b.step(37)
        pa = _same(a, b, what)
        assert pa["n_covered"] + pa["n_uncovered"] > 0, what
        a.close()
        b.close()


def test_noalloc_and_plain_steps_alternate(Sim):
    """Both entry points on one context (ensemble of three uneven replicas)."""
    import torch
    reps = [workloads.channel(16, 24, kT=1e-5, radius=3.0, g=(0, 0, 5e-5), seed=7, replica=0),
            workloads.channel(14, 20, kT=1e-5, radius=2.5, g=(0, 0, 5e-5), seed=7, replica=1,
                              U0=(0.0, 0.02, 0.08)),
            workloads.full(dict(nx=12, ny=10, nz=18, walls=3, kT=1e-5, init_amp=1e-3, G=1.5, seed=7,
                                replica=2))]
    a = Sim(reps, "fp32", stream=torch.cuda.Stream())
    b = Sim(reps, "fp32", stream=torch.cuda.Stream())
    for n in (3, 5, 8):
        a.step_noalloc(n)
        a.step(n)
        b.step(2 * n)
    for r in range(3):
        assert np.array_equal(a.populations(r), b.populations(r)), r
        pa, pb = a.particle_state(r), b.particle_state(r)
        for k in ("X", "U", "W"):
            assert np.array_equal(pa[k], pb[k]), (r, k)


def test_noalloc_rejects_a_context_beyond_the_array(Sim):
    """300 replicas with R = 4 spheres need about 50 MiB of step scratch:
    LBM_EINVAL before any device work, and the context still steps."""
    from paper_1909_01092_amd._capi import LBM_EINVAL, LbmError
    reps = [workloads.channel(16, 20, kT=1e-5, radius=4.0, g=(0, 0, 5e-5), seed=9, replica=k, series_cap=8)
            for k in range(300)]
    sim = Sim(reps, "fp32")
    with pytest.raises(LbmError) as e:
        sim.step_noalloc(1)
    assert e.value.code == LBM_EINVAL
    assert sim.particle_state(0)["step"] == 0
    sim.step(2)
    assert sim.particle_state(299)["step"] == 2
