"""The paper's own setup on the GPU path (Sec. 3): a closed box with walls on
every axis and the immiscible-side densities rho_A = 2.21, rho_B = 0.09 at
G = 1.5 (G rho_tot = 3.45).

  * parity with the FP64 oracle on a small closed box at these densities
    (the other parity cases use the miscible 0.95 / 0.05 mixture);
  * the full 60 x 60 x 900 box in FP32: stable over 2000 steps, mass of each
    component conserved to FP32 rounding, the sphere settling along +g.
"""
import numpy as np
import pytest

from oracle.oracle import OracleSim
from paper_1909_01092_amd import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def Sim():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1909_01092_amd.sim import Simulation
    return Simulation


def test_paper_densities_parity(Sim):
    p = workloads.paper_box(n=16, nz=28, radius=3.5, kT=1e-4, g=5e-5)
    sim, ref = Sim(p, "fp64"), OracleSim(p)
    sim.step(100)
    ref.step(100)
    f, fr = sim.populations(), ref.populations()
    err = np.abs(f - fr).max() / np.abs(fr).max()
    print(f"closed 16x16x28 box, rho 2.21/0.09: 100 steps, rel err {err:.2e}", flush=True)
    assert err < 1e-12
    pg, po = sim.particle_state(), ref.particle()
    assert np.abs(pg["X"] - po["X"]).max() < 1e-12


def test_paper_box_runs(Sim):
    import torch
    p = workloads.paper_box()
    sim = Sim(p, "fp32", stream=torch.cuda.Stream())
    m0 = sim.observables()["mass"]
    sim.step(2000)
    st = sim.particle_state()
    m1 = sim.observables()["mass"]
    print(f"60x60x900 closed box: mass drift {np.abs(m1 - m0) / m0}, U {st['U']}, X {st['X']}", flush=True)
    assert not st["unstable"]
    assert np.all(np.abs(m1 - m0) <= 1e-5 * m0)
    assert st["U"][2] > 0


def test_paper_box_langevin_statistics(Sim):
    """The Langevin picture in the paper's own regime: 12 noise replicas of the
    closed 60 x 60 x 900 box (rho 2.21 / 0.09, kT = 1e-4, R = 8), 5000 steps.
    In the steady state the velocity variance along each axis is kT / m_p
    (Sec. 3), the sphere settles along +g, and the standardized velocity is
    Gaussian.  With a velocity relaxation time of about 100 steps, 12 x 4000
    steps give a standard error of about 6% on the variance."""
    import math
    import torch
    steps, skip, nrep = 5000, 1000, 12
    reps = [dict(workloads.paper_box(steps_cap=steps), replica=k) for k in range(nrep)]
    sim = Sim(reps, "fp32", stream=torch.cuda.Stream())
    sim.step(steps)
    assert not any(sim.particle_state(r)["unstable"] for r in range(nrep))
    U = np.stack([sim.u_series(r)[skip:] for r in range(nrep)])
    q = reps[0]
    mp = 4.0 / 3.0 * math.pi * q["radius"] ** 3 * q["rho_p"]
    ratios = [float(U[:, :, a].var(axis=1).mean() / (q["kT"] / mp)) for a in range(3)]
    x = U[:, :, 2] - U[:, :, 2].mean(axis=1, keepdims=True)
    x = (x / x.std(axis=1, keepdims=True)).ravel()
    skew, kurt = float((x ** 3).mean()), float((x ** 4).mean())
    print(f"paper box: Var(U)/(kT/m_p) = {ratios}, <U_z> = {U[:, :, 2].mean():.3e}, "
          f"skewness {skew:.3f}, kurtosis {kurt:.3f}", flush=True)
    for rt in ratios:
        assert 0.85 < rt < 1.25
    assert U[:, :, 2].mean() > 0
    assert abs(skew) < 0.15 and abs(kurt - 3.0) < 0.4
