"""The single run's parameter grid on the GPU path: the 64 x 64 x 256 channel
with an R = 8 sphere at every kT in {1e-6, 1e-5, 1e-4}, g in {1e-5, 3e-5,
1e-4} and Delta rho in {-0.5, 0, 0.5}, 27 replicas in one context, FP32.

  * every replica stays stable and conserves each component's mass to FP32
    rounding;
  * the mean settling velocity is proportional to the driving (linear
    friction, Sec. 3: <U> = F_p / gamma) and independent of kT (the thermal
    noise has zero mean); the wetting offset shifts it by a few percent, the
    same way at every kT;
  * the two extreme replicas (kT = 1e-4, g = 1e-4, Delta rho = -+0.5) take one
    more step on the GPU and, from the same state, in the FP64 oracle: they
    agree to the FP32 tolerance.
"""
import numpy as np
import pytest

from oracle.oracle import OracleSim
from paper_1909_01092_amd import workloads

pytestmark = pytest.mark.gpu
STEPS, TAIL = 3000, 2000


@pytest.fixture(scope="module")
def grid():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1909_01092_amd.sim import Simulation
    reps = workloads.single_grid()
    sim = Simulation(reps, "fp32", stream=torch.cuda.Stream())
    sim.set_launch(256, 4)
    m0 = [sim.observables(r)["mass"] for r in range(len(reps))]
    sim.step(STEPS)
    out = {}
    for r, q in enumerate(reps):
        st = sim.particle_state(r, allow_unstable=True)
        u = sim.u_series(r)[-TAIL:, 2]
        m = sim.observables(r)["mass"] if not st["unstable"] else np.full(2, np.nan)
        out[q["grid"]] = dict(r=r, unstable=st["unstable"], U=float(u.mean()),
                              drift=float(np.abs(m / m0[r] - 1).max()))
        print(f"kT {q['kT']:.0e} g {q['g'][2]:.0e} drho {q['wet_drho']:+.1f}: <U_z> {u.mean():.4e}, "
              f"mass drift {out[q['grid']]['drift']:.1e}", flush=True)
    yield sim, reps, out
    sim.close()


def test_grid_stable_and_conservative(grid):
    _, _, out = grid
    for key, v in out.items():
        assert not v["unstable"], key
        assert v["drift"] < 1e-5, (key, v["drift"])
        assert v["U"] > 0.0, key


def test_mean_velocity_linear_in_g_and_independent_of_kT(grid):
    _, _, out = grid
    for kT in workloads.GRID_KT:
        for d in workloads.GRID_DRHO:
            u = [out[(kT, g, d)]["U"] for g in workloads.GRID_G]
            assert 2.6 < u[1] / u[0] < 3.4, (kT, d, u)
            assert 8.5 < u[2] / u[0] < 11.5, (kT, d, u)
    for g in workloads.GRID_G[1:]:
        for d in workloads.GRID_DRHO:
            u = [out[(kT, g, d)]["U"] for kT in workloads.GRID_KT]
            assert max(u) / min(u) < 1.06, (g, d, u)
    for kT in workloads.GRID_KT:
        u = [out[(kT, 1e-4, d)]["U"] for d in workloads.GRID_DRHO]
        assert u[0] < u[1] < u[2], (kT, u)
        assert u[2] / u[0] < 1.25


def test_extreme_replicas_one_step_against_oracle(grid):
    sim, reps, out = grid
    for d in (-0.5, 0.5):
        r = out[(1e-4, 1e-4, d)]["r"]
        f0, p0 = sim.populations(r), sim.particle_state(r)
        ref = OracleSim(reps[r])
        ref.set_populations(f0)
        ref.set_particle({k: p0[k] for k in ("X", "U", "W", "Pev", "Lev", "delta", "step", "n_fluid")})
        ref.step(1)
        sim.step(1)
        f, fr = sim.populations(r), ref.populations()
        err = np.abs(f - fr).max() / np.abs(fr).max()
        print(f"drho {d:+.1f}: one step from the GPU state, rel err {err:.2e}", flush=True)
        assert err < 1e-7
        assert np.abs(sim.particle_state(r)["X"] - ref.particle()["X"]).max() < 1e-8
