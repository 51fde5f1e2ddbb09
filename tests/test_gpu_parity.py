"""Parity of the HIP path with the FP64 oracle, through the C ABI.

Tolerances (written here, derived in the design notes):
  * FP64 storage: max |f_gpu - f_ref| / max |f_ref| < 1e-12 after 200 steps
    (only the rounding order differs; every decision uses the same FP64
    predicate);
  * FP32 storage of deviations: max |d_gpu - d_ref| / max |d_ref| < 1e-5 per
    field after 200 steps, with d = f - w_i rho0_l;
  * FP16 relative-deviation storage: error reported, bounded loosely.
Cases span several workgroup tiles and z-chunks with ragged tails, walls and
periodic axes, with and without the sphere, with cover/uncover events.
"""
import numpy as np
import pytest

from oracle.oracle import OracleSim
from paper_1909_01092_amd import workloads

pytestmark = pytest.mark.gpu

W = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)


@pytest.fixture(scope="module")
def Sim():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1909_01092_amd.sim import Simulation
    return Simulation


def dev(f, rho0):
    return f - W[None, :, None, None, None] * np.array(rho0)[:, None, None, None, None]


def rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def solid_mask(f):
    return f.sum(axis=(0, 1)) == 0


def compare(sim, ref, tol, tol_dev=None, rep=0, what=""):
    f, fr = sim.populations(rep), ref.populations()
    assert np.array_equal(solid_mask(f), solid_mask(fr)), f"{what}: particle nodes differ"
    e = rel(f, fr)
    rho0 = ref.params.get("rho0", (0.95, 0.05))
    ed = rel(dev(f, rho0), dev(fr, rho0))
    print(f"{what}: rel err f {e:.3e}, deviations {ed:.3e}", flush=True)
    assert e < tol, (what, e)
    if tol_dev is not None:
        assert ed < tol_dev, (what, ed)
    return e, ed


def compare_particle(sim, ref, tol, rep=0, what=""):
    pg, po = sim.particle_state(rep), ref.particle()
    assert pg["step"] == po["step"]
    assert pg["n_covered"] == po["n_covered"] and pg["n_uncovered"] == po["n_uncovered"], what
    for k in ("X", "U", "W", "F", "T"):
        scale = max(np.abs(po[k]).max(), 1e-300)
        err = np.abs(pg[k] - po[k]).max() / scale
        if k == "X":
            err = np.abs(pg[k] - po[k]).max()
        print(f"{what}: particle {k} err {err:.3e}", flush=True)
        assert err < tol, (what, k, err)
    return pg, po


def test_initial_state(Sim):
    p = workloads.channel(20, 18, kT=1e-5, radius=4.0, seed=9)
    sim, ref = Sim(p, "fp64"), OracleSim(p)
    compare(sim, ref, 1e-15, 1e-12, what="init")
    compare_particle(sim, ref, 1e-15, what="init")


@pytest.mark.parametrize("walls,kT,G", [(3, 1e-5, 1.5), (0, 1e-4, 0.0), (7, 1e-5, 1.5)])
def test_fluid_fp64(Sim, walls, kT, G):
    p = workloads.full(dict(nx=16, ny=12, nz=21, walls=walls, kT=kT, G=G, init_amp=1e-3,
                            g=(1e-5, 0.0, 2e-5), force_mode=1, seed=4))
    sim, ref = Sim(p, "fp64"), OracleSim(p)
    sim.set_launch(256, 8)       # 3 z-chunks, the last one ragged
    for n in (1, 4, 25):
        sim.step(n)
        ref.step(n)
        compare(sim, ref, 1e-13, 1e-9, what=f"fluid walls={walls} kT={kT} after +{n}")


def test_sphere_fp64_parity_small_channel(Sim):
    """24 x 24 x 48 channel, R = 4, kT = 1e-5, g = 1e-5, 200 steps (FP64)."""
    p = workloads.PARITY_SMALL
    sim, ref = Sim(p, "fp64"), OracleSim(p)
    for n in (1, 9, 40, 150):
        sim.step(n)
        ref.step(n)
        compare(sim, ref, 1e-12, 1e-12, what=f"sphere after +{n}")
    compare_particle(sim, ref, 1e-9, what="sphere 200 steps")
    pg = sim.particle_state()
    print(f"events: covered {pg['n_covered']} uncovered {pg['n_uncovered']}", flush=True)


def test_events_prescribed_motion_fp64(Sim):
    """A sphere driven at a prescribed velocity sweeps nodes: cover and uncover
    events every few steps, with wetting and noise."""
    p = workloads.channel(16, 24, kT=1e-5, radius=3.3, wet_drho=0.2, fixed_velocity=1,
                          U0=(0.01, -0.02, 0.07), W0=(0.0, 0.01, 0.0), seed=5)
    sim, ref = Sim(p, "fp64"), OracleSim(p)
    for n in (3, 17, 40):
        sim.step(n)
        ref.step(n)
        compare(sim, ref, 1e-12, what=f"events +{n}")
        compare_particle(sim, ref, 1e-9, what=f"events +{n}")
    assert sim.particle_state()["n_covered"] > 10


def test_free_sphere_periodic_fp64(Sim):
    p = workloads.full(dict(nx=14, ny=14, nz=15, walls=0, G=1.5, kT=1e-5, init_amp=1e-3,
                            radius=2.5, wet_drho=0.1, U0=(0.02, -0.03, 0.05), seed=6))
    sim, ref = Sim(p, "fp64"), OracleSim(p)
    sim.step(60)
    ref.step(60)
    compare(sim, ref, 1e-12, what="periodic free sphere")
    compare_particle(sim, ref, 1e-9, what="periodic free sphere")


def test_fp32_parity_small_channel(Sim):
    p = workloads.PARITY_SMALL
    sim, ref = Sim(p, "fp32"), OracleSim(p)
    sim.step(200)
    ref.step(200)
    compare(sim, ref, 1e-6, 1e-5, what="fp32 200 steps")
    pg, po = sim.particle_state(), ref.particle()
    errU = np.abs(pg["U"] - po["U"]).max() / np.abs(po["U"]).max()
    errX = np.abs(pg["X"] - po["X"]).max()
    print(f"fp32 particle U rel err {errU:.3e}, X abs err {errX:.3e}", flush=True)
    assert errU < 1e-5 and errX < 1e-7


def test_fp32_parity_single_run_slice(Sim):
    """A 64 x 64 x 64 slice of the single-run channel (R = 8, kT = 1e-5,
    g = 1e-4) in the benchmark's launch shape (full 64-node rows, 256 x 4):
    200 FP32 steps against the oracle."""
    p = dict(workloads.SINGLE_RUN, nz=64, X0=None)
    p = workloads.full(p)
    sim, ref = Sim(p, "fp32"), OracleSim(p)
    sim.set_launch(256, 4)
    sim.step(200)
    ref.step(200)
    compare(sim, ref, 1e-6, 1e-5, what="64x64x64 slice, fp32 200 steps")
    pg, po = sim.particle_state(), ref.particle()
    errU = np.abs(pg["U"] - po["U"]).max() / np.abs(po["U"]).max()
    print(f"slice particle U rel err {errU:.3e}", flush=True)
    assert errU < 1e-5


def test_fp32_parity_single_run_full_size(Sim):
    """The whole single-run channel, 64 x 64 x 256 (R = 8, kT = 1e-5,
    g = 1e-4), in the benchmark's launch shape (1024 x 4): 200 FP32 steps
    against the oracle, every population compared (about half a minute of
    oracle time on 16 threads)."""
    import time
    p = workloads.SINGLE_RUN
    sim, ref = Sim(p, "fp32"), OracleSim(p)
    sim.set_launch(1024, 4)
    sim.step(200)
    t0 = time.perf_counter()
    ref.step(200)
    print(f"oracle: 200 steps of 64x64x256 in {time.perf_counter() - t0:.1f} s", flush=True)
    compare(sim, ref, 1e-6, 1e-5, what="64x64x256 single run, fp32 200 steps")
    pg, po = sim.particle_state(), ref.particle()
    assert (pg["n_covered"], pg["n_uncovered"]) == (po["n_covered"], po["n_uncovered"])
    errU = np.abs(pg["U"] - po["U"]).max() / np.abs(po["U"]).max()
    # the position to FP32's relative bar on the distance travelled (about
    # 0.4 lattice units here): its error is the sum of the velocity errors
    moved = np.asarray(po["X"]) - np.asarray(p["X0"])
    errX = np.abs(pg["X"] - po["X"]).max() / np.abs(moved).max()
    print(f"single run particle U rel err {errU:.3e}, displacement rel err {errX:.3e}", flush=True)
    assert errU < 1e-5 and errX < 1e-5


# distinct relaxation times per mode group (shear, bulk, momentum, ghost),
# the brute-force pin's set: the general MRT collision of Sec. 2
MRT_TAUS = dict(tau_shear=0.8, tau_bulk=1.1, tau_mom=0.9, tau_ghost=1.3)


@pytest.mark.parametrize("prec,tol,tol_dev", [("fp64", 1e-12, 1e-12), ("fp32", 1e-6, 1e-5)])
def test_general_mrt_rates_with_events(Sim, prec, tol, tol_dev):
    """The MRT collision with a distinct relaxation rate per mode group (Sec. 2,
    MRT paragraph) on a walled channel whose sphere is driven through cover /
    uncover events, with wetting, noise and a body force: 200 steps against
    the oracle, FP64 at 1e-12 and FP32 deviations at 1e-5."""
    p = workloads.channel(16, 24, kT=1e-5, radius=3.3, wet_drho=0.2, fixed_velocity=1,
                          U0=(0.01, -0.02, 0.07), W0=(0.0, 0.01, 0.0), g=(0.0, 0.0, 1e-4), seed=5,
                          **MRT_TAUS)
    sim, ref = Sim(p, prec), OracleSim(p)
    sim.set_launch(256, 5)
    for n in (7, 193):
        sim.step(n)
        ref.step(n)
        compare(sim, ref, tol, tol_dev, what=f"MRT rates {prec} +{n}")
    pg, po = compare_particle(sim, ref, 1e-9 if prec == "fp64" else 1e-5, what=f"MRT rates {prec}")
    assert po["n_covered"] > 10 and po["n_uncovered"] > 10


@pytest.mark.parametrize("prec,tol_dev,tol_u", [("fp64", 1e-12, 1e-10), ("fp32", 1e-5, 1e-5)])
def test_general_mrt_rates_free_sphere_parity_channel(Sim, prec, tol_dev, tol_u):
    """The 24 x 24 x 48 parity channel with a free sphere and distinct
    relaxation rates per mode group, 200 steps."""
    p = dict(workloads.PARITY_SMALL, **MRT_TAUS)
    sim, ref = Sim(p, prec), OracleSim(p)
    sim.step(200)
    ref.step(200)
    compare(sim, ref, 1e-6 if prec == "fp32" else 1e-12, tol_dev, what=f"MRT rates parity channel {prec}")
    pg, po = sim.particle_state(), ref.particle()
    errU = np.abs(pg["U"] - po["U"]).max() / np.abs(po["U"]).max()
    print(f"MRT rates {prec}: particle U rel err {errU:.3e}", flush=True)
    assert errU < tol_u


def test_rejected_launch_shape_leaves_the_context_unchanged(Sim):
    """A shape whose LDS does not fit (FP64, 200-node rows, 1024 threads) is
    rejected with LBM_EINVAL, and the context keeps its previous shape:
    lbm_get_launch reports it and the following steps match the oracle."""
    from paper_1909_01092_amd._capi import LbmError
    p = workloads.full(dict(nx=200, ny=6, nz=9, walls=3, G=1.5, kT=1e-5, init_amp=1e-3,
                            g=(0.0, 0.0, 1e-5), force_mode=1, seed=21))
    sim, ref = Sim(p, "fp64"), OracleSim(p)
    sim.set_launch(256, 4)
    with pytest.raises(LbmError):
        sim.set_launch(1024, 2)
    assert sim.get_launch() == (256, 4)
    sim.step(12)
    ref.step(12)
    compare(sim, ref, 1e-12, 1e-12, what="after a rejected launch shape")


def test_fp16_error_reported(Sim):
    p = workloads.PARITY_SMALL
    sim, ref = Sim(p, "fp16"), OracleSim(p)
    sim.step(50)
    ref.step(50)
    e, ed = compare(sim, ref, 1e-3, what="fp16 50 steps")
    assert ed < 5e-2


def test_checkpoint_resume_bitwise(Sim):
    p = workloads.channel(16, 24, kT=1e-5, radius=3.3, wet_drho=0.2, fixed_velocity=1,
                          U0=(0.01, -0.02, 0.07), seed=5)
    a = Sim(p, "fp32")
    a.step(10)
    ck = a.checkpoint()
    a.step(30)
    fa, pa = a.populations(), a.particle_state()
    a.restore(ck)
    a.step(30)
    fb, pb = a.populations(), a.particle_state()
    assert np.array_equal(fa, fb)
    assert np.array_equal(pa["X"], pb["X"]) and np.array_equal(pa["U"], pb["U"])


def test_graph_replay_equals_plain_launches(Sim):
    import torch
    p = workloads.channel(16, 24, kT=1e-5, radius=3.0, g=(0, 0, 1e-4), seed=8)
    s = torch.cuda.Stream()
    a = Sim(p, "fp32", stream=s)
    b = Sim(p, "fp32", stream=s)
    b.set_graph(4)
    for _ in range(3):
        a.step(9)
        b.step(9)
        fa, fb = a.populations(), b.populations()
        assert np.array_equal(fa, fb)
        assert np.array_equal(a.particle_state()["U"], b.particle_state()["U"])


def test_fields_and_observables(Sim):
    p = workloads.channel(16, 20, kT=1e-5, radius=3.0, g=(0, 0, 1e-4), wet_drho=0.1, seed=2)
    sim, ref = Sim(p, "fp64"), OracleSim(p)
    sim.step(12)
    ref.step(12)
    rho, u = sim.fields()
    rr, ur = ref.fields()
    assert rel(rho, rr) < 1e-12
    assert np.abs(u - ur).max() < 1e-12 * max(np.abs(ur).max(), 1e-6)
    o = sim.observables(profile=True)
    m, j = ref.observables()
    assert np.abs(o["mass"] / m - 1).max() < 1e-12
    assert np.abs(o["momentum"] - j).max() < 1e-10 * np.abs(m).sum()
    fl = rr.sum(0) > 0
    assert o["n_fluid"] == fl.sum()
    assert abs(o["u2_mean"] - (ur ** 2).sum(0)[fl].mean()) < 1e-10 * (ur ** 2).sum(0)[fl].mean()


def test_ensemble_of_uneven_replicas(Sim):
    reps = [workloads.channel(16, 24, kT=1e-5, radius=3.0, g=(0, 0, 5e-5), seed=7, replica=0),
            workloads.channel(14, 20, kT=1e-5, radius=2.5, g=(0, 0, 5e-5), seed=7, replica=1),
            workloads.full(dict(nx=12, ny=10, nz=18, walls=3, kT=1e-5, init_amp=1e-3, G=1.5,
                                seed=7, replica=2))]
    sim = Sim(reps, "fp64")
    refs = [OracleSim(q) for q in reps]
    sim.step(25)
    for k, r in enumerate(refs):
        r.step(25)
        compare(sim, r, 1e-12, rep=k, what=f"ensemble replica {k}")


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-6)])
def test_noise_free_replica_among_noisy_ones(Sim, prec, tol):
    """A kT = 0 replica launched with noisy ones runs the noisy kernel form
    with zero amplitudes: it matches the oracle, and equals (as numbers; only
    the sign of an exact zero may differ) the same replica run alone, which
    takes the noise-free form."""
    quiet = workloads.channel(16, 24, kT=0.0, radius=3.0, g=(0, 0, 5e-5), seed=7, replica=1,
                              U0=(0.0, 0.01, 0.05))
    reps = [workloads.channel(14, 20, kT=1e-5, radius=2.5, g=(0, 0, 5e-5), seed=7, replica=0), quiet,
            workloads.full(dict(nx=12, ny=10, nz=18, walls=3, kT=1e-4, init_amp=1e-3, G=1.5,
                                seed=7, replica=2))]
    sim, alone = Sim(reps, prec), Sim(quiet, prec)
    refs = [OracleSim(q) for q in reps]
    sim.step(30)
    alone.step(30)
    for k, r in enumerate(refs):
        r.step(30)
        compare(sim, r, tol, rep=k, what=f"{prec} mixed-noise replica {k}")
    assert np.array_equal(sim.populations(1), alone.populations(0))
    pm, pa = sim.particle_state(1), alone.particle_state(0)
    for key in ("X", "U", "W", "F", "T"):
        assert np.array_equal(pm[key], pa[key]), key


def test_timing_samples_every_kth_step(Sim):
    from paper_1909_01092_amd._capi import LbmError
    sim = Sim(workloads.channel(16, 24, kT=1e-5, radius=3.0, g=(0, 0, 5e-5)), "fp32")
    sim.timing(3)
    sim.step(9)
    ms, n = sim.timing_read()
    assert n == 3 and ms > 0.0
    sim.timing(1)
    sim.step(4)
    assert sim.timing_read()[1] == 4
    sim.timing(0)
    sim.step(2)
    assert sim.timing_read()[1] == 0
    with pytest.raises(LbmError):
        sim.timing(-1)


def test_many_replicas_finish_apart_fp64(Sim):
    """Forty replicas, enough particle workgroups (273) that the step is
    finished by its own launch rather than by the last workgroup: every
    sphere moves fast enough for cover / uncover events, one replica has no
    sphere; three of them against the oracle."""
    reps = []
    for k in range(40):
        if k == 20:
            reps.append(workloads.full(dict(nx=12, ny=12, nz=16, walls=3, kT=1e-5, init_amp=1e-3,
                                            G=1.5, seed=11, replica=k)))
            continue
        reps.append(workloads.channel(12, 16, kT=1e-5, radius=2.5, g=(0, 0, 5e-5), seed=11, replica=k,
                                      U0=(0.0, 0.01 * (k % 3), 0.1), wet_drho=0.05 * (k % 4)))
    sim = Sim(reps, "fp64")
    sim.step(25)
    for k in (0, 20, 39):
        ref = OracleSim(reps[k])
        ref.step(25)
        compare(sim, ref, 1e-12, rep=k, what=f"replica {k} of 40")
        if k != 20:
            pg, po = compare_particle(sim, ref, 1e-10, rep=k, what=f"replica {k} of 40")
            assert po["n_covered"] > 0 and po["n_uncovered"] > 0


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16"])
def test_finishing_launch_equals_last_workgroup_bitwise(Sim, prec):
    """A replica stepped alone (its step finished by the last particle
    workgroup) and as the first of forty (finished by the separate finishing
    launch, which sums the partials through LDS over a whole workgroup) in the
    same launch shape: the same sums in the same order, so bit for bit the
    same populations and sphere state, through cover / uncover events."""
    reps = [workloads.channel(12, 16, kT=1e-5, radius=2.5, g=(0, 0, 5e-5), seed=11, replica=k,
                              U0=(0.0, 0.01 * (k % 3), 0.1), wet_drho=0.05 * (k % 4)) for k in range(40)]
    alone, many = Sim(reps[:1], prec), Sim(reps, prec)
    for s in (alone, many):
        s.set_launch(256, 4)
        s.step(25)
    assert np.array_equal(alone.populations(0), many.populations(0))
    pa, pm = alone.particle_state(0), many.particle_state(0)
    assert pa["n_covered"] > 0 and pa["n_uncovered"] > 0
    for key in ("X", "U", "W", "F", "T", "Pev", "Lev", "delta", "n_fluid"):
        assert np.array_equal(pa[key], pm[key]), key
    assert np.array_equal(alone.u_series(0), many.u_series(0))


@pytest.mark.timeout(900)
def test_large_full_size_one_step_fp16(Sim):
    """192 x 192 x 1024, R = 16, kT = 1e-4, FP16 relative-deviation storage in
    the large workload's launch shape (1024 threads, z-chunk 32): the GPU
    state after 20 steps is handed to the oracle, which takes one step; the
    GPU's next step must agree to FP16's storage rounding.  Each stored
    relative deviation is rounded to 11 bits (error <= 2^-12 of itself), so
    the deviations agree to 2^-12 = 2.4e-4 normwise plus FP32 arithmetic;
    asserted at 3e-4.  The full populations differ only by their deviations
    (w_i rho0_l is exact on both sides) and the largest deviation is of the
    order of the largest population, so they take the same bound."""
    p = workloads.LARGE
    sim = Sim(p, "fp16")
    sim.set_launch(1024, 32)
    sim.step(20)
    f0, p0 = sim.populations(), sim.particle_state()
    ref = OracleSim(p)
    ref.set_populations(f0)
    del f0
    ref.set_particle({k: p0[k] for k in ("X", "U", "W", "Pev", "Lev", "step", "n_fluid")})
    sim.step(1)
    ref.step(1)
    compare(sim, ref, 3e-4, 3e-4, what="192x192x1024 FP16 one step from the GPU state")
    pg, po = sim.particle_state(), ref.particle()
    errU = np.abs(pg["U"] - po["U"]).max() / np.abs(po["U"]).max()
    print(f"192x192x1024 one step: particle U rel err {errU:.3e}", flush=True)
    assert errU < 1e-3


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_launch_shape_does_not_change_results(Sim, prec):
    """Block sizes 256 / 512 / 1024 and z-chunks with ragged tails and both
    march directions give the same populations."""
    p = workloads.channel(16, 24, kT=1e-5, radius=3.3, seed=11)
    shapes = [(256, 3), (256, 24), (512, 5), (1024, 2), (1024, 7)]
    sims = [Sim(p, prec) for _ in shapes]
    for s, (blk, cz) in zip(sims, shapes):
        s.set_launch(blk, cz)
        assert s.get_launch() == (blk, cz)
        s.step(20)
    f0 = sims[0].populations()
    for s, shape in zip(sims[1:], shapes[1:]):
        e = rel(s.populations(), f0)
        print(f"{prec} launch {shape}: rel diff {e:.2e}", flush=True)
        assert e < 1e-14, shape


def test_autotune_keeps_the_run_where_it_was(Sim):
    p = workloads.channel(16, 24, kT=1e-5, radius=3.0, g=(0, 0, 1e-4), seed=12)
    a, b = Sim(p, "fp32"), Sim(p, "fp32")
    a.step(5)
    b.step(5)
    blk, cz, ms = a.autotune(steps_per_trial=2, preserve=True)
    print(f"autotune: block {blk} zchunk {cz} {ms * 1e3:.1f} us", flush=True)
    assert blk in (256, 512, 1024) and cz >= 2 and ms > 0
    assert a.get_launch() == (blk, cz)
    assert a.particle_state()["step"] == 5
    a.step(10)
    b.step(10)
    assert rel(a.populations(), b.populations()) < 1e-14


def test_single_run_full_size_one_step_fp32(Sim):
    """64 x 64 x 256, R = 8, FP32 storage, in the benchmark's launch shape: the
    GPU state after 30 steps is handed to the oracle, which takes one step;
    the GPU's next step must agree to the FP32 tolerance."""
    p = workloads.SINGLE_RUN
    sim = Sim(p, "fp32")
    sim.set_launch(256, 4)
    sim.step(30)
    f0, p0 = sim.populations(), sim.particle_state()
    ref = OracleSim(p)
    ref.set_populations(f0)
    ref.set_particle({k: p0[k] for k in ("X", "U", "W", "Pev", "Lev", "step", "n_fluid")})
    sim.step(1)
    ref.step(1)
    compare(sim, ref, 1e-7, 2e-5, what="64x64x256 one step from the GPU state")


@pytest.mark.parametrize("case", ["smallest", "widest_row", "no_noise", "sphere_without_nodes"])
def test_degenerate_and_extreme_shapes_fp64(Sim, case):
    """The smallest lattice (2 x 2 x 2, periodic), an x-row at the 256-node
    maximum (one row per workgroup), kT = 0 (no noise), and a sphere too
    small to cover any node (only its external force acts)."""
    if case == "smallest":
        p = workloads.full(dict(nx=2, ny=2, nz=2, walls=0, G=1.5, kT=1e-4, init_amp=1e-3, seed=3))
    elif case == "widest_row":
        p = workloads.full(dict(nx=256, ny=3, nz=4, walls=3, G=1.5, kT=1e-5, init_amp=1e-3,
                                g=(0.0, 0.0, 1e-5), force_mode=1, seed=3))
    elif case == "no_noise":
        p = workloads.channel(16, 24, kT=0.0, radius=3.3, g=(0, 0, 1e-4), seed=3)
    else:
        p = workloads.channel(12, 20, kT=1e-5, radius=0.3, g=(0, 0, 1e-4), seed=3)
    sim, ref = Sim(p, "fp64"), OracleSim(p)
    sim.step(12)
    ref.step(12)
    compare(sim, ref, 1e-12, what=f"{case} after 12 steps")
    if p["radius"] > 0:
        compare_particle(sim, ref, 1e-9, what=case)


def test_instability_is_reported(Sim):
    """A driving force that pushes the sphere past |U| = 1/2 sets the sticky
    unstable flag; the state query then returns LBM_EUNSTABLE."""
    from paper_1909_01092_amd import _capi
    p = workloads.channel(16, 24, kT=0.0, radius=2.5, g=(0.0, 0.0, 1.0), seed=3)
    sim = Sim(p, "fp32")
    sim.step(3)   # |U| passes 1/2 at the second step; stop well before the run blows up
    with pytest.raises(_capi.LbmError) as e:
        sim.particle_state()
    assert e.value.code == _capi.LBM_EUNSTABLE
    assert sim.particle_state(allow_unstable=True)["unstable"]


def test_ensemble_full_size_one_step_fp32(Sim):
    """The full 192-replica ensemble (32.7 M nodes, three lattice sizes) in
    FP32: after 20 steps one replica of each size is handed to the oracle,
    which takes one step; the GPU's next step must agree to the FP32
    tolerance."""
    reps = workloads.ensemble(steps_cap=64)
    sim = Sim(reps, "fp32")
    sim.set_launch(256, 4)
    sim.step(20)
    picks = (0, 128, 160)
    states = {r: (sim.populations(r), sim.particle_state(r)) for r in picks}
    sim.step(1)
    for r in picks:
        f0, p0 = states[r]
        ref = OracleSim(reps[r])
        ref.set_populations(f0)
        ref.set_particle({k: p0[k] for k in ("X", "U", "W", "Pev", "Lev", "step", "n_fluid")})
        ref.step(1)
        compare(sim, ref, 1e-7, 2e-5, rep=r, what=f"ensemble replica {r} one step from the GPU state")


def test_ensemble_full_size_200_steps_fp32(Sim):
    """The full 192-replica ensemble in FP32 and in the benchmark's launch
    shape (512 x 8), 200 steps from the initial state; the first replica of
    each size (32 x 32 x 128, 24 x 24 x 96, 48 x 48 x 192) against the oracle
    run alone over the same 200 steps."""
    reps = workloads.ensemble(steps_cap=256)
    sim = Sim(reps, "fp32")
    sim.set_launch(512, 8)
    sim.step(200)
    for r in (0, 128, 160):
        ref = OracleSim(reps[r])
        ref.step(200)
        compare(sim, ref, 1e-6, 1e-5, rep=r, what=f"ensemble replica {r}, 200 steps")
        pg, po = sim.particle_state(r), ref.particle()
        assert (pg["n_covered"], pg["n_uncovered"]) == (po["n_covered"], po["n_uncovered"])
        errU = np.abs(pg["U"] - po["U"]).max() / np.abs(po["U"]).max()
        print(f"ensemble replica {r}: particle U rel err {errU:.3e}", flush=True)
        assert errU < 1e-5


def test_adjoint_channel_200_steps_fp32(Sim):
    """The adjoint form's channel, 48 x 48 x 192 (R = 6, kT = 1e-5,
    g = 5e-5), 200 plain FP32 steps against the oracle."""
    p = workloads.ADJOINT
    sim, ref = Sim(p, "fp32"), OracleSim(p)
    sim.step(200)
    ref.step(200)
    compare(sim, ref, 1e-6, 1e-5, what="48x48x192 adjoint channel, fp32 200 steps")
    pg, po = sim.particle_state(), ref.particle()
    errU = np.abs(pg["U"] - po["U"]).max() / np.abs(po["U"]).max()
    print(f"adjoint channel particle U rel err {errU:.3e}", flush=True)
    assert errU < 1e-5


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16"])
def test_no_unwritten_memory_is_read(Sim, prec):
    """Every slot a step pulls from has been written: with the workspace
    filled with NaN bytes (0xff) before initialisation the run has no NaN and
    is bitwise the run on a zero-filled workspace, through walls, periodic
    wrap, a moving sphere with cover / uncover events and the wetting layer."""
    import torch
    reps = [workloads.channel(16, 24, kT=1e-5, radius=3.3, wet_drho=0.2, seed=8, replica=0,
                              U0=(0.02, -0.01, 0.08)),
            workloads.full(dict(nx=12, ny=14, nz=16, walls=7, kT=1e-5, init_amp=1e-3, G=1.5,
                                radius=2.5, rho_p=2.0, wet_drho=-0.1, U0=(0.0, 0.03, -0.06),
                                seed=8, replica=1))]
    runs = []
    for fill in (0xFF, 0x00):
        sim = Sim(reps, prec, stream=torch.cuda.Stream(), fill=fill)
        sim.step(30)
        runs.append([(sim.populations(r), sim.particle_state(r)) for r in range(len(reps))])
        sim.close()
    for (fa, pa), (fb, pb) in zip(*runs):
        assert not np.isnan(fa).any()
        assert np.array_equal(fa, fb)
        for k in ("X", "U", "W", "F", "T"):
            assert np.array_equal(pa[k], pb[k])
        assert pa["n_covered"] > 0 and pa["n_uncovered"] > 0


def test_poisoned_checkpoint_is_reported(Sim):
    """A checkpoint whose population block carries NaN bytes restores, and the
    next step sets the sticky unstable flag (LBM_EUNSTABLE on the state
    query) instead of running on silently."""
    from paper_1909_01092_amd import _capi
    sim = Sim(workloads.channel(16, 24, kT=1e-5, radius=3.0, g=(0, 0, 5e-5), seed=4), "fp32")
    sim.step(5)
    ck = sim.checkpoint()
    mid = (ck.numel() // 2) // 256 * 256
    ck[mid:mid + 4096].fill_(0xFF)
    sim.restore(ck)
    sim.particle_state()  # the restored state itself is not flagged yet
    sim.step(1)
    with pytest.raises(_capi.LbmError) as e:
        sim.particle_state()
    assert e.value.code == _capi.LBM_EUNSTABLE


def test_contexts_are_independent(Sim):
    """Two contexts in one process, on two streams, stepped in turn, give
    bitwise the results each gives alone (no library-global state)."""
    import torch
    pa = workloads.channel(16, 24, kT=1e-5, radius=3.0, g=(0, 0, 5e-5), seed=12)
    pb = workloads.full(dict(nx=12, ny=14, nz=16, walls=7, kT=1e-4, init_amp=1e-3, G=1.5, radius=2.5,
                             rho_p=2.0, wet_drho=0.1, U0=(0.0, 0.02, -0.04), seed=13))
    alone = []
    for p in (pa, pb):
        s = Sim(p, "fp32", stream=torch.cuda.Stream())
        s.step(40)
        alone.append((s.populations(), s.particle_state()["X"]))
        s.close()
    a, b = Sim(pa, "fp32", stream=torch.cuda.Stream()), Sim(pb, "fp32", stream=torch.cuda.Stream())
    for _ in range(8):
        a.step(5)
        b.step(5)
    for s, (f, X) in zip((a, b), alone):
        assert np.array_equal(s.populations(), f)
        assert np.array_equal(s.particle_state()["X"], X)


def test_fp16_storage_error_on_the_large_channel(Sim):
    """The large channel (192 x 192 x 1024, R = 16, kT = 1e-4) for 2000 steps
    with FP16 relative-deviation storage against FP32 storage on the same
    noise: the time-averaged u_z(x, y) profile, the particle's mean velocity
    and its velocity variance (measured 3e-4, 4e-6 and 3e-5)."""
    import os
    import sys
    import torch
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    from paper_1909_01092_amd import studies
    out = studies.fp16_error(torch, 2000)
    print({k: out[k] for k in ("uz_profile_rel_l2", "mean_Uz_rel", "var_Uz_rel", "unstable")}, flush=True)
    assert not out["unstable"]
    assert out["uz_profile_rel_l2"] < 2e-3
    assert out["mean_Uz_rel"] < 1e-4
    assert out["var_Uz_rel"] < 1e-3
