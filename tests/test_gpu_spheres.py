"""Several spheres in one fluid on the GPU against the FP64 oracle (the
multi-particle follow-up of Sec. 5; each sphere follows the particle
paragraph of Sec. 2: its own links, wetting layer, events and Newton-Euler
step, with a global mass correction and, under balanced driving, the fluid
carrying minus the sum of the spheres' external forces).

Bars, as for one sphere: FP64 storage 1e-12 relative on populations and
deviations, each sphere's X to 1e-12 absolute and U, W, F, T to 1e-12
relative, event counts and link counts exact; FP32 storage 1e-5 on
deviations.  Every case has cover and uncover events on every sphere.
"""
import math

import numpy as np
import pytest

from oracle.oracle import OracleSim

from test_gpu_parity import dev, rel, solid_mask  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def Sim():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1909_01092_amd.sim import Simulation
    return Simulation


def _oracle(p):
    from oracle import oracle as om
    q = dict(om.DEFAULTS)
    q.update(p)
    return OracleSim(q)


def two_walled():
    """Walled 12 x 12 x 40 duct, distinct MRT rates, noise, two spheres of
    distinct radii, densities and wetting offsets."""
    return dict(nx=12, ny=12, nz=40, walls=3, init_amp=1e-3, G=1.5, tau_shear=0.8, tau_bulk=1.1,
                tau_mom=0.9, tau_ghost=1.3, kT=1e-4, seed=12, g=(0.0, 0.0, 2e-4), radius=2.5,
                rho_p=2.0, wet_drho=0.1, X0=(5.6, 5.3, 8.4), U0=(0.03, -0.02, 0.05),
                W0=(0.05, 0.02, 0.03),
                spheres=[dict(radius=2.2, rho_p=1.6, wet_drho=-0.15, X0=(6.2, 6.7, 27.5),
                              U0=(-0.02, 0.03, -0.04), W0=(-0.02, 0.0, 0.01))])


def three_periodic():
    """Fully periodic 16 x 16 x 48 box, all relaxation times 1, three spheres."""
    return dict(nx=16, ny=16, nz=48, walls=0, init_amp=1e-3, G=1.2, kT=1e-4, seed=21,
                g=(0.0, 0.0, 1e-4), radius=2.5, rho_p=2.0, wet_drho=0.1, X0=(7.3, 8.1, 6.3),
                U0=(0.04, -0.03, 0.06), W0=(0.02, -0.03, 0.01),
                spheres=[dict(radius=2.1, rho_p=1.5, wet_drho=-0.1, X0=(8.45, 7.48, 22.47),
                              U0=(-0.05, 0.05, -0.06), W0=(0.0, 0.02, -0.02)),
                         dict(radius=2.8, rho_p=2.5, wet_drho=0.05, X0=(7.9, 8.4, 38.6),
                              U0=(0.02, 0.04, 0.07), W0=(0.01, 0.0, 0.03))])


def compare_fluid(sim, ref, entry, tol, tol_dev, what):
    f, fr = sim.populations(entry), ref.populations()
    assert np.array_equal(solid_mask(f), solid_mask(fr)), f"{what}: particle nodes differ"
    rho0 = ref.params.get("rho0", (0.95, 0.05))
    e, ed = rel(f, fr), rel(dev(f, rho0), dev(fr, rho0))
    print(f"{what}: rel err f {e:.3e}, deviations {ed:.3e}", flush=True)
    assert e < tol and ed < tol_dev, (what, e, ed)


def compare_spheres(sim, ref, first, tol, what, need_events=True):
    K = ref.n_spheres()
    for k in range(K):
        pg, po = sim.particle_state(first + k), ref.sphere(k)
        assert pg["step"] == po["step"], (what, k)
        for key in ("n_covered", "n_uncovered", "n_links"):
            assert pg[key] == po[key], (what, k, key, pg[key], po[key])
        if need_events:
            assert po["n_covered"] > 0 and po["n_uncovered"] > 0, (what, k)
        assert abs(pg["n_fluid"] - po["n_fluid"]) == 0.0, (what, k)
        assert np.abs(pg["X"] - po["X"]).max() < tol, (what, k, "X")
        for key in ("U", "W", "F", "T", "Pev", "Lev", "delta"):
            scale = max(np.abs(po[key]).max(), 1e-300)
            err = np.abs(pg[key] - po[key]).max() / scale
            lim = tol if key in ("U", "W", "F", "T") else max(tol, 1e-12)
            if key in ("Pev", "Lev") and np.abs(po[key]).max() == 0.0:
                assert np.abs(pg[key]).max() == 0.0, (what, k, key)
                continue
            print(f"{what}: sphere {k} {key} err {err:.3e}", flush=True)
            assert err < lim * (10.0 if key == "delta" else 1.0), (what, k, key, err)


def test_two_spheres_general_mrt_fp64(Sim):
    p = two_walled()
    ref = _oracle(p)
    sim = Sim(p, "fp64")
    assert len(sim.replicas) == 2 and sim.replicas[1]["shared_fluid"] == 1
    for n in (1, 29, 30):
        sim.step(n)
        ref.step(n)
        compare_fluid(sim, ref, 0, 1e-12, 1e-12, f"two walled fp64 step {ref.particle()['step']}")
    compare_spheres(sim, ref, 0, 1e-12, "two walled fp64")
    # the second entry reports the same fluid
    assert np.array_equal(sim.populations(1), sim.populations(0))
    sim.close()


@pytest.mark.parametrize("prec,tol,tol_dev", [("fp64", 1e-12, 1e-12), ("fp32", 1e-5, 1e-5)])
def test_three_spheres_periodic(Sim, prec, tol, tol_dev):
    p = three_periodic()
    ref = _oracle(p)
    sim = Sim(p, prec)
    sim.step(60)
    ref.step(60)
    compare_fluid(sim, ref, 0, tol, tol_dev, f"three periodic {prec}")
    if prec == "fp64":
        compare_spheres(sim, ref, 0, 1e-12, "three periodic fp64")
    else:
        for k in range(3):
            pg, po = sim.particle_state(k), ref.sphere(k)
            assert np.abs(pg["X"] - po["X"]).max() < 1e-4, k
            assert np.abs(pg["U"] - po["U"]).max() < 1e-4 * np.abs(po["U"]).max(), k
    sim.close()


def test_groups_series_and_observables(Sim):
    """Each sphere's U series (ring wrapped) against the oracle's, and the
    shared fluid's observables the same from every entry of the group."""
    p = dict(three_periodic(), series_cap=25)
    ref = _oracle(p)
    sim = Sim(p, "fp64")
    sim.step(60)
    ref.step(60)
    for k in range(3):
        u = sim.u_series(k)
        ur = ref.sphere_u_series(k)[-25:]
        assert u.shape == (25, 3)
        assert np.abs(u - ur).max() < 1e-12 * np.abs(ur).max(), k
    o = [sim.observables(k) for k in range(3)]
    m, j = ref.observables()
    for k in range(3):
        assert np.array_equal(o[k]["mass"], o[0]["mass"]) and o[k]["n_fluid"] == o[0]["n_fluid"]
    assert np.abs(o[0]["mass"] - m).max() < 1e-12 * np.abs(m).max()
    assert np.abs(o[0]["momentum"] - j).max() < 1e-10 * np.abs(m).sum()
    sim.close()


def ensemble_mixed():
    """Three replicas in one context: two spheres, one sphere, three spheres.
    Six boxes of edge 14 give 258 particle workgroups, so the group state is
    published by the separate finishing launch."""
    base = dict(nx=14, ny=14, nz=50, walls=3, init_amp=1e-3, G=1.3, kT=1e-4, g=(0.0, 0.0, 1e-4))
    a = dict(base, seed=5, replica=0, radius=4.0, rho_p=2.0, wet_drho=0.1, X0=(6.4, 6.7, 8.3),
             U0=(0.03, 0.02, 0.05), W0=(0.01, 0.02, 0.0),
             spheres=[dict(radius=3.6, rho_p=1.7, wet_drho=-0.1, X0=(6.8, 6.2, 30.6),
                           U0=(-0.02, 0.03, -0.05), W0=(0.0, -0.01, 0.02))])
    b = dict(base, seed=6, replica=1, radius=4.0, rho_p=2.2, wet_drho=0.05, X0=(6.6, 6.4, 20.2),
             U0=(0.02, -0.03, 0.06))
    c = dict(base, nz=56, seed=7, replica=2, radius=4.0, rho_p=2.0, wet_drho=0.1, X0=(6.3, 6.6, 7.4),
             U0=(0.03, -0.02, 0.06), W0=(0.02, 0.0, 0.01),
             spheres=[dict(radius=3.5, rho_p=1.8, wet_drho=-0.05, X0=(6.7, 6.5, 26.3),
                           U0=(-0.03, 0.02, 0.05), W0=(0.0, 0.01, 0.0)),
                      dict(radius=3.2, rho_p=2.4, wet_drho=0.12, X0=(6.5, 6.9, 44.6),
                           U0=(0.02, 0.03, -0.06), W0=(0.01, -0.02, 0.0))])
    return [a, b, c]


def test_ensemble_of_groups_fp64(Sim):
    reps = ensemble_mixed()
    sim = Sim(reps, "fp64")
    assert len(sim.replicas) == 6
    refs = [_oracle(q) for q in reps]
    sim.step(40)
    first = [0, 2, 3]
    for r, ref in enumerate(refs):
        ref.step(40)
        compare_fluid(sim, ref, first[r], 1e-12, 1e-12, f"ensemble replica {r}")
        compare_spheres(sim, ref, first[r], 1e-12, f"ensemble replica {r}", need_events=False)
        for k in range(ref.n_spheres()):
            s = ref.sphere(k)
            assert s["n_covered"] + s["n_uncovered"] > 0, (r, k)
    sim.close()


def _box(X, R):
    return [math.floor(X[a] - R) - 2 for a in range(3)], 2 * math.ceil(R) + 6


def _boxes_meet(oa, Sa, ob, Sb, n3, walls):
    for ax in range(3):
        d1, d2 = ob[ax] - oa[ax], oa[ax] - ob[ax]
        if walls & (1 << ax):
            meet = d1 < Sa and d2 < Sb
        else:
            meet = (d1 % n3[ax]) < Sa or (d2 % n3[ax]) < Sb
        if not meet:
            return False
    return True


def test_contact_reported(Sim):
    """Two prescribed spheres closing in along the periodic axis: the state
    queries turn to LBM_ECONTACT at the first step whose bounding boxes share
    a node (host restatement of the box rule), not before, and stay there."""
    from paper_1909_01092_amd import _capi
    p = dict(nx=12, ny=12, nz=40, walls=3, fixed_velocity=1, radius=2.5, X0=(5.5, 5.5, 8.0),
             U0=(0.0, 0.0, 0.1), spheres=[dict(radius=2.5, X0=(5.5, 5.5, 28.0), U0=(0.0, 0.0, -0.1))])
    sim = Sim(p, "fp32")
    seen = None
    for n in range(1, 80):
        if seen is not None and n > seen + 5:
            break
        sim.step(1)
        s0 = sim.particle_state(0, allow_unstable=True)
        s1 = sim.particle_state(1, allow_unstable=True)
        ob0, S0 = _box(s0["X"], 2.5)
        ob1, S1 = _box(s1["X"], 2.5)
        meet = _boxes_meet(ob0, S0, ob1, S1, (12, 12, 40), 3)
        assert s0["contact"] == s1["contact"], n
        if seen is None:
            assert s0["contact"] == meet, (n, ob0, ob1)
            if meet:
                seen = n
        else:
            assert s0["contact"], n
    assert seen is not None and 20 < seen < 80
    with pytest.raises(_capi.LbmError) as e:
        sim.particle_state(0)
    assert e.value.code == _capi.LBM_ECONTACT
    sim.close()


def test_groups_graph_noalloc_and_resume_bitwise(Sim):
    """A fluid with three spheres steps bitwise alike with plain launches, HIP
    graph replay (10 steps per graph) and the no-allocation entry point (the
    whole checkpoint), and after restoring a checkpoint (populations and the
    spheres' states)."""
    import torch
    p = three_periodic()
    stream = torch.cuda.Stream()
    sims = [Sim(p, "fp32", stream=stream, fill=0) for _ in range(3)]
    sims[1].set_graph(10)
    sims[0].step(30)
    sims[1].step(30)
    sims[2].step_noalloc(30)
    cks = [s.checkpoint() for s in sims]
    torch.cuda.synchronize()
    assert torch.equal(cks[1], cks[0]) and torch.equal(cks[2], cks[0])
    # resume: populations and every sphere's state (the raw checkpoint bytes
    # also hold the never-read slots of particle nodes, whose stale contents
    # depend on which buffer a step wrote)
    a = sims[0]
    mid = a.checkpoint()
    a.step(15)
    f_end = a.populations()
    s_end = [a.particle_state(k) for k in range(3)]
    a.restore(mid)
    a.step(15)
    assert np.array_equal(a.populations(), f_end)
    for k in range(3):
        s = a.particle_state(k)
        assert s["step"] == 45
        for key in ("X", "U", "W", "F", "T", "Pev", "Lev", "delta"):
            assert np.array_equal(s[key], s_end[k][key]), (k, key)
    for s in sims:
        s.close()
