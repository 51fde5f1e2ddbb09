"""Pins of the oracle with several spheres in one fluid (the multi-particle
follow-up of Sec. 5; the particle paragraph of Sec. 2 applied to each sphere).

Each sphere keeps its own moving-wall links, wetting layer, reaction force,
cover / uncover events and Newton-Euler step; the fluid's mass correction and
balanced driving are global.  Pinned by:
  * a brute-force restatement with two spheres (tests/brute_force.py);
  * periodic images: two identical spheres in a channel doubled along its
    periodic axis reproduce one sphere in the original channel;
  * per-component mass and total momentum (fluid + spheres + pending events)
    conserved with two spheres crossing nodes;
  * a co-moving pair in a uniform stream feels no force.
"""
import numpy as np

from oracle import oracle as om

from test_oracle_pins import _feq_pop  # noqa: E402  (uniform-flow equilibrium)


def _two(p, spheres):
    q = dict(om.DEFAULTS)
    q.update(p)
    q["spheres"] = spheres
    return q


def test_brute_force_two_spheres():
    """30 steps of the oracle with two moving spheres (distinct radii, densities
    and wetting offsets, cover / uncover events on both, noise, distinct
    relaxation rates) against the brute-force restatement."""
    import sys
    import os
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    from brute_force import BruteForce
    p = _two(dict(nx=6, ny=6, nz=12, walls=3, init_amp=1e-3, G=1.5, tau_shear=0.8, tau_bulk=1.1,
                  tau_mom=0.9, tau_ghost=1.3, kT=1e-4, seed=12, g=(0.0, 0.0, 2e-4), radius=1.3,
                  rho_p=2.0, wet_drho=0.2, X0=(2.6, 2.4, 2.7), U0=(0.03, -0.02, 0.09),
                  W0=(0.05, 0.02, 0.03)),
             [dict(radius=1.45, rho_p=1.6, wet_drho=-0.15, X0=(2.3, 2.7, 8.4), U0=(-0.02, 0.03, -0.08),
                   W0=(-0.02, 0.0, 0.01))])
    sim = om.OracleSim(p)
    assert sim.n_spheres() == 2
    f0 = sim.populations()
    bf = BruteForce(dict(p, M0=float(f0.sum())), f0, [sim.sphere(0), sim.sphere(1)], sim.normals)
    for _ in range(30):
        sim.step(1)
        bf.step()
    f = sim.populations()
    assert np.abs(f - bf.f).max() <= 1e-13 * np.abs(f).max()
    for k in range(2):
        P, sp = sim.sphere(k), bf.sph[k]
        assert (P["n_covered"], P["n_uncovered"]) == (sp["n_cov"], sp["n_unc"]), k
        assert sp["n_cov"] > 0 and sp["n_unc"] > 0, k
        for key, v in (("X", sp["X"]), ("U", sp["U"]), ("W", sp["W"]), ("F", sp["F"]), ("T", sp["T"])):
            assert np.abs(P[key] - v).max() <= 1e-12 * max(np.abs(P[key]).max(), 1e-300), (k, key)


def test_two_periodic_images_equal_one_sphere():
    """A channel periodic in z of length L with one sphere, and the same channel
    of length 2 L with the sphere and its image L further: with a uniform start
    and no noise the doubled system is invariant under the shift by L, so each
    of its spheres moves, feels forces and meets events exactly as the single
    one, and the populations are the single channel's twice over (to the
    rounding of the longer sums)."""
    base = dict(nx=10, ny=10, nz=14, walls=3, G=1.5, kT=0.0, init_amp=0.0, g=(0.0, 0.0, 2e-4),
                radius=2.6, rho_p=2.0, wet_drho=0.1, X0=(4.3, 4.6, 6.2), U0=(0.01, -0.02, 0.06),
                W0=(0.01, 0.02, 0.0))
    one = om.OracleSim(base)
    X1 = (base["X0"][0], base["X0"][1], base["X0"][2] + 14.0)
    two = om.OracleSim(_two(dict(base, nz=28), [dict(radius=2.6, rho_p=2.0, wet_drho=0.1, X0=X1,
                                                      U0=base["U0"], W0=base["W0"])]))
    for _ in range(4):
        one.step(10)
        two.step(10)
        P = one.particle()
        for k in range(2):
            Q = two.sphere(k)
            X = np.array(Q["X"]) - np.array([0.0, 0.0, 14.0 * k])
            assert np.abs(X - P["X"]).max() < 1e-12
            for key in ("U", "W", "F", "T"):
                assert np.abs(Q[key] - P[key]).max() <= 1e-11 * np.abs(P[key]).max(), (k, key)
            assert (Q["n_covered"], Q["n_uncovered"]) == (P["n_covered"], P["n_uncovered"])
    f1, f2 = one.populations(), two.populations()
    assert np.abs(f2 - np.concatenate([f1, f1], axis=2)).max() <= 1e-13 * np.abs(f1).max()
    assert P["n_covered"] > 0 and P["n_uncovered"] > 0


def _pair_periodic():
    return _two(dict(nx=12, ny=12, nz=20, walls=0, G=1.5, kT=1e-5, init_amp=1e-3, seed=13, radius=2.5,
                     rho_p=2.0, wet_drho=0.1, X0=(5.5, 5.2, 4.4), U0=(0.02, -0.03, 0.05)),
                [dict(radius=2.2, rho_p=1.7, wet_drho=-0.2, X0=(6.1, 6.6, 14.3), U0=(-0.03, 0.02, -0.04),
                      W0=(0.0, 0.01, -0.01))])


def test_mass_conserved_with_two_spheres():
    sim = om.OracleSim(_pair_periodic())
    m0, _ = sim.observables()
    worst = 0.0
    for _ in range(8):
        sim.step(15)
        m, _ = sim.observables()
        worst = max(worst, np.abs(m / m0 - 1).max())
    assert all(sim.sphere(k)["n_covered"] + sim.sphere(k)["n_uncovered"] > 0 for k in range(2))
    assert worst < 1e-13, worst


def test_momentum_conserved_with_two_spheres():
    """Fully periodic, no driving: fluid momentum + sum of m_k U_k + pending event
    momenta is constant to rounding."""
    p = _pair_periodic()
    sim = om.OracleSim(p)
    mk = [p["rho_p"] * 4.0 / 3.0 * np.pi * p["radius"] ** 3] + \
         [e["rho_p"] * 4.0 / 3.0 * np.pi * e["radius"] ** 3 for e in p["spheres"]]

    def total():
        _, j = sim.observables()
        t = j.copy()
        for k in range(2):
            s = sim.sphere(k)
            t = t + mk[k] * s["U"] + s["Pev"]
        return t

    P0 = total()
    scale = mk[0] * 0.05
    for _ in range(8):
        sim.step(15)
        assert np.abs(total() - P0).max() < 1e-13 * scale * 100
    assert all(sim.sphere(k)["n_covered"] + sim.sphere(k)["n_uncovered"] > 0 for k in range(2))


def test_co_moving_pair_feels_no_force():
    """A uniform stream at U carrying two spheres that move at U: every link
    term cancels on both, so their forces and torques vanish."""
    e, w, b, c = om.basis()
    cf = c.astype(float)
    U = np.array([0.002, -0.001, 0.003])
    sim = om.OracleSim(_two(dict(nx=12, ny=12, nz=22, radius=3.0, X0=(5.5, 5.5, 4.5), U0=tuple(U)),
                            [dict(radius=2.0, rho_p=1.5, X0=(5.5, 6.5, 15.5), U0=tuple(U))]))
    f = sim.populations()
    for l, r0 in enumerate((0.95, 0.05)):
        feq = _feq_pop(r0, U, w, cf)
        solid = f[l].sum(0) == 0
        f[l] = np.where(solid[None], 0.0, feq[:, None, None, None])
    sim.set_populations(f)
    for _ in range(5):
        sim.step(1)
        for k in range(2):
            s = sim.sphere(k)
            assert np.abs(s["F"]).max() < 1e-14, k
            assert np.abs(s["T"]).max() < 1e-13, k
            np.testing.assert_allclose(s["U"], U, rtol=1e-12)
    assert all(sim.sphere(k)["n_covered"] == 0 for k in range(2))
