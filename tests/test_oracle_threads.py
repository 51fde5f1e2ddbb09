"""The oracle's plane-parallel loops give bitwise the run of one thread.

Its sums over nodes (wetting-layer reaction, link momentum exchange, torque,
bounce-back mass flux) are taken per z-plane in a fixed order and the plane
sums added in z order, so the thread count cannot change a bit.  Cases: a
walled channel with a sphere driven through cover / uncover events, wetting
and noise; a fully periodic box whose free sphere crosses a face.
"""
import numpy as np

from oracle import oracle as om
from paper_1909_01092_amd import workloads

CASES = [
    workloads.channel(16, 24, kT=1e-5, radius=3.3, wet_drho=0.2, fixed_velocity=1,
                      U0=(0.01, -0.02, 0.07), W0=(0.0, 0.01, 0.0), seed=5),
    workloads.full(dict(nx=14, ny=14, nz=15, walls=0, G=1.5, kT=1e-5, init_amp=1e-3, radius=2.5,
                        wet_drho=0.1, U0=(0.02, -0.03, 0.05), tau_shear=0.8, tau_bulk=1.1,
                        tau_mom=0.9, tau_ghost=1.3, seed=6)),
]


def _run(p, threads, steps=30):
    om.set_threads(threads)
    s = om.OracleSim(p)
    s.step(steps)
    return s.populations(), s.particle(), s.u_series()


def test_thread_count_does_not_change_the_run():
    before = om.set_threads(0)
    try:
        for p in CASES:
            f1, P1, u1 = _run(p, 1)
            for t in (2, 5, 8):
                ft, Pt, ut = _run(p, t)
                assert np.array_equal(f1, ft), t
                assert np.array_equal(u1, ut), t
                for k in ("X", "U", "W", "F", "T", "Pev", "Lev", "delta"):
                    assert np.array_equal(P1[k], Pt[k]), (t, k)
                assert (P1["n_covered"], P1["n_uncovered"], P1["n_links"]) == \
                    (Pt["n_covered"], Pt["n_uncovered"], Pt["n_links"])
            assert P1["n_covered"] + P1["n_uncovered"] > 0
    finally:
        om.set_threads(before)
