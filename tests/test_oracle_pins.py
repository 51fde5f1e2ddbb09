"""Pins of the FP64 CPU oracle against facts fixed outside it.

Each test checks the oracle against mathematics or numbers the paper prints,
never against a re-typed copy of the oracle's own formula:
  * lattice isotropy and mode orthogonality in exact rational arithmetic;
  * Philox4x32-10 against rocRAND's independent implementation;
  * Box-Muller output against the standard normal law;
  * the mode-space collision against the population-space BGK + Guo forcing
    special case (all relaxation times equal, no noise);
  * the Shan-Chen force of a linear profile (exact: -G rho_A c_s^2 grad rho_B);
  * the wetting-layer force in a uniform fluid (closed form in Delta rho);
  * transport coefficients D = 1/6 and eta = 0.383 (rho_tot = 2.30) that the
    paper states for its relaxation times (Sec. 2, after the bulk pressure);
  * equipartition <u_a^2> = kT/rho, <drho_l^2> = 3 kT rho_l (fluctuation-
    dissipation, Sec. 2 noise paragraph);
  * the textbook series of Poiseuille flow in a square duct;
  * invariants: per-component mass with a moving sphere and cover/uncover
    events, total momentum of fluid + particle, zero force on a co-moving
    sphere;
  * the A <-> B mirror symmetry of a sphere at a flat interface between the
    two demixed phases: Delta rho = 0 keeps it on the interface, +-Delta rho
    give mirror-image motions, and Delta rho > 0 (affinity to A) draws it
    into the A phase;
  * brute force: an independent dense-matrix, population-space restatement
    of the whole step (tests/brute_force.py) on a tiny walled channel with a
    moving sphere, which planted mistakes in the oracle fail;
  * the adjoint against central differences of the forward step and the
    linear-response limit dJ/dg_z = J/g_z.
"""
import os
import shutil
import subprocess
import tempfile
from fractions import Fraction as Fr

import numpy as np
import pytest

Q = 19


def _exact_basis(om):
    e, w, b, c = om.basis()
    E = np.rint(e).astype(np.int64)
    assert np.array_equal(E, e), "mode polynomials must be integer on the lattice"
    W = [Fr(x).limit_denominator(1000) for x in w]
    for x, y in zip(W, w):
        assert float(x) == y
    return E, W, b, c


def test_lattice_isotropy_exact(oracle_lib):
    E, W, b, c = _exact_basis(oracle_lib)
    assert sum(W) == 1
    d = lambda i, j: 1 if i == j else 0  # noqa: E731
    for a in range(3):
        assert sum(W[i] * c[i, a] for i in range(Q)) == 0
        for bb in range(3):
            assert sum(W[i] * c[i, a] * c[i, bb] for i in range(Q)) == Fr(d(a, bb), 3)
            for g in range(3):
                assert sum(W[i] * c[i, a] * c[i, bb] * c[i, g] for i in range(Q)) == 0
                for h in range(3):
                    m4 = sum(W[i] * c[i, a] * c[i, bb] * c[i, g] * c[i, h] for i in range(Q))
                    assert m4 == Fr(d(a, bb) * d(g, h) + d(a, g) * d(bb, h) + d(a, h) * d(bb, g), 9)
    # velocity set: rest + 6 axis + 12 planar diagonal links, listed in opposite pairs
    assert sorted(int((c[i] ** 2).sum()) for i in range(Q)) == [0] + [1] * 6 + [2] * 12
    for i in range(1, Q, 2):
        assert np.array_equal(c[i], -c[i + 1])


def test_modes_orthogonal_exact(oracle_lib):
    E, W, b, c = _exact_basis(oracle_lib)
    for k in range(Q):
        for m in range(Q):
            s = sum(W[i] * int(E[k, i]) * int(E[m, i]) for i in range(Q))
            if k == m:
                assert s > 0 and float(s) == pytest.approx(b[k], rel=1e-15)
            else:
                assert s == 0, (k, m)
    # the hydrodynamic (conserved) modes are mass and the three momenta
    assert np.all(E[0] == 1)
    assert np.array_equal(E[1:4].T, c)
    assert [Fr(x).limit_denominator(100) for x in b] == [
        Fr(1), Fr(1, 3), Fr(1, 3), Fr(1, 3), Fr(2, 3), Fr(4, 3), Fr(4, 9), Fr(1, 9), Fr(1, 9),
        Fr(1, 9), Fr(2, 3), Fr(2, 3), Fr(2, 3), Fr(2, 9), Fr(2, 9), Fr(2, 9), Fr(2), Fr(4, 3),
        Fr(4, 9)]


def test_equilibrium_moments_exact(oracle_lib):
    """Second-order equilibrium: Maxwellian moments up to the stress, zero ghosts."""
    E, W, b, c = _exact_basis(oracle_lib)
    rng = np.random.default_rng(1)
    for _ in range(4):
        rho = Fr(int(rng.integers(1, 50)), 17)
        u = [Fr(int(rng.integers(-9, 9)), 97) for _ in range(3)]
        uu = sum(x * x for x in u)
        feq = []
        for i in range(Q):
            cu = sum(int(c[i, a]) * u[a] for a in range(3))
            feq.append(W[i] * rho * (1 + 3 * cu + Fr(9, 2) * cu * cu - Fr(3, 2) * uu))
        assert sum(feq) == rho
        for a in range(3):
            assert sum(feq[i] * int(c[i, a]) for i in range(Q)) == rho * u[a]
            for bb in range(3):
                pab = sum(feq[i] * int(c[i, a]) * int(c[i, bb]) for i in range(Q))
                assert pab == rho * u[a] * u[bb] + (rho / 3 if a == bb else 0)
        for k in range(10, Q):
            assert sum(int(E[k, i]) * feq[i] for i in range(Q)) == 0, k


ROCRAND_PROBE = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
struct Probe : rocrand_device::philox4x32_10_engine {
  uint4 rounds(uint4 c, uint2 k) { return ten_rounds(c, k); }
};
int main() {
  Probe p; unsigned c0, c1, c2, c3, k0, k1;
  while (scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    uint4 c = {c0, c1, c2, c3}; uint2 k = {k0, k1};
    uint4 r = p.rounds(c, k);
    printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
"""


def test_philox_matches_rocrand(oracle_lib):
    """The oracle's Philox4x32-10 agrees word for word with rocRAND's engine."""
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    hdr = "/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"
    if not (os.path.exists(hipcc) and os.path.exists(hdr)):
        pytest.skip("rocRAND headers / hipcc not available")
    with tempfile.TemporaryDirectory() as td:
        src = os.path.join(td, "probe.cpp")
        exe = os.path.join(td, "probe")
        with open(src, "w") as fh:
            fh.write(ROCRAND_PROBE)
        subprocess.run([hipcc, "-O1", "-I/opt/rocm/include", src, "-o", exe], check=True,
                       capture_output=True)
        rng = np.random.default_rng(123)
        cases = rng.integers(0, 2**32, size=(600, 6), dtype=np.uint64).tolist()
        cases += [[0] * 6, [2**32 - 1] * 6, [5, 17, 3, 0, 0, 0], [27647, 199, 8, 0, 0, 1]]
        inp = "\n".join(" ".join(str(int(v)) for v in cs) for cs in cases) + "\n"
        out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
    ref = [list(map(int, line.split())) for line in out.strip().splitlines()]
    assert len(ref) == len(cases)
    for cs, r in zip(cases, ref):
        assert oracle_lib.philox(cs[:4], cs[4:]) == r


def test_normals_are_standard_gaussian(oracle_lib):
    from scipy import stats
    sim = oracle_lib.OracleSim(dict(nx=4, ny=4, nz=4, seed=77))
    z = np.array([sim.normals(node, step) for node in range(200) for step in range(60)])
    assert z.shape == (12000, 36)
    flat = z.ravel()
    assert abs(flat.mean()) < 4.0 / np.sqrt(flat.size)
    assert abs(flat.var() - 1.0) < 4.0 * np.sqrt(2.0 / flat.size)
    assert stats.kstest(flat, "norm").pvalue > 1e-4
    corr = np.corrcoef(z.T)
    off = corr[~np.eye(36, dtype=bool)]
    assert np.abs(off).max() < 5.0 / np.sqrt(z.shape[0])


def _feq_pop(rho, u, w, c):
    cu = c @ u
    return w * rho * (1 + 3 * cu + 4.5 * cu * cu - 1.5 * (u @ u))


@pytest.mark.parametrize("tau", [1.0, 0.8, 1.7])
def test_collision_equals_bgk_guo_when_rates_equal(oracle_lib, tau):
    """All relaxation times equal and kT = 0: MRT reduces to BGK with Guo forcing
    (population form, Guo-Zheng-Shi 2002) for each component at the common
    velocity u = (j_A + j_B + (F_A + F_B)/2) / rho."""
    e, w, b, c = oracle_lib.basis()
    cf = c.astype(float)
    sim = oracle_lib.OracleSim(dict(nx=4, ny=4, nz=4, tau_shear=tau, tau_bulk=tau, tau_mom=tau,
                                    tau_ghost=tau, kT=0.0))
    rng = np.random.default_rng(5)
    for _ in range(20):
        fin = np.empty((2, Q))
        for l, r0 in enumerate((0.95, 0.05)):
            fin[l] = _feq_pop(r0 * (1 + 0.05 * rng.standard_normal()), 0.05 * rng.standard_normal(3),
                              w, cf) + 1e-3 * r0 * w * rng.standard_normal(Q)
        F = 1e-3 * rng.standard_normal((2, 3))
        rho_l = fin.sum(1)
        j = fin @ cf
        u = (j.sum(0) + 0.5 * F.sum(0)) / rho_l.sum()
        out = sim.collide_node(fin, F, np.zeros(36))
        for l in range(2):
            S = w * (3 * ((cf - u) @ F[l]) + 9 * (cf @ u) * (cf @ F[l]))
            ref = fin[l] - (fin[l] - _feq_pop(rho_l[l], u, w, cf)) / tau + (1 - 0.5 / tau) * S
            np.testing.assert_allclose(out[l], ref, rtol=0, atol=1e-15)


def test_shan_chen_force_of_linear_profile(oracle_lib):
    """F_A = -G rho_A sum_i w_i rho_B(x+c_i) c_i is exactly -G rho_A c_s^2 grad rho_B
    for a linear rho_B (and vice versa), at nodes whose stencil stays linear."""
    e, w, b, c = oracle_lib.basis()
    nx, ny, nz, G = 16, 4, 4, 1.3
    sim = oracle_lib.OracleSim(dict(nx=nx, ny=ny, nz=nz, G=G))
    x = np.arange(nx)
    rA = 0.9 + 0.002 * x
    rB = 0.07 - 0.001 * x
    f = np.zeros((2, Q, nz, ny, nx))
    for i in range(Q):
        f[0, i] = w[i] * rA[None, None, :]
        f[1, i] = w[i] * rB[None, None, :]
    sim.set_populations(f)
    F = sim.forces()
    inner = slice(1, nx - 1)
    shape = F[0, 0][:, :, inner].shape
    np.testing.assert_allclose(F[0, 0][:, :, inner],
                               np.broadcast_to((-G * rA * (-0.001) / 3)[inner], shape),
                               rtol=1e-12, atol=0)
    np.testing.assert_allclose(F[1, 0][:, :, inner],
                               np.broadcast_to((-G * rB * 0.002 / 3)[inner], shape),
                               rtol=1e-12, atol=0)
    assert np.abs(F[:, 1:]).max() < 1e-16


def test_wetting_layer_force_closed_form(oracle_lib):
    """Uniform fluid around a sphere: the virtual layer holds rho_A + drho and
    rho_B - drho, so a fluid node x feels F_A = G rho_A drho sum_{solid} w_i c_i and
    F_B = -G rho_B drho sum_{solid} w_i c_i (sum over links into particle nodes)."""
    e, w, b, c = oracle_lib.basis()
    n, R, G, dr = 12, 2.6, 1.5, 0.08
    rA, rB = 0.95, 0.05
    sim = oracle_lib.OracleSim(dict(nx=n, ny=n, nz=n, G=G, radius=R, wet_drho=dr,
                                    rho0=(rA, rB)))
    F = sim.forces()
    X = np.array([(n - 1) / 2.0] * 3)
    grid = np.stack(np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij"), -1)
    solid = (((grid - X) ** 2).sum(-1) < R * R)  # [x, y, z]
    checked = 0
    for (xi, yi, zi) in np.argwhere(~solid):
        s = np.zeros(3)
        for i in range(1, Q):
            p = (np.array([xi, yi, zi]) + c[i]) % n
            if solid[tuple(p)]:
                s += w[i] * c[i]
        fa = F[0, :, zi, yi, xi]
        fb = F[1, :, zi, yi, xi]
        np.testing.assert_allclose(fa, G * rA * dr * s, rtol=0, atol=1e-15)
        np.testing.assert_allclose(fb, -G * rB * dr * s, rtol=0, atol=1e-15)
        checked += int(np.any(s != 0))
    assert checked > 50


def _paper(key):
    """A value the paper prints (tests/golden/paper_sec2_parameters.json, with its place)."""
    import json
    path = os.path.join(os.path.dirname(__file__), "golden", "paper_sec2_parameters.json")
    with open(path) as fh:
        return json.load(fh)[key]["value"]


def _decay_rate(series, t0, t1):
    return -np.log(series[t1] / series[t0]) / (t1 - t0)


@pytest.mark.parametrize("tau", [1.0, 0.8])
def test_shear_viscosity(oracle_lib, tau):
    """A shear wave decays at nu k^2 with nu = c_s^2 (tau_shear - 1/2).  At tau = 1 and
    rho_tot = 2.30 this is eta = rho_tot nu = 0.383, the value the paper fixes."""
    e, w, b, c = oracle_lib.basis()
    cf = c.astype(float)
    nx, A = 32, 1e-4
    rA, rB = _paper("rho_A"), _paper("rho_B")
    sim = oracle_lib.OracleSim(dict(nx=nx, ny=2, nz=2, rho0=(rA, rB), tau_shear=tau))
    k = 2 * np.pi / nx
    f = np.zeros((2, Q, 2, 2, nx))
    for x in range(nx):
        u = np.array([0.0, A * np.sin(k * x), 0.0])
        f[0, :, :, :, x] = _feq_pop(rA, u, w, cf)[:, None, None]
        f[1, :, :, :, x] = _feq_pop(rB, u, w, cf)[:, None, None]
    sim.set_populations(f)
    amp = []
    for t in range(121):
        rho, u = sim.fields()
        amp.append(2.0 / nx * np.sum(u[1, 0, 0] * np.sin(k * np.arange(nx))))
        sim.step(1)
    nu = _decay_rate(np.array(amp), 20, 120) / k**2
    assert nu == pytest.approx((tau - 0.5) / 3.0, rel=0.01)
    if tau == 1.0:
        assert (rA + rB) * nu == pytest.approx(_paper("eta"), abs=6e-4)


def test_interdiffusion_coefficient(oracle_lib):
    """A composition wave (total density uniform, G = 0) decays at D k^2 with
    D = c_s^2 (tau_mom - 1/2) = 1/6, the paper's value."""
    e, w, b, c = oracle_lib.basis()
    nx, A = 32, 1e-4
    sim = oracle_lib.OracleSim(dict(nx=nx, ny=2, nz=2, rho0=(0.5, 0.5)))
    k = 2 * np.pi / nx
    f = np.zeros((2, Q, 2, 2, nx))
    for x in range(nx):
        d = A * np.sin(k * x)
        f[0, :, :, :, x] = (w * (0.5 + d))[:, None, None]
        f[1, :, :, :, x] = (w * (0.5 - d))[:, None, None]
    sim.set_populations(f)
    amp = []
    for t in range(121):
        rho, u = sim.fields()
        amp.append(2.0 / nx * np.sum((rho[0, 0, 0] - 0.5) * np.sin(k * np.arange(nx))))
        sim.step(1)
    D = _decay_rate(np.array(amp), 20, 120) / k**2
    assert D == pytest.approx(_paper("D"), rel=0.01)


def _block_se(x, nblocks=25):
    x = np.asarray(x)
    m = len(x) // nblocks
    blocks = x[: m * nblocks].reshape(nblocks, m).mean(1)
    return blocks.std(ddof=1) / np.sqrt(nblocks)


def test_equipartition(oracle_lib):
    """Fluctuation-dissipation: at rest in a periodic box <u_a^2> = kT/rho and
    <(rho_l - <rho_l>)^2> = 3 kT rho_l, up to the 1 - 1/N of the conserved totals."""
    n, kT = 8, 1e-4
    rA, rB = 0.95, 0.05
    sim = oracle_lib.OracleSim(dict(nx=n, ny=n, nz=n, kT=kT, rho0=(rA, rB), seed=11))
    sim.step(150)
    N = n**3
    u2, dA, dB = [], [], []
    for t in range(1350):
        sim.step(1)
        rho, u = sim.fields()
        u2.append((u**2).mean(axis=(1, 2, 3)).mean())
        dA.append(((rho[0] - rho[0].mean()) ** 2).mean())
        dB.append(((rho[1] - rho[1].mean()) ** 2).mean())
    corr = 1.0 - 1.0 / N
    for series, expect in ((u2, kT / (rA + rB) * corr), (dA, 3 * kT * rA * corr),
                           (dB, 3 * kT * rB * corr)):
        m, se = np.mean(series), _block_se(series)
        assert abs(m - expect) < 4 * se + 0.01 * expect, (m, expect, se)
        assert abs(m / expect - 1) < 0.04, (m, expect)


def _duct_series(N, g, nu, nterms=101):
    a = b = N / 2.0
    x = np.arange(N) - (N - 1) / 2.0
    X, Y = np.meshgrid(x, x, indexing="xy")  # Y rows, X columns -> [y, x]
    u = np.zeros_like(X)
    for n in range(1, 2 * nterms, 2):
        u += ((-1) ** ((n - 1) // 2) / n**3 *
              (1 - np.cosh(n * np.pi * Y / (2 * a)) / np.cosh(n * np.pi * b / (2 * a))) *
              np.cos(n * np.pi * X / (2 * a)))
    return 16 * a * a * g / (nu * np.pi**3) * u


def _duct_error(om, N, steps):
    g = 1e-6
    sim = om.OracleSim(dict(nx=N, ny=N, nz=2, walls=3, G=1.5, force_mode=1, g=(0, 0, g)))
    sim.step(steps)
    rho, u = sim.fields()
    uz = u[2, 0]
    ref = _duct_series(N, g, 1.0 / 6.0)
    sim.step(50)
    uz2 = sim.fields()[1][2, 0]
    assert np.abs(uz2 - uz).max() < 1e-6 * np.abs(ref).max(), "not converged"
    assert np.abs(u[0]).max() < 1e-5 * np.abs(ref).max()
    return np.sqrt(((uz - ref) ** 2).sum() / (ref**2).sum())


def test_poiseuille_square_duct(oracle_lib):
    """Steady duct flow against the Fourier series solution; half-way bounce-back
    at tau = 1 leaves a second-order wall error."""
    e12 = _duct_error(oracle_lib, 12, 900)
    e24 = _duct_error(oracle_lib, 24, 3200)
    assert e24 < 5e-3, e24
    assert 3.0 < e12 / e24 < 5.0, (e12, e24)


def test_mass_conserved_with_moving_sphere_and_events(oracle_lib):
    """Per-component mass is conserved to rounding through moving bounce-back,
    cover / uncover events, noise and the wetting layer."""
    sim = oracle_lib.OracleSim(dict(nx=14, ny=14, nz=20, walls=3, G=1.5, kT=1e-5, radius=3.3,
                                    wet_drho=0.2, init_amp=1e-3, fixed_velocity=1,
                                    U0=(0.01, -0.02, 0.07), W0=(0.0, 0.01, 0.0)))
    m0, _ = sim.observables()
    worst = 0.0
    for _ in range(10):
        sim.step(10)
        m, _ = sim.observables()
        worst = max(worst, np.abs(m / m0 - 1).max())
    p = sim.particle()
    assert p["n_covered"] > 20 and p["n_uncovered"] > 20
    assert worst < 1e-13, worst


def test_momentum_conserved_fluid_plus_particle(oracle_lib):
    """Fully periodic, no external driving: fluid momentum + m_p U + pending event
    momentum is constant to rounding (Shan-Chen pairs cancel, the wetting-layer
    reaction goes to the particle, diffusive noise is antisymmetric)."""
    R, rho_p = 2.5, 2.0
    sim = oracle_lib.OracleSim(dict(nx=12, ny=12, nz=12, G=1.5, kT=1e-5, radius=R, rho_p=rho_p,
                                    wet_drho=0.1, init_amp=1e-3, U0=(0.02, -0.03, 0.05)))
    mp = rho_p * 4.0 / 3.0 * np.pi * R**3

    def total():
        _, j = sim.observables()
        p = sim.particle()
        return j + mp * p["U"] + p["Pev"]

    P0 = total()
    scale = mp * 0.05
    for _ in range(8):
        sim.step(15)
        assert np.abs(total() - P0).max() < 1e-13 * scale * 100
    p = sim.particle()
    assert p["n_covered"] + p["n_uncovered"] > 0


def test_co_moving_sphere_feels_no_force(oracle_lib):
    """Uniform fluid at velocity U carried with a sphere moving at U: every link
    term cancels by the lattice symmetry, so force and torque vanish."""
    e, w, b, c = oracle_lib.basis()
    cf = c.astype(float)
    n, U = 12, np.array([0.002, -0.001, 0.003])
    sim = oracle_lib.OracleSim(dict(nx=n, ny=n, nz=n, radius=3.0, U0=tuple(U)))
    f = sim.populations()
    for l, r0 in enumerate((0.95, 0.05)):
        feq = _feq_pop(r0, U, w, cf)
        solid = f[l].sum(0) == 0
        f[l] = np.where(solid[None], 0.0, feq[:, None, None, None])
    sim.set_populations(f)
    for _ in range(5):
        sim.step(1)
        p = sim.particle()
        assert np.abs(p["F"]).max() < 1e-14
        assert np.abs(p["T"]).max() < 1e-13
        np.testing.assert_allclose(p["U"], U, rtol=1e-12)
    assert p["n_covered"] == 0 and p["n_uncovered"] == 0


_IFACE = dict(nx=10, ny=10, nz=16, walls=7, rho0=(2.21, 0.09), G=1.5, init_split=8, radius=2.5,
              rho_p=4.6)


def test_sphere_at_interface_mirror_symmetry(oracle_lib):
    """Closed box, A phase below z = 7.5 and B phase above (the paper's
    demixed densities), sphere centred on the interface, no noise, no
    driving.  Mirroring z about the interface and exchanging A and B maps the
    problem onto itself with Delta rho -> -Delta rho (the wetting layer adds
    +Delta rho to A and -Delta rho to B, Sec. 2 particle paragraph), so:
    Delta rho = 0 leaves the sphere on the interface, +-Delta rho move it by
    mirror-image displacements, and it stays on the box axis.  A positive
    offset (affinity to A) draws it into the A phase."""
    z0 = (_IFACE["nz"] - 1) / 2.0
    runs = {}
    for d in (0.0, 0.3, -0.3):
        s = oracle_lib.OracleSim(dict(_IFACE, wet_drho=d))
        s.step(100)
        runs[d] = s.particle()
    p0 = runs[0.0]
    assert abs(p0["X"][2] - z0) < 1e-13 and np.abs(p0["U"]).max() < 1e-14
    up, dn = runs[0.3], runs[-0.3]
    assert abs((up["X"][2] - z0) + (dn["X"][2] - z0)) < 1e-12
    assert abs(up["U"][2] + dn["U"][2]) < 1e-13
    for p in (up, dn):
        np.testing.assert_allclose(p["X"][:2], [4.5, 4.5], atol=1e-12)
    assert up["X"][2] < z0 - 0.5, up["X"]
    assert up["n_covered"] > 0 and up["n_uncovered"] > 0


# ---------------------------------------------------------------- adjoint
_ADJ_CASE = dict(nx=10, ny=12, nz=14, walls=3, rho0=(0.95, 0.05), init_amp=1e-3, G=1.5, kT=1e-5,
                 seed=3, g=(0.0, 0.0, 5e-5), force_mode=0, radius=2.7, rho_p=2.0, wet_drho=0.1,
                 X0=(4.6, 5.4, 7.3), U0=(0.02, -0.03, 0.06), W0=(0.01, 0.02, -0.01))


def _J(oracle_lib, params, nsteps):
    s = oracle_lib.OracleSim(params)
    s.step(nsteps)
    p = s.particle()
    return s.u_series()[:, 2].mean(), (p["n_covered"], p["n_uncovered"])


def test_adjoint_matches_central_differences(oracle_lib):
    """dJ/d(g, G, Delta rho) of J = mean U_z^{n+1/2} against central
    differences of the forward step, in a walled channel with noise, a
    wetting layer and a spinning sphere that covers and uncovers nodes
    (the event sets are the same at +h and -h, so J is smooth there)."""
    ns = 30
    sim = oracle_lib.OracleSim(_ADJ_CASE)
    J, grad = sim.adjoint(ns)
    J0, events = _J(oracle_lib, _ADJ_CASE, ns)
    assert J == pytest.approx(J0, rel=1e-14)
    assert min(events) > 0
    steps = [("g", 0, 1e-6, 0), ("g", 1, 1e-6, 1), ("g", 2, 1e-6, 2),
             ("G", None, 1e-4, 3), ("wet_drho", None, 1e-4, 4)]
    for key, idx, h, k in steps:
        vals = []
        for sg in (1.0, -1.0):
            p = dict(_ADJ_CASE)
            if idx is None:
                p[key] = p[key] + sg * h
            else:
                g = list(p["g"])
                g[idx] += sg * h
                p["g"] = tuple(g)
            v, ev = _J(oracle_lib, p, ns)
            assert ev == events
            vals.append(v)
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(grad[k] - fd) <= 1e-6 * abs(fd), (key, idx, grad[k], fd)


def test_adjoint_linear_response(oracle_lib):
    """Slow settling from rest in a uniform, noise-free fluid without a
    wetting offset: J is linear in g up to O(Re), so dJ/dg_z = J / g_z."""
    p = dict(nx=12, ny=12, nz=16, walls=3, G=1.5, kT=0.0, g=(0.0, 0.0, 1e-6), radius=3.0,
             rho_p=2.0, X0=(5.5, 5.5, 7.5))
    sim = oracle_lib.OracleSim(p)
    J, grad = sim.adjoint(20)
    assert J > 0
    assert abs(grad[2] - J / 1e-6) <= 1e-4 * abs(J / 1e-6)


def test_adjoint_rejects_unsupported(oracle_lib):
    sim = oracle_lib.OracleSim(dict(_ADJ_CASE, tau_shear=0.8))
    with pytest.raises(ValueError):
        sim.adjoint(2)
    sim = oracle_lib.OracleSim(dict(_ADJ_CASE, radius=0.0))
    with pytest.raises(ValueError):
        sim.adjoint(2)


def test_brute_force_step(oracle_lib):
    """20 steps of the oracle against an independent brute-force restatement
    (tests/brute_force.py): dense 19 x 19 mode matrix and its inverse
    diag(w) M^T diag(1/b), Guo source and f_eq in population space, distinct
    relaxation rates for every group, noise, Shan-Chen forces with wall
    mirrors and a wetting layer, naive per-link loops for the moving sphere
    (momentum exchange, torque), cover/uncover and the mass correction, on a
    6 x 6 x 8 walled channel with a small sphere in motion."""
    from brute_force import BruteForce
    p = dict(oracle_lib.DEFAULTS)
    p.update(nx=6, ny=6, nz=8, walls=3, init_amp=1e-3, G=1.5, tau_shear=0.8, tau_bulk=1.1,
             tau_mom=0.9, tau_ghost=1.3, kT=1e-4, seed=11, g=(0.0, 0.0, 2e-4), radius=1.3,
             rho_p=2.0, wet_drho=0.2, X0=(2.6, 2.4, 3.7), U0=(0.03, -0.02, 0.09),
             W0=(0.01, 0.02, 0.03))
    sim = oracle_lib.OracleSim(p)
    f0 = sim.populations()
    bf = BruteForce(dict(p, M0=float(f0.sum())), f0, sim.particle(), sim.normals)
    for _ in range(20):
        sim.step(1)
        bf.step()
    f = sim.populations()
    assert np.abs(f - bf.f).max() <= 1e-13 * np.abs(f).max()
    P = sim.particle()
    assert (P["n_covered"], P["n_uncovered"]) == (bf.n_cov, bf.n_unc)
    assert bf.n_cov > 0 and bf.n_unc > 0
    for key, v in (("X", bf.X), ("U", bf.U), ("W", bf.Wv), ("F", bf.F), ("T", bf.T)):
        assert np.abs(P[key] - v).max() <= 1e-12 * max(np.abs(P[key]).max(), 1e-300), key


_PLANTS = {
    # Guo term of mode 5 with the wrong sign of u.F
    "guo": ("phi[5] = 2.0 * (3.0 * u[0] * Fl[0] - uF);", "phi[5] = 2.0 * (3.0 * u[0] * Fl[0] + uF);"),
    # wetting offset added to component B instead of subtracted
    "wetting": ("s->rt[N + n] = sum[1] / cnt - drho;", "s->rt[N + n] = sum[1] / cnt + drho;"),
    # link torque with the operands of the cross product swapped
    "torque": ("                        cross(r, lp, t);", "                        cross(lp, r, t);"),
}


@pytest.mark.parametrize("plant", sorted(_PLANTS))
def test_brute_force_detects_planted_mistake(oracle_lib, plant, tmp_path):
    """The brute-force pin is not vacuous: an oracle built with one planted
    mistake (a sign, an operand order) no longer matches it."""
    from brute_force import BruteForce
    src = open(os.path.join(os.path.dirname(oracle_lib.LIB_PATH), "lbm_oracle.c")).read()
    old, new = _PLANTS[plant]
    assert src.count(old) == 1
    path = tmp_path / "planted.c"
    path.write_text(src.replace(old, new))
    lib = tmp_path / "libplanted.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off", "-fPIC", "-shared",
                    "-I" + os.path.dirname(oracle_lib.LIB_PATH), "-o", str(lib), str(path), "-lm"],
                   check=True)
    saved = oracle_lib._lib
    try:
        oracle_lib._lib = None
        keep = oracle_lib.LIB_PATH
        oracle_lib.LIB_PATH = str(lib)
        p = dict(oracle_lib.DEFAULTS)
        p.update(nx=6, ny=6, nz=8, walls=3, init_amp=1e-3, G=1.5, tau_shear=0.8, tau_bulk=1.1,
                 tau_mom=0.9, tau_ghost=1.3, kT=1e-4, seed=11, g=(0.0, 0.0, 2e-4), radius=1.3,
                 rho_p=2.0, wet_drho=0.2, X0=(2.6, 2.4, 3.7), U0=(0.03, -0.02, 0.09),
                 W0=(0.01, 0.02, 0.03))
        sim = oracle_lib.OracleSim(p)
        f0 = sim.populations()
        bf = BruteForce(dict(p, M0=float(f0.sum())), f0, sim.particle(), sim.normals)
        for _ in range(10):
            sim.step(1)
            bf.step()
        f = sim.populations()
        err = np.abs(f - bf.f).max() / np.abs(f).max()
        assert not err <= 1e-13
        del sim
    finally:
        oracle_lib.LIB_PATH = keep
        oracle_lib._lib = saved
