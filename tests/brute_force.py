"""Brute-force FP64 restatement of one step of the method, for pinning the
oracle on tiny lattices (test code only).

Xue, Biferale, Sbragaglia, Toschi, "A lattice Boltzmann study of particle
settling in a fluctuating multicomponent fluid under confinement", Sec. 2
(eq. density, eq. lbe, MRT paragraph, eq. sc-force, noise paragraph, particle
paragraph) and Sec. 3 eq. (fp), under the readings listed in the design notes
(basis, forcing, noise layout, wetting layer, bounce-back, events, mass
correction).

Written independently of the oracle's arithmetic:
  * the collision works in population space through a dense 19 x 19 mode
    matrix M and its inverse diag(w) M^T diag(1/b): m* = m - S (m - M f_eq)
    + (I - S/2) M S_Guo + noise, with the Guo source S_Guo and f_eq built
    per population, and S the diagonal of the group rates 1/tau;
  * moments, the wetting layer, forces, streaming with bounce-back and
    momentum exchange, Newton-Euler, cover/uncover and the mass correction are
    naive loops over nodes and links.
Only the standard normals come from the oracle (Philox4x32-10 and Box-Muller,
each pinned on its own).
"""
import numpy as np

# D3Q19 in the storage order: rest, axis pairs, xy, xz, yz diagonal pairs
C = np.array([[0, 0, 0],
              [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
              [1, 1, 0], [-1, -1, 0], [1, -1, 0], [-1, 1, 0],
              [1, 0, 1], [-1, 0, -1], [1, 0, -1], [-1, 0, 1],
              [0, 1, 1], [0, -1, -1], [0, 1, -1], [0, -1, 1]])
Q = 19
W = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
OPP = [0] + [i + 1 if i % 2 else i - 1 for i in range(1, Q)]


def _poly(c):
    x, y, z = (float(v) for v in c)
    c2 = x * x + y * y + z * z
    return [1, x, y, z, c2 - 1, 3 * x * x - c2, y * y - z * z, x * y, y * z, x * z,
            (3 * c2 - 5) * x, (3 * c2 - 5) * y, (3 * c2 - 5) * z,
            (y * y - z * z) * x, (z * z - x * x) * y, (x * x - y * y) * z,
            3 * c2 * c2 - 6 * c2 + 1, (2 * c2 - 3) * (3 * x * x - c2), (2 * c2 - 3) * (y * y - z * z)]


M = np.array([_poly(c) for c in C]).T          # M[k, i] = e_k(c_i)
B = (M * M) @ W                                # b_k = sum_i w_i e_k(c_i)^2
MINV = np.diag(W) @ M.T @ np.diag(1.0 / B)     # f_i = w_i sum_k e_k(c_i) m_k / b_k


class BruteForce:
    """One replica; state copied from an oracle simulation at step n.  Several
    spheres: params["spheres"] lists the further ones (radius, rho_p,
    wet_drho) and `particle` is then the list of all sphere states; a node
    inside several spheres belongs to the first of them."""

    def __init__(self, params, f, particle, normals):
        self.p = dict(params)
        self.nx, self.ny, self.nz = params["nx"], params["ny"], params["nz"]
        self.walled = [bool(params["walls"] & (1 << a)) for a in range(3)]
        self.f = np.array(f, dtype=np.float64)          # [2][19][nz][ny][nx]
        states = particle if isinstance(particle, (list, tuple)) else [particle]
        geo = [dict(radius=params["radius"], rho_p=params["rho_p"], wet_drho=params["wet_drho"])]
        geo += [dict(radius=e["radius"], rho_p=e.get("rho_p", params["rho_p"]), wet_drho=e.get("wet_drho", 0.0))
                for e in params.get("spheres", [])]
        self.sph = []
        for g, st in zip(geo, states):
            R = g["radius"]
            Vp = 4.0 / 3.0 * np.pi * R ** 3
            mp = g["rho_p"] * Vp
            self.sph.append(dict(R=R, rho_p=g["rho_p"], drho=g["wet_drho"], Vp=Vp, mp=mp, Ip=0.4 * mp * R * R,
                                 X=np.array(st["X"], dtype=float), U=np.array(st["U"], dtype=float),
                                 W=np.array(st["W"], dtype=float), Pev=np.array(st["Pev"], dtype=float),
                                 Lev=np.array(st["Lev"], dtype=float), F=np.zeros(3), T=np.zeros(3),
                                 n_cov=0, n_unc=0))
        self.step_no = int(states[0]["step"])
        self.normals = normals                           # (node, step) -> 36 standard normals
        self.owner = self._owner([s["X"] for s in self.sph])
        # initial fluid mass (balanced driving divides the external force by it)
        self.M0 = params["M0"]

    # sphere 0, as the single-sphere form names it
    X = property(lambda self: self.sph[0]["X"])
    U = property(lambda self: self.sph[0]["U"])
    Wv = property(lambda self: self.sph[0]["W"])
    F = property(lambda self: self.sph[0]["F"])
    T = property(lambda self: self.sph[0]["T"])
    n_cov = property(lambda self: self.sph[0]["n_cov"])
    n_unc = property(lambda self: self.sph[0]["n_unc"])

    # ------------------------------------------------------------ geometry
    def _sep(self, d, a):
        n = (self.nx, self.ny, self.nz)[a]
        if not self.walled[a]:
            if d > 0.5 * n:
                d -= n
            elif d < -0.5 * n:
                d += n
        return d

    def _r(self, pos, X):
        return np.array([self._sep(pos[a] - X[a], a) for a in range(3)])

    def _owner(self, Xs):
        """-1 for fluid nodes, else the first sphere containing the node."""
        own = np.full((self.nz, self.ny, self.nx), -1, dtype=np.int64)
        for z in range(self.nz):
            for y in range(self.ny):
                for x in range(self.nx):
                    for k, X in enumerate(Xs):
                        dx = self._sep(x - X[0], 0)
                        dy = self._sep(y - X[1], 1)
                        dz = self._sep(z - X[2], 2)
                        d2 = dx * dx + dy * dy
                        d2 = d2 + dz * dz
                        if d2 < self.sph[k]["R"] ** 2:
                            own[z, y, x] = k
                            break
        return own

    def _nb(self, x, y, z, i):
        """(neighbour, crossed_wall): x + c_i wrapped on periodic axes."""
        q = [x + C[i][0], y + C[i][1], z + C[i][2]]
        n = (self.nx, self.ny, self.nz)
        crossed = False
        for a in range(3):
            if q[a] < 0 or q[a] >= n[a]:
                if self.walled[a]:
                    crossed = True
                    q[a] = 0 if q[a] < 0 else n[a] - 1   # neutral wall: the adjacent node
                else:
                    q[a] %= n[a]
        return tuple(q), crossed

    def _nodes(self):
        for z in range(self.nz):
            for y in range(self.ny):
                for x in range(self.nx):
                    yield x, y, z

    # ---------------------------------------------------------------- step
    def step(self):
        p = self.p
        f, owner = self.f, self.owner
        solid = owner >= 0
        K = len(self.sph)
        G, kT = p["G"], p["kT"]
        rho = f.sum(axis=1) * ~solid                         # [2][nz][ny][nx]
        jm = np.einsum("lizyx,ia->lazyx", f, C.astype(float)) * ~solid
        # wetting layer: particle nodes see the mean of their fluid neighbours
        # +- the wetting offset of the sphere holding them
        rt = rho.copy()
        for x, y, z in self._nodes():
            if not solid[z, y, x]:
                continue
            dr = self.sph[owner[z, y, x]]["drho"]
            acc, cnt = np.zeros(2), 0
            for i in range(1, Q):
                (qx, qy, qz), crossed = self._nb(x, y, z, i)
                if crossed or solid[qz, qy, qx]:
                    continue
                acc += rho[:, qz, qy, qx]
                cnt += 1
            rt[:, z, y, x] = (acc / cnt + np.array([dr, -dr])) if cnt else 0.0
        # external force on each sphere (Sec. 3 eq. fp) and the fluid's acceleration
        g = np.array(p["g"], dtype=float)
        rho_tot0 = p["rho0"][0] + p["rho0"][1]
        if p["force_mode"] == 1:
            af = g.copy()
            Fext = [s["Vp"] * s["rho_p"] * g for s in self.sph]
        else:
            Fext = [s["Vp"] * (s["rho_p"] - rho_tot0) * g for s in self.sph]
            af = -sum(Fext) / self.M0
        # Shan-Chen forces and their reaction on the spheres
        F = np.zeros((2, 3, self.nz, self.ny, self.nx))
        Fv, Tv = np.zeros((K, 3)), np.zeros((K, 3))
        for x, y, z in self._nodes():
            if solid[z, y, x]:
                continue
            for i in range(1, Q):
                (qx, qy, qz), crossed = self._nb(x, y, z, i)
                link = np.zeros(3)
                for l in range(2):
                    fl = -G * rho[l, z, y, x] * W[i] * rt[1 - l, qz, qy, qx] * C[i]
                    F[l, :, z, y, x] += fl
                    link += fl
                if not crossed and solid[qz, qy, qx]:
                    k = owner[qz, qy, qx]
                    r = self._r(np.array([x, y, z]) + 0.5 * C[i], self.sph[k]["X"])
                    Fv[k] += link
                    Tv[k] += np.cross(r, link)
            for l in range(2):
                F[l, :, z, y, x] += rho[l, z, y, x] * af
        # collision in population space through the dense mode matrix
        taus = (p["tau_shear"], p["tau_bulk"], p["tau_mom"], p["tau_ghost"])
        s = np.zeros(Q)
        s[1:4] = 1 / taus[2]
        s[4] = 1 / taus[1]
        s[5:10] = 1 / taus[0]
        s[10:] = 1 / taus[3]
        gam = 1 - s
        mu = 3.0 * kT
        fpost = np.zeros_like(f)
        for x, y, z in self._nodes():
            if solid[z, y, x]:
                continue
            node = x + self.nx * (y + self.ny * z)
            zz = self.normals(node, self.step_no) if kT > 0 else np.zeros(36)
            rl = rho[:, z, y, x]
            rtot = rl.sum()
            u = (jm[0, :, z, y, x] + jm[1, :, z, y, x] + 0.5 * (F[0, :, z, y, x] + F[1, :, z, y, x])) / rtot
            ra, rb = max(rl[0], 0.0), max(rl[1], 0.0)
            xid = np.zeros(3)
            if mu > 0 and p["noise_diffusive"] and rtot > 0:
                xid = np.sqrt(mu * B[1] * (1 - gam[1] ** 2) * ra * rb / rtot) * zz[32:35]
            cu = C @ u
            for l in range(2):
                fl = f[l, :, z, y, x]
                Fl = F[l, :, z, y, x]
                feq = W * rl[l] * (1 + 3 * cu + 4.5 * cu * cu - 1.5 * (u @ u))
                guo = W * (3 * ((C - u) @ Fl) + 9 * cu * (C @ Fl))
                m = M @ fl
                ms = m - s * (m - M @ feq) + (1 - s / 2) * (M @ guo)
                ms[1:4] += (1.0 if l == 0 else -1.0) * xid
                if mu > 0:
                    rp = max(rl[l], 0.0)
                    for k in range(4, Q):
                        ms[k] += np.sqrt(mu * rp * B[k] * (1 - gam[k] ** 2)) * zz[16 * l + k - 4]
                fpost[l, :, z, y, x] = MINV @ ms
        # streaming, half-way bounce-back on walls, moving-wall bounce-back on the spheres
        fnew = np.zeros_like(f)
        dp, dl, dMbb = np.zeros((K, 3)), np.zeros((K, 3)), np.zeros(2)
        for x, y, z in self._nodes():
            if solid[z, y, x]:
                continue
            fnew[:, 0, z, y, x] = fpost[:, 0, z, y, x]
            for i in range(1, Q):
                (qx, qy, qz), crossed = self._nb(x, y, z, i)
                if crossed:
                    fnew[:, OPP[i], z, y, x] = fpost[:, i, z, y, x]
                elif solid[qz, qy, qx]:
                    k = owner[qz, qy, qx]
                    sp = self.sph[k]
                    r = self._r(np.array([x, y, z]) + 0.5 * C[i], sp["X"])
                    ub = sp["U"] + np.cross(sp["W"], r)
                    lp = np.zeros(3)
                    for l in range(2):
                        corr = 6 * W[i] * rho[l, z, y, x] * (C[i] @ ub)
                        fnew[l, OPP[i], z, y, x] = fpost[l, i, z, y, x] - corr
                        lp += (2 * fpost[l, i, z, y, x] - corr) * C[i]
                        dMbb[l] -= corr
                    dp[k] += lp
                    dl[k] += np.cross(r, lp)
                else:
                    fnew[:, i, qz, qy, qx] = fpost[:, i, z, y, x]
        # leap-frog Newton-Euler of each sphere
        n3 = (self.nx, self.ny, self.nz)
        for k, sp in enumerate(self.sph):
            Ftot = dp[k] - Fv[k] + Fext[k] + sp["Pev"]
            Ttot = dl[k] - Tv[k] + sp["Lev"]
            if not p["fixed_velocity"]:
                sp["U"] = sp["U"] + Ftot / sp["mp"]
                sp["W"] = sp["W"] + Ttot / sp["Ip"]
            Xn = sp["X"] + sp["U"]
            for a in range(3):
                if not self.walled[a]:
                    if Xn[a] >= n3[a]:
                        Xn[a] -= n3[a]
                    elif Xn[a] < 0:
                        Xn[a] += n3[a]
            sp["X"] = Xn
            sp["F"], sp["T"] = Ftot, Ttot
            sp["Pev"], sp["Lev"] = np.zeros(3), np.zeros(3)
        # cover / uncover against the particle nodes at X^{n+1}: a covered node
        # feeds the sphere now holding it, an uncovered one takes the rigid
        # velocity of the sphere that held it
        onew = self._owner([sp["X"] for sp in self.sph])
        snew = onew >= 0
        dMcov, dMunc = np.zeros(2), np.zeros(2)
        for x, y, z in self._nodes():
            if not solid[z, y, x] and snew[z, y, x]:
                sp = self.sph[onew[z, y, x]]
                j = np.einsum("li,ia->a", fnew[:, :, z, y, x], C.astype(float))
                r = self._r(np.array([x, y, z], dtype=float), sp["X"])
                sp["Pev"] = sp["Pev"] + j
                sp["Lev"] = sp["Lev"] + np.cross(r, j)
                dMcov -= fnew[:, :, z, y, x].sum(axis=1)
                sp["n_cov"] += 1
        for x, y, z in self._nodes():
            if not (solid[z, y, x] and not snew[z, y, x]):
                continue
            sp = self.sph[owner[z, y, x]]
            acc, cnt = np.zeros(2), 0
            for i in range(1, Q):
                (qx, qy, qz), crossed = self._nb(x, y, z, i)
                if crossed or solid[qz, qy, qx] or snew[qz, qy, qx]:
                    continue
                acc += fnew[:, :, qz, qy, qx].sum(axis=1)
                cnt += 1
            rbar = acc / cnt if cnt else np.array(p["rho0"], dtype=float)
            r = self._r(np.array([x, y, z], dtype=float), sp["X"])
            u = sp["U"] + np.cross(sp["W"], r)
            cu = C @ u
            for l in range(2):
                fnew[l, :, z, y, x] = W * rbar[l] * (1 + 3 * cu + 4.5 * cu * cu - 1.5 * (u @ u))
            dMunc += rbar
            mom = rbar.sum() * u
            sp["Pev"] = sp["Pev"] - mom
            sp["Lev"] = sp["Lev"] - np.cross(r, mom)
            sp["n_unc"] += 1
        fnew[:, :, snew] = 0.0
        # global mass correction over the fluid nodes of step n+1
        nf = float((~snew).sum())
        delta = -(dMbb + dMcov + dMunc) / nf
        fnew += (W[None, :, None, None, None] * delta[:, None, None, None, None]) * (~snew)[None, None]
        self.f, self.owner = fnew, onew
        self.step_no += 1
