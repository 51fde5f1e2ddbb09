// Adjoint kernels: reverse-mode derivative of the step (every relaxation
// time 1) with respect to the body force g, the Shan-Chen coupling G and
// the wetting offset Delta rho, for J = time average of U_z^{n+1/2}.
//
// Paper: Xue, Biferale, Sbragaglia, Toschi, "A lattice Boltzmann study of
// particle settling in a fluctuating multicomponent fluid under
// confinement".  Sec. 2: eq. (density), eq. (lbe), eq. (sc-force), the noise
// paragraph (amplitudes sqrt(mu rho_l b_k) on modes 4..18, species-momentum
// noise) and the particle paragraph (moving-wall bounce-back with momentum
// exchange, leap-frog Newton-Euler, cover/uncover, mass correction, virtual
// wetting layer).  Sec. 3, eq. (fp): external force on the sphere.
//
// With every relaxation time 1 the post-collision populations of a node are
// a function of its densities rho_l, momenta j_l and forces F_l only, so the
// adjoint of a state is carried as 8 numbers per node: a population adjoint
// fbar_{l i}(x) = Abar_rho_l(x) + c_i . Abar_j_l(x).  Events, bounce-back,
// wall reflection and the mass correction all keep that form.
//
// The noise normals are a function of (node, step) and are regenerated
// unchanged; particle-node, link and event sets are held fixed (their
// derivative vanishes between events).
//
// One reversed step: k_adj_events and k_adj_kept over the box of X^n (mass
// correction, cover/uncover, wetting-layer densities of step n; then the
// Newton-Euler step back), k_adj_local and k_adj_gather over all nodes
// (collision, force and link adjoints; Shan-Chen gather from the
// neighbours' force adjoints; k_adj_mirror over the walled faces for the
// wall-mirror sources), k_adj_links over the box (moving-wall and
// wetting-reaction terms of the sphere links), and k_adj_chain over the box
// (wetting-layer chain; its last workgroup makes the fixed-order sums into
// the adjoint state).
#include <utility>
#include "lbm_adjoint.h"
#include "lbm_kernels_impl.h"

namespace lbm {
namespace {

constexpr int NB = 256;  // node-kernel block

// f(integral_constant<int, i>) for i = 1 .. Q - 1, in that order
template <typename F, int... I>
__device__ __forceinline__ void for_each_dir(F &&f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I + 1>{}), ...);
}

__device__ __forceinline__ bool solid_at(int x, int y, int z, const RepDesc &D, const int32_t *org,
                                         const double *X, const Geo &g, int &b) {
    b = D.has_particle ? bbox_index(x, y, z, org, D.S, g) : -1;
    return b >= 0 && pnode(x, y, z, X, D.R2, g);
}

// p + c_i inside the lattice (periodic axes wrapped); false across a wall
__device__ __forceinline__ bool step_in(const int (&p)[3], int i, const Geo &g, int (&q)[3]) {
    q[0] = p[0] + cx(i); q[1] = p[1] + cy(i); q[2] = p[2] + cz(i);
    return wrap1(q[0], g.nx, g.wx) && wrap1(q[1], g.ny, g.wy) && wrap1(q[2], g.nz, g.wz);
}

// Node p lies within one node of the box at org (edge S) on every axis: only
// then can p or one of its neighbours be a particle node.
__device__ __forceinline__ bool near_box(const int (&p)[3], const RepDesc &D, const int32_t *org,
                                         const Geo &g) {
    if (!D.has_particle) return false;
    const int n3[3] = {g.nx, g.ny, g.nz};
    const bool w3[3] = {g.wx, g.wy, g.wz};
    for (int ax = 0; ax < 3; ax++) {
        int v = p[ax] - org[ax];
        if (!w3[ax]) {
            v %= n3[ax];
            if (v < 0) v += n3[ax];
            if (v == n3[ax] - 1) v = -1;
        }
        if (v < -1 || v > D.S) return false;
    }
    return true;
}

__device__ __forceinline__ int64_t lin(const int (&q)[3], const Geo &g) {
    return (int64_t)q[0] + (int64_t)g.nx * ((int64_t)q[1] + (int64_t)g.ny * q[2]);
}

__device__ __forceinline__ void cross3(const double *a, const double *b, double *c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

// ============================================================ k_adj_record
// Moments of every node as the main kernel forms them (pulled populations,
// density deviation plus the mass correction) and a copy of the state.
template <typename S, typename T>
__global__ __launch_bounds__(NB) void k_adj_record(RecArgs a) {
    const RepDesc &D = a.desc[0];
    const RepState &st = *a.state;
    const Geo g = geo_of(D);
    const int64_t n = (int64_t)blockIdx.x * NB + threadIdx.x;
    if (n == 0) *a.st_out = st;
    if (n >= g.N) return;
    const int x = (int)(n % g.nx), y = (int)((n / g.nx) % g.ny);
    const int z = (int)(n / ((int64_t)g.nx * g.ny));
    const PullCtx<S, T> pc = pull_ctx<S, T>(a.src, D, g);
    T d[2][Q];
    pull_node(pc, pidx(x, y, z, g), d);
    NodeM<T, true> m;
    node_moments(d, m);
    T *rec = static_cast<T *>(a.rec);
    const int64_t N = g.N;
    rec[n] = m.rd[0] + T(st.delta[0]);
    rec[N + n] = m.rd[1] + T(st.delta[1]);
    for (int q = 0; q < 3; q++) {
        rec[(2 + q) * N + n] = m.j[0][q];
        rec[(5 + q) * N + n] = m.j[1][q];
    }
}

// ============================================================ k_adj_events
// One thread per node of the box of X^n.
//  1. Mass correction: f^{n+1} = fnew + w_i delta_l on the fluid nodes of
//     step n+1, delta_l = -(sum of mass fluxes)_l / |Phi^{n+1}|, so each flux
//     gets the adjoint -sum(Abar_rho) / |Phi^{n+1}|.
//  2. Covered nodes (fluid at X^n, particle at X^{n+1}): their populations
//     only fed Pev += j, Lev += r x j and the mass flux, so their adjoint is
//     Abar_rho_l = -dMb_l, Abar_j = Pevb + Levb x r.
//  3. Uncovered nodes: f_eq(rho_bar, u_b) with u_b = U + Omega x r; by the
//     lattice moments of f_eq the density adjoint is Abar_rho + Abar_j . u_b
//     and the velocity adjoint sum_l rho_bar_l Abar_j_l.  rho_bar is the mean
//     over neighbours fluid at both times: each gets the adjoint / count
//     (gathered by those neighbours in k_adj_kept).
//  Also the wetting-layer densities of step n (mean of fluid neighbours
//  +/- Delta rho) for the node kernels.  Partials: the events' share of the
//  adjoints of U^{n+1/2}, Omega^{n+1/2} and X^{n+1}.
template <typename T>
__global__ __launch_bounds__(NB) void k_adj_events(AdjArgs a) {
    __shared__ double red[(NB / 64) * ADJ_PE];
    const RepDesc D = a.desc[0];
    const RepState sn = *a.stn, s1 = *a.stn1;
    const AdjState ad = *a.adj;
    const Geo g = geo_of(D);
    const int64_t N = g.N;
    const int Sx = D.S, S3 = Sx * Sx * Sx;
    const T *recn = static_cast<const T *>(a.recn);
    const T *rec1 = static_cast<const T *>(a.recn1);
    T *A1 = static_cast<T *>(a.Anext);
    const double nf1 = s1.n_fluid;
    const double dMb[2] = {-ad.dsum[0] / nf1, -ad.dsum[1] / nf1};
    double acc[ADJ_PE];
#pragma unroll
    for (int k = 0; k < ADJ_PE; k++) acc[k] = 0.0;
    const int b = blockIdx.x * NB + threadIdx.x;
    int bb[3], p[3];
    const bool in = b < S3 && bbox_pos(b, sn.org, Sx, g, bb, p);
    if (b < S3) {
        a.ubn[b] = 0.0;
        a.ubn[S3 + b] = 0.0;
        a.vt[b] = 0.0;
        a.vt[S3 + b] = 0.0;
        a.vinv[b] = 0.0;
    }
    const bool so = in && pnode(p[0], p[1], p[2], sn.X, D.R2, g);
    const bool sn1 = in && pnode(p[0], p[1], p[2], s1.X, D.R2, g);
    const int64_t m = in ? lin(p, g) : 0;
    if (so) {
        double s0 = 0.0, s1v = 0.0;
        int cnt = 0;
#pragma unroll
        for (int i = 1; i < Q; i++) {
            int q[3];
            if (!step_in(p, i, g, q) || pnode(q[0], q[1], q[2], sn.X, D.R2, g)) continue;
            const int64_t qi = lin(q, g);
            s0 += D.rho0[0] + (double)recn[qi];
            s1v += D.rho0[1] + (double)recn[N + qi];
            cnt++;
        }
        if (cnt > 0) {
            a.vt[b] = s0 / cnt + D.drho;
            a.vt[S3 + b] = s1v / cnt - D.drho;
            a.vinv[b] = 1.0 / cnt;
        }
    }
    if (in && !so && sn1) {  // covered
        const double r[3] = {sepd(p[0] - s1.X[0], g.nx, g.wx), sepd(p[1] - s1.X[1], g.ny, g.wy),
                             sepd(p[2] - s1.X[2], g.nz, g.wz)};
        double jv[3], Jb[3], c[3];
        for (int q = 0; q < 3; q++) jv[q] = (double)rec1[(2 + q) * N + m] + (double)rec1[(5 + q) * N + m];
        cross3(ad.Levb, r, c);
        for (int q = 0; q < 3; q++) Jb[q] = ad.Pevb[q] + c[q];
        A1[m] = T(-dMb[0]);
        A1[N + m] = T(-dMb[1]);
        for (int q = 0; q < 3; q++) {
            A1[(2 + q) * N + m] = T(Jb[q]);
            A1[(5 + q) * N + m] = T(Jb[q]);
        }
        cross3(jv, ad.Levb, c);
        for (int q = 0; q < 3; q++) acc[6 + q] -= c[q];
    }
    if (so && !sn1) {  // uncovered
        const double r[3] = {sepd(p[0] - s1.X[0], g.nx, g.wx), sepd(p[1] - s1.X[1], g.ny, g.wy),
                             sepd(p[2] - s1.X[2], g.nz, g.wz)};
        const double rb[2] = {D.rho0[0] + (double)rec1[m] - s1.delta[0],
                              D.rho0[1] + (double)rec1[N + m] - s1.delta[1]};
        double u[3], c[3];
        cross3(s1.W, r, c);
        for (int q = 0; q < 3; q++) u[q] = s1.U[q] + c[q];
        double Ar[2], Aj[2][3];
        for (int l = 0; l < 2; l++) {
            Ar[l] = (double)A1[l * N + m];
            for (int q = 0; q < 3; q++) Aj[l][q] = (double)A1[(2 + 3 * l + q) * N + m];
        }
        // Pev -= mom, Lev -= r x mom, mom = (rb_A + rb_B) u_b
        double mb[3];
        cross3(ad.Levb, r, c);
        for (int q = 0; q < 3; q++) mb[q] = -(ad.Pevb[q] + c[q]);
        const double um = u[0] * mb[0] + u[1] * mb[1] + u[2] * mb[2];
        double rbb[2], ub[3];
        for (int l = 0; l < 2; l++)
            rbb[l] = Ar[l] + (Aj[l][0] * u[0] + Aj[l][1] * u[1] + Aj[l][2] * u[2]) + dMb[l] + um;
        for (int q = 0; q < 3; q++) ub[q] = rb[0] * Aj[0][q] + rb[1] * Aj[1][q] + (rb[0] + rb[1]) * mb[q];
        for (int q = 0; q < 3; q++) acc[q] += ub[q];
        cross3(r, ub, c);
        for (int q = 0; q < 3; q++) acc[3 + q] += c[q];
        // lever arm r = p - X^{n+1}: d/dr of u_b and of r x mom
        double mom[3], c2[3];
        for (int q = 0; q < 3; q++) mom[q] = (rb[0] + rb[1]) * u[q];
        cross3(ub, s1.W, c);
        cross3(mom, ad.Levb, c2);
        for (int q = 0; q < 3; q++) acc[6 + q] -= c[q] - c2[q];
        int cnt = 0;
        for (int i = 1; i < Q; i++) {
            int q[3];
            if (!step_in(p, i, g, q)) continue;
            if (pnode(q[0], q[1], q[2], sn.X, D.R2, g) || pnode(q[0], q[1], q[2], s1.X, D.R2, g)) continue;
            cnt++;
        }
        if (cnt > 0) {
            a.ubn[b] = rbb[0] / cnt;
            a.ubn[S3 + b] = rbb[1] / cnt;
        }
    }
    block_sum<NB, ADJ_PE>(acc, red);
    if (threadIdx.x == 0)
        for (int k = 0; k < ADJ_PE; k++) a.partE[(int64_t)blockIdx.x * PART + k] = acc[k];
}

// ============================================================== k_adj_kept
// One thread per box node: nodes fluid at both times collect the
// uncovered-node adjoints of their neighbours.  The first wave of workgroup
// 0 then sums the event partials (fixed order) and takes the Newton-Euler
// step back: U^{n+1/2} = U^{n-1/2} + F/m_p, Omega likewise with T/I_p,
// X^{n+1} = X^n + U^{n+1/2}; J picks U_z^{n+1/2}.
template <typename T>
__global__ __launch_bounds__(NB) void k_adj_kept(AdjArgs a) {
    const RepDesc D = a.desc[0];
    const RepState sn = *a.stn, s1 = *a.stn1;
    const Geo g = geo_of(D);
    const int64_t N = g.N;
    const int Sx = D.S, S3 = Sx * Sx * Sx;
    T *A1 = static_cast<T *>(a.Anext);
    const int b = blockIdx.x * NB + threadIdx.x;
    int bb[3], p[3];
    const bool in = b < S3 && bbox_pos(b, sn.org, Sx, g, bb, p);
    if (in && !pnode(p[0], p[1], p[2], sn.X, D.R2, g) && !pnode(p[0], p[1], p[2], s1.X, D.R2, g)) {
        double s[2] = {0.0, 0.0};
        bool any = false;
#pragma unroll
        for (int i = 1; i < Q; i++) {
            int q[3];
            if (!step_in(p, i, g, q)) continue;
            const int bq = bbox_index(q[0], q[1], q[2], sn.org, Sx, g);
            if (bq < 0) continue;
            const double u0 = a.ubn[bq], u1 = a.ubn[S3 + bq];
            if (u0 != 0.0 || u1 != 0.0) {
                s[0] += u0;
                s[1] += u1;
                any = true;
            }
        }
        if (any) {
            const int64_t m = lin(p, g);
            A1[m] = T((double)A1[m] + s[0]);
            A1[N + m] = T((double)A1[N + m] + s[1]);
        }
    }
    if (blockIdx.x != 0 || threadIdx.x >= 64) return;
    double ev[ADJ_PE];
    sum_partials<ADJ_PE>(a.partE, a.nbw, 0, ev);
    if (threadIdx.x != 0) return;
    const AdjState ad = *a.adj;
    AdjState *o = a.adj;
    double Ub1[3], Wb1[3], Xb1[3], Fb[3], Tb[3];
    for (int q = 0; q < 3; q++) {
        Xb1[q] = ad.Xb[q] + ev[6 + q];
        Ub1[q] = ad.Ub[q] + ev[q] + Xb1[q] + (q == 2 ? a.invN : 0.0);
        Wb1[q] = ad.Wb[q] + ev[3 + q];
        Fb[q] = D.fixed_velocity ? 0.0 : Ub1[q] / D.mp;
        Tb[q] = D.fixed_velocity ? 0.0 : Wb1[q] / D.Ip;
    }
    for (int q = 0; q < 3; q++) {
        o->Ub[q] = Ub1[q];
        o->Wb[q] = Wb1[q];
        o->Xb[q] = Xb1[q];
        o->Pevb[q] = Fb[q];
        o->Levb[q] = Tb[q];
        o->Fb[q] = Fb[q];
        o->Tb[q] = Tb[q];
        o->grad[q] = ad.grad[q] + a.cF * Fb[q];
    }
    const double nf1 = s1.n_fluid;
    o->dMb[0] = -ad.dsum[0] / nf1;
    o->dMb[1] = -ad.dsum[1] / nf1;
    o->Jsum = ad.Jsum + s1.U[2];
}

// ============================================================ node adjoint
// Forward values of a fluid node at step n rebuilt from the recorded
// moments: densities, momenta, forces (from the neighbours' densities seen
// by the force), velocity and species-momentum noise as the main kernel
// forms them; plus which links leave through a wall or into the sphere.

// nbr(i, rt) gives the densities the force reads at the neighbour along c_i
// (wrapped on periodic axes, clamped onto the lattice across a wall; the
// wetting layer's on particle nodes).
template <typename T, typename NbrRt>
__device__ __forceinline__ void node_forward(const AdjArgs &a, const RepDesc &D, const RepState &sn,
                                             const Geo &g, const int (&p)[3], int64_t n, bool near,
                                             const Coef<T> &cf, NodeFwd<T> &f, NbrRt &&nbr) {
    const int64_t N = g.N;
    const T *rec = static_cast<const T *>(a.recn);
    for (int l = 0; l < 2; l++) {
        f.rd[l] = rec[l * N + n];
        f.rl[l] = T(D.rho0[l]) + f.rd[l];
        for (int q = 0; q < 3; q++) f.jl[l][q] = rec[(2 + 3 * l + q) * N + n];
    }
    for (int l = 0; l < 2; l++)
        for (int q = 0; q < 3; q++) f.sv[l][q] = T(0);
    f.wall = 0;
    f.link = 0;
    const int n3[3] = {g.nx, g.ny, g.nz};
    const bool w3[3] = {g.wx, g.wy, g.wz};
#pragma unroll
    for (int i = 1; i < Q; i++) {
        const int c3[3] = {cx(i), cy(i), cz(i)};
        int m3[3];
        bool out = false;
        for (int ax = 0; ax < 3; ax++) {
            int v = p[ax] + c3[ax];
            if (v < 0 || v >= n3[ax]) {
                if (w3[ax]) { out = true; v = v < 0 ? 0 : n3[ax] - 1; }
                else v = v < 0 ? v + n3[ax] : v - n3[ax];
            }
            m3[ax] = v;
        }
        int bm = -1;
        const bool ms = near && solid_at(m3[0], m3[1], m3[2], D, sn.org, sn.X, g, bm);
        T rt[2];
        nbr(i, rt);
        const T w = T(wgt(i));
        for (int l = 0; l < 2; l++)
            for (int q = 0; q < 3; q++)
                if (c3[q]) f.sv[l][q] += c3[q] > 0 ? w * rt[l] : -(w * rt[l]);
        if (out) f.wall |= 1u << i;
        else if (ms) f.link |= 1u << i;
    }
    const T G = T(D.G);
    for (int q = 0; q < 3; q++) {
        f.F[0][q] = -G * f.rl[0] * f.sv[1][q] + f.rl[0] * T(D.af[q]);
        f.F[1][q] = -G * f.rl[1] * f.sv[0][q] + f.rl[1] * T(D.af[q]);
    }
    for (int k = 0; k < 4; k++) f.zd[k] = T(0);
    if (cf.noise) noise_block<T>((uint32_t)n, (uint32_t)sn.step, 8u, D.key0, D.key1, f.zd);
    const T inv = recip(f.rl[0] + f.rl[1]);
    for (int q = 0; q < 3; q++) f.u[q] = (f.jl[0][q] + f.jl[1][q] + T(0.5) * (f.F[0][q] + f.F[1][q])) * inv;
    f.ampf = (cf.noise && cf.diffusive) ? cf.ampd * sqrt(tmax0(f.rl[0]) * tmax0(f.rl[1]) * inv) : T(0);
    for (int q = 0; q < 3; q++) f.xid[q] = f.ampf * f.zd[q];
}

template <typename T>
__device__ __forceinline__ void comp_noise(const RepDesc &D, const RepState &sn, int64_t n, int l,
                                           const Coef<T> &cf, T (&zl)[16]) {
    if (cf.noise) {
#pragma unroll
        for (int b4 = 0; b4 < 4; b4++)
            noise_block<T>((uint32_t)n, (uint32_t)sn.step, (uint32_t)(4 * l + b4), D.key0, D.key1, zl + 4 * b4);
    } else {
#pragma unroll
        for (int k = 0; k < 16; k++) zl[k] = T(0);
    }
}

// Collision adjoint of one component (every relaxation time 1): from the
// adjoint fpb of its post-collision populations to the adjoints of its
// density (rbl), force (Fbl), and contributions to the velocity (ub) and
// species-momentum noise (xb) adjoints.  Mode adjoints
// Mb_k = (1/b_k) sum_i w_i e_k(c_i) fpb_i; modes 4..9 hold
// r u^T K u / 2 + u^T K F / 2 with K symmetric; noise sqrt(mu rho_l b_k) z.
template <typename T>
__device__ __forceinline__ void comp_adjoint(const NodeFwd<T> &f, int l, const T (&fpb)[Q],
                                             const T (&zl)[16], const Coef<T> &cf, T &rbl, T (&Fbl)[3],
                                             T (&ub)[3], T (&xb)[3]) {
    const T rll = l ? f.rl[1] : f.rl[0];
    const T Fl[3] = {l ? f.F[1][0] : f.F[0][0], l ? f.F[1][1] : f.F[0][1], l ? f.F[1][2] : f.F[0][2]};
    const T sig = l ? T(-1) : T(1);
    const T *u = f.u;
    T gw[Q];
#pragma unroll
    for (int i = 0; i < Q; i++) gw[i] = T(wgt(i)) * fpb[i];
    T a0, aj[3], am[Q];
    component_modes(gw, a0, aj, am);
    const T Jb[3] = {T(3) * aj[0], T(3) * aj[1], T(3) * aj[2]};
    const T M4 = T(inv_norm(4)) * am[4], M5 = T(inv_norm(5)) * am[5], M6 = T(inv_norm(6)) * am[6];
    const T M7 = T(inv_norm(7)) * am[7], M8 = T(inv_norm(8)) * am[8], M9 = T(inv_norm(9)) * am[9];
    const T Kxx = T(2) * M4 + T(4) * M5, Kyy = T(2) * M4 - T(2) * M5 + T(2) * M6;
    const T Kzz = T(2) * M4 - T(2) * M5 - T(2) * M6;
    const T Kxy = M7, Kyz = M8, Kxz = M9;
    const T Ku[3] = {Kxx * u[0] + Kxy * u[1] + Kxz * u[2], Kxy * u[0] + Kyy * u[1] + Kyz * u[2],
                     Kxz * u[0] + Kyz * u[1] + Kzz * u[2]};
    const T KF[3] = {Kxx * Fl[0] + Kxy * Fl[1] + Kxz * Fl[2], Kxy * Fl[0] + Kyy * Fl[1] + Kyz * Fl[2],
                     Kxz * Fl[0] + Kyz * Fl[1] + Kzz * Fl[2]};
    rbl = a0 + (u[0] * Jb[0] + u[1] * Jb[1] + u[2] * Jb[2]) +
          T(0.5) * (u[0] * Ku[0] + u[1] * Ku[1] + u[2] * Ku[2]);
    for (int q = 0; q < 3; q++) {
        ub[q] += rll * (Jb[q] + Ku[q]) + T(0.5) * KF[q];
        Fbl[q] = T(0.5) * (Jb[q] + Ku[q]);
        xb[q] += sig * Jb[q];
    }
    if (cf.noise && rll > T(0)) {
        const T sqmu[3] = {cf.nb, cf.ns, cf.ng};
        T s = T(0);
#pragma unroll
        for (int k = 4; k < Q; k++) {
            const T sm = k == 4 ? sqmu[0] : (k <= 9 ? sqmu[1] : sqmu[2]);
            s += T(inv_norm(k) * sqrt_norm(k)) * am[k] * sm * zl[k - 4];
        }
        rbl += s / (T(2) * sqrt(rll));
    }
}

// Rest of the node adjoint (linear in its inputs): species-momentum noise
// amp z_{32+a} with amp = ampd sqrt(rho_A rho_B / rho), the velocity
// u = (j_A + j_B + (F_A + F_B)/2) / rho, and the node-local part of the
// force F_l = -G rho_l s_l' + rho_l a_f.  Outputs the density and momentum
// adjoints; acc gets the G and a_f adjoints.
template <typename T>
__device__ __forceinline__ void node_finish(const NodeFwd<T> &f, const RepDesc &D, const Coef<T> &cf,
                                            T (&rb)[2], T (&Fbv)[2][3], const T (&ub)[3], const T (&xb)[3],
                                            T (&jb)[3], double *acc) {
    const T rho = f.rl[0] + f.rl[1];
    if (cf.noise && cf.diffusive && f.rl[0] > T(0) && f.rl[1] > T(0)) {
        const T ab = xb[0] * f.zd[0] + xb[1] * f.zd[1] + xb[2] * f.zd[2];
        rb[0] += ab * f.ampf * f.rl[1] / (T(2) * f.rl[0] * rho);
        rb[1] += ab * f.ampf * f.rl[0] / (T(2) * f.rl[1] * rho);
    }
    const T ubu = (ub[0] * f.u[0] + ub[1] * f.u[1] + ub[2] * f.u[2]) / rho;
    for (int q = 0; q < 3; q++) jb[q] = ub[q] / rho;
    for (int l = 0; l < 2; l++) {
        rb[l] -= ubu;
        for (int q = 0; q < 3; q++) Fbv[l][q] += T(0.5) * jb[q];
    }
    const T G = T(D.G);
    for (int l = 0; l < 2; l++) {
        const T *so = f.sv[1 - l];
        rb[l] += Fbv[l][0] * (T(D.af[0]) - G * so[0]) + Fbv[l][1] * (T(D.af[1]) - G * so[1]) +
                 Fbv[l][2] * (T(D.af[2]) - G * so[2]);
        acc[0] += -(double)f.rl[l] * ((double)Fbv[l][0] * (double)so[0] + (double)Fbv[l][1] * (double)so[1] +
                                      (double)Fbv[l][2] * (double)so[2]);
        for (int q = 0; q < 3; q++) acc[1 + q] += (double)f.rl[l] * (double)Fbv[l][q];
    }
}

// ============================================================ k_adj_local
// Tile = ty full x-rows of one plane z.  The densities the force reads
// (recorded, or the wetting layer's on particle nodes) and the adjoint state
// after the step (8 values) of the tile plus a one-node halo (rows y0-1 and
// y0+rows, planes z-1 and z+1; mirrored across walls, wrapped on periodic
// axes) are staged in LDS, so a node's 18-neighbour gathers read LDS.  Per
// fluid node: the adjoint of f*_i(x) from where streaming took it (a
// neighbour's Abar; the node's own reflected Abar for links through a wall
// or into the sphere, whose moving-wall terms k_adj_links adds), then the
// collision and node-local force adjoints.
// FP32: held to 128 VGPRs (four waves per SIMD).
constexpr int LV = 10;  // staged values per node: rt_A, rt_B, Abar_rho_A, Abar_rho_B, Abar_j_A (3), Abar_j_B (3)

template <typename T>
__global__ __launch_bounds__(NB) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 1))) void k_adj_local(AdjArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[(NB / 64) * ADJ_PA];
    T *lds = reinterpret_cast<T *>(smem);
    const RepDesc D = a.desc[0];
    const RepState sn = *a.stn;
    const Geo g = geo_of(D);
    const int64_t N = g.N;
    const int nx = g.nx, ty = a.lty, nty = (g.ny + ty - 1) / ty;
    const int yt = blockIdx.x % nty, z = blockIdx.x / nty;
    const int y0 = yt * ty, rows = min(ty, g.ny - y0);
    const int t = threadIdx.x, nin = nx * rows;
    const bool inner = t < nin;
    const int x = inner ? t % nx : 0, yl = inner ? t / nx : 0, y = y0 + yl;
    const int pr = (ty + 2) * nx;  // LDS elements per plane and staged value
    const T *rec = static_cast<const T *>(a.recn);
    const T *A1 = static_cast<const T *>(a.Anext);
    // slot dz + 1 holds plane z + dz
    auto L = [&](int dz, int v, int row, int xx) -> T & {
        return lds[((dz + 1) * LV + v) * pr + (row + 1) * nx + xx];
    };
    {
        // stage planes z - 1, z, z + 1: rows -1 .. rows of the tile, every x
        const int S3 = D.S * D.S * D.S;
        const int per = (rows + 2) * nx;
        for (int e = t; e < 3 * per; e += NB) {
            const int dz = e / per - 1, r = e % per;
            const int row = r / nx - 1, xx = r % nx;
            const int q[3] = {xx, mirror1(y0 + row, g.ny, g.wy), mirror1(z + dz, g.nz, g.wz)};
            const int64_t m = lin(q, g);
            int bm = -1;
            const bool ms = near_box(q, D, sn.org, g) && solid_at(q[0], q[1], q[2], D, sn.org, sn.X, g, bm);
            L(dz, 0, row, xx) = ms ? T(a.vt[bm] - D.rho0[0]) : rec[m];
            L(dz, 1, row, xx) = ms ? T(a.vt[S3 + bm] - D.rho0[1]) : rec[N + m];
#pragma unroll
            for (int k = 0; k < 8; k++) L(dz, 2 + k, row, xx) = A1[k * N + m];
        }
    }
    __syncthreads();
    double acc[ADJ_PA];
#pragma unroll
    for (int k = 0; k < ADJ_PA; k++) acc[k] = 0.0;
    T *A0 = static_cast<T *>(a.Acur);
    T *Fo = static_cast<T *>(a.Fb);
    const int p[3] = {x, y, z};
    const int64_t n = lin(p, g);
    int bs = -1;
    const bool near = inner && near_box(p, D, sn.org, g);
    const bool solid = near && solid_at(x, y, z, D, sn.org, sn.X, g, bs);
    if (inner && solid) {
        for (int k = 0; k < 8; k++) A0[k * N + n] = T(0);
        for (int k = 0; k < 6; k++) Fo[k * N + n] = T(0);
    }
    if (inner && !solid) {
        const int xm = mirror1(x - 1, nx, g.wx), xp = mirror1(x + 1, nx, g.wx);
        const Coef<T> cf = make_coef_dev<T>(D);
        NodeFwd<T> f;
        node_forward(a, D, sn, g, p, n, near, cf, f, [&](int i, T (&rt)[2]) {
            const int xx = cx(i) > 0 ? xp : (cx(i) < 0 ? xm : x);
            rt[0] = L(cz(i), 0, yl + cy(i), xx);
            rt[1] = L(cz(i), 1, yl + cy(i), xx);
        });
        if (f.link) static_cast<NodeFwd<T> *>(a.nfw)[bbox_index(x, y, z, sn.org, D.S, g)] = f;
        T rb[2], Fbv[2][3];
        T ub[3] = {T(0), T(0), T(0)}, xb[3] = {T(0), T(0), T(0)};
#pragma unroll 1
        for (int l = 0; l < 2; l++) {
            T zl[16];
            comp_noise(D, sn, n, l, cf, zl);
            const T Ar = L(0, 2 + l, yl, x);
            const T Aj[3] = {L(0, 4 + 3 * l, yl, x), L(0, 5 + 3 * l, yl, x), L(0, 6 + 3 * l, yl, x)};
            T fpb[Q];
            fpb[0] = Ar;
#pragma unroll
            for (int i = 1; i < Q; i++) {
                if ((f.wall | f.link) >> i & 1u) {
                    fpb[i] = Ar - (T(cx(i)) * Aj[0] + T(cy(i)) * Aj[1] + T(cz(i)) * Aj[2]);
                    continue;
                }
                const int xx = cx(i) > 0 ? xp : (cx(i) < 0 ? xm : x);
                const int rt = yl + cy(i);
                T v = L(cz(i), 2 + l, rt, xx);
                if (cx(i)) v += cx(i) > 0 ? L(cz(i), 4 + 3 * l, rt, xx) : -L(cz(i), 4 + 3 * l, rt, xx);
                if (cy(i)) v += cy(i) > 0 ? L(cz(i), 5 + 3 * l, rt, xx) : -L(cz(i), 5 + 3 * l, rt, xx);
                if (cz(i)) v += cz(i) > 0 ? L(cz(i), 6 + 3 * l, rt, xx) : -L(cz(i), 6 + 3 * l, rt, xx);
                fpb[i] = v;
            }
            T rbl, Fbl[3];
            comp_adjoint(f, l, fpb, zl, cf, rbl, Fbl, ub, xb);
            if (l) {
                rb[1] = rbl;
                for (int q = 0; q < 3; q++) Fbv[1][q] = Fbl[q];
            } else {
                rb[0] = rbl;
                for (int q = 0; q < 3; q++) Fbv[0][q] = Fbl[q];
            }
        }
        T jb[3];
        node_finish(f, D, cf, rb, Fbv, ub, xb, jb, acc);
        for (int l = 0; l < 2; l++) {
            A0[l * N + n] = rb[l];
            for (int q = 0; q < 3; q++) {
                A0[(2 + 3 * l + q) * N + n] = jb[q];
                Fo[(3 * l + q) * N + n] = f.rl[l] * Fbv[l][q];
            }
        }
    }
    block_sum<NB, ADJ_PA>(acc, red);
    if (threadIdx.x == 0)
        for (int k = 0; k < ADJ_PA; k++) a.partA[(int64_t)blockIdx.x * ADJ_PA + k] = acc[k];
}

// ============================================================ k_adj_links
// Two lanes per box node fluid at X^n with links into the sphere, one per
// component.  For a link i: f_opp(i)(x) = f*_i(x) - 6 w_i rho_l (c_i . u_b),
// u_b = U + Omega x d (d = x - X^n; c_i . (Omega x c_i) = 0), exchanged
// momentum (2 f*_i - 6 w_i rho_l c_i . u_b) c_i with torque about X^n,
// bounce-back mass flux, and the wetting-layer reaction
// -G rho_l w_i rho~_l'(x + c_i) c_i on the sphere.  k_adj_local took the
// reflected Abar for f*_i (and left the node's rebuilt forward values in the
// box array); the rest of its adjoint (2 q, q = c_i . (Fbar + Tbar x d)) goes
// through the same node adjoint here, which is linear: each lane applies it
// to its component's share and the pair's sums are added to the node's
// outputs, with the density adjoint of the link terms and the sphere
// adjoints.
template <typename T>
__global__ __launch_bounds__(NB) void k_adj_links(AdjArgs a) {
    __shared__ double red[(NB / 64) * ADJ_PA];
    const RepDesc D = a.desc[0];
    const RepState sn = *a.stn;
    const AdjState ad = *a.adj;
    const Geo g = geo_of(D);
    const int64_t N = g.N;
    const int Sx = D.S, S3 = Sx * Sx * Sx;
    const T *A1 = static_cast<const T *>(a.Anext);
    T *A0 = static_cast<T *>(a.Acur);
    T *Fo = static_cast<T *>(a.Fb);
    double acc[ADJ_PA];
#pragma unroll
    for (int k = 0; k < ADJ_PA; k++) acc[k] = 0.0;
    const int tid = blockIdx.x * NB + threadIdx.x;
    const int b = tid >> 1, l = tid & 1;
    int bb[3], p[3];
    const bool in = b < S3 && bbox_pos(b, sn.org, Sx, g, bb, p);
    // links of a fluid node (the predicate combined as pnode combines it)
    uint32_t lk = 0;
    if (in) {
        Nbr nb;
        nbr_of(p, sn.X, D.R2, g, nb);
        if (!pnode_nb(nb, 0))
            for (int i = 1; i < Q; i++)
                if (nbr_ok(nb, i) && pnode_nb(nb, i)) lk |= 1u << i;
    }
    if (lk) {  // both lanes of the pair
        const int64_t n = lin(p, g);
        const Coef<T> cf = make_coef_dev<T>(D);
        // forward values of this node as k_adj_local rebuilt them
        const NodeFwd<T> f = static_cast<const NodeFwd<T> *>(a.nfw)[b];
        const double d3[3] = {sepd(p[0] - sn.X[0], g.nx, g.wx), sepd(p[1] - sn.X[1], g.ny, g.wy),
                              sepd(p[2] - sn.X[2], g.nz, g.wz)};
        double V[3], TxD[3];
        cross3(sn.W, d3, V);
        for (int q = 0; q < 3; q++) V[q] += sn.U[q];
        cross3(ad.Tb, d3, TxD);
        T zl[16];
        comp_noise(D, sn, n, l, cf, zl);
        const T jc[3] = {l ? f.jl[1][0] : f.jl[0][0], l ? f.jl[1][1] : f.jl[0][1], l ? f.jl[1][2] : f.jl[0][2]};
        const T Fc[3] = {l ? f.F[1][0] : f.F[0][0], l ? f.F[1][1] : f.F[0][1], l ? f.F[1][2] : f.F[0][2]};
        const T rdl = l ? f.rd[1] : f.rd[0];
        T fo[Q];
        relax_tau1(T(l ? D.rho0[1] : D.rho0[0]), l ? T(-1) : T(1), rdl, jc, Fc, f.u, f.xid, zl, cf, fo);
        const T Ar = A1[l * N + n];
        const T Aj[3] = {A1[(2 + 3 * l) * N + n], A1[(3 + 3 * l) * N + n], A1[(4 + 3 * l) * N + n]};
        const double rld = (double)(l ? f.rl[1] : f.rl[0]);
        const double dMbl = l ? ad.dMb[1] : ad.dMb[0];
        const double r0l = l ? D.rho0[1] : D.rho0[0];
        double rlkl = 0.0;
        T dfp[Q];
#pragma unroll
        for (int i = 0; i < Q; i++) dfp[i] = T(0);
#pragma unroll 1
        for (int i = 1; i < Q; i++) {
            if (!(f.link >> i & 1u)) continue;
            const double c3[3] = {(double)cx(i), (double)cy(i), (double)cz(i)};
            int q3[3];
            step_in(p, i, g, q3);
            const int bm = bbox_index(q3[0], q3[1], q3[2], sn.org, Sx, g);
            const double vo = a.vt[(1 - l) * S3 + bm];
            const double cu = c3[0] * V[0] + c3[1] * V[1] + c3[2] * V[2];
            const double qv = c3[0] * (ad.Fb[0] + TxD[0]) + c3[1] * (ad.Fb[1] + TxD[1]) +
                              c3[2] * (ad.Fb[2] + TxD[2]);
            const double fs = wgt(i) * r0l + (double)fo[i];
            const double corr = 6.0 * wgt(i) * rld * cu;
            const double lpm = 2.0 * fs - corr;
            const double al = (double)Ar - (c3[0] * (double)Aj[0] + c3[1] * (double)Aj[1] +
                                            c3[2] * (double)Aj[2]);
            dfp[i] = T(2.0 * qv);
            const double corrb = -al - qv - dMbl;
            const double cub = 6.0 * wgt(i) * rld * corrb;
            const double flm = -D.G * rld * wgt(i) * vo;
            rlkl += 6.0 * wgt(i) * cu * corrb + D.G * wgt(i) * vo * qv;
            acc[0] += rld * wgt(i) * vo * qv;
            double cW[3], cT[3], dc[3];
            cross3(c3, sn.W, cW);
            cross3(c3, ad.Tb, cT);
            cross3(d3, c3, dc);
            for (int q = 0; q < 3; q++) {
                acc[4 + q] += cub * c3[q];
                acc[7 + q] += cub * dc[q];
                acc[10 + q] += -(cub * cW[q] + lpm * cT[q]) + flm * cT[q];
            }
        }
        T rbl, Fbl[3];
        T ub[3] = {T(0), T(0), T(0)}, xb[3] = {T(0), T(0), T(0)};
        comp_adjoint(f, l, dfp, zl, cf, rbl, Fbl, ub, xb);
        // this lane's share of the node adjoint (the other component's inputs are zero)
        T rb[2] = {l ? T(0) : rbl, l ? rbl : T(0)};
        T Fbv[2][3];
        for (int q = 0; q < 3; q++) {
            Fbv[0][q] = l ? T(0) : Fbl[q];
            Fbv[1][q] = l ? Fbl[q] : T(0);
        }
        T jb[3];
        node_finish(f, D, cf, rb, Fbv, ub, xb, jb, acc);
        double out[13];
        out[0] = (double)rb[0] + (l ? 0.0 : rlkl);
        out[1] = (double)rb[1] + (l ? rlkl : 0.0);
        for (int q = 0; q < 3; q++) {
            out[2 + q] = (double)jb[q];
            out[5 + q] = (double)Fbv[0][q];
            out[8 + q] = (double)Fbv[1][q];
        }
        for (int k = 0; k < 11; k++) out[k] += __shfl_xor(out[k], 1);
        if (l == 0) {
            for (int c = 0; c < 2; c++) {
                A0[c * N + n] = T((double)A0[c * N + n] + out[c]);
                for (int q = 0; q < 3; q++) {
                    A0[(2 + 3 * c + q) * N + n] += T(out[2 + q]);
                    Fo[(3 * c + q) * N + n] += f.rl[c] * T(out[5 + 3 * c + q]);
                }
            }
        }
    }
    block_sum<NB, ADJ_PA>(acc, red);
    if (threadIdx.x == 0)
        for (int k = 0; k < ADJ_PA; k++) a.partL[(int64_t)blockIdx.x * PART + k] = acc[k];
}

// =========================================================== k_adj_gather
// One thread per node y.  F_l(x) reads rho~_l'(m_i(x)), m_i(x) = x + c_i
// wrapped, or clamped onto the box across a wall; so y collects
// -G rho_l(x) w_i c_i . Fbar_l(x) from every fluid x with m_i(x) = y.  Here
// the plain sources x = y - c_i; k_adj_mirror adds those whose x + c_i left
// the box through a wall next to y.  Particle nodes y also collect the
// wetting-layer reaction of their links (adjoint -q along c_i) and store the
// sum for the chain to their fluid neighbours.
template <typename T>
__global__ __launch_bounds__(NB) void k_adj_gather(AdjArgs a) {
    __shared__ double red[(NB / 64) * ADJ_PB];
    const RepDesc D = a.desc[0];
    const RepState sn = *a.stn;
    const AdjState ad = *a.adj;
    const Geo g = geo_of(D);
    const int64_t N = g.N;
    const int S3 = D.S * D.S * D.S;
    const int64_t n = (int64_t)blockIdx.x * NB + threadIdx.x;
    const T *rec = static_cast<const T *>(a.recn);
    const T *Fb = static_cast<const T *>(a.Fb);
    T *A0 = static_cast<T *>(a.Acur);
    double acc[ADJ_PB] = {0.0, 0.0};
    if (n < N) {
        const int p[3] = {(int)(n % g.nx), (int)((n / g.nx) % g.ny), (int)(n / ((int64_t)g.nx * g.ny))};
        int bs = -1;
        const bool near = near_box(p, D, sn.org, g);
        const bool solid = near && solid_at(p[0], p[1], p[2], D, sn.org, sn.X, g, bs);
        const int n3[3] = {g.nx, g.ny, g.nz};
        const bool w3[3] = {g.wx, g.wy, g.wz};
        const T G = T(D.G);
        T s[2] = {T(0), T(0)};
        double lk[2] = {0.0, 0.0};
        // sources x of y for direction i, per axis: the plain one y - c (wrapped
        // on periodic axes; inside the box on walled ones) and, on a walled face
        // that c points out of, y itself (x + c left the box and was clamped)
        auto source = [&](int i, const int (&xs)[3], bool mirrored) {
            int bx;
            if (near && solid_at(xs[0], xs[1], xs[2], D, sn.org, sn.X, g, bx)) return;
            const int64_t si = lin(xs, g);
            const T w = T(wgt(i));
            // Fb holds rho_l(x) times the force adjoint of x
            T cFA = T(0), cFB = T(0);
            if (cx(i)) { cFA += cx(i) > 0 ? Fb[si] : -Fb[si]; cFB += cx(i) > 0 ? Fb[3 * N + si] : -Fb[3 * N + si]; }
            if (cy(i)) { cFA += cy(i) > 0 ? Fb[N + si] : -Fb[N + si]; cFB += cy(i) > 0 ? Fb[4 * N + si] : -Fb[4 * N + si]; }
            if (cz(i)) { cFA += cz(i) > 0 ? Fb[2 * N + si] : -Fb[2 * N + si]; cFB += cz(i) > 0 ? Fb[5 * N + si] : -Fb[5 * N + si]; }
            // F_A(x) reads rho~_B(y), F_B(x) reads rho~_A(y)
            s[1] += -G * w * cFA;
            s[0] += -G * w * cFB;
            if (solid && !mirrored) {
                const T rA = T(D.rho0[0]) + rec[si], rB = T(D.rho0[1]) + rec[N + si];
                const double d3[3] = {sepd(xs[0] - sn.X[0], g.nx, g.wx), sepd(xs[1] - sn.X[1], g.ny, g.wy),
                                      sepd(xs[2] - sn.X[2], g.nz, g.wz)};
                double TxD[3];
                cross3(ad.Tb, d3, TxD);
                const double qv = cx(i) * (ad.Fb[0] + TxD[0]) + cy(i) * (ad.Fb[1] + TxD[1]) +
                                  cz(i) * (ad.Fb[2] + TxD[2]);
                lk[1] += D.G * (double)rA * wgt(i) * qv;
                lk[0] += D.G * (double)rB * wgt(i) * qv;
            }
        };
#pragma unroll
        for (int i = 1; i < Q; i++) {
            int pl[3];
            if (!step_in(p, opp(i), g, pl)) continue;  // plain source y - c_i
            source(i, pl, false);
        }
        if (!solid) {
            const T v0 = A0[n] + s[0], v1 = A0[N + n] + s[1];
            A0[n] = v0;
            A0[N + n] = v1;
            acc[0] = (double)v0;
            acc[1] = (double)v1;
        } else {
            a.vtb[bs] = (double)s[0] + lk[0];
            a.vtb[S3 + bs] = (double)s[1] + lk[1];
        }
    }
    block_sum<NB, ADJ_PB>(acc, red);
    if (threadIdx.x == 0)
        for (int k = 0; k < ADJ_PB; k++) a.partB[(int64_t)blockIdx.x * ADJ_PB + k] = acc[k];
}

// ============================================================ k_adj_mirror
// One thread per node y on a walled face (each node once: it belongs to the
// first walled axis, in x, y, z order, on whose face it lies).  Sources x
// whose x + c_i left the box across the wall next to y on at least one axis
// and was clamped back onto y there (the neutral-wall mirror of the force);
// on the other axes x is the plain y - c.  Adds to the density adjoint
// (fluid y) or to the wetting-layer adjoint (particle y); partials: the
// density-adjoint additions.
template <typename T>
__global__ __launch_bounds__(NB) void k_adj_mirror(AdjArgs a) {
    __shared__ double red[(NB / 64) * 2];
    const RepDesc D = a.desc[0];
    const RepState sn = *a.stn;
    const Geo g = geo_of(D);
    const int64_t N = g.N;
    const int S3 = D.S * D.S * D.S;
    const T *Fb = static_cast<const T *>(a.Fb);
    T *A0 = static_cast<T *>(a.Acur);
    const int n3[3] = {g.nx, g.ny, g.nz};
    const bool w3[3] = {g.wx, g.wy, g.wz};
    double acc[2] = {0.0, 0.0};
    int p[3] = {0, 0, 0};
    bool valid = false;
    int64_t k = (int64_t)blockIdx.x * NB + threadIdx.x;
    for (int ax = 0; ax < 3; ax++) {
        if (!w3[ax]) continue;
        const int b1 = ax == 0 ? 1 : 0, b2 = ax == 2 ? 1 : 2;
        const int64_t fsz = (int64_t)n3[b1] * n3[b2];
        if (k < 2 * fsz) {
            p[ax] = k >= fsz ? n3[ax] - 1 : 0;
            const int64_t r = k % fsz;
            p[b1] = (int)(r % n3[b1]);
            p[b2] = (int)(r / n3[b1]);
            valid = true;
            for (int e = 0; e < ax; e++)
                if (w3[e] && (p[e] == 0 || p[e] == n3[e] - 1)) valid = false;
            break;
        }
        k -= 2 * fsz;
    }
    if (valid) {
        const bool near = near_box(p, D, sn.org, g);
        int bs = -1;
        const bool solid = near && solid_at(p[0], p[1], p[2], D, sn.org, sn.X, g, bs);
        const T G = T(D.G);
        T s[2] = {T(0), T(0)};
        // every direction expanded at compile time (in ascending order, as a
        // loop would add them): the subsets m that use an axis the direction
        // does not move along drop out, and the loads of the remaining
        // candidates are issued together
        auto dir_term = [&](auto ic) {
            constexpr int i = decltype(ic)::value;
            const int c3[3] = {cx(i), cy(i), cz(i)};
            int pl[3];
            bool cl[3];
#pragma unroll
            for (int ax = 0; ax < 3; ax++) {
                int v = p[ax] - c3[ax];
                if (!w3[ax]) v = v < 0 ? v + n3[ax] : (v >= n3[ax] ? v - n3[ax] : v);
                pl[ax] = v;
                cl[ax] = w3[ax] && ((c3[ax] == -1 && p[ax] == 0) || (c3[ax] == 1 && p[ax] == n3[ax] - 1));
            }
            if (!(cl[0] || cl[1] || cl[2])) return;
            const T w = T(wgt(i));
#pragma unroll
            for (int m = 1; m < 8; m++) {
                int xs[3];
                bool ok = true;
#pragma unroll
                for (int ax = 0; ax < 3; ax++) {
                    const bool use = (m >> ax) & 1;
                    if (use && !cl[ax]) ok = false;
                    xs[ax] = use ? p[ax] : pl[ax];
                    if (xs[ax] < 0 || xs[ax] >= n3[ax]) ok = false;
                }
                if (!ok) continue;
                int bx;
                if (near && solid_at(xs[0], xs[1], xs[2], D, sn.org, sn.X, g, bx)) continue;
                const int64_t si = lin(xs, g);
                T cFA = T(0), cFB = T(0);  // Fb holds rho_l(x) times the force adjoint of x
                for (int q = 0; q < 3; q++) {
                    if (!c3[q]) continue;
                    const T fa = Fb[q * N + si], fb = Fb[(3 + q) * N + si];
                    cFA += c3[q] > 0 ? fa : -fa;
                    cFB += c3[q] > 0 ? fb : -fb;
                }
                s[1] += -G * w * cFA;
                s[0] += -G * w * cFB;
            }
        };
        for_each_dir(dir_term, std::make_integer_sequence<int, Q - 1>{});
        if (!solid) {
            const int64_t m = lin(p, g);
            const T v0 = A0[m] + s[0], v1 = A0[N + m] + s[1];
            acc[0] = (double)v0 - (double)A0[m];
            acc[1] = (double)v1 - (double)A0[N + m];
            A0[m] = v0;
            A0[N + m] = v1;
        } else {
            a.vtb[bs] += (double)s[0];
            a.vtb[S3 + bs] += (double)s[1];
        }
    }
    block_sum<NB, 2>(acc, red);
    if (threadIdx.x == 0) {
        a.partM[(int64_t)blockIdx.x * PART] = acc[0];
        a.partM[(int64_t)blockIdx.x * PART + 1] = acc[1];
    }
}

// Fixed-order sums (one workgroup of NB threads; the order depends on the
// partial indices only) of the node-kernel, link, wall-mirror and chain
// partials into the adjoint state: G, a_f, U, Omega, X adjoints; the
// density-adjoint sum of the reversed state for the next mass correction;
// Delta rho.  Resets the completion counter.
__device__ __forceinline__ void adj_sums(const AdjArgs &a, double *red) {
    const int t = threadIdx.x;
    double acc[18];
#pragma unroll
    for (int k = 0; k < 18; k++) acc[k] = 0.0;
    for (int w = t; w < a.nlt; w += NB)
        for (int k = 0; k < ADJ_PA; k++) acc[k] += a.partA[(int64_t)w * ADJ_PA + k];
    for (int w = t; w < a.nwg; w += NB)
        for (int k = 0; k < ADJ_PB; k++) acc[ADJ_PA + k] += a.partB[(int64_t)w * ADJ_PB + k];
    for (int w = t; w < a.nmw; w += NB)
        for (int k = 0; k < 2; k++) acc[15 + k] += a.partM[(int64_t)w * PART + k];
    for (int w = t; w < 2 * a.nbw; w += NB)
        for (int k = 0; k < ADJ_PA; k++) acc[k] += a.partL[(int64_t)w * PART + k];
    for (int w = t; w < a.nbw; w += NB)
        for (int k = 0; k < ADJ_PC; k++) acc[15 + k] += a.partC[(int64_t)w * PART + k];
    block_sum<NB, 18>(acc, red);
    if (t != 0) return;
    AdjState *o = a.adj;
    o->done = 0u;
    o->grad[3] += acc[0];
    for (int q = 0; q < 3; q++) {
        o->afb[q] += acc[1 + q];
        o->Ub[q] += acc[4 + q];
        o->Wb[q] += acc[7 + q];
        o->Xb[q] += acc[10 + q];
    }
    o->dsum[0] = acc[13] + acc[15];
    o->dsum[1] = acc[14] + acc[16];
    o->grad[4] += acc[17];
}


// ============================================================= k_adj_chain
// One thread per box node.  Wetting layer: rho~_l(s) = mean over fluid
// neighbours of rho_l +/- Delta rho on particle nodes s, so each fluid
// neighbour gets vtb_l(s) / count (gathered here by the fluid box nodes)
// and Delta rho gets vtb_A - vtb_B.  Partials: the density adjoint added
// per component, the Delta rho adjoint.
template <typename T>
__global__ __launch_bounds__(NB) void k_adj_chain(AdjArgs a) {
    __shared__ double red[(NB / 64) * ADJ_PC];
    __shared__ double red2[(NB / 64) * 18];
    const RepDesc D = a.desc[0];
    const RepState sn = *a.stn;
    const Geo g = geo_of(D);
    const int64_t N = g.N;
    const int Sx = D.S, S3 = Sx * Sx * Sx;
    T *A0 = static_cast<T *>(a.Acur);
    double acc[ADJ_PC] = {0.0, 0.0, 0.0};
    const int b = blockIdx.x * NB + threadIdx.x;
    int bb[3], p[3];
    const bool in = b < S3 && bbox_pos(b, sn.org, Sx, g, bb, p);
    if (in && pnode(p[0], p[1], p[2], sn.X, D.R2, g)) {
        if (a.vinv[b] > 0.0) acc[2] = a.vtb[b] - a.vtb[S3 + b];
    } else if (in) {
        double s[2] = {0.0, 0.0};
        bool any = false;
#pragma unroll
        for (int i = 1; i < Q; i++) {
            int q[3];
            if (!step_in(p, i, g, q)) continue;
            const int bq = bbox_index(q[0], q[1], q[2], sn.org, Sx, g);
            if (bq < 0 || a.vinv[bq] == 0.0) continue;
            if (!pnode(q[0], q[1], q[2], sn.X, D.R2, g)) continue;
            s[0] += a.vtb[bq] * a.vinv[bq];
            s[1] += a.vtb[S3 + bq] * a.vinv[bq];
            any = true;
        }
        if (any) {
            const int64_t m = lin(p, g);
            const T v0 = T((double)A0[m] + s[0]), v1 = T((double)A0[N + m] + s[1]);
            acc[0] = (double)v0 - (double)A0[m];
            acc[1] = (double)v1 - (double)A0[N + m];
            A0[m] = v0;
            A0[N + m] = v1;
        }
    }
    block_sum<NB, ADJ_PC>(acc, red);
    if (threadIdx.x == 0)
        for (int k = 0; k < ADJ_PC; k++) a.partC[(int64_t)blockIdx.x * PART + k] = acc[k];
    // the last workgroup to finish sums every partial of the reversed step
    __shared__ int last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) last = atomicAdd(&a.adj->done, 1u) == (unsigned)(a.nbw - 1);
    __syncthreads();
    if (!last) return;
    __threadfence();
    adj_sums(a, red2);
}

template <typename S, typename T>
hipError_t launch_record_t(const RecArgs &a, int64_t N, hipStream_t s) {
    hipLaunchKernelGGL((k_adj_record<S, T>), dim3((int)((N + NB - 1) / NB)), dim3(NB), 0, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_step_t(const AdjArgs &a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    hipLaunchKernelGGL((k_adj_events<T>), dim3(a.nbw), dim3(NB), 0, s, a);
    hipLaunchKernelGGL((k_adj_kept<T>), dim3(a.nbw), dim3(NB), 0, s, a);
    if (e0) {
        const hipError_t e = hipEventRecord(e0, s);
        if (e != hipSuccess) return e;
    }
    const size_t lds = (size_t)3 * LV * (a.lty + 2) * a.desc_nx * sizeof(T);
    hipLaunchKernelGGL((k_adj_local<T>), dim3(a.nlt), dim3(NB), lds, s, a);
    if (e1) {
        const hipError_t e = hipEventRecord(e1, s);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_adj_links<T>), dim3(2 * a.nbw), dim3(NB), 0, s, a);
    hipLaunchKernelGGL((k_adj_gather<T>), dim3(a.nwg), dim3(NB), 0, s, a);
    hipLaunchKernelGGL((k_adj_mirror<T>), dim3(a.nmw), dim3(NB), 0, s, a);
    hipLaunchKernelGGL((k_adj_chain<T>), dim3(a.nbw), dim3(NB), 0, s, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_adj_record(int prec, const RecArgs &a, int64_t N, hipStream_t s) {
    if (prec == 0) return launch_record_t<double, double>(a, N, s);
    if (prec == 1) return launch_record_t<float, float>(a, N, s);
    return launch_record_t<_Float16, float>(a, N, s);
}

hipError_t launch_adj_step(int prec, const AdjArgs &a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    return prec == 0 ? launch_step_t<double>(a, s, e0, e1) : launch_step_t<float>(a, s, e0, e1);
}

}  // namespace lbm
