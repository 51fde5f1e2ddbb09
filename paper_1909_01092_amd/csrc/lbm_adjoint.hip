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
// One reversed step = k_adj_pre (box: mass correction, events,
// Newton-Euler; wetting-layer densities of step n) + k_adj_local (all
// nodes: collision, force and link adjoints) + k_adj_gather (all nodes:
// Shan-Chen gather from the neighbours' force adjoints) + k_adj_post (box:
// wetting-layer chain, fixed-order sums).
#include "lbm_adjoint.h"
#include "lbm_kernels_impl.h"

namespace lbm {
namespace {

constexpr int NB = 256;  // node-kernel block

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

// ============================================================== k_adj_pre
// One workgroup over the box of X^n.
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
//     (gathered by those neighbours in a second pass).
//  4. Newton-Euler: U^{n+1/2} = U^{n-1/2} + F/m_p, X^{n+1} = X^n + U^{n+1/2}.
//  Also the wetting-layer densities of step n (mean of fluid neighbours
//  +/- Delta rho) for the node kernels.
template <typename T>
__global__ __launch_bounds__(ADJ_BOX) void k_adj_pre(AdjArgs a) {
    __shared__ double red[(ADJ_BOX / 64) * 9];
    const RepDesc D = a.desc[0];
    const RepState sn = *a.stn, s1 = *a.stn1;
    const AdjState ad = *a.adj;
    const Geo g = geo_of(D);
    const int64_t N = g.N;
    const int t = threadIdx.x;
    const int Sx = D.S, S3 = Sx * Sx * Sx;
    const T *recn = static_cast<const T *>(a.recn);
    const T *rec1 = static_cast<const T *>(a.recn1);
    T *A1 = static_cast<T *>(a.Anext);
    const double nf1 = s1.n_fluid;
    const double dMb[2] = {-ad.dsum[0] / nf1, -ad.dsum[1] / nf1};
    double acc[9];
#pragma unroll
    for (int k = 0; k < 9; k++) acc[k] = 0.0;

    for (int b = t; b < S3; b += ADJ_BOX) {
        a.ubn[b] = 0.0;
        a.ubn[S3 + b] = 0.0;
        a.vt[b] = 0.0;
        a.vt[S3 + b] = 0.0;
        a.vinv[b] = 0.0;
        int bb[3], p[3];
        if (!bbox_pos(b, sn.org, Sx, g, bb, p)) continue;
        const bool so = pnode(p[0], p[1], p[2], sn.X, D.R2, g);
        const bool sn1 = pnode(p[0], p[1], p[2], s1.X, D.R2, g);
        const int64_t m = lin(p, g);
        if (so) {
            double s0 = 0.0, s1v = 0.0;
            int cnt = 0;
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
        if (!so && sn1) {  // covered
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
    }
    __syncthreads();
    // neighbours fluid at both times collect the uncovered-node adjoints
    for (int b = t; b < S3; b += ADJ_BOX) {
        int bb[3], p[3];
        if (!bbox_pos(b, sn.org, Sx, g, bb, p)) continue;
        if (pnode(p[0], p[1], p[2], sn.X, D.R2, g) || pnode(p[0], p[1], p[2], s1.X, D.R2, g)) continue;
        double s[2] = {0.0, 0.0};
        bool any = false;
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
    block_sum<ADJ_BOX, 9>(acc, red);
    if (t != 0) return;
    // Newton-Euler (J picks U_z^{n+1/2}; X^{n+1} = X^n + U^{n+1/2})
    AdjState *o = a.adj;
    double Ub1[3], Wb1[3], Xb1[3], Fb[3], Tb[3];
    for (int q = 0; q < 3; q++) {
        Xb1[q] = ad.Xb[q] + acc[6 + q];
        Ub1[q] = ad.Ub[q] + acc[q] + Xb1[q] + (q == 2 ? a.invN : 0.0);
        Wb1[q] = ad.Wb[q] + acc[3 + q];
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
    o->dMb[0] = dMb[0];
    o->dMb[1] = dMb[1];
    o->Jsum = ad.Jsum + s1.U[2];
}

// ============================================================ k_adj_local
// One thread per node, fluid at X^n.  Forward values are rebuilt from the
// recorded moments (forces from the neighbours' densities, the velocity and
// the regenerated normals); then, in reverse: the adjoint of f*_i(x) from
// where streaming took it (a neighbour's Abar, the node's own reflected Abar
// at walls, the moving-wall bounce-back at links), the collision adjoint in
// mode space, and the node-local part of the force adjoint.
template <typename T>
__global__ __launch_bounds__(NB) void k_adj_local(AdjArgs a) {
    __shared__ double red[(NB / 64) * ADJ_PA];
    const RepDesc D = a.desc[0];
    const RepState sn = *a.stn;
    const AdjState ad = *a.adj;
    const Geo g = geo_of(D);
    const int64_t N = g.N;
    const int S3 = D.S * D.S * D.S;
    const int64_t n = (int64_t)blockIdx.x * NB + threadIdx.x;
    double acc[ADJ_PA];
#pragma unroll
    for (int k = 0; k < ADJ_PA; k++) acc[k] = 0.0;
    const T *rec = static_cast<const T *>(a.recn);
    const T *A1 = static_cast<const T *>(a.Anext);
    T *A0 = static_cast<T *>(a.Acur);
    T *Fo = static_cast<T *>(a.Fb);
    int bs = -1;
    const int x = (int)(n % g.nx), y = (int)((n / g.nx) % g.ny);
    const int z = (int)(n / ((int64_t)g.nx * g.ny));
    const bool live = n < N;
    const bool solid = live && solid_at(x, y, z, D, sn.org, sn.X, g, bs);
    if (live && solid) {
        for (int k = 0; k < 8; k++) A0[k * N + n] = T(0);
        for (int k = 0; k < 6; k++) Fo[k * N + n] = T(0);
    }
    if (live && !solid) {
        const int p[3] = {x, y, z};
        const T r0[2] = {T(D.rho0[0]), T(D.rho0[1])};
        T rd[2], jl[2][3];
        for (int l = 0; l < 2; l++) {
            rd[l] = rec[l * N + n];
            for (int q = 0; q < 3; q++) jl[l][q] = rec[(2 + 3 * l + q) * N + n];
        }
        const T rl[2] = {r0[0] + rd[0], r0[1] + rd[1]};
        // neighbours: wall crossings (reflected), sphere links, plain targets;
        // sums sum_i w_i rho~_l(x + c_i) c_i of density deviations
        T sv[2][3] = {{T(0), T(0), T(0)}, {T(0), T(0), T(0)}};
        uint32_t wall = 0, link = 0;
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
            int bm;
            const bool ms = solid_at(m3[0], m3[1], m3[2], D, sn.org, sn.X, g, bm);
            const int64_t mi = lin(m3, g);
            T rt[2];
            if (ms) {
                rt[0] = T(a.vt[bm] - D.rho0[0]);
                rt[1] = T(a.vt[S3 + bm] - D.rho0[1]);
            } else {
                rt[0] = rec[mi];
                rt[1] = rec[N + mi];
            }
            const T w = T(wgt(i));
            for (int l = 0; l < 2; l++)
                for (int q = 0; q < 3; q++)
                    if (c3[q]) sv[l][q] += c3[q] > 0 ? w * rt[l] : -(w * rt[l]);
            if (out) wall |= 1u << i;
            else if (ms) link |= 1u << i;
        }
        const T G = T(D.G);
        const T af[3] = {T(D.af[0]), T(D.af[1]), T(D.af[2])};
        T F[2][3];
        for (int q = 0; q < 3; q++) {
            F[0][q] = -G * rl[0] * sv[1][q] + rl[0] * af[q];
            F[1][q] = -G * rl[1] * sv[0][q] + rl[1] * af[q];
        }
        const Coef<T> cf = make_coef_dev<T>(D);
        T zz[36];
        if (cf.noise) noise36<T>((uint32_t)n, (uint32_t)sn.step, D.key0, D.key1, zz);
        else
            for (int k = 0; k < 36; k++) zz[k] = T(0);
        T u[3], xid[3];
        common_velocity(rd, jl, F, zz, cf, u, xid);

        // adjoint of the post-collision populations
        T fpb[2][Q];
        T Ar[2], Aj[2][3];
        for (int l = 0; l < 2; l++) {
            Ar[l] = A1[l * N + n];
            for (int q = 0; q < 3; q++) Aj[l][q] = A1[(2 + 3 * l + q) * N + n];
            fpb[l][0] = Ar[l];
        }
#pragma unroll
        for (int i = 1; i < Q; i++) {
            const T c3[3] = {T(cx(i)), T(cy(i)), T(cz(i))};
            if ((wall | link) >> i & 1u) {
                for (int l = 0; l < 2; l++)
                    fpb[l][i] = Ar[l] - (c3[0] * Aj[l][0] + c3[1] * Aj[l][1] + c3[2] * Aj[l][2]);
                continue;
            }
            int q3[3];
            step_in(p, i, g, q3);
            const int64_t tg = lin(q3, g);
            for (int l = 0; l < 2; l++) {
                T v = A1[l * N + tg];
                if (cx(i)) v += c3[0] * A1[(2 + 3 * l) * N + tg];
                if (cy(i)) v += c3[1] * A1[(3 + 3 * l) * N + tg];
                if (cz(i)) v += c3[2] * A1[(4 + 3 * l) * N + tg];
                fpb[l][i] = v;
            }
        }
        // moving-wall links (FP64): f_opp(i)(x) = f*_i(x) - 6 w_i rho_l (c_i . u_b);
        // exchanged momentum sum_l (2 f*_i - 6 w_i rho_l c_i . u_b) c_i, its torque
        // about X^n; wetting-layer reaction -G rho_l w_i rho~_l'(x + c_i) c_i
        double rlk[2] = {0.0, 0.0};
        if (link) {
            T fo[2][Q];
            for (int l = 0; l < 2; l++) {
                T zl[16];
                for (int k = 0; k < 16; k++) zl[k] = zz[16 * l + k];
                relax_tau1(r0[l], l ? T(-1) : T(1), rd[l], jl[l], F[l], u, xid, zl, cf, fo[l]);
            }
            const double d3[3] = {sepd(x - sn.X[0], g.nx, g.wx), sepd(y - sn.X[1], g.ny, g.wy),
                                  sepd(z - sn.X[2], g.nz, g.wz)};
            double V[3], TxD[3];
            cross3(sn.W, d3, V);
            for (int q = 0; q < 3; q++) V[q] += sn.U[q];
            cross3(ad.Tb, d3, TxD);
            for (int i = 1; i < Q; i++) {
                if (!(link >> i & 1u)) continue;
                const double c3[3] = {(double)cx(i), (double)cy(i), (double)cz(i)};
                int q3[3];
                step_in(p, i, g, q3);
                const int bm = bbox_index(q3[0], q3[1], q3[2], sn.org, D.S, g);
                const double vl[2] = {a.vt[bm], a.vt[S3 + bm]};
                const double cu = c3[0] * V[0] + c3[1] * V[1] + c3[2] * V[2];
                const double qv = c3[0] * (ad.Fb[0] + TxD[0]) + c3[1] * (ad.Fb[1] + TxD[1]) +
                                  c3[2] * (ad.Fb[2] + TxD[2]);
                double lpm = 0.0, cub = 0.0, flm = 0.0;
                for (int l = 0; l < 2; l++) {
                    const double rld = (double)rl[l];
                    const double fs = wgt(i) * D.rho0[l] + (double)fo[l][i];
                    const double corr = 6.0 * wgt(i) * rld * cu;
                    lpm += 2.0 * fs - corr;
                    const double al = (double)fpb[l][i];
                    fpb[l][i] = T(al + 2.0 * qv);
                    const double corrb = -al - qv - ad.dMb[l];
                    rlk[l] += 6.0 * wgt(i) * cu * corrb;
                    cub += 6.0 * wgt(i) * rld * corrb;
                    const double vo = vl[1 - l];
                    rlk[l] += D.G * wgt(i) * vo * qv;
                    acc[0] += rld * wgt(i) * vo * qv;
                    flm += -D.G * rld * wgt(i) * vo;
                }
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
        }

        // collision adjoint: ms_k = b_k sum_i w_i e_k(c_i) fpb_i / b_k^2 ...
        // mode adjoints Mb_k = (1/b_k) sum_i w_i e_k(c_i) fpb_i
        T rb[2], jb[2][3], Fbv[2][3];
        T ub[3] = {T(0), T(0), T(0)}, xb[3] = {T(0), T(0), T(0)};
        const T sqmu[3] = {cf.nb, cf.ns, cf.ng};
        for (int l = 0; l < 2; l++) {
            T gw[Q];
#pragma unroll
            for (int i = 0; i < Q; i++) gw[i] = T(wgt(i)) * fpb[l][i];
            T a0, aj[3], am[Q];
            component_modes(gw, a0, aj, am);
            const T Jb[3] = {T(3) * aj[0], T(3) * aj[1], T(3) * aj[2]};
            const T M4 = T(inv_norm(4)) * am[4], M5 = T(inv_norm(5)) * am[5], M6 = T(inv_norm(6)) * am[6];
            const T M7 = T(inv_norm(7)) * am[7], M8 = T(inv_norm(8)) * am[8], M9 = T(inv_norm(9)) * am[9];
            // m_eq + Phi/2 of modes 4..9 = u^T K u r / 2 + u^T K F / 2 with K symmetric
            const T Kxx = T(2) * M4 + T(4) * M5, Kyy = T(2) * M4 - T(2) * M5 + T(2) * M6;
            const T Kzz = T(2) * M4 - T(2) * M5 - T(2) * M6;
            const T Kxy = M7, Kyz = M8, Kxz = M9;
            const T Ku[3] = {Kxx * u[0] + Kxy * u[1] + Kxz * u[2], Kxy * u[0] + Kyy * u[1] + Kyz * u[2],
                             Kxz * u[0] + Kyz * u[1] + Kzz * u[2]};
            const T *Fl = F[l];
            const T KF[3] = {Kxx * Fl[0] + Kxy * Fl[1] + Kxz * Fl[2], Kxy * Fl[0] + Kyy * Fl[1] + Kyz * Fl[2],
                             Kxz * Fl[0] + Kyz * Fl[1] + Kzz * Fl[2]};
            const T sig = l ? T(-1) : T(1);
            rb[l] = a0 + (u[0] * Jb[0] + u[1] * Jb[1] + u[2] * Jb[2]) +
                    T(0.5) * (u[0] * Ku[0] + u[1] * Ku[1] + u[2] * Ku[2]);
            for (int q = 0; q < 3; q++) {
                ub[q] += rl[l] * (Jb[q] + Ku[q]) + T(0.5) * KF[q];
                Fbv[l][q] = T(0.5) * (Jb[q] + Ku[q]);
                xb[q] += sig * Jb[q];
            }
            // noise amplitude sqrt(mu rho_l b_k): d/d rho_l = sqrt(mu b_k) z / (2 sqrt rho_l)
            if (cf.noise && rl[l] > T(0)) {
                T s = T(0);
#pragma unroll
                for (int k = 4; k < Q; k++) {
                    const T sm = k == 4 ? sqmu[0] : (k <= 9 ? sqmu[1] : sqmu[2]);
                    s += T(inv_norm(k) * sqrt_norm(k)) * am[k] * sm * zz[16 * l + k - 4];
                }
                rb[l] += s / (T(2) * sqrt(rl[l]));
            }
        }
        // species-momentum noise amp z_{32+a}, amp = ampd sqrt(rho_A rho_B / rho)
        const T rho = rl[0] + rl[1];
        if (cf.noise && cf.diffusive && rl[0] > T(0) && rl[1] > T(0)) {
            const T amp = cf.ampd * sqrt(rl[0] * rl[1] / rho);
            const T ab = xb[0] * zz[32] + xb[1] * zz[33] + xb[2] * zz[34];
            rb[0] += ab * amp * rl[1] / (T(2) * rl[0] * rho);
            rb[1] += ab * amp * rl[0] / (T(2) * rl[1] * rho);
        }
        // u = (j_A + j_B + (F_A + F_B)/2) / rho
        const T ubu = (ub[0] * u[0] + ub[1] * u[1] + ub[2] * u[2]) / rho;
        for (int l = 0; l < 2; l++) {
            rb[l] -= ubu;
            for (int q = 0; q < 3; q++) {
                jb[l][q] = ub[q] / rho;
                Fbv[l][q] += T(0.5) * ub[q] / rho;
            }
        }
        // node-local part of the force adjoint: F_l = -G rho_l s_l' + rho_l a_f
        for (int l = 0; l < 2; l++) {
            const T *so = sv[1 - l];
            rb[l] += Fbv[l][0] * (af[0] - G * so[0]) + Fbv[l][1] * (af[1] - G * so[1]) +
                     Fbv[l][2] * (af[2] - G * so[2]);
            acc[0] += -(double)rl[l] * ((double)Fbv[l][0] * (double)so[0] + (double)Fbv[l][1] * (double)so[1] +
                                        (double)Fbv[l][2] * (double)so[2]);
            for (int q = 0; q < 3; q++) acc[1 + q] += (double)rl[l] * (double)Fbv[l][q];
        }
        for (int l = 0; l < 2; l++) {
            A0[l * N + n] = T((double)rb[l] + rlk[l]);
            for (int q = 0; q < 3; q++) {
                A0[(2 + 3 * l + q) * N + n] = jb[l][q];
                Fo[(3 * l + q) * N + n] = Fbv[l][q];
            }
        }
    }
    block_sum<NB, ADJ_PA>(acc, red);
    if (threadIdx.x == 0)
        for (int k = 0; k < ADJ_PA; k++) a.partA[(int64_t)blockIdx.x * ADJ_PA + k] = acc[k];
}

// =========================================================== k_adj_gather
// One thread per node y.  F_l(x) reads rho~_l'(m_i(x)), m_i(x) = x + c_i
// wrapped, or clamped onto the box across a wall; so y collects
// -G rho_l(x) w_i c_i . Fbar_l(x) from every fluid x with m_i(x) = y (per
// axis: y - c_i, plus y itself when x + c_i left the box through the wall
// next to y).  Particle nodes y also collect the wetting-layer reaction of
// their links (adjoint -q along c_i) and store the sum for the chain to
// their fluid neighbours.
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
        int bs;
        const bool solid = solid_at(p[0], p[1], p[2], D, sn.org, sn.X, g, bs);
        const int n3[3] = {g.nx, g.ny, g.nz};
        const bool w3[3] = {g.wx, g.wy, g.wz};
        const T G = T(D.G);
        T s[2] = {T(0), T(0)};
        double lk[2] = {0.0, 0.0};
        for (int i = 1; i < Q; i++) {
            const int c3[3] = {cx(i), cy(i), cz(i)};
            int cand[3][2], nc[3];
            bool clamp[3][2];
            for (int ax = 0; ax < 3; ax++) {
                const int c = c3[ax], v = p[ax] - c;
                nc[ax] = 0;
                if (!w3[ax]) {
                    cand[ax][0] = v < 0 ? v + n3[ax] : (v >= n3[ax] ? v - n3[ax] : v);
                    clamp[ax][0] = false;
                    nc[ax] = 1;
                    continue;
                }
                if (v >= 0 && v < n3[ax]) {
                    cand[ax][nc[ax]] = v;
                    clamp[ax][nc[ax]] = false;
                    nc[ax]++;
                }
                if ((c == -1 && p[ax] == 0) || (c == 1 && p[ax] == n3[ax] - 1)) {
                    cand[ax][nc[ax]] = p[ax];
                    clamp[ax][nc[ax]] = true;
                    nc[ax]++;
                }
            }
            const T w = T(wgt(i));
            for (int i0 = 0; i0 < nc[0]; i0++)
                for (int i1 = 0; i1 < nc[1]; i1++)
                    for (int i2 = 0; i2 < nc[2]; i2++) {
                        const int xs[3] = {cand[0][i0], cand[1][i1], cand[2][i2]};
                        int bx;
                        if (solid_at(xs[0], xs[1], xs[2], D, sn.org, sn.X, g, bx)) continue;
                        const int64_t si = lin(xs, g);
                        const T rA = T(D.rho0[0]) + rec[si], rB = T(D.rho0[1]) + rec[N + si];
                        T cFA = T(0), cFB = T(0);
                        for (int q = 0; q < 3; q++) {
                            if (!c3[q]) continue;
                            const T fa = Fb[q * N + si], fb = Fb[(3 + q) * N + si];
                            cFA += c3[q] > 0 ? fa : -fa;
                            cFB += c3[q] > 0 ? fb : -fb;
                        }
                        // F_A(x) reads rho~_B(y), F_B(x) reads rho~_A(y)
                        s[1] += -G * rA * w * cFA;
                        s[0] += -G * rB * w * cFB;
                        const bool mirrored = clamp[0][i0] || clamp[1][i1] || clamp[2][i2];
                        if (solid && !mirrored) {
                            const double d3[3] = {sepd(xs[0] - sn.X[0], g.nx, g.wx),
                                                  sepd(xs[1] - sn.X[1], g.ny, g.wy),
                                                  sepd(xs[2] - sn.X[2], g.nz, g.wz)};
                            double TxD[3];
                            cross3(ad.Tb, d3, TxD);
                            double qv = 0.0;
                            for (int q = 0; q < 3; q++) qv += c3[q] * (ad.Fb[q] + TxD[q]);
                            lk[1] += D.G * (double)rA * wgt(i) * qv;
                            lk[0] += D.G * (double)rB * wgt(i) * qv;
                        }
                    }
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

// ============================================================= k_adj_post
// One workgroup.  Wetting layer: rho~_l(s) = mean over fluid neighbours of
// rho_l +/- Delta rho on particle nodes s, so each fluid neighbour gets
// vtb_l(s) / count (gathered here by the fluid box nodes) and Delta rho
// gets vtb_A - vtb_B.  Then the fixed-order sums of the node-kernel
// partials go into the adjoint state.
template <typename T>
__global__ __launch_bounds__(ADJ_BOX) void k_adj_post(AdjArgs a) {
    __shared__ double red[(ADJ_BOX / 64) * 18];
    const RepDesc D = a.desc[0];
    const RepState sn = *a.stn;
    const Geo g = geo_of(D);
    const int64_t N = g.N;
    const int t = threadIdx.x;
    const int Sx = D.S, S3 = Sx * Sx * Sx;
    T *A0 = static_cast<T *>(a.Acur);
    double acc[18];
#pragma unroll
    for (int k = 0; k < 18; k++) acc[k] = 0.0;
    for (int w = t; w < a.nwg; w += ADJ_BOX) {
        for (int k = 0; k < ADJ_PA; k++) acc[k] += a.partA[(int64_t)w * ADJ_PA + k];
        for (int k = 0; k < ADJ_PB; k++) acc[ADJ_PA + k] += a.partB[(int64_t)w * ADJ_PB + k];
    }
    if (D.has_particle) {
        for (int b = t; b < S3; b += ADJ_BOX) {
            int bb[3], p[3];
            if (!bbox_pos(b, sn.org, Sx, g, bb, p)) continue;
            if (pnode(p[0], p[1], p[2], sn.X, D.R2, g)) {
                if (a.vinv[b] > 0.0) acc[17] += a.vtb[b] - a.vtb[S3 + b];
                continue;
            }
            double s[2] = {0.0, 0.0};
            bool any = false;
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
                acc[15] += (double)v0 - (double)A0[m];
                acc[16] += (double)v1 - (double)A0[N + m];
                A0[m] = v0;
                A0[N + m] = v1;
            }
        }
    }
    block_sum<ADJ_BOX, 18>(acc, red);
    if (t != 0) return;
    AdjState *o = a.adj;
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

template <typename S, typename T>
hipError_t launch_record_t(const RecArgs &a, int64_t N, hipStream_t s) {
    hipLaunchKernelGGL((k_adj_record<S, T>), dim3((int)((N + NB - 1) / NB)), dim3(NB), 0, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_step_t(const AdjArgs &a, hipStream_t s) {
    hipLaunchKernelGGL((k_adj_pre<T>), dim3(1), dim3(ADJ_BOX), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_adj_local<T>), dim3(a.nwg), dim3(NB), 0, s, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_adj_gather<T>), dim3(a.nwg), dim3(NB), 0, s, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_adj_post<T>), dim3(1), dim3(ADJ_BOX), 0, s, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_adj_record(int prec, const RecArgs &a, int64_t N, hipStream_t s) {
    if (prec == 0) return launch_record_t<double, double>(a, N, s);
    if (prec == 1) return launch_record_t<float, float>(a, N, s);
    return launch_record_t<_Float16, float>(a, N, s);
}

hipError_t launch_adj_step(int prec, const AdjArgs &a, hipStream_t s) {
    return prec == 0 ? launch_step_t<double>(a, s) : launch_step_t<float>(a, s);
}

}  // namespace lbm
