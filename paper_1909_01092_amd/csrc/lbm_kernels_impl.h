// HIP kernels (gfx950) of the fluctuating two-component D3Q19 step with one
// finite-size sphere per replica.  Instantiated once per storage precision
// by lbm_k_f64.hip / lbm_k_f32.hip / lbm_k_f16.hip.
//
// Paper: Xue, Biferale, Sbragaglia, Toschi, "A lattice Boltzmann study of
// particle settling in a fluctuating multicomponent fluid under
// confinement".  Sec. 2: eq. (density), eq. (lbe), MRT paragraph,
// eq. (sc-force), noise paragraph, particle paragraph (particle nodes,
// leap-frog Newton, moving bounce-back with momentum exchange,
// cover/uncover, mass correction, virtual wetting layer).  Sec. 3: eq. (fp).
//
// One step = k_main (all nodes of all replicas) + k_particle (bounding box
// of each sphere; the last workgroup per replica finishes the step).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm_kernels.h"
#include "lbm_math.h"
#include "lbm_types.h"

namespace lbm {

template <typename T>
__device__ __forceinline__ Coef<T> make_coef_dev(const RepDesc &D) {
    return make_coef<T>(D.rho0[0], D.rho0[1], D.tau[0], D.tau[1], D.tau[2], D.tau[3], D.kT,
                        D.noise_diffusive);
}

// ------------------------------------------------------------ storage forms
template <typename S> struct Rel { static constexpr bool value = false; };
template <> struct Rel<_Float16> { static constexpr bool value = true; };

template <typename S, typename T>
__device__ __forceinline__ T ld_dev(const S *p, T scale) {
    if constexpr (Rel<S>::value) return T((float)(*p)) * scale;
    else return T(*p);
}
template <typename S, typename T>
__device__ __forceinline__ void st_dev(S *p, T v, T inv_scale) {
    if constexpr (Rel<S>::value) *p = (S)(float)(v * inv_scale);
    else *p = (S)v;
}

// ------------------------------------------------------------------ geometry
struct Geo {
    int nx, ny, nz;
    bool wx, wy, wz;
    int64_t N;
};

__device__ __forceinline__ Geo geo_of(const RepDesc &D) {
    Geo g;
    g.nx = D.nx; g.ny = D.ny; g.nz = D.nz;
    g.wx = D.walls & 1u; g.wy = D.walls & 2u; g.wz = D.walls & 4u;
    g.N = D.N;
    return g;
}

// bring a coordinate one layer outside the box back in; false = wall layer
__device__ __forceinline__ bool wrap1(int &v, int n, bool wall) {
    if (v < 0 || v >= n) {
        if (wall) return false;
        v = v < 0 ? v + n : v - n;
    }
    return true;
}
// wall layers mirror onto the adjacent node, periodic axes wrap
__device__ __forceinline__ int mirror1(int v, int n, bool wall) {
    if (v < 0) return wall ? 0 : v + n;
    if (v >= n) return wall ? n - 1 : v - n;
    return v;
}

// minimum-image separation along one axis (periodic axes only)
__device__ __forceinline__ double sepd(double d, int n, bool wall) {
#pragma clang fp contract(off)
    if (!wall) {
        const double h = 0.5 * (double)n;
        if (d > h) d = d - (double)n;
        else if (d < -h) d = d + (double)n;
    }
    return d;
}

// particle-node predicate |x - X|^2 < R^2 in FP64 with every product rounded
// on its own (no contraction), so every implementation decides identically.
__device__ __forceinline__ bool pnode(int x, int y, int z, const double *X, double R2,
                                      const Geo &g) {
#pragma clang fp contract(off)
    const double dx = sepd((double)x - X[0], g.nx, g.wx);
    const double dy = sepd((double)y - X[1], g.ny, g.wy);
    const double dz = sepd((double)z - X[2], g.nz, g.wz);
    double d2 = dx * dx + dy * dy;
    d2 = d2 + dz * dz;
    return d2 < R2;
}

// cheap conservative test: within lim of X along every axis
__device__ __forceinline__ bool near_box(int x, int y, int z, const double *X, double lim,
                                         const Geo &g) {
    return fabs(sepd((double)x - X[0], g.nx, g.wx)) < lim &&
           fabs(sepd((double)y - X[1], g.ny, g.wy)) < lim &&
           fabs(sepd((double)z - X[2], g.nz, g.wz)) < lim;
}

// node index inside a replica (a replica block of 38 N elements fits 32 bits)
__device__ __forceinline__ uint32_t nidx(int x, int y, int z, const Geo &g) {
    return (uint32_t)x + (uint32_t)g.nx * ((uint32_t)y + (uint32_t)g.ny * (uint32_t)z);
}

// Integer box around the sphere centre X, widened by lim on every side, in
// which exact particle predicates are evaluated.  Periodic axes test the
// three images of a coordinate.
struct NearBox {
    int lo[3], hi[3];
};
__device__ __forceinline__ NearBox near_bounds(const double *X, double lim) {
    NearBox b;
    for (int a = 0; a < 3; a++) {
        b.lo[a] = (int)floor(X[a] - lim);
        b.hi[a] = (int)ceil(X[a] + lim);
    }
    return b;
}
__device__ __forceinline__ bool in_range(int v, int lo, int hi, int n, bool wall) {
    if (v >= lo && v <= hi) return true;
    if (wall) return false;
    return (v + n >= lo && v + n <= hi) || (v - n >= lo && v - n <= hi);
}
__device__ __forceinline__ bool near_int(int x, int y, int z, const NearBox &b, const Geo &g) {
    return in_range(x, b.lo[0], b.hi[0], g.nx, g.wx) && in_range(y, b.lo[1], b.hi[1], g.ny, g.wy) &&
           in_range(z, b.lo[2], b.hi[2], g.nz, g.wz);
}

__device__ __forceinline__ int find_rep(const int32_t *begin, int nrep, int wg) {
    int lo = 0, hi = nrep - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (begin[mid] <= wg) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// bbox array index of a box node, -1 when outside the array
__device__ __forceinline__ int bbox_index(int x, int y, int z, const int32_t *org, int S,
                                          const Geo &g) {
    int bx = x - org[0], by = y - org[1], bz = z - org[2];
    if (!g.wx) { if (bx < 0) bx += g.nx; else if (bx >= g.nx) bx -= g.nx; }
    if (!g.wy) { if (by < 0) by += g.ny; else if (by >= g.ny) by -= g.ny; }
    if (!g.wz) { if (bz < 0) bz += g.nz; else if (bz >= g.nz) bz -= g.nz; }
    if (bx < 0 || by < 0 || bz < 0 || bx >= S || by >= S || bz >= S) return -1;
    return (bz * S + by) * S + bx;
}

// ------------------------------------------------------------------ pulling
// Populations f_{l i}(x, n) of a fluid node in deviation form: each comes from
// the post-collision slot i of x - c_i, or - when x - c_i is a wall layer or a
// particle node at X^{n-1} (bit i of the node mask) - from the node's own slot
// opp(i), which the previous step stored already bounced.  Nodes uncovered
// at this step (MASK_LOCAL), and every node right after initialisation, hold
// their populations in their own slots.  The mass correction of the previous
// step adds w_i delta_l.
template <typename S, typename T>
struct PullCtx {
    const S *src;          // replica block
    Geo g;
    bool local_read;
    T delta[2];
    T scale[2];            // FP16 relative storage: rho0_l (times w_i per slot)
};

template <typename S, typename T>
__device__ __forceinline__ PullCtx<S, T> pull_ctx(const void *buf, const RepDesc &D,
                                                  const RepState &st, bool with_delta) {
    PullCtx<S, T> pc;
    pc.src = reinterpret_cast<const S *>(buf) + D.pop_off;
    pc.g = geo_of(D);
    pc.local_read = st.local_read != 0;
    for (int l = 0; l < 2; l++) {
        pc.delta[l] = with_delta ? T(st.delta[l]) : T(0);
        pc.scale[l] = Rel<S>::value ? T(D.rho0[l]) : T(1);
    }
    return pc;
}

template <typename S, typename T>
__device__ __forceinline__ void pull_node(const PullCtx<S, T> &c, int x, int y, int z, uint32_t mask,
                                          T (&d)[2][Q]) {
    const uint32_t own = nidx(x, y, z, c.g);
    const uint32_t N = (uint32_t)c.g.N;
    const bool loc = c.local_read || (mask & MASK_LOCAL);
#pragma unroll
    for (int i = 0; i < Q; i++) {
        uint32_t idx = own;
        int slot = i;
        if (!loc && i != 0) {
            int sx = x - cx(i), sy = y - cy(i), sz = z - cz(i);
            bool ok = !((mask >> i) & 1u);
            if (cx(i) != 0) ok = ok && wrap1(sx, c.g.nx, c.g.wx);
            if (cy(i) != 0) ok = ok && wrap1(sy, c.g.ny, c.g.wy);
            if (cz(i) != 0) ok = ok && wrap1(sz, c.g.nz, c.g.wz);
            if (ok) idx = nidx(sx, sy, sz, c.g);
            else slot = opp(i);
        }
        const T w = T(wgt(i));
#pragma unroll
        for (int l = 0; l < 2; l++)
            d[l][i] = ld_dev<S, T>(c.src + ((uint32_t)(l * Q + slot) * N + idx), w * c.scale[l]) +
                      w * c.delta[l];
    }
}

// mask of a box node for the current step (0 outside the bounding box)
__device__ __forceinline__ uint32_t node_mask(int x, int y, int z, const uint32_t *pmask,
                                              const int32_t *org, int S, const Geo &g, int &b) {
    b = bbox_index(x, y, z, org, S, g);
    return b >= 0 ? pmask[b] : 0u;
}

// What a collision needs from the pulled populations of a node: density
// deviations, momenta and (unless every relaxation time is 1, when the
// post-collision state depends on density and momentum only) modes 4..18.
template <typename T, bool TAU1>
struct NodeM {
    T rd[2];
    T j[2][3];
    T m[2][TAU1 ? 1 : Q];
};

template <typename T, bool TAU1>
__device__ __forceinline__ void node_moments(const T (&d)[2][Q], NodeM<T, TAU1> &s) {
#pragma unroll
    for (int l = 0; l < 2; l++) {
        if constexpr (TAU1) {
            T r = T(0), jx = T(0), jy = T(0), jz = T(0);
#pragma unroll
            for (int i = 0; i < Q; i++) {
                r += d[l][i];
                if (cx(i) > 0) jx += d[l][i]; else if (cx(i) < 0) jx -= d[l][i];
                if (cy(i) > 0) jy += d[l][i]; else if (cy(i) < 0) jy -= d[l][i];
                if (cz(i) > 0) jz += d[l][i]; else if (cz(i) < 0) jz -= d[l][i];
            }
            s.rd[l] = r; s.j[l][0] = jx; s.j[l][1] = jy; s.j[l][2] = jz;
        } else {
            component_modes(d[l], s.rd[l], s.j[l], s.m[l]);
        }
    }
}

// ------------------------------------------------------- block reductions
template <int NV>
__device__ __forceinline__ void wave_sum(double (&v)[NV]) {
#pragma unroll
    for (int k = 0; k < NV; k++) {
        double x = v[k];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        v[k] = x;
    }
}

// fixed-order sum over the workgroup, result in every thread
template <int B, int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double *red /* [B/64][NV] */) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    wave_sum<NV>(v);
    __syncthreads();
    if (lane == 0)
        for (int k = 0; k < NV; k++) red[wave * NV + k] = v[k];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 0; k < NV; k++) {
            double s = 0.0;
            for (int w = 0; w < B / 64; w++) s += red[w * NV + k];
            red[k] = s;
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; k++) v[k] = red[k];
    __syncthreads();
}

// position of bbox entry b (origin org, edge S); false when it lies in a wall layer
__device__ __forceinline__ bool bbox_pos(int b, const int32_t *org, int S, const Geo &g, int (&bb)[3],
                                         int (&p)[3]) {
    bb[0] = b % S; bb[1] = (b / S) % S; bb[2] = b / (S * S);
    const int n3[3] = {g.nx, g.ny, g.nz};
    const bool w3[3] = {g.wx, g.wy, g.wz};
    bool in = true;
    for (int q = 0; q < 3; q++) {
        int v = org[q] + bb[q];
        if (v < 0 || v >= n3[q]) {
            if (w3[q]) in = false;
            else v = ((v % n3[q]) + n3[q]) % n3[q];
        }
        p[q] = v;
    }
    return in;
}

// ================================================================ k_main
// Workgroup = ty full x-rows of one replica, marching over cz z-planes.
// Density deviations of the tile plus a one-node halo (rows y0-1 and
// y0+rows, planes z-1 and z+1) sit in a 3-plane LDS ring; halo densities are
// recomputed from pulled populations, so no density field goes through HBM.
// The density and momenta of the next plane stay in registers while the
// current plane collides.  The sphere enters only through the integer node
// masks and the wetting-layer densities of its bounding box; every FP64
// particle computation lives in k_links / k_particle.
template <typename S, typename T, int B, bool TAU1>
__global__ __launch_bounds__(B) void k_main(MainArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    T *lds = reinterpret_cast<T *>(smem);

    const int wg = blockIdx.x;
    const int r = find_rep(a.wg_begin, a.nrep, wg);
    const RepDesc &D = a.desc[r];
    RepState *stp = a.state + r;
    const Geo g = geo_of(D);
    const int nx = g.nx;
    const int local = wg - D.wg_begin;
    const int yt = local % D.nty, ch = local / D.nty;
    const int y0 = yt * D.ty, rows = min(D.ty, g.ny - y0);
    const int z0 = ch * D.cz, z1 = min(z0 + D.cz, g.nz);
    const int t = threadIdx.x;
    const int nin = nx * rows;
    const bool inner = t < nin;
    const int x = inner ? t % nx : 0, yl = inner ? t / nx : 0;
    const int y = y0 + yl;
    const int pr = (D.ty + 2) * nx;  // LDS elements per plane and component

    const bool hp = D.has_particle;
    const PullCtx<S, T> pc = pull_ctx<S, T>(a.src, D, *stp, true);
    const double dl[2] = {stp->delta[0], stp->delta[1]};
    const uint32_t step = (uint32_t)stp->step;
    const int32_t org[3] = {stp->org[0], stp->org[1], stp->org[2]};
    const int Sx = D.S, S3 = Sx * Sx * Sx;
    const uint32_t *pmask = a.pmask + D.bbox_off;
    const double *vrho = a.vrho + D.bbox_off * 2;
    double *rho_n = a.rho_n + D.bbox_off * 2;
    S *dst = reinterpret_cast<S *>(a.dst) + D.pop_off;
    const uint32_t N32 = (uint32_t)g.N;

    auto L = [&](int zp, int l, int row, int xx) -> T & {
        const int slot = ((zp % 3) + 3) % 3;
        return lds[(slot * 2 + l) * pr + (row + 1) * nx + xx];
    };

    // density deviation of a box node: pulled, or the wetting-layer value on
    // particle nodes; fluid nodes also return their moments
    auto node_density = [&](int xx, int yy, int zz, NodeM<T, TAU1> &s, T &rA, T &rB) -> bool {
        int b = -1;
        const uint32_t m = hp ? node_mask(xx, yy, zz, pmask, org, Sx, g, b) : 0u;
        if (!(m & MASK_SOLID)) {
            T d[2][Q];
            pull_node(pc, xx, yy, zz, m, d);
            node_moments(d, s);
            rA = s.rd[0];
            rB = s.rd[1];
            return true;
        }
        rA = T(vrho[b] + dl[0] - D.rho0[0]);
        rB = T(vrho[S3 + b] + dl[1] - D.rho0[1]);
        return false;
    };

    NodeM<T, TAU1> nxt;
    bool nxt_fluid = false;

    // fill LDS plane zp (unmapped index); the interior node's moments go to nxt
    auto fill = [&](int zp) {
        const int zz = mirror1(zp, g.nz, g.wz);
        if (inner) {
            T rA, rB;
            nxt_fluid = node_density(x, y, zz, nxt, rA, rB);
            L(zp, 0, yl, x) = rA;
            L(zp, 1, yl, x) = rB;
        }
        for (int h = t - nin; h < 2 * nx; h += B) {
            if (h < 0) continue;
            const int row = h < nx ? -1 : rows;
            const int xx = h < nx ? h : h - nx;
            const int yy = mirror1(y0 + row, g.ny, g.wy);
            NodeM<T, TAU1> hd;
            T rA, rB;
            node_density(xx, yy, zz, hd, rA, rB);
            L(zp, 0, row, xx) = rA;
            L(zp, 1, row, xx) = rB;
        }
    };

    const T G = T(D.G);
    const Coef<T> cf = make_coef_dev<T>(D);
    const int xm = mirror1(x - 1, nx, g.wx), xp = mirror1(x + 1, nx, g.wx);

    // plane zp is filled while plane zp - 1 collides
    for (int zp = z0 - 1; zp <= z1; zp++) {
        const NodeM<T, TAU1> cur = nxt;
        const bool cur_fluid = nxt_fluid;
        fill(zp);
        __syncthreads();
        if (zp <= z0) continue;
        const int z = zp - 1;
        const bool active = inner && cur_fluid;
        if (active) {
            const uint32_t own = nidx(x, y, z, g);
            const T(&rd)[2] = cur.rd;
            const T(&j)[2][3] = cur.j;
            // Shan-Chen: F_l = -G rho_l sum_i w_i rho~_l'(x + c_i) c_i + rho_l a_f
            T grad[2][3] = {{T(0), T(0), T(0)}, {T(0), T(0), T(0)}};
#pragma unroll
            for (int i = 1; i < Q; i++) {
                const int xx = cx(i) > 0 ? xp : (cx(i) < 0 ? xm : x);
                const T w = T(wgt(i));
#pragma unroll
                for (int l = 0; l < 2; l++) {
                    const T v = w * L(z + cz(i), l, yl + cy(i), xx);
                    if (cx(i)) grad[l][0] += cx(i) > 0 ? v : -v;
                    if (cy(i)) grad[l][1] += cy(i) > 0 ? v : -v;
                    if (cz(i)) grad[l][2] += cz(i) > 0 ? v : -v;
                }
            }
            const T rl[2] = {cf.rho0[0] + rd[0], cf.rho0[1] + rd[1]};
            if (!(rl[0] > T(0)) || !(rl[1] >= T(0))) atomicOr(&stp->flags, FLAG_UNSTABLE);
            if (hp) {  // densities near the sphere, for the link kernel
                const int b = bbox_index(x, y, z, org, Sx, g);
                if (b >= 0) {
                    rho_n[b] = (double)rl[0];
                    rho_n[S3 + b] = (double)rl[1];
                }
            }
            T F[2][3];
#pragma unroll
            for (int q = 0; q < 3; q++) {
                F[0][q] = -G * rl[0] * grad[1][q] + rl[0] * T(D.af[q]);
                F[1][q] = -G * rl[1] * grad[0][q] + rl[1] * T(D.af[q]);
            }
            T u[3], xid[3];
            T zz[36];
            if (cf.noise) noise_block<T>(own, step, 8u, D.key0, D.key1, zz + 32);
            else zz[32] = zz[33] = zz[34] = T(0);
            common_velocity(rd, j, F, zz, cf, u, xid);
#pragma unroll
            for (int l = 0; l < 2; l++) {
                if (cf.noise) {
#pragma unroll
                    for (int b = 0; b < 4; b++)
                        noise_block<T>(own, step, (uint32_t)(4 * l + b), D.key0, D.key1,
                                       zz + 16 * l + 4 * b);
                } else {
#pragma unroll
                    for (int k = 0; k < 16; k++) zz[16 * l + k] = T(0);
                }
                T out[Q];
                if constexpr (TAU1) relax_tau1(l, rd[l], j[l], F[l], u, xid, zz, cf, out);
                else relax_component(l, rd[l], j[l], cur.m[l], F[l], u, xid, zz, cf, out);
                const T sc = Rel<S>::value ? cf.rho0[l] : T(1);
#pragma unroll
                for (int i = 0; i < Q; i++)
                    st_dev<S, T>(dst + ((uint32_t)(l * Q + i) * N32 + own), out[i],
                                 Rel<S>::value ? T(1) / (T(wgt(i)) * sc) : T(1));
            }
        }
        __syncthreads();
    }
}

// =============================================================== k_links
// Links from fluid nodes into the sphere at X^n (one thread per bbox entry):
// moving-wall bounce-back f_opp(i)(x) = f*_i(x) - 6 w_i rho_l(x) (c_i . u_b)
// written over the stored slot i, momentum exchange
// sum_l (2 f*_i - 6 w_i rho_l c_i . u_b) c_i with its torque about X^n, the
// bounce-back mass flux, and the reaction of the wetting layer on the
// sphere.  Per-workgroup FP64 sums, fixed order.
template <typename S, typename T, int B>
__global__ __launch_bounds__(B) void k_links(LinkArgs a) {
    __shared__ double red[(B / 64) * 16];
    const int r = find_rep(a.k3_begin, a.nrep, blockIdx.x);
    const RepDesc &D = a.desc[r];
    if (!D.has_particle) return;
    const RepState &st = a.state[r];
    const Geo g = geo_of(D);
    const int t = threadIdx.x;
    const int local = blockIdx.x - D.k3_begin;
    const int Sx = D.S, S3 = Sx * Sx * Sx;
    const int32_t org[3] = {st.org[0], st.org[1], st.org[2]};
    const uint32_t *pmask = a.pmask + D.bbox_off;
    const double *vrho = a.vrho + D.bbox_off * 2;
    const double *rho_n = a.rho_n + D.bbox_off * 2;
    S *buf = reinterpret_cast<S *>(a.buf) + D.pop_off;
    const uint32_t N32 = (uint32_t)g.N;
    double acc[15];
    for (int k = 0; k < 15; k++) acc[k] = 0.0;
    const int b = local * B + t;
    if (b < S3) {
        int bb[3], p[3];
        const bool in = bbox_pos(b, org, Sx, g, bb, p);
        const uint32_t m = pmask[b];
        if (in && !(m & MASK_SOLID)) {
            const double X[3] = {st.X[0], st.X[1], st.X[2]};
            const double U[3] = {st.U[0], st.U[1], st.U[2]};
            const double W[3] = {st.W[0], st.W[1], st.W[2]};
            const double rA = rho_n[b], rB = rho_n[S3 + b];
            const uint32_t own = nidx(p[0], p[1], p[2], g);
#pragma unroll
            for (int i = 1; i < Q; i++) {
                const int qx = bb[0] + cx(i), qy = bb[1] + cy(i), qz = bb[2] + cz(i);
                if (qx < 0 || qy < 0 || qz < 0 || qx >= Sx || qy >= Sx || qz >= Sx) continue;
                const int qb = (qz * Sx + qy) * Sx + qx;
                if (!(pmask[qb] & MASK_SOLID)) continue;
                const double rr[3] = {sepd(p[0] + 0.5 * cx(i) - X[0], g.nx, g.wx),
                                      sepd(p[1] + 0.5 * cy(i) - X[1], g.ny, g.wy),
                                      sepd(p[2] + 0.5 * cz(i) - X[2], g.nz, g.wz)};
                const double ub[3] = {U[0] + W[1] * rr[2] - W[2] * rr[1],
                                      U[1] + W[2] * rr[0] - W[0] * rr[2],
                                      U[2] + W[0] * rr[1] - W[1] * rr[0]};
                const double cu = cx(i) * ub[0] + cy(i) * ub[1] + cz(i) * ub[2];
                const double rl[2] = {rA, rB};
                double mom = 0.0;
#pragma unroll
                for (int l = 0; l < 2; l++) {
                    S *ptr = buf + ((uint32_t)(l * Q + i) * N32 + own);
                    const double wr = wgt(i) * D.rho0[l];
                    const double fs = wr + (double)ld_dev<S, T>(ptr, Rel<S>::value ? T(wr) : T(1));
                    const double corr = 6.0 * wgt(i) * rl[l] * cu;
                    mom += 2.0 * fs - corr;
                    acc[6 + l] -= corr;
                    st_dev<S, T>(ptr, T(fs - corr - wr), Rel<S>::value ? T(1.0 / wr) : T(1));
                }
                const double lp[3] = {mom * cx(i), mom * cy(i), mom * cz(i)};
                acc[0] += lp[0]; acc[1] += lp[1]; acc[2] += lp[2];
                acc[3] += rr[1] * lp[2] - rr[2] * lp[1];
                acc[4] += rr[2] * lp[0] - rr[0] * lp[2];
                acc[5] += rr[0] * lp[1] - rr[1] * lp[0];
                acc[14] += 1.0;
                // wetting-layer reaction: the fluid's Shan-Chen force from this particle node
                const double s = -D.G * wgt(i) * (rA * (vrho[S3 + qb] + st.delta[1]) +
                                                  rB * (vrho[qb] + st.delta[0]));
                const double fl[3] = {s * cx(i), s * cy(i), s * cz(i)};
                acc[8] += fl[0]; acc[9] += fl[1]; acc[10] += fl[2];
                acc[11] += rr[1] * fl[2] - rr[2] * fl[1];
                acc[12] += rr[2] * fl[0] - rr[0] * fl[2];
                acc[13] += rr[0] * fl[1] - rr[1] * fl[0];
            }
        }
    }
    block_sum<B, 15>(acc, red);
    if (t == 0) {
        double *p = a.part1 + D.part3_off + (int64_t)local * PART;
        for (int k = 0; k < 15; k++) p[k] = acc[k];
    }
}

// =========================================================== k_particle_a
// Per replica, one thread per node of the sphere's new bounding box.  Every
// workgroup redundantly reduces the link partials (fixed order) and advances
// the sphere (leap-frog Newton-Euler under F = links - wetting reaction +
// F_ext + pending event momentum); workgroup 0 records the update.  Each
// thread then builds its node's mask for step n+1 and, for nodes fluid at
// X^n, pulls the step-(n+1) populations: densities for the wetting layer and
// uncovered nodes, momentum and mass of nodes the sphere covers.
template <typename S, typename T, int B>
__global__ __launch_bounds__(B) void k_particle_a(ParticleArgs a) {
    __shared__ double red[(B / 64) * 16];
    const int wg = blockIdx.x;
    const int r = find_rep(a.k3_begin, a.nrep, wg);
    const RepDesc &D = a.desc[r];
    if (!D.has_particle) return;
    RepState *st = a.state + r;
    const Geo g = geo_of(D);
    const int t = threadIdx.x;
    const int local = wg - D.k3_begin;

    double X[3], U[3], Wv[3];
    for (int q = 0; q < 3; q++) { X[q] = st->X[q]; U[q] = st->U[q]; Wv[q] = st->W[q]; }
    // 1. link momentum exchange and wetting-layer reaction of step n
    double sum[15];
    for (int k = 0; k < 15; k++) sum[k] = 0.0;
    for (int w = t; w < D.k3_count; w += B) {
        const double *p = a.part1 + D.part3_off + (int64_t)w * PART;
        for (int q = 0; q < 15; q++) sum[q] += p[q];
    }
    block_sum<B, 15>(sum, red);
    // 2. Newton-Euler, leap-frog
    double F[3], Tq[3], Un[3], Wn[3], Xn[3];
    const int n3[3] = {g.nx, g.ny, g.nz};
    const bool w3[3] = {g.wx, g.wy, g.wz};
    for (int q = 0; q < 3; q++) {
        F[q] = sum[q] - sum[8 + q] + D.Fext[q] + st->Pev[q];
        Tq[q] = sum[3 + q] - sum[11 + q] + st->Lev[q];
        Un[q] = D.fixed_velocity ? U[q] : U[q] + F[q] / D.mp;
        Wn[q] = D.fixed_velocity ? Wv[q] : Wv[q] + Tq[q] / D.Ip;
    }
    for (int q = 0; q < 3; q++) {
        Xn[q] = X[q] + Un[q];
        if (!w3[q]) {
            if (Xn[q] >= n3[q]) Xn[q] -= n3[q];
            else if (Xn[q] < 0.0) Xn[q] += n3[q];
        }
    }
    // 3. bounding box of X^n and X^{n+1}
    int org[3];
    for (int q = 0; q < 3; q++) {
        double lo = X[q];
        double xn = Xn[q];
        if (!w3[q]) {  // unwrap X^{n+1} next to X^n
            if (xn - lo > 0.5 * n3[q]) xn -= n3[q];
            else if (lo - xn > 0.5 * n3[q]) xn += n3[q];
        }
        lo = fmin(lo, xn);
        org[q] = (int)floor(lo - D.radius) - 2;
    }
    if (local == 0 && t == 0) {
        for (int q = 0; q < 3; q++) {
            st->Xn[q] = Xn[q]; st->Un[q] = Un[q]; st->Wn[q] = Wn[q];
            st->Fn[q] = F[q]; st->Tn[q] = Tq[q]; st->orgn[q] = org[q];
        }
        st->dMbb[0] = sum[6];
        st->dMbb[1] = sum[7];
        st->nlinks = sum[14];
    }
    const int Sx = D.S, S3 = Sx * Sx * Sx;
    double *raw = a.raw + D.bbox_off * 2;
    uint8_t *flags = a.flags + D.bbox_off;
    uint32_t *pmask = a.pmask + D.bbox_off;
    PullCtx<S, T> pc = pull_ctx<S, T>(a.buf, D, *st, false);
    pc.local_read = false;

    // 4. node masks of step n+1; covered nodes (fluid at X^n, particle at
    // X^{n+1}) with the momentum of their step-(n+1) populations
    double cov[10];
    for (int k = 0; k < 10; k++) cov[k] = 0.0;
    const int b = local * B + t;
    if (b < S3) {
        int bb[3], p[3];
        const bool in = bbox_pos(b, org, Sx, g, bb, p);
        const bool fo = in && !pnode(p[0], p[1], p[2], X, D.R2, g);
        const bool fn = in && !pnode(p[0], p[1], p[2], Xn, D.R2, g);
        uint32_t m = 0u;
        if (in) {
            if (!fn) m |= MASK_SOLID;
            if (!fo && fn) m |= MASK_LOCAL;
#pragma unroll
            for (int i = 1; i < Q; i++) {
                int sx = p[0] - cx(i), sy = p[1] - cy(i), sz = p[2] - cz(i);
                if (!(wrap1(sx, g.nx, g.wx) && wrap1(sy, g.ny, g.wy) && wrap1(sz, g.nz, g.wz)))
                    continue;
                if (pnode(sx, sy, sz, X, D.R2, g)) m |= 1u << i;
            }
        }
        pmask[b] = m;
        if (fo) {
            T d[2][Q];
            pull_node(pc, p[0], p[1], p[2], m & ~(MASK_SOLID | MASK_LOCAL), d);
            double jt[3] = {0.0, 0.0, 0.0}, rho[2];
            for (int l = 0; l < 2; l++) {
                T rd, jl[3], mm[Q];
                component_modes(d[l], rd, jl, mm);
                rho[l] = D.rho0[l] + (double)rd;
                for (int q = 0; q < 3; q++) jt[q] += (double)jl[q];
            }
            raw[b] = rho[0];
            raw[S3 + b] = rho[1];
            if (!fn) {
                const double rr[3] = {sepd(p[0] - Xn[0], g.nx, g.wx), sepd(p[1] - Xn[1], g.ny, g.wy),
                                      sepd(p[2] - Xn[2], g.nz, g.wz)};
                cov[0] += jt[0]; cov[1] += jt[1]; cov[2] += jt[2];
                cov[3] += rr[1] * jt[2] - rr[2] * jt[1];
                cov[4] += rr[2] * jt[0] - rr[0] * jt[2];
                cov[5] += rr[0] * jt[1] - rr[1] * jt[0];
                cov[6] += rho[0];
                cov[7] += rho[1];
                cov[9] += 1.0;
            }
        }
        if (in && !fn) cov[8] += 1.0;
        flags[b] = (uint8_t)((in ? 1 : 0) | (fo ? 2 : 0) | (fn ? 4 : 0));
    }
    block_sum<B, 10>(cov, red);
    if (t == 0) {
        double *p = a.part3 + D.part3_off + (int64_t)local * PART;
        for (int k = 0; k < 10; k++) p[k] = cov[k];
    }
}

// mean density of the nodes around bbox entry bb that are fluid at X^n and
// at X^{n+1}; rho0 when there is none
__device__ __forceinline__ void mean_kept_neighbours(const int (&bb)[3], int Sx, int S3,
                                                     const uint8_t *flags, const double *raw,
                                                     const double *rho0, double (&rb)[2]) {
    double s0 = 0.0, s1 = 0.0;
    int cnt = 0;
#pragma unroll
    for (int i = 1; i < Q; i++) {
        const int qx = bb[0] + cx(i), qy = bb[1] + cy(i), qz = bb[2] + cz(i);
        if (qx < 0 || qy < 0 || qz < 0 || qx >= Sx || qy >= Sx || qz >= Sx) continue;
        const int qb = (qz * Sx + qy) * Sx + qx;
        if ((flags[qb] & 7) != 7) continue;
        s0 += raw[qb];
        s1 += raw[S3 + qb];
        cnt++;
    }
    rb[0] = cnt > 0 ? s0 / cnt : rho0[0];
    rb[1] = cnt > 0 ? s1 / cnt : rho0[1];
}

// =========================================================== k_particle_b
// One thread per node of the new bounding box.  Uncovered nodes (particle at
// X^n, fluid at X^{n+1}) get f_eq(rho_bar, u_b) in their own slots, rho_bar
// being the mean density of their neighbours fluid at both times; particle
// nodes at X^{n+1} get the wetting-layer density: mean of their fluid
// neighbours + / - Delta rho (the mass correction delta is added where it is
// read).  The last workgroup sums the event partials, computes the global
// mass correction and publishes the state of step n+1.
template <typename S, typename T, int B>
__global__ __launch_bounds__(B) void k_particle_b(ParticleArgs a) {
    __shared__ double red[(B / 64) * 20];
    __shared__ int last;
    const int wg = blockIdx.x;
    const int r = find_rep(a.k3_begin, a.nrep, wg);
    const RepDesc &D = a.desc[r];
    RepState *st = a.state + r;
    const Geo g = geo_of(D);
    const int t = threadIdx.x;
    const int local = wg - D.k3_begin;
    double *series = a.series + D.series_off;

    if (!D.has_particle) {
        if (t == 0) {
            const int64_t n = st->step;
            double *s = series + 3 * (n % D.series_cap);
            s[0] = s[1] = s[2] = 0.0;
            st->delta[0] = st->delta[1] = 0.0;
            st->local_read = 0;
            st->step = n + 1;
        }
        return;
    }
    const int32_t org[3] = {st->orgn[0], st->orgn[1], st->orgn[2]};
    const double Xn[3] = {st->Xn[0], st->Xn[1], st->Xn[2]};
    const double Un[3] = {st->Un[0], st->Un[1], st->Un[2]};
    const double Wn[3] = {st->Wn[0], st->Wn[1], st->Wn[2]};
    const int Sx = D.S, S3 = Sx * Sx * Sx;
    const double *raw = a.raw + D.bbox_off * 2;
    double *vrho = a.vrho + D.bbox_off * 2;
    const uint8_t *flags = a.flags + D.bbox_off;
    S *buf = reinterpret_cast<S *>(a.buf) + D.pop_off;
    const uint32_t N32 = (uint32_t)g.N;

    double unc[10];
    for (int k = 0; k < 10; k++) unc[k] = 0.0;
    const int b = local * B + t;
    if (b < S3) {
        const int f = flags[b];
        int bb[3], p[3];
        bbox_pos(b, org, Sx, g, bb, p);
        if ((f & 1) && !(f & 2) && (f & 4)) {  // uncovered
            double rb[2];
            mean_kept_neighbours(bb, Sx, S3, flags, raw, D.rho0, rb);
            const double rr[3] = {sepd(p[0] - Xn[0], g.nx, g.wx), sepd(p[1] - Xn[1], g.ny, g.wy),
                                  sepd(p[2] - Xn[2], g.nz, g.wz)};
            const double u[3] = {Un[0] + Wn[1] * rr[2] - Wn[2] * rr[1],
                                 Un[1] + Wn[2] * rr[0] - Wn[0] * rr[2],
                                 Un[2] + Wn[0] * rr[1] - Wn[1] * rr[0]};
            const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
            const uint32_t own = nidx(p[0], p[1], p[2], g);
            for (int i = 0; i < Q; i++) {
                const double cu = cx(i) * u[0] + cy(i) * u[1] + cz(i) * u[2];
                const double e = 1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu;
                for (int l = 0; l < 2; l++) {
                    const double wr = wgt(i) * D.rho0[l];
                    const double dev = wgt(i) * rb[l] * e - wr;
                    st_dev<S, T>(buf + ((uint32_t)(l * Q + i) * N32 + own), T(dev),
                                 Rel<S>::value ? T(1.0 / wr) : T(1));
                }
            }
            const double mom[3] = {(rb[0] + rb[1]) * u[0], (rb[0] + rb[1]) * u[1],
                                   (rb[0] + rb[1]) * u[2]};
            unc[0] += mom[0]; unc[1] += mom[1]; unc[2] += mom[2];
            unc[3] += rr[1] * mom[2] - rr[2] * mom[1];
            unc[4] += rr[2] * mom[0] - rr[0] * mom[2];
            unc[5] += rr[0] * mom[1] - rr[1] * mom[0];
            unc[6] += rb[0];
            unc[7] += rb[1];
            unc[9] += 1.0;
        } else if ((f & 1) && !(f & 4)) {  // particle node at X^{n+1}: wetting layer
            double s0 = 0.0, s1 = 0.0;
            int cnt = 0;
#pragma unroll
            for (int i = 1; i < Q; i++) {
                const int qx = bb[0] + cx(i), qy = bb[1] + cy(i), qz = bb[2] + cz(i);
                if (qx < 0 || qy < 0 || qz < 0 || qx >= Sx || qy >= Sx || qz >= Sx) continue;
                const int qb = (qz * Sx + qy) * Sx + qx;
                const int fq = flags[qb];
                if (!((fq & 1) && (fq & 4))) continue;
                double r0, r1;
                if (fq & 2) {
                    r0 = raw[qb];
                    r1 = raw[S3 + qb];
                } else {  // neighbour uncovered at this step: its f_eq density
                    const int qq[3] = {qx, qy, qz};
                    double rb[2];
                    mean_kept_neighbours(qq, Sx, S3, flags, raw, D.rho0, rb);
                    r0 = rb[0];
                    r1 = rb[1];
                }
                s0 += r0;
                s1 += r1;
                cnt++;
            }
            vrho[b] = cnt > 0 ? s0 / cnt + D.drho : 0.0;
            vrho[S3 + b] = cnt > 0 ? s1 / cnt - D.drho : 0.0;
        }
    }
    block_sum<B, 10>(unc, red);
    if (t == 0) {
        double *p = a.part3b + D.part3_off + (int64_t)local * PART;
        for (int k = 0; k < 10; k++) p[k] = unc[k];
    }
    __threadfence();
    __syncthreads();
    if (t == 0) last = (atomicAdd(&st->k3_done, 1u) == (unsigned)(D.k3_count - 1));
    __syncthreads();
    if (!last) return;
    __threadfence();

    // ---- last workgroup: event sums (fixed order), mass correction, new state
    double tot[20];
    for (int k = 0; k < 20; k++) tot[k] = 0.0;
    for (int w = t; w < D.k3_count; w += B) {
        const double *pa = a.part3 + D.part3_off + (int64_t)w * PART;
        const double *pb = a.part3b + D.part3_off + (int64_t)w * PART;
        for (int k = 0; k < 10; k++) {
            tot[k] += pa[k];
            tot[10 + k] += pb[k];
        }
    }
    block_sum<B, 20>(tot, red);
    if (t != 0) return;
    const double *utot = tot + 10;
    const double nf = (double)D.N - tot[8];
    const int64_t n = st->step;
    double *s = series + 3 * (n % D.series_cap);
    const int n3[3] = {g.nx, g.ny, g.nz};
    const bool w3[3] = {g.wx, g.wy, g.wz};
    bool bad = false;
    for (int l = 0; l < 2; l++)
        st->delta[l] = -(st->dMbb[l] - tot[6 + l] + utot[6 + l]) / nf;
    for (int q = 0; q < 3; q++) {
        st->Xp[q] = st->X[q];
        st->X[q] = Xn[q];
        st->U[q] = Un[q];
        st->W[q] = Wn[q];
        st->F[q] = st->Fn[q];
        st->T[q] = st->Tn[q];
        st->Pev[q] = tot[q] - utot[q];
        st->Lev[q] = tot[3 + q] - utot[3 + q];
        st->org[q] = org[q];
        s[q] = Un[q];
        if (!(fabs(Un[q]) < 0.5) || !isfinite(st->Fn[q])) bad = true;
        if (w3[q] && (Xn[q] - D.radius < -0.5 || Xn[q] + D.radius > n3[q] - 0.5)) bad = true;
    }
    st->n_fluid = nf;
    st->n_cov += (int64_t)tot[9];
    st->n_unc += (int64_t)utot[9];
    st->n_links = (int64_t)st->nlinks;
    st->local_read = 0;
    if (bad) st->flags |= FLAG_UNSTABLE;
    st->k3_done = 0;
    st->step = n + 1;
    __threadfence();
}

// ================================================================ k_init
// f(0) = w_i rho_l(x) with rho_l = rho0_l + amp (2u - 1), u from Philox with
// counter (node, 0, 0, 1), word l; written to the node's own slots.
template <typename S>
__global__ __launch_bounds__(256) void k_init(InitArgs a) {
    __shared__ double red[4 * 2];
    const int wg = blockIdx.x;
    const int r = find_rep(a.init_begin, a.nrep, wg);
    const RepDesc &D = a.desc[r];
    const RepState &st = a.state[r];
    const Geo g = geo_of(D);
    const int64_t n = (int64_t)(wg - a.init_begin[r]) * 256 + threadIdx.x;
    double m[2] = {0.0, 0.0};
    if (n < g.N) {
        const int x = (int)(n % g.nx), y = (int)((n / g.nx) % g.ny);
        const int z = (int)(n / ((int64_t)g.nx * g.ny));
        const bool solid = D.has_particle && pnode(x, y, z, st.X, D.R2, g);
        uint32_t c0 = (uint32_t)n, c1 = 0u, c2 = 0u, c3 = 1u;
        philox4x32_10(c0, c1, c2, c3, D.key0, D.key1);
        const uint32_t w[2] = {c0, c1};
        S *dst = reinterpret_cast<S *>(a.buf) + D.pop_off;
        for (int l = 0; l < 2; l++) {
            const double rho = D.rho0[l] + D.init_amp * (2.0 * (((double)w[l] + 0.5) * 0x1p-32) - 1.0);
            if (!solid) m[l] = rho;
            for (int i = 0; i < Q; i++) {
                const double wr = wgt(i) * D.rho0[l];
                const double dev = solid ? 0.0 : wgt(i) * rho - wr;
                st_dev<S, double>(dst + (int64_t)(l * Q + i) * g.N + n, dev,
                                  Rel<S>::value ? 1.0 / wr : 1.0);
            }
        }
    }
    block_sum<256, 2>(m, red);
    if (threadIdx.x == 0) {
        a.mass[2 * wg] = m[0];
        a.mass[2 * wg + 1] = m[1];
    }
}

// ============================================================= k_export
// f_{l i}(x, n) in FP64 for the nodes of planes [z_begin, z_end) of one
// replica (particle nodes: 0).
template <typename S, typename T>
__global__ __launch_bounds__(256) void k_export(ExportArgs a) {
    const RepDesc &D = a.desc[a.rep];
    const RepState &st = a.state[a.rep];
    const Geo g = geo_of(D);
    const int64_t plane = (int64_t)g.nx * g.ny;
    const int64_t cnt = plane * (a.z_end - a.z_begin);
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= cnt) return;
    const int x = (int)(k % g.nx), y = (int)((k / g.nx) % g.ny), z = a.z_begin + (int)(k / plane);
    const PullCtx<S, T> pc = pull_ctx<S, T>(a.src, D, st, true);
    int b = -1;
    const uint32_t m = D.has_particle ? node_mask(x, y, z, a.pmask + D.bbox_off, st.org, D.S, g, b) : 0u;
    const bool solid = m & MASK_SOLID;
    T d[2][Q];
    if (!solid) pull_node(pc, x, y, z, m, d);
    for (int l = 0; l < 2; l++)
        for (int i = 0; i < Q; i++)
            a.out[(int64_t)(l * Q + i) * cnt + k] = solid ? 0.0 : wgt(i) * D.rho0[l] + (double)d[l][i];
}

// ============================================================= k_fields_a
// Density seen by the Shan-Chen force (wetting layer on particle nodes),
// total momentum and a solid flag per node, into scratch.
template <typename S, typename T>
__global__ __launch_bounds__(256) void k_fields_a(FieldArgs a) {
    const RepDesc &D = a.desc[a.rep];
    const RepState &st = a.state[a.rep];
    const Geo g = geo_of(D);
    const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (n >= g.N) return;
    const int x = (int)(n % g.nx), y = (int)((n / g.nx) % g.ny);
    const int z = (int)(n / ((int64_t)g.nx * g.ny));
    double *rt = a.scratch, *jt = a.scratch + 2 * g.N, *sol = a.scratch + 8 * g.N;
    int b = -1;
    const uint32_t m = D.has_particle ? node_mask(x, y, z, a.pmask + D.bbox_off, st.org, D.S, g, b) : 0u;
    if (m & MASK_SOLID) {
        const int S3 = D.S * D.S * D.S;
        const double *vrho = a.vrho + D.bbox_off * 2;
        rt[n] = vrho[b] + st.delta[0];
        rt[g.N + n] = vrho[S3 + b] + st.delta[1];
        for (int q = 0; q < 3; q++) jt[q * g.N + n] = 0.0;
        sol[n] = 1.0;
        return;
    }
    const PullCtx<S, T> pc = pull_ctx<S, T>(a.src, D, st, true);
    T d[2][Q];
    pull_node(pc, x, y, z, m, d);
    double jtot[3] = {0.0, 0.0, 0.0};
    for (int l = 0; l < 2; l++) {
        T rd, jl[3], mm[Q];
        component_modes(d[l], rd, jl, mm);
        rt[l * g.N + n] = D.rho0[l] + (double)rd;
        for (int q = 0; q < 3; q++) jtot[q] += (double)jl[q];
    }
    for (int q = 0; q < 3; q++) jt[q * g.N + n] = jtot[q];
    sol[n] = 0.0;
}

// ============================================================== launchers
template <typename S, typename T>
hipError_t launch_main_t(const MainArgs &a, int grid, int block, size_t lds, hipStream_t s) {
    const bool tau1 = a.tau1 != 0;
    switch (block) {
    case 256:
        if (tau1) hipLaunchKernelGGL((k_main<S, T, 256, true>), dim3(grid), dim3(256), lds, s, a);
        else hipLaunchKernelGGL((k_main<S, T, 256, false>), dim3(grid), dim3(256), lds, s, a);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename S, typename T>
hipError_t launch_links_t(const LinkArgs &a, int grid, hipStream_t s) {
    hipLaunchKernelGGL((k_links<S, T, 256>), dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <typename S, typename T>
hipError_t launch_particle_t(const ParticleArgs &a, int grid, hipStream_t s) {
    hipLaunchKernelGGL((k_particle_a<S, T, 256>), dim3(grid), dim3(256), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_particle_b<S, T, 256>), dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <typename S, typename T>
hipError_t launch_init_t(const InitArgs &a, int grid, hipStream_t s) {
    hipLaunchKernelGGL(k_init<S>, dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <typename S, typename T>
hipError_t launch_export_t(const ExportArgs &a, int64_t count, hipStream_t s) {
    hipLaunchKernelGGL((k_export<S, T>), dim3((int)((count + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <typename S, typename T>
hipError_t launch_fields_a_t(const FieldArgs &a, int64_t N, hipStream_t s) {
    hipLaunchKernelGGL((k_fields_a<S, T>), dim3((int)((N + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

#define LBM_INSTANTIATE(SUFFIX, S, T)                                                              \
    hipError_t launch_main_##SUFFIX(const MainArgs &a, int grid, int block, size_t lds,          \
                                    hipStream_t s) {                                               \
        return launch_main_t<S, T>(a, grid, block, lds, s);                                        \
    }                                                                                              \
    hipError_t launch_links_##SUFFIX(const LinkArgs &a, int grid, hipStream_t s) {                 \
        return launch_links_t<S, T>(a, grid, s);                                                   \
    }                                                                                              \
    hipError_t launch_particle_##SUFFIX(const ParticleArgs &a, int grid, hipStream_t s) {          \
        return launch_particle_t<S, T>(a, grid, s);                                                \
    }                                                                                              \
    hipError_t launch_init_##SUFFIX(const InitArgs &a, int grid, hipStream_t s) {                  \
        return launch_init_t<S, T>(a, grid, s);                                                    \
    }                                                                                              \
    hipError_t launch_export_##SUFFIX(const ExportArgs &a, int64_t count, hipStream_t s) {         \
        return launch_export_t<S, T>(a, count, s);                                                 \
    }                                                                                              \
    hipError_t launch_fields_a_##SUFFIX(const FieldArgs &a, int64_t N, hipStream_t s) {            \
        return launch_fields_a_t<S, T>(a, N, s);                                                   \
    }

}  // namespace lbm
