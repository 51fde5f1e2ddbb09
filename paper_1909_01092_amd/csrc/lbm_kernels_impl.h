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
// Storage.  Each replica keeps its populations on a lattice padded by one
// ghost layer per side, [component][direction][z+1][y+1][x+1].  Node x pulls
// population i of step n from the padded position x - c_i, slot i.  Whoever
// produces a value that does not arrive by plain streaming writes it into
// exactly that slot: a node next to a wall writes its bounced value into the
// wall's ghost, a node next to a periodic face writes the wrapped copy into
// the ghost, the link kernel writes the sphere's moving-wall bounce-back into
// the particle node's slot, and uncovered nodes get f_eq written into the
// slots they pull from.  Every pull is therefore 38 loads at wave-uniform
// offsets from the node's own index.
//
// One step = k_main (all nodes of all replicas) + k_links + k_particle
// (bounding box of each sphere).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm_kernels.h"
#include "lbm_math.h"
#include "lbm_types.h"

namespace lbm {

template <typename T>
__device__ __forceinline__ Coef<T> make_coef_dev(const RepDesc &D) {
    return coef_of<T>(D);
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
    int64_t N;          // nodes
    int PX, PY;         // padded row and plane widths (nx + 2, ny + 2)
    uint32_t NP;        // padded nodes per component and direction
};

__device__ __forceinline__ Geo geo_of(const RepDesc &D) {
    Geo g;
    g.nx = D.nx; g.ny = D.ny; g.nz = D.nz;
    g.wx = D.walls & 1u; g.wy = D.walls & 2u; g.wz = D.walls & 4u;
    g.N = D.N;
    g.PX = D.nx + 2;
    g.PY = D.ny + 2;
    g.NP = (uint32_t)D.NP;
    return g;
}

// padded index of lattice position (x, y, z), -1 <= x <= nx etc.
__device__ __forceinline__ uint32_t pidx(int x, int y, int z, const Geo &g) {
    return (uint32_t)(x + 1) + (uint32_t)g.PX * ((uint32_t)(y + 1) + (uint32_t)g.PY * (uint32_t)(z + 1));
}
// unpadded node index (noise counter, fields)
__device__ __forceinline__ uint32_t nidx(int x, int y, int z, const Geo &g) {
    return (uint32_t)x + (uint32_t)g.nx * ((uint32_t)y + (uint32_t)g.ny * (uint32_t)z);
}
// bring a coordinate one layer outside the box back in; false = wall layer
__device__ __forceinline__ bool wrap1(int &v, int n, bool wall) {
    if (v < 0 || v >= n) {
        if (wall) return false;
        v = v < 0 ? v + n : v - n;
    }
    return true;
}
// padded-index offset of direction i
__device__ __forceinline__ int32_t doff(int i, const Geo &g) {
    return cx(i) + g.PX * (cy(i) + g.PY * cz(i));
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

// ------------------------------------------------------------------ pulling
// Populations f_{l i}(x, n) of a fluid node in deviation form: slot i at the
// padded position x - c_i (see the storage note at the top).
template <typename S, typename T>
struct PullCtx {
    const S *src;          // replica block
    int32_t NP, PX, PXY;   // padded sizes
    T scale[2];            // FP16 relative storage: rho0_l (times w_i per slot)
};

template <typename S, typename T>
__device__ __forceinline__ PullCtx<S, T> pull_ctx(const void *buf, const RepDesc &D, const Geo &g) {
    PullCtx<S, T> pc;
    pc.src = reinterpret_cast<const S *>(buf) + D.pop_off;
    pc.NP = (int32_t)g.NP;
    pc.PX = g.PX;
    pc.PXY = g.PX * g.PY;
    for (int l = 0; l < 2; l++) pc.scale[l] = Rel<S>::value ? T(D.rho0[l]) : T(1);
    return pc;
}

// element at a wave-uniform base plus a per-lane byte offset (lets the
// compiler use scalar-base + 32-bit vector-offset addressing)
template <typename S>
__device__ __forceinline__ const S &at(const S *base, uint32_t byte_off) {
    return *reinterpret_cast<const S *>(reinterpret_cast<const char *>(base) + byte_off);
}
template <typename S>
__device__ __forceinline__ S &at(S *base, uint32_t byte_off) {
    return *reinterpret_cast<S *>(reinterpret_cast<char *>(base) + byte_off);
}

template <typename S, typename T>
__device__ __forceinline__ void pull_node(const PullCtx<S, T> &c, uint32_t own, T (&d)[2][Q]) {
    const S *b0 = c.src, *b1 = c.src + Q * c.NP;
#pragma unroll
    for (int i = 0; i < Q; i++) {
        const T w = T(wgt(i));
        const int32_t off = cx(i) + c.PX * cy(i) + c.PXY * cz(i);
        const uint32_t vo = (own + (uint32_t)(i * c.NP - off)) * (uint32_t)sizeof(S);
        d[0][i] = ld_dev<S, T>(&at(b0, vo), w * c.scale[0]);
        d[1][i] = ld_dev<S, T>(&at(b1, vo), w * c.scale[1]);
    }
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
// x + (x moved across lanes by the DPP pattern CTRL), FP64 as two 32-bit moves
template <int CTRL>
__device__ __forceinline__ double dpp_add(double x) {
    const int lo = __double2loint(x), hi = __double2hiint(x);
    const int plo = __builtin_amdgcn_update_dpp(0, lo, CTRL, 0xf, 0xf, false);
    const int phi = __builtin_amdgcn_update_dpp(0, hi, CTRL, 0xf, 0xf, false);
    return x + __hiloint2double(phi, plo);
}

// x + (x of the lane 16 or 32 apart), the lower lane's value first in every
// lane, FP64 as two 32-bit swaps (v_permlane16_swap / v_permlane32_swap:
// rows 0-1 and 2-3, or the two halves of the wave, exchanged)
__device__ __forceinline__ double add_row_pair(double x) {
    const int lo = __double2loint(x), hi = __double2hiint(x);
    const auto l = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    const auto h = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    return __hiloint2double(h[0], l[0]) + __hiloint2double(h[1], l[1]);
}
__device__ __forceinline__ double add_half_pair(double x) {
    const int lo = __double2loint(x), hi = __double2hiint(x);
    const auto l = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    const auto h = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    return __hiloint2double(h[0], l[0]) + __hiloint2double(h[1], l[1]);
}

// Sum over the 64 lanes of a wave, in a fixed order and bitwise the same in
// every lane: lane pairs, then quads, 8-lane halves and 16-lane rows are
// combined with DPP permutations (quad swaps, half-row and row mirrors; each
// step adds two equal partial sums in either order, so all lanes agree), then
// rows 0 + 1 and 2 + 3 and the two halves with lane swaps (lower part first).
// Everything stays in vector registers.  All lanes of the wave must be active.
template <int NV>
__device__ __forceinline__ void wave_sum(double (&v)[NV]) {
#pragma unroll
    for (int k = 0; k < NV; k++) {
        double x = v[k];
        x = dpp_add<0xB1>(x);   // quad_perm [1,0,3,2]
        x = dpp_add<0x4E>(x);   // quad_perm [2,3,0,1]
        x = dpp_add<0x141>(x);  // row_half_mirror
        x = dpp_add<0x140>(x);  // row_mirror
        x = add_row_pair(x);
        v[k] = add_half_pair(x);
    }
}

// fixed-order sum over the workgroup, result in every thread
template <int B, int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double *red /* [B/64][NV] */) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    wave_sum<NV>(v);
    __syncthreads();  // earlier readers of red are done
    if (lane == 0)
        for (int k = 0; k < NV; k++) red[wave * NV + k] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; k++) {
        double s = 0.0;
        for (int w = 0; w < B / 64; w++) s += red[w * NV + k];
        v[k] = s;
    }
}

// Workgroups are dispatched to the 8 XCDs round-robin; give each XCD a
// contiguous run of logical tiles so halo rows and planes shared by
// neighbouring tiles are read through the same L2.
__device__ __forceinline__ int xcd_logical(int b, int G) {
    const int q = G >> 3, r = G & 7, xcd = b & 7, slot = b >> 3;
    return xcd < r ? xcd * (q + 1) + slot : r * (q + 1) + (xcd - r) * q + slot;
}

// ================================================================ k_main
// Workgroup = ty full x-rows of one replica, marching over cz z-planes.
// Density deviations of the tile plus a one-node halo (rows y0-1 and
// y0+rows, planes z-1 and z+1) sit in a 4-plane LDS ring; halo densities are
// recomputed from pulled populations, so no density field goes through HBM.
// The density and momenta of the next plane stay in registers while the
// current plane collides.  The sphere enters only through the solid flags
// and wetting-layer densities of its bounding box; every FP64 particle
// computation lives in the bounding-box kernels.
// FP32 arithmetic with all relaxation times 1 (FP32 or FP16 storage): both
// components unrolled and the kernel held to 128 VGPRs (four waves per SIMD).
// Other forms keep the component loop rolled and their natural allocation.
template <typename S, typename T, bool TAU1>
constexpr bool main_fast_form = sizeof(T) == 4 && TAU1;
template <typename S, typename T, bool TAU1>
constexpr bool main_unroll = sizeof(T) == 4 && TAU1;

// GROUP: fluids may hold several spheres (their boxes are searched too); a
// separate instantiation, so the single-sphere form keeps its registers.
// NOISE: some replica of the launch has kT > 0.  Every node then draws its
// normals; a replica with kT = 0 has zero amplitudes and takes none of them
// (products with zero).  Without it no normals are drawn.  Being a compile-
// time choice, the noise-free form costs the noisy one nothing.
template <typename S, typename T, int B, bool TAU1, bool GROUP, bool NOISE>
__global__ __launch_bounds__(B) __attribute__((amdgpu_waves_per_eu(main_fast_form<S, T, TAU1> ? 4 : 1)))
void k_main(MainArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    T *lds = reinterpret_cast<T *>(smem);

    const int wg = xcd_logical(blockIdx.x, gridDim.x);
    const int r = find_rep(a.wg_begin, a.nrep, wg);
    const RepDesc D = a.desc[r];  // by value: no reload after stores
    RepState *stp = a.state + r;
    const Geo g = geo_of(D);
    const int nx = g.nx, ty = D.ty, zc = D.cz;
    const int local = wg - D.wg_begin;
    const int yt = local % D.nty, ch = local / D.nty;
    const int y0 = yt * ty, rows = min(ty, g.ny - y0);
    const int z0 = ch * zc, z1 = min(z0 + zc, g.nz);
    const int t = threadIdx.x;
    const int nin = nx * rows;
    const bool inner = t < nin;
    const int x = inner ? t % nx : 0, yl = inner ? t / nx : 0;
    const int y = y0 + yl;
    const int pr = (ty + 2) * nx;  // LDS elements per plane and component

    const bool hp = D.has_particle;
    const int nsph = GROUP ? D.n_sph : 1;
    const bool ghost_fill = D.ghost_fill;
    const PullCtx<S, T> pc = pull_ctx<S, T>(a.src, D, g);
    const T dl[2] = {T(stp->delta[0]), T(stp->delta[1])};
    const double dld[2] = {stp->delta[0], stp->delta[1]};
    const uint32_t step = (uint32_t)stp->step;
    const int32_t org[3] = {stp->org[0], stp->org[1], stp->org[2]};
    const int Sx = D.S, S3 = Sx * Sx * Sx;
    const uint32_t *__restrict__ pmask = a.pmask + D.bbox_off;
    const double *__restrict__ vrho = a.vrho + D.bbox_off * 2;
    double *__restrict__ rho_n = a.rho_n + D.bbox_off * 2;
    S *__restrict__ dst = reinterpret_cast<S *>(a.dst) + D.pop_off;
    const uint32_t NP = g.NP;
    const double rho0d[2] = {D.rho0[0], D.rho0[1]};
    const T G = sizeof(T) == 4 ? T(D.G32) : T(D.G);
    const T af[3] = {sizeof(T) == 4 ? T(D.af32[0]) : T(D.af[0]), sizeof(T) == 4 ? T(D.af32[1]) : T(D.af[1]),
                     sizeof(T) == 4 ? T(D.af32[2]) : T(D.af[2])};
    const uint32_t key0 = D.key0, key1 = D.key1;
    const Coef<T> cf = make_coef_dev<T>(D);
    uint32_t k0 = key0, k1 = key1;
    PullCtx<S, T> pcl = pc;

    // four plane slots: the fill of the next plane never lands on a slot the
    // collision of the current plane still reads, so one barrier per plane
    auto L = [&](int zp, int l, int row, int xx) -> T & {
        const int slot = zp & 3;
        return lds[(slot * 2 + l) * pr + (row + 1) * nx + xx];
    };

    // density deviation of a box node: pulled (plus the mass correction), or
    // the wetting-layer value on particle nodes; fluid nodes also return
    // their moments
    auto node_density = [&](int xx, int yy, int zz, NodeM<T, TAU1> &s, T &rA, T &rB) -> bool {
        int b = -1;
        if (hp) b = bbox_index(xx, yy, zz, org, Sx, g);
        if (b < 0 || !(pmask[b] & MASK_SOLID)) {
            // the group's other spheres (their boxes are disjoint from this
            // one's and from each other, so at most one holds the node)
            int64_t vi = -1;
            int vs = 0;
            if (GROUP && nsph > 1 && b < 0) {
                for (int e = 1; e < nsph; e++) {
                    const RepDesc *De = a.desc + r + e;
                    const int Se = De->S;
                    const int be = bbox_index(xx, yy, zz, a.state[r + e].org, Se, g);
                    if (be < 0) continue;
                    if (a.pmask[De->bbox_off + be] & MASK_SOLID) {
                        vi = 2 * De->bbox_off + be;
                        vs = Se * Se * Se;
                    }
                    break;
                }
            }
            if (vi < 0) {
                T d[2][Q];
                pull_node(pcl, pidx(xx, yy, zz, g), d);
                node_moments(d, s);
                s.rd[0] += dl[0];
                s.rd[1] += dl[1];
                rA = s.rd[0];
                rB = s.rd[1];
                return true;
            }
            rA = T(a.vrho[vi] + dld[0] - rho0d[0]);
            rB = T(a.vrho[vi + vs] + dld[1] - rho0d[1]);
            return false;
        }
        rA = T(vrho[b] + dld[0] - rho0d[0]);
        rB = T(vrho[S3 + b] + dld[1] - rho0d[1]);
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

    const int xm = mirror1(x - 1, nx, g.wx), xp = mirror1(x + 1, nx, g.wx);
    // x / y faces of this lane's node as bits (x low, x high, y low, y high)
    uint32_t xyface = (x == 0 ? 1u : 0u) | (x == nx - 1 ? 2u : 0u) | (y == 0 ? 4u : 0u) |
                      (y == g.ny - 1 ? 8u : 0u);

    // Plane zp is filled while the plane filled before it collides.  Odd
    // z-chunks march downwards, so two neighbouring chunks read the halo
    // planes they share at the same time (both at their start or both at
    // their end) and the second read hits L2.
    const int dir = (ch & 1) ? -1 : 1;
    const int zfirst = dir > 0 ? z0 - 1 : z1;
    const int nplanes = z1 - z0 + 2;
    for (int k = 0; k < nplanes; k++) {
        // keep uniform values derived from these roots inside the loop (scalar
        // recomputation is cheaper than spilling hoisted copies)
        asm volatile("" : "+s"(k0), "+s"(k1), "+s"(pcl.NP), "+s"(pcl.PX), "+s"(pcl.PXY));
        // face tests are redone per plane from these bits instead of being
        // hoisted as lane masks that would crowd the scalar registers
        asm volatile("" : "+v"(xyface));
        const int zp = zfirst + dir * k;
        const NodeM<T, TAU1> cur = nxt;
        const bool cur_fluid = nxt_fluid;
        fill(zp);
        __syncthreads();
        if (k < 2) continue;
        const int z = zp - dir;
        if (inner && cur_fluid) {
            const uint32_t own = pidx(x, y, z, g);
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
            if (hp) {  // densities near the spheres, for the link kernel
                const int b = bbox_index(x, y, z, org, Sx, g);
                if (b >= 0) {
                    rho_n[b] = (double)rl[0];
                    rho_n[S3 + b] = (double)rl[1];
                } else if (GROUP && nsph > 1) {
                    for (int e = 1; e < nsph; e++) {
                        const RepDesc *De = a.desc + r + e;
                        const int Se = De->S;
                        const int be = bbox_index(x, y, z, a.state[r + e].org, Se, g);
                        if (be < 0) continue;
                        double *rn = a.rho_n + 2 * De->bbox_off;
                        rn[be] = (double)rl[0];
                        rn[Se * Se * Se + be] = (double)rl[1];
                        break;
                    }
                }
            }
            T F[2][3];
#pragma unroll
            for (int q = 0; q < 3; q++) {
                F[0][q] = -G * rl[0] * grad[1][q] + rl[0] * af[q];
                F[1][q] = -G * rl[1] * grad[0][q] + rl[1] * af[q];
            }
            const uint32_t node = (uint32_t)(x + nx * (y + g.ny * z));
            T u[3], xid[3];
            T zz[36];
            if constexpr (NOISE) noise_block<T>(node, step, 8u, k0, k1, zz + 32);
            else zz[32] = zz[33] = zz[34] = T(0);
            common_velocity(rd, j, F, zz, cf, u, xid);
            const bool zlo = z == 0, zhi = z == g.nz - 1;
            const bool yzface = (xyface & 12u) != 0u || zlo || zhi;
            const bool xonly = !yzface && (xyface & 3u) != 0u;
            constexpr int kCompUnroll = main_unroll<S, T, TAU1> ? 2 : 1;
#pragma unroll kCompUnroll
            for (int l = 0; l < 2; l++) {
                // this component's values (selected, so nothing is indexed by l)
                const T rdl = l ? rd[1] : rd[0];
                const T jl[3] = {l ? j[1][0] : j[0][0], l ? j[1][1] : j[0][1], l ? j[1][2] : j[0][2]};
                const T Fl[3] = {l ? F[1][0] : F[0][0], l ? F[1][1] : F[0][1], l ? F[1][2] : F[0][2]};
                const T r0l = l ? cf.rho0[1] : cf.rho0[0];
                const T sig = l ? T(-1) : T(1);
                T zl[16];
                if constexpr (NOISE) {
#pragma unroll
                    for (int b = 0; b < 4; b++)
                        noise_block<T>(node, step, (uint32_t)(4 * l + b), k0, k1, zl + 4 * b);
                } else {
#pragma unroll
                    for (int k = 0; k < 16; k++) zl[k] = T(0);
                }
                T out[Q];
                if constexpr (TAU1) {
                    relax_tau1(r0l, sig, rdl, jl, Fl, u, xid, zl, cf, out);
                } else {
                    T ml[Q];
#pragma unroll
                    for (int k = 4; k < Q; k++) ml[k] = l ? cur.m[1][k] : cur.m[0][k];
                    relax_component(r0l, sig, rdl, jl, ml, Fl, u, xid, zl, cf, out);
                }
                const T sc = Rel<S>::value ? r0l : T(1);
                S *dl_base = dst + l * Q * pcl.NP;
                const uint32_t own4 = own * (uint32_t)sizeof(S);
#pragma unroll
                for (int i = 0; i < Q; i++) {
                    const T inv = Rel<S>::value ? T(1) / (T(wgt(i)) * sc) : T(1);
                    S *col = dl_base + i * pcl.NP;
                    st_dev<S, T>(&at(col, own4), out[i], inv);
                }
                // Narrow rows: the two x-ghost elements between consecutive rows
                // share a cache line with both rows' ends, and a line left partly
                // unwritten costs a read-modify-write in HBM.  The x-face nodes
                // then also fill the ghost slots no node ever pulls from (c_x <= 0
                // beside x = 0, c_x >= 0 beside x = nx - 1), so every such line is
                // written whole.
                if (ghost_fill && (xyface & 3u) != 0u) {
                    const bool hi = xyface & 2u;
#pragma unroll
                    for (int i = 0; i < Q; i++) {
                        const T inv = Rel<S>::value ? T(1) / (T(wgt(i)) * sc) : T(1);
                        if (hi ? cx(i) >= 0 : cx(i) <= 0) {
                            const uint32_t e = (uint32_t)((int32_t)own + (hi ? 1 : -1) + i * pcl.NP);
                            st_dev<S, T>(&at(dl_base, e * (uint32_t)sizeof(S)), out[i], inv);
                        }
                    }
                }
                // A link that leaves the box also writes its value where the
                // receiver pulls it from: the wall ghost x + c_i, slot opp(i)
                // (half-way bounce-back), or the periodic image of x, slot i.
                // Only nodes on a face do.  Nodes on an x-face alone (the
                // common case: two per row) write the links with c_x pointing
                // out, at offsets uniform over the wave; nodes on a y- or
                // z-face take the general form.
                if (xonly) {
                    const bool hi = xyface & 2u;
#pragma unroll
                    for (int i = 1; i < Q; i++) {
                        if (cx(i) == 0) continue;
                        const T inv = Rel<S>::value ? T(1) / (T(wgt(i)) * sc) : T(1);
                        const int32_t so = g.wx ? opp(i) * pcl.NP + pcl.PX * cy(i) + pcl.PXY * cz(i) + cx(i)
                                                : i * pcl.NP - cx(i) * nx;
                        if ((cx(i) > 0) == hi) {
                            const uint32_t e = (uint32_t)((int32_t)own + so);
                            st_dev<S, T>(&at(dl_base, e * (uint32_t)sizeof(S)), out[i], inv);
                        }
                    }
                }
                if (yzface) {
                    const bool xlo = xyface & 1u, xhi = xyface & 2u, ylo = xyface & 4u, yhi = xyface & 8u;
#pragma unroll
                    for (int i = 1; i < Q; i++) {
                        const T inv = Rel<S>::value ? T(1) / (T(wgt(i)) * sc) : T(1);
                        const bool ex = cx(i) > 0 ? xhi : (cx(i) < 0 ? xlo : false);
                        const bool ey = cy(i) > 0 ? yhi : (cy(i) < 0 ? ylo : false);
                        const bool ez = cz(i) > 0 ? zhi : (cz(i) < 0 ? zlo : false);
                        if (ex || ey || ez) {
                            // element index from the component base: slot * NP + target,
                            // never negative (x + c_i lies in the ghost layer, the
                            // periodic image x - n c_i inside the box)
                            const bool bounce = (ex && g.wx) || (ey && g.wy) || (ez && g.wz);
                            const int32_t so = bounce ? opp(i) * pcl.NP + pcl.PX * cy(i) + pcl.PXY * cz(i) + cx(i)
                                                      : i * pcl.NP + (ex ? -cx(i) * nx : 0) +
                                                            (ey ? -cy(i) * g.ny * g.PX : 0) +
                                                            (ez ? -cz(i) * g.nz * g.PX * g.PY : 0);
                            const uint32_t e = (uint32_t)((int32_t)own + so);
                            st_dev<S, T>(&at(dl_base, e * (uint32_t)sizeof(S)), out[i], inv);
                        }
                    }
                }
            }
        }
    }
}

// ---------------------------------------------------- sphere-box helpers
// Sum of NV values over per-workgroup partials [count][PART] starting at k0,
// in a fixed order independent of the launch: lane l adds partials l, l + 64,
// ..., then a butterfly over the wave.  Every lane of every wave holds the
// same result, so no LDS or barrier is needed.
// A lane's partials are loaded CH at a time before they are added (in the
// same order), so a long list costs 1/CH of the dependent round trips.
template <int NV>
__device__ __forceinline__ void sum_partials(const double *part, int count, int k0, double (&v)[NV]) {
    constexpr int CH = NV > 16 ? 2 : 4;
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < NV; k++) v[k] = 0.0;
    for (int w0 = lane; w0 < count; w0 += CH * 64) {
        double c[CH][NV];
#pragma unroll
        for (int j = 0; j < CH; j++) {
            const int w = w0 + 64 * j;
            const double *p = part + (int64_t)(w < count ? w : 0) * PART + k0;
#pragma unroll
            for (int k = 0; k < NV; k++) c[j][k] = p[k];
        }
#pragma unroll
        for (int j = 0; j < CH; j++) {
            if (w0 + 64 * j >= count) break;
#pragma unroll
            for (int k = 0; k < NV; k++) v[k] += c[j][k];
        }
    }
    wave_sum<NV>(v);
}

// Neighbourhood of a box node p for the particle predicate: for p itself
// (bit 0) and each neighbour p + c_i (bit i), whether it lies inside the
// lattice (not a wall layer) and whether it is a particle node of the
// sphere at Xc.  The squared minimum-image separations along each axis are
// formed once for the positions p + {-1, 0, 1} (wrapped on periodic axes) and
// combined in the order pnode uses, so every decision is bitwise the one
// pnode takes for that node.  Held as two bit masks, not as arrays, so that
// nothing of it is kept in scratch memory.
struct Nbr {
    uint32_t ok;      // bit i: p + c_i inside the lattice
    uint32_t solid;   // bit i: p + c_i a particle node
};

__device__ __forceinline__ void nbr_of(const int (&p)[3], const double *Xc, double R2, const Geo &g,
                                       Nbr &nb) {
#pragma clang fp contract(off)
    const int n3[3] = {g.nx, g.ny, g.nz};
    const bool w3[3] = {g.wx, g.wy, g.wz};
    double sq[3][3];
    bool in[3][3];
#pragma unroll
    for (int ax = 0; ax < 3; ax++) {
#pragma unroll
        for (int k = 0; k < 3; k++) {
            int q = p[ax] + k - 1;
            in[ax][k] = w3[ax] ? (q >= 0 && q < n3[ax]) : true;
            if (!w3[ax]) q = q < 0 ? q + n3[ax] : (q >= n3[ax] ? q - n3[ax] : q);
            const double d = sepd((double)q - Xc[ax], n3[ax], w3[ax]);
            sq[ax][k] = d * d;
        }
    }
    nb.ok = 0u;
    nb.solid = 0u;
#pragma unroll
    for (int i = 0; i < Q; i++) {
        double d2 = sq[0][cx(i) + 1] + sq[1][cy(i) + 1];
        d2 = d2 + sq[2][cz(i) + 1];
        if (in[0][cx(i) + 1] && in[1][cy(i) + 1] && in[2][cz(i) + 1]) nb.ok |= 1u << i;
        if (d2 < R2) nb.solid |= 1u << i;
    }
}

__device__ __forceinline__ bool nbr_ok(const Nbr &nb, int i) { return (nb.ok >> i) & 1u; }

__device__ __forceinline__ bool pnode_nb(const Nbr &nb, int i) { return (nb.solid >> i) & 1u; }

// box coordinates of lattice node p in the box at org (periodic axes
// unwrapped next to it); false when p lies outside the box
__device__ __forceinline__ bool box_coords(const int (&p)[3], const int32_t *org, int S, const Geo &g,
                                           int (&bb)[3]) {
    const int n3[3] = {g.nx, g.ny, g.nz};
    const bool w3[3] = {g.wx, g.wy, g.wz};
    bool in = true;
#pragma unroll
    for (int ax = 0; ax < 3; ax++) {
        int v = p[ax] - org[ax];
        if (!w3[ax]) { if (v < 0) v += n3[ax]; else if (v >= n3[ax]) v -= n3[ax]; }
        bb[ax] = v;
        in = in && v >= 0 && v < S;
    }
    return in;
}

// box index of neighbour p + c_i from p's box coordinates; -1 outside the box
__device__ __forceinline__ int box_nb(const int (&bb)[3], int i, int S) {
    const int qx = bb[0] + cx(i), qy = bb[1] + cy(i), qz = bb[2] + cz(i);
    if (qx < 0 || qy < 0 || qz < 0 || qx >= S || qy >= S || qz >= S) return -1;
    return (qz * S + qy) * S + qx;
}

// lattice position of neighbour p + c_i (wrapped on periodic axes)
__device__ __forceinline__ void nb_pos(const int (&p)[3], int i, const Geo &g, int (&q)[3]) {
    q[0] = mirror1(p[0] + cx(i), g.nx, false);
    q[1] = mirror1(p[1] + cy(i), g.ny, false);
    q[2] = mirror1(p[2] + cz(i), g.nz, false);
}

// storage form of a deviation (as st_dev writes it) and the value a pull of
// it returns (as ld_dev reads it with the pull's scale)
template <typename S, typename T>
__device__ __forceinline__ T store_round(double v, T inv_scale, T scale, S &sv) {
    if constexpr (Rel<S>::value) {
        sv = (S)(float)(T(v) * inv_scale);
        return T((float)sv) * scale;
    } else {
        sv = (S)T(v);
        return T(sv);
    }
}

// Mean post-streaming density of the neighbours of p that are fluid at X^n
// and at X^{n+1} (raw of the box at orgo); rho0 when there is none.  Every
// argument is passed by value, so that no caller keeps its locals in scratch
// memory for the call.
struct Rho2 {
    double a, b;
};
struct Pos3 {
    double v[3];
};
struct Org3 {
    int32_t v[3];
};

__device__ __forceinline__ Rho2 mean_kept(int px, int py, int pz, Pos3 Xo, Pos3 Xn, double R2,
                                        const double *raw, Org3 orgo, int Sx, int S3, Geo g,
                                        double rho0A, double rho0B) {
    const int p[3] = {px, py, pz};
    Nbr no, nn;
    nbr_of(p, Xo.v, R2, g, no);
    nbr_of(p, Xn.v, R2, g, nn);
    int bo[3];
    const bool inbox = box_coords(p, orgo.v, Sx, g, bo);
    int idx[Q];
    uint32_t keep = 0;
#pragma unroll
    for (int i = 1; i < Q; i++) {
        idx[i] = inbox ? box_nb(bo, i, Sx) : -1;
        if (idx[i] >= 0 && nbr_ok(no, i) && !pnode_nb(no, i) && !pnode_nb(nn, i))
            keep |= 1u << i;
    }
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int i = 1; i < Q; i++) {
        if (!((keep >> i) & 1u)) continue;
        s0 += raw[idx[i]];
        s1 += raw[S3 + idx[i]];
    }
    const int cnt = __builtin_popcount(keep);
    Rho2 rb;
    rb.a = cnt > 0 ? s0 / cnt : rho0A;
    rb.b = cnt > 0 ? s1 / cnt : rho0B;
    return rb;
}

// =============================================================== k_links
// One thread per node of the box of X^n.  A node p fluid at X^n with links
// to the sphere (p + c_i a particle node) applies the moving-wall
// bounce-back f_opp(i)(p) = f*_i(p) - 6 w_i rho_l(p) (c_i . u_b), u_b the
// rigid velocity at the link midpoint, and writes it into the slot p pulls
// from (opp(i) at p + c_i) for the next step; it sums the exchanged momentum
// sum_l (2 f*_i - 6 w_i rho_l c_i . u_b) c_i and its torque about X^n, the
// bounce-back mass flux and the reaction of the wetting layer on the sphere.
// Every fluid box node then forms its step-(n+1) populations (plain pulls,
// its own bounced values on links) and stores their densities and momentum
// for the particle kernel.  Per-workgroup FP64 sums, fixed order.
template <typename S, typename T, int B>
__global__ __launch_bounds__(B) void k_links(LinkArgs a) {
    __shared__ double red[(B / 64) * 16];
    const int r = find_rep(a.k3_begin, a.nrep, blockIdx.x);
    const RepDesc *__restrict__ dp = a.desc + r;  // read-only in this kernel
    const RepDesc &D = *dp;
    const RepState st = a.state[r];
    if (!D.has_particle) return;
    const Geo g = geo_of(D);
    const int t = threadIdx.x;
    const int local = blockIdx.x - D.k3_begin;
    const int Sx = D.S, S3 = Sx * Sx * Sx;
    const int32_t org[3] = {st.org[0], st.org[1], st.org[2]};
    const double X[3] = {st.X[0], st.X[1], st.X[2]};
    const double *vrho = a.vrho + D.bbox_off * 2;
    const double *rho_n = a.rho_n + D.bbox_off * 2;
    double *raw = a.raw + D.bbox_off * RAW;
    S *buf = reinterpret_cast<S *>(a.buf) + D.pop_off;
    const PullCtx<S, T> pc = pull_ctx<S, T>(a.buf, D, g);
    const uint32_t NP = g.NP;
    double acc[15];
#pragma unroll
    for (int k = 0; k < 15; k++) acc[k] = 0.0;
    const int b = local * B + t;
    int bb[3], p[3];
    const bool in = b < S3 && bbox_pos(b, org, Sx, g, bb, p);
    Nbr nb;
    nbr_of(p, X, D.R2, g, nb);
    const bool fluid = in && !pnode_nb(nb, 0);
    // Loads, arithmetic and stores are kept in three separate phases: on this
    // architecture loads and stores share one wait counter, so a store issued
    // before a later load's wait would turn that wait into a write round trip.
    uint32_t links = 0;
    uint32_t own = 0;
    S sv[2][Q];
    double rw[RAW];
    if (fluid) {
        // fluid node: links to neighbours that are particle nodes at X^n
#pragma unroll
        for (int i = 1; i < Q; i++)
            if (box_nb(bb, i, Sx) >= 0 && nbr_ok(nb, i) && pnode_nb(nb, i)) links |= 1u << i;
        // plain pulls, own post-collision values (own slots are always valid,
        // so they are loaded unconditionally), own densities
        own = pidx(p[0], p[1], p[2], g);
        T d[2][Q];
        pull_node(pc, own, d);
        T fo[2][Q];
#pragma unroll
        for (int i = 1; i < Q; i++) {
#pragma unroll
            for (int l = 0; l < 2; l++) {
                const T sc = Rel<S>::value ? T(wgt(i) * D.rho0[l]) : T(1);
                fo[l][i] = ld_dev<S, T>(buf + ((uint32_t)(l * Q + i) * NP + own), sc);
            }
        }
        const double rA = rho_n[b], rB = rho_n[S3 + b];
        if (links) {
            // rigid velocity at the link midpoint p + c_i/2: c_i . u_b = c_i . (U + W x d)
            // with d = p - X, since c_i . (W x c_i) = 0; the torque of the summed
            // link momentum P about X is d x P for the same reason
            const double dd[3] = {sepd(p[0] - X[0], g.nx, g.wx), sepd(p[1] - X[1], g.ny, g.wy),
                                  sepd(p[2] - X[2], g.nz, g.wz)};
            const double V[3] = {st.U[0] + st.W[1] * dd[2] - st.W[2] * dd[1],
                                 st.U[1] + st.W[2] * dd[0] - st.W[0] * dd[2],
                                 st.U[2] + st.W[0] * dd[1] - st.W[1] * dd[0]};
            const double rl[2] = {rA, rB};
            double P[3] = {0.0, 0.0, 0.0};
#pragma unroll
            for (int i = 1; i < Q; i++) {
                if (!((links >> i) & 1u)) continue;
                const double cu = cx(i) * V[0] + cy(i) * V[1] + cz(i) * V[2];
                double mom = 0.0;
#pragma unroll
                for (int l = 0; l < 2; l++) {
                    const double wr = wgt(i) * D.rho0[l];
                    const double fs = wr + (double)fo[l][i];
                    const double corr = 6.0 * wgt(i) * rl[l] * cu;
                    mom += 2.0 * fs - corr;
                    acc[6 + l] -= corr;
                    d[l][opp(i)] = store_round<S, T>(fs - corr - wr, T(1.0 / wr), T(wgt(i)) * pc.scale[l], sv[l][i]);
                }
                if (cx(i)) P[0] += cx(i) > 0 ? mom : -mom;
                if (cy(i)) P[1] += cy(i) > 0 ? mom : -mom;
                if (cz(i)) P[2] += cz(i) > 0 ? mom : -mom;
                acc[14] += 1.0;
            }
            acc[0] += P[0]; acc[1] += P[1]; acc[2] += P[2];
            acc[3] += dd[1] * P[2] - dd[2] * P[1];
            acc[4] += dd[2] * P[0] - dd[0] * P[2];
            acc[5] += dd[0] * P[1] - dd[1] * P[0];
        }
        // densities and momentum of step n+1 at this node
        NodeM<T, true> m;
        node_moments(d, m);
        rw[0] = D.rho0[0] + (double)m.rd[0];
        rw[1] = D.rho0[1] + (double)m.rd[1];
#pragma unroll
        for (int q = 0; q < 3; q++) rw[2 + q] = (double)m.j[0][q] + (double)m.j[1][q];
    }
    if (in && !fluid) {
        // particle node s: reaction of the wetting layer, i.e. the Shan-Chen
        // force -G rho_l(x) w_k rho~_l'(s) c on each fluid neighbour x = s + c_k
        // (link direction c = -c_k), summed here from the particle side
        const double vA = vrho[b] + st.delta[0], vB = vrho[S3 + b] + st.delta[1];
        double rn[2][Q];
        uint32_t fl = 0;
#pragma unroll
        for (int k = 1; k < Q; k++) {
            rn[0][k] = rn[1][k] = 0.0;
            const int xb = box_nb(bb, k, Sx);
            if (xb < 0 || !nbr_ok(nb, k) || pnode_nb(nb, k)) continue;
            fl |= 1u << k;
            rn[0][k] = rho_n[xb];
            rn[1][k] = rho_n[S3 + xb];
        }
        // force on the fluid neighbour x = s + c_k is -sw c_k; its torque about X
        // is (d_s + c_k/2) x (-sw c_k) = d_s x (-sw c_k), d_s = s - X
        double Fw[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 1; k < Q; k++) {
            if (!((fl >> k) & 1u)) continue;
            const double sw = -D.G * wgt(k) * (rn[0][k] * vB + rn[1][k] * vA);
            if (cx(k)) Fw[0] += cx(k) > 0 ? -sw : sw;
            if (cy(k)) Fw[1] += cy(k) > 0 ? -sw : sw;
            if (cz(k)) Fw[2] += cz(k) > 0 ? -sw : sw;
        }
        const double ds[3] = {sepd(p[0] - X[0], g.nx, g.wx), sepd(p[1] - X[1], g.ny, g.wy),
                              sepd(p[2] - X[2], g.nz, g.wz)};
        acc[8] += Fw[0]; acc[9] += Fw[1]; acc[10] += Fw[2];
        acc[11] += ds[1] * Fw[2] - ds[2] * Fw[1];
        acc[12] += ds[2] * Fw[0] - ds[0] * Fw[2];
        acc[13] += ds[0] * Fw[1] - ds[1] * Fw[0];
    }
    if (fluid) {
        // stores: bounced values into the slots p pulls from at p + c_i (a
        // ghost when the link crosses a periodic face), then the node's raw
#pragma unroll
        for (int i = 1; i < Q; i++) {
            if (!((links >> i) & 1u)) continue;
            const uint32_t tgt = own + (uint32_t)doff(i, g);
#pragma unroll
            for (int l = 0; l < 2; l++) buf[(uint32_t)(l * Q + opp(i)) * NP + tgt] = sv[l][i];
        }
#pragma unroll
        for (int k = 0; k < RAW; k++) raw[k * S3 + b] = rw[k];
    }
    block_sum<B, 15>(acc, red);
    if (t == 0) {
        double *pp = a.part1 + D.part3_off + (int64_t)local * PART;
        for (int k = 0; k < 15; k++) pp[k] = acc[k];
    }
}

// ============================================================ k_particle
// One thread per node of the box of X^{n+1}.  Every wave reduces the link
// sums (fixed order) and advances the sphere: leap-frog Newton-Euler under
// F = links - wetting reaction + F_ext + pending event momentum.  Each node
// then takes its flags at X^{n+1} (the FP64 predicate, evaluated here for
// both positions), and
//  * covered (fluid at X^n, particle at X^{n+1}): adds its momentum and
//    mass to the event sums;
//  * uncovered (particle at X^n, fluid at X^{n+1}): gets f_eq(rho_bar, u_b)
//    written into the slots it pulls from, rho_bar the mean density of its
//    neighbours fluid at both times;
//  * particle node at X^{n+1}: gets the wetting-layer density, mean of its
//    fluid neighbours +/- Delta rho (the mass correction delta is added
//    where it is read).
// Each workgroup leaves its event sums as a partial.  They are combined, with
// the global mass correction and the new state of step n+1, either by the
// last workgroup to finish (one device-scope fence and atomic per workgroup)
// or, for large grids, by the separate k_finish launch (finish_apart): each
// such fence writes back the XCD's L2, which costs more than a launch once
// many workgroups share an XCD.
// Leap-frog Newton-Euler step of one sphere from the link sums of step n
// (momentum exchange minus wetting-layer reaction, plus F_ext and the
// pending event momentum), and the bounding-box origin of X^{n+1}.  Every
// caller evaluates it on the same inputs, so all agree bitwise.
struct Motion {
    double F[3], Tq[3], Un[3], Wn[3], Xn[3];
    int org[3];
};

__device__ __forceinline__ void newton_euler(const RepDesc &D, const RepState *st, const Geo &g,
                                             const double (&sum)[15], Motion &m) {
    const int n3[3] = {g.nx, g.ny, g.nz};
    const bool w3[3] = {g.wx, g.wy, g.wz};
    for (int q = 0; q < 3; q++) {
        m.F[q] = sum[q] - sum[8 + q] + D.Fext[q] + st->Pev[q];
        m.Tq[q] = sum[3 + q] - sum[11 + q] + st->Lev[q];
        m.Un[q] = D.fixed_velocity ? st->U[q] : st->U[q] + m.F[q] / D.mp;
        m.Wn[q] = D.fixed_velocity ? st->W[q] : st->W[q] + m.Tq[q] / D.Ip;
    }
    for (int q = 0; q < 3; q++) {
        m.Xn[q] = st->X[q] + m.Un[q];
        if (!w3[q]) {
            if (m.Xn[q] >= n3[q]) m.Xn[q] -= n3[q];
            else if (m.Xn[q] < 0.0) m.Xn[q] += n3[q];
        }
        m.org[q] = (int)floor(m.Xn[q] - D.radius) - 2;  // box of X^{n+1}
    }
}

// A replica without a sphere: record U = 0 and advance the step counter.
__device__ __forceinline__ void advance_empty(const ParticleArgs &a, const RepDesc &D, RepState *st) {
    const int64_t n = st->step;
    double *s = a.series + D.series_off + 3 * (n % D.series_cap);
    s[0] = s[1] = s[2] = 0.0;
    st->delta[0] = st->delta[1] = 0.0;
    st->step = n + 1;
}

// Motion of step n+1 of one sphere (one thread): position, velocities,
// forces, bounding-box origin, pending event momentum, the U series entry and
// the event counters.  Returns whether the sphere went unstable (|U| >= 1/2,
// a non-finite force) or reached a wall.
__device__ __forceinline__ bool publish_motion(const ParticleArgs &a, const RepDesc &D, RepState *st,
                                               const Geo &g, const double (&sum)[15], const Motion &mo,
                                               const double (&tot)[20]) {
    const int n3[3] = {g.nx, g.ny, g.nz};
    const bool w3[3] = {g.wx, g.wy, g.wz};
    const double Xold[3] = {st->X[0], st->X[1], st->X[2]};
    const double *utot = tot + 10;
    const int64_t n = st->step;
    double *s = a.series + D.series_off + 3 * (n % D.series_cap);
    bool bad = false;
    for (int q = 0; q < 3; q++) {
        st->Xp[q] = Xold[q];
        st->X[q] = mo.Xn[q];
        st->U[q] = mo.Un[q];
        st->W[q] = mo.Wn[q];
        st->F[q] = mo.F[q];
        st->T[q] = mo.Tq[q];
        st->Pev[q] = tot[q] - utot[q];
        st->Lev[q] = tot[3 + q] - utot[3 + q];
        st->org[q] = mo.org[q];
        s[q] = mo.Un[q];
        if (q == 2) st->uz_sum += mo.Un[2];
        if (!(fabs(mo.Un[q]) < 0.5) || !isfinite(mo.F[q])) bad = true;
        if (w3[q] && (mo.Xn[q] - D.radius < -0.5 || mo.Xn[q] + D.radius > n3[q] - 0.5)) bad = true;
    }
    st->n_cov += (int64_t)tot[8];
    st->n_unc += (int64_t)utot[8];
    st->n_links = (int64_t)sum[14];
    return bad;
}

// Publish step n+1 of one replica with a single sphere from the link sums,
// the motion and the event totals (one thread): global mass correction
// delta_l = -(bounce-back flux - covered + uncovered mass)_l / |Phi^{n+1}|,
// then the sphere's motion, the step counter and the stability flag.
__device__ __forceinline__ void publish_step(const ParticleArgs &a, const RepDesc &D, RepState *st,
                                             const Geo &g, const double (&sum)[15], const Motion &mo,
                                             const double (&tot)[20]) {
    const double *utot = tot + 10;
    const double nf = (double)D.N - tot[9];
    for (int l = 0; l < 2; l++) st->delta[l] = -(sum[6 + l] - tot[6 + l] + utot[6 + l]) / nf;
    const bool bad = publish_motion(a, D, st, g, sum, mo, tot);
    st->n_fluid = nf;
    if (bad) st->flags |= FLAG_UNSTABLE;
    st->step = st->step + 1;
}

// Publish step n+1 of a group of spheres in one fluid (one wave; lane 0
// writes).  The mass correction is global: the bounce-back, covered and
// uncovered fluxes and the particle nodes of every sphere are summed before
// delta_l and |Phi^{n+1}| are formed.  Each sphere then takes its own
// Newton-Euler step, and every entry of the group receives the shared fields
// (delta, fluid nodes, step, flags).  Two boxes that now share a node set
// FLAG_CONTACT on the group.
__device__ __forceinline__ void publish_group(const ParticleArgs &a, int prim, const Geo &g) {
    const RepDesc *P = a.desc + prim;
    const int K = P->n_sph;
    double dm[2] = {0.0, 0.0}, nsol = 0.0;
    for (int e = prim; e < prim + K; e++) {
        const RepDesc *De = a.desc + e;
        double sum[15], tot[20];
        sum_partials<15>(a.part1 + De->part3_off, De->k3_count, 0, sum);
        sum_partials<20>(a.part3 + De->part3_off, De->k3_count, 0, tot);
        for (int l = 0; l < 2; l++) dm[l] += sum[6 + l] - tot[6 + l] + tot[16 + l];
        nsol += tot[9];
    }
    const double nf = (double)P->N - nsol;
    const double delta[2] = {-dm[0] / nf, -dm[1] / nf};
    uint32_t flags = 0u;
    for (int e = prim; e < prim + K; e++) flags |= a.state[e].flags;
    const bool lead = (threadIdx.x & 63) == 0;
    for (int e = prim; e < prim + K; e++) {
        const RepDesc &De = a.desc[e];
        RepState *se = a.state + e;
        double sum[15], tot[20];
        sum_partials<15>(a.part1 + De.part3_off, De.k3_count, 0, sum);
        sum_partials<20>(a.part3 + De.part3_off, De.k3_count, 0, tot);
        Motion mo;
        newton_euler(De, se, g, sum, mo);
        if (lead && publish_motion(a, De, se, g, sum, mo, tot)) flags |= FLAG_UNSTABLE;
    }
    if (!lead) return;
    const int32_t n3[3] = {g.nx, g.ny, g.nz};
    for (int e = prim; e < prim + K; e++)
        for (int f = e + 1; f < prim + K; f++)
            if (boxes_overlap(a.state[e].org, a.desc[e].S, a.state[f].org, a.desc[f].S, n3, P->walls))
                flags |= FLAG_CONTACT;
    const int64_t step = a.state[prim].step + 1;
    for (int e = prim; e < prim + K; e++) {
        RepState *se = a.state + e;
        se->delta[0] = delta[0];
        se->delta[1] = delta[1];
        se->n_fluid = nf;
        se->flags = flags;
        se->step = step;
    }
}

template <typename S, typename T, int B, bool APART>
__global__ __launch_bounds__(B) void k_particle(ParticleArgs a) {
    static_assert(B == 64, "the uncovered-density jobs are shared within one wave");
    __shared__ double red[(B / 64) * 20];
    __shared__ int last;
    __shared__ int job_desc[64];   // owner lane | direction << 8 (0: the owner itself)
    __shared__ int job_pos[64][3];
    __shared__ Rho2 job_res[64];
    const int wg = blockIdx.x;
    const int r = find_rep(a.k3_begin, a.nrep, wg);
    const RepDesc *__restrict__ dp = a.desc + r;  // read-only in this kernel
    const RepDesc &D = *dp;
    RepState *st = a.state + r;
    const Geo g = geo_of(D);
    const int t = threadIdx.x;
    const int local = wg - D.k3_begin;
    if (!D.has_particle) {
        if (!APART && t == 0) advance_empty(a, D, st);
        return;
    }
    double X[3];
    int32_t orgo[3];
    for (int q = 0; q < 3; q++) {
        X[q] = st->X[q]; orgo[q] = st->org[q];
    }
    // 1. link momentum exchange and wetting-layer reaction of step n
    double sum[15];
    sum_partials<15>(a.part1 + D.part3_off, D.k3_count, 0, sum);
    // 2. Newton-Euler, leap-frog
    Motion mo;
    newton_euler(D, st, g, sum, mo);
    const double(&Un)[3] = mo.Un;
    const double(&Wn)[3] = mo.Wn;
    const double(&Xn)[3] = mo.Xn;
    const int(&org)[3] = mo.org;
    const int Sx = D.S, S3 = Sx * Sx * Sx;
    const double *raw = a.raw + D.bbox_off * RAW;
    double *vrho = a.vrho + D.bbox_off * 2;
    uint32_t *pmask = a.pmask + D.bbox_off;
    S *buf = reinterpret_cast<S *>(a.buf) + D.pop_off;
    const uint32_t NP = g.NP;

    // 3. events and wetting layer
    double ev[20];
#pragma unroll
    for (int k = 0; k < 20; k++) ev[k] = 0.0;
    const int b = local * B + t;
    int bb[3] = {0, 0, 0}, p[3] = {0, 0, 0};
    const bool in = b < S3 && bbox_pos(b, org, Sx, g, bb, p);
    Nbr no, nn;
    nbr_of(p, X, D.R2, g, no);
    nbr_of(p, Xn, D.R2, g, nn);
    const bool fo = in && !pnode_nb(no, 0);
    const bool fn = in && !pnode_nb(nn, 0);
    int bo[3];
    const bool inbox = box_coords(p, orgo, Sx, g, bo);
    // Loads and arithmetic first, every store last (loads and stores share
    // one wait counter here).
    //
    // A particle node at X^{n+1} (covered ones included) takes the wetting
    // layer: the mean density of its neighbours fluid at X^{n+1}.  A neighbour
    // uncovered at this step carries the mean density of its own kept
    // neighbours (its f_eq density), and an uncovered node needs that mean for
    // itself.  Those means are jobs shared out over the wave's lanes, 64 per
    // round, so that a lane with several of them does not run them one after
    // another while the rest of the wave waits.
    const bool pn = in && !fn;         // particle node at X^{n+1}
    const bool unc = in && !fo && fn;  // uncovered at this step
    int idx[Q];
    uint32_t kept = 0, fresh = 0;  // fluid at X^{n+1}; of those, uncovered now
    if (pn) {
#pragma unroll
        for (int i = 1; i < Q; i++) {
            idx[i] = -1;
            if (!nbr_ok(nn, i) || pnode_nb(nn, i)) continue;
            if (pnode_nb(no, i)) {
                fresh |= 1u << i;
            } else {
                idx[i] = inbox ? box_nb(bo, i, Sx) : -1;
                if (idx[i] < 0) continue;
            }
            kept |= 1u << i;
        }
    }
    const uint32_t jobs = pn ? fresh : (unc ? 1u : 0u);  // bit i: neighbour i; bit 0: itself
    double fs[2] = {0.0, 0.0};  // fresh neighbours' densities, summed in direction order
    Rho2 rself = {0.0, 0.0};    // an uncovered node's own mean
    {
        const int cnt = __builtin_popcount(jobs);
        int incl = cnt;  // inclusive prefix sum of the job counts over the wave
        for (int d = 1; d < 64; d <<= 1) {
            const int v = __shfl_up(incl, d);
            if (t >= d) incl += v;
        }
        const int excl = incl - cnt;
        const int total = __shfl(incl, 63);
        if (total > 0) {  // uniform over the wave (one wave per workgroup)
            job_pos[t][0] = p[0];
            job_pos[t][1] = p[1];
            job_pos[t][2] = p[2];
            for (int base = 0; base < total; base += 64) {
                int m = excl;
                for (uint32_t w = jobs; w; w &= w - 1, m++)
                    if (m >= base && m < base + 64) job_desc[m - base] = t | (__builtin_ctz(w) << 8);
                __syncthreads();
                if (t < total - base) {
                    const int d = job_desc[t], owner = d & 255, i = d >> 8;
                    const int o[3] = {job_pos[owner][0], job_pos[owner][1], job_pos[owner][2]};
                    int q[3] = {o[0], o[1], o[2]};
                    if (i > 0) nb_pos(o, i, g, q);
                    job_res[t] = mean_kept(q[0], q[1], q[2], Pos3{{X[0], X[1], X[2]}}, Pos3{{Xn[0], Xn[1], Xn[2]}},
                                           D.R2, raw, Org3{{orgo[0], orgo[1], orgo[2]}}, Sx, S3, g,
                                           D.rho0[0], D.rho0[1]);
                }
                __syncthreads();
                m = excl;
                for (uint32_t w = jobs; w; w &= w - 1, m++) {
                    if (m < base || m >= base + 64) continue;
                    const Rho2 rb = job_res[m - base];
                    if (__builtin_ctz(w) == 0) {
                        rself = rb;
                    } else {
                        fs[0] += rb.a;
                        fs[1] += rb.b;
                    }
                }
                __syncthreads();
            }
        }
    }
    double vw[2] = {0.0, 0.0};
    if (pn) {
        ev[9] += 1.0;
        double r0[Q], r1[Q];
#pragma unroll
        for (int i = 1; i < Q; i++) {
            r0[i] = r1[i] = 0.0;
            if (((kept & ~fresh) >> i) & 1u) {
                r0[i] = raw[idx[i]];
                r1[i] = raw[S3 + idx[i]];
            }
        }
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int i = 1; i < Q; i++) {
            if (!(((kept & ~fresh) >> i) & 1u)) continue;
            s0 += r0[i];
            s1 += r1[i];
        }
        s0 += fs[0];
        s1 += fs[1];
        const int cnt = __builtin_popcount(kept);
        vw[0] = cnt > 0 ? s0 / cnt + D.drho : 0.0;
        vw[1] = cnt > 0 ? s1 / cnt - D.drho : 0.0;
    }
    if (fo && !fn && inbox) {  // covered
        const int ob = (bo[2] * Sx + bo[1]) * Sx + bo[0];
        const double rho[2] = {raw[ob], raw[S3 + ob]};
        const double jt[3] = {raw[2 * S3 + ob], raw[3 * S3 + ob], raw[4 * S3 + ob]};
        const double rr[3] = {sepd(p[0] - Xn[0], g.nx, g.wx), sepd(p[1] - Xn[1], g.ny, g.wy),
                              sepd(p[2] - Xn[2], g.nz, g.wz)};
        ev[0] += jt[0]; ev[1] += jt[1]; ev[2] += jt[2];
        ev[3] += rr[1] * jt[2] - rr[2] * jt[1];
        ev[4] += rr[2] * jt[0] - rr[0] * jt[2];
        ev[5] += rr[0] * jt[1] - rr[1] * jt[0];
        ev[6] += rho[0];
        ev[7] += rho[1];
        ev[8] += 1.0;
    }
    if (b < S3) {
        pmask[b] = (in && !fn) ? MASK_SOLID : 0u;
        if (in && !fn) {
            vrho[b] = vw[0];
            vrho[S3 + b] = vw[1];
        }
    }
    if (unc) {  // uncovered (rare): f_eq of its neighbours' mean density and u_b
        const double rb[2] = {rself.a, rself.b};
        const double rr[3] = {sepd(p[0] - Xn[0], g.nx, g.wx), sepd(p[1] - Xn[1], g.ny, g.wy),
                              sepd(p[2] - Xn[2], g.nz, g.wz)};
        const double u[3] = {Un[0] + Wn[1] * rr[2] - Wn[2] * rr[1],
                             Un[1] + Wn[2] * rr[0] - Wn[0] * rr[2],
                             Un[2] + Wn[0] * rr[1] - Wn[1] * rr[0]};
        const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
        const uint32_t own = pidx(p[0], p[1], p[2], g);
        for (int i = 0; i < Q; i++) {
            const double cu = cx(i) * u[0] + cy(i) * u[1] + cz(i) * u[2];
            const double e = 1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu;
            const uint32_t src = own - (uint32_t)doff(i, g);
            for (int l = 0; l < 2; l++) {
                const double wr = wgt(i) * D.rho0[l];
                const double dev = wgt(i) * rb[l] * e - wr;
                st_dev<S, T>(buf + ((uint32_t)(l * Q + i) * NP + src), T(dev),
                             Rel<S>::value ? T(1.0 / wr) : T(1));
            }
        }
        const double mom[3] = {(rb[0] + rb[1]) * u[0], (rb[0] + rb[1]) * u[1],
                               (rb[0] + rb[1]) * u[2]};
        ev[10] += mom[0]; ev[11] += mom[1]; ev[12] += mom[2];
        ev[13] += rr[1] * mom[2] - rr[2] * mom[1];
        ev[14] += rr[2] * mom[0] - rr[0] * mom[2];
        ev[15] += rr[0] * mom[1] - rr[1] * mom[0];
        ev[16] += rb[0];
        ev[17] += rb[1];
        ev[18] += 1.0;
    }
    block_sum<B, 20>(ev, red);
    if (t == 0) {
        double *pp = a.part3 + D.part3_off + (int64_t)local * PART;
        for (int k = 0; k < 20; k++) pp[k] = ev[k];
    }
    if constexpr (APART) return;
    // the counter of the group's primary entry counts the workgroups of every
    // sphere in the fluid (a single sphere: its own)
    RepState *sp = a.state + D.primary;
    __threadfence();
    __syncthreads();
    if (t == 0) last = (atomicAdd(&sp->k3_done, 1u) == (unsigned)(D.k3_total - 1));
    __syncthreads();
    if (!last) return;
    __threadfence();
    // the next launch sees the stores below: kernel boundaries order them
    if (D.n_sph > 1) {
        publish_group(a, D.primary, g);
        if (t == 0) sp->k3_done = 0;
        return;
    }
    // last workgroup: event sums (fixed order), then the new state
    double tot[20];
    sum_partials<20>(a.part3 + D.part3_off, D.k3_count, 0, tot);
    if (t != 0) return;
    st->k3_done = 0;
    publish_step(a, D, st, g, sum, mo, tot);
}

// ============================================================== k_finish
// One wave per entry after k_particle (finish_apart): sums the link and
// event partials in the same fixed order, repeats the Newton-Euler step of
// k_particle on the same inputs and publishes the state of step n+1 (a
// group of spheres in one fluid: its primary's wave publishes them all).
template <int B>
__global__ __launch_bounds__(B) void k_finish(ParticleArgs a) {
    const int r = blockIdx.x;
    const RepDesc *__restrict__ dp = a.desc + r;  // read-only in this kernel
    const RepDesc &D = *dp;
    RepState *st = a.state + r;
    if (!D.has_particle) {
        if (threadIdx.x == 0) advance_empty(a, D, st);
        return;
    }
    const Geo g = geo_of(D);
    if (D.n_sph > 1) {
        if (D.primary == r) publish_group(a, r, g);
        return;
    }
    double sum[15], tot[20];
    sum_partials<15>(a.part1 + D.part3_off, D.k3_count, 0, sum);
    sum_partials<20>(a.part3 + D.part3_off, D.k3_count, 0, tot);
    Motion mo;
    newton_euler(D, st, g, sum, mo);
    if (threadIdx.x == 0) publish_step(a, D, st, g, sum, mo, tot);
}

// ================================================================ k_init
// f(0) = w_i rho_l(x) with rho_l = rho0_l + amp (2u - 1), u from Philox with
// counter (node, 0, 0, 1), word l, written into the slots x pulls from; the
// planes z >= init_split (when set) start from the swapped pair rho0_{1-l}.
template <typename S>
__global__ __launch_bounds__(256) void k_init(InitArgs a) {
    __shared__ double red[4 * 2];
    const int wg = blockIdx.x;
    const int r = find_rep(a.init_begin, a.nrep, wg);
    const RepDesc &D = a.desc[r];
    const Geo g = geo_of(D);
    const int64_t n = (int64_t)(wg - a.init_begin[r]) * 256 + threadIdx.x;
    double m[2] = {0.0, 0.0};
    if (n < g.N) {
        const int x = (int)(n % g.nx), y = (int)((n / g.nx) % g.ny);
        const int z = (int)(n / ((int64_t)g.nx * g.ny));
        bool solid = false;  // inside any sphere of the replica
        for (int e = r; e < r + D.n_sph; e++)
            solid = solid || (a.desc[e].has_particle && pnode(x, y, z, a.state[e].X, a.desc[e].R2, g));
        uint32_t c0 = (uint32_t)n, c1 = 0u, c2 = 0u, c3 = 1u;
        philox4x32_10(c0, c1, c2, c3, D.key0, D.key1);
        const uint32_t w[2] = {c0, c1};
        S *dst = reinterpret_cast<S *>(a.buf) + D.pop_off;
        const uint32_t own = pidx(x, y, z, g);
        const bool swap = D.init_split > 0 && z >= D.init_split;  // other phase above the split
        for (int l = 0; l < 2; l++) {
            const double base = swap ? D.rho0[1 - l] : D.rho0[l];
            const double rho = base + D.init_amp * (2.0 * (((double)w[l] + 0.5) * 0x1p-32) - 1.0);
            if (solid) continue;
            m[l] = rho;
            for (int i = 0; i < Q; i++) {
                const double wr = wgt(i) * D.rho0[l];
                st_dev<S, double>(dst + ((uint32_t)(l * Q + i) * g.NP + own - (uint32_t)doff(i, g)),
                                  wgt(i) * rho - wr, Rel<S>::value ? 1.0 / wr : 1.0);
            }
        }
    }
    block_sum<256, 2>(m, red);
    if (threadIdx.x == 0) {
        a.mass[2 * wg] = m[0];
        a.mass[2 * wg + 1] = m[1];
    }
}

// The entry of the group of primary entry prim whose sphere holds node
// (x, y, z) for the current step (b: its box index), or -1 for a fluid node.
__device__ __forceinline__ int solid_entry(int x, int y, int z, const RepDesc *desc, const RepState *state,
                                           const uint32_t *pmask, int prim, const Geo &g, int &b) {
    for (int e = prim; e < prim + desc[prim].n_sph; e++) {
        const RepDesc &D = desc[e];
        if (!D.has_particle) continue;
        b = bbox_index(x, y, z, state[e].org, D.S, g);
        if (b >= 0 && (pmask[D.bbox_off + b] & MASK_SOLID)) return e;
    }
    b = -1;
    return -1;
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
    const PullCtx<S, T> pc = pull_ctx<S, T>(a.src, D, g);
    int b;
    const bool solid = solid_entry(x, y, z, a.desc, a.state, a.pmask, D.primary, g, b) >= 0;
    T d[2][Q];
    if (!solid) pull_node(pc, pidx(x, y, z, g), d);
    for (int l = 0; l < 2; l++)
        for (int i = 0; i < Q; i++)
            a.out[(int64_t)(l * Q + i) * cnt + k] =
                solid ? 0.0 : wgt(i) * (D.rho0[l] + st.delta[l]) + (double)d[l][i];
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
    int b;
    const int e = solid_entry(x, y, z, a.desc, a.state, a.pmask, D.primary, g, b);
    if (e >= 0) {
        const int S3 = a.desc[e].S * a.desc[e].S * a.desc[e].S;
        const double *vrho = a.vrho + a.desc[e].bbox_off * 2;
        rt[n] = vrho[b] + st.delta[0];
        rt[g.N + n] = vrho[S3 + b] + st.delta[1];
        for (int q = 0; q < 3; q++) jt[q * g.N + n] = 0.0;
        sol[n] = 1.0;
        return;
    }
    const PullCtx<S, T> pc = pull_ctx<S, T>(a.src, D, g);
    T d[2][Q];
    pull_node(pc, pidx(x, y, z, g), d);
    double jtot[3] = {0.0, 0.0, 0.0};
    for (int l = 0; l < 2; l++) {
        T rd, jl[3], mm[Q];
        component_modes(d[l], rd, jl, mm);
        rt[l * g.N + n] = D.rho0[l] + st.delta[l] + (double)rd;
        for (int q = 0; q < 3; q++) jtot[q] += (double)jl[q];
    }
    for (int q = 0; q < 3; q++) jt[q * g.N + n] = jtot[q];
    sol[n] = 0.0;
}

// ============================================================== launchers
template <typename S, typename T, int B, bool GROUP>
void launch_main_b(const MainArgs &a, int grid, size_t lds, hipStream_t s) {
    if (a.tau1) {
        if (a.noise) hipLaunchKernelGGL((k_main<S, T, B, true, GROUP, true>), dim3(grid), dim3(B), lds, s, a);
        else hipLaunchKernelGGL((k_main<S, T, B, true, GROUP, false>), dim3(grid), dim3(B), lds, s, a);
    } else {
        if (a.noise) hipLaunchKernelGGL((k_main<S, T, B, false, GROUP, true>), dim3(grid), dim3(B), lds, s, a);
        else hipLaunchKernelGGL((k_main<S, T, B, false, GROUP, false>), dim3(grid), dim3(B), lds, s, a);
    }
}

template <typename S, typename T, bool GROUP>
hipError_t launch_main_g(const MainArgs &a, int grid, int block, size_t lds, hipStream_t s) {
    switch (block) {
    case 256: launch_main_b<S, T, 256, GROUP>(a, grid, lds, s); break;
    case 512: launch_main_b<S, T, 512, GROUP>(a, grid, lds, s); break;
    case 1024: launch_main_b<S, T, 1024, GROUP>(a, grid, lds, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename S, typename T>
hipError_t launch_main_t(const MainArgs &a, int grid, int block, size_t lds, hipStream_t s) {
    return a.groups ? launch_main_g<S, T, true>(a, grid, block, lds, s)
                    : launch_main_g<S, T, false>(a, grid, block, lds, s);
}

template <typename S, typename T>
hipError_t launch_links_t(const LinkArgs &a, int grid, hipStream_t s) {
    hipLaunchKernelGGL((k_links<S, T, K3_THREADS>), dim3(grid), dim3(K3_THREADS), 0, s, a);
    return hipGetLastError();
}

template <typename S, typename T>
hipError_t launch_particle_t(const ParticleArgs &a, int grid, hipStream_t s) {
    if (a.finish_apart) hipLaunchKernelGGL((k_particle<S, T, K3_THREADS, true>), dim3(grid), dim3(K3_THREADS), 0, s, a);
    else hipLaunchKernelGGL((k_particle<S, T, K3_THREADS, false>), dim3(grid), dim3(K3_THREADS), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !a.finish_apart) return e;
    hipLaunchKernelGGL(k_finish<64>, dim3(a.nrep), dim3(64), 0, s, a);
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
