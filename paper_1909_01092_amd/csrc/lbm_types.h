// Device-side data layout of the library (workspace contents).
//
// Populations: two ping-pong buffers; replica r owns a block of 38 NP_r
// elements laid out [component][direction][z+1][y+1][x+1] on its lattice
// padded by one ghost layer per side (x fastest).  A buffer holds the
// post-collision values f*_i of the last step in the slot each node pulls
// from (slot i at padded position x - c_i); values that reach a node by
// bounce-back or across a periodic face are written there by their
// producer.  Elements are stored as deviations from w_i rho0_l (FP64, FP32)
// or as relative deviations (f - w_i rho0_l) / (w_i rho0_l) (FP16).
#pragma once
#include <stdint.h>
#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#endif

#include "lbm_math.h"

namespace lbm {

struct RepDesc {
    int32_t nx, ny, nz;
    uint32_t walls;          // bit0 x, bit1 y, bit2 z
    int64_t N;               // nodes
    int64_t NP;              // padded nodes (nx + 2)(ny + 2)(nz + 2)
    int64_t pop_off;         // element offset of the replica block (38 NP) in a population buffer
    int32_t ty;              // rows (y) per main-kernel tile; tiles span full x rows
    int32_t nty, nchunk;     // tiles along y, z-chunks
    int32_t wg_begin;        // first main-kernel workgroup of this replica
    int32_t k3_begin, k3_count;  // particle-kernel workgroups
    int32_t S;               // edge of the particle bounding box (nodes), 2 ceil(R) + 6
    int32_t has_particle;
    int64_t bbox_off;        // element offset of this replica in the bbox arrays (S^3 each)
    int64_t part3_off;       // double offset of the link and particle partials (PART per workgroup)
    int64_t series_off;      // double offset of the U series ring (3 per entry)
    int32_t series_cap;
    int32_t cz;              // z-chunk of the main kernel
    double rho0[2];
    double G;
    double af[3];            // body-force acceleration of the fluid
    double Fext[3];          // external force on the particle
    double M0;               // initial fluid mass (balanced driving)
    double radius, R2, rho_p, mp, Ip, drho;
    double tau[4];           // shear, bulk, momentum, ghost
    double kT;
    double init_amp;
    uint32_t key0, key1;
    int32_t noise_diffusive, fixed_velocity;
    int32_t init_split;      // first plane of the swapped initial phase (0: none)
    int32_t ghost_fill;      // main kernel also writes the never-pulled x-ghost slots
    // collision coefficients and forcing in both arithmetic precisions, made
    // once on the host (kernels load them as wave-uniform values)
    Coef<float> cf32;
    Coef<double> cf64;
    float G32, af32[3];
    // Several spheres in one fluid: each sphere is an entry; the first entry
    // of a group (the primary) owns the populations and the main-kernel
    // tiles, the others (k = 1 .. n_sph - 1, at primary + k) share them and
    // carry only their sphere, box and partials.  Every entry of a group
    // holds the same fluid fields.
    int32_t primary;         // index of the group's first entry
    int32_t n_sph;           // entries in the group (1: a single sphere or none)
    int32_t k3_total;        // particle-kernel workgroups of the whole group
    int32_t pad_grp;
};

template <typename T> __host__ __device__ __forceinline__ const Coef<T> &coef_of(const RepDesc &D);
template <> __host__ __device__ __forceinline__ const Coef<float> &coef_of<float>(const RepDesc &D) { return D.cf32; }
template <> __host__ __device__ __forceinline__ const Coef<double> &coef_of<double>(const RepDesc &D) { return D.cf64; }

struct RepState {
    double X[3], Xp[3];      // X^n and X^{n-1}
    double U[3], W[3];       // U^{n-1/2}, Omega^{n-1/2}
    double F[3], T[3];       // total force / torque of the last step
    double Pev[3], Lev[3];   // pending cover/uncover momentum, angular momentum
    double delta[2];         // mass correction applied when pulling step n
    double n_fluid;
    double uz_sum;           // running sum of U_z^{n+1/2} over the steps taken
    int64_t step, n_cov, n_unc, n_links;
    int32_t org[3];          // origin of the bounding box of X^n
    int32_t pad_org;
    uint32_t flags;          // FLAG_UNSTABLE, FLAG_CONTACT
    uint32_t k3_done;        // particle-kernel completion counter (0 between steps)
    uint32_t pad1[2];
};

constexpr uint32_t FLAG_UNSTABLE = 1u;
// two spheres of one group whose bounding boxes share a node (the per-sphere
// box work then no longer sees every particle node near it)
constexpr uint32_t FLAG_CONTACT = 2u;
// Node flag of a bounding-box node for one step: MASK_SOLID = particle node at X^n.
constexpr uint32_t MASK_SOLID = 1u << 19;
constexpr int PART = 24;     // doubles per workgroup partial
constexpr int RAW = 5;       // doubles per box node: rho_A, rho_B, j (post-streaming, step n+1)
constexpr int MAX_GROUP = 16;  // spheres per fluid

// Whether the boxes of edge Sa at oa and of edge Sb at ob share a node: per
// axis, half-open intervals on a ring of n nodes (periodic axes, n >= Sa, Sb)
// or on a line (walled axes); they share a node when they meet on all three.
__host__ __device__ inline bool boxes_overlap(const int32_t *oa, int Sa, const int32_t *ob, int Sb,
                                              const int32_t *n3, uint32_t walls) {
    for (int ax = 0; ax < 3; ax++) {
        int d1 = ob[ax] - oa[ax], d2 = oa[ax] - ob[ax];
        bool meet;
        if (walls & (1u << ax)) {
            meet = d1 < Sa && d2 < Sb;
        } else {
            d1 = ((d1 % n3[ax]) + n3[ax]) % n3[ax];
            d2 = ((d2 % n3[ax]) + n3[ax]) % n3[ax];
            meet = d1 < Sa || d2 < Sb;
        }
        if (!meet) return false;
    }
    return true;
}

}  // namespace lbm
