// Launch interface between the C-ABI host code and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm_types.h"

namespace lbm {

struct MainArgs {
    const RepDesc *desc;
    RepState *state;
    const int32_t *wg_begin;   // nrep entries
    int32_t nrep;
    const void *src;           // populations of step n (post-collision of n-1)
    void *dst;                 // post-collision populations of step n
    const uint32_t *pmask;     // node masks of step n (bbox)
    const double *vrho;        // wetting-layer densities of step n (bbox)
    double *rho_n;             // densities of step n near the sphere (bbox), written
    int32_t tau1;              // every relaxation time of every replica is 1
    int32_t groups;            // some fluid holds several spheres
    int32_t noise;             // some replica has kT > 0
};

struct LinkArgs {
    const RepDesc *desc;
    const RepState *state;
    const int32_t *k3_begin;
    int32_t nrep;
    void *buf;                 // post-collision populations of step n (bounced values written)
    const double *vrho;        // wetting-layer densities of step n (bbox)
    const double *rho_n;       // densities of step n (bbox)
    double *raw;               // post-streaming densities and momenta of fluid box nodes, written
    double *part1;             // per-workgroup link partials
};

// Threads per workgroup of the bounding-box kernels k_links / k_particle: one
// wave.  The box chain is latency-bound on a few thousand nodes, so more,
// smaller workgroups spread it over more CUs (64x64x256 channel: 0.1365
// against 0.1394 ms per step with 256 threads).
constexpr int K3_THREADS = 64;

struct ParticleArgs {
    const RepDesc *desc;
    RepState *state;
    const int32_t *k3_begin;
    int32_t nrep;
    void *buf;                 // populations of step n+1 (uncovered-node values written)
    const double *part1;       // link partials
    double *part3;             // cover / uncover partials
    uint32_t *pmask;           // node masks of step n+1, written
    const double *raw;
    double *vrho;              // wetting-layer densities of step n+1, written
    double *series;
    int32_t finish_apart;      // 1: k_finish publishes the step; 0: the last workgroup does
};

struct InitArgs {
    const RepDesc *desc;
    RepState *state;
    const int32_t *init_begin;
    int32_t nrep;
    void *buf;
    double *mass;              // 2 per init workgroup
    double *vrho;
    uint32_t *pmask;
};

struct ExportArgs {
    const RepDesc *desc;
    const RepState *state;
    int32_t rep;
    int32_t z_begin, z_end;
    const void *src;
    const uint32_t *pmask;
    double *out;
};

struct FieldArgs {
    const RepDesc *desc;
    const RepState *state;
    int32_t rep;
    const void *src;
    const uint32_t *pmask;
    const double *vrho;
    double *scratch;           // 9 N doubles
    double *columns;           // 8 nx ny doubles, or null
};

// dispatch on the storage precision (0 FP64, 1 FP32, 2 FP16)
hipError_t launch_main(int prec, const MainArgs &a, int grid, int block, size_t lds, hipStream_t s);
hipError_t launch_links(int prec, const LinkArgs &a, int grid, hipStream_t s);
hipError_t launch_particle(int prec, const ParticleArgs &a, int grid, hipStream_t s);
hipError_t launch_init(int prec, const InitArgs &a, int grid, int nrep, hipStream_t s);
hipError_t launch_export(int prec, const ExportArgs &a, int64_t count, hipStream_t s);
hipError_t launch_fields(int prec, const FieldArgs &a, int64_t N, int64_t plane, hipStream_t s);

#define LBM_DECLARE(SUFFIX)                                                                        \
    hipError_t launch_main_##SUFFIX(const MainArgs &, int, int, size_t, hipStream_t);              \
    hipError_t launch_links_##SUFFIX(const LinkArgs &, int, hipStream_t);                          \
    hipError_t launch_particle_##SUFFIX(const ParticleArgs &, int, hipStream_t);                   \
    hipError_t launch_init_##SUFFIX(const InitArgs &, int, hipStream_t);                           \
    hipError_t launch_export_##SUFFIX(const ExportArgs &, int64_t, hipStream_t);                   \
    hipError_t launch_fields_a_##SUFFIX(const FieldArgs &, int64_t, hipStream_t);
LBM_DECLARE(f64)
LBM_DECLARE(f32)
LBM_DECLARE(f16)

}  // namespace lbm
