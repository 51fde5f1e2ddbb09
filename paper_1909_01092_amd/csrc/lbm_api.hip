// Host implementation of the C ABI declared in include/lbm.h: validation,
// workspace layout, initial state, step scheduling (plain launches or HIP
// graph replays), state queries and checkpoints.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "lbm.h"
#include "lbm_adjoint.h"
#include "lbm_kernels.h"
#include "lbm_types.h"

using namespace lbm;

namespace {

thread_local std::string g_init_error;

// Static per-step scratch for lbm_step_noalloc.  In host code `scratch`
// names a host-side stand-in: its device address comes from
// hipGetSymbolAddress, taken once per device with that device current.
constexpr size_t STATIC_SCRATCH_BYTES = size_t(16) << 20;
constexpr int MAX_DEVICES = 64;
__device__ __align__(256) unsigned char scratch[STATIC_SCRATCH_BYTES];
std::mutex g_scratch_mutex;
void *g_scratch_ptr[MAX_DEVICES] = {};

constexpr size_t ALIGN = 256;
constexpr int MAIN_BLOCK_MIN = 256;
constexpr size_t MAIN_LDS_MAX = 64 * 1024;
constexpr int K3_BLOCK = K3_THREADS;
constexpr int K3_FINISH_APART = 256;  // particle workgroups above which k_finish runs apart
constexpr int INIT_BLOCK = 256;

size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

size_t elem_size(int prec) { return prec == LBM_FP64 ? 8 : prec == LBM_FP32 ? 4 : 2; }

bool has_sphere(const lbm_params &p) { return p.radius > 0.0; }

int bbox_edge(const lbm_params &p) {
    return has_sphere(p) ? 2 * (int)std::ceil(p.radius) + 6 : 0;
}

// Entries grouped into fluids: an entry with shared_fluid = 1 is one more
// sphere in the fluid of the entry before it.  q holds the entries with the
// fluid fields of each group's primary (the sphere fields stay their own).
struct Groups {
    std::vector<lbm_params> q;
    std::vector<int> prim, nsph;
};

// initial bounding-box origin of a sphere (as the device forms it)
void init_org(const lbm_params &q, int32_t org[3]) {
    for (int a = 0; a < 3; a++) org[a] = (int32_t)std::floor(q.X0[a] - q.radius) - 2;
}

struct Layout {
    size_t tables, desc, state, pop[2], part1, part3, raw, vrho, rho_n, pmask, series, aux, total;
    std::vector<int64_t> pop_off, bbox_off, part3_off, series_off, init_wg;
    std::vector<int> S, k3_count;
    int64_t Ntot = 0, NPtot = 0, S3tot = 0, part3_tot = 0, series_tot = 0, init_tot = 0;
    size_t aux_doubles = 0;
};

// populations, fluid nodes and initial-state workgroups per group (its
// primary); boxes, partials and U series per entry
Layout plan(const Groups &G, int prec) {
    Layout L;
    const lbm_params *p = G.q.data();
    const int n = (int)G.q.size();
    const size_t es = elem_size(prec);
    L.pop_off.resize(n); L.bbox_off.resize(n); L.part3_off.resize(n);
    L.series_off.resize(n); L.S.resize(n); L.k3_count.resize(n); L.init_wg.resize(n);
    size_t max_cols = 0;
    for (int r = 0; r < n; r++) {
        const bool primary = G.prim[r] == r;
        const int64_t N = (int64_t)p[r].nx * p[r].ny * p[r].nz;
        const int64_t NP = (int64_t)(p[r].nx + 2) * (p[r].ny + 2) * (p[r].nz + 2);
        if (primary) {
            L.pop_off[r] = 38 * L.NPtot;
            L.NPtot += NP;
            L.Ntot += N;
        } else {
            L.pop_off[r] = L.pop_off[G.prim[r]];
        }
        L.S[r] = bbox_edge(p[r]);
        const int64_t S3 = (int64_t)L.S[r] * L.S[r] * L.S[r];
        L.bbox_off[r] = L.S3tot;
        L.S3tot += S3;
        L.k3_count[r] = has_sphere(p[r]) ? (int)((S3 + K3_BLOCK - 1) / K3_BLOCK) : 1;
        L.part3_off[r] = L.part3_tot;
        L.part3_tot += (int64_t)L.k3_count[r] * PART;
        L.series_off[r] = L.series_tot;
        L.series_tot += 3 * (int64_t)p[r].series_cap;
        L.init_wg[r] = primary ? (N + INIT_BLOCK - 1) / INIT_BLOCK : 0;
        L.init_tot += L.init_wg[r];
        max_cols = std::max(max_cols, (size_t)8 * p[r].nx * p[r].ny);
    }
    L.aux_doubles = std::max(max_cols, (size_t)(2 * L.init_tot));
    size_t o = 0;
    auto take = [&](size_t bytes) { const size_t at = o; o = align_up(o + bytes); return at; };
    L.tables = take(sizeof(int32_t) * 3 * (n + 1));
    L.desc = take(sizeof(RepDesc) * n);
    L.state = take(sizeof(RepState) * n);
    L.pop[0] = take(38 * L.NPtot * es);
    L.pop[1] = take(38 * L.NPtot * es);
    L.part1 = take(sizeof(double) * std::max<int64_t>(L.part3_tot, 1));
    L.part3 = take(sizeof(double) * std::max<int64_t>(L.part3_tot, 1));
    L.raw = take(sizeof(double) * std::max<int64_t>(RAW * L.S3tot, 1));
    L.vrho = take(sizeof(double) * std::max<int64_t>(2 * L.S3tot, 1));
    L.rho_n = take(sizeof(double) * std::max<int64_t>(2 * L.S3tot, 1));
    L.pmask = take(sizeof(uint32_t) * std::max<int64_t>(L.S3tot, 1));
    L.series = take(sizeof(double) * std::max<int64_t>(L.series_tot, 1));
    L.aux = take(sizeof(double) * L.aux_doubles);
    L.total = o;
    return L;
}

std::string fmt(const char *f, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, f);
    vsnprintf(buf, sizeof(buf), f, ap);
    va_end(ap);
    return buf;
}

std::string validate(const lbm_params *praw, int n, int prec, Groups &G) {
    if (!praw) return "params is NULL";
    if (n < 1) return "n_replicas must be >= 1";
    if (prec < LBM_FP64 || prec > LBM_FP16) return "precision must be LBM_FP64, LBM_FP32 or LBM_FP16";
    G.q.assign(praw, praw + n);
    G.prim.assign(n, 0);
    G.nsph.assign(n, 1);
    for (int r = 0; r < n; r++) {
        const int32_t sf = praw[r].shared_fluid;
        if (sf != 0 && sf != 1) return fmt("entry %d: shared_fluid must be 0 or 1", r);
        if (sf == 0) {
            G.prim[r] = r;
            continue;
        }
        if (r == 0) return "entry 0: shared_fluid needs an entry before it";
        const int pr = G.prim[r - 1];
        G.prim[r] = pr;
        if (!has_sphere(praw[pr]) || !has_sphere(praw[r]))
            return fmt("entry %d: spheres sharing a fluid need radius > 0 (and so does entry %d)", r, pr);
        if (r - pr + 1 > MAX_GROUP) return fmt("entry %d: more than %d spheres in one fluid", r, MAX_GROUP);
        lbm_params q = praw[pr];  // the fluid is the primary's
        q.radius = praw[r].radius;
        q.rho_p = praw[r].rho_p;
        q.wet_drho = praw[r].wet_drho;
        for (int a = 0; a < 3; a++) {
            q.X0[a] = praw[r].X0[a];
            q.U0[a] = praw[r].U0[a];
            q.W0[a] = praw[r].W0[a];
        }
        q.shared_fluid = 1;
        G.q[r] = q;
    }
    for (int r = 0; r < n; r++) G.nsph[G.prim[r]] = r - G.prim[r] + 1;
    for (int r = 0; r < n; r++) G.nsph[r] = G.nsph[G.prim[r]];
    const lbm_params *p = G.q.data();
    for (int r = 0; r < n; r++) {
        const lbm_params &q = p[r];
        const int nn[3] = {q.nx, q.ny, q.nz};
        if (q.nx < 2 || q.ny < 2 || q.nz < 2) return fmt("replica %d: every axis needs >= 2 nodes", r);
        if (q.nx > MAIN_BLOCK_MIN) return fmt("replica %d: nx = %d exceeds %d", r, q.nx, MAIN_BLOCK_MIN);
        // element offsets of a replica block (38 NP) are 32-bit signed, byte
        // offsets within one component (19 NP elements) 32-bit unsigned
        const int64_t np = (int64_t)(q.nx + 2) * (q.ny + 2) * (q.nz + 2);
        const int64_t es = prec == LBM_FP64 ? 8 : prec == LBM_FP32 ? 4 : 2;
        if (np >= (int64_t(1) << 31) / 38 || 19 * np * es >= (int64_t(1) << 32))
            return fmt("replica %d: lattice too large for one replica at this precision", r);
        if (q.walls > 7u) return fmt("replica %d: walls must be a 3-bit mask", r);
        if (!(q.rho0[0] > 0.0) || !(q.rho0[1] > 0.0)) return fmt("replica %d: rho0 must be > 0", r);
        if (!(q.init_amp >= 0.0) || q.init_amp >= std::min(q.rho0[0], q.rho0[1]))
            return fmt("replica %d: init_amp must be in [0, min(rho0))", r);
        if (q.init_split < 0 || q.init_split >= q.nz)
            return fmt("replica %d: init_split must be in [0, nz)", r);
        const double taus[4] = {q.tau_shear, q.tau_bulk, q.tau_mom, q.tau_ghost};
        for (double t : taus)
            if (!(t > 0.5) || !std::isfinite(t)) return fmt("replica %d: relaxation times must be > 1/2", r);
        if (!(q.kT >= 0.0) || !std::isfinite(q.kT)) return fmt("replica %d: kT must be >= 0", r);
        if (!std::isfinite(q.G)) return fmt("replica %d: G must be finite", r);
        if (q.force_mode != 0 && q.force_mode != 1) return fmt("replica %d: force_mode must be 0 or 1", r);
        if (q.series_cap < 1) return fmt("replica %d: series_cap must be >= 1", r);
        for (int a = 0; a < 3; a++)
            if (!std::isfinite(q.g[a]) || !std::isfinite(q.U0[a]) || !std::isfinite(q.W0[a]) ||
                !std::isfinite(q.X0[a]))
                return fmt("replica %d: non-finite vector parameter", r);
        if (has_sphere(q)) {
            if (!(q.rho_p > 0.0)) return fmt("replica %d: rho_p must be > 0", r);
            const int S = bbox_edge(q);
            for (int a = 0; a < 3; a++) {
                const bool wall = q.walls & (1u << a);
                if (wall) {
                    if (q.X0[a] - q.radius < 1.0 || q.X0[a] + q.radius > nn[a] - 2.0)
                        return fmt("replica %d: sphere needs one node of clearance from the walls on axis %d", r, a);
                } else {
                    if (S > nn[a]) return fmt("replica %d: periodic axis %d shorter than 2 ceil(R) + 6", r, a);
                    if (q.X0[a] < 0.0 || q.X0[a] >= nn[a]) return fmt("replica %d: X0 outside the box", r);
                }
                if (!(std::fabs(q.U0[a]) < 0.5)) return fmt("replica %d: |U0| must be < 0.5", r);
            }
        }
    }
    // spheres in one fluid start with disjoint bounding boxes
    for (int r = 0; r < n; r++) {
        if (G.prim[r] == r) continue;
        const int32_t n3[3] = {p[r].nx, p[r].ny, p[r].nz};
        int32_t oa[3];
        init_org(p[r], oa);
        for (int e = G.prim[r]; e < r; e++) {
            int32_t ob[3];
            init_org(p[e], ob);
            if (boxes_overlap(oa, bbox_edge(p[r]), ob, bbox_edge(p[e]), n3, p[r].walls))
                return fmt("entries %d and %d: the spheres' bounding boxes (edge 2 ceil(R) + 6) overlap", e, r);
        }
    }
    return "";
}

}  // namespace

struct lbm_ctx {
    std::vector<lbm_params> p;     // entries, fluid fields resolved to each group's primary
    std::vector<int> prim, nsph;   // group primary and group size of each entry
    int nrep = 0, prec = 0;
    size_t es = 0;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    hipStream_t stream = nullptr;
    int device = 0;           // device current at lbm_init (the stream's)
    Layout L;
    std::vector<RepDesc> desc;
    std::vector<int32_t> tables;
    int block = 256, cz = 8, maxnx = 0;
    int main_grid = 0, k3_grid = 0, init_grid = 0;
    size_t lds = 0;
    int cur = 0;
    int tau1 = 0;
    int noise = 0;            // some replica has kT > 0
    int groups = 0;           // some fluid holds several spheres
    int graph_steps = 0, graph_parity = -1;
    hipGraphExec_t gexec = nullptr;
    bool timing = false;
    int timing_every = 1;     // plain-launch steps: events around every k-th main launch
    int64_t timing_step = 0;  // plain-launch steps since timing was enabled
    std::vector<hipEvent_t> ev;
    size_t ev_used = 0;
    // adjoint tape left by lbm_adjoint_forward for lbm_adjoint_backward
    struct {
        bool valid = false;
        int32_t nsteps = 0, segment = 0;
        char *buf = nullptr;
        size_t bytes = 0;
        int64_t step_end = 0;
    } tape;
    std::string err;

    RepDesc *d_desc() { return reinterpret_cast<RepDesc *>(ws + L.desc); }
    RepState *d_state() { return reinterpret_cast<RepState *>(ws + L.state); }
    int32_t *d_tables() { return reinterpret_cast<int32_t *>(ws + L.tables); }
    void *d_pop(int k) { return ws + L.pop[k]; }
    double *d_part1() { return reinterpret_cast<double *>(ws + L.part1); }
    double *d_part3() { return reinterpret_cast<double *>(ws + L.part3); }
    double *d_raw() { return reinterpret_cast<double *>(ws + L.raw); }
    double *d_vrho() { return reinterpret_cast<double *>(ws + L.vrho); }
    double *d_rho_n() { return reinterpret_cast<double *>(ws + L.rho_n); }
    uint32_t *d_pmask() { return reinterpret_cast<uint32_t *>(ws + L.pmask); }
    double *d_series() { return reinterpret_cast<double *>(ws + L.series); }
    double *d_aux() { return reinterpret_cast<double *>(ws + L.aux); }
};

namespace {

int fail(lbm_ctx *c, int code, const std::string &m) {
    if (c) c->err = m;
    else g_init_error = m;
    return code;
}

int hip_fail(lbm_ctx *c, hipError_t e, const char *what) {
    return fail(c, LBM_EDEVICE, fmt("%s: %s", what, hipGetErrorString(e)));
}

#define HIP_TRY(c, call)                                                                           \
    do {                                                                                           \
        hipError_t e_ = (call);                                                                    \
        if (e_ != hipSuccess) return hip_fail((c), e_, #call);                                     \
    } while (0)

// rows of one main-kernel tile of replica q for the context's block
int tile_rows(const lbm_ctx *c, const lbm_params &q) { return std::max(1, std::min(q.ny, c->block / q.nx)); }

// LDS of the main kernel for the context's block: a 4-plane ring of both
// components' densities over the tile rows plus a one-row halo on each side
size_t main_lds_bytes(const lbm_ctx *c) {
    size_t elems = 0;
    for (int r = 0; r < c->nrep; r++)
        elems = std::max(elems, (size_t)8 * (tile_rows(c, c->p[r]) + 2) * c->p[r].nx);
    return elems * (c->prec == LBM_FP64 ? 8 : 4);
}

// tiling of the main kernel and the workgroup tables
void build_tiling(lbm_ctx *c) {
    const int n = c->nrep;
    c->tables.assign(3 * (n + 1), 0);
    int32_t *wg_begin = c->tables.data(), *k3_begin = wg_begin + (n + 1), *init_begin = k3_begin + (n + 1);
    int wg = 0, k3 = 0, iw = 0;
    for (int r = 0; r < n; r++) {
        RepDesc &D = c->desc[r];
        const lbm_params &q = c->p[r];
        D.ty = tile_rows(c, q);
        D.nty = (q.ny + D.ty - 1) / D.ty;
        D.cz = std::min(c->cz, q.nz);
        D.nchunk = (q.nz + D.cz - 1) / D.cz;
        // main-kernel tiles for a group's primary only (an entry with none is
        // never the last one at or below a workgroup's index)
        D.wg_begin = wg;
        wg_begin[r] = wg;
        if (c->prim[r] == r) wg += D.nty * D.nchunk;
        D.k3_begin = k3;
        k3_begin[r] = k3;
        D.k3_count = c->L.k3_count[r];
        k3 += D.k3_count;
        init_begin[r] = iw;
        iw += (int)c->L.init_wg[r];
    }
    for (int r = 0; r < n; r++) {
        RepDesc &D = c->desc[r];
        D.k3_total = 0;
        for (int e = c->prim[r]; e < c->prim[r] + c->nsph[r]; e++) D.k3_total += c->L.k3_count[e];
    }
    wg_begin[n] = wg;
    k3_begin[n] = k3;
    init_begin[n] = iw;
    c->main_grid = wg;
    c->k3_grid = k3;
    c->init_grid = iw;
    c->lds = main_lds_bytes(c);
}

// Longest z-chunk (a power of two up to 16) that still gives the main
// kernel about four resident waves per SIMD on 256 CUs; 2 if none does.
int auto_zchunk(lbm_ctx *c) {
    const int64_t want = 256 * 16 / (c->block / 64);
    for (int cz = 16; cz >= 2; cz /= 2) {
        int64_t wgs = 0;
        for (int r = 0; r < c->nrep; r++) {
            if (c->prim[r] != r) continue;
            const lbm_params &q = c->p[r];
            const int ty = tile_rows(c, q);
            wgs += (int64_t)((q.ny + ty - 1) / ty) * ((q.nz + cz - 1) / cz);
        }
        if (wgs >= want) return cz;
    }
    return 2;
}

int upload_desc(lbm_ctx *c) {
    HIP_TRY(c, hipMemcpyAsync(c->d_desc(), c->desc.data(), sizeof(RepDesc) * c->nrep,
                              hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->d_tables(), c->tables.data(), sizeof(int32_t) * c->tables.size(),
                              hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return LBM_OK;
}

void drop_graph(lbm_ctx *c) {
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);  // teardown: nothing to report
    c->gexec = nullptr;
    c->graph_parity = -1;
}

// Per-step scratch of the step kernels: link and event partials, the box
// nodes' post-streaming moments and step densities.  Written and consumed
// within one step; nothing in it carries over.
struct StepScratch {
    double *part1, *part3, *raw, *rho_n;
};

StepScratch workspace_scratch(lbm_ctx *c) {
    return {c->d_part1(), c->d_part3(), c->d_raw(), c->d_rho_n()};
}

int enqueue_step(lbm_ctx *c, bool timed, const StepScratch &sc) {
    MainArgs m;
    m.desc = c->d_desc();
    m.state = c->d_state();
    m.wg_begin = c->d_tables();
    m.nrep = c->nrep;
    m.src = c->d_pop(c->cur);
    m.dst = c->d_pop(1 - c->cur);
    m.pmask = c->d_pmask();
    m.vrho = c->d_vrho();
    m.rho_n = sc.rho_n;
    m.tau1 = c->tau1;
    m.noise = c->noise;
    m.groups = c->groups;
    if (timed && c->ev_used + 2 > c->ev.size()) {
        for (int k = 0; k < 256; k++) {
            hipEvent_t e;
            HIP_TRY(c, hipEventCreate(&e));
            c->ev.push_back(e);
        }
    }
    if (timed) HIP_TRY(c, hipEventRecord(c->ev[c->ev_used], c->stream));
    hipError_t e = launch_main(c->prec, m, c->main_grid, c->block, c->lds, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "main kernel launch");
    if (timed) {
        HIP_TRY(c, hipEventRecord(c->ev[c->ev_used + 1], c->stream));
        c->ev_used += 2;
    }
    LinkArgs la;
    la.desc = c->d_desc();
    la.state = c->d_state();
    la.k3_begin = c->d_tables() + (c->nrep + 1);
    la.nrep = c->nrep;
    la.buf = c->d_pop(1 - c->cur);
    la.vrho = c->d_vrho();
    la.rho_n = sc.rho_n;
    la.raw = sc.raw;
    la.part1 = sc.part1;
    e = launch_links(c->prec, la, c->k3_grid, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "link kernel launch");
    ParticleArgs pa;
    pa.desc = c->d_desc();
    pa.state = c->d_state();
    pa.k3_begin = c->d_tables() + (c->nrep + 1);
    pa.nrep = c->nrep;
    pa.buf = c->d_pop(1 - c->cur);
    pa.part1 = sc.part1;
    pa.part3 = sc.part3;
    pa.pmask = c->d_pmask();
    pa.raw = sc.raw;
    pa.vrho = c->d_vrho();
    pa.series = c->d_series();
    // many particle workgroups: a separate finishing launch beats one
    // device-scope fence per workgroup (192-replica ensemble: 4.02 against
    // 4.30 ms per step); few: the fences are cheaper than the extra launch
    // (64x64x256 channel, 168 workgroups: 0.1365 against 0.1403 ms per step)
    pa.finish_apart = c->k3_grid > K3_FINISH_APART ? 1 : 0;
    e = launch_particle(c->prec, pa, c->k3_grid, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "particle kernel launch");
    c->cur = 1 - c->cur;
    return LBM_OK;
}

// status of a replica's sticky flags
int flag_status(lbm_ctx *c, uint32_t flags) {
    if (flags & FLAG_UNSTABLE) return fail(c, LBM_EUNSTABLE, "run went unstable");
    if (flags & FLAG_CONTACT)
        return fail(c, LBM_ECONTACT, "two spheres in one fluid came close enough for their bounding boxes to overlap");
    return LBM_OK;
}

int check_rep(lbm_ctx *c, int r) {
    if (!c) return LBM_EINVAL;
    if (r < 0 || r >= c->nrep) return fail(c, LBM_EINVAL, fmt("replica %d out of range", r));
    return LBM_OK;
}

int read_state(lbm_ctx *c, int r, RepState *s) {
    HIP_TRY(c, hipMemcpyAsync(s, c->d_state() + r, sizeof(RepState), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return LBM_OK;
}

// ------------------------------------------------------------------ adjoint
// Device memory of one adjoint call, in the caller's buffer: checkpoints at
// the start of every segment and after the last step, the moments and states
// recorded while a segment is replayed, two adjoint states of 8 values per
// node, the node-force adjoint, bounding-box arrays and partial sums.
// rows per tile of the adjoint's node kernel (one plane per tile) and its
// LDS bytes (10 staged values over the tile rows plus a one-row halo on each
// side, on the tile's plane and the planes above and below).  A workgroup
// holds at most 160 KiB of LDS on gfx950; 1 KiB of it is left for the
// kernel's static reduction array (416 bytes).
constexpr size_t ADJ_LDS_MAX = 160 * 1024 - 1024;
int adj_tile_rows(const lbm_params &q) { return std::max(1, std::min(q.ny, 256 / q.nx)); }
size_t adj_lds_bytes(const lbm_params &q, int prec) {
    return (size_t)3 * 10 * (adj_tile_rows(q) + 2) * q.nx * (prec == LBM_FP64 ? 8 : 4);
}

struct AdjLayout {
    int nseg = 0, seg = 0, nwg = 0, nbw = 0, nmw = 0, lty = 0, nlt = 0;
    size_t ckb = 0, recb = 0, Ab = 0;
    size_t ck = 0, rec = 0, rst = 0, A[2] = {0, 0}, Fb = 0, vt = 0, vinv = 0, vtb = 0, ubn = 0, nfw = 0,
           partA = 0, partB = 0, partE = 0, partC = 0, partL = 0, partM = 0, adj = 0, total = 0;
};

int adj_check(lbm_ctx *c, int32_t nsteps, int32_t segment) {
    if (!c) return LBM_EINVAL;
    if (c->nrep != 1) return fail(c, LBM_EINVAL, "the adjoint takes a single-replica, single-sphere context");
    if (!c->tau1) return fail(c, LBM_EINVAL, "the adjoint needs every relaxation time equal to 1");
    if (!c->desc[0].has_particle) return fail(c, LBM_EINVAL, "the adjoint needs a sphere (radius > 0)");
    if (nsteps < 1) return fail(c, LBM_EINVAL, "nsteps must be >= 1");
    if (segment < 0) return fail(c, LBM_EINVAL, "segment must be >= 0 (0: 50 steps)");
    if (adj_lds_bytes(c->p[0], c->prec) > ADJ_LDS_MAX)
        return fail(c, LBM_EINVAL, "x-rows too long for the adjoint's LDS tiles at this precision "
                                   "(FP64: nx <= 226)");
    return LBM_OK;
}

AdjLayout adj_plan(lbm_ctx *c, int32_t nsteps, int32_t segment) {
    AdjLayout A;
    A.seg = std::min(segment > 0 ? segment : 50, nsteps);
    A.nseg = (nsteps + A.seg - 1) / A.seg;
    const int64_t N = c->desc[0].N;
    const size_t te = c->prec == LBM_FP64 ? 8 : 4;
    const int64_t S3 = c->L.S3tot;
    A.nwg = (int)((N + 255) / 256);
    A.nbw = (int)((S3 + 255) / 256);
    {
        // node-kernel tiles: ty full x-rows of one plane
        const lbm_params &q = c->p[0];
        A.lty = adj_tile_rows(q);
        A.nlt = (int)((int64_t)((q.ny + A.lty - 1) / A.lty) * q.nz);
    }
    {
        const lbm_params &q = c->p[0];
        const int64_t nn[3] = {q.nx, q.ny, q.nz};
        int64_t faces = 0;
        for (int ax = 0; ax < 3; ax++)
            if (q.walls & (1u << ax)) faces += 2 * nn[(ax + 1) % 3] * nn[(ax + 2) % 3];
        A.nmw = (int)std::max<int64_t>(1, (faces + 255) / 256);
    }
    lbm_checkpoint_bytes(c, &A.ckb);
    A.ckb = align_up(A.ckb);
    A.recb = align_up(8 * N * te);
    A.Ab = align_up(8 * N * te);
    size_t o = 0;
    auto take = [&](size_t bytes) { const size_t at = o; o = align_up(o + bytes); return at; };
    A.ck = take(A.ckb * (A.nseg + 1));
    A.rec = take(A.recb * (A.seg + 1));
    A.rst = take(sizeof(RepState) * (A.seg + 1));
    A.A[0] = take(A.Ab);
    A.A[1] = take(A.Ab);
    A.Fb = take(6 * N * te);
    A.vt = take(sizeof(double) * 2 * S3);
    A.vinv = take(sizeof(double) * S3);
    A.vtb = take(sizeof(double) * 2 * S3);
    A.ubn = take(sizeof(double) * 2 * S3);
    A.nfw = take(NODE_FWD_BYTES * S3);
    A.partA = take(sizeof(double) * ADJ_PA * A.nlt);
    A.partB = take(sizeof(double) * ADJ_PB * A.nwg);
    A.partE = take(sizeof(double) * PART * A.nbw);
    A.partC = take(sizeof(double) * PART * A.nbw);
    A.partL = take(sizeof(double) * PART * 2 * A.nbw);
    A.partM = take(sizeof(double) * PART * A.nmw);
    A.adj = take(sizeof(AdjState));
    A.total = o;
    return A;
}

}  // namespace

extern "C" {
#define LBM_API __attribute__((visibility("default")))

LBM_API int lbm_workspace_bytes(const lbm_params *p, int32_t n_replicas, int32_t precision, size_t *bytes) {
    Groups G;
    const std::string v = validate(p, n_replicas, precision, G);
    if (!v.empty()) return fail(nullptr, LBM_EINVAL, v);
    if (!bytes) return fail(nullptr, LBM_EINVAL, "bytes is NULL");
    *bytes = plan(G, precision).total;
    return LBM_OK;
}

LBM_API int lbm_init(const lbm_params *p_in, int32_t n_replicas, int32_t precision, void *dev_ws,
             size_t ws_bytes, void *hip_stream, lbm_ctx **out) {
    if (!out) return fail(nullptr, LBM_EINVAL, "out is NULL");
    *out = nullptr;
    Groups G;
    const std::string v = validate(p_in, n_replicas, precision, G);
    if (!v.empty()) return fail(nullptr, LBM_EINVAL, v);
    if (!dev_ws || ((uintptr_t)dev_ws % ALIGN) != 0)
        return fail(nullptr, LBM_ENOMEM, "workspace must be a 256-byte aligned device pointer");
    const lbm_params *p = G.q.data();
    Layout L = plan(G, precision);
    if (ws_bytes < L.total)
        return fail(nullptr, LBM_ENOMEM, fmt("workspace of %zu bytes is smaller than the %zu needed",
                                             ws_bytes, L.total));
    lbm_ctx *c = new lbm_ctx();
    c->p.assign(p, p + n_replicas);
    c->nrep = n_replicas;
    c->prec = precision;
    c->es = elem_size(precision);
    c->ws = reinterpret_cast<char *>(dev_ws);
    c->ws_bytes = ws_bytes;
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return fail(nullptr, LBM_EDEVICE, "hipGetDevice failed");
    }
    c->L = L;
    c->prim = G.prim;
    c->nsph = G.nsph;
    for (int r = 0; r < n_replicas; r++) c->groups = c->groups || G.nsph[r] > 1;
    c->desc.resize(n_replicas);
    c->tau1 = 1;
    std::vector<RepState> st(n_replicas);
    for (int r = 0; r < n_replicas; r++) {
        const lbm_params &q = p[r];
        RepDesc &D = c->desc[r];
        std::memset(&D, 0, sizeof(D));
        D.nx = q.nx; D.ny = q.ny; D.nz = q.nz; D.walls = q.walls;
        D.N = (int64_t)q.nx * q.ny * q.nz;
        D.NP = (int64_t)(q.nx + 2) * (q.ny + 2) * (q.nz + 2);
        D.pop_off = L.pop_off[r];
        D.S = L.S[r];
        D.has_particle = has_sphere(q);
        D.bbox_off = L.bbox_off[r];
        D.part3_off = L.part3_off[r];
        D.series_off = L.series_off[r];
        D.series_cap = q.series_cap;
        D.rho0[0] = q.rho0[0]; D.rho0[1] = q.rho0[1];
        D.G = q.G;
        D.radius = D.has_particle ? q.radius : 0.0;
        D.R2 = D.radius * D.radius;
        D.rho_p = q.rho_p;
        const double V = D.has_particle ? 4.0 / 3.0 * M_PI * q.radius * q.radius * q.radius : 0.0;
        D.mp = q.rho_p * V;
        D.Ip = 0.4 * D.mp * q.radius * q.radius;
        D.drho = q.wet_drho;
        D.tau[0] = q.tau_shear; D.tau[1] = q.tau_bulk; D.tau[2] = q.tau_mom; D.tau[3] = q.tau_ghost;
        for (double t : D.tau)
            if (t != 1.0) c->tau1 = 0;
        D.kT = q.kT;
        if (q.kT > 0.0) c->noise = 1;
        D.init_amp = q.init_amp;
        D.init_split = q.init_split;
        // rows of at most two cache lines (padded): their x-ghost elements sit in
        // lines shared with row ends, so filling them saves a read-modify-write
        // per line (32x32x128 replicas: 2055 -> 1677 us per main kernel; rows
        // of 264 bytes and more are faster without)
        D.ghost_fill = (int32_t)((size_t)(q.nx + 2) * elem_size(precision) <= 256);
        D.key0 = (uint32_t)(q.seed & 0xffffffffu);
        D.key1 = (uint32_t)(q.seed >> 32) ^ (uint32_t)q.replica;
        D.noise_diffusive = q.noise_diffusive;
        D.fixed_velocity = q.fixed_velocity;
        D.primary = G.prim[r];
        D.n_sph = G.nsph[r];
        RepState &s = st[r];
        std::memset(&s, 0, sizeof(s));
        for (int a = 0; a < 3; a++) {
            s.X[a] = q.X0[a]; s.Xp[a] = q.X0[a];
            s.U[a] = D.has_particle ? q.U0[a] : 0.0;
            s.W[a] = D.has_particle ? q.W0[a] : 0.0;
        }
    }
    for (int r = 0; r < n_replicas; r++) c->maxnx = std::max(c->maxnx, p[r].nx);
    c->cz = auto_zchunk(c);
    build_tiling(c);
    int rc = upload_desc(c);
    if (rc != LBM_OK) { g_init_error = c->err; delete c; return rc; }
    hipError_t e = hipMemcpyAsync(c->d_state(), st.data(), sizeof(RepState) * n_replicas,
                                  hipMemcpyHostToDevice, c->stream);
    InitArgs ia;
    ia.desc = c->d_desc();
    ia.state = c->d_state();
    ia.init_begin = c->d_tables() + 2 * (n_replicas + 1);
    ia.nrep = n_replicas;
    ia.buf = c->d_pop(0);
    ia.mass = c->d_aux();
    ia.vrho = c->d_vrho();
    ia.pmask = c->d_pmask();
    if (e == hipSuccess) e = launch_init(precision, ia, c->init_grid, n_replicas, c->stream);
    std::vector<double> mass(2 * L.init_tot);
    if (e == hipSuccess)
        e = hipMemcpyAsync(mass.data(), c->d_aux(), sizeof(double) * mass.size(),
                           hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        g_init_error = fmt("initialisation: %s", hipGetErrorString(e));
        delete c;
        return LBM_EDEVICE;
    }
    // initial fluid mass per group (its primary's workgroups), external force
    // per sphere; under balanced driving the fluid carries minus the sum over
    // the group's spheres, spread over its mass
    int64_t w = 0;
    for (int r = 0; r < n_replicas; r++) {
        const lbm_params &q = p[r];
        RepDesc &D = c->desc[r];
        double M = 0.0;
        for (int64_t k = 0; k < L.init_wg[r]; k++, w++) M += mass[2 * w] + mass[2 * w + 1];
        D.M0 = G.prim[r] == r ? M : c->desc[G.prim[r]].M0;
        const double V = D.has_particle ? 4.0 / 3.0 * M_PI * q.radius * q.radius * q.radius : 0.0;
        const double rho_tot0 = q.rho0[0] + q.rho0[1];
        for (int a = 0; a < 3; a++)
            D.Fext[a] = q.force_mode == 1 ? V * q.rho_p * q.g[a] : V * (q.rho_p - rho_tot0) * q.g[a];
    }
    for (int r = 0; r < n_replicas; r++) {
        const lbm_params &q = p[r];
        RepDesc &D = c->desc[r];
        const int pr = G.prim[r];
        for (int a = 0; a < 3; a++) {
            double tot = 0.0;
            for (int e = pr; e < pr + G.nsph[r]; e++) tot += c->desc[e].Fext[a];
            if (q.force_mode == 1) D.af[a] = q.g[a];
            else D.af[a] = D.M0 > 0.0 ? -tot / D.M0 : 0.0;
        }
    }
    for (int r = 0; r < n_replicas; r++) {
        RepDesc &D = c->desc[r];
        D.cf32 = make_coef<float>(D.rho0[0], D.rho0[1], D.tau[0], D.tau[1], D.tau[2], D.tau[3], D.kT,
                                  D.noise_diffusive);
        D.cf64 = make_coef<double>(D.rho0[0], D.rho0[1], D.tau[0], D.tau[1], D.tau[2], D.tau[3], D.kT,
                                   D.noise_diffusive);
        D.G32 = (float)D.G;
        for (int a = 0; a < 3; a++) D.af32[a] = (float)D.af[a];
    }
    rc = upload_desc(c);
    if (rc != LBM_OK) { g_init_error = c->err; delete c; return rc; }
    // fluid nodes of a group: every sphere's initial layer counted its own
    // particle nodes only
    bool groups = false;
    for (int r = 0; r < n_replicas; r++) groups = groups || G.nsph[r] > 1;
    if (groups) {
        e = hipMemcpyAsync(st.data(), c->d_state(), sizeof(RepState) * n_replicas, hipMemcpyDeviceToHost,
                           c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e == hipSuccess) {
            for (int r = 0; r < n_replicas; r++) {
                if (G.prim[r] != r || G.nsph[r] == 1) continue;
                const double N = (double)c->desc[r].N;
                double solid = 0.0;
                for (int k = r; k < r + G.nsph[r]; k++) solid += N - st[k].n_fluid;
                for (int k = r; k < r + G.nsph[r]; k++) st[k].n_fluid = N - solid;
            }
            e = hipMemcpyAsync(c->d_state(), st.data(), sizeof(RepState) * n_replicas, hipMemcpyHostToDevice,
                               c->stream);
        }
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) {
            g_init_error = fmt("initialisation: %s", hipGetErrorString(e));
            delete c;
            return LBM_EDEVICE;
        }
    }
    c->cur = 0;
    *out = c;
    return LBM_OK;
}

LBM_API int lbm_step(lbm_ctx *c, int32_t nsteps) {
    if (!c) return LBM_EINVAL;
    if (nsteps < 0) return fail(c, LBM_EINVAL, "nsteps must be >= 0");
    c->tape.valid = false;
    int32_t left = nsteps;
    if (c->graph_steps > 0 && !c->timing) {
        while (left >= c->graph_steps) {
            if (!c->gexec || c->graph_parity != c->cur) {
                drop_graph(c);
                const int parity = c->cur;
                HIP_TRY(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
                int rc = LBM_OK;
                for (int k = 0; k < c->graph_steps && rc == LBM_OK; k++) rc = enqueue_step(c, false, workspace_scratch(c));
                hipGraph_t graph = nullptr;
                hipError_t e = hipStreamEndCapture(c->stream, &graph);
                c->cur = parity;  // capture only recorded the launches
                if (rc != LBM_OK) { if (graph) (void)hipGraphDestroy(graph); return rc; }
                if (e != hipSuccess) return hip_fail(c, e, "hipStreamEndCapture");
                e = hipGraphInstantiate(&c->gexec, graph, nullptr, nullptr, 0);
                (void)hipGraphDestroy(graph);  // the executable graph keeps what it needs
                if (e != hipSuccess) { c->gexec = nullptr; return hip_fail(c, e, "hipGraphInstantiate"); }
                c->graph_parity = parity;
            }
            HIP_TRY(c, hipGraphLaunch(c->gexec, c->stream));
            if (c->graph_steps % 2) c->cur = 1 - c->cur;
            left -= c->graph_steps;
        }
    }
    for (int32_t k = 0; k < left; k++) {
        const bool timed = c->timing && (c->timing_step++ % c->timing_every) == 0;
        const int rc = enqueue_step(c, timed, workspace_scratch(c));
        if (rc != LBM_OK) return rc;
    }
    return LBM_OK;
}

LBM_API int lbm_step_noalloc(lbm_ctx *c, int32_t nsteps) {
    if (!c) return LBM_EINVAL;
    if (nsteps < 0) return fail(c, LBM_EINVAL, "nsteps must be >= 0");
    c->tape.valid = false;
    // the per-step scratch this context needs, carved as in the workspace
    const size_t b1 = align_up(sizeof(double) * std::max<int64_t>(c->L.part3_tot, 1));
    const size_t b3 = b1;
    const size_t braw = align_up(sizeof(double) * std::max<int64_t>(RAW * c->L.S3tot, 1));
    const size_t brho = align_up(sizeof(double) * std::max<int64_t>(2 * c->L.S3tot, 1));
    const size_t need = b1 + b3 + braw + brho;
    if (need > STATIC_SCRATCH_BYTES)
        return fail(c, LBM_EINVAL, fmt("lbm_step_noalloc: the context needs %zu bytes of step scratch, "
                                       "more than the %zu of the static array", need, STATIC_SCRATCH_BYTES));
    if (c->device < 0 || c->device >= MAX_DEVICES) return fail(c, LBM_EDEVICE, "device index out of range");
    char *base = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mutex);
        if (!g_scratch_ptr[c->device]) {
            int cur = 0;
            HIP_TRY(c, hipGetDevice(&cur));
            if (cur != c->device) HIP_TRY(c, hipSetDevice(c->device));
            void *ptr = nullptr;
            const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
            if (cur != c->device) HIP_TRY(c, hipSetDevice(cur));
            if (e != hipSuccess) return hip_fail(c, e, "hipGetSymbolAddress(scratch)");
            g_scratch_ptr[c->device] = ptr;
        }
        base = reinterpret_cast<char *>(g_scratch_ptr[c->device]);
    }
    StepScratch sc;
    sc.part1 = reinterpret_cast<double *>(base);
    sc.part3 = reinterpret_cast<double *>(base + b1);
    sc.raw = reinterpret_cast<double *>(base + b1 + b3);
    sc.rho_n = reinterpret_cast<double *>(base + b1 + b3 + braw);
    for (int32_t k = 0; k < nsteps; k++) {
        const bool timed = c->timing && (c->timing_step++ % c->timing_every) == 0;
        const int rc = enqueue_step(c, timed, sc);
        if (rc != LBM_OK) return rc;
    }
    return LBM_OK;
}

LBM_API int lbm_sync(lbm_ctx *c) {
    if (!c) return LBM_EINVAL;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return LBM_OK;
}

LBM_API int lbm_particle_state(lbm_ctx *c, int32_t replica, lbm_particle *out) {
    int rc = check_rep(c, replica);
    if (rc != LBM_OK) return rc;
    if (!out) return fail(c, LBM_EINVAL, "out is NULL");
    RepState s;
    rc = read_state(c, replica, &s);
    if (rc != LBM_OK) return rc;
    for (int a = 0; a < 3; a++) {
        out->X[a] = s.X[a]; out->U[a] = s.U[a]; out->W[a] = s.W[a];
        out->F[a] = s.F[a]; out->T[a] = s.T[a]; out->Pev[a] = s.Pev[a]; out->Lev[a] = s.Lev[a];
    }
    out->delta[0] = s.delta[0];
    out->delta[1] = s.delta[1];
    out->n_fluid = s.n_fluid;
    out->step = s.step;
    out->n_covered = s.n_cov;
    out->n_uncovered = s.n_unc;
    out->n_links = s.n_links;
    return flag_status(c, s.flags);
}

LBM_API int lbm_populations(lbm_ctx *c, int32_t replica, double *host_f) {
    int rc = check_rep(c, replica);
    if (rc != LBM_OK) return rc;
    if (!host_f) return fail(c, LBM_EINVAL, "host_f is NULL");
    const lbm_params &q = c->p[replica];
    const int64_t plane = (int64_t)q.nx * q.ny, N = plane * q.nz;
    const size_t cap = 38 * c->L.NPtot * c->es;  // the free population buffer is the scratch
    int zs = (int)std::max<int64_t>(1, std::min<int64_t>(q.nz, cap / (38 * plane * sizeof(double))));
    std::vector<double> host((size_t)38 * plane * zs);
    for (int z0 = 0; z0 < q.nz; z0 += zs) {
        const int z1 = std::min(q.nz, z0 + zs);
        const int64_t cnt = plane * (z1 - z0);
        ExportArgs a;
        a.desc = c->d_desc();
        a.state = c->d_state();
        a.rep = replica;
        a.z_begin = z0;
        a.z_end = z1;
        a.src = c->d_pop(c->cur);
        a.pmask = c->d_pmask();
        a.out = reinterpret_cast<double *>(c->d_pop(1 - c->cur));
        hipError_t e = launch_export(c->prec, a, cnt, c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "export kernel launch");
        HIP_TRY(c, hipMemcpyAsync(host.data(), a.out, sizeof(double) * 38 * cnt,
                                  hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        for (int k = 0; k < 38; k++)
            std::memcpy(host_f + (int64_t)k * N + plane * z0, host.data() + (int64_t)k * cnt,
                        sizeof(double) * cnt);
    }
    return LBM_OK;
}

namespace {
int run_fields(lbm_ctx *c, int r, bool columns) {
    const lbm_params &q = c->p[r];
    const int64_t plane = (int64_t)q.nx * q.ny, N = plane * q.nz;
    FieldArgs a;
    a.desc = c->d_desc();
    a.state = c->d_state();
    a.rep = r;
    a.src = c->d_pop(c->cur);
    a.pmask = c->d_pmask();
    a.vrho = c->d_vrho();
    a.scratch = reinterpret_cast<double *>(c->d_pop(1 - c->cur));
    a.columns = columns ? c->d_aux() : nullptr;
    hipError_t e = launch_fields(c->prec, a, N, plane, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "field kernels launch");
    return LBM_OK;
}
}  // namespace

LBM_API int lbm_fields(lbm_ctx *c, int32_t replica, double *host_rho, double *host_u) {
    int rc = check_rep(c, replica);
    if (rc != LBM_OK) return rc;
    if (!host_rho || !host_u) return fail(c, LBM_EINVAL, "output is NULL");
    rc = run_fields(c, replica, false);
    if (rc != LBM_OK) return rc;
    const lbm_params &q = c->p[replica];
    const int64_t N = (int64_t)q.nx * q.ny * q.nz;
    const double *s = reinterpret_cast<const double *>(c->d_pop(1 - c->cur));
    std::vector<double> sol(N);
    HIP_TRY(c, hipMemcpyAsync(host_rho, s, sizeof(double) * 2 * N, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(host_u, s + 5 * N, sizeof(double) * 3 * N, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(sol.data(), s + 8 * N, sizeof(double) * N, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (int64_t n = 0; n < N; n++)
        if (sol[n] != 0.0) host_rho[n] = host_rho[N + n] = 0.0;
    return LBM_OK;
}

LBM_API int lbm_observables(lbm_ctx *c, int32_t replica, lbm_obs *o) {
    int rc = check_rep(c, replica);
    if (rc != LBM_OK) return rc;
    if (!o) return fail(c, LBM_EINVAL, "o is NULL");
    rc = run_fields(c, replica, true);
    if (rc != LBM_OK) return rc;
    const lbm_params &q = c->p[replica];
    const int64_t plane = (int64_t)q.nx * q.ny;
    std::vector<double> col(8 * plane);
    HIP_TRY(c, hipMemcpyAsync(col.data(), c->d_aux(), sizeof(double) * col.size(),
                              hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int k = 0; k < 8; k++)
        for (int64_t i = 0; i < plane; i++) s[k] += col[k * plane + i];
    o->mass[0] = s[0];
    o->mass[1] = s[1];
    for (int a = 0; a < 3; a++) o->momentum[a] = s[2 + a];
    o->n_fluid = s[7];
    o->u2_mean = s[7] > 0 ? s[5] / s[7] : 0.0;
    o->uz_mean = s[7] > 0 ? s[6] / s[7] : 0.0;
    if (o->uz_profile)
        for (int64_t i = 0; i < plane; i++)
            o->uz_profile[i] = col[7 * plane + i] > 0 ? col[6 * plane + i] / col[7 * plane + i] : 0.0;
    RepState st;
    rc = read_state(c, replica, &st);
    if (rc != LBM_OK) return rc;
    return flag_status(c, st.flags);
}

LBM_API int lbm_u_series(lbm_ctx *c, int32_t replica, double *host_u3, int64_t cap, int64_t *count) {
    int rc = check_rep(c, replica);
    if (rc != LBM_OK) return rc;
    if (!host_u3 || !count || cap < 0) return fail(c, LBM_EINVAL, "bad output arguments");
    RepState st;
    rc = read_state(c, replica, &st);
    if (rc != LBM_OK) return rc;
    const int64_t ring = c->p[replica].series_cap;
    const int64_t avail = std::min<int64_t>(st.step, ring);
    const int64_t n = std::min<int64_t>(avail, cap);
    std::vector<double> buf(3 * ring);
    HIP_TRY(c, hipMemcpyAsync(buf.data(), c->d_series() + c->L.series_off[replica],
                              sizeof(double) * 3 * ring, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    const int64_t first = st.step - n;  // oldest step index returned
    for (int64_t k = 0; k < n; k++) {
        const int64_t slot = (first + k) % ring;
        for (int a = 0; a < 3; a++) host_u3[3 * k + a] = buf[3 * slot + a];
    }
    *count = n;
    return LBM_OK;
}

LBM_API int lbm_checkpoint_bytes(lbm_ctx *c, size_t *bytes) {
    if (!c || !bytes) return LBM_EINVAL;
    *bytes = 38 * c->L.NPtot * c->es + sizeof(RepState) * c->nrep +
             (sizeof(double) * 2 + sizeof(uint32_t)) * c->L.S3tot;
    return LBM_OK;
}

LBM_API int lbm_checkpoint(lbm_ctx *c, void *dev_dst) {
    if (!c || !dev_dst) return LBM_EINVAL;
    char *d = reinterpret_cast<char *>(dev_dst);
    const size_t pb = 38 * c->L.NPtot * c->es, sb = sizeof(RepState) * c->nrep;
    HIP_TRY(c, hipMemcpyAsync(d, c->d_pop(c->cur), pb, hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(d + pb, c->d_state(), sb, hipMemcpyDeviceToDevice, c->stream));
    if (c->L.S3tot) {
        HIP_TRY(c, hipMemcpyAsync(d + pb + sb, c->d_vrho(), sizeof(double) * 2 * c->L.S3tot,
                                  hipMemcpyDeviceToDevice, c->stream));
        HIP_TRY(c, hipMemcpyAsync(d + pb + sb + sizeof(double) * 2 * c->L.S3tot, c->d_pmask(),
                                  sizeof(uint32_t) * c->L.S3tot, hipMemcpyDeviceToDevice, c->stream));
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return LBM_OK;
}

LBM_API int lbm_restore(lbm_ctx *c, const void *dev_src) {
    if (!c || !dev_src) return LBM_EINVAL;
    c->tape.valid = false;
    const char *d = reinterpret_cast<const char *>(dev_src);
    const size_t pb = 38 * c->L.NPtot * c->es, sb = sizeof(RepState) * c->nrep;
    HIP_TRY(c, hipMemcpyAsync(c->d_pop(c->cur), d, pb, hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->d_state(), d + pb, sb, hipMemcpyDeviceToDevice, c->stream));
    if (c->L.S3tot) {
        HIP_TRY(c, hipMemcpyAsync(c->d_vrho(), d + pb + sb, sizeof(double) * 2 * c->L.S3tot,
                                  hipMemcpyDeviceToDevice, c->stream));
        HIP_TRY(c, hipMemcpyAsync(c->d_pmask(), d + pb + sb + sizeof(double) * 2 * c->L.S3tot,
                                  sizeof(uint32_t) * c->L.S3tot, hipMemcpyDeviceToDevice, c->stream));
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return LBM_OK;
}

LBM_API int lbm_set_launch(lbm_ctx *c, int32_t block, int32_t zchunk) {
    if (!c) return LBM_EINVAL;
    if (block != 256 && block != 512 && block != 1024)
        return fail(c, LBM_EINVAL, "block must be 256, 512 or 1024");
    if (zchunk < 0) return fail(c, LBM_EINVAL, "zchunk must be >= 0 (0: automatic)");
    if (block < c->maxnx) return fail(c, LBM_EINVAL, "block must hold one x-row of every replica");
    // build the new tiling aside and commit it only when it fits, so a
    // rejected shape leaves the context (and lbm_get_launch) as it was
    const int old_block = c->block, old_cz = c->cz;
    c->block = block;
    c->cz = zchunk > 0 ? zchunk : auto_zchunk(c);
    if (main_lds_bytes(c) > MAIN_LDS_MAX) {
        c->block = old_block;
        c->cz = old_cz;
        return fail(c, LBM_EINVAL, "launch shape needs too much LDS");
    }
    build_tiling(c);
    drop_graph(c);
    return upload_desc(c);
}

LBM_API int lbm_autotune(lbm_ctx *c, int32_t steps_per_trial, void *dev_ckpt, int32_t *block_out,
                         int32_t *zchunk_out, double *best_ms) {
    if (!c) return LBM_EINVAL;
    c->tape.valid = false;
    if (steps_per_trial < 1) return fail(c, LBM_EINVAL, "steps_per_trial must be >= 1");
    int rc = LBM_OK;
    if (dev_ckpt && (rc = lbm_checkpoint(c, dev_ckpt)) != LBM_OK) return rc;
    const bool timing_was = c->timing;
    const int graph_was = c->graph_steps;
    c->graph_steps = 0;
    // mean main-kernel time of one shape over steps_per_trial timed steps
    auto trial = [&](int blk, int cz, double &ms) -> int {
        c->block = blk;
        c->cz = cz;
        if (main_lds_bytes(c) > MAIN_LDS_MAX) { ms = -1.0; return LBM_OK; }
        build_tiling(c);
        drop_graph(c);
        int r = upload_desc(c);
        if (r != LBM_OK) return r;
        c->timing = false;
        if ((r = enqueue_step(c, false, workspace_scratch(c))) != LBM_OK) return r;  // first launch of this shape
        c->timing = true;
        c->ev_used = 0;
        for (int k = 0; k < steps_per_trial && r == LBM_OK; k++) r = enqueue_step(c, true, workspace_scratch(c));
        if (r != LBM_OK) return r;
        int64_t n = 0;
        return lbm_timing_read(c, &ms, &n);
    };
    struct Cand { int blk, cz; double ms; };
    std::vector<Cand> cands;
    const int blocks[3] = {256, 512, 1024};
    const int chunks[5] = {2, 4, 8, 16, 32};
    for (int bi = 0; bi < 3 && rc == LBM_OK; bi++) {
        if (blocks[bi] < c->maxnx) continue;
        for (int ci = 0; ci < 5 && rc == LBM_OK; ci++) {
            double ms = -1.0;
            rc = trial(blocks[bi], chunks[ci], ms);
            if (rc == LBM_OK && ms > 0.0) cands.push_back({blocks[bi], chunks[ci], ms});
        }
    }
    // the three fastest are timed again; each keeps the better of its two means
    std::sort(cands.begin(), cands.end(), [](const Cand &a, const Cand &b) { return a.ms < b.ms; });
    for (size_t k = 0; k < cands.size() && k < 3 && rc == LBM_OK; k++) {
        double ms = -1.0;
        rc = trial(cands[k].blk, cands[k].cz, ms);
        if (rc == LBM_OK && ms > 0.0) cands[k].ms = std::min(cands[k].ms, ms);
    }
    std::sort(cands.begin(), cands.end(), [](const Cand &a, const Cand &b) { return a.ms < b.ms; });
    int best_b = cands.empty() ? 256 : cands[0].blk, best_cz = cands.empty() ? auto_zchunk(c) : cands[0].cz;
    const double best = cands.empty() ? -1.0 : cands[0].ms;
    c->timing = timing_was;
    c->ev_used = 0;
    c->graph_steps = graph_was;
    c->block = best_b;
    c->cz = best_cz;
    build_tiling(c);
    drop_graph(c);
    const int rc2 = upload_desc(c);
    if (rc == LBM_OK) rc = rc2;
    if (dev_ckpt && rc == LBM_OK) rc = lbm_restore(c, dev_ckpt);
    if (rc != LBM_OK) return rc;
    if (block_out) *block_out = best_b;
    if (zchunk_out) *zchunk_out = best_cz;
    if (best_ms) *best_ms = best;
    return LBM_OK;
}

LBM_API int lbm_get_launch(lbm_ctx *c, int32_t *block, int32_t *zchunk) {
    if (!c || !block || !zchunk) return LBM_EINVAL;
    *block = c->block;
    *zchunk = c->cz;
    return LBM_OK;
}

LBM_API int lbm_set_graph(lbm_ctx *c, int32_t steps_per_graph) {
    if (!c) return LBM_EINVAL;
    if (steps_per_graph < 0) return fail(c, LBM_EINVAL, "steps_per_graph must be >= 0");
    if (steps_per_graph > 0 && c->stream == nullptr)
        return fail(c, LBM_EINVAL, "graph replay needs a non-default stream");
    drop_graph(c);
    c->graph_steps = steps_per_graph;
    return LBM_OK;
}

LBM_API int lbm_timing(lbm_ctx *c, int32_t every) {
    if (!c) return LBM_EINVAL;
    if (every < 0) return fail(c, LBM_EINVAL, "timing interval must be >= 0");
    c->timing = every != 0;
    c->timing_every = every > 0 ? every : 1;
    c->timing_step = 0;
    c->ev_used = 0;
    return LBM_OK;
}

LBM_API int lbm_timing_read(lbm_ctx *c, double *mean_ms, int64_t *count) {
    if (!c || !mean_ms || !count) return LBM_EINVAL;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    double sum = 0.0;
    for (size_t k = 0; k + 1 < c->ev_used; k += 2) {
        float ms = 0.0f;
        HIP_TRY(c, hipEventElapsedTime(&ms, c->ev[k], c->ev[k + 1]));
        sum += ms;
    }
    *count = (int64_t)(c->ev_used / 2);
    *mean_ms = *count ? sum / (double)*count : 0.0;
    return LBM_OK;
}

LBM_API int lbm_step_bytes(lbm_ctx *c, double *bytes) {
    if (!c || !bytes) return LBM_EINVAL;
    *bytes = 2.0 * 38.0 * (double)c->L.Ntot * (double)c->es;
    return LBM_OK;
}

LBM_API int lbm_adjoint_bytes(lbm_ctx *c, int32_t nsteps, int32_t segment, size_t *bytes) {
    const int rc = adj_check(c, nsteps, segment);
    if (rc != LBM_OK) return rc;
    if (!bytes) return fail(c, LBM_EINVAL, "bytes is NULL");
    *bytes = adj_plan(c, nsteps, segment).total;
    return LBM_OK;
}

namespace {
// K steps from the current state, recording the moments and the sphere
// state before every step and after the last (into the tape's record area)
int record_segment(lbm_ctx *c, const AdjLayout &A, char *w, RepState *rst, int K) {
    for (int k = 0; k <= K; k++) {
        RecArgs ra;
        ra.desc = c->d_desc();
        ra.state = c->d_state();
        ra.src = c->d_pop(c->cur);
        ra.rec = w + A.rec + (size_t)k * A.recb;
        ra.st_out = rst + k;
        hipError_t e = launch_adj_record(c->prec, ra, c->desc[0].N, c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "adjoint record launch");
        int r;
        if (k < K && (r = enqueue_step(c, false, workspace_scratch(c))) != LBM_OK) return r;
    }
    return LBM_OK;
}
}  // namespace

namespace {
// Forward sweep of the adjoint form: nsteps steps from the current state with
// a checkpoint at the start of every segment and after the last step; the
// last segment's moments and sphere states are recorded on the way.  Leaves
// the context after the nsteps steps and the tape for adjoint_backward.
int adjoint_forward(lbm_ctx *c, int32_t nsteps, int32_t segment, void *dev_adj, size_t adj_bytes, double *J) {
    c->tape.valid = false;
    int rc = adj_check(c, nsteps, segment);
    if (rc != LBM_OK) return rc;
    const AdjLayout A = adj_plan(c, nsteps, segment);
    if (!dev_adj || ((uintptr_t)dev_adj % ALIGN) != 0)
        return fail(c, LBM_ENOMEM, "adjoint buffer must be a 256-byte aligned device pointer");
    if (adj_bytes < A.total)
        return fail(c, LBM_ENOMEM, fmt("adjoint buffer of %zu bytes is smaller than the %zu needed",
                                       adj_bytes, A.total));
    RepState st0;
    rc = read_state(c, 0, &st0);
    if (rc != LBM_OK) return rc;
    if (st0.flags & FLAG_UNSTABLE) return fail(c, LBM_EUNSTABLE, "the run is unstable");
    char *w = reinterpret_cast<char *>(dev_adj);
    struct TimingOff {
        lbm_ctx *c;
        bool was;
        ~TimingOff() { c->timing = was; }
    } keep{c, c->timing};
    c->timing = false;
    auto ck = [&](int s) { return w + A.ck + (size_t)s * A.ckb; };
    auto seg_len = [&](int s) { return std::min(A.seg, nsteps - s * A.seg); };
    RepState *rst = reinterpret_cast<RepState *>(w + A.rst);
    for (int s = 0; s < A.nseg; s++) {
        if ((rc = lbm_checkpoint(c, ck(s))) != LBM_OK) return rc;
        rc = s + 1 < A.nseg ? lbm_step(c, seg_len(s)) : record_segment(c, A, w, rst, seg_len(s));
        if (rc != LBM_OK) return rc;
    }
    if ((rc = lbm_checkpoint(c, ck(A.nseg))) != LBM_OK) return rc;
    RepState st1;
    if ((rc = read_state(c, 0, &st1)) != LBM_OK) return rc;
    if (J) *J = (st1.uz_sum - st0.uz_sum) / nsteps;
    if (st1.flags & FLAG_UNSTABLE) return fail(c, LBM_EUNSTABLE, "the run went unstable");
    c->tape.valid = true;
    c->tape.nsteps = nsteps;
    c->tape.segment = segment;
    c->tape.buf = w;
    c->tape.bytes = adj_bytes;
    c->tape.step_end = st1.step;
    return LBM_OK;
}

// Reverse sweep over the tape of adjoint_forward: last segment first, each
// segment's steps reversed, every other segment replayed from its checkpoint
// and recorded first.  Leaves the context where the forward sweep left it.
int adjoint_backward(lbm_ctx *c, double grad[5], double *J) {
    if (!c->tape.valid) return fail(c, LBM_ESTATE, "no adjoint tape: call lbm_adjoint_forward first");
    const int32_t nsteps = c->tape.nsteps;
    const AdjLayout A = adj_plan(c, nsteps, c->tape.segment);
    char *w = c->tape.buf;
    RepState stc;
    int rc = read_state(c, 0, &stc);
    if (rc != LBM_OK) return rc;
    if (stc.step != c->tape.step_end)
        return fail(c, LBM_ESTATE, "the context moved since lbm_adjoint_forward");
    c->tape.valid = false;  // the sweep replays and restores: one backward per forward
    const bool timed = c->timing;
    struct TimingOff {
        lbm_ctx *c;
        bool was;
        ~TimingOff() { c->timing = was; }
    } keep{c, c->timing};
    c->timing = false;
    auto ck = [&](int s) { return w + A.ck + (size_t)s * A.ckb; };
    auto seg_len = [&](int s) { return std::min(A.seg, nsteps - s * A.seg); };
    RepState *rst = reinterpret_cast<RepState *>(w + A.rst);
    HIP_TRY(c, hipMemsetAsync(w + A.adj, 0, sizeof(AdjState), c->stream));
    HIP_TRY(c, hipMemsetAsync(w + A.A[0], 0, A.Ab, c->stream));

    const lbm_params &q = c->p[0];
    const RepDesc &D = c->desc[0];
    const double V = 4.0 / 3.0 * M_PI * q.radius * q.radius * q.radius;
    const double cF = q.force_mode == 1 ? V * q.rho_p : V * (q.rho_p - (q.rho0[0] + q.rho0[1]));
    const double caf = q.force_mode == 1 ? 1.0 : (D.M0 > 0.0 ? -cF / D.M0 : 0.0);
    AdjArgs aa;
    aa.desc = c->d_desc();
    aa.adj = reinterpret_cast<AdjState *>(w + A.adj);
    aa.cF = cF;
    aa.invN = 1.0 / nsteps;
    aa.Fb = w + A.Fb;
    aa.vt = reinterpret_cast<double *>(w + A.vt);
    aa.vinv = reinterpret_cast<double *>(w + A.vinv);
    aa.vtb = reinterpret_cast<double *>(w + A.vtb);
    aa.ubn = reinterpret_cast<double *>(w + A.ubn);
    aa.nfw = w + A.nfw;
    aa.partA = reinterpret_cast<double *>(w + A.partA);
    aa.partB = reinterpret_cast<double *>(w + A.partB);
    aa.partE = reinterpret_cast<double *>(w + A.partE);
    aa.partC = reinterpret_cast<double *>(w + A.partC);
    aa.partL = reinterpret_cast<double *>(w + A.partL);
    aa.partM = reinterpret_cast<double *>(w + A.partM);
    aa.nwg = A.nwg;
    aa.lty = A.lty;
    aa.nlt = A.nlt;
    aa.desc_nx = q.nx;
    aa.nbw = A.nbw;
    aa.nmw = A.nmw;
    int an = 0;  // buffer holding the adjoint of the state after the step being reversed
    for (int s = A.nseg - 1; s >= 0; s--) {
        const int K = seg_len(s);
        if (s + 1 < A.nseg) {  // replay (the last segment was recorded by the sweep)
            if ((rc = lbm_restore(c, ck(s))) != LBM_OK) return rc;
            if ((rc = record_segment(c, A, w, rst, K)) != LBM_OK) return rc;
        }
        for (int k = K - 1; k >= 0; k--) {
            aa.stn = rst + k;
            aa.stn1 = rst + k + 1;
            aa.recn = w + A.rec + (size_t)k * A.recb;
            aa.recn1 = w + A.rec + (size_t)(k + 1) * A.recb;
            aa.Anext = w + A.A[an];
            aa.Acur = w + A.A[1 - an];
            hipEvent_t e0 = nullptr, e1 = nullptr;
            if (timed) {
                if (c->ev_used + 2 > c->ev.size()) {
                    for (int q = 0; q < 256; q++) {
                        hipEvent_t ev;
                        HIP_TRY(c, hipEventCreate(&ev));
                        c->ev.push_back(ev);
                    }
                }
                e0 = c->ev[c->ev_used];
                e1 = c->ev[c->ev_used + 1];
                c->ev_used += 2;
            }
            hipError_t e = launch_adj_step(c->prec, aa, c->stream, e0, e1);
            if (e != hipSuccess) return hip_fail(c, e, "adjoint step launch");
            an = 1 - an;
        }
    }
    if ((rc = lbm_restore(c, ck(A.nseg))) != LBM_OK) return rc;
    AdjState h;
    HIP_TRY(c, hipMemcpyAsync(&h, w + A.adj, sizeof(AdjState), hipMemcpyDeviceToHost, c->stream));
    RepState st1;
    if ((rc = read_state(c, 0, &st1)) != LBM_OK) return rc;
    for (int a = 0; a < 3; a++) grad[a] = h.grad[a] + caf * h.afb[a];
    grad[3] = h.grad[3];
    grad[4] = h.grad[4];
    if (J) *J = h.Jsum / nsteps;
    if (st1.flags & FLAG_UNSTABLE) return fail(c, LBM_EUNSTABLE, "the run went unstable");
    return LBM_OK;
}
}  // namespace

LBM_API int lbm_adjoint_forward(lbm_ctx *c, int32_t nsteps, int32_t segment, void *dev_adj, size_t adj_bytes,
                                double *J) {
    if (!c) return LBM_EINVAL;
    if (!J) return fail(c, LBM_EINVAL, "J must not be NULL");
    return adjoint_forward(c, nsteps, segment, dev_adj, adj_bytes, J);
}

LBM_API int lbm_adjoint_backward(lbm_ctx *c, double grad[5]) {
    if (!c) return LBM_EINVAL;
    if (!grad) return fail(c, LBM_EINVAL, "grad must not be NULL");
    return adjoint_backward(c, grad, nullptr);
}

LBM_API int lbm_adjoint(lbm_ctx *c, int32_t nsteps, int32_t segment, void *dev_adj, size_t adj_bytes,
                        double grad[5], double *J) {
    if (!c) return LBM_EINVAL;
    if (!grad || !J) return fail(c, LBM_EINVAL, "grad and J must not be NULL");
    int rc = adjoint_forward(c, nsteps, segment, dev_adj, adj_bytes, nullptr);
    if (rc != LBM_OK) return rc;
    return adjoint_backward(c, grad, J);
}



LBM_API void lbm_destroy(lbm_ctx *c) {
    if (!c) return;
    drop_graph(c);
    // teardown: errors here have no caller to go to
    for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
    delete c;
}

LBM_API const char *lbm_last_error(const lbm_ctx *c) {
    return c ? c->err.c_str() : g_init_error.c_str();
}

}  // extern "C"
