/*
 * lbm.h — C ABI of the MI355X (gfx950) library for the fluctuating
 * two-component D3Q19 lattice Boltzmann step with a settling, wettable,
 * finite-size sphere (Xue, Biferale, Sbragaglia, Toschi, "A lattice
 * Boltzmann study of particle settling in a fluctuating multicomponent fluid
 * under confinement").
 *
 * What one step computes (Sec. 2 of the paper, "Methodology"):
 *   - moments rho_l, rho_tot v of the populations f_{l i} (eq. density);
 *   - the Shan-Chen force between components (eq. sc-force) plus the body
 *     force, with a virtual wetting layer on particle nodes (mean density of
 *     the fluid neighbours + / - Delta rho) and neutral (mirror) walls;
 *   - MRT collision in an orthogonal mode basis with Guo forcing at the
 *     hydrodynamic velocity v + (F_A + F_B)/(2 rho_tot), and thermal noise on
 *     every non-conserved mode obeying fluctuation-dissipation (eq. lbe);
 *   - streaming with half-way bounce-back on the walls and moving-wall
 *     bounce-back on the sphere, with momentum exchange on every link;
 *   - leap-frog Newton-Euler update of the sphere under the external force
 *     of Sec. 3, eq. (fp), cover/uncover of nodes, global mass correction.
 *
 * Conventions.  Lattice units.  Node (x, y, z), 0 <= x < nx etc., sits at
 * position (x, y, z); a walled axis has its walls half-way outside the first
 * and last node.  Populations exchanged with the host are FP64 arrays laid
 * out [component 2][direction 19][z][y][x].  Direction order: rest;
 * +x, -x, +y, -y, +z, -z; (1,1,0), (-1,-1,0), (1,-1,0), (-1,1,0);
 * (1,0,1), (-1,0,-1), (1,0,-1), (-1,0,1); (0,1,1), (0,-1,-1), (0,1,-1),
 * (0,-1,1).
 *
 * Memory ownership.  The caller allocates one device workspace of
 * lbm_workspace_bytes() bytes (256-byte aligned) and keeps it alive until
 * lbm_destroy(); the library never allocates or frees device memory.  The
 * library copies the parameters and owns the host context.  Every host array
 * is caller-owned.
 *
 * Errors.  Every call returns an lbm_status; nothing is thrown or aborted
 * across the ABI.  Invalid arguments return LBM_EINVAL before any device
 * work.  lbm_last_error() gives a message.  A step that produces a
 * non-finite or negative density, or a sphere that leaves its channel, sets
 * a sticky flag: the state queries then return LBM_EUNSTABLE (after filling
 * their outputs) until lbm_restore().  Spheres of one fluid whose bounding
 * boxes meet set another (LBM_ECONTACT, see "Several spheres").
 *
 * Streams.  All device work is enqueued on the hip_stream given to
 * lbm_init (NULL = the default stream).  lbm_step is asynchronous; the query
 * calls synchronise that stream.  A context is not thread-safe.
 */
#ifndef LBM_H
#define LBM_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx;

enum {
    LBM_OK = 0,
    LBM_EINVAL = -1,    /* invalid argument or configuration            */
    LBM_ENOMEM = -2,    /* workspace too small or misaligned            */
    LBM_EDEVICE = -3,   /* HIP runtime error                            */
    LBM_EUNSTABLE = -4, /* the run went unstable (sticky)               */
    LBM_ESTATE = -5,    /* call not valid in the current context state  */
    LBM_ECONTACT = -6   /* spheres in one fluid came into contact (sticky) */
};

enum { LBM_FP64 = 0, LBM_FP32 = 1, LBM_FP16 = 2 };

/* One replica of the problem (Sec. 3 set-up: square channel, sphere at the
 * centre of the cross-section, body force along z). */
typedef struct lbm_params {
    int32_t nx, ny, nz;        /* nodes per axis, 2 <= n, nx <= 256; with NP =            */
                               /* (nx+2)(ny+2)(nz+2): 38 NP < 2^31 and 19 NP bytes(elem)  */
                               /* < 2^32 (FP64: NP < 28.2M, FP32/FP16: NP < 56.5M)         */
    uint32_t walls;            /* bit0 x, bit1 y, bit2 z walls; other axes periodic       */
    double rho0[2];            /* reference densities of A (majority) and B               */
    double init_amp;           /* initial densities rho0_l + init_amp (2u - 1), u uniform */
    double G;                  /* Shan-Chen coupling (eq. sc-force)                       */
    double tau_shear, tau_bulk, tau_mom, tau_ghost; /* relaxation times, > 1/2            */
    double kT;                 /* thermal energy (>= 0)                                   */
    uint64_t seed;             /* Philox key = (lo32(seed), hi32(seed) ^ replica)         */
    int32_t replica;           /* replica index entering the key                          */
    double g[3];               /* body-force acceleration g (Sec. 3)                      */
    int32_t force_mode;        /* 0: sphere gets F_p = V (rho_p - rho_tot0) g (eq. fp),
                                     fluid gets -F_p / M_fluid (net zero); 1: fluid rho g,
                                     sphere rho_p V g                                       */
    double radius;             /* sphere radius d/2 (<= 0: no sphere); a periodic axis     */
                               /* needs n >= 2 ceil(R) + 6, a wall axis one node of       */
                               /* clearance around the initial sphere                     */
    double rho_p;              /* sphere density                                          */
    double wet_drho;           /* wetting-layer offset Delta rho (+A, -B)                 */
    double X0[3], U0[3], W0[3];/* initial centre, velocity, angular velocity              */
    int32_t noise_diffusive;   /* 1: noise on the species-momentum (diffusion) mode       */
    int32_t fixed_velocity;    /* 1: sphere moves with U0, W0 (prescribed)                */
    int32_t series_cap;        /* length of the per-step U ring buffer (>= 1)             */
    int32_t init_split;        /* 0: every node starts from rho0; k in [1, nz): nodes with */
                               /* z >= k start from the swapped pair (rho0[1], rho0[0]),   */
                               /* i.e. the other phase of a demixed mixture, which puts a  */
                               /* flat A|B interface at z = k - 1/2.  LBM_FP16 storage is  */
                               /* relative to rho0, so it holds the swapped phase to about */
                               /* 1e-3 of rho0[0] / rho0[1] only: use FP32 or FP64 there   */
    int32_t shared_fluid;      /* 0: this entry starts a replica (its own fluid); 1: one   */
                               /* more sphere in the fluid of the entry before it (several */
                               /* spheres per fluid, the multi-particle follow-up of Sec. 5)*/
                               /* -- see "Several spheres" below                            */
} lbm_params;

/* Several spheres.  The parameter array passed to lbm_init is a list of
 * entries.  An entry with shared_fluid = 0 starts a replica: its fluid, and
 * its sphere when radius > 0.  Each following entry with shared_fluid = 1
 * adds one sphere to that fluid, up to 16 spheres per fluid: its radius,
 * rho_p, wet_drho, X0, U0 and W0 are its own, and every other field is
 * taken from the replica's first entry.  All spheres of a fluid need
 * radius > 0.  Every sphere keeps its own moving-wall links, wetting layer,
 * cover / uncover events and Newton-Euler step (Sec. 2, applied to each).
 * The mass correction is global: the fluxes of all the spheres are summed,
 * then spread over the fluid nodes that are in no sphere.  Under balanced
 * driving (force_mode 0) the fluid carries minus the sum of the spheres'
 * external forces.  The replica argument of the query calls is an entry
 * index.  lbm_particle_state and lbm_u_series report that entry's sphere;
 * lbm_populations, lbm_fields and lbm_observables report the shared fluid
 * for every entry of a replica.  Each sphere's work covers its bounding box
 * of edge 2 ceil(R) + 6, and the boxes of one fluid must be disjoint:
 * lbm_init rejects spheres whose initial boxes share a node (LBM_EINVAL),
 * and a step that brings two boxes together sets a sticky flag, after which
 * the state queries return LBM_ECONTACT.  Boxes meet when the gap between
 * two spheres falls below 4 to 8 lattice units along an axis (the exact
 * value depends on the radii and on the centres' fractional parts). */

/* Sphere state after the last completed step n. */
typedef struct lbm_particle {
    double X[3], U[3], W[3];   /* X^n, U^{n-1/2}, Omega^{n-1/2}                           */
    double F[3], T[3];         /* total force / torque of step n-1                        */
    double Pev[3], Lev[3];     /* cover/uncover momentum pending for the next step        */
    double delta[2];           /* mass correction per component                           */
    double n_fluid;            /* fluid nodes |Phi^n|                                      */
    int64_t step;              /* n                                                       */
    int64_t n_covered, n_uncovered, n_links;
} lbm_particle;

/* Global observables of the current state of one replica: the fluid's
 * per-component mass and momentum (the moments of eq. density, Sec. 2), the
 * mean square of the hydrodynamic velocity v_H = v + (F_A + F_B)/(2 rho_tot)
 * (Sec. 2, force paragraph) and the settling-direction profile of v_H,z over
 * the channel cross-section, the fluid flow around the particle the set-up
 * of Sec. 3 (Fig. 1 caption) drives.  Sums run over fluid nodes in a fixed
 * order: per (x, y) column along z on the device, then the columns in order
 * on the host. */
typedef struct lbm_obs {
    double mass[2];            /* sum of rho_l over fluid nodes                            */
    double momentum[3];        /* sum of (j_A + j_B) over fluid nodes                      */
    double u2_mean;            /* mean |v_H|^2 over fluid nodes                            */
    double uz_mean;            /* mean v_H,z over fluid nodes                              */
    double n_fluid;
    double *uz_profile;        /* optional [ny][nx]: mean v_H,z over fluid nodes of each
                                  (x, y) column; caller-owned, may be NULL                  */
} lbm_obs;

/* Workspace size for n_replicas parameter sets p[0..n_replicas-1] stored in
 * the given precision (LBM_FP64 / LBM_FP32 / LBM_FP16). */
int lbm_workspace_bytes(const lbm_params *p, int32_t n_replicas, int32_t precision,
                        size_t *bytes);

/* Validate, lay out the workspace, write the initial state (densities
 * rho0_l + init_amp (2u - 1) from Philox counter (node, 0, 0, 1), with rho0
 * swapped on the planes z >= init_split when init_split > 0; fluid at rest)
 * and return a context.  dev_ws: device pointer, 256-byte aligned. */
int lbm_init(const lbm_params *p, int32_t n_replicas, int32_t precision, void *dev_ws,
             size_t ws_bytes, void *hip_stream, lbm_ctx **out);

/* Advance every replica by nsteps (asynchronous). */
int lbm_step(lbm_ctx *c, int32_t nsteps);

/* lbm_step for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation):
 * the same steps, bitwise, with the per-step scratch of the step kernels
 * (link and event partial sums, the sphere box's post-streaming moments and
 * step densities) taken from a static device array of the library
 * (16 MiB; each GPU the library runs on holds its own until the process
 * ends) instead of the context workspace.  Makes no allocation and no
 * library call that allocates.  Plain launches only (lbm_set_graph is not
 * used).  Every call on one GPU shares that GPU's array: calls whose steps
 * overlap on one GPU (two contexts on two streams) race and must be
 * serialised by the caller.  LBM_EINVAL for nsteps < 0 or a context whose
 * step scratch exceeds 16 MiB (56 bytes per sphere-box node, summed over
 * the replicas, plus 384 bytes per 64 box nodes, each rounded up to 256);
 * LBM_EDEVICE if the array's address cannot be obtained. */
int lbm_step_noalloc(lbm_ctx *c, int32_t nsteps);

/* Blocks until the context's stream has drained. */
int lbm_sync(lbm_ctx *c);

int lbm_particle_state(lbm_ctx *c, int32_t replica, lbm_particle *out);
/* Fills *o; o->uz_profile, when not NULL, receives nx * ny values (row-major
 * [y][x], a column with no fluid node gives 0).  Synchronises the context
 * stream.  LBM_EINVAL for a bad replica or NULL o; LBM_EUNSTABLE (after
 * filling *o) when the run went unstable. */
int lbm_observables(lbm_ctx *c, int32_t replica, lbm_obs *o);

/* f_{l i}(x, n) (after streaming and mass correction, particle nodes 0) of one
 * replica into host_f[2][19][nz][ny][nx]. */
int lbm_populations(lbm_ctx *c, int32_t replica, double *host_f);

/* rho_l and the hydrodynamic velocity v_H per node (particle nodes 0):
 * host_rho[2][nz][ny][nx], host_u[3][nz][ny][nx]. */
int lbm_fields(lbm_ctx *c, int32_t replica, double *host_rho, double *host_u);

/* The particle velocity time series the paper tracks (Fig. 1 caption) and
 * whose mean and variance it analyses (Sec. 4, eq. MEANVARIANCE and eq.
 * FLUCTUATIONSSCALING): U^{n+1/2} of each step, kept on the device in a ring
 * of series_cap entries that the step writes at slot n mod series_cap.
 * Copies the last min(steps, series_cap, cap) entries, oldest first, into
 * host_u3[k][3] (caller-owned, 3 cap doubles); *count = number written.
 * Synchronises the context stream.  LBM_EINVAL for a bad replica, NULL
 * outputs or cap < 0. */
int lbm_u_series(lbm_ctx *c, int32_t replica, double *host_u3, int64_t cap, int64_t *count);

/* Checkpoint: the complete state needed to resume bit-for-bit. */
int lbm_checkpoint_bytes(lbm_ctx *c, size_t *bytes);
int lbm_checkpoint(lbm_ctx *c, void *dev_dst);
int lbm_restore(lbm_ctx *c, const void *dev_src);

/* Launch shape of the main kernel: block threads (256, 512 or 1024; at least
 * the longest x-row) and z-chunk length (>= 1; 0 picks the default: the
 * longest power-of-two chunk up to 16 that keeps about four waves per SIMD
 * resident).  Rebuilds the tiling; results do not depend on the shape.
 * LBM_EINVAL for other blocks or a shape needing more than 64 KiB of LDS. */
int lbm_set_launch(lbm_ctx *c, int32_t block, int32_t zchunk);
int lbm_get_launch(lbm_ctx *c, int32_t *block, int32_t *zchunk);

/* Autotuner of the main-kernel launch shape.  Every block (256, 512, 1024;
 * at least the longest x-row) and z-chunk (2 ... 32) whose LDS fits is run
 * for one untimed step plus steps_per_trial steps timed with HIP events on
 * the context stream; the three fastest are timed once more, and the shape
 * with the shortest mean main-kernel time is kept.  The trial steps are real steps of the run (results do not depend on
 * the shape).  With dev_ckpt non-NULL (a device buffer of
 * lbm_checkpoint_bytes) the state is checkpointed first and restored after,
 * leaving the run where it was.  Outputs (may be NULL): chosen block and
 * z-chunk, its mean main-kernel time in ms.  Synchronises the stream. */
int lbm_autotune(lbm_ctx *c, int32_t steps_per_trial, void *dev_ckpt, int32_t *block_out,
                 int32_t *zchunk_out, double *best_ms);

/* 0: plain launches; k > 0: lbm_step replays a HIP graph of k steps (needs a
 * non-default stream); leftover steps run as plain launches, and so do all
 * steps while lbm_timing is on.  An even k replays one captured graph; an
 * odd k swaps the roles of the two population buffers at every replay, so
 * the graph is captured again each time.  Results equal plain launches. */
int lbm_set_graph(lbm_ctx *c, int32_t steps_per_graph);

/* Timing of the main kernel.  every = 0 turns it off; every = k >= 1 makes
 * every k-th plain-launch step from now on (the first, the (k+1)-th, ...)
 * record HIP events around its main-kernel launch on the context stream.  A sparse sample keeps
 * the events' own cost out of the other steps.  lbm_timing_read returns the
 * mean duration (ms) and the number of timed launches since it was enabled.
 * EINVAL for every < 0. */
int lbm_timing(lbm_ctx *c, int32_t every);
int lbm_timing_read(lbm_ctx *c, double *mean_ms, int64_t *count);

/* Algorithmic bytes one main-kernel launch moves per step: read + write of
 * 2 x 19 populations of the storage precision per node of every replica. */
int lbm_step_bytes(lbm_ctx *c, double *bytes);

/* Adjoint form (reverse-mode derivative through Sec. 2 eq. lbe, eq.
 * sc-force, the noise paragraph and the particle paragraph, and the external
 * force of Sec. 3 eq. fp).  Runs nsteps steps from the current state and
 * returns
 *   *J      = (1/nsteps) sum over those steps of U_z^{n+1/2} (time-averaged
 *             settling velocity, Sec. 4),
 *   grad[5] = dJ/d(g_x, g_y, g_z, G, Delta rho).
 * The noise normals of each (node, step) are held fixed (counter-based, so
 * the replay regenerates them); particle-node, link and cover/uncover sets
 * are held fixed (they change only at events, where J is not
 * differentiable); every value those sets carry is differentiated.
 * Schedule: forward sweep with a checkpoint every `segment` steps (0: 50)
 * and after the last step; the sweep records the last segment's per-node
 * densities and momenta (8 values per node and step) and sphere states.
 * Then, last segment first, each segment's steps are reversed, every other
 * segment being replayed from its checkpoint and recorded first.  With
 * segment >= nsteps the forward steps run once.
 * Arithmetic: FP64 for LBM_FP64 contexts, FP32 node adjoints otherwise; the
 * sphere and parameter adjoints are always FP64.
 * Requirements (else LBM_EINVAL): one replica, every relaxation time 1, a
 * sphere, and (FP64 contexts) nx <= 226: the node kernel stages a tile of
 * full x-rows over three planes in the 160 KiB of LDS a workgroup can hold.  dev_adj: caller-owned device buffer, 256-byte aligned, of at
 * least lbm_adjoint_bytes(c, nsteps, segment) bytes (LBM_ENOMEM otherwise);
 * the library keeps no reference to it after the call.  On success the
 * context holds the state after the nsteps steps, as lbm_step(c, nsteps)
 * leaves it; after LBM_EDEVICE it may hold any state the call passed
 * through (restore a checkpoint taken before the call).  LBM_EUNSTABLE if the run is or goes unstable.  Synchronises
 * the context stream.  While lbm_timing is enabled, the launches this call
 * times (lbm_timing_read) are those of the adjoint's node kernel, one per
 * reversed step; its forward sweep and replays run untimed. */
int lbm_adjoint_bytes(lbm_ctx *c, int32_t nsteps, int32_t segment, size_t *bytes);
int lbm_adjoint(lbm_ctx *c, int32_t nsteps, int32_t segment, void *dev_adj, size_t adj_bytes,
                double grad[5], double *J);

/* The two halves of lbm_adjoint, for a caller (an autograd function) that
 * needs J now and the gradient only later.
 * lbm_adjoint_forward: the forward sweep alone (the nsteps steps with the
 * checkpoints and the recorded last segment, about the cost of nsteps plain
 * steps); *J = the mean of U_z^{n+1/2} over those steps (from the running
 * sum the step keeps).  The context then holds the state after the steps and
 * a tape in dev_adj, which the caller keeps alive and untouched.
 * lbm_adjoint_backward: the reverse sweep over that tape; grad[5] as for
 * lbm_adjoint; the context is left where the forward sweep left it.  One
 * backward per forward; LBM_ESTATE when no tape is pending or the context
 * was stepped, restored or autotuned since the forward sweep.  Arguments,
 * requirements and errors of the forward sweep are those of lbm_adjoint. */
int lbm_adjoint_forward(lbm_ctx *c, int32_t nsteps, int32_t segment, void *dev_adj, size_t adj_bytes,
                        double *J);
int lbm_adjoint_backward(lbm_ctx *c, double grad[5]);

void lbm_destroy(lbm_ctx *c);
const char *lbm_last_error(const lbm_ctx *c);  /* NULL ctx: the calling thread's last error of a call with no context (lbm_init, lbm_workspace_bytes) */

#ifdef __cplusplus
}
#endif
#endif
