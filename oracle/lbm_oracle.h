/*
 * Plain FP64 CPU oracle of the fluctuating two-component D3Q19 lattice
 * Boltzmann step with one moving wettable sphere (Xue, Biferale, Sbragaglia,
 * Toschi, "A lattice Boltzmann study of particle settling in a fluctuating
 * multicomponent fluid under confinement", Section 2 "Methodology").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may include, link
 * or call this code: only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark use it.  It shares no header, table or helper with the HIP
 * library; its declarations here are its own.
 *
 * Every routine is a straightforward, sequential transcription of the method
 * (no blocking, no fusion); see lbm_oracle.c for the per-step citations.
 */
#ifndef LBM_ORACLE_H
#define LBM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAX_EXTRA 7  /* spheres beyond the first                        */

/* A further sphere in the same fluid (several particles, Sec. 5 follow-up) */
typedef struct orc_sphere {
    double radius, rho_p, wet_drho;
    double X0[3], U0[3], W0[3];
} orc_sphere;

typedef struct orc_params {
    int32_t nx, ny, nz;        /* lattice nodes per axis                              */
    uint32_t walls;            /* bit0: x walls, bit1: y walls, bit2: z walls          */
    double rho0[2];            /* reference densities of components A and B           */
    double init_amp;           /* uniform +/- amplitude of the initial densities      */
    double G;                  /* Shan-Chen coupling                                  */
    double tau_shear, tau_bulk, tau_mom, tau_ghost;
    double kT;                 /* thermal energy                                      */
    uint64_t seed;             /* Philox key = (lo32(seed), hi32(seed) ^ replica)     */
    int32_t replica;
    double g[3];               /* body-force acceleration                             */
    int32_t force_mode;        /* 0 balanced driving, 1 fluid rho*g / particle rho_p*V*g */
    double radius, rho_p, wet_drho;
    double X0[3], U0[3], W0[3];
    int32_t noise_diffusive;   /* 1: antisymmetric species-momentum noise              */
    int32_t fixed_velocity;    /* 1: sphere keeps U0, W0 (prescribed motion)          */
    int32_t init_split;        /* > 0: planes z >= init_split start from the swapped  */
                               /* densities (rho0[1], rho0[0]), the other phase       */
    int32_t n_extra;           /* further spheres (radius > 0 of the first required)  */
    orc_sphere extra[ORC_MAX_EXTRA];
} orc_params;

typedef struct orc_particle {
    double X[3], U[3], W[3];   /* X^n, U^{n-1/2}, Omega^{n-1/2}                        */
    double F[3], T[3];         /* total force / torque of the last step               */
    double Pev[3], Lev[3];     /* pending cover/uncover momentum and angular momentum */
    double delta[2];           /* last mass correction per component                  */
    double n_fluid;            /* |Phi^n|                                             */
    int64_t step;              /* n                                                   */
    int64_t n_covered, n_uncovered; /* cumulative event counts                        */
    int64_t n_links;           /* boundary links of the last step                     */
} orc_particle;

typedef struct orc_sim orc_sim;

orc_sim *orc_create(const orc_params *p);
void orc_destroy(orc_sim *s);
void orc_step(orc_sim *s, int32_t nsteps);
/* Threads of the per-node loops (n > 0 sets them; n <= 0 only queries);
 * returns the count in effect (1 without OpenMP).  Results do not depend
 * on it. */
int orc_set_threads(int32_t n);
/* f = [2][19][nz][ny][nx] populations f_{l i}(x, n) after streaming and mass
 * correction (solid nodes hold zero).                                        */
void orc_get_populations(const orc_sim *s, double *f);
void orc_set_populations(orc_sim *s, const double *f);
void orc_get_particle(const orc_sim *s, orc_particle *out);
void orc_set_particle(orc_sim *s, const orc_particle *in);
/* Sphere k (0 = the first) of several: state, and U^{n+1/2} series.  A node
 * inside several spheres belongs to the first of them.                      */
int32_t orc_n_spheres(const orc_sim *s);
void orc_get_sphere(const orc_sim *s, int32_t k, orc_particle *out);
void orc_set_sphere(orc_sim *s, int32_t k, const orc_particle *in);
int64_t orc_u_series_sphere(const orc_sim *s, int32_t k, double *u3, int64_t cap);
/* Per-node fields of the current state: rho[2][N], u[3][N] = v^(H) (solid: 0) */
void orc_get_fields(const orc_sim *s, double *rho, double *u);
/* Global observables: mass[2], fluid momentum[3] (sum of raw j over fluid nodes) */
void orc_observables(const orc_sim *s, double mass[2], double mom[3]);
/* U^{n+1/2}_z series of the run so far (length = steps taken; caller sizes it) */
int64_t orc_u_series(const orc_sim *s, double *u3, int64_t cap);

/* Adjoint of nsteps steps from the current state (every relaxation time 1,
 * one sphere, radius > 0): J = (1/nsteps) sum_n U_z^{n+1/2} and
 * grad = dJ/d(g_x, g_y, g_z, G, Delta rho).  Runs the steps forward (the
 * simulation ends after them, as orc_step would leave it).  Returns 0, -1 for
 * an unsupported configuration, -2 when memory runs out.                   */
int orc_adjoint(orc_sim *s, int32_t nsteps, double grad[5], double *J);

/* Building blocks exposed for the pins */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void orc_normals(const orc_sim *s, int64_t node, int64_t step, double z[36]);
void orc_basis(double e[19][19], double w[19], double b[19], int32_t c[19][3]);
/* collide one node (both components): fin[2][19] -> fout[2][19] given forces  */
void orc_collide_node(const orc_sim *s, const double fin[2][19], const double F[2][3],
                      const double noise[36], double fout[2][19]);
/* Shan-Chen + body force at every node of the current state: F[2][3][N]   */
void orc_forces(const orc_sim *s, double *F);

#ifdef __cplusplus
}
#endif
#endif
