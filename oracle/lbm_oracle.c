/*
 * Plain, sequential FP64 CPU oracle of the fluctuating two-component D3Q19
 * lattice Boltzmann step with one moving, wettable, finite-size sphere.
 *
 * TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the CPU
 * baseline of the benchmark.  The HIP product path never includes, links or
 * calls it, and it includes nothing of the product.
 *
 * Paper: Xue, Biferale, Sbragaglia, Toschi, "A lattice Boltzmann study of
 * particle settling in a fluctuating multicomponent fluid under confinement".
 *   Sec. 2, eq. (density)      moments rho_l, rho_tot v
 *   Sec. 2, eq. (lbe)          stream + collide + deterministic source + noise
 *   Sec. 2, MRT paragraph      modes relaxed separately; momentum-mode rate
 *                              sets D, stress-mode rate sets eta
 *   Sec. 2, eq. (sc-force)     Shan-Chen inter-component force
 *   Sec. 2, noise paragraph    no noise on mass, FDT noise on the other modes;
 *                              hydrodynamic velocity v + (F_A+F_B)/(2 rho_tot)
 *   Sec. 2, particle paragraph particle nodes, leap-frog Newton, moving
 *                              bounce-back with momentum exchange, cover /
 *                              uncover, global mass correction, virtual
 *                              wetting layer (+Delta rho)
 *   Sec. 3, eq. (fp)           external force on the particle
 *   Sec. 4, Langevin paragraph particle mass m_p = pi d^3 rho_p / 6
 * Where the paper is silent the readings listed in the design notes are
 * used (basis, forcing scheme, noise layout, generator, event rules).
 *
 * Every loop is written in the order of the method; nothing is fused or
 * blocked.  Compile with -ffp-contract=off: the particle-node predicate must
 * round identically on every implementation.
 *
 * Threads.  Built with OpenMP, the per-node loops run over z-planes in
 * parallel.  Every sum over nodes (the wetting-layer reaction, the link
 * momentum exchange, its torque and mass flux) is taken per z-plane in
 * (y, x, link) order and the plane sums are then added in z order, whatever
 * the thread count, so one thread and many give bitwise the same run.
 */
#include "lbm_oracle.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define Q 19

/* ---------------------------------------------------------------- lattice */
/* D3Q19: rest, 6 axis links (+,- pairs), 12 planar diagonals (opposite pairs) */
static const int CV[Q][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

static int opposite(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

static double weight(int i) {
    int c2 = CV[i][0] * CV[i][0] + CV[i][1] * CV[i][1] + CV[i][2] * CV[i][2];
    return c2 == 0 ? 1.0 / 3.0 : (c2 == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
}

/* Orthogonal mode polynomials e_k(c) (Duenweg-Schiller-Ladd set) */
static double mode_poly(int k, const int c[3]) {
    double x = c[0], y = c[1], z = c[2];
    double c2 = x * x + y * y + z * z;
    switch (k) {
    case 0: return 1.0;
    case 1: return x;
    case 2: return y;
    case 3: return z;
    case 4: return c2 - 1.0;
    case 5: return 3.0 * x * x - c2;
    case 6: return y * y - z * z;
    case 7: return x * y;
    case 8: return y * z;
    case 9: return x * z;
    case 10: return (3.0 * c2 - 5.0) * x;
    case 11: return (3.0 * c2 - 5.0) * y;
    case 12: return (3.0 * c2 - 5.0) * z;
    case 13: return (y * y - z * z) * x;
    case 14: return (z * z - x * x) * y;
    case 15: return (x * x - y * y) * z;
    case 16: return 3.0 * c2 * c2 - 6.0 * c2 + 1.0;
    case 17: return (2.0 * c2 - 3.0) * (3.0 * x * x - c2);
    case 18: return (2.0 * c2 - 3.0) * (y * y - z * z);
    }
    return 0.0;
}

/* ------------------------------------------------------------------ state */
struct orc_sim {
    orc_params p;
    int64_t N;
    double E[Q][Q];     /* E[k][i] = e_k(c_i)                */
    double W[Q];        /* lattice weights                   */
    double B[Q];        /* b_k = sum_i w_i e_k(c_i)^2         */
    double *f;          /* [2][Q][N] current populations     */
    double *fpost;      /* [2][Q][N] post-collision          */
    double *fnew;       /* [2][Q][N] after streaming         */
    double *rho;        /* [2][N]                            */
    double *jm;         /* [2][3][N]                         */
    double *rt;         /* [2][N] densities seen by SC force */
    double *F;          /* [2][3][N]                         */
    /* particle nodes at X^n / X^{n+1}: 0 fluid, k + 1 inside sphere k (the
     * first sphere that contains the node)                                  */
    unsigned char *solid;
    unsigned char *solid_new;
    int K;                              /* spheres (0: none)                  */
    double Rk[ORC_MAX_EXTRA + 1], rhopk[ORC_MAX_EXTRA + 1], drhok[ORC_MAX_EXTRA + 1];
    orc_particle P[ORC_MAX_EXTRA + 1];  /* sphere states (global fields alike) */
    double M_fluid0;
    double *series[ORC_MAX_EXTRA + 1];  /* U^{n+1/2} of each sphere, 3 per step */
    int64_t series_len, series_cap;
};

static int64_t node_index(const orc_sim *s, int x, int y, int z) {
    return (int64_t)x + (int64_t)s->p.nx * ((int64_t)y + (int64_t)s->p.ny * z);
}

/* Resolve a lattice position against walls / periodic axes.  Returns 0 when
 * the position lies in a wall layer (outside the box on a walled axis).   */
static int resolve(const orc_sim *s, int *x, int *y, int *z) {
    int n[3] = {s->p.nx, s->p.ny, s->p.nz};
    int *v[3] = {x, y, z};
    for (int a = 0; a < 3; a++) {
        if (*v[a] < 0 || *v[a] >= n[a]) {
            if (s->p.walls & (1u << a)) return 0;
            *v[a] = (*v[a] % n[a] + n[a]) % n[a];
        }
    }
    return 1;
}

/* Mirror of a wall-layer position onto the adjacent box node (clamp). */
static void mirror(const orc_sim *s, int *x, int *y, int *z) {
    int n[3] = {s->p.nx, s->p.ny, s->p.nz};
    int *v[3] = {x, y, z};
    for (int a = 0; a < 3; a++) {
        if (*v[a] < 0 || *v[a] >= n[a]) {
            if (s->p.walls & (1u << a)) *v[a] = *v[a] < 0 ? 0 : n[a] - 1;
            else *v[a] = (*v[a] % n[a] + n[a]) % n[a];
        }
    }
}

/* minimum-image separation along one axis */
static double sep(double d, int n, int periodic) {
    if (periodic) {
        if (d > 0.5 * n) d -= n;
        else if (d < -0.5 * n) d += n;
    }
    return d;
}

static void separation(const orc_sim *s, double px, double py, double pz,
                       const double X[3], double r[3]) {
    r[0] = sep(px - X[0], s->p.nx, !(s->p.walls & 1u));
    r[1] = sep(py - X[1], s->p.ny, !(s->p.walls & 2u));
    r[2] = sep(pz - X[2], s->p.nz, !(s->p.walls & 4u));
}

/* particle node predicate |x - X|^2 < R^2 (strict), FP64, no contraction */
static int particle_node(const orc_sim *s, int x, int y, int z, const double X[3]) {
    if (s->p.radius <= 0.0) return 0;
    double r[3];
    separation(s, (double)x, (double)y, (double)z, X, r);
    double d2 = r[0] * r[0] + r[1] * r[1];
    d2 = d2 + r[2] * r[2];
    return d2 < s->p.radius * s->p.radius;
}

/* the same predicate for sphere k */
static int sphere_node(const orc_sim *s, int k, int x, int y, int z, const double X[3]) {
    double r[3];
    separation(s, (double)x, (double)y, (double)z, X, r);
    double d2 = r[0] * r[0] + r[1] * r[1];
    d2 = d2 + r[2] * r[2];
    return d2 < s->Rk[k] * s->Rk[k];
}

/* 0 for a fluid node, else 1 + the first sphere (centres Xs[k]) containing it */
static unsigned char owner_of(const orc_sim *s, int x, int y, int z, const orc_particle *Ps) {
    for (int k = 0; k < s->K; k++)
        if (sphere_node(s, k, x, y, z, Ps[k].X)) return (unsigned char)(k + 1);
    return 0;
}

static double sphere_volume(const orc_sim *s, int k) {
    return 4.0 / 3.0 * M_PI * s->Rk[k] * s->Rk[k] * s->Rk[k];
}

static void cross(const double a[3], const double b[3], double c[3]) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

static double particle_volume(const orc_sim *s) {
    return 4.0 / 3.0 * M_PI * s->p.radius * s->p.radius * s->p.radius;
}

/* ------------------------------------------------------------ Philox4x32-10
 * Counter-based generator of Salmon, Moraes, Dror, Shaw (SC'11): ten rounds
 * of two 32x32->64 multiplications with a Weyl key schedule.               */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; round++) {
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void philox_key(const orc_sim *s, uint32_t key[2]) {
    key[0] = (uint32_t)(s->p.seed & 0xffffffffu);
    key[1] = (uint32_t)(s->p.seed >> 32) ^ (uint32_t)s->p.replica;
}

static double unit_open(uint32_t w) { return ((double)w + 0.5) * ldexp(1.0, -32); }

/* 36 standard normals for (node, step): 9 Philox blocks, Box-Muller pairs.
 * Block b gives normals 4b..4b+3.  Normals 16 l + (k - 4) drive mode k of
 * component l (k = 4..18); normals 32..34 the species-momentum noise.      */
void orc_normals(const orc_sim *s, int64_t node, int64_t step, double z[36]) {
    uint32_t key[2];
    philox_key(s, key);
    for (int b = 0; b < 9; b++) {
        uint32_t ctr[4] = {(uint32_t)node, (uint32_t)step, (uint32_t)b, 0u}, w[4];
        orc_philox4x32_10(ctr, key, w);
        for (int h = 0; h < 2; h++) {
            double u1 = unit_open(w[2 * h]), u2 = unit_open(w[2 * h + 1]);
            double r = sqrt(-2.0 * log(u1));
            double a = 2.0 * M_PI * u2;
            z[4 * b + 2 * h] = r * cos(a);
            z[4 * b + 2 * h + 1] = r * sin(a);
        }
    }
}

void orc_basis(double e[19][19], double w[19], double b[19], int32_t c[19][3]) {
    for (int i = 0; i < Q; i++) {
        w[i] = weight(i);
        for (int a = 0; a < 3; a++) c[i][a] = CV[i][a];
    }
    for (int k = 0; k < Q; k++) {
        b[k] = 0.0;
        for (int i = 0; i < Q; i++) {
            e[k][i] = mode_poly(k, CV[i]);
            b[k] += w[i] * e[k][i] * e[k][i];
        }
    }
}

/* ----------------------------------------------------------- construction */
orc_sim *orc_create(const orc_params *p) {
    orc_sim *s = (orc_sim *)calloc(1, sizeof(orc_sim));
    s->p = *p;
    s->N = (int64_t)p->nx * p->ny * p->nz;
    int32_t cdummy[19][3];
    orc_basis(s->E, s->W, s->B, cdummy);
    int64_t N = s->N;
    s->f = (double *)calloc((size_t)(2 * Q * N), sizeof(double));
    s->fpost = (double *)calloc((size_t)(2 * Q * N), sizeof(double));
    s->fnew = (double *)calloc((size_t)(2 * Q * N), sizeof(double));
    s->rho = (double *)calloc((size_t)(2 * N), sizeof(double));
    s->jm = (double *)calloc((size_t)(6 * N), sizeof(double));
    s->rt = (double *)calloc((size_t)(2 * N), sizeof(double));
    s->F = (double *)calloc((size_t)(6 * N), sizeof(double));
    s->solid = (unsigned char *)calloc((size_t)N, 1);
    s->solid_new = (unsigned char *)calloc((size_t)N, 1);
    s->K = p->radius > 0.0 ? 1 + (p->n_extra > 0 ? (p->n_extra < ORC_MAX_EXTRA ? p->n_extra : ORC_MAX_EXTRA) : 0) : 0;
    s->series_cap = 1024;
    for (int k = 0; k < s->K || k == 0; k++)
        s->series[k] = (double *)calloc((size_t)(3 * s->series_cap), sizeof(double));
    for (int k = 0; k < s->K; k++) {
        const orc_sphere e0 = {p->radius, p->rho_p, p->wet_drho, {p->X0[0], p->X0[1], p->X0[2]},
                               {p->U0[0], p->U0[1], p->U0[2]}, {p->W0[0], p->W0[1], p->W0[2]}};
        const orc_sphere *e = k == 0 ? &e0 : &p->extra[k - 1];
        s->Rk[k] = e->radius;
        s->rhopk[k] = e->rho_p;
        s->drhok[k] = e->wet_drho;
        for (int a = 0; a < 3; a++) {
            s->P[k].X[a] = e->X0[a];
            s->P[k].U[a] = e->U0[a];
            s->P[k].W[a] = e->W0[a];
        }
    }
    if (s->K == 0)
        for (int a = 0; a < 3; a++) {
            s->P[0].X[a] = p->X0[a];
            s->P[0].U[a] = p->U0[a];
            s->P[0].W[a] = p->W0[a];
        }
    /* initial particle nodes and densities rho_l0 + amp (2u - 1) (Philox tag 1) */
    uint32_t key[2];
    philox_key(s, key);
    s->M_fluid0 = 0.0;
    for (int z = 0; z < p->nz; z++)
        for (int y = 0; y < p->ny; y++)
            for (int x = 0; x < p->nx; x++) {
                int64_t n = node_index(s, x, y, z);
                s->solid[n] = owner_of(s, x, y, z, s->P);
                if (s->solid[n]) continue;
                uint32_t ctr[4] = {(uint32_t)n, 0u, 0u, 1u}, w[4];
                orc_philox4x32_10(ctr, key, w);
                /* a demixed start: the planes above the split hold the other phase */
                const int swap = p->init_split > 0 && z >= p->init_split;
                for (int l = 0; l < 2; l++) {
                    double base = swap ? p->rho0[1 - l] : p->rho0[l];
                    double r = base + p->init_amp * (2.0 * unit_open(w[l]) - 1.0);
                    for (int i = 0; i < Q; i++) s->f[((int64_t)l * Q + i) * N + n] = s->W[i] * r;
                    s->M_fluid0 += r;
                }
                s->P[0].n_fluid += 1.0;
            }
    for (int k = 1; k < s->K; k++) s->P[k].n_fluid = s->P[0].n_fluid;
    return s;
}

void orc_destroy(orc_sim *s) {
    if (!s) return;
    free(s->f); free(s->fpost); free(s->fnew); free(s->rho); free(s->jm);
    free(s->rt); free(s->F); free(s->solid); free(s->solid_new);
    for (int k = 0; k <= ORC_MAX_EXTRA; k++) free(s->series[k]);
    free(s);
}

#define FI(arr, l, i, n) (arr)[((int64_t)(l) * Q + (i)) * N + (n)]

/* ----------------------------------------------------- step 1: moments */
static void moments(orc_sim *s) {
    int64_t N = s->N;
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; n++)
        for (int l = 0; l < 2; l++) {
            double r = 0.0, j[3] = {0.0, 0.0, 0.0};
            if (!s->solid[n])
                for (int i = 0; i < Q; i++) {
                    double fi = FI(s->f, l, i, n);
                    r += fi;
                    for (int a = 0; a < 3; a++) j[a] += fi * CV[i][a];
                }
            s->rho[l * N + n] = r;
            for (int a = 0; a < 3; a++) s->jm[(l * 3 + a) * N + n] = j[a];
        }
}

/* ------------------------------------------ step 2: virtual wetting layer
 * Fluid nodes see their own density.  A particle node with at least one
 * fluid neighbour carries the mean density of its fluid neighbours plus
 * +Delta rho (component A) / -Delta rho (component B).                   */
static void virtual_densities(orc_sim *s) {
    int64_t N = s->N;
    const orc_params *p = &s->p;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < p->nz; z++)
        for (int y = 0; y < p->ny; y++)
            for (int x = 0; x < p->nx; x++) {
                int64_t n = node_index(s, x, y, z);
                if (!s->solid[n]) {
                    s->rt[n] = s->rho[n];
                    s->rt[N + n] = s->rho[N + n];
                    continue;
                }
                double sum[2] = {0.0, 0.0};
                int cnt = 0;
                for (int i = 1; i < Q; i++) {
                    int xn = x + CV[i][0], yn = y + CV[i][1], zn = z + CV[i][2];
                    if (!resolve(s, &xn, &yn, &zn)) continue;
                    int64_t m = node_index(s, xn, yn, zn);
                    if (s->solid[m]) continue;
                    sum[0] += s->rho[m];
                    sum[1] += s->rho[N + m];
                    cnt++;
                }
                if (cnt > 0) {
                    const double drho = s->drhok[s->solid[n] - 1];
                    s->rt[n] = sum[0] / cnt + drho;
                    s->rt[N + n] = sum[1] / cnt - drho;
                } else {
                    s->rt[n] = 0.0;
                    s->rt[N + n] = 0.0;
                }
            }
}

/* body-force acceleration of the fluid and external force on each sphere
 * (Fext[k][3]); with several spheres the fluid balances their sum        */
static void driving(const orc_sim *s, double af[3], double Fext[][3]) {
    const orc_params *p = &s->p;
    double rho_tot0 = p->rho0[0] + p->rho0[1];
    double tot[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < s->K; k++) {
        double V = sphere_volume(s, k);
        for (int a = 0; a < 3; a++) {
            Fext[k][a] = p->force_mode == 1 ? V * s->rhopk[k] * p->g[a] : V * (s->rhopk[k] - rho_tot0) * p->g[a];
            tot[a] += Fext[k][a];
        }
    }
    for (int a = 0; a < 3; a++) {
        if (p->force_mode == 1) af[a] = p->g[a];
        else af[a] = s->M_fluid0 > 0.0 ? -tot[a] / s->M_fluid0 : 0.0;
    }
}

/* --------------------------------------------------- step 3: forces
 * F_l(x) = -G rho_l(x) sum_i w_i rt_{l'}(x + c_i) c_i + rho_l(x) a_f.
 * Wall layers mirror the adjacent fluid node (neutral walls).  The share
 * of the force coming from particle nodes is returned for the reaction
 * on the particle (force Fv, torque Tv about X^n).                       */
static void forces_impl(const orc_sim *s, double *F, double Fv[][3], double Tv[][3]) {
    int64_t N = s->N;
    const orc_params *p = &s->p;
    const int K = s->K > 0 ? s->K : 1;
    double af[3], Fext[ORC_MAX_EXTRA + 1][3];
    driving(s, af, Fext);
    /* per-plane sums of the particle-node share: [nz][K][6] = Fv, Tv of each sphere */
    double *pv = (double *)calloc((size_t)p->nz * K * 6, sizeof(double));
#pragma omp parallel for schedule(static)
    for (int z = 0; z < p->nz; z++)
        for (int y = 0; y < p->ny; y++)
            for (int x = 0; x < p->nx; x++) {
                int64_t n = node_index(s, x, y, z);
                for (int l = 0; l < 2; l++)
                    for (int a = 0; a < 3; a++) F[(l * 3 + a) * N + n] = 0.0;
                if (s->solid[n]) continue;
                double sumo[2][3] = {{0, 0, 0}, {0, 0, 0}};
                for (int i = 1; i < Q; i++) {
                    int xn = x + CV[i][0], yn = y + CV[i][1], zn = z + CV[i][2];
                    int inside = resolve(s, &xn, &yn, &zn);
                    if (!inside) {
                        xn = x + CV[i][0]; yn = y + CV[i][1]; zn = z + CV[i][2];
                        mirror(s, &xn, &yn, &zn);
                    }
                    int64_t m = node_index(s, xn, yn, zn);
                    double link[2][3];
                    for (int l = 0; l < 2; l++) {
                        double other = s->rt[(1 - l) * N + m];
                        for (int a = 0; a < 3; a++) {
                            link[l][a] = -p->G * s->rho[l * N + n] * s->W[i] * other * CV[i][a];
                            sumo[l][a] += link[l][a];
                        }
                    }
                    if (inside && s->solid[m]) {
                        const int k = s->solid[m] - 1;
                        double *Fvz = pv + ((int64_t)z * K + k) * 6, *Tvz = Fvz + 3;
                        double fl[3], r[3], t[3];
                        for (int a = 0; a < 3; a++) fl[a] = link[0][a] + link[1][a];
                        separation(s, x + 0.5 * CV[i][0], y + 0.5 * CV[i][1], z + 0.5 * CV[i][2],
                                   s->P[k].X, r);
                        cross(r, fl, t);
                        for (int a = 0; a < 3; a++) { Fvz[a] += fl[a]; Tvz[a] += t[a]; }
                    }
                }
                for (int l = 0; l < 2; l++)
                    for (int a = 0; a < 3; a++)
                        F[(l * 3 + a) * N + n] = sumo[l][a] + s->rho[l * N + n] * af[a];
            }
    for (int k = 0; k < K; k++) {
        for (int a = 0; a < 3; a++) { Fv[k][a] = 0.0; Tv[k][a] = 0.0; }
        for (int z = 0; z < p->nz; z++) {
            const double *v = pv + ((int64_t)z * K + k) * 6;
            for (int a = 0; a < 3; a++) { Fv[k][a] += v[a]; Tv[k][a] += v[3 + a]; }
        }
    }
    free(pv);
}

void orc_forces(const orc_sim *s, double *F) {
    orc_sim *m = (orc_sim *)s; /* moments / virtual densities are scratch */
    moments(m);
    virtual_densities(m);
    double Fv[ORC_MAX_EXTRA + 1][3], Tv[ORC_MAX_EXTRA + 1][3];
    forces_impl(s, F, Fv, Tv);
}

/* ---------------------------------------------- steps 4-6: collision
 * Both components share the hydrodynamic velocity
 *   u = (j_A + j_B + (F_A + F_B)/2) / rho.
 * Per component the modes m_k = sum_i e_k(c_i) f_i relax separately;
 * stress modes get Guo forcing in mode space; non-conserved modes get
 * noise sqrt(mu rho_l b_k (1 - gamma_k^2)) r with mu = kT / c_s^2.       */
void orc_collide_node(const orc_sim *s, const double fin[2][19], const double F[2][3],
                      const double noise[36], double fout[2][19]) {
    const orc_params *p = &s->p;
    double gs = 1.0 - 1.0 / p->tau_shear, gb = 1.0 - 1.0 / p->tau_bulk;
    double gj = 1.0 - 1.0 / p->tau_mom, gg = 1.0 - 1.0 / p->tau_ghost;
    double mu = 3.0 * p->kT;
    double m[2][Q], rl[2], jl[2][3];
    for (int l = 0; l < 2; l++) {
        for (int k = 0; k < Q; k++) {
            m[l][k] = 0.0;
            for (int i = 0; i < Q; i++) m[l][k] += s->E[k][i] * fin[l][i];
        }
        rl[l] = m[l][0];
        for (int a = 0; a < 3; a++) jl[l][a] = m[l][1 + a];
    }
    double rho = rl[0] + rl[1];
    double u[3];
    for (int a = 0; a < 3; a++) u[a] = (jl[0][a] + jl[1][a] + 0.5 * (F[0][a] + F[1][a])) / rho;
    double ra = rl[0] > 0.0 ? rl[0] : 0.0, rb = rl[1] > 0.0 ? rl[1] : 0.0;
    double xid[3] = {0.0, 0.0, 0.0};
    if (mu > 0.0 && p->noise_diffusive && rho > 0.0) {
        double amp = sqrt(mu * s->B[1] * (1.0 - gj * gj) * ra * rb / rho);
        for (int a = 0; a < 3; a++) xid[a] = amp * noise[32 + a];
    }
    for (int l = 0; l < 2; l++) {
        double ms[Q];
        double r = rl[l], rp = r > 0.0 ? r : 0.0;
        const double *Fl = F[l];
        double sigma = l == 0 ? 1.0 : -1.0;
        ms[0] = r;
        for (int a = 0; a < 3; a++)
            ms[1 + a] = r * u[a] + gj * (jl[l][a] + 0.5 * Fl[a] - r * u[a]) + 0.5 * Fl[a] +
                        sigma * xid[a];
        double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
        double uF = u[0] * Fl[0] + u[1] * Fl[1] + u[2] * Fl[2];
        double meq[10], phi[10], gam[10];
        meq[4] = r * uu;
        meq[5] = r * (3.0 * u[0] * u[0] - uu);
        meq[6] = r * (u[1] * u[1] - u[2] * u[2]);
        meq[7] = r * u[0] * u[1];
        meq[8] = r * u[1] * u[2];
        meq[9] = r * u[0] * u[2];
        phi[4] = 2.0 * uF;
        phi[5] = 2.0 * (3.0 * u[0] * Fl[0] - uF);
        phi[6] = 2.0 * (u[1] * Fl[1] - u[2] * Fl[2]);
        phi[7] = u[0] * Fl[1] + u[1] * Fl[0];
        phi[8] = u[1] * Fl[2] + u[2] * Fl[1];
        phi[9] = u[0] * Fl[2] + u[2] * Fl[0];
        gam[4] = gb;
        for (int k = 5; k <= 9; k++) gam[k] = gs;
        for (int k = 4; k <= 9; k++) {
            ms[k] = meq[k] + gam[k] * (m[l][k] - meq[k]) + 0.5 * (1.0 + gam[k]) * phi[k];
            if (mu > 0.0) ms[k] += sqrt(mu * rp * s->B[k] * (1.0 - gam[k] * gam[k])) * noise[16 * l + k - 4];
        }
        for (int k = 10; k < Q; k++) {
            ms[k] = gg * m[l][k];
            if (mu > 0.0) ms[k] += sqrt(mu * rp * s->B[k] * (1.0 - gg * gg)) * noise[16 * l + k - 4];
        }
        for (int i = 0; i < Q; i++) {
            double acc = 0.0;
            for (int k = 0; k < Q; k++) acc += s->E[k][i] * ms[k] / s->B[k];
            fout[l][i] = s->W[i] * acc;
        }
    }
}

static void collide(orc_sim *s) {
    int64_t N = s->N;
    double zero[36];
    memset(zero, 0, sizeof(zero));
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; n++) {
        if (s->solid[n]) {
            for (int l = 0; l < 2; l++)
                for (int i = 0; i < Q; i++) FI(s->fpost, l, i, n) = 0.0;
            continue;
        }
        double fin[2][Q], fout[2][Q], F[2][3], z[36];
        for (int l = 0; l < 2; l++) {
            for (int i = 0; i < Q; i++) fin[l][i] = FI(s->f, l, i, n);
            for (int a = 0; a < 3; a++) F[l][a] = s->F[(l * 3 + a) * N + n];
        }
        if (s->p.kT > 0.0) orc_normals(s, n, s->P[0].step, z);
        else memcpy(z, zero, sizeof(z));
        orc_collide_node(s, fin, F, z, fout);
        for (int l = 0; l < 2; l++)
            for (int i = 0; i < Q; i++) FI(s->fpost, l, i, n) = fout[l][i];
    }
}

static void series_push(orc_sim *s) {
    if (s->series_len == s->series_cap) {
        s->series_cap *= 2;
        for (int k = 0; k < s->K || k == 0; k++)
            s->series[k] = (double *)realloc(s->series[k], (size_t)(3 * s->series_cap) * sizeof(double));
    }
    for (int k = 0; k < s->K || k == 0; k++)
        for (int a = 0; a < 3; a++) s->series[k][3 * s->series_len + a] = s->P[k].U[a];
    s->series_len++;
}

/* ------------------------------------------------------------ step 7
 * Streaming of fpost into fnew with half-way bounce-back on walls and
 * moving-wall bounce-back on particle nodes (momentum exchange per link:
 * dp[k], torque dl[k] about X_k^n of the sphere k that owns the particle
 * node, bounce-back mass flux dMbb).  links[k]: boundary links of sphere k. */
static void stream_bounce(orc_sim *s, double dp[][3], double dl[][3], double dMbb[2], int64_t *links) {
    int64_t N = s->N;
    const orc_params *p = &s->p;
    const int K = s->K > 0 ? s->K : 1;
    const int NV = 7 * K + 2;  /* per plane: dp, dl, links of each sphere; dMbb */
    memset(s->fnew, 0, (size_t)(2 * Q * N) * sizeof(double));
    /* per-plane sums; every destination slot has exactly one writer, so
     * planes stream independently */
    double *pv = (double *)calloc((size_t)p->nz * NV, sizeof(double));
#pragma omp parallel for schedule(static)
    for (int z = 0; z < p->nz; z++)
        for (int y = 0; y < p->ny; y++)
            for (int x = 0; x < p->nx; x++) {
                double *vz = pv + (int64_t)z * NV, *dMz = vz + 7 * K;
                int64_t n = node_index(s, x, y, z);
                if (s->solid[n]) continue;
                for (int l = 0; l < 2; l++) FI(s->fnew, l, 0, n) = FI(s->fpost, l, 0, n);
                for (int i = 1; i < Q; i++) {
                    int xn = x + CV[i][0], yn = y + CV[i][1], zn = z + CV[i][2];
                    int io = opposite(i);
                    if (!resolve(s, &xn, &yn, &zn)) {
                        for (int l = 0; l < 2; l++) FI(s->fnew, l, io, n) = FI(s->fpost, l, i, n);
                        continue;
                    }
                    int64_t m = node_index(s, xn, yn, zn);
                    if (s->solid[m]) {
                        const int k = s->solid[m] - 1;
                        const orc_particle *P = &s->P[k];
                        double *dpz = vz + 7 * k, *dlz = dpz + 3;
                        double r[3], w[3], ub[3];
                        separation(s, x + 0.5 * CV[i][0], y + 0.5 * CV[i][1], z + 0.5 * CV[i][2],
                                   P->X, r);
                        cross(P->W, r, w);
                        for (int a = 0; a < 3; a++) ub[a] = P->U[a] + w[a];
                        double cu = CV[i][0] * ub[0] + CV[i][1] * ub[1] + CV[i][2] * ub[2];
                        double lp[3] = {0, 0, 0};
                        for (int l = 0; l < 2; l++) {
                            double corr = 6.0 * s->W[i] * s->rho[l * N + n] * cu;
                            double fs = FI(s->fpost, l, i, n);
                            FI(s->fnew, l, io, n) = fs - corr;
                            for (int a = 0; a < 3; a++) lp[a] += (2.0 * fs - corr) * CV[i][a];
                            dMz[l] -= corr;
                        }
                        double t[3];
                        cross(r, lp, t);
                        for (int a = 0; a < 3; a++) { dpz[a] += lp[a]; dlz[a] += t[a]; }
                        dpz[6] += 1.0;
                        continue;
                    }
                    for (int l = 0; l < 2; l++) FI(s->fnew, l, i, m) = FI(s->fpost, l, i, n);
                }
            }
    dMbb[0] = dMbb[1] = 0.0;
    for (int k = 0; k < K; k++) {
        for (int a = 0; a < 3; a++) { dp[k][a] = 0.0; dl[k][a] = 0.0; }
        links[k] = 0;
    }
    for (int z = 0; z < p->nz; z++) {
        const double *v = pv + (int64_t)z * NV;
        for (int k = 0; k < K; k++) {
            for (int a = 0; a < 3; a++) { dp[k][a] += v[7 * k + a]; dl[k][a] += v[7 * k + 3 + a]; }
            links[k] += (int64_t)v[7 * k + 6];
        }
        dMbb[0] += v[7 * K];
        dMbb[1] += v[7 * K + 1];
    }
    free(pv);
}

/* ------------------------------------------------------------ one step */
static void one_step(orc_sim *s) {
    int64_t N = s->N;
    const orc_params *p = &s->p;
    const int K = s->K;

    moments(s);                 /* 1 */
    virtual_densities(s);       /* 2 */
    double Fv[ORC_MAX_EXTRA + 1][3], Tv[ORC_MAX_EXTRA + 1][3];
    forces_impl(s, s->F, Fv, Tv); /* 3 */
    collide(s);                 /* 4-6 */

    /* 7: streaming with half-way bounce-back on walls and moving-wall
     * bounce-back on particle nodes (momentum exchange on each link)     */
    double dp[ORC_MAX_EXTRA + 1][3], dl[ORC_MAX_EXTRA + 1][3], dMbb[2];
    int64_t links[ORC_MAX_EXTRA + 1];
    stream_bounce(s, dp, dl, dMbb, links);

    /* 8: leap-frog Newton-Euler update of each sphere */
    double af[3], Fext[ORC_MAX_EXTRA + 1][3];
    driving(s, af, Fext);
    int n3[3] = {p->nx, p->ny, p->nz};
    for (int k = 0; k < K; k++) {
        orc_particle *P = &s->P[k];
        double mp = s->rhopk[k] * sphere_volume(s, k);
        double Ip = 0.4 * mp * s->Rk[k] * s->Rk[k];
        for (int a = 0; a < 3; a++) {
            P->F[a] = dp[k][a] - Fv[k][a] + Fext[k][a] + P->Pev[a];
            P->T[a] = dl[k][a] - Tv[k][a] + P->Lev[a];
            if (!p->fixed_velocity) {
                P->U[a] += P->F[a] / mp;
                P->W[a] += P->T[a] / Ip;
            }
        }
        for (int a = 0; a < 3; a++) {
            P->X[a] += P->U[a];
            if (!(p->walls & (1u << a))) {
                if (P->X[a] >= n3[a]) P->X[a] -= n3[a];
                else if (P->X[a] < 0.0) P->X[a] += n3[a];
            }
            P->Pev[a] = 0.0;
            P->Lev[a] = 0.0;
        }
        P->n_links = links[k];
    }
    if (K == 0) s->P[0].n_links = 0;
    series_push(s);

    /* 9: cover / uncover against the particle nodes at X^{n+1}; a covered
     * node's momentum goes to the sphere that now holds it, an uncovered
     * node takes the rigid velocity of the sphere that held it           */
    double dMcov[2] = {0, 0}, dMunc[2] = {0, 0};
#pragma omp parallel for schedule(static)
    for (int z = 0; z < p->nz; z++)
        for (int y = 0; y < p->ny; y++)
            for (int x = 0; x < p->nx; x++) {
                int64_t n = node_index(s, x, y, z);
                s->solid_new[n] = owner_of(s, x, y, z, s->P);
            }
    for (int z = 0; z < p->nz; z++)
        for (int y = 0; y < p->ny; y++)
            for (int x = 0; x < p->nx; x++) {
                int64_t n = node_index(s, x, y, z);
                if (!s->solid[n] && s->solid_new[n]) { /* covered */
                    orc_particle *P = &s->P[s->solid_new[n] - 1];
                    double j[3] = {0, 0, 0}, r[3], t[3];
                    for (int l = 0; l < 2; l++) {
                        double rl = 0.0;
                        for (int i = 0; i < Q; i++) {
                            double fi = FI(s->fnew, l, i, n);
                            rl += fi;
                            for (int a = 0; a < 3; a++) j[a] += fi * CV[i][a];
                        }
                        dMcov[l] -= rl;
                    }
                    separation(s, x, y, z, P->X, r);
                    cross(r, j, t);
                    for (int a = 0; a < 3; a++) { P->Pev[a] += j[a]; P->Lev[a] += t[a]; }
                    P->n_covered++;
                }
            }
    for (int z = 0; z < p->nz; z++)
        for (int y = 0; y < p->ny; y++)
            for (int x = 0; x < p->nx; x++) {
                int64_t n = node_index(s, x, y, z);
                if (!(s->solid[n] && !s->solid_new[n])) continue; /* uncovered only */
                orc_particle *P = &s->P[s->solid[n] - 1];
                double rb[2] = {0, 0};
                int cnt = 0;
                for (int i = 1; i < Q; i++) {
                    int xn = x + CV[i][0], yn = y + CV[i][1], zn = z + CV[i][2];
                    if (!resolve(s, &xn, &yn, &zn)) continue;
                    int64_t m = node_index(s, xn, yn, zn);
                    if (s->solid[m] || s->solid_new[m]) continue;
                    for (int l = 0; l < 2; l++)
                        for (int k = 0; k < Q; k++) rb[l] += FI(s->fnew, l, k, m);
                    cnt++;
                }
                for (int l = 0; l < 2; l++) rb[l] = cnt > 0 ? rb[l] / cnt : p->rho0[l];
                double r[3], w[3], u[3];
                separation(s, x, y, z, P->X, r);
                cross(P->W, r, w);
                for (int a = 0; a < 3; a++) u[a] = P->U[a] + w[a];
                double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
                for (int l = 0; l < 2; l++) {
                    for (int i = 0; i < Q; i++) {
                        double cu = CV[i][0] * u[0] + CV[i][1] * u[1] + CV[i][2] * u[2];
                        FI(s->fnew, l, i, n) = s->W[i] * rb[l] * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
                    }
                    dMunc[l] += rb[l];
                }
                double mom[3], t[3];
                for (int a = 0; a < 3; a++) mom[a] = (rb[0] + rb[1]) * u[a];
                cross(r, mom, t);
                for (int a = 0; a < 3; a++) { P->Pev[a] -= mom[a]; P->Lev[a] -= t[a]; }
                P->n_uncovered++;
            }
    /* covered nodes drop their populations */
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; n++)
        if (s->solid_new[n])
            for (int l = 0; l < 2; l++)
                for (int i = 0; i < Q; i++) FI(s->fnew, l, i, n) = 0.0;

    /* 10: global mass correction over Phi^{n+1} */
    double nf = 0.0;
    for (int64_t n = 0; n < N; n++) nf += s->solid_new[n] ? 0.0 : 1.0;
    double delta[2];
    for (int l = 0; l < 2; l++) delta[l] = -(dMbb[l] + dMcov[l] + dMunc[l]) / nf;
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; n++) {
        if (s->solid_new[n]) continue;
        for (int l = 0; l < 2; l++)
            for (int i = 0; i < Q; i++) FI(s->fnew, l, i, n) += s->W[i] * delta[l];
    }
    for (int k = 0; k < K || k == 0; k++) {
        s->P[k].delta[0] = delta[0];
        s->P[k].delta[1] = delta[1];
        s->P[k].n_fluid = nf;
        s->P[k].step++;
    }

    double *t = s->f; s->f = s->fnew; s->fnew = t;
    unsigned char *u8 = s->solid; s->solid = s->solid_new; s->solid_new = u8;
}

int orc_set_threads(int32_t n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

void orc_step(orc_sim *s, int32_t nsteps) {
    for (int32_t k = 0; k < nsteps; k++) one_step(s);
}

void orc_get_populations(const orc_sim *s, double *f) {
    memcpy(f, s->f, (size_t)(2 * Q * s->N) * sizeof(double));
}

void orc_set_populations(orc_sim *s, const double *f) {
    memcpy(s->f, f, (size_t)(2 * Q * s->N) * sizeof(double));
}

void orc_get_particle(const orc_sim *s, orc_particle *out) { *out = s->P[0]; }

static void reset_solid(orc_sim *s) {
    const orc_params *p = &s->p;
    for (int z = 0; z < p->nz; z++)
        for (int y = 0; y < p->ny; y++)
            for (int x = 0; x < p->nx; x++)
                s->solid[node_index(s, x, y, z)] = owner_of(s, x, y, z, s->P);
}

void orc_set_particle(orc_sim *s, const orc_particle *in) {
    s->P[0] = *in;
    reset_solid(s);
}

int32_t orc_n_spheres(const orc_sim *s) { return s->K; }

void orc_get_sphere(const orc_sim *s, int32_t k, orc_particle *out) {
    *out = s->P[k >= 0 && k < s->K ? k : 0];
}

void orc_set_sphere(orc_sim *s, int32_t k, const orc_particle *in) {
    if (k < 0 || k >= s->K) return;
    s->P[k] = *in;
    reset_solid(s);
}

void orc_get_fields(const orc_sim *s, double *rho, double *u) {
    orc_sim *m = (orc_sim *)s;
    int64_t N = s->N;
    double *F = (double *)malloc((size_t)(6 * N) * sizeof(double));
    orc_forces(s, F);
    for (int64_t n = 0; n < N; n++) {
        double rt = s->rho[n] + s->rho[N + n];
        rho[n] = s->rho[n];
        rho[N + n] = s->rho[N + n];
        for (int a = 0; a < 3; a++) {
            if (m->solid[n] || rt == 0.0) { u[a * N + n] = 0.0; continue; }
            u[a * N + n] = (s->jm[a * N + n] + s->jm[(3 + a) * N + n] +
                            0.5 * (F[a * N + n] + F[(3 + a) * N + n])) / rt;
        }
    }
    free(F);
}

void orc_observables(const orc_sim *s, double mass[2], double mom[3]) {
    int64_t N = s->N;
    mass[0] = mass[1] = 0.0;
    mom[0] = mom[1] = mom[2] = 0.0;
    for (int64_t n = 0; n < N; n++) {
        if (s->solid[n]) continue;
        for (int l = 0; l < 2; l++)
            for (int i = 0; i < Q; i++) {
                double fi = FI(s->f, l, i, n);
                mass[l] += fi;
                for (int a = 0; a < 3; a++) mom[a] += fi * CV[i][a];
            }
    }
}

int64_t orc_u_series(const orc_sim *s, double *u3, int64_t cap) {
    return orc_u_series_sphere(s, 0, u3, cap);
}

int64_t orc_u_series_sphere(const orc_sim *s, int32_t k, double *u3, int64_t cap) {
    if (k < 0 || (k >= s->K && k > 0)) return 0;
    int64_t n = s->series_len < cap ? s->series_len : cap;
    memcpy(u3, s->series[k], (size_t)(3 * n) * sizeof(double));
    return s->series_len;
}

/* ===================================================================
 * Adjoint (reverse-mode derivative) of nsteps steps.
 *
 * Objective: J = (1/nsteps) sum_{n} U_z^{n+1/2}, the time-averaged settling
 * velocity over the steps of this call.  Parameters: the body-force vector
 * g (three components), the Shan-Chen coupling G and the wetting offset
 * Delta rho; grad = dJ/d(g_x, g_y, g_z, G, Delta rho).
 *
 * Readings.  Every relaxation time is 1.  The noise normals depend on
 * (node, step) only and are held fixed; their amplitudes sqrt(mu rho_l b_k)
 * are differentiated.  The particle-node, link and cover/uncover sets are
 * piecewise constant in the particle position and are held fixed (their
 * derivative vanishes between events); the values those sets carry
 * (moving-wall terms, event momenta, equilibria of uncovered nodes, mass
 * fluxes, lever arms) are differentiated.
 *
 * Plain form: every forward state is stored, each step is replayed, and
 * its operations (steps 1-10 of one_step) are differentiated one by one in
 * reverse order on full population arrays.  Parity unpinned beyond what
 * the tests check: central differences of the forward step and the
 * linear-response limit dJ/dg_z -> J/g_z.
 * =================================================================== */

typedef struct {
    double *fb;        /* [2][Q][N] adjoint of the state f^{n+1} (then of f^n)   */
    double *fnewb;     /* [2][Q][N] adjoint of fnew after streaming              */
    double *fpostb;    /* [2][Q][N] adjoint of fpost                             */
    double *rhob;      /* [2][N]    adjoint of the moments rho_l                 */
    double *rtb;       /* [2][N]    adjoint of the densities seen by the force   */
    double *Fb;        /* [2][3][N] adjoint of the node forces                   */
} adj_arrays;

static void add_cross(double out[3], const double a[3], const double b[3], double sgn) {
    double c[3];
    cross(a, b, c);
    for (int a_ = 0; a_ < 3; a_++) out[a_] += sgn * c[a_];
}

/* Adjoint of the collision of one node (all relaxation times 1):
 * fpostb[2][Q] -> adjoint of the node's populations finb[2][Q] and of its
 * forces Fbn[2][3].                                                        */
static void collide_node_adjoint(const orc_sim *s, const double fin[2][Q], const double F[2][3],
                                 const double z[36], const double fpostb[2][Q],
                                 double finb[2][Q], double Fbn[2][3]) {
    const orc_params *p = &s->p;
    double mu = 3.0 * p->kT;
    double rl[2], jl[2][3];
    for (int l = 0; l < 2; l++) {
        rl[l] = 0.0;
        for (int a = 0; a < 3; a++) jl[l][a] = 0.0;
        for (int i = 0; i < Q; i++) {
            rl[l] += s->E[0][i] * fin[l][i];
            for (int a = 0; a < 3; a++) jl[l][a] += s->E[1 + a][i] * fin[l][i];
        }
    }
    double rho = rl[0] + rl[1];
    double u[3];
    for (int a = 0; a < 3; a++) u[a] = (jl[0][a] + jl[1][a] + 0.5 * (F[0][a] + F[1][a])) / rho;
    double ra = rl[0] > 0.0 ? rl[0] : 0.0, rb = rl[1] > 0.0 ? rl[1] : 0.0;
    double amp = 0.0;
    if (mu > 0.0 && p->noise_diffusive && rho > 0.0) amp = sqrt(mu * s->B[1] * ra * rb / rho);

    double rlb[2] = {0.0, 0.0}, jlb[2][3] = {{0, 0, 0}, {0, 0, 0}};
    double ub[3] = {0, 0, 0}, xidb[3] = {0, 0, 0};
    for (int l = 0; l < 2; l++) for (int a = 0; a < 3; a++) Fbn[l][a] = 0.0;

    for (int l = 0; l < 2; l++) {
        /* fout_i = w_i sum_k e_k(c_i) ms_k / b_k */
        double msb[Q];
        for (int k = 0; k < Q; k++) {
            msb[k] = 0.0;
            for (int i = 0; i < Q; i++) msb[k] += fpostb[l][i] * s->W[i] * s->E[k][i] / s->B[k];
        }
        double r = rl[l], sigma = l == 0 ? 1.0 : -1.0;
        const double *Fl = F[l];
        /* ms_0 = r */
        rlb[l] += msb[0];
        /* ms_{1+a} = r u_a + F_a / 2 + sigma xid_a */
        for (int a = 0; a < 3; a++) {
            rlb[l] += msb[1 + a] * u[a];
            ub[a] += msb[1 + a] * r;
            Fbn[l][a] += 0.5 * msb[1 + a];
            xidb[a] += sigma * msb[1 + a];
        }
        /* m_eq: 4 r u.u, 5 r(3ux^2 - u.u), 6 r(uy^2 - uz^2), 7 r ux uy, 8 r uy uz, 9 r ux uz */
        double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
        rlb[l] += msb[4] * uu;
        for (int a = 0; a < 3; a++) ub[a] += msb[4] * r * 2.0 * u[a];
        rlb[l] += msb[5] * (3.0 * u[0] * u[0] - uu);
        ub[0] += msb[5] * r * (6.0 * u[0] - 2.0 * u[0]);
        ub[1] += msb[5] * r * (-2.0 * u[1]);
        ub[2] += msb[5] * r * (-2.0 * u[2]);
        rlb[l] += msb[6] * (u[1] * u[1] - u[2] * u[2]);
        ub[1] += msb[6] * r * 2.0 * u[1];
        ub[2] += msb[6] * r * (-2.0 * u[2]);
        rlb[l] += msb[7] * u[0] * u[1];
        ub[0] += msb[7] * r * u[1];
        ub[1] += msb[7] * r * u[0];
        rlb[l] += msb[8] * u[1] * u[2];
        ub[1] += msb[8] * r * u[2];
        ub[2] += msb[8] * r * u[1];
        rlb[l] += msb[9] * u[0] * u[2];
        ub[0] += msb[9] * r * u[2];
        ub[2] += msb[9] * r * u[0];
        /* Guo terms Phi_k / 2: 4 u.F, 5 3uxFx - u.F, 6 uyFy - uzFz,
         * 7 (uxFy + uyFx)/2, 8 (uyFz + uzFy)/2, 9 (uxFz + uzFx)/2 */
        for (int a = 0; a < 3; a++) {
            ub[a] += msb[4] * Fl[a];
            Fbn[l][a] += msb[4] * u[a];
            ub[a] -= msb[5] * Fl[a];
            Fbn[l][a] -= msb[5] * u[a];
        }
        ub[0] += msb[5] * 3.0 * Fl[0];
        Fbn[l][0] += msb[5] * 3.0 * u[0];
        ub[1] += msb[6] * Fl[1];
        Fbn[l][1] += msb[6] * u[1];
        ub[2] -= msb[6] * Fl[2];
        Fbn[l][2] -= msb[6] * u[2];
        ub[0] += 0.5 * msb[7] * Fl[1]; ub[1] += 0.5 * msb[7] * Fl[0];
        Fbn[l][1] += 0.5 * msb[7] * u[0]; Fbn[l][0] += 0.5 * msb[7] * u[1];
        ub[1] += 0.5 * msb[8] * Fl[2]; ub[2] += 0.5 * msb[8] * Fl[1];
        Fbn[l][2] += 0.5 * msb[8] * u[1]; Fbn[l][1] += 0.5 * msb[8] * u[2];
        ub[0] += 0.5 * msb[9] * Fl[2]; ub[2] += 0.5 * msb[9] * Fl[0];
        Fbn[l][2] += 0.5 * msb[9] * u[0]; Fbn[l][0] += 0.5 * msb[9] * u[2];
        /* noise sqrt(mu r b_k) z on modes 4..18: d/dr = sqrt(mu b_k) z / (2 sqrt(r)) */
        if (mu > 0.0 && r > 0.0)
            for (int k = 4; k < Q; k++)
                rlb[l] += msb[k] * sqrt(mu * s->B[k]) * z[16 * l + k - 4] / (2.0 * sqrt(r));
    }
    /* species-momentum noise xid = amp z_{32+a}, amp^2 = mu b_1 ra rb / rho */
    if (amp > 0.0) {
        double ampb = 0.0;
        for (int a = 0; a < 3; a++) ampb += xidb[a] * z[32 + a];
        double K0 = mu * s->B[1];
        double dKa = K0 * (rb / rho - ra * rb / (rho * rho));
        double dKb = K0 * (ra / rho - ra * rb / (rho * rho));
        rlb[0] += ampb * dKa / (2.0 * amp);
        rlb[1] += ampb * dKb / (2.0 * amp);
    }
    /* u = (j_A + j_B + (F_A + F_B)/2) / rho */
    double ubu = ub[0] * u[0] + ub[1] * u[1] + ub[2] * u[2];
    for (int l = 0; l < 2; l++) {
        for (int a = 0; a < 3; a++) {
            jlb[l][a] += ub[a] / rho;
            Fbn[l][a] += 0.5 * ub[a] / rho;
        }
        rlb[l] -= ubu / rho;
    }
    /* moments rho_l = sum_i e_0 f_i, j_l = sum_i e_{1..3} f_i */
    for (int l = 0; l < 2; l++)
        for (int i = 0; i < Q; i++) {
            double v = s->E[0][i] * rlb[l];
            for (int a = 0; a < 3; a++) v += s->E[1 + a][i] * jlb[l][a];
            finb[l][i] = v;
        }
}

static void load_snapshot(orc_sim *s, const double *f, const orc_particle *P) {
    memcpy(s->f, f, (size_t)(2 * Q * s->N) * sizeof(double));
    orc_set_particle(s, P);
}

int orc_adjoint(orc_sim *s, int32_t nsteps, double grad[5], double *J) {
    const orc_params *p = &s->p;
    if (nsteps < 1 || p->radius <= 0.0 || s->K != 1 || p->tau_shear != 1.0 || p->tau_bulk != 1.0 ||
        p->tau_mom != 1.0 || p->tau_ghost != 1.0)
        return -1;
    int64_t N = s->N;
    size_t popn = (size_t)(2 * Q * N);
    double *snapf = (double *)malloc((size_t)(nsteps + 1) * popn * sizeof(double));
    orc_particle *snapP = (orc_particle *)malloc((size_t)(nsteps + 1) * sizeof(orc_particle));
    adj_arrays A;
    A.fb = (double *)calloc(popn, sizeof(double));
    A.fnewb = (double *)calloc(popn, sizeof(double));
    A.fpostb = (double *)calloc(popn, sizeof(double));
    A.rhob = (double *)calloc((size_t)(2 * N), sizeof(double));
    A.rtb = (double *)calloc((size_t)(2 * N), sizeof(double));
    A.Fb = (double *)calloc((size_t)(6 * N), sizeof(double));
    unsigned char *solid_next = (unsigned char *)calloc((size_t)N, 1);
    if (!snapf || !snapP || !A.fb || !A.fnewb || !A.fpostb || !A.rhob || !A.rtb || !A.Fb ||
        !solid_next) {
        free(snapf); free(snapP); free(A.fb); free(A.fnewb); free(A.fpostb); free(A.rhob);
        free(A.rtb); free(A.Fb); free(solid_next);
        return -2;
    }

    /* forward sweep, storing every state */
    double Jsum = 0.0;
    for (int32_t k = 0; k < nsteps; k++) {
        memcpy(snapf + (size_t)k * popn, s->f, popn * sizeof(double));
        snapP[k] = s->P[0];
        one_step(s);
        Jsum += s->P[0].U[2];
    }
    memcpy(snapf + (size_t)nsteps * popn, s->f, popn * sizeof(double));
    snapP[nsteps] = s->P[0];
    *J = Jsum / nsteps;

    double mp = p->rho_p * particle_volume(s);
    double Ip = 0.4 * mp * p->radius * p->radius;
    double Vp = particle_volume(s);
    double rho_tot0 = p->rho0[0] + p->rho0[1];
    /* d Fext / d g and d a_f / d g (both proportional to g) */
    double cF = p->force_mode == 1 ? Vp * p->rho_p : Vp * (p->rho_p - rho_tot0);
    double caf = p->force_mode == 1 ? 1.0 : (s->M_fluid0 > 0.0 ? -cF / s->M_fluid0 : 0.0);

    double Ub[3] = {0, 0, 0}, Wb[3] = {0, 0, 0}, Xb[3] = {0, 0, 0};
    double Pevb[3] = {0, 0, 0}, Levb[3] = {0, 0, 0};
    double gb[3] = {0, 0, 0}, Gb = 0.0, drhob = 0.0, afb[3] = {0, 0, 0};
    memset(A.fb, 0, popn * sizeof(double));

    for (int32_t n = nsteps - 1; n >= 0; n--) {
        /* replay steps 1-7 of step n */
        load_snapshot(s, snapf + (size_t)n * popn, &snapP[n]);
        const orc_particle *Pn = &snapP[n], *P1 = &snapP[n + 1];
        moments(s);
        virtual_densities(s);
        double Fv[1][3], Tv[1][3];
        forces_impl(s, s->F, Fv, Tv);
        collide(s);
        double dp[1][3], dl[1][3], dMbb[2];
        int64_t links[1];
        stream_bounce(s, dp, dl, dMbb, links);
        for (int z = 0; z < p->nz; z++)
            for (int y = 0; y < p->ny; y++)
                for (int x = 0; x < p->nx; x++)
                    solid_next[node_index(s, x, y, z)] = (unsigned char)particle_node(s, x, y, z, P1->X);

        /* 10: fnew_final = fnew + w_i delta_l on Phi^{n+1},
         * delta_l = -(dMbb + dMcov + dMunc)_l / nf                         */
        double nf = 0.0;
        for (int64_t m = 0; m < N; m++) nf += solid_next[m] ? 0.0 : 1.0;
        double deltab[2] = {0.0, 0.0};
        for (int64_t m = 0; m < N; m++) {
            if (solid_next[m]) continue;
            for (int l = 0; l < 2; l++)
                for (int i = 0; i < Q; i++) deltab[l] += s->W[i] * FI(A.fb, l, i, m);
        }
        double dMb[2] = {-deltab[0] / nf, -deltab[1] / nf};
        /* adjoint of fnew after the events: fb on Phi^{n+1}, zero elsewhere
         * (covered nodes are cleared, so nothing flows back through them)  */
        for (int64_t m = 0; m < N; m++)
            for (int l = 0; l < 2; l++)
                for (int i = 0; i < Q; i++)
                    FI(A.fnewb, l, i, m) = solid_next[m] ? 0.0 : FI(A.fb, l, i, m);

        /* 9: events (adjoints of U^{n+1/2}, Omega^{n+1/2}, X^{n+1} collect here) */
        double Ub1[3], Wb1[3], Xb1[3];
        for (int a = 0; a < 3; a++) { Ub1[a] = Ub[a]; Wb1[a] = Wb[a]; Xb1[a] = Xb[a]; }
        for (int z = 0; z < p->nz; z++)
            for (int y = 0; y < p->ny; y++)
                for (int x = 0; x < p->nx; x++) {
                    int64_t m = node_index(s, x, y, z);
                    double r[3];
                    separation(s, x, y, z, P1->X, r);
                    if (s->solid[m] && !solid_next[m]) {
                        /* uncovered: fnew(x) = f_eq(rb, u_b), u_b = U + Omega x r */
                        double rbv[2] = {0, 0};
                        int cnt = 0;
                        for (int i = 1; i < Q; i++) {
                            int xn = x + CV[i][0], yn = y + CV[i][1], zn = z + CV[i][2];
                            if (!resolve(s, &xn, &yn, &zn)) continue;
                            int64_t q = node_index(s, xn, yn, zn);
                            if (s->solid[q] || solid_next[q]) continue;
                            for (int l = 0; l < 2; l++)
                                for (int k = 0; k < Q; k++) rbv[l] += FI(s->fnew, l, k, q);
                            cnt++;
                        }
                        for (int l = 0; l < 2; l++) rbv[l] = cnt > 0 ? rbv[l] / cnt : p->rho0[l];
                        double w[3], u[3];
                        cross(P1->W, r, w);
                        for (int a = 0; a < 3; a++) u[a] = P1->U[a] + w[a];
                        double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
                        double rbb[2] = {0, 0}, ub[3] = {0, 0, 0};
                        for (int l = 0; l < 2; l++)
                            for (int i = 0; i < Q; i++) {
                                double cu = CV[i][0] * u[0] + CV[i][1] * u[1] + CV[i][2] * u[2];
                                double fbv = FI(A.fb, l, i, m);
                                rbb[l] += fbv * s->W[i] * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
                                for (int a = 0; a < 3; a++)
                                    ub[a] += fbv * s->W[i] * rbv[l] *
                                             (3.0 * CV[i][a] + 9.0 * cu * CV[i][a] - 3.0 * u[a]);
                            }
                        /* dMunc_l += rb_l */
                        for (int l = 0; l < 2; l++) rbb[l] += dMb[l];
                        /* Pev -= mom, Lev -= r x mom, mom = (rb_A + rb_B) u */
                        double mom[3], momb[3];
                        for (int a = 0; a < 3; a++) { mom[a] = (rbv[0] + rbv[1]) * u[a]; momb[a] = -Pevb[a]; }
                        add_cross(momb, Levb, r, -1.0);
                        double rbar[3] = {0, 0, 0};
                        add_cross(rbar, mom, Levb, -1.0);
                        for (int a = 0; a < 3; a++) {
                            ub[a] += (rbv[0] + rbv[1]) * momb[a];
                            rbb[0] += u[a] * momb[a];
                            rbb[1] += u[a] * momb[a];
                        }
                        /* u = U + Omega x r */
                        for (int a = 0; a < 3; a++) Ub1[a] += ub[a];
                        add_cross(Wb1, r, ub, 1.0);
                        add_cross(rbar, ub, P1->W, 1.0);
                        for (int a = 0; a < 3; a++) Xb1[a] -= rbar[a];
                        /* rb_l = mean over kept fluid neighbours of sum_k fnew */
                        if (cnt > 0)
                            for (int i = 1; i < Q; i++) {
                                int xn = x + CV[i][0], yn = y + CV[i][1], zn = z + CV[i][2];
                                if (!resolve(s, &xn, &yn, &zn)) continue;
                                int64_t q = node_index(s, xn, yn, zn);
                                if (s->solid[q] || solid_next[q]) continue;
                                for (int l = 0; l < 2; l++)
                                    for (int k = 0; k < Q; k++) FI(A.fnewb, l, k, q) += rbb[l] / cnt;
                            }
                        /* the populations fnew(x) before the overwrite are not used */
                        for (int l = 0; l < 2; l++)
                            for (int i = 0; i < Q; i++) FI(A.fnewb, l, i, m) = 0.0;
                    } else if (!s->solid[m] && solid_next[m]) {
                        /* covered: Pev += j, Lev += r x j, dMcov_l -= rho_l */
                        double j[3] = {0, 0, 0};
                        for (int l = 0; l < 2; l++)
                            for (int i = 0; i < Q; i++)
                                for (int a = 0; a < 3; a++) j[a] += FI(s->fnew, l, i, m) * CV[i][a];
                        double jb[3];
                        for (int a = 0; a < 3; a++) jb[a] = Pevb[a];
                        add_cross(jb, Levb, r, 1.0);
                        double rbar[3] = {0, 0, 0};
                        add_cross(rbar, j, Levb, 1.0);
                        for (int a = 0; a < 3; a++) Xb1[a] -= rbar[a];
                        for (int l = 0; l < 2; l++)
                            for (int i = 0; i < Q; i++)
                                FI(A.fnewb, l, i, m) = -dMb[l] + CV[i][0] * jb[0] + CV[i][1] * jb[1] +
                                                       CV[i][2] * jb[2];
                    }
                }

        /* 8: Newton-Euler.  J picks U_z^{n+1/2}; X^{n+1} = X^n + U^{n+1/2} */
        Ub1[2] += 1.0 / nsteps;
        for (int a = 0; a < 3; a++) Ub1[a] += Xb1[a];
        double Fb[3] = {0, 0, 0}, Tb[3] = {0, 0, 0};
        if (!p->fixed_velocity)
            for (int a = 0; a < 3; a++) { Fb[a] = Ub1[a] / mp; Tb[a] = Wb1[a] / Ip; }
        /* F = dp - Fv + Fext + Pev^n, T = dl - Tv + Lev^n; U^{n-1/2}, Omega^{n-1/2}
         * pass through                                                       */
        double Ub0[3], Wb0[3], Xb0[3];
        for (int a = 0; a < 3; a++) {
            gb[a] += cF * Fb[a];
            Ub0[a] = Ub1[a];
            Wb0[a] = Wb1[a];
            Xb0[a] = Xb1[a];
        }

        /* 7: streaming adjoint */
        memset(A.fpostb, 0, popn * sizeof(double));
        memset(A.rhob, 0, (size_t)(2 * N) * sizeof(double));
        for (int z = 0; z < p->nz; z++)
            for (int y = 0; y < p->ny; y++)
                for (int x = 0; x < p->nx; x++) {
                    int64_t m = node_index(s, x, y, z);
                    if (s->solid[m]) continue;
                    for (int l = 0; l < 2; l++) FI(A.fpostb, l, 0, m) += FI(A.fnewb, l, 0, m);
                    for (int i = 1; i < Q; i++) {
                        int xn = x + CV[i][0], yn = y + CV[i][1], zn = z + CV[i][2];
                        int io = opposite(i);
                        if (!resolve(s, &xn, &yn, &zn)) {
                            for (int l = 0; l < 2; l++) FI(A.fpostb, l, i, m) += FI(A.fnewb, l, io, m);
                            continue;
                        }
                        int64_t q = node_index(s, xn, yn, zn);
                        if (s->solid[q]) {
                            double r[3], w[3], ubv[3];
                            separation(s, x + 0.5 * CV[i][0], y + 0.5 * CV[i][1], z + 0.5 * CV[i][2],
                                       Pn->X, r);
                            cross(Pn->W, r, w);
                            for (int a = 0; a < 3; a++) ubv[a] = Pn->U[a] + w[a];
                            double cu = CV[i][0] * ubv[0] + CV[i][1] * ubv[1] + CV[i][2] * ubv[2];
                            /* lp = sum_l (2 fs_l - corr_l) c_i; dp += lp; dl += r x lp */
                            double lp[3] = {0, 0, 0}, corr[2];
                            for (int l = 0; l < 2; l++) {
                                corr[l] = 6.0 * s->W[i] * s->rho[l * N + m] * cu;
                                for (int a = 0; a < 3; a++)
                                    lp[a] += (2.0 * FI(s->fpost, l, i, m) - corr[l]) * CV[i][a];
                            }
                            double lpb[3];
                            for (int a = 0; a < 3; a++) lpb[a] = Fb[a];
                            add_cross(lpb, Tb, r, 1.0);
                            double rbar[3] = {0, 0, 0};
                            add_cross(rbar, lp, Tb, 1.0);
                            double clpb = CV[i][0] * lpb[0] + CV[i][1] * lpb[1] + CV[i][2] * lpb[2];
                            double cub = 0.0;
                            for (int l = 0; l < 2; l++) {
                                double a_ = FI(A.fnewb, l, io, m);
                                FI(A.fpostb, l, i, m) += a_ + 2.0 * clpb;
                                double corrb = -a_ - clpb - dMb[l];
                                A.rhob[l * N + m] += 6.0 * s->W[i] * cu * corrb;
                                cub += 6.0 * s->W[i] * s->rho[l * N + m] * corrb;
                            }
                            double ubb[3] = {cub * CV[i][0], cub * CV[i][1], cub * CV[i][2]};
                            for (int a = 0; a < 3; a++) Ub0[a] += ubb[a];
                            add_cross(Wb0, r, ubb, 1.0);
                            add_cross(rbar, ubb, Pn->W, 1.0);
                            for (int a = 0; a < 3; a++) Xb0[a] -= rbar[a];
                            continue;
                        }
                        for (int l = 0; l < 2; l++) FI(A.fpostb, l, i, m) += FI(A.fnewb, l, i, q);
                    }
                }

        /* 4-6: collision adjoint per fluid node */
        memset(A.fb, 0, popn * sizeof(double));
        for (int64_t m = 0; m < N; m++) {
            for (int l = 0; l < 2; l++) for (int a = 0; a < 3; a++) A.Fb[(l * 3 + a) * N + m] = 0.0;
            if (s->solid[m]) continue;
            double fin[2][Q], F[2][3], zz[36], fpb[2][Q], finb[2][Q], Fbn[2][3];
            for (int l = 0; l < 2; l++) {
                for (int i = 0; i < Q; i++) { fin[l][i] = FI(s->f, l, i, m); fpb[l][i] = FI(A.fpostb, l, i, m); }
                for (int a = 0; a < 3; a++) F[l][a] = s->F[(l * 3 + a) * N + m];
            }
            if (p->kT > 0.0) orc_normals(s, m, Pn->step, zz);
            else memset(zz, 0, sizeof(zz));
            collide_node_adjoint(s, fin, F, zz, fpb, finb, Fbn);
            for (int l = 0; l < 2; l++) {
                for (int i = 0; i < Q; i++) FI(A.fb, l, i, m) = finb[l][i];
                for (int a = 0; a < 3; a++) A.Fb[(l * 3 + a) * N + m] = Fbn[l][a];
            }
        }

        /* 3: forces F_l(x) = sum_i -G rho_l(x) w_i rt_l'(x + c_i) c_i + rho_l(x) a_f;
         * reaction Fv, Tv (about X^n) on links into particle nodes          */
        double af[3], Fext[1][3];
        driving(s, af, Fext);
        double Fvb[3] = {-Fb[0], -Fb[1], -Fb[2]}, Tvb[3] = {-Tb[0], -Tb[1], -Tb[2]};
        memset(A.rtb, 0, (size_t)(2 * N) * sizeof(double));
        for (int z = 0; z < p->nz; z++)
            for (int y = 0; y < p->ny; y++)
                for (int x = 0; x < p->nx; x++) {
                    int64_t m = node_index(s, x, y, z);
                    if (s->solid[m]) continue;
                    for (int l = 0; l < 2; l++)
                        for (int a = 0; a < 3; a++) {
                            A.rhob[l * N + m] += af[a] * A.Fb[(l * 3 + a) * N + m];
                            afb[a] += s->rho[l * N + m] * A.Fb[(l * 3 + a) * N + m];
                        }
                    for (int i = 1; i < Q; i++) {
                        int xn = x + CV[i][0], yn = y + CV[i][1], zn = z + CV[i][2];
                        int inside = resolve(s, &xn, &yn, &zn);
                        if (!inside) {
                            xn = x + CV[i][0]; yn = y + CV[i][1]; zn = z + CV[i][2];
                            mirror(s, &xn, &yn, &zn);
                        }
                        int64_t q = node_index(s, xn, yn, zn);
                        double linkb[2][3];
                        for (int l = 0; l < 2; l++)
                            for (int a = 0; a < 3; a++) linkb[l][a] = A.Fb[(l * 3 + a) * N + m];
                        if (inside && s->solid[q]) {
                            double r[3], fl[3] = {0, 0, 0};
                            separation(s, x + 0.5 * CV[i][0], y + 0.5 * CV[i][1], z + 0.5 * CV[i][2],
                                       Pn->X, r);
                            for (int l = 0; l < 2; l++)
                                for (int a = 0; a < 3; a++)
                                    fl[a] += -p->G * s->rho[l * N + m] * s->W[i] * s->rt[(1 - l) * N + q] * CV[i][a];
                            double flb[3];
                            for (int a = 0; a < 3; a++) flb[a] = Fvb[a];
                            add_cross(flb, Tvb, r, 1.0);
                            double rbar[3] = {0, 0, 0};
                            add_cross(rbar, fl, Tvb, 1.0);
                            for (int a = 0; a < 3; a++) Xb0[a] -= rbar[a];
                            for (int l = 0; l < 2; l++)
                                for (int a = 0; a < 3; a++) linkb[l][a] += flb[a];
                        }
                        for (int l = 0; l < 2; l++) {
                            double sl = CV[i][0] * linkb[l][0] + CV[i][1] * linkb[l][1] + CV[i][2] * linkb[l][2];
                            double other = s->rt[(1 - l) * N + q];
                            A.rhob[l * N + m] += -p->G * s->W[i] * other * sl;
                            A.rtb[(1 - l) * N + q] += -p->G * s->rho[l * N + m] * s->W[i] * sl;
                            Gb += -s->rho[l * N + m] * s->W[i] * other * sl;
                        }
                    }
                }

        /* 2: virtual densities (fluid: rt = rho; particle node: mean over fluid
         * neighbours +/- Delta rho)                                           */
        for (int z = 0; z < p->nz; z++)
            for (int y = 0; y < p->ny; y++)
                for (int x = 0; x < p->nx; x++) {
                    int64_t m = node_index(s, x, y, z);
                    if (!s->solid[m]) {
                        for (int l = 0; l < 2; l++) A.rhob[l * N + m] += A.rtb[l * N + m];
                        continue;
                    }
                    int cnt = 0;
                    for (int i = 1; i < Q; i++) {
                        int xn = x + CV[i][0], yn = y + CV[i][1], zn = z + CV[i][2];
                        if (!resolve(s, &xn, &yn, &zn)) continue;
                        if (s->solid[node_index(s, xn, yn, zn)]) continue;
                        cnt++;
                    }
                    if (cnt == 0) continue;
                    drhob += A.rtb[m] - A.rtb[N + m];
                    for (int i = 1; i < Q; i++) {
                        int xn = x + CV[i][0], yn = y + CV[i][1], zn = z + CV[i][2];
                        if (!resolve(s, &xn, &yn, &zn)) continue;
                        int64_t q = node_index(s, xn, yn, zn);
                        if (s->solid[q]) continue;
                        for (int l = 0; l < 2; l++) A.rhob[l * N + q] += A.rtb[l * N + m] / cnt;
                    }
                }

        /* 1: moments rho_l = sum_i f_{l i} */
        for (int64_t m = 0; m < N; m++) {
            if (s->solid[m]) continue;
            for (int l = 0; l < 2; l++)
                for (int i = 0; i < Q; i++) FI(A.fb, l, i, m) += A.rhob[l * N + m];
        }

        for (int a = 0; a < 3; a++) {
            Ub[a] = Ub0[a];
            Wb[a] = Wb0[a];
            Xb[a] = Xb0[a];
            Pevb[a] = Fb[a];
            Levb[a] = Tb[a];
        }
    }
    for (int a = 0; a < 3; a++) gb[a] += caf * afb[a];
    grad[0] = gb[0];
    grad[1] = gb[1];
    grad[2] = gb[2];
    grad[3] = Gb;
    grad[4] = drhob;

    /* leave the simulation at the state after the last step */
    load_snapshot(s, snapf + (size_t)nsteps * popn, &snapP[nsteps]);
    free(snapf); free(snapP); free(A.fb); free(A.fnewb); free(A.fpostb); free(A.rhob);
    free(A.rtb); free(A.Fb); free(solid_next);
    return 0;
}
