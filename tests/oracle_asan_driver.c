/* Drives the FP64 oracle through the code paths the tests use, for a build
 * with the host address and undefined-behaviour sanitizers: a walled channel
 * with noise, distinct relaxation times, a moving and spinning sphere with
 * cover / uncover events and a wetting offset; a fully periodic box whose
 * sphere crosses a face; a demixed start; then the adjoint (every relaxation
 * time 1).  Exit status 0 when every call returns and the results are
 * finite. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "lbm_oracle.h"

static orc_params base(int nx, int ny, int nz, unsigned walls) {
    orc_params p;
    memset(&p, 0, sizeof(p));
    p.nx = nx; p.ny = ny; p.nz = nz; p.walls = walls;
    p.rho0[0] = 0.95; p.rho0[1] = 0.05;
    p.init_amp = 1e-3; p.G = 1.5;
    p.tau_shear = p.tau_bulk = p.tau_mom = p.tau_ghost = 1.0;
    p.kT = 1e-4; p.seed = 7; p.rho_p = 2.0; p.noise_diffusive = 1;
    return p;
}

static int run(orc_params p, int steps, int adjoint) {
    orc_sim *s = orc_create(&p);
    if (!s) return 1;
    orc_step(s, steps);
    const long n = (long)p.nx * p.ny * p.nz;
    double *f = malloc(sizeof(double) * 2 * 19 * n), *rho = malloc(sizeof(double) * 2 * n),
           *u = malloc(sizeof(double) * 3 * n), *F = malloc(sizeof(double) * 6 * n);
    orc_get_populations(s, f);
    orc_get_fields(s, rho, u);
    orc_forces(s, F);
    double m[2], j[3], u3[3 * 64];
    orc_observables(s, m, j);
    orc_u_series(s, u3, 64);
    orc_particle q;
    orc_get_particle(s, &q);
    int bad = !(isfinite(m[0]) && isfinite(m[1]) && isfinite(q.X[2]) && isfinite(f[0]));
    if (adjoint) {
        double grad[5], J = 0.0;
        bad |= orc_adjoint(s, 12, grad, &J) != 0;
        for (int k = 0; k < 5; k++) bad |= !isfinite(grad[k]);
    }
    printf("%dx%dx%d walls %u: covered %lld uncovered %lld%s\n", p.nx, p.ny, p.nz, p.walls,
           (long long)q.n_covered, (long long)q.n_uncovered, bad ? " BAD" : "");
    free(f); free(rho); free(u); free(F);
    orc_destroy(s);
    return bad;
}

int main(void) {
    int bad = 0;
    orc_params a = base(10, 12, 14, 3);
    a.tau_shear = 0.8; a.tau_bulk = 1.1; a.tau_mom = 0.9; a.tau_ghost = 1.3;
    a.g[2] = 5e-5; a.radius = 2.7; a.wet_drho = 0.1;
    a.X0[0] = 4.6; a.X0[1] = 5.4; a.X0[2] = 7.3;
    a.U0[0] = 0.02; a.U0[1] = -0.03; a.U0[2] = 0.06;
    a.W0[0] = 0.01; a.W0[1] = 0.02; a.W0[2] = -0.01;
    bad |= run(a, 25, 0);
    orc_params b = base(14, 14, 14, 0);
    b.radius = 2.5; b.wet_drho = -0.1;
    b.X0[0] = 0.1; b.X0[1] = 13.2; b.X0[2] = 6.5;
    b.U0[0] = -0.05; b.U0[1] = 0.04; b.U0[2] = 0.05;
    bad |= run(b, 20, 1);
    orc_params c = base(10, 10, 16, 7);
    c.rho0[0] = 2.21; c.rho0[1] = 0.09; c.init_amp = 0.0; c.kT = 0.0;
    c.init_split = 8; c.radius = 2.5; c.rho_p = 4.6; c.wet_drho = 0.3;
    c.X0[0] = 4.5; c.X0[1] = 4.5; c.X0[2] = 7.5;
    bad |= run(c, 20, 1);
    return bad;
}
