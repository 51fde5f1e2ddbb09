/* A plain C program on the library's C ABI alone (no Python, no torch):
 * device memory from hipMalloc, the default stream, one context.
 *
 *   c_abi_driver <params.bin> <n_entries> <precision> <steps> <out.bin>
 *
 * params.bin holds n_entries lbm_params structs as the caller laid them out.
 * The program runs lbm_workspace_bytes, lbm_init, lbm_step(steps) and
 * lbm_step_noalloc(steps), then writes entry 0's lbm_particle and its
 * populations (double, [2][19][nz][ny][nx]) to out.bin.  Exit status: 0, or
 * 1 + the first failing call's position, with lbm_last_error on stderr. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "lbm.h"

static int fail(int where, const lbm_ctx *c) {
    const char *m = lbm_last_error(c);
    fprintf(stderr, "c_abi_driver: call %d failed: %s\n", where, m ? m : "(no message)");
    return 1 + where;
}

int main(int argc, char **argv) {
    if (argc != 6) {
        fprintf(stderr, "usage: %s params.bin n_entries precision steps out.bin\n", argv[0]);
        return 1;
    }
    const int n = atoi(argv[2]), prec = atoi(argv[3]), steps = atoi(argv[4]);
    if (n < 1) return 1;
    lbm_params *p = (lbm_params *)calloc((size_t)n, sizeof(lbm_params));
    FILE *f = fopen(argv[1], "rb");
    if (!p || !f || fread(p, sizeof(lbm_params), (size_t)n, f) != (size_t)n) {
        fprintf(stderr, "c_abi_driver: cannot read %d parameter sets from %s\n", n, argv[1]);
        return 1;
    }
    fclose(f);
    size_t bytes = 0;
    if (lbm_workspace_bytes(p, n, prec, &bytes) != LBM_OK) return fail(1, NULL);
    void *ws = NULL;
    if (hipMalloc(&ws, bytes) != hipSuccess) {
        fprintf(stderr, "c_abi_driver: hipMalloc of %zu bytes failed\n", bytes);
        return 2;
    }
    lbm_ctx *c = NULL;
    if (lbm_init(p, n, prec, ws, bytes, NULL, &c) != LBM_OK) return fail(2, NULL);
    if (lbm_step(c, steps) != LBM_OK) return fail(3, c);
    if (lbm_step_noalloc(c, steps) != LBM_OK) return fail(4, c);
    lbm_particle st;
    memset(&st, 0, sizeof st);
    const int rc = lbm_particle_state(c, 0, &st);
    if (rc != LBM_OK && rc != LBM_EUNSTABLE) return fail(5, c);
    const size_t nf = (size_t)2 * 19 * (size_t)p[0].nx * (size_t)p[0].ny * (size_t)p[0].nz;
    double *pop = (double *)malloc(nf * sizeof(double));
    if (!pop || lbm_populations(c, 0, pop) != LBM_OK) return fail(6, c);
    FILE *o = fopen(argv[5], "wb");
    if (!o || fwrite(&st, sizeof st, 1, o) != 1 || fwrite(pop, sizeof(double), nf, o) != nf) {
        fprintf(stderr, "c_abi_driver: cannot write %s\n", argv[5]);
        return 8;
    }
    fclose(o);
    lbm_destroy(c);
    hipFree(ws);
    free(pop);
    free(p);
    return 0;
}
