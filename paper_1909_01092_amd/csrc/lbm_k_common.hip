// Precision-independent kernels (initial wetting layer, hydrodynamic velocity,
// column sums) and the dispatch on storage precision.
#include "lbm_kernels_impl.h"

namespace lbm {

// Wetting-layer densities, bbox origin and fluid count of the initial state
// (one workgroup per replica).
__global__ __launch_bounds__(256) void k_init_layer(InitArgs a) {
    __shared__ double red[4];
    const int r = blockIdx.x;
    const RepDesc &D = a.desc[r];
    RepState *st = a.state + r;
    const Geo g = geo_of(D);
    if (!D.has_particle) {
        if (threadIdx.x == 0) st->n_fluid = (double)D.N;
        return;
    }
    const int n3[3] = {g.nx, g.ny, g.nz};
    const bool w3[3] = {g.wx, g.wy, g.wz};
    const double X[3] = {st->X[0], st->X[1], st->X[2]};
    int org[3];
    for (int q = 0; q < 3; q++) org[q] = (int)floor(X[q] - D.radius) - 2;
    const int Sx = D.S, S3 = Sx * Sx * Sx;
    double *vrho = a.vrho + D.bbox_off * 2;
    uint32_t *pmask = a.pmask + D.bbox_off;
    auto init_rho = [&](int x, int y, int z, int l) {
        uint32_t c0 = (uint32_t)nidx(x, y, z, g), c1 = 0u, c2 = 0u, c3 = 1u;
        philox4x32_10(c0, c1, c2, c3, D.key0, D.key1);
        const uint32_t w = l == 0 ? c0 : c1;
        const bool swap = D.init_split > 0 && z >= D.init_split;  // other phase above the split
        return (swap ? D.rho0[1 - l] : D.rho0[l]) + D.init_amp * (2.0 * (((double)w + 0.5) * 0x1p-32) - 1.0);
    };
    double ns[1] = {0.0};
    for (int b = threadIdx.x; b < S3; b += 256) {
        int p[3];
        const int bb[3] = {b % Sx, (b / Sx) % Sx, b / (Sx * Sx)};
        bool in = true;
        for (int q = 0; q < 3; q++) {
            int v = org[q] + bb[q];
            if (v < 0 || v >= n3[q]) {
                if (w3[q]) in = false;
                else v = ((v % n3[q]) + n3[q]) % n3[q];
            }
            p[q] = v;
        }
        const bool solid = in && pnode(p[0], p[1], p[2], X, D.R2, g);
        pmask[b] = solid ? MASK_SOLID : 0u;  // populations of step 0 sit in own slots
        if (!solid) continue;
        ns[0] += 1.0;
        double s0 = 0.0, s1 = 0.0;
        int cnt = 0;
        for (int i = 1; i < Q; i++) {
            int qx = p[0] + cx(i), qy = p[1] + cy(i), qz = p[2] + cz(i);
            if (!(wrap1(qx, g.nx, g.wx) && wrap1(qy, g.ny, g.wy) && wrap1(qz, g.nz, g.wz))) continue;
            if (pnode(qx, qy, qz, X, D.R2, g)) continue;
            s0 += init_rho(qx, qy, qz, 0);
            s1 += init_rho(qx, qy, qz, 1);
            cnt++;
        }
        vrho[b] = cnt > 0 ? s0 / cnt + D.drho : 0.0;
        vrho[S3 + b] = cnt > 0 ? s1 / cnt - D.drho : 0.0;
    }
    block_sum<256, 1>(ns, red);
    if (threadIdx.x == 0) {
        st->n_fluid = (double)D.N - ns[0];
        for (int q = 0; q < 3; q++) st->org[q] = org[q];
    }
}

// Hydrodynamic velocity v + (F_A + F_B) / (2 rho) per node from the scratch
// written by k_fields_a.
__global__ __launch_bounds__(256) void k_fields_b(FieldArgs a) {
    const RepDesc &D = a.desc[a.rep];
    const Geo g = geo_of(D);
    const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (n >= g.N) return;
    const int x = (int)(n % g.nx), y = (int)((n / g.nx) % g.ny);
    const int z = (int)(n / ((int64_t)g.nx * g.ny));
    const double *rt = a.scratch, *jt = a.scratch + 2 * g.N, *sol = a.scratch + 8 * g.N;
    double *u = a.scratch + 5 * g.N;
    if (sol[n] != 0.0) {
        for (int q = 0; q < 3; q++) u[q * g.N + n] = 0.0;
        return;
    }
    double grad[2][3] = {{0, 0, 0}, {0, 0, 0}};
    for (int i = 1; i < Q; i++) {
        const int qx = mirror1(x + cx(i), g.nx, g.wx), qy = mirror1(y + cy(i), g.ny, g.wy);
        const int qz = mirror1(z + cz(i), g.nz, g.wz);
        const int64_t m = nidx(qx, qy, qz, g);
        for (int l = 0; l < 2; l++) {
            const double v = wgt(i) * rt[l * g.N + m];
            grad[l][0] += v * cx(i); grad[l][1] += v * cy(i); grad[l][2] += v * cz(i);
        }
    }
    const double rA = rt[n], rB = rt[g.N + n];
    for (int q = 0; q < 3; q++) {
        const double FA = -D.G * rA * grad[1][q] + rA * D.af[q];
        const double FB = -D.G * rB * grad[0][q] + rB * D.af[q];
        u[q * g.N + n] = (jt[q * g.N + n] + 0.5 * (FA + FB)) / (rA + rB);
    }
}

// Column sums over z: mass_A, mass_B, j (3), sum |u|^2, sum u_z, fluid count.
__global__ __launch_bounds__(256) void k_columns(FieldArgs a) {
    const RepDesc &D = a.desc[a.rep];
    const Geo g = geo_of(D);
    const int64_t plane = (int64_t)g.nx * g.ny;
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= plane) return;
    const double *rt = a.scratch, *jt = a.scratch + 2 * g.N, *u = a.scratch + 5 * g.N,
                 *sol = a.scratch + 8 * g.N;
    double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int z = 0; z < g.nz; z++) {
        const int64_t n = c + plane * z;
        if (sol[n] != 0.0) continue;
        s[0] += rt[n];
        s[1] += rt[g.N + n];
        for (int q = 0; q < 3; q++) s[2 + q] += jt[q * g.N + n];
        const double ux = u[n], uy = u[g.N + n], uz = u[2 * g.N + n];
        s[5] += ux * ux + uy * uy + uz * uz;
        s[6] += uz;
        s[7] += 1.0;
    }
    for (int k = 0; k < 8; k++) a.columns[k * plane + c] = s[k];
}

hipError_t launch_main(int prec, const MainArgs &a, int grid, int block, size_t lds, hipStream_t s) {
    if (prec == 0) return launch_main_f64(a, grid, block, lds, s);
    if (prec == 1) return launch_main_f32(a, grid, block, lds, s);
    return launch_main_f16(a, grid, block, lds, s);
}

hipError_t launch_links(int prec, const LinkArgs &a, int grid, hipStream_t s) {
    if (prec == 0) return launch_links_f64(a, grid, s);
    if (prec == 1) return launch_links_f32(a, grid, s);
    return launch_links_f16(a, grid, s);
}

hipError_t launch_particle(int prec, const ParticleArgs &a, int grid, hipStream_t s) {
    if (prec == 0) return launch_particle_f64(a, grid, s);
    if (prec == 1) return launch_particle_f32(a, grid, s);
    return launch_particle_f16(a, grid, s);
}

hipError_t launch_init(int prec, const InitArgs &a, int grid, int nrep, hipStream_t s) {
    hipError_t e = prec == 0 ? launch_init_f64(a, grid, s)
                 : prec == 1 ? launch_init_f32(a, grid, s) : launch_init_f16(a, grid, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_init_layer, dim3(nrep), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_export(int prec, const ExportArgs &a, int64_t count, hipStream_t s) {
    if (prec == 0) return launch_export_f64(a, count, s);
    if (prec == 1) return launch_export_f32(a, count, s);
    return launch_export_f16(a, count, s);
}

hipError_t launch_fields(int prec, const FieldArgs &a, int64_t N, int64_t plane, hipStream_t s) {
    hipError_t e = prec == 0 ? launch_fields_a_f64(a, N, s)
                 : prec == 1 ? launch_fields_a_f32(a, N, s) : launch_fields_a_f16(a, N, s);
    if (e != hipSuccess) return e;
    const int grid = (int)((N + 255) / 256);
    hipLaunchKernelGGL(k_fields_b, dim3(grid), dim3(256), 0, s, a);
    e = hipGetLastError();
    if (e != hipSuccess || a.columns == nullptr) return e;
    hipLaunchKernelGGL(k_columns, dim3((int)((plane + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace lbm
