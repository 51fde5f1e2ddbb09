// Per-node arithmetic of the fluctuating two-component D3Q19 step:
// counter-based noise, the orthogonal mode transform and the MRT collision
// with Guo forcing.  Everything here is __host__ __device__ and free of
// memory traffic so that kernels (and a host-side unit check) share it.
//
// Paper: Xue, Biferale, Sbragaglia, Toschi, "A lattice Boltzmann study of
// particle settling in a fluctuating multicomponent fluid under
// confinement", Sec. 2 (eq. lbe, MRT paragraph, noise paragraph).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

constexpr int Q = 19;

// D3Q19 velocities: rest, axis links in (+,-) pairs, planar diagonals in
// opposite pairs (xy, xz, yz).
__host__ __device__ __forceinline__ constexpr int cx(int i) {
    return (i == 1 || i == 7 || i == 9 || i == 11 || i == 13) ? 1
         : (i == 2 || i == 8 || i == 10 || i == 12 || i == 14) ? -1 : 0;
}
__host__ __device__ __forceinline__ constexpr int cy(int i) {
    return (i == 3 || i == 7 || i == 10 || i == 15 || i == 17) ? 1
         : (i == 4 || i == 8 || i == 9 || i == 16 || i == 18) ? -1 : 0;
}
__host__ __device__ __forceinline__ constexpr int cz(int i) {
    return (i == 5 || i == 11 || i == 14 || i == 15 || i == 18) ? 1
         : (i == 6 || i == 12 || i == 13 || i == 16 || i == 17) ? -1 : 0;
}
__host__ __device__ __forceinline__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }
__host__ __device__ __forceinline__ constexpr double wgt(int i) {
    return i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
}

// ------------------------------------------------------------ Philox4x32-10
// Salmon et al. (SC'11): 10 rounds of two 32x32->64 products, Weyl key bumps.
// three-way xor: one v_bitop3_b32 (truth table 0x96) on gfx950
__host__ __device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
#else
    return a ^ b ^ c;
#endif
}

__host__ __device__ inline void philox4x32_10(uint32_t &c0, uint32_t &c1, uint32_t &c2,
                                              uint32_t &c3, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; r++) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = xor3((uint32_t)(p1 >> 32), c1, k0);
        const uint32_t n2 = xor3((uint32_t)(p0 >> 32), c3, k1);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// Box-Muller on two 32-bit words, u = (w + 1/2) 2^-32 in (0, 1):
//   z0 = sqrt(-2 ln u1) cos(2 pi u2),  z1 = sqrt(-2 ln u1) sin(2 pi u2).
__host__ __device__ inline void box_muller(uint32_t w1, uint32_t w2, double &z0, double &z1) {
    const double u1 = ((double)w1 + 0.5) * 0x1p-32;
    const double u2 = ((double)w2 + 0.5) * 0x1p-32;
    const double r = sqrt(-2.0 * log(u1));
    const double a = 2.0 * 3.14159265358979323846 * u2;
    z0 = r * cos(a);
    z1 = r * sin(a);
}

// FP32 form.  ln u1 keeps full relative accuracy for u1 near 1: with
// v = 1 - u1 (exact from the complemented word) and t = fl(1 - v), the
// rounding error e = (1 - t) - v is exact (Sterbenz), and
// ln(1 - v) = ln(t + e) = ln t + e / t + O(e^2) = ln t + e (1 + O(v)),
// so ln u1 = ln t + e to a few FP32 ulps; for u1 < 1/2 e = 0.  Angles are
// taken in revolutions, which is what the hardware sine / cosine consume.
__host__ __device__ inline void box_muller(uint32_t w1, uint32_t w2, float &z0, float &z1) {
    const bool big = w1 >= 0x80000000u;
    const float v = __builtin_fmaf((float)(big ? ~w1 : w1), 0x1p-32f, 0x1p-33f);
    const float t = big ? 1.0f - v : v;
    const float e = big ? (1.0f - t) - v : 0.0f;
#if defined(__HIP_DEVICE_COMPILE__)
    const float m2lnu = __builtin_fmaf(__builtin_amdgcn_logf(t), -1.3862943611198906f, -2.0f * e);
#else
    const float m2lnu = -2.0f * (logf(t) + e);
#endif
    const float u2 = __builtin_fmaf((float)w2, 0x1p-32f, 0x1p-33f);
#if defined(__HIP_DEVICE_COMPILE__)
    const float r = __builtin_amdgcn_sqrtf(m2lnu);
    const float c = __builtin_amdgcn_cosf(u2);
    const float s = __builtin_amdgcn_sinf(u2);
#else
    const float r = sqrtf(m2lnu);
    const float c = (float)cos(6.283185307179586 * u2);
    const float s = (float)sin(6.283185307179586 * u2);
#endif
    z0 = r * c;
    z1 = r * s;
}

// Standard normals for (node, step): Philox block b = 0..8 with counter
// (node, step, b, 0); words (0,1) and (2,3) of each block form Box-Muller
// pairs, so block b yields normals 4b..4b+3.  Blocks 0-3 drive modes 4..18 of
// component A (normals 0..14), blocks 4-7 those of component B (normals
// 16..30), block 8 the antisymmetric species-momentum noise (normals 32..34).
template <typename T>
__host__ __device__ inline void noise_block(uint32_t node, uint32_t step, uint32_t b, uint32_t k0,
                                            uint32_t k1, T *z4) {
    uint32_t c0 = node, c1 = step, c2 = b, c3 = 0u;
    philox4x32_10(c0, c1, c2, c3, k0, k1);
    box_muller(c0, c1, z4[0], z4[1]);
    box_muller(c2, c3, z4[2], z4[3]);
}


// ------------------------------------------------------------- collision
template <typename T>
struct Coef {
    T rho0[2];
    T gs, gb, gj, gg;   // gamma = 1 - 1/tau for shear, bulk, momentum, ghost modes
    T nb, ns, ng;       // sqrt(mu (1 - gamma^2)) for bulk, shear, ghost modes
    T ampd;             // sqrt(mu b_1 (1 - gamma_j^2)) for the species-momentum noise
    int noise;          // kT > 0
    int diffusive;      // species-momentum noise on
};

// b_k = sum_i w_i e_k(c_i)^2 of the mode set used by modes_hi / back_transform
__host__ __device__ __forceinline__ constexpr double mode_norm(int k) {
    return k == 0 ? 1.0 : k <= 3 ? 1.0 / 3.0 : k == 4 ? 2.0 / 3.0 : k == 5 ? 4.0 / 3.0
         : k == 6 ? 4.0 / 9.0 : k <= 9 ? 1.0 / 9.0 : k <= 12 ? 2.0 / 3.0 : k <= 15 ? 2.0 / 9.0
         : k == 16 ? 2.0 : k == 17 ? 4.0 / 3.0 : 4.0 / 9.0;
}
// sqrt(b_k), 1 / b_k as literals
__host__ __device__ __forceinline__ constexpr double sqrt_norm(int k) {
    return k == 0 ? 1.0 : k <= 3 ? 0.57735026918962576 : k == 4 ? 0.81649658092772603
         : k == 5 ? 1.1547005383792515 : k == 6 ? 0.66666666666666667 : k <= 9 ? 0.33333333333333333
         : k <= 12 ? 0.81649658092772603 : k <= 15 ? 0.47140452079103169 : k == 16 ? 1.4142135623730951
         : k == 17 ? 1.1547005383792515 : 0.66666666666666667;
}
__host__ __device__ __forceinline__ constexpr double inv_norm(int k) {
    return k == 0 ? 1.0 : k <= 3 ? 3.0 : k == 4 ? 1.5 : k == 5 ? 0.75 : k == 6 ? 2.25
         : k <= 9 ? 9.0 : k <= 12 ? 1.5 : k <= 15 ? 4.5 : k == 16 ? 0.5 : k == 17 ? 0.75 : 2.25;
}

// Relaxation factors and noise amplitudes from relaxation times and kT.
template <typename T>
__host__ __device__ inline Coef<T> make_coef(double rho0A, double rho0B, double tau_shear,
                                             double tau_bulk, double tau_mom, double tau_ghost,
                                             double kT, int diffusive) {
    Coef<T> c;
    const double gs = 1.0 - 1.0 / tau_shear, gb = 1.0 - 1.0 / tau_bulk;
    const double gj = 1.0 - 1.0 / tau_mom, gg = 1.0 - 1.0 / tau_ghost;
    const double mu = 3.0 * kT;
    c.rho0[0] = T(rho0A);
    c.rho0[1] = T(rho0B);
    c.gs = T(gs); c.gb = T(gb); c.gj = T(gj); c.gg = T(gg);
    c.nb = T(sqrt(mu * (1.0 - gb * gb)));
    c.ns = T(sqrt(mu * (1.0 - gs * gs)));
    c.ng = T(sqrt(mu * (1.0 - gg * gg)));
    c.ampd = T(sqrt(mu * mode_norm(1) * (1.0 - gj * gj)));
    c.noise = kT > 0.0;
    c.diffusive = diffusive;
    return c;
}

template <typename T>
__host__ __device__ inline T tmax0(T a) { return a > T(0) ? a : T(0); }

// 1/a: exact division in FP64, the hardware reciprocal (about 1 ulp) in FP32
__host__ __device__ inline double recip(double a) { return 1.0 / a; }
__host__ __device__ inline float recip(float a) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rcpf(a);
#else
    return 1.0f / a;
#endif
}

// Density deviation, momentum and modes 4..18 of one component (orthogonal
// polynomial basis; modes of the deviation from w_i rho0 equal those of f for
// k >= 1).
template <typename T>
__host__ __device__ inline void component_modes(const T (&f)[Q], T &rd, T (&j)[3], T (&m)[Q]) {
    const T sx = f[1] + f[2], sy = f[3] + f[4], sz = f[5] + f[6];
    const T dx = f[1] - f[2], dy = f[3] - f[4], dz = f[5] - f[6];
    const T p7 = f[7] + f[8], q7 = f[7] - f[8], p9 = f[9] + f[10], q9 = f[9] - f[10];
    const T p11 = f[11] + f[12], q11 = f[11] - f[12], p13 = f[13] + f[14], q13 = f[13] - f[14];
    const T p15 = f[15] + f[16], q15 = f[15] - f[16], p17 = f[17] + f[18], q17 = f[17] - f[18];
    const T Exy = p7 + p9, Exz = p11 + p13, Eyz = p15 + p17;
    rd = f[0] + sx + sy + sz + Exy + Exz + Eyz;
    const T ax = q7 + q9 + q11 + q13, ay = q7 - q9 + q15 + q17, az = q11 - q13 + q15 - q17;
    j[0] = dx + ax;
    j[1] = dy + ay;
    j[2] = dz + az;
    m[4] = -f[0] + Exy + Exz + Eyz;
    m[5] = T(2) * sx - sy - sz + Exy + Exz - T(2) * Eyz;
    m[6] = sy - sz + Exy - Exz;
    m[7] = p7 - p9;
    m[8] = p15 - p17;
    m[9] = p11 - p13;
    m[10] = T(-2) * dx + ax;
    m[11] = T(-2) * dy + ay;
    m[12] = T(-2) * dz + az;
    m[13] = q7 + q9 - q11 - q13;
    m[14] = -q7 + q9 + q15 + q17;
    m[15] = q11 - q13 - q15 + q17;
    m[16] = f[0] - T(2) * (sx + sy + sz) + Exy + Exz + Eyz;
    m[17] = T(-2) * sx + sy + sz + Exy + Exz - T(2) * Eyz;
    m[18] = -sy + sz + Exy - Exz;
}

// f_i = w_i sum_k e_k(c_i) a_k with a_k = m_k / b_k.
template <typename T>
__host__ __device__ inline void back_transform(const T (&a)[Q], T (&f)[Q]) {
    const T w0 = T(1.0 / 3.0), w1 = T(1.0 / 18.0), w2 = T(1.0 / 36.0);
    f[0] = w0 * (a[0] - a[4] + a[16]);
    const T Ex = w1 * (a[0] + T(2) * a[5] - T(2) * a[16] - T(2) * a[17]);
    const T Ox = w1 * (a[1] - T(2) * a[10]);
    const T Ey = w1 * (a[0] - a[5] + a[6] - T(2) * a[16] + a[17] - a[18]);
    const T Oy = w1 * (a[2] - T(2) * a[11]);
    const T Ez = w1 * (a[0] - a[5] - a[6] - T(2) * a[16] + a[17] + a[18]);
    const T Oz = w1 * (a[3] - T(2) * a[12]);
    f[1] = Ex + Ox; f[2] = Ex - Ox;
    f[3] = Ey + Oy; f[4] = Ey - Oy;
    f[5] = Ez + Oz; f[6] = Ez - Oz;
    const T Exy = w2 * (a[0] + a[4] + a[5] + a[6] + a[16] + a[17] + a[18]);
    const T Pxy = w2 * a[7];
    const T Ax = w2 * (a[1] + a[10] + a[13]);
    const T Ay = w2 * (a[2] + a[11] - a[14]);
    f[7] = Exy + Pxy + Ax + Ay;  f[8] = Exy + Pxy - Ax - Ay;
    f[9] = Exy - Pxy + Ax - Ay;  f[10] = Exy - Pxy - Ax + Ay;
    const T Exz = w2 * (a[0] + a[4] + a[5] - a[6] + a[16] + a[17] - a[18]);
    const T Pxz = w2 * a[9];
    const T Bx = w2 * (a[1] + a[10] - a[13]);
    const T Bz = w2 * (a[3] + a[12] + a[15]);
    f[11] = Exz + Pxz + Bx + Bz; f[12] = Exz + Pxz - Bx - Bz;
    f[13] = Exz - Pxz + Bx - Bz; f[14] = Exz - Pxz - Bx + Bz;
    const T Eyz = w2 * (a[0] + a[4] - T(2) * a[5] + a[16] - T(2) * a[17]);
    const T Pyz = w2 * a[8];
    const T Cy = w2 * (a[2] + a[11] + a[14]);
    const T Cz = w2 * (a[3] + a[12] - a[15]);
    f[15] = Eyz + Pyz + Cy + Cz; f[16] = Eyz + Pyz - Cy - Cz;
    f[17] = Eyz - Pyz + Cy - Cz; f[18] = Eyz - Pyz - Cy + Cz;
}

// Barycentric velocity u = (j_A + j_B + (F_A + F_B)/2) / rho shared by both
// components, and the species-momentum noise xi_d (normals 32..34 of z).
template <typename T>
__host__ __device__ inline void common_velocity(const T (&rd)[2], const T (&j)[2][3],
                                                const T (&F)[2][3], const T (&z)[36],
                                                const Coef<T> &c, T (&u)[3], T (&xid)[3]) {
    const T rA = c.rho0[0] + rd[0], rB = c.rho0[1] + rd[1];
    const T inv = recip(rA + rB);
    for (int a = 0; a < 3; a++) u[a] = (j[0][a] + j[1][a] + T(0.5) * (F[0][a] + F[1][a])) * inv;
    const T amp = (c.noise && c.diffusive) ? c.ampd * sqrt(tmax0(rA) * tmax0(rB) * inv) : T(0);
    for (int a = 0; a < 3; a++) xid[a] = amp * z[32 + a];
}

// Post-collision deviations of one component (sigma = +1 for A, -1 for B;
// zl = its normals 0..14 for modes 4..18):
//   j*  = rho_l u + g_j (j_l + F_l/2 - rho_l u) + F_l/2 + sigma xi_d
//   m*_k = m_eq + g_k (m_k - m_eq) + (1 + g_k)/2 Phi_k + noise,   k = 4..9
//   m*_k = g_g m_k + noise,                                         k = 10..18
// noise amplitude sqrt(mu rho_l b_k (1 - g_k^2)), mu = kT / c_s^2.
template <typename T>
__host__ __device__ inline void relax_component(T rho0l, T sig, T rd, const T (&j)[3],
                                                const T (&m)[Q], const T (&Fl)[3], const T (&u)[3],
                                                const T (&xid)[3], const T (&zl)[16],
                                                const Coef<T> &c, T (&out)[Q]) {
    const T r = rho0l + rd;
    const T sq = c.noise ? sqrt(tmax0(r)) : T(0);
    const T nb = c.nb * sq, ns = c.ns * sq, ng = c.ng * sq;
    const T uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    T a[Q];
    a[0] = rd;
    for (int q = 0; q < 3; q++) {
        const T ru = r * u[q];
        a[1 + q] = T(3) * (ru + c.gj * (j[q] + T(0.5) * Fl[q] - ru) + T(0.5) * Fl[q] + sig * xid[q]);
    }
    const T uF = u[0] * Fl[0] + u[1] * Fl[1] + u[2] * Fl[2];
    const T hb = T(0.5) * (T(1) + c.gb), hs = T(0.5) * (T(1) + c.gs);
    const T e4 = r * uu, e5 = r * (T(3) * u[0] * u[0] - uu), e6 = r * (u[1] * u[1] - u[2] * u[2]);
    const T e7 = r * u[0] * u[1], e8 = r * u[1] * u[2], e9 = r * u[0] * u[2];
    const T f4 = T(2) * uF, f5 = T(2) * (T(3) * u[0] * Fl[0] - uF);
    const T f6 = T(2) * (u[1] * Fl[1] - u[2] * Fl[2]);
    const T f7 = u[0] * Fl[1] + u[1] * Fl[0], f8 = u[1] * Fl[2] + u[2] * Fl[1];
    const T f9 = u[0] * Fl[2] + u[2] * Fl[0];
    a[4] = T(inv_norm(4)) * (e4 + c.gb * (m[4] - e4) + hb * f4) + T(inv_norm(4) * sqrt_norm(4)) * nb * zl[0];
    a[5] = T(inv_norm(5)) * (e5 + c.gs * (m[5] - e5) + hs * f5) + T(inv_norm(5) * sqrt_norm(5)) * ns * zl[1];
    a[6] = T(inv_norm(6)) * (e6 + c.gs * (m[6] - e6) + hs * f6) + T(inv_norm(6) * sqrt_norm(6)) * ns * zl[2];
    a[7] = T(inv_norm(7)) * (e7 + c.gs * (m[7] - e7) + hs * f7) + T(inv_norm(7) * sqrt_norm(7)) * ns * zl[3];
    a[8] = T(inv_norm(8)) * (e8 + c.gs * (m[8] - e8) + hs * f8) + T(inv_norm(8) * sqrt_norm(8)) * ns * zl[4];
    a[9] = T(inv_norm(9)) * (e9 + c.gs * (m[9] - e9) + hs * f9) + T(inv_norm(9) * sqrt_norm(9)) * ns * zl[5];
#pragma unroll
    for (int k = 10; k < Q; k++)
        a[k] = T(inv_norm(k)) * c.gg * m[k] + T(inv_norm(k) * sqrt_norm(k)) * ng * zl[k - 4];
    back_transform(a, out);
}

// relax_component for gamma_k = 0 on every mode (all relaxation times 1): the
// post-collision state depends on density and momentum only.
template <typename T>
__host__ __device__ inline void relax_tau1(T rho0l, T sig, T rd, const T (&j)[3], const T (&Fl)[3],
                                           const T (&u)[3], const T (&xid)[3], const T (&zl)[16],
                                           const Coef<T> &c, T (&out)[Q]) {
    const T r = rho0l + rd;
    const T sq = c.noise ? sqrt(tmax0(r)) : T(0);
    const T nb = c.nb * sq, ns = c.ns * sq, ng = c.ng * sq;
    const T uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    T a[Q];
    a[0] = rd;
    for (int q = 0; q < 3; q++) a[1 + q] = T(3) * (r * u[q] + T(0.5) * Fl[q] + sig * xid[q]);
    const T uF = u[0] * Fl[0] + u[1] * Fl[1] + u[2] * Fl[2];
    const T e4 = r * uu, e5 = r * (T(3) * u[0] * u[0] - uu), e6 = r * (u[1] * u[1] - u[2] * u[2]);
    const T e7 = r * u[0] * u[1], e8 = r * u[1] * u[2], e9 = r * u[0] * u[2];
    const T f4 = uF, f5 = T(3) * u[0] * Fl[0] - uF, f6 = u[1] * Fl[1] - u[2] * Fl[2];
    const T f7 = T(0.5) * (u[0] * Fl[1] + u[1] * Fl[0]), f8 = T(0.5) * (u[1] * Fl[2] + u[2] * Fl[1]);
    const T f9 = T(0.5) * (u[0] * Fl[2] + u[2] * Fl[0]);
    a[4] = T(inv_norm(4)) * (e4 + f4) + T(inv_norm(4) * sqrt_norm(4)) * nb * zl[0];
    a[5] = T(inv_norm(5)) * (e5 + f5) + T(inv_norm(5) * sqrt_norm(5)) * ns * zl[1];
    a[6] = T(inv_norm(6)) * (e6 + f6) + T(inv_norm(6) * sqrt_norm(6)) * ns * zl[2];
    a[7] = T(inv_norm(7)) * (e7 + f7) + T(inv_norm(7) * sqrt_norm(7)) * ns * zl[3];
    a[8] = T(inv_norm(8)) * (e8 + f8) + T(inv_norm(8) * sqrt_norm(8)) * ns * zl[4];
    a[9] = T(inv_norm(9)) * (e9 + f9) + T(inv_norm(9) * sqrt_norm(9)) * ns * zl[5];
#pragma unroll
    for (int k = 10; k < Q; k++) a[k] = T(inv_norm(k) * sqrt_norm(k)) * ng * zl[k - 4];
    back_transform(a, out);
}

}  // namespace lbm
