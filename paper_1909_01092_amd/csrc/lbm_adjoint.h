// Launch interface of the adjoint kernels (reverse-mode derivative of the
// step with respect to g, G and Delta rho; single replica, every relaxation
// time 1).
//
// Paper: Xue, Biferale, Sbragaglia, Toschi, "A lattice Boltzmann study of
// particle settling in a fluctuating multicomponent fluid under
// confinement".  The derivative is taken through the step of Sec. 2
// (eq. lbe, eq. sc-force, noise paragraph, particle paragraph) and the
// external force of Sec. 3, eq. (fp); the objective is the time-averaged
// settling velocity of Sec. 4.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm_types.h"

namespace lbm {

// Adjoint of the sphere and of the parameters, FP64.
struct AdjState {
    double Ub[3], Wb[3], Xb[3];  // adjoints of U^{n+1/2}, Omega^{n+1/2}, X^{n+1} entering the
                                 // reverse of step n; of U^{n-1/2}, Omega^{n-1/2}, X^n after it
    double Pevb[3], Levb[3];     // adjoints of the event momentum / angular momentum made by step n
    double Fb[3], Tb[3];         // adjoints of the force and torque of step n
    double dMb[2];               // adjoint of each mass flux of step n: -(adjoint of delta) / |Phi^{n+1}|
    double dsum[2];              // sum over fluid nodes of the density adjoint of the last reversed state
    double grad[5];              // dJ/d(g_x, g_y, g_z, G, Delta rho) so far (g: external-force part)
    double afb[3];               // adjoint of the body-force acceleration of the fluid
    double Jsum;                 // sum of U_z^{n+1/2} over the reversed steps
};

constexpr int ADJ_PA = 13;   // doubles per workgroup partial of the local kernel
constexpr int ADJ_PB = 2;    // doubles per workgroup partial of the gather kernel
constexpr int ADJ_BOX = 1024;  // threads of the bounding-box kernels

struct AdjArgs {
    const RepDesc *desc;
    const RepState *stn;     // recorded state before step n
    const RepState *stn1;    // recorded state after step n
    AdjState *adj;
    double cF;               // d F_ext / d g (force on the sphere per unit g)
    double invN;             // 1 / number of steps in J
    const void *recn;        // moments before step n: [8][N] (rho_A - rho0_A, rho_B - rho0_B, j_A, j_B)
    const void *recn1;       // moments after step n
    void *Anext;             // adjoint of the state after step n: [8][N] (rho_A, rho_B, j_A, j_B)
    void *Acur;              // adjoint of the state before step n, written
    void *Fb;                // adjoint of the node forces of step n: [6][N]
    double *vt;              // box of X^n: wetting-layer densities of step n [2][S^3]
    double *vinv;            // box: 1 / fluid-neighbour count of particle nodes (0: none) [S^3]
    double *vtb;             // box: adjoint of the wetting-layer densities [2][S^3]
    double *ubn;             // box: uncovered-node density adjoint per kept neighbour [2][S^3]
    double *partA;           // [nwg][ADJ_PA]
    double *partB;           // [nwg][ADJ_PB]
    int32_t nwg;             // workgroups of the node kernels (256 threads, one node each)
};

struct RecArgs {
    const RepDesc *desc;
    const RepState *state;
    const void *src;         // populations before the step
    void *rec;               // [8][N] moments, written
    RepState *st_out;        // copy of the state, written
};

hipError_t launch_adj_record(int prec, const RecArgs &a, int64_t N, hipStream_t s);
hipError_t launch_adj_step(int prec, const AdjArgs &a, hipStream_t s);

}  // namespace lbm
