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
    uint32_t done;               // completion counter of the wetting-chain kernel (0 between steps)
    uint32_t pad;
};

// Forward values of a fluid node at step n rebuilt from the recorded
// moments: density deviations and densities, momenta, forces, the sums
// sum_i w_i rho~_l(x + c_i) c_i, velocity, species-momentum noise and its
// normals and amplitude; links through a wall / into the sphere (bit i).
template <typename T>
struct NodeFwd {
    T rd[2], rl[2], jl[2][3], F[2][3], sv[2][3], u[3], xid[3], zd[4], ampf;
    uint32_t wall, link;
};
constexpr size_t NODE_FWD_BYTES = sizeof(NodeFwd<double>);

constexpr int ADJ_PA = 13;   // doubles per workgroup partial of the local kernel
constexpr int ADJ_PB = 2;    // doubles per workgroup partial of the gather kernel
constexpr int ADJ_PE = 9;    // doubles of an event partial (stride PART per workgroup)
constexpr int ADJ_PC = 3;    // doubles of a wetting-chain partial (stride PART per workgroup)

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
    void *Fb;                // rho_l(x) times the adjoint of the node force F_l(x) of step n: [6][N]
    double *vt;              // box of X^n: wetting-layer densities of step n [2][S^3]
    double *vinv;            // box: 1 / fluid-neighbour count of particle nodes (0: none) [S^3]
    double *vtb;             // box: adjoint of the wetting-layer densities [2][S^3]
    double *ubn;             // box: uncovered-node density adjoint per kept neighbour [2][S^3]
    void *nfw;               // box: NodeFwd<T> of the nodes with sphere links [S^3]
    double *partA;           // [nlt][ADJ_PA]
    double *partB;           // [nwg][ADJ_PB]
    double *partE;           // [nbw][PART] event partials
    double *partC;           // [nbw][PART] wetting-chain partials
    double *partL;           // [2 nbw][PART] link partials (same slots as partA)
    double *partM;           // [nmw][PART] wall-mirror partials
    int32_t nwg;             // workgroups of the gather kernel (256 threads, one node each)
    int32_t lty, nlt;        // local kernel: tile rows (of one plane), tiles (one workgroup each)
    int32_t desc_nx;         // nodes per x-row (host copy, for the local kernel's LDS size)
    int32_t nbw;             // workgroups of the box kernels (256 threads, one box node each)
    int32_t nmw;             // workgroups of the wall-face kernel (256 threads, one face node each)
};

struct RecArgs {
    const RepDesc *desc;
    const RepState *state;
    const void *src;         // populations before the step
    void *rec;               // [8][N] moments, written
    RepState *st_out;        // copy of the state, written
};

hipError_t launch_adj_record(int prec, const RecArgs &a, int64_t N, hipStream_t s);
// one reversed step; e0 / e1 (optional) are recorded around the node kernel k_adj_local
hipError_t launch_adj_step(int prec, const AdjArgs &a, hipStream_t s, hipEvent_t e0, hipEvent_t e1);

}  // namespace lbm
