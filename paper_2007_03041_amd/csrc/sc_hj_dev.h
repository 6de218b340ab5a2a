// sc_hj_dev.h -- argument blocks and constants of the Hamilton-Jacobi and proposer kernels
// (library internal).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace scx {

enum { HJ_LINEAR = 0, HJ_WENOZ = 1, HJ_LEARNED = 2 };

constexpr double HJ_EPS_Z = 1e-6;  // WENO-Z epsilon

// proposer: features (8) -> 32 -> 32 -> 3; FP32 master parameters, row-major
// (out, in) weights followed by their biases
constexpr int MLP_IN = 8, MLP_H = 32, MLP_OUT = 3;
constexpr int MLP_W1 = 0;
constexpr int MLP_B1 = MLP_W1 + MLP_H * MLP_IN;
constexpr int MLP_W2 = MLP_B1 + MLP_H;
constexpr int MLP_B2 = MLP_W2 + MLP_H * MLP_H;
constexpr int MLP_W3 = MLP_B2 + MLP_H;
constexpr int MLP_B3 = MLP_W3 + MLP_OUT * MLP_H;
constexpr int MLP_NPARAM = MLP_B3 + MLP_OUT;

// device-side state of a run (doubles)
enum { HJ_S_C = 0, HJ_S_T = 1, HJ_S_STEPS = 2, HJ_S_FALLBACK = 3, HJ_S_ERRSUM = 4, HJ_S_JUDGED = 5, HJ_S_SIZE = 8 };

struct HjQuadArgs {
    int64_t nx, ny;
    int32_t axis;    // 0: x (contiguous), 1: y
    int32_t pad_;
    double c[3][3];  // substencil weights, node order x_{i-3+r}, x_{i-2+r}, x_{i-1+r} (J_R)
    double d[3];     // linear weights
    double theta;    // largest accepted |proposal - WENO-Z| per weight
};

enum { HJ_H_QUADRATIC = 0, HJ_H_EX3 = 1 };

struct HjStepArgs {
    int64_t nx, ny, npts;
    double dx, dy;
    double alpha_x, alpha_y;
    double cfl_h;  // CFL min(dx, dy): dt = cfl_h / c
    double t_end;
    int32_t hamiltonian;  // HJ_H_QUADRATIC: (p^2 + q^2) / 2; HJ_H_EX3: (1 + p + q)^2 / 2 - S(x, y, t)
    int32_t pad_;
};

// Fused step of the separable Hamiltonian (p^2 + q^2) / 2 (linear or WENO-Z weights): each wave owns
// HJF_C points of one line plus HJF_KW window points on either side, over which the periodic
// line's sweeps are summed from zero (taken where d^{HJF_KW} < 2^-60).
constexpr int HJF_C = 512;
constexpr int HJF_KW = 64;
constexpr int HJF_PPL = (HJF_C + 2 * HJF_KW) / 64;  // points a lane sweeps
constexpr int HJF_ROW = HJF_C + 2 * HJF_KW + 6;     // tile points per line (stencil halo of 3 each side)
struct HjFusedArgs {
    double alpha[2];             // per axis
    double d[2];                 // e^{-alpha dx} per axis
    double dpow[2][HJF_PPL + 1]; // d^t, t = 0..HJF_PPL
    double dscan[2][6];          // d^{HJF_PPL 2^s}: decay across 2^s lanes
};
// the number of workgroups of the x and y passes (their wave-speed maxima go to part[])
int64_t hj_fused_blocks(int64_t nx, int64_t ny, int axis);
hipError_t launch_hj_fused_pass(int axis, int weights, const double *u, const double *w_in, double *out,
                                const HjQuadArgs &Q, const HjFusedArgs &F, const HjStepArgs &A, const double *state,
                                double *part, hipStream_t st);

hipError_t launch_hj_weno_quad(int mode, const double *u, double *JL, double *JR, const HjQuadArgs &A,
                               const float *P, double *stats, hipStream_t st);
hipError_t launch_hj_update(double *u, const double *DmX, const double *DpX, const double *DmY, const double *DpY,
                            const HjStepArgs &A, const double *state, double *part, hipStream_t st);
hipError_t launch_hj_init_speed(const double *u, const HjStepArgs &A, double *part, hipStream_t st);
hipError_t launch_hj_finish(const double *part, int64_t nparts, const double *stats, int64_t nstats,
                            const HjStepArgs &A, double *state, int mode, hipStream_t st);
hipError_t launch_hj_harvest(const double *u, const HjQuadArgs &A, float *X, float *Y, hipStream_t st);
int64_t mlp_train_slots(int64_t n);
hipError_t launch_mlp_forward(const float *P, const float *X, float *Y, int64_t n, hipStream_t st);
hipError_t launch_mlp_grad(const float *P, const float *X, const float *Y, int64_t n, float *partial, float *grad,
                           float *loss, hipStream_t st);
hipError_t launch_mlp_adam(float *P, const float *grad, float *M, float *V, int t, float lr, hipStream_t st);

}  // namespace scx
