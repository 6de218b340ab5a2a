// sc_hj_kernels.hip -- kernels of the nonlinear Hamilton-Jacobi example (u_t + |grad u|^2 / 2 = 0, periodic,
// 2-D) and of the learned quadrature-weight proposer.
//
//   hj_weno_quad     per point: the two 5-point local integrals J_L, J_R along one axis from three
//                    3-point substencils (Sec. 2.4) with linear, WENO-Z or proposed weights; the
//                    proposer is a 3-layer MLP evaluated on the matrix cores (BF16 operands, FP32
//                    accumulation), its proposal judged against the WENO-Z weights and replaced by
//                    them when it is off by more than a threshold
//   hj_update        per point: the Lax-Friedrichs numerical Hamiltonian of the one-sided
//                    derivatives (Sec. 2.5) and the forward-Euler update, with the time step and the
//                    dissipation taken from the lagged wave speed held on the device
//   hj_finish_step   reduces the new wave speed and advances the device-side time (the paper's
//                    adaptive rule: the reduction of one step feeds the next)
//   mlp_forward / mlp_train_tile / mlp_reduce_grads / mlp_adam: inference and training of the proposer
#include <hip/hip_runtime.h>

#include <cmath>
#include <stdint.h>

#include "sc_hj_dev.h"

namespace scx {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// float -> bfloat16 bits, round to nearest even: the gfx950 conversion instruction (two values per
// instruction where the compiler pairs them)
__device__ __forceinline__ short f2bf(float x)
{
    return __builtin_bit_cast(short, (__bf16)x);
}

__device__ __forceinline__ f32x4 mfma16(bf16x4 a, bf16x4 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// ------------------------------------------------------------------------------------------
// The proposer on the matrix cores.  A 16x16x16 product: lane l = 16 g + m holds A[m][4g..4g+3],
// B[4g..4g+3][m] and the result D[4g..4g+3][m].  Weights are read into B operands once per wave:
// B[k][n] = W[n][k] for W stored (out, in) row-major.
// ------------------------------------------------------------------------------------------
struct MlpOperands {
    bf16x4 w1[2];     // layer 1: N-tiles 0, 1 (K = 16, features 0..7 real)
    bf16x4 w2[2][2];  // layer 2: [N-tile][K-step]
    bf16x4 w3[2];     // layer 3: [K-step] (N = 3 real of 16)
    float b1[2], b2[2], b3;
};

__device__ __forceinline__ MlpOperands mlp_load(const float *__restrict__ P, int lane)
{
    MlpOperands o;
    const int m = lane & 15, g = lane >> 4;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int n = 16 * t + m;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int k = 4 * g + j;
            o.w1[t][j] = k < MLP_IN ? f2bf(P[MLP_W1 + n * MLP_IN + k]) : (short)0;
        }
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int j = 0; j < 4; ++j) o.w2[t][s][j] = f2bf(P[MLP_W2 + n * MLP_H + 16 * s + 4 * g + j]);
        o.b1[t] = P[MLP_B1 + n];
        o.b2[t] = P[MLP_B2 + n];
    }
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int j = 0; j < 4; ++j) o.w3[s][j] = m < MLP_OUT ? f2bf(P[MLP_W3 + m * MLP_H + 16 * s + 4 * g + j]) : (short)0;
    o.b3 = m < MLP_OUT ? P[MLP_B3 + m] : 0.f;
    return o;
}

// Forward of 16 samples whose features are rows feat[0..15][0..7] (LDS).  hid: 16 x 33 LDS
// scratch of the calling wave; the logits go to z[0..15][0..3] (LDS).  Every lane of the wave calls
// it; `bar` synchronises the writers and readers of the scratch.  If keep != nullptr the layer
// inputs and pre-activations are copied there for the backward pass (keep: z1[16][33], h1[16][33],
// z2[16][33], h2[16][33]).
template <typename Bar>
__device__ __forceinline__ void mlp_tile_forward(const MlpOperands &o, const float (*feat)[MLP_IN], float (*hid)[33],
                                                 float (*z)[4], float (*keep)[16][33], int lane, Bar bar)
{
    const int m = lane & 15, g = lane >> 4;
    bf16x4 a;
#pragma unroll
    for (int j = 0; j < 4; ++j) a[j] = (4 * g + j) < MLP_IN ? f2bf(feat[m][4 * g + j]) : (short)0;
    f32x4 z1[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const f32x4 c = {o.b1[t], o.b1[t], o.b1[t], o.b1[t]};
        z1[t] = mfma16(a, o.w1[t], c);
    }
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            hid[4 * g + j][16 * t + m] = fmaxf(z1[t][j], 0.f);
            if (keep) keep[0][4 * g + j][16 * t + m] = z1[t][j];
        }
    bar();
    bf16x4 a2[2];
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int j = 0; j < 4; ++j) a2[s][j] = f2bf(hid[m][16 * s + 4 * g + j]);
    bar();
    f32x4 z2[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const f32x4 c = {o.b2[t], o.b2[t], o.b2[t], o.b2[t]};
        z2[t] = mfma16(a2[0], o.w2[t][0], c);
        z2[t] = mfma16(a2[1], o.w2[t][1], z2[t]);
    }
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            hid[4 * g + j][16 * t + m] = fmaxf(z2[t][j], 0.f);
            if (keep) keep[2][4 * g + j][16 * t + m] = z2[t][j];
        }
    bar();
    bf16x4 a3[2];
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int j = 0; j < 4; ++j) a3[s][j] = f2bf(hid[m][16 * s + 4 * g + j]);
    bar();
    const f32x4 c3 = {o.b3, o.b3, o.b3, o.b3};
    f32x4 z3 = mfma16(a3[0], o.w3[0], c3);
    z3 = mfma16(a3[1], o.w3[1], z3);
    if (m < MLP_OUT)
#pragma unroll
        for (int j = 0; j < 4; ++j) z[4 * g + j][m] = z3[j];
    bar();
}

// Inference of 16 samples with every product transposed: the weights are the A operand and the
// samples the B operand, so a layer's result -- lane 16 g + m holding units 4g..4g+3 of sample m --
// is the next layer's B operand as it stands and the hidden activations stay in registers (the
// weight registers of mlp_load serve unchanged: A[m][4g..4g+3] of a unit block is what they hold).
// Each product sums the same terms as mlp_tile_forward's.  The logits of sample m go to
// z[m][0..2] (LDS) from lanes 0..15.
struct MlpRowBias {
    f32x4 b1[2], b2[2], b3;  // biases of units 16 t + 4 g + j (layer 3: unit 4 g + j)
};

__device__ __forceinline__ MlpRowBias mlp_row_bias(const float *__restrict__ P, int lane)
{
    MlpRowBias r;
    const int g = lane >> 4;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            r.b1[t][j] = P[MLP_B1 + 16 * t + 4 * g + j];
            r.b2[t][j] = P[MLP_B2 + 16 * t + 4 * g + j];
        }
        r.b3[j] = (4 * g + j) < MLP_OUT ? P[MLP_B3 + 4 * g + j] : 0.f;
    }
    return r;
}

__device__ __forceinline__ void mlp_tile_infer(const MlpOperands &o, const MlpRowBias &rb, const float (*feat)[MLP_IN],
                                               float (*z)[4], int lane)
{
    const int m = lane & 15, g = lane >> 4;
    bf16x4 x;
#pragma unroll
    for (int j = 0; j < 4; ++j) x[j] = (4 * g + j) < MLP_IN ? f2bf(feat[m][4 * g + j]) : (short)0;
    bf16x4 h1[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const f32x4 r = mfma16(o.w1[t], x, rb.b1[t]);
#pragma unroll
        for (int j = 0; j < 4; ++j) h1[t][j] = f2bf(fmaxf(r[j], 0.f));
    }
    bf16x4 h2[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        f32x4 r = mfma16(o.w2[t][0], h1[0], rb.b2[t]);
        r = mfma16(o.w2[t][1], h1[1], r);
#pragma unroll
        for (int j = 0; j < 4; ++j) h2[t][j] = f2bf(fmaxf(r[j], 0.f));
    }
    f32x4 r3 = mfma16(o.w3[0], h2[0], rb.b3);
    r3 = mfma16(o.w3[1], h2[1], r3);
    if (g == 0)
#pragma unroll
        for (int j = 0; j < MLP_OUT; ++j) z[m][j] = r3[j];
}

__device__ __forceinline__ void softmax3(const float *zz, double *om)
{
    const double a = zz[0], b = zz[1], c = zz[2];
    const double mx = fmax(a, fmax(b, c));
    const double ea = exp(a - mx), eb = exp(b - mx), ec = exp(c - mx);
    const double s = ea + eb + ec;
    om[0] = ea / s;
    om[1] = eb / s;
    om[2] = ec / s;
}

// Features of a 5-point stencil (ETA5 order): the substencils' second differences over their
// largest magnitude, that magnitude against the WENO-Z epsilon (log scale), and the deviations of
// the outer values from the centre value over their largest magnitude.
__device__ __forceinline__ void stencil_features(const double *s, float *f)
{
    double q[3], Q = 0.0;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        q[r] = s[r] - 2.0 * s[r + 1] + s[r + 2];
        Q = fmax(Q, fabs(q[r]));
    }
#pragma unroll
    for (int r = 0; r < 3; ++r) f[r] = Q > 0.0 ? (float)(q[r] / Q) : 0.f;
    double lg = Q > 0.0 ? log10(Q * Q / HJ_EPS_Z) : -8.0;
    lg = fmin(fmax(lg, -8.0), 8.0);
    f[3] = (float)(lg / 8.0);
    const double e[4] = {s[0] - s[2], s[1] - s[2], s[3] - s[2], s[4] - s[2]};
    double E = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) E = fmax(E, fabs(e[k]));
#pragma unroll
    for (int k = 0; k < 4; ++k) f[4 + k] = E > 0.0 ? (float)(e[k] / E) : 0.f;
}

// WENO-Z weights of a 5-point stencil: smoothness = squared second difference per substencil.
__device__ __forceinline__ void wenoz(const double *s, const double *d, double *om)
{
    double beta[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const double q = s[r] - 2.0 * s[r + 1] + s[r + 2];
        beta[r] = q * q;
    }
    const double tau = fabs(beta[0] - beta[2]);
    double sum = 0.0;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        om[r] = d[r] * (1.0 + tau / (HJ_EPS_Z + beta[r]));
        sum += om[r];
    }
#pragma unroll
    for (int r = 0; r < 3; ++r) om[r] /= sum;
}

// ------------------------------------------------------------------------------------------
// hj_weno_quad: block of 256 points (4 waves); each point has two stencils (J_R: nodes
// x_{i-3}..x_{i+1}; J_L: the mirror x_{i+3}..x_{i-1}).
// ------------------------------------------------------------------------------------------
template <int MODE>
__global__ void __launch_bounds__(256) hj_weno_quad(const double *__restrict__ u, double *__restrict__ JL,
                                                    double *__restrict__ JR, const HjQuadArgs A,
                                                    const float *__restrict__ P, double *__restrict__ stats)
{
    __shared__ float feat[512][MLP_IN];
    __shared__ float zo[512][4];
    __shared__ double red[2][4];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6;
    const int64_t p = (int64_t)blockIdx.x * 256 + tid;
    const bool ok = p < A.nx * A.ny;
    const int64_t pj = ok ? p / A.nx : 0, pi = ok ? p % A.nx : 0;
    double v[7];
#pragma unroll
    for (int k = 0; k < 7; ++k) {
        int64_t idx;
        if (A.axis == 0) {
            int64_t i2 = pi + (k - 3);
            i2 = i2 < 0 ? i2 + A.nx : (i2 >= A.nx ? i2 - A.nx : i2);
            idx = pj * A.nx + i2;
        } else {
            int64_t j2 = pj + (k - 3);
            j2 = j2 < 0 ? j2 + A.ny : (j2 >= A.ny ? j2 - A.ny : j2);
            idx = j2 * A.nx + pi;
        }
        v[k] = ok ? u[idx] : 0.0;
    }
    double sR[5], sL[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        sR[k] = v[k];      // node offset k - 3
        sL[k] = v[6 - k];  // mirror: offset 3 - k
    }
    double oR[3], oL[3];
    double err_sum = 0.0, nfall = 0.0;
    if (MODE == HJ_LINEAR) {
#pragma unroll
        for (int r = 0; r < 3; ++r) oR[r] = oL[r] = A.d[r];
    } else {
        wenoz(sR, A.d, oR);
        wenoz(sL, A.d, oL);
    }
    if (MODE == HJ_LEARNED) {
        // Every tile below reads and writes only its own wave's rows of feat and zo (tile T of wave
        // wv covers its points wv*64 + 16 (T mod 4) ..., stencil R for T < 4, L after), so the
        // waves synchronise with themselves only: LDS accesses of one wave complete in order, and
        // the fences keep the compiler from moving accesses across the sync points.
        auto bar = [] {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        };
        stencil_features(sR, feat[tid]);
        stencil_features(sL, feat[256 + tid]);
        bar();
        const MlpOperands o = mlp_load(P, lane);
        const MlpRowBias rb = mlp_row_bias(P, lane);
        for (int T = 0; T < 8; ++T) {
            const int base = (T >> 2) * 256 + wv * 64 + 16 * (T & 3);
            mlp_tile_infer(o, rb, &feat[base], &zo[base], lane);
        }
        bar();
        double pR[3], pL[3];
        softmax3(zo[tid], pR);
        softmax3(zo[256 + tid], pL);
        double eR = 0.0, eL = 0.0;
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            eR = fmax(eR, fabs(pR[r] - oR[r]));
            eL = fmax(eL, fabs(pL[r] - oL[r]));
        }
        if (ok) {
            err_sum = eR + eL;
            nfall = (eR > A.theta ? 1.0 : 0.0) + (eL > A.theta ? 1.0 : 0.0);
        }
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            if (eR <= A.theta) oR[r] = pR[r];
            if (eL <= A.theta) oL[r] = pL[r];
        }
        // per-block statistics: proposals judged, fallbacks, summed judged error (sums within each
        // wave by shuffles, then across the four waves)
#pragma unroll
        for (int sft = 32; sft > 0; sft >>= 1) {
            nfall += __shfl_down(nfall, sft, 64);
            err_sum += __shfl_down(err_sum, sft, 64);
        }
        if (lane == 0) {
            red[0][wv] = nfall;
            red[1][wv] = err_sum;
        }
        __syncthreads();
        if (tid == 0) {
            const int64_t nb = blockIdx.x;
            stats[3 * nb + 0] = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
            stats[3 * nb + 1] = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
            stats[3 * nb + 2] = (double)(((int64_t)A.nx * A.ny - (int64_t)blockIdx.x * 256) < 256
                                             ? 2 * ((int64_t)A.nx * A.ny - (int64_t)blockIdx.x * 256)
                                             : 512);
        }
    }
    if (!ok) return;
    double jr = 0.0, jl = 0.0;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        double qR = 0.0, qL = 0.0;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            qR = fma(A.c[r][j], sR[r + j], qR);
            qL = fma(A.c[r][j], sL[r + j], qL);
        }
        jr = fma(oR[r], qR, jr);
        jl = fma(oL[r], qL, jl);
    }
    JR[p] = jr;
    JL[p] = jl;
}

// ------------------------------------------------------------------------------------------
// Update and the adaptive rule
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ double hj_dt(const HjStepArgs &A, const double *state)
{
    double dt = A.cfl_h / state[HJ_S_C];
    const double left = A.t_end - state[HJ_S_T];
    return dt < left ? dt : (left > 0.0 ? left : 0.0);
}

// u <- u - dt H^(p-, p+, q-, q+); D* hold u - L^{-1}[u] from the sweeps: p- = alpha Dm, p+ = -alpha Dp
__global__ void __launch_bounds__(256) hj_update(double *__restrict__ u, const double *__restrict__ DmX,
                                                 const double *__restrict__ DpX, const double *__restrict__ DmY,
                                                 const double *__restrict__ DpY, const HjStepArgs A,
                                                 const double *__restrict__ state, double *__restrict__ part)
{
    __shared__ double red[256];
    const int tid = threadIdx.x;
    const int64_t p = (int64_t)blockIdx.x * 256 + tid;
    const double c = state[HJ_S_C];
    const double dt = hj_dt(A, state);
    double m = 0.0;
    if (p < A.npts) {
        const double pm = A.alpha_x * DmX[p], pp = -A.alpha_x * DpX[p];
        const double qm = A.alpha_y * DmY[p], qp = -A.alpha_y * DpY[p];
        const double px = 0.5 * (pm + pp), qy = 0.5 * (qm + qp);
        double H;
        if (A.hamiltonian == HJ_H_EX3) {
            // Example 3 (Sec. 5.1): H = (1 + p + q)^2 / 2 and the source of the manufactured
            // solution u = t (sin x + sin y), S = sin x + sin y + (1 + t cos x + t cos y)^2 / 2,
            // at the old time; the wave speed is the largest |H_p| = |1 + p + q| over the four
            // one-sided combinations
            const double s = 1.0 + px + qy;
            const double t = state[HJ_S_T];
            const double x = (double)(p % A.nx) * A.dx, y = (double)(p / A.nx) * A.dy;
            const double sx = sin(x), sy = sin(y);
            const double w = 1.0 + t * cos(x) + t * cos(y);
            const double S = sx + sy + 0.5 * w * w;
            H = 0.5 * s * s + c * 0.5 * (pm - pp) + c * 0.5 * (qm - qp) - S;
            m = fmax(fmax(fabs(1.0 + pm + qm), fabs(1.0 + pm + qp)), fmax(fabs(1.0 + pp + qm), fabs(1.0 + pp + qp)));
        } else {
            H = 0.5 * (px * px + qy * qy) + c * 0.5 * (pm - pp) + c * 0.5 * (qm - qp);
            m = fmax(fmax(fabs(pm), fabs(pp)), fmax(fabs(qm), fabs(qp)));
        }
        u[p] = u[p] - dt * H;
    }
    red[tid] = m;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) red[tid] = fmax(red[tid], red[tid + s]);
        __syncthreads();
    }
    if (tid == 0) part[blockIdx.x] = red[0];
}

// Initial wave speed: max of |H_p|, |H_q| at periodic central differences of u0.
__global__ void __launch_bounds__(256) hj_init_speed(const double *__restrict__ u, const HjStepArgs A,
                                                     double *__restrict__ part)
{
    __shared__ double red[256];
    const int tid = threadIdx.x;
    const int64_t p = (int64_t)blockIdx.x * 256 + tid;
    double m = 0.0;
    if (p < A.npts) {
        const int64_t j = p / A.nx, i = p % A.nx;
        const int64_t ip = i + 1 == A.nx ? 0 : i + 1, im = i == 0 ? A.nx - 1 : i - 1;
        const int64_t jp = j + 1 == A.ny ? 0 : j + 1, jm = j == 0 ? A.ny - 1 : j - 1;
        const double gx = (u[j * A.nx + ip] - u[j * A.nx + im]) / (2.0 * A.dx);
        const double gy = (u[jp * A.nx + i] - u[jm * A.nx + i]) / (2.0 * A.dy);
        m = A.hamiltonian == HJ_H_EX3 ? fabs(1.0 + gx + gy) : fmax(fabs(gx), fabs(gy));
    }
    red[tid] = m;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) red[tid] = fmax(red[tid], red[tid + s]);
        __syncthreads();
    }
    if (tid == 0) part[blockIdx.x] = red[0];
}

// ------------------------------------------------------------------------------------------
// Fused step of the separable Hamiltonian H(p, q) = (p^2 + q^2) / 2: its Lax-Friedrichs numerical
// Hamiltonian splits into an x part (p_mean^2 / 2 + c (p- - p+) / 2) and a y part, so one step is
// two line passes: along x, w = u - dt Hx; along y, u <- w - dt Hy, each computing its weights,
// local integrals, sweeps and one-sided derivatives in registers.  One wave per line chunk of
// HJF_C points; its lanes sweep HJF_PPL consecutive points each over the chunk and HJF_KW window
// points on either side, and the sweeps of the periodic line are summed from zero at the window's
// ends: the dropped remainder is below d^{HJF_KW} < 2^-60 of the result (Sec. 3.1, the N-N
// criterion at that tolerance), so no wave needs another's totals.  AXIS 0: lines along x, TC of
// them per workgroup, tile [line][point]; AXIS 1: TC adjacent y lines, tile [point][line] so the
// loads and stores run along rows.
// ------------------------------------------------------------------------------------------
template <int AXIS, int TC, int MODE>
__global__ void __launch_bounds__(TC * 64) hj_fused_pass(const double *__restrict__ u, const double *w_in,
                                                         double *out, const HjQuadArgs Q, const HjFusedArgs F,
                                                         const HjStepArgs A, const double *__restrict__ state,
                                                         double *__restrict__ part)
{
    constexpr int LS = AXIS == 0 ? HJF_ROW : TC + 1;  // LDS stride: x between lines, y between points
    __shared__ double tile[TC * HJF_ROW + (AXIS == 0 ? 0 : HJF_ROW)];
    __shared__ double red[TC];
    auto TI = [](int line, int q) { return AXIS == 0 ? line * LS + q : q * LS + line; };
    const int tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t n = AXIS == 0 ? A.nx : A.ny;       // points per line
    const int64_t nlines = AXIS == 0 ? A.ny : A.nx;
    const int64_t nch = (n + HJF_C - 1) / HJF_C;
    const int64_t chunk = (int64_t)blockIdx.x % nch;
    const int64_t line0 = ((int64_t)blockIdx.x / nch) * TC;
    const int64_t c0 = chunk * HJF_C;
    const int64_t q0 = c0 - HJF_KW - 3;  // line point of tile point 0 (wrapped below)
    auto wrap = [n](int64_t p) {
        p %= n;
        return p < 0 ? p + n : p;
    };
    auto gidx = [&](int64_t line, int64_t p) { return AXIS == 0 ? line * A.nx + p : p * A.nx + line; };

    // 1. the tile: TC lines x HJF_ROW points (lines past the grid read line 0; they store nothing)
    if (AXIS == 0) {
        const int64_t L = line0 + wv < nlines ? line0 + wv : 0;
        for (int q = lane; q < HJF_ROW; q += 64) tile[TI(wv, q)] = u[gidx(L, wrap(q0 + q))];
    } else {
        for (int e = tid; e < TC * HJF_ROW; e += TC * 64) {
            const int q = e / TC, cc = e % TC;
            const int64_t L = line0 + cc < nlines ? line0 + cc : 0;
            tile[TI(cc, q)] = u[gidx(L, wrap(q0 + q))];
        }
    }
    __syncthreads();

    // 2. this lane's points t = 0..PPL-1 sit at tile points 3 + lane PPL + t; v[k] = tile point
    //    lane PPL + k, k = 0..PPL+5 (the stencil halo of 3 on either side)
    constexpr int PPL = HJF_PPL;
    double v[PPL + 6];
#pragma unroll
    for (int k = 0; k < PPL + 6; ++k) v[k] = tile[TI(wv, lane * PPL + k)];
    const double alpha = F.alpha[AXIS], d = F.d[AXIS];
    double JR[PPL], JL[PPL];
#pragma unroll
    for (int t = 0; t < PPL; ++t) {
        // J_R from the nodes x_{i-3} .. x_{i+1}, J_L from the mirror x_{i+3} .. x_{i-1}
        double sR[5], sL[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            sR[k] = v[t + k];
            sL[k] = v[t + 6 - k];
        }
        double oR[3], oL[3];
        if (MODE == HJ_LINEAR) {
#pragma unroll
            for (int r = 0; r < 3; ++r) oR[r] = oL[r] = Q.d[r];
        } else {
            wenoz(sR, Q.d, oR);
            wenoz(sL, Q.d, oL);
        }
        double jr = 0.0, jl = 0.0;
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            double qR = 0.0, qL = 0.0;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                qR = fma(Q.c[r][j], sR[r + j], qR);
                qL = fma(Q.c[r][j], sL[r + j], qL);
            }
            jr = fma(oR[r], qR, jr);
            jl = fma(oL[r], qL, jl);
        }
        JR[t] = jr;
        JL[t] = jl;
    }

    // 3. sweeps: lane totals, their scans across the wave (decay d^{PPL} a lane), then the re-sweep
    //    from the carry into the lane
    double fR = 0.0, fL = 0.0;
#pragma unroll
    for (int t = 0; t < PPL; ++t) fR = fma(d, fR, JR[t]);
#pragma unroll
    for (int t = PPL - 1; t >= 0; --t) fL = fma(d, fL, JL[t]);
#pragma unroll
    for (int s = 0; s < 6; ++s) {
        const int k = 1 << s;
        const double yR = __shfl_up(fR, k, 64), yL = __shfl_down(fL, k, 64);
        if (lane >= k) fR = fma(F.dscan[AXIS][s], yR, fR);
        if (lane + k < 64) fL = fma(F.dscan[AXIS][s], yL, fL);
    }
    double cR = __shfl_up(fR, 1, 64), cL = __shfl_down(fL, 1, 64);
    if (lane == 0) cR = 0.0;
    if (lane == 63) cL = 0.0;
    double IR[PPL];
#pragma unroll
    for (int t = 0; t < PPL; ++t) {
        cR = fma(d, cR, JR[t]);
        IR[t] = cR;
    }

    // 4. one-sided derivatives p- = alpha (u - I_R), p+ = -alpha (u - I_L), the x or y part of the
    //    numerical Hamiltonian, the time step from the lagged speed, and the new values
    const double c = state[HJ_S_C];
    const double dt = hj_dt(A, state);
    double m = 0.0, res[PPL];
#pragma unroll
    for (int t = PPL - 1; t >= 0; --t) {
        cL = fma(d, cL, JL[t]);
        const double ui = v[t + 3];
        const double pm = alpha * (ui - IR[t]), pp = -alpha * (ui - cL);
        const double pmean = 0.5 * (pm + pp);
        const double H = 0.5 * pmean * pmean + c * 0.5 * (pm - pp);
        res[t] = AXIS == 0 ? ui - dt * H : dt * H;
        const int64_t p = c0 - HJF_KW + lane * PPL + t;  // line point (before the chunk: window only)
        if (p >= c0 && p < c0 + HJF_C && p < n) m = fmax(m, fmax(fabs(pm), fabs(pp)));
    }
    if (line0 + wv >= nlines) m = 0.0;
    // (each wave reads and writes only its own line of the tile)
#pragma unroll
    for (int t = 0; t < PPL; ++t) tile[TI(wv, 3 + lane * PPL + t)] = res[t];
#pragma unroll
    for (int k = 32; k > 0; k >>= 1) m = fmax(m, __shfl_xor(m, k, 64));
    if (lane == 0) red[wv] = m;
    __syncthreads();

    // 5. stores of the chunk's points, along rows: x writes w = u - dt Hx, y writes u = w - dt Hy
    const int64_t cn = (c0 + HJF_C < n ? c0 + HJF_C : n) - c0;  // points of this chunk
    if (AXIS == 0) {
        if (line0 + wv < nlines)
            for (int j = lane; j < cn; j += 64) out[gidx(line0 + wv, c0 + j)] = tile[TI(wv, 3 + HJF_KW + j)];
    } else {
        for (int e = tid; e < TC * cn; e += TC * 64) {
            const int j = e / TC, cc = e % TC;
            if (line0 + cc < nlines) {
                const int64_t g = gidx(line0 + cc, c0 + j);
                out[g] = w_in[g] - tile[TI(cc, 3 + HJF_KW + j)];
            }
        }
    }
    if (tid == 0) {
        double M = 0.0;
        for (int k = 0; k < TC; ++k) M = fmax(M, red[k]);
        part[blockIdx.x] = M;
    }
}

// One block: reduce the per-block maxima (and the proposer statistics), then advance the state.
// mode 0: initialise (c = max, t = 0, counters = 0); mode 1: after an update (t += dt with the old c,
// then c = max).  1024 threads with four independent loads in flight each, so the reduction of the
// per-block partials is not one latency-bound walk; wave shuffles, then one exchange across waves.
constexpr int HJ_FIN_THREADS = 1024;
__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int s = 32; s > 0; s >>= 1) v = fmax(v, __shfl_down(v, s, 64));
    return v;
}
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int s = 32; s > 0; s >>= 1) v += __shfl_down(v, s, 64);
    return v;
}
__global__ void __launch_bounds__(HJ_FIN_THREADS) hj_finish_step(const double *__restrict__ part, int64_t nparts,
                                                                 const double *__restrict__ stats, int64_t nstats,
                                                                 const HjStepArgs A, double *__restrict__ state,
                                                                 int mode)
{
    constexpr int NT = HJ_FIN_THREADS, U = 4;
    __shared__ double red[4][NT / 64];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    double mu[U] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t i = tid; i < nparts; i += U * NT) {
#pragma unroll
        for (int k = 0; k < U; ++k)
            if (i + k * NT < nparts) mu[k] = fmax(mu[k], part[i + k * NT]);
    }
    double s0[U] = {0.0, 0.0, 0.0, 0.0}, s1[U] = {0.0, 0.0, 0.0, 0.0}, s2[U] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t i = tid; i < nstats; i += U * NT) {
#pragma unroll
        for (int k = 0; k < U; ++k)
            if (i + k * NT < nstats) {
                const double *q = stats + 3 * (i + k * NT);
                s0[k] += q[0];
                s1[k] += q[1];
                s2[k] += q[2];
            }
    }
    const double m = wave_max(fmax(fmax(mu[0], mu[1]), fmax(mu[2], mu[3])));
    const double t0 = wave_sum((s0[0] + s0[1]) + (s0[2] + s0[3]));
    const double t1 = wave_sum((s1[0] + s1[1]) + (s1[2] + s1[3]));
    const double t2 = wave_sum((s2[0] + s2[1]) + (s2[2] + s2[3]));
    if (lane == 0) {
        red[0][wv] = m;
        red[1][wv] = t0;
        red[2][wv] = t1;
        red[3][wv] = t2;
    }
    __syncthreads();
    if (tid == 0) {
        double M = 0.0, S0 = 0.0, S1 = 0.0, S2 = 0.0;
        for (int w = 0; w < NT / 64; ++w) {
            M = fmax(M, red[0][w]);
            S0 += red[1][w];
            S1 += red[2][w];
            S2 += red[3][w];
        }
        if (mode == 0) {
            state[HJ_S_C] = M;
            state[HJ_S_T] = 0.0;
            state[HJ_S_STEPS] = 0.0;
            state[HJ_S_FALLBACK] = 0.0;
            state[HJ_S_ERRSUM] = 0.0;
            state[HJ_S_JUDGED] = 0.0;
        } else {
            // steps past t_end (dt = 0) leave u and the state unchanged
            const double dt = hj_dt(A, state);
            if (dt > 0.0) {
                state[HJ_S_T] += dt;
                state[HJ_S_STEPS] += 1.0;
                state[HJ_S_C] = M;
                state[HJ_S_FALLBACK] += S0;
                state[HJ_S_ERRSUM] += S1;
                state[HJ_S_JUDGED] += S2;
            }
        }
    }
}

// ------------------------------------------------------------------------------------------
// Training samples: features and WENO-Z weights of the stencils of a field along one axis
// (both sides of every point: rows 2p (J_R) and 2p + 1 (J_L)).
// ------------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) hj_harvest(const double *__restrict__ u, const HjQuadArgs A,
                                                  float *__restrict__ X, float *__restrict__ Y)
{
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= A.nx * A.ny) return;
    const int64_t pj = p / A.nx, pi = p % A.nx;
    double v[7];
#pragma unroll
    for (int k = 0; k < 7; ++k) {
        int64_t idx;
        if (A.axis == 0) {
            int64_t i2 = pi + (k - 3);
            i2 = i2 < 0 ? i2 + A.nx : (i2 >= A.nx ? i2 - A.nx : i2);
            idx = pj * A.nx + i2;
        } else {
            int64_t j2 = pj + (k - 3);
            j2 = j2 < 0 ? j2 + A.ny : (j2 >= A.ny ? j2 - A.ny : j2);
            idx = j2 * A.nx + pi;
        }
        v[k] = u[idx];
    }
    for (int side = 0; side < 2; ++side) {
        double s[5], om[3];
        float f[MLP_IN];
#pragma unroll
        for (int k = 0; k < 5; ++k) s[k] = side == 0 ? v[k] : v[6 - k];
        stencil_features(s, f);
        wenoz(s, A.d, om);
        const int64_t row = 2 * p + side;
#pragma unroll
        for (int k = 0; k < MLP_IN; ++k) X[row * MLP_IN + k] = f[k];
#pragma unroll
        for (int r = 0; r < 3; ++r) Y[row * 3 + r] = (float)om[r];
    }
}

// ------------------------------------------------------------------------------------------
// Proposer inference and training.  Blocks of 256 threads, each wave a tile of 16 samples per
// step (samples beyond n are zero features and carry no loss).
// ------------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) mlp_forward(const float *__restrict__ P, const float *__restrict__ X,
                                                   float *__restrict__ Y, int64_t n)
{
    __shared__ float feat[4][16][MLP_IN];
    __shared__ float zo[4][16][4];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const MlpOperands o = mlp_load(P, lane);
    const MlpRowBias rb = mlp_row_bias(P, lane);
    const int64_t ntiles = (n + 15) / 16;
    const int64_t per_block = 4;
    for (int64_t t0 = (int64_t)blockIdx.x * per_block; t0 < ntiles; t0 += (int64_t)gridDim.x * per_block) {
        const int64_t tile = t0 + wv;
        // features of this wave's tile
        for (int e = lane; e < 16 * MLP_IN; e += 64) {
            const int64_t row = tile * 16 + e / MLP_IN;
            feat[wv][e / MLP_IN][e % MLP_IN] = (tile < ntiles && row < n) ? X[row * MLP_IN + e % MLP_IN] : 0.f;
        }
        __syncthreads();
        mlp_tile_infer(o, rb, feat[wv], zo[wv], lane);
        __syncthreads();
        if (lane < 16) {
            const int64_t row = tile * 16 + lane;
            if (tile < ntiles && row < n) {
                double om[3];
                softmax3(zo[wv][lane], om);
                Y[row * 3 + 0] = (float)om[0];
                Y[row * 3 + 1] = (float)om[1];
                Y[row * 3 + 2] = (float)om[2];
            }
        }
        __syncthreads();
    }
}

// Fused forward + backward of the loss mean_i sum_r (omega_ir - target_ir)^2 over a batch; each wave
// accumulates its gradient contributions and writes them to its slot of `partial` (MLP_NPARAM
// floats per wave) plus its summed squared error at partial[slot * MLP_NPARAM + MLP_NPARAM - 1 + 1]
// -- the slot holds MLP_NPARAM + 1 floats.
__global__ void __launch_bounds__(256) mlp_train_tile(const float *__restrict__ P, const float *__restrict__ X,
                                                      const float *__restrict__ Yt, int64_t n,
                                                      float *__restrict__ partial)
{
    __shared__ float feat[4][16][MLP_IN];
    __shared__ float hid[4][16][33];
    __shared__ float zo[4][16][4];
    __shared__ float keep[4][4][16][33];  // z1, h1 (bf16-valued), z2, h2 per wave
    __shared__ float gz[4][16][33];       // upstream gradient of the layer being processed
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int m = lane & 15, g = lane >> 4;
    const MlpOperands o = mlp_load(P, lane);
    auto bar = [] { __syncthreads(); };
    // gradient accumulators in MFMA result layout
    f32x4 gW3[2] = {};     // D[out 4g+j][unit 16t+m]  (M = out padded to 16, N = 32)
    f32x4 gW2[2][2] = {};  // [M-tile a][N-tile t]: D[unit 16a+4g+j][unit 16t+m]
    f32x4 gW1[2] = {};     // [M-tile a]: D[unit 16a+4g+j][feature m]
    float gb1[2] = {0.f, 0.f}, gb2[2] = {0.f, 0.f}, gb3 = 0.f, sq = 0.f;
    const int64_t ntiles = (n + 15) / 16;
    const float inv_n = 1.0f / (float)n;
    for (int64_t t0 = (int64_t)blockIdx.x * 4; t0 < ntiles; t0 += (int64_t)gridDim.x * 4) {
        const int64_t tile = t0 + wv;
        const bool tile_ok = tile < ntiles;
        for (int e = lane; e < 16 * MLP_IN; e += 64) {
            const int64_t row = tile * 16 + e / MLP_IN;
            feat[wv][e / MLP_IN][e % MLP_IN] = (tile_ok && row < n) ? X[row * MLP_IN + e % MLP_IN] : 0.f;
        }
        __syncthreads();
        mlp_tile_forward(o, feat[wv], hid[wv], zo[wv], keep[wv], lane, bar);
        // keep[1] = bf16(relu(z1)), keep[3] = bf16(relu(z2)): the operands the forward used
        for (int e = lane; e < 16 * 32; e += 64) {
            const int r = e >> 5, c = e & 31;
            const short h1 = f2bf(fmaxf(keep[wv][0][r][c], 0.f));
            const short h2 = f2bf(fmaxf(keep[wv][2][r][c], 0.f));
            keep[wv][1][r][c] = __uint_as_float((uint32_t)(uint16_t)h1 << 16);
            keep[wv][3][r][c] = __uint_as_float((uint32_t)(uint16_t)h2 << 16);
        }
        // output gradient: softmax Jacobian of 2 (om - y) / n
        if (lane < 16) {
            const int64_t row = tile * 16 + lane;
            float g3[3] = {0.f, 0.f, 0.f};
            if (tile_ok && row < n) {
                double om[3];
                softmax3(zo[wv][lane], om);
                double go[3], dot = 0.0;
                for (int r = 0; r < 3; ++r) {
                    const double e = om[r] - (double)Yt[row * 3 + r];
                    sq += (float)(e * e);
                    go[r] = 2.0 * e * (double)inv_n;
                    dot += go[r] * om[r];
                }
                for (int r = 0; r < 3; ++r) g3[r] = (float)(om[r] * (go[r] - dot));
            }
            for (int c = 0; c < 16; ++c) gz[wv][lane][c] = c < 3 ? g3[c] : 0.f;
        }
        __syncthreads();
        // dW3 += G3^T H2: A[out][sample] = G3[sample][out], B[sample][unit] = H2[sample][unit]
        {
            bf16x4 a;
#pragma unroll
            for (int j = 0; j < 4; ++j) a[j] = f2bf(gz[wv][4 * g + j][m]);
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                bf16x4 b;
#pragma unroll
                for (int j = 0; j < 4; ++j) b[j] = f2bf(keep[wv][3][4 * g + j][16 * t + m]);
                gW3[t] = mfma16(a, b, gW3[t]);
            }
        }
        if (lane < MLP_OUT)
            for (int r = 0; r < 16; ++r) gb3 += gz[wv][r][lane];
        // dH2 = G3 W3: A[sample][out] = G3, B[out][unit] = W3[out][unit] (rows >= 3 zero)
        f32x4 dh2[2];
        {
            bf16x4 a;
#pragma unroll
            for (int j = 0; j < 4; ++j) a[j] = f2bf(gz[wv][m][4 * g + j]);
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                bf16x4 b;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int k = 4 * g + j;
                    b[j] = k < MLP_OUT ? f2bf(P[MLP_W3 + k * MLP_H + 16 * t + m]) : (short)0;
                }
                const f32x4 zc = {0.f, 0.f, 0.f, 0.f};
                dh2[t] = mfma16(a, b, zc);
            }
        }
        __syncthreads();
        // G2 = dH2 * (z2 > 0) -> gz
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int r = 4 * g + j, c = 16 * t + m;
                gz[wv][r][c] = keep[wv][2][r][c] > 0.f ? dh2[t][j] : 0.f;
            }
        __syncthreads();
        for (int t = 0; t < 2; ++t)
            if (lane < 16)
                for (int r = 0; r < 16; ++r) gb2[t] += gz[wv][r][16 * t + lane];
        // dW2 += G2^T H1: A[unit a][sample] = G2[sample][unit], B[sample][unit'] = H1
        {
#pragma unroll
            for (int a_ = 0; a_ < 2; ++a_) {
                bf16x4 a;
#pragma unroll
                for (int j = 0; j < 4; ++j) a[j] = f2bf(gz[wv][4 * g + j][16 * a_ + m]);
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    bf16x4 b;
#pragma unroll
                    for (int j = 0; j < 4; ++j) b[j] = f2bf(keep[wv][1][4 * g + j][16 * t + m]);
                    gW2[a_][t] = mfma16(a, b, gW2[a_][t]);
                }
            }
        }
        // dH1 = G2 W2: A[sample][unit k] = G2, B[k][unit n] = W2[k][n]
        f32x4 dh1[2];
        {
            bf16x4 a[2];
#pragma unroll
            for (int s = 0; s < 2; ++s)
#pragma unroll
                for (int j = 0; j < 4; ++j) a[s][j] = f2bf(gz[wv][m][16 * s + 4 * g + j]);
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int s = 0; s < 2; ++s) {
                    bf16x4 b;
#pragma unroll
                    for (int j = 0; j < 4; ++j) b[j] = f2bf(P[MLP_W2 + (16 * s + 4 * g + j) * MLP_H + 16 * t + m]);
                    acc = mfma16(a[s], b, acc);
                }
                dh1[t] = acc;
            }
        }
        __syncthreads();
        // G1 = dH1 * (z1 > 0) -> gz
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int r = 4 * g + j, c = 16 * t + m;
                gz[wv][r][c] = keep[wv][0][r][c] > 0.f ? dh1[t][j] : 0.f;
            }
        __syncthreads();
        for (int t = 0; t < 2; ++t)
            if (lane < 16)
                for (int r = 0; r < 16; ++r) gb1[t] += gz[wv][r][16 * t + lane];
        // dW1 += G1^T X: A[unit][sample] = G1[sample][unit], B[sample][feature] = X (features < 8)
#pragma unroll
        for (int a_ = 0; a_ < 2; ++a_) {
            bf16x4 a, b;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                a[j] = f2bf(gz[wv][4 * g + j][16 * a_ + m]);
                b[j] = m < MLP_IN ? f2bf(feat[wv][4 * g + j][m]) : (short)0;
            }
            gW1[a_] = mfma16(a, b, gW1[a_]);
        }
        __syncthreads();
    }
    // write this wave's partial gradient (slot = global wave index)
    float *dst = partial + ((int64_t)blockIdx.x * 4 + wv) * (MLP_NPARAM + 1);
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int out = 4 * g + j;
            if (out < MLP_OUT) dst[MLP_W3 + out * MLP_H + 16 * t + m] = gW3[t][j];
        }
#pragma unroll
    for (int a_ = 0; a_ < 2; ++a_)
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int j = 0; j < 4; ++j) dst[MLP_W2 + (16 * a_ + 4 * g + j) * MLP_H + 16 * t + m] = gW2[a_][t][j];
#pragma unroll
    for (int a_ = 0; a_ < 2; ++a_)
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (m < MLP_IN) dst[MLP_W1 + (16 * a_ + 4 * g + j) * MLP_IN + m] = gW1[a_][j];
    if (lane < 16) {
        dst[MLP_B1 + lane] = gb1[0];
        dst[MLP_B1 + 16 + lane] = gb1[1];
        dst[MLP_B2 + lane] = gb2[0];
        dst[MLP_B2 + 16 + lane] = gb2[1];
    }
    if (lane < MLP_OUT) dst[MLP_B3 + lane] = gb3;
    // squared error of this wave's samples (lanes 0..15 hold them)
    __shared__ float sqs[256];
    sqs[tid] = sq;
    __syncthreads();
    if (lane == 0) {
        float s = 0.f;
        for (int k = 0; k < 16; ++k) s += sqs[wv * 64 + k];
        dst[MLP_NPARAM] = s;
    }
}

// grad[k] = sum over slots of partial[slot][k] (k < MLP_NPARAM); loss = sum of the squared errors / n
__global__ void __launch_bounds__(256) mlp_reduce_grads(const float *__restrict__ partial, int64_t nslots, int64_t n,
                                                        float *__restrict__ grad, float *__restrict__ loss)
{
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k > MLP_NPARAM) return;
    double s = 0.0;
    for (int64_t i = 0; i < nslots; ++i) s += (double)partial[i * (MLP_NPARAM + 1) + k];
    if (k < MLP_NPARAM)
        grad[k] = (float)s;
    else
        loss[0] = (float)(s / (double)n);
}

// Adam (Kingma & Ba) on the FP32 master parameters; t = step number (>= 1).
// Adam (Kingma & Ba) in FP32.  The constants b1, 1 - b1, b2, 1 - b2 and the bias corrections
// 1 / (1 - b^t) are formed in FP64 on the host and rounded once: 1 - fl32(0.999) alone is 1.3e-5
// away from 0.001.
__global__ void __launch_bounds__(256) mlp_adam(float *__restrict__ P, const float *__restrict__ grad,
                                                float *__restrict__ M, float *__restrict__ V, float lr, float b1,
                                                float omb1, float b2, float omb2, float c1, float c2, float eps)
{
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= MLP_NPARAM) return;
    const float gk = grad[k];
    const float mk = b1 * M[k] + omb1 * gk;
    const float vk = b2 * V[k] + omb2 * gk * gk;
    M[k] = mk;
    V[k] = vk;
    const float mh = mk * c1;
    const float vh = vk * c2;
    P[k] = P[k] - lr * mh / (sqrtf(vh) + eps);
}

// ------------------------------------------------------------------------------------------
// Launchers
// ------------------------------------------------------------------------------------------
hipError_t launch_hj_weno_quad(int mode, const double *u, double *JL, double *JR, const HjQuadArgs &A,
                               const float *P, double *stats, hipStream_t st)
{
    const int64_t npts = A.nx * A.ny;
    const dim3 grid((unsigned)((npts + 255) / 256));
    if (mode == HJ_LINEAR)
        hipLaunchKernelGGL(hj_weno_quad<HJ_LINEAR>, grid, dim3(256), 0, st, u, JL, JR, A, P, stats);
    else if (mode == HJ_WENOZ)
        hipLaunchKernelGGL(hj_weno_quad<HJ_WENOZ>, grid, dim3(256), 0, st, u, JL, JR, A, P, stats);
    else
        hipLaunchKernelGGL(hj_weno_quad<HJ_LEARNED>, grid, dim3(256), 0, st, u, JL, JR, A, P, stats);
    return hipGetLastError();
}

hipError_t launch_hj_update(double *u, const double *DmX, const double *DpX, const double *DmY, const double *DpY,
                            const HjStepArgs &A, const double *state, double *part, hipStream_t st)
{
    const dim3 grid((unsigned)((A.npts + 255) / 256));
    hipLaunchKernelGGL(hj_update, grid, dim3(256), 0, st, u, DmX, DpX, DmY, DpY, A, state, part);
    return hipGetLastError();
}

hipError_t launch_hj_init_speed(const double *u, const HjStepArgs &A, double *part, hipStream_t st)
{
    const dim3 grid((unsigned)((A.npts + 255) / 256));
    hipLaunchKernelGGL(hj_init_speed, grid, dim3(256), 0, st, u, A, part);
    return hipGetLastError();
}

hipError_t launch_hj_finish(const double *part, int64_t nparts, const double *stats, int64_t nstats,
                            const HjStepArgs &A, double *state, int mode, hipStream_t st)
{
    hipLaunchKernelGGL(hj_finish_step, dim3(1), dim3(HJ_FIN_THREADS), 0, st, part, nparts, stats, nstats, A, state, mode);
    return hipGetLastError();
}

constexpr int HJF_TCX = 4, HJF_TCY = 16;

int64_t hj_fused_blocks(int64_t nx, int64_t ny, int axis)
{
    const int64_t n = axis == 0 ? nx : ny, nlines = axis == 0 ? ny : nx;
    const int TC = axis == 0 ? HJF_TCX : HJF_TCY;
    return ((nlines + TC - 1) / TC) * ((n + HJF_C - 1) / HJF_C);
}

hipError_t launch_hj_fused_pass(int axis, int weights, const double *u, const double *w_in, double *out,
                                const HjQuadArgs &Q, const HjFusedArgs &F, const HjStepArgs &A, const double *state,
                                double *part, hipStream_t st)
{
    const dim3 grid((unsigned)hj_fused_blocks(A.nx, A.ny, axis));
    if (axis == 0) {
        if (weights == HJ_LINEAR)
            hipLaunchKernelGGL((hj_fused_pass<0, HJF_TCX, HJ_LINEAR>), grid, dim3(HJF_TCX * 64), 0, st, u, w_in, out, Q, F,
                               A, state, part);
        else
            hipLaunchKernelGGL((hj_fused_pass<0, HJF_TCX, HJ_WENOZ>), grid, dim3(HJF_TCX * 64), 0, st, u, w_in, out, Q, F,
                               A, state, part);
    } else {
        if (weights == HJ_LINEAR)
            hipLaunchKernelGGL((hj_fused_pass<1, HJF_TCY, HJ_LINEAR>), grid, dim3(HJF_TCY * 64), 0, st, u, w_in, out, Q, F,
                               A, state, part);
        else
            hipLaunchKernelGGL((hj_fused_pass<1, HJF_TCY, HJ_WENOZ>), grid, dim3(HJF_TCY * 64), 0, st, u, w_in, out, Q, F,
                               A, state, part);
    }
    return hipGetLastError();
}

hipError_t launch_hj_harvest(const double *u, const HjQuadArgs &A, float *X, float *Y, hipStream_t st)
{
    const int64_t npts = A.nx * A.ny;
    hipLaunchKernelGGL(hj_harvest, dim3((unsigned)((npts + 255) / 256)), dim3(256), 0, st, u, A, X, Y);
    return hipGetLastError();
}

int64_t mlp_train_slots(int64_t n)
{
    const int64_t ntiles = (n + 15) / 16;
    int64_t blocks = (ntiles + 3) / 4;
    if (blocks > 1024) blocks = 1024;
    return blocks * 4;
}

hipError_t launch_mlp_forward(const float *P, const float *X, float *Y, int64_t n, hipStream_t st)
{
    const int64_t ntiles = (n + 15) / 16;
    int64_t blocks = (ntiles + 3) / 4;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(mlp_forward, dim3((unsigned)blocks), dim3(256), 0, st, P, X, Y, n);
    return hipGetLastError();
}

hipError_t launch_mlp_grad(const float *P, const float *X, const float *Y, int64_t n, float *partial, float *grad,
                           float *loss, hipStream_t st)
{
    const int64_t slots = mlp_train_slots(n);
    hipLaunchKernelGGL(mlp_train_tile, dim3((unsigned)(slots / 4)), dim3(256), 0, st, P, X, Y, n, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(mlp_reduce_grads, dim3((MLP_NPARAM + 1 + 255) / 256), dim3(256), 0, st, partial, slots, n, grad,
                       loss);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(float *P, const float *grad, float *M, float *V, int t, float lr, hipStream_t st)
{
    const double b1 = 0.9, b2 = 0.999;
    const float c1 = (float)(1.0 / (1.0 - std::pow(b1, (double)t)));
    const float c2 = (float)(1.0 / (1.0 - std::pow(b2, (double)t)));
    hipLaunchKernelGGL(mlp_adam, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, st, P, grad, M, V, lr, (float)b1,
                       (float)(1.0 - b1), (float)b2, (float)(1.0 - b2), c1, c2, 1e-8f);
    return hipGetLastError();
}

}  // namespace scx
