// sc_device.h -- internal argument blocks shared by the host launchers and the HIP kernels of the
// successive-convolution library.  Not part of the public ABI (include/sc.h is).
#pragma once
#include <stdint.h>

namespace scx {

constexpr int WAVE = 64;   // CDNA wavefront width
constexpr int MAXS = 16;   // largest per-thread segment length any kernel variant uses

// One operator application inside a line pass.  Everything here is per (axis, operator, alpha)
// and uniform across the launch, so it travels as a kernel argument (scalar registers).
struct OpArgs {
    double wR[6];          // interior J_R weights on window offsets 0..order-1; J_L uses the mirror
    double bRl[2][6];      // Dirichlet one-sided J_R weights at i = 1 .. H-1   (nodes 0..order-1)
    double bRr[2][6];      // Dirichlet one-sided J_R weights at i = n-H+1 .. n-1 (nodes n-order..n-1)
    double bLl[2][6];      // Dirichlet one-sided J_L weights at i = 0 .. H-2   (nodes 0..order-1)
    double bLr[2][6];      // Dirichlet one-sided J_L weights at i = n-H .. n-2 (nodes n-order..n-1)
    double d;              // e^{-nu}, nu = alpha dx
    double nu;
    double dpow[MAXS + 1]; // d^t, t = 0..S
    double dseg[8];        // d^{S 2^j}: decay across 2^j whole segments
    double dpart;          // d^{S GW}: decay across one wave-part of segments
    double dchunk;         // d^{C}: decay across one whole chunk
    double inv1mmu;        // 1 / (1 - mu), mu = e^{-alpha (b - a)}
    double mu;
    double scale;          // result multiplier
    int32_t op;            // 0 = L_L^{-1}, 1 = L_R^{-1}, 2 = L_0^{-1}
    int32_t k;             // 0: result is L^{-1}[v]; k >= 1: result is sum_{p=1..k} D^p[v]
};

struct PassArgs {
    const void *v;         // operand
    const void *acc;       // acc_mode 2: added to the result (may equal out)
    void *out;
    const double *g;       // Dirichlet values, 2 per line, or nullptr (= 0)
    double *agg;           // chunked: per (op, line, chunk) [fwd total, bwd total, J_R[0]]
    const double *carry;   // chunked: per (op, line, chunk) [fwd carry in, bwd carry in], then per
                           // (op, line) [A', B']
    int64_t n;             // points per line
    int64_t stride;        // element stride along the line
    int64_t nlines;
    int64_t ncells;        // n (periodic) or n - 1 (Dirichlet)
    int64_t nchunks;
    int32_t bc;            // 0 periodic, 1 Dirichlet
    int32_t acc_mode;      // 0 none, 1 add the operand v, 2 add acc
    int32_t nops;          // 1 or 2
    int32_t pad_;
    OpArgs ops[2];
};

}  // namespace scx
