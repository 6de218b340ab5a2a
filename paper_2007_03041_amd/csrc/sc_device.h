// sc_device.h -- internal argument blocks shared by the host launchers and the HIP kernels of the
// successive-convolution library.  Not part of the public ABI (include/sc.h is).
#pragma once
#include <stdint.h>

namespace scx {

constexpr int WAVE = 64;        // CDNA wavefront width
constexpr int MAXS = 16;        // largest per-thread segment length any kernel variant uses
constexpr int MAXWIN = MAXS + 6; // largest register window (segment + stencil halo)

// One operator application inside a line pass.  Everything here is per (axis, operator, alpha,
// kernel variant) and uniform across the launch, so it travels as a kernel argument and lives in
// scalar registers.
struct OpArgs {
    double wR[6];           // interior J_R weights on window offsets 0..order-1; J_L uses the mirror
    // The segment totals of the two sweeps are linear in the segment's window of S + order operand
    // values: sum_t d^{S-1-t} J_R[t] = sum_w kR[w] win[w] and sum_t d^t J_L[t] = sum_w kL[w] win[w].
    double kR[MAXWIN];
    double kL[MAXWIN];
    double d;               // e^{-nu}, nu = alpha dx
    double nu;
    double dpow[MAXS + 1];  // d^t, t = 0..S
    double dseg[12];        // d^{S 2^j}: decay across 2^j whole segments
    double dpart;           // d^{S GW}: decay across one wave-part of segments
    double dchunk;          // d^{C}: decay across one whole chunk
    double dlp_full;        // decay from the start of the last real wave-part of a tile to the tile's
    double dlp_last;        //   last real point: full tile (or whole line) / last chunk of a line
    double inv1mmu;         // 1 / (1 - mu), mu = e^{-alpha (b - a)}
    double mu;
    double scale;           // result multiplier
    int32_t op;             // 0 = L_L^{-1}, 1 = L_R^{-1}, 2 = L_0^{-1}
    int32_t k;              // 0: result is L^{-1}[v]; k >= 1: result is sum_{p=1..k} D^p[v]
};

struct PassArgs {
    const void *v;          // operand
    const void *acc;        // acc_mode 2: added to the result (may equal out)
    void *out;
    const double *g;        // Dirichlet values, 2 per line, or nullptr (= 0)
    double *agg;            // chunked: per (op, line, chunk) [fwd total, bwd total, J_R[0]]
    const double *carry;    // chunked: per (op, line, chunk) [fwd carry in, bwd carry in], then per
                            // (op, line) [A', B']
    int64_t n;              // points per line
    int64_t stride;         // element stride along the line
    int64_t nlines;
    int64_t ncells;         // n (periodic) or n - 1 (Dirichlet)
    int64_t nchunks;
    int32_t bc;             // 0 periodic, 1 Dirichlet
    int32_t acc_mode;       // 0 none, 1 add the operand v, 2 add acc
    int32_t nops;           // 1 or 2
    int32_t pad_;
    // Dirichlet ends: the one-sided stencils of the order/2 points nearest an end integrate the
    // interpolant through the `order` end values; extending the line by that interpolant's values
    // at m = 1..order/2 points beyond the end makes the centred interior stencil integrate the same
    // polynomial.  ext[m-1][j] = l_j(-m), the Lagrange basis on nodes 0..order-1 (the right end
    // uses the mirrored nodes).
    double ext[3][6];
    OpArgs ops[2];
};

// Tile shape of a kernel variant.
struct Variant {
    int S;       // points per thread segment
    int TC;      // lines per tile
    bool contig; // lanes along the line (contiguous axis) or across lines (strided axis)
    int NT;      // threads per workgroup
    int G() const { return NT / TC; }
    int C() const { return G() * S; }
    int GW() const { return contig ? (G() < WAVE ? G() : WAVE) : WAVE / TC; }
};

}  // namespace scx
