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
    double dchunk_last;     // decay across the last chunk of a line (its real length)
    double dlp_full;        // decay from the start of the last real wave-part of a tile to the tile's
    double dlp_last;        //   last real point: full tile (or whole line) / last chunk of a line
    double inv1mmu;         // 1 / (1 - mu), mu = e^{-alpha (b - a)}
    double mu;
    double dir2inv;         // 2 / (1 - mu^2): the 2x2 end-value system of L_0 on Dirichlet lines
    double scale;           // result multiplier
    int32_t op;             // 0 = L_L^{-1}, 1 = L_R^{-1}, 2 = L_0^{-1}
    int32_t k;              // 0: result is L^{-1}[v]; k >= 1: result is sum_{p=1..k} D^p[v]
    // FP32 passes: the per-point coefficients rounded once from the FP64 values above, and the
    // in-wave scan decays split as hi + lo (hi = fl32(d^{S 2^j}), lo = fl32(d^{S 2^j} - hi))
    float wRf[6];
    float kRf[MAXWIN];
    float kLf[MAXWIN];
    float df;
    float dlo;              // d - fl32(d): the FP32 sweeps apply d as df + dlo
    float dpowf[MAXS + 1];
    float dseg_hi[12];
    float dseg_lo[12];
};

struct PassArgs {
    const void *v;          // operand
    const void *acc;        // acc_mode bit 1: aw acc added to the result (may equal out)
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
    int32_t acc_mode;       // bit 0: add vw v (the operand); bit 1: add aw acc
    int32_t nops;           // 1 or 2
    int32_t fuse_carry;     // chunked apply: each tile forms its chunk carries from the aggregates
    uint32_t *sync;         // single-pass chunked launches: the tile claim counter
    int32_t spin_limit;     // single-pass: polls of the other chunks' totals before a tile gives up
    int32_t nn_cpb;         // > 0: nearest-neighbour virtual blocks of this many chunks (carry launch
                            // and apply); 0: exact carries over the whole line
    int32_t win_k;          // > 0: windowed apply of chunked one-line tiles: the carries are the
                            // sweeps over the win_k points before and after the chunk
    int32_t pad_;
    double vw, aw;          // weights of the operand and of acc in the result (acc_mode)
    // Dirichlet ends: the one-sided stencils of the order/2 points nearest an end integrate the
    // interpolant through the `order` end values; extending the line by that interpolant's values
    // at m = 1..order/2 points beyond the end makes the centred interior stencil integrate the same
    // polynomial.  ext[m-1][j] = l_j(-m), the Lagrange basis on nodes 0..order-1 (the right end
    // uses the mirrored nodes).
    double ext[3][6];
    OpArgs ops[2];
};

// One instance of a batched pass: its argument block (array pointers unused) and the element offsets
// of its arrays in the batch buffers: operand and result at v_off, Dirichlet values at g_off (< 0:
// zero), chunk aggregates and carries at agg_off / carry_off doubles into the workspace.
struct BatchArgs {
    PassArgs a;
    int64_t v_off;
    int64_t g_off;
    int64_t agg_off;
    int64_t carry_off;
};

// One work item of a batched launch: tile `tile` (line tile, times chunks for chunked passes) of
// instance `item`.
struct BatchWork {
    int32_t item;
    int32_t pad_;
    int64_t tile;
};

// Tile shape of a kernel variant.
struct Variant {
    int S;       // points per thread segment
    int TC;      // lines per tile
    bool contig; // lanes along the line (contiguous axis) or across lines (strided axis)
    int NT;      // threads per workgroup
    constexpr int G() const { return NT / TC; }
    constexpr int C() const { return G() * S; }
    constexpr int GW() const { return contig ? (G() < WAVE ? G() : WAVE) : WAVE / TC; }
    constexpr int NP() const { return G() / GW(); }
    // static LDS of the line pass with this shape: the tile (line stride as in the kernel), line bases,
    // four carry tables, J_R(x_0), boundary terms and two decay tables
    constexpr int lds_bytes(int elem, int order, int nops) const
    {
        const int W = C() + order;
        const int LS = (!contig && elem == 8) ? (((W + 31) & ~31) + 1) : ((W + W / S + 1) | 1);
        return TC * LS * elem + TC * 8 + 4 * nops * TC * NP() * 8 + nops * TC * 8 + nops * TC * 3 * 8 +
               nops * (GW() + 1) * 8 + nops * (NP() + 1) * 8;
    }
};

constexpr int LDS_LIMIT = 160 * 1024;  // LDS per workgroup on gfx950

// The kernel variants: X(id, S, TC, CONTIG, NT).  A variant is built for an element type only where
// its LDS fits (Variant::lds_bytes with two operators).
#define SC_VARIANTS(X)             \
    X(0, 16, 16, true, 256)        \
    X(1, 16, 4, true, 256)         \
    X(2, 16, 1, true, 256)         \
    X(3, 16, 1, true, 512)         \
    X(4, 16, 16, false, 256)       \
    X(5, 16, 16, false, 512)       \
    X(6, 16, 16, false, 1024)      \
    X(7, 16, 4, false, 1024)       \
    X(8, 8, 16, false, 1024)       \
    X(9, 8, 1, true, 512)          \
    X(10, 16, 8, true, 256)        \
    X(11, 16, 32, false, 512)      \
    X(12, 16, 32, false, 1024)     \
    X(13, 8, 32, false, 1024)      \
    X(14, 16, 1, true, 64)         \
    X(15, 16, 1, true, 1024)       \
    X(16, 16, 2, true, 256)

}  // namespace scx
