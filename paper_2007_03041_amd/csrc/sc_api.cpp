// sc_api.cpp -- the C ABI of include/sc.h: validation, coefficient set-up, pass planning and the
// time-step driver.  All arithmetic on array data happens in the HIP kernels (sc_kernels.hip);
// this file only prepares per-axis constants (quadrature weights, decay powers, mu) in FP64 and
// enqueues launches on the caller's stream.
#include "sc.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <limits>
#include <mutex>
#include <string>
#include <vector>

#include "sc_device.h"
#include "sc_host.h"
#include "sc_launch.h"

thread_local std::string g_err;

namespace scx {
namespace host {

std::mutex g_tmu;
bool g_timing = false;
std::vector<std::string> g_timing_only;
std::vector<TimedLaunch> g_records;
std::vector<std::pair<hipEvent_t, hipEvent_t>> g_pool;
size_t g_pool_used = 0;

sc_status fail(sc_status s, const std::string &msg)
{
    g_err = msg;
    return s;
}

// ------------------------------------------------------------------------------------------
// grid helpers
// ------------------------------------------------------------------------------------------

// Tile index arithmetic along a line is 32-bit (a chunk start plus a halo and a thread offset).
constexpr int64_t kMaxLine = (int64_t(1) << 31) - 65536;

sc_status check_grid(const sc_grid *g)
{
    if (!g) return fail(SC_ERR_ARG, "grid is NULL");
    if (g->ndim < 1 || g->ndim > 3) return fail(SC_ERR_ARG, "ndim must be 1, 2 or 3");
    if (g->dtype != SC_F64 && g->dtype != SC_F32_MIXED) return fail(SC_ERR_ARG, "unknown dtype");
    int64_t total = 1;
    for (int e = 0; e < g->ndim; ++e) {
        if (g->n[e] < 1) return fail(SC_ERR_SHAPE, "n must be >= 1 on every axis");
        if (g->n[e] > kMaxLine) return fail(SC_ERR_SHAPE, "more than 2^31 - 2^16 points on one axis");
        if (g->bc[e] != SC_BC_PERIODIC && g->bc[e] != SC_BC_DIRICHLET) return fail(SC_ERR_ARG, "unknown bc");
        if (!(g->hi[e] > g->lo[e]) || !std::isfinite(g->hi[e] - g->lo[e]))
            return fail(SC_ERR_ARG, "each axis needs lo < hi");
        if (total > (int64_t(1) << 40) / g->n[e]) return fail(SC_ERR_SHAPE, "array too large");
        total *= g->n[e];
    }
    return SC_OK;
}

Axis axis_of(const sc_grid *g, int dim)
{
    Axis a;
    a.n = g->n[dim];
    a.stride = 1;
    for (int e = 0; e < dim; ++e) a.stride *= g->n[e];
    a.total = 1;
    for (int e = 0; e < g->ndim; ++e) a.total *= g->n[e];
    a.nlines = a.total / a.n;
    a.bc = g->bc[dim];
    a.ncells = a.bc == SC_BC_PERIODIC ? a.n : a.n - 1;
    a.len = g->hi[dim] - g->lo[dim];
    a.dx = a.len / (double)a.ncells;
    return a;
}

size_t elem_bytes(const sc_grid *g) { return g->dtype == SC_F64 ? 8 : 4; }

size_t round256(size_t b) { return (b + 255) & ~size_t(255); }

bool overlap(const void *a, const void *b, size_t bytes)
{
    const char *x = (const char *)a, *y = (const char *)b;
    return x < y + bytes && y < x + bytes;
}

// Kernel variant for a line pass along an axis of n points (contiguous or strided) with elements
// of `elem` bytes.  The choice can be overridden for tuning with SC_VARIANT_CONTIG /
// SC_VARIANT_STRIDED (variant ids).
int pick_variant(bool contig, int64_t n, int elem)
{
    const char *env = std::getenv(contig ? "SC_VARIANT_CONTIG" : "SC_VARIANT_STRIDED");
    if (env && *env) {
        const int id = std::atoi(env);
        if (scx::variant_built(id, elem) && scx::variant(id).contig == contig) return id;
    }
    if (contig) {
        if (n <= 256) return 0;   // 16 lines x 256
        if (n <= 512) return 10;  // 8 lines x 512
        if (n <= 1024) return 1;  // 4 lines x 1024
        if (n <= 2048) return 16; // 2 lines x 2048
        if (n <= 4096) return 2;  // 1 line x 4096
        return 3;                 // 1 line x 8192; longer lines chunked
    }
    if (elem == 4) {
        // 32 adjacent float lines = 128-byte row segments
        if (n <= 256) return 11;
        return 12;  // 32 lines x 512; longer lines chunked
    }
    if (n <= 256) return 4;
    // 16 lines x 512 (two workgroups per CU); longer lines chunked, their carries formed inside the
    // apply launch up to 16 chunks
    if (n <= 8192) return 5;
    return 6;  // 16 lines x 1024
}

// SC_PIPE=0: never the pipelined strided form; SC_PIPE=1: wherever its shape conditions hold;
// unset: where it measured faster (see run_pass)
int pipe_mode()
{
    const char *env = std::getenv("SC_PIPE");
    if (env && env[0] == '0') return 0;
    if (env && env[0] == '1') return 1;
    return 2;
}

// decay from the start of the last real wave-part of a tile to the tile's last real point
double last_part_decay(double nu, int64_t n_loc, const scx::Variant &V)
{
    const int64_t span = (int64_t)V.S * V.GW();
    const int64_t part_last = ((n_loc - 1) / V.S) / V.GW();
    return std::exp(-nu * (double)(n_loc - part_last * span));
}

// Per-(axis, operator, alpha) constants for the variant chosen for the pass.
void fill_op(scx::OpArgs *P, int op, int order, double alpha, const Axis &ax, int vid, double scale, int k, int identity)
{
    std::memset(P, 0, sizeof(*P));
    const scx::Variant &V = scx::variant(vid);
    const int H = order / 2;
    const double nu = alpha * ax.dx;
    int eta[8];
    // interior: window offset j <-> node x_{i-H+j} <-> eta = H - j (J_R); J_L uses the mirror
    for (int j = 0; j < order; ++j) eta[j] = H - j;
    if (identity) {
        // the operand is the local integral itself: J_R[i] = v[i] and, by the mirror layout, J_L[i] = v[i]
        for (int j = 0; j < order; ++j) P->wR[j] = (j == H) ? 1.0 : 0.0;
    } else {
        scx::quad_weights(nu, order, eta, P->wR);
    }
    const int S = V.S;
    // segment totals as linear functionals of the window (S + order values):
    //   sum_t d^{S-1-t} J_R[t] = sum_w kR[w] win[w],  J_R[t] = sum_j wR[j] win[t+j]
    //   sum_t d^t J_L[t]       = sum_w kL[w] win[w],  J_L[t] = sum_j wR[order-1-j] win[t+1+j]
    for (int w = 0; w < S + order; ++w) {
        double kr = 0.0, kl = 0.0;
        for (int j = 0; j < order; ++j) {
            const int tr = w - j;
            if (tr >= 0 && tr < S) kr += P->wR[j] * std::exp(-nu * (double)(S - 1 - tr));
            const int tl = w - 1 - j;
            if (tl >= 0 && tl < S) kl += P->wR[order - 1 - j] * std::exp(-nu * (double)tl);
        }
        P->kR[w] = kr;
        P->kL[w] = kl;
    }
    const int64_t C = V.C();
    const int64_t nch = (ax.n + C - 1) / C;
    P->d = std::exp(-nu);
    P->df = (float)P->d;
    P->dlo = (float)(P->d - (double)P->df);
    P->nu = nu;
    for (int t = 0; t <= scx::MAXS; ++t) P->dpow[t] = std::exp(-nu * t);
    for (int j = 0; j < 12; ++j) P->dseg[j] = std::exp(-nu * (double)S * (double)(1 << j));
    for (int j = 0; j < order; ++j) P->wRf[j] = (float)P->wR[j];
    for (int w = 0; w < scx::MAXWIN; ++w) {
        P->kRf[w] = (float)P->kR[w];
        P->kLf[w] = (float)P->kL[w];
    }
    for (int t = 0; t <= scx::MAXS; ++t) P->dpowf[t] = (float)P->dpow[t];
    for (int j = 0; j < 12; ++j) {
        P->dseg_hi[j] = (float)P->dseg[j];
        P->dseg_lo[j] = (float)(P->dseg[j] - (double)P->dseg_hi[j]);
    }
    P->dpart = std::exp(-nu * (double)S * (double)V.GW());
    P->dchunk = std::exp(-nu * (double)C);
    P->dchunk_last = std::exp(-nu * (double)(ax.n - (nch - 1) * C));
    P->dlp_full = last_part_decay(nu, std::min<int64_t>(ax.n, C), V);
    P->dlp_last = last_part_decay(nu, ax.n - (nch - 1) * C, V);
    const double x = nu * (double)ax.ncells;  // alpha (b - a)
    P->mu = std::exp(-x);
    P->inv1mmu = 1.0 / (-std::expm1(-x));
    P->dir2inv = 2.0 / (1.0 - P->mu * P->mu);
    P->scale = scale;
    P->op = op;
    P->k = k;
}

// Lagrange basis on nodes 0..order-1 evaluated at -m, m = 1..order/2: the values that extend a
// Dirichlet line beyond its ends by the interpolant of its `order` end values.
void fill_ext(scx::PassArgs *a, int order)
{
    for (int m = 1; m <= order / 2; ++m)
        for (int j = 0; j < order; ++j) {
            double l = 1.0;
            for (int q = 0; q < order; ++q)
                if (q != j) l *= (double)(-m - q) / (double)(j - q);
            a->ext[m - 1][j] = l;
        }
}


size_t chunk_ws_bytes(int64_t nlines, int64_t nchunks, int nops)
{
    if (nchunks <= 1) return 0;
    const int64_t ent = (int64_t)nops * nlines * nchunks;
    return round256(sizeof(double) * (size_t)(3 * ent)) +
           round256(sizeof(double) * (size_t)(2 * ent + 2 * (int64_t)nops * nlines));
}

int64_t chunk_points(const Axis &ax, int elem) { return scx::variant(pick_variant(ax.stride == 1, ax.n, elem)).C(); }

int64_t nchunks_for(const Axis &ax, int elem)
{
    const int64_t C = chunk_points(ax, elem);
    return (ax.n + C - 1) / C;
}

// chunked passes with at most this many chunks per line form their carries inside the apply launch
constexpr int64_t kFuseCarryChunks = 16;
// ... and with at most this many run as one single-pass launch (the gathered totals sit in registers)
constexpr int64_t kSingleChunks = 8;

// Windowed chunk carries (chunked contiguous one-line tiles of one operator): the carries into a
// chunk are the sweeps over the K points on either side of it, K = ceil(60 ln 2 / nu), so that the
// dropped remainder is below 2^-60 of the carry.  Used where K <= 128 and the first and last chunks
// are longer than K plus the stencil (the end constants then act on their own chunks only, and
// Dirichlet windows stay inside the line).  Returns K, or 0 where the exact carries are taken.
// SC_WINDOW=0 always takes the exact carries.
int window_k(const scx::PassArgs &a, int order, const scx::Variant &V, bool multi)
{
    const char *env = std::getenv("SC_WINDOW");
    if (env && env[0] == '0') return 0;
    if (!V.contig || V.TC != 1 || a.nops != 1 || multi || a.nchunks < 2 || a.stride != 1) return 0;
    const double nu = a.ops[0].nu;
    const double kd = std::ceil(60.0 * std::log(2.0) / nu);
    if (!(kd <= 128.0)) return 0;
    const int64_t K = (int64_t)kd;
    const int64_t C = V.C();
    const int64_t last = a.n - (a.nchunks - 1) * C;
    if (C < K + order + 1 || last < K + order + 1) return 0;
    return (int)K;
}

// SC_SINGLE=1 selects the single-read form for chunked passes of at most kSingleChunks chunks.  It
// is not the default: at 4096^2 FP64 its y pass measured slower than the aggregate + apply launches
// (one operator 0.095 vs 0.089 ms; the advection-diffusion pair 0.097 vs 0.096 ms), because a tile's
// wait for its line's other chunk totals (published and polled at device scope, across the chips'
// separate L2 caches) costs more than the second read of the field.
bool single_pass_enabled()
{
    const char *env = std::getenv("SC_SINGLE");
    return env && env[0] == '1';
}

// polls of the other chunks' totals before a single-pass tile gives up and writes NaN (SC_SPIN_LIMIT;
// each poll sleeps about 128 cycles, so the default bound is about a quarter second).  A negative
// value -m makes every tile ignore the published totals and give up after m polls: a host-side way
// for tests to exercise the give-up path without any wait that cannot end.
int spin_limit()
{
    const char *env = std::getenv("SC_SPIN_LIMIT");
    if (env && *env) {
        const long v = std::strtol(env, nullptr, 10);
        if (v > -(1L << 30) && v < (1L << 30)) return (int)v;
    }
    return 1 << 22;
}

// One pass along `dim`: out = acc_term + sum_ops scale * result(op).
sc_status run_pass(const sc_grid *g, int dim, int order, const OpSpec *ops, int nops, const void *v,
                   const void *acc, int acc_mode, void *out, const double *dg, char *wsp, size_t ws_bytes,
                   hipStream_t st, int64_t nn_cpb, double vw, double aw)
{
    const Axis ax = axis_of(g, dim);
    const int elem = (int)elem_bytes(g);
    const int vid = pick_variant(ax.stride == 1, ax.n, elem);
    const int64_t C = scx::variant(vid).C();
    scx::PassArgs a;
    std::memset(&a, 0, sizeof(a));
    a.v = v;
    a.acc = acc;
    a.out = out;
    a.g = dg;
    a.n = ax.n;
    a.stride = ax.stride;
    a.nlines = ax.nlines;
    a.ncells = ax.ncells;
    a.nchunks = (ax.n + C - 1) / C;
    a.bc = ax.bc;
    a.acc_mode = acc_mode;
    a.vw = vw;
    a.aw = aw;
    a.nops = nops;
    fill_ext(&a, order);
    bool multi = false;
    for (int o = 0; o < nops; ++o) {
        fill_op(&a.ops[o], ops[o].op, order, ops[o].alpha, ax, vid, ops[o].scale, ops[o].k, ops[o].identity);
        multi = multi || ops[o].k > 1;
        if (nn_cpb > 0) {
            // nearest-neighbour blocks: the two ends of the line are more than one block apart
            // (e^{-alpha (b - a)} below the N-N tolerance), so their coupling is dropped
            a.ops[o].mu = 0.0;
            a.ops[o].inv1mmu = 1.0;
            a.ops[o].dir2inv = 2.0;
        }
    }
    if (nn_cpb > 0 && (multi || nn_cpb > INT32_MAX)) return fail(SC_ERR_ARG, "internal: bad nearest-neighbour block");
    if (multi && (nops != 1 || a.nchunks != 1 || ax.bc != SC_BC_PERIODIC))
        return fail(SC_ERR_UNSUPPORTED, "internal: fused powers of D need one periodic operator on whole lines");
    const int64_t tiles = (ax.nlines + scx::variant(vid).TC - 1) / scx::variant(vid).TC;
    if (tiles * a.nchunks > (int64_t)INT32_MAX) return fail(SC_ERR_SHAPE, "too many lines for one launch");
    // timing names carry the axis: its stride decides the memory access pattern
    static const char *const kFused[3] = {"line_pass_fused_x", "line_pass_fused_y", "line_pass_fused_z"};
    static const char *const kAgg[3] = {"line_pass_agg_x", "line_pass_agg_y", "line_pass_agg_z"};
    static const char *const kApply[3] = {"line_pass_apply_x", "line_pass_apply_y", "line_pass_apply_z"};
    hipError_t e;
    if (a.nchunks == 1) {
        // Strided lines of exactly one tile whose tiles are adjacent, aligned lines: the pipelined
        // persistent form, where it measured faster (512^3, per pass): FP32 (0.40 -> 0.35 ms: its
        // arithmetic is the longer part and overlaps the loads there).  FP64 passes, whose plain
        // form streams its strided loads and stores, run z in 0.52 ms against 0.54 pipelined.
        // SC_PIPE overrides (pipe_mode).
        const scx::Variant &V = scx::variant(vid);
        const bool pipe = !V.contig && !multi && scx::pipe_variant(vid, elem) && ax.n == V.C() && ax.nlines % V.TC == 0 &&
                          ax.stride % V.TC == 0 && ((uintptr_t)v & 15) == 0 && pipe_mode() != 0 &&
                          (pipe_mode() == 1 || elem == 4);
        e = timed(kFused[dim], st, [&](const char **) {
            return pipe ? scx::launch_line_pass_pipe(a, elem, order, vid, st)
                        : scx::launch_line_pass(a, elem, order, vid, scx::LMODE_FUSED, multi, st);
        });
        if (e != hipSuccess) return fail(SC_ERR_DEVICE, std::string("launch failed: ") + hipGetErrorString(e));
        return SC_OK;
    }
    if (nn_cpb == 0) {
        const int K = window_k(a, order, scx::variant(vid), multi);
        if (K > 0) {
            // windowed carries: one launch, no workspace; the two ends' coupling (below 2^-60 here,
            // since the line is longer than K) is dropped
            a.win_k = K;
            a.ops[0].mu = 0.0;
            a.ops[0].inv1mmu = 1.0;
            a.ops[0].dir2inv = 2.0;
            e = timed(kApply[dim], st, [&](const char **) {
                return scx::launch_line_pass(a, elem, order, vid, scx::LMODE_WIN, false, st);
            });
            if (e != hipSuccess) return fail(SC_ERR_DEVICE, std::string("launch failed: ") + hipGetErrorString(e));
            return SC_OK;
        }
    }
    const size_t need = chunk_ws_bytes(ax.nlines, a.nchunks, nops);
    if (!wsp || ws_bytes < need) return fail(SC_ERR_WORKSPACE, "workspace too small for a chunked pass");
    const int64_t ent = (int64_t)nops * ax.nlines * a.nchunks;
    a.agg = (double *)wsp;
    a.carry = (const double *)(wsp + round256(sizeof(double) * (size_t)(3 * ent)));
    if (a.nchunks <= kSingleChunks && single_pass_enabled() && nn_cpb == 0) {
        // lines of at most 8 chunks: one launch reads the field once; its tiles publish their chunk
        // totals and gather those of the other chunks of their lines (the slots and the claim
        // counter are reset first, by a kernel on the same stream)
        static const char *const kSingle[3] = {"line_pass_single_x", "line_pass_single_y", "line_pass_single_z"};
        a.sync = (uint32_t *)(wsp + round256(sizeof(double) * (size_t)(3 * ent)));
        a.spin_limit = spin_limit();
        e = timed("single_pass_reset", st, [&](const char **) {
            return scx::launch_single_pass_reset(a.agg, 3 * ent, a.sync, st);
        });
        if (e == hipSuccess)
            e = timed(kSingle[dim], st, [&](const char **) {
                return scx::launch_line_pass(a, elem, order, vid, scx::LMODE_SINGLE, false, st);
            });
        if (e != hipSuccess) return fail(SC_ERR_DEVICE, std::string("launch failed: ") + hipGetErrorString(e));
        return SC_OK;
    }
    // lines of few chunks: every apply tile forms its own carries from the chunk totals (one launch
    // less); longer lines go through the carry launch
    // (nearest-neighbour blocks always take the carry launch)
    a.nn_cpb = (int32_t)nn_cpb;
    a.fuse_carry = (a.nchunks <= kFuseCarryChunks && nn_cpb == 0) ? 1 : 0;
    e = timed(kAgg[dim], st, [&](const char **) {
        return scx::launch_line_pass(a, elem, order, vid, scx::LMODE_AGG, false, st);
    });
    if (e == hipSuccess && !a.fuse_carry)
        e = timed("chunk_carry", st, [&](const char **) { return scx::launch_chunk_carry(a, st); });
    if (e == hipSuccess)
        e = timed(kApply[dim], st, [&](const char **) {
            return scx::launch_line_pass(a, elem, order, vid, scx::LMODE_APPLY, false, st);
        });
    if (e != hipSuccess) return fail(SC_ERR_DEVICE, std::string("launch failed: ") + hipGetErrorString(e));
    return SC_OK;
}

sc_status check_line_args(const sc_grid *g, int dim, int order, double alpha)
{
    sc_status s = check_grid(g);
    if (s != SC_OK) return s;
    if (dim < 0 || dim >= g->ndim) return fail(SC_ERR_ARG, "dim out of range");
    if (order != 4 && order != 6) return fail(SC_ERR_UNSUPPORTED, "order must be 4 or 6");
    if (!(alpha > 0.0) || !std::isfinite(alpha)) return fail(SC_ERR_ARG, "alpha must be finite and > 0");
    if (g->n[dim] < order + 1) return fail(SC_ERR_SHAPE, "line shorter than the stencil (n < order + 1)");
    const double nu = alpha * (axis_of(g, dim).dx);
    if (!(nu < 700.0)) return fail(SC_ERR_ARG, "alpha * dx too large (> 700)");
    return SC_OK;
}

double nn_bound(const sc_grid *g, const sc_linear_pde *p)
{
    const double eps = p->nn_eps > 0.0 ? p->nn_eps : 1e-16;
    const double le = std::log(eps);
    double b = std::numeric_limits<double>::infinity();
    for (int d = 0; d < g->ndim; ++d) {
        const double Lm = p->block_len > 0.0 ? p->block_len : (g->hi[d] - g->lo[d]);
        if (p->c[d] != 0.0) b = std::min(b, -p->beta * Lm / (std::fabs(p->c[d]) * le));
        if (p->nu_diff > 0.0) b = std::min(b, (1.0 / p->nu_diff) * (p->beta * Lm / le) * (p->beta * Lm / le));
    }
    return b;
}

}  // namespace host
}  // namespace scx

using namespace scx::host;

// ------------------------------------------------------------------------------------------
// ABI
// ------------------------------------------------------------------------------------------
extern "C" {

const char *sc_last_error(void) { return g_err.c_str(); }

sc_status sc_local_quad(const sc_grid *grid, int dim, int order, double alpha, const void *v, void *JL,
                        void *JR, sc_stream_t stream)
{
    sc_status s = check_line_args(grid, dim, order, alpha);
    if (s != SC_OK) return s;
    if (!v || !JL || !JR) return fail(SC_ERR_ARG, "null array pointer");
    const Axis ax = axis_of(grid, dim);
    const size_t bytes = (size_t)ax.total * elem_bytes(grid);
    if (overlap(v, JL, bytes) || overlap(v, JR, bytes) || overlap(JL, JR, bytes))
        return fail(SC_ERR_ARG, "v, JL and JR must not overlap");
    scx::PassArgs a;
    std::memset(&a, 0, sizeof(a));
    a.v = v;
    a.n = ax.n;
    a.stride = ax.stride;
    a.nlines = ax.nlines;
    a.ncells = ax.ncells;
    a.bc = ax.bc;
    a.nops = 1;
    fill_ext(&a, order);
    fill_op(&a.ops[0], SC_OP_0, order, alpha, ax, 0, 1.0, 0);
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = timed("local_quad", st, [&](const char **) { return scx::launch_local_quad(a, (int)elem_bytes(grid), order, JL, JR, st); });
    if (e != hipSuccess) return fail(SC_ERR_DEVICE, std::string("launch failed: ") + hipGetErrorString(e));
    return SC_OK;
}

sc_status sc_sweep_LR(const sc_grid *grid, int dim, double alpha, const void *JL, const void *JR, void *IL,
                      void *IR, double *line_ends, sc_stream_t stream)
{
    sc_status s = check_line_args(grid, dim, 4, alpha);
    if (s != SC_OK) return s;
    if (!JL || !JR || !IL || !IR || !line_ends) return fail(SC_ERR_ARG, "null array pointer");
    const Axis ax = axis_of(grid, dim);
    const size_t bytes = (size_t)ax.total * elem_bytes(grid);
    if (overlap(IL, IR, bytes) || overlap(IL, JL, bytes) || overlap(IL, JR, bytes) || overlap(IR, JL, bytes) ||
        overlap(IR, JR, bytes))
        return fail(SC_ERR_ARG, "outputs must not overlap the inputs or each other");
    scx::PassArgs a;
    std::memset(&a, 0, sizeof(a));
    a.n = ax.n;
    a.stride = ax.stride;
    a.nlines = ax.nlines;
    a.ncells = ax.ncells;
    a.bc = ax.bc;
    a.nops = 1;
    a.ops[0].d = std::exp(-alpha * ax.dx);
    a.ops[0].nu = alpha * ax.dx;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = timed("sweep", st, [&](const char **) { return scx::launch_sweep(a, (int)elem_bytes(grid), JL, JR, IL, IR, line_ends, st); });
    if (e != hipSuccess) return fail(SC_ERR_DEVICE, std::string("launch failed: ") + hipGetErrorString(e));
    return SC_OK;
}

size_t sc_workspace_bytes(const sc_grid *grid, int dim, int which, int k)
{
    if (check_grid(grid) != SC_OK) return 0;
    if (which == 2) {
        size_t b = round256((size_t)axis_of(grid, 0).total * elem_bytes(grid));
        if (k >= 2) {
            // Runge-Kutta stages: two stage fields, then the partial sums' own
            size_t ps = 0;
            for (int d = 0; d < grid->ndim; ++d) ps = std::max(ps, sc_workspace_bytes(grid, d, 1, k));
            return 2 * b + ps + 256;
        }
        size_t extra = 0;
        for (int d = 0; d < grid->ndim; ++d) {
            const Axis ax = axis_of(grid, d);
            extra = std::max(extra, chunk_ws_bytes(ax.nlines, nchunks_for(ax, (int)elem_bytes(grid)), 2));
        }
        return b + extra + 256;
    }
    if (dim < 0 || dim >= grid->ndim) return 0;
    const Axis ax = axis_of(grid, dim);
    const int64_t nch = nchunks_for(ax, (int)elem_bytes(grid));
    size_t b = chunk_ws_bytes(ax.nlines, nch, 1);
    if (which == 1 && nch > 1 && k > 1) b += 2 * round256((size_t)ax.total * elem_bytes(grid));
    return b + 256;
}

sc_status sc_apply_invL(const sc_grid *grid, int dim, int op, int order, double alpha, const double *dirichlet_g,
                        const void *v, void *out, void *ws, size_t ws_bytes, sc_stream_t stream)
{
    sc_status s = check_line_args(grid, dim, order, alpha);
    if (s != SC_OK) return s;
    if (op < SC_OP_L || op > SC_OP_0) return fail(SC_ERR_ARG, "op must be SC_OP_L, SC_OP_R or SC_OP_0");
    if (!v || !out) return fail(SC_ERR_ARG, "null array pointer");
    const Axis ax = axis_of(grid, dim);
    if (overlap(v, out, (size_t)ax.total * elem_bytes(grid))) return fail(SC_ERR_ARG, "out overlaps v");
    if (ws && ((uintptr_t)ws & 255)) return fail(SC_ERR_ARG, "workspace must be 256-byte aligned");
    OpSpec o{(int)op, alpha, 1.0, 0};
    return run_pass(grid, dim, order, &o, 1, v, nullptr, 0, out, dirichlet_g, (char *)ws, ws_bytes,
                    (hipStream_t)stream);
}

int64_t sc_chunk_points(const sc_grid *grid, int dim)
{
    if (check_grid(grid) != SC_OK || dim < 0 || dim >= grid->ndim) return -1;
    return chunk_points(axis_of(grid, dim), (int)elem_bytes(grid));
}

sc_status sc_apply_invL_nn(const sc_grid *grid, int dim, int op, int order, double alpha, int64_t block_points,
                           const double *dirichlet_g, const void *v, void *out, void *ws, size_t ws_bytes,
                           sc_stream_t stream)
{
    sc_status s = check_line_args(grid, dim, order, alpha);
    if (s != SC_OK) return s;
    if (op < SC_OP_L || op > SC_OP_0) return fail(SC_ERR_ARG, "op must be SC_OP_L, SC_OP_R or SC_OP_0");
    if (!v || !out) return fail(SC_ERR_ARG, "null array pointer");
    const Axis ax = axis_of(grid, dim);
    if (overlap(v, out, (size_t)ax.total * elem_bytes(grid))) return fail(SC_ERR_ARG, "out overlaps v");
    if (ws && ((uintptr_t)ws & 255)) return fail(SC_ERR_ARG, "workspace must be 256-byte aligned");
    const int64_t C = chunk_points(ax, (int)elem_bytes(grid));
    if (block_points < 1) return fail(SC_ERR_ARG, "block_points must be positive");
    if (block_points < ax.n && block_points % C != 0)
        return fail(SC_ERR_ARG, "block_points must be a multiple of sc_chunk_points (" + std::to_string(C) +
                                    " on this axis) or at least the line length");
    const int64_t nch = (ax.n + C - 1) / C;
    const int64_t cpb = std::min<int64_t>(block_points >= ax.n ? nch : block_points / C, nch);
    OpSpec o{(int)op, alpha, 1.0, 0};
    return run_pass(grid, dim, order, &o, 1, v, nullptr, 0, out, dirichlet_g, (char *)ws, ws_bytes,
                    (hipStream_t)stream, cpb);
}

// out = aw acc + scale S_k[v] along `dim` (acc may be out; nullptr: none) for lines longer than one
// tile: the Horner form of the fused passes, S_k = D (I + D (I + ... + D)), one pass per power --
// u_1 = v, u_{p+1} = v + D[u_p] (each pass adds v to its result), the last pass writing
// scale D[u_k] + aw acc.  ws: two fields and the chunk totals (sc_workspace_bytes(grid, dim, 1, k)).
static sc_status partial_sum_chunked(const sc_grid *grid, int dim, int op, int order, double alpha, int k,
                                     double scale, const double *dirichlet_g, const void *v, const void *acc,
                                     double aw, void *out, char *ws, size_t ws_bytes, hipStream_t st)
{
    const size_t bytes = (size_t)axis_of(grid, dim).total * elem_bytes(grid);
    const size_t need = sc_workspace_bytes(grid, dim, 1, k);
    if (!ws || ws_bytes < need) return fail(SC_ERR_WORKSPACE, "workspace too small");
    char *w0 = ws;
    char *w1 = w0 + round256(bytes);
    char *rest = w1 + round256(bytes);
    const size_t rest_bytes = ws_bytes - 2 * round256(bytes);
    const void *u = v;
    for (int p = 1; p <= k; ++p) {
        const bool last = p == k;
        void *dst = last ? out : (void *)((p % 2) ? w0 : w1);
        OpSpec o{op, alpha, last ? scale : 1.0, 1};
        const sc_status s = last ? run_pass(grid, dim, order, &o, 1, u, acc, acc ? 2 : 0, dst, dirichlet_g, rest,
                                            rest_bytes, st, 0, 1.0, aw)
                                 : run_pass(grid, dim, order, &o, 1, u, v, 2, dst, dirichlet_g, rest, rest_bytes, st);
        if (s != SC_OK) return s;
        u = dst;
    }
    return SC_OK;
}

sc_status sc_apply_D_partial_sum(const sc_grid *grid, int dim, int op, int order, double alpha, int k,
                                 double scale, const double *dirichlet_g, const void *v, void *out, void *ws,
                                 size_t ws_bytes, sc_stream_t stream)
{
    sc_status s = check_line_args(grid, dim, order, alpha);
    if (s != SC_OK) return s;
    if (op < SC_OP_L || op > SC_OP_0) return fail(SC_ERR_ARG, "op must be SC_OP_L, SC_OP_R or SC_OP_0");
    if (k < 1 || k > 8) return fail(SC_ERR_ARG, "k must be in 1..8");
    if (!std::isfinite(scale)) return fail(SC_ERR_ARG, "scale must be finite");
    if (!v || !out) return fail(SC_ERR_ARG, "null array pointer");
    if (grid->bc[dim] == SC_BC_DIRICHLET && k > 1)
        return fail(SC_ERR_UNSUPPORTED, "Dirichlet axes support k = 1 only");
    const Axis ax = axis_of(grid, dim);
    const size_t bytes = (size_t)ax.total * elem_bytes(grid);
    if (overlap(v, out, bytes)) return fail(SC_ERR_ARG, "out overlaps v");
    if (ws && ((uintptr_t)ws & 255)) return fail(SC_ERR_ARG, "workspace must be 256-byte aligned");
    hipStream_t st = (hipStream_t)stream;
    if (nchunks_for(ax, (int)elem_bytes(grid)) == 1 || k == 1) {
        OpSpec o{(int)op, alpha, scale, k};
        return run_pass(grid, dim, order, &o, 1, v, nullptr, 0, out, dirichlet_g, (char *)ws, ws_bytes, st);
    }
    return partial_sum_chunked(grid, dim, op, order, alpha, k, scale, dirichlet_g, v, nullptr, 0.0, out, (char *)ws,
                               ws_bytes, st);
}

double sc_effective_dt(const sc_grid *grid, const sc_linear_pde *pde)
{
    if (check_grid(grid) != SC_OK || !pde || !(pde->dt > 0.0) || !(pde->beta > 0.0)) return -1.0;
    if (pde->nn_policy == 1) return std::min(pde->dt, nn_bound(grid, pde));
    return pde->dt;
}

sc_status sc_time_step(const sc_grid *grid, const sc_linear_pde *pde, int nsteps, void *u, void *ws,
                       size_t ws_bytes, sc_stream_t stream)
{
    sc_status s = check_grid(grid);
    if (s != SC_OK) return s;
    if (!pde || !u) return fail(SC_ERR_ARG, "null argument");
    if (nsteps < 0) return fail(SC_ERR_ARG, "nsteps must be >= 0");
    if (pde->order != 4 && pde->order != 6) return fail(SC_ERR_UNSUPPORTED, "order must be 4 or 6");
    if (!(pde->dt > 0.0) || !(pde->beta > 0.0) || !(pde->nu_diff >= 0.0))
        return fail(SC_ERR_ARG, "dt and beta must be > 0 and nu_diff >= 0");
    if (pde->nn_policy < 0 || pde->nn_policy > 2) return fail(SC_ERR_ARG, "nn_policy must be 0, 1 or 2");
    if (pde->split != 0 && pde->split != 1) return fail(SC_ERR_ARG, "split must be 0 or 1");
    if (pde->stages < 0 || pde->stages > 3) return fail(SC_ERR_ARG, "stages must be 0..3");
    const int stages = pde->stages < 1 ? 1 : pde->stages;
    if (stages > 1) {
        if (pde->split) return fail(SC_ERR_UNSUPPORTED, "Runge-Kutta stages use the unsplit form");
        for (int d = 0; d < grid->ndim; ++d)
            if (grid->bc[d] != SC_BC_PERIODIC) return fail(SC_ERR_UNSUPPORTED, "Runge-Kutta stages need periodic axes");
    }
    double dt = pde->dt;
    if (pde->nn_policy != 0) {
        const double bound = nn_bound(grid, pde);
        if (dt > bound) {
            if (pde->nn_policy == 2) return fail(SC_ERR_ARG, "dt exceeds the nearest-neighbour bound");
            dt = bound;
        }
    }
    for (int d = 0; d < grid->ndim; ++d)
        if (grid->n[d] < pde->order + 1) return fail(SC_ERR_SHAPE, "line shorter than the stencil");
    const size_t need = sc_workspace_bytes(grid, 0, 2, stages) - 256;
    if (!ws || ws_bytes < need) return fail(SC_ERR_WORKSPACE, "workspace too small (see sc_workspace_bytes)");
    if ((uintptr_t)ws & 255) return fail(SC_ERR_ARG, "workspace must be 256-byte aligned");
    const Axis ax0 = axis_of(grid, 0);
    const size_t fbytes = (size_t)ax0.total * elem_bytes(grid);
    if (overlap(u, ws, fbytes)) return fail(SC_ERR_ARG, "workspace overlaps u");
    hipStream_t st = (hipStream_t)stream;
    char *wsp = (char *)ws;
    void *cur = u, *nxt = wsp;
    char *rest = wsp + round256(fbytes);
    const size_t rest_bytes = ws_bytes - round256(fbytes);
    // per-axis operators (Sec. 2.1 alpha choices)
    OpSpec ops[3][2];
    int nops[3] = {0, 0, 0};
    for (int d = 0; d < grid->ndim; ++d) {
        const double c = pde->c[d];
        if (c != 0.0) {
            const double a = pde->beta / (std::fabs(c) * dt);
            ops[d][nops[d]++] = OpSpec{c > 0.0 ? SC_OP_R : SC_OP_L, a, -std::fabs(c) * dt * a, 1};
        }
        if (pde->nu_diff > 0.0) {
            const double a = pde->beta / std::sqrt(pde->nu_diff * dt);
            ops[d][nops[d]++] = OpSpec{SC_OP_0, a, -pde->nu_diff * dt * a * a, 1};
        }
        for (int o = 0; o < nops[d]; ++o) {
            const double nu = ops[d][o].alpha * axis_of(grid, d).dx;
            if (!(nu < 700.0) || !std::isfinite(nu)) return fail(SC_ERR_ARG, "alpha * dx too large (> 700)");
        }
    }
    if (stages > 1) {
        // s-stage SSP Runge-Kutta with every D replaced by S_s (Sec. 2.5): each stage is
        // out = ca acc + cb E(v), E(v) = v + sum over axes and operators of scale S_s[v].  The
        // partial-sum passes form it themselves: the first one adds cb v (and ca acc) to its
        // cb scale S_s[v], each later one adds its own term onto out.  Lines longer than one tile
        // take their powers of D one chunked pass each, the last adding the term onto out (a first
        // term with ca != 0 starts out as ca acc + cb v).
        const int elem = (int)elem_bytes(grid);
        const int64_t nel = ax0.total;
        char *U1 = wsp, *B = wsp + round256(fbytes);
        char *psw = B + round256(fbytes);
        const size_t psw_bytes = ws_bytes - 2 * round256(fbytes);
        auto lin = [&](double a, const void *x, double b, const void *y, void *o) -> sc_status {
            const hipError_t e = timed("lincomb", st, [&](const char **) {
                return scx::launch_lincomb(nel, elem, a, x, b, y, o, st);
            });
            return e == hipSuccess ? SC_OK : fail(SC_ERR_DEVICE, std::string("launch failed: ") + hipGetErrorString(e));
        };
        // out = ca acc + cb E(v); acc is read only when ca != 0 and may be out; v is not out
        auto stage = [&](const void *v, double ca, const void *acc, double cb, void *out) -> sc_status {
            bool first = true;
            for (int d = 0; d < grid->ndim; ++d)
                for (int k = 0; k < nops[d]; ++k) {
                    const OpSpec &op = ops[d][k];
                    sc_status r;
                    if (nchunks_for(axis_of(grid, d), elem) == 1) {
                        const OpSpec o{op.op, op.alpha, cb * op.scale, stages};
                        r = first ? run_pass(grid, d, pde->order, &o, 1, v, acc, ca != 0.0 ? 3 : 1, out, nullptr, psw,
                                             psw_bytes, st, 0, cb, ca)
                                  : run_pass(grid, d, pde->order, &o, 1, v, out, 2, out, nullptr, psw, psw_bytes, st);
                    } else {
                        const double sc = cb * op.scale;
                        if (first && ca == 0.0) {
                            r = partial_sum_chunked(grid, d, op.op, pde->order, op.alpha, stages, sc, nullptr, v, v, cb,
                                                    out, psw, psw_bytes, st);
                        } else {
                            r = first ? lin(ca, acc, cb, v, out) : SC_OK;
                            if (r == SC_OK)
                                r = partial_sum_chunked(grid, d, op.op, pde->order, op.alpha, stages, sc, nullptr, v,
                                                        out, 1.0, out, psw, psw_bytes, st);
                        }
                    }
                    if (r != SC_OK) return r;
                    first = false;
                }
            if (first) return ca == 0.0 ? lin(cb, v, 0.0, v, out) : lin(ca, acc, cb, v, out);  // no operators
            return SC_OK;
        };
        for (int step = 0; step < nsteps; ++step) {
            s = stage(u, 0.0, nullptr, 1.0, U1);
            if (s != SC_OK) return s;
            if (stages == 2) {
                s = stage(U1, 0.5, u, 0.5, u);
            } else {
                s = stage(U1, 0.75, u, 0.25, B);
                if (s == SC_OK) s = stage(B, 1.0 / 3.0, u, 2.0 / 3.0, u);
            }
            if (s != SC_OK) return s;
        }
        return SC_OK;
    }
    // Dimension-split steps alternate between u and the workspace pass by pass; after an odd number
    // of passes the result would sit in the workspace and need a copy back (a full-field read and
    // write).  A pass whose lines fit one tile reads all of its operand into the tile before it
    // writes, so it can run in place: the last such pass of the call does, and the result ends in u.
    int64_t inplace_pass = -1;
    if (pde->split) {
        int per_step = 0, last_fused = -1;
        for (int d = 0; d < grid->ndim; ++d)
            if (nops[d]) {
                if (nchunks_for(axis_of(grid, d), (int)elem_bytes(grid)) == 1) last_fused = per_step;
                ++per_step;
            }
        const int64_t passes = (int64_t)per_step * nsteps;
        if ((passes & 1) && last_fused >= 0) inplace_pass = passes - per_step + last_fused;
    }
    int64_t pass = 0;
    for (int step = 0; step < nsteps; ++step) {
        bool first = true;
        for (int d = 0; d < grid->ndim; ++d) {
            if (!nops[d]) continue;
            if (pde->split) {
                // one 1-D step on the current state: nxt = cur + sum_ops scale * D[cur]
                const bool inplace = pass++ == inplace_pass;
                s = run_pass(grid, d, pde->order, ops[d], nops[d], cur, nullptr, 1, inplace ? cur : nxt, nullptr, rest,
                             rest_bytes, st);
                if (s != SC_OK) return s;
                if (!inplace) std::swap(cur, nxt);
                continue;
            }
            // unsplit: every axis reads u^n (cur); nxt accumulates u^n + all D terms
            s = run_pass(grid, d, pde->order, ops[d], nops[d], cur, first ? nullptr : nxt, first ? 1 : 2, nxt, nullptr,
                         rest, rest_bytes, st);
            if (s != SC_OK) return s;
            first = false;
        }
        if (!pde->split && !first) std::swap(cur, nxt);
    }
    if (cur != u) {
        hipError_t e = hipMemcpyAsync(u, cur, fbytes, hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return fail(SC_ERR_DEVICE, std::string("copy failed: ") + hipGetErrorString(e));
    }
    return SC_OK;
}

sc_status sc_timing_enable(int on)
{
    std::lock_guard<std::mutex> lk(g_tmu);
    g_timing = on != 0;
    return SC_OK;
}

sc_status sc_timing_select(const char *names)
{
    std::vector<std::string> sel;
    if (names) {
        const std::string all(names);
        if (all.size() > 1023) return fail(SC_ERR_ARG, "timing selection longer than 1023 bytes");
        size_t p = 0;
        while (p <= all.size()) {
            const size_t q = std::min(all.find(',', p), all.size());
            if (q > p) sel.push_back(all.substr(p, q - p));
            p = q + 1;
        }
    }
    std::lock_guard<std::mutex> lk(g_tmu);
    g_timing_only = std::move(sel);
    return SC_OK;
}

void sc_timing_reset(void)
{
    std::lock_guard<std::mutex> lk(g_tmu);
    for (auto &r : g_records) (void)hipEventSynchronize(r.stop);
    g_records.clear();
    g_pool_used = 0;
}

int sc_timing_read(char names[][64], double *ms, int *counts, int max_entries)
{
    std::lock_guard<std::mutex> lk(g_tmu);
    std::vector<std::string> nm;
    std::vector<double> t;
    std::vector<int> cnt;
    for (auto &r : g_records) {
        float el = 0.f;
        if (hipEventSynchronize(r.stop) != hipSuccess || hipEventElapsedTime(&el, r.start, r.stop) != hipSuccess)
            el = 0.f;
        size_t i = 0;
        for (; i < nm.size(); ++i)
            if (nm[i] == r.name) break;
        if (i == nm.size()) {
            nm.push_back(r.name);
            t.push_back(0.0);
            cnt.push_back(0);
        }
        t[i] += el;
        cnt[i] += 1;
    }
    int m = 0;
    for (size_t i = 0; i < nm.size() && m < max_entries; ++i, ++m) {
        std::snprintf(names[m], 64, "%s", nm[i].c_str());
        ms[m] = t[i];
        counts[m] = cnt[i];
    }
    return m;
}

}  // extern "C"
