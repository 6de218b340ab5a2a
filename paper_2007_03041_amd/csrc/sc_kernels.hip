// sc_kernels.hip -- the non-templated kernels of the successive-convolution library (chunk carries,
// stand-alone stages, helpers) and the dispatch of line passes to the per-(element type, order)
// instantiation units sc_lp_*.hip.
#include "sc_line_pass.h"

namespace scx {

extern template hipError_t launch_line_pass_t<double, 4, false>(const PassArgs &, int, int, bool, hipStream_t);
extern template hipError_t launch_line_pass_t<double, 4, true>(const PassArgs &, int, int, bool, hipStream_t);
extern template hipError_t launch_line_pass_t<double, 6, false>(const PassArgs &, int, int, bool, hipStream_t);
extern template hipError_t launch_line_pass_t<double, 6, true>(const PassArgs &, int, int, bool, hipStream_t);
extern template hipError_t launch_line_pass_t<float, 4, false>(const PassArgs &, int, int, bool, hipStream_t);
extern template hipError_t launch_line_pass_t<float, 4, true>(const PassArgs &, int, int, bool, hipStream_t);
extern template hipError_t launch_line_pass_t<float, 6, false>(const PassArgs &, int, int, bool, hipStream_t);
extern template hipError_t launch_line_pass_t<float, 6, true>(const PassArgs &, int, int, bool, hipStream_t);
extern template hipError_t launch_line_pass_pipe_t<double, 4>(const PassArgs &, int, hipStream_t);
extern template hipError_t launch_line_pass_pipe_t<double, 6>(const PassArgs &, int, hipStream_t);
extern template hipError_t launch_line_pass_pipe_t<float, 4>(const PassArgs &, int, hipStream_t);
extern template hipError_t launch_line_pass_pipe_t<float, 6>(const PassArgs &, int, hipStream_t);
extern template hipError_t launch_line_pass_batch_t<double, 4, false>(const BatchLaunch &, int, hipStream_t);
extern template hipError_t launch_line_pass_batch_t<double, 4, true>(const BatchLaunch &, int, hipStream_t);
extern template hipError_t launch_line_pass_batch_t<double, 6, false>(const BatchLaunch &, int, hipStream_t);
extern template hipError_t launch_line_pass_batch_t<double, 6, true>(const BatchLaunch &, int, hipStream_t);
extern template hipError_t launch_line_pass_batch_t<float, 4, false>(const BatchLaunch &, int, hipStream_t);
extern template hipError_t launch_line_pass_batch_t<float, 4, true>(const BatchLaunch &, int, hipStream_t);
extern template hipError_t launch_line_pass_batch_t<float, 6, false>(const BatchLaunch &, int, hipStream_t);
extern template hipError_t launch_line_pass_batch_t<float, 6, true>(const BatchLaunch &, int, hipStream_t);
extern template int line_pass_batch_occupancy_t<double, 4, false>(int, int);
extern template int line_pass_batch_occupancy_t<double, 4, true>(int, int);
extern template int line_pass_batch_occupancy_t<double, 6, false>(int, int);
extern template int line_pass_batch_occupancy_t<double, 6, true>(int, int);
extern template int line_pass_batch_occupancy_t<float, 4, false>(int, int);
extern template int line_pass_batch_occupancy_t<float, 4, true>(int, int);
extern template int line_pass_batch_occupancy_t<float, 6, false>(int, int);
extern template int line_pass_batch_occupancy_t<float, 6, true>(int, int);

// Nearest-neighbour carries (Sec. 3.2/3.3 block operators under the N-N criterion): the line is cut
// into virtual blocks of cpb chunks.  Within a block the chunks chain exactly; the first chunk of
// block b > 0 receives block b-1's own total (its sweep from zero), the last chunk of block b < last
// receives block b+1's own total, and nothing comes from further away.  Periodic lines take the
// periodic choice for the wrap (the last block's own I_R at b, the first block's own I_L at a);
// Dirichlet lines impose their end values on the end blocks' operators, whose end integrals are
// the carried sweeps at the end points.  The operator's mu terms are zero here (set on the host).
__device__ void chunk_carry_nn(const PassArgs &a, const OpArgs &P, const double *ag, double *cr, double ga,
                               double gb, double &Ap, double &Bp)
{
    const int64_t nch = a.nchunks, cpb = a.nn_cpb;
    double E = 0.0, T = 0.0;  // carried sweep, and the current block's own sweep
    for (int64_t ch = 0; ch < nch; ++ch) {
        if (ch % cpb == 0) {
            E = T;  // the previous block's own total (zero before block 0)
            T = 0.0;
        }
        cr[2 * ch + 0] = E;
        const double dc = ch == nch - 1 ? P.dchunk_last : P.dchunk;
        E = fma(dc, E, ag[3 * ch + 0]);
        T = fma(dc, T, ag[3 * ch + 0]);
    }
    double F = 0.0, U = 0.0;
    for (int64_t ch = nch - 1; ch >= 0; --ch) {
        if (ch == nch - 1 || (ch + 1) % cpb == 0) {
            F = U;  // the next block's own total (zero after the last block)
            U = 0.0;
        }
        cr[2 * ch + 1] = F;
        const double dc = ch == nch - 1 ? P.dchunk_last : P.dchunk;
        F = fma(dc, F, ag[3 * ch + 1]);
        U = fma(dc, U, ag[3 * ch + 1]);
    }
    if (a.bc == 0)
        boundary_constants(P, 0, T, U, ag[2], 0.0, 0.0, Ap, Bp);
    else
        boundary_constants(P, 1, E, F, ag[2], ga, gb, Ap, Bp);
}

// Chunk carries of chunked passes: one thread per (op, line) walks the chunk totals in both
// directions (Sec. 3, eqs. (Left-/Right-moving integral DD) with exact attenuation factors) and
// forms the boundary constants.
__device__ void chunk_carry_one(const PassArgs &a, const double *agg, double *carry, const double *g, int64_t idx)
{
    const int o = (int)(idx / a.nlines);
    const int64_t L = idx % a.nlines;
    const OpArgs &P = a.ops[o];
    const int64_t nch = a.nchunks;
    const double *ag = agg + ((int64_t)o * a.nlines + L) * nch * 3;
    double *cr = carry + ((int64_t)o * a.nlines + L) * nch * 2;
    if (a.nn_cpb > 0) {
        const double ga = (a.bc == 1 && g) ? g[2 * L + 0] : 0.0;
        const double gb = (a.bc == 1 && g) ? g[2 * L + 1] : 0.0;
        double Ap = 0.0, Bp = 0.0;
        chunk_carry_nn(a, P, ag, cr, ga, gb, Ap, Bp);
        double *ab = carry + 2 * (int64_t)a.nops * a.nlines * nch + 2 * idx;
        ab[0] = Ap;
        ab[1] = Bp;
        return;
    }
    double E = 0.0;
    for (int64_t ch = 0; ch < nch; ++ch) {
        cr[2 * ch + 0] = E;
        E = fma(ch == nch - 1 ? P.dchunk_last : P.dchunk, E, ag[3 * ch + 0]);
    }
    double F = 0.0;
    for (int64_t ch = nch - 1; ch >= 0; --ch) {
        cr[2 * ch + 1] = F;
        F = fma(ch == nch - 1 ? P.dchunk_last : P.dchunk, F, ag[3 * ch + 1]);
    }
    const double ga = (a.bc == 1 && g) ? g[2 * L + 0] : 0.0;
    const double gb = (a.bc == 1 && g) ? g[2 * L + 1] : 0.0;
    double Ap = 0.0, Bp = 0.0;
    boundary_constants(P, a.bc, E, F, ag[2], ga, gb, Ap, Bp);
    double *ab = carry + 2 * (int64_t)a.nops * a.nlines * nch + 2 * idx;
    ab[0] = Ap;
    ab[1] = Bp;
}

__global__ void __launch_bounds__(256) chunk_carry(const PassArgs a)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)a.nops * a.nlines) return;
    chunk_carry_one(a, a.agg, const_cast<double *>(a.carry), a.g, idx);
}

// Batched chunk carries: workgroup b serves every (operator, line) of instance items[b].
__global__ void __launch_bounds__(256) chunk_carry_batch(const BatchArgs *__restrict__ table,
                                                         const int32_t *__restrict__ items, const double *gbase,
                                                         double *wsbase)
{
    const BatchArgs &b = table[items[blockIdx.x]];
    const int64_t cnt = (int64_t)b.a.nops * b.a.nlines;
    for (int64_t idx = threadIdx.x; idx < cnt; idx += blockDim.x)
        chunk_carry_one(b.a, wsbase + b.agg_off, wsbase + b.carry_off, b.g_off >= 0 ? gbase + b.g_off : nullptr, idx);
}

// ------------------------------------------------------------------------------------------
// Stand-alone stages (sc_local_quad, sc_sweep_LR) and small helpers.
// ------------------------------------------------------------------------------------------
template <typename T, int ORDER>
__global__ void __launch_bounds__(256) local_quad_kernel(const PassArgs a, T *JL, T *JR)
{
    constexpr int H = ORDER / 2;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = a.n * a.nlines;
    if (gid >= total) return;
    // gid enumerates elements in memory order; recover (line, i)
    const int64_t s = a.stride, n = a.n;
    const int64_t outer = gid / (s * n), rem = gid % (s * n);
    const int64_t i = rem / s, inner = rem % s;
    const int64_t base = outer * s * n + inner;
    const T *v = (const T *)a.v;
    const OpArgs &P = a.ops[0];
    double sr = 0.0, sl = 0.0;
#pragma unroll
    for (int j = 0; j < ORDER; ++j) {
        sr = fma(P.wR[j], (double)line_value<T, ORDER>(a, v, base, i - H + j), sr);
        sl = fma(P.wR[ORDER - 1 - j], (double)line_value<T, ORDER>(a, v, base, i - H + 1 + j), sl);
    }
    if (a.bc == 1 && i == 0) sr = 0.0;
    if (a.bc == 1 && i == n - 1) sl = 0.0;
    JR[gid] = (T)sr;
    JL[gid] = (T)sl;
}

// Raw sweeps: one workgroup per line, each thread a contiguous segment, serial carries between
// the segments -- the stand-alone debugging stage, not the fused hot path.
template <typename T>
__global__ void __launch_bounds__(256) sweep_kernel(const PassArgs a, const T *JL, const T *JR,
                                                    T *IL, T *IR, double *ends)
{
    __shared__ double sf[256], sb[256], dp[256], cinf[256], cinb[256];
    const int64_t L = blockIdx.x;
    const int tid = threadIdx.x;
    const int64_t n = a.n, s = a.stride;
    const int64_t base = (L / s) * s * n + (L % s);
    const OpArgs &P = a.ops[0];
    const double d = P.d;
    const int64_t seg = (n + 255) / 256;
    const int64_t i0 = tid * seg, i1 = (i0 + seg < n) ? i0 + seg : n;
    // local sweeps (J_R[0] excluded from the forward sweep; J_L of the last point excluded for
    // Dirichlet lines)
    double f = 0.0;
    for (int64_t i = i0; i < i1; ++i) f = fma(d, f, i == 0 ? 0.0 : (double)JR[base + i * s]);
    double b = 0.0;
    for (int64_t i = i1 - 1; i >= i0; --i)
        b = fma(d, b, (a.bc == 1 && i == n - 1) ? 0.0 : (double)JL[base + i * s]);
    const int64_t len = i1 > i0 ? i1 - i0 : 0;
    sf[tid] = f;
    sb[tid] = b;
    dp[tid] = exp(-P.nu * (double)len);  // decay across this segment
    __syncthreads();
    if (tid == 0) {
        double cc = 0.0;
        for (int t = 0; t < 256; ++t) {
            cinf[t] = cc;
            cc = fma(dp[t], cc, sf[t]);
        }
        double cb2 = 0.0;
        for (int t = 255; t >= 0; --t) {
            cinb[t] = cb2;
            cb2 = fma(dp[t], cb2, sb[t]);
        }
    }
    __syncthreads();
    f = cinf[tid];
    for (int64_t i = i0; i < i1; ++i) {
        f = fma(d, f, i == 0 ? 0.0 : (double)JR[base + i * s]);
        IR[base + i * s] = (T)f;
    }
    b = cinb[tid];
    for (int64_t i = i1 - 1; i >= i0; --i) {
        b = fma(d, b, (a.bc == 1 && i == n - 1) ? 0.0 : (double)JL[base + i * s]);
        IL[base + i * s] = (T)b;
    }
    __syncthreads();
    if (tid == 0) {
        const double IRn = (double)IR[base + (n - 1) * s];
        ends[2 * L + 0] = (double)IL[base];
        ends[2 * L + 1] = (a.bc == 0) ? fma(d, IRn, (double)JR[base]) : IRn;
    }
}

// out = a x + b y (element-wise; out may be x or y)
template <typename T>
__global__ void __launch_bounds__(256) lincomb_kernel(int64_t nel, double a, const T *x, double b, const T *y, T *out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nel) out[i] = (T)fma(a, (double)x[i], b * (double)y[i]);
}

// ------------------------------------------------------------------------------------------
// Host launchers
// ------------------------------------------------------------------------------------------

// ------------------------------------------------------------------------------------------
// Host launchers
// ------------------------------------------------------------------------------------------
static const Variant kVariants[] = {
#define SC_ROW(id, S, TC, CONTIG, NT) {S, TC, CONTIG, NT},
    SC_VARIANTS(SC_ROW)
#undef SC_ROW
};
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

int num_variants() { return kNumVariants; }
const Variant &variant(int id) { return kVariants[id]; }
bool variant_built(int vid, int elem)
{
    if (vid < 0 || vid >= kNumVariants) return false;
    // both orders and operator counts must fit: the order-6 two-operator shape is the largest
    return kVariants[vid].lds_bytes(elem, 6, 2) <= LDS_LIMIT;
}

hipError_t launch_line_pass(const PassArgs &a, int elem, int order, int vid, int mode, bool multi, hipStream_t st)
{
    if (!variant_built(vid, elem)) return hipErrorInvalidValue;
    // lines that are a whole number of chunks have no segment past their end: the kernels without
    // the per-point end rules keep fewer registers live and reach a higher occupancy.  Windowed
    // applies take a ragged last chunk as the full tile ending at the line's end, so all their tiles
    // are full.
    const bool full = a.n % variant(vid).C() == 0 || (mode == LMODE_WIN && a.n >= variant(vid).C());
    if (elem == 8) {
        if (order == 4)
            return full ? launch_line_pass_t<double, 4, true>(a, vid, mode, multi, st)
                        : launch_line_pass_t<double, 4, false>(a, vid, mode, multi, st);
        return full ? launch_line_pass_t<double, 6, true>(a, vid, mode, multi, st)
                    : launch_line_pass_t<double, 6, false>(a, vid, mode, multi, st);
    }
    if (order == 4)
        return full ? launch_line_pass_t<float, 4, true>(a, vid, mode, multi, st)
                    : launch_line_pass_t<float, 4, false>(a, vid, mode, multi, st);
    return full ? launch_line_pass_t<float, 6, true>(a, vid, mode, multi, st)
                : launch_line_pass_t<float, 6, false>(a, vid, mode, multi, st);
}

// Resets the chunk totals of a single-pass chunked launch to "not yet published" and its claim
// counter to 0 (a kernel rather than a memset, so the pair can sit in a captured graph).
__global__ void __launch_bounds__(256) single_pass_reset(double *__restrict__ agg, int64_t n, uint32_t *sync)
{
    const double e = __longlong_as_double((long long)CHUNK_EMPTY);
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) agg[i] = e;
    if (blockIdx.x == 0 && threadIdx.x == 0) *sync = 0u;
}

hipError_t launch_single_pass_reset(double *agg, int64_t n, uint32_t *sync, hipStream_t st)
{
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(single_pass_reset, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(256), 0, st, agg, n, sync);
    return hipGetLastError();
}

bool pipe_variant(int vid, int elem) { return (vid == 5 && elem == 8) || vid == 12; }

hipError_t launch_line_pass_pipe(const PassArgs &a, int elem, int order, int vid, hipStream_t st)
{
    if (!pipe_variant(vid, elem) || !variant_built(vid, elem)) return hipErrorInvalidValue;
    const Variant &V = variant(vid);
    // the shape the pipelined loads assume (checked again here, whatever the caller checked)
    if (V.contig || a.n != V.C() || a.nlines % V.TC || a.stride % V.TC || ((uintptr_t)a.v & 15) || a.nops < 1 ||
        a.nops > 2)
        return hipErrorInvalidValue;
    if (elem == 8) return order == 4 ? launch_line_pass_pipe_t<double, 4>(a, vid, st) : launch_line_pass_pipe_t<double, 6>(a, vid, st);
    return order == 4 ? launch_line_pass_pipe_t<float, 4>(a, vid, st) : launch_line_pass_pipe_t<float, 6>(a, vid, st);
}

hipError_t launch_line_pass_batch(const BatchLaunch &b, int elem, int order, int vid, hipStream_t st)
{
    if (!variant_built(vid, elem) || !batch_built(variant(vid))) return hipErrorInvalidValue;
    if (b.nwork <= 0) return hipSuccess;
    if (elem == 8) {
        if (order == 4)
            return b.full ? launch_line_pass_batch_t<double, 4, true>(b, vid, st)
                          : launch_line_pass_batch_t<double, 4, false>(b, vid, st);
        return b.full ? launch_line_pass_batch_t<double, 6, true>(b, vid, st)
                      : launch_line_pass_batch_t<double, 6, false>(b, vid, st);
    }
    if (order == 4)
        return b.full ? launch_line_pass_batch_t<float, 4, true>(b, vid, st)
                      : launch_line_pass_batch_t<float, 4, false>(b, vid, st);
    return b.full ? launch_line_pass_batch_t<float, 6, true>(b, vid, st)
                  : launch_line_pass_batch_t<float, 6, false>(b, vid, st);
}

int line_pass_batch_occupancy(int elem, int order, int vid, int mode, int full)
{
    if (!variant_built(vid, elem) || !batch_built(variant(vid))) return 0;
    if (elem == 8) {
        if (order == 4)
            return full ? line_pass_batch_occupancy_t<double, 4, true>(vid, mode)
                        : line_pass_batch_occupancy_t<double, 4, false>(vid, mode);
        return full ? line_pass_batch_occupancy_t<double, 6, true>(vid, mode)
                    : line_pass_batch_occupancy_t<double, 6, false>(vid, mode);
    }
    if (order == 4)
        return full ? line_pass_batch_occupancy_t<float, 4, true>(vid, mode)
                    : line_pass_batch_occupancy_t<float, 4, false>(vid, mode);
    return full ? line_pass_batch_occupancy_t<float, 6, true>(vid, mode)
                : line_pass_batch_occupancy_t<float, 6, false>(vid, mode);
}

hipError_t launch_chunk_carry_batch(const BatchArgs *table, const int32_t *items, int nitems,
                                    const double *g, double *ws, hipStream_t st)
{
    if (nitems <= 0) return hipSuccess;
    hipLaunchKernelGGL(chunk_carry_batch, dim3(nitems), dim3(256), 0, st, table, items, g, ws);
    return hipGetLastError();
}

hipError_t launch_chunk_carry(const PassArgs &a, hipStream_t st)
{
    const int64_t nthr = (int64_t)a.nops * a.nlines;
    hipLaunchKernelGGL(chunk_carry, dim3((nthr + 255) / 256), dim3(256), 0, st, a);
    return hipGetLastError();
}

template <typename T>
static hipError_t local_quad_t(const PassArgs &a, int order, void *JL, void *JR, hipStream_t st)
{
    const int64_t total = a.n * a.nlines;
    const dim3 grid((total + 255) / 256);
    if (order == 4)
        hipLaunchKernelGGL((local_quad_kernel<T, 4>), grid, dim3(256), 0, st, a, (T *)JL, (T *)JR);
    else
        hipLaunchKernelGGL((local_quad_kernel<T, 6>), grid, dim3(256), 0, st, a, (T *)JL, (T *)JR);
    return hipGetLastError();
}

hipError_t launch_local_quad(const PassArgs &a, int elem, int order, void *JL, void *JR, hipStream_t st)
{
    return elem == 8 ? local_quad_t<double>(a, order, JL, JR, st) : local_quad_t<float>(a, order, JL, JR, st);
}

hipError_t launch_sweep(const PassArgs &a, int elem, const void *JL, const void *JR, void *IL, void *IR, double *ends,
                        hipStream_t st)
{
    if (elem == 8)
        hipLaunchKernelGGL((sweep_kernel<double>), dim3(a.nlines), dim3(256), 0, st, a, (const double *)JL,
                           (const double *)JR, (double *)IL, (double *)IR, ends);
    else
        hipLaunchKernelGGL((sweep_kernel<float>), dim3(a.nlines), dim3(256), 0, st, a, (const float *)JL,
                           (const float *)JR, (float *)IL, (float *)IR, ends);
    return hipGetLastError();
}

hipError_t launch_lincomb(int64_t nel, int elem, double a, const void *x, double b, const void *y, void *out,
                          hipStream_t st)
{
    const dim3 grid((nel + 255) / 256);
    if (elem == 8)
        hipLaunchKernelGGL((lincomb_kernel<double>), grid, dim3(256), 0, st, nel, a, (const double *)x, b,
                           (const double *)y, (double *)out);
    else
        hipLaunchKernelGGL((lincomb_kernel<float>), grid, dim3(256), 0, st, nel, a, (const float *)x, b,
                           (const float *)y, (float *)out);
    return hipGetLastError();
}

}  // namespace scx
