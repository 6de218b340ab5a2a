// sc_line_pass.h -- the line-pass kernel of the successive-convolution fast summation (gfx950),
// included by one instantiation unit per (element type, order).
//
// One pass applies up to two operators L_op^{-1} (or D = I - L_op^{-1} and its partial sums) along
// one axis of a dense array, line by line (Sec. 2.2: the directions stay uncoupled).
//
//   workgroup = a tile of TC lines x one chunk of C = G*S points of each line (+ order/2 halo)
//   thread    = one segment of S consecutive points of one line (G segments per line)
//
// Per workgroup, with one HBM read of the operand and one write of the result:
//   1. coalesced load of the tile into LDS in [line][point] layout (one pad element per segment
//      against bank conflicts).  Along x the lanes run along the line; along y/z they run across TC
//      adjacent lines, so y/z tiles are transposed through LDS.  Each thread then holds the window
//      of S + order operand values around its segment in registers.
//   2. segment totals of the two sweeps (Sec. 2.4 recurrences).  In the interior they are linear
//      in the window, so each is one dot product with coefficients precomputed on the host (kR,
//      kL); segments at line ends and in the padding use the point-by-point local integrals of
//      Sec. 2.4, eqs. (JR), (JL).  A Dirichlet line's one-sided end stencils are realised by
//      extending the line beyond each end with the interpolant of its end values, so the centred
//      stencil integrates the same polynomial there.
//   3. the segments are combined by a first-order linear-recurrence scan over (decay, value) pairs:
//      Kogge-Stone with wavefront shuffles inside a wave (decay d^{S 2^j}) and one LDS exchange
//      between the waves of a line (Sec. 3, eqs. (Left-/Right-moving integral DD): a block's
//      integral = its own sweep + attenuated contributions of the others).  Lines longer than one
//      tile are chunked: an aggregate launch, a carry launch and an apply launch.
//   4. the line totals give the boundary constants in FP64 (Sec. 2.3 periodic constants; Dirichlet
//      end values through the 2x2 system whose inverse has the form of Sec. 3.3).
//   5. each thread re-sweeps its segment from the exact carries: the forward sweep adds its share
//      of the result, the backward sweep the rest (L_0^{-1} = (I_L + I_R)/2 + A e^{-alpha(x-a)}
//      + B e^{-alpha(b-x)} is linear in the two sweeps), scaled, as D = I - L^{-1} (Sec. 2.2) and
//      plus an accumulator (the explicit update of Sec. 2.5).  Only the S outputs stay in registers.
//
// The boundary terms are folded in as A' d^i and B' d^{N-i} with A' = I_R(b)/(1-mu),
// B' = I_L(a)/(1-mu) for periodic lines (for L_0 these are twice the paper's A, B because the
// sweep average carries the factor 1/2).
//
// Precision.  T is the element type in memory and the arithmetic type of all per-point work (local
// integrals, segment totals, re-sweeps, combine).  With T = float the in-wave scan of the segment
// totals runs on (hi, lo) float pairs with error-free transformations (compensated carries), and
// everything across wave-parts and chunks -- carries, line totals, boundary constants -- is FP64.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sc_device.h"
#include "sc_launch.h"

namespace scx {

enum { MODE_FUSED = 0, MODE_AGG = 1, MODE_APPLY = 2 };

template <typename R>
__device__ __forceinline__ R shfl_up_r(R x, int delta)
{
    return __shfl_up(x, (unsigned)delta, WAVE);
}
template <typename R>
__device__ __forceinline__ R shfl_down_r(R x, int delta)
{
    return __shfl_down(x, (unsigned)delta, WAVE);
}

__device__ __forceinline__ double fmx(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmx(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// Per-point coefficients in the arithmetic type of the pass.
template <typename R>
struct Coef;
template <>
struct Coef<double> {
    static __device__ __forceinline__ double wR(const OpArgs &P, int j) { return P.wR[j]; }
    static __device__ __forceinline__ double kR(const OpArgs &P, int w) { return P.kR[w]; }
    static __device__ __forceinline__ double kL(const OpArgs &P, int w) { return P.kL[w]; }
    static __device__ __forceinline__ double dpow(const OpArgs &P, int t) { return P.dpow[t]; }
    static __device__ __forceinline__ double d(const OpArgs &P) { return P.d; }
    static __device__ __forceinline__ double dlo(const OpArgs &) { return 0.0; }
};
template <>
struct Coef<float> {
    static __device__ __forceinline__ float wR(const OpArgs &P, int j) { return P.wRf[j]; }
    static __device__ __forceinline__ float kR(const OpArgs &P, int w) { return P.kRf[w]; }
    static __device__ __forceinline__ float kL(const OpArgs &P, int w) { return P.kLf[w]; }
    static __device__ __forceinline__ float dpow(const OpArgs &P, int t) { return P.dpowf[t]; }
    static __device__ __forceinline__ float d(const OpArgs &P) { return P.df; }
    static __device__ __forceinline__ float dlo(const OpArgs &P) { return P.dlo; }
};

// One step x <- d x + J of a sweep.  FP32 applies d as hi + lo: the rounding of d alone would bias
// every step of a segment the same way (up to S ulp at its end).
template <typename R>
__device__ __forceinline__ R sweep_step(R d, R dl, R x, R J)
{
    if constexpr (sizeof(R) == 4)
        return fmx(d, x, fmx(dl, x, J));
    else
        return fmx(d, x, J);
}

// x <- D y + x on (hi, lo) float pairs with D = Dh + Dl.  Dh yh is split exactly by an FMA
// (TwoProduct), its sum with xh exactly by Knuth's TwoSum; the remaining small terms go to the low
// part and the pair is renormalised.  Contraction is off so the transformations stay error-free.
__device__ __forceinline__ void comp_axpy(float Dh, float Dl, float yh, float yl, float &xh, float &xl)
{
#pragma clang fp contract(off)
    const float p = Dh * yh;
    const float pe = __builtin_fmaf(Dh, yh, -p);
    const float s = p + xh;
    const float bv = s - p;
    const float se = (p - (s - bv)) + (xh - bv);
    const float lo = ((pe + se) + xl) + __builtin_fmaf(Dh, yl, Dl * yh);
    const float h = s + lo;
    xl = lo - (h - s);
    xh = h;
}

// d^{S m} for 0 <= m < 2^12 from the binary powers d^{S 2^j}
__device__ __forceinline__ double dseg_pow(const OpArgs &P, int m)
{
    double r = 1.0;
#pragma unroll
    for (int j = 0; j < 12; ++j)
        if ((m >> j) & 1) r *= P.dseg[j];
    return r;
}

// A e^{-nu m} for an integer distance m >= 0, skipping exp when it underflows or A == 0
__device__ __forceinline__ double decayed(double A, double nu, int64_t m)
{
    if (A == 0.0 || m < 0) return 0.0;
    const double x = nu * (double)m;
    return x > 745.0 ? 0.0 : A * exp(-x);
}

template <typename T>
__device__ __forceinline__ T ldg(const T *p)
{
    return __builtin_nontemporal_load(p);
}

// Value at point p of the line at `base`: periodic wrap, or for Dirichlet lines the extension of
// the end interpolant to the order/2 points beyond each end (PassArgs::ext).
template <typename T, int ORDER>
__device__ __forceinline__ T line_value(const PassArgs &a, const T *v, int64_t base, int64_t p)
{
    const int64_t n = a.n;
    if (a.bc == 0) {
        if (p < 0) p += n;
        if (p >= n) p -= n;
        if (p < 0 || p >= n) {
            p %= n;
            if (p < 0) p += n;
        }
        return ldg(v + base + p * a.stride);
    }
    if (p >= 0 && p < n) return ldg(v + base + p * a.stride);
    const int m = p < 0 ? (int)(-p) : (int)(p - n + 1);  // distance beyond the end, 1..order/2
    if (m > ORDER / 2) return T(0);
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < ORDER; ++j) {
        const int64_t node = p < 0 ? j : n - 1 - j;
        s = fma(a.ext[m - 1][j], (double)ldg(v + base + node * a.stride), s);
    }
    return (T)s;
}

// ------------------------------------------------------------------------------------------
// The line pass.
//   T       element type in memory and per-point arithmetic type (double or float)
//   ORDER   4 or 6 (stencil width; halo H = ORDER/2)
//   S       points per thread segment
//   TC      lines per workgroup tile
//   CONTIG  true: the axis is contiguous (lanes run along the line);
//           false: strided axis (lanes run across TC adjacent lines)
//   MODE    FUSED: whole line in the tile; AGG: write chunk aggregates; APPLY: use chunk carries
//   NT      threads per workgroup
//   NOPS    operators applied to the same operand (1 or 2)
//   MULTI   partial sums with k > 1 (FUSED, periodic, one operator): the new operand of each
//           power is shared through the tile
// ------------------------------------------------------------------------------------------
template <bool B>
struct BoolC {
    static constexpr bool value = B;
};

template <typename T, int ORDER, int S, int TC, bool CONTIG, int MODE, int NT, int NOPS, bool MULTI>
__global__ void __launch_bounds__(NT) line_pass(const PassArgs a)
{
    using R = T;                                     // per-point arithmetic
    using K = Coef<T>;
    constexpr bool F32 = sizeof(T) == 4;
    constexpr int H = ORDER / 2;
    constexpr int NWIN = S + ORDER;                  // window: points seg0-H .. seg0+S+H-1
    constexpr int G = NT / TC;                       // segments per line in the tile
    constexpr int C = G * S;                         // chunk length
    constexpr int W = C + 2 * H;                     // tile points per line incl. halos
    constexpr int LS = (W + W / S + 1) | 1;          // padded, odd LDS line stride
    constexpr int GW = CONTIG ? (G < WAVE ? G : WAVE) : (WAVE / TC);  // segments per wave-part
    constexpr int NP = G / GW;                       // wave-parts per line
    constexpr int SL = CONTIG ? 1 : TC;              // lane distance between adjacent segments
    static_assert(G * TC == NT, "tile shape");
    static_assert(S <= MAXS && NWIN <= MAXWIN, "segment too long");
    static_assert(!MULTI || (MODE == MODE_FUSED && NOPS == 1), "powers of D are fused for one operator on whole lines");

    __shared__ T tile[TC * LS];
    __shared__ int64_t lbase[TC];
    __shared__ double xf_s[NOPS][TC][NP];   // per wave-part totals of the forward sweep
    __shared__ double xb_s[NOPS][TC][NP];   //                     ... of the backward sweep
    __shared__ double j0_s[NOPS][TC];       // J_R at x_0 (periodic: the wrapped last cell)
    __shared__ double cf_s[NOPS][TC][NP];   // forward carry into each wave-part
    __shared__ double cb_s[NOPS][TC][NP];   // backward carry into each wave-part
    __shared__ double ab_s[NOPS][TC][3];    // A' d^{cstart}, B' d^{N-(cstart+C-1)}, B' (see below)
    __shared__ double pw_s[NOPS][GW + 1];   // d^{S m}, m = 0..GW
    __shared__ double pp_s[NOPS][NP + 1];   // d^{S GW p}, p = 0..NP

    const int tid = threadIdx.x;
    const int c = CONTIG ? tid / G : tid % TC;
    const int g = CONTIG ? tid % G : tid / TC;
    const int gl = g % GW;
    const int part = g / GW;

    const int64_t n = a.n;
    const int64_t nchunks = (MODE == MODE_FUSED) ? 1 : a.nchunks;
    const int64_t blk = blockIdx.x;
    const int64_t chunk = (MODE == MODE_FUSED) ? 0 : blk % nchunks;
    const int64_t line0 = ((MODE == MODE_FUSED) ? blk : blk / nchunks) * TC;
    const int64_t cstart = chunk * C;
    const T *__restrict__ v = (const T *)a.v;

    if (tid < TC) {
        const int64_t L = line0 + tid;
        int64_t b = 0;
        if (L < a.nlines) b = (L / a.stride) * a.stride * n + (L % a.stride);
        lbase[tid] = b;
    }
    // decay tables (binary powers, computed once per workgroup)
    for (int e = tid; e < NOPS * (GW + 1 + NP + 1); e += NT) {
        const int o = e / (GW + 1 + NP + 1), m = e % (GW + 1 + NP + 1);
        if (m <= GW)
            pw_s[o][m] = dseg_pow(a.ops[o], m);
        else
            pp_s[o][m - GW - 1] = dseg_pow(a.ops[o], (m - GW - 1) * GW);
    }
    __syncthreads();

    // 1. tile load: all loads of a thread are issued before any LDS write; periodic halos wrap,
    //    Dirichlet halos are filled from the end interpolant afterwards
    {
        constexpr int FILL = (TC * W + NT - 1) / NT;
        const int ni = (int)n;
        const bool wrap_many = (a.bc == 0) && (ni < C + 2 * H);
        T vals[FILL];
        if (CONTIG && TC == 1) {
            // element e = tid + k NT is point p = cstart - H + e of the one line of the tile
            const int p0 = (int)cstart - H + tid;
            const T *rowp = v + lbase[0] + p0;
            const bool lok = line0 < a.nlines;
#pragma unroll
            for (int k = 0; k < FILL; ++k) {
                const int e = tid + k * NT;
                const int p = p0 + k * NT;
                T val = T(0);
                if (lok && e < W) {
                    if (p >= 0 && p < ni) {
                        val = ldg(rowp + k * NT);
                    } else if (a.bc == 0) {
                        int pw = p;
                        if (wrap_many) {
                            pw %= ni;
                            if (pw < 0) pw += ni;
                        } else {
                            pw = p < 0 ? p + ni : p - ni;
                        }
                        val = ldg(v + lbase[0] + pw);
                    }
                }
                vals[k] = val;
            }
        } else {
            const int64_t st = CONTIG ? 1 : a.stride;  // contiguous variants only run on stride-1 axes
            const int c0 = (int)cstart - H;
#pragma unroll
            for (int k = 0; k < FILL; ++k) {
                const int e = tid + k * NT;
                const int cc = CONTIG ? e / W : e % TC;
                const int q = CONTIG ? e % W : e / TC;
                int p = c0 + q;
                bool ok = (e < TC * W) && (line0 + cc < a.nlines);
                if (a.bc == 0) {
                    if (wrap_many) {
                        p %= ni;
                        if (p < 0) p += ni;
                    } else {
                        p = (p < 0) ? p + ni : (p >= ni ? p - ni : p);
                    }
                } else {
                    ok = ok && (p >= 0 && p < ni);
                }
                vals[k] = ok ? ldg(v + lbase[cc] + (int64_t)p * st) : T(0);
            }
        }
#pragma unroll
        for (int k = 0; k < FILL; ++k) {
            const int e = tid + k * NT;
            const int cc = CONTIG ? e / W : e % TC;
            const int q = CONTIG ? e % W : e / TC;
            if (e < TC * W) tile[cc * LS + q + q / S] = vals[k];
        }
    }
    if (a.bc == 1 && (cstart == 0 || cstart + C + H > n)) {
        __syncthreads();
        for (int e = tid; e < TC * 2 * H; e += NT) {
            const int cc = e / (2 * H), h = e % (2 * H);
            const int64_t p = (h < H) ? (int64_t)(-1 - h) : n + (h - H);
            const int64_t q = p - cstart + H;
            if (line0 + cc < a.nlines && q >= 0 && q < W) {
                const int qi = (int)q;
                tile[cc * LS + qi + qi / S] = line_value<T, ORDER>(a, v, lbase[cc], p);
            }
        }
    }
    __syncthreads();

    const bool line_ok = (line0 + c) < a.nlines;
    const int64_t seg0 = cstart + (int64_t)g * S;    // first point of this segment
    const int64_t n_loc = ((cstart + C < n) ? cstart + C : n) - cstart;  // real points in the tile
    const int s_last = (int)((n_loc - 1) / S);       // segment holding the tile's last real point
    const int t_last = (int)(n_loc - 1 - (int64_t)s_last * S);
    const int part_last = s_last / GW;
    // The general per-point rules (below) are needed only by waves holding padding past the line
    // end; elsewhere the two end rules are single corrections of a linear sweep: J_R(x_0) is
    // removed at t = 0 of the first segment, and on Dirichlet lines J_L(x_{n-1}) at t = S-1 of
    // the segment ending at x_{n-1}.  The choice is uniform per wave, so no wave runs both paths.
    const bool edge = __any(seg0 + S > n);
    const bool first_seg = (seg0 == 0);
    const bool dir_last = (a.bc == 1) && (seg0 + S == n);
    const int wbase = c * LS + g * (S + 1);

    T win[NWIN];
#pragma unroll
    for (int w = 0; w < NWIN; ++w) win[w] = tile[wbase + w + w / S];

    // the operand enters the result once: acc_mode 1 adds v, each D = v - L^{-1} v adds scale v
    double vc = (a.acc_mode == 1) ? 1.0 : 0.0;
    if (!MULTI) {
#pragma unroll
        for (int o = 0; o < NOPS; ++o)
            if (a.ops[o].k >= 1) vc += a.ops[o].scale;
    }
    const R vcoef = (R)vc;
    R outv[S];
#pragma unroll
    for (int t = 0; t < S; ++t) outv[t] = vcoef * win[t + H];

    // per-point rules of edge segments: J_R(x_0) = 0 (the cell left of x_0 is not part of the sweep;
    // periodic lines add it to I_R(b)), J_L(x_{n-1}) = 0 on Dirichlet lines, nothing past the end
    auto keepR = [&](int t) { const int64_t i = seg0 + t; return i > 0 && i < n; };
    auto keepL = [&](int t) { const int64_t i = seg0 + t; return i < n && !(a.bc == 1 && i == n - 1); };

    const int kk = MULTI ? a.ops[0].k : 1;
    for (int it = 0; it < kk; ++it) {
        // 2. segment totals of the forward and backward sweeps
        R aF[NOPS], aB[NOPS], jr0[NOPS];
#pragma unroll
        for (int o = 0; o < NOPS; ++o) {
            const OpArgs &P = a.ops[o];
            R sf = 0, sb = 0, j0 = 0;
            if (!edge) {
                if (P.op != 0) {
#pragma unroll
                    for (int w = 0; w < NWIN; ++w) sf = fmx(K::kR(P, w), win[w], sf);
                    // J_R at the segment's first point; excluded at x_0
                    R J0 = 0;
#pragma unroll
                    for (int j = 0; j < ORDER; ++j) J0 = fmx(K::wR(P, j), win[j], J0);
                    if (first_seg) {
                        sf = fmx(-K::dpow(P, S - 1), J0, sf);
                        j0 = J0;
                    }
                } else if (first_seg) {
#pragma unroll
                    for (int j = 0; j < ORDER; ++j) j0 = fmx(K::wR(P, j), win[j], j0);
                }
                if (P.op != 1) {
#pragma unroll
                    for (int w = 0; w < NWIN; ++w) sb = fmx(K::kL(P, w), win[w], sb);
                    if (a.bc == 1) {
                        // J_L at the segment's last point; excluded at x_{n-1} on Dirichlet lines
                        R JN = 0;
#pragma unroll
                        for (int j = 0; j < ORDER; ++j) JN = fmx(K::wR(P, ORDER - 1 - j), win[S + j], JN);
                        if (dir_last) sb = fmx(-K::dpow(P, S - 1), JN, sb);
                    }
                }
            } else {
#pragma unroll
                for (int t = 0; t < S; ++t) {
                    R JR = 0, JL = 0;
#pragma unroll
                    for (int j = 0; j < ORDER; ++j) {
                        JR = fmx(K::wR(P, j), win[t + j], JR);
                        JL = fmx(K::wR(P, ORDER - 1 - j), win[t + 1 + j], JL);
                    }
                    if (t == 0 && seg0 == 0) j0 = JR;
                    const int64_t i = seg0 + t;
                    if (i < n) sf = sweep_step(K::d(P), K::dlo(P), sf, keepR(t) ? JR : R(0));  // total at the last real point
                    sb = fmx(K::dpow(P, t), keepL(t) ? JL : R(0), sb);
                }
                if (P.op == 0) sf = 0;
                if (P.op == 1) sb = 0;
            }
            aF[o] = sf;
            aB[o] = sb;
            jr0[o] = j0;
        }

        // 3. scan of the segment totals along the line: within a wave by shuffles ...
        double ef[NOPS], eb[NOPS];
#pragma unroll
        for (int o = 0; o < NOPS; ++o) {
            const OpArgs &P = a.ops[o];
            double xf = (double)aF[o], xb = (double)aB[o];
            double e1 = 0.0, e2 = 0.0;
            if (P.op != 0) {
                if constexpr (F32) {
                    float xh = aF[o], xl = 0.f;
#pragma unroll
                    for (int s = 0, kx = 1; kx < GW; ++s, kx <<= 1) {
                        const float yh = shfl_up_r(xh, kx * SL), yl = shfl_up_r(xl, kx * SL);
                        if (gl >= kx) comp_axpy(P.dseg_hi[s], P.dseg_lo[s], yh, yl, xh, xl);
                    }
                    const float eh = shfl_up_r(xh, SL), el = shfl_up_r(xl, SL);
                    xf = (double)xh + (double)xl;
                    e1 = (gl == 0) ? 0.0 : (double)eh + (double)el;
                } else {
#pragma unroll
                    for (int s = 0, kx = 1; kx < GW; ++s, kx <<= 1) {
                        const double yf = shfl_up_r(xf, kx * SL);
                        if (gl >= kx) xf = fma(P.dseg[s], yf, xf);
                    }
                    e1 = shfl_up_r(xf, SL);
                    if (gl == 0) e1 = 0.0;
                }
            }
            if (P.op != 1) {
                if constexpr (F32) {
                    float xh = aB[o], xl = 0.f;
#pragma unroll
                    for (int s = 0, kx = 1; kx < GW; ++s, kx <<= 1) {
                        const float yh = shfl_down_r(xh, kx * SL), yl = shfl_down_r(xl, kx * SL);
                        if (gl + kx < GW) comp_axpy(P.dseg_hi[s], P.dseg_lo[s], yh, yl, xh, xl);
                    }
                    const float eh = shfl_down_r(xh, SL), el = shfl_down_r(xl, SL);
                    xb = (double)xh + (double)xl;
                    e2 = (gl == GW - 1) ? 0.0 : (double)eh + (double)el;
                } else {
#pragma unroll
                    for (int s = 0, kx = 1; kx < GW; ++s, kx <<= 1) {
                        const double yb = shfl_down_r(xb, kx * SL);
                        if (gl + kx < GW) xb = fma(P.dseg[s], yb, xb);
                    }
                    e2 = shfl_down_r(xb, SL);
                    if (gl == GW - 1) e2 = 0.0;
                }
            }
            ef[o] = e1;
            eb[o] = e2;
            if (line_ok) {
                if (part == part_last) {
                    if (g == s_last) xf_s[o][c][part] = fma(P.dpow[t_last + 1], e1, (double)aF[o]);
                } else if (gl == GW - 1) {
                    xf_s[o][c][part] = xf;
                }
                if (gl == 0) xb_s[o][c][part] = xb;
                if (g == 0) j0_s[o][c] = (cstart == 0) ? (double)jr0[o] : 0.0;
            }
        }
        __syncthreads();

        // ... and across the wave-parts and chunks by one thread per (operator, line), which also
        // forms the boundary constants
        if (tid < NOPS * TC) {
            const int o = tid / TC, cc = tid % TC;
            const OpArgs &P = a.ops[o];
            const int64_t L = line0 + cc;
            if (L < a.nlines) {
                const int64_t cidx = ((int64_t)o * a.nlines + L) * nchunks + chunk;
                double cf = 0.0, cb = 0.0;
                if (MODE == MODE_APPLY) {
                    cf = a.carry[2 * cidx + 0];
                    cb = a.carry[2 * cidx + 1];
                }
                double IRn = 0.0;
                for (int p2 = 0; p2 < NP; ++p2) {
                    cf_s[o][cc][p2] = cf;
                    if (p2 == part_last) {
                        const double dlp = (chunk == nchunks - 1) ? P.dlp_last : P.dlp_full;
                        IRn = fma(dlp, cf, xf_s[o][cc][p2]);  // I_R at the tile's last point
                    }
                    cf = fma(P.dpart, cf, xf_s[o][cc][p2]);
                }
                for (int p2 = NP - 1; p2 >= 0; --p2) {
                    cb_s[o][cc][p2] = cb;
                    cb = fma(P.dpart, cb, xb_s[o][cc][p2]);
                }
                const double IL0 = cb;  // I_L at the tile's first point
                double Ap = 0.0, Bp = 0.0;
                if (MODE == MODE_AGG) {
                    a.agg[3 * cidx + 0] = IRn;
                    a.agg[3 * cidx + 1] = IL0;
                    a.agg[3 * cidx + 2] = j0_s[o][cc];
                } else if (MODE == MODE_FUSED) {
                    if (a.bc == 0) {
                        Ap = fma(P.d, IRn, j0_s[o][cc]) * P.inv1mmu;
                        Bp = IL0 * P.inv1mmu;
                    } else {
                        const double ga = a.g ? a.g[2 * L + 0] : 0.0;
                        const double gb = a.g ? a.g[2 * L + 1] : 0.0;
                        if (P.op == 1) {
                            Ap = ga;
                        } else if (P.op == 0) {
                            Bp = gb;
                        } else {
                            // 0.5 I_L(a) + A + B mu = ga ; 0.5 I_R(b) + A mu + B = gb
                            const double r0 = ga - 0.5 * IL0, r1 = gb - 0.5 * IRn;
                            const double det = 1.0 - P.mu * P.mu;
                            Ap = 2.0 * (r0 - P.mu * r1) / det;
                            Bp = 2.0 * (r1 - P.mu * r0) / det;
                        }
                    }
                } else {
                    const int64_t ab = 2 * (int64_t)NOPS * a.nlines * nchunks + 2 * ((int64_t)o * a.nlines + L);
                    Ap = a.carry[ab + 0];
                    Bp = a.carry[ab + 1];
                }
                // boundary terms at the tile's first point and at the end of its last segment
                ab_s[o][cc][0] = decayed(Ap, P.nu, cstart);
                const int64_t eB = a.ncells - (cstart + C - 1);
                ab_s[o][cc][1] = (eB >= 0) ? decayed(Bp, P.nu, eB) : 0.0;
                ab_s[o][cc][2] = (eB >= 0) ? 0.0 : Bp;  // tiles reaching past N: per-segment powers
            }
        }
        __syncthreads();
        if (MODE == MODE_AGG) return;

        // 5. re-sweep from the exact carries and accumulate the result
        R fw[MULTI ? S : 1];
#pragma unroll
        for (int o = 0; o < NOPS; ++o) {
            const OpArgs &P = a.ops[o];
            const R d = K::d(P), dl = K::dlo(P);
            const double sgn = (P.k == 0) ? P.scale : -P.scale;
            const R cR = (R)((P.op == 1) ? sgn : (P.op == 2 ? 0.5 * sgn : 0.0));
            const R cL = (R)((P.op == 0) ? sgn : (P.op == 2 ? 0.5 * sgn : 0.0));
            // FP32 passes of L_0 on Dirichlet lines: the constants of the 2x2 end-value system can
            // exceed the result by ~1/(1 - mu) and cancel in it, so their terms are summed per point
            // in FP64 below and enter the result once, instead of riding through the FP32 sweeps
            const bool sepB = F32 && a.bc == 1 && P.op == 2;
            const int tsb = (a.ncells - seg0 < S - 1) ? (int)(a.ncells - seg0) : S - 1;
            if (P.op != 0) {
                // I_R at seg0 - 1; A' d^i obeys the same recurrence, so it enters once, at seg0
                R f = (R)fma(pw_s[o][gl], cf_s[o][c][part], ef[o]);
                const R a0 = sepB ? R(0) : (R)(ab_s[o][c][0] * pp_s[o][part] * pw_s[o][gl]);
                auto fwd = [&](auto E) {
#pragma unroll
                    for (int t = 0; t < S; ++t) {
                        R JR = 0;
#pragma unroll
                        for (int j = 0; j < ORDER; ++j) JR = fmx(K::wR(P, j), win[t + j], JR);
                        if (decltype(E)::value) {
                            if (!keepR(t)) JR = 0;
                        } else if (t == 0 && first_seg) {
                            JR = 0;
                        }
                        f = sweep_step(d, dl, f, JR);
                        if (t == 0) f += a0;
                        const R r = f;
                        if (MULTI)
                            fw[MULTI ? t : 0] = r;
                        else
                            outv[t] = fmx(cR, r, outv[t]);
                    }
                };
                if (edge)
                    fwd(BoolC<true>{});
                else
                    fwd(BoolC<false>{});
            }
            if (P.op != 1) {
                // I_L at seg0 + S and B' d^{N-i} at the segment's last point
                R b = (R)fma(pw_s[o][GW - 1 - gl], cb_s[o][c][part], eb[o]);
                // B' d^{N-i} obeys the same recurrence: it enters once, at the segment's last point
                // at or before x_N (tsb)
                const R b0 = sepB ? R(0)
                                  : (R)((ab_s[o][c][2] == 0.0)
                                            ? ab_s[o][c][1] * pp_s[o][NP - 1 - part] * pw_s[o][GW - 1 - gl]
                                            : decayed(ab_s[o][c][2], P.nu, a.ncells - seg0 - tsb));
                auto bwd = [&](auto E) {
#pragma unroll
                    for (int t = S - 1; t >= 0; --t) {
                        R JL = 0;
#pragma unroll
                        for (int j = 0; j < ORDER; ++j) JL = fmx(K::wR(P, ORDER - 1 - j), win[t + 1 + j], JL);
                        if (decltype(E)::value) {
                            if (!keepL(t)) JL = 0;
                        } else if (t == S - 1 && dir_last) {
                            JL = 0;
                        }
                        b = sweep_step(d, dl, b, JL);
                        if (decltype(E)::value) {
                            if (t == tsb) b += b0;
                        } else if (t == S - 1) {
                            b += b0;
                        }
                        const R r = b;
                        if (MULTI) {
                            const R rr = (P.op == 2) ? R(0.5) * (fw[MULTI ? t : 0] + r) : r;
                            const R wn = win[t + H] - rr;
                            outv[t] = fmx((R)P.scale, wn, outv[t]);
                            fw[MULTI ? t : 0] = wn;
                        } else {
                            outv[t] = fmx(cL, r, outv[t]);
                        }
                    }
                };
                if (edge)
                    bwd(BoolC<true>{});
                else
                    bwd(BoolC<false>{});
            } else if (MULTI) {
#pragma unroll
                for (int t = 0; t < S; ++t) {
                    const R wn = win[t + H] - fw[MULTI ? t : 0];
                    outv[t] = fmx((R)P.scale, wn, outv[t]);
                    fw[MULTI ? t : 0] = wn;
                }
            }
            if constexpr (F32) {
                if (sepB) {
                    // A' d^i (forward) and B' d^{N-i} (backward, from the last point at or before x_N)
                    const double ea = ab_s[o][c][0] * pp_s[o][part] * pw_s[o][gl];
                    const double eb0 = (ab_s[o][c][2] == 0.0)
                                           ? ab_s[o][c][1] * pp_s[o][NP - 1 - part] * pw_s[o][GW - 1 - gl]
                                           : decayed(ab_s[o][c][2], P.nu, a.ncells - seg0 - tsb);
                    const double h = 0.5 * sgn;
                    double eb = 0.0;
#pragma unroll
                    for (int t = S - 1; t >= 0; --t) {
                        eb *= P.d;
                        if (t == tsb) eb += eb0;
                        outv[t] += (R)(h * fma(ea, P.dpow[t], eb));
                    }
                }
            }
        }

        if (MULTI && it + 1 < kk) {
            // the new operand D^{it+1}[v] goes through the tile to the neighbouring segments
#pragma unroll
            for (int t = 0; t < S; ++t) {
                const int q = H + g * S + t;
                tile[c * LS + q + q / S] = (T)fw[MULTI ? t : 0];
            }
            __syncthreads();
            for (int e = tid; e < TC * W; e += NT) {
                const int cc = e / W;
                const int q = e % W;
                const int64_t p = (int64_t)q - H;
                if (p < 0 || p >= n) {
                    int64_t pw = p % n;
                    if (pw < 0) pw += n;
                    const int qs = (int)pw + H;
                    tile[cc * LS + q + q / S] = tile[cc * LS + qs + qs / S];
                }
            }
            __syncthreads();
#pragma unroll
            for (int w = 0; w < NWIN; ++w) win[w] = tile[wbase + w + w / S];
        }
    }

    // store: along x staged through the tile so that the global writes are coalesced; along y/z
    // the lanes of a wave already write full row segments of TC adjacent lines
    T *__restrict__ out = (T *)a.out;
    const T *acc = (const T *)a.acc;
    if (CONTIG) {
        __syncthreads();
#pragma unroll
        for (int t = 0; t < S; ++t) {
            const int q = H + g * S + t;
            tile[c * LS + q + q / S] = (T)outv[t];
        }
        __syncthreads();
        constexpr int STO = (TC * C + NT - 1) / NT;
        const int nl = (int)n_loc;
        if (TC == 1) {
            if (line0 < a.nlines) {
                T *op = out + lbase[0] + cstart + tid;
                const T *ap = acc + lbase[0] + cstart + tid;
#pragma unroll
                for (int k = 0; k < STO; ++k) {
                    const int q = tid + k * NT;
                    if (q < nl) {
                        T val = tile[(q + H) + (q + H) / S];
                        if (a.acc_mode == 2) val += ap[k * NT];
                        op[k * NT] = val;
                    }
                }
            }
        } else {
#pragma unroll
            for (int k = 0; k < STO; ++k) {
                const int e = tid + k * NT;
                const int cc = e / C;
                const int q = e % C;
                if (e < TC * C && line0 + cc < a.nlines && q < nl) {
                    const int64_t idx = lbase[cc] + cstart + q;
                    T val = tile[cc * LS + (q + H) + (q + H) / S];
                    if (a.acc_mode == 2) val += acc[idx];
                    out[idx] = val;
                }
            }
        }
    } else if (line_ok) {
        const int64_t st = a.stride;
        const int64_t i0 = lbase[c] + seg0 * st;
#pragma unroll
        for (int t = 0; t < S; ++t) {
            if (seg0 + t < n) {
                R val = outv[t];
                if (a.acc_mode == 2) val += acc[i0 + t * st];
                out[i0 + t * st] = (T)val;
            }
        }
    }
}


// ------------------------------------------------------------------------------------------
// Launch of one variant; variants whose LDS does not fit for T are not instantiated.
// ------------------------------------------------------------------------------------------
template <typename T, int ORDER, int S, int TC, bool CONTIG, int NT, int NOPS>
static hipError_t launch_shape(const PassArgs &a, int mode, bool multi, hipStream_t st)
{
    constexpr Variant V{S, TC, CONTIG, NT};
    if constexpr (V.lds_bytes((int)sizeof(T), ORDER, 2) > LDS_LIMIT) {
        return hipErrorInvalidValue;
    } else {
        const int64_t tiles = (a.nlines + TC - 1) / TC;
        if (mode == MODE_FUSED) {
            if (NOPS == 1 && multi)
                hipLaunchKernelGGL((line_pass<T, ORDER, S, TC, CONTIG, MODE_FUSED, NT, 1, true>), dim3(tiles), dim3(NT),
                                   0, st, a);
            else
                hipLaunchKernelGGL((line_pass<T, ORDER, S, TC, CONTIG, MODE_FUSED, NT, NOPS, false>), dim3(tiles),
                                   dim3(NT), 0, st, a);
            return hipGetLastError();
        }
        const dim3 grid(tiles * a.nchunks);
        if (mode == MODE_AGG)
            hipLaunchKernelGGL((line_pass<T, ORDER, S, TC, CONTIG, MODE_AGG, NT, NOPS, false>), grid, dim3(NT), 0, st, a);
        else
            hipLaunchKernelGGL((line_pass<T, ORDER, S, TC, CONTIG, MODE_APPLY, NT, NOPS, false>), grid, dim3(NT), 0, st,
                               a);
        return hipGetLastError();
    }
}

template <typename T, int ORDER, int S, int TC, bool CONTIG, int NT>
static hipError_t launch_variant(const PassArgs &a, int mode, bool multi, hipStream_t st)
{
    if (a.nops == 2) return launch_shape<T, ORDER, S, TC, CONTIG, NT, 2>(a, mode, false, st);
    return launch_shape<T, ORDER, S, TC, CONTIG, NT, 1>(a, mode, multi, st);
}

template <typename T, int ORDER>
hipError_t launch_line_pass_t(const PassArgs &a, int vid, int mode, bool multi, hipStream_t st)
{
    switch (vid) {
#define SC_CASE(id, S, TC, CONTIG, NT) \
    case id: return launch_variant<T, ORDER, S, TC, CONTIG, NT>(a, mode, multi, st);
        SC_VARIANTS(SC_CASE)
#undef SC_CASE
    }
    return hipErrorInvalidValue;
}

}  // namespace scx
