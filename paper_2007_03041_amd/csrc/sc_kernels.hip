// sc_kernels.hip -- gfx950 kernels of the successive-convolution fast summation.
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
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sc_device.h"
#include "sc_launch.h"

namespace scx {

enum { MODE_FUSED = 0, MODE_AGG = 1, MODE_APPLY = 2 };

__device__ __forceinline__ double shfl_up_d(double x, int delta)
{
    return __shfl_up(x, (unsigned)delta, WAVE);
}
__device__ __forceinline__ double shfl_down_d(double x, int delta)
{
    return __shfl_down(x, (unsigned)delta, WAVE);
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
//   T       element type in memory (double)
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
    const int64_t myline = line0 + c;
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
    double vcoef = (a.acc_mode == 1) ? 1.0 : 0.0;
    if (!MULTI) {
#pragma unroll
        for (int o = 0; o < NOPS; ++o)
            if (a.ops[o].k >= 1) vcoef += a.ops[o].scale;
    }
    double outv[S];
#pragma unroll
    for (int t = 0; t < S; ++t) outv[t] = vcoef * (double)win[t + H];

    // per-point rules of edge segments: J_R(x_0) = 0 (the cell left of x_0 is not part of the sweep;
    // periodic lines add it to I_R(b)), J_L(x_{n-1}) = 0 on Dirichlet lines, nothing past the end
    auto keepR = [&](int t) { const int64_t i = seg0 + t; return i > 0 && i < n; };
    auto keepL = [&](int t) { const int64_t i = seg0 + t; return i < n && !(a.bc == 1 && i == n - 1); };

    const int kk = MULTI ? a.ops[0].k : 1;
    for (int it = 0; it < kk; ++it) {
        // 2. segment totals of the forward and backward sweeps
        double aF[NOPS], aB[NOPS], jr0[NOPS];
#pragma unroll
        for (int o = 0; o < NOPS; ++o) {
            const OpArgs &P = a.ops[o];
            double sf = 0.0, sb = 0.0, j0 = 0.0;
            if (!edge) {
                if (P.op != 0) {
#pragma unroll
                    for (int w = 0; w < NWIN; ++w) sf = fma(P.kR[w], (double)win[w], sf);
                    // J_R at the segment's first point; excluded at x_0
                    double J0 = 0.0;
#pragma unroll
                    for (int j = 0; j < ORDER; ++j) J0 = fma(P.wR[j], (double)win[j], J0);
                    if (first_seg) {
                        sf = fma(-P.dpow[S - 1], J0, sf);
                        j0 = J0;
                    }
                } else if (first_seg) {
#pragma unroll
                    for (int j = 0; j < ORDER; ++j) j0 = fma(P.wR[j], (double)win[j], j0);
                }
                if (P.op != 1) {
#pragma unroll
                    for (int w = 0; w < NWIN; ++w) sb = fma(P.kL[w], (double)win[w], sb);
                    if (a.bc == 1) {
                        // J_L at the segment's last point; excluded at x_{n-1} on Dirichlet lines
                        double JN = 0.0;
#pragma unroll
                        for (int j = 0; j < ORDER; ++j) JN = fma(P.wR[ORDER - 1 - j], (double)win[S + j], JN);
                        if (dir_last) sb = fma(-P.dpow[S - 1], JN, sb);
                    }
                }
            } else {
#pragma unroll
                for (int t = 0; t < S; ++t) {
                    double JR = 0.0, JL = 0.0;
#pragma unroll
                    for (int j = 0; j < ORDER; ++j) {
                        JR = fma(P.wR[j], (double)win[t + j], JR);
                        JL = fma(P.wR[ORDER - 1 - j], (double)win[t + 1 + j], JL);
                    }
                    if (t == 0 && seg0 == 0) j0 = JR;
                    const int64_t i = seg0 + t;
                    if (i < n) sf = fma(P.d, sf, keepR(t) ? JR : 0.0);  // total at the last real point
                    sb = fma(P.dpow[t], keepL(t) ? JL : 0.0, sb);
                }
                if (P.op == 0) sf = 0.0;
                if (P.op == 1) sb = 0.0;
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
            double xf = aF[o], xb = aB[o];
            double e1 = 0.0, e2 = 0.0;
            if (P.op != 0) {
#pragma unroll
                for (int s = 0, kx = 1; kx < GW; ++s, kx <<= 1) {
                    const double yf = shfl_up_d(xf, kx * SL);
                    if (gl >= kx) xf = fma(P.dseg[s], yf, xf);
                }
                e1 = shfl_up_d(xf, SL);
                if (gl == 0) e1 = 0.0;
            }
            if (P.op != 1) {
#pragma unroll
                for (int s = 0, kx = 1; kx < GW; ++s, kx <<= 1) {
                    const double yb = shfl_down_d(xb, kx * SL);
                    if (gl + kx < GW) xb = fma(P.dseg[s], yb, xb);
                }
                e2 = shfl_down_d(xb, SL);
                if (gl == GW - 1) e2 = 0.0;
            }
            ef[o] = e1;
            eb[o] = e2;
            if (line_ok) {
                if (part == part_last) {
                    if (g == s_last) xf_s[o][c][part] = fma(P.dpow[t_last + 1], e1, aF[o]);
                } else if (gl == GW - 1) {
                    xf_s[o][c][part] = xf;
                }
                if (gl == 0) xb_s[o][c][part] = xb;
                if (g == 0) j0_s[o][c] = (cstart == 0) ? jr0[o] : 0.0;
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
        double fw[MULTI ? S : 1];
#pragma unroll
        for (int o = 0; o < NOPS; ++o) {
            const OpArgs &P = a.ops[o];
            const double d = P.d;
            const double sgn = (P.k == 0) ? P.scale : -P.scale;
            const double cR = (P.op == 1) ? sgn : (P.op == 2 ? 0.5 * sgn : 0.0);
            const double cL = (P.op == 0) ? sgn : (P.op == 2 ? 0.5 * sgn : 0.0);
            if (P.op != 0) {
                // I_R at seg0 - 1; A' d^i obeys the same recurrence, so it enters once, at seg0
                double f = fma(pw_s[o][gl], cf_s[o][c][part], ef[o]);
                const double a0 = ab_s[o][c][0] * pp_s[o][part] * pw_s[o][gl];
                auto fwd = [&](auto E) {
#pragma unroll
                    for (int t = 0; t < S; ++t) {
                        double JR = 0.0;
#pragma unroll
                        for (int j = 0; j < ORDER; ++j) JR = fma(P.wR[j], (double)win[t + j], JR);
                        if (decltype(E)::value) {
                            if (!keepR(t)) JR = 0.0;
                        } else if (t == 0 && first_seg) {
                            JR = 0.0;
                        }
                        f = fma(d, f, JR);
                        if (t == 0) f += a0;
                        const double r = f;
                        if (MULTI)
                            fw[MULTI ? t : 0] = r;
                        else
                            outv[t] = fma(cR, r, outv[t]);
                    }
                };
                if (edge)
                    fwd(BoolC<true>{});
                else
                    fwd(BoolC<false>{});
            }
            if (P.op != 1) {
                // I_L at seg0 + S and B' d^{N-i} at the segment's last point
                double b = fma(pw_s[o][GW - 1 - gl], cb_s[o][c][part], eb[o]);
                // B' d^{N-i} obeys the same recurrence: it enters once, at the segment's last point
                // at or before x_N (tsb)
                const int tsb = (a.ncells - seg0 < S - 1) ? (int)(a.ncells - seg0) : S - 1;
                const double b0 = (ab_s[o][c][2] == 0.0)
                                      ? ab_s[o][c][1] * pp_s[o][NP - 1 - part] * pw_s[o][GW - 1 - gl]
                                      : decayed(ab_s[o][c][2], P.nu, a.ncells - seg0 - tsb);
                auto bwd = [&](auto E) {
#pragma unroll
                    for (int t = S - 1; t >= 0; --t) {
                        double JL = 0.0;
#pragma unroll
                        for (int j = 0; j < ORDER; ++j) JL = fma(P.wR[ORDER - 1 - j], (double)win[t + 1 + j], JL);
                        if (decltype(E)::value) {
                            if (!keepL(t)) JL = 0.0;
                        } else if (t == S - 1 && dir_last) {
                            JL = 0.0;
                        }
                        b = fma(d, b, JL);
                        if (decltype(E)::value) {
                            if (t == tsb) b += b0;
                        } else if (t == S - 1) {
                            b += b0;
                        }
                        const double r = b;
                        if (MULTI) {
                            const double rr = (P.op == 2) ? 0.5 * (fw[MULTI ? t : 0] + r) : r;
                            const double wn = (double)win[t + H] - rr;
                            outv[t] = fma(P.scale, wn, outv[t]);
                            fw[MULTI ? t : 0] = wn;
                        } else {
                            outv[t] = fma(cL, r, outv[t]);
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
                    const double wn = (double)win[t + H] - fw[MULTI ? t : 0];
                    outv[t] = fma(P.scale, wn, outv[t]);
                    fw[MULTI ? t : 0] = wn;
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
                double val = outv[t];
                if (a.acc_mode == 2) val += (double)acc[i0 + t * st];
                out[i0 + t * st] = (T)val;
            }
        }
    }
}

// Chunk carries of chunked passes: one thread per (op, line) walks the chunk totals in both
// directions (Sec. 3, eqs. (Left-/Right-moving integral DD) with exact attenuation factors) and
// forms the boundary constants.
__global__ void __launch_bounds__(256) chunk_carry(const PassArgs a, int64_t chunk_len)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)a.nops * a.nlines) return;
    const int o = (int)(idx / a.nlines);
    const int64_t L = idx % a.nlines;
    const OpArgs &P = a.ops[o];
    const int64_t nch = a.nchunks;
    const double *ag = a.agg + ((int64_t)o * a.nlines + L) * nch * 3;
    double *cr = const_cast<double *>(a.carry) + ((int64_t)o * a.nlines + L) * nch * 2;
    const int64_t len_last = a.n - (nch - 1) * chunk_len;
    const double d_last = exp(-P.nu * (double)len_last);
    double E = 0.0;
    for (int64_t ch = 0; ch < nch; ++ch) {
        cr[2 * ch + 0] = E;
        E = fma(ch == nch - 1 ? d_last : P.dchunk, E, ag[3 * ch + 0]);
    }
    double F = 0.0;
    for (int64_t ch = nch - 1; ch >= 0; --ch) {
        cr[2 * ch + 1] = F;
        F = fma(ch == nch - 1 ? d_last : P.dchunk, F, ag[3 * ch + 1]);
    }
    const double IRn = E, IL0 = F, J0 = ag[2];
    double Ap = 0.0, Bp = 0.0;
    if (a.bc == 0) {
        Ap = fma(P.d, IRn, J0) * P.inv1mmu;
        Bp = IL0 * P.inv1mmu;
    } else {
        const double ga = a.g ? a.g[2 * L + 0] : 0.0;
        const double gb = a.g ? a.g[2 * L + 1] : 0.0;
        if (P.op == 1) {
            Ap = ga;
        } else if (P.op == 0) {
            Bp = gb;
        } else {
            const double r0 = ga - 0.5 * IL0, r1 = gb - 0.5 * IRn;
            const double det = 1.0 - P.mu * P.mu;
            Ap = 2.0 * (r0 - P.mu * r1) / det;
            Bp = 2.0 * (r1 - P.mu * r0) / det;
        }
    }
    double *ab = const_cast<double *>(a.carry) + 2 * (int64_t)a.nops * a.nlines * nch + 2 * idx;
    ab[0] = Ap;
    ab[1] = Bp;
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

template <typename T>
__global__ void __launch_bounds__(256) axpy_kernel(int64_t nel, double s, const T *x, T *y, int init)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nel) y[i] = init ? (T)(s * (double)x[i]) : (T)fma(s, (double)x[i], (double)y[i]);
}

// ------------------------------------------------------------------------------------------
// Host launchers
// ------------------------------------------------------------------------------------------
static const Variant kVariants[] = {
    {16, 16, true, 256},    // 0: contiguous, lines <= 256
    {16, 4, true, 256},     // 1: contiguous, lines <= 1024
    {16, 1, true, 256},     // 2: contiguous, lines <= 4096
    {16, 1, true, 512},     // 3: contiguous, lines <= 8192 (chunked beyond)
    {16, 16, false, 256},   // 4: strided, 16 lines x 256
    {16, 16, false, 512},   // 5: strided, 16 lines x 512
    {16, 16, false, 1024},  // 6: strided, 16 lines x 1024 (chunked beyond 4096)
    {16, 4, false, 1024},   // 7: strided, 4 lines x 4096
    {8, 16, false, 1024},   // 8: strided, 16 lines x 512, short segments
    {8, 1, true, 512},      // 9: contiguous, lines <= 4096, short segments
};
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

int num_variants() { return kNumVariants; }
const Variant &variant(int id) { return kVariants[id]; }

template <int ORDER, int S, int TC, bool CONTIG, int NT, int NOPS>
static hipError_t launch_v2(const PassArgs &a, int mode, bool multi, hipStream_t st)
{
    const int64_t tiles = (a.nlines + TC - 1) / TC;
    if (mode == MODE_FUSED) {
        if (NOPS == 1 && multi)
            hipLaunchKernelGGL((line_pass<double, ORDER, S, TC, CONTIG, MODE_FUSED, NT, 1, true>), dim3(tiles), dim3(NT), 0, st, a);
        else
            hipLaunchKernelGGL((line_pass<double, ORDER, S, TC, CONTIG, MODE_FUSED, NT, NOPS, false>), dim3(tiles), dim3(NT), 0, st, a);
        return hipGetLastError();
    }
    const dim3 grid(tiles * a.nchunks);
    if (mode == MODE_AGG)
        hipLaunchKernelGGL((line_pass<double, ORDER, S, TC, CONTIG, MODE_AGG, NT, NOPS, false>), grid, dim3(NT), 0, st, a);
    else
        hipLaunchKernelGGL((line_pass<double, ORDER, S, TC, CONTIG, MODE_APPLY, NT, NOPS, false>), grid, dim3(NT), 0, st, a);
    return hipGetLastError();
}

template <int ORDER, int S, int TC, bool CONTIG, int NT>
static hipError_t launch_v(const PassArgs &a, int mode, bool multi, hipStream_t st)
{
    if (a.nops == 2) return launch_v2<ORDER, S, TC, CONTIG, NT, 2>(a, mode, false, st);
    return launch_v2<ORDER, S, TC, CONTIG, NT, 1>(a, mode, multi, st);
}

template <int ORDER>
static hipError_t launch_order(const PassArgs &a, int vid, int mode, bool multi, hipStream_t st)
{
    switch (vid) {
    case 0: return launch_v<ORDER, 16, 16, true, 256>(a, mode, multi, st);
    case 1: return launch_v<ORDER, 16, 4, true, 256>(a, mode, multi, st);
    case 2: return launch_v<ORDER, 16, 1, true, 256>(a, mode, multi, st);
    case 3: return launch_v<ORDER, 16, 1, true, 512>(a, mode, multi, st);
    case 4: return launch_v<ORDER, 16, 16, false, 256>(a, mode, multi, st);
    case 5: return launch_v<ORDER, 16, 16, false, 512>(a, mode, multi, st);
    case 6: return launch_v<ORDER, 16, 16, false, 1024>(a, mode, multi, st);
    case 7: return launch_v<ORDER, 16, 4, false, 1024>(a, mode, multi, st);
    case 8: return launch_v<ORDER, 8, 16, false, 1024>(a, mode, multi, st);
    case 9: return launch_v<ORDER, 8, 1, true, 512>(a, mode, multi, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_line_pass(const PassArgs &a, int order, int vid, int mode, bool multi, hipStream_t st)
{
    if (order == 4) return launch_order<4>(a, vid, mode, multi, st);
    return launch_order<6>(a, vid, mode, multi, st);
}

hipError_t launch_chunk_carry(const PassArgs &a, int64_t chunk_len, hipStream_t st)
{
    const int64_t nthr = (int64_t)a.nops * a.nlines;
    hipLaunchKernelGGL(chunk_carry, dim3((nthr + 255) / 256), dim3(256), 0, st, a, chunk_len);
    return hipGetLastError();
}

hipError_t launch_local_quad(const PassArgs &a, int order, void *JL, void *JR, hipStream_t st)
{
    const int64_t total = a.n * a.nlines;
    const dim3 grid((total + 255) / 256);
    if (order == 4)
        hipLaunchKernelGGL((local_quad_kernel<double, 4>), grid, dim3(256), 0, st, a, (double *)JL, (double *)JR);
    else
        hipLaunchKernelGGL((local_quad_kernel<double, 6>), grid, dim3(256), 0, st, a, (double *)JL, (double *)JR);
    return hipGetLastError();
}

hipError_t launch_sweep(const PassArgs &a, const void *JL, const void *JR, void *IL, void *IR, double *ends, hipStream_t st)
{
    hipLaunchKernelGGL((sweep_kernel<double>), dim3(a.nlines), dim3(256), 0, st, a, (const double *)JL,
                       (const double *)JR, (double *)IL, (double *)IR, ends);
    return hipGetLastError();
}

hipError_t launch_axpy(int64_t nel, double s, const void *x, void *y, int init, hipStream_t st)
{
    hipLaunchKernelGGL((axpy_kernel<double>), dim3((nel + 255) / 256), dim3(256), 0, st, nel, s,
                       (const double *)x, (double *)y, init);
    return hipGetLastError();
}

}  // namespace scx
