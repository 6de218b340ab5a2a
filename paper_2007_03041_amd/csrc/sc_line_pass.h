// sc_line_pass.h -- the line-pass kernel of the successive-convolution fast summation (gfx950),
// included by one instantiation unit per (element type, order, full tiles or not).
//
// One pass applies up to two operators L_op^{-1} (or D = I - L_op^{-1} and its partial sums) along
// one axis of a dense array, line by line (Sec. 2.2: the directions stay uncoupled).
//
//   workgroup = a tile of TC lines x one chunk of C = G*S points of each line (+ order/2 halo)
//   thread    = one segment of S consecutive points of one line (G segments per line)
//
// Per workgroup, with one HBM read of the operand and one write of the result:
//   1. coalesced load of the tile into LDS in [line][point] layout.  Along x the lanes run along the
//      line and the tile transposes the data into per-thread segments (one pad element per segment
//      against bank conflicts); along y/z the lanes run across TC adjacent lines, the FP64 tile is
//      unpadded with a line stride of 1 mod 32, and the read-only aggregate launch skips the tile
//      and reads each window straight from memory.  Each thread then holds the window of S + order
//      operand values around its segment in registers.
//   2. segment totals of the two sweeps (Sec. 2.4 recurrences).  In the interior they are linear
//      in the window, so each is one dot product with coefficients precomputed on the host (kR,
//      kL); segments at line ends and in the padding use the point-by-point local integrals of
//      Sec. 2.4, eqs. (JR), (JL).  A Dirichlet line's one-sided end stencils are realised by
//      extending the line beyond each end with the interpolant of its end values, so the centred
//      stencil integrates the same polynomial there.
//   3. the segments are combined by a first-order linear-recurrence scan over (decay, value) pairs:
//      Kogge-Stone inside a wave (decay d^{S 2^j}; DPP lane moves on x tiles, shuffles on y/z
//      tiles) and one LDS exchange between the waves of a line (Sec. 3, eqs. (Left-/Right-moving
//      integral DD): a block's integral = its own sweep + attenuated contributions of the others).
//      Lines longer than one tile are chunked: an aggregate launch, then an apply launch that forms
//      its carries from the chunk totals (lines of more than 16 chunks: a carry launch between).
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

#include <algorithm>
#include <type_traits>

#include "sc_device.h"
#include "sc_launch.h"

namespace scx {

enum { MODE_FUSED = 0, MODE_AGG = 1, MODE_APPLY = 2, MODE_SINGLE = 3, MODE_WIN = 4 };

// Single-pass chunked launches: the chunk totals slots hold this bit pattern (a signalling NaN, which
// arithmetic never produces) until their tile publishes them.
constexpr uint64_t CHUNK_EMPTY = 0x7FF4DEADBEEF0001ull;
__device__ __forceinline__ bool chunk_empty(double x) { return (uint64_t)__double_as_longlong(x) == CHUNK_EMPTY; }
__device__ __forceinline__ void publish_agent(double *p, double v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double read_agent(const double *p)
{
    return __hip_atomic_load(const_cast<double *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

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

// A double moved between lanes by one DPP pattern (both halves alike).  Lanes whose source lies
// outside the pattern's range, or whose row is not in ROW_MASK, receive 0.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_d(double x)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, ROW_MASK, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, ROW_MASK, 0xF, true);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double readlane_d(double x, int lane)
{
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(x), lane),
                            __builtin_amdgcn_readlane(__double2loint(x), lane));
}
enum : int {
    DPP_ROW_SHL0 = 0x100,  // + k: row_shl:k (lane i of a row of 16 reads lane i + k of its row)
    DPP_ROW_SHR0 = 0x110,  // + k: row_shr:k (lane i reads lane i - k of its row)
    DPP_WAVE_SHL1 = 0x130, // lane i reads lane i + 1
    DPP_WAVE_SHR1 = 0x138, // lane i reads lane i - 1
    DPP_ROW_BCAST15 = 0x142, // the rows in the mask read lane 15 of the row below them
    DPP_ROW_BCAST31 = 0x143, // the rows in the mask read lane 31
};

// Inclusive scans x_i <- sum_j D^{|i-j|} a_j over the GW consecutive lanes of each wave part
// (GW = 16, 32 or 64; gl = lane mod GW), for the segment totals of contiguous tiles:
// Kogge-Stone with DPP row shifts inside each row of 16 lanes (decays D^k from dseg), then the
// carries across rows with per-lane decays pw[m] = D^m.  Forward: rows 1 and 3 take lane 15 of the
// row below by row broadcast, then rows 2 and 3 take lane 31.  Backward: row r takes the first
// lane of row r + 1, read as a scalar, from the top row down.
template <int GW, class OA>
__device__ __forceinline__ double scan_fwd_dpp(double x, const OA &P, const double *pw, int gl)
{
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        if ((1 << s) < GW) {
            double y;
            if (s == 0) y = dpp_d<DPP_ROW_SHR0 + 1, 0xF>(x);
            else if (s == 1) y = dpp_d<DPP_ROW_SHR0 + 2, 0xF>(x);
            else if (s == 2) y = dpp_d<DPP_ROW_SHR0 + 4, 0xF>(x);
            else y = dpp_d<DPP_ROW_SHR0 + 8, 0xF>(x);
            x = fma(P.dseg[s], y, x);
        }
    }
    if constexpr (GW > 16) x = fma(pw[(gl & 15) + 1], dpp_d<DPP_ROW_BCAST15, 0xA>(x), x);
    if constexpr (GW > 32) x = fma(pw[gl >= 32 ? gl - 31 : 0], dpp_d<DPP_ROW_BCAST31, 0xC>(x), x);
    return x;
}
template <int GW, class OA>
__device__ __forceinline__ double scan_bwd_dpp(double x, const OA &P, const double *pw, int gl)
{
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        if ((1 << s) < GW) {
            double y;
            if (s == 0) y = dpp_d<DPP_ROW_SHL0 + 1, 0xF>(x);
            else if (s == 1) y = dpp_d<DPP_ROW_SHL0 + 2, 0xF>(x);
            else if (s == 2) y = dpp_d<DPP_ROW_SHL0 + 4, 0xF>(x);
            else y = dpp_d<DPP_ROW_SHL0 + 8, 0xF>(x);
            x = fma(P.dseg[s], y, x);
        }
    }
    const int lane = (int)(__lane_id());
    if constexpr (GW == 32) {
        // two wave parts per wave: rows 0 and 2 take the first lane of rows 1 and 3
        const double c1 = readlane_d(x, 16), c3 = readlane_d(x, 48);
        if ((lane & 16) == 0) x = fma(pw[16 - (gl & 15)], lane < 32 ? c1 : c3, x);
    } else if constexpr (GW == 64) {
        const double c3 = readlane_d(x, 48);
        if ((lane >> 4) == 2) x = fma(pw[48 - gl], c3, x);
        const double c2 = readlane_d(x, 32);
        if ((lane >> 4) == 1) x = fma(pw[32 - gl], c2, x);
        const double c1 = readlane_d(x, 16);
        if ((lane >> 4) == 0) x = fma(pw[16 - gl], c1, x);
    }
    return x;
}

__device__ __forceinline__ double fmx(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmx(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// Per-point coefficients in the arithmetic type of the pass.
template <typename R>
struct Coef;
// (templated on the argument block's type so that blocks read through the constant address space
// keep their scalar loads)
template <>
struct Coef<double> {
    template <class OA> static __device__ __forceinline__ double wR(const OA &P, int j) { return P.wR[j]; }
    template <class OA> static __device__ __forceinline__ double kR(const OA &P, int w) { return P.kR[w]; }
    template <class OA> static __device__ __forceinline__ double kL(const OA &P, int w) { return P.kL[w]; }
    template <class OA> static __device__ __forceinline__ double dpow(const OA &P, int t) { return P.dpow[t]; }
    template <class OA> static __device__ __forceinline__ double d(const OA &P) { return P.d; }
    template <class OA> static __device__ __forceinline__ double dlo(const OA &) { return 0.0; }
};
template <>
struct Coef<float> {
    template <class OA> static __device__ __forceinline__ float wR(const OA &P, int j) { return P.wRf[j]; }
    template <class OA> static __device__ __forceinline__ float kR(const OA &P, int w) { return P.kRf[w]; }
    template <class OA> static __device__ __forceinline__ float kL(const OA &P, int w) { return P.kLf[w]; }
    template <class OA> static __device__ __forceinline__ float dpow(const OA &P, int t) { return P.dpowf[t]; }
    template <class OA> static __device__ __forceinline__ float d(const OA &P) { return P.df; }
    template <class OA> static __device__ __forceinline__ float dlo(const OA &P) { return P.dlo; }
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

// The scans above on (hi, lo) float pairs with the compensated step comp_axpy, for FP32 tiles.  A
// lane whose source lies outside the pattern keeps its pair, as in the shuffle form; per-lane decays
// pw[m] (FP64) enter as hi + lo.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_f(float x)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROW_MASK, 0xF, true));
}
__device__ __forceinline__ void comp_axpy_d(double D, float yh, float yl, float &xh, float &xl)
{
    const float Dh = (float)D;
    comp_axpy(Dh, (float)(D - (double)Dh), yh, yl, xh, xl);
}
template <int GW, class OA>
__device__ __forceinline__ void scan_fwd_dpp_f(float &xh, float &xl, const OA &P, const double *pw, int gl)
{
    const int r16 = gl & 15;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        if ((1 << s) < GW) {
            float yh, yl;
            if (s == 0) yh = dpp_f<DPP_ROW_SHR0 + 1, 0xF>(xh), yl = dpp_f<DPP_ROW_SHR0 + 1, 0xF>(xl);
            else if (s == 1) yh = dpp_f<DPP_ROW_SHR0 + 2, 0xF>(xh), yl = dpp_f<DPP_ROW_SHR0 + 2, 0xF>(xl);
            else if (s == 2) yh = dpp_f<DPP_ROW_SHR0 + 4, 0xF>(xh), yl = dpp_f<DPP_ROW_SHR0 + 4, 0xF>(xl);
            else yh = dpp_f<DPP_ROW_SHR0 + 8, 0xF>(xh), yl = dpp_f<DPP_ROW_SHR0 + 8, 0xF>(xl);
            if (r16 >= (1 << s)) comp_axpy(P.dseg_hi[s], P.dseg_lo[s], yh, yl, xh, xl);
        }
    }
    if constexpr (GW > 16) {
        const float yh = dpp_f<DPP_ROW_BCAST15, 0xA>(xh), yl = dpp_f<DPP_ROW_BCAST15, 0xA>(xl);
        if (gl & 16) comp_axpy_d(pw[r16 + 1], yh, yl, xh, xl);
    }
    if constexpr (GW > 32) {
        const float yh = dpp_f<DPP_ROW_BCAST31, 0xC>(xh), yl = dpp_f<DPP_ROW_BCAST31, 0xC>(xl);
        if (gl >= 32) comp_axpy_d(pw[gl - 31], yh, yl, xh, xl);
    }
}
template <int GW, class OA>
__device__ __forceinline__ void scan_bwd_dpp_f(float &xh, float &xl, const OA &P, const double *pw, int gl)
{
    const int r16 = gl & 15;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        if ((1 << s) < GW) {
            float yh, yl;
            if (s == 0) yh = dpp_f<DPP_ROW_SHL0 + 1, 0xF>(xh), yl = dpp_f<DPP_ROW_SHL0 + 1, 0xF>(xl);
            else if (s == 1) yh = dpp_f<DPP_ROW_SHL0 + 2, 0xF>(xh), yl = dpp_f<DPP_ROW_SHL0 + 2, 0xF>(xl);
            else if (s == 2) yh = dpp_f<DPP_ROW_SHL0 + 4, 0xF>(xh), yl = dpp_f<DPP_ROW_SHL0 + 4, 0xF>(xl);
            else yh = dpp_f<DPP_ROW_SHL0 + 8, 0xF>(xh), yl = dpp_f<DPP_ROW_SHL0 + 8, 0xF>(xl);
            if (r16 + (1 << s) < 16 && r16 + (1 << s) < GW) comp_axpy(P.dseg_hi[s], P.dseg_lo[s], yh, yl, xh, xl);
        }
    }
    const int lane = (int)(__lane_id());
    auto rd = [](float v, int l) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l)); };
    if constexpr (GW == 32) {
        const float h1 = rd(xh, 16), l1 = rd(xl, 16), h3 = rd(xh, 48), l3 = rd(xl, 48);
        if ((lane & 16) == 0) comp_axpy_d(pw[16 - r16], lane < 32 ? h1 : h3, lane < 32 ? l1 : l3, xh, xl);
    } else if constexpr (GW == 64) {
        const float h3 = rd(xh, 48), l3 = rd(xl, 48);
        if ((lane >> 4) == 2) comp_axpy_d(pw[48 - gl], h3, l3, xh, xl);
        const float h2 = rd(xh, 32), l2 = rd(xl, 32);
        if ((lane >> 4) == 1) comp_axpy_d(pw[32 - gl], h2, l2, xh, xl);
        const float h1 = rd(xh, 16), l1 = rd(xl, 16);
        if ((lane >> 4) == 0) comp_axpy_d(pw[16 - gl], h1, l1, xh, xl);
    }
}

// d^{S m} for 0 <= m < 2^12 from the binary powers d^{S 2^j}
template <class OA>
__device__ __forceinline__ double dseg_pow(const OA &P, int m)
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
    if (m == 0) return A;
    const double x = nu * (double)m;
    return x > 745.0 ? 0.0 : A * exp(-x);
}

// d^m for 0 <= m < 128 by binary powers of the operator's decay table (no exp on the device)
template <class OA>
__device__ __forceinline__ double dpow_small(const OA &P, int m)
{
    static_assert(MAXS >= 16, "decay table reaches d^16");
    const double d16 = P.dpow[16], d32 = d16 * d16, d64 = d32 * d32;
    double r = (m & 1) ? P.dpow[1] : 1.0;
    if (m & 2) r *= P.dpow[2];
    if (m & 4) r *= P.dpow[4];
    if (m & 8) r *= P.dpow[8];
    if (m & 16) r *= d16;
    if (m & 32) r *= d32;
    if (m & 64) r *= d64;
    return r;
}

// Boundary constants A', B' of one line from its sweep totals: I_R at the last point (IRn), I_L at
// the first point (IL0) and J_R at x_0 (J0).  Periodic lines (Sec. 2.3): A' = (d IRn + J0)/(1 - mu),
// B' = IL0/(1 - mu).  Dirichlet lines: the end values ga, gb fix them; for L_0 through the 2x2
// system 0.5 I_L(a) + A + B mu = ga, 0.5 I_R(b) + A mu + B = gb (A' = 2A, B' = 2B).
template <class OA>
__device__ __forceinline__ void boundary_constants(const OA &P, int bc, double IRn, double IL0, double J0, double ga,
                                                   double gb, double &Ap, double &Bp)
{
    Ap = 0.0;
    Bp = 0.0;
    if (bc == 0) {
        Ap = fma(P.d, IRn, J0) * P.inv1mmu;
        Bp = IL0 * P.inv1mmu;
    } else if (P.op == 1) {
        Ap = ga;
    } else if (P.op == 0) {
        Bp = gb;
    } else {
        const double r0 = ga - 0.5 * IL0, r1 = gb - 0.5 * IRn;
        Ap = (r0 - P.mu * r1) * P.dir2inv;
        Bp = (r1 - P.mu * r0) * P.dir2inv;
    }
}

// Chunk carries of line L, operator P, from the per-chunk totals ag[3 ch + {0, 1, 2}] (forward,
// backward, J_R at the chunk's first point) of its nch chunks: the forward carry into chunk `want`
// (cf), the backward carry into it (cb), and the line totals IRn = I_R at the last point and
// IL0 = I_L at the first (Sec. 3: a block's integral is its own sweep plus the attenuated sweeps
// of the blocks before it).
// The totals are read four chunks at a time, so their loads overlap instead of each waiting behind
// the previous step of the recurrence.
template <class OA>
__device__ __forceinline__ void chunk_scan(const OA &P, const double *ag, int64_t nch, int64_t want, double &cf,
                                           double &cb, double &IRn, double &IL0)
{
    constexpr int B = 4;
    double E = 0.0;
    for (int64_t c0 = 0; c0 < nch; c0 += B) {
        double t[B];
#pragma unroll
        for (int j = 0; j < B; ++j) t[j] = (c0 + j < nch) ? ag[3 * (c0 + j) + 0] : 0.0;
#pragma unroll
        for (int j = 0; j < B; ++j) {
            const int64_t ch = c0 + j;
            if (ch < nch) {
                if (ch == want) cf = E;
                E = fma(ch == nch - 1 ? P.dchunk_last : P.dchunk, E, t[j]);
            }
        }
    }
    double F = 0.0;
    for (int64_t c1 = nch - 1; c1 >= 0; c1 -= B) {
        double t[B];
#pragma unroll
        for (int j = 0; j < B; ++j) t[j] = (c1 - j >= 0) ? ag[3 * (c1 - j) + 1] : 0.0;
#pragma unroll
        for (int j = 0; j < B; ++j) {
            const int64_t ch = c1 - j;
            if (ch >= 0) {
                if (ch == want) cb = F;
                F = fma(ch == nch - 1 ? P.dchunk_last : P.dchunk, F, t[j]);
            }
        }
    }
    IRn = E;
    IL0 = F;
}

// chunk_scan over totals already in registers: forward totals tf[ch], backward totals tb[ch] of
// nch <= M chunks (same operations in the same order)
template <int M, class OA>
__device__ __forceinline__ void chunk_scan_regs(const OA &P, const double (&tf)[M], const double (&tb)[M], int64_t nch,
                                                int64_t want, double &cf, double &cb, double &IRn, double &IL0)
{
    double E = 0.0;
#pragma unroll
    for (int ch = 0; ch < M; ++ch) {
        if (ch < nch) {
            if (ch == want) cf = E;
            E = fma(ch == nch - 1 ? P.dchunk_last : P.dchunk, E, tf[ch]);
        }
    }
    double F = 0.0;
#pragma unroll
    for (int ch = M - 1; ch >= 0; --ch) {
        if (ch < nch) {
            if (ch == want) cb = F;
            F = fma(ch == nch - 1 ? P.dchunk_last : P.dchunk, F, tb[ch]);
        }
    }
    IRn = E;
    IL0 = F;
}

// A wave-uniform 64-bit value the compiler cannot see through (the asm exists in the device pass
// only; the host pass never runs kernel bodies).
__device__ __forceinline__ uint64_t launder_sgpr(uint64_t x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    asm volatile("" : "+s"(x));
#endif
    return x;
}

// Direct global-to-LDS load of 16 bytes a lane: lane l's bytes land at lds_dst + 16 l (lds_dst
// wave-uniform).  (The builtin exists in the device pass only.)
template <typename T>
__device__ __forceinline__ void load_lds16(const T *src, T *lds_dst)
{
#if defined(__HIP_DEVICE_COMPILE__)
    // (cache policy nt: the pipelined strided tiles' operand is read once)
    __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void *)lds_dst, 16, 0, 2);
#endif
}

// Workgroup barrier for LDS traffic only: waits for this wave's LDS operations, not for its
// outstanding global loads -- a direct-to-LDS prefetch of the next tile keeps streaming across it
// (a __syncthreads fence would wait for it).  The memory clobber keeps the compiler from moving
// memory accesses across.
__device__ __forceinline__ void barrier_lds()
{
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Operand loads are ordinary cached loads: a window's halo rows are read again by the neighbouring
// segment's thread, and a streaming (non-temporal) hint evicted them before that second read (the
// aggregate launch then fetched 14 % more than the field and ran 25 % longer).
template <typename T>
__device__ __forceinline__ T ldg(const T *p)
{
    return *p;
}

// streaming load (non-temporal): operands that no other tile of the pass reads again
template <typename T>
__device__ __forceinline__ T ldg_stream(const T *p)
{
    return __builtin_nontemporal_load(p);
}

// Value at point p of the line at `base`: periodic wrap, or for Dirichlet lines the extension of
// the end interpolant to the order/2 points beyond each end (PassArgs::ext).
template <typename T, int ORDER, class PA>
__device__ __forceinline__ T line_value(const PA &a, const T *v, int64_t base, int64_t p)
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

// Operand values each thread of a tile loads: TC lines x (C + order) points over NT threads.
constexpr int tile_fill(int order, int S, int TC, int NT) { return (TC * ((NT / TC) * S + order) + NT - 1) / NT; }

// Issues the global loads of one tile's operand values into registers: element e = tid + k NT of
// the tile (line e / W, point cstart - order/2 + e % W along x; line e % TC, point e / TC along
// y/z) goes to vals[k].  lb holds the TC line bases.  Periodic halos wrap; points outside a
// Dirichlet line read 0 (they are filled from the end interpolant once the tile is in LDS).
// FULL: the line length is a whole number of chunks, so on one-line tiles only the first and the
// last group of NT elements can fall outside the line.
// STREAM: strided tiles of whole lines read with streaming loads (no other tile of the pass reads
// their operand again).
template <typename T, int ORDER, int S, int TC, bool CONTIG, int NT, bool FULL, class PA, bool STREAM = false>
__device__ __forceinline__ void load_tile(T (&vals)[tile_fill(ORDER, S, TC, NT)], const PA &a, const T *v,
                                          const int64_t *lb, int64_t line0, int64_t cstart, int tid)
{
    auto ld = [](const T *p) { return STREAM ? ldg_stream(p) : ldg(p); };
    constexpr int H = ORDER / 2;
    constexpr int C = (NT / TC) * S;
    constexpr int W = C + 2 * H;
    constexpr int FILL = tile_fill(ORDER, S, TC, NT);
    const int ni = (int)a.n;
    const bool wrap_many = (a.bc == 0) && (ni < C + 2 * H);
    if (CONTIG && TC == 1) {
        // element e = tid + k NT is point p = cstart - H + e of the one line of the tile
        const int p0 = (int)cstart - H + tid;
        const T *rowp = v + lb[0] + p0;
        // (the tile's line exists or not for the whole workgroup: one uniform branch, so no element's
        // load sits in a branch of its own)
        if (line0 >= a.nlines) {
#pragma unroll
            for (int k = 0; k < FILL; ++k) vals[k] = T(0);
            return;
        }
        // one load per element, from the in-line address plus the wrap of a periodic halo point: two
        // alternative loads into one register would serialise the loads behind register reuse
#pragma unroll
        for (int k = 0; k < FILL; ++k) {
            const int e = tid + k * NT;
            const int p = p0 + k * NT;
            if (FULL && NT >= ORDER && k > 0 && k < FILL - 1) {
                // elements NT .. C - 1 of the tile: points cstart - H + NT .. cstart + C - H - 1
                vals[k] = ldg(rowp + k * NT);
                continue;
            }
            bool ok = e < W;
            int dp = 0;
            if (p < 0 || p >= ni) {
                if (a.bc == 0) {
                    int pw = p;
                    if (wrap_many) {
                        pw %= ni;
                        if (pw < 0) pw += ni;
                    } else {
                        pw = p < 0 ? p + ni : p - ni;
                    }
                    dp = pw - p;
                } else {
                    ok = false;
                }
            }
            vals[k] = ok ? ldg(rowp + k * NT + dp) : T(0);
        }
    } else if (CONTIG && FULL && NT >= ORDER * TC) {
        // full multi-line x tiles: thread tid serves line tid / TPL, points q = tid % TPL + k TPL of
        // it (TPL = NT / TC threads per line, coalesced along the line); the middle groups lie inside
        // the line.  A thread whose line does not exist reads line 0 instead (its results are never
        // stored), so no load depends on a per-lane condition.
        constexpr int TPL = NT / TC;
        const int cc = tid / TPL;
        const int q0 = tid % TPL;
        const int64_t lbase_c = (line0 + cc < a.nlines) ? lb[cc] : lb[0];
        const T *rowp = v + lbase_c + ((int)cstart - H + q0);
#pragma unroll
        for (int k = 0; k < FILL; ++k) {
            const int q = q0 + k * TPL;
            if (k > 0 && k < FILL - 1) {
                vals[k] = ldg(rowp + k * TPL);
                continue;
            }
            const int p = (int)cstart - H + q;
            bool ok = q < W;
            int dp = 0;
            if (p < 0 || p >= ni) {
                if (a.bc == 0) {
                    int pw = p;
                    if (wrap_many) {
                        pw %= ni;
                        if (pw < 0) pw += ni;
                    } else {
                        pw = p < 0 ? p + ni : p - ni;
                    }
                    dp = pw - p;
                } else {
                    ok = false;
                }
            }
            vals[k] = ok ? ldg(rowp + k * TPL + dp) : T(0);
        }
    } else if (!CONTIG && (int)cstart - H >= 0 && (int)cstart - H + W <= ni) {
        // strided tile inside its lines: thread tid loads line tid % TC, rows tid / TC + k NT / TC
        const int cc = tid % TC;
        const bool ok = line0 + cc < a.nlines;
        const T *q = v + lb[cc] + (int64_t)((int)cstart - H + tid / TC) * a.stride;
        const int64_t step = (int64_t)(NT / TC) * a.stride;
#pragma unroll
        for (int k = 0; k < FILL; ++k) {
            vals[k] = (ok && tid + k * NT < TC * W) ? ld(q) : T(0);
            q += step;
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
            vals[k] = ok ? ld(v + lb[cc] + (int64_t)p * st) : T(0);
        }
    }
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
//   FULL    every tile of the launch is full (the line length is a multiple of the chunk length):
//           no segment reaches past a line end, and the per-point end rules are compiled out
// ------------------------------------------------------------------------------------------
template <bool B>
struct BoolC {
    static constexpr bool value = B;
};

// Array pointers of one pass.
struct Ptrs {
    const void *v;
    const void *acc;
    void *out;
    const double *g;
    double *agg;
    const double *carry;
};

// Workgroups are dealt to the 8 XCDs of the chip round-robin (block b on XCD b mod 8).  The apply
// tiles of one line group read the same chunk totals; numbering the logical tiles XCD by XCD keeps a
// line group's chunks on one XCD, so those totals come from its L2 once.
__device__ __forceinline__ int64_t xcd_grouped(int64_t b, int64_t nblocks)
{
    constexpr int64_t NX = 8;
    const int64_t whole = (nblocks / NX) * NX;
    return b < whole ? (b % NX) * (whole / NX) + b / NX : b;
}

// Single-power passes are held to 128 VGPRs (4 waves per SIMD): left alone, the compiler gave the
// one-operator x passes 129-131 and so one workgroup per CU less.  The fused powers of D keep their
// registers (about 190-230 in FP64, 2 waves): held to 168 they spill, and measured slower along
// every axis (512^3 FP64 S_3: x 0.85 -> 0.96, y 1.08 -> 1.16, z 1.20 -> 1.31 ms).
template <typename T, int ORDER, int S, int TC, bool CONTIG, int MODE, int NT, int NOPS, bool MULTI, bool FULL>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(MULTI ? 1 : 4)))
line_pass(const PassArgs a)
{
    constexpr bool PIPE = false;
    constexpr bool pipe_first = false;
    constexpr int64_t pipe_next = -1;
    const Ptrs pt{a.v, a.acc, a.out, a.g, a.agg, a.carry};
    int64_t blk = (MODE == MODE_APPLY || MODE == MODE_WIN) ? xcd_grouped(blockIdx.x, gridDim.x) : (int64_t)blockIdx.x;
    if constexpr (MODE == MODE_SINGLE) {
        // tiles are claimed in order (line group by line group, its chunks in turn), so every tile
        // a tile waits for has been claimed by a running workgroup or will be by the next one to start
        __shared__ uint32_t claim_s;
        if (threadIdx.x == 0) claim_s = atomicAdd(a.sync, 1u);
        __syncthreads();
        blk = claim_s;
    }
    const int tid_in = threadIdx.x;
#include "sc_line_pass_body.inc"
}


// Persistent strided pass over whole lines (y/z lines that fit one tile): workgroup b takes line
// tiles b, b + grid, ...  Each tile's operand goes straight from memory to LDS; the loads of the
// next tile are issued as soon as the windows of the current one are in registers, so they stream
// in during the current tile's scans, re-sweeps and stores.
template <typename T, int ORDER, int S, int TC, int NT, int NOPS>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4)))
line_pass_pipe(const PassArgs a_arg, int64_t ntiles)
{
    constexpr bool CONTIG = false;
    constexpr int MODE = MODE_FUSED;
    constexpr bool MULTI = false;
    constexpr bool FULL = true;
    constexpr bool PIPE = true;
    (void)a_arg;
    // The argument block is read through the kernel-argument segment (the explicit arguments start
    // at its offset 0), with the pointer laundered per tile: otherwise the loop-invariant coefficient
    // reads are hoisted out of the loop and their scalar registers spill.
    typedef const PassArgs __attribute__((address_space(4))) CPassArgs;
    for (int64_t blk = blockIdx.x; blk < ntiles; blk += gridDim.x) {
        const bool pipe_first = blk == (int64_t)blockIdx.x;
        const int64_t pipe_next = blk + gridDim.x < ntiles ? blk + gridDim.x : -1;
        const auto &a = *(const CPassArgs *)launder_sgpr((uint64_t)__builtin_amdgcn_kernarg_segment_ptr());
        const Ptrs pt{a.v, a.acc, a.out, a.g, a.agg, a.carry};
        // the thread index is laundered per tile, as in the batched kernel
        int tid_in = threadIdx.x;
        asm volatile("" : "+v"(tid_in));
        {
#include "sc_line_pass_body.inc"
        }
        barrier_lds();  // the next tile reuses the LDS tables (its loads are waited for at its start)
    }
}

// Persistent pass over a batch of independent instances: workgroup b takes work items b, b + grid,
// ... of the list; each item is one tile of one instance, whose argument block (coefficients, sizes,
// element offsets of its arrays) lives in a device table.  Items of one launch share the tile shape.
// FULL: every item's tile ends inside its line.  Register budgets as measured on the ragged batch:
// 168 VGPRs (3 waves per SIMD) for general tiles and for FP64 exact-carry applies, whose
// 128-register form spills (3.43 vs 3.06 ms); 128 for the rest (FP32 applies 2.29 vs 2.59 ms,
// FP64 windowed applies 3.02 vs 2.91 ms).
template <typename T, int ORDER, int S, int TC, bool CONTIG, int MODE, int NT, bool FULL>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu((FULL && (MODE != MODE_APPLY || sizeof(T) == 4)) ? 4 : 3)))
line_pass_batch(const BatchArgs *__restrict__ table,
                                                     const BatchWork *__restrict__ work, int64_t nwork,
                                                     const T *vbase, T *obase, const double *gbase, double *wsbase)
{
    constexpr int NOPS = 1;
    constexpr bool MULTI = false;
    constexpr bool PIPE = false;
    constexpr bool pipe_first = false;
    constexpr int64_t pipe_next = -1;
    // the table and work list are read-only for the whole launch: reading them through the constant
    // address space makes every per-instance parameter a scalar load, as for kernel arguments
    typedef const BatchArgs __attribute__((address_space(4))) CBatchArgs;
    typedef const BatchWork __attribute__((address_space(4))) CBatchWork;
    const CBatchArgs *ctab = (const CBatchArgs *)table;
    const CBatchWork *cwork = (const CBatchWork *)work;
    for (int64_t w = blockIdx.x; w < nwork; w += gridDim.x) {
        const int32_t item = cwork[w].item;
        const int64_t tile_id = cwork[w].tile;
        const auto &b = ctab[item];
        const auto &a = b.a;
        const Ptrs pt{vbase + b.v_off, nullptr, obase + b.v_off, b.g_off >= 0 ? gbase + b.g_off : nullptr,
                      wsbase + b.agg_off, wsbase + b.carry_off};
        const int64_t blk = tile_id;
        // the thread index is laundered per item: computations on it are then not hoisted out of
        // the loop, where they would stay live across the whole tile (+40 VGPRs)
        int tid_in = threadIdx.x;
        asm volatile("" : "+v"(tid_in));
        {
#include "sc_line_pass_body.inc"
        }
        __syncthreads();  // the next item reuses the LDS tables
    }
}

// ------------------------------------------------------------------------------------------
// Launch of one variant; variants whose LDS does not fit for T are not instantiated.
// ------------------------------------------------------------------------------------------
template <typename T, int ORDER, bool FULL, int S, int TC, bool CONTIG, int NT, int NOPS>
static hipError_t launch_shape(const PassArgs &a, int mode, bool multi, hipStream_t st)
{
    constexpr Variant V{S, TC, CONTIG, NT};
    if constexpr (V.lds_bytes((int)sizeof(T), ORDER, 2) > LDS_LIMIT) {
        return hipErrorInvalidValue;
    } else {
        const int64_t tiles = (a.nlines + TC - 1) / TC;
        if (mode == MODE_FUSED) {
            if (NOPS == 1 && multi)
                hipLaunchKernelGGL((line_pass<T, ORDER, S, TC, CONTIG, MODE_FUSED, NT, 1, true, FULL>), dim3(tiles), dim3(NT),
                                   0, st, a);
            else
                hipLaunchKernelGGL((line_pass<T, ORDER, S, TC, CONTIG, MODE_FUSED, NT, NOPS, false, FULL>), dim3(tiles),
                                   dim3(NT), 0, st, a);
            return hipGetLastError();
        }
        const dim3 grid(tiles * a.nchunks);
        if (mode == MODE_AGG)
            hipLaunchKernelGGL((line_pass<T, ORDER, S, TC, CONTIG, MODE_AGG, NT, NOPS, false, FULL>), grid, dim3(NT), 0, st, a);
        else if (mode == MODE_SINGLE)
            hipLaunchKernelGGL((line_pass<T, ORDER, S, TC, CONTIG, MODE_SINGLE, NT, NOPS, false, FULL>), grid, dim3(NT), 0,
                               st, a);
        else if (mode == MODE_WIN) {
            if constexpr (CONTIG && TC == 1 && NOPS == 1)
                hipLaunchKernelGGL((line_pass<T, ORDER, S, TC, CONTIG, MODE_WIN, NT, 1, false, FULL>), grid, dim3(NT), 0, st, a);
            else
                return hipErrorInvalidValue;
        } else
            hipLaunchKernelGGL((line_pass<T, ORDER, S, TC, CONTIG, MODE_APPLY, NT, NOPS, false, FULL>), grid, dim3(NT), 0, st,
                               a);
        return hipGetLastError();
    }
}

template <typename T, int ORDER, bool FULL, int S, int TC, bool CONTIG, int NT>
static hipError_t launch_variant(const PassArgs &a, int mode, bool multi, hipStream_t st)
{
    if (FULL && a.n % ((NT / TC) * S) != 0 && !(mode == MODE_WIN && a.n >= (NT / TC) * S)) return hipErrorInvalidValue;
    if (a.nops == 2) return launch_shape<T, ORDER, FULL, S, TC, CONTIG, NT, 2>(a, mode, false, st);
    return launch_shape<T, ORDER, FULL, S, TC, CONTIG, NT, 1>(a, mode, multi, st);
}

template <typename T, int ORDER, bool FULL>
hipError_t launch_line_pass_t(const PassArgs &a, int vid, int mode, bool multi, hipStream_t st)
{
    switch (vid) {
#define SC_CASE(id, S, TC, CONTIG, NT) \
    case id: return launch_variant<T, ORDER, FULL, S, TC, CONTIG, NT>(a, mode, multi, st);
        SC_VARIANTS(SC_CASE)
#undef SC_CASE
    }
    return hipErrorInvalidValue;
}


// ------------------------------------------------------------------------------------------
// Pipelined strided passes (whole lines of C points, FULL tiles)
// ------------------------------------------------------------------------------------------
// static LDS of a pipelined tile: [point][line] tile without padding plus the tables of Variant
template <typename T, int ORDER, int S, int TC, int NT, int NOPS>
constexpr int pipe_lds_bytes()
{
    constexpr Variant V{S, TC, false, NT};
    return V.lds_bytes((int)sizeof(T), ORDER, NOPS) - TC * ((((V.C() + ORDER + 31) & ~31) + 1)) * (int)sizeof(T) +
           (V.C() + ORDER) * TC * (int)sizeof(T) + 64;
}

template <typename T, int ORDER, int S, int TC, int NT, int NOPS>
static hipError_t launch_pipe_shape(const PassArgs &a, hipStream_t st)
{
    if constexpr (pipe_lds_bytes<T, ORDER, S, TC, NT, NOPS>() > LDS_LIMIT) {
        return hipErrorInvalidValue;
    } else {
    const int64_t ntiles = a.nlines / TC;
    // resident workgroups of the whole device (one grid's worth), found once per process
    static const int64_t resident = [] {
        int dev = 0, cus = 0, occ = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &occ, reinterpret_cast<const void *>(&line_pass_pipe<T, ORDER, S, TC, NT, NOPS>), NT, 0) != hipSuccess)
            return int64_t(0);
        return (int64_t)(occ > 0 ? occ : 1) * cus;
    }();
    if (resident <= 0) return hipErrorInvalidValue;
    const int64_t grid = std::min<int64_t>(ntiles, resident);
    hipLaunchKernelGGL((line_pass_pipe<T, ORDER, S, TC, NT, NOPS>), dim3((unsigned)grid), dim3(NT), 0, st, a, ntiles);
    return hipGetLastError();
    }
}

template <typename T, int ORDER>
hipError_t launch_line_pass_pipe_t(const PassArgs &a, int vid, hipStream_t st)
{
    constexpr bool F64 = sizeof(T) == 8;
    if (vid == 5 && F64) return a.nops == 2 ? launch_pipe_shape<T, ORDER, 16, 16, 512, 2>(a, st)
                                            : launch_pipe_shape<T, ORDER, 16, 16, 512, 1>(a, st);
    if (vid == 12) return a.nops == 2 ? launch_pipe_shape<T, ORDER, 16, 32, 1024, 2>(a, st)
                                      : launch_pipe_shape<T, ORDER, 16, 32, 1024, 1>(a, st);
    return hipErrorInvalidValue;
}

// ------------------------------------------------------------------------------------------
// Batched launches (contiguous variants only)
// ------------------------------------------------------------------------------------------
// Shapes the batched kernel is instantiated for: every x-line tile, and the strided tiles of 16 or 32
// lines with S = 16 (the shapes of single y/z passes).
constexpr bool batch_built(const Variant &V) { return V.contig || (V.S == 16 && (V.TC == 16 || V.TC == 32)); }

template <typename T, int ORDER, int S, int TC, bool CONTIG, int NT, bool FULL>
static hipError_t launch_batch_shape(const BatchLaunch &b, hipStream_t st)
{
    constexpr Variant V{S, TC, CONTIG, NT};
    if constexpr (!batch_built(V) || V.lds_bytes((int)sizeof(T), ORDER, 2) > LDS_LIMIT) {
        return hipErrorInvalidValue;
    } else {
        const dim3 grid((unsigned)b.grid), block(NT);
        const T *v = (const T *)b.v;
        T *o = (T *)b.out;
        if (b.mode == MODE_FUSED)
            hipLaunchKernelGGL((line_pass_batch<T, ORDER, S, TC, CONTIG, MODE_FUSED, NT, FULL>), grid, block, 0, st, b.table,
                               b.work, b.nwork, v, o, b.g, b.ws);
        else if (b.mode == MODE_AGG)
            hipLaunchKernelGGL((line_pass_batch<T, ORDER, S, TC, CONTIG, MODE_AGG, NT, FULL>), grid, block, 0, st, b.table,
                               b.work, b.nwork, v, o, b.g, b.ws);
        else if (b.mode == MODE_WIN) {
            if constexpr (TC == 1)
                hipLaunchKernelGGL((line_pass_batch<T, ORDER, S, TC, CONTIG, MODE_WIN, NT, FULL>), grid, block, 0, st, b.table,
                                   b.work, b.nwork, v, o, b.g, b.ws);
            else
                return hipErrorInvalidValue;
        } else
            hipLaunchKernelGGL((line_pass_batch<T, ORDER, S, TC, CONTIG, MODE_APPLY, NT, FULL>), grid, block, 0, st, b.table,
                               b.work, b.nwork, v, o, b.g, b.ws);
        return hipGetLastError();
    }
}

template <typename T, int ORDER, int S, int TC, bool CONTIG, int NT, bool FULL>
static int batch_occupancy_shape(int mode)
{
    constexpr Variant V{S, TC, CONTIG, NT};
    if constexpr (!batch_built(V) || V.lds_bytes((int)sizeof(T), ORDER, 2) > LDS_LIMIT) {
        return 0;
    } else {
        int occ = 0;
        hipError_t e;
        if (mode == MODE_FUSED)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &occ, reinterpret_cast<const void *>(&line_pass_batch<T, ORDER, S, TC, CONTIG, MODE_FUSED, NT, FULL>), NT, 0);
        else if (mode == MODE_AGG)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &occ, reinterpret_cast<const void *>(&line_pass_batch<T, ORDER, S, TC, CONTIG, MODE_AGG, NT, FULL>), NT, 0);
        else if (mode == MODE_WIN) {
            if constexpr (TC == 1)
                e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
                    &occ, reinterpret_cast<const void *>(&line_pass_batch<T, ORDER, S, TC, CONTIG, MODE_WIN, NT, FULL>), NT,
                    0);
            else
                return 0;
        } else
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &occ, reinterpret_cast<const void *>(&line_pass_batch<T, ORDER, S, TC, CONTIG, MODE_APPLY, NT, FULL>), NT, 0);
        return e == hipSuccess ? occ : 0;
    }
}

template <typename T, int ORDER, bool FULL>
hipError_t launch_line_pass_batch_t(const BatchLaunch &b, int vid, hipStream_t st)
{
    switch (vid) {
#define SC_CASE(id, S, TC, CONTIG, NT) \
    case id: return launch_batch_shape<T, ORDER, S, TC, CONTIG, NT, FULL>(b, st);
        SC_VARIANTS(SC_CASE)
#undef SC_CASE
    }
    return hipErrorInvalidValue;
}

template <typename T, int ORDER, bool FULL>
int line_pass_batch_occupancy_t(int vid, int mode)
{
    switch (vid) {
#define SC_CASE(id, S, TC, CONTIG, NT) \
    case id: return batch_occupancy_shape<T, ORDER, S, TC, CONTIG, NT, FULL>(mode);
        SC_VARIANTS(SC_CASE)
#undef SC_CASE
    }
    return 0;
}

}  // namespace scx
