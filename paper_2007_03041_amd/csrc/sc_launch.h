// sc_launch.h -- host launchers of the library's kernels (library internal).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sc_device.h"

namespace scx {

enum { LMODE_FUSED = 0, LMODE_AGG = 1, LMODE_APPLY = 2, LMODE_SINGLE = 3, LMODE_WIN = 4 };

int num_variants();
const Variant &variant(int id);
// true if variant `vid` is built for elements of `elem` bytes (its LDS fits)
bool variant_built(int vid, int elem);

// elem = 8 (FP64) or 4 (FP32 data, mixed-precision carries)
hipError_t launch_line_pass(const PassArgs &a, int elem, int order, int vid, int mode, bool multi, hipStream_t st);
hipError_t launch_chunk_carry(const PassArgs &a, hipStream_t st);
// resets the chunk totals (n doubles) and the claim counter of a single-pass chunked launch
hipError_t launch_single_pass_reset(double *agg, int64_t n, uint32_t *sync, hipStream_t st);
// Pipelined strided pass (variants 5 and 12; lines of exactly C points, line count and stride
// multiples of TC, operand 16-byte aligned): see line_pass_pipe.
hipError_t launch_line_pass_pipe(const PassArgs &a, int elem, int order, int vid, hipStream_t st);
bool pipe_variant(int vid, int elem);
hipError_t launch_local_quad(const PassArgs &a, int elem, int order, void *JL, void *JR, hipStream_t st);
hipError_t launch_sweep(const PassArgs &a, int elem, const void *JL, const void *JR, void *IL, void *IR,
                        double *ends, hipStream_t st);
hipError_t launch_lincomb(int64_t nel, int elem, double a, const void *x, double b, const void *y, void *out,
                          hipStream_t st);

// One launch of the persistent batched pass (x lines of many instances, one tile shape).
struct BatchLaunch {
    const BatchArgs *table;  // device
    const BatchWork *work;   // device
    int64_t nwork;
    int64_t grid;            // workgroups (<= nwork)
    const void *v;
    void *out;
    const double *g;
    double *ws;
    int mode;                // LMODE_*
    int full;                // every work item's tile ends inside its line (no per-point end rules)
};

hipError_t launch_line_pass_batch(const BatchLaunch &b, int elem, int order, int vid, hipStream_t st);
// resident workgroups per CU of the batched pass (0 if the variant is not built for x lines)
int line_pass_batch_occupancy(int elem, int order, int vid, int mode, int full);
hipError_t launch_chunk_carry_batch(const BatchArgs *table, const int32_t *items, int nitems,
                                    const double *g, double *ws, hipStream_t st);

// one instantiation unit per (element type, order, full tiles or not): sc_lp_<type>_o<order>[_full].hip
template <typename T, int ORDER, bool FULL>
hipError_t launch_line_pass_t(const PassArgs &a, int vid, int mode, bool multi, hipStream_t st);
template <typename T, int ORDER>
hipError_t launch_line_pass_pipe_t(const PassArgs &a, int vid, hipStream_t st);
template <typename T, int ORDER, bool FULL>
hipError_t launch_line_pass_batch_t(const BatchLaunch &b, int vid, hipStream_t st);
template <typename T, int ORDER, bool FULL>
int line_pass_batch_occupancy_t(int vid, int mode);

double moment(int q, double nu);
void quad_weights(double nu, int m, const int *eta, double *w);

}  // namespace scx
