// sc_launch.h -- host launchers of the kernels in sc_kernels.hip (library internal).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sc_device.h"

namespace scx {

enum { LMODE_FUSED = 0, LMODE_AGG = 1, LMODE_APPLY = 2 };

int num_variants();
const Variant &variant(int id);

hipError_t launch_line_pass(const PassArgs &a, int order, int vid, int mode, bool multi, hipStream_t st);
hipError_t launch_chunk_carry(const PassArgs &a, int64_t chunk_len, hipStream_t st);
hipError_t launch_local_quad(const PassArgs &a, int order, void *JL, void *JR, hipStream_t st);
hipError_t launch_sweep(const PassArgs &a, const void *JL, const void *JR, void *IL, void *IR,
                        double *ends, hipStream_t st);
hipError_t launch_axpy(int64_t nel, double s, const void *x, void *y, int init, hipStream_t st);

double moment(int q, double nu);
void quad_weights(double nu, int m, const int *eta, double *w);

}  // namespace scx
