// Line-pass kernels for double elements, order-4 local quadrature, on lines that are a whole number
// of chunks (no segment past a line end), and batched tiles that end inside their line.
#include "sc_line_pass.h"

namespace scx {
template hipError_t launch_line_pass_t<double, 4, true>(const PassArgs &, int, int, bool, hipStream_t);
template hipError_t launch_line_pass_pipe_t<double, 4>(const PassArgs &, int, hipStream_t);
template hipError_t launch_line_pass_batch_t<double, 4, true>(const BatchLaunch &, int, hipStream_t);
template int line_pass_batch_occupancy_t<double, 4, true>(int, int);
}  // namespace scx
