// Line-pass kernels for float elements, order-6 local quadrature, on lines that are a whole number
// of chunks (no segment past a line end), and batched tiles that end inside their line.
#include "sc_line_pass.h"

namespace scx {
template hipError_t launch_line_pass_t<float, 6, true>(const PassArgs &, int, int, bool, hipStream_t);
template hipError_t launch_line_pass_pipe_t<float, 6>(const PassArgs &, int, hipStream_t);
template hipError_t launch_line_pass_batch_t<float, 6, true>(const BatchLaunch &, int, hipStream_t);
template int line_pass_batch_occupancy_t<float, 6, true>(int, int);
}  // namespace scx
