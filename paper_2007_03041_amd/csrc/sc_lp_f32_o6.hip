// Line-pass kernels for float elements, order-6 local quadrature (one unit per element type and
// order so the variants compile in parallel).
#include "sc_line_pass.h"

namespace scx {
template hipError_t launch_line_pass_t<float, 6, false>(const PassArgs &, int, int, bool, hipStream_t);
template hipError_t launch_line_pass_batch_t<float, 6, false>(const BatchLaunch &, int, hipStream_t);
template int line_pass_batch_occupancy_t<float, 6, false>(int, int);
}  // namespace scx
