// Line-pass kernels for double elements, order-4 local quadrature (one unit per element type and
// order so the variants compile in parallel).
#include "sc_line_pass.h"

namespace scx {
template hipError_t launch_line_pass_t<double, 4, false>(const PassArgs &, int, int, bool, hipStream_t);
template hipError_t launch_line_pass_batch_t<double, 4, false>(const BatchLaunch &, int, hipStream_t);
template int line_pass_batch_occupancy_t<double, 4, false>(int, int);
}  // namespace scx
