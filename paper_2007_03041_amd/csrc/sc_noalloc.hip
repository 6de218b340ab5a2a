// sc_noalloc.hip -- sc_apply_invL_noalloc: sc_apply_invL for callers that cannot allocate device
// memory (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
//
// The chunked passes of sc_apply_invL keep per-(line, chunk) sweep totals and carries in a
// workspace.  Here that workspace is a fixed array in the library's device image, one copy per
// GPU, held until the process ends.  Its device address is resolved once per device, with that
// device current, on the first call there; host code uses only that address (the array's name
// in host code is a host-side stand-in, not a device address).
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "sc.h"
#include "sc_host.h"

namespace {

static __device__ __align__(256) unsigned char scratch[SC_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_scratch[kMaxDevices] = {};  // device address of `scratch` per device (nullptr: not resolved)

// Device address of the current device's copy of the scratch array, resolved on first use.
sc_status scratch_ptr(void **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return scx::host::fail(SC_ERR_DEVICE, std::string("hipGetDevice failed: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return scx::host::fail(SC_ERR_DEVICE, "device index out of range for the scratch table");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return scx::host::fail(SC_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return SC_OK;
}

}  // namespace

extern "C" sc_status sc_apply_invL_noalloc(const sc_grid *grid, int dim, int op, int order, double alpha,
                                           const double *dirichlet_g, const void *v, void *out, sc_stream_t stream)
{
    using namespace scx::host;
    sc_status s = check_line_args(grid, dim, order, alpha);
    if (s != SC_OK) return s;
    if (op < SC_OP_L || op > SC_OP_0) return fail(SC_ERR_ARG, "op must be SC_OP_L, SC_OP_R or SC_OP_0");
    if (!v || !out) return fail(SC_ERR_ARG, "null array pointer");
    const Axis ax = axis_of(grid, dim);
    const size_t need = chunk_ws_bytes(ax.nlines, nchunks_for(ax, (int)elem_bytes(grid)), 1);
    if (need > (size_t)SC_NOALLOC_SCRATCH_BYTES)
        return fail(SC_ERR_WORKSPACE, "sc_apply_invL_noalloc: this pass needs " + std::to_string(need) +
                                          " bytes of scratch, more than the fixed " +
                                          std::to_string((size_t)SC_NOALLOC_SCRATCH_BYTES) +
                                          " (use sc_apply_invL with a workspace)");
    void *ws = nullptr;
    if (need > 0) {
        s = scratch_ptr(&ws);
        if (s != SC_OK) return s;
    }
    // the same passes as sc_apply_invL; every scratch entry a pass reads is written earlier in the
    // same call (chunk totals by the aggregate launch, carries by the carry launch)
    return sc_apply_invL(grid, dim, op, order, alpha, dirichlet_g, v, out, ws, need > 0 ? (size_t)SC_NOALLOC_SCRATCH_BYTES : 0,
                         stream);
}
