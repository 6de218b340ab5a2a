// sc_host.h -- host-side helpers shared by the C ABI units (library internal): error reporting,
// per-launch timing, axis geometry, argument checks and the per-operator constants of a pass.
#pragma once
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "sc.h"
#include "sc_device.h"

namespace scx {
namespace host {

sc_status fail(sc_status s, const std::string &msg);

// ------------------------------------------------------------------------------------------
// optional per-kernel timing (events on the caller's stream)
// ------------------------------------------------------------------------------------------
struct TimedLaunch {
    std::string name;
    hipEvent_t start, stop;
};
extern std::mutex g_tmu;
extern bool g_timing;
extern std::vector<std::string> g_timing_only;  // empty: every launch is timed
extern std::vector<TimedLaunch> g_records;
extern std::vector<std::pair<hipEvent_t, hipEvent_t>> g_pool;
extern size_t g_pool_used;

template <typename F>
hipError_t timed(const char *fallback_name, hipStream_t st, F &&launch)
{
    if (!g_timing) {
        const char *nm = fallback_name;
        return launch(&nm);
    }
    std::unique_lock<std::mutex> lk(g_tmu);
    bool selected = g_timing_only.empty();
    for (const auto &s : g_timing_only) selected = selected || s == fallback_name;
    if (!selected) {
        lk.unlock();
        const char *nm = fallback_name;
        return launch(&nm);
    }
    if (g_pool_used == g_pool.size()) {
        hipEvent_t a, b;
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return hipErrorOutOfMemory;
        g_pool.emplace_back(a, b);
    }
    auto ev = g_pool[g_pool_used++];
    hipError_t e = hipEventRecord(ev.first, st);
    if (e != hipSuccess) return e;
    const char *nm = fallback_name;
    e = launch(&nm);
    if (e != hipSuccess) return e;
    e = hipEventRecord(ev.second, st);
    if (e != hipSuccess) return e;
    g_records.push_back({nm ? std::string(nm) : std::string(fallback_name), ev.first, ev.second});
    return e;
}

// ------------------------------------------------------------------------------------------
// geometry and pass set-up
// ------------------------------------------------------------------------------------------
struct Axis {
    int64_t n, stride, nlines, ncells, total;
    double dx, len;
    int bc;
};

struct OpSpec {
    int op;
    double alpha, scale;
    int k;
    int identity = 0;  // 1: the operand already holds the local integrals (J_R for L_R, J_L for L_L)
};

sc_status check_grid(const sc_grid *g);
Axis axis_of(const sc_grid *g, int dim);
size_t elem_bytes(const sc_grid *g);
size_t round256(size_t b);
bool overlap(const void *a, const void *b, size_t bytes);
int pick_variant(bool contig, int64_t n, int elem);
void fill_op(OpArgs *P, int op, int order, double alpha, const Axis &ax, int vid, double scale, int k,
             int identity = 0);
void fill_ext(PassArgs *a, int order);
size_t chunk_ws_bytes(int64_t nlines, int64_t nchunks, int nops);
int64_t nchunks_for(const Axis &ax, int elem);
// nn_cpb > 0: nearest-neighbour virtual blocks of nn_cpb chunks (the line's mu terms dropped)
sc_status run_pass(const sc_grid *g, int dim, int order, const OpSpec *ops, int nops, const void *v, const void *acc,
                   int acc_mode, void *out, const double *dg, char *wsp, size_t ws_bytes, hipStream_t st,
                   int64_t nn_cpb = 0, double vw = 1.0, double aw = 1.0);
int64_t chunk_points(const Axis &ax, int elem);
// K of the windowed chunk carries for this pass and tile shape, or 0 (exact carries)
int window_k(const PassArgs &a, int order, const Variant &V, bool multi);
sc_status check_line_args(const sc_grid *g, int dim, int order, double alpha);

}  // namespace host
}  // namespace scx
