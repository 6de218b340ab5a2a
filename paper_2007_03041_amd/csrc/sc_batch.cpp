// sc_batch.cpp -- batched application over many independent instances: the lines of every
// instance (own length, line count, alpha, boundary, operator; contiguous or interleaved lines) in
// one pass per tile shape.
//
// A plan groups the instances by the tile shape chosen for them; each group is one launch of the
// persistent batched line pass over a work list of (instance, tile) items (chunked groups: an
// aggregate launch, a carry launch and an apply launch).  Shapes come from an autotuner that times
// every variant of the instances' layout, persistent or one workgroup per item, per class of
// instances (layout, line length rounded up to a power of two, single- or multi-line), and remembers
// the winners for the process.
// The launches of a plan can be captured once into a HIP graph and replayed as one launch.
#include "sc.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "sc_device.h"
#include "sc_host.h"
#include "sc_launch.h"

using namespace scx;
using namespace scx::host;

namespace {

// variants a batch may use (see SC_VARIANTS): contiguous lines (axis 0) take the x-line tiles,
// interleaved lines (axis 1) the strided 16- and 32-line tiles
const int kBatchVariants[] = {14, 0, 10, 1, 16, 9, 2, 3, 15};
const int kBatchStridedVariants[] = {4, 5, 6, 11, 12};

std::vector<int> batch_variants(int axis)
{
    return axis == 0 ? std::vector<int>(std::begin(kBatchVariants), std::end(kBatchVariants))
                     : std::vector<int>(std::begin(kBatchStridedVariants), std::end(kBatchStridedVariants));
}

struct Choice {
    int vid = -1;
    int persistent = 0;
    int exact = 0;  // 1: exact chunk carries even where the windowed carries apply
};

struct ClassKey {
    int elem, order, nbits, multi, axis;
    bool operator<(const ClassKey &o) const
    {
        return std::tie(axis, elem, order, nbits, multi) < std::tie(o.axis, o.elem, o.order, o.nbits, o.multi);
    }
};

std::mutex g_tune_mu;
std::map<ClassKey, Choice> g_tuned;  // winners of sc_batch_tune, per class, for the whole process

int ceil_log2(int64_t n)
{
    int b = 0;
    while ((int64_t(1) << b) < n) ++b;
    return b;
}

ClassKey class_of(const sc_batch_item &it, int elem, int order)
{
    return ClassKey{elem, order, ceil_log2(it.n), it.nlines >= 4 ? 1 : 0, it.axis};
}

Choice default_choice(const sc_batch_item &it, int elem)
{
    Choice c;
    // SC_BATCH_VARIANT=<variant>[p]: every untuned instance of that variant's layout takes it
    // (p: persistent)
    if (const char *env = std::getenv("SC_BATCH_VARIANT")) {
        const int vid = std::atoi(env);
        for (int v : batch_variants(it.axis))
            if (v == vid && variant_built(vid, elem)) {
                c.vid = vid;
                c.persistent = std::strchr(env, 'p') ? 1 : 0;
                return c;
            }
    }
    if (it.axis == 1) {
        // the tiles of single y/z passes (a strided shape the batch is not built for: 16 x 512)
        const int vid = pick_variant(false, it.n, elem);
        bool ok = false;
        for (int v : kBatchStridedVariants) ok = ok || v == vid;
        c.vid = ok ? vid : 5;
        return c;
    }
    if (it.nlines >= 4) {
        c.vid = it.n <= 256 ? 0 : it.n <= 512 ? 10 : it.n <= 1024 ? 1 : it.n <= 2048 ? 16 : it.n <= 4096 ? 2 : 3;
    } else {
        c.vid = it.n <= 1024 ? 14 : it.n <= 4096 ? 2 : 3;
    }
    if (elem == 4 && it.n > 8192 && it.n <= 16384) c.vid = 15;
    return c;
}

Axis item_axis(const sc_batch_item &it)
{
    Axis ax;
    ax.n = it.n;
    ax.stride = it.axis == 1 ? it.nlines : 1;
    ax.nlines = it.nlines;
    ax.total = it.n * it.nlines;
    ax.bc = it.bc;
    ax.ncells = it.bc == SC_BC_PERIODIC ? it.n : it.n - 1;
    ax.len = it.hi - it.lo;
    ax.dx = ax.len / (double)ax.ncells;
    return ax;
}

size_t item_chunk_doubles(const sc_batch_item &it, int64_t C)
{
    const int64_t nch = (it.n + C - 1) / C;
    if (nch <= 1) return 0;
    const int64_t ent = it.nlines * nch;
    return (size_t)(3 * ent) + (size_t)(2 * ent + 2 * it.nlines);
}

struct Launch {
    int kind = 0;  // 0: line pass, 1: chunk carry
    int vid = 0, mode = 0;
    int full = 0;  // line pass over tiles that end inside their line (the lean instantiation)
    int64_t nwork = 0, grid = 0;
    size_t off = 0;  // byte offset of the work list / item list in the device buffer
};

}  // namespace

struct sc_batch_plan_s {
    int elem = 8, order = 6, dtype = SC_F64;
    std::vector<sc_batch_item> items;
    std::vector<Choice> choice;
    std::vector<Launch> launches;
    char *dev = nullptr;  // device: instance table, then work and item lists
    size_t dev_bytes = 0;
    size_t ws_need = 0;   // workspace of the current choices (doubles)
    size_t ws_bound = 0;  // bytes: enough for any choice and for one-launch-per-instance runs
    int64_t extent = 0;   // elements of v / out the instances span
    int64_t g_extent = 0; // doubles of g the Dirichlet instances span
    int num_cu = 0;
    hipStream_t cap = nullptr;
    hipGraphExec_t exec = nullptr;
    const void *gv = nullptr;
    void *gout = nullptr;
    const double *gg = nullptr;
    void *gws = nullptr;
};

namespace {

void drop_graph(sc_batch_plan p)
{
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    p->exec = nullptr;
}

// Instance table, work lists and launches for the current choices; uploads them to the device.
sc_status build(sc_batch_plan p)
{
    const int count = (int)p->items.size();
    std::vector<BatchArgs> table(count);
    // (vid, persistent, chunked: 0 whole lines, 1 exact chunk carries, 2 windowed carries) -> items
    std::map<std::tuple<int, int, int>, std::vector<int>> groups;
    size_t wsd = 0;
    for (int i = 0; i < count; ++i) {
        const sc_batch_item &it = p->items[i];
        const Choice ch = p->choice[i];
        const Variant &V = variant(ch.vid);
        const Axis ax = item_axis(it);
        BatchArgs &b = table[i];
        std::memset(&b, 0, sizeof(b));
        PassArgs &a = b.a;
        a.n = it.n;
        a.stride = ax.stride;
        a.nlines = it.nlines;
        a.ncells = ax.ncells;
        a.nchunks = (it.n + V.C() - 1) / V.C();
        a.bc = it.bc;
        a.acc_mode = 0;
        a.nops = 1;
        fill_ext(&a, p->order);
        fill_op(&a.ops[0], it.op, p->order, it.alpha, ax, ch.vid, it.k >= 1 ? it.scale : 1.0, it.k);
        b.v_off = it.offset;
        b.g_off = it.g_offset;
        b.agg_off = b.carry_off = 0;
        int chunked = a.nchunks > 1 ? 1 : 0;
        if (chunked) {
            const int K = ch.exact ? 0 : window_k(a, p->order, V, false);
            if (K > 0) {
                // windowed carries: the apply launch alone, no workspace
                a.win_k = K;
                a.ops[0].mu = 0.0;
                a.ops[0].inv1mmu = 1.0;
                a.ops[0].dir2inv = 2.0;
                chunked = 2;
            } else {
                const int64_t ent = it.nlines * a.nchunks;
                b.agg_off = (int64_t)wsd;
                b.carry_off = (int64_t)wsd + 3 * ent;
                wsd += item_chunk_doubles(it, V.C());
            }
        }
        groups[std::make_tuple(ch.vid, ch.persistent, chunked)].push_back(i);
    }
    // work lists, in launch order: every fused group, then the chunked groups' phases
    std::vector<char> host(round256(sizeof(BatchArgs) * (size_t)count));
    std::memcpy(host.data(), table.data(), sizeof(BatchArgs) * (size_t)count);
    std::vector<Launch> launches;
    auto occ_grid = [&](int vid, int mode, int full, int pers, int64_t nwork) {
        int64_t grid = nwork;
        if (pers) {
            const int occ = std::max(1, line_pass_batch_occupancy(p->elem, p->order, vid, mode, full));
            grid = std::min<int64_t>(nwork, (int64_t)occ * p->num_cu);
        }
        return std::max<int64_t>(1, std::min<int64_t>(grid, INT32_MAX));
    };
    auto add_work = [&](const std::vector<BatchWork> &w) {
        const size_t off = host.size();
        host.resize(off + round256(sizeof(BatchWork) * w.size()));
        std::memcpy(host.data() + off, w.data(), sizeof(BatchWork) * w.size());
        return off;
    };
    for (int phase = 0; phase < 4; ++phase) {
        for (auto &kv : groups) {
            const int vid = std::get<0>(kv.first), pers = std::get<1>(kv.first), chunked = std::get<2>(kv.first);
            if ((phase == 0) != (chunked == 0)) continue;
            if (chunked == 2 && phase != 3) continue;  // windowed: the apply launch only
            const Variant &V = variant(vid);
            Launch L;
            L.vid = vid;
            if (phase == 2) {
                std::vector<int32_t> ids(kv.second.begin(), kv.second.end());
                const size_t off = host.size();
                host.resize(off + round256(sizeof(int32_t) * ids.size()));
                std::memcpy(host.data() + off, ids.data(), sizeof(int32_t) * ids.size());
                L.kind = 1;
                L.nwork = (int64_t)ids.size();
                L.off = off;
                launches.push_back(L);
                continue;
            }
            // tiles that end inside their line (every chunk but a ragged last one) run the lean
            // instantiation without the per-point end rules; the others the general one
            std::vector<BatchWork> w[2];
            for (int i : kv.second) {
                const BatchArgs &b = table[i];
                const int64_t tiles = (b.a.nlines + V.TC - 1) / V.TC;
                // (windowed items take a ragged last chunk as the full tile ending at the line's end)
                const bool ragged = b.a.n % V.C() != 0 && b.a.win_k == 0;
                for (int64_t t = 0; t < tiles * b.a.nchunks; ++t) {
                    const bool last = t % b.a.nchunks == b.a.nchunks - 1;
                    w[(ragged && last) ? 0 : 1].push_back(BatchWork{i, 0, t});
                }
            }
            L.mode = phase == 0 ? LMODE_FUSED : phase == 1 ? LMODE_AGG : chunked == 2 ? LMODE_WIN : LMODE_APPLY;
            for (int full = 1; full >= 0; --full) {
                if (w[full].empty()) continue;
                L.full = full;
                L.nwork = (int64_t)w[full].size();
                L.grid = occ_grid(vid, L.mode, full, pers, L.nwork);
                L.off = add_work(w[full]);
                launches.push_back(L);
            }
        }
    }
    drop_graph(p);
    // launches already enqueued may still read the old tables
    if (p->dev && hipDeviceSynchronize() != hipSuccess) return fail(SC_ERR_DEVICE, "device synchronisation failed");
    if (host.size() > p->dev_bytes) {
        if (p->dev) (void)hipFree(p->dev);
        p->dev = nullptr;
        p->dev_bytes = 0;
        if (hipMalloc((void **)&p->dev, host.size()) != hipSuccess) return fail(SC_ERR_DEVICE, "hipMalloc of the plan tables failed");
        p->dev_bytes = host.size();
    }
    if (hipMemcpy(p->dev, host.data(), host.size(), hipMemcpyHostToDevice) != hipSuccess)
        return fail(SC_ERR_DEVICE, "upload of the plan tables failed");
    p->launches = launches;
    p->ws_need = wsd * sizeof(double);
    return SC_OK;
}

hipError_t enqueue(sc_batch_plan p, const void *v, void *out, const double *g, void *ws, hipStream_t st, bool time_it)
{
    const BatchArgs *table = (const BatchArgs *)p->dev;
    for (const Launch &L : p->launches) {
        hipError_t e;
        auto run = [&](const char **) -> hipError_t {
            if (L.kind == 1)
                return launch_chunk_carry_batch(table, (const int32_t *)(p->dev + L.off), (int)L.nwork, g,
                                                (double *)ws, st);
            BatchLaunch b{table, (const BatchWork *)(p->dev + L.off), L.nwork, L.grid, v, out, g, (double *)ws, L.mode,
                          L.full};
            return launch_line_pass_batch(b, p->elem, p->order, L.vid, st);
        };
        if (time_it) {
            // timing names carry the launch's shape: batch_<phase>_v<variant><p: persistent, o: one
            // workgroup per item>[f: tiles that end inside their line]
            std::string nm = L.kind == 1                ? "batch_chunk_carry"
                             : L.mode == LMODE_FUSED ? "batch_fused"
                             : L.mode == LMODE_AGG   ? "batch_agg"
                             : L.mode == LMODE_WIN   ? "batch_window"
                                                     : "batch_apply";
            if (L.kind == 0) nm += "_v" + std::to_string(L.vid) + (L.grid < L.nwork ? "p" : "o") + (L.full ? "f" : "");
            e = timed(nm.c_str(), st, run);
        } else {
            e = run(nullptr);
        }
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

sc_status check_buffers(sc_batch_plan p, const void *v, void *out, const double *g, void *ws, size_t ws_bytes)
{
    if (!v || !out) return fail(SC_ERR_ARG, "null array pointer");
    if (overlap(v, out, (size_t)p->extent * (size_t)p->elem)) return fail(SC_ERR_ARG, "out overlaps v");
    if (p->g_extent > 0 && !g) return fail(SC_ERR_ARG, "instances with Dirichlet values need g");
    if (p->ws_need > 0 && (!ws || ws_bytes < p->ws_need)) return fail(SC_ERR_WORKSPACE, "workspace too small");
    if (ws && ((uintptr_t)ws & 255)) return fail(SC_ERR_ARG, "workspace must be 256-byte aligned");
    return SC_OK;
}

}  // namespace

extern "C" {

sc_status sc_batch_plan_create(const sc_batch_item *items, int count, int dtype, int order, sc_batch_plan *plan)
{
    if (!plan) return fail(SC_ERR_ARG, "plan is NULL");
    *plan = nullptr;
    if (!items || count < 1) return fail(SC_ERR_ARG, "need at least one instance");
    if (dtype != SC_F64 && dtype != SC_F32_MIXED) return fail(SC_ERR_ARG, "unknown dtype");
    if (order != 4 && order != 6) return fail(SC_ERR_UNSUPPORTED, "order must be 4 or 6");
    const int elem = dtype == SC_F64 ? 8 : 4;
    int64_t extent = 0, g_extent = 0;
    size_t bound = 0, per_max = 0;
    for (int i = 0; i < count; ++i) {
        const sc_batch_item &it = items[i];
        char where[64];
        std::snprintf(where, sizeof(where), "instance %d: ", i);
        if (it.n < order + 1) return fail(SC_ERR_SHAPE, std::string(where) + "line shorter than the stencil");
        if (it.nlines < 1 || it.offset < 0) return fail(SC_ERR_SHAPE, std::string(where) + "bad line count or offset");
        if (it.axis != 0 && it.axis != 1) return fail(SC_ERR_ARG, std::string(where) + "axis must be 0 or 1");
        if (it.n > (int64_t(1) << 40) / it.nlines) return fail(SC_ERR_SHAPE, std::string(where) + "too large");
        // tile index arithmetic along a line is 32-bit
        if (it.n > (int64_t(1) << 31) - 65536) return fail(SC_ERR_SHAPE, std::string(where) + "line longer than 2^31 - 2^16");
        if (it.bc != SC_BC_PERIODIC && it.bc != SC_BC_DIRICHLET) return fail(SC_ERR_ARG, std::string(where) + "unknown bc");
        if (it.op < SC_OP_L || it.op > SC_OP_0) return fail(SC_ERR_ARG, std::string(where) + "unknown op");
        if (it.k != 0 && it.k != 1) return fail(SC_ERR_UNSUPPORTED, std::string(where) + "batches take k = 0 or 1");
        if (!(it.hi > it.lo) || !std::isfinite(it.hi - it.lo)) return fail(SC_ERR_ARG, std::string(where) + "lo < hi");
        if (!(it.alpha > 0.0) || !std::isfinite(it.alpha)) return fail(SC_ERR_ARG, std::string(where) + "alpha must be > 0");
        if (!std::isfinite(it.scale)) return fail(SC_ERR_ARG, std::string(where) + "scale must be finite");
        if (it.g_offset < -1 || (it.g_offset >= 0 && it.bc != SC_BC_DIRICHLET))
            return fail(SC_ERR_ARG, std::string(where) + "g_offset must be -1, or >= 0 on Dirichlet instances");
        const Axis ax = item_axis(it);
        if (!(it.alpha * ax.dx < 700.0)) return fail(SC_ERR_ARG, std::string(where) + "alpha * dx too large (> 700)");
        extent = std::max(extent, it.offset + it.n * it.nlines);
        if (it.g_offset >= 0) g_extent = std::max(g_extent, it.g_offset + 2 * it.nlines);
        size_t worst = 0;
        for (int vid : batch_variants(it.axis))
            if (variant_built(vid, elem)) worst = std::max(worst, item_chunk_doubles(it, variant(vid).C()));
        bound += worst * sizeof(double);
        const int64_t C1 = variant(pick_variant(it.axis == 0, it.n, elem)).C();
        per_max = std::max(per_max, chunk_ws_bytes(it.nlines, (it.n + C1 - 1) / C1, 1));
    }
    sc_batch_plan p = new sc_batch_plan_s;
    p->elem = elem;
    p->order = order;
    p->dtype = dtype;
    p->items.assign(items, items + count);
    p->extent = extent;
    p->g_extent = g_extent;
    p->ws_bound = std::max(round256(bound), per_max);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&p->num_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || p->num_cu < 1) {
        delete p;
        return fail(SC_ERR_DEVICE, "no HIP device");
    }
    p->choice.resize(count);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        for (int i = 0; i < count; ++i) {
            auto f = g_tuned.find(class_of(items[i], elem, order));
            p->choice[i] = f != g_tuned.end() ? f->second : default_choice(items[i], elem);
        }
    }
    if (hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking) != hipSuccess) {
        delete p;
        return fail(SC_ERR_DEVICE, "stream creation failed");
    }
    sc_status s = build(p);
    if (s != SC_OK) {
        sc_batch_plan_destroy(p);
        return s;
    }
    *plan = p;
    return SC_OK;
}

sc_status sc_batch_plan_destroy(sc_batch_plan plan)
{
    if (!plan) return SC_OK;
    drop_graph(plan);
    if (plan->cap) (void)hipStreamDestroy(plan->cap);
    if (plan->dev) (void)hipFree(plan->dev);
    delete plan;
    return SC_OK;
}

size_t sc_batch_workspace_bytes(sc_batch_plan plan) { return plan ? plan->ws_bound : 0; }

int64_t sc_batch_elements(sc_batch_plan plan) { return plan ? plan->extent : -1; }

sc_status sc_batch_apply(sc_batch_plan plan, const void *v, void *out, const double *g, void *ws, size_t ws_bytes,
                         int use_graph, sc_stream_t stream)
{
    if (!plan) return fail(SC_ERR_ARG, "plan is NULL");
    sc_status s = check_buffers(plan, v, out, g, ws, ws_bytes);
    if (s != SC_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e;
    if (!use_graph) {
        e = enqueue(plan, v, out, g, ws, st, true);
        if (e != hipSuccess) return fail(SC_ERR_DEVICE, std::string("launch failed: ") + hipGetErrorString(e));
        return SC_OK;
    }
    if (!plan->exec || plan->gv != v || plan->gout != out || plan->gg != g || plan->gws != ws) {
        drop_graph(plan);
        hipGraph_t graph = nullptr;
        e = hipStreamBeginCapture(plan->cap, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            const hipError_t e1 = enqueue(plan, v, out, g, ws, plan->cap, false);
            e = hipStreamEndCapture(plan->cap, &graph);
            if (e1 != hipSuccess) e = e1;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&plan->exec, graph, nullptr, nullptr, 0);
        if (graph) (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            plan->exec = nullptr;
            return fail(SC_ERR_DEVICE, std::string("graph capture failed: ") + hipGetErrorString(e));
        }
        plan->gv = v;
        plan->gout = out;
        plan->gg = g;
        plan->gws = ws;
    }
    e = timed("batch_graph", st, [&](const char **) { return hipGraphLaunch(plan->exec, st); });
    if (e != hipSuccess) return fail(SC_ERR_DEVICE, std::string("graph launch failed: ") + hipGetErrorString(e));
    return SC_OK;
}

sc_status sc_batch_apply_per_instance(sc_batch_plan plan, const void *v, void *out, const double *g, void *ws,
                                      size_t ws_bytes, sc_stream_t stream)
{
    if (!plan) return fail(SC_ERR_ARG, "plan is NULL");
    sc_status s = check_buffers(plan, v, out, g, ws, ws_bytes);
    if (s != SC_OK) return s;
    for (size_t i = 0; i < plan->items.size(); ++i) {
        const sc_batch_item &it = plan->items[i];
        sc_grid gr;
        std::memset(&gr, 0, sizeof(gr));
        // the instance as a 2-D grid whose axis `d` holds its lines
        const int d = it.axis;
        gr.ndim = 2;
        gr.n[d] = it.n;
        gr.n[1 - d] = it.nlines;
        gr.n[2] = 1;
        gr.lo[d] = it.lo;
        gr.hi[d] = it.hi;
        gr.lo[1 - d] = 0.0;
        gr.hi[1 - d] = 1.0;
        gr.bc[d] = it.bc;
        gr.bc[1 - d] = SC_BC_PERIODIC;
        gr.dtype = plan->dtype;
        const char *vi = (const char *)v + (size_t)it.offset * plan->elem;
        char *oi = (char *)out + (size_t)it.offset * plan->elem;
        const double *gi = it.g_offset >= 0 ? g + it.g_offset : nullptr;
        if (it.k == 0)
            s = sc_apply_invL(&gr, d, it.op, plan->order, it.alpha, gi, vi, oi, ws, ws_bytes, stream);
        else
            s = sc_apply_D_partial_sum(&gr, d, it.op, plan->order, it.alpha, 1, it.scale, gi, vi, oi, ws, ws_bytes,
                                       stream);
        if (s != SC_OK) return s;
    }
    return SC_OK;
}

sc_status sc_batch_tune(sc_batch_plan plan, const void *v, void *out, const double *g, void *ws, size_t ws_bytes,
                        int reps, sc_stream_t stream)
{
    if (!plan) return fail(SC_ERR_ARG, "plan is NULL");
    if (reps < 1) return fail(SC_ERR_ARG, "reps must be >= 1");
    if (ws_bytes < plan->ws_bound || !ws) return fail(SC_ERR_WORKSPACE, "tuning needs sc_batch_workspace_bytes()");
    sc_status s = check_buffers(plan, v, out, g, ws, ws_bytes);
    if (s != SC_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    std::map<ClassKey, std::vector<int>> classes;
    for (size_t i = 0; i < plan->items.size(); ++i)
        classes[class_of(plan->items[i], plan->elem, plan->order)].push_back((int)i);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(SC_ERR_DEVICE, "event creation failed");
    std::map<ClassKey, Choice> won;
    for (auto &kv : classes) {
        // a plan holding this class only, timed for every candidate shape
        sc_batch_plan_s sub;
        sub.elem = plan->elem;
        sub.order = plan->order;
        sub.dtype = plan->dtype;
        sub.num_cu = plan->num_cu;
        for (int i : kv.second) sub.items.push_back(plan->items[i]);
        sub.choice.resize(sub.items.size());
        float best = 1e30f;
        Choice best_c = plan->choice[kv.second[0]];
        for (int vid : batch_variants(kv.first.axis)) {
            if (!variant_built(vid, plan->elem)) continue;
            for (int cand = 0; cand < 4; ++cand) {
                const int pers = cand & 1, exact = cand >> 1;
                // the exact carries are a separate candidate only where the windowed ones apply
                if (exact) {
                    bool any = false;
                    for (int i : kv.second) {
                        const sc_batch_item &it = plan->items[i];
                        PassArgs a;
                        std::memset(&a, 0, sizeof(a));
                        a.n = it.n;
                        a.stride = item_axis(it).stride;
                        a.nlines = it.nlines;
                        a.nops = 1;
                        a.nchunks = (it.n + variant(vid).C() - 1) / variant(vid).C();
                        fill_op(&a.ops[0], it.op, plan->order, it.alpha, item_axis(it), vid, 1.0, it.k);
                        any = any || window_k(a, plan->order, variant(vid), false) > 0;
                    }
                    if (!any) continue;
                }
                for (auto &c : sub.choice) c = Choice{vid, pers, exact};
                s = build(&sub);
                if (s != SC_OK) break;
                hipError_t e = enqueue(&sub, v, out, g, ws, st, false);  // warm-up
                if (e == hipSuccess) e = hipEventRecord(e0, st);
                for (int r = 0; r < reps && e == hipSuccess; ++r) e = enqueue(&sub, v, out, g, ws, st, false);
                if (e == hipSuccess) e = hipEventRecord(e1, st);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                float ms = 0.f;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                if (e != hipSuccess) {
                    s = fail(SC_ERR_DEVICE, std::string("tuning launch failed: ") + hipGetErrorString(e));
                    break;
                }
                if (ms < best) {
                    best = ms;
                    best_c = Choice{vid, pers, exact};
                }
            }
            if (s != SC_OK) break;
        }
        if (sub.dev) (void)hipFree(sub.dev);
        sub.dev = nullptr;
        if (s != SC_OK) break;
        won[kv.first] = best_c;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (s != SC_OK) return s;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        for (auto &kv : won) g_tuned[kv.first] = kv.second;
    }
    for (size_t i = 0; i < plan->items.size(); ++i)
        plan->choice[i] = won[class_of(plan->items[i], plan->elem, plan->order)];
    return build(plan);
}

int sc_batch_tune_export(char *buf, int len)
{
    std::string txt;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        for (auto &kv : g_tuned) {
            char line[112];
            std::snprintf(line, sizeof(line), "%d %d %d %d %d %d %d %d\n", kv.first.elem, kv.first.order,
                          kv.first.nbits, kv.first.multi, kv.second.vid, kv.second.persistent, kv.second.exact,
                          kv.first.axis);
            txt += line;
        }
    }
    if (buf && len > 0) std::snprintf(buf, (size_t)len, "%s", txt.c_str());
    return (int)txt.size();
}

sc_status sc_batch_tune_import(const char *text)
{
    if (!text) return fail(SC_ERR_ARG, "text is NULL");
    std::map<ClassKey, Choice> got;
    const char *p = text;
    int lineno = 0;
    while (*p) {
        const char *e = std::strchr(p, '\n');
        const std::string line(p, e ? (size_t)(e - p) : std::strlen(p));
        p = e ? e + 1 : p + line.size();
        ++lineno;
        if (line.find_first_not_of(" \t\r") == std::string::npos) continue;
        ClassKey k{};
        Choice c;
        char extra = 0;
        // (lines of seven integers, written before the layout field, are contiguous-line classes)
        const int got_n = std::sscanf(line.c_str(), "%d %d %d %d %d %d %d %d %c", &k.elem, &k.order, &k.nbits,
                                      &k.multi, &c.vid, &c.persistent, &c.exact, &k.axis, &extra);
        if (got_n != 7 && got_n != 8)
            return fail(SC_ERR_ARG, "tune table line " + std::to_string(lineno) + ": expected 8 integers");
        if (got_n == 7) k.axis = 0;
        bool known = false;
        if (k.axis == 0 || k.axis == 1)
            for (int v : batch_variants(k.axis)) known = known || v == c.vid;
        if ((k.elem != 4 && k.elem != 8) || (k.order != 4 && k.order != 6) || k.nbits < 0 || k.nbits > 31 ||
            (k.multi != 0 && k.multi != 1) || !known || !variant_built(c.vid, k.elem) ||
            (c.persistent != 0 && c.persistent != 1) || (c.exact != 0 && c.exact != 1))
            return fail(SC_ERR_ARG, "tune table line " + std::to_string(lineno) + ": value out of range");
        got[k] = c;
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (auto &kv : got) g_tuned[kv.first] = kv.second;
    return SC_OK;
}

int sc_batch_describe(sc_batch_plan plan, char *buf, int len)
{
    if (!plan) return -1;
    std::map<std::tuple<int, int, int>, int> use;  // (the variant also tells the layout)
    for (const Choice &c : plan->choice) use[std::make_tuple(c.vid, c.persistent, c.exact)] += 1;
    std::string js = "{\"launches\": " + std::to_string(plan->launches.size()) + ", \"shapes\": [";
    bool first = true;
    for (auto &kv : use) {
        const Variant &V = variant(std::get<0>(kv.first));
        char tmp[200];
        std::snprintf(tmp, sizeof(tmp),
                      "%s{\"variant\": %d, \"S\": %d, \"TC\": %d, \"NT\": %d, \"chunk\": %d, \"axis\": %d, "
                      "\"persistent\": %d, \"exact_carries\": %d, \"instances\": %d}",
                      first ? "" : ", ", std::get<0>(kv.first), V.S, V.TC, V.NT, V.C(), V.contig ? 0 : 1,
                      std::get<1>(kv.first), std::get<2>(kv.first), kv.second);
        js += tmp;
        first = false;
    }
    js += "]}";
    if (buf && len > 0) std::snprintf(buf, (size_t)len, "%s", js.c_str());
    return (int)js.size();
}

}  // extern "C"
