// sc_hj.cpp -- C ABI of the nonlinear Hamilton-Jacobi example and of the learned weight proposer:
// validation, quadrature constants, workspace layout and the order of launches of one step.
#include "sc.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <string>

#include "sc_device.h"
#include "sc_hj_dev.h"
#include "sc_host.h"
#include "sc_launch.h"

using namespace scx;
using namespace scx::host;

namespace {

struct HjLayout {
    size_t JL, JR, D[4], part, stats, chunk, total;
    int64_t nblocks;
};

HjLayout hj_layout(const sc_grid *g)
{
    HjLayout L;
    const int64_t npts = g->n[0] * g->n[1];
    const size_t f = round256(sizeof(double) * (size_t)npts);
    L.nblocks = (npts + 255) / 256;
    size_t off = 0;
    L.JL = off;
    off += f;
    L.JR = off;
    off += f;
    for (int k = 0; k < 4; ++k) {
        L.D[k] = off;
        off += f;
    }
    L.part = off;
    // per-block wave-speed maxima: of the update's blocks, or of the fused passes' workgroups
    const int64_t nparts = std::max<int64_t>(L.nblocks, hj_fused_blocks(g->n[0], g->n[1], 0) +
                                                            hj_fused_blocks(g->n[0], g->n[1], 1));
    off += round256(sizeof(double) * (size_t)nparts);
    L.stats = off;
    off += round256(sizeof(double) * 6 * (size_t)L.nblocks);
    L.chunk = off;
    size_t ch = 0;
    for (int d = 0; d < 2; ++d) {
        const Axis ax = axis_of(g, d);
        ch = std::max(ch, chunk_ws_bytes(ax.nlines, nchunks_for(ax, 8), 1));
    }
    off += round256(ch);
    L.total = off;
    return L;
}

sc_status check_hj(const sc_grid *g, const sc_hj_params *p)
{
    sc_status s = check_grid(g);
    if (s != SC_OK) return s;
    if (!p) return fail(SC_ERR_ARG, "params is NULL");
    if (g->ndim != 2) return fail(SC_ERR_UNSUPPORTED, "the Hamilton-Jacobi solver is 2-D");
    if (g->dtype != SC_F64) return fail(SC_ERR_UNSUPPORTED, "the Hamilton-Jacobi solver is FP64");
    if (g->bc[0] != SC_BC_PERIODIC || g->bc[1] != SC_BC_PERIODIC)
        return fail(SC_ERR_UNSUPPORTED, "the Hamilton-Jacobi solver is periodic");
    if (g->n[0] < 7 || g->n[1] < 7) return fail(SC_ERR_SHAPE, "need at least 7 points per axis");
    if (!(p->beta > 0.0) || !(p->cfl > 0.0) || !std::isfinite(p->beta) || !std::isfinite(p->cfl))
        return fail(SC_ERR_ARG, "beta and cfl must be finite and > 0");
    if (!(p->t_end >= 0.0)) return fail(SC_ERR_ARG, "t_end must be >= 0");
    if (p->weights < 0 || p->weights > 2) return fail(SC_ERR_ARG, "weights must be 0, 1 or 2");
    if (p->hamiltonian < 0 || p->hamiltonian > 1) return fail(SC_ERR_ARG, "hamiltonian must be 0 or 1");
    if (!(p->theta >= 0.0)) return fail(SC_ERR_ARG, "theta must be >= 0");
    const double h = std::min(axis_of(g, 0).dx, axis_of(g, 1).dx);
    const double alpha = p->beta / (p->cfl * h);
    for (int d = 0; d < 2; ++d)
        if (!(alpha * axis_of(g, d).dx < 700.0)) return fail(SC_ERR_ARG, "alpha * dx too large (> 700)");
    return SC_OK;
}

HjStepArgs step_args(const sc_grid *g, const sc_hj_params *p)
{
    HjStepArgs A;
    A.nx = g->n[0];
    A.ny = g->n[1];
    A.npts = A.nx * A.ny;
    A.dx = axis_of(g, 0).dx;
    A.dy = axis_of(g, 1).dx;
    const double h = std::min(A.dx, A.dy);
    A.alpha_x = A.alpha_y = p->beta / (p->cfl * h);
    A.cfl_h = p->cfl * h;
    A.t_end = p->t_end;
    A.hamiltonian = p->hamiltonian;
    A.pad_ = 0;
    return A;
}

// substencil weights c[r] on eta = {3 - r, 2 - r, 1 - r} and the linear weights d: the 5-point rule on
// eta = {3, 2, 1, 0, -1} equals sum_r d_r c[r]; its first node only appears in S_0 and its last
// only in S_2, which fixes d_0 and d_2, and the weights sum to one
HjQuadArgs quad_args(const sc_grid *g, const sc_hj_params *p, int axis)
{
    HjQuadArgs Q;
    std::memset(&Q, 0, sizeof(Q));
    Q.nx = g->n[0];
    Q.ny = g->n[1];
    Q.axis = axis;
    const double h = std::min(axis_of(g, 0).dx, axis_of(g, 1).dx);
    const double nu = p->beta / (p->cfl * h) * axis_of(g, axis).dx;
    for (int r = 0; r < 3; ++r) {
        const int eta[3] = {3 - r, 2 - r, 1 - r};
        quad_weights(nu, 3, eta, Q.c[r]);
    }
    const int eta5[5] = {3, 2, 1, 0, -1};
    double w5[5];
    quad_weights(nu, 5, eta5, w5);
    Q.d[0] = w5[0] / Q.c[0][0];
    Q.d[2] = w5[4] / Q.c[2][2];
    Q.d[1] = 1.0 - Q.d[0] - Q.d[2];
    Q.theta = p->theta;
    return Q;
}

// The fused two-pass step applies to the separable quadratic Hamiltonian with linear or WENO-Z
// weights where the sweeps' decay over the window, d^{HJF_KW}, is below 2^-60 on both axes.
// SC_HJ_FUSED=0 always takes the step of separate launches.
bool hj_fused_ok(const sc_grid *g, const sc_hj_params *p, const HjStepArgs &A)
{
    const char *env = std::getenv("SC_HJ_FUSED");
    if (env && env[0] == '0') return false;
    if (p->weights == HJ_LEARNED || p->hamiltonian != HJ_H_QUADRATIC) return false;
    const double nu_min = std::min(A.alpha_x * A.dx, A.alpha_y * A.dy);
    (void)g;
    return nu_min * HJF_KW >= 60.0 * std::log(2.0);
}

HjFusedArgs fused_args(const HjStepArgs &A)
{
    HjFusedArgs F;
    std::memset(&F, 0, sizeof(F));
    for (int ax = 0; ax < 2; ++ax) {
        const double nu = ax == 0 ? A.alpha_x * A.dx : A.alpha_y * A.dy;
        F.alpha[ax] = ax == 0 ? A.alpha_x : A.alpha_y;
        F.d[ax] = std::exp(-nu);
        for (int t = 0; t <= HJF_PPL; ++t) F.dpow[ax][t] = std::exp(-nu * t);
        for (int k = 0; k < 6; ++k) F.dscan[ax][k] = std::exp(-nu * (double)HJF_PPL * (double)(1 << k));
    }
    return F;
}

}  // namespace

extern "C" {

size_t sc_hj_workspace_bytes(const sc_grid *grid)
{
    if (!grid || check_grid(grid) != SC_OK || grid->ndim != 2) return 0;
    return hj_layout(grid).total + 256;
}

sc_status sc_hj_init(const sc_grid *grid, const sc_hj_params *p, const void *u, double *state, void *ws,
                     size_t ws_bytes, sc_stream_t stream)
{
    sc_status s = check_hj(grid, p);
    if (s != SC_OK) return s;
    if (!u || !state) return fail(SC_ERR_ARG, "null pointer");
    const HjLayout L = hj_layout(grid);
    if (!ws || ws_bytes < L.total) return fail(SC_ERR_WORKSPACE, "workspace too small");
    if ((uintptr_t)ws & 255) return fail(SC_ERR_ARG, "workspace must be 256-byte aligned");
    hipStream_t st = (hipStream_t)stream;
    char *w = (char *)ws;
    const HjStepArgs A = step_args(grid, p);
    hipError_t e = launch_hj_init_speed((const double *)u, A, (double *)(w + L.part), st);
    if (e == hipSuccess) e = launch_hj_finish((const double *)(w + L.part), L.nblocks, nullptr, 0, A, state, 0, st);
    if (e != hipSuccess) return fail(SC_ERR_DEVICE, std::string("launch failed: ") + hipGetErrorString(e));
    return SC_OK;
}

sc_status sc_hj_step(const sc_grid *grid, const sc_hj_params *p, int nsteps, void *u, double *state,
                     const float *mlp_params, void *ws, size_t ws_bytes, sc_stream_t stream)
{
    sc_status s = check_hj(grid, p);
    if (s != SC_OK) return s;
    if (!u || !state) return fail(SC_ERR_ARG, "null pointer");
    if (nsteps < 0) return fail(SC_ERR_ARG, "nsteps must be >= 0");
    if (p->weights == HJ_LEARNED && !mlp_params) return fail(SC_ERR_ARG, "learned weights need the proposer's parameters");
    const HjLayout L = hj_layout(grid);
    if (!ws || ws_bytes < L.total) return fail(SC_ERR_WORKSPACE, "workspace too small");
    if ((uintptr_t)ws & 255) return fail(SC_ERR_ARG, "workspace must be 256-byte aligned");
    const size_t fbytes = sizeof(double) * (size_t)(grid->n[0] * grid->n[1]);
    if (overlap(u, ws, fbytes)) return fail(SC_ERR_ARG, "workspace overlaps u");
    hipStream_t st = (hipStream_t)stream;
    char *w = (char *)ws;
    double *JL = (double *)(w + L.JL), *JR = (double *)(w + L.JR);
    double *D[4];
    for (int k = 0; k < 4; ++k) D[k] = (double *)(w + L.D[k]);
    double *part = (double *)(w + L.part), *stats = (double *)(w + L.stats);
    const HjStepArgs A = step_args(grid, p);
    const HjQuadArgs Q[2] = {quad_args(grid, p, 0), quad_args(grid, p, 1)};
    const double alpha = A.alpha_x;
    if (hj_fused_ok(grid, p, A)) {
        // two passes a step, alternating between u and a workspace field: x: dst = src - dt Hx(src);
        // y: dst -= dt Hy(src).  An odd step count ends with a copy back into u.
        const HjFusedArgs F = fused_args(A);
        const int64_t nbx = hj_fused_blocks(A.nx, A.ny, 0), nby = hj_fused_blocks(A.nx, A.ny, 1);
        double *bufs[2] = {(double *)u, D[0]};
        for (int step = 0; step < nsteps; ++step) {
            const double *src = bufs[step & 1];
            double *dst = bufs[(step + 1) & 1];
            hipError_t e = timed("hj_fused_x", st, [&](const char **) {
                return launch_hj_fused_pass(0, p->weights, src, nullptr, dst, Q[0], F, A, state, part, st);
            });
            if (e == hipSuccess)
                e = timed("hj_fused_y", st, [&](const char **) {
                    return launch_hj_fused_pass(1, p->weights, src, dst, dst, Q[1], F, A, state, part + nbx, st);
                });
            if (e == hipSuccess)
                e = timed("hj_finish_step", st, [&](const char **) {
                    return launch_hj_finish(part, nbx + nby, stats, 0, A, state, 1, st);
                });
            if (e != hipSuccess) return fail(SC_ERR_DEVICE, std::string("launch failed: ") + hipGetErrorString(e));
        }
        if (nsteps & 1) {
            const hipError_t e = hipMemcpyAsync(u, D[0], fbytes, hipMemcpyDeviceToDevice, st);
            if (e != hipSuccess) return fail(SC_ERR_DEVICE, std::string("copy failed: ") + hipGetErrorString(e));
        }
        return SC_OK;
    }
    for (int step = 0; step < nsteps; ++step) {
        for (int axis = 0; axis < 2; ++axis) {
            hipError_t e = timed("hj_weno_quad", st, [&](const char **) {
                return launch_hj_weno_quad(p->weights, (const double *)u, JL, JR, Q[axis], mlp_params,
                                           stats + 3 * axis * L.nblocks, st);
            });
            if (e != hipSuccess) return fail(SC_ERR_DEVICE, std::string("launch failed: ") + hipGetErrorString(e));
            // u - L_R^{-1}[u] and u - L_L^{-1}[u] from the local integrals (sweeps, periodic constants)
            OpSpec oR{SC_OP_R, alpha, -1.0, 0, 1}, oL{SC_OP_L, alpha, -1.0, 0, 1};
            s = run_pass(grid, axis, 4, &oR, 1, JR, u, 2, D[2 * axis + 0], nullptr, w + L.chunk, L.total - L.chunk, st);
            if (s == SC_OK)
                s = run_pass(grid, axis, 4, &oL, 1, JL, u, 2, D[2 * axis + 1], nullptr, w + L.chunk, L.total - L.chunk,
                             st);
            if (s != SC_OK) return s;
        }
        hipError_t e = timed("hj_update", st, [&](const char **) {
            return launch_hj_update((double *)u, D[0], D[1], D[2], D[3], A, state, part, st);
        });
        if (e == hipSuccess)
            e = timed("hj_finish_step", st, [&](const char **) {
                return launch_hj_finish(part, L.nblocks, stats, p->weights == HJ_LEARNED ? 2 * L.nblocks : 0, A, state,
                                        1, st);
            });
        if (e != hipSuccess) return fail(SC_ERR_DEVICE, std::string("launch failed: ") + hipGetErrorString(e));
    }
    return SC_OK;
}

sc_status sc_hj_harvest(const sc_grid *grid, const sc_hj_params *p, const void *u, int axis, float *X, float *Y,
                        sc_stream_t stream)
{
    sc_status s = check_hj(grid, p);
    if (s != SC_OK) return s;
    if (axis < 0 || axis > 1) return fail(SC_ERR_ARG, "axis must be 0 or 1");
    if (!u || !X || !Y) return fail(SC_ERR_ARG, "null pointer");
    const HjQuadArgs Q = quad_args(grid, p, axis);
    hipError_t e = launch_hj_harvest((const double *)u, Q, X, Y, (hipStream_t)stream);
    if (e != hipSuccess) return fail(SC_ERR_DEVICE, std::string("launch failed: ") + hipGetErrorString(e));
    return SC_OK;
}

int sc_mlp_param_count(void) { return MLP_NPARAM; }

sc_status sc_mlp_forward(const float *params, int64_t n, const float *X, float *Y, sc_stream_t stream)
{
    if (!params || !X || !Y) return fail(SC_ERR_ARG, "null pointer");
    if (n < 1) return fail(SC_ERR_ARG, "n must be >= 1");
    hipError_t e = launch_mlp_forward(params, X, Y, n, (hipStream_t)stream);
    if (e != hipSuccess) return fail(SC_ERR_DEVICE, std::string("launch failed: ") + hipGetErrorString(e));
    return SC_OK;
}

size_t sc_mlp_grad_workspace_bytes(int64_t n)
{
    if (n < 1) return 0;
    return sizeof(float) * (size_t)mlp_train_slots(n) * (MLP_NPARAM + 1);
}

sc_status sc_mlp_grad(const float *params, int64_t n, const float *X, const float *Y, float *grad, float *loss,
                      void *ws, size_t ws_bytes, sc_stream_t stream)
{
    if (!params || !X || !Y || !grad || !loss) return fail(SC_ERR_ARG, "null pointer");
    if (n < 1) return fail(SC_ERR_ARG, "n must be >= 1");
    if (!ws || ws_bytes < sc_mlp_grad_workspace_bytes(n)) return fail(SC_ERR_WORKSPACE, "workspace too small");
    hipError_t e = launch_mlp_grad(params, X, Y, n, (float *)ws, grad, loss, (hipStream_t)stream);
    if (e != hipSuccess) return fail(SC_ERR_DEVICE, std::string("launch failed: ") + hipGetErrorString(e));
    return SC_OK;
}

sc_status sc_mlp_adam(float *params, const float *grad, float *m, float *v, int step, float lr, sc_stream_t stream)
{
    if (!params || !grad || !m || !v) return fail(SC_ERR_ARG, "null pointer");
    if (step < 1 || !(lr > 0.f)) return fail(SC_ERR_ARG, "step must be >= 1 and lr > 0");
    hipError_t e = launch_mlp_adam(params, grad, m, v, step, lr, (hipStream_t)stream);
    if (e != hipSuccess) return fail(SC_ERR_DEVICE, std::string("launch failed: ") + hipGetErrorString(e));
    return SC_OK;
}

}  // extern "C"
