/*
 * sc.h -- C ABI of the MI355X (gfx950) successive-convolution library.
 *
 * The library applies, line by line along one axis of a dense 1-3 dimensional array, the
 * exponential-kernel convolution operators of Christlieb, Guthrey, Sands & Thavappiragasm (2020),
 * "Parallel Algorithms for Successive Convolution":
 *   L_L^{-1}[v](x) = alpha int_x^b e^{-alpha(s-x)} v ds + B e^{-alpha(b-x)}          (Sec. 2.1)
 *   L_R^{-1}[v](x) = alpha int_a^x e^{-alpha(x-s)} v ds + A e^{-alpha(x-a)}          (Sec. 2.1)
 *   L_0^{-1}[v](x) = alpha/2 int_a^b e^{-alpha|x-s|} v ds + A e^{-alpha(x-a)} + B e^{-alpha(b-x)}
 * computed in O(N) per line by local quadrature (Sec. 2.4, eqs. (JR), (JL); sixth-order rule of
 * Sec. 2.4 / App. C, or its centred fourth-order substencil), two recursive sweeps
 * I_R(x_i) = e^{-alpha dx} I_R(x_{i-1}) + J_R(x_i), I_L(x_i) = e^{-alpha dx} I_L(x_{i+1}) + J_L(x_i)
 * (Sec. 2.4), and the boundary constants A, B (Sec. 2.3 periodic; Dirichlet values enforced at the
 * two ends, App. A).  D = I - L^{-1} and its partial sums (Sec. 2.2) stand in for derivatives.
 *
 * Memory and ownership
 *   - All array pointers are DEVICE pointers owned by the caller (hipMalloc or torch tensors),
 *     dense, C order, axis 0 (x) contiguous: element (i0, i1, i2) at i0 + n0*(i1 + n1*i2).
 *   - Pointers to arrays of the data type must be aligned to the element size.  The library
 *     allocates no device memory and keeps no state between calls except read-only tables, with
 *     one exception: a batch plan (sc_batch_plan_create, sc_batch_tune) holds its launch tables
 *     in device memory it allocates (hipMalloc) and frees in sc_batch_plan_destroy; rebuilding them
 *     (creation, tuning) synchronises the device.
 *   - Every call is asynchronous on `stream` (0 = the null stream); SC_OK means "validated and
 *     enqueued".  Device-side faults surface at the caller's next synchronisation.
 *   - `out` must not overlap `v`.  Workspace buffers (`ws`) are caller-owned device memory of at
 *     least sc_workspace_bytes() bytes, 256-byte aligned; their contents on entry are ignored.
 *
 * Grid conventions (SC_BC_PERIODIC): n stored points x_i = lo + i*dx, dx = (hi-lo)/n, the point
 * x_n = x_0 is not stored.  SC_BC_DIRICHLET: n stored points including both ends, dx = (hi-lo)/(n-1).
 * "Lines" of axis d are numbered row-major over the remaining axes (highest axis slowest); Dirichlet
 * values are given as 2 doubles per line (value at lo, value at hi), NULL meaning zero.
 *
 * Errors: every function returns an sc_status; on failure nothing is enqueued and sc_last_error()
 * returns a message (thread-local, valid until the next call on the same thread).  No C++
 * exception crosses this interface.
 */
#ifndef SC_H
#define SC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t *sc_stream_t; /* hipStream_t */

typedef enum {
    SC_OK = 0,
    SC_ERR_ARG = -1,         /* invalid argument (null pointer, alpha <= 0, bad dim/op/k, overlap) */
    SC_ERR_SHAPE = -2,       /* line too short for the stencil, or sizes out of range */
    SC_ERR_UNSUPPORTED = -3, /* valid request the library does not implement */
    SC_ERR_WORKSPACE = -4,   /* workspace missing or smaller than sc_workspace_bytes() */
    SC_ERR_DEVICE = -5       /* a HIP call or kernel launch failed */
} sc_status;

typedef enum {
    SC_F64 = 0,      /* FP64 data and arithmetic */
    SC_F32_MIXED = 1 /* FP32 data, quadrature and in-segment sweeps; in-wave carries as compensated
                        FP32 (hi, lo) pairs; FP64 boundary constants (A,B) and carries across
                        wave-parts and chunks.  sc_local_quad / sc_sweep_LR accumulate in FP64 and
                        round their FP32 outputs once. */
} sc_dtype;

/* L_L^{-1}, L_R^{-1}, L_0^{-1}.  Entry points take the operator as an int holding one of these
 * values (any other value is rejected with SC_ERR_ARG). */
typedef enum { SC_OP_L = 0, SC_OP_R = 1, SC_OP_0 = 2 } sc_op;
typedef enum { SC_BC_PERIODIC = 0, SC_BC_DIRICHLET = 1 } sc_bc;

typedef struct {
    int32_t ndim;     /* 1..3 */
    int64_t n[3];     /* stored points per axis; n[0] = x (contiguous); unused axes = 1 */
    double lo[3];     /* domain [lo, hi] per axis */
    double hi[3];
    int32_t bc[3];    /* sc_bc per axis */
    int32_t dtype;    /* sc_dtype: element type of every array argument */
} sc_grid;

/* Local integrals along axis `dim` (Sec. 2.4, eqs. (JR), (JL)); order 4 or 6.
 * JR[i] integrates cell [x_{i-1}, x_i], JL[i] cell [x_i, x_{i+1}] (periodic: wrapped cells at the
 * ends; Dirichlet: JR = 0 at the first and JL = 0 at the last point, one-sided 6/4-point stencils
 * within order/2 points of an end).  v, JL, JR: arrays of the grid's shape and dtype. */
sc_status sc_local_quad(const sc_grid *grid, int dim, int order, double alpha, const void *v,
                        void *JL, void *JR, sc_stream_t stream);

/* Raw recursive sweeps along `dim` (Sec. 2.4): IR[0] = 0, IR[i] = d IR[i-1] + JR[i];
 * IL[last] = JL[last], IL[i] = d IL[i+1] + JL[i], d = e^{-alpha dx}.  line_ends (FP64, 2 per line):
 * [I_L(a), I_R(b)] with I_R(b) = d IR[n-1] + JR[0] for periodic axes.  No boundary constants. */
sc_status sc_sweep_LR(const sc_grid *grid, int dim, double alpha, const void *JL, const void *JR,
                      void *IL, void *IR, double *line_ends, sc_stream_t stream);

/* out = L_op^{-1}[v] along `dim` with the boundary constants of Sec. 2.3 (periodic) or the
 * Dirichlet values (2 per line, FP64, device; NULL = 0).  ws: see sc_workspace_bytes(). */
sc_status sc_apply_invL(const sc_grid *grid, int dim, int op, int order, double alpha,
                        const double *dirichlet_g, const void *v, void *out, void *ws,
                        size_t ws_bytes, sc_stream_t stream);

/* sc_apply_invL for callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same operation, arguments and errors
 * as sc_apply_invL, without a workspace.  The per-(line, chunk) sweep totals and carries of
 * chunked passes go to a fixed scratch array of SC_NOALLOC_SCRATCH_BYTES in the library's device
 * image, one per GPU, held until the process ends; a pass that needs more (sc_workspace_bytes
 * with which = 0, less its 256 bytes of alignment slack) fails with SC_ERR_WORKSPACE before
 * anything is enqueued.  The call allocates nothing.  It uses the copy of the current device (the
 * stream must belong to it).  All calls on one GPU share that array: calls that overlap in time on
 * one GPU (different streams, or threads) race and give wrong results; calls ordered on one stream
 * are safe, each writes every entry it reads. */
#define SC_NOALLOC_SCRATCH_BYTES (8u << 20)
sc_status sc_apply_invL_noalloc(const sc_grid *grid, int dim, int op, int order, double alpha,
                                const double *dirichlet_g, const void *v, void *out, sc_stream_t stream);

/* Points per chunk of the passes along `dim` for this grid (the length of the line segment one
 * workgroup tile sweeps; lines longer than this are chunked), or -1 for an invalid grid or dim. */
int64_t sc_chunk_points(const sc_grid *grid, int dim);

/* out = L_op^{-1}[v] along `dim` in the nearest-neighbour block form of Sec. 3: each line is cut
 * into virtual blocks of block_points points (the last block takes the remainder), the one-GPU
 * stand-in for the blocks of a domain decomposition.  Each block sweeps its own local integrals
 * from zero; block i > 0 receives only block i-1's right-moving block-end integral and block
 * i < last only block i+1's left-moving one (Sec. 3.2/3.3 block operators with the N-N
 * constants); the line's boundary constants act on the end blocks only: periodic lines take the
 * periodic choice of Sec. 3.2 (the last block's own I_R at b, the first block's own I_L at a);
 * Dirichlet lines impose their end values on the end blocks' operators.  The coupling
 * e^{-alpha (b - a)} between the two ends is dropped.  When every block spans L_m with
 * e^{-alpha L_m} <= eps (the N-N criterion, eq. (NN constraint general)) the result equals
 * sc_apply_invL's within eps * max|I| plus rounding; shorter blocks give the truncated operator.
 * block_points: a positive multiple of sc_chunk_points(grid, dim), or at least the line length
 * (one block); otherwise SC_ERR_ARG.  Other arguments, layout and the workspace
 * (sc_workspace_bytes with which = 0) as for sc_apply_invL. */
sc_status sc_apply_invL_nn(const sc_grid *grid, int dim, int op, int order, double alpha, int64_t block_points,
                           const double *dirichlet_g, const void *v, void *out, void *ws, size_t ws_bytes,
                           sc_stream_t stream);

/* out = scale * sum_{p=1..k} D^p[v], D = I - L_op^{-1} (Sec. 2.2, successive relation), k in 1..8.
 * scale = +alpha, -alpha, -alpha^2 gives the left-biased, right-biased and second derivative
 * representations.  Dirichlet axes support k = 1 only (SC_ERR_UNSUPPORTED otherwise). */
sc_status sc_apply_D_partial_sum(const sc_grid *grid, int dim, int op, int order, double alpha,
                                 int k, double scale, const double *dirichlet_g, const void *v,
                                 void *out, void *ws, size_t ws_bytes, sc_stream_t stream);

/* u_t + c . grad u = nu_diff lap u, advanced `nsteps` forward-Euler steps in place:
 *   u <- u - sum_d |c_d| dt alpha_d D_{R or L, d}[u] - sum_d nu_diff dt alpha_nu^2 D_{0,d}[u]
 * with alpha_d = beta/(|c_d| dt) (D_R if c_d > 0, D_L if c_d < 0) and alpha_nu = beta/sqrt(nu dt)
 * (Sec. 2.1 alpha choices; Sec. 2.2 first-order representations; Sec. 2.5 explicit coupling).
 * split = 0: all D terms act on u^n and are summed (the coupling of Sec. 2.5; its amplification
 * of grid-scale modes is 1 - d (beta + beta^2) with both operators on d axes, so |.| <= 1 needs
 * d (beta + beta^2) <= 2).  split = 1: dimension splitting -- the same 1-D step applied to each
 * axis in turn, x then y then z, each acting on the previous one's result (per-axis factors of
 * modulus <= 1 at beta = 1).  Dirichlet axes hold u = 0 at both ends.  nn_policy applies the
 * nearest-neighbour time-step bound of Sec. 3.1 with tolerance nn_eps over blocks of length
 * block_len (0 = the whole axis):
 * 0 = ignore, 1 = reduce dt to the bound, 2 = fail with SC_ERR_ARG if dt exceeds it.
 * stages = s in {2, 3} (Sec. 2.5): an s-stage explicit Runge-Kutta method coupled to partial sums of
 * the same order -- every D above replaced by S_s = sum_{p=1..s} D^p -- in the strong-stability-
 * preserving Shu-Osher forms (E = the additive Euler step with S_s; s = 2: u1 = E(u), u <- u/2 +
 * E(u1)/2; s = 3: u1 = E(u), u2 = 3u/4 + E(u1)/4, u <- u/3 + 2E(u2)/3); O(dt^s).  Unsplit, periodic
 * axes only (SC_ERR_UNSUPPORTED otherwise).  Stability needs beta small enough that the Euler
 * increment of every mode stays in the method's region: a d-dimensional diffusion increment reaches
 * -d s beta^2 (s = 2: >= -2; s = 3: >= -2.51). */
typedef struct {
    double c[3];
    double nu_diff;
    double beta;
    double dt;
    int32_t order;    /* 4 or 6 */
    int32_t nn_policy;
    double nn_eps;    /* 0 -> 1e-16 */
    double block_len; /* 0 -> axis length */
    int32_t split;    /* 0 additive (unsplit), 1 dimension-split x, y, z */
    int32_t stages;   /* 0 or 1: the Euler step above; 2, 3: s-stage SSP Runge-Kutta (see above) */
} sc_linear_pde;

sc_status sc_time_step(const sc_grid *grid, const sc_linear_pde *pde, int nsteps, void *u,
                       void *ws, size_t ws_bytes, sc_stream_t stream);

/* Workspace bytes needed by one call: which = 0 sc_apply_invL, 1 sc_apply_D_partial_sum (for k),
 * 2 sc_time_step (k = the number of stages; 1 for the Euler step).  Returns 0 on invalid arguments. */
size_t sc_workspace_bytes(const sc_grid *grid, int dim, int which, int k);

/* The time step actually used by sc_time_step for this pde (after the nearest-neighbour policy),
 * or a negative value on invalid arguments. */
double sc_effective_dt(const sc_grid *grid, const sc_linear_pde *pde);

const char *sc_last_error(void);

/* ------------------------------------------------------------------------------------------------
 * Batches of independent instances.  Instance i is nlines lines of n points at element offset
 * `offset` of the batch arrays v and out (the same offset in both; dtype of the plan): axis 0, the
 * points of line l are contiguous (point p at offset + l n + p: x lines); axis 1, the lines are
 * interleaved (point p at offset + p nlines + l: the y lines of an array of n rows of nlines points).
 * Each line is on [lo, hi] with the grid convention of sc_grid, with its instance's alpha, boundary
 * and operator.  The plan applies, along every instance's lines, L_op^{-1} (k = 0) or scale * D
 * (k = 1) -- the operations of sc_apply_invL / sc_apply_D_partial_sum -- in one launch per tile shape.
 * ---------------------------------------------------------------------------------------------- */
typedef struct {
    int64_t offset;   /* element offset of the instance's first point in v and out */
    int64_t n;        /* points per line, >= order + 1 */
    int64_t nlines;   /* >= 1 */
    double lo, hi;
    double alpha;     /* > 0, alpha dx < 700 */
    double scale;     /* result multiplier for k = 1 */
    int64_t g_offset; /* Dirichlet values: 2 per line (a, b) from this FP64 offset of g; -1 = zero */
    int32_t bc;       /* sc_bc */
    int32_t op;       /* sc_op */
    int32_t k;        /* 0 or 1 */
    int32_t axis;     /* 0: contiguous lines; 1: interleaved lines (see above) */
} sc_batch_item;

typedef struct sc_batch_plan_s *sc_batch_plan;

/* Validates the instances (copied) and prepares the launches with the tile shapes the autotuner
 * chose earlier in this process for instances of the same class (axis; line length rounded up to a
 * power of two; single- or multi-line), default shapes otherwise.  Allocates the plan's device
 * tables (hipMalloc) on the current device and a private capture stream.  dtype: sc_dtype. */
sc_status sc_batch_plan_create(const sc_batch_item *items, int count, int dtype, int order, sc_batch_plan *plan);
sc_status sc_batch_plan_destroy(sc_batch_plan plan);
/* Workspace bytes enough for any tile shape and for sc_batch_apply_per_instance. */
size_t sc_batch_workspace_bytes(sc_batch_plan plan);
/* Elements of v and out the instances span (max of offset + n * nlines). */
int64_t sc_batch_elements(sc_batch_plan plan);
/* Enqueues the batch on `stream`.  use_graph = 1: the launches are captured once into a HIP graph
 * (re-captured when an array pointer changes) and replayed with one hipGraphLaunch.  out must not
 * overlap v; g (FP64 device) is needed if any instance has g_offset >= 0. */
sc_status sc_batch_apply(sc_batch_plan plan, const void *v, void *out, const double *g, void *ws, size_t ws_bytes,
                         int use_graph, sc_stream_t stream);
/* The same results through one sc_apply_invL / sc_apply_D_partial_sum call per instance. */
sc_status sc_batch_apply_per_instance(sc_batch_plan plan, const void *v, void *out, const double *g, void *ws,
                                      size_t ws_bytes, sc_stream_t stream);
/* Autotuner: times every candidate tile shape (chunk length and lines per tile of the variants of
 * the class's axis: x-line tiles, or strided tiles of 16 or 32 lines; persistent or one workgroup
 * per work item; windowed or exact chunk carries where the windowed ones apply) on each class of
 * the plan's instances, `reps` runs each, on the caller's arrays (out is overwritten), keeps the
 * fastest per class for this plan and for plans created later in the process
 * (sc_batch_tune_export saves the table).
 * Synchronises `stream`; needs ws_bytes >= sc_batch_workspace_bytes(plan). */
sc_status sc_batch_tune(sc_batch_plan plan, const void *v, void *out, const double *g, void *ws, size_t ws_bytes,
                        int reps, sc_stream_t stream);
/* JSON description of the plan's launches and tile shapes; returns its length (buf may be NULL). */
int sc_batch_describe(sc_batch_plan plan, char *buf, int len);
/* The autotuner's table of this process as text, one class a line: "elem order nbits multi variant
 * persistent exact axis" (elem 8 or 4 bytes; nbits = ceil(log2 n); multi = nlines >= 4; exact = 1:
 * exact chunk carries where the windowed ones would apply; axis of the instances; import also takes
 * lines without the axis, as axis 0).  Returns its length; writes at most len - 1
 * characters and a terminating 0 to buf (buf may be NULL). */
int sc_batch_tune_export(char *buf, int len);
/* Merges such a table (e.g. saved from an earlier process) into this process's; plans created
 * afterwards use it.  Rejects the whole text with SC_ERR_ARG if a line is malformed or names a
 * shape not built for its element type. */
sc_status sc_batch_tune_import(const char *text);

/* ------------------------------------------------------------------------------------------------
 * Nonlinear Hamilton-Jacobi equation u_t + H(u_x, u_y) = S on a periodic 2-D grid (FP64,
 * shape (n[1], n[0])), first order in time (Sec. 2.5): u <- u - dt H^ with the Lax-Friedrichs
 * numerical Hamiltonian H^ of the one-sided derivatives u_x^- = alpha D_R[u], u_x^+ = -alpha D_L[u]
 * (and likewise in y).  The local integrals use a 5-point WENO quadrature built from three 3-point
 * substencils (Sec. 2.4) with
 *   weights = 0: the linear weights d_r (smooth data),
 *             1: WENO-Z nonlinear weights (smoothness: squared second difference per substencil),
 *             2: weights proposed by the learned MLP (sc_mlp_*), each proposal judged against the
 *                WENO-Z weights and replaced by them when some weight differs by more than theta.
 * Adaptive step with one lagged wave speed c (held on the device): dt = cfl min(dx, dy) / c, the
 * last step shortened to land on t_end; alpha = beta / (cfl min(dx, dy)) on both axes; the LF
 * dissipation is c; c is then replaced by the largest |H_p|, |H_q| over the step's one-sided
 * derivatives.  This is the adaptive rule of Sec. 4.5 with its wave speeds taken equal (as the
 * paper's own examples do); where max |H_p| = max |H_q| on a square grid -- Example 3, the data
 * sin x + sin y -- it coincides with the per-axis rule dt = cfl min(dx / c_x, dy / c_y). 
 * state (device, 8 doubles): [c, t, steps, fallbacks, summed judged error, proposals judged, -, -].
 * ---------------------------------------------------------------------------------------------- */
typedef struct {
    double beta;      /* > 0 */
    double cfl;       /* > 0 */
    double t_end;     /* steps stop advancing past t_end */
    double theta;     /* learned weights: largest accepted |proposal - WENO-Z| per weight */
    int32_t weights;  /* 0 linear, 1 WENO-Z, 2 learned */
    int32_t hamiltonian; /* 0: (u_x^2 + u_y^2) / 2; 1: Example 3 of Sec. 5.1, (1 + u_x + u_y)^2 / 2 with
                            the source S = sin x + sin y + (1 + t cos x + t cos y)^2 / 2 of the
                            manufactured solution u = t (sin x + sin y) on the right-hand side */
} sc_hj_params;

size_t sc_hj_workspace_bytes(const sc_grid *grid);
/* state <- initial wave speed (max of periodic central differences of u), t = 0, counters 0. */
sc_status sc_hj_init(const sc_grid *grid, const sc_hj_params *p, const void *u, double *state, void *ws,
                     size_t ws_bytes, sc_stream_t stream);
/* nsteps steps in place (no host synchronisation: dt is read from state on the device).
 * mlp_params: device FP32 parameters of the proposer (weights = 2), else may be NULL. */
sc_status sc_hj_step(const sc_grid *grid, const sc_hj_params *p, int nsteps, void *u, double *state,
                     const float *mlp_params, void *ws, size_t ws_bytes, sc_stream_t stream);
/* Training samples from a field: for every point and side (rows 2p: J_R stencil, 2p + 1: J_L) the
 * proposer's 8 features (X, FP32) and the WENO-Z weights (Y, 3 FP32) along `axis`. */
sc_status sc_hj_harvest(const sc_grid *grid, const sc_hj_params *p, const void *u, int axis, float *X, float *Y,
                        sc_stream_t stream);

/* The proposer: features (8) -> 32 -> 32 -> 3 with ReLU and softmax; FP32 master parameters on
 * the device, row-major (out, in) weights each followed by its bias (W1 b1 W2 b2 W3 b3); the matrix
 * products run on the matrix cores with BF16 operands and FP32 accumulation. */
int sc_mlp_param_count(void);
sc_status sc_mlp_forward(const float *params, int64_t n, const float *X, float *Y, sc_stream_t stream);
size_t sc_mlp_grad_workspace_bytes(int64_t n);
/* grad = d loss / d params, loss = mean over the n samples of sum_r (omega_r - Y_r)^2 (device). */
sc_status sc_mlp_grad(const float *params, int64_t n, const float *X, const float *Y, float *grad, float *loss,
                      void *ws, size_t ws_bytes, sc_stream_t stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8); step >= 1 is the update count. */
sc_status sc_mlp_adam(float *params, const float *grad, float *m, float *v, int step, float lr, sc_stream_t stream);

/* Optional per-kernel timing with HIP events recorded on the caller's stream around every launch
 * the library makes (for benchmarks).  sc_timing_read returns the number of kernel names written;
 * ms[i] is the summed elapsed time and counts[i] the launches of names[i] since the last reset.
 * Reading synchronises the events. */
sc_status sc_timing_enable(int on);
/* Restrict the timing to the launches whose kernel names appear in `names` (comma-separated, e.g.
 * "line_pass_apply_y,line_pass_fused_x"); NULL or "" times every launch.  Each timed launch adds
 * two event records to the stream, so a benchmark that times one kernel inside its measured region
 * selects just that kernel.  The string is copied; SC_ERR_ARG if it is longer than 1023 bytes. */
sc_status sc_timing_select(const char *names);
int sc_timing_read(char names[][64], double *ms, int *counts, int max_entries);
void sc_timing_reset(void);

#ifdef __cplusplus
}
#endif
#endif
