/*
 * sc_oracle.c -- plain, slow, obviously-correct FP64 CPU oracle of the successive-convolution
 * fast summation (Christlieb, Guthrey, Sands, Thavappiragasm 2020, "Parallel Algorithms for
 * Successive Convolution").
 *
 * TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT: only the tests, the smoke check and the CPU
 * baseline of the benchmark load this file's library.  It shares nothing with the GPU library.
 *
 * Every function follows the paper's steps in the paper's order:
 *   quadrature weights  -> Sec. 2.4 (interpolation on each stencil, eqs. (JR)/(JL)), App. C
 *                          (mirror symmetry for J_L); computed here by direct numerical
 *                          integration of kernel x Lagrange basis, not from App. C's formulas
 *   local integrals     -> Sec. 2.4, eqs. (JR), (JL)
 *   sweeps              -> Sec. 2.4, the two O(N) recurrences
 *   boundary constants  -> Sec. 2.3 (periodic A, B); App. A (Dirichlet value A = u(a)); for L_0
 *                          with Dirichlet data the two end conditions form the 2x2 system of the
 *                          same shape as Sec. 3.3
 *   combine             -> Sec. 2.1 inverse-operator definitions, L_0 as the average of the left
 *                          and right sweeps (Sec. 2.4, Sec. 3.3)
 *   D partial sums      -> Sec. 2.2, eq. (D operators) and the successive relation
 *   time step           -> Sec. 2.1 (alpha choices), Sec. 2.5 (explicit coupling), Sec. 2.2
 *                          first-order representations
 *
 * Readings where the paper is silent (one-sided stencils at Dirichlet ends, the grid convention,
 * which (A,B) conditions hold for Dirichlet L_0) are listed in the design notes of the repository.
 * Built with -O2 -ffp-contract=off: round-to-nearest, no contraction.
 */
#include "sc_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define GL_POINTS 20
static const long double PI_L = 3.141592653589793238462643383279502884L;

/* Gauss-Legendre rule on [-1,1]: Newton iteration on the three-term recurrence of P_n. */
static void gl_rule(int n, long double *x, long double *w)
{
    for (int i = 0; i < (n + 1) / 2; ++i) {
        long double z = cosl(PI_L * ((long double)i + 0.75L) / ((long double)n + 0.5L));
        long double pp = 1.0L;
        for (int it = 0; it < 200; ++it) {
            long double p1 = 1.0L, p2 = 0.0L;
            for (int j = 1; j <= n; ++j) {
                long double p3 = p2;
                p2 = p1;
                p1 = ((2.0L * j - 1.0L) * z * p2 - (j - 1.0L) * p3) / (long double)j;
            }
            pp = (long double)n * (z * p1 - p2) / (z * z - 1.0L);
            long double z1 = z;
            z = z1 - p1 / pp;
            if (fabsl(z - z1) <= 1e-19L * fabsl(z)) {
                /* recompute the derivative at the converged node */
                p1 = 1.0L; p2 = 0.0L;
                for (int j = 1; j <= n; ++j) {
                    long double p3 = p2;
                    p2 = p1;
                    p1 = ((2.0L * j - 1.0L) * z * p2 - (j - 1.0L) * p3) / (long double)j;
                }
                pp = (long double)n * (z * p1 - p2) / (z * z - 1.0L);
                break;
            }
        }
        x[i] = -z;
        x[n - 1 - i] = z;
        w[i] = w[n - 1 - i] = 2.0L / ((1.0L - z * z) * pp * pp);
    }
}

/* Lagrange basis polynomial l_j on nodes eta[0..m-1], evaluated at t. */
static long double lagrange(int m, const int *eta, int j, long double t)
{
    long double p = 1.0L;
    for (int k = 0; k < m; ++k)
        if (k != j) p *= (t - (long double)eta[k]) / (long double)(eta[j] - eta[k]);
    return p;
}

int sco_weights(double nu, int nnodes, const int *eta, double *w)
{
    if (!(nu > 0.0) || nnodes < 1 || nnodes > 16) return -1;
    long double gx[GL_POINTS], gw[GL_POINTS];
    gl_rule(GL_POINTS, gx, gw);
    /* panels of width h with nu*h <= 1/2 so each panel integrand is a gentle exponential */
    int panels = 4 + (int)ceil(2.0 * nu);
    long double h = 1.0L / (long double)panels;
    long double acc[16];
    for (int j = 0; j < nnodes; ++j) acc[j] = 0.0L;
    for (int p = 0; p < panels; ++p) {
        long double a = h * p;
        for (int q = 0; q < GL_POINTS; ++q) {
            long double t = a + 0.5L * h * (gx[q] + 1.0L);
            long double kern = (long double)nu * expl(-(long double)nu * t) * 0.5L * h * gw[q];
            for (int j = 0; j < nnodes; ++j) acc[j] += kern * lagrange(nnodes, eta, j, t);
        }
    }
    for (int j = 0; j < nnodes; ++j) w[j] = (double)acc[j];
    return 0;
}

/* ---------------------------------------------------------------------------------------- */
/* One line                                                                                 */
/* ---------------------------------------------------------------------------------------- */

/* Stencil of the local integral at point i: offsets m (node x_{i+m}).
 * Sixth order: J_R uses x_{i-3..i+2} (Sec. 2.4, the six-point stencil S(i)); J_L the mirror
 * x_{i-2..i+3}.  Fourth order: the centred four-point substencil S_1 = x_{i-2..i+1} for J_R and
 * its mirror x_{i-1..i+2} for J_L. */
static int stencil_lo(int order, int right) { return order == 6 ? (right ? -3 : -2) : (right ? -2 : -1); }

/* Weights for the local integral at point i of a line of n points.  For Dirichlet lines a stencil
 * that would leave [0, n-1] is shifted to the nearest in-range node set of the same width.
 * first[0] receives the absolute index of the first node (periodic: may be negative/wrapped). */
static void local_weights(int bc, int order, int right, double nu, int64_t n, int64_t i,
                          double *w, int64_t *first)
{
    int width = order;
    int64_t lo = i + stencil_lo(order, right);
    if (bc == SCO_BC_DIRICHLET) {
        if (lo < 0) lo = 0;
        if (lo + width - 1 > n - 1) lo = n - width;
    }
    int eta[8];
    for (int j = 0; j < width; ++j) {
        int64_t node = lo + j;
        /* J_R: s = x_i - eta*dx  => eta = i - node;  J_L: s = x_i + eta*dx => eta = node - i */
        eta[j] = right ? (int)(i - node) : (int)(node - i);
    }
    sco_weights(nu, width, eta, w);
    *first = lo;
}

static double vat(const double *v, int64_t n, int64_t idx)
{
    int64_t k = idx % n;
    if (k < 0) k += n;
    return v[k];
}

int sco_line_quad(int bc, int order, double alpha, double dx, int64_t n, const double *v,
                  double *JL, double *JR)
{
    if (order != 4 && order != 6) return -1;
    if (n < order + 1) return -2;
    double nu = alpha * dx;
    /* interior weights are the same at every point of a uniform grid (Sec. 2.4: computed once
     * per direction and reused); only shifted Dirichlet stencils need their own */
    double wRi[8], wLi[8], w[8];
    int64_t first;
    local_weights(SCO_BC_PERIODIC, order, 1, nu, n, 0, wRi, &first);
    local_weights(SCO_BC_PERIODIC, order, 0, nu, n, 0, wLi, &first);
    int edge = order; /* points within this distance of an end may need a shifted stencil */
    for (int64_t i = 0; i < n; ++i) {
        int near_end = (bc == SCO_BC_DIRICHLET) && (i < edge || i > n - 1 - edge);
        /* J_R[i]: cell [x_{i-1}, x_i]; absent at i = 0 for Dirichlet */
        double sR = 0.0;
        if (!(bc == SCO_BC_DIRICHLET && i == 0)) {
            const double *ww = wRi;
            first = i + stencil_lo(order, 1);
            if (near_end) { local_weights(bc, order, 1, nu, n, i, w, &first); ww = w; }
            for (int j = 0; j < order; ++j) sR += ww[j] * vat(v, n, first + j);
        }
        JR[i] = sR;
        /* J_L[i]: cell [x_i, x_{i+1}]; absent at i = n-1 for Dirichlet */
        double sL = 0.0;
        if (!(bc == SCO_BC_DIRICHLET && i == n - 1)) {
            const double *ww = wLi;
            first = i + stencil_lo(order, 0);
            if (near_end) { local_weights(bc, order, 0, nu, n, i, w, &first); ww = w; }
            for (int j = 0; j < order; ++j) sL += ww[j] * vat(v, n, first + j);
        }
        JL[i] = sL;
    }
    return 0;
}

int sco_line_sweep(int bc, double alpha, double dx, int64_t n, const double *JL, const double *JR,
                   double *IL, double *IR, double *ends)
{
    double d = exp(-alpha * dx);
    IR[0] = 0.0;
    for (int64_t i = 1; i < n; ++i) IR[i] = d * IR[i - 1] + JR[i];
    IL[n - 1] = (bc == SCO_BC_PERIODIC) ? JL[n - 1] : 0.0;
    for (int64_t i = n - 2; i >= 0; --i) IL[i] = d * IL[i + 1] + JL[i];
    ends[0] = IL[0];
    /* periodic: I_R(b) adds the wrapped last cell [x_{n-1}, x_n], whose local integral is J_R[0] */
    ends[1] = (bc == SCO_BC_PERIODIC) ? d * IR[n - 1] + JR[0] : IR[n - 1];
    return 0;
}

int sco_line_invL(int bc, int op, int order, double alpha, double dx, int64_t n, const double *v,
                  double ga, double gb, double *out)
{
    if (op < 0 || op > 2) return -1;
    double *JL = malloc(sizeof(double) * n), *JR = malloc(sizeof(double) * n);
    double *IL = malloc(sizeof(double) * n), *IR = malloc(sizeof(double) * n);
    double ends[2];
    int rc = sco_line_quad(bc, order, alpha, dx, n, v, JL, JR);
    if (rc == 0) rc = sco_line_sweep(bc, alpha, dx, n, JL, JR, IL, IR, ends);
    if (rc == 0) {
        int64_t ncell = (bc == SCO_BC_PERIODIC) ? n : n - 1;
        double mu = exp(-alpha * dx * (double)ncell);
        double A = 0.0, B = 0.0;
        if (bc == SCO_BC_PERIODIC) {
            double s = (op == SCO_OP_0) ? 0.5 : 1.0;
            A = s * ends[1] / (1.0 - mu);
            B = s * ends[0] / (1.0 - mu);
        } else if (op == SCO_OP_R) {
            A = ga; /* the value at a is A itself */
        } else if (op == SCO_OP_L) {
            B = gb;
        } else {
            /* L_0^{-1}[v](a) = 0.5 I_L(a) + A + B mu = ga ;  L_0^{-1}[v](b) = 0.5 I_R(b) + A mu + B = gb */
            double r0 = ga - 0.5 * ends[0], r1 = gb - 0.5 * ends[1];
            double det = 1.0 - mu * mu;
            A = (r0 - mu * r1) / det;
            B = (r1 - mu * r0) / det;
        }
        for (int64_t i = 0; i < n; ++i) {
            double ea = exp(-alpha * dx * (double)i);            /* e^{-alpha (x_i - a)} */
            double eb = exp(-alpha * dx * (double)(ncell - i));  /* e^{-alpha (b - x_i)} */
            if (op == SCO_OP_R)
                out[i] = IR[i] + A * ea;
            else if (op == SCO_OP_L)
                out[i] = IL[i] + B * eb;
            else
                out[i] = 0.5 * (IL[i] + IR[i]) + A * ea + B * eb;
        }
    }
    free(JL); free(JR); free(IL); free(IR);
    return rc;
}

/* Nearest-neighbour block form of one application of L_op^{-1} (Sec. 3).  The line is cut into
 * blocks of `block` points (the last takes the remainder); block i holds the local integrals J of
 * its own points.  Steps, in the order of Sec. 3:
 *   1. the local integrals J_R, J_L with the global stencils (the quadrature halo of Sec. 3);
 *   2. each block sweeps its own J from zero (the block-local integrals I_{R,i}, I_{L,i});
 *   3. the N-N constants: block i > 0 receives A_i = the right-moving local integral of block i-1 at
 *      their shared end, block i < last receives B_i = the left-moving local integral of block i+1
 *      at their shared end (Sec. 3.2, the compact forms after the N-N criterion; the left-moving
 *      one read as I_L of the next block);
 *   4. the line constants: A acts on block 0 only and B on the last block only.  Periodic lines take
 *      the periodic choice of Sec. 3.2: A = the last block's own right-moving integral at b (its
 *      sweep continued over the wrapped cell), B = the first block's own left-moving integral at a.
 *      Dirichlet lines impose the end values on the block operators at the end points, with the
 *      coupling e^{-alpha (b - a)} of the two ends dropped (the line is at least one block long);
 *   5. combine as in sco_line_invL, each block with its own constants (Sec. 3.2/3.3 block operators).
 * The result equals sco_line_invL's within e^{-alpha L_m} max|I| when every block spans L_m with
 * e^{-alpha L_m} <= eps (the N-N criterion, eq. (NN constraint general)). */
int sco_line_invL_nn(int bc, int op, int order, double alpha, double dx, int64_t n, int64_t block,
                     const double *v, double ga, double gb, double *out)
{
    if (op < 0 || op > 2 || block < 1) return -1;
    double *JL = malloc(sizeof(double) * n), *JR = malloc(sizeof(double) * n);
    double *IL = malloc(sizeof(double) * n), *IR = malloc(sizeof(double) * n);
    int64_t nb = (n + block - 1) / block;
    double *TR = malloc(sizeof(double) * nb), *TL = malloc(sizeof(double) * nb);
    int rc = sco_line_quad(bc, order, alpha, dx, n, v, JL, JR);
    if (rc == 0) {
        double d = exp(-alpha * dx);
        int64_t ncell = (bc == SCO_BC_PERIODIC) ? n : n - 1;
        /* 2. block-local sweeps from zero; J_R[0] (periodic: the wrapped cell) stays out of the
         *    sweeps as in the global form, J_L[n-1] is the wrapped cell or zero */
        for (int64_t ib = 0; ib < nb; ++ib) {
            int64_t s = ib * block, e = (s + block < n) ? s + block : n;
            IR[s] = (s == 0) ? 0.0 : JR[s];
            for (int64_t i = s + 1; i < e; ++i) IR[i] = d * IR[i - 1] + JR[i];
            IL[e - 1] = (e == n) ? ((bc == SCO_BC_PERIODIC) ? JL[n - 1] : 0.0) : JL[e - 1];
            for (int64_t i = e - 2; i >= s; --i) IL[i] = d * IL[i + 1] + JL[i];
            TR[ib] = IR[e - 1];
            TL[ib] = IL[s];
        }
        /* 3. the neighbours' block-end integrals, carried into each block */
        for (int64_t ib = 0; ib < nb; ++ib) {
            int64_t s = ib * block, e = (s + block < n) ? s + block : n;
            double Ai = (ib > 0) ? TR[ib - 1] : 0.0;
            double Bi = (ib < nb - 1) ? TL[ib + 1] : 0.0;
            for (int64_t i = s; i < e; ++i) {
                IR[i] += Ai * exp(-alpha * dx * (double)(i - s + 1));
                IL[i] += Bi * exp(-alpha * dx * (double)(e - i));
            }
        }
        /* 4. the line constants */
        double A = 0.0, B = 0.0;
        if (bc == SCO_BC_PERIODIC) {
            double sc = (op == SCO_OP_0) ? 0.5 : 1.0;
            A = sc * (d * TR[nb - 1] + JR[0]);
            B = sc * TL[0];
        } else if (op == SCO_OP_R) {
            A = ga;
        } else if (op == SCO_OP_L) {
            B = gb;
        } else {
            A = ga - 0.5 * IL[0];
            B = gb - 0.5 * IR[n - 1];
        }
        /* 5. combine */
        int64_t last0 = (nb - 1) * block;
        for (int64_t i = 0; i < n; ++i) {
            double ea = (i < block) ? exp(-alpha * dx * (double)i) : 0.0;
            double eb = (i >= last0) ? exp(-alpha * dx * (double)(ncell - i)) : 0.0;
            if (op == SCO_OP_R)
                out[i] = IR[i] + A * ea;
            else if (op == SCO_OP_L)
                out[i] = IL[i] + B * eb;
            else
                out[i] = 0.5 * (IL[i] + IR[i]) + A * ea + B * eb;
        }
    }
    free(JL); free(JR); free(IL); free(IR); free(TR); free(TL);
    return rc;
}

/* ---------------------------------------------------------------------------------------- */
/* Whole arrays                                                                             */
/* ---------------------------------------------------------------------------------------- */

static int grid_ok(const sco_grid *g, int dim)
{
    if (!g || g->ndim < 1 || g->ndim > 3 || dim < 0 || dim >= g->ndim) return 0;
    for (int e = 0; e < g->ndim; ++e) if (g->n[e] < 1) return 0;
    return 1;
}

static int64_t total_points(const sco_grid *g)
{
    int64_t t = 1;
    for (int e = 0; e < g->ndim; ++e) t *= g->n[e];
    return t;
}

static int64_t axis_stride(const sco_grid *g, int dim)
{
    int64_t s = 1;
    for (int e = 0; e < dim; ++e) s *= g->n[e];
    return s;
}

static double axis_dx(const sco_grid *g, int dim)
{
    double len = g->hi[dim] - g->lo[dim];
    return g->bc[dim] == SCO_BC_PERIODIC ? len / (double)g->n[dim] : len / (double)(g->n[dim] - 1);
}

/* first element of line L along axis dim */
static int64_t line_base(const sco_grid *g, int dim, int64_t L)
{
    int64_t s = axis_stride(g, dim);
    int64_t inner = L % s, outer = L / s;
    return outer * s * g->n[dim] + inner;
}

int sco_local_quad(const sco_grid *g, int dim, int order, double alpha, const double *v,
                   double *JL, double *JR)
{
    if (!grid_ok(g, dim) || !(alpha > 0.0)) return -1;
    int64_t n = g->n[dim], s = axis_stride(g, dim), lines = total_points(g) / n;
    double dx = axis_dx(g, dim);
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int64_t L = 0; L < lines; ++L) {
        double *buf = malloc(sizeof(double) * 3 * n);
        double *a = buf, *jl = buf + n, *jr = buf + 2 * n;
        int64_t b = line_base(g, dim, L);
        for (int64_t i = 0; i < n; ++i) a[i] = v[b + i * s];
        bad |= (sco_line_quad(g->bc[dim], order, alpha, dx, n, a, jl, jr) != 0);
        for (int64_t i = 0; i < n; ++i) { JL[b + i * s] = jl[i]; JR[b + i * s] = jr[i]; }
        free(buf);
    }
    return bad ? -2 : 0;
}

int sco_sweep_LR(const sco_grid *g, int dim, double alpha, const double *JL, const double *JR,
                 double *IL, double *IR, double *ends)
{
    if (!grid_ok(g, dim) || !(alpha > 0.0)) return -1;
    int64_t n = g->n[dim], s = axis_stride(g, dim), lines = total_points(g) / n;
    double dx = axis_dx(g, dim);
#pragma omp parallel for schedule(static)
    for (int64_t L = 0; L < lines; ++L) {
        double *buf = malloc(sizeof(double) * 4 * n);
        double *jl = buf, *jr = buf + n, *il = buf + 2 * n, *ir = buf + 3 * n;
        int64_t b = line_base(g, dim, L);
        for (int64_t i = 0; i < n; ++i) { jl[i] = JL[b + i * s]; jr[i] = JR[b + i * s]; }
        sco_line_sweep(g->bc[dim], alpha, dx, n, jl, jr, il, ir, ends + 2 * L);
        for (int64_t i = 0; i < n; ++i) { IL[b + i * s] = il[i]; IR[b + i * s] = ir[i]; }
        free(buf);
    }
    return 0;
}

int sco_apply_invL(const sco_grid *g, int dim, int op, int order, double alpha,
                   const double *gvals, const double *v, double *out)
{
    return sco_apply_D_partial_sum(g, dim, op, order, alpha, 0, 1.0, gvals, v, out);
}

/* k == 0 is the internal spelling of "return L^{-1}[v]" */
int sco_apply_D_partial_sum(const sco_grid *g, int dim, int op, int order, double alpha, int k,
                            double scale, const double *gvals, const double *v, double *out)
{
    if (!grid_ok(g, dim) || !(alpha > 0.0) || op < 0 || op > 2 || k < 0) return -1;
    int64_t n = g->n[dim], s = axis_stride(g, dim), lines = total_points(g) / n;
    double dx = axis_dx(g, dim);
    int bc = g->bc[dim];
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int64_t L = 0; L < lines; ++L) {
        double *buf = malloc(sizeof(double) * 3 * n);
        double *w = buf, *t = buf + n, *acc = buf + 2 * n;
        int64_t b = line_base(g, dim, L);
        double ga = gvals ? gvals[2 * L] : 0.0, gb = gvals ? gvals[2 * L + 1] : 0.0;
        for (int64_t i = 0; i < n; ++i) { w[i] = v[b + i * s]; acc[i] = 0.0; }
        if (k == 0) {
            bad |= (sco_line_invL(bc, op, order, alpha, dx, n, w, ga, gb, t) != 0);
            for (int64_t i = 0; i < n; ++i) acc[i] = t[i];
        } else {
            for (int p = 1; p <= k; ++p) {
                /* w_p = D[w_{p-1}] = w_{p-1} - L^{-1}[w_{p-1}] */
                bad |= (sco_line_invL(bc, op, order, alpha, dx, n, w, ga, gb, t) != 0);
                for (int64_t i = 0; i < n; ++i) { w[i] = w[i] - t[i]; acc[i] += w[i]; }
            }
        }
        for (int64_t i = 0; i < n; ++i) out[b + i * s] = scale * acc[i];
        free(buf);
    }
    return bad ? -2 : 0;
}

int sco_apply_invL_nn(const sco_grid *g, int dim, int op, int order, double alpha, int64_t block,
                      const double *gvals, const double *v, double *out)
{
    if (!grid_ok(g, dim) || !(alpha > 0.0) || op < 0 || op > 2 || block < 1) return -1;
    int64_t n = g->n[dim], s = axis_stride(g, dim), lines = total_points(g) / n;
    double dx = axis_dx(g, dim);
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int64_t L = 0; L < lines; ++L) {
        double *buf = malloc(sizeof(double) * 2 * n);
        int64_t b = line_base(g, dim, L);
        double ga = gvals ? gvals[2 * L] : 0.0, gb = gvals ? gvals[2 * L + 1] : 0.0;
        for (int64_t i = 0; i < n; ++i) buf[i] = v[b + i * s];
        bad |= (sco_line_invL_nn(g->bc[dim], op, order, alpha, dx, n, block, buf, ga, gb, buf + n) != 0);
        for (int64_t i = 0; i < n; ++i) out[b + i * s] = buf[n + i];
        free(buf);
    }
    return bad ? -2 : 0;
}

int sco_time_step(const sco_grid *g, const sco_pde *p, int nsteps, double *u)
{
    if (!g || !p || g->ndim < 1 || g->ndim > 3 || !(p->dt > 0.0) || !(p->beta > 0.0)) return -1;
    int64_t tot = total_points(g);
    double *acc = malloc(sizeof(double) * tot), *dterm = malloc(sizeof(double) * tot);
    int rc = 0;
    for (int step = 0; step < nsteps && rc == 0; ++step) {
        memcpy(acc, u, sizeof(double) * tot);
        for (int dim = 0; dim < g->ndim && rc == 0; ++dim) {
            if (p->split && dim > 0) memcpy(u, acc, sizeof(double) * tot); /* next axis acts on the result */
            double c = p->c[dim];
            if (c != 0.0) {
                /* alpha = beta / (|c| dt); c > 0 uses the left-biased d/dx ~ alpha D_R, c < 0 the
                 * right-biased d/dx ~ -alpha D_L; dt * (-c d/dx u) = -|c| dt alpha D[u] */
                double a = p->beta / (fabs(c) * p->dt);
                int op = c > 0.0 ? SCO_OP_R : SCO_OP_L;
                rc = sco_apply_D_partial_sum(g, dim, op, p->order, a, 1, 1.0, NULL, u, dterm);
                double coef = -fabs(c) * p->dt * a;
                for (int64_t q = 0; q < tot; ++q) acc[q] += coef * dterm[q];
            }
            if (p->nu_diff > 0.0 && rc == 0) {
                /* alpha = beta / sqrt(nu dt); dt * nu * d_xx u ~ -nu dt alpha^2 D_0[u] */
                double a = p->beta / sqrt(p->nu_diff * p->dt);
                rc = sco_apply_D_partial_sum(g, dim, SCO_OP_0, p->order, a, 1, 1.0, NULL, u, dterm);
                double coef = -p->nu_diff * p->dt * a * a;
                for (int64_t q = 0; q < tot; ++q) acc[q] += coef * dterm[q];
            }
        }
        memcpy(u, acc, sizeof(double) * tot);
    }
    free(acc); free(dterm);
    return rc;
}

int sco_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the OpenMP loops over lines (for timing single-thread and all-core runs). */
int sco_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}
