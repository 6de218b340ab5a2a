/*
 * sc_oracle.h -- plain FP64 CPU oracle of the successive-convolution fast summation.
 *
 * TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code, header, table or
 * constant generator with the GPU library; the two are independent derivations of the same
 * mathematics (Christlieb, Guthrey, Sands, Thavappiragasm, "Parallel Algorithms for Successive
 * Convolution", 2020).
 *
 * Conventions (used identically by the GPU library, but restated here on purpose):
 *   - arrays are dense, shape [n2][n1][n0], axis 0 (x) contiguous;
 *   - periodic axis: n stored points x_i = a + i*dx, i = 0..n-1, dx = (b-a)/n, x_n == x_0 not stored;
 *   - Dirichlet axis: n stored points including both ends, dx = (b-a)/(n-1);
 *   - "lines" of axis d are enumerated row-major over the remaining axes (highest axis slowest);
 *   - op 0 = L_L^{-1} (left-moving), op 1 = L_R^{-1} (right-moving), op 2 = L_0^{-1} (second
 *     derivative), the operators of Sec. 2.1, eqs. for the inverse operators.
 */
#ifndef SC_ORACLE_H
#define SC_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { SCO_OP_L = 0, SCO_OP_R = 1, SCO_OP_0 = 2 };
enum { SCO_BC_PERIODIC = 0, SCO_BC_DIRICHLET = 1 };

typedef struct {
    int32_t ndim;
    int64_t n[3];
    double lo[3], hi[3];
    int32_t bc[3];
} sco_grid;

/* Quadrature weights w_j = nu * int_0^1 exp(-nu*eta) l_j(eta) d eta, where l_j is the Lagrange
 * basis polynomial on the nodes eta[0..nnodes-1] (node positions in units of dx, measured from the
 * evaluation point into the cell; Sec. 2.4 eqs. (JR), (JL) and the interpolation step on each
 * stencil).  Composite Gauss-Legendre in long double.  Returns 0 on success. */
int sco_weights(double nu, int nnodes, const int *eta, double *w);

/* Local integrals J_R, J_L of one line (Sec. 2.4, eqs. (JR), (JL)); order 4 or 6.
 * Periodic: J_R[0] is the wrapped cell [x_{n-1}, x_n]; J_L[n-1] the wrapped cell [x_{n-1}, x_n].
 * Dirichlet: J_R[0] = 0 and J_L[n-1] = 0 (no such cells); one-sided stencils near the ends. */
int sco_line_quad(int bc, int order, double alpha, double dx, int64_t n, const double *v,
                  double *JL, double *JR);

/* Raw sweeps of one line (Sec. 2.4 recurrences): I_R[0] = 0, I_R[i] = d I_R[i-1] + J_R[i];
 * I_L[n-1] = J_L[n-1], I_L[i] = d I_L[i+1] + J_L[i]; ends[0] = I_L(a), ends[1] = I_R(b). */
int sco_line_sweep(int bc, double alpha, double dx, int64_t n, const double *JL, const double *JR,
                   double *IL, double *IR, double *ends);

/* One application of L_op^{-1} to one line, with boundary coefficients A, B (Sec. 2.3 periodic
 * constants; Dirichlet values ga, gb enforced at the ends). */
int sco_line_invL(int bc, int op, int order, double alpha, double dx, int64_t n, const double *v,
                  double ga, double gb, double *out);

/* Nearest-neighbour block form of sco_line_invL (Sec. 3): blocks of `block` points sweep their own
 * local integrals from zero and exchange only their block-end integrals with their neighbours;
 * the line constants act on the end blocks only (periodic choice of Sec. 3.2; Dirichlet end
 * values imposed on the end blocks' operators). */
int sco_line_invL_nn(int bc, int op, int order, double alpha, double dx, int64_t n, int64_t block,
                     const double *v, double ga, double gb, double *out);

/* Whole-array drivers (line by line along axis `dim`).  g: Dirichlet values, 2 per line
 * (g_a, g_b), NULL = 0.  Return 0 on success, negative on invalid arguments. */
int sco_local_quad(const sco_grid *g, int dim, int order, double alpha, const double *v,
                   double *JL, double *JR);
int sco_sweep_LR(const sco_grid *g, int dim, double alpha, const double *JL, const double *JR,
                 double *IL, double *IR, double *ends);
int sco_apply_invL(const sco_grid *g, int dim, int op, int order, double alpha,
                   const double *gvals, const double *v, double *out);
/* sco_line_invL_nn along every line of axis `dim`. */
int sco_apply_invL_nn(const sco_grid *g, int dim, int op, int order, double alpha, int64_t block,
                      const double *gvals, const double *v, double *out);
/* out = scale * sum_{p=1..k} D^p[v], D = I - L_op^{-1} (Sec. 2.2, successive relation). */
int sco_apply_D_partial_sum(const sco_grid *g, int dim, int op, int order, double alpha, int k,
                            double scale, const double *gvals, const double *v, double *out);

/* Forward-Euler step of u_t + c . grad u = nu_diff * lap u with D operators (Sec. 2.1 alpha
 * choices, Sec. 2.5 coupling, first-order representations); Dirichlet axes use g = 0.
 * split = 0: every axis' D terms act on u^n and are added (the explicit coupling of Sec. 2.5);
 * split = 1: dimension splitting, one such 1-D step per axis in turn (x, then y, then z). */
typedef struct {
    double c[3];
    double nu_diff;
    double beta;
    double dt;
    int32_t order;
    int32_t split;
} sco_pde;
int sco_time_step(const sco_grid *g, const sco_pde *p, int nsteps, double *u);

/* Number of threads the OpenMP loops use (for reporting). */
int sco_num_threads(void);

#ifdef __cplusplus
}
#endif
#endif
