// sc_coeffs.cpp -- host-side FP64 quadrature weights of the local integrals.
//
// J_R(x_i) = alpha int_{x_{i-1}}^{x_i} e^{-alpha(x_i - s)} v(s) ds  (Sec. 2.4, eq. (JR)) with v
// replaced by its Lagrange interpolant on a stencil becomes, in the variable eta = (x_i - s)/dx,
//     J_R(x_i) = sum_j w_j v_j,   w_j = nu int_0^1 e^{-nu eta} l_j(eta) d eta,   nu = alpha dx,
// where node x_{i+m} sits at eta = -m (J_L mirrors this: s = x_i + eta dx, node x_{i+m} at
// eta = +m; App. C, mirror symmetry).  Expanding l_j(eta) = sum_q a_{jq} eta^q gives
//     w_j = sum_q a_{jq} E_q(nu),   E_q(nu) = nu int_0^1 e^{-nu eta} eta^q d eta,
// and E_q is evaluated from the all-positive series  E_q = q! e^{-nu} sum_{l>=1} nu^l / (q+l)!
// (no cancellation at small nu, unlike the closed forms of App. C) or, for nu > 30, the upward
// recurrence E_q = (q/nu) E_{q-1} - e^{-nu}, E_0 = 1 - e^{-nu}, which is stable for nu > q.
// The weights are computed once per (axis, alpha) and reused for every line (Sec. 2.4, uniform
// grids).
#include <cmath>

namespace scx {

double moment(int q, double nu)
{
    if (nu <= 30.0) {
        double term = nu / (q + 1.0);
        double sum = term;
        for (int l = 2; l < 1000; ++l) {
            term *= nu / (double)(q + l);
            sum += term;
            if (term < 1e-18 * sum) break;
        }
        return std::exp(-nu) * sum;
    }
    double e = std::exp(-nu);
    double E = -std::expm1(-nu);
    for (int j = 1; j <= q; ++j) E = (j / nu) * E - e;
    return E;
}

// w[j] for nodes eta[0..m-1] (distinct integers), m <= 8.
void quad_weights(double nu, int m, const int *eta, double *w)
{
    double E[8];
    for (int q = 0; q < m; ++q) E[q] = moment(q, nu);
    for (int j = 0; j < m; ++j) {
        // coefficients of prod_{k != j} (eta - eta_k), highest degree m-1
        double poly[8] = {1.0, 0, 0, 0, 0, 0, 0, 0};
        int deg = 0;
        double den = 1.0;
        for (int k = 0; k < m; ++k) {
            if (k == j) continue;
            // multiply by (eta - eta_k)
            for (int q = deg + 1; q >= 1; --q) poly[q] = poly[q - 1] - eta[k] * poly[q];
            poly[0] = -eta[k] * poly[0];
            ++deg;
            den *= (double)(eta[j] - eta[k]);
        }
        double acc = 0.0;
        for (int q = 0; q <= deg; ++q) acc += poly[q] * E[q];
        w[j] = acc / den;
    }
}

}  // namespace scx
