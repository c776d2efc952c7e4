// dg_lgl.cpp -- host-side operator setup: Legendre-Gauss-Lobatto nodes and
// weights and the nodal differentiation matrix, in FP64, once per solver.
//
// Nodes (Sec. 2.1: the solutions of (1 - xi^2) P_N'(xi) = 0) are found with
// the fixed-point Newton iteration on x P_N(x) - P_{N-1}(x), whose zeros are
// exactly the LGL nodes including +-1 (it is proportional to (1 - x^2) P_N'):
//   x <- x - (x P_N - P_{N-1}) / ((N + 1) P_N),
// started from the Chebyshev-Gauss-Lobatto points. Weights are
// w_j = 2 / (N (N+1) P_N(xi_j)^2) and the differentiation matrix
// D_ij = h_j'(xi_i) of the Lagrange basis of eq. lagrange_pol has the closed form
//   D_ij = P_N(xi_i) / (P_N(xi_j) (xi_i - xi_j))  (i != j),
//   D_00 = -N(N+1)/4,  D_NN = N(N+1)/4,  D_ii = 0 otherwise.
#include <cmath>

#include "dg_host.hpp"

namespace dg {

static void legendre_pair(int n, double x, double &pn, double &pnm1)
{
    // P_n and P_{n-1} by the three-term recurrence
    double a = 1.0, b = x;   // P_0, P_1
    if (n == 0) { pn = 1.0; pnm1 = 0.0; return; }
    for (int k = 2; k <= n; ++k) {
        const double c = ((2.0 * k - 1.0) * x * b - (k - 1.0) * a) / k;
        a = b;
        b = c;
    }
    pn = b;
    pnm1 = a;
}

void lgl_operator(int N, double *xi, double *w, double *D)
{
    const int n1 = N + 1;
    double x[kMaxNP1], pn[kMaxNP1];
    for (int j = 0; j < n1; ++j) x[j] = -std::cos(M_PI * j / N);
    for (int it = 0; it < 200; ++it) {
        double dmax = 0.0;
        for (int j = 0; j < n1; ++j) {
            double p, pm;
            legendre_pair(N, x[j], p, pm);
            const double dx = (x[j] * p - pm) / ((N + 1.0) * p);
            x[j] -= dx;
            dmax = std::fmax(dmax, std::fabs(dx));
        }
        if (dmax < 1e-16) break;
    }
    x[0] = -1.0;
    x[N] = 1.0;
    for (int j = 1; j < N; ++j) {      // symmetric pairs
        const int k = N - j;
        if (j < k) {
            const double m = 0.5 * (x[k] - x[j]);
            x[j] = -m;
            x[k] = m;
        } else if (j == k) {
            x[j] = 0.0;
        }
    }
    for (int j = 0; j < n1; ++j) {
        double p, pm;
        legendre_pair(N, x[j], p, pm);
        pn[j] = p;
        xi[j] = x[j];
        w[j] = 2.0 / (N * (N + 1.0) * p * p);
    }
    for (int i = 0; i < n1; ++i)
        for (int j = 0; j < n1; ++j) {
            double v = 0.0;
            if (i != j) v = pn[i] / (pn[j] * (x[i] - x[j]));
            else if (i == 0) v = -0.25 * N * (N + 1.0);
            else if (i == N) v = 0.25 * N * (N + 1.0);
            D[i * n1 + j] = v;
        }
}

}  // namespace dg
