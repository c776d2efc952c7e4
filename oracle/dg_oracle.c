/*
 * dg_oracle.c -- plain, slow, obviously-correct CPU FP64 reference ("the
 * oracle") for the nodal discontinuous Galerkin (NDG) right-hand side and its
 * explicit Runge-Kutta time stepping, after Sporykhin & Homann, "Performance
 * of a high-order MPI-Kokkos accelerated fluid solver" (arXiv:2510.05254).
 *
 * TEST INFRASTRUCTURE ONLY. The tests, the smoke check and the benchmark's
 * CPU-baseline leg are the only code that may load this library. It shares no
 * source, header, table or helper with the GPU library, and the GPU library
 * never calls it.
 *
 * Everything here is double precision, round-to-nearest, built with
 * -ffp-contract=off and without fast-math. Loops are plain; OpenMP is used
 * only to split the outer element loop (and elementwise RK combinations)
 * across host cores so that full-size cases finish in reasonable time. No
 * blocking, fusion or reordering beyond what the definitions below state.
 *
 * Notation (paper Sec. 2.1): N = polynomial degree, N+1 Legendre-Gauss-Lobatto
 * (LGL) nodes xi_0..xi_N per direction; K_d elements along direction d on the
 * periodic unit interval/square/cube; dx_d = 1/K_d.
 *
 * State layout (shared with the tests): u[v][e][n], with
 *   e = ex + Kx*(ey + Ky*ez)   (element index, x fastest)
 *   n = i + (N+1)*(j + (N+1)*k) (node index inside the element, x fastest)
 * and v the conserved variable: advection (U); isothermal Euler
 * (rho, rho*u_1, .., rho*u_dim).
 *
 * Parity status of each function is listed in oracle/__init__.py; every
 * function here is pinned by a CPU test (see tests/test_oracle_*.py).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_MAXN 8
#define OR_MAXNP1 (OR_MAXN + 1)
#define OR_ADVECTION 0
#define OR_EULER 1

/* ------------------------------------------------------------------------ */
/* Threads                                                                  */
/* ------------------------------------------------------------------------ */

void or_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int or_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Legendre polynomials (Sec. 2.1, the P_N appearing in eq. lagrange_pol)   */
/* ------------------------------------------------------------------------ */

/* P_n(x) and P_n'(x) by Bonnet's recurrence
 *   (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1},
 * and the derivative recurrence P'_{k+1} = P'_{k-1} + (2k+1) P_k. */
static void legendre(int n, double x, double *p_out, double *dp_out)
{
    double pm1 = 1.0, p = x;        /* P_0, P_1 */
    double dpm1 = 0.0, dp = 1.0;    /* P_0', P_1' */
    if (n == 0) { *p_out = 1.0; *dp_out = 0.0; return; }
    for (int k = 1; k < n; ++k) {
        double pp1 = ((2.0 * k + 1.0) * x * p - k * pm1) / (k + 1.0);
        double dpp1 = dpm1 + (2.0 * k + 1.0) * p;
        pm1 = p; p = pp1;
        dpm1 = dp; dp = dpp1;
    }
    *p_out = p;
    *dp_out = dp;
}

/* ------------------------------------------------------------------------ */
/* LGL nodes and weights (Sec. 2.1: nodes solve (1 - xi^2) P_N'(xi) = 0;    */
/* weights of the (N+1)-point quadrature in eq. lag_coefs)                 */
/* ------------------------------------------------------------------------ */

/* Nodes: xi_0 = -1, xi_N = +1 and the N-1 roots of P_N' found by Newton's
 * method on g = P_N', with g' = P_N'' taken from Legendre's equation
 * (1 - x^2) P'' = 2 x P' - N(N+1) P. Starting guesses are the
 * Chebyshev-Gauss-Lobatto points -cos(pi j / N), which interlace the roots.
 * The result is sorted ascending and made exactly antisymmetric.
 * Weights: w_j = 2 / (N (N+1) P_N(xi_j)^2), the textbook LGL weight
 * (the paper relies on it through eq. lag_coefs but does not print it). */
int or_lgl(int N, double *xi, double *w)
{
    if (N < 1 || N > OR_MAXN || !xi || !w) return -1;
    xi[0] = -1.0;
    xi[N] = 1.0;
    for (int j = 1; j < N; ++j) {
        double x = -cos(M_PI * j / N);
        for (int it = 0; it < 100; ++it) {
            double p, dp;
            legendre(N, x, &p, &dp);
            double d2p = (2.0 * x * dp - N * (N + 1.0) * p) / (1.0 - x * x);
            double dx = dp / d2p;
            x -= dx;
            if (fabs(dx) <= 1e-17) break;
        }
        xi[j] = x;
    }
    /* sort ascending (insertion sort; N <= 8) */
    for (int a = 1; a <= N; ++a) {
        double t = xi[a];
        int b = a - 1;
        while (b >= 0 && xi[b] > t) { xi[b + 1] = xi[b]; --b; }
        xi[b + 1] = t;
    }
    /* exact antisymmetry xi_{N-j} = -xi_j */
    for (int j = 0; j <= N / 2; ++j) {
        double s = 0.5 * (xi[N - j] - xi[j]);
        xi[j] = -s;
        xi[N - j] = s;
    }
    if (N % 2 == 0) xi[N / 2] = 0.0;
    for (int j = 0; j <= N; ++j) {
        double p, dp;
        legendre(N, xi[j], &p, &dp);
        w[j] = 2.0 / (N * (N + 1.0) * p * p);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Differentiation matrix (Sec. 2.1, the dh_l/dx after integration by parts) */
/* ------------------------------------------------------------------------ */

/* D[i*(N+1) + l] = h_l'(xi_i), where h_l is the Lagrange cardinal polynomial
 * of eq. lagrange_pol (h_l(xi_m) = delta_lm, eq. ortho_at_roots). Written
 * out from the product form h_l(x) = prod_{m != l} (x - xi_m)/(xi_l - xi_m):
 *   i != l:  h_l'(xi_i) = prod_{m != l, i} (xi_i - xi_m) / prod_{m != l} (xi_l - xi_m)
 *   i == l:  h_l'(xi_l) = sum_{m != l} 1 / (xi_l - xi_m).                   */
int or_dmat(int N, const double *xi, double *D)
{
    if (N < 1 || N > OR_MAXN || !xi || !D) return -1;
    const int n1 = N + 1;
    for (int i = 0; i < n1; ++i) {
        for (int l = 0; l < n1; ++l) {
            double v;
            if (i == l) {
                v = 0.0;
                for (int m = 0; m < n1; ++m)
                    if (m != l) v += 1.0 / (xi[l] - xi[m]);
            } else {
                double num = 1.0, den = 1.0;
                for (int m = 0; m < n1; ++m) {
                    if (m == l) continue;
                    den *= (xi[l] - xi[m]);
                    if (m != i) num *= (xi[i] - xi[m]);
                }
                v = num / den;
            }
            D[i * n1 + l] = v;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Mesh (Sec. 2.1 element partition and eq. transformation)                 */
/* ------------------------------------------------------------------------ */

/* 1-D node coordinates along one axis: x[e*(N+1) + i] for element e of K on
 * the periodic unit interval, x = x_{e-1/2} + (dx/2)(xi_i + 1) with
 * x_{e-1/2} = e*dx, dx = 1/K. (The paper's map omits the element offset.) */
int or_axis_coords(int N, int64_t K, double *x)
{
    double xi[OR_MAXNP1], w[OR_MAXNP1];
    if (K < 1 || !x || or_lgl(N, xi, w)) return -1;
    const double dx = 1.0 / (double)K;
    for (int64_t e = 0; e < K; ++e)
        for (int i = 0; i <= N; ++i)
            x[e * (N + 1) + i] = (double)e * dx + 0.5 * dx * (xi[i] + 1.0);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Physical fluxes (eq. advection1d, eq. advection2d, eq. eulerIso2d)       */
/* ------------------------------------------------------------------------ */

static int nvar_of(int dim, int eq) { return eq == OR_ADVECTION ? 1 : 1 + dim; }

/* Flux along direction d of the state U (nvar values) into F.
 * Advection: F_d = a_d U.
 * Isothermal Euler, U = (rho, m_1..m_dim), u_k = m_k / rho:
 *   F_d = (m_d, m_d u_1 + delta_{d1} rho c^2, ..., m_d u_dim + delta_{d,dim} rho c^2).
 * (The 1-D Euler system is the 2-D one restricted to (rho, rho u_x).) */
static void phys_flux(int dim, int d, int eq, const double *par,
                      const double *U, double *F)
{
    if (eq == OR_ADVECTION) {
        F[0] = par[d] * U[0];
        return;
    }
    const double c = par[0];
    const double rho = U[0];
    F[0] = U[1 + d];
    for (int k = 0; k < dim; ++k) {
        double uk = U[1 + k] / rho;
        F[1 + k] = U[1 + d] * uk;
        if (k == d) F[1 + k] = F[1 + k] + rho * c * c;
    }
}

/* Largest absolute eigenvalue of the flux Jacobian dF_d/dU at U (the
 * alpha_max of eq. LF): |a_d| for advection; |u_d| + c for isothermal Euler,
 * whose eigenvalues along d are u_d - c, u_d (multiplicity dim-1), u_d + c. */
static double max_speed(int dim, int d, int eq, const double *par, const double *U)
{
    (void)dim;
    if (eq == OR_ADVECTION) return fabs(par[d]);
    return fabs(U[1 + d] / U[0]) + par[0];
}

/* Lax-Friedrichs (Rusanov) numerical flux, eq. LF, at one face point whose
 * left/lower trace is UL (the paper's U^-) and right/upper trace is UR (U^+):
 *   Fhat = 1/2 [ F(UL) + F(UR) - alpha (UR - UL) ],
 * with alpha the larger of the two traces' maximal wave speeds. */
static void num_flux(int dim, int d, int eq, const double *par,
                     const double *UL, const double *UR, double *Fh)
{
    double FL[4], FR[4];
    const int nv = nvar_of(dim, eq);
    phys_flux(dim, d, eq, par, UL, FL);
    phys_flux(dim, d, eq, par, UR, FR);
    double aL = max_speed(dim, d, eq, par, UL);
    double aR = max_speed(dim, d, eq, par, UR);
    double alpha = aL > aR ? aL : aR;
    for (int v = 0; v < nv; ++v)
        Fh[v] = 0.5 * ((FL[v] + FR[v]) - alpha * (UR[v] - UL[v]));
}

/* Exported single-point versions for the tests. */
int or_flux(int dim, int d, int eq, const double *par, const double *U, double *F)
{
    if (dim < 1 || dim > 3 || d < 0 || d >= dim || (eq != 0 && eq != 1)) return -1;
    phys_flux(dim, d, eq, par, U, F);
    return 0;
}

int or_numflux(int dim, int d, int eq, const double *par,
               const double *UL, const double *UR, double *Fh)
{
    if (dim < 1 || dim > 3 || d < 0 || d >= dim || (eq != 0 && eq != 1)) return -1;
    num_flux(dim, d, eq, par, UL, UR, Fh);
    return 0;
}

double or_max_speed(int dim, int d, int eq, const double *par, const double *U)
{
    return max_speed(dim, d, eq, par, U);
}

/* ------------------------------------------------------------------------ */
/* Right-hand side of the semi-discrete system (Sec. 2.1, the evolution     */
/* equation for the nodal coefficients, tensor-product in dim dimensions)  */
/* ------------------------------------------------------------------------ */

typedef struct {
    int dim, N, eq, nvar, n1, np;
    int64_t K[3], E;
    double par[3];
    double xi[OR_MAXNP1], w[OR_MAXNP1], D[OR_MAXNP1 * OR_MAXNP1];
} or_mesh;

static int mesh_init(or_mesh *m, int dim, int N, const int64_t *K, int eq,
                     const double *par)
{
    if (dim < 1 || dim > 3 || N < 1 || N > OR_MAXN || !K || !par) return -1;
    if (eq != OR_ADVECTION && eq != OR_EULER) return -1;
    memset(m, 0, sizeof(*m));
    m->dim = dim; m->N = N; m->eq = eq;
    m->nvar = nvar_of(dim, eq);
    m->n1 = N + 1;
    m->np = 1;
    for (int d = 0; d < dim; ++d) m->np *= m->n1;
    m->E = 1;
    for (int d = 0; d < 3; ++d) {
        m->K[d] = d < dim ? K[d] : 1;
        if (m->K[d] < 1) return -1;
        m->E *= m->K[d];
    }
    if (eq == OR_ADVECTION) for (int d = 0; d < dim; ++d) m->par[d] = par[d];
    else m->par[0] = par[0];
    if (or_lgl(N, m->xi, m->w)) return -1;
    if (or_dmat(N, m->xi, m->D)) return -1;
    return 0;
}

/* Element multi-index <-> linear index. */
static void elem_coords(const or_mesh *m, int64_t e, int64_t c[3])
{
    c[0] = e % m->K[0];
    c[1] = (e / m->K[0]) % m->K[1];
    c[2] = e / (m->K[0] * m->K[1]);
}

static int64_t elem_index(const or_mesh *m, const int64_t c[3])
{
    return c[0] + m->K[0] * (c[1] + m->K[1] * c[2]);
}

/* Periodic neighbour of element e along d: step = +1 (upper) or -1 (lower). */
static int64_t neighbour(const or_mesh *m, int64_t e, int d, int step)
{
    int64_t c[3];
    elem_coords(m, e, c);
    c[d] = (c[d] + step + m->K[d]) % m->K[d];
    return elem_index(m, c);
}

static void node_coords(const or_mesh *m, int n, int ijk[3])
{
    ijk[0] = n % m->n1;
    ijk[1] = (n / m->n1) % m->n1;
    ijk[2] = n / (m->n1 * m->n1);
    for (int d = m->dim; d < 3; ++d) ijk[d] = 0;
}

static int node_index(const or_mesh *m, const int ijk[3])
{
    return ijk[0] + m->n1 * (ijk[1] + m->n1 * ijk[2]);
}

static void gather(const or_mesh *m, const double *U, int64_t e, int n, double *out)
{
    const int64_t stride = m->E * m->np;
    for (int v = 0; v < m->nvar; ++v) out[v] = U[v * stride + e * m->np + n];
}

/* R = dU/dt for the whole mesh.
 *
 * form 0 (weak form, normative; Sec. 2.1 evolution equation): for element e,
 * node l = (l_1..l_dim) and each direction d, with the 1-D sums running over
 * the nodes i of the line through l along d,
 *   R_l += (2/dx_d) (1/w_{l_d}) [ sum_i w_i D_{i,l_d} F_d(U_i)
 *                                 - delta_{l_d,N} Fhat_{d,upper}
 *                                 + delta_{l_d,0} Fhat_{d,lower} ].
 * The sum is the LGL quadrature of the volume integral of F dh_l/dx, the
 * bracket terms are [Fhat h_l] at the element's two borders along d, and the
 * factor 1/((dx/2) w_l) inverts the lumped (diagonal) mass of eq. lag_coefs.
 * Fhat_{d,upper} at a node on the upper face uses UL = this element's trace,
 * UR = the upper neighbour's trace at the matching node (periodic wrap);
 * Fhat_{d,lower} uses UL = the lower neighbour's trace, UR = this element's.
 *
 * form 1 (strong form; used only to check that the two agree): the same
 * quantity after one more integration by parts,
 *   R_l += (2/dx_d) [ - sum_i D_{l_d,i} F_d(U_i)
 *                     + delta_{l_d,N} (1/w_N) (F_d(U_l) - Fhat_{d,upper})
 *                     + delta_{l_d,0} (1/w_0) (Fhat_{d,lower} - F_d(U_l)) ]. */
static void rhs_mesh(const or_mesh *m, int form, const double *U, double *R)
{
    const int nv = m->nvar, n1 = m->n1, np = m->np, dim = m->dim, N = m->N;
    const int64_t stride = m->E * np;

#pragma omp parallel
    {
        /* nodal fluxes of the current element, Fn[(d*nv + v)*np + n] */
        double *Fn = (double *)malloc(sizeof(double) * 3 * 4 * np);
        double *Rl = (double *)malloc(sizeof(double) * 4 * np);
#pragma omp for schedule(static)
        for (int64_t e = 0; e < m->E; ++e) {
            double Un[4], Fd[4];
            for (int n = 0; n < np; ++n) {
                gather(m, U, e, n, Un);
                for (int d = 0; d < dim; ++d) {
                    phys_flux(dim, d, m->eq, m->par, Un, Fd);
                    for (int v = 0; v < nv; ++v) Fn[(d * nv + v) * np + n] = Fd[v];
                }
            }
            for (int i = 0; i < nv * np; ++i) Rl[i] = 0.0;

            for (int d = 0; d < dim; ++d) {
                const double jac = 2.0 * (double)m->K[d]; /* 2/dx_d */
                for (int l = 0; l < np; ++l) {
                    int ijk[3];
                    node_coords(m, l, ijk);
                    const int ld = ijk[d];
                    double acc[4];
                    for (int v = 0; v < nv; ++v) acc[v] = 0.0;
                    /* volume term along the line through l */
                    for (int i = 0; i < n1; ++i) {
                        int q[3] = {ijk[0], ijk[1], ijk[2]};
                        q[d] = i;
                        const int ni = node_index(m, q);
                        for (int v = 0; v < nv; ++v) {
                            if (form == 0)
                                acc[v] += m->w[i] * m->D[i * n1 + ld] * Fn[(d * nv + v) * np + ni];
                            else
                                acc[v] += m->D[ld * n1 + i] * Fn[(d * nv + v) * np + ni];
                        }
                    }
                    /* surface terms at the two borders along d */
                    double Fh[4], Uo[4], Unb[4];
                    double bnd[4] = {0.0, 0.0, 0.0, 0.0};
                    if (ld == N) {
                        int q[3] = {ijk[0], ijk[1], ijk[2]};
                        q[d] = 0;
                        gather(m, U, e, l, Uo);
                        gather(m, U, neighbour(m, e, d, +1), node_index(m, q), Unb);
                        num_flux(dim, d, m->eq, m->par, Uo, Unb, Fh);
                        for (int v = 0; v < nv; ++v) {
                            if (form == 0) bnd[v] -= Fh[v];
                            else bnd[v] += (1.0 / m->w[N]) * (Fn[(d * nv + v) * np + l] - Fh[v]);
                        }
                    }
                    if (ld == 0) {
                        int q[3] = {ijk[0], ijk[1], ijk[2]};
                        q[d] = N;
                        gather(m, U, e, l, Uo);
                        gather(m, U, neighbour(m, e, d, -1), node_index(m, q), Unb);
                        num_flux(dim, d, m->eq, m->par, Unb, Uo, Fh);
                        for (int v = 0; v < nv; ++v) {
                            if (form == 0) bnd[v] += Fh[v];
                            else bnd[v] += (1.0 / m->w[0]) * (Fh[v] - Fn[(d * nv + v) * np + l]);
                        }
                    }
                    for (int v = 0; v < nv; ++v) {
                        double r;
                        if (form == 0) r = jac * (1.0 / m->w[ld]) * (acc[v] + bnd[v]);
                        else r = jac * (bnd[v] - acc[v]);
                        Rl[v * np + l] += r;
                    }
                }
            }
            for (int v = 0; v < nv; ++v)
                for (int n = 0; n < np; ++n) R[v * stride + e * np + n] = Rl[v * np + n];
        }
        free(Fn);
        free(Rl);
    }
}

int or_rhs(int dim, int N, const int64_t *K, int eq, const double *par, int form,
           const double *U, double *R)
{
    or_mesh m;
    if (mesh_init(&m, dim, N, K, eq, par) || !U || !R || (form != 0 && form != 1)) return -1;
    rhs_mesh(&m, form, U, R);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Explicit Runge-Kutta schemes (Sec. 2.3, eqs. RK3, RK4, RK6)              */
/* ------------------------------------------------------------------------ */

/* Butcher form with every stage increment stored: k_s = dt F(Y_s),
 *   Y_1 = U,  Y_s = U + (sum_{j<s} num[s][j] k_j) / den[s],
 *   U_next = U + (sum_j bnum[j] k_j) / bden.
 * Numerators and denominators are kept as the paper groups them.
 *
 * RK4 (eq. RK4): the classical scheme as printed.
 * RK6 (eq. RK6): Luther's seven-stage scheme as printed.
 * RK3 (eq. RK3): as printed, the third line applies dt to k_1 (already a
 *   multiple of dt) and fails first-order consistency; the coefficients
 *   1/3, 2/3, 1/4, 3/4 are those of Heun's third-order method, which is the
 *   reading used: Y_2 = U + k_1/3, Y_3 = U + 2 k_2/3, U_next = U + (k_1 + 3 k_3)/4. */
typedef struct {
    int stages;
    double num[7][7], den[7];
    double bnum[7], bden;
} or_tableau;

static int tableau(int rk, or_tableau *t)
{
    memset(t, 0, sizeof(*t));
    const double s21 = sqrt(21.0);
    if (rk == 3) {
        t->stages = 3;
        t->den[1] = 3.0; t->num[1][0] = 1.0;
        t->den[2] = 3.0; t->num[2][1] = 2.0;
        t->bden = 4.0; t->bnum[0] = 1.0; t->bnum[2] = 3.0;
    } else if (rk == 4) {
        t->stages = 4;
        t->den[1] = 2.0; t->num[1][0] = 1.0;
        t->den[2] = 2.0; t->num[2][1] = 1.0;
        t->den[3] = 1.0; t->num[3][2] = 1.0;
        t->bden = 6.0;
        t->bnum[0] = 1.0; t->bnum[1] = 2.0; t->bnum[2] = 2.0; t->bnum[3] = 1.0;
    } else if (rk == 6) {
        t->stages = 7;
        t->den[1] = 1.0; t->num[1][0] = 1.0;
        t->den[2] = 8.0; t->num[2][0] = 3.0; t->num[2][1] = 1.0;
        t->den[3] = 27.0; t->num[3][0] = 8.0; t->num[3][1] = 2.0; t->num[3][2] = 8.0;
        t->den[4] = 392.0;
        t->num[4][0] = 3.0 * (3.0 * s21 - 7.0);
        t->num[4][1] = -8.0 * (7.0 - s21);
        t->num[4][2] = 48.0 * (7.0 - s21);
        t->num[4][3] = -3.0 * (21.0 - s21);
        t->den[5] = 1960.0;
        t->num[5][0] = -5.0 * (231.0 + 51.0 * s21);
        t->num[5][1] = -40.0 * (7.0 + s21);
        t->num[5][2] = -320.0 * s21;
        t->num[5][3] = 3.0 * (21.0 + 121.0 * s21);
        t->num[5][4] = 392.0 * (6.0 + s21);
        t->den[6] = 180.0;
        t->num[6][0] = 15.0 * (22.0 + 7.0 * s21);
        t->num[6][1] = 120.0;
        t->num[6][2] = 40.0 * (7.0 * s21 - 5.0);
        t->num[6][3] = -63.0 * (3.0 * s21 - 2.0);
        t->num[6][4] = -14.0 * (49.0 + 9.0 * s21);
        t->num[6][5] = 70.0 * (7.0 - s21);
        t->bden = 180.0;
        t->bnum[0] = 9.0; t->bnum[2] = 64.0; t->bnum[4] = 49.0; t->bnum[5] = 49.0;
        t->bnum[6] = 9.0;
    } else {
        return -1;
    }
    return 0;
}

/* Butcher coefficients a[s][j] = num[s][j]/den[s], b[j] = bnum[j]/bden,
 * exported so the tests can check the order conditions. */
int or_rk_tableau(int rk, int *stages, double *a /*7x7*/, double *b /*7*/)
{
    or_tableau t;
    if (tableau(rk, &t) || !stages || !a || !b) return -1;
    *stages = t.stages;
    for (int s = 0; s < 7; ++s) {
        for (int j = 0; j < 7; ++j) a[s * 7 + j] = s > 0 && t.den[s] != 0.0 ? t.num[s][j] / t.den[s] : 0.0;
        b[s] = t.bnum[s] / t.bden;
    }
    return 0;
}

typedef void (*or_rhs_fn)(void *ctx, const double *Y, double *R);

/* nsteps steps of scheme rk with step dt on the n-vector U (in place),
 * F evaluated by f(ctx, Y, R). Work arrays are allocated here. */
static int rk_integrate(int rk, double dt, int64_t nsteps, int64_t n, double *U,
                        or_rhs_fn f, void *ctx)
{
    or_tableau t;
    if (tableau(rk, &t)) return -1;
    const int S = t.stages;
    double *Y = (double *)malloc(sizeof(double) * (size_t)n);
    double *k = (double *)malloc(sizeof(double) * (size_t)n * (size_t)S);
    if (!Y || !k) { free(Y); free(k); return -2; }
    for (int64_t step = 0; step < nsteps; ++step) {
        for (int s = 0; s < S; ++s) {
            const double *Ys = U;
            if (s > 0) {
#pragma omp parallel for schedule(static)
                for (int64_t i = 0; i < n; ++i) {
                    double sum = 0.0;
                    for (int j = 0; j < s; ++j) sum += t.num[s][j] * k[(int64_t)j * n + i];
                    Y[i] = U[i] + sum / t.den[s];
                }
                Ys = Y;
            }
            double *ks = k + (int64_t)s * n;
            f(ctx, Ys, ks);
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < n; ++i) ks[i] = dt * ks[i];
        }
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            double sum = 0.0;
            for (int j = 0; j < S; ++j) sum += t.bnum[j] * k[(int64_t)j * n + i];
            U[i] = U[i] + sum / t.bden;
        }
    }
    free(Y);
    free(k);
    return 0;
}

static void mesh_rhs_cb(void *ctx, const double *Y, double *R)
{
    rhs_mesh((const or_mesh *)ctx, 0, Y, R);
}

/* nsteps RK steps of the NDG system (weak-form RHS) on U, in place. */
int or_step(int dim, int N, const int64_t *K, int eq, const double *par, int rk,
            double dt, int64_t nsteps, double *U)
{
    or_mesh m;
    if (mesh_init(&m, dim, N, K, eq, par) || !U || nsteps < 0) return -1;
    const int64_t n = (int64_t)m.nvar * m.E * m.np;
    return rk_integrate(rk, dt, nsteps, n, U, mesh_rhs_cb, &m);
}

/* Scalar test ODEs stepped by the same RK routine:
 * kind 0: y' = lam * y;  kind 1: y' = y (1 - y) (logistic). */
typedef struct { int kind; double lam; } ode_ctx;

static void ode_cb(void *ctx, const double *Y, double *R)
{
    const ode_ctx *c = (const ode_ctx *)ctx;
    R[0] = c->kind == 0 ? c->lam * Y[0] : Y[0] * (1.0 - Y[0]);
}

int or_ode_solve(int rk, int kind, double lam, double y0, double dt, int64_t nsteps,
                 double *y_out)
{
    ode_ctx c = {kind, lam};
    double y = y0;
    int rc = rk_integrate(rk, dt, nsteps, 1, &y, ode_cb, &c);
    *y_out = y;
    return rc;
}

/* ------------------------------------------------------------------------ */
/* L2 error and mass (Sec. 3.1 L2 norm; integrals by the nodal LGL rule)    */
/* ------------------------------------------------------------------------ */

/* Quadrature weight of node n: prod_d (dx_d/2) w_{n_d}. */
static double node_weight(const or_mesh *m, int n)
{
    int ijk[3];
    node_coords(m, n, ijk);
    double q = 1.0;
    for (int d = 0; d < m->dim; ++d) q *= (0.5 / (double)m->K[d]) * m->w[ijk[d]];
    return q;
}

/* sq_err[v] = integral of (U_v - Uref_v)^2 and sq_ref[v] = integral of
 * Uref_v^2 over the periodic domain. Element partial sums, then a serial sum
 * over elements in index order. */
int or_l2(int dim, int N, const int64_t *K, int eq, const double *U,
          const double *Uref, double *sq_err, double *sq_ref)
{
    double par[3] = {1.0, 1.0, 1.0};
    or_mesh m;
    if (mesh_init(&m, dim, N, K, eq, par) || !U || !Uref) return -1;
    const int64_t stride = m.E * m.np;
    for (int v = 0; v < m.nvar; ++v) {
        double se = 0.0, sr = 0.0;
        for (int64_t e = 0; e < m.E; ++e) {
            double pe = 0.0, pr = 0.0;
            for (int n = 0; n < m.np; ++n) {
                const double q = node_weight(&m, n);
                const double diff = U[v * stride + e * m.np + n] - Uref[v * stride + e * m.np + n];
                const double ref = Uref[v * stride + e * m.np + n];
                pe += q * diff * diff;
                pr += q * ref * ref;
            }
            se += pe;
            sr += pr;
        }
        sq_err[v] = se;
        sq_ref[v] = sr;
    }
    return 0;
}

/* mass[v] = integral of U_v over the periodic domain. */
int or_mass(int dim, int N, const int64_t *K, int eq, const double *U, double *mass)
{
    double par[3] = {1.0, 1.0, 1.0};
    or_mesh m;
    if (mesh_init(&m, dim, N, K, eq, par) || !U || !mass) return -1;
    const int64_t stride = m.E * m.np;
    for (int v = 0; v < m.nvar; ++v) {
        double s = 0.0;
        for (int64_t e = 0; e < m.E; ++e) {
            double pe = 0.0;
            for (int n = 0; n < m.np; ++n) pe += node_weight(&m, n) * U[v * stride + e * m.np + n];
            s += pe;
        }
        mass[v] = s;
    }
    return 0;
}
