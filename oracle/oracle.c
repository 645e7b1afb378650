/*
 * oracle.c -- plain, slow FP64 CPU oracle for the lumped DG S_N transport
 * sweep and the Second Moment (SM) thermal radiative transfer step of
 * Olivier, Warsa & Park, "Efficient, Nonlinear Second Moment Methods for
 * Multigroup Thermal Radiative Transfer".
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may load this
 * library: only the test-suite, the smoke check and the benchmark's CPU
 * baseline leg use it.  It shares no code, header, table or helper with
 * the GPU library.
 *
 * Everything is written from the paper's definitions in the most direct
 * form: local matrices assembled term by term from the weak forms with
 * the trapezoid (2-point Gauss-Lobatto) lumping, solved by Gaussian
 * elimination with partial pivoting; moments and closures summed
 * direction by direction; the low-order operator applied from an
 * explicitly assembled sparse divergence matrix.  Single threaded, except
 * that the sweep may run its independent (direction, group) pairs on
 * several OpenMP threads (the results do not depend on the thread count).
 *
 * Conventions.
 *   cell c = i + nx*j; local node l = lx + 2*ly (1D: l = lx);
 *   node n = npc*c + l with npc = 2^dim.
 *   Angular arrays are [d][g][node].
 *   Boundary face nodes (general inflow arrays): 1D: x- = 0, x+ = 1.
 *   2D: x- side 2*j+ly, x+ side 2*ny+2*j+ly, y- side 4*ny+2*i+lx,
 *   y+ side 4*ny+2*nx+2*i+lx.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846264338327950288
#endif

#define ORC_OK 0
#define ORC_E_NONPHYSICAL 5
#define ORC_E_NOT_CONVERGED 4

typedef struct {
    int dim, nx, ny;
    const double *xe, *ye;
    int nang;
    const double *om; /* [nang][3] */
    const double *w;  /* [nang] */
    int G;
    const double *nu; /* [G+1] stated group bounds */
    double a, c;
} orc_geom;

typedef struct {
    const int *region;     /* [ncell] */
    int model;             /* 0: sigma0[r*G+g]; 1: sigma0[r]/(nubar^3 T^3) clipped */
    const double *sigma0;
    double clip_lo, clip_hi;
    const double *cv;      /* [nregion] */
} orc_mat;

typedef struct {
    int kind[4];           /* 0 vacuum, 1 Planck at T_bdr, 2 explicit isotropic per group, 3 reflective */
    double T_bdr[4];
    const double *inflow_g[4];
} orc_bc;

typedef struct {
    double eps_outer, eps_inner, cg_rtol, elim_rtol;
    int max_outer, max_inner, max_cg, max_elim;
    int scheme;            /* 0 consistent SM, 1 independent SM, 2 unaccelerated */
    int lo_time_edge;      /* 0: E*,F* from HO sums (default), 1: from LO solution */
    int fixup;             /* 1: zero-and-scale negative-flux fixup in the sweep */
    double T_floor;        /* > 0: temperature floor of the energy balance */
} orc_opts;

typedef struct {
    int outer, inner_total, cg_total, elim_max, hit_max;
} orc_stats;

/* ------------------------------------------------------------------------ */
/* small helpers                                                            */
/* ------------------------------------------------------------------------ */

static int ncell(const orc_geom *g) { return g->nx * (g->dim == 2 ? g->ny : 1); }
static int npc(const orc_geom *g) { return g->dim == 2 ? 4 : 2; }
static int nnode(const orc_geom *g) { return ncell(g) * npc(g); }
static double hx_of(const orc_geom *g, int i) { return g->xe[i + 1] - g->xe[i]; }
static double hy_of(const orc_geom *g, int j) { return g->dim == 2 ? g->ye[j + 1] - g->ye[j] : 1.0; }

/* lumped volume weight of every node of cell (i,j): |K| / 2^dim */
static double vol_weight(const orc_geom *g, int i, int j)
{
    return hx_of(g, i) * hy_of(g, j) / (double)npc(g);
}

/* Derivative along axis `ax` of the nodal basis function of local node l,
 * evaluated at local node m.  Q1 (1D: P1) Lagrange basis on the vertices:
 *   phi_l(x,y) = L_lx(x) L_ly(y), L_0(s) = (s1 - s)/h, L_1(s) = (s - s0)/h. */
static double dbasis(const orc_geom *g, int i, int j, int l, int m, int ax)
{
    int lx = l & 1, ly = l >> 1, mx = m & 1, my = m >> 1;
    double hx = hx_of(g, i), hy = hy_of(g, j);
    double dLx = (lx ? 1.0 : -1.0) / hx;
    double dLy = (ly ? 1.0 : -1.0) / hy;
    double Lx_at_m = (lx == mx) ? 1.0 : 0.0;
    double Ly_at_m = (ly == my) ? 1.0 : 0.0;
    if (g->dim == 1) return ax == 0 ? dLx : 0.0;
    return ax == 0 ? dLx * Ly_at_m : Lx_at_m * dLy;
}

/* Face of cell (i,j) on axis ax, side sd (0: lower, 1: upper) contains local
 * node l iff the node's coordinate index along ax equals sd. */
static int node_on_face(int l, int ax, int sd) { return ((ax == 0 ? (l & 1) : (l >> 1)) == sd); }

/* lumped face weight per face node: |f| / 2^(dim-1) */
static double face_weight(const orc_geom *g, int i, int j, int ax)
{
    if (g->dim == 1) return 1.0;
    return ax == 0 ? 0.5 * hy_of(g, j) : 0.5 * hx_of(g, i);
}

/* neighbour across face (ax, sd); returns -1 on the domain boundary */
static int neighbour(const orc_geom *g, int i, int j, int ax, int sd)
{
    int ni = i, nj = j;
    if (ax == 0) ni += sd ? 1 : -1; else nj += sd ? 1 : -1;
    if (ni < 0 || ni >= g->nx) return -1;
    if (g->dim == 2 && (nj < 0 || nj >= g->ny)) return -1;
    if (g->dim == 1 && nj != 0) return -1;
    return ni + g->nx * nj;
}

/* local node coincident with l across the face on axis ax */
static int mirror(int l, int ax) { return ax == 0 ? (l ^ 1) : (l ^ 2); }

/* boundary face-node index (see header) */
static int bnode_index(const orc_geom *g, int i, int j, int ax, int sd, int l)
{
    if (g->dim == 1) return sd;
    if (ax == 0) return (sd ? 2 * g->ny : 0) + 2 * j + (l >> 1);
    return 4 * g->ny + (sd ? 2 * g->nx : 0) + 2 * i + (l & 1);
}

static int nbnode(const orc_geom *g) { return g->dim == 1 ? 2 : 4 * (g->nx + g->ny); }

/* Omega . e_ax */
static double om_ax(const orc_geom *g, int d, int ax) { return g->om[3 * d + ax]; }

/* alpha_n = sum_d w_d |Omega_d . n| / sum_d w_d  (Eq. alpha) */
static double alpha_axis(const orc_geom *g, int ax)
{
    double s = 0.0, sw = 0.0;
    for (int d = 0; d < g->nang; ++d) { s += g->w[d] * fabs(om_ax(g, d, ax)); sw += g->w[d]; }
    return s / sw;
}

/* Dense Gaussian elimination with partial pivoting, n <= 8.  A is
 * overwritten; x receives the solution.  Returns 0 on success. */
static int lu_solve(int n, double *A, double *b, double *x)
{
    for (int k = 0; k < n; ++k) {
        int p = k;
        for (int r = k + 1; r < n; ++r) if (fabs(A[r * n + k]) > fabs(A[p * n + k])) p = r;
        if (A[p * n + k] == 0.0) return -1;
        if (p != k) {
            for (int c = 0; c < n; ++c) { double t = A[k * n + c]; A[k * n + c] = A[p * n + c]; A[p * n + c] = t; }
            double t = b[k]; b[k] = b[p]; b[p] = t;
        }
        for (int r = k + 1; r < n; ++r) {
            double f = A[r * n + k] / A[k * n + k];
            for (int c = k; c < n; ++c) A[r * n + c] -= f * A[k * n + c];
            b[r] -= f * b[k];
        }
    }
    for (int k = n - 1; k >= 0; --k) {
        double s = b[k];
        for (int c = k + 1; c < n; ++c) s -= A[k * n + c] * x[c];
        x[k] = s / A[k * n + k];
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Spectra: normalised Planck b_g(T) and Rosseland r_g(T) (Sec. 2, Eqs.     */
/* planck/black_body and the Rosseland fraction).  Integrated here by       */
/* adaptive Gauss-Kronrod (7,15) in FP64 -- deliberately not the series     */
/* method the paper cites.  The first group's lower bound is taken as 0 and */
/* the last group's upper bound as infinity, so that sum_g b_g = 1.         */
/* ------------------------------------------------------------------------ */

static double planck_density(double x)
{
    if (x <= 0.0) return 0.0;
    if (x > 700.0) return 0.0;
    return 15.0 / pow(M_PI, 4) * x * x * x / expm1(x);
}

static double rosseland_density(double x)
{
    if (x <= 0.0) return 0.0;
    if (x > 700.0) return 0.0;
    double em = -expm1(-x);          /* 1 - e^{-x} */
    return 15.0 / (4.0 * pow(M_PI, 4)) * pow(x, 4) * exp(-x) / (em * em);
}

static const double gk_x[8] = {0.991455371120812639206854697526329, 0.949107912342758524526189684047851,
                               0.864864423359769072789712788640926, 0.741531185599394439863864773280788,
                               0.586087235467691130294144845693013, 0.405845151377397166906606412076961,
                               0.207784955007898467600689403773245, 0.000000000000000000000000000000000};
static const double gk_wk[8] = {0.022935322010529224963732008058970, 0.063092092629978553290700663189204,
                                0.104790010322250183839876322541518, 0.140653259715525918745189590510238,
                                0.169004726639267902826583426598550, 0.190350578064785409913256402421014,
                                0.204432940075298892414161999234649, 0.209482141084727828012999174891714};

static double gk15(double (*f)(double), double a, double b)
{
    double c = 0.5 * (a + b), h = 0.5 * (b - a);
    double rk = f(c) * gk_wk[7];
    for (int k = 0; k < 7; ++k) rk += gk_wk[k] * (f(c - h * gk_x[k]) + f(c + h * gk_x[k]));
    return rk * h;
}

/* Integral of a spectral density over [lo, hi] by composite Gauss-Kronrod 15
 * on a fixed panel grid (width 1/4 on [0, 64], width 2 on [64, 750]); the
 * densities are analytic and negligible (< 1e-250) beyond x = 750, so this
 * is accurate to rounding.  Bounded work: no adaptive recursion. */
static double integrate_density(double (*f)(double), double lo, double hi)
{
    if (hi > 750.0) hi = 750.0;
    if (lo < 0.0) lo = 0.0;
    if (hi <= lo) return 0.0;
    double s = 0.0;
    for (int k = 0; k < 256 + 343; ++k) {
        double a = k < 256 ? 0.25 * k : 64.0 + 2.0 * (k - 256);
        double b = k < 256 ? a + 0.25 : a + 2.0;
        if (b <= lo) continue;
        if (a >= hi) break;
        double x0 = a > lo ? a : lo, x1 = b < hi ? b : hi;
        if (x1 > x0) s += gk15(f, x0, x1);
    }
    return s;
}

/* b_g(T), r_g(T) for all groups at scalar T > 0 */
void orc_spectra(int G, const double *nu, double T, double *b, double *r)
{
    if (G == 1) { b[0] = 1.0; r[0] = 1.0; return; }   /* one group spans [0, inf) */
    for (int g = 0; g < G; ++g) {
        double lo = (g == 0) ? 0.0 : nu[g] / T;
        double hi = (g == G - 1) ? 1e300 : nu[g + 1] / T;
        b[g] = integrate_density(planck_density, lo, hi);
        r[g] = integrate_density(rosseland_density, lo, hi);
    }
}

/* ------------------------------------------------------------------------ */
/* Opacity: sigma_g per cell from the cell-average temperature (Sec. 3).    */
/* ------------------------------------------------------------------------ */

void orc_opacity(const orc_geom *g, const orc_mat *m, const double *T_nodes, double *sig)
{
    int nc = ncell(g), np = npc(g), G = g->G;
    for (int c = 0; c < nc; ++c) {
        double Tc = 0.0;
        for (int l = 0; l < np; ++l) Tc += T_nodes[np * c + l];
        Tc /= np;
        int r = m->region[c];
        for (int k = 0; k < G; ++k) {
            double s;
            if (m->model == 0) s = m->sigma0[r * G + k];
            else {
                double nubar = sqrt(g->nu[k] * g->nu[k + 1]);
                s = m->sigma0[r] / (pow(nubar, 3) * pow(Tc, 3));
                if (s < m->clip_lo) s = m->clip_lo;
                if (s > m->clip_hi) s = m->clip_hi;
            }
            sig[(size_t)c * G + k] = s;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Zero-and-scale negative-flux fixup (Sec. 6, after Hamilton, Benzi and   */
/* Warsa).  The particle balance of a cell is the sum of the rows of its    */
/* local system A x = b:  sum_m colsum_m x_m = sum_l b_l  (absorption plus  */
/* outflow equals source plus inflow).  When x has a negative entry, every  */
/* negative entry is set to zero and the rest multiplied by the one factor  */
/* that restores that sum; if no factor can (the source side or the scaled  */
/* sum is not positive) the whole cell is set to zero.                      */
/* ------------------------------------------------------------------------ */

static void zero_and_scale(int np, const double *colsum, double src, double *x)
{
    int neg = 0;
    for (int l = 0; l < np; ++l) if (x[l] < 0.0) neg = 1;
    if (!neg) return;
    double den = 0.0;
    for (int m = 0; m < np; ++m) den += colsum[m] * (x[m] > 0.0 ? x[m] : 0.0);
    double f = (src > 0.0 && den > 0.0) ? src / den : 0.0;
    for (int m = 0; m < np; ++m) x[m] = x[m] > 0.0 ? f * x[m] : 0.0;
}

/* ------------------------------------------------------------------------ */
/* Sweep: lumped upwind DG S_N (Eq. dgsn_transport with every form lumped  */
/* by the trapezoid rule).  For each (d,g) the cells are visited in upwind  */
/* order and the local system                                              */
/*   A_lm = sigt w_l delta_lm - w_m Omega.grad(phi_l)(x_m)                 */
/*        + delta_lm sum_{outflow faces f of l} (Omega.n_f) fw_f            */
/*   b_l  = w_l q_l - sum_{inflow faces f of l} (Omega.n_f) fw_f I_up       */
/* is assembled and solved by Gaussian elimination; with fixup != 0 the   */
/* solution then goes through zero_and_scale.                               */
/*   q_l = q_iso[l][g] + inv_c_dt * psi_prev[d][g][l]                       */
/* ------------------------------------------------------------------------ */

/* one (direction d, group k) pair of orc_sweep */
static int sweep_pair(const orc_geom *g, int d, int k, const double *sig_t, const double *q_iso,
                      const double *psi_prev, double inv_c_dt, const double *inflow, int fixup, double *psi)
{
    int nx = g->nx, ny = g->dim == 2 ? g->ny : 1, np = npc(g), G = g->G, nn = nnode(g), NB = nbnode(g);
    int fwdx = om_ax(g, d, 0) > 0.0, fwdy = g->dim == 2 ? om_ax(g, d, 1) > 0.0 : 1;
    const double *pp = psi_prev ? psi_prev + ((size_t)d * G + k) * nn : NULL;
    double *out = psi + ((size_t)d * G + k) * nn;
    const double *inf = inflow ? inflow + ((size_t)d * G + k) * NB : NULL;
    for (int jj = 0; jj < ny; ++jj) {
        int j = fwdy ? jj : ny - 1 - jj;
        for (int ii = 0; ii < nx; ++ii) {
            int i = fwdx ? ii : nx - 1 - ii;
            int c = i + nx * j;
            double A[16], b[4], x[4];
            double wv = vol_weight(g, i, j), st = sig_t[(size_t)c * G + k];
            for (int l = 0; l < np; ++l) {
                double q = q_iso[(size_t)(np * c + l) * G + k];
                if (pp) q += inv_c_dt * pp[np * c + l];
                b[l] = wv * q;
                for (int m = 0; m < np; ++m) {
                    double og = 0.0;
                    for (int ax = 0; ax < g->dim; ++ax) og += om_ax(g, d, ax) * dbasis(g, i, j, l, m, ax);
                    A[l * np + m] = (l == m ? st * wv : 0.0) - wv * og;
                }
                for (int ax = 0; ax < g->dim; ++ax) {
                    for (int sd = 0; sd < 2; ++sd) {
                        if (!node_on_face(l, ax, sd)) continue;
                        double on = om_ax(g, d, ax) * (sd ? 1.0 : -1.0);
                        double fw = face_weight(g, i, j, ax);
                        if (on > 0.0) {
                            A[l * np + l] += on * fw;
                        } else {
                            int nb = neighbour(g, i, j, ax, sd);
                            double up;
                            if (nb >= 0) up = out[np * nb + mirror(l, ax)];
                            else up = inf ? inf[bnode_index(g, i, j, ax, sd, l)] : 0.0;
                            b[l] -= on * fw * up;
                        }
                    }
                }
            }
            double colsum[4], src = 0.0;
            for (int m = 0; m < np; ++m) {
                colsum[m] = 0.0;
                for (int l = 0; l < np; ++l) colsum[m] += A[l * np + m];
                src += b[m];
            }
            if (lu_solve(np, A, b, x)) return -1;
            if (fixup) zero_and_scale(np, colsum, src, x);
            for (int l = 0; l < np; ++l) out[np * c + l] = x[l];
        }
    }
    return ORC_OK;
}

/* The (d, g) pairs are independent (each writes only its own psi[d][g]),
 * so they may run on several threads (OpenMP, when compiled with it):
 * every result is the same whatever the thread count. */
int orc_sweep(const orc_geom *g, const double *sig_t, const double *q_iso, const double *psi_prev,
              double inv_c_dt, const double *inflow, int fixup, double *psi)
{
    int npairs = g->nang * g->G, fail = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : fail)
    for (int pk = 0; pk < npairs; ++pk)
        fail |= sweep_pair(g, pk / g->G, pk % g->G, sig_t, q_iso, psi_prev, inv_c_dt, inflow, fixup, psi) != ORC_OK;
    return fail ? -1 : ORC_OK;
}

/* threads of the parallel sweep (OpenMP builds; 0 = the runtime default);
 * returns the count the next sweep uses (1 without OpenMP) */
int orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Adjoint sweep: solves L^T lambda = b for each (d,g), L the operator of    */
/* orc_sweep (zero inflow), b_l = w_l src_l.  L is block lower-triangular   */
/* in upwind order: row (c,l) holds the local block A^c and, for every      */
/* inflow face f of l, the coupling (Omega.n_f) fw to the upwind neighbour's */
/* coincident node.  So L^T is block upper-triangular: row (c,m) holds      */
/* (A^c)^T and, for every outflow face f of m, the coupling                 */
/* (-Omega.n_f) fw to the downwind neighbour's coincident node.  The cells  */
/* are visited in reverse (downwind first); each transposed local system is */
/* assembled from the same terms as orc_sweep and solved by Gaussian        */
/* elimination.  Optionally                                                  */
/*   dsig[c][g] = sum_d sum_{l in c} w_l lambda_l (emis_{l,g} - psi_fwd_l).   */
/* ------------------------------------------------------------------------ */

int orc_adjoint_sweep(const orc_geom *g, const double *sig_t, const double *src, const double *emis,
                      const double *psi_fwd, double *lambda, double *dsig)
{
    int nx = g->nx, ny = g->dim == 2 ? g->ny : 1, np = npc(g), G = g->G, nn = nnode(g);
    for (int d = 0; d < g->nang; ++d) {
        int fwdx = om_ax(g, d, 0) > 0.0, fwdy = g->dim == 2 ? om_ax(g, d, 1) > 0.0 : 1;
        for (int k = 0; k < G; ++k) {
            const double *s = src + ((size_t)d * G + k) * nn;
            double *out = lambda + ((size_t)d * G + k) * nn;
            for (int jj = ny - 1; jj >= 0; --jj) {
                int j = fwdy ? jj : ny - 1 - jj;
                for (int ii = nx - 1; ii >= 0; --ii) {
                    int i = fwdx ? ii : nx - 1 - ii;
                    int c = i + nx * j;
                    double A[16], At[16], b[4], x[4];
                    double wv = vol_weight(g, i, j), st = sig_t[(size_t)c * G + k];
                    for (int l = 0; l < np; ++l) {
                        for (int m = 0; m < np; ++m) {
                            double og = 0.0;
                            for (int ax = 0; ax < g->dim; ++ax) og += om_ax(g, d, ax) * dbasis(g, i, j, l, m, ax);
                            A[l * np + m] = (l == m ? st * wv : 0.0) - wv * og;
                        }
                        for (int ax = 0; ax < g->dim; ++ax)
                            for (int sd = 0; sd < 2; ++sd) {
                                if (!node_on_face(l, ax, sd)) continue;
                                double on = om_ax(g, d, ax) * (sd ? 1.0 : -1.0);
                                if (on > 0.0) A[l * np + l] += on * face_weight(g, i, j, ax);
                            }
                    }
                    for (int l = 0; l < np; ++l)
                        for (int m = 0; m < np; ++m) At[m * np + l] = A[l * np + m];
                    for (int m = 0; m < np; ++m) {
                        b[m] = wv * s[np * c + m];
                        for (int ax = 0; ax < g->dim; ++ax)
                            for (int sd = 0; sd < 2; ++sd) {
                                if (!node_on_face(m, ax, sd)) continue;
                                double on = om_ax(g, d, ax) * (sd ? 1.0 : -1.0);
                                if (on <= 0.0) continue;            /* only outflow faces of m */
                                int nb = neighbour(g, i, j, ax, sd);
                                if (nb < 0) continue;               /* homogeneous adjoint boundary */
                                b[m] -= -on * face_weight(g, i, j, ax) * out[np * nb + mirror(m, ax)];
                            }
                    }
                    if (lu_solve(np, At, b, x)) return -1;
                    for (int l = 0; l < np; ++l) out[np * c + l] = x[l];
                }
            }
        }
    }
    if (dsig) {
        int nc = ncell(g);
        for (int c = 0; c < nc; ++c) {
            int i = c % nx, j = c / nx;
            double wv = vol_weight(g, i, j);
            for (int k = 0; k < G; ++k) {
                double acc = 0.0;
                for (int d = 0; d < g->nang; ++d) {
                    const double *L = lambda + ((size_t)d * G + k) * nn;
                    const double *I = psi_fwd + ((size_t)d * G + k) * nn;
                    for (int l = 0; l < np; ++l)
                        acc += wv * L[np * c + l] * (emis[(size_t)(np * c + l) * G + k] - I[np * c + l]);
                }
                dsig[(size_t)c * G + k] = acc;
            }
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Moments in the comparison format (sums over directions by definition).  */
/* 2D, per node: for quadrant q (0:(+,+) 1:(-,+) 2:(-,-) 3:(+,-)) the six  */
/* sums of w*{1, mu, eta, mu^2, mu*eta, eta^2}*I over d in q and all g, at */
/* index 6q+k; then 24..26 = sum_g sigma_g sum_d w*{1,mu,eta}*I.           */
/* 1D: half h (0: mu>0, 1: mu<0), index 3h+k for w*{1,mu,mu^2}; 6,7 =      */
/* sigma-weighted {1, mu}.                                                 */
/* ------------------------------------------------------------------------ */

int orc_n_moments(int dim) { return dim == 2 ? 27 : 8; }

void orc_moments(const orc_geom *g, const double *sig, const double *psi, double *mom)
{
    int nn = nnode(g), np = npc(g), G = g->G, NM = orc_n_moments(g->dim);
    memset(mom, 0, sizeof(double) * (size_t)NM * nn);
    for (int d = 0; d < g->nang; ++d) {
        double mu = om_ax(g, d, 0), eta = g->dim == 2 ? om_ax(g, d, 1) : 0.0, w = g->w[d];
        for (int k = 0; k < G; ++k) {
            const double *I = psi + ((size_t)d * G + k) * nn;
            for (int n = 0; n < nn; ++n) {
                double s = sig[(size_t)(n / np) * G + k], v = I[n];
                if (g->dim == 2) {
                    int q = (mu > 0 && eta > 0) ? 0 : (mu < 0 && eta > 0) ? 1 : (mu < 0 && eta < 0) ? 2 : 3;
                    double f[6] = {1.0, mu, eta, mu * mu, mu * eta, eta * eta};
                    for (int m = 0; m < 6; ++m) mom[(size_t)(6 * q + m) * nn + n] += w * f[m] * v;
                    mom[(size_t)24 * nn + n] += s * w * v;
                    mom[(size_t)25 * nn + n] += s * w * mu * v;
                    mom[(size_t)26 * nn + n] += s * w * eta * v;
                } else {
                    int h = mu > 0 ? 0 : 1;
                    double f[3] = {1.0, mu, mu * mu};
                    for (int m = 0; m < 3; ++m) mom[(size_t)(3 * h + m) * nn + n] += w * f[m] * v;
                    mom[(size_t)6 * nn + n] += s * w * v;
                    mom[(size_t)7 * nn + n] += s * w * mu * v;
                }
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Boundary inflow from the boundary description: B_g(T_bdr)/4pi (Eq. for  */
/* the inflow boundary condition) or the explicit per-group value; 0 for   */
/* vacuum.  Fills a general [d][g][NB] inflow array.                       */
/* ------------------------------------------------------------------------ */

void orc_inflow_from_bc(const orc_geom *g, const orc_bc *bc, double *inflow)
{
    int G = g->G, NB = nbnode(g);
    int nsides = 2 * g->dim;
    double *val = calloc((size_t)4 * G, sizeof(double));
    double *b = malloc(sizeof(double) * G), *r = malloc(sizeof(double) * G);
    for (int s = 0; s < nsides; ++s) {
        if (bc->kind[s] == 1 && bc->T_bdr[s] > 0.0) {
            orc_spectra(G, g->nu, bc->T_bdr[s], b, r);
            double B = g->a * g->c * pow(bc->T_bdr[s], 4);
            for (int k = 0; k < G; ++k) val[s * G + k] = B * b[k] / (4.0 * M_PI);
        } else if (bc->kind[s] == 2) {
            for (int k = 0; k < G; ++k) val[s * G + k] = bc->inflow_g[s][k];
        }
    }
    for (int d = 0; d < g->nang; ++d)
        for (int k = 0; k < G; ++k) {
            double *o = inflow + ((size_t)d * G + k) * NB;
            if (g->dim == 1) { o[0] = val[0 * G + k]; o[1] = val[1 * G + k]; continue; }
            for (int t = 0; t < 2 * g->ny; ++t) { o[t] = val[0 * G + k]; o[2 * g->ny + t] = val[1 * G + k]; }
            for (int t = 0; t < 2 * g->nx; ++t) { o[4 * g->ny + t] = val[2 * G + k]; o[4 * g->ny + 2 * g->nx + t] = val[3 * G + k]; }
        }
    free(val); free(b); free(r);
}

/* ------------------------------------------------------------------------ */
/* Reflective sides (specular reflection, the symmetry planes of Sec. 6):  */
/* at a boundary node of a reflective side, the inflow of a direction      */
/* entering through that side is the intensity, at the same node, of the   */
/* mirrored direction (mu -> -mu on the x sides, eta -> -eta on the y     */
/* sides), taken from psi [d][g][node].  Entries of other sides and of     */
/* leaving directions are not touched.  Returns -1 if a mirrored direction */
/* is missing from the quadrature.                                          */
/* ------------------------------------------------------------------------ */

static int mirror_direction(const orc_geom *g, int d, int ax)
{
    for (int e = 0; e < g->nang; ++e) {
        int same = 1;
        for (int k = 0; k < g->dim; ++k) {
            double want = k == ax ? -om_ax(g, d, k) : om_ax(g, d, k);
            if (fabs(om_ax(g, e, k) - want) > 1e-12) same = 0;
        }
        if (same && fabs(g->w[e] - g->w[d]) <= 1e-12 * g->w[d]) return e;
    }
    return -1;
}

int orc_reflect_inflow(const orc_geom *g, const orc_bc *bc, const double *psi, double *inflow)
{
    int nx = g->nx, ny = g->dim == 2 ? g->ny : 1, np = npc(g), G = g->G, nn = nnode(g), NB = nbnode(g);
    for (int s = 0; s < 2 * g->dim; ++s) {
        if (bc->kind[s] != 3) continue;
        int ax = s / 2, sd = s % 2;
        for (int d = 0; d < g->nang; ++d) {
            double on = (sd ? 1.0 : -1.0) * om_ax(g, d, ax);
            if (on >= 0.0) continue;                 /* leaves through this side */
            int e = mirror_direction(g, d, ax);
            if (e < 0) return -1;
            for (int k = 0; k < G; ++k) {
                const double *I = psi + ((size_t)e * G + k) * nn;
                double *o = inflow + ((size_t)d * G + k) * NB;
                /* every node of every cell on this side */
                int ncs = ax == 0 ? ny : nx;
                for (int t = 0; t < ncs; ++t) {
                    int i = ax == 0 ? (sd ? nx - 1 : 0) : t, j = ax == 0 ? t : (sd ? ny - 1 : 0);
                    for (int l = 0; l < np; ++l) {
                        if (!node_on_face(l, ax, sd)) continue;
                        o[bnode_index(g, i, j, ax, sd, l)] = I[np * (i + nx * j) + l];
                    }
                }
            }
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Low-order LDG operators (Sec. 4, lumped).  D is assembled row by row   */
/* into a small per-row table with merged columns: for node i in cell K    */
/*   (D F)_i = - sum_{m in K} w_m grad(phi_i)(x_m) . F_m                    */
/*           + sum_{interior faces f of K at i} fw [u] (((1+s)/2) F_K1.n    */
/*                                                 + ((1-s)/2) F_K2.n)      */
/* with n = +e_ax pointing from the lower cell K1 to the upper cell K2,    */
/* [u] = +1 for i in K1 and -1 for i in K2, and s = sign(wv . n) for the   */
/* fixed upwinding vector wv = (1, 1).  The penalty P collects             */
/* (c alpha/2) [u][E] on interior faces and c alpha u E on the boundary.   */
/* Columns of D index F as (node, component) -> node*dim + comp.           */
/* ------------------------------------------------------------------------ */

#define MAXROW 16
typedef struct { int n; int col[MAXROW]; double val[MAXROW]; } orc_row;

static void row_add(orc_row *r, int col, double v)
{
    for (int k = 0; k < r->n; ++k) if (r->col[k] == col) { r->val[k] += v; return; }
    if (r->n >= MAXROW) { fprintf(stderr, "oracle: row overflow\n"); abort(); }
    r->col[r->n] = col; r->val[r->n] = v; r->n++;
}

typedef struct {
    int nn, dim;
    orc_row *D;   /* [nn] rows of D */
    orc_row *P;   /* [nn] rows of the penalty */
    double *wv;   /* [nn] lumped node weights */
} orc_lo_ops;

static void lo_ops_build(const orc_geom *g, orc_lo_ops *ops)
{
    int nx = g->nx, ny = g->dim == 2 ? g->ny : 1, np = npc(g), nn = nnode(g), dim = g->dim;
    const double upw[2] = {1.0, 1.0};
    ops->nn = nn; ops->dim = dim;
    ops->D = calloc(nn, sizeof(orc_row));
    ops->P = calloc(nn, sizeof(orc_row));
    ops->wv = calloc(nn, sizeof(double));
    double alpha[2] = {alpha_axis(g, 0), dim == 2 ? alpha_axis(g, 1) : 0.0};
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            int c = i + nx * j;
            double wv = vol_weight(g, i, j);
            for (int l = 0; l < np; ++l) {
                int n = np * c + l;
                ops->wv[n] = wv;
                for (int m = 0; m < np; ++m)
                    for (int ax = 0; ax < dim; ++ax)
                        row_add(&ops->D[n], (np * c + m) * dim + ax, -wv * dbasis(g, i, j, l, m, ax));
                for (int ax = 0; ax < dim; ++ax)
                    for (int sd = 0; sd < 2; ++sd) {
                        if (!node_on_face(l, ax, sd)) continue;
                        double fw = face_weight(g, i, j, ax);
                        double cal = g->c * alpha[ax];
                        int nb = neighbour(g, i, j, ax, sd);
                        if (nb < 0) { row_add(&ops->P[n], n, fw * cal); continue; }
                        int nbn = np * nb + mirror(l, ax);
                        double jmp = sd ? 1.0 : -1.0;        /* [u] for this node */
                        int k1 = sd ? n : nbn, k2 = sd ? nbn : n;   /* nodes in K1, K2 */
                        double s = upw[ax] > 0 ? 1.0 : -1.0;
                        row_add(&ops->D[n], k1 * dim + ax, fw * jmp * 0.5 * (1.0 + s));
                        row_add(&ops->D[n], k2 * dim + ax, fw * jmp * 0.5 * (1.0 - s));
                        row_add(&ops->P[n], k1, fw * 0.5 * cal * jmp);
                        row_add(&ops->P[n], k2, -fw * 0.5 * cal * jmp);
                    }
            }
        }
}

static void lo_ops_free(orc_lo_ops *ops) { free(ops->D); free(ops->P); free(ops->wv); }

/* y = D x  (x indexed node*dim+comp) */
static void apply_D(const orc_lo_ops *o, const double *x, double *y)
{
    for (int n = 0; n < o->nn; ++n) {
        double s = 0.0;
        for (int k = 0; k < o->D[n].n; ++k) s += o->D[n].val[k] * x[o->D[n].col[k]];
        y[n] = s;
    }
}

/* y = D^T x */
static void apply_DT(const orc_lo_ops *o, const double *x, double *y)
{
    memset(y, 0, sizeof(double) * (size_t)o->nn * o->dim);
    for (int n = 0; n < o->nn; ++n)
        for (int k = 0; k < o->D[n].n; ++k) y[o->D[n].col[k]] += o->D[n].val[k] * x[n];
}

static void apply_P(const orc_lo_ops *o, const double *x, double *y)
{
    for (int n = 0; n < o->nn; ++n) {
        double s = 0.0;
        for (int k = 0; k < o->P[n].n; ++k) s += o->P[n].val[k] * x[o->P[n].col[k]];
        y[n] = s;
    }
}

/* ------------------------------------------------------------------------ */
/* Closures and low-order sources (Sec. 2 gray collapse; Sec. 4 consistent */
/* and independent LDG right-hand sides).  Output per node:                */
/*   sigE, sigF, sigP, qE, qF[dim]                                          */
/* qE = w Estar/dt - 2 sum_bfaces fw F_in + R0 (consistent only)           */
/* qF = w Fstar/(c dt) - [consistent] sum_bfaces fw P_in + R1              */
/* HO quantities are summed direction by direction from psi.               */
/* T_l is the nodal temperature of the current outer iterate.               */
/* ------------------------------------------------------------------------ */

int orc_closures(const orc_geom *g, const orc_bc *bc, int scheme, double dt, const double *sig,
                 const double *T_l, const double *Estar, const double *Fstar, const double *psi,
                 const double *inflow, double *sigE, double *sigF, double *sigP, double *qE, double *qF)
{
    int nx = g->nx, ny = g->dim == 2 ? g->ny : 1, np = npc(g), nn = nnode(g), G = g->G, dim = g->dim;
    int NB = nbnode(g);
    double c = g->c;
    double alpha[2] = {alpha_axis(g, 0), dim == 2 ? alpha_axis(g, 1) : 0.0};
    (void)bc;
    /* nodal HO quantities */
    double *E = calloc(nn, sizeof(double));            /* (1/c) sum w I */
    double *F = calloc((size_t)nn * 2, sizeof(double));    /* sum w Omega I */
    double *Pi = calloc((size_t)nn * 4, sizeof(double));   /* sum w Omega Omega I (2x2, row major) */
    double *sphi = calloc(nn, sizeof(double));          /* sum_g sigma_g sum_d w I */
    double *sF = calloc((size_t)nn * 2, sizeof(double));   /* sum_g sigma_g sum_d w Omega I */
    double *phi = calloc(nn, sizeof(double));
    double *bg = malloc(sizeof(double) * G), *rg = malloc(sizeof(double) * G);
    for (int d = 0; d < g->nang; ++d)
        for (int k = 0; k < G; ++k) {
            const double *I = psi + ((size_t)d * G + k) * nn;
            double om[2] = {om_ax(g, d, 0), dim == 2 ? om_ax(g, d, 1) : 0.0};
            for (int n = 0; n < nn; ++n) {
                double wI = g->w[d] * I[n], s = sig[(size_t)(n / np) * G + k];
                phi[n] += wI;
                sphi[n] += s * wI;
                for (int a = 0; a < dim; ++a) {
                    F[2 * n + a] += om[a] * wI;
                    sF[2 * n + a] += s * om[a] * wI;
                    for (int b2 = 0; b2 < dim; ++b2) Pi[4 * n + 2 * a + b2] += om[a] * om[b2] * wI;
                }
            }
        }
    for (int n = 0; n < nn; ++n) E[n] = phi[n] / c;
    /* gray opacities (Eqs. sigmaE, sigmaF and the Planck collapse); nodes are
       independent (OpenMP threads, when built with it) */
#pragma omp parallel for schedule(static)
    for (int n = 0; n < nn; ++n) {
        int cc = n / np;
        double bg[G], rg[G];
        orc_spectra(G, g->nu, T_l[n], bg, rg);
        double sb = 0, sr = 0, sbs = 0, srs = 0;
        for (int k = 0; k < G; ++k) {
            double s = sig[(size_t)cc * G + k];
            sb += bg[k]; sbs += bg[k] * s; sr += rg[k]; srs += rg[k] * s;
        }
        sigP[n] = sbs / sb;
        sigF[n] = srs / sr;
        sigE[n] = phi[n] > 0.0 ? sphi[n] / phi[n] : sigP[n];
    }
    /* sources */
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            int cc = i + nx * j;
            double wv = vol_weight(g, i, j);
            for (int l = 0; l < np; ++l) {
                int n = np * cc + l;
                double r0 = 0.0, r1[2] = {0.0, 0.0};
                double qe = wv * Estar[n] / dt, qf[2] = {0.0, 0.0};
                for (int a = 0; a < dim; ++a) qf[a] = wv * Fstar[dim * n + a] / (c * dt);
                /* multigroup additive correction, lumped: w (sigF F - sum_g sigma_g F_g) */
                for (int a = 0; a < dim; ++a) r1[a] += wv * (sigF[n] * F[2 * n + a] - sF[2 * n + a]);
                /* volume closure: sum_m w_m (T_m grad phi_l(x_m)), T = Pi - (phi/3) I */
                for (int m = 0; m < np; ++m) {
                    int nm = np * cc + m;
                    for (int a = 0; a < dim; ++a)
                        for (int b2 = 0; b2 < dim; ++b2) {
                            double Tab = Pi[4 * nm + 2 * a + b2] - (a == b2 ? phi[nm] / 3.0 : 0.0);
                            r1[a] += wv * Tab * dbasis(g, i, j, l, m, b2);
                        }
                }
                for (int ax = 0; ax < dim; ++ax)
                    for (int sd = 0; sd < 2; ++sd) {
                        if (!node_on_face(l, ax, sd)) continue;
                        double fw = face_weight(g, i, j, ax);
                        double sgn = sd ? 1.0 : -1.0;   /* outward normal = sgn e_ax */
                        int nb = neighbour(g, i, j, ax, sd);
                        if (nb >= 0) {
                            int nbn = np * nb + mirror(l, ax);
                            int n1 = sd ? n : nbn, n2 = sd ? nbn : n;   /* K1 (lower), K2 (upper) nodes */
                            double jmp = sgn;                            /* [u] for this node */
                            double s = 1.0;                              /* wv = (1,1) */
                            /* half-range sums w.r.t. n = +e_ax at n1 and n2 */
                            double beta1 = 0, beta2 = 0, Fn1 = F[2 * n1 + ax], Fn2 = F[2 * n2 + ax];
                            double Pp1[2] = {0, 0}, Pm1[2] = {0, 0}, Pp2[2] = {0, 0}, Pm2[2] = {0, 0};
                            for (int d = 0; d < g->nang; ++d) {
                                double on = om_ax(g, d, ax);
                                double om[2] = {om_ax(g, d, 0), dim == 2 ? om_ax(g, d, 1) : 0.0};
                                for (int k = 0; k < G; ++k) {
                                    const double *I = psi + ((size_t)d * G + k) * nn;
                                    double w1 = g->w[d] * I[n1], w2 = g->w[d] * I[n2];
                                    beta1 += (fabs(on) - alpha[ax]) * w1;
                                    beta2 += (fabs(on) - alpha[ax]) * w2;
                                    for (int a = 0; a < dim; ++a) {
                                        if (on > 0) { Pp1[a] += om[a] * on * w1; Pp2[a] += om[a] * on * w2; }
                                        else { Pm1[a] += om[a] * on * w1; Pm2[a] += om[a] * on * w2; }
                                    }
                                }
                            }
                            if (scheme == 0) r0 += fw * jmp * (0.5 * s * (Fn1 - Fn2) - 0.5 * (beta1 - beta2));
                            for (int a = 0; a < dim; ++a) {
                                double Tn1 = 0, Tn2 = 0;   /* (T n)_a with n = e_ax */
                                Tn1 = Pi[4 * n1 + 2 * a + ax] - (a == ax ? phi[n1] / 3.0 : 0.0);
                                Tn2 = Pi[4 * n2 + 2 * a + ax] - (a == ax ? phi[n2] / 3.0 : 0.0);
                                double v = -0.5 * (Tn1 + Tn2);
                                if (scheme == 0) {
                                    v += -0.5 * ((Pp1[a] - Pm1[a]) - (Pp2[a] - Pm2[a]));
                                    v += -(c / 6.0) * s * (a == ax ? 1.0 : 0.0) * (E[n1] - E[n2]);
                                }
                                r1[a] += fw * jmp * v;
                            }
                        } else {
                            const double *inf = inflow;
                            int bi = bnode_index(g, i, j, ax, sd, l);
                            double Jp = 0, Fin = 0, Pp[2] = {0, 0}, Pin[2] = {0, 0};
                            for (int d = 0; d < g->nang; ++d) {
                                double on = sgn * om_ax(g, d, ax);  /* Omega . n_K */
                                double om[2] = {om_ax(g, d, 0), dim == 2 ? om_ax(g, d, 1) : 0.0};
                                for (int k = 0; k < G; ++k) {
                                    double Iown = psi[((size_t)d * G + k) * nn + n];
                                    double Ib = inf ? inf[((size_t)d * G + k) * NB + bi] : 0.0;
                                    if (on > 0) {
                                        Jp += g->w[d] * on * Iown;
                                        for (int a = 0; a < dim; ++a) Pp[a] += g->w[d] * om[a] * on * Iown;
                                    } else {
                                        Fin += g->w[d] * on * Ib;
                                        for (int a = 0; a < dim; ++a) Pin[a] += g->w[d] * om[a] * on * Ib;
                                    }
                                }
                            }
                            qe += -2.0 * fw * Fin;
                            if (scheme == 0) {
                                r0 += -fw * (Jp - c * alpha[ax] * E[n] - Fin);
                                for (int a = 0; a < dim; ++a) {
                                    qf[a] += -fw * Pin[a];
                                    r1[a] += fw * ((c / 3.0) * (a == ax ? sgn : 0.0) * E[n] - Pp[a]);
                                }
                            }
                        }
                    }
                qE[n] = qe + r0;
                for (int a = 0; a < dim; ++a) qF[dim * n + a] = qf[a] + r1[a];
            }
        }
    free(E); free(F); free(Pi); free(sphi); free(sF); free(phi); free(bg); free(rg);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Pointwise energy balance (nonlinear elimination, Eq. nonlinear_T_update)*/
/*   cv T/dt + sigP a c T^4 = rhs,  rhs = c sigE E + cv Tstar/dt           */
/* Newton safeguarded by bisection on the bracket [0, rhs dt/cv].          */
/* Stop when |f(T)| <= rtol |rhs|.  Returns iterations, or -1 if rhs <= 0. */
/* ------------------------------------------------------------------------ */

int orc_energy_solve(double cv_dt, double k4, double rhs, double T0, double rtol, int maxit, double *T)
{
    if (!(rhs > 0.0)) return -1;
    double lo = 0.0, hi = rhs / cv_dt;
    double t = T0;
    if (!(t > lo && t < hi)) t = 0.5 * (lo + hi);
    for (int it = 1; it <= maxit; ++it) {
        double f = cv_dt * t + k4 * t * t * t * t - rhs;
        if (fabs(f) <= rtol * fabs(rhs)) { *T = t; return it - 1; }
        if (f > 0) hi = t; else lo = t;
        double fp = cv_dt + 4.0 * k4 * t * t * t;
        double tn = t - f / fp;
        if (!(tn > lo && tn < hi)) tn = 0.5 * (lo + hi);
        t = tn;
    }
    *T = t;
    return maxit;
}

/* Temperature floor (Sec. 6): with T_floor > 0 the balance's temperature  */
/* is max(root, T_floor), and T_floor when it has no positive root (it < 0  */
/* from orc_energy_solve).  Returns 1 for a missing root without a floor.   */
static int floor_temperature(double T_floor, int it, double *T)
{
    if (it < 0) {
        if (!(T_floor > 0.0)) return 1;
        *T = T_floor;
        return 0;
    }
    if (T_floor > 0.0 && *T < T_floor) *T = T_floor;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Low-order Newton with nonlinear elimination of T (Sec. 5):              */
/*   S = (c/3) D M_F^-1 D^T + M_E + P - dB dBt^-1 M_a                       */
/*   S E = qE + B(T0) - D M_F^-1 qF + dB dBt^-1 (qT - Bt(T0))               */
/*   F = M_F^-1 (qF + (c/3) D^T E);  T from the pointwise balance.          */
/* Jacobi-preconditioned CG.  E, T are in/out (initial guess in), F out.   */
/* ------------------------------------------------------------------------ */

static double dot(int n, const double *a, const double *b)
{
    double s = 0;
    for (int i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

typedef struct {
    const orc_lo_ops *ops;
    const double *MF;     /* [nn*dim] */
    const double *diagE;  /* [nn] */
    double c3;
    double *tmpF, *tmpF2, *tmpE;
} orc_schur;

static void schur_apply(const orc_schur *S, const double *x, double *y)
{
    int nn = S->ops->nn, dim = S->ops->dim;
    apply_DT(S->ops, x, S->tmpF);
    for (int k = 0; k < nn * dim; ++k) S->tmpF[k] /= S->MF[k];
    apply_D(S->ops, S->tmpF, y);
    apply_P(S->ops, x, S->tmpE);
    for (int n = 0; n < nn; ++n) y[n] = S->c3 * y[n] + S->tmpE[n] + S->diagE[n] * x[n];
}

/* Returns the iteration count; *capped = 1 when maxit iterations ran and the
 * residual still exceeds the threshold (the paper's tables mark such capped
 * counts). */
static int pcg(const orc_schur *S, const double *b, double *x, const double *Minv, double rtol, int maxit,
               int *capped)
{
    int n = S->ops->nn;
    double *r = malloc(sizeof(double) * n), *z = malloc(sizeof(double) * n);
    double *p = malloc(sizeof(double) * n), *Ap = malloc(sizeof(double) * n);
    schur_apply(S, x, Ap);
    for (int i = 0; i < n; ++i) r[i] = b[i] - Ap[i];
    double bn = sqrt(dot(n, b, b));
    if (bn == 0.0) bn = 1.0;
    for (int i = 0; i < n; ++i) { z[i] = Minv[i] * r[i]; p[i] = z[i]; }
    double rz = dot(n, r, z);
    int it = 0;
    while (it < maxit && sqrt(dot(n, r, r)) > rtol * bn) {
        schur_apply(S, p, Ap);
        double al = rz / dot(n, p, Ap);
        for (int i = 0; i < n; ++i) { x[i] += al * p[i]; r[i] -= al * Ap[i]; }
        for (int i = 0; i < n; ++i) z[i] = Minv[i] * r[i];
        double rzn = dot(n, r, z);
        for (int i = 0; i < n; ++i) p[i] = z[i] + (rzn / rz) * p[i];
        rz = rzn;
        ++it;
    }
    *capped = it >= maxit && sqrt(dot(n, r, r)) > rtol * bn;
    free(r); free(z); free(p); free(Ap);
    return it;
}

/* Solve the low-order system for fixed closures.  cvn: nodal c_v.
 * Returns ORC_OK / ORC_E_NONPHYSICAL; fills stats (inner, cg, elim). */
static int lo_solve_ops(const orc_geom *g, const orc_lo_ops *ops, const orc_opts *op, double dt,
                        const double *cvn, const double *Tstar, const double *sigE, const double *sigF,
                        const double *sigP, const double *qE, const double *qF, double *E, double *F,
                        double *T, orc_stats *st)
{
    int nn = ops->nn, dim = ops->dim;
    double a = g->a, c = g->c;
    double *MF = malloc(sizeof(double) * nn * dim), *diagE = malloc(sizeof(double) * nn);
    double *rhs = malloc(sizeof(double) * nn), *tF = malloc(sizeof(double) * nn * dim);
    double *tF2 = malloc(sizeof(double) * nn * dim), *tE = malloc(sizeof(double) * nn);
    double *Minv = malloc(sizeof(double) * nn), *DqF = malloc(sizeof(double) * nn);
    double *Eold = malloc(sizeof(double) * nn), *Told = malloc(sizeof(double) * nn);
    for (int n = 0; n < nn; ++n)
        for (int k = 0; k < dim; ++k) MF[n * dim + k] = ops->wv[n] * (sigF[n] + 1.0 / (c * dt));
    for (int k = 0; k < nn * dim; ++k) tF[k] = qF[k] / MF[k];
    apply_D(ops, tF, DqF);
    orc_schur S = {ops, MF, diagE, c / 3.0, tF, tF2, tE};
    double first = -1.0;
    int status = ORC_OK;
    for (int m = 1; m <= op->max_inner; ++m) {
        memcpy(Eold, E, sizeof(double) * nn);
        memcpy(Told, T, sizeof(double) * nn);
        for (int n = 0; n < nn; ++n) {
            double wv = ops->wv[n], T0 = T[n];
            double dB = wv * 4.0 * sigP[n] * a * c * T0 * T0 * T0;
            double dBt = wv * (cvn[n] / dt) + dB;
            double B0 = wv * sigP[n] * a * c * pow(T0, 4);
            double Bt0 = wv * cvn[n] * T0 / dt + B0;
            double Ma = wv * c * sigE[n];
            double qT = wv * cvn[n] * Tstar[n] / dt;
            diagE[n] = wv * c * (sigE[n] + 1.0 / (c * dt)) - dB * Ma / dBt;
            rhs[n] = qE[n] + B0 - DqF[n] + dB / dBt * (qT - Bt0);
        }
        /* Jacobi diagonal: (c/3) sum_k D_{n,k}^2 / MF_k + P_nn + diagE_n */
        for (int n = 0; n < nn; ++n) {
            double dd = 0.0;
            for (int k = 0; k < ops->D[n].n; ++k) dd += ops->D[n].val[k] * ops->D[n].val[k] / MF[ops->D[n].col[k]];
            double pp = 0.0;
            for (int k = 0; k < ops->P[n].n; ++k) if (ops->P[n].col[k] == n) pp += ops->P[n].val[k];
            Minv[n] = 1.0 / ((c / 3.0) * dd + pp + diagE[n]);
        }
        int cg_capped = 0;
        st->cg_total += pcg(&S, rhs, E, Minv, op->cg_rtol, op->max_cg, &cg_capped);
        if (cg_capped) st->hit_max = 1;
        /* back substitution for F */
        apply_DT(ops, E, tF);
        for (int k = 0; k < nn * dim; ++k) F[k] = (qF[k] + (c / 3.0) * tF[k]) / MF[k];
        /* nonlinear elimination of T */
        for (int n = 0; n < nn; ++n) {
            double r = c * sigE[n] * E[n] + cvn[n] * Tstar[n] / dt;
            int it = orc_energy_solve(cvn[n] / dt, sigP[n] * a * c, r, T[n], op->elim_rtol, op->max_elim, &T[n]);
            if (floor_temperature(op->T_floor, it, &T[n])) { status = ORC_E_NONPHYSICAL; break; }
            if (it > st->elim_max) st->elim_max = it;
            if (it >= op->max_elim) st->hit_max = 1;   /* this node's Newton ran to its cap */
        }
        st->inner_total++;
        if (status) break;
        double diff = 0.0;
        for (int n = 0; n < nn; ++n) diff += (T[n] - Told[n]) * (T[n] - Told[n]) + (E[n] - Eold[n]) * (E[n] - Eold[n]);
        diff = sqrt(diff);
        if (m == 1) first = diff;
        if (diff == 0.0 || (m > 1 && diff < op->eps_inner * first) ) break;
        if (m == op->max_inner) st->hit_max = 1;
    }
    free(MF); free(diagE); free(rhs); free(tF); free(tF2); free(tE); free(Minv); free(DqF); free(Eold); free(Told);
    return status;
}

static void nodal_cv(const orc_geom *g, const orc_mat *m, double *cvn)
{
    int np = npc(g), nn = nnode(g);
    for (int n = 0; n < nn; ++n) cvn[n] = m->cv[m->region[n / np]];
}

int orc_lo_solve(const orc_geom *g, const orc_mat *m, const orc_opts *op, double dt, const double *Tstar,
                 const double *sigE, const double *sigF, const double *sigP, const double *qE,
                 const double *qF, double *E, double *F, double *T, orc_stats *st)
{
    orc_lo_ops ops;
    lo_ops_build(g, &ops);
    double *cvn = malloc(sizeof(double) * ops.nn);
    nodal_cv(g, m, cvn);
    memset(st, 0, sizeof *st);
    int r = lo_solve_ops(g, &ops, op, dt, cvn, Tstar, sigE, sigF, sigP, qE, qF, E, F, T, st);
    free(cvn);
    lo_ops_free(&ops);
    return r;
}

/* Dense Schur complement for tiny meshes (SPD pin): S[nn][nn] */
void orc_schur_dense(const orc_geom *g, double dt, const double *sigE, const double *sigF, const double *sigP,
                     const double *cvn, const double *T0, double *Sout)
{
    orc_lo_ops ops;
    lo_ops_build(g, &ops);
    int nn = ops.nn, dim = ops.dim;
    double a = g->a, c = g->c;
    double *MF = malloc(sizeof(double) * nn * dim), *diagE = malloc(sizeof(double) * nn);
    double *tF = malloc(sizeof(double) * nn * dim), *tF2 = malloc(sizeof(double) * nn * dim);
    double *tE = malloc(sizeof(double) * nn), *e = calloc(nn, sizeof(double)), *col = malloc(sizeof(double) * nn);
    for (int n = 0; n < nn; ++n) {
        for (int k = 0; k < dim; ++k) MF[n * dim + k] = ops.wv[n] * (sigF[n] + 1.0 / (c * dt));
        double wv = ops.wv[n], t = T0[n];
        double dB = wv * 4.0 * sigP[n] * a * c * t * t * t, dBt = wv * cvn[n] / dt + dB, Ma = wv * c * sigE[n];
        diagE[n] = wv * c * (sigE[n] + 1.0 / (c * dt)) - dB * Ma / dBt;
    }
    orc_schur S = {&ops, MF, diagE, c / 3.0, tF, tF2, tE};
    for (int k = 0; k < nn; ++k) {
        e[k] = 1.0;
        schur_apply(&S, e, col);
        for (int n = 0; n < nn; ++n) Sout[(size_t)n * nn + k] = col[n];
        e[k] = 0.0;
    }
    free(MF); free(diagE); free(tF); free(tF2); free(tE); free(e); free(col);
    lo_ops_free(&ops);
}

/* Export D, P in dense form (tiny meshes) for structural tests. */
void orc_lo_dense(const orc_geom *g, double *Dd /*[nn][nn*dim]*/, double *Pd /*[nn][nn]*/, double *wv)
{
    orc_lo_ops ops;
    lo_ops_build(g, &ops);
    int nn = ops.nn, dim = ops.dim;
    memset(Dd, 0, sizeof(double) * (size_t)nn * nn * dim);
    memset(Pd, 0, sizeof(double) * (size_t)nn * nn);
    for (int n = 0; n < nn; ++n) {
        for (int k = 0; k < ops.D[n].n; ++k) Dd[(size_t)n * nn * dim + ops.D[n].col[k]] += ops.D[n].val[k];
        for (int k = 0; k < ops.P[n].n; ++k) Pd[(size_t)n * nn + ops.P[n].col[k]] += ops.P[n].val[k];
        wv[n] = ops.wv[n];
    }
    lo_ops_free(&ops);
}

/* ------------------------------------------------------------------------ */
/* One backward-Euler step (Algorithm 1).                                   */
/* State in/out: psi [d][g][node] (I^k -> I^{k+1}), T, E_lo, F_lo (nodal).  */
/* scheme 0/1: SM consistent/independent; 2: unaccelerated (sweep +        */
/* pointwise elimination against sum_g sigma_g E_g from the sweep).        */
/* ------------------------------------------------------------------------ */

int orc_step(const orc_geom *g, const orc_mat *mt, const orc_bc *bc, const orc_opts *op, double dt,
             double *psi, double *T, double *E_lo, double *F_lo, orc_stats *st)
{
    int nn = nnode(g), np = npc(g), G = g->G, nc = ncell(g), dim = g->dim, NB = nbnode(g);
    size_t npsi = (size_t)g->nang * G * nn;
    double a = g->a, c = g->c;
    memset(st, 0, sizeof *st);
    double *sig = malloc(sizeof(double) * (size_t)nc * G), *sigt = malloc(sizeof(double) * (size_t)nc * G);
    double *psi_prev = malloc(sizeof(double) * npsi), *q = malloc(sizeof(double) * (size_t)nn * G);
    double *inflow = malloc(sizeof(double) * (size_t)g->nang * G * NB);
    double *Tstar = malloc(sizeof(double) * nn), *Estar = calloc(nn, sizeof(double));
    double *Fstar = calloc((size_t)nn * dim, sizeof(double)), *cvn = malloc(sizeof(double) * nn);
    double *sigE = malloc(sizeof(double) * nn), *sigF = malloc(sizeof(double) * nn), *sigP = malloc(sizeof(double) * nn);
    double *qE = malloc(sizeof(double) * nn), *qF = malloc(sizeof(double) * nn * dim);
    double *Tl = malloc(sizeof(double) * nn), *El = malloc(sizeof(double) * nn);
    double *bg = malloc(sizeof(double) * G), *rg = malloc(sizeof(double) * G);
    double *sphi = malloc(sizeof(double) * nn);
    orc_lo_ops ops;
    lo_ops_build(g, &ops);
    nodal_cv(g, mt, cvn);
    memcpy(psi_prev, psi, sizeof(double) * npsi);
    memcpy(Tstar, T, sizeof(double) * nn);
    orc_opacity(g, mt, T, sig);
    for (size_t k = 0; k < (size_t)nc * G; ++k) sigt[k] = sig[k] + 1.0 / (c * dt);
    orc_inflow_from_bc(g, bc, inflow);
    int refl_bad = orc_reflect_inflow(g, bc, psi_prev, inflow);
    /* time-edge sources: HO sums of I^k (default) or the LO solution */
    if (op->lo_time_edge) {
        memcpy(Estar, E_lo, sizeof(double) * nn);
        memcpy(Fstar, F_lo, sizeof(double) * nn * dim);
    } else {
        for (int d = 0; d < g->nang; ++d)
            for (int k = 0; k < G; ++k)
                for (int n = 0; n < nn; ++n) {
                    double wI = g->w[d] * psi_prev[((size_t)d * G + k) * nn + n];
                    Estar[n] += wI / c;
                    for (int ax = 0; ax < dim; ++ax) Fstar[dim * n + ax] += om_ax(g, d, ax) * wI;
                }
    }
    memcpy(Tl, T, sizeof(double) * nn);
    if (op->scheme == 2) memcpy(El, Estar, sizeof(double) * nn);
    else memcpy(El, E_lo, sizeof(double) * nn);
    double first = -1.0;
    int status = refl_bad ? -2 : ORC_OK;
    int maxo = refl_bad ? 0 : op->max_outer;
    for (int l = 1; l <= maxo; ++l) {
        /* emission source at the current temperature iterate (nodes are
           independent: OpenMP threads, when built with it) */
#pragma omp parallel for schedule(static)
        for (int n = 0; n < nn; ++n) {
            double bg[G], rg[G];
            orc_spectra(G, g->nu, Tl[n], bg, rg);
            double B = a * c * pow(Tl[n], 4);
            for (int k = 0; k < G; ++k) q[(size_t)n * G + k] = sig[(size_t)(n / np) * G + k] * B * bg[k] / (4.0 * M_PI);
        }
        orc_sweep(g, sigt, q, psi_prev, 1.0 / (c * dt), inflow, op->fixup, psi);
        /* reflective sides: the inflow now mirrors this sweep's intensity (the
           closures below and the next sweep use it) */
        orc_reflect_inflow(g, bc, psi, inflow);
        st->outer++;
        double *Tn = malloc(sizeof(double) * nn), *En = malloc(sizeof(double) * nn);
        if (op->scheme == 2) {
            memset(sphi, 0, sizeof(double) * nn);
            memset(En, 0, sizeof(double) * nn);
            for (int d = 0; d < g->nang; ++d)
                for (int k = 0; k < G; ++k)
                    for (int n = 0; n < nn; ++n) {
                        double wI = g->w[d] * psi[((size_t)d * G + k) * nn + n];
                        En[n] += wI / c;
                        sphi[n] += sig[(size_t)(n / np) * G + k] * wI;
                    }
            for (int n = 0; n < nn; ++n) {
                orc_spectra(G, g->nu, Tl[n], bg, rg);
                double sb = 0, sbs = 0;
                for (int k = 0; k < G; ++k) { sb += bg[k]; sbs += bg[k] * sig[(size_t)(n / np) * G + k]; }
                double r = sphi[n] + cvn[n] * Tstar[n] / dt;
                Tn[n] = Tl[n];
                int it = orc_energy_solve(cvn[n] / dt, (sbs / sb) * a * c, r, Tl[n], op->elim_rtol, op->max_elim, &Tn[n]);
                if (floor_temperature(op->T_floor, it, &Tn[n])) { status = ORC_E_NONPHYSICAL; break; }
                if (it > st->elim_max) st->elim_max = it;
                if (it >= op->max_elim) st->hit_max = 1;
            }
            memcpy(E_lo, En, sizeof(double) * nn);
        } else {
            orc_closures(g, bc, op->scheme, dt, sig, Tl, Estar, Fstar, psi, inflow, sigE, sigF, sigP, qE, qF);
            memcpy(Tn, Tl, sizeof(double) * nn);
            memcpy(En, El, sizeof(double) * nn);
            orc_stats s2;
            memset(&s2, 0, sizeof s2);
            status = lo_solve_ops(g, &ops, op, dt, cvn, Tstar, sigE, sigF, sigP, qE, qF, En, F_lo, Tn, &s2);
            st->inner_total += s2.inner_total;
            st->cg_total += s2.cg_total;
            if (s2.elim_max > st->elim_max) st->elim_max = s2.elim_max;
            if (s2.hit_max) st->hit_max = 1;
        }
        double diff = 0.0;
        for (int n = 0; n < nn; ++n) diff += (Tn[n] - Tl[n]) * (Tn[n] - Tl[n]) + (En[n] - El[n]) * (En[n] - El[n]);
        diff = sqrt(diff);
        memcpy(Tl, Tn, sizeof(double) * nn);
        memcpy(El, En, sizeof(double) * nn);
        free(Tn); free(En);
        if (status) break;
        if (l == 1) first = diff;
        if (diff == 0.0 || (l > 1 && diff < op->eps_outer * first)) break;
        if (l == maxo) st->hit_max = 1;
    }
    memcpy(T, Tl, sizeof(double) * nn);
    if (op->scheme != 2) memcpy(E_lo, El, sizeof(double) * nn);
    lo_ops_free(&ops);
    free(sig); free(sigt); free(psi_prev); free(q); free(inflow); free(Tstar); free(Estar); free(Fstar);
    free(cvn); free(sigE); free(sigF); free(sigP); free(qE); free(qF); free(Tl); free(El); free(bg); free(rg);
    free(sphi);
    return status;
}

/* initial isotropic equilibrium intensity B_g(T_n)/4pi at every node */
void orc_equilibrium_psi(const orc_geom *g, const double *T, double *psi)
{
    int nn = nnode(g), G = g->G;
#pragma omp parallel for schedule(static)
    for (int n = 0; n < nn; ++n) {
        double b[G], r[G];
        orc_spectra(G, g->nu, T[n], b, r);
        double B = g->a * g->c * pow(T[n], 4);
        for (int d = 0; d < g->nang; ++d)
            for (int k = 0; k < G; ++k) psi[((size_t)d * G + k) * nn + n] = B * b[k] / (4.0 * M_PI);
    }
}

/* ------------------------------------------------------------------------ */
/* Adjoint gradient of the time-integrated right-boundary outflow            */
/*   J = sum_k dt sum_g sum_{d: mu_d > 0} w_d mu_d sum_{n on x+} fw_n I^k_n  */
/* with respect to log sigma0_r and log c_v,r, taken at the converged fixed  */
/* point of every step (implicit function theorem).  The fixed point of a   */
/* step solves the lumped DG transport with emission sigma_g B_g(T)/4pi and */
/* time-edge source I^{k-1}/(c dt) (Sec. 3) together with the lumped nodal  */
/* energy balance c_v (T - T^{k-1})/dt = sum_g sigma_g (phi_g - 4 pi E_g(T)),*/
/* E_g = a c T^4 b_g / 4pi (Sec. 2), with sigma_g from the start-of-step     */
/* cell temperature.  Forward: orc_step with the options given (tight       */
/* tolerances), keeping I^k, T^k, sigma^k.  Reverse, k = N..1: the adjoint  */
/* of the step solves                                                        */
/*   L^T lam_{d,g} = S^I_{d,g} + sigma_g w_d tau                              */
/*   D tau - w sum_g sigma_g E'_g(T) sum_d lam_{d,g} = S^T,                   */
/*   D = c_v/dt + sum_g sigma_g 4 pi E'_g(T),  4 pi E'_g = 4 a c T^3 r_g      */
/* by source iteration (adjoint sweep, then pointwise tau), with            */
/*   S^I = dJ/dI^k + (w/(c dt)) lam^{k+1},                                    */
/*   S^T = (c_v/dt) tau^{k+1} - sum_g dsigma^{k+1}_g/dT^k G^{k+1}_g,          */
/*   G_{c,g} = lam^T dR/dsigma_{c,g}                                          */
/*          = sum_d sum_{l in c} w_l lam (I - E_g)                             */
/*            - sum_{l in c} tau_l (phi_g - 4 pi E_g),                         */
/* and dJ/dlog sigma0_r = -sum_k sum_{c in r, g unclipped} sigma G,          */
/*     dJ/dlog c_v,r    = -sum_k sum_{n in r} tau_n c_v (T^k - T^{k-1})/dt.  */
/* Objectives: 0, the time-integrated outflow through x+,                    */
/*   J = sum_k dt sum_{d: mu>0} w_d mu_d sum_g sum_{n on x+} fw_n I^k        */
/*   (dJ/dI^k the outflow weights, no direct T dependence);                   */
/* 1, the material energy at the final step, J = sum_n w_n c_v,n T^N_n       */
/*   (dJ/dI = 0; S^T at step N gains w c_v; dJ/dlog c_v,r gains the direct  */
/*   term sum_{n in r} w c_v T^N).                                             */
/* ------------------------------------------------------------------------ */

int orc_adjoint_gradient(const orc_geom *g, const orc_mat *mt, const orc_bc *bc, const orc_opts *op, double dt,
                         int n_steps, int objective, const double *psi0, const double *T0, double *J_out,
                         double *grad_s0, double *grad_cv, int n_regions, int *adj_iters)
{
    if (objective != 0 && objective != 1) return -2;
    if (op->fixup || op->T_floor != 0.0) return -2;   /* the adjoint of the linear, unfloored step */
    for (int s = 0; s < 2 * g->dim; ++s)
        if (bc->kind[s] == 3) return -2;               /* vacuum and given inflow only */
    int nn = nnode(g), np = npc(g), G = g->G, nc = ncell(g), nd = g->nang, dim = g->dim;
    int nx = g->nx;
    size_t npsi = (size_t)nd * G * nn;
    double a = g->a, c = g->c;
    int N = n_steps;
    double *ck_psi = malloc(sizeof(double) * npsi * (N + 1));
    double *ck_T = malloc(sizeof(double) * (size_t)nn * (N + 1));
    double *ck_sig = malloc(sizeof(double) * (size_t)nc * G * (N + 1));
    double *E = malloc(sizeof(double) * nn), *F = calloc((size_t)nn * dim, sizeof(double));
    double *cvn = malloc(sizeof(double) * nn), *wsp = malloc(sizeof(double) * nn);
    double *dJdI = calloc(npsi, sizeof(double));
    int rc = ORC_OK;
    nodal_cv(g, mt, cvn);
    for (int cc = 0; cc < nc; ++cc)
        for (int l = 0; l < np; ++l) wsp[np * cc + l] = vol_weight(g, cc % nx, cc / nx);
    /* objective 0 weights: outflow through x+ (objective 1 leaves dJ/dI = 0) */
    for (int d = 0; d < nd && objective == 0; ++d) {
        double mu = om_ax(g, d, 0);
        if (mu <= 0.0) continue;
        for (int k = 0; k < G; ++k)
            for (int cc = 0; cc < nc; ++cc) {
                int i = cc % nx, j = cc / nx;
                if (i != nx - 1) continue;
                for (int l = 0; l < np; ++l)
                    if (node_on_face(l, 0, 1))
                        dJdI[((size_t)d * G + k) * nn + np * cc + l] = dt * g->w[d] * mu * face_weight(g, i, j, 0);
            }
    }
    /* forward with checkpoints */
    memcpy(ck_psi, psi0, sizeof(double) * npsi);
    memcpy(ck_T, T0, sizeof(double) * nn);
    for (int n = 0; n < nn; ++n) E[n] = a * pow(T0[n], 4);
    double J = 0.0;
    for (int k = 1; k <= N && rc == ORC_OK; ++k) {
        double *psi = ck_psi + npsi * k, *T = ck_T + (size_t)nn * k;
        memcpy(psi, ck_psi + npsi * (k - 1), sizeof(double) * npsi);
        memcpy(T, ck_T + (size_t)nn * (k - 1), sizeof(double) * nn);
        orc_opacity(g, mt, T, ck_sig + (size_t)nc * G * k);    /* start-of-step temperature */
        orc_stats st;
        rc = orc_step(g, mt, bc, op, dt, psi, T, E, F, &st);
        for (size_t t = 0; t < npsi; ++t) J += dJdI[t] * psi[t];
    }
    if (objective == 1) {
        const double *TN = ck_T + (size_t)nn * N;
        for (int n = 0; n < nn; ++n) J += wsp[n] * cvn[n] * TN[n];
    }
    *J_out = J;
    if (rc != ORC_OK) goto done;
    {
        for (int r = 0; r < n_regions; ++r) { grad_s0[r] = 0.0; grad_cv[r] = 0.0; }
        double *lam = calloc(npsi, sizeof(double)), *lam_next = calloc(npsi, sizeof(double));
        double *src = malloc(sizeof(double) * npsi), *sigt = malloc(sizeof(double) * (size_t)nc * G);
        double *tau = calloc(nn, sizeof(double)), *ST = calloc(nn, sizeof(double)), *ST_prev = calloc(nn, sizeof(double));
        double *emis = malloc(sizeof(double) * (size_t)nn * G), *dE = malloc(sizeof(double) * (size_t)nn * G);
        double *phi = malloc(sizeof(double) * (size_t)nn * G), *D = malloc(sizeof(double) * nn);
        double *Gs = malloc(sizeof(double) * (size_t)nc * G), *dsig = malloc(sizeof(double) * (size_t)nc * G);
        double *bg = malloc(sizeof(double) * G), *rg = malloc(sizeof(double) * G), *tau_new = malloc(sizeof(double) * nn);
        int iters = 0;
        if (objective == 1)   /* dJ/dT^N enters the energy-balance adjoint of the last step */
            for (int n = 0; n < nn; ++n) ST[n] = wsp[n] * cvn[n];
        for (int k = N; k >= 1; --k) {
            const double *psi = ck_psi + npsi * k, *T = ck_T + (size_t)nn * k, *Tp = ck_T + (size_t)nn * (k - 1);
            const double *sig = ck_sig + (size_t)nc * G * k;
            for (size_t t = 0; t < (size_t)nc * G; ++t) sigt[t] = sig[t] + 1.0 / (c * dt);
            for (int n = 0; n < nn; ++n) {
                orc_spectra(G, g->nu, T[n], bg, rg);
                double T3 = pow(T[n], 3), T4 = T3 * T[n];
                D[n] = cvn[n] / dt;
                for (int q = 0; q < G; ++q) {
                    emis[(size_t)n * G + q] = a * c * T4 * bg[q] / (4.0 * M_PI);
                    dE[(size_t)n * G + q] = 4.0 * a * c * T3 * rg[q] / (4.0 * M_PI);
                    D[n] += sig[(size_t)(n / np) * G + q] * 4.0 * M_PI * dE[(size_t)n * G + q];
                    double s = 0.0;
                    for (int d = 0; d < nd; ++d) s += g->w[d] * psi[((size_t)d * G + q) * nn + n];
                    phi[(size_t)n * G + q] = s;
                }
            }
            /* adjoint source iteration */
            for (int n = 0; n < nn; ++n) tau[n] = 0.0;
            for (int it = 0; it < 500; ++it) {
                for (int d = 0; d < nd; ++d)
                    for (int q = 0; q < G; ++q)
                        for (int n = 0; n < nn; ++n) {
                            size_t t = ((size_t)d * G + q) * nn + n;
                            double SI = dJdI[t] + wsp[n] / (c * dt) * lam_next[t];
                            src[t] = (SI + sig[(size_t)(n / np) * G + q] * g->w[d] * tau[n]) / wsp[n];
                        }
                if (orc_adjoint_sweep(g, sigt, src, NULL, NULL, lam, NULL)) { rc = -1; break; }
                double num = 0.0, den = 0.0;
                for (int n = 0; n < nn; ++n) {
                    double s = ST[n];
                    for (int q = 0; q < G; ++q) {
                        double ls = 0.0;
                        for (int d = 0; d < nd; ++d) ls += lam[((size_t)d * G + q) * nn + n];
                        s += wsp[n] * sig[(size_t)(n / np) * G + q] * dE[(size_t)n * G + q] * ls;
                    }
                    tau_new[n] = s / D[n];
                    num += (tau_new[n] - tau[n]) * (tau_new[n] - tau[n]);
                    den += tau_new[n] * tau_new[n];
                }
                memcpy(tau, tau_new, sizeof(double) * nn);
                ++iters;
                if (num <= 1e-30 * den || den == 0.0) break;
            }
            if (rc) break;
            /* lam consistent with the final tau */
            for (int d = 0; d < nd; ++d)
                for (int q = 0; q < G; ++q)
                    for (int n = 0; n < nn; ++n) {
                        size_t t = ((size_t)d * G + q) * nn + n;
                        double SI = dJdI[t] + wsp[n] / (c * dt) * lam_next[t];
                        src[t] = (SI + sig[(size_t)(n / np) * G + q] * g->w[d] * tau[n]) / wsp[n];
                    }
            if (orc_adjoint_sweep(g, sigt, src, emis, psi, lam, dsig)) { rc = -1; break; }
            /* G = lam^T dR/dsigma, gradient contributions, S^T for step k-1 */
            for (int cc = 0; cc < nc; ++cc)
                for (int q = 0; q < G; ++q) {
                    double v = -dsig[(size_t)cc * G + q];
                    for (int l = 0; l < np; ++l) {
                        int n = np * cc + l;
                        v -= tau[n] * (phi[(size_t)n * G + q] - 4.0 * M_PI * emis[(size_t)n * G + q]);
                    }
                    Gs[(size_t)cc * G + q] = v;
                }
            for (int cc = 0; cc < nc; ++cc) {
                int r = mt->region[cc];
                double Tc = 0.0;
                for (int l = 0; l < np; ++l) Tc += Tp[np * cc + l];
                Tc /= np;
                for (int q = 0; q < G; ++q) {
                    double s = sig[(size_t)cc * G + q];
                    int free_ = mt->model == 0 || (s > mt->clip_lo && s < mt->clip_hi);
                    if (free_) grad_s0[r] -= s * Gs[(size_t)cc * G + q];
                }
                for (int l = 0; l < np; ++l) {
                    int n = np * cc + l;
                    grad_cv[r] -= tau[n] * cvn[n] * (T[n] - Tp[n]) / dt;
                    double sT = cvn[n] / dt * tau[n];
                    if (mt->model == 1)
                        for (int q = 0; q < G; ++q) {
                            double s = sig[(size_t)cc * G + q];
                            if (s > mt->clip_lo && s < mt->clip_hi)
                                sT -= (-3.0 * s / (np * Tc)) * Gs[(size_t)cc * G + q];
                        }
                    ST_prev[n] = sT;
                }
            }
            memcpy(ST, ST_prev, sizeof(double) * nn);
            memcpy(lam_next, lam, sizeof(double) * npsi);
        }
        if (objective == 1 && rc == ORC_OK) {   /* direct dependence of J on c_v */
            const double *TN = ck_T + (size_t)nn * N;
            for (int cc = 0; cc < nc; ++cc)
                for (int l = 0; l < np; ++l) {
                    int n = np * cc + l;
                    grad_cv[mt->region[cc]] += wsp[n] * cvn[n] * TN[n];
                }
        }
        if (adj_iters) *adj_iters = iters;
        free(lam); free(lam_next); free(src); free(sigt); free(tau); free(ST); free(ST_prev); free(emis); free(dE);
        free(phi); free(D); free(Gs); free(dsig); free(bg); free(rg); free(tau_new);
    }
done:
    free(ck_psi); free(ck_T); free(ck_sig); free(E); free(F); free(cvn); free(wsp); free(dJdI);
    return rc;
}

/* J alone (forward only), for finite differences: objective 0 the
   time-integrated outflow through x+, 1 the final material energy */
int orc_objective(const orc_geom *g, const orc_mat *mt, const orc_bc *bc, const orc_opts *op, double dt, int n_steps,
                  int objective, const double *psi0, const double *T0, double *J_out)
{
    int nn = nnode(g), np = npc(g), G = g->G, nc = ncell(g), nd = g->nang, dim = g->dim, nx = g->nx;
    size_t npsi = (size_t)nd * G * nn;
    if (objective != 0 && objective != 1) return -2;
    double *psi = malloc(sizeof(double) * npsi), *T = malloc(sizeof(double) * nn);
    double *E = malloc(sizeof(double) * nn), *F = calloc((size_t)nn * dim, sizeof(double));
    memcpy(psi, psi0, sizeof(double) * npsi);
    memcpy(T, T0, sizeof(double) * nn);
    for (int n = 0; n < nn; ++n) E[n] = g->a * pow(T0[n], 4);
    double J = 0.0;
    int rc = ORC_OK;
    for (int k = 1; k <= n_steps && rc == ORC_OK; ++k) {
        orc_stats st;
        rc = orc_step(g, mt, bc, op, dt, psi, T, E, F, &st);
        for (int d = 0; d < nd && objective == 0; ++d) {
            double mu = om_ax(g, d, 0);
            if (mu <= 0.0) continue;
            for (int q = 0; q < G; ++q)
                for (int cc = 0; cc < nc; ++cc) {
                    int i = cc % nx, j = cc / nx;
                    if (i != nx - 1) continue;
                    for (int l = 0; l < np; ++l)
                        if (node_on_face(l, 0, 1))
                            J += dt * g->w[d] * mu * face_weight(g, i, j, 0) * psi[((size_t)d * G + q) * nn + np * cc + l];
                }
        }
    }
    if (objective == 1) {
        double *cvn = malloc(sizeof(double) * nn);
        nodal_cv(g, mt, cvn);
        for (int cc = 0; cc < nc; ++cc)
            for (int l = 0; l < np; ++l) J += vol_weight(g, cc % nx, cc / nx) * cvn[np * cc + l] * T[np * cc + l];
        free(cvn);
    }
    *J_out = J;
    free(psi); free(T); free(E); free(F);
    return rc;
}

/* ======================================================================== */
/* Unstructured quadrilateral meshes: the lumped bilinear DG sweep of       */
/* Eq. dgsn_transport on general convex quadrilaterals (the paper's refined */
/* meshes use trapezoidal corner cells), cells taken in a dependency order  */
/* per direction.                                                           */
/*                                                                          */
/* Mesh: nv vertices xy[v][2]; nc cells cv[c][4] listed counter-clockwise.  */
/* Node n = 4 c + l is the cell's l-th vertex.  The bilinear map from the   */
/* reference square (vertices (0,0), (1,0), (1,1), (0,1)) gives at vertex m */
/* the Jacobian J_m; the trapezoid (vertex) quadrature gives the lumped     */
/* weight w_m = det J_m / 4 and grad phi_l(x_m) = J_m^-T grad_ref phi_l.    */
/* Edge e joins local vertices e and e+1 (mod 4) with outward normal times  */
/* length nL_e; each endpoint gets half of it (trapezoid).  Local system    */
/*   A_lm = sigt w_l delta_lm - w_m Omega.grad(phi_l)(x_m)                 */
/*        + delta_lm sum_{edges e of l, Omega.nL_e > 0} Omega.nL_e / 2      */
/*   b_l  = w_l q_l - sum_{edges e of l, Omega.nL_e < 0} Omega.nL_e/2 I_up  */
/* I_up the neighbour's node at the same vertex, or the inflow of the       */
/* boundary node.  Boundary edges are numbered in (cell, edge) order; the   */
/* boundary node 2 k + j is the j-th endpoint of boundary edge k.           */
/* ======================================================================== */

typedef struct {
    int nv, nc;
    const double *xy;   /* [nv][2] */
    const int *cv;      /* [nc][4] counter-clockwise */
    int nang;
    const double *om;   /* [nang][3] */
    const double *w;
    int G;
} orc_qgeom;

typedef struct { int a, b, c, e; } orc_qedge;

static int qedge_cmp(const void *x, const void *y)
{
    const orc_qedge *p = x, *q = y;
    if (p->a != q->a) return p->a < q->a ? -1 : 1;
    if (p->b != q->b) return p->b < q->b ? -1 : 1;
    if (p->c != q->c) return p->c < q->c ? -1 : 1;
    return p->e - q->e;
}

/* nb[4c+e] = neighbour cell across edge e (-1 on the boundary); bedge[4c+e] = boundary edge index or -1 */
static int qmesh_connect(const orc_qgeom *q, int *nb, int *bedge)
{
    int ne = 4 * q->nc, nbnd = 0;
    orc_qedge *E = malloc(sizeof(orc_qedge) * ne);
    for (int c = 0; c < q->nc; ++c)
        for (int e = 0; e < 4; ++e) {
            int v0 = q->cv[4 * c + e], v1 = q->cv[4 * c + (e + 1) % 4];
            E[4 * c + e] = (orc_qedge){v0 < v1 ? v0 : v1, v0 < v1 ? v1 : v0, c, e};
            nb[4 * c + e] = -1;
        }
    qsort(E, ne, sizeof(orc_qedge), qedge_cmp);
    for (int k = 0; k < ne; ++k) {
        if (k + 1 < ne && E[k].a == E[k + 1].a && E[k].b == E[k + 1].b) {
            if (k + 2 < ne && E[k + 2].a == E[k].a && E[k + 2].b == E[k].b) { free(E); return -1; }  /* non-manifold */
            nb[4 * E[k].c + E[k].e] = E[k + 1].c;
            nb[4 * E[k + 1].c + E[k + 1].e] = E[k].c;
            ++k;
        }
    }
    free(E);
    for (int c = 0; c < q->nc; ++c)
        for (int e = 0; e < 4; ++e) bedge[4 * c + e] = nb[4 * c + e] < 0 ? nbnd++ : -1;
    return nbnd;
}

int orc_qmesh_nbnodes(const orc_qgeom *q)
{
    int *nb = malloc(sizeof(int) * 4 * q->nc), *be = malloc(sizeof(int) * 4 * q->nc);
    int n = qmesh_connect(q, nb, be);
    free(nb); free(be);
    return n < 0 ? n : 2 * n;
}

/* reference gradient of phi_l at reference vertex m (vertices (0,0),(1,0),(1,1),(0,1)) */
static void qref_grad(int l, int m, double g[2])
{
    static const double V[4][2] = {{0, 0}, {1, 0}, {1, 1}, {0, 1}};
    double xi = V[m][0], eta = V[m][1];
    switch (l) {
        case 0: g[0] = -(1 - eta); g[1] = -(1 - xi); break;
        case 1: g[0] = 1 - eta; g[1] = -xi; break;
        case 2: g[0] = eta; g[1] = xi; break;
        default: g[0] = -eta; g[1] = 1 - xi; break;
    }
}

/* per cell: w[m], G[l][m][2] = grad phi_l(x_m), nL[e][2]; returns -1 if not positively oriented */
static int qcell_terms(const orc_qgeom *q, int c, double w[4], double G[4][4][2], double nL[4][2])
{
    double X[4][2];
    for (int l = 0; l < 4; ++l) { X[l][0] = q->xy[2 * q->cv[4 * c + l]]; X[l][1] = q->xy[2 * q->cv[4 * c + l] + 1]; }
    for (int m = 0; m < 4; ++m) {
        double J[2][2] = {{0, 0}, {0, 0}};   /* J[i][k] = d x_i / d ref_k */
        for (int l = 0; l < 4; ++l) {
            double g[2];
            qref_grad(l, m, g);
            for (int i = 0; i < 2; ++i) for (int k = 0; k < 2; ++k) J[i][k] += X[l][i] * g[k];
        }
        double det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
        if (!(det > 0.0)) return -1;
        w[m] = det / 4.0;
        for (int l = 0; l < 4; ++l) {
            double g[2];
            qref_grad(l, m, g);
            /* solve J^T y = g */
            G[l][m][0] = (J[1][1] * g[0] - J[1][0] * g[1]) / det;
            G[l][m][1] = (-J[0][1] * g[0] + J[0][0] * g[1]) / det;
        }
    }
    for (int e = 0; e < 4; ++e) {
        int b = (e + 1) % 4;
        nL[e][0] = X[b][1] - X[e][1];
        nL[e][1] = -(X[b][0] - X[e][0]);
    }
    return 0;
}

int orc_qsweep(const orc_qgeom *q, const double *sig_t, const double *q_iso, const double *psi_prev,
               double inv_c_dt, const double *inflow, double *psi)
{
    int nc = q->nc, G = q->G, nn = 4 * nc;
    int *nb = malloc(sizeof(int) * 4 * nc), *be = malloc(sizeof(int) * 4 * nc);
    int nbe = qmesh_connect(q, nb, be), NB = 2 * nbe;
    int *indeg = malloc(sizeof(int) * nc), *order = malloc(sizeof(int) * nc);
    int status = nbe < 0 ? -1 : ORC_OK;
    for (int d = 0; d < q->nang && status == ORC_OK; ++d) {
        double mu = q->om[3 * d], eta = q->om[3 * d + 1];
        /* dependency order (Kahn): a cell waits for the neighbours across its inflow edges */
        for (int c = 0; c < nc; ++c) indeg[c] = 0;
        for (int c = 0; c < nc && status == ORC_OK; ++c) {
            double w[4], Gr[4][4][2], nL[4][2];
            if (qcell_terms(q, c, w, Gr, nL)) { status = -2; break; }
            for (int e = 0; e < 4; ++e)
                if (nb[4 * c + e] >= 0 && mu * nL[e][0] + eta * nL[e][1] < 0.0) indeg[c]++;
        }
        int head = 0, tail = 0;
        for (int c = 0; c < nc; ++c) if (indeg[c] == 0) order[tail++] = c;
        while (head < tail && status == ORC_OK) {
            int c = order[head++];
            double w[4], Gr[4][4][2], nL[4][2];
            qcell_terms(q, c, w, Gr, nL);
            for (int k = 0; k < G; ++k) {
                const double *pp = psi_prev ? psi_prev + ((size_t)d * G + k) * nn : NULL;
                double *out = psi + ((size_t)d * G + k) * nn;
                const double *inf = inflow ? inflow + ((size_t)d * G + k) * NB : NULL;
                double A[16], b[4], x[4], st = sig_t[(size_t)c * G + k];
                for (int l = 0; l < 4; ++l) {
                    double ql = q_iso[(size_t)(4 * c + l) * G + k];
                    if (pp) ql += inv_c_dt * pp[4 * c + l];
                    b[l] = w[l] * ql;
                    for (int m = 0; m < 4; ++m)
                        A[4 * l + m] = (l == m ? st * w[l] : 0.0) - w[m] * (mu * Gr[l][m][0] + eta * Gr[l][m][1]);
                }
                for (int e = 0; e < 4; ++e) {
                    double on = 0.5 * (mu * nL[e][0] + eta * nL[e][1]);
                    for (int j = 0; j < 2; ++j) {
                        int l = (e + j) % 4;
                        if (on > 0.0) { A[4 * l + l] += on; continue; }
                        /* a face parallel to the direction carries nothing (and its
                           neighbour is not upwind, so it may not be swept yet) */
                        if (on == 0.0) continue;
                        double up = 0.0;
                        int n2 = nb[4 * c + e];
                        if (n2 >= 0) {
                            int v = q->cv[4 * c + l], l2 = 0;
                            while (l2 < 4 && q->cv[4 * n2 + l2] != v) ++l2;
                            up = out[4 * n2 + l2];
                        } else if (inf) {
                            up = inf[2 * be[4 * c + e] + j];
                        }
                        b[l] -= on * up;
                    }
                }
                if (lu_solve(4, A, b, x)) { status = -1; break; }
                for (int l = 0; l < 4; ++l) out[4 * c + l] = x[l];
            }
            for (int e = 0; e < 4; ++e) {
                int n2 = nb[4 * c + e];
                if (n2 >= 0 && mu * nL[e][0] + eta * nL[e][1] > 0.0 && --indeg[n2] == 0) order[tail++] = n2;
            }
        }
        if (status == ORC_OK && tail != nc) status = -3;   /* a dependency cycle */
    }
    free(nb); free(be); free(indeg); free(order);
    return status;
}

/* ------------------------------------------------------------------------ */
/* One backward-Euler step of the unaccelerated scheme of Algorithm 1 (no   */
/* low-order solve: every outer iteration sweeps with the emission source   */
/* at the current temperature iterate and solves the pointwise energy       */
/* balance cv T/dt + sigma_P a c T^4 = sum_g sigma_g phi_g + cv Tstar/dt)   */
/* on an unstructured quadrilateral mesh, with a fixed boundary inflow.     */
/* The opacity is taken once per step at the start-of-step temperature     */
/* (cell mean of the nodal values, as on the rectilinear mesh); node n of   */
/* cell n/4 has that cell's c_v.  psi: in I*, out I; T in/out; E out       */
/* (sum_d w I / c).  Same outer test and caps as orc_step.                 */
/* ------------------------------------------------------------------------ */
int orc_qstep_unacc(const orc_qgeom *q, const double *nu, double a, double c, const orc_mat *m,
                    const double *inflow, const orc_opts *op, double dt, double *psi, double *T, double *E,
                    orc_stats *st)
{
    int nc = q->nc, G = q->G, nn = 4 * nc, nang = q->nang;
    size_t npsi = (size_t)nang * G * nn;
    orc_geom g;   /* only what orc_opacity reads: nc cells of 4 nodes, the groups */
    memset(&g, 0, sizeof g);
    g.dim = 2; g.nx = nc; g.ny = 1; g.G = G; g.nu = nu; g.a = a; g.c = c;
    memset(st, 0, sizeof *st);
    double *sig = malloc(sizeof(double) * nc * G), *sigt = malloc(sizeof(double) * nc * G);
    double *qs = malloc(sizeof(double) * nn * G), *prev = malloc(sizeof(double) * npsi);
    double *out = calloc(npsi, sizeof(double)), *Tstar = malloc(sizeof(double) * nn);
    double *Tl = malloc(sizeof(double) * nn), *El = malloc(sizeof(double) * nn);
    double *Tn = malloc(sizeof(double) * nn), *En = malloc(sizeof(double) * nn);
    double *sphi = malloc(sizeof(double) * nn), *cvn = malloc(sizeof(double) * nn);
    orc_opacity(&g, m, T, sig);
    for (size_t k = 0; k < (size_t)nc * G; ++k) sigt[k] = sig[k] + 1.0 / (c * dt);
    for (int n = 0; n < nn; ++n) cvn[n] = m->cv[m->region[n / 4]];
    memcpy(prev, psi, sizeof(double) * npsi);
    memcpy(Tstar, T, sizeof(double) * nn);
    memcpy(Tl, T, sizeof(double) * nn);
    /* first energy iterate: the intensity's own E* */
    memset(El, 0, sizeof(double) * nn);
    for (int d = 0; d < nang; ++d)
        for (int k = 0; k < G; ++k)
            for (int n = 0; n < nn; ++n) El[n] += q->w[d] * prev[((size_t)d * G + k) * nn + n] / c;
    double first = -1.0;
    int status = ORC_OK;
    for (int l = 1; l <= op->max_outer; ++l) {
#pragma omp parallel for schedule(static)
        for (int n = 0; n < nn; ++n) {
            double bg[G], rg[G];
            orc_spectra(G, nu, Tl[n], bg, rg);
            double B = a * c * pow(Tl[n], 4);
            for (int k = 0; k < G; ++k) qs[(size_t)n * G + k] = sig[(size_t)(n / 4) * G + k] * B * bg[k] / (4.0 * M_PI);
        }
        int r = orc_qsweep(q, sigt, qs, prev, 1.0 / (c * dt), inflow, out);
        if (r) { status = r; break; }
        st->outer++;
        memset(En, 0, sizeof(double) * nn);
        memset(sphi, 0, sizeof(double) * nn);
        for (int d = 0; d < nang; ++d)
            for (int k = 0; k < G; ++k)
                for (int n = 0; n < nn; ++n) {
                    double wI = q->w[d] * out[((size_t)d * G + k) * nn + n];
                    En[n] += wI / c;
                    sphi[n] += sig[(size_t)(n / 4) * G + k] * wI;
                }
        for (int n = 0; n < nn && status == ORC_OK; ++n) {
            double bg[G], rg[G];
            orc_spectra(G, nu, Tl[n], bg, rg);
            double sb = 0, sbs = 0;
            for (int k = 0; k < G; ++k) { sb += bg[k]; sbs += bg[k] * sig[(size_t)(n / 4) * G + k]; }
            double rhs = sphi[n] + cvn[n] * Tstar[n] / dt;
            Tn[n] = Tl[n];
            int it = orc_energy_solve(cvn[n] / dt, (sbs / sb) * a * c, rhs, Tl[n], op->elim_rtol, op->max_elim, &Tn[n]);
            if (floor_temperature(op->T_floor, it, &Tn[n])) { status = ORC_E_NONPHYSICAL; break; }
            if (it > st->elim_max) st->elim_max = it;
            if (it >= op->max_elim) st->hit_max = 1;
        }
        double diff = 0.0;
        for (int n = 0; n < nn; ++n) diff += (Tn[n] - Tl[n]) * (Tn[n] - Tl[n]) + (En[n] - El[n]) * (En[n] - El[n]);
        diff = sqrt(diff);
        memcpy(Tl, Tn, sizeof(double) * nn);
        memcpy(El, En, sizeof(double) * nn);
        if (status) break;
        if (l == 1) first = diff;
        if (diff == 0.0 || (l > 1 && diff < op->eps_outer * first)) break;
        if (l == op->max_outer) st->hit_max = 1;
    }
    memcpy(T, Tl, sizeof(double) * nn);
    memcpy(E, El, sizeof(double) * nn);
    memcpy(psi, out, sizeof(double) * npsi);
    free(sig); free(sigt); free(qs); free(prev); free(out); free(Tstar); free(Tl); free(El); free(Tn); free(En);
    free(sphi); free(cvn);
    return status;
}
