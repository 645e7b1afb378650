// FP64 closure post-pass and low-order (LO) solve of the SM method (gfx950).
//
// Closures (Sec. 2 gray collapse; Sec. 4 consistent and independent LDG
// sources).  Per node, from the HO moments of the last sweep:
//   sigma_E = sum_g sigma_g phi_g / phi   (sigma_P where phi = 0),
//   sigma_F, sigma_P from the Rosseland / Planck fractions at the outer
//   iterate's temperature (computed by the source kernel),
//   qE = w E*/dt - 2 sum_bfaces fw F_in + R0_cons,
//   qF = w F*/(c dt) - sum_bfaces fw P_in (consistent) + R1,
// where, with n = +e_ax from the lower cell K1 to the upper cell K2 and the
// LDG upwinding s = +1 (upwind vector (1,1)),
//   R0_cons = fw [u] ( (s/2)[F.n] - [beta]/2 )                  (interior)
//           - fw ( J+ - c alpha E_HO - F_in )                    (boundary)
//   R1      = w (sigma_F F - sum_g sigma_g F_g) + sum_m w (T_m grad phi)(x_m)
//           - fw [v] . {T n}                                     (both schemes)
//           - fw [v] . ( [(Pi+ - Pi-) n]/2 + (c/6) s n [E] )     (consistent)
//           + fw ( (c/3) n E_HO - Pi+ n )                         (consistent, boundary)
// T = Pi - (phi/3) I, beta = sum w (|Omega.n| - alpha) I, Pi = sum w Omega Omega I.
// Half-range sums come from the quadrant moments of the sweep.
//
// Low-order Newton with nonlinear elimination of T (Sec. 5), lumped:
//   S = (c/3) D M_F^-1 D^T + M_E + P - diag(dB dBt^-1 M_a)  (SPD),
//   S E = qE + B(T0) - D M_F^-1 qF + dB dBt^-1 (qT - Bt(T0)),
//   F = M_F^-1 (qF + (c/3) D^T E),
//   cv T/dt + sigma_P a c T^4 = c sigma_E E + cv T*/dt at every node,
// with preconditioned CG on S (Jacobi, or the aggregation multigrid of
// mg_precond.inc); D (divergence) and P (penalty, kappa = alpha/2) are
// geometric and assembled once on the host in CSR form, and the CG applies S
// in stencil form.  One host wait per Newton iteration when a block of CG
// iterations suffices.
#include <cmath>
#include <cstring>

#include "lo.h"

namespace smrt {

// ---------------------------------------------------------------------------
// Closure kernels
// ---------------------------------------------------------------------------
struct NodeMom2D {
    double phi, F[2], Pi[2][2];     // full range
    double Fp[2][2];                // Fp[ax][a]: sum over Omega_ax > 0 of w Omega_a I
    double Pp[2][2];                // Pp[ax][a]: sum over Omega_ax > 0 of w Omega_a Omega_ax I
    double sphi, sF[2];
};

__device__ inline NodeMom2D load_mom2d(const double *mom, int nn, int n) {
    double m[27];
#pragma unroll
    for (int k = 0; k < 27; ++k) m[k] = mom[(int64_t)k * nn + n];
    NodeMom2D r;
    r.phi = m[0] + m[6] + m[12] + m[18];
    r.F[0] = m[1] + m[7] + m[13] + m[19];
    r.F[1] = m[2] + m[8] + m[14] + m[20];
    r.Pi[0][0] = m[3] + m[9] + m[15] + m[21];
    r.Pi[0][1] = r.Pi[1][0] = m[4] + m[10] + m[16] + m[22];
    r.Pi[1][1] = m[5] + m[11] + m[17] + m[23];
    // mu > 0: quadrants 0, 3; eta > 0: quadrants 0, 1
    r.Fp[0][0] = m[1] + m[19];
    r.Fp[0][1] = m[2] + m[20];
    r.Fp[1][0] = m[1] + m[7];
    r.Fp[1][1] = m[2] + m[8];
    r.Pp[0][0] = m[3] + m[21];   // Pi_xx over mu > 0
    r.Pp[0][1] = m[4] + m[22];   // Pi_yx over mu > 0
    r.Pp[1][0] = m[4] + m[10];   // Pi_xy over eta > 0
    r.Pp[1][1] = m[5] + m[11];   // Pi_yy over eta > 0
    r.sphi = m[24];
    r.sF[0] = m[25];
    r.sF[1] = m[26];
    return r;
}

__device__ inline double Tten(const NodeMom2D &m, int a, int b) { return m.Pi[a][b] - (a == b ? m.phi / 3.0 : 0.0); }

__global__ void k_closures2d(ClosureArgs A) {
    const int nn = 4 * A.nx * A.ny;
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= nn || (A.gate && !*A.gate)) return;
    const int cell = n >> 2, l = n & 3, lx = l & 1, ly = l >> 1;
    const int i = cell % A.nx, j = cell / A.nx;
    const double hx = A.hx[i], hy = A.hy[j], w = 0.25 * hx * hy, c = A.c;
    const bool cons = A.scheme == 0;
    const NodeMom2D me = load_mom2d(A.mom, nn, n);
    const NodeMom2D px = load_mom2d(A.mom, nn, n ^ 1), py = load_mom2d(A.mom, nn, n ^ 2);
    const double E = me.phi / c;
    const double sigP = A.sigP[n], sigF = A.sigF[n];
    const double sigE = me.phi > 0.0 ? me.sphi / me.phi : sigP;
    double qE = w * A.Estar[n] / A.dt;
    double qF[2] = {w * A.Fstar[2 * n] / (c * A.dt), w * A.Fstar[2 * n + 1] / (c * A.dt)};
    double r0 = 0.0, r1[2];
    // multigroup additive correction and volume closure sum_m w (T_m grad phi_l)(x_m)
    const double sx = lx ? 1.0 : -1.0, sy = ly ? 1.0 : -1.0;
    for (int a = 0; a < 2; ++a) {
        r1[a] = w * (sigF * me.F[a] - me.sF[a]);
        r1[a] += w * (sx / hx) * (Tten(me, a, 0) + Tten(px, a, 0)) + w * (sy / hy) * (Tten(me, a, 1) + Tten(py, a, 1));
    }
    for (int ax = 0; ax < 2; ++ax) {
        const int sd = ax == 0 ? lx : ly;
        const double fw = ax == 0 ? 0.5 * hy : 0.5 * hx;
        const double sgn = sd ? 1.0 : -1.0;
        const double alpha = A.alpha[ax];
        int nbc = -1;
        if (ax == 0) { const int ii = i + (sd ? 1 : -1); if (ii >= 0 && ii < A.nx) nbc = ii + A.nx * j; }
        else { const int jj = j + (sd ? 1 : -1); if (jj >= 0 && jj < A.ny) nbc = i + A.nx * jj; }
        if (nbc >= 0) {
            const int nbn = 4 * nbc + (l ^ (ax == 0 ? 1 : 2));
            const NodeMom2D nb = load_mom2d(A.mom, nn, nbn);
            const NodeMom2D &m1 = sd ? me : nb;   // lower cell K1
            const NodeMom2D &m2 = sd ? nb : me;   // upper cell K2
            const double jmp = sgn;
            const double s = 1.0;
            if (cons) {
                const double b1 = (2.0 * m1.Fp[ax][ax] - m1.F[ax]) - alpha * m1.phi;
                const double b2 = (2.0 * m2.Fp[ax][ax] - m2.F[ax]) - alpha * m2.phi;
                r0 += fw * jmp * (0.5 * s * (m1.F[ax] - m2.F[ax]) - 0.5 * (b1 - b2));
            }
            for (int a = 0; a < 2; ++a) {
                double v = -0.5 * (Tten(m1, a, ax) + Tten(m2, a, ax));
                if (cons) {
                    const double d1 = 2.0 * m1.Pp[ax][a] - m1.Pi[a][ax];
                    const double d2 = 2.0 * m2.Pp[ax][a] - m2.Pi[a][ax];
                    v += -0.5 * (d1 - d2) - (c / 6.0) * s * (a == ax ? 1.0 : 0.0) * (m1.phi - m2.phi) / c;
                }
                r1[a] += fw * jmp * v;
            }
        } else {
            const int side = 2 * ax + sd;
            // incoming moments: isotropic side inflow, or per node (reflective side)
            double Fin, Pin2[2];
            if ((A.refl >> side) & 1) {
                const int b = side == 0 ? 2 * j + ly
                            : side == 1 ? 2 * A.ny + 2 * j + ly
                            : side == 2 ? 4 * A.ny + 2 * i + lx
                                        : 4 * A.ny + 2 * A.nx + 2 * i + lx;
                Fin = A.bmom[3 * b];
                Pin2[0] = A.bmom[3 * b + 1];
                Pin2[1] = A.bmom[3 * b + 2];
            } else {
                Fin = A.Itot[side] * A.S1[side];
                Pin2[0] = A.Itot[side] * A.S2[2 * side];
                Pin2[1] = A.Itot[side] * A.S2[2 * side + 1];
            }
            qE += -2.0 * fw * Fin;
            if (cons) {
                const double Jp = sd ? me.Fp[ax][ax] : -(me.F[ax] - me.Fp[ax][ax]);
                r0 += -fw * (Jp - c * alpha * E - Fin);
                for (int a = 0; a < 2; ++a) {
                    const double Pin = Pin2[a];
                    const double Ppn = sd ? me.Pp[ax][a] : -(me.Pi[a][ax] - me.Pp[ax][a]);
                    qF[a] += -fw * Pin;
                    r1[a] += fw * ((c / 3.0) * (a == ax ? sgn : 0.0) * E - Ppn);
                }
            }
        }
    }
    A.out[n] = sigE;
    A.out[(int64_t)nn + n] = sigF;
    A.out[(int64_t)2 * nn + n] = sigP;
    A.out[(int64_t)3 * nn + n] = qE + r0;
    A.out[(int64_t)4 * nn + n] = qF[0] + r1[0];
    A.out[(int64_t)5 * nn + n] = qF[1] + r1[1];
}

__global__ void k_closures1d(ClosureArgs A) {
    const int nn = 2 * A.nx;
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= nn) return;
    const int cell = n >> 1, l = n & 1;
    const double h = A.hx[cell], w = 0.5 * h, c = A.c;
    const bool cons = A.scheme == 0;
    struct M1 { double phi, F, Pi, Fp, Pp, sphi, sF; };
    auto get = [&](int k) {
        M1 r;
        double m[8];
        for (int q = 0; q < 8; ++q) m[q] = A.mom[(int64_t)q * nn + k];
        r.phi = m[0] + m[3]; r.F = m[1] + m[4]; r.Pi = m[2] + m[5]; r.Fp = m[1]; r.Pp = m[2];
        r.sphi = m[6]; r.sF = m[7];
        return r;
    };
    const M1 me = get(n), pr = get(n ^ 1);
    const double E = me.phi / c;
    const double sigP = A.sigP[n], sigF = A.sigF[n];
    const double sigE = me.phi > 0.0 ? me.sphi / me.phi : sigP;
    double qE = w * A.Estar[n] / A.dt, qF = w * A.Fstar[n] / (c * A.dt);
    const double s = 1.0, sl = l ? 1.0 : -1.0, alpha = A.alpha[0];
    double r0 = 0.0;
    double r1 = w * (sigF * me.F - me.sF) + w * (sl / h) * ((me.Pi - me.phi / 3.0) + (pr.Pi - pr.phi / 3.0));
    const int cc = cell + (l ? 1 : -1);
    if (cc >= 0 && cc < A.nx) {
        const M1 nb = get(2 * cc + (l ^ 1));
        const M1 &m1 = l ? me : nb;
        const M1 &m2 = l ? nb : me;
        if (cons) {
            const double b1 = (2.0 * m1.Fp - m1.F) - alpha * m1.phi, b2 = (2.0 * m2.Fp - m2.F) - alpha * m2.phi;
            r0 += sl * (0.5 * s * (m1.F - m2.F) - 0.5 * (b1 - b2));
        }
        double v = -0.5 * ((m1.Pi - m1.phi / 3.0) + (m2.Pi - m2.phi / 3.0));
        if (cons) v += -0.5 * ((2.0 * m1.Pp - m1.Pi) - (2.0 * m2.Pp - m2.Pi)) - (s / 6.0) * (m1.phi - m2.phi);
        r1 += sl * v;
    } else {
        const int side = l;
        const bool rf = (A.refl >> side) & 1;
        const double Fin = rf ? A.bmom[3 * side] : A.Itot[side] * A.S1[side];
        qE += -2.0 * Fin;
        if (cons) {
            const double Jp = l ? me.Fp : -(me.F - me.Fp);
            r0 += -(Jp - c * alpha * E - Fin);
            const double Pin = rf ? A.bmom[3 * side + 1] : A.Itot[side] * A.S2[2 * side];
            const double Ppn = l ? me.Pp : -(me.Pi - me.Pp);
            qF += -Pin;
            r1 += (c / 3.0) * sl * E - Ppn;
        }
    }
    A.out[n] = sigE;
    A.out[(int64_t)nn + n] = sigF;
    A.out[(int64_t)2 * nn + n] = sigP;
    A.out[(int64_t)3 * nn + n] = qE + r0;
    A.out[(int64_t)4 * nn + n] = qF + r1;
}

void run_closures(hipStream_t s, const ClosureArgs &a) {
    const int nn = a.dim == 2 ? 4 * a.nx * a.ny : 2 * a.nx;
    if (a.dim == 2) hipLaunchKernelGGL(k_closures2d, dim3((nn + 127) / 128), dim3(128), 0, s, a);
    else hipLaunchKernelGGL(k_closures1d, dim3((nn + 127) / 128), dim3(128), 0, s, a);
    SMRT_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// CSR assembly of the lumped LDG divergence D and penalty P (host).
// D row n, column (m, a) = m*dim + a, such that (D F)_n equals the lumped
//   - sum_m w grad(phi_n)(x_m) . F_m + interior-face upwinded fluxes.
// On a rectangle grad(phi_l)(x_m) is nonzero only for m = l and the partner
// node across the cell in that direction, with value +-1/h.
// ---------------------------------------------------------------------------
static void csr_from_rows(const std::vector<std::vector<std::pair<int, double>>> &rows, Csr &m, int ncols) {
    m.nrows = (int)rows.size();
    m.ncols = ncols;
    m.rowptr.assign(m.nrows + 1, 0);
    m.col.clear();
    m.val.clear();
    for (int r = 0; r < m.nrows; ++r) {
        // merge duplicate columns, keep column order of first appearance sorted
        std::vector<std::pair<int, double>> e = rows[r];
        std::sort(e.begin(), e.end(), [](auto &x, auto &y) { return x.first < y.first; });
        for (size_t k = 0; k < e.size(); ++k) {
            if (!m.col.empty() && (int)m.col.size() > m.rowptr[r] && m.col.back() == e[k].first) m.val.back() += e[k].second;
            else { m.col.push_back(e[k].first); m.val.push_back(e[k].second); }
        }
        m.rowptr[r + 1] = (int)m.col.size();
    }
}

void assemble_lo_operators(int dim, int nx, int ny, const std::vector<double> &xe, const std::vector<double> &ye,
                           const double alpha[2], double c, Csr &D, Csr &DT, Csr &P, std::vector<double> &wnode) {
    const int npc = dim == 2 ? 4 : 2;
    const int nyy = dim == 2 ? ny : 1;
    const int nn = nx * nyy * npc;
    std::vector<std::vector<std::pair<int, double>>> Dr(nn), Pr(nn);
    wnode.assign(nn, 0.0);
    for (int j = 0; j < nyy; ++j)
        for (int i = 0; i < nx; ++i) {
            const int cell = i + nx * j;
            const double hx = xe[i + 1] - xe[i], hy = dim == 2 ? ye[j + 1] - ye[j] : 1.0;
            const double w = hx * hy / npc;
            for (int l = 0; l < npc; ++l) {
                const int n = npc * cell + l;
                wnode[n] = w;
                const int lx = l & 1, ly = l >> 1;
                // volume: x derivative couples l and its x partner (same y level)
                const double sx = lx ? 1.0 : -1.0;
                Dr[n].push_back({n * dim + 0, -w * sx / hx});
                Dr[n].push_back({(npc * cell + (l ^ 1)) * dim + 0, -w * sx / hx});
                if (dim == 2) {
                    const double sy = ly ? 1.0 : -1.0;
                    Dr[n].push_back({n * dim + 1, -w * sy / hy});
                    Dr[n].push_back({(npc * cell + (l ^ 2)) * dim + 1, -w * sy / hy});
                }
                for (int ax = 0; ax < dim; ++ax) {
                    const int sd = ax == 0 ? lx : ly;
                    const double fw = dim == 1 ? 1.0 : (ax == 0 ? 0.5 * hy : 0.5 * hx);
                    int nbc = -1;
                    if (ax == 0) { const int ii = i + (sd ? 1 : -1); if (ii >= 0 && ii < nx) nbc = ii + nx * j; }
                    else { const int jj = j + (sd ? 1 : -1); if (jj >= 0 && jj < ny) nbc = i + nx * jj; }
                    const double cal = c * alpha[ax];
                    if (nbc < 0) {
                        Pr[n].push_back({n, fw * cal});
                        continue;
                    }
                    const int nbn = npc * nbc + (l ^ (ax == 0 ? 1 : 2));
                    // upwinding s = +1: the flux across the face is the lower cell's F.n
                    const int lower = sd ? n : nbn;
                    const double jmp = sd ? 1.0 : -1.0;
                    Dr[n].push_back({lower * dim + ax, fw * jmp});
                    Pr[n].push_back({n, 0.5 * fw * cal});
                    Pr[n].push_back({nbn, -0.5 * fw * cal});
                }
            }
        }
    csr_from_rows(Dr, D, nn * dim);
    csr_from_rows(Pr, P, nn);
    std::vector<std::vector<std::pair<int, double>>> Tr(nn * dim);
    for (int r = 0; r < nn; ++r)
        for (int k = D.rowptr[r]; k < D.rowptr[r + 1]; ++k) Tr[D.col[k]].push_back({r, D.val[k]});
    csr_from_rows(Tr, DT, nn);
}

// ---------------------------------------------------------------------------
// LO kernels
// ---------------------------------------------------------------------------
__device__ __forceinline__ void d_lo_outer_setup(int bid, int nn, int dim, double icdt, const double *wn, const double *sigF, const double *qF,
                                 double *MFinv, double *tmpF) {
    const int n = bid * 256 + threadIdx.x;
    if (n >= nn) return;
    const double mi = 1.0 / (wn[n] * (sigF[n] + icdt));
    MFinv[n] = mi;
    for (int a = 0; a < dim; ++a) tmpF[dim * n + a] = qF[(int64_t)a * nn + n] * mi;
}
__global__ void k_lo_outer_setup(int nn, int dim, double icdt, const double *wn, const double *sigF, const double *qF,
                                 double *MFinv, double *tmpF) { d_lo_outer_setup(blockIdx.x, nn, dim, icdt, wn, sigF, qF, MFinv, tmpF); }

// y = A x (CSR), optionally y = alpha A x + beta y
__device__ __forceinline__ void d_spmv(int bid, int nrows, const int *rp, const int *col, const double *val, const double *x, double *y) {
    const int r = bid * 256 + threadIdx.x;
    if (r >= nrows) return;
    double s = 0.0;
    for (int k = rp[r]; k < rp[r + 1]; ++k) s += val[k] * x[col[k]];
    y[r] = s;
}
__global__ void k_spmv(int nrows, const int *rp, const int *col, const double *val, const double *x, double *y) { d_spmv(blockIdx.x, nrows, rp, col, val, x, y); }

// dDD_n = (c/3) sum_k D_nk^2 MFinv(col node) + P_nn
__device__ __forceinline__ void d_jacobi_base(int bid, int nn, int dim, double c3, const int *drp, const int *dcol, const double *dval,
                              const int *prp, const int *pcol, const double *pval, const double *MFinv, double *base) {
    const int n = bid * 256 + threadIdx.x;
    if (n >= nn) return;
    double s = 0.0;
    for (int k = drp[n]; k < drp[n + 1]; ++k) s += dval[k] * dval[k] * MFinv[dcol[k] / dim];
    double p = 0.0;
    for (int k = prp[n]; k < prp[n + 1]; ++k)
        if (pcol[k] == n) p += pval[k];
    base[n] = c3 * s + p;
}
__global__ void k_jacobi_base(int nn, int dim, double c3, const int *drp, const int *dcol, const double *dval,
                              const int *prp, const int *pcol, const double *pval, const double *MFinv, double *base) { d_jacobi_base(blockIdx.x, nn, dim, c3, drp, dcol, dval, prp, pcol, pval, MFinv, base); }

// Newton linearisation at T0: diagE, rhs, Jacobi inverse
__device__ __forceinline__ void d_newton_prep(int bid, int nn, double a, double c, double dt, const double *wn, const double *cvn,
                              const double *T0, const double *Tstar, const double *sigE, const double *sigP,
                              const double *qE, const double *DqF, const double *jbase, double *diagE, double *rhs,
                              double *Minv, const double *E, double *Eold, double *Told) {
    const int n = bid * 256 + threadIdx.x;
    if (n >= nn) return;
    const double w = wn[n], t = T0[n];
    Told[n] = t;      // the iterate this Newton step starts from (for the stopping test)
    Eold[n] = E[n];
    const double dB = w * 4.0 * sigP[n] * a * c * t * t * t;
    const double dBt = w * cvn[n] / dt + dB;
    const double B0 = w * sigP[n] * a * c * t * t * t * t;
    const double Bt0 = w * cvn[n] * t / dt + B0;
    const double Ma = w * c * sigE[n];
    const double qT = w * cvn[n] * Tstar[n] / dt;
    const double de = w * c * (sigE[n] + 1.0 / (c * dt)) - dB * Ma / dBt;
    diagE[n] = de;
    rhs[n] = qE[n] + B0 - DqF[n] + dB / dBt * (qT - Bt0);
    Minv[n] = 1.0 / (jbase[n] + de);
}
__global__ void k_newton_prep(int nn, double a, double c, double dt, const double *wn, const double *cvn,
                              const double *T0, const double *Tstar, const double *sigE, const double *sigP,
                              const double *qE, const double *DqF, const double *jbase, double *diagE, double *rhs,
                              double *Minv, const double *E, double *Eold, double *Told) { d_newton_prep(blockIdx.x, nn, a, c, dt, wn, cvn, T0, Tstar, sigE, sigP, qE, DqF, jbase, diagE, rhs, Minv, E, Eold, Told); }

// tmpF = (c/3) MFinv * (D^T x)  (D^T rows are F dofs)
__global__ void k_dt_scaled(int nrows, int dim, double c3, const int *rp, const int *col, const double *val,
                            const double *x, const double *MFinv, double *tmpF) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrows) return;
    double s = 0.0;
    for (int k = rp[r]; k < rp[r + 1]; ++k) s += val[k] * x[col[k]];
    tmpF[r] = c3 * MFinv[r / dim] * s;
}

// y = D tmpF + P x + diagE x
__global__ void k_schur_rows(int nn, const int *drp, const int *dcol, const double *dval, const int *prp, const int *pcol,
                             const double *pval, const double *tmpF, const double *x, const double *diagE, double *y) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= nn) return;
    double s = 0.0;
    for (int k = drp[n]; k < drp[n + 1]; ++k) s += dval[k] * tmpF[dcol[k]];
    for (int k = prp[n]; k < prp[n + 1]; ++k) s += pval[k] * x[pcol[k]];
    y[n] = s + diagE[n] * x[n];
}

// The same two products as k_dt_scaled and k_schur_rows(_dot), computed from
// the mesh instead of the CSR arrays (the operators of assemble_lo_operators
// written as stencils: every entry follows from hx, hy, the local node and
// whether the face is interior), so an application reads only the vectors.
//   (D^T x)(m, a) = -(w/h_a) s_a(m) (x_m - x_{partner_a(m)})
//                   + [m on the cell's upper a-face, face interior] fw_a (x_m - x_{coincident node above})
//   (D f)_n = -(w/h_x) s_x (f(n,x) + f(n^1,x)) - (w/h_y) s_y (f(n,y) + f(n^2,y))
//             + sum over n's faces a: interior: fw_a jmp f(lower, a)
//   (P x)_n = sum over n's faces a: interior 0.5 fw_a c alpha_a (x_n - x_nb), boundary fw_a c alpha_a x_n

__device__ inline void lo_node(const LoGeom &g, int n, int &cell, int &l, int &i, int &j, double &hx, double &hy,
                               double &w) {
    const int npc = g.dim == 2 ? 4 : 2;
    cell = n / npc;
    l = n - npc * cell;
    i = cell % g.nx;
    j = cell / g.nx;
    hx = g.hx[i];
    hy = g.dim == 2 ? g.hy[j] : 1.0;
    w = hx * hy / npc;
}

__device__ __forceinline__ void d_dt_stencil(int bid, int nn, LoGeom g, double c3, const double *x, const double *MFinv, double *tmpF) {
    const int m = bid * 256 + threadIdx.x;
    if (m >= nn) return;
    int cell, l, i, j;
    double hx, hy, w;
    lo_node(g, m, cell, l, i, j, hx, hy, w);
    const int npc = g.dim == 2 ? 4 : 2;
    const double xm = x[m], sc = c3 * MFinv[m];
    {
        const int lx = l & 1;
        double v = -(w / hx) * (lx ? 1.0 : -1.0) * (xm - x[m ^ 1]);
        if (lx && i + 1 < g.nx) v += (g.dim == 2 ? 0.5 * hy : 1.0) * (xm - x[npc * (cell + 1) + (l ^ 1)]);
        tmpF[(int64_t)m * g.dim] = sc * v;
    }
    if (g.dim == 2) {
        const int ly = l >> 1;
        double v = -(w / hy) * (ly ? 1.0 : -1.0) * (xm - x[m ^ 2]);
        if (ly && j + 1 < g.ny) v += 0.5 * hx * (xm - x[npc * (cell + g.nx) + (l ^ 2)]);
        tmpF[(int64_t)m * 2 + 1] = sc * v;
    }
}
__global__ void k_dt_stencil(int nn, LoGeom g, double c3, const double *x, const double *MFinv, double *tmpF) { d_dt_stencil(blockIdx.x, nn, g, c3, x, MFinv, tmpF); }

__device__ __forceinline__ void d_schur_stencil_dot(int bid, int nn, LoGeom g, const double *tmpF, const double *x,
                                                           const double *diagE, double *y, double *part) {
    __shared__ double sh[256];
    const int n = bid * 256 + threadIdx.x;
    double v = 0.0;
    if (n < nn) {
        int cell, l, i, j;
        double hx, hy, w;
        lo_node(g, n, cell, l, i, j, hx, hy, w);
        const int npc = g.dim == 2 ? 4 : 2, dim = g.dim;
        const double xn = x[n];
        const int lx = l & 1;
        double s = -(w / hx) * (lx ? 1.0 : -1.0) * (tmpF[(int64_t)n * dim] + tmpF[(int64_t)(n ^ 1) * dim]);
        double pp = 0.0;
        {
            const double fw = dim == 2 ? 0.5 * hy : 1.0, cal = g.c * g.alpha[0];
            const int ii = i + (lx ? 1 : -1);
            if (ii >= 0 && ii < g.nx) {
                const int nbn = npc * (cell + (lx ? 1 : -1)) + (l ^ 1);
                s += fw * (lx ? tmpF[(int64_t)n * dim] : -tmpF[(int64_t)nbn * dim]);
                pp += 0.5 * fw * cal * (xn - x[nbn]);
            } else {
                pp += fw * cal * xn;
            }
        }
        if (dim == 2) {
            const int ly = l >> 1;
            s += -(w / hy) * (ly ? 1.0 : -1.0) * (tmpF[(int64_t)n * 2 + 1] + tmpF[(int64_t)(n ^ 2) * 2 + 1]);
            const double fw = 0.5 * hx, cal = g.c * g.alpha[1];
            const int jj = j + (ly ? 1 : -1);
            if (jj >= 0 && jj < g.ny) {
                const int nbn = npc * (cell + (ly ? g.nx : -g.nx)) + (l ^ 2);
                s += fw * (ly ? tmpF[(int64_t)n * 2 + 1] : -tmpF[(int64_t)nbn * 2 + 1]);
                pp += 0.5 * fw * cal * (xn - x[nbn]);
            } else {
                pp += fw * cal * xn;
            }
        }
        const double yn = s + pp + diagE[n] * xn;
        y[n] = yn;
        v = xn * yn;
    }
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0 && part) part[bid] = sh[0];
}
__global__ void __launch_bounds__(256) k_schur_stencil_dot(int nn, LoGeom g, const double *tmpF, const double *x,
                                                           const double *diagE, double *y, double *part) { d_schur_stencil_dot(blockIdx.x, nn, g, tmpF, x, diagE, y, part); }

// S x fused with the block partials of x . (S x) (one partial per 256-row block)
__global__ void __launch_bounds__(256) k_schur_rows_dot(int nn, const int *drp, const int *dcol, const double *dval,
                                                        const int *prp, const int *pcol, const double *pval,
                                                        const double *tmpF, const double *x, const double *diagE,
                                                        double *y, double *part) {
    __shared__ double sh[256];
    const int n = blockIdx.x * 256 + threadIdx.x;
    double v = 0.0;
    if (n < nn) {
        double s = 0.0;
        for (int k = drp[n]; k < drp[n + 1]; ++k) s += dval[k] * tmpF[dcol[k]];
        for (int k = prp[n]; k < prp[n + 1]; ++k) s += pval[k] * x[pcol[k]];
        s += diagE[n] * x[n];
        y[n] = s;
        v = x[n] * s;
    }
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// Fixed-order sum of nb block partials (stride apart; a second sequence at +1
// when two) by a 256-thread block: thread k sums k, k+256, .., then a tree.
// Every block that calls it on the same partials gets the same bits.
__device__ void block_sum_partials(int nb, int stride, bool two, const double *part, double (*sh)[256], double &a,
                                   double &b) {
    double x = 0.0, y = 0.0;
    for (int k = threadIdx.x; k < nb; k += 256) {
        x += part[stride * k];
        if (two) y += part[stride * k + 1];
    }
    sh[0][threadIdx.x] = x;
    sh[1][threadIdx.x] = y;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + k];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + k];
        }
        __syncthreads();
    }
    a = sh[0][0];
    b = sh[1][0];
    __syncthreads();   // sh may be reused by the caller
}

// CG scalar slots: 0 rz, 2 rr, 3 rz_new, 4 |b|^2, 8 stop flag (1: converged,
// 2: iteration cap, 3: converged or capped before the first iteration),
// 9 iterations done, 10 tolerance on rr, 11 iteration cap.
// Once the stop flag is set the update kernels leave x, r, z, p unchanged, so
// the host checks convergence only every few iterations.
// CG update x += al p, r -= al Ap, z = M^-1 r (al = rz / pAp, pAp summed here from
// the block partials apart of p.Ap) fused with the block partials of r.z and r.r
__device__ __forceinline__ void d_cg_xr_dot(int bid, int n, int nbk, const double *sc, const double *apart,
                                                   const double *p, const double *Ap, double *x, double *r,
                                                   const double *Minv, double *z, double *part) {
    __shared__ double sh[2][256];
    const int i = bid * 256 + threadIdx.x;
    const bool frozen = sc[8] != 0.0;
    double pAp = 0.0, unused;
    block_sum_partials(nbk, 1, false, apart, sh, pAp, unused);
    double rz = 0.0, rr = 0.0;
    if (i < n) {
        double ri = r[i];
        if (!frozen) {
            const double al = sc[0] / pAp;
            x[i] += al * p[i];
            ri -= al * Ap[i];
            r[i] = ri;
            z[i] = Minv[i] * ri;
        }
        rz = ri * z[i];
        rr = ri * ri;
    }
    sh[0][threadIdx.x] = rz;
    sh[1][threadIdx.x] = rr;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + k];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + k];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * bid] = sh[0][0];
        part[2 * bid + 1] = sh[1][0];
    }
}
__global__ void __launch_bounds__(256) k_cg_xr_dot(int n, int nbk, const double *sc, const double *apart,
                                                   const double *p, const double *Ap, double *x, double *r,
                                                   const double *Minv, double *z, double *part) { d_cg_xr_dot(blockIdx.x, n, nbk, sc, apart, p, Ap, x, r, Minv, z, part); }

// deterministic block reduction of sum_i a_i b_i (b == nullptr: sum a_i^2 of (a - c))
constexpr int RED_BLOCKS = 256, RED_THREADS = 256;
__device__ __forceinline__ void d_dot_partial(int bid, int n, const double *a, const double *b, const double *cdiff, double *part) {
    __shared__ double sh[RED_THREADS];
    double s = 0.0;
    for (int i = bid * RED_THREADS + threadIdx.x; i < n; i += RED_BLOCKS * RED_THREADS) {
        if (cdiff) { const double d = a[i] - cdiff[i]; s += d * d; }
        else s += a[i] * (b ? b[i] : a[i]);
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int k = RED_THREADS / 2; k > 0; k >>= 1) {
        if (threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[bid] = sh[0];
}
__global__ void k_dot_partial(int n, const double *a, const double *b, const double *cdiff, double *part) { d_dot_partial(blockIdx.x, n, a, b, cdiff, part); }
__device__ __forceinline__ void d_dot_finish(int bid, const double *part, double *out, int slot, int accumulate) {
    __shared__ double sh[RED_BLOCKS];
    sh[threadIdx.x] = part[threadIdx.x];
    __syncthreads();
    for (int k = RED_BLOCKS / 2; k > 0; k >>= 1) {
        if (threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[slot] = accumulate ? out[slot] + sh[0] : sh[0];
}
__global__ void k_dot_finish(const double *part, double *out, int slot, int accumulate) { d_dot_finish(blockIdx.x, part, out, slot, accumulate); }

// Several sums in one pass over the vectors (the CG start: b.b, r.z, r.r;
// the Newton iterate change: |T - T_old|^2 + |E - E_old|^2), as block
// partials part[j][block], then k_dot_finish_n adds each row in a fixed
// order into its scalar slot.
__device__ __forceinline__ void d_dot3_partial(int bid, int n, const double *b, const double *r, const double *z, double *part) {
    __shared__ double sh[3][RED_THREADS];
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int i = bid * RED_THREADS + threadIdx.x; i < n; i += RED_BLOCKS * RED_THREADS) {
        const double ri = r[i];
        s0 += b[i] * b[i];
        s1 += ri * z[i];
        s2 += ri * ri;
    }
    sh[0][threadIdx.x] = s0;
    sh[1][threadIdx.x] = s1;
    sh[2][threadIdx.x] = s2;
    __syncthreads();
    for (int k = RED_THREADS / 2; k > 0; k >>= 1) {
        if (threadIdx.x < k)
            for (int j = 0; j < 3; ++j) sh[j][threadIdx.x] += sh[j][threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int j = 0; j < 3; ++j) part[j * RED_BLOCKS + bid] = sh[j][0];
}
__global__ void k_dot3_partial(int n, const double *b, const double *r, const double *z, double *part) { d_dot3_partial(blockIdx.x, n, b, r, z, part); }
__device__ __forceinline__ void d_diff2_partial(int bid, int n, const double *T, const double *To, const double *E, const double *Eo,
                                double *part) {
    __shared__ double sh[RED_THREADS];
    double s = 0.0;
    for (int i = bid * RED_THREADS + threadIdx.x; i < n; i += RED_BLOCKS * RED_THREADS) {
        const double dT = T[i] - To[i], dE = E[i] - Eo[i];
        s += dT * dT + dE * dE;
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int k = RED_THREADS / 2; k > 0; k >>= 1) {
        if (threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[bid] = sh[0];
}
__global__ void k_diff2_partial(int n, const double *T, const double *To, const double *E, const double *Eo,
                                double *part) { d_diff2_partial(blockIdx.x, n, T, To, E, Eo, part); }
__device__ __forceinline__ void d_dot_finish_n(int bid, const double *part, double *out, int m, int slot0, int slot1, int slot2) {
    __shared__ double sh[RED_BLOCKS];
    const int slots[3] = {slot0, slot1, slot2};
    for (int j = 0; j < m; ++j) {
        sh[threadIdx.x] = part[j * RED_BLOCKS + threadIdx.x];
        __syncthreads();
        for (int k = RED_BLOCKS / 2; k > 0; k >>= 1) {
            if (threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[slots[j]] = sh[0];
        __syncthreads();
    }
}
__global__ void k_dot_finish_n(const double *part, double *out, int m, int slot0, int slot1, int slot2) { d_dot_finish_n(blockIdx.x, part, out, m, slot0, slot1, slot2); }

// CG vector updates with device-side scalars: sc[0]=rz, sc[1]=pAp, sc[2]=rr, sc[3]=rz_new
// p = z + (rz_new / rz) p, rz_new summed here from the r.z block partials
__device__ __forceinline__ void d_cg_p(int bid, int n, int nbk, const double *sc, const double *part, const double *z,
                                              double *p) {
    __shared__ double sh[2][256];
    if (sc[8] != 0.0) return;   // uniform over the grid
    double rzn, unused;
    block_sum_partials(nbk, 2, false, part, sh, rzn, unused);
    const int i = bid * 256 + threadIdx.x;
    if (i < n) p[i] = z[i] + (rzn / sc[0]) * p[i];
}
__global__ void __launch_bounds__(256) k_cg_p(int n, int nbk, const double *sc, const double *part, const double *z,
                                              double *p) { d_cg_p(blockIdx.x, n, nbk, sc, part, z, p); }
__device__ __forceinline__ void d_cg_init(int bid, int n, const double *b, const double *Ax, double *r, const double *Minv, double *z, double *p) {
    const int i = bid * 256 + threadIdx.x;
    if (i >= n) return;
    r[i] = b[i] - Ax[i];
    z[i] = Minv[i] * r[i];
    p[i] = z[i];
}
__global__ void k_cg_init(int n, const double *b, const double *Ax, double *r, const double *Minv, double *z, double *p) { d_cg_init(blockIdx.x, n, b, Ax, r, Minv, z, p); }
// one 256-thread block: (rz_new, rr) from the block partials, then the scalars
__device__ __forceinline__ void d_cg_step_end(int bid, int nbk, const double *part, double *sc) {
    __shared__ double sh[2][256];
    if (sc[8] != 0.0) return;   // uniform over the block
    double rzn, rr;
    block_sum_partials(nbk, 2, true, part, sh, rzn, rr);
    if (threadIdx.x != 0) return;
    sc[3] = rzn;
    sc[2] = rr;
    sc[0] = sc[3];
    sc[9] += 1.0;
    if (sc[2] <= sc[10]) sc[8] = 1.0;
    else if (sc[9] >= sc[11]) sc[8] = 2.0;
}
__global__ void __launch_bounds__(256) k_cg_step_end(int nbk, const double *part, double *sc) { d_cg_step_end(blockIdx.x, nbk, part, sc); }
// stopping threshold rtol^2 |b|^2 (|b|^2 in sc[4], 1 if b = 0) and the stop
// flag before the first iteration (already converged, or no iterations allowed)
__device__ __forceinline__ void d_cg_start(int bid, double *sc, double rtol, int maxit) {
    const double bb = sc[4];
    const double tol2 = rtol * rtol * (bb > 0 ? bb : 1.0);
    sc[8] = (!(sc[2] > tol2) || maxit <= 0) ? 3.0 : 0.0;
    sc[9] = 0.0;
    sc[10] = tol2;
    sc[11] = (double)maxit;
}
__global__ void k_cg_start(double *sc, double rtol, int maxit) { d_cg_start(blockIdx.x, sc, rtol, maxit); }

// F = MFinv (qF + (c/3) D^T E)  (qF rows [a][n], F node-major [n][a])
__device__ __forceinline__ void d_backsub(int bid, int nn, int dim, double c3, const int *rp, const int *col, const double *val, const double *E,
                          const double *qF, const double *MFinv, double *F) {
    const int r = bid * 256 + threadIdx.x;
    if (r >= nn * dim) return;
    double s = 0.0;
    for (int k = rp[r]; k < rp[r + 1]; ++k) s += val[k] * E[col[k]];
    const int n = r / dim, a = r % dim;
    F[r] = MFinv[n] * (qF[(int64_t)a * nn + n] + c3 * s);
}
__global__ void k_backsub(int nn, int dim, double c3, const int *rp, const int *col, const double *val, const double *E,
                          const double *qF, const double *MFinv, double *F) { d_backsub(blockIdx.x, nn, dim, c3, rp, col, val, E, qF, MFinv, F); }

// pointwise energy balance: cv T/dt + sigP a c T^4 = c sigE E + cv T*/dt
// (Newton safeguarded by bisection on [0, rhs dt/cv]; stop at |f| <= rtol |rhs|).
// T_floor > 0 floors the temperature (Sec. 6): T = max(root, T_floor), and
// T_floor where the balance has no positive root; T_floor = 0 leaves the root
// as it is and flags a node without one.
// flags: [0] a node without a positive root (no floor), [1] the largest
// iteration count, [2] a node that hit maxit; the count is reduced over the
// wave first, and a wave whose count is already stored skips its atomic.
__device__ __forceinline__ void d_eliminate(int bid, int nn, double a, double c, double dt, double rtol, int maxit, double T_floor,
                            const double *cvn, const double *sigE, const double *sigP, const double *E,
                            const double *Tstar, double *T, int *flags) {
    const int n = bid * 256 + threadIdx.x;
    int it = 0;
    bool bad = false, capped = false;
    if (n < nn) {
        const double cv_dt = cvn[n] / dt, k4 = sigP[n] * a * c;
        const double rhs = c * sigE[n] * E[n] + cv_dt * Tstar[n];
        if (!(rhs > 0.0)) {
            if (T_floor > 0.0) T[n] = T_floor;
            else bad = true;
        } else {
            double lo = 0.0, hi = rhs / cv_dt, t = T[n];
            if (!(t > lo && t < hi)) t = 0.5 * (lo + hi);
            for (; it < maxit; ++it) {
                const double f = cv_dt * t + k4 * t * t * t * t - rhs;
                if (fabs(f) <= rtol * fabs(rhs)) break;
                if (f > 0) hi = t; else lo = t;
                double tn = t - f / (cv_dt + 4.0 * k4 * t * t * t);
                if (!(tn > lo && tn < hi)) tn = 0.5 * (lo + hi);
                t = tn;
            }
            T[n] = T_floor > 0.0 ? fmax(t, T_floor) : t;
            capped = it == maxit;
        }
    }
    // wave maximum of the iteration count (every lane of the wave takes part)
    int m = it;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = max(m, __shfl_xor(m, off, 64));
    const bool any_bad = __builtin_amdgcn_ballot_w64(bad) != 0;
    const bool any_capped = __builtin_amdgcn_ballot_w64(capped) != 0;
    if ((threadIdx.x & 63) == 0) {
        if (any_bad) atomicOr(&flags[0], 1);
        // a count at or below the one already stored needs no atomic (most
        // waves, once a few have stored theirs): one address, thousands of waves
        if (m > __hip_atomic_load(&flags[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(&flags[1], m);
        if (any_capped) atomicOr(&flags[2], 1);
    }
}
__global__ void k_eliminate(int nn, double a, double c, double dt, double rtol, int maxit, double T_floor,
                            const double *cvn, const double *sigE, const double *sigP, const double *E,
                            const double *Tstar, double *T, int *flags) { d_eliminate(blockIdx.x, nn, a, c, dt, rtol, maxit, T_floor, cvn, sigE, sigP, E, Tstar, T, flags); }

__global__ void k_zero4(int *p) { p[threadIdx.x] = 0; }

void run_eliminate(hipStream_t s, int nn, double a, double c, double dt, double rtol, int maxit, double T_floor,
                   const double *cvn, const double *sigE, const double *sigP, const double *E, const double *Tstar,
                   double *T, int *flags) {
    hipLaunchKernelGGL(k_eliminate, dim3((nn + 255) / 256), dim3(256), 0, s, nn, a, c, dt, rtol, maxit, T_floor, cvn,
                       sigE, sigP, E, Tstar, T, flags);
}

// ---------------------------------------------------------------------------
// host driver of the LO solve
// ---------------------------------------------------------------------------
static inline int nb(int64_t n, int b = 256) { return (int)((n + b - 1) / b); }

void LoSolver::init(int dim_, int nx, int ny, const std::vector<double> &xe, const std::vector<double> &ye,
                    const double alpha[2], double c_, double a_) {
    dim = dim_;
    c = c_;
    a = a_;
    gnx = nx;
    gny = ny;
    gxe = xe;
    gye = ye;
    galpha[0] = alpha[0];
    galpha[1] = alpha[1];
    Csr D, DT, P;
    std::vector<double> wv;
    assemble_lo_operators(dim, nx, ny, xe, ye, alpha, c, D, DT, P, wv);
    nn = D.nrows;
    {
        std::vector<double> hx(nx), hy(dim == 2 ? ny : 1, 1.0);
        for (int i = 0; i < nx; ++i) hx[i] = xe[i + 1] - xe[i];
        if (dim == 2)
            for (int j = 0; j < ny; ++j) hy[j] = ye[j + 1] - ye[j];
        dhx.alloc(nx);
        dhy.alloc((int64_t)hy.size());
        SMRT_HIP(hipMemcpy(dhx.p, hx.data(), sizeof(double) * nx, hipMemcpyHostToDevice));
        SMRT_HIP(hipMemcpy(dhy.p, hy.data(), sizeof(double) * hy.size(), hipMemcpyHostToDevice));
    }
    dD.upload(D);
    dDT.upload(DT);
    dP.upload(P);
    wn.alloc(nn);
    SMRT_HIP(hipMemcpy(wn.p, wv.data(), sizeof(double) * nn, hipMemcpyHostToDevice));
    for (auto *v : {&MFinv, &DqF, &jbase, &diagE, &rhs, &Minv, &r, &z, &p, &Ap, &Eold, &Told}) v->alloc(nn);
    tmpF.alloc((int64_t)nn * dim);
    part.alloc(3 * RED_BLOCKS);
    sc.alloc(12);
    sc2.alloc(12);
    bpart.alloc(2 * (int64_t)((nn + 255) / 256));
    apart.alloc((int64_t)((nn + 255) / 256));
    flags.alloc(4);
}

// the same sum, skipped while *gate is 0
__global__ void k_dot_partial_g(const int *gate, int n, const double *a, const double *b, const double *cdiff,
                                double *part) {
    if (!*gate) return;
    d_dot_partial(blockIdx.x, n, a, b, cdiff, part);
}
__global__ void k_dot_finish_g(const int *gate, const double *part, double *out, int slot, int accumulate) {
    if (!*gate) return;
    d_dot_finish(blockIdx.x, part, out, slot, accumulate);
}
void LoSolver::dot_gated(hipStream_t s, const int *gate, const double *x, const double *y, const double *cdiff,
                         int slot, bool accumulate) {
    hipLaunchKernelGGL(k_dot_partial_g, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s, gate, nn, x, y, cdiff, part.p);
    hipLaunchKernelGGL(k_dot_finish_g, dim3(1), dim3(RED_BLOCKS), 0, s, gate, (const double *)part.p, sc.p, slot,
                       accumulate ? 1 : 0);
}

double LoSolver::dot(hipStream_t s, const double *x, const double *y, const double *cdiff, int slot, bool accumulate) {
    hipLaunchKernelGGL(k_dot_partial, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s, nn, x, y, cdiff, part.p);
    hipLaunchKernelGGL(k_dot_finish, dim3(1), dim3(RED_BLOCKS), 0, s, part.p, sc.p, slot, accumulate ? 1 : 0);
    return 0.0;
}

// Every small device-to-host read of the LO goes through the pinned buffer
// hbuf (slots 0-1 CG status, 2-3 elimination flags, 4 iterate change, 5 a
// fetched scalar, 6-7 the flags of a caller's elimination), never through
// pageable stack memory.
void LoSolver::ensure_hbuf() {
    if (!hbuf) SMRT_HIP(hipHostMalloc((void **)&hbuf, 8 * sizeof(double), hipHostMallocDefault));
}

double LoSolver::fetch(hipStream_t s, int slot) {
    ensure_hbuf();
    SMRT_HIP(hipMemcpyAsync(hbuf + 5, sc.p + slot, sizeof(double), hipMemcpyDeviceToHost, s));
    SMRT_HIP(hipStreamSynchronize(s));
    return hbuf[5];
}

void LoSolver::fetch_flags(hipStream_t s, int fl[4]) {
    ensure_hbuf();
    SMRT_HIP(hipMemcpyAsync(hbuf + 6, flags.p, 4 * sizeof(int), hipMemcpyDeviceToHost, s));
    SMRT_HIP(hipStreamSynchronize(s));
    std::memcpy(fl, hbuf + 6, 4 * sizeof(int));
}

LoGeom LoSolver::geom() const {
    LoGeom g{};
    g.dim = dim; g.nx = gnx; g.ny = dim == 2 ? gny : 1;
    g.hx = dhx.p; g.hy = dhy.p;
    g.c = c; g.alpha[0] = galpha[0]; g.alpha[1] = galpha[1];
    return g;
}

void LoSolver::schur(hipStream_t s, const double *x, double *y) {
    const LoGeom g = geom();
    hipLaunchKernelGGL(k_dt_stencil, dim3(nb(nn)), dim3(256), 0, s, nn, g, c / 3.0, x, MFinv.p, tmpF.p);
    hipLaunchKernelGGL(k_schur_stencil_dot, dim3(nb(nn)), dim3(256), 0, s, nn, g, tmpF.p, x, diagE.p, y,
                       (double *)nullptr);
}

// Queues the start of a PCG solve of S x = rhs (x holds the initial guess):
// the residual, the preconditioned residual, the scalars, the threshold and
// the initial convergence test (all on the device; a solve that starts
// converged runs frozen blocks and reports 0 iterations), then its first
// block of CG_CHECK iterations.  Nothing is waited for.
void LoSolver::pcg_begin(hipStream_t s, double *x, double rtol, int maxit) {
    schur(s, x, Ap.p);
    hipLaunchKernelGGL(k_cg_init, dim3(nb(nn)), dim3(256), 0, s, nn, rhs.p, Ap.p, r.p, Minv.p, z.p, p.p);
    if (precond == 1) mg_cg_init(s);               // z = M^-1 r, p = z by a V-cycle
    // |b|^2, rz, rr into slots 4, 0, 2
    hipLaunchKernelGGL(k_dot3_partial, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s, nn, rhs.p, r.p, z.p, part.p);
    hipLaunchKernelGGL(k_dot_finish_n, dim3(1), dim3(RED_BLOCKS), 0, s, part.p, sc.p, 3, 4, 0, 2);
    hipLaunchKernelGGL(k_cg_start, dim3(1), dim3(1), 0, s, sc.p, rtol, maxit);
    if (use_graphs && !graph_failed && (cg_exec == nullptr || cg_stream != s || cg_x != x || cg_precond != precond)) {
        // record CG_CHECK iterations once (kernels only) and replay them;
        // streams that cannot capture fall back to direct launches
        drop_graph();
        if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) == hipSuccess) {
            cg_block(s, x, CG_CHECK);
            hipGraph_t g = nullptr;
            if (hipStreamEndCapture(s, &g) == hipSuccess && g &&
                hipGraphInstantiate(&cg_exec, g, nullptr, nullptr, 0) == hipSuccess) {
                cg_graph = g;
                cg_stream = s;
                cg_x = x;
                cg_precond = precond;
            } else {
                if (g) (void)hipGraphDestroy(g);
                cg_exec = nullptr;
                graph_failed = true;
            }
        } else {
            (void)hipGetLastError();
            graph_failed = true;
        }
    }
    pcg_block(s, x);
}

// Queues one more block of CG_CHECK iterations (frozen once converged).
void LoSolver::pcg_block(hipStream_t s, double *x) {
    if (use_graphs && cg_exec) SMRT_HIP(hipGraphLaunch(cg_exec, s));
    else cg_block(s, x, CG_CHECK);
}

// Queues the copy of the CG stop flag and iteration count to the host.
void LoSolver::pcg_status_async(hipStream_t s) {
    SMRT_HIP(hipMemcpyAsync(hbuf, sc.p + 8, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
}

// One CG iteration = 5 launches: D^T p; S p with the p.Sp block partials (both
// in stencil form); the
// x/r/z update (each block sums the p.Sp partials itself) with the r.z and r.r
// partials; the new direction (each block sums r.z); the scalars and the stop test.
void LoSolver::cg_block(hipStream_t s, double *x, int iters) {
    const int nbk = nb(nn);
    if (precond == 1) {
        for (int k = 0; k < iters; ++k) mg_cg_iteration(s, x);
        return;
    }
    const LoGeom g = geom();
    for (int k = 0; k < iters; ++k) {
        hipLaunchKernelGGL(k_dt_stencil, dim3(nbk), dim3(256), 0, s, nn, g, c / 3.0, p.p, MFinv.p, tmpF.p);
        hipLaunchKernelGGL(k_schur_stencil_dot, dim3(nbk), dim3(256), 0, s, nn, g, tmpF.p, p.p, diagE.p, Ap.p,
                           apart.p);
        hipLaunchKernelGGL(k_cg_xr_dot, dim3(nbk), dim3(256), 0, s, nn, nbk, sc.p, apart.p, p.p, Ap.p, x, r.p, Minv.p,
                           z.p, bpart.p);
        hipLaunchKernelGGL(k_cg_p, dim3(nbk), dim3(256), 0, s, nn, nbk, sc.p, bpart.p, z.p, p.p);
        hipLaunchKernelGGL(k_cg_step_end, dim3(1), dim3(256), 0, s, nbk, bpart.p, sc.p);
    }
}

void LoSolver::drop_graph() {
    // the last replay may still be queued on its stream: let it finish first
    if (cg_exec && cg_stream) (void)hipStreamSynchronize(cg_stream);
    if (cg_exec) (void)hipGraphExecDestroy(cg_exec);
    if (cg_graph) (void)hipGraphDestroy(cg_graph);
    cg_exec = nullptr;
    cg_graph = nullptr;
    cg_stream = nullptr;
    cg_x = nullptr;
    cg_precond = -1;
}


smrt_status LoSolver::solve(hipStream_t s, const LoInputs &in, double *E, double *F, double *T, smrt_step_stats *st,
                            std::string &err) {
    const double icdt = 1.0 / (c * in.dt);
    hipLaunchKernelGGL(k_lo_outer_setup, dim3(nb(nn)), dim3(256), 0, s, nn, dim, icdt, wn.p, in.sigF, in.qF, MFinv.p, tmpF.p);
    hipLaunchKernelGGL(k_spmv, dim3(nb(nn)), dim3(256), 0, s, nn, dD.rp, dD.col, dD.val, tmpF.p, DqF.p);
    hipLaunchKernelGGL(k_jacobi_base, dim3(nb(nn)), dim3(256), 0, s, nn, dim, c / 3.0, dD.rp, dD.col, dD.val, dP.rp,
                       dP.col, dP.val, MFinv.p, jbase.p);
    ensure_hbuf();
    // F from E, then the pointwise temperature from the energy balance
    // (starting from T as it was at the linearisation), then the iterate
    // change |T - T_old|^2 + |E - E_old|^2 into scalar slot 5; the stop flag
    // and count of the CG, the elimination flags and the change are copied
    // to the host together
    auto tail = [&]() {
        hipLaunchKernelGGL(k_backsub, dim3(nb((int64_t)nn * dim)), dim3(256), 0, s, nn, dim, c / 3.0, dDT.rp, dDT.col,
                           dDT.val, E, in.qF, MFinv.p, F);
        hipLaunchKernelGGL(k_zero4, dim3(1), dim3(4), 0, s, flags.p);
        hipLaunchKernelGGL(k_eliminate, dim3(nb(nn)), dim3(256), 0, s, nn, a, c, in.dt, in.elim_rtol, in.max_elim,
                           in.T_floor, in.cvn, in.sigE, in.sigP, E, in.Tstar, T, flags.p);
        hipLaunchKernelGGL(k_diff2_partial, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s, nn, T, Told.p, E, Eold.p,
                           part.p);
        hipLaunchKernelGGL(k_dot_finish_n, dim3(1), dim3(RED_BLOCKS), 0, s, part.p, sc.p, 1, 5, 5, 5);
        pcg_status_async(s);
        SMRT_HIP(hipMemcpyAsync(hbuf + 2, flags.p, 4 * sizeof(int), hipMemcpyDeviceToHost, s));
        SMRT_HIP(hipMemcpyAsync(hbuf + 4, sc.p + 5, sizeof(double), hipMemcpyDeviceToHost, s));
        SMRT_HIP(hipStreamSynchronize(s));
    };
    double first = -1.0;
    smrt_status status = SMRT_OK;
    for (int m = 1; m <= in.max_inner; ++m) {
        hipLaunchKernelGGL(k_newton_prep, dim3(nb(nn)), dim3(256), 0, s, nn, a, c, in.dt, wn.p, in.cvn, T, in.Tstar,
                           in.sigE, in.sigP, in.qE, DqF.p, jbase.p, diagE.p, rhs.p, Minv.p, E, Eold.p, Told.p);
        precond = in.precond;
        if (precond == 1) {
            init_mg();                              // once per context
            setup_mg(s);                            // coarse operators of this linearisation
        }
        // one block of CG iterations and the rest of the Newton iteration are
        // queued before the first wait; a CG that needs more than one block
        // runs on and the rest is redone from the saved temperature
        pcg_begin(s, E, in.cg_rtol, in.max_cg);
        tail();
        if (hbuf[0] == 0.0) {
            do {
                pcg_block(s, E);
                pcg_status_async(s);
                SMRT_HIP(hipStreamSynchronize(s));
            } while (hbuf[0] == 0.0);
            SMRT_HIP(hipMemcpyAsync(T, Told.p, sizeof(double) * nn, hipMemcpyDeviceToDevice, s));
            tail();
        }
        st->cg_total += (int)hbuf[1];
        // a CG stopped by its iteration cap (stop flag 2), or a node whose
        // pointwise Newton ran to its cap (elimination flag 2), is a capped
        // iteration of this step
        if (hbuf[0] == 2.0) st->hit_max = 1;
        int fl[4];
        std::memcpy(fl, hbuf + 2, sizeof(fl));
        const double diff = std::sqrt(hbuf[4]);
        st->inner_total++;
        if (fl[1] > st->elim_max) st->elim_max = fl[1];
        if (fl[2]) st->hit_max = 1;
        if (fl[0]) {
            err = "no positive temperature root in the energy balance";
            status = SMRT_E_NONPHYSICAL;
            break;
        }
        if (!std::isfinite(diff)) {
            err = "non-finite low-order iterate";
            status = SMRT_E_NONPHYSICAL;
            break;
        }
        if (m == 1) first = diff;
        if (diff == 0.0 || (m > 1 && diff < in.eps_inner * first)) break;
        if (m == in.max_inner) st->hit_max = 1;
    }
    return status;
}

}  // namespace smrt

#include "mg_precond.inc"
#include "lo_batch.inc"
