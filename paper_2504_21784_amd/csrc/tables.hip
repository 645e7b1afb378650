// Per-step and per-outer-iteration tables of the SM-TRT step (gfx950):
//  * opacity table: sigma_g per cell from the cell-average temperature of
//    the previous step (Sec. 3), and sigma_t = sigma + 1/(c dt) (Sec. 2);
//  * emission source: q_iso = sigma_g a c T^4 b_g(T) / (4 pi) at every node
//    (Eq. planck / black_body), plus the Planck- and Rosseland-collapsed
//    gray opacities sigma_P and sigma_F at the node (Sec. 2, Eq. sigmaF);
//  * boundary inflow table B_g(T_bdr)/(4 pi) or explicit values;
//  * layout conversions between the ABI and the sweep's internal layout;
//  * the 2D moment finalisation (sum of per-workgroup partials, FP64);
//  * the 1D sweep (lanes = (angle, group) pairs) and its moments.
//
// The group fractions use the cumulative Planck function
//   P(x) = 15/pi^4 int_0^x t^3/(e^t - 1) dt
// evaluated with the Bernoulli-number series for x < 2 and the exponential
// series 1 - 15/pi^4 sum_k e^{-kx}(x^3/k + 3x^2/k^2 + 6x/k^3 + 6/k^4) for
// x >= 2 (both follow from expanding the integrand), and the Rosseland
// cumulative R(x) = P(x) - 15/(4 pi^4) x^4/(e^x - 1) (integration by parts
// of x^4 e^x/(e^x-1)^2).  b_g = P(x_{g+1}) - P(x_g), r_g likewise, with the
// first lower bound at 0 and the last upper bound at infinity.
#include <cmath>
#include <type_traits>

#include "smrt_internal.h"
#include "tables.h"

namespace smrt {

__constant__ double c_bern[NBERN];   // B_{2k} / ((2k)! (2k+3)), k = 1..NBERN

// 1/k for the exponential series (no division in the loop)
struct InvTable {
    double v[201];
    constexpr InvTable() : v() {
        for (int k = 1; k <= 200; ++k) v[k] = 1.0 / k;
    }
};
__constant__ InvTable c_inv = InvTable();

// Cumulative normalised Planck and Rosseland spectra at x = nu/T, from one
// evaluation of the Planck integral:
//   P(x) = 15/pi^4 int_0^x t^3/(e^t-1) dt,
//   R(x) = 15/(4 pi^4) int_0^x t^4 e^t/(e^t-1)^2 dt = P(x) - 15/(4 pi^4) x^4 e^{-x}/(1-e^{-x})
// (integration by parts).  P by the Bernoulli series for x < 2; above, the
// upper tail 1 - P by the exponential series sum_k e^{-kx} (x^3/k + 3x^2/k^2
// + 6x/k^3 + 6/k^4).  Each side is returned together with its complement,
// so that a fraction between two bounds above x = 2 is taken as the
// difference of the tails, which keeps its relative precision where the
// fraction is tiny (1 - P near 1 would lose it).
struct PR {
    double P, R, Pc, Rc;   // P, R and the tails 1 - P, 1 - R
};
__device__ PR planck_rosseland_cum(double x) {
    constexpr double c15 = 15.0 / (M_PI * M_PI * M_PI * M_PI);
    constexpr double c15_4 = 15.0 / (4.0 * M_PI * M_PI * M_PI * M_PI);
    if (!(x > 0.0)) return {0.0, 0.0, 1.0, 1.0};
    if (x >= 1e300) return {1.0, 1.0, 0.0, 0.0};
    if (x < 2.0) {
        // int_0^x t^3/(e^t-1) dt = x^3/3 - x^4/8 + sum_k B_2k x^(2k+3) / ((2k)! (2k+3))
        const double x2 = x * x, x3 = x2 * x;
        double s = 0.0, p = x3 * x2;   // x^(2k+3) for k = 1
        for (int k = 0; k < NBERN; ++k) {
            s += c_bern[k] * p;
            p *= x2;
        }
        const double P = c15 * (x3 / 3.0 - x3 * x / 8.0 + s);
        const double R = P - c15_4 * x3 * x * exp(-x) / -expm1(-x);
        return {P, R, 1.0 - P, 1.0 - R};
    }
    double s = 0.0;
    const double e = exp(-x), em = 1.0 - e;
    const double x2 = x * x, x3 = x2 * x;
    double ek = e;
    for (int k = 1; k <= 200; ++k) {
        const double ik = c_inv.v[k];
        const double term = ek * (ik * (x3 + ik * (3.0 * x2 + ik * (6.0 * x + 6.0 * ik))));
        s += term;
        if (term < 1e-18 * s) break;
        ek *= e;
        if (ek == 0.0) break;
    }
    const double Q = c15 * s;
    const double Qr = x > 700.0 ? 0.0 : Q + c15_4 * x3 * x * e / em;
    return {1.0 - Q, 1.0 - Qr, Q, Qr};
}

// Group fractions at temperature T, produced one group at a time in group
// order (no per-thread arrays, which would live in scratch memory):
// b_g = P(x_{g+1}) - P(x_g), r_g likewise, with x_0 = 0 and x_G = infinity
// (so a single group gets b = r = 1); a group whose lower bound lies at
// x >= 2 takes the difference of the upper tails.
struct GroupFractions {
    const double *nu;
    double T, Pl = 0.0, Rl = 0.0, Pcl = 1.0, Rcl = 1.0, xl = 0.0;
    int G, g = 0;
    __device__ GroupFractions(int G_, const double *nu_, double T_) : nu(nu_), T(T_), G(G_) {}
    __device__ void next(double &b, double &r) {
        PR u{1.0, 1.0, 0.0, 0.0};
        double xu = 1e308;
        if (g < G - 1) {
            xu = nu[g + 1] / T;
            u = planck_rosseland_cum(xu);
        }
        if (xl >= 2.0) {
            b = Pcl - u.Pc;
            r = Rcl - u.Rc;
        } else {
            b = u.P - Pl;
            r = u.R - Rl;
        }
        Pl = u.P;
        Rl = u.R;
        Pcl = u.Pc;
        Rcl = u.Rc;
        xl = xu;
        ++g;
    }
};

// ---------------------------------------------------------------------------
// Opacity table (once per step)
// ---------------------------------------------------------------------------
// cell-average temperature (arithmetic mean of the nodal values) and the
// group opacity of a cell at it: model 0 sigma0[r][g], model 1
// sigma0[r] / (nu_g^3 T^3) with nu_g the geometric mean of the group bounds,
// clipped to [clip_lo, clip_hi]
__device__ inline double cell_mean_T(int npc, const double *T, int c) {
    double Tc = 0.0;
    for (int l = 0; l < npc; ++l) Tc += T[npc * c + l];
    return Tc / npc;
}
__device__ inline double group_opacity(int model, int G, int r, int g, const double *sigma0, const double *nu,
                                       double Tc, double clip_lo, double clip_hi) {
    if (model == 0) return sigma0[r * G + g];
    const double nb = sqrt(nu[g] * nu[g + 1]);
    const double s = sigma0[r] / (nb * nb * nb * Tc * Tc * Tc);
    return fmin(fmax(s, clip_lo), clip_hi);
}

template <typename real>
__global__ void k_opacity(int ncell, int npc, int G, const double *T, const int *region, int model,
                          const double *sigma0, double clip_lo, double clip_hi, const double *nu,
                          double inv_c_dt, double *sig, real *sig2) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    const double Tc = cell_mean_T(npc, T, c);
    const int r = region[c];
    for (int g = 0; g < G; ++g) {
        const double s = group_opacity(model, G, r, g, sigma0, nu, Tc, clip_lo, clip_hi);
        sig[(int64_t)c * G + g] = s;
        if (sig2) {
            sig2[2 * ((int64_t)g * ncell + c)] = (real)(s + inv_c_dt);
            sig2[2 * ((int64_t)g * ncell + c) + 1] = (real)s;
        }
    }
}

// ---------------------------------------------------------------------------
// Emission source and gray collapse (once per outer iteration)
// ---------------------------------------------------------------------------
template <typename real>
__global__ void k_source(int nn, int npc, int G, const double *T, const double *nu, double a, double c,
                         const double *sig, real *qiso, real *qnat, double *sigP, double *sigF, const int *gate) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= nn || (gate && !*gate)) return;
    const double Tn = T[n];
    GroupFractions fr(G, nu, Tn);
    const int cell = n / npc, l = n - cell * npc;
    const int ncell = nn / npc;
    const double B = a * c * Tn * Tn * Tn * Tn / (4.0 * M_PI);
    double sb = 0, sbs = 0, sr = 0, srs = 0;
    for (int g = 0; g < G; ++g) {
        double bg, rg;
        fr.next(bg, rg);
        const double s = sig[(int64_t)cell * G + g];
        if (qiso) qiso[((int64_t)g * ncell + cell) * npc + l] = (real)(s * B * bg);
        if (qnat) qnat[(int64_t)g * nn + n] = (real)(s * B * bg);
        sb += bg;
        sbs += bg * s;
        sr += rg;
        srs += rg * s;
    }
    sigP[n] = sbs / sb;
    sigF[n] = srs / sr;
}

// ---------------------------------------------------------------------------
// 2D sweep tables in the skewed band layout of the sweep, one copy per
// quadrant: slot (band, t, r) of quadrant q holds the canonical cell
// (t - r, 16 band + r); entries outside the mesh are padding.
// ---------------------------------------------------------------------------
__device__ inline bool skew_to_cell(int nx, int ny, int q, int64_t slot, int &cell, int &flip) {
    const int NT = nx + BAND_ROWS - 1;
    const int r = (int)(slot % BAND_ROWS);
    const int64_t bt = slot / BAND_ROWS;
    const int t = (int)(bt % NT), band = (int)(bt / NT);
    const int ic = t - r, jc = band * BAND_ROWS + r;
    if (ic < 0 || ic >= nx || jc >= ny) return false;
    const bool fx = (q == 1 || q == 2), fy = (q == 2 || q == 3);
    cell = (fx ? nx - 1 - ic : ic) + nx * (fy ? ny - 1 - jc : jc);
    flip = (fx ? 1 : 0) | (fy ? 2 : 0);
    return true;
}

// (sigma_t, sigma) per (quadrant, group, skewed cell) from sigma [cell][G]
// (and sigma_t if given).  One thread per (quadrant, skewed slot) walks the
// groups in blocks of GB, issuing a block's gathers before its stores; its
// writes for each group are coalesced across the slots.  A padding slot
// reads cell 0 and stores (1, 0).
constexpr int TAB_GB = 4;
template <typename real>
__global__ void k_stab2d(int nx, int ny, int G, const double *__restrict__ sig, const double *__restrict__ sigt,
                         double icdt, real *__restrict__ stab) {
    const int64_t cs = cell_slab(nx, ny);
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= 4 * cs) return;
    const int64_t slot = i % cs;
    const int q = (int)(i / cs);
    int cell = 0, flip;
    const bool on = skew_to_cell(nx, ny, q, slot, cell, flip);
    if (!on) cell = 0;
    using r2 = typename std::conditional<sizeof(real) == 4, float2, double2>::type;
    r2 *__restrict__ out = reinterpret_cast<r2 *>(stab);
    const double *__restrict__ st_src = sigt ? sigt : sig;   // sigma_t given, or sigma + 1/(c dt)
    const double add = sigt ? 0.0 : icdt;
    const double *row = sig + (int64_t)cell * G, *strow = st_src + (int64_t)cell * G;
    for (int g0 = 0; g0 < G; g0 += TAB_GB) {
        double sg[TAB_GB], st[TAB_GB];
#pragma unroll
        for (int k = 0; k < TAB_GB; ++k) {
            const int g = g0 + k < G ? g0 + k : G - 1;
            sg[k] = row[g];
            st[k] = strow[g];
        }
#pragma unroll
        for (int k = 0; k < TAB_GB; ++k) {
            if (g0 + k < G) {   // uniform across the grid
                r2 v;
                v.x = on ? (real)(st[k] + add) : real(1);
                v.y = on ? (real)sg[k] : real(0);
                out[((int64_t)q * G + g0 + k) * cs + slot] = v;
            }
        }
    }
}

// 2D opacity and its skewed per-quadrant tables in one pass: one thread per
// (quadrant, skewed slot) evaluates its cell's opacities from the nodal
// temperatures (four quadrants recompute a cell's values, cheaper than
// reading them back), writes (sigma + 1/(c dt), sigma) for every group, and
// the quadrant-0 thread of the cell also writes sigma[cell][G].  A padding
// slot stores (1, 0).
template <typename real>
__global__ void k_opacity_tab2d(int nx, int ny, int G, const double *__restrict__ T, const int *__restrict__ region,
                                int model, const double *__restrict__ sigma0, double clip_lo, double clip_hi,
                                const double *__restrict__ nu, double icdt, double *__restrict__ sig,
                                real *__restrict__ stab) {
    const int64_t cs = cell_slab(nx, ny);
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= 4 * cs) return;
    const int64_t slot = i % cs;
    const int q = (int)(i / cs);
    int cell = 0, flip;
    const bool on = skew_to_cell(nx, ny, q, slot, cell, flip);
    using r2 = typename std::conditional<sizeof(real) == 4, float2, double2>::type;
    r2 *__restrict__ out = reinterpret_cast<r2 *>(stab);
    if (!on) {
        for (int g = 0; g < G; ++g) {
            r2 v;
            v.x = real(1);
            v.y = real(0);
            out[((int64_t)q * G + g) * cs + slot] = v;
        }
        return;
    }
    const double Tc = cell_mean_T(4, T, cell);
    const int r = region[cell];
    // a cell's G opacities are contiguous in sig: with G even they go out in
    // 16-byte pairs (half the store instructions of the scattered cells)
    const bool pairs = (G & 1) == 0;
    double s_even = 0.0;
    for (int g = 0; g < G; ++g) {
        const double s = group_opacity(model, G, r, g, sigma0, nu, Tc, clip_lo, clip_hi);
        r2 v;
        v.x = (real)(s + icdt);
        v.y = (real)s;
        out[((int64_t)q * G + g) * cs + slot] = v;
        if (q == 0) {
            if (!pairs) sig[(int64_t)cell * G + g] = s;
            else if (g & 1) *reinterpret_cast<double2 *>(sig + (int64_t)cell * G + g - 1) = make_double2(s_even, s);
            else s_even = s;
        }
    }
}

// Emission table in the skewed per-quadrant layout (canonical node order) from
// a natural-order field q[n * sn + g * sg] (FP64, or already at the sweep
// precision); one thread per (quadrant, skewed slot) walks the groups in
// blocks of TAB_GB (gathers first, then stores).  A padding slot stores zeros.
template <typename real, typename src_t>
__global__ void k_qtab2d(int nx, int ny, int G, const src_t *__restrict__ q, int64_t sn, int64_t sg,
                         real *__restrict__ qtab, const int *gate) {
    const int64_t cs = cell_slab(nx, ny);
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= 4 * cs || (gate && !*gate)) return;
    const int64_t slot = i % cs;
    const int qd = (int)(i / cs);
    int cell = 0, flip = 0;
    const bool on = skew_to_cell(nx, ny, qd, slot, cell, flip);
    if (!on) cell = 0;
    using r4 = typename std::conditional<sizeof(real) == 4, float4, double4>::type;
    r4 *__restrict__ out = reinterpret_cast<r4 *>(qtab);
    const src_t *base = q + (int64_t)4 * cell * sn;
    for (int g0 = 0; g0 < G; g0 += TAB_GB) {
        src_t v[TAB_GB][4];
        using s4 = typename std::conditional<sizeof(src_t) == 4, float4, double4>::type;
#pragma unroll
        for (int k = 0; k < TAB_GB; ++k) {
            const int g = g0 + k < G ? g0 + k : G - 1;
            if (sn == 1) {   // a cell's 4 nodes are contiguous (and 4-value aligned)
                const s4 t4 = *reinterpret_cast<const s4 *>(base + (int64_t)g * sg);
                v[k][0] = t4.x; v[k][1] = t4.y; v[k][2] = t4.z; v[k][3] = t4.w;
            } else {
#pragma unroll
                for (int l = 0; l < 4; ++l) v[k][l] = base[(int64_t)g * sg + l * sn];
            }
        }
#pragma unroll
        for (int k = 0; k < TAB_GB; ++k) {
            if (g0 + k < G) {   // uniform across the grid
                r4 w;
                w.x = on ? (real)v[k][0 ^ flip] : real(0);
                w.y = on ? (real)v[k][1 ^ flip] : real(0);
                w.z = on ? (real)v[k][2 ^ flip] : real(0);
                w.w = on ? (real)v[k][3 ^ flip] : real(0);
                out[((int64_t)qd * G + g0 + k) * cs + slot] = w;
            }
        }
    }
}

// Isotropic equilibrium intensity B_g(T_n)/(4 pi) in the ABI layout [d][g][node]
// (FP64) -- used to initialise a state.
__global__ void k_equilibrium(int nn, int G, int nang, const double *T, const double *nu, double a, double c,
                              double *psi) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= nn) return;
    GroupFractions fr(G, nu, T[n]);
    const double B = a * c * pow(T[n], 4) / (4.0 * M_PI);
    for (int g = 0; g < G; ++g) {
        double bg, rg;
        fr.next(bg, rg);
        for (int d = 0; d < nang; ++d) psi[((int64_t)d * G + g) * nn + n] = B * bg;
    }
}

// Side values of the isotropic inflow: val[side][g]
__global__ void k_side_inflow(int G, const double *nu, double a, double c, const int *kind, const double *Tb,
                              const double *explicit_g, double *val) {
    const int side = blockIdx.x;
    if (threadIdx.x != 0) return;
    for (int g = 0; g < G; ++g) val[side * G + g] = 0.0;
    if (kind[side] == 1 && Tb[side] > 0.0) {
        GroupFractions fr(G, nu, Tb[side]);
        const double B = a * c * pow(Tb[side], 4) / (4.0 * M_PI);
        for (int g = 0; g < G; ++g) {
            double bg, rg;
            fr.next(bg, rg);
            val[side * G + g] = B * bg;
        }
    } else if (kind[side] == 2) {
        for (int g = 0; g < G; ++g) val[side * G + g] = explicit_g[side * G + g];
    }
}

// General inflow table [d][g][NB] from the side values
template <typename real>
__global__ void k_fill_inflow(int dim, int nx, int ny, int G, int nang, const double *val, real *inflow) {
    const int NB = dim == 1 ? 2 : 4 * (nx + ny);
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= (int64_t)nang * G * NB) return;
    const int b = (int)(i % NB);
    const int g = (int)((i / NB) % G);
    int side;
    if (dim == 1) side = b;
    else side = b < 2 * ny ? 0 : b < 4 * ny ? 1 : b < 4 * ny + 2 * nx ? 2 : 3;
    inflow[i] = (real)val[side * G + g];
}

template <typename real>
__global__ void k_copy_to(int64_t n, const double *src, real *dst) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) dst[i] = (real)src[i];
}
template <typename real>
__global__ void k_copy_from(int64_t n, const real *src, double *dst) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) dst[i] = (double)src[i];
}

// q_iso ABI [node][G] -> internal [G][cell][npc]
template <typename real>
__global__ void k_qiso_to_internal(int nn, int G, const double *q, real *qi, int npc) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= (int64_t)nn * G) return;
    const int n = (int)(i / G), g = (int)(i % G);
    const int cell = n / npc, l = n % npc;
    qi[((int64_t)g * (nn / npc) + cell) * npc + l] = (real)q[i];
}

// sig_t, sig ABI [cell][G] -> internal (sigma_t, sigma) pairs [G][cell]
template <typename real>
__global__ void k_sig_to_internal(int ncell, int G, const double *st, const double *s, real *sig2) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= (int64_t)ncell * G) return;
    const int c = (int)(i / G), g = (int)(i % G);
    sig2[2 * ((int64_t)g * ncell + c)] = (real)st[i];
    sig2[2 * ((int64_t)g * ncell + c) + 1] = (real)s[i];
}

// ---------------------------------------------------------------------------
// Angular flux layout conversion (2D): ABI [d][g][node] <-> internal
// [d][g][band][t][r][canonical node].  dir_quad[d] gives the quadrant.
// ---------------------------------------------------------------------------
__device__ inline int64_t internal_index(int nx, int ny, int q, int i, int j, int l, int64_t slab_base) {
    const bool fx = (q == 1 || q == 2), fy = (q == 2 || q == 3);
    const int ic = fx ? nx - 1 - i : i, jc = fy ? ny - 1 - j : j;
    const int lc = l ^ ((fx ? 1 : 0) | (fy ? 2 : 0));
    const int band = jc / BAND_ROWS, r = jc % BAND_ROWS, t = ic + r;
    const int NT = nx + BAND_ROWS - 1;
    return slab_base + (((int64_t)band * NT + t) * BAND_ROWS + r) * 4 + lc;
}

template <typename real, typename src_t, bool TO_INTERNAL>
__global__ void k_psi_convert(int nx, int ny, int G, int nang, const int *dir_quad, const src_t *in, real *out_or_in_real,
                              double *out_abi) {
    const int nn = nx * ny * 4;
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= (int64_t)nang * G * nn) return;
    const int n = (int)(i % nn);
    const int dg = (int)(i / nn);
    const int d = dg / G;
    const int cell = n >> 2, l = n & 3;
    const int ii = cell % nx, jj = cell / nx;
    const int64_t slab = (int64_t)dg * psi_slab(nx, ny);
    const int64_t k = internal_index(nx, ny, dir_quad[d], ii, jj, l, slab);
    if (TO_INTERNAL) out_or_in_real[k] = (real)in[i];
    else out_abi[i] = (double)out_or_in_real[k];
}

// ---------------------------------------------------------------------------
// Reflective sides (specular reflection: the symmetry planes of Sec. 6).
// A boundary node b of the general inflow table [d][g][NB] lies on side
// `side` at cell (ci, cj), local node l.  For a direction d entering through
// a reflective side, the inflow is the intensity of its mirror image e
// (mu -> -mu on the x sides, eta -> -eta on the y sides) at the same node,
// read from the sweep's angular flux (2D: internal layout; 1D: [d][g][node]).
// refl has bit s set for a reflective side s; mirror[ax * nang + d] = e.
// ---------------------------------------------------------------------------
__device__ inline void boundary_node(int dim, int nx, int ny, int b, int &side, int &ci, int &cj, int &l) {
    if (dim == 1) { side = b; ci = b ? nx - 1 : 0; cj = 0; l = b; return; }
    if (b < 2 * ny) { side = 0; ci = 0; cj = b >> 1; l = (b & 1) << 1; return; }
    b -= 2 * ny;
    if (b < 2 * ny) { side = 1; ci = nx - 1; cj = b >> 1; l = 1 | ((b & 1) << 1); return; }
    b -= 2 * ny;
    if (b < 2 * nx) { side = 2; ci = b >> 1; cj = 0; l = b & 1; return; }
    b -= 2 * nx;
    side = 3; ci = b >> 1; cj = ny - 1; l = 2 | (b & 1);
}

// one thread per (d, g, boundary node); entries of other sides and of
// directions leaving through the side are left as they are
template <typename real>
__global__ void k_reflect(int dim, int nx, int ny, int G, int nang, int refl, const int *mirror, const double *om,
                          const int *dir_quad, const real *psi, real *inflow) {
    const int NB = dim == 1 ? 2 : 4 * (nx + ny);
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= (int64_t)nang * G * NB) return;
    const int b = (int)(i % NB);
    const int g = (int)((i / NB) % G);
    const int d = (int)(i / ((int64_t)NB * G));
    int side, ci, cj, l;
    boundary_node(dim, nx, ny, b, side, ci, cj, l);
    if (!((refl >> side) & 1)) return;
    const int ax = side >> 1;
    if ((side & 1 ? 1.0 : -1.0) * om[3 * d + ax] >= 0.0) return;
    const int e = mirror[ax * nang + d];
    const int64_t pair = (int64_t)e * G + g;
    if (dim == 1) inflow[i] = psi[pair * 2 * nx + 2 * ci + l];
    else inflow[i] = psi[internal_index(nx, ny, dir_quad[e], ci, cj, l, pair * psi_slab(nx, ny))];
}

// Incoming moments of the inflow at each boundary node of a reflective side,
//   bmom[b] = (sum_{Omega.n<0} sum_g w (Omega.n) I_b, the same weighted by
//   mu, by eta),
// the closures' boundary terms F_in and P_in for an inflow that is neither
// isotropic nor uniform along the side.  One 64-thread block per node: the
// (d, g) pairs are strided over the lanes, summed in FP64 and reduced over
// the wave.
template <typename real>
__global__ void __launch_bounds__(64) k_inflow_moments(int dim, int nx, int ny, int G, int nang, int refl,
                                                       const double *om, const double *w, const real *inflow,
                                                       double *bmom) {
    const int NB = dim == 1 ? 2 : 4 * (nx + ny);
    const int b = blockIdx.x;
    int side, ci, cj, l;
    boundary_node(dim, nx, ny, b, side, ci, cj, l);
    if (!((refl >> side) & 1)) return;     // uniform over the block
    const int ax = side >> 1;
    const double sgn = side & 1 ? 1.0 : -1.0;
    double f = 0.0, p0 = 0.0, p1 = 0.0;
    for (int k = threadIdx.x; k < nang * G; k += 64) {
        const int d = k / G, g = k - d * G;
        const double on = sgn * om[3 * d + ax];
        if (on < 0.0) {
            const double v = w[d] * on * (double)inflow[((int64_t)d * G + g) * NB + b];
            f += v;
            p0 += om[3 * d] * v;
            p1 += (dim == 2 ? om[3 * d + 1] : 0.0) * v;
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        f += __shfl_xor(f, off, 64);
        p0 += __shfl_xor(p0, off, 64);
        p1 += __shfl_xor(p1, off, 64);
    }
    if (threadIdx.x == 0) {
        bmom[3 * b] = f;
        bmom[3 * b + 1] = p0;
        bmom[3 * b + 2] = p1;
    }
}

// ---------------------------------------------------------------------------
// Adjoint helpers: direction permutation (out[d] = in[map[d]]) of [d][per]
// arrays, and the opacity sensitivity of a sweep,
//   dsig[c][g] = sum_d sum_{l in c} w_l lambda_{d,g,l} (emis_{l,g} - I_{d,g,l}),
// w_l the lumped nodal weight |cell| / 2^dim (one thread per (cell, group),
// directions summed in index order).
// ---------------------------------------------------------------------------
__global__ void k_permute_dirs(int nang, int64_t per, const int *map, const double *in, double *out) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= nang * per) return;
    const int d = (int)(i / per);
    out[i] = in[(int64_t)map[d] * per + (i - d * per)];
}

__global__ void k_adjoint_dsig(int dim, int nx, int ny, int G, int nang, const double *hx, const double *hy,
                               const double *lam, const double *emis, const double *psi, double *dsig) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int ncell = nx * ny, npc = dim == 2 ? 4 : 2;
    if (i >= (int64_t)ncell * G) return;
    const int c = (int)(i / G), g = (int)(i % G);
    const double wl = dim == 2 ? hx[c % nx] * hy[c / nx] * 0.25 : hx[c] * 0.5;
    const int64_t nn = (int64_t)ncell * npc;
    double s = 0.0;
    for (int d = 0; d < nang; ++d) {
        const double *L = lam + ((int64_t)d * G + g) * nn + (int64_t)npc * c;
        const double *I = psi + ((int64_t)d * G + g) * nn + (int64_t)npc * c;
        for (int l = 0; l < npc; ++l) s += L[l] * (emis[((int64_t)npc * c + l) * G + g] - I[l]);
    }
    dsig[i] = wl * s;
}

// ---------------------------------------------------------------------------
// Adjoint of a time step (implicit function theorem at the converged step):
// per-node quantities of the step, adjoint source assembly, the pointwise
// temperature adjoint, sigma-sensitivities and per-region gradient sums.
// Nodal weights: 2D |cell|/4 = hx hy / 4, 1D hx / 2.
// ---------------------------------------------------------------------------
__device__ inline double nodal_weight(int dim, int nx, const double *hx, const double *hy, int cell) {
    return dim == 2 ? hx[cell % nx] * hy[cell / nx] * 0.25 : hx[cell] * 0.5;
}

// emis = a c T^4 b_g / 4pi, dE = 4 a c T^3 r_g / 4pi, D = c_v/dt + sum_g sigma_g 4pi dE,
// phi_g = sum_d w_d I_{d,g}
__global__ void k_adj_prep(int nn, int npc, int G, int nang, const double *nu, double a, double c, double dt,
                           const double *T, const double *sig, const double *cvn, const double *w, const double *psi,
                           double *emis, double *dE, double *D, double *phi) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= nn) return;
    const double Tn = T[n];
    GroupFractions fr(G, nu, Tn);
    const double T3 = Tn * Tn * Tn, T4 = T3 * Tn;
    double dsum = cvn[n] / dt;
    for (int g = 0; g < G; ++g) {
        double bg, rg;
        fr.next(bg, rg);
        const double e = a * c * T4 * bg / (4.0 * M_PI), de = 4.0 * a * c * T3 * rg / (4.0 * M_PI);
        emis[(int64_t)n * G + g] = e;
        dE[(int64_t)n * G + g] = de;
        dsum += sig[(int64_t)(n / npc) * G + g] * 4.0 * M_PI * de;
        double ph = 0.0;
        for (int d = 0; d < nang; ++d) ph += w[d] * psi[((int64_t)d * G + g) * nn + n];
        phi[(int64_t)n * G + g] = ph;
    }
    D[n] = dsum;
}

// final-material-energy weights w_n c_v,n (dJ/dT^N of J = sum_n w_n c_v,n T^N_n)
__global__ void k_adj_energy_weights(int dim, int nx, int npc, int nn, const double *hx, const double *hy,
                                     const double *cvn, double *wc) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= nn) return;
    wc[n] = nodal_weight(dim, nx, hx, hy, n / npc) * cvn[n];
}
__global__ void k_mul(int64_t n, const double *a, const double *b, double *out) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) out[i] = a[i] * b[i];
}

// right-boundary outflow weights dJ/dI = dt w_d mu_d fw_n (mu_d > 0, n on x+)
__global__ void k_adj_dJdI(int dim, int nx, int ny, int G, int nang, const double *om, const double *w, const double *hy,
                           double dt, double *out) {
    const int npc = dim == 2 ? 4 : 2, nn = nx * ny * npc;
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= (int64_t)nang * G * nn) return;
    const int n = (int)(i % nn), d = (int)(i / ((int64_t)G * nn));
    const int cell = n / npc, l = n % npc;
    const double mu = om[3 * d];
    double v = 0.0;
    if (mu > 0.0 && cell % nx == nx - 1 && (l & 1)) v = dt * w[d] * mu * (dim == 2 ? 0.5 * hy[cell / nx] : 1.0);
    out[i] = v;
}

// src = (dJ/dI + w/(c dt) lam_next + sigma_g w_d tau) / w
__global__ void k_adj_src(int dim, int nx, int ny, int G, int nang, const double *hx, const double *hy, const double *wang,
                          const double *dJdI, const double *lam_next, double icdt, const double *sig, const double *tau,
                          double *src) {
    const int npc = dim == 2 ? 4 : 2, nn = nx * ny * npc;
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= (int64_t)nang * G * nn) return;
    const int n = (int)(i % nn);
    const int64_t dg = i / nn;
    const int d = (int)(dg / G), g = (int)(dg % G);
    const int cell = n / npc;
    const double wl = nodal_weight(dim, nx, hx, hy, cell);
    src[i] = (dJdI[i] + wl * icdt * lam_next[i] + sig[(int64_t)cell * G + g] * wang[d] * tau[n]) / wl;
}

// tau_new = (ST + w sum_g sigma_g dE_g sum_d lam) / D; block partials of |tau_new - tau|^2 and |tau_new|^2
__global__ void k_adj_tau(int dim, int nx, int ny, int G, int nang, const double *hx, const double *hy,
                          const double *sig, const double *dE, const double *ST, const double *D, const double *lam,
                          const double *tau, double *tau_new, double *part) {
    __shared__ double sh[2][256];
    const int npc = dim == 2 ? 4 : 2, nn = nx * ny * npc;
    const int n = blockIdx.x * 256 + threadIdx.x;
    double e1 = 0.0, e2 = 0.0;
    if (n < nn) {
        const int cell = n / npc;
        double s = ST[n];
        for (int g = 0; g < G; ++g) {
            double ls = 0.0;
            for (int d = 0; d < nang; ++d) ls += lam[((int64_t)d * G + g) * nn + n];
            s += nodal_weight(dim, nx, hx, hy, cell) * sig[(int64_t)cell * G + g] * dE[(int64_t)n * G + g] * ls;
        }
        const double t = s / D[n];
        tau_new[n] = t;
        e1 = (t - tau[n]) * (t - tau[n]);
        e2 = t * t;
    }
    sh[0][threadIdx.x] = e1;
    sh[1][threadIdx.x] = e2;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + k];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + k];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = sh[0][0];
        part[2 * blockIdx.x + 1] = sh[1][0];
    }
}

// Anderson acceleration of the adjoint temperature iteration tau <- g(tau):
// f = g - tau; unless first, dF = f - f_prev and dG = g - g_prev (a new
// history column); then f_prev = f, g_prev = g.
__global__ void k_aa_columns(int nn, const double *tau, const double *g, double *fprev, double *gprev, double *dF,
                             double *dG, int first) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= nn) return;
    const double gn = g[n], f = gn - tau[n];
    if (!first) {
        dF[n] = f - fprev[n];
        dG[n] = gn - gprev[n];
    }
    fprev[n] = f;
    gprev[n] = gn;
}
// block partials of <col_c, a> and <col_c, b> for the ncols history columns
// col_c = cols + slot[c] * nn: part[(2 c + j) * nblocks + block]
__global__ void __launch_bounds__(256) k_aa_dots(int nn, int ncols, AASlots sl, const double *cols, const double *a,
                                                 const double *b, double *part) {
    __shared__ double sh[256];
    const int n = blockIdx.x * 256 + threadIdx.x;
    for (int q = 0; q < 2 * ncols; ++q) {
        const double *col = cols + (int64_t)sl.s[q >> 1] * nn;
        const double *v = (q & 1) ? b : a;
        sh[threadIdx.x] = n < nn ? col[n] * v[n] : 0.0;
        __syncthreads();
        for (int k = 128; k > 0; k >>= 1) {
            if (threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
            __syncthreads();
        }
        if (threadIdx.x == 0) part[(int64_t)q * gridDim.x + blockIdx.x] = sh[0];
        __syncthreads();
    }
}
// out[q] = sum over blocks of part[q * nb + block] (fixed order), q < nq
__global__ void k_aa_dots_finish(int nb, int nq, const double *part, double *out) {
    const int q = threadIdx.x;
    if (q >= nq) return;
    double s = 0.0;
    for (int k = 0; k < nb; ++k) s += part[(int64_t)q * nb + k];
    out[q] = s;
}
// tau = g - sum_c gamma_c dG[slot c]
__global__ void k_aa_update(int nn, int ncols, AASlots sl, AACoef gm, const double *dG, const double *g, double *tau) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= nn) return;
    double t = g[n];
    for (int c = 0; c < ncols; ++c) t -= gm.v[c] * dG[(int64_t)sl.s[c] * nn + n];
    tau[n] = t;
}

// sum of nb pairs of block partials in a fixed order (one thread)
__global__ void k_sum_pairs(int nb, const double *part, double *out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double a = 0.0, b = 0.0;
    for (int k = 0; k < nb; ++k) {
        a += part[2 * k];
        b += part[2 * k + 1];
    }
    out[0] = a;
    out[1] = b;
}

// G_{c,g} = lam^T dR/dsigma_{c,g} = -dsig - sum_{l in c} tau_l (phi_g - 4pi emis_g); then per cell the
// log-sigma0 sensitivity, per node the log-c_v sensitivity and the temperature source of the step before
__global__ void k_adj_cell(int npc, int ncell, int G, int model, double clip_lo, double clip_hi, double dt,
                           const double *dsig, const double *tau, const double *phi, const double *emis,
                           const double *sig, const double *cvn, const double *T, const double *Tp, double *gs_cell,
                           double *gcv_node, double *ST_prev) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    double Tc = 0.0;
    for (int l = 0; l < npc; ++l) Tc += Tp[npc * c + l];
    Tc /= npc;
    double gsum = 0.0, dTsum = 0.0;   // sum_g free sigma G ; sum_g free dsigma/dT G
    for (int g = 0; g < G; ++g) {
        double Gv = -dsig[(int64_t)c * G + g];
        for (int l = 0; l < npc; ++l) {
            const int n = npc * c + l;
            Gv -= tau[n] * (phi[(int64_t)n * G + g] - 4.0 * M_PI * emis[(int64_t)n * G + g]);
        }
        const double s = sig[(int64_t)c * G + g];
        const bool free_ = model == 0 || (s > clip_lo && s < clip_hi);
        if (free_) gsum += s * Gv;
        if (model == 1 && s > clip_lo && s < clip_hi) dTsum += (-3.0 * s / (npc * Tc)) * Gv;
    }
    gs_cell[c] = -gsum;
    for (int l = 0; l < npc; ++l) {
        const int n = npc * c + l;
        gcv_node[n] = -tau[n] * cvn[n] * (T[n] - Tp[n]) / dt;
        ST_prev[n] = cvn[n] / dt * tau[n] - dTsum;
    }
}

// per-region sums in cell order (one thread per region); accumulated into grad_s0, grad_cv
__global__ void k_region_sums(int nreg, int ncell, int npc, const int *region, const double *gs_cell,
                              const double *gcv_node, double *grad_s0, double *grad_cv) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nreg) return;
    double a = 0.0, b = 0.0;
    for (int c = 0; c < ncell; ++c) {
        if (region[c] != r) continue;
        a += gs_cell[c];
        for (int l = 0; l < npc; ++l) b += gcv_node[npc * c + l];
    }
    grad_s0[r] += a;
    grad_cv[r] += b;
}

// deterministic dot product of two long arrays (block partials, fixed-order sum)
__global__ void k_dot_blocks(int64_t n, const double *a, const double *b, double *part) {
    __shared__ double sh[256];
    double s = 0.0;
    for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) s += a[i] * b[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}
__global__ void k_sum_blocks(int nb, const double *part, double *out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (int k = 0; k < nb; ++k) s += part[k];
    out[0] = s;
}
__global__ void k_add_scalar(int64_t n, const double *a, double v, double *out) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) out[i] = a[i] + v;
}

// ---------------------------------------------------------------------------
// Moment finalisation (2D), deterministic (fixed summation order).
// Partials: [chunk][band][step t][canonical node lc][row] pairs (sum_g I,
// sum_g sigma_g I) over the chunk's groups, the cell of (t, row) being
// canonical column t - row; a chunk is one direction and chunks are grouped by
// quadrant.  The angular weights enter here, in FP64:
//   quadrant moments  sum_{d in q} w_d {1, mu, eta, mu^2, mu eta, eta^2}_d S_I,
//   sigma-weighted    sum_d w_d {1, mu, eta}_d S_sigma.
// Pass 1 works in each quadrant's own skewed coordinates (thread = (quadrant,
// band, step, canonical node, row), so the 16 rows of a wave read contiguous
// partials), sums the quadrant's chunks in FP64 in chunk order and writes the
// 6 angular moments of that quadrant into mom and its 3 sigma-weighted ones
// into a per-quadrant buffer; pass 2 sums those over the 4 quadrants.
// ---------------------------------------------------------------------------
template <typename real>
__global__ void __launch_bounds__(256) k_moments_quadrant(int nx, int ny, ChunkRanges cr, const int *qc_dir,
                                                          const double *dirs, const real *part, double *mom,
                                                          double *sigq, const int *gate) {
    using r2 = typename std::conditional<sizeof(real) == 4, float2, double2>::type;
    using e2 = __attribute__((ext_vector_type(2))) real;
    if (gate && !*gate) return;   // uniform over the grid
    const int nb = (ny + BAND_ROWS - 1) / BAND_ROWS, NT = nx + BAND_ROWS - 1;
    const int ntb = (NT + 3) / 4;
    int b = blockIdx.x;
    const int tb = b % ntb;
    b /= ntb;
    const int band = b % nb, q = b / nb;
    const int rc = threadIdx.x & 15, lc = (threadIdx.x >> 4) & 3;
    const int t = tb * 4 + (threadIdx.x >> 6);
    const int ic = t - rc, jc = band * BAND_ROWS + rc;
    if (t >= NT || ic < 0 || ic >= nx || jc >= ny) return;
    double acc[NMOM2D];
#pragma unroll
    for (int k = 0; k < NMOM2D; ++k) acc[k] = 0.0;
    const r2 *pp = reinterpret_cast<const r2 *>(part);
    // the quadrant's chunks in order, loads issued 8 chunks at a time so that
    // several are in flight (the sum keeps the chunk order)
    constexpr int U = 8;
    const int64_t stride = (int64_t)nb * NT * 64;
    const r2 *base = pp + ((int64_t)band * NT + t) * 64 + lc * BAND_ROWS + rc;
    for (int qc0 = cr.start[q]; qc0 < cr.start[q + 1]; qc0 += U) {
        r2 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int qc = qc0 + u < cr.start[q + 1] ? qc0 + u : qc0;
            // each partial is read once: a streaming load (not kept in the caches)
            const e2 t = __builtin_nontemporal_load(reinterpret_cast<const e2 *>(base + qc * stride));
            v[u].x = t[0];
            v[u].y = t[1];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (qc0 + u >= cr.start[q + 1]) break;
            const double *cw = dirs + 8 * qc_dir[qc0 + u] + 2;   // w, w mu, w eta, w mu^2, w mu eta, w eta^2
            const double sI = (double)v[u].x, sS = (double)v[u].y;
#pragma unroll
            for (int k = 0; k < 6; ++k) acc[k] += cw[k] * sI;
#pragma unroll
            for (int k = 0; k < 3; ++k) acc[6 + k] += cw[k] * sS;
        }
    }
    const bool fx = (q == 1 || q == 2), fy = (q == 2 || q == 3);
    const int i = fx ? nx - 1 - ic : ic, j = fy ? ny - 1 - jc : jc;
    const int l = lc ^ ((fx ? 1 : 0) | (fy ? 2 : 0));
    const int64_t nn = (int64_t)nx * ny * 4;
    const int64_t n = 4 * (i + (int64_t)nx * j) + l;
#pragma unroll
    for (int k = 0; k < 6; ++k) mom[(6 * q + k) * nn + n] = acc[k];
#pragma unroll
    for (int k = 0; k < 3; ++k) sigq[(3 * q + k) * nn + n] = acc[6 + k];
}

__global__ void k_moments_sigma(int64_t nn, const double *sigq, double *mom, const int *gate) {
    const int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (n >= nn || (gate && !*gate)) return;
#pragma unroll
    for (int k = 0; k < 3; ++k)
        mom[(24 + k) * nn + n] = ((sigq[k * nn + n] + sigq[(3 + k) * nn + n]) + sigq[(6 + k) * nn + n]) +
                                 sigq[(9 + k) * nn + n];
}

// ---------------------------------------------------------------------------
// 1D sweep: one thread per (direction, group); cells in upwind order.
// Lumped linear DG, nodes (L, R); for mu > 0 (canonical):
//   [[d, m/2], [-m/2, d]] [I_L, I_R] = [w q_L + m I_up, w q_R],
//   d = m/2 + sigt h/2, w = h/2, m = |mu|  ->  inverse (dI - (m/2)J)/(d^2 + m^2/4)
// Optional zero-and-scale fixup (Sec. 6, Hamilton et al.): the columns sum to
// (sigt w, sigt w + m), so a cell with a negative entry keeps its balance
//   sigt w (I_u + I_d) + m I_d = r0 + r1
// when its negative entry is zeroed and the other scaled to match (zero if the
// right side is not positive).
// ---------------------------------------------------------------------------
template <typename real>
__global__ void k_sweep1d(Sweep1DArgs A) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= A.nang * A.G) return;
    const int d = i / A.G, g = i % A.G;
    const real *mw = static_cast<const real *>(A.mu_w);
    const real *hx = static_cast<const real *>(A.hx);
    const real *sig2 = static_cast<const real *>(A.sig2);
    const real *qi = static_cast<const real *>(A.qiso);
    const real *pp = static_cast<const real *>(A.psi_prev);
    real *po = static_cast<real *>(A.psi_out);
    const real *inf = static_cast<const real *>(A.inflow);
    const real mu = mw[2 * d];
    const bool fwd = mu > 0;
    const real m = fabs(mu);
    const int nn = 2 * A.nx;
    const int64_t base = ((int64_t)d * A.G + g) * nn;
    real up = inf[((int64_t)d * A.G + g) * 2 + (fwd ? 0 : 1)];
    const real icdt = (real)A.inv_c_dt;
    for (int s = 0; s < A.nx; ++s) {
        const int c = fwd ? s : A.nx - 1 - s;
        const real h = hx[c];
        const real w = real(0.5) * h;
        const real st = sig2[2 * ((int64_t)g * A.nx + c)];
        const int nu_ = fwd ? 0 : 1, nd_ = fwd ? 1 : 0;     // upwind / downwind node
        real qu = qi[((int64_t)g * A.nx + c) * 2 + nu_], qd = qi[((int64_t)g * A.nx + c) * 2 + nd_];
        if (pp) {
            qu += icdt * pp[base + 2 * c + nu_];
            qd += icdt * pp[base + 2 * c + nd_];
        }
        const real r0 = w * qu + m * up, r1 = w * qd;
        const real dg = real(0.5) * m + st * w, hm = real(0.5) * m;
        const real inv = real(1) / (dg * dg + hm * hm);
        real Iu = (dg * r0 - hm * r1) * inv;
        real Id = (dg * r1 + hm * r0) * inv;
        if (A.fixup && fmin(Iu, Id) < real(0)) {
            const real pu = fmax(Iu, real(0)), pd = fmax(Id, real(0));
            const real src = r0 + r1, den = st * w * (pu + pd) + m * pd;
            const real f = (src > real(0) && den > real(0)) ? src / den : real(0);
            Iu = f * pu;
            Id = f * pd;
        }
        po[base + 2 * c + nu_] = Iu;
        po[base + 2 * c + nd_] = Id;
        up = Id;
    }
}

// 1D moments [8][node] from psi [d][g][node] (sum over d, g in a fixed order)
template <typename real>
__global__ void k_moments1d(int nx, int G, int nang, const real *mu_w, const double *sig, const real *psi, double *mom) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    const int nn = 2 * nx;
    if (n >= nn) return;
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const int c = n >> 1;
    for (int d = 0; d < nang; ++d) {
        const double mu = mu_w[2 * d], w = mu_w[2 * d + 1];
        const int h = mu > 0 ? 0 : 1;
        for (int g = 0; g < G; ++g) {
            const double v = psi[((int64_t)d * G + g) * nn + n];
            acc[3 * h] += w * v;
            acc[3 * h + 1] += w * mu * v;
            acc[3 * h + 2] += w * mu * mu * v;
            const double s = sig[(int64_t)c * G + g];
            acc[6] += s * w * v;
            acc[7] += s * w * mu * v;
        }
    }
    for (int m = 0; m < 8; ++m) mom[(int64_t)m * nn + n] = acc[m];
}

// HO energy density and flux of an ABI-layout psi (FP64): E = (1/c) sum w I,
// F = sum w Omega I  (used at set_state)
__global__ void k_psi_EF(int nn, int dim, int G, int nang, const double *om, const double *w, double c,
                         const double *psi, double *E, double *F) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= nn) return;
    double e = 0, fx = 0, fy = 0;
    for (int d = 0; d < nang; ++d)
        for (int g = 0; g < G; ++g) {
            const double v = w[d] * psi[((int64_t)d * G + g) * nn + n];
            e += v;
            fx += om[3 * d] * v;
            fy += om[3 * d + 1] * v;
        }
    E[n] = e / c;
    F[dim * n] = fx;
    if (dim == 2) F[dim * n + 1] = fy;
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
static inline int nblk(int64_t n, int b) { return (int)((n + b - 1) / b); }

// Bernoulli coefficients B_2k / ((2k)! (2k+3)) = (-1)^(k+1) 2 zeta(2k) / ((2 pi)^(2k) (2k+3))
void upload_series_coefficients() {
    double coef[NBERN];
    for (int k = 1; k <= NBERN; ++k) {
        double z;
        if (k == 1) z = M_PI * M_PI / 6.0;
        else {
            z = 0.0;
            const int N = 20000;
            for (int n = N; n >= 1; --n) z += std::pow((double)n, -2.0 * k);
            z += std::pow((double)N, 1.0 - 2.0 * k) / (2.0 * k - 1.0) - 0.5 * std::pow((double)N, -2.0 * k);
        }
        const double sign = (k % 2 == 1) ? 1.0 : -1.0;
        coef[k - 1] = sign * 2.0 * z / (std::pow(2.0 * M_PI, 2.0 * k) * (2.0 * k + 3.0));
    }
    SMRT_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_bern), coef, sizeof(double) * NBERN));
}


template <typename real>
void run_opacity(hipStream_t s, int ncell, int npc, int G, const double *T, const int *region, int model,
                 const double *sigma0, double lo, double hi, const double *nu, double icdt, double *sig, real *sig2) {
    hipLaunchKernelGGL(k_opacity<real>, dim3(nblk(ncell, 256)), dim3(256), 0, s, ncell, npc, G, T, region, model,
                       sigma0, lo, hi, nu, icdt, sig, sig2);
}
template <typename real>
void run_source(hipStream_t s, int nn, int npc, int G, const double *T, const double *nu, double a, double c,
                const double *sig, real *qiso, real *qnat, double *sigP, double *sigF, const int *gate) {
    hipLaunchKernelGGL(k_source<real>, dim3(nblk(nn, 128)), dim3(128), 0, s, nn, npc, G, T, nu, a, c, sig, qiso, qnat, sigP, sigF, gate);
}
template <typename real>
void run_opacity_tab2d(hipStream_t s, int nx, int ny, int G, const double *T, const int *region, int model,
                       const double *sigma0, double lo, double hi, const double *nu, double icdt, double *sig,
                       real *stab) {
    const int64_t n = 4 * cell_slab(nx, ny);
    hipLaunchKernelGGL(k_opacity_tab2d<real>, dim3(nblk(n, 256)), dim3(256), 0, s, nx, ny, G, T, region, model, sigma0,
                       lo, hi, nu, icdt, sig, stab);
}
template <typename real>
void run_stab2d(hipStream_t s, int nx, int ny, int G, const double *sig, const double *sigt, double icdt, real *stab) {
    const int64_t n = 4 * cell_slab(nx, ny);
    hipLaunchKernelGGL(k_stab2d<real>, dim3(nblk(n, 256)), dim3(256), 0, s, nx, ny, G, sig, sigt, icdt, stab);
}
template <typename real, typename src_t>
void run_qtab2d(hipStream_t s, int nx, int ny, int G, const src_t *q, int64_t sn, int64_t sg, real *qtab,
                const int *gate) {
    const int64_t n = 4 * cell_slab(nx, ny);
    hipLaunchKernelGGL((k_qtab2d<real, src_t>), dim3(nblk(n, 256)), dim3(256), 0, s, nx, ny, G, q, sn, sg, qtab, gate);
}
void run_equilibrium(hipStream_t s, int nn, int G, int nang, const double *T, const double *nu, double a, double c,
                     double *psi) {
    hipLaunchKernelGGL(k_equilibrium, dim3(nblk(nn, 128)), dim3(128), 0, s, nn, G, nang, T, nu, a, c, psi);
}
void run_side_inflow(hipStream_t s, int nsides, int G, const double *nu, double a, double c, const int *kind,
                     const double *Tb, const double *explicit_g, double *val) {
    hipLaunchKernelGGL(k_side_inflow, dim3(nsides), dim3(64), 0, s, G, nu, a, c, kind, Tb, explicit_g, val);
}
template <typename real>
void run_fill_inflow(hipStream_t s, int dim, int nx, int ny, int G, int nang, const double *val, real *inflow) {
    const int NB = dim == 1 ? 2 : 4 * (nx + ny);
    hipLaunchKernelGGL(k_fill_inflow<real>, dim3(nblk((int64_t)nang * G * NB, 256)), dim3(256), 0, s, dim, nx, ny, G,
                       nang, val, inflow);
}
template <typename real>
void run_reflect(hipStream_t s, int dim, int nx, int ny, int G, int nang, int refl, const int *mirror, const double *om,
                 const double *w, const int *dir_quad, const real *psi, real *inflow, double *bmom) {
    if (!refl) return;
    const int NB = dim == 1 ? 2 : 4 * (nx + ny);
    hipLaunchKernelGGL(k_reflect<real>, dim3(nblk((int64_t)nang * G * NB, 256)), dim3(256), 0, s, dim, nx, ny, G, nang,
                       refl, mirror, om, dir_quad, psi, inflow);
    hipLaunchKernelGGL(k_inflow_moments<real>, dim3(NB), dim3(64), 0, s, dim, nx, ny, G, nang, refl, om, w,
                       (const real *)inflow, bmom);
}
template <typename real>
void run_copy_to(hipStream_t s, int64_t n, const double *src, real *dst) {
    hipLaunchKernelGGL(k_copy_to<real>, dim3(nblk(n, 256)), dim3(256), 0, s, n, src, dst);
}
template <typename real>
void run_qiso_to_internal(hipStream_t s, int nn, int G, int npc, const double *q, real *qi) {
    hipLaunchKernelGGL(k_qiso_to_internal<real>, dim3(nblk((int64_t)nn * G, 256)), dim3(256), 0, s, nn, G, q, qi, npc);
}
template <typename real>
void run_sig_to_internal(hipStream_t s, int ncell, int G, const double *st, const double *sg, real *sig2) {
    hipLaunchKernelGGL(k_sig_to_internal<real>, dim3(nblk((int64_t)ncell * G, 256)), dim3(256), 0, s, ncell, G, st, sg, sig2);
}
template <typename real>
void run_psi_to_internal(hipStream_t s, int nx, int ny, int G, int nang, const int *dq, const double *abi, real *in) {
    const int64_t n = (int64_t)nang * G * nx * ny * 4;
    hipLaunchKernelGGL((k_psi_convert<real, double, true>), dim3(nblk(n, 256)), dim3(256), 0, s, nx, ny, G, nang, dq, abi,
                       in, (double *)nullptr);
}
template <typename real>
void run_psi_from_internal(hipStream_t s, int nx, int ny, int G, int nang, const int *dq, const real *in, double *abi) {
    const int64_t n = (int64_t)nang * G * nx * ny * 4;
    hipLaunchKernelGGL((k_psi_convert<real, double, false>), dim3(nblk(n, 256)), dim3(256), 0, s, nx, ny, G, nang, dq,
                       (const double *)nullptr, const_cast<real *>(in), abi);
}
void run_permute_dirs(hipStream_t s, int nang, int64_t per, const int *map, const double *in, double *out) {
    hipLaunchKernelGGL(k_permute_dirs, dim3(nblk(nang * per, 256)), dim3(256), 0, s, nang, per, map, in, out);
}
void run_adjoint_dsig(hipStream_t s, int dim, int nx, int ny, int G, int nang, const double *hx, const double *hy,
                      const double *lam, const double *emis, const double *psi, double *dsig) {
    hipLaunchKernelGGL(k_adjoint_dsig, dim3(nblk((int64_t)nx * ny * G, 128)), dim3(128), 0, s, dim, nx, ny, G, nang, hx,
                       hy, lam, emis, psi, dsig);
}
void run_adj_prep(hipStream_t s, int nn, int npc, int G, int nang, const double *nu, double a, double c, double dt,
                  const double *T, const double *sig, const double *cvn, const double *w, const double *psi, double *emis,
                  double *dE, double *D, double *phi) {
    hipLaunchKernelGGL(k_adj_prep, dim3(nblk(nn, 128)), dim3(128), 0, s, nn, npc, G, nang, nu, a, c, dt, T, sig, cvn, w,
                       psi, emis, dE, D, phi);
}
void run_adj_dJdI(hipStream_t s, int dim, int nx, int ny, int G, int nang, const double *om, const double *w,
                  const double *hy, double dt, double *out) {
    const int64_t n = (int64_t)nang * G * nx * ny * (dim == 2 ? 4 : 2);
    hipLaunchKernelGGL(k_adj_dJdI, dim3(nblk(n, 256)), dim3(256), 0, s, dim, nx, ny, G, nang, om, w, hy, dt, out);
}
void run_adj_src(hipStream_t s, int dim, int nx, int ny, int G, int nang, const double *hx, const double *hy,
                 const double *wang, const double *dJdI, const double *lam_next, double icdt, const double *sig,
                 const double *tau, double *src) {
    const int64_t n = (int64_t)nang * G * nx * ny * (dim == 2 ? 4 : 2);
    hipLaunchKernelGGL(k_adj_src, dim3(nblk(n, 256)), dim3(256), 0, s, dim, nx, ny, G, nang, hx, hy, wang, dJdI,
                       lam_next, icdt, sig, tau, src);
}
void run_adj_tau(hipStream_t s, int dim, int nx, int ny, int G, int nang, const double *hx, const double *hy,
                 const double *sig, const double *dE, const double *ST, const double *D, const double *lam,
                 const double *tau, double *tau_new, double *part, double *out2) {
    const int nn = nx * ny * (dim == 2 ? 4 : 2), nb = nblk(nn, 256);
    hipLaunchKernelGGL(k_adj_tau, dim3(nb), dim3(256), 0, s, dim, nx, ny, G, nang, hx, hy, sig, dE, ST, D, lam, tau,
                       tau_new, part);
    hipLaunchKernelGGL(k_sum_pairs, dim3(1), dim3(64), 0, s, nb, part, out2);
}
void run_aa_columns(hipStream_t s, int nn, const double *tau, const double *g, double *fprev, double *gprev,
                    double *dF, double *dG, bool first) {
    hipLaunchKernelGGL(k_aa_columns, dim3(nblk(nn, 256)), dim3(256), 0, s, nn, tau, g, fprev, gprev, dF, dG,
                       first ? 1 : 0);
}
void run_aa_dots(hipStream_t s, int nn, int ncols, const AASlots &sl, const double *cols, const double *a,
                 const double *b, double *part, double *out) {
    const int nb = nblk(nn, 256);
    hipLaunchKernelGGL(k_aa_dots, dim3(nb), dim3(256), 0, s, nn, ncols, sl, cols, a, b, part);
    hipLaunchKernelGGL(k_aa_dots_finish, dim3(1), dim3(64), 0, s, nb, 2 * ncols, part, out);
}
void run_aa_update(hipStream_t s, int nn, int ncols, const AASlots &sl, const AACoef &gm, const double *dG,
                   const double *g, double *tau) {
    hipLaunchKernelGGL(k_aa_update, dim3(nblk(nn, 256)), dim3(256), 0, s, nn, ncols, sl, gm, dG, g, tau);
}
void run_adj_cell(hipStream_t s, int npc, int ncell, int G, int model, double clip_lo, double clip_hi, double dt,
                  const double *dsig, const double *tau, const double *phi, const double *emis, const double *sig,
                  const double *cvn, const double *T, const double *Tp, double *gs_cell, double *gcv_node,
                  double *ST_prev) {
    hipLaunchKernelGGL(k_adj_cell, dim3(nblk(ncell, 128)), dim3(128), 0, s, npc, ncell, G, model, clip_lo, clip_hi, dt,
                       dsig, tau, phi, emis, sig, cvn, T, Tp, gs_cell, gcv_node, ST_prev);
}
void run_region_sums(hipStream_t s, int nreg, int ncell, int npc, const int *region, const double *gs_cell,
                     const double *gcv_node, double *grad_s0, double *grad_cv) {
    hipLaunchKernelGGL(k_region_sums, dim3(nblk(nreg, 64)), dim3(64), 0, s, nreg, ncell, npc, region, gs_cell, gcv_node,
                       grad_s0, grad_cv);
}
void run_adj_energy_weights(hipStream_t s, int dim, int nx, int npc, int nn, const double *hx, const double *hy,
                            const double *cvn, double *wc) {
    hipLaunchKernelGGL(k_adj_energy_weights, dim3(nblk(nn, 256)), dim3(256), 0, s, dim, nx, npc, nn, hx, hy, cvn, wc);
}
void run_mul(hipStream_t s, int64_t n, const double *a, const double *b, double *out) {
    hipLaunchKernelGGL(k_mul, dim3(nblk(n, 256)), dim3(256), 0, s, n, a, b, out);
}
void run_dot(hipStream_t s, int64_t n, const double *a, const double *b, double *part256, double *out) {
    hipLaunchKernelGGL(k_dot_blocks, dim3(256), dim3(256), 0, s, n, a, b, part256);
    hipLaunchKernelGGL(k_sum_blocks, dim3(1), dim3(64), 0, s, 256, part256, out);
}
void run_add_scalar(hipStream_t s, int64_t n, const double *a, double v, double *out) {
    hipLaunchKernelGGL(k_add_scalar, dim3(nblk(n, 256)), dim3(256), 0, s, n, a, v, out);
}
template <typename real>
void run_copy_from(hipStream_t s, int64_t n, const real *src, double *dst) {
    hipLaunchKernelGGL(k_copy_from<real>, dim3(nblk(n, 256)), dim3(256), 0, s, n, src, dst);
}
template <typename real>
void run_moments_finalize(hipStream_t s, int nx, int ny, const ChunkRanges &cr, const int *qc_dir, const double *dirs,
                          const real *part, double *sigq, double *mom, const int *gate) {
    const int nb = (ny + BAND_ROWS - 1) / BAND_ROWS, NT = nx + BAND_ROWS - 1;
    hipLaunchKernelGGL(k_moments_quadrant<real>, dim3(4 * nb * ((NT + 3) / 4)), dim3(256), 0, s, nx, ny, cr, qc_dir,
                       dirs, part, mom, sigq, gate);
    const int64_t nn = (int64_t)nx * ny * 4;
    hipLaunchKernelGGL(k_moments_sigma, dim3(nblk(nn, 256)), dim3(256), 0, s, nn, (const double *)sigq, mom, gate);
}
template <typename real>
void launch_sweep1d(const Sweep1DArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_sweep1d<real>, dim3(nblk(a.nang * a.G, 64)), dim3(64), 0, s, a);
    SMRT_HIP(hipGetLastError());
}
template <typename real>
void run_moments1d(hipStream_t s, int nx, int G, int nang, const real *mw, const double *sig, const real *psi, double *mom) {
    hipLaunchKernelGGL(k_moments1d<real>, dim3(nblk(2 * nx, 128)), dim3(128), 0, s, nx, G, nang, mw, sig, psi, mom);
}
void run_psi_EF(hipStream_t s, int nn, int dim, int G, int nang, const double *om, const double *w, double c,
                const double *psi, double *E, double *F) {
    hipLaunchKernelGGL(k_psi_EF, dim3(nblk(nn, 128)), dim3(128), 0, s, nn, dim, G, nang, om, w, c, psi, E, F);
}

#define INST(real)                                                                                                  \
    template void run_opacity<real>(hipStream_t, int, int, int, const double *, const int *, int, const double *,  \
                                    double, double, const double *, double, double *, real *);                      \
    template void run_source<real>(hipStream_t, int, int, int, const double *, const double *, double, double,      \
                                   const double *, real *, real *, double *, double *, const int *);                \
    template void run_fill_inflow<real>(hipStream_t, int, int, int, int, int, const double *, real *);              \
    template void run_reflect<real>(hipStream_t, int, int, int, int, int, int, const int *, const double *,         \
                                    const double *, const int *, const real *, real *, double *);                   \
    template void run_stab2d<real>(hipStream_t, int, int, int, const double *, const double *, double, real *);     \
    template void run_opacity_tab2d<real>(hipStream_t, int, int, int, const double *, const int *, int,            \
                                          const double *, double, double, const double *, double, double *, real *); \
    template void run_qtab2d<real, double>(hipStream_t, int, int, int, const double *, int64_t, int64_t, real *,   \
                                           const int *);                                                          \
    template void run_copy_to<real>(hipStream_t, int64_t, const double *, real *);                                  \
    template void run_copy_from<real>(hipStream_t, int64_t, const real *, double *);                                \
    template void run_qiso_to_internal<real>(hipStream_t, int, int, int, const double *, real *);                   \
    template void run_sig_to_internal<real>(hipStream_t, int, int, const double *, const double *, real *);         \
    template void run_psi_to_internal<real>(hipStream_t, int, int, int, int, const int *, const double *, real *);  \
    template void run_psi_from_internal<real>(hipStream_t, int, int, int, int, const int *, const real *, double *); \
    template void run_moments_finalize<real>(hipStream_t, int, int, const ChunkRanges &, const int *,              \
                                              const double *, const real *, double *, double *, const int *);                                                        \
    template void launch_sweep1d<real>(const Sweep1DArgs &, hipStream_t);                                           \
    template void run_moments1d<real>(hipStream_t, int, int, int, const real *, const double *, const real *, double *);
INST(float)
template void run_qtab2d<float, float>(hipStream_t, int, int, int, const float *, int64_t, int64_t, float *,
                                       const int *);
INST(double)

}  // namespace smrt
