// Lumped bilinear DG S_N sweep on unstructured quadrilateral meshes.
//
// What is computed (Eq. dgsn_transport on general convex quadrilaterals,
// every form lumped by the vertex (trapezoid) rule): for every (direction
// d, group g) and cell K, the 4x4 local system
//   A_lm = sigt w_l delta_lm - w_m Omega.grad(phi_l)(x_m)
//        + delta_lm sum_{edges e of l, Omega.nL_e > 0} Omega.nL_e / 2
//   b_l  = w_l (q_l + inv_c_dt I*_l) - sum_{edges e of l, Omega.nL_e < 0} Omega.nL_e / 2 I_up
// with, at vertex m of the bilinear map from the reference square,
// w_m = det J_m / 4 and w_m grad(phi_l)(x_m) = w_m J_m^-T grad_ref(phi_l)(m);
// nL_e is edge e's outward normal times its length; I_up is the upwind
// neighbour's value at the same vertex, or the boundary inflow.
//
// Schedule.  The paper's refined meshes (trapezoidal corner cells) break the
// diagonal wavefront of the rectilinear kernel, so cells are ordered per
// direction by their upwind dependencies: the host assigns every (direction,
// cell) pair a level (one more than the deepest upwind neighbour, Kahn's
// algorithm; a cycle is an error) and lists each direction's cells level
// by level.  One launch sweeps everything: a workgroup of 1024 threads takes
// one direction and a block of 4 groups and walks that direction's levels,
// 256 cells x 4 groups at a time, with a workgroup barrier between levels
// (the upwind values a level reads were written by the same workgroup), so
// a level costs a barrier and one round of loads instead of a launch.  The
// host also classifies each edge of each pair as inflow or outflow, so the
// device never disagrees with the schedule about an edge nearly parallel to
// the direction.  The local system is solved in registers by Gaussian
// elimination with partial pivoting.  Angular flux layout [d][g][node],
// node = 4 cell + local vertex (counter-clockwise), as the ABI's.
#include <cmath>
#include <type_traits>
#include <cstring>
#include <memory>
#include <numeric>

#include "lo.h"
#include "tables.h"

namespace smrt {

struct QGeomCell {
    double K[4][2][2];   // K_m = w_m J_m^-T (w_m grad phi_l(x_m) = K_m grad_ref phi_l(m))
    double w[4];         // lumped weights
    double nL[4][2];     // edge e (vertex e -> e+1): outward normal x length
};

struct QArgs {
    int nc, G, nang, NB;
    const QGeomCell *geo;
    const int *dcell;             // [d][nc]: direction d's cells, level by level
    const int *dlev;              // level offsets into a direction's cells, direction d's at dlev_base[d]
    const int *dlev_base;         // [nang + 1]: direction d has levels dlev_base[d+1] - dlev_base[d] - 1
    const unsigned char *flags;   // [d][cell]: bit e inflow edge, bit 4+e outflow edge
    const int *upw;               // [cell][edge][2]: upwind node (>= 0) or -(1 + boundary node)
    const double *om;             // [nang][3]
    const void *sig_t;            // [cell][G], sweep precision
    const void *q;                // [g][node], sweep precision
    const void *psi_prev;         // [d][g][node], sweep precision
    const void *inflow;           // [d][g][NB], sweep precision
    const double *par;            // [0] inv_c_dt, [1] 1 if psi_prev holds I*, else 0 (set per sweep)
    void *psi;                    // [d][g][node], sweep precision
};

// reference gradient of phi_l at reference vertex m ((0,0), (1,0), (1,1), (0,1))
__host__ __device__ inline void qref_grad(int l, int m, double &gx, double &gy) {
    const double xi = (m == 1 || m == 2) ? 1.0 : 0.0, eta = (m >= 2) ? 1.0 : 0.0;
    switch (l) {
        case 0: gx = -(1 - eta); gy = -(1 - xi); break;
        case 1: gx = 1 - eta; gy = -xi; break;
        case 2: gx = eta; gy = xi; break;
        default: gx = -eta; gy = 1 - xi; break;
    }
}

// the unit (direction d, group g, cell c): local system, elimination, store
template <typename real>
__device__ __forceinline__ void qsolve_unit(const QArgs &A, int d, int g, int c) {
    const int nn = 4 * A.nc;
    const real mu = (real)A.om[3 * d], eta = (real)A.om[3 * d + 1];
    const QGeomCell &K = A.geo[c];
    const unsigned fl = A.flags[(int64_t)d * A.nc + c];
    real *psi = static_cast<real *>(A.psi);
    const int64_t slab = ((int64_t)d * A.G + g) * nn;
    const real *sig_t = static_cast<const real *>(A.sig_t), *q = static_cast<const real *>(A.q);
    const real *psi_prev = static_cast<const real *>(A.psi_prev), *inflow = static_cast<const real *>(A.inflow);
    const real st = sig_t[(int64_t)c * A.G + g];
    real M[4][4], b[4];
    const real icdt = (real)A.par[0];
    const bool has_prev = A.par[1] != 0.0;
    // the cell's 4 nodes are contiguous and 4-value aligned in every [d][g][node] slab
    using r4 = typename std::conditional<sizeof(real) == 4, float4, double4>::type;
    r4 pv{};
    if (has_prev) pv = *reinterpret_cast<const r4 *>(psi_prev + slab + 4 * c);
    // the cell's 8 upwind entries, loaded with its flags rather than after them
    // (one dependent round trip fewer before the upwind values)
    const int4 ua = *reinterpret_cast<const int4 *>(A.upw + 8 * (int64_t)c);
    const int4 ub = *reinterpret_cast<const int4 *>(A.upw + 8 * (int64_t)c + 4);
    const int upw8[8] = {ua.x, ua.y, ua.z, ua.w, ub.x, ub.y, ub.z, ub.w};
    const real pp[4] = {pv.x, pv.y, pv.z, pv.w};
    const r4 qv = *reinterpret_cast<const r4 *>(q + (int64_t)g * nn + 4 * c);
    const real qa[4] = {qv.x, qv.y, qv.z, qv.w};
#pragma unroll
    for (int l = 0; l < 4; ++l) {
        real ql = qa[l];
        if (has_prev) ql += icdt * pp[l];
        b[l] = (real)K.w[l] * ql;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            double gx, gy;
            qref_grad(l, m, gx, gy);
            // w_m grad phi_l(x_m) = K_m grad_ref phi_l(m)
            const real ax = (real)(K.K[m][0][0] * gx + K.K[m][0][1] * gy);
            const real ay = (real)(K.K[m][1][0] * gx + K.K[m][1][1] * gy);
            M[l][m] = (l == m ? st * (real)K.w[l] : real(0)) - (mu * ax + eta * ay);
        }
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const real on = real(0.5) * (mu * (real)K.nL[e][0] + eta * (real)K.nL[e][1]);
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int l = (e + j) & 3;
            if ((fl >> (4 + e)) & 1) {
                M[l][l] += on;
            } else if ((fl >> e) & 1) {
                const int u = upw8[2 * e + j];
                const real up = u >= 0 ? psi[slab + u] : inflow[((int64_t)d * A.G + g) * A.NB + (-u - 1)];
                b[l] -= on * up;
            }
        }
    }
    // Gaussian elimination with partial pivoting (4x4, in registers)
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        int p = k;
#pragma unroll
        for (int r = k + 1; r < 4; ++r)
            if (fabs(M[r][k]) > fabs(M[p][k])) p = r;
#pragma unroll
        for (int r = k + 1; r < 4; ++r) {
            if (r != p) continue;
#pragma unroll
            for (int cc = 0; cc < 4; ++cc) { const real tmp = M[k][cc]; M[k][cc] = M[r][cc]; M[r][cc] = tmp; }
            const real tmp = b[k]; b[k] = b[r]; b[r] = tmp;
        }
#pragma unroll
        for (int r = k + 1; r < 4; ++r) {
            const real f = M[r][k] / M[k][k];
#pragma unroll
            for (int cc = k; cc < 4; ++cc) M[r][cc] -= f * M[k][cc];
            b[r] -= f * b[k];
        }
    }
    real x[4];
#pragma unroll
    for (int k = 3; k >= 0; --k) {
        real s = b[k];
#pragma unroll
        for (int cc = k + 1; cc < 4; ++cc) s -= M[k][cc] * x[cc];
        x[k] = s / M[k][k];
    }
    r4 xv;
    xv.x = x[0]; xv.y = x[1]; xv.z = x[2]; xv.w = x[3];
    *reinterpret_cast<r4 *>(psi + slab + 4 * c) = xv;
}


// One workgroup per (direction, block of QGB groups): the direction's levels
// in order, a workgroup barrier between levels.
constexpr int QGB = 4, QSWEEP_THREADS = 1024, QCELLS = QSWEEP_THREADS / QGB;
template <typename real>
__global__ void __launch_bounds__(QSWEEP_THREADS) k_qsweep_dir(QArgs A) {
    const int ngb = (A.G + QGB - 1) / QGB;
    const int d = blockIdx.x / ngb, g = (blockIdx.x % ngb) * QGB + (int)(threadIdx.x % QGB);
    const int slot = threadIdx.x / QGB;
    const int *cells = A.dcell + (int64_t)d * A.nc;
    const int l0 = A.dlev_base[d], l1 = A.dlev_base[d + 1];
    for (int L = l0; L + 1 < l1; ++L) {
        const int c0 = A.dlev[L], c1 = A.dlev[L + 1];
        for (int k = c0 + slot; k < c1; k += QCELLS)
            if (g < A.G) qsolve_unit<real>(A, d, g, cells[k]);
        __syncthreads();   // this level's outflow before the next level reads it
    }
}

// double inputs to the sweep's precision
__global__ void k_qto_f32(int64_t n, const double *in, float *out) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) out[i] = (float)in[i];
}

template <typename real>
__global__ void k_qcopy_out(int64_t n, const real *in, double *out) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) out[i] = (double)in[i];
}

// Gray angular moments of a swept intensity per node (Sec. 2's moment sums
// with the quadrature weights, over all groups), split by the quadrant of the
// direction as on the rectilinear path: rows 6q..6q+5 hold the sums of
// w f I with f = 1, mu, eta, mu^2, mu eta, eta^2 over the directions of
// quadrant q (0: mu, eta > 0; 1: mu < 0 < eta; 2: both < 0; 3: the rest),
// rows 24..26 the sums of sigma w (1, mu, eta) I with sigma the cell's
// group opacity.  A dependency-level sweep cannot fuse these sums: the
// directions of one node are solved in different launches.
//
// A workgroup is 4 waves over the same 64 nodes, wave q taking the
// directions of quadrant q (so every wave streams a quarter of the
// intensity, 4x the waves of one thread per node).  Each wave writes its
// quadrant's six rows; the opacity-weighted sums of the four quadrants meet
// in LDS and are added in quadrant order.  Directions, then groups, are
// summed in index order in FP64, every intensity value read once (coalesced
// along the nodes).
template <typename real>
__global__ void __launch_bounds__(256) k_qmoments(int nang, int G, int nn, const double *om, const double *wq,
                                                  const double *sig, const real *psi, double *mom) {
    __shared__ double part[4][3][64];
    const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int n = blockIdx.x * 64 + lane;
    const bool live = n < nn;
    const int nc = live ? n : nn - 1;       // a clamped node keeps the loads in range; its sums are not stored
    double s0[6] = {0, 0, 0, 0, 0, 0}, s1[3] = {0, 0, 0};
    const double *sg = sig + (int64_t)(nc >> 2) * G;
    for (int d = 0; d < nang; ++d) {
        const double mu = om[3 * d], eta = om[3 * d + 1];
        const int qd = (mu > 0 && eta > 0) ? 0 : (mu < 0 && eta > 0) ? 1 : (mu < 0 && eta < 0) ? 2 : 3;
        if (qd != q) continue;              // uniform over the wave
        const double w = wq[d];
        const double f[6] = {1.0, mu, eta, mu * mu, mu * eta, eta * eta};
        const real *I = psi + (int64_t)d * G * nn + nc;
        double t = 0.0, a = 0.0;
#pragma unroll 4
        for (int g = 0; g < G; ++g) {
            const double v = (double)I[(int64_t)g * nn];
            t += v;
            a += sg[g] * v;
        }
#pragma unroll
        for (int m = 0; m < 6; ++m) s0[m] += w * f[m] * t;
        s1[0] += w * a;
        s1[1] += w * mu * a;
        s1[2] += w * eta * a;
    }
    if (live) {
#pragma unroll
        for (int m = 0; m < 6; ++m) mom[(int64_t)(6 * q + m) * nn + n] = s0[m];
    }
#pragma unroll
    for (int m = 0; m < 3; ++m) part[q][m][lane] = s1[m];
    __syncthreads();
    if (q == 0 && live) {
#pragma unroll
        for (int m = 0; m < 3; ++m)
            mom[(int64_t)(24 + m) * nn + n] = ((part[0][m][lane] + part[1][m][lane]) + part[2][m][lane]) + part[3][m][lane];
    }
}

// ---------------------------------------------------------------------------
// The unaccelerated time step on the mesh (Algorithm 1 without the
// low-order solve): small kernels around the sweep and the moments.
// ---------------------------------------------------------------------------
// the ABI's emission q[node][G] to the sweep's q[g][node] (a cell's 4 nodes
// contiguous, one vector load per unit), in the sweep precision
template <typename real>
__global__ void k_qtranspose(int nn, int G, const double *q_ng, real *q) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= (int64_t)nn * G) return;
    const int64_t g = i / nn, n = i - g * nn;
    q[i] = (real)q_ng[n * G + g];
}
// sigma_t = sigma + 1/(c dt) per (cell, group), in the sweep precision
template <typename real>
__global__ void k_qsigt(int64_t n, const double *sig, double icdt, real *sigt) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) sigt[i] = (real)(sig[i] + icdt);
}
// equilibrium intensity: every direction takes B_g(T_n)/4pi (qn[g][node])
template <typename real>
__global__ void k_qequilibrium(int nang, int G, int nn, const double *qn, real *psi) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= (int64_t)nang * G * nn) return;
    psi[i] = (real)qn[i % ((int64_t)G * nn)];
}
// E = phi / c and sigma_E = sum_g sigma_g phi_g / phi (sigma_P where phi = 0)
// from the 27 nodal moments (phi: the four quadrants' rows 0, 6, 12, 18)
__global__ void k_qho(int nn, double c, const double *mom, const double *sigP, double *E, double *sigE) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= nn) return;
    const double phi = ((mom[n] + mom[6 * (int64_t)nn + n]) + mom[12 * (int64_t)nn + n]) + mom[18 * (int64_t)nn + n];
    E[n] = phi / c;
    if (sigE) sigE[n] = phi > 0.0 ? mom[24 * (int64_t)nn + n] / phi : sigP[n];
}
// |Ta - Tb|^2 + |Ea - Eb|^2: 256 block partials, then one block sums them (fixed order)
constexpr int QRED = 256;
__global__ void k_qdiff2(int n, const double *Ta, const double *Tb, const double *Ea, const double *Eb, double *part) {
    __shared__ double sh[QRED];
    double s = 0.0;
    for (int i = blockIdx.x * QRED + threadIdx.x; i < n; i += QRED * QRED) {
        const double dT = Ta[i] - Tb[i], dE = Ea[i] - Eb[i];
        s += dT * dT + dE * dE;
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int k = QRED / 2; k > 0; k >>= 1) {
        if (threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}
__global__ void k_qsum(const double *part, double *out) {
    __shared__ double sh[QRED];
    sh[threadIdx.x] = part[threadIdx.x];
    __syncthreads();
    for (int k = QRED / 2; k > 0; k >>= 1) {
        if (threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0];
}
__global__ void k_qzero4(int *p) { if (threadIdx.x < 4) p[threadIdx.x] = 0; }

}  // namespace smrt

using namespace smrt;

struct smrt_qmesh {
    std::string err;
    int nv = 0, nc = 0, nang = 0, G = 0, NB = 0, nlev = 0;
    bool fp32 = false;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    DevBuf<QGeomCell> geo;
    DevBuf<int> dcell, dlev, dlev_base;   // per direction: cells by level, level offsets
    DevBuf<unsigned char> flags, psi;
    DevBuf<int> upw;
    DevBuf<double> om, sig_t, q, psi_prev, inflow, out, par, wq, sig_m, mom;
    DevBuf<float> sig_t32, q32, psi_prev32, inflow32;   // FP32 sweeps read their inputs in FP32
    bool swept = false;       // psi holds the intensity of a finished sweep
    // time step: materials, state (T, E, I at nodes; I in the sweep precision)
    bool have_mat = false, have_state = false;
    int nreg = 0, model = 1;
    double clip_lo = 0.0, clip_hi = 0.0, a = 1.0, c = 1.0;
    DevBuf<int> region, eflags;
    DevBuf<double> sigma0, nu, cvn, T, E, Tstar, Tl, El, Tn, En, sig_step, qn, sigP, sigF, sigE, ones, red;
    DevBuf<unsigned char> psi_state;
    double *hbuf = nullptr;   // pinned: [0] iterate change, [1..4] elimination flags (as ints)
    ~smrt_qmesh() {
        if (hbuf) (void)hipHostFree(hbuf);
        if (own_stream && stream) (void)hipStreamDestroy(stream);
    }
    // the sweep from I* = prev (nullptr: the uploaded psi_prev) into out (nullptr: psi)
    void launch_sweep(hipStream_t s, const void *prev = nullptr, void *out = nullptr);
};

void smrt_qmesh::launch_sweep(hipStream_t s, const void *prev, void *out_psi) {
    QArgs A{};
    A.nc = nc; A.G = G; A.nang = nang; A.NB = NB;
    A.geo = geo.p; A.dcell = dcell.p; A.dlev = dlev.p; A.dlev_base = dlev_base.p; A.flags = flags.p; A.upw = upw.p;
    A.om = om.p;
    if (fp32) {
        A.sig_t = sig_t32.p; A.q = q32.p; A.psi_prev = psi_prev32.p; A.inflow = inflow32.p;
    } else {
        A.sig_t = sig_t.p; A.q = q.p; A.psi_prev = psi_prev.p; A.inflow = inflow.p;
    }
    A.par = par.p; A.psi = psi.p;
    if (prev) A.psi_prev = prev;
    if (out_psi) A.psi = out_psi;
    const dim3 grid((unsigned)(nang * ((G + QGB - 1) / QGB)));
    if (fp32) hipLaunchKernelGGL(k_qsweep_dir<float>, grid, dim3(QSWEEP_THREADS), 0, s, A);
    else hipLaunchKernelGGL(k_qsweep_dir<double>, grid, dim3(QSWEEP_THREADS), 0, s, A);
}

static thread_local std::string g_qmesh_error;

template <typename F>
static smrt_status qguard(smrt_qmesh *m, F &&f) {
    try {
        f();
        return SMRT_OK;
    } catch (const smrt::Error &e) {
        if (m) m->err = e.msg;
        g_qmesh_error = e.msg;
        return e.st;
    } catch (const std::bad_alloc &) {
        if (m) m->err = "host allocation failed";
        g_qmesh_error = "host allocation failed";
        return SMRT_E_OUT_OF_MEMORY;
    } catch (...) {
        if (m) m->err = "unexpected exception";
        g_qmesh_error = "unexpected exception";
        return SMRT_E_DEVICE;
    }
}

static void qrequire(bool ok, const std::string &msg) {
    if (!ok) throw smrt::Error(SMRT_E_INVALID_ARG, msg);
}

extern "C" smrt_status smrt_qmesh_create(int n_vertices, const double *xy, int n_cells, const int32_t *cells,
                                         const smrt_quad_desc *quad, int G, smrt_precision precision, void *hip_stream,
                                         smrt_qmesh **out) {
    if (!out) { g_qmesh_error = "out is NULL"; return SMRT_E_INVALID_ARG; }
    *out = nullptr;
    std::unique_ptr<smrt_qmesh> h(new (std::nothrow) smrt_qmesh());
    if (!h) { g_qmesh_error = "host allocation failed"; return SMRT_E_OUT_OF_MEMORY; }
    smrt_qmesh *m = h.get();
    const smrt_status st = qguard(m, [&] {
        qrequire(n_vertices > 0 && n_cells > 0 && xy && cells && quad && quad->omega && quad->w, "NULL or empty mesh");
        qrequire(G >= 1, "G must be >= 1");
        qrequire(precision == SMRT_FP64 || precision == SMRT_FP32, "unknown precision");
        qrequire((int64_t)n_cells * 4 < (1ll << 30), "mesh too large");
        const int nang = quad->n_angles;
        qrequire(nang > 0, "no directions");
        double ws = 0.0;
        for (int d = 0; d < nang; ++d) {
            qrequire(quad->w[d] > 0.0, "quadrature weights must be > 0");
            ws += quad->w[d];
        }
        qrequire(std::fabs(ws - 4.0 * M_PI) <= 1e-12 * 4.0 * M_PI, "quadrature weights must sum to 4 pi");
        m->nv = n_vertices; m->nc = n_cells; m->nang = nang; m->G = G; m->fp32 = precision == SMRT_FP32;
        const int nc = n_cells;
        for (int k = 0; k < 4 * nc; ++k) qrequire(cells[k] >= 0 && cells[k] < n_vertices, "vertex index out of range");
        // geometry
        std::vector<QGeomCell> geo(nc);
        for (int c = 0; c < nc; ++c) {
            double X[4][2];
            for (int l = 0; l < 4; ++l) { X[l][0] = xy[2 * cells[4 * c + l]]; X[l][1] = xy[2 * cells[4 * c + l] + 1]; }
            for (int mv = 0; mv < 4; ++mv) {
                double J[2][2] = {{0, 0}, {0, 0}};
                for (int l = 0; l < 4; ++l) {
                    double gx, gy;
                    qref_grad(l, mv, gx, gy);
                    for (int i = 0; i < 2; ++i) { J[i][0] += X[l][i] * gx; J[i][1] += X[l][i] * gy; }
                }
                const double det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
                qrequire(det > 0.0, "cells must be convex quadrilaterals listed counter-clockwise");
                const double w = det / 4.0;
                geo[c].w[mv] = w;
                // w J^-T = (1/4) [[J11, -J10], [-J01, J00]]
                geo[c].K[mv][0][0] = J[1][1] / 4.0;
                geo[c].K[mv][0][1] = -J[1][0] / 4.0;
                geo[c].K[mv][1][0] = -J[0][1] / 4.0;
                geo[c].K[mv][1][1] = J[0][0] / 4.0;
            }
            for (int e = 0; e < 4; ++e) {
                const int b = (e + 1) & 3;
                geo[c].nL[e][0] = X[b][1] - X[e][1];
                geo[c].nL[e][1] = -(X[b][0] - X[e][0]);
            }
        }
        // connectivity: pair edges by their sorted vertex pair
        struct E { int a, b, c, e; };
        std::vector<E> es(4 * (size_t)nc);
        for (int c = 0; c < nc; ++c)
            for (int e = 0; e < 4; ++e) {
                const int v0 = cells[4 * c + e], v1 = cells[4 * c + ((e + 1) & 3)];
                es[4 * c + e] = {std::min(v0, v1), std::max(v0, v1), c, e};
            }
        std::sort(es.begin(), es.end(), [](const E &x, const E &y) {
            return x.a != y.a ? x.a < y.a : x.b != y.b ? x.b < y.b : x.c != y.c ? x.c < y.c : x.e < y.e;
        });
        std::vector<int> nb(4 * (size_t)nc, -1);
        for (size_t k = 0; k < es.size(); ++k) {
            if (k + 1 < es.size() && es[k].a == es[k + 1].a && es[k].b == es[k + 1].b) {
                qrequire(!(k + 2 < es.size() && es[k + 2].a == es[k].a && es[k + 2].b == es[k].b),
                         "an edge is shared by more than two cells");
                nb[4 * es[k].c + es[k].e] = es[k + 1].c;
                nb[4 * es[k + 1].c + es[k + 1].e] = es[k].c;
                ++k;
            }
        }
        std::vector<int> upw(8 * (size_t)nc);
        int nbe = 0;
        for (int c = 0; c < nc; ++c)
            for (int e = 0; e < 4; ++e) {
                const int n2 = nb[4 * c + e];
                for (int j = 0; j < 2; ++j) {
                    const int l = (e + j) & 3;
                    if (n2 >= 0) {
                        int l2 = 0;
                        while (l2 < 4 && cells[4 * n2 + l2] != cells[4 * c + l]) ++l2;
                        upw[(4 * c + e) * 2 + j] = 4 * n2 + l2;
                    } else {
                        upw[(4 * c + e) * 2 + j] = -(1 + 2 * nbe + j);
                    }
                }
                if (n2 < 0) ++nbe;
            }
        m->NB = 2 * nbe;
        // per direction: edge classes and levels (Kahn); then the (d, cell) pairs by level
        std::vector<unsigned char> flags((size_t)nang * nc, 0);
        std::vector<int> level((size_t)nang * nc, 0), indeg(nc), queue(nc);
        int maxlev = 0;
        for (int d = 0; d < nang; ++d) {
            const double mu = quad->omega[3 * d], eta = quad->omega[3 * d + 1];
            for (int c = 0; c < nc; ++c) {
                unsigned f = 0;
                int deg = 0;
                for (int e = 0; e < 4; ++e) {
                    const double on = mu * geo[c].nL[e][0] + eta * geo[c].nL[e][1];
                    if (on < 0.0) {
                        f |= 1u << e;
                        if (nb[4 * c + e] >= 0) ++deg;
                    } else if (on > 0.0) {
                        f |= 1u << (4 + e);
                    }
                }
                flags[(size_t)d * nc + c] = (unsigned char)f;
                indeg[c] = deg;
            }
            int head = 0, tail = 0;
            for (int c = 0; c < nc; ++c) if (indeg[c] == 0) { queue[tail++] = c; level[(size_t)d * nc + c] = 0; }
            while (head < tail) {
                const int c = queue[head++];
                const int lv = level[(size_t)d * nc + c];
                maxlev = std::max(maxlev, lv);
                for (int e = 0; e < 4; ++e) {
                    const int n2 = nb[4 * c + e];
                    if (n2 < 0 || !((flags[(size_t)d * nc + c] >> (4 + e)) & 1)) continue;
                    int &ln = level[(size_t)d * nc + n2];
                    ln = std::max(ln, lv + 1);
                    if (--indeg[n2] == 0) queue[tail++] = n2;
                }
            }
            qrequire(tail == nc, "the upwind dependencies of a direction form a cycle");
        }
        m->nlev = maxlev + 1;
        // per direction: its cells sorted by level and the level offsets
        std::vector<int> dcell((size_t)nang * nc), dlev, dlev_base(nang + 1, 0);
        for (int d = 0; d < nang; ++d) {
            int nl = 0;
            for (int c = 0; c < nc; ++c) nl = std::max(nl, level[(size_t)d * nc + c] + 1);
            std::vector<int> count(nl + 1, 0);
            for (int c = 0; c < nc; ++c) count[level[(size_t)d * nc + c] + 1]++;
            std::partial_sum(count.begin(), count.end(), count.begin());
            std::vector<int> fill(count.begin(), count.end() - 1);
            for (int c = 0; c < nc; ++c) dcell[(size_t)d * nc + fill[level[(size_t)d * nc + c]]++] = c;
            dlev.insert(dlev.end(), count.begin(), count.end());
            dlev_base[d + 1] = (int)dlev.size();
        }
        // device
        if (hip_stream) m->stream = static_cast<hipStream_t>(hip_stream);
        else { SMRT_HIP(hipStreamCreate(&m->stream)); m->own_stream = true; }
        const int64_t nn = 4 * (int64_t)nc, npsi = (int64_t)nang * G * nn;
        m->geo.alloc(nc);
        m->dcell.alloc((int64_t)dcell.size());
        m->dlev.alloc((int64_t)dlev.size());
        m->dlev_base.alloc(nang + 1);
        m->flags.alloc((int64_t)flags.size());
        m->upw.alloc((int64_t)upw.size());
        m->om.alloc(3 * (int64_t)nang);
        SMRT_HIP(hipMemcpy(m->geo.p, geo.data(), sizeof(QGeomCell) * nc, hipMemcpyHostToDevice));
        SMRT_HIP(hipMemcpy(m->dcell.p, dcell.data(), sizeof(int) * dcell.size(), hipMemcpyHostToDevice));
        SMRT_HIP(hipMemcpy(m->dlev.p, dlev.data(), sizeof(int) * dlev.size(), hipMemcpyHostToDevice));
        SMRT_HIP(hipMemcpy(m->dlev_base.p, dlev_base.data(), sizeof(int) * (nang + 1), hipMemcpyHostToDevice));
        SMRT_HIP(hipMemcpy(m->flags.p, flags.data(), flags.size(), hipMemcpyHostToDevice));
        SMRT_HIP(hipMemcpy(m->upw.p, upw.data(), sizeof(int) * upw.size(), hipMemcpyHostToDevice));
        SMRT_HIP(hipMemcpy(m->om.p, quad->omega, sizeof(double) * 3 * nang, hipMemcpyHostToDevice));
        m->wq.alloc(nang);
        SMRT_HIP(hipMemcpy(m->wq.p, quad->w, sizeof(double) * nang, hipMemcpyHostToDevice));
        m->sig_t.alloc((int64_t)nc * G);
        m->q.alloc(nn * G);
        m->psi_prev.alloc(npsi);
        m->inflow.alloc(std::max<int64_t>((int64_t)nang * G * m->NB, 1));
        m->out.alloc(npsi);
        m->par.alloc(2);
        m->psi.alloc(npsi * (m->fp32 ? 4 : 8));
        if (m->fp32) {
            m->sig_t32.alloc((int64_t)nc * G);
            m->q32.alloc(nn * G);
            m->psi_prev32.alloc(npsi);
            m->inflow32.alloc(std::max<int64_t>((int64_t)nang * G * m->NB, 1));
        }
    });
    if (st != SMRT_OK) return st;
    *out = h.release();
    return SMRT_OK;
}

extern "C" void smrt_qmesh_destroy(smrt_qmesh *m) { delete m; }

extern "C" const char *smrt_qmesh_last_error(const smrt_qmesh *m) { return m ? m->err.c_str() : g_qmesh_error.c_str(); }

extern "C" smrt_status smrt_qmesh_info(const smrt_qmesh *m, int *n_boundary_nodes, int *n_levels) {
    if (!m) { g_qmesh_error = "mesh is NULL"; return SMRT_E_INVALID_ARG; }
    if (n_boundary_nodes) *n_boundary_nodes = m->NB;
    if (n_levels) *n_levels = m->nlev;
    return SMRT_OK;
}

extern "C" smrt_status smrt_qmesh_sweep(smrt_qmesh *m, const double *sig_t, const double *q_iso, const double *psi_prev,
                                        double inv_c_dt, const double *inflow, double *psi_out, double *ms_kernel) {
    if (!m) { g_qmesh_error = "mesh is NULL"; return SMRT_E_INVALID_ARG; }
    return qguard(m, [&] {
        qrequire(sig_t && q_iso && psi_out, "NULL input or output");
        qrequire(std::isfinite(inv_c_dt) && inv_c_dt >= 0.0, "inv_c_dt must be finite and >= 0");
        const int64_t nn = 4 * (int64_t)m->nc, npsi = (int64_t)m->nang * m->G * nn;
        for (int64_t k = 0; k < (int64_t)m->nc * m->G; ++k)
            qrequire(std::isfinite(sig_t[k]) && sig_t[k] > 0.0, "sig_t must be finite and > 0");
        hipStream_t s = m->stream;
        m->swept = false;
        SMRT_HIP(hipMemcpyAsync(m->sig_t.p, sig_t, sizeof(double) * m->nc * m->G, hipMemcpyHostToDevice, s));
        // q_iso is staged in the output buffer (free until the sweep's copy-out) and
        // transposed to the sweep's [g][node] layout below
        SMRT_HIP(hipMemcpyAsync(m->out.p, q_iso, sizeof(double) * nn * m->G, hipMemcpyHostToDevice, s));
        {
            const dim3 gq((unsigned)((nn * m->G + 255) / 256));
            if (m->fp32) hipLaunchKernelGGL(k_qtranspose<float>, gq, dim3(256), 0, s, (int)nn, m->G,
                                            (const double *)m->out.p, m->q32.p);
            else hipLaunchKernelGGL(k_qtranspose<double>, gq, dim3(256), 0, s, (int)nn, m->G, (const double *)m->out.p,
                                    m->q.p);
        }
        if (psi_prev) SMRT_HIP(hipMemcpyAsync(m->psi_prev.p, psi_prev, sizeof(double) * npsi, hipMemcpyHostToDevice, s));
        if (inflow) SMRT_HIP(hipMemcpyAsync(m->inflow.p, inflow, sizeof(double) * m->nang * m->G * m->NB,
                                            hipMemcpyHostToDevice, s));
        else if (m->NB) SMRT_HIP(hipMemsetAsync(m->inflow.p, 0, sizeof(double) * m->nang * m->G * m->NB, s));
        if (m->fp32) {
            auto to32 = [&](int64_t n, const double *in, float *out) {
                if (n > 0) hipLaunchKernelGGL(k_qto_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, in, out);
            };
            to32((int64_t)m->nc * m->G, m->sig_t.p, m->sig_t32.p);
            if (psi_prev) to32(npsi, m->psi_prev.p, m->psi_prev32.p);
            to32((int64_t)m->nang * m->G * m->NB, m->inflow.p, m->inflow32.p);
        }
        const double par[2] = {inv_c_dt, psi_prev ? 1.0 : 0.0};
        SMRT_HIP(hipMemcpyAsync(m->par.p, par, sizeof(par), hipMemcpyHostToDevice, s));
        hipEvent_t e0, e1;
        SMRT_HIP(hipEventCreate(&e0));
        if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); throw Error(SMRT_E_DEVICE, "hipEventCreate failed"); }
        SMRT_HIP(hipEventRecord(e0, s));
        m->launch_sweep(s);
        SMRT_HIP(hipGetLastError());
        SMRT_HIP(hipEventRecord(e1, s));
        if (m->fp32) hipLaunchKernelGGL(k_qcopy_out<float>, dim3((unsigned)((npsi + 255) / 256)), dim3(256), 0, s, npsi,
                                        (const float *)m->psi.p, m->out.p);
        else hipLaunchKernelGGL(k_qcopy_out<double>, dim3((unsigned)((npsi + 255) / 256)), dim3(256), 0, s, npsi,
                                (const double *)m->psi.p, m->out.p);
        SMRT_HIP(hipMemcpyAsync(psi_out, m->out.p, sizeof(double) * npsi, hipMemcpyDeviceToHost, s));
        SMRT_HIP(hipStreamSynchronize(s));
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (ms_kernel) *ms_kernel = ms;
        m->swept = true;
    });
}

extern "C" smrt_status smrt_qmesh_moments(smrt_qmesh *m, const double *sig, double *mom_out, double *ms_kernel) {
    if (!m) { g_qmesh_error = "mesh is NULL"; return SMRT_E_INVALID_ARG; }
    return qguard(m, [&] {
        qrequire(sig && mom_out, "NULL input or output");
        qrequire(m->swept, "no sweep has run on this mesh");
        for (int64_t k = 0; k < (int64_t)m->nc * m->G; ++k)
            qrequire(std::isfinite(sig[k]) && sig[k] >= 0.0, "sig must be finite and >= 0");
        const int nn = 4 * m->nc;
        if (!m->sig_m.p) m->sig_m.alloc((int64_t)m->nc * m->G);
        if (!m->mom.p) m->mom.alloc(27 * (int64_t)nn);
        hipStream_t s = m->stream;
        SMRT_HIP(hipMemcpyAsync(m->sig_m.p, sig, sizeof(double) * m->nc * m->G, hipMemcpyHostToDevice, s));
        hipEvent_t e0, e1;
        SMRT_HIP(hipEventCreate(&e0));
        if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); throw Error(SMRT_E_DEVICE, "hipEventCreate failed"); }
        SMRT_HIP(hipEventRecord(e0, s));
        const dim3 grid((unsigned)((nn + 63) / 64));     // 64 nodes per workgroup of 4 quadrant waves
        if (m->fp32) hipLaunchKernelGGL(k_qmoments<float>, grid, dim3(256), 0, s, m->nang, m->G, nn, m->om.p, m->wq.p,
                                        m->sig_m.p, (const float *)m->psi.p, m->mom.p);
        else hipLaunchKernelGGL(k_qmoments<double>, grid, dim3(256), 0, s, m->nang, m->G, nn, m->om.p, m->wq.p,
                                m->sig_m.p, (const double *)m->psi.p, m->mom.p);
        SMRT_HIP(hipGetLastError());
        SMRT_HIP(hipEventRecord(e1, s));
        SMRT_HIP(hipMemcpyAsync(mom_out, m->mom.p, sizeof(double) * 27 * nn, hipMemcpyDeviceToHost, s));
        SMRT_HIP(hipStreamSynchronize(s));
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (ms_kernel) *ms_kernel = ms;
    });
}

// ---------------------------------------------------------------------------
// Time step on the mesh: the unaccelerated scheme of Algorithm 1
// ---------------------------------------------------------------------------
extern "C" smrt_status smrt_qmesh_set_materials(smrt_qmesh *m, const int32_t *region, int n_regions, int model,
                                                const double *sigma0, double clip_lo, double clip_hi, const double *cv,
                                                const double *nu_edges, double a, double c) {
    if (!m) { g_qmesh_error = "mesh is NULL"; return SMRT_E_INVALID_ARG; }
    return qguard(m, [&] {
        qrequire(region && sigma0 && cv && nu_edges, "NULL input");
        upload_series_coefficients();   // the emission's Planck series, as at context creation
        qrequire(n_regions >= 1, "n_regions must be >= 1");
        qrequire(model == 0 || model == 1, "model must be 0 (tabulated) or 1 (power law)");
        qrequire(std::isfinite(a) && a > 0.0 && std::isfinite(c) && c > 0.0, "a and c must be finite and > 0");
        const int nc = m->nc, G = m->G, nn = 4 * nc;
        for (int k = 0; k < nc; ++k) qrequire(region[k] >= 0 && region[k] < n_regions, "region index out of range");
        const int ns = model == 0 ? n_regions * G : n_regions;
        for (int k = 0; k < ns; ++k) qrequire(std::isfinite(sigma0[k]) && sigma0[k] >= 0.0, "sigma0 must be >= 0");
        if (model == 1) qrequire(clip_lo > 0.0 && clip_hi >= clip_lo, "clip bounds must satisfy 0 < lo <= hi");
        for (int r = 0; r < n_regions; ++r) qrequire(std::isfinite(cv[r]) && cv[r] > 0.0, "c_v must be > 0");
        qrequire(nu_edges[0] >= 0.0, "group bounds must be >= 0");
        for (int g = 0; g < G; ++g) qrequire(nu_edges[g + 1] > nu_edges[g], "group bounds must increase");
        hipStream_t s = m->stream;
        SMRT_HIP(hipStreamSynchronize(s));
        m->nreg = n_regions; m->model = model; m->clip_lo = clip_lo; m->clip_hi = clip_hi; m->a = a; m->c = c;
        m->region.alloc(nc);
        m->sigma0.alloc(ns);
        m->nu.alloc(G + 1);
        std::vector<double> cvn(nn);
        for (int n = 0; n < nn; ++n) cvn[n] = cv[region[n / 4]];
        m->cvn.alloc(nn);
        SMRT_HIP(hipMemcpy(m->region.p, region, sizeof(int) * nc, hipMemcpyHostToDevice));
        SMRT_HIP(hipMemcpy(m->sigma0.p, sigma0, sizeof(double) * ns, hipMemcpyHostToDevice));
        SMRT_HIP(hipMemcpy(m->nu.p, nu_edges, sizeof(double) * (G + 1), hipMemcpyHostToDevice));
        SMRT_HIP(hipMemcpy(m->cvn.p, cvn.data(), sizeof(double) * nn, hipMemcpyHostToDevice));
        if (!m->T.p) {
            for (auto *v : {&m->T, &m->E, &m->Tstar, &m->Tl, &m->El, &m->Tn, &m->En, &m->sigP, &m->sigF, &m->sigE})
                v->alloc(nn);
            m->sig_step.alloc((int64_t)nc * G);
            m->qn.alloc((int64_t)nn * G);
            m->red.alloc(QRED + 1);
            m->eflags.alloc(4);
            m->psi_state.alloc((int64_t)m->nang * G * nn * (m->fp32 ? 4 : 8));
            if (!m->mom.p) m->mom.alloc(27 * (int64_t)nn);
            std::vector<double> ones((size_t)nc * G, 1.0);
            m->ones.alloc((int64_t)nc * G);
            SMRT_HIP(hipMemcpy(m->ones.p, ones.data(), sizeof(double) * ones.size(), hipMemcpyHostToDevice));
            SMRT_HIP(hipHostMalloc((void **)&m->hbuf, 8 * sizeof(double), hipHostMallocDefault));
        }
        m->have_mat = true;
        m->have_state = false;
    });
}

extern "C" smrt_status smrt_qmesh_set_state(smrt_qmesh *m, const double *T, const double *psi) {
    if (!m) { g_qmesh_error = "mesh is NULL"; return SMRT_E_INVALID_ARG; }
    return qguard(m, [&] {
        qrequire(m->have_mat, "smrt_qmesh_set_materials must come first");
        qrequire(T != nullptr, "T is NULL");
        const int nc = m->nc, G = m->G, nang = m->nang, nn = 4 * nc;
        const int64_t npsi = (int64_t)nang * G * nn;
        for (int n = 0; n < nn; ++n) qrequire(std::isfinite(T[n]) && T[n] > 0.0, "T must be finite and > 0");
        hipStream_t s = m->stream;
        SMRT_HIP(hipMemcpyAsync(m->T.p, T, sizeof(double) * nn, hipMemcpyHostToDevice, s));
        if (psi) {
            SMRT_HIP(hipMemcpyAsync(m->psi_prev.p, psi, sizeof(double) * npsi, hipMemcpyHostToDevice, s));
            if (m->fp32) hipLaunchKernelGGL(k_qto_f32, dim3((unsigned)((npsi + 255) / 256)), dim3(256), 0, s, npsi,
                                            (const double *)m->psi_prev.p, (float *)m->psi_state.p);
            else SMRT_HIP(hipMemcpyAsync(m->psi_state.p, m->psi_prev.p, sizeof(double) * npsi, hipMemcpyDeviceToDevice, s));
        } else {
            // isotropic equilibrium B_g(T_n)/4pi: the emission of a unit opacity
            run_source<double>(s, nn, 4, G, m->T.p, m->nu.p, m->a, m->c, m->ones.p, nullptr, m->qn.p, m->sigP.p,
                               m->sigF.p);
            const dim3 grid((unsigned)((npsi + 255) / 256));
            if (m->fp32) hipLaunchKernelGGL(k_qequilibrium<float>, grid, dim3(256), 0, s, nang, G, nn,
                                            (const double *)m->qn.p, (float *)m->psi_state.p);
            else hipLaunchKernelGGL(k_qequilibrium<double>, grid, dim3(256), 0, s, nang, G, nn, (const double *)m->qn.p,
                                    (double *)m->psi_state.p);
        }
        // E = sum_d w_d sum_g I / c of the state's intensity
        const dim3 gm((unsigned)((nn + 63) / 64));
        if (m->fp32) hipLaunchKernelGGL(k_qmoments<float>, gm, dim3(256), 0, s, nang, G, nn, m->om.p, m->wq.p,
                                        m->ones.p, (const float *)m->psi_state.p, m->mom.p);
        else hipLaunchKernelGGL(k_qmoments<double>, gm, dim3(256), 0, s, nang, G, nn, m->om.p, m->wq.p, m->ones.p,
                                (const double *)m->psi_state.p, m->mom.p);
        hipLaunchKernelGGL(k_qho, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s, nn, m->c,
                           (const double *)m->mom.p, (const double *)nullptr, m->E.p, (double *)nullptr);
        SMRT_HIP(hipGetLastError());
        SMRT_HIP(hipStreamSynchronize(s));
        m->have_state = true;
    });
}

extern "C" smrt_status smrt_qmesh_get_state(smrt_qmesh *m, double *T, double *E, double *psi) {
    if (!m) { g_qmesh_error = "mesh is NULL"; return SMRT_E_INVALID_ARG; }
    return qguard(m, [&] {
        qrequire(m->have_state, "no state (smrt_qmesh_set_state)");
        const int nn = 4 * m->nc;
        const int64_t npsi = (int64_t)m->nang * m->G * nn;
        hipStream_t s = m->stream;
        if (T) SMRT_HIP(hipMemcpyAsync(T, m->T.p, sizeof(double) * nn, hipMemcpyDeviceToHost, s));
        if (E) SMRT_HIP(hipMemcpyAsync(E, m->E.p, sizeof(double) * nn, hipMemcpyDeviceToHost, s));
        if (psi) {
            const dim3 grid((unsigned)((npsi + 255) / 256));
            if (m->fp32) hipLaunchKernelGGL(k_qcopy_out<float>, grid, dim3(256), 0, s, npsi,
                                            (const float *)m->psi_state.p, m->out.p);
            else hipLaunchKernelGGL(k_qcopy_out<double>, grid, dim3(256), 0, s, npsi, (const double *)m->psi_state.p,
                                    m->out.p);
            SMRT_HIP(hipMemcpyAsync(psi, m->out.p, sizeof(double) * npsi, hipMemcpyDeviceToHost, s));
        }
        SMRT_HIP(hipStreamSynchronize(s));
    });
}

extern "C" smrt_status smrt_qmesh_step(smrt_qmesh *m, double dt, const double *inflow, const smrt_options *opt,
                                       smrt_step_stats *stats) {
    if (!m) { g_qmesh_error = "mesh is NULL"; return SMRT_E_INVALID_ARG; }
    smrt_status result = SMRT_OK;
    const smrt_status st0 = qguard(m, [&] {
        qrequire(m->have_state, "no state (smrt_qmesh_set_state)");
        qrequire(opt != nullptr, "options are NULL");
        qrequire(std::isfinite(dt) && dt > 0.0, "dt must be finite and > 0");
        qrequire(opt->scheme == SMRT_UNACCELERATED,
                 "unstructured meshes step with the unaccelerated scheme only (the SM closures need half-range "
                 "sums for every face normal)");
        qrequire(!opt->fixup, "the unstructured sweep has no negative-flux fixup");
        qrequire(opt->max_outer >= 1 && opt->max_elim >= 1, "iteration caps must be >= 1");
        const int nc = m->nc, G = m->G, nang = m->nang, nn = 4 * nc;
        const int64_t npsi = (int64_t)nang * G * nn, nin = (int64_t)nang * G * m->NB;
        hipStream_t s = m->stream;
        hipEvent_t e0, e1;
        SMRT_HIP(hipEventCreate(&e0));
        if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); throw Error(SMRT_E_DEVICE, "hipEventCreate failed"); }
        struct Ev { hipEvent_t a, b; ~Ev() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); } } ev{e0, e1};
        SMRT_HIP(hipEventRecord(e0, s));
        const double icdt = 1.0 / (m->c * dt);
        // fixed inflow of the step (vacuum when NULL), in the sweep precision
        if (inflow) SMRT_HIP(hipMemcpyAsync(m->inflow.p, inflow, sizeof(double) * nin, hipMemcpyHostToDevice, s));
        else if (nin) SMRT_HIP(hipMemsetAsync(m->inflow.p, 0, sizeof(double) * nin, s));
        if (m->fp32 && nin)
            hipLaunchKernelGGL(k_qto_f32, dim3((unsigned)((nin + 255) / 256)), dim3(256), 0, s, nin,
                               (const double *)m->inflow.p, m->inflow32.p);
        const double par[2] = {icdt, 1.0};
        SMRT_HIP(hipMemcpyAsync(m->par.p, par, sizeof(par), hipMemcpyHostToDevice, s));
        // opacity at the start-of-step temperature, sigma_t in the sweep precision
        run_opacity<double>(s, nc, 4, G, m->T.p, m->region.p, m->model, m->sigma0.p, m->clip_lo, m->clip_hi, m->nu.p,
                            0.0, m->sig_step.p, (double *)nullptr);
        const int64_t ncg = (int64_t)nc * G;
        const dim3 gcg((unsigned)((ncg + 255) / 256));
        if (m->fp32) hipLaunchKernelGGL(k_qsigt<float>, gcg, dim3(256), 0, s, ncg, (const double *)m->sig_step.p, icdt,
                                        m->sig_t32.p);
        else hipLaunchKernelGGL(k_qsigt<double>, gcg, dim3(256), 0, s, ncg, (const double *)m->sig_step.p, icdt,
                                m->sig_t.p);
        SMRT_HIP(hipMemcpyAsync(m->Tstar.p, m->T.p, sizeof(double) * nn, hipMemcpyDeviceToDevice, s));
        SMRT_HIP(hipMemcpyAsync(m->Tl.p, m->T.p, sizeof(double) * nn, hipMemcpyDeviceToDevice, s));
        SMRT_HIP(hipMemcpyAsync(m->El.p, m->E.p, sizeof(double) * nn, hipMemcpyDeviceToDevice, s));
        smrt_step_stats st{};
        const dim3 gn((unsigned)((nn + 255) / 256)), gm((unsigned)((nn + 63) / 64));
        const dim3 gq((unsigned)(((int64_t)nn * G + 255) / 256));
        double first = -1.0;
        for (int l = 1; l <= opt->max_outer; ++l) {
            run_source<double>(s, nn, 4, G, m->Tl.p, m->nu.p, m->a, m->c, m->sig_step.p, nullptr, m->qn.p, m->sigP.p,
                               m->sigF.p);
            if (m->fp32) {
                hipLaunchKernelGGL(k_qto_f32, gq, dim3(256), 0, s, (int64_t)nn * G, (const double *)m->qn.p, m->q32.p);
                m->launch_sweep(s, m->psi_state.p, m->psi.p);
                hipLaunchKernelGGL(k_qmoments<float>, gm, dim3(256), 0, s, nang, G, nn, m->om.p, m->wq.p,
                                   (const double *)m->sig_step.p, (const float *)m->psi.p, m->mom.p);
            } else {
                SMRT_HIP(hipMemcpyAsync(m->q.p, m->qn.p, sizeof(double) * nn * G, hipMemcpyDeviceToDevice, s));
                m->launch_sweep(s, m->psi_state.p, m->psi.p);
                hipLaunchKernelGGL(k_qmoments<double>, gm, dim3(256), 0, s, nang, G, nn, m->om.p, m->wq.p,
                                   (const double *)m->sig_step.p, (const double *)m->psi.p, m->mom.p);
            }
            hipLaunchKernelGGL(k_qho, gn, dim3(256), 0, s, nn, m->c, (const double *)m->mom.p,
                               (const double *)m->sigP.p, m->En.p, m->sigE.p);
            SMRT_HIP(hipMemcpyAsync(m->Tn.p, m->Tl.p, sizeof(double) * nn, hipMemcpyDeviceToDevice, s));
            hipLaunchKernelGGL(k_qzero4, dim3(1), dim3(64), 0, s, m->eflags.p);
            run_eliminate(s, nn, m->a, m->c, dt, opt->elim_rtol, opt->max_elim, opt->T_floor, m->cvn.p, m->sigE.p,
                          m->sigP.p, m->En.p, m->Tstar.p, m->Tn.p, m->eflags.p);
            hipLaunchKernelGGL(k_qdiff2, dim3(QRED), dim3(QRED), 0, s, nn, (const double *)m->Tn.p,
                               (const double *)m->Tl.p, (const double *)m->En.p, (const double *)m->El.p, m->red.p);
            hipLaunchKernelGGL(k_qsum, dim3(1), dim3(QRED), 0, s, (const double *)m->red.p, m->red.p + QRED);
            SMRT_HIP(hipGetLastError());
            SMRT_HIP(hipMemcpyAsync(m->hbuf, m->red.p + QRED, sizeof(double), hipMemcpyDeviceToHost, s));
            SMRT_HIP(hipMemcpyAsync(m->hbuf + 1, m->eflags.p, 4 * sizeof(int), hipMemcpyDeviceToHost, s));
            SMRT_HIP(hipMemcpyAsync(m->Tl.p, m->Tn.p, sizeof(double) * nn, hipMemcpyDeviceToDevice, s));
            SMRT_HIP(hipMemcpyAsync(m->El.p, m->En.p, sizeof(double) * nn, hipMemcpyDeviceToDevice, s));
            SMRT_HIP(hipStreamSynchronize(s));
            st.outer++;
            int fl[4];
            std::memcpy(fl, m->hbuf + 1, sizeof(fl));
            const double diff = std::sqrt(m->hbuf[0]);
            if (fl[1] > st.elim_max) st.elim_max = fl[1];
            if (fl[2]) st.hit_max = 1;
            if (fl[0]) {
                m->err = "no positive temperature root in the energy balance";
                result = SMRT_E_NONPHYSICAL;
                break;
            }
            if (!std::isfinite(diff)) {
                m->err = "non-finite outer iterate";
                result = SMRT_E_NONPHYSICAL;
                break;
            }
            if (opt->fixed_outer > 0) {
                if (l >= opt->fixed_outer) break;
                continue;
            }
            if (l == 1) first = diff;
            if (diff == 0.0 || (l > 1 && diff < opt->eps_outer * first)) break;
            if (l == opt->max_outer) st.hit_max = 1;
        }
        // the new state: the last iterate and the last sweep's intensity (a
        // non-physical iterate leaves the state as it was before the step)
        if (result == SMRT_OK) {
            SMRT_HIP(hipMemcpyAsync(m->T.p, m->Tl.p, sizeof(double) * nn, hipMemcpyDeviceToDevice, s));
            SMRT_HIP(hipMemcpyAsync(m->E.p, m->El.p, sizeof(double) * nn, hipMemcpyDeviceToDevice, s));
            SMRT_HIP(hipMemcpyAsync(m->psi_state.p, m->psi.p, npsi * (m->fp32 ? 4 : 8), hipMemcpyDeviceToDevice, s));
        }
        SMRT_HIP(hipEventRecord(e1, s));
        SMRT_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        st.t_total_ms = ms;
        m->swept = true;
        if (stats) *stats = st;
        if (result == SMRT_OK && opt->strict && st.hit_max) {
            result = SMRT_E_NOT_CONVERGED;
            m->err = "iteration cap reached";
        }
    });
    if (st0 != SMRT_OK) return st0;
    if (result != SMRT_OK) g_qmesh_error = m->err;
    return result;
}
