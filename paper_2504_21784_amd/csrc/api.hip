// C ABI and host runtime of the SM-TRT library: context creation and
// validation, device memory, the launch plan of the sweep, and the
// backward-Euler step driver (Algorithm 1 of the paper).
#include <cmath>
#include <cstring>
#include <memory>
#include <numeric>
#include <algorithm>
#include <cstdio>
#include <mutex>

#include "lo.h"
#include "tables.h"

using namespace smrt;

static thread_local std::string g_last_error;

struct smrt_ctx {
    std::string err;
    // problem description (host copies)
    int dim = 0, nx = 0, ny = 0, nang = 0, G = 0, nn = 0, ncell = 0, npc = 0, NB = 0, nreg = 0;
    std::vector<double> xe, ye, om, w, nu;
    double a = 1, c = 1;
    std::vector<int> region;
    int model = 0;
    std::vector<double> sigma0, cv;
    double clip_lo = 0, clip_hi = 0;
    int bc_kind[4] = {0, 0, 0, 0};
    double bc_T[4] = {0, 0, 0, 0};
    std::vector<double> bc_explicit;   // [4][G]
    smrt_options opt{};
    hipStream_t stream = nullptr;
    bool own_stream = false;
    bool fp32 = false;
    size_t rs = 8;
    // geometry on the device
    DevBuf<double> d_nu, d_hx64, d_hy64, d_sigma0, d_cvn, d_om, d_w, d_sideval, d_Tb, d_explicit;
    DevBuf<int> d_region, d_dir_quad, d_kind;
    DevBuf<int> d_opposite;       // direction with -Omega (adjoint sweeps)
    bool have_opposite = false;
    DevBuf<int> d_mirror;         // [2][nang]: direction with mu -> -mu (x sides), eta -> -eta (y sides); -1 if none
    bool have_mirror[2] = {false, false};
    int refl = 0;                 // bit s: side s is reflective
    DevBuf<double> d_bmom;        // [NB][3] incoming moments of the reflective sides' inflow
    DevBuf<unsigned char> d_hx, d_hy, d_dirs, d_mu_w;
    // sweep plan
    int NW = 0, NBW = 1, K = 1, R = 0, NQC = 0, nbands = 0, NT = 0, n_bgroups = 0, n_wg = 0;
    int user_NW = 0, user_NBW = 0, user_K = 0, wg_per_cu = 0;
    std::vector<int> qc_quad;
    std::vector<int> slot_pair;   // pairs (d, g)
    ChunkRanges chunks{};         // chunk range of each quadrant
    DevBuf<int> d_qc_quad, d_qc_dir, d_slot_pair, d_ctr, d_lctr;
    DevBuf<double> d_dirs64;      // per direction, FP64: mu, eta, w, w mu, w eta, w mu^2, w mu eta, w eta^2
    std::vector<int> qc_dir;      // direction of each chunk
    DevBuf<int2> d_tasks;         // single-problem task list (0, band group * NQC + chunk)
    DevBuf<unsigned char> d_psi[2], d_part, d_qiso, d_sig2, d_inflow;
    DevBuf<uint64_t> d_trace;
    int cur = 0;
    // FP64 state and work arrays
    DevBuf<double> d_qnat;   // q_iso [G][node] at the sweep precision (2D: gathered into the skewed tables)
    DevBuf<double> d_sigq;   // per-quadrant sigma-weighted moments [4][3][node] (2D finalisation)
    DevBuf<double> d_T, d_E, d_F, d_Eho, d_Fho, d_mom, d_sig, d_sigP, d_sigF, d_clos, d_Tl, d_El, d_Tn, d_En, d_Tstar,
        d_Estar, d_Fstar, d_sigEho;
    LoSolver lo;
    double alpha[2] = {0, 0}, S1[4] = {0, 0, 0, 0}, S2[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    bool have_state = false;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    int *h_ctr = nullptr;          // pinned copy of the sweep's protocol counters
    double *h_small = nullptr;     // pinned staging for small device-to-host reads (32 doubles)
    ~smrt_ctx() {
        if (stream) (void)hipStreamSynchronize(stream);
        if (h_ctr) (void)hipHostFree(h_ctr);
        if (h_small) (void)hipHostFree(h_small);
        if (ev0) (void)hipEventDestroy(ev0);
        if (ev1) (void)hipEventDestroy(ev1);
        if (own_stream && stream) (void)hipStreamDestroy(stream);
    }
};

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
template <typename F>
static smrt_status guard(smrt_ctx *ctx, F &&f) {
    try {
        f();
        return SMRT_OK;
    } catch (const smrt::Error &e) {
        if (ctx) ctx->err = e.msg;
        g_last_error = e.msg;
        return e.st;
    } catch (const std::bad_alloc &) {
        if (ctx) ctx->err = "host allocation failed";
        g_last_error = "host allocation failed";
        return SMRT_E_OUT_OF_MEMORY;
    } catch (...) {
        if (ctx) ctx->err = "unexpected exception";
        g_last_error = "unexpected exception";
        return SMRT_E_DEVICE;
    }
}

static void require(bool ok, const std::string &msg) {
    if (!ok) throw smrt::Error(SMRT_E_INVALID_ARG, msg);
}

static void h2d(void *dst, const void *src, size_t bytes, hipStream_t s) {
    if (bytes) SMRT_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s));
}
static void d2h(void *dst, const void *src, size_t bytes, hipStream_t s) {
    if (bytes) SMRT_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s));
}

__global__ void k_zero_int(int *p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}
__global__ void k_init_ctr(int *p) {
    p[0] = 0;
    p[1] = 0;
    p[2] = 1;
    p[3] = 0;
}
// HO energy density and sigma_E from moments (2D rows 0,6,12,18 / 24; 1D rows 0,3 / 6)
__global__ void k_ho_from_mom(int nn, int dim, double c, const double *mom, const double *sigP, double *E, double *F,
                              double *sigE) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= nn) return;
    double phi, fx, fy = 0.0, sp;
    if (dim == 2) {
        phi = mom[n] + mom[6 * (int64_t)nn + n] + mom[12 * (int64_t)nn + n] + mom[18 * (int64_t)nn + n];
        fx = mom[1 * (int64_t)nn + n] + mom[7 * (int64_t)nn + n] + mom[13 * (int64_t)nn + n] + mom[19 * (int64_t)nn + n];
        fy = mom[2 * (int64_t)nn + n] + mom[8 * (int64_t)nn + n] + mom[14 * (int64_t)nn + n] + mom[20 * (int64_t)nn + n];
        sp = mom[24 * (int64_t)nn + n];
    } else {
        phi = mom[n] + mom[3 * (int64_t)nn + n];
        fx = mom[1 * (int64_t)nn + n] + mom[4 * (int64_t)nn + n];
        sp = mom[6 * (int64_t)nn + n];
    }
    if (E) E[n] = phi / c;
    if (F) {
        F[dim * n] = fx;
        if (dim == 2) F[dim * n + 1] = fy;
    }
    if (sigE) sigE[n] = phi > 0.0 ? sp / phi : sigP[n];
}

static int nblk(int64_t n, int b = 256) { return (int)((n + b - 1) / b); }

// ---------------------------------------------------------------------------
// launch plan of the 2D sweep
// ---------------------------------------------------------------------------
// waves a sweep workgroup may have: a wave's registers bound it (16 bytes of
// intensity per lane and node take twice the registers)
static int max_waves(bool fp32, int k) { return (fp32 ? 4 : 8) * k >= 16 ? 8 : 16; }

static void plan_sweep(smrt_ctx *x) {
    if (x->dim != 2) return;
    std::vector<std::vector<int>> qdirs(4);
    for (int d = 0; d < x->nang; ++d) {
        const double mu = x->om[3 * d], eta = x->om[3 * d + 1];
        const int q = (mu > 0 && eta > 0) ? 0 : (mu < 0 && eta > 0) ? 1 : (mu < 0 && eta < 0) ? 2 : 3;
        qdirs[q].push_back(d);
    }
    // A chunk = (quadrant, direction, block of 4 K NW groups): group block w
    // of a band sweeps groups 4K w .. 4K w + 4K - 1 of the chunk's block, its
    // channel c the groups 4k + c of that range.  Slots past G are inactive
    // (-1, -1).  A workgroup sweeps one chunk on NBW consecutive bands.
    int K = x->user_K ? x->user_K : 1, NW = x->user_NW ? x->user_NW : 1;
    x->nbands = (x->ny + BAND_ROWS - 1) / BAND_ROWS;
    int NBW = x->user_NBW;
    if (!NBW) {
        // the fewest bands (a power of two) that cover the mesh, within 16
        // waves; when they do not, band groups stacked across workgroups, each
        // with at most 8 compute waves (beside its publishing and receiving waves)
        // (FP64: at most 4 bands per group, which leaves each wave registers for
        // a deeper prefetch; measured faster at 256^2 S8 G16, 1.09 against 1.25 ms)
        const int cap = x->fp32 ? max_waves(x->fp32, K) : 4;
        NBW = 1;
        while (NBW < x->nbands && NW * NBW < cap) NBW *= 2;
        if (NBW < x->nbands)
            while (NBW > 1 && NW * NBW > 8) NBW /= 2;
    }
    require(NBW >= x->nbands || NW * NBW <= 8,
            "a chunk spanning several band groups allows at most 8 waves per band group (waves per band x bands)");
    x->NW = NW;
    x->NBW = NBW;
    x->K = K;
    x->R = 4 * NW * K;
    x->NT = x->nx + BAND_ROWS - 1;
    x->n_bgroups = (x->nbands + NBW - 1) / NBW;
    // a sweep wave addresses its 4K group slabs through 32-bit byte offsets
    // below 2^31 (offsets from 2^31 up mark lanes with no work)
    require((int64_t)CHANNELS * K * x->nbands * x->NT * BAND_ROWS * 4 * x->rs < (int64_t(1) << 31),
            "mesh too large for the sweep's 31-bit per-wave offsets");
    x->qc_quad.clear();
    x->qc_dir.clear();
    x->slot_pair.clear();
    const int GB = 4 * K * NW;
    const int ngb = (x->G + GB - 1) / GB;
    for (int q = 0; q < 4; ++q) {
        const int nd = (int)qdirs[q].size();
        for (int dq = 0; dq < nd; ++dq)
            for (int gb = 0; gb < ngb; ++gb) {
                x->qc_quad.push_back(q);
                x->qc_dir.push_back(qdirs[q][dq]);
                for (int w = 0; w < NW; ++w)
                    for (int c = 0; c < CHANNELS; ++c)
                        for (int k = 0; k < K; ++k) {
                            const int g = gb * GB + w * CHANNELS * K + CHANNELS * k + c;
                            const bool on = g < x->G;
                            x->slot_pair.push_back(on ? qdirs[q][dq] : -1);
                            x->slot_pair.push_back(on ? g : -1);
                        }
            }
    }
    x->NQC = (int)x->qc_quad.size();
    for (int q = 0; q <= 4; ++q) x->chunks.start[q] = 0;
    for (int qc = 0; qc < x->NQC; ++qc) x->chunks.start[x->qc_quad[qc] + 1] = qc + 1;
    for (int q = 1; q <= 4; ++q) x->chunks.start[q] = std::max(x->chunks.start[q], x->chunks.start[q - 1]);
    x->n_wg = x->NQC * x->n_bgroups;
    x->d_qc_quad.alloc(x->NQC);
    x->d_qc_dir.alloc(x->NQC);
    SMRT_HIP(hipMemcpy(x->d_qc_dir.p, x->qc_dir.data(), sizeof(int) * x->NQC, hipMemcpyHostToDevice));
    x->d_slot_pair.alloc((int64_t)x->slot_pair.size());
    SMRT_HIP(hipMemcpy(x->d_qc_quad.p, x->qc_quad.data(), sizeof(int) * x->NQC, hipMemcpyHostToDevice));
    SMRT_HIP(hipMemcpy(x->d_slot_pair.p, x->slot_pair.data(), sizeof(int) * x->slot_pair.size(), hipMemcpyHostToDevice));
    const int TW = x->fp32 ? 1 : 2;
    x->d_part.alloc((int64_t)x->NQC * x->nbands * x->NT * BAND_ROWS * PART_PER_CELL * x->rs);
    x->d_trace.alloc((int64_t)x->NQC * x->nbands * x->R * x->nx * 2 * TW);
    SMRT_HIP(hipMemset(x->d_trace.p, 0, sizeof(uint64_t) * x->d_trace.n));
    x->d_ctr.alloc(4);
    hipLaunchKernelGGL(k_init_ctr, dim3(1), dim3(1), 0, x->stream, x->d_ctr.p);
    // band-group-major task list: a band group is claimed only after every group below it
    std::vector<int2> tasks(x->n_wg);
    for (int t = 0; t < x->n_wg; ++t) tasks[t] = make_int2(0, t);
    if (x->n_bgroups == 1) {
        // No workgroup waits on another, so workgroup b sweeps tasks[b].  The
        // hardware hands workgroup b to XCD b mod 8; give each XCD a run of
        // chunks that read the same opacity and source tables (one quadrant
        // and group block, successive directions), so those tables are
        // fetched into each XCD's L2 once and shared by its workgroups.
        std::vector<int> by_table;
        for (int q = 0; q < 4; ++q)
            for (int gb = 0; gb < ngb; ++gb)
                for (int qc = x->chunks.start[q]; qc < x->chunks.start[q + 1]; ++qc)
                    if ((qc - x->chunks.start[q]) % ngb == gb) by_table.push_back(qc);
        const int n = x->n_wg, per = n / N_XCD, extra = n % N_XCD;
        for (int b = 0; b < n; ++b) {
            const int xcd = b % N_XCD, local = b / N_XCD;
            const int first = xcd < extra ? xcd * (per + 1) : extra * (per + 1) + (xcd - extra) * per;
            tasks[b] = make_int2(0, by_table[first + local]);
        }
    }
    x->d_tasks.alloc(x->n_wg);
    SMRT_HIP(hipMemcpy(x->d_tasks.p, tasks.data(), sizeof(int2) * x->n_wg, hipMemcpyHostToDevice));
    x->d_lctr.alloc(2);
    SMRT_HIP(hipMemset(x->d_lctr.p, 0, 2 * sizeof(int)));
    SMRT_HIP(hipStreamSynchronize(x->stream));
}

static int64_t psi_count(const smrt_ctx *x) {
    if (x->dim == 2) return (int64_t)x->nang * x->G * psi_slab(x->nx, x->ny);
    return (int64_t)x->nang * x->G * x->nn;
}

// ---------------------------------------------------------------------------
// sweep launch (2D: band kernel + moment finalisation; 1D: pair kernel + moments)
// ---------------------------------------------------------------------------
// Work memory of the 2D sweep kernels beyond inputs and outputs: moment
// partials, band trace words, the problem's counters and the launch ticket.
// By default the context's own buffers; the allocation-free entry point
// passes regions of its static array instead.
struct SweepScratch {
    void *part = nullptr;
    uint64_t *trace = nullptr;
    int *ctr = nullptr;    // [4]
    int *lctr = nullptr;   // [2]
};

static Sweep2DArgs sweep_args(const smrt_ctx *x, const void *psi_prev, void *psi_out, const void *sig2,
                              const void *qiso, const void *inflow, double icdt, const SweepScratch *ws = nullptr) {
    Sweep2DArgs a{};
    a.nx = x->nx; a.ny = x->ny; a.G = x->G; a.nbands = x->nbands; a.NT = x->NT;
    a.NW = x->NW; a.K = x->K; a.R = x->R; a.NQC = x->NQC; a.n_wg = x->n_wg; a.NB = x->NB;
    a.qc_quad = x->d_qc_quad.p;
    a.slot_pair = reinterpret_cast<const int2 *>(x->d_slot_pair.p);
    a.dirs = x->d_dirs.p; a.hx = x->d_hx.p; a.hy = x->d_hy.p;
    a.sig2 = sig2; a.qiso = qiso; a.psi_prev = psi_prev; a.psi_out = psi_out; a.inflow = inflow;
    a.inv_c_dt = icdt; a.part = x->d_part.p; a.trace = x->d_trace.p; a.ctr = x->d_ctr.p;
    if (ws) {
        a.part = ws->part;
        a.trace = ws->trace;
        a.ctr = ws->ctr;
    }
    return a;
}

static void finalize_moments(smrt_ctx *x, double *mom, const void *part = nullptr, const int *gate = nullptr) {
    if (!part) part = x->d_part.p;
    if (x->fp32) run_moments_finalize<float>(x->stream, x->nx, x->ny, x->chunks, x->d_qc_dir.p, x->d_dirs64.p, (const float *)part, x->d_sigq.p, mom, gate);
    else run_moments_finalize<double>(x->stream, x->nx, x->ny, x->chunks, x->d_qc_dir.p, x->d_dirs64.p, (const double *)part, x->d_sigq.p, mom, gate);
}

static void run_sweep(smrt_ctx *x, const void *psi_prev, void *psi_out, const void *sig2, const void *qiso,
                      const void *inflow, double icdt, const double *sig64, double *mom, bool finalize = true,
                      const SweepScratch *ws = nullptr) {
    if (x->dim == 2) {
        const Sweep2DArgs a = sweep_args(x, psi_prev, psi_out, sig2, qiso, inflow, icdt, ws);
        SweepLaunch L{};
        L.single = a;
        L.probs = nullptr;
        L.tasks = x->d_tasks.p;
        L.n_tasks = x->n_wg;
        L.NW = x->NW;
        L.NBW = x->NBW;
        L.K = x->K;
        L.wg_per_cu = x->wg_per_cu;
        L.lctr = ws ? ws->lctr : x->d_lctr.p;
        L.fixup = x->opt.fixup;
        L.xw = x->n_bgroups > 1 ? 1 : 0;
        L.static_order = x->n_bgroups == 1 ? 1 : 0;
        if (x->fp32) launch_sweep2d<float>(L, x->stream);
        else launch_sweep2d<double>(L, x->stream);
        if (finalize) finalize_moments(x, mom, ws ? ws->part : nullptr);
    } else {
        Sweep1DArgs a{};
        a.nx = x->nx; a.G = x->G; a.nang = x->nang; a.mu_w = x->d_mu_w.p; a.hx = x->d_hx.p;
        a.sig2 = sig2; a.qiso = qiso; a.psi_prev = psi_prev; a.psi_out = psi_out; a.inflow = inflow; a.inv_c_dt = icdt;
        a.fixup = x->opt.fixup;
        if (x->fp32) {
            launch_sweep1d<float>(a, x->stream);
            if (finalize) run_moments1d<float>(x->stream, x->nx, x->G, x->nang, (const float *)x->d_mu_w.p, sig64, (const float *)psi_out, mom);
        } else {
            launch_sweep1d<double>(a, x->stream);
            if (finalize) run_moments1d<double>(x->stream, x->nx, x->G, x->nang, (const double *)x->d_mu_w.p, sig64, (const double *)psi_out, mom);
        }
    }
}

// The sweep's error flag (counter 3) is set when a band-trace wait exceeded
// its bound.  fetch_sweep_flag queues its copy to pinned host memory;
// raise_sweep_flag reads it after the caller's wait, resets the protocol
// state so the context stays usable, and reports.
// A small device-to-host read (at most 32 doubles) that waits for the
// context stream: staged through the context's pinned buffer, never copied
// asynchronously into pageable (stack) memory.
static void read_small(smrt_ctx *x, void *dst, const void *src, size_t bytes) {
    if (bytes > 32 * sizeof(double)) throw smrt::Error(SMRT_E_INVALID_ARG, "read_small: more than 32 doubles");
    SMRT_HIP(hipMemcpyAsync(x->h_small, src, bytes, hipMemcpyDeviceToHost, x->stream));
    SMRT_HIP(hipStreamSynchronize(x->stream));
    std::memcpy(dst, x->h_small, bytes);
}

static void fetch_sweep_flag(smrt_ctx *x) {
    if (x->dim == 2) SMRT_HIP(hipMemcpyAsync(x->h_ctr, x->d_ctr.p, 4 * sizeof(int), hipMemcpyDeviceToHost, x->stream));
}

static void raise_sweep_flag(smrt_ctx *x) {
    if (x->dim != 2 || !x->h_ctr[3]) return;
    hipLaunchKernelGGL(k_init_ctr, dim3(1), dim3(1), 0, x->stream, x->d_ctr.p);
    SMRT_HIP(hipMemsetAsync(x->d_trace.p, 0, sizeof(uint64_t) * x->d_trace.n, x->stream));
    SMRT_HIP(hipStreamSynchronize(x->stream));
    const int bits = x->h_ctr[3];
    x->h_ctr[3] = 0;
    std::string which;
    if (bits & WAIT_START_GATE) which += " (band start)";
    if (bits & WAIT_TRACE) which += " (band trace)";
    throw smrt::Error(SMRT_E_DEVICE, "sweep band-trace wait exceeded its bound" + which);
}

static void check_sweep_flag(smrt_ctx *x) {
    if (x->dim != 2) return;
    fetch_sweep_flag(x);
    SMRT_HIP(hipStreamSynchronize(x->stream));
    raise_sweep_flag(x);
}

// rebuild the per-side inflow tables from the boundary description
// Reflective sides: the inflow of the directions entering through them is
// set from the mirrored directions of psi (the newest intensity), with the
// incoming moments the closures need.  Nothing when no side reflects.
static void reflect_update(smrt_ctx *x, const void *psi) {
    if (!x->refl) return;
    if (x->fp32)
        run_reflect<float>(x->stream, x->dim, x->nx, x->ny, x->G, x->nang, x->refl, x->d_mirror.p, x->d_om.p, x->d_w.p,
                           x->d_dir_quad.p, (const float *)psi, (float *)x->d_inflow.p, x->d_bmom.p);
    else
        run_reflect<double>(x->stream, x->dim, x->nx, x->ny, x->G, x->nang, x->refl, x->d_mirror.p, x->d_om.p,
                            x->d_w.p, x->d_dir_quad.p, (const double *)psi, (double *)x->d_inflow.p, x->d_bmom.p);
}

static void build_inflow(smrt_ctx *x) {
    const int nsides = 2 * x->dim;
    h2d(x->d_kind.p, x->bc_kind, sizeof(int) * 4, x->stream);
    h2d(x->d_Tb.p, x->bc_T, sizeof(double) * 4, x->stream);
    h2d(x->d_explicit.p, x->bc_explicit.data(), sizeof(double) * 4 * x->G, x->stream);
    run_side_inflow(x->stream, nsides, x->G, x->d_nu.p, x->a, x->c, x->d_kind.p, x->d_Tb.p, x->d_explicit.p, x->d_sideval.p);
    if (x->fp32) run_fill_inflow<float>(x->stream, x->dim, x->nx, x->ny, x->G, x->nang, x->d_sideval.p, (float *)x->d_inflow.p);
    else run_fill_inflow<double>(x->stream, x->dim, x->nx, x->ny, x->G, x->nang, x->d_sideval.p, (double *)x->d_inflow.p);
    if (x->have_state) reflect_update(x, x->d_psi[x->cur].p);
}

// per-side total isotropic inflow intensity sum_g I_g (Planck: a c T^4 / 4pi since sum_g b_g = 1)
static void side_totals(const smrt_ctx *x, double Itot[4]) {
    for (int s = 0; s < 4; ++s) {
        Itot[s] = 0.0;
        if (s >= 2 * x->dim) continue;
        if (x->bc_kind[s] == 1 && x->bc_T[s] > 0) Itot[s] = x->a * x->c * std::pow(x->bc_T[s], 4) / (4.0 * M_PI);
        else if (x->bc_kind[s] == 2)
            for (int g = 0; g < x->G; ++g) Itot[s] += x->bc_explicit[s * x->G + g];
    }
}

static ClosureArgs closure_args(smrt_ctx *x, int scheme, double dt, const double *mom, const double *sigP,
                                const double *sigF, const double *Estar, const double *Fstar, double *out) {
    ClosureArgs a{};
    a.dim = x->dim; a.nx = x->nx; a.ny = x->ny; a.scheme = scheme; a.c = x->c; a.dt = dt;
    a.hx = x->d_hx64.p; a.hy = x->d_hy64.p;
    a.alpha[0] = x->alpha[0]; a.alpha[1] = x->alpha[1];
    a.refl = x->refl;
    a.bmom = x->d_bmom.p;
    side_totals(x, a.Itot);
    for (int s = 0; s < 4; ++s) a.S1[s] = x->S1[s];
    for (int s = 0; s < 8; ++s) a.S2[s] = x->S2[s];
    a.mom = mom; a.sigP = sigP; a.sigF = sigF; a.Estar = Estar; a.Fstar = Fstar; a.out = out;
    return a;
}

static LoInputs lo_inputs(smrt_ctx *x, double dt, const double *clos) {
    x->lo.use_graphs = x->opt.lo_graphs != 0;
    LoInputs in{};
    in.dt = dt; in.eps_inner = x->opt.eps_inner; in.cg_rtol = x->opt.cg_rtol; in.elim_rtol = x->opt.elim_rtol;
    in.max_inner = x->opt.max_inner; in.max_cg = x->opt.max_cg; in.max_elim = x->opt.max_elim;
    in.T_floor = x->opt.T_floor;
    in.precond = x->opt.lo_precond;
    const int64_t nn = x->nn;
    in.sigE = clos; in.sigF = clos + nn; in.sigP = clos + 2 * nn; in.qE = clos + 3 * nn; in.qF = clos + 4 * nn;
    in.cvn = x->d_cvn.p;
    return in;
}

static double diff_norm(smrt_ctx *x, const double *Ta, const double *Tb, const double *Ea, const double *Eb) {
    x->lo.dot(x->stream, Ta, nullptr, Tb, 6, false);
    x->lo.dot(x->stream, Ea, nullptr, Eb, 6, true);
    return std::sqrt(x->lo.fetch(x->stream, 6));
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" void smrt_default_options(smrt_options *o) {
    if (!o) return;
    std::memset(o, 0, sizeof *o);
    o->eps_outer = 1e-3; o->eps_inner = 1e-3; o->cg_rtol = 1e-10; o->elim_rtol = 1e-10;
    o->lo_graphs = 1;
    o->max_outer = 100; o->max_inner = 30; o->max_cg = 50; o->max_elim = 40;
    o->precision = SMRT_FP64; o->scheme = SMRT_SM_CONSISTENT;
}

extern "C" const char *smrt_last_error(const smrt_ctx *ctx) { return ctx ? ctx->err.c_str() : g_last_error.c_str(); }

static void set_boundary_impl(smrt_ctx *x, const smrt_boundary_desc *bc) {
    require(bc != nullptr, "boundary descriptor is NULL");
    // validate every side before changing any
    int refl = 0;
    for (int s = 0; s < 2 * x->dim; ++s) {
        require(bc->kind[s] >= 0 && bc->kind[s] <= 3, "boundary kind must be 0, 1, 2 or 3");
        require(bc->kind[s] != 3 || x->have_mirror[s / 2],
                "a reflective side needs the mirror image of every direction in the quadrature");
        require(bc->kind[s] != 1 || bc->T_bdr[s] >= 0.0, "boundary temperature must be >= 0");
        require(bc->kind[s] != 2 || bc->inflow_g[s] != nullptr, "explicit inflow needs inflow_g");
        for (int g = 0; g < x->G && bc->kind[s] == 2; ++g)
            require(bc->inflow_g[s][g] >= 0.0, "explicit inflow must be >= 0");
        if (bc->kind[s] == 3) refl |= 1 << s;
    }
    for (int s = 0; s < 2 * x->dim; ++s) {
        x->bc_kind[s] = bc->kind[s];
        x->bc_T[s] = bc->T_bdr[s];
        for (int g = 0; g < x->G; ++g) x->bc_explicit[s * x->G + g] = bc->kind[s] == 2 ? bc->inflow_g[s][g] : 0.0;
    }
    x->refl = refl;
    build_inflow(x);
}

static void validate_options(const smrt_options *o) {
    require(o->eps_outer > 0 && o->eps_inner > 0 && o->cg_rtol > 0 && o->elim_rtol > 0, "tolerances must be > 0");
    require(o->max_outer > 0 && o->max_inner > 0 && o->max_cg > 0 && o->max_elim > 0, "iteration caps must be > 0");
    require(o->scheme >= 0 && o->scheme <= 2, "unknown scheme");
    require(o->precision == SMRT_FP64 || o->precision == SMRT_FP32, "unknown precision");
    require(o->lo_graphs == 0 || o->lo_graphs == 1, "lo_graphs must be 0 or 1");
    require(o->fixup == 0 || o->fixup == 1, "fixup must be 0 or 1");
    require(std::isfinite(o->T_floor) && o->T_floor >= 0.0, "T_floor must be finite and >= 0");
    require(o->lo_precond == 0 || o->lo_precond == 1, "lo_precond must be 0 (Jacobi) or 1 (multigrid)");
}

extern "C" smrt_status smrt_create(const smrt_mesh_desc *mesh, const smrt_quad_desc *quad, const smrt_groups_desc *groups,
                                   const smrt_material_desc *mat, const smrt_boundary_desc *bc, const smrt_options *opt,
                                   void *hip_stream, smrt_ctx **out) {
    if (!out) { g_last_error = "out is NULL"; return SMRT_E_INVALID_ARG; }
    *out = nullptr;
    std::unique_ptr<smrt_ctx> x(new (std::nothrow) smrt_ctx());
    if (!x) { g_last_error = "host allocation failed"; return SMRT_E_OUT_OF_MEMORY; }
    smrt_ctx *p = x.get();
    smrt_status st = guard(p, [&] {
        require(mesh && quad && groups && mat && bc && opt, "NULL descriptor");
        require(mesh->dim == 1 || mesh->dim == 2, "dim must be 1 or 2");
        require(mesh->nx >= 1 && (mesh->dim == 1 || mesh->ny >= 1), "mesh needs at least one cell");
        require(mesh->x_edges != nullptr && (mesh->dim == 1 || mesh->y_edges != nullptr), "mesh edges are NULL");
        p->dim = mesh->dim; p->nx = mesh->nx; p->ny = mesh->dim == 2 ? mesh->ny : 1;
        p->xe.assign(mesh->x_edges, mesh->x_edges + p->nx + 1);
        for (int i = 0; i < p->nx; ++i) require(p->xe[i + 1] > p->xe[i], "x_edges must increase strictly");
        if (p->dim == 2) {
            p->ye.assign(mesh->y_edges, mesh->y_edges + p->ny + 1);
            for (int j = 0; j < p->ny; ++j) require(p->ye[j + 1] > p->ye[j], "y_edges must increase strictly");
        }
        require(quad->n_angles >= 1 && quad->omega && quad->w, "quadrature arrays are NULL");
        p->nang = quad->n_angles;
        p->om.assign(quad->omega, quad->omega + 3 * p->nang);
        p->w.assign(quad->w, quad->w + p->nang);
        double sw = 0.0;
        for (int d = 0; d < p->nang; ++d) {
            sw += p->w[d];
            require(p->w[d] > 0.0, "quadrature weights must be > 0");
            require(p->om[3 * d] != 0.0, "a direction has mu = 0");
            if (p->dim == 2) {
                require(p->om[3 * d + 1] != 0.0, "a direction has eta = 0");
                const double nrm = std::sqrt(p->om[3 * d] * p->om[3 * d] + p->om[3 * d + 1] * p->om[3 * d + 1] +
                                             p->om[3 * d + 2] * p->om[3 * d + 2]);
                require(std::fabs(nrm - 1.0) <= 1e-12, "directions must be unit vectors");
            } else {
                require(std::fabs(p->om[3 * d]) <= 1.0, "|mu| must be <= 1");
            }
        }
        require(std::fabs(sw - 4.0 * M_PI) <= 1e-12 * 4.0 * M_PI, "quadrature weights must sum to 4 pi");
        require(groups->G >= 1 && groups->G <= MAXG && groups->nu_edges, "G must be in [1, 64]");
        p->G = groups->G;
        p->nu.assign(groups->nu_edges, groups->nu_edges + p->G + 1);
        for (int g = 0; g < p->G; ++g) require(p->nu[g + 1] > p->nu[g] && p->nu[g] >= 0.0, "nu_edges must increase strictly");
        require(groups->a > 0 && groups->c > 0, "a and c must be > 0");
        p->a = groups->a; p->c = groups->c;
        p->npc = p->dim == 2 ? 4 : 2;
        p->ncell = p->nx * p->ny;
        p->nn = p->ncell * p->npc;
        p->NB = p->dim == 1 ? 2 : 4 * (p->nx + p->ny);
        require(mat->n_regions >= 1 && mat->region_of_cell && mat->sigma0 && mat->cv, "material arrays are NULL");
        require(mat->model == 0 || mat->model == 1, "material model must be 0 or 1");
        p->nreg = mat->n_regions;
        p->region.assign(mat->region_of_cell, mat->region_of_cell + p->ncell);
        for (int r : p->region) require(r >= 0 && r < p->nreg, "region index out of range");
        p->model = mat->model;
        const int ns = p->model == 0 ? p->nreg * p->G : p->nreg;
        p->sigma0.assign(mat->sigma0, mat->sigma0 + ns);
        for (double v : p->sigma0) require(v >= 0.0 && std::isfinite(v), "sigma0 must be finite and >= 0");
        p->cv.assign(mat->cv, mat->cv + p->nreg);
        for (double v : p->cv) require(v > 0.0, "cv must be > 0");
        p->clip_lo = mat->clip_lo; p->clip_hi = mat->clip_hi;
        require(p->model == 0 || (p->clip_lo >= 0 && p->clip_hi >= p->clip_lo), "clip range must satisfy 0 <= lo <= hi");
        validate_options(opt);
        p->opt = *opt;
        p->fp32 = opt->precision == SMRT_FP32;
        p->rs = p->fp32 ? 4 : 8;
        int ndev = 0;
        SMRT_HIP(hipGetDeviceCount(&ndev));
        require(ndev > 0, "no HIP device");
        int dev = 0;
        SMRT_HIP(hipGetDevice(&dev));
        hipDeviceProp_t prop;
        SMRT_HIP(hipGetDeviceProperties(&prop, dev));
        if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
            throw smrt::Error(SMRT_E_DEVICE, std::string("this library is built for gfx950, device is ") + prop.gcnArchName);
        if (hip_stream) p->stream = static_cast<hipStream_t>(hip_stream);
        else { SMRT_HIP(hipStreamCreateWithFlags(&p->stream, hipStreamNonBlocking)); p->own_stream = true; }
        SMRT_HIP(hipEventCreate(&p->ev0));
        SMRT_HIP(hipEventCreate(&p->ev1));
        SMRT_HIP(hipHostMalloc((void **)&p->h_ctr, 4 * sizeof(int), hipHostMallocDefault));
        SMRT_HIP(hipHostMalloc((void **)&p->h_small, 32 * sizeof(double), hipHostMallocDefault));
        upload_series_coefficients();
        // quadrature sums used by the closures
        for (int ax = 0; ax < p->dim; ++ax) {
            double s = 0.0;
            for (int d = 0; d < p->nang; ++d) s += p->w[d] * std::fabs(p->om[3 * d + ax]);
            p->alpha[ax] = s / sw;
            for (int sd = 0; sd < 2; ++sd) {
                const int side = 2 * ax + sd;
                const double sgn = sd ? 1.0 : -1.0;
                double s1 = 0.0, s2[2] = {0.0, 0.0};
                for (int d = 0; d < p->nang; ++d) {
                    const double on = sgn * p->om[3 * d + ax];
                    if (on < 0) {
                        s1 += p->w[d] * on;
                        for (int a = 0; a < p->dim; ++a) s2[a] += p->w[d] * p->om[3 * d + a] * on;
                    }
                }
                p->S1[side] = s1;
                p->S2[2 * side] = s2[0];
                p->S2[2 * side + 1] = s2[1];
            }
        }
        // geometry and materials on the device
        std::vector<double> hx(p->nx), hy(p->ny, 1.0);
        for (int i = 0; i < p->nx; ++i) hx[i] = p->xe[i + 1] - p->xe[i];
        if (p->dim == 2)
            for (int j = 0; j < p->ny; ++j) hy[j] = p->ye[j + 1] - p->ye[j];
        p->d_hx64.alloc(p->nx); p->d_hy64.alloc(p->ny);
        h2d(p->d_hx64.p, hx.data(), 8 * p->nx, p->stream);
        h2d(p->d_hy64.p, hy.data(), 8 * p->ny, p->stream);
        p->d_hx.alloc(p->nx * p->rs); p->d_hy.alloc(p->ny * p->rs);
        std::vector<double> dirs((size_t)p->nang * 8), mw((size_t)p->nang * 2);
        std::vector<int> dq(p->nang);
        for (int d = 0; d < p->nang; ++d) {
            const double mu = p->om[3 * d], eta = p->dim == 2 ? p->om[3 * d + 1] : 0.0, ww = p->w[d];
            const double v[8] = {mu, eta, ww, ww * mu, ww * eta, ww * mu * mu, ww * mu * eta, ww * eta * eta};
            for (int k = 0; k < 8; ++k) dirs[8 * d + k] = v[k];
            mw[2 * d] = mu; mw[2 * d + 1] = ww;
            dq[d] = (mu > 0 && eta > 0) ? 0 : (mu < 0 && eta > 0) ? 1 : (mu < 0 && eta < 0) ? 2 : 3;
        }
        DevBuf<double> tmp;
        tmp.alloc(std::max<int64_t>((int64_t)p->nang * 8, std::max(p->nx, p->ny)));
        auto to_real = [&](const std::vector<double> &src, DevBuf<unsigned char> &dst) {
            dst.alloc(src.size() * p->rs);
            SMRT_HIP(hipMemcpy(tmp.p, src.data(), 8 * src.size(), hipMemcpyHostToDevice));
            if (p->fp32) run_copy_to<float>(p->stream, (int64_t)src.size(), tmp.p, (float *)dst.p);
            else run_copy_to<double>(p->stream, (int64_t)src.size(), tmp.p, (double *)dst.p);
            SMRT_HIP(hipStreamSynchronize(p->stream));
        };
        to_real(hx, p->d_hx);
        to_real(hy, p->d_hy);
        to_real(dirs, p->d_dirs);
        p->d_dirs64.alloc((int64_t)dirs.size());
        SMRT_HIP(hipMemcpy(p->d_dirs64.p, dirs.data(), 8 * dirs.size(), hipMemcpyHostToDevice));
        to_real(mw, p->d_mu_w);
        p->d_dir_quad.alloc(p->nang);
        SMRT_HIP(hipMemcpy(p->d_dir_quad.p, dq.data(), sizeof(int) * p->nang, hipMemcpyHostToDevice));
        // opposite directions (-mu, -eta): the adjoint sweep of d is the sweep of its opposite
        std::vector<int> opp(p->nang, -1);
        for (int d = 0; d < p->nang; ++d)
            for (int e = 0; e < p->nang; ++e) {
                const double dm = p->om[3 * e] + p->om[3 * d];
                const double de = p->dim == 2 ? p->om[3 * e + 1] + p->om[3 * d + 1] : 0.0;
                if (std::fabs(dm) < 1e-12 && std::fabs(de) < 1e-12) { opp[d] = e; break; }
            }
        p->have_opposite = std::all_of(opp.begin(), opp.end(), [](int e) { return e >= 0; });
        if (p->have_opposite) {
            p->d_opposite.alloc(p->nang);
            SMRT_HIP(hipMemcpy(p->d_opposite.p, opp.data(), sizeof(int) * p->nang, hipMemcpyHostToDevice));
        }
        // mirror images for reflective sides: (-mu, eta) for the x sides, (mu, -eta) for the y sides,
        // with the same weight
        std::vector<int> mir(2 * (size_t)p->nang, -1);
        for (int ax = 0; ax < p->dim; ++ax) {
            for (int d = 0; d < p->nang; ++d)
                for (int e = 0; e < p->nang; ++e) {
                    bool same = std::fabs(p->w[e] - p->w[d]) <= 1e-12 * p->w[d];
                    for (int k = 0; k < p->dim; ++k) {
                        const double want = k == ax ? -p->om[3 * d + k] : p->om[3 * d + k];
                        same = same && std::fabs(p->om[3 * e + k] - want) <= 1e-12;
                    }
                    if (same) { mir[(size_t)ax * p->nang + d] = e; break; }
                }
            p->have_mirror[ax] = std::all_of(mir.begin() + (size_t)ax * p->nang, mir.begin() + (size_t)(ax + 1) * p->nang,
                                             [](int e) { return e >= 0; });
        }
        p->d_mirror.alloc(2 * (int64_t)p->nang);
        SMRT_HIP(hipMemcpy(p->d_mirror.p, mir.data(), sizeof(int) * mir.size(), hipMemcpyHostToDevice));
        p->d_bmom.alloc(3 * (int64_t)(p->dim == 1 ? 2 : 4 * (p->nx + p->ny)));
        p->d_nu.alloc(p->G + 1);
        SMRT_HIP(hipMemcpy(p->d_nu.p, p->nu.data(), 8 * (p->G + 1), hipMemcpyHostToDevice));
        p->d_region.alloc(p->ncell);
        SMRT_HIP(hipMemcpy(p->d_region.p, p->region.data(), sizeof(int) * p->ncell, hipMemcpyHostToDevice));
        p->d_sigma0.alloc(ns);
        SMRT_HIP(hipMemcpy(p->d_sigma0.p, p->sigma0.data(), 8 * ns, hipMemcpyHostToDevice));
        std::vector<double> cvn(p->nn);
        for (int n = 0; n < p->nn; ++n) cvn[n] = p->cv[p->region[n / p->npc]];
        p->d_cvn.alloc(p->nn);
        SMRT_HIP(hipMemcpy(p->d_cvn.p, cvn.data(), 8 * p->nn, hipMemcpyHostToDevice));
        p->d_om.alloc(3 * p->nang); p->d_w.alloc(p->nang);
        SMRT_HIP(hipMemcpy(p->d_om.p, p->om.data(), 8 * 3 * p->nang, hipMemcpyHostToDevice));
        SMRT_HIP(hipMemcpy(p->d_w.p, p->w.data(), 8 * p->nang, hipMemcpyHostToDevice));
        p->d_sideval.alloc(4 * p->G); p->d_Tb.alloc(4); p->d_explicit.alloc(4 * p->G); p->d_kind.alloc(4);
        p->bc_explicit.assign(4 * p->G, 0.0);
        // state and work arrays
        const int NM = p->dim == 2 ? 27 : 8;
        p->d_psi[0].alloc(psi_count(p) * p->rs);
        p->d_psi[1].alloc(psi_count(p) * p->rs);
        p->d_psi[0].zero(p->stream);
        p->d_psi[1].zero(p->stream);
        // sweep tables: 2D per-quadrant skewed layout, 1D natural layout
        const int64_t tab_cells = p->dim == 2 ? 4 * cell_slab(p->nx, p->ny) : p->ncell;
        p->d_qiso.alloc(tab_cells * p->G * p->npc * p->rs);
        p->d_sig2.alloc(tab_cells * p->G * 2 * p->rs);
        if (p->dim == 2) p->d_qnat.alloc((int64_t)p->nn * p->G);
        if (p->dim == 2) p->d_sigq.alloc((int64_t)12 * p->nn);
        p->d_inflow.alloc((int64_t)p->nang * p->G * p->NB * p->rs);
        for (auto *b : {&p->d_T, &p->d_E, &p->d_Eho, &p->d_sigP, &p->d_sigF, &p->d_Tl, &p->d_El, &p->d_Tn, &p->d_En,
                        &p->d_Tstar, &p->d_Estar, &p->d_sigEho})
            b->alloc(p->nn);
        for (auto *b : {&p->d_F, &p->d_Fho, &p->d_Fstar}) b->alloc((int64_t)p->nn * p->dim);
        p->d_mom.alloc((int64_t)NM * p->nn);
        p->d_sig.alloc((int64_t)p->ncell * p->G);
        p->d_clos.alloc((int64_t)(4 + p->dim) * p->nn);
        p->lo.init(p->dim, p->nx, p->ny, p->xe, p->ye, p->alpha, p->c, p->a);
        plan_sweep(p);
        set_boundary_impl(p, bc);
        SMRT_HIP(hipStreamSynchronize(p->stream));
    });
    if (st != SMRT_OK) {
        g_last_error = p->err;
        return st;
    }
    *out = x.release();
    return SMRT_OK;
}

extern "C" void smrt_destroy(smrt_ctx *ctx) { delete ctx; }

extern "C" smrt_status smrt_set_options(smrt_ctx *x, const smrt_options *o) {
    if (!x) { g_last_error = "ctx is NULL"; return SMRT_E_INVALID_ARG; }
    return guard(x, [&] {
        require(o != nullptr, "options are NULL");
        validate_options(o);
        require(o->precision == x->opt.precision, "precision cannot change after create");
        x->opt = *o;
    });
}

extern "C" smrt_status smrt_set_boundary(smrt_ctx *x, const smrt_boundary_desc *bc) {
    if (!x) { g_last_error = "ctx is NULL"; return SMRT_E_INVALID_ARG; }
    return guard(x, [&] {
        set_boundary_impl(x, bc);
        SMRT_HIP(hipStreamSynchronize(x->stream));
    });
}

// a launch shape the sweep kernels are built for (0 = automatic per field)
static void check_shape(bool fp32, int nw, int nbw, int k, bool allow_auto) {
    const int lo = allow_auto ? 0 : 1;
    require((nw >= lo && nw <= 2) || nw == 4, "waves per band must be 1, 2 or 4 (0: automatic)");
    require((nbw >= lo && nbw <= 2) || nbw == 4 || nbw == 8 || nbw == 16,
            "bands per workgroup must be 1, 2, 4, 8 or 16 (0: automatic)");
    require((k >= lo && k <= 2) || (k == 4 && fp32), "pairs per lane must be 1, 2, or 4 (FP32 only) (0: automatic)");
    require(std::max(nw, 1) * std::max(nbw, 1) <= 16, "a sweep workgroup has at most 16 waves (waves per band x bands)");
    require(std::max(nw, 1) * std::max(nbw, 1) <= max_waves(fp32, std::max(k, 1)),
            "with 16 bytes per lane and node (FP32 with four pairs per lane, FP64 with two) a sweep workgroup has at most 8 waves");
}

extern "C" smrt_status smrt_set_launch(smrt_ctx *x, int waves_per_band, int bands_per_group, int pairs_per_lane) {
    if (!x) { g_last_error = "ctx is NULL"; return SMRT_E_INVALID_ARG; }
    return guard(x, [&] {
        check_shape(x->fp32, waves_per_band, bands_per_group, pairs_per_lane, true);
        SMRT_HIP(hipStreamSynchronize(x->stream));
        const int old[3] = {x->user_NW, x->user_NBW, x->user_K};
        x->user_NW = waves_per_band;
        x->user_NBW = bands_per_group;
        x->user_K = pairs_per_lane;
        try {
            plan_sweep(x);
        } catch (...) {
            // a shape this mesh cannot take: keep the previous one
            x->user_NW = old[0];
            x->user_NBW = old[1];
            x->user_K = old[2];
            plan_sweep(x);
            throw;
        }
    });
}

extern "C" smrt_status smrt_set_occupancy(smrt_ctx *x, int workgroups_per_cu) {
    if (!x) { g_last_error = "ctx is NULL"; return SMRT_E_INVALID_ARG; }
    return guard(x, [&] {
        require(workgroups_per_cu >= 0 && workgroups_per_cu <= 8, "workgroups per CU must be in [0, 8]");
        x->wg_per_cu = workgroups_per_cu;
    });
}

extern "C" smrt_status smrt_get_info(const smrt_ctx *x, smrt_info *info) {
    if (!x || !info) { g_last_error = "NULL argument"; return SMRT_E_INVALID_ARG; }
    info->dim = x->dim; info->nx = x->nx; info->ny = x->ny; info->n_angles = x->nang; info->G = x->G;
    info->n_nodes = x->nn; info->n_cells = x->ncell;
    info->units_per_sweep = (int64_t)x->ncell * x->nang * x->G;
    info->algorithmic_bytes_per_sweep = info->units_per_sweep * 2 * x->npc * (int64_t)x->rs;
    info->band_rows = BAND_ROWS; info->waves_per_band = x->NW; info->pairs_per_lane = x->K;
    info->pairs_per_chunk = x->R; info->n_chunks = x->NQC; info->n_workgroups = x->n_wg;
    info->bands_per_group = x->NBW;
    return SMRT_OK;
}

extern "C" smrt_status smrt_set_state(smrt_ctx *x, const double *T_nodes, const double *psi) {
    if (!x) { g_last_error = "ctx is NULL"; return SMRT_E_INVALID_ARG; }
    return guard(x, [&] {
        require(T_nodes != nullptr, "T is NULL");
        for (int n = 0; n < x->nn; ++n) require(T_nodes[n] > 0.0 && std::isfinite(T_nodes[n]), "T must be finite and > 0");
        h2d(x->d_T.p, T_nodes, 8 * x->nn, x->stream);
        DevBuf<double> abi;
        const int64_t na = (int64_t)x->nang * x->G * x->nn;
        abi.alloc(na);
        if (psi) h2d(abi.p, psi, 8 * na, x->stream);
        else run_equilibrium(x->stream, x->nn, x->G, x->nang, x->d_T.p, x->d_nu.p, x->a, x->c, abi.p);
        if (x->dim == 2) {
            if (x->fp32) run_psi_to_internal<float>(x->stream, x->nx, x->ny, x->G, x->nang, x->d_dir_quad.p, abi.p, (float *)x->d_psi[x->cur].p);
            else run_psi_to_internal<double>(x->stream, x->nx, x->ny, x->G, x->nang, x->d_dir_quad.p, abi.p, (double *)x->d_psi[x->cur].p);
        } else {
            if (x->fp32) run_copy_to<float>(x->stream, na, abi.p, (float *)x->d_psi[x->cur].p);
            else run_copy_to<double>(x->stream, na, abi.p, (double *)x->d_psi[x->cur].p);
        }
        run_psi_EF(x->stream, x->nn, x->dim, x->G, x->nang, x->d_om.p, x->d_w.p, x->c, abi.p, x->d_Eho.p, x->d_Fho.p);
        SMRT_HIP(hipMemcpyAsync(x->d_E.p, x->d_Eho.p, 8 * x->nn, hipMemcpyDeviceToDevice, x->stream));
        SMRT_HIP(hipMemcpyAsync(x->d_F.p, x->d_Fho.p, 8 * x->nn * x->dim, hipMemcpyDeviceToDevice, x->stream));
        reflect_update(x, x->d_psi[x->cur].p);
        SMRT_HIP(hipStreamSynchronize(x->stream));
        x->have_state = true;
    });
}

extern "C" smrt_status smrt_get_state(smrt_ctx *x, double *T, double *E, double *F, double *psi) {
    if (!x) { g_last_error = "ctx is NULL"; return SMRT_E_INVALID_ARG; }
    return guard(x, [&] {
        if (T) d2h(T, x->d_T.p, 8 * x->nn, x->stream);
        if (E) d2h(E, x->d_E.p, 8 * x->nn, x->stream);
        if (F) d2h(F, x->d_F.p, 8 * x->nn * x->dim, x->stream);
        if (psi) {
            const int64_t na = (int64_t)x->nang * x->G * x->nn;
            DevBuf<double> abi;
            abi.alloc(na);
            if (x->dim == 2) {
                if (x->fp32) run_psi_from_internal<float>(x->stream, x->nx, x->ny, x->G, x->nang, x->d_dir_quad.p, (const float *)x->d_psi[x->cur].p, abi.p);
                else run_psi_from_internal<double>(x->stream, x->nx, x->ny, x->G, x->nang, x->d_dir_quad.p, (const double *)x->d_psi[x->cur].p, abi.p);
            } else {
                // 1D internal layout equals the ABI layout
                DevBuf<double> t;
                if (x->fp32) {
                    std::vector<float> h(na);
                    d2h(h.data(), x->d_psi[x->cur].p, 4 * na, x->stream);
                    SMRT_HIP(hipStreamSynchronize(x->stream));
                    for (int64_t k = 0; k < na; ++k) psi[k] = h[k];
                    return;
                }
                SMRT_HIP(hipMemcpyAsync(abi.p, x->d_psi[x->cur].p, 8 * na, hipMemcpyDeviceToDevice, x->stream));
            }
            d2h(psi, abi.p, 8 * na, x->stream);
            SMRT_HIP(hipStreamSynchronize(x->stream));
        }
        SMRT_HIP(hipStreamSynchronize(x->stream));
    });
}

// One sweep from device-resident FP64 arrays in the ABI layouts: sig_t, sig
// [cell][G]; q [node][G]; prev (psi_prev, or nullptr) [d][g][node]; inflow
// (nullptr: the context's boundary inflow) [d][g][NB]; out [d][g][node];
// mom (or nullptr) [27|8][node].
// Device scratch of a raw sweep (tables, internal-layout intensities, inflow,
// moments); a caller that sweeps many times keeps one and passes it in.
struct RawScratch {
    DevBuf<unsigned char> sig2, qiso, in, out, inflow;
    DevBuf<double> mom;
};
template <typename T>
static void ensure(DevBuf<T> &b, int64_t n) {
    if (b.n != n) b.alloc(n);
}

// Work arrays of one raw sweep: the inputs in the sweep's internal layouts
// and precision, the internal output, and moments when the caller wants none.
struct RawBufs {
    void *sig2, *qiso, *in, *out, *inflow;
    double *mom;
};
static int64_t raw_tab_cells(const smrt_ctx *x) { return x->dim == 2 ? 4 * cell_slab(x->nx, x->ny) : x->ncell; }

// The sweep of explicit inputs (FP64, caller layouts) into out/mom through
// the work arrays B; ws: kernel work memory (nullptr: the context's).
static void raw_sweep_with(smrt_ctx *x, const double *sig_t, const double *sig, const double *q, const double *prev,
                           double inv_c_dt, const double *inflow64, double *out, double *mom, const RawBufs &B,
                           const SweepScratch *ws) {
    const int64_t na = (int64_t)x->nang * x->G * x->nn;
    auto tables = [&](auto zero) {
        using real = decltype(zero);
        if (x->dim == 2) {
            run_stab2d<real>(x->stream, x->nx, x->ny, x->G, sig, sig_t, 0.0, (real *)B.sig2);
            run_qtab2d<real, double>(x->stream, x->nx, x->ny, x->G, q, x->G, 1, (real *)B.qiso);
        } else {
            run_sig_to_internal<real>(x->stream, x->ncell, x->G, sig_t, sig, (real *)B.sig2);
            run_qiso_to_internal<real>(x->stream, x->nn, x->G, x->npc, q, (real *)B.qiso);
        }
        if (prev) {
            if (x->dim == 2) run_psi_to_internal<real>(x->stream, x->nx, x->ny, x->G, x->nang, x->d_dir_quad.p, prev, (real *)B.in);
            else run_copy_to<real>(x->stream, na, prev, (real *)B.in);
        }
        if (inflow64) run_copy_to<real>(x->stream, (int64_t)x->nang * x->G * x->NB, inflow64, (real *)B.inflow);
    };
    if (x->fp32) tables(0.0f);
    else tables(0.0);
    if (!mom) mom = B.mom;
    run_sweep(x, prev ? B.in : nullptr, B.out, B.sig2, B.qiso, inflow64 ? B.inflow : x->d_inflow.p, inv_c_dt, sig, mom,
              true, ws);
    if (!ws) check_sweep_flag(x);
    auto back = [&](auto zero) {
        using real = decltype(zero);
        if (x->dim == 2) run_psi_from_internal<real>(x->stream, x->nx, x->ny, x->G, x->nang, x->d_dir_quad.p, (const real *)B.out, out);
        else run_copy_from<real>(x->stream, na, (const real *)B.out, out);
    };
    if (x->fp32) back(0.0f);
    else back(0.0);
}

static void raw_sweep(smrt_ctx *x, const double *sig_t, const double *sig, const double *q, const double *prev,
                      double inv_c_dt, const double *inflow64, double *out, double *mom, RawScratch *scratch = nullptr) {
    const int64_t tab_cells = raw_tab_cells(x);
    RawScratch local;
    RawScratch &R = scratch ? *scratch : local;
    ensure(R.sig2, tab_cells * x->G * 2 * x->rs);
    ensure(R.qiso, tab_cells * x->G * x->npc * x->rs);
    ensure(R.in, psi_count(x) * x->rs);
    ensure(R.out, psi_count(x) * x->rs);
    ensure(R.inflow, (int64_t)x->nang * x->G * x->NB * x->rs);
    if (!mom) ensure(R.mom, (int64_t)(x->dim == 2 ? 27 : 8) * x->nn);
    const RawBufs B{R.sig2.p, R.qiso.p, R.in.p, R.out.p, R.inflow.p, R.mom.p};
    raw_sweep_with(x, sig_t, sig, q, prev, inv_c_dt, inflow64, out, mom, B, nullptr);
    SMRT_HIP(hipStreamSynchronize(x->stream));
}

extern "C" smrt_status smrt_sweep(smrt_ctx *x, const double *sig_t, const double *sig, const double *q_iso,
                                  const double *psi_prev, double inv_c_dt, const double *psi_inflow, double *psi_out,
                                  double *moments_out) {
    if (!x) { g_last_error = "ctx is NULL"; return SMRT_E_INVALID_ARG; }
    return guard(x, [&] {
        require(sig_t && sig && q_iso, "sig_t, sig and q_iso are required");
        require(std::isfinite(inv_c_dt) && inv_c_dt >= 0.0, "inv_c_dt must be finite and >= 0");
        const int64_t na = (int64_t)x->nang * x->G * x->nn;
        const int64_t ng = (int64_t)x->ncell * x->G;
        for (int64_t k = 0; k < ng; ++k) require(sig_t[k] > 0.0 && sig[k] >= 0.0, "sig_t must be > 0 and sig >= 0");
        DevBuf<double> t_st, t_s, t_q, t_prev, t_inf, t_out, mom;
        t_st.alloc(ng); t_s.alloc(ng); t_q.alloc((int64_t)x->nn * x->G); t_out.alloc(na);
        h2d(t_st.p, sig_t, 8 * ng, x->stream);
        h2d(t_s.p, sig, 8 * ng, x->stream);
        h2d(t_q.p, q_iso, 8 * x->nn * x->G, x->stream);
        if (psi_prev) {
            t_prev.alloc(na);
            h2d(t_prev.p, psi_prev, 8 * na, x->stream);
        }
        if (psi_inflow) {
            t_inf.alloc((int64_t)x->nang * x->G * x->NB);
            h2d(t_inf.p, psi_inflow, 8 * t_inf.n, x->stream);
        }
        mom.alloc((int64_t)(x->dim == 2 ? 27 : 8) * x->nn);
        raw_sweep(x, t_st.p, t_s.p, t_q.p, t_prev.p, inv_c_dt, t_inf.p, t_out.p, mom.p);
        if (moments_out) d2h(moments_out, mom.p, 8 * mom.n, x->stream);
        if (psi_out) d2h(psi_out, t_out.p, 8 * na, x->stream);
        SMRT_HIP(hipStreamSynchronize(x->stream));
    });
}

// 1 in *bad if some sig_t <= 0 or sig < 0 (device-side input check)
__global__ void k_check_opacities(int64_t n, const double *sig_t, const double *sig, int *bad) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const bool b = i < n && !(sig_t[i] > 0.0 && sig[i] >= 0.0);
    if (__builtin_amdgcn_ballot_w64(b) != 0 && (threadIdx.x & 63) == 0) atomicOr(bad, 1);
}

extern "C" smrt_status smrt_sweep_dev(smrt_ctx *x, const double *sig_t, const double *sig, const double *q_iso,
                                      const double *psi_prev, double inv_c_dt, const double *psi_inflow,
                                      double *psi_out, double *moments_out) {
    if (!x) { g_last_error = "ctx is NULL"; return SMRT_E_INVALID_ARG; }
    return guard(x, [&] {
        require(sig_t && sig && q_iso && psi_out, "sig_t, sig, q_iso and psi_out are required");
        require(std::isfinite(inv_c_dt) && inv_c_dt >= 0.0, "inv_c_dt must be finite and >= 0");
        const int64_t ng = (int64_t)x->ncell * x->G;
        DevBuf<int> bad;
        bad.alloc(1);
        bad.zero(x->stream);
        hipLaunchKernelGGL(k_check_opacities, dim3((unsigned)((ng + 255) / 256)), dim3(256), 0, x->stream, ng, sig_t,
                           sig, bad.p);
        int hb = 0;
        read_small(x, &hb, bad.p, sizeof(int));
        require(hb == 0, "sig_t must be > 0 and sig >= 0");
        raw_sweep(x, sig_t, sig, q_iso, psi_prev, inv_c_dt, psi_inflow, psi_out, moments_out);
    });
}

// ---------------------------------------------------------------------------
// Allocation-free sweep (smrt_sweep_dev_static): every per-call work array of
// smrt_sweep_dev (input tables, internal intensities, moment partials, trace
// words, counters, the opacity check flag) lives in one static device array,
// so the call allocates nothing.  The array's device address is looked up
// once per device; host code uses that address, never the array's name.
// ---------------------------------------------------------------------------
constexpr size_t SWEEP_SCRATCH_BYTES = (size_t)64 << 20;   // per GPU, held until the process ends
static __device__ __align__(256) unsigned char scratch[SWEEP_SCRATCH_BYTES];
constexpr int SCRATCH_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static unsigned char *g_scratch_ptr[SCRATCH_MAX_DEVICES] = {};

// the static array's address on the current device (looked up on first use)
static unsigned char *static_scratch() {
    int dev = 0;
    SMRT_HIP(hipGetDevice(&dev));
    require(dev >= 0 && dev < SCRATCH_MAX_DEVICES, "device index beyond the static scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        SMRT_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        require(p != nullptr, "hipGetSymbolAddress returned no address for the static scratch");
        g_scratch_ptr[dev] = static_cast<unsigned char *>(p);
    }
    return g_scratch_ptr[dev];
}

__global__ void k_fill_u64(int64_t n, uint64_t *p, uint64_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void k_fill_i32(int n, int *p, int v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Regions of the static array, 256-byte aligned, in a fixed order.
struct ScratchPlan {
    size_t off = 0;
    size_t take(size_t bytes) {
        const size_t at = off;
        off += (bytes + 255) / 256 * 256;
        return at;
    }
};

extern "C" smrt_status smrt_sweep_dev_static(smrt_ctx *x, const double *sig_t, const double *sig, const double *q_iso,
                                             const double *psi_prev, double inv_c_dt, const double *psi_inflow,
                                             double *psi_out, double *moments_out) {
    if (!x) { g_last_error = "ctx is NULL"; return SMRT_E_INVALID_ARG; }
    return guard(x, [&] {
        require(sig_t && sig && q_iso && psi_out, "sig_t, sig, q_iso and psi_out are required");
        require(std::isfinite(inv_c_dt) && inv_c_dt >= 0.0, "inv_c_dt must be finite and >= 0");
        const int64_t tab_cells = raw_tab_cells(x);
        const bool two_d = x->dim == 2;
        ScratchPlan plan;
        const size_t o_sig2 = plan.take((size_t)(tab_cells * x->G * 2 * x->rs));
        const size_t o_qiso = plan.take((size_t)(tab_cells * x->G * x->npc * x->rs));
        const size_t o_in = plan.take(psi_prev ? (size_t)(psi_count(x) * x->rs) : 0);
        const size_t o_out = plan.take((size_t)(psi_count(x) * x->rs));
        const size_t o_inflow = plan.take(psi_inflow ? (size_t)((int64_t)x->nang * x->G * x->NB * x->rs) : 0);
        const size_t o_mom = plan.take(moments_out ? 0 : (size_t)((two_d ? 27 : 8) * x->nn) * sizeof(double));
        const size_t o_part = plan.take(two_d ? (size_t)x->d_part.n : 0);
        const size_t o_trace = plan.take(two_d ? (size_t)x->d_trace.n * sizeof(uint64_t) : 0);
        const size_t o_flags = plan.take(8 * sizeof(int));   // ctr[4], lctr[2], opacity flag
        if (plan.off > SWEEP_SCRATCH_BYTES)
            throw smrt::Error(SMRT_E_INVALID_ARG, "the problem needs " + std::to_string(plan.off) +
                                                      " bytes of sweep work memory; the static scratch holds " +
                                                      std::to_string(SWEEP_SCRATCH_BYTES) + " (use smrt_sweep_dev)");
        unsigned char *base = static_scratch();
        int *flags = reinterpret_cast<int *>(base + o_flags);
        // clear what must start at zero, with fill kernels (no memset)
        hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, x->stream, 8, flags, 0);
        SweepScratch ws;
        if (two_d) {
            ws.part = base + o_part;
            ws.trace = reinterpret_cast<uint64_t *>(base + o_trace);
            ws.ctr = flags;
            ws.lctr = flags + 4;
            hipLaunchKernelGGL(k_init_ctr, dim3(1), dim3(1), 0, x->stream, ws.ctr);
            const int64_t nt = x->d_trace.n;
            if (nt > 0)
                hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)std::min<int64_t>((nt + 255) / 256, 1024)), dim3(256), 0,
                                   x->stream, nt, ws.trace, (uint64_t)0);
        }
        const int64_t ng = (int64_t)x->ncell * x->G;
        hipLaunchKernelGGL(k_check_opacities, dim3((unsigned)((ng + 255) / 256)), dim3(256), 0, x->stream, ng, sig_t, sig,
                           flags + 6);
        int hb = 0;
        read_small(x, &hb, flags + 6, sizeof(int));
        require(hb == 0, "sig_t must be > 0 and sig >= 0");
        const RawBufs B{base + o_sig2, base + o_qiso, psi_prev ? base + o_in : nullptr, base + o_out,
                        psi_inflow ? base + o_inflow : nullptr, reinterpret_cast<double *>(base + o_mom)};
        raw_sweep_with(x, sig_t, sig, q_iso, psi_prev, inv_c_dt, psi_inflow, psi_out, moments_out, B,
                       two_d ? &ws : nullptr);
        if (two_d) {
            int fl = 0;
            read_small(x, &fl, ws.ctr + 3, sizeof(int));
            if (fl) throw smrt::Error(SMRT_E_DEVICE, "sweep band-trace wait exceeded its bound");
        }
        SMRT_HIP(hipStreamSynchronize(x->stream));
    });
}

// Adjoint sweep (transpose of the lumped upwind DG operator).  With every
// form lumped on a rectilinear mesh the transpose of the operator of
// direction Omega is the operator of -Omega (the local matrices are
// dI + (a/2)Kx + (b/2)Ky with antisymmetric Kx, Ky, and the upwind
// couplings swap sides), so lambda_d = L_{-Omega_d}^{-1} (w . src_d) is one
// forward sweep of the opposite direction with zero inflow, its source
// carried in the time-edge slot (inv_c_dt = 1, q = 0).
extern "C" smrt_status smrt_adjoint_sweep(smrt_ctx *x, const double *sig_t, const double *src, const double *emis,
                                          const double *psi_fwd, double *lambda_out, double *dsig_out) {
    if (!x) { g_last_error = "ctx is NULL"; return SMRT_E_INVALID_ARG; }
    return guard(x, [&] {
        require(sig_t && src && lambda_out, "sig_t, src and lambda_out are required");
        require(!dsig_out || (emis && psi_fwd), "dsig_out needs emis and psi_fwd");
        require(x->have_opposite, "the quadrature has a direction without its opposite: no adjoint sweep");
        const int64_t na = (int64_t)x->nang * x->G * x->nn;
        const int64_t ng = (int64_t)x->ncell * x->G;
        for (int64_t k = 0; k < ng; ++k) require(sig_t[k] > 0.0, "sig_t must be > 0");
        DevBuf<double> t_st, t_q, t_src, t_prev, t_inf, t_out, t_lam;
        t_st.alloc(ng); t_q.alloc((int64_t)x->nn * x->G); t_src.alloc(na); t_prev.alloc(na);
        t_inf.alloc((int64_t)x->nang * x->G * x->NB); t_out.alloc(na); t_lam.alloc(na);
        h2d(t_st.p, sig_t, 8 * ng, x->stream);
        h2d(t_src.p, src, 8 * na, x->stream);
        t_q.zero(x->stream);
        t_inf.zero(x->stream);
        const int64_t per = (int64_t)x->G * x->nn;
        run_permute_dirs(x->stream, x->nang, per, x->d_opposite.p, t_src.p, t_prev.p);
        raw_sweep(x, t_st.p, t_st.p, t_q.p, t_prev.p, 1.0, t_inf.p, t_out.p, nullptr);
        run_permute_dirs(x->stream, x->nang, per, x->d_opposite.p, t_out.p, t_lam.p);
        d2h(lambda_out, t_lam.p, 8 * na, x->stream);
        if (dsig_out) {
            DevBuf<double> t_e, t_f, t_d;
            t_e.alloc((int64_t)x->nn * x->G); t_f.alloc(na); t_d.alloc(ng);
            h2d(t_e.p, emis, 8 * t_e.n, x->stream);
            h2d(t_f.p, psi_fwd, 8 * na, x->stream);
            run_adjoint_dsig(x->stream, x->dim, x->nx, x->dim == 2 ? x->ny : 1, x->G, x->nang, x->d_hx64.p,
                             x->dim == 2 ? x->d_hy64.p : nullptr, t_lam.p, t_e.p, t_f.p, t_d.p);
            d2h(dsig_out, t_d.p, 8 * ng, x->stream);
        }
        SMRT_HIP(hipStreamSynchronize(x->stream));
    });
}

extern "C" smrt_status smrt_compute_closures(smrt_ctx *x, const double *moments, const double *T_l, const double *Estar,
                                             const double *Fstar, const double *sig, double dt, double *closures_out) {
    if (!x) { g_last_error = "ctx is NULL"; return SMRT_E_INVALID_ARG; }
    return guard(x, [&] {
        require(moments && T_l && Estar && Fstar && sig && closures_out, "NULL argument");
        require(dt > 0.0, "dt must be > 0");
        const int NM = x->dim == 2 ? 27 : 8;
        DevBuf<double> m, Tl, Es, Fs, sg, sP, sF, out;
        DevBuf<unsigned char> q;
        m.alloc((int64_t)NM * x->nn); Tl.alloc(x->nn); Es.alloc(x->nn); Fs.alloc((int64_t)x->nn * x->dim);
        sg.alloc((int64_t)x->ncell * x->G); sP.alloc(x->nn); sF.alloc(x->nn); out.alloc((int64_t)(4 + x->dim) * x->nn);
        q.alloc((int64_t)x->nn * x->G * x->rs);
        h2d(m.p, moments, 8 * m.n, x->stream); h2d(Tl.p, T_l, 8 * x->nn, x->stream); h2d(Es.p, Estar, 8 * x->nn, x->stream);
        h2d(Fs.p, Fstar, 8 * Fs.n, x->stream); h2d(sg.p, sig, 8 * sg.n, x->stream);
        if (x->fp32) run_source<float>(x->stream, x->nn, x->npc, x->G, Tl.p, x->d_nu.p, x->a, x->c, sg.p, (float *)q.p, nullptr, sP.p, sF.p);
        else run_source<double>(x->stream, x->nn, x->npc, x->G, Tl.p, x->d_nu.p, x->a, x->c, sg.p, (double *)q.p, nullptr, sP.p, sF.p);
        run_closures(x->stream, closure_args(x, x->opt.scheme == SMRT_SM_INDEPENDENT ? 1 : 0, dt, m.p, sP.p, sF.p, Es.p, Fs.p, out.p));
        d2h(closures_out, out.p, 8 * out.n, x->stream);
        SMRT_HIP(hipStreamSynchronize(x->stream));
    });
}

extern "C" smrt_status smrt_lo_solve(smrt_ctx *x, const double *closures, const double *Tstar, double dt, double *E,
                                     double *F, double *T, smrt_step_stats *stats) {
    if (!x) { g_last_error = "ctx is NULL"; return SMRT_E_INVALID_ARG; }
    smrt_status inner = SMRT_OK;
    smrt_status st = guard(x, [&] {
        require(closures && Tstar && E && F && T, "NULL argument");
        require(dt > 0.0, "dt must be > 0");
        DevBuf<double> cl, Ts, dE, dF, dT;
        cl.alloc((int64_t)(4 + x->dim) * x->nn); Ts.alloc(x->nn); dE.alloc(x->nn); dF.alloc((int64_t)x->nn * x->dim); dT.alloc(x->nn);
        h2d(cl.p, closures, 8 * cl.n, x->stream); h2d(Ts.p, Tstar, 8 * x->nn, x->stream);
        h2d(dE.p, E, 8 * x->nn, x->stream); h2d(dT.p, T, 8 * x->nn, x->stream);
        smrt_step_stats s{};
        LoInputs in = lo_inputs(x, dt, cl.p);
        in.Tstar = Ts.p;
        inner = x->lo.solve(x->stream, in, dE.p, dF.p, dT.p, &s, x->err);
        d2h(E, dE.p, 8 * x->nn, x->stream); d2h(F, dF.p, 8 * dF.n, x->stream); d2h(T, dT.p, 8 * x->nn, x->stream);
        SMRT_HIP(hipStreamSynchronize(x->stream));
        if (stats) *stats = s;
        if (inner == SMRT_OK && x->opt.strict && s.hit_max) {
            inner = SMRT_E_NOT_CONVERGED;
            x->err = "low-order iteration cap reached";
        }
    });
    return st != SMRT_OK ? st : inner;
}

// prepare the per-step opacity table and return 1/(c dt)
static double prepare_step_tables(smrt_ctx *x, double dt) {
    const double icdt = 1.0 / (x->c * dt);
    const bool d2 = x->dim == 2;
    if (x->fp32) {
        if (d2) run_opacity_tab2d<float>(x->stream, x->nx, x->ny, x->G, x->d_T.p, x->d_region.p, x->model, x->d_sigma0.p, x->clip_lo, x->clip_hi, x->d_nu.p, icdt, x->d_sig.p, (float *)x->d_sig2.p);
        else run_opacity<float>(x->stream, x->ncell, x->npc, x->G, x->d_T.p, x->d_region.p, x->model, x->d_sigma0.p, x->clip_lo, x->clip_hi, x->d_nu.p, icdt, x->d_sig.p, (float *)x->d_sig2.p);
    } else {
        if (d2) run_opacity_tab2d<double>(x->stream, x->nx, x->ny, x->G, x->d_T.p, x->d_region.p, x->model, x->d_sigma0.p, x->clip_lo, x->clip_hi, x->d_nu.p, icdt, x->d_sig.p, (double *)x->d_sig2.p);
        else run_opacity<double>(x->stream, x->ncell, x->npc, x->G, x->d_T.p, x->d_region.p, x->model, x->d_sigma0.p, x->clip_lo, x->clip_hi, x->d_nu.p, icdt, x->d_sig.p, (double *)x->d_sig2.p);
    }
    return icdt;
}

static void run_source_at(smrt_ctx *x, const double *T, const int *gate = nullptr) {
    const bool d2 = x->dim == 2;
    if (x->fp32) {
        run_source<float>(x->stream, x->nn, x->npc, x->G, T, x->d_nu.p, x->a, x->c, x->d_sig.p, d2 ? nullptr : (float *)x->d_qiso.p, d2 ? (float *)x->d_qnat.p : nullptr, x->d_sigP.p, x->d_sigF.p, gate);
        if (d2) run_qtab2d<float, float>(x->stream, x->nx, x->ny, x->G, (const float *)x->d_qnat.p, 1, x->nn, (float *)x->d_qiso.p, gate);
    } else {
        run_source<double>(x->stream, x->nn, x->npc, x->G, T, x->d_nu.p, x->a, x->c, x->d_sig.p, d2 ? nullptr : (double *)x->d_qiso.p, d2 ? x->d_qnat.p : nullptr, x->d_sigP.p, x->d_sigF.p, gate);
        if (d2) run_qtab2d<double, double>(x->stream, x->nx, x->ny, x->G, x->d_qnat.p, 1, x->nn, (double *)x->d_qiso.p, gate);
    }
}

// One backward-Euler step (Algorithm 1) split into phases, so that a batch
// can run the outer iterations of many problems in lock-step with one
// batched sweep per outer iteration.
struct StepRun {
    smrt_ctx *x = nullptr;
    double dt = 0, icdt = 0, first = -1.0;
    int l = 0, maxo = 0;
    bool unacc = false, done = false;
    smrt_status result = SMRT_OK;
    smrt_step_stats s{};
    void *pin = nullptr, *pout = nullptr;
    float t_sweep = 0.f;

    void begin(smrt_ctx *ctx, double step_dt) {
        x = ctx;
        dt = step_dt;
        require(dt > 0.0 && std::isfinite(dt), "dt must be finite and > 0");
        require(x->have_state, "smrt_set_state must be called before smrt_step");
        hipStream_t S = x->stream;
        const int64_t nn = x->nn;
        SMRT_HIP(hipEventRecord(x->ev0, S));
        icdt = prepare_step_tables(x, dt);
        SMRT_HIP(hipMemcpyAsync(x->d_Tstar.p, x->d_T.p, 8 * nn, hipMemcpyDeviceToDevice, S));
        if (x->opt.lo_time_edge) {
            SMRT_HIP(hipMemcpyAsync(x->d_Estar.p, x->d_E.p, 8 * nn, hipMemcpyDeviceToDevice, S));
            SMRT_HIP(hipMemcpyAsync(x->d_Fstar.p, x->d_F.p, 8 * nn * x->dim, hipMemcpyDeviceToDevice, S));
        } else {
            SMRT_HIP(hipMemcpyAsync(x->d_Estar.p, x->d_Eho.p, 8 * nn, hipMemcpyDeviceToDevice, S));
            SMRT_HIP(hipMemcpyAsync(x->d_Fstar.p, x->d_Fho.p, 8 * nn * x->dim, hipMemcpyDeviceToDevice, S));
        }
        SMRT_HIP(hipMemcpyAsync(x->d_Tl.p, x->d_T.p, 8 * nn, hipMemcpyDeviceToDevice, S));
        unacc = x->opt.scheme == SMRT_UNACCELERATED;
        SMRT_HIP(hipMemcpyAsync(x->d_El.p, unacc ? x->d_Estar.p : x->d_E.p, 8 * nn, hipMemcpyDeviceToDevice, S));
        maxo = x->opt.fixed_outer > 0 ? x->opt.fixed_outer : x->opt.max_outer;
        pin = x->d_psi[x->cur].p;
        pout = x->d_psi[1 - x->cur].p;
    }
    // emission tables at the current outer temperature
    void pre_sweep() {
        ++l;
        run_source_at(x, x->d_Tl.p);
    }
    // LO (or pointwise elimination) after the sweep; returns true once the
    // outer iteration of this step is finished
    bool post_sweep() {
        hipStream_t S = x->stream;
        const int64_t nn = x->nn;
        s.outer++;
        reflect_update(x, pout);   // reflective sides mirror this sweep's intensity from here on
        SMRT_HIP(hipMemcpyAsync(x->d_Tn.p, x->d_Tl.p, 8 * nn, hipMemcpyDeviceToDevice, S));
        if (unacc) {
            // pointwise elimination against sum_g sigma_g phi_g of the sweep
            hipLaunchKernelGGL(k_ho_from_mom, dim3(nblk(nn)), dim3(256), 0, S, (int)nn, x->dim, x->c, x->d_mom.p,
                               x->d_sigP.p, x->d_En.p, (double *)nullptr, x->d_sigEho.p);
            LoSolver &L = x->lo;
            hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, S, L.flags.p, 4);
            run_eliminate(S, (int)nn, x->a, x->c, dt, x->opt.elim_rtol, x->opt.max_elim, x->opt.T_floor, x->d_cvn.p,
                          x->d_sigEho.p,
                          x->d_sigP.p, x->d_En.p, x->d_Tstar.p, x->d_Tn.p, L.flags.p);
            int fl[4];
            L.fetch_flags(S, fl);
            if (fl[1] > s.elim_max) s.elim_max = fl[1];
            if (fl[2]) s.hit_max = 1;             // a node's pointwise Newton ran to its cap
            if (fl[0]) { x->err = "no positive temperature root in the energy balance"; result = SMRT_E_NONPHYSICAL; }
        } else {
            SMRT_HIP(hipMemcpyAsync(x->d_En.p, x->d_El.p, 8 * nn, hipMemcpyDeviceToDevice, S));
            run_closures(S, closure_args(x, x->opt.scheme == SMRT_SM_INDEPENDENT ? 1 : 0, dt, x->d_mom.p, x->d_sigP.p,
                                         x->d_sigF.p, x->d_Estar.p, x->d_Fstar.p, x->d_clos.p));
            LoInputs in = lo_inputs(x, dt, x->d_clos.p);
            in.Tstar = x->d_Tstar.p;
            smrt_step_stats ls{};
            const smrt_status r = x->lo.solve(S, in, x->d_En.p, x->d_F.p, x->d_Tn.p, &ls, x->err);
            s.inner_total += ls.inner_total;
            s.cg_total += ls.cg_total;
            s.elim_max = std::max(s.elim_max, ls.elim_max);
            s.hit_max |= ls.hit_max;
            if (r != SMRT_OK) result = r;
        }
        fetch_sweep_flag(x);                       // read after the change norm's own wait
        const double diff = diff_norm(x, x->d_Tn.p, x->d_Tl.p, x->d_En.p, x->d_El.p);
        raise_sweep_flag(x);
        SMRT_HIP(hipMemcpyAsync(x->d_Tl.p, x->d_Tn.p, 8 * nn, hipMemcpyDeviceToDevice, S));
        SMRT_HIP(hipMemcpyAsync(x->d_El.p, x->d_En.p, 8 * nn, hipMemcpyDeviceToDevice, S));
        if (result != SMRT_OK) return done = true;
        if (!std::isfinite(diff)) { x->err = "non-finite outer iterate"; result = SMRT_E_NONPHYSICAL; return done = true; }
        if (x->opt.fixed_outer > 0) return done = (l >= maxo);
        if (l == 1) first = diff;
        if (diff == 0.0 || (l > 1 && diff < x->opt.eps_outer * first)) return done = true;
        if (l == maxo) { s.hit_max = 1; return done = true; }
        return false;
    }
    smrt_status end(smrt_step_stats *stats) {
        hipStream_t S = x->stream;
        const int64_t nn = x->nn;
        // new state: T, E from the last outer iterate; psi and HO moments from the last sweep
        SMRT_HIP(hipMemcpyAsync(x->d_T.p, x->d_Tl.p, 8 * nn, hipMemcpyDeviceToDevice, S));
        SMRT_HIP(hipMemcpyAsync(x->d_E.p, x->d_El.p, 8 * nn, hipMemcpyDeviceToDevice, S));
        hipLaunchKernelGGL(k_ho_from_mom, dim3(nblk(nn)), dim3(256), 0, S, (int)nn, x->dim, x->c, x->d_mom.p, x->d_sigP.p,
                           x->d_Eho.p, x->d_Fho.p, (double *)nullptr);
        x->cur = 1 - x->cur;
        SMRT_HIP(hipEventRecord(x->ev1, S));
        SMRT_HIP(hipEventSynchronize(x->ev1));
        float tot = 0.f;
        SMRT_HIP(hipEventElapsedTime(&tot, x->ev0, x->ev1));
        s.t_total_ms = tot;
        s.t_sweep_ms = t_sweep;
        s.t_lo_ms = tot - t_sweep;
        if (stats) *stats = s;
        if (result == SMRT_OK && x->opt.strict && s.hit_max) {
            result = SMRT_E_NOT_CONVERGED;
            x->err = "iteration cap reached";
        }
        return result;
    }
};

// time one stream-ordered section (ms)
// a pair of events released on every exit path
struct EventPair {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    EventPair() {
        SMRT_HIP(hipEventCreate(&e0));
        if (hipEventCreate(&e1) != hipSuccess) {
            (void)hipEventDestroy(e0);
            throw Error(SMRT_E_DEVICE, "hipEventCreate failed");
        }
    }
    ~EventPair() {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    }
    EventPair(const EventPair &) = delete;
    EventPair &operator=(const EventPair &) = delete;
};

template <typename F>
static float timed(hipStream_t S, F &&f) {
    EventPair ev;
    SMRT_HIP(hipEventRecord(ev.e0, S));
    f();
    SMRT_HIP(hipEventRecord(ev.e1, S));
    SMRT_HIP(hipEventSynchronize(ev.e1));
    float ms = 0.f;
    SMRT_HIP(hipEventElapsedTime(&ms, ev.e0, ev.e1));
    return ms;
}

extern "C" smrt_status smrt_step(smrt_ctx *x, double dt, smrt_step_stats *stats) {
    if (!x) { g_last_error = "ctx is NULL"; return SMRT_E_INVALID_ARG; }
    StepRun run;
    smrt_status st = guard(x, [&] {
        run.begin(x, dt);
        for (;;) {
            run.pre_sweep();
            run.t_sweep += timed(x->stream, [&] {
                run_sweep(x, run.pin, run.pout, x->d_sig2.p, x->d_qiso.p, x->d_inflow.p, run.icdt, x->d_sig.p, x->d_mom.p);
            });
            if (run.post_sweep()) break;
        }
        run.end(stats);
    });
    return st != SMRT_OK ? st : run.result;
}

extern "C" smrt_status smrt_sweep_resident(smrt_ctx *x, double dt, int n_times, double *ms_per_pass,
                                           double *ms_sweep_kernel) {
    if (!x) { g_last_error = "ctx is NULL"; return SMRT_E_INVALID_ARG; }
    return guard(x, [&] {
        require(dt > 0.0 && n_times >= 1 && ms_per_pass && ms_sweep_kernel, "invalid argument");
        require(x->have_state, "smrt_set_state must be called first");
        void *pin = x->d_psi[x->cur].p, *pout = x->d_psi[1 - x->cur].p;
        std::vector<EventPair> evp(n_times);   // released on every exit path
        SMRT_HIP(hipEventRecord(x->ev0, x->stream));
        for (int k = 0; k < n_times; ++k) {
            const double icdt = prepare_step_tables(x, dt);
            run_source_at(x, x->d_T.p);
            SMRT_HIP(hipEventRecord(evp[k].e0, x->stream));
            run_sweep(x, pin, pout, x->d_sig2.p, x->d_qiso.p, x->d_inflow.p, icdt, x->d_sig.p, x->d_mom.p, false);
            SMRT_HIP(hipEventRecord(evp[k].e1, x->stream));
            if (x->dim == 2) {
                finalize_moments(x, x->d_mom.p);
            } else {
                if (x->fp32) run_moments1d<float>(x->stream, x->nx, x->G, x->nang, (const float *)x->d_mu_w.p, x->d_sig.p, (const float *)pout, x->d_mom.p);
                else run_moments1d<double>(x->stream, x->nx, x->G, x->nang, (const double *)x->d_mu_w.p, x->d_sig.p, (const double *)pout, x->d_mom.p);
            }
            reflect_update(x, pout);
            run_closures(x->stream, closure_args(x, x->opt.scheme == SMRT_SM_INDEPENDENT ? 1 : 0, dt, x->d_mom.p,
                                                 x->d_sigP.p, x->d_sigF.p, x->d_Eho.p, x->d_Fho.p, x->d_clos.p));
        }
        SMRT_HIP(hipEventRecord(x->ev1, x->stream));
        fetch_sweep_flag(x);                       // one wait for the passes and the flag
        SMRT_HIP(hipStreamSynchronize(x->stream));
        float ms = 0.f, ks = 0.f;
        SMRT_HIP(hipEventElapsedTime(&ms, x->ev0, x->ev1));
        for (int k = 0; k < n_times; ++k) {
            float t = 0.f;
            SMRT_HIP(hipEventElapsedTime(&t, evp[k].e0, evp[k].e1));
            ks += t;
        }
        *ms_per_pass = ms / n_times;
        *ms_sweep_kernel = ks / n_times;
        raise_sweep_flag(x);
    });
}

extern "C" smrt_status smrt_get_moments(smrt_ctx *x, double *moments) {
    if (!x) { g_last_error = "ctx is NULL"; return SMRT_E_INVALID_ARG; }
    return guard(x, [&] {
        require(moments != nullptr, "moments is NULL");
        d2h(moments, x->d_mom.p, 8 * x->d_mom.n, x->stream);
        SMRT_HIP(hipStreamSynchronize(x->stream));
    });
}

// ---------------------------------------------------------------------------
// Launch-shape autotuner (one problem): time one sweep per candidate
// (waves per workgroup, groups per lane) on the context's current state and
// keep the fastest.
// ---------------------------------------------------------------------------
struct Shape {
    int nw, nbw, k;
};
static std::vector<Shape> launch_candidates(bool fp32, int G, int nbands) {
    // (waves per band, bands per workgroup, groups per lane): every shape
    // whose chunk covers at most twice the groups a direction has and whose
    // workgroup covers at most twice the bands (beyond that only idle waves
    // are added), within 16 waves
    std::vector<Shape> c;
    for (int k : {1, 2, 4}) {
        if (k == 4 && !fp32) break;
        for (int nw : {1, 2, 4}) {
            const int gb = 4 * k * nw;
            if (gb > 4 && gb >= 2 * std::max(G, 4)) break;
            for (int nbw : {1, 2, 4, 8, 16}) {
                if (nw * nbw > max_waves(fp32, k)) break;
                if (nbw > 1 && nbw >= 2 * nbands) break;
                if (nbw < nbands && nw * nbw > 8) break;   // stacked band groups: at most 8 waves each
                c.push_back({nw, nbw, k});
            }
        }
    }
    return c;
}

extern "C" smrt_status smrt_autotune(smrt_ctx *x, double dt, int *waves_per_band, int *bands_per_group,
                                     int *pairs_per_lane, int *workgroups_per_cu, double *ms_best) {
    if (!x) { g_last_error = "ctx is NULL"; return SMRT_E_INVALID_ARG; }
    return guard(x, [&] {
        require(x->dim == 2, "the launch shape applies to 2D sweeps");
        require(x->have_state, "smrt_set_state must be called first");
        require(dt > 0.0, "dt must be > 0");
        const double icdt = prepare_step_tables(x, dt);
        run_source_at(x, x->d_T.p);
        void *pin = x->d_psi[x->cur].p, *pout = x->d_psi[1 - x->cur].p;
        float best = 1e30f;
        Shape bs{1, 1, 1};
        int bo = 0;
        for (const Shape &c : launch_candidates(x->fp32, x->G, (x->ny + BAND_ROWS - 1) / BAND_ROWS)) {
            SMRT_HIP(hipStreamSynchronize(x->stream));
            x->user_NW = c.nw;
            x->user_NBW = c.nbw;
            x->user_K = c.k;
            plan_sweep(x);
            for (int occ : {0, 1, 2}) {
                x->wg_per_cu = occ;
                auto once = [&] { run_sweep(x, pin, pout, x->d_sig2.p, x->d_qiso.p, x->d_inflow.p, icdt, x->d_sig.p, x->d_mom.p, false); };
                once();   // warm-up
                const float ms = std::min(timed(x->stream, once), timed(x->stream, once));
                check_sweep_flag(x);
                if (ms < best) { best = ms; bs = c; bo = occ; }
            }
        }
        SMRT_HIP(hipStreamSynchronize(x->stream));
        x->user_NW = bs.nw;
        x->user_NBW = bs.nbw;
        x->user_K = bs.k;
        x->wg_per_cu = bo;
        plan_sweep(x);
        if (waves_per_band) *waves_per_band = bs.nw;
        if (bands_per_group) *bands_per_group = bs.nbw;
        if (pairs_per_lane) *pairs_per_lane = bs.k;
        if (workgroups_per_cu) *workgroups_per_cu = bo;
        if (ms_best) *ms_best = best;
    });
}

extern "C" smrt_status smrt_device_name(char *buf, int len, int *n_compute_units) {
    if (!buf || len < 1) { g_last_error = "invalid argument"; return SMRT_E_INVALID_ARG; }
    int dev = 0;
    hipDeviceProp_t pr{};
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&pr, dev) != hipSuccess) {
        g_last_error = "no HIP device";
        return SMRT_E_DEVICE;
    }
    std::snprintf(buf, (size_t)len, "%s %s", pr.name, pr.gcnArchName);
    if (n_compute_units) *n_compute_units = pr.multiProcessorCount;
    return SMRT_OK;
}

// ---------------------------------------------------------------------------
// Batches: every sweep task of many 2D problems in one persistent launch.
// ---------------------------------------------------------------------------
// Device state of smrt_batch_run (its control blocks, LO descriptors and
// barrier, the captured block of outer iterations, per-step events).
struct BatchRunState {
    DevBuf<RunCtl> ctl;      // [n] this step's control blocks
    DevBuf<RunCtl> hist;     // [n_steps][n] control blocks at the end of every step
    DevBuf<LoProb> lo;       // [n]
    DevBuf<unsigned> bar;    // [LO_BAR_WORDS] the batched LO kernel's grid barrier
    DevBuf<int> flags;       // [0] a batched-LO barrier wait past its bound, [1] problems still iterating
    int *h_flags = nullptr;  // pinned: the two flags
    RunCtl *h_ctl = nullptr; // pinned: the control blocks at the end of a step
    std::vector<LoProb> h_lo;
    LoBatch lb{};
    int grid = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<double> graph_dt;   // time steps the captured block of outer iterations was recorded with
    std::vector<hipEvent_t> ev;
    ~BatchRunState() {
        drop();
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
        if (h_flags) (void)hipHostFree(h_flags);
        if (h_ctl) (void)hipHostFree(h_ctl);
    }
    void drop() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
        graph_dt.clear();
    }
};

struct smrt_batch {
    std::string err;
    std::vector<smrt_ctx *> P;
    hipStream_t stream = nullptr;   // the batch's own stream (default priority)
    bool fp32 = false;
    int NW = 0, NBW = 1, K = 1, wg_per_cu = 0;
    DevBuf<Sweep2DArgs> d_args;
    DevBuf<int2> d_tasks;
    DevBuf<int> d_lctr;
    std::vector<Sweep2DArgs> h_args;
    std::vector<int> task_set;    // active set the uploaded task list was built for
    int n_tasks = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    std::unique_ptr<BatchRunState> run;   // device state of smrt_batch_run (made on first use)
    ~smrt_batch() {
        drop_graph();
        if (stream) (void)hipStreamDestroy(stream);
    }
    void drop_graph() {
        if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
        if (graph) (void)hipGraphDestroy(graph);
        graph_exec = nullptr;
        graph = nullptr;
    }
};

// For the duration of a batch call every problem works on the batch stream:
// each problem's own stream is drained first and the batch stream is drained
// before the problems get their streams back.
struct BatchStreams {
    smrt_batch *b;
    std::vector<hipStream_t> saved;
    explicit BatchStreams(smrt_batch *bb) : b(bb) {
        for (smrt_ctx *x : b->P) {
            SMRT_HIP(hipStreamSynchronize(x->stream));
            saved.push_back(x->stream);
            x->stream = b->stream;
        }
    }
    ~BatchStreams() {
        (void)hipStreamSynchronize(b->stream);
        for (size_t i = 0; i < saved.size(); ++i) b->P[i]->stream = saved[i];
    }
};

template <typename F>
static smrt_status bguard(smrt_batch *b, F &&f) {
    try {
        f();
        return SMRT_OK;
    } catch (const smrt::Error &e) {
        if (b) b->err = e.msg;
        g_last_error = e.msg;
        return e.st;
    } catch (const std::bad_alloc &) {
        g_last_error = "host allocation failed";
        return SMRT_E_OUT_OF_MEMORY;
    } catch (...) {
        g_last_error = "unexpected exception";
        return SMRT_E_DEVICE;
    }
}

// re-plan every problem with the batch's launch shape (0 = automatic per field)
static void batch_plan(smrt_batch *b, int nw, int nbw, int k) {
    SMRT_HIP(hipStreamSynchronize(b->stream));
    b->drop_graph();
    b->task_set.clear();
    for (smrt_ctx *x : b->P) {
        x->user_NW = nw;
        x->user_NBW = nbw;
        x->user_K = k;
        plan_sweep(x);
    }
    b->NW = b->P[0]->NW;
    b->NBW = b->P[0]->NBW;
    b->K = b->P[0]->K;
    for (smrt_ctx *x : b->P)
        require(x->NW == b->NW && x->NBW == b->NBW && x->K == b->K,
                "problems of a batch need one launch shape: set it explicitly");
}

// Task list over the given problems: band-group level by level (so every
// band group follows the group below it), and within a level the problems
// with the longest bands first (their pipelines are the critical paths).
static void batch_upload_tasks(smrt_batch *b, const std::vector<int> &active) {
    if (active == b->task_set) return;
    std::vector<int> order(active.size());
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int i, int j) { return b->P[active[i]]->NT > b->P[active[j]]->NT; });
    int maxg = 0;
    for (int p : active) maxg = std::max(maxg, b->P[p]->n_bgroups);
    std::vector<int2> tasks;
    for (int bg = 0; bg < maxg; ++bg)
        for (int i : order) {
            const smrt_ctx *x = b->P[active[i]];
            if (bg >= x->n_bgroups) continue;
            for (int qc = 0; qc < x->NQC; ++qc) tasks.push_back(make_int2(i, bg * x->NQC + qc));
        }
    b->n_tasks = (int)tasks.size();
    b->d_tasks.alloc(std::max<int64_t>(1, b->n_tasks));
    SMRT_HIP(hipMemcpyAsync(b->d_tasks.p, tasks.data(), sizeof(int2) * tasks.size(), hipMemcpyHostToDevice, b->stream));
    SMRT_HIP(hipStreamSynchronize(b->stream));
    b->task_set = active;
}

// argument blocks of the active problems (position i in the launch = active[i])
static void batch_upload_args(smrt_batch *b, const std::vector<int> &active, const std::vector<double> &icdt,
                              const int *const *gates = nullptr) {
    b->h_args.resize(active.size());
    for (size_t i = 0; i < active.size(); ++i) {
        smrt_ctx *x = b->P[active[i]];
        b->h_args[i] = sweep_args(x, x->d_psi[x->cur].p, x->d_psi[1 - x->cur].p, x->d_sig2.p, x->d_qiso.p,
                                  x->d_inflow.p, icdt[active[i]]);
        if (gates) b->h_args[i].gate = gates[active[i]];
    }
    if (b->d_args.n < (int64_t)active.size()) b->d_args.alloc((int64_t)b->P.size());
    SMRT_HIP(hipMemcpyAsync(b->d_args.p, b->h_args.data(), sizeof(Sweep2DArgs) * active.size(), hipMemcpyHostToDevice,
                            b->stream));
    SMRT_HIP(hipStreamSynchronize(b->stream));
}

static void batch_launch(smrt_batch *b) {
    SweepLaunch L{};
    L.probs = b->d_args.p;
    L.tasks = b->d_tasks.p;
    L.n_tasks = b->n_tasks;
    L.NW = b->NW;
    L.NBW = b->NBW;
    L.K = b->K;
    L.wg_per_cu = b->wg_per_cu;
    L.lctr = b->d_lctr.p;
    // one kernel serves the whole batch, so its problems share the fixup setting
    L.fixup = b->P[0]->opt.fixup;
    L.xw = 0;
    for (const smrt_ctx *x : b->P) L.xw |= x->n_bgroups > 1 ? 1 : 0;
    for (const smrt_ctx *x : b->P) require(x->opt.fixup == L.fixup, "problems of a batch share one fixup setting");
    if (b->fp32) launch_sweep2d<float>(L, b->stream);
    else launch_sweep2d<double>(L, b->stream);
}

static std::vector<int> all_problems(const smrt_batch *b) {
    std::vector<int> a(b->P.size());
    std::iota(a.begin(), a.end(), 0);
    return a;
}

extern "C" smrt_status smrt_batch_create(int n, smrt_ctx *const *problems, smrt_batch **out) {
    if (!out || !problems || n < 1) { g_last_error = "invalid argument"; return SMRT_E_INVALID_ARG; }
    *out = nullptr;
    auto b = std::make_unique<smrt_batch>();
    smrt_status st = bguard(b.get(), [&] {
        for (int i = 0; i < n; ++i) {
            smrt_ctx *x = problems[i];
            require(x != nullptr, "NULL problem");
            require(x->dim == 2, "batched sweeps are 2D");
            require(x->have_state, "every problem needs a state (smrt_set_state) before batching");
            require(x->fp32 == problems[0]->fp32, "problems of a batch share one precision");
            for (int j = 0; j < i; ++j) require(problems[j] != x, "a problem appears twice in the batch");
            b->P.push_back(x);
        }
        SMRT_HIP(hipStreamCreate(&b->stream));
        b->fp32 = problems[0]->fp32;
        BatchStreams on(b.get());
        b->d_lctr.alloc(2);
        SMRT_HIP(hipMemsetAsync(b->d_lctr.p, 0, 2 * sizeof(int), b->stream));
        // default shape: the largest problem's automatic one, shared by all
        int big = 0;
        for (int i = 1; i < n; ++i)
            if ((int64_t)b->P[i]->ncell * b->P[i]->nang * b->P[i]->G > (int64_t)b->P[big]->ncell * b->P[big]->nang * b->P[big]->G) big = i;
        smrt_ctx *xb = b->P[big];
        xb->user_NW = 0;
        xb->user_NBW = 0;
        xb->user_K = 0;
        plan_sweep(xb);
        batch_plan(b.get(), xb->NW, xb->NBW, xb->K);
    });
    if (st != SMRT_OK) return st;
    *out = b.release();
    return SMRT_OK;
}

extern "C" void smrt_batch_destroy(smrt_batch *b) {
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    delete b;
}

extern "C" const char *smrt_batch_last_error(const smrt_batch *b) { return b ? b->err.c_str() : g_last_error.c_str(); }

extern "C" smrt_status smrt_batch_set_launch(smrt_batch *b, int waves_per_band, int bands_per_group,
                                             int pairs_per_lane) {
    if (!b) { g_last_error = "batch is NULL"; return SMRT_E_INVALID_ARG; }
    return bguard(b, [&] {
        BatchStreams on(b);
        check_shape(b->fp32, waves_per_band, bands_per_group, pairs_per_lane, false);
        batch_plan(b, waves_per_band, bands_per_group, pairs_per_lane);
    });
}

extern "C" smrt_status smrt_batch_set_occupancy(smrt_batch *b, int workgroups_per_cu) {
    if (!b) { g_last_error = "batch is NULL"; return SMRT_E_INVALID_ARG; }
    return bguard(b, [&] {
        require(workgroups_per_cu >= 0 && workgroups_per_cu <= 8, "workgroups per CU must be in [0, 8]");
        b->drop_graph();
        b->wg_per_cu = workgroups_per_cu;
    });
}

extern "C" smrt_status smrt_batch_info(const smrt_batch *b, int64_t *units_per_sweep, int *n_tasks,
                                       int *waves_per_band, int *bands_per_group, int *pairs_per_lane) {
    if (!b) { g_last_error = "batch is NULL"; return SMRT_E_INVALID_ARG; }
    int64_t u = 0, t = 0;
    for (const smrt_ctx *x : b->P) {
        u += (int64_t)x->ncell * x->nang * x->G;
        t += x->n_wg;
    }
    if (units_per_sweep) *units_per_sweep = u;
    if (n_tasks) *n_tasks = (int)t;
    if (waves_per_band) *waves_per_band = b->NW;
    if (bands_per_group) *bands_per_group = b->NBW;
    if (pairs_per_lane) *pairs_per_lane = b->K;
    return SMRT_OK;
}

// tables, sources and one batched sweep of every problem (+ finalisation and closures)
static void batch_tables(smrt_batch *b, double dt, std::vector<double> &icdt) {
    icdt.assign(b->P.size(), 0.0);
    for (size_t i = 0; i < b->P.size(); ++i) {
        smrt_ctx *x = b->P[i];
        icdt[i] = prepare_step_tables(x, dt);
        run_source_at(x, x->d_T.p);
    }
}
static void batch_post(smrt_batch *b, double dt) {
    for (smrt_ctx *x : b->P) {
        finalize_moments(x, x->d_mom.p);
        reflect_update(x, x->d_psi[1 - x->cur].p);
        run_closures(x->stream, closure_args(x, x->opt.scheme == SMRT_SM_INDEPENDENT ? 1 : 0, dt, x->d_mom.p,
                                             x->d_sigP.p, x->d_sigF.p, x->d_Eho.p, x->d_Fho.p, x->d_clos.p));
    }
}

extern "C" smrt_status smrt_batch_sweep_resident(smrt_batch *b, double dt, int n_times, int capture_graph,
                                                 double *ms_per_pass, double *ms_sweep_kernel) {
    if (!b) { g_last_error = "batch is NULL"; return SMRT_E_INVALID_ARG; }
    return bguard(b, [&] {
        BatchStreams on(b);
        require(dt > 0.0 && n_times >= 1 && ms_per_pass && ms_sweep_kernel, "invalid argument");
        const std::vector<int> all = all_problems(b);
        std::vector<double> icdt(b->P.size());
        for (size_t i = 0; i < b->P.size(); ++i) icdt[i] = 1.0 / (b->P[i]->c * dt);
        batch_upload_tasks(b, all);
        batch_upload_args(b, all, icdt);
        // the batched sweep alone (eager), for the kernel time
        batch_tables(b, dt, icdt);
        batch_launch(b);
        SMRT_HIP(hipStreamSynchronize(b->stream));
        float ks = 1e30f;
        for (int r = 0; r < 2; ++r) ks = std::min(ks, timed(b->stream, [&] { batch_launch(b); }));
        for (smrt_ctx *x : b->P) check_sweep_flag(x);
        auto pass = [&] {
            std::vector<double> ic;
            batch_tables(b, dt, ic);
            batch_launch(b);
            batch_post(b, dt);
        };
        float ms = 0.f;
        if (capture_graph) {
            b->drop_graph();
            SMRT_HIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
            try {
                pass();
            } catch (...) {
                hipGraph_t g = nullptr;
                (void)hipStreamEndCapture(b->stream, &g);
                if (g) (void)hipGraphDestroy(g);
                throw;
            }
            SMRT_HIP(hipStreamEndCapture(b->stream, &b->graph));
            SMRT_HIP(hipGraphInstantiate(&b->graph_exec, b->graph, nullptr, nullptr, 0));
            SMRT_HIP(hipGraphLaunch(b->graph_exec, b->stream));   // warm-up replay
            SMRT_HIP(hipStreamSynchronize(b->stream));
            ms = timed(b->stream, [&] {
                for (int k = 0; k < n_times; ++k) SMRT_HIP(hipGraphLaunch(b->graph_exec, b->stream));
            });
        } else {
            ms = timed(b->stream, [&] {
                for (int k = 0; k < n_times; ++k) pass();
            });
        }
        for (smrt_ctx *x : b->P) check_sweep_flag(x);
        *ms_per_pass = ms / n_times;
        *ms_sweep_kernel = ks;
    });
}

extern "C" smrt_status smrt_batch_autotune(smrt_batch *b, double dt, int *waves_per_band, int *bands_per_group,
                                           int *pairs_per_lane, int *workgroups_per_cu, double *ms_best) {
    if (!b) { g_last_error = "batch is NULL"; return SMRT_E_INVALID_ARG; }
    return bguard(b, [&] {
        BatchStreams on(b);
        require(dt > 0.0, "dt must be > 0");
        int maxg = 0, maxb = 0;
        for (const smrt_ctx *x : b->P) {
            maxg = std::max(maxg, x->G);
            maxb = std::max(maxb, x->nbands);
        }
        float best = 1e30f;
        Shape bs{b->NW, b->NBW, b->K};
        const std::vector<int> all = all_problems(b);
        int bo = 0;
        for (const Shape &c : launch_candidates(b->fp32, maxg, maxb)) {
            batch_plan(b, c.nw, c.nbw, c.k);
            std::vector<double> icdt;
            batch_tables(b, dt, icdt);
            batch_upload_tasks(b, all);
            batch_upload_args(b, all, icdt);
            for (int occ : {0, 1, 2}) {
                b->wg_per_cu = occ;
                batch_launch(b);   // warm-up
                const float ms = std::min(timed(b->stream, [&] { batch_launch(b); }), timed(b->stream, [&] { batch_launch(b); }));
                for (smrt_ctx *x : b->P) check_sweep_flag(x);
                if (ms < best) { best = ms; bs = c; bo = occ; }
            }
        }
        batch_plan(b, bs.nw, bs.nbw, bs.k);
        b->wg_per_cu = bo;
        if (waves_per_band) *waves_per_band = bs.nw;
        if (bands_per_group) *bands_per_group = bs.nbw;
        if (pairs_per_lane) *pairs_per_lane = bs.k;
        if (workgroups_per_cu) *workgroups_per_cu = bo;
        if (ms_best) *ms_best = best;
    });
}

extern "C" smrt_status smrt_batch_step(smrt_batch *b, const double *dt, smrt_step_stats *stats) {
    if (!b) { g_last_error = "batch is NULL"; return SMRT_E_INVALID_ARG; }
    const size_t n = b->P.size();
    std::vector<StepRun> runs(n);
    smrt_status result = SMRT_OK;
    smrt_status st = bguard(b, [&] {
        BatchStreams on(b);
        require(dt != nullptr, "dt is NULL");
        for (size_t i = 0; i < n; ++i) runs[i].begin(b->P[i], dt[i]);
        std::vector<int> active = all_problems(b);
        while (!active.empty()) {
            std::vector<double> icdt(n, 0.0);
            for (int p : active) {
                runs[p].pre_sweep();
                icdt[p] = runs[p].icdt;
            }
            batch_upload_tasks(b, active);
            batch_upload_args(b, active, icdt);
            const float ms = timed(b->stream, [&] {
                batch_launch(b);
                for (int p : active) finalize_moments(b->P[p], b->P[p]->d_mom.p);
            });
            std::vector<int> next;
            for (int p : active) {
                runs[p].t_sweep += ms;
                if (!runs[p].post_sweep()) next.push_back(p);
            }
            active.swap(next);
        }
        for (size_t i = 0; i < n; ++i) {
            const smrt_status r = runs[i].end(stats ? stats + i : nullptr);
            if (r != SMRT_OK && result == SMRT_OK) {
                result = r;
                b->err = "problem " + std::to_string(i) + ": " + b->P[i]->err;
            }
        }
    });
    if (st == SMRT_OK && result != SMRT_OK) g_last_error = b->err;
    return st != SMRT_OK ? st : result;
}

// ---------------------------------------------------------------------------
// Multi-step batched run with device-side convergence control
// ---------------------------------------------------------------------------
// Each problem's outer iteration (Algorithm 1) is decided on the device from
// its control block, and its LO solve (Newton and CG, Sec. 5) runs inside the
// batched LO kernel, so the host queues blocks of RUN_BLOCK outer iterations
// and waits once per block to learn whether any problem still iterates.  A
// problem whose step has converged skips every kernel of the remaining
// outer iterations of the block: each takes the problem's control-block flag
// as a gate (the batched sweep and LO per problem, the per-problem kernels
// as a whole).
constexpr int RUN_BLOCK = 4;

__global__ void k_run_begin(RunCtl *ctl, int n) {
    const int p = threadIdx.x;
    if (p >= n) return;
    RunCtl c{};
    c.active = 1;
    c.first = -1.0;
    c.first_in = -1.0;
    ctl[p] = c;
}

// The end of one outer iteration of one problem: the checks StepRun::post_sweep
// makes on the host, on the iterate change |T - T_l|^2 + |E - E_l|^2 in sc[6].
__global__ void k_outer_decide(RunCtl *ctl, const double *sc, const int *sweep_ctr, int fixed_outer, int maxo,
                               double eps_outer) {
    RunCtl &c = *ctl;
    if (!c.active) return;
    c.l += 1;
    c.outer += 1;
    const double diff = sqrt(sc[6]);
    bool done = false;
    if (c.status != SMRT_OK) {
        done = true;                                   // its LO solve failed
    } else if (sweep_ctr[3]) {
        c.status = SMRT_E_DEVICE;
        c.reason = RUN_SWEEP_WAIT;
        done = true;
    } else if (!isfinite(diff)) {
        c.status = SMRT_E_NONPHYSICAL;
        c.reason = RUN_OUTER_NONFINITE;
        done = true;
    } else if (fixed_outer > 0) {
        done = c.l >= maxo;
    } else {
        if (c.l == 1) c.first = diff;
        if (diff == 0.0 || (c.l > 1 && diff < eps_outer * c.first)) done = true;
        else if (c.l == maxo) {
            c.hit_max = 1;
            done = true;
        }
    }
    if (done) c.active = 0;
}

// a = b and c = d (n doubles each), skipped while *gate is 0
__global__ void k_copy2_gated(const int *gate, int64_t n, double *a, const double *b, double *c, const double *d) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n || !*gate) return;
    a[i] = b[i];
    c[i] = d[i];
}

// flags[1] = problems still iterating (one thread)
__global__ void k_run_count(const RunCtl *ctl, int n, int *flags) {
    int a = 0;
    for (int p = 0; p < n; ++p) a += ctl[p].active;
    flags[1] = a;
}

// One outer iteration of every problem; a converged problem (its control
// block no longer active) skips every kernel of it.
static void run_outer_iteration(smrt_batch *b, BatchRunState &R, const std::vector<double> &dt) {
    hipStream_t S = b->stream;
    const size_t n = b->P.size();
    for (size_t i = 0; i < n; ++i) run_source_at(b->P[i], b->P[i]->d_Tl.p, &R.ctl.p[i].active);
    batch_launch(b);
    for (size_t i = 0; i < n; ++i) {
        smrt_ctx *x = b->P[i];
        const int *on = &R.ctl.p[i].active;
        finalize_moments(x, x->d_mom.p, nullptr, on);
        hipLaunchKernelGGL(k_copy2_gated, dim3(nblk(x->nn)), dim3(256), 0, S, on, (int64_t)x->nn, x->d_Tn.p,
                           (const double *)x->d_Tl.p, x->d_En.p, (const double *)x->d_El.p);
        ClosureArgs ca = closure_args(x, x->opt.scheme == SMRT_SM_INDEPENDENT ? 1 : 0, dt[i], x->d_mom.p, x->d_sigP.p,
                                      x->d_sigF.p, x->d_Estar.p, x->d_Fstar.p, x->d_clos.p);
        ca.gate = on;
        run_closures(S, ca);
    }
    run_lo_batch(S, R.lb, R.grid);
    for (size_t i = 0; i < n; ++i) {
        smrt_ctx *x = b->P[i];
        const int *on = &R.ctl.p[i].active;
        x->lo.dot_gated(S, on, x->d_Tn.p, nullptr, x->d_Tl.p, 6, false);
        x->lo.dot_gated(S, on, x->d_En.p, nullptr, x->d_El.p, 6, true);
        // the copies precede the decision, which may clear the flag that gates them
        hipLaunchKernelGGL(k_copy2_gated, dim3(nblk(x->nn)), dim3(256), 0, S, on, (int64_t)x->nn, x->d_Tl.p,
                           (const double *)x->d_Tn.p, x->d_El.p, (const double *)x->d_En.p);
        const int maxo = x->opt.fixed_outer > 0 ? x->opt.fixed_outer : x->opt.max_outer;
        hipLaunchKernelGGL(k_outer_decide, dim3(1), dim3(1), 0, S, R.ctl.p + i, (const double *)x->lo.sc.p,
                           (const int *)x->d_ctr.p, x->opt.fixed_outer, maxo, x->opt.eps_outer);
    }
}

static LoProb lo_prob(smrt_ctx *x, double dt, RunCtl *ctl) {
    LoSolver &L = x->lo;
    const LoInputs in = lo_inputs(x, dt, x->d_clos.p);
    LoProb q{};
    q.nn = L.nn;
    q.dim = L.dim;
    q.nbk = (L.nn + 255) / 256;
    q.nbkd = (L.nn * L.dim + 255) / 256;
    q.g = L.geom();
    q.a = L.a;
    q.c = L.c;
    q.dt = dt;
    q.eps_inner = in.eps_inner;
    q.cg_rtol = in.cg_rtol;
    q.elim_rtol = in.elim_rtol;
    q.T_floor = in.T_floor;
    q.max_inner = in.max_inner;
    q.max_cg = in.max_cg;
    q.max_elim = in.max_elim;
    q.drp = L.dD.rp; q.dcol = L.dD.col; q.dval = L.dD.val;
    q.dtrp = L.dDT.rp; q.dtcol = L.dDT.col; q.dtval = L.dDT.val;
    q.prp = L.dP.rp; q.pcol = L.dP.col; q.pval = L.dP.val;
    q.wn = L.wn.p;
    q.MFinv = L.MFinv.p; q.DqF = L.DqF.p; q.jbase = L.jbase.p; q.diagE = L.diagE.p; q.rhs = L.rhs.p;
    q.Minv = L.Minv.p; q.r = L.r.p; q.z = L.z.p; q.p = L.p.p; q.Ap = L.Ap.p; q.Eold = L.Eold.p; q.Told = L.Told.p;
    q.tmpF = L.tmpF.p; q.part = L.part.p; q.sc = L.sc.p; q.bpart = L.bpart.p; q.apart = L.apart.p; q.sc2 = L.sc2.p;
    q.flags = L.flags.p;
    q.sigE = in.sigE; q.sigF = in.sigF; q.sigP = in.sigP; q.qE = in.qE; q.qF = in.qF; q.cvn = in.cvn;
    q.Tstar = x->d_Tstar.p;
    q.E = x->d_En.p;
    q.F = x->d_F.p;
    q.T = x->d_Tn.p;
    q.ctl = ctl;
    return q;
}

static const char *run_reason(int r) {
    switch (r) {
    case RUN_NO_ROOT: return "no positive temperature root in the energy balance";
    case RUN_LO_NONFINITE: return "non-finite low-order iterate";
    case RUN_OUTER_NONFINITE: return "non-finite outer iterate";
    case RUN_SWEEP_WAIT: return "sweep band-trace wait exceeded its bound";
    default: return "step failed";
    }
}

extern "C" smrt_status smrt_batch_run(smrt_batch *b, int n_steps, const double *dt, smrt_step_stats *stats,
                                      int capture_graph) {
    if (!b) { g_last_error = "batch is NULL"; return SMRT_E_INVALID_ARG; }
    const size_t n = b->P.size();
    smrt_status result = SMRT_OK;
    smrt_status st = bguard(b, [&] {
        require(n_steps >= 1 && dt != nullptr, "n_steps must be >= 1 and dt non-NULL");
        require(n <= (size_t)LO_BATCH_MAX, "a batched run takes at most 64 problems");
        for (int64_t k = 0; k < (int64_t)n_steps * (int64_t)n; ++k)
            require(dt[k] > 0.0 && std::isfinite(dt[k]), "dt must be finite and > 0");
        for (const smrt_ctx *x : b->P) {
            require(x->opt.scheme != SMRT_UNACCELERATED, "a batched run needs an SM scheme (the LO solve)");
            require(x->opt.lo_precond == 0, "a batched run uses the Jacobi-preconditioned LO (lo_precond = 0)");
            require(!x->refl, "a batched run has no reflective sides");
        }
        BatchStreams on(b);
        hipStream_t S = b->stream;
        if (!b->run) b->run = std::make_unique<BatchRunState>();
        BatchRunState &R = *b->run;
        R.drop();
        if (R.ctl.n != (int64_t)n) {
            R.ctl.alloc((int64_t)n);
            R.lo.alloc((int64_t)n);
        }
        if (R.hist.n < (int64_t)n_steps * (int64_t)n) R.hist.alloc((int64_t)n_steps * (int64_t)n);
        if (!R.bar.p) R.bar.alloc(LO_BAR_WORDS);
        if (!R.flags.p) R.flags.alloc(2);
        if (!R.h_flags) SMRT_HIP(hipHostMalloc((void **)&R.h_flags, 2 * sizeof(int), hipHostMallocDefault));
        if (!R.h_ctl) SMRT_HIP(hipHostMalloc((void **)&R.h_ctl, LO_BATCH_MAX * sizeof(RunCtl), hipHostMallocDefault));
        while ((int)R.ev.size() < n_steps + 1) {
            hipEvent_t e;
            SMRT_HIP(hipEventCreate(&e));
            R.ev.push_back(e);
        }
        hipLaunchKernelGGL(k_zero_int, dim3(nblk(LO_BAR_WORDS)), dim3(256), 0, S, (int *)R.bar.p, LO_BAR_WORDS);
        hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, S, R.flags.p, 2);
        R.lb = LoBatch{};
        R.lb.P = R.lo.p;
        R.lb.np = (int)n;
        R.lb.bar = R.bar.p;
        R.lb.abort = R.flags.p;
        R.h_lo.resize(n);
        for (size_t i = 0; i < n; ++i) R.lb.vb_n[i + 1] = R.lb.vb_n[i] + (b->P[i]->lo.nn + 255) / 256;
        if (!R.grid) R.grid = lo_batch_grid(R.lb.vb_n[n]);
        std::vector<const int *> gates(n);
        for (size_t i = 0; i < n; ++i) gates[i] = &R.ctl.p[i].active;
        const std::vector<int> all = all_problems(b);
        batch_upload_tasks(b, all);
        SMRT_HIP(hipEventRecord(R.ev[0], S));
        int steps_done = 0;
        for (int s = 0; s < n_steps; ++s) {
            const std::vector<double> dts(dt + (int64_t)s * n, dt + (int64_t)(s + 1) * n);
            std::vector<StepRun> runs(n);
            std::vector<double> icdt(n);
            for (size_t i = 0; i < n; ++i) {
                runs[i].begin(b->P[i], dts[i]);
                icdt[i] = runs[i].icdt;
                R.h_lo[i] = lo_prob(b->P[i], dts[i], R.ctl.p + i);
            }
            hipLaunchKernelGGL(k_run_begin, dim3(1), dim3(LO_BATCH_MAX), 0, S, R.ctl.p, (int)n);
            SMRT_HIP(hipMemcpyAsync(R.lo.p, R.h_lo.data(), sizeof(LoProb) * n, hipMemcpyHostToDevice, S));
            batch_upload_args(b, all, icdt, gates.data());   // waits for the uploads
            // blocks of outer iterations until no problem iterates
            int max_blocks = 0;
            for (const smrt_ctx *x : b->P) {
                const int maxo = x->opt.fixed_outer > 0 ? x->opt.fixed_outer : x->opt.max_outer;
                max_blocks = std::max(max_blocks, (maxo + RUN_BLOCK - 1) / RUN_BLOCK);
            }
            for (int blk = 0;; ++blk) {
                require(blk < max_blocks, "batched run: outer iterations past every problem's cap");
                if (capture_graph) {
                    if (!R.exec || R.graph_dt != dts) {
                        R.drop();
                        SMRT_HIP(hipStreamBeginCapture(S, hipStreamCaptureModeThreadLocal));
                        try {
                            for (int k = 0; k < RUN_BLOCK; ++k) run_outer_iteration(b, R, dts);
                        } catch (...) {
                            hipGraph_t g = nullptr;
                            (void)hipStreamEndCapture(S, &g);
                            if (g) (void)hipGraphDestroy(g);
                            throw;
                        }
                        SMRT_HIP(hipStreamEndCapture(S, &R.graph));
                        SMRT_HIP(hipGraphInstantiate(&R.exec, R.graph, nullptr, nullptr, 0));
                        R.graph_dt = dts;
                    }
                    SMRT_HIP(hipGraphLaunch(R.exec, S));
                } else {
                    for (int k = 0; k < RUN_BLOCK; ++k) run_outer_iteration(b, R, dts);
                }
                hipLaunchKernelGGL(k_run_count, dim3(1), dim3(1), 0, S, R.ctl.p, (int)n, R.flags.p);
                SMRT_HIP(hipMemcpyAsync(R.h_flags, R.flags.p, 2 * sizeof(int), hipMemcpyDeviceToHost, S));
                SMRT_HIP(hipStreamSynchronize(S));
                if (R.h_flags[0]) throw smrt::Error(SMRT_E_DEVICE, "batched LO: a grid-barrier wait exceeded its bound");
                if (R.h_flags[1] == 0) break;
            }
            // the new state of every problem (StepRun::end, without its wait)
            for (size_t i = 0; i < n; ++i) {
                smrt_ctx *x = b->P[i];
                const int64_t nn = x->nn;
                SMRT_HIP(hipMemcpyAsync(x->d_T.p, x->d_Tl.p, 8 * nn, hipMemcpyDeviceToDevice, S));
                SMRT_HIP(hipMemcpyAsync(x->d_E.p, x->d_El.p, 8 * nn, hipMemcpyDeviceToDevice, S));
                hipLaunchKernelGGL(k_ho_from_mom, dim3(nblk(nn)), dim3(256), 0, S, (int)nn, x->dim, x->c, x->d_mom.p,
                                   x->d_sigP.p, x->d_Eho.p, x->d_Fho.p, (double *)nullptr);
                x->cur = 1 - x->cur;
            }
            SMRT_HIP(hipMemcpyAsync(R.hist.p + (int64_t)s * n, R.ctl.p, sizeof(RunCtl) * n, hipMemcpyDeviceToDevice, S));
            SMRT_HIP(hipMemcpyAsync(R.h_ctl, R.ctl.p, sizeof(RunCtl) * n, hipMemcpyDeviceToHost, S));
            SMRT_HIP(hipEventRecord(R.ev[s + 1], S));
            SMRT_HIP(hipStreamSynchronize(S));
            steps_done = s + 1;
            bool failed = false;
            for (size_t i = 0; i < n; ++i) {
                const RunCtl &c = R.h_ctl[i];
                smrt_ctx *x = b->P[i];
                if (c.reason == RUN_SWEEP_WAIT) {
                    // clear the sweep's wait flag and trace words, as a single step does
                    hipLaunchKernelGGL(k_init_ctr, dim3(1), dim3(1), 0, S, x->d_ctr.p);
                    SMRT_HIP(hipMemsetAsync(x->d_trace.p, 0, sizeof(uint64_t) * x->d_trace.n, S));
                }
                smrt_status ps = (smrt_status)c.status;
                std::string why = ps != SMRT_OK ? run_reason(c.reason) : "";
                if (ps == SMRT_OK && x->opt.strict && c.hit_max) {
                    ps = SMRT_E_NOT_CONVERGED;
                    why = "iteration cap reached";
                }
                if (ps != SMRT_OK && result == SMRT_OK) {
                    result = ps;
                    b->err = "step " + std::to_string(s) + ", problem " + std::to_string(i) + ": " + why;
                }
                if (ps != SMRT_OK) failed = true;
            }
            SMRT_HIP(hipStreamSynchronize(S));
            if (failed) break;
        }
        if (stats) {
            std::vector<RunCtl> h((size_t)steps_done * n);
            if (!h.empty())
                SMRT_HIP(hipMemcpy(h.data(), R.hist.p, sizeof(RunCtl) * h.size(), hipMemcpyDeviceToHost));
            for (int s = 0; s < n_steps; ++s) {
                float ms = 0.f;
                if (s < steps_done) SMRT_HIP(hipEventElapsedTime(&ms, R.ev[s], R.ev[s + 1]));
                for (size_t i = 0; i < n; ++i) {
                    smrt_step_stats &o = stats[(int64_t)s * n + i];
                    o = smrt_step_stats{};
                    if (s >= steps_done) continue;
                    const RunCtl &c = h[(size_t)s * n + i];
                    o.outer = c.outer;
                    o.inner_total = c.inner_total;
                    o.cg_total = c.cg_total;
                    o.elim_max = c.elim_max;
                    o.hit_max = c.hit_max;
                    o.t_total_ms = ms;
                }
            }
        }
        R.drop();
    });
    if (st == SMRT_OK && result != SMRT_OK) g_last_error = b->err;
    return st != SMRT_OK ? st : result;
}

// ---------------------------------------------------------------------------
// Materials update (per-region sigma0 and c_v), e.g. between gradient steps
// ---------------------------------------------------------------------------
extern "C" smrt_status smrt_set_materials(smrt_ctx *x, const double *sigma0, const double *cv) {
    if (!x) { g_last_error = "ctx is NULL"; return SMRT_E_INVALID_ARG; }
    return guard(x, [&] {
        require(sigma0 != nullptr || cv != nullptr, "nothing to set");
        if (sigma0) {
            const size_t ns = x->sigma0.size();
            for (size_t k = 0; k < ns; ++k) require(std::isfinite(sigma0[k]) && sigma0[k] >= 0.0, "sigma0 must be >= 0");
            std::copy(sigma0, sigma0 + ns, x->sigma0.begin());
            SMRT_HIP(hipMemcpy(x->d_sigma0.p, x->sigma0.data(), 8 * ns, hipMemcpyHostToDevice));
        }
        if (cv) {
            for (int r = 0; r < x->nreg; ++r) require(std::isfinite(cv[r]) && cv[r] > 0.0, "c_v must be > 0");
            std::copy(cv, cv + x->nreg, x->cv.begin());
            std::vector<double> cvn(x->nn);
            for (int n = 0; n < x->nn; ++n) cvn[n] = x->cv[x->region[n / x->npc]];
            SMRT_HIP(hipMemcpy(x->d_cvn.p, cvn.data(), 8 * x->nn, hipMemcpyHostToDevice));
        }
    });
}

// ---------------------------------------------------------------------------
// Adjoint gradient of the time-integrated right-boundary outflow
//   J = sum_k dt sum_g sum_{mu_d > 0} w_d mu_d sum_{n on x+} fw_n I^k_n
// with respect to log sigma0_r and log c_v,r, at the converged fixed point of
// every step (implicit function theorem): forward steps with checkpoints of
// (I^k, T^k, sigma^k), then, backwards, the adjoint of each step by source
// iteration (adjoint sweep + pointwise temperature adjoint) and the
// sensitivities of the opacity and heat-capacity terms.
// ---------------------------------------------------------------------------
static void adjoint_sweep_dev(smrt_ctx *x, const double *sigt, const double *src, double *lam, double *prev_tmp,
                              double *out_tmp, const double *zq, const double *zinf, RawScratch *scratch = nullptr) {
    const int64_t per = (int64_t)x->G * x->nn;
    run_permute_dirs(x->stream, x->nang, per, x->d_opposite.p, src, prev_tmp);
    raw_sweep(x, sigt, sigt, zq, prev_tmp, 1.0, zinf, out_tmp, nullptr, scratch);
    run_permute_dirs(x->stream, x->nang, per, x->d_opposite.p, out_tmp, lam);
}

static void psi_state_to_abi(smrt_ctx *x, double *out) {
    const int64_t na = (int64_t)x->nang * x->G * x->nn;
    if (x->dim == 2) {
        if (x->fp32) run_psi_from_internal<float>(x->stream, x->nx, x->ny, x->G, x->nang, x->d_dir_quad.p, (const float *)x->d_psi[x->cur].p, out);
        else run_psi_from_internal<double>(x->stream, x->nx, x->ny, x->G, x->nang, x->d_dir_quad.p, (const double *)x->d_psi[x->cur].p, out);
    } else {
        if (x->fp32) run_copy_from<float>(x->stream, na, (const float *)x->d_psi[x->cur].p, out);
        else run_copy_from<double>(x->stream, na, (const double *)x->d_psi[x->cur].p, out);
    }
}

extern "C" smrt_status smrt_adjoint(smrt_ctx *x, int objective, int n_steps, double dt, double *J_out,
                                    double *grad_log_sigma0, double *grad_log_cv, int *adjoint_iterations) {
    if (!x) { g_last_error = "ctx is NULL"; return SMRT_E_INVALID_ARG; }
    return guard(x, [&] {
        require(objective == 0 || objective == 1,
                "objective must be 0 (time-integrated right-boundary outflow) or 1 (final material energy)");
        require(n_steps >= 1 && dt > 0.0 && std::isfinite(dt), "n_steps >= 1 and dt > 0 required");
        require(J_out && grad_log_sigma0 && grad_log_cv, "NULL output");
        require(x->have_state, "smrt_set_state must be called first");
        require(x->have_opposite, "the quadrature has a direction without its opposite: no adjoint sweep");
        require(x->model == 1, "the gradient is defined for the power-law opacity model (one sigma0 per region)");
        require(x->opt.fixup == 0 && x->opt.T_floor == 0.0,
                "the adjoint differentiates the linear sweep and the unfloored energy balance: fixup and T_floor must be off");
        require(x->refl == 0, "the adjoint takes vacuum or given inflow on every side (no reflective side)");
        hipStream_t S = x->stream;
        const int N = n_steps, nn = x->nn, nc = x->ncell, G = x->G, npc = x->npc, nreg = x->nreg;
        const int64_t npsi = (int64_t)x->nang * G * nn, ncg = (int64_t)nc * G;
        const int ny1 = x->dim == 2 ? x->ny : 1;
        const double *hy = x->dim == 2 ? x->d_hy64.p : nullptr;
        DevBuf<double> ck_psi, ck_T, ck_sig, dJdI, part, scal, wc;
        ck_psi.alloc(npsi * (N + 1));
        ck_T.alloc((int64_t)nn * (N + 1));
        ck_sig.alloc(ncg * (N + 1));
        dJdI.alloc(npsi);
        part.alloc(std::max<int64_t>(256, 2 * ((nn + 255) / 256)));
        scal.alloc(4);
        wc.alloc(nn);
        if (objective == 0) {
            run_adj_dJdI(S, x->dim, x->nx, ny1, G, x->nang, x->d_om.p, x->d_w.p, hy, dt, dJdI.p);
        } else {
            // J = sum_n w_n c_v,n T^N_n: no direct dependence on I
            dJdI.zero(S);
            run_adj_energy_weights(S, x->dim, x->nx, npc, nn, x->d_hx64.p, hy, x->d_cvn.p, wc.p);
        }
        // forward with checkpoints
        psi_state_to_abi(x, ck_psi.p);
        SMRT_HIP(hipMemcpyAsync(ck_T.p, x->d_T.p, 8 * nn, hipMemcpyDeviceToDevice, S));
        double J = 0.0;
        for (int k = 1; k <= N; ++k) {
            StepRun run;
            run.begin(x, dt);
            SMRT_HIP(hipMemcpyAsync(ck_sig.p + ncg * k, x->d_sig.p, 8 * ncg, hipMemcpyDeviceToDevice, S));
            for (;;) {
                run.pre_sweep();
                run.t_sweep += timed(S, [&] {
                    run_sweep(x, run.pin, run.pout, x->d_sig2.p, x->d_qiso.p, x->d_inflow.p, run.icdt, x->d_sig.p, x->d_mom.p);
                });
                if (run.post_sweep()) break;
            }
            const smrt_status r = run.end(nullptr);
            if (r != SMRT_OK) throw smrt::Error(r, "forward step " + std::to_string(k) + ": " + x->err);
            psi_state_to_abi(x, ck_psi.p + npsi * k);
            SMRT_HIP(hipMemcpyAsync(ck_T.p + (int64_t)nn * k, x->d_T.p, 8 * nn, hipMemcpyDeviceToDevice, S));
            if (objective == 0) {
                run_dot(S, npsi, dJdI.p, ck_psi.p + npsi * k, part.p, scal.p);
                double jk = 0.0;
                read_small(x, &jk, scal.p, 8);
                J += jk;
            }
        }
        const double *TN = ck_T.p + (int64_t)nn * N;
        if (objective == 1) {
            run_dot(S, nn, wc.p, TN, part.p, scal.p);
            read_small(x, &J, scal.p, 8);
        }
        // reverse
        DevBuf<double> lam, lam_next, src, prev_tmp, out_tmp, zq, zinf, sigt, tau, tau_new, ST, ST_prev, emis, dE, phi, D,
            dsig, gs_cell, gcv_node, gs, gc;
        lam.alloc(npsi); lam_next.alloc(npsi); src.alloc(npsi); prev_tmp.alloc(npsi); out_tmp.alloc(npsi);
        zq.alloc((int64_t)nn * G); zinf.alloc((int64_t)x->nang * G * x->NB);
        sigt.alloc(ncg); tau.alloc(nn); tau_new.alloc(nn); ST.alloc(nn); ST_prev.alloc(nn);
        emis.alloc((int64_t)nn * G); dE.alloc((int64_t)nn * G); phi.alloc((int64_t)nn * G); D.alloc(nn);
        dsig.alloc(ncg); gs_cell.alloc(nc); gcv_node.alloc(nn); gs.alloc(nreg); gc.alloc(nreg);
        lam_next.zero(S); zq.zero(S); zinf.zero(S); ST.zero(S); gs.zero(S); gc.zero(S);
        // Anderson acceleration of each step's temperature iteration (window AA_M)
        constexpr int AA_M = 5;
        static_assert(AA_M <= AA_MAX, "Anderson window too large");
        DevBuf<double> dFr, dGr, fprev, gprev, aapart, aaout;
        dFr.alloc((int64_t)AA_M * nn); dGr.alloc((int64_t)AA_M * nn); fprev.alloc(nn); gprev.alloc(nn);
        aapart.alloc((int64_t)2 * AA_M * ((nn + 255) / 256)); aaout.alloc(2 * AA_M);
        RawScratch rsc;   // the adjoint sweeps' scratch, allocated once
        // objective 1: dJ/dT^N = w c_v enters the energy-balance adjoint of the last step
        if (objective == 1) run_add_scalar(S, nn, wc.p, 0.0, ST.p);
        const double icdt = 1.0 / (x->c * dt);
        int iters = 0;
        for (int k = N; k >= 1; --k) {
            const double *psi = ck_psi.p + npsi * k, *T = ck_T.p + (int64_t)nn * k, *Tp = ck_T.p + (int64_t)nn * (k - 1);
            const double *sig = ck_sig.p + ncg * k;
            run_add_scalar(S, ncg, sig, icdt, sigt.p);
            run_adj_prep(S, nn, npc, G, x->nang, x->d_nu.p, x->a, x->c, dt, T, sig, x->d_cvn.p, x->d_w.p, psi, emis.p,
                         dE.p, D.p, phi.p);
            // tau <- g(tau) = (pointwise temperature adjoint)(adjoint sweep(tau)), a linear
            // fixed point, solved by Anderson acceleration: tau_{k+1} = g_k - dG gamma with
            // gamma = argmin |f_k - dF gamma| over the last AA_M differences of f = g - tau
            // and g (normal equations, Cholesky); a failed solve restarts the window.
            tau.zero(S);
            int win[AA_M], nwin = 0, next_slot = 0;
            double Mg[AA_M][AA_M] = {};
            for (int it = 0; it < 500; ++it) {
                run_adj_src(S, x->dim, x->nx, ny1, G, x->nang, x->d_hx64.p, hy, x->d_w.p, dJdI.p, lam_next.p, icdt, sig,
                            tau.p, src.p);
                adjoint_sweep_dev(x, sigt.p, src.p, lam.p, prev_tmp.p, out_tmp.p, zq.p, zinf.p, &rsc);
                run_adj_tau(S, x->dim, x->nx, ny1, G, x->nang, x->d_hx64.p, hy, sig, dE.p, ST.p, D.p, lam.p, tau.p,
                            tau_new.p, part.p, scal.p);
                double nd[2];
                read_small(x, nd, scal.p, 16);
                ++iters;
                if (!(nd[0] > 1e-30 * nd[1]) || nd[1] == 0.0) {   // |g - tau| small: keep g
                    std::swap(tau.p, tau_new.p);
                    break;
                }
                const int slot = next_slot;
                run_aa_columns(S, nn, tau.p, tau_new.p, fprev.p, gprev.p, dFr.p + (int64_t)slot * nn,
                               dGr.p + (int64_t)slot * nn, it == 0);
                if (it == 0) {   // no history yet: a plain step
                    std::swap(tau.p, tau_new.p);
                    continue;
                }
                if (nwin == AA_M) {
                    for (int c = 0; c + 1 < AA_M; ++c) win[c] = win[c + 1];
                    --nwin;
                }
                win[nwin++] = slot;
                next_slot = (slot + 1) % AA_M;
                AASlots sl{};
                for (int c = 0; c < nwin; ++c) sl.s[c] = win[c];
                run_aa_dots(S, nn, nwin, sl, dFr.p, dFr.p + (int64_t)slot * nn, fprev.p, aapart.p, aaout.p);
                double dots[2 * AA_M];
                read_small(x, dots, aaout.p, sizeof(double) * 2 * nwin);
                double b[AA_M], A[AA_M][AA_M], L[AA_M][AA_M] = {};
                for (int c = 0; c < nwin; ++c) {
                    Mg[win[c]][slot] = Mg[slot][win[c]] = dots[2 * c];
                    b[c] = dots[2 * c + 1];
                }
                double dmax = 0.0;
                for (int i = 0; i < nwin; ++i) dmax = std::max(dmax, Mg[win[i]][win[i]]);
                for (int i = 0; i < nwin; ++i)
                    for (int j = 0; j < nwin; ++j) A[i][j] = Mg[win[i]][win[j]] + (i == j ? 1e-13 * dmax : 0.0);
                bool ok = dmax > 0.0;
                for (int i = 0; i < nwin && ok; ++i)   // Cholesky A = L L^T
                    for (int j = 0; j <= i; ++j) {
                        double v = A[i][j];
                        for (int k2 = 0; k2 < j; ++k2) v -= L[i][k2] * L[j][k2];
                        if (i == j) {
                            if (!(v > 0.0)) { ok = false; break; }
                            L[i][i] = std::sqrt(v);
                        } else {
                            L[i][j] = v / L[j][j];
                        }
                    }
                if (!ok) {   // restart the history with a plain step
                    nwin = 0;
                    std::swap(tau.p, tau_new.p);
                    continue;
                }
                double y[AA_M];
                for (int i = 0; i < nwin; ++i) {
                    double v = b[i];
                    for (int k2 = 0; k2 < i; ++k2) v -= L[i][k2] * y[k2];
                    y[i] = v / L[i][i];
                }
                AACoef gm{};
                for (int i = nwin - 1; i >= 0; --i) {
                    double v = y[i];
                    for (int k2 = i + 1; k2 < nwin; ++k2) v -= L[k2][i] * gm.v[k2];
                    gm.v[i] = v / L[i][i];
                }
                run_aa_update(S, nn, nwin, sl, gm, dGr.p, tau_new.p, tau.p);
            }
            // lam consistent with the final tau, then the sensitivities of this step
            run_adj_src(S, x->dim, x->nx, ny1, G, x->nang, x->d_hx64.p, hy, x->d_w.p, dJdI.p, lam_next.p, icdt, sig,
                        tau.p, src.p);
            adjoint_sweep_dev(x, sigt.p, src.p, lam.p, prev_tmp.p, out_tmp.p, zq.p, zinf.p, &rsc);
            run_adjoint_dsig(S, x->dim, x->nx, ny1, G, x->nang, x->d_hx64.p, hy, lam.p, emis.p, psi, dsig.p);
            run_adj_cell(S, npc, nc, G, x->model, x->clip_lo, x->clip_hi, dt, dsig.p, tau.p, phi.p, emis.p, sig,
                         x->d_cvn.p, T, Tp, gs_cell.p, gcv_node.p, ST_prev.p);
            run_region_sums(S, nreg, nc, npc, x->d_region.p, gs_cell.p, gcv_node.p, gs.p, gc.p);
            std::swap(ST.p, ST_prev.p);
            std::swap(lam_next.p, lam.p);
        }
        if (objective == 1) {
            // direct dependence of J on c_v: sum over the region of w c_v T^N
            gs_cell.zero(S);
            run_mul(S, nn, wc.p, TN, gcv_node.p);
            run_region_sums(S, nreg, nc, npc, x->d_region.p, gs_cell.p, gcv_node.p, gs.p, gc.p);
        }
        d2h(grad_log_sigma0, gs.p, 8 * nreg, S);
        d2h(grad_log_cv, gc.p, 8 * nreg, S);
        SMRT_HIP(hipStreamSynchronize(S));
        *J_out = J;
        if (adjoint_iterations) *adjoint_iterations = iters;
    });
}
