// FP64 closure post-pass and low-order solver (lo.hip).
#pragma once
#include <algorithm>
#include <memory>
#include <string>
#include <vector>

#include "smrt_internal.h"

namespace smrt {

// Owning device buffer.
template <typename T>
struct DevBuf {
    T *p = nullptr;
    int64_t n = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { release(); }
    void alloc(int64_t count) {
        release();
        n = count;
        if (count > 0) {
            hipError_t e = hipMalloc(&p, sizeof(T) * count);
            if (e != hipSuccess) {
                p = nullptr;
                throw Error(SMRT_E_OUT_OF_MEMORY, "hipMalloc of " + std::to_string(sizeof(T) * count) + " bytes failed");
            }
        }
    }
    void zero(hipStream_t s = nullptr) {
        if (p) SMRT_HIP(hipMemsetAsync(p, 0, sizeof(T) * n, s));
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
};

struct Csr {
    int nrows = 0, ncols = 0;
    std::vector<int> rowptr, col;
    std::vector<double> val;
};

struct DevCsr {
    DevBuf<int> rp_, col_;
    DevBuf<double> val_;
    int *rp = nullptr, *col = nullptr;
    double *val = nullptr;
    int nrows = 0;
    void upload(const Csr &m) {
        nrows = m.nrows;
        rp_.alloc(m.rowptr.size());
        col_.alloc(std::max<size_t>(m.col.size(), 1));
        val_.alloc(std::max<size_t>(m.val.size(), 1));
        SMRT_HIP(hipMemcpy(rp_.p, m.rowptr.data(), sizeof(int) * m.rowptr.size(), hipMemcpyHostToDevice));
        if (!m.col.empty()) {
            SMRT_HIP(hipMemcpy(col_.p, m.col.data(), sizeof(int) * m.col.size(), hipMemcpyHostToDevice));
            SMRT_HIP(hipMemcpy(val_.p, m.val.data(), sizeof(double) * m.val.size(), hipMemcpyHostToDevice));
        }
        rp = rp_.p;
        col = col_.p;
        val = val_.p;
    }
};

struct ClosureArgs {
    int dim, nx, ny, scheme;
    double c, dt;
    const double *hx, *hy;        // cell sizes
    double alpha[2];
    double Itot[4];               // per side: sum_g inflow intensity (isotropic)
    double S1[4];                 // per side: sum_{Omega.n<0} w (Omega.n)
    double S2[8];                 // per side, component: sum_{Omega.n<0} w Omega_a (Omega.n)
    int refl;                     // bit s: side s is reflective; its F_in, P_in come from bmom
    const double *bmom;           // [NB][3] incoming moments (F_in, P_in,x, P_in,y) per boundary node
    const double *mom;            // [27|8][nn]
    const double *sigP, *sigF;    // [nn] at the outer iterate's T
    const double *Estar, *Fstar;  // [nn], [nn][dim]
    double *out;                  // [3+1+dim][nn]
    const int *gate;              // nullptr, or a device flag: no work while it is 0
};
void run_closures(hipStream_t s, const ClosureArgs &a);
void run_eliminate(hipStream_t s, int nn, double a, double c, double dt, double rtol, int maxit, double T_floor,
                   const double *cvn, const double *sigE, const double *sigP, const double *E, const double *Tstar,
                   double *T, int *flags);

void assemble_lo_operators(int dim, int nx, int ny, const std::vector<double> &xe, const std::vector<double> &ye,
                           const double alpha[2], double c, Csr &D, Csr &DT, Csr &P, std::vector<double> &wnode);

struct LoInputs {
    double dt, eps_inner, cg_rtol, elim_rtol;
    double T_floor;                               // > 0: temperature floor of the elimination
    int max_inner, max_cg, max_elim;
    int precond;                                  // 0: Jacobi; 1: aggregation multigrid V-cycle
    const double *sigE, *sigF, *sigP, *qE, *qF;   // closure rows (qF: [dim][nn])
    const double *cvn, *Tstar;
};

struct MgHierarchy;   // aggregation multigrid levels (built on first use)

// mesh of the stencil form of the LO operators
struct LoGeom {
    int dim, nx, ny;
    const double *hx, *hy;
    double c, alpha[2];
};

// Device-side control of one problem in a multi-step batched run: the outer
// iteration of the step (Algorithm 1) and the Newton and CG iterations of its
// LO solve (Sec. 5) are decided on the device from these fields.
struct RunCtl {
    int active;          // 1 while the step's outer iteration runs
    int l;               // outer iterations done in this step
    int status;          // SMRT_OK, or the failure that ended this step
    int reason;          // RUN_* code of a failure (its message on the host)
    int m;               // Newton iteration of the current LO solve
    int nt_on;           // 1 while the LO's Newton iteration runs
    int cg_on;           // 1 while the current CG runs
    int cg_par;          // the current CG scalars are in sc (0) or sc2 (1)
    int outer, inner_total, cg_total, elim_max, hit_max;   // statistics of the step
    double first;        // first outer change of the step
    double first_in;     // first Newton change of the current LO solve
};
enum { RUN_NO_ROOT = 1, RUN_LO_NONFINITE = 2, RUN_OUTER_NONFINITE = 3, RUN_SWEEP_WAIT = 4 };

// One problem of the batched LO kernel: its operators, the work vectors of its
// LoSolver, the closure inputs, the iterate and its control block.
struct LoProb {
    int nn, dim, nbk, nbkd;                  // nodes, 256-node blocks of nodes and of F rows
    LoGeom g;
    double a, c, dt, eps_inner, cg_rtol, elim_rtol, T_floor;
    int max_inner, max_cg, max_elim;
    const int *drp, *dcol, *dtrp, *dtcol, *prp, *pcol;   // D, D^T and P (CSR)
    const double *dval, *dtval, *pval, *wn;
    double *MFinv, *DqF, *jbase, *diagE, *rhs, *Minv, *r, *z, *p, *Ap, *Eold, *Told, *tmpF, *part, *sc, *bpart,
        *apart, *sc2;
    int *flags;
    const double *sigE, *sigF, *sigP, *qE, *qF, *cvn, *Tstar;
    double *E, *F, *T;
    RunCtl *ctl;
};

constexpr int LO_BATCH_MAX = 64;   // problems of one batched LO launch
constexpr int LO_BAR_WORDS = 512;  // words of the batched LO's grid barrier
// Launch arguments of the batched LO kernel: the problems and where each
// problem's node blocks start in the launch's sequence of node blocks.
struct LoBatch {
    const LoProb *P;
    int np;
    int vb_n[LO_BATCH_MAX + 1];    // prefix sums of nbk
    unsigned *bar;                 // [LO_BAR_WORDS] grid barrier: generation, top and group counters
    int *abort;                    // set when a barrier wait exceeds its bound
};
// One LO solve (Newton with nonlinear elimination, Jacobi-PCG) of every
// problem whose control block is active, in one persistent launch whose
// workgroups meet at grid barriers; the same arithmetic, block by block, as
// LoSolver::solve.  grid: workgroups that are all resident at once.
void run_lo_batch(hipStream_t s, const LoBatch &b, int grid);
int lo_batch_grid(int total_blocks);   // persistent grid for a batch of that many node blocks

struct LoSolver {
    int dim = 0, nn = 0;
    double c = 1, a = 1;
    // mesh, kept to re-assemble the geometric operators for the multigrid set-up
    int gnx = 0, gny = 0;
    std::vector<double> gxe, gye;
    double galpha[2] = {0, 0};
    std::unique_ptr<MgHierarchy> mg;
    int precond = 0;               // preconditioner of the current solve
    DevBuf<double> dhx, dhy;       // cell sizes (the stencil form of S)
    DevCsr dD, dDT, dP;
    DevBuf<double> wn, MFinv, DqF, jbase, diagE, rhs, Minv, r, z, p, Ap, Eold, Told, tmpF, part, sc, bpart, apart;
    DevBuf<double> sc2;            // second set of CG scalars (the batched LO alternates between sc and sc2)
    DevBuf<int> flags;
    // captured HIP graph of a block of CG iterations (kernels only), per (stream, x)
    hipGraph_t cg_graph = nullptr;
    hipGraphExec_t cg_exec = nullptr;
    hipStream_t cg_stream = nullptr;
    const double *cg_x = nullptr;
    int cg_precond = -1;
    bool use_graphs = true, graph_failed = false;
    LoSolver();
    ~LoSolver();
    void init_mg();
    void setup_mg(hipStream_t s);
    void vcycle(hipStream_t s, const double *r, double *z);
    void mg_cg_init(hipStream_t s);
    void mg_cg_iteration(hipStream_t s, double *x);
    void drop_graph();
    void cg_block(hipStream_t s, double *x, int iters);
    void init(int dim, int nx, int ny, const std::vector<double> &xe, const std::vector<double> &ye,
              const double alpha[2], double c, double a);
    double dot(hipStream_t s, const double *x, const double *y, const double *cdiff, int slot, bool accumulate);
    // dot(), skipped while the device flag *gate is 0
    void dot_gated(hipStream_t s, const int *gate, const double *x, const double *y, const double *cdiff, int slot,
                   bool accumulate);
    double fetch(hipStream_t s, int slot);
    void fetch_flags(hipStream_t s, int fl[4]);   // the elimination flags, through pinned memory
    void ensure_hbuf();
    void schur(hipStream_t s, const double *x, double *y);
    struct LoGeom geom() const;
    static constexpr int CG_CHECK = 4;   // CG iterations queued between host checks
    double *hbuf = nullptr;              // pinned: CG stop flag and count, elimination flags, iterate change
    void pcg_begin(hipStream_t s, double *x, double rtol, int maxit);
    void pcg_block(hipStream_t s, double *x);
    void pcg_status_async(hipStream_t s);
    smrt_status solve(hipStream_t s, const LoInputs &in, double *E, double *F, double *T, smrt_step_stats *st,
                      std::string &err);
};

}  // namespace smrt
