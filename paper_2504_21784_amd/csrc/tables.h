// Host launchers of the table, conversion and 1D kernels (tables.hip).
#pragma once
#include "smrt_internal.h"

namespace smrt {

// A launcher's gate (nullptr: always) is a device flag: while it is 0 the
// kernels return at once (a converged problem of a multi-step batched run).

constexpr int NBERN = 24;   // Bernoulli terms of the small-argument Planck series
constexpr int MAXG = 64;    // largest group count

// computes the small-argument Planck series coefficients and uploads them to
// the current device (every entry point that creates device state calls it)
void upload_series_coefficients();
template <typename real>
void run_opacity(hipStream_t s, int ncell, int npc, int G, const double *T, const int *region, int model,
                 const double *sigma0, double lo, double hi, const double *nu, double icdt, double *sig, real *sig2);
template <typename real>
void run_source(hipStream_t s, int nn, int npc, int G, const double *T, const double *nu, double a, double c,
                const double *sig, real *qiso, real *qnat, double *sigP, double *sigF,
                const int *gate = nullptr);
template <typename real>
void run_stab2d(hipStream_t s, int nx, int ny, int G, const double *sig, const double *sigt, double icdt, real *stab);
// 2D: opacity sigma[cell][G] and its skewed per-quadrant (sigma_t, sigma) tables in one pass
template <typename real>
void run_opacity_tab2d(hipStream_t s, int nx, int ny, int G, const double *T, const int *region, int model,
                       const double *sigma0, double lo, double hi, const double *nu, double icdt, double *sig,
                       real *stab);
template <typename real, typename src_t>
void run_qtab2d(hipStream_t s, int nx, int ny, int G, const src_t *q, int64_t sn, int64_t sg, real *qtab,
                const int *gate = nullptr);
void run_equilibrium(hipStream_t s, int nn, int G, int nang, const double *T, const double *nu, double a, double c,
                     double *psi);
void run_side_inflow(hipStream_t s, int nsides, int G, const double *nu, double a, double c, const int *kind,
                     const double *Tb, const double *explicit_g, double *val);
template <typename real>
void run_fill_inflow(hipStream_t s, int dim, int nx, int ny, int G, int nang, const double *val, real *inflow);
// reflective sides (bit s of refl): inflow [d][g][NB] from the mirrored
// directions of psi (2D internal layout, 1D [d][g][node]) and the incoming
// moments bmom [NB][3] of the result (nothing when refl == 0)
template <typename real>
void run_reflect(hipStream_t s, int dim, int nx, int ny, int G, int nang, int refl, const int *mirror, const double *om,
                 const double *w, const int *dir_quad, const real *psi, real *inflow, double *bmom);
template <typename real>
void run_copy_to(hipStream_t s, int64_t n, const double *src, real *dst);
template <typename real>
void run_copy_from(hipStream_t s, int64_t n, const real *src, double *dst);
void run_adj_prep(hipStream_t s, int nn, int npc, int G, int nang, const double *nu, double a, double c, double dt,
                  const double *T, const double *sig, const double *cvn, const double *w, const double *psi, double *emis,
                  double *dE, double *D, double *phi);
void run_adj_dJdI(hipStream_t s, int dim, int nx, int ny, int G, int nang, const double *om, const double *w,
                  const double *hy, double dt, double *out);
void run_adj_src(hipStream_t s, int dim, int nx, int ny, int G, int nang, const double *hx, const double *hy,
                 const double *wang, const double *dJdI, const double *lam_next, double icdt, const double *sig,
                 const double *tau, double *src);
// part: scratch of 2 * ceil(nodes / 256) doubles; out2: [|tau_new - tau|^2, |tau_new|^2]
void run_adj_tau(hipStream_t s, int dim, int nx, int ny, int G, int nang, const double *hx, const double *hy,
                 const double *sig, const double *dE, const double *ST, const double *D, const double *lam,
                 const double *tau, double *tau_new, double *part, double *out2);
void run_adj_cell(hipStream_t s, int npc, int ncell, int G, int model, double clip_lo, double clip_hi, double dt,
                  const double *dsig, const double *tau, const double *phi, const double *emis, const double *sig,
                  const double *cvn, const double *T, const double *Tp, double *gs_cell, double *gcv_node,
                  double *ST_prev);
void run_region_sums(hipStream_t s, int nreg, int ncell, int npc, const int *region, const double *gs_cell,
                     const double *gcv_node, double *grad_s0, double *grad_cv);
// wc[n] = (lumped nodal weight) c_v,n; out = a * b elementwise
void run_adj_energy_weights(hipStream_t s, int dim, int nx, int npc, int nn, const double *hx, const double *hy,
                            const double *cvn, double *wc);
void run_mul(hipStream_t s, int64_t n, const double *a, const double *b, double *out);
// Anderson acceleration of the adjoint temperature iteration: history columns
// (ring of AA_MAX slots of nn doubles), their dot products, the update.
constexpr int AA_MAX = 8;
struct AASlots { int s[AA_MAX]; };
struct AACoef { double v[AA_MAX]; };
void run_aa_columns(hipStream_t s, int nn, const double *tau, const double *g, double *fprev, double *gprev,
                    double *dF, double *dG, bool first);
// out[2c] = <col_c, a>, out[2c+1] = <col_c, b>; part: scratch of 2 * ncols * ceil(nn / 256) doubles
void run_aa_dots(hipStream_t s, int nn, int ncols, const AASlots &sl, const double *cols, const double *a,
                 const double *b, double *part, double *out);
void run_aa_update(hipStream_t s, int nn, int ncols, const AASlots &sl, const AACoef &gm, const double *dG,
                   const double *g, double *tau);
// part256: scratch of 256 doubles
void run_dot(hipStream_t s, int64_t n, const double *a, const double *b, double *part256, double *out);
void run_add_scalar(hipStream_t s, int64_t n, const double *a, double v, double *out);
void run_permute_dirs(hipStream_t s, int nang, int64_t per, const int *map, const double *in, double *out);
void run_adjoint_dsig(hipStream_t s, int dim, int nx, int ny, int G, int nang, const double *hx, const double *hy,
                      const double *lam, const double *emis, const double *psi, double *dsig);
template <typename real>
void run_qiso_to_internal(hipStream_t s, int nn, int G, int npc, const double *q, real *qi);
template <typename real>
void run_sig_to_internal(hipStream_t s, int ncell, int G, const double *st, const double *sg, real *sig2);
template <typename real>
void run_psi_to_internal(hipStream_t s, int nx, int ny, int G, int nang, const int *dq, const double *abi, real *in);
template <typename real>
void run_psi_from_internal(hipStream_t s, int nx, int ny, int G, int nang, const int *dq, const real *in, double *abi);
template <typename real>
// sigq: scratch of 12 * n_nodes doubles (per-quadrant sigma-weighted moments)
// qc_dir: direction of each chunk; dirs: FP64 per-direction table (mu, eta, w, w mu, w eta, w mu^2, w mu eta, w eta^2)
void run_moments_finalize(hipStream_t s, int nx, int ny, const ChunkRanges &cr, const int *qc_dir, const double *dirs,
                          const real *part, double *sigq, double *mom,
                          const int *gate = nullptr);
template <typename real>
void run_moments1d(hipStream_t s, int nx, int G, int nang, const real *mw, const double *sig, const real *psi, double *mom);
void run_psi_EF(hipStream_t s, int nn, int dim, int G, int nang, const double *om, const double *w, double c,
                const double *psi, double *E, double *F);

}  // namespace smrt
