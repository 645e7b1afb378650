// Internal declarations of the MI355X SM-TRT library (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/smrt.h"

namespace smrt {

constexpr int BAND_ROWS = 16;       // rows of cells per band (lanes per channel)
constexpr int CHANNELS = 4;         // (angle, group) channels per wave (64 / BAND_ROWS)
constexpr int N_XCD = 8;            // accelerator dies (XCDs), each with its own L2; workgroup b runs on XCD b mod 8
constexpr int NMOM2D = 9;           // per node per quadrant: 6 quadrant sums + 3 sigma-weighted
constexpr int PART_PER_CELL = 4 * 2;         // per cell per chunk: sum_g I and sum_g sigma_g I of 4 nodes
constexpr int SPIN_LIMIT = 1 << 20;          // bounded wait on a band trace
// bits of a sweep's error flag: which bounded wait ran out
constexpr int WAIT_START_GATE = 1;           // a band waiting for the band below to start
constexpr int WAIT_TRACE = 2;                // a row-0 lane waiting for the band below's trace
constexpr int TRACE_LAG = 8;                 // columns a band stays behind the band below
constexpr int LDS_PER_CU = 160 * 1024;       // gfx950 LDS per compute unit (bytes)

#define SMRT_HIP(call)                                                                   \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess) throw smrt::Error(SMRT_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

struct Error {
    smrt_status st;
    std::string msg;
    Error(smrt_status s, std::string m) : st(s), msg(std::move(m)) {}
};

// Chunks of a 2D sweep are ordered by quadrant: quadrant q owns chunks
// [start[q], start[q+1]).
struct ChunkRanges {
    int start[5];
};

// Device-side description of one 2D sweep (one problem).
struct Sweep2DArgs {
    int nx, ny, G, nbands, NT;       // NT = nx + BAND_ROWS - 1 steps per band
    int NW, K, R, NQC;               // waves per band (group blocks of one direction), pairs/lane, pairs/chunk, chunk count
    int n_wg;                        // workgroups of this problem (NQC * band groups)
    int NB;                          // boundary face nodes
    const int *qc_quad;              // [NQC] quadrant of each chunk
    const int2 *slot_pair;           // [NQC*R] (direction, group) or (-1,-1)
    const void *dirs;                // per direction: real[8] = mu, eta, w, w*mu, w*eta, w*mu^2, w*mu*eta, w*eta^2
    const void *hx, *hy;             // real[nx], real[ny]
    const void *sig2;                // real2 [4 quad][G][band][t][r] = (sigma_t, sigma), skewed canonical
    const void *qiso;                // real4 [4 quad][G][band][t][r], canonical node order
    const void *psi_prev;            // internal layout or nullptr
    void *psi_out;                   // internal layout
    const void *inflow;              // real [d][G][NB]
    double inv_c_dt;
    void *part;                      // real2 [NQC][nbands][NT][4 nodes][16 rows]: (sum_g I, sum_g sigma_g I)
    uint64_t *trace;                 // [NQC][nbands][slot = (wave, k, channel)][nx][2 values][words]
    int *ctr;                        // [4]: (unused), workgroups done, epoch, error flag
    const int *gate;                 // nullptr, or a flag: the problem is swept only while it is nonzero
};

// One sweep launch: one problem (args by value) or a batch of problems
// (device array), and the launch's task list.  A task is (problem, band group
// * NQC + chunk); the list is band-group-major, so a workgroup that claims a
// ticket only ever waits on tasks claimed before it by running workgroups:
// deadlock-free at any residency.
struct SweepLaunch {
    Sweep2DArgs single;              // used when probs == nullptr
    const Sweep2DArgs *probs;        // [n_probs] device array (batch) or nullptr
    const int2 *tasks;               // [n_tasks]
    int n_tasks;
    int NW, NBW, K;                  // launch shape shared by every problem: waves per band,
                                     // bands per workgroup (NW * NBW <= 16), pairs per lane
    int wg_per_cu;                   // 0: as many as fit; n: pad LDS so at most n workgroups share a CU
    int *lctr;                       // [2]: ticket, workgroups done (both reset by the last workgroup)
    int fixup;                       // 1: zero-and-scale negative-flux fixup in every cell
    int xw;                          // 1: some chunk spans several band groups (publishing and
                                     //    receiving waves in every workgroup)
    int static_order;                // 1: workgroup b sweeps tasks[b] (no workgroup waits on
                                     //    another); 0: tasks are claimed through the ticket lctr[0]
};

// Internal angular-flux layout (both precisions): [d][g][band][t][r][4 canonical nodes].
__host__ __device__ inline int64_t psi_slab(int nx, int ny) {
    int nb = (ny + BAND_ROWS - 1) / BAND_ROWS;
    return (int64_t)nb * (nx + BAND_ROWS - 1) * BAND_ROWS * 4;
}

// Per-(quadrant, group) cell tables use the same skewed band layout as the
// angular flux so that a wave's diagonal of cells is contiguous in memory.
__host__ __device__ inline int64_t cell_slab(int nx, int ny) {
    int nb = (ny + BAND_ROWS - 1) / BAND_ROWS;
    return (int64_t)nb * (nx + BAND_ROWS - 1) * BAND_ROWS;
}

template <typename real>
void launch_sweep2d(const SweepLaunch &L, hipStream_t s);

struct Sweep1DArgs {
    int nx, G, nang;
    const void *mu_w;       // real[2*nang]: mu, w
    const void *hx;
    const void *sig2;       // real2 [G][cell]
    const void *qiso;       // real [G][cell][2]
    const void *psi_prev;   // [d][g][node]
    void *psi_out;
    const void *inflow;     // [d][G][2]
    double inv_c_dt;
    int fixup;              // 1: zero-and-scale negative-flux fixup in every cell
};
template <typename real>
void launch_sweep1d(const Sweep1DArgs &a, hipStream_t s);

}  // namespace smrt
