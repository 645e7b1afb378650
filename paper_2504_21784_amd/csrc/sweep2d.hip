// Lumped bilinear DG S_N sweep on a rectilinear 2D mesh for gfx950.
//
// What is computed (Eq. dgsn_transport with every form lumped by the
// trapezoid rule): for every (direction d, group g) and every cell, in
// upwind order, the 4x4 local system
//     A I = w (q_iso + inv_c_dt I*) + upwind face terms
// with A = dI + (a/2)Kx + (b/2)Ky in canonical (mu>0, eta>0) node order,
// a = |mu| hy/2, b = |eta| hx/2, d = (a+b)/2 + sigt hx hy/4, Kx = I(x)J,
// Ky = J(x)I, J = [[0,1],[-1,0]].  Because Kx, Ky commute and square to -I,
//     A^-1 = (dI - (a/2)Kx - (b/2)Ky)(alpha I + beta M) / (alpha^2 - beta^2)
// with alpha = d^2 + (a^2+b^2)/4, beta = ab/2, M = Kx Ky; the solve costs
// ~30 flops instead of a pivoted LU.  Fused with the solve, each lane
// accumulates the angular moments of its intensities (per quadrant:
// w{1,mu,eta,mu^2,mu eta,eta^2} I; and sigma_g w{1,mu,eta} I).
//
// Work decomposition (CDNA4, wave64):
//  * The mesh is viewed per quadrant in canonical coordinates (flipped so
//    the sweep runs +x,+y) and cut into bands of 16 rows.
//  * A wave = 4 channels x 16 rows: lane = channel*16 + row.  Each channel
//    is one (direction, group) pair (times K pairs handled in sequence by
//    the lane).  At step t the lane of row r handles column t - r, so a
//    band is a diagonal wavefront inside the wave: the x-upwind trace stays
//    in the lane's registers and the y-upwind trace moves one lane up with
//    a DPP row shift.
//  * A workgroup = NW waves on the same band of the same quadrant with
//    disjoint (direction, group) pairs; their moment contributions are
//    reduced through LDS every step (summed in FP64 in a fixed order) and
//    one partial per cell and workgroup is written.
//  * Bands hand their top-row outflow to the band above through a trace
//    buffer of 64-bit words that carry (sweep epoch, value bits), written
//    and polled with relaxed device-scope atomics: a word is valid when
//    its epoch matches, so no cache flushes are needed.  Workgroups take
//    tasks from a ticket counter in band-major order, so a workgroup only
//    ever waits on a band whose workgroup started earlier: no deadlock,
//    whatever the residency.  Every wait is bounded (SPIN_LIMIT) and sets an
//    error flag instead of hanging.
//  * Angular-flux layout [d][g][band][t][r][node]: at step t a channel's 16
//    lanes read and write 16 consecutive 4-node cells (256 B in FP32).
#include "smrt_internal.h"

namespace smrt {

template <typename real> struct vec2;
template <> struct vec2<float> { using type = float2; };
template <> struct vec2<double> { using type = double2; };

template <typename real> struct vec4;
template <> struct vec4<float> { using type = float4; };
template <> struct vec4<double> { using type = double4; };

// Trace words: FP32 value -> 1 word, FP64 value -> 2 words (lo, hi halves).
template <typename real> struct trace_words { static constexpr int n = sizeof(real) / 4; };

__device__ __forceinline__ uint64_t pack_word(uint32_t epoch, uint32_t bits) {
    return ((uint64_t)epoch << 32) | bits;
}

__device__ __forceinline__ void put_trace(uint64_t *p, float v, uint32_t ep) {
    __hip_atomic_store(p, pack_word(ep, __float_as_uint(v)), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void put_trace(uint64_t *p, double v, uint32_t ep) {
    uint64_t b = __double_as_longlong(v);
    __hip_atomic_store(p, pack_word(ep, (uint32_t)b), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(p + 1, pack_word(ep, (uint32_t)(b >> 32)), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t poll_word(const uint64_t *p) {
    return __hip_atomic_load(const_cast<uint64_t *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ float word_value(const uint64_t *w, float) { return __uint_as_float((uint32_t)w[0]); }
__device__ __forceinline__ double word_value(const uint64_t *w, double) {
    return __longlong_as_double((long long)(((uint64_t)(uint32_t)w[1] << 32) | (uint32_t)w[0]));
}

template <typename real>
__device__ __forceinline__ real shift_up_one_row(real v);   // lane r <- lane r-1 within 16-lane rows

template <>
__device__ __forceinline__ float shift_up_one_row<float>(float v) {
    // DPP row_shr:1 (0x111); lane 0 of every row keeps 0 (bound_ctrl).
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x111, 0xf, 0xf, true));
}
template <>
__device__ __forceinline__ double shift_up_one_row<double>(double v) {
    long long b = __builtin_bit_cast(long long, v);
    int lo = __builtin_amdgcn_update_dpp(0, (int)b, 0x111, 0xf, 0xf, true);
    int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x111, 0xf, 0xf, true);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}

template <typename real, int K>
struct StepIn {
    // raw loaded values only: any reordering happens at use, so the loads of
    // several steps can stay in flight
    real psi[K][4];     // I* (canonical node order)
    real qn[K][4];      // q_iso (canonical node order)
    real st[K], sg[K];  // sigma_t, sigma
    real bot[K][2];     // y- boundary inflow for canonical nodes 0, 1 (band 0)
    uint64_t tw[K][2 * trace_words<real>::n];   // band trace words (band > 0)
    real hx;
};

template <typename real, int K, int PF>
__global__ void __launch_bounds__(MAX_WG_THREADS) sweep2d_kernel(Sweep2DArgs A) {
    using r2 = typename vec2<real>::type;
    using r4 = typename vec4<real>::type;
    constexpr int TW = trace_words<real>::n;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    real *red = reinterpret_cast<real *>(smem_raw);
    __shared__ int s_task, s_epoch;

    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int ch = lane >> 4;
    const int r = lane & 15;
    const int nthr = A.NW * 64;
    const int red_stride = nthr + 1;

    if (threadIdx.x == 0) {
        s_task = atomicAdd(&A.ctr[0], 1);
        s_epoch = __hip_atomic_load(&A.ctr[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    const int task = s_task;
    const uint32_t epoch = (uint32_t)s_epoch;
    const int band = task / A.NQC;
    const int qc = task - band * A.NQC;
    const int quad = A.qc_quad[qc];
    const bool fx = (quad == 1 || quad == 2);
    const bool fy = (quad == 2 || quad == 3);
    const int nx = A.nx, ny = A.ny, G = A.G, NT = A.NT, nbands = A.nbands;
    const int jc = band * BAND_ROWS + r;
    const bool row_ok = jc < ny;
    const int jn = fy ? ny - 1 - jc : jc;

    const real *dirs = static_cast<const real *>(A.dirs);
    const real *hxa = static_cast<const real *>(A.hx);
    const real *hya = static_cast<const real *>(A.hy);
    const r2 *sig2 = static_cast<const r2 *>(A.sig2);
    const r4 *qiso = static_cast<const r4 *>(A.qiso);
    const r4 *pprev = static_cast<const r4 *>(A.psi_prev);
    r4 *pout = static_cast<r4 *>(A.psi_out);
    const real *inflow = static_cast<const real *>(A.inflow);

    int dd[K], gg[K];
    bool act[K];
    real am[K], bm[K];            // |mu|, |eta|
    real cw[K][6];                // w*{1, mu, eta, mu^2, mu eta, eta^2}
    int64_t slab[K];              // offset of this (d,g) band slab in units of cells
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int slot = (wv * CHANNELS + ch) * K + k;
        const int2 pg = A.slot_pair[qc * A.R + slot];
        dd[k] = pg.x < 0 ? 0 : pg.x;      // inactive slots (-1) address direction 0
        gg[k] = pg.y < 0 ? 0 : pg.y;
        act[k] = pg.x >= 0 && row_ok;
        const int d = pg.x < 0 ? 0 : pg.x;
        const real *dr = dirs + 8 * d;
        am[k] = fabs(dr[0]);
        bm[k] = fabs(dr[1]);
#pragma unroll
        for (int m = 0; m < 6; ++m) cw[k][m] = dr[2 + m];
        slab[k] = (((int64_t)d * G + gg[k]) * nbands + band) * NT * BAND_ROWS;
    }
    const real hy = row_ok ? hya[jn] : real(1);
    const int64_t tslab = (int64_t)nbands * NT * BAND_ROWS;   // cells per (quadrant, group) table slab
    const real icdt = (real)A.inv_c_dt;

    // boundary side bases in the general inflow array [d][g][NB]
    const int xside = fx ? 2 * ny : 0;                 // canonical x- side
    const int yside = 4 * ny + (fy ? 2 * nx : 0);      // canonical y- side
    const int traces_per_band = A.R * nx * 2 * TW;
    uint64_t *trace_in = A.trace + ((int64_t)qc * nbands + (band > 0 ? band - 1 : 0)) * traces_per_band;
    uint64_t *trace_out = A.trace + ((int64_t)qc * nbands + band) * traces_per_band;
    const bool produce = (r == BAND_ROWS - 1) && (band + 1 < nbands);
    const bool consume = (r == 0) && (band > 0);

    // All prefetch loads are issued unconditionally from clamped (always
    // valid) addresses into raw registers, so several steps of loads stay in
    // flight: a load under a branch, or a reordering of its result, makes the
    // compiler wait for every outstanding memory operation.
    // psi_prev may be absent (raw sweep without a time-edge source): loads then
    // read psi_out (valid memory) and the values are discarded at use.
    const bool has_prev = pprev != nullptr;
    const r4 *pp_eff = has_prev ? pprev : pout;
    auto load_step = [&](int t, StepIn<real, K> &S) {
        const int ic = t - r;
        const bool col_ok = ic >= 0 && ic < nx;
        const int icc = col_ok ? ic : 0;
        const int in = fx ? nx - 1 - icc : icc;
        S.hx = hxa[in];
        // band trace words first (band > 0, row 0): issued before the other loads.
        // Every lane of a channel reads the word its row-0 lane needs (column t),
        // so a wave touches one address per channel and no word is contended.
        const int tcol = t < nx ? t : nx - 1;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const uint64_t *src = trace_in + (((int64_t)(wv * CHANNELS + ch) * K + k) * nx + tcol) * 2 * TW;
#pragma unroll
            for (int u = 0; u < 2 * TW; ++u) S.tw[k][u] = poll_word(src + u);
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const bool ok = act[k] && col_ok;
            // (quadrant, group) tables in the skewed layout: contiguous per channel
            const int64_t ti = ((int64_t)quad * G + gg[k]) * tslab + ((int64_t)band * NT + t) * BAND_ROWS + r;
            const r2 s = sig2[ti];
            S.st[k] = s.x;
            S.sg[k] = s.y;
            const r4 qn = qiso[ti];
            S.qn[k][0] = qn.x; S.qn[k][1] = qn.y; S.qn[k][2] = qn.z; S.qn[k][3] = qn.w;
            const r4 p = pp_eff[ok ? slab[k] + (int64_t)t * BAND_ROWS + r : 0];
            S.psi[k][0] = p.x; S.psi[k][1] = p.y; S.psi[k][2] = p.z; S.psi[k][3] = p.w;
            // y- boundary inflow (band 0, row 0) -- other lanes read one shared valid word
            const int64_t ib = ((int64_t)dd[k] * G + gg[k]) * A.NB;
            const int bnd = (band == 0 && r == 0 && ok) ? 1 : 0;
            const int lx0 = fx ? 1 : 0;
            const int64_t bbase = ib + yside + bnd * (2 * in);   // always a valid index
            S.bot[k][0] = inflow[bbase + bnd * lx0];
            S.bot[k][1] = inflow[bbase + bnd * (1 - lx0)];
        }
    };

    real xl[K][2], yb[K][2];   // x-upwind (nodes 1,3 of the left cell), y-upwind (nodes 2,3 of the cell below)
    real left[K][2];           // canonical x- boundary inflow of this row (nodes 0, 2)
#pragma unroll
    for (int k = 0; k < K; ++k) {
        xl[k][0] = xl[k][1] = yb[k][0] = yb[k][1] = 0;
        const int64_t ib = ((int64_t)dd[k] * G + gg[k]) * A.NB;
        const int ly0 = fy ? 1 : 0;
        const int jv = row_ok ? jn : 0;
        left[k][0] = inflow[ib + xside + 2 * jv + ly0];
        left[k][1] = inflow[ib + xside + 2 * jv + (1 - ly0)];
    }
    StepIn<real, K> buf[PF + 1];
#pragma unroll
    for (int u = 0; u <= PF; ++u)
        if (u < NT) load_step(u, buf[u]);
    // One full wait after the prologue: the loop then starts from a state with
    // no pending loads, so the per-step waits only cover the slot being used.
    __builtin_amdgcn_s_waitcnt(0);
    int err = 0;

    // Start gate: a band begins only once the band below has published the
    // trace of column TRACE_LAG, so that in steady state each prefetched
    // trace word was written several steps before it is needed.
    if (band > 0) {
        const int gcol = TRACE_LAG < nx - 1 ? TRACE_LAG : nx - 1;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const uint64_t *g = trace_in + (((int64_t)(wv * CHANNELS + ch) * K + k) * nx + gcol) * 2 * TW;
            bool waiting = (r == 0) && act[k];
            int spins = 0;
            while (waiting) {
                bool rd = true;
#pragma unroll
                for (int u2 = 0; u2 < 2 * TW; ++u2) rd &= (uint32_t)(poll_word(g + u2) >> 32) == epoch;
                if (rd) break;
                if (++spins > SPIN_LIMIT ||
                    __hip_atomic_load(&A.ctr[3], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                    err = 1;
                    atomicOr(&A.ctr[3], 1);
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
        }
    }

    for (int t0 = 0; t0 < NT; t0 += PF + 1) {
#pragma unroll
        for (int u = 0; u <= PF; ++u) {
            const int t = t0 + u;
            if (t < NT) {
                StepIn<real, K> &S = buf[u];
                const int ic = t - r;
                const bool col_ok = ic >= 0 && ic < nx;
                const real hx = S.hx;
                const real wgt = hx * hy * real(0.25);
                real acc[PART_PER_CELL];
#pragma unroll
                for (int m = 0; m < PART_PER_CELL; ++m) acc[m] = 0;
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const bool ok = act[k] && col_ok;
                    // y-upwind values: from the lane below (already shifted), the band
                    // below (trace words) or the boundary.
                    real yin0 = yb[k][0], yin1 = yb[k][1];
                    if (r == 0 && band == 0) {
                        yin0 = S.bot[k][0];
                        yin1 = S.bot[k][1];
                    } else if (r == 0) {
                        uint64_t *tw = S.tw[k];
                        bool ready = true;
#pragma unroll
                        for (int u2 = 0; u2 < 2 * TW; ++u2) ready &= (uint32_t)(tw[u2] >> 32) == epoch;
                        const bool wait_here = ok && !ready && !err;
                        if (__builtin_amdgcn_ballot_w64(wait_here) != 0) {   // rare: trace not yet valid
                            const uint64_t *src = trace_in + (((int64_t)(wv * CHANNELS + ch) * K + k) * nx + (ok ? ic : 0)) * 2 * TW;
                            int spins = 0;
                            bool waiting = wait_here;
                            while (waiting) {
                                // bounded wait; a timed-out wave raises ctr[3] and every other
                                // waiter gives up at once
                                if (++spins > SPIN_LIMIT ||
                                    __hip_atomic_load(&A.ctr[3], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                                    err = 1;
                                    atomicOr(&A.ctr[3], 1);
                                    break;
                                }
                                __builtin_amdgcn_s_sleep(1);
                                bool rd = true;
#pragma unroll
                                for (int u2 = 0; u2 < 2 * TW; ++u2) {
                                    tw[u2] = poll_word(src + u2);
                                    rd &= (uint32_t)(tw[u2] >> 32) == epoch;
                                }
                                waiting = !rd;
                            }
                        }
                        if (ok) {
                            yin0 = word_value(tw, real(0));
                            yin1 = word_value(tw + TW, real(0));
                        }
                    }
                    const real xin0 = (ic == 0) ? left[k][0] : xl[k][0];
                    const real xin2 = (ic == 0) ? left[k][1] : xl[k][1];
                    const real a = am[k] * hy * real(0.5);
                    const real b = bm[k] * hx * real(0.5);
                    const real q0 = S.qn[k][0], q1 = S.qn[k][1], q2 = S.qn[k][2], q3 = S.qn[k][3];
                    const real ps0 = has_prev ? S.psi[k][0] : real(0), ps1 = has_prev ? S.psi[k][1] : real(0);
                    const real ps2 = has_prev ? S.psi[k][2] : real(0), ps3 = has_prev ? S.psi[k][3] : real(0);
                    real rh0 = wgt * (q0 + icdt * ps0) + a * xin0 + b * yin0;
                    real rh1 = wgt * (q1 + icdt * ps1) + b * yin1;
                    real rh2 = wgt * (q2 + icdt * ps2) + a * xin2;
                    real rh3 = wgt * (q3 + icdt * ps3);
                    const real dg = real(0.5) * (a + b) + S.st[k] * wgt;
                    const real ha = real(0.5) * a, hb = real(0.5) * b;
                    const real y0 = dg * rh0 - ha * rh1 - hb * rh2;
                    const real y1 = dg * rh1 + ha * rh0 - hb * rh3;
                    const real y2 = dg * rh2 - ha * rh3 + hb * rh0;
                    const real y3 = dg * rh3 + ha * rh2 + hb * rh1;
                    const real al = dg * dg + ha * ha + hb * hb;
                    const real be = real(2) * ha * hb;
                    const real inv = real(1) / (al * al - be * be);
                    const real ai = al * inv, bi = be * inv;
                    const real I0 = ai * y0 + bi * y3;
                    const real I1 = ai * y1 - bi * y2;
                    const real I2 = ai * y2 - bi * y1;
                    const real I3 = ai * y3 + bi * y0;
                    if (ok) {
                        r4 o;
                        o.x = I0; o.y = I1; o.z = I2; o.w = I3;
                        pout[slab[k] + (int64_t)t * BAND_ROWS + r] = o;
                        if (produce) {
                            uint64_t *dst = trace_out + (((int64_t)(wv * CHANNELS + ch) * K + k) * nx + ic) * 2 * TW;
                            put_trace(dst, I2, epoch);
                            put_trace(dst + TW, I3, epoch);
                        }
                        const real Iv[4] = {I0, I1, I2, I3};
#pragma unroll
                        for (int l = 0; l < 4; ++l) {
                            const real v = Iv[l];
                            real *m = acc + l * NMOM2D;
#pragma unroll
                            for (int j = 0; j < 6; ++j) m[j] += cw[k][j] * v;
                            const real sv = S.sg[k] * v;
                            m[6] += cw[k][0] * sv;
                            m[7] += cw[k][1] * sv;
                            m[8] += cw[k][2] * sv;
                        }
                    }
                    xl[k][0] = I1;
                    xl[k][1] = I3;
                    yb[k][0] = shift_up_one_row<real>(I2);
                    yb[k][1] = shift_up_one_row<real>(I3);
                }
                // prefetch the step PF+1 ahead into the slot just consumed
                if (t + PF + 1 < NT) load_step(t + PF + 1, buf[u]);

                // workgroup reduction of the moment contributions of this step
#pragma unroll
                for (int m = 0; m < PART_PER_CELL; ++m) red[m * red_stride + threadIdx.x] = acc[m];
                __syncthreads();
                real *part = static_cast<real *>(A.part) + (((int64_t)qc * nbands + band) * NT + t) * (BAND_ROWS * PART_PER_CELL);
                for (int o = threadIdx.x; o < BAND_ROWS * PART_PER_CELL; o += nthr) {
                    const int rr = o / PART_PER_CELL;
                    const int m = o - rr * PART_PER_CELL;
                    const int icc = t - rr;
                    if (icc >= 0 && icc < nx && band * BAND_ROWS + rr < ny) {
                        double s = 0.0;
                        const real *src = red + m * red_stride + rr;
                        for (int w2 = 0; w2 < A.NW; ++w2)
#pragma unroll
                            for (int c2 = 0; c2 < CHANNELS; ++c2) s += (double)src[w2 * 64 + c2 * BAND_ROWS];
                        part[o] = (real)s;
                    }
                }
                __syncthreads();
            }
        }
    }

    // the last workgroup to finish resets the ticket counters and advances the epoch
    __syncthreads();
    if (threadIdx.x == 0) {
        const int done = atomicAdd(&A.ctr[1], 1);
        if (done == A.n_wg - 1) {
            __hip_atomic_store(&A.ctr[0], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&A.ctr[1], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(&A.ctr[2], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

template <typename real, int K>
static void launch_k(const Sweep2DArgs &a, hipStream_t s) {
    constexpr int PF = sizeof(real) == 4 ? 2 : 1;
    const size_t lds = (size_t)PART_PER_CELL * (a.NW * 64 + 1) * sizeof(real);
    SMRT_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&sweep2d_kernel<real, K, PF>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL((sweep2d_kernel<real, K, PF>), dim3(a.n_wg), dim3(a.NW * 64), lds, s, a);
}

template <typename real>
void launch_sweep2d(const Sweep2DArgs &a, hipStream_t s) {
    if (a.K == 1) { launch_k<real, 1>(a, s); SMRT_HIP(hipGetLastError()); return; }
    if constexpr (sizeof(real) == 4) {
        if (a.K == 2) { launch_k<real, 2>(a, s); SMRT_HIP(hipGetLastError()); return; }
    }
    throw Error(SMRT_E_INVALID_ARG, "pairs per lane must be 1 (FP64) or 1, 2 (FP32)");
}

template void launch_sweep2d<float>(const Sweep2DArgs &, hipStream_t);
template void launch_sweep2d<double>(const Sweep2DArgs &, hipStream_t);

}  // namespace smrt
