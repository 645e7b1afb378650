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
//  * A wave = one direction and 4 channels x 16 rows: lane = channel*16 +
//    row; channel c handles groups c, c+4, .. (K groups per lane, in
//    sequence).  At step t the lane of row r handles column t - r, so a band
//    is a diagonal wavefront inside the wave: the x-upwind trace stays in the
//    lane's registers and the y-upwind trace moves one lane up with a DPP
//    row shift.
//  * Moments: because the direction is uniform across the wave, its
//    contribution to every moment of a node is (wave-uniform coefficient) x
//    (sum over the wave's groups of I) or x (sum of sigma_g I).  Each lane
//    accumulates these two sums (4 nodes each), three gfx950 permlane swaps
//    reduce-scatter them over the 4 channels so that channel c holds node c's
//    totals, and channel c forms the 9 moments of canonical node c.  A
//    workgroup = NW waves = NW directions of one quadrant on the same band
//    and the same 4K groups; their 9-value
//    contributions are reduced through double-buffered LDS every step
//    (summed at the sweep precision in a fixed order, one barrier per step)
//    into one partial per cell and workgroup; partials are summed in FP64
//    by the finalisation kernels.
//  * Bands hand their top-row outflow to the band above through a trace
//    buffer of 64-bit words that carry (sweep epoch, value bits), written
//    with single 64-bit device-coherent stores (the form a relaxed
//    device-scope atomic store takes) and read with device-coherent loads:
//    a word is valid when its epoch matches, so no cache flushes are needed.  Workgroups take
//    tasks (problem, band, chunk) from a ticket counter over a task list in
//    which every band follows the band below it, so a workgroup only ever
//    waits on a band whose workgroup started earlier: no deadlock, whatever
//    the residency.  One launch may sweep many problems (a batch): each
//    problem keeps its own epoch, done counter and error flag.  Every wait
//    is bounded (SPIN_LIMIT) and sets an error flag instead of hanging.
//  * Angular-flux layout [d][g][band][t][r][node]: at step t a channel's 16
//    lanes read and write 16 consecutive 4-node cells (256 B in FP32).
//  * Optional zero-and-scale negative-flux fixup (Sec. 6, after Hamilton et
//    al.), compiled in only when asked for: a cell solution with a negative
//    entry is replaced before it is stored, traced or summed into moments.
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

// Buffer-resource access: a wave-uniform base (SGPRs) + a per-lane 32-bit
// byte offset fixed for the whole band + a wave-uniform per-step byte offset,
// so a step's loads and stores need no per-lane address arithmetic.  A lane
// with no work (a slot past the group or direction count, a row past the
// mesh) gets the per-lane offset OOB, at or past every resource's size: the
// hardware's range check for raw buffers then returns zeros to its loads and
// drops its stores, so the step needs no per-lane masking.  Every other
// access stays inside its resource.
using rsrc_t = __amdgpu_buffer_rsrc_t;
constexpr int RSRC_DWORD3 = 0x00020000;   // gfx9-family raw buffer, 32-bit data format
constexpr int CPOL_SC1 = 16;              // coherent at device scope (trace words)
constexpr uint32_t OOB = 0x80000000u;     // resources are smaller than 2^31 bytes (checked by the host)
__device__ __forceinline__ rsrc_t make_rsrc(const void *base, uint64_t bytes) {
    // base and size are wave-uniform by construction; say so, so the resource
    // lives in scalar registers (a divergent resource would need a waterfall loop)
    const uint64_t b = (uint64_t)base;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)b), hi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
    const int n = __builtin_amdgcn_readfirstlane((int)(bytes < 0xffffffffull ? bytes : 0xffffffffull));
    return __builtin_amdgcn_make_buffer_rsrc((void *)(((uint64_t)hi << 32) | lo), 0, n, RSRC_DWORD3);
}
__device__ __forceinline__ void bload(float2 &v, rsrc_t r, uint32_t vo, uint32_t so) {
    v = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 0));
}
__device__ __forceinline__ void bload(float4 &v, rsrc_t r, uint32_t vo, uint32_t so) {
    v = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(r, vo, so, 0));
}
__device__ __forceinline__ void bload(double2 &v, rsrc_t r, uint32_t vo, uint32_t so) {
    v = __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, vo, so, 0));
}
__device__ __forceinline__ void bload(double4 &v, rsrc_t r, uint32_t vo, uint32_t so) {
    const double2 a = __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, vo, so, 0));
    const double2 b = __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, vo, so + 16, 0));
    v.x = a.x; v.y = a.y; v.z = b.x; v.w = b.y;
}
__device__ __forceinline__ void bstore(const float4 &v, rsrc_t r, uint32_t vo, uint32_t so) {
    using u4 = __attribute__((ext_vector_type(4))) unsigned int;
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4, v), r, vo, so, 0);
}
__device__ __forceinline__ void bstore(const double4 &v, rsrc_t r, uint32_t vo, uint32_t so) {
    using u4 = __attribute__((ext_vector_type(4))) unsigned int;
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4, make_double2(v.x, v.y)), r, vo, so, 0);
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4, make_double2(v.z, v.w)), r, vo, so + 16, 0);
}
// trace words (device-coherent loads; the bounded spin path re-polls atomically)
// A trace word holds (epoch, value bits) and is written with one 64-bit
// device-coherent store, the form a relaxed device-scope atomic store takes.
__device__ __forceinline__ void bstore_word(uint64_t w, rsrc_t r, uint32_t vo, uint32_t so) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned int, w), r, vo,
                                          so, CPOL_SC1);
}
__device__ __forceinline__ void put_trace_words(float v, uint32_t ep, rsrc_t r, uint32_t vo, uint32_t so) {
    bstore_word(pack_word(ep, __float_as_uint(v)), r, vo, so);
}
__device__ __forceinline__ void put_trace_words(double v, uint32_t ep, rsrc_t r, uint32_t vo, uint32_t so) {
    const uint64_t b = __double_as_longlong(v);
    bstore_word(pack_word(ep, (uint32_t)b), r, vo, so);
    bstore_word(pack_word(ep, (uint32_t)(b >> 32)), r, vo, so + 8);
}
__device__ __forceinline__ void bload_words(uint64_t *w, int n, rsrc_t r, uint32_t vo, uint32_t so) {
    if (n == 2) {
        const auto a = __builtin_amdgcn_raw_buffer_load_b128(r, vo, so, CPOL_SC1);
        w[0] = ((uint64_t)a[1] << 32) | a[0];
        w[1] = ((uint64_t)a[3] << 32) | a[2];
    } else {
        const auto a = __builtin_amdgcn_raw_buffer_load_b128(r, vo, so, CPOL_SC1);
        const auto b = __builtin_amdgcn_raw_buffer_load_b128(r, vo, so + 16, CPOL_SC1);
        w[0] = ((uint64_t)a[1] << 32) | a[0];
        w[1] = ((uint64_t)a[3] << 32) | a[2];
        w[2] = ((uint64_t)b[1] << 32) | b[0];
        w[3] = ((uint64_t)b[3] << 32) | b[2];
    }
}
// two adjacent boundary values
__device__ __forceinline__ void bload_pair(float &a, float &b, rsrc_t r, uint32_t vo, uint32_t so) {
    const float2 v = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 0));
    a = v.x; b = v.y;
}
__device__ __forceinline__ void bload_pair(double &a, double &b, rsrc_t r, uint32_t vo, uint32_t so) {
    const double2 v = __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, vo, so, 0));
    a = v.x; b = v.y;
}

// A batch problem's arguments, read from the device array and made
// wave-uniform dword by dword so they live in scalar registers.
__device__ __forceinline__ Sweep2DArgs load_uniform_args(const Sweep2DArgs *p) {
    constexpr int N = sizeof(Sweep2DArgs) / 4;
    static_assert(sizeof(Sweep2DArgs) % 4 == 0, "argument block must be dword-sized");
    int w[N];
    __builtin_memcpy(w, p, sizeof(Sweep2DArgs));
#pragma unroll
    for (int i = 0; i < N; ++i) w[i] = __builtin_amdgcn_readfirstlane(w[i]);
    Sweep2DArgs a;
    __builtin_memcpy(&a, w, sizeof(Sweep2DArgs));
    return a;
}

template <typename real, int K>
struct StepIn {
    // raw loaded values only: any reordering happens at use, so the loads of
    // several steps can stay in flight
    real psi[K][4];     // I* (canonical node order)
    real qn[K][4];      // q_iso (canonical node order)
    real st[K], sg[K];  // sigma_t, sigma
    real bot[K][2];     // y- boundary inflow at natural nodes (2 in, 2 in + 1) of row 0's column (band 0)
    uint64_t tw[K][2 * trace_words<real>::n];   // band trace words (band > 0)
    real hx0;           // width of row 0's column (other rows take it from the row above)
};

// reciprocal: the hardware's 1-ulp v_rcp_f32 in FP32, a correctly rounded
// division in FP64
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }

// Reduce-scatter over the 4 channels (rows of 16 lanes) of a wave: given each
// lane's values v[0..3] (one per canonical node), every lane of channel c gets
// the sum over the 4 channels of v[c].  gfx950 permlane swaps: the 32-lane swap
// exchanges the upper half of its first operand with the lower half of its
// second, the 16-lane swap the odd rows of its first operand with the even rows
// of its second; in both cases the two results sum to the wanted partial.
__device__ __forceinline__ uint2 swap32(uint32_t a, uint32_t b) {
    const auto r = __builtin_amdgcn_permlane32_swap(a, b, false, false);
    return make_uint2(r[0], r[1]);
}
__device__ __forceinline__ uint2 swap16(uint32_t a, uint32_t b) {
    const auto r = __builtin_amdgcn_permlane16_swap(a, b, false, false);
    return make_uint2(r[0], r[1]);
}
__device__ __forceinline__ float sum_swapped32(float a, float b) {
    const uint2 r = swap32(__float_as_uint(a), __float_as_uint(b));
    return __uint_as_float(r.x) + __uint_as_float(r.y);
}
__device__ __forceinline__ float sum_swapped16(float a, float b) {
    const uint2 r = swap16(__float_as_uint(a), __float_as_uint(b));
    return __uint_as_float(r.x) + __uint_as_float(r.y);
}
__device__ __forceinline__ double sum_swapped32(double a, double b) {
    const uint64_t ua = __double_as_longlong(a), ub = __double_as_longlong(b);
    const uint2 lo = swap32((uint32_t)ua, (uint32_t)ub), hi = swap32((uint32_t)(ua >> 32), (uint32_t)(ub >> 32));
    return __longlong_as_double(((uint64_t)hi.x << 32) | lo.x) + __longlong_as_double(((uint64_t)hi.y << 32) | lo.y);
}
__device__ __forceinline__ double sum_swapped16(double a, double b) {
    const uint64_t ua = __double_as_longlong(a), ub = __double_as_longlong(b);
    const uint2 lo = swap16((uint32_t)ua, (uint32_t)ub), hi = swap16((uint32_t)(ua >> 32), (uint32_t)(ub >> 32));
    return __longlong_as_double(((uint64_t)hi.x << 32) | lo.x) + __longlong_as_double(((uint64_t)hi.y << 32) | lo.y);
}
template <typename real>
__device__ __forceinline__ real channel_scatter_sum(const real (&v)[4]) {
    // lower half keeps nodes 0,1 and upper half nodes 2,3 ...
    const real h0 = sum_swapped32(v[0], v[2]);
    const real h1 = sum_swapped32(v[1], v[3]);
    // ... then even channels keep their even node, odd channels their odd node
    return sum_swapped16(h0, h1);
}

// Zero-and-scale fixup of one cell (Sec. 6, Hamilton et al.): when the cell
// solution has a negative entry, the negative entries become zero and the
// others are scaled by one factor chosen so that the cell's particle balance,
// the sum of the rows of its local system, still holds.  In canonical node
// order the columns of A sum to (sw, sw + a, sw + b, sw + a + b) with
// sw = sigma_t hx hy/4, so the balance reads
//     sw (I0 + I1 + I2 + I3) + a (I1 + I3) + b (I2 + I3) = src,
// src the sum of the right-hand sides.  When no non-negative solution keeps
// it (src <= 0), the cell is set to zero.
template <typename real>
__device__ __forceinline__ void zero_and_scale(real &I0, real &I1, real &I2, real &I3, real sw, real a, real b,
                                               real src) {
    if (fmin(fmin(I0, I1), fmin(I2, I3)) < real(0)) {
        const real p0 = fmax(I0, real(0)), p1 = fmax(I1, real(0)), p2 = fmax(I2, real(0)), p3 = fmax(I3, real(0));
        const real den = sw * (p0 + p1 + p2 + p3) + a * (p1 + p3) + b * (p2 + p3);
        const real f = (src > real(0) && den > real(0)) ? src * recip(den) : real(0);
        I0 = f * p0; I1 = f * p1; I2 = f * p2; I3 = f * p3;
    }
}

__device__ __forceinline__ void bstore_pair(float a, float b, rsrc_t r, uint32_t vo, uint32_t so) {
    using u2 = __attribute__((ext_vector_type(2))) unsigned int;
    u2 w;
    w[0] = __float_as_uint(a); w[1] = __float_as_uint(b);
    __builtin_amdgcn_raw_buffer_store_b64(w, r, vo, so, 0);
}
__device__ __forceinline__ void bstore_pair(double a, double b, rsrc_t r, uint32_t vo, uint32_t so) {
    using u4 = __attribute__((ext_vector_type(4))) unsigned int;
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4, make_double2(a, b)), r, vo, so, 0);
}

// LDS ring through which the NW waves of a workgroup (the group blocks of one
// direction) combine their per-node group sums: RING steps deep, one slot
// per step holding every wave's two sums per lane, an arrival count and a
// consumed count per slot.
constexpr int RING = 8;
template <typename real, int NW>
constexpr size_t ring_bytes() {
    return NW > 1 ? (size_t)RING * NW * 64 * 2 * sizeof(real) + 2 * RING * sizeof(unsigned) : 0;
}

// One workgroup = one task (problem, band, chunk): a chunk is one direction
// of a quadrant and a block of 4*K*NW groups; wave w sweeps groups
// 4K w .. 4K w + 4K - 1 of the block (channel c, pair k -> group 4k + c).
template <typename real, int K, int PF, int NW, bool BATCH, bool FIX>
__global__ void __launch_bounds__(NW * 64) sweep2d_kernel(SweepLaunch L) {
    using r2 = typename vec2<real>::type;
    using r4 = typename vec4<real>::type;
    constexpr int TW = trace_words<real>::n;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ int s_prob, s_task, s_epoch;

    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int wvu = __builtin_amdgcn_readfirstlane(wv);   // the same value, known wave-uniform
    const int ch = lane >> 4;
    const int r = lane & 15;

    if (threadIdx.x == 0) {
        const int2 tk = L.tasks[atomicAdd(&L.lctr[0], 1)];
        s_prob = tk.x;
        s_task = tk.y;
        int *pc = BATCH ? L.probs[tk.x].ctr : L.single.ctr;
        s_epoch = __hip_atomic_load(&pc[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    // the ring's counters start at zero
    r2 *ring = reinterpret_cast<r2 *>(smem_raw);
    unsigned *arrived = reinterpret_cast<unsigned *>(smem_raw + (size_t)RING * NW * 64 * sizeof(r2));
    unsigned *consumed = arrived + RING;
    if constexpr (NW > 1) {
        if (threadIdx.x < 2 * RING) arrived[threadIdx.x] = 0;
    }
    __syncthreads();
    const int prob = __builtin_amdgcn_readfirstlane(s_prob);
    // problem arguments: kernel arguments (one problem) or the batch's device
    // array (uniform index, so they live in scalar registers either way)
    const Sweep2DArgs A = BATCH ? load_uniform_args(L.probs + prob) : L.single;
    const int task = __builtin_amdgcn_readfirstlane(s_task);
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

    // the chunk's direction (slot 0 of wave 0 is always active); this wave's
    // first group, or -1 when the block has no group for it
    const int d = __builtin_amdgcn_readfirstlane(A.slot_pair[qc * A.R].x);
    const int2 pg0 = A.slot_pair[qc * A.R + wv * CHANNELS * K];
    const bool wave_on = __builtin_amdgcn_readfirstlane(pg0.x) >= 0;
    const real *dr = dirs + 8 * d;
    const real am = fabs(dr[0]), bm = fabs(dr[1]);
    const int gb0 = wave_on ? __builtin_amdgcn_readfirstlane(pg0.y) : 0;
    bool act[K];
    int gl[K];                    // group within the wave's block (0 for an inactive slot)
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int slot = (wv * CHANNELS + ch) * K + k;
        const int2 pg = A.slot_pair[qc * A.R + slot];
        act[k] = pg.x >= 0 && row_ok;
        gl[k] = pg.y >= 0 ? pg.y - gb0 : 0;
    }
    const real hy = row_ok ? hya[jn] : real(1);
    const int64_t gslab = (int64_t)nbands * NT * BAND_ROWS;   // cells per (direction or quadrant, group) slab
    const real icdt = (real)A.inv_c_dt;

    // boundary side bases in the general inflow array [d][g][NB]
    const int xside = fx ? 2 * ny : 0;                 // canonical x- side
    const int yside = 4 * ny + (fy ? 2 * nx : 0);      // canonical y- side
    // band trace words of a (chunk, band): [slot (wave, k, channel)][column][2 values][TW]
    const int64_t traces_per_band = (int64_t)A.R * nx * 2 * TW;
    uint64_t *trace_in = A.trace + ((int64_t)qc * nbands + (band > 0 ? band - 1 : 0)) * traces_per_band;
    uint64_t *trace_out = A.trace + ((int64_t)qc * nbands + band) * traces_per_band;
    const bool produce = (r == BAND_ROWS - 1) && (band + 1 < nbands);

    // buffer resources (wave-uniform bases) and per-lane byte offsets
    const bool has_prev = pprev != nullptr;
    const int64_t pbase = (((int64_t)d * G + gb0) * nbands + band) * NT * BAND_ROWS;
    const int64_t tbase = ((int64_t)quad * G + gb0) * gslab + (int64_t)band * NT * BAND_ROWS;
    const uint64_t span = (uint64_t)CHANNELS * K * gslab;           // cells covered from a base
    // psi_prev may be absent (raw sweep without a time-edge source): an empty
    // resource then makes every load of it return zeros.
    const rsrc_t rs_prev = make_rsrc((has_prev ? pprev : pout) + pbase, has_prev ? span * sizeof(r4) : 0);
    const rsrc_t rs_out = make_rsrc(pout + pbase, span * sizeof(r4));
    const rsrc_t rs_sig = make_rsrc(sig2 + tbase, span * sizeof(r2));
    const rsrc_t rs_q = make_rsrc(qiso + tbase, span * sizeof(r4));
    const rsrc_t rs_inf = make_rsrc(inflow + ((int64_t)d * G + gb0) * A.NB, (uint64_t)CHANNELS * K * A.NB * sizeof(real));
    const uint64_t band_trace_bytes = (uint64_t)traces_per_band * sizeof(uint64_t);
    const rsrc_t rs_tr = make_rsrc(trace_in, band_trace_bytes);
    const rsrc_t rs_tw = make_rsrc(trace_out, band_trace_bytes);
    // moment partials of the (chunk, band): [t][channel = node][row][2]
    r2 *part_band = static_cast<r2 *>(A.part) + ((int64_t)qc * nbands + band) * NT * 64;
    const rsrc_t rs_part = make_rsrc(part_band, (uint64_t)NT * 64 * sizeof(r2));
    const uint32_t vo_part = (uint32_t)(lane * sizeof(r2));
    // lane byte offsets, OOB for a lane with no work (see make_rsrc)
    uint32_t vo4[K], vo2[K];   // cell gl * gslab + r in the 4-value and 2-value slabs
    uint32_t vo_inf[K], vo_tr[K], vo_tw[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const uint32_t cell = (uint32_t)(gl[k] * gslab + r);
        const uint32_t slot_bytes = (uint32_t)((((wv * K + k) * CHANNELS + ch) * nx * 2 * TW) * sizeof(uint64_t));
        vo4[k] = act[k] ? cell * (uint32_t)sizeof(r4) : OOB;
        vo2[k] = act[k] ? cell * (uint32_t)sizeof(r2) : OOB;
        vo_inf[k] = act[k] ? (uint32_t)((gl[k] * A.NB + yside) * sizeof(real)) : OOB;
        vo_tr[k] = act[k] ? slot_bytes : OOB;
        vo_tw[k] = act[k] && produce ? slot_bytes : OOB;
    }
    const uint32_t col_bytes = (uint32_t)(2 * TW * sizeof(uint64_t));   // one column of one slot

    // All prefetch loads are issued unconditionally (in bounds, or at the
    // out-of-range offset of a lane with no work, which reads zeros) into raw
    // registers, so several steps of loads stay in flight: a load under a
    // branch, or a reordering of its result, makes the compiler wait for every
    // outstanding memory operation.
    auto load_step = [&](int t, StepIn<real, K> &S) {
        // steps past NT (padding of the last group of PF+1 steps) touch no cell
        // and read the tables of step NT-1
        const int tt = t < NT ? t : NT - 1;
        const int c0 = t < nx ? t : nx - 1;               // row 0's column (clamped)
        const int in0 = fx ? nx - 1 - c0 : c0;            // ... in natural order
        // band trace words first (band > 0, row 0): every lane of a channel reads
        // the words its row-0 lane needs, so a wave touches one address per channel
#pragma unroll
        for (int k = 0; k < K; ++k) bload_words(S.tw[k], 2 * TW, rs_tr, vo_tr[k], (uint32_t)c0 * col_bytes);
        S.hx0 = hxa[in0];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            r2 sv;
            bload(sv, rs_sig, vo2[k], (uint32_t)(tt * BAND_ROWS * sizeof(r2)));
            S.st[k] = sv.x;
            S.sg[k] = sv.y;
            r4 qn;
            bload(qn, rs_q, vo4[k], (uint32_t)(tt * BAND_ROWS * sizeof(r4)));
            S.qn[k][0] = qn.x; S.qn[k][1] = qn.y; S.qn[k][2] = qn.z; S.qn[k][3] = qn.w;
            r4 p;
            bload(p, rs_prev, vo4[k], (uint32_t)(tt * BAND_ROWS * sizeof(r4)));
            S.psi[k][0] = p.x; S.psi[k][1] = p.y; S.psi[k][2] = p.z; S.psi[k][3] = p.w;
            // y- boundary inflow at row 0's column (used by band 0, row 0 only)
            bload_pair(S.bot[k][0], S.bot[k][1], rs_inf, vo_inf[k], (uint32_t)(2 * in0 * sizeof(real)));
        }
    };

    real xl[K][2], yb[K][2];   // x-upwind (nodes 1,3 of the left cell), y-upwind (nodes 2,3 of the cell below)
    real left[K][2];           // canonical x- boundary inflow of this row (nodes 0, 2)
    real hx_sh = 0;            // width of the column of the row above at the previous step
#pragma unroll
    for (int k = 0; k < K; ++k) {
        xl[k][0] = xl[k][1] = yb[k][0] = yb[k][1] = 0;
        const int64_t ib = ((int64_t)d * G + gb0 + gl[k]) * A.NB;
        const int ly0 = fy ? 1 : 0;
        const int jv = row_ok ? jn : 0;
        left[k][0] = act[k] ? inflow[ib + xside + 2 * jv + ly0] : real(0);
        left[k][1] = act[k] ? inflow[ib + xside + 2 * jv + (1 - ly0)] : real(0);
    }
    StepIn<real, K> buf[PF + 1];
#pragma unroll
    for (int u = 0; u <= PF; ++u) load_step(u, buf[u]);
    // One full wait after the prologue: the loop then starts from a state with
    // no pending loads, so the per-step waits only cover the slot being used.
    __builtin_amdgcn_s_waitcnt(0);
    int err = 0;

    // word index of (column, this lane's slot k) in a band's trace block
    auto trace_word = [&](int column, int k) -> int64_t {
        return ((int64_t)((wv * K + k) * CHANNELS + ch) * nx + column) * 2 * TW;
    };

    // Start gate: a band begins only once the band below has published the
    // trace of column TRACE_LAG, so that in steady state each prefetched
    // trace word was written several steps before it is needed.
    if (band > 0) {
        const int gcol = TRACE_LAG < nx - 1 ? TRACE_LAG : nx - 1;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const uint64_t *g = trace_in + trace_word(gcol, k);
            bool waiting = (r == 0) && act[k];
            int spins = 0;
            while (waiting) {
                bool rd = true;
#pragma unroll
                for (int u2 = 0; u2 < 2 * TW; ++u2) rd &= (uint32_t)(poll_word(g + u2) >> 32) == epoch;
                if (rd) break;
                if (++spins > SPIN_LIMIT) {
                    err = 1;
                    atomicOr(&A.ctr[3], WAIT_START_GATE);
                    break;
                }
                if (__hip_atomic_load(&A.ctr[3], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                    err = 1;   // another wave timed out: give up at once
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
        }
    }

    // rows 0 of active slots: the lanes that read the band below's trace
    uint64_t row0_mask[K];
#pragma unroll
    for (int k = 0; k < K; ++k) row0_mask[k] = __builtin_amdgcn_ballot_w64(r == 0 && act[k]);
    // The step loop runs in whole groups of PF+1 steps with no per-step
    // condition (a conditional step or prefetch would merge register values
    // and force a wait on every outstanding load); padding steps t >= NT have
    // no valid column, so they store nothing.
    for (int t0 = 0; t0 < NT; t0 += PF + 1) {
#pragma unroll
        for (int u = 0; u <= PF; ++u) {
            const int t = t0 + u;
            {
                StepIn<real, K> &S = buf[u];
                const int ic = t - r;
                const real hx = (r == 0) ? S.hx0 : hx_sh;
                const real wgt = hx * hy * real(0.25);
                const real a = am * hy * real(0.5);
                const real b = bm * hx * real(0.5);
                real sumI[4], sumS[4];   // sum_k I, sum_k sigma I
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    // y-upwind values: the lane below (already shifted) or, in row 0, the
                    // band below (trace words) or the y- boundary (band 0); branch-free
                    // except for the rare wait on a trace word that is not yet valid.
                    uint64_t *tw = S.tw[k];
                    // row 0 has a column at this step exactly when t < nx (ic = t)
                    if (band > 0 && t < nx) {
                        bool ready = true;
#pragma unroll
                        for (int u2 = 0; u2 < 2 * TW; ++u2) ready &= (uint32_t)(tw[u2] >> 32) == epoch;
                        const uint64_t need = __builtin_amdgcn_ballot_w64(!ready) & row0_mask[k];
                        if (need != 0) {
                            const uint64_t *src = trace_in + trace_word(t, k);
                            int spins = 0;
                            bool waiting = ((need >> lane) & 1) && !err;
                            while (waiting) {
                                // bounded wait; a timed-out wave raises ctr[3] and every other
                                // waiter gives up at once
                                if (++spins > SPIN_LIMIT) {
                                    err = 1;
                                    atomicOr(&A.ctr[3], WAIT_TRACE);
                                    break;
                                }
                                if (__hip_atomic_load(&A.ctr[3], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                                    err = 1;
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
                    }
                    const real bv0 = fx ? S.bot[k][1] : S.bot[k][0];   // canonical node 0 is natural lx = fx
                    const real bv1 = fx ? S.bot[k][0] : S.bot[k][1];
                    const real e0 = band == 0 ? bv0 : word_value(tw, real(0));
                    const real e1 = band == 0 ? bv1 : word_value(tw + TW, real(0));
                    const real yin0 = (r == 0) ? e0 : yb[k][0];
                    const real yin1 = (r == 0) ? e1 : yb[k][1];
                    const real xin0 = (ic == 0) ? left[k][0] : xl[k][0];
                    const real xin2 = (ic == 0) ? left[k][1] : xl[k][1];
                    const real ps0 = S.psi[k][0], ps1 = S.psi[k][1], ps2 = S.psi[k][2], ps3 = S.psi[k][3];
                    real rh0 = wgt * (S.qn[k][0] + icdt * ps0) + a * xin0 + b * yin0;
                    real rh1 = wgt * (S.qn[k][1] + icdt * ps1) + b * yin1;
                    real rh2 = wgt * (S.qn[k][2] + icdt * ps2) + a * xin2;
                    real rh3 = wgt * (S.qn[k][3] + icdt * ps3);
                    const real dg = real(0.5) * (a + b) + S.st[k] * wgt;
                    const real ha = real(0.5) * a, hb = real(0.5) * b;
                    const real y0 = dg * rh0 - ha * rh1 - hb * rh2;
                    const real y1 = dg * rh1 + ha * rh0 - hb * rh3;
                    const real y2 = dg * rh2 - ha * rh3 + hb * rh0;
                    const real y3 = dg * rh3 + ha * rh2 + hb * rh1;
                    const real al = dg * dg + ha * ha + hb * hb;
                    const real be = real(2) * ha * hb;
                    const real inv = recip(al * al - be * be);
                    const real ai = al * inv, bi = be * inv;
                    real I0 = ai * y0 + bi * y3;
                    real I1 = ai * y1 - bi * y2;
                    real I2 = ai * y2 - bi * y1;
                    real I3 = ai * y3 + bi * y0;
                    if constexpr (FIX) zero_and_scale(I0, I1, I2, I3, S.st[k] * wgt, a, b, (rh0 + rh1) + (rh2 + rh3));
                    // A cell outside the mesh (ic < 0 or ic >= nx, or a row past ny)
                    // is a padding slot of the skewed layout: its store lands
                    // there and its sums are never read, so neither needs a
                    // per-lane test.  Padding steps (t >= NT) store nothing.
                    if (t < NT) {
                        r4 o;
                        o.x = I0; o.y = I1; o.z = I2; o.w = I3;
                        bstore(o, rs_out, vo4[k], (uint32_t)(t * BAND_ROWS * sizeof(r4)));
                    }
                    // the top row publishes its column ic = t - 15 while it lies in the mesh
                    if (t >= BAND_ROWS - 1 && t < NT) {
                        const uint32_t so = (uint32_t)(t - (BAND_ROWS - 1)) * col_bytes;
                        put_trace_words(I2, epoch, rs_tw, vo_tw[k], so);
                        put_trace_words(I3, epoch, rs_tw, vo_tw[k], so + TW * (uint32_t)sizeof(uint64_t));
                    }
                    const real sg = S.sg[k];
                    if (k == 0) {
                        sumI[0] = I0; sumI[1] = I1; sumI[2] = I2; sumI[3] = I3;
                        sumS[0] = sg * I0; sumS[1] = sg * I1; sumS[2] = sg * I2; sumS[3] = sg * I3;
                    } else {
                        sumI[0] += I0; sumI[1] += I1; sumI[2] += I2; sumI[3] += I3;
                        sumS[0] += sg * I0; sumS[1] += sg * I1; sumS[2] += sg * I2; sumS[3] += sg * I3;
                    }
                    xl[k][0] = I1;
                    xl[k][1] = I3;
                    yb[k][0] = shift_up_one_row<real>(I2);
                    yb[k][1] = shift_up_one_row<real>(I3);
                }
                hx_sh = shift_up_one_row<real>(hx);
                // prefetch the step PF+1 ahead into the slot just consumed
                load_step(t + PF + 1, buf[u]);

                // channel sums: channel c gets node c's sums over the wave's groups
                const real nI = channel_scatter_sum<real>(sumI);
                const real nS = channel_scatter_sum<real>(sumS);
                if (t < NT) {
                    if constexpr (NW == 1) {
                        bstore_pair(nI, nS, rs_part, vo_part, (uint32_t)(t * 64 * sizeof(r2)));
                    } else {
                        // Combine the workgroup's waves through the LDS ring: each
                        // wave deposits its sums; the last to arrive at this step
                        // adds them in wave order and stores the partial.
                        const int slot = t & (RING - 1);
                        const unsigned round = (unsigned)(t / RING);
                        if (round > 0 && !err) {
                            // the slot's previous step must have been consumed
                            int spins = 0;
                            while (__hip_atomic_load(&consumed[slot], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) <
                                   round) {
                                if (++spins > SPIN_LIMIT) {
                                    err = 1;
                                    atomicOr(&A.ctr[3], WAIT_RING);
                                    break;
                                }
                                if (__hip_atomic_load(&A.ctr[3], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                                    err = 1;
                                    break;
                                }
                                __builtin_amdgcn_s_sleep(1);
                            }
                        }
                        r2 mine;
                        mine.x = nI;
                        mine.y = nS;
                        ring[(slot * NW + wvu) * 64 + lane] = mine;
                        unsigned prev = 0;
                        if (lane == 0)
                            prev = __hip_atomic_fetch_add(&arrived[slot], 1u, __ATOMIC_ACQ_REL,
                                                          __HIP_MEMORY_SCOPE_WORKGROUP);
                        prev = __builtin_amdgcn_readfirstlane(prev);
                        if (prev == round * NW + (NW - 1)) {
                            real sI = 0, sS = 0;   // fixed order over the waves
#pragma unroll
                            for (int w2 = 0; w2 < NW; ++w2) {
                                const r2 v = ring[(slot * NW + w2) * 64 + lane];
                                sI += v.x;
                                sS += v.y;
                            }
                            bstore_pair(sI, sS, rs_part, vo_part, (uint32_t)(t * 64 * sizeof(r2)));
                            if (lane == 0)
                                __hip_atomic_fetch_add(&consumed[slot], 1u, __ATOMIC_RELEASE,
                                                       __HIP_MEMORY_SCOPE_WORKGROUP);
                        }
                    }
                }
            }
        }
    }

    // completion: per-problem epoch, per-launch ticket
    __syncthreads();
    if (threadIdx.x == 0) {
        // the problem's last workgroup advances its epoch (every workgroup of the
        // problem read the epoch before this point)
        const int done = atomicAdd(&A.ctr[1], 1);
        if (done == A.n_wg - 1) {
            __hip_atomic_store(&A.ctr[1], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(&A.ctr[2], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        // the launch's last workgroup resets the ticket
        const int ldone = atomicAdd(&L.lctr[1], 1);
        if (ldone == L.n_tasks - 1) {
            __hip_atomic_store(&L.lctr[0], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&L.lctr[1], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// prefetch depth: PF + 1 steps of loads in flight (fewer when K pairs per
// lane make a step's loads larger)
template <typename real, int K>
constexpr int prefetch_depth() {
    return sizeof(real) == 4 ? (K == 1 ? 4 : K == 2 ? 3 : 1) : (K == 1 ? 2 : 1);
}

template <typename real, int K, int NW, bool BATCH, bool FIX>
static void launch_knwbf(const SweepLaunch &L, hipStream_t s) {
    constexpr int PF = prefetch_depth<real, K>();
    // LDS: the wave ring, or more when the launch asks for fewer workgroups
    // per CU (a workgroup alone on a CU runs each step faster)
    size_t lds = ring_bytes<real, NW>();
    if (L.wg_per_cu > 0) lds = std::max(lds, (size_t)(LDS_PER_CU / L.wg_per_cu - 1024));
    static bool lds_attr_set = false;   // once per instantiation (so a launch can be graph-captured)
    if (!lds_attr_set) {
        SMRT_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&sweep2d_kernel<real, K, PF, NW, BATCH, FIX>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, LDS_PER_CU - 1024));
        lds_attr_set = true;
    }
    hipLaunchKernelGGL((sweep2d_kernel<real, K, PF, NW, BATCH, FIX>), dim3(L.n_tasks), dim3(NW * 64), lds, s, L);
}
template <typename real, int K, int NW, bool BATCH>
static void launch_knwb(const SweepLaunch &L, hipStream_t s) {
    if (L.fixup) launch_knwbf<real, K, NW, BATCH, true>(L, s);
    else launch_knwbf<real, K, NW, BATCH, false>(L, s);
}
template <typename real, int K, int NW>
static void launch_knw(const SweepLaunch &L, hipStream_t s) {
    if (L.probs) launch_knwb<real, K, NW, true>(L, s);
    else launch_knwb<real, K, NW, false>(L, s);
}

template <typename real, int K>
static void launch_k(const SweepLaunch &L, hipStream_t s) {
    switch (L.NW) {
        case 1: launch_knw<real, K, 1>(L, s); return;
        case 2: launch_knw<real, K, 2>(L, s); return;
        case 4: launch_knw<real, K, 4>(L, s); return;
        case 8: launch_knw<real, K, 8>(L, s); return;
        default: throw Error(SMRT_E_INVALID_ARG, "waves per workgroup must be 1, 2, 4 or 8");
    }
}

template <typename real>
void launch_sweep2d(const SweepLaunch &L, hipStream_t s) {
    if (L.n_tasks <= 0) return;
    if (L.K == 1) { launch_k<real, 1>(L, s); SMRT_HIP(hipGetLastError()); return; }
    if (L.K == 2) { launch_k<real, 2>(L, s); SMRT_HIP(hipGetLastError()); return; }
    if constexpr (sizeof(real) == 4) {
        if (L.K == 4) { launch_k<real, 4>(L, s); SMRT_HIP(hipGetLastError()); return; }
    }
    throw Error(SMRT_E_INVALID_ARG, "pairs per lane must be 1, 2 (FP64) or 1, 2, 4 (FP32)");
}

template void launch_sweep2d<float>(const SweepLaunch &, hipStream_t);
template void launch_sweep2d<double>(const SweepLaunch &, hipStream_t);

}  // namespace smrt
