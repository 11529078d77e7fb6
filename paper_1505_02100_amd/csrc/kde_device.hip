// Device code of libkdeplugin: one persistent kernel that walks an ordered
// work list of (sample, stage, tile) items and carries every sample through
// Algorithm 1 (Steps I-VII), plus a small init kernel.
//
// Pair stages (Steps IV and VI).  The strict upper triangle i < j of the
// n x n pair matrix (the symmetric form of equations (6)-(7)) is cut into
// items of TI = BLOCK * R rows by W columns.  A block keeps its TI row values
// in registers (R per lane; each wave owns 64 R consecutive rows) and streams
// the item's columns through LDS in tiles of TJ values; every lane reads the
// same column value (LDS broadcast) and evaluates R pairs with it.  Columns
// left of a wave's rows are skipped, columns inside its row span are masked
// (j > i per lane), and columns right of it run unmasked, so the mask costs
// 64 R columns per wave per diagonal item only.
//
// FP32 pair arithmetic.  The samples are prescaled once per tile load,
// v = (x - c) / g, in FP64 and then rounded to FP32, so d = v_i - v_j is the
// kernel argument y = (x_i - x_j)/g of Steps IV and VI.  With Y = y^2:
//     He6(y) = ((Y - 15) Y + 45) Y - 15,    He4(y) = (Y - 6) Y + 3,
// whose coefficients are small integers, exact in FP32, and the Gaussian
// factor exp(-Y/2) = 2^(-k Y), k = log2(e)/2, is one v_exp_f32.  Per pair
// (r = 6):
//     d = vi - vj; Y = d d; a = k Y; e = exp2(-a);
//     q = Y - 15; q = fma(q, Y, 45); p = fma(q, Y, -15); acc = fma(p, e, acc)
// which is 7 VALU + 1 transcendental (r = 4 drops one fma: 6 + 1); 1/sqrt(2 pi)
// is applied once to the FP64 total.  The default precision evaluates Step IV
// in the depressed form instead (Z = Y - 5, He6 = (Z^2 - 30) Z - 40, 6 + 1):
// h depends on Psi6 only through g2^(1/7) and Psi4's weak dependence on g2,
// so the small absorption bias of that form costs about 1e-8 in h.
//
// Why this form.  The sums of K6 and K4 over all pairs cancel heavily:
// sum |K| / |sum K| is in the hundreds at n = 1024 and grows like g^-6, to
// about 1e4 at n = 2^20.  A systematic error of relative size b per term
// therefore costs b times that factor, while errors that vary randomly from
// pair to pair average out.  Measured on gfx950 at n = 2^20, the systematic
// sources were, in order: FP32 running sums that take many terms (rounding
// of a growing partial sum is not unbiased; 32 terms per accumulator cost
// 2e-5 on Psi6), irrational polynomial coefficients rounded to FP32 (this
// is why all coefficients are integers here), the absorption of a small
// y^2 into an additive shift (why the polynomial is not depressed), and a
// small bias of v_exp_f32 (mean relative error about -3e-9).  So each row
// keeps four FP32 accumulators (one per column of an LDS b128 read) that take
// at most kFold terms each; the four are then added pairwise in FP32 (a
// 16-term pairwise sum) and the result goes into the lane's FP64 sum.
// The one systematic error left by construction is the FP32 rounding of k
// (relative 1.3e-8, i.e. the Gaussian taken at a bandwidth 7e-9 larger than
// the polynomial's); the EXACT_K variant removes it with a two-term k,
// a = fma(Y, k_hi, Y k_lo), at one more VALU op per pair.
//
// Each item also centres its rows and columns on its own offset,
// c = mean + g tau(row block) with tau a generic value in [-1/4, 1/4) (a
// golden-ratio sequence): the differences are unchanged, but a sample's FP32
// rounding differs from item to item instead of entering all its n pairs
// the same way.
//
// FP64 pair arithmetic is the plain printed form: t = y^2,
// p = ((t - 15) t + 45) t - 15 (resp. (t - 6) t + 3), exp(-t/2), FP64 sums.
//
// Cross-block reduction is deterministic.  Step I takes one pass: a moment
// item writes its chunk's sum, squared deviations from the chunk's own mean,
// minimum and maximum into two slots, and the block that completes the last
// chunk (atomic counter) merges the chunks in a fixed order with the update
// of Chan, Golub and LeVeque and publishes both Step I stages at once (the
// second stage's items only count).  A pair item's FP64
// partial is added exactly, as a 128-bit fixed-point integer, into the
// block's accumulator, which goes into the stage's accumulator with
// integer atomics; integer addition does not depend on order, so the sum
// is the same for every schedule and the finaliser reads it in one step.
// The finaliser runs the stage's scalar formulas (Steps I-III, V, VII) in
// FP64 and publishes them with a release flag.
// Items of a later stage wait (acquire, bounded by a wall-clock limit) for
// that flag.  Items of earlier stages always hold smaller tickets, and no
// item waits on a later ticket, so the wait always ends.
#include <hip/hip_runtime.h>

#include <math.h>

#include <type_traits>

#include "kde_exp2_poly.h"
#include "kde_internal.h"

namespace kde {

constexpr int WAVE = 64;
constexpr int TJ = 1024;  // column tile (values) in LDS
// Largest |u| for which the FP32 pair term cannot overflow: |d| <= 2e6 gives
// s <= 4e12 and p(s) < 7e37.  Samples spread wider take the clamped variant.
constexpr double kSafeLimit = 1.0e6;

__device__ __forceinline__ uint32_t ld_acquire(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_release(uint32_t* p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_relaxed(uint32_t* p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_f64(const double* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_f64(double* p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t ld_i32(const int32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void set_status(State* st, int32_t code) {
    int32_t expect = 0;
    __hip_atomic_compare_exchange_strong(&st->status, &expect, code, __ATOMIC_RELAXED,
                                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ double load_x(const void* x, int32_t dtype, int64_t i) {
    return dtype == 0 ? static_cast<const double*>(x)[i]
                      : static_cast<double>(static_cast<const float*>(x)[i]);
}


// The fields of a sample's descriptor an item needs, read once per item
// (no copy of the whole descriptor, whose per-stage arrays would otherwise be
// indexed dynamically in private memory).
struct View {
    const void* x;
    int64_t n;
    int64_t W;
    double psi_g;
    int64_t base;   // first slot of this item's stage
    int32_t dtype;
    int32_t mode;
    int32_t chunk;
    int32_t cnt;    // items of this item's stage
};

__device__ __forceinline__ View load_view(const Desc* dp, int32_t stage) {
    View v;
    v.x = dp->x;
    v.n = dp->n;
    v.W = dp->W;
    v.psi_g = dp->psi_g;
    v.base = dp->slot_base[stage];
    v.dtype = dp->dtype;
    v.mode = dp->mode;
    v.chunk = dp->chunk;
    v.cnt = dp->n_items[stage];
    return v;
}

// ------------------------------------------------------------ reductions
template <int BLOCK>
__device__ __forceinline__ double block_sum(double v, double* red) {
    // fixed butterfly inside the wave, then waves in index order
#pragma unroll
    for (int off = WAVE / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
    const int lane = threadIdx.x & (WAVE - 1), wave = threadIdx.x / WAVE;
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double tot = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int w = 0; w < BLOCK / WAVE; ++w) tot += red[w];
    }
    __syncthreads();
    return tot;  // valid in thread 0
}

template <int BLOCK>
__device__ __forceinline__ double block_max(double v, double* red) {
#pragma unroll
    for (int off = WAVE / 2; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, WAVE));
    const int lane = threadIdx.x & (WAVE - 1), wave = threadIdx.x / WAVE;
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double m = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int w = 0; w < BLOCK / WAVE; ++w) m = fmax(m, red[w]);
    }
    __syncthreads();
    return m;
}

template <int BLOCK>
__device__ __forceinline__ double block_max_signed(double v, double* red) {
#pragma unroll
    for (int off = WAVE / 2; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, WAVE));
    const int lane = threadIdx.x & (WAVE - 1), wave = threadIdx.x / WAVE;
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double m = v;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int w = 0; w < BLOCK / WAVE; ++w) m = fmax(m, red[w]);
    }
    __syncthreads();
    return m;  // valid in thread 0
}

// ------------------------------------------------------------- moments
// Each thread reads U values per round so that the loads of a round are in
// flight together; per-thread order is fixed, so the result is deterministic.
constexpr int kMomentUnroll = 8;

// Step I in one pass over chunk chunk_idx: the sum of x - x[0] (every chunk
// takes the same shift, so the chunk means the merge compares are small
// numbers and keep their accuracy when the sample sits far from 0), the
// sum of squared deviations from the chunk's own mean (the data are read
// again for that, from cache), and the chunk's minimum and maximum.
// Per-thread order is fixed, so the result is deterministic.  All four are
// valid in thread 0.
template <int BLOCK>
__device__ void moment_stats(const View& d, int32_t chunk_idx, double* red, double* out_sum, double* out_m2,
                             double* out_min, double* out_max) {
    const int64_t a = (int64_t)chunk_idx * d.chunk;
    const int64_t b = min(a + (int64_t)d.chunk, d.n);
    const double x0 = load_x(d.x, d.dtype, 0);
    double s = 0.0, lo = INFINITY, hi = -INFINITY;
    for (int64_t i0 = a + threadIdx.x; i0 < b; i0 += (int64_t)BLOCK * kMomentUnroll) {
        double v[kMomentUnroll];
#pragma unroll
        for (int u = 0; u < kMomentUnroll; ++u) {
            const int64_t i = i0 + (int64_t)u * BLOCK;
            v[u] = i < b ? load_x(d.x, d.dtype, i) : x0;
        }
#pragma unroll
        for (int u = 0; u < kMomentUnroll; ++u) {
            s += v[u] - x0;
            lo = fmin(lo, v[u]);
            hi = fmax(hi, v[u]);
        }
    }
    const double sum = block_sum<BLOCK>(s, red);
    if (threadIdx.x == 0) red[0] = sum / (double)(b - a);
    __syncthreads();
    const double mc = red[0];
    __syncthreads();
    double q = 0.0;
    for (int64_t i0 = a + threadIdx.x; i0 < b; i0 += (int64_t)BLOCK * kMomentUnroll) {
        double v[kMomentUnroll];
#pragma unroll
        for (int u = 0; u < kMomentUnroll; ++u) {
            const int64_t i = i0 + (int64_t)u * BLOCK;
            v[u] = i < b ? (load_x(d.x, d.dtype, i) - x0) - mc : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kMomentUnroll; ++u) q = fma(v[u], v[u], q);
    }
    *out_sum = sum;
    *out_m2 = block_sum<BLOCK>(q, red);
    *out_min = -block_max_signed<BLOCK>(-lo, red);
    *out_max = block_max_signed<BLOCK>(hi, red);
}

// Merge of two (count, mean, sum of squared deviations) triples, the
// pairwise update of Chan, Golub and LeVeque: exact in real arithmetic and
// stable in floating point whatever the spread of the two means.
__device__ __forceinline__ void chan_merge(double& n, double& mean, double& m2, double nb, double meanb,
                                           double m2b) {
    if (nb == 0.0) return;
    if (n == 0.0) {
        n = nb;
        mean = meanb;
        m2 = m2b;
        return;
    }
    const double t = n + nb;
    const double delta = meanb - mean;
    mean += delta * (nb / t);
    m2 += m2b + delta * delta * (n * nb / t);
    n = t;
}

// ---------------------------------------------------- FP32 pair evaluation
// Largest Y kept by the clamped variant: exp2(-k Y) is exactly 0 there and
// Y^3 stays finite.
constexpr float kYClamp = 1.0e12f;
// Terms an FP32 accumulator takes before it is added into the FP64 lane sum.
constexpr int kFold = 4;

// 2^t from the minimax polynomial of degree kExp2PolyDegree (Remez exchange,
// FP32 coefficients) on the FMA pipes instead of the transcendental unit:
// t = n + f with n = round(t), f in [-1/2, 1/2], 2^t = 2^n p(f).  Arguments
// below -200 give 0, as 2^t is below FP32's range there.
__device__ __forceinline__ float exp2_poly(float t) {
    t = fmaxf(t, -200.0f);
    const float n = __builtin_rintf(t);
    const float f = t - n;
    float p = kExp2Poly[kExp2PolyDegree];
#pragma unroll
    for (int k = kExp2PolyDegree - 1; k >= 0; --k) p = fmaf(p, f, kExp2Poly[k]);
    return __builtin_ldexpf(p, (int)n);
}

template <int RO, bool SAFE, bool EXACT_K, bool PEXP = false>
__device__ __forceinline__ float pair_poly_exp(float vi, float vj, const PolyConsts& pc, float* e_out) {
    const float d = vi - vj;
    float p;
    if (RO == 6 && !EXACT_K) {
        // Step IV, default precision: the depressed form Z = Y - 5,
        // He6 = (Z^2 - 30) Z - 40 and exp(-Y/2) = 2^(-k Z) 2^(-5k), one VALU op
        // less per pair.  Its absorption of a tiny Y into -5 biases Psi6 by a
        // few 1e-6 at n = 2^20, which reaches h only through g2^(1/7) and
        // Psi4's weak dependence on g2 (about 1e-8 in h).
        float Z = fmaf(d, d, -5.0f);
        if (SAFE) Z = fminf(Z, kYClamp);
        *e_out = PEXP ? exp2_poly(-(Z * pc.k_hi)) : __builtin_amdgcn_exp2f(-(Z * pc.k_hi));
        const float q = fmaf(Z, Z, -30.0f);
        p = fmaf(q, Z, -40.0f);
        return p;
    }
    float Y = d * d;
    if (SAFE) Y = fminf(Y, kYClamp);
    const float a = EXACT_K ? fmaf(Y, pc.k_hi, Y * pc.k_lo) : Y * pc.k_hi;
    *e_out = PEXP ? exp2_poly(-a) : __builtin_amdgcn_exp2f(-a);
    if (RO == 6) {
        float q = Y - 15.0f;
        q = fmaf(q, Y, 45.0f);
        p = fmaf(q, Y, -15.0f);
    } else {
        const float q = Y - 6.0f;
        p = fmaf(q, Y, 3.0f);
    }
    return p;
}

template <int RO, bool SAFE, bool EXACT_K, bool PEXP = false>
__device__ __forceinline__ float pair_term_f32(float vi, float vj, const PolyConsts& pc) {
    float e;
    const float p = pair_poly_exp<RO, SAFE, EXACT_K, PEXP>(vi, vj, pc, &e);
    return p * e;
}

template <int RO, bool SAFE, bool EXACT_K, bool PEXP = false>
__device__ __forceinline__ void pair_acc_f32(float vi, float vj, float& acc, const PolyConsts& pc) {
    float e;
    const float p = pair_poly_exp<RO, SAFE, EXACT_K, PEXP>(vi, vj, pc, &e);
    acc = fmaf(p, e, acc);
}

template <int RO, bool SAFE, bool EXACT_K, int R, bool PEXP = false>
__device__ __forceinline__ void pair_b128_f32(const float (&ui)[R], float4 v, float (&acc)[R][4],
                                              const PolyConsts& pc) {
#pragma unroll
    for (int k = 0; k < R; ++k) {
        pair_acc_f32<RO, SAFE, EXACT_K, PEXP>(ui[k], v.x, acc[k][0], pc);
        pair_acc_f32<RO, SAFE, EXACT_K, PEXP>(ui[k], v.y, acc[k][1], pc);
        pair_acc_f32<RO, SAFE, EXACT_K, PEXP>(ui[k], v.z, acc[k][2], pc);
        pair_acc_f32<RO, SAFE, EXACT_K, PEXP>(ui[k], v.w, acc[k][3], pc);
    }
}

template <int R>
__device__ __forceinline__ void fold_f64(float (&acc)[R][4], double (&tot)[R]) {
#pragma unroll
    for (int k = 0; k < R; ++k) {
        tot[k] += (double)((acc[k][0] + acc[k][1]) + (acc[k][2] + acc[k][3]));
        acc[k][0] = acc[k][1] = acc[k][2] = acc[k][3] = 0.0f;
    }
}

// Step VI at R = 1 without the clamp (the default FP32 path), over cnt >= 1
// groups of 16 columns starting at LDS byte address addr (16-byte aligned),
// one row per lane, written out as a fixed loop.  The operations are exactly
// those of pair_acc_f32 and fold_f64 (per pair d = ui - xj, Y = d d,
// q = fma(d, d, -6), p = fma(q, Y, 3), e = 2^(Y (-k)); column c of every read
// into accumulator c in read order; then (a0 + a1) + (a2 + a3) into the FP64
// lane total), so the result is bitwise that of the generic loop.  Only the
// order differs: the compiler's schedule of this step ran at 5.3e12 pairs/s
// on MI355X, and timing valid orders of the step's dependency graph found this
// one at 6.1e12.  Here the first VALU instruction sits on an 8-byte boundary,
// the faster placement for this order.  An s_nop separates a v_exp_f32 from a
// VALU op that reads its result in the next instruction (gfx950 needs one
// wait state there).
__device__ __forceinline__ void pair16_loop_r4_f32(uint32_t addr, int32_t cnt, float ui, float k, double& tot) {
    asm volatile(
        ".p2align 6\n"
        "s_nop 0\n"
        "s_nop 0\n"
        "s_nop 0\n"
        "s_nop 0\n"
        "1:\n"
        "v_mov_b32_e32 v45, %[addr]\n"
        "ds_read_b128 v[40:43], v45 offset:16\n"
        "ds_read_b128 v[46:49], v45 offset:48\n"
        "ds_read_b128 v[50:53], v45\n"
        "ds_read_b128 v[54:57], v45 offset:32\n"
        "s_add_u32 %[addr], %[addr], 64\n"
        "s_sub_u32 %[cnt], %[cnt], 1\n"
        "s_waitcnt lgkmcnt(0)\n"
        "v_sub_f32_e32 v42, %[ui], v42\n"
        "v_sub_f32_e32 v56, %[ui], v56\n"
        "v_sub_f32_e32 v46, %[ui], v46\n"
        "v_sub_f32_e32 v51, %[ui], v51\n"
        "v_fmaak_f32 v59, v46, v46, 0xc0c00000\n"
        "v_sub_f32_e32 v41, %[ui], v41\n"
        "v_sub_f32_e32 v49, %[ui], v49\n"
        "v_fmaak_f32 v60, v41, v41, 0xc0c00000\n"
        "v_sub_f32_e32 v43, %[ui], v43\n"
        "v_sub_f32_e32 v57, %[ui], v57\n"
        "v_mul_f32_e32 v41, v41, v41\n"
        "v_fmaak_f32 v61, v43, v43, 0xc0c00000\n"
        "v_mul_f32_e32 v85, v57, v57\n"
        "v_fmaak_f32 v92, v51, v51, 0xc0c00000\n"
        "v_mul_f32_e32 v43, v43, v43\n"
        "v_mul_f32_e32 v93, v42, v42\n"
        "v_fmaak_f32 v60, v60, v41, 0x40400000\n"
        "v_sub_f32_e32 v52, %[ui], v52\n"
        "v_sub_f32_e32 v47, %[ui], v47\n"
        "v_mul_f32_e32 v94, v49, v49\n"
        "v_fmaak_f32 v95, v56, v56, 0xc0c00000\n"
        "v_mul_f32_e64 v41, v41, -%[k]\n"
        "v_sub_f32_e32 v48, %[ui], v48\n"
        "v_mul_f32_e32 v56, v56, v56\n"
        "v_fmaak_f32 v61, v61, v43, 0x40400000\n"
        "v_mul_f32_e32 v96, v47, v47\n"
        "v_mul_f32_e32 v97, v48, v48\n"
        "v_fmaak_f32 v98, v52, v52, 0xc0c00000\n"
        "v_mul_f32_e32 v51, v51, v51\n"
        "v_sub_f32_e32 v54, %[ui], v54\n"
        "v_fmaak_f32 v99, v54, v54, 0xc0c00000\n"
        "v_sub_f32_e32 v40, %[ui], v40\n"
        "v_sub_f32_e32 v53, %[ui], v53\n"
        "v_mul_f32_e32 v100, v53, v53\n"
        "v_fmaak_f32 v57, v57, v57, 0xc0c00000\n"
        "v_fmaak_f32 v48, v48, v48, 0xc0c00000\n"
        "v_fmaak_f32 v95, v95, v56, 0x40400000\n"
        "v_mul_f32_e32 v46, v46, v46\n"
        "v_fmaak_f32 v101, v40, v40, 0xc0c00000\n"
        "v_fmaak_f32 v47, v47, v47, 0xc0c00000\n"
        "v_mul_f32_e32 v40, v40, v40\n"
        "v_mul_f32_e32 v54, v54, v54\n"
        "v_fmaak_f32 v49, v49, v49, 0xc0c00000\n"
        "v_fmaak_f32 v99, v99, v54, 0x40400000\n"
        "v_fmaak_f32 v53, v53, v53, 0xc0c00000\n"
        "v_sub_f32_e32 v55, %[ui], v55\n"
        "v_fmaak_f32 v92, v92, v51, 0x40400000\n"
        "v_fmaak_f32 v102, v55, v55, 0xc0c00000\n"
        "v_fmaak_f32 v49, v49, v94, 0x40400000\n"
        "v_fmaak_f32 v57, v57, v85, 0x40400000\n"
        "v_sub_f32_e32 v50, %[ui], v50\n"
        "v_fmaak_f32 v59, v59, v46, 0x40400000\n"
        "v_fmaak_f32 v53, v53, v100, 0x40400000\n"
        "v_fmaak_f32 v103, v50, v50, 0xc0c00000\n"
        "v_fmaak_f32 v101, v101, v40, 0x40400000\n"
        "v_mul_f32_e32 v50, v50, v50\n"
        "v_fmaak_f32 v42, v42, v42, 0xc0c00000\n"
        "v_fmaak_f32 v48, v48, v97, 0x40400000\n"
        "v_fmaak_f32 v42, v42, v93, 0x40400000\n"
        "v_fmaak_f32 v103, v103, v50, 0x40400000\n"
        "v_mul_f32_e32 v55, v55, v55\n"
        "v_mul_f32_e64 v46, v46, -%[k]\n"
        "v_mul_f32_e64 v100, v100, -%[k]\n"
        "v_mul_f32_e64 v50, v50, -%[k]\n"
        "v_mul_f32_e64 v85, v85, -%[k]\n"
        "v_mul_f32_e64 v93, v93, -%[k]\n"
        "v_mul_f32_e64 v43, v43, -%[k]\n"
        "v_mul_f32_e64 v51, v51, -%[k]\n"
        "v_mul_f32_e64 v54, v54, -%[k]\n"
        "v_mul_f32_e64 v94, v94, -%[k]\n"
        "v_mul_f32_e64 v97, v97, -%[k]\n"
        "v_mul_f32_e64 v56, v56, -%[k]\n"
        "v_mul_f32_e64 v40, v40, -%[k]\n"
        "v_exp_f32_e32 v100, v100\n"
        "v_exp_f32_e32 v56, v56\n"
        "v_exp_f32_e32 v46, v46\n"
        "v_exp_f32_e32 v93, v93\n"
        "v_exp_f32_e32 v40, v40\n"
        "v_exp_f32_e32 v50, v50\n"
        "v_exp_f32_e32 v51, v51\n"
        "v_exp_f32_e32 v41, v41\n"
        "v_exp_f32_e32 v43, v43\n"
        "v_exp_f32_e32 v97, v97\n"
        "v_exp_f32_e32 v94, v94\n"
        "v_exp_f32_e32 v85, v85\n"
        "v_exp_f32_e32 v54, v54\n"
        "v_fmaak_f32 v47, v47, v96, 0x40400000\n"
        "v_fmaak_f32 v102, v102, v55, 0x40400000\n"
        "v_mul_f32_e32 v53, v53, v100\n"
        "v_mul_f32_e32 v100, v92, v51\n"
        "v_mul_f32_e32 v92, v52, v52\n"
        "v_fmaak_f32 v51, v98, v92, 0x40400000\n"
        "v_fmac_f32_e32 v53, v61, v43\n"
        "v_fmac_f32_e32 v53, v57, v85\n"
        "v_fmac_f32_e32 v100, v60, v41\n"
        "v_mul_f32_e32 v52, v103, v50\n"
        "v_fmac_f32_e32 v52, v101, v40\n"
        "v_fmac_f32_e32 v52, v99, v54\n"
        "v_fmac_f32_e32 v53, v49, v94\n"
        "v_fmac_f32_e32 v52, v59, v46\n"
        "v_mul_f32_e64 v98, v55, -%[k]\n"
        "v_mul_f32_e64 v61, v92, -%[k]\n"
        "v_mul_f32_e64 v43, v96, -%[k]\n"
        "v_exp_f32_e32 v57, v43\n"
        "v_exp_f32_e32 v85, v98\n"
        "v_exp_f32_e32 v60, v61\n"
        "s_nop 0\n"
        "v_mul_f32_e32 v41, v51, v60\n"
        "v_fmac_f32_e32 v41, v42, v93\n"
        "v_fmac_f32_e32 v41, v95, v56\n"
        "v_fmac_f32_e32 v41, v48, v97\n"
        "v_fmac_f32_e32 v100, v102, v85\n"
        "v_fmac_f32_e32 v100, v47, v57\n"
        "v_add_f32_e32 v103, v52, v100\n"
        "v_add_f32_e32 v50, v41, v53\n"
        "v_add_f32_e32 v101, v103, v50\n"
        "v_cvt_f64_f32_e32 v[42:43], v101\n"
        "s_cmp_lg_u32 %[cnt], 0\n"
        "v_add_f64 %[tot], %[tot], v[42:43]\n"
        "s_cbranch_scc1 1b\n"
        : [tot] "+{v[34:35]}"(tot), [addr] "+s"(addr), [cnt] "+s"(cnt)
        : [ui] "{v44}"(ui), [k] "s"(k)
        : "v40", "v41", "v42", "v43", "v45", "v46", "v47", "v48", "v49", "v50", "v51", "v52", "v53", "v54", "v55", "v56", "v57", "v59", "v60", "v61", "v85", "v92", "v93", "v94", "v95", "v96", "v97", "v98", "v99", "v100", "v101", "v102", "v103", "scc", "memory");
}

// Step IV at R = 1 without the clamp (the default FP32 path), over cnt >= 1
// groups of 16 columns starting at LDS byte address addr (16-byte aligned),
// one row per lane.  Per group: four b128 reads, then the operations of
// pair_acc_f32 in its depressed form (per pair d = ui - xj, Z = fma(d, d, -5),
// q = fma(Z, Z, -30), p = fma(q, Z, -40), e = 2^(Z (-k)); column c of every
// read into accumulator c in read order) and of fold_f64 ((a0 + a1) + (a2 + a3)
// into the FP64 lane total), so the result is bitwise that of the generic
// loop.  The instructions and registers are the compiler's own code for this
// step, whose order was as fast as any tried; the loop is written out whole
// so that neither its order nor its placement moves with changes elsewhere
// in the kernel.  Placement matters on MI355X: the same loop ran 12% slower
// with its first VALU instruction on an 8-byte boundary than 4 bytes past
// one, where the alignment directive before the loop label puts it here.
__device__ __forceinline__ void pair16_loop_r6_f32(uint32_t addr, int32_t cnt, float ui, float k, double& tot) {
    asm volatile(
        ".p2align 6\n"
        "s_nop 0\n"
        "s_nop 0\n"
        "s_nop 0\n"
        "s_nop 0\n"
        "1:\n"
        "v_mov_b32_e32 v45, %[addr]\n"
        "ds_read_b128 v[40:43], v45\n"
        "ds_read_b128 v[46:49], v45 offset:16\n"
        "ds_read_b128 v[50:53], v45 offset:32\n"
        "ds_read_b128 v[54:57], v45 offset:48\n"
        "s_add_u32 %[addr], %[addr], 64\n"
        "s_waitcnt lgkmcnt(0)\n"
        "v_sub_f32_e32 v40, %[ui], v40\n"
        "v_sub_f32_e32 v41, %[ui], v41\n"
        "v_sub_f32_e32 v42, %[ui], v42\n"
        "v_sub_f32_e32 v43, %[ui], v43\n"
        "v_sub_f32_e32 v45, %[ui], v46\n"
        "v_sub_f32_e32 v46, %[ui], v47\n"
        "v_sub_f32_e32 v47, %[ui], v48\n"
        "v_sub_f32_e32 v48, %[ui], v49\n"
        "v_fmaak_f32 v40, v40, v40, 0xc0a00000\n"
        "v_fmaak_f32 v41, v41, v41, 0xc0a00000\n"
        "v_fmaak_f32 v42, v42, v42, 0xc0a00000\n"
        "v_fmaak_f32 v43, v43, v43, 0xc0a00000\n"
        "v_sub_f32_e32 v49, %[ui], v50\n"
        "v_sub_f32_e32 v50, %[ui], v51\n"
        "v_sub_f32_e32 v51, %[ui], v52\n"
        "v_sub_f32_e32 v52, %[ui], v53\n"
        "v_sub_f32_e32 v53, %[ui], v54\n"
        "v_sub_f32_e32 v54, %[ui], v55\n"
        "v_sub_f32_e32 v55, %[ui], v56\n"
        "v_sub_f32_e32 v56, %[ui], v57\n"
        "v_fmaak_f32 v45, v45, v45, 0xc0a00000\n"
        "v_fmaak_f32 v46, v46, v46, 0xc0a00000\n"
        "v_fmaak_f32 v47, v47, v47, 0xc0a00000\n"
        "v_fmaak_f32 v48, v48, v48, 0xc0a00000\n"
        "v_fmaak_f32 v57, v40, v40, 0xc1f00000\n"
        "v_fmaak_f32 v58, v41, v41, 0xc1f00000\n"
        "v_fmaak_f32 v59, v42, v42, 0xc1f00000\n"
        "v_fmaak_f32 v60, v43, v43, 0xc1f00000\n"
        "v_mul_f32_e64 v61, v40, -%[k]\n"
        "v_mul_f32_e64 v85, v41, -%[k]\n"
        "v_mul_f32_e64 v92, v42, -%[k]\n"
        "v_mul_f32_e64 v93, v43, -%[k]\n"
        "v_fmaak_f32 v49, v49, v49, 0xc0a00000\n"
        "v_fmaak_f32 v50, v50, v50, 0xc0a00000\n"
        "v_fmaak_f32 v51, v51, v51, 0xc0a00000\n"
        "v_fmaak_f32 v52, v52, v52, 0xc0a00000\n"
        "v_mul_f32_e64 v98, v45, -%[k]\n"
        "v_mul_f32_e64 v99, v46, -%[k]\n"
        "v_mul_f32_e64 v100, v47, -%[k]\n"
        "v_mul_f32_e64 v101, v48, -%[k]\n"
        "v_fmaak_f32 v40, v57, v40, 0xc2200000\n"
        "v_fmaak_f32 v41, v58, v41, 0xc2200000\n"
        "v_fmaak_f32 v42, v59, v42, 0xc2200000\n"
        "v_fmaak_f32 v43, v60, v43, 0xc2200000\n"
        "v_exp_f32_e32 v57, v61\n"
        "v_exp_f32_e32 v58, v85\n"
        "v_exp_f32_e32 v59, v92\n"
        "v_exp_f32_e32 v60, v93\n"
        "v_fmaak_f32 v53, v53, v53, 0xc0a00000\n"
        "v_fmaak_f32 v54, v54, v54, 0xc0a00000\n"
        "v_fmaak_f32 v55, v55, v55, 0xc0a00000\n"
        "v_fmaak_f32 v56, v56, v56, 0xc0a00000\n"
        "v_fmaak_f32 v94, v45, v45, 0xc1f00000\n"
        "v_fmaak_f32 v95, v46, v46, 0xc1f00000\n"
        "v_fmaak_f32 v96, v47, v47, 0xc1f00000\n"
        "v_fmaak_f32 v97, v48, v48, 0xc1f00000\n"
        "v_mul_f32_e64 v106, v49, -%[k]\n"
        "v_mul_f32_e64 v107, v50, -%[k]\n"
        "v_mul_f32_e64 v108, v51, -%[k]\n"
        "v_mul_f32_e64 v109, v52, -%[k]\n"
        "v_exp_f32_e32 v61, v98\n"
        "v_exp_f32_e32 v85, v99\n"
        "v_exp_f32_e32 v92, v100\n"
        "v_exp_f32_e32 v93, v101\n"
        "v_mul_f32_e64 v114, v53, -%[k]\n"
        "v_mul_f32_e64 v115, v54, -%[k]\n"
        "v_mul_f32_e64 v116, v55, -%[k]\n"
        "v_mul_f32_e64 v117, v56, -%[k]\n"
        "v_fmaak_f32 v45, v94, v45, 0xc2200000\n"
        "v_fmaak_f32 v46, v95, v46, 0xc2200000\n"
        "v_fmaak_f32 v47, v96, v47, 0xc2200000\n"
        "v_fmaak_f32 v48, v97, v48, 0xc2200000\n"
        "v_exp_f32_e32 v94, v106\n"
        "v_exp_f32_e32 v95, v107\n"
        "v_exp_f32_e32 v96, v108\n"
        "v_exp_f32_e32 v97, v109\n"
        "v_exp_f32_e32 v98, v114\n"
        "v_exp_f32_e32 v99, v115\n"
        "v_exp_f32_e32 v100, v116\n"
        "v_exp_f32_e32 v101, v117\n"
        "v_fmaak_f32 v102, v49, v49, 0xc1f00000\n"
        "v_fmaak_f32 v103, v50, v50, 0xc1f00000\n"
        "v_fmaak_f32 v104, v51, v51, 0xc1f00000\n"
        "v_fmaak_f32 v105, v52, v52, 0xc1f00000\n"
        "v_fma_f32 v40, v40, v57, 0\n"
        "v_fma_f32 v41, v41, v58, 0\n"
        "v_fma_f32 v42, v42, v59, 0\n"
        "v_fma_f32 v43, v43, v60, 0\n"
        "v_fmaak_f32 v110, v53, v53, 0xc1f00000\n"
        "v_fmaak_f32 v111, v54, v54, 0xc1f00000\n"
        "v_fmaak_f32 v112, v55, v55, 0xc1f00000\n"
        "v_fmaak_f32 v113, v56, v56, 0xc1f00000\n"
        "v_fmaak_f32 v49, v102, v49, 0xc2200000\n"
        "v_fmaak_f32 v50, v103, v50, 0xc2200000\n"
        "v_fmaak_f32 v51, v104, v51, 0xc2200000\n"
        "v_fmaak_f32 v52, v105, v52, 0xc2200000\n"
        "v_fmac_f32_e32 v40, v45, v61\n"
        "v_fmac_f32_e32 v41, v46, v85\n"
        "v_fmac_f32_e32 v42, v47, v92\n"
        "v_fmac_f32_e32 v43, v48, v93\n"
        "v_fmaak_f32 v53, v110, v53, 0xc2200000\n"
        "v_fmaak_f32 v54, v111, v54, 0xc2200000\n"
        "v_fmaak_f32 v55, v112, v55, 0xc2200000\n"
        "v_fmaak_f32 v56, v113, v56, 0xc2200000\n"
        "v_fmac_f32_e32 v40, v49, v94\n"
        "v_fmac_f32_e32 v41, v50, v95\n"
        "v_fmac_f32_e32 v42, v51, v96\n"
        "v_fmac_f32_e32 v43, v52, v97\n"
        "v_fmac_f32_e32 v40, v53, v98\n"
        "v_fmac_f32_e32 v41, v54, v99\n"
        "v_fmac_f32_e32 v42, v55, v100\n"
        "v_fmac_f32_e32 v43, v56, v101\n"
        "v_add_f32_e32 v40, v40, v41\n"
        "v_add_f32_e32 v41, v42, v43\n"
        "s_sub_u32 %[cnt], %[cnt], 1\n"
        "v_add_f32_e32 v40, v40, v41\n"
        "v_cvt_f64_f32_e32 v[40:41], v40\n"
        "s_cmp_lg_u32 %[cnt], 0\n"
        "v_add_f64 %[tot], %[tot], v[40:41]\n"
        "s_cbranch_scc1 1b\n"
        : [tot] "+{v[34:35]}"(tot), [addr] "+s"(addr), [cnt] "+s"(cnt)
        : [ui] "{v44}"(ui), [k] "s"(k)
        : "v40", "v41", "v42", "v43", "v45", "v46", "v47", "v48", "v49", "v50", "v51", "v52", "v53", "v54", "v55", "v56", "v57", "v58", "v59", "v60", "v61", "v85", "v92", "v93", "v94", "v95", "v96", "v97", "v98", "v99", "v100", "v101", "v102", "v103", "v104", "v105", "v106", "v107", "v108", "v109", "v110", "v111", "v112", "v113", "v114", "v115", "v116", "v117", "scc", "memory");
}

// The exact-k variant (KDE_FP32_COMP_EXACT) of the Step IV loop above:
// per pair d = ui - xj, Y = d d, a = fma(Y, k_hi, Y k_lo), e = 2^(-a),
// p = ((Y - 15) Y + 45) Y - 15, column c into accumulator c, the same fold.
// The compiler's own code for the step, registers included, written out
// whole for the same reason: left to the compiler, its schedule moved with
// unrelated changes to the kernel and ran 20% slower.
__device__ __forceinline__ void pair16_loop_r6x_f32(uint32_t addr, int32_t cnt, float ui, float khi, float klo,
                                                 double& tot) {
    asm volatile(
        ".p2align 6\n"
        "s_nop 0\n"
        "s_nop 0\n"
        "s_nop 0\n"
        "s_nop 0\n"
        "1:\n"
        "v_mov_b32_e32 v43, %[addr]\n"
        "ds_read_b128 v[38:41], v43\n"
        "ds_read_b128 v[44:47], v43 offset:16\n"
        "ds_read_b128 v[48:51], v43 offset:32\n"
        "ds_read_b128 v[52:55], v43 offset:48\n"
        "s_add_u32 %[addr], %[addr], 64\n"
        "s_waitcnt lgkmcnt(0)\n"
        "v_sub_f32_e32 v38, %[ui], v38\n"
        "v_sub_f32_e32 v39, %[ui], v39\n"
        "v_sub_f32_e32 v40, %[ui], v40\n"
        "v_sub_f32_e32 v41, %[ui], v41\n"
        "v_sub_f32_e32 v43, %[ui], v44\n"
        "v_sub_f32_e32 v44, %[ui], v45\n"
        "v_sub_f32_e32 v45, %[ui], v46\n"
        "v_sub_f32_e32 v46, %[ui], v47\n"
        "v_sub_f32_e32 v47, %[ui], v48\n"
        "v_sub_f32_e32 v48, %[ui], v49\n"
        "v_sub_f32_e32 v49, %[ui], v50\n"
        "v_sub_f32_e32 v50, %[ui], v51\n"
        "v_sub_f32_e32 v51, %[ui], v52\n"
        "v_sub_f32_e32 v52, %[ui], v53\n"
        "v_sub_f32_e32 v53, %[ui], v54\n"
        "v_sub_f32_e32 v54, %[ui], v55\n"
        "v_mul_f32_e32 v55, v38, v38\n"
        "v_mul_f32_e32 v56, v39, v39\n"
        "v_mul_f32_e32 v57, v40, v40\n"
        "v_mul_f32_e32 v58, v41, v41\n"
        "v_fmaak_f32 v38, v38, v38, 0xc1700000\n"
        "v_fmaak_f32 v39, v39, v39, 0xc1700000\n"
        "v_fmaak_f32 v40, v40, v40, 0xc1700000\n"
        "v_fmaak_f32 v41, v41, v41, 0xc1700000\n"
        "v_mul_f32_e32 v59, v43, v43\n"
        "v_mul_f32_e32 v83, v44, v44\n"
        "v_mul_f32_e32 v90, v45, v45\n"
        "v_mul_f32_e32 v91, v46, v46\n"
        "v_mul_f32_e32 v100, %[klo], v55\n"
        "v_mul_f32_e32 v101, %[klo], v56\n"
        "v_mul_f32_e32 v102, %[klo], v57\n"
        "v_mul_f32_e32 v103, %[klo], v58\n"
        "v_fmaak_f32 v43, v43, v43, 0xc1700000\n"
        "v_fmaak_f32 v44, v44, v44, 0xc1700000\n"
        "v_fmaak_f32 v45, v45, v45, 0xc1700000\n"
        "v_fmaak_f32 v46, v46, v46, 0xc1700000\n"
        "v_mul_f32_e32 v92, v47, v47\n"
        "v_mul_f32_e32 v93, v48, v48\n"
        "v_mul_f32_e32 v94, v49, v49\n"
        "v_mul_f32_e32 v95, v50, v50\n"
        "v_fmaak_f32 v38, v38, v55, 0x42340000\n"
        "v_fmaak_f32 v39, v39, v56, 0x42340000\n"
        "v_fmaak_f32 v40, v40, v57, 0x42340000\n"
        "v_fmaak_f32 v41, v41, v58, 0x42340000\n"
        "v_mul_f32_e32 v104, %[klo], v59\n"
        "v_mul_f32_e32 v105, %[klo], v83\n"
        "v_mul_f32_e32 v106, %[klo], v90\n"
        "v_mul_f32_e32 v107, %[klo], v91\n"
        "v_fmac_f32_e32 v100, %[khi], v55\n"
        "v_fmac_f32_e32 v101, %[khi], v56\n"
        "v_fmac_f32_e32 v102, %[khi], v57\n"
        "v_fmac_f32_e32 v103, %[khi], v58\n"
        "v_fmaak_f32 v47, v47, v47, 0xc1700000\n"
        "v_fmaak_f32 v48, v48, v48, 0xc1700000\n"
        "v_fmaak_f32 v49, v49, v49, 0xc1700000\n"
        "v_fmaak_f32 v50, v50, v50, 0xc1700000\n"
        "v_mul_f32_e32 v96, v51, v51\n"
        "v_mul_f32_e32 v97, v52, v52\n"
        "v_mul_f32_e32 v98, v53, v53\n"
        "v_mul_f32_e32 v99, v54, v54\n"
        "v_fmaak_f32 v43, v43, v59, 0x42340000\n"
        "v_fmaak_f32 v44, v44, v83, 0x42340000\n"
        "v_fmaak_f32 v45, v45, v90, 0x42340000\n"
        "v_fmaak_f32 v46, v46, v91, 0x42340000\n"
        "v_mul_f32_e32 v108, %[klo], v92\n"
        "v_mul_f32_e32 v109, %[klo], v93\n"
        "v_mul_f32_e32 v110, %[klo], v94\n"
        "v_mul_f32_e32 v111, %[klo], v95\n"
        "v_fmaak_f32 v38, v38, v55, 0xc1700000\n"
        "v_fmaak_f32 v39, v39, v56, 0xc1700000\n"
        "v_fmaak_f32 v40, v40, v57, 0xc1700000\n"
        "v_fmaak_f32 v41, v41, v58, 0xc1700000\n"
        "v_fmac_f32_e32 v104, %[khi], v59\n"
        "v_fmac_f32_e32 v105, %[khi], v83\n"
        "v_fmac_f32_e32 v106, %[khi], v90\n"
        "v_fmac_f32_e32 v107, %[khi], v91\n"
        "v_exp_f32_e64 v55, -v100\n"
        "v_exp_f32_e64 v56, -v101\n"
        "v_exp_f32_e64 v57, -v102\n"
        "v_exp_f32_e64 v58, -v103\n"
        "v_fmaak_f32 v51, v51, v51, 0xc1700000\n"
        "v_fmaak_f32 v52, v52, v52, 0xc1700000\n"
        "v_fmaak_f32 v53, v53, v53, 0xc1700000\n"
        "v_fmaak_f32 v54, v54, v54, 0xc1700000\n"
        "v_fmaak_f32 v47, v47, v92, 0x42340000\n"
        "v_fmaak_f32 v48, v48, v93, 0x42340000\n"
        "v_fmaak_f32 v49, v49, v94, 0x42340000\n"
        "v_fmaak_f32 v50, v50, v95, 0x42340000\n"
        "v_mul_f32_e32 v112, %[klo], v96\n"
        "v_mul_f32_e32 v113, %[klo], v97\n"
        "v_mul_f32_e32 v114, %[klo], v98\n"
        "v_mul_f32_e32 v115, %[klo], v99\n"
        "v_fmaak_f32 v43, v43, v59, 0xc1700000\n"
        "v_fmaak_f32 v44, v44, v83, 0xc1700000\n"
        "v_fmaak_f32 v45, v45, v90, 0xc1700000\n"
        "v_fmaak_f32 v46, v46, v91, 0xc1700000\n"
        "v_fmac_f32_e32 v108, %[khi], v92\n"
        "v_fmac_f32_e32 v109, %[khi], v93\n"
        "v_fmac_f32_e32 v110, %[khi], v94\n"
        "v_fmac_f32_e32 v111, %[khi], v95\n"
        "v_exp_f32_e64 v59, -v104\n"
        "v_exp_f32_e64 v83, -v105\n"
        "v_exp_f32_e64 v90, -v106\n"
        "v_exp_f32_e64 v91, -v107\n"
        "v_fmaak_f32 v51, v51, v96, 0x42340000\n"
        "v_fmaak_f32 v52, v52, v97, 0x42340000\n"
        "v_fmaak_f32 v53, v53, v98, 0x42340000\n"
        "v_fmaak_f32 v54, v54, v99, 0x42340000\n"
        "v_fmaak_f32 v47, v47, v92, 0xc1700000\n"
        "v_fmaak_f32 v48, v48, v93, 0xc1700000\n"
        "v_fmaak_f32 v49, v49, v94, 0xc1700000\n"
        "v_fmaak_f32 v50, v50, v95, 0xc1700000\n"
        "v_fmac_f32_e32 v112, %[khi], v96\n"
        "v_fmac_f32_e32 v113, %[khi], v97\n"
        "v_fmac_f32_e32 v114, %[khi], v98\n"
        "v_fmac_f32_e32 v115, %[khi], v99\n"
        "v_exp_f32_e64 v92, -v108\n"
        "v_exp_f32_e64 v93, -v109\n"
        "v_exp_f32_e64 v94, -v110\n"
        "v_exp_f32_e64 v95, -v111\n"
        "v_fmaak_f32 v51, v51, v96, 0xc1700000\n"
        "v_fmaak_f32 v52, v52, v97, 0xc1700000\n"
        "v_fmaak_f32 v53, v53, v98, 0xc1700000\n"
        "v_fmaak_f32 v54, v54, v99, 0xc1700000\n"
        "v_exp_f32_e64 v96, -v112\n"
        "v_exp_f32_e64 v97, -v113\n"
        "v_exp_f32_e64 v98, -v114\n"
        "v_exp_f32_e64 v99, -v115\n"
        "v_fma_f32 v38, v38, v55, 0\n"
        "v_fma_f32 v39, v39, v56, 0\n"
        "v_fma_f32 v40, v40, v57, 0\n"
        "v_fma_f32 v41, v41, v58, 0\n"
        "v_fmac_f32_e32 v38, v43, v59\n"
        "v_fmac_f32_e32 v39, v44, v83\n"
        "v_fmac_f32_e32 v40, v45, v90\n"
        "v_fmac_f32_e32 v41, v46, v91\n"
        "v_fmac_f32_e32 v38, v47, v92\n"
        "v_fmac_f32_e32 v39, v48, v93\n"
        "v_fmac_f32_e32 v40, v49, v94\n"
        "v_fmac_f32_e32 v41, v50, v95\n"
        "v_fmac_f32_e32 v38, v51, v96\n"
        "v_fmac_f32_e32 v39, v52, v97\n"
        "v_fmac_f32_e32 v40, v53, v98\n"
        "v_fmac_f32_e32 v41, v54, v99\n"
        "v_add_f32_e32 v38, v38, v39\n"
        "v_add_f32_e32 v39, v40, v41\n"
        "s_sub_u32 %[cnt], %[cnt], 1\n"
        "v_add_f32_e32 v38, v38, v39\n"
        "v_cvt_f64_f32_e32 v[38:39], v38\n"
        "s_cmp_lg_u32 %[cnt], 0\n"
        "v_add_f64 %[tot], %[tot], v[38:39]\n"
        "s_cbranch_scc1 1b\n"
        : [tot] "+{v[32:33]}"(tot), [addr] "+s"(addr), [cnt] "+s"(cnt)
        : [ui] "{v42}"(ui), [khi] "s"(khi), [klo] "s"(klo)
        : "v38", "v39", "v40", "v41", "v43", "v44", "v45", "v46", "v47", "v48", "v49", "v50", "v51", "v52", "v53", "v54", "v55", "v56", "v57", "v58", "v59", "v83", "v90", "v91", "v92", "v93", "v94", "v95", "v96", "v97", "v98", "v99", "v100", "v101", "v102", "v103", "v104", "v105", "v106", "v107", "v108", "v109", "v110", "v111", "v112", "v113", "v114", "v115", "scc", "memory");
}

// The exact-k variant of the Step VI loop: as above with
// p = (Y - 6) Y + 3.
__device__ __forceinline__ void pair16_loop_r4x_f32(uint32_t addr, int32_t cnt, float ui, float khi, float klo,
                                                 double& tot) {
    asm volatile(
        ".p2align 6\n"
        "s_nop 0\n"
        "s_nop 0\n"
        "s_nop 0\n"
        "s_nop 0\n"
        "1:\n"
        "v_mov_b32_e32 v43, %[addr]\n"
        "ds_read_b128 v[38:41], v43\n"
        "ds_read_b128 v[44:47], v43 offset:16\n"
        "ds_read_b128 v[48:51], v43 offset:32\n"
        "ds_read_b128 v[52:55], v43 offset:48\n"
        "s_add_u32 %[addr], %[addr], 64\n"
        "s_waitcnt lgkmcnt(0)\n"
        "v_sub_f32_e32 v38, %[ui], v38\n"
        "v_sub_f32_e32 v39, %[ui], v39\n"
        "v_sub_f32_e32 v40, %[ui], v40\n"
        "v_sub_f32_e32 v41, %[ui], v41\n"
        "v_sub_f32_e32 v43, %[ui], v44\n"
        "v_sub_f32_e32 v44, %[ui], v45\n"
        "v_sub_f32_e32 v45, %[ui], v46\n"
        "v_sub_f32_e32 v46, %[ui], v47\n"
        "v_sub_f32_e32 v47, %[ui], v48\n"
        "v_sub_f32_e32 v48, %[ui], v49\n"
        "v_sub_f32_e32 v49, %[ui], v50\n"
        "v_sub_f32_e32 v50, %[ui], v51\n"
        "v_sub_f32_e32 v51, %[ui], v52\n"
        "v_sub_f32_e32 v52, %[ui], v53\n"
        "v_sub_f32_e32 v53, %[ui], v54\n"
        "v_sub_f32_e32 v54, %[ui], v55\n"
        "v_mul_f32_e32 v55, v38, v38\n"
        "v_mul_f32_e32 v56, v39, v39\n"
        "v_mul_f32_e32 v57, v40, v40\n"
        "v_mul_f32_e32 v58, v41, v41\n"
        "v_mul_f32_e32 v59, v43, v43\n"
        "v_mul_f32_e32 v83, v44, v44\n"
        "v_mul_f32_e32 v90, v45, v45\n"
        "v_mul_f32_e32 v91, v46, v46\n"
        "v_mul_f32_e32 v100, %[klo], v55\n"
        "v_mul_f32_e32 v101, %[klo], v56\n"
        "v_mul_f32_e32 v102, %[klo], v57\n"
        "v_mul_f32_e32 v103, %[klo], v58\n"
        "v_fmaak_f32 v38, v38, v38, 0xc0c00000\n"
        "v_fmaak_f32 v39, v39, v39, 0xc0c00000\n"
        "v_fmaak_f32 v40, v40, v40, 0xc0c00000\n"
        "v_fmaak_f32 v41, v41, v41, 0xc0c00000\n"
        "v_mul_f32_e32 v92, v47, v47\n"
        "v_mul_f32_e32 v93, v48, v48\n"
        "v_mul_f32_e32 v94, v49, v49\n"
        "v_mul_f32_e32 v95, v50, v50\n"
        "v_mul_f32_e32 v104, %[klo], v59\n"
        "v_mul_f32_e32 v105, %[klo], v83\n"
        "v_mul_f32_e32 v106, %[klo], v90\n"
        "v_mul_f32_e32 v107, %[klo], v91\n"
        "v_fmac_f32_e32 v100, %[khi], v55\n"
        "v_fmac_f32_e32 v101, %[khi], v56\n"
        "v_fmac_f32_e32 v102, %[khi], v57\n"
        "v_fmac_f32_e32 v103, %[khi], v58\n"
        "v_fmaak_f32 v43, v43, v43, 0xc0c00000\n"
        "v_fmaak_f32 v44, v44, v44, 0xc0c00000\n"
        "v_fmaak_f32 v45, v45, v45, 0xc0c00000\n"
        "v_fmaak_f32 v46, v46, v46, 0xc0c00000\n"
        "v_mul_f32_e32 v96, v51, v51\n"
        "v_mul_f32_e32 v97, v52, v52\n"
        "v_mul_f32_e32 v98, v53, v53\n"
        "v_mul_f32_e32 v99, v54, v54\n"
        "v_fmaak_f32 v38, v38, v55, 0x40400000\n"
        "v_fmaak_f32 v39, v39, v56, 0x40400000\n"
        "v_fmaak_f32 v40, v40, v57, 0x40400000\n"
        "v_fmaak_f32 v41, v41, v58, 0x40400000\n"
        "v_mul_f32_e32 v108, %[klo], v92\n"
        "v_mul_f32_e32 v109, %[klo], v93\n"
        "v_mul_f32_e32 v110, %[klo], v94\n"
        "v_mul_f32_e32 v111, %[klo], v95\n"
        "v_fmac_f32_e32 v104, %[khi], v59\n"
        "v_fmac_f32_e32 v105, %[khi], v83\n"
        "v_fmac_f32_e32 v106, %[khi], v90\n"
        "v_fmac_f32_e32 v107, %[khi], v91\n"
        "v_exp_f32_e64 v55, -v100\n"
        "v_exp_f32_e64 v56, -v101\n"
        "v_exp_f32_e64 v57, -v102\n"
        "v_exp_f32_e64 v58, -v103\n"
        "v_fmaak_f32 v47, v47, v47, 0xc0c00000\n"
        "v_fmaak_f32 v48, v48, v48, 0xc0c00000\n"
        "v_fmaak_f32 v49, v49, v49, 0xc0c00000\n"
        "v_fmaak_f32 v50, v50, v50, 0xc0c00000\n"
        "v_fmaak_f32 v43, v43, v59, 0x40400000\n"
        "v_fmaak_f32 v44, v44, v83, 0x40400000\n"
        "v_fmaak_f32 v45, v45, v90, 0x40400000\n"
        "v_fmaak_f32 v46, v46, v91, 0x40400000\n"
        "v_mul_f32_e32 v112, %[klo], v96\n"
        "v_mul_f32_e32 v113, %[klo], v97\n"
        "v_mul_f32_e32 v114, %[klo], v98\n"
        "v_mul_f32_e32 v115, %[klo], v99\n"
        "v_fmac_f32_e32 v108, %[khi], v92\n"
        "v_fmac_f32_e32 v109, %[khi], v93\n"
        "v_fmac_f32_e32 v110, %[khi], v94\n"
        "v_fmac_f32_e32 v111, %[khi], v95\n"
        "v_exp_f32_e64 v59, -v104\n"
        "v_exp_f32_e64 v83, -v105\n"
        "v_exp_f32_e64 v90, -v106\n"
        "v_exp_f32_e64 v91, -v107\n"
        "v_fmaak_f32 v51, v51, v51, 0xc0c00000\n"
        "v_fmaak_f32 v52, v52, v52, 0xc0c00000\n"
        "v_fmaak_f32 v53, v53, v53, 0xc0c00000\n"
        "v_fmaak_f32 v54, v54, v54, 0xc0c00000\n"
        "v_fmaak_f32 v47, v47, v92, 0x40400000\n"
        "v_fmaak_f32 v48, v48, v93, 0x40400000\n"
        "v_fmaak_f32 v49, v49, v94, 0x40400000\n"
        "v_fmaak_f32 v50, v50, v95, 0x40400000\n"
        "v_fmac_f32_e32 v112, %[khi], v96\n"
        "v_fmac_f32_e32 v113, %[khi], v97\n"
        "v_fmac_f32_e32 v114, %[khi], v98\n"
        "v_fmac_f32_e32 v115, %[khi], v99\n"
        "v_exp_f32_e64 v92, -v108\n"
        "v_exp_f32_e64 v93, -v109\n"
        "v_exp_f32_e64 v94, -v110\n"
        "v_exp_f32_e64 v95, -v111\n"
        "v_fmaak_f32 v51, v51, v96, 0x40400000\n"
        "v_fmaak_f32 v52, v52, v97, 0x40400000\n"
        "v_fmaak_f32 v53, v53, v98, 0x40400000\n"
        "v_fmaak_f32 v54, v54, v99, 0x40400000\n"
        "v_exp_f32_e64 v96, -v112\n"
        "v_exp_f32_e64 v97, -v113\n"
        "v_exp_f32_e64 v98, -v114\n"
        "v_exp_f32_e64 v99, -v115\n"
        "v_fma_f32 v38, v38, v55, 0\n"
        "v_fma_f32 v39, v39, v56, 0\n"
        "v_fma_f32 v40, v40, v57, 0\n"
        "v_fma_f32 v41, v41, v58, 0\n"
        "v_fmac_f32_e32 v38, v43, v59\n"
        "v_fmac_f32_e32 v39, v44, v83\n"
        "v_fmac_f32_e32 v40, v45, v90\n"
        "v_fmac_f32_e32 v41, v46, v91\n"
        "v_fmac_f32_e32 v38, v47, v92\n"
        "v_fmac_f32_e32 v39, v48, v93\n"
        "v_fmac_f32_e32 v40, v49, v94\n"
        "v_fmac_f32_e32 v41, v50, v95\n"
        "v_fmac_f32_e32 v38, v51, v96\n"
        "v_fmac_f32_e32 v39, v52, v97\n"
        "v_fmac_f32_e32 v40, v53, v98\n"
        "v_fmac_f32_e32 v41, v54, v99\n"
        "v_add_f32_e32 v38, v38, v39\n"
        "v_add_f32_e32 v39, v40, v41\n"
        "s_sub_u32 %[cnt], %[cnt], 1\n"
        "v_add_f32_e32 v38, v38, v39\n"
        "v_cvt_f64_f32_e32 v[38:39], v38\n"
        "s_cmp_lg_u32 %[cnt], 0\n"
        "v_add_f64 %[tot], %[tot], v[38:39]\n"
        "s_cbranch_scc1 1b\n"
        : [tot] "+{v[32:33]}"(tot), [addr] "+s"(addr), [cnt] "+s"(cnt)
        : [ui] "{v42}"(ui), [khi] "s"(khi), [klo] "s"(klo)
        : "v38", "v39", "v40", "v41", "v43", "v44", "v45", "v46", "v47", "v48", "v49", "v50", "v51", "v52", "v53", "v54", "v55", "v56", "v57", "v58", "v59", "v83", "v90", "v91", "v92", "v93", "v94", "v95", "v96", "v97", "v98", "v99", "v100", "v101", "v102", "v103", "v104", "v105", "v106", "v107", "v108", "v109", "v110", "v111", "v112", "v113", "v114", "v115", "scc", "memory");
}

// Columns [c0, c1) of pair item cb of the row block starting at row r0
// (row_chunks gives the chunk width; the host enumerates items with it).
__device__ __forceinline__ void item_columns(int64_t n, int64_t r0, int64_t W, int32_t cb,
                                             int64_t* c0, int64_t* c1) {
    int64_t m, w;
    row_chunks(n, r0, W, &m, &w);
    *c0 = r0 + (int64_t)cb * w;
    *c1 = min(*c0 + w, n);
}

// Generic centring offset of row block rb (see the header comment).
__device__ __forceinline__ double centre_offset(int32_t rb) {
    const double f = (double)rb * 0.6180339887498949;
    return 0.5 * (f - floor(f)) - 0.25;
}

// Column tiles are software-pipelined: the values of the next tile are
// loaded into registers (TJ / BLOCK per thread, all in flight together)
// while the current tile is evaluated, then converted and stored to LDS.
template <int BLOCK>
__device__ __forceinline__ void load_cols(const View& d, int64_t cj, int64_t c1, double (&v)[TJ / BLOCK]) {
#pragma unroll
    for (int q = 0; q < TJ / BLOCK; ++q) {
        const int64_t j = cj + threadIdx.x + (int64_t)q * BLOCK;
        v[q] = j < c1 ? load_x(d.x, d.dtype, j) : 0.0;
    }
}

template <typename T, int BLOCK>
__device__ __forceinline__ void store_cols(T* tile, const double (&v)[TJ / BLOCK], int len, double mean,
                                           double scale, double tau) {
#pragma unroll
    for (int q = 0; q < TJ / BLOCK; ++q) {
        const int e = threadIdx.x + q * BLOCK;
        if (e < len) tile[e] = (T)((v[q] - mean) * scale - tau);
    }
}

template <int RO, bool SAFE, bool EXACT_K, int R, int BLOCK, bool PEXP = false>
__device__ double pair_item_f32(const View& d, int32_t rb, int32_t cb, double mean, double scale,
                                const PolyConsts& pc, float* tile, double* red) {
    constexpr int TI = BLOCK * R;
    const double tau = centre_offset(rb);
    // the wave index is the same in all lanes of a wave: readfirstlane tells the
    // compiler so, and the column loops then run on scalar counters
    const int tid = threadIdx.x, lane = tid & (WAVE - 1);
    const int wave = __builtin_amdgcn_readfirstlane(tid / WAVE);
    const int64_t n = d.n;
    const int64_t r0 = (int64_t)rb * TI;
    const int64_t wlo = r0 + (int64_t)wave * WAVE * R;
    const int64_t whi = wlo + WAVE * R;

    float ui[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int64_t i = wlo + lane + (int64_t)WAVE * k;
        ui[k] = i < n ? (float)((load_x(d.x, d.dtype, i) - mean) * scale - tau) : 0.0f;
    }
    float acc[R][4];
    double tot[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        acc[k][0] = acc[k][1] = acc[k][2] = acc[k][3] = 0.0f;
        tot[k] = 0.0;
    }

    int64_t c0, c1;
    item_columns(n, r0, d.W, cb, &c0, &c1);
    double nv[TJ / BLOCK];
    load_cols<BLOCK>(d, c0, c1, nv);
    for (int64_t cj = c0; cj < c1; cj += TJ) {
        const int len = (int)min((int64_t)TJ, c1 - cj);
        __syncthreads();
        store_cols<float, BLOCK>(tile, nv, len, mean, scale, tau);
        __syncthreads();
        if (cj + TJ < c1) load_cols<BLOCK>(d, cj + TJ, c1, nv);

        // columns inside this wave's row span: only j > i counts
        const int64_t ma = max(cj, wlo + 1), mb = min(cj + (int64_t)len, whi);
        for (int64_t j = ma; j < mb; ++j) {
            const float uj = tile[j - cj];
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const float t = pair_term_f32<RO, SAFE, EXACT_K, PEXP>(ui[k], uj, pc);
                const bool live = j > wlo + lane + (int64_t)WAVE * k;
                tot[k] += live ? (double)t : 0.0;
            }
        }
        // columns right of this wave's rows: every pair counts
        const int64_t ua = max(cj, whi);
        if (ua < cj + len) {
            int jj = (int)(ua - cj);
            const float4* t4 = reinterpret_cast<const float4*>(tile);
            if constexpr ((RO == 4 || RO == 6) && R == 1 && !SAFE && !EXACT_K && !PEXP && kFold == 4) {
                // jj is a multiple of 64 here (row blocks, waves and chunk
                // starts all are), so the group reads are 16-byte aligned
                const int32_t groups = (len - jj) >> 4;
                if (groups > 0) {
                    const uint32_t lds = (uint32_t)(size_t)((__attribute__((address_space(3))) float*)tile) + 4u * (uint32_t)jj;
                    if constexpr (RO == 4) pair16_loop_r4_f32(lds, groups, ui[0], pc.k_hi, tot[0]);
                    else pair16_loop_r6_f32(lds, groups, ui[0], pc.k_hi, tot[0]);
                    jj += groups << 4;
                }
            } else if constexpr ((RO == 4 || RO == 6) && R == 1 && !SAFE && EXACT_K && !PEXP && kFold == 4) {
                const int32_t groups = (len - jj) >> 4;
                if (groups > 0) {
                    const uint32_t lds = (uint32_t)(size_t)((__attribute__((address_space(3))) float*)tile) + 4u * (uint32_t)jj;
                    if constexpr (RO == 4) pair16_loop_r4x_f32(lds, groups, ui[0], pc.k_hi, pc.k_lo, tot[0]);
                    else pair16_loop_r6x_f32(lds, groups, ui[0], pc.k_hi, pc.k_lo, tot[0]);
                    jj += groups << 4;
                }
            } else {
                for (; jj + 4 * kFold <= len; jj += 4 * kFold) {
#pragma unroll
                    for (int q = 0; q < kFold; ++q) pair_b128_f32<RO, SAFE, EXACT_K, R, PEXP>(ui, t4[(jj >> 2) + q], acc, pc);
                    fold_f64<R>(acc, tot);
                }
            }
            for (; jj + 4 <= len; jj += 4) pair_b128_f32<RO, SAFE, EXACT_K, R, PEXP>(ui, t4[jj >> 2], acc, pc);
            fold_f64<R>(acc, tot);
            for (; jj < len; ++jj) {
                const float uj = tile[jj];
#pragma unroll
                for (int k = 0; k < R; ++k) tot[k] += (double)pair_term_f32<RO, SAFE, EXACT_K, PEXP>(ui[k], uj, pc);
            }
        }
    }
    double lane_tot = 0.0;
#pragma unroll
    for (int k = 0; k < R; ++k) lane_tot += tot[k];
    return lane_tot;  // this lane's partial: the caller reduces over the block
}

// ---------------------------------------------------- FP64 pair evaluation
template <int RO>
__device__ __forceinline__ double pair_term_f64(double ui, double uj) {
    const double y = ui - uj;
    const double t = y * y;
    double p;
    if (RO == 6)
        p = ((t - 15.0) * t + 45.0) * t - 15.0;
    else
        p = (t - 6.0) * t + 3.0;
    return p * exp(-0.5 * t);
}

template <int RO, int R, int BLOCK>
__device__ double pair_item_f64(const View& d, int32_t rb, int32_t cb, double mean, double scale,
                                double* tile, double* red) {
    constexpr int TI = BLOCK * R;
    // the wave index is the same in all lanes of a wave: readfirstlane tells the
    // compiler so, and the column loops then run on scalar counters
    const int tid = threadIdx.x, lane = tid & (WAVE - 1);
    const int wave = __builtin_amdgcn_readfirstlane(tid / WAVE);
    const int64_t n = d.n;
    const int64_t r0 = (int64_t)rb * TI;
    const int64_t wlo = r0 + (int64_t)wave * WAVE * R;
    const int64_t whi = wlo + WAVE * R;

    double ui[R], acc[R][2];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int64_t i = wlo + lane + (int64_t)WAVE * k;
        ui[k] = i < n ? (load_x(d.x, d.dtype, i) - mean) * scale : 0.0;
        acc[k][0] = acc[k][1] = 0.0;
    }
    int64_t c0, c1;
    item_columns(n, r0, d.W, cb, &c0, &c1);
    double nv[TJ / BLOCK];
    load_cols<BLOCK>(d, c0, c1, nv);
    for (int64_t cj = c0; cj < c1; cj += TJ) {
        const int len = (int)min((int64_t)TJ, c1 - cj);
        __syncthreads();
        store_cols<double, BLOCK>(tile, nv, len, mean, scale, 0.0);
        __syncthreads();
        if (cj + TJ < c1) load_cols<BLOCK>(d, cj + TJ, c1, nv);
        const int64_t ma = max(cj, wlo + 1), mb = min(cj + (int64_t)len, whi);
        for (int64_t j = ma; j < mb; ++j) {
            const double uj = tile[j - cj];
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const double t = pair_term_f64<RO>(ui[k], uj);
                const bool live = j > wlo + lane + (int64_t)WAVE * k;
                acc[k][0] += live ? t : 0.0;
            }
        }
        const int64_t ua = max(cj, whi);
        if (ua < cj + len) {
            int jj = (int)(ua - cj);
            const double2* t2 = reinterpret_cast<const double2*>(tile);
            for (; jj + 2 <= len; jj += 2) {
                const double2 v = t2[jj >> 1];
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    acc[k][0] += pair_term_f64<RO>(ui[k], v.x);
                    acc[k][1] += pair_term_f64<RO>(ui[k], v.y);
                }
            }
            for (; jj < len; ++jj) {
                const double uj = tile[jj];
#pragma unroll
                for (int k = 0; k < R; ++k) acc[k][0] += pair_term_f64<RO>(ui[k], uj);
            }
        }
    }
    double lane_tot = 0.0;
#pragma unroll
    for (int k = 0; k < R; ++k) lane_tot += acc[k][0] + acc[k][1];
    return block_sum<BLOCK>(lane_tot, red);
}

// ---------------------------------------------- Q32.32 fixed point (emulation)
// The arithmetic of the paper's FPGA design (Section 4.2): z-scored samples
// and every pair-stage quantity in Q32.32, value = i / 2^32 in a signed 64-bit
// integer (sign, 31 integer and 32 fraction bits); products truncate (floor),
// sums are exact; the Gaussian factor comes from a minimax polynomial (Remez
// exchange) after range reduction.  Terms with |u| >= 16 are 0: their
// Gaussian factor is below 2^-128, far below Q32.32's resolution, and the
// polynomial would leave Q32.32's range.  Lane sums stay in Q32.32 (at most
// 15 times the lane's pairs, far inside 2^31); block sums are exact 64-bit
// integer sums, and the stage sum is the exact fixed-point accumulator.
using q32 = int64_t;
constexpr q32 kQOne = (q32)1 << 32;

__device__ __forceinline__ q32 q_mul(q32 a, q32 b) { return (q32)(((__int128)a * (__int128)b) >> 32); }

__device__ __forceinline__ q32 q_from(double v) { return (q32)floor(v * 4294967296.0); }

// 2^-a for a >= 0: a = n + f with n = round(a), 2^-a = 2^-n p(-f), -f in [-1/2, 1/2]
__device__ __forceinline__ q32 q_exp2_neg(q32 a) {
    const q32 n = (a + (kQOne >> 1)) >> 32;
    const q32 x = n * kQOne - a;
    q32 p = kExp2PolyQ[kExp2PolyQDegree];
#pragma unroll
    for (int k = kExp2PolyQDegree - 1; k >= 0; --k) p = q_mul(p, x) + kExp2PolyQ[k];
    return n >= 62 ? 0 : (p >> n);
}

template <int RO>
__device__ __forceinline__ q32 q_term(q32 zi, q32 zj, q32 ginv) {
    const q32 u = q_mul(zi - zj, ginv);
    if (u >= 16 * kQOne || u <= -16 * kQOne) return 0;
    const q32 t = q_mul(u, u);
    q32 p;
    if (RO == 6)
        p = q_mul(q_mul(t - 15 * kQOne, t) + 45 * kQOne, t) - 15 * kQOne;
    else
        p = q_mul(t - 6 * kQOne, t) + 3 * kQOne;
    // exp(-t/2) = 2^(-(t/2) log2(e))
    return q_mul(p, q_exp2_neg(q_mul(t >> 1, 2 * kQLog2eHalf)));
}

template <int BLOCK>
__device__ __forceinline__ q32 block_sum_q(q32 v, q32* red) {
#pragma unroll
    for (int off = WAVE / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
    const int lane = threadIdx.x & (WAVE - 1), wave = threadIdx.x / WAVE;
    if (lane == 0) red[wave] = v;
    __syncthreads();
    q32 tot = 0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int w = 0; w < BLOCK / WAVE; ++w) tot += red[w];
    }
    __syncthreads();
    return tot;  // valid in thread 0
}

// One pair item in Q32.32; returns the item's exact sum (thread 0).
template <int RO, int R, int BLOCK>
__device__ q32 pair_item_q32(const View& d, int32_t rb, int32_t cb, double mean, double scale, double sigma,
                             q32* tile, q32* red) {
    constexpr int TI = BLOCK * R;
    const int tid = threadIdx.x, lane = tid & (WAVE - 1);
    const int wave = __builtin_amdgcn_readfirstlane(tid / WAVE);
    const int64_t n = d.n;
    const int64_t r0 = (int64_t)rb * TI;
    const int64_t wlo = r0 + (int64_t)wave * WAVE * R;
    const int64_t whi = wlo + WAVE * R;
    // z-scores (the reciprocal of sigma, not a division) and the reciprocal
    // bandwidth in z units.  Psi_r(g) of a sample without spread (n = 1 or
    // ties only) has no z-score: its values are then taken in units of g.
    const double zs = sigma > 0.0 && isfinite(sigma) ? sigma : 1.0 / scale;
    const double inv_sigma = 1.0 / zs;
    const q32 ginv = q_from(zs * scale);

    q32 zi[R], acc[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int64_t i = wlo + lane + (int64_t)WAVE * k;
        zi[k] = i < n ? q_from((load_x(d.x, d.dtype, i) - mean) * inv_sigma) : 0;
        acc[k] = 0;
    }
    int64_t c0, c1;
    item_columns(n, r0, d.W, cb, &c0, &c1);
    for (int64_t cj = c0; cj < c1; cj += TJ) {
        const int len = (int)min((int64_t)TJ, c1 - cj);
        __syncthreads();
        for (int e = tid; e < len; e += BLOCK) tile[e] = q_from((load_x(d.x, d.dtype, cj + e) - mean) * inv_sigma);
        __syncthreads();
        const int64_t ma = max(cj, wlo + 1), mb = min(cj + (int64_t)len, whi);
        for (int64_t j = ma; j < mb; ++j) {
            const q32 zj = tile[j - cj];
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const q32 t = q_term<RO>(zi[k], zj, ginv);
                acc[k] += j > wlo + lane + (int64_t)WAVE * k ? t : 0;
            }
        }
        for (int64_t j = max(cj, whi); j < cj + len; ++j) {
            const q32 zj = tile[j - cj];
#pragma unroll
            for (int k = 0; k < R; ++k) acc[k] += q_term<RO>(zi[k], zj, ginv);
        }
    }
    q32 lane_tot = 0;
#pragma unroll
    for (int k = 0; k < R; ++k) lane_tot += acc[k];
    return block_sum_q<BLOCK>(lane_tot, red);
}

// ------------------------------------------------------------ finalisers
// Scalar formulas of Algorithm 1 in FP64, written in scale-free form so that
// samples with very large or small spread do not overflow sigma^9 or g^7:
//   g1 = sigma (-2 K6(0) 32 sqrt(pi) / (105 n))^(1/9)          (Steps II-III)
//   g2 = g1 (-2 K4(0) n / A6)^(1/7),  A6 = 2 S6 + n K6(0)       (Steps IV-V)
//   h  = g2 (R(K) n / A4)^(1/5),      A4 = 2 S4 + n K4(0)       (Steps VI-VII)
// which are the printed formulas with Psi8, Psi6(g1), Psi4(g2) substituted.
// Values of earlier stages a finaliser needs, loaded together as soon as it
// knows it is the finaliser.
struct Prior {
    int32_t status, safe;
    double g1, g2, maxdev, mean, scale;
};

__device__ __forceinline__ Prior load_prior(State* st) {
    Prior p;
    p.status = ld_i32(&st->status);
    p.safe = __hip_atomic_load(&st->safe, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    p.g1 = ld_f64(&st->g1);
    p.g2 = ld_f64(&st->g2);
    p.maxdev = ld_f64(&st->maxdev);
    p.mean = ld_f64(&st->mean);
    p.scale = ld_f64(&st->scale);
    return p;
}

// What a finaliser publishes to the items of later stages.
struct Published {
    int32_t status, safe;
    double mean, scale;
};

template <int PREC>
__device__ Published finalize_stage(const View& d, State* st, int32_t stage, double tot, double aux,
                                    const Prior& pr, const PolyConsts& pc) {
    const double pi = 3.14159265358979323846;
    const double rt2pi = sqrt(2.0 * pi);
    const double K6_0 = -15.0 / rt2pi, K4_0 = 3.0 / rt2pi, RK = 1.0 / (2.0 * sqrt(pi));
    const double nd = (double)d.n;
    int32_t status = pr.status;
    Published out{pr.status, pr.safe, pr.mean, pr.scale};
    switch (stage) {
    case ST_SUM: {
        if (!isfinite(tot)) { set_status(st, KDE_ENONFINITE); status = KDE_ENONFINITE; }
        out.mean = tot / nd;
        st_f64(&st->mean, out.mean);
        break;
    }
    case ST_SSQ: {
        const double sigma = sqrt(tot / (nd - 1.0));
        st_f64(&st->sigma, sigma);
        st_f64(&st->maxdev, aux);
        // sigma = 0 makes Psi8 of Step II infinite: only the full selection
        // needs it.  For Psi_r(g) with a given g, Step I only centres the
        // data, and n = 1 or a sample of ties is an ordinary input whose
        // pairs are K(0) terms (equations (6)-(7)).
        if (d.mode == MODE_PLUGIN && status == 0 && !(sigma > 0.0 && isfinite(sigma))) {
            set_status(st, KDE_EDEGENERATE);
            status = KDE_EDEGENERATE;
        }
        double g;
        if (d.mode == MODE_PLUGIN) {
            st_f64(&st->psi8, 105.0 / (32.0 * sqrt(pi) * pow(sigma, 9.0)));
            g = sigma * pow(-2.0 * K6_0 * 32.0 * sqrt(pi) / (105.0 * nd), 1.0 / 9.0);
            st_f64(&st->g1, g);
        } else {
            g = d.psi_g;
        }
        out.scale = 1.0 / g;
        out.safe = aux * out.scale > kSafeLimit ? 1 : 0;
        st_f64(&st->scale, out.scale);
        __hip_atomic_store(&st->safe, out.safe, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
    }
    case ST_PSI6: {
        // the default FP32 path evaluates Step IV with exp2(-k Z), Z = Y - 5
        const double S6 = (PREC == 1 || PREC == 3 ? exp2(-5.0 * (double)pc.k_hi) : 1.0) * tot / rt2pi;
        st_f64(&st->S6, S6);
        const double A6 = 2.0 * S6 + nd * K6_0;
        const double g1 = d.mode == MODE_PLUGIN ? pr.g1 : d.psi_g;
        st_f64(&st->psi6, A6 / (nd * nd * pow(g1, 7.0)));
        if (d.mode == MODE_PLUGIN) {
            if (status == 0 && !(A6 < 0.0)) { set_status(st, KDE_EDEGENERATE); status = KDE_EDEGENERATE; }
            const double g2 = g1 * pow(-2.0 * K4_0 * nd / A6, 1.0 / 7.0);
            st_f64(&st->g2, g2);
            out.scale = 1.0 / g2;
            out.safe = pr.maxdev * out.scale > kSafeLimit ? 1 : 0;
            st_f64(&st->scale, out.scale);
            __hip_atomic_store(&st->safe, out.safe, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        break;
    }
    case ST_PSI4: {
        const double S4 = tot / rt2pi;
        st_f64(&st->S4, S4);
        const double A4 = 2.0 * S4 + nd * K4_0;
        const double g2 = d.mode == MODE_PLUGIN ? pr.g2 : d.psi_g;
        st_f64(&st->psi4, A4 / (nd * nd * pow(g2, 5.0)));
        if (d.mode == MODE_PLUGIN) {
            if (status == 0 && !(A4 > 0.0)) { set_status(st, KDE_EDEGENERATE); status = KDE_EDEGENERATE; }
            st_f64(&st->h, g2 * pow(RK * nd / A4, 1.0 / 5.0));
        }
        break;
    }
    default:
        break;
    }
    out.status = status;
    return out;
}

// --------------------------------------------------------------- kernels
__global__ void k_init(State* states, Pub* pubs, int32_t count, uint32_t* ticket) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) {
        State s = {};
        states[i] = s;
    }
    if (i < (int64_t)count * kPubReplicas) {
        Pub q = {};
        pubs[i] = q;
    }
    if (i == 0) *ticket = 0u;
}

// Exact accumulation of pair-item partials.  A partial v with |v| < 2^62 is
// taken as the integer V = trunc(v 2^64) (two's complement over 128 bits),
// cut into four 32-bit limbs, the top one signed, and each limb is added
// into its own 64-bit integer: below 2^31 additions nothing overflows, and
// the exact total is recovered by carrying once at the end.  The truncation
// costs at most 2^-64 per item.
constexpr double kFxLimit = 4611686018427387904.0;  // 2^62

__device__ __forceinline__ void fx_add(int64_t (&acc)[4], double v) {
    const uint64_t bits = (uint64_t)__double_as_longlong(v);
    const int e = (int)((bits >> 52) & 0x7ff);
    if (e == 0) return;  // zero or below 2^-1022: truncates to 0
    const uint64_t mant = (bits & 0xfffffffffffffull) | (1ull << 52);
    // v = mant 2^(e - 1075), so V = mant 2^s with s = e - 1011
    const int sh = e - 1011;
    uint64_t lo, hi;
    if (sh <= -53) {
        return;
    } else if (sh < 0) {
        lo = mant >> (-sh);
        hi = 0;
    } else if (sh == 0) {
        lo = mant;
        hi = 0;
    } else if (sh < 64) {
        lo = mant << sh;
        hi = mant >> (64 - sh);
    } else {
        lo = 0;
        hi = mant << (sh - 64);  // sh < 74 since |v| < 2^62
    }
    if (bits >> 63) {
        lo = ~lo + 1ull;
        hi = ~hi + (lo == 0ull ? 1ull : 0ull);
    }
    acc[0] += (int64_t)(lo & 0xffffffffull);
    acc[1] += (int64_t)(lo >> 32);
    acc[2] += (int64_t)(hi & 0xffffffffull);
    acc[3] += (int64_t)(int32_t)(uint32_t)(hi >> 32);
}

// Exact accumulation of a Q32.32 partial v (value v / 2^32): V = v 2^32.
__device__ __forceinline__ void fx_add_q(int64_t (&acc)[4], int64_t v) {
    const __int128 V = (__int128)v << 32;
    const uint64_t lo = (uint64_t)V, hi = (uint64_t)(V >> 64);
    acc[0] += (int64_t)(lo & 0xffffffffull);
    acc[1] += (int64_t)(lo >> 32);
    acc[2] += (int64_t)(hi & 0xffffffffull);
    acc[3] += (int64_t)(int32_t)(uint32_t)(hi >> 32);
}

// The value of accumulated limbs, rounded to FP64.
__device__ __forceinline__ double fx_value(const int64_t (&a)[4]) {
    const __int128 V = ((__int128)a[3] << 96) + ((__int128)a[2] << 64) + ((__int128)a[1] << 32) + (__int128)a[0];
    const int64_t hi = (int64_t)(V >> 64);
    const uint64_t lo = (uint64_t)V;
    return (double)hi + ldexp((double)lo, -64);
}

// Completion of `cnt` items of one (sample, stage) whose slots this block
// has written: one release read-modify-write on the stage's counter.  The
// block that brings the counter to the stage's item count merges Step I's
// chunks (first stage) or reads the exact pair sum, and runs the stage's
// scalar formulas.
template <int PREC, int BLOCK>
__device__ void complete_items(const LaunchArgs& A, int32_t ds, const View& d, State* st, int32_t stage,
                               uint32_t cnt, int64_t (&pacc)[4], double* red, int32_t* sh_last,
                               Published* pub) {
    const int tid = threadIdx.x;
    if (tid == 0) {
        if (stage >= ST_PSI6) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (pacc[q] != 0)
                    __hip_atomic_fetch_add(&st->acc[stage - ST_PSI6][q], pacc[q], __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                pacc[q] = 0;
            }
        }
        const uint32_t old = __hip_atomic_fetch_add(&st->done[stage], cnt, __ATOMIC_RELEASE,
                                                    __HIP_MEMORY_SCOPE_AGENT);
        *sh_last = (old + cnt == (uint32_t)d.cnt) ? 1 : 0;
    }
    __syncthreads();
    // Step I's second stage has no work of its own: the first stage's
    // finaliser published it (its items only count)
    if (*sh_last && stage != ST_SSQ) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        Prior pr{};
        int64_t a[4] = {0, 0, 0, 0};
        if (tid == 0) {
            pr = load_prior(st);
            if (stage >= ST_PSI6)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    a[q] = __hip_atomic_load(&st->acc[stage - ST_PSI6][q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        double tot = 0.0, mx = 0.0, mean = 0.0;
        if (stage == ST_SUM) {
            // Step I: every thread merges a contiguous range of chunks in
            // index order, the lanes of a wave merge lower group with upper
            // group (both lanes of a pair compute the same merge), thread 0
            // the waves in order; then the largest deviation from the mean
            // from each chunk's minimum and maximum
            __shared__ double sm[3 * (BLOCK / WAVE)];
            const int64_t base = d.base, base2 = A.descs[ds].slot_base[ST_SSQ];
            const int32_t m = d.cnt, per = (m + BLOCK - 1) / BLOCK;
            const int32_t k0 = min(m, tid * per), k1 = min(m, k0 + per);
            double cn = 0.0, cm = 0.0, c2 = 0.0;
            for (int32_t k = k0; k < k1; ++k) {
                const Slot sl = A.slots[base + k];
                const double nk = (double)min((int64_t)d.chunk, d.n - (int64_t)k * d.chunk);
                chan_merge(cn, cm, c2, nk, sl.v / nk, sl.aux);
            }
#pragma unroll
            for (int off = 1; off < WAVE; off <<= 1) {
                const double on = __shfl_xor(cn, off, WAVE), om = __shfl_xor(cm, off, WAVE);
                const double o2 = __shfl_xor(c2, off, WAVE);
                if (tid & off) {
                    double ln = on, lm = om, l2 = o2;
                    chan_merge(ln, lm, l2, cn, cm, c2);
                    cn = ln;
                    cm = lm;
                    c2 = l2;
                } else {
                    chan_merge(cn, cm, c2, on, om, o2);
                }
            }
            if ((tid & (WAVE - 1)) == 0) {
                sm[3 * (tid / WAVE)] = cn;
                sm[3 * (tid / WAVE) + 1] = cm;
                sm[3 * (tid / WAVE) + 2] = c2;
            }
            __syncthreads();
            if (tid == 0) {
                double N = 0.0, M = 0.0, Q = 0.0;
                for (int w = 0; w < BLOCK / WAVE; ++w) chan_merge(N, M, Q, sm[3 * w], sm[3 * w + 1], sm[3 * w + 2]);
                sm[0] = load_x(d.x, d.dtype, 0) + M;  // the chunks' sums were taken about x[0]
                sm[1] = Q;
            }
            __syncthreads();
            mean = sm[0];
            tot = sm[1];
            double dm = 0.0;
            for (int32_t k = k0; k < k1; ++k) {
                const Slot sl = A.slots[base2 + k];
                dm = fmax(dm, fmax(sl.aux - mean, mean - sl.v));
            }
            mx = block_max<BLOCK>(dm, red);
        }
        if (tid == 0) {
            int32_t flag = stage;
            if (stage >= ST_PSI6) tot = fx_value(a);
            if (stage == ST_SUM) {
                // mean, then sigma and Steps II-III as the second stage's finaliser
                if (!(isfinite(mean) && isfinite(tot))) {
                    set_status(st, KDE_ENONFINITE);
                    pr.status = KDE_ENONFINITE;
                }
                st_f64(&st->mean, mean);
                pr.mean = mean;
                *pub = finalize_stage<PREC>(d, st, ST_SSQ, tot, mx, pr, A.pc);
                flag = ST_SSQ;
                const uint64_t now = wall_clock64();
                __hip_atomic_store(&st->t_fin[ST_SUM], now, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&st->t_fin[ST_SSQ], now, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                st_relaxed(&st->ready[ST_SUM], 1u);
            } else {
                *pub = finalize_stage<PREC>(d, st, stage, tot, mx, pr, A.pc);
                __hip_atomic_store(&st->t_fin[stage], (uint64_t)wall_clock64(), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            }
            // read by the host after the launch only; waiting blocks poll the
            // replicas below, whose release orders everything written here
            st_relaxed(&st->ready[flag], 1u);
        }
        __syncthreads();
        if (tid < kPubReplicas) {
            // every replica gets the values, then its flag(s) with release order
            Pub* q = A.pubs + (int64_t)ds * kPubReplicas + tid;
            __hip_atomic_store(&q->status, pub->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&q->safe, pub->safe, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            st_f64(&q->mean, pub->mean);
            st_f64(&q->scale, pub->scale);
            if (stage == ST_SUM) st_release(&q->ready[ST_SUM], 1u);
            st_release(&q->ready[stage == ST_SUM ? ST_SSQ : stage], 1u);
        }
    }
    __syncthreads();
}

// Memory-model cost on a multi-XCD device: an agent-scope release writes
// back the XCD's L2 and an agent-scope acquire invalidates it, for every CU of
// that XCD.  The loop therefore (i) takes tickets with a relaxed atomic,
// (ii) waits with relaxed polling and issues one acquire per (block, sample,
// stage) it has not seen published yet, caching the published scalars in
// LDS, and (iii) counts its finished items of one run of (sample, stage)
// items with a single release read-modify-write, as soon as its next ticket
// lies past the run (or there is none); only a stage's finaliser acquires
// the slots.
//
// A block takes its next ticket when it has finished an item, not when it
// starts one: the three blocks on a CU progress at different rates (the
// oldest waves issue first), and a ticket taken a whole item ahead by a slow
// block left that item waiting while faster blocks ran dry at the end of
// every stage.
//
// Progress.  A block holds uncounted items of one (sample, stage) only, and
// it counts them before it starts an item of another (sample, stage) (the
// run rule does so at the end of the run; the check at the top of the loop
// covers work lists whose runs are marked shorter).  So a block that waits
// for a stage flag holds no uncounted items, a block that does not wait
// finishes its item and takes the next ticket, and a block without tickets
// has counted everything: every stage counter reaches its item count and
// every flag is published.
template <int PREC, int R, int BLOCK, int WAVES>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(WAVES))) void k_persistent(LaunchArgs A) {
    using TileT = typename std::conditional<PREC >= 1 && PREC <= 3, float, double>::type;
    __shared__ __align__(16) TileT tile[TJ];
    __shared__ double red[BLOCK / WAVE];
    __shared__ uint32_t sh_ticket;
    __shared__ int32_t sh_status, sh_safe, sh_last, sh_flush;
    __shared__ int32_t sh_cds, sh_cwait;  // (sample, stage) whose published scalars are cached
    __shared__ double sh_mean, sh_scale;
    __shared__ Published sh_pub;  // a finaliser's values, for its replica writers

    const int tid = threadIdx.x;
    uint32_t next = 0;  // thread 0: the block's next ticket
    if (tid == 0) {
        next = atomicAdd(A.ticket, 1u);
        sh_cds = -1;
        sh_cwait = -1;
    }
    // finished items not yet counted (same values in every thread) and, in
    // LDS, their exact sum if they are pair items
    int32_t pend_ds = -1, pend_stage = 0;
    uint32_t pend_cnt = 0;
    __shared__ int64_t pacc[4];
    if (tid < 4) pacc[tid] = 0;
    // the view of the last item's (sample, stage): consecutive items of one
    // stage share it, so it is read again only when the pair changes
    View d = {};
    int32_t d_ds = -1, d_stage = -1;
    for (;;) {
        if (tid == 0) {
            sh_ticket = next;
        }
        __syncthreads();
        const uint32_t t = sh_ticket;
        const bool have = t < A.n_items;
        Item it = {};
        if (have) it = A.items[t];
        if (pend_cnt != 0u && (!have || it.ds != pend_ds || it.stage != pend_stage)) {
            complete_items<PREC, BLOCK>(A, pend_ds, load_view(A.descs + pend_ds, pend_stage),
                                        A.states + pend_ds, pend_stage, pend_cnt, pacc, red, &sh_last,
                                        &sh_pub);
            pend_cnt = 0u;
        }
        if (!have) break;

        if (it.ds != d_ds || it.stage != d_stage) {
            d = load_view(A.descs + it.ds, it.stage);
            d_ds = it.ds;
            d_stage = it.stage;
        }
        State* st = A.states + it.ds;

        if (tid == 0) {
            if (it.stage == ST_SUM && it.a == 0) {
                __hip_atomic_store(&st->t_first, (uint64_t)wall_clock64(), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            }
            if (it.wait < 0) {
                sh_status = ld_i32(&st->status);
            } else if (sh_cds != it.ds || sh_cwait != it.wait) {
                const Pub* q = A.pubs + (int64_t)it.ds * kPubReplicas + (blockIdx.x & (kPubReplicas - 1));
                const uint64_t t0 = wall_clock64();
                bool ready = true;
                for (uint32_t spin = 1;
                     __hip_atomic_load(&q->ready[it.wait], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u;
                     ++spin) {
                    __builtin_amdgcn_s_sleep(8);
                    if ((spin & 63u) == 0u &&
                        (ld_i32(&st->status) == KDE_ETIMEOUT || wall_clock64() - t0 > A.timeout_ticks)) {
                        set_status(st, KDE_ETIMEOUT);  // keeps an earlier status if one is set
                        ready = false;
                        break;
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                if (ready) {
                    sh_status = __hip_atomic_load(&q->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    sh_mean = ld_f64(&q->mean);
                    sh_scale = ld_f64(&q->scale);
                    sh_safe = __hip_atomic_load(&q->safe, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    sh_cds = it.ds;
                    sh_cwait = it.wait;
                } else {
                    sh_status = ld_i32(&st->status);  // nonzero: the item is skipped
                    sh_cds = -1;
                    sh_cwait = -1;
                }
            }
        }
        __syncthreads();
        const int32_t status = sh_status;
        const double mean = sh_mean, scale = sh_scale;
        const int32_t safe = sh_safe;

        double v = 0.0;
        bool lane_partial = false;  // v holds this lane's part of an FP32 pair item
        q32 vq = 0;  // Q32.32 item sum (fixed-point mode)
        if (status == 0) {
            switch (it.stage) {
            case ST_SUM: {
                // the chunk's (sum, squared deviations) in its own slot, its
                // (min, max) in the slot of the same chunk in the second stage
                double sum, m2, lo, hi;
                moment_stats<BLOCK>(d, it.a, red, &sum, &m2, &lo, &hi);
                if (tid == 0) {
                    A.slots[it.slot] = Slot{sum, m2};
                    A.slots[A.descs[it.ds].slot_base[ST_SSQ] + it.a] = Slot{lo, hi};
                }
                break;
            }
            case ST_SSQ:
                break;  // Step I's first finaliser has done this stage's work
            case ST_PSI6:
            case ST_PSI4:
                if constexpr (PREC == 4) {
                    // sigma was written by Step I's finaliser before the flag this item waited for
                    const double sigma = ld_f64(&st->sigma);
                    q32* tl = reinterpret_cast<q32*>(tile);
                    q32* rq = reinterpret_cast<q32*>(red);
                    vq = it.stage == ST_PSI6 ? pair_item_q32<6, R, BLOCK>(d, it.a, it.b, mean, scale, sigma, tl, rq)
                                             : pair_item_q32<4, R, BLOCK>(d, it.a, it.b, mean, scale, sigma, tl, rq);
                } else if constexpr (PREC >= 1) {
                    constexpr bool XK = PREC == 2;
                    constexpr bool PX = PREC == 3;
                    float* tl = reinterpret_cast<float*>(tile);
                    if (it.stage == ST_PSI6)
                        v = safe ? pair_item_f32<6, true, XK, R, BLOCK, PX>(d, it.a, it.b, mean, scale, A.pc, tl, red)
                                 : pair_item_f32<6, false, XK, R, BLOCK, PX>(d, it.a, it.b, mean, scale, A.pc, tl, red);
                    else
                        v = safe ? pair_item_f32<4, true, XK, R, BLOCK, PX>(d, it.a, it.b, mean, scale, A.pc, tl, red)
                                 : pair_item_f32<4, false, XK, R, BLOCK, PX>(d, it.a, it.b, mean, scale, A.pc, tl, red);
                    lane_partial = true;
                } else {
                    double* tl = reinterpret_cast<double*>(tile);
                    if (it.stage == ST_PSI6)
                        v = pair_item_f64<6, R, BLOCK>(d, it.a, it.b, mean, scale, tl, red);
                    else
                        v = pair_item_f64<4, R, BLOCK>(d, it.a, it.b, mean, scale, tl, red);
                }
                break;
            default:
                break;
            }
        }

        // the next ticket's round trip overlaps the block reduction of an
        // FP32 pair item
        if (tid == 0) next = atomicAdd(A.ticket, 1u);
        if (__builtin_amdgcn_readfirstlane(lane_partial)) v = block_sum<BLOCK>(v, red);
        if (tid == 0) {
            if (PREC == 4 && it.stage >= ST_PSI6) {
                fx_add_q(pacc, vq);
            } else if (it.stage >= ST_PSI6) {
                if (fabs(v) < kFxLimit)
                    fx_add(pacc, v);
                else if (status == 0)
                    set_status(st, KDE_EDEGENERATE);  // non-finite or out of range partial
            }
            sh_flush = next >= (uint32_t)it.run_end ? 1 : 0;
        }
        pend_ds = it.ds;
        pend_stage = it.stage;
        ++pend_cnt;
        __syncthreads();
        if (sh_flush) {
            complete_items<PREC, BLOCK>(A, it.ds, d, st, it.stage, pend_cnt, pacc, red, &sh_last, &sh_pub);
            pend_cnt = 0u;
        }
    }
}

// ---------------------------------------------------------- host entry
hipError_t launch_init(State* states, Pub* pubs, int32_t count, uint32_t* ticket, hipStream_t s) {
    const int threads = 256;
    const int64_t cover = (int64_t)count * kPubReplicas;
    const int blocks = cover > 0 ? (int)((cover + threads - 1) / threads) : 1;
    hipLaunchKernelGGL(k_init, dim3(blocks), dim3(threads), 0, s, states, pubs, count, ticket);
    return hipGetLastError();
}

// Results of an asynchronous batch call, written where the caller asked
// (device memory or pinned host memory): out[k] from state outmap[2k], or a
// sample the host rejected with status outmap[2k + 1].  The same fields as the
// host read-back fills, so both routes give the same bits.
__global__ void k_results(const State* states, const int32_t* outmap, int64_t n_out, kde_result* out) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_out) return;
    const int32_t q = outmap[2 * k];
    kde_result r = {};
    if (q < 0) {
        r.h = __longlong_as_double(0x7ff8000000000000ll);
        r.status = outmap[2 * k + 1];
    } else {
        const State& s = states[q];
        r.h = s.status ? __longlong_as_double(0x7ff8000000000000ll) : s.h;
        r.mean = s.mean;
        r.sigma = s.sigma;
        r.psi8 = s.psi8;
        r.g1 = s.g1;
        r.psi6 = s.psi6;
        r.g2 = s.g2;
        r.psi4 = s.psi4;
        r.status = s.status;
    }
    out[k] = r;
}

hipError_t launch_results(const State* states, const int32_t* outmap, int64_t n_out, kde_result* out,
                          hipStream_t s) {
    if (n_out <= 0) return hipSuccess;
    const int threads = 64;
    hipLaunchKernelGGL(k_results, dim3((unsigned)((n_out + threads - 1) / threads)), dim3(threads), 0, s, states,
                       outmap, n_out, out);
    return hipGetLastError();
}

template <int PREC, int R, int WAVES>
static hipError_t launch_one(int grid, hipStream_t s, const LaunchArgs& a) {
    hipLaunchKernelGGL((k_persistent<PREC, R, 256, WAVES>), dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <int PREC, int R, int WAVES>
static hipError_t occ_one(int* blocks) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k_persistent<PREC, R, 256, WAVES>, 256, 0);
}

// Every (precision, R) has a kernel held to three waves per SIMD (at most
// 168 VGPRs); the default precision at R = 1 also has one held to four (at
// most 128 VGPRs, some spilled outside the pair loops), the faster one for
// large samples.
bool wide_available(int prec, int R) { return prec == 1 && R == 1; }

hipError_t launch_persistent(int prec, int R, bool wide, int grid, hipStream_t s, const LaunchArgs& a) {
    if (wide) return wide_available(prec, R) ? launch_one<1, 1, 4>(grid, s, a) : hipErrorInvalidValue;
    switch (prec * 8 + R) {
    case 0 * 8 + 1: return launch_one<0, 1, 3>(grid, s, a);
    case 0 * 8 + 2: return launch_one<0, 2, 3>(grid, s, a);
    case 0 * 8 + 4: return launch_one<0, 4, 3>(grid, s, a);
    case 1 * 8 + 1: return launch_one<1, 1, 3>(grid, s, a);
    case 1 * 8 + 2: return launch_one<1, 2, 3>(grid, s, a);
    case 1 * 8 + 4: return launch_one<1, 4, 3>(grid, s, a);
    case 2 * 8 + 1: return launch_one<2, 1, 3>(grid, s, a);
    case 2 * 8 + 2: return launch_one<2, 2, 3>(grid, s, a);
    case 2 * 8 + 4: return launch_one<2, 4, 3>(grid, s, a);
    case 3 * 8 + 1: return launch_one<3, 1, 3>(grid, s, a);
    case 3 * 8 + 2: return launch_one<3, 2, 3>(grid, s, a);
    case 3 * 8 + 4: return launch_one<3, 4, 3>(grid, s, a);
    case 4 * 8 + 1: return launch_one<4, 1, 3>(grid, s, a);
    case 4 * 8 + 2: return launch_one<4, 2, 3>(grid, s, a);
    case 4 * 8 + 4: return launch_one<4, 4, 3>(grid, s, a);
    default: return hipErrorInvalidValue;
    }
}

const void* persistent_kernel(int prec, int R, bool wide) {
    if (wide) return wide_available(prec, R) ? (const void*)k_persistent<1, 1, 256, 4> : nullptr;
    switch (prec * 8 + R) {
    case 0 * 8 + 1: return (const void*)k_persistent<0, 1, 256, 3>;
    case 0 * 8 + 2: return (const void*)k_persistent<0, 2, 256, 3>;
    case 0 * 8 + 4: return (const void*)k_persistent<0, 4, 256, 3>;
    case 1 * 8 + 1: return (const void*)k_persistent<1, 1, 256, 3>;
    case 1 * 8 + 2: return (const void*)k_persistent<1, 2, 256, 3>;
    case 1 * 8 + 4: return (const void*)k_persistent<1, 4, 256, 3>;
    case 2 * 8 + 1: return (const void*)k_persistent<2, 1, 256, 3>;
    case 2 * 8 + 2: return (const void*)k_persistent<2, 2, 256, 3>;
    case 2 * 8 + 4: return (const void*)k_persistent<2, 4, 256, 3>;
    case 3 * 8 + 1: return (const void*)k_persistent<3, 1, 256, 3>;
    case 3 * 8 + 2: return (const void*)k_persistent<3, 2, 256, 3>;
    case 3 * 8 + 4: return (const void*)k_persistent<3, 4, 256, 3>;
    case 4 * 8 + 1: return (const void*)k_persistent<4, 1, 256, 3>;
    case 4 * 8 + 2: return (const void*)k_persistent<4, 2, 256, 3>;
    case 4 * 8 + 4: return (const void*)k_persistent<4, 4, 256, 3>;
    default: return nullptr;
    }
}

hipError_t persistent_occupancy(int prec, int R, bool wide, int* blocks_per_cu) {
    if (wide) return wide_available(prec, R) ? occ_one<1, 1, 4>(blocks_per_cu) : hipErrorInvalidValue;
    switch (prec * 8 + R) {
    case 0 * 8 + 1: return occ_one<0, 1, 3>(blocks_per_cu);
    case 0 * 8 + 2: return occ_one<0, 2, 3>(blocks_per_cu);
    case 0 * 8 + 4: return occ_one<0, 4, 3>(blocks_per_cu);
    case 1 * 8 + 1: return occ_one<1, 1, 3>(blocks_per_cu);
    case 1 * 8 + 2: return occ_one<1, 2, 3>(blocks_per_cu);
    case 1 * 8 + 4: return occ_one<1, 4, 3>(blocks_per_cu);
    case 2 * 8 + 1: return occ_one<2, 1, 3>(blocks_per_cu);
    case 2 * 8 + 2: return occ_one<2, 2, 3>(blocks_per_cu);
    case 2 * 8 + 4: return occ_one<2, 4, 3>(blocks_per_cu);
    case 3 * 8 + 1: return occ_one<3, 1, 3>(blocks_per_cu);
    case 3 * 8 + 2: return occ_one<3, 2, 3>(blocks_per_cu);
    case 3 * 8 + 4: return occ_one<3, 4, 3>(blocks_per_cu);
    case 4 * 8 + 1: return occ_one<4, 1, 3>(blocks_per_cu);
    case 4 * 8 + 2: return occ_one<4, 2, 3>(blocks_per_cu);
    case 4 * 8 + 4: return occ_one<4, 4, 3>(blocks_per_cu);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace kde
