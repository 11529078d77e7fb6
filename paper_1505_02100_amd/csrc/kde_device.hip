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
// v = (x - mean) / g, in FP64 and then rounded to FP32, so d = v_i - v_j is
// the kernel argument y = (x_i - x_j)/g of Steps IV and VI.  The Hermite
// factors are depressed in Y = y^2 (Z = Y - 5, resp. Z = Y - 3):
//     He6(y) = y^6 - 15 y^4 + 45 y^2 - 15 = Z^3 - 30 Z - 40,
//     He4(y) = y^4 - 6 y^2 + 3            = Z^2 - 6,
// so every polynomial coefficient is a small integer, exact in FP32.  The
// Gaussian factor is exp(-Y/2) = 2^(-k Y), k = log2(e)/2, evaluated as
// exp2(-k Z) (one v_exp_f32) times the constant 2^(-5k) (resp. 2^(-3k)),
// which is applied once to the FP64 total together with 1/sqrt(2 pi).  Per
// pair (r = 6):
//     d = vi - vj; Z = fma(d, d, -5); a = k Z; e = exp2(-a);
//     q = fma(Z, Z, -30); p = fma(q, Z, -40); acc = fma(p, e, acc)
// which is 6 VALU + 1 transcendental (r = 4 drops q: 5 + 1).  Why this form:
// the sums of K6 and K4 over all pairs cancel heavily (sum |K| / |sum K| is
// in the hundreds already at n = 1024 and grows as g shrinks), so any
// systematic error in the kernel's shape is amplified by that factor, while
// rounding errors that vary from pair to pair average out.  With integer
// coefficients the only systematic error left is the FP32 rounding of k
// (relative 1.3e-8), i.e. the Gaussian evaluated at a bandwidth larger by
// 7e-9 than the polynomial.  The EXACT_K variant removes even that with a
// two-term k (a = fma(Z, k_hi, Z k_lo)) at one more VALU op per pair.
// The FP32 value of a sample carries a rounding error that enters every
// pair of that sample the same way; summed over its n pairs it no longer
// averages out, and the cancellation factor makes it the dominant error at
// large n.  Each item therefore centres its rows and columns on its own
// offset, mean + g tau(row block) with tau a generic value in [-1/4, 1/4)
// (a golden-ratio sequence): the differences are unchanged, but a sample's
// rounding differs from item to item, so those errors average out too.
// Per lane, each row keeps FP32 partial sums over chunks of 64 columns that
// are folded into a Kahan-compensated FP32 (sum, compensation) pair.  The
// lane totals are reduced in FP64 in a fixed order.
//
// FP64 pair arithmetic is the plain printed form: t = y^2,
// p = ((t - 15) t + 45) t - 15 (resp. (t - 6) t + 3), exp(-t/2), FP64 sums.
//
// Cross-block reduction is deterministic: every item writes its own slot;
// the block that completes the last item of a stage (atomic counter) sums
// that stage's slots in index order and runs the stage's scalar formulas
// (Steps I-III, V, VII) in FP64, then publishes them with a release flag.
// Items of a later stage wait (acquire, bounded by a wall-clock limit) for
// that flag.  Items of earlier stages always hold smaller tickets, and no
// item waits on a later ticket, so the wait always ends.
#include <hip/hip_runtime.h>

#include <math.h>

#include <type_traits>

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

// ------------------------------------------------------------- moments
template <int BLOCK>
__device__ double moment_sum(const View& d, int32_t chunk_idx, double* red) {
    const int64_t a = (int64_t)chunk_idx * d.chunk;
    const int64_t b = min(a + (int64_t)d.chunk, d.n);
    double s = 0.0;
    for (int64_t i = a + threadIdx.x; i < b; i += BLOCK) s += load_x(d.x, d.dtype, i);
    return block_sum<BLOCK>(s, red);
}

template <int BLOCK>
__device__ void moment_ssq(const View& d, int32_t chunk_idx, double mean, double* red,
                           double* out_ssq, double* out_max) {
    const int64_t a = (int64_t)chunk_idx * d.chunk;
    const int64_t b = min(a + (int64_t)d.chunk, d.n);
    double s = 0.0, m = 0.0;
    for (int64_t i = a + threadIdx.x; i < b; i += BLOCK) {
        double v = load_x(d.x, d.dtype, i) - mean;
        s = fma(v, v, s);
        m = fmax(m, fabs(v));
    }
    *out_ssq = block_sum<BLOCK>(s, red);
    *out_max = block_max<BLOCK>(m, red);
}

// ---------------------------------------------------- FP32 pair evaluation
// Largest |Z| kept by the clamped variant: exp2(-k Z) is exactly 0 there and
// Z^3 stays finite.
constexpr float kZClamp = 1.0e12f;

template <int RO, bool SAFE, bool EXACT_K>
__device__ __forceinline__ float pair_term_f32(float vi, float vj, const PolyConsts& pc) {
    const float d = vi - vj;
    float Z = fmaf(d, d, RO == 6 ? -5.0f : -3.0f);
    if (SAFE) Z = fminf(Z, kZClamp);
    const float a = EXACT_K ? fmaf(Z, pc.k_hi, Z * pc.k_lo) : Z * pc.k_hi;
    const float e = __builtin_amdgcn_exp2f(-a);
    float p;
    if (RO == 6) {
        const float q = fmaf(Z, Z, -30.0f);
        p = fmaf(q, Z, -40.0f);
    } else {
        p = fmaf(Z, Z, -6.0f);
    }
    return p * e;
}

template <int RO, bool SAFE, bool EXACT_K>
__device__ __forceinline__ void pair_acc_f32(float vi, float vj, float& acc, const PolyConsts& pc) {
    const float d = vi - vj;
    float Z = fmaf(d, d, RO == 6 ? -5.0f : -3.0f);
    if (SAFE) Z = fminf(Z, kZClamp);
    const float a = EXACT_K ? fmaf(Z, pc.k_hi, Z * pc.k_lo) : Z * pc.k_hi;
    const float e = __builtin_amdgcn_exp2f(-a);
    float p;
    if (RO == 6) {
        const float q = fmaf(Z, Z, -30.0f);
        p = fmaf(q, Z, -40.0f);
    } else {
        p = fmaf(Z, Z, -6.0f);
    }
    acc = fmaf(p, e, acc);
}

template <int R>
__device__ __forceinline__ void kahan_fold(float (&acc)[R][2], float (&ks)[R], float (&kc)[R]) {
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const float chunk = acc[k][0] + acc[k][1];
        acc[k][0] = 0.0f;
        acc[k][1] = 0.0f;
        const float y = chunk - kc[k];
        const float t = ks[k] + y;
        kc[k] = (t - ks[k]) - y;
        ks[k] = t;
    }
}

template <int RO, bool SAFE, bool EXACT_K, int R>
__device__ __forceinline__ void pair_b128_f32(const float (&ui)[R], float4 v, float (&acc)[R][2],
                                              const PolyConsts& pc) {
#pragma unroll
    for (int k = 0; k < R; ++k) {
        pair_acc_f32<RO, SAFE, EXACT_K>(ui[k], v.x, acc[k][0], pc);
        pair_acc_f32<RO, SAFE, EXACT_K>(ui[k], v.y, acc[k][1], pc);
        pair_acc_f32<RO, SAFE, EXACT_K>(ui[k], v.z, acc[k][0], pc);
        pair_acc_f32<RO, SAFE, EXACT_K>(ui[k], v.w, acc[k][1], pc);
    }
}

// Generic centring offset of row block rb (see the header comment).
__device__ __forceinline__ double centre_offset(int32_t rb) {
    const double f = (double)rb * 0.6180339887498949;
    return 0.5 * (f - floor(f)) - 0.25;
}

template <int RO, bool SAFE, bool EXACT_K, int R, int BLOCK>
__device__ double pair_item_f32(const View& d, int32_t rb, int32_t cb, double mean, double scale,
                                const PolyConsts& pc, float* tile, double* red) {
    constexpr int TI = BLOCK * R;
    const double tau = centre_offset(rb);
    const int tid = threadIdx.x, lane = tid & (WAVE - 1), wave = tid / WAVE;
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
    float acc[R][2], ks[R], kc[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        acc[k][0] = acc[k][1] = 0.0f;
        ks[k] = kc[k] = 0.0f;
    }

    const int64_t c0 = r0 + (int64_t)cb * d.W;
    const int64_t c1 = min(c0 + d.W, n);
    for (int64_t cj = c0; cj < c1; cj += TJ) {
        const int len = (int)min((int64_t)TJ, c1 - cj);
        __syncthreads();
        for (int e = tid; e < len; e += BLOCK)
            tile[e] = (float)((load_x(d.x, d.dtype, cj + e) - mean) * scale - tau);
        __syncthreads();

        // columns inside this wave's row span: only j > i counts
        const int64_t ma = max(cj, wlo + 1), mb = min(cj + (int64_t)len, whi);
        for (int64_t j = ma; j < mb; ++j) {
            const float uj = tile[j - cj];
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const float t = pair_term_f32<RO, SAFE, EXACT_K>(ui[k], uj, pc);
                const bool live = j > wlo + lane + (int64_t)WAVE * k;
                acc[k][0] += live ? t : 0.0f;
            }
        }
        // columns right of this wave's rows: every pair counts
        const int64_t ua = max(cj, whi);
        if (ua < cj + len) {
            int jj = (int)(ua - cj);
            const float4* t4 = reinterpret_cast<const float4*>(tile);
            for (; jj + 64 <= len; jj += 64) {
#pragma unroll
                for (int q = 0; q < 16; ++q) pair_b128_f32<RO, SAFE, EXACT_K, R>(ui, t4[(jj >> 2) + q], acc, pc);
                kahan_fold<R>(acc, ks, kc);
            }
            for (; jj + 4 <= len; jj += 4) pair_b128_f32<RO, SAFE, EXACT_K, R>(ui, t4[jj >> 2], acc, pc);
            for (; jj < len; ++jj) {
                const float uj = tile[jj];
#pragma unroll
                for (int k = 0; k < R; ++k) pair_acc_f32<RO, SAFE, EXACT_K>(ui[k], uj, acc[k][0], pc);
            }
        }
        kahan_fold<R>(acc, ks, kc);
    }
    double lane_tot = 0.0;
#pragma unroll
    for (int k = 0; k < R; ++k) lane_tot += (double)ks[k] - (double)kc[k];
    return block_sum<BLOCK>(lane_tot, red);
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
    const int tid = threadIdx.x, lane = tid & (WAVE - 1), wave = tid / WAVE;
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
    const int64_t c0 = r0 + (int64_t)cb * d.W;
    const int64_t c1 = min(c0 + d.W, n);
    for (int64_t cj = c0; cj < c1; cj += TJ) {
        const int len = (int)min((int64_t)TJ, c1 - cj);
        __syncthreads();
        for (int e = tid; e < len; e += BLOCK) tile[e] = (load_x(d.x, d.dtype, cj + e) - mean) * scale;
        __syncthreads();
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

// ------------------------------------------------------------ finalisers
// Scalar formulas of Algorithm 1 in FP64, written in scale-free form so that
// samples with very large or small spread do not overflow sigma^9 or g^7:
//   g1 = sigma (-2 K6(0) 32 sqrt(pi) / (105 n))^(1/9)          (Steps II-III)
//   g2 = g1 (-2 K4(0) n / A6)^(1/7),  A6 = 2 S6 + n K6(0)       (Steps IV-V)
//   h  = g2 (R(K) n / A4)^(1/5),      A4 = 2 S4 + n K4(0)       (Steps VI-VII)
// which are the printed formulas with Psi8, Psi6(g1), Psi4(g2) substituted.
template <int PREC>
__device__ void finalize_stage(const View& d, State* st, int32_t stage, double tot, double aux,
                               const PolyConsts& pc) {
    const double pi = 3.14159265358979323846;
    const double rt2pi = sqrt(2.0 * pi);
    const double K6_0 = -15.0 / rt2pi, K4_0 = 3.0 / rt2pi, RK = 1.0 / (2.0 * sqrt(pi));
    const double nd = (double)d.n;
    int32_t status = ld_i32(&st->status);
    switch (stage) {
    case ST_SUM: {
        if (!isfinite(tot)) { set_status(st, KDE_ENONFINITE); status = KDE_ENONFINITE; }
        st_f64(&st->mean, tot / nd);
        break;
    }
    case ST_SSQ: {
        const double sigma = sqrt(tot / (nd - 1.0));
        st_f64(&st->sigma, sigma);
        st_f64(&st->maxdev, aux);
        if (status == 0 && !(sigma > 0.0 && isfinite(sigma))) { set_status(st, KDE_EDEGENERATE); status = KDE_EDEGENERATE; }
        double g;
        if (d.mode == MODE_PLUGIN) {
            st_f64(&st->psi8, 105.0 / (32.0 * sqrt(pi) * pow(sigma, 9.0)));
            g = sigma * pow(-2.0 * K6_0 * 32.0 * sqrt(pi) / (105.0 * nd), 1.0 / 9.0);
            st_f64(&st->g1, g);
        } else {
            g = d.psi_g;
        }
        const double scale = 1.0 / g;
        st_f64(&st->scale, scale);
        __hip_atomic_store(&st->safe, (int32_t)(aux * scale > kSafeLimit ? 1 : 0), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        break;
    }
    case ST_PSI6: {
        const double S6 = PREC == 2 ? pc.f6x * tot : PREC == 1 ? pc.f6 * tot : tot / rt2pi;
        st_f64(&st->S6, S6);
        const double A6 = 2.0 * S6 + nd * K6_0;
        const double g1 = d.mode == MODE_PLUGIN ? ld_f64(&st->g1) : d.psi_g;
        st_f64(&st->psi6, A6 / (nd * nd * pow(g1, 7.0)));
        if (d.mode == MODE_PLUGIN) {
            if (status == 0 && !(A6 < 0.0)) { set_status(st, KDE_EDEGENERATE); status = KDE_EDEGENERATE; }
            const double g2 = g1 * pow(-2.0 * K4_0 * nd / A6, 1.0 / 7.0);
            st_f64(&st->g2, g2);
            const double scale = 1.0 / g2;
            st_f64(&st->scale, scale);
            __hip_atomic_store(&st->safe, (int32_t)(ld_f64(&st->maxdev) * scale > kSafeLimit ? 1 : 0),
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        break;
    }
    case ST_PSI4: {
        const double S4 = PREC == 2 ? pc.f4x * tot : PREC == 1 ? pc.f4 * tot : tot / rt2pi;
        st_f64(&st->S4, S4);
        const double A4 = 2.0 * S4 + nd * K4_0;
        const double g2 = d.mode == MODE_PLUGIN ? ld_f64(&st->g2) : d.psi_g;
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
}

// --------------------------------------------------------------- kernels
__global__ void k_init(State* states, int32_t count, uint32_t* ticket) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) {
        State s = {};
        states[i] = s;
    }
    if (i == 0) *ticket = 0u;
}

template <int PREC, int R, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_persistent(LaunchArgs A) {
    using TileT = typename std::conditional<PREC >= 1, float, double>::type;
    __shared__ __align__(16) TileT tile[TJ];
    __shared__ double red[BLOCK / WAVE];
    __shared__ uint32_t sh_ticket;
    __shared__ int32_t sh_status, sh_safe, sh_last;
    __shared__ double sh_mean, sh_scale;

    const int tid = threadIdx.x;
    for (;;) {
        if (tid == 0) sh_ticket = atomicAdd(A.ticket, 1u);
        __syncthreads();
        const uint32_t t = sh_ticket;
        __syncthreads();
        if (t >= A.n_items) break;

        const Item it = A.items[t];
        const View d = load_view(A.descs + it.ds, it.stage);
        State* st = A.states + it.ds;

        if (tid == 0) {
            if (it.wait >= 0) {
                const uint64_t t0 = wall_clock64();
                while (ld_acquire(&st->ready[it.wait]) == 0u) {
                    __builtin_amdgcn_s_sleep(8);
                    if (ld_i32(&st->status) == KDE_ETIMEOUT) break;  // an earlier wait gave up
                    if (wall_clock64() - t0 > A.timeout_ticks) {
                        set_status(st, KDE_ETIMEOUT);
                        break;
                    }
                }
            }
            if (it.stage == ST_SUM && it.a == 0) {
                __hip_atomic_store(&st->t_first, (uint64_t)wall_clock64(), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            }
            sh_status = ld_i32(&st->status);
            sh_mean = ld_f64(&st->mean);
            sh_scale = ld_f64(&st->scale);
            sh_safe = __hip_atomic_load(&st->safe, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
        const int32_t status = sh_status;
        const double mean = sh_mean, scale = sh_scale;
        const int32_t safe = sh_safe;

        double v = 0.0, aux = 0.0;
        if (status == 0) {
            switch (it.stage) {
            case ST_SUM:
                v = moment_sum<BLOCK>(d, it.a, red);
                break;
            case ST_SSQ:
                moment_ssq<BLOCK>(d, it.a, mean, red, &v, &aux);
                break;
            case ST_PSI6:
            case ST_PSI4:
                if constexpr (PREC >= 1) {
                    constexpr bool XK = PREC == 2;
                    float* tl = reinterpret_cast<float*>(tile);
                    if (it.stage == ST_PSI6)
                        v = safe ? pair_item_f32<6, true, XK, R, BLOCK>(d, it.a, it.b, mean, scale, A.pc, tl, red)
                                 : pair_item_f32<6, false, XK, R, BLOCK>(d, it.a, it.b, mean, scale, A.pc, tl, red);
                    else
                        v = safe ? pair_item_f32<4, true, XK, R, BLOCK>(d, it.a, it.b, mean, scale, A.pc, tl, red)
                                 : pair_item_f32<4, false, XK, R, BLOCK>(d, it.a, it.b, mean, scale, A.pc, tl, red);
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

        if (tid == 0) {
            Slot s;
            s.v = v;
            s.aux = aux;
            A.slots[it.slot] = s;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            const uint32_t old = __hip_atomic_fetch_add(&st->done[it.stage], 1u, __ATOMIC_ACQ_REL,
                                                        __HIP_MEMORY_SCOPE_AGENT);
            sh_last = (old + 1u == (uint32_t)d.cnt) ? 1 : 0;
        }
        __syncthreads();
        if (sh_last) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            const int64_t base = d.base;
            const int32_t cnt = d.cnt;
            double s = 0.0, c = 0.0, m = 0.0;
            for (int32_t k = tid; k < cnt; k += BLOCK) {
                const Slot sl = A.slots[base + k];
                const double tt = s + sl.v;  // Neumaier step in slot order
                c += fabs(s) >= fabs(sl.v) ? (s - tt) + sl.v : (sl.v - tt) + s;
                s = tt;
                m = fmax(m, sl.aux);
            }
            const double tot = block_sum<BLOCK>(s + c, red);
            const double mx = block_max<BLOCK>(m, red);
            if (tid == 0) {
                finalize_stage<PREC>(d, st, it.stage, tot, mx, A.pc);
                __hip_atomic_store(&st->t_fin[it.stage], (uint64_t)wall_clock64(), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
                st_release(&st->ready[it.stage], 1u);
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------- host entry
hipError_t launch_init(State* states, int32_t count, uint32_t* ticket, hipStream_t s) {
    const int threads = 256;
    const int blocks = (count + threads - 1) / threads > 0 ? (count + threads - 1) / threads : 1;
    hipLaunchKernelGGL(k_init, dim3(blocks), dim3(threads), 0, s, states, count, ticket);
    return hipGetLastError();
}

template <int PREC, int R>
static hipError_t launch_one(int grid, hipStream_t s, const LaunchArgs& a) {
    hipLaunchKernelGGL((k_persistent<PREC, R, 256>), dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <int PREC, int R>
static hipError_t occ_one(int* blocks) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k_persistent<PREC, R, 256>, 256, 0);
}

hipError_t launch_persistent(int prec, int R, int grid, hipStream_t s, const LaunchArgs& a) {
    switch (prec * 8 + R) {
    case 0 * 8 + 1: return launch_one<0, 1>(grid, s, a);
    case 0 * 8 + 2: return launch_one<0, 2>(grid, s, a);
    case 0 * 8 + 4: return launch_one<0, 4>(grid, s, a);
    case 1 * 8 + 1: return launch_one<1, 1>(grid, s, a);
    case 1 * 8 + 2: return launch_one<1, 2>(grid, s, a);
    case 1 * 8 + 4: return launch_one<1, 4>(grid, s, a);
    case 2 * 8 + 1: return launch_one<2, 1>(grid, s, a);
    case 2 * 8 + 2: return launch_one<2, 2>(grid, s, a);
    case 2 * 8 + 4: return launch_one<2, 4>(grid, s, a);
    default: return hipErrorInvalidValue;
    }
}

hipError_t persistent_occupancy(int prec, int R, int* blocks_per_cu) {
    switch (prec * 8 + R) {
    case 0 * 8 + 1: return occ_one<0, 1>(blocks_per_cu);
    case 0 * 8 + 2: return occ_one<0, 2>(blocks_per_cu);
    case 0 * 8 + 4: return occ_one<0, 4>(blocks_per_cu);
    case 1 * 8 + 1: return occ_one<1, 1>(blocks_per_cu);
    case 1 * 8 + 2: return occ_one<1, 2>(blocks_per_cu);
    case 1 * 8 + 4: return occ_one<1, 4>(blocks_per_cu);
    case 2 * 8 + 1: return occ_one<2, 1>(blocks_per_cu);
    case 2 * 8 + 2: return occ_one<2, 2>(blocks_per_cu);
    case 2 * 8 + 4: return occ_one<2, 4>(blocks_per_cu);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace kde
