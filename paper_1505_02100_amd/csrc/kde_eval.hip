// Density evaluation with a selected bandwidth: the kernel estimator of
// equation (1) with the Gaussian kernel of equation (2),
//     f(y_k) = (n h)^-1 sum_i phi((y_k - x_i) / h),   k < m,
// on a grid of points or at the samples themselves.
//
// Work decomposition.  The m evaluation points are cut into tiles of 256
// (one point per thread) and the n samples into chunks of W columns; a
// block evaluates one (tile, chunk) item, streaming its chunk through LDS in
// tiles of TJ values read as b128 broadcasts, and writes one partial sum per
// point.  A second kernel adds a point's partials in chunk order (so results
// are deterministic) and applies the normalisation 1 / (n h sqrt(2 pi)).
//
// FP32 arithmetic.  With k = log2(e)/2 and s = sqrt(k) / h, the scaled
// values v = (x - c) s (computed in FP64, then rounded) give
//     phi-factor exp(-((y - x)/h)^2 / 2) = 2^(-(v_y - v_x)^2),
// so a pair costs a subtraction, a square, one v_exp_f32 and an add.  The
// centre c is the midrange of the tile's points, so the rounding of v_y and
// of the columns that matter (within a few bandwidths of the tile) stays at
// a few ulp of small numbers.  A tile whose points spread over more than
// kEvalSpan scaled units takes the difference y - x in FP64 instead (then
// squares it in FP64 and rounds once before the exp2); this is the case for
// unsorted evaluation points.  Each point keeps four FP32 accumulators that
// take at most kEvalFold terms each, adds them pairwise in FP32 and folds
// the result into an FP64 sum.  There is no cancellation (every term is
// positive), so the relative error per point is that of the terms: a few
// times 1e-7.
//
// FP64 arithmetic is the plain definition: u = (y - x) / h, exp(-u^2 / 2).
#include <hip/hip_runtime.h>

#include <math.h>

#include "kde_internal.h"
#include "kde_eval.h"

namespace kde {
namespace eval {

constexpr int BLOCK = 256;
constexpr int TJ = 1024;        // column values per LDS tile
constexpr int kEvalFold = 4;    // b128 reads per FP32 accumulator before the FP64 fold
constexpr double kEvalSpan = 8.0;

__device__ __forceinline__ double load_x(const void* x, int32_t dtype, int64_t i) {
    return dtype == 0 ? static_cast<const double*>(x)[i] : static_cast<double>(static_cast<const float*>(x)[i]);
}

__device__ __forceinline__ double block_min_max(double lo, double hi, double* red, double* out_hi) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        lo = fmin(lo, __shfl_xor(lo, off, 64));
        hi = fmax(hi, __shfl_xor(hi, off, 64));
    }
    if (lane == 0) {
        red[2 * wave] = lo;
        red[2 * wave + 1] = hi;
    }
    __syncthreads();
    double a = red[0], b = red[1];
#pragma unroll
    for (int w = 1; w < BLOCK / 64; ++w) {
        a = fmin(a, red[2 * w]);
        b = fmax(b, red[2 * w + 1]);
    }
    __syncthreads();
    *out_hi = b;
    return a;
}

__device__ __forceinline__ void flag_nonfinite(int32_t* flag) {
    __hip_atomic_store(flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One (tile, chunk) item.  PREC 0: FP64 plain; 1: FP32 (centred, or FP64
// differences for a wide tile).
template <int PREC>
__global__ __launch_bounds__(BLOCK) void k_eval(EvalArgs a) {
    __shared__ __align__(16) double tile64[TJ];
    __shared__ double red[2 * BLOCK / 64];
    float* tile32 = reinterpret_cast<float*>(tile64);

    const int tid = threadIdx.x;
    const int32_t rt = (int32_t)(blockIdx.x / a.n_cc);
    const int32_t cc = (int32_t)(blockIdx.x % a.n_cc);
    const int64_t k = (int64_t)rt * BLOCK + tid;
    const bool live = k < a.m;
    double y = live ? a.y[k] : 0.0;
    if (live && !isfinite(y)) {
        flag_nonfinite(a.flag);
        y = 0.0;
    }
    const int64_t c0 = (int64_t)cc * a.W;
    const int64_t c1 = min(c0 + a.W, a.n);

    double tot = 0.0;
    if constexpr (PREC == 0) {
        const double inv_h = 1.0 / a.h;
        for (int64_t cj = c0; cj < c1; cj += TJ) {
            const int len = (int)min((int64_t)TJ, c1 - cj);
            __syncthreads();
            for (int e = tid; e < TJ; e += BLOCK) {
                double v = INFINITY;
                if (e < len) {
                    v = load_x(a.x, a.dtype, cj + e);
                    if (!isfinite(v)) {
                        flag_nonfinite(a.flag);
                        v = INFINITY;
                    }
                }
                tile64[e] = v;
            }
            __syncthreads();
            const double2* t2 = reinterpret_cast<const double2*>(tile64);
            for (int j = 0; j < len; j += 2) {
                const double2 v = t2[j >> 1];
                const double u0 = (y - v.x) * inv_h, u1 = (y - v.y) * inv_h;
                tot += exp(-0.5 * u0 * u0);
                tot += exp(-0.5 * u1 * u1);
            }
        }
    } else {
        // centre and spread of this tile's points
        double hi;
        const double lo = block_min_max(live ? y : INFINITY, live ? y : -INFINITY, red, &hi);
        const double c = 0.5 * lo + 0.5 * hi;
        const bool narrow = (hi - lo) * a.s <= kEvalSpan;
        const float vy = (float)((y - c) * a.s);
        const double uy = (y - c) * a.s;
        float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        for (int64_t cj = c0; cj < c1; cj += TJ) {
            const int len = (int)min((int64_t)TJ, c1 - cj);
            __syncthreads();
            for (int e = tid; e < TJ; e += BLOCK) {
                double v = INFINITY;
                if (e < len) {
                    v = load_x(a.x, a.dtype, cj + e);
                    if (!isfinite(v)) {
                        flag_nonfinite(a.flag);
                        v = INFINITY;
                    } else {
                        v = (v - c) * a.s;
                    }
                }
                if (narrow)
                    tile32[e] = (float)v;
                else
                    tile64[e] = v;
            }
            __syncthreads();
            const int groups = (len + 4 * kEvalFold - 1) / (4 * kEvalFold);
            if (narrow) {
                const float4* t4 = reinterpret_cast<const float4*>(tile32);
                for (int g = 0; g < groups; ++g) {
#pragma unroll
                    for (int q = 0; q < kEvalFold; ++q) {
                        const float4 v = t4[g * kEvalFold + q];
                        const float d0 = vy - v.x, d1 = vy - v.y, d2 = vy - v.z, d3 = vy - v.w;
                        acc[0] += __builtin_amdgcn_exp2f(-(d0 * d0));
                        acc[1] += __builtin_amdgcn_exp2f(-(d1 * d1));
                        acc[2] += __builtin_amdgcn_exp2f(-(d2 * d2));
                        acc[3] += __builtin_amdgcn_exp2f(-(d3 * d3));
                    }
                    tot += (double)((acc[0] + acc[1]) + (acc[2] + acc[3]));
                    acc[0] = acc[1] = acc[2] = acc[3] = 0.0f;
                }
            } else {
                const double2* t2 = reinterpret_cast<const double2*>(tile64);
                for (int g = 0; g < groups; ++g) {
#pragma unroll
                    for (int q = 0; q < 2 * kEvalFold; ++q) {
                        const double2 v = t2[g * 2 * kEvalFold + q];
                        const double d0 = uy - v.x, d1 = uy - v.y;
                        acc[(2 * q) & 3] += __builtin_amdgcn_exp2f(-(float)(d0 * d0));
                        acc[(2 * q + 1) & 3] += __builtin_amdgcn_exp2f(-(float)(d1 * d1));
                    }
                    tot += (double)((acc[0] + acc[1]) + (acc[2] + acc[3]));
                    acc[0] = acc[1] = acc[2] = acc[3] = 0.0f;
                }
            }
        }
    }
    if (live) {
        if (a.n_cc == 1)
            a.out[k] = tot * a.norm;
        else
            a.part[(int64_t)cc * a.m + k] = tot;
    }
}

// out[k] = norm * sum over chunks, in chunk order.
__global__ __launch_bounds__(BLOCK) void k_eval_reduce(const double* part, int32_t n_cc, int64_t m, double norm,
                                                       double* out) {
    const int64_t k = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (k >= m) return;
    double s = 0.0;
    for (int32_t c = 0; c < n_cc; ++c) s += part[(int64_t)c * m + k];
    out[k] = s * norm;
}

hipError_t launch(const EvalArgs& a, hipStream_t s) {
    const int64_t items = (int64_t)a.n_rt * a.n_cc;
    if (a.prec == 0)
        hipLaunchKernelGGL(k_eval<0>, dim3((unsigned)items), dim3(BLOCK), 0, s, a);
    else
        hipLaunchKernelGGL(k_eval<1>, dim3((unsigned)items), dim3(BLOCK), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || a.n_cc == 1) return e;
    const unsigned blocks = (unsigned)((a.m + BLOCK - 1) / BLOCK);
    hipLaunchKernelGGL(k_eval_reduce, dim3(blocks), dim3(BLOCK), 0, s, a.part, a.n_cc, a.m, a.norm, a.out);
    return hipGetLastError();
}

}  // namespace eval
}  // namespace kde
