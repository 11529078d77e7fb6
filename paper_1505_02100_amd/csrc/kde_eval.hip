// Density evaluation with a selected bandwidth: the kernel estimator of
// equation (1) with the Gaussian kernel of equation (2),
//     f(y_k) = (n h)^-1 sum_i phi((y_k - x_i) / h),   k < m,
// on a grid of points or at the samples themselves.
//
// Work decomposition.  The m evaluation points are cut into tiles (256
// points for FP64, one per thread; 4096 for FP32, runs of 32 consecutive
// points, each run shared by two threads) and the n samples into chunks of W
// columns; a block evaluates one (tile, chunk) item, streaming its chunk
// through LDS in tiles of column values read as b128 broadcasts, and writes
// one partial sum per point.  A
// second kernel adds a point's partials in a fixed order (so results are
// deterministic) and applies the normalisation 1 / (n h sqrt(2 pi)).
//
// FP32 arithmetic works in scaled units: with k = log2(e)/2 and
// s = sqrt(k) / h, v = x s, and the kernel factor exp(-((y - x)/h)^2 / 2) is
// 2^(-(v_y - v_x)^2).
//
// Evenly spaced runs (grids).  When a tile cuts into evenly spaced runs of
// 32 points, each run is two sub-runs of 16 with reference points u_0 and
// u_1 = u_0 + 16 ds, point j of sub-run b at u_b + j ds (j = -8 .. 7), and a
// column's 32 terms come from four exp2: with d_b = u_b - v_x,
//     2^(-(d_b + j ds)^2) = 2^(-K - j^2 ds^2 - 32 b j ds^2) * E_b R^j,
//     E_b = 2^(K - d_b^2),  R = 2^(-2 ds d_0),
// R^j by repeated multiplication in both directions (R and 1/R, shared by
// the two sub-runs), so a pair costs one multiply and one add instead of an
// exp2; the factor 2^(-K - ...) is applied once per point at the end.  d_b is
// formed in FP64 (exact for the columns that matter whatever the offset of
// the data) and the exponents are rounded to FP32 once.  The offset K = 24
// keeps E_b in FP32's normal range for every column within about 12 scaled
// units of the reference, so the terms that it would otherwise flush are
// below 2^-100 of a nearby sample's; the span of a sub-run is limited to 4
// scaled units (points at most 8 steps from their reference), which bounds
// the terms (at most 2^(K + 20)) and the error of R^j.  The two threads of a
// run take every other group of kRunFold columns; their FP32 sums take
// kRunFold columns before they are folded into FP64, and the two FP64 sums
// are added at the end.  The derivation of the error bound (about 6.4e-6
// relative per point, measured 1e-7) is in the tests of this kernel.
//
// Other points (unsorted, uneven, or spaced more widely than 0.3 h) take the
// per-point path in sub-tiles of 512, two adjacent points per thread (each
// column read from LDS serves both): for 2^(-(v_y - v_x)^2) =
// 2^(-v_y^2) 2^(v_x (2 v_y) - v_x^2), with (v_x, -v_x^2) stored per column a
// pair costs one fma, one v_exp_f32 and an add, and each point's sum is
// scaled by 2^(-v_y^2) once.  The exponent v_y^2 - (v_y - v_x)^2 never
// exceeds v_y^2, so nothing overflows, and far columns underflow to 0 as
// they should.  Each group of 32 lanes (64 points, half a wave) has its own
// centre c, the midrange of its points, and its own FP32 copy of the column
// tile in LDS, centred on it: the rounding of v_y and of the columns that
// matter (within a few bandwidths of the group) then stays at a few ulp of
// small numbers.  A sub-tile with a group whose points spread over more than
// kEvalSpan scaled units (about 9.4 h) takes the difference y - x in FP64
// instead (then squares it in FP64 and rounds once before the exp2); this
// is the case for unsorted evaluation points.  Each point keeps four FP32
// accumulators that take at most kEvalFold terms each, adds them pairwise
// in FP32 and folds the result into an FP64 sum.  There is no cancellation
// (every term is positive), so the relative error per point is that of the
// terms: a few times 1e-7.
//
// FP64 arithmetic is the plain definition: u = (y - x) / h, exp(-u^2 / 2).
#include <hip/hip_runtime.h>

#include <math.h>

#include "kde_internal.h"
#include "kde_eval.h"

namespace kde {
namespace eval {

constexpr int BLOCK = 256;
constexpr int TJ = 1024;        // column values per LDS tile (FP64 paths)
constexpr int GROUP = 32;       // lanes sharing a centre (FP32 per-point path)
constexpr int NGROUP = BLOCK / GROUP;
constexpr int TJN = 256;        // columns per LDS tile and group (FP32 path; two floats each)
constexpr int kEvalFold = 4;    // b128 reads per FP32 accumulator before the FP64 fold
constexpr double kEvalSpan = 8.0;
constexpr int PPT = 2;               // points per thread on the per-point path (FP32)
constexpr int SUBTILE = BLOCK * PPT; // points per sub-tile of that path
constexpr int RUN = 32;              // points of an evenly spaced run (two threads share one)
constexpr int SUB = 16;              // points per sub-run (one reference point each)
constexpr int SUB_REF = 8;           // a sub-run's reference point
constexpr int RUNS = BLOCK / 2;      // runs per FP32 tile
constexpr int TP32 = RUNS * RUN;     // points per FP32 tile
static_assert(RUN == 2 * SUB && TP32 % SUBTILE == 0, "run layout");
static_assert(SUB * RUNS <= NGROUP * TJN, "the exchange of half sums fits the column tile");
static_assert(TP32 == kTilePoints32 && BLOCK == kTilePoints64, "tile sizes the host assumes");
static_assert(NGROUP * TJN >= TJ, "the FP64 column tile fits the group tiles");
constexpr double kRunTol = 1e-9;     // evenly spaced to this many scaled units
constexpr double kRunSpan = 4.0;     // largest span of a sub-run, scaled units
constexpr double kRunK = 24.0;       // exponent offset of the run terms
constexpr float kRunArgMax = 60.0f;  // clamp of the ratio's exponent
constexpr double kRunPad = 1e30;     // column value of a padded (or non-finite) sample
constexpr double kRunRefMax = 1048576.0;  // largest |reference| of a run, scaled units
constexpr int kRunFold = 32;         // columns per FP32 run accumulator before the FP64 fold

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

// FP32, one sub-tile of SUBTILE points of an item whose points are not
// evenly spaced runs: points k_first + PPT tid + p (p < PPT, adjacent points
// in a lane) against columns [c0, c1), centred per group of 32 lanes (narrow
// groups) or with FP64 differences (wide blocks).  Each column read from LDS
// serves the lane's PPT points.
__device__ void eval_subtile_f32(const EvalArgs& a, int32_t cc, int64_t k_first, int64_t c0, int64_t c1,
                                 double* tile64, double* red, double* gcen, int32_t* gwide) {
    const int tid = threadIdx.x;
    const int64_t kt = k_first + (int64_t)PPT * tid;
    double y[PPT], tot[PPT];
    bool live[PPT];
    double glo = INFINITY, ghi = -INFINITY;
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
        live[p] = kt + p < a.m;
        y[p] = live[p] ? a.y[kt + p] : 0.0;
        if (live[p] && !isfinite(y[p])) {
            flag_nonfinite(a.flag);
            y[p] = 0.0;
        }
        tot[p] = 0.0;
        if (live[p]) {
            glo = fmin(glo, y[p]);
            ghi = fmax(ghi, y[p]);
        }
    }
    // centre and spread of each group of 32 lanes (lanes 0-31 and 32-63 of
    // a wave); a group without live points is narrow
#pragma unroll
    for (int off = GROUP / 2; off > 0; off >>= 1) {
        glo = fmin(glo, __shfl_xor(glo, off, 64));
        ghi = fmax(ghi, __shfl_xor(ghi, off, 64));
    }
    const int grp = tid / GROUP;
    __syncthreads();  // the previous sub-tile is done with gcen, gwide and the tiles
    if (tid == 0) *gwide = 0;
    __syncthreads();
    if ((tid & (GROUP - 1)) == 0) {
        const bool any = glo <= ghi;
        gcen[grp] = any ? 0.5 * glo + 0.5 * ghi : 0.0;
        if (any && (ghi - glo) * a.s > kEvalSpan) atomicOr(gwide, 1);
    }
    __syncthreads();
    const bool narrow = *gwide == 0;
    if (narrow) {
        // 2^(-(v_y - v_x)^2) = 2^(-v_y^2) 2^(fma(v_x, 2 v_y, -v_x^2)): the
        // column tile holds (v_x, -v_x^2), the argument is at most v_y^2
        // (<= 16 here), and the point's factor 2^(-v_y^2) is applied once
        // at the end in FP64, so a pair costs an fma, the exp2 and an add
        float vy[PPT], vy2[PPT], acc[PPT][4];
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
            vy[p] = (float)((y[p] - gcen[grp]) * a.s);
            vy2[p] = 2.0f * vy[p];
            acc[p][0] = acc[p][1] = acc[p][2] = acc[p][3] = 0.0f;
        }
        float2* tile2 = reinterpret_cast<float2*>(tile64);
        const float4* t4 = reinterpret_cast<const float4*>(tile2 + grp * TJN);
        for (int64_t cj = c0; cj < c1; cj += TJN) {
            const int len = (int)min((int64_t)TJN, c1 - cj);
            __syncthreads();
            for (int e = tid; e < TJN; e += BLOCK) {
                double v = 0.0;
                bool pad = true;
                if (e < len) {
                    v = load_x(a.x, a.dtype, cj + e);
                    if (!isfinite(v))
                        flag_nonfinite(a.flag);
                    else
                        pad = false;
                }
#pragma unroll
                for (int g = 0; g < NGROUP; ++g) {
                    // a column too far away for v_x^2 to stay finite contributes 0
                    const double vxd = (v - gcen[g]) * a.s;
                    const bool zero = pad || !(fabs(vxd) < 1e15);
                    const float vx = zero ? 0.0f : (float)vxd;
                    tile2[g * TJN + e] = make_float2(vx, zero ? -INFINITY : -(vx * vx));
                }
            }
            __syncthreads();
            const int groups = (len + 4 * kEvalFold - 1) / (4 * kEvalFold);
            for (int g = 0; g < groups; ++g) {
#pragma unroll
                for (int q = 0; q < 2 * kEvalFold; ++q) {
                    const float4 v = t4[g * 2 * kEvalFold + q];
#pragma unroll
                    for (int p = 0; p < PPT; ++p) {
                        acc[p][(2 * q) & 3] += __builtin_amdgcn_exp2f(__builtin_fmaf(v.x, vy2[p], v.y));
                        acc[p][(2 * q + 1) & 3] += __builtin_amdgcn_exp2f(__builtin_fmaf(v.z, vy2[p], v.w));
                    }
                }
#pragma unroll
                for (int p = 0; p < PPT; ++p) {
                    tot[p] += (double)((acc[p][0] + acc[p][1]) + (acc[p][2] + acc[p][3]));
                    acc[p][0] = acc[p][1] = acc[p][2] = acc[p][3] = 0.0f;
                }
            }
        }
#pragma unroll
        for (int p = 0; p < PPT; ++p) tot[p] *= exp2(-((double)vy[p] * (double)vy[p]));
    } else {
        // one centre for the block, differences in FP64
        double hi;
        const double lo = block_min_max(glo, ghi, red, &hi);
        const double c = 0.5 * lo + 0.5 * hi;
        double uy[PPT];
        float acc[PPT][4];
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
            uy[p] = (y[p] - c) * a.s;
            acc[p][0] = acc[p][1] = acc[p][2] = acc[p][3] = 0.0f;
        }
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
                tile64[e] = v;
            }
            __syncthreads();
            const int groups = (len + 4 * kEvalFold - 1) / (4 * kEvalFold);
            const double2* t2 = reinterpret_cast<const double2*>(tile64);
            for (int g = 0; g < groups; ++g) {
#pragma unroll
                for (int q = 0; q < 2 * kEvalFold; ++q) {
                    const double2 v = t2[g * 2 * kEvalFold + q];
#pragma unroll
                    for (int p = 0; p < PPT; ++p) {
                        const double d0 = uy[p] - v.x, d1 = uy[p] - v.y;
                        acc[p][(2 * q) & 3] += __builtin_amdgcn_exp2f(-(float)(d0 * d0));
                        acc[p][(2 * q + 1) & 3] += __builtin_amdgcn_exp2f(-(float)(d1 * d1));
                    }
                }
#pragma unroll
                for (int p = 0; p < PPT; ++p) {
                    tot[p] += (double)((acc[p][0] + acc[p][1]) + (acc[p][2] + acc[p][3]));
                    acc[p][0] = acc[p][1] = acc[p][2] = acc[p][3] = 0.0f;
                }
            }
        }
    }
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
        if (live[p]) {
            if (a.n_cc == 1)
                a.out[kt + p] = tot[p] * a.norm;
            else
                a.part[(int64_t)cc * a.m + kt + p] = tot[p];
        }
    }
}

// One (tile, chunk) item, FP64 plain: a tile of 256 points, one per thread.
__global__ __launch_bounds__(BLOCK) void k_eval64(EvalArgs a) {
    __shared__ __align__(16) double tile64[TJ];
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
    const double inv_h = 1.0 / a.h;
    double tot = 0.0;
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
    if (live) {
        if (a.n_cc == 1)
            a.out[k] = tot * a.norm;
        else
            a.part[(int64_t)cc * a.m + k] = tot;
    }
}

// One step of an evenly spaced run: column v_x (scaled, centred) against the
// run's RUN points, two sub-runs of SUB points with reference points u_b =
// u_0 + b SUB ds (b = 0, 1); point i of sub-run b sits at u_b + j ds,
// j = i - SUB_REF.  With d_b = u_b - v_x,
//     -(d_b + j ds)^2 = -d_b^2 - 2 j ds d_b - j^2 ds^2,
// and d_b = d_0 + b SUB ds, so with E_b = 2^(K - d_b^2) and one ratio
// R = 2^(-2 ds d_0) for both sub-runs,
//     E_b R^j = 2^(K - (d_b + j ds)^2 + j^2 ds^2 + 2 j b SUB ds^2):
// four exp2 per column (E_0, E_1, R, 1/R), then one multiply and one add per
// point; the factor 2^(-K - j^2 ds^2 - 2 j b SUB ds^2) is applied to the
// point's sum at the end.  The exponents are formed in FP64 and rounded once;
// the R exponent is clamped to +-kRunArgMax, which only changes columns whose
// E_0 and E_1 are both 0.
__device__ __forceinline__ void run_chain(float e, float r, float ri, float* acc) {
    acc[SUB_REF] += e;
    float t = e;
#pragma unroll
    for (int j = 1; j < SUB - SUB_REF; ++j) {
        t *= r;
        acc[SUB_REF + j] += t;
    }
    t = e;
#pragma unroll
    for (int j = 1; j <= SUB_REF; ++j) {
        t *= ri;
        acc[SUB_REF - j] += t;
    }
}

__device__ __forceinline__ void run_step(double vx, double u0, double u1, double m2ds, float (&acc)[RUN]) {
    const double d0 = u0 - vx, d1 = u1 - vx;
    const float ea0 = (float)__builtin_fma(-d0, d0, kRunK);
    const float ea1 = (float)__builtin_fma(-d1, d1, kRunK);
    const float ra = __builtin_amdgcn_fmed3f((float)(d0 * m2ds), -kRunArgMax, kRunArgMax);
    const float e0 = __builtin_amdgcn_exp2f(ea0);
    const float e1 = __builtin_amdgcn_exp2f(ea1);
    const float r = __builtin_amdgcn_exp2f(ra);
    const float ri = __builtin_amdgcn_exp2f(-ra);
    run_chain(e0, r, ri, acc);
    run_chain(e1, r, ri, acc + SUB);
}

// One (tile, chunk) item, FP32: a tile of TP32 points.  If the tile cuts into
// evenly spaced runs of RUN consecutive points (each to kRunTol scaled units,
// a sub-run spanning at most kRunSpan) the block takes the run path: threads
// t and t + RUNS share run t, each taking every other group of kRunFold
// columns, and add their sums at the end.  Otherwise it evaluates the tile as
// sub-tiles of SUBTILE points, PPT adjacent points per thread.
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(4))) void k_eval32(EvalArgs a) {
    __shared__ __align__(16) double tile64[NGROUP * TJN];
    __shared__ double red[2 * BLOCK / 64];
    __shared__ double gcen[NGROUP];
    __shared__ int32_t gwide;

    const int tid = threadIdx.x;
    const int run = tid % RUNS, half = tid / RUNS;  // half is the same across a wave
    const int32_t rt = (int32_t)(blockIdx.x / a.n_cc);
    const int32_t cc = (int32_t)(blockIdx.x % a.n_cc);
    const int64_t kb = (int64_t)rt * TP32;
    const int64_t c0 = (int64_t)cc * a.W;
    const int64_t c1 = min(c0 + a.W, a.n);

    // the run's points k0 .. k0 + live_n - 1: evenly spaced?  Each half of
    // the pair checks its sub-run against the line through the run's ends.
    const int64_t k0 = kb + (int64_t)run * RUN;
    const int live_n = (int)max((int64_t)0, min((int64_t)RUN, a.m - k0));
    bool ok = true;
    double y0 = 0.0, dy = 0.0;
    if (live_n > 0) {
        y0 = a.y[k0];
        if (live_n > 1) dy = (a.y[k0 + live_n - 1] - y0) / (double)(live_n - 1);
        for (int i = half * SUB; i < min(live_n, (half + 1) * SUB); ++i) {
            const double yi = a.y[k0 + i];
            if (!isfinite(yi)) {
                flag_nonfinite(a.flag);
                ok = false;
            } else if (!(fabs((yi - (y0 + (double)i * dy)) * a.s) <= kRunTol)) {
                ok = false;
            }
        }
        if (!(fabs(dy * a.s) * (double)(SUB - 1) <= kRunSpan)) ok = false;
        // the references relative to the block's first point: within
        // kRunRefMax scaled units their FP64 rounding (and that of the centred
        // columns near them) stays below 2^-32 units; a grid tile spans at
        // most about 1100
        const double u0 = (y0 - a.y[kb]) * a.s + (double)SUB_REF * dy * a.s;
        if (!(fabs(u0) < kRunRefMax && fabs(u0 + (double)SUB * dy * a.s) < kRunRefMax)) ok = false;
    }
    if (!__syncthreads_and(ok)) {
        for (int sub = 0; sub < TP32 / SUBTILE; ++sub) {
            const int64_t kf = kb + (int64_t)sub * SUBTILE;
            if (kf >= a.m) break;  // the same for every thread
            eval_subtile_f32(a, cc, kf, c0, c1, tile64, red, gcen, &gwide);
        }
        return;
    }

    // run path: columns centred on the block's first point, in FP64
    const double cb = a.y[kb];
    const double ds = dy * a.s;
    const double u0 = (y0 - cb) * a.s + (double)SUB_REF * ds;
    const double u1 = u0 + (double)SUB * ds;
    const double m2ds = -2.0 * ds;
    double tot[RUN];
#pragma unroll
    for (int i = 0; i < RUN; ++i) tot[i] = 0.0;
    const double2* t2 = reinterpret_cast<const double2*>(tile64);
    for (int64_t cj = c0; cj < c1; cj += TJ) {
        const int len = (int)min((int64_t)TJ, c1 - cj);
        __syncthreads();
        for (int e = tid; e < TJ; e += BLOCK) {
            double v = kRunPad;
            if (e < len) {
                const double x = load_x(a.x, a.dtype, cj + e);
                // a finite sample whose scaled distance overflows is as far
                // away as a pad (an infinite one would make the ratio's
                // exponent inf * 0 in a run of zero spacing)
                if (!isfinite(x))
                    flag_nonfinite(a.flag);
                else
                    v = fmin(fmax((x - cb) * a.s, -kRunPad), kRunPad);
            }
            tile64[e] = v;
        }
        __syncthreads();
        const int groups = (len + kRunFold - 1) / kRunFold;
        for (int g = half; g < groups; g += 2) {
            float acc[RUN];
#pragma unroll
            for (int i = 0; i < RUN; ++i) acc[i] = 0.0f;
#pragma unroll
            for (int q = 0; q < kRunFold / 2; ++q) {
                const double2 v = t2[g * (kRunFold / 2) + q];
                run_step(v.x, u0, u1, m2ds, acc);
                run_step(v.y, u0, u1, m2ds, acc);
            }
#pragma unroll
            for (int i = 0; i < RUN; ++i) tot[i] += (double)acc[i];
        }
    }
    // the two halves add their sums through LDS: half 0 finishes sub-run 0,
    // half 1 sub-run 1 (a + b == b + a, so the result does not depend on
    // which half adds)
    double* xch = tile64;
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        __syncthreads();
        if (half != b) {
#pragma unroll
            for (int i = 0; i < SUB; ++i) xch[i * RUNS + run] = tot[b * SUB + i];
        }
        __syncthreads();
        if (half == b) {
#pragma unroll
            for (int i = 0; i < SUB; ++i) tot[b * SUB + i] += xch[i * RUNS + run];
        }
    }
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        if (half != b) continue;
#pragma unroll
        for (int i = 0; i < SUB; ++i) {
            const int p = b * SUB + i;
            if (p < live_n) {
                const double j = (double)(i - SUB_REF);
                const double t = tot[p] * exp2(-(double)kRunK - j * j * ds * ds - 2.0 * j * (double)(b * SUB) * ds * ds);
                if (a.n_cc == 1)
                    a.out[k0 + p] = t * a.norm;
                else
                    a.part[(int64_t)cc * a.m + k0 + p] = t;
            }
        }
    }
}

// out[k] = norm * sum over chunks in a fixed order: RLANES threads per point,
// lane q adding chunks q + RLANES (RILP i + r) into its r-th sum (RILP sums in
// flight, so a thread keeps RILP loads outstanding), the sums then added in
// order r = 0, 1, ..., and lane 0 adding the RLANES lane sums in lane order
// (deterministic).  Consecutive threads take consecutive points, so each load
// instruction reads whole lines of one chunk's partials.
constexpr int RLANES = 16;
constexpr int RPOINTS = BLOCK / RLANES;
constexpr int RILP = 8;

__global__ __launch_bounds__(BLOCK) void k_eval_reduce(const double* part, int32_t n_cc, int64_t m, double norm,
                                                       double* out) {
    __shared__ double red[RLANES][RPOINTS];
    const int p = threadIdx.x % RPOINTS, q = threadIdx.x / RPOINTS;
    const int64_t k = (int64_t)blockIdx.x * RPOINTS + p;
    double s = 0.0;
    if (k < m) {
        double r[RILP];
#pragma unroll
        for (int i = 0; i < RILP; ++i) r[i] = 0.0;
        int32_t c = q;
        for (; c + (RILP - 1) * RLANES < n_cc; c += RILP * RLANES) {
#pragma unroll
            for (int i = 0; i < RILP; ++i) r[i] += part[(int64_t)(c + i * RLANES) * m + k];
        }
#pragma unroll
        for (int i = 0; i < RILP; ++i)
            if (c + i * RLANES < n_cc) r[i] += part[(int64_t)(c + i * RLANES) * m + k];
#pragma unroll
        for (int i = 0; i < RILP; ++i) s += r[i];
    }
    red[q][p] = s;
    __syncthreads();
    if (q == 0 && k < m) {
        double t = 0.0;
#pragma unroll
        for (int l = 0; l < RLANES; ++l) t += red[l][p];
        out[k] = t * norm;
    }
}

hipError_t launch(const EvalArgs& a, hipStream_t s) {
    const int64_t items = (int64_t)a.n_rt * a.n_cc;
    if (a.prec == 0)
        hipLaunchKernelGGL(k_eval64, dim3((unsigned)items), dim3(BLOCK), 0, s, a);
    else
        hipLaunchKernelGGL(k_eval32, dim3((unsigned)items), dim3(BLOCK), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || a.n_cc == 1) return e;
    const unsigned blocks = (unsigned)((a.m + RPOINTS - 1) / RPOINTS);
    hipLaunchKernelGGL(k_eval_reduce, dim3(blocks), dim3(BLOCK), 0, s, a.part, a.n_cc, a.m, a.norm, a.out);
    return hipGetLastError();
}

hipError_t blocks_per_cu(int prec, int* out) {
    return prec == 0 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(out, k_eval64, BLOCK, 0)
                     : hipOccupancyMaxActiveBlocksPerMultiprocessor(out, k_eval32, BLOCK, 0);
}

}  // namespace eval
}  // namespace kde
