// Issue-rate microbenchmark for the pair stages' instruction mix on gfx950.
//
// Measures, with register-only loops (no memory traffic inside the timed
// loops), the device-wide rate of:
//   fma, mul, sub   FP32 VALU instructions (VOP2/VOP3, VGPR and inline
//                   constant operands), 8 independent chains per lane;
//   exp             v_exp_f32 (x <- 2^(-|x|), the modifiers are free);
//   pair_r6         one Step IV term: sub, fma, mul, exp, fma, fma, fma
//                   (the depressed He6 form of the kernel);
//   pair_r4         one Step VI term: sub, mul, fma, fma, mul, exp, fma;
//   pair_r6_noexp   the Step IV term without its exp (the exp's argument is
//                   used in its place), to see whether the exp overlaps the
//                   other VALU work;
// in the pair loops each lane holds 8 row values and their sums, and one
// column value per step is shared by the 8 pairs (one add per 8 pairs, as the
// kernel's LDS read serves 4 pairs), so only the sums carry from step to step;
// and the shader clock under that load: thread 0 of every block reads the
// shader cycle counter (s_memtime) and the 100 MHz wall clock
// (s_memrealtime) around its loop, and the ratio of the two deltas is the
// clock the SIMD actually ran at.
//
// Output: one JSON object on stdout.  Usage: issue_rate [waves_per_simd ...]
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <vector>

#define CHK(x)                                                                      \
    do {                                                                            \
        hipError_t e_ = (x);                                                        \
        if (e_ != hipSuccess) {                                                     \
            std::fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));            \
            std::exit(1);                                                           \
        }                                                                           \
    } while (0)

constexpr int kChains = 8;
constexpr int kThreads = 256;

struct Clocks {
    unsigned long long cyc, wall;
};

enum Op { OP_FMA, OP_MUL, OP_SUB, OP_EXP, OP_PAIR6, OP_PAIR4, OP_PAIR6_NOEXP, NUM_OPS };
static const char* kNames[NUM_OPS] = {"fma", "mul", "sub", "exp", "pair_r6", "pair_r4", "pair_r6_noexp"};
// VALU instructions (exp counted as one) per loop step of one chain
static const int kInsts[NUM_OPS] = {1, 1, 1, 1, 7, 7, 6};

template <int OP>
__global__ __launch_bounds__(kThreads) void k_loop(float* out, Clocks* clk, int iters, float seed) {
    float a[kChains], b[kChains];
    for (int c = 0; c < kChains; ++c) {
        a[c] = seed + 0.001f * (float)(threadIdx.x + c);
        b[c] = 0.25f + 0.0001f * (float)c;
    }
    float col = 0.0f;
    unsigned long long c0 = 0, w0 = 0;
    if (threadIdx.x == 0) {
        c0 = clock64();
        w0 = wall_clock64();
    }
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) {
            if constexpr (OP == OP_FMA) {
                a[c] = __builtin_fmaf(a[c], 0.999f, b[c]);
            } else if constexpr (OP == OP_MUL) {
                a[c] = a[c] * 0.999f;
            } else if constexpr (OP == OP_SUB) {
                a[c] = a[c] - b[c];
            } else if constexpr (OP == OP_EXP) {
                a[c] = __builtin_amdgcn_exp2f(-__builtin_fabsf(a[c]));
            } else if constexpr (OP == OP_PAIR6) {
                // a[c] is the lane's row value, b[c] its running sum; the column
                // value col changes every step, as an LDS column would
                const float d = a[c] - col;
                const float z = __builtin_fmaf(d, d, -5.0f);
                const float e = __builtin_amdgcn_exp2f(z * -0.72134752f);
                const float p = __builtin_fmaf(__builtin_fmaf(z, z, -30.0f), z, -40.0f);
                b[c] = __builtin_fmaf(p, e, b[c]);
            } else if constexpr (OP == OP_PAIR4) {
                const float d = a[c] - col;
                const float y = d * d;
                const float p = __builtin_fmaf(__builtin_fmaf(d, d, -6.0f), y, 3.0f);
                const float e = __builtin_amdgcn_exp2f(y * -0.72134752f);
                b[c] = __builtin_fmaf(p, e, b[c]);
            } else {
                const float d = a[c] - col;
                const float z = __builtin_fmaf(d, d, -5.0f);
                const float e = z * -0.72134752f;
                const float p = __builtin_fmaf(__builtin_fmaf(z, z, -30.0f), z, -40.0f);
                b[c] = __builtin_fmaf(p, e, b[c]);
            }
        }
        col += 0.0009765625f;
    }
    float s = 0.0f;
    for (int c = 0; c < kChains; ++c) s += a[c] + b[c];
    out[(size_t)blockIdx.x * kThreads + threadIdx.x] = s;
    if (threadIdx.x == 0) {
        clk[blockIdx.x].cyc = clock64() - c0;
        clk[blockIdx.x].wall = wall_clock64() - w0;
    }
}

template <int OP>
static void launch(int blocks, float* out, Clocks* clk, int iters, hipStream_t s) {
    hipLaunchKernelGGL(k_loop<OP>, dim3(blocks), dim3(kThreads), 0, s, out, clk, iters, 0.5f);
}

static void run(int op, int blocks, float* out, Clocks* clk, int iters, hipStream_t s) {
    switch (op) {
    case OP_FMA: launch<OP_FMA>(blocks, out, clk, iters, s); break;
    case OP_MUL: launch<OP_MUL>(blocks, out, clk, iters, s); break;
    case OP_SUB: launch<OP_SUB>(blocks, out, clk, iters, s); break;
    case OP_EXP: launch<OP_EXP>(blocks, out, clk, iters, s); break;
    case OP_PAIR6: launch<OP_PAIR6>(blocks, out, clk, iters, s); break;
    case OP_PAIR4: launch<OP_PAIR4>(blocks, out, clk, iters, s); break;
    default: launch<OP_PAIR6_NOEXP>(blocks, out, clk, iters, s); break;
    }
}

int main(int argc, char** argv) {
    std::vector<int> waves;
    for (int k = 1; k < argc; ++k) waves.push_back(std::atoi(argv[k]));
    if (waves.empty()) waves = {2, 3, 4, 8};
    hipDeviceProp_t prop;
    CHK(hipGetDeviceProperties(&prop, 0));
    const int cus = prop.multiProcessorCount;
    const int max_blocks = cus * 8;  // 8 waves per SIMD at 4 waves per block
    float* out = nullptr;
    Clocks* clk = nullptr;
    CHK(hipMalloc(&out, sizeof(float) * (size_t)max_blocks * kThreads));
    CHK(hipMalloc(&clk, sizeof(Clocks) * (size_t)max_blocks));
    std::vector<Clocks> hclk((size_t)max_blocks);
    hipStream_t s;
    CHK(hipStreamCreate(&s));
    hipEvent_t e0, e1;
    CHK(hipEventCreate(&e0));
    CHK(hipEventCreate(&e1));
    const int iters = 20000;
    std::printf("{\"device\": \"%s\", \"cus\": %d, \"threads_per_block\": %d, \"chains\": %d, \"iters\": %d, "
                "\"results\": [",
                prop.gcnArchName, cus, kThreads, kChains, iters);
    bool first = true;
    for (int w : waves) {
        if (w < 1 || w > 8) continue;
        const int blocks = cus * w;  // a block is 4 waves: w waves per SIMD
        for (int op = 0; op < NUM_OPS; ++op) {
            run(op, blocks, out, clk, iters, s);  // warm-up
            CHK(hipStreamSynchronize(s));
            float best = 1e30f;
            for (int rep = 0; rep < 5; ++rep) {
                CHK(hipEventRecord(e0, s));
                run(op, blocks, out, clk, iters, s);
                CHK(hipEventRecord(e1, s));
                CHK(hipEventSynchronize(e1));
                float ms = 0.0f;
                CHK(hipEventElapsedTime(&ms, e0, e1));
                if (ms < best) best = ms;
            }
            CHK(hipGetLastError());
            CHK(hipMemcpy(hclk.data(), clk, sizeof(Clocks) * (size_t)blocks, hipMemcpyDeviceToHost));
            double cyc = 0.0, wall = 0.0;
            for (int b = 0; b < blocks; ++b) {
                cyc += (double)hclk[(size_t)b].cyc;
                wall += (double)hclk[(size_t)b].wall;
            }
            const double sclk_mhz = wall > 0 ? 100.0 * cyc / wall : 0.0;
            const double steps = (double)blocks * kThreads * iters * kChains;  // lane loop steps
            const double lane_insts = steps * kInsts[op];
            std::printf("%s{\"waves_per_simd\": %d, \"op\": \"%s\", \"ms\": %.4f, \"lane_steps_per_s\": %.4e, "
                        "\"lane_insts_per_s\": %.4e, \"insts_per_cu_cycle\": %.3f, \"sclk_mhz\": %.1f}",
                        first ? "" : ", ", w, kNames[op], best, steps / (best * 1e-3),
                        lane_insts / (best * 1e-3),
                        sclk_mhz > 0 ? lane_insts / (best * 1e-3) / (cus * sclk_mhz * 1e6) : 0.0, sclk_mhz);
            first = false;
        }
    }
    std::printf("]}\n");
    CHK(hipFree(out));
    CHK(hipFree(clk));
    return 0;
}
