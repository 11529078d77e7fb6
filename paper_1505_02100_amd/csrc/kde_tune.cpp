// Autotuner of libkdeplugin's tile configuration.
//
// The persistent kernel has three free parameters that do not change any
// result's definition: rows per lane R (tile height 256 R), persistent blocks
// per CU, and the number of pair items a stage is cut into (which sets the
// item width W for each sample size).  R and the block count are fixed per
// context (they pick the kernel instantiation and grid); the item count is
// chosen per sample size.  For the FP32 precision there is a fourth: how
// 2^t is evaluated, on the transcendental unit (v_exp_f32) or by the Remez
// minimax polynomial on the FMA pipes (the paper's exponential); the two
// agree to rounding level, well inside the FP32 bound.  The search times
// complete selections of synthetic samples with HIP events around each
// launch and writes the best configuration as a table that kde_ctx_create
// reads back.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include <unistd.h>

#include "kdeplugin.h"

namespace {

// Synthetic timing samples: SplitMix64 uniforms through Box-Muller.  Their
// values only have to look like data; no result depends on them.
std::vector<double> normal_sample(int64_t n, uint64_t seed) {
    std::vector<double> x((size_t)n);
    uint64_t z = seed;
    auto next = [&z]() {
        z += 0x9E3779B97F4A7C15ull;
        uint64_t w = z;
        w = (w ^ (w >> 30)) * 0xBF58476D1CE4E5B9ull;
        w = (w ^ (w >> 27)) * 0x94D049BB133111EBull;
        w ^= w >> 31;
        return (double)(w >> 11) * (1.0 / 9007199254740992.0);
    };
    const double two_pi = 6.283185307179586;
    for (int64_t i = 0; i < n; i += 2) {
        const double u1 = 1.0 - next(), u2 = next();
        const double r = std::sqrt(-2.0 * std::log(u1));
        x[(size_t)i] = r * std::cos(two_pi * u2);
        if (i + 1 < n) x[(size_t)i + 1] = r * std::sin(two_pi * u2);
    }
    return x;
}

constexpr int kWarmupMs = 300;  // load before the first timed candidate

// Blocks per CU to try: 0 (the context's own choice: the occupancy limit, and
// the four-wave kernel for large samples where it has one), the occupancy
// limit, and one below it.  A table with 0 leaves the choice to the context.
std::vector<int> bpc_candidates(int occ) {
    std::vector<int> v{0, occ};
    if (occ > 1) v.push_back(occ - 1);
    return v;
}

// Median device time (ms) of `reps` selections on a context, or -1 on error.
double time_ctx(kde_ctx* c, const void* dx, int64_t n, int reps) {
    kde_result r;
    if (kde_plugin_bandwidth_ex(c, dx, n, KDE_MEM_DEVICE, KDE_F64, nullptr, &r) != KDE_OK) return -1.0;
    std::vector<double> t;
    for (int k = 0; k < reps; ++k) {
        if (kde_plugin_bandwidth_ex(c, dx, n, KDE_MEM_DEVICE, KDE_F64, nullptr, &r) != KDE_OK) return -1.0;
        t.push_back(kde_ctx_last_device_ms(c));
    }
    std::sort(t.begin(), t.end());
    return t[t.size() / 2];
}

int floor_log2(int64_t n) {
    int lg = 0;
    while (lg < 62 && ((int64_t)2 << lg) <= n) ++lg;
    return lg;
}

// Median device time (ms) of `reps` batch launches over samples dx[0..m).
double time_batch(kde_ctx* c, const std::vector<void*>& dx, const std::vector<int64_t>& ns, int reps) {
    std::vector<kde_result> out(ns.size());
    std::vector<const void*> xs(dx.begin(), dx.end());
    if (kde_plugin_bandwidth_batch(c, xs.data(), ns.data(), (int64_t)ns.size(), KDE_MEM_DEVICE, out.data(),
                                   nullptr) != KDE_OK)
        return -1.0;
    std::vector<double> t;
    for (int k = 0; k < reps; ++k) {
        if (kde_plugin_bandwidth_batch(c, xs.data(), ns.data(), (int64_t)ns.size(), KDE_MEM_DEVICE, out.data(),
                                       nullptr) != KDE_OK)
            return -1.0;
        t.push_back(kde_ctx_last_device_ms(c));
    }
    std::sort(t.begin(), t.end());
    return t[t.size() / 2];
}

int write_table(const char* out_path, int precision, int R, int bpc, double total,
                const std::vector<std::pair<int, int64_t>>& ent, int64_t budget, int exp_poly = -1) {
    FILE* f = std::fopen(out_path, "w");
    if (!f) return KDE_EINVAL;
    std::fprintf(f, "{\n \"precision\": %d,\n \"rows_per_lane\": %d,\n \"blocks_per_cu\": %d,\n", precision, R,
                 bpc);
    if (exp_poly >= 0) std::fprintf(f, " \"exp_poly\": %d,\n", exp_poly);
    std::fprintf(f, " \"total_ms\": %.6f,\n", total);
    if (budget > 0) {
        std::fprintf(f, " \"pair_budget\": %lld\n}\n", (long long)budget);
    } else {
        std::fprintf(f, " \"targets\": [");
        for (size_t q = 0; q < ent.size(); ++q)
            std::fprintf(f, "%s[%d, %lld]", q ? ", " : "", ent[q].first, (long long)ent[q].second);
        std::fprintf(f, "]\n}\n");
    }
    std::fclose(f);
    return KDE_OK;
}

}  // namespace

extern "C" int kde_autotune(const kde_options* opt, const int64_t* ns, int32_t count, int32_t mode,
                            int32_t reps, const char* out_path, int32_t verbose) {
    if (!ns || count < 1 || !out_path) return KDE_EINVAL;
    kde_options base;
    kde_options_init(&base);
    if (opt) base = *opt;
    base.tune_table = nullptr;
    if (reps < 1) reps = 5;
    std::vector<int64_t> sizes(ns, ns + count);
    for (int64_t n : sizes)
        if (n < 2) return KDE_EINVAL;
    if (hipSetDevice(base.device) != hipSuccess) return KDE_EDEVICE;
    // device copies of one timing sample per size
    std::vector<void*> dx(sizes.size(), nullptr);
    int st = KDE_OK;
    for (size_t q = 0; q < sizes.size() && st == KDE_OK; ++q) {
        std::vector<double> h = normal_sample(sizes[q], 1234 + q);
        if (hipMalloc(&dx[q], h.size() * 8) != hipSuccess ||
            hipMemcpy(dx[q], h.data(), h.size() * 8, hipMemcpyHostToDevice) != hipSuccess)
            st = KDE_EDEVICE;
    }
    // bring the GPU to its clock under load before anything is timed: the first
    // tens of milliseconds of load run at a lower clock, which made the first
    // candidates look slower than later ones
    if (st == KDE_OK) {
        kde_ctx* w = nullptr;
        if (kde_ctx_create(&w, &base) == KDE_OK) {
            size_t big = 0;
            for (size_t q = 1; q < sizes.size(); ++q)
                if (sizes[q] > sizes[big]) big = q;
            const auto t0 = std::chrono::steady_clock::now();
            kde_result r;
            for (int k = 0; k < 100000; ++k) {
                if (kde_plugin_bandwidth_ex(w, dx[big], sizes[big], KDE_MEM_DEVICE, KDE_F64, nullptr, &r) != KDE_OK)
                    break;
                if (std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(kWarmupMs)) break;
            }
            kde_ctx_destroy(w);
        }
    }
    const int Rs[] = {1, 2, 4};
    // the FP32 precision also tries the polynomial exponential (its kernels are
    // those of KDE_FP32_POLYEXP); other precisions have one way to evaluate it
    const bool try_poly = base.precision == KDE_FP32_COMP;
    const int exp_choices = try_poly ? 2 : 1;
    if (st == KDE_OK && mode == 1) {
        // batch objective: one launch over all samples; item size = pair budget
        const int64_t budgets[] = {1 << 18, 1 << 19, 1 << 20, 1 << 21, 1 << 22, 1 << 23};
        double bt = 1e300;
        int bR = 1, bB = 0, bP = 0;
        int64_t bbud = 0;
        for (int ep = 0; ep < exp_choices; ++ep)
        for (int R : Rs) {
            kde_options o = base;
            o.rows_per_lane = R;
            if (ep) o.precision = KDE_FP32_POLYEXP;
            kde_ctx* probe = nullptr;
            if (kde_ctx_create(&probe, &o) != KDE_OK) {
                st = KDE_EDEVICE;
                break;
            }
            int32_t occ = 1;
            kde_ctx_config(probe, nullptr, nullptr, nullptr, &occ);
            kde_ctx_destroy(probe);
            for (int bpc : bpc_candidates(occ)) {
                for (int64_t B : budgets) {
                    // a candidate is a table with this pair budget, read back by kde_ctx_create
                    char path[64];
                    std::snprintf(path, sizeof path, "/tmp/kde_tune_probe_%d.json", (int)getpid());
                    o.blocks_per_cu = bpc;
                    std::vector<std::pair<int, int64_t>> none;
                    if (write_table(path, o.precision, R, bpc, 0.0, none, B) != KDE_OK) continue;
                    kde_options ot = o;
                    ot.tune_table = path;
                    kde_ctx* c = nullptr;
                    if (kde_ctx_create(&c, &ot) != KDE_OK) continue;
                    const double ms = time_batch(c, dx, sizes, reps);
                    kde_ctx_destroy(c);
                    std::remove(path);
                    if (verbose)
                        std::fprintf(stderr, "autotune batch exp=%s R=%d bpc=%d budget=%lld: %.4f ms\n",
                                     ep ? "poly" : "hw", R, bpc, (long long)B, ms);
                    if (ms > 0 && ms < bt) {
                        bt = ms;
                        bR = R;
                        bB = bpc;
                        bbud = B;
                        bP = ep;
                    }
                }
            }
        }
        for (void* p : dx)
            if (p) (void)hipFree(p);
        if (st) return st;
        std::vector<std::pair<int, int64_t>> none;
        return write_table(out_path, base.precision, bR, bB, bt, none, bbud, try_poly ? bP : -1);
    }
    const int64_t targets[] = {1024, 2048, 4096, 8192, 16384, 32768, 65536};
    struct Best {
        double total = 1e300;
        int R = 1, bpc = 0, poly = 0;
        std::vector<int64_t> tgt;
    } best;
    for (int ep = 0; ep < exp_choices; ++ep)
    for (int R : Rs) {
        if (st) break;
        // blocks per CU: the occupancy limit and one below it
        kde_options o = base;
        o.rows_per_lane = R;
        if (ep) o.precision = KDE_FP32_POLYEXP;
        kde_ctx* probe = nullptr;
        if (kde_ctx_create(&probe, &o) != KDE_OK) {
            st = KDE_EDEVICE;
            break;
        }
        int32_t occ = 1;
        kde_ctx_config(probe, nullptr, nullptr, nullptr, &occ);
        kde_ctx_destroy(probe);
        for (int bpc : bpc_candidates(occ)) {
            double total = 0.0;
            std::vector<int64_t> tgt(sizes.size(), 0);
            for (size_t q = 0; q < sizes.size(); ++q) {
                double bt = 1e300;
                for (int64_t T : targets) {
                    o.blocks_per_cu = bpc;
                    o.target_items = (int32_t)T;
                    kde_ctx* c = nullptr;
                    if (kde_ctx_create(&c, &o) != KDE_OK) continue;
                    const double ms = time_ctx(c, dx[q], sizes[q], reps);
                    kde_ctx_destroy(c);
                    if (verbose)
                        std::fprintf(stderr, "autotune exp=%s R=%d bpc=%d n=%lld items=%lld: %.4f ms\n",
                                     ep ? "poly" : "hw", R, bpc, (long long)sizes[q], (long long)T, ms);
                    if (ms > 0 && ms < bt) {
                        bt = ms;
                        tgt[q] = T;
                    }
                }
                total += bt;
            }
            if (total < best.total) {
                best.total = total;
                best.R = R;
                best.bpc = bpc;
                best.tgt = tgt;
                best.poly = ep;
            }
        }
    }
    for (void* p : dx)
        if (p) (void)hipFree(p);
    if (st) return st;
    // one entry per measured size, keyed by floor(log2 n), in increasing order
    std::vector<std::pair<int, int64_t>> ent;
    for (size_t q = 0; q < sizes.size(); ++q) ent.emplace_back(floor_log2(sizes[q]), best.tgt[q]);
    std::sort(ent.begin(), ent.end());
    return write_table(out_path, base.precision, best.R, best.bpc, best.total, ent, 0, try_poly ? best.poly : -1);
}
