// Exercises libkdeplugin's host runtime through its C ABI, for a build whose
// host code carries AddressSanitizer and UndefinedBehaviorSanitizer (device
// code unchanged): contexts and their options, single, shard, batch
// (synchronous and asynchronous) and no-allocation calls on host and device
// samples, tune tables (written by the autotuner, and malformed ones), the
// server (admission, budget, cancellation, a failed step, draining), density
// evaluation, and the error paths.  Prints "host runtime under sanitizers:
// ok" and exits 0 when every call returned what it should; a sanitizer
// report aborts the process.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "kdeplugin.h"

static int g_fail = 0;
#define CHECK(c)                                                          \
    do {                                                                  \
        if (!(c)) {                                                       \
            std::fprintf(stderr, "check failed line %d: %s (%s)\n", __LINE__, #c, \
                         kde_last_error_message());                       \
            ++g_fail;                                                     \
        }                                                                 \
    } while (0)

// deterministic test samples (xorshift uniforms summed to a rough bell shape)
static std::vector<double> sample(int64_t n, uint64_t seed) {
    std::vector<double> x((size_t)n);
    uint64_t s = seed * 0x9E3779B97F4A7C15ull + 7;
    for (auto& v : x) {
        double t = 0;
        for (int k = 0; k < 4; ++k) {
            s ^= s << 13;
            s ^= s >> 7;
            s ^= s << 17;
            t += (double)(s >> 11) * 0x1.0p-53;
        }
        v = t - 2.0;
    }
    return x;
}

static double* to_device(const std::vector<double>& x) {
    double* d = nullptr;
    if (hipMalloc(&d, x.size() * sizeof(double)) != hipSuccess) return nullptr;
    if (hipMemcpy(d, x.data(), x.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) return nullptr;
    return d;
}

static void write_file(const std::string& path, const std::string& text) {
    FILE* f = std::fopen(path.c_str(), "wb");
    if (!f) return;
    std::fwrite(text.data(), 1, text.size(), f);
    std::fclose(f);
}

static void literal_calls() {
    auto x = sample(3000, 1);
    const double h = kde_plugin_bandwidth(x.data(), (int64_t)x.size());
    CHECK(std::isfinite(h) && h > 0);
    CHECK(kde_psi(x.data(), (int64_t)x.size(), 4, 0.3) > 0);
    CHECK(kde_psi(x.data(), 1, 6, 0.3) < 0);
    CHECK(std::isnan(kde_psi(x.data(), 0, 4, 0.3)));
    CHECK(std::isnan(kde_plugin_bandwidth(nullptr, 10)));
    std::vector<double> y = {-1, 0, 1}, f(3);
    CHECK(kde_eval(x.data(), (int64_t)x.size(), y.data(), 3, h, f.data()) == KDE_OK && f[1] > 0);
    for (int c = 1; c >= -8; --c) CHECK(kde_strerror(c) != nullptr);
}

static void context_calls(int prec) {
    kde_options o;
    kde_options_init(&o);
    o.precision = prec;
    kde_ctx* c = nullptr;
    CHECK(kde_ctx_create(&c, &o) == KDE_OK && c);
    if (!c) return;
    int32_t R = 0, bt = 0, tr = 0, bpc = 0;
    CHECK(kde_ctx_config(c, &R, &bt, &tr, &bpc) == KDE_OK && R >= 1 && bpc >= 1);
    for (int64_t n : {2, 3, 65, 257, 4097, 20000}) {
        auto x = sample(n, (uint64_t)n);
        kde_result r{};
        CHECK(kde_plugin_bandwidth_ex(c, x.data(), n, KDE_MEM_HOST, KDE_F64, nullptr, &r) == KDE_OK && r.h > 0);
        double* d = to_device(x);
        CHECK(d != nullptr);
        kde_result rd{};
        CHECK(kde_plugin_bandwidth_ex(c, d, n, KDE_MEM_DEVICE, KDE_F64, nullptr, &rd) == KDE_OK && rd.h == r.h);
        double ms[KDE_NUM_STAGES];
        CHECK(kde_ctx_last_timeline(c, 0, ms) == KDE_OK);
        CHECK(kde_ctx_last_timeline(c, 5, ms) == KDE_EINVAL);
        CHECK(kde_ctx_last_device_ms(c) >= 0);
        double p = 0;
        CHECK(kde_psi_ex(c, d, n, 6, 0.4, KDE_MEM_DEVICE, KDE_F64, nullptr, &p) == KDE_OK && p < 0);
        const int64_t items = kde_psi_num_items(c, n);
        CHECK(items >= 1);
        int64_t r0, r1, c0, c1;
        CHECK(kde_psi_item_geometry(c, n, items - 1, &r0, &r1, &c0, &c1) == KDE_OK && r1 <= n && c1 <= n);
        CHECK(kde_psi_item_geometry(c, n, items, &r0, &r1, &c0, &c1) == KDE_EINVAL);
        double part = 0;
        CHECK(kde_psi_range(c, d, n, 4, 0.4, KDE_MEM_DEVICE, KDE_F64, 0, items, nullptr, &part) == KDE_OK);
        CHECK(kde_psi_range(c, d, n, 4, 0.4, KDE_MEM_DEVICE, KDE_F64, 0, items + 1, nullptr, &part) == KDE_EINVAL);
        // no-allocation entry point: device and pinned results
        kde_result* dres = nullptr;
        kde_result* hres = nullptr;
        CHECK(hipMalloc(&dres, sizeof(kde_result)) == hipSuccess);
        CHECK(hipHostMalloc((void**)&hres, sizeof(kde_result), hipHostMallocDefault) == hipSuccess);
        CHECK(kde_plugin_bandwidth_noalloc(c, d, n, KDE_F64, nullptr, hres) == KDE_OK);
        CHECK(hipDeviceSynchronize() == hipSuccess);
        CHECK(hres->h == r.h);
        CHECK(kde_plugin_bandwidth_noalloc(c, d, n, KDE_F64, nullptr, dres) == KDE_OK);
        CHECK(kde_plugin_bandwidth_noalloc(c, x.data(), n, KDE_F64, nullptr, dres) == KDE_EINVAL);
        CHECK(kde_plugin_bandwidth_noalloc(c, d, n, KDE_F64, nullptr, &r) == KDE_EINVAL);
        CHECK(hipDeviceSynchronize() == hipSuccess);
        // density evaluation on host and device arrays
        std::vector<double> y = {-2, -0.5, 0, 0.5, 2}, f(5);
        CHECK(kde_eval_ex(c, d, n, KDE_MEM_DEVICE, KDE_F64, y.data(), 5, KDE_MEM_HOST, 0.3, nullptr, f.data()) ==
              KDE_OK);
        CHECK(kde_eval_ex(c, d, n, KDE_MEM_DEVICE, KDE_F64, y.data(), 5, KDE_MEM_HOST, -1.0, nullptr, f.data()) ==
              KDE_EINVAL);
        (void)hipFree(dres);
        (void)hipHostFree(hres);
        (void)hipFree(d);
    }
    // FP32 input, a NaN sample, a constant sample, bad arguments
    {
        std::vector<float> xf(1000);
        auto x = sample(1000, 3);
        for (size_t i = 0; i < xf.size(); ++i) xf[i] = (float)x[i];
        kde_result r{};
        CHECK(kde_plugin_bandwidth_ex(c, xf.data(), 1000, KDE_MEM_HOST, KDE_F32, nullptr, &r) == KDE_OK);
        x[500] = NAN;
        CHECK(kde_plugin_bandwidth_ex(c, x.data(), 1000, KDE_MEM_HOST, KDE_F64, nullptr, &r) == KDE_ENONFINITE);
        std::vector<double> k(50, 3.0);
        CHECK(kde_plugin_bandwidth_ex(c, k.data(), 50, KDE_MEM_HOST, KDE_F64, nullptr, &r) == KDE_EDEGENERATE);
        CHECK(kde_plugin_bandwidth_ex(c, x.data(), 1, KDE_MEM_HOST, KDE_F64, nullptr, &r) == KDE_EINVAL);
        CHECK(kde_plugin_bandwidth_ex(c, x.data(), 10, 7, KDE_F64, nullptr, &r) == KDE_EINVAL);
        double p;
        CHECK(kde_psi_ex(c, k.data(), 50, 4, 0.2, KDE_MEM_HOST, KDE_F64, nullptr, &p) == KDE_OK && p > 0);
        CHECK(kde_psi_ex(c, k.data(), 50, 5, 0.2, KDE_MEM_HOST, KDE_F64, nullptr, &p) == KDE_EINVAL);
    }
    // batches: host and device samples, invalid members, asynchronous results
    {
        std::vector<std::vector<double>> xs;
        std::vector<const void*> hp;
        std::vector<int64_t> ns;
        for (int k = 0; k < 24; ++k) {
            xs.push_back(sample(200 + 377 * k, 100 + (uint64_t)k));
            ns.push_back((int64_t)xs.back().size());
        }
        for (auto& v : xs) hp.push_back(v.data());
        std::vector<kde_result> out(xs.size());
        CHECK(kde_plugin_bandwidth_batch(c, hp.data(), ns.data(), (int64_t)xs.size(), KDE_MEM_HOST, out.data(),
                                         nullptr) == KDE_OK);
        for (auto& r : out) CHECK(r.status == KDE_OK && r.h > 0);
        std::vector<const void*> dp;
        for (auto& v : xs) dp.push_back(to_device(v));
        ns[3] = 1;                      // invalid member
        dp[5] = nullptr;                // invalid member
        std::vector<kde_result> out2(xs.size());
        CHECK(kde_plugin_bandwidth_batch(c, dp.data(), ns.data(), (int64_t)xs.size(), KDE_MEM_DEVICE, out2.data(),
                                         nullptr) == KDE_OK);
        CHECK(out2[3].status == KDE_EINVAL && out2[5].status == KDE_EINVAL && out2[4].h == out[4].h);
        kde_result* hres = nullptr;
        CHECK(hipHostMalloc((void**)&hres, sizeof(kde_result) * xs.size(), hipHostMallocDefault) == hipSuccess);
        hipStream_t st;
        CHECK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess);
        CHECK(kde_plugin_bandwidth_batch(c, dp.data(), ns.data(), (int64_t)xs.size(), KDE_MEM_DEVICE, hres,
                                         (kde_stream)st) == KDE_OK);
        CHECK(hipStreamSynchronize(st) == hipSuccess);
        for (size_t k = 0; k < xs.size(); ++k) CHECK(hres[k].status == out2[k].status && (k == 3 || k == 5 || hres[k].h == out2[k].h));
        CHECK(kde_plugin_bandwidth_batch(c, dp.data(), ns.data(), 0, KDE_MEM_DEVICE, out2.data(), nullptr) ==
              KDE_EINVAL);
        (void)hipStreamDestroy(st);
        (void)hipHostFree(hres);
        for (auto p : dp)
            if (p) (void)hipFree((void*)p);
    }
    kde_ctx_destroy(c);
}

static void options_and_tune_tables(const std::string& dir) {
    kde_options o;
    kde_options_init(&o);
    kde_ctx* c = nullptr;
    o.precision = 9;
    CHECK(kde_ctx_create(&c, &o) == KDE_EINVAL);
    kde_options_init(&o);
    o.rows_per_lane = 3;
    CHECK(kde_ctx_create(&c, &o) == KDE_EINVAL);
    kde_options_init(&o);
    o.device = 99;
    CHECK(kde_ctx_create(&c, &o) == KDE_EINVAL);
    CHECK(kde_ctx_create(nullptr, nullptr) == KDE_EINVAL);
    // a table written by the autotuner, then read back
    const std::string tuned = dir + "/san_tune.json";
    kde_options_init(&o);
    o.precision = KDE_FP32_COMP;
    const int64_t ns[2] = {300, 2000};
    CHECK(kde_autotune(&o, ns, 2, KDE_TUNE_SINGLE, 1, tuned.c_str(), 0) == KDE_OK);
    o.tune_table = tuned.c_str();
    CHECK(kde_ctx_create(&c, &o) == KDE_OK);
    if (c) {
        auto x = sample(2000, 9);
        kde_result r{};
        CHECK(kde_plugin_bandwidth_ex(c, x.data(), 2000, KDE_MEM_HOST, KDE_F64, nullptr, &r) == KDE_OK);
        kde_ctx_destroy(c);
        c = nullptr;
    }
    // malformed tables are rejected, not read past their end
    const char* bad[] = {"", "{", "{\"targets\": [[3, 100]", "{\"targets\": [[3, 100], [x, y]]}",
                         "{\"rows_per_lane\": 3}", "{\"blocks_per_cu\": 99}", "{\"precision\": 0}",
                         "{\"targets\": [[", "\"targets\"]]"};
    int k = 0;
    for (const char* t : bad) {
        const std::string p = dir + "/san_bad" + std::to_string(k++) + ".json";
        write_file(p, t);
        o.tune_table = p.c_str();
        const int st = kde_ctx_create(&c, &o);
        if (st == KDE_OK) {
            kde_ctx_destroy(c);  // a table without errors is accepted
            c = nullptr;
        } else {
            CHECK(st == KDE_EINVAL);
        }
    }
    o.tune_table = "/nonexistent/table.json";
    CHECK(kde_ctx_create(&c, &o) == KDE_EINVAL);
}

static void server_calls() {
    kde_options o;
    kde_options_init(&o);
    o.precision = KDE_FP32_COMP;
    kde_ctx* c = nullptr;
    CHECK(kde_ctx_create(&c, &o) == KDE_OK);
    if (!c) return;
    for (int fill : {KDE_FILL_SHARE, KDE_FILL_PRIORITY}) {
        kde_server_options so;
        kde_server_options_init(&so);
        so.mem_budget = 4 << 20;
        so.max_active = 4;
        so.step_pairs = 1 << 24;
        so.policy = fill == KDE_FILL_PRIORITY ? KDE_SERVE_SJF : KDE_SERVE_FCFS;
        so.aging_ms = 5;
        so.fill = fill;
        kde_server* s = nullptr;
        CHECK(kde_server_create(&s, c, &so) == KDE_OK);
        if (!s) continue;
        std::vector<std::vector<double>> xs;
        for (int k = 0; k < 10; ++k) xs.push_back(sample(500 + 1500 * k, 40 + (uint64_t)k));
        double* d = to_device(xs[9]);
        std::vector<int64_t> ids;
        for (auto& v : xs) {
            int64_t id = 0;
            CHECK(kde_server_submit(s, v.data(), (int64_t)v.size(), KDE_MEM_HOST, nullptr, &id) == KDE_OK);
            ids.push_back(id);
        }
        int64_t idd = 0;
        CHECK(kde_server_submit(s, d, (int64_t)xs[9].size(), KDE_MEM_DEVICE, nullptr, &idd) == KDE_OK);
        std::vector<double> huge_host(1);
        int64_t idh = 0;
        CHECK(kde_server_submit(s, huge_host.data(), (int64_t)1 << 30, KDE_MEM_HOST, nullptr, &idh) == KDE_ENOMEM);
        CHECK(kde_server_cancel(s, ids.back()) == KDE_OK);
        kde_server_stats st{};
        CHECK(kde_server_step(s, 0, &st) == KDE_OK);
        CHECK(kde_server_fail_next_step(s, KDE_EDEVICE) == KDE_OK);
        CHECK(kde_server_fail_next_step(s, 1) == KDE_EINVAL);
        CHECK(kde_server_step(s, 1, &st) == KDE_OK);
        CHECK(kde_server_drain(s) == KDE_OK);
        std::vector<kde_completion> done(64);
        int32_t got = 0;
        CHECK(kde_server_poll(s, done.data(), 64, &got) == KDE_OK);
        CHECK(got == 10);  // 11 submitted, one cancelled
        int ok = 0, failed = 0;
        for (int q = 0; q < got; ++q) {
            if (done[(size_t)q].result.status == KDE_OK)
                ++ok;
            else if (done[(size_t)q].result.status == KDE_EDEVICE)
                ++failed;
        }
        CHECK(ok + failed == got && failed >= 1);
        CHECK(kde_server_cancel(s, ids[0]) == KDE_EBUSY);
        kde_server_destroy(s);
        (void)hipFree(d);
    }
    kde_server_options bad;
    kde_server_options_init(&bad);
    bad.fill = 7;
    kde_server* s = nullptr;
    CHECK(kde_server_create(&s, c, &bad) == KDE_EINVAL);
    kde_ctx_destroy(c);
}

int main(int argc, char** argv) {
    const std::string dir = argc > 1 ? argv[1] : "/tmp";
    literal_calls();
    context_calls(KDE_FP64_PLAIN);
    context_calls(KDE_FP32_COMP);
    options_and_tune_tables(dir);
    server_calls();
    // Leave without running the HIP runtime's own teardown: a kernel that
    // spills registers makes the runtime hold scratch memory, and releasing it
    // from the runtime's exit handlers trips AddressSanitizer's device
    // allocator after the runtime has been marked unloaded (an ordering
    // between the sanitizer and the runtime, after every check here has run).
    if (g_fail) {
        std::fprintf(stderr, "%d checks failed\n", g_fail);
        std::fflush(stderr);
        std::_Exit(1);
    }
    std::printf("host runtime under sanitizers: ok\n");
    std::fflush(stdout);
    std::_Exit(0);
}
