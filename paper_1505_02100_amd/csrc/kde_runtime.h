// Host-side internals shared by the translation units of libkdeplugin's
// runtime (contexts, plans, the work decomposition, the server).  Not part of
// the public interface.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <list>
#include <memory>
#include <string>
#include <vector>

#include "kde_internal.h"

namespace kde {
hipError_t launch_init(State* states, Pub* pubs, int32_t count, uint32_t* ticket, hipStream_t s);
hipError_t launch_results(const State* states, const int32_t* outmap, int64_t n_out, kde_result* out,
                          hipStream_t s);
// The persistent kernel for (precision, R), held to three waves per SIMD, or
// (wide) to four, which only the default precision at R = 1 has.
bool wide_available(int prec, int R);
hipError_t launch_persistent(int prec, int R, bool wide, int grid, hipStream_t s, const LaunchArgs& a);
// The instantiation itself, for graph nodes; nullptr if none.
const void* persistent_kernel(int prec, int R, bool wide);
hipError_t persistent_occupancy(int prec, int R, bool wide, int* blocks_per_cu);
}  // namespace kde

namespace kde {
namespace rt {

// Thread-local last error (kde_last_error / kde_last_error_message).
int set_err(int code, const std::string& msg);
int ok();
int hip_fail(hipError_t e, const char* what);

#define HIPCHK(call)                                           \
    do {                                                       \
        hipError_t _e = (call);                                \
        if (_e != hipSuccess) return ::kde::rt::hip_fail(_e, #call); \
    } while (0)

constexpr int kBlock = 256;             // threads per block of the persistent kernel
constexpr int64_t kMomentChunk = 2048;  // elements per moment item (8 per thread)
constexpr uint64_t kTimeoutTicks = 20ull * 100000000ull;  // 20 s at the 100 MHz wall clock
// A wait for an earlier stage's flag lasts at most as long as that stage's
// slowest item still in flight (plus its finaliser), so the bound adds the
// time of the launch's largest pair item at kSlowPairsPerS, a per-block rate
// far below any measured one: huge samples, whose items take seconds, are
// not cut off, and a hang still ends.
constexpr double kSlowPairsPerS = 2e7;
// Launches whose pair stage holds at least this many pairs (over all their
// samples) run on the four-wave kernel when the context chose its own tile
// configuration.  Measured on MI355X against the three-wave kernel: -1.6% at
// n = 2^20, -1.2% at 2^19, -1.4% at 2^18 (3.4e10 pairs), equal at 2^17
// (8.6e9), +0.8% at 2^16 with three blocks per CU and +3% with four (2.1e9:
// the stage ends and the spill code weigh more there), -1.6% for the
// 512-sample batch (1e11 pairs per stage in one launch).
constexpr double kWideMinPairs = 17179869184.0;  // 2^34
// Pair items of samples this large (FP64 sample of 4 MiB, an XCD's L2) are
// listed band-wise, chunk-major inside bands of kBandRows row blocks.
constexpr int64_t kBandMinN = (int64_t)1 << 19;
constexpr int64_t kBandRows = 512;

// Grow-only device buffer.
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
    int ensure(size_t need, const char* what);
};

// Everything one launch of the persistent kernel needs for a fixed shape.
struct Plan {
    std::string key;
    int32_t count = 0;                // samples
    std::vector<Item> items;
    std::vector<Desc> descs;          // host copy of what is on the device
    DevBuf d_items, d_descs, d_states, d_pubs, d_slots, d_ticket;
    State* h_states = nullptr;        // pinned
    Desc* h_descs = nullptr;          // pinned staging of descriptor uploads
    bool descs_dirty = true;          // descs differ from what the device holds
    hipEvent_t ev_upload = nullptr;   // recorded after the last upload from h_descs
    // Batch results written on the device (asynchronous batch calls): out[k]
    // takes the state of sample outmap[2k] >= 0, or the status outmap[2k + 1]
    // of a sample the host already rejected.
    std::vector<int32_t> outmap;
    DevBuf d_outmap;
    int64_t n_slots = 0;
    hipGraphExec_t exec = nullptr;
    bool primed = false;              // states reset once before the first replay
    hipEvent_t ev_reset = nullptr;    // recorded after the reset that follows each replay
    hipStream_t reset_stream = nullptr;  // the stream that reset was issued on
    int grid = 0;
    bool wide = false;                // launched with the four-wave kernel
    ~Plan() {
        // a replay may still be in flight (asynchronous calls): let it finish
        if (ev_reset) (void)hipEventSynchronize(ev_reset);
        if (exec) (void)hipGraphExecDestroy(exec);
        if (ev_reset) (void)hipEventDestroy(ev_reset);
        if (ev_upload) (void)hipEventDestroy(ev_upload);
        if (h_states) (void)hipHostFree(h_states);
        if (h_descs) (void)hipHostFree(h_descs);
    }
    size_t device_bytes() const {
        return d_items.bytes + d_descs.bytes + d_states.bytes + d_pubs.bytes + d_slots.bytes + d_ticket.bytes +
               d_outmap.bytes;
    }
};

// Pair-item decomposition of the strict upper triangle for a sample of size n.
struct PairGeom {
    int64_t n, TI, W, RB;
};

// One sample of a launch.
struct SampleSpec {
    const void* x;
    int64_t n;
    int32_t dtype;
    int32_t mode;
    int32_t psi_r;
    double psi_g;
    int64_t item_begin, item_end;  // pair-item range (MODE_PSI); [0, -1) = all
};

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev);
    ~DeviceGuard();
};

PolyConsts make_consts();
int64_t moment_chunk(int64_t n);
int64_t pair_items_in_row(const PairGeom& g, int64_t rb);
int64_t pair_chunk_width(const PairGeom& g, int64_t rb);
int64_t pair_item_count(const PairGeom& g);
bool pair_item_at(const PairGeom& g, int64_t k, int64_t* rb, int64_t* cb);
void fill_result(const State& s, kde_result* r);
int check_x(const void* x, int64_t n, int64_t nmin, int mem_kind, int dtype);

}  // namespace rt
}  // namespace kde

struct kde_ctx {
    std::vector<kde::State> last_states;      // device state records of the last call
    hipEvent_t ev0 = nullptr, ev1 = nullptr;  // bracket each launch on the caller's stream
    double last_device_ms = -1.0;             // init + persistent kernel time of the last call
    int device = 0;
    int precision = KDE_FP64_PLAIN;
    int64_t mem_budget = 0;
    int R = 1;
    int blocks_per_cu = 0;
    int blocks_per_cu_wide = 0;               // > 0: large samples use the four-wave kernel with this many blocks per CU
    int last_grid = 0, last_waves = 0;        // launch shape of the last synchronous call
    int64_t target_items = 0;                 // 0 = by sample size
    int64_t bucket_target[64] = {0};          // from a tune table: by floor(log2 n)
    int64_t pair_budget = 0;                  // from a tune table: pairs per item for every n
    int cus = 0;
    kde::PolyConsts pc{};
    std::list<std::unique_ptr<kde::rt::Plan>> plans;  // most recently used first
    size_t max_plans = 16;
    kde::rt::DevBuf x_stage;                  // host samples copied here
    kde::rt::DevBuf ev_y, ev_out, ev_part, ev_flag;  // density evaluation buffers
    int64_t eval32_resident = 0;              // FP32 evaluation blocks the device holds at once (0: not yet asked)
    uint64_t wait_limit_ticks = 0;            // kde_options.wait_limit_us in wall-clock ticks; 0 = by item size
};

namespace kde {
namespace rt {
// The wall-clock bound of an in-kernel wait for a launch whose largest pair
// item has max_item_pairs pairs: the context's own limit, else kTimeoutTicks
// plus that item's time at kSlowPairsPerS.
inline uint64_t wait_ticks(const kde_ctx* c, int64_t max_item_pairs) {
    if (c->wait_limit_ticks) return c->wait_limit_ticks;
    return kTimeoutTicks + (uint64_t)((double)max_item_pairs / kSlowPairsPerS * 1e8);
}
PairGeom pair_geom(const kde_ctx* c, int64_t n);
int grid_for(const kde_ctx* c, int64_t work, bool wide);
// Whether a launch whose pair stage holds stage_pairs pairs takes the four-wave kernel.
inline bool use_wide(const kde_ctx* c, double stage_pairs) {
    return c->blocks_per_cu_wide > 0 && stage_pairs >= kWideMinPairs;
}
// Items of one sample, stage by stage, appended to `out` (slot numbers from
// slot_base[] of `d`, which must already be filled).  Used by the server.
void sample_items(const kde_ctx* c, int32_t ds, const Desc& d, const SampleSpec& ss,
                  std::vector<Item>* per_stage);
// Fill the descriptor of one sample (everything but slot_base) and return the
// number of slots it needs.
int64_t describe_sample(const kde_ctx* c, const SampleSpec& ss, Desc* d);
// Device-accessible address of a result buffer (device memory on the
// context's GPU, or pinned host memory), or nullptr.
kde_result* device_view(const kde_ctx* c, kde_result* out);
bool on_device(const kde_ctx* c, const void* p);
// Take the device address of the no-allocation scratch on `device` (once per
// device; kde_ctx_create calls it).
int noalloc_init(int device);
}  // namespace rt
}  // namespace kde
