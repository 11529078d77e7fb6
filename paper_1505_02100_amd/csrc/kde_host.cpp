// Host runtime and C ABI of libkdeplugin.
//
// A context owns a small cache of "plans".  A plan is everything one launch
// of the persistent kernel needs for a fixed problem shape: the ordered work
// list, the per-sample descriptors, state records, partial-sum slots, the
// work ticket, and a hipGraph (persistent kernel + state read-back) that is
// replayed whenever the same shape comes back, followed by the init kernel
// that readies the states for the next call.  Only the descriptors (sample
// pointers) are refreshed between replays, and only when they changed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <list>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "kde_eval.h"
#include "kde_runtime.h"

using namespace kde;

namespace kde {
namespace rt {

// ----------------------------------------------------------------- errors
namespace {
thread_local int t_err = KDE_OK;
thread_local std::string t_msg;
}  // namespace

int set_err(int code, const std::string& msg) {
    t_err = code;
    t_msg = msg;
    return code;
}
int ok() {
    t_err = KDE_OK;
    t_msg.clear();
    return KDE_OK;
}
int hip_fail(hipError_t e, const char* what) {
    return set_err(KDE_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}
int last_error_code() { return t_err; }
const char* last_error_text() { return t_msg.c_str(); }

const double kPi = 3.14159265358979323846;

int DevBuf::ensure(size_t need, const char* what) {
    if (need <= bytes) return KDE_OK;
    if (p) {
        (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    hipError_t e = hipMalloc(&p, need);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return set_err(KDE_ENOMEM, std::string("hipMalloc ") + what + ": " + hipGetErrorString(e));
    }
    bytes = need;
    return KDE_OK;
}

PolyConsts make_consts() {
    // exp(-y^2/2) = 2^(-k y^2) with k = log2(e)/2 (see kde_device.hip)
    const double k = 0.5 / std::log(2.0);
    PolyConsts pc{};
    pc.k_hi = (float)k;
    pc.k_lo = (float)(k - (double)pc.k_hi);
    return pc;
}

DeviceGuard::DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
}
DeviceGuard::~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
}

// Pair work items per stage: small samples favour fewer, larger items (less
// per-item latency), large ones more items (a shorter tail at the end of each
// stage).  Measured on MI355X for the FP32 kernel with 256-row tiles; a
// context option or tune table overrides it.
int64_t target_items_for(const kde_ctx* c, int64_t n) {
    if (c->pair_budget > 0) {
        const double P = 0.5 * (double)n * (double)(n - 1);
        return std::max<int64_t>(1, (int64_t)(P / (double)c->pair_budget));
    }
    if (c->target_items > 0) return c->target_items;
    int lg = 0;
    while (lg < 62 && ((int64_t)2 << lg) <= n) ++lg;
    for (int b = lg; b >= 0; --b)
        if (c->bucket_target[b] > 0) return c->bucket_target[b];
    // about n/32 items per stage, i.e. chunks of about n/16 columns (rounded
    // up to a power of two) for 256-row tiles; up to n = 2048 the narrowest
    // chunks (1024 items), and at most 65536 so the work list stays small
    // (beyond n = 2^18 the count hardly matters)
    if (n <= 2048) return 1024;
    return std::min<int64_t>(65536, (n + 31) / 32);
}

// Tune table (written by kde_autotune): a small JSON object
//   {"precision": p, "rows_per_lane": R, "blocks_per_cu": b,
//    "targets": [[log2n, items], ...]}          (tuned per sample size), or
//   {..., "pair_budget": B}                     (tuned for batches)
// A [log2n, items] entry applies to samples with floor(log2 n) >= log2n up
// to the next entry; a pair budget sizes every sample's items to about B
// pairs.
struct TuneTable {
    int precision = -1, R = 0, bpc = 0;
    int exp_poly = -1;  // FP32: 1 = the polynomial exponential won the search
    int64_t bucket[64] = {0};
    int64_t pair_budget = 0;
};

bool json_int(const std::string& t, const char* key, long long* v) {
    const size_t k = t.find(std::string("\"") + key + "\"");
    if (k == std::string::npos) return false;
    const size_t c = t.find(':', k);
    if (c == std::string::npos) return false;
    char* end = nullptr;
    *v = std::strtoll(t.c_str() + c + 1, &end, 10);
    return end != t.c_str() + c + 1;
}

int load_tune_table(const char* path, TuneTable* tt) {
    FILE* f = std::fopen(path, "rb");
    if (!f) return set_err(KDE_EINVAL, std::string("cannot open tune table ") + path);
    std::string t;
    char buf[4096];
    size_t r;
    while ((r = std::fread(buf, 1, sizeof buf, f)) > 0) t.append(buf, r);
    std::fclose(f);
    long long v;
    if (json_int(t, "precision", &v)) tt->precision = (int)v;
    if (json_int(t, "rows_per_lane", &v)) tt->R = (int)v;
    if (json_int(t, "blocks_per_cu", &v)) tt->bpc = (int)v;
    if (json_int(t, "pair_budget", &v)) tt->pair_budget = v;
    if (json_int(t, "exp_poly", &v)) tt->exp_poly = (int)v;
    const size_t k = t.find("\"targets\"");
    if (k != std::string::npos) {
        const size_t open = t.find('[', k);
        const size_t close = t.find("]]", k);
        if (open == std::string::npos || close == std::string::npos || close < open)
            return set_err(KDE_EINVAL, std::string("malformed targets in tune table ") + path);
        size_t pos = open + 1;
        while (pos < close) {
            const size_t lb = t.find('[', pos);
            if (lb == std::string::npos || lb > close) break;
            long long lg = -1, items = 0;
            if (std::sscanf(t.c_str() + lb, "[%lld , %lld]", &lg, &items) != 2)
                return set_err(KDE_EINVAL, std::string("malformed targets in tune table ") + path);
            if (lg >= 0 && lg < 64 && items > 0) tt->bucket[lg] = items;
            pos = t.find(']', lb);
            if (pos == std::string::npos) break;
            ++pos;
        }
    }
    if ((tt->R != 0 && tt->R != 1 && tt->R != 2 && tt->R != 4) || tt->bpc < 0 || tt->bpc > 16 ||
        tt->exp_poly < -1 || tt->exp_poly > 1 || (tt->exp_poly == 1 && tt->precision != KDE_FP32_COMP))
        return set_err(KDE_EINVAL, std::string("malformed tune table ") + path);
    return KDE_OK;
}

PairGeom pair_geom(const kde_ctx* c, int64_t n) {
    PairGeom g{};
    g.n = n;
    g.TI = (int64_t)kBlock * c->R;
    g.RB = (n + g.TI - 1) / g.TI;
    const double P = 0.5 * (double)n * (double)(n - 1);
    const double want = P / ((double)g.TI * (double)std::max<int64_t>(1, target_items_for(c, n)));
    int64_t W = 64;
    while ((double)W < want && W < ((int64_t)1 << 40)) W <<= 1;
    g.W = W;
    return g;
}

// Row block rb's columns [rb TI, n) in chunks (row_chunks; the device
// computes the same widths).
int64_t pair_items_in_row(const PairGeom& g, int64_t rb) {
    int64_t m, w;
    row_chunks(g.n, rb * g.TI, g.W, &m, &w);
    return m;
}

int64_t pair_chunk_width(const PairGeom& g, int64_t rb) {
    int64_t m, w;
    row_chunks(g.n, rb * g.TI, g.W, &m, &w);
    return w;
}

int64_t pair_item_count(const PairGeom& g) {
    int64_t tot = 0;
    for (int64_t rb = 0; rb < g.RB; ++rb) tot += pair_items_in_row(g, rb);
    return tot;
}

// Item k of the pair enumeration (row-block major) -> (rb, cb).
bool pair_item_at(const PairGeom& g, int64_t k, int64_t* rb, int64_t* cb) {
    for (int64_t r = 0; r < g.RB; ++r) {
        const int64_t m = pair_items_in_row(g, r);
        if (k < m) {
            *rb = r;
            *cb = k;
            return true;
        }
        k -= m;
    }
    return false;
}

int64_t moment_chunk(int64_t n) {
    // at most 4096 moment items per sample
    return std::max<int64_t>(kMomentChunk, (n + 4095) / 4096);
}

int64_t describe_sample(const kde_ctx* c, const SampleSpec& ss, Desc* d) {
    *d = Desc{};
    d->x = ss.x;
    d->n = ss.n;
    d->dtype = ss.dtype;
    d->mode = ss.mode;
    d->psi_r = ss.psi_r;
    d->psi_g = ss.psi_g;
    d->chunk = (int32_t)moment_chunk(ss.n);
    const PairGeom g = pair_geom(c, ss.n);
    d->W = g.W;
    const int64_t nm = (ss.n + d->chunk - 1) / d->chunk;
    d->n_items[ST_SUM] = (int32_t)nm;
    d->n_items[ST_SSQ] = (int32_t)nm;
    const int64_t np = pair_item_count(g);
    if (ss.mode == MODE_PLUGIN) {
        d->n_items[ST_PSI6] = (int32_t)np;
        d->n_items[ST_PSI4] = (int32_t)np;
    } else {
        const int64_t b = std::max<int64_t>(0, ss.item_begin);
        const int64_t e = ss.item_end < 0 ? np : std::min(np, ss.item_end);
        const int st = ss.psi_r == 6 ? ST_PSI6 : ST_PSI4;
        d->n_items[st] = (int32_t)std::max<int64_t>(0, e - b);
    }
    int64_t slots = 0;
    for (int s = 0; s < NUM_STAGES; ++s) slots += d->n_items[s];
    return slots;
}

void sample_items(const kde_ctx* c, int32_t ds, const Desc& d, const SampleSpec& ss,
                  std::vector<Item>* per_stage) {
    for (int s = 0; s < NUM_STAGES; ++s) {
        std::vector<Item>& out = per_stage[s];
        const int32_t cnt = d.n_items[s];
        if (cnt == 0) continue;
        int32_t wait = -1;
        if (s == ST_SSQ) wait = ST_SUM;
        if (s == ST_PSI6) wait = ST_SSQ;
        if (s == ST_PSI4) wait = d.mode == MODE_PLUGIN ? ST_PSI6 : ST_SSQ;
        if (s == ST_SUM || s == ST_SSQ) {
            for (int32_t q = 0; q < cnt; ++q) out.push_back(Item{ds, s, wait, q, 0, 0, d.slot_base[s] + q});
        } else if (d.mode == MODE_PLUGIN && d.n >= kBandMinN) {
            // large samples: bands of kBandRows row blocks, chunk-major inside
            // a band (the blocks in flight then share a few column chunks,
            // which each XCD's L2 holds), the last band row-major (its small
            // items end the stage)
            const PairGeom g = pair_geom(c, d.n);
            int32_t q = 0;
            for (int64_t b0 = 0; b0 < g.RB; b0 += kBandRows) {
                const int64_t b1 = std::min<int64_t>(g.RB, b0 + kBandRows);
                if (b1 == g.RB) {
                    for (int64_t rb = b0; rb < b1; ++rb)
                        for (int64_t cb = 0, m = pair_items_in_row(g, rb); cb < m; ++cb)
                            out.push_back(Item{ds, s, wait, (int32_t)rb, (int32_t)cb, 0, d.slot_base[s] + q++});
                } else {
                    int64_t mmax = 0;  // chunks per row change at the width levels
                    for (int64_t rb = b0; rb < b1; ++rb) mmax = std::max(mmax, pair_items_in_row(g, rb));
                    for (int64_t cb = 0; cb < mmax; ++cb)
                        for (int64_t rb = b0; rb < b1; ++rb)
                            if (cb < pair_items_in_row(g, rb))
                                out.push_back(Item{ds, s, wait, (int32_t)rb, (int32_t)cb, 0, d.slot_base[s] + q++});
                }
            }
        } else {
            const PairGeom g = pair_geom(c, d.n);
            const int64_t first = d.mode == MODE_PLUGIN ? 0 : std::max<int64_t>(0, ss.item_begin);
            int64_t rb = 0, cb = 0;
            pair_item_at(g, first, &rb, &cb);
            for (int32_t q = 0; q < cnt; ++q) {
                out.push_back(Item{ds, s, wait, (int32_t)rb, (int32_t)cb, 0, d.slot_base[s] + q});
                if (++cb >= pair_items_in_row(g, rb)) {
                    ++rb;
                    cb = 0;
                }
            }
        }
    }
}

// Build the ordered work list: stage-major over samples (largest first), so
// that every item a later stage waits on is handed out long before it.
void build_items(const kde_ctx* c, Plan& p, const std::vector<SampleSpec>& ss) {
    const int32_t m = (int32_t)ss.size();
    p.count = m;
    p.descs.assign(m, Desc{});
    std::vector<int32_t> order(m);
    for (int32_t k = 0; k < m; ++k) order[k] = k;
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t a, int32_t b) { return ss[a].n > ss[b].n; });
    int64_t slot = 0;
    for (int32_t k = 0; k < m; ++k) {
        describe_sample(c, ss[k], &p.descs[k]);
        for (int s = 0; s < NUM_STAGES; ++s) {  // slots: contiguous per (sample, stage)
            p.descs[k].slot_base[s] = slot;
            slot += p.descs[k].n_items[s];
        }
    }
    p.n_slots = slot;
    std::vector<Item> per_stage[NUM_STAGES];
    for (int32_t oi = 0; oi < m; ++oi) sample_items(c, order[oi], p.descs[order[oi]], ss[order[oi]], per_stage);
    p.items.clear();
    p.items.reserve((size_t)slot);
    for (int s = 0; s < NUM_STAGES; ++s) p.items.insert(p.items.end(), per_stage[s].begin(), per_stage[s].end());
    // runs of consecutive items of one (sample, stage): a block counts its
    // finished items of a run once its next ticket lies past the run
    const int64_t total = (int64_t)p.items.size();
    for (int64_t e = total; e > 0;) {
        int64_t b = e - 1;
        while (b > 0 && p.items[b - 1].ds == p.items[e - 1].ds && p.items[b - 1].stage == p.items[e - 1].stage) --b;
        for (int64_t q = b; q < e; ++q) p.items[q].run_end = (int32_t)e;
        e = b;
    }
}

// Persistent blocks for a launch whose widest stage has `work` items: the
// context's blocks per CU on every CU, but no more than half that many items
// (blocks of a small launch then take two items per stage, and the CUs keep
// some of their VALU share for the others) and never more than there are items.
int grid_for(const kde_ctx* c, int64_t work, bool wide) {
    const int64_t full = (int64_t)c->cus * std::max(1, wide ? c->blocks_per_cu_wide : c->blocks_per_cu);
    const int64_t w = std::max<int64_t>(1, work);
    return (int)std::min(full, std::max(std::min<int64_t>(c->cus, w), w / 2));
}

int total_plan_bytes(const kde_ctx* c, size_t extra, size_t* out) {
    size_t tot = extra + c->x_stage.bytes + c->ev_y.bytes + c->ev_out.bytes + c->ev_part.bytes + c->ev_flag.bytes;
    for (auto& p : c->plans) tot += p->device_bytes();
    *out = tot;
    return KDE_OK;
}

// Allocate and upload a freshly built plan; the work list goes up on the
// call's stream, ahead of the plan's first launch there.
int upload_plan(kde_ctx* c, Plan& p, hipStream_t s) {
    const size_t need = sizeof(Item) * std::max<size_t>(1, p.items.size()) +
                        sizeof(Desc) * std::max(1, p.count) + sizeof(State) * std::max(1, p.count) +
                        sizeof(Pub) * kPubReplicas * std::max(1, p.count) +
                        sizeof(Slot) * (size_t)std::max<int64_t>(1, p.n_slots) + 256;
    if (c->mem_budget > 0) {
        size_t have = 0;
        total_plan_bytes(c, need, &have);
        while (have > (size_t)c->mem_budget && !c->plans.empty()) {
            c->plans.pop_back();  // evict least recently used
            total_plan_bytes(c, need, &have);
        }
        if (have > (size_t)c->mem_budget)
            return set_err(KDE_ENOMEM, "work list and partial sums exceed the context's memory budget");
    }
    int st;
    if ((st = p.d_items.ensure(sizeof(Item) * std::max<size_t>(1, p.items.size()), "work list"))) return st;
    if ((st = p.d_descs.ensure(sizeof(Desc) * std::max(1, p.count), "descriptors"))) return st;
    if ((st = p.d_states.ensure(sizeof(State) * std::max(1, p.count), "states"))) return st;
    if ((st = p.d_pubs.ensure(sizeof(Pub) * kPubReplicas * std::max(1, p.count), "published scalars"))) return st;
    if ((st = p.d_slots.ensure(sizeof(Slot) * (size_t)std::max<int64_t>(1, p.n_slots), "slots"))) return st;
    if ((st = p.d_ticket.ensure(256, "ticket"))) return st;
    HIPCHK(hipHostMalloc((void**)&p.h_states, sizeof(State) * std::max(1, p.count), hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void**)&p.h_descs, sizeof(Desc) * std::max(1, p.count), hipHostMallocDefault));
    HIPCHK(hipEventCreateWithFlags(&p.ev_upload, hipEventDisableTiming));
    if (!p.items.empty())
        HIPCHK(hipMemcpyAsync(p.d_items.p, p.items.data(), sizeof(Item) * p.items.size(), hipMemcpyHostToDevice,
                              s));
    if (!p.outmap.empty()) {
        if ((st = p.d_outmap.ensure(sizeof(int32_t) * p.outmap.size(), "batch output map"))) return st;
        HIPCHK(hipMemcpyAsync(p.d_outmap.p, p.outmap.data(), sizeof(int32_t) * p.outmap.size(),
                              hipMemcpyHostToDevice, s));
    }
    int64_t per_stage[NUM_STAGES] = {0};
    for (const Item& it : p.items) ++per_stage[it.stage];
    double stage_pairs = 0.0;
    for (const Desc& d : p.descs) stage_pairs += 0.5 * (double)d.n * (double)(d.n - 1);
    p.wide = use_wide(c, stage_pairs);
    p.grid = grid_for(c, *std::max_element(per_stage, per_stage + NUM_STAGES), p.wide);
    return KDE_OK;
}

LaunchArgs args_for(const kde_ctx* c, Plan& p) {
    LaunchArgs a{};
    a.items = (const Item*)p.d_items.p;
    a.n_items = (uint32_t)p.items.size();
    a.descs = (const Desc*)p.d_descs.p;
    a.states = (State*)p.d_states.p;
    a.slots = (Slot*)p.d_slots.p;
    a.pubs = (Pub*)p.d_pubs.p;
    a.ticket = (uint32_t*)p.d_ticket.p;
    a.pc = c->pc;
    int64_t wmax = 0;
    for (const Desc& d : p.descs) wmax = std::max<int64_t>(wmax, d.W);
    a.timeout_ticks = wait_ticks(c, (int64_t)kBlock * c->R * (wmax + 4));
    return a;
}

// Record the persistent kernel and the read-back of the per-sample states
// into pinned host memory as one graph on first use; replay after.  With
// the copy in the graph it follows the kernel without a separate
// submission (-8% wall time per call at n = 1024, -0.7% at 65536).  The init
// kernel that resets the states runs after the replay, for the next call
// (once before the first): the caller waits for the event recorded between
// the two only, and the next call's kernel starts without a kernel boundary
// in front of it.
//
// Everything a call changes on the device is ordered on the caller's stream
// after the previous replay of the plan (and the reset behind it): the
// descriptors go up from pinned staging by a stream-ordered copy, so a call
// may return before its launch has run (asynchronous batch calls) and the
// next call still cannot overwrite what a replay in flight reads.  out, when
// given, is device-accessible memory that receives the batch results on the
// stream (k_results) before the reset.
int run_plan(kde_ctx* c, Plan& p, hipStream_t s, kde_result* out = nullptr, bool timed = true) {
    if (!p.exec) {
        // the graph is built node by node, not captured from a stream: a
        // capture would collide with legacy-stream calls that other threads'
        // contexts make meanwhile
        hipGraph_t graph = nullptr;
        HIPCHK(hipGraphCreate(&graph, 0));
        LaunchArgs a = args_for(c, p);
        void* kargs[] = {&a};
        hipKernelNodeParams kn{};
        kn.func = const_cast<void*>(persistent_kernel(c->precision, c->R, p.wide));
        kn.gridDim = dim3((unsigned)p.grid);
        kn.blockDim = dim3(kBlock);
        kn.sharedMemBytes = 0;
        kn.kernelParams = kargs;
        kn.extra = nullptr;
        hipGraphNode_t knode = nullptr, mnode = nullptr;
        hipError_t e = kn.func ? hipGraphAddKernelNode(&knode, graph, nullptr, 0, &kn) : hipErrorInvalidValue;
        if (e == hipSuccess)
            e = hipGraphAddMemcpyNode1D(&mnode, graph, &knode, 1, p.h_states, p.d_states.p, sizeof(State) * p.count,
                                        hipMemcpyDeviceToHost);
        if (e == hipSuccess) e = hipGraphInstantiate(&p.exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            p.exec = nullptr;
            return hip_fail(e, "graph of the persistent kernel");
        }
    }
    if (!p.ev_reset) HIPCHK(hipEventCreateWithFlags(&p.ev_reset, hipEventDisableTiming));
    if (!p.primed) {
        HIPCHK(launch_init((State*)p.d_states.p, (Pub*)p.d_pubs.p, p.count, (uint32_t*)p.d_ticket.p, s));
        p.primed = true;
    } else if (s != p.reset_stream) {
        // the reset after the previous replay ran on another stream
        HIPCHK(hipStreamWaitEvent(s, p.ev_reset, 0));
    }
    if (p.descs_dirty) {
        // the staging buffer is rewritten only once its previous upload has
        // been done (long ago, as a rule)
        HIPCHK(hipEventSynchronize(p.ev_upload));
        std::memcpy(p.h_descs, p.descs.data(), sizeof(Desc) * p.count);
        HIPCHK(hipMemcpyAsync(p.d_descs.p, p.h_descs, sizeof(Desc) * p.count, hipMemcpyHostToDevice, s));
        HIPCHK(hipEventRecord(p.ev_upload, s));
        p.descs_dirty = false;
    }
    if (timed) HIPCHK(hipEventRecord(c->ev0, s));
    HIPCHK(hipGraphLaunch(p.exec, s));
    c->last_grid = p.grid;
    c->last_waves = p.wide ? 4 : 3;
    if (timed) HIPCHK(hipEventRecord(c->ev1, s));
    if (out)
        HIPCHK(launch_results((const State*)p.d_states.p, (const int32_t*)p.d_outmap.p,
                              (int64_t)p.outmap.size() / 2, out, s));
    HIPCHK(launch_init((State*)p.d_states.p, (Pub*)p.d_pubs.p, p.count, (uint32_t*)p.d_ticket.p, s));
    HIPCHK(hipEventRecord(p.ev_reset, s));
    p.reset_stream = s;
    return KDE_OK;
}

Plan* find_plan(kde_ctx* c, const std::string& key) {
    for (auto it = c->plans.begin(); it != c->plans.end(); ++it) {
        if ((*it)->key == key) {
            if (it != c->plans.begin()) c->plans.splice(c->plans.begin(), c->plans, it);
            return c->plans.front().get();
        }
    }
    return nullptr;
}

int get_plan(kde_ctx* c, const std::string& key, const std::vector<SampleSpec>& ss, hipStream_t s, Plan** out,
             const std::vector<int32_t>* outmap = nullptr) {
    Plan* p = find_plan(c, key);
    if (!p) {
        auto np = std::make_unique<Plan>();
        np->key = key;
        build_items(c, *np, ss);
        if (outmap) np->outmap = *outmap;
        int st = upload_plan(c, *np, s);
        if (st) return st;
        c->plans.push_front(std::move(np));
        while (c->plans.size() > c->max_plans) c->plans.pop_back();
        p = c->plans.front().get();
    }
    // descriptors are uploaded again (in run_plan, ordered on the call's
    // stream) if the sample pointers (or psi parameters) changed
    for (size_t k = 0; k < ss.size(); ++k) {
        if (p->descs[k].x != ss[k].x || p->descs[k].psi_g != ss[k].psi_g) {
            p->descs[k].x = ss[k].x;
            p->descs[k].psi_g = ss[k].psi_g;
            p->descs_dirty = true;
        }
    }
    *out = p;
    return KDE_OK;
}

void fill_result(const State& s, kde_result* r) {
    r->h = s.h;
    r->mean = s.mean;
    r->sigma = s.sigma;
    r->psi8 = s.psi8;
    r->g1 = s.g1;
    r->psi6 = s.psi6;
    r->g2 = s.g2;
    r->psi4 = s.psi4;
    r->status = s.status;
    r->reserved = 0;
}

int check_x(const void* x, int64_t n, int64_t nmin, int mem_kind, int dtype) {
    if (!x) return set_err(KDE_EINVAL, "null sample pointer");
    if (n < nmin)
        return set_err(KDE_EINVAL, nmin == 2 ? "n must be at least 2 (Step I divides by n - 1)"
                                            : "n must be at least 1");
    if (n > ((int64_t)1 << 31) - 1) return set_err(KDE_EINVAL, "n must be below 2^31");
    if (mem_kind != KDE_MEM_HOST && mem_kind != KDE_MEM_DEVICE) return set_err(KDE_EINVAL, "bad mem_kind");
    if (dtype != KDE_F64 && dtype != KDE_F32) return set_err(KDE_EINVAL, "bad dtype");
    return KDE_OK;
}

// Stage host samples into the context's device buffer (or pass device data).
int stage_x(kde_ctx* c, const void* x, int64_t n, int mem_kind, int dtype, hipStream_t s,
            const void** dev) {
    if (mem_kind == KDE_MEM_DEVICE) {
        *dev = x;
        return KDE_OK;
    }
    const size_t bytes = (size_t)n * (dtype == KDE_F64 ? 8 : 4);
    int st = c->x_stage.ensure(bytes, "sample staging buffer");
    if (st) return st;
    HIPCHK(hipMemcpyAsync(c->x_stage.p, x, bytes, hipMemcpyHostToDevice, s));
    *dev = c->x_stage.p;
    return KDE_OK;
}

// Device-accessible address of out for the results kernel, or nullptr when out
// is ordinary (pageable) host memory, which only the host can fill.
kde_result* device_view(const kde_ctx* c, kde_result* out) {
    hipPointerAttribute_t a{};
    if (hipPointerGetAttributes(&a, out) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    if (a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged)
        return a.device == c->device ? out : nullptr;
    if (a.type == hipMemoryTypeHost) return (kde_result*)(a.devicePointer ? a.devicePointer : (void*)out);
    return nullptr;
}

// True when p points into memory on the context's GPU.
bool on_device(const kde_ctx* c, const void* p) {
    hipPointerAttribute_t a{};
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return (a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged) && a.device == c->device;
}

int finish(kde_ctx* c, Plan& p, hipStream_t s) {
    (void)s;
    HIPCHK(hipEventSynchronize(c->ev1));
    c->last_states.assign(p.h_states, p.h_states + p.count);
    float ms = -1.0f;
    if (hipEventElapsedTime(&ms, c->ev0, c->ev1) == hipSuccess) c->last_device_ms = ms;
    return KDE_OK;
}

std::string key_single(const char* tag, int64_t n, int dtype, int extra1 = 0, int64_t e2 = 0,
                       int64_t e3 = 0) {
    char buf[160];
    std::snprintf(buf, sizeof buf, "%s:n=%lld:t=%d:%d:%lld:%lld", tag, (long long)n, dtype, extra1,
                  (long long)e2, (long long)e3);
    return buf;
}

std::mutex g_default_mu;
kde_ctx* g_default = nullptr;

kde_ctx* default_ctx() {
    if (!g_default) {
        kde_ctx* c = nullptr;
        if (kde_ctx_create(&c, nullptr) == KDE_OK) g_default = c;
    }
    return g_default;
}

int psi_common(kde_ctx* c, const void* x, int64_t n, int mem_kind, int dtype, int r, double g,
               int64_t b, int64_t e, hipStream_t s, State* out) {
    int st = check_x(x, n, 1, mem_kind, dtype);
    if (st) return st;
    if (r != 4 && r != 6) return set_err(KDE_EINVAL, "r must be 4 or 6");
    if (!(g > 0.0) || !std::isfinite(g)) return set_err(KDE_EINVAL, "g must be finite and positive");
    DeviceGuard dg(c->device);
    const void* dx = nullptr;
    if ((st = stage_x(c, x, n, mem_kind, dtype, s, &dx))) return st;
    SampleSpec sp{dx, n, dtype, MODE_PSI, r, g, b, e};
    Plan* p = nullptr;
    if ((st = get_plan(c, key_single("psi", n, dtype, r, b, e), {sp}, s, &p))) return st;
    if ((st = run_plan(c, *p, s))) return st;
    if ((st = finish(c, *p, s))) return st;
    *out = p->h_states[0];
    return KDE_OK;
}

}  // namespace rt
}  // namespace kde

using namespace kde::rt;

// ================================================================ C ABI
extern "C" {

const char* kde_version(void) { return "libkdeplugin 0.1 (gfx950)"; }

int kde_last_error(void) { return last_error_code(); }

const char* kde_last_error_message(void) { return last_error_text(); }

const char* kde_strerror(int code) {
    switch (code) {
    case KDE_OK: return "ok";
    case KDE_EINVAL: return "invalid argument";
    case KDE_ENONFINITE: return "non-finite sample value";
    case KDE_EDEGENERATE: return "degenerate sample (zero spread or failed sign invariant)";
    case KDE_ENOMEM: return "out of memory or over budget";
    case KDE_EDEVICE: return "HIP runtime error";
    case KDE_ETIMEOUT: return "in-kernel stage wait timed out";
    case KDE_EBUSY: return "busy";
    default: return "unknown status";
    }
}

void kde_options_init(kde_options* opt) {
    if (!opt) return;
    std::memset(opt, 0, sizeof(*opt));
    opt->device = 0;
    opt->precision = KDE_FP64_PLAIN;
}

int kde_ctx_create(kde_ctx** out, const kde_options* opt) {
    if (!out) return set_err(KDE_EINVAL, "null output pointer");
    *out = nullptr;
    kde_options o;
    kde_options_init(&o);
    if (opt) o = *opt;
    if (o.precision != KDE_FP64_PLAIN && o.precision != KDE_FP32_COMP &&
        o.precision != KDE_FP32_COMP_EXACT && o.precision != KDE_FP32_POLYEXP && o.precision != KDE_Q32_32)
        return set_err(KDE_EINVAL, "bad precision");
    if (o.rows_per_lane != 0 && o.rows_per_lane != 1 && o.rows_per_lane != 2 && o.rows_per_lane != 4)
        return set_err(KDE_EINVAL, "rows_per_lane must be 0, 1, 2 or 4");
    if (o.blocks_per_cu < 0 || o.blocks_per_cu > 16) return set_err(KDE_EINVAL, "blocks_per_cu out of range");
    if (o.mem_budget < 0 || o.target_items < 0 || o.pair_budget < 0 || o.wait_limit_us < 0)
        return set_err(KDE_EINVAL, "negative option");
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev == 0) return set_err(KDE_EDEVICE, "no HIP device available");
    if (o.device < 0 || o.device >= ndev) return set_err(KDE_EINVAL, "device ordinal out of range");
    TuneTable tt;
    if (o.tune_table) {
        const int st = load_tune_table(o.tune_table, &tt);
        if (st) return st;
        if (tt.precision >= 0 && tt.precision != o.precision)
            return set_err(KDE_EINVAL, "tune table was made for another precision");
    }
    auto c = std::make_unique<kde_ctx>();
    for (int b = 0; b < 64; ++b) c->bucket_target[b] = tt.bucket[b];
    c->pair_budget = o.pair_budget > 0 ? o.pair_budget : tt.pair_budget;
    c->device = o.device;
    // an FP32 tune table may select the polynomial exponential's kernels
    c->precision = (o.precision == KDE_FP32_COMP && tt.exp_poly == 1) ? KDE_FP32_POLYEXP : o.precision;
    c->mem_budget = o.mem_budget;
    c->R = o.rows_per_lane ? o.rows_per_lane : (tt.R ? tt.R : 1);
    c->target_items = o.target_items;
    c->wait_limit_ticks = (uint64_t)o.wait_limit_us * 100u;  // 100 MHz wall clock
    c->pc = make_consts();
    DeviceGuard dg(c->device);
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, c->device));
    c->cus = prop.multiProcessorCount;
    HIPCHK(hipEventCreate(&c->ev0));
    HIPCHK(hipEventCreate(&c->ev1));
    int occ = 0;
    HIPCHK(persistent_occupancy(c->precision, c->R, false, &occ));
    if (o.blocks_per_cu == 0 && tt.bpc == 0 && wide_available(c->precision, c->R)) {
        int occ4 = 0;
        HIPCHK(persistent_occupancy(c->precision, c->R, true, &occ4));
        if (occ4 > occ) c->blocks_per_cu_wide = occ4;
    }
    {
        // device address of the static scratch of kde_plugin_bandwidth_noalloc
        const int st = noalloc_init(c->device);
        if (st) return st;
    }
    c->blocks_per_cu = o.blocks_per_cu ? o.blocks_per_cu : (tt.bpc ? std::min(tt.bpc, std::max(1, occ)) : std::max(1, occ));
    *out = c.release();
    return ok();
}

void kde_ctx_destroy(kde_ctx* ctx) {
    if (!ctx) return;
    DeviceGuard dg(ctx->device);
    // each plan waits for its last replay (and the reset after it) when it is
    // destroyed; the other calls return only when their work is done
    if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
    if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
    delete ctx;
}

int kde_ctx_config(const kde_ctx* c, int32_t* rows_per_lane, int32_t* block_threads,
                   int32_t* tile_rows, int32_t* blocks_per_cu) {
    if (!c) return set_err(KDE_EINVAL, "null context");
    if (rows_per_lane) *rows_per_lane = c->R;
    if (block_threads) *block_threads = kBlock;
    if (tile_rows) *tile_rows = kBlock * c->R;
    if (blocks_per_cu) *blocks_per_cu = c->blocks_per_cu;
    return ok();
}

int64_t kde_psi_num_items(const kde_ctx* c, int64_t n) {
    if (!c || n < 1) {
        set_err(KDE_EINVAL, "null context or n < 1");
        return -1;
    }
    ok();
    return pair_item_count(pair_geom(c, n));
}

int kde_psi_item_geometry(const kde_ctx* c, int64_t n, int64_t item, int64_t* r0, int64_t* r1,
                          int64_t* c0, int64_t* c1) {
    if (!c || n < 1 || item < 0) return set_err(KDE_EINVAL, "bad arguments");
    const PairGeom g = pair_geom(c, n);
    int64_t rb, cb;
    if (!pair_item_at(g, item, &rb, &cb)) return set_err(KDE_EINVAL, "item index out of range");
    const int64_t a = rb * g.TI;
    const int64_t w = pair_chunk_width(g, rb);
    const int64_t cs = a + cb * w;
    if (r0) *r0 = a;
    if (r1) *r1 = std::min(a + g.TI, n);
    if (c0) *c0 = cs;
    if (c1) *c1 = std::min(cs + w, n);
    return ok();
}

int kde_psi_ex(kde_ctx* ctx, const void* x, int64_t n, int r, double g, int mem_kind, int dtype,
               kde_stream stream, double* out) {
    if (!ctx || !out) return set_err(KDE_EINVAL, "null context or output");
    State s{};
    int st = psi_common(ctx, x, n, mem_kind, dtype, r, g, 0, -1, (hipStream_t)stream, &s);
    if (st) return st;
    if (s.status) return set_err(s.status, "Psi evaluation failed on the device");
    *out = r == 6 ? s.psi6 : s.psi4;
    return ok();
}

int kde_psi_range(kde_ctx* ctx, const void* x, int64_t n, int r, double g, int mem_kind, int dtype,
                  int64_t item_begin, int64_t item_end, kde_stream stream, double* partial) {
    if (!ctx || !partial) return set_err(KDE_EINVAL, "null context or output");
    const int64_t np = n >= 1 ? pair_item_count(pair_geom(ctx, n)) : 0;
    if (item_begin < 0 || item_end < item_begin || item_end > np)
        return set_err(KDE_EINVAL, "item range outside [0, kde_psi_num_items)");
    if (item_begin == item_end) {
        *partial = 0.0;
        return ok();
    }
    State s{};
    int st = psi_common(ctx, x, n, mem_kind, dtype, r, g, item_begin, item_end, (hipStream_t)stream, &s);
    if (st) return st;
    if (s.status) return set_err(s.status, "Psi range evaluation failed on the device");
    *partial = r == 6 ? s.S6 : s.S4;
    return ok();
}

int kde_plugin_bandwidth_ex(kde_ctx* c, const void* x, int64_t n, int mem_kind, int dtype,
                            kde_stream stream, kde_result* out) {
    if (!c || !out) return set_err(KDE_EINVAL, "null context or output");
    std::memset(out, 0, sizeof(*out));
    out->h = NAN;
    int st = check_x(x, n, 2, mem_kind, dtype);
    if (st) {
        out->status = st;
        return st;
    }
    hipStream_t s = (hipStream_t)stream;
    DeviceGuard dg(c->device);
    const void* dx = nullptr;
    if ((st = stage_x(c, x, n, mem_kind, dtype, s, &dx))) return out->status = st;
    SampleSpec sp{dx, n, dtype, MODE_PLUGIN, 0, 0.0, 0, -1};
    Plan* p = nullptr;
    if ((st = get_plan(c, key_single("plugin", n, dtype), {sp}, s, &p))) return out->status = st;
    if ((st = run_plan(c, *p, s))) return out->status = st;
    if ((st = finish(c, *p, s))) return out->status = st;
    fill_result(p->h_states[0], out);
    if (out->status) {
        out->h = NAN;
        return set_err(out->status, "bandwidth selection failed on the device");
    }
    return ok();
}

int kde_plugin_bandwidth_batch(kde_ctx* c, const void* const* xs, const int64_t* ns, int64_t count,
                               int mem_kind, kde_result* out, kde_stream stream) {
    if (!c || !xs || !ns || !out || count < 1) return set_err(KDE_EINVAL, "bad batch arguments");
    if (count > (1 << 24)) return set_err(KDE_EINVAL, "batch too large");
    if (mem_kind != KDE_MEM_HOST && mem_kind != KDE_MEM_DEVICE) return set_err(KDE_EINVAL, "bad mem_kind");
    hipStream_t s = (hipStream_t)stream;
    DeviceGuard dg(c->device);
    // asynchronous when the samples are on the device and out is
    // device-accessible: the results are then written by the device, on s
    kde_result* dout = mem_kind == KDE_MEM_DEVICE ? device_view(c, out) : nullptr;
    std::vector<int32_t> status((size_t)count, KDE_OK);
    std::vector<int64_t> valid;
    std::string key = dout ? "batch-async" : "batch";
    key.reserve(16 * (size_t)count);
    size_t host_bytes = 0;
    for (int64_t k = 0; k < count; ++k) {
        const int st = check_x(xs[k], ns[k], 2, mem_kind, KDE_F64);
        status[(size_t)k] = st;
        if (st == KDE_OK) {
            valid.push_back(k);
            host_bytes += (size_t)ns[k] * 8;
        }
        if (!dout) {
            std::memset(&out[k], 0, sizeof(kde_result));
            out[k].h = NAN;
            out[k].status = st;
        }
    }
    if (valid.empty()) return set_err(KDE_EINVAL, "no valid sample in the batch");
    // host samples are packed into one device arena
    size_t off = 0;
    if (mem_kind == KDE_MEM_HOST) {
        int st = c->x_stage.ensure(host_bytes, "batch staging arena");
        if (st) return st;
    }
    std::vector<SampleSpec> vs;
    vs.reserve(valid.size());
    for (int64_t k : valid) {
        const void* dx = xs[k];
        if (mem_kind == KDE_MEM_HOST) {
            dx = (char*)c->x_stage.p + off;
            HIPCHK(hipMemcpyAsync((void*)dx, xs[k], (size_t)ns[k] * 8, hipMemcpyHostToDevice, s));
            off += (size_t)ns[k] * 8;
        }
        vs.push_back(SampleSpec{dx, ns[k], KDE_F64, MODE_PLUGIN, 0, 0.0, 0, -1});
        key += ":" + std::to_string(ns[k]);
    }
    std::vector<int32_t> outmap;
    if (dout) {
        // the output map is part of the plan: the positions and statuses of
        // rejected samples go into the key
        outmap.assign(2 * (size_t)count, 0);
        int32_t q = 0;
        for (int64_t k = 0; k < count; ++k) {
            if (status[(size_t)k] == KDE_OK) {
                outmap[2 * k] = q++;
            } else {
                outmap[2 * k] = -1;
                outmap[2 * k + 1] = status[(size_t)k];
                key += "|x" + std::to_string(k) + "=" + std::to_string(status[(size_t)k]);
            }
        }
    }
    Plan* p = nullptr;
    int st;
    if ((st = get_plan(c, key, vs, s, &p, dout ? &outmap : nullptr))) return st;
    if (dout) {
        if ((st = run_plan(c, *p, s, dout, false))) return st;
        return ok();
    }
    if ((st = run_plan(c, *p, s))) return st;
    if ((st = finish(c, *p, s))) return st;
    for (size_t q = 0; q < valid.size(); ++q) {
        fill_result(p->h_states[q], &out[valid[q]]);
        if (out[valid[q]].status) out[valid[q]].h = NAN;
    }
    return ok();
}

double kde_ctx_last_device_ms(const kde_ctx* c) {
    if (!c) {
        set_err(KDE_EINVAL, "null context");
        return -1.0;
    }
    return c->last_device_ms;
}

int kde_ctx_last_launch(const kde_ctx* c, int32_t* blocks, int32_t* waves_per_simd) {
    if (!c) return set_err(KDE_EINVAL, "null context");
    if (c->last_grid == 0) return set_err(KDE_EINVAL, "nothing launched on this context yet");
    if (blocks) *blocks = c->last_grid;
    if (waves_per_simd) *waves_per_simd = c->last_waves;
    return ok();
}

static_assert(NUM_STAGES == KDE_NUM_STAGES, "the timeline has one entry per stage");

int kde_ctx_last_timeline(const kde_ctx* c, int64_t sample, double* ms) {
    if (!c || !ms) return set_err(KDE_EINVAL, "null context or output");
    if (sample < 0 || sample >= (int64_t)c->last_states.size())
        return set_err(KDE_EINVAL, "sample index outside the last call");
    const State& s = c->last_states[(size_t)sample];
    for (int k = 0; k < NUM_STAGES; ++k)
        ms[k] = s.t_fin[k] >= s.t_first && s.t_fin[k] ? (double)(s.t_fin[k] - s.t_first) * 1e-5 : -1.0;
    return ok();
}

double kde_psi(const double* x, int64_t n, int r, double g) {
    std::lock_guard<std::mutex> lk(g_default_mu);
    kde_ctx* c = default_ctx();
    if (!c) return NAN;
    double v = NAN;
    if (kde_psi_ex(c, x, n, r, g, KDE_MEM_HOST, KDE_F64, nullptr, &v) != KDE_OK) return NAN;
    return v;
}

double kde_plugin_bandwidth(const double* x, int64_t n) {
    std::lock_guard<std::mutex> lk(g_default_mu);
    kde_ctx* c = default_ctx();
    if (!c) return NAN;
    kde_result r;
    if (kde_plugin_bandwidth_ex(c, x, n, KDE_MEM_HOST, KDE_F64, nullptr, &r) != KDE_OK) return NAN;
    return r.h;
}

// Density evaluation (equation (1)): see kde_eval.hip for the kernels.
int kde_eval_ex(kde_ctx* c, const void* x, int64_t n, int mem_kind, int dtype, const double* y, int64_t m,
                int y_mem_kind, double h, kde_stream stream, double* out) {
    if (!c) return set_err(KDE_EINVAL, "null context");
    int st = check_x(x, n, 1, mem_kind, dtype);
    if (st) return st;
    if (m < 0) return set_err(KDE_EINVAL, "m must not be negative");
    if (m > ((int64_t)1 << 31) - 1) return set_err(KDE_EINVAL, "m must be below 2^31");
    if (y_mem_kind != KDE_MEM_HOST && y_mem_kind != KDE_MEM_DEVICE) return set_err(KDE_EINVAL, "bad y_mem_kind");
    if (!(std::isfinite(h) && h > 0.0)) return set_err(KDE_EINVAL, "h must be finite and positive");
    if (m == 0) return ok();
    if (!y || !out) return set_err(KDE_EINVAL, "null evaluation point or output pointer");
    hipStream_t s = (hipStream_t)stream;
    DeviceGuard dg(c->device);

    // tiles of points times chunks of W samples.  FP64 plain: tiles of 256
    // points, at least ~4096 items, at most 2^24 pairs per item, chunks of at
    // least 1024 samples.  FP32: tiles of 4096 points, items of at most 2^26
    // pairs, as many as fill whole rounds of the blocks the GPU holds at once
    // (the items of a round take equal time), chunks of at least 512 samples
    eval::EvalArgs a{};
    a.n = n;
    a.m = m;
    a.dtype = dtype == KDE_F64 ? 0 : 1;
    a.prec = c->precision == KDE_FP64_PLAIN ? 0 : 1;
    a.h = h;
    a.s = std::sqrt(0.5 * 1.4426950408889634) / h;
    a.norm = 1.0 / ((double)n * h * std::sqrt(2.0 * 3.14159265358979323846));
    const bool f32 = a.prec != 0;
    const int64_t tp = f32 ? eval::kTilePoints32 : eval::kTilePoints64;
    const int64_t wmin = f32 ? 512 : 1024;
    const int lg_pairs = f32 ? 26 : 24;
    const int64_t n_rt = (m + tp - 1) / tp;
    int64_t n_cc = (tp * n + ((int64_t)1 << lg_pairs) - 1) >> lg_pairs;
    if (!f32) {
        n_cc = std::max<int64_t>(n_cc, (4096 + n_rt - 1) / n_rt);
    } else {
        if (c->eval32_resident == 0) {
            int bpc = 0;
            HIPCHK(eval::blocks_per_cu(1, &bpc));
            c->eval32_resident = (int64_t)std::max(1, bpc) * c->cus;
        }
        const int64_t res = c->eval32_resident;
        const int64_t rounds = (n_rt * n_cc + res - 1) / res;
        n_cc = std::max<int64_t>(n_cc, (rounds * res + n_rt - 1) / n_rt);
    }
    n_cc = std::max<int64_t>(1, std::min<int64_t>(n_cc, (n + wmin - 1) / wmin));
    a.W = ((((n + n_cc - 1) / n_cc) + 15) / 16) * 16;
    n_cc = (n + a.W - 1) / a.W;
    if (n_rt * n_cc > ((int64_t)1 << 31) - 1) return set_err(KDE_EINVAL, "too many evaluation items");
    a.n_rt = (int32_t)n_rt;
    a.n_cc = (int32_t)n_cc;

    // device buffers (budget-checked like the work lists)
    const size_t ybytes = (size_t)m * 8, pbytes = n_cc > 1 ? (size_t)n_cc * (size_t)m * 8 : 0;
    const size_t xbytes = mem_kind == KDE_MEM_HOST ? (size_t)n * (dtype == KDE_F64 ? 8 : 4) : 0;
    if (c->mem_budget > 0) {
        size_t have = 0;
        const size_t grow = std::max(xbytes, c->x_stage.bytes) - c->x_stage.bytes +
                            (y_mem_kind == KDE_MEM_HOST ? 2 * ybytes : 0) + pbytes + 256;
        total_plan_bytes(c, grow, &have);
        if (have > (size_t)c->mem_budget)
            return set_err(KDE_ENOMEM, "density evaluation buffers exceed the context's memory budget");
    }
    const void* dx = nullptr;
    if ((st = stage_x(c, x, n, mem_kind, dtype, s, &dx))) return st;
    a.x = dx;
    if (y_mem_kind == KDE_MEM_HOST) {
        if ((st = c->ev_y.ensure(ybytes, "evaluation points"))) return st;
        if ((st = c->ev_out.ensure(ybytes, "evaluation output"))) return st;
        HIPCHK(hipMemcpyAsync(c->ev_y.p, y, ybytes, hipMemcpyHostToDevice, s));
        a.y = (const double*)c->ev_y.p;
        a.out = (double*)c->ev_out.p;
    } else {
        a.y = y;
        a.out = out;
    }
    if (pbytes && (st = c->ev_part.ensure(pbytes, "evaluation partial sums"))) return st;
    a.part = (double*)c->ev_part.p;
    if ((st = c->ev_flag.ensure(256, "evaluation flag"))) return st;
    a.flag = (int32_t*)c->ev_flag.p;
    HIPCHK(hipMemsetAsync(a.flag, 0, sizeof(int32_t), s));
    HIPCHK(hipEventRecord(c->ev0, s));
    HIPCHK(eval::launch(a, s));
    HIPCHK(hipEventRecord(c->ev1, s));
    int32_t flag = 0;
    HIPCHK(hipMemcpyAsync(&flag, a.flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    if (y_mem_kind == KDE_MEM_HOST) HIPCHK(hipMemcpyAsync(out, a.out, ybytes, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    float ms = -1.0f;
    if (hipEventElapsedTime(&ms, c->ev0, c->ev1) == hipSuccess) c->last_device_ms = ms;
    if (flag) return set_err(KDE_ENONFINITE, "NaN or Inf among the samples or evaluation points");
    return ok();
}

int kde_eval(const double* x, int64_t n, const double* y, int64_t m, double h, double* out) {
    std::lock_guard<std::mutex> lk(g_default_mu);
    kde_ctx* c = default_ctx();
    if (!c) return last_error_code() ? last_error_code() : KDE_EDEVICE;
    return kde_eval_ex(c, x, n, KDE_MEM_HOST, KDE_F64, y, m, KDE_MEM_HOST, h, nullptr, out);
}

}  // extern "C"
