// Continuous-batching server of libkdeplugin.
//
// Requests (one sample each) are submitted at any time.  The server admits
// them into a fixed number of slots against a device-memory budget, keeps
// admitted samples resident in a device arena, and runs "steps": one launch
// of the persistent kernel over a work list that takes the next work items of
// every active request in round-robin order, up to a pair budget per step
// (processor sharing).  A request's per-stage counters, flags and partial-sum
// slots live on the device across steps, so requests join and leave between
// launches while the others keep going, and a request's items and their
// arithmetic are the ones a single call would use: every result is bitwise
// the same alone or in any mix.
//
// Steps are queued two deep on the server's stream, so the host prepares and
// admits while the device computes.  Host samples are copied into the arena
// on a second stream; the compute stream waits for that copy only in the
// step that first lists the request.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <vector>

#include "kde_runtime.h"

using namespace kde;
using namespace kde::rt;

namespace {

double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// First-fit allocator over [0, size) with coalescing; offsets aligned to 256.
class Arena {
public:
    explicit Arena(size_t size) { free_[0] = size; }
    bool alloc(size_t bytes, size_t* off) {
        bytes = (bytes + 255) & ~(size_t)255;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes, start = it->first + bytes;
                free_.erase(it);
                if (rest) free_[start] = rest;
                used_ += bytes;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = (bytes + 255) & ~(size_t)255;
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t used() const { return used_; }

private:
    std::map<size_t, size_t> free_;
    size_t used_ = 0;
};

struct Request {
    int64_t id = 0;
    const void* x_user = nullptr;
    int64_t n = 0;
    int mem_kind = KDE_MEM_HOST;
    double t_submit = 0, t_admit = -1, t_done = -1;
    int32_t slot = -1;
    size_t off = 0, bytes = 0;        // arena block: [slots | sample copy]
    Desc desc{};
    PairGeom geom{};
    int stage = 0;                    // issue cursor: stage, ordinal within it,
    int64_t next = 0;                 // and (row block, chunk) for pair stages
    int64_t rb = 0, cb = 0;
    double pairs = 0;                 // pair evaluations of the whole selection
    hipEvent_t copied = nullptr;      // sample ready: host copy done, or the producer's work (device samples)
    bool wait_copy = false;           // the compute stream has yet to wait for `copied`
    int64_t last_step = -1;           // sequence number of the step that listed its last items
    int64_t launched_step = -1;       // sequence number of the last launched step listing any of its items
    double listed_pairs = 0;          // pair evaluations of the items listed so far
    int32_t fail = 0;                 // KDE_E* code once a step listing its items failed to run
};

struct Step {
    hipEvent_t done = nullptr;
    int buf = 0;
    int64_t seq = 0;
};

}  // namespace

struct kde_server {
    kde_ctx* ctx = nullptr;
    kde_server_options opt{};
    hipStream_t stream = nullptr, copy_stream = nullptr;
    DevBuf arena_buf, d_descs, d_states, d_pubs, d_items[2], d_ticket;
    std::unique_ptr<Arena> arena;
    Desc* h_descs = nullptr;          // pinned mirrors
    State* h_states[2] = {nullptr, nullptr};  // state read-back of the steps using list buffer 0 / 1
    Item* h_items[2] = {nullptr, nullptr};
    size_t items_cap = 0;
    hipEvent_t items_free[2] = {nullptr, nullptr};  // the pinned list buffer may be rewritten
    int next_buf = 0;
    std::vector<int32_t> free_slots;
    std::vector<std::unique_ptr<Request>> active;   // admission order
    std::deque<std::unique_ptr<Request>> queue;
    std::deque<Step> inflight;
    std::vector<kde_completion> done;
    int64_t next_id = 1;
    size_t rr = 0;                    // round-robin start
    double pairs_done = 0;
    int64_t steps = 0;
    size_t device_sample_bytes = 0;   // admitted samples that live in caller memory
    double pairs_issued = 0;          // pair evaluations of all launched items
    int32_t fail_next = 0;            // injected failure of the next step (kde_server_fail_next_step)
    int32_t failed_steps = 0;
};

namespace {

size_t slots_bytes(const Desc& d) {
    int64_t s = 0;
    for (int k = 0; k < NUM_STAGES; ++k) s += d.n_items[k];
    return (size_t)std::max<int64_t>(1, s) * sizeof(Slot);
}

// Arena bytes of a request: its partial-sum slots, plus its sample when the
// sample is copied in from host memory.
size_t request_bytes(const Request& r) {
    const size_t sample = r.mem_kind == KDE_MEM_HOST ? (size_t)r.n * sizeof(double) : 0;
    return ((slots_bytes(r.desc) + 255) & ~(size_t)255) + sample;
}

// Device bytes a request counts against the budget: the arena block, plus a
// device-resident sample the caller keeps in its own memory.
size_t budget_bytes(const Request& r) {
    return r.bytes + (r.mem_kind == KDE_MEM_DEVICE ? (size_t)r.n * sizeof(double) : 0);
}

int admit_one(kde_server* s, std::unique_ptr<Request>& rp) {
    Request& r = *rp;
    size_t off = 0;
    if (s->arena->used() + s->device_sample_bytes + budget_bytes(r) > (size_t)s->opt.mem_budget)
        return KDE_ENOMEM;
    if (!s->arena->alloc(r.bytes, &off)) return KDE_ENOMEM;
    if (r.mem_kind == KDE_MEM_DEVICE) s->device_sample_bytes += (size_t)r.n * sizeof(double);
    r.off = off;
    r.slot = s->free_slots.back();
    s->free_slots.pop_back();
    char* base = (char*)s->arena_buf.p;
    const int64_t slot0 = (int64_t)(off / sizeof(Slot));
    int64_t acc = slot0;
    for (int k = 0; k < NUM_STAGES; ++k) {
        r.desc.slot_base[k] = acc;
        acc += r.desc.n_items[k];
    }
    if (r.mem_kind == KDE_MEM_HOST) {
        void* dst = base + off + ((slots_bytes(r.desc) + 255) & ~(size_t)255);
        HIPCHK(hipMemcpyAsync(dst, r.x_user, (size_t)r.n * sizeof(double), hipMemcpyHostToDevice, s->copy_stream));
        if (!r.copied) HIPCHK(hipEventCreateWithFlags(&r.copied, hipEventDisableTiming));
        HIPCHK(hipEventRecord(r.copied, s->copy_stream));
        r.wait_copy = true;
        r.desc.x = dst;
    } else {
        r.desc.x = r.x_user;
        r.wait_copy = r.copied != nullptr;  // the producer stream's event recorded at submission
    }
    r.geom = pair_geom(s->ctx, r.n);
    r.stage = 0;
    r.next = r.rb = r.cb = 0;
    s->h_descs[r.slot] = r.desc;
    HIPCHK(hipMemcpyAsync((Desc*)s->d_descs.p + r.slot, s->h_descs + r.slot, sizeof(Desc), hipMemcpyHostToDevice,
                          s->stream));
    HIPCHK(hipMemsetAsync((State*)s->d_states.p + r.slot, 0, sizeof(State), s->stream));
    HIPCHK(hipMemsetAsync((Pub*)s->d_pubs.p + (size_t)r.slot * kPubReplicas, 0, sizeof(Pub) * kPubReplicas,
                          s->stream));
    r.t_admit = now_ms();
    return KDE_OK;
}

// Admission key of smallest-first: log2 of the request's pair count, minus
// one for every aging_ms it has waited, so a large request overtakes newer
// small ones after waiting (aging_ms = 0: no aging, pure smallest-first).
double sjf_key(const kde_server* s, const Request& r, double now) {
    double k = std::log2(std::max(1.0, r.pairs));
    if (s->opt.aging_ms > 0) k -= (now - r.t_submit) / (double)s->opt.aging_ms;
    return k;
}

// The same key on the pair evaluations a request still has to list (the
// priority fill order of a step).
double remaining_key(const kde_server* s, const Request& r, double now) {
    double k = std::log2(std::max(1.0, r.pairs - r.listed_pairs));
    if (s->opt.aging_ms > 0) k -= (now - r.t_submit) / (double)s->opt.aging_ms;
    return k;
}

int admit(kde_server* s) {
    const double now = now_ms();
    while (!s->queue.empty() && !s->free_slots.empty()) {
        auto pick = s->queue.begin();
        if (s->opt.policy == KDE_SERVE_SJF)
            pick = std::min_element(s->queue.begin(), s->queue.end(),
                                    [&](const std::unique_ptr<Request>& a, const std::unique_ptr<Request>& b) {
                                        return sjf_key(s, *a, now) < sjf_key(s, *b, now);
                                    });
        const int st = admit_one(s, *pick);
        if (st == KDE_ENOMEM) break;  // wait for memory to free up
        if (st) return st;
        s->active.push_back(std::move(*pick));
        s->queue.erase(pick);
    }
    return KDE_OK;
}

// Pair evaluations of a pair item: rows [r0, r1) x columns [c0, c1) with
// column > row (diagonal items are partly empty).
double item_pairs(const Request& r, const Item& it) {
    if (it.stage == ST_SUM || it.stage == ST_SSQ) return 0.0;
    const PairGeom& g = r.geom;
    const int64_t r0 = (int64_t)it.a * g.TI, r1 = std::min(r0 + g.TI, r.n);
    const int64_t w = pair_chunk_width(g, it.a);
    const int64_t c0 = r0 + (int64_t)it.b * w, c1 = std::min(c0 + w, r.n);
    if (c0 >= r1) return (double)(r1 - r0) * (double)(c1 - c0);
    double p = 0.0;
    for (int64_t i = r0; i < r1; ++i) p += (double)std::max<int64_t>(0, c1 - std::max(c0, i + 1));
    return p;
}

// The next unlisted item of a request (its cursor must not be past the end).
Item next_item(Request& r) {
    const Desc& d = r.desc;
    const int s = r.stage;
    int32_t wait = -1;
    if (s == ST_SSQ) wait = ST_SUM;
    if (s == ST_PSI6) wait = ST_SSQ;
    if (s == ST_PSI4) wait = ST_PSI6;
    Item it{r.slot, s, wait, 0, 0, 0, d.slot_base[s] + r.next};
    if (s == ST_SUM || s == ST_SSQ) {
        it.a = (int32_t)r.next;
    } else {
        it.a = (int32_t)r.rb;
        it.b = (int32_t)r.cb;
        if (++r.cb >= pair_items_in_row(r.geom, r.rb)) {
            ++r.rb;
            r.cb = 0;
        }
    }
    ++r.next;
    return it;
}

// A step's items come from many requests, one pair item per request per
// turn: one block per item up to the context's full grid.
int step_grid(const kde_ctx* c, int64_t items, bool wide) {
    const int bpc = wide ? c->blocks_per_cu_wide : c->blocks_per_cu;
    return (int)std::min<int64_t>((int64_t)c->cus * std::max(1, bpc), std::max<int64_t>(1, items));
}

int launch_step(kde_server* s) {
    if (s->active.empty()) return KDE_OK;
    std::vector<Item> stage_lists[NUM_STAGES];
    double budget = (double)s->opt.step_pairs;
    const size_t m = s->active.size();
    std::vector<bool> exhausted(m, false);
    size_t left = m;
    std::vector<bool> listed(m, false);
    for (size_t k = 0; k < m; ++k)
        if (s->active[k]->stage >= NUM_STAGES || s->active[k]->fail) {
            exhausted[k] = true;
            --left;
        }
    double step_pairs = 0.0;
    // A request's cursor always points at its next unlisted item; when the last
    // one is listed, last_step records the step being built.  Moment items
    // ride free (they count no pairs).
    auto advance = [](Request& r) {
        while (r.stage < NUM_STAGES && r.next >= r.desc.n_items[r.stage]) {
            ++r.stage;
            r.next = 0;
            r.rb = r.cb = 0;
        }
    };
    // List the next items of active request k up to `max_pair_items` pair
    // items (or until the budget runs out); true once it has none left.
    auto take = [&](size_t k, int64_t max_pair_items) {
        Request& r = *s->active[k];
        int64_t got = 0;
        for (;;) {
            advance(r);
            if (r.stage >= NUM_STAGES || got >= max_pair_items || budget <= 0) break;
            const Item it = next_item(r);
            stage_lists[it.stage].push_back(it);
            listed[k] = true;
            const double p = item_pairs(r, it);
            budget -= p;
            step_pairs += p;
            r.listed_pairs += p;
            if (p > 0) ++got;
        }
        if (r.stage >= NUM_STAGES) {
            exhausted[k] = true;
            --left;
            r.last_step = s->steps;  // the step being built
            return true;
        }
        return false;
    };
    if (s->opt.fill == KDE_FILL_PRIORITY) {
        // the budget goes to the requests in admission-key order, each taking
        // as much as it can use before the next one gets any
        std::vector<size_t> order;
        for (size_t k = 0; k < m; ++k)
            if (!exhausted[k]) order.push_back(k);
        const double now = now_ms();
        std::vector<double> key(m, 0.0);
        for (size_t k : order) {
            const Request& r = *s->active[k];
            key[k] = s->opt.policy == KDE_SERVE_SJF ? remaining_key(s, r, now) : (double)r.id;
        }
        std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return key[a] < key[b]; });
        for (size_t k : order) {
            if (budget <= 0) break;
            take(k, INT64_MAX);
        }
    } else {
        // round-robin, one pair item per request per turn (processor sharing)
        const size_t turn = s->rr % std::max<size_t>(1, m);
        while (left > 0 && budget > 0) {
            for (size_t q = 0; q < m && budget > 0; ++q) {
                const size_t k = (turn + q) % m;
                if (!exhausted[k]) take(k, 1);
            }
        }
    }
    s->rr = (s->rr + 1) % std::max<size_t>(1, m);
    size_t total = 0;
    for (auto& v : stage_lists) total += v.size();
    if (total == 0) return KDE_OK;
    // A step that cannot run (its launch failed, or a failure injected for
    // tests) fails the requests it lists: their device state misses these
    // items, so they complete with the failure once no earlier step can still
    // write their memory; the other requests go on.
    auto fail_step = [&](int32_t code) {
        for (size_t k = 0; k < m; ++k)
            if (listed[k] && !s->active[k]->fail) s->active[k]->fail = code;
        ++s->failed_steps;
        ++s->steps;
        return KDE_OK;
    };
    if (s->fail_next) {
        const int32_t code = s->fail_next;
        s->fail_next = 0;
        return fail_step(code);
    }
    // the compute stream waits for sample copies of newly listed requests
    for (auto& rp : s->active)
        if (rp->wait_copy) {
            HIPCHK(hipStreamWaitEvent(s->stream, rp->copied, 0));
            rp->wait_copy = false;
        }
    const int b = s->next_buf;
    s->next_buf ^= 1;
    if (total > s->items_cap) {
        // grow both list buffers (no step may be using them: drain first)
        for (auto& st : s->inflight) HIPCHK(hipEventSynchronize(st.done));
        size_t cap = std::max<size_t>(total, 2 * s->items_cap);
        for (int q = 0; q < 2; ++q) {
            if (s->h_items[q]) HIPCHK(hipHostFree(s->h_items[q]));
            HIPCHK(hipHostMalloc((void**)&s->h_items[q], cap * sizeof(Item), hipHostMallocDefault));
            int st = s->d_items[q].ensure(cap * sizeof(Item), "server work list");
            if (st) return st;
        }
        s->items_cap = cap;
    }
    HIPCHK(hipEventSynchronize(s->items_free[b]));  // the previous copy out of this buffer is done
    Item* dst = s->h_items[b];
    for (auto& v : stage_lists) {
        if (v.empty()) continue;
        std::memcpy(dst, v.data(), v.size() * sizeof(Item));
        dst += v.size();
    }
    HIPCHK(hipMemcpyAsync(s->d_items[b].p, s->h_items[b], total * sizeof(Item), hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipEventRecord(s->items_free[b], s->stream));
    uint32_t* ticket = (uint32_t*)s->d_ticket.p + 64 * b;
    HIPCHK(hipMemsetAsync(ticket, 0, sizeof(uint32_t), s->stream));
    LaunchArgs a{};
    a.items = (const Item*)s->d_items[b].p;
    a.n_items = (uint32_t)total;
    a.descs = (const Desc*)s->d_descs.p;
    a.states = (State*)s->d_states.p;
    a.slots = (Slot*)s->arena_buf.p;
    a.pubs = (Pub*)s->d_pubs.p;
    a.ticket = ticket;
    a.pc = s->ctx->pc;
    int64_t widest_item = 0;
    for (size_t k = 0; k < m; ++k)
        if (listed[k]) widest_item = std::max(widest_item, s->active[k]->geom.TI * (s->active[k]->geom.W + 4));
    a.timeout_ticks = wait_ticks(s->ctx, widest_item);
    const bool wide = use_wide(s->ctx, step_pairs);  // the four-wave kernel for large steps
    if (launch_persistent(s->ctx->precision, s->ctx->R, wide, step_grid(s->ctx, (int64_t)total, wide), s->stream, a) !=
        hipSuccess) {
        (void)hipGetLastError();
        return fail_step(KDE_EDEVICE);
    }
    for (size_t k = 0; k < m; ++k)
        if (listed[k]) s->active[k]->launched_step = s->steps;
    s->pairs_issued += step_pairs;
    HIPCHK(hipMemcpyAsync(s->h_states[b], s->d_states.p, sizeof(State) * (size_t)s->opt.max_active,
                          hipMemcpyDeviceToHost, s->stream));
    Step st;
    HIPCHK(hipEventCreateWithFlags(&st.done, hipEventDisableTiming));
    HIPCHK(hipEventRecord(st.done, s->stream));
    st.buf = b;
    st.seq = s->steps;
    s->inflight.push_back(st);
    ++s->steps;
    return KDE_OK;
}

// Hand active request k to the caller with result c and free its slot,
// arena block and budget.
void complete(kde_server* s, size_t k, kde_completion c, double t) {
    Request& r = *s->active[k];
    c.id = r.id;
    c.n = r.n;
    c.t_submit_ms = r.t_submit;
    c.t_admit_ms = r.t_admit;
    c.t_done_ms = t;
    s->done.push_back(c);
    s->arena->release(r.off, r.bytes);
    if (r.mem_kind == KDE_MEM_DEVICE) s->device_sample_bytes -= (size_t)r.n * sizeof(double);
    s->free_slots.push_back(r.slot);
    if (r.copied) (void)hipEventDestroy(r.copied);
    s->active.erase(s->active.begin() + (long)k);
}

// Retire the oldest step and collect the requests whose last stage has
// published in its state read-back.  Returns KDE_EBUSY (without error state)
// when the step is still running and block == false.
int retire_step(kde_server* s, bool block) {
    Step st = s->inflight.front();
    if (block) {
        HIPCHK(hipEventSynchronize(st.done));
    } else {
        const hipError_t q = hipEventQuery(st.done);
        if (q == hipErrorNotReady) return KDE_EBUSY;
        if (q != hipSuccess) return hip_fail(q, "hipEventQuery");
    }
    (void)hipEventDestroy(st.done);
    s->inflight.pop_front();
    const State* hs = s->h_states[st.buf];
    const double t = now_ms();
    for (size_t k = 0; k < s->active.size();) {
        Request& r = *s->active[k];
        const State& h = hs[r.slot];
        // only a read-back taken after the step that listed the request's last
        // items can show its final flag (older ones may still hold the state of
        // the slot's previous request)
        if (!r.fail && r.stage >= NUM_STAGES && r.last_step >= 0 && st.seq >= r.last_step && h.ready[ST_PSI4]) {
            kde_completion c{};
            fill_result(h, &c.result);
            if (c.result.status) c.result.h = NAN;
            s->pairs_done += r.pairs;
            complete(s, k, c, t);  // erases active[k]: r is gone after this
        } else {
            ++k;
        }
    }
    return KDE_OK;
}

// Complete the failed requests that no step in flight can still touch.
void reap_failed(kde_server* s) {
    const int64_t oldest = s->inflight.empty() ? INT64_MAX : s->inflight.front().seq;
    const double t = now_ms();
    for (size_t k = 0; k < s->active.size();) {
        Request& r = *s->active[k];
        if (r.fail && r.launched_step < oldest) {
            kde_completion c{};
            c.result.h = NAN;
            c.result.status = r.fail;
            complete(s, k, c, t);
        } else {
            ++k;
        }
    }
}

}  // namespace

extern "C" {

void kde_server_options_init(kde_server_options* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->mem_budget = (int64_t)8 << 30;
    o->max_active = 64;
    o->step_pairs = (int64_t)1 << 34;
    o->policy = KDE_SERVE_FCFS;
    o->aging_ms = 0;
    o->fill = KDE_FILL_SHARE;
}

int kde_server_create(kde_server** out, kde_ctx* ctx, const kde_server_options* opt) {
    if (!out || !ctx) return set_err(KDE_EINVAL, "null server output or context");
    *out = nullptr;
    kde_server_options o;
    kde_server_options_init(&o);
    if (opt) o = *opt;
    if (o.mem_budget < ((int64_t)1 << 20) || o.max_active < 1 || o.max_active > 65536 || o.step_pairs < 1 ||
        (o.policy != KDE_SERVE_FCFS && o.policy != KDE_SERVE_SJF) || o.aging_ms < 0 ||
        (o.fill != KDE_FILL_SHARE && o.fill != KDE_FILL_PRIORITY))
        return set_err(KDE_EINVAL, "bad server options");
    DeviceGuard dg(ctx->device);
    auto s = std::make_unique<kde_server>();
    s->ctx = ctx;
    s->opt = o;
    HIPCHK(hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking));
    HIPCHK(hipStreamCreateWithFlags(&s->copy_stream, hipStreamNonBlocking));
    int st;
    if ((st = s->arena_buf.ensure((size_t)o.mem_budget, "server arena"))) return st;
    if ((st = s->d_descs.ensure(sizeof(Desc) * (size_t)o.max_active, "server descriptors"))) return st;
    if ((st = s->d_states.ensure(sizeof(State) * (size_t)o.max_active, "server states"))) return st;
    if ((st = s->d_pubs.ensure(sizeof(Pub) * kPubReplicas * (size_t)o.max_active, "server published scalars")))
        return st;
    if ((st = s->d_ticket.ensure(512, "server tickets"))) return st;
    s->arena = std::make_unique<Arena>((size_t)o.mem_budget);
    HIPCHK(hipHostMalloc((void**)&s->h_descs, sizeof(Desc) * (size_t)o.max_active, hipHostMallocDefault));
    for (int q = 0; q < 2; ++q) {
        HIPCHK(hipHostMalloc((void**)&s->h_states[q], sizeof(State) * (size_t)o.max_active, hipHostMallocDefault));
        std::memset(s->h_states[q], 0, sizeof(State) * (size_t)o.max_active);
    }
    for (int q = 0; q < 2; ++q) {
        HIPCHK(hipEventCreateWithFlags(&s->items_free[q], hipEventDisableTiming));
        HIPCHK(hipEventRecord(s->items_free[q], s->stream));
    }
    for (int32_t k = o.max_active - 1; k >= 0; --k) s->free_slots.push_back(k);
    *out = s.release();
    return ok();
}

void kde_server_destroy(kde_server* s) {
    if (!s) return;
    DeviceGuard dg(s->ctx->device);
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    if (s->copy_stream) (void)hipStreamSynchronize(s->copy_stream);
    for (auto& st : s->inflight) (void)hipEventDestroy(st.done);
    for (auto& r : s->active)
        if (r->copied) (void)hipEventDestroy(r->copied);
    for (auto& r : s->queue)
        if (r->copied) (void)hipEventDestroy(r->copied);
    for (int q = 0; q < 2; ++q) {
        if (s->h_items[q]) (void)hipHostFree(s->h_items[q]);
        if (s->items_free[q]) (void)hipEventDestroy(s->items_free[q]);
    }
    if (s->h_descs) (void)hipHostFree(s->h_descs);
    for (int q = 0; q < 2; ++q)
        if (s->h_states[q]) (void)hipHostFree(s->h_states[q]);
    if (s->stream) (void)hipStreamDestroy(s->stream);
    if (s->copy_stream) (void)hipStreamDestroy(s->copy_stream);
    delete s;
}

int kde_server_submit(kde_server* s, const void* x, int64_t n, int mem_kind, kde_stream producer, int64_t* id) {
    if (!s || !id) return set_err(KDE_EINVAL, "null server or id");
    int st = check_x(x, n, 2, mem_kind, KDE_F64);
    if (st) return st;
    auto r = std::make_unique<Request>();
    r->x_user = x;
    r->n = n;
    r->mem_kind = mem_kind;
    SampleSpec sp{x, n, KDE_F64, MODE_PLUGIN, 0, 0.0, 0, -1};
    describe_sample(s->ctx, sp, &r->desc);
    r->bytes = request_bytes(*r);
    if (budget_bytes(*r) > (size_t)s->opt.mem_budget)
        return set_err(KDE_ENOMEM, "request larger than the server's memory budget");
    if (mem_kind == KDE_MEM_DEVICE) {
        // the sample may still be being written on the producer's stream: the
        // server's stream waits for the work enqueued there so far before the
        // first step that lists the request
        DeviceGuard dg(s->ctx->device);
        HIPCHK(hipEventCreateWithFlags(&r->copied, hipEventDisableTiming));
        const hipError_t e = hipEventRecord(r->copied, (hipStream_t)producer);
        if (e != hipSuccess) {
            (void)hipEventDestroy(r->copied);
            return hip_fail(e, "hipEventRecord on the producer stream");
        }
    }
    r->id = s->next_id++;
    r->t_submit = now_ms();
    r->pairs = (double)n * (double)(n - 1);
    *id = r->id;
    s->queue.push_back(std::move(r));
    return ok();
}

int kde_server_cancel(kde_server* s, int64_t id) {
    if (!s) return set_err(KDE_EINVAL, "null server");
    for (auto it = s->queue.begin(); it != s->queue.end(); ++it)
        if ((*it)->id == id) {
            if ((*it)->copied) (void)hipEventDestroy((*it)->copied);
            s->queue.erase(it);
            return ok();
        }
    return set_err(KDE_EBUSY, "request is not queued (admitted, finished or unknown)");
}

int kde_server_step(kde_server* s, int32_t block, kde_server_stats* stats) {
    if (!s) return set_err(KDE_EINVAL, "null server");
    DeviceGuard dg(s->ctx->device);
    int st;
    while (!s->inflight.empty()) {  // retire every step that has finished
        st = retire_step(s, false);
        if (st == KDE_EBUSY) break;
        if (st) return st;
    }
    if (s->inflight.size() >= 2 && block && (st = retire_step(s, true))) return st;
    reap_failed(s);
    if ((st = admit(s))) return st;
    const int64_t before = s->steps;
    if (s->inflight.size() < 2 && (st = launch_step(s))) return st;
    // nothing new to launch (every active request's items are queued): wait for
    // the oldest step, then admit into whatever it freed and launch again
    if (block && s->steps == before && !s->inflight.empty()) {
        if ((st = retire_step(s, true))) return st;
        reap_failed(s);
        if ((st = admit(s))) return st;
        if (s->inflight.size() < 2 && (st = launch_step(s))) return st;
    }
    if (stats) {
        stats->active = (int32_t)s->active.size();
        stats->queued = (int32_t)s->queue.size();
        stats->inflight_steps = (int32_t)s->inflight.size();
        stats->failed_steps = s->failed_steps;
        stats->steps = s->steps;
        stats->arena_used = (int64_t)(s->arena->used() + s->device_sample_bytes);
        stats->pairs_done = s->pairs_done;
        stats->pairs_issued = s->pairs_issued;
        stats->completed_unread = (int64_t)s->done.size();
    }
    return ok();
}

int kde_server_poll(kde_server* s, kde_completion* out, int32_t max, int32_t* got) {
    if (!s || !got || (max > 0 && !out)) return set_err(KDE_EINVAL, "bad poll arguments");
    const int32_t k = std::min<int32_t>(max, (int32_t)s->done.size());
    for (int32_t q = 0; q < k; ++q) out[q] = s->done[(size_t)q];
    s->done.erase(s->done.begin(), s->done.begin() + k);
    *got = k;
    return ok();
}

int kde_server_fail_next_step(kde_server* s, int32_t code) {
    if (!s || code >= 0) return set_err(KDE_EINVAL, "null server or non-negative failure code");
    s->fail_next = code;
    return ok();
}

int kde_server_drain(kde_server* s) {
    if (!s) return set_err(KDE_EINVAL, "null server");
    kde_server_stats st{};
    for (;;) {
        const int rc = kde_server_step(s, 1, &st);
        if (rc) return rc;
        if (st.active == 0 && st.queued == 0 && st.inflight_steps == 0) break;
        if (st.active == 0 && st.queued > 0 && st.inflight_steps == 0)
            return set_err(KDE_ENOMEM, "queued requests cannot be admitted");
    }
    return ok();
}

}  // extern "C"
