// Bandwidth selection that allocates nothing: kde_plugin_bandwidth_noalloc.
//
// For callers that cannot call hipMalloc (code under HIP graph capture,
// tight serving loops, harnesses that forbid allocation).  Everything one
// launch of the persistent kernel needs besides the caller's sample and
// result -- the work list, the sample's descriptor, its state record and
// published-value lines, the per-item slots and the work ticket -- lives in
// `scratch`, a static device array of fixed size that every GPU the library
// runs on holds once, for the life of the process.  Its device address is
// taken once per device with hipGetSymbolAddress when a context is created
// there (kde_ctx_create calls noalloc_init); host code uses that address,
// never the array's name.
//
// A call enqueues five kernels on the caller's stream and returns:
//   k_na_prepare  zeroes the state, its published-value lines and the
//                 ticket, writes the descriptor and the output map, and
//                 scans the pair items per row block (first item of each);
//   k_na_items    writes the work list, one thread per item of each stage;
//   k_persistent  Steps I-VII, exactly as kde_plugin_bandwidth_ex runs them;
//   k_results     the kde_result into the caller's device-accessible memory.
// The work list holds the items kde_plugin_bandwidth_ex lists for the same n
// and context (the moment items with the same slots), row-block major
// (kde_plugin_bandwidth_ex orders the pair items of samples of 2^19 or more
// band-wise instead); each item's partial enters an exact fixed-point sum,
// so the results are bitwise the same.
#include <hip/hip_runtime.h>

#include <cstddef>
#include <mutex>
#include <string>

#include "kde_runtime.h"

namespace kde {
namespace noalloc {

constexpr int64_t kMaxItems = 262144;  // work items of one selection, all four stages

constexpr size_t up256(size_t b) { return (b + 255) & ~(size_t)255; }
constexpr size_t kOffTicket = 0;
constexpr size_t kOffState = 256;
constexpr size_t kOffPub = kOffState + up256(sizeof(State));
constexpr size_t kOffDesc = kOffPub + up256(sizeof(Pub) * kPubReplicas);
constexpr size_t kOffOutmap = kOffDesc + up256(sizeof(Desc));
constexpr size_t kOffRowFirst = kOffOutmap + 256;
constexpr size_t kOffItems = kOffRowFirst + up256(sizeof(int32_t) * (kMaxItems + 1));
constexpr size_t kOffSlots = kOffItems + up256(sizeof(Item) * kMaxItems);
constexpr size_t kBytes = kOffSlots + up256(sizeof(Slot) * kMaxItems);
static_assert(KDE_NOALLOC_MAX_ITEMS == kMaxItems, "public limit");
static_assert(KDE_NOALLOC_SCRATCH_BYTES == kBytes, "public size");

}  // namespace noalloc
}  // namespace kde

static __device__ __align__(256) unsigned char scratch[kde::noalloc::kBytes];

namespace kde {
namespace noalloc {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
unsigned char* g_ptr[kMaxDevices] = {};

struct Parts {
    uint32_t* ticket;
    State* state;
    Pub* pubs;
    Desc* desc;
    int32_t* outmap;
    int32_t* rb_first;
    Item* items;
    Slot* slots;
};

__host__ __device__ inline Parts parts(unsigned char* base) {
    Parts p;
    p.ticket = (uint32_t*)(base + kOffTicket);
    p.state = (State*)(base + kOffState);
    p.pubs = (Pub*)(base + kOffPub);
    p.desc = (Desc*)(base + kOffDesc);
    p.outmap = (int32_t*)(base + kOffOutmap);
    p.rb_first = (int32_t*)(base + kOffRowFirst);
    p.items = (Item*)(base + kOffItems);
    p.slots = (Slot*)(base + kOffSlots);
    return p;
}

constexpr int kPrepThreads = 1024;

// One block.  Clears what must start at zero, writes the descriptor and the
// output map (result 0 from state 0), and the exclusive prefix sums of the
// pair items per row block: rb_first[rb] is the index (within a pair stage)
// of row block rb's first item, rb_first[RB] the stage's item count.
__global__ __launch_bounds__(kPrepThreads) void k_na_prepare(unsigned char* base, Desc d, int64_t TI,
                                                            int64_t RB) {
    const Parts p = parts(base);
    const int tid = threadIdx.x;
    if (tid == 0) {
        State s = {};
        *p.state = s;
        *p.ticket = 0u;
        *p.desc = d;
        p.outmap[0] = 0;
        p.outmap[1] = 0;
    }
    if (tid < kPubReplicas) {
        Pub q = {};
        p.pubs[tid] = q;
    }
    __shared__ int32_t wave_tot[kPrepThreads / 64];
    const int lane = tid & 63, wave = tid >> 6;
    int32_t carry = 0;
    for (int64_t b0 = 0; b0 < RB; b0 += kPrepThreads) {
        const int64_t rb = b0 + tid;
        int64_t m = 0, w = 0;
        if (rb < RB) row_chunks(d.n, rb * TI, d.W, &m, &w);
        // inclusive scan within the wave, then over the waves' totals
        int32_t v = (int32_t)m;
        for (int off = 1; off < 64; off <<= 1) {
            const int32_t u = __shfl_up(v, off, 64);
            if (lane >= off) v += u;
        }
        if (lane == 63) wave_tot[wave] = v;
        __syncthreads();
        int32_t before = carry;
        for (int k = 0; k < wave; ++k) before += wave_tot[k];
        if (rb < RB) p.rb_first[rb] = before + v - (int32_t)m;
        int32_t all = 0;
        for (int k = 0; k < kPrepThreads / 64; ++k) all += wave_tot[k];
        carry += all;
        __syncthreads();  // wave_tot is rewritten by the next round
    }
    if (tid == 0) p.rb_first[RB] = carry;
}

// One thread per item index q of each stage.  The list is stage-major
// (Step I's two stages, then Step IV's and Step VI's pair items, row blocks
// in increasing order, column chunks in increasing order within a row
// block); every stage of the one sample is a single run, and item k's slot
// is k (the context's plans list the same items in this order below 2^19
// samples, band-wise above; pair items use no slot).
__global__ void k_na_items(unsigned char* base, int32_t nm, int32_t np, int64_t RB) {
    const Parts p = parts(base);
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t s1 = nm, s2 = 2 * nm, s3 = 2 * nm + np, s4 = 2 * nm + 2 * np;
    if (q < nm) {
        p.items[q] = Item{0, ST_SUM, -1, (int32_t)q, 0, s1, (int64_t)q};
        p.items[s1 + q] = Item{0, ST_SSQ, ST_SUM, (int32_t)q, 0, s2, (int64_t)(s1 + q)};
    }
    if (q < np) {
        // the row block holding item q: the last rb with rb_first[rb] <= q
        int64_t lo = 0, hi = RB - 1;
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) >> 1;
            if (p.rb_first[mid] <= q)
                lo = mid;
            else
                hi = mid - 1;
        }
        const int32_t rb = (int32_t)lo, cb = (int32_t)(q - p.rb_first[lo]);
        p.items[s2 + q] = Item{0, ST_PSI6, ST_SSQ, rb, cb, s3, (int64_t)(s2 + q)};
        p.items[s3 + q] = Item{0, ST_PSI4, ST_PSI6, rb, cb, s4, (int64_t)(s3 + q)};
    }
}

}  // namespace noalloc

namespace rt {

int noalloc_init(int device) {
    if (device < 0 || device >= noalloc::kMaxDevices)
        return set_err(KDE_EINVAL, "device ordinal beyond the no-allocation scratch table");
    std::lock_guard<std::mutex> lk(noalloc::g_mu);
    if (noalloc::g_ptr[device]) return KDE_OK;
    DeviceGuard dg(device);
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
        (void)hipGetLastError();
        return set_err(KDE_EDEVICE, std::string("hipGetSymbolAddress of the no-allocation scratch: ") +
                                        hipGetErrorString(e));
    }
    noalloc::g_ptr[device] = (unsigned char*)ptr;
    return KDE_OK;
}

}  // namespace rt
}  // namespace kde

using namespace kde;
using namespace kde::rt;

extern "C" int kde_plugin_bandwidth_noalloc(kde_ctx* c, const void* x, int64_t n, int dtype,
                                            kde_stream stream, kde_result* out) {
    if (!c || !out) return set_err(KDE_EINVAL, "null context or output");
    int st = check_x(x, n, 2, KDE_MEM_DEVICE, dtype);
    if (st) return st;
    DeviceGuard dg(c->device);
    unsigned char* base = nullptr;
    {
        std::lock_guard<std::mutex> lk(noalloc::g_mu);
        base = c->device < noalloc::kMaxDevices ? noalloc::g_ptr[c->device] : nullptr;
    }
    if (!base) return set_err(KDE_EDEVICE, "no-allocation scratch not set up on the context's device");
    if (!on_device(c, x)) return set_err(KDE_EINVAL, "x must be device memory on the context's GPU");
    kde_result* dout = device_view(c, out);
    if (!dout)
        return set_err(KDE_EINVAL, "out must be device memory on the context's GPU or pinned host memory");

    SampleSpec sp{x, n, dtype, MODE_PLUGIN, 0, 0.0, 0, -1};
    Desc d;
    describe_sample(c, sp, &d);
    int64_t total = 0;
    for (int s = 0; s < NUM_STAGES; ++s) {
        d.slot_base[s] = total;
        total += d.n_items[s];
    }
    if (total > noalloc::kMaxItems)
        return set_err(KDE_EINVAL, "the work list of " + std::to_string(total) +
                                       " items exceeds the no-allocation scratch (" +
                                       std::to_string(noalloc::kMaxItems) + " items)");
    const PairGeom g = pair_geom(c, n);
    const int32_t nm = d.n_items[ST_SUM], np = d.n_items[ST_PSI6];
    hipStream_t s = (hipStream_t)stream;
    const noalloc::Parts p = noalloc::parts(base);

    hipLaunchKernelGGL(noalloc::k_na_prepare, dim3(1), dim3(noalloc::kPrepThreads), 0, s, base, d, g.TI, g.RB);
    HIPCHK(hipGetLastError());
    const int64_t widest = nm > np ? nm : np;
    hipLaunchKernelGGL(noalloc::k_na_items, dim3((unsigned)((widest + 255) / 256)), dim3(256), 0, s, base, nm, np,
                       g.RB);
    HIPCHK(hipGetLastError());
    LaunchArgs a{};
    a.items = p.items;
    a.n_items = (uint32_t)total;
    a.descs = p.desc;
    a.states = p.state;
    a.slots = p.slots;
    a.pubs = p.pubs;
    a.ticket = p.ticket;
    a.pc = c->pc;
    a.timeout_ticks = wait_ticks(c, g.TI * (g.W + 4));
    // always the three-wave kernel: it needs no scratch (private) memory, so
    // its launch never makes the HIP runtime grow its scratch pool; the
    // four-wave kernel spills registers (same results, bitwise)
    const int grid = grid_for(c, widest, false);
    HIPCHK(launch_persistent(c->precision, c->R, false, grid, s, a));
    c->last_grid = grid;
    c->last_waves = 3;
    HIPCHK(launch_results(p.state, p.outmap, 1, dout, s));
    return ok();
}
