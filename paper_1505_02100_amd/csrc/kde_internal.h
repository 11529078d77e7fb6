// Internal layout shared by the host runtime and the device code of
// libkdeplugin.  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kdeplugin.h"

namespace kde {

// Column chunks of a pair stage.  The row block starting at row r0 owns the
// columns [r0, n) of the upper triangle, L = n - r0 of them, and cuts them
// into m = ceil(L / Wr) chunks of equal width w (rounded up to a multiple of
// 4 for the b128 column reads).  Wr is the stage's chunk width W for row
// blocks with L > n/2, W/2 for n/4 < L <= n/2, W/4 for n/8 < L <= n/4 and
// W/8 below (not under min(W, 256)): the work list runs row blocks in
// increasing order, so the last quarter of a stage's pairs comes in smaller
// items and the blocks of the device run out of work at nearly the same
// time.  Host and device compute the chunks with this one function.
__host__ __device__ inline void row_chunks(int64_t n, int64_t r0, int64_t W, int64_t* m, int64_t* w) {
    const int64_t L = n - r0;
    if (L <= 0) {
        *m = 0;
        *w = 0;
        return;
    }
    int64_t Wr = W;
    if (2 * L <= n) Wr >>= 1;
    if (4 * L <= n) Wr >>= 1;
    if (8 * L <= n) Wr >>= 1;
    const int64_t lo = W < 256 ? W : 256;
    if (Wr < lo) Wr = lo;
    *m = (L + Wr - 1) / Wr;
    *w = (((L + *m - 1) / *m) + 3) & ~(int64_t)3;
}

// Stages of one bandwidth selection, in dependency order (Algorithm 1).
enum Stage : int32_t {
    ST_SUM = 0,   // Step I, pass 1: sum of the samples -> mean
    ST_SSQ = 1,   // Step I, pass 2: sum of squared deviations -> sigma; Steps II-III -> g1
    ST_PSI6 = 2,  // Step IV pair sum; finaliser runs Step V -> g2
    ST_PSI4 = 3,  // Step VI pair sum; finaliser runs Step VII -> h
    NUM_STAGES = 4
};

enum Mode : int32_t {
    MODE_PLUGIN = 0,  // Steps I-VII
    MODE_PSI = 1,     // Steps I (for centring) + one pair stage with a given g
};

// Work item: one unit of one stage of one sample.  For the moment stages,
// `a` is the chunk index.  For a pair stage, `a` is the row block and `b`
// the column chunk within that row block's part of the upper triangle.
struct Item {
    int32_t ds;     // sample index in the descriptor table
    int32_t stage;  // Stage
    int32_t wait;   // stage whose finaliser must have published first, or -1
    int32_t a;
    int32_t b;
    // One past the ticket of the last item of the run of consecutive items
    // of the same (sample, stage) this item belongs to in its work list;
    // 0 makes the block count this item as soon as it is finished.
    int32_t run_end;
    int64_t slot;   // index of this item's partial-sum slot
};
static_assert(sizeof(Item) == 32, "Item layout");

// Per-sample description written by the host.
struct Desc {
    const void* x;          // samples on the device
    int64_t n;
    int32_t dtype;          // 0 = f64, 1 = f32
    int32_t mode;           // Mode
    int32_t psi_r;          // MODE_PSI: 4 or 6
    int32_t chunk;          // elements per moment item
    int64_t W;              // columns per pair item
    int32_t n_items[NUM_STAGES];   // items of each stage present in the work list
    int64_t slot_base[NUM_STAGES]; // first slot of each stage
    double psi_g;           // MODE_PSI: the bandwidth g
};

// Per-sample state, zeroed by the init kernel and updated by the
// persistent kernel (counters, flags and published scalars).
struct State {
    uint32_t done[NUM_STAGES];   // items finished per stage
    uint32_t ready[NUM_STAGES];  // 1 once the stage's finaliser has published
    int32_t status;
    int32_t safe;                // clamp pair arguments (extreme spread)
    double mean;
    double scale;                // u = (x - mean) * scale for the current pair stage
    double sigma, psi8, g1, psi6, g2, psi4, h;
    double S6, S4;               // strict-upper-triangle kernel sums
    double maxdev;               // max |x - mean|
    uint64_t t_first;            // wall clock (100 MHz ticks) when the first item started
    uint64_t t_fin[NUM_STAGES];  // wall clock when each stage's finaliser published
    // Exact sums of the pair stages' item partials (Steps IV and VI) in fixed
    // point, units of 2^-64, as four 32-bit limbs added in 64-bit integers
    int64_t acc[2][4];
};

// Replicated copy of the scalars a stage's finaliser publishes for the items
// of later stages.  Each sample has kPubReplicas of them, one 128-byte line
// each; block b waits on and reads replica b mod kPubReplicas, so the blocks
// of the device do not all poll and load one line at a stage boundary.
constexpr int kPubReplicas = 16;
struct alignas(128) Pub {
    uint32_t ready[NUM_STAGES];  // 1 once the stage's finaliser has published
    int32_t status;
    int32_t safe;
    double mean;
    double scale;
    uint8_t pad[88];
};
static_assert(sizeof(Pub) == 128, "Pub layout");

// Partial result of one work item.
struct Slot {
    double v;    // Step I chunk: its sum of x - x[0] (first stage's slot) or its minimum (second stage's)
    double aux;  // its squared deviations from its own mean (first) or its maximum (second)
};

// Constants of the FP32 pair evaluation (derivation in kde_device.hip).
struct PolyConsts {
    float k_hi;    // log2(e)/2 rounded to FP32
    float k_lo;    // log2(e)/2 - k_hi rounded to FP32 (exact-k variant)
};

// Arguments of the persistent kernel.
struct LaunchArgs {
    const Item* items;
    uint32_t n_items;
    uint32_t pad0;
    const Desc* descs;
    State* states;
    Slot* slots;
    Pub* pubs;               // kPubReplicas per sample
    uint32_t* ticket;
    PolyConsts pc;
    uint64_t timeout_ticks;  // wall-clock ticks (100 MHz) an in-kernel wait may take
};

}  // namespace kde
