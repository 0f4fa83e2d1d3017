// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>

#include "rafi.h"

#define RAFI_HIP_CHECK(expr)                                                        \
    do {                                                                            \
        hipError_t rafi_e_ = (expr);                                                \
        if (rafi_e_ != hipSuccess) {                                                \
            std::fprintf(stderr, "librafi: %s failed: %s (%s:%d)\n", #expr,         \
                         hipGetErrorString(rafi_e_), __FILE__, __LINE__);           \
            return RAFI_ERR_HIP;                                                    \
        }                                                                           \
    } while (0)

#define RAFI_LAUNCH_CHECK()                                                         \
    do {                                                                            \
        hipError_t rafi_e_ = hipGetLastError();                                     \
        if (rafi_e_ != hipSuccess) {                                                \
            std::fprintf(stderr, "librafi: launch failed: %s (%s:%d)\n",            \
                         hipGetErrorString(rafi_e_), __FILE__, __LINE__);           \
            return RAFI_ERR_HIP;                                                    \
        }                                                                           \
    } while (0)

namespace rafi {

// ------------------------------------------------------------ split plan ---
// The forward step runs as: per-tile destination histogram -> exclusive scan
// over the (destination-major, tile-minor) count table -> stable scatter.
struct SplitPlan {
    uint64_t n = 0;          // slots
    int32_t D = 0;           // domains
    uint32_t S = 0;          // item bytes
    uint32_t tile = 0;       // slots per tile
    uint32_t n_tiles = 0;
    uint64_t rows = 0;       // D + 2 (domains, done, bad)
    uint64_t M = 0;          // rows * n_tiles table entries
    uint32_t scan_blocks = 0;
    uint64_t off_table = 0, off_part = 0, off_dummy = 0, off_done = 0, bytes = 0;  // workspace layout
    // the item array may be read up to 16 bytes past its end (allocations the
    // library pads for this: context queues)
    bool padded = false;
    // off_dummy: 16 bytes any scatter lane may overwrite; off_done: the finished-tile
    // counter of the fused histogram + scan launch (zero between launches)
    // Lockstep scatter (large splits of items that are not whole 16-byte
    // pieces): tiles of `lock` chunks of 2048 slots; the workspace at
    // off_pre holds, per chunk and destination, the items bound there in the
    // earlier chunks of the chunk's tile (u16). lock = 0: off.
    uint32_t lock = 0;
    uint32_t n_chunks = 0;
    uint64_t off_pre = 0;
};

// allow_lock: the plan may use the lockstep scatter (its workspace grows by
// 2 bytes per chunk and destination).
SplitPlan split_plan(uint64_t n, int32_t D, uint32_t S, bool allow_lock = true);
// Select the staged scatter shape (0 = automatic, 1..17 = fixed shapes).
int split_set_variant(int v);
// A plan whose workspace covers every n <= cap.
SplitPlan split_plan_bound(uint64_t cap, int32_t D, uint32_t S);

// Optional events recorded around the split's passes (on the split stream).
struct SplitEvents {
    hipEvent_t begin = nullptr, before_scatter = nullptr, end = nullptr;
};

// Run the split. offsets: device u64 [D+1]; summary: device u64 [4], or [5]
// with dropped: {total, done, bad, n_tiles_app, dropped}; tile_offsets
// (optional): device u32 [D+1] built for tiles of tile_items. dropped
// (optional): device counter read into summary[4] and reset. fused: allow the
// one-launch histogram + scan + finalize for small tables (the workspace's
// first 4 bytes must be zero, as the context keeps them).
int split_run(const SplitPlan &p, const void *items, const int32_t *dest, void *out,
              uint64_t *offsets, uint64_t *summary, uint32_t *tile_offsets, uint32_t tile_items,
              void *workspace, hipStream_t stream, const SplitEvents *ev = nullptr,
              unsigned long long *dropped = nullptr, bool fused = false);

}  // namespace rafi

// ------------------------------------------------------------- context ---
struct rafi_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int32_t D = 0;
    uint32_t S = 0;
    uint64_t cap = 0;
    void *buf[2] = {nullptr, nullptr};
    int cur_in = 0;                     // buf[cur_in] is the input queue
    int32_t *dest = nullptr;            // [cap]
    uint64_t *offsets = nullptr;        // [D+1]
    uint32_t *tile_offsets = nullptr;   // [D+1]
    uint64_t *summary = nullptr;        // [4] device
    unsigned long long *dropped = nullptr;  // device counter
    // Persistent domain kernels: [0] next queue index to hand out, [1] waves
    // that have exited. Zero between launches: the last wave to exit resets both.
    unsigned long long *work = nullptr;
    unsigned long long *append = nullptr;  // slots taken by rafi_emit since the last rafi_open
    uint64_t *host_summary = nullptr;   // pinned [8]
    hipEvent_t summary_ready = nullptr; // recorded after each round's summary copy
    void *ws = nullptr;
    uint64_t ws_bytes = 0;
    uint64_t n_in = 0, n_slots = 0;
    uint64_t wave_slots = 0;            // n_slots of the last rafi_begin (item ids stay below it)
    uint32_t tile_items = 256, n_tiles = 0;
    int debug = 0;
    rafi_stats_t stats{};
    // profiling: event pairs waiting to be resolved
    int prof_on = 0;
    rafi_profile prof{};
    struct Pending {
        int kind;  // 0 split (3 events), 1 domain (2 events)
        hipEvent_t e[3];
        uint64_t slots;
    };
    static constexpr int kMaxPending = 64;
    Pending pending[kMaxPending];
    int n_pending = 0;
    hipEvent_t pool[3 * kMaxPending];
    int pool_size = 0;
};

namespace rafi {
int ctx_fill_poison(rafi_ctx *ctx, uint64_t n);
// Domain-kernel timing: prof_domain_begin returns a handle (or -1 when off)
// to pass to prof_domain_end after the launch.
int prof_domain_begin(rafi_ctx *ctx);
void prof_domain_end(rafi_ctx *ctx, int h);
// Resolve pending event pairs: all of them after synchronising the context
// stream (wait), or only those already complete, in order.
int prof_resolve(rafi_ctx *ctx, bool wait);
// The two halves of rafi_round: enqueue the split of the current output slots
// and the copy of its summary to the host (no wait); then wait for that copy
// only and take the results (queue length, statistics). Work enqueued between
// the two keeps running. round_finish does not touch the output slots.
int round_enqueue(rafi_ctx *ctx);
int round_finish(rafi_ctx *ctx, uint64_t *total);

// The round loop with the host one step ahead of the device. After a forward
// step is enqueued, the next domain launch is enqueued at once as
// launch(bound), with bound >= the queue length that step will produce (the
// kernel reads the exact length on the device), and only then does the host
// wait for the step's total; so the device never waits for the host between
// the two. slots(n): output slots a launch over n queued items writes. The
// last launch, over an empty queue, does nothing. *rounds: forward steps;
// *forwarded: items they delivered.
template <typename Launch, typename Slots>
int run_rounds(rafi_ctx *c, int32_t max_rounds, int32_t *rounds, uint64_t *forwarded, Launch launch, Slots slots)
{
    int32_t r = 0;
    uint64_t fwd = 0;
    int rc = round_enqueue(c);
    uint64_t bound = c->n_slots;
    while (rc == RAFI_OK) {
        ++r;
        const bool more = r < max_rounds;
        const int lrc = more ? launch(bound) : RAFI_OK;
        uint64_t total = 0;
        rc = round_finish(c, &total);
        fwd += total;
        if (rc == RAFI_OK) rc = lrc;
        if (rc != RAFI_OK || total == 0) break;
        if (!more) {
            rc = RAFI_ERR_MAX_ROUNDS;
            break;
        }
        c->n_slots = slots(total);
        bound = c->n_slots;
        rc = round_enqueue(c);
    }
    if (rounds) *rounds = r;
    if (forwarded) *forwarded = fwd;
    return rc;
}
}
