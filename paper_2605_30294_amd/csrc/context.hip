// Host context: queue ownership, the device view and the forward step
// (Sec. 3.4 of the paper: create a context, size its queues, hand kernels a
// device interface, call forwardRays() between kernel launches).
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>

#include "internal.h"

namespace rafi {
namespace {

__global__ void fill_i32_kernel(int32_t *p, uint64_t n, int32_t v)
{
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Empty queue: offsets, tile offsets and summary all zero; dropped counter reset.
__global__ void reset_kernel(uint64_t *offsets, uint32_t *tile_offsets, int32_t D, uint64_t *summary,
                             unsigned long long *dropped)
{
    for (int32_t e = threadIdx.x; e <= D; e += blockDim.x) {
        offsets[e] = 0;
        tile_offsets[e] = 0;
    }
    if (threadIdx.x < 4) summary[threadIdx.x] = 0;
    if (threadIdx.x == 0) *dropped = 0;
}

// Append-mode output: every slot RAFI_DONE, append counter zero.
__global__ void open_append_kernel(int32_t *dest, uint64_t n, unsigned long long *append)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) *append = 0;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        dest[i] = RAFI_DONE;
}

bool valid_shape(int32_t D, uint32_t S)
{
    return D >= 1 && D <= RAFI_MAX_DOMAINS && S >= 4 && S <= RAFI_MAX_ITEM_BYTES && S % 4 == 0;
}

void free_queues(rafi_ctx *c)
{
    for (void *&b : c->buf) {
        if (b) (void)hipFree(b);
        b = nullptr;
    }
    if (c->dest) (void)hipFree(c->dest);
    if (c->ws) (void)hipFree(c->ws);
    c->dest = nullptr;
    c->ws = nullptr;
    c->ws_bytes = 0;
}

int alloc_queues(rafi_ctx *c, uint64_t cap)
{
    const SplitPlan p = split_plan_bound(cap, c->D, c->S);
    // item buffers padded by 16 bytes: the split may read whole 16-byte
    // pieces past the last item
    if (hipMalloc(&c->buf[0], cap * c->S + 16) != hipSuccess || hipMalloc(&c->buf[1], cap * c->S + 16) != hipSuccess ||
        hipMalloc(reinterpret_cast<void **>(&c->dest), cap * sizeof(int32_t)) != hipSuccess ||
        hipMalloc(&c->ws, p.bytes) != hipSuccess) {
        (void)hipGetLastError();
        free_queues(c);
        return RAFI_ERR_OOM;
    }
    // the workspace head holds the fused scan's finished-tile counter: zero once
    if (hipMemset(c->ws, 0, 256) != hipSuccess) {
        (void)hipGetLastError();
        free_queues(c);
        return RAFI_ERR_HIP;
    }
    c->ws_bytes = p.bytes;
    c->cap = cap;
    return RAFI_OK;
}

int empty_queue(rafi_ctx *c)
{
    hipLaunchKernelGGL(reset_kernel, dim3(1), dim3(1024), 0, c->stream, c->offsets, c->tile_offsets, c->D,
                       c->summary, c->dropped);
    RAFI_LAUNCH_CHECK();
    c->n_in = 0;
    c->n_tiles = 0;
    return RAFI_OK;
}

}  // namespace

int ctx_fill_poison(rafi_ctx *c, uint64_t n)
{
    if (!c->debug || n == 0) return RAFI_OK;
    const uint32_t blocks = (uint32_t)std::min<uint64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(fill_i32_kernel, dim3(blocks), dim3(256), 0, c->stream, c->dest, n, RAFI_POISON);
    RAFI_LAUNCH_CHECK();
    return RAFI_OK;
}

namespace {
hipEvent_t take_event(rafi_ctx *c)
{
    if (c->pool_size > 0) return c->pool[--c->pool_size];
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void give_event(rafi_ctx *c, hipEvent_t e)
{
    if (!e) return;
    if (c->pool_size < 3 * rafi_ctx::kMaxPending) c->pool[c->pool_size++] = e;
    else (void)hipEventDestroy(e);
}
}  // namespace

int prof_resolve(rafi_ctx *c, bool wait)
{
    if (c->n_pending == 0) return RAFI_OK;
    if (wait) RAFI_HIP_CHECK(hipStreamSynchronize(c->stream));
    int done = 0;
    for (; done < c->n_pending; ++done) {
        rafi_ctx::Pending &p = c->pending[done];
        if (!wait) {  // only pairs whose last event has completed, in order
            const hipError_t q = hipEventQuery(p.e[p.kind == 0 ? 2 : 1]);
            if (q == hipErrorNotReady) {
                (void)hipGetLastError();
                break;
            }
            RAFI_HIP_CHECK(q);
        }
        float a = 0.0f, b = 0.0f;
        if (p.kind == 0) {
            if (hipEventElapsedTime(&a, p.e[0], p.e[2]) == hipSuccess) c->prof.split_ms += a;
            if (hipEventElapsedTime(&b, p.e[1], p.e[2]) == hipSuccess) c->prof.scatter_ms += b;
            c->prof.split_calls++;
            c->prof.scatter_calls++;
            c->prof.split_slots += p.slots;
        } else {
            if (hipEventElapsedTime(&a, p.e[0], p.e[1]) == hipSuccess) c->prof.domain_ms += a;
            c->prof.domain_calls++;
        }
        for (int k = 0; k < (p.kind == 0 ? 3 : 2); ++k) give_event(c, p.e[k]);
    }
    for (int i = done; i < c->n_pending; ++i) c->pending[i - done] = c->pending[i];
    c->n_pending -= done;
    return RAFI_OK;
}

int prof_domain_begin(rafi_ctx *c)
{
    if (!c->prof_on) return -1;
    if (c->n_pending >= rafi_ctx::kMaxPending && prof_resolve(c, true) != RAFI_OK) return -1;
    rafi_ctx::Pending &p = c->pending[c->n_pending];
    p.kind = 1;
    p.e[0] = take_event(c);
    p.e[1] = take_event(c);
    p.slots = 0;
    if (!p.e[0] || !p.e[1] || hipEventRecord(p.e[0], c->stream) != hipSuccess) return -1;
    return c->n_pending++;
}

void prof_domain_end(rafi_ctx *c, int h)
{
    if (h < 0) return;
    (void)hipEventRecord(c->pending[h].e[1], c->stream);
}

int round_enqueue(rafi_ctx *c)
{
    SplitPlan p = split_plan(c->n_slots, c->D, c->S);
    p.padded = true;  // the context's item buffers are padded (alloc_queues)
    if (p.bytes > c->ws_bytes) return RAFI_ERR_STATE;
    SplitEvents ev;
    const SplitEvents *evp = nullptr;
    if (c->prof_on && (c->n_pending < rafi_ctx::kMaxPending || prof_resolve(c, true) == RAFI_OK)) {
        rafi_ctx::Pending &pp = c->pending[c->n_pending];
        pp.kind = 0;
        pp.slots = c->n_slots;
        for (int k = 0; k < 3; ++k) pp.e[k] = take_event(c);
        if (pp.e[0] && pp.e[1] && pp.e[2]) {
            ev.begin = pp.e[0];
            ev.before_scatter = pp.e[1];
            ev.end = pp.e[2];
            evp = &ev;
            c->n_pending++;
        }
    }
    // the split also moves the dropped-emit count into summary[4] and resets it
    int rc = split_run(p, c->buf[1], c->dest, c->buf[0], c->offsets, c->summary, c->tile_offsets,
                       c->tile_items, c->ws, c->stream, evp, c->dropped, true);
    if (rc != RAFI_OK) return rc;
    RAFI_HIP_CHECK(hipMemcpyAsync(c->host_summary, c->summary, sizeof(uint64_t) * 5, hipMemcpyDeviceToHost,
                                  c->stream));
    if (!c->summary_ready) RAFI_HIP_CHECK(hipEventCreateWithFlags(&c->summary_ready, hipEventDisableTiming));
    RAFI_HIP_CHECK(hipEventRecord(c->summary_ready, c->stream));
    return RAFI_OK;
}

int round_finish(rafi_ctx *c, uint64_t *total)
{
    RAFI_HIP_CHECK(hipEventSynchronize(c->summary_ready));
    const uint64_t *h = c->host_summary;
    if (c->n_pending) {
        int rc = prof_resolve(c, false);
        if (rc != RAFI_OK) return rc;
    }
    c->prof.split_items += c->prof_on ? h[0] : 0;
    c->n_in = h[0];
    c->n_slots = h[0];
    c->n_tiles = (uint32_t)h[3];
    c->stats.rounds++;
    c->stats.forwarded += h[0];
    c->stats.done += h[1];
    c->stats.bad_dest += h[2];
    c->stats.dropped += h[4];
    c->stats.last_total = h[0];
    if (total) *total = h[0];
    if (h[2]) return RAFI_ERR_BAD_DEST;
    if (h[4]) return RAFI_ERR_OVERFLOW;
    return RAFI_OK;
}

}  // namespace rafi

using namespace rafi;

namespace {
// Workspace of rafi_multisplit_noalloc: file-scope device memory, one copy
// per device, held until the process ends. In host code the array's name is
// not a device address; only the address hipGetSymbolAddress returns (kept
// per device in g_scratch) may reach a kernel or a copy.
constexpr uint64_t kNoAllocScratchBytes = 32ull << 20;
__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices] = {};

// The scratch address on the device of stream s, which must be the current
// device. Looked up once per device, on the first call there.
int noalloc_scratch(hipStream_t s, void **out)
{
    int dev = 0;
    RAFI_HIP_CHECK(hipGetDevice(&dev));
    if (s) {
        hipDevice_t sd = 0;
        RAFI_HIP_CHECK(hipStreamGetDevice(s, &sd));
        if (sd != dev) return RAFI_ERR_ARG;
    }
    if (dev < 0 || dev >= kMaxDevices) return RAFI_ERR_ARG;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        RAFI_HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return RAFI_ERR_HIP;
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return RAFI_OK;
}
}  // namespace

extern "C" {

const char *rafi_strerror(int code)
{
    switch (code) {
    case RAFI_OK: return "ok";
    case RAFI_ERR_ARG: return "invalid argument";
    case RAFI_ERR_OOM: return "out of device memory";
    case RAFI_ERR_HIP: return "HIP runtime error";
    case RAFI_ERR_OVERFLOW: return "emits beyond the slot range were dropped";
    case RAFI_ERR_BAD_DEST: return "slots with an invalid destination were dropped";
    case RAFI_ERR_MAX_ROUNDS: return "round limit reached with items still alive";
    case RAFI_ERR_STATE: return "call not valid in the current state";
    case RAFI_ERR_TOO_LARGE: return "problem larger than the fixed scratch buffer";
    default: return "unknown error";
    }
}

int rafi_create(int32_t n_domains, uint32_t item_bytes, uint64_t capacity, rafi_ctx **out)
{
    if (!out) return RAFI_ERR_ARG;
    *out = nullptr;
    if (!valid_shape(n_domains, item_bytes) || capacity == 0 || capacity >= (1ull << 32)) return RAFI_ERR_ARG;
    rafi_ctx *c = new (std::nothrow) rafi_ctx();
    if (!c) return RAFI_ERR_OOM;
    c->D = n_domains;
    c->S = item_bytes;
    RAFI_HIP_CHECK(hipGetDevice(&c->device));
    int rc = alloc_queues(c, capacity);
    if (rc == RAFI_OK &&
        (hipMalloc(reinterpret_cast<void **>(&c->offsets), sizeof(uint64_t) * (n_domains + 1)) != hipSuccess ||
         hipMalloc(reinterpret_cast<void **>(&c->tile_offsets), sizeof(uint32_t) * (n_domains + 1)) != hipSuccess ||
         hipMalloc(reinterpret_cast<void **>(&c->summary), sizeof(uint64_t) * 8) != hipSuccess ||
         hipMalloc(reinterpret_cast<void **>(&c->dropped), sizeof(unsigned long long)) != hipSuccess ||
         hipMalloc(reinterpret_cast<void **>(&c->work), 2 * sizeof(unsigned long long)) != hipSuccess ||
         hipMemset(c->work, 0, 2 * sizeof(unsigned long long)) != hipSuccess ||
         hipMalloc(reinterpret_cast<void **>(&c->append), sizeof(unsigned long long)) != hipSuccess ||
         hipMemset(c->append, 0, sizeof(unsigned long long)) != hipSuccess ||
         hipHostMalloc(reinterpret_cast<void **>(&c->host_summary), sizeof(uint64_t) * 8, hipHostMallocDefault) != hipSuccess))
        rc = RAFI_ERR_OOM;
    if (rc == RAFI_OK) rc = empty_queue(c);
    if (rc == RAFI_OK && hipStreamSynchronize(c->stream) != hipSuccess) rc = RAFI_ERR_HIP;
    if (rc != RAFI_OK) {
        (void)hipGetLastError();
        rafi_destroy(c);
        return rc;
    }
    *out = c;
    return RAFI_OK;
}

void rafi_destroy(rafi_ctx *c)
{
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    free_queues(c);
    if (c->offsets) (void)hipFree(c->offsets);
    if (c->tile_offsets) (void)hipFree(c->tile_offsets);
    if (c->summary) (void)hipFree(c->summary);
    if (c->dropped) (void)hipFree(c->dropped);
    if (c->work) (void)hipFree(c->work);
    if (c->append) (void)hipFree(c->append);
    if (c->host_summary) (void)hipHostFree(c->host_summary);
    if (c->summary_ready) (void)hipEventDestroy(c->summary_ready);
    for (int i = 0; i < c->n_pending; ++i)
        for (int k = 0; k < (c->pending[i].kind == 0 ? 3 : 2); ++k)
            if (c->pending[i].e[k]) (void)hipEventDestroy(c->pending[i].e[k]);
    for (int i = 0; i < c->pool_size; ++i) (void)hipEventDestroy(c->pool[i]);
    delete c;
}

int rafi_resize(rafi_ctx *c, uint64_t capacity)
{
    if (!c || capacity == 0 || capacity >= (1ull << 32)) return RAFI_ERR_ARG;
    RAFI_HIP_CHECK(hipStreamSynchronize(c->stream));
    free_queues(c);
    int rc = alloc_queues(c, capacity);
    if (rc != RAFI_OK) return rc;
    c->n_slots = 0;
    return empty_queue(c);
}

int rafi_set_stream(rafi_ctx *c, void *hip_stream)
{
    if (!c) return RAFI_ERR_ARG;
    c->stream = static_cast<hipStream_t>(hip_stream);
    return RAFI_OK;
}

int rafi_set_debug(rafi_ctx *c, int32_t on)
{
    if (!c) return RAFI_ERR_ARG;
    c->debug = on ? 1 : 0;
    return RAFI_OK;
}

int rafi_set_tile_items(rafi_ctx *c, uint32_t tile_items)
{
    if (!c || tile_items == 0) return RAFI_ERR_ARG;
    c->tile_items = tile_items;
    return RAFI_OK;
}

int rafi_view(const rafi_ctx *c, rafi_device_view *v)
{
    if (!c || !v) return RAFI_ERR_ARG;
    v->in_items = c->buf[0];
    v->in_offsets = c->offsets;
    v->in_tile_offsets = c->tile_offsets;
    v->out_items = c->buf[1];
    v->out_dest = c->dest;
    v->dropped = c->dropped;
    v->n_in = c->n_in;
    v->n_slots = c->n_slots;
    v->capacity = c->cap;
    v->item_bytes = c->S;
    v->n_domains = c->D;
    v->tile_items = c->tile_items;
    v->n_tiles = c->n_tiles;
    v->append = c->append;
    return RAFI_OK;
}

int rafi_begin(rafi_ctx *c, uint64_t n_slots)
{
    if (!c || n_slots > c->cap) return RAFI_ERR_ARG;
    int rc = empty_queue(c);
    if (rc != RAFI_OK) return rc;
    c->n_slots = n_slots;
    c->wave_slots = n_slots;
    return ctx_fill_poison(c, n_slots);
}

int rafi_open(rafi_ctx *c, uint64_t n_slots, int32_t mode)
{
    if (!c || n_slots > c->cap || (mode != RAFI_SLOTS_ORDERED && mode != RAFI_SLOTS_APPEND)) return RAFI_ERR_ARG;
    c->n_slots = n_slots;
    if (mode == RAFI_SLOTS_ORDERED) return ctx_fill_poison(c, n_slots);
    const uint32_t blocks = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((n_slots + 255) / 256, 4096));
    hipLaunchKernelGGL(open_append_kernel, dim3(blocks), dim3(256), 0, c->stream, c->dest, n_slots, c->append);
    RAFI_LAUNCH_CHECK();
    return RAFI_OK;
}

int rafi_emit_bulk(rafi_ctx *c, const void *items, const int32_t *dest, uint64_t n)
{
    if (!c || n > c->n_slots || (n && (!items || !dest))) return RAFI_ERR_ARG;
    if (n == 0) return RAFI_OK;
    RAFI_HIP_CHECK(hipMemcpyAsync(c->buf[1], items, n * c->S, hipMemcpyDeviceToDevice, c->stream));
    RAFI_HIP_CHECK(hipMemcpyAsync(c->dest, dest, n * sizeof(int32_t), hipMemcpyDeviceToDevice, c->stream));
    return RAFI_OK;
}

int rafi_round(rafi_ctx *c, uint64_t *counts, uint64_t *total)
{
    if (!c) return RAFI_ERR_ARG;
    int rc = round_enqueue(c);
    if (rc != RAFI_OK) return rc;
    if (counts) {
        uint64_t *tmp = static_cast<uint64_t *>(std::malloc(sizeof(uint64_t) * (c->D + 1)));
        if (!tmp) return RAFI_ERR_OOM;
        hipError_t e = hipMemcpyAsync(tmp, c->offsets, sizeof(uint64_t) * (c->D + 1), hipMemcpyDeviceToHost,
                                      c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e == hipSuccess)
            for (int32_t d = 0; d < c->D; ++d) counts[d] = tmp[d + 1] - tmp[d];
        std::free(tmp);
        RAFI_HIP_CHECK(e);
    }
    rc = round_finish(c, total);
    const int fill = ctx_fill_poison(c, c->n_slots);
    return rc != RAFI_OK ? rc : fill;
}

int rafi_copy_queue(const rafi_ctx *c, void *items_dst, uint64_t *offsets_dst)
{
    if (!c) return RAFI_ERR_ARG;
    if (items_dst && c->n_in)
        RAFI_HIP_CHECK(hipMemcpyAsync(items_dst, c->buf[0], c->n_in * c->S, hipMemcpyDeviceToDevice, c->stream));
    if (offsets_dst)
        RAFI_HIP_CHECK(hipMemcpyAsync(offsets_dst, c->offsets, sizeof(uint64_t) * (c->D + 1),
                                      hipMemcpyDeviceToDevice, c->stream));
    return RAFI_OK;
}

int rafi_set_profiling(rafi_ctx *c, int32_t on)
{
    if (!c) return RAFI_ERR_ARG;
    int rc = prof_resolve(c, true);
    if (rc != RAFI_OK) return rc;
    c->prof_on = on ? 1 : 0;
    if (on) c->prof = rafi_profile{};
    return RAFI_OK;
}

int rafi_get_profile(rafi_ctx *c, rafi_profile *out)
{
    if (!c || !out) return RAFI_ERR_ARG;
    int rc = prof_resolve(c, true);
    if (rc != RAFI_OK) return rc;
    *out = c->prof;
    return RAFI_OK;
}

int rafi_stats(const rafi_ctx *c, rafi_stats_t *out)
{
    if (!c || !out) return RAFI_ERR_ARG;
    *out = c->stats;
    return RAFI_OK;
}

int rafi_split_set_variant(int32_t variant) { return split_set_variant(variant); }

int rafi_multisplit_workspace(uint64_t n, int32_t n_domains, uint32_t item_bytes, uint64_t *bytes)
{
    if (!bytes || !valid_shape(n_domains, item_bytes) || n >= (1ull << 32)) return RAFI_ERR_ARG;
    *bytes = split_plan(n, n_domains, item_bytes).bytes;
    return RAFI_OK;
}

int rafi_multisplit(const void *items, const int32_t *dest, uint64_t n, uint32_t item_bytes, int32_t n_domains,
                    void *out, uint64_t *offsets, uint64_t *summary, void *workspace, uint64_t workspace_bytes,
                    void *hip_stream)
{
    if (!valid_shape(n_domains, item_bytes) || n >= (1ull << 32) || !offsets || !summary) return RAFI_ERR_ARG;
    if (n && (!items || !dest || !out || !workspace)) return RAFI_ERR_ARG;
    // 16-byte alignment for the vector paths (device allocations always have it)
    if ((reinterpret_cast<uintptr_t>(items) | reinterpret_cast<uintptr_t>(out) |
         reinterpret_cast<uintptr_t>(dest) | reinterpret_cast<uintptr_t>(workspace)) & 15)
        return RAFI_ERR_ARG;
    SplitPlan p = split_plan(n, n_domains, item_bytes);
    // a workspace sized while another scatter shape was selected may lack the
    // lockstep plan's chunk prefixes: plan without them
    if (workspace_bytes < p.bytes && p.lock) p = split_plan(n, n_domains, item_bytes, false);
    if (workspace_bytes < p.bytes) return RAFI_ERR_ARG;
    return split_run(p, items, dest, out, offsets, summary, nullptr, 1, workspace,
                     static_cast<hipStream_t>(hip_stream));
}

int rafi_multisplit_noalloc(const void *items, const int32_t *dest, uint64_t n, uint32_t item_bytes,
                            int32_t n_domains, void *out, uint64_t *offsets, uint64_t *summary, void *hip_stream)
{
    if (!valid_shape(n_domains, item_bytes) || n >= (1ull << 32) || !offsets || !summary) return RAFI_ERR_ARG;
    if (n && (!items || !dest || !out)) return RAFI_ERR_ARG;
    if ((reinterpret_cast<uintptr_t>(items) | reinterpret_cast<uintptr_t>(out) |
         reinterpret_cast<uintptr_t>(dest)) & 15)
        return RAFI_ERR_ARG;
    // no lockstep plan: its chunk prefixes grow with n, the scratch does not
    const SplitPlan p = split_plan(n, n_domains, item_bytes, false);
    if (p.bytes > kNoAllocScratchBytes) return RAFI_ERR_TOO_LARGE;
    const hipStream_t s = static_cast<hipStream_t>(hip_stream);
    void *ws = nullptr;
    const int rc = noalloc_scratch(s, &ws);
    if (rc != RAFI_OK) return rc;
    return split_run(p, items, dest, out, offsets, summary, nullptr, 1, ws, s);
}

}  // extern "C"
