/*
 * rafi_device.h -- device side of the forwarding interface (HIP, gfx950).
 *
 * The device interface of Sec. 3.3: a kernel receives a rafi_device_view by
 * value, reads how many items each domain has and the items themselves, and
 * emits every item it handles with a destination domain (or RAFI_DONE).
 *
 * Emission is slot-ordered: the thread that handles input item i (or, in a
 * generator kernel, work unit i) writes output slot i exactly once. This is
 * the paper's first queue design (Sec. 3.2: an item written back to the
 * position it was read from, destination pre-set to -1), which makes the
 * order of items within each destination reproducible from run to run.
 * Emits to a slot outside [0, n_slots) are dropped and counted, as emits
 * beyond the queue capacity are dropped in Sec. 3.3.
 */
#ifndef RAFI_DEVICE_H
#define RAFI_DEVICE_H

#include <hip/hip_runtime.h>

#include "rafi.h"

/* Number of input items of domain d (numIncoming, Sec. 3.3). */
__device__ inline uint64_t rafi_num_incoming(const rafi_device_view &v, int32_t d)
{
    return v.in_offsets[d + 1] - v.in_offsets[d];
}

/* Number of items in the input queue, read on the device (the view's n_in
 * is the host's copy). Domain kernels that the library launches before the
 * host has read the forward step's total use this, with a grid sized for an
 * upper bound; threads at or past it do nothing. */
__device__ inline uint64_t rafi_queue_length(const rafi_device_view &v)
{
    return v.in_offsets[v.n_domains];
}

/* Pointer to input item i of domain d (getIncoming, Sec. 3.3). */
__device__ inline const void *rafi_incoming(const rafi_device_view &v, int32_t d, uint64_t i)
{
    return static_cast<const char *>(v.in_items) + (v.in_offsets[d] + i) * v.item_bytes;
}

/* Emit `item` (item_bytes bytes, 4-byte aligned) into output slot `slot`
 * bound for domain `dest` (emitOutgoing, Sec. 3.3). Sending to one's own
 * domain is valid. */
__device__ inline void rafi_forward(const rafi_device_view &v, uint64_t slot, const void *item,
                                    int32_t dest)
{
    if (slot >= v.n_slots) {
        atomicAdd(v.dropped, 1ull);
        return;
    }
    const uint32_t *src = static_cast<const uint32_t *>(item);
    uint32_t *dst = reinterpret_cast<uint32_t *>(static_cast<char *>(v.out_items) + slot * v.item_bytes);
    for (uint32_t w = 0; w < v.item_bytes / 4; ++w) dst[w] = src[w];
    v.out_dest[slot] = dest;
}

/* Typed emit: one aligned store of T (sizeof(T) must equal item_bytes). */
template <typename T>
__device__ inline void rafi_forward_t(const rafi_device_view &v, uint64_t slot, const T &item,
                                      int32_t dest)
{
    if (slot >= v.n_slots) {
        atomicAdd(v.dropped, 1ull);
        return;
    }
    static_cast<T *>(v.out_items)[slot] = item;
    v.out_dest[slot] = dest;
}

/* Append emit (emitOutgoing with the paper's atomic queue, Sec. 3.2-3.3),
 * for output opened with rafi_open(..., RAFI_SLOTS_APPEND): the item goes to
 * the next free slot. Lanes of a wave that emit together take consecutive
 * slots in lane order with one atomic per wave. May be called any number of
 * times per thread and from divergent code. */
template <typename T>
__device__ inline void rafi_emit_t(const rafi_device_view &v, const T &item, int32_t dest)
{
    const uint64_t active = __ballot(1);
    const int lane = (int)__lane_id();
    const int leader = __ffsll((long long)active) - 1;
    unsigned long long base = 0;
    if (lane == leader) base = atomicAdd(v.append, (unsigned long long)__popcll(active));
    base = __shfl(base, leader);
    rafi_forward_t(v, base + (uint64_t)__popcll(active & ((1ull << lane) - 1ull)), item, dest);
}

/* Untyped append emit (item_bytes bytes, 4-byte aligned). */
__device__ inline void rafi_emit(const rafi_device_view &v, const void *item, int32_t dest)
{
    const uint64_t active = __ballot(1);
    const int lane = (int)__lane_id();
    const int leader = __ffsll((long long)active) - 1;
    unsigned long long base = 0;
    if (lane == leader) base = atomicAdd(v.append, (unsigned long long)__popcll(active));
    base = __shfl(base, leader);
    rafi_forward(v, base + (uint64_t)__popcll(active & ((1ull << lane) - 1ull)), item, dest);
}

/* Mark slot `slot` as leaving the system (destination RAFI_DONE). */
__device__ inline void rafi_done(const rafi_device_view &v, uint64_t slot)
{
    if (slot >= v.n_slots) {
        atomicAdd(v.dropped, 1ull);
        return;
    }
    v.out_dest[slot] = RAFI_DONE;
}

/* Domain and item range of workgroup-sized tile `tile` (0 <= tile < n_tiles):
 * returns the domain; [*begin, *end) are input-queue indices. */
__device__ inline int32_t rafi_tile(const rafi_device_view &v, uint32_t tile, uint64_t *begin,
                                    uint64_t *end)
{
    int32_t lo = 0, hi = v.n_domains; /* find last d with in_tile_offsets[d] <= tile */
    while (hi - lo > 1) {
        int32_t mid = (lo + hi) >> 1;
        if (v.in_tile_offsets[mid] <= tile) lo = mid; else hi = mid;
    }
    uint64_t first = v.in_offsets[lo] + (uint64_t)(tile - v.in_tile_offsets[lo]) * v.tile_items;
    uint64_t last = first + v.tile_items;
    if (last > v.in_offsets[lo + 1]) last = v.in_offsets[lo + 1];
    *begin = first;
    *end = last;
    return lo;
}

/* Launch helper for domain kernels (not part of the paper's interface).
 * The GPU deals workgroups to its 8 XCDs round-robin (workgroup b to XCD
 * b % 8), and each XCD has its own L2. Numbering workgroups with
 * rafi_xcd_block(blockIdx.x, gridDim.x) instead gives each XCD a contiguous
 * range of logical workgroups, so the workgroups resident on one XCD read
 * neighbouring parts of the domain-sorted input queue, and therefore the same
 * few bricks. It is a bijection on [0, nb) for any nb. */
__device__ inline uint32_t rafi_xcd_block(uint32_t b, uint32_t nb)
{
    const uint32_t per = nb / 8u, rem = nb % 8u, x = b % 8u;
    return x * per + (x < rem ? x : rem) + b / 8u;
}

#endif /* RAFI_DEVICE_H */
