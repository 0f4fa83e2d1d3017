// Stable multi-split by destination: the forward step of the library.
//
// What it computes (Sec. 4.2.1-4.2.2 of the paper, collapsed to one device):
// slot i with destination e in [0, D) lands at
//     offset[e] + #{ j < i : dest[j] == e },
// offset[] being the exclusive prefix of the per-destination counts; slots
// with RAFI_DONE leave, slots with any other out-of-range value are dropped;
// both are counted. The paper reaches the same placement with a radix sort of
// (dest << 32 | i) keys, a gather and a begin/end tally; here it is three
// HBM-streaming passes:
//
//   1. hist    per tile of T slots, a destination histogram (LDS atomics),
//              written destination-major: table[e * n_tiles + tile].
//   2. scan    one exclusive scan over the flattened table. Entry
//              (e, tile) then holds the output position of the tile's first
//              item bound for e, and row starts are the offsets.
//   3. scatter per tile, each wavefront owns a contiguous quarter; per-wave
//              counts give each wave its base per destination, and inside a
//              wave the rank of a lane among same-destination lanes comes from
//              a ballot match over the destination bits. Items are copied as
//              4-byte words (16-byte vectors when the size allows).
#include "internal.h"
#include "split_device.h"

#include <algorithm>

namespace rafi {
namespace {

constexpr int kScanThreads = 256;
constexpr int kScanPer = 16;                       // elements per thread
constexpr int kScanChunk = kScanThreads * kScanPer;  // 4096
constexpr int kPartThreads = 1024;
constexpr int kPartMax = kPartThreads * kScanPer;  // 16384 partial sums
// Up to this many scan chunks, each chunk of the apply pass sums the earlier
// chunks' totals itself (at most 2 MiB read over the whole launch), which
// saves the launch that scans the partial sums.
constexpr uint32_t kDirectMaxBlocks = 1024;

using dev::block_excl_scan;
using dev::bucket_of;
using dev::load_nt4;
using dev::match_peers;

// ---------------------------------------------------------------- pass 1 ---
// Destination histogram of tile blockIdx.x into column blockIdx.x of table.
__device__ inline void hist_tile(const int32_t *__restrict__ dest, uint64_t n, int32_t D, uint32_t T,
                                 uint32_t n_tiles, uint32_t *__restrict__ table, uint32_t *h)
{
    const uint32_t rows = (uint32_t)D + 2u;
    for (uint32_t e = threadIdx.x; e < rows; e += blockDim.x) h[e] = 0;
    __syncthreads();
    const uint64_t start = (uint64_t)blockIdx.x * T;
    const uint64_t end = min(start + T, n);
    // T is a multiple of 1024 and dest is 16-byte aligned: whole int4 groups,
    // loaded kU at a time before the LDS atomics so the loads overlap.
    constexpr int kU = 8;
    const uint64_t vend = start + ((end - start) & ~(uint64_t)3);
    const uint64_t stride = 4ull * blockDim.x;
    uint64_t i = start + 4ull * threadIdx.x;
    for (; i + (kU - 1) * stride < vend; i += kU * stride) {
        uint4 d4[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) d4[u] = load_nt4(dest + i + u * stride);
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            atomicAdd(&h[bucket_of((int32_t)d4[u].x, D)], 1u);
            atomicAdd(&h[bucket_of((int32_t)d4[u].y, D)], 1u);
            atomicAdd(&h[bucket_of((int32_t)d4[u].z, D)], 1u);
            atomicAdd(&h[bucket_of((int32_t)d4[u].w, D)], 1u);
        }
    }
    for (; i < vend; i += stride) {
        int4 d4 = *reinterpret_cast<const int4 *>(dest + i);
        atomicAdd(&h[bucket_of(d4.x, D)], 1u);
        atomicAdd(&h[bucket_of(d4.y, D)], 1u);
        atomicAdd(&h[bucket_of(d4.z, D)], 1u);
        atomicAdd(&h[bucket_of(d4.w, D)], 1u);
    }
    for (uint64_t j = vend + threadIdx.x; j < end; j += blockDim.x) atomicAdd(&h[bucket_of(dest[j], D)], 1u);
    __syncthreads();
    for (uint32_t e = threadIdx.x; e < rows; e += blockDim.x)
        table[(uint64_t)e * n_tiles + blockIdx.x] = h[e];
}

__global__ void __launch_bounds__(256)
hist_kernel(const int32_t *__restrict__ dest, uint64_t n, int32_t D, uint32_t T, uint32_t n_tiles,
            uint32_t *__restrict__ table)
{
    extern __shared__ uint32_t h[];  // D + 2
    hist_tile(dest, n, D, T, n_tiles, table, h);
}

// Lockstep plans: tiles of kLockTile chunks of kLockChunk slots. Besides the
// tile's column of the table, pre[c * D + e] = items of chunk c's tile bound
// for e in the chunks before c (at most (kLockTile - 1) * kLockChunk, which
// fits 16 bits).
constexpr uint32_t kLockChunk = 2048;  // slots per chunk: 8 waves x 4 rounds x 64 lanes
constexpr uint32_t kLockTile = 32;     // chunks per tile: one per CU of an XCD
constexpr uint32_t kLockXcds = 8;
static_assert((kLockTile - 1) * kLockChunk < 65536, "chunk prefixes are 16-bit");

// s_waitcnt immediate for lgkmcnt(0) alone (vmcnt and expcnt at their
// maxima, i.e. not waited on).
constexpr int kWaitLds = 0xc07f;

__global__ void __launch_bounds__(256)
hist_lock_kernel(const int32_t *__restrict__ dest, uint64_t n, int32_t D, uint32_t n_tiles, uint32_t n_chunks,
                 uint32_t *__restrict__ table, uint16_t *__restrict__ pre)
{
    extern __shared__ uint32_t h[];  // D + 2
    const uint32_t rows = (uint32_t)D + 2u;
    for (uint32_t e = threadIdx.x; e < rows; e += blockDim.x) h[e] = 0;
    __syncthreads();
    const uint32_t c_first = blockIdx.x * kLockTile;
    const uint32_t c_end = min(c_first + kLockTile, n_chunks);
    static_assert(kLockChunk == 2 * 4 * 256, "two int4 groups per thread per chunk");
    for (uint32_t c = c_first; c < c_end; ++c) {
        const uint64_t s0 = (uint64_t)c * kLockChunk;
        const bool full = s0 + kLockChunk <= n;
        // dest is 16-byte aligned and chunks start at multiples of 2048
        uint4 a = make_uint4(0, 0, 0, 0), b = make_uint4(0, 0, 0, 0);
        if (full) {
            a = load_nt4(dest + s0 + 4 * threadIdx.x);
            b = load_nt4(dest + s0 + 1024 + 4 * threadIdx.x);
        }
        for (uint32_t e = threadIdx.x; e < (uint32_t)D; e += blockDim.x)
            pre[(uint64_t)c * (uint32_t)D + e] = (uint16_t)h[e];
        __syncthreads();  // every count read before it changes
        if (full) {
            atomicAdd(&h[bucket_of((int32_t)a.x, D)], 1u);
            atomicAdd(&h[bucket_of((int32_t)a.y, D)], 1u);
            atomicAdd(&h[bucket_of((int32_t)a.z, D)], 1u);
            atomicAdd(&h[bucket_of((int32_t)a.w, D)], 1u);
            atomicAdd(&h[bucket_of((int32_t)b.x, D)], 1u);
            atomicAdd(&h[bucket_of((int32_t)b.y, D)], 1u);
            atomicAdd(&h[bucket_of((int32_t)b.z, D)], 1u);
            atomicAdd(&h[bucket_of((int32_t)b.w, D)], 1u);
        } else {
            for (uint64_t i = s0 + threadIdx.x; i < n; i += blockDim.x) atomicAdd(&h[bucket_of(dest[i], D)], 1u);
        }
        // Every wave's LDS atomics complete before the barrier: LDS requests
        // of different waves can complete out of order, and the compiler
        // has been seen to drop this wait when the next read of the counts
        // is reached through the loop's back edge.
        __builtin_amdgcn_s_waitcnt(kWaitLds);
        __syncthreads();
    }
    for (uint32_t e = threadIdx.x; e < rows; e += blockDim.x)
        table[(uint64_t)e * n_tiles + blockIdx.x] = h[e];
}

// ---------------------------------------------------------------- pass 2 ---
__device__ inline void load16(const uint32_t *__restrict__ a, uint64_t M, uint64_t base, uint32_t v[kScanPer])
{
    if (base + kScanPer <= M) {
        const uint4 *p = reinterpret_cast<const uint4 *>(a + base);
#pragma unroll
        for (int k = 0; k < kScanPer / 4; ++k) {
            uint4 q = p[k];
            v[4 * k] = q.x; v[4 * k + 1] = q.y; v[4 * k + 2] = q.z; v[4 * k + 3] = q.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) v[k] = (base + k < M) ? a[base + k] : 0u;
    }
}

// a[base + k] = run + v[0] + ... + v[k - 1] for the thread's 16 entries
__device__ inline void store16_excl(uint32_t *__restrict__ a, uint64_t M, uint64_t base, const uint32_t v[kScanPer],
                                    uint32_t run)
{
    if (base + kScanPer <= M) {
        uint4 *p = reinterpret_cast<uint4 *>(a + base);
#pragma unroll
        for (int k = 0; k < kScanPer / 4; ++k) {
            uint4 q;
            q.x = run; run += v[4 * k];
            q.y = run; run += v[4 * k + 1];
            q.z = run; run += v[4 * k + 2];
            q.w = run; run += v[4 * k + 3];
            p[k] = q;
        }
    } else {
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) {
            if (base + k < M) a[base + k] = run;
            run += v[k];
        }
    }
}

__global__ void __launch_bounds__(kScanThreads)
scan_reduce_kernel(const uint32_t *__restrict__ a, uint64_t M, uint32_t *__restrict__ part)
{
    __shared__ uint32_t lds[kScanThreads / 64 + 1];
    uint32_t v[kScanPer];
    load16(a, M, (uint64_t)blockIdx.x * kScanChunk + (uint64_t)threadIdx.x * kScanPer, v);
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) s += v[k];
    uint32_t tot;
    block_excl_scan<kScanThreads>(s, lds, &tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(kPartThreads)
scan_partials_kernel(uint32_t *__restrict__ part, uint32_t nb)
{
    __shared__ uint32_t lds[kPartThreads / 64 + 1];
    uint32_t v[kScanPer];
    const uint64_t base = (uint64_t)threadIdx.x * kScanPer;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) v[k] = (base + k < nb) ? part[base + k] : 0u;
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) s += v[k];
    uint32_t tot;
    uint32_t run = block_excl_scan<kPartThreads>(s, lds, &tot);
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        if (base + k < nb) part[base + k] = run;
        run += v[k];
    }
}

__global__ void __launch_bounds__(kScanThreads)
scan_apply_kernel(uint32_t *__restrict__ a, uint64_t M, const uint32_t *__restrict__ part)
{
    __shared__ uint32_t lds[kScanThreads / 64 + 1];
    uint32_t v[kScanPer];
    const uint64_t base = (uint64_t)blockIdx.x * kScanChunk + (uint64_t)threadIdx.x * kScanPer;
    load16(a, M, base, v);
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) s += v[k];
    uint32_t tot;
    uint32_t run = block_excl_scan<kScanThreads>(s, lds, &tot) + part[blockIdx.x];
    store16_excl(a, M, base, v, run);
}

// scan_apply_kernel with the chunk's offset summed here from the chunks'
// totals (part as scan_reduce_kernel left it) instead of by a separate scan.
__global__ void __launch_bounds__(kScanThreads)
scan_apply_direct_kernel(uint32_t *__restrict__ a, uint64_t M, const uint32_t *__restrict__ part)
{
    __shared__ uint32_t lds[kScanThreads / 64 + 1];
    uint32_t before = 0;
    for (uint32_t j = threadIdx.x; j < blockIdx.x; j += kScanThreads) before += part[j];
    uint32_t off;
    (void)block_excl_scan<kScanThreads>(before, lds, &off);
    uint32_t v[kScanPer];
    const uint64_t base = (uint64_t)blockIdx.x * kScanChunk + (uint64_t)threadIdx.x * kScanPer;
    load16(a, M, base, v);
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) s += v[k];
    uint32_t tot;
    uint32_t run = block_excl_scan<kScanThreads>(s, lds, &tot) + off;
    store16_excl(a, M, base, v, run);
}

// Offsets, summary and the tile table for domain-pure launches, from the
// scanned table; with `dropped`, its count goes to summary[4] and is reset
// (the domain kernels that add to it have completed).
template <int NT>
__device__ inline void finalize_body(const uint32_t *__restrict__ table, uint32_t n_tiles, int32_t D, uint64_t n,
                                     uint64_t *__restrict__ offsets, uint64_t *__restrict__ summary,
                                     uint32_t *__restrict__ tile_offsets, uint32_t tile_items,
                                     unsigned long long *__restrict__ dropped, uint32_t *lds)
{
    auto row_start = [&](int32_t e) -> uint64_t {
        return n_tiles ? (uint64_t)table[(uint64_t)e * n_tiles] : 0ull;
    };
    for (int32_t e = threadIdx.x; e <= D; e += NT) offsets[e] = row_start(e);
    const uint64_t total = row_start(D);
    const uint64_t done_end = n_tiles ? row_start(D + 1) : 0ull;
    // per-domain tile counts, scanned (each thread owns a contiguous run)
    const int32_t per = (D + NT - 1) / NT;
    const int32_t e0 = threadIdx.x * per;
    uint32_t local = 0;
    for (int32_t e = e0; e < min(e0 + per, D); ++e) {
        uint64_t c = row_start(e + 1) - row_start(e);
        local += (uint32_t)((c + tile_items - 1) / tile_items);
    }
    uint32_t tot;
    uint32_t run = block_excl_scan<NT>(local, lds, &tot);
    if (tile_offsets) {
        for (int32_t e = e0; e < min(e0 + per, D); ++e) {
            tile_offsets[e] = run;
            uint64_t c = row_start(e + 1) - row_start(e);
            run += (uint32_t)((c + tile_items - 1) / tile_items);
        }
        if (threadIdx.x == 0) tile_offsets[D] = tot;
    }
    if (threadIdx.x == 0) {
        summary[0] = total;
        summary[1] = done_end - total;
        summary[2] = n - done_end;
        summary[3] = tot;
        if (dropped) {
            summary[4] = *dropped;
            *dropped = 0;
        }
    }
}

__global__ void __launch_bounds__(1024)
finalize_kernel(const uint32_t *__restrict__ table, uint32_t n_tiles, int32_t D, uint64_t n,
                uint64_t *__restrict__ offsets, uint64_t *__restrict__ summary,
                uint32_t *__restrict__ tile_offsets, uint32_t tile_items, unsigned long long *__restrict__ dropped)
{
    __shared__ uint32_t lds[1024 / 64 + 1];
    finalize_body<1024>(table, n_tiles, D, n, offsets, summary, tile_offsets, tile_items, dropped, lds);
}

// True in exactly one workgroup of the launch: the last to get here. Each
// workgroup's global writes before the call are visible to that one (device
// fences around a count of finished workgroups). The counter is zero between
// launches: the last workgroup resets it.
__device__ inline bool last_workgroup(uint32_t *counter, uint32_t n_groups)
{
    __shared__ uint32_t is_last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) is_last = atomicAdd(counter, 1u) == n_groups - 1 ? 1u : 0u;
    __syncthreads();
    if (!is_last) return false;
    __threadfence();
    if (threadIdx.x == 0) atomicExch(counter, 0u);
    return true;
}

// Exclusive scan of a[0, m) in place by one workgroup of NT threads, each
// owning a contiguous run (m small).
template <int NT>
__device__ inline void block_scan_inplace(uint32_t *a, uint64_t m, uint32_t *lds)
{
    const uint64_t per = (m + NT - 1) / NT;
    const uint64_t b0 = min((uint64_t)threadIdx.x * per, m), b1 = min(b0 + per, m);
    uint32_t sum = 0;
    for (uint64_t k = b0; k < b1; ++k) sum += a[k];
    uint32_t tot;
    uint32_t run = block_excl_scan<NT>(sum, lds, &tot);
    for (uint64_t k = b0; k < b1; ++k) {
        const uint32_t v = a[k];
        a[k] = run;
        run += v;
    }
    __syncthreads();
}

// ----------------------------------------------------- passes 1 + 2 fused ---
// For a small count table (M entries): every workgroup writes its tile's
// histogram, and the last one to finish (a device-scope fence, then an atomic
// count of finished tiles) scans the whole table in place and finalizes. No
// workgroup waits for another. The counter is zero between launches: the last
// workgroup resets it.
constexpr uint64_t kFusedMaxM = 4096;     // at most 16 entries per thread in the last workgroup's scan
constexpr uint32_t kFusedMaxTiles = 512;  // workgroups, each with its own fence

__global__ void __launch_bounds__(256)
hist_scan_kernel(const int32_t *__restrict__ dest, uint64_t n, int32_t D, uint32_t T, uint32_t n_tiles,
                 uint32_t *__restrict__ table, uint64_t M, uint32_t *__restrict__ counter,
                 uint64_t *__restrict__ offsets, uint64_t *__restrict__ summary,
                 uint32_t *__restrict__ tile_offsets, uint32_t tile_items, unsigned long long *__restrict__ dropped)
{
    extern __shared__ uint32_t h[];  // D + 2
    __shared__ uint32_t lds[256 / 64 + 1];
    hist_tile(dest, n, D, T, n_tiles, table, h);
    if (!last_workgroup(counter, n_tiles)) return;
    block_scan_inplace<256>(table, M, lds);
    finalize_body<256>(table, n_tiles, D, n, offsets, summary, tile_offsets, tile_items, dropped, lds);
}

// ---------------------------------------------------------------- pass 3 ---
template <int NW>
__device__ inline void copy_item(const uint32_t *__restrict__ src, uint32_t *__restrict__ dst)
{
    if constexpr (NW % 4 == 0) {
        const uint4 *s = reinterpret_cast<const uint4 *>(src);
        uint4 *d = reinterpret_cast<uint4 *>(dst);
#pragma unroll
        for (int k = 0; k < NW / 4; ++k) d[k] = s[k];
    } else if constexpr (NW % 2 == 0) {
        const uint2 *s = reinterpret_cast<const uint2 *>(src);
        uint2 *d = reinterpret_cast<uint2 *>(dst);
#pragma unroll
        for (int k = 0; k < NW / 2; ++k) d[k] = s[k];
    } else {
#pragma unroll
        for (int k = 0; k < NW; ++k) dst[k] = src[k];
    }
}

template <int NW>
__global__ void __launch_bounds__(256)
scatter_kernel(const uint32_t *__restrict__ items, const int32_t *__restrict__ dest, uint64_t n,
               int32_t D, int nbits, uint32_t T, uint32_t n_tiles, const uint32_t *__restrict__ table,
               uint32_t *__restrict__ out, uint32_t nw_runtime)
{
    extern __shared__ uint32_t cnt[];  // [4][D]
    const uint32_t nw = NW > 0 ? (uint32_t)NW : nw_runtime;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const uint64_t start = (uint64_t)blockIdx.x * T;
    const uint64_t end = min(start + T, n);
    const uint64_t q = T / 4;
    const uint64_t wstart = min(start + w * q, end), wend = min(wstart + q, end);
    uint32_t *mycnt = cnt + (uint64_t)w * D;

    for (uint32_t e = tid; e < 4u * (uint32_t)D; e += 256) cnt[e] = 0;
    __syncthreads();
    for (uint64_t i = wstart + lane; i < wend; i += 64) {
        const int32_t d = dest[i];
        if (d >= 0 && d < D) atomicAdd(&mycnt[d], 1u);
    }
    __syncthreads();
    for (int32_t e = tid; e < D; e += 256) {
        uint32_t run = table[(uint64_t)e * n_tiles + blockIdx.x];
#pragma unroll
        for (int ww = 0; ww < 4; ++ww) {
            const uint32_t c = cnt[ww * D + e];
            cnt[ww * D + e] = run;
            run += c;
        }
    }
    __syncthreads();
    const uint64_t lt = (1ull << lane) - 1ull;
    for (uint64_t b = wstart; b < wend; b += 64) {
        const uint64_t i = b + lane;
        const bool in = i < wend;
        const int32_t d = in ? dest[i] : RAFI_DONE;
        const bool ok = in && d >= 0 && d < D;
        const uint64_t peers = match_peers((uint32_t)d, ok, nbits);
        uint32_t pos = 0;
        if (ok) pos = mycnt[d] + (uint32_t)__popcll(peers & lt);
        __builtin_amdgcn_wave_barrier();
        if (ok && (peers & lt) == 0ull) mycnt[d] = pos + (uint32_t)__popcll(peers);
        // positions of kept items are < n by construction; the guard keeps a
        // corrupted table from ever writing outside the output buffer
        if (ok && pos < n) {
            const uint32_t *src = items + i * nw;
            uint32_t *dst = out + (uint64_t)pos * nw;
            if constexpr (NW > 0) {
                copy_item<NW>(src, dst);
            } else {
                for (uint32_t k = 0; k < nw; ++k) dst[k] = src[k];
            }
        }
    }
}

// ------------------------------------------------------- pass 3, staged ---
template <int NW, int R, int W, int OCC, bool DB>
__global__ void __launch_bounds__(64 * W, OCC)
scatter_staged_kernel(const uint32_t *__restrict__ items, const int32_t *__restrict__ dest, uint64_t n,
                      int32_t D, int nbits, uint32_t T, uint32_t n_tiles, const uint32_t *__restrict__ table,
                      uint32_t *__restrict__ out)
{
    extern __shared__ __align__(16) uint32_t lds[];
    const uint64_t tstart = (uint64_t)blockIdx.x * T;
    const uint64_t tend = min(tstart + T, n);
    const uint32_t tile = blockIdx.x;
    dev::staged_scatter_tile<NW, R, W, DB>(
        items, dest, tstart, tend, D, 0, nbits,
        [&](int32_t e) { return table[(uint64_t)e * n_tiles + tile]; }, out, n, lds);
}

// One (rounds, waves, workgroups per CU) shape of the staged scatter; it is
// launched only if its LDS fits that many workgroups per CU.
template <int NW, int R, int W, int BPC, bool DB = false>
bool try_staged(const SplitPlan &p, const uint32_t *items, const int32_t *dest, const uint32_t *table,
                uint32_t *out, hipStream_t s)
{
    const size_t lds = dev::staged_lds_bytes<NW, R, W>(p.D) + 64;
    if (p.D > dev::kStagedMaxD || lds * BPC > dev::kStagedLdsPerCu) return false;
    int nbits = 1;
    while ((1 << nbits) < p.D) ++nbits;
    constexpr int OCC = (W * BPC + 3) / 4;  // waves per SIMD
    hipLaunchKernelGGL((scatter_staged_kernel<NW, R, W, OCC, DB>), dim3(p.n_tiles), dim3(64 * W), lds, s, items, dest,
                       p.n, p.D, nbits, p.tile, p.n_tiles, table, out);
    return true;
}

template <int NW, int R, int W, int OCC>
__global__ void __launch_bounds__(64 * W, OCC)
scatter_gather_kernel(const uint32_t *__restrict__ items, const int32_t *__restrict__ dest, uint64_t n,
                      int32_t D, int nbits, uint32_t T, uint32_t n_tiles, const uint32_t *__restrict__ table,
                      uint32_t *__restrict__ out)
{
    extern __shared__ __align__(16) uint32_t lds[];
    const uint64_t tstart = (uint64_t)blockIdx.x * T;
    const uint64_t tend = min(tstart + T, n);
    const uint32_t tile = blockIdx.x;
    dev::gather_scatter_tile<NW, R, W>(
        items, dest, tstart, tend, D, 0, nbits,
        [&](int32_t e) { return table[(uint64_t)e * n_tiles + tile]; }, out, n, lds);
}

template <int NW, int R, int W, int BPC>
bool try_gather(const SplitPlan &p, const uint32_t *items, const int32_t *dest, const uint32_t *table,
                uint32_t *out, hipStream_t s)
{
    const size_t lds = dev::gather_lds_bytes<R, W>(p.D) + 64;
    if (p.D > dev::kStagedMaxD || lds * BPC > dev::kStagedLdsPerCu) return false;
    int nbits = 1;
    while ((1 << nbits) < p.D) ++nbits;
    constexpr int OCC = (W * BPC + 3) / 4;
    hipLaunchKernelGGL((scatter_gather_kernel<NW, R, W, OCC>), dim3(p.n_tiles), dim3(64 * W), lds, s, items, dest,
                       p.n, p.D, nbits, p.tile, p.n_tiles, table, out);
    return true;
}

template <int NW, int R, int W, bool DB>
__global__ void __launch_bounds__(64 * W, (W + 3) / 4)
scatter_wide_kernel(const uint32_t *__restrict__ items, const int32_t *__restrict__ dest, uint64_t n,
                    int32_t D, int nbits, uint32_t T, uint32_t n_tiles, const uint32_t *__restrict__ table,
                    uint32_t *__restrict__ out, uint32_t *__restrict__ dummy)
{
    extern __shared__ __align__(16) uint32_t lds[];
    const uint64_t tstart = (uint64_t)blockIdx.x * T;
    const uint64_t tend = min(tstart + T, n);
    const uint32_t tile = blockIdx.x;
    dev::wide_scatter_tile<NW, R, W, DB>(
        items, dest, tstart, tend, D, 0, nbits,
        [&](int32_t e) { return table[(uint64_t)e * n_tiles + tile]; }, out, n, dummy, lds);
}

// The wide shape: one workgroup per CU with a chunk as large as LDS allows.
template <int NW, int R, int W, bool DB>
bool try_wide(const SplitPlan &p, const uint32_t *items, const int32_t *dest, const uint32_t *table,
              uint32_t *out, uint32_t *dummy, hipStream_t s)
{
    const size_t lds = dev::wide_lds_bytes_c<NW, R, W>(p.D) + 64;
    if (p.D > dev::kStagedMaxD || lds > dev::kStagedLdsPerCu) return false;
    int nbits = 1;
    while ((1 << nbits) < p.D) ++nbits;
    hipLaunchKernelGGL((scatter_wide_kernel<NW, R, W, DB>), dim3(p.n_tiles), dim3(64 * W), lds, s, items, dest,
                       p.n, p.D, nbits, p.tile, p.n_tiles, table, out, dummy);
    return true;
}

// The line-aligned shape: one workgroup per CU, each over a group of
// consecutive histogram tiles, so that only the two ends of a destination's
// run per group are partial lines.
template <int NW, int R, int W, int PMAX, bool DB>
__global__ void __launch_bounds__(64 * W)
scatter_line_kernel(const uint32_t *__restrict__ items, const int32_t *__restrict__ dest, uint64_t n,
                    int32_t D, int nbits, uint32_t T, uint32_t n_tiles, uint32_t group,
                    const uint32_t *__restrict__ table, uint32_t *__restrict__ out)
{
    extern __shared__ __align__(16) uint32_t lds[];
    const uint32_t tile = blockIdx.x * group;
    const uint64_t tstart = (uint64_t)tile * T;
    const uint64_t tend = min(tstart + (uint64_t)group * T, n);
    dev::line_scatter_tile<NW, R, W, PMAX, DB>(
        items, dest, tstart, tend, D, nbits,
        [&](int32_t e) { return table[(uint64_t)e * n_tiles + tile]; }, out, n, lds);
}

// The wide shape with raw staging (item sizes that are not a multiple of 16
// bytes): one workgroup per CU, the chunk's bytes in LDS in load order.
template <int NW, int R, int W>
__global__ void __launch_bounds__(64 * W, (W + 3) / 4)
scatter_wide_raw_kernel(const uint32_t *__restrict__ items, const int32_t *__restrict__ dest, uint64_t n,
                        uint64_t words, int32_t D, int nbits, uint32_t T, uint32_t n_tiles,
                        const uint32_t *__restrict__ table, uint32_t *__restrict__ out, uint32_t *__restrict__ dummy)
{
    extern __shared__ __align__(16) uint32_t lds[];
    const uint64_t tstart = (uint64_t)blockIdx.x * T;
    const uint64_t tend = min(tstart + T, n);
    const uint32_t tile = blockIdx.x;
    dev::wide_raw_scatter_tile<NW, R, W>(
        items, dest, tstart, tend, words, D, nbits,
        [&](int32_t e) { return table[(uint64_t)e * n_tiles + tile]; }, out, n, dummy, lds);
}

template <int NW, int R, int W>
bool try_wide_raw(const SplitPlan &p, const uint32_t *items, const int32_t *dest, const uint32_t *table,
                  uint32_t *out, uint32_t *dummy, hipStream_t s)
{
    const size_t lds = dev::wide_raw_lds_bytes_c<NW, R, W>(p.D) + 64;
    if (p.D > dev::kStagedMaxD || lds > dev::kStagedLdsPerCu) return false;
    // readable words: the array, rounded up to whole 16-byte pieces where
    // the allocation is padded for that
    uint64_t words = p.n * (uint64_t)NW;
    if (p.padded) words = (words + 3) & ~3ull;
    if (words % 4 != 0 || words < 4) return false;
    int nbits = 1;
    while ((1 << nbits) < p.D) ++nbits;
    hipLaunchKernelGGL((scatter_wide_raw_kernel<NW, R, W>), dim3(p.n_tiles), dim3(64 * W), lds, s, items, dest, p.n,
                       words, p.D, nbits, p.tile, p.n_tiles, table, out, dummy);
    return true;
}

// The raw shape over a lockstep schedule: kLockXcds * kLockTile persistent
// workgroups, one per CU. The dispatcher deals workgroups to the XCDs in
// turn, so workgroup b runs on XCD b % 8 as its (b / 8)-th. At step j the 32
// workgroups of XCD x take the 32 chunks of tile 8 j + x: the line a
// destination's runs in two neighbouring chunks share is then written twice
// into one L2 within the same step and leaves it whole, where chunks far
// apart in time would each send a partial line to HBM. Every workgroup loads
// its next chunk (and that chunk's run bases) while it writes the current one.
template <int NW, int R, int W>
__global__ void __launch_bounds__(64 * W, (W + 3) / 4)
scatter_lock_raw_kernel(const uint32_t *__restrict__ items, const int32_t *__restrict__ dest, uint64_t n,
                        uint64_t words, int32_t D, int nbits, uint32_t n_tiles, uint32_t n_chunks,
                        const uint32_t *__restrict__ table, const uint16_t *__restrict__ pre,
                        uint32_t *__restrict__ out, uint32_t *__restrict__ dummy)
{
    static_assert(W * 64 * R == (int)kLockChunk, "a chunk of the schedule is one chunk of the kernel");
    extern __shared__ __align__(16) uint32_t lds[];
    const uint32_t x = blockIdx.x % kLockXcds, k = blockIdx.x / kLockXcds;
    const dev::LockChunks<kLockChunk, kLockTile> sched{n, x * kLockTile + k, kLockXcds * kLockTile, n_chunks,
                                                       n_tiles, D, table, pre};
    dev::wide_raw_scatter<NW, R, W>(items, dest, words, D, nbits, sched, out, n, dummy, lds);
}

template <int NW>
bool try_lock_raw(const SplitPlan &p, const uint32_t *items, const int32_t *dest, const uint32_t *table,
                  const uint16_t *pre, uint32_t *out, uint32_t *dummy, hipStream_t s)
{
    constexpr int R = 4, W = 8;
    const size_t lds = dev::wide_raw_lds_bytes_c<NW, R, W>(p.D) + 64;
    if (p.lock != kLockTile || p.D > dev::kStagedMaxD || lds > dev::kStagedLdsPerCu) return false;
    uint64_t words = p.n * (uint64_t)NW;
    if (p.padded) words = (words + 3) & ~3ull;
    if (words % 4 != 0 || words < 4) return false;
    int nbits = 1;
    while ((1 << nbits) < p.D) ++nbits;
    hipLaunchKernelGGL((scatter_lock_raw_kernel<NW, R, W>), dim3(kLockXcds * kLockTile), dim3(64 * W), lds, s,
                       items, dest, p.n, words, p.D, nbits, p.n_tiles, p.n_chunks, table, pre, out, dummy);
    return true;
}

int g_cus = 0;

int cu_count()
{
    if (g_cus == 0) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v < 1)
            v = 256;
        g_cus = v;
    }
    return g_cus;
}

// Whether one workgroup per CU covers at least two histogram tiles and
// 16384 slots: then the partial lines at the ends of each workgroup's runs
// are few and the line-aligned shape pays.
bool line_spans_tiles(const SplitPlan &p)
{
    const uint32_t cus = (uint32_t)cu_count();
    const uint64_t group = (p.n_tiles + cus - 1) / cus;
    return p.n_tiles >= 2u * cus && group * p.tile >= 16384;
}

template <int NW, int R, int W, int PMAX, bool DB>
bool try_line(const SplitPlan &p, const uint32_t *items, const int32_t *dest, const uint32_t *table,
              uint32_t *out, hipStream_t s)
{
    const size_t lds = dev::line_lds_bytes_c<NW, R, W, PMAX>(p.D) + 64;
    if (p.D > dev::kStagedMaxD || lds > dev::kStagedLdsPerCu) return false;
    if ((reinterpret_cast<uintptr_t>(out) & 127) != 0) return false;
    if (p.n * (uint64_t)p.S > 0xfffffff0ull) return false;  // 32-bit buffer offsets
    const uint32_t cus = (uint32_t)cu_count();
    const uint32_t group = (p.n_tiles + cus - 1) / cus;
    const uint32_t grid = (p.n_tiles + group - 1) / group;
    int nbits = 1;
    while ((1 << nbits) < p.D) ++nbits;
    hipLaunchKernelGGL((scatter_line_kernel<NW, R, W, PMAX, DB>), dim3(grid), dim3(64 * W), lds, s, items, dest,
                       p.n, p.D, nbits, p.tile, p.n_tiles, group, table, out);
    return true;
}

// Process-wide choice among the scatter shapes (0 = automatic).
int g_split_variant = 0;

template <int NW>
bool launch_staged(const SplitPlan &p, const uint32_t *items, const int32_t *dest, const uint32_t *table,
                   const uint16_t *pre, uint32_t *out, uint32_t *dummy, hipStream_t s)
{
    int v = g_split_variant;
    if constexpr (NW >= 11) {
        // automatic: items of 44 bytes and more, few destinations and at most
        // 64 MiB: the plain per-thread scatter (each wave's run of a
        // destination is already long; the staged shapes' ranking costs
        // more than it saves there, 5-15% at 1M slots)
        if (v == 0 && p.D <= 128 && p.n * (uint64_t)p.S <= (1ull << 26) && !p.lock) return false;
    }
    if constexpr (NW % 4 != 0 && NW >= 3 && NW <= 15) {
        // large splits: the lockstep schedule (its plan has the chunk prefixes)
        if ((v == 0 || v == 17) && p.lock && try_lock_raw<NW>(p, items, dest, table, pre, out, dummy, s))
            return true;
    }
    if (v == 17) v = 0;  // no lockstep plan for this split: automatic
    if constexpr (NW % 4 != 0 && NW >= 3 && NW <= 15) {
        // item sizes that are not a multiple of 16 bytes: raw staging, one
        // workgroup per CU (automatic when a tile fills a 2048-slot chunk)
        if ((v == 16 || (v == 0 && p.tile >= 8 * 64 * 4)) &&
            try_wide_raw<NW, 4, 8>(p, items, dest, table, out, dummy, s))
            return true;
    }
    if (v == 16) v = 0;  // shape 16 does not take this item size: automatic
    if (v >= 14) {  // line-aligned writes, one workgroup per CU over a group of tiles
        if constexpr (NW == 8) {
            if (v == 14 && try_line<8, 4, 8, 1792, false>(p, items, dest, table, out, s)) return true;
            if (v == 15 && try_line<8, 4, 8, 1792, true>(p, items, dest, table, out, s)) return true;
        } else if constexpr (NW == 4) {
            if (v == 14 && try_line<4, 6, 8, 3840, false>(p, items, dest, table, out, s)) return true;
            if (v == 15 && try_line<4, 6, 8, 3840, true>(p, items, dest, table, out, s)) return true;
        }
        v = 0;  // item size or output alignment the line shapes do not take
    }
    if (v >= 12) {  // one workgroup per CU, 4096-slot (32-byte) or 6144-slot (16-byte) chunks
        if constexpr (NW == 8) {
            if (v == 12) return try_wide<8, 8, 8, false>(p, items, dest, table, out, dummy, s);
            if (v == 13) return try_wide<8, 8, 8, true>(p, items, dest, table, out, dummy, s);
        } else if constexpr (NW == 4) {
            if (v == 12) return try_wide<4, 12, 8, false>(p, items, dest, table, out, dummy, s);
            if (v == 13) return try_wide<4, 12, 8, true>(p, items, dest, table, out, dummy, s);
        }
        return false;
    }
    if (v == 0) {
        // automatic: few destinations and at most 256 MiB of items (every
        // context round of the workloads here): 1024-slot chunks give each
        // destination a run of about 1024 / D items per chunk, long enough
        // that the small staged shapes write whole lines without the
        // line-aligned shape's carry (16-byte items: shape 4, 32-byte items:
        // shape 2, 25-40% faster than the others there); else line-aligned
        // writes when each workgroup spans several tiles, else the wide shape
        // when a tile fills at least one of its chunks
        if (p.D <= 128 && p.n * (uint64_t)p.S <= (1ull << 28)) {
            if constexpr (NW == 8) {
                if (try_staged<8, 4, 4, 3>(p, items, dest, table, out, s)) return true;
            } else if constexpr (NW == 4) {
                if (try_staged<4, 4, 4, 4>(p, items, dest, table, out, s)) return true;
            }
        }
        if (line_spans_tiles(p)) {
            if constexpr (NW == 8) {
                if (try_line<8, 4, 8, 1792, false>(p, items, dest, table, out, s)) return true;
            } else if constexpr (NW == 4) {
                if (try_line<4, 6, 8, 3840, false>(p, items, dest, table, out, s)) return true;
            }
        }
        if constexpr (NW == 8) {
            if (p.tile >= 8 * 8 * 64 && try_wide<8, 8, 8, false>(p, items, dest, table, out, dummy, s)) return true;
        } else if constexpr (NW == 4) {
            if (p.tile >= 8 * 12 * 64 && try_wide<4, 12, 8, false>(p, items, dest, table, out, dummy, s)) return true;
        }
    }
    if (v >= 8) {  // shapes 1-4 with double-buffered chunk loads
        if constexpr (NW == 8) {
            if (v == 8) return try_staged<8, 7, 4, 2, true>(p, items, dest, table, out, s);
            if (v == 9) return try_staged<8, 4, 4, 3, true>(p, items, dest, table, out, s);
            if (v == 10) return try_staged<8, 3, 8, 2, true>(p, items, dest, table, out, s);
            if (v == 11) return try_staged<8, 2, 4, 4, true>(p, items, dest, table, out, s);
        } else if constexpr (NW == 4) {
            if (v == 8) return try_staged<4, 12, 4, 2, true>(p, items, dest, table, out, s);
            if (v == 9) return try_staged<4, 8, 4, 3, true>(p, items, dest, table, out, s);
            if (v == 10) return try_staged<4, 5, 8, 2, true>(p, items, dest, table, out, s);
            if (v == 11) return try_staged<4, 4, 4, 4, true>(p, items, dest, table, out, s);
        }
        return false;
    }
    if (v >= 5) {
        if (v == 5) return try_gather<NW, 16, 4, 4>(p, items, dest, table, out, s);  // 4096-slot chunks
        if (v == 6) return try_gather<NW, 32, 4, 2>(p, items, dest, table, out, s);  // 8192-slot chunks
        if (v == 7) return try_gather<NW, 16, 8, 2>(p, items, dest, table, out, s);  // 8192, 8 waves
        return false;
    }
    if constexpr (NW == 8) {
        if ((v == 0 || v == 1) && try_staged<8, 7, 4, 2>(p, items, dest, table, out, s)) return true;
        if ((v == 0 || v == 2) && try_staged<8, 4, 4, 3>(p, items, dest, table, out, s)) return true;
        if ((v == 0 || v == 3) && try_staged<8, 3, 8, 2>(p, items, dest, table, out, s)) return true;
        if ((v == 0 || v == 4) && try_staged<8, 2, 4, 4>(p, items, dest, table, out, s)) return true;
        return false;
    } else if constexpr (NW == 4) {
        if ((v == 0 || v == 1) && try_staged<4, 12, 4, 2>(p, items, dest, table, out, s)) return true;
        if ((v == 0 || v == 2) && try_staged<4, 8, 4, 3>(p, items, dest, table, out, s)) return true;
        if ((v == 0 || v == 3) && try_staged<4, 5, 8, 2>(p, items, dest, table, out, s)) return true;
        if ((v == 0 || v == 4) && try_staged<4, 4, 4, 4>(p, items, dest, table, out, s)) return true;
        return false;
    } else if constexpr (NW <= 3) {
        return try_staged<NW, 16, 4, 2>(p, items, dest, table, out, s);
    } else if constexpr (56 / NW > 0) {
        return try_staged<NW, 56 / NW, 4, 2>(p, items, dest, table, out, s);
    } else {
        return false;
    }
}

template <int NW>
void launch_scatter(const SplitPlan &p, const uint32_t *items, const int32_t *dest,
                    const uint32_t *table, const uint16_t *pre, uint32_t *out, uint32_t *dummy, hipStream_t s)
{
    if constexpr (NW > 0) {
        if (launch_staged<NW>(p, items, dest, table, pre, out, dummy, s)) return;
    }
    int nbits = 1;
    while ((1 << nbits) < p.D) ++nbits;
    const size_t lds = sizeof(uint32_t) * 4 * (size_t)p.D;
    hipLaunchKernelGGL(scatter_kernel<NW>, dim3(p.n_tiles), dim3(256), lds, s, items, dest, p.n,
                       p.D, nbits, p.tile, p.n_tiles, table, out, p.S / 4);
}

}  // namespace

namespace {
constexpr uint64_t kMaxTiles = 4096;

uint64_t min_tile(int32_t D)
{
    // at least 1024 slots and about one table byte per slot
    const uint64_t t = std::max<uint64_t>(1024, 4ull * (uint64_t)(D + 2));
    return (t + 1023) / 1024 * 1024;
}

void finish_plan(SplitPlan &p)
{
    p.rows = (uint64_t)p.D + 2;
    p.M = p.rows * p.n_tiles;
    p.scan_blocks = (uint32_t)((p.M + kScanChunk - 1) / kScanChunk);
    // fixed head: the fused scan's finished-tile counter, then the dummy slot
    p.off_done = 0;
    p.off_dummy = 256;
    p.off_table = 512;
    p.off_part = p.off_table + (p.M * 4 + 255) / 256 * 256;
    p.bytes = p.off_part + ((uint64_t)std::max<uint32_t>(p.scan_blocks, 1) * 4 + 255) / 256 * 256;
    p.off_pre = p.bytes;
    if (p.lock) p.bytes += ((uint64_t)p.n_chunks * (uint64_t)p.D * 2 + 255) / 256 * 256;
}

// The lockstep scatter takes items that are not whole 16-byte pieces (the
// raw shape's sizes), at most the staged shapes' destination count, and
// splits of at least 2^21 slots (four chunks per workgroup) whose table the
// scan takes in one partial-sum pass.
constexpr uint64_t kLockMinN = 1ull << 21;

bool lock_eligible(uint64_t n, int32_t D, uint32_t S)
{
    const uint32_t NW = S / 4;
    const uint64_t tiles = (n + kLockTile * kLockChunk - 1) / (kLockTile * kLockChunk);
    return S % 4 == 0 && NW % 4 != 0 && NW >= 3 && NW <= 15 && D <= dev::kStagedMaxD && n >= kLockMinN &&
           ((uint64_t)D + 2) * tiles <= (uint64_t)kPartMax * kScanChunk;
}

SplitPlan lock_plan(uint64_t n, int32_t D, uint32_t S)
{
    SplitPlan p;
    p.n = n;
    p.D = D;
    p.S = S;
    p.tile = kLockTile * kLockChunk;
    p.n_tiles = (uint32_t)((n + p.tile - 1) / p.tile);
    p.lock = kLockTile;
    p.n_chunks = (uint32_t)((n + kLockChunk - 1) / kLockChunk);
    finish_plan(p);
    return p;
}
}  // namespace

int split_set_variant(int v)
{
    if (v < 0 || v > 17) return RAFI_ERR_ARG;
    g_split_variant = v;
    return RAFI_OK;
}

SplitPlan split_plan(uint64_t n, int32_t D, uint32_t S, bool allow_lock)
{
    if (allow_lock && (g_split_variant == 0 || g_split_variant == 17) && lock_eligible(n, D, S))
        return lock_plan(n, D, S);
    SplitPlan p;
    p.n = n;
    p.D = D;
    p.S = S;
    uint64_t t = std::max<uint64_t>(min_tile(D), (n + kMaxTiles - 1) / kMaxTiles);
    t = (t + 1023) / 1024 * 1024;
    p.tile = (uint32_t)t;
    p.n_tiles = (uint32_t)((n + t - 1) / t);
    finish_plan(p);
    return p;
}

SplitPlan split_plan_bound(uint64_t cap, int32_t D, uint32_t S)
{
    // every n <= cap uses a tile >= min_tile(D) and at most kMaxTiles tiles
    SplitPlan p;
    p.n = cap;
    p.D = D;
    p.S = S;
    p.tile = (uint32_t)min_tile(D);
    p.n_tiles = (uint32_t)std::min<uint64_t>(kMaxTiles, (cap + p.tile - 1) / p.tile);
    finish_plan(p);
    // a lockstep plan for some n <= cap (whatever shape is selected later):
    // its workspace grows with n
    if (lock_eligible(cap, D, S)) p.bytes = std::max(p.bytes, lock_plan(cap, D, S).bytes);
    return p;
}

int split_run(const SplitPlan &p, const void *items, const int32_t *dest, void *out,
              uint64_t *offsets, uint64_t *summary, uint32_t *tile_offsets, uint32_t tile_items,
              void *workspace, hipStream_t s, const SplitEvents *ev, unsigned long long *dropped, bool fused)
{
    if (p.scan_blocks > (uint32_t)kPartMax) return RAFI_ERR_ARG;
    if (ev) RAFI_HIP_CHECK(hipEventRecord(ev->begin, s));
    uint32_t *table = reinterpret_cast<uint32_t *>(static_cast<char *>(workspace) + p.off_table);
    uint32_t *part = reinterpret_cast<uint32_t *>(static_cast<char *>(workspace) + p.off_part);
    uint32_t *dummy = reinterpret_cast<uint32_t *>(static_cast<char *>(workspace) + p.off_dummy);
    uint32_t *counters = reinterpret_cast<uint32_t *>(static_cast<char *>(workspace) + p.off_done);
    uint16_t *pre = reinterpret_cast<uint16_t *>(static_cast<char *>(workspace) + p.off_pre);
    const uint32_t ti = tile_items ? tile_items : 1u;
    // The fused launch costs one device-scope fence (an L2 write-back on this
    // multi-XCD part) per workgroup: worth it only for small tables.
    if (p.n_tiles > 0 && fused && !p.lock && p.M <= kFusedMaxM && p.n_tiles <= kFusedMaxTiles) {
        hipLaunchKernelGGL(hist_scan_kernel, dim3(p.n_tiles), dim3(256), sizeof(uint32_t) * p.rows, s, dest, p.n,
                           p.D, p.tile, p.n_tiles, table, p.M, counters, offsets, summary, tile_offsets, ti,
                           dropped);
        RAFI_LAUNCH_CHECK();
    } else {
        if (p.n_tiles > 0) {
            if (p.lock)
                hipLaunchKernelGGL(hist_lock_kernel, dim3(p.n_tiles), dim3(256), sizeof(uint32_t) * p.rows, s,
                                   dest, p.n, p.D, p.n_tiles, p.n_chunks, table, pre);
            else
                hipLaunchKernelGGL(hist_kernel, dim3(p.n_tiles), dim3(256), sizeof(uint32_t) * p.rows, s,
                                   dest, p.n, p.D, p.tile, p.n_tiles, table);
            RAFI_LAUNCH_CHECK();
            hipLaunchKernelGGL(scan_reduce_kernel, dim3(p.scan_blocks), dim3(kScanThreads), 0, s, table,
                               p.M, part);
            if (p.scan_blocks <= kDirectMaxBlocks) {
                hipLaunchKernelGGL(scan_apply_direct_kernel, dim3(p.scan_blocks), dim3(kScanThreads), 0, s,
                                   table, p.M, part);
            } else {
                hipLaunchKernelGGL(scan_partials_kernel, dim3(1), dim3(kPartThreads), 0, s, part,
                                   p.scan_blocks);
                hipLaunchKernelGGL(scan_apply_kernel, dim3(p.scan_blocks), dim3(kScanThreads), 0, s, table,
                                   p.M, part);
            }
            RAFI_LAUNCH_CHECK();
        }
        hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(1024), 0, s, table, p.n_tiles, p.D, p.n,
                           offsets, summary, tile_offsets, ti, dropped);
        RAFI_LAUNCH_CHECK();
    }
    if (ev) RAFI_HIP_CHECK(hipEventRecord(ev->before_scatter, s));
    if (p.n_tiles == 0) {
        if (ev) RAFI_HIP_CHECK(hipEventRecord(ev->end, s));
        return RAFI_OK;
    }
    const uint32_t *it = static_cast<const uint32_t *>(items);
    uint32_t *o = static_cast<uint32_t *>(out);
    switch (p.S / 4) {
    case 1: launch_scatter<1>(p, it, dest, table, pre, o, dummy, s); break;
    case 2: launch_scatter<2>(p, it, dest, table, pre, o, dummy, s); break;
    case 3: launch_scatter<3>(p, it, dest, table, pre, o, dummy, s); break;
    case 4: launch_scatter<4>(p, it, dest, table, pre, o, dummy, s); break;
    case 6: launch_scatter<6>(p, it, dest, table, pre, o, dummy, s); break;
    case 8: launch_scatter<8>(p, it, dest, table, pre, o, dummy, s); break;
    case 10: launch_scatter<10>(p, it, dest, table, pre, o, dummy, s); break;
    case 11: launch_scatter<11>(p, it, dest, table, pre, o, dummy, s); break;
    case 12: launch_scatter<12>(p, it, dest, table, pre, o, dummy, s); break;
    case 16: launch_scatter<16>(p, it, dest, table, pre, o, dummy, s); break;
    default: launch_scatter<0>(p, it, dest, table, pre, o, dummy, s); break;
    }
    RAFI_LAUNCH_CHECK();
    if (ev) RAFI_HIP_CHECK(hipEventRecord(ev->end, s));
    return RAFI_OK;
}

}  // namespace rafi
