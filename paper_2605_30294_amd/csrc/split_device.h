// Device building blocks of the stable multi-split, shared by the plain
// forward step (multisplit.hip) and the segmented one of the batched form
// (batched.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "rafi.h"

namespace rafi {
namespace dev {

// Inclusive scan over the 64 lanes of a wave (all lanes active): a
// Hillis-Steele scan inside each row of 16 lanes with DPP row shifts (lanes
// shifted in from outside the row read 0), then the totals of rows 0..2
// (lanes 15, 31, 47) added to the rows after them.
__device__ inline uint32_t wave_incl_scan(uint32_t v)
{
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false);  // row_shr:1
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false);  // row_shr:2
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false);  // row_shr:4
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false);  // row_shr:8
    const uint32_t row = (threadIdx.x & 63) >> 4;
    const uint32_t r0 = (uint32_t)__builtin_amdgcn_readlane((int)v, 15);
    const uint32_t r1 = (uint32_t)__builtin_amdgcn_readlane((int)v, 31);
    const uint32_t r2 = (uint32_t)__builtin_amdgcn_readlane((int)v, 47);
    return v + (row >= 1 ? r0 : 0u) + (row >= 2 ? r1 : 0u) + (row >= 3 ? r2 : 0u);
}

// Exclusive block scan; lds needs NT/64 + 1 words. Returns the exclusive
// prefix of v and the block total in *total.
template <int NT>
__device__ inline uint32_t block_excl_scan(uint32_t v, uint32_t *lds, uint32_t *total)
{
    constexpr int NW = NT / 64;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    uint32_t incl = wave_incl_scan(v);
    if (lane == 63) lds[wave] = incl;
    __syncthreads();
    if (tid < 64) {
        uint32_t w = tid < NW ? lds[tid] : 0u;
        uint32_t wi = wave_incl_scan(w);
        if (tid < NW) lds[tid] = wi - w;
        if (tid == NW - 1) lds[NW] = wi;
    }
    __syncthreads();
    uint32_t res = lds[wave] + incl - v;
    *total = lds[NW];
    __syncthreads();
    return res;
}

typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

// 16-byte streaming load (read once; not kept in the caches).
__device__ inline uint4 load_nt4(const void *p)
{
    const u32x4_t v = __builtin_nontemporal_load(reinterpret_cast<const u32x4_t *>(p));
    return make_uint4(v.x, v.y, v.z, v.w);
}

__device__ inline uint32_t bucket_of(int32_t d, int32_t D)
{
    if (d >= 0 && d < D) return (uint32_t)d;
    return d == RAFI_DONE ? (uint32_t)D : (uint32_t)D + 1u;
}

// Lanes of this wave whose key equals mine (only lanes with ok set take part).
__device__ inline uint64_t match_peers(uint32_t key, bool ok, int nbits)
{
    uint64_t peers = __ballot(ok);
    for (int b = 0; b < nbits; ++b) {
        const bool bit = (key >> b) & 1u;
        const uint64_t m = __ballot(bit);
        peers &= bit ? m : ~m;
    }
    return peers;
}

// ------------------------------------------------ staged stable scatter ---
// A tile of slots [tstart, tend) is processed in chunks of CH = W waves x R
// rounds x 64 slots. Per chunk:
//   rank   each wave owns a contiguous 1/W of the chunk; round r, lane l takes
//          slot wave_base + 64 r + l, so slot order = (round, lane) order. A
//          ballot match gives the lane's rank among same-destination lanes,
//          and a per-wave LDS counter carries it across rounds.
//   scan   chunk-local offsets over destinations (block scan), turned into
//          per-wave bases.
//   place  items move from registers into LDS at their chunk-sorted slot,
//          together with that slot's output position.
//   write  consecutive threads write consecutive 16-byte pieces of the
//          sorted chunk, so every destination run goes out as whole lines.
// The next chunk's loads are issued before the write phase.
constexpr int kStagedMaxD = 1024;
constexpr size_t kStagedLdsPerCu = 160 * 1024;

template <int NW, int R, int W>
constexpr size_t staged_lds_bytes_c(int32_t D)
{
    constexpr int CH = W * 64 * R;
    return sizeof(uint32_t) * ((size_t)CH * NW + D + CH) + sizeof(uint16_t) * ((size_t)W * D + 1);
}

template <int NW, int R, int W>
inline size_t staged_lds_bytes(int32_t D)
{
    return staged_lds_bytes_c<NW, R, W>(D);
}

// Destination of slot i is dest[i] - dbase, valid when in [0, D). run_base(e)
// gives the output slot of the tile's first item bound for e. Output slots
// >= out_cap are never written (they cannot occur for a consistent table).
//
// DB = false: one register buffer; the next chunk's loads are issued after
// the place phase and overlap the write phase only.
// DB = true: two register buffers; the next chunk's loads are issued before
// the current chunk is ranked, so they overlap all of its phases (the shape
// needs 2 x R x NW item registers per lane).
template <int NW, int R, int W, bool DB = false, typename RunBase>
__device__ inline void staged_scatter_tile(const uint32_t *__restrict__ items, const int32_t *__restrict__ dest,
                                           uint64_t tstart, uint64_t tend, int32_t D, int32_t dbase, int nbits,
                                           RunBase run_base, uint32_t *__restrict__ out, uint64_t out_cap,
                                           uint32_t *lds)
{
    constexpr int NT = 64 * W, SEG = 64 * R, CH = W * SEG;
    constexpr int PIECE = (NW % 4 == 0) ? 4 : ((NW % 2 == 0) ? 2 : 1);  // words per store
    constexpr int PPI = NW / PIECE;                                    // pieces per item
    constexpr int EPT = (kStagedMaxD + NT - 1) / NT;                   // max destinations per thread
    uint32_t *stage = lds;                                             // [CH * NW]
    uint32_t *run = stage + CH * NW;                                   // [D] next output slot per dest
    uint32_t *gpos = run + D;                                          // [CH] output slot of sorted slot j
    uint16_t *cnt = reinterpret_cast<uint16_t *>(gpos + CH);           // [W * D]
    __shared__ uint32_t scan_lds[NT / 64 + 1];

    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const uint64_t lt = (1ull << lane) - 1ull;
    const int per = (D + NT - 1) / NT;  // destinations per thread in the scans
    const int e0 = tid * per;

    for (int32_t e = tid; e < D; e += NT) run[e] = run_base(e);

    typedef uint32_t Items[R][NW];
    typedef int32_t Dests[R];
    auto load_chunk = [&](Items &item, Dests &dd, uint64_t cbase) {
        const uint64_t qbase = cbase + (uint64_t)w * SEG;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint64_t i = qbase + 64 * r + lane;
            dd[r] = i < tend ? __builtin_nontemporal_load(dest + i) - dbase : -1;
            if (i < tend) {
                const uint32_t *src = items + i * NW;
                if constexpr (NW % 4 == 0) {
#pragma unroll
                    for (int k = 0; k < NW / 4; ++k) {
                        const uint4 q = load_nt4(src + 4 * k);
                        item[r][4 * k] = q.x; item[r][4 * k + 1] = q.y;
                        item[r][4 * k + 2] = q.z; item[r][4 * k + 3] = q.w;
                    }
                } else {
#pragma unroll
                    for (int k = 0; k < NW; ++k) item[r][k] = __builtin_nontemporal_load(src + k);
                }
            }
        }
    };

    // One chunk; `after_place` runs once the chunk's registers are free.
    auto process = [&](Items &item, Dests &dd, auto after_place) {
        uint16_t rank[R];
        for (int k = tid; k < (W * D + 1) / 2; k += NT) reinterpret_cast<uint32_t *>(cnt)[k] = 0;
        __syncthreads();

        // rank
        uint16_t *mycnt = cnt + w * D;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int32_t d = dd[r];
            const bool ok = d >= 0 && d < D;
            const uint64_t peers = match_peers((uint32_t)d, ok, nbits);
            uint16_t before = 0;
            if (ok) before = mycnt[d];
            __builtin_amdgcn_wave_barrier();
            rank[r] = (uint16_t)(before + __popcll(peers & lt));
            if (ok && (peers & lt) == 0ull) mycnt[d] = (uint16_t)(before + __popcll(peers));
            __builtin_amdgcn_wave_barrier();
        }
        __syncthreads();

        // scan: chunk totals per destination -> chunk offsets -> per-wave
        // bases; the wave-0 base is the chunk offset excl[e], and the output
        // slot of chunk-sorted slot j bound for e is run[e] - excl[e] + j
        uint32_t tot_e[EPT];
        uint32_t local = 0;
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
            const int32_t e = e0 + k;
            uint32_t t = 0;
            if (k < per && e < D)
#pragma unroll
                for (int ww = 0; ww < W; ++ww) t += cnt[ww * D + e];
            tot_e[k] = t;
            local += t;
        }
        uint32_t chunk_total;
        uint32_t base = block_excl_scan<NT>(local, scan_lds, &chunk_total);
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
            const int32_t e = e0 + k;
            if (k < per && e < D) {
                uint32_t b = base;
#pragma unroll
                for (int ww = 0; ww < W; ++ww) {
                    const uint32_t c = cnt[ww * D + e];
                    cnt[ww * D + e] = (uint16_t)b;
                    b += c;
                }
            }
            base += tot_e[k];
        }
        __syncthreads();

        // place: items go to their chunk-sorted slot in LDS
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int32_t d = dd[r];
            if (d >= 0 && d < D) {
                const uint32_t pos = (uint32_t)cnt[w * D + d] + rank[r];
                uint32_t *dst = stage + pos * NW;
                if constexpr (NW % 4 == 0) {
#pragma unroll
                    for (int k = 0; k < NW / 4; ++k)
                        reinterpret_cast<uint4 *>(dst)[k] =
                            make_uint4(item[r][4 * k], item[r][4 * k + 1], item[r][4 * k + 2], item[r][4 * k + 3]);
                } else {
#pragma unroll
                    for (int k = 0; k < NW; ++k) dst[k] = item[r][k];
                }
                gpos[pos] = run[d] - (uint32_t)cnt[d] + pos;
            }
        }
        __syncthreads();

        after_place();

        // advance the per-destination output slots past this chunk
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
            const int32_t e = e0 + k;
            if (k < per && e < D) run[e] += tot_e[k];
        }

        // write: whole destination runs, consecutive lanes on consecutive pieces
        const uint32_t n_pieces = chunk_total * PPI;
        for (uint32_t q = tid; q < n_pieces; q += NT) {
            const uint32_t j = q / PPI, part = q - j * PPI;
            const uint32_t g = gpos[j];
            if (g < out_cap) {
                const uint32_t *src = stage + j * NW + part * PIECE;
                uint32_t *dst = out + (uint64_t)g * NW + part * PIECE;
                if constexpr (PIECE == 4)
                    *reinterpret_cast<uint4 *>(dst) = *reinterpret_cast<const uint4 *>(src);
                else if constexpr (PIECE == 2)
                    *reinterpret_cast<uint2 *>(dst) = *reinterpret_cast<const uint2 *>(src);
                else
                    *dst = *src;
            }
        }
        __syncthreads();
    };

    Items itemA;
    Dests ddA;
    if (tstart < tend) load_chunk(itemA, ddA, tstart);
    if constexpr (!DB) {
        for (uint64_t cbase = tstart; cbase < tend; cbase += CH)
            process(itemA, ddA, [&] {
                // the registers are free again: start loading the next chunk so
                // its latency overlaps the write phase
                if (cbase + CH < tend) load_chunk(itemA, ddA, cbase + CH);
            });
    } else {
        Items itemB;
        Dests ddB;
        for (uint64_t cbase = tstart; cbase < tend; cbase += 2 * CH) {
            const uint64_t c1 = cbase + CH;
            if (c1 < tend) load_chunk(itemB, ddB, c1);
            process(itemA, ddA, [] {});
            if (c1 >= tend) break;
            if (c1 + CH < tend) load_chunk(itemA, ddA, c1 + CH);
            process(itemB, ddB, [] {});
        }
    }
}

// ------------------------------------------------- wide staged scatter ---
// One workgroup per CU stages a chunk of CH = W x R x 64 slots (4096 for
// 32-byte items), so that a destination's run in a chunk averages CH / D
// items: 128 bytes at 1024 destinations. The output slot of chunk-sorted
// slot j bound for e is rb[e] + j, so LDS holds only the items, the per-wave
// counters, rb[D] and a 16-bit destination per sorted slot; each thread keeps
// the output cursors of the destinations it scans in registers.
// Every global load and store is issued unconditionally (reads past the tile
// are clamped to its last slot, surplus store lanes repeat the last piece of
// the chunk or write the 16-byte dummy), so the compiler can count
// outstanding memory operations exactly and waits for a chunk's loads never
// wait for the previous chunk's stores.
// DB = true issues the next chunk's loads before the current chunk is ranked.
template <int NW, int R, int W>
constexpr size_t wide_lds_bytes_c(int32_t D)
{
    constexpr int CH = W * 64 * R;
    return sizeof(uint32_t) * ((size_t)CH * NW + D) + sizeof(uint16_t) * ((size_t)W * D + 1 + CH);
}

template <int NW, int R, int W, bool DB, typename RunBase>
__device__ inline void wide_scatter_tile(const uint32_t *__restrict__ items, const int32_t *__restrict__ dest,
                                         uint64_t tstart, uint64_t tend, int32_t D, int32_t dbase, int nbits,
                                         RunBase run_base, uint32_t *__restrict__ out, uint64_t out_cap,
                                         uint32_t *__restrict__ dummy, uint32_t *lds)
{
    constexpr int NT = 64 * W, SEG = 64 * R, CH = W * SEG;
    static_assert(NW % 4 == 0, "16-byte pieces");
    static_assert(CH <= 65536, "chunk-local indices are 16-bit");
    constexpr int PPI = NW / 4;                          // 16-byte pieces per item
    constexpr int NPT = CH * PPI / NT;                   // store pieces per thread per chunk
    constexpr int EPT = (kStagedMaxD + NT - 1) / NT;     // max destinations per thread
    uint32_t *stage = lds;                               // [CH * NW]
    uint32_t *rb = stage + CH * NW;                      // [D]
    uint16_t *cnt = reinterpret_cast<uint16_t *>(rb + D);  // [W * D (+1)]
    uint16_t *sdst = cnt + W * D + 1;                    // [CH] destination of sorted slot j
    __shared__ uint32_t scan_lds[NT / 64 + 1];

    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const uint64_t lt = (1ull << lane) - 1ull;
    const int per = (D + NT - 1) / NT;
    const int e0 = tid * per;

    uint32_t cursor[EPT];
#pragma unroll
    for (int k = 0; k < EPT; ++k) cursor[k] = (k < per && e0 + k < D) ? run_base(e0 + k) : 0u;

    typedef uint32_t Items[R][NW];
    typedef int32_t Dests[R];
    auto load_chunk = [&](Items &item, Dests &dd, uint64_t cbase) {
        const uint64_t qbase = cbase + (uint64_t)w * SEG;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint64_t i = qbase + 64 * r + lane;
            const uint64_t ic = i < tend ? i : tend - 1;
            const int32_t x = __builtin_nontemporal_load(dest + ic);
            dd[r] = i < tend ? x - dbase : -1;
            const uint32_t *src = items + ic * NW;
#pragma unroll
            for (int k = 0; k < NW / 4; ++k) {
                const uint4 q = load_nt4(src + 4 * k);
                item[r][4 * k] = q.x; item[r][4 * k + 1] = q.y;
                item[r][4 * k + 2] = q.z; item[r][4 * k + 3] = q.w;
            }
        }
        // keep these loads ahead of the memory operations that follow
        __asm__ __volatile__("" ::: "memory");
    };

    auto process = [&](Items &item, Dests &dd, auto after_place) {
        uint16_t rank[R];
        for (int k = tid; k < (W * D + 1) / 2; k += NT) reinterpret_cast<uint32_t *>(cnt)[k] = 0;
        __syncthreads();

        uint16_t *mycnt = cnt + w * D;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int32_t d = dd[r];
            const bool ok = d >= 0 && d < D;
            const uint64_t peers = match_peers((uint32_t)d, ok, nbits);
            uint16_t before = 0;
            if (ok) before = mycnt[d];
            __builtin_amdgcn_wave_barrier();
            rank[r] = (uint16_t)(before + __popcll(peers & lt));
            if (ok && (peers & lt) == 0ull) mycnt[d] = (uint16_t)(before + __popcll(peers));
            __builtin_amdgcn_wave_barrier();
        }
        __syncthreads();

        uint32_t tot_e[EPT];
        uint32_t local = 0;
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
            const int32_t e = e0 + k;
            uint32_t t = 0;
            if (k < per && e < D)
#pragma unroll
                for (int ww = 0; ww < W; ++ww) t += cnt[ww * D + e];
            tot_e[k] = t;
            local += t;
        }
        uint32_t chunk_total;
        uint32_t base = block_excl_scan<NT>(local, scan_lds, &chunk_total);
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
            const int32_t e = e0 + k;
            if (k < per && e < D) {
                rb[e] = cursor[k] - base;  // output slot = rb[e] + chunk-sorted index
                cursor[k] += tot_e[k];
                uint32_t b = base;
#pragma unroll
                for (int ww = 0; ww < W; ++ww) {
                    const uint32_t c = cnt[ww * D + e];
                    cnt[ww * D + e] = (uint16_t)b;
                    b += c;
                }
            }
            base += tot_e[k];
        }
        __syncthreads();

#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int32_t d = dd[r];
            if (d >= 0 && d < D) {
                const uint32_t pos = (uint32_t)cnt[w * D + d] + rank[r];
                uint32_t *dst = stage + pos * NW;
#pragma unroll
                for (int k = 0; k < NW / 4; ++k)
                    reinterpret_cast<uint4 *>(dst)[k] =
                        make_uint4(item[r][4 * k], item[r][4 * k + 1], item[r][4 * k + 2], item[r][4 * k + 3]);
                sdst[pos] = (uint16_t)d;
            }
        }
        __syncthreads();

        after_place();

        // write: NPT pieces per thread, all issued
        const uint32_t n_pieces = chunk_total * PPI;
#pragma unroll
        for (int u = 0; u < NPT; ++u) {
            const uint32_t q = (uint32_t)(u * NT + tid);
            const uint32_t qq = q < n_pieces ? q : (n_pieces ? n_pieces - 1 : 0);
            const uint32_t j = qq / PPI, part = qq - j * PPI;
            // sdst[0] may be stale when the chunk is empty; keep the LDS index
            // in range (the store then goes to the dummy)
            const uint32_t e = min((uint32_t)sdst[j], (uint32_t)(D - 1));
            const uint32_t g = rb[e] + j;
            const uint4 v = *reinterpret_cast<const uint4 *>(stage + j * NW + part * 4);
            uint32_t *dst = (n_pieces && g < out_cap) ? out + (uint64_t)g * NW + part * 4 : dummy;
            *reinterpret_cast<uint4 *>(dst) = v;
        }
        __syncthreads();
    };

    Items itemA;
    Dests ddA;
    if (tstart >= tend) return;
    load_chunk(itemA, ddA, tstart);
    if constexpr (!DB) {
        for (uint64_t cbase = tstart; cbase < tend; cbase += CH)
            process(itemA, ddA, [&] { load_chunk(itemA, ddA, cbase + CH); });
    } else {
        Items itemB;
        Dests ddB;
        for (uint64_t cbase = tstart; cbase < tend; cbase += 2 * CH) {
            load_chunk(itemB, ddB, cbase + CH);
            process(itemA, ddA, [] {});
            if (cbase + CH >= tend) break;
            load_chunk(itemA, ddA, cbase + 2 * CH);
            process(itemB, ddB, [] {});
        }
    }
}

// ------------------------------------------------ line-aligned scatter ---
// The wide shape, except that each destination's output run is written in
// whole 128-byte lines only. Writes that cover part of a line cost about as
// much as whole lines on this memory system, and a chunk's run for one
// destination is a few items long and starts anywhere in a line, so the
// wide shape spends most of its write time on partial lines. Here the items
// of a run's last, unfinished line are not written: the thread that owns the
// destination keeps them in registers and stages them again, in front of the
// destination's new items, in the next chunk. Only the first and the last
// line of a destination's run over [tstart, tend) can be partial writes.
// [tstart, tend) may span several histogram tiles: a destination's runs of
// consecutive tiles are adjacent in the output, so the cursor runs on.
//
// The stage holds a chunk of CH items plus the carried ones, and for each
// stage slot the output slot it is written to (all ones while held back), so
// that the write phase reads two independent LDS words per piece. When more
// than PMAX items would be carried into the next chunk, every destination
// writes its carried items as a partial line instead, so the stage never
// holds more than CH + PMAX. Output lines are counted from item 0: `out`
// must be 128-byte aligned, NW in {4, 8, 16}, and the output at most
// 0xfffffff0 bytes (it is written through a buffer resource with 32-bit
// offsets).
template <int NW, int R, int W, int PMAX>
constexpr size_t line_lds_bytes_c(int32_t D)
{
    constexpr int SC = W * 64 * R + PMAX;
    return sizeof(uint32_t) * ((size_t)SC * (NW + 1) + 2 * (size_t)D) + sizeof(uint16_t) * ((size_t)W * D + 2);
}

template <int NW, int R, int W, int PMAX, bool DB, typename RunBase>
__device__ inline void line_scatter_tile(const uint32_t *__restrict__ items, const int32_t *__restrict__ dest,
                                         uint64_t tstart, uint64_t tend, int32_t D, int nbits, RunBase run_base,
                                         uint32_t *__restrict__ out, uint64_t out_cap, uint32_t *lds)
{
    constexpr int NT = 64 * W, SEG = 64 * R, CH = W * SEG, SC = CH + PMAX;
    static_assert(NW == 4 || NW == 8 || NW == 16, "items that tile a 128-byte line in 16-byte pieces");
    static_assert(SC < 65536, "stage indices and the packed scan are 16-bit");
    constexpr int L = 32 / NW;                           // items per 128-byte line
    constexpr int LC = L - 1;                            // most items one destination carries
    constexpr int PPI = NW / 4;                          // 16-byte pieces per item
    constexpr int NPT = (SC * PPI + NT - 1) / NT;        // store pieces per thread per chunk
    constexpr int EPT = (kStagedMaxD + NT - 1) / NT;     // max destinations per thread
    static_assert((size_t)LC * kStagedMaxD < 65536, "carried count fits the packed scan");
    static_assert(SC * (NW + 1) % 2 == 0, "8-byte aligned destination table");
    static_assert(W % 4 == 0, "the count table is cleared in 8-byte words");
    constexpr uint32_t HELD = 0xffffffffu;
    uint32_t *stage = lds;                               // [SC * NW]
    uint32_t *gidx = stage + SC * NW;                    // [SC] output slot of stage slot j, or HELD
    uint2 *rbw = reinterpret_cast<uint2 *>(gidx + SC);   // [D] {output slot of stage slot 0, first slot held}
    uint16_t *cnt = reinterpret_cast<uint16_t *>(rbw + D);  // [W * D (+2)]
    __shared__ uint32_t scan_lds[NT / 64 + 1];

    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const uint64_t lt = (1ull << lane) - 1ull;
    const int per = (D + NT - 1) / NT;
    const int e0 = tid * per;

    // per owned destination: output slot of its next new item, the items it
    // carries (those of slots [cur - pend, cur)) and where they sit in the stage
    uint32_t cur[EPT], pend[EPT], keep[EPT];
    uint32_t carry[EPT][LC][NW];
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
        cur[k] = (k < per && e0 + k < D) ? run_base(e0 + k) : 0u;
        pend[k] = 0;
        keep[k] = 0;
    }

    typedef uint32_t Items[R][NW];
    typedef int32_t Dests[R];
    auto load_chunk = [&](Items &item, Dests &dd, uint64_t cbase) {
        const uint64_t qbase = cbase + (uint64_t)w * SEG;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint64_t i = qbase + 64 * r + lane;
            const uint64_t ic = i < tend ? i : tend - 1;
            const int32_t x = __builtin_nontemporal_load(dest + ic);
            dd[r] = i < tend ? x : -1;
            const uint32_t *src = items + ic * NW;
#pragma unroll
            for (int k = 0; k < NW / 4; ++k) {
                const uint4 q = load_nt4(src + 4 * k);
                item[r][4 * k] = q.x; item[r][4 * k + 1] = q.y;
                item[r][4 * k + 2] = q.z; item[r][4 * k + 3] = q.w;
            }
        }
        __asm__ __volatile__("" ::: "memory");
    };

    auto store_item = [&](uint32_t g, const uint32_t *v) {
        if (g < out_cap) {
            uint4 *dst = reinterpret_cast<uint4 *>(out + (uint64_t)g * NW);
#pragma unroll
            for (int k = 0; k < PPI; ++k) dst[k] = make_uint4(v[4 * k], v[4 * k + 1], v[4 * k + 2], v[4 * k + 3]);
        }
    };

    auto process = [&](Items &item, Dests &dd, auto after_place) {
        uint16_t rank[R];
        for (int k = tid; k < W * D / 4; k += NT) reinterpret_cast<uint64_t *>(cnt)[k] = 0ull;
        __syncthreads();

        uint16_t *mycnt = cnt + w * D;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int32_t d = dd[r];
            const bool ok = d >= 0 && d < D;
            const uint64_t peers = match_peers((uint32_t)d, ok, nbits);
            uint16_t before = 0;
            if (ok) before = mycnt[d];
            __builtin_amdgcn_wave_barrier();
            rank[r] = (uint16_t)(before + __popcll(peers & lt));
            if (ok && (peers & lt) == 0ull) mycnt[d] = (uint16_t)(before + __popcll(peers));
            __builtin_amdgcn_wave_barrier();
        }
        __syncthreads();

        // a destination's stage segment: its carried items, then its new ones;
        // one scan gives the segment bases (low half) and the carried total
        // of the next chunk (high half)
        // per-wave counts of the owned destinations, kept for the rewrite
        // below; two adjacent 16-bit counts are one 32-bit word when a
        // thread owns an even-aligned pair
        uint32_t cv[EPT][W];
        uint32_t *cnt32 = reinterpret_cast<uint32_t *>(cnt);
        const bool pairs = EPT == 2 && per == 2 && (D & 1) == 0;
        if (pairs) {
#pragma unroll
            for (int ww = 0; ww < W; ++ww) {
                const uint32_t pr = e0 < D ? cnt32[(ww * D + e0) >> 1] : 0u;
                cv[0][ww] = pr & 0xffffu;
                cv[EPT - 1][ww] = pr >> 16;
            }
        } else {
#pragma unroll
            for (int k = 0; k < EPT; ++k)
#pragma unroll
                for (int ww = 0; ww < W; ++ww) cv[k][ww] = (k < per && e0 + k < D) ? cnt[ww * D + e0 + k] : 0u;
        }
        uint32_t tot_e[EPT];
        uint32_t seg_sum = 0, carry_sum = 0;
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
            const int32_t e = e0 + k;
            uint32_t t = 0;
            if (k < per && e < D) {
#pragma unroll
                for (int ww = 0; ww < W; ++ww) t += cv[k][ww];
                const uint32_t a = cur[k] - pend[k], end = cur[k] + t;
                const uint32_t lend = end & ~(uint32_t)(L - 1);
                const uint32_t wl = lend > a ? lend : a;
                seg_sum += pend[k] + t;
                carry_sum += end - wl;
            }
            tot_e[k] = t;
        }
        uint32_t packed_total;
        const uint32_t packed = block_excl_scan<NT>(seg_sum | (carry_sum << 16), scan_lds, &packed_total);
        uint32_t base = packed & 0xffffu;
        const uint32_t staged = packed_total & 0xffffu, carried_next = packed_total >> 16;
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
            const int32_t e = e0 + k;
            if (k < per && e < D) {
                const uint32_t a = cur[k] - pend[k], end = cur[k] + tot_e[k];
                const uint32_t lend = end & ~(uint32_t)(L - 1);
                const uint32_t wl = lend > a ? lend : a;
                rbw[e] = make_uint2(a - base, wl);
#pragma unroll
                for (int i = 0; i < LC; ++i)
                    if ((uint32_t)i < pend[k]) {
                        uint4 *dst = reinterpret_cast<uint4 *>(stage + (base + i) * NW);
#pragma unroll
                        for (int q = 0; q < PPI; ++q)
                            dst[q] = make_uint4(carry[k][i][4 * q], carry[k][i][4 * q + 1], carry[k][i][4 * q + 2],
                                                carry[k][i][4 * q + 3]);
                        gidx[base + i] = a + i < wl ? a + i : HELD;
                    }
                uint32_t b = base + pend[k];
#pragma unroll
                for (int ww = 0; ww < W; ++ww) {
                    const uint32_t c = cv[k][ww];
                    cv[k][ww] = b;
                    b += c;
                }
                if (!pairs) {
#pragma unroll
                    for (int ww = 0; ww < W; ++ww) cnt[ww * D + e] = (uint16_t)cv[k][ww];
                }
                keep[k] = base + (wl - a);  // stage slot of the first item carried on
                base += pend[k] + tot_e[k];
                pend[k] = end - wl;
                cur[k] = end;
            }
        }
        if (pairs && e0 < D) {
#pragma unroll
            for (int ww = 0; ww < W; ++ww) cnt32[(ww * D + e0) >> 1] = cv[0][ww] | (cv[EPT - 1][ww] << 16);
        }
        __syncthreads();

#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int32_t d = dd[r];
            if (d >= 0 && d < D) {
                const uint32_t pos = (uint32_t)cnt[w * D + d] + rank[r];
                const uint2 bw = rbw[d];
                uint32_t *dst = stage + pos * NW;
#pragma unroll
                for (int k = 0; k < NW / 4; ++k)
                    reinterpret_cast<uint4 *>(dst)[k] =
                        make_uint4(item[r][4 * k], item[r][4 * k + 1], item[r][4 * k + 2], item[r][4 * k + 3]);
                const uint32_t g = bw.x + pos;
                gidx[pos] = g < bw.y ? g : HELD;
            }
        }
        __syncthreads();

        after_place();

        // write every staged piece that lies in a finished line, WB pieces
        // at a time with all their LDS reads issued together
        const uint32_t n_pieces = staged * PPI;
        constexpr int WB = 8;
        const __amdgpu_buffer_rsrc_t orsrc =
            __builtin_amdgcn_make_buffer_rsrc(out, (short)0, (int)(uint32_t)(out_cap * (uint64_t)(NW * 4)), 0x00020000);
#pragma unroll
        for (int u0 = 0; u0 < NPT; u0 += WB) {
            uint32_t g[WB], col[WB];
            uint4 v[WB];
#pragma unroll
            for (int b = 0; b < WB; ++b) {
                const uint32_t q = (uint32_t)((u0 + b) * NT + tid);
                const bool ok = u0 + b < NPT && q < n_pieces;
                const uint32_t qq = ok ? q : 0u;
                const uint32_t j = qq / PPI;
                col[b] = qq - j * PPI;
                g[b] = ok ? gidx[j] : HELD;
                v[b] = *reinterpret_cast<const uint4 *>(stage + j * NW + col[b] * 4);
            }
            // every lane issues its store; a held piece gets an offset past
            // the buffer's end, which the hardware drops. Stores issued in
            // every case let the compiler count outstanding memory
            // operations, so the next chunk's loads are not held behind them.
#pragma unroll
            for (int b = 0; b < WB; ++b) {
                const uint32_t off = g[b] < out_cap ? g[b] * (uint32_t)(NW * 4) + col[b] * 16u : 0xfffffff0u;
                const u32x4_t x = {v[b].x, v[b].y, v[b].z, v[b].w};
                __builtin_amdgcn_raw_buffer_store_b128(x, orsrc, (int)off, 0, 0);
            }
        }
        // pick up the items carried into the next chunk; if there are too
        // many for the stage, write them now (partial lines) instead
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
#pragma unroll
            for (int i = 0; i < LC; ++i)
                if ((uint32_t)i < pend[k]) {
#pragma unroll
                    for (int q = 0; q < PPI; ++q) {
                        const uint4 x = *reinterpret_cast<const uint4 *>(stage + (keep[k] + i) * NW + 4 * q);
                        carry[k][i][4 * q] = x.x; carry[k][i][4 * q + 1] = x.y;
                        carry[k][i][4 * q + 2] = x.z; carry[k][i][4 * q + 3] = x.w;
                    }
                    if (carried_next > (uint32_t)PMAX) store_item(cur[k] - pend[k] + i, carry[k][i]);
                }
            if (carried_next > (uint32_t)PMAX) pend[k] = 0;
        }
        __syncthreads();
    };

    if (tstart >= tend) return;
    Items itemA;
    Dests ddA;
    load_chunk(itemA, ddA, tstart);
    if constexpr (!DB) {
        for (uint64_t cbase = tstart; cbase < tend; cbase += CH)
            process(itemA, ddA, [&] { load_chunk(itemA, ddA, cbase + CH); });
    } else {
        Items itemB;
        Dests ddB;
        for (uint64_t cbase = tstart; cbase < tend; cbase += 2 * CH) {
            load_chunk(itemB, ddB, cbase + CH);
            process(itemA, ddA, [] {});
            if (cbase + CH >= tend) break;
            load_chunk(itemA, ddA, cbase + 2 * CH);
            process(itemB, ddB, [] {});
        }
    }
    // the last line of every run
#pragma unroll
    for (int k = 0; k < EPT; ++k)
#pragma unroll
        for (int i = 0; i < LC; ++i)
            if ((uint32_t)i < pend[k]) store_item(cur[k] - pend[k] + i, carry[k][i]);
}

// ------------------------------------- gather-read, coalesced-write scatter ---
// Same ranking as staged_scatter_tile, but LDS keeps only, per chunk-sorted
// slot, the chunk-local source index and the output slot (6 bytes instead of
// the item), so a chunk can hold many more slots and every destination run
// of a chunk is long. The write phase reads each item from global memory in
// sorted order (the chunk's lines come from HBM once and are then served by
// L2) and writes consecutive pieces of the sorted chunk with consecutive
// lanes.
template <int R, int W>
inline size_t gather_lds_bytes(int32_t D)
{
    constexpr int CH = W * 64 * R;
    return sizeof(uint32_t) * ((size_t)D + CH) + sizeof(uint16_t) * ((size_t)CH + (size_t)W * D + 1);
}

template <int NW, int R, int W, typename RunBase>
__device__ inline void gather_scatter_tile(const uint32_t *__restrict__ items, const int32_t *__restrict__ dest,
                                           uint64_t tstart, uint64_t tend, int32_t D, int32_t dbase, int nbits,
                                           RunBase run_base, uint32_t *__restrict__ out, uint64_t out_cap,
                                           uint32_t *lds)
{
    constexpr int NT = 64 * W, SEG = 64 * R, CH = W * SEG;
    constexpr int PIECE = (NW % 4 == 0) ? 4 : ((NW % 2 == 0) ? 2 : 1);
    constexpr int PPI = NW / PIECE;
    constexpr int EPT = (kStagedMaxD + NT - 1) / NT;
    constexpr int UNROLL = 8;
    static_assert(CH <= 65536, "chunk-local indices are 16-bit");
    uint32_t *run = lds;                                               // [D]
    uint32_t *gpos = run + D;                                          // [CH]
    uint16_t *src = reinterpret_cast<uint16_t *>(gpos + CH);           // [CH]
    uint16_t *cnt = src + CH;                                          // [W * D]
    __shared__ uint32_t scan_lds[NT / 64 + 1];

    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const uint64_t lt = (1ull << lane) - 1ull;
    const int per = (D + NT - 1) / NT;
    const int e0 = tid * per;

    for (int32_t e = tid; e < D; e += NT) run[e] = run_base(e);

    int32_t dd[R];
    uint16_t rank[R];
    auto load_dest = [&](uint64_t cbase) {
        const uint64_t qbase = cbase + (uint64_t)w * SEG;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint64_t i = qbase + 64 * r + lane;
            dd[r] = i < tend ? __builtin_nontemporal_load(dest + i) - dbase : -1;
        }
    };
    if (tstart < tend) load_dest(tstart);

    for (uint64_t cbase = tstart; cbase < tend; cbase += CH) {
        for (int k = tid; k < (W * D + 1) / 2; k += NT) reinterpret_cast<uint32_t *>(cnt)[k] = 0;
        __syncthreads();

        uint16_t *mycnt = cnt + w * D;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int32_t d = dd[r];
            const bool ok = d >= 0 && d < D;
            const uint64_t peers = match_peers((uint32_t)d, ok, nbits);
            uint16_t before = 0;
            if (ok) before = mycnt[d];
            __builtin_amdgcn_wave_barrier();
            rank[r] = (uint16_t)(before + __popcll(peers & lt));
            if (ok && (peers & lt) == 0ull) mycnt[d] = (uint16_t)(before + __popcll(peers));
            __builtin_amdgcn_wave_barrier();
        }
        __syncthreads();

        uint32_t tot_e[EPT];
        uint32_t local = 0;
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
            const int32_t e = e0 + k;
            uint32_t t = 0;
            if (k < per && e < D)
#pragma unroll
                for (int ww = 0; ww < W; ++ww) t += cnt[ww * D + e];
            tot_e[k] = t;
            local += t;
        }
        uint32_t chunk_total;
        uint32_t base = block_excl_scan<NT>(local, scan_lds, &chunk_total);
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
            const int32_t e = e0 + k;
            if (k < per && e < D) {
                uint32_t b = base;
#pragma unroll
                for (int ww = 0; ww < W; ++ww) {
                    const uint32_t c = cnt[ww * D + e];
                    cnt[ww * D + e] = (uint16_t)b;
                    b += c;
                }
            }
            base += tot_e[k];
        }
        __syncthreads();

#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int32_t d = dd[r];
            if (d >= 0 && d < D) {
                const uint32_t pos = (uint32_t)cnt[w * D + d] + rank[r];
                src[pos] = (uint16_t)(w * SEG + 64 * r + lane);
                gpos[pos] = run[d] - (uint32_t)cnt[d] + pos;
            }
        }
        __syncthreads();

        if (cbase + CH < tend) load_dest(cbase + CH);
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
            const int32_t e = e0 + k;
            if (k < per && e < D) run[e] += tot_e[k];
        }

        // write: UNROLL pieces per thread in flight (loads first, then stores)
        const uint32_t n_pieces = chunk_total * PPI;
        for (uint32_t q0 = 0; q0 < n_pieces; q0 += NT * UNROLL) {
            uint32_t v[UNROLL][PIECE];
            uint32_t g[UNROLL], part[UNROLL];
#pragma unroll
            for (int u = 0; u < UNROLL; ++u) {
                const uint32_t q = q0 + u * NT + tid;
                g[u] = 0xffffffffu;
                if (q < n_pieces) {
                    const uint32_t j = q / PPI;
                    part[u] = q - j * PPI;
                    g[u] = gpos[j];
                    const uint32_t *s = items + (cbase + src[j]) * NW + part[u] * PIECE;
                    if constexpr (PIECE == 4) {
                        const uint4 x = *reinterpret_cast<const uint4 *>(s);
                        v[u][0] = x.x; v[u][1] = x.y; v[u][2] = x.z; v[u][3] = x.w;
                    } else if constexpr (PIECE == 2) {
                        const uint2 x = *reinterpret_cast<const uint2 *>(s);
                        v[u][0] = x.x; v[u][1] = x.y;
                    } else {
                        v[u][0] = *s;
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < UNROLL; ++u) {
                if (g[u] < out_cap) {
                    uint32_t *dst = out + (uint64_t)g[u] * NW + part[u] * PIECE;
                    if constexpr (PIECE == 4)
                        *reinterpret_cast<uint4 *>(dst) = make_uint4(v[u][0], v[u][1], v[u][2], v[u][3]);
                    else if constexpr (PIECE == 2)
                        *reinterpret_cast<uint2 *>(dst) = make_uint2(v[u][0], v[u][1]);
                    else
                        *dst = v[u][0];
                }
            }
        }
        __syncthreads();
    }
}

// ------------------------------------------ wide scatter, raw staging ---
// The wide shape for items whose size is not a multiple of 16 bytes (the
// 44-byte rays of the paper's forwarding benchmark, the 40- and 24-byte
// N-body items). A chunk's bytes are read as consecutive 16-byte pieces and
// kept in LDS in load order: the chunk starts on a 16-byte boundary because
// CH and every tile start are multiples of 4 items. Ranking moves indices
// only: for each chunk-sorted slot j, its output slot and the chunk-local
// item it takes. The write phase gives consecutive 4-byte words of the
// sorted chunk to consecutive lanes, so a destination's run goes out as
// contiguous words. All stores are issued (surplus lanes write the dummy
// word), so the compiler counts outstanding memory operations exactly and
// the next chunk's loads, issued before the write phase, never wait for
// this chunk's stores.
template <int NW, int R, int W>
constexpr size_t wide_raw_lds_bytes_c(int32_t D)
{
    constexpr int CH = W * 64 * R;
    return sizeof(uint32_t) * ((size_t)CH * NW + D + CH) + sizeof(uint16_t) * ((size_t)W * D + 2 + CH);
}

// Chunk schedules of the raw scatter. A schedule names the chunks one
// workgroup processes, in order (chunk j covers slots [begin(j), end(j)), at
// most CH of them), and each destination's output slot for the first of its
// items in a chunk: base(j, e), read for every chunk when kRebase, else only
// for the first chunk, after which the cursor runs on.
//
// TileChunks: the consecutive chunks of one tile [tstart, tend).
template <int CH, typename RunBase>
struct TileChunks {
    static constexpr bool kRebase = false;
    uint64_t tstart, tend;
    RunBase run_base;
    __device__ bool has(uint32_t j) const { return tstart + (uint64_t)j * CH < tend; }
    __device__ uint64_t begin(uint32_t j) const { return tstart + (uint64_t)j * CH; }
    __device__ uint64_t end(uint32_t j) const { return min(begin(j) + CH, tend); }
    __device__ uint32_t base(uint32_t, int32_t e) const { return run_base(e); }
};

// LockChunks: chunk c0 + j * stride, for every such chunk below n_chunks.
// base(j, e) = the tile's run base (tiles of LC consecutive chunks) plus the
// items bound for e in the earlier chunks of the same tile (pre: u16 per
// chunk and destination).
template <int CH, int LC>
struct LockChunks {
    static constexpr bool kRebase = true;
    uint64_t n;
    uint32_t c0, stride, n_chunks, n_tiles;
    int32_t D;
    const uint32_t *__restrict__ table;
    const uint16_t *__restrict__ pre;
    __device__ uint32_t chunk(uint32_t j) const { return c0 + j * stride; }
    __device__ bool has(uint32_t j) const { return chunk(j) < n_chunks; }
    __device__ uint64_t begin(uint32_t j) const { return (uint64_t)chunk(j) * CH; }
    __device__ uint64_t end(uint32_t j) const { return min(begin(j) + CH, n); }
    __device__ uint32_t base(uint32_t j, int32_t e) const
    {
        const uint32_t c = chunk(j);
        return table[(uint64_t)e * n_tiles + c / LC] + (uint32_t)pre[(uint64_t)c * (uint32_t)D + (uint32_t)e];
    }
};

// words: 32-bit words of `items` that may be read, a multiple of 4 (at
// least 4); the host rounds the array's length up to it only where the
// allocation is padded for that.
template <int NW, int R, int W, typename Sched>
__device__ inline void wide_raw_scatter(const uint32_t *__restrict__ items, const int32_t *__restrict__ dest,
                                        uint64_t words, int32_t D, int nbits, const Sched &sched,
                                        uint32_t *__restrict__ out, uint64_t out_cap, uint32_t *__restrict__ dummy,
                                        uint32_t *lds)
{
    constexpr int NT = 64 * W, SEG = 64 * R, CH = W * SEG;
    static_assert((R * NW) % 4 == 0, "a chunk is a whole number of 16-byte pieces per thread");
    static_assert(CH <= 65536, "chunk-local indices are 16-bit");
    constexpr int PPT = R * NW / 4;                      // 16-byte load pieces per thread per chunk
    constexpr int WPT = R * NW;                          // 4-byte store words per thread per chunk
    constexpr int EPT = (kStagedMaxD + NT - 1) / NT;     // max destinations per thread
    uint32_t *stage = lds;                               // [CH * NW] the chunk's words in load order
    uint32_t *rb = stage + CH * NW;                      // [D]
    uint32_t *gpos = rb + D;                             // [CH] output slot of sorted slot j
    uint16_t *cnt = reinterpret_cast<uint16_t *>(gpos + CH);  // [W * D (+2)]
    uint16_t *ssrc = cnt + W * D + 2;                    // [CH] chunk-local item of sorted slot j
    __shared__ uint32_t scan_lds[NT / 64 + 1];

    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const uint64_t lt = (1ull << lane) - 1ull;
    const int per = (D + NT - 1) / NT;
    const int e0 = tid * per;

    // cursor: output slot of the next item bound for each owned destination;
    // nbase: the same for the next chunk, read with its items (kRebase)
    uint32_t cursor[EPT], nbase[EPT];
    auto load_bases = [&](uint32_t j) {
#pragma unroll
        for (int k = 0; k < EPT; ++k) nbase[k] = (k < per && e0 + k < D) ? sched.base(j, e0 + k) : 0u;
    };

    typedef uint4 Pieces[PPT];
    typedef int32_t Dests[R];
    // Slots [cbase, cend) of the chunk; pieces past the chunk's last word
    // (rounded up to a whole piece: chunk ends are multiples of 4 items
    // except at the array's end, whose padding `words` covers) read that
    // piece instead: they belong to no item of the chunk and are never stored.
    auto load_chunk = [&](Pieces &pc, Dests &dd, uint64_t cbase, uint64_t cend) {
        const uint64_t qbase = cbase + (uint64_t)w * SEG;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint64_t i = qbase + 64 * r + lane;
            const uint64_t ic = i < cend ? i : cend - 1;
            const int32_t x = __builtin_nontemporal_load(dest + ic);
            dd[r] = i < cend ? x : -1;
        }
        const uint64_t wb = cbase * NW;  // a multiple of 4
        const uint64_t we = (cend * NW + 3) & ~3ull;
        const uint64_t wlim = we < words ? we : words;
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const uint64_t w0 = wb + 4ull * (uint64_t)(k * NT + tid);
            pc[k] = load_nt4(items + (w0 + 4 <= wlim ? w0 : wlim - 4));
        }
        __asm__ __volatile__("" ::: "memory");
    };

    auto process = [&](Pieces &pc, Dests &dd, auto after_place) {
        // the chunk's bytes into LDS, in load order
#pragma unroll
        for (int k = 0; k < PPT; ++k) reinterpret_cast<uint4 *>(stage)[k * NT + tid] = pc[k];
        uint16_t rank[R];
        for (int k = tid; k < (W * D + 2) / 2; k += NT) reinterpret_cast<uint32_t *>(cnt)[k] = 0;
        __syncthreads();

        uint16_t *mycnt = cnt + w * D;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int32_t d = dd[r];
            const bool ok = d >= 0 && d < D;
            const uint64_t peers = match_peers((uint32_t)d, ok, nbits);
            uint16_t before = 0;
            if (ok) before = mycnt[d];
            __builtin_amdgcn_wave_barrier();
            rank[r] = (uint16_t)(before + __popcll(peers & lt));
            if (ok && (peers & lt) == 0ull) mycnt[d] = (uint16_t)(before + __popcll(peers));
            __builtin_amdgcn_wave_barrier();
        }
        __syncthreads();

        uint32_t tot_e[EPT];
        uint32_t local = 0;
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
            const int32_t e = e0 + k;
            uint32_t t = 0;
            if (k < per && e < D)
#pragma unroll
                for (int ww = 0; ww < W; ++ww) t += cnt[ww * D + e];
            tot_e[k] = t;
            local += t;
        }
        uint32_t chunk_total;
        uint32_t base = block_excl_scan<NT>(local, scan_lds, &chunk_total);
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
            const int32_t e = e0 + k;
            if (k < per && e < D) {
                rb[e] = cursor[k] - base;  // output slot = rb[e] + chunk-sorted index
                cursor[k] += tot_e[k];
                uint32_t b = base;
#pragma unroll
                for (int ww = 0; ww < W; ++ww) {
                    const uint32_t c = cnt[ww * D + e];
                    cnt[ww * D + e] = (uint16_t)b;
                    b += c;
                }
            }
            base += tot_e[k];
        }
        __syncthreads();

#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int32_t d = dd[r];
            if (d >= 0 && d < D) {
                const uint32_t pos = (uint32_t)cnt[w * D + d] + rank[r];
                gpos[pos] = rb[d] + pos;
                ssrc[pos] = (uint16_t)(w * SEG + 64 * r + lane);
            }
        }
        __syncthreads();

        after_place();

        // write: WPT words per thread, all issued
        const uint32_t n_words = chunk_total * NW;
#pragma unroll
        for (int u = 0; u < WPT; ++u) {
            const uint32_t q = (uint32_t)(u * NT + tid);
            const uint32_t qq = q < n_words ? q : (n_words ? n_words - 1 : 0);
            const uint32_t j = qq / NW, part = qq - j * NW;
            const uint32_t g = gpos[j];
            // (ssrc[0] may be stale when the chunk is empty: keep the index in range)
            const uint32_t v = stage[min((uint32_t)ssrc[j], (uint32_t)(CH - 1)) * NW + part];
            uint32_t *dst = (q < n_words && g < out_cap) ? out + (uint64_t)g * NW + part : dummy;
            *dst = v;
        }
        __syncthreads();
    };

    if (!sched.has(0)) return;
    Pieces pc;
    Dests dd;
    load_chunk(pc, dd, sched.begin(0), sched.end(0));
    load_bases(0);
#pragma unroll
    for (int k = 0; k < EPT; ++k) cursor[k] = nbase[k];
    for (uint32_t j = 0; sched.has(j); ++j) {
        if constexpr (Sched::kRebase) {
#pragma unroll
            for (int k = 0; k < EPT; ++k) cursor[k] = nbase[k];
        }
        const bool more = sched.has(j + 1);  // the same for the whole workgroup
        process(pc, dd, [&] {
            if (more) {
                load_chunk(pc, dd, sched.begin(j + 1), sched.end(j + 1));
                if constexpr (Sched::kRebase) load_bases(j + 1);
            }
        });
    }
}

template <int NW, int R, int W, typename RunBase>
__device__ inline void wide_raw_scatter_tile(const uint32_t *__restrict__ items, const int32_t *__restrict__ dest,
                                             uint64_t tstart, uint64_t tend, uint64_t words, int32_t D, int nbits,
                                             RunBase run_base, uint32_t *__restrict__ out, uint64_t out_cap,
                                             uint32_t *__restrict__ dummy, uint32_t *lds)
{
    const TileChunks<W * 64 * R, RunBase> sched{tstart, tend, run_base};
    wide_raw_scatter<NW, R, W>(items, dest, words, D, nbits, sched, out, out_cap, dummy, lds);
}

}  // namespace dev
}  // namespace rafi
