// Batched form: many independent emission-absorption scenes advance together,
// one launch per kernel per round for all of them.
//
// Global domain ids are scene-major (dom_base_s + local) and so are global ray
// ids. Items never change scene, so after every forward step scene s's items
// occupy one contiguous run of the queue, and the stable split over all
// global domains equals a *segmented* split: tiles never straddle a scene and
// see at most that scene's domain count of destinations. Concretely, per
// round (all sizes on the device, so the round is captured once in a hipGraph):
//   plan      per scene: its slot run (from the previous offsets), tiles, and
//             its block of the count table (destination-major, tile-minor)
//   hist      per tile: destination counts -> table; per-domain totals
//   scan      exclusive scan of the table = output slot of each (tile, dest)
//   finalize  exclusive scan of the per-domain totals -> new queue offsets
//   scatter   per tile: the staged stable scatter of split_device.h
//   march     persistent kernel over all items of all scenes
#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "ea_device.h"
#include "internal.h"
#include "rafi_device.h"
#include "split_device.h"

namespace rafi {
namespace {

using ea::Geo;
using ea::Item;

constexpr int kMaxSceneDomains = 64;
constexpr int kScanChunk = 4096;  // 256 threads x 16
constexpr int kPartMax = 16384;

// summary words (u64)
enum { S_TOTAL = 0, S_DONE, S_BAD, S_TILES, S_TABLE, S_SLOTS, S_ROUNDS, S_COUNT };

struct BatchDev {
    const rafi_ea_scene *scenes;   // [S]
    const int32_t *dom_scene;      // [Dt]
    const int32_t *scene_dom;      // [S+1] domain prefix
    const uint32_t *scene_ray;     // [S+1] ray prefix
    uint64_t *offsets;             // [Dt+1]
    uint32_t *dom_count;           // [Dt]
    uint32_t *seg_begin, *seg_n;   // [S]
    uint32_t *seg_tiles;           // [S+1]
    uint32_t *seg_table;           // [S+1]
    uint32_t *table;               // [table_cap]
    uint32_t *part;                // [part_cap]
    unsigned long long *summary;   // [S_COUNT]
    void *items_in, *items_out;    // queues
    int32_t *dest;                 // [cap]
    int32_t S, Dt;
    uint32_t tile;                 // split tile (slots)
    uint64_t table_cap;
    uint32_t part_cap;
    float dt, c;
};

// ------------------------------------------------------------- raygen ---
__device__ inline int32_t scene_of_ray(const uint32_t *scene_ray, int32_t S, uint32_t r)
{
    int32_t lo = 0, hi = S;  // last s with scene_ray[s] <= r
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (scene_ray[mid] <= r) lo = mid; else hi = mid;
    }
    return lo;
}

__global__ void __launch_bounds__(256)
batch_raygen_kernel(BatchDev b, const float *__restrict__ volumes, float *__restrict__ image, uint32_t n_rays)
{
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_rays) return;
    const int32_t s = scene_of_ray(b.scene_ray, b.S, r);
    const rafi_ea_scene &sc = b.scenes[s];
    const Geo g = ea::make_geo(sc.n, sc.grid);
    float org[3], dir[3];
    int32_t K, owner = -1;
    ea::ray_setup(sc.view, (int32_t)(r - sc.ray_base), org, dir, &K);
    const int32_t k0 = ea::first_inside(g, org, dir, K, b.dt, &owner);
    Item *out = static_cast<Item *>(b.items_out);
    if (k0 >= 0) {
        out[r] = Item{(int32_t)r, k0, 0.0f, 0.0f};
        b.dest[r] = sc.dom_base + owner;
    } else {
        image[r] = 0.0f;
        b.dest[r] = RAFI_DONE;
    }
}

// Offsets standing for "the previous round" of ray generation: scene s's
// slots are its rays [ray_base_s, ray_base_{s+1}), attributed to its first
// domain. Only the offsets at scene boundaries are read by the planner.
__global__ void batch_seed_offsets_kernel(BatchDev b)
{
    for (int32_t d = blockIdx.x * blockDim.x + threadIdx.x; d <= b.Dt; d += gridDim.x * blockDim.x) {
        if (d == b.Dt) {
            b.offsets[d] = b.scene_ray[b.S];
        } else {
            const int32_t s = b.dom_scene[d];
            b.offsets[d] = d == b.scene_dom[s] ? b.scene_ray[s] : b.scene_ray[s + 1];
        }
    }
    if (blockIdx.x == 0 && threadIdx.x < S_COUNT) b.summary[threadIdx.x] = 0;
}

// --------------------------------------------------------------- plan ---
__global__ void __launch_bounds__(1024)
batch_plan_kernel(BatchDev b)
{
    __shared__ uint32_t lds[1024 / 64 + 1];
    const int32_t per = (b.S + 1023) / 1024;
    const int32_t s0 = threadIdx.x * per;
    uint32_t tiles_local = 0, table_local = 0;
    for (int32_t s = s0; s < min(s0 + per, b.S); ++s) {
        const uint64_t beg = b.offsets[b.scene_dom[s]];
        const uint64_t end = b.offsets[b.scene_dom[s + 1]];
        const uint32_t n = (uint32_t)(end - beg);
        b.seg_begin[s] = (uint32_t)beg;
        b.seg_n[s] = n;
        const uint32_t t = (n + b.tile - 1) / b.tile;
        tiles_local += t;
        table_local += t * (uint32_t)(b.scene_dom[s + 1] - b.scene_dom[s]);
    }
    uint32_t tiles_total, table_total;
    uint32_t tiles_run = dev::block_excl_scan<1024>(tiles_local, lds, &tiles_total);
    uint32_t table_run = dev::block_excl_scan<1024>(table_local, lds, &table_total);
    for (int32_t s = s0; s < min(s0 + per, b.S); ++s) {
        b.seg_tiles[s] = tiles_run;
        b.seg_table[s] = table_run;
        const uint32_t t = (b.seg_n[s] + b.tile - 1) / b.tile;
        tiles_run += t;
        table_run += t * (uint32_t)(b.scene_dom[s + 1] - b.scene_dom[s]);
    }
    if (threadIdx.x == 0) {
        b.seg_tiles[b.S] = tiles_total;
        b.seg_table[b.S] = table_total;
        b.summary[S_TILES] = tiles_total;
        b.summary[S_TABLE] = min((uint64_t)table_total, b.table_cap);
        b.summary[S_SLOTS] = b.offsets[b.Dt];
        b.summary[S_DONE] = 0;
        b.summary[S_BAD] = 0;
    }
}

// Tile t of the round -> scene, local tile, slot range.
struct TileRef {
    int32_t s;
    uint32_t local, ntiles;
    uint64_t begin, end;
};

__device__ inline TileRef tile_ref(const BatchDev &b, uint32_t t)
{
    int32_t lo = 0, hi = b.S;  // last s with seg_tiles[s] <= t
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (b.seg_tiles[mid] <= t) lo = mid; else hi = mid;
    }
    TileRef r;
    r.s = lo;
    r.local = t - b.seg_tiles[lo];
    r.ntiles = b.seg_tiles[lo + 1] - b.seg_tiles[lo];
    r.begin = (uint64_t)b.seg_begin[lo] + (uint64_t)r.local * b.tile;
    r.end = min(r.begin + b.tile, (uint64_t)b.seg_begin[lo] + b.seg_n[lo]);
    return r;
}

// --------------------------------------------------------------- hist ---
__global__ void __launch_bounds__(256)
batch_hist_kernel(BatchDev b)
{
    __shared__ uint32_t h[kMaxSceneDomains + 2];
    const uint32_t t = blockIdx.x;
    if (t >= b.seg_tiles[b.S]) return;
    const TileRef tr = tile_ref(b, t);
    const int32_t dbase = b.scene_dom[tr.s];
    const int32_t D = b.scene_dom[tr.s + 1] - dbase;
    for (int32_t e = threadIdx.x; e < D + 2; e += blockDim.x) h[e] = 0;
    __syncthreads();
    for (uint64_t i = tr.begin + threadIdx.x; i < tr.end; i += blockDim.x) {
        const int32_t d = b.dest[i];
        uint32_t bucket = (uint32_t)D + 1u;  // invalid
        if (d == RAFI_DONE) bucket = (uint32_t)D;
        else if (d >= dbase && d < dbase + D) bucket = (uint32_t)(d - dbase);
        atomicAdd(&h[bucket], 1u);
    }
    __syncthreads();
    const uint64_t tb = b.seg_table[tr.s];
    for (int32_t e = threadIdx.x; e < D; e += blockDim.x) {
        const uint64_t idx = tb + (uint64_t)e * tr.ntiles + tr.local;
        if (idx < b.table_cap) b.table[idx] = h[e];
        if (h[e]) atomicAdd(&b.dom_count[dbase + e], h[e]);
    }
    if (threadIdx.x == 0) {
        if (h[D]) atomicAdd(&b.summary[S_DONE], (unsigned long long)h[D]);
        if (h[D + 1]) atomicAdd(&b.summary[S_BAD], (unsigned long long)h[D + 1]);
    }
}

// --------------------------------------------------------------- scan ---
// Exclusive scan of table[0, M) with M read from the device; the grid covers
// the largest table and blocks past M exit.
__device__ inline void load16(const uint32_t *__restrict__ a, uint64_t M, uint64_t base, uint32_t v[16])
{
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = (base + k < M) ? a[base + k] : 0u;
}

__global__ void __launch_bounds__(256)
batch_scan_reduce_kernel(BatchDev b)
{
    __shared__ uint32_t lds[256 / 64 + 1];
    const uint64_t M = b.summary[S_TABLE];
    if ((uint64_t)blockIdx.x * kScanChunk >= M) return;
    uint32_t v[16];
    load16(b.table, M, (uint64_t)blockIdx.x * kScanChunk + threadIdx.x * 16ull, v);
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) s += v[k];
    uint32_t tot;
    dev::block_excl_scan<256>(s, lds, &tot);
    if (threadIdx.x == 0) b.part[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(1024)
batch_scan_partials_kernel(BatchDev b)
{
    __shared__ uint32_t lds[1024 / 64 + 1];
    const uint64_t M = b.summary[S_TABLE];
    const uint32_t nb = (uint32_t)((M + kScanChunk - 1) / kScanChunk);
    const uint32_t base = threadIdx.x * 16;
    uint32_t v[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = (base + k < nb) ? b.part[base + k] : 0u;
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) s += v[k];
    uint32_t tot;
    uint32_t run = dev::block_excl_scan<1024>(s, lds, &tot);
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        if (base + k < nb) b.part[base + k] = run;
        run += v[k];
    }
}

__global__ void __launch_bounds__(256)
batch_scan_apply_kernel(BatchDev b)
{
    __shared__ uint32_t lds[256 / 64 + 1];
    const uint64_t M = b.summary[S_TABLE];
    if ((uint64_t)blockIdx.x * kScanChunk >= M) return;
    const uint64_t base = (uint64_t)blockIdx.x * kScanChunk + threadIdx.x * 16ull;
    uint32_t v[16];
    load16(b.table, M, base, v);
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) s += v[k];
    uint32_t tot;
    uint32_t run = dev::block_excl_scan<256>(s, lds, &tot) + b.part[blockIdx.x];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        if (base + k < M) b.table[base + k] = run;
        run += v[k];
    }
}

// ----------------------------------------------------------- finalize ---
__global__ void __launch_bounds__(1024)
batch_finalize_kernel(BatchDev b)
{
    __shared__ uint32_t lds[1024 / 64 + 1];
    const int32_t per = (b.Dt + 1023) / 1024;
    const int32_t d0 = threadIdx.x * per;
    uint32_t local = 0;
    for (int32_t d = d0; d < min(d0 + per, b.Dt); ++d) local += b.dom_count[d];
    uint32_t total;
    uint32_t run = dev::block_excl_scan<1024>(local, lds, &total);
    for (int32_t d = d0; d < min(d0 + per, b.Dt); ++d) {
        b.offsets[d] = run;
        run += b.dom_count[d];
        b.dom_count[d] = 0;
    }
    if (threadIdx.x == 0) {
        b.offsets[b.Dt] = total;
        b.summary[S_TOTAL] = total;
        if (total) b.summary[S_ROUNDS] += 1;
    }
}

// ------------------------------------------------------------ scatter ---
constexpr int kNW = RAFI_EA_ITEM_BYTES / 4;
constexpr int kR = 4, kW = 4;  // 1024-slot chunks, four workgroups per CU

__global__ void __launch_bounds__(64 * kW, 4)
batch_scatter_kernel(BatchDev b, uint64_t cap)
{
    extern __shared__ __align__(16) uint32_t lds[];
    const uint32_t t = blockIdx.x;
    if (t >= b.seg_tiles[b.S]) return;
    const TileRef tr = tile_ref(b, t);
    const int32_t dbase = b.scene_dom[tr.s];
    const int32_t D = b.scene_dom[tr.s + 1] - dbase;
    int nbits = 1;
    while ((1 << nbits) < D) ++nbits;
    const uint64_t tb = b.seg_table[tr.s];
    const uint32_t *table = b.table;
    const uint64_t tcap = b.table_cap;
    dev::staged_scatter_tile<kNW, kR, kW>(
        static_cast<const uint32_t *>(b.items_out), b.dest, tr.begin, tr.end, D, dbase, nbits,
        [&](int32_t e) {
            const uint64_t idx = tb + (uint64_t)e * tr.ntiles + tr.local;
            return idx < tcap ? table[idx] : 0xffffffffu;
        },
        static_cast<uint32_t *>(b.items_in), cap, lds);
}

// -------------------------------------------------------------- march ---
__global__ void batch_march_kernel(BatchDev b, const float *__restrict__ volumes, float *__restrict__ image,
                                   uint32_t n_rays)
{
    const uint64_t n_in = b.summary[S_TOTAL];
    const Item *in = static_cast<const Item *>(b.items_in);
    Item *out = static_cast<Item *>(b.items_out);
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n_in;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const int32_t d = ea::find_domain(b.offsets, b.Dt, i);
        const int32_t s = b.dom_scene[d];
        const rafi_ea_scene &sc = b.scenes[s];
        Item it = in[i];
        if ((uint32_t)it.ray >= n_rays || (uint32_t)it.ray < sc.ray_base) {  // never for emitted items
            b.dest[i] = RAFI_POISON;
            continue;
        }
        const Geo g = ea::make_geo(sc.n, sc.grid);
        float org[3], dir[3];
        int32_t K;
        ea::ray_setup(sc.view, (int32_t)(it.ray - sc.ray_base), org, dir, &K);
        const int32_t local = ea::march_through(volumes + sc.volume_offset, g, ea::box_of(d - sc.dom_base, g),
                                                org, dir, K, b.dt, b.c, it);
        if (local >= 0) {
            out[i] = it;
            b.dest[i] = sc.dom_base + local;
        } else {
            image[it.ray] = it.I;
            b.dest[i] = RAFI_DONE;
        }
    }
}

}  // namespace
}  // namespace rafi

// ------------------------------------------------------------------ host ---
struct rafi_batch {
    hipStream_t stream = nullptr;
    int32_t S = 0, Dt = 0;
    uint64_t n_rays = 0;
    float dt = 0.5f, c = 0.025f;
    std::vector<rafi_ea_scene> scenes;
    std::vector<uint32_t> rays_per_scene;
    rafi_batch_tuning tune{4096, 256, 2048, 1, 4};
    // device
    rafi_ea_scene *d_scenes = nullptr;
    int32_t *d_dom_scene = nullptr, *d_scene_dom = nullptr;
    uint32_t *d_scene_ray = nullptr;
    uint64_t *d_offsets = nullptr;
    uint32_t *d_dom_count = nullptr, *d_seg = nullptr, *d_table = nullptr, *d_part = nullptr;
    unsigned long long *d_summary = nullptr;
    void *d_buf[2] = {nullptr, nullptr};
    int32_t *d_dest = nullptr;
    uint64_t *h_summary = nullptr;
    uint64_t table_cap = 0;
    uint32_t part_cap = 0, tiles_cap = 0;
    // captured round
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    const float *graph_volumes = nullptr;
    float *graph_image = nullptr;
    hipStream_t graph_stream = nullptr;
    rafi_batch_tuning graph_tune{};
};

namespace rafi {
namespace {

BatchDev make_dev(rafi_batch *b)
{
    BatchDev d;
    d.scenes = b->d_scenes;
    d.dom_scene = b->d_dom_scene;
    d.scene_dom = b->d_scene_dom;
    d.scene_ray = b->d_scene_ray;
    d.offsets = b->d_offsets;
    d.dom_count = b->d_dom_count;
    d.seg_begin = b->d_seg;
    d.seg_n = b->d_seg + b->S;
    d.seg_tiles = b->d_seg + 2 * b->S;
    d.seg_table = b->d_seg + 3 * b->S + 1;
    d.table = b->d_table;
    d.part = b->d_part;
    d.summary = b->d_summary;
    d.items_in = b->d_buf[0];
    d.items_out = b->d_buf[1];
    d.dest = b->d_dest;
    d.S = b->S;
    d.Dt = b->Dt;
    d.tile = b->tune.split_tile;
    d.table_cap = b->table_cap;
    d.part_cap = b->part_cap;
    d.dt = b->dt;
    d.c = b->c;
    return d;
}

void free_graph(rafi_batch *b)
{
    if (b->graph_exec) (void)hipGraphExecDestroy(b->graph_exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->graph_exec = nullptr;
    b->graph = nullptr;
}

// Sizes that bound every round for the current tile size.
int size_workspace(rafi_batch *b)
{
    uint64_t tiles = 0, table = 0;
    for (int32_t s = 0; s < b->S; ++s) {
        const uint64_t t = (b->rays_per_scene[s] + b->tune.split_tile - 1) / b->tune.split_tile;
        tiles += t;
        table += t * (uint64_t)(b->scenes[s].grid[0] * b->scenes[s].grid[1] * b->scenes[s].grid[2]);
    }
    const uint32_t parts = (uint32_t)((table + kScanChunk - 1) / kScanChunk);
    if (parts > (uint32_t)kPartMax || table >= (1ull << 32)) return RAFI_ERR_ARG;
    if (table > b->table_cap) {
        if (b->d_table) (void)hipFree(b->d_table);
        b->d_table = nullptr;
        if (hipMalloc(reinterpret_cast<void **>(&b->d_table), std::max<uint64_t>(table, 1) * 4) != hipSuccess)
            return RAFI_ERR_OOM;
        b->table_cap = table;
    }
    if (parts > b->part_cap) {
        if (b->d_part) (void)hipFree(b->d_part);
        b->d_part = nullptr;
        if (hipMalloc(reinterpret_cast<void **>(&b->d_part), std::max<uint32_t>(parts, 1) * 4) != hipSuccess)
            return RAFI_ERR_OOM;
        b->part_cap = parts;
    }
    b->tiles_cap = (uint32_t)tiles;
    return RAFI_OK;
}

// All launches of one round on stream st.
int launch_round(rafi_batch *b, const float *volumes, float *image, hipStream_t st)
{
    const BatchDev d = make_dev(b);
    const uint32_t tiles = std::max<uint32_t>(b->tiles_cap, 1);
    const uint32_t scan_blocks = std::max<uint32_t>((uint32_t)((b->table_cap + kScanChunk - 1) / kScanChunk), 1);
    hipLaunchKernelGGL(batch_plan_kernel, dim3(1), dim3(1024), 0, st, d);
    hipLaunchKernelGGL(batch_hist_kernel, dim3(tiles), dim3(256), 0, st, d);
    hipLaunchKernelGGL(batch_scan_reduce_kernel, dim3(scan_blocks), dim3(256), 0, st, d);
    hipLaunchKernelGGL(batch_scan_partials_kernel, dim3(1), dim3(1024), 0, st, d);
    hipLaunchKernelGGL(batch_scan_apply_kernel, dim3(scan_blocks), dim3(256), 0, st, d);
    hipLaunchKernelGGL(batch_finalize_kernel, dim3(1), dim3(1024), 0, st, d);
    const size_t lds = dev::staged_lds_bytes<kNW, kR, kW>(kMaxSceneDomains);
    hipLaunchKernelGGL(batch_scatter_kernel, dim3(tiles), dim3(64 * kW), lds, st, d, (uint64_t)b->n_rays);
    hipLaunchKernelGGL(batch_march_kernel, dim3(b->tune.march_grid), dim3(b->tune.march_block), 0, st, d, volumes,
                       image, (uint32_t)b->n_rays);
    RAFI_LAUNCH_CHECK();
    return RAFI_OK;
}

bool same_tuning(const rafi_batch_tuning &a, const rafi_batch_tuning &b)
{
    return std::memcmp(&a, &b, sizeof(a)) == 0;
}

int ensure_graph(rafi_batch *b, const float *volumes, float *image)
{
    if (b->graph_exec && b->graph_volumes == volumes && b->graph_image == image && b->graph_stream == b->stream &&
        same_tuning(b->graph_tune, b->tune))
        return RAFI_OK;
    free_graph(b);
    // capture on a private stream, then replay on the batch's stream
    hipStream_t cap = nullptr;
    RAFI_HIP_CHECK(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    int rc = RAFI_OK;
    if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) rc = RAFI_ERR_HIP;
    if (rc == RAFI_OK) {
        rc = launch_round(b, volumes, image, cap);
        hipGraph_t g = nullptr;
        if (hipStreamEndCapture(cap, &g) != hipSuccess) rc = RAFI_ERR_HIP;
        b->graph = g;
    }
    if (rc == RAFI_OK && hipGraphInstantiate(&b->graph_exec, b->graph, nullptr, nullptr, 0) != hipSuccess)
        rc = RAFI_ERR_HIP;
    (void)hipStreamDestroy(cap);
    if (rc != RAFI_OK) {
        (void)hipGetLastError();
        free_graph(b);
        return rc;
    }
    b->graph_volumes = volumes;
    b->graph_image = image;
    b->graph_stream = b->stream;
    b->graph_tune = b->tune;
    return RAFI_OK;
}

void destroy_batch(rafi_batch *b)
{
    if (!b) return;
    (void)hipStreamSynchronize(b->stream);
    free_graph(b);
    void *ptrs[] = {b->d_scenes, b->d_dom_scene, b->d_scene_dom, b->d_scene_ray, b->d_offsets, b->d_dom_count,
                    b->d_seg, b->d_table, b->d_part, b->d_summary, b->d_buf[0], b->d_buf[1], b->d_dest};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    if (b->h_summary) (void)hipHostFree(b->h_summary);
    delete b;
}

}  // namespace
}  // namespace rafi

using namespace rafi;

extern "C" {

int rafi_batch_create(rafi_ea_scene *scenes, int32_t n_scenes, float dt, float c, rafi_batch **out)
{
    if (!out || !scenes || n_scenes < 1 || n_scenes > 65535 || !(dt > 0.0f)) return RAFI_ERR_ARG;
    *out = nullptr;
    std::vector<int32_t> dom_scene, scene_dom(n_scenes + 1), scene_ray_v;
    std::vector<uint32_t> scene_ray(n_scenes + 1), rays(n_scenes);
    uint64_t R = 0;
    int32_t Dt = 0;
    for (int32_t s = 0; s < n_scenes; ++s) {
        rafi_ea_scene &sc = scenes[s];
        if (sc.n < 2 || sc.view.width < 1 || sc.view.height < 1 || sc.view.n_samples < 0) return RAFI_ERR_ARG;
        int32_t D = 1;
        for (int a = 0; a < 3; ++a) {
            if (sc.grid[a] < 1 || sc.n % sc.grid[a] != 0) return RAFI_ERR_ARG;
            D *= sc.grid[a];
        }
        if (D > kMaxSceneDomains) return RAFI_ERR_ARG;
        sc.ray_base = (uint32_t)R;
        sc.dom_base = Dt;
        scene_ray[s] = (uint32_t)R;
        scene_dom[s] = Dt;
        rays[s] = (uint32_t)((uint64_t)sc.view.width * sc.view.height);
        R += rays[s];
        for (int32_t k = 0; k < D; ++k) dom_scene.push_back(s);
        Dt += D;
        if (R >= (1ull << 31)) return RAFI_ERR_ARG;
    }
    scene_ray[n_scenes] = (uint32_t)R;
    scene_dom[n_scenes] = Dt;

    rafi_batch *b = new (std::nothrow) rafi_batch();
    if (!b) return RAFI_ERR_OOM;
    b->S = n_scenes;
    b->Dt = Dt;
    b->n_rays = R;
    b->dt = dt;
    b->c = c;
    b->scenes.assign(scenes, scenes + n_scenes);
    b->rays_per_scene = rays;
    const uint64_t cap = std::max<uint64_t>(R, 1);
    bool ok = hipMalloc(reinterpret_cast<void **>(&b->d_scenes), sizeof(rafi_ea_scene) * n_scenes) == hipSuccess &&
              hipMalloc(reinterpret_cast<void **>(&b->d_dom_scene), sizeof(int32_t) * Dt) == hipSuccess &&
              hipMalloc(reinterpret_cast<void **>(&b->d_scene_dom), sizeof(int32_t) * (n_scenes + 1)) == hipSuccess &&
              hipMalloc(reinterpret_cast<void **>(&b->d_scene_ray), sizeof(uint32_t) * (n_scenes + 1)) == hipSuccess &&
              hipMalloc(reinterpret_cast<void **>(&b->d_offsets), sizeof(uint64_t) * (Dt + 1)) == hipSuccess &&
              hipMalloc(reinterpret_cast<void **>(&b->d_dom_count), sizeof(uint32_t) * Dt) == hipSuccess &&
              hipMalloc(reinterpret_cast<void **>(&b->d_seg), sizeof(uint32_t) * (4 * (size_t)n_scenes + 2)) == hipSuccess &&
              hipMalloc(reinterpret_cast<void **>(&b->d_summary), sizeof(unsigned long long) * S_COUNT) == hipSuccess &&
              hipMalloc(&b->d_buf[0], cap * RAFI_EA_ITEM_BYTES) == hipSuccess &&
              hipMalloc(&b->d_buf[1], cap * RAFI_EA_ITEM_BYTES) == hipSuccess &&
              hipMalloc(reinterpret_cast<void **>(&b->d_dest), cap * sizeof(int32_t)) == hipSuccess &&
              hipHostMalloc(reinterpret_cast<void **>(&b->h_summary), sizeof(uint64_t) * S_COUNT,
                            hipHostMallocDefault) == hipSuccess;
    int rc = ok ? RAFI_OK : RAFI_ERR_OOM;
    if (rc == RAFI_OK) rc = size_workspace(b);
    if (rc == RAFI_OK) {
        ok = hipMemcpy(b->d_scenes, scenes, sizeof(rafi_ea_scene) * n_scenes, hipMemcpyHostToDevice) == hipSuccess &&
             hipMemcpy(b->d_dom_scene, dom_scene.data(), sizeof(int32_t) * Dt, hipMemcpyHostToDevice) == hipSuccess &&
             hipMemcpy(b->d_scene_dom, scene_dom.data(), sizeof(int32_t) * (n_scenes + 1), hipMemcpyHostToDevice) ==
                 hipSuccess &&
             hipMemcpy(b->d_scene_ray, scene_ray.data(), sizeof(uint32_t) * (n_scenes + 1), hipMemcpyHostToDevice) ==
                 hipSuccess &&
             hipMemset(b->d_dom_count, 0, sizeof(uint32_t) * Dt) == hipSuccess &&
             hipDeviceSynchronize() == hipSuccess;
        if (!ok) rc = RAFI_ERR_HIP;
    }
    if (rc != RAFI_OK) {
        (void)hipGetLastError();
        destroy_batch(b);
        return rc;
    }
    *out = b;
    return RAFI_OK;
}

void rafi_batch_destroy(rafi_batch *b) { destroy_batch(b); }

int rafi_batch_set_stream(rafi_batch *b, void *hip_stream)
{
    if (!b) return RAFI_ERR_ARG;
    b->stream = static_cast<hipStream_t>(hip_stream);
    return RAFI_OK;
}

int rafi_batch_set_tuning(rafi_batch *b, const rafi_batch_tuning *t)
{
    if (!b || !t) return RAFI_ERR_ARG;
    if (t->split_tile < 1024 || t->split_tile % 256 != 0 || t->march_grid < 1 || t->march_grid > 65535 ||
        t->rounds_per_sync < 1)
        return RAFI_ERR_ARG;
    if (t->march_block != 64 && t->march_block != 128 && t->march_block != 256 && t->march_block != 512)
        return RAFI_ERR_ARG;
    RAFI_HIP_CHECK(hipStreamSynchronize(b->stream));
    const rafi_batch_tuning old = b->tune;
    b->tune = *t;
    const int rc = size_workspace(b);
    if (rc != RAFI_OK) {
        b->tune = old;
        size_workspace(b);
        return rc;
    }
    return RAFI_OK;
}

int rafi_batch_info(const rafi_batch *b, uint64_t *n_rays, int32_t *n_domains)
{
    if (!b) return RAFI_ERR_ARG;
    if (n_rays) *n_rays = b->n_rays;
    if (n_domains) *n_domains = b->Dt;
    return RAFI_OK;
}

int rafi_batch_render(rafi_batch *b, const float *volumes, float *image, int32_t max_rounds, int32_t *rounds)
{
    if (!b || !volumes || !image || max_rounds < 1) return RAFI_ERR_ARG;
    const BatchDev d = make_dev(b);
    hipLaunchKernelGGL(batch_seed_offsets_kernel, dim3(std::max<int32_t>((b->Dt + 256) / 256, 1)), dim3(256), 0,
                       b->stream, d);
    if (b->n_rays)
        hipLaunchKernelGGL(batch_raygen_kernel, dim3((uint32_t)((b->n_rays + 255) / 256)), dim3(256), 0, b->stream,
                           d, volumes, image, (uint32_t)b->n_rays);
    RAFI_LAUNCH_CHECK();
    if (b->tune.use_graph) {
        int rc = ensure_graph(b, volumes, image);
        if (rc != RAFI_OK) return rc;
    }
    int32_t launched = 0;
    for (;;) {
        for (int k = 0; k < b->tune.rounds_per_sync && launched < max_rounds; ++k, ++launched) {
            if (b->tune.use_graph) {
                RAFI_HIP_CHECK(hipGraphLaunch(b->graph_exec, b->stream));
            } else {
                int rc = launch_round(b, volumes, image, b->stream);
                if (rc != RAFI_OK) return rc;
            }
        }
        RAFI_HIP_CHECK(hipMemcpyAsync(b->h_summary, b->d_summary, sizeof(uint64_t) * S_COUNT, hipMemcpyDeviceToHost,
                                      b->stream));
        RAFI_HIP_CHECK(hipStreamSynchronize(b->stream));
        if (b->h_summary[S_TOTAL] == 0) break;
        if (launched >= max_rounds) {
            if (rounds) *rounds = (int32_t)b->h_summary[S_ROUNDS] + 1;
            return RAFI_ERR_MAX_ROUNDS;
        }
    }
    if (rounds) *rounds = (int32_t)b->h_summary[S_ROUNDS] + 1;
    return b->h_summary[S_BAD] ? RAFI_ERR_BAD_DEST : RAFI_OK;
}

}  // extern "C"
