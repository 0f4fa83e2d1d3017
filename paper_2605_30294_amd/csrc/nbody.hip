// Multi-context, multi-phase forwarding: one step of the distributed
// Barnes-Hut N-body code of Sec. 5.5, with the three item types of that
// section's listing in three contexts of their own (particles 40 bytes,
// virtual particles 24 bytes, refinement requests 4 bytes).
//
// A step, all on one stream:
//   1. particle context: half-kick, drift, periodic wrap, and a forward to
//      the domain owning the new position (a range of 30-bit Morton keys);
//   2. each domain's particles put in key order (three stable 10-bit splits
//      of the whole queue by key digit: a domain is a key range);
//   3. the domain hierarchy: Morton cells of level L (runs of one key prefix
//      within a domain) and the domain root, with mass and centre of mass;
//      the domain's bounding box;
//   4. virtual-particle context, first round: every root to every other
//      non-empty domain;
//   5. request context: a receiver keeps a root it accepts (Barnes-Hut
//      acceptance against its own box) and sends a refinement request to
//      the owner of one it does not;
//   6. virtual-particle context, second round: the accepted roots, and each
//      owner's answer to each request: its cells that the requester
//      accepts, and the particles of those it does not. Answers take fixed
//      slots after a prefix sum of their sizes, so the queues are the same
//      on every run;
//   7. forces (the domain's own particles, then its remote list) and the
//      second half-kick.
#include <vector>

#include "internal.h"
#include "ea_device.h"
#include "rafi_device.h"
#include "split_device.h"

namespace rafi {
namespace {

struct NBParticle {
    float pos[3], vel[3], acc[3], mass;
};
struct NBVirtual {
    float pos[3], mass, smax;
    int32_t src;
};
struct NBRequest {
    int32_t sender;
};
static_assert(sizeof(NBParticle) == RAFI_NB_PARTICLE_BYTES, "particle layout");
static_assert(sizeof(NBVirtual) == RAFI_NB_VIRTUAL_BYTES, "virtual particle layout");
static_assert(sizeof(NBRequest) == RAFI_NB_REQUEST_BYTES, "request layout");

struct NBNode {
    float com[3], mass;
    uint32_t first, count;
};
struct NBBox {
    float lo[3], hi[3], size;
};

constexpr int kNBThreads = 256;
constexpr uint32_t kDigitBuckets = 1024;  // 10-bit key digits

// Spread the low 10 bits of v to every third bit.
__device__ inline uint32_t spread3(uint32_t v)
{
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000ffu;
    v = (v | (v << 8)) & 0x0300f00fu;
    v = (v | (v << 4)) & 0x030c30c3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

__device__ inline uint32_t cell_coord(float c)
{
    const int32_t q = (int32_t)(c * 1024.0f);
    return (uint32_t)min(max(q, 0), 1023);
}

__device__ inline uint32_t morton_key(const float p[3])
{
    return spread3(cell_coord(p[0])) | (spread3(cell_coord(p[1])) << 1) | (spread3(cell_coord(p[2])) << 2);
}

// The largest d in [0, D) with K[d] <= key (K[0] = 0).
__device__ inline int32_t key_owner(const uint32_t *__restrict__ K, int32_t D, uint32_t key)
{
    int32_t lo = 0, hi = D - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (K[mid] <= key) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ inline float wrap_unit(float x)
{
    x = x - floorf(x);
    return x < 1.0f ? x : 0.0f;
}

// size^2 < theta^2 d^2, d = distance from c to the box
__device__ inline bool accepts(const float c[3], float size, const NBBox &b, float theta)
{
    float d[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) d[a] = fmaxf(fmaxf(b.lo[a] - c[a], c[a] - b.hi[a]), 0.0f);
    const float d2 = __fmaf_rn(d[2], d[2], __fmaf_rn(d[1], d[1], d[0] * d[0]));
    return size * size < (theta * theta) * d2;
}

// ----------------------------------------------------------- workspace ---
struct NBLayout {
    uint64_t off_tmp, off_digit, off_split, off_offsets, off_summary, off_flags, off_cell_of, off_cell_start,
        off_cells, off_roots, off_boxes, off_dcell, off_acc, off_cnt, off_aoff, off_part, off_counters, bytes;
};

constexpr uint32_t kScanTile = 1024;  // elements per block of the scan helper

NBLayout nb_layout(uint64_t n, int32_t D)
{
    NBLayout L;
    const uint64_t n1 = std::max<uint64_t>(n, 1);
    const uint64_t nr = std::max<uint64_t>((uint64_t)D * (uint64_t)(D > 1 ? D - 1 : 1), 1);
    const uint64_t scan_n = std::max(n1, nr);
    // every split of up to n1 slots fits the bound plan's workspace
    const uint64_t split_bytes = std::max(split_plan_bound(n1, (int32_t)kDigitBuckets, RAFI_NB_PARTICLE_BYTES).bytes,
                                          split_plan_bound(n1, (int32_t)kDigitBuckets, 4).bytes);
    uint64_t o = 0;
    auto take = [&](uint64_t bytes) {
        const uint64_t at = o;
        o += (bytes + 255) / 256 * 256;
        return at;
    };
    L.off_tmp = take(n1 * sizeof(NBParticle));
    L.off_digit = take(n1 * sizeof(int32_t));
    L.off_split = take(split_bytes);
    L.off_offsets = take((kDigitBuckets + 1) * sizeof(uint64_t));
    L.off_summary = take(8 * sizeof(uint64_t));
    L.off_flags = take(n1 * sizeof(uint32_t));
    L.off_cell_of = take(n1 * sizeof(uint32_t));
    L.off_cell_start = take(n1 * sizeof(uint32_t));
    L.off_cells = take(n1 * sizeof(NBNode));
    L.off_roots = take((uint64_t)D * sizeof(NBNode));
    L.off_boxes = take((uint64_t)D * sizeof(NBBox));
    L.off_dcell = take((uint64_t)D * 2 * sizeof(uint32_t));
    L.off_acc = take(nr * sizeof(int32_t));
    L.off_cnt = take(nr * sizeof(uint32_t));
    L.off_aoff = take(nr * sizeof(uint32_t));
    L.off_part = take(((scan_n + kScanTile - 1) / kScanTile + 1) * sizeof(uint32_t));
    L.off_counters = take(4 * sizeof(uint32_t));
    L.bytes = o;
    return L;
}

template <typename T>
T *at(void *ws, uint64_t off)
{
    return reinterpret_cast<T *>(static_cast<char *>(ws) + off);
}

// ------------------------------------------------- exclusive scan, u32 ---
// out[i] = sum of in[0..i); *total = the sum of all n. Blocks of kScanTile
// elements scan locally, one block scans the block sums, a last pass adds
// them. n < 2^32 and the sum fits 32 bits.
__global__ void __launch_bounds__(256) scan_tiles_kernel(const uint32_t *__restrict__ in, uint32_t *__restrict__ out,
                                                        uint64_t n, uint32_t *__restrict__ part)
{
    __shared__ uint32_t lds[256 / 64 + 1];
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile + threadIdx.x * 4;
    uint32_t v[4], s = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        v[k] = base + k < n ? in[base + k] : 0u;
        s += v[k];
    }
    uint32_t tot;
    uint32_t run = dev::block_excl_scan<256>(s, lds, &tot);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (base + k < n) out[base + k] = run;
        run += v[k];
    }
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(1024) scan_parts_kernel(uint32_t *__restrict__ part, uint32_t nb,
                                                         uint32_t *__restrict__ total)
{
    __shared__ uint32_t lds[1024 / 64 + 1];
    uint32_t carry = 0;
    for (uint32_t b0 = 0; b0 < nb; b0 += 1024) {
        const uint32_t b = b0 + threadIdx.x;
        const uint32_t v = b < nb ? part[b] : 0u;
        uint32_t tot;
        const uint32_t run = dev::block_excl_scan<1024>(v, lds, &tot);
        if (b < nb) part[b] = carry + run;
        carry += tot;
    }
    if (threadIdx.x == 0) *total = carry;
}

__global__ void __launch_bounds__(256) scan_add_kernel(uint32_t *__restrict__ out, uint64_t n,
                                                      const uint32_t *__restrict__ part)
{
    const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) out[i] += part[i / kScanTile];
}

int scan_u32(const uint32_t *in, uint32_t *out, uint64_t n, uint32_t *part, uint32_t *total, hipStream_t s)
{
    const uint32_t nb = (uint32_t)std::max<uint64_t>(1, (n + kScanTile - 1) / kScanTile);
    hipLaunchKernelGGL(scan_tiles_kernel, dim3(nb), dim3(256), 0, s, in, out, n, part);
    hipLaunchKernelGGL(scan_parts_kernel, dim3(1), dim3(1024), 0, s, part, nb, total);
    if (n) hipLaunchKernelGGL(scan_add_kernel, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, s, out, n, part);
    RAFI_LAUNCH_CHECK();
    return RAFI_OK;
}

// ------------------------------------------------------------- kernels ---
__global__ void __launch_bounds__(kNBThreads) nb_seed_kernel(rafi_device_view P, const uint32_t *__restrict__ K,
                                                            const NBParticle *__restrict__ in, uint64_t n)
{
    const uint64_t i = (uint64_t)blockIdx.x * kNBThreads + threadIdx.x;
    if (i >= n) return;
    const NBParticle p = in[i];
    rafi_forward_t(P, i, p, key_owner(K, P.n_domains, morton_key(p.pos)));
}

__global__ void __launch_bounds__(kNBThreads) nb_drift_kernel(rafi_device_view P, const uint32_t *__restrict__ K,
                                                             float dt, float hdt)
{
    const uint64_t i = (uint64_t)blockIdx.x * kNBThreads + threadIdx.x;
    if (i >= P.n_in) return;
    NBParticle p = static_cast<const NBParticle *>(P.in_items)[i];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        p.vel[a] = __fmaf_rn(hdt, p.acc[a], p.vel[a]);
        p.pos[a] = wrap_unit(__fmaf_rn(dt, p.vel[a], p.pos[a]));
    }
    rafi_forward_t(P, i, p, key_owner(K, P.n_domains, morton_key(p.pos)));
}

__global__ void __launch_bounds__(kNBThreads) nb_key_kernel(const NBParticle *__restrict__ q, uint64_t n,
                                                           uint32_t *__restrict__ key)
{
    const uint64_t i = (uint64_t)blockIdx.x * kNBThreads + threadIdx.x;
    if (i < n) key[i] = morton_key(q[i].pos);
}

__global__ void __launch_bounds__(kNBThreads) nb_key_digit_kernel(const uint32_t *__restrict__ key, uint64_t n,
                                                                 int shift, int32_t *__restrict__ digit)
{
    const uint64_t i = (uint64_t)blockIdx.x * kNBThreads + threadIdx.x;
    if (i < n) digit[i] = (int32_t)((key[i] >> shift) & (kDigitBuckets - 1));
}

// K[0] = 0, K[d] = sorted[d n / D], K[D] = 2^30
__global__ void __launch_bounds__(kNBThreads) nb_pick_kernel(const uint32_t *__restrict__ sorted, uint64_t n,
                                                            int32_t D, uint32_t *__restrict__ K)
{
    const int32_t d = blockIdx.x * kNBThreads + threadIdx.x;
    if (d > D) return;
    K[d] = d == 0 ? 0u : (d == D ? (1u << 30) : sorted[(uint64_t)d * n / (uint64_t)D]);
}

__global__ void __launch_bounds__(kNBThreads) nb_digit_kernel(const NBParticle *__restrict__ q, uint64_t n,
                                                             int shift, int32_t *__restrict__ digit)
{
    const uint64_t i = (uint64_t)blockIdx.x * kNBThreads + threadIdx.x;
    if (i < n) digit[i] = (int32_t)((morton_key(q[i].pos) >> shift) & (kDigitBuckets - 1));
}

// Key order within each domain in one launch: workgroup d sorts its domain's
// (key, queue position) pairs in LDS with a bitonic network (the pairs are
// distinct, so this is exactly the stable sort by key) and gathers the
// particles in that order into dst. For domains of at most kSortMax
// particles; the host takes the three digit passes otherwise.
constexpr uint32_t kSortMax = 8192;
constexpr uint32_t kSortThreads = 1024;

__global__ void __launch_bounds__(kSortThreads) nb_domain_sort_kernel(const NBParticle *__restrict__ src,
                                                                      const uint64_t *__restrict__ off,
                                                                      NBParticle *__restrict__ dst)
{
    __shared__ uint64_t s_key[kSortMax];
    const uint32_t d = blockIdx.x;
    const uint32_t first = (uint32_t)off[d], count = (uint32_t)(off[d + 1] - off[d]);
    uint32_t m = 1;  // a power of two >= count (count <= kSortMax)
    while (m < count) m <<= 1;
    for (uint32_t i = threadIdx.x; i < m; i += kSortThreads)
        s_key[i] = i < count ? ((uint64_t)morton_key(src[first + i].pos) << 32) | i : ~0ull;
    __syncthreads();
    for (uint32_t k = 2; k <= m; k <<= 1)
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            for (uint32_t i = threadIdx.x; i < m; i += kSortThreads) {
                const uint32_t l = i ^ j;
                if (l > i) {
                    const uint64_t a = s_key[i], b = s_key[l];
                    if ((a > b) == ((i & k) == 0)) {
                        s_key[i] = b;
                        s_key[l] = a;
                    }
                }
            }
            __syncthreads();
        }
    for (uint32_t i = threadIdx.x; i < count; i += kSortThreads) dst[first + i] = src[first + (uint32_t)s_key[i]];
}

// flags[i] = 1 where a new cell starts: a new level-L key prefix or a new domain
__global__ void __launch_bounds__(kNBThreads) nb_flag_kernel(const NBParticle *__restrict__ q, uint64_t n,
                                                            const uint32_t *__restrict__ K, int32_t D, int shift,
                                                            uint32_t *__restrict__ flags)
{
    const uint64_t i = (uint64_t)blockIdx.x * kNBThreads + threadIdx.x;
    if (i >= n) return;
    const uint32_t k = morton_key(q[i].pos);
    uint32_t f = 1;
    if (i > 0) {
        const uint32_t kp = morton_key(q[i - 1].pos);
        f = ((k >> shift) != (kp >> shift) || key_owner(K, D, k) != key_owner(K, D, kp)) ? 1u : 0u;
    }
    flags[i] = f;
}

__global__ void __launch_bounds__(kNBThreads) nb_cell_start_kernel(const uint32_t *__restrict__ flags,
                                                                  const uint32_t *__restrict__ cell_of, uint64_t n,
                                                                  uint32_t *__restrict__ cell_start)
{
    const uint64_t i = (uint64_t)blockIdx.x * kNBThreads + threadIdx.x;
    if (i < n && flags[i]) cell_start[cell_of[i]] = (uint32_t)i;
}

// First virtual-particle round: slot s (D - 1) + k carries root s to domain
// r = k (+1 from s on), if both domains hold particles.
__global__ void __launch_bounds__(kNBThreads) nb_roots_kernel(rafi_device_view V, const NBNode *__restrict__ roots,
                                                             const NBBox *__restrict__ boxes, int32_t D)
{
    const uint64_t slot = (uint64_t)blockIdx.x * kNBThreads + threadIdx.x;
    const uint64_t n = (uint64_t)D * (uint64_t)(D - 1);
    if (slot >= n) return;
    const int32_t s = (int32_t)(slot / (uint64_t)(D - 1)), k = (int32_t)(slot % (uint64_t)(D - 1));
    const int32_t r = k < s ? k : k + 1;
    if (roots[s].count == 0 || roots[r].count == 0) {
        rafi_done(V, slot);
        return;
    }
    NBVirtual v;
    v.pos[0] = roots[s].com[0];
    v.pos[1] = roots[s].com[1];
    v.pos[2] = roots[s].com[2];
    v.mass = roots[s].mass;
    v.smax = boxes[s].size;
    v.src = s;
    rafi_forward_t(V, slot, v, r);
}

// A receiver accepts a root or asks its owner for more (request at the same slot).
__global__ void __launch_bounds__(kNBThreads) nb_accept_kernel(rafi_device_view V, rafi_device_view Rq,
                                                              const NBBox *__restrict__ boxes, float theta,
                                                              int32_t *__restrict__ acc)
{
    const uint64_t i = (uint64_t)blockIdx.x * kNBThreads + threadIdx.x;
    if (i >= V.n_in) return;
    const int32_t r = ea::find_domain(V.in_offsets, V.n_domains, i);
    const NBVirtual v = static_cast<const NBVirtual *>(V.in_items)[i];
    const bool a = accepts(v.pos, v.smax, boxes[r], theta);
    acc[i] = a ? 1 : 0;
    if (a) {
        rafi_done(Rq, i);
    } else {
        rafi_forward_t(Rq, i, NBRequest{r}, v.src);
    }
}

// Second virtual-particle round, first n1 slots: the accepted roots stay with their receiver.
__global__ void __launch_bounds__(kNBThreads) nb_keep_kernel(rafi_device_view V, const int32_t *__restrict__ acc)
{
    const uint64_t i = (uint64_t)blockIdx.x * kNBThreads + threadIdx.x;
    if (i >= V.n_in) return;
    if (acc[i]) {
        const int32_t r = ea::find_domain(V.in_offsets, V.n_domains, i);
        rafi_forward_t(V, i, static_cast<const NBVirtual *>(V.in_items)[i], r);
    } else {
        rafi_done(V, i);
    }
}

// ------------------------------------------- one wave per item forms ---
// Wave w handles request w; each lane takes one of the owner's cells, and a
// wave scan of the cells' answer sizes gives every cell its slots, in cell
// order (the same slots as one thread walking the cells).
__device__ inline int32_t wave_id() { return (int32_t)((blockIdx.x * kNBThreads + threadIdx.x) >> 6); }

__global__ void __launch_bounds__(kNBThreads) nb_answer_size_wave_kernel(rafi_device_view Rq,
                                                                        const NBNode *__restrict__ cells,
                                                                        const uint32_t *__restrict__ dcell,
                                                                        const NBBox *__restrict__ boxes, float theta,
                                                                        float csize, uint32_t *__restrict__ cnt)
{
    const uint64_t j = (uint64_t)wave_id();
    if (j >= Rq.n_in) return;  // whole waves
    const int lane = threadIdx.x & 63;
    const int32_t s = ea::find_domain(Rq.in_offsets, Rq.n_domains, j);
    const NBBox b = boxes[static_cast<const NBRequest *>(Rq.in_items)[j].sender];
    uint32_t c = 0;
    for (uint32_t k0 = dcell[2 * s]; k0 < dcell[2 * s + 1]; k0 += 64) {
        const uint32_t k = k0 + lane;
        if (k < dcell[2 * s + 1]) c += accepts(cells[k].com, csize, b, theta) ? 1u : cells[k].count;
    }
    const uint32_t tot = (uint32_t)__builtin_amdgcn_readlane((int)dev::wave_incl_scan(c), 63);
    if (lane == 0) cnt[j] = tot;
}

// Lane o's copy of v (every lane of the wave active).
__device__ inline uint32_t lane_value(uint32_t v, uint32_t o)
{
    return (uint32_t)__builtin_amdgcn_ds_bpermute((int)(o << 2), (int)v);
}

// The answer items of 64 cells at a time (the same slots as the size kernel's
// count, cell by cell): a lane per cell finds each cell's item count and the
// wave scans them; then the wave writes those items 64 at a time, each lane
// finding the cell its item belongs to by a binary search over the scan, so
// an opened cell with many particles is copied by the whole wave.
__global__ void __launch_bounds__(kNBThreads) nb_answer_wave_kernel(rafi_device_view V, rafi_device_view Rq,
                                                                   const NBParticle *__restrict__ q,
                                                                   const NBNode *__restrict__ cells,
                                                                   const uint32_t *__restrict__ dcell,
                                                                   const NBBox *__restrict__ boxes, float theta,
                                                                   float csize, const uint32_t *__restrict__ aoff,
                                                                   uint64_t n1)
{
    const uint64_t j = (uint64_t)wave_id();
    if (j >= Rq.n_in) return;  // whole waves
    const uint32_t lane = threadIdx.x & 63;
    const int32_t s = ea::find_domain(Rq.in_offsets, Rq.n_domains, j);
    const int32_t r = static_cast<const NBRequest *>(Rq.in_items)[j].sender;
    const NBBox b = boxes[r];
    uint64_t base = n1 + aoff[j];
    const uint32_t kend = dcell[2 * s + 1];
    for (uint32_t k0 = dcell[2 * s]; k0 < kend; k0 += 64) {
        const uint32_t k = k0 + lane;
        const bool valid = k < kend;
        NBNode c{};
        if (valid) c = cells[k];
        const bool a = valid && accepts(c.com, csize, b, theta);
        const uint32_t sz = valid ? (a ? 1u : c.count) : 0u;
        const uint32_t incl = dev::wave_incl_scan(sz);
        const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
        // per lane, for the search below: its cell's first item (wave-relative),
        // first particle, and whether it answers with its moments
        const uint32_t first_item = incl - sz, first_particle = c.first, accepted = a ? 1u : 0u;
        for (uint32_t t0 = 0; t0 < total; t0 += 64) {
            const uint32_t t = min(t0 + lane, total - 1);
            // o = number of cells whose items all lie before t: the owner of item t
            uint32_t o = 0;
#pragma unroll
            for (uint32_t st = 32; st > 0; st >>= 1)
                if (lane_value(incl, o + st - 1) <= t) o += st;
            const uint32_t off = t - lane_value(first_item, o);
            const uint32_t p0 = lane_value(first_particle, o), acc = lane_value(accepted, o);
            const uint32_t kk = k0 + o;
            if (t0 + lane >= total) continue;
            NBVirtual v;
            if (acc) {
                const NBNode &cn = cells[kk];
                v.pos[0] = cn.com[0];
                v.pos[1] = cn.com[1];
                v.pos[2] = cn.com[2];
                v.mass = cn.mass;
                v.smax = csize;
            } else {
                const NBParticle &pq = q[p0 + off];
                v.pos[0] = pq.pos[0];
                v.pos[1] = pq.pos[1];
                v.pos[2] = pq.pos[2];
                v.mass = pq.mass;
                v.smax = 0.0f;
            }
            v.src = s;
            rafi_forward_t(V, base + t, v, r);
        }
        base += total;
    }
}

// Workgroup d handles domain d. Its four waves each add one of the moments
// (mass, then mass times x, y, z) over the domain's particles in key order:
// coalesced loads of 64 particles at a time, the next chunk's issued before
// this chunk is summed, each lane taking the values from the lane that holds
// them. Wave 0 also takes the box (a min/max: exact in any order).
template <int A>
__device__ inline float domain_moment(const NBParticle *__restrict__ q, uint32_t first, uint32_t count, int lane,
                                      float lo[3], float hi[3])
{
    float sum = 0.0f;
    float nw = 0.0f, npos[3] = {0.0f, 0.0f, 0.0f};
    if ((uint32_t)lane < count) {
        nw = q[first + lane].mass;
#pragma unroll
        for (int a = 0; a < 3; ++a) npos[a] = q[first + lane].pos[a];
    }
    for (uint32_t c0 = 0; c0 < count; c0 += 64) {
        const float pw = nw, pc = A > 0 ? npos[A - 1] : 0.0f;
        if (A == 0 && c0 + lane < count)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                lo[a] = fminf(lo[a], npos[a]);
                hi[a] = fmaxf(hi[a], npos[a]);
            }
        const uint32_t nx = c0 + 64 + lane;
        if (nx < count) {
            nw = q[first + nx].mass;
#pragma unroll
            for (int a = 0; a < 3; ++a) npos[a] = q[first + nx].pos[a];
        }
        auto add = [&](uint32_t t) {
            const float w = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(pw), t));
            if (A == 0) {
                sum = sum + w;
            } else {
                const float c = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(pc), t));
                sum = __fmaf_rn(w, c, sum);
            }
        };
        if (count - c0 >= 64) {  // a full chunk: straight-line code, constant lanes
#pragma unroll
            for (uint32_t t = 0; t < 64; ++t) add(t);
        } else {
            for (uint32_t t = 0; t < count - c0; ++t) add(t);
        }
    }
    return sum;
}

__global__ void __launch_bounds__(256) nb_domain_kernel(const NBParticle *__restrict__ q,
                                                        const uint64_t *__restrict__ off, int32_t D, uint64_t n,
                                                        const uint32_t *__restrict__ cell_of,
                                                        const uint32_t *__restrict__ n_cells,
                                                        NBNode *__restrict__ roots, NBBox *__restrict__ boxes,
                                                        uint32_t *__restrict__ dcell)
{
    __shared__ float s_sum[4];
    const int32_t d = blockIdx.x;  // the grid has D workgroups
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)), lane = threadIdx.x & 63;
    const uint32_t first = (uint32_t)off[d], count = (uint32_t)(off[d + 1] - off[d]);
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    float sum;
    if (w == 0) sum = domain_moment<0>(q, first, count, lane, lo, hi);
    else if (w == 1) sum = domain_moment<1>(q, first, count, lane, lo, hi);
    else if (w == 2) sum = domain_moment<2>(q, first, count, lane, lo, hi);
    else sum = domain_moment<3>(q, first, count, lane, lo, hi);
    if (lane == 0) s_sum[w] = sum;
    __syncthreads();
    if (w != 0) return;
#pragma unroll
    for (int a = 0; a < 3; ++a)
        for (int o = 32; o > 0; o >>= 1) {
            lo[a] = fminf(lo[a], __shfl_xor(lo[a], o, 64));
            hi[a] = fmaxf(hi[a], __shfl_xor(hi[a], o, 64));
        }
    if (lane != 0) return;
    const float m = s_sum[0], mx = s_sum[1], my = s_sum[2], mz = s_sum[3];
    NBNode r{};
    NBBox b{};
    if (count) {
        r.com[0] = mx / m;
        r.com[1] = my / m;
        r.com[2] = mz / m;
        r.mass = m;
        r.first = first;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            b.lo[a] = lo[a];
            b.hi[a] = hi[a];
        }
        b.size = fmaxf(fmaxf(b.hi[0] - b.lo[0], b.hi[1] - b.lo[1]), b.hi[2] - b.lo[2]);
        dcell[2 * d] = cell_of[first];
        dcell[2 * d + 1] = (uint64_t)first + count < n ? cell_of[first + count] : *n_cells;
    } else {
        dcell[2 * d] = dcell[2 * d + 1] = 0;
    }
    r.count = count;
    roots[d] = r;
    boxes[d] = b;
}

// Chunked force sums. A particle's sources (its domain's particles in key
// order, then its remote list) are cut into chunks of kForceChunk; workgroup
// (tile, chunk) adds one chunk's terms in order from zero for the tile's
// particles (the self term masked, as above) and stores the chunk sum;
// nb_fold_kernel then adds a particle's chunk sums in chunk order. The
// inverse distance is the hardware reciprocal square root (about 1 ulp):
// a float32 sum in any order differs from the exact force by rounding of the
// order of the terms' magnitudes times a few 1e-7, and the pair loop is bound
// by instruction issue, where a correctly rounded root and division cost
// about 25 instructions per pair.
constexpr uint32_t kForceChunk = 1024;

__global__ void __launch_bounds__(kNBThreads) nb_force_chunk_kernel(const NBParticle *__restrict__ q,
                                                                   rafi_device_view P, rafi_device_view V,
                                                                   float eps2, uint64_t n,
                                                                   float *__restrict__ part)
{
    __shared__ float4 src[kNBThreads];
    uint64_t begin, end;
    const int32_t r = rafi_tile(P, blockIdx.x, &begin, &end);
    const uint64_t l0 = P.in_offsets[r], nloc = P.in_offsets[r + 1] - l0;
    const uint64_t v0 = V.in_offsets[r], len = nloc + (V.in_offsets[r + 1] - v0);
    const uint64_t c0 = (uint64_t)blockIdx.y * kForceChunk;
    if (c0 >= len) return;  // whole workgroup
    const uint64_t c1 = min<uint64_t>(c0 + kForceChunk, len);
    const uint64_t i = begin + threadIdx.x;
    const bool mine = i < end;
    const uint64_t ii = mine ? i : begin;
    const float p[3] = {q[ii].pos[0], q[ii].pos[1], q[ii].pos[2]};
    const NBVirtual *rem = static_cast<const NBVirtual *>(V.in_items);
    const int64_t self_k = (int64_t)(i - l0);  // position of the particle itself in the sequence
    float A[3] = {0.0f, 0.0f, 0.0f};
    for (uint64_t t = c0; t < c1; t += kNBThreads) {
        const uint64_t k = t + threadIdx.x;
        __syncthreads();
        if (k < c1) {
            if (k < nloc) {
                const NBParticle &o = q[l0 + k];
                src[threadIdx.x] = make_float4(o.pos[0], o.pos[1], o.pos[2], o.mass);
            } else {
                const NBVirtual &o = rem[v0 + (k - nloc)];
                src[threadIdx.x] = make_float4(o.pos[0], o.pos[1], o.pos[2], o.mass);
            }
        }
        __syncthreads();
        const int cnt = (int)min<uint64_t>(kNBThreads, c1 - t);
        const int self = (int)(self_k - (int64_t)t);
#pragma unroll 4
        for (int k2 = 0; k2 < cnt; ++k2) {
            const float4 sv = src[k2];
            const float dx = sv.x - p[0], dy = sv.y - p[1], dz = sv.z - p[2];
            const float r2 = __fmaf_rn(dz, dz, __fmaf_rn(dy, dy, __fmaf_rn(dx, dx, eps2)));
            const float inv = __builtin_amdgcn_rsqf(r2);
            const float f = sv.w * (inv * inv * inv);
            const float sc = __int_as_float(__float_as_int(f) & -(int32_t)(k2 != self));
            A[0] = __fmaf_rn(sc, dx, A[0]);
            A[1] = __fmaf_rn(sc, dy, A[1]);
            A[2] = __fmaf_rn(sc, dz, A[2]);
        }
    }
    if (mine) {
        float *o = part + ((uint64_t)blockIdx.y * n + i) * 3;
        o[0] = A[0];
        o[1] = A[1];
        o[2] = A[2];
    }
}

__global__ void __launch_bounds__(kNBThreads) nb_fold_kernel(NBParticle *__restrict__ q, const uint64_t *__restrict__ off,
                                                            int32_t D, uint64_t n, rafi_device_view V,
                                                            const float *__restrict__ part, float hdt)
{
    const uint64_t i = (uint64_t)blockIdx.x * kNBThreads + threadIdx.x;
    if (i >= n) return;
    const int32_t r = ea::find_domain(off, D, i);
    const uint64_t len = (off[r + 1] - off[r]) + (V.in_offsets[r + 1] - V.in_offsets[r]);
    float a[3] = {0.0f, 0.0f, 0.0f};
    for (uint64_t c = 0; c * kForceChunk < len; ++c) {
        const float *o = part + (c * n + i) * 3;
        a[0] = a[0] + o[0];
        a[1] = a[1] + o[1];
        a[2] = a[2] + o[2];
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        q[i].acc[k] = a[k];
        q[i].vel[k] = __fmaf_rn(hdt, a[k], q[i].vel[k]);
    }
}

// Workgroup c handles cell c: its four waves each add one of the cell's
// moments (mass, then mass times x, y, z) over its particles in key order from
// zero (the same sums as the domain moments above); then the centre of mass
// is the first moment over the mass.
__global__ void __launch_bounds__(256) nb_cells_kernel(const NBParticle *__restrict__ q, uint64_t n,
                                                       const uint32_t *__restrict__ n_cells,
                                                       const uint32_t *__restrict__ cell_start,
                                                       NBNode *__restrict__ cells)
{
    __shared__ float s_sum[4];
    const uint32_t c = blockIdx.x;
    const uint32_t nc = *n_cells;
    if (c >= nc) return;  // the whole workgroup
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)), lane = threadIdx.x & 63;
    const uint32_t first = cell_start[c];
    const uint32_t count = (c + 1 < nc ? cell_start[c + 1] : (uint32_t)n) - first;
    float lo[3], hi[3];  // unused here
    float sum;
    if (w == 0) sum = domain_moment<0>(q, first, count, lane, lo, hi);
    else if (w == 1) sum = domain_moment<1>(q, first, count, lane, lo, hi);
    else if (w == 2) sum = domain_moment<2>(q, first, count, lane, lo, hi);
    else sum = domain_moment<3>(q, first, count, lane, lo, hi);
    if (lane == 0) s_sum[w] = sum;
    __syncthreads();
    if (threadIdx.x != 0) return;
    const float m = s_sum[0];
    NBNode nd;
    nd.com[0] = s_sum[1] / m;
    nd.com[1] = s_sum[2] / m;
    nd.com[2] = s_sum[3] / m;
    nd.mass = m;
    nd.first = first;
    nd.count = count;
    cells[c] = nd;
}

uint32_t blocks_for(uint64_t n) { return (uint32_t)std::max<uint64_t>(1, (n + kNBThreads - 1) / kNBThreads); }
// blocks that give every one of n items a wave of its own
uint32_t waves_blocks(uint64_t n) { return (uint32_t)std::max<uint64_t>(1, (n + kNBThreads / 64 - 1) / (kNBThreads / 64)); }

bool job_ok(const rafi_nb_job *j)
{
    return j && j->n_domains >= 1 && j->n_domains <= 1024 && j->cell_level >= 1 && j->cell_level <= 10 &&
           j->splitters && j->workspace && j->theta >= 0.0f && j->eps >= 0.0f;
}

}  // namespace
}  // namespace rafi

using namespace rafi;

extern "C" {

int rafi_nb_workspace(uint64_t n_particles, int32_t n_domains, uint64_t *bytes)
{
    if (!bytes || n_domains < 1 || n_domains > 1024 || n_particles >= (1ull << 31)) return RAFI_ERR_ARG;
    *bytes = nb_layout(n_particles, n_domains).bytes;
    return RAFI_OK;
}

int rafi_nb_splitters(const void *particles, uint64_t n, int32_t n_domains, uint32_t *splitters, void *workspace,
                      void *hip_stream)
{
    if (!particles || !splitters || !workspace || n == 0 || n_domains < 1 || n_domains > 1024 ||
        n >= (1ull << 31))
        return RAFI_ERR_ARG;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const NBLayout L = nb_layout(n, n_domains);
    // the keys, in two arrays inside the particle staging area (8 <= 40 bytes per particle)
    uint32_t *ka = at<uint32_t>(workspace, L.off_tmp), *kb = ka + n;
    int32_t *digit = at<int32_t>(workspace, L.off_digit);
    hipLaunchKernelGGL(nb_key_kernel, dim3(blocks_for(n)), dim3(kNBThreads), 0, s,
                       static_cast<const NBParticle *>(particles), n, ka);
    RAFI_LAUNCH_CHECK();
    const SplitPlan plan = split_plan(n, (int32_t)kDigitBuckets, 4);
    uint32_t *src = ka, *dst = kb;
    for (int pass = 0; pass < 3; ++pass) {
        hipLaunchKernelGGL(nb_key_digit_kernel, dim3(blocks_for(n)), dim3(kNBThreads), 0, s, src, n, 10 * pass,
                           digit);
        RAFI_LAUNCH_CHECK();
        const int rc = split_run(plan, src, digit, dst, at<uint64_t>(workspace, L.off_offsets),
                                 at<uint64_t>(workspace, L.off_summary), nullptr, 0,
                                 at<void>(workspace, L.off_split), s);
        if (rc != RAFI_OK) return rc;
        std::swap(src, dst);
    }
    hipLaunchKernelGGL(nb_pick_kernel, dim3(blocks_for((uint64_t)n_domains + 1)), dim3(kNBThreads), 0, s, src, n,
                       n_domains, splitters);
    RAFI_LAUNCH_CHECK();
    return RAFI_OK;
}

int rafi_nb_seed(rafi_ctx *P, const rafi_nb_job *job, const void *particles, uint64_t n)
{
    if (!P || !job_ok(job) || P->S != RAFI_NB_PARTICLE_BYTES || P->D != job->n_domains || n > P->cap ||
        (n && !particles) || n >= (1ull << 31))
        return RAFI_ERR_ARG;
    int rc = rafi_begin(P, n);
    if (rc != RAFI_OK) return rc;
    rafi_device_view v;
    rafi_view(P, &v);
    if (n)
        hipLaunchKernelGGL(nb_seed_kernel, dim3(blocks_for(n)), dim3(kNBThreads), 0, P->stream, v, job->splitters,
                           static_cast<const NBParticle *>(particles), n);
    RAFI_LAUNCH_CHECK();
    uint64_t total = 0;
    return rafi_round(P, nullptr, &total);
}

int rafi_nb_step(rafi_ctx *P, rafi_ctx *V, rafi_ctx *Rq, const rafi_nb_job *job, uint64_t *round_counts,
                 uint64_t *sizes)
{
    if (!P || !V || !Rq || !job_ok(job) || P->S != RAFI_NB_PARTICLE_BYTES || V->S != RAFI_NB_VIRTUAL_BYTES ||
        Rq->S != RAFI_NB_REQUEST_BYTES || P->D != job->n_domains || V->D != job->n_domains ||
        Rq->D != job->n_domains || P->stream != V->stream || P->stream != Rq->stream || P->n_in > job->capacity)
        return RAFI_ERR_ARG;
    const int32_t D = job->n_domains;
    const uint64_t n1_slots = (uint64_t)D * (uint64_t)(D - 1);
    if (V->cap < n1_slots || Rq->cap < n1_slots) return RAFI_ERR_ARG;
    hipStream_t s = P->stream;
    const NBLayout L = nb_layout(job->capacity, D);
    void *ws = job->workspace;
    const float dt = job->dt, hdt = 0.5f * job->dt, eps2 = job->eps * job->eps, theta = job->theta;
    const float csize = ldexpf(1.0f, -job->cell_level);
    const uint64_t n = P->n_in;
    std::vector<uint64_t> own_counts(round_counts ? 0 : (size_t)4 * D);
    uint64_t *counts4 = round_counts ? round_counts : own_counts.data();
    auto counts_at = [&](int k) { return counts4 + (size_t)k * D; };
    const uint64_t *pcount = counts_at(0), *vcount = counts_at(3);

    // 1. kick, drift, wrap; forward each particle to its owner
    int rc = rafi_open(P, n, RAFI_SLOTS_ORDERED);
    if (rc != RAFI_OK) return rc;
    rafi_device_view pv;
    rafi_view(P, &pv);
    if (n)
        hipLaunchKernelGGL(nb_drift_kernel, dim3(blocks_for(n)), dim3(kNBThreads), 0, s, pv, job->splitters, dt, hdt);
    RAFI_LAUNCH_CHECK();
    uint64_t total = 0;
    rc = rafi_round(P, counts_at(0), &total);
    if (rc != RAFI_OK) return rc;
    if (total != n) return RAFI_ERR_BAD_DEST;  // every particle has an owner
    rafi_view(P, &pv);
    NBParticle *q = static_cast<NBParticle *>(const_cast<void *>(pv.in_items));

    // 2. key order within each domain: one sorting workgroup per domain, or
    // three stable passes over 10-bit digits when a domain is too large
    NBParticle *tmp = at<NBParticle>(ws, L.off_tmp);
    int32_t *digit = at<int32_t>(ws, L.off_digit);
    uint64_t largest = 0;
    for (int32_t e = 0; e < D; ++e) largest = std::max(largest, pcount[e]);
    if (n && largest <= kSortMax) {
        hipLaunchKernelGGL(nb_domain_sort_kernel, dim3((uint32_t)D), dim3(kSortThreads), 0, s, q, pv.in_offsets,
                           tmp);
        RAFI_LAUNCH_CHECK();
        RAFI_HIP_CHECK(hipMemcpyAsync(q, tmp, n * sizeof(NBParticle), hipMemcpyDeviceToDevice, s));
    } else if (n) {
        const SplitPlan plan = split_plan(n, (int32_t)kDigitBuckets, RAFI_NB_PARTICLE_BYTES);
        NBParticle *src = q, *dst = tmp;
        for (int pass = 0; pass < 3; ++pass) {
            hipLaunchKernelGGL(nb_digit_kernel, dim3(blocks_for(n)), dim3(kNBThreads), 0, s, src, n, 10 * pass,
                               digit);
            RAFI_LAUNCH_CHECK();
            rc = split_run(plan, src, digit, dst, at<uint64_t>(ws, L.off_offsets), at<uint64_t>(ws, L.off_summary),
                           nullptr, 0, at<void>(ws, L.off_split), s);
            if (rc != RAFI_OK) return rc;
            std::swap(src, dst);
        }
        RAFI_HIP_CHECK(hipMemcpyAsync(q, src, n * sizeof(NBParticle), hipMemcpyDeviceToDevice, s));
    }

    // 3. cells, roots, boxes
    uint32_t *flags = at<uint32_t>(ws, L.off_flags), *cell_of = at<uint32_t>(ws, L.off_cell_of);
    uint32_t *cell_start = at<uint32_t>(ws, L.off_cell_start), *counters = at<uint32_t>(ws, L.off_counters);
    uint32_t *part = at<uint32_t>(ws, L.off_part);
    NBNode *cells = at<NBNode>(ws, L.off_cells), *roots = at<NBNode>(ws, L.off_roots);
    NBBox *boxes = at<NBBox>(ws, L.off_boxes);
    uint32_t *dcell = at<uint32_t>(ws, L.off_dcell);
    if (n) {
        hipLaunchKernelGGL(nb_flag_kernel, dim3(blocks_for(n)), dim3(kNBThreads), 0, s, q, n, job->splitters, D,
                           30 - 3 * job->cell_level, flags);
        RAFI_LAUNCH_CHECK();
        rc = scan_u32(flags, cell_of, n, part, counters, s);
        if (rc != RAFI_OK) return rc;
        hipLaunchKernelGGL(nb_cell_start_kernel, dim3(blocks_for(n)), dim3(kNBThreads), 0, s, flags, cell_of, n,
                           cell_start);
        hipLaunchKernelGGL(nb_cells_kernel, dim3((uint32_t)std::max<uint64_t>(n, 1)), dim3(256), 0, s, q, n,
                           counters, cell_start, cells);
        RAFI_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(nb_domain_kernel, dim3((uint32_t)D), dim3(256), 0, s, q, pv.in_offsets, D, n, cell_of,
                       counters, roots, boxes, dcell);
    RAFI_LAUNCH_CHECK();

    // 4. virtual particles, first round: the roots
    rc = rafi_open(V, n1_slots, RAFI_SLOTS_ORDERED);
    if (rc != RAFI_OK) return rc;
    rafi_device_view vv;
    rafi_view(V, &vv);
    if (n1_slots)
        hipLaunchKernelGGL(nb_roots_kernel, dim3(blocks_for(n1_slots)), dim3(kNBThreads), 0, s, vv, roots, boxes, D);
    RAFI_LAUNCH_CHECK();
    uint64_t n1 = 0;
    rc = rafi_round(V, counts_at(1), &n1);
    if (rc != RAFI_OK) return rc;
    rafi_view(V, &vv);
    if (job->log_vp1 && n1)
        RAFI_HIP_CHECK(hipMemcpyAsync(job->log_vp1, vv.in_items, std::min<uint64_t>(n1, job->log_vp1_cap) *
                                      RAFI_NB_VIRTUAL_BYTES, hipMemcpyDeviceToDevice, s));

    // 5. accept, or request refinement from the root's owner
    int32_t *acc = at<int32_t>(ws, L.off_acc);
    rc = rafi_open(Rq, n1, RAFI_SLOTS_ORDERED);
    if (rc != RAFI_OK) return rc;
    rafi_device_view rv;
    rafi_view(Rq, &rv);
    if (n1)
        hipLaunchKernelGGL(nb_accept_kernel, dim3(blocks_for(n1)), dim3(kNBThreads), 0, s, vv, rv, boxes, theta, acc);
    RAFI_LAUNCH_CHECK();
    uint64_t nr = 0;
    rc = rafi_round(Rq, counts_at(2), &nr);
    if (rc != RAFI_OK) return rc;
    rafi_view(Rq, &rv);

    // 6. answer sizes, their prefix, then the second virtual round
    uint32_t *cnt = at<uint32_t>(ws, L.off_cnt), *aoff = at<uint32_t>(ws, L.off_aoff);
    uint32_t answers = 0;
    if (nr) {
        hipLaunchKernelGGL(nb_answer_size_wave_kernel, dim3(waves_blocks(nr)), dim3(kNBThreads), 0, s, rv, cells,
                           dcell, boxes, theta, csize, cnt);
        RAFI_LAUNCH_CHECK();
        rc = scan_u32(cnt, aoff, nr, part, counters + 1, s);
        if (rc != RAFI_OK) return rc;
        RAFI_HIP_CHECK(hipMemcpyAsync(&answers, counters + 1, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        RAFI_HIP_CHECK(hipStreamSynchronize(s));
    }
    const uint64_t n2_slots = n1 + answers;
    if (n2_slots > V->cap) return RAFI_ERR_OVERFLOW;
    rc = rafi_open(V, n2_slots, RAFI_SLOTS_ORDERED);
    if (rc != RAFI_OK) return rc;
    rafi_view(V, &vv);
    if (n1) hipLaunchKernelGGL(nb_keep_kernel, dim3(blocks_for(n1)), dim3(kNBThreads), 0, s, vv, acc);
    if (nr)
        hipLaunchKernelGGL(nb_answer_wave_kernel, dim3(waves_blocks(nr)), dim3(kNBThreads), 0, s, vv, rv, q, cells,
                           dcell, boxes, theta, csize, aoff, n1);
    RAFI_LAUNCH_CHECK();
    uint64_t n2 = 0;
    rc = rafi_round(V, counts_at(3), &n2);
    if (rc != RAFI_OK) return rc;
    rafi_view(V, &vv);

    // 7. forces in chunks (a workgroup per particle tile and chunk), then
    // the ordered sum of the chunk sums and the second half-kick
    if (n) {
        if (pv.tile_items != (uint32_t)kNBThreads || !pv.n_tiles) return RAFI_ERR_STATE;
        uint64_t chunks = 0;
        for (int32_t d = 0; d < D; ++d)
            chunks = std::max<uint64_t>(chunks, (pcount[d] + vcount[d] + kForceChunk - 1) / kForceChunk);
        float *part = nullptr;
        RAFI_HIP_CHECK(hipMallocAsync(reinterpret_cast<void **>(&part), std::max<uint64_t>(chunks, 1) * n * 3 *
                                      sizeof(float), s));
        if (chunks)
            hipLaunchKernelGGL(nb_force_chunk_kernel, dim3(pv.n_tiles, (uint32_t)chunks), dim3(kNBThreads), 0, s, q,
                               pv, vv, eps2, n, part);
        hipLaunchKernelGGL(nb_fold_kernel, dim3(blocks_for(n)), dim3(kNBThreads), 0, s, q, pv.in_offsets, D, n, vv,
                           part, hdt);
        const hipError_t launched = hipGetLastError();
        const hipError_t freed = hipFreeAsync(part, s);  // freed whatever the launches reported
        if (launched != hipSuccess || freed != hipSuccess) return RAFI_ERR_HIP;
    }
    if (sizes) {
        sizes[0] = n1;
        sizes[1] = nr;
        sizes[2] = n2;
    }
    return RAFI_OK;
}

}  // extern "C"
