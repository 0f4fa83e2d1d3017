// Emission-absorption ray march over bricked domains: ray generation (round
// 0), the brick kernel that advances rays through their current brick and
// forwards them at its boundary (the VoPaT / Lander pattern, Sec. 5.1-5.2:
// each forwarded ray carries its partial integration state), and the adjoint
// that replays every ray backwards through the same bricks. The per-sample
// arithmetic is in ea_device.h.
#include <algorithm>

#include "ea_device.h"
#include "internal.h"
#include "rafi_device.h"

namespace rafi {
namespace {

using ea::Box;
using ea::Geo;
using ea::Item;
using ea::Tri;

__device__ inline Geo job_geo(const rafi_ea_job &j) { return ea::make_geo(j.n, j.grid); }

__device__ inline void job_ray(const rafi_ea_job &j, int32_t ray, float org[3], float dir[3], int32_t *K)
{
    const int32_t per = j.width * j.height;
    const int32_t v = ray / per;
    ea::ray_setup(j.views[v], ray - v * per, org, dir, K);
}

__device__ inline void log_visit(const rafi_ea_job &j, int32_t ray, int32_t d)
{
    if (!j.visit_log) return;
    const int32_t c = j.visit_count[ray];
    if (c < j.visit_stride) j.visit_log[(int64_t)ray * j.visit_stride + c] = d;
    j.visit_count[ray] = c + 1;
}

// ------------------------------------------------------------- raygen ---
__global__ void __launch_bounds__(256)
raygen_kernel(rafi_device_view view, rafi_ea_job job, uint64_t n_rays)
{
    const uint64_t r = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (r >= n_rays) return;
    const Geo g = job_geo(job);
    float org[3], dir[3];
    int32_t K, owner = -1;
    job_ray(job, (int32_t)r, org, dir, &K);
    const int32_t k0 = ea::first_inside(g, org, dir, K, job.dt, &owner);
    if (job.visit_count) job.visit_count[r] = 0;
    if (k0 >= 0) {
        if (job.kfirst) job.kfirst[r] = k0;
        rafi_forward_t(view, r, Item{(int32_t)r, k0, 0.0f, 0.0f}, owner);
    } else {
        if (job.kfirst) job.kfirst[r] = 0;
        job.image[r] = 0.0f;
        if (job.tau) job.tau[r] = 0.0f;
        if (job.klast) job.klast[r] = 0;
        rafi_done(view, r);
    }
}

// Emission of a marched ray from input slot i: to its own output slot, or
// appended (rafi_open append mode, where every slot starts as RAFI_DONE).
__device__ inline void emit_item(const rafi_device_view &view, const rafi_ea_job &job, uint64_t i, const Item &it,
                                 int32_t dest)
{
    if (job.emit_mode == RAFI_SLOTS_APPEND) rafi_emit_t(view, it, dest);
    else rafi_forward_t(view, i, it, dest);
}

// A ray leaving brick d: forwarded to `dest`, or finished (dest < 0) with its
// integral, optical depth and end sample written out.
__device__ inline void emit_ray(const rafi_device_view &view, const rafi_ea_job &job, uint64_t i, const Item &it,
                                int32_t dest)
{
    if (dest >= 0) {
        emit_item(view, job, i, it, dest);
        return;
    }
    job.image[it.ray] = it.I;
    if (job.tau) job.tau[it.ray] = it.tau;
    if (job.klast) job.klast[it.ray] = it.k;
    if (job.emit_mode != RAFI_SLOTS_APPEND) rafi_done(view, i);
}

// ------------------------------------------------------------- march ----
// One lane per ray. A wave marches until the longest chord among its 64 rays
// ends, so each workgroup first orders its rays by the samples each has left
// in its brick (a counting sort through LDS), where chords can differ and
// unless they all fall in one bucket. Every ray is marched as if alone and written to its own output
// slot, so results do not depend on the lane.
__global__ void __launch_bounds__(256)
march_kernel(rafi_device_view view, rafi_ea_job job, uint32_t n_rays)
{
    constexpr uint32_t kThreads = 256, kWaves = kThreads / 64, kBuckets = 16;
    __shared__ Item s_item[kThreads];
    __shared__ uint32_t s_slot[kThreads];
    __shared__ int32_t s_d[kThreads];
    __shared__ uint32_t s_cnt[kWaves][kBuckets];
    // the grid may be sized for an upper bound: number the live workgroups only
    const uint64_t n_in = rafi_queue_length(view);
    const uint32_t nb = (uint32_t)((n_in + kThreads - 1) / kThreads);
    if (blockIdx.x >= nb) return;
    const uint32_t t = threadIdx.x, w = t >> 6, lane = t & 63;
    const uint64_t base = rafi_xcd_block(blockIdx.x, nb) * (uint64_t)kThreads;
    const Geo g = job_geo(job);
    uint64_t slot = base + t;
    int32_t d = 0;
    Item it{};
    uint32_t key = kBuckets - 1;
    // Order the lanes only where chords can differ much: bricks whose chord
    // can exceed 64 samples, and rays not along an axis (the same decision in
    // every thread, taken from the workgroup's first ray; any choice gives the
    // same results).
    bool order = (float)(g.b0 + g.b1 + g.b2) >= 64.0f * job.dt;
    if (order) {
        const int32_t r0 = static_cast<const Item *>(view.in_items)[base].ray;
        if ((uint32_t)r0 < n_rays) {
            const float *dir0 = job.views[r0 / (job.width * job.height)].dir;
            order = (dir0[0] != 0.0f) + (dir0[1] != 0.0f) + (dir0[2] != 0.0f) > 1;
        }
    }
    if (!order) {
        if (slot >= n_in) return;
        d = ea::find_domain(view.in_offsets, view.n_domains, slot);
        it = static_cast<const Item *>(view.in_items)[slot];
        if ((uint32_t)it.ray >= n_rays) {  // never true for items this library emitted
            emit_item(view, job, slot, it, RAFI_POISON);
            return;
        }
        log_visit(job, it.ray, d);
        float org[3], dir[3];
        int32_t K;
        job_ray(job, it.ray, org, dir, &K);
        const int32_t dest = ea::march_through(job.volume, g, ea::box_of(d, g), org, dir, K, job.dt, job.c, it);
        emit_ray(view, job, slot, it, dest);
        return;
    }
    if (slot < n_in) {
        d = ea::find_domain(view.in_offsets, view.n_domains, slot);
        it = static_cast<const Item *>(view.in_items)[slot];
        if ((uint32_t)it.ray >= n_rays) {  // never true for items this library emitted
            emit_item(view, job, slot, it, RAFI_POISON);
        } else {
            // samples left in the brick along a straight line (an estimate: it
            // only orders the lanes)
            float org[3], dir[3];
            int32_t K;
            job_ray(job, it.ray, org, dir, &K);
            const Box box = ea::box_of(d, g);
            const float lo[3] = {box.lo0, box.lo1, box.lo2}, hi[3] = {box.hi0, box.hi1, box.hi2};
            float texit = 3.0e38f;
#pragma unroll
            for (int a = 0; a < 3; ++a)
                if (dir[a] != 0.0f)
                    texit = fminf(texit, ((dir[a] > 0.0f ? hi[a] : lo[a]) - org[a]) * __builtin_amdgcn_rcpf(dir[a]));
            const float span = (float)(g.b0 + g.b1 + g.b2) * __builtin_amdgcn_rcpf(job.dt);
            const float left = fminf(texit * __builtin_amdgcn_rcpf(job.dt) - 0.5f - (float)it.k, (float)(K - it.k));
            key = (uint32_t)fminf(fmaxf(left * ((float)(kBuckets - 1) / span), 0.0f), (float)(kBuckets - 2));
        }
    }
    // Stable counting sort of the workgroup's lanes by key, through LDS: lanes
    // with a similar number of samples left share a wave.
    uint32_t rank = 0;
#pragma unroll
    for (uint32_t k = 0; k < kBuckets; ++k) {
        const uint64_t m = __ballot(key == k);
        if (lane == 0) s_cnt[w][k] = (uint32_t)__popcll(m);
        if (key == k) rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
    }
    __syncthreads();
    uint32_t pos = rank, n_live = 0, n_full = 0;
    for (uint32_t k = 0; k < kBuckets; ++k) {
        uint32_t tot = 0;
#pragma unroll
        for (uint32_t ww = 0; ww < kWaves; ++ww) {
            const uint32_t c = s_cnt[ww][k];
            pos += (k < key || (k == key && ww < w)) ? c : 0;
            tot += c;
        }
        n_live += k < kBuckets - 1 ? tot : 0;
        n_full += (k < kBuckets - 1 && tot > 0) ? 1 : 0;
    }
    // One bucket (or none) holds every live ray: the order stays (the same
    // decision in every thread, so the barrier below is met by all or none).
    if (n_full > 1) {
        s_item[pos] = it;
        s_slot[pos] = (uint32_t)(slot - base);
        s_d[pos] = d;
        __syncthreads();
        if (t >= n_live) return;  // no barrier follows
        it = s_item[t];
        slot = base + s_slot[t];
        d = s_d[t];
    } else if (key == kBuckets - 1) {
        return;
    }
    log_visit(job, it.ray, d);
    float org[3], dir[3];
    int32_t K;
    job_ray(job, it.ray, org, dir, &K);
    const int32_t dest = ea::march_through(job.volume, g, ea::box_of(d, g), org, dir, K, job.dt, job.c, it);
    emit_ray(view, job, slot, it, dest);
}

// LDS-staged march: one workgroup per domain-pure tile of the input queue
// stages its brick's densities (plus a one-voxel rim) in LDS once and marches
// all the tile's rays against it.
constexpr int kMarchLdsThreads = 1024;

__global__ void __launch_bounds__(kMarchLdsThreads)
march_lds_kernel(rafi_device_view view, rafi_ea_job job, uint32_t n_rays)
{
    extern __shared__ float vl[];
    uint64_t tb, te;
    const int32_t d = rafi_tile(view, rafi_xcd_block(blockIdx.x, gridDim.x), &tb, &te);
    const Geo g = job_geo(job);
    const Box box = ea::box_of(d, g);
    const ea::Region reg = ea::region_of(box, g);
    ea::load_region(vl, job.volume, g.n, reg);
    __syncthreads();
    for (uint64_t i = tb + threadIdx.x; i < te; i += blockDim.x) {
        Item it = static_cast<const Item *>(view.in_items)[i];
        if ((uint32_t)it.ray >= n_rays) {
            emit_item(view, job, i, it, RAFI_POISON);
            continue;
        }
        log_visit(job, it.ray, d);
        float org[3], dir[3];
        int32_t K;
        job_ray(job, it.ray, org, dir, &K);
        const int32_t dest = ea::march_through_lds(vl, reg, g, box, org, dir, K, job.dt, job.c, it);
        emit_ray(view, job, i, it, dest);
    }
}

// ----------------------------------------------------------- adjoint ----
// Round 0 of the backward pass: every ray that sampled the volume starts at
// its last inside sample, in that sample's brick, with tau = tau_N, B = 0.
__global__ void __launch_bounds__(256)
bwd_seed_kernel(rafi_device_view view, rafi_ea_job job, uint64_t n_rays)
{
    const uint64_t r = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (r >= n_rays) return;
    if (job.visit_count) job.visit_count[r] = 0;
    const int32_t kl = job.klast[r];
    if (kl <= 0) {
        rafi_done(view, r);
        return;
    }
    const Geo g = job_geo(job);
    float org[3], dir[3];
    int32_t K;
    job_ray(job, (int32_t)r, org, dir, &K);
    float p[3];
    ea::sample_pos(org, dir, job.dt, kl - 1, p);
    rafi_forward_t(view, r, Item{(int32_t)r, kl - 1, job.tau[r], 0.0f}, ea::owner_of(p, g));
}

__device__ inline void scatter8(float *__restrict__ grad, int32_t n, const Tri &t, float s)
{
    const int64_t sy = n, sz = (int64_t)n * n;
    const float gx0 = 1.0f - t.f0, gy0 = 1.0f - t.f1, gz0 = 1.0f - t.f2;
    const float a00 = s * gz0 * gy0, a01 = s * gz0 * t.f1, a10 = s * t.f2 * gy0, a11 = s * t.f2 * t.f1;
    float *b = grad + t.base;
    unsafeAtomicAdd(b, a00 * gx0);
    unsafeAtomicAdd(b + 1, a00 * t.f0);
    unsafeAtomicAdd(b + sy, a01 * gx0);
    unsafeAtomicAdd(b + sy + 1, a01 * t.f0);
    unsafeAtomicAdd(b + sz, a10 * gx0);
    unsafeAtomicAdd(b + sz + 1, a10 * t.f0);
    unsafeAtomicAdd(b + sz + sy, a11 * gx0);
    unsafeAtomicAdd(b + sz + sy + 1, a11 * t.f0);
}

// Walk the ray's samples backwards through its brick:
//   tau <- tau - sigma_k (now the depth in front of k), T = exp(-tau),
//   a = 1 - exp(-sigma_k), dI/drho_k = T (a + c (1 - a)(rho_k - B)),
//   scatter dL/dI * dI/drho_k to the 8 voxels, B <- a rho_k + (1 - a) B.
__global__ void __launch_bounds__(256)
bwd_march_kernel(rafi_device_view view, rafi_ea_job job, const float *__restrict__ grad_image,
                 float *__restrict__ grad, uint32_t n_rays)
{
    // the grid may be sized for an upper bound: number the live workgroups only
    const uint64_t n_in = rafi_queue_length(view);
    const uint32_t nb = (uint32_t)((n_in + blockDim.x - 1) / blockDim.x);
    if (blockIdx.x >= nb) return;
    const uint64_t i = rafi_xcd_block(blockIdx.x, nb) * (uint64_t)blockDim.x + threadIdx.x;
    if (i >= n_in) return;
    const Geo g = job_geo(job);
    const int32_t d = ea::find_domain(view.in_offsets, view.n_domains, i);
    const Box box = ea::box_of(d, g);
    Item it = static_cast<const Item *>(view.in_items)[i];
    if ((uint32_t)it.ray >= n_rays) {
        rafi_forward_t(view, i, it, RAFI_POISON);
        return;
    }
    log_visit(job, it.ray, d);
    float org[3], dir[3];
    int32_t K;
    job_ray(job, it.ray, org, dir, &K);
    const float gI = grad_image[it.ray];
    const float c = job.c;
    float tau = it.tau, ctau = 0.0f, B = it.I;
    int32_t k = it.k;
    int32_t dest = RAFI_DONE;
    ea::Corners cc;
    for (; k >= 0; --k) {
        float p[3];
        ea::sample_pos(org, dir, job.dt, k, p);
        if (!box.contains(p)) {
            dest = ea::owner_of(p, g);
            break;
        }
        const Tri t = ea::tri_setup(g.n, p);
        const float rho = ea::density_cached(job.volume, g.n, t, cc);
        const float sigma = c * rho;
        // compensated tau -= sigma
        const float yt = -sigma - ctau;
        const float tt = tau + yt;
        ctau = (tt - tau) - yt;
        tau = tt;
        const float T = __expf(-tau);
        const float a = ea::one_minus_exp_neg(sigma);
        const float dIdrho = T * __fmaf_rn(c * (1.0f - a), rho - B, a);
        if (gI != 0.0f) scatter8(grad, g.n, t, gI * dIdrho);
        B = __fmaf_rn(a, rho - B, B);
    }
    it.k = k;
    it.tau = tau - ctau;
    it.I = B;
    if (k >= 0 && dest >= 0) rafi_forward_t(view, i, it, dest);
    else rafi_done(view, i);
}

// LDS-privatised backward: one workgroup per domain-pure tile of the input
// queue. The workgroup accumulates dL/dV for the voxels its brick's samples
// touch -- the brick plus a one-voxel rim, (b+2)^3 floats -- in LDS, and each
// lane first sums its ray's contributions in registers while consecutive
// samples stay in the same trilinear cell. At the end the non-zero LDS
// entries are added to the global gradient.
constexpr int kBwdThreads = 1024;

// Add v to a float in LDS as a compare-and-swap loop on the word's bits: the
// same single rounded float addition as an atomic add, in the same
// unspecified order. On gfx950 the native LDS float32 add (ds_add_f32) costs
// about 200 cycles per full wave, some 3 per active lane, while a 32-bit
// compare-and-swap costs about 27 (measured, 64 distinct words per wave).
__device__ inline void lds_add(float *p, float v)
{
    uint32_t *q = reinterpret_cast<uint32_t *>(p);
    uint32_t old = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    for (;;) {
        uint32_t seen = old;
        if (__hip_atomic_compare_exchange_strong(q, &seen, __float_as_uint(__uint_as_float(old) + v), __ATOMIC_RELAXED,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP))
            return;
        old = seen;
    }
}

// Add acc[q] to the LDS words base[o[q]] for the corners q with fl[q]: every
// word read, then every compare-and-swap issued, then one wait, so a cell
// change pays two LDS round trips instead of two per corner. A corner that
// is not flushed takes a swap of its read value's bits with one bit flipped
// for that same value: it fails, or rewrites the word unchanged. Corners
// whose swap lost a race to another lane are added again one by one.
__device__ inline void lds_add_corners(float *base, const int32_t o[8], const float acc[8], const bool fl[8])
{
    uint32_t *w = reinterpret_cast<uint32_t *>(base);
    uint32_t old[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) old[q] = __hip_atomic_load(w + o[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    // seen[q]: the word as each swap found it (equal to old[q] when it took)
    uint32_t seen[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        seen[q] = fl[q] ? old[q] : old[q] ^ 1u;
        const uint32_t want = fl[q] ? __float_as_uint(__uint_as_float(old[q]) + acc[q]) : seen[q];
        (void)__hip_atomic_compare_exchange_strong(w + o[q], &seen[q], want, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    bool ok[8], all = true;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        ok[q] = !fl[q] || seen[q] == old[q];
        all &= ok[q];
    }
    if (!all) {
#pragma unroll
        for (int q = 0; q < 8; ++q)
            if (!ok[q]) lds_add(base + o[q], acc[q]);
    }
}

// The backward of the queue items [first, last), all in domain d, by the whole
// workgroup: zero the brick's gradient region in LDS, march every ray back
// through the brick accumulating into it, then add its non-zero entries to
// the global gradient. kSmall: the volume has at most kSmallN^3 voxels.
template <bool kSmall>
__device__ inline void bwd_segment(const rafi_device_view &view, const rafi_ea_job &job,
                                   const float *__restrict__ grad_image, float *__restrict__ grad, uint32_t n_rays,
                                   int32_t d, uint64_t first, uint64_t last, float *gl)
{
    const Geo g = job_geo(job);
    const Box box = ea::box_of(d, g);
    const int32_t ox = (int32_t)box.lo0 - 1, oy = (int32_t)box.lo1 - 1, oz = (int32_t)box.lo2 - 1;
    const int32_t ex = g.b0 + 2, ey = g.b1 + 2, ez = g.b2 + 2;
    const int32_t nl = ex * ey * ez, sxy = ex * ey;
    for (int32_t k = threadIdx.x; k < nl; k += blockDim.x) gl[k] = 0.0f;
    __syncthreads();

    const float c = job.c;
    for (uint64_t i = first + threadIdx.x; i < last; i += blockDim.x) {
        Item it = static_cast<const Item *>(view.in_items)[i];
        if ((uint32_t)it.ray >= n_rays) {
            rafi_forward_t(view, i, it, RAFI_POISON);
            continue;
        }
        log_visit(job, it.ray, d);
        float org[3], dir[3];
        int32_t K;
        job_ray(job, it.ray, org, dir, &K);
        const float gI = grad_image[it.ray];
        float tau = it.tau, ctau = 0.0f, B = it.I;
        int32_t k = it.k;
        int32_t dest = RAFI_DONE;
        // acc[q]: this lane's pending gradient for corner q = (q&1, q>>1&1, q>>2)
        // of the cell whose corner (0,0,0) is local voxel (cx, cy, cz)
        int32_t cell = -1, cx = 0, cy = 0, cz = 0;
        ea::Corners cc;
        float acc[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[q] = 0.0f;
        const int32_t o[8] = {0, 1, ex, ex + 1, sxy, sxy + 1, sxy + ex, sxy + ex + 1};
        auto flush = [&]() {
            if (cell < 0) return;
            bool fl[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) fl[q] = acc[q] != 0.0f;
            lds_add_corners(gl + cell, o, acc, fl);
        };
        // Move to the cell with corner (tx, ty, tz). Across one face the 4
        // shared corners stay in registers (renumbered); only the other 4 are
        // added to LDS. Any other move adds all 8.
        auto move_to = [&](int32_t tx, int32_t ty, int32_t tz) {
            const int32_t mx = tx - cx, my = ty - cy, mz = tz - cz;
            const bool face = cell >= 0 && abs(mx) + abs(my) + abs(mz) == 1;
            const int bit = mx ? 1 : (my ? 2 : 4);
            const bool up = mx + my + mz > 0;
            float keep[8];
            bool fl[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                // a corner on the far side of the crossed face survives as corner q ^ bit
                const bool kept = face && (((q & bit) != 0) == up);
                fl[q] = !kept && acc[q] != 0.0f;
                keep[q] = kept ? acc[q] : 0.0f;
            }
            if (cell >= 0) lds_add_corners(gl + cell, o, acc, fl);
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const float from = bit == 1 ? keep[q ^ 1] : (bit == 2 ? keep[q ^ 2] : keep[q ^ 4]);
                acc[q] = face ? from : 0.0f;
            }
            cx = tx;
            cy = ty;
            cz = tz;
            cell = tx + ex * (ty + ey * tz);
        };
        for (; k >= 0; --k) {
            float p[3];
            ea::sample_pos(org, dir, job.dt, k, p);
            if (!box.contains(p)) {
                dest = ea::owner_of(p, g);
                break;
            }
            // the forward march's per-sample forms: cached corners, the
            // hardware exponential, the series for 1 - exp(-sigma)
            const Tri t = kSmall ? ea::tri_setup_small(g.n, p) : ea::tri_setup(g.n, p);
            ea::fetch_corners(job.volume, g.n, t, cc);
            // local corner (i0, j0, k0) of the sample's cell. A move flushes
            // the corners the lane leaves, which hold only earlier samples'
            // terms: its LDS round trips overlap the gathers just issued.
            const int32_t tx = t.x - ox, ty = t.y - oy, tz = t.z - oz;
            if (gI != 0.0f && (cell < 0 || tx != cx || ty != cy || tz != cz)) move_to(tx, ty, tz);
            const float rho = ea::interp_corners(cc, t);
            const float sigma = c * rho;
            const float yt = -sigma - ctau;
            const float tt = tau + yt;
            ctau = (tt - tau) - yt;
            tau = tt;
            const float T = __expf(-tau);
            const float a = ea::one_minus_exp_neg(sigma);
            const float dIdrho = T * __fmaf_rn(c * (1.0f - a), rho - B, a);
            B = __fmaf_rn(a, rho - B, B);
            if (gI == 0.0f) continue;
            const float s = gI * dIdrho;
            const float gx0 = 1.0f - t.f0, gy0 = 1.0f - t.f1, gz0 = 1.0f - t.f2;
            const float a00 = s * gz0 * gy0, a01 = s * gz0 * t.f1, a10 = s * t.f2 * gy0, a11 = s * t.f2 * t.f1;
            acc[0] += a00 * gx0;
            acc[1] += a00 * t.f0;
            acc[2] += a01 * gx0;
            acc[3] += a01 * t.f0;
            acc[4] += a10 * gx0;
            acc[5] += a10 * t.f0;
            acc[6] += a11 * gx0;
            acc[7] += a11 * t.f0;
        }
        flush();
        it.k = k;
        it.tau = tau - ctau;
        it.I = B;
        if (k >= 0 && dest >= 0) rafi_forward_t(view, i, it, dest);
        else rafi_done(view, i);
    }
    __syncthreads();
    for (int32_t k = threadIdx.x; k < nl; k += blockDim.x) {
        const float v = gl[k];
        if (v != 0.0f) {
            const int32_t lz = k / sxy, ly = (k - lz * sxy) / ex, lx = k - lz * sxy - ly * ex;
            const int64_t idx = (ox + lx) + (int64_t)g.n * ((oy + ly) + (int64_t)g.n * (oz + lz));
            unsafeAtomicAdd(&grad[idx], v);
        }
    }
    __syncthreads();  // the region is reused by the next segment
}

// One workgroup per domain-pure tile of the input queue.
__global__ void __launch_bounds__(kBwdThreads)
bwd_march_lds_kernel(rafi_device_view view, rafi_ea_job job, const float *__restrict__ grad_image,
                     float *__restrict__ grad, uint32_t n_rays)
{
    extern __shared__ float gl[];
    uint64_t tb, te;
    const int32_t d = rafi_tile(view, rafi_xcd_block(blockIdx.x, gridDim.x), &tb, &te);
    if (job.n <= ea::kSmallN)
        bwd_segment<true>(view, job, grad_image, grad, n_rays, d, tb, te, gl);
    else
        bwd_segment<false>(view, job, grad_image, grad, n_rays, d, tb, te, gl);
}

// One workgroup per CU, each taking an equal contiguous slice of the queue
// and working through the brick segments it spans (usually one or two), so
// every CU is busy for the whole launch and the gradient region is flushed
// about once per workgroup.
__global__ void __launch_bounds__(kBwdThreads)
bwd_march_range_kernel(rafi_device_view view, rafi_ea_job job, const float *__restrict__ grad_image,
                       float *__restrict__ grad, uint32_t n_rays)
{
    extern __shared__ float gl[];
    const uint64_t w = rafi_xcd_block(blockIdx.x, gridDim.x);
    const uint64_t n = rafi_queue_length(view);
    uint64_t i = n * w / gridDim.x;
    const uint64_t end = n * (w + 1) / gridDim.x;
    while (i < end) {
        const int32_t d = ea::find_domain(view.in_offsets, view.n_domains, i);
        const uint64_t seg_end = min(end, view.in_offsets[d + 1]);
        if (job.n <= ea::kSmallN)
            bwd_segment<true>(view, job, grad_image, grad, n_rays, d, i, seg_end, gl);
        else
            bwd_segment<false>(view, job, grad_image, grad, n_rays, d, i, seg_end, gl);
        i = seg_end;
    }
}

// Bytes of a brick region (brick + one-voxel rim) in LDS.
size_t region_bytes(const rafi_ea_job *j)
{
    return sizeof(float) * (size_t)(j->n / j->grid[0] + 2) * (j->n / j->grid[1] + 2) * (j->n / j->grid[2] + 2);
}

size_t max_lds_bytes()
{
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return 0;
    return (size_t)v;
}

bool job_ok(const rafi_ctx *c, const rafi_ea_job *j)
{
    if (!c || !j || !j->volume || !j->views || !j->image) return false;
    if (j->n < 2 || j->n_views < 1 || j->width < 1 || j->height < 1) return false;
    for (int a = 0; a < 3; ++a)
        if (j->grid[a] < 1 || j->n % j->grid[a] != 0) return false;
    if (c->D != j->grid[0] * j->grid[1] * j->grid[2] || c->S != RAFI_EA_ITEM_BYTES) return false;
    if (j->visit_log && (!j->visit_count || j->visit_stride < 1)) return false;
    if (j->emit_mode != RAFI_SLOTS_ORDERED && j->emit_mode != RAFI_SLOTS_APPEND) return false;
    const uint64_t rays = (uint64_t)j->n_views * j->width * j->height;
    return rays <= c->cap && rays < (1ull << 31);
}

uint32_t n_rays_of(const rafi_ea_job *j) { return (uint32_t)((uint64_t)j->n_views * j->width * j->height); }

}  // namespace
}  // namespace rafi

using namespace rafi;

extern "C" {

int rafi_ea_raygen(rafi_ctx *c, const rafi_ea_job *job)
{
    if (!job_ok(c, job)) return RAFI_ERR_ARG;
    const uint64_t rays = n_rays_of(job);
    int rc = rafi_begin(c, rays);
    if (rc != RAFI_OK) return rc;
    rafi_device_view v;
    rafi_view(c, &v);
    if (rays)
        hipLaunchKernelGGL(raygen_kernel, dim3((uint32_t)((rays + 255) / 256)), dim3(256), 0, c->stream, v,
                           *job, rays);
    RAFI_LAUNCH_CHECK();
    return RAFI_OK;
}

int rafi_ea_march(rafi_ctx *c, const rafi_ea_job *job)
{
    if (!job_ok(c, job)) return RAFI_ERR_ARG;
    rafi_device_view v;
    rafi_view(c, &v);
    // The LDS-staged kernel pays one brick load per workgroup, so it is used
    // when the tile table was built with large tiles and the brick fits.
    const size_t lds = region_bytes(job);
    const bool staged = v.tile_items >= 512 && lds <= max_lds_bytes();
    const int ph = prof_domain_begin(c);
    if (v.n_in) {
        if (staged)
            hipLaunchKernelGGL(march_lds_kernel, dim3(v.n_tiles), dim3(kMarchLdsThreads), lds, c->stream, v, *job,
                               n_rays_of(job));
        else
            hipLaunchKernelGGL(march_kernel, dim3((uint32_t)((v.n_in + 255) / 256)), dim3(256), 0, c->stream, v,
                               *job, n_rays_of(job));
    }
    prof_domain_end(c, ph);
    RAFI_LAUNCH_CHECK();
    return RAFI_OK;
}

int rafi_ea_render(rafi_ctx *c, const rafi_ea_job *job, int32_t max_rounds, int32_t *rounds)
{
    if (!job_ok(c, job) || max_rounds < 1) return RAFI_ERR_ARG;
    int rc = rafi_ea_raygen(c, job);
    if (rc != RAFI_OK) return rc;
    // Tiles of 512 or more (rafi_set_tile_items) select the LDS-staged march,
    // whose grid is the host's tile count: rounds then wait for each total.
    if (c->tile_items >= 512 && region_bytes(job) <= max_lds_bytes()) {
        int32_t r = 0;
        for (;;) {
            uint64_t total = 0;
            rc = rafi_round(c, nullptr, &total);
            ++r;
            if (rc != RAFI_OK || total == 0) break;
            if (r >= max_rounds) { rc = RAFI_ERR_MAX_ROUNDS; break; }
            if (job->emit_mode == RAFI_SLOTS_APPEND && (rc = rafi_open(c, c->n_slots, RAFI_SLOTS_APPEND)) != RAFI_OK)
                break;
            if ((rc = rafi_ea_march(c, job)) != RAFI_OK) break;
        }
        if (rounds) *rounds = r;
        return rc;
    }
    // The gather march, launched one step ahead of the host (run_rounds).
    const uint32_t n_rays = n_rays_of(job);
    auto launch = [&](uint64_t bound) -> int {
        const int orc = rafi_open(c, bound, job->emit_mode);
        if (orc != RAFI_OK) return orc;
        rafi_device_view v;
        rafi_view(c, &v);
        v.n_in = bound;
        const int ph = prof_domain_begin(c);
        if (bound)
            hipLaunchKernelGGL(march_kernel, dim3((uint32_t)((bound + 255) / 256)), dim3(256), 0, c->stream, v,
                               *job, n_rays);
        prof_domain_end(c, ph);
        RAFI_LAUNCH_CHECK();
        return RAFI_OK;
    };
    return run_rounds(c, max_rounds, rounds, nullptr, launch, [](uint64_t n) { return n; });
}

int rafi_ea_backward(rafi_ctx *c, const rafi_ea_job *job, const float *grad_image, float *grad_volume,
                     int32_t max_rounds, int32_t *rounds)
{
    if (!job_ok(c, job) || !job->tau || !job->klast || !grad_image || !grad_volume || max_rounds < 1)
        return RAFI_ERR_ARG;
    const uint64_t rays = n_rays_of(job);
    int rc = rafi_begin(c, rays);
    if (rc != RAFI_OK) return rc;
    rafi_device_view v;
    rafi_view(c, &v);
    if (rays)
        hipLaunchKernelGGL(bwd_seed_kernel, dim3((uint32_t)((rays + 255) / 256)), dim3(256), 0, c->stream, v,
                           *job, rays);
    RAFI_LAUNCH_CHECK();
    // LDS privatisation when the brick's region fits a workgroup's LDS
    const size_t lds = region_bytes(job);
    const bool use_lds = lds <= max_lds_bytes();
    int cus = 0, dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
        return RAFI_ERR_HIP;
    if (use_lds && job->bwd_tile_items) {  // tile per workgroup: the host's tile count sizes the grid
        const uint32_t saved_tile = c->tile_items;
        c->tile_items = job->bwd_tile_items;
        int32_t r = 0;
        for (;;) {
            uint64_t total = 0;
            rc = rafi_round(c, nullptr, &total);
            ++r;
            if (rc != RAFI_OK || total == 0) break;
            if (r >= max_rounds) { rc = RAFI_ERR_MAX_ROUNDS; break; }
            rafi_view(c, &v);
            const int ph = prof_domain_begin(c);
            hipLaunchKernelGGL(bwd_march_lds_kernel, dim3(v.n_tiles), dim3(kBwdThreads), lds, c->stream, v, *job,
                               grad_image, grad_volume, (uint32_t)rays);
            prof_domain_end(c, ph);
            rc = hipGetLastError() == hipSuccess ? RAFI_OK : RAFI_ERR_HIP;
            if (rc != RAFI_OK) break;
        }
        c->tile_items = saved_tile;
        if (rounds) *rounds = r;
        return rc;
    }
    // one workgroup per CU over slices of the queue (or global atomics when the
    // brick's region does not fit), launched one step ahead of the host
    auto launch = [&](uint64_t bound) -> int {
        const int orc = rafi_open(c, bound, RAFI_SLOTS_ORDERED);
        if (orc != RAFI_OK) return orc;
        rafi_device_view lv;
        rafi_view(c, &lv);
        lv.n_in = bound;
        const int ph = prof_domain_begin(c);
        if (bound && use_lds) {
            const uint64_t want = (bound + kBwdThreads - 1) / kBwdThreads;
            const uint32_t blocks = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(want, cus));
            hipLaunchKernelGGL(bwd_march_range_kernel, dim3(blocks), dim3(kBwdThreads), lds, c->stream, lv, *job,
                               grad_image, grad_volume, (uint32_t)rays);
        } else if (bound) {
            hipLaunchKernelGGL(bwd_march_kernel, dim3((uint32_t)((bound + 255) / 256)), dim3(256), 0, c->stream,
                               lv, *job, grad_image, grad_volume, (uint32_t)rays);
        }
        prof_domain_end(c, ph);
        RAFI_LAUNCH_CHECK();
        return RAFI_OK;
    };
    return run_rounds(c, max_rounds, rounds, nullptr, launch, [](uint64_t n) { return n; });
}

}  // extern "C"
