// Delta-tracking volume path tracing over bricked domains (the stochastic
// brick transport of Sec. 5.1): ray generation (round 0), the brick kernel
// that walks paths and shadow rays through their current brick with
// Woodcock / ratio tracking, and the resolve step that sums the shadow-ray
// contributions per path. A visit to a brick ends when the item leaves the
// brick or the volume or, for a path, at a real collision, which spawns a
// shadow ray and a bounced path: fixed fan-out 2 (input slot i writes output
// slots 2i and 2i + 1), so queue order is reproducible.
//
// All positions and decisions are float32 with every operation written out;
// the random numbers are counter based (Philox4x32-10) and the logarithm is
// a fixed float32 series, so a path's walk does not depend on the bricks,
// the launch shape or the device.
#include <algorithm>

#include "ea_device.h"
#include "internal.h"
#include "rafi_device.h"

namespace rafi {
namespace {

struct DTItem {
    float px, py, pz;  // pending tentative point
    float dx, dy, dz;  // unit direction
    float w;           // path: throughput; shadow: weight incl. light and phase
    int32_t path;
    uint32_t stream, count;
    int32_t bounce, kind;  // kind 0 path, 1 shadow ray
};
static_assert(sizeof(DTItem) == RAFI_DT_ITEM_BYTES, "item layout");

constexpr int32_t kPath = 0, kShadow = 1;
// Tentative points per visit before the item is forwarded to its own brick
// (its walk continues unchanged next round): every visit ends.
constexpr uint32_t kMaxPoints = 65536;

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC 2011), first output word.
__device__ inline uint32_t philox_w0(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // each 32 x 32 -> 64-bit product as one multiply giving both halves
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c0;
}

__device__ inline float draw(const rafi_dt_job &job, DTItem &it)
{
    const uint32_t w = philox_w0(it.stream, it.count, 0u, 0u, job.seed, (uint32_t)it.path);
    it.count++;
    return (float)(w >> 8) * 5.9604644775390625e-08f;  // 2^-24
}

// ln x for normal x in (0, 1]: x = m 2^e, m in [sqrt(1/2), sqrt(2)),
// ln m = 2 atanh(s), s = (m - 1)/(m + 1), series to s^13; ln2 in two parts.
__device__ inline float dt_logf(float x)
{
    const uint32_t b = __float_as_uint(x);
    int32_t e = (int32_t)(b >> 23) - 127;
    float m = __uint_as_float((b & 0x007FFFFFu) | 0x3F800000u);
    if (m > 1.41421354f) {
        m = m * 0.5f;
        e += 1;
    }
    const float f = m - 1.0f;
    const float s = f / (2.0f + f);
    const float z = s * s;
    float q = __fmaf_rn(z, 1.0f / 13.0f, 1.0f / 11.0f);
    q = __fmaf_rn(z, q, 1.0f / 9.0f);
    q = __fmaf_rn(z, q, 1.0f / 7.0f);
    q = __fmaf_rn(z, q, 1.0f / 5.0f);
    q = __fmaf_rn(z, q, 1.0f / 3.0f);
    q = q * z;
    const float s2 = s + s;
    const float lnm = __fmaf_rn(s2, q, s2);
    const float fe = (float)e;
    return __fmaf_rn(fe, 0.693145751953125f, __fmaf_rn(fe, 1.42860677e-06f, lnm));
}

// Next tentative point: p += s d, s = -ln(1 - u) / smax.
__device__ inline void fly(const rafi_dt_job &job, DTItem &it)
{
    const float s = -dt_logf(1.0f - draw(job, it)) / job.smax;
    it.px = __fmaf_rn(s, it.dx, it.px);
    it.py = __fmaf_rn(s, it.dy, it.py);
    it.pz = __fmaf_rn(s, it.dz, it.pz);
}

// Isotropic direction, Marsaglia (1972): (x1, x2) uniform in the unit disc,
// d = (2 x1 sqrt(1 - s), 2 x2 sqrt(1 - s), 1 - 2 s), s = x1^2 + x2^2.
__device__ inline void isotropic(const rafi_dt_job &job, DTItem &it)
{
    for (int tries = 0; tries < 64; ++tries) {
        const float x1 = __fmaf_rn(2.0f, draw(job, it), -1.0f);
        const float x2 = __fmaf_rn(2.0f, draw(job, it), -1.0f);
        const float s = __fmaf_rn(x1, x1, x2 * x2);
        if (s < 1.0f && s > 0.0f) {
            const float t = 2.0f * sqrtf(1.0f - s);
            it.dx = x1 * t;
            it.dy = x2 * t;
            it.dz = __fmaf_rn(-2.0f, s, 1.0f);
            return;
        }
    }
    it.dx = 0.0f;
    it.dy = 0.0f;
    it.dz = 1.0f;
}

__device__ inline int32_t owner(const DTItem &it, const ea::Geo &g)
{
    const float p[3] = {it.px, it.py, it.pz};
    return ea::owner_of(p, g);
}

__device__ inline float sigma_at(const rafi_dt_job &job, const DTItem &it)
{
    const float p[3] = {it.px, it.py, it.pz};
    return job.kappa * ea::density(job.volume, job.n, ea::tri_setup(job.n, p));
}

__device__ inline void put_contrib(const rafi_dt_job &job, const DTItem &it)
{
    job.contrib[(int64_t)it.path * job.max_bounce + it.bounce] = it.w;
}

// ------------------------------------------------------------- raygen ---
__global__ void __launch_bounds__(256)
dt_raygen_kernel(rafi_device_view view, rafi_dt_job job, uint64_t n_paths)
{
    const uint64_t r = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (r >= n_paths) return;
    for (int32_t b = 0; b < job.max_bounce; ++b) job.contrib[r * job.max_bounce + b] = 0.0f;
    const ea::Geo g = ea::make_geo(job.n, job.grid);
    const int32_t per = job.width * job.height;
    const int32_t vi = (int32_t)(r / per);
    float o[3], d[3];
    int32_t K;
    ea::ray_setup(job.views[vi], (int32_t)r - vi * per, o, d, &K);
    DTItem it{};
    it.path = (int32_t)r;
    it.w = 1.0f;
    it.kind = kPath;
    const float fn = (float)job.n;
    float t0 = 0.0f, t1 = INFINITY;
    bool miss = false;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (d[a] != 0.0f) {
            const float ta = (0.0f - o[a]) / d[a], tb = (fn - o[a]) / d[a];
            t0 = fmaxf(t0, fminf(ta, tb));
            t1 = fminf(t1, fmaxf(ta, tb));
        } else if (!(o[a] >= 0.0f && o[a] < fn)) {
            miss = true;
        }
    }
    int32_t e = -1;
    if (!miss && t0 < t1) {
        it.dx = d[0];
        it.dy = d[1];
        it.dz = d[2];
        it.px = __fmaf_rn(t0, d[0], o[0]);
        it.py = __fmaf_rn(t0, d[1], o[1]);
        it.pz = __fmaf_rn(t0, d[2], o[2]);
        fly(job, it);
        e = owner(it, g);
    }
    if (e >= 0) rafi_forward_t(view, r, it, e);
    else rafi_done(view, r);
}

// -------------------------------------------------------------- trace ----
// Outcome of one visit: what goes into slots 2i and 2i + 1 (dest -1 = DONE).
__global__ void __launch_bounds__(256)
dt_trace_kernel(rafi_device_view view, rafi_dt_job job, uint64_t n_paths)
{
    constexpr uint32_t kThreads = 256, kWaves = kThreads / 64, kBuckets = 16;
    __shared__ uint32_t s_slot[kThreads];
    __shared__ int32_t s_d[kThreads];
    __shared__ uint32_t s_cnt[kWaves][kBuckets];
    // the grid may be sized for an upper bound: number the live workgroups only
    const uint64_t n_in = rafi_queue_length(view);
    const uint32_t nb = (uint32_t)((n_in + kThreads - 1) / kThreads);
    if (blockIdx.x >= nb) return;  // whole workgroups: no lane is left out of the counter sums
    const uint32_t t = threadIdx.x, w = t >> 6, lane = t & 63;
    const uint64_t base = rafi_xcd_block(blockIdx.x, nb) * (uint64_t)kThreads;
    const ea::Geo g = ea::make_geo(job.n, job.grid);
    // Order the workgroup's items into lanes by the tentative points they can
    // expect in their brick (the straight-line chord times the majorant),
    // through LDS; results do not depend on the lane.
    uint64_t i = base + t;
    int32_t d = 0;
    uint32_t key = kBuckets - 1;
    if (i < n_in) {
        d = ea::find_domain(view.in_offsets, view.n_domains, i);
        const DTItem q = static_cast<const DTItem *>(view.in_items)[i];
        const ea::Box bx = ea::box_of(d, g);
        const float lo[3] = {bx.lo0, bx.lo1, bx.lo2}, hi[3] = {bx.hi0, bx.hi1, bx.hi2};
        const float p[3] = {q.px, q.py, q.pz}, dv[3] = {q.dx, q.dy, q.dz};
        float texit = 3.0e38f;
#pragma unroll
        for (int a = 0; a < 3; ++a)
            if (dv[a] != 0.0f)
                texit = fminf(texit, ((dv[a] > 0.0f ? hi[a] : lo[a]) - p[a]) * __builtin_amdgcn_rcpf(dv[a]));
        const float span = (float)(g.b0 + g.b1 + g.b2);
        key = (uint32_t)fminf(fmaxf(texit * ((float)(kBuckets - 1) / span), 0.0f), (float)(kBuckets - 2));
    }
    uint32_t rank = 0;
#pragma unroll
    for (uint32_t k = 0; k < kBuckets; ++k) {
        const uint64_t m = __ballot(key == k);
        if (lane == 0) s_cnt[w][k] = (uint32_t)__popcll(m);
        if (key == k) rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
    }
    __syncthreads();
    uint32_t pos = rank, n_live = 0;
    for (uint32_t k = 0; k < kBuckets; ++k) {
#pragma unroll
        for (uint32_t ww = 0; ww < kWaves; ++ww) {
            const uint32_t c = s_cnt[ww][k];
            pos += (k < key || (k == key && ww < w)) ? c : 0;
            n_live += k < kBuckets - 1 ? c : 0;
        }
    }
    s_slot[pos] = (uint32_t)(i - base);
    s_d[pos] = d;
    __syncthreads();
    // no barrier follows: lanes without an item stay for the counter sums
    const bool live = t < n_live;
    uint32_t points = 0, hits = 0;
    if (live) {
        i = base + s_slot[t];
        d = s_d[t];
        const ea::Box box = ea::box_of(d, g);
        DTItem it = static_cast<const DTItem *>(view.in_items)[i];
        DTItem out0 = it;
        int32_t dest0 = RAFI_DONE, dest1 = RAFI_DONE;
        if ((uint64_t)(uint32_t)it.path >= n_paths || it.bounce < 0 || it.bounce >= job.max_bounce) {
            dest0 = RAFI_POISON;  // never true for items this library emitted
        } else {
            for (;;) {
                if (points == kMaxPoints) {  // bounded visit: continue next round in this brick
                    out0 = it;
                    dest0 = d;
                    break;
                }
                ++points;
                const float sigma = sigma_at(job, it);
                if (it.kind == kPath) {
                    const float u = draw(job, it);
                    if (u * job.smax < sigma) {
                        // real collision: shadow ray into slot 2i, bounced path into 2i + 1
                        ++hits;
                        const float w = it.w * job.albedo;
                        DTItem sh = it;
                        sh.kind = kShadow;
                        sh.stream = 2u * (uint32_t)it.bounce + 1u;
                        sh.count = 0;
                        sh.w = w * job.radiance * 0.0795774715f;  // 1 / (4 pi)
                        sh.dx = job.light[0];
                        sh.dy = job.light[1];
                        sh.dz = job.light[2];
                        fly(job, sh);
                        const int32_t es = owner(sh, g);
                        if (es >= 0) {
                            out0 = sh;
                            dest0 = es;
                        } else {
                            put_contrib(job, sh);
                        }
                        if (it.bounce + 1 < job.max_bounce) {
                            it.bounce += 1;
                            it.stream = 2u * (uint32_t)it.bounce;
                            it.count = 0;
                            it.w = w;
                            isotropic(job, it);
                            fly(job, it);
                            dest1 = owner(it, g);
                        }
                        break;
                    }
                } else {
                    it.w = it.w * (1.0f - sigma / job.smax);
                }
                fly(job, it);
                const float p[3] = {it.px, it.py, it.pz};
                if (box.contains(p)) continue;
                const int32_t e = ea::owner_of(p, g);
                if (e >= 0) {
                    out0 = it;
                    dest0 = e;
                } else if (it.kind == kShadow) {
                    put_contrib(job, it);
                }
                break;
            }
        }
        if (dest0 == RAFI_DONE) rafi_done(view, 2 * i);
        else rafi_forward_t(view, 2 * i, out0, dest0);
        if (dest1 >= 0) rafi_forward_t(view, 2 * i + 1, it, dest1);
        else rafi_done(view, 2 * i + 1);
    }
    if (job.counters) {  // the whole wave is here: one atomic pair per wave
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            points += __shfl_xor(points, o);
            hits += __shfl_xor(hits, o);
        }
        if ((threadIdx.x & 63) == 0) {
            atomicAdd(&job.counters[0], (unsigned long long)points);
            atomicAdd(&job.counters[1], (unsigned long long)hits);
        }
    }
}

// image[path] = sum over scattering events, in event order
__global__ void dt_resolve_kernel(rafi_dt_job job, uint64_t n_paths)
{
    const uint64_t r = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (r >= n_paths) return;
    float s = 0.0f;
    for (int32_t b = 0; b < job.max_bounce; ++b) s += job.contrib[r * job.max_bounce + b];
    job.image[r] = s;
}

uint64_t n_paths_of(const rafi_dt_job *j) { return (uint64_t)j->n_views * j->width * j->height; }

bool job_ok(const rafi_ctx *c, const rafi_dt_job *j)
{
    if (!c || !j || !j->volume || !j->views || !j->contrib) return false;
    if (j->n < 2 || j->n_views < 1 || j->width < 1 || j->height < 1 || j->max_bounce < 1) return false;
    if (!(j->smax > 0.0f) || !(j->kappa >= 0.0f) || !(j->albedo >= 0.0f && j->albedo <= 1.0f)) return false;
    for (int a = 0; a < 3; ++a)
        if (j->grid[a] < 1 || j->n % j->grid[a] != 0) return false;
    if ((uint64_t)j->n * j->n * j->n >= (1ull << 62)) return false;
    if (c->D != j->grid[0] * j->grid[1] * j->grid[2] || c->S != RAFI_DT_ITEM_BYTES) return false;
    const uint64_t paths = n_paths_of(j);
    return paths <= c->cap && paths < (1ull << 31) && paths * (uint64_t)j->max_bounce < (1ull << 62);
}

}  // namespace
}  // namespace rafi

using namespace rafi;

extern "C" {

int rafi_dt_capacity(uint64_t n_paths, int32_t max_bounce, uint64_t *capacity)
{
    if (!capacity || max_bounce < 1 || n_paths >= (1ull << 31)) return RAFI_ERR_ARG;
    *capacity = 2 * n_paths * ((uint64_t)max_bounce + 1);
    return RAFI_OK;
}

int rafi_dt_raygen(rafi_ctx *c, const rafi_dt_job *job)
{
    if (!job_ok(c, job)) return RAFI_ERR_ARG;
    const uint64_t paths = n_paths_of(job);
    int rc = rafi_begin(c, paths);
    if (rc != RAFI_OK) return rc;
    rafi_device_view v;
    rafi_view(c, &v);
    if (paths)
        hipLaunchKernelGGL(dt_raygen_kernel, dim3((uint32_t)((paths + 255) / 256)), dim3(256), 0, c->stream, v,
                           *job, paths);
    RAFI_LAUNCH_CHECK();
    return RAFI_OK;
}

int rafi_dt_trace(rafi_ctx *c, const rafi_dt_job *job)
{
    if (!job_ok(c, job) || 2 * c->n_in > c->cap) return RAFI_ERR_ARG;
    int rc = rafi_open(c, 2 * c->n_in, RAFI_SLOTS_ORDERED);
    if (rc != RAFI_OK) return rc;
    rafi_device_view v;
    rafi_view(c, &v);
    const int ph = prof_domain_begin(c);
    if (v.n_in)
        hipLaunchKernelGGL(dt_trace_kernel, dim3((uint32_t)((v.n_in + 255) / 256)), dim3(256), 0, c->stream, v,
                           *job, n_paths_of(job));
    prof_domain_end(c, ph);
    RAFI_LAUNCH_CHECK();
    return RAFI_OK;
}

int rafi_dt_render(rafi_ctx *c, const rafi_dt_job *job, int32_t max_rounds, int32_t *rounds)
{
    if (max_rounds < 1) return RAFI_ERR_ARG;
    int rc = rafi_dt_raygen(c, job);
    if (rc != RAFI_OK) return rc;
    const uint64_t paths = n_paths_of(job);
    // Each trace launch is enqueued one step ahead of the host (run_rounds).
    // bound (the slots just split) only bounds the queue length, so the
    // output is clamped to the capacity: a queue that really needs more than
    // capacity slots has its excess emits dropped and counted
    // (RAFI_ERR_OVERFLOW), while the grid still covers every queued item.
    const uint64_t cap = c->cap;
    auto launch = [&](uint64_t bound) -> int {
        const int orc = rafi_open(c, std::min<uint64_t>(2 * bound, cap), RAFI_SLOTS_ORDERED);
        if (orc != RAFI_OK) return orc;
        rafi_device_view v;
        rafi_view(c, &v);
        v.n_in = bound;
        const int ph = prof_domain_begin(c);
        if (bound)
            hipLaunchKernelGGL(dt_trace_kernel, dim3((uint32_t)((bound + 255) / 256)), dim3(256), 0, c->stream, v,
                               *job, paths);
        prof_domain_end(c, ph);
        RAFI_LAUNCH_CHECK();
        return RAFI_OK;
    };
    rc = run_rounds(c, max_rounds, rounds, nullptr, launch,
                    [cap](uint64_t n) { return std::min<uint64_t>(2 * n, cap); });
    if (rc == RAFI_OK && job->image) {
        if (paths)
            hipLaunchKernelGGL(dt_resolve_kernel, dim3((uint32_t)((paths + 255) / 256)), dim3(256), 0, c->stream,
                               *job, paths);
        RAFI_LAUNCH_CHECK();
    }
    return rc;
}

}  // extern "C"
