// Emission-absorption ray march over bricked domains: ray generation (round
// 0), the brick kernel that advances rays through their current brick and
// forwards them at its boundary (the VoPaT / Lander pattern, Sec. 5.1-5.2:
// each forwarded ray carries its partial integration state), and the adjoint
// that replays every ray backwards through the same bricks.
//
// Per sample k of a ray (all float32):
//   t_k = (k + 0.5) * dt,   p_k = fma(t_k, dir, org),
//   rho_k = trilinear(volume, p_k) (clamp to edge; lerp x, then y, then z),
//   sigma_k = c * rho_k,
//   I   += exp(-tau) * (1 - exp(-sigma_k)) * rho_k,   tau += sigma_k.
// The opacity 1 - exp(-sigma) is taken as -expm1(-sigma) and both sums are
// compensated (Kahan) within a brick visit, so the float32 integral stays
// within a few ulps of the exact value over hundreds of samples.
#include "internal.h"
#include "rafi_device.h"

namespace rafi {
namespace {

struct EAItem {
    int32_t ray;
    int32_t k;
    float tau;
    float I;  // forward: partial integral; backward: B, the integral behind sample k
};
static_assert(sizeof(EAItem) == RAFI_EA_ITEM_BYTES, "item layout");

struct Geo {
    int32_t n;
    int32_t g0, g1, g2;
    int32_t b0, b1, b2;  // brick edge per axis
};

__device__ inline Geo make_geo(const rafi_ea_job &j)
{
    Geo g;
    g.n = j.n;
    g.g0 = j.grid[0];
    g.g1 = j.grid[1];
    g.g2 = j.grid[2];
    g.b0 = j.n / j.grid[0];
    g.b1 = j.n / j.grid[1];
    g.b2 = j.n / j.grid[2];
    return g;
}

// Owning brick of p, or -1 outside [0, n)^3. Bricks are half-open.
__device__ inline int32_t owner_of(const float p[3], const Geo &g)
{
    const float fn = (float)g.n;
#pragma unroll
    for (int a = 0; a < 3; ++a)
        if (!(p[a] >= 0.0f) || !(p[a] < fn)) return -1;
    const int32_t bx = (int32_t)floorf(p[0]) / g.b0;
    const int32_t by = (int32_t)floorf(p[1]) / g.b1;
    const int32_t bz = (int32_t)floorf(p[2]) / g.b2;
    return bx + g.g0 * (by + g.g1 * bz);
}

// Brick bounds of domain d: a point is in d iff lo <= p < hi on every axis
// (the bounds are integers, so this equals owner_of(p) == d).
struct Box {
    float lo0, hi0, lo1, hi1, lo2, hi2;
    __device__ bool contains(const float p[3]) const
    {
        return p[0] >= lo0 && p[0] < hi0 && p[1] >= lo1 && p[1] < hi1 && p[2] >= lo2 && p[2] < hi2;
    }
};

__device__ inline Box box_of(int32_t d, const Geo &g)
{
    const int32_t bx = d % g.g0, by = (d / g.g0) % g.g1, bz = d / (g.g0 * g.g1);
    return Box{(float)(bx * g.b0), (float)((bx + 1) * g.b0), (float)(by * g.b1), (float)((by + 1) * g.b1),
               (float)(bz * g.b2), (float)((bz + 1) * g.b2)};
}

__device__ inline void ray_setup(const rafi_ea_job &j, int32_t ray, float org[3], float dir[3],
                                 int32_t *n_samples)
{
    const int32_t per = j.width * j.height;
    const int32_t v = ray / per;
    const int32_t local = ray - v * per;
    const int32_t py = local / j.width;
    const int32_t px = local - py * j.width;
    const rafi_ortho_view &V = j.views[v];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        org[a] = __fmaf_rn((float)py, V.dv[a], __fmaf_rn((float)px, V.du[a], V.org0[a]));
        dir[a] = V.dir[a];
    }
    *n_samples = V.n_samples;
}

__device__ inline void sample_pos(const float org[3], const float dir[3], float dt, int32_t k, float p[3])
{
    const float t = ((float)k + 0.5f) * dt;
#pragma unroll
    for (int a = 0; a < 3; ++a) p[a] = __fmaf_rn(t, dir[a], org[a]);
}

__device__ inline float lerpf(float a, float b, float t) { return __fmaf_rn(t, b - a, a); }

// Trilinear setup at p: corner (i0, j0, k0) and fractional weights.
struct Tri {
    int64_t base;
    float f0, f1, f2;
};

__device__ inline Tri tri_setup(int32_t n, const float p[3])
{
    int32_t i0[3];
    float f[3];
    const float hi = (float)(n - 1);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float u = fminf(fmaxf(p[a] - 0.5f, 0.0f), hi);
        const int32_t i = min((int32_t)floorf(u), n - 2);
        i0[a] = i;
        f[a] = u - (float)i;
    }
    return Tri{i0[0] + (int64_t)n * (i0[1] + (int64_t)n * i0[2]), f[0], f[1], f[2]};
}

// Trilinear density at p from the global volume (voxel centres at i + 0.5).
__device__ inline float density(const float *__restrict__ vol, int32_t n, const Tri &t)
{
    const int64_t sx = 1, sy = n, sz = (int64_t)n * n;
    const float *b = vol + t.base;
    const float x00 = lerpf(b[0], b[sx], t.f0);
    const float x10 = lerpf(b[sy], b[sy + sx], t.f0);
    const float x01 = lerpf(b[sz], b[sz + sx], t.f0);
    const float x11 = lerpf(b[sz + sy], b[sz + sy + sx], t.f0);
    const float y0 = lerpf(x00, x10, t.f1);
    const float y1 = lerpf(x01, x11, t.f1);
    return lerpf(y0, y1, t.f2);
}

__device__ inline void log_visit(const rafi_ea_job &j, int32_t ray, int32_t d)
{
    if (!j.visit_log) return;
    const int32_t c = j.visit_count[ray];
    if (c < j.visit_stride) j.visit_log[(int64_t)ray * j.visit_stride + c] = d;
    j.visit_count[ray] = c + 1;
}

// First k in [0, K] for which pred(k) flips from `from` to !from (K if never).
template <typename Pred>
__device__ inline int32_t first_flip(int32_t K, bool from, Pred pred)
{
    int32_t lo = 0, hi = K;
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (pred(mid) != from) hi = mid; else lo = mid + 1;
    }
    return lo;
}

// ------------------------------------------------------------- raygen ---
// Every coordinate of p_k is monotone in k (fma and the product are
// correctly rounded, hence monotone), so "sample k is inside the box" holds on
// one interval of k; its first index comes from a binary search per face.
__global__ void __launch_bounds__(256)
raygen_kernel(rafi_device_view view, rafi_ea_job job, uint64_t n_rays)
{
    const uint64_t r = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (r >= n_rays) return;
    const Geo g = make_geo(job);
    float org[3], dir[3];
    int32_t K;
    ray_setup(job, (int32_t)r, org, dir, &K);
    const float fn = (float)g.n;
    int32_t k_lo = 0, k_hi = K;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        auto coord = [&](int32_t k) {
            const float t = ((float)k + 0.5f) * job.dt;
            return __fmaf_rn(t, dir[a], org[a]);
        };
        auto ge0 = [&](int32_t k) { return coord(k) >= 0.0f; };
        auto ltn = [&](int32_t k) { return coord(k) < fn; };
        if (dir[a] > 0.0f) {
            k_lo = max(k_lo, first_flip(K, false, ge0));   // becomes true
            k_hi = min(k_hi, first_flip(K, true, ltn));    // becomes false
        } else if (dir[a] < 0.0f) {
            k_lo = max(k_lo, first_flip(K, false, ltn));
            k_hi = min(k_hi, first_flip(K, true, ge0));
        } else if (!(org[a] >= 0.0f && org[a] < fn)) {
            k_hi = 0;
        }
    }
    if (job.visit_count) job.visit_count[r] = 0;
    EAItem it{(int32_t)r, 0, 0.0f, 0.0f};
    if (k_lo < k_hi) {
        float p[3];
        sample_pos(org, dir, job.dt, k_lo, p);
        it.k = k_lo;
        if (job.kfirst) job.kfirst[r] = k_lo;
        rafi_forward_t(view, r, it, owner_of(p, g));
    } else {
        if (job.kfirst) job.kfirst[r] = 0;
        job.image[r] = 0.0f;
        if (job.tau) job.tau[r] = 0.0f;
        if (job.klast) job.klast[r] = 0;
        rafi_done(view, r);
    }
}

// ------------------------------------------------------------- march ----
__device__ inline int32_t find_domain(const uint64_t *__restrict__ off, int32_t D, uint64_t i)
{
    int32_t lo = 0, hi = D;  // last d with off[d] <= i
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (off[mid] <= i) lo = mid; else hi = mid;
    }
    return lo;
}

__global__ void __launch_bounds__(256)
march_kernel(rafi_device_view view, rafi_ea_job job, uint32_t n_rays)
{
    const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (i >= view.n_in) return;
    const Geo g = make_geo(job);
    const int32_t d = find_domain(view.in_offsets, view.n_domains, i);
    const Box box = box_of(d, g);

    EAItem it = static_cast<const EAItem *>(view.in_items)[i];
    if ((uint32_t)it.ray >= n_rays) {  // never true for items this library emitted
        rafi_forward_t(view, i, it, RAFI_POISON);
        return;
    }
    log_visit(job, it.ray, d);
    float org[3], dir[3];
    int32_t K;
    ray_setup(job, it.ray, org, dir, &K);
    float tau = it.tau, I = it.I, ctau = 0.0f, cI = 0.0f;
    int32_t k = it.k;
    int32_t dest = RAFI_DONE;
    for (; k < K; ++k) {
        float p[3];
        sample_pos(org, dir, job.dt, k, p);
        if (!box.contains(p)) {
            dest = owner_of(p, g);
            break;
        }
        const float rho = density(job.volume, g.n, tri_setup(g.n, p));
        const float sigma = job.c * rho;
        const float w = expf(-tau) * -expm1f(-sigma);
        // compensated I += w * rho
        const float yI = w * rho - cI;
        const float tI = I + yI;
        cI = (tI - I) - yI;
        I = tI;
        // compensated tau += sigma
        const float yt = sigma - ctau;
        const float tt = tau + yt;
        ctau = (tt - tau) - yt;
        tau = tt;
    }
    it.k = k;
    it.tau = tau - ctau;
    it.I = I - cI;
    if (dest >= 0) {
        rafi_forward_t(view, i, it, dest);
    } else {
        job.image[it.ray] = it.I;
        if (job.tau) job.tau[it.ray] = it.tau;
        if (job.klast) job.klast[it.ray] = it.k;
        rafi_done(view, i);
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
    const Geo g = make_geo(job);
    float org[3], dir[3];
    int32_t K;
    ray_setup(job, (int32_t)r, org, dir, &K);
    float p[3];
    sample_pos(org, dir, job.dt, kl - 1, p);
    const EAItem it{(int32_t)r, kl - 1, job.tau[r], 0.0f};
    rafi_forward_t(view, r, it, owner_of(p, g));
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

__global__ void __launch_bounds__(256)
bwd_march_kernel(rafi_device_view view, rafi_ea_job job, const float *__restrict__ grad_image,
                 float *__restrict__ grad, uint32_t n_rays)
{
    const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (i >= view.n_in) return;
    const Geo g = make_geo(job);
    const int32_t d = find_domain(view.in_offsets, view.n_domains, i);
    const Box box = box_of(d, g);
    EAItem it = static_cast<const EAItem *>(view.in_items)[i];
    if ((uint32_t)it.ray >= n_rays) {
        rafi_forward_t(view, i, it, RAFI_POISON);
        return;
    }
    log_visit(job, it.ray, d);
    float org[3], dir[3];
    int32_t K;
    ray_setup(job, it.ray, org, dir, &K);
    const float gI = grad_image[it.ray];
    const float c = job.c;
    float tau = it.tau, ctau = 0.0f, B = it.I;
    int32_t k = it.k;
    int32_t dest = RAFI_DONE;
    for (; k >= 0; --k) {
        float p[3];
        sample_pos(org, dir, job.dt, k, p);
        if (!box.contains(p)) {
            dest = owner_of(p, g);
            break;
        }
        const Tri t = tri_setup(g.n, p);
        const float rho = density(job.volume, g.n, t);
        const float sigma = c * rho;
        // compensated tau -= sigma: tau becomes tau_k, the depth in front of sample k
        const float yt = -sigma - ctau;
        const float tt = tau + yt;
        ctau = (tt - tau) - yt;
        tau = tt;
        const float T = expf(-tau);
        const float a = -expm1f(-sigma);
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

bool job_ok(const rafi_ctx *c, const rafi_ea_job *j)
{
    if (!c || !j || !j->volume || !j->views || !j->image) return false;
    if (j->n < 2 || j->n_views < 1 || j->width < 1 || j->height < 1) return false;
    for (int a = 0; a < 3; ++a)
        if (j->grid[a] < 1 || j->n % j->grid[a] != 0) return false;
    if (c->D != j->grid[0] * j->grid[1] * j->grid[2] || c->S != RAFI_EA_ITEM_BYTES) return false;
    if (j->visit_log && (!j->visit_count || j->visit_stride < 1)) return false;
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
    const int ph = prof_domain_begin(c);
    if (v.n_in)
        hipLaunchKernelGGL(march_kernel, dim3((uint32_t)((v.n_in + 255) / 256)), dim3(256), 0, c->stream, v,
                           *job, n_rays_of(job));
    prof_domain_end(c, ph);
    RAFI_LAUNCH_CHECK();
    return RAFI_OK;
}

int rafi_ea_render(rafi_ctx *c, const rafi_ea_job *job, int32_t max_rounds, int32_t *rounds)
{
    if (!job_ok(c, job) || max_rounds < 1) return RAFI_ERR_ARG;
    int rc = rafi_ea_raygen(c, job);
    if (rc != RAFI_OK) return rc;
    int32_t r = 0;
    for (;;) {
        uint64_t total = 0;
        rc = rafi_round(c, nullptr, &total);
        ++r;
        if (rc != RAFI_OK) break;
        if (total == 0) break;
        if (r >= max_rounds) { rc = RAFI_ERR_MAX_ROUNDS; break; }
        rc = rafi_ea_march(c, job);
        if (rc != RAFI_OK) break;
    }
    if (rounds) *rounds = r;
    return rc;
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
    int32_t r = 0;
    for (;;) {
        uint64_t total = 0;
        rc = rafi_round(c, nullptr, &total);
        ++r;
        if (rc != RAFI_OK) break;
        if (total == 0) break;
        if (r >= max_rounds) { rc = RAFI_ERR_MAX_ROUNDS; break; }
        rafi_view(c, &v);
        const int ph = prof_domain_begin(c);
        hipLaunchKernelGGL(bwd_march_kernel, dim3((uint32_t)((v.n_in + 255) / 256)), dim3(256), 0, c->stream, v,
                           *job, grad_image, grad_volume, (uint32_t)rays);
        prof_domain_end(c, ph);
        RAFI_LAUNCH_CHECK();
    }
    if (rounds) *rounds = r;
    return rc;
}

}  // extern "C"
