// Device building blocks of the emission-absorption march, shared by the
// plain render (ea.hip) and the batched form (batched.hip).
//
// Per sample k of a ray (all float32):
//   t_k = (k + 0.5) * dt,   p_k = fma(t_k, dir, org),
//   rho_k = trilinear(volume, p_k) (clamp to edge; lerp x, then y, then z),
//   sigma_k = c * rho_k,
//   I   += exp(-tau) * (1 - exp(-sigma_k)) * rho_k,   tau += sigma_k.
// The opacity 1 - exp(-sigma) is taken as -expm1(-sigma) and both sums are
// compensated (Kahan) within a brick visit, so the float32 integral stays
// within a few ulps of the exact value over hundreds of samples.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "rafi.h"

namespace rafi {
namespace ea {

struct Item {
    int32_t ray;
    int32_t k;
    float tau;
    float I;  // forward: partial integral; backward: B, the integral behind sample k
};
static_assert(sizeof(Item) == RAFI_EA_ITEM_BYTES, "item layout");

struct Geo {
    int32_t n;
    int32_t g0, g1, g2;
    int32_t b0, b1, b2;  // brick edge per axis
};

__device__ inline Geo make_geo(int32_t n, const int32_t grid[3])
{
    return Geo{n, grid[0], grid[1], grid[2], n / grid[0], n / grid[1], n / grid[2]};
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
    // the six compares combined without short-circuit branches
    __device__ bool contains(const float p[3]) const
    {
        return (p[0] >= lo0) & (p[0] < hi0) & (p[1] >= lo1) & (p[1] < hi1) & (p[2] >= lo2) & (p[2] < hi2);
    }
};

__device__ inline Box box_of(int32_t d, const Geo &g)
{
    const int32_t bx = d % g.g0, by = (d / g.g0) % g.g1, bz = d / (g.g0 * g.g1);
    return Box{(float)(bx * g.b0), (float)((bx + 1) * g.b0), (float)(by * g.b1), (float)((by + 1) * g.b1),
               (float)(bz * g.b2), (float)((bz + 1) * g.b2)};
}

// Ray `local` of a view (row-major pixels): origin, direction, sample count.
__device__ inline void ray_setup(const rafi_ortho_view &V, int32_t local, float org[3], float dir[3],
                                 int32_t *n_samples)
{
    const int32_t py = local / V.width;
    const int32_t px = local - py * V.width;
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

// Trilinear setup at p: corner (i0, j0, k0), its linear index and the
// fractional weights.
struct Tri {
    int64_t base;
    int32_t x, y, z;
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
    return Tri{i0[0] + (int64_t)n * (i0[1] + (int64_t)n * i0[2]), i0[0], i0[1], i0[2], f[0], f[1], f[2]};
}

// tri_setup for volumes of at most 1290^3 voxels (n^3 < 2^31, the caller's
// test): the same cell and weights, the clamp as one med3 (the clamp for any
// non-NaN value), the floor limited to n - 2 in float (exact: an integer
// below 2^24) and the corner's linear index from full-rate 24-bit
// multiplies (every factor below 2^24, the sum below 2^31).
constexpr int32_t kSmallN = 1290;

__device__ inline Tri tri_setup_small(int32_t n, const float p[3])
{
    const float hi = (float)(n - 1), top = (float)(n - 2);
    uint32_t i0[3];
    float f[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float u = __builtin_amdgcn_fmed3f(p[a] - 0.5f, 0.0f, hi);
        const float fl = fminf(floorf(u), top);
        i0[a] = (uint32_t)fl;
        f[a] = u - fl;
    }
    const uint32_t nn = (uint32_t)n;
    const uint32_t base = i0[0] + __umul24(i0[1], nn) + __umul24(i0[2], nn * nn);
    return Tri{(int64_t)base, (int32_t)i0[0], (int32_t)i0[1], (int32_t)i0[2], f[0], f[1], f[2]};
}

// 1 - exp(-s). For |s| below 1/16, the Maclaurin series of the function to
// the s^6 term (Horner form; the truncated terms are below 1.2e-11 |s|):
// five fused multiply-adds and a product instead of the library's expm1.
// Larger |s|, or a NaN, take the library call.
__device__ inline float one_minus_exp_neg(float s)
{
    if (fabsf(s) < 0.0625f) {
        float q = __fmaf_rn(s, -1.0f / 720.0f, 1.0f / 120.0f);
        q = __fmaf_rn(s, q, -1.0f / 24.0f);
        q = __fmaf_rn(s, q, 1.0f / 6.0f);
        q = __fmaf_rn(s, q, -0.5f);
        q = __fmaf_rn(s, q, 1.0f);
        return s * q;
    }
    return -expm1f(-s);
}

// Trilinear density from the volume (voxel centres at i + 0.5).
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

// The 8 voxels of the last sampled cell, kept in registers. Samples half a
// voxel apart along a ray often fall in the same cell, and then no memory is
// read: on the 64-view render the texture-address unit's work drops by about
// a third. The values and the interpolation are those of density(), so the
// result is bit-identical.
struct Corners {
    int64_t base = -1;  // linear index of the cached cell's corner; -1 = empty
    float v[8];
};

// density_cached in two halves: the loads of a new cell's corners (issued,
// not waited for), and the interpolation that uses them.
__device__ inline void fetch_corners(const float *__restrict__ vol, int32_t n, const Tri &t, Corners &cc)
{
    if (t.base != cc.base) {
        const int64_t sy = n, sz = (int64_t)n * n;
        const float *b = vol + t.base;
        cc.v[0] = b[0];
        cc.v[1] = b[1];
        cc.v[2] = b[sy];
        cc.v[3] = b[sy + 1];
        cc.v[4] = b[sz];
        cc.v[5] = b[sz + 1];
        cc.v[6] = b[sz + sy];
        cc.v[7] = b[sz + sy + 1];
        cc.base = t.base;
    }
}

__device__ inline float interp_corners(const Corners &cc, const Tri &t)
{
    const float x00 = lerpf(cc.v[0], cc.v[1], t.f0);
    const float x10 = lerpf(cc.v[2], cc.v[3], t.f0);
    const float x01 = lerpf(cc.v[4], cc.v[5], t.f0);
    const float x11 = lerpf(cc.v[6], cc.v[7], t.f0);
    const float y0 = lerpf(x00, x10, t.f1);
    const float y1 = lerpf(x01, x11, t.f1);
    return lerpf(y0, y1, t.f2);
}

__device__ inline float density_cached(const float *__restrict__ vol, int32_t n, const Tri &t, Corners &cc)
{
    fetch_corners(vol, n, t, cc);
    return interp_corners(cc, t);
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

// Ray generation: the first sample index inside [0, n)^3, or -1 if none.
// Every coordinate of p_k is monotone in k (the product and the fma are
// correctly rounded, hence monotone), so the inside samples form one interval
// of k, found by a binary search per face; *owner is the brick of that sample.
__device__ inline int32_t first_inside(const Geo &g, const float org[3], const float dir[3], int32_t K, float dt,
                                       int32_t *owner)
{
    const float fn = (float)g.n;
    int32_t k_lo = 0, k_hi = K;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        auto coord = [&](int32_t k) {
            const float t = ((float)k + 0.5f) * dt;
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
    if (k_lo >= k_hi) return -1;
    float p[3];
    sample_pos(org, dir, dt, k_lo, p);
    *owner = owner_of(p, g);
    return k_lo;
}

// Advance a ray through its brick (box) from sample it.k: accumulates tau and
// I and leaves it.k at the first sample not taken. Returns the brick that owns
// that sample, or -1 when the ray left the volume or ran out of samples.
// kSmall: the volume has at most kSmallN^3 voxels (tri_setup_small).
// The transmittance exp(-tau) is the hardware exponential (a base-2
// exponential of -tau log2(e)); its relative error, about 1e-6 for the
// optical depths of a ray, stays well inside the integrals' tolerance; the
// emission weight 1 - exp(-sigma) keeps full relative accuracy for small
// sigma (one_minus_exp_neg).
template <bool kSmall>
__device__ inline int32_t march_through_n(const float *__restrict__ vol, const Geo &g, const Box &box,
                                          const float org[3], const float dir[3], int32_t K, float dt, float c,
                                          Item &it)
{
    float tau = it.tau, I = it.I, ctau = 0.0f, cI = 0.0f;
    int32_t k = it.k;
    int32_t dest = -1;
    Corners cc;
    for (; k < K; ++k) {
        float p[3];
        sample_pos(org, dir, dt, k, p);
        if (!box.contains(p)) {
            dest = owner_of(p, g);
            break;
        }
        const float rho = density_cached(vol, g.n, kSmall ? tri_setup_small(g.n, p) : tri_setup(g.n, p), cc);
        const float sigma = c * rho;
        const float w = __expf(-tau) * one_minus_exp_neg(sigma);
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
    return dest;
}

__device__ inline int32_t march_through(const float *__restrict__ vol, const Geo &g, const Box &box,
                                        const float org[3], const float dir[3], int32_t K, float dt, float c,
                                        Item &it)
{
    return g.n <= kSmallN ? march_through_n<true>(vol, g, box, org, dir, K, dt, c, it)
                          : march_through_n<false>(vol, g, box, org, dir, K, dt, c, it);
}

// A brick's voxels plus a one-voxel rim, staged in LDS: region origin
// o = lo - 1 per axis, extent e = b + 2. Samples inside the brick only touch
// voxels [max(lo-1, 0), min(hi, n-1)], all inside the region.
struct Region {
    int32_t ox, oy, oz, ex, ey, ez;
};

__device__ inline Region region_of(const Box &box, const Geo &g)
{
    return Region{(int32_t)box.lo0 - 1, (int32_t)box.lo1 - 1, (int32_t)box.lo2 - 1, g.b0 + 2, g.b1 + 2, g.b2 + 2};
}

// Corner (i0, j0, k0) of a trilinear setup -> region index.
__device__ inline int32_t region_index(const Region &r, const Tri &t)
{
    return (t.x - r.ox) + r.ex * ((t.y - r.oy) + r.ey * (t.z - r.oz));
}

// Load the region of `vol` into lds (voxels outside the volume are never read).
__device__ inline void load_region(float *lds, const float *__restrict__ vol, int32_t n, const Region &r)
{
    const int32_t total = r.ex * r.ey * r.ez, sxy = r.ex * r.ey;
    for (int32_t k = threadIdx.x; k < total; k += blockDim.x) {
        const int32_t lz = k / sxy, ly = (k - lz * sxy) / r.ex, lx = k - lz * sxy - ly * r.ex;
        const int32_t x = r.ox + lx, y = r.oy + ly, z = r.oz + lz;
        float v = 0.0f;
        if (x >= 0 && x < n && y >= 0 && y < n && z >= 0 && z < n) v = vol[x + (int64_t)n * (y + (int64_t)n * z)];
        lds[k] = v;
    }
}

// Trilinear density from a staged region: the same values and operations as
// density(), so the result is bit-identical.
__device__ inline float density_lds(const float *lds, const Region &r, int32_t li, const Tri &t)
{
    const int32_t sy = r.ex, sz = r.ex * r.ey;
    const float *b = lds + li;
    const float x00 = lerpf(b[0], b[1], t.f0);
    const float x10 = lerpf(b[sy], b[sy + 1], t.f0);
    const float x01 = lerpf(b[sz], b[sz + 1], t.f0);
    const float x11 = lerpf(b[sz + sy], b[sz + sy + 1], t.f0);
    const float y0 = lerpf(x00, x10, t.f1);
    const float y1 = lerpf(x01, x11, t.f1);
    return lerpf(y0, y1, t.f2);
}

// march_through with the brick's densities read from a staged region.
__device__ inline int32_t march_through_lds(const float *lds, const Region &reg, const Geo &g, const Box &box,
                                            const float org[3], const float dir[3], int32_t K, float dt, float c,
                                            Item &it)
{
    float tau = it.tau, I = it.I, ctau = 0.0f, cI = 0.0f;
    int32_t k = it.k;
    int32_t dest = -1;
    for (; k < K; ++k) {
        float p[3];
        sample_pos(org, dir, dt, k, p);
        if (!box.contains(p)) {
            dest = owner_of(p, g);
            break;
        }
        const Tri t = tri_setup(g.n, p);
        const float rho = density_lds(lds, reg, region_index(reg, t), t);
        const float sigma = c * rho;
        const float w = expf(-tau) * -expm1f(-sigma);
        const float yI = w * rho - cI;
        const float tI = I + yI;
        cI = (tI - I) - yI;
        I = tI;
        const float yt = sigma - ctau;
        const float tt = tau + yt;
        ctau = (tt - tau) - yt;
        tau = tt;
    }
    it.k = k;
    it.tau = tau - ctau;
    it.I = I - cI;
    return dest;
}

__device__ inline int32_t find_domain(const uint64_t *__restrict__ off, int32_t D, uint64_t i)
{
    int32_t lo = 0, hi = D;  // last d with off[d] <= i
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (off[mid] <= i) lo = mid; else hi = mid;
    }
    return lo;
}

}  // namespace ea
}  // namespace rafi
