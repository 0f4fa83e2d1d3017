// RK4 streamlines over bricked domains (particle tracing, Sec. 5.4 of the
// paper): one thread per particle integrates with classical RK4 while the
// particle stays in its brick, then forwards it to the brick it entered, or
// finishes it (did not move / left the field / step limit).
//
// Every operation that decides routing or step counts is float32 with the
// fused operations written out, so results are bitwise reproducible:
//   k1 = V(p); k2 = V(fma(h/2, k1, p)); k3 = V(fma(h/2, k2, p)); k4 = V(fma(h, k3, p))
//   s = fma(2, k2, k1); s = fma(2, k3, s); s = s + k4;  p' = fma(h/6, s, p)
// with V trilinear over the voxel-centred field, clamp-to-edge, lerping x,
// then y, then z (lerp(a, b, t) = fma(t, b - a, a)).
#include "internal.h"
#include "rafi_device.h"

namespace rafi {
namespace {

struct SLItem {
    float x, y, z;
    int32_t id;
};
static_assert(sizeof(SLItem) == RAFI_SL_ITEM_BYTES, "item layout");

__device__ inline float lerpf(float a, float b, float t) { return __fmaf_rn(t, b - a, a); }

// Velocity of one voxel as stored: FW = 4 floats per voxel (the padded layout
// written by rafi_sl_pack, 16-byte loads) or FW = 3 (the caller's n^3 x 3
// field as is; 25% fewer bytes per voxel, 12-byte loads).
struct V3 {
    float x, y, z;
};
template <int FW> struct Voxel;
template <> struct Voxel<4> { typedef float4 type; };
template <> struct Voxel<3> { typedef V3 type; };

template <int FW>
__device__ inline V3 load_voxel(const typename Voxel<FW>::type *__restrict__ f, int32_t i)
{
    const typename Voxel<FW>::type v = f[i];
    return V3{v.x, v.y, v.z};
}

// The 8 voxels around the last sample point, kept in registers: consecutive
// RK4 stages and steps usually fall in the same cell (a step moves a particle
// by a fraction of a voxel), and then no memory is touched. Reuse is exact.
struct CellCache {
    int32_t base = -1;  // corner (i0, j0, k0): linear index, or byte offset (buffer loads); -1 = empty
    V3 c[8];
};

// Cell index and weight along one axis of sample coordinate q: the sample
// shifted by half a voxel, clamped to [0, n-1], its floor limited to n-2.
// (med3 is the clamp for any non-NaN value; the floor is an integer below
// 2^24, so taking the limit in float is exact.)
__device__ inline float cell_axis(float q, float hi, float top, int32_t &i)
{
    const float uc = __builtin_amdgcn_fmed3f(q - 0.5f, 0.0f, hi);
    const float fl = fminf(floorf(uc), top);
    i = (int32_t)fl;
    return uc - fl;
}

// Linear voxel index i0 + n i1 + n^2 i2. The entry points check n^3 < 2^31,
// so n <= 1290 and every factor is below 2^24: the full-rate 24-bit
// multiplies are exact.
__device__ inline int32_t voxel_index(int32_t i0, int32_t i1, int32_t i2, int32_t sy, int32_t sz)
{
    return i0 + (int32_t)__umul24((uint32_t)i1, (uint32_t)sy) + (int32_t)__umul24((uint32_t)i2, (uint32_t)sz);
}

template <int FW>
__device__ inline void field_at(const typename Voxel<FW>::type *__restrict__ f, int32_t n, CellCache &cc, float qx,
                                float qy, float qz, float &vx, float &vy, float &vz)
{
    const float hi = (float)(n - 1), top = (float)(n - 2);
    int32_t i0[3];
    float w[3];
    w[0] = cell_axis(qx, hi, top, i0[0]);
    w[1] = cell_axis(qy, hi, top, i0[1]);
    w[2] = cell_axis(qz, hi, top, i0[2]);
    const int32_t sy = n, sz = n * n;  // n^3 < 2^31 (checked by the entry points)
    const int32_t base = voxel_index(i0[0], i0[1], i0[2], sy, sz);
    if (base != cc.base) {
        const typename Voxel<FW>::type *b = f + base;
        cc.c[0] = load_voxel<FW>(b, 0);
        cc.c[1] = load_voxel<FW>(b, 1);
        cc.c[2] = load_voxel<FW>(b, sy);
        cc.c[3] = load_voxel<FW>(b, sy + 1);
        cc.c[4] = load_voxel<FW>(b, sz);
        cc.c[5] = load_voxel<FW>(b, sz + 1);
        cc.c[6] = load_voxel<FW>(b, sz + sy);
        cc.c[7] = load_voxel<FW>(b, sz + sy + 1);
        cc.base = base;
    }
    const V3 *c = cc.c;
#define TRI(comp)                                                                                   \
    lerpf(lerpf(lerpf(c[0].comp, c[1].comp, w[0]), lerpf(c[2].comp, c[3].comp, w[0]), w[1]),        \
          lerpf(lerpf(c[4].comp, c[5].comp, w[0]), lerpf(c[6].comp, c[7].comp, w[0]), w[1]), w[2])
    vx = TRI(x);
    vy = TRI(y);
    vz = TRI(z);
#undef TRI
}

// The same sampler reading the field through a buffer resource, for fields
// of at most 2^31 - 1 bytes: a cell's 8 corners are loaded with one per-lane
// byte offset (the corner voxel), a wave-uniform offset per row (0, n, n^2,
// n^2 + n voxels) and an immediate of 0 or 1 voxel, so the loads need one
// address register instead of four 64-bit pointers. Same values.
struct FieldBuf {
    __amdgpu_buffer_rsrc_t r;
    int32_t row[4];  // byte offsets of the rows (0, n, n^2, n^2 + n voxels)
};

template <int FW>
__device__ inline V3 load_voxel_buf(const FieldBuf &fb, int32_t voff, int32_t soff)
{
    if constexpr (FW == 4) {
        const auto v = __builtin_amdgcn_raw_buffer_load_b128(fb.r, voff, soff, 0);
        return V3{__uint_as_float(v[0]), __uint_as_float(v[1]), __uint_as_float(v[2])};
    } else {
        const auto v = __builtin_amdgcn_raw_buffer_load_b96(fb.r, voff, soff, 0);
        return V3{__uint_as_float(v[0]), __uint_as_float(v[1]), __uint_as_float(v[2])};
    }
}

template <int FW>
__device__ inline void field_at_buf(const FieldBuf &fb, int32_t n, CellCache &cc, float qx, float qy, float qz,
                                    float &vx, float &vy, float &vz)
{
    const float hi = (float)(n - 1), top = (float)(n - 2);
    int32_t i0[3];
    float w[3];
    w[0] = cell_axis(qx, hi, top, i0[0]);
    w[1] = cell_axis(qy, hi, top, i0[1]);
    w[2] = cell_axis(qz, hi, top, i0[2]);
    // Byte offset of the corner voxel, which also names the cell. This path
    // runs for fields of at most 2^31 - 1 bytes (checked at launch), so
    // n <= 894 and the plane stride is at most 16 * 812^2 < 2^24 bytes: every
    // factor of the full-rate 24-bit multiplies is below 2^24 and the sum
    // below 2^31.
    const int32_t vo = (int32_t)(__umul24((uint32_t)i0[0], FW * 4u) + __umul24((uint32_t)i0[1], (uint32_t)fb.row[1]) +
                                 __umul24((uint32_t)i0[2], (uint32_t)fb.row[2]));
    if (vo != cc.base) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            cc.c[2 * r] = load_voxel_buf<FW>(fb, vo, fb.row[r]);
            cc.c[2 * r + 1] = load_voxel_buf<FW>(fb, vo + FW * 4, fb.row[r]);
        }
        cc.base = vo;
    }
    const V3 *c = cc.c;
#define TRI(comp)                                                                                   \
    lerpf(lerpf(lerpf(c[0].comp, c[1].comp, w[0]), lerpf(c[2].comp, c[3].comp, w[0]), w[1]),        \
          lerpf(lerpf(c[4].comp, c[5].comp, w[0]), lerpf(c[6].comp, c[7].comp, w[0]), w[1]), w[2])
    vx = TRI(x);
    vy = TRI(y);
    vz = TRI(z);
#undef TRI
}

// rk4_step over any sampler S(qx, qy, qz, vx, vy, vz).
template <typename S>
__device__ inline void rk4_step_with(S &&sample, float h, float hh, float h6, float x, float y, float z, float &nx,
                                     float &ny, float &nz)
{
    float k1x, k1y, k1z, k2x, k2y, k2z, k3x, k3y, k3z, k4x, k4y, k4z;
    sample(x, y, z, k1x, k1y, k1z);
    sample(__fmaf_rn(hh, k1x, x), __fmaf_rn(hh, k1y, y), __fmaf_rn(hh, k1z, z), k2x, k2y, k2z);
    sample(__fmaf_rn(hh, k2x, x), __fmaf_rn(hh, k2y, y), __fmaf_rn(hh, k2z, z), k3x, k3y, k3z);
    sample(__fmaf_rn(h, k3x, x), __fmaf_rn(h, k3y, y), __fmaf_rn(h, k3z, z), k4x, k4y, k4z);
    const float sx = __fmaf_rn(2.0f, k3x, __fmaf_rn(2.0f, k2x, k1x)) + k4x;
    const float sy = __fmaf_rn(2.0f, k3y, __fmaf_rn(2.0f, k2y, k1y)) + k4y;
    const float sz = __fmaf_rn(2.0f, k3z, __fmaf_rn(2.0f, k2z, k1z)) + k4z;
    nx = __fmaf_rn(h6, sx, x);
    ny = __fmaf_rn(h6, sy, y);
    nz = __fmaf_rn(h6, sz, z);
}

// One classical RK4 step from (x, y, z), with the operation order fixed above.
template <int FW>
__device__ inline void rk4_step(const typename Voxel<FW>::type *__restrict__ F, int32_t n, CellCache &cc, float h,
                                float hh, float h6, float x, float y, float z, float &nx, float &ny, float &nz)
{
    float k1x, k1y, k1z, k2x, k2y, k2z, k3x, k3y, k3z, k4x, k4y, k4z;
    field_at<FW>(F, n, cc, x, y, z, k1x, k1y, k1z);
    field_at<FW>(F, n, cc, __fmaf_rn(hh, k1x, x), __fmaf_rn(hh, k1y, y), __fmaf_rn(hh, k1z, z), k2x, k2y, k2z);
    field_at<FW>(F, n, cc, __fmaf_rn(hh, k2x, x), __fmaf_rn(hh, k2y, y), __fmaf_rn(hh, k2z, z), k3x, k3y, k3z);
    field_at<FW>(F, n, cc, __fmaf_rn(h, k3x, x), __fmaf_rn(h, k3y, y), __fmaf_rn(h, k3z, z), k4x, k4y, k4z);
    const float sx = __fmaf_rn(2.0f, k3x, __fmaf_rn(2.0f, k2x, k1x)) + k4x;
    const float sy = __fmaf_rn(2.0f, k3y, __fmaf_rn(2.0f, k2y, k1y)) + k4y;
    const float sz = __fmaf_rn(2.0f, k3z, __fmaf_rn(2.0f, k2z, k1z)) + k4z;
    nx = __fmaf_rn(h6, sx, x);
    ny = __fmaf_rn(h6, sy, y);
    nz = __fmaf_rn(h6, sz, z);
}

struct Geo {
    int32_t n, g0, g1, g2, b0, b1, b2;
};

__device__ inline Geo make_geo(const rafi_sl_job &j)
{
    return Geo{j.n, j.grid[0], j.grid[1], j.grid[2], j.n / j.grid[0], j.n / j.grid[1], j.n / j.grid[2]};
}

__device__ inline int32_t owner_of(float x, float y, float z, const Geo &g)
{
    const float fn = (float)g.n;
    if (!(x >= 0.0f) || !(x < fn) || !(y >= 0.0f) || !(y < fn) || !(z >= 0.0f) || !(z < fn)) return -1;
    const int32_t bx = (int32_t)floorf(x) / g.b0;
    const int32_t by = (int32_t)floorf(y) / g.b1;
    const int32_t bz = (int32_t)floorf(z) / g.b2;
    return bx + g.g0 * (by + g.g1 * bz);
}

// Owner of a position just left the brick [lo, hi) of domain d. Each axis's
// brick index moves by at most one when the position lies within one brick
// edge of the old brick (a step is a fraction of a voxel in any field a brick
// can hold without forwarding every step); the bounds are integers below
// 2^24, so the float compares are exact and give floor(x) / b. Positions
// farther away take the divisions. -1 outside the field (or NaN).
__device__ inline int32_t owner_after_step(float x, float y, float z, const Geo &g, int32_t d, float lo0,
                                           float hi0, float lo1, float hi1, float lo2, float hi2)
{
    const float fn = (float)g.n;
    if (!(x >= 0.0f) || !(x < fn) || !(y >= 0.0f) || !(y < fn) || !(z >= 0.0f) || !(z < fn)) return -1;
    const float b0 = (float)g.b0, b1 = (float)g.b1, b2 = (float)g.b2;
    if (x >= lo0 - b0 && x < hi0 + b0 && y >= lo1 - b1 && y < hi1 + b1 && z >= lo2 - b2 && z < hi2 + b2) {
        const int32_t cx = (int32_t)(x >= hi0) - (int32_t)(x < lo0);
        const int32_t cy = (int32_t)(y >= hi1) - (int32_t)(y < lo1);
        const int32_t cz = (int32_t)(z >= hi2) - (int32_t)(z < lo2);
        return d + cx + g.g0 * (cy + g.g1 * cz);
    }
    return owner_of(x, y, z, g);
}

__global__ void pack_kernel(const float *__restrict__ f3, uint64_t nvox, float4 *__restrict__ f4)
{
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < nvox;
         i += (uint64_t)gridDim.x * blockDim.x)
        f4[i] = make_float4(f3[3 * i], f3[3 * i + 1], f3[3 * i + 2], 0.0f);
}

__global__ void __launch_bounds__(256)
seed_kernel(rafi_device_view view, rafi_sl_job job, const float *__restrict__ seeds, uint64_t n_seeds)
{
    const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (i >= n_seeds) return;
    const Geo g = make_geo(job);
    SLItem it{seeds[3 * i], seeds[3 * i + 1], seeds[3 * i + 2], (int32_t)i};
    job.steps[i] = 0;
    const int32_t e = owner_of(it.x, it.y, it.z, g);
    if (e >= 0) {
        rafi_forward_t(view, i, it, e);
    } else {
        job.endpoint[3 * i] = it.x;
        job.endpoint[3 * i + 1] = it.y;
        job.endpoint[3 * i + 2] = it.z;
        if (job.reason) job.reason[i] = RAFI_SL_EXITED;
        rafi_done(view, i);
    }
}

__device__ inline int32_t find_domain(const uint64_t *__restrict__ off, int32_t D, uint64_t i)
{
    int32_t lo = 0, hi = D;
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (off[mid] <= i) lo = mid; else hi = mid;
    }
    return lo;
}

__device__ inline void count_forwards(unsigned long long *counters, bool cross, bool self_fwd)
{
    // one atomic per wave and counter
    const uint64_t mc = __ballot(cross), ms = __ballot(self_fwd);
    const int lane = threadIdx.x & 63;
    const int leader = __ffsll((long long)__ballot(1)) - 1;
    if (lane == leader) {
        if (mc) atomicAdd(&counters[0], (unsigned long long)__popcll(mc));
        if (ms) atomicAdd(&counters[1], (unsigned long long)__popcll(ms));
    }
}

// One lane per particle. A wave runs until the longest visit among its 64
// particles ends, so each workgroup first orders its particles by an estimate
// of their visit (a counting sort through LDS) and gives each wave particles
// of similar length. Every particle is integrated as if alone and written to
// its own output slot, so results do not depend on the lane it runs in.
template <int FW, bool BUF>
__global__ void __launch_bounds__(256)
advance_kernel(rafi_device_view view, rafi_sl_job job, uint64_t n_ids)
{
    constexpr uint32_t kThreads = 256, kWaves = kThreads / 64, kBuckets = 16;
    __shared__ float s_x[kThreads], s_y[kThreads], s_z[kThreads];
    __shared__ int32_t s_steps[kThreads], s_d[kThreads];
    __shared__ uint32_t s_slot[kThreads];
    __shared__ uint32_t s_cnt[kWaves][kBuckets];
    // the grid may be sized for an upper bound: number the live workgroups only
    const uint64_t n_in = rafi_queue_length(view);
    const uint32_t nb = (uint32_t)((n_in + kThreads - 1) / kThreads);
    if (blockIdx.x >= nb) return;
    const uint32_t t = threadIdx.x, w = t >> 6, lane = t & 63;
    const uint64_t base = rafi_xcd_block(blockIdx.x, nb) * (uint64_t)kThreads;
    const Geo g = make_geo(job);
    const typename Voxel<FW>::type *__restrict__ F = reinterpret_cast<const typename Voxel<FW>::type *>(job.field4);
    const bool capped = job.steps_per_visit > 0 && n_in > job.tail_items;
    const int32_t cap = capped ? job.steps_per_visit : 0x7fffffff;

    // Load this lane's particle and bucket it by a straight-line estimate of
    // its visit: the steps to the brick's faces at the nearest voxel's
    // velocity, capped by the steps it may still take (over the first
    // launch's particles this estimate correlates 0.98 with the visit). Empty
    // lanes take the last bucket. Only the lane order depends on it.
    uint64_t slot = base + t;
    bool live = slot < n_in;
    float x = 0.0f, y = 0.0f, z = 0.0f;
    int32_t steps = 0, d = 0;
    uint32_t key = kBuckets - 1;
    if (live) {
        const SLItem it = static_cast<const SLItem *>(view.in_items)[slot];
        if ((uint64_t)(uint32_t)it.id >= n_ids) {  // never true for items this library emitted
            rafi_forward_t(view, slot, it, RAFI_POISON);
            live = false;
        } else {
            x = it.x;
            y = it.y;
            z = it.z;
            steps = job.steps[it.id];
            d = find_domain(view.in_offsets, view.n_domains, slot);
            const int32_t bx = d % g.g0, by = (d / g.g0) % g.g1, bz = d / (g.g0 * g.g1);
            const int32_t i0 = min(max((int32_t)x, 0), g.n - 1), i1 = min(max((int32_t)y, 0), g.n - 1),
                          i2 = min(max((int32_t)z, 0), g.n - 1);
            const V3 v = load_voxel<FW>(F, voxel_index(i0, i1, i2, g.n, g.n * g.n));
            const float lo0 = (float)(bx * g.b0), lo1 = (float)(by * g.b1), lo2 = (float)(bz * g.b2);
            const float e0 = v.x > 0.0f ? (lo0 + (float)g.b0 - x) : (x - lo0);
            const float e1 = v.y > 0.0f ? (lo1 + (float)g.b1 - y) : (y - lo1);
            const float e2 = v.z > 0.0f ? (lo2 + (float)g.b2 - z) : (z - lo2);
            const float tx = e0 * __builtin_amdgcn_rcpf(fabsf(v.x)), ty = e1 * __builtin_amdgcn_rcpf(fabsf(v.y)),
                        tz = e2 * __builtin_amdgcn_rcpf(fabsf(v.z));
            const float span = (float)min(cap, job.max_steps);
            const float est = fminf(fminf(fminf(tx, ty), tz) * __builtin_amdgcn_rcpf(job.h),
                                    fminf((float)(job.max_steps - steps), span));
            key = (uint32_t)fminf(fmaxf(est * ((float)(kBuckets - 1) / span), 0.0f), (float)(kBuckets - 2));
        }
    }
    // Stable counting sort of the workgroup's lanes by key, through LDS. Every
    // thread reaches both barriers; threads left without a particle return
    // after the second, and no barrier follows.
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
    s_x[pos] = x;
    s_y[pos] = y;
    s_z[pos] = z;
    s_steps[pos] = steps;
    s_d[pos] = d;
    s_slot[pos] = (uint32_t)(slot - base);
    __syncthreads();
    if (t >= n_live) return;  // no barrier follows
    slot = base + s_slot[t];
    x = s_x[t];
    y = s_y[t];
    z = s_z[t];
    steps = s_steps[t];
    d = s_d[t];

    const int32_t bx = d % g.g0, by = (d / g.g0) % g.g1, bz = d / (g.g0 * g.g1);
    const float lo0 = (float)(bx * g.b0), hi0 = (float)((bx + 1) * g.b0);
    const float lo1 = (float)(by * g.b1), hi1 = (float)((by + 1) * g.b1);
    const float lo2 = (float)(bz * g.b2), hi2 = (float)((bz + 1) * g.b2);
    const float h = job.h, hh = job.h * 0.5f, h6 = (float)((double)job.h / 6.0);
    int32_t dest = d, why = 0;
    CellCache cc;
    FieldBuf fb;
    if constexpr (BUF) {
        const int32_t row = g.n * FW * 4, plane = g.n * row;
        fb.r = __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(job.field4), (short)0, plane * g.n, 0x00020000);
        fb.row[0] = 0;
        fb.row[1] = row;
        fb.row[2] = plane;
        fb.row[3] = plane + row;
    }
    for (int32_t taken = 0;;) {
        float nx, ny, nz;
        if constexpr (BUF)
            rk4_step_with(
                [&](float qx, float qy, float qz, float &vx, float &vy, float &vz) {
                    field_at_buf<FW>(fb, g.n, cc, qx, qy, qz, vx, vy, vz);
                },
                h, hh, h6, x, y, z, nx, ny, nz);
        else
            rk4_step<FW>(F, g.n, cc, h, hh, h6, x, y, z, nx, ny, nz);
        ++steps;
        ++taken;
        const bool same = __float_as_uint(nx) == __float_as_uint(x) && __float_as_uint(ny) == __float_as_uint(y) &&
                          __float_as_uint(nz) == __float_as_uint(z);
        x = nx;
        y = ny;
        z = nz;
        if (same) { why = RAFI_SL_STAGNANT; break; }
        const bool inside = x >= lo0 && x < hi0 && y >= lo1 && y < hi1 && z >= lo2 && z < hi2;
        const int32_t e = inside ? d : owner_after_step(x, y, z, g, d, lo0, hi0, lo1, hi1, lo2, hi2);
        if (e < 0) { why = RAFI_SL_EXITED; break; }
        if (steps >= job.max_steps) { why = RAFI_SL_MAXSTEPS; break; }
        if (e != d || taken >= cap) { dest = e; break; }
    }
    // the particle id again, rather than keeping it live through the loop
    const int32_t id = static_cast<const SLItem *>(view.in_items)[slot].id;
    job.steps[id] = steps;
    if (job.counters) count_forwards(job.counters, why == 0 && dest != d, why == 0 && dest == d);
    if (why) {
        job.endpoint[3 * (size_t)id] = x;
        job.endpoint[3 * (size_t)id + 1] = y;
        job.endpoint[3 * (size_t)id + 2] = z;
        if (job.reason) job.reason[id] = why;
        rafi_done(view, slot);
    } else {
        rafi_forward_t(view, slot, SLItem{x, y, z, id}, dest);
    }
}

// ------------------------------------------------ four lanes per particle ---
// Launches over few particles are bound by the latency of each particle's
// chain of RK4 steps, not by throughput. There a quad of lanes carries one
// particle: lane a (a < 3) holds coordinate a of the position, computes that
// axis's cell and weight, gathers component a of the 8 corners and
// interpolates it; lane 3 repeats lane 2. The weights and the step tests are
// exchanged within the quad by DPP moves. Every component's arithmetic is the
// one-lane kernel's, in the same order, so the results are bit-identical;
// each lane runs about a third of the chain.
//
// A lone wave issues about one instruction per 4.5 cycles, a DPP move that
// feeds the next instruction costs about 12 more, and any branch 30-60
// cycles (compare, exec or condition, redirect). So the common path of a
// sample and of a step is straight-line code: the rare events (a sample
// leaving the cached cell, a step that may stop or forward the particle)
// each sit behind one wave-uniform branch, laid out of line, that only
// tests a per-lane candidate flag and is not taken.
constexpr int kQuadThreads = 256;

// DPP quad permutations (lane j of a quad reads lane p[j]): 0xb1 = [1,0,3,2],
// 0x4e = [2,3,0,1], 0x55 * k = [k,k,k,k]. All four lanes of a quad must be
// active (the quad kernel branches only on quad-uniform values).
template <int CTRL>
__device__ inline int32_t quad_read(int32_t v)
{
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xf, 0xf, true);
}

__device__ inline int32_t quad_sum(int32_t v)
{
    v += quad_read<0xb1>(v);
    return v + quad_read<0x4e>(v);
}

__device__ inline int32_t quad_all(bool b)
{
    int32_t v = b ? 1 : 0;
    v &= quad_read<0xb1>(v);
    return v & quad_read<0x4e>(v);
}

template <int K>
__device__ inline float quad_lane(float v)
{
    return __int_as_float(quad_read<0x55 * K>(__float_as_int(v)));
}

// s_waitcnt immediate for vmcnt(0) alone (expcnt and lgkmcnt at their
// maxima, i.e. not waited on).
constexpr int kWaitLoads = 0x0f70;

// This lane's component of the 8 corners of one cell.
struct QuadCell {
    int32_t base = -1;  // linear index of corner (i0, j0, k0), the same on the 4 lanes; -1: empty
    float c[8];
};

// Lane geometry of the quad kernel: f points at component a of voxel 0, o[]
// holds the 8 corner offsets in floats, stride is the voxel stride of axis a
// (0 on lane 3, whose axis repeats lane 2's).
struct QuadAxis {
    const float *f;
    int32_t o[8];
    float hi;   // n - 1
    float top;  // n - 2
    int32_t stride;
};

// Cell (quad-uniform linear index) and this lane's weight of coordinate q,
// as the one-lane sampler computes them.
__device__ inline int32_t quad_cell(const QuadAxis &ax, float q, float &w)
{
    int32_t i;
    w = cell_axis(q, ax.hi, ax.top, i);
    return quad_sum((int32_t)__umul24((uint32_t)i, (uint32_t)ax.stride));
}

template <int FW>
__device__ inline void quad_gather(const QuadAxis &ax, int32_t base, QuadCell &dst)
{
    const float *b = ax.f + (size_t)base * FW;
#pragma unroll
    for (int k = 0; k < 8; ++k) dst.c[k] = b[ax.o[k]];
    dst.base = base;
}

// The cell in use: this lane's component of the 8 corners, kept as
// c[2k] = corner 2k and c[2k+1] = corner 2k+1 - corner 2k (the x-lerp's
// difference, the same float the lerp forms, so reuse is exact), the floor of
// this lane's axis (a float) and the quad's linear corner index.
struct QuadCache {
    float fl = -1.0f;
    int32_t base = -1;
    float c[8];
};

__device__ inline void cache_fill(QuadCache &cc, const QuadCell &s, float fl)
{
#pragma unroll
    for (int k = 0; k < 8; k += 2) {
        cc.c[k] = s.c[k];
        cc.c[k + 1] = s.c[k + 1] - s.c[k];
    }
    cc.base = s.base;
    cc.fl = fl;
}

// The one-lane sampler's 7 lerps (x, then y, then z) on the cached cell.
__device__ inline float interp_cached(const QuadCache &cc, float w0, float w1, float w2)
{
    const float *c = cc.c;
    const float x0 = __fmaf_rn(w0, c[1], c[0]), x1 = __fmaf_rn(w0, c[3], c[2]);
    const float x2 = __fmaf_rn(w0, c[5], c[4]), x3 = __fmaf_rn(w0, c[7], c[6]);
    return lerpf(lerpf(x0, x1, w1), lerpf(x2, x3, w1), w2);
}

// One sample of this lane's component at coordinate q. The interpolation runs
// on the cached cell at once. A lane whose axis floor differs from the cached
// one flags its wave; only then do the quads that left their cell take the
// corners from a look-ahead slot (pnow: gathered for this step, normally
// arrived; pnext: gathered for the next step) or gather them, and
// interpolate again.
template <int FW>
__device__ inline float sample_quad(const QuadAxis &ax, QuadCache &cc, const QuadCell &pnow, const QuadCell &pnext,
                                    float q)
{
    const float uc = __builtin_amdgcn_fmed3f(q - 0.5f, 0.0f, ax.hi);
    const float fl = fminf(floorf(uc), ax.top);
    const float w = uc - fl;
    const float w0 = quad_lane<0>(w), w1 = quad_lane<1>(w), w2 = quad_lane<2>(w);
    float r = interp_cached(cc, w0, w1, w2);
    if (__builtin_expect(__builtin_amdgcn_ballot_w64(fl != cc.fl) != 0, 0)) {
        const int32_t moved = quad_sum(fl != cc.fl ? 1 : 0);
        const int32_t base = quad_sum((int32_t)__umul24((uint32_t)(int32_t)fl, (uint32_t)ax.stride));
        if (moved) {
            if (base == pnow.base) {
                cache_fill(cc, pnow, fl);
            } else if (base == pnext.base) {
                cache_fill(cc, pnext, fl);
            } else {
                QuadCell g;
                quad_gather<FW>(ax, base, g);
                __builtin_amdgcn_s_waitcnt(kWaitLoads);
                cache_fill(cc, g, fl);
            }
            r = interp_cached(cc, w0, w1, w2);
        }
    }
    return r;
}

// Particle state of the quad kernel (lane a holds coordinate a). A particle
// that is done keeps running with step 0, so its position no longer moves,
// and its results are kept aside; the wave loops until no particle is live.
struct QuadRun {
    float x, sum;
    float h, hh, h6;  // job.h, h/2, h/6; all 0 once done
    int32_t steps, taken;
    bool live;
    float out_x;
    int32_t out_steps, out_why, out_dest;
};

// One RK4 step. The stop and forward tests run exactly (quad-wide, as the
// one-lane kernel decides them) only when some live lane of the wave sees a
// candidate: a coordinate that did not change, a coordinate outside the
// brick's range, or a step count at its limit.
template <int FW>
__device__ inline void quad_step(const QuadAxis &ax, QuadCache &cc, const QuadCell &pnow, const QuadCell &pnext,
                                 QuadRun &s, float lo, float hi, float fn, int32_t bsz, int32_t dmul, int32_t d,
                                 int32_t max_steps, int32_t cap, bool &any_live)
{
    const float x = s.x;
    const float k1 = sample_quad<FW>(ax, cc, pnow, pnext, x);
    const float k2 = sample_quad<FW>(ax, cc, pnow, pnext, __fmaf_rn(s.hh, k1, x));
    const float k3 = sample_quad<FW>(ax, cc, pnow, pnext, __fmaf_rn(s.hh, k2, x));
    const float k4 = sample_quad<FW>(ax, cc, pnow, pnext, __fmaf_rn(s.h, k3, x));
    const float sum = __fmaf_rn(2.0f, k3, __fmaf_rn(2.0f, k2, k1)) + k4;
    const float nx = __fmaf_rn(s.h6, sum, x);
    const int32_t steps = s.steps + 1, taken = s.taken + 1;
    s.x = nx;
    s.sum = sum;
    s.steps = steps;
    s.taken = taken;
    const bool cand = __float_as_uint(nx) == __float_as_uint(x) || !(nx >= lo && nx < hi) || steps >= max_steps ||
                      taken >= cap;
    if (__builtin_expect(__builtin_amdgcn_ballot_w64(s.live && cand) != 0, 0)) {
        const bool stag = quad_all(__float_as_uint(nx) == __float_as_uint(x));
        int32_t e = d;
        if (!quad_all(nx >= lo && nx < hi)) {
            const bool ok = nx >= 0.0f && nx < fn;
            const int32_t all_ok = quad_all(ok);
            const int32_t idx = quad_sum(ok ? ((int32_t)floorf(nx) / bsz) * dmul : 0);
            e = all_ok ? idx : -1;
        }
        const int32_t why = stag ? RAFI_SL_STAGNANT : e < 0 ? RAFI_SL_EXITED : steps >= max_steps ? RAFI_SL_MAXSTEPS : 0;
        const bool forward = why == 0 && (e != d || taken >= cap);
        if (s.live && (why != 0 || forward)) {
            s.live = false;
            s.out_x = nx;
            s.out_steps = steps;
            s.out_why = why;
            s.out_dest = forward ? e : d;
            s.h = 0.0f;
            s.hh = 0.0f;
            s.h6 = 0.0f;
        }
        any_live = __builtin_amdgcn_ballot_w64(s.live) != 0;
    }
}

// Settle the slot gathered a step ago (normally arrived), then gather into
// `slot` the cell two steps ahead along the last step's mean velocity. Done
// particles gather too (clamped into the field, never read), so that every
// path of the loop issues the same loads and the compiler's count of pending
// loads stays exact.
template <int FW>
__device__ inline void quad_look_ahead(const QuadAxis &ax, const QuadRun &s, float h6x2, QuadCell &slot)
{
    __builtin_amdgcn_s_waitcnt(kWaitLoads);
    float w;
    quad_gather<FW>(ax, quad_cell(ax, __fmaf_rn(h6x2, s.sum, s.x), w), slot);
}

template <int FW>
__global__ void __launch_bounds__(kQuadThreads)
advance_quad_kernel(rafi_device_view view, rafi_sl_job job, uint64_t n_ids)
{
    constexpr uint32_t kPer = kQuadThreads / 4;  // particles per workgroup
    const uint64_t n_in = rafi_queue_length(view);
    const uint32_t nb = (uint32_t)((n_in + kPer - 1) / kPer);
    if (blockIdx.x >= nb) return;
    const uint64_t i = rafi_xcd_block(blockIdx.x, nb) * (uint64_t)kPer + (threadIdx.x >> 2);
    if (i >= n_in) return;  // the same on the 4 lanes of a quad
    const int32_t lane = threadIdx.x & 3, a = min(lane, 2);
    const Geo g = make_geo(job);
    const int32_t d = find_domain(view.in_offsets, view.n_domains, i);
    const int32_t bsz = a == 0 ? g.b0 : a == 1 ? g.b1 : g.b2;
    const int32_t bc = a == 0 ? d % g.g0 : a == 1 ? (d / g.g0) % g.g1 : d / (g.g0 * g.g1);
    const float lo = (float)(bc * bsz), hi = (float)((bc + 1) * bsz);
    // weight of this axis's brick coordinate in the domain index
    const int32_t dmul = lane == 3 ? 0 : a == 0 ? 1 : a == 1 ? g.g0 : g.g0 * g.g1;
    const int32_t sy = g.n, sz = g.n * g.n;
    const QuadAxis ax{static_cast<const float *>(job.field4) + a,
                      {0, FW, sy * FW, (sy + 1) * FW, sz * FW, (sz + 1) * FW, (sz + sy) * FW, (sz + sy + 1) * FW},
                      (float)(g.n - 1), (float)(g.n - 2), lane == 3 ? 0 : a == 0 ? 1 : a == 1 ? sy : sz};
    const float fn = (float)g.n;

    SLItem it = static_cast<const SLItem *>(view.in_items)[i];
    if ((uint64_t)(uint32_t)it.id >= n_ids) {  // never true for items this library emitted
        if (lane == 0) rafi_forward_t(view, i, it, RAFI_POISON);
        return;
    }
    const float h6 = (float)((double)job.h / 6.0);
    const bool capped = job.steps_per_visit > 0 && n_in > job.tail_items;
    const int32_t cap = capped ? job.steps_per_visit : 0x7fffffff;
    QuadRun s{a == 0 ? it.x : a == 1 ? it.y : it.z, 0.0f, job.h, job.h * 0.5f, h6, job.steps[it.id], 0, true,
              0.0f, 0, 0, d};
    QuadCache cc;
    QuadCell pa, pb;
    bool any_live = true;
    // Nothing loaded so far may still be pending in the loop: a load first read
    // there would make every trip wait for all loads in flight.
    __builtin_amdgcn_s_waitcnt(kWaitLoads);
    // two steps per trip, so that the two look-ahead slots swap roles without
    // copies (every live particle stops within max_steps, so the loop ends)
    do {
        quad_step<FW>(ax, cc, pa, pb, s, lo, hi, fn, bsz, dmul, d, job.max_steps, cap, any_live);
        quad_look_ahead<FW>(ax, s, 2.0f * h6, pa);
        quad_step<FW>(ax, cc, pb, pa, s, lo, hi, fn, bsz, dmul, d, job.max_steps, cap, any_live);
        quad_look_ahead<FW>(ax, s, 2.0f * h6, pb);
    } while (any_live);
    const float x = s.out_x;
    const int32_t steps = s.out_steps, why = s.out_why, dest = s.out_dest;
    const float px = quad_lane<0>(x), py = quad_lane<1>(x), pz = quad_lane<2>(x);
    if (why && lane < 3) job.endpoint[3 * (size_t)it.id + lane] = x;
    if (lane != 0) return;
    job.steps[it.id] = steps;
    if (job.counters) count_forwards(job.counters, why == 0 && dest != d, why == 0 && dest == d);
    if (why) {
        if (job.reason) job.reason[it.id] = why;
        rafi_done(view, i);
    } else {
        it.x = px;
        it.y = py;
        it.z = pz;
        rafi_forward_t(view, i, it, dest);
    }
}

constexpr int kSLThreads = 256;

// Persistent form of advance_kernel. Each wave keeps 64 particles in flight:
// whenever at least job.refill_lanes lanes are idle, lane 0 takes that many
// queue indices from work[0] and the idle lanes load them. A particle is
// integrated exactly as in advance_kernel and written to its own slot, so
// results and routing are the same; only the assignment of particles to lanes
// changes. Every wave exits once the queue is handed out and its lanes are
// idle; each particle needs at most max_steps steps, so every wave ends.
// The last wave to exit (work[1] reaching n_waves - 1) resets both counters.
template <int FW>
__global__ void __launch_bounds__(kSLThreads)
advance_persistent_kernel(rafi_device_view view, rafi_sl_job job, uint64_t n_ids, unsigned long long *work,
                          uint32_t n_waves)
{
    const Geo g = make_geo(job);
    const typename Voxel<FW>::type *__restrict__ F = reinterpret_cast<const typename Voxel<FW>::type *>(job.field4);
    const uint64_t n = rafi_queue_length(view);
    const int lane = threadIdx.x & 63;
    const uint64_t lanes_below = (1ull << lane) - 1;
    const float h = job.h, hh = job.h * 0.5f, h6 = (float)((double)job.h / 6.0);
    const bool capped = job.steps_per_visit > 0 && n > job.tail_items;
    const int32_t cap = capped ? job.steps_per_visit : 0x7fffffff;
    const int refill = job.refill_lanes;

    bool has = false, exhausted = false;
    uint64_t i = 0;
    SLItem it{};
    int32_t d = 0, steps = 0, taken = 0;
    float lo0 = 0, hi0 = 0, lo1 = 0, hi1 = 0, lo2 = 0, hi2 = 0;
    uint32_t n_cross = 0, n_self = 0;
    CellCache cc;
    for (;;) {
        uint64_t idle = __ballot(!has);
        if (!exhausted && __popcll(idle) >= refill) {
            const uint32_t grab = (uint32_t)__popcll(idle);
            unsigned long long base = 0;
            if (lane == 0) base = atomicAdd(&work[0], (unsigned long long)grab);
            base = __shfl(base, 0);
            if (base + grab >= n) exhausted = true;
            if (!has) {
                const uint64_t j = base + (uint64_t)__popcll(idle & lanes_below);
                if (j < n) {
                    i = j;
                    it = static_cast<const SLItem *>(view.in_items)[j];
                    if ((uint64_t)(uint32_t)it.id >= n_ids) {  // never true for items this library emitted
                        rafi_forward_t(view, j, it, RAFI_POISON);
                    } else {
                        d = find_domain(view.in_offsets, view.n_domains, j);
                        const int32_t bx = d % g.g0, by = (d / g.g0) % g.g1, bz = d / (g.g0 * g.g1);
                        lo0 = (float)(bx * g.b0);
                        hi0 = (float)((bx + 1) * g.b0);
                        lo1 = (float)(by * g.b1);
                        hi1 = (float)((by + 1) * g.b1);
                        lo2 = (float)(bz * g.b2);
                        hi2 = (float)((bz + 1) * g.b2);
                        steps = job.steps[it.id];
                        taken = 0;
                        has = true;
                    }
                }
            }
            idle = __ballot(!has);
        }
        if (idle == ~0ull) {
            if (exhausted) break;
            continue;
        }
        if (has) {
            float nx, ny, nz;
            rk4_step<FW>(F, g.n, cc, h, hh, h6, it.x, it.y, it.z, nx, ny, nz);
            ++steps;
            ++taken;
            const bool same = __float_as_uint(nx) == __float_as_uint(it.x) &&
                              __float_as_uint(ny) == __float_as_uint(it.y) &&
                              __float_as_uint(nz) == __float_as_uint(it.z);
            it.x = nx;
            it.y = ny;
            it.z = nz;
            int32_t why = 0, dest = -1;
            if (same) {
                why = RAFI_SL_STAGNANT;
            } else {
                const bool inside = nx >= lo0 && nx < hi0 && ny >= lo1 && ny < hi1 && nz >= lo2 && nz < hi2;
                const int32_t e = inside ? d : owner_after_step(nx, ny, nz, g, d, lo0, hi0, lo1, hi1, lo2, hi2);
                if (e < 0) why = RAFI_SL_EXITED;
                else if (steps >= job.max_steps) why = RAFI_SL_MAXSTEPS;
                else if (e != d || taken >= cap) dest = e;
            }
            if (why || dest >= 0) {
                job.steps[it.id] = steps;
                if (why) {
                    job.endpoint[3 * (size_t)it.id] = nx;
                    job.endpoint[3 * (size_t)it.id + 1] = ny;
                    job.endpoint[3 * (size_t)it.id + 2] = nz;
                    if (job.reason) job.reason[it.id] = why;
                    rafi_done(view, i);
                } else {
                    n_cross += dest != d;
                    n_self += dest == d;
                    rafi_forward_t(view, i, it, dest);
                }
                has = false;
            }
        }
    }
    // all lanes are converged here (the exit test is wave-uniform)
    if (job.counters) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            n_cross += __shfl_xor(n_cross, o);
            n_self += __shfl_xor(n_self, o);
        }
        if (lane == 0) {
            if (n_cross) atomicAdd(&job.counters[0], (unsigned long long)n_cross);
            if (n_self) atomicAdd(&job.counters[1], (unsigned long long)n_self);
        }
    }
    if (lane == 0) {
        const unsigned long long done = atomicAdd(&work[1], 1ull);
        if (done == n_waves - 1) {
            atomicExch(&work[0], 0ull);
            atomicExch(&work[1], 0ull);
        }
    }
}

// Workgroups of the persistent kernel that fit on the device at once.
uint32_t persistent_blocks()
{
    static int cached_dev = -1;
    static uint32_t cached = 0;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (dev != cached_dev) {
        int per_cu = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, advance_persistent_kernel<4>, kSLThreads, 0) !=
                hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            return 0;
        cached = (uint32_t)std::max(1, per_cu) * (uint32_t)std::max(1, cus);
        cached_dev = dev;
    }
    return cached;
}

bool job_ok(const rafi_ctx *c, const rafi_sl_job *j)
{
    if (!c || !j || !j->field4 || !j->endpoint || !j->steps) return false;
    if (j->n < 2 || j->n > 1290 || j->max_steps < 1 || !(j->h > 0.0f) || j->steps_per_visit < 0) return false;
    if (j->refill_lanes < 0 || j->refill_lanes > 64) return false;
    if (j->field_stride != 0 && j->field_stride != 3 && j->field_stride != 4) return false;
    for (int a = 0; a < 3; ++a)
        if (j->grid[a] < 1 || j->n % j->grid[a] != 0) return false;
    return c->D == j->grid[0] * j->grid[1] * j->grid[2] && c->S == RAFI_SL_ITEM_BYTES;
}

// One domain launch over the queue in view v; v.n_in sizes the grid and may
// be an upper bound (the kernels read the queue length on the device).
int launch_advance(rafi_ctx *c, const rafi_sl_job *job, const rafi_device_view &v)
{
    const uint64_t one_per_item = (v.n_in + kSLThreads - 1) / kSLThreads;
    const uint32_t resident = job->refill_lanes > 0 ? persistent_blocks() : 1;
    if (!resident) return RAFI_ERR_HIP;
    const int ph = prof_domain_begin(c);
    if (v.n_in && job->refill_lanes > 0) {
        const uint32_t blocks = (uint32_t)std::min<uint64_t>(one_per_item, resident);
        if (job->field_stride == 3)
            hipLaunchKernelGGL(advance_persistent_kernel<3>, dim3(blocks), dim3(kSLThreads), 0, c->stream, v, *job,
                               c->wave_slots, c->work, blocks * (kSLThreads / 64));
        else
            hipLaunchKernelGGL(advance_persistent_kernel<4>, dim3(blocks), dim3(kSLThreads), 0, c->stream, v, *job,
                               c->wave_slots, c->work, blocks * (kSLThreads / 64));
    } else if (v.n_in && v.n_in <= job->quad_items) {
        const uint32_t blocks = (uint32_t)((v.n_in + kQuadThreads / 4 - 1) / (kQuadThreads / 4));
        if (job->field_stride == 3)
            hipLaunchKernelGGL(advance_quad_kernel<3>, dim3(blocks), dim3(kQuadThreads), 0, c->stream, v, *job,
                               c->wave_slots);
        else
            hipLaunchKernelGGL(advance_quad_kernel<4>, dim3(blocks), dim3(kQuadThreads), 0, c->stream, v, *job,
                               c->wave_slots);
    } else if (v.n_in) {
        // buffer loads while the field's byte offsets fit a signed 32-bit register
        const uint64_t n = (uint64_t)job->n;
        const bool buf = n * n * n * (uint64_t)(job->field_stride == 3 ? 12 : 16) <= 0x7fffffffull;
        static_assert(kSLThreads == 256, "advance_kernel sorts workgroups of 256 threads");
        const dim3 grid((uint32_t)one_per_item), block(kSLThreads);
        if (job->field_stride == 3) {
            if (buf)
                hipLaunchKernelGGL((advance_kernel<3, true>), grid, block, 0, c->stream, v, *job, c->wave_slots);
            else
                hipLaunchKernelGGL((advance_kernel<3, false>), grid, block, 0, c->stream, v, *job, c->wave_slots);
        } else {
            if (buf)
                hipLaunchKernelGGL((advance_kernel<4, true>), grid, block, 0, c->stream, v, *job, c->wave_slots);
            else
                hipLaunchKernelGGL((advance_kernel<4, false>), grid, block, 0, c->stream, v, *job, c->wave_slots);
        }
    }
    prof_domain_end(c, ph);
    RAFI_LAUNCH_CHECK();
    return RAFI_OK;
}

}  // namespace
}  // namespace rafi

using namespace rafi;

extern "C" {

int rafi_sl_pack(const float *field, int32_t n, float *field4, void *hip_stream)
{
    if (!field || !field4 || n < 2 || n > 1290) return RAFI_ERR_ARG;
    const uint64_t nvox = (uint64_t)n * n * n;
    const uint32_t blocks = (uint32_t)std::min<uint64_t>((nvox + 255) / 256, 65536);
    hipLaunchKernelGGL(pack_kernel, dim3(blocks), dim3(256), 0, static_cast<hipStream_t>(hip_stream), field, nvox,
                       reinterpret_cast<float4 *>(field4));
    RAFI_LAUNCH_CHECK();
    return RAFI_OK;
}

int rafi_sl_seed(rafi_ctx *c, const rafi_sl_job *job, const float *seeds, uint64_t n_seeds)
{
    if (!job_ok(c, job) || (n_seeds && !seeds) || n_seeds > c->cap || n_seeds >= (1ull << 31)) return RAFI_ERR_ARG;
    int rc = rafi_begin(c, n_seeds);
    if (rc != RAFI_OK) return rc;
    rafi_device_view v;
    rafi_view(c, &v);
    if (n_seeds)
        hipLaunchKernelGGL(seed_kernel, dim3((uint32_t)((n_seeds + 255) / 256)), dim3(256), 0, c->stream, v, *job,
                           seeds, n_seeds);
    RAFI_LAUNCH_CHECK();
    return RAFI_OK;
}

int rafi_sl_advance(rafi_ctx *c, const rafi_sl_job *job)
{
    if (!job_ok(c, job)) return RAFI_ERR_ARG;
    rafi_device_view v;
    rafi_view(c, &v);
    return launch_advance(c, job, v);
}

int rafi_sl_trace(rafi_ctx *c, const rafi_sl_job *job, const float *seeds, uint64_t n_seeds, int32_t max_rounds,
                  int32_t *rounds, uint64_t *forwarded)
{
    if (max_rounds < 1) return RAFI_ERR_ARG;
    int rc = rafi_sl_seed(c, job, seeds, n_seeds);
    if (rc != RAFI_OK) return rc;
    // each advance launch is enqueued one step ahead of the host (run_rounds)
    auto launch = [&](uint64_t bound) -> int {
        const int orc = rafi_open(c, bound, RAFI_SLOTS_ORDERED);
        if (orc != RAFI_OK) return orc;
        rafi_device_view v;
        rafi_view(c, &v);
        v.n_in = bound;
        return launch_advance(c, job, v);
    };
    return run_rounds(c, max_rounds, rounds, forwarded, launch, [](uint64_t n) { return n; });
}

}  // extern "C"
