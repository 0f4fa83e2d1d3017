/*
 * rafi_oracle.c -- CPU oracle for the work-forwarding hot path.
 *
 * TEST INFRASTRUCTURE ONLY. This is a plain, slow, obviously-correct CPU
 * statement of what the forwarding path computes. Only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg load it; the product
 * library never calls it, and it shares no source, header, table or constant
 * with the HIP path. Single-threaded by default; oracle_set_threads(n)
 * runs the items of one (domain, round) on n OpenMP threads for timing.
 * Every item's work reads only shared inputs and writes only its own output
 * slot and its own per-item results, so the results are the same bits for
 * any thread count.
 *
 * Precision: floating point that decides an integer (sample positions, which
 * brick owns a point, RK4 trajectories that decide routing and step counts) is
 * carried in float32 with every operation spelled out (fmaf where the method
 * fuses), exactly as the GPU kernels take those decisions. Integrals and
 * gradients, which decide nothing, are carried in float64.
 *
 * Compile with -ffp-contract=off and without -ffast-math so that every
 * float32 operation below is rounded exactly once.
 *
 * Paper references are to "RaFI" (arXiv 2605.30294): Sec. 3.2 ray queues,
 * Sec. 3.3 device interface, Sec. 3.4 host context, Sec. 4.2.1 sorting by
 * destination, Sec. 4.2.2 exchanging rays, Sec. 4.2.3 wrap-up, Sec. 5.1
 * VoPaT (ray-march-and-forward), Sec. 5.4 particle tracing.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_DONE (-1)

/* Threads for the per-item loops (1: plain sequential loops). */
static int g_threads = 1;

void oracle_set_threads(int32_t n) { g_threads = n < 1 ? 1 : n; }
int32_t oracle_get_threads(void) { return g_threads; }

/* ======================================================================
 * O1. The forward step = a stable counting sort by destination.
 *
 * Sec. 4.2.1 sorts the emitted items by the 64-bit key (dest << 32 | i) and
 * gathers them, so items bound for the same destination keep their emission
 * order. Sec. 4.2.2 tallies per-destination begin/end (empty destinations get
 * zero) and exchanges count and offset arrays. On one device the result of
 * all of this is: item i with destination e lands at
 *     offset[e] + #{ j < i : dest[j] == e },
 * with offset[] the exclusive prefix sum of the per-destination counts.
 * That is counting sort (CLRS 8.2), written out directly here.
 *
 * dest == -1 (ORC_DONE) means "leaves the system"; any other value outside
 * [0, n_domains) is an invalid destination: both kinds are dropped and counted.
 * Items are opaque bytes (Sec. 3.1: the library never looks inside).
 * ====================================================================== */
int oracle_multisplit(uint64_t n, uint32_t item_bytes, const uint8_t *items,
                      const int32_t *dest, int32_t n_domains, uint8_t *out,
                      uint64_t *counts, uint64_t *offsets, uint64_t *n_done,
                      uint64_t *n_bad)
{
    if (n_domains <= 0) return -1;
    uint64_t done = 0, bad = 0;
    for (int32_t e = 0; e < n_domains; ++e) counts[e] = 0;
    for (uint64_t i = 0; i < n; ++i) {
        int32_t d = dest[i];
        if (d == ORC_DONE) done++;
        else if (d < 0 || d >= n_domains) bad++;
        else counts[d]++;
    }
    offsets[0] = 0;
    for (int32_t e = 0; e < n_domains; ++e) offsets[e + 1] = offsets[e] + counts[e];
    uint64_t *cursor = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n_domains);
    if (!cursor) return -2;
    for (int32_t e = 0; e < n_domains; ++e) cursor[e] = offsets[e];
    for (uint64_t i = 0; i < n; ++i) {
        int32_t d = dest[i];
        if (d < 0 || d >= n_domains) continue;
        memcpy(out + cursor[d] * item_bytes, items + i * item_bytes, item_bytes);
        cursor[d]++;
    }
    free(cursor);
    if (n_done) *n_done = done;
    if (n_bad) *n_bad = bad;
    return 0;
}

/* ======================================================================
 * Geometry shared by the volume and the field workloads (oracle-local).
 *
 * Cube of n^3 voxels, voxel centres at i + 0.5, world box [0, n)^3, split into
 * g[0] x g[1] x g[2] equal bricks ("domains", the paper's ranks) of edge
 * n / g[a]. Domain id d = bx + g0 * (by + g1 * bz). A point belongs to the
 * brick containing it (half-open bricks: a point on a brick plane belongs to
 * the upper brick); a point outside the box belongs to nobody (-1).
 * ====================================================================== */
static int32_t owner_of(const float p[3], int32_t n, const int32_t g[3])
{
    const float fn = (float)n;
    int32_t b[3];
    for (int a = 0; a < 3; ++a) {
        if (!(p[a] >= 0.0f) || !(p[a] < fn)) return -1;
        int32_t cell = (int32_t)floorf(p[a]);
        b[a] = cell / (n / g[a]);
    }
    return b[0] + g[0] * (b[1] + g[1] * b[2]);
}

/* Trilinear interpolation of voxel-centred samples with clamp-to-edge, in
 * float64: the plain definition, sum over the 8 corners of the product of the
 * per-axis weights. Weights come from u = clamp(q - 1/2, 0, n - 1),
 * i0 = min(floor(u), n - 2), f = u - i0. */
static void tri_setup(const float q[3], int32_t n, int32_t i0[3], double f[3])
{
    for (int a = 0; a < 3; ++a) {
        double u = (double)q[a] - 0.5;
        if (u < 0.0) u = 0.0;
        if (u > (double)(n - 1)) u = (double)(n - 1);
        int32_t i = (int32_t)floor(u);
        if (i > n - 2) i = n - 2;
        i0[a] = i;
        f[a] = u - (double)i;
    }
}

static double tri_scalar(const double *vol, int32_t n, const float q[3])
{
    int32_t i0[3];
    double f[3];
    tri_setup(q, n, i0, f);
    double s = 0.0;
    for (int c = 0; c < 8; ++c) {
        int32_t dx = c & 1, dy = (c >> 1) & 1, dz = (c >> 2) & 1;
        double w = (dx ? f[0] : 1.0 - f[0]) * (dy ? f[1] : 1.0 - f[1]) * (dz ? f[2] : 1.0 - f[2]);
        size_t idx = (size_t)(i0[0] + dx) + (size_t)n * ((size_t)(i0[1] + dy) + (size_t)n * (size_t)(i0[2] + dz));
        s += w * vol[idx];
    }
    return s;
}

/* Exposed for the interpolation pins (linear fields, voxel centres, clamping). */
double oracle_trilinear(const double *vol, int32_t n, float qx, float qy, float qz)
{
    float q[3] = {qx, qy, qz};
    return tri_scalar(vol, n, q);
}

/* ======================================================================
 * O3. Emission-absorption ray march through a bricked scalar volume.
 *
 * Each brick advances the rays it owns sample by sample while the samples stay
 * inside it, carrying the partial integral in the item (the pattern of the
 * volume renderers in Sec. 5.1-5.3: a forwarded ray packages its integration
 * state and continues in the next domain); on leaving it is forwarded to the
 * owner of its next sample, or finishes when it leaves the volume.
 *
 * Sample k of a ray: t_k = (k + 1/2) dt, p_k = fma(t_k, dir, org) in float32,
 * with org = fma(py, dv, fma(px, du, org0)). The sample density is
 * rho_k = V(p_k); with sigma_k = c * rho_k (c = kappa * dt),
 *     I = sum_k exp(-tau_k) (1 - exp(-sigma_k)) rho_k,   tau_k = sum_{j<k} sigma_j,
 * over the samples inside the volume (emission equal to density).
 * ====================================================================== */
typedef struct {
    float org0[3], du[3], dv[3], dir[3];
    int32_t width, height, n_samples, pad;
} orc_view;

static void ray_origin(const orc_view *v, int32_t px, int32_t py, float org[3])
{
    for (int a = 0; a < 3; ++a)
        org[a] = fmaf((float)py, v->dv[a], fmaf((float)px, v->du[a], v->org0[a]));
}

static void sample_pos(const float org[3], const float dir[3], float dt, int32_t k, float p[3])
{
    float t = ((float)k + 0.5f) * dt;
    for (int a = 0; a < 3; ++a) p[a] = fmaf(t, dir[a], org[a]);
}

static void ray_of(const orc_view *views, int64_t r, const orc_view **v, int32_t *px, int32_t *py)
{
    int64_t per = 0, base = 0;
    int32_t vi = 0;
    for (;;) {
        per = (int64_t)views[vi].width * views[vi].height;
        if (r < base + per) break;
        base += per;
        vi++;
    }
    *v = &views[vi];
    int64_t local = r - base;
    *px = (int32_t)(local % views[vi].width);
    *py = (int32_t)(local / views[vi].width);
}

/* The oracle's own work item: ray id, next sample, optical depth and the
 * partial integral in float64. */
typedef struct {
    int64_t ray;
    int32_t k;
    int32_t pad;
    double tau;
    double I;
} orc_ray;

typedef struct {
    int32_t n;
    int32_t g[3];
    float dt;
    float c;
} orc_ea_params;

/* Advance one ray inside domain d; returns the destination (ORC_DONE when it
 * leaves the volume or runs out of samples). Optionally records the number of
 * samples taken in this brick. */
static int32_t ea_advance(const double *vol, const orc_ea_params *P, const orc_view *v,
                          const float org[3], orc_ray *it, int32_t d)
{
    const double c = (double)P->c;
    for (;;) {
        if (it->k >= v->n_samples) return ORC_DONE;
        float p[3];
        sample_pos(org, v->dir, P->dt, it->k, p);
        int32_t e = owner_of(p, P->n, P->g);
        if (e < 0) return ORC_DONE;
        if (e != d) return e;
        double rho = tri_scalar(vol, P->n, p);
        double sigma = c * rho;
        it->I += exp(-it->tau) * (-expm1(-sigma)) * rho;
        it->tau += sigma;
        it->k++;
    }
}

/* First sample index inside the volume (the ray generator's job), or -1. */
static int32_t ea_first_inside(const orc_ea_params *P, const orc_view *v, const float org[3],
                               int32_t *owner)
{
    for (int32_t k = 0; k < v->n_samples; ++k) {
        float p[3];
        sample_pos(org, v->dir, P->dt, k, p);
        int32_t e = owner_of(p, P->n, P->g);
        if (e >= 0) { *owner = e; return k; }
    }
    return -1;
}

/*
 * O2 + O3: the round loop of Sec. 3.4 / 4.2.3 with per-domain queues.
 *
 * Round 0 generates one item per ray and sends it to the owner of its first
 * inside sample (rays that miss the volume finish with I = 0). Every later
 * round walks the domains in order and each domain's queue in order, advances
 * every item, and collects the emitted items in that order; the forward step
 * (O1) then regroups them by destination. The loop ends when no item is left
 * (the returned total of Sec. 3.4), or fails at max_rounds.
 *
 * Outputs (any may be NULL):
 *   image[r]        final integral per ray (0 for rays that miss)
 *   tau_out[r]      final optical depth per ray
 *   klast_out[r]    index one past the last inside sample (0 for misses)
 *   round_counts    [max_rounds][D] number of items per domain delivered by
 *                   each forward step (round 0 = after ray generation)
 *   queue_log       ray ids in queue order after every forward step,
 *                   concatenated over rounds; capacity queue_cap entries
 *   visit_log       [n_rays][visit_stride] domain ids each ray visited, -1 padded
 * Returns the number of forward steps taken, or a negative error.
 */
int oracle_ea_render(const double *vol, const orc_ea_params *P, const orc_view *views,
                     int32_t n_views, double *image, double *tau_out, int32_t *klast_out,
                     int32_t max_rounds, uint64_t *round_counts, int64_t *queue_log,
                     uint64_t queue_cap, uint64_t *queue_len, int32_t *visit_log,
                     int32_t visit_stride)
{
    const int32_t D = P->g[0] * P->g[1] * P->g[2];
    int64_t n_rays = 0;
    for (int32_t i = 0; i < n_views; ++i) n_rays += (int64_t)views[i].width * views[i].height;

    orc_ray *O = (orc_ray *)malloc(sizeof(orc_ray) * (size_t)(n_rays ? n_rays : 1));
    orc_ray *Q = (orc_ray *)malloc(sizeof(orc_ray) * (size_t)(n_rays ? n_rays : 1));
    int32_t *odest = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n_rays ? n_rays : 1));
    uint64_t *counts = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)D);
    uint64_t *offs = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(D + 1));
    int32_t *nvis = (int32_t *)calloc((size_t)(n_rays ? n_rays : 1), sizeof(int32_t));
    if (!O || !Q || !odest || !counts || !offs || !nvis) return -2;
    if (visit_log)
        for (int64_t i = 0; i < n_rays * visit_stride; ++i) visit_log[i] = -1;
    uint64_t qlen = 0;

    /* Round 0: ray generation; one output slot per ray. */
    uint64_t n_out = 0;
    for (int64_t r = 0; r < n_rays; ++r) {
        const orc_view *v;
        int32_t px, py, own = -1;
        ray_of(views, r, &v, &px, &py);
        float org[3];
        ray_origin(v, px, py, org);
        int32_t k0 = ea_first_inside(P, v, org, &own);
        orc_ray it = {r, k0 < 0 ? 0 : k0, 0, 0.0, 0.0};
        O[n_out] = it;
        odest[n_out] = (k0 < 0) ? ORC_DONE : own;
        n_out++;
        if (k0 < 0) {
            if (image) image[r] = 0.0;
            if (tau_out) tau_out[r] = 0.0;
            if (klast_out) klast_out[r] = 0;
        }
    }

    int32_t rounds = 0;
    uint64_t total = 0;
    for (;;) {
        /* Forward step (O1) on the emitted slots. */
        oracle_multisplit(n_out, (uint32_t)sizeof(orc_ray), (const uint8_t *)O, odest, D,
                          (uint8_t *)Q, counts, offs, NULL, NULL);
        total = offs[D];
        if (rounds >= max_rounds) { rounds = -6; break; }
        if (round_counts)
            for (int32_t e = 0; e < D; ++e) round_counts[(size_t)rounds * D + e] = counts[e];
        for (uint64_t i = 0; i < total; ++i) {
            if (queue_log && qlen < queue_cap) queue_log[qlen] = Q[i].ray;
            qlen++;
        }
        /* Record the visit of every delivered item. */
        for (int32_t d = 0; d < D; ++d)
            for (uint64_t i = offs[d]; i < offs[d + 1]; ++i) {
                int64_t r = Q[i].ray;
                if (visit_log && nvis[r] < visit_stride) visit_log[r * visit_stride + nvis[r]] = d;
                nvis[r]++;
            }
        rounds++;
        if (total == 0) break;

        /* Domain kernels: walk domains in order, items in queue order; the
         * item at queue position i emits into output slot i. */
        for (int32_t d = 0; d < D; ++d) {
            const int64_t b = (int64_t)offs[d], end = (int64_t)offs[d + 1];
#pragma omp parallel for schedule(dynamic, 64) num_threads(g_threads) if (g_threads > 1)
            for (int64_t i = b; i < end; ++i) {
                orc_ray it = Q[i];
                const orc_view *v;
                int32_t px, py;
                ray_of(views, it.ray, &v, &px, &py);
                float org[3];
                ray_origin(v, px, py, org);
                int32_t e = ea_advance(vol, P, v, org, &it, d);
                O[i] = it;
                odest[i] = e;
                if (e == ORC_DONE) {
                    if (image) image[it.ray] = it.I;
                    if (tau_out) tau_out[it.ray] = it.tau;
                    if (klast_out) klast_out[it.ray] = it.k;
                }
            }
        }
        n_out = total;
    }
    if (queue_len) *queue_len = qlen;
    free(O); free(Q); free(odest); free(counts); free(offs); free(nvis);
    return rounds;
}

/*
 * Unpartitioned brute force: march every ray through all of its samples in
 * one go, never forwarding. The paper states that forwarding changes neither
 * which rays are traced nor what they compute (Sec. 5.1), so the partitioned
 * round loop must reproduce this bit for bit. The visit sequence is the
 * run-length-compressed sequence of owning bricks along the samples.
 * ray_ids selects a subset of rays (NULL = all, in order); outputs are indexed
 * by position in that list.
 */
int oracle_ea_brute(const double *vol, const orc_ea_params *P, const orc_view *views,
                    int32_t n_views, const int64_t *ray_ids, int64_t n_ids, double *image,
                    double *tau_out, int32_t *visit_log, int32_t visit_stride)
{
    const double c = (double)P->c;
    int64_t n_rays = 0;
    for (int32_t i = 0; i < n_views; ++i) n_rays += (int64_t)views[i].width * views[i].height;
    if (!ray_ids) n_ids = n_rays;
#pragma omp parallel for schedule(dynamic, 256) num_threads(g_threads) if (g_threads > 1)
    for (int64_t q = 0; q < n_ids; ++q) {
        int64_t r = ray_ids ? ray_ids[q] : q;
        const orc_view *v;
        int32_t px, py;
        ray_of(views, r, &v, &px, &py);
        float org[3];
        ray_origin(v, px, py, org);
        double tau = 0.0, I = 0.0;
        int32_t last = -2, nv = 0;
        if (visit_log)
            for (int32_t s = 0; s < visit_stride; ++s) visit_log[q * visit_stride + s] = -1;
        for (int32_t k = 0; k < v->n_samples; ++k) {
            float p[3];
            sample_pos(org, v->dir, P->dt, k, p);
            int32_t e = owner_of(p, P->n, P->g);
            if (e < 0) continue;
            if (e != last) {
                if (visit_log && nv < visit_stride) visit_log[q * visit_stride + nv] = e;
                nv++;
                last = e;
            }
            double rho = tri_scalar(vol, P->n, p);
            double sigma = c * rho;
            I += exp(-tau) * (-expm1(-sigma)) * rho;
            tau += sigma;
        }
        if (image) image[q] = I;
        if (tau_out) tau_out[q] = tau;
    }
    return 0;
}

/* Per-sample densities of one ray (inside samples only, in order), for the
 * compositing-identity pin. Returns the number written. */
int32_t oracle_ea_ray_samples(const double *vol, const orc_ea_params *P, const orc_view *views,
                              int32_t n_views, int64_t ray, double *rho_out, int32_t cap)
{
    const orc_view *v;
    int32_t px, py, m = 0;
    (void)n_views;
    ray_of(views, ray, &v, &px, &py);
    float org[3];
    ray_origin(v, px, py, org);
    for (int32_t k = 0; k < v->n_samples; ++k) {
        float p[3];
        sample_pos(org, v->dir, P->dt, k, p);
        if (owner_of(p, P->n, P->g) < 0) continue;
        if (m < cap) rho_out[m] = tri_scalar(vol, P->n, p);
        m++;
    }
    return m;
}

/* ======================================================================
 * O6. Gradient of the image loss L = sum_r (I_r - I*_r)^2 with respect to the
 * voxel densities (the adjoint of O3), float64.
 *
 * With T_k = exp(-tau_k), a_k = 1 - exp(-sigma_k) and I = sum_k T_k a_k rho_k,
 *   dI/drho_k = T_k [ a_k + c exp(-sigma_k) (rho_k - B_{k+1}) ],
 * where B_{k+1} = sum_{j>k} (T_j / T_{k+1}) a_j rho_j is the part of the
 * integral behind sample k, obeying B_k = a_k rho_k + (1 - a_k) B_{k+1},
 * B_end = 0. Densities are trilinear in the voxels, so
 *   dL/dV_v = sum_r 2 (I_r - I*_r) sum_k dI_r/drho_k w_v(p_k).
 * Each ray is swept front to back (storing tau_k and rho_k), then back to front.
 * ray_ids selects a subset (NULL = all rays); target is indexed by ray id.
 * ====================================================================== */
int oracle_ea_loss_grad(const double *vol, const orc_ea_params *P, const orc_view *views,
                        int32_t n_views, const double *target, const int64_t *ray_ids,
                        int64_t n_ids, double *image, double *grad, double *loss)
{
    const double c = (double)P->c;
    const int32_t n = P->n;
    int64_t n_rays = 0;
    int32_t maxs = 0;
    for (int32_t i = 0; i < n_views; ++i) {
        n_rays += (int64_t)views[i].width * views[i].height;
        if (views[i].n_samples > maxs) maxs = views[i].n_samples;
    }
    if (!ray_ids) n_ids = n_rays;
    double *tau_k = (double *)malloc(sizeof(double) * (size_t)(maxs + 1));
    double *rho_k = (double *)malloc(sizeof(double) * (size_t)(maxs + 1));
    int32_t *ks = (int32_t *)malloc(sizeof(int32_t) * (size_t)(maxs + 1));
    if (!tau_k || !rho_k || !ks) return -2;
    double L = 0.0;
    for (int64_t q = 0; q < n_ids; ++q) {
        int64_t r = ray_ids ? ray_ids[q] : q;
        const orc_view *v;
        int32_t px, py;
        ray_of(views, r, &v, &px, &py);
        float org[3];
        ray_origin(v, px, py, org);
        double tau = 0.0, I = 0.0;
        int32_t m = 0;
        for (int32_t k = 0; k < v->n_samples; ++k) {
            float p[3];
            sample_pos(org, v->dir, P->dt, k, p);
            if (owner_of(p, n, P->g) < 0) continue;
            double rho = tri_scalar(vol, n, p);
            double sigma = c * rho;
            tau_k[m] = tau;
            rho_k[m] = rho;
            ks[m] = k;
            m++;
            I += exp(-tau) * (-expm1(-sigma)) * rho;
            tau += sigma;
        }
        if (image) image[q] = I;
        double resid = I - target[r];
        L += resid * resid;
        if (!grad) continue;
        double gI = 2.0 * resid;
        double B = 0.0;
        for (int32_t s = m - 1; s >= 0; --s) {
            double rho = rho_k[s], sigma = c * rho;
            double T = exp(-tau_k[s]);
            double a = -expm1(-sigma);
            double dIdrho = T * (a + c * exp(-sigma) * (rho - B));
            float p[3];
            sample_pos(org, v->dir, P->dt, ks[s], p);
            int32_t i0[3];
            double f[3];
            tri_setup(p, n, i0, f);
            for (int cc = 0; cc < 8; ++cc) {
                int32_t dx = cc & 1, dy = (cc >> 1) & 1, dz = (cc >> 2) & 1;
                double w = (dx ? f[0] : 1.0 - f[0]) * (dy ? f[1] : 1.0 - f[1]) * (dz ? f[2] : 1.0 - f[2]);
                size_t idx = (size_t)(i0[0] + dx) + (size_t)n * ((size_t)(i0[1] + dy) + (size_t)n * (size_t)(i0[2] + dz));
                grad[idx] += gI * dIdrho * w;
            }
            B = a * rho + (1.0 - a) * B;
        }
    }
    if (loss) *loss = L;
    free(tau_k); free(rho_k); free(ks);
    return 0;
}

/* ======================================================================
 * O4. RK4 streamlines through a bricked vector field (Sec. 5.4).
 *
 * One item per particle: id, position (float3) and step count. A brick
 * integrates its particles with classical RK4 (step h) while they stay inside
 * it; a particle finishes when a step does not move it, when it leaves the
 * field, or at max_steps; otherwise it is forwarded to the brick that now owns
 * it. All of this decides integers (routing, step counts), so it runs in
 * float32 with each operation written out:
 *   k1 = V(p), k2 = V(p + (h/2) k1), k3 = V(p + (h/2) k2), k4 = V(p + h k3)
 *   s = k1 + 2 k2 + 2 k3 + k4 (as fma(2,k2,k1), fma(2,k3,.), + k4)
 *   p' = fma(h/6, s, p)                       componentwise.
 * V is float32 trilinear interpolation of the voxel-centred field with
 * clamp-to-edge, lerping along x, then y, then z, lerp(a,b,t) = fma(t, b-a, a).
 * ====================================================================== */
typedef struct {
    int32_t n;
    int32_t g[3];
    float h;
    int32_t max_steps;
} orc_sl_params;

enum { ORC_SL_LIVE = 0, ORC_SL_STAGNANT = 1, ORC_SL_EXITED = 2, ORC_SL_MAXSTEPS = 3 };

static float lerpf(float a, float b, float t) { return fmaf(t, b - a, a); }

static void tri_vec3(const float *field, int32_t n, const float q[3], float out[3])
{
    int32_t i0[3];
    float f[3];
    for (int a = 0; a < 3; ++a) {
        float u = q[a] - 0.5f;
        u = fminf(fmaxf(u, 0.0f), (float)(n - 1));
        int32_t i = (int32_t)floorf(u);
        if (i > n - 2) i = n - 2;
        i0[a] = i;
        f[a] = u - (float)i;
    }
#define FV(dx, dy, dz, comp) field[3 * ((size_t)(i0[0] + (dx)) + (size_t)n * ((size_t)(i0[1] + (dy)) + (size_t)n * (size_t)(i0[2] + (dz)))) + (comp)]
    for (int comp = 0; comp < 3; ++comp) {
        float x00 = lerpf(FV(0, 0, 0, comp), FV(1, 0, 0, comp), f[0]);
        float x10 = lerpf(FV(0, 1, 0, comp), FV(1, 1, 0, comp), f[0]);
        float x01 = lerpf(FV(0, 0, 1, comp), FV(1, 0, 1, comp), f[0]);
        float x11 = lerpf(FV(0, 1, 1, comp), FV(1, 1, 1, comp), f[0]);
        float y0 = lerpf(x00, x10, f[1]);
        float y1 = lerpf(x01, x11, f[1]);
        out[comp] = lerpf(y0, y1, f[2]);
    }
#undef FV
}

/* Exposed for the sampler pins (linear fields, clamp band, component order). */
void oracle_tri_vec3(const float *field, int32_t n, float qx, float qy, float qz, float *out)
{
    const float q[3] = {qx, qy, qz};
    tri_vec3(field, n, q, out);
}

/* One RK4 step from p into pn. */
static void rk4_step(const float *field, int32_t n, float h, const float p[3], float pn[3])
{
    const float hh = h * 0.5f;
    const float h6 = (float)((double)h / 6.0);
    float k1[3], k2[3], k3[3], k4[3], q[3];
    tri_vec3(field, n, p, k1);
    for (int a = 0; a < 3; ++a) q[a] = fmaf(hh, k1[a], p[a]);
    tri_vec3(field, n, q, k2);
    for (int a = 0; a < 3; ++a) q[a] = fmaf(hh, k2[a], p[a]);
    tri_vec3(field, n, q, k3);
    for (int a = 0; a < 3; ++a) q[a] = fmaf(h, k3[a], p[a]);
    tri_vec3(field, n, q, k4);
    for (int a = 0; a < 3; ++a) {
        float s = fmaf(2.0f, k2[a], k1[a]);
        s = fmaf(2.0f, k3[a], s);
        s = s + k4[a];
        pn[a] = fmaf(h6, s, p[a]);
    }
}

typedef struct {
    int32_t id;
    int32_t steps;
    float p[3];
    int32_t pad;
} orc_particle;

/* Advance one particle inside brick d. Returns its destination; on finish
 * sets *reason. With cap > 0, at most cap RK4 steps are taken and a particle
 * still inside d is then forwarded to d itself; cap = 1 is the paper's one
 * update per round (Sec. 5.4), cap = 0 integrates until the particle leaves. */
static int32_t sl_advance(const float *field, const orc_sl_params *P, orc_particle *it,
                          int32_t d, int32_t cap, int32_t *reason)
{
    for (int32_t taken = 1;; ++taken) {
        float pn[3];
        rk4_step(field, P->n, P->h, it->p, pn);
        it->steps++;
        int same = memcmp(pn, it->p, sizeof(pn)) == 0;
        memcpy(it->p, pn, sizeof(pn));
        if (same) { *reason = ORC_SL_STAGNANT; return ORC_DONE; }
        int32_t e = owner_of(pn, P->n, P->g);
        if (e < 0) { *reason = ORC_SL_EXITED; return ORC_DONE; }
        if (it->steps >= P->max_steps) { *reason = ORC_SL_MAXSTEPS; return ORC_DONE; }
        if (e != d || (cap > 0 && taken >= cap)) return e;
    }
}

/*
 * O2 + O4: the streamline round loop. Round 0 sends every seed to its owning
 * brick (seeds outside the field finish immediately with 0 steps, reason
 * "exited"). Outputs per particle id: endpoint, step count, finish reason.
 * round_counts / queue_log (particle ids) / visit_log as in oracle_ea_render.
 */
int oracle_streamlines(const float *field, const orc_sl_params *P, const float *seeds,
                       int64_t n_seeds, int32_t steps_per_visit, float *endpoint, int32_t *steps,
                       int32_t *reason, int32_t max_rounds, uint64_t *round_counts,
                       int32_t *queue_log, uint64_t queue_cap, uint64_t *queue_len,
                       int32_t *visit_log, int32_t visit_stride)
{
    const int32_t D = P->g[0] * P->g[1] * P->g[2];
    size_t cap = (size_t)(n_seeds ? n_seeds : 1);
    orc_particle *O = (orc_particle *)malloc(sizeof(orc_particle) * cap);
    orc_particle *Q = (orc_particle *)malloc(sizeof(orc_particle) * cap);
    int32_t *odest = (int32_t *)malloc(sizeof(int32_t) * cap);
    uint64_t *counts = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)D);
    uint64_t *offs = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(D + 1));
    int32_t *nvis = (int32_t *)calloc(cap, sizeof(int32_t));
    if (!O || !Q || !odest || !counts || !offs || !nvis) return -2;
    if (visit_log)
        for (int64_t i = 0; i < n_seeds * visit_stride; ++i) visit_log[i] = -1;
    uint64_t qlen = 0, n_out = 0;

    for (int64_t i = 0; i < n_seeds; ++i) {
        orc_particle it;
        memset(&it, 0, sizeof(it));
        it.id = (int32_t)i;
        memcpy(it.p, seeds + 3 * i, sizeof(it.p));
        int32_t e = owner_of(it.p, P->n, P->g);
        O[n_out] = it;
        odest[n_out] = e;
        n_out++;
        if (e < 0) {
            memcpy(endpoint + 3 * i, it.p, sizeof(it.p));
            steps[i] = 0;
            if (reason) reason[i] = ORC_SL_EXITED;
        }
    }
    int32_t rounds = 0;
    for (;;) {
        oracle_multisplit(n_out, (uint32_t)sizeof(orc_particle), (const uint8_t *)O, odest, D,
                          (uint8_t *)Q, counts, offs, NULL, NULL);
        uint64_t total = offs[D];
        if (rounds >= max_rounds) { rounds = -6; break; }
        if (round_counts)
            for (int32_t e = 0; e < D; ++e) round_counts[(size_t)rounds * D + e] = counts[e];
        for (uint64_t i = 0; i < total; ++i) {
            if (queue_log && qlen < queue_cap) queue_log[qlen] = Q[i].id;
            qlen++;
        }
        for (int32_t d = 0; d < D; ++d)
            for (uint64_t i = offs[d]; i < offs[d + 1]; ++i) {
                int32_t id = Q[i].id;
                if (visit_log && nvis[id] < visit_stride) visit_log[(size_t)id * visit_stride + nvis[id]] = d;
                nvis[id]++;
            }
        rounds++;
        if (total == 0) break;
        /* the particle at queue position i emits into output slot i */
        for (int32_t d = 0; d < D; ++d) {
            const int64_t b = (int64_t)offs[d], end = (int64_t)offs[d + 1];
#pragma omp parallel for schedule(dynamic, 64) num_threads(g_threads) if (g_threads > 1)
            for (int64_t i = b; i < end; ++i) {
                orc_particle it = Q[i];
                int32_t why = ORC_SL_LIVE;
                int32_t e = sl_advance(field, P, &it, d, steps_per_visit, &why);
                O[i] = it;
                odest[i] = e;
                if (e == ORC_DONE) {
                    memcpy(endpoint + 3 * (size_t)it.id, it.p, sizeof(it.p));
                    steps[it.id] = it.steps;
                    if (reason) reason[it.id] = why;
                }
            }
        }
        n_out = total;
    }
    if (queue_len) *queue_len = qlen;
    free(O); free(Q); free(odest); free(counts); free(offs); free(nvis);
    return rounds;
}

/* Unpartitioned brute force: integrate every seed to completion without ever
 * forwarding; the visit sequence is the run-length-compressed owner sequence
 * of the positions the particle occupies between steps. */
int oracle_streamlines_brute(const float *field, const orc_sl_params *P, const float *seeds,
                             int64_t n_seeds, float *endpoint, int32_t *steps, int32_t *reason,
                             int32_t *visit_log, int32_t visit_stride)
{
#pragma omp parallel for schedule(dynamic, 64) num_threads(g_threads) if (g_threads > 1)
    for (int64_t i = 0; i < n_seeds; ++i) {
        float p[3];
        memcpy(p, seeds + 3 * i, sizeof(p));
        int32_t st = 0, why = ORC_SL_LIVE, nv = 0;
        if (visit_log)
            for (int32_t s = 0; s < visit_stride; ++s) visit_log[(size_t)i * visit_stride + s] = -1;
        int32_t e = owner_of(p, P->n, P->g);
        if (e < 0) why = ORC_SL_EXITED;
        int32_t last = -2;
        while (why == ORC_SL_LIVE) {
            if (e != last) {
                if (visit_log && nv < visit_stride) visit_log[(size_t)i * visit_stride + nv] = e;
                nv++;
                last = e;
            }
            float pn[3];
            rk4_step(field, P->n, P->h, p, pn);
            st++;
            int same = memcmp(pn, p, sizeof(pn)) == 0;
            memcpy(p, pn, sizeof(p));
            if (same) { why = ORC_SL_STAGNANT; break; }
            e = owner_of(p, P->n, P->g);
            if (e < 0) { why = ORC_SL_EXITED; break; }
            if (st >= P->max_steps) { why = ORC_SL_MAXSTEPS; break; }
        }
        memcpy(endpoint + 3 * i, p, sizeof(p));
        steps[i] = st;
        if (reason) reason[i] = why;
    }
    return 0;
}

/* ======================================================================
 * O7. Delta-tracking volume path tracing over bricks.
 *
 * The volume path tracer of Sec. 5.1 traces rays through the local brick with
 * delta (Woodcock) tracking; a ray that scatters is forwarded to its own
 * rank for the next round, a ray that leaves the brick to the rank owning
 * the point it reached, and a shading event may spawn a shadow ray beside the
 * bounced ray (Sec. 5.1 figure, Sec. 5.2 Lander with volumetric shadows,
 * Sec. 6.3 on one item spawning several). Reading used here:
 *
 *   medium    sigma_t(x) = kappa * V(x), V the float32 trilinear density;
 *             one global majorant smax >= kappa * max V, so the sequence of
 *             tentative collisions along a ray does not depend on the bricks;
 *   path      tentative points p += s d, s = -ln(1 - u) / smax; at a
 *             tentative point inside brick D a path collides for real when
 *             u * smax < sigma_t(p) (u a fresh draw), else continues;
 *             leaving the volume ends it (black background);
 *   scatter   weight w *= albedo; a shadow ray toward the light starts at the
 *             collision point with weight w * radiance / (4 pi) (isotropic
 *             phase); the path takes a new isotropic direction (Marsaglia
 *             1972) unless it has scattered max_bounce times;
 *   shadow    ratio tracking: at each tentative point the weight is
 *             multiplied by 1 - sigma_t(p) / smax; on leaving the volume its
 *             weight is the contribution of that scattering event;
 *   output    contrib[path * max_bounce + b] for the shadow ray of the b-th
 *             scattering event (0 where there was none);
 *   slots     fixed fan-out 2: the item in input slot i owns output slots 2i
 *             (the item itself, or the shadow ray of its scattering event)
 *             and 2i + 1 (the bounced path, or DONE);
 *   random    Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC 2011), key
 *             (seed, path id), counter (stream, draw index, 0, 0), word 0,
 *             u = (word >> 8) * 2^-24; stream 2b is the path after b
 *             scattering events, 2b + 1 the shadow ray of event b.
 * Positions, draws and every decision are float32 with each operation
 * written out; weights are float64.
 * ====================================================================== */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        const uint32_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static float f32_of(uint32_t b) { float f; memcpy(&f, &b, 4); return f; }
static uint32_t bits_of(float f) { uint32_t b; memcpy(&b, &f, 4); return b; }

/* Natural logarithm of a normal float32 x in (0, 1], from x = m 2^e with
 * m in [sqrt(1/2), sqrt(2)) and ln m = 2 atanh(s), s = (m - 1) / (m + 1),
 * summed as 2s + 2s (s^2/3 + s^4/5 + ... + s^12/13) (|s| < 0.172, so the
 * first omitted term is below 2^-40 relative); ln x = e ln2 + ln m with ln2
 * split in two parts. Each operation is one float32 rounding. */
float oracle_dt_logf(float x)
{
    const uint32_t b = bits_of(x);
    int32_t e = (int32_t)(b >> 23) - 127;
    float m = f32_of((b & 0x007FFFFFu) | 0x3F800000u);
    if (m > 1.41421354f) {
        m = m * 0.5f;
        e += 1;
    }
    const float f = m - 1.0f;
    const float s = f / (2.0f + f);
    const float z = s * s;
    float q = fmaf(z, 1.0f / 13.0f, 1.0f / 11.0f);
    q = fmaf(z, q, 1.0f / 9.0f);
    q = fmaf(z, q, 1.0f / 7.0f);
    q = fmaf(z, q, 1.0f / 5.0f);
    q = fmaf(z, q, 1.0f / 3.0f);
    q = q * z;
    const float s2 = s + s;
    const float lnm = fmaf(s2, q, s2);
    const float fe = (float)e;
    return fmaf(fe, 0.693145751953125f, fmaf(fe, 1.42860677e-06f, lnm));
}

typedef struct {
    int32_t n;
    int32_t g[3];
    float kappa, smax, albedo;
    float light[3];
    float radiance;
    int32_t max_bounce;
    uint32_t seed;
} orc_dt_params;

enum { DT_PATH = 0, DT_SHADOW = 1 };
/* tentative points evaluated per brick visit before the item is forwarded to
 * its own brick (its walk then continues unchanged in the next round) */
#define DT_MAX_POINTS 65536u

typedef struct {
    float p[3], d[3];
    double w;
    int32_t path;
    uint32_t stream, count;
    int32_t bounce, kind;
} orc_dt_item;

static float dt_draw(const orc_dt_params *P, orc_dt_item *it)
{
    const uint32_t ctr[4] = {it->stream, it->count, 0u, 0u};
    const uint32_t key[2] = {P->seed, (uint32_t)it->path};
    uint32_t o[4];
    oracle_philox4x32_10(ctr, key, o);
    it->count++;
    return (float)(o[0] >> 8) * 5.9604644775390625e-08f; /* 2^-24 */
}

static void dt_fly(const orc_dt_params *P, orc_dt_item *it)
{
    const float s = -oracle_dt_logf(1.0f - dt_draw(P, it)) / P->smax;
    for (int a = 0; a < 3; ++a) it->p[a] = fmaf(s, it->d[a], it->p[a]);
}

/* float32 trilinear, clamp-to-edge, lerping x, then y, then z */
static float dt_density(const float *vol, int32_t n, const float q[3])
{
    int32_t i0[3];
    float f[3];
    const float hi = (float)(n - 1);
    for (int a = 0; a < 3; ++a) {
        const float u = fminf(fmaxf(q[a] - 0.5f, 0.0f), hi);
        int32_t i = (int32_t)floorf(u);
        if (i > n - 2) i = n - 2;
        i0[a] = i;
        f[a] = u - (float)i;
    }
    const size_t sy = (size_t)n, sz = (size_t)n * n;
    const float *b = vol + (size_t)i0[0] + sy * (size_t)i0[1] + sz * (size_t)i0[2];
    const float x00 = lerpf(b[0], b[1], f[0]), x01 = lerpf(b[sy], b[sy + 1], f[0]);
    const float x10 = lerpf(b[sz], b[sz + 1], f[0]), x11 = lerpf(b[sz + sy], b[sz + sy + 1], f[0]);
    return lerpf(lerpf(x00, x01, f[1]), lerpf(x10, x11, f[1]), f[2]);
}

/* Exposed for the sampler pins (linear data, clamp band, strides). */
float oracle_dt_density(const float *vol, int32_t n, float qx, float qy, float qz)
{
    const float q[3] = {qx, qy, qz};
    return dt_density(vol, n, q);
}

static void dt_isotropic(const orc_dt_params *P, orc_dt_item *it)
{
    for (int tries = 0; tries < 64; ++tries) {
        const float x1 = fmaf(2.0f, dt_draw(P, it), -1.0f);
        const float x2 = fmaf(2.0f, dt_draw(P, it), -1.0f);
        const float s = fmaf(x1, x1, x2 * x2);
        if (s < 1.0f && s > 0.0f) {
            const float t = 2.0f * sqrtf(1.0f - s);
            it->d[0] = x1 * t;
            it->d[1] = x2 * t;
            it->d[2] = fmaf(-2.0f, s, 1.0f);
            return;
        }
    }
    it->d[0] = 0.0f; it->d[1] = 0.0f; it->d[2] = 1.0f;
}

/* Primary ray of path r: entry into [0,n)^3 by the slab test, then its
 * first tentative point. Returns the owner of that point (-1: no collision
 * possible, the path is done). */
static int32_t dt_raygen(const orc_dt_params *P, const orc_view *views, int64_t r, orc_dt_item *it)
{
    const orc_view *v;
    int32_t px, py;
    ray_of(views, r, &v, &px, &py);
    float o[3];
    ray_origin(v, px, py, o);
    memset(it, 0, sizeof(*it));
    it->path = (int32_t)r;
    it->w = 1.0;
    it->kind = DT_PATH;
    const float fn = (float)P->n;
    float t0 = 0.0f, t1 = INFINITY;
    for (int a = 0; a < 3; ++a) {
        it->d[a] = v->dir[a];
        if (v->dir[a] != 0.0f) {
            const float ta = (0.0f - o[a]) / v->dir[a], tb = (fn - o[a]) / v->dir[a];
            t0 = fmaxf(t0, fminf(ta, tb));
            t1 = fminf(t1, fmaxf(ta, tb));
        } else if (!(o[a] >= 0.0f && o[a] < fn)) {
            return -1;
        }
    }
    if (!(t0 < t1)) return -1;
    for (int a = 0; a < 3; ++a) it->p[a] = fmaf(t0, it->d[a], o[a]);
    dt_fly(P, it);
    return owner_of(it->p, P->n, P->g);
}

/* One visit of item `it` to brick `d` (its tentative point lies in d). Writes
 * the content of the item's two output slots: out[0] / dest[0] and
 * out[1] / dest[1] (ORC_DONE when a slot carries nothing). */
static void dt_visit(const float *vol, const orc_dt_params *P, int32_t d, orc_dt_item it, double *contrib,
                     orc_dt_item out[2], int32_t dest[2])
{
    dest[0] = ORC_DONE;
    dest[1] = ORC_DONE;
    for (uint32_t points = 0;; ++points) {
        if (points == DT_MAX_POINTS) { /* bounded visit: continue next round in the same brick */
            out[0] = it;
            dest[0] = d;
            return;
        }
        const float sigma = P->kappa * dt_density(vol, P->n, it.p);
        if (it.kind == DT_PATH) {
            const float u = dt_draw(P, &it);
            if (u * P->smax < sigma) {
                const int32_t b = it.bounce;
                const double w = it.w * (double)P->albedo;
                orc_dt_item sh = it;
                sh.kind = DT_SHADOW;
                sh.stream = 2u * (uint32_t)b + 1u;
                sh.count = 0;
                sh.w = w * (double)P->radiance / (4.0 * 3.14159265358979323846);
                for (int a = 0; a < 3; ++a) sh.d[a] = P->light[a];
                dt_fly(P, &sh);
                const int32_t es = owner_of(sh.p, P->n, P->g);
                if (es < 0) contrib[(size_t)sh.path * P->max_bounce + b] = sh.w;
                else { out[0] = sh; dest[0] = es; }
                if (b + 1 < P->max_bounce) {
                    orc_dt_item pa = it;
                    pa.bounce = b + 1;
                    pa.stream = 2u * (uint32_t)(b + 1);
                    pa.count = 0;
                    pa.w = w;
                    dt_isotropic(P, &pa);
                    dt_fly(P, &pa);
                    const int32_t ep = owner_of(pa.p, P->n, P->g);
                    if (ep >= 0) { out[1] = pa; dest[1] = ep; }
                }
                return;
            }
        } else {
            it.w *= 1.0 - (double)sigma / (double)P->smax;
        }
        dt_fly(P, &it);
        const int32_t e = owner_of(it.p, P->n, P->g);
        if (e == d) continue;
        if (e < 0) {
            if (it.kind == DT_SHADOW) contrib[(size_t)it.path * P->max_bounce + it.bounce] = it.w;
            return;
        }
        out[0] = it;
        dest[0] = e;
        return;
    }
}

/* The round loop for delta tracking (O2 with fan-out 2): round 0 emits every
 * path to the owner of its first tentative point; each later round visits
 * the domains in order and their queued items in order, and the 2 slots of
 * each item go through the stable counting sort of O1. Logged per forward
 * step: counts per domain, and every queued item as 11 words (p, d as float32
 * bits; path, stream, count, bounce, kind) in queue order. */
int oracle_dt_render(const float *vol, const orc_dt_params *P, const orc_view *views, int32_t n_views,
                     double *contrib, double *weights_log, int32_t max_rounds, uint64_t *round_counts,
                     uint32_t *queue_log, uint64_t queue_cap, uint64_t *queue_len)
{
    const int32_t D = P->g[0] * P->g[1] * P->g[2];
    int64_t n_paths = 0;
    for (int32_t v = 0; v < n_views; ++v) n_paths += (int64_t)views[v].width * views[v].height;
    memset(contrib, 0, sizeof(double) * (size_t)n_paths * P->max_bounce);
    /* a path has at most itself and one shadow ray per scattering event alive */
    const size_t live = (size_t)n_paths * (size_t)(P->max_bounce + 1) + 1;
    orc_dt_item *slots = (orc_dt_item *)malloc(sizeof(orc_dt_item) * 2 * live);
    orc_dt_item *queue = (orc_dt_item *)malloc(sizeof(orc_dt_item) * live);
    int32_t *sdest = (int32_t *)malloc(sizeof(int32_t) * 2 * live);
    uint64_t *counts = (uint64_t *)calloc((size_t)D, sizeof(uint64_t));
    uint64_t *offs = (uint64_t *)calloc((size_t)D + 1, sizeof(uint64_t));
    if (!slots || !queue || !sdest || !counts || !offs) return -2;
    uint64_t n_slots = (uint64_t)n_paths, qlen = 0;
    for (int64_t r = 0; r < n_paths; ++r) sdest[r] = dt_raygen(P, views, r, &slots[r]);
    int32_t rounds = 0;
    for (;;) {
        /* forward step: stable counting sort of the slots by destination */
        for (int32_t e = 0; e < D; ++e) counts[e] = 0;
        for (uint64_t i = 0; i < n_slots; ++i)
            if (sdest[i] >= 0) counts[sdest[i]]++;
        offs[0] = 0;
        for (int32_t e = 0; e < D; ++e) offs[e + 1] = offs[e] + counts[e];
        uint64_t *fill = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)D);
        for (int32_t e = 0; e < D; ++e) fill[e] = offs[e];
        for (uint64_t i = 0; i < n_slots; ++i)
            if (sdest[i] >= 0) queue[fill[sdest[i]]++] = slots[i];
        free(fill);
        const uint64_t total = offs[D];
        if (total >= live) return -3; /* cannot happen: see the bound above */
        if (round_counts && rounds < max_rounds)
            for (int32_t e = 0; e < D; ++e) round_counts[(size_t)rounds * D + e] = counts[e];
        for (uint64_t i = 0; i < total; ++i, ++qlen) {
            if (!queue_log || qlen >= queue_cap) continue;
            uint32_t *q = queue_log + qlen * 11;
            for (int a = 0; a < 3; ++a) { q[a] = bits_of(queue[i].p[a]); q[3 + a] = bits_of(queue[i].d[a]); }
            q[6] = (uint32_t)queue[i].path; q[7] = queue[i].stream; q[8] = queue[i].count;
            q[9] = (uint32_t)queue[i].bounce; q[10] = (uint32_t)queue[i].kind;
            if (weights_log) weights_log[qlen] = queue[i].w;
        }
        rounds++;
        if (total == 0) break;
        if (rounds >= max_rounds) { rounds = -1; break; }
        /* domain kernels, fan-out 2 (each (path, event) contribution is
         * written by the one item that finishes it) */
        for (int32_t e = 0; e < D; ++e) {
            const int64_t b = (int64_t)offs[e], end = (int64_t)offs[e + 1];
#pragma omp parallel for schedule(dynamic, 64) num_threads(g_threads) if (g_threads > 1)
            for (int64_t i = b; i < end; ++i)
                dt_visit(vol, P, e, queue[i], contrib, &slots[2 * i], &sdest[2 * i]);
        }
        n_slots = 2 * total;
    }
    if (queue_len) *queue_len = qlen;
    free(slots); free(queue); free(sdest); free(counts); free(offs);
    return rounds;
}

/* ======================================================================
 * O8. Multi-context, multi-phase forwarding: one step of the distributed
 * Barnes-Hut N-body code of Sec. 5.5, with the three item types of that
 * section's listing, each in its own context:
 *   Particle         {pos[3], vel[3], force[3], mass}          40 bytes
 *   VirtualParticle  {pos[3], mass, smax, sourceRank}          24 bytes
 *   RefinementReq    {senderRank}                               4 bytes
 *
 * Readings (the section describes the protocol, not its arithmetic):
 *   - Domains are ranges of 30-bit Morton keys (10 bits per axis over the
 *     unit box; Sec. 5.5 uses a Morton-order decomposition so that the owner
 *     of any position is computed on the device). The D+1 splitters are the
 *     keys of ranks floor(d N / D) of the sorted initial keys, K[0] = 0,
 *     K[D] = 2^30; owner(key) = the largest d with K[d] <= key.
 *   - The force slot of a Particle holds the acceleration (G = 1); the
 *     integrator is kick-drift-kick leapfrog, positions wrap periodically
 *     into [0, 1) and gravity is the open-boundary Plummer-softened sum.
 *   - The per-domain hierarchy is the domain root and one level of Morton
 *     cells (level L: key >> (30 - 3L)), in key order; cuBQL's BVH is not
 *     rebuilt here. A node's mass is the float32 sum of its particles'
 *     masses in key order and its centre of mass the fmaf-accumulated
 *     first moment divided by that mass. A cell's size is its edge 2^-L;
 *     the root's is the largest edge of the domain's particle bounding box.
 *   - Acceptance (the multipole acceptance criterion of Barnes-Hut, tested
 *     against the receiving domain's bounding box): size^2 < theta^2 d^2,
 *     d the distance from the node's centre of mass to the box.
 *   - Essential-tree exchange: every domain sends its root to every other
 *     non-empty domain; a receiver that does not accept it returns a
 *     RefinementReq; the owner answers with its cells that the requester
 *     accepts, and with the particles (size 0) of those it does not. The
 *     received nodes, in queue order, are the requester's remote list.
 *   - Force on a particle: the softened point-mass terms of its domain's
 *     other particles in key order, then of its remote list in order, each
 *     term evaluated and added in float64 (the section fixes no order and
 *     no precision; this is the plain sum over that source sequence). The
 *     float64 total, rounded to float32, is the stored acceleration.
 *   - Slots: the forward step keeps slot order within a destination (O1),
 *     and fan-out uses fixed slots: root s -> r at s (D-1) + k; a request at
 *     the slot of the root it answers; answers after the n1 slots of the
 *     first VirtualParticle round, at n1 + the exclusive prefix of the
 *     answer sizes in request-queue order.
 * ====================================================================== */
typedef struct {
    int32_t n_domains, cell_level;
    float dt, theta, eps;
} orc_nb_params;

typedef struct {
    float pos[3], vel[3], acc[3], mass;
} orc_nb_particle;

typedef struct {
    float pos[3], mass, smax;
    int32_t src;
} orc_nb_vp;

uint32_t oracle_morton30(float x, float y, float z)
{
    const float c[3] = {x, y, z};
    uint32_t key = 0;
    for (int a = 0; a < 3; ++a) {
        int32_t q = (int32_t)(c[a] * 1024.0f);
        if (q < 0) q = 0;
        if (q > 1023) q = 1023;
        for (int b = 0; b < 10; ++b) key |= (uint32_t)((q >> b) & 1) << (3 * b + a);
    }
    return key;
}

static int32_t nb_owner(const uint32_t *K, int32_t D, uint32_t key)
{
    int32_t d = 0;
    while (d + 1 < D && K[d + 1] <= key) ++d;
    return d;
}

static int cmp_u32(const void *a, const void *b)
{
    const uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

int oracle_nb_splitters(const float *pos, int64_t n, int32_t D, uint32_t *K)
{
    if (D < 1 || n < 1) return -1;
    uint32_t *keys = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n);
    if (!keys) return -2;
    for (int64_t i = 0; i < n; ++i) keys[i] = oracle_morton30(pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]);
    qsort(keys, (size_t)n, sizeof(uint32_t), cmp_u32);
    K[0] = 0;
    for (int32_t d = 1; d < D; ++d) K[d] = keys[(int64_t)d * n / D];
    K[D] = 1u << 30;
    free(keys);
    return 0;
}

static float nb_wrap(float x)
{
    x = x - floorf(x);
    return x < 1.0f ? x : 0.0f;
}

static uint32_t nb_key(const orc_nb_particle *p) { return oracle_morton30(p->pos[0], p->pos[1], p->pos[2]); }

/* a += m (q - p) / (|q - p|^2 + eps^2)^(3/2), in float64; mag += |term|
 * per component (the scale of the sum's rounding error, for tolerances) */
static void nb_term(const float p[3], const float q[3], float m, double eps2, double a[3], double mag[3])
{
    const double dx = (double)q[0] - p[0], dy = (double)q[1] - p[1], dz = (double)q[2] - p[2];
    const double r2 = dx * dx + dy * dy + dz * dz + eps2;
    const double s = m / (r2 * sqrt(r2));
    a[0] += s * dx;
    a[1] += s * dy;
    a[2] += s * dz;
    mag[0] += fabs(s * dx);
    mag[1] += fabs(s * dy);
    mag[2] += fabs(s * dz);
}

/* size^2 < theta^2 d^2, d = distance from c to the box [lo, hi] */
static int nb_accept(const float c[3], float size, const float lo[3], const float hi[3], float theta)
{
    float d[3];
    for (int a = 0; a < 3; ++a) d[a] = fmaxf(fmaxf(lo[a] - c[a], c[a] - hi[a]), 0.0f);
    const float d2 = fmaf(d[2], d[2], fmaf(d[1], d[1], d[0] * d[0]));
    return size * size < (theta * theta) * d2;
}

typedef struct {
    int64_t first, count;   /* particle range in the sorted queue */
    float com[3], mass;
} nb_node;

static void nb_moments(const orc_nb_particle *q, int64_t first, int64_t count, nb_node *nd)
{
    float m = 0.0f, mx = 0.0f, my = 0.0f, mz = 0.0f;
    for (int64_t i = first; i < first + count; ++i) {
        m = m + q[i].mass;
        mx = fmaf(q[i].mass, q[i].pos[0], mx);
        my = fmaf(q[i].mass, q[i].pos[1], my);
        mz = fmaf(q[i].mass, q[i].pos[2], mz);
    }
    nd->first = first;
    nd->count = count;
    nd->mass = m;
    nd->com[0] = mx / m;
    nd->com[1] = my / m;
    nd->com[2] = mz / m;
}

/* Round 0: every particle of the input (any order) to the domain owning it. */
int oracle_nb_seed(const orc_nb_params *P, const uint32_t *K, const orc_nb_particle *in, int64_t n,
                   orc_nb_particle *queue, uint64_t *counts)
{
    const int32_t D = P->n_domains;
    int32_t *dest = (int32_t *)calloc((size_t)(n ? n : 1), sizeof(int32_t));
    uint64_t *offs = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(D + 1));
    if (!dest || !offs) return -2;
    for (int64_t i = 0; i < n; ++i) dest[i] = nb_owner(K, D, nb_key(&in[i]));
    oracle_multisplit((uint64_t)n, sizeof(orc_nb_particle), (const uint8_t *)in, dest, D, (uint8_t *)queue,
                      counts, offs, NULL, NULL);
    free(dest); free(offs);
    return 0;
}

/* order by key, then by position in the queue (a stable sort by key) */
static const uint32_t *nb_cmp_keys;
static int cmp_key_index(const void *a, const void *b)
{
    const int64_t i = *(const int64_t *)a, j = *(const int64_t *)b;
    if (nb_cmp_keys[i] != nb_cmp_keys[j]) return nb_cmp_keys[i] < nb_cmp_keys[j] ? -1 : 1;
    return i < j ? -1 : (i > j ? 1 : 0);
}

/*
 * One step. queue: in, the particle queue the previous step (or the seed)
 * left, grouped by domain; out, the new queue (grouped by domain, each
 * domain in key order), with positions drifted and velocities and
 * accelerations updated. Logs (any may be NULL): counts per domain of the
 * four forward rounds in the order particle, virtual 1, request, virtual 2
 * (round_counts[4][D]); the three exchange queues (vp1 [cap_vp1], rr
 * [cap_rr], vp2 [cap_vp2]) and their lengths (lens[3]); per particle of the
 * new queue, the sum of the force terms' magnitudes per component
 * (acc_mag[n][3], float64).
 */
int oracle_nb_step(const orc_nb_params *P, const uint32_t *K, orc_nb_particle *queue, int64_t n,
                   uint64_t *round_counts, orc_nb_vp *vp1_log, uint64_t cap_vp1, int32_t *rr_log,
                   uint64_t cap_rr, orc_nb_vp *vp2_log, uint64_t cap_vp2, uint64_t *lens, double *acc_mag)
{
    const int32_t D = P->n_domains, L = P->cell_level;
    const float dt = P->dt, hdt = 0.5f * P->dt;
    const double eps2 = (double)P->eps * P->eps;
    const size_t nn = (size_t)(n ? n : 1);
    orc_nb_particle *tmp = (orc_nb_particle *)malloc(sizeof(orc_nb_particle) * nn);
    int32_t *dest = (int32_t *)calloc(nn, sizeof(int32_t));
    uint64_t *counts = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)D);
    uint64_t *offs = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(D + 1));
    uint32_t *keys = (uint32_t *)malloc(sizeof(uint32_t) * nn);
    int64_t *idx = (int64_t *)malloc(sizeof(int64_t) * nn);
    nb_node *cells = (nb_node *)malloc(sizeof(nb_node) * nn);
    int64_t *cell_first = (int64_t *)malloc(sizeof(int64_t) * (size_t)(D + 1));
    nb_node *root = (nb_node *)malloc(sizeof(nb_node) * (size_t)D);
    float *lo = (float *)malloc(sizeof(float) * 3 * (size_t)D), *hi = (float *)malloc(sizeof(float) * 3 * (size_t)D);
    float *rsize = (float *)malloc(sizeof(float) * (size_t)D);
    if (!tmp || !dest || !counts || !offs || !keys || !idx || !cells || !cell_first || !root || !lo || !hi || !rsize)
        return -2;

    /* 1. kick (half), drift, wrap, owner: the Particle context's forward */
    for (int64_t i = 0; i < n; ++i) {
        orc_nb_particle *p = &queue[i];
        for (int a = 0; a < 3; ++a) {
            p->vel[a] = fmaf(hdt, p->acc[a], p->vel[a]);
            p->pos[a] = nb_wrap(fmaf(dt, p->vel[a], p->pos[a]));
        }
        dest[i] = nb_owner(K, D, nb_key(p));
    }
    oracle_multisplit((uint64_t)n, sizeof(orc_nb_particle), (const uint8_t *)queue, dest, D, (uint8_t *)tmp,
                      counts, offs, NULL, NULL);
    if (round_counts) for (int32_t d = 0; d < D; ++d) round_counts[d] = counts[d];

    /* 2. each domain in key order (stable): one sort of the whole queue by
     * key, since a domain is a key range */
    for (int64_t i = 0; i < n; ++i) { keys[i] = nb_key(&tmp[i]); idx[i] = i; }
    nb_cmp_keys = keys;
    qsort(idx, (size_t)n, sizeof(int64_t), cmp_key_index);
    for (int64_t i = 0; i < n; ++i) queue[i] = tmp[idx[i]];
    for (int64_t i = 0; i < n; ++i) keys[i] = nb_key(&queue[i]);

    /* 3. cells (runs of one level-L prefix within a domain), roots, boxes */
    const int sh = 30 - 3 * L;
    const float csize = ldexpf(1.0f, -L);
    int64_t nc = 0;
    for (int32_t d = 0; d < D; ++d) {
        cell_first[d] = nc;
        int64_t i = (int64_t)offs[d];
        const int64_t e = (int64_t)offs[d + 1];
        while (i < e) {
            int64_t j = i + 1;
            while (j < e && (keys[j] >> sh) == (keys[i] >> sh)) ++j;
            nb_moments(queue, i, j - i, &cells[nc++]);
            i = j;
        }
        if (e > (int64_t)offs[d]) {
            nb_moments(queue, (int64_t)offs[d], e - (int64_t)offs[d], &root[d]);
            for (int a = 0; a < 3; ++a) { lo[3 * d + a] = queue[offs[d]].pos[a]; hi[3 * d + a] = queue[offs[d]].pos[a]; }
            for (int64_t k = (int64_t)offs[d]; k < e; ++k)
                for (int a = 0; a < 3; ++a) {
                    lo[3 * d + a] = fminf(lo[3 * d + a], queue[k].pos[a]);
                    hi[3 * d + a] = fmaxf(hi[3 * d + a], queue[k].pos[a]);
                }
            rsize[d] = fmaxf(fmaxf(hi[3 * d] - lo[3 * d], hi[3 * d + 1] - lo[3 * d + 1]), hi[3 * d + 2] - lo[3 * d + 2]);
        } else {
            root[d].count = 0;
        }
    }
    cell_first[D] = nc;

    /* 4. VirtualParticle round 1: every root to every other non-empty domain */
    const int64_t n_r1 = (int64_t)D * (D - 1);
    orc_nb_vp *vo = (orc_nb_vp *)malloc(sizeof(orc_nb_vp) * (size_t)(n_r1 ? n_r1 : 1));
    orc_nb_vp *v1 = (orc_nb_vp *)malloc(sizeof(orc_nb_vp) * (size_t)(n_r1 ? n_r1 : 1));
    int32_t *vdest = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n_r1 ? n_r1 : 1));
    uint64_t *o1 = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(D + 1));
    if (!vo || !v1 || !vdest || !o1) return -2;
    for (int32_t s = 0; s < D; ++s)
        for (int32_t k = 0; k < D - 1; ++k) {
            const int32_t r = k < s ? k : k + 1;
            const int64_t slot = (int64_t)s * (D - 1) + k;
            memset(&vo[slot], 0, sizeof(orc_nb_vp));
            vdest[slot] = ORC_DONE;
            if (root[s].count > 0 && counts[r] > 0) {
                for (int a = 0; a < 3; ++a) vo[slot].pos[a] = root[s].com[a];
                vo[slot].mass = root[s].mass;
                vo[slot].smax = rsize[s];
                vo[slot].src = s;
                vdest[slot] = r;
            }
        }
    oracle_multisplit((uint64_t)n_r1, sizeof(orc_nb_vp), (const uint8_t *)vo, vdest, D, (uint8_t *)v1, counts, o1,
                      NULL, NULL);
    const int64_t n1 = (int64_t)o1[D];
    if (round_counts) for (int32_t d = 0; d < D; ++d) round_counts[D + d] = counts[d];
    if (vp1_log) for (int64_t i = 0; i < n1 && (uint64_t)i < cap_vp1; ++i) vp1_log[i] = v1[i];

    /* 5. accept a root, or return a RefinementReq to its owner */
    int32_t *acc = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n1 ? n1 : 1));
    int32_t *ro = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n1 ? n1 : 1));
    int32_t *rq = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n1 ? n1 : 1));
    int32_t *rdest = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n1 ? n1 : 1));
    uint64_t *orr = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(D + 1));
    if (!acc || !ro || !rq || !rdest || !orr) return -2;
    for (int32_t r = 0; r < D; ++r)
        for (int64_t i = (int64_t)o1[r]; i < (int64_t)o1[r + 1]; ++i) {
            acc[i] = nb_accept(v1[i].pos, v1[i].smax, &lo[3 * r], &hi[3 * r], P->theta);
            ro[i] = r;
            rdest[i] = acc[i] ? ORC_DONE : v1[i].src;
        }
    oracle_multisplit((uint64_t)n1, sizeof(int32_t), (const uint8_t *)ro, rdest, D, (uint8_t *)rq, counts, orr,
                      NULL, NULL);
    const int64_t nr = (int64_t)orr[D];
    if (round_counts) for (int32_t d = 0; d < D; ++d) round_counts[2 * D + d] = counts[d];
    if (rr_log) for (int64_t i = 0; i < nr && (uint64_t)i < cap_rr; ++i) rr_log[i] = rq[i];

    /* 6. answers: sizes, prefix, then the nodes */
    int64_t *aoff = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nr + 1));
    if (!aoff) return -2;
    aoff[0] = 0;
    for (int32_t s = 0; s < D; ++s)
        for (int64_t j = (int64_t)orr[s]; j < (int64_t)orr[s + 1]; ++j) {
            const int32_t r = rq[j];
            int64_t c = 0;
            for (int64_t k = cell_first[s]; k < cell_first[s + 1]; ++k)
                c += nb_accept(cells[k].com, csize, &lo[3 * r], &hi[3 * r], P->theta) ? 1 : cells[k].count;
            aoff[j + 1] = aoff[j] + c;
        }
    const int64_t n2 = n1 + aoff[nr];
    orc_nb_vp *wo = (orc_nb_vp *)malloc(sizeof(orc_nb_vp) * (size_t)(n2 ? n2 : 1));
    orc_nb_vp *v2 = (orc_nb_vp *)malloc(sizeof(orc_nb_vp) * (size_t)(n2 ? n2 : 1));
    int32_t *wdest = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n2 ? n2 : 1));
    uint64_t *o2 = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(D + 1));
    if (!wo || !v2 || !wdest || !o2) return -2;
    for (int64_t i = 0; i < n1; ++i) { wo[i] = v1[i]; wdest[i] = acc[i] ? ro[i] : ORC_DONE; }
    for (int32_t s = 0; s < D; ++s)
        for (int64_t j = (int64_t)orr[s]; j < (int64_t)orr[s + 1]; ++j) {
            const int32_t r = rq[j];
            int64_t slot = n1 + aoff[j];
            for (int64_t k = cell_first[s]; k < cell_first[s + 1]; ++k) {
                if (nb_accept(cells[k].com, csize, &lo[3 * r], &hi[3 * r], P->theta)) {
                    orc_nb_vp *v = &wo[slot];
                    for (int a = 0; a < 3; ++a) v->pos[a] = cells[k].com[a];
                    v->mass = cells[k].mass; v->smax = csize; v->src = s;
                    wdest[slot++] = r;
                } else {
                    for (int64_t q = cells[k].first; q < cells[k].first + cells[k].count; ++q) {
                        orc_nb_vp *v = &wo[slot];
                        for (int a = 0; a < 3; ++a) v->pos[a] = queue[q].pos[a];
                        v->mass = queue[q].mass; v->smax = 0.0f; v->src = s;
                        wdest[slot++] = r;
                    }
                }
            }
        }
    oracle_multisplit((uint64_t)n2, sizeof(orc_nb_vp), (const uint8_t *)wo, wdest, D, (uint8_t *)v2, counts, o2,
                      NULL, NULL);
    if (round_counts) for (int32_t d = 0; d < D; ++d) round_counts[3 * D + d] = counts[d];
    if (vp2_log) for (int64_t i = 0; i < (int64_t)o2[D] && (uint64_t)i < cap_vp2; ++i) vp2_log[i] = v2[i];
    if (lens) { lens[0] = (uint64_t)n1; lens[1] = (uint64_t)nr; lens[2] = o2[D]; }

    /* 7. forces (own domain's other particles, then the remote list) and the second half-kick */
    for (int32_t r = 0; r < D; ++r)
        for (int64_t i = (int64_t)offs[r]; i < (int64_t)offs[r + 1]; ++i) {
            double a[3] = {0.0, 0.0, 0.0}, mag[3] = {0.0, 0.0, 0.0};
            for (int64_t j = (int64_t)offs[r]; j < (int64_t)offs[r + 1]; ++j)
                if (j != i) nb_term(queue[i].pos, queue[j].pos, queue[j].mass, eps2, a, mag);
            for (int64_t v = (int64_t)o2[r]; v < (int64_t)o2[r + 1]; ++v)
                nb_term(queue[i].pos, v2[v].pos, v2[v].mass, eps2, a, mag);
            if (acc_mag) for (int c = 0; c < 3; ++c) acc_mag[3 * i + c] = mag[c];
            for (int c = 0; c < 3; ++c) {
                queue[i].acc[c] = (float)a[c];
                queue[i].vel[c] = fmaf(hdt, queue[i].acc[c], queue[i].vel[c]);
            }
        }
    free(tmp); free(dest); free(counts); free(offs); free(keys); free(idx); free(cells); free(cell_first); free(root);
    free(lo); free(hi); free(rsize); free(vo); free(v1); free(vdest); free(o1); free(acc); free(ro); free(rq);
    free(rdest); free(orr); free(aoff); free(wo); free(v2); free(wdest); free(o2);
    return 0;
}
