/*
 * rafi.h -- host C ABI of the single-GPU work-forwarding library (librafi.so).
 *
 * The library follows the forwarding model of RaFI (arXiv 2605.30294):
 * application kernels read work items from an input queue and emit each item
 * with a destination domain (Sec. 3.2, 3.3); a forward step then regroups the
 * emitted items by destination and hands every domain its new input queue,
 * returning the number of items still alive (Sec. 3.4, 4.2). Here all domains
 * live on one GPU, so the forward step is a device-local stable multi-split.
 *
 * Conventions for every call below:
 *   - Pointers documented as "device" are HIP device allocations the caller
 *     owns; "host" pointers are ordinary host memory. No call takes ownership
 *     of caller memory. A context owns its queues (Sec. 3.2: the library
 *     manages the arrays itself once told their capacity).
 *   - Work is stream-ordered on the context's stream (rafi_set_stream;
 *     default: the null stream). Calls that return host-visible results
 *     (rafi_round's counts and total) synchronise that stream.
 *   - A context is not thread-safe: one host thread per context.
 *   - Every int-returning call returns RAFI_OK (0) or a negative RAFI_ERR_*
 *     code; rafi_strerror() names it. On RAFI_ERR_ARG nothing was launched.
 *
 * The device-side half (reading inputs and emitting items from a kernel) is
 * in rafi_device.h.
 */
#ifndef RAFI_H
#define RAFI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    RAFI_OK = 0,
    RAFI_ERR_ARG = -1,        /* invalid argument; nothing was done */
    RAFI_ERR_OOM = -2,        /* device allocation failed */
    RAFI_ERR_HIP = -3,        /* a HIP runtime call failed */
    RAFI_ERR_OVERFLOW = -4,   /* emits beyond the slot range were dropped (Sec. 3.3) */
    RAFI_ERR_BAD_DEST = -5,   /* slots carried a destination outside {-1} U [0, n_domains) */
    RAFI_ERR_MAX_ROUNDS = -6, /* a driver loop hit its round limit with items still alive */
    RAFI_ERR_STATE = -7,      /* call not valid in the context's current state */
    RAFI_ERR_TOO_LARGE = -8   /* problem larger than a fixed buffer; nothing was done */
};

/* Destination of an item that leaves the system (the -1 of Sec. 3.2). */
#define RAFI_DONE (-1)
/* Destination pre-filled into unwritten slots in debug mode. */
#define RAFI_POISON (-2)

/* Largest number of domains one context or split supports. */
#define RAFI_MAX_DOMAINS 8192
/* Largest item size in bytes (items are copied as 4-byte words). */
#define RAFI_MAX_ITEM_BYTES 256

typedef struct rafi_ctx rafi_ctx;

/*
 * Plain-old-data view of a context's queues, passed by value to kernels
 * (the device interface of Sec. 3.3). Valid until the next rafi_round,
 * rafi_begin or rafi_resize on the context.
 *
 * Input queue: n_in items; those of domain d are items
 *   [in_offsets[d], in_offsets[d+1]) of in_items, in forward order.
 * Output: n_slots slots. The kernel that handles input item i owns slot i
 *   and writes it exactly once, with rafi_forward or rafi_done (slot-ordered
 *   emission: the destination order within a domain is then deterministic).
 * in_tile_offsets[d] is the index of domain d's first tile when every
 *   domain's items are cut into tiles of tile_items; in_tile_offsets[D] is
 *   the number of tiles (a launch grid for domain-pure workgroups).
 */
typedef struct rafi_device_view {
    const void *in_items;             /* device */
    const uint64_t *in_offsets;       /* device [n_domains + 1] */
    const uint32_t *in_tile_offsets;  /* device [n_domains + 1] */
    void *out_items;                  /* device [capacity * item_bytes] */
    int32_t *out_dest;                /* device [capacity] */
    unsigned long long *dropped;      /* device counter of emits to slots >= n_slots */
    uint64_t n_in;                    /* number of input items */
    uint64_t n_slots;                 /* output slots the next rafi_round consumes */
    uint64_t capacity;                /* queue capacity in items */
    uint32_t item_bytes;
    int32_t n_domains;
    uint32_t tile_items;
    uint32_t n_tiles;                 /* host copy of in_tile_offsets[n_domains] */
    unsigned long long *append;       /* device counter of slots taken by rafi_emit (append mode) */
} rafi_device_view;

typedef struct rafi_stats_t {
    uint64_t rounds;     /* rafi_round calls since creation */
    uint64_t forwarded;  /* items delivered to a domain queue, summed over rounds */
    uint64_t done;       /* slots that carried RAFI_DONE */
    uint64_t bad_dest;   /* slots with an invalid destination (poison included) */
    uint64_t dropped;    /* emits to a slot outside [0, n_slots) */
    uint64_t last_total; /* total returned by the last rafi_round */
} rafi_stats_t;

/*
 * Create a context for n_domains domains of items of item_bytes bytes, with
 * queues of `capacity` items (host context creation + resizeRayQueues,
 * Sec. 3.4). n_domains in [1, RAFI_MAX_DOMAINS]; item_bytes a multiple of 4
 * in [4, RAFI_MAX_ITEM_BYTES]; capacity in [1, 2^32 - 1]. Allocates two
 * item buffers, the destination array and the split workspace on the current
 * HIP device. *out receives the context (NULL on failure).
 */
int rafi_create(int32_t n_domains, uint32_t item_bytes, uint64_t capacity, rafi_ctx **out);

/* Free a context and everything it allocated. NULL is ignored. */
void rafi_destroy(rafi_ctx *ctx);

/* Change the queue capacity (resizeRayQueues, Sec. 3.4). Drops the current
 * queue contents. */
int rafi_resize(rafi_ctx *ctx, uint64_t capacity);

/* Stream for all later work on this context (a hipStream_t, passed as void*).
 * The stream must outlive its use by the context. The paper's library runs on
 * one stream and leaves several asynchronous streams to future work (Sec. 7);
 * here each context has one stream of the caller's choice, so contexts on
 * different streams (and the batched form) can overlap. */
int rafi_set_stream(rafi_ctx *ctx, void *hip_stream);

/* Debug mode: when on, every rafi_begin/rafi_round pre-fills the output
 * destinations with RAFI_POISON, so slots a kernel never wrote are counted
 * as bad destinations. */
int rafi_set_debug(rafi_ctx *ctx, int32_t on);

/* Tile size used to build in_tile_offsets (default 256; any value >= 1). */
int rafi_set_tile_items(rafi_ctx *ctx, uint32_t tile_items);

/* Fill *out with the current device view (getDeviceInterface, Sec. 3.4). */
int rafi_view(const rafi_ctx *ctx, rafi_device_view *out);

/* Start a new wave of work: empty the input queue and open n_slots output
 * slots (n_slots <= capacity) for a generator kernel (ray generation /
 * seeding) that emits into slots [0, n_slots). */
int rafi_begin(rafi_ctx *ctx, uint64_t n_slots);

/* Output modes of rafi_open. */
#define RAFI_SLOTS_ORDERED 0
#define RAFI_SLOTS_APPEND 1

/* Reopen the output slots of the current round before a domain kernel runs,
 * leaving the input queue as it is (rafi_begin and rafi_round open
 * slot-ordered output with n_slots = the number of work units / input items).
 *   RAFI_SLOTS_ORDERED: the thread handling work unit i writes slot i with
 *     rafi_forward / rafi_done (fan-out k: unit i owns slots k*i .. k*i+k-1).
 *   RAFI_SLOTS_APPEND: the paper's append queue (Sec. 3.2-3.3): every slot
 *     starts as RAFI_DONE, the append counter starts at 0, and rafi_emit takes
 *     the next free slot; any number of emits per thread. Emits beyond
 *     n_slots are dropped and counted (rafi_round then returns
 *     RAFI_ERR_OVERFLOW). The order of items within a destination depends on
 *     the order in which waves reach their emits; the multiset does not.
 * n_slots <= capacity, else RAFI_ERR_ARG; other modes: RAFI_ERR_ARG.
 * Stream-ordered (one small fill kernel; no host synchronisation). */
int rafi_open(rafi_ctx *ctx, uint64_t n_slots, int32_t mode);

/* Bulk emission from device arrays: copy items [n * item_bytes] and dest [n]
 * (both device) into output slots [0, n) (n <= n_slots), as a generator
 * kernel would with rafi_forward. Stream-ordered device-to-device copies. */
int rafi_emit_bulk(rafi_ctx *ctx, const void *items, const int32_t *dest, uint64_t n);

/*
 * Forward step (forwardRays, Sec. 3.4 and 4.2): stable multi-split of the
 * n_slots output slots by destination into the next input queue. An item
 * with destination e lands at in_offsets[e] + (number of earlier slots with
 * destination e). RAFI_DONE slots leave the system; slots with invalid
 * destinations are dropped and counted. Afterwards n_slots = n_in = total.
 *   counts: host [n_domains] items per domain, or NULL.
 *   total:  host, items now alive (the distributed-termination total, Sec. 4.2.3), or NULL.
 * Synchronises the context stream. Returns RAFI_ERR_BAD_DEST or
 * RAFI_ERR_OVERFLOW (after completing the split) if such slots occurred in
 * this round.
 */
int rafi_round(rafi_ctx *ctx, uint64_t *counts, uint64_t *total);

/* Copy the current input queue (n_in items, device-to-device, stream-ordered)
 * into items_dst (device, >= n_in * item_bytes bytes) and its per-domain
 * offsets into offsets_dst (device, n_domains + 1 uint64); either may be NULL. */
int rafi_copy_queue(const rafi_ctx *ctx, void *items_dst, uint64_t *offsets_dst);

/* Cumulative statistics (host copy, updated by rafi_round): the counts that
 * Sec. 3.3 and 4.2 leave to the application (dropped emits, invalid
 * destinations) besides the per-round totals of Sec. 4.2.3. */
int rafi_stats(const rafi_ctx *ctx, rafi_stats_t *out);

/*
 * Per-phase GPU time, measured with HIP events recorded on the context stream
 * around every launch while profiling is on (rafi_set_profiling). Times are
 * sums in milliseconds; *_calls count launches. "split" is the whole forward
 * step, "scatter" its final pass alone, "domain" the domain kernels
 * (rafi_ea_march, rafi_sl_advance, ...). Event pairs are resolved at the
 * next rafi_round or rafi_get_profile (which synchronises the stream).
 */
typedef struct rafi_profile {
    double split_ms, scatter_ms, domain_ms;
    uint64_t split_calls, scatter_calls, domain_calls;
    uint64_t split_slots;  /* slots consumed by the timed forward steps */
    uint64_t split_items;  /* items they delivered */
} rafi_profile;

/* Turn event timing on (1) or off (0); turning it on clears the totals. */
int rafi_set_profiling(rafi_ctx *ctx, int32_t on);
int rafi_get_profile(rafi_ctx *ctx, rafi_profile *out);

/* Static string naming an error code. */
const char *rafi_strerror(int code);

/*
 * Stateless split (the forward step without a context). items: device
 * [n * item_bytes]; dest: device [n]; out: device [n * item_bytes], receives
 * the kept items grouped by destination, stable; offsets: device
 * [n_domains + 1] uint64 exclusive prefix of the per-destination counts;
 * summary: device [4] uint64 = {total kept, done, bad, 0}. workspace: device,
 * at least rafi_multisplit_workspace() bytes. item_bytes, n_domains as for
 * rafi_create; n < 2^32. Follows Sec. 4.2.1-4.2.2.
 */
int rafi_multisplit_workspace(uint64_t n, int32_t n_domains, uint32_t item_bytes,
                              uint64_t *bytes);

/* Process-wide choice of the scatter pass's workgroup shape (chunk size,
 * waves per workgroup, workgroups per CU): 0 = automatic (for at most 128
 * destinations: up to 256 MiB of 16- or 32-byte items shape 4 or 2, up to
 * 64 MiB of items of 44 bytes or more the plain per-thread scatter; else
 * shape 14 when one workgroup per CU spans at least two tiles and 16384
 * slots, else shape 12 when a tile holds at least one of its chunks, else
 * the first of 1..4 that fits the LDS); 1..4 stage items
 * in LDS; 5..7 stage only indices and read items in sorted order; 8..11 are
 * shapes 1..4 with the next chunk's loads issued before the current chunk is
 * ranked; 12..13 use one workgroup per CU with 4096-slot chunks (32-byte
 * items), 13 with the next chunk's loads issued early; 14..15 (16- and
 * 32-byte items, 128-byte aligned output of at most 0xfffffff0 bytes, else
 * as 0) use one workgroup per
 * CU over a group of tiles and write each destination's output in whole
 * 128-byte lines, keeping a run's unfinished line for the next chunk; 15
 * issues the next chunk's loads early; 16 (item sizes of 12 to 60 bytes
 * that are not a multiple of 16, else as 0) uses one workgroup per CU with
 * 2048-slot chunks whose bytes are staged in LDS in load order and written
 * as consecutive 4-byte words (automatic for those sizes when a tile holds a
 * chunk); 17 (the sizes of 16, splits of at least 2^21 slots and at most
 * 1024 destinations, else as 0) runs shape 16's chunks on a lockstep
 * schedule: 256 persistent workgroups, the 32 of one XCD taking the 32
 * consecutive chunks of one tile at a time, with each chunk's run bases
 * from the histogram pass (automatic where it applies; its plan needs 2
 * more workspace bytes per 2048 slots and destination, which
 * rafi_multisplit_workspace includes while 0 or 17 is selected). For
 * tuning. Every shape gives the same bytes. Not synchronised: set it while
 * no split is being launched. Outside 0..17: RAFI_ERR_ARG. */
int rafi_split_set_variant(int32_t variant);
int rafi_multisplit(const void *items, const int32_t *dest, uint64_t n, uint32_t item_bytes,
                    int32_t n_domains, void *out, uint64_t *offsets, uint64_t *summary,
                    void *workspace, uint64_t workspace_bytes, void *hip_stream);

/*
 * The stateless split for callers that cannot allocate device memory (code
 * under stream capture, tight serving loops, harnesses that forbid
 * hipMalloc): rafi_multisplit with the workspace taken from a fixed 32 MiB
 * buffer of the library's own (static device memory, one copy per device,
 * held until the process ends). Arguments, layout, results and errors as
 * rafi_multisplit; it calls no allocating routine. Problems whose workspace
 * (rafi_multisplit_workspace) exceeds 32 MiB return RAFI_ERR_TOO_LARGE
 * before anything is enqueued. Every n fits for n_domains <= 2045, and
 * n <= 2^24 fits for every n_domains; D = 2046 and more fail above about
 * 2^25 slots (the table holds up to 4096 tiles of D + 2 counts). hip_stream (or the
 * null stream) must belong to the current device, else RAFI_ERR_ARG. The
 * buffer needs no clearing: every split writes each workspace entry it reads.
 * All calls on one device share the buffer: calls that overlap on that
 * device (different streams, or host threads) race and must be ordered by
 * the caller; calls in one stream are ordered already.
 */
int rafi_multisplit_noalloc(const void *items, const int32_t *dest, uint64_t n, uint32_t item_bytes,
                            int32_t n_domains, void *out, uint64_t *offsets, uint64_t *summary,
                            void *hip_stream);

/* ------------------------------------------------------------------------
 * Emission-absorption volume ray march over bricked domains (the
 * march-and-forward pattern of Sec. 5.1-5.3).
 *
 * Volume: n^3 float32 densities at voxel centres (i + 1/2), x fastest, split
 * into grid[0] x grid[1] x grid[2] bricks of n/grid[a] voxels (domain id
 * bx + grid0*(by + grid1*bz); a point on a brick plane belongs to the upper
 * brick). Ray (px, py) of view v starts at org = org0 + py*dv + px*du
 * (computed as fma(py, dv, fma(px, du, org0))) and sample k sits at
 * p_k = fma((k + 1/2) dt, dir, org), k < n_samples. With rho_k the trilinear
 * (clamp-to-edge) density at p_k and sigma_k = c rho_k,
 *   I = sum over inside samples of exp(-tau_k) (1 - exp(-sigma_k)) rho_k,
 *   tau_k = sum_{j<k} sigma_j.
 * Each brick advances its rays while their samples stay inside it and then
 * forwards them to the owner of the next sample, or finishes them.
 * ------------------------------------------------------------------------ */
typedef struct rafi_ortho_view {
    float org0[3], du[3], dv[3], dir[3];
    int32_t width, height, n_samples, pad;
} rafi_ortho_view; /* 64 bytes */

typedef struct rafi_ea_job {
    const float *volume;            /* device [n^3] */
    const rafi_ortho_view *views;   /* device [n_views], all width x height */
    float *image;                   /* device [n_views * height * width] result per ray */
    float *tau;                     /* device, optional: final optical depth per ray */
    int32_t *klast;                 /* device, optional: one past the last inside sample */
    int32_t *kfirst;                /* device, optional: first inside sample (0 for misses) */
    int32_t *visit_log;             /* device, optional [n_rays * visit_stride]: domains visited,
                                       in order (forward) or as replayed (backward) */
    int32_t *visit_count;           /* device [n_rays], required with visit_log; zeroed by raygen */
    int32_t n;
    int32_t grid[3];
    int32_t n_views, width, height;
    float dt;                       /* sample spacing along the ray */
    float c;                        /* extinction per unit density per sample (kappa * dt) */
    int32_t visit_stride;
    int32_t emit_mode;              /* RAFI_SLOTS_ORDERED (0): ray in input slot i is emitted to
                                       output slot i; RAFI_SLOTS_APPEND: forwarded rays are
                                       appended (rafi_emit) and finished rays take no slot.
                                       rafi_ea_render opens every march round's output in this
                                       mode; callers of rafi_ea_march open it themselves
                                       (rafi_open). Same images either way; the order of rays
                                       within a domain queue is reproducible only when ordered.
                                       Other values: RAFI_ERR_ARG. */
    uint32_t bwd_tile_items;        /* LDS-privatised backward: 0 = one workgroup per CU, each
                                       taking an equal contiguous slice of the queue and
                                       flushing its brick's gradient once per brick it spans;
                                       k > 0 = one workgroup per k-ray domain-pure tile. Same
                                       gradients up to float32 atomic summation order. */
} rafi_ea_job;

/* Item size a context needs for the march (16 bytes: ray id, next sample,
 * optical depth, partial integral). */
#define RAFI_EA_ITEM_BYTES 16

/* Ray generation (round 0): opens one slot per ray (rafi_begin) and emits
 * every ray to the owner of its first inside sample; rays that miss the
 * volume finish with image = 0. The context needs n_domains = grid volume,
 * item_bytes = RAFI_EA_ITEM_BYTES, capacity >= number of rays. */
int rafi_ea_raygen(rafi_ctx *ctx, const rafi_ea_job *job);

/* One domain-kernel launch: every input item advances through its brick and
 * is forwarded or finished (result written to job->image). */
int rafi_ea_march(rafi_ctx *ctx, const rafi_ea_job *job);

/* Whole render: raygen, then rafi_round / rafi_ea_march until no item is
 * left. *rounds receives the number of forward steps taken. */
int rafi_ea_render(rafi_ctx *ctx, const rafi_ea_job *job, int32_t max_rounds, int32_t *rounds);

/*
 * Adjoint of the march (reverse replay): accumulates dL/dV into grad_volume
 * (device [n^3] float32, added to; the caller zeroes it) given
 * grad_image = dL/dI per ray (device [n_rays]). job must be the forward job
 * after rafi_ea_render with job->tau and job->klast recorded; job->visit_log,
 * when set, receives the backward visit sequence (the forward one reversed).
 *
 * Each ray re-enters the domains in reverse order, starting at its last
 * inside sample with the forward's final optical depth tau_N and B = 0, and
 * walks its samples backwards. With T = exp(-tau_k), a = 1 - exp(-sigma_k):
 *   dI/drho_k = T (a + c exp(-sigma_k) (rho_k - B)),   B <- a rho_k + (1 - a) B,
 * B being the part of the integral behind sample k; dI/drho_k * dL/dI is
 * scattered to the 8 voxels of sample k with their trilinear weights
 * (float32 atomic adds, so the summation order is not fixed). The item is 16
 * bytes (ray id, sample, tau, B); the context is the forward's.
 */
int rafi_ea_backward(rafi_ctx *ctx, const rafi_ea_job *job, const float *grad_image, float *grad_volume,
                     int32_t max_rounds, int32_t *rounds);

/* ------------------------------------------------------------------------
 * Batched form: many independent scenes advance together, one launch per
 * kernel per round for all of them (an extension; not in the paper).
 *
 * Scene s has its own volume (n_s^3 float32 at volume_offset in one device
 * buffer), domain grid and view; its domains get global ids
 * dom_base_s + local and its rays global ids ray_base_s + local (both filled
 * in by rafi_batch_create, in scene order). Items never change scene, so the
 * forward step is a segmented split: tiles never straddle a scene, each has
 * at most the scene's domain count of destinations, and the result equals the
 * stable split over all global domains. Every size the kernels need lives on
 * the device, so a round is captured once in a hipGraph and replayed.
 * ------------------------------------------------------------------------ */
typedef struct rafi_ea_scene {
    uint64_t volume_offset;   /* first float of the scene's volume in the volume buffer */
    rafi_ortho_view view;     /* the scene's view: width * height rays */
    int32_t n;
    int32_t grid[3];
    uint32_t ray_base;        /* set by rafi_batch_create */
    int32_t dom_base;         /* set by rafi_batch_create */
} rafi_ea_scene; /* 96 bytes */

typedef struct rafi_batch rafi_batch;

typedef struct rafi_batch_tuning {
    uint32_t split_tile;      /* slots per split tile, multiple of 256, >= 1024 (default 4096) */
    uint32_t march_block;     /* threads per march workgroup: 64, 128, 256 or 512 (default 256) */
    uint32_t march_grid;      /* persistent march workgroups (default 2048) */
    int32_t use_graph;        /* 1: rounds replayed from a captured hipGraph (default 1) */
    int32_t rounds_per_sync;  /* rounds launched between host checks of the total (default 4) */
} rafi_batch_tuning;

/* Create a batch over n_scenes scenes (host array; copied, bases filled in
 * the copy and in `scenes` itself). n_s >= 2, n_s % grid_a == 0, at most 64
 * domains per scene, total rays < 2^31. dt, c as for rafi_ea_job. */
int rafi_batch_create(rafi_ea_scene *scenes, int32_t n_scenes, float dt, float c, rafi_batch **out);
void rafi_batch_destroy(rafi_batch *b);
int rafi_batch_set_stream(rafi_batch *b, void *hip_stream);
int rafi_batch_set_tuning(rafi_batch *b, const rafi_batch_tuning *t);
/* Total rays and global domains of the batch. */
int rafi_batch_info(const rafi_batch *b, uint64_t *n_rays, int32_t *n_domains);
/* Render every scene: volumes device (the buffer the scenes' offsets index),
 * image device [n_rays] (ray r of scene s at ray_base_s + r). *rounds gets the
 * number of forward steps until no item was left. */
int rafi_batch_render(rafi_batch *b, const float *volumes, float *image, int32_t max_rounds, int32_t *rounds);

/* ------------------------------------------------------------------------
 * RK4 streamlines over bricked domains (particle tracing, Sec. 5.4).
 *
 * Field: n^3 float32 velocity triples at voxel centres, x fastest, in voxels
 * per unit time; packed once by rafi_sl_pack into a 16-byte-per-voxel copy.
 * Step: k1 = V(p), k2 = V(p + h/2 k1), k3 = V(p + h/2 k2), k4 = V(p + h k3),
 * p' = fma(h/6, fma(2,k3,fma(2,k2,k1)) + k4, p), componentwise, V trilinear
 * with clamp-to-edge (lerp x, then y, then z; lerp(a,b,t) = fma(t,b-a,a)).
 * A particle finishes when a step leaves it bitwise unchanged (stagnant), when
 * it leaves the box [0,n)^3 (exited), or at max_steps; otherwise it is
 * forwarded when it crosses into another brick.
 * ------------------------------------------------------------------------ */
typedef struct rafi_sl_job {
    const float *field4;   /* device field: [n^3 * 4] from rafi_sl_pack (field_stride 0 or 4),
                              or the [n^3 * 3] field itself (field_stride 3) */
    float *endpoint;       /* device [n_seeds * 3] final position per particle id */
    int32_t *steps;        /* device [n_seeds] steps taken */
    int32_t *reason;       /* device [n_seeds] 1 stagnant, 2 exited, 3 max steps; optional */
    unsigned long long *counters; /* device [2], optional, accumulated: forwards to another
                                     brick, forwards to the same brick (step cap) */
    int32_t n;
    int32_t grid[3];
    float h;
    int32_t max_steps;
    int32_t steps_per_visit; /* 0: integrate until the particle leaves its brick; k > 0: at
                                most k steps per domain-kernel launch, then the particle is
                                forwarded even to its own brick (k = 1 is the paper's one
                                update per round). Results do not depend on k. */
    uint32_t tail_items;     /* the cap is not applied in launches whose input queue holds at
                                most this many particles (0: always applied) */
    int32_t refill_lanes;    /* 0: one thread per queued particle; 1..64: persistent waves,
                                each taking new particles from the queue whenever at least
                                this many of its 64 lanes are idle (lanes stay busy while
                                their neighbours cross the brick). Results do not depend on
                                it. Outside 0..64: RAFI_ERR_ARG. */
    int32_t field_stride;    /* floats per voxel of field4: 0 or 4 = the padded layout of
                                rafi_sl_pack (16-byte loads), 3 = the unpadded field (12-byte
                                loads, 3/4 of the bytes). Same results either way; other
                                values: RAFI_ERR_ARG. */
    uint32_t quad_items;     /* launches whose input queue holds at most this many particles
                                (with refill_lanes 0) run four lanes per particle, one per
                                coordinate, exchanging weights within the lane quad (and cell
                                indices and tests when a lane flags a cell change or a
                                possible stop: about a third of the dependent instructions
                                per step), and gather each particle's cell two steps ahead
                                while it integrates: for launches too small to fill the GPU,
                                which are bound by each particle's step latency. 0: never.
                                Same results either way. */
} rafi_sl_job;

/* Item: position (3 x float32) and particle id; the step count lives in
 * job->steps[id] between visits. */
#define RAFI_SL_ITEM_BYTES 16
#define RAFI_SL_STAGNANT 1
#define RAFI_SL_EXITED 2
#define RAFI_SL_MAXSTEPS 3

/* Repack field [n^3 * 3] (device) into field4 [n^3 * 4] (device); n^3 < 2^31. */
int rafi_sl_pack(const float *field, int32_t n, float *field4, void *hip_stream);

/* Round 0: opens one slot per seed and emits seed i (id i, position
 * seeds[3i..3i+2], device) to its owning brick. */
int rafi_sl_seed(rafi_ctx *ctx, const rafi_sl_job *job, const float *seeds, uint64_t n_seeds);

/* One domain-kernel launch: every particle integrates until it leaves its
 * brick, finishes, or has taken job->steps_per_visit steps in this launch. */
int rafi_sl_advance(rafi_ctx *ctx, const rafi_sl_job *job);

/* Whole trace: seed, then rafi_round / rafi_sl_advance until no particle is
 * left. *rounds receives the number of forward steps; *forwarded (optional)
 * the number of items delivered over all forward steps. */
int rafi_sl_trace(rafi_ctx *ctx, const rafi_sl_job *job, const float *seeds, uint64_t n_seeds,
                  int32_t max_rounds, int32_t *rounds, uint64_t *forwarded);

/* ------------------------------------------------------------------------
 * Delta-tracking volume path tracing over bricked domains (the stochastic
 * transport of Sec. 5.1: Woodcock tracking inside the local brick, scattered
 * and shadow rays forwarded between rounds; one item may spawn two).
 *
 * Medium sigma_t(x) = kappa V(x) with V the float32 trilinear density (as for
 * the emission-absorption march); one global majorant smax >= kappa max V.
 * A path draws tentative points p += s d with s = -ln(1 - u) / smax; at a
 * point inside its brick it collides for real when u' smax < sigma_t(p),
 * otherwise it continues; leaving the volume ends it (black background). At a
 * real collision its weight is multiplied by the albedo, a shadow ray leaves
 * toward the light with weight w radiance / (4 pi) (isotropic phase) and is
 * ratio-tracked (weight times 1 - sigma_t / smax per tentative point) until it
 * leaves the volume, where its weight is the contribution of that scattering
 * event; the path takes a new isotropic direction (Marsaglia 1972) unless it
 * has scattered max_bounce times.
 * Random numbers: Philox4x32-10 (Salmon et al., SC 2011) with key
 * (seed, path id) and counter (stream, draw index, 0, 0), first word,
 * u = (word >> 8) 2^-24; stream 2b is the path after b scattering events,
 * 2b + 1 the shadow ray of event b. Logarithms use a fixed float32 series
 * (range reduction to [sqrt(1/2), sqrt(2)) and 2 atanh((m-1)/(m+1)) to s^13),
 * so the random walk is reproducible bit for bit.
 * Slots: fixed fan-out 2 per visit (input slot i owns output slots 2i, 2i+1).
 * ------------------------------------------------------------------------ */
typedef struct rafi_dt_job {
    const float *volume;            /* device [n^3] densities, x fastest */
    const rafi_ortho_view *views;   /* device [n_views], all width x height; path id =
                                       ray id = (view * height + py) * width + px */
    float *contrib;                 /* device [n_paths * max_bounce]: contribution of the
                                       shadow ray of each scattering event (0: none);
                                       zeroed by rafi_dt_raygen */
    float *image;                   /* device [n_paths], optional: sum of contrib over the
                                       events, in event order, written by rafi_dt_render */
    int32_t n;
    int32_t grid[3];
    int32_t n_views, width, height;
    float kappa;                    /* extinction per unit density per unit length */
    float smax;                     /* global majorant, >= kappa * max density, > 0 */
    float albedo;                   /* in [0, 1] */
    float light[3];                 /* unit direction toward the (directional) light */
    float radiance;                 /* light radiance */
    int32_t max_bounce;             /* scattering events per path, >= 1 */
    uint32_t seed;
    unsigned long long *counters;   /* device [2], optional, accumulated: tentative points
                                       evaluated, real collisions */
} rafi_dt_job;

/* Item size a context needs (position, direction, weight, path id, stream,
 * draw count, scattering events, kind). */
#define RAFI_DT_ITEM_BYTES 48

/* Context capacity that always suffices: a path has at most itself and one
 * shadow ray per scattering event alive, and each visit opens 2 slots. */
int rafi_dt_capacity(uint64_t n_paths, int32_t max_bounce, uint64_t *capacity);

/* Round 0: one slot per path; each primary ray enters the volume (slab test)
 * and goes to the owner of its first tentative point, or finishes. */
int rafi_dt_raygen(rafi_ctx *ctx, const rafi_dt_job *job);

/* One domain-kernel launch: opens 2 ordered slots per queued item and traces
 * every item through its brick until it leaves the brick, leaves the volume,
 * or (paths) collides for real. RAFI_ERR_ARG if 2 n_in exceeds the capacity. */
int rafi_dt_trace(rafi_ctx *ctx, const rafi_dt_job *job);

/* Whole render: raygen, then rafi_round / rafi_dt_trace until nothing is
 * left; then image (if set). *rounds receives the number of forward steps. */
int rafi_dt_render(rafi_ctx *ctx, const rafi_dt_job *job, int32_t max_rounds, int32_t *rounds);

/* ======================================================================
 * Multi-context, multi-phase forwarding: the N-body essential-tree exchange
 * (Sec. 5.5). Three contexts with the three item types of that section's
 * listing, on one stream, with the same n_domains:
 *   particles  Particle {float pos[3], vel[3], force[3], mass}   40 bytes
 *   virtuals   VirtualParticle {float pos[3], mass, smax;
 *                               int32 sourceRank}                 24 bytes
 *   requests   RefinementReq {int32 senderRank}                    4 bytes
 * The force slot holds the acceleration (G = 1). Domains are ranges of
 * 30-bit Morton keys over the unit box (10 bits per axis, the cell of a
 * coordinate c being min(1023, (int)(c * 1024))); owner(key) = the largest
 * d with splitters[d] <= key.
 * ====================================================================== */
#define RAFI_NB_PARTICLE_BYTES 40
#define RAFI_NB_VIRTUAL_BYTES 24
#define RAFI_NB_REQUEST_BYTES 4

typedef struct rafi_nb_job {
    int32_t n_domains;            /* 1..1024, the three contexts' n_domains */
    int32_t cell_level;           /* 1..10: the hierarchy's cells are Morton cells of edge 2^-cell_level */
    float dt;                     /* leapfrog step (kick-drift-kick) */
    float theta;                  /* acceptance: node size^2 < theta^2 distance^2 to the receiver's box */
    float eps;                    /* Plummer softening length */
    const uint32_t *splitters;    /* device [n_domains + 1], from rafi_nb_splitters */
    void *workspace;              /* device, rafi_nb_workspace(capacity, n_domains) bytes */
    uint64_t capacity;            /* particles the workspace was sized for */
    void *log_vp1;                /* device, optional: receives the first virtual-particle queue */
    uint64_t log_vp1_cap;         /* items log_vp1 holds */
} rafi_nb_job;

/* Workspace bytes for up to n_particles particles (< 2^31) over n_domains. */
int rafi_nb_workspace(uint64_t n_particles, int32_t n_domains, uint64_t *bytes);

/* Morton-order decomposition: splitters[0] = 0, splitters[d] = the key of
 * rank floor(d n / D) among the n particles' keys, splitters[D] = 2^30.
 * particles: device [n] Particle records; splitters: device [D + 1];
 * workspace as for rafi_nb_workspace(n, D). Enqueued on hip_stream. */
int rafi_nb_splitters(const void *particles, uint64_t n, int32_t n_domains, uint32_t *splitters,
                      void *workspace, void *hip_stream);

/* Round 0 of the particle context: every particle (device [n], any order)
 * to the domain owning its position, then one rafi_round. */
int rafi_nb_seed(rafi_ctx *particles, const rafi_nb_job *job, const void *in, uint64_t n);

/* One step on the particle queue the last seed or step left:
 *   1. half-kick, drift, periodic wrap into [0, 1); forward to the owner
 *      (particle round);
 *   2. each domain's particles in Morton-key order (stable);
 *   3. per domain: cells (runs of one level-cell_level key prefix) and a
 *      root, each with its mass and centre of mass (float32 sums in key
 *      order); the particles' bounding box (root size = its largest edge,
 *      cell size = 2^-cell_level);
 *   4. first virtual round: root s to every other non-empty domain r at slot
 *      s (D - 1) + (r < s ? r : r - 1);
 *   5. request round: receiver r keeps a root it accepts, else sends
 *      RefinementReq{r} to its owner from the root's slot;
 *   6. second virtual round: kept roots at their slots, then each request's
 *      answer (the owner's cells r accepts, the particles of the others,
 *      in key order) after the n1 round-1 slots, at the exclusive prefix of
 *      the answer sizes in request-queue order;
 *   7. forces: for each particle the softened sum over its domain's other
 *      particles in key order, then its remote list in queue order; then
 *      the second half-kick.
 * Afterwards the particle context's queue holds the particles (domain
 * grouped, key ordered within a domain), the request context's the
 * requests and the virtual context's the remote lists. round_counts (host
 * [4][D], optional): per-domain counts of the particle, virtual 1, request
 * and virtual 2 rounds; sizes (host [3], optional): the lengths of the
 * virtual 1, request and virtual 2 queues. RAFI_ERR_OVERFLOW if the
 * answers do not fit the virtual context (nothing of the second virtual
 * round is emitted);
 * RAFI_ERR_ARG for mismatched contexts, streams or sizes. */
int rafi_nb_step(rafi_ctx *particles, rafi_ctx *virtuals, rafi_ctx *requests, const rafi_nb_job *job,
                 uint64_t *round_counts, uint64_t *sizes);

#ifdef __cplusplus
}
#endif

#endif /* RAFI_H */
