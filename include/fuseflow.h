/*
 * fuseflow.h — C ABI of the MI355X (gfx950) fusion library for FUSE-Flow
 * (frame-wise confidence- and consistency-weighted multi-view point fusion with an
 * adaptive spatial hash).
 *
 * What one call computes (paper Sec. II):
 *   Sec. II.1, Eq. 1   input: N cameras with intrinsics K_i, extrinsics T_i, depth D_i,
 *                      per-pixel confidence C_i (Sec. II.2, Eq. 2) and optional RGB I_i;
 *                      output: one fused point cloud per time step, frame-wise and stateless.
 *   Sec. II.4, Eq. 8-9 pixel-wise back-projection and confidence gating (C > tau).
 *   Sec. II.5(1) a-e   world transform, extents, coarse density grid, density-adaptive
 *                      refinement, assignment of every point to its cell (spatial hash).
 *   Sec. II.5(2) a-c   per cell the three most confident points; for each, distance
 *                      consistency V (Eq. 4-7) against at most K locally relevant views;
 *                      joint weight w = C V (Eq. 10).
 *   Sec. II.5(3)       weighted fusion of each cell's representatives (Eq. 11).
 *
 * Readings of points the paper leaves open (all fixed here, bit-for-bit):
 *   - world_to_cam is [R | t] (world -> camera); Eq. 8 applies its inverse.
 *   - depth is z-depth; pixel (x, y) has its centre at integer coordinates.
 *   - a pixel is kept when depth is finite and > 0, C > tau (strict) and the
 *     back-projected point is finite; otherwise it is dropped (Eq. 9's "0").
 *   - coarse grid: coarse_res cells along the longest extent, edge rounded up to a power of
 *     two; level L = smallest L <= max_level with count <= target_per_cell * 4^L.
 *   - representatives: C descending, then x, y, z ascending, then pixel id.
 *   - local views: other cameras whose image contains the nearest-pixel projection (point
 *     in front), ranked by squared distance to the camera centre (ties: centre x, y, z,
 *     camera index); the first min(K, N) - 1 are used; a view with no finite positive depth
 *     at that pixel is skipped; V = exp(-sum d^2 / (m sigma^2)) over the m views used.
 *   - fusion: xyz = sum(w p) / sum(w); weight = mean w; rgb = rint(sum(w rgb) / sum(w)).
 *
 * Conventions for every call:
 *   - All image pointers in ff_view and all pointers in ff_output are DEVICE pointers on the
 *     context's device.  Images are row-major with pitch = width (no padding).
 *   - ff_camera, ff_view, ff_frame, ff_params and ff_output structs themselves are HOST
 *     memory, read during the call only (they may be reused as soon as the call returns).
 *   - Calls are asynchronous and ordered on the given stream (a hipStream_t passed as
 *     void*, NULL = the null stream).  The caller owns inputs and outputs and must keep them
 *     alive until the work queued on the stream completes.
 *   - Return values report errors the host can detect (bad arguments, allocation failure,
 *     HIP errors).  Data-dependent outcomes are written to device memory: *count receives
 *     the number of fused points S; if S > capacity only the first `capacity` points are
 *     written and *status becomes FF_DEV_OVERFLOW.  capacity >= sum(W*H) never overflows.
 *     FF_DEV_ERROR in *status reports a failed internal bounds check (see the enum).
 *   - Pixel ids are frame-global: camera-major (cameras in the order given), then y*W + x.
 *     A frame must have fewer than 2^32 pixels.
 *   - A context is not thread-safe: calls on one context must not overlap from several
 *     host threads; work of successive calls on different streams is ordered by the
 *     library (it reuses one workspace).
 */
#ifndef FUSEFLOW_H
#define FUSEFLOW_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum ff_status {
    FF_OK = 0,
    FF_ERR_INVALID_ARG = 1,   /* a pointer, size or parameter is out of range */
    FF_ERR_OOM = 2,           /* device or pinned allocation failed, or over the budget */
    FF_ERR_BUSY = 3,          /* server: no free slot right now (non-blocking submit) */
    FF_ERR_HIP = 4,           /* a HIP runtime call failed */
    FF_ERR_NOT_FOUND = 5      /* server: unknown ticket */
} ff_status;

/* ff_params.flags: the paper's ablations (Sec. III, Table II), and the confidence source */
enum {
    FF_NO_MF = 1u,   /* no measurement confidence: C := 1, gate on depth only */
    FF_NO_DC = 2u,   /* no distance consistency: V := 1 */
    FF_NO_SA = 4u,   /* no spatial-hash aggregation: every gated point is its own output,
                        in pixel-id order, with V computed per point; keys = pixel ids */
    FF_CONF_EQ3 = 8u /* the confidence is computed on the device from the depth maps by
                        Eq. 3 (Sec. II.2) with the paper's weights, as ff_confidence does;
                        ff_view.conf is ignored and may be NULL */
};

/* values of *ff_output.status */
enum {
    FF_DEV_OK = 0,
    FF_DEV_OVERFLOW = 1,   /* S > capacity (or M > member_capacity): output truncated */
    FF_DEV_ERROR = 2       /* an internal consistency check of the device path failed (an
                              index out of its bounds); raised for every frame of the call
                              that found it, since the frames of a call share the
                              workspace.  Outputs of that call are unreliable. */
};

/* Fusion calls reject (FF_ERR_INVALID_ARG) a camera with a non-finite parameter, a side
 * above 16384 px, a principal point beyond +-16384 px or a focal length outside
 * [2^-20, 2^20] px in magnitude: the range in which the per-cell kernel's approximate
 * field-of-view pre-test is proven to take the exact float32 decisions. */
typedef struct ff_camera {
    int32_t width, height;        /* pixels, 1..16384 */
    float fx, fy, cx, cy;         /* intrinsics K (pixel units) */
    float world_to_cam[12];       /* [R | t] row-major 3x4: X_cam = R X_world + t */
} ff_camera;

typedef struct ff_view {
    const float* depth;           /* device, height*width FP32 z-depth (m); <= 0 or NaN = none */
    const float* conf;            /* device, height*width FP32 confidence in [0, 1] */
    const uint8_t* rgb;           /* device, height*width*3 uint8, or NULL */
} ff_view;

typedef struct ff_params {
    float tau;                    /* Eq. 9 gate threshold (paper: 0.6) */
    int32_t k_views;              /* K of Eq. 7, own camera included, 1..8 (default 4) */
    float sigma;                  /* Eq. 7 tolerance in metres (default 0.02) */
    int32_t coarse_res;           /* coarse cells on the longest axis, power of two <= 128 (64) */
    int32_t max_level;            /* deepest refinement level (6) */
    int32_t target_per_cell;      /* refinement target occupancy (16) */
    int32_t level_override;       /* -1, or a level used in every coarse cell */
    uint32_t flags;               /* FF_NO_MF | FF_NO_DC | FF_NO_SA | FF_CONF_EQ3 */
} ff_params;

typedef struct ff_output {
    float* xyz;                   /* device [capacity][3] fused points (world, m) */
    float* weight;                /* device [capacity] mean joint weight of the cell */
    uint8_t* rgb;                 /* device [capacity][3] or NULL (needs rgb on every view) */
    uint32_t* n_members;          /* device [capacity] gated points in the cell, or NULL */
    uint32_t* reps;               /* device [capacity][3] representative pixel ids,
                                     0xFFFFFFFF padded, or NULL */
    uint64_t* keys;               /* device [capacity] cell key, or NULL:
                                     (coarse << 3Lmax) | (lz << 2Lmax) | (ly << Lmax) | lx */
    uint32_t* member_offsets;     /* device [capacity + 1] or NULL: cell s owns
                                     member_ids[member_offsets[s] .. member_offsets[s+1]) */
    uint32_t* member_ids;         /* device [member_capacity] or NULL: pixel ids of every
                                     gated point grouped by cell, pixel-id order inside */
    uint32_t capacity;            /* entries available in the per-point arrays */
    uint32_t member_capacity;     /* entries available in member_ids */
    uint32_t* count;              /* device [1]: S, the number of fused points */
    int32_t* status;              /* device [1]: FF_DEV_OK, FF_DEV_OVERFLOW or FF_DEV_ERROR */
    uint32_t* info;               /* device [4] or NULL: M (gated points), S, R
                                     (representatives), sort key bits */
} ff_output;

typedef struct ff_frame {
    int32_t n_cams;
    const ff_camera* cams;        /* host [n_cams] */
    const ff_view* views;         /* host [n_cams] */
} ff_frame;

typedef struct ff_context ff_context;

/* Launch/tuning knobs of the device path (chosen by ff_autotune or set by hand).  None of
 * them changes a result, only the time it takes. */
typedef struct ff_tuning {
    int32_t radix_bits;           /* widest digit of the LSD radix sort, 6..10 (the key bits
                                     are spread evenly over the fewest passes) */
    int32_t sort_items;           /* keys per thread per sort tile: 8 or 16 */
    int32_t hist_tiles;           /* 4096-pixel tiles per coarse-histogram workgroup: 1..8,
                                     or 0 (default): about 900 workgroups, i.e. the batch's
                                     tiles / 900 rounded, within 1..8 */
    int32_t cell_groups;          /* workgroups of the per-cell phase, 64..4096, or 0
                                     (default): as many as the device holds resident at
                                     once for the launch (1280 on MI355X: 256 CUs x 5) for
                                     batches of at most 7,372,800 pixels, else twice that */
    int32_t use_graph;            /* 1: ff_fuse_batch replays a cached HIP graph (default) */
} ff_tuning;

/* Library version string. */
const char* ff_version(void);
const char* ff_status_string(ff_status s);

/* Paper constants and this library's defaults (tau 0.6, K 4, sigma 0.02, 64, 6, 16, -1, 0). */
void ff_params_default(ff_params* p);

/* Create a context on `device` able to take batches of up to max_frames frames holding
 * max_pixels pixels and max_cameras cameras in total.  All device workspace is allocated
 * here (nothing is allocated per call afterwards).  FF_ERR_OOM if it does not fit. */
ff_status ff_context_create(ff_context** out, int device, uint64_t max_pixels,
                            int32_t max_cameras, int32_t max_frames);
void ff_context_destroy(ff_context* ctx);

/* Device workspace bytes a context with these limits allocates. */
uint64_t ff_workspace_bytes(uint64_t max_pixels, int32_t max_cameras, int32_t max_frames);

/* Fuse one frame (Sec. II) with one kernel per step. */
ff_status ff_fuse(ff_context* ctx, int32_t n_cams, const ff_camera* cams,
                  const ff_view* views, const ff_params* params, const ff_output* out,
                  void* stream);

/* Fuse n_frames independent frames together: every step runs once over all cameras of all
 * frames (uneven resolutions welcome; the frames are kept apart by disjoint key ranges), and
 * the launches are replayed from a HIP graph cached per batch shape (resolution mix, grid
 * parameters, tuning).  outs[f] receives exactly what ff_fuse would produce for frame f. */
ff_status ff_fuse_batch(ff_context* ctx, int32_t n_frames, const ff_frame* frames,
                        const ff_params* params, const ff_output* outs, void* stream);

/* Tuning.  A context keeps a default tuning (get/set) and a cache of tunings keyed by the
 * batch shape: the frames' camera resolutions in order, the grid and level limits, the
 * flags and the view-list size.  A call uses the cached tuning of its shape, else the
 * default.  ff_autotune times candidate settings on the given batch (one knob at a time:
 * digit width x keys per thread, then histogram tiles, then per-cell workgroups; each
 * candidate once untimed and three times timed, which synchronises the stream and leaves
 * the batch's results in `outs`), caches the fastest for the batch's shape and returns
 * it in *chosen. */
ff_status ff_get_tuning(const ff_context* ctx, ff_tuning* t);
ff_status ff_set_tuning(ff_context* ctx, const ff_tuning* t);
ff_status ff_autotune(ff_context* ctx, int32_t n_frames, const ff_frame* frames,
                      const ff_params* params, const ff_output* outs, void* stream,
                      ff_tuning* chosen);
/* The tuning cached for this batch's shape: *found = 1 and *t filled, or *found = 0. */
ff_status ff_tuning_lookup(const ff_context* ctx, int32_t n_frames, const ff_frame* frames,
                           const ff_params* params, ff_tuning* t, int32_t* found);
/* The shape cache as JSON text ({"device": name, "entries": [{"shape": ..., knobs}, ...]}),
 * for persisting it.  Writes at most cap bytes including the terminating zero into buf
 * (buf may be NULL with cap 0) and the size it needs, terminating zero included, into
 * *needed.  FF_ERR_INVALID_ARG when it does not fit. */
ff_status ff_tuning_export(const ff_context* ctx, char* buf, uint64_t cap, uint64_t* needed);
/* Merge entries of such a JSON text into the shape cache.  Entries recorded for another
 * device name are skipped (*imported counts the rest); a malformed text or knob out of
 * range gives FF_ERR_INVALID_ARG and changes nothing. */
ff_status ff_tuning_import(ff_context* ctx, const char* json, int32_t* imported);

/* Per-kernel timing.  While enabled, ff_fuse brackets every kernel it launches with HIP
 * events on the call's stream (ff_fuse_batch then launches directly instead of replaying a
 * graph).  Slots: 0 back-project + AABB partials, 1 per-frame reduce, 2 coarse histogram,
 * 3..5 coarse scan, 6 keys, 10..12 cell heads, 13 cells (top-3, consistency, fusion),
 * 14 final, 15 camera prep, 16 + 3k + {0, 1, 2}: radix pass k (tile histograms, scan,
 * scatter). */
#define FF_TRACE_SLOTS 32
typedef struct ff_trace {
    double total_ms[FF_TRACE_SLOTS];   /* summed kernel time per slot */
    uint64_t launches[FF_TRACE_SLOTS]; /* launches timed per slot */
    uint64_t calls;                    /* ff_fuse / ff_fuse_batch calls timed */
} ff_trace;
ff_status ff_trace_enable(ff_context* ctx, int32_t on);   /* on resets the totals */
ff_status ff_trace_read(ff_context* ctx, ff_trace* out);  /* waits for the timed work */
const char* ff_trace_slot_name(int32_t slot);

/* Probe: the duration of ONE kernel (a trace slot) in every call, graph replays included.
 * Events are recorded on the call's stream just before and after that kernel; in a graph
 * replay the graph is split around it (the launches before and after it are replayed from
 * graphs cached per segment), so the rest of the call keeps its launch structure.  While
 * per-kernel tracing is on, the probe records nothing.  Totals accumulate from
 * ff_probe_enable (which resets them; slot -1 switches the probe off) until the next enable. */
typedef struct ff_probe {
    int32_t slot;                 /* probed trace slot, -1 = off */
    int32_t reserved;
    uint64_t launches;            /* timed launches of that kernel */
    uint64_t frames;              /* frames those launches processed */
    uint64_t pixels;              /* input pixels of those frames */
    double total_ms;              /* summed kernel time */
} ff_probe;
ff_status ff_probe_enable(ff_context* ctx, int32_t slot); /* waits for recorded launches */
ff_status ff_probe_read(ff_context* ctx, ff_probe* out);  /* waits for recorded launches */

/* ------------------------------------------------------------ measurement confidence
 * Sec. II.2, Eq. 2-3: C = alpha / (1 + beta G) + gamma / (1 + delta sigma_local), divided
 * by alpha + gamma so that C lies in (0, 1] as Eq. 2 states (the printed weights alpha =
 * beta = 0.5, gamma = delta = 1 would span (0, 1.5]).  Readings of what the paper leaves
 * open: G is the magnitude of the central-difference depth gradient in metres per pixel
 * (one-sided where only one neighbour along an axis has a valid depth, 0 where none has);
 * sigma_local is the population standard deviation of the valid depths of the 3x3
 * window around the pixel; pixels without a valid depth (not finite or <= 0) get 0.
 * Computed in float32 with one rounding per operation in a fixed order (the gate and the
 * ranking downstream decide on C exactly). */
typedef struct ff_conf_params {
    float alpha, beta, gamma, delta;   /* Eq. 3 weights (paper: 0.5, 0.5, 1, 1) */
} ff_conf_params;
void ff_conf_params_default(ff_conf_params* p);
/* conf_out[k]: device, height*width FP32 written for camera k, from views[k].depth (the
 * other view fields are not read).  Stream-ordered; no context, nothing allocated.
 * FF_ERR_INVALID_ARG for null pointers, empty images, >= 2^32 pixels per camera or
 * non-finite weights. */
ff_status ff_confidence(int32_t n_cams, const ff_camera* cams, const ff_view* views,
                        float* const* conf_out, const ff_conf_params* params, void* stream);

/* ------------------------------------------------------------ E_MC evaluator
 * Sec. III, Eq. 12: E_MC = mean over the points P of a fused cloud of the mean, over the
 * cameras i that see P, of |z(T_i P) - D_i(pi(T_i P))|.  Readings: a camera sees P when P
 * is in front of it, its nearest pixel (Eq. 4) is inside the image, the depth there is
 * valid, and P is not occluded: z <= D + c_occ z^2.  Points seen by no camera are left
 * out; rho is every `stride`-th point of the cloud.  Decisions in float32 (as the fusion
 * path projects), error sums in double, summed per workgroup and then in a fixed order
 * (deterministic). */
typedef struct ff_emc_params {
    float c_occ;                  /* occlusion tolerance coefficient, 1/m (0.003) */
    int32_t stride;               /* evaluate every stride-th point (1) */
} ff_emc_params;
void ff_emc_params_default(ff_emc_params* p);
/* xyz: device [capacity][3] fused points (e.g. ff_output.xyz), count: device number of
 * points (e.g. ff_output.count, clamped to capacity).  out: device double[3] = {E_MC in
 * metres, points used, mean number of cameras seeing a used point}.  Uses the context's
 * descriptor and a partial-sum workspace; ordered after the context's previous calls.
 * FF_ERR_INVALID_ARG for null pointers, stride < 1, negative c_occ, n_cams outside
 * 1..max_cameras. */
ff_status ff_emc(ff_context* ctx, int32_t n_cams, const ff_camera* cams, const ff_view* views,
                 const float* xyz, const uint32_t* count, uint32_t capacity,
                 const ff_emc_params* params, double* out, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): ff_emc without a context.  Same
 * arguments and result as ff_emc (the same kernels, bit-identical output), on the calling
 * thread's current device.  The camera records and the partial sums live in one static
 * device array of the library (about 64 KiB per device, held until the process ends);
 * nothing is allocated per call.  At most 64 cameras (FF_ERR_INVALID_ARG beyond).  Calls
 * that overlap on one device share that array and race: order them on one stream. */
ff_status ff_emc_noalloc(int32_t n_cams, const ff_camera* cams, const ff_view* views,
                         const float* xyz, const uint32_t* count, uint32_t capacity,
                         const ff_emc_params* params, double* out, void* stream);

/* ------------------------------------------------------------------------------ serving
 * A streaming loop over several rigs (the paper's per-frame statelessness, Sec. II.1, is
 * what makes frames of different rigs independent work).  Frames are admitted as they
 * arrive into batches sized by the device memory budget, run on `lanes` concurrent
 * workspaces/streams (buffers and tables stay resident), and their latency (completion minus
 * arrival) is recorded.  A frame's result is bit-identical to ff_fuse on the same frame.
 * All HIP work of a server happens on its own scheduler thread. */

typedef struct ff_server ff_server;

typedef struct ff_server_config {
    uint64_t hbm_budget_bytes;    /* device memory for all lane workspaces together: frames
                                     are admitted by their workspace footprint against what
                                     the running batches leave of it */
    int32_t lanes;                /* concurrent batches (one stream + workspace each), 1..8 */
    int32_t max_batch_frames;     /* frames per batch, 1..64 */
    int32_t max_cameras;          /* cameras per batch, 1..1024 */
    int32_t max_pending;          /* submitted but not started frames; beyond: FF_ERR_BUSY */
    int32_t plain;                /* 1: baseline loop, one frame at a time through ff_fuse,
                                     the next frame starts after the previous completed */
    int32_t autotune;             /* 1: the first batch of every new batch shape is autotuned
                                     (ff_autotune on its lane, which holds the scheduler for
                                     the search) and the tuning is shared by all lanes */
} ff_server_config;

typedef struct ff_stats {
    uint64_t frames;              /* completed frames */
    uint64_t pixels;              /* their input pixels */
    uint64_t batches;             /* launches (batches) */
    double first_arrival_s;       /* server clock of the first completed frame's arrival */
    double last_done_s;           /* server clock of the last completion */
    double p50_ms, p99_ms, mean_ms, max_ms;   /* frame latency: completion - arrival */
    double px_per_s;              /* pixels / (last_done - first_arrival) */
    double mean_batch_frames;
    uint64_t hbm_used_bytes;      /* device bytes of the lanes' workspaces now */
    uint64_t hbm_peak_bytes;      /* and at most so far (never above the budget) */
} ff_stats;

/* Defaults: 2 lanes, 16 frames per batch, 256 cameras, 4096 pending, not plain, no
 * autotuning. */
void ff_server_config_default(ff_server_config* cfg);

/* Creates the lanes (streams); their workspaces are made when a lane first takes a batch,
 * sized by it (ff_workspace_bytes of the batch's pixels, cameras and frames), and grown
 * when a later batch needs more.  The workspaces of all lanes together never exceed the
 * budget: a frame joins a batch only while the batch still fits what the other lanes leave,
 * otherwise it waits (FIFO) until running batches complete; idle lanes give their
 * workspaces back when the next frame fits nowhere else.  A frame whose own workspace
 * exceeds the whole budget is refused at submit with FF_ERR_OOM.  FF_ERR_OOM here if not
 * even one 4096-pixel frame fits. */
ff_status ff_server_create(ff_server** out, int device, const ff_server_config* cfg);
void ff_server_destroy(ff_server* s);

/* Largest single frame (pixels, with the configured camera limit) the budget admits. */
uint64_t ff_server_max_pixels(const ff_server* s);

/* Size every idle lane's workspace now for a batch of `frames` frames with `pixels` pixels
 * and `cameras` cameras in all (lanes already that large are left as they are), so that
 * streams of such frames meet no workspace creation later.  Lanes are sized in order while
 * the budget allows: FF_ERR_OOM if it ran out before the last lane (the lanes sized so far
 * keep their workspaces), FF_ERR_BUSY if a lane was running a batch (call it before
 * submitting or after a drain), FF_ERR_INVALID_ARG for sizes beyond the configured camera
 * or batch limits. */
ff_status ff_server_reserve(ff_server* s, uint64_t pixels, int32_t cameras, int32_t frames);

/* Seconds on the server clock (steady clock, zero at creation). */
double ff_server_now(const ff_server* s);

/* Queue one frame of rig `rig_id` arriving at `arrival_s` on the server clock (a time in the
 * past, e.g. a negative one, means the moment of this call).  An event is recorded on
 * `stream` (the caller's stream, NULL = the null stream) and the frame's batch waits for
 * it, so work queued there before the submit (writing the images, clearing the outputs)
 * is complete before the frame is read.  The host structs are copied; the device images
 * and `out` buffers must stay valid until the frame is done.  Returns, for this frame
 * only: FF_ERR_INVALID_ARG when the host checks of ff_fuse_batch reject it, FF_ERR_OOM
 * when its workspace exceeds the budget, FF_ERR_BUSY when max_pending frames wait already.
 * Nothing about one frame affects the acceptance of other frames. */
ff_status ff_server_submit(ff_server* s, int32_t rig_id, const ff_frame* frame,
                           const ff_params* params, const ff_output* out, double arrival_s,
                           void* stream, uint64_t* ticket);

/* done = 1 once the frame's results are in its output buffers (its batch's device work has
 * finished).  Once done is reported, the call returns the frame's own status (FF_OK, or the
 * error its batch's launch met) and forgets the ticket: a later poll or wait on it returns
 * FF_ERR_NOT_FOUND. */
ff_status ff_server_poll(ff_server* s, uint64_t ticket, int32_t* done);
/* Block until the frame is done; returns its status and forgets the ticket. */
ff_status ff_server_wait(ff_server* s, uint64_t ticket);
/* Wait until every submitted frame is done and forget all tickets.  Returns FF_OK, or the
 * first error a frame completed with since the previous drain. */
ff_status ff_server_drain(ff_server* s);

ff_status ff_server_stats(const ff_server* s, ff_stats* st);
/* Forget completed frames' latencies (stats restart from zero). */
ff_status ff_server_reset_stats(ff_server* s);
/* The latency of every frame completed since the last reset, in completion order, with
 * its rig: the first min(cap, *n) go to rig_ids and latency_ms (host arrays; either may be
 * NULL), *n is set to how many there are.  For per-rig percentiles beside ff_stats. */
ff_status ff_server_latencies(const ff_server* s, uint64_t cap, int32_t* rig_ids,
                              double* latency_ms, uint64_t* n);
/* The probe on every lane (see ff_probe_enable); read sums the lanes.  Both wait for the
 * lanes' recorded launches to finish. */
ff_status ff_server_probe_enable(ff_server* s, int32_t slot);
ff_status ff_server_probe_read(ff_server* s, ff_probe* out);

#ifdef __cplusplus
}
#endif
#endif /* FUSEFLOW_H */
