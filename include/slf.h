/*
 * slf — superpixel-plane matching cost for sparse light fields on MI355X.
 *
 * Implements the depth path of Chuchvara, Barsi, Gotchev, "Fast and Accurate
 * Depth Estimation from Sparse Light Fields": per-superpixel statistics
 * (Sec. III-A), the partly randomised fronto-parallel plane sweep with the
 * truncated SSD cost (Sec. III-B, eqs. 1-2), the iterative refinement by
 * propagation over a shrinking kernel and triangle normals maximising
 * E = E_c E_s (Sec. III-C, eqs. 3-11, Jacobi ping-pong as in Sec. III-E), and
 * the per-pixel depth readout of the superpixel planes (Sec. III-A: the
 * method's result is one depth map per view).
 *
 * Conventions
 *  - Every call returns an int status: SLF_OK (0) or a negative SLF_E* code.
 *    No exception crosses the ABI.  slf_last_error() gives a message for the
 *    last failing call on a context.
 *  - A context is used by one host thread at a time.  There is no global
 *    state shared between contexts.
 *  - Host buffers are owned by the caller and copied during the call.
 *    Device buffers (is_device = 1) are read or written asynchronously on the
 *    context's stream: the caller keeps them alive and unmodified until
 *    slf_synchronize() (or until later work on that stream has completed).
 *  - Arrays are row-major.  Pixel (u, v): u = column, v = row, centres at
 *    integer coordinates.
 *  - Cameras: X_cam = R X_world + t, pixel ~ K X_cam, K's last row (0,0,1).
 *    Depth is camera-frame z.
 *  - Superpixel labels are seed-grid ids: label k of a grid_w x grid_h grid
 *    is cell (k mod grid_w, k div grid_w); cells may be empty.
 *  - A plane is stored per superpixel as 4 floats (d, nx, ny, nz): the unit
 *    normal n in the view's camera frame and the depth d of the plane at the
 *    superpixel's centroid (Sec. III-A: each superpixel's plane is given by
 *    its depth and orientation at the centroid).  Empty cells hold zeros.
 */
#ifndef SLF_H
#define SLF_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    SLF_OK = 0,
    SLF_EINVAL = -1,       /* bad argument: range, size, non-finite value, invalid plane */
    SLF_ESTATE = -2,       /* call out of order (e.g. sweep before images and labels) */
    SLF_ENOMEM = -3,       /* device or host allocation failed */
    SLF_EDEVICE = -4,      /* HIP runtime error */
    SLF_EUNSUPPORTED = -5  /* valid but not supported (e.g. dimensions above 65535) */
};

/* Method parameters.  struct_size must be sizeof(slf_params). */
typedef struct {
    uint32_t struct_size;
    int32_t levels;             /* L sweep levels (Sec. III-B), >= 1 */
    double d_min, d_max;        /* sweep depth range, 0 < d_min < d_max */
    uint64_t seed;              /* seed of the per-superpixel level jitter */
    int32_t jitter;             /* 1: level k of superpixel s lies at q_min + (k + u) Delta in inverse
                                   depth, u in [0,1) drawn per (view, superpixel, level) (Sec. III-B);
                                   0: u = 0 */
    float tssd_T;               /* truncation T of eq. (1): squared RGB distance, colours in [0,1] */
    float sigma;                /* depth Gaussian sigma of eqs. (6) and (10), scene units */
    float alpha;                /* colour Gaussian alpha of eq. (7), colours in [0,1] */
    float eta;                  /* occlusion regulariser of eq. (11) (0.5 in the paper) */
    float occ_tol;              /* relative tolerance tau: a sample is visible (set X of eq. 10) if
                                   z_i <= D(p^i) (1 + tau), else occluded (set Y of eq. 11) */
    int32_t kernel_step;        /* spacing of far propagation samples in superpixels (5 in Sec. IV-A) */
    int32_t kernel_radius_init; /* initial kernel radius in grid cells; <= 0: floor(min(W,H) / (2 S)),
                                   S = sqrt(W H / (grid_w grid_h)) (kernel size = smallest image
                                   dimension, Sec. IV-A); radius at iteration I is floor(R_init / I) (eq. 4) */
    uint32_t term_mask;         /* bit0 smoothness E_s, bit1 consistency E_c, bit2 occlusion O (Fig. 6) */
    int32_t image_precision;    /* device storage of images: SLF_IMAGE_U8 (default), SLF_IMAGE_F16,
                                   SLF_IMAGE_F32 */
    int32_t homography_fp64;    /* must be 1: refinement composes each candidate's homographies in FP64 on
                                   the device, re-centred on the superpixel (per-sample work is FP32) */
    int32_t energy_mode;        /* 0: E = E_c E_s (eq. 3); 1: E = -normalised TSSD (data-only test mode) */
    int32_t exact_margin;       /* work skipped by exact bounds.  The sweep stops a level once its
                                   partial cost (a sum of terms >= 0) exceeds a complete level's cost;
                                   the refinement stops a candidate once its energy bound falls below
                                   an evaluated candidate's energy.  0 (default): against the best so
                                   far, so the chosen level or candidate, plane and cost or energy are
                                   exact, and the margin (second best against best) is an upper bound
                                   of the exact one, the second best being taken over what was
                                   evaluated in full; 1: against the second best, so the margins are
                                   exact too, at more work.  No stage reads a margin. */
} slf_params;

enum { SLF_IMAGE_U8 = 0, SLF_IMAGE_F16 = 1, SLF_IMAGE_F32 = 2 };

/* Fills p with the defaults: levels 64, [2, 8], seed 0x5EED, jitter on,
 * T = 0.04, sigma = 0.05, alpha = 0.1, eta = 0.5, tau = 1e-3, step 5, radius
 * derived, all terms, U8 images, FP64 homography composition, paper energy,
 * margins as upper bounds (exact_margin 0). */
void slf_default_params(slf_params *p);

typedef struct slf_ctx slf_ctx;

/* Creates a context on HIP device `device_ordinal`; *out receives it.
 * Errors: SLF_EINVAL (bad ordinal or out == NULL), SLF_EDEVICE, SLF_ENOMEM. */
int slf_create(int device_ordinal, slf_ctx **out);
/* Releases the context and every device buffer it owns (waits for its stream). */
int slf_destroy(slf_ctx *ctx);
/* Runs all later work on `hip_stream` (a hipStream_t; NULL = the default stream).
 * The stream must outlive its use by the context. */
int slf_set_stream(slf_ctx *ctx, void *hip_stream);
/* Validates and copies the parameters.  SLF_EINVAL on any bad field. */
int slf_set_params(slf_ctx *ctx, const slf_params *p);

/* Cameras of all n_views views (Sec. III-A: a calibrated camera system).
 * wh[n][2] = (W, H) with 2 <= W, H <= 65535; K[n][9], R[n][9] row-major with
 * R orthonormal (within 1e-6) and K's last row (0,0,1); t[n][3].  Resets
 * images, labels, neighbour lists (to all other views, ascending) and planes.
 * SLF_EINVAL for a side below 2, a count outside [2, 4096] or non-finite
 * values; SLF_EUNSUPPORTED for a side above 65535.  The kernels' per-sample
 * FP32 arithmetic works on pixel offsets re-centred per superpixel (constants
 * composed in FP64), so its accuracy does not depend on the image size. */
int slf_set_cameras(slf_ctx *ctx, int n_views, const int32_t *wh, const double *K, const double *R,
                    const double *t);
/* Neighbour views N(r) of view `view` used by eqs. (2) and (8); n >= 1
 * distinct views other than `view`.  Default: all other views, ascending.
 * N(r) is a set: the kernels visit it in decreasing distance between camera
 * centres (ties in the given order), so the views with the widest baselines,
 * which separate depth hypotheses most, come first and the exact bounds of
 * the sweep and the refinement stop earlier.  The order changes no decision,
 * only the FP32 rounding of the per-view sums. */
int slf_set_neighbors(slf_ctx *ctx, int view, int n, const int32_t *views);
/* RGB8 image of a view, H rows of W * 3 bytes separated by row_stride_bytes
 * (>= 3 W).  is_device = 1: rgb is a device pointer read on the stream. */
int slf_set_image_rgb8(slf_ctx *ctx, int view, const uint8_t *rgb, int64_t row_stride_bytes, int is_device);
/* Superpixel labels of a view (Sec. III-A: the SLIC segmentation, read as
 * an approximately regular grid of cells with a conventional neighbour
 * system), int32, H rows separated by row_stride_elems (>= W); grid_w *
 * grid_h <= 2^24 cells.  Host labels are range-checked here
 * (SLF_EINVAL); device labels are checked when superpixels are built and an
 * out-of-range label makes slf_sweep / slf_propagate fail with SLF_EINVAL. */
int slf_set_labels(slf_ctx *ctx, int view, const int32_t *labels, int64_t row_stride_elems, int grid_w,
                   int grid_h, int is_device);

/* Segments the view's image (set with slf_set_image_rgb8) on the GPU into
 * grid_w x grid_h SLIC superpixels and makes them the view's labels, as
 * slf_set_labels would (Sec. III-A: SLIC superpixels read as a regular grid of
 * cells; Sec. III-E: the segmentation runs on the GPU).  Cluster k = gy gw +
 * gx starts at the centre of grid cell (gx, gy) with the colour of the nearest
 * pixel; each of `iterations` passes assigns every pixel to the closest centre
 * of the 3 x 3 cells around its own, D = |rgb - rgb_k|^2 + ((u - u_k)^2 + (v
 * - v_k)^2) (2.55 compactness)^2 gw gh / (W H) with colours in 0..255 (ties:
 * the first centre in row-major order of the 3 x 3 cells), and moves each
 * centre to the mean position and colour of its pixels between passes.  Then
 * each label keeps only its largest 4-connected component (equal sizes: the
 * one whose first pixel in raster order comes first); every other component
 * takes the final label of the component holding the pixel left of its first
 * pixel, or above it in the first column (the component holding pixel (0,0)
 * keeps its label).  Results are deterministic.  SLF_ESTATE without an image;
 * SLF_EINVAL unless 1 <= grid_w <= W, 1 <= grid_h <= H, grid_w grid_h <=
 * 2^24, iterations >= 1 and compactness finite and >= 0.  Allocates its
 * working buffers (12 bytes per pixel, 28 per cluster) on first use.
 * Asynchronous. */
int slf_segment(slf_ctx *ctx, int view, int grid_w, int grid_h, int iterations, float compactness);
/* Copies a view's labels (set or segmented): H rows separated by
 * row_stride_elems (>= W).  is_device = 0: host buffer, synchronises; 1:
 * device buffer, asynchronous.  SLF_ESTATE if the view has no labels. */
int slf_get_labels(slf_ctx *ctx, int view, int32_t *out, int64_t row_stride_elems, int is_device);

/* Builds the device image texels and the superpixel pixel lists and
 * statistics (Sec. III-A, III-C-1: area, centroid, mean colour) for the
 * current images and labels.  slf_sweep, slf_set_planes and slf_propagate do
 * this themselves when inputs changed; calling it first separates the setup
 * from the sweep.  Synchronises (label range errors surface here as
 * SLF_EINVAL).  SLF_ESTATE unless cameras, images and labels are set;
 * SLF_EUNSUPPORTED if the image texels of all views would exceed 4 GiB
 * ((W+1)(H+1) entries per view of 8 bytes for SLF_IMAGE_U8 and
 * SLF_IMAGE_F16, 16 bytes for SLF_IMAGE_F32). */
int slf_prepare(slf_ctx *ctx);
/* Plane sweep (Sec. III-B) over all superpixels of all views: builds the
 * superpixel pixel lists and statistics if images or labels changed, then for
 * each superpixel picks the level minimising eq. (2) (ties: smallest level)
 * and stores the fronto-parallel plane as the current state.  Per-superpixel
 * outputs: normalised cost C / (|Omega| |N(r)| T) in [0,1], level index and
 * margin (second best minus best normalised cost).
 * SLF_ESTATE unless cameras, images and labels are set for every view. */
int slf_sweep(slf_ctx *ctx);
/* Replaces the current planes of a view ([grid_w * grid_h][4] host floats,
 * see the plane convention; Sec. III-E: the state the next refinement
 * iteration reads, as the initial planes of Sec. III-B are).  Non-empty cells need a finite d > 0 and a unit
 * normal (within 1e-3) facing the camera at the cell's centroid; SLF_EINVAL
 * otherwise.  Entries of empty cells are ignored.  Needs cameras, images and
 * labels (SLF_ESTATE). */
int slf_set_planes(slf_ctx *ctx, int view, const float *planes);
/* Refinement iterations I = first_iter .. first_iter + n_iters - 1 (Sec.
 * III-C), all superpixels of all views in parallel, reading the current state
 * and writing the next (ping-pong), then making it current.  Per superpixel:
 * candidates in slot order (0 current plane, 1 + j ring neighbour j, 9 + 8 (m /
 * step - 1) + j the cell m cells away in ring direction j for m = step, 2
 * step, ... <= floor(R_init / I); then 1000 + j the plane through the
 * superpixel's 3D centroid at the winner's depth and the 3D centroids of ring
 * neighbours j and j + 1); a candidate replaces the best only if its energy
 * is strictly larger.  Outputs energy, winning slot and margin (best minus
 * second-best energy).  SLF_ESTATE before slf_sweep or slf_set_planes for
 * every view; SLF_EINVAL if first_iter < 1 or n_iters < 0. */
int slf_propagate(slf_ctx *ctx, int first_iter, int n_iters);
/* Copies the current state of a view to host arrays of grid_w * grid_h
 * entries; any output pointer may be NULL.  energy_or_cost receives the sweep
 * cost after slf_sweep and the energy after slf_propagate; choice the level or
 * slot (-1 for empty cells); margin as described above.  Synchronises. */
int slf_get_planes(slf_ctx *ctx, int view, float *planes, float *energy_or_cost, int32_t *choice, float *margin);
/* Per-pixel depth D(p) of the view from its superpixel's plane (Sec. III-A:
 * the depth values of each superpixel are described by its plane; the
 * method outputs one depth map per view), 0 where the plane does not face
 * the camera: H rows separated by row_stride_elems.
 * is_device = 0 synchronises and copies to the host; 1 writes the device
 * buffer asynchronously. */
int slf_get_depth(slf_ctx *ctx, int view, float *out, int64_t row_stride_elems, int is_device);
/* Superpixel statistics of a view (after slf_sweep / slf_set_planes): area
 * [K] int32, centroid [K][2] (u, v), mean colour [K][3] in [0,1]; NULL skips
 * an output.  Synchronises. */
int slf_get_superpixels(slf_ctx *ctx, int view, int32_t *area, float *centroid, float *colour);
/* Work done since the last reset; any output may be NULL.  evals: SP-plane
 * hypotheses decided (one (view, superpixel, plane) score: a sweep level or
 * a refinement candidate).  samples: px-view samples computed (one pixel
 * tested in one neighbour view under one plane).  pruned: refinement
 * candidates decided before their consistency term (eq. 8) was complete:
 * after each neighbour view, the smoothness times an upper bound of the
 * consistency term (views left contributing at most 1 + occlusion weight)
 * lay below the floor, so the candidate could not change the result.  The
 * floor is the best energy so far by default (exact_margin = 0: winner,
 * plane and energy are exact and the margin is an upper bound of the exact
 * one) or the second best (exact_margin = 1: the margin is exact too).
 * Pruned candidates count in evals; only the samples of the views computed
 * count in samples.  Sweep levels are decided the same way (see
 * slf_get_sweep_work): every level counts in evals, only the samples
 * computed count in samples.  Synchronises. */
int slf_get_work(slf_ctx *ctx, uint64_t *evals, uint64_t *samples, uint64_t *pruned);
/* Sweep work since the last reset; either output may be NULL.  The sweep
 * (Sec. III-B, eq. 2) scores levels in chunks; each px-view sample costs
 * >= 0, so a level's partial cost bounds its cost from below, and a chunk
 * stops once every level in it is bounded above a complete level's cost:
 * the best so far by default (exact_margin = 0: level, plane and cost are
 * those of the full sweep and the margin is an upper bound of the exact
 * one), the second best with exact_margin = 1 (the margin is exact too).
 * computed: px-view samples the sweeps computed (the coarse pre-pass that
 * orders the chunks included); total: the samples of a sweep without that
 * bound (pixels x neighbour views x levels).  Synchronises. */
int slf_get_sweep_work(slf_ctx *ctx, uint64_t *computed, uint64_t *total);
/* Sweep levels since the last reset (Sec. III-B): scored, those whose cost
 * (eq. 2) was summed over every pixel and neighbour view, i.e. not stopped by
 * the level bound of slf_get_sweep_work; decided, every level of every
 * non-empty superpixel (the sweep's share of slf_get_work's evals).  Either
 * output may be NULL.  Synchronises. */
int slf_get_sweep_levels(slf_ctx *ctx, uint64_t *scored, uint64_t *decided);
int slf_reset_work(slf_ctx *ctx);
/* Waits for all work enqueued by the context. */
int slf_synchronize(slf_ctx *ctx);

/* Warm start for a new frame of a static rig: after new images and labels
 * were set on the same cameras and label grids, each grid cell keeps its 3D
 * plane from the previous frame's current state, with the depth taken at
 * the cell's new centroid.  A cell that was empty in the previous frame, or
 * whose plane does not face the camera at its new centroid, starts as the
 * fronto-parallel plane at depth 2 / (1/d_min + 1/d_max).  Refinement then
 * continues with slf_propagate, usually from I = 1.  (Not part of the paper,
 * which processes frames independently (Sec. IV); a serving form.)
 * SLF_ESTATE unless every view had planes when the new images or labels
 * were set, with unchanged cameras and grids. */
int slf_warm_start(slf_ctx *ctx);
/* Device bytes the context holds once set up for its cameras, label grids
 * and image precision (images, labels, texels, superpixel lists, plane
 * state); the figure a pool admits against.  SLF_ESTATE before cameras and
 * labels are set. */
int slf_get_footprint(slf_ctx *ctx, uint64_t *bytes);

/* Stability-based depth fusion (Sec. III-D), the two passes per reference
 * view of Sec. III-E run for every view at once.  Pass 1: each pixel of every
 * view with a depth is lifted to its 3D point and projected into every other
 * view; the nearest pixel (round half up) of that reference receives the
 * point's depth in the reference camera as this view's candidate, the closest
 * point winning when several land on one pixel.  Pass 2: at each reference
 * pixel the candidates are its own depth and one per other view; a non-zero
 * candidate c_j gains one for every other non-zero candidate c_k with
 * |c_k - c_j| <= agree_tol c_j and loses one for every other; the fused depth
 * is the smallest candidate whose stability is >= 0 (equal depths: the
 * smaller view index), 0 where there is none.  Depth maps and candidates are
 * FP32; the projection is FP64 as one fixed sequence of correctly rounded
 * operations (ray by Cramer's rule on K's upper 2 x 2 block, world point, the
 * reference's camera, projection); the agreement test is FP32.
 *
 * slf_fuse: fuses the depth maps of the current planes of all views (those
 * slf_get_depth returns) and keeps the result in the context.  Needs planes
 * for every view (SLF_ESTATE).  agree_tol >= 0, finite (SLF_EINVAL); at most
 * 64 views (SLF_EUNSUPPORTED).  On first use it allocates 12 bytes per pixel
 * plus 4 (V - 1) bytes per pixel of candidate layers; these are not part of
 * slf_get_footprint.  Asynchronous. */
int slf_fuse(slf_ctx *ctx, float agree_tol);
/* Fused depth of a view after slf_fuse: H rows separated by row_stride_elems
 * (>= W) into out (may be NULL), and, if votes is not NULL, the pass-2 record
 * of each pixel in the same layout: bits 0-7 the winning view (255: none),
 * bits 8-15 the number of non-zero candidates, bits 16-31 the winner's
 * stability as a signed 16-bit value (0 if none).  is_device = 1: out and
 * votes are device buffers written asynchronously; 0: host buffers, the call
 * synchronises.  SLF_ESTATE before slf_fuse. */
int slf_get_fused_depth(slf_ctx *ctx, int view, float *out, int64_t row_stride_elems, int32_t *votes, int is_device);
/* The same fusion on caller depth maps: depth[v], fused[v] (and votes[v] if
 * votes is not NULL, layout as above) are device buffers of H_v x W_v values
 * (row stride W_v) for every view v of the context's cameras; depths <= 0,
 * NaN or inf are no depth.  Only the cameras need to be set (SLF_ESTATE).
 * The candidate layers (4 (V - 1) bytes per pixel) are the context's,
 * allocated on first use.  Asynchronous on the context's stream: the caller
 * keeps the buffers alive until it completes. */
int slf_fuse_depth(slf_ctx *ctx, const float *const *depth, float *const *fused, int32_t *const *votes,
                   float agree_tol);

/* slf_fuse_depth for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops, harnesses that forbid hipMalloc): the same
 * kernels and results as slf_fuse_depth, run one reference view at a time, with
 * the camera table and that view's candidate layers in a fixed device array of
 * 64 MiB that the library holds on each device it runs on until the process
 * ends.  The call allocates nothing (no hipMalloc, no host-pinned memory); the
 * caller still passes the depth, fused and votes buffers.  Each view v needs
 * 4 (V - 1) W_v H_v <= 64 MiB - 16 KiB bytes of layers (about 16.7 M entries:
 * 8 views of 1920 x 1080 or 16 views of 1280 x 720 fit), else SLF_EUNSUPPORTED
 * before anything runs.  Every call on a device shares that device's array and
 * leaves its last contents there; each call clears what it reads, but calls
 * that overlap on one device (other streams, other contexts, other threads)
 * race and give undefined results.  Asynchronous on the context's stream;
 * other errors as slf_fuse_depth. */
int slf_fuse_depth_static(slf_ctx *ctx, const float *const *depth, float *const *fused, int32_t *const *votes,
                          float agree_tol);

const char *slf_status_string(int status);
/* Message of the last failing call on ctx ("" if none); valid until the next call. */
const char *slf_last_error(const slf_ctx *ctx);

/* ------------------------------------------------------------------------
 * Rig pool: many contexts ("rigs") driven together on one device.
 *
 * A pool accounts the footprint of attached rigs against an HBM budget
 * (admission) and runs their work in stages.  A stage runs, for every
 * active request, its next operation (the sweep or one refinement
 * iteration); requests of the same operation and image format share one
 * persistent launch whose waves pull (rig, superpixel-tile) items from a
 * device work queue, XCD by XCD.  The arithmetic per superpixel is that of
 * slf_sweep / slf_propagate, so a rig's results are identical whether it runs
 * alone, through a pool, alone in a pool or in a mix.
 *
 * Ordering: a request's stages start after all work enqueued on the rig's
 * stream before slf_pool_submit; once its last stage is launched, the rig's
 * stream waits for it, so later calls on the rig see its result.  Between
 * submit and the launch of its last stage every call on the rig returns
 * SLF_ESTATE.  A pool is used by one host thread at a time.
 * ---------------------------------------------------------------------- */
typedef struct slf_pool slf_pool;

enum {
    SLF_POOL_SOLVE = 0,      /* the sweep, then the iterations */
    SLF_POOL_PROPAGATE = 1   /* the iterations only, from the current planes */
};

/* Launch shape of pooled stages.  struct_size must be sizeof(slf_pool_config). */
typedef struct {
    int32_t struct_size;
    int32_t sweep_level_chunk;  /* sweep levels scored per pass over the pixels: 4, 8 or 16 (default 8) */
    int32_t sweep_tile;         /* superpixels per work item in sweep stages, 1..64 (default 1) */
    int32_t refine_tile;        /* superpixels per work item in refinement stages, 1..64 (default 1) */
    int32_t blocks_per_cu;      /* persistent workgroups per compute unit; 0 = as many as are resident */
    int32_t use_graph;          /* 1: slf_pool_run captures its stage sequence as a HIP graph, replayed
                                   while the sequence's shape repeats (default 1) */
    int32_t sweep_level_split;  /* sweep work items cover 1/split of a tile's levels (hypothesis chunks;
                                   the parts are merged in level order), 1..16 (default 1) */
} slf_pool_config;

void slf_pool_default_config(slf_pool_config *cfg);
/* A pool on device_ordinal with hbm_budget_bytes of admission budget (0: the
 * device's total memory) and a stream of its own. */
int slf_pool_create(int device_ordinal, uint64_t hbm_budget_bytes, slf_pool **out);
/* Waits for the pool's work, detaches every rig and frees the pool. */
int slf_pool_destroy(slf_pool *pool);
/* Runs the pool's work on `stream` (hipStream_t; NULL: the pool's own).
 * SLF_ESTATE while requests are active. */
int slf_pool_set_stream(slf_pool *pool, void *stream);
int slf_pool_set_config(slf_pool *pool, const slf_pool_config *cfg);
int slf_pool_get_config(slf_pool *pool, slf_pool_config *cfg);
/* Admits a rig whose cameras and label grids are set: SLF_ENOMEM, with no
 * change, if its footprint does not fit the budget left; SLF_EUNSUPPORTED
 * beyond 64 rigs; SLF_ESTATE if it is attached already. */
int slf_pool_attach(slf_pool *pool, slf_ctx *rig);
/* Releases a rig's footprint; SLF_ESTATE while it has a request in flight. */
int slf_pool_detach(slf_pool *pool, slf_ctx *rig);
/* Budget, bytes admitted, rigs attached and requests active; NULL skips. */
int slf_pool_usage(slf_pool *pool, uint64_t *budget, uint64_t *used, int *n_rigs, int *n_active);
/* Queues a request for an attached rig (one at a time per rig): op
 * SLF_POOL_SOLVE or SLF_POOL_PROPAGATE, iterations first_iter ..
 * first_iter + n_iters - 1.  Builds the rig's superpixels if its inputs
 * changed (synchronising the rig's stream).  Nothing is launched until
 * slf_pool_step or slf_pool_run.  SLF_ENOMEM if the rig's footprint grew past
 * the budget; SLF_ESTATE for PROPAGATE without planes. */
int slf_pool_submit(slf_pool *pool, slf_ctx *rig, int op, int first_iter, int n_iters, uint64_t tag);
/* Launches one stage of every active request; *n_active (may be NULL)
 * receives the number still active afterwards.  Asynchronous. */
int slf_pool_step(slf_pool *pool, int *n_active);
/* Launches every active request to its end (one graph replay when
 * use_graph = 1 and the schedule fits 64 groups, else stage by stage).
 * Asynchronous. */
int slf_pool_run(slf_pool *pool);
/* Tags of requests whose work has completed (at most max per call, each
 * reported once); does not block. */
int slf_pool_poll(slf_pool *pool, uint64_t *done_tags, int max, int *n_done);
/* Waits for all work launched by the pool. */
int slf_pool_synchronize(slf_pool *pool);
/* Picks sweep_level_chunk, sweep_tile, sweep_level_split and refine_tile by timing sweep and
 * refinement stages over the attached rigs (each trial capped at 2048
 * superpixels per rig), then keeps the fastest; results are cached per set of
 * (resolution, neighbours, levels, precision, views) and *from_cache (may be
 * NULL) is set to 1 on a hit.  Leaves every rig as after slf_sweep, with its
 * work counters unchanged.  SLF_ESTATE while requests are active. */
int slf_pool_autotune(slf_pool *pool, int *from_cache);
const char *slf_pool_last_error(const slf_pool *pool);

#ifdef __cplusplus
}
#endif
#endif
