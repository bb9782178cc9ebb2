/*
 * slf — superpixel-plane matching cost for sparse light fields on MI355X.
 *
 * Implements the depth path of Chuchvara, Barsi, Gotchev, "Fast and Accurate
 * Depth Estimation from Sparse Light Fields": per-superpixel statistics
 * (Sec. III-A), the partly randomised fronto-parallel plane sweep with the
 * truncated SSD cost (Sec. III-B, eqs. 1-2), the iterative refinement by
 * propagation over a shrinking kernel and triangle normals maximising
 * E = E_c E_s (Sec. III-C, eqs. 3-11, Jacobi ping-pong as in Sec. III-E), and
 * the per-pixel depth readout of the superpixel planes (Sec. III-A: "the
 * output is a set of corresponding depth maps").
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
 *    superpixel's centroid (Sec. II: planes are "a single depth value at a
 *    superpixel centroid and a normal vector").  Empty cells hold zeros.
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
} slf_params;

enum { SLF_IMAGE_U8 = 0, SLF_IMAGE_F16 = 1, SLF_IMAGE_F32 = 2 };

/* Fills p with the defaults: levels 64, [2, 8], seed 0x5EED, jitter on,
 * T = 0.04, sigma = 0.05, alpha = 0.1, eta = 0.5, tau = 1e-3, step 5, radius
 * derived, all terms, U8 images, FP64 homography composition, paper energy. */
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
 * SLF_EINVAL on bad sizes or non-finite values. */
int slf_set_cameras(slf_ctx *ctx, int n_views, const int32_t *wh, const double *K, const double *R,
                    const double *t);
/* Neighbour views N(r) of view `view` used by eqs. (2) and (8); n >= 1
 * distinct views other than `view`.  Default: all other views, ascending. */
int slf_set_neighbors(slf_ctx *ctx, int view, int n, const int32_t *views);
/* RGB8 image of a view, H rows of W * 3 bytes separated by row_stride_bytes
 * (>= 3 W).  is_device = 1: rgb is a device pointer read on the stream. */
int slf_set_image_rgb8(slf_ctx *ctx, int view, const uint8_t *rgb, int64_t row_stride_bytes, int is_device);
/* Superpixel labels of a view, int32, H rows separated by row_stride_elems
 * (>= W); grid_w * grid_h <= 2^24 cells.  Host labels are range-checked here
 * (SLF_EINVAL); device labels are checked when superpixels are built and an
 * out-of-range label makes slf_sweep / slf_propagate fail with SLF_EINVAL. */
int slf_set_labels(slf_ctx *ctx, int view, const int32_t *labels, int64_t row_stride_elems, int grid_w,
                   int grid_h, int is_device);

/* Builds the device image texels and the superpixel pixel lists and
 * statistics (Sec. III-A, III-C-1: area, centroid, mean colour) for the
 * current images and labels.  slf_sweep, slf_set_planes and slf_propagate do
 * this themselves when inputs changed; calling it first separates the setup
 * from the sweep.  Synchronises (label range errors surface here as
 * SLF_EINVAL).  SLF_ESTATE unless cameras, images and labels are set. */
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
 * see the plane convention).  Non-empty cells need a finite d > 0 and a unit
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
/* Per-pixel depth D(p) of the view from its superpixel's plane (0 where the
 * plane does not face the camera): H rows separated by row_stride_elems.
 * is_device = 0 synchronises and copies to the host; 1 writes the device
 * buffer asynchronously. */
int slf_get_depth(slf_ctx *ctx, int view, float *out, int64_t row_stride_elems, int is_device);
/* Superpixel statistics of a view (after slf_sweep / slf_set_planes): area
 * [K] int32, centroid [K][2] (u, v), mean colour [K][3] in [0,1]; NULL skips
 * an output.  Synchronises. */
int slf_get_superpixels(slf_ctx *ctx, int view, int32_t *area, float *centroid, float *colour);
/* Work done since the last reset: SP-plane hypothesis evaluations (one
 * (view, superpixel, plane) score) and px-view samples (one pixel tested in
 * one neighbour view under one plane).  Synchronises. */
int slf_get_work(slf_ctx *ctx, uint64_t *evals, uint64_t *samples);
int slf_reset_work(slf_ctx *ctx);
/* Waits for all work enqueued by the context. */
int slf_synchronize(slf_ctx *ctx);

const char *slf_status_string(int status);
/* Message of the last failing call on ctx ("" if none); valid until the next call. */
const char *slf_last_error(const slf_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif
