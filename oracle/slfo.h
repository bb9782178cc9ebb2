/*
 * slfo — plain FP64 CPU oracle of the superpixel-plane matching cost
 * (Chuchvara, Barsi, Gotchev, "Fast and Accurate Depth Estimation from Sparse
 * Light Fields", Sec. III-A to III-C, eqs. (1)-(11)).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header or constant table with the HIP library and never calls it.
 *
 * Conventions (also stated where each is used):
 *  - pixels: u = column, v = row, centres at integers, p~ = (u, v, 1);
 *  - cameras: X_c = R X_w + t, pixel ~ K X_c, K last row (0, 0, 1); depth =
 *    camera z; R_ri = R_i R_r^T, t_ri = t_i - R_ri t_r;
 *  - colour: rgb / 255 in [0, 1]^3;
 *  - superpixel labels are seed-grid ids k <-> cell (k mod gw, k div gw);
 *  - a plane of superpixel s in view r is stored as (d, nx, ny, nz): unit
 *    normal n and depth d at the centroid c_s; the 3D plane is n.X = delta
 *    with delta = d (n . K_r^-1 c~_s) > 0.
 * Every function returns 0 on success or a negative code on bad arguments.
 */
#ifndef SLFO_H
#define SLFO_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t levels;             /* L sweep levels (Sec. III-B) */
    double d_min, d_max;        /* sweep depth range */
    uint64_t seed;              /* jitter hash seed */
    int32_t jitter;             /* 1: per-superpixel random offset inside each level bin */
    double tssd_T;              /* truncation T of eq. (1), squared [0,1]^3 colour distance */
    double sigma;               /* depth Gaussian sigma, eqs. (6), (10) */
    double alpha;               /* colour Gaussian alpha, eq. (7) */
    double eta;                 /* occlusion regulariser, eq. (11) */
    double occ_tol;             /* relative tolerance tau of the D(p) <= D(p^i) split */
    int32_t kernel_step;        /* spacing of far propagation samples, superpixels */
    int32_t kernel_radius_init; /* <= 0: floor(min(W,H) / (2 S)) */
    uint32_t term_mask;         /* bit0 smoothness, bit1 consistency, bit2 occlusion */
    int32_t energy_mode;        /* 0: E = E_c E_s (eq. 3); 1: E = -normalised TSSD */
} slfo_params;

typedef struct {
    int32_t n_views;
    const int32_t *width, *height;   /* [V] */
    const int32_t *grid_w, *grid_h;  /* [V] */
    const double *K, *R, *t;         /* [V][9], [V][9], [V][3] row-major */
    const uint8_t *rgb;              /* views concatenated, each H x W x 3 */
    const int32_t *labels;           /* views concatenated, each H x W */
    const int64_t *pix_off;          /* [V+1] pixel offset of each view */
    const int32_t *nbr_off, *nbr;    /* neighbour view lists, CSR: [V+1], [nbr_off[V]] */
} slfo_rig;

typedef struct slfo_ctx slfo_ctx;

/* Builds per-superpixel pixel lists and statistics.  The rig's arrays must
 * outlive the context (they are not copied).  *err receives 0 or a negative
 * code (-1 bad argument, -2 label out of range, -3 out of memory). */
slfo_ctx *slfo_create(const slfo_rig *rig, const slfo_params *p, int *err);
void slfo_destroy(slfo_ctx *c);
int slfo_set_params(slfo_ctx *c, const slfo_params *p);
void slfo_set_threads(int n);

int64_t slfo_sp_offset(const slfo_ctx *c, int view); /* first global superpixel index of a view */
int64_t slfo_sp_total(const slfo_ctx *c);
/* area [S], centroid [S][2] (u, v), colour [S][3] in [0,1], over all views */
int slfo_sp_stats(const slfo_ctx *c, int32_t *area, double *centroid, double *colour);

uint64_t slfo_mix64(uint64_t z);
double slfo_level_q(const slfo_ctx *c, int view, int sp, int k);
int slfo_kernel_radius(const slfo_ctx *c, int view, int iter);
int slfo_homography(const slfo_ctx *c, int r, int i, const double n[3], double delta, double H[9]);

/* normalised TSSD cost C / (A N T) of an arbitrary stored plane (d, n) for (view, sp) */
double slfo_sweep_cost_plane(const slfo_ctx *c, int view, int sp, const double plane[4]);

/* sweep of one superpixel / of all superpixels of all views.  Outputs per
 * superpixel: plane (d, 0, 0, 1), normalised cost, level index, margin
 * (second-best minus best normalised cost; +inf for one level).  Empty
 * superpixels get plane 0, cost 0, choice -1, margin 0. */
int slfo_sweep_sp(const slfo_ctx *c, int view, int sp, double plane[4], double *cost, int32_t *choice,
                  double *margin);
int slfo_sweep_all(const slfo_ctx *c, double *planes, double *cost, int32_t *choice, double *margin);

/* energy (eq. 3) of stored plane `plane` for (view, sp) given state A [S][4] */
double slfo_energy(const slfo_ctx *c, const double *A, int view, int sp, const double plane[4]);

/* Parity instrument: an upper bound of the change of the energy of `plane`
 * when sample decisions of eqs. (9)-(11) that lie within eps_px of a
 * nearest-pixel threshold or within eps_rel of the visibility split flip; 0 if
 * none is that close. */
double slfo_energy_flip_bound(const slfo_ctx *c, const double *A, int view, int sp, const double plane[4],
                              double eps_px, double eps_rel);

/* one refinement iteration (propagation then normals, Jacobi in A -> B) */
int slfo_refine_sp(const slfo_ctx *c, const double *A, int iter, int view, int sp, double plane[4],
                   double *energy, int32_t *choice, double *margin);
int slfo_refine_all(const slfo_ctx *c, const double *A, int iter, double *B, double *energy, int32_t *choice,
                    double *margin);
/* every evaluated slot of one refinement step, in evaluation order; returns count or < 0 */
int slfo_refine_trace(const slfo_ctx *c, const double *A, int iter, int view, int sp, int32_t *slots,
                      double *planes, double *energies, int cap);

/* Test hook: the refinement step with its propagation stage resolved toward
 * `pivot_slot` (an evaluated propagation slot), as a tie-break would: the
 * normals pivot at that candidate and replace it only on strict improvement.
 * Fills the final plane / energy / choice and the trace (propagation slots,
 * then the normals); returns the trace length, -2 if the slot was not
 * evaluated, or < 0 on bad arguments. */
int slfo_refine_pivot(const slfo_ctx *c, const double *A, int iter, int view, int sp, int pivot_slot, double plane[4],
                      double *energy, int32_t *choice, int32_t *slots, double *planes, double *energies, int cap);

/* per-pixel depth of view `view` from planes [S][4]; 0 where undefined */
int slfo_render_depth(const slfo_ctx *c, const double *planes, int view, double *out);

/* Stability-based depth fusion (Sec. III-D; two passes per reference view,
 * Sec. III-E).  Cameras as in slfo_rig: wh [V][2], K, R [V][9], t [V][3];
 * depth: FP32 depth maps of all views concatenated (H x W each, <= 0 = none).
 *
 * slfo_fuse_project: pass 1 for one (reference, source) pair: cand [H_r][W_r]
 * receives, per reference pixel, the smallest camera-r depth of the source
 * pixels whose 3D points project to it (nearest pixel, round half up), 0 if
 * none.
 * slfo_fuse_vote: pass 2 on one pixel: candidates c[n] (0 = none) in view
 * order; stability[j] = #agreeing - #disagreeing other non-zero candidates,
 * agreement |c_k - c_j| <= tau c_j in FP32; returns the index of the smallest
 * candidate with stability >= 0 (equal depths: smaller index) or -1.
 * slfo_fuse_view: both passes for reference view `ref` (the reference's own
 * depth is its candidate); fused [H_r][W_r]; winner (view index or -1),
 * stability (the winner's, 0 if none) and n_cand (non-zero candidates) may
 * be NULL.  V <= 64. */
int slfo_fuse_project(int n_views, const int32_t *wh, const double *K, const double *R, const double *t,
                      const float *depth, int ref, int src, float *cand);
int slfo_fuse_vote(int n, const float *c, float tau, int32_t *stability);
int slfo_fuse_view(int n_views, const int32_t *wh, const double *K, const double *R, const double *t,
                   const float *depth, int ref, float tau, float *fused, int32_t *winner, int32_t *stability,
                   int32_t *n_cand);

/* Grid-seeded SLIC segmentation (Sec. III-A; its GPU form, Sec. III-E); the
 * definition is in slfo_slic.c.  rgb H x W x 3; labels H x W; centres [gw gh][5]
 * = (u, v, r, g, b) in FP32.  slfo_slic: `iterations` assignment passes with a
 * centre update between consecutive ones, then (connectivity != 0) the
 * connectivity step.  Returns 0, -1 bad arguments, -2 a label out of range,
 * -3 out of memory. */
float slfo_slic_weight(int W, int H, int gw, int gh, double compactness);
int slfo_slic_centres_init(int W, int H, const uint8_t *rgb, int gw, int gh, float *cen);
int slfo_slic_assign(int W, int H, const uint8_t *rgb, int gw, int gh, const float *cen, double compactness,
                     int32_t *labels);
int slfo_slic_update(int W, int H, const uint8_t *rgb, int gw, int gh, const int32_t *labels, float *cen);
int slfo_slic_connectivity(int W, int H, int gw, int gh, int32_t *labels);
int slfo_slic(int W, int H, const uint8_t *rgb, int gw, int gh, int iterations, double compactness,
              int connectivity, int32_t *labels);

#ifdef __cplusplus
}
#endif
#endif
