// Internal device-side layout shared by the kernels and the host layer of libslf.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "slf.h"

namespace slf {

constexpr int kWave = 64;
constexpr int kWavesPerBlock = 4;
constexpr int kBlock = kWave * kWavesPerBlock;
constexpr int kMaxNeighbors = 64;

// Device image storage formats (texel = the four bilinear taps of a pixel).
enum { SLF_FMT_U8 = SLF_IMAGE_U8, SLF_FMT_F16 = SLF_IMAGE_F16, SLF_FMT_F32 = SLF_IMAGE_F32 };

// Per-view geometry and buffer offsets, in device memory.
struct ViewDev {
  int W, H, gw, gh;
  int sp_off;          // first global superpixel index of this view
  int pair_off;        // first entry of this view's neighbour list in the pair table
  int n_pairs;         // |N(r)|
  int kr_init;         // initial propagation kernel radius, grid cells
  int64_t pix_off;     // first pixel of this view in per-pixel arrays (labels, rgb)
  int64_t quad_off;    // first texel of this view in the texel array ((W+1) x (H+1) texels)
  float Kinv[9];       // K^-1 rounded to FP32
  float pad1[3];
  double Kinv_d[9];    // K^-1 in FP64
  double pad2;
};

// Geometry of one (reference r, neighbour i) pair: for a plane with
// inverse-depth row g (1/D(p) = g . p~) in camera r, the plane-induced
// homography is H = A + b g^T with A = K_i R_ri K_r^-1 and b = K_i t_ri.
struct PairDev {
  float A[9];
  float b[3];
  int i;               // neighbour view
  int pad[3];
  double A_d[9];
  double b_d[3];
};

// Packed pixel-list entry: x = u | v << 16, y = RGBA8 of the pixel.
using PixEntry = uint2;

struct SweepArgs {
  const ViewDev *views;
  const PairDev *pairs;
  const int *sp_view;
  const int *order;     // claim c of the launch takes superpixel order[c] (nullptr: superpixel c)
  const int *area;
  const int *px_off;
  const PixEntry *px;
  const int4 *bbox;     // per superpixel pixel bounding box (x0, y0, x1, y1)
  const void *quads;
  uint32_t quad_bytes;  // bytes of texels over all views (< 4 GiB)
  int S;
  int levels;
  double qmin, dq;     // inverse-depth range start and bin width
  uint64_t seed;
  int jitter;
  float T255;          // truncation in squared 0..255 units
  int exact_margin;    // 1: levels stop against the second-best complete cost (exact margin), 0: the best
  const float4 *colour;  // mean colour per superpixel
  float4 *planes;      // out
  float4 *tab;         // out: per superpixel {colour, inverse-depth row (g0, g1, g2, 0)}
  float *cost;         // out
  int *choice;         // out
  float *margin;       // out
  unsigned long long *work;  // [3] += px-view samples computed (the level bound skips the rest),
                             // [4] += levels scored over all pixels and views
};

struct RefineArgs {
  const ViewDev *views;
  const PairDev *pairs;
  const int *sp_view;
  const int *order;     // claim c of the launch takes superpixel order[c] (nullptr: superpixel c)
  const int *area;
  const int *px_off;
  const PixEntry *px;
  const double2 *centroid_d;  // centroids in FP64
  const float4 *colour;   // mean colour in [0,1]
  const int *labels;      // all views
  const uint16_t *lab16;  // the same labels as 16 bits, or null when a view has more than 65536 cells
  const void *quads;      // images (data-only energy mode)
  uint32_t quad_bytes;    // bytes of texels over all views (< 4 GiB)
  const float4 *planesA;  // state read
  const float4 *tabA;     // per superpixel {colour, inverse-depth row} of state A
  float4 *planesB;        // state written
  float4 *tabB;
  float *energy;
  int *choice;
  float *margin;
  unsigned long long *work;  // [0] evals, [1] samples, [2] candidates pruned
  int S;
  int iter;
  int kernel_step;
  int energy_mode;
  int exact_margin;  // 1: candidates stop against the second-best energy (exact margin), 0: the best
  unsigned term_mask;
  float inv2sig2, inv2alpha2, eta, occ_tol, T255;
  float inv2sig2_log2e, inv2alpha2_log2e;  // the same scales times log2(e), for exp2
};

// One rig's work in a pooled persistent launch: a sweep or one refinement
// iteration over the rig's superpixels, cut into items of `tile` superpixels.
enum { SLF_OP_SWEEP = 0, SLF_OP_REFINE = 1 };
struct PoolJob {
  int item_begin;  // first work item of this job within the stage
  int S;           // superpixels of the rig
  int split;       // sweep stages: level parts per superpixel (items = tiles x split)
  int sp_begin;    // first superpixel of this job in the stage's superpixel order
  int64_t part_base;  // sweep stages with split > 1: first part record of this job
  SweepArgs sweep;     // used by sweep stages
  RefineArgs refine;   // used by refinement stages
};
constexpr int kPoolQueues = 8;      // one per XCD
constexpr int kPoolMaxJobs = 64;    // rigs in one stage
constexpr int kWorkCounters = 5;      // per-context device work counters (slf_ctx::d_work)
constexpr int kPoolCounterStride = 16;  // ints between claim counters (one 64-byte line each)
// A stage: every job runs the same op in the same image format.  Items
// [qbegin[q], qend[q]) form queue q; the waves of XCD q drain it first.
// Read-only while the stage runs; the claim counters live elsewhere.
struct PoolStage {
  int njobs, tile, total_sp, pad;
  float4 *parts;   // per (superpixel, part) {best, second, level} of split sweeps
  int qbegin[kPoolQueues], qend[kPoolQueues];
  PoolJob jobs[kPoolMaxJobs];
};

// Host-side launchers (slf_kernels.hip).
hipError_t launch_quads(int fmt, const uint8_t *rgb, int64_t rgb_stride, int W, int H, void *quads,
                        int64_t quad_off, hipStream_t st);
hipError_t launch_sp_build(const ViewDev *views_d, const ViewDev *views_h, int V, const int *labels, uint16_t *lab16,
                           const uint8_t *rgb, int S, int *count, int4 *bbox, int *px_off, int *scan_tmp,
                           PixEntry *px, int *area, float2 *centroid, double2 *centroid_d, float4 *colour,
                           int *sp_view, int *err, hipStream_t st);
// Persistent sweep launch; counters: kPoolQueues x kPoolCounterStride ints of claim counters.
hipError_t launch_sweep(int fmt, const SweepArgs &a, int *counters, int n_cu, hipStream_t st);
// `slot`: device memory for the refinement's arguments (written on the stream
// before the kernel, which reads them from there).
hipError_t launch_refine(int fmt, const RefineArgs &a, RefineArgs *slot, int *counters, int n_cu, hipStream_t st);
hipError_t launch_depth(const ViewDev *views_d, const ViewDev &vh, int view, const int *labels,
                        const float4 *tab, float *out, int64_t stride, hipStream_t st);
size_t quad_bytes(int fmt);
hipError_t launch_warm(const ViewDev *views, const int *sp_view, const int *area, const double2 *cen,
                       const float4 *colour, float4 *planes, float4 *tab, int S, double d_fb, hipStream_t st);
// One pooled stage: a kernel that clears the stage's claim counters, then
// the persistent kernel over `blocks` workgroups, then (sweeps split into
// level parts) the kernel merging the parts.
hipError_t launch_pool(int op, int fmt, int kc, bool merge, const PoolStage *stage, int *counters, int blocks,
                       hipStream_t st);
// Workgroups of the pooled kernel resident per compute unit.
int pool_occupancy(int op, int fmt, int kc);

}  // namespace slf
