// Host-side state of one rig (slf_ctx) and the helpers that the per-rig
// entry points (slf_api.hip) and the pool (slf_pool.hip) share.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "slf.h"
#include "slf_internal.h"

struct slf_pool;

namespace slf {

struct ViewHost {
  int W = 0, H = 0;
  double K[9], R[9], t[3], Kinv[9];
  int gw = 0, gh = 0;
  bool has_img = false, has_lab = false, has_planes = false;
  std::vector<int> nbrs;
};

template <typename T>
void dfree(T *&p) {
  if (p) (void)hipFree((void *)p);
  p = nullptr;
}

}  // namespace slf

struct slf_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  slf_params p;
  std::string err;
  std::vector<slf::ViewHost> vh;
  int V = 0;

  // per-pixel device buffers
  uint8_t *d_rgb = nullptr;
  int *d_labels = nullptr;
  uint16_t *d_lab16 = nullptr;  // the labels as 16 bits, for the refinement's gathers
  bool lab16_ok = false;        // every view has at most 65536 grid cells
  void *d_quads = nullptr;
  size_t quads_bytes = 0;
  int quads_fmt = -1;
  bool quads_dirty = true;
  int64_t total_px = 0;

  // geometry tables
  std::vector<slf::ViewDev> views_h;
  std::vector<slf::PairDev> pairs_h;
  slf::ViewDev *d_views = nullptr;
  slf::PairDev *d_pairs = nullptr;
  bool geom_dirty = true;

  // superpixel buffers
  int S = 0, S_cap = 0;
  bool sp_dirty = true;
  int *d_count = nullptr, *d_sp_view = nullptr, *d_area = nullptr, *d_px_off = nullptr, *d_scan = nullptr;
  int *d_err = nullptr;
  int4 *d_bbox = nullptr;
  float2 *d_centroid = nullptr;
  double2 *d_centroid_d = nullptr;
  int *d_order = nullptr;  // claim order of the per-superpixel launches (strip order, see strip_order)
  bool order_ok = false;   // d_order holds the order of the current grids
  std::vector<int> order_h;  // its host copy (the source of the upload, kept alive)
  float4 *d_colour = nullptr;
  slf::PixEntry *d_px = nullptr;
  float4 *d_planes[2] = {nullptr, nullptr};
  float4 *d_tab[2] = {nullptr, nullptr};  // per superpixel {colour, inverse-depth row}
  float *d_energy = nullptr, *d_margin = nullptr;
  int *d_choice = nullptr;
  // device work counters: [0] refinement evals, [1] refinement samples,
  // [2] refinement candidates pruned, [3] sweep samples computed, [4] sweep
  // levels scored over all pixels and views
  unsigned long long *d_work = nullptr;
  int *d_claims = nullptr;  // claim counters of the persistent sweep launch
  slf::RefineArgs *d_refine_args = nullptr;  // refinement launch arguments, written on the stream before each launch
  int n_cu = 0;             // compute units of the device
  float *d_depth_tmp = nullptr;
  int64_t depth_tmp_n = 0;
  // depth fusion (slf_fusion.hip), allocated on first use: candidate layers,
  // the device camera table (and its host copy), the depth maps read out of
  // the planes, the fused depth and the votes
  void *d_fz = nullptr, *d_fcams = nullptr, *d_fdepth = nullptr, *d_fused = nullptr, *d_fvotes = nullptr;
  int64_t fz_bytes = 0, fcams_bytes = 0, fdepth_bytes = 0, fused_bytes = 0, fvotes_bytes = 0;
  std::vector<unsigned char> fcams_h;
  bool has_fused = false;
  // GPU SLIC (slf_slic.hip), allocated on first use: centres, per-label best
  // component, and per-pixel working labels, union-find parents and sizes
  void *d_slic_cen = nullptr, *d_slic_best = nullptr, *d_slic_work = nullptr;
  int64_t slic_cen_bytes = 0, slic_best_bytes = 0, slic_work_bytes = 0;
  int cur = 0;
  std::vector<int> area_h;
  std::vector<double2> cen_h;   // centroids and colours: read back on first use after a rebuild
  std::vector<float4> col_h;
  bool stats_h_ok = false;
  uint64_t host_evals = 0;        // sweep hypotheses (levels x non-empty superpixels)
  uint64_t host_sweep_total = 0;  // sweep px-view samples without the level bound

  // Warm start: every view had planes when the superpixels were last rebuilt
  // for new images on the same cameras and grids.
  bool warm_ok = false;

  // pool membership
  slf_pool *pool = nullptr;
  uint64_t pool_bytes = 0;  // footprint accounted to the pool
  bool in_flight = false;   // a pool request has stages not yet launched

  int fail(int code, const char *fmt, ...) __attribute__((format(printf, 3, 4)));
};

#define HIP_OR_FAIL(ctx, call)                                                                          \
  do {                                                                                                  \
    hipError_t e_ = (call);                                                                             \
    if (e_ != hipSuccess)                                                                               \
      return (ctx)->fail(e_ == hipErrorOutOfMemory ? SLF_ENOMEM : SLF_EDEVICE, "%s: %s", #call,         \
                         hipGetErrorString(e_));                                                        \
  } while (0)

namespace slf {

// Geometry tables, image texels and superpixel lists, rebuilt when inputs
// changed (slf_api.hip).  Synchronises the rig's stream when it rebuilds.
int ensure_setup(slf_ctx *c);
// Device bytes the rig holds once set up: images, labels, texels, geometry,
// superpixel lists and plane state.  Needs cameras and label grids.
int footprint(const slf_ctx *c, uint64_t *bytes);
// Kernel arguments of a sweep / of refinement iteration `iter` on the rig's
// current state (planes[cur] -> planes[1 - cur]).
void sweep_args(const slf_ctx *c, SweepArgs &a);
void refine_args(const slf_ctx *c, int iter, RefineArgs &a);
// Bookkeeping after a sweep / an iteration was enqueued.
void after_sweep(slf_ctx *c);
void after_refine(slf_ctx *c);
// SLF_ESTATE when the rig has pool stages not yet launched.
int check_idle(slf_ctx *c);
// Takes the device address of the static fusion scratch on `device` (which
// must be current), once per device; SLF_OK, SLF_EDEVICE or SLF_EUNSUPPORTED.
int static_scratch_init(int device);

}  // namespace slf
