// Host layer of libslf: the C ABI declared in include/slf.h.  Validates
// arguments, owns device buffers, composes per-view-pair geometry in FP64 and
// enqueues the kernels of slf_kernels.hip on the context's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "slf.h"
#include "slf_ctx.h"
#include "slf_internal.h"

using namespace slf;

namespace {

void inv3(const double *m, double *o) {
  const double a = m[0], b = m[1], c = m[2], d = m[3], e = m[4], f = m[5], g = m[6], h = m[7], i = m[8];
  const double c00 = e * i - f * h, c01 = f * g - d * i, c02 = d * h - e * g;
  const double det = a * c00 + b * c01 + c * c02;
  o[0] = c00 / det;
  o[1] = (c * h - b * i) / det;
  o[2] = (b * f - c * e) / det;
  o[3] = c01 / det;
  o[4] = (a * i - c * g) / det;
  o[5] = (c * d - a * f) / det;
  o[6] = c02 / det;
  o[7] = (b * g - a * h) / det;
  o[8] = (a * e - b * d) / det;
}

void mul3(const double *a, const double *b, double *o) {
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) o[3 * r + c] = a[3 * r] * b[c] + a[3 * r + 1] * b[3 + c] + a[3 * r + 2] * b[6 + c];
}

bool finite_all(const double *x, int n) {
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(x[i])) return false;
  return true;
}

}  // namespace

int slf_ctx::fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  err = buf;
  return code;
}

namespace {

int params_check(slf_ctx *c, const slf_params *p) {
  if (!p) return c->fail(SLF_EINVAL, "params is NULL");
  if (p->struct_size != sizeof(slf_params))
    return c->fail(SLF_EINVAL, "struct_size %u != %zu", p->struct_size, sizeof(slf_params));
  if (p->levels < 1 || p->levels > (1 << 20)) return c->fail(SLF_EINVAL, "levels %d out of [1, 2^20]", p->levels);
  if (!(p->d_min > 0) || !(p->d_max > p->d_min) || !std::isfinite(p->d_max))
    return c->fail(SLF_EINVAL, "need 0 < d_min < d_max < inf");
  if (!(p->tssd_T > 0) || !std::isfinite(p->tssd_T)) return c->fail(SLF_EINVAL, "tssd_T must be > 0");
  if (!(p->sigma > 0) || !std::isfinite(p->sigma)) return c->fail(SLF_EINVAL, "sigma must be > 0");
  if (!(p->alpha > 0) || !std::isfinite(p->alpha)) return c->fail(SLF_EINVAL, "alpha must be > 0");
  if (!(p->eta >= 0) || !std::isfinite(p->eta)) return c->fail(SLF_EINVAL, "eta must be >= 0");
  if (!(p->occ_tol >= 0) || !std::isfinite(p->occ_tol)) return c->fail(SLF_EINVAL, "occ_tol must be >= 0");
  if (p->kernel_step < 1) return c->fail(SLF_EINVAL, "kernel_step must be >= 1");
  if (p->term_mask > 7u) return c->fail(SLF_EINVAL, "term_mask must be in [0, 7]");
  if (p->image_precision < 0 || p->image_precision > 2) return c->fail(SLF_EINVAL, "bad image_precision");
  if (p->energy_mode < 0 || p->energy_mode > 1) return c->fail(SLF_EINVAL, "bad energy_mode");
  if (p->exact_margin < 0 || p->exact_margin > 1) return c->fail(SLF_EINVAL, "bad exact_margin");
  if (p->homography_fp64 != 1) return c->fail(SLF_EUNSUPPORTED, "homography_fp64 must be 1");
  return SLF_OK;
}

int ensure_alloc(slf_ctx *c, size_t bytes, void **ptr) {
  hipError_t e = hipMalloc(ptr, bytes ? bytes : 16);
  if (e != hipSuccess) {
    *ptr = nullptr;
    return c->fail(SLF_ENOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
  }
  return SLF_OK;
}

void free_sp(slf_ctx *c) {
  dfree(c->d_count);
  dfree(c->d_order);
  c->order_ok = false;
  dfree(c->d_sp_view);
  dfree(c->d_area);
  dfree(c->d_px_off);
  dfree(c->d_scan);
  dfree(c->d_bbox);
  dfree(c->d_centroid);
  dfree(c->d_centroid_d);
  dfree(c->d_colour);
  dfree(c->d_px);
  for (int j = 0; j < 2; ++j) {
    dfree(c->d_planes[j]);
    dfree(c->d_tab[j]);
  }
  dfree(c->d_energy);
  dfree(c->d_margin);
  dfree(c->d_choice);
  c->S_cap = 0;
}

void free_all(slf_ctx *c) {
  free_sp(c);
  dfree(c->d_rgb);
  dfree(c->d_labels);
  dfree(c->d_lab16);
  if (c->d_quads) (void)hipFree(c->d_quads);
  c->d_quads = nullptr;
  c->quads_bytes = 0;
  dfree(c->d_views);
  dfree(c->d_pairs);
  dfree(c->d_err);
  dfree(c->d_work);
  dfree(c->d_claims);
  dfree(c->d_refine_args);
  dfree(c->d_depth_tmp);
  for (void **f : {&c->d_fz, &c->d_fcams, &c->d_fdepth, &c->d_fused, &c->d_fvotes, &c->d_slic_cen, &c->d_slic_best,
                   &c->d_slic_work})
    dfree(*f);
  c->slic_cen_bytes = c->slic_best_bytes = c->slic_work_bytes = 0;
  c->fz_bytes = c->fcams_bytes = c->fdepth_bytes = c->fused_bytes = c->fvotes_bytes = 0;
  c->fcams_h.clear();
  c->has_fused = false;
}

bool views_ready(const slf_ctx *c) {
  if (c->V < 2) return false;
  for (const auto &v : c->vh)
    if (!v.has_img || !v.has_lab) return false;
  return true;
}

// Per-view and per-pair geometry, composed in FP64 and rounded once.
int build_geometry(slf_ctx *c) {
  const int V = c->V;
  c->order_ok = false;  // the claim order follows the grids
  c->views_h.assign(V, ViewDev{});
  c->pairs_h.clear();
  int sp = 0;
  int64_t px = 0, qd = 0;
  for (int v = 0; v < V; ++v) {
    const ViewHost &h = c->vh[v];
    ViewDev &d = c->views_h[v];
    d.W = h.W;
    d.H = h.H;
    d.gw = h.gw;
    d.gh = h.gh;
    d.sp_off = sp;
    d.pix_off = px;
    d.quad_off = qd;
    d.pair_off = (int)c->pairs_h.size();
    d.n_pairs = (int)h.nbrs.size();
    if (c->p.kernel_radius_init > 0) {
      d.kr_init = c->p.kernel_radius_init;
    } else {
      const double S = std::sqrt((double)h.W * h.H / ((double)h.gw * h.gh));
      d.kr_init = (int)std::floor(std::min(h.W, h.H) / (2.0 * S));
    }
    for (int j = 0; j < 9; ++j) {
      d.Kinv[j] = (float)h.Kinv[j];
      d.Kinv_d[j] = h.Kinv[j];
    }
    const int64_t K = (int64_t)h.gw * h.gh;
    if ((int64_t)sp + K > (int64_t)1 << 30) return c->fail(SLF_EUNSUPPORTED, "too many superpixels");
    sp += (int)K;
    px += (int64_t)h.W * h.H;
    qd += (int64_t)(h.W + 1) * (h.H + 1);
    // pairs: A = K_i R_ri K_r^-1, b = K_i t_ri, R_ri = R_i R_r^T, t_ri = t_i - R_ri t_r
    // N(r) in decreasing distance between camera centres (stable): the
    // widest baselines separate depth hypotheses most, so the exact bounds
    // of the sweep (over level chunks) and of the refinement (over views)
    // stop earlier; the order changes only the rounding of per-view sums
    // (full-HD sweep 20.3 -> 19.5 ms, refinement 27.1 -> 26.7 ms)
    std::vector<int> order = h.nbrs;
    {
      auto centre = [&](const ViewHost &q, double *C) {
        for (int a = 0; a < 3; ++a) C[a] = -(q.R[a] * q.t[0] + q.R[3 + a] * q.t[1] + q.R[6 + a] * q.t[2]);
      };
      double Cr[3];
      centre(h, Cr);
      std::vector<double> dist(c->V, 0.0);
      for (int i : order) {
        double Ci[3];
        centre(c->vh[i], Ci);
        dist[i] = (Ci[0] - Cr[0]) * (Ci[0] - Cr[0]) + (Ci[1] - Cr[1]) * (Ci[1] - Cr[1]) + (Ci[2] - Cr[2]) * (Ci[2] - Cr[2]);
      }
      std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return dist[x] > dist[y]; });
    }
    for (int i : order) {
      const ViewHost &hi = c->vh[i];
      double RrT[9], Rri[9], tri[3], T1[9], A[9];
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) RrT[3 * a + b] = h.R[3 * b + a];
      mul3(hi.R, RrT, Rri);
      for (int a = 0; a < 3; ++a)
        tri[a] = hi.t[a] - (Rri[3 * a] * h.t[0] + Rri[3 * a + 1] * h.t[1] + Rri[3 * a + 2] * h.t[2]);
      mul3(hi.K, Rri, T1);
      mul3(T1, h.Kinv, A);
      PairDev pd{};
      for (int j = 0; j < 9; ++j) {
        pd.A[j] = (float)A[j];
        pd.A_d[j] = A[j];
      }
      for (int a = 0; a < 3; ++a) {
        const double bb = hi.K[3 * a] * tri[0] + hi.K[3 * a + 1] * tri[1] + hi.K[3 * a + 2] * tri[2];
        pd.b[a] = (float)bb;
        pd.b_d[a] = bb;
      }
      pd.i = i;
      c->pairs_h.push_back(pd);
    }
  }
  c->S = sp;
  c->total_px = px;
  dfree(c->d_views);
  dfree(c->d_pairs);
  int rc;
  if ((rc = ensure_alloc(c, sizeof(ViewDev) * V, (void **)&c->d_views))) return rc;
  if ((rc = ensure_alloc(c, sizeof(PairDev) * std::max<size_t>(1, c->pairs_h.size()), (void **)&c->d_pairs)))
    return rc;
  HIP_OR_FAIL(c, hipMemcpyAsync(c->d_views, c->views_h.data(), sizeof(ViewDev) * V, hipMemcpyHostToDevice,
                                c->stream));
  HIP_OR_FAIL(c, hipMemcpyAsync(c->d_pairs, c->pairs_h.data(), sizeof(PairDev) * c->pairs_h.size(),
                                hipMemcpyHostToDevice, c->stream));
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  c->geom_dirty = false;
  return SLF_OK;
}

// The order in which the per-superpixel launches claim superpixels: strips
// of kStripCellRows grid rows, each strip over every view (raster order
// within a view), strips top to bottom.  The claim queues cut this order into
// one contiguous range per XCD, so an XCD works through a band of rows of
// every view at once: what its superpixels read in the other views (their
// texels for the sweep, their labels and plane records for the refinement)
// lies in the same rows, shared by the reference views of the strip instead
// of streamed once per view through that XCD's L2.  Superpixels are
// independent within a launch, so the order changes no result.
#ifndef SLF_STRIP_ROWS
#define SLF_STRIP_ROWS 2
#endif
constexpr int kStripCellRows = SLF_STRIP_ROWS;
std::vector<int> strip_order(const slf_ctx *c) {
  std::vector<std::pair<int64_t, int>> key;
  key.reserve(c->S);
  for (int v = 0; v < c->V; ++v) {
    const ViewDev &d = c->views_h[v];
    for (int s = 0; s < d.gw * d.gh; ++s) {
      const int strip = (s / d.gw) / kStripCellRows;
      key.emplace_back(((int64_t)strip * c->V + v) * (int64_t)(1 << 24) + s, d.sp_off + s);
    }
  }
  std::sort(key.begin(), key.end());
  std::vector<int> order(key.size());
  for (size_t i = 0; i < key.size(); ++i) order[i] = key[i].second;
  return order;
}

// Superpixel buffers for c->S superpixels; *kept is set when the existing
// buffers (and the plane state in them) were large enough to stay.
int alloc_sp(slf_ctx *c, bool *kept) {
  *kept = c->S <= c->S_cap && c->d_px;
  if (*kept) return SLF_OK;
  free_sp(c);
  const size_t S = (size_t)c->S;
  const size_t nb = (S + 4095) / 4096 + 1;
  int rc;
  if ((rc = ensure_alloc(c, sizeof(int) * S, (void **)&c->d_count))) return rc;
  if ((rc = ensure_alloc(c, sizeof(int) * S, (void **)&c->d_sp_view))) return rc;
  if ((rc = ensure_alloc(c, sizeof(int) * S, (void **)&c->d_order))) return rc;
  if ((rc = ensure_alloc(c, sizeof(int) * S, (void **)&c->d_area))) return rc;
  if ((rc = ensure_alloc(c, sizeof(int) * (S + 1), (void **)&c->d_px_off))) return rc;
  if ((rc = ensure_alloc(c, sizeof(int) * nb, (void **)&c->d_scan))) return rc;
  if ((rc = ensure_alloc(c, sizeof(int4) * S, (void **)&c->d_bbox))) return rc;
  if ((rc = ensure_alloc(c, sizeof(float2) * S, (void **)&c->d_centroid))) return rc;
  if ((rc = ensure_alloc(c, sizeof(double2) * S, (void **)&c->d_centroid_d))) return rc;
  if ((rc = ensure_alloc(c, sizeof(float4) * S, (void **)&c->d_colour))) return rc;
  if ((rc = ensure_alloc(c, sizeof(PixEntry) * (size_t)c->total_px, (void **)&c->d_px))) return rc;
  for (int j = 0; j < 2; ++j) {
    if ((rc = ensure_alloc(c, sizeof(float4) * S, (void **)&c->d_planes[j]))) return rc;
    if ((rc = ensure_alloc(c, 2 * sizeof(float4) * S, (void **)&c->d_tab[j]))) return rc;
  }
  if ((rc = ensure_alloc(c, sizeof(float) * S, (void **)&c->d_energy))) return rc;
  if ((rc = ensure_alloc(c, sizeof(float) * S, (void **)&c->d_margin))) return rc;
  if ((rc = ensure_alloc(c, sizeof(int) * S, (void **)&c->d_choice))) return rc;
  c->S_cap = c->S;
  return SLF_OK;
}

}  // namespace

// Geometry tables, image texels and superpixel lists, rebuilt when inputs changed.
int slf::ensure_setup(slf_ctx *c) {
  if (!views_ready(c)) return c->fail(SLF_ESTATE, "cameras, images and labels must be set for every view");
  int rc;
  bool same_cells = true;  // every view keeps its grid cells (and so its plane state)
  if (c->geom_dirty) {
    const int old_S = c->S;
    if ((rc = build_geometry(c))) return rc;
    if (c->S != old_S) {
      c->sp_dirty = true;
      same_cells = false;
    }
  }
  const int fmt = c->p.image_precision;
  if (c->quads_dirty || c->quads_fmt != fmt) {
    int64_t texels = 0;
    for (const auto &v : c->vh) texels += (int64_t)(v.W + 1) * (v.H + 1);
    const size_t need = (size_t)texels * quad_bytes(fmt);
    // one 32-bit buffer resource covers every view's texels
    if (need > 0xFFFFFFF0ull)
      return c->fail(SLF_EUNSUPPORTED,
                     "texel storage of %zu bytes exceeds 4 GiB (8 bytes per pixel for RGBA8 and FP16, 16 for FP32)",
                     need);
    if (need > c->quads_bytes) {
      if (c->d_quads) (void)hipFree(c->d_quads);
      c->d_quads = nullptr;
      c->quads_bytes = 0;
      if ((rc = ensure_alloc(c, need, &c->d_quads))) return rc;
      c->quads_bytes = need;
    }
    for (int v = 0; v < c->V; ++v) {
      const ViewDev &d = c->views_h[v];
      HIP_OR_FAIL(c, launch_quads(fmt, c->d_rgb + 3 * d.pix_off, 3 * (int64_t)d.W, d.W, d.H, c->d_quads, d.quad_off,
                                  c->stream));
    }
    c->quads_fmt = fmt;
    c->quads_dirty = false;
  }
  if (c->sp_dirty) {
    bool kept = false;
    if ((rc = alloc_sp(c, &kept))) return rc;
    bool all_planes = true;
    for (const auto &v : c->vh) all_planes = all_planes && v.has_planes;
    c->warm_ok = kept && same_cells && all_planes;
    c->lab16_ok = true;
    for (const auto &v : c->vh) c->lab16_ok = c->lab16_ok && (int64_t)v.gw * v.gh <= 65536;
    if (!c->order_ok) {  // depends on the grids only, not on the labels: built once per geometry
      c->order_h = strip_order(c);
      HIP_OR_FAIL(c, hipMemcpyAsync(c->d_order, c->order_h.data(), sizeof(int) * c->order_h.size(),
                                    hipMemcpyHostToDevice, c->stream));
      c->order_ok = true;
    }
    HIP_OR_FAIL(c, launch_sp_build(c->d_views, c->views_h.data(), c->V, c->d_labels,
                                   c->lab16_ok ? c->d_lab16 : nullptr, c->d_rgb, c->S, c->d_count,
                                   c->d_bbox, c->d_px_off, c->d_scan, c->d_px, c->d_area, c->d_centroid,
                                   c->d_centroid_d, c->d_colour, c->d_sp_view, c->d_err, c->stream));
    int herr = 0;
    HIP_OR_FAIL(c, hipMemcpyAsync(&herr, c->d_err, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    c->area_h.resize(c->S);
    HIP_OR_FAIL(c, hipMemcpyAsync(c->area_h.data(), c->d_area, sizeof(int) * c->S, hipMemcpyDeviceToHost, c->stream));
    c->stats_h_ok = false;  // centroids and colours are read back when a host call needs them
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    for (auto &v : c->vh) v.has_planes = false;
    if (herr & 1) {
      c->warm_ok = false;
      return c->fail(SLF_EINVAL, "a label is outside [0, grid_w * grid_h)");
    }
    if (herr) return c->fail(SLF_EDEVICE, "superpixel list build inconsistent (flag %d)", herr);
    c->sp_dirty = false;
  }
  return SLF_OK;
}

int slf::footprint(const slf_ctx *c, uint64_t *bytes) {
  if (c->V < 2) return SLF_ESTATE;
  uint64_t px = 0, S = 0, pairs = 0, max_px = 0, texels = 0;
  for (const auto &v : c->vh) {
    if (v.gw < 1 || v.gh < 1) return SLF_ESTATE;
    px += (uint64_t)v.W * v.H;
    texels += (uint64_t)(v.W + 1) * (v.H + 1);
    max_px = std::max<uint64_t>(max_px, (uint64_t)v.W * v.H);
    S += (uint64_t)v.gw * v.gh;
    pairs += v.nbrs.size();
  }
  uint64_t b = 0;
  b += px * (3 + sizeof(int) + sizeof(uint16_t));                 // images, labels (32 and 16 bits)
  b += texels * quad_bytes(c->p.image_precision);                 // bilinear texels
  b += sizeof(ViewDev) * c->V + sizeof(PairDev) * pairs + 64;     // geometry, flags, counters
  b += S * (4 * sizeof(int) + sizeof(int4) + sizeof(float2) + sizeof(double2) + sizeof(float4));
  b += sizeof(int) * ((S + 4095) / 4096 + 2);                     // scan blocks, offsets
  b += px * sizeof(PixEntry);                                     // pixel lists
  b += S * 2 * (sizeof(float4) + 2 * sizeof(float4));             // plane state, ping-pong
  b += S * (2 * sizeof(float) + sizeof(int));                     // energy, margin, choice
  b += max_px * sizeof(float);                                    // host depth readout staging
  *bytes = b;
  return SLF_OK;
}

void slf::sweep_args(const slf_ctx *c, SweepArgs &a) {
  a = SweepArgs{};
  a.views = c->d_views;
  a.pairs = c->d_pairs;
  a.sp_view = c->d_sp_view;
  a.order = c->d_order;
  a.area = c->d_area;
  a.px_off = c->d_px_off;
  a.px = c->d_px;
  a.bbox = c->d_bbox;
  a.quads = c->d_quads;
  a.quad_bytes = (uint32_t)c->quads_bytes;
  a.S = c->S;
  a.levels = c->p.levels;
  a.qmin = 1.0 / c->p.d_max;
  a.dq = (1.0 / c->p.d_min - 1.0 / c->p.d_max) / c->p.levels;
  a.seed = c->p.seed;
  a.jitter = c->p.jitter;
  a.T255 = c->p.tssd_T * 255.f * 255.f;
  a.exact_margin = c->p.exact_margin;
  a.planes = c->d_planes[c->cur];
  a.colour = c->d_colour;
  a.tab = c->d_tab[c->cur];
  a.cost = c->d_energy;
  a.choice = c->d_choice;
  a.margin = c->d_margin;
  a.work = c->d_work;
}

// Host copies of the superpixel centroids and colours (set_planes and
// get_superpixels use them); read back once per superpixel rebuild.
static int fetch_stats(slf_ctx *c) {
  if (c->stats_h_ok) return SLF_OK;
  c->cen_h.resize(c->S);
  c->col_h.resize(c->S);
  HIP_OR_FAIL(c, hipMemcpyAsync(c->col_h.data(), c->d_colour, sizeof(float4) * c->S, hipMemcpyDeviceToHost,
                                c->stream));
  HIP_OR_FAIL(c, hipMemcpyAsync(c->cen_h.data(), c->d_centroid_d, sizeof(double2) * c->S, hipMemcpyDeviceToHost,
                                c->stream));
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  c->stats_h_ok = true;
  return SLF_OK;
}

void slf::after_sweep(slf_ctx *c) {
  for (int v = 0; v < c->V; ++v) {
    const ViewDev &d = c->views_h[v];
    uint64_t nonempty = 0, px = 0;
    for (int s = 0; s < d.gw * d.gh; ++s) {
      const int A = c->area_h[d.sp_off + s];
      nonempty += A > 0;
      px += (uint64_t)A;
    }
    c->host_evals += nonempty * (uint64_t)c->p.levels;
    c->host_sweep_total += px * (uint64_t)d.n_pairs * (uint64_t)c->p.levels;
    c->vh[v].has_planes = true;
  }
}

void slf::refine_args(const slf_ctx *c, int iter, RefineArgs &a) {
  a = RefineArgs{};
  a.views = c->d_views;
  a.pairs = c->d_pairs;
  a.sp_view = c->d_sp_view;
  a.order = c->d_order;
  a.area = c->d_area;
  a.px_off = c->d_px_off;
  a.px = c->d_px;
  a.centroid_d = c->d_centroid_d;
  a.colour = c->d_colour;
  a.labels = c->d_labels;
  a.lab16 = c->lab16_ok ? c->d_lab16 : nullptr;
  a.quads = c->d_quads;
  a.quad_bytes = (uint32_t)c->quads_bytes;
  a.energy = c->d_energy;
  a.choice = c->d_choice;
  a.margin = c->d_margin;
  a.work = c->d_work;
  a.S = c->S;
  a.kernel_step = c->p.kernel_step;
  a.energy_mode = c->p.energy_mode;
  a.exact_margin = c->p.exact_margin;
  a.term_mask = c->p.term_mask;
  a.inv2sig2 = 1.f / (2.f * c->p.sigma * c->p.sigma);
  a.inv2alpha2 = 1.f / (2.f * c->p.alpha * c->p.alpha);
  a.inv2sig2_log2e = (float)(1.4426950408889634 / (2.0 * (double)c->p.sigma * (double)c->p.sigma));
  a.inv2alpha2_log2e = (float)(1.4426950408889634 / (2.0 * (double)c->p.alpha * (double)c->p.alpha));
  a.eta = c->p.eta;
  a.occ_tol = c->p.occ_tol;
  a.T255 = c->p.tssd_T * 255.f * 255.f;
  a.iter = iter;
  a.planesA = c->d_planes[c->cur];
  a.tabA = c->d_tab[c->cur];
  a.planesB = c->d_planes[1 - c->cur];
  a.tabB = c->d_tab[1 - c->cur];
}

void slf::after_refine(slf_ctx *c) { c->cur = 1 - c->cur; }

int slf::check_idle(slf_ctx *c) {
  if (c->in_flight) return c->fail(SLF_ESTATE, "the rig has pool work not yet launched");
  return SLF_OK;
}

// ===================================================================== C ABI

extern "C" {

void slf_default_params(slf_params *p) {
  if (!p) return;
  std::memset(p, 0, sizeof *p);
  p->struct_size = sizeof(slf_params);
  p->levels = 64;
  p->d_min = 2.0;
  p->d_max = 8.0;
  p->seed = 0x5EED;
  p->jitter = 1;
  p->tssd_T = 0.04f;
  p->sigma = 0.05f;
  p->alpha = 0.1f;
  p->eta = 0.5f;
  p->occ_tol = 1e-3f;
  p->kernel_step = 5;
  p->kernel_radius_init = 0;
  p->term_mask = 7u;
  p->image_precision = SLF_IMAGE_U8;
  p->homography_fp64 = 1;
  p->energy_mode = 0;
  p->exact_margin = 0;
}

const char *slf_status_string(int s) {
  switch (s) {
    case SLF_OK: return "SLF_OK";
    case SLF_EINVAL: return "SLF_EINVAL: invalid argument";
    case SLF_ESTATE: return "SLF_ESTATE: call out of order";
    case SLF_ENOMEM: return "SLF_ENOMEM: out of memory";
    case SLF_EDEVICE: return "SLF_EDEVICE: HIP runtime error";
    case SLF_EUNSUPPORTED: return "SLF_EUNSUPPORTED: not supported";
    default: return "unknown status";
  }
}

const char *slf_last_error(const slf_ctx *ctx) { return ctx ? ctx->err.c_str() : "context is NULL"; }

int slf_create(int device_ordinal, slf_ctx **out) {
  if (!out) return SLF_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n == 0) return SLF_EDEVICE;
  if (device_ordinal < 0 || device_ordinal >= n) return SLF_EINVAL;
  slf_ctx *c = new (std::nothrow) slf_ctx();
  if (!c) return SLF_ENOMEM;
  c->device = device_ordinal;
  slf_default_params(&c->p);
  if (hipSetDevice(device_ordinal) != hipSuccess) {
    delete c;
    return SLF_EDEVICE;
  }
  if (hipMalloc((void **)&c->d_err, sizeof(int)) != hipSuccess ||
      hipMalloc((void **)&c->d_work, kWorkCounters * sizeof(unsigned long long)) != hipSuccess ||
      hipMemset(c->d_work, 0, kWorkCounters * sizeof(unsigned long long)) != hipSuccess ||
      hipMalloc((void **)&c->d_claims, kPoolQueues * kPoolCounterStride * sizeof(int)) != hipSuccess ||
      hipMalloc((void **)&c->d_refine_args, sizeof(RefineArgs)) != hipSuccess) {
    free_all(c);
    delete c;
    return SLF_ENOMEM;
  }
  if (hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, device_ordinal) != hipSuccess ||
      c->n_cu < 1 || static_scratch_init(device_ordinal) != SLF_OK) {
    free_all(c);
    delete c;
    return SLF_EDEVICE;
  }
  *out = c;
  return SLF_OK;
}

int slf_destroy(slf_ctx *c) {
  if (!c) return SLF_EINVAL;
  if (c->pool) return c->fail(SLF_ESTATE, "detach the rig from its pool first");
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  free_all(c);
  delete c;
  return SLF_OK;
}

int slf_set_stream(slf_ctx *c, void *stream) {
  if (!c) return SLF_EINVAL;
  if (int rc = check_idle(c)) return rc;
  // the refinement's argument slot is rewritten on the new stream: let the old one finish with it
  HIP_OR_FAIL(c, hipSetDevice(c->device));
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  c->stream = (hipStream_t)stream;
  return SLF_OK;
}

int slf_set_params(slf_ctx *c, const slf_params *p) {
  if (!c) return SLF_EINVAL;
  if (int rc = check_idle(c)) return rc;
  int rc = params_check(c, p);
  if (rc) return rc;
  const bool radius_changed = p->kernel_radius_init != c->p.kernel_radius_init;
  c->p = *p;
  if (radius_changed) c->geom_dirty = true;
  return SLF_OK;
}

int slf_set_cameras(slf_ctx *c, int n_views, const int32_t *wh, const double *K, const double *R, const double *t) {
  if (!c) return SLF_EINVAL;
  if (int rc = check_idle(c)) return rc;
  if (n_views < 2 || n_views > 4096) return c->fail(SLF_EINVAL, "n_views %d out of [2, 4096]", n_views);
  if (!wh || !K || !R || !t) return c->fail(SLF_EINVAL, "NULL camera array");
  std::vector<ViewHost> vh(n_views);
  int64_t total = 0;
  for (int v = 0; v < n_views; ++v) {
    ViewHost &h = vh[v];
    h.W = wh[2 * v];
    h.H = wh[2 * v + 1];
    if (h.W < 2 || h.H < 2) return c->fail(SLF_EINVAL, "view %d: W, H must be >= 2", v);
    if (h.W > 65535 || h.H > 65535) return c->fail(SLF_EUNSUPPORTED, "view %d: W, H must be <= 65535", v);
    std::memcpy(h.K, K + 9 * v, sizeof h.K);
    std::memcpy(h.R, R + 9 * v, sizeof h.R);
    std::memcpy(h.t, t + 3 * v, sizeof h.t);
    if (!finite_all(h.K, 9) || !finite_all(h.R, 9) || !finite_all(h.t, 3))
      return c->fail(SLF_EINVAL, "view %d: non-finite camera", v);
    if (h.K[6] != 0.0 || h.K[7] != 0.0 || h.K[8] != 1.0) return c->fail(SLF_EINVAL, "view %d: K's last row must be (0,0,1)", v);
    const double det = h.K[0] * (h.K[4] * h.K[8] - h.K[5] * h.K[7]) - h.K[1] * (h.K[3] * h.K[8] - h.K[5] * h.K[6]) +
                       h.K[2] * (h.K[3] * h.K[7] - h.K[4] * h.K[6]);
    if (!(std::fabs(det) > 0.0)) return c->fail(SLF_EINVAL, "view %d: K is singular", v);
    double RRt[9], Rt[9];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) Rt[3 * a + b] = h.R[3 * b + a];
    mul3(h.R, Rt, RRt);
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b)
        if (std::fabs(RRt[3 * a + b] - (a == b ? 1.0 : 0.0)) > 1e-6)
          return c->fail(SLF_EINVAL, "view %d: R is not orthonormal", v);
    const double detR = h.R[0] * (h.R[4] * h.R[8] - h.R[5] * h.R[7]) - h.R[1] * (h.R[3] * h.R[8] - h.R[5] * h.R[6]) +
                        h.R[2] * (h.R[3] * h.R[7] - h.R[4] * h.R[6]);
    if (!(detR > 0.0)) return c->fail(SLF_EINVAL, "view %d: R is not a rotation", v);
    inv3(h.K, h.Kinv);
    total += (int64_t)h.W * h.H;
    for (int i = 0; i < n_views; ++i)
      if (i != v) h.nbrs.push_back(i);
  }
  if (total >= ((int64_t)1 << 31)) return c->fail(SLF_EUNSUPPORTED, "more than 2^31 pixels in total");
  HIP_OR_FAIL(c, hipSetDevice(c->device));
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  free_sp(c);
  dfree(c->d_rgb);
  dfree(c->d_labels);
  dfree(c->d_lab16);
  if (c->d_quads) (void)hipFree(c->d_quads);
  c->d_quads = nullptr;
  c->quads_bytes = 0;
  c->vh = vh;
  c->V = n_views;
  c->total_px = total;
  int rc;
  if ((rc = ensure_alloc(c, (size_t)total * 3, (void **)&c->d_rgb))) return rc;
  if ((rc = ensure_alloc(c, (size_t)total * sizeof(int), (void **)&c->d_labels))) return rc;
  if ((rc = ensure_alloc(c, (size_t)total * sizeof(uint16_t), (void **)&c->d_lab16))) return rc;
  c->geom_dirty = true;
  c->sp_dirty = true;
  c->quads_dirty = true;
  c->S = 0;
  c->has_fused = false;
  return SLF_OK;
}

int slf_set_neighbors(slf_ctx *c, int view, int n, const int32_t *views) {
  if (!c) return SLF_EINVAL;
  if (int rc = check_idle(c)) return rc;
  if (view < 0 || view >= c->V) return c->fail(SLF_EINVAL, "view %d out of range", view);
  if (n < 1 || n > c->V - 1 || !views) return c->fail(SLF_EINVAL, "need 1 <= n <= n_views - 1 neighbour views");
  std::vector<int> nb(views, views + n);
  for (int j = 0; j < n; ++j) {
    if (nb[j] < 0 || nb[j] >= c->V || nb[j] == view) return c->fail(SLF_EINVAL, "bad neighbour view %d", nb[j]);
    for (int k = 0; k < j; ++k)
      if (nb[k] == nb[j]) return c->fail(SLF_EINVAL, "neighbour view %d repeated", nb[j]);
  }
  c->vh[view].nbrs = nb;
  c->geom_dirty = true;
  return SLF_OK;
}

static int64_t pix_off_of(const slf_ctx *c, int view) {
  int64_t o = 0;
  for (int v = 0; v < view; ++v) o += (int64_t)c->vh[v].W * c->vh[v].H;
  return o;
}

int slf_set_image_rgb8(slf_ctx *c, int view, const uint8_t *rgb, int64_t stride, int is_device) {
  if (!c) return SLF_EINVAL;
  if (int rc = check_idle(c)) return rc;
  if (view < 0 || view >= c->V) return c->fail(SLF_EINVAL, "view %d out of range", view);
  const ViewHost &h = c->vh[view];
  if (!rgb) return c->fail(SLF_EINVAL, "rgb is NULL");
  if (stride < 3 * (int64_t)h.W) return c->fail(SLF_EINVAL, "row stride %lld < 3 W", (long long)stride);
  HIP_OR_FAIL(c, hipSetDevice(c->device));
  uint8_t *dst = c->d_rgb + 3 * pix_off_of(c, view);
  HIP_OR_FAIL(c, hipMemcpy2DAsync(dst, 3 * (size_t)h.W, rgb, (size_t)stride, 3 * (size_t)h.W, (size_t)h.H,
                                  is_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream));
  if (!is_device) HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  c->vh[view].has_img = true;
  c->quads_dirty = true;
  c->sp_dirty = true;  // pixel entries carry the reference colours
  return SLF_OK;
}

int slf_set_labels(slf_ctx *c, int view, const int32_t *labels, int64_t stride, int gw, int gh, int is_device) {
  if (!c) return SLF_EINVAL;
  if (int rc = check_idle(c)) return rc;
  if (view < 0 || view >= c->V) return c->fail(SLF_EINVAL, "view %d out of range", view);
  const ViewHost &h = c->vh[view];
  if (!labels) return c->fail(SLF_EINVAL, "labels is NULL");
  if (stride < h.W) return c->fail(SLF_EINVAL, "row stride %lld < W", (long long)stride);
  if (gw < 1 || gh < 1 || (int64_t)gw * gh > (1 << 24)) return c->fail(SLF_EINVAL, "grid %d x %d invalid", gw, gh);
  if (!is_device) {
    const int K = gw * gh;
    for (int y = 0; y < h.H; ++y)
      for (int x = 0; x < h.W; ++x) {
        const int l = labels[(int64_t)y * stride + x];
        if (l < 0 || l >= K) return c->fail(SLF_EINVAL, "label %d at (%d, %d) outside [0, %d)", l, x, y, K);
      }
  }
  HIP_OR_FAIL(c, hipSetDevice(c->device));
  int *dst = c->d_labels + pix_off_of(c, view);
  HIP_OR_FAIL(c, hipMemcpy2DAsync(dst, sizeof(int) * (size_t)h.W, labels, sizeof(int) * (size_t)stride,
                                  sizeof(int) * (size_t)h.W, (size_t)h.H,
                                  is_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream));
  if (!is_device) HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  ViewHost &hv = c->vh[view];
  if (hv.gw != gw || hv.gh != gh) c->geom_dirty = true;
  hv.gw = gw;
  hv.gh = gh;
  hv.has_lab = true;
  c->sp_dirty = true;
  return SLF_OK;
}

int slf_prepare(slf_ctx *c) {
  if (!c) return SLF_EINVAL;
  if (int rc = check_idle(c)) return rc;
  HIP_OR_FAIL(c, hipSetDevice(c->device));
  return ensure_setup(c);
}

int slf_sweep(slf_ctx *c) {
  if (!c) return SLF_EINVAL;
  if (int rc = check_idle(c)) return rc;
  HIP_OR_FAIL(c, hipSetDevice(c->device));
  int rc = ensure_setup(c);
  if (rc) return rc;
  SweepArgs a;
  sweep_args(c, a);
  HIP_OR_FAIL(c, launch_sweep(c->p.image_precision, a, c->d_claims, c->n_cu, c->stream));
  after_sweep(c);
  return SLF_OK;
}

int slf_set_planes(slf_ctx *c, int view, const float *planes) {
  if (!c) return SLF_EINVAL;
  if (int rc = check_idle(c)) return rc;
  if (view < 0 || view >= c->V) return c->fail(SLF_EINVAL, "view %d out of range", view);
  if (!planes) return c->fail(SLF_EINVAL, "planes is NULL");
  HIP_OR_FAIL(c, hipSetDevice(c->device));
  int rc = ensure_setup(c);
  if (rc) return rc;
  if ((rc = fetch_stats(c))) return rc;
  const ViewDev &d = c->views_h[view];
  const ViewHost &h = c->vh[view];
  const int K = d.gw * d.gh;
  std::vector<float4> pl(K), tab(2 * (size_t)K);
  for (int s = 0; s < K; ++s) {
    const int g = d.sp_off + s;
    tab[2 * s] = c->col_h[g];
    if (c->area_h[g] == 0) {
      pl[s] = make_float4(0.f, 0.f, 0.f, 0.f);
      tab[2 * s + 1] = make_float4(0.f, 0.f, 0.f, 0.f);
      continue;
    }
    const double dd = planes[4 * s], n0 = planes[4 * s + 1], n1 = planes[4 * s + 2], n2 = planes[4 * s + 3];
    if (!std::isfinite(dd) || !(dd > 0) || !std::isfinite(n0) || !std::isfinite(n1) || !std::isfinite(n2))
      return c->fail(SLF_EINVAL, "view %d cell %d: plane not finite or d <= 0", view, s);
    if (std::fabs(std::sqrt(n0 * n0 + n1 * n1 + n2 * n2) - 1.0) > 1e-3)
      return c->fail(SLF_EINVAL, "view %d cell %d: normal is not unit length", view, s);
    const double cu = c->cen_h[g].x, cv = c->cen_h[g].y;
    const double rx = h.Kinv[0] * cu + h.Kinv[1] * cv + h.Kinv[2];
    const double ry = h.Kinv[3] * cu + h.Kinv[4] * cv + h.Kinv[5];
    const double rz = h.Kinv[6] * cu + h.Kinv[7] * cv + h.Kinv[8];
    const double tt = n0 * rx + n1 * ry + n2 * rz;
    if (!(tt > 0)) return c->fail(SLF_EINVAL, "view %d cell %d: plane does not face the camera", view, s);
    const double delta = dd * tt;
    pl[s] = make_float4((float)dd, (float)n0, (float)n1, (float)n2);
    tab[2 * s + 1] = make_float4((float)((n0 * h.Kinv[0] + n1 * h.Kinv[3] + n2 * h.Kinv[6]) / delta),
                                 (float)((n0 * h.Kinv[1] + n1 * h.Kinv[4] + n2 * h.Kinv[7]) / delta),
                                 (float)((n0 * h.Kinv[2] + n1 * h.Kinv[5] + n2 * h.Kinv[8]) / delta), 0.f);
  }
  HIP_OR_FAIL(c, hipMemcpyAsync(c->d_planes[c->cur] + d.sp_off, pl.data(), sizeof(float4) * K, hipMemcpyHostToDevice,
                                c->stream));
  HIP_OR_FAIL(c, hipMemcpyAsync(c->d_tab[c->cur] + 2 * (size_t)d.sp_off, tab.data(), 2 * sizeof(float4) * K,
                                hipMemcpyHostToDevice, c->stream));
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  c->vh[view].has_planes = true;
  return SLF_OK;
}

int slf_propagate(slf_ctx *c, int first_iter, int n_iters) {
  if (!c) return SLF_EINVAL;
  if (int rc = check_idle(c)) return rc;
  if (first_iter < 1 || n_iters < 0) return c->fail(SLF_EINVAL, "need first_iter >= 1 and n_iters >= 0");
  HIP_OR_FAIL(c, hipSetDevice(c->device));
  int rc = ensure_setup(c);
  if (rc) return rc;
  for (const auto &v : c->vh)
    if (!v.has_planes) return c->fail(SLF_ESTATE, "every view needs planes (slf_sweep or slf_set_planes)");
  for (int it = first_iter; it < first_iter + n_iters; ++it) {
    RefineArgs a;
    refine_args(c, it, a);
    HIP_OR_FAIL(c, launch_refine(c->p.image_precision, a, c->d_refine_args, c->d_claims, c->n_cu, c->stream));
    after_refine(c);
  }
  return SLF_OK;
}

int slf_warm_start(slf_ctx *c) {
  if (!c) return SLF_EINVAL;
  if (int rc = check_idle(c)) return rc;
  HIP_OR_FAIL(c, hipSetDevice(c->device));
  int rc = ensure_setup(c);
  if (rc) return rc;
  if (!c->warm_ok)
    return c->fail(SLF_ESTATE, "no previous plane state on these cameras and grids to start from");
  const double q_mid = 0.5 * (1.0 / c->p.d_min + 1.0 / c->p.d_max);
  HIP_OR_FAIL(c, launch_warm(c->d_views, c->d_sp_view, c->d_area, c->d_centroid_d, c->d_colour, c->d_planes[c->cur],
                             c->d_tab[c->cur], c->S, 1.0 / q_mid, c->stream));
  for (auto &v : c->vh) v.has_planes = true;
  c->warm_ok = false;
  return SLF_OK;
}

int slf_get_footprint(slf_ctx *c, uint64_t *bytes) {
  if (!c || !bytes) return SLF_EINVAL;
  if (footprint(c, bytes)) return c->fail(SLF_ESTATE, "cameras and label grids must be set first");
  return SLF_OK;
}

int slf_get_planes(slf_ctx *c, int view, float *planes, float *energy, int32_t *choice, float *margin) {
  if (!c) return SLF_EINVAL;
  if (int rc = check_idle(c)) return rc;
  if (view < 0 || view >= c->V) return c->fail(SLF_EINVAL, "view %d out of range", view);
  if (c->sp_dirty || c->views_h.empty() || !c->vh[view].has_planes)
    return c->fail(SLF_ESTATE, "no planes for view %d", view);
  HIP_OR_FAIL(c, hipSetDevice(c->device));
  const ViewDev &d = c->views_h[view];
  const size_t K = (size_t)d.gw * d.gh;
  if (planes)
    HIP_OR_FAIL(c, hipMemcpyAsync(planes, c->d_planes[c->cur] + d.sp_off, sizeof(float4) * K, hipMemcpyDeviceToHost,
                                  c->stream));
  if (energy)
    HIP_OR_FAIL(c, hipMemcpyAsync(energy, c->d_energy + d.sp_off, sizeof(float) * K, hipMemcpyDeviceToHost, c->stream));
  if (choice)
    HIP_OR_FAIL(c, hipMemcpyAsync(choice, c->d_choice + d.sp_off, sizeof(int) * K, hipMemcpyDeviceToHost, c->stream));
  if (margin)
    HIP_OR_FAIL(c, hipMemcpyAsync(margin, c->d_margin + d.sp_off, sizeof(float) * K, hipMemcpyDeviceToHost, c->stream));
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  return SLF_OK;
}

int slf_get_depth(slf_ctx *c, int view, float *out, int64_t stride, int is_device) {
  if (!c) return SLF_EINVAL;
  if (int rc = check_idle(c)) return rc;
  if (view < 0 || view >= c->V) return c->fail(SLF_EINVAL, "view %d out of range", view);
  if (!out) return c->fail(SLF_EINVAL, "out is NULL");
  if (c->sp_dirty || c->views_h.empty() || !c->vh[view].has_planes)
    return c->fail(SLF_ESTATE, "no planes for view %d", view);
  const ViewDev &d = c->views_h[view];
  if (stride < d.W) return c->fail(SLF_EINVAL, "row stride %lld < W", (long long)stride);
  HIP_OR_FAIL(c, hipSetDevice(c->device));
  if (is_device) {
    HIP_OR_FAIL(c, launch_depth(c->d_views, d, view, c->d_labels, c->d_tab[c->cur], out, stride, c->stream));
    return SLF_OK;
  }
  const int64_t n = (int64_t)d.W * d.H;
  if (n > c->depth_tmp_n) {
    dfree(c->d_depth_tmp);
    int rc = ensure_alloc(c, sizeof(float) * n, (void **)&c->d_depth_tmp);
    if (rc) return rc;
    c->depth_tmp_n = n;
  }
  HIP_OR_FAIL(c, launch_depth(c->d_views, d, view, c->d_labels, c->d_tab[c->cur], c->d_depth_tmp, d.W, c->stream));
  HIP_OR_FAIL(c, hipMemcpy2DAsync(out, sizeof(float) * stride, c->d_depth_tmp, sizeof(float) * d.W,
                                  sizeof(float) * d.W, d.H, hipMemcpyDeviceToHost, c->stream));
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  return SLF_OK;
}

int slf_get_superpixels(slf_ctx *c, int view, int32_t *area, float *centroid, float *colour) {
  if (!c) return SLF_EINVAL;
  if (int rc = check_idle(c)) return rc;
  if (view < 0 || view >= c->V) return c->fail(SLF_EINVAL, "view %d out of range", view);
  if (c->sp_dirty || c->views_h.empty()) return c->fail(SLF_ESTATE, "superpixels not built yet");
  HIP_OR_FAIL(c, hipSetDevice(c->device));
  if (int rc = fetch_stats(c)) return rc;
  const ViewDev &d = c->views_h[view];
  const size_t K = (size_t)d.gw * d.gh;
  if (area) std::memcpy(area, c->area_h.data() + d.sp_off, sizeof(int) * K);
  if (centroid)
    for (size_t s = 0; s < K; ++s) {
      centroid[2 * s] = (float)c->cen_h[d.sp_off + s].x;
      centroid[2 * s + 1] = (float)c->cen_h[d.sp_off + s].y;
    }
  if (colour)
    for (size_t s = 0; s < K; ++s) {
      colour[3 * s] = c->col_h[d.sp_off + s].x;
      colour[3 * s + 1] = c->col_h[d.sp_off + s].y;
      colour[3 * s + 2] = c->col_h[d.sp_off + s].z;
    }
  return SLF_OK;
}

int slf_get_work(slf_ctx *c, uint64_t *evals, uint64_t *samples, uint64_t *pruned) {
  if (!c) return SLF_EINVAL;
  if (int rc = check_idle(c)) return rc;
  HIP_OR_FAIL(c, hipSetDevice(c->device));
  unsigned long long w[kWorkCounters] = {};
  HIP_OR_FAIL(c, hipMemcpyAsync(w, c->d_work, sizeof w, hipMemcpyDeviceToHost, c->stream));
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  if (evals) *evals = c->host_evals + w[0];
  if (samples) *samples = w[1] + w[3];
  if (pruned) *pruned = w[2];
  return SLF_OK;
}

int slf_get_sweep_work(slf_ctx *c, uint64_t *computed, uint64_t *total) {
  if (!c) return SLF_EINVAL;
  if (int rc = check_idle(c)) return rc;
  HIP_OR_FAIL(c, hipSetDevice(c->device));
  unsigned long long w = 0;
  HIP_OR_FAIL(c, hipMemcpyAsync(&w, c->d_work + 3, sizeof w, hipMemcpyDeviceToHost, c->stream));
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  if (computed) *computed = w;
  if (total) *total = c->host_sweep_total;
  return SLF_OK;
}

int slf_get_sweep_levels(slf_ctx *c, uint64_t *scored, uint64_t *decided) {
  if (!c) return SLF_EINVAL;
  if (int rc = check_idle(c)) return rc;
  HIP_OR_FAIL(c, hipSetDevice(c->device));
  unsigned long long w = 0;
  HIP_OR_FAIL(c, hipMemcpyAsync(&w, c->d_work + 4, sizeof w, hipMemcpyDeviceToHost, c->stream));
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  if (scored) *scored = w;
  if (decided) *decided = c->host_evals;
  return SLF_OK;
}

int slf_reset_work(slf_ctx *c) {
  if (!c) return SLF_EINVAL;
  if (int rc = check_idle(c)) return rc;
  HIP_OR_FAIL(c, hipSetDevice(c->device));
  HIP_OR_FAIL(c, hipMemsetAsync(c->d_work, 0, kWorkCounters * sizeof(unsigned long long), c->stream));
  c->host_evals = c->host_sweep_total = 0;
  return SLF_OK;
}

int slf_synchronize(slf_ctx *c) {
  if (!c) return SLF_EINVAL;
  HIP_OR_FAIL(c, hipSetDevice(c->device));
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  return SLF_OK;
}

}  // extern "C"
