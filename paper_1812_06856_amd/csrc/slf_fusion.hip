// Stability-based depth fusion of the views' depth maps (Sec. III-D), as the
// two passes per reference view of Sec. III-E, run for all reference views at
// once:
//
//  1. k_fuse_project: one thread per source pixel.  The pixel's 3D point is
//     formed once and projected into every other view; the nearest pixel p of
//     reference r receives the point's camera-r depth in source view i's
//     layer of r's candidate buffer, through an atomic minimum on the FP32 bit
//     pattern (positive floats order like their bits), so of several points
//     of view i landing on p the closest is kept whatever the order.
//  2. k_fuse_vote: one thread per reference pixel.  Its candidates are its own
//     depth and one per other view; each non-zero candidate c_j scores +1 for
//     every other candidate within tau c_j of it and -1 for every other one;
//     the smallest candidate with a score >= 0 is the fused depth (equal
//     depths: the smaller view index), 0 if there is none.
//
// Precision.  Depth maps and candidates are FP32 (the paper's depth maps are
// FP32 textures).  The projection is FP64, in one fixed sequence of
// operations, and this file is compiled with -ffp-contract=off, so every
// candidate and pixel decision is the correctly rounded result of that
// sequence.  The agreement test is one FP32 subtraction and one FP32
// multiplication.  Integer outputs (winner, score, count) are exact.
//
// HBM traffic per frame (P pixels over V views of one size): the depth maps
// read once per pass, the candidate layers cleared, updated by atomics and
// read once ((V-1) P entries of 4 bytes each), the fused depth and the votes
// written once.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "slf_ctx.h"

namespace slf {
namespace {

constexpr uint32_t kNoCand = 0x7F800000u;  // +inf: no candidate yet
constexpr int kFuseMaxViews = 64;

// One view's camera and buffers for the fusion kernels (device table).
struct FuseView {
  double K[6];         // first two rows of K: a b c / d e f (last row 0 0 1)
  double R[9];         // X_cam = R X_world + t
  double t[3];
  int W, H;
  int64_t zoff;        // first entry of this reference's (V-1) candidate layers
  const float *depth;  // H x W, row stride W
  float *fused;        // H x W
  int *votes;          // H x W or null
};

// Fixed device scratch of slf_fuse_depth_static (callers that cannot
// allocate): the camera table, then the candidate layers of one reference
// view.  Each device holds its own copy until the process ends.
constexpr int64_t kStaticScratchBytes = 64ll << 20;
constexpr int64_t kStaticTableBytes = 16 << 10;
constexpr int64_t kStaticLayerBytes = kStaticScratchBytes - kStaticTableBytes;
static_assert(sizeof(FuseView) * kFuseMaxViews <= kStaticTableBytes, "camera table does not fit");
constexpr int kMaxDevices = 64;

__global__ __launch_bounds__(256) void k_fuse_clear(uint32_t *z, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) z[k] = kNoCand;
}

// Pass 1.  blockIdx.y = source view i; each thread one pixel of view i.
// ref >= 0: only into reference `ref`, whose layers start at z[0];
// ref < 0: into every other view r, whose layers start at z[views[r].zoff].
__global__ __launch_bounds__(256) void k_fuse_project(const FuseView *__restrict__ views, int V, int ref,
                                                      uint32_t *__restrict__ z) {
  const int i = blockIdx.y;
  if (i == ref) return;
  const FuseView &S = views[i];
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)S.W * S.H) return;
  const float D = S.depth[idx];
  if (!(D > 0.f) || isinf(D)) return;
  const int u = (int)(idx % S.W), v = (int)(idx / S.W);
  // the ray (x, y, 1) through (u, v) solves [[a b] [d e]] (x, y) = (u - c, v - f) by Cramer's rule
  const double du = (double)u - S.K[2], dv = (double)v - S.K[5];
  const double det = S.K[0] * S.K[4] - S.K[1] * S.K[3];
  const double x = (S.K[4] * du - S.K[1] * dv) / det;
  const double y = (S.K[0] * dv - S.K[3] * du) / det;
  const double Dd = (double)D;
  const double Y0 = Dd * x - S.t[0], Y1 = Dd * y - S.t[1], Y2 = Dd - S.t[2];
  // world point R_i^T (X_i - t_i)
  double Xw[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) Xw[j] = S.R[0 + j] * Y0 + S.R[3 + j] * Y1 + S.R[6 + j] * Y2;
  const int r_lo = ref >= 0 ? ref : 0, r_hi = ref >= 0 ? ref + 1 : V;
  for (int r = r_lo; r < r_hi; ++r) {
    if (r == i) continue;
    const FuseView &Rv = views[r];
    double Xr[3];
#pragma unroll
    for (int j = 0; j < 3; ++j)
      Xr[j] = Rv.R[3 * j + 0] * Xw[0] + Rv.R[3 * j + 1] * Xw[1] + Rv.R[3 * j + 2] * Xw[2] + Rv.t[j];
    if (!(Xr[2] > 0.0)) continue;
    const double px = (Rv.K[0] * Xr[0] + Rv.K[1] * Xr[1] + Rv.K[2] * Xr[2]) / Xr[2];
    const double py = (Rv.K[3] * Xr[0] + Rv.K[4] * Xr[1] + Rv.K[5] * Xr[2]) / Xr[2];
    const double fu = floor(px + 0.5), fv = floor(py + 0.5);
    if (!(fu >= 0.0 && fu <= (double)(Rv.W - 1) && fv >= 0.0 && fv <= (double)(Rv.H - 1))) continue;
    const float zf = (float)Xr[2];
    if (!(zf > 0.f) || isinf(zf)) continue;
    const int layer = i < r ? i : i - 1;
    const int64_t base = ref >= 0 ? 0 : Rv.zoff;
    uint32_t *slot = z + base + (int64_t)layer * Rv.W * Rv.H + (int64_t)(int)fv * Rv.W + (int)fu;
    atomicMin(slot, __float_as_uint(zf));
  }
}

// Writes up to kTableChunk table entries passed by value (the launch copies
// its arguments, so no host buffer has to outlive the call).
constexpr int kTableChunk = 8;
struct TableChunk {
  FuseView v[kTableChunk];
};
__global__ void k_fuse_put_table(FuseView *dst, TableChunk chunk, int n) {
  const int k = threadIdx.x;
  if (k < n) dst[k] = chunk.v[k];
}

__device__ inline float own_depth(float d) { return (d > 0.f && !isinf(d)) ? d : 0.f; }

__device__ inline int pack_votes(int winner, int n, int s) {
  return (int)(((uint32_t)(uint16_t)(int16_t)s << 16) | ((uint32_t)n << 8) | (uint32_t)(winner < 0 ? 255 : winner));
}

// Pass 2.  blockIdx.y = reference view (or `ref` alone); each thread one pixel.
// VMAX > 0: candidates in registers (V <= VMAX, loops unrolled); VMAX = 0: any V <= 64.
template <int VMAX>
__global__ __launch_bounds__(256) void k_fuse_vote(const FuseView *__restrict__ views, int V, int ref,
                                                   const uint32_t *__restrict__ z, float tau) {
  const int r = ref >= 0 ? ref : (int)blockIdx.y;
  const FuseView &Rv = views[r];
  const int64_t P = (int64_t)Rv.W * Rv.H;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= P) return;
  const uint32_t *zr = z + (ref >= 0 ? 0 : Rv.zoff);
  constexpr int N = VMAX > 0 ? VMAX : kFuseMaxViews;
  constexpr int UNR = VMAX > 0 ? VMAX : 1;  // unrolled only for the register form
  float c[N];
  int m = 0;
#pragma unroll UNR
  for (int k = 0; k < N; ++k) {
    float ck = 0.f;
    if (k < V) {
      if (k == r) {
        ck = own_depth(Rv.depth[idx]);
      } else {
        const uint32_t b = zr[(int64_t)(k < r ? k : k - 1) * P + idx];
        ck = b == kNoCand ? 0.f : __uint_as_float(b);
      }
    }
    c[k] = ck;
    m += ck > 0.f;
  }
  int best = -1, best_s = 0;
  float best_c = 0.f;
#pragma unroll UNR
  for (int j = 0; j < N; ++j) {
    if (j >= V) break;
    const float cj = c[j];
    if (!(cj > 0.f)) continue;
    const float lim = tau * cj;
    int s = 0;
#pragma unroll UNR
    for (int k = 0; k < N; ++k) {
      if (k >= V) break;
      const float ck = c[k];
      if (k == j || !(ck > 0.f)) continue;
      float d = ck - cj;
      if (d < 0.f) d = -d;
      s += (d <= lim) ? 1 : -1;
    }
    if (s >= 0 && (best < 0 || cj < best_c)) {
      best = j;
      best_c = cj;
      best_s = s;
    }
  }
  Rv.fused[idx] = best >= 0 ? best_c : 0.f;
  if (Rv.votes) Rv.votes[idx] = pack_votes(best, m, best_s);
}

// Fills the host table: cameras of the context, the buffers given, and the
// candidate-layer offsets for the all-references pass.  Returns the number of
// candidate entries that pass needs.
int64_t fuse_table(const slf_ctx *c, const float *const *depth, float *const *fused, int32_t *const *votes,
                   FuseView *tab) {
  const int V = c->V;
  for (int r = 0; r < V; ++r) tab[r] = FuseView{};
  int64_t off = 0;
  for (int r = 0; r < V; ++r) {
    const ViewHost &h = c->vh[r];
    FuseView &f = tab[r];
    for (int k = 0; k < 6; ++k) f.K[k] = h.K[k];
    for (int k = 0; k < 9; ++k) f.R[k] = h.R[k];
    for (int k = 0; k < 3; ++k) f.t[k] = h.t[k];
    f.W = h.W;
    f.H = h.H;
    f.zoff = off;
    f.depth = depth[r];
    f.fused = fused[r];
    f.votes = votes ? votes[r] : nullptr;
    off += (int64_t)(V - 1) * h.W * h.H;
  }
  return off;
}

int max_pixels(const FuseView *tab, int V) {
  int64_t m = 1;
  for (int r = 0; r < V; ++r) m = std::max<int64_t>(m, (int64_t)tab[r].W * tab[r].H);
  return (int)m;
}

hipError_t launch_vote(const FuseView *d_tab, int V, int ref, const uint32_t *z, float tau, int64_t maxP, int ny,
                       hipStream_t st) {
  const dim3 grid((unsigned)((maxP + 255) / 256), (unsigned)ny);
  if (V <= 8)
    hipLaunchKernelGGL(k_fuse_vote<8>, grid, dim3(256), 0, st, d_tab, V, ref, z, tau);
  else if (V <= 16)
    hipLaunchKernelGGL(k_fuse_vote<16>, grid, dim3(256), 0, st, d_tab, V, ref, z, tau);
  else
    hipLaunchKernelGGL(k_fuse_vote<0>, grid, dim3(256), 0, st, d_tab, V, ref, z, tau);
  return hipGetLastError();
}

// Both passes for all reference views: one clear, one projection launch over
// the pixels of all views, one vote launch over the pixels of all views.
hipError_t fuse_all(const FuseView *d_tab, const std::vector<FuseView> &tab, uint32_t *z, int64_t nz, float tau,
                    hipStream_t st) {
  const int V = (int)tab.size();
  const int64_t maxP = max_pixels(tab.data(), V);
  hipLaunchKernelGGL(k_fuse_clear, dim3((unsigned)std::min<int64_t>((nz + 255) / 256, 65536)), dim3(256), 0, st, z,
                     nz);
  hipLaunchKernelGGL(k_fuse_project, dim3((unsigned)((maxP + 255) / 256), (unsigned)V), dim3(256), 0, st, d_tab, V,
                     -1, z);
  return launch_vote(d_tab, V, -1, z, tau, maxP, V, st);
}

int check_fuse_args(slf_ctx *c, float tau) {
  if (c->V < 2 || c->vh.empty()) return c->fail(SLF_ESTATE, "cameras must be set first");
  if (c->V > kFuseMaxViews) return c->fail(SLF_EUNSUPPORTED, "fusion supports at most %d views", kFuseMaxViews);
  if (!(tau >= 0.f) || !std::isfinite(tau)) return c->fail(SLF_EINVAL, "agree_tol must be finite and >= 0");
  return SLF_OK;
}

int grow(slf_ctx *c, void **p, int64_t *have, int64_t need_bytes) {
  if (need_bytes <= *have) return SLF_OK;
  if (*p) (void)hipFree(*p);
  *p = nullptr;
  *have = 0;
  hipError_t e = hipMalloc(p, (size_t)std::max<int64_t>(need_bytes, 16));
  if (e != hipSuccess) {
    *p = nullptr;
    return c->fail(SLF_ENOMEM, "hipMalloc(%lld): %s", (long long)need_bytes, hipGetErrorString(e));
  }
  *have = need_bytes;
  return SLF_OK;
}

// Uploads the table when it changed since the last upload.  The host copy
// lives in the context until the next change, which first waits for the
// stream, so an upload in flight never reads a buffer being rewritten.
int upload_table(slf_ctx *c, const std::vector<FuseView> &tab) {
  const size_t bytes = sizeof(FuseView) * tab.size();
  if (c->fcams_h.size() == bytes && c->d_fcams && std::memcmp(c->fcams_h.data(), tab.data(), bytes) == 0)
    return SLF_OK;
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  int rc;
  if ((rc = grow(c, (void **)&c->d_fcams, &c->fcams_bytes, (int64_t)bytes))) return rc;
  c->fcams_h.resize(bytes);
  std::memcpy(c->fcams_h.data(), tab.data(), bytes);
  HIP_OR_FAIL(c, hipMemcpyAsync(c->d_fcams, c->fcams_h.data(), bytes, hipMemcpyHostToDevice, c->stream));
  return SLF_OK;
}

// Runs both passes for the given device buffers with buffers the context owns
// (candidate layers and the device table).
int fuse_into(slf_ctx *c, const float *const *depth, float *const *fused, int32_t *const *votes, float tau) {
  std::vector<FuseView> tab(c->V);
  const int64_t nz = fuse_table(c, depth, fused, votes, tab.data());
  int rc;
  if ((rc = grow(c, (void **)&c->d_fz, &c->fz_bytes, nz * (int64_t)sizeof(uint32_t)))) return rc;
  if ((rc = upload_table(c, tab))) return rc;
  HIP_OR_FAIL(c, fuse_all((const FuseView *)c->d_fcams, tab, (uint32_t *)c->d_fz, nz, tau, c->stream));
  return SLF_OK;
}

}  // namespace
}  // namespace slf

// The scratch itself.  Host code never passes `scratch` to a kernel or a copy:
// on the host the name stands in for the symbol, not for a device address.
// Its address on each device is taken once, at context creation with that
// device current, and kept in scratch_ptr.
static __device__ __align__(256) unsigned char scratch[slf::kStaticScratchBytes];

namespace {
std::mutex scratch_mu;
void *scratch_ptr[slf::kMaxDevices] = {};
}  // namespace

int slf::static_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return SLF_EUNSUPPORTED;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (scratch_ptr[device]) return SLF_OK;
  void *p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return SLF_EDEVICE;
  scratch_ptr[device] = p;
  return SLF_OK;
}

namespace {
void *static_scratch(int device) {
  if (device < 0 || device >= slf::kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(scratch_mu);
  return scratch_ptr[device];
}
}  // namespace

using namespace slf;

extern "C" {

int slf_fuse(slf_ctx *c, float agree_tol) {
  if (!c) return SLF_EINVAL;
  if (int rc = check_idle(c)) return rc;
  if (int rc = check_fuse_args(c, agree_tol)) return rc;
  if (c->sp_dirty || c->views_h.empty()) return c->fail(SLF_ESTATE, "no planes: sweep or set planes first");
  for (int v = 0; v < c->V; ++v)
    if (!c->vh[v].has_planes) return c->fail(SLF_ESTATE, "no planes for view %d", v);
  HIP_OR_FAIL(c, hipSetDevice(c->device));
  const int64_t n = c->total_px;
  int rc;
  if ((rc = grow(c, (void **)&c->d_fdepth, &c->fdepth_bytes, n * 4))) return rc;
  if ((rc = grow(c, (void **)&c->d_fused, &c->fused_bytes, n * 4))) return rc;
  if ((rc = grow(c, (void **)&c->d_fvotes, &c->fvotes_bytes, n * 4))) return rc;
  std::vector<const float *> din(c->V);
  std::vector<float *> dout(c->V);
  std::vector<int32_t *> dvotes(c->V);
  for (int v = 0; v < c->V; ++v) {
    const ViewDev &d = c->views_h[v];
    float *dep = (float *)c->d_fdepth + d.pix_off;
    HIP_OR_FAIL(c, launch_depth(c->d_views, d, v, c->d_labels, c->d_tab[c->cur], dep, d.W, c->stream));
    din[v] = dep;
    dout[v] = (float *)c->d_fused + d.pix_off;
    dvotes[v] = (int32_t *)c->d_fvotes + d.pix_off;
  }
  c->has_fused = false;
  if ((rc = fuse_into(c, din.data(), dout.data(), dvotes.data(), agree_tol))) return rc;
  c->has_fused = true;
  return SLF_OK;
}

int slf_get_fused_depth(slf_ctx *c, int view, float *out, int64_t stride, int32_t *votes, int is_device) {
  if (!c) return SLF_EINVAL;
  if (int rc = check_idle(c)) return rc;
  if (view < 0 || view >= c->V) return c->fail(SLF_EINVAL, "view %d out of range", view);
  if (!c->has_fused) return c->fail(SLF_ESTATE, "no fused depth: call slf_fuse first");
  const ViewHost &h = c->vh[view];
  if ((out || votes) && stride < h.W) return c->fail(SLF_EINVAL, "row stride %lld < W", (long long)stride);
  HIP_OR_FAIL(c, hipSetDevice(c->device));
  const int64_t off = c->views_h[view].pix_off;
  const hipMemcpyKind kind = is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (out)
    HIP_OR_FAIL(c, hipMemcpy2DAsync(out, sizeof(float) * stride, (const float *)c->d_fused + off, sizeof(float) * h.W,
                                    sizeof(float) * h.W, h.H, kind, c->stream));
  if (votes)
    HIP_OR_FAIL(c, hipMemcpy2DAsync(votes, sizeof(int32_t) * stride, (const int32_t *)c->d_fvotes + off,
                                    sizeof(int32_t) * h.W, sizeof(int32_t) * h.W, h.H, kind, c->stream));
  if (!is_device) HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  return SLF_OK;
}

int slf_fuse_depth(slf_ctx *c, const float *const *depth, float *const *fused, int32_t *const *votes,
                   float agree_tol) {
  if (!c) return SLF_EINVAL;
  if (int rc = check_idle(c)) return rc;
  if (int rc = check_fuse_args(c, agree_tol)) return rc;
  if (!depth || !fused) return c->fail(SLF_EINVAL, "depth and fused must not be NULL");
  for (int v = 0; v < c->V; ++v) {
    if (!depth[v] || !fused[v]) return c->fail(SLF_EINVAL, "depth or fused buffer of view %d is NULL", v);
    if (votes && !votes[v]) return c->fail(SLF_EINVAL, "votes buffer of view %d is NULL", v);
  }
  HIP_OR_FAIL(c, hipSetDevice(c->device));
  return fuse_into(c, depth, fused, votes, agree_tol);
}

int slf_fuse_depth_static(slf_ctx *c, const float *const *depth, float *const *fused, int32_t *const *votes,
                          float agree_tol) {
  if (!c) return SLF_EINVAL;
  if (int rc = check_idle(c)) return rc;
  if (int rc = check_fuse_args(c, agree_tol)) return rc;
  if (!depth || !fused) return c->fail(SLF_EINVAL, "depth and fused must not be NULL");
  for (int v = 0; v < c->V; ++v) {
    if (!depth[v] || !fused[v]) return c->fail(SLF_EINVAL, "depth or fused buffer of view %d is NULL", v);
    if (votes && !votes[v]) return c->fail(SLF_EINVAL, "votes buffer of view %d is NULL", v);
    const int64_t need = (int64_t)(c->V - 1) * c->vh[v].W * c->vh[v].H * (int64_t)sizeof(uint32_t);
    if (need > kStaticLayerBytes)
      return c->fail(SLF_EUNSUPPORTED, "view %d needs %lld bytes of candidate layers, above the %lld of the static scratch",
                     v, (long long)need, (long long)kStaticLayerBytes);
  }
  unsigned char *base = (unsigned char *)static_scratch(c->device);
  if (!base) return c->fail(SLF_EDEVICE, "static scratch of device %d not set up", c->device);
  HIP_OR_FAIL(c, hipSetDevice(c->device));
  FuseView tab[kFuseMaxViews];  // host copy on the stack: the call allocates nothing
  fuse_table(c, depth, fused, votes, tab);
  FuseView *d_tab = (FuseView *)base;
  uint32_t *z = (uint32_t *)(base + kStaticTableBytes);
  const int V = c->V;
  for (int k0 = 0; k0 < V; k0 += kTableChunk) {
    TableChunk ch{};
    const int n = std::min(kTableChunk, V - k0);
    for (int k = 0; k < n; ++k) ch.v[k] = tab[k0 + k];
    hipLaunchKernelGGL(k_fuse_put_table, dim3(1), dim3(64), 0, c->stream, d_tab + k0, ch, n);
  }
  HIP_OR_FAIL(c, hipGetLastError());
  const int64_t maxP = max_pixels(tab, V);
  // one reference view at a time: its candidate layers fill the scratch
  for (int r = 0; r < V; ++r) {
    const int64_t P = (int64_t)tab[r].W * tab[r].H;
    const int64_t nz = (int64_t)(V - 1) * P;
    hipLaunchKernelGGL(k_fuse_clear, dim3((unsigned)std::min<int64_t>((nz + 255) / 256, 65536)), dim3(256), 0,
                       c->stream, z, nz);
    hipLaunchKernelGGL(k_fuse_project, dim3((unsigned)((maxP + 255) / 256), (unsigned)V), dim3(256), 0, c->stream,
                       (const FuseView *)d_tab, V, r, z);
    HIP_OR_FAIL(c, launch_vote(d_tab, V, r, z, agree_tol, P, 1, c->stream));
  }
  return SLF_OK;
}

}  // extern "C"
