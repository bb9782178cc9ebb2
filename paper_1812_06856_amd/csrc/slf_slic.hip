// Grid-seeded SLIC segmentation on the GPU (Sec. III-A: SLIC superpixels,
// read as a regular grid of cells whose ids are the labels; Sec. III-E: the
// segmentation runs on the GPU before the plane sweep).
//
//  - k_slic_init: one thread per cluster; the centre starts at its cell's
//    centre with the colour of the nearest pixel (round half up).
//  - k_slic_assign: one thread per pixel; the pixel compares the centres of
//    the 3 x 3 cells around its own cell, D = |rgb - rgb_k|^2 + ((u - u_k)^2 +
//    (v - v_k)^2) w, colours in 0..255; ties go to the first centre in the
//    order dy = -1..1, dx = -1..1.
//  - k_slic_update: one wavefront per cluster gathers the pixels of its 3 x 3
//    cell window that carry its label and sums their positions and colours as
//    exact integers; the centre becomes sum / count in FP32 (no float
//    atomics: the result does not depend on the order).
//  - connectivity: union-find over 4-neighbours of equal label (links go from
//    the larger root to the smaller, so a component's root is its first pixel
//    in raster order), component sizes, the largest component per label by a
//    64-bit atomic maximum of (size, ~root), then every pixel walks from its
//    component to the first component that keeps its label: a component that
//    does not takes the final label of the component left of its first pixel
//    (above it in the first column), whose root comes earlier, so the walk
//    ends.  The component of the image's first pixel keeps its label.
//
// Every decision is integer and taken in FP32 from exactly represented
// inputs in one fixed order of operations; this file is compiled with
// -ffp-contract=off, so the labels are the same on every run.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "slf_ctx.h"

namespace slf {
namespace {

__device__ __forceinline__ int cell_of(int p, int n, int g) {
  // floor((p + 0.5) g / n) in integers
  const int c = (int)(((long long)(2 * p + 1) * g) / (2 * (long long)n));
  return c < g ? c : g - 1;
}

__global__ __launch_bounds__(256) void k_slic_init(const uint8_t *__restrict__ rgb, int W, int H, int gw, int gh,
                                                   float *__restrict__ cen, unsigned long long *__restrict__ best) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= gw * gh) return;
  const int gx = k % gw, gy = k / gw;
  const double u = (gx + 0.5) * (double)W / gw - 0.5, v = (gy + 0.5) * (double)H / gh - 0.5;
  int iu = (int)floor(u + 0.5), iv = (int)floor(v + 0.5);
  iu = min(iu, W - 1);
  iv = min(iv, H - 1);
  const uint8_t *p = rgb + 3 * ((long long)iv * W + iu);
  cen[5 * k + 0] = (float)u;
  cen[5 * k + 1] = (float)v;
  cen[5 * k + 2] = (float)p[0];
  cen[5 * k + 3] = (float)p[1];
  cen[5 * k + 4] = (float)p[2];
  best[k] = 0ull;
}

__global__ __launch_bounds__(256) void k_slic_assign(const uint8_t *__restrict__ rgb, int W, int H, int gw, int gh,
                                                     const float *__restrict__ cen, float wsp,
                                                     int *__restrict__ labels) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x, v = blockIdx.y;
  if (u >= W) return;
  const int cx = cell_of(u, W, gw), cy = cell_of(v, H, gh);
  const uint8_t *p = rgb + 3 * ((long long)v * W + u);
  const float r = (float)p[0], g = (float)p[1], b = (float)p[2];
  float best = INFINITY;
  int bk = cy * gw + cx;
  for (int dy = -1; dy <= 1; ++dy) {
    const int yy = cy + dy;
    if (yy < 0 || yy >= gh) continue;
    for (int dx = -1; dx <= 1; ++dx) {
      const int xx = cx + dx;
      if (xx < 0 || xx >= gw) continue;
      const int k = yy * gw + xx;
      const float *c = cen + 5 * k;
      const float du = (float)u - c[0], dv = (float)v - c[1];
      const float d0 = r - c[2], d1 = g - c[3], d2 = b - c[4];
      const float dc = d0 * d0 + d1 * d1 + d2 * d2;
      const float ds = du * du + dv * dv;
      const float D = dc + ds * wsp;
      if (D < best) {
        best = D;
        bk = k;
      }
    }
  }
  labels[(long long)v * W + u] = bk;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// One wavefront per cluster; blockDim = 256 (4 clusters per block).
__global__ __launch_bounds__(256) void k_slic_update(const uint8_t *__restrict__ rgb, const int *__restrict__ labels,
                                                     int W, int H, int gw, int gh, float *__restrict__ cen) {
  const int k = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (k >= gw * gh) return;
  const int gx = k % gw, gy = k / gw;
  // pixel window of cells gx-1..gx+1, gy-1..gy+1 (a safe superset; other labels are skipped)
  const int x0 = max(0, (int)((long long)max(gx - 1, 0) * W / gw) - 1);
  const int x1 = min(W - 1, (int)(((long long)min(gx + 2, gw) * W + gw - 1) / gw));
  const int y0 = max(0, (int)((long long)max(gy - 1, 0) * H / gh) - 1);
  const int y1 = min(H - 1, (int)(((long long)min(gy + 2, gh) * H + gh - 1) / gh));
  const int ww = x1 - x0 + 1, n = ww * (y1 - y0 + 1);
  unsigned long long su = 0, sv = 0, sr = 0, sg = 0, sb = 0, cnt = 0;
  for (int q = lane; q < n; q += 64) {
    const int u = x0 + q % ww, v = y0 + q / ww;
    const long long i = (long long)v * W + u;
    if (labels[i] == k) {
      su += u;
      sv += v;
      sr += rgb[3 * i];
      sg += rgb[3 * i + 1];
      sb += rgb[3 * i + 2];
      ++cnt;
    }
  }
  su = wave_sum_u64(su);
  sv = wave_sum_u64(sv);
  sr = wave_sum_u64(sr);
  sg = wave_sum_u64(sg);
  sb = wave_sum_u64(sb);
  cnt = wave_sum_u64(cnt);
  if (lane == 0 && cnt > 0) {
    const float fn = (float)cnt;
    cen[5 * k + 0] = (float)su / fn;
    cen[5 * k + 1] = (float)sv / fn;
    cen[5 * k + 2] = (float)sr / fn;
    cen[5 * k + 3] = (float)sg / fn;
    cen[5 * k + 4] = (float)sb / fn;
  }
}

// ---- connectivity

__device__ __forceinline__ int load_parent(const int *p, int x) {
  return __hip_atomic_load(p + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int find_root(const int *p, int x) {
  int y = load_parent(p, x);
  while (y != x) {  // parents only decrease, so the walk ends at the current root
    x = y;
    y = load_parent(p, x);
  }
  return x;
}

// Joins the trees of a and b, the larger root under the smaller.  If another
// thread changed b's parent first, the atomic returns that parent and the
// loop continues from it, so no link is lost; every pass moves to a smaller
// root, so the loop ends.
__device__ void unite(int *p, int a, int b) {
  while (true) {
    a = find_root(p, a);
    b = find_root(p, b);
    if (a == b) return;
    if (a > b) {
      const int t = a;
      a = b;
      b = t;
    }
    const int old = atomicMin(p + b, a);
    if (old == b) return;
    b = old;
  }
}

__global__ __launch_bounds__(256) void k_cc_init(int *__restrict__ parent, int *__restrict__ csize, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  parent[i] = (int)i;
  csize[i] = 0;
}

__global__ __launch_bounds__(256) void k_cc_link(const int *__restrict__ lab, int W, int H, int *parent) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x, v = blockIdx.y;
  if (u >= W) return;
  const int i = v * W + u;
  const int l = lab[i];
  if (u > 0 && lab[i - 1] == l) unite(parent, i, i - 1);
  if (v > 0 && lab[i - W] == l) unite(parent, i, i - W);
}

__global__ __launch_bounds__(256) void k_cc_flatten(int *parent, int *__restrict__ csize, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int r = find_root(parent, (int)i);
  atomicAdd(csize + r, 1);
  parent[i] = r;
}

__global__ __launch_bounds__(256) void k_cc_best(const int *__restrict__ lab, const int *__restrict__ parent,
                                                 const int *__restrict__ csize, unsigned long long *best, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || parent[i] != (int)i) return;
  // larger size wins; equal sizes: the smaller root (larger ~root)
  const unsigned long long key = ((unsigned long long)(unsigned)csize[i] << 32) | (unsigned)(~(unsigned)i);
  atomicMax(best + lab[i], key);
}

__global__ __launch_bounds__(256) void k_cc_final(const int *__restrict__ lab, const int *__restrict__ parent,
                                                  const unsigned long long *__restrict__ best, int W, long long n,
                                                  int *__restrict__ out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int x = parent[i];
  while (true) {  // roots strictly decrease along the walk, which ends at root 0 at the latest
    const int k = lab[x];
    if (x == 0 || (unsigned)(best[k] & 0xffffffffull) == ~(unsigned)x) {
      out[i] = k;
      return;
    }
    const int nb = (x % W) > 0 ? x - 1 : x - W;
    x = parent[nb];
  }
}

int grow(slf_ctx *c, void **p, int64_t *have, int64_t need) {
  if (need <= *have) return SLF_OK;
  if (*p) (void)hipFree(*p);
  *p = nullptr;
  *have = 0;
  hipError_t e = hipMalloc(p, (size_t)std::max<int64_t>(need, 16));
  if (e != hipSuccess) {
    *p = nullptr;
    return c->fail(SLF_ENOMEM, "hipMalloc(%lld): %s", (long long)need, hipGetErrorString(e));
  }
  *have = need;
  return SLF_OK;
}

}  // namespace
}  // namespace slf

using namespace slf;

extern "C" {

int slf_segment(slf_ctx *c, int view, int gw, int gh, int iterations, float compactness) {
  if (!c) return SLF_EINVAL;
  if (int rc = check_idle(c)) return rc;
  if (view < 0 || view >= c->V) return c->fail(SLF_EINVAL, "view %d out of range", view);
  ViewHost &h = c->vh[view];
  if (!h.has_img) return c->fail(SLF_ESTATE, "view %d has no image", view);
  if (gw < 1 || gh < 1 || gw > h.W || gh > h.H || (int64_t)gw * gh > (1 << 24))
    return c->fail(SLF_EINVAL, "grid %d x %d invalid for a %d x %d image", gw, gh, h.W, h.H);
  if (iterations < 1) return c->fail(SLF_EINVAL, "iterations must be >= 1");
  if (!(compactness >= 0.f) || !std::isfinite(compactness)) return c->fail(SLF_EINVAL, "compactness must be >= 0");
  HIP_OR_FAIL(c, hipSetDevice(c->device));
  const int W = h.W, H = h.H, K = gw * gh;
  const long long n = (long long)W * H;
  int rc;
  if ((rc = grow(c, &c->d_slic_cen, &c->slic_cen_bytes, 5 * sizeof(float) * (int64_t)K))) return rc;
  if ((rc = grow(c, &c->d_slic_best, &c->slic_best_bytes, sizeof(unsigned long long) * (int64_t)K))) return rc;
  if ((rc = grow(c, &c->d_slic_work, &c->slic_work_bytes, 3 * sizeof(int) * (int64_t)n))) return rc;
  int64_t pix = 0;
  for (int v = 0; v < view; ++v) pix += (int64_t)c->vh[v].W * c->vh[v].H;
  const uint8_t *rgb = c->d_rgb + 3 * pix;
  int *out = c->d_labels + pix;
  float *cen = (float *)c->d_slic_cen;
  unsigned long long *best = (unsigned long long *)c->d_slic_best;
  int *wlab = (int *)c->d_slic_work, *parent = wlab + n, *csize = parent + n;
  // spatial weight (2.55 m)^2 gw gh / (W H): colours in 0..255, the same as 0..100 with m^2 / S^2
  const double m = 2.55 * (double)compactness;
  const float wsp = (float)(m * m * (double)gw * (double)gh / ((double)W * (double)H));
  const dim3 rows((W + 255) / 256, H);
  const unsigned nb = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(k_slic_init, dim3((K + 255) / 256), dim3(256), 0, c->stream, rgb, W, H, gw, gh, cen, best);
  for (int it = 0; it < iterations; ++it) {
    hipLaunchKernelGGL(k_slic_assign, rows, dim3(256), 0, c->stream, rgb, W, H, gw, gh, (const float *)cen, wsp, wlab);
    if (it + 1 < iterations)
      hipLaunchKernelGGL(k_slic_update, dim3((K + 3) / 4), dim3(256), 0, c->stream, rgb, (const int *)wlab, W, H, gw,
                         gh, cen);
  }
  hipLaunchKernelGGL(k_cc_init, dim3(nb), dim3(256), 0, c->stream, parent, csize, n);
  hipLaunchKernelGGL(k_cc_link, rows, dim3(256), 0, c->stream, (const int *)wlab, W, H, parent);
  hipLaunchKernelGGL(k_cc_flatten, dim3(nb), dim3(256), 0, c->stream, parent, csize, n);
  hipLaunchKernelGGL(k_cc_best, dim3(nb), dim3(256), 0, c->stream, (const int *)wlab, (const int *)parent,
                     (const int *)csize, best, n);
  hipLaunchKernelGGL(k_cc_final, dim3(nb), dim3(256), 0, c->stream, (const int *)wlab, (const int *)parent,
                     (const unsigned long long *)best, W, n, out);
  HIP_OR_FAIL(c, hipGetLastError());
  if (h.gw != gw || h.gh != gh) c->geom_dirty = true;
  h.gw = gw;
  h.gh = gh;
  h.has_lab = true;
  c->sp_dirty = true;
  return SLF_OK;
}

int slf_get_labels(slf_ctx *c, int view, int32_t *out, int64_t stride, int is_device) {
  if (!c) return SLF_EINVAL;
  if (int rc = check_idle(c)) return rc;
  if (view < 0 || view >= c->V) return c->fail(SLF_EINVAL, "view %d out of range", view);
  const ViewHost &h = c->vh[view];
  if (!h.has_lab) return c->fail(SLF_ESTATE, "view %d has no labels", view);
  if (!out) return c->fail(SLF_EINVAL, "out is NULL");
  if (stride < h.W) return c->fail(SLF_EINVAL, "row stride %lld < W", (long long)stride);
  HIP_OR_FAIL(c, hipSetDevice(c->device));
  int64_t pix = 0;
  for (int v = 0; v < view; ++v) pix += (int64_t)c->vh[v].W * c->vh[v].H;
  HIP_OR_FAIL(c, hipMemcpy2DAsync(out, sizeof(int32_t) * stride, c->d_labels + pix, sizeof(int) * h.W,
                                  sizeof(int) * h.W, h.H, is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                                  c->stream));
  if (!is_device) HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  return SLF_OK;
}

}  // extern "C"
