// HIP kernels for gfx950: superpixel setup, plane sweep (TSSD), refinement
// energy, depth readout.  One wavefront (64 lanes) owns one superpixel in the
// sweep and refinement; lanes stride over the superpixel's pixel list and
// partial sums are combined with a fixed butterfly, so results do not depend
// on scheduling.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <limits.h>
#include <math.h>

#include <algorithm>
#include <type_traits>

#include "slf_internal.h"

namespace slf {

// Ring R8 around a grid cell (gy pointing down); entry j + 1 is adjacent to
// entry j.  Kept as 2-bit fields (offset + 1) of one constant, so a lane's
// offset is a shift and a mask rather than a table load.
constexpr int kRingDxTab[8] = {1, 1, 0, -1, -1, -1, 0, 1};
constexpr int kRingDyTab[8] = {0, 1, 1, 1, 0, -1, -1, -1};
constexpr unsigned pack_ring(const int *d) {
  unsigned p = 0;
  for (int j = 0; j < 8; ++j) p |= (unsigned)(d[j] + 1) << (2 * j);
  return p;
}
constexpr unsigned kRingDxBits = pack_ring(kRingDxTab);
constexpr unsigned kRingDyBits = pack_ring(kRingDyTab);
__device__ __forceinline__ int ring_dx(int j) { return (int)((kRingDxBits >> (2 * j)) & 3u) - 1; }
__device__ __forceinline__ int ring_dy(int j) { return (int)((kRingDyBits >> (2 * j)) & 3u) - 1; }

// ------------------------------------------------------------------ helpers

// SplitMix64 output function (Steele, Lea, Flood 2014).
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

// Inverse depth of sweep level k of superpixel s in view r (Sec. III-B):
// bin k of width dq starting at qmin, offset by a per-(view, superpixel,
// level) uniform draw taken from the top 24 bits of mix64.
__device__ __forceinline__ double level_q(uint64_t seed, int jitter, double qmin, double dq, int r, int s, int k) {
  double u = 0.0;
  if (jitter) {
    uint64_t key = seed ^ ((uint64_t)r << 48) ^ ((uint64_t)s << 24) ^ (uint64_t)k;
    u = (double)(mix64(key) >> 40) * (1.0 / 16777216.0);
  }
  return qmin + ((double)k + u) * dq;
}

// Wave reductions in a fixed order (so results do not depend on
// scheduling): DPP steps inside each row of 16 lanes (xor 1, xor 2, half-row
// mirror, row mirror), then the four row sums are read out and added.  The
// whole wave must be active; the result is uniform.
template <int CTRL>
__device__ __forceinline__ int dpp_i(int x) {
  return __builtin_amdgcn_update_dpp(0, x, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ float dpp_f(float x) {
  return __int_as_float(dpp_i<CTRL>(__float_as_int(x)));
}
constexpr int kDppXor1 = 0xB1;        // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;        // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141; // row_half_mirror
constexpr int kDppMirror = 0x140;     // row_mirror

__device__ __forceinline__ float rd_f(float x, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}

__device__ __forceinline__ float wave_sum(float x) {
  x += dpp_f<kDppXor1>(x);
  x += dpp_f<kDppXor2>(x);
  x += dpp_f<kDppHalfMirror>(x);
  x += dpp_f<kDppMirror>(x);
  return (rd_f(x, 0) + rd_f(x, 16)) + (rd_f(x, 32) + rd_f(x, 48));
}
// Sums of two values over the wave at once: v_permlane32_swap exchanges the
// upper half of a with the lower half of b, so one add leaves the 32-lane
// partial sums of a in lanes 0..31 and of b in lanes 32..63; the row steps
// then reduce both together.  Fixed order; the whole wave must be active.
__device__ __forceinline__ void wave_sum2(float a, float b, float &sa, float &sb) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  float x = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  x += dpp_f<kDppXor1>(x);
  x += dpp_f<kDppXor2>(x);
  x += dpp_f<kDppHalfMirror>(x);
  x += dpp_f<kDppMirror>(x);
  sa = rd_f(x, 0) + rd_f(x, 16);
  sb = rd_f(x, 32) + rd_f(x, 48);
}
__device__ __forceinline__ int wave_sum_i(int x) {
  x += dpp_i<kDppXor1>(x);
  x += dpp_i<kDppXor2>(x);
  x += dpp_i<kDppHalfMirror>(x);
  x += dpp_i<kDppMirror>(x);
  return (__builtin_amdgcn_readlane(x, 0) + __builtin_amdgcn_readlane(x, 16)) +
         (__builtin_amdgcn_readlane(x, 32) + __builtin_amdgcn_readlane(x, 48));
}
__device__ __forceinline__ long long wave_sum_ll(long long x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, kWave);
  return x;
}
// Reductions over the ring lanes 0..7, read from lane 0 (uniform result):
// quad xor 1, quad xor 2, half-row mirror.  Lanes 8.. do not take part; the
// whole wave must be active.
__device__ __forceinline__ float ring_min(float x) {
  x = fminf(x, dpp_f<kDppXor1>(x));
  x = fminf(x, dpp_f<kDppXor2>(x));
  x = fminf(x, dpp_f<kDppHalfMirror>(x));
  return rd_f(x, 0);
}
__device__ __forceinline__ float ring_max(float x) {
  x = fmaxf(x, dpp_f<kDppXor1>(x));
  x = fmaxf(x, dpp_f<kDppXor2>(x));
  x = fmaxf(x, dpp_f<kDppHalfMirror>(x));
  return rd_f(x, 0);
}
__device__ __forceinline__ float ring_sum(float x) {
  x += dpp_f<kDppXor1>(x);
  x += dpp_f<kDppXor2>(x);
  x += dpp_f<kDppHalfMirror>(x);
  return rd_f(x, 0);
}

// Makes earlier LDS writes of any lane of this wave visible to its later reads.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// 1 / x in FP64 from the hardware reciprocal and one Newton step (a few ulp;
// the plane geometry it serves is rounded to FP32 before any sample uses it).
__device__ __forceinline__ double rcp_d(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  return fma(r, fma(-x, r, 1.0), r);
}

// floor(x + 0.5) as an integer, the sum taken exactly (v_cvt_rpi_i32_f32; a
// NaN gives 0).  The compiler does not form this instruction by itself.
__device__ __forceinline__ int round_half_up(float x) {
  int r;
  asm("v_cvt_rpi_i32_f32 %0, %1" : "=v"(r) : "v"(x));
  return r;
}

// floor(x) as an integer in one instruction (v_cvt_flr_i32_f32; a NaN gives
// 0).  The compiler emits a floor and a conversion for (int)floorf(x).
__device__ __forceinline__ int floor_to_int(float x) {
  int r;
  asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(x));
  return r;
}

// Lane `l`'s value, uniform over the wave (l must be wave-uniform).
__device__ __forceinline__ float bcast(float x, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}

// ------------------------------------------------------------------ image texels
// Per view (W+1) x (H+1) entries, entry (x, y) at index y (W+1) + x, the last
// column and row replicated.  FP16 / FP32: the entry is the RGBA texel
// (x, y), 8 / 16 bytes, and a bilinear footprint takes one load per row.
// RGBA8: the entry is the texel pair (x, y), (x, y+1), 8 bytes, so entries
// (x0, y0) and (x0+1, y0), 16 contiguous bytes, hold all four taps and a
// sample takes a single load (the address path, not the bytes, limits the
// sweep's gathers).
size_t quad_bytes(int fmt) { return fmt == SLF_FMT_F32 ? 16 : 8; }
template <int FMT>
constexpr int kQuadBytes = FMT == SLF_FMT_F32 ? 16 : 8;

// An entry of a table that no kernel writes while it reads it (geometry,
// superpixel statistics, the state being read), accessed through the
// constant address space: at a wave-uniform index the compiler then always
// emits a scalar load, whatever it can prove about the stores around it.
template <class T>
__device__ __forceinline__ const T &ro_at(const T *p, int64_t i) {
  typedef const __attribute__((address_space(4))) T CT;
  return *(const T *)&((CT *)p)[i];
}

// Raw buffer resource over `bytes` bytes at p (gfx9-family descriptor word 3):
// loads past the end return 0.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(const void *p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, 0x00020000);
}

__device__ __forceinline__ uint4 load_u4(__amdgpu_buffer_rsrc_t rs, uint32_t off) {
  return __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(rs, (int)off, 0, 0));
}

// The four bilinear taps (x0, y0), (x0+1, y0), (x0, y0+1), (x0+1, y0+1) as
// 4 x RGB floats: two loads of two adjacent texels, `off` the byte offset
// of texel (x0, y0) and `row` the bytes of one texel row.
template <int FMT>
__device__ __forceinline__ void fetch_quad(__amdgpu_buffer_rsrc_t rs, uint32_t off, uint32_t row, float (&t)[12]);

template <>
__device__ __forceinline__ void fetch_quad<SLF_FMT_U8>(__amdgpu_buffer_rsrc_t rs, uint32_t off, uint32_t row,
                                                       float (&t)[12]) {
  const uint4 q = load_u4(rs, off);  // (x0, y0), (x0, y0+1), (x0+1, y0), (x0+1, y0+1)
  const uint32_t w[4] = {q.x, q.z, q.y, q.w};
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    t[3 * j + 0] = (float)(w[j] & 255u);
    t[3 * j + 1] = (float)((w[j] >> 8) & 255u);
    t[3 * j + 2] = (float)((w[j] >> 16) & 255u);
  }
}

template <>
__device__ __forceinline__ void fetch_quad<SLF_FMT_F16>(__amdgpu_buffer_rsrc_t rs, uint32_t off, uint32_t row,
                                                        float (&t)[12]) {
  const uint4 a = load_u4(rs, off), b = load_u4(rs, off + row);
  const uint32_t w[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    __half2 rg = *reinterpret_cast<const __half2 *>(&w[2 * j]);
    __half2 ba = *reinterpret_cast<const __half2 *>(&w[2 * j + 1]);
    t[3 * j + 0] = __low2float(rg);
    t[3 * j + 1] = __high2float(rg);
    t[3 * j + 2] = __low2float(ba);
  }
}

template <>
__device__ __forceinline__ void fetch_quad<SLF_FMT_F32>(__amdgpu_buffer_rsrc_t rs, uint32_t off, uint32_t row,
                                                        float (&t)[12]) {
  const uint32_t o[4] = {off, off + 16u, off + row, off + row + 16u};
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const float4 c = __builtin_bit_cast(float4, load_u4(rs, o[j]));
    t[3 * j + 0] = c.x;
    t[3 * j + 1] = c.y;
    t[3 * j + 2] = c.z;
  }
}

__global__ __launch_bounds__(256) void k_quads(const uint8_t *rgb, int W, int H, void *quads, int64_t quad_off,
                                               int fmt) {
  const int Wp = W + 1;
  const int64_t n = (int64_t)Wp * (H + 1);
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n) return;
  const int yr = (int)(idx / Wp);
  const int x = min((int)(idx % Wp), W - 1), y = min(yr, H - 1);  // replicated edge
  const uint8_t *c = rgb + 3 * ((int64_t)y * W + x);
  if (fmt == SLF_FMT_U8) {
    const uint8_t *d = rgb + 3 * ((int64_t)min(yr + 1, H - 1) * W + x);  // the texel below
    static_cast<uint2 *>(quads)[quad_off + idx] =
        make_uint2((uint32_t)c[0] | ((uint32_t)c[1] << 8) | ((uint32_t)c[2] << 16),
                   (uint32_t)d[0] | ((uint32_t)d[1] << 8) | ((uint32_t)d[2] << 16));
  } else if (fmt == SLF_FMT_F16) {
    __half2 rg = __floats2half2_rn((float)c[0], (float)c[1]);
    __half2 ba = __floats2half2_rn((float)c[2], 0.f);
    static_cast<uint2 *>(quads)[quad_off + idx] =
        make_uint2(*reinterpret_cast<uint32_t *>(&rg), *reinterpret_cast<uint32_t *>(&ba));
  } else {
    static_cast<float4 *>(quads)[quad_off + idx] = make_float4((float)c[0], (float)c[1], (float)c[2], 0.f);
  }
}

hipError_t launch_quads(int fmt, const uint8_t *rgb, int64_t, int W, int H, void *quads, int64_t quad_off,
                        hipStream_t st) {
  const int64_t n = (int64_t)(W + 1) * (H + 1);
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_quads, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, rgb, W, H, quads, quad_off, fmt);
  return hipGetLastError();
}

// ------------------------------------------------------------------ superpixel setup (a1)

__global__ __launch_bounds__(256) void k_sp_reset(const ViewDev *views, int V, int S, int *count, int4 *bbox,
                                                  int *sp_view, int *err) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g == 0) *err = 0;
  if (g >= S) return;
  int v = 0;
  while (v + 1 < V && views[v + 1].sp_off <= g) ++v;
  sp_view[g] = v;
  count[g] = 0;
  bbox[g] = make_int4(INT_MAX, INT_MAX, -1, -1);
}

// Pixel counts and bounding boxes.  One wave per tile of 16 x 4 pixels
// (lane = 16 row + column): for each distinct label of the tile, one lane
// adds the label's pixel count, column range and row range there, all read
// off the ballot mask of its pixels, with integer atomics (their order does
// not matter).  With lab16 non-null (K <= 65536) every pixel also stores its
// label as 16 bits.
constexpr int kCountTileW = 16, kCountTileH = kWave / kCountTileW;
__global__ __launch_bounds__(256) void k_sp_count(const int *labels, uint16_t *lab16, int W, int H, int K, int sp_off,
                                                  int *count, int4 *bbox, int *err) {
  const int lane = threadIdx.x & (kWave - 1);
  const int tiles_x = (W + kCountTileW - 1) / kCountTileW;
  const int tiles = tiles_x * ((H + kCountTileH - 1) / kCountTileH);
  const int tile = blockIdx.x * (blockDim.x / kWave) + (threadIdx.x >> 6);
  if (tile >= tiles) return;  // the whole wave
  const int x0 = (tile % tiles_x) * kCountTileW, y0 = (tile / tiles_x) * kCountTileH;
  const int x = x0 + (lane & (kCountTileW - 1)), y = y0 + lane / kCountTileW;
  int l = -1;
  if (x < W && y < H) {
    const int64_t idx = (int64_t)y * W + x;
    l = labels[idx];
    if (l < 0 || l >= K) {
      atomicOr(err, 1);
      l = -1;
    } else if (lab16) {
      lab16[idx] = (uint16_t)l;
    }
  }
  uint64_t pending = __ballot(l >= 0);
  while (pending) {
    const int leader = __ffsll((long long)pending) - 1;
    const int L = __shfl(l, leader, kWave);
    const uint64_t same = __ballot(l == L);
    pending &= ~same;
    if (lane == leader) {
      const uint32_t cols = (uint32_t)((same | same >> 16 | same >> 32 | same >> 48) & 0xffffu);
      int ylo = kCountTileH, yhi = -1;
      for (int r = 0; r < kCountTileH; ++r)
        if ((same >> (kCountTileW * r)) & 0xffffull) {
          ylo = min(ylo, r);
          yhi = r;
        }
      const int g = sp_off + L;
      int *b = reinterpret_cast<int *>(bbox + g);
      atomicAdd(count + g, __popcll(same));
      atomicMin(b + 0, x0 + __ffs(cols) - 1);
      atomicMin(b + 1, y0 + ylo);
      atomicMax(b + 2, x0 + 31 - __clz(cols));
      atomicMax(b + 3, y0 + yhi);
    }
  }
}

// Exclusive scan of count[0..S) into off[0..S], 4096 items per block.
constexpr int kScanThreads = 1024, kScanItems = 4;

__device__ int block_excl_scan(int x, int *sh, int *total) {
  const int t = threadIdx.x;
  sh[t] = x;
  __syncthreads();
  for (int o = 1; o < kScanThreads; o <<= 1) {
    const int y = t >= o ? sh[t - o] : 0;
    __syncthreads();
    sh[t] += y;
    __syncthreads();
  }
  const int incl = sh[t];
  *total = sh[kScanThreads - 1];
  __syncthreads();
  return incl - x;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_local(const int *in, int *out, int *blocksum, int n) {
  __shared__ int sh[kScanThreads];
  const int64_t base = (int64_t)blockIdx.x * kScanThreads * kScanItems + (int64_t)threadIdx.x * kScanItems;
  int v[kScanItems], s = 0;
  for (int j = 0; j < kScanItems; ++j) {
    v[j] = base + j < n ? in[base + j] : 0;
    s += v[j];
  }
  int total;
  int run = block_excl_scan(s, sh, &total);
  for (int j = 0; j < kScanItems; ++j) {
    if (base + j < n) out[base + j] = run;
    run += v[j];
  }
  if (threadIdx.x == 0) blocksum[blockIdx.x] = total;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_top(int *blocksum, int nb, int *out_total) {
  __shared__ int sh[kScanThreads];
  const int base = threadIdx.x * kScanItems;
  int v[kScanItems], s = 0;
  for (int j = 0; j < kScanItems; ++j) {
    v[j] = base + j < nb ? blocksum[base + j] : 0;
    s += v[j];
  }
  int total;
  int run = block_excl_scan(s, sh, &total);
  for (int j = 0; j < kScanItems; ++j) {
    if (base + j < nb) blocksum[base + j] = run;
    run += v[j];
  }
  if (threadIdx.x == 0) *out_total = total;
}

__global__ __launch_bounds__(256) void k_scan_add(int *out, const int *blocksum, int n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] += blocksum[i / (kScanThreads * kScanItems)];
}

// One wavefront per superpixel scans its bounding box in raster order and
// appends matching pixels with a ballot prefix, so every pixel list is in
// raster order and the build is deterministic.  Also computes area,
// centroid and mean colour (Sec. III-C-1: superpixel colour = mean colour).
__global__ __launch_bounds__(kBlock) void k_sp_fill(const ViewDev *views, const int *labels, const uint8_t *rgb,
                                                   int S, const int *sp_view, const int *count, const int4 *bbox,
                                                   const int *px_off, PixEntry *px, int *area, float2 *centroid,
                                                   double2 *centroid_d, float4 *colour, int *err) {
  const int lane = threadIdx.x & (kWave - 1);
  const int g = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  if (g >= S) return;
  const int v = sp_view[g];
  const ViewDev &vw = views[v];
  const int s = g - vw.sp_off;
  const int cnt = count[g];
  if (cnt == 0) {
    if (lane == 0) {
      area[g] = 0;
      centroid[g] = make_float2(0.f, 0.f);
      centroid_d[g] = make_double2(0.0, 0.0);
      colour[g] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    return;
  }
  const int4 box = bbox[g];
  const int base = px_off[g];
  const int *lab = labels + vw.pix_off;
  const uint8_t *img = rgb + 3 * vw.pix_off;
  int written = 0;
  long long sx = 0, sy = 0;
  int sr = 0, sg = 0, sb = 0;
  // pixel (x, y) of the box, taken when `in`; the lanes of one call visit
  // pixels in raster order, so the ballot prefix appends in raster order
  auto visit = [&](int x, int y, bool in) {
    const int64_t pidx = (int64_t)y * vw.W + x;
    const bool m = in && lab[pidx] == s;
    const uint64_t mask = __ballot(m);
    if (m) {
      const int pre = __popcll(mask & ((1ull << lane) - 1ull));
      const uint8_t *c = img + 3 * pidx;
      const uint32_t rgba = (uint32_t)c[0] | ((uint32_t)c[1] << 8) | ((uint32_t)c[2] << 16);
      if (written + pre < cnt) px[base + written + pre] = make_uint2((uint32_t)x | ((uint32_t)y << 16), rgba);
      sx += x;
      sy += y;
      sr += c[0];
      sg += c[1];
      sb += c[2];
    }
    written += __popcll(mask);
  };
  // the box as one raster sequence of bw bh pixels, 64 per pass: lane j of
  // a pass takes pixel i0 + j at (xo, yo), advanced by 64 pixels each pass
  const int bw = box.z - box.x + 1;
  const int64_t n = (int64_t)bw * (box.w - box.y + 1);
  const int dq = kWave / bw, dr = kWave % bw;
  int xo = lane % bw, yo = lane / bw;
  for (int64_t i0 = 0; i0 < n; i0 += kWave) {
    visit(box.x + xo, box.y + yo, i0 + lane < n);
    xo += dr;
    yo += dq;
    if (xo >= bw) {  // xo < 2 bw here
      xo -= bw;
      ++yo;
    }
  }
  sx = wave_sum_ll(sx);
  sy = wave_sum_ll(sy);
  sr = wave_sum_i(sr);
  sg = wave_sum_i(sg);
  sb = wave_sum_i(sb);
  if (lane == 0) {
    if (written != cnt) atomicOr(err, 2);
    area[g] = cnt;
    const double n = (double)cnt;
    centroid_d[g] = make_double2((double)sx / n, (double)sy / n);
    centroid[g] = make_float2((float)((double)sx / n), (float)((double)sy / n));
    const float cr = (float)(sr / (255.0 * n)), cg = (float)(sg / (255.0 * n)), cb = (float)(sb / (255.0 * n));
    colour[g] = make_float4(cr, cg, cb, fmaf(cb, cb, fmaf(cg, cg, cr * cr)));  // w = |C|^2 (eq. 7's weight)
  }
}

hipError_t launch_sp_build(const ViewDev *views_d, const ViewDev *views_h, int V, const int *labels, uint16_t *lab16,
                           const uint8_t *rgb, int S, int *count, int4 *bbox, int *px_off, int *scan_tmp,
                           PixEntry *px, int *area, float2 *centroid, double2 *centroid_d, float4 *colour,
                           int *sp_view, int *err, hipStream_t st) {
  if (S <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_sp_reset, dim3((S + 255) / 256), dim3(256), 0, st, views_d, V, S, count, bbox, sp_view, err);
  for (int v = 0; v < V; ++v) {
    const ViewDev &vw = views_h[v];
    const int64_t tiles = (int64_t)((vw.W + kCountTileW - 1) / kCountTileW) * ((vw.H + kCountTileH - 1) / kCountTileH);
    hipLaunchKernelGGL(k_sp_count, dim3((unsigned)((tiles + 3) / 4)), dim3(256), 0, st, labels + vw.pix_off,
                       lab16 ? lab16 + vw.pix_off : nullptr, vw.W, vw.H, vw.gw * vw.gh, vw.sp_off, count, bbox, err);
  }
  const int per = kScanThreads * kScanItems;
  const int nb = (S + per - 1) / per;
  if (nb > per) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_scan_local, dim3(nb), dim3(kScanThreads), 0, st, count, px_off, scan_tmp, S);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanThreads), 0, st, scan_tmp, nb, px_off + S);
  hipLaunchKernelGGL(k_scan_add, dim3((S + 255) / 256), dim3(256), 0, st, px_off, scan_tmp, S);
  hipLaunchKernelGGL(k_sp_fill, dim3((S + kWavesPerBlock - 1) / kWavesPerBlock), dim3(kBlock), 0, st, views_d,
                     labels, rgb, S, sp_view, count, bbox, px_off, px, area, centroid, centroid_d, colour, err);
  return hipGetLastError();
}

// ------------------------------------------------------------------ sweep sample
// Byte offset of view i's texels in the texel array (which the host keeps
// under 4 GiB, so that one wave-uniform buffer resource covers every view).
template <int FMT>
__device__ __forceinline__ uint32_t quad_base(const ViewDev &vi) {
  return (uint32_t)vi.quad_off * (uint32_t)kQuadBytes<FMT>;
}

// Where the samples in one neighbour view land.  Positions are taken relative
// to an integer pixel (X0, Y0) of that view (0 for absolute positions), so
// that the FP32 per-sample arithmetic works on small numbers at any image
// size: the image [0, W-1] x [0, H-1] is [xlo, xhi] x [ylo, yhi] in these
// coordinates, and vbase is the byte offset of texel entry (X0, Y0), modulo
// 2^32 like every offset formed from it (the texel array is below 4 GiB).
struct SampleFrame {
  float xlo, xhi, ylo, yhi;
  int Wi;  // view width: a texel row holds W + 1 entries
  uint32_t vbase;
};

template <int FMT>
__device__ __forceinline__ SampleFrame frame_at(const ViewDev &vi, int X0, int Y0) {
  SampleFrame f;
  f.xlo = (float)(-X0);
  f.xhi = (float)(vi.W - 1 - X0);
  f.ylo = (float)(-Y0);
  f.yhi = (float)(vi.H - 1 - Y0);
  f.Wi = vi.W;
  f.vbase = quad_base<FMT>(vi) + ((uint32_t)Y0 * (uint32_t)(vi.W + 1) + (uint32_t)X0) * (uint32_t)kQuadBytes<FMT>;
  return f;
}

// Byte offset of texel entry (X0 + x0, Y0 + y0).  |x0|, |y0| < 2^16 and
// W + 1 <= 2^16, so the signed 24-bit multiply (full rate) forms the index;
// its low 32 bits are all the modular offset needs.
template <int FMT>
__device__ __forceinline__ uint32_t texel_offset(const SampleFrame &f, int x0, int y0) {
  return f.vbase + (uint32_t)(__mul24(y0, f.Wi + 1) + x0) * (uint32_t)kQuadBytes<FMT>;
}

// One px-view sample of eq. (1): homogeneous projection (x, y, w), bilinear
// RGB of the neighbour image, SSD against the reference colour, truncation.
// Samples behind the camera or outside [0, W-1] x [0, H-1] cost T.  The texel
// address is clamped into the image whatever the coordinates, so the load is
// always in bounds and issued unconditionally.
//
// With check = false the caller guarantees w > 0 and a position inside the
// image (see sweep_levels): the clamp would be the identity, so it and the
// test are skipped and the result is the same.
template <int FMT>
__device__ __forceinline__ float tssd_sample(float x, float y, float w, const SampleFrame &f,
                                             __amdgpu_buffer_rsrc_t quads, float r0, float g0, float b0, float T,
                                             bool check = true) {
  const float rw = rcp(w);
  const float xs = x * rw, ys = y * rw;
  // Clamp into the image; the sample counts only if unclamped (a NaN fails
  // the equality, and converts to entry (X0, Y0), so the load stays in bounds).
  const float xc = check ? __builtin_amdgcn_fmed3f(xs, f.xlo, f.xhi) : xs;
  const float yc = check ? __builtin_amdgcn_fmed3f(ys, f.ylo, f.yhi) : ys;
  const bool in = !check || ((w > 0.f) & (xc == xs) & (yc == ys));
  // Taps at floor(x) and floor(x)+1 with weight fract(x); at x = W-1 the
  // replicated column has weight 0, which equals clamping the left tap to W-2.
  const int x0 = floor_to_int(xc), y0 = floor_to_int(yc);
  const float fx = __builtin_amdgcn_fractf(xc), fy = __builtin_amdgcn_fractf(yc);
  float t[12];
  const uint32_t row = (uint32_t)(f.Wi + 1) * (uint32_t)kQuadBytes<FMT>;
  fetch_quad<FMT>(quads, texel_offset<FMT>(f, x0, y0), row, t);
  // bilinear weights of the four taps (FP16 taps feed mixed-precision FMAs directly)
  const float ofx = 1.f - fx, ofy = 1.f - fy;
  const float w00 = ofx * ofy, w10 = fx * ofy, w01 = ofx * fy, w11 = fx * fy;
  float b[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) b[c] = fmaf(w11, t[9 + c], fmaf(w01, t[6 + c], fmaf(w10, t[3 + c], w00 * t[c])));
  const float d0 = r0 - b[0], d1 = g0 - b[1], d2 = b0 - b[2];
  const float ssd = fmaf(d2, d2, fmaf(d1, d1, d0 * d0));
  return in ? fminf(ssd, T) : T;
}

// The RGBA8 sample in two phases, so that a caller can issue the texel
// loads of several samples before it waits for the first: `fetch` projects,
// clamps and issues the 16-byte load, `finish` interpolates and scores.
// fetch + finish performs exactly the operations of tssd_sample<SLF_FMT_U8>.
struct U8Tap {
  uint4 q;
  float fx, fy;
  bool in;
};

__device__ __forceinline__ U8Tap u8_fetch(float x, float y, float w, const SampleFrame &f,
                                          __amdgpu_buffer_rsrc_t quads, bool check) {
  U8Tap t;
  const float rw = rcp(w);
  const float xs = x * rw, ys = y * rw;
  const float xc = check ? __builtin_amdgcn_fmed3f(xs, f.xlo, f.xhi) : xs;
  const float yc = check ? __builtin_amdgcn_fmed3f(ys, f.ylo, f.yhi) : ys;
  t.in = !check || ((w > 0.f) & (xc == xs) & (yc == ys));
  const int x0 = floor_to_int(xc), y0 = floor_to_int(yc);
  t.fx = __builtin_amdgcn_fractf(xc);
  t.fy = __builtin_amdgcn_fractf(yc);
  t.q = load_u4(quads, texel_offset<SLF_FMT_U8>(f, x0, y0));
  return t;
}

__device__ __forceinline__ float u8_finish(const U8Tap &tp, float r0, float g0, float b0, float T) {
  const uint32_t wd[4] = {tp.q.x, tp.q.z, tp.q.y, tp.q.w};  // (x0, y0), (x0+1, y0), (x0, y0+1), (x0+1, y0+1)
  float t[12];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    t[3 * j + 0] = (float)(wd[j] & 255u);
    t[3 * j + 1] = (float)((wd[j] >> 8) & 255u);
    t[3 * j + 2] = (float)((wd[j] >> 16) & 255u);
  }
  const float ofx = 1.f - tp.fx, ofy = 1.f - tp.fy;
  const float w00 = ofx * ofy, w10 = tp.fx * ofy, w01 = ofx * tp.fy, w11 = tp.fx * tp.fy;
  float b[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) b[c] = fmaf(w11, t[9 + c], fmaf(w01, t[6 + c], fmaf(w10, t[3 + c], w00 * t[c])));
  const float d0 = r0 - b[0], d1 = g0 - b[1], d2 = b0 - b[2];
  const float ssd = fmaf(d2, d2, fmaf(d1, d1, d0 * d0));
  return tp.in ? fminf(ssd, T) : T;
}

template <>
__device__ __forceinline__ float tssd_sample<SLF_FMT_U8>(float x, float y, float w, const SampleFrame &f,
                                                         __amdgpu_buffer_rsrc_t quads, float r0, float g0, float b0,
                                                         float T, bool check) {
  return u8_finish(u8_fetch(x, y, w, f, quads, check), r0, g0, b0, T);
}

// FP16 texels: each tap enters an FMA as an FP16 operand widened exactly
// inside the instruction (v_fma_mix_f32), so the interpolation is the FP32
// one with no separate conversions.  Two phases as for RGBA8 (two 16-byte
// loads, one per texel row).
struct F16Tap {
  uint4 lo, hi;
  float fx, fy;
  bool in;
};

__device__ __forceinline__ F16Tap f16_fetch(float x, float y, float w, const SampleFrame &f,
                                            __amdgpu_buffer_rsrc_t quads, bool check) {
  F16Tap t;
  const float rw = rcp(w);
  const float xs = x * rw, ys = y * rw;
  const float xc = check ? __builtin_amdgcn_fmed3f(xs, f.xlo, f.xhi) : xs;
  const float yc = check ? __builtin_amdgcn_fmed3f(ys, f.ylo, f.yhi) : ys;
  t.in = !check || ((w > 0.f) & (xc == xs) & (yc == ys));
  const int x0 = floor_to_int(xc), y0 = floor_to_int(yc);
  t.fx = __builtin_amdgcn_fractf(xc);
  t.fy = __builtin_amdgcn_fractf(yc);
  const uint32_t off = texel_offset<SLF_FMT_F16>(f, x0, y0);
  t.lo = load_u4(quads, off);
  t.hi = load_u4(quads, off + (uint32_t)(f.Wi + 1) * 8u);
  return t;
}

__device__ __forceinline__ float f16_finish(const F16Tap &tp, float r0, float g0, float b0, float T) {
  const uint4 lo = tp.lo, hi = tp.hi;
  const float fx = tp.fx, fy = tp.fy;
  const bool in = tp.in;
  typedef _Float16 h2 __attribute__((ext_vector_type(2)));
  const h2 rg00 = __builtin_bit_cast(h2, lo.x), b00 = __builtin_bit_cast(h2, lo.y);
  const h2 rg10 = __builtin_bit_cast(h2, lo.z), b10 = __builtin_bit_cast(h2, lo.w);
  const h2 rg01 = __builtin_bit_cast(h2, hi.x), b01 = __builtin_bit_cast(h2, hi.y);
  const h2 rg11 = __builtin_bit_cast(h2, hi.z), b11 = __builtin_bit_cast(h2, hi.w);
  const float ofx = 1.f - fx, ofy = 1.f - fy;
  const float w00 = ofx * ofy, w10 = fx * ofy, w01 = ofx * fy, w11 = fx * fy;
  // w00 t00 as an FMA with a +0 addend (taps and weights are >= 0, so it
  // equals the product) keeps the first tap in the mixed-precision form too
  const float br = fmaf(w11, (float)rg11.x, fmaf(w01, (float)rg01.x, fmaf(w10, (float)rg10.x, fmaf(w00, (float)rg00.x, 0.f))));
  const float bg = fmaf(w11, (float)rg11.y, fmaf(w01, (float)rg01.y, fmaf(w10, (float)rg10.y, fmaf(w00, (float)rg00.y, 0.f))));
  const float bb = fmaf(w11, (float)b11.x, fmaf(w01, (float)b01.x, fmaf(w10, (float)b10.x, fmaf(w00, (float)b00.x, 0.f))));
  const float d0 = r0 - br, d1 = g0 - bg, d2 = b0 - bb;
  const float ssd = fmaf(d2, d2, fmaf(d1, d1, d0 * d0));
  return in ? fminf(ssd, T) : T;
}

template <>
__device__ __forceinline__ float tssd_sample<SLF_FMT_F16>(float x, float y, float w, const SampleFrame &f,
                                                          __amdgpu_buffer_rsrc_t quads, float r0, float g0, float b0,
                                                          float T, bool check) {
  return f16_finish(f16_fetch(x, y, w, f, quads, check), r0, g0, b0, T);
}

// levels whose texel loads are issued together (RGBA8: 4 loads; FP16, two loads each: 8)
#ifndef SLF_SWEEP_BATCH
#define SLF_SWEEP_BATCH 4
#endif
#ifndef SLF_SWEEP_BATCH_F16
#define SLF_SWEEP_BATCH_F16 4
#endif
template <int KC>
constexpr int kSweepBatchOf = KC < SLF_SWEEP_BATCH ? KC : SLF_SWEEP_BATCH;
template <int KC>
constexpr int kSweepBatchF16Of = KC < SLF_SWEEP_BATCH_F16 ? KC : SLF_SWEEP_BATCH_F16;

// acc[k] += the sample of one pixel in one view at levels q[0..KC): the
// homogeneous position is (ax, ay, aw) + q (bx, by, bw).  For RGBA8 and FP16
// texels the loads of a batch of levels are issued before the first is
// consumed (with one sample after another the compiler waits on each load
// in the bounds-tested form); the arithmetic of each sample is unchanged.
template <int FMT, int KC>
__device__ __forceinline__ void sample_levels(const float (&q)[KC], float (&acc)[KC], float ax, float ay, float aw,
                                              float bx, float by, float bw, const SampleFrame &f,
                                              __amdgpu_buffer_rsrc_t qrs, float r0, float g0, float b0, float T,
                                              bool check) {
  if constexpr (FMT == SLF_FMT_U8 || FMT == SLF_FMT_F16) {
    constexpr int B = FMT == SLF_FMT_U8 ? kSweepBatchOf<KC> : kSweepBatchF16Of<KC>;
#pragma unroll
    for (int k0 = 0; k0 < KC; k0 += B) {
      if constexpr (FMT == SLF_FMT_U8) {
        U8Tap t[B];
#pragma unroll
        for (int j = 0; j < B; ++j)
          t[j] = u8_fetch(fmaf(q[k0 + j], bx, ax), fmaf(q[k0 + j], by, ay), fmaf(q[k0 + j], bw, aw), f, qrs, check);
#pragma unroll
        for (int j = 0; j < B; ++j) acc[k0 + j] += u8_finish(t[j], r0, g0, b0, T);
      } else {
        F16Tap t[B];
#pragma unroll
        for (int j = 0; j < B; ++j)
          t[j] = f16_fetch(fmaf(q[k0 + j], bx, ax), fmaf(q[k0 + j], by, ay), fmaf(q[k0 + j], bw, aw), f, qrs, check);
#pragma unroll
        for (int j = 0; j < B; ++j) acc[k0 + j] += f16_finish(t[j], r0, g0, b0, T);
      }
    }
  } else {
#pragma unroll
    for (int kk = 0; kk < KC; ++kk)
      acc[kk] += tssd_sample<FMT>(fmaf(q[kk], bx, ax), fmaf(q[kk], by, ay), fmaf(q[kk], bw, aw), f, qrs, r0, g0, b0, T,
                                  check);
  }
}

constexpr int kXcds = 8;  // MI355X: 8 accelerator complex dies, each with its own L2
static_assert(kPoolQueues == kXcds, "one claim queue per XCD");

// Persistent sweep launch over superpixels 0..S-1: they are cut into kXcds
// contiguous queues (raster order within a view); the waves of workgroup b,
// which the hardware places on XCD b mod 8, drain queue b mod 8 first, so
// each XCD's gathers stay inside its own L2, and then steal from the other
// queues.  One claim is one superpixel, so superpixels of uneven cost (area,
// chunks stopped early by the level bound) balance across the chip, and
// every wave exits once all queues are empty.  The same counters serve the
// pooled kernel below.
__global__ void k_pool_reset(int *counters) {
  if (threadIdx.x < kPoolQueues) counters[threadIdx.x * kPoolCounterStride] = 0;
}

// Claims the next index of a queue for the whole wave.  Every lane takes
// part in the atomic (lane 0 adds one, the others zero) and the wave takes
// the first lane's old value.  A form with the atomic under `lane == 0`
// lets the compiler send lanes 1..63 past it on their own (for them it adds
// nothing), which splits the wave across the claim and, where the caller's
// body also branches on lane 0, leaves those lanes re-claiming the same
// index without end.
__device__ __forceinline__ int claim(int *next) {
  const int lane = threadIdx.x & (kWave - 1);
  return __builtin_amdgcn_readfirstlane(atomicAdd(next, lane == 0 ? 1 : 0));
}

template <class F>
__device__ __forceinline__ void for_each_claimed(const int S, int *counters, F &&body) {
  const int home = (int)(blockIdx.x % kPoolQueues);
  for (int k = 0; k < kPoolQueues; ++k) {
    const int q = (home + k) % kPoolQueues;
    const int begin = (int)((int64_t)S * q / kPoolQueues), end = (int)((int64_t)S * (q + 1) / kPoolQueues);
    int *next = counters + q * kPoolCounterStride;
    for (;;) {
      const int g = begin + claim(next);
      if (g >= end) break;
      body(g);
    }
  }
}

// Workgroups of a persistent launch over S items: as many as are resident at
// once on every CU, but no more than one wave per item (rounded up to whole
// multiples of kXcds, so each XCD gets its share of workgroups).
static int persistent_blocks(const void *kernel, int n_cu, int S) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kBlock, 0) != hipSuccess || per_cu < 1) per_cu = 1;
  const int resident = per_cu * (n_cu > 0 ? n_cu : 1);
  const int needed = ((S + kWavesPerBlock - 1) / kWavesPerBlock + kXcds - 1) / kXcds * kXcds;
  return std::max(1, std::min(resident, needed));
}

// ------------------------------------------------------------------ plane sweep (a2-a5)
// Level-chunked: each lane takes (neighbour view, pixel) pairs of the
// superpixel; for a pair, a = A p~ is formed once and the KC levels of the
// chunk give (x, y, w) = a + q_k b (the fronto-parallel plane at inverse
// depth q_k has inverse-depth row (0, 0, q_k)).  Per-level lane partials are
// summed by a butterfly and the running argmin keeps the smallest level on
// ties.
// Costs of levels [k_begin, k_end) of superpixel g: the smallest (ties: the
// lowest level) and the second smallest, uniform over the wave.
// Every kBoundCheck pixel passes the chunk's partial costs are compared with
// a complete level's cost: the second best when a.exact_margin is set (once
// two levels are complete), else the best.  Each sample costs >= 0, so a
// partial cost bounds the level's cost from below (per lane the sums only
// grow, and FP addition is monotone, so this holds for the rounded sums as
// well); when every level of the chunk is bounded above the reference
// (times kBoundMargin, a further margin) none of them can be the best, nor
// tie with it, nor (with exact_margin) be the second best, and the chunk
// stops.  The levels that finish are summed exactly as without the bound, so
// the level, plane and cost are unchanged; without exact_margin the second
// best is taken over the levels that finished, an upper bound of the exact
// one.  *computed receives the px-view samples computed for levels below
// k_end.
#ifndef SLF_BOUND_CHECK
#define SLF_BOUND_CHECK 2
#endif
constexpr int kBoundCheck = SLF_BOUND_CHECK;
constexpr float kBoundMargin = 1.00001f;

// Sweep constants of one (superpixel, neighbour view) pair.  Pixel offsets
// (du, dv) from the centre (ub, vb) of the superpixel's bounding box go in,
// and positions relative to (X0, Y0), the pixel nearest the box centre's
// projection at the middle of the inverse-depth range, come out:
//   x - X0 = (h0 du + h1 dv + h2 + q bx) / (h6 du + h7 dv + h8 + q bw),
// and y - Y0 likewise with h3..h5 and by.  Row x is row x of A minus X0 times
// row w (row y with Y0), moved to (ub, vb); the rows are composed in FP64 from
// the pair's A and b and then rounded, so every FP32 quantity of a sample is
// of the size of the superpixel and its disparity range, not of the image.
struct alignas(16) SweepPair {
  float h[9];
  float b[3];
  SampleFrame f;
  int pad[2];
};

// The pixel of view i nearest (hx, hy) / hw, clamped into the image; (0, 0)
// unless hw > 0.  Any pixel near the projection serves as a re-centring
// pixel, so FP32 suffices (a NaN fails both tests and gives 0).
__device__ __forceinline__ void near_pixel(double hx, double hy, double hw, const ViewDev &vi, int &X0, int &Y0) {
  X0 = Y0 = 0;
  if (hw > 0.0) {
    const float r = rcp((float)hw);
    const float cx = rintf((float)hx * r), cy = rintf((float)hy * r);
    X0 = cx > 0.f ? (cx < (float)(vi.W - 1) ? (int)cx : vi.W - 1) : 0;
    Y0 = cy > 0.f ? (cy < (float)(vi.H - 1) ? (int)cy : vi.H - 1) : 0;
  }
}

template <int FMT>
__device__ __forceinline__ SweepPair sweep_pair(const PairDev &pg, const ViewDev &vi, int ub, int vb, double qm) {
  const double hx = pg.A_d[0] * ub + pg.A_d[1] * vb + pg.A_d[2];
  const double hy = pg.A_d[3] * ub + pg.A_d[4] * vb + pg.A_d[5];
  const double hw = pg.A_d[6] * ub + pg.A_d[7] * vb + pg.A_d[8];
  int X0, Y0;
  near_pixel(hx + qm * pg.b_d[0], hy + qm * pg.b_d[1], hw + qm * pg.b_d[2], vi, X0, Y0);
  SweepPair p;
  p.h[0] = (float)(pg.A_d[0] - X0 * pg.A_d[6]);
  p.h[1] = (float)(pg.A_d[1] - X0 * pg.A_d[7]);
  p.h[2] = (float)(hx - X0 * hw);
  p.h[3] = (float)(pg.A_d[3] - Y0 * pg.A_d[6]);
  p.h[4] = (float)(pg.A_d[4] - Y0 * pg.A_d[7]);
  p.h[5] = (float)(hy - Y0 * hw);
  p.h[6] = (float)pg.A_d[6];
  p.h[7] = (float)pg.A_d[7];
  p.h[8] = (float)hw;
  p.b[0] = (float)(pg.b_d[0] - X0 * pg.b_d[2]);
  p.b[1] = (float)(pg.b_d[1] - Y0 * pg.b_d[2]);
  p.b[2] = (float)pg.b_d[2];
  p.f = frame_at<FMT>(vi, X0, Y0);
  p.pad[0] = p.pad[1] = 0;
  return p;
}

// The pairs of the superpixel a wave sweeps: the first kSweepPairsLds are
// composed once per superpixel, one per lane, into the wave's LDS; a
// superpixel with more neighbour views composes the others where a lane
// reaches them.
constexpr int kSweepPairsLds = kWave;
struct SweepPairs {
  const SweepPair *lds;
  const SweepArgs *a;
  const ViewDev *vw;
  int ub, vb;
  double qm;
  template <int FMT>
  __device__ __forceinline__ SweepPair at(int iv) const {
    if (iv < kSweepPairsLds) return lds[iv];
    const PairDev &pg = a->pairs[vw->pair_off + iv];
    return sweep_pair<FMT>(pg, a->views[pg.i], ub, vb, qm);
  }
};

// Chunk order.  Bounded against the best complete cost, a chunk stops early
// once a good level is known, so a coarse pre-pass first scores one level per
// chunk (its middle one) on every kCoarseStride-th pixel pass, and the chunks
// then run in increasing coarse cost (one byte per chunk in the wave's LDS).
// The order changes only which samples the bound skips: the tie rule below
// (a lower cost, or an equal one at a lower level) gives the level a pass in
// level order gives.  Returns false (level order) for fewer than 3 or more
// than 64 chunks, or fewer than 2 kCoarseStride pixel passes.  The pre-pass
// samples are added to *computed.
#ifndef SLF_COARSE_STRIDE
#define SLF_COARSE_STRIDE 8
#endif
constexpr int kCoarseStride = SLF_COARSE_STRIDE;  // 0: chunks in level order

template <int FMT, int KC>
__device__ __forceinline__ bool coarse_order(const SweepArgs &a, const int g, const int v, const int s,
                                             const ViewDev &vw, const int A, const int k_begin, const int k_end,
                                             const SweepPairs &pairs, uint8_t *order, uint64_t &computed) {
  const int lane = threadIdx.x & (kWave - 1);
  const int P = A * vw.n_pairs;
  const int n_pass = (P + kWave - 1) / kWave;
  const int n_chunks = (k_end - k_begin + KC - 1) / KC;
  if (kCoarseStride <= 0 || n_chunks < 3 || n_chunks > kWave || n_pass < 2 * kCoarseStride) return false;
  const int poff = a.px_off[g];
  const __amdgpu_buffer_rsrc_t qrs = buffer_rsrc(a.quads, a.quad_bytes);
  float mine = 0.f;  // lane c: coarse cost of chunk c
  for (int c0 = 0; c0 < n_chunks; c0 += KC) {
    float q[KC], acc[KC];
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
      const int cb = k_begin + min(c0 + kk, n_chunks - 1) * KC;
      q[kk] = (float)level_q(a.seed, a.jitter, a.qmin, a.dq, v, s, cb + min(KC / 2, k_end - cb - 1));
      acc[kk] = 0.f;
    }
    for (int it = 0; it < n_pass; it += kCoarseStride) {
      const int j = lane + it * kWave;
      if (j < P) {
        const int iv = j / A, p = j - iv * A;
        const SweepPair sp = pairs.at<FMT>(iv);
        const PixEntry e = a.px[poff + p];
        const float du = (float)((int)(e.x & 0xffffu) - pairs.ub), dv = (float)((int)(e.x >> 16) - pairs.vb);
        const float r0 = (float)(e.y & 255u), g0 = (float)((e.y >> 8) & 255u), b0 = (float)((e.y >> 16) & 255u);
        const float ax = fmaf(sp.h[0], du, fmaf(sp.h[1], dv, sp.h[2]));
        const float ay = fmaf(sp.h[3], du, fmaf(sp.h[4], dv, sp.h[5]));
        const float aw = fmaf(sp.h[6], du, fmaf(sp.h[7], dv, sp.h[8]));
        sample_levels<FMT, KC>(q, acc, ax, ay, aw, sp.b[0], sp.b[1], sp.b[2], sp.f, qrs, r0, g0, b0, a.T255, true);
      }
    }
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
      const float sum = wave_sum(acc[kk]);
      if (lane == c0 + kk) mine = sum;
    }
    const int used = (n_pass + kCoarseStride - 1) / kCoarseStride, last = (used - 1) * kCoarseStride;
    computed += (uint64_t)((used - 1) * kWave + min(kWave, P - last * kWave)) * (uint64_t)min(KC, n_chunks - c0);
  }
  // rank of chunk `lane` in increasing coarse cost (ties: lower chunk first)
  int rank = 0;
  for (int c = 0; c < n_chunks; ++c) {
    const float other = __shfl(mine, c, kWave);
    rank += (other < mine || (other == mine && c < lane)) ? 1 : 0;
  }
  if (lane < n_chunks) order[rank] = (uint8_t)lane;
  wave_lds_sync();
  return true;
}

template <int FMT, int KC>
__device__ __forceinline__ void sweep_levels(const SweepArgs &a, const int g, const int v, const int s,
                                             const ViewDev &vw, const int A, const int k_begin, const int k_end,
                                             float &best, float &second, int &kbest, uint64_t &computed,
                                             uint32_t &scored) {
  const int lane = threadIdx.x & (kWave - 1);
  const int N = vw.n_pairs;
  const int P = A * N;
  const int poff = a.px_off[g];
  const int4 bb = ro_at(a.bbox, g);  // pixel bounding box (x0, y0, x1, y1)
  __shared__ uint8_t s_order[kWavesPerBlock][kWave];  // chunk order of each wave of the workgroup
  __shared__ SweepPair s_pairs[kWavesPerBlock][kSweepPairsLds];  // pair constants of each wave's superpixel
  uint8_t *order = s_order[threadIdx.x >> 6];
  SweepPair *lds_pairs = s_pairs[threadIdx.x >> 6];
  const SweepPairs pairs{lds_pairs, &a, &vw, (bb.x + bb.z) >> 1, (bb.y + bb.w) >> 1,
                         a.qmin + a.dq * (0.5 * (double)a.levels)};
  wave_lds_sync();  // the previous superpixel's reads are done
  if (lane < min(N, kSweepPairsLds)) {
    const PairDev &pg = a.pairs[vw.pair_off + lane];
    lds_pairs[lane] = sweep_pair<FMT>(pg, a.views[pg.i], pairs.ub, pairs.vb, pairs.qm);
  }
  wave_lds_sync();
  const bool ordered = coarse_order<FMT, KC>(a, g, v, s, vw, A, k_begin, k_end, pairs, order, computed);
  const int n_chunks = (k_end - k_begin + KC - 1) / KC;
  for (int ci = 0; ci < n_chunks; ++ci) {
    const int k0 = k_begin + KC * (ordered ? __builtin_amdgcn_readfirstlane((int)order[ci]) : ci);
    float q[KC];
#pragma unroll
    for (int j = 0; j < KC; ++j) q[j] = (float)level_q(a.seed, a.jitter, a.qmin, a.dq, v, s, k0 + j);
    // Lane j < N: does every sample of neighbour view j at this chunk's
    // levels land inside the image, at least half a pixel from its border,
    // with w > 0?  x, y, w are affine in the pixel for fixed q and in q for
    // fixed pixel, and every level of the chunk (also one past `levels`)
    // has q in [q_min + k0 dq, q_min + (k0 + KC) dq]: so w is smallest, and
    // the image positions (a projective map of the box, moving monotonically
    // along epipolar lines as q changes) are extreme, at the 8 corners of
    // box x q-range.  The test takes absolute positions from the pair table
    // in FP32; they and the re-centred positions the samples use differ by
    // rounding of at most about 0.01 px at the largest image side, far below
    // the half-pixel margin.
    bool inner = false;
    if (lane < N) {
      const PairDev &pg = a.pairs[vw.pair_off + lane];
      const ViewDev &vi = a.views[pg.i];
      const float qlo = (float)(a.qmin + (double)k0 * a.dq), qhi = (float)(a.qmin + (double)(k0 + KC) * a.dq);
      const float xmax = (float)vi.W - 1.5f, ymax = (float)vi.H - 1.5f;
      inner = true;
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const float cu = (float)((c & 1) ? bb.z : bb.x), cv = (float)((c & 2) ? bb.w : bb.y), cq = (c & 4) ? qhi : qlo;
        const float cx = fmaf(cq, pg.b[0], fmaf(pg.A[0], cu, fmaf(pg.A[1], cv, pg.A[2])));
        const float cy = fmaf(cq, pg.b[1], fmaf(pg.A[3], cu, fmaf(pg.A[4], cv, pg.A[5])));
        const float cw = fmaf(cq, pg.b[2], fmaf(pg.A[6], cu, fmaf(pg.A[7], cv, pg.A[8])));
        inner = inner && cw > 1e-3f && cx >= 0.5f * cw && cx <= xmax * cw && cy >= 0.5f * cw && cy <= ymax * cw;
      }
    }
    const uint64_t inner_views = __ballot(inner);
    float acc[KC];
#pragma unroll
    for (int j = 0; j < KC; ++j) acc[j] = 0.f;
    int iv = 0, p = lane;
    while (p >= A) {
      p -= A;
      ++iv;
    }
    int cur = -1;
    SweepPair sp = {};
    const __amdgpu_buffer_rsrc_t qrs = buffer_rsrc(a.quads, a.quad_bytes);
    const int n_pass = (P + kWave - 1) / kWave;
    int passes = n_pass;
    const float bound_ref = a.exact_margin ? second : best;  // complete levels change only between chunks
    for (int it = 0; it < n_pass; ++it) {
      if (lane + it * kWave < P) {
      if (iv != cur) {
        sp = pairs.at<FMT>(iv);
        cur = iv;
      }
      const PixEntry e = a.px[poff + p];
      const float du = (float)((int)(e.x & 0xffffu) - pairs.ub), dv = (float)((int)(e.x >> 16) - pairs.vb);
      const float r0 = (float)(e.y & 255u), g0 = (float)((e.y >> 8) & 255u), b0 = (float)((e.y >> 16) & 255u);
      const float ax = fmaf(sp.h[0], du, fmaf(sp.h[1], dv, sp.h[2]));
      const float ay = fmaf(sp.h[3], du, fmaf(sp.h[4], dv, sp.h[5]));
      const float aw = fmaf(sp.h[6], du, fmaf(sp.h[7], dv, sp.h[8]));
      // every active lane in an inner view (neighbours past the 64th are
      // never taken as inner): samples without the bounds test
      if (__ballot(iv >= kWave || ((inner_views >> iv) & 1ull) == 0ull) == 0ull)
        sample_levels<FMT, KC>(q, acc, ax, ay, aw, sp.b[0], sp.b[1], sp.b[2], sp.f, qrs, r0, g0, b0, a.T255, false);
      else
        sample_levels<FMT, KC>(q, acc, ax, ay, aw, sp.b[0], sp.b[1], sp.b[2], sp.f, qrs, r0, g0, b0, a.T255, true);
      p += kWave;
      while (p >= A) {
        p -= A;
        ++iv;
      }
      }
      if ((it & (kBoundCheck - 1)) == kBoundCheck - 1 && it + 1 < n_pass && bound_ref < INFINITY) {
        const float lim = bound_ref * kBoundMargin;
        bool bounded = true;
#pragma unroll
        for (int kk = 0; kk < KC; ++kk)
          if (bounded && k0 + kk < k_end) bounded = wave_sum(acc[kk]) > lim;
        if (bounded) {
          passes = it + 1;
          break;
        }
      }
    }
    computed += (uint64_t)min(P, passes * kWave) * (uint64_t)min(KC, k_end - k0);
    if (passes < n_pass) continue;  // no level of this chunk can be the best (or, with exact_margin, the second best)
    scored += (uint32_t)min(KC, k_end - k0);
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
      const float C = wave_sum(acc[kk]);
      if (k0 + kk < k_end) {
        if (C < best || (C == best && k0 + kk < kbest)) {
          second = best;
          best = C;
          kbest = k0 + kk;
        } else if (C < second) {
          second = C;
        }
      }
    }
  }
}

// Sweep outputs of superpixel g (one lane): the fronto-parallel plane of
// the best level, its {colour, inverse-depth row} record, normalised cost,
// level and margin.
__device__ __forceinline__ void sweep_finish(const SweepArgs &a, const int g, const int v, const int s, const int A,
                                             const int N, const float best, const float second, const int kbest) {
  const double qb = level_q(a.seed, a.jitter, a.qmin, a.dq, v, s, kbest);
  a.planes[g] = make_float4((float)(1.0 / qb), 0.f, 0.f, 1.f);
  a.tab[2 * g] = a.colour[g];
  a.tab[2 * g + 1] = make_float4(0.f, 0.f, (float)qb, 0.f);
  const float norm = 1.f / ((float)A * (float)N * a.T255);
  a.cost[g] = best * norm;
  a.choice[g] = kbest;
  a.margin[g] = a.levels > 1 ? (second - best) * norm : INFINITY;
}

__device__ __forceinline__ void sweep_empty(const SweepArgs &a, const int g) {
  a.planes[g] = make_float4(0.f, 0.f, 0.f, 0.f);
  a.tab[2 * g] = make_float4(0.f, 0.f, 0.f, 0.f);
  a.tab[2 * g + 1] = make_float4(0.f, 0.f, 0.f, 0.f);
  a.cost[g] = 0.f;
  a.choice[g] = -1;
  a.margin[g] = 0.f;
}

template <int FMT, int KC>
__device__ __forceinline__ void sweep_sp(const SweepArgs &a, const int g) {
  const int lane = threadIdx.x & (kWave - 1);
  const int v = a.sp_view[g];
  const ViewDev &vw = a.views[v];
  const int s = g - vw.sp_off;
  const int A = a.area[g];
  if (A == 0) {
    if (lane == 0) sweep_empty(a, g);
    return;
  }
  float best = INFINITY, second = INFINITY;
  int kbest = 0;
  uint64_t computed = 0;
  uint32_t scored = 0;
  sweep_levels<FMT, KC>(a, g, v, s, vw, A, 0, a.levels, best, second, kbest, computed, scored);
  if (lane == 0) {
    sweep_finish(a, g, v, s, A, vw.n_pairs, best, second, kbest);
    atomicAdd(&a.work[3], (unsigned long long)computed);
    atomicAdd(&a.work[4], (unsigned long long)scored);
  }
}

// Levels of part `part` of `split` (contiguous, whole level chunks) of
// superpixel g; writes {best, second, level} to parts[part].  Empty
// superpixels are written by the finalize step.
__device__ __forceinline__ int part_levels(int levels, int split, int kc) {
  return ((levels + split - 1) / split + kc - 1) / kc * kc;
}
template <int FMT, int KC>
__device__ __forceinline__ void sweep_part(const SweepArgs &a, const int g, const int part, const int split,
                                           float4 *parts) {
  const int lane = threadIdx.x & (kWave - 1);
  const int v = a.sp_view[g];
  const ViewDev &vw = a.views[v];
  const int s = g - vw.sp_off;
  const int A = a.area[g];
  if (A == 0) return;
  const int per = part_levels(a.levels, split, KC);
  const int kb = part * per, ke = min(a.levels, kb + per);
  float best = INFINITY, second = INFINITY;
  int kbest = 0;
  uint64_t computed = 0;  // the bound references this part's own complete levels (best, or second best
                          // with exact_margin), so the part's best stays exact and the merge is too
  uint32_t scored = 0;
  if (kb < ke) sweep_levels<FMT, KC>(a, g, v, s, vw, A, kb, ke, best, second, kbest, computed, scored);
  if (lane == 0) {
    parts[part] = make_float4(best, second, __int_as_float(kbest), 0.f);
    atomicAdd(&a.work[3], (unsigned long long)computed);
    atomicAdd(&a.work[4], (unsigned long long)scored);
  }
}

// Merges the parts of superpixel g in level order: the two smallest costs
// and the level of the first smallest, as one pass over all levels gives.
__device__ __forceinline__ void sweep_merge(const SweepArgs &a, const int g, const int split, const float4 *parts) {
  const int v = a.sp_view[g];
  const ViewDev &vw = a.views[v];
  const int A = a.area[g];
  if (A == 0) {
    sweep_empty(a, g);
    return;
  }
  float best = INFINITY, second = INFINITY;
  int kbest = 0;
  for (int p = 0; p < split; ++p) {
    const float4 r = parts[p];
    if (r.x < best) {
      second = fminf(best, r.y);
      best = r.x;
      kbest = __float_as_int(r.z);
    } else {
      second = fminf(second, r.x);
    }
  }
  sweep_finish(a, g, v, g - vw.sp_off, A, vw.n_pairs, best, second, kbest);
}

#ifndef SLF_LEVEL_CHUNK
#define SLF_LEVEL_CHUNK 8
#endif
constexpr int kLevelChunk = SLF_LEVEL_CHUNK;

// Waves per SIMD the sweep's registers are sized for (128 VGPRs; 3 and 5
// waves measured slower).
constexpr int kSweepWaves = 4;

template <int FMT, int KC>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(kSweepWaves))) void k_sweep(SweepArgs a, int *__restrict__ counters) {
  for_each_claimed(a.S, counters, [&](int c) { sweep_sp<FMT, KC>(a, a.order ? ro_at(a.order, c) : c); });
}

// Writes one launch's arguments into device memory (the launch copies its
// own arguments, so no host buffer has to outlive the call; stream order
// puts the write after every earlier kernel and before the one that reads)
// and clears the claim counters of the launch that follows.
template <class T>
__global__ void k_put_args_reset(T *dst, T v, int *counters) {
  if (threadIdx.x == 0) *dst = v;
  if (threadIdx.x < kPoolQueues) counters[threadIdx.x * kPoolCounterStride] = 0;
}

hipError_t launch_sweep(int fmt, const SweepArgs &a, int *counters, int n_cu, hipStream_t st) {
  const void *k = fmt == SLF_FMT_U8    ? (const void *)k_sweep<SLF_FMT_U8, kLevelChunk>
                  : fmt == SLF_FMT_F16 ? (const void *)k_sweep<SLF_FMT_F16, kLevelChunk>
                                       : (const void *)k_sweep<SLF_FMT_F32, kLevelChunk>;
  hipLaunchKernelGGL(k_pool_reset, dim3(1), dim3(64), 0, st, counters);
  SweepArgs args = a;
  void *kargs[] = {(void *)&args, (void *)&counters};
  return hipLaunchKernel(k, dim3(persistent_blocks(k, n_cu, a.S)), dim3(kBlock), kargs, 0, st);
}

// ------------------------------------------------------------------ refinement (a6-a8)


constexpr int kLdsPix = 1024;  // pixels of a superpixel staged in LDS (the rest read from the list)
#ifndef SLF_REFINE_CHAINS
#define SLF_REFINE_CHAINS 3
#endif
// independent gather chains per lane in the energy loop: 3 (passes of 192
// pixels; a median superpixel of 350 pixels pads to two) measured 1.5 %
// faster than 2 on the full-HD refinement, the extra registers spilling only
// outside the sample loops
constexpr int kChains = SLF_REFINE_CHAINS;
#ifndef SLF_REFINE_WAVES
#define SLF_REFINE_WAVES 5
#endif
constexpr int kRefineWaves = SLF_REFINE_WAVES;  // waves per SIMD the refinement's registers are sized for
static_assert(kLdsPix % kWave == 0, "the staged pixel list pads to whole waves");

typedef __attribute__((address_space(3))) uint32_t LdsU32;
typedef __attribute__((address_space(3))) float LdsF32;
typedef __attribute__((address_space(3))) uint8_t LdsU8;

__device__ __forceinline__ float3 load_f3(__amdgpu_buffer_rsrc_t rs, int off) {
  typedef float f3v __attribute__((ext_vector_type(3)));
  const f3v v = __builtin_bit_cast(f3v, __builtin_amdgcn_raw_buffer_load_b96(rs, off, 0, 0));
  return make_float3(v.x, v.y, v.z);
}

__device__ __forceinline__ float4 load_f4(__amdgpu_buffer_rsrc_t rs, int off) {
  typedef float f4v __attribute__((ext_vector_type(4)));
  const f4v v = __builtin_bit_cast(f4v, __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0));
  return make_float4(v.x, v.y, v.z, v.w);
}

// The best plane so far (in the wave's LDS) and its depth at the centroid.
struct BestPlane {
  double nx, ny, nz, delta, d;
};
typedef __attribute__((address_space(3))) BestPlane LdsBest;

// Energies, slot and counters of the running winner (uniform, in scalar registers).
struct Best {
  float E, second;
  int slot, evaluated, pruned, view_samples;
  bool ordered;  // views are visited in the order of the first candidate's terms (vorder)
};

// Ring neighbour j of the superpixel (eq. 5), held in LDS.
struct RingEntry {
  double rx, ry, rz;  // K_r^-1 (c_j, 1)
  double d;           // centroid depth in state A
  float w;            // omega(C_s, C_j) scaled by 1 / max_j omega (same ratio in eq. 5)
  int cell;           // -1 if outside the grid or empty
};
// Per-(candidate, neighbour view) projection constants, composed in FP64 and
// stored in FP32 (see energy()).
struct ViewConst {
  float ax, axu, axv, ay, ayu, ayv, aw, awu, awv;
  int X0, Y0, pad;
};
constexpr int kViewsPerPass = 16;  // neighbour views whose constants are composed at once
typedef __attribute__((address_space(3))) RingEntry LdsRing;
typedef __attribute__((address_space(3))) ViewConst LdsViewConst;

// Field-wise copies between registers and LDS.
__device__ __forceinline__ RingEntry lds_get(const LdsRing *p) {
  RingEntry r;
  r.rx = p->rx;
  r.ry = p->ry;
  r.rz = p->rz;
  r.d = p->d;
  r.w = p->w;
  r.cell = p->cell;
  return r;
}
__device__ __forceinline__ void lds_put(LdsRing *p, const RingEntry &r) {
  p->rx = r.rx;
  p->ry = r.ry;
  p->rz = r.rz;
  p->d = r.d;
  p->w = r.w;
  p->cell = r.cell;
}
__device__ __forceinline__ ViewConst lds_get(const LdsViewConst *p) {
  ViewConst q;
  q.ax = p->ax;
  q.axu = p->axu;
  q.axv = p->axv;
  q.ay = p->ay;
  q.ayu = p->ayu;
  q.ayv = p->ayv;
  q.aw = p->aw;
  q.awu = p->awu;
  q.awv = p->awv;
  q.X0 = p->X0;
  q.Y0 = p->Y0;
  q.pad = 0;
  return q;
}
__device__ __forceinline__ void lds_put(LdsViewConst *p, const ViewConst &q) {
  p->ax = q.ax;
  p->axu = q.axu;
  p->axv = q.axv;
  p->ay = q.ay;
  p->ayu = q.ayu;
  p->ayv = q.ayv;
  p->aw = q.aw;
  p->awu = q.awu;
  p->awv = q.awv;
  p->X0 = q.X0;
  p->Y0 = q.Y0;
}

// Per-superpixel data the energy needs, uniform over the wave.  Geometry
// that defines candidate planes (rays through centroids, normals) is FP64.
// Per-lane tables live in the wave's LDS space, so that they hold no
// registers while the samples run.
struct SpCtx {
  int g, v, s, A, N, poff;
  int ub, vb;                // centroid rounded to the nearest pixel
  float invA;                // 1 / |Omega|
  const LdsU32 *pix_lds;     // pixels 0..n_lds-1 as FP16 pairs (u - ub, v - vb), staged in LDS
  int n_lds;                 // staged pixels (0 if an offset exceeds 2048: FP16 holds integers exactly up to there)
  int n_pad;                 // n_lds rounded up to whole waves; entries n_lds..n_pad-1 hold a NaN pair
  const LdsRing *ring;       // ring neighbours 0..7
  LdsViewConst *vc;          // constants of up to kViewsPerPass neighbour views
  LdsBest *best;             // plane of the running winner
  LdsF32 *tview;             // per-view terms of the first evaluated candidate (N <= kViewsPerPass)
  LdsU8 *vorder;             // views in increasing order of those terms
  double rsx, rsy, rsz;      // K_r^-1 (c_s, 1)
  float4 Cs;                 // mean colour
  float omega_min;           // min over ring neighbours of omega(C_s, C_j); 1 without neighbours
  int M;                     // number of non-empty ring neighbours
};

__device__ __forceinline__ float uni_f(float x) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}

__device__ __forceinline__ double bcast_d(double x, int l) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Energy E = E_c E_s (eqs. 3-11) of the 3D plane n . X = delta in camera r.
// `e_floor` is an energy already reached (the best or the second best so
// far).  Each view's term of E_c is at most 1 + occ (every S_i, V_i and
// Gaussian mean is at most 1), so after j of the N views E_c <= (their sum +
// (N - j)(1 + occ)) / N.  Once E_s times that bound lies below e_floor, with a
// margin far above FP32 rounding, the candidate cannot reach e_floor: it can
// change neither the winner nor (with the second best as floor) the margin.
// *pruned is set and the remaining views are skipped.  *views receives the
// number of neighbour views sampled.
template <int FMT>
__device__ float energy(const RefineArgs &a, const SpCtx &c, const ViewDev &vw, double nx, double ny, double nz,
                        double delta, float e_floor, bool &pruned, int &views, bool record, bool ordered) {
  pruned = false;
  views = 0;
  const int lane = threadIdx.x & (kWave - 1);

  if (a.energy_mode == 1) {  // data-only: -normalised TSSD of this plane
    const double idl = 1.0 / delta;
    const double gg[3] = {(nx * vw.Kinv_d[0] + ny * vw.Kinv_d[3] + nz * vw.Kinv_d[6]) * idl,
                          (nx * vw.Kinv_d[1] + ny * vw.Kinv_d[4] + nz * vw.Kinv_d[7]) * idl,
                          (nx * vw.Kinv_d[2] + ny * vw.Kinv_d[5] + nz * vw.Kinv_d[8]) * idl};
    float acc = 0.f;
    for (int iv = 0; iv < c.N; ++iv) {
      const PairDev &pg = ro_at(a.pairs, vw.pair_off + iv);
      const ViewDev &vi = ro_at(a.views, pg.i);
      double H[9];
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int q = 0; q < 3; ++q) H[3 * r + q] = pg.A_d[3 * r + q] + pg.b_d[r] * gg[q];
      // re-centred as in the sweep: offsets from the rounded centroid in,
      // positions relative to the pixel nearest its projection out
      const double hx = H[0] * c.ub + H[1] * c.vb + H[2];
      const double hy = H[3] * c.ub + H[4] * c.vb + H[5];
      const double hw = H[6] * c.ub + H[7] * c.vb + H[8];
      int X0, Y0;
      near_pixel(hx, hy, hw, vi, X0, Y0);
      const float h0 = (float)(H[0] - X0 * H[6]), h1 = (float)(H[1] - X0 * H[7]), h2 = (float)(hx - X0 * hw);
      const float h3 = (float)(H[3] - Y0 * H[6]), h4 = (float)(H[4] - Y0 * H[7]), h5 = (float)(hy - Y0 * hw);
      const float h6 = (float)H[6], h7 = (float)H[7], h8 = (float)hw;
      const SampleFrame f = frame_at<FMT>(vi, X0, Y0);
      for (int p = lane; p < c.A; p += kWave) {
        const PixEntry e = a.px[c.poff + p];
        const float du = (float)((int)(e.x & 0xffffu) - c.ub), dv = (float)((int)(e.x >> 16) - c.vb);
        acc += tssd_sample<FMT>(fmaf(h0, du, fmaf(h1, dv, h2)), fmaf(h3, du, fmaf(h4, dv, h5)),
                                fmaf(h6, du, fmaf(h7, dv, h8)), f, buffer_rsrc(a.quads, a.quad_bytes),
                                (float)(e.y & 255u), (float)((e.y >> 8) & 255u), (float)((e.y >> 16) & 255u), a.T255);
      }
    }
    views = c.N;
    return -wave_sum(acc) / ((float)c.A * (float)c.N * a.T255);
  }

  // Smoothness, eqs. (5)-(6): this plane extrapolated to neighbour j's centroid
  float Es = 1.f;
  if ((a.term_mask & 1u) && c.M > 0) {
    float num = 0.f, den = 0.f;
    if (lane < 8) {
      const RingEntry r = lds_get(c.ring + lane);
      if (r.cell >= 0) {
        const double t = nx * r.rx + ny * r.ry + nz * r.rz;
        float sj = 0.f;
        if (t > 0.0) {
          const float dd = (float)(r.d - delta * rcp_d(t));
          sj = __expf(-dd * dd * a.inv2sig2);
        }
        num = r.w * sj;
        den = r.w;
      }
    }
    Es = ring_sum(num) * rcp(ring_sum(den));  // the nearest colour has weight 1, so den >= 1
  }

  const float occ = (a.term_mask & 4u) ? a.eta * (1.f - c.omega_min) : 0.f;
  const float ec_max = (a.term_mask & 2u) ? (1.f + occ) * 1.001f : 1.f;
  if (Es * ec_max < e_floor) {
    pruned = true;
    return 0.f;
  }

  // Consistency, eqs. (8)-(11).  Pixels are taken relative to the rounded
  // centroid (ub, vb) and projections relative to the integer pixel (X0, Y0)
  // nearest to the projected centroid, so the FP32 per-sample arithmetic
  // works on small offsets and the nearest-pixel decision of eq. (9) keeps
  // ~1e-6 px accuracy at any image size.  The per-(candidate, view)
  // constants are composed in FP64 (lane j composes neighbour view base + j,
  // into LDS) and read back into scalar registers view by view.
  float Ec = 1.f;
  if (a.term_mask & 2u) {
    const double idl = rcp_d(delta);
    const double gd0 = (nx * vw.Kinv_d[0] + ny * vw.Kinv_d[3] + nz * vw.Kinv_d[6]) * idl;
    const double gd1 = (nx * vw.Kinv_d[1] + ny * vw.Kinv_d[4] + nz * vw.Kinv_d[7]) * idl;
    const double gd2 = (nx * vw.Kinv_d[2] + ny * vw.Kinv_d[5] + nz * vw.Kinv_d[8]) * idl;
    const float i0 = (float)(gd0 * c.ub + gd1 * c.vb + gd2);  // 1 / D at the rounded centroid
    const float gu = (float)gd0, gv = (float)gd1;
    float sum = 0.f;
    const float tau = a.occ_tol;
    // omega of eq. (7) as exp2(k (2 C_s . C_l - |C_l|^2 - |C_s|^2)) = exp2(-k |C_s - C_l|^2):
    // the records carry |C_l|^2, so a sample spends three FMAs on the colour
    const float kc = a.inv2alpha2_log2e, cw0 = -kc * c.Cs.w;
    const float c2r = 2.f * c.Cs.x, c2g = 2.f * c.Cs.y, c2b = 2.f * c.Cs.z;
    const __amdgpu_buffer_rsrc_t px_rs = buffer_rsrc(a.px + c.poff, 8u * (uint32_t)c.A);
    for (int base = 0; base < c.N; base += kViewsPerPass) {
      const int nv = min(kViewsPerPass, c.N - base);
      wave_lds_sync();  // the previous pass's reads are done
      if (lane < nv) {
        float ax = 0.f, axu = 0.f, axv = 0.f, ay = 0.f, ayu = 0.f, ayv = 0.f, aw = 0.f, awu = 0.f, awv = 0.f;
        int X0 = 0, Y0 = 0;
        const PairDev &pg = a.pairs[vw.pair_off + base + lane];
        double H[9];
        const double gg[3] = {gd0, gd1, gd2};
        for (int r = 0; r < 3; ++r)
          for (int q = 0; q < 3; ++q) H[3 * r + q] = pg.A_d[3 * r + q] + pg.b_d[r] * gg[q];
        const double hx = H[0] * c.ub + H[1] * c.vb + H[2];
        const double hy = H[3] * c.ub + H[4] * c.vb + H[5];
        const double hw = H[6] * c.ub + H[7] * c.vb + H[8];
        if (hw > 0.0) {
          // only the re-centring pixel: any nearby integer serves, so FP32 suffices
          const float rhw = rcp((float)hw);
          const double xc = (double)((float)hx * rhw), yc = (double)((float)hy * rhw);
          if (fabs(xc) < 1.0e7 && fabs(yc) < 1.0e7) {
            X0 = (int)floor(xc + 0.5);
            Y0 = (int)floor(yc + 0.5);
          }
        }
        ax = (float)(hx - X0 * hw);
        axu = (float)(H[0] - X0 * H[6]);
        axv = (float)(H[1] - X0 * H[7]);
        ay = (float)(hy - Y0 * hw);
        ayu = (float)(H[3] - Y0 * H[6]);
        ayv = (float)(H[4] - Y0 * H[7]);
        aw = (float)hw;
        awu = (float)H[6];
        awv = (float)H[7];
        lds_put(c.vc + lane, ViewConst{ax, axu, axv, ay, ayu, ayv, aw, awu, awv, X0, Y0, 0});
      }
      wave_lds_sync();
      for (int jo = 0; jo < nv; ++jo) {
        // the jo-th view of this pass (in vorder once it is set), uniform over the wave
        const int jv = ordered ? __builtin_amdgcn_readfirstlane((int)c.vorder[jo]) : jo;
        const ViewConst q = lds_get(c.vc + jv);
        // The multipliers go to scalar registers.  The three addends stay
        // in vector registers (every lane read the same LDS word): an FMA
        // can read only one scalar operand, so scalar addends would be
        // copied back into vector registers on every pass.
        const float cax = q.ax, caxu = uni_f(q.axu), caxv = uni_f(q.axv);
        const float cay = q.ay, cayu = uni_f(q.ayu), cayv = uni_f(q.ayv);
        const float caw = q.aw, cawu = uni_f(q.awu), cawv = uni_f(q.awv);
        const int iX0 = __builtin_amdgcn_readfirstlane(q.X0), iY0 = __builtin_amdgcn_readfirstlane(q.Y0);
        const float fX0 = (float)iX0, fY0 = (float)iY0;
        const ViewDev &vi = ro_at(a.views, ro_at(a.pairs, vw.pair_off + base + jv).i);
        const uint32_t Wv = (uint32_t)vi.W, Hv = (uint32_t)vi.H;
        // 16-bit labels when every view has at most 65536 cells: half the
        // bytes of the label windows the gathers touch.
        const uint32_t npx = (uint32_t)vi.W * (uint32_t)vi.H;
        const __amdgpu_buffer_rsrc_t lab_rs =
            a.lab16 ? buffer_rsrc(a.lab16 + vi.pix_off, 2u * npx) : buffer_rsrc(a.labels + vi.pix_off, 4u * npx);
        const __amdgpu_buffer_rsrc_t tab_rs = buffer_rsrc(a.tabA + 2 * vi.sp_off, 32u * (uint32_t)(vi.gw * vi.gh));
        float sw = 0.f, gx = 0.f;
        // |X_i| and whether Y_i is non-empty are exact integer results, so
        // they are kept per wave in scalar registers (a ballot per sample)
        // rather than per lane and reduced afterwards.
        int nX = 0;
        uint64_t occluded = 0;
        // Branch-free samples in three phases: project the pixel into view
        // i (clamped into the image), gather its label, gather the label's
        // record; the gathers are raw buffer loads bounded by their arrays.
        // Predicates decide what is accumulated.
        // Predicates are carried as wave masks (a ballot of each compare is
        // the compare's own result), so they combine in scalar registers and
        // feed the per-lane selects and the wave-level counts directly.
        struct Proj {
          float iota, w, dx, dy;
          uint64_t seen;  // lanes whose pixel lands inside view i, in front of both cameras
          uint32_t pix;
        };
        // (du, dv): the pixel relative to (ub, vb).  The staged FP16 offsets
        // enter the FMAs as mixed-precision operands, converted exactly.
        auto project = [&](float du, float dv) {
          Proj q;
          q.iota = fmaf(gu, du, fmaf(gv, dv, i0));  // 1 / D(p)
          q.w = fmaf(cawu, du, fmaf(cawv, dv, caw));  // z_i(P) = w / iota
          const float rw = rcp(q.w);
          q.dx = fmaf(caxu, du, fmaf(caxv, dv, cax)) * rw;
          q.dy = fmaf(cayu, du, fmaf(cayv, dv, cay)) * rw;
          // nearest pixel (round half up, in one instruction and without
          // rounding x + 0.5 first); inside the image iff 0 <= u < W, 0 <= v < H
          const int ui = iX0 + round_half_up(q.dx), vi = iY0 + round_half_up(q.dy);
          q.seen = __builtin_amdgcn_ballot_w64(q.iota > 0.f) & __builtin_amdgcn_ballot_w64(q.w > 0.f) &
                   __builtin_amdgcn_ballot_w64((uint32_t)ui < Wv) & __builtin_amdgcn_ballot_w64((uint32_t)vi < Hv);
          // outside the image (not seen) the offset is arbitrary: the gathers
          // are bounded by their buffer resources and the sample is masked out
          q.pix = __umul24((uint32_t)vi, Wv) + (uint32_t)ui;  // sides below 2^16
          return q;
        };
        auto label = [&](const Proj &q, auto narrow) -> uint32_t {
          if constexpr (decltype(narrow)::value)
            return (uint32_t)__builtin_amdgcn_raw_buffer_load_b16(lab_rs, (int)(2u * q.pix), 0, 0);
          else
            return (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(lab_rs, (int)(4u * q.pix), 0, 0);
        };
        auto accumulate = [&](const Proj &q, const float4 Cl, const float3 gt) {
          const float cl = fmaf(c2r, Cl.x, fmaf(c2g, Cl.y, fmaf(c2b, Cl.z, -Cl.w)));
          const float om = __builtin_amdgcn_exp2f(fmaf(cl, kc, cw0));
          const float den = fmaf(gt.x, fX0 + q.dx, fmaf(gt.y, fY0 + q.dy, gt.z));  // 1 / D(p^i)
          const uint64_t back = __builtin_amdgcn_ballot_w64(!(den > 0.f));
          // z <= D(p^i) (1 + tau)  <=>  w den - iota <= tau iota   (iota, den > 0);
          // the residual is one FMA and also the numerator of z - D(p^i)
          const float num = fmaf(q.w, den, -q.iota);
          const uint64_t vis = q.seen & (back | __builtin_amdgcn_ballot_w64(num <= tau * q.iota));
          const float dz = num * rcp(q.iota * den);  // z - D(p^i)
          const float gk = __builtin_amdgcn_exp2f(-dz * dz * a.inv2sig2_log2e);
          sw += __builtin_amdgcn_inverse_ballot_w64(q.seen) ? om : 0.f;
          nX += __popcll(vis);
          gx += __builtin_amdgcn_inverse_ballot_w64(vis & ~back) ? gk : 0.f;
          occluded |= q.seen & ~vis;
        };
        auto staged = [&](int p) {
          const __half2 h = __builtin_bit_cast(__half2, (uint32_t)c.pix_lds[p]);
          return project(__low2float(h), __high2float(h));
        };
        auto listed = [&](int p) {
          const uint32_t uv = (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(px_rs, (int)(8u * (uint32_t)p), 0, 0);
          return project((float)((int)(uv & 0xffffu) - c.ub), (float)((int)(uv >> 16) - c.vb));
        };
        auto one = [&](int p, bool in, auto narrow) {
          Proj q = listed(p);
          q.seen &= __builtin_amdgcn_ballot_w64(in);
          const uint32_t l = label(q, narrow);
          accumulate(q, load_f4(tab_rs, (int)(32u * l)), load_f3(tab_rs, (int)(32u * l + 16u)));
        };
        // kChains pixels per lane per pass keep that many gather chains in
        // flight; each lane still accumulates its pixels in order.  The
        // staged list is padded to whole waves with NaN offsets: a NaN pixel
        // projects to iota = NaN, so it is never seen and adds +0, which
        // leaves the lane's sums unchanged, and its clamped gathers stay in
        // bounds.  The trip counts are uniform (whole passes, then fewer than
        // kChains waves of pixels on one chain), and the wave-level counts
        // stay in scalar registers.
        // K waves of staged pixels, one gather chain each
        auto pass = [&](int p0, auto narrow, auto chains) {
          constexpr int K = decltype(chains)::value;
          Proj q[K];
          uint32_t l[K];
          float4 C[K];
          float3 G[K];
#pragma unroll
          for (int k = 0; k < K; ++k) q[k] = staged(p0 + k * kWave + lane);
#pragma unroll
          for (int k = 0; k < K; ++k) l[k] = label(q[k], narrow);
#pragma unroll
          for (int k = 0; k < K; ++k) {
            C[k] = load_f4(tab_rs, (int)(32u * l[k]));
            G[k] = load_f3(tab_rs, (int)(32u * l[k] + 16u));
          }
#pragma unroll
          for (int k = 0; k < K; ++k) accumulate(q[k], C[k], G[k]);
        };
        auto samples = [&](auto narrow) {
          const int n_pad = c.n_pad;
          int p0 = 0;
          for (; p0 + kChains * kWave <= n_pad; p0 += kChains * kWave)
            pass(p0, narrow, std::integral_constant<int, kChains>{});
          // the staged list pads to whole waves: two waves left take two
          // chains, one wave one
          if (kChains > 2 && p0 + 2 * kWave <= n_pad) {
            pass(p0, narrow, std::integral_constant<int, 2>{});
            p0 += 2 * kWave;
          }
          for (; p0 < n_pad; p0 += kWave) {
            const Proj q = staged(p0 + lane);
            const uint32_t l = label(q, narrow);
            accumulate(q, load_f4(tab_rs, (int)(32u * l)), load_f3(tab_rs, (int)(32u * l + 16u)));
          }
          for (int p0 = c.n_lds; p0 < c.A; p0 += kWave) {
            const int p = p0 + lane;
            one(p < c.A ? p : p0, p < c.A, narrow);
          }
        };
        if (a.lab16)
          samples(std::true_type{});
        else
          samples(std::false_type{});
        float swt, gxt;
        wave_sum2(sw, gx, swt, gxt);
        const int nXt = nX;
        const bool Y = occluded != 0ull;
        const float Si = swt * c.invA;
        const float Vi = nXt > 0 ? Si * gxt * rcp((float)nXt) : 0.f;
        const float term = Vi + (Y ? occ : 0.f);
        if (record && lane == 0) c.tview[base + jv] = term;
        sum += term;
        ++views;
        const float left = (float)(c.N - views);
        if (Es * (sum + left * (1.f + occ)) * rcp((float)c.N) * 1.001f < e_floor) {
          pruned = true;
          return 0.f;
        }
      }
    }
    Ec = sum * rcp((float)c.N);
  }
  return Ec * Es;
}

__device__ __forceinline__ void ray_of(const ViewDev &vw, double2 cp, double &x, double &y, double &z) {
  x = vw.Kinv_d[0] * cp.x + vw.Kinv_d[1] * cp.y + vw.Kinv_d[2];
  y = vw.Kinv_d[3] * cp.x + vw.Kinv_d[4] * cp.y + vw.Kinv_d[5];
  z = vw.Kinv_d[6] * cp.x + vw.Kinv_d[7] * cp.y + vw.Kinv_d[8];
}

// One candidate plane n . X = delta of camera r, its depth d at the
// superpixel's centroid and its slot number.
struct Cand {
  double nx, ny, nz, delta;
  int slot, pad;
};
constexpr int kCandBatch = kWave;  // candidates generated per batch (one per lane)

// Wave-uniform copies (the value of the first active lane, held in SGPRs).
__device__ __forceinline__ double uni_d(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffll));
  const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Appends this lane's candidate (if valid) to list[base..] keeping lane
// order; returns the number appended (uniform).
__device__ __forceinline__ int append_cand(Cand *list, int base, bool valid, const Cand &cd) {
  const int lane = threadIdx.x & (kWave - 1);
  const uint64_t mask = __ballot(valid);
  if (valid) list[base + __popcll(mask & ((1ull << lane) - 1ull))] = cd;
  return __popcll(mask);
}

// Evaluates list[0..n) in order; a candidate replaces the best only on a
// strictly larger energy (Sec. III-C), so ties keep the earlier slot.
template <int FMT>
__device__ void evaluate(const RefineArgs &a, const SpCtx &c, const ViewDev &vw, const Cand *list, int n, Best &b) {
  for (int k = 0; k < n; ++k) {
    Cand cd = list[k];
    cd.nx = uni_d(cd.nx);
    cd.ny = uni_d(cd.ny);
    cd.nz = uni_d(cd.nz);
    cd.delta = uni_d(cd.delta);
    cd.slot = __builtin_amdgcn_readfirstlane(cd.slot);
    bool pruned;
    int views;
    // A candidate whose energy bound falls below the floor cannot replace the
    // best (a strictly larger energy does), nor tie with it; with exact_margin
    // the floor is the second best, so it cannot be the second best either.
    const float floor_E = a.exact_margin ? b.second : (b.slot >= 0 ? b.E : -INFINITY);
    // The first candidate (never pruned: the floor is still -inf) records its
    // per-view terms of E_c; later candidates visit the views in increasing
    // order of those terms.  Views where even the running winner scores low
    // (pixels outside the image, occluded, or in other superpixels) bring a
    // candidate's bound down fastest; the bound holds in any order, and only
    // the FP32 rounding order of the view sum changes.
    const bool record = !b.ordered && b.evaluated == 0 && a.energy_mode == 0 && (a.term_mask & 2u) &&
                        c.N <= kViewsPerPass;
    const float E =
        uni_f(energy<FMT>(a, c, vw, cd.nx, cd.ny, cd.nz, cd.delta, floor_E, pruned, views, record, b.ordered));
    if (record && !pruned && views == c.N) {
      wave_lds_sync();
      const int lane = threadIdx.x & (kWave - 1);
      if (lane < c.N) {
        const float t = c.tview[lane];
        int rank = 0;
        for (int j = 0; j < c.N; ++j) {
          const float u = c.tview[j];
          rank += (u < t || (u == t && j < lane)) ? 1 : 0;
        }
        c.vorder[rank] = (uint8_t)lane;
      }
      wave_lds_sync();
      b.ordered = true;
    }
    ++b.evaluated;
    b.view_samples += views;
    if (pruned) {  // bounded below the second best: no change
      ++b.pruned;
      continue;
    }
    if (b.slot < 0 || E > b.E) {
      if (b.slot >= 0) b.second = b.E;
      b.E = E;
      b.slot = cd.slot;
      c.best->nx = cd.nx;
      c.best->ny = cd.ny;
      c.best->nz = cd.nz;
      c.best->delta = cd.delta;
      c.best->d = cd.delta * rcp_d(cd.nx * c.rsx + cd.ny * c.rsy + cd.nz * c.rsz);  // depth at the centroid
    } else if (E > b.second) {
      b.second = E;
    }
  }
}

// One refinement step per superpixel (Sec. III-C): propagation over the
// kernel, then 8 triangle normals pivoting at the winner's centroid depth.
// Candidates are generated lane-parallel in slot order into an LDS list and
// evaluated in that order by one energy loop.
// The LDS space of one wave in the refinement.
struct WaveLds {
  float tview[kViewsPerPass];
  uint8_t vorder[kViewsPerPass];
  Cand list[kCandBatch];
  uint32_t pix[kLdsPix];
  ViewConst vc[kViewsPerPass];
  RingEntry ring[8];
  BestPlane best;
};

template <int FMT>
__device__ __forceinline__ void refine_sp(const RefineArgs &a, const int g, WaveLds &wl) {
  Cand *list = wl.list;
  uint32_t *pix_lds = wl.pix;
  const int lane = threadIdx.x & (kWave - 1);
  SpCtx c;
  c.g = g;
  c.v = ro_at(a.sp_view, g);
  const ViewDev &vw = ro_at(a.views, c.v);
  c.s = g - vw.sp_off;
  c.A = ro_at(a.area, g);
  if (c.A == 0) {
    if (lane == 0) {
      a.planesB[g] = make_float4(0.f, 0.f, 0.f, 0.f);
      a.tabB[2 * g] = make_float4(0.f, 0.f, 0.f, 0.f);
      a.tabB[2 * g + 1] = make_float4(0.f, 0.f, 0.f, 0.f);
      a.energy[g] = 0.f;
      a.choice[g] = -1;
      a.margin[g] = 0.f;
    }
    return;
  }
  c.N = vw.n_pairs;
  c.poff = ro_at(a.px_off, g);
  c.invA = 1.f / (float)c.A;
  const double2 cs = ro_at(a.centroid_d, g);
  ray_of(vw, cs, c.rsx, c.rsy, c.rsz);
  c.Cs = ro_at(a.colour, g);
  c.ub = (int)floor(cs.x + 0.5);
  c.vb = (int)floor(cs.y + 0.5);
  bool fits = true;
  const int n_stage = min(c.A, kLdsPix);
  const int n_pad = (n_stage + kWave - 1) / kWave * kWave;
  for (int p = lane; p < n_pad; p += kWave) {
    uint32_t h = 0x7e007e00u;  // FP16 NaN pair: a pixel that is never seen
    if (p < n_stage) {
      const uint32_t uv = a.px[c.poff + p].x;
      const int du = (int)(uv & 0xffffu) - c.ub, dv = (int)(uv >> 16) - c.vb;
      fits = fits && abs(du) <= 2048 && abs(dv) <= 2048;
      h = __builtin_bit_cast(uint32_t, __floats2half2_rn((float)du, (float)dv));
    }
    pix_lds[p] = h;
  }
  c.n_lds = __ballot(!fits) == 0ull ? n_stage : 0;
  c.n_pad = c.n_lds > 0 ? n_pad : 0;
  c.pix_lds = (const LdsU32 *)pix_lds;
  wave_lds_sync();
  const int gx = c.s % vw.gw, gy = c.s / vw.gw;

  // ring neighbour j on lane j, then into LDS
  int ring_cell = -1;
  double rrx = 0.0, rry = 0.0, rrz = 0.0, ring_d = 0.0;
  float dist2 = INFINITY;
  if (lane < 8) {
    const int x = gx + ring_dx(lane), y = gy + ring_dy(lane);
    if (x >= 0 && x < vw.gw && y >= 0 && y < vw.gh) {
      const int k = y * vw.gw + x;
      const int gk = vw.sp_off + k;
      if (a.area[gk] > 0) {
        ring_cell = k;
        ray_of(vw, a.centroid_d[gk], rrx, rry, rrz);
        ring_d = a.planesA[gk].x;
        const float4 Ck = a.colour[gk];
        const float dr = c.Cs.x - Ck.x, dg = c.Cs.y - Ck.y, db = c.Cs.z - Ck.z;
        dist2 = dr * dr + dg * dg + db * db;
      }
    }
  }
  c.M = __popcll(__ballot(ring_cell >= 0));
  const float dmin2 = ring_min(dist2);
  const float dmax2 = ring_max(ring_cell >= 0 ? dist2 : -INFINITY);
  const float ring_w = ring_cell >= 0 ? __expf(-(dist2 - dmin2) * a.inv2alpha2) : 0.f;
  c.omega_min = c.M > 0 ? __expf(-dmax2 * a.inv2alpha2) : 1.f;
  LdsRing *ring = (LdsRing *)wl.ring;
  if (lane < 8) lds_put(ring + lane, RingEntry{rrx, rry, rrz, ring_d, ring_w, ring_cell});
  c.ring = ring;
  c.vc = (LdsViewConst *)wl.vc;
  c.best = (LdsBest *)&wl.best;
  c.tview = (LdsF32 *)wl.tview;
  c.vorder = (LdsU8 *)wl.vorder;
  wave_lds_sync();

  Best b;
  b.E = -INFINITY;
  b.second = -INFINITY;
  b.slot = -1;
  b.evaluated = 0;
  b.pruned = 0;
  b.view_samples = 0;
  b.ordered = false;

  // Propagation (Sec. III-C, eq. 4): slot r = 0 the current plane, 1 + j ring
  // neighbour j, 9 + 8 (m / step - 1) + j the cell m cells away along ring
  // direction j, m = step, 2 step, ... <= floor(R_init / I).  A candidate is
  // the neighbour's 3D plane; it is skipped when its cell is outside the
  // grid or empty, or when the plane does not face camera r at this centroid.
  const int R = vw.kr_init / a.iter;
  const int n_raw = 9 + 8 * (R / a.kernel_step);
  for (int r0 = 0; r0 < n_raw; r0 += kCandBatch) {
    const int r = r0 + lane;
    bool valid = false;
    Cand cd;
    cd.slot = r;
    cd.pad = 0;
    if (r < n_raw) {
      int x = gx, y = gy;
      if (r >= 1 && r <= 8) {
        x += ring_dx(r - 1);
        y += ring_dy(r - 1);
      } else if (r >= 9) {
        const int m = a.kernel_step * ((r - 9) / 8 + 1), j = (r - 9) % 8;
        x += m * ring_dx(j);
        y += m * ring_dy(j);
      }
      if (x >= 0 && x < vw.gw && y >= 0 && y < vw.gh) {
        const int gk = vw.sp_off + y * vw.gw + x;
        if (a.area[gk] > 0) {
          const float4 pk = a.planesA[gk];
          double rx, ry, rz;
          ray_of(vw, a.centroid_d[gk], rx, ry, rz);
          cd.nx = pk.y;
          cd.ny = pk.z;
          cd.nz = pk.w;
          cd.delta = (double)pk.x * (cd.nx * rx + cd.ny * ry + cd.nz * rz);
          const double tt = cd.nx * c.rsx + cd.ny * c.rsy + cd.nz * c.rsz;
          valid = tt > 0.0 && cd.delta > 0.0;
        }
      }
    }
    const int n = append_cand(list, 0, valid, cd);
    wave_lds_sync();
    evaluate<FMT>(a, c, vw, list, n, b);
    wave_lds_sync();
  }

  // Triangle normals (Sec. III-C): lane j < 8 forms the plane through X_s
  // (the winner's centroid depth) and the 3D centroids of ring neighbours j
  // and j+1 at their depths in the state, in FP64.
  if (b.slot >= 0) {
    bool valid = false;
    Cand cd;
    cd.slot = 1000 + lane;
    cd.pad = 0;
    cd.nx = cd.ny = cd.nz = cd.delta = 0.0;
    RingEntry ra, rb;
    ra.cell = rb.cell = -1;
    if (lane < 8) {
      ra = lds_get(c.ring + lane);
      rb = lds_get(c.ring + ((lane + 1) & 7));
    }
    if (lane < 8 && ra.cell >= 0 && rb.cell >= 0) {
      const double dbb = rb.d, rbx = rb.rx, rby = rb.ry, rbz = rb.rz;
      const double bd = c.best->d;
      const double Xs0 = bd * c.rsx, Xs1 = bd * c.rsy, Xs2 = bd * c.rsz;
      const double ea0 = ra.d * ra.rx - Xs0, ea1 = ra.d * ra.ry - Xs1, ea2 = ra.d * ra.rz - Xs2;
      const double eb0 = dbb * rbx - Xs0, eb1 = dbb * rby - Xs1, eb2 = dbb * rbz - Xs2;
      double n0 = ea1 * eb2 - ea2 * eb1;
      double n1 = ea2 * eb0 - ea0 * eb2;
      double n2 = ea0 * eb1 - ea1 * eb0;
      const double len = sqrt(n0 * n0 + n1 * n1 + n2 * n2);
      const double la = sqrt(ea0 * ea0 + ea1 * ea1 + ea2 * ea2), lb = sqrt(eb0 * eb0 + eb1 * eb1 + eb2 * eb2);
      if (len > 1e-12 * la * lb) {
        n0 /= len;
        n1 /= len;
        n2 /= len;
        double tt = n0 * c.rsx + n1 * c.rsy + n2 * c.rsz;
        if (tt < 0.0) {
          n0 = -n0;
          n1 = -n1;
          n2 = -n2;
          tt = -tt;
        }
        cd.nx = n0;
        cd.ny = n1;
        cd.nz = n2;
        cd.delta = n0 * Xs0 + n1 * Xs1 + n2 * Xs2;
        valid = tt > 0.0 && cd.delta > 0.0;
      }
    }
    const int n = append_cand(list, 0, valid, cd);
    wave_lds_sync();
    evaluate<FMT>(a, c, vw, list, n, b);
  }

  if (lane == 0) {
    if (b.slot < 0) {  // no valid candidate: keep the current plane
      a.planesB[g] = a.planesA[g];
      a.tabB[2 * g] = a.tabA[2 * g];
      a.tabB[2 * g + 1] = a.tabA[2 * g + 1];
      a.energy[g] = -INFINITY;
      a.choice[g] = -1;
      a.margin[g] = 0.f;
    } else {
      const double bnx = c.best->nx, bny = c.best->ny, bnz = c.best->nz;
      a.planesB[g] = make_float4((float)c.best->d, (float)bnx, (float)bny, (float)bnz);
      const double id = 1.0 / c.best->delta;
      a.tabB[2 * g] = c.Cs;
      a.tabB[2 * g + 1] = make_float4((float)((bnx * vw.Kinv_d[0] + bny * vw.Kinv_d[3] + bnz * vw.Kinv_d[6]) * id),
                                      (float)((bnx * vw.Kinv_d[1] + bny * vw.Kinv_d[4] + bnz * vw.Kinv_d[7]) * id),
                                      (float)((bnx * vw.Kinv_d[2] + bny * vw.Kinv_d[5] + bnz * vw.Kinv_d[8]) * id),
                                      0.f);
      a.energy[g] = b.E;
      a.choice[g] = b.slot;
      a.margin[g] = b.evaluated > 1 ? b.E - b.second : INFINITY;
    }
    atomicAdd(&a.work[0], (unsigned long long)b.evaluated);
    atomicAdd(&a.work[1], (unsigned long long)b.view_samples * (unsigned long long)c.A);
    atomicAdd(&a.work[2], (unsigned long long)b.pruned);
  }
}

// Five waves per SIMD (at most 96 VGPRs): the sample loop waits on dependent
// gathers, and the extra wave hides more of that latency than the few
// registers it costs (spilled only around candidate generation).
//
// Persistent: a grid that fills the chip once, each wave claiming superpixels
// from its XCD's queue (for_each_claimed: contiguous ranges in raster order
// per XCD, so a queue's gathers stay inside that XCD's L2, then the other
// queues once its own is drained).  Superpixel costs vary with area and with
// how many candidates survive the bound, and a static one-wave-per-superpixel
// grid left the last waves of each view running alone (on the 4x4 720p rig
// the claim loop takes a frame from 58.1 to 52.7 ms; with the arguments read
// through the constant address space the loop fits in 96 VGPRs).
template <int FMT>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(kRefineWaves))) void k_refine(
    const RefineArgs *__restrict__ args, int *__restrict__ counters) {
  __shared__ WaveLds s_wave[kWavesPerBlock];
  // The arguments sit in device memory, read through the constant address
  // space: fields load into scalar registers where they are used instead of
  // all at entry, which halves the scalar registers spilled around the
  // candidate loop (the sweep, whose loops read its arguments throughout,
  // ran 35 % slower this way and keeps them as kernel arguments).
  typedef const __attribute__((address_space(4))) RefineArgs ConstRefine;
  const RefineArgs &a = *(const RefineArgs *)&*(ConstRefine *)args;
  const int wid = threadIdx.x >> 6;
  for_each_claimed(a.S, counters, [&](int c) { refine_sp<FMT>(a, a.order ? ro_at(a.order, c) : c, s_wave[wid]); });
}

hipError_t launch_refine(int fmt, const RefineArgs &a, RefineArgs *slot, int *counters, int n_cu, hipStream_t st) {
  const void *k = fmt == SLF_FMT_U8    ? (const void *)k_refine<SLF_FMT_U8>
                  : fmt == SLF_FMT_F16 ? (const void *)k_refine<SLF_FMT_F16>
                                       : (const void *)k_refine<SLF_FMT_F32>;
  hipLaunchKernelGGL(k_put_args_reset<RefineArgs>, dim3(1), dim3(64), 0, st, slot, a, counters);
  const RefineArgs *args = slot;
  void *kargs[] = {(void *)&args, (void *)&counters};
  return hipLaunchKernel(k, dim3(persistent_blocks(k, n_cu, a.S)), dim3(kBlock), kargs, 0, st);
}

// ------------------------------------------------------------------ pooled persistent launch
// Many rigs in one launch.  Work items (`tile` consecutive superpixels of
// one job) are claimed from kPoolQueues queues; a wave drains the queue of
// its own XCD (workgroup b runs on XCD b mod 8) and then steals from the
// others in turn, so every wave exits once all queues are empty.  Each item
// runs the same per-superpixel device functions as the per-rig kernels.

typedef const __attribute__((address_space(4))) PoolStage ConstStage;

template <int OP, int FMT, int KC>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(OP == SLF_OP_REFINE ? kRefineWaves : KC <= 8 ? kSweepWaves : 1))) void k_pool(const PoolStage *__restrict__ stage_ptr, int *__restrict__ counters) {
  __shared__ WaveLds s_wave[OP == SLF_OP_REFINE ? kWavesPerBlock : 1];
  // The stage table does not change during the launch: read it through the
  // constant address space, as kernel arguments are, so that its fields are
  // loaded into scalar registers.
  ConstStage &st = *(ConstStage *)stage_ptr;
  const int wid = OP == SLF_OP_REFINE ? (int)(threadIdx.x >> 6) : 0;
  const int home = (int)(blockIdx.x % kPoolQueues);
  const int njobs = st.njobs, tile = st.tile;
  for (int k = 0; k < kPoolQueues; ++k) {
    const int q = (home + k) % kPoolQueues;
    const int begin = st.qbegin[q], end = st.qend[q];
    int *next = counters + q * kPoolCounterStride;
    for (;;) {
      const int item = begin + claim(next);
      if (item >= end) break;
      int lo = 0, hi = njobs - 1;  // the job holding the item
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (st.jobs[mid].item_begin <= item) lo = mid;
        else hi = mid - 1;
      }
      lo = __builtin_amdgcn_readfirstlane(lo);
      const PoolJob &J = *(const PoolJob *)&st.jobs[lo];
      if constexpr (OP == SLF_OP_SWEEP) {
        const int split = J.split;
        const int t = item - J.item_begin;
        const int part = t % split;
        const int g0 = (t / split) * tile;
        const int g1 = min(g0 + tile, J.S);
        for (int c = g0; c < g1; ++c) {  // claims in the rig's strip order (index order without one)
          const int g = J.sweep.order ? ro_at(J.sweep.order, c) : c;
          if (split == 1)
            sweep_sp<FMT, KC>(J.sweep, g);
          else
            sweep_part<FMT, KC>(J.sweep, g, part, split, st.parts + J.part_base + (int64_t)g * split);
        }
      } else {
        const int g0 = (item - J.item_begin) * tile;
        const int g1 = min(g0 + tile, J.S);
        for (int c = g0; c < g1; ++c) refine_sp<FMT>(J.refine, J.refine.order ? ro_at(J.refine.order, c) : c, s_wave[wid]);
      }
    }
  }
}

template <int OP, int FMT>
static const void *pool_kernel(int kc) {
  if constexpr (OP == SLF_OP_REFINE) {  // the refinement has no level chunk
    return (const void *)k_pool<OP, FMT, 8>;
  } else {
    switch (kc) {
      case 4: return (const void *)k_pool<OP, FMT, 4>;
      case 16: return (const void *)k_pool<OP, FMT, 16>;
      default: return (const void *)k_pool<OP, FMT, 8>;
    }
  }
}

static const void *pool_kernel(int op, int fmt, int kc) {
  if (op == SLF_OP_SWEEP) {
    switch (fmt) {
      case SLF_FMT_U8: return pool_kernel<SLF_OP_SWEEP, SLF_FMT_U8>(kc);
      case SLF_FMT_F16: return pool_kernel<SLF_OP_SWEEP, SLF_FMT_F16>(kc);
      default: return pool_kernel<SLF_OP_SWEEP, SLF_FMT_F32>(kc);
    }
  }
  switch (fmt) {
    case SLF_FMT_U8: return pool_kernel<SLF_OP_REFINE, SLF_FMT_U8>(kc);
    case SLF_FMT_F16: return pool_kernel<SLF_OP_REFINE, SLF_FMT_F16>(kc);
    default: return pool_kernel<SLF_OP_REFINE, SLF_FMT_F32>(kc);
  }
}

int pool_occupancy(int op, int fmt, int kc) {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, pool_kernel(op, fmt, kc), kBlock, 0) != hipSuccess) return 0;
  return n;
}

// Merges the level parts of every superpixel of a split sweep stage (one
// thread per superpixel, grid-stride, so the launch shape does not depend on
// the batch).
__global__ __launch_bounds__(256) void k_sweep_merge(const PoolStage *__restrict__ stage_ptr) {
  ConstStage &st = *(ConstStage *)stage_ptr;
  const int njobs = st.njobs, total = st.total_sp;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (st.jobs[mid].sp_begin <= i) lo = mid;
      else hi = mid - 1;
    }
    const PoolJob &J = *(const PoolJob *)&st.jobs[lo];
    if (J.split <= 1) continue;
    const int g = i - J.sp_begin;
    sweep_merge(J.sweep, g, J.split, st.parts + J.part_base + (int64_t)g * J.split);
  }
}

hipError_t launch_pool(int op, int fmt, int kc, bool merge, const PoolStage *stage, int *counters, int blocks,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_pool_reset, dim3(1), dim3(64), 0, st, counters);
  void *args[] = {(void *)&stage, (void *)&counters};
  const hipError_t e = hipLaunchKernel(pool_kernel(op, fmt, kc), dim3(blocks), dim3(kBlock), args, 0, st);
  if (e != hipSuccess) return e;
  if (merge) hipLaunchKernelGGL(k_sweep_merge, dim3(1024), dim3(256), 0, st, stage);
  return hipGetLastError();
}

// ------------------------------------------------------------------ warm start
// Each grid cell keeps its 3D plane from the previous frame: the stored
// inverse-depth row g (1/D(p) = g . p~) is unchanged, and the depth at the
// new centroid is 1 / (g . c~).  A cell that was empty before, or whose plane
// no longer faces the camera at its new centroid, starts fronto-parallel at
// depth d_fb.
__global__ void k_warm(const ViewDev *__restrict__ views, const int *__restrict__ sp_view,
                       const int *__restrict__ area, const double2 *__restrict__ cen,
                       const float4 *__restrict__ colour, float4 *planes, float4 *tab, int S, double d_fb) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= S) return;
  const float4 C = colour[g];
  if (area[g] == 0) {
    planes[g] = make_float4(0.f, 0.f, 0.f, 0.f);
    tab[2 * g] = C;
    tab[2 * g + 1] = make_float4(0.f, 0.f, 0.f, 0.f);
    return;
  }
  const float4 P = planes[g];
  const float4 G = tab[2 * g + 1];
  const double2 c = cen[g];
  const double inv = (double)G.x * c.x + (double)G.y * c.y + (double)G.z;
  float4 outP, outG;
  if (P.x > 0.f && inv > 0.0) {
    outP = make_float4((float)(1.0 / inv), P.y, P.z, P.w);
    outG = G;
  } else {
    const ViewDev &vw = views[sp_view[g]];
    outP = make_float4((float)d_fb, 0.f, 0.f, 1.f);
    outG = make_float4((float)(vw.Kinv_d[6] / d_fb), (float)(vw.Kinv_d[7] / d_fb), (float)(vw.Kinv_d[8] / d_fb), 0.f);
  }
  planes[g] = outP;
  tab[2 * g] = C;
  tab[2 * g + 1] = outG;
}

hipError_t launch_warm(const ViewDev *views, const int *sp_view, const int *area, const double2 *cen,
                       const float4 *colour, float4 *planes, float4 *tab, int S, double d_fb, hipStream_t st) {
  hipLaunchKernelGGL(k_warm, dim3((S + 255) / 256), dim3(256), 0, st, views, sp_view, area, cen, colour, planes, tab,
                     S, d_fb);
  return hipGetLastError();
}

// ------------------------------------------------------------------ depth readout (a9)
// D(p) = 1 / (g_s . p~) for s = label(p), 0 where the plane does not face the camera.
__global__ __launch_bounds__(256) void k_depth(const int *labels, int W, int H, int K, int sp_off, const float4 *tab,
                                               float *out, int64_t stride) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)W * H) return;
  const int x = (int)(idx % W), y = (int)(idx / W);
  int l = labels[idx];
  l = min(max(l, 0), K - 1);
  const float4 gt = tab[2 * (sp_off + l) + 1];
  const float den = fmaf(gt.x, (float)x, fmaf(gt.y, (float)y, gt.z));
  out[(int64_t)y * stride + x] = den > 0.f ? 1.f / den : 0.f;
}

hipError_t launch_depth(const ViewDev *, const ViewDev &vh, int, const int *labels, const float4 *tab, float *out,
                        int64_t stride, hipStream_t st) {
  const int64_t n = (int64_t)vh.W * vh.H;
  hipLaunchKernelGGL(k_depth, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, labels + vh.pix_off, vh.W, vh.H,
                     vh.gw * vh.gh, vh.sp_off, tab, out, stride);
  return hipGetLastError();
}

}  // namespace slf
