// VALU issue-rate probe for gfx950: each kernel runs one instruction form on
// eight independent register chains per lane, on 4096 workgroups of 256
// threads (16 waves per CU for the whole launch), and reports wave
// instructions per CU-clock at the nominal 2.4 GHz.  The forms are the ones
// the sweep and refinement loops are made of; the figures bound what an
// issue-limited kernel of that mix can reach, which the published FP32
// vector peak (counting packed FP32 and FMAs as two operations) does not
// show.  Every form is an ALU instruction written in inline assembly (no
// memory access inside the timed loops); the result of each lane is stored
// once so the chains stay live.
//
// Output: one JSON object per line, {"form": ..., "class": ..., "ms": ...,
// "wave_instr_per_cu_clock": ...}, then a summary line.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>

namespace {

constexpr int kChains = 8;
constexpr int kBlocks = 256 * 16;
constexpr int kThreads = 256;
constexpr int kIters = 2048;

#define PROBE(NAME, T, INIT, ASM, ...)                                                                 \
  __global__ __launch_bounds__(kThreads) void NAME(float *out, int n, float fb, float fc) {            \
    T x[kChains];                                                                                      \
    const float b = fb, c = fc;                                                                        \
    const uint32_t ub = __float_as_uint(fb), uc = __float_as_uint(fc);                                 \
    (void)b; (void)c; (void)ub; (void)uc;                                                              \
    for (int i = 0; i < kChains; ++i) x[i] = INIT;                                                     \
    for (int it = 0; it < n; ++it) {                                                                   \
      _Pragma("unroll") for (int i = 0; i < kChains; ++i) asm volatile(ASM : "+v"(x[i]) : __VA_ARGS__); \
    }                                                                                                  \
    float s = 0.f;                                                                                     \
    for (int i = 0; i < kChains; ++i) s += (float)x[i];                                                \
    out[blockIdx.x * kThreads + threadIdx.x] = s;                                                      \
  }

#define FI (threadIdx.x * 1e-3f + i)
#define UI (threadIdx.x + i)

// FP32 arithmetic, vector operands only
PROBE(p_fmac, float, FI, "v_fmac_f32 %0, %1, %2", "v"(b), "v"(c))
PROBE(p_fma, float, FI, "v_fma_f32 %0, %0, %1, %2", "v"(b), "v"(c))
PROBE(p_mul, float, FI, "v_mul_f32 %0, %0, %1", "v"(b))
PROBE(p_add, float, FI, "v_add_f32 %0, %0, %1", "v"(b))
PROBE(p_add_u32, uint32_t, UI, "v_add_u32 %0, %0, %1", "v"(ub))
// the same with a scalar operand
PROBE(p_fmac_s, float, FI, "v_fmac_f32 %0, %1, %2", "s"(b), "v"(c))
PROBE(p_mul_s, float, FI, "v_mul_f32 %0, %1, %0", "s"(b))
// conversions, min/max, integer multiplies, packed and mixed precision
PROBE(p_cvt_ubyte, float, FI, "v_cvt_f32_ubyte1 %0, %0", "v"(b))
PROBE(p_cvt_rpi, uint32_t, UI, "v_cvt_rpi_i32_f32 %0, %0", "v"(ub))
PROBE(p_fract, float, FI, "v_fract_f32 %0, %0", "v"(b))
PROBE(p_min, float, FI, "v_min_f32 %0, %0, %1", "v"(b))
PROBE(p_mad24, uint32_t, UI, "v_mad_u32_u24 %0, %0, %1, %2", "v"(ub), "v"(uc))
PROBE(p_fma_mix, float, FI, "v_fma_mix_f32 %0, %1, %2, %0 op_sel_hi:[1,0,0]", "v"(ub), "v"(c))
PROBE(p_dot2, float, FI, "v_dot2_f32_f16 %0, %1, %2, %0", "v"(ub), "v"(uc))
PROBE(p_pk_fma16, uint32_t, UI, "v_pk_fma_f16 %0, %0, %1, %2", "v"(ub), "v"(uc))
PROBE(p_dpp, float, FI, "v_add_f32_dpp %0, %0, %0 quad_perm:[1,0,3,2] row_mask:0xf bank_mask:0xf", "v"(b))
PROBE(p_fma64, double, (threadIdx.x * 1e-3 + i), "v_fma_f64 %0, %0, %1, %2", "v"((double)fb), "v"((double)fc))
// transcendentals
PROBE(p_exp, float, FI, "v_exp_f32 %0, %0", "v"(b))
PROBE(p_rcp, float, FI, "v_rcp_f32 %0, %0", "v"(b))
// mixed streams: two instructions per asm block on two chains
#define PROBE2(NAME, ASM)                                                                              \
  __global__ __launch_bounds__(kThreads) void NAME(float *out, int n, float fb, float fc) {            \
    float x[kChains], y[kChains];                                                                      \
    const float b = fb, c = fc;                                                                        \
    for (int i = 0; i < kChains; ++i) {                                                                \
      x[i] = FI;                                                                                       \
      y[i] = FI + 0.5f;                                                                                \
    }                                                                                                  \
    for (int it = 0; it < n; ++it) {                                                                   \
      _Pragma("unroll") for (int i = 0; i < kChains; ++i) asm volatile(ASM : "+v"(x[i]), "+v"(y[i]) : "v"(b), "v"(c), "s"(b)); \
    }                                                                                                  \
    float s = 0.f;                                                                                     \
    for (int i = 0; i < kChains; ++i) s += x[i] + y[i];                                                \
    out[blockIdx.x * kThreads + threadIdx.x] = s;                                                      \
  }
PROBE2(p_fast_slow, "v_fmac_f32 %0, %2, %3\n v_cvt_rpi_i32_f32 %1, %1")
PROBE2(p_fast_exp, "v_fmac_f32 %0, %2, %3\n v_exp_f32 %1, %1")
PROBE2(p_slow_slow, "v_cvt_rpi_i32_f32 %0, %0\n v_cvt_rpi_i32_f32 %1, %1")

typedef void (*Kernel)(float *, int, float, float);
struct Form {
  const char *name, *cls;
  Kernel k;
  int per_block;  // instructions per asm block
};

}  // namespace

int main() {
  float *d = nullptr;
  if (hipMalloc(&d, sizeof(float) * kBlocks * kThreads) != hipSuccess) {
    fprintf(stderr, "hipMalloc failed\n");
    return 1;
  }
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return 1;
  const Form forms[] = {
      {"v_fmac_f32 v,v", "fp32 vector operands", p_fmac, 1},
      {"v_fma_f32 v,v,v", "fp32 vector operands", p_fma, 1},
      {"v_mul_f32 v,v", "fp32 vector operands", p_mul, 1},
      {"v_add_f32 v,v", "fp32 vector operands", p_add, 1},
      {"v_add_u32 v,v", "int32 vector operands", p_add_u32, 1},
      {"v_fmac_f32 s,v", "scalar operand", p_fmac_s, 1},
      {"v_mul_f32 s,v", "scalar operand", p_mul_s, 1},
      {"v_cvt_f32_ubyte1", "conversion", p_cvt_ubyte, 1},
      {"v_cvt_rpi_i32_f32", "conversion", p_cvt_rpi, 1},
      {"v_fract_f32", "fract", p_fract, 1},
      {"v_min_f32", "min/max", p_min, 1},
      {"v_mad_u32_u24", "int multiply", p_mad24, 1},
      {"v_fma_mix_f32", "mixed precision", p_fma_mix, 1},
      {"v_dot2_f32_f16", "packed fp16", p_dot2, 1},
      {"v_pk_fma_f16", "packed fp16", p_pk_fma16, 1},
      {"v_add_f32_dpp", "dpp", p_dpp, 1},
      {"v_fma_f64", "fp64", p_fma64, 1},
      {"v_exp_f32", "transcendental", p_exp, 1},
      {"v_rcp_f32", "transcendental", p_rcp, 1},
      {"v_fmac_f32 + v_cvt_rpi_i32_f32", "mixed stream", p_fast_slow, 2},
      {"v_fmac_f32 + v_exp_f32", "mixed stream", p_fast_exp, 2},
      {"v_cvt_rpi_i32_f32 x2", "mixed stream", p_slow_slow, 2},
  };
  for (const Form &f : forms) {
    float ms = 0.f;
    for (int rep = 0; rep < 3; ++rep) {  // the last of three launches is reported
      if (hipEventRecord(e0) != hipSuccess) return 2;
      hipLaunchKernelGGL(f.k, dim3(kBlocks), dim3(kThreads), 0, 0, d, kIters, 0.999f, 1e-3f);
      if (hipGetLastError() != hipSuccess || hipEventRecord(e1) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
        return 2;
      if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return 2;
    }
    const double waves_instr = (double)kBlocks * kThreads / 64.0 * kIters * kChains * f.per_block;
    const double rate = waves_instr / (ms * 1e-3) / 256.0 / 2.4e9;
    printf("{\"form\": \"%s\", \"class\": \"%s\", \"ms\": %.4f, \"wave_instr_per_cu_clock\": %.3f}\n", f.name, f.cls,
           ms, rate);
  }
  printf("{\"summary\": \"wave64 VALU instructions per CU-clock at 2.4 GHz; 2.0 would be 78.6 T lane-ops/s\"}\n");
  (void)hipFree(d);
  return 0;
}
