// VALU issue-rate microbenchmark behind the ALU ceilings that the benchmark
// reports for the sweeps.  Not part of the near-field library: built into a
// library of its own and loaded only by the benchmark.
//
// Each kernel runs independent dependency chains of one instruction mix, so that
// the issue rate and not the latency bounds it; the loop bodies are written
// instruction by instruction (register-only VALU operations in inline assembly,
// so that the compiler neither fuses nor drops any).  The benchmark times every
// mix on the same launch shape with HIP events: lane-operations per second, and
// each mix's cost relative to the FMA mix, in FMA issue slots.
//
// Mixes (per loop trip of one lane; every chain carried from trip to trip):
//   0 fma    16 FP32 FMAs
//   1 trans  16 transcendentals (sin, cos, rsq in turn)
//   2 pair   the FP32 sweep's algorithmic work for one pair: 15 FP32 VALU
//            operations (multiply-adds) and rsq, sin, cos
//   3 issued about the instruction mix the FP32 sweep issues per pair (its
//            counters): 6 FMA, 5 multiplies, 1 add, 4 integer, 4 conversions and
//            3 transcendentals (23 VALU instructions)
//   4 int    16 integer subtractions
//   5 cvt    16 int <-> float conversions and 8 integer subtractions
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kThreads = 256;

#define FMA(x) asm volatile("v_fma_f32 %0, %0, %1, %2" : "+v"(x) : "v"(m), "v"(c))
#define MUL(x) asm volatile("v_mul_f32 %0, %0, %1" : "+v"(x) : "v"(m))
#define ADD(x) asm volatile("v_add_f32 %0, %0, %1" : "+v"(x) : "v"(c))
#define SUB(x, y) asm volatile("v_sub_u32 %0, %0, %1" : "+v"(x) : "v"(y))
#define SIN(x) asm volatile("v_sin_f32 %0, %0" : "+v"(x))
#define COS(x) asm volatile("v_cos_f32 %0, %0" : "+v"(x))
#define RSQ(x) asm volatile("v_rsq_f32 %0, %0" : "+v"(x))
#define CVT_I(y, x) asm volatile("v_cvt_i32_f32 %0, %1" : "=v"(y) : "v"(x))
#define CVT_F(x, y) asm volatile("v_cvt_f32_i32 %0, %1" : "=v"(x) : "v"(y))

template <int MIX>
__global__ void __launch_bounds__(kThreads) k_mix(int iters, float seed, float* __restrict__ sink) {
  const int tid = blockIdx.x * kThreads + threadIdx.x;
  float a[16];
  int b[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    a[i] = 1.0f + seed * (float)(tid + i) * 1e-9f;
    b[i] = tid * 7 + i;
  }
  const float m = 0.999f + seed * 1e-6f, c = 1e-3f * seed;
  for (int it = 0; it < iters; ++it) {
    if constexpr (MIX == 0) {
#pragma unroll
      for (int i = 0; i < 16; ++i) FMA(a[i]);
    } else if constexpr (MIX == 1) {
#pragma unroll
      for (int i = 0; i < 16; i += 4) {
        SIN(a[i]);
        COS(a[i + 1]);
        RSQ(a[i + 2]);  // rsq chains stay positive and tend to 1
        SIN(a[i + 3]);
      }
    } else if constexpr (MIX == 2) {
      // 15 multiply-adds over five chains, three transcendentals on three others
#pragma unroll
      for (int i = 0; i < 15; ++i) {
        FMA(a[i % 5]);
        if (i == 4) RSQ(a[5]);
        if (i == 9) SIN(a[6]);
        if (i == 14) COS(a[7]);
      }
    } else if constexpr (MIX == 3) {
#pragma unroll
      for (int i = 0; i < 6; ++i) FMA(a[i]);
      RSQ(a[14]);
#pragma unroll
      for (int i = 6; i < 11; ++i) MUL(a[i]);
      SIN(a[15]);
      ADD(a[11]);
#pragma unroll
      for (int i = 0; i < 4; ++i) SUB(b[i], b[i + 4]);
      COS(a[13]);
      CVT_I(b[8], a[12]);
      CVT_I(b[9], a[11]);
      CVT_F(a[12], b[10]);
      CVT_F(a[10], b[11]);
    } else if constexpr (MIX == 4) {
#pragma unroll
      for (int i = 0; i < 16; ++i) SUB(b[i], b[(i + 7) & 15]);
    } else {
#pragma unroll
      for (int i = 0; i < 8; ++i) CVT_I(b[i], a[i]);
#pragma unroll
      for (int i = 0; i < 8; ++i) SUB(b[i], b[8]);
#pragma unroll
      for (int i = 0; i < 8; ++i) CVT_F(a[i], b[i]);
    }
  }
  float s = 0.0f;
#pragma unroll
  for (int i = 0; i < 16; ++i) s += a[i] + (float)b[i];
  sink[tid] = s;
}

}  // namespace

extern "C" {

// Work counts per loop trip and lane: VALU operations (transcendentals included)
// and transcendentals, for mix `mix`; -1 for an unknown mix.
int p2p_issue_counts(int mix, int* valu, int* trans) {
  static const int kValu[6] = {16, 16, 18, 23, 16, 24}, kTrans[6] = {0, 16, 3, 3, 0, 0};
  if (mix < 0 || mix > 5 || !valu || !trans) return -1;
  *valu = kValu[mix];
  *trans = kTrans[mix];
  return 0;
}

// Runs mix `mix` on `blocks` workgroups of 256 threads for `iters` loop trips.
// sink: device float[blocks * 256].  *ms: the launch's wall time from HIP events.
// Returns 0, or -1 for a bad argument, or the HIP error code.
int p2p_issue_run(int mix, int blocks, int iters, float* sink, float* ms) {
  if (mix < 0 || mix > 5 || blocks < 1 || iters < 1 || !sink || !ms) return -1;
  void (*kern[6])(int, float, float*) = {k_mix<0>, k_mix<1>, k_mix<2>, k_mix<3>, k_mix<4>, k_mix<5>};
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return (int)hipGetLastError();
  if (hipEventCreate(&e1) != hipSuccess) {
    hipEventDestroy(e0);
    return (int)hipGetLastError();
  }
  hipEventRecord(e0, nullptr);
  hipLaunchKernelGGL(kern[mix], dim3(blocks), dim3(kThreads), 0, nullptr, iters, 1.0f, sink);
  hipEventRecord(e1, nullptr);
  hipError_t e = hipEventSynchronize(e1);
  if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  return e == hipSuccess ? (int)hipGetLastError() : (int)e;
}

}  // extern "C"
