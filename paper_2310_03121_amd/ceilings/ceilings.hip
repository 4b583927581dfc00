// Microbenchmarks of the compute ceilings the roofline objects of the
// benchmark are measured against (a measurement tool, not part of the
// energy/force path):
//   kind 0: v_mfma_f32_16x16x32_bf16 issue loop (16,384 FLOP per instruction)
//   kind 1: v_mfma_f32_16x16x4_f32 issue loop (2,048 FLOP per instruction)
//   kind 2: v_fma_f32 loop (2 FLOP per lane and instruction; packed FP32
//           instructions are switched off in every build, as in the library)
//   kind 3: v_exp_f32 loop (one transcendental per lane and instruction)
// Each wave runs eight independent chains, so issue rather than latency
// bounds the loop; the results are folded into `sink` so nothing is dead.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

constexpr int kChains = 8;

// Eight named accumulators (an array invites the register allocator to
// shuffle them between iterations).
#define NNP_CEIL_ACCS f32x4_t c0 = {0.f, 0.f, 0.f, 0.f}, c1 = c0, c2 = c0, c3 = c0, c4 = c0, \
                              c5 = c0, c6 = c0, c7 = c0
#define NNP_CEIL_FOLD                                                                     \
  const f32x4_t t = ((c0 + c1) + (c2 + c3)) + ((c4 + c5) + (c6 + c7));                  \
  const float s = t[0] + t[1] + t[2] + t[3];                                              \
  if (s == 12345.678f) sink[blockIdx.x] = s;  // never true for these inputs

__global__ __launch_bounds__(256) void k_mfma_bf16(int iters, float* sink) {
  const int lane = threadIdx.x & 63;
  bf16x8_t a, b;
  for (int e = 0; e < 8; ++e) {
    a[e] = (__bf16)(0.001f * (float)(lane + e));
    b[e] = (__bf16)(0.002f * (float)(lane - e));
  }
  NNP_CEIL_ACCS;
#pragma unroll 1
  for (int it = 0; it < iters; ++it) {
    c0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c0, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c1, 0, 0, 0);
    c2 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c2, 0, 0, 0);
    c3 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c3, 0, 0, 0);
    c4 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c4, 0, 0, 0);
    c5 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c5, 0, 0, 0);
    c6 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c6, 0, 0, 0);
    c7 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c7, 0, 0, 0);
  }
  NNP_CEIL_FOLD
}

__global__ __launch_bounds__(256) void k_mfma_f32(int iters, float* sink) {
  const int lane = threadIdx.x & 63;
  const float a = 0.001f * (float)lane, b = 0.002f * (float)(64 - lane);
  NNP_CEIL_ACCS;
#pragma unroll 1
  for (int it = 0; it < iters; ++it) {
    c0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c0, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c1, 0, 0, 0);
    c2 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c2, 0, 0, 0);
    c3 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c3, 0, 0, 0);
    c4 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c4, 0, 0, 0);
    c5 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c5, 0, 0, 0);
    c6 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c6, 0, 0, 0);
    c7 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c7, 0, 0, 0);
  }
  NNP_CEIL_FOLD
}

__global__ __launch_bounds__(256) void k_fma(int iters, float* sink) {
  float x[kChains];
  const float m = 0.999f, q = 1e-4f * (float)(threadIdx.x & 63);
  for (int c = 0; c < kChains; ++c) x[c] = 0.5f + 0.01f * (float)c;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = __builtin_fmaf(x[c], m, q);
  }
  float s = 0.f;
  for (int c = 0; c < kChains; ++c) s += x[c];
  if (s == 12345.678f) sink[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_exp(int iters, float* sink) {
  float x[kChains];
  for (int c = 0; c < kChains; ++c) x[c] = -0.5f - 0.01f * (float)c;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = -__builtin_amdgcn_exp2f(x[c]);  // stays in [-1, -0.5]
  }
  float s = 0.f;
  for (int c = 0; c < kChains; ++c) s += x[c];
  if (s == 12345.678f) sink[blockIdx.x] = s;
}

}  // namespace

extern "C" {

// Work of one launch, in FLOP (kinds 0-2) or transcendentals (kind 3).
double nnp_ceiling_work(int kind, int blocks, int iters) {
  const double waves = (double)blocks * 4.0, lanes = waves * 64.0;
  const double per = (double)iters * kChains;
  switch (kind) {
    case 0: return waves * per * 16384.0;
    case 1: return waves * per * 2048.0;
    case 2: return lanes * per * 2.0;
    case 3: return lanes * per;
  }
  return 0.0;
}

// Enqueues one launch of `kind` (blocks of 256 threads) on `stream`; sink is
// a device float [blocks] that is never written in practice.  Returns 0, or
// -1 for a bad argument or launch.
int nnp_ceiling_launch(int kind, int blocks, int iters, float* sink, void* stream) {
  if (blocks < 1 || iters < 1 || !sink) return -1;
  hipStream_t st = static_cast<hipStream_t>(stream);
  switch (kind) {
    case 0: hipLaunchKernelGGL(k_mfma_bf16, dim3(blocks), dim3(256), 0, st, iters, sink); break;
    case 1: hipLaunchKernelGGL(k_mfma_f32, dim3(blocks), dim3(256), 0, st, iters, sink); break;
    case 2: hipLaunchKernelGGL(k_fma, dim3(blocks), dim3(256), 0, st, iters, sink); break;
    case 3: hipLaunchKernelGGL(k_exp, dim3(blocks), dim3(256), 0, st, iters, sink); break;
    default: return -1;
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // extern "C"
