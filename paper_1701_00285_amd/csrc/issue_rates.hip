// Issue-rate probe for the pair kernels' instruction mix on gfx950: cycles per
// instruction group per SIMD for the matrix-core forms the distance Gram uses,
// for the kernel-value VALU sequence (sqrt, exp2, two FMAs), and for the two
// interleaved in one wave.  It shows which MFMA forms execute beside the
// VALU (their mixed cost is close to the larger of the two) and which hold
// it (the mixed cost is the sum).
//
//   paper_1701_00285_amd/issue_rates        (built with the library)
//
// Every kernel writes one float per thread into a buffer sized for the
// largest grid; nothing else is read or written.
#include <hip/hip_runtime.h>

#include <cstdio>

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef short s4 __attribute__((ext_vector_type(4)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));

constexpr int kThreads = 256;

// the kernel-value work of one pair in the matrix-core kernel
#define PAIR_VALUE(s, r)                                                                 \
  {                                                                                      \
    const float e = __builtin_amdgcn_exp2f(-__builtin_amdgcn_sqrtf(fabsf(s)));          \
    r = fmaf(e, 0.5f, r);                                                                \
    c0 = fmaf(e, s, c0);                                                                 \
    s += 1e-7f;                                                                          \
  }

// four independent accumulators keep the matrix core busy back to back
#define MFMA4(OP, a, b) \
  g0 = OP(a, b, g0, 0, 0, 0); g1 = OP(a, b, g1, 0, 0, 0); g2 = OP(a, b, g2, 0, 0, 0); g3 = OP(a, b, g3, 0, 0, 0);

// one MFMA, then VALU instructions, four times
#define INTERLEAVE(nv)                                      \
  for (int q = 0; q < 4; ++q) {                             \
    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);      \
    __builtin_amdgcn_sched_group_barrier(0x002, nv, 0);     \
  }

__global__ __launch_bounds__(kThreads) void mfma_f32(float* out, int iters, float a0) {
  f4 g0 = {0, 0, 0, 0}, g1 = g0, g2 = g0, g3 = g0;
  const float a = a0 + threadIdx.x, b = a0 * 2.0f;
  for (int i = 0; i < iters; ++i) { MFMA4(__builtin_amdgcn_mfma_f32_16x16x4f32, a, b) }
  out[blockIdx.x * kThreads + threadIdx.x] = g0[0] + g1[1] + g2[2] + g3[3];
}

__global__ __launch_bounds__(kThreads) void mfma_bf16_k16(float* out, int iters, float a0) {
  f4 g0 = {0, 0, 0, 0}, g1 = g0, g2 = g0, g3 = g0;
  const s4 a = {(short)threadIdx.x, 1, 2, 3}, b = {4, 5, 6, (short)a0};
  for (int i = 0; i < iters; ++i) { MFMA4(__builtin_amdgcn_mfma_f32_16x16x16bf16_1k, a, b) }
  out[blockIdx.x * kThreads + threadIdx.x] = g0[0] + g1[1] + g2[2] + g3[3];
}

__global__ __launch_bounds__(kThreads) void mfma_f16_k32(float* out, int iters, float a0) {
  f4 g0 = {0, 0, 0, 0}, g1 = g0, g2 = g0, g3 = g0;
  h8 a, b;
  for (int e = 0; e < 8; ++e) {
    a[e] = (_Float16)(a0 + threadIdx.x + e);
    b[e] = (_Float16)(a0 * e);
  }
  for (int i = 0; i < iters; ++i) { MFMA4(__builtin_amdgcn_mfma_f32_16x16x32_f16, a, b) }
  out[blockIdx.x * kThreads + threadIdx.x] = g0[0] + g1[1] + g2[2] + g3[3];
}

__global__ __launch_bounds__(kThreads) void pair_values(float* out, int iters, float a0) {
  float s0 = a0 + threadIdx.x * 1e-3f, s1 = s0 + 1, s2 = s0 + 2, s3 = s0 + 3;
  float r0 = 0, r1 = 0, r2 = 0, r3 = 0, c0 = 0;
  for (int i = 0; i < iters; ++i) { PAIR_VALUE(s0, r0) PAIR_VALUE(s1, r1) PAIR_VALUE(s2, r2) PAIR_VALUE(s3, r3) }
  out[blockIdx.x * kThreads + threadIdx.x] = r0 + r1 + r2 + r3 + c0;
}

__global__ __launch_bounds__(kThreads) void fma_only(float* out, int iters, float a0) {
  float r0 = a0, r1 = a0 + 1, r2 = a0 + 2, r3 = a0 + 3;
  const float b = threadIdx.x * 1e-3f;
  for (int i = 0; i < iters; ++i) {
    r0 = fmaf(r0, b, 0.5f);
    r1 = fmaf(r1, b, 0.5f);
    r2 = fmaf(r2, b, 0.5f);
    r3 = fmaf(r3, b, 0.5f);
  }
  out[blockIdx.x * kThreads + threadIdx.x] = r0 + r1 + r2 + r3;
}

__global__ __launch_bounds__(kThreads) void fma_f64(float* out, int iters, float a0) {
  double r0 = a0, r1 = a0 + 1, r2 = a0 + 2, r3 = a0 + 3;
  const double b = threadIdx.x * 1e-3;
  for (int i = 0; i < iters; ++i) {
    r0 = fma(r0, b, 0.5);
    r1 = fma(r1, b, 0.5);
    r2 = fma(r2, b, 0.5);
    r3 = fma(r3, b, 0.5);
  }
  out[blockIdx.x * kThreads + threadIdx.x] = (float)(r0 + r1 + r2 + r3);
}

// the FP64 pair kernels' one hardware transcendental: reciprocal square root
__global__ __launch_bounds__(kThreads) void rsq_f64(float* out, int iters, float a0) {
  double r0 = a0 + threadIdx.x, r1 = r0 + 1, r2 = r0 + 2, r3 = r0 + 3;
  for (int i = 0; i < iters; ++i) {
    r0 = __builtin_amdgcn_rsq(r0) + 1.0;
    r1 = __builtin_amdgcn_rsq(r1) + 1.0;
    r2 = __builtin_amdgcn_rsq(r2) + 1.0;
    r3 = __builtin_amdgcn_rsq(r3) + 1.0;
  }
  out[blockIdx.x * kThreads + threadIdx.x] = (float)(r0 + r1 + r2 + r3);
}

// FP32 sqrt and exp2 alone (with one add each to keep the chains live)
__global__ __launch_bounds__(kThreads) void trans_f32(float* out, int iters, float a0) {
  float r0 = a0 + threadIdx.x, r1 = r0 + 1, r2 = r0 + 2, r3 = r0 + 3;
  for (int i = 0; i < iters; ++i) {
    r0 = __builtin_amdgcn_exp2f(-__builtin_amdgcn_sqrtf(r0)) + 1.0f;
    r1 = __builtin_amdgcn_exp2f(-__builtin_amdgcn_sqrtf(r1)) + 1.0f;
    r2 = __builtin_amdgcn_exp2f(-__builtin_amdgcn_sqrtf(r2)) + 1.0f;
    r3 = __builtin_amdgcn_exp2f(-__builtin_amdgcn_sqrtf(r3)) + 1.0f;
  }
  out[blockIdx.x * kThreads + threadIdx.x] = r0 + r1 + r2 + r3;
}

__global__ __launch_bounds__(kThreads) void mix_f32(float* out, int iters, float a0) {
  f4 g0 = {0, 0, 0, 0}, g1 = g0, g2 = g0, g3 = g0;
  const float a = a0 + threadIdx.x, b = a0 * 2.0f;
  float s0 = a0 + threadIdx.x * 1e-3f, s1 = s0 + 1, s2 = s0 + 2, s3 = s0 + 3;
  float r0 = 0, r1 = 0, r2 = 0, r3 = 0, c0 = 0;
  for (int i = 0; i < iters; ++i) {
    MFMA4(__builtin_amdgcn_mfma_f32_16x16x4f32, a, b)
    PAIR_VALUE(s0, r0) PAIR_VALUE(s1, r1) PAIR_VALUE(s2, r2) PAIR_VALUE(s3, r3)
    INTERLEAVE(5)
  }
  out[blockIdx.x * kThreads + threadIdx.x] = g0[0] + g1[1] + g2[2] + g3[3] + r0 + r1 + r2 + r3 + c0;
}

__global__ __launch_bounds__(kThreads) void mix_f32_fma(float* out, int iters, float a0) {
  f4 g0 = {0, 0, 0, 0}, g1 = g0, g2 = g0, g3 = g0;
  const float a = a0 + threadIdx.x, b = a0 * 2.0f;
  float r0 = a0, r1 = a0 + 1, r2 = a0 + 2, r3 = a0 + 3;
  const float c = threadIdx.x * 1e-3f;
  for (int i = 0; i < iters; ++i) {
    MFMA4(__builtin_amdgcn_mfma_f32_16x16x4f32, a, b)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      r0 = fmaf(r0, c, 0.5f);
      r1 = fmaf(r1, c, 0.5f);
      r2 = fmaf(r2, c, 0.5f);
      r3 = fmaf(r3, c, 0.5f);
    }
    INTERLEAVE(4)
  }
  out[blockIdx.x * kThreads + threadIdx.x] = g0[0] + g1[1] + g2[2] + g3[3] + r0 + r1 + r2 + r3;
}

__global__ __launch_bounds__(kThreads) void mix_bf16_k16(float* out, int iters, float a0) {
  f4 g0 = {0, 0, 0, 0}, g1 = g0, g2 = g0, g3 = g0;
  const s4 a = {(short)threadIdx.x, 1, 2, 3}, b = {4, 5, 6, (short)a0};
  float s0 = a0 + threadIdx.x * 1e-3f, s1 = s0 + 1, s2 = s0 + 2, s3 = s0 + 3;
  float r0 = 0, r1 = 0, r2 = 0, r3 = 0, c0 = 0;
  for (int i = 0; i < iters; ++i) {
    MFMA4(__builtin_amdgcn_mfma_f32_16x16x16bf16_1k, a, b)
    PAIR_VALUE(s0, r0) PAIR_VALUE(s1, r1) PAIR_VALUE(s2, r2) PAIR_VALUE(s3, r3)
    INTERLEAVE(5)
  }
  out[blockIdx.x * kThreads + threadIdx.x] = g0[0] + g1[1] + g2[2] + g3[3] + r0 + r1 + r2 + r3 + c0;
}

__global__ __launch_bounds__(kThreads) void mix_f16_k32(float* out, int iters, float a0) {
  f4 g0 = {0, 0, 0, 0}, g1 = g0, g2 = g0, g3 = g0;
  h8 a, b;
  for (int e = 0; e < 8; ++e) {
    a[e] = (_Float16)(a0 + threadIdx.x + e);
    b[e] = (_Float16)(a0 * e);
  }
  float s0 = a0 + threadIdx.x * 1e-3f, s1 = s0 + 1, s2 = s0 + 2, s3 = s0 + 3;
  float r0 = 0, r1 = 0, r2 = 0, r3 = 0, c0 = 0;
  for (int i = 0; i < iters; ++i) {
    MFMA4(__builtin_amdgcn_mfma_f32_16x16x32_f16, a, b)
    PAIR_VALUE(s0, r0) PAIR_VALUE(s1, r1) PAIR_VALUE(s2, r2) PAIR_VALUE(s3, r3)
    INTERLEAVE(5)
  }
  out[blockIdx.x * kThreads + threadIdx.x] = g0[0] + g1[1] + g2[2] + g3[3] + r0 + r1 + r2 + r3 + c0;
}

}  // namespace

int main() {
  constexpr int kMaxWavesPerSimd = 8, kSimds = 1024, kIters = 20000;
  const int max_blocks = kSimds * kMaxWavesPerSimd / (kThreads / 64);
  float* out = nullptr;
  if (hipMalloc(&out, (size_t)max_blocks * kThreads * sizeof(float)) != hipSuccess) {
    printf("hipMalloc failed\n");
    return 1;
  }
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return 1;
  struct Case {
    const char* name;
    void (*k)(float*, int, float);
  };
  const Case cases[] = {
      {"mfma 16x16x4 f32", mfma_f32},
      {"mfma 16x16x16 bf16", mfma_bf16_k16},
      {"mfma 16x16x32 f16", mfma_f16_k32},
      {"pair values (sqrt, exp2, 2 fma, add)", pair_values},
      {"fma", fma_only},
      {"fma f64", fma_f64},
      {"rsq f64 + add f64", rsq_f64},
      {"sqrt f32 + exp2 f32 + add", trans_f32},
      {"mfma f32 + pair values", mix_f32},
      {"mfma f32 + 4 fma", mix_f32_fma},
      {"mfma bf16 k16 + pair values", mix_bf16_k16},
      {"mfma f16 k32 + pair values", mix_f16_k32},
  };
  printf("cycles per group per SIMD at 2.4 GHz (group: one MFMA and/or one pair's VALU work, or the named "
         "instructions)\n");
  for (int waves : {8, 2}) {
    const int blocks = kSimds * waves / (kThreads / 64);
    printf("--- %d waves per SIMD\n", waves);
    for (const Case& c : cases) {
      float best = 1e30f;
      for (int rep = 0; rep < 3; ++rep) {
        if (hipEventRecord(e0) != hipSuccess) return 1;
        hipLaunchKernelGGL(c.k, dim3(blocks), dim3(kThreads), 0, 0, out, kIters, 1.0f);
        if (hipEventRecord(e1) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return 1;
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return 1;
        best = ms < best ? ms : best;
      }
      const double groups_per_simd = (double)waves * kIters * 4.0;
      printf("%-40s %8.3f ms  %6.2f cycles\n", c.name, best, best * 1e-3 * 2.4e9 / groups_per_simd);
    }
  }
  if (hipFree(out) != hipSuccess) return 1;
  printf("done\n");
  return 0;
}
