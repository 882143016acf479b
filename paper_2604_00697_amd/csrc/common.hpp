// Shared device helpers for the gfx950 kernels: operand types, MFMA wrappers,
// wave reductions.  Every kernel in this library is written for CDNA4
// (64-wide wavefronts, 16x16 MFMA tiles, 160 KB LDS per CU).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#define IFS_DEV __device__ __forceinline__

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------- conversions
template <typename T> IFS_DEV T from_f32(float x);
template <> IFS_DEV float from_f32<float>(float x) { return x; }
template <> IFS_DEV __bf16 from_f32<__bf16>(float x) { return (__bf16)x; }
template <> IFS_DEV _Float16 from_f32<_Float16>(float x) { return (_Float16)x; }

IFS_DEV float to_f32(float x) { return x; }
IFS_DEV float to_f32(__bf16 x) { return (float)x; }
IFS_DEV float to_f32(_Float16 x) { return (float)x; }

// 16 bytes of operands as the MFMA source vector for one lane.
template <typename T> struct Vec16;
template <> struct Vec16<float> { typedef f32x4 type; };
template <> struct Vec16<__bf16> { typedef bf16x8 type; };
template <> struct Vec16<_Float16> { typedef f16x8 type; };

// ---------------------------------------------------------------- MFMA
// One 16x16 output tile, contraction over the 16 bytes each lane holds:
// fp32: 4 successive v_mfma_f32_16x16x4_f32 (k = 16 per call),
// bf16/fp16: one v_mfma_f32_16x16x32 (k = 32 per call).
// Lane l supplies row (l % 16) of A and column (l % 16) of B; the k slot it
// feeds is the same for A and B, so any lane/k assignment contracts exactly.
// Result: acc[i] = C[4*(l/16) + i][l % 16].
IFS_DEV f32x4 mfma16(const f32x4 &a, const f32x4 &b, f32x4 acc) {
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[0], b[0], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[1], b[1], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[2], b[2], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[3], b[3], acc, 0, 0, 0);
  return acc;
}
IFS_DEV f32x4 mfma16(const bf16x8 &a, const bf16x8 &b, f32x4 acc) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
}
IFS_DEV f32x4 mfma16(const f16x8 &a, const f16x8 &b, f32x4 acc) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, acc, 0, 0, 0);
}

// ---------------------------------------------------------------- reductions
IFS_DEV float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
IFS_DEV double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Block-wide sum of one double per thread; result valid in thread 0.
template <int NT>
IFS_DEV double block_sum(double v, double *sh /* >= NT/64 */) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) r += sh[i];
  }
  __syncthreads();
  return r;
}

// Device-side error flags (sticky until read by the host).
enum : int { FLAG_DOMAIN = 1, FLAG_NONFINITE = 2 };
