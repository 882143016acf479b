// Shared device helpers for the gfx950 kernels: operand types, MFMA wrappers,
// wave reductions.  Every kernel in this library is written for CDNA4
// (64-wide wavefronts, 16x16 MFMA tiles, 160 KB LDS per CU).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#define IFS_DEV __device__ __forceinline__

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
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
// fp32 operands contracted on the fp64 matrix cores: each fp32 value is
// widened exactly, so the products are exact and only the fp64 sums round.
// Operands in the fp32 form's lane layout; the result rows interleave
// across the lane groups instead: acc[i] = C[4*i + l/16][l % 16].
IFS_DEV f64x4 mfma16(const f32x4 &a, const f32x4 &b, f64x4 acc) {
  acc = __builtin_amdgcn_mfma_f64_16x16x4f64((double)a[0], (double)b[0], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f64_16x16x4f64((double)a[1], (double)b[1], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f64_16x16x4f64((double)a[2], (double)b[2], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f64_16x16x4f64((double)a[3], (double)b[3], acc, 0, 0, 0);
  return acc;
}
IFS_DEV f32x4 mfma16(const bf16x8 &a, const bf16x8 &b, f32x4 acc) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
}
IFS_DEV f32x4 mfma16(const f16x8 &a, const f16x8 &b, f32x4 acc) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, acc, 0, 0, 0);
}

// ---------------------------------------------------------------- grouped launches
// A grouped launch runs one kernel for G independent problems at once, the
// problem index in blockIdx.z; problem g's workspace is problem 0's moved by
// g * gs bytes, so every workspace pointer a kernel receives is moved by
// goff(gs) (null pointers stay null).  gs = 0 is the ungrouped launch.
template <class P>
IFS_DEV P *gsh(P *p, long o) {
  return p ? (P *)((char *)p + o) : p;
}
IFS_DEV long goff(long gs) { return (long)blockIdx.z * gs; }

// ---------------------------------------------------------------- guarded loads
// p[i] if ok, else 0, without a branch around the load: the address falls back
// to p[0] (every array passed here is non-empty), so loads issued back to back
// stay in flight together instead of each waiting behind its own branch.
template <typename F>
IFS_DEV F ld_or0(const F *p, long i, bool ok) {
  const F v = p[ok ? i : 0];
  return ok ? v : F(0);
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

// Row dot product of one wave: sum_{j < cend} a[j] (x[j] - xs[j]) (xs optional),
// 4 floats per lane per load.
IFS_DEV float row_dot(const float *a, const float *x, const float *xs, int cend) {
  // U 16-byte chunks per lane in flight together (one round trip for rows of
  // up to 2048); a chunk past the last whole one re-reads chunk 0 and is
  // skipped, which needs cend >= 4 (true whenever the loop runs)
  constexpr int U = 8;
  const int lane = threadIdx.x & 63;
  const int c4 = cend & ~3;  // whole chunks end here
  float t = 0.f;             // the last cend - c4 elements, one per lane
  if (c4 + lane < cend) t = a[c4 + lane] * (x[c4 + lane] - (xs ? xs[c4 + lane] : 0.f));
  float s[U];
#pragma unroll
  for (int q = 0; q < U; ++q) s[q] = 0.f;
  for (int j0 = 4 * lane; j0 < c4 + 4 * lane; j0 += 256 * U) {
    f32x4 v[U], u[U];
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int j = j0 + 256 * q, jc = j < c4 ? j : 0;
      v[q] = *(const f32x4 *)(a + jc);
      u[q] = *(const f32x4 *)(x + jc);
    }
    if (xs) {
#pragma unroll
      for (int q = 0; q < U; ++q) {
        const int j = j0 + 256 * q, jc = j < c4 ? j : 0;
        u[q] -= *(const f32x4 *)(xs + jc);
      }
    }
#pragma unroll
    for (int q = 0; q < U; ++q)
      if (j0 + 256 * q < c4) {
#pragma unroll
        for (int e = 0; e < 4; ++e) s[q] = fmaf(v[q][e], u[q][e], s[q]);
      }
  }
#pragma unroll
  for (int w = U / 2; w > 0; w /= 2)
#pragma unroll
    for (int q = 0; q < w; ++q) s[q] += s[q + w];
  return wave_sum(s[0] + t);
}

// Block-wide sums of N doubles per thread with one LDS exchange (the same
// summation order as N separate block_sum calls); results valid in thread 0.
template <int NT, int N>
IFS_DEV void block_sums(double (&v)[N], double *sh /* >= N * NT/64 */) {
  const int w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < N; ++k) v[k] = wave_sum(v[k]);
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int k = 0; k < N; ++k) sh[k * (NT / 64) + w] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < N; ++k) {
      double r = 0.0;
#pragma unroll
      for (int i = 0; i < NT / 64; ++i) r += sh[k * (NT / 64) + i];
      v[k] = r;
    }
  }
  __syncthreads();
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

// Stages rows [g0, g0 + R) of a row-major [n][D] array into LDS as [R][ld]
// (ld > D).  The real rows are one contiguous run of floats in global memory,
// read as 16-byte vectors, up to 8 in flight per thread; every other element
// (columns >= D, rows >= n) is written as 0, except column onecol (if >= D),
// which holds 1 on real rows and turns a row sum into one more output column
// of a reduction product.  Rows whose start is not 16-byte aligned are read
// with scalar loads.
template <int NT>
IFS_DEV void stage_rows(float *dst, int ld, const float *src, int g0, int R, int n, int D,
                        int onecol) {
  const int tid = threadIdx.x;
  const int rows = max(0, min(R, n - g0));
  const int nreal = rows * D;
  const float *sp = src + (long)g0 * D;
  const int n4 = ((uintptr_t)sp & 15) ? 0 : nreal / 4;
  for (int b0 = 0; b0 < n4; b0 += 8 * NT) {
    f32x4 v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int q = b0 + u * NT + tid;
      v[u] = *(const f32x4 *)(sp + 4 * (q < n4 ? q : 0));
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int q = b0 + u * NT + tid;
      if (q < n4)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int e = 4 * q + j;
          dst[(e / D) * ld + e % D] = v[u][j];
        }
    }
  }
  for (int e0 = 4 * n4; e0 < nreal; e0 += 8 * NT) {
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = ld_or0(sp, e0 + u * NT + tid, e0 + u * NT + tid < nreal);
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * NT + tid;
      if (e < nreal) dst[(e / D) * ld + e % D] = v[u];
    }
  }
  const int padc = ld - D;
  for (int i = tid; i < R * padc; i += NT) {
    const int r = i / padc, d = D + i % padc;
    dst[r * ld + d] = (r < rows && d == onecol) ? 1.f : 0.f;
  }
  for (int i = tid; i < (R - rows) * D; i += NT) dst[(rows + i / D) * ld + i % D] = 0.f;
}

// ---------------------------------------------------------------- SE kernel tiles
// exp of the kernel matrices.  ACC (the fp32 form): the accurate device
// library exp, since the gradient's sums amplify relative errors of K_uu and
// K_uf by their condition; otherwise the hardware exp, whose error is far
// below the rounding of the reduced-precision operands.
template <bool ACC>
IFS_DEV float kexp(float x) {
  if constexpr (ACC) return expf(x);
  else return __expf(x);
}

// Squared scaled distance from norms and cross term (the cross term comes from
// fp32 MFMA); clamped at 0 against rounding.  Used by the reduced-precision
// forms; the fp32 form forms the distances from differences (sqdist).
IFS_DEV float kern_se(float sf2, float zn, float xn, float cross) {
  return sf2 * __expf(-0.5f * fmaxf(zn + xn - 2.f * cross, 0.f));
}

// sum_d (a_d - b_d)^2 over D values of two LDS rows: no cancellation, unlike
// |a|^2 + |b|^2 - 2 a.b, whose rounding grows with the norms of the scaled
// inputs rather than with their distance.
IFS_DEV float sqdist(const float *a, const float *b, int D) {
  float s0 = 0.f, s1 = 0.f;
  int d = 0;
  for (; d + 1 < D; d += 2) {
    const float e0 = a[d] - b[d], e1 = a[d + 1] - b[d + 1];
    s0 = fmaf(e0, e0, s0);
    s1 = fmaf(e1, e1, s1);
  }
  if (d < D) {
    const float e = a[d] - b[d];
    s0 = fmaf(e, e, s0);
  }
  return s0 + s1;
}

// Cross terms C[i][j] = sum_d A[i][d] B[j][d] of a (16 TI) x (16 TJ) block
// from LDS rows A (stride lda) and B (stride ldb), d < D4 (a multiple of 4,
// zero-padded), with 16x16x4 MFMA on TI x TJ independent accumulators:
// acc[i][j][q] = C[16 i + r(q)][16 j + lane % 16] with r(q) = 4 (lane/16) + q
// (fp32 MFMA) or, F64 (fp64 MFMA on the widened values, rounded to fp32 at
// the end), r(q) = 4 q + lane/16: the row layout of the fp64 accumulators.
template <int TI, int TJ, bool F64 = false>
IFS_DEV void cross_block(const float *A, int lda, const float *B, int ldb, int D4,
                         f32x4 (&acc)[TI][TJ]) {
  const int lane = threadIdx.x & 63, l16 = lane & 15, l4 = lane >> 4;
  using Acc = typename std::conditional<F64, f64x4, f32x4>::type;
  Acc c[TI][TJ];
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j) c[i][j] = Acc{0, 0, 0, 0};
  for (int d0 = 0; d0 < D4; d0 += 4) {
    float a[TI], b[TJ];
#pragma unroll
    for (int i = 0; i < TI; ++i) a[i] = A[(i * 16 + l16) * lda + d0 + l4];
#pragma unroll
    for (int j = 0; j < TJ; ++j) b[j] = B[(j * 16 + l16) * ldb + d0 + l4];
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
      for (int j = 0; j < TJ; ++j) {
        if constexpr (F64)
          c[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)a[i], (double)b[j], c[i][j], 0,
                                                         0, 0);
        else
          c[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], c[i][j], 0, 0, 0);
      }
  }
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[i][j][q] = (float)c[i][j][q];
}

// Device-side error flags (sticky until read by the host).
enum : int { FLAG_DOMAIN = 1, FLAG_NONFINITE = 2 };

// Caller arguments of one library call, copied into device memory by k_latch
// at the start of the call.  Kernels take the caller's buffers and scalars
// from here, so their launch arguments name only the context's workspace and
// a recorded launch sequence (a HIP graph) replays for any caller buffers.
constexpr int MAX_NG_LATCH = 64;  // natural-gradient step sizes per latch
struct CallArgs {
  const float *X, *y, *ell, *sf2, *noise, *Z, *m, *s;
  float *L;                     // caller's L (read by the set-up, written by the last NG step)
  const double *grad_scale;     // or null
  double *out_bound, *out_terms, *out_resid;
  float *g_ell, *g_sf2, *g_noise, *g_Z, *g_m, *g_s;
  double c;                     // N / B, the data term's scale
  float ng_tol;                 // stopping threshold of an adaptive NG loop
  float gap_sigma2;             // split sigma^2 of S~ for the variance-gap rule
  int *out_steps;               // NG updates applied by an adaptive loop, or null
  float gammas[MAX_NG_LATCH];   // NG step sizes, from the latch's first step on
};

__global__ void k_latch(CallArgs a, CallArgs *dst) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *dst = a;
}
