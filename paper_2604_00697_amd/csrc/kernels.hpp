// Non-GEMM kernels of the iteration: set-up (validation, kernel matrix, layout
// copies), K_uf generation, matrix-vector products, likelihood expectations
// with the fp64 finalisation of the bound, and the gradient reductions.
// Small reductions finish in the last workgroup of the producing kernel
// (device-scope fence + atomic arrival counter; no workgroup ever waits).
#pragma once
#include "common.hpp"

#define NTB 256  // threads per block of the elementwise kernels

// Scalar slots of the context's fp64 buffer.
enum : int {
  S_SUMLOGS = 0,   // sum_i log s~_i
  S_LOGDET = 1,    // log|T| = 2 sum log|L_ii|
  S_QUAD = 2,      // b^T Wu b   (= m~^T P K_uu P m~)
  S_RESID = 3,     // residual of the last NG step
  S_LPD = 4,       // running sum of log predictive densities over a prediction's chunks
  S_NSLOT = 8
};

// Arrival counters (one int each, reset to 0 by the last arriving workgroup).
enum : int { CNT_VEC = 0, CNT_LIK = 1, CNT_GRAD = 2, CNT_N = 4 };

// True in exactly one workgroup of the grid (of one problem's part of a
// grouped grid, whose problems have counters of their own): the last to
// arrive.  Every such workgroup's global writes before the call are visible
// to it.
IFS_DEV bool arrive_last(int *counter, int *s_flag) {
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    const int prev = atomicAdd(counter, 1);
    *s_flag = prev == (int)(gridDim.x * gridDim.y) - 1;
  }
  __syncthreads();
  const bool last = *s_flag != 0;
  if (last) {
    __threadfence();
    if (threadIdx.x == 0) atomicExch(counter, 0);
  }
  return last;
}

// ---------------------------------------------------------------- set-up
// One launch per iteration before any product:
//  * blocks [0, nK): lower 64 x 64 tiles of K~ = sf2 exp(-1/2 |zs_i - zs_j|^2) + diag(s~)
//    and their mirrors
//    (fp32, plus the operand type), zs = Z / ell; the first tile column also
//    writes Zs and the zero-padded copy of s~; block 0 validates ell, sf2,
//    noise_var, s~ and forms 1/ell and sum log s~;
//  * blocks [nK, nK + nL): 64 x 64 tiles of the caller's L: fp32 master (lower
//    triangle, strict upper 0), operand copy, both transposes, and the
//    transpose scaled by s~ along k (operand of L^T S~ L).
struct SetupArgs {
  CallArgs cav;        // the call's arguments when latch is set
  int latch;           // 1: read cav and copy it to *ca; 0: *ca already holds them
  CallArgs *ca;        // Z, ell, sf2, noise, s~ and the caller's L
  int M, D, need_noise;
  float *Zs, *inv_ell, *sP, *Kt;
  float *sfn;          // workspace copies {sf2, noise_var} for the later kernels
  void *KtT;
  long ld;
  float *L32, *Lt32;
  void *LT, *LtT, *LstT;
  double *scal;
  int *flag;
  int *ngskip;         // stop flag of an adaptive NG loop, cleared for the call
  int nKx, nK, nLx;
  // inputs of the generated K_uf tiles (KufGen), when nG > 0: the blocks
  // after workgroup 0, the nK K~ tiles and the nL tiles of L take first
  // 64 rows of Z each (nGz blocks), then 64 rows of the batch (B rows), which
  // also write Xs = X / ell
  int nG, nGz, B, ldk;
  __bf16 *Zh, *Zl, *Xh, *Xl;
  float *zc, *xr, *Xs;
  long gs;             // grouped launch: bytes between the problems' workspaces
  IFS_DEV void shift(long o) {
    ca = gsh(ca, o); Zs = gsh(Zs, o); inv_ell = gsh(inv_ell, o); sP = gsh(sP, o);
    Kt = gsh(Kt, o); sfn = gsh(sfn, o); KtT = gsh((char *)KtT, o); L32 = gsh(L32, o);
    Lt32 = gsh(Lt32, o); LT = gsh((char *)LT, o); LtT = gsh((char *)LtT, o);
    LstT = gsh((char *)LstT, o); scal = gsh(scal, o); flag = gsh(flag, o);
    ngskip = gsh(ngskip, o);
    Zh = gsh(Zh, o); Zl = gsh(Zl, o); Xh = gsh(Xh, o); Xl = gsh(Xl, o); zc = gsh(zc, o);
    xr = gsh(xr, o); Xs = gsh(Xs, o);
  }
};

// sqrt(log2(e) / 2): exp(-d^2 / 2) = 2^(-(c d)^2)
constexpr float KUF_C = 0.84932180028801904272f;

// One row of the generator's inputs: v = c * (row / ell) over d < D, written
// as the hi / lo bf16 split of s v (s = 2 for Z rows, 1 for batch rows;
// zeros for D <= d < ldk); returns |v|^2 (fp32) to the row's four threads.
// Thread q of the row handles d = q, q + 4, ...
IFS_DEV float gen_row(const float *src, const float *ellc, int D, int ldk, float s, int q,
                      __bf16 *hi, __bf16 *lo, float *xs_out) {
  float nrm = 0.f;
  for (int d = q; d < ldk; d += 4) {
    float v = 0.f;
    if (d < D) {
      const float x = src[d] * (1.0f / ellc[d]);
      if (xs_out) xs_out[d] = x;
      v = KUF_C * x;
    }
    nrm = fmaf(v, v, nrm);
    const float w = s * v;
    const __bf16 h = (__bf16)w;
    hi[d] = h;
    lo[d] = (__bf16)(w - (float)h);
  }
  nrm += __shfl_xor(nrm, 1);
  nrm += __shfl_xor(nrm, 2);
  return nrm;
}

// The call's inputs that the set-up reads, taken by value: a pointer into
// the kernel's argument block would make the compiler keep a private copy of
// the whole block in scratch memory.
struct SetupIn {
  const float *X, *ell, *sf2, *noise, *Z, *s, *L;
};
IFS_DEV SetupIn setup_in(const CallArgs &c) {
  return {c.X, c.ell, c.sf2, c.noise, c.Z, c.s, c.L};
}

template <int MAXD, typename T>
__global__ __launch_bounds__(NTB) void k_setup(SetupArgs a) {
  __shared__ float zi[64][MAXD + 1], zj[64][MAXD + 1];
  __shared__ double sh[NTB / 64];
  if (a.gs) a.shift(goff(a.gs));
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (a.latch) *a.ca = a.cav;
    // a stop of an earlier call must not skip this call's first products
    *a.ngskip = 0;
  }
  const int M = a.M, D = a.D;
  const SetupIn ca = a.latch ? setup_in(a.cav) : setup_in(*a.ca);
  const float *Zc = ca.Z, *ellc = ca.ell, *sc = ca.s;
  // workgroup 0: the call's scalars, 1/ell, the domain checks and sum log s~
  // (dispatched first, beside the tiles)
  if (blockIdx.x == 0) {
    int bad = 0;
    for (int d = threadIdx.x; d < D; d += NTB) {
      const float l = ellc[d];
      if (!(l > 0.f) || !isfinite(l)) bad = 1;
      a.inv_ell[d] = 1.0f / l;
    }
    if (threadIdx.x == 0) {
      const float v = *ca.sf2;
      if (!(v > 0.f) || !isfinite(v)) bad = 1;
      a.sfn[0] = v;
      if (a.need_noise) {
        const float n = *ca.noise;
        if (!(n > 0.f) || !isfinite(n)) bad = 1;
        a.sfn[1] = n;
      }
    }
    double acc = 0.0;
    for (int q = threadIdx.x; q < M; q += NTB) {
      const float v = sc[q];
      if (!(v > 0.f) || !isfinite(v)) bad = 1;
      acc += log((double)v);
    }
    acc = block_sum<NTB>(acc, sh);
    if (threadIdx.x == 0) a.scal[S_SUMLOGS] = acc;
    if (bad) atomicOr(a.flag, FLAG_DOMAIN);
    return;
  }
  const int b = (int)blockIdx.x - 1;
  if (b < a.nK) {
    // lower 64 x 64 tile (bi >= bj), its mirror written through LDS; thread
    // (tx, ty) owns rows ty + 16 p and columns tx + 16 q
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    int bi = (int)((sqrtf(8.0f * b + 1.0f) - 1.0f) * 0.5f);
    while ((bi + 1) * (bi + 2) / 2 <= b) ++bi;
    while (bi * (bi + 1) / 2 > b) --bi;
    const int bj = b - bi * (bi + 1) / 2;
    const int i0 = bi * 64, j0 = bj * 64;
    for (int e0 = 0; e0 < 64 * D; e0 += 4 * NTB) {
      float vi[4], vj[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = e0 + u * NTB + (int)threadIdx.x, r = e / D, d = e % D;
        const bool in = e < 64 * D;
        const float il = 1.0f / ld_or0(ellc, d, in);
        vi[u] = ld_or0(Zc, (long)(i0 + r) * D + d, in && i0 + r < M) * il;
        vj[u] = ld_or0(Zc, (long)(j0 + r) * D + d, in && j0 + r < M) * il;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = e0 + u * NTB + (int)threadIdx.x, r = e / D, d = e % D;
        if (e < 64 * D) {
          zi[r][d] = vi[u];
          zj[r][d] = vj[u];
          if (bj == 0 && i0 + r < M) a.Zs[(long)(i0 + r) * D + d] = vi[u];
        }
      }
    }
    if (bj == 0 && threadIdx.x < 64 && i0 + threadIdx.x < M)
      a.sP[i0 + threadIdx.x] = sc[i0 + threadIdx.x];
    __syncthreads();
    float d2[4][4];
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
      for (int q = 0; q < 4; ++q) d2[p][q] = 0.f;
    for (int d = 0; d < D; ++d) {
      float zr[4], zc[4];
#pragma unroll
      for (int p = 0; p < 4; ++p) zr[p] = zi[ty + 16 * p][d];
#pragma unroll
      for (int q = 0; q < 4; ++q) zc[q] = zj[tx + 16 * q][d];
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const float df = zr[p] - zc[q];
          d2[p][q] = fmaf(df, df, d2[p][q]);
        }
    }
    const float sf2 = *ca.sf2;
    float kv[4][4];
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const int i = i0 + ty + 16 * p;
      const float si = ld_or0(sc, i, i < M);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int j = j0 + tx + 16 * q;
        float v = sf2 * kexp<std::is_same<T, float>::value>(-0.5f * d2[p][q]);
        if (i == j) v += si;
        kv[p][q] = v;
        if (i < M && j < M) {
          a.Kt[(long)i * a.ld + j] = v;
          if constexpr (!std::is_same<T, float>::value)
            ((T *)a.KtT)[(long)i * a.ld + j] = from_f32<T>(v);
        }
      }
    }
    if (bi != bj) {
      // the mirror tile [j][i] through LDS (zi is free once the distances are
      // formed)
      __syncthreads();
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) zi[ty + 16 * p][tx + 16 * q] = kv[p][q];
      __syncthreads();
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        const int j = j0 + ty + 16 * p;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int i = i0 + tx + 16 * q;
          if (i < M && j < M) {
            const float v = zi[tx + 16 * q][ty + 16 * p];
            a.Kt[(long)j * a.ld + i] = v;
            if constexpr (!std::is_same<T, float>::value)
              ((T *)a.KtT)[(long)j * a.ld + i] = from_f32<T>(v);
          }
        }
      }
    }
    return;
  }
  const int nL = a.nLx * (a.nLx + 1) / 2;
  if (b >= a.nK + nL) {
    // generator inputs: 64 rows per block, four threads per row
    const int g = b - a.nK - nL, r = threadIdx.x >> 2, q = threadIdx.x & 3;
    // rows past M (or B) within the last block get norm terms of -1e30, so
    // that their generated entries come out as exactly 0 with no mask
    if (g < a.nGz) {
      const int m = g * 64 + r;
      if (m < M) {
        const long o = (long)m * a.ldk;
        const float n = gen_row(Zc + (long)m * D, ellc, D, a.ldk, 2.f, q, a.Zh + o, a.Zl + o,
                                nullptr);
        if (q == 0) a.zc[m] = -n;
      } else if (q == 0) {
        a.zc[m] = -1e30f;
      }
    } else {
      const int n0 = (g - a.nGz) * 64 + r;
      if (n0 < a.B) {
        const long o = (long)n0 * a.ldk;
        const float n = gen_row(ca.X + (long)n0 * D, ellc, D, a.ldk, 1.f, q, a.Xh + o,
                                a.Xl + o, a.Xs + (long)n0 * D);
        const float l2 = log2f(*ca.sf2);
        if (q == 0) a.xr[n0] = l2 - n;
      } else if (q == 0) {
        a.xr[n0] = -1e30f;
      }
    }
    return;
  }
  // caller's L -> L32, LT, LtT, Lt32, LstT on the 64 x 64 tiles with I >= J
  // only (zi serves as the transpose buffer): the strictly upper tiles of L
  // (and the strictly lower ones of the transposes) are zero from the
  // workspace's allocation and no kernel ever writes them
  const int bl = b - a.nK;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;  // 64 x 4
  int I = (int)((sqrtf(8.0f * bl + 1.0f) - 1.0f) * 0.5f);
  while ((I + 1) * (I + 2) / 2 <= bl) ++I;
  while (I * (I + 1) / 2 > bl) --I;
  const int i0 = I * 64, j0 = (bl - I * (I + 1) / 2) * 64;
  float lv[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int i = i0 + ty + 4 * u, j = j0 + tx;
    lv[u] = ld_or0(ca.L, (long)i * M + j, i < M && j < M && i >= j);
  }
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int r = ty + 4 * u;
    const int i = i0 + r, j = j0 + tx;
    const float v = lv[u];
    zi[r][tx] = v;
    if (i < M && j < M) {
      a.L32[(long)i * a.ld + j] = v;
      if constexpr (!std::is_same<T, float>::value) ((T *)a.LT)[(long)i * a.ld + j] = from_f32<T>(v);
    }
  }
  __syncthreads();
  const float si = ld_or0(sc, i0 + tx, i0 + tx < M);
  for (int r = ty; r < 64; r += 4) {
    const int j = j0 + r, i = i0 + tx;  // transposes: [j][i] = L[i][j]
    if (i < M && j < M) {
      const float v = zi[tx][r];
      ((T *)a.LtT)[(long)j * a.ld + i] = from_f32<T>(v);
      ((T *)a.LstT)[(long)j * a.ld + i] = from_f32<T>(v * si);
      if constexpr (!std::is_same<T, float>::value) a.Lt32[(long)j * a.ld + i] = v;
    }
  }
}

// ---------------------------------------------------------------- K_uf
// K_uf[k][n] = sf2 exp(-1/2 |zs_k - xs_n|^2) for a block of 128 inducing
// points x 128 data points, written transposed in the operand type (Kft[n][k],
// the B operand layout of V = L^T K_uf; zero outside k < M, n < B).
// xs = X / ell is formed here; the first block row writes it.  Each wave owns
// a 64 (k) x 64 (n) sub-block; the MFMA lane layout gives every lane 4
// consecutive k of one n, stored straight from registers, so the workgroup
// needs only the staged inputs in LDS (kuf_smem(D) bytes) and several
// workgroups share a CU.  It depends on nothing but Z / ell and the batch, so
// it runs alongside the natural-gradient and Gram products.
constexpr int KUF_T = 128;
__host__ __device__ inline int kuf_ldz(int D) { return ((D + 3) & ~3) + 1; }
__host__ __device__ inline int kuf_smem(int D) { return (2 * KUF_T * kuf_ldz(D) + 2 * KUF_T + D) * 4; }
template <typename T>
__global__ __launch_bounds__(NTB) void k_kuf(const float *Zs, const CallArgs *ca,
                                             const float *inv_ell, int M, int B, int D,
                                             const float *sf2, float *Xs, T *Kft, long ld,
                                             long gs) {
  extern __shared__ __attribute__((aligned(16))) float ksm[];
  if (gs) {
    const long o = goff(gs);
    Zs = gsh(Zs, o); ca = gsh(ca, o); inv_ell = gsh(inv_ell, o); sf2 = gsh(sf2, o);
    Xs = gsh(Xs, o); Kft = gsh(Kft, o);
  }
  const int D4 = (D + 3) & ~3, LDZ = kuf_ldz(D);
  float *zs = ksm;                    // [128][LDZ]
  float *xs = zs + KUF_T * LDZ;       // [128][LDZ]
  float *zn = xs + KUF_T * LDZ;       // [128]
  float *xn = zn + KUF_T;             // [128]
  float *il = xn + KUF_T;             // [D]: 1 / ell
  const int t = threadIdx.x;
  const int k0 = blockIdx.y * KUF_T, n0 = blockIdx.x * KUF_T;
  if (t < D) il[t] = inv_ell[t];
  // stage Zs rows and raw X rows, then scale X by 1/ell in LDS
  stage_rows<NTB>(zs, LDZ, Zs, k0, KUF_T, M, D, -1);
  stage_rows<NTB>(xs, LDZ, ca->X, n0, KUF_T, B, D, -1);
  __syncthreads();
  for (int i = t; i < KUF_T * D; i += NTB) {
    const int r = i / D, d = i % D;
    const float v = xs[r * LDZ + d] * il[d];
    xs[r * LDZ + d] = v;
    if (blockIdx.y == 0 && n0 + r < B) Xs[(long)(n0 + r) * D + d] = v;
  }
  __syncthreads();
  {
    const float *row = t < KUF_T ? zs + t * LDZ : xs + (t - KUF_T) * LDZ;
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
    for (int d = 0; d < D4; d += 4) {
      s0 = fmaf(row[d], row[d], s0);
      s1 = fmaf(row[d + 1], row[d + 1], s1);
      s2 = fmaf(row[d + 2], row[d + 2], s2);
      s3 = fmaf(row[d + 3], row[d + 3], s3);
    }
    (t < KUF_T ? zn : xn)[t % KUF_T] = (s0 + s1) + (s2 + s3);
  }
  __syncthreads();
  const float s2 = *sf2;
  const int lane = t & 63, wave = t >> 6, l16 = lane & 15, l4 = lane >> 4;
  const int kb0 = (wave >> 1) * 64, nb0 = (wave & 1) * 64;
  constexpr bool F32 = std::is_same<T, float>::value;
  f32x4 c[4][4];
  if constexpr (!F32) cross_block<4, 4>(zs + kb0 * LDZ, LDZ, xs + nb0 * LDZ, LDZ, D4, c);
  float zr[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int q = 0; q < 4; ++q) zr[i][q] = zn[kb0 + 16 * i + 4 * l4 + q];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int n = nb0 + 16 * j + l16;
    const bool nok = n0 + n < B;
    const float xv = xn[n];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int kq = kb0 + 16 * i + 4 * l4;  // first of this lane's 4 consecutive k
      T e[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        // the fp32 form: distances from differences and the accurate exp
        float kv;
        if constexpr (F32)
          kv = s2 * kexp<true>(-0.5f * sqdist(zs + (kq + q) * LDZ, xs + n * LDZ, D));
        else
          kv = kern_se(s2, zr[i][q], xv, c[i][j][q]);
        e[q] = from_f32<T>((nok && k0 + kq + q < M) ? kv : 0.f);
      }
      T *dst = Kft + (long)(n0 + n) * ld + k0 + kq;
      if constexpr (sizeof(T) == 4) {
        *(f32x4 *)dst = f32x4{(float)e[0], (float)e[1], (float)e[2], (float)e[3]};
      } else {
        uint2 raw;
        __builtin_memcpy(&raw, e, 8);
        *(uint2 *)dst = raw;
      }
    }
  }
}

// sum_{k < np} p[k * stride], accumulated in A: each round issues W loads
// (clamped to an in-bounds slot, masked afterwards) before the first add uses
// them.
template <int W = 16, typename F, typename A = F>
IFS_DEV A slot_sum(const F *p, int np, long stride) {
  A a[W];
#pragma unroll
  for (int u = 0; u < W; ++u) a[u] = 0;
  for (int k = 0; k < np; k += W) {
    F v[W];
#pragma unroll
    for (int u = 0; u < W; ++u) v[u] = p[(long)min(k + u, np - 1) * stride];
#pragma unroll
    for (int u = 0; u < W; ++u) a[u] += k + u < np ? (A)v[u] : A(0);
  }
#pragma unroll
  for (int w = W / 2; w > 0; w /= 2)
#pragma unroll
    for (int u = 0; u < w; ++u) a[u] += a[u + w];
  return a[0];
}

// Two slot sums at once (uf side: nu slots, uu side: nz slots), all loads of
// a round in flight together.
// A: the accumulation type (fp64 for the gradient's cross-tile sums); P: the
// partials' type.
template <typename A = float, typename P = float>
IFS_DEV void slot_sum2(const P *pu, int nu, long su, const P *pz, int nz, long sz,
                       A &ru, A &rz) {
  constexpr int W = 16;
  A a[W], b[W];
#pragma unroll
  for (int u = 0; u < W; ++u) a[u] = b[u] = A(0);
  const int n = nu > nz ? nu : nz;
  for (int k = 0; k < n; k += W) {
    P va[W], vb[W];
#pragma unroll
    for (int u = 0; u < W; ++u) {
      va[u] = pu[(long)max(0, min(k + u, nu - 1)) * su];
      vb[u] = pz[(long)max(0, min(k + u, nz - 1)) * sz];
    }
#pragma unroll
    for (int u = 0; u < W; ++u) {
      a[u] += k + u < nu ? (A)va[u] : A(0);
      b[u] += k + u < nz ? (A)vb[u] : A(0);
    }
  }
#pragma unroll
  for (int w = W / 2; w > 0; w /= 2)
#pragma unroll
    for (int u = 0; u < w; ++u) {
      a[u] += a[u + w];
      b[u] += b[u + w];
    }
  ru = a[0];
  rz = b[0];
}

// ---------------------------------------------------------------- matrix-vector
// y[i] = scale * sum_j A[i][j] (x[j] - xs[j]) over j < Cn (lower: j <= i;
// xs and scale optional); one wave per row.
__global__ void k_gemv_rows(const float *A, long ld, int R, int Cn, const float *x,
                            const float *xs, int lower, const double *scale, float *y,
                            long gs = 0) {
  if (gs) {
    const long o = goff(gs);
    A = gsh(A, o); x = gsh(x, o); xs = gsh(xs, o); y = gsh(y, o);
  }
  const int row = blockIdx.x * (NTB / 64) + (threadIdx.x >> 6);
  if (row >= R) return;
  const float s = row_dot(A + (long)row * ld, x, xs, lower ? min(Cn, row + 1) : Cn);
  if ((threadIdx.x & 63) == 0) y[row] = scale ? (float)(*scale * s) : s;
}

// a = L^T m~ (rows of the fp32 transpose Lt), m~ from the call's arguments.
__global__ void k_lt_m(const float *Lt, long ld, int M, const CallArgs *ca, float *a,
                       long gs = 0) {
  if (gs) {
    const long o = goff(gs);
    Lt = gsh(Lt, o); ca = gsh(ca, o); a = gsh(a, o);
  }
  const int row = blockIdx.x * (NTB / 64) + (threadIdx.x >> 6);
  if (row >= M) return;
  const float s = row_dot(Lt + (long)row * ld, ca->m, nullptr, M);
  if ((threadIdx.x & 63) == 0) a[row] = s;
}

// Lb = L b (lower) for rows [0, M) and Wub = Wu b for rows [M, 2M), one wave
// per row, with workgroup partials part[blk] = {sum b_i Wub_i, sum log|L_ii|}
// (fp64) over the workgroup's rows; the bound's finalisation sums them.
__global__ void k_vec_lb_wub(const float *L, const float *Wu, long ld, int M, const float *b,
                             float *Lb, float *Wub, double *part, int *flag, long gs = 0) {
  __shared__ double sq[NTB / 64], sl[NTB / 64];
  if (gs) {
    const long o = goff(gs);
    L = gsh(L, o); Wu = gsh(Wu, o); b = gsh(b, o); Lb = gsh(Lb, o); Wub = gsh(Wub, o);
    part = gsh(part, o); flag = gsh(flag, o);
  }
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int row = blockIdx.x * (NTB / 64) + w;
  double q = 0.0, ldt = 0.0;
  if (row < M) {
    const float s = row_dot(L + (long)row * ld, b, nullptr, row + 1);
    if (lane == 0) {
      Lb[row] = s;
      const float d = L[(long)row * ld + row];
      if (d == 0.f || !isfinite(d)) atomicOr(flag, FLAG_DOMAIN);
      ldt = log(fabs((double)d));
    }
  } else if (row < 2 * M) {
    const int r = row - M;
    const float s = row_dot(Wu + (long)r * ld, b, nullptr, M);
    if (lane == 0) {
      Wub[r] = s;
      q = (double)b[r] * (double)s;
    }
  }
  if (lane == 0) {
    sq[w] = q;
    sl[w] = ldt;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, c = 0.0;
    for (int k = 0; k < NTB / 64; ++k) {
      a += sq[k];
      c += sl[k];
    }
    part[2 * blockIdx.x] = a;
    part[2 * blockIdx.x + 1] = c;
  }
}

// ---------------------------------------------------------------- likelihood + bound
// Per datum: mu = sum of mean partials, var = sf2 - sum of variance partials,
// E_n and alpha_n = c dE/dmu, beta_n = c dE/dvar (c = N/B), sqrt(-beta_n);
// workgroup partials of [sum E, sum var, sum dE/dnoise, sum beta] in fp64.
// The grid covers the padded batch: padded entries get alpha = beta = 0.
// The last workgroup forms F = c sum E - KL with
//   KL = 1/2 (-tr(Q Wu) + tr W - M + quad - log|T| - sum log s~).
struct LikArgs {
  const float *mu_part; int n_mu; const float *var_part; int n_var; long ldp;
  const CallArgs *ca;  // y, N / B, out_bound, out_terms
  int B; int Bp; const float *sfn;  // {sf2, noise_var}
  int lik; const double *gh; int ngh;  // gh: nodes[ngh] then weights[ngh]
  float *mu, *var, *alpha, *beta, *sqnb;  // sqnb = sqrt(max(0, -beta))
  double *part;  // [nblocks][4]
  const double *gram_part; int n_gram;  // [n_gram][3]: tr W, sum Q o Wu, ||W - I||^2
  const double *vec_part; int n_vec;    // [n_vec][2]: b^T Wu b, sum log|L_ii|
  double *scal; int M;
  int *flag, *counter;
  long gs;  // grouped launch: bytes between the problems' workspaces
  int defer_final;  // 1: F is formed by the next kernel (k_valpha), not here
  IFS_DEV void shift(long o) {
    mu_part = gsh(mu_part, o); var_part = gsh(var_part, o); ca = gsh(ca, o); sfn = gsh(sfn, o);
    gh = gsh(gh, o); mu = gsh(mu, o); var = gsh(var, o); alpha = gsh(alpha, o);
    beta = gsh(beta, o); sqnb = gsh(sqnb, o); part = gsh(part, o);
    gram_part = gsh(gram_part, o); vec_part = gsh(vec_part, o); scal = gsh(scal, o);
    flag = gsh(flag, o); counter = gsh(counter, o);
  }
};

__device__ __forceinline__ void probit_terms(double y, double mu, double v, const double *gh,
                                             int ngh, double &E, double &dmu, double &dv) {
  // E = pi^{-1/2} sum_k w_k log Phi(y (mu + sqrt(2 v) t_k)); exact partials of that sum.
  const double sd = sqrt(v > 0.0 ? v : 0.0);
  const double inv_sqrt_pi = 0.56418958354775628695;
  const double sq2 = 1.41421356237309504880;
  const double sq2_over_pi = 0.79788456080286535588;  // sqrt(2/pi)
  E = 0.0; dmu = 0.0; dv = 0.0;
  double dsd = 0.0;
  for (int k = 0; k < ngh; ++k) {
    const double t = gh[k], w = gh[ngh + k] * inv_sqrt_pi;
    const double z = y * (mu + sq2 * sd * t);
    const double u = -z / sq2;
    double logPhi, lam;  // log Phi(z) and phi(z)/Phi(z)
    if (z < 0.0) {
      const double ex = erfcx(u);  // Phi(z) = erfcx(u) exp(-u^2) / 2
      logPhi = log(0.5 * ex) - u * u;
      lam = sq2_over_pi / ex;
    } else {
      logPhi = log1p(-0.5 * erfc(-u));
      lam = sq2_over_pi * exp(-u * u) / erfc(u);
    }
    E += w * logPhi;
    dmu += w * lam * y;
    dsd += w * lam * y * sq2 * t;  // d/dsd
  }
  dv = sd > 0.0 ? dsd / (2.0 * sd) : 0.0;
}

// One datum n of the padded batch: mu, var, E_n, alpha, beta, sqrt(-beta)
// written; contributions to the block sums of [E, var, dE/dnoise, beta]
// returned (zero for padded entries, whose alpha, beta, sqnb are zeroed).
IFS_DEV void lik_datum(const LikArgs &a, int n, double &e, double &vs, double &dn, double &bs) {
  e = vs = dn = bs = 0.0;
  if (n < a.B) {
    float m, vp;
    slot_sum2(a.mu_part + n, a.n_mu, a.ldp, a.var_part + n, a.n_var, a.ldp, m, vp);
    const double mu = m, var = (double)a.sfn[0] - (double)vp;
    const double y = a.ca->y[n];
    double E, dmu, dv;
    if (a.lik == 0) {
      const double s2 = a.sfn[1];
      const double r = y - mu;
      E = -0.5 * log(2.0 * M_PI * s2) - (r * r + var) / (2.0 * s2);
      dmu = r / s2;
      dv = -0.5 / s2;
      dn = -0.5 / s2 + (r * r + var) / (2.0 * s2 * s2);
    } else {
      probit_terms(y, mu, var, a.gh, a.ngh, E, dmu, dv);
    }
    a.mu[n] = (float)mu;
    a.var[n] = (float)var;
    const double c = a.ca->c;
    a.alpha[n] = (float)(c * dmu);
    a.beta[n] = (float)(c * dv);
    a.sqnb[n] = (float)sqrt(fmax(0.0, -c * dv));
    e = E;
    vs = var;
    bs = c * dv;
  } else if (n < a.Bp) {
    a.alpha[n] = 0.f;
    a.beta[n] = 0.f;
    a.sqnb[n] = 0.f;
  }
}

// F = c sum E - KL with
//   KL = 1/2 (-tr(Q Wu) + tr W - M + quad - log|T| - sum log s~)
// from the likelihood's block partials part[nblk][4] and the earlier kernels'
// partials (traces, ||W - I||^2, b^T Wu b, log|L_ii|).  Called by every
// thread of one block of NT threads; sh holds >= 7 * NT / 64 doubles.
template <int NT>
IFS_DEV void lik_final(const LikArgs &a, int nblk, double *sh) {
  double v[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < nblk; i += NT) {
    v[0] += a.part[4 * i];
    v[1] += a.part[4 * i + 1];
  }
  for (int i = threadIdx.x; i < a.n_gram; i += NT) {
    v[2] += a.gram_part[3 * i];
    v[3] += a.gram_part[3 * i + 1];
    v[4] += a.gram_part[3 * i + 2];
  }
  for (int i = threadIdx.x; i < a.n_vec; i += NT) {
    v[5] += a.vec_part[2 * i];
    v[6] += a.vec_part[2 * i + 1];
  }
  block_sums<NT, 7>(v, sh);
  if (threadIdx.x == 0) {
    const double e = v[0], vs = v[1], trw = v[2], qwu = v[3], r2 = v[4];
    const double quad = v[5], logdet = 2.0 * v[6], sls = a.scal[S_SUMLOGS];
    a.scal[S_QUAD] = quad;
    a.scal[S_LOGDET] = logdet;
    const double KL = 0.5 * (-qwu + trw - (double)a.M + quad - logdet - sls);
    const double data = a.ca->c * e;
    const double F = data - KL;
    if (!isfinite(F)) atomicOr(a.flag, FLAG_NONFINITE);
    if (a.ca->out_bound) *a.ca->out_bound = F;
    if (a.ca->out_terms) {
      double *o = a.ca->out_terms;
      o[0] = data; o[1] = KL; o[2] = vs; o[3] = sqrt(r2 / a.M);
      o[4] = trw; o[5] = qwu; o[6] = quad; o[7] = logdet;
    }
  }
}

// Likelihood over the padded batch, one datum per thread; the last block
// forms F.
__global__ void k_lik(LikArgs a) {
  __shared__ double sh[7 * (NTB / 64)];
  __shared__ int s_last;
  if (a.gs) a.shift(goff(a.gs));
  double v[4];
  lik_datum(a, blockIdx.x * NTB + threadIdx.x, v[0], v[1], v[2], v[3]);
  block_sums<NTB, 4>(v, sh);
  if (threadIdx.x == 0) {
    double *p = a.part + 4 * blockIdx.x;
    p[0] = v[0]; p[1] = v[1]; p[2] = v[2]; p[3] = v[3];
  }
  if (a.defer_final) return;
  if (!arrive_last(a.counter, &s_last)) return;
  lik_final<NTB>(a, gridDim.x, sh);
}

// ---------------------------------------------------------------- prediction
// Predictive marginals at test inputs (one chunk of at most B_max points):
//   mu_* = k_*u P m~ = a^T U_*,  sigma_*^2 = k_** - k_*u P k_u* = sf2 - sum V_* o U_*,
// from the per-128-row partials of the U epilogue, and with targets the log
// predictive density of each point,
//   Gaussian: log N(y; mu_*, sigma_*^2 + noise),
//   probit:   log Phi(y mu_* / sqrt(1 + sigma_*^2)),
// with fp64 per-workgroup partial sums of it.
struct PredArgs {
  const float *mu_part; int n_mu; const float *var_part; int n_var; long ldp;
  int n; const float *sfn; int lik;
  const float *y;            // chunk targets (optional)
  float *mu, *var, *lpd;     // chunk outputs (lpd optional, needs y)
  double *part;              // [blocks] partial sums of the log densities
};

// log Phi(z), in the two forms that keep it accurate on either side of 0
__device__ __forceinline__ double log_Phi(double z) {
  const double u = -z * 0.70710678118654752440;  // -z / sqrt(2)
  if (z < 0.0) return log(0.5 * erfcx(u)) - u * u;  // Phi(z) = erfcx(u) exp(-u^2) / 2
  return log1p(-0.5 * erfc(-u));
}

__global__ void k_predict(PredArgs a) {
  __shared__ double sh[NTB / 64];
  const int n = blockIdx.x * NTB + threadIdx.x;
  double l = 0.0;
  if (n < a.n) {
    float m, vp;
    slot_sum2(a.mu_part + n, a.n_mu, a.ldp, a.var_part + n, a.n_var, a.ldp, m, vp);
    const double mu = m, var = (double)a.sfn[0] - (double)vp;
    a.mu[n] = (float)mu;
    a.var[n] = (float)var;
    if (a.y) {
      const double y = a.y[n];
      if (a.lik == 0) {
        const double vy = var + (double)a.sfn[1], r = y - mu;
        l = -0.5 * log(2.0 * M_PI * vy) - r * r / (2.0 * vy);
      } else {
        l = log_Phi(y * mu / sqrt(1.0 + var));
      }
      if (a.lpd) a.lpd[n] = (float)l;
    }
  }
  if (!a.y) return;
  l = block_sum<NTB>(l, sh);
  if (threadIdx.x == 0) a.part[blockIdx.x] = l;
}

// Adds one chunk's partials to the running sum in scal[S_LPD] (first chunk:
// starts it) and, after the last chunk, writes NLPD = -sum / n_total.
__global__ void k_predict_sum(const double *part, int nparts, double *scal, int first,
                              int last, double n_total, double *nlpd) {
  __shared__ double sh[NTB / 64];
  double s = 0.0;
  for (int i = threadIdx.x; i < nparts; i += NTB) s += part[i];
  s = block_sum<NTB>(s, sh);
  if (threadIdx.x == 0) {
    const double tot = (first ? 0.0 : scal[S_LPD]) + s;
    scal[S_LPD] = tot;
    if (last && nlpd) *nlpd = -tot / n_total;
  }
}

// ---------------------------------------------------------------- Hutchinson bound
// Bound evaluation with the cubic traces replaced by probe estimates.  With
// Xc = [V | Omega | a] (columns: the batch, the K probes, a = L^T m~) and
// WX = L^T K~ L Xc, EX = L^T S~ L Omega (fp32, stored transposed [column][row]):
//   U = 2V - W V gives sigma^2_n = sf2 - sum_i V_in U_in and mu_n = a^T U_n
//   (U kept for the backward's R = L U),
//   per probe w: w^T W w, w^T E w, |W w|^2, (W w)^T (E w) for the estimates of
//   tr W, tr Wu = tr(W - E) and tr(W Wu), and b = 2a - W a.
// The probes as operands: rows [B, B + K) of the batch operand take Omega^T,
// row B + K takes a; k >= M is zero.
template <typename T>
__global__ void k_hutch_fill(T *Vt, long ld, int B, int K, const float *Omt, const float *a,
                             int M, int Mp) {
  for (int r = blockIdx.y; r <= K; r += gridDim.y)  // 0..K: probe rows, then a
  for (int i = blockIdx.x * NTB + threadIdx.x; i < Mp; i += gridDim.x * NTB) {
    float v = 0.f;
    if (i < M) v = r < K ? Omt[(long)r * M + i] : a[i];
    Vt[(long)(B + r) * ld + i] = from_f32<T>(v);
  }
}

struct HutchArgs {
  const void *Vt; long ld;  // batch operand rows (type T) [n][i]
  void *Ut;                 // rows [0, B) get U = 2V - W V (type T, zero beyond M)
  const float *wx, *ex;     // [B + K + 1][ld], [K][ld]
  const float *Omt;         // caller's probes [K][M]
  const float *a;           // L^T m~
  int M, B, K;
  float *var_part, *mu_part;  // [n]: sum_i V o U and sum_i a o U
  double *hp;                 // [K][4]
  float *b;                   // 2a - W a, zero-padded to ld
};

template <typename T>
__global__ void k_hutch_rows(HutchArgs h) {
  const int row = blockIdx.x * (NTB / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= h.B + h.K + 1) return;
  const float *wx = h.wx + (long)row * h.ld;
  if (row < h.B) {
    const T *vt = (const T *)h.Vt + (long)row * h.ld;
    T *ut = (T *)h.Ut + (long)row * h.ld;
    float sv = 0.f, sm = 0.f;
    for (int i = lane; i < (int)h.ld; i += 64) {
      if (i >= h.M) {
        ut[i] = from_f32<T>(0.f);
        continue;
      }
      const float v = to_f32(vt[i]);
      const float u = 2.f * v - wx[i];
      ut[i] = from_f32<T>(u);
      sv = fmaf(v, u, sv);
      sm = fmaf(h.a[i], u, sm);
    }
    sv = wave_sum(sv);
    sm = wave_sum(sm);
    if (lane == 0) {
      h.var_part[row] = sv;
      h.mu_part[row] = sm;
    }
  } else if (row < h.B + h.K) {
    const int k = row - h.B;
    const float *om = h.Omt + (long)k * h.M, *ex = h.ex + (long)k * h.ld;
    double w1 = 0.0, w2 = 0.0, w3 = 0.0, w4 = 0.0;
    for (int i = lane; i < h.M; i += 64) {
      const double o = om[i], w = wx[i], e = ex[i];
      w1 += o * w;
      w2 += o * e;
      w3 += w * w;
      w4 += w * e;
    }
    w1 = wave_sum(w1);
    w2 = wave_sum(w2);
    w3 = wave_sum(w3);
    w4 = wave_sum(w4);
    if (lane == 0) {
      double *p = h.hp + 4 * (long)k;
      p[0] = w1; p[1] = w2; p[2] = w3; p[3] = w4;
    }
  } else {
    for (int i = lane; i < (int)h.ld; i += 64) h.b[i] = i < h.M ? 2.f * h.a[i] - wx[i] : 0.f;
  }
}

// The trace estimates as the bound's Gram partial {tr W, tr(Q Wu), 0}, with
// tr(Q Wu) = 2 tr Wu - tr(W Wu) (one block).
__global__ void k_hutch_final(const double *hp, int K, double *gram_part) {
  __shared__ double sh[3 * (NTB / 64)];
  double v[3] = {0.0, 0.0, 0.0};
  for (int k = threadIdx.x; k < K; k += NTB) {
    const double *p = hp + 4 * (long)k;
    v[0] += p[0];
    v[1] += p[0] - p[1];
    v[2] += p[2] - p[3];
  }
  block_sums<NTB, 3>(v, sh);
  if (threadIdx.x == 0) {
    gram_part[0] = v[0] / K;
    gram_part[1] = 2.0 * v[1] / K - v[2] / K;
    gram_part[2] = 0.0;
  }
}

// The backward's low-rank form of C (the adjoint of G_uu = L C L^T in
// L-space): C = X S X^T with the r = B + 2K + 3 columns
//   X = [V | Omega | Omega - G | x | a | b],  G = 2 W Omega - E Omega,
//   x = V alpha - Wu b, b = Q a,
// and S pairing them: beta_n on V_n, 1/(4K) between Omega_k and
// (Omega - G)_k, -1/2 between x and a, -1/2 on b.  This kernel writes X^T in
// the operand type, rows [0, rp) of length Mp (zero beyond M and r).
template <typename T>
__global__ void k_hutch_X(const T *Vt, const float *Omt, const float *wx, const float *ex,
                          const float *Va, const float *Wub, const float *a, const float *b,
                          int B, int K, int M, int Mp, int rows, T *Xt) {
  const long ld = Mp;
  for (int q = blockIdx.y; q < rows; q += gridDim.y)
  for (int i = blockIdx.x * NTB + threadIdx.x; i < Mp; i += gridDim.x * NTB) {
    float v = 0.f;
    if (i < M) {
      if (q < B) {
        v = to_f32(Vt[(long)q * ld + i]);
      } else if (q < B + K) {
        v = Omt[(long)(q - B) * M + i];
      } else if (q < B + 2 * K) {
        const int k = q - B - K;
        v = Omt[(long)k * M + i] - (2.f * wx[(long)(B + k) * ld + i] - ex[(long)k * ld + i]);
      } else if (q == B + 2 * K) {
        v = Va[i] - Wub[i];
      } else if (q == B + 2 * K + 1) {
        v = a[i];
      } else if (q == B + 2 * K + 2) {
        v = b[i];
      }
    }
    Xt[(long)q * ld + i] = from_f32<T>(v);
  }
}

// Y2 = Y1 S for Y1 = L X ([Mp][ldr], columns as in X): column c of Y2 takes
// S's partner column of Y1 times its coefficient; zero beyond M and r.
template <typename TW>
__global__ void k_hutch_mix(const TW *Y1, TW *Y2, long ldr, int M, int Mp, int B, int K,
                            const float *beta, float inv4k) {
  const int r = B + 2 * K + 3;
  const long n = (long)Mp * ldr;
  for (long e = blockIdx.x * (long)NTB + threadIdx.x; e < n; e += (long)gridDim.x * NTB) {
    const int i = (int)(e / ldr), c = (int)(e % ldr);
    float v = 0.f;
    if (i < M && c < r) {
      int src;
      float w;
      if (c < B) { src = c; w = beta[c]; }
      else if (c < B + K) { src = c + K; w = inv4k; }
      else if (c < B + 2 * K) { src = c - K; w = inv4k; }
      else if (c == B + 2 * K) { src = c + 1; w = -0.5f; }
      else if (c == B + 2 * K + 1) { src = c - 1; w = -0.5f; }
      else { src = c; w = -0.5f; }
      v = w * to_f32(Y1[(long)i * ldr + src]);
    }
    Y2[e] = from_f32<TW>(v);
  }
}

// t2 = Q x = 2x - W x for x = V alpha - Wu b, given W x = L^T K~ L x
__global__ void k_hutch_t2(float *t2, const float *Va, const float *Wub, const float *Wx, int M) {
  const int i = blockIdx.x * NTB + threadIdx.x;
  if (i < M) t2[i] = 2.f * (Va[i] - Wub[i]) - Wx[i];
}

// y -= s~ o x  (K~ L b -> K_uu L b)
__global__ void k_hutch_sub_diag(float *y, const float *sP, const float *x, int M) {
  const int i = blockIdx.x * NTB + threadIdx.x;
  if (i < M) y[i] -= sP[i] * x[i];
}

// The bound's vector partial {b^T Wu b, sum log|L_ii|} in one block, with the
// domain check on the diagonal of L.
__global__ void k_hutch_quad(const float *b, const float *Wub, const float *L, long ld, int M,
                             double *vec_part, int *flag) {
  __shared__ double sh[2 * (NTB / 64)];
  double v[2] = {0.0, 0.0};
  int bad = 0;
  for (int i = threadIdx.x; i < M; i += NTB) {
    v[0] += (double)b[i] * (double)Wub[i];
    const float d = L[(long)i * ld + i];
    if (d == 0.f || !isfinite(d)) bad = 1;
    v[1] += log(fabs((double)d));
  }
  if (bad) atomicOr(flag, FLAG_DOMAIN);
  block_sums<NTB, 2>(v, sh);
  if (threadIdx.x == 0) {
    vec_part[0] = v[0];
    vec_part[1] = v[1];
  }
}

// ---------------------------------------------------------------- backward
// C = -sym((V alpha) a^T) + V diag(beta) V^T - 1/2 (Wu + I - Wub a^T - a Wub^T)
//     + 1/2 (Q - b b^T), with V diag(beta) V^T = -sum_s Ys[s] (split-K pieces
// of (V D)(V D)^T, D = diag(sqrt(-beta)); beta <= 0 for both likelihoods),
// written in the operand type TC over the M x M block.  The pieces hold the
// lower 64 x 64 tiles only: one workgroup per lower tile sums them in split
// order, forms the tile of C from the symmetric inputs and writes it and,
// through LDS, its mirror.  Entries outside the M x M block are zeros.
template <typename TC>
struct alignas(8 * sizeof(TC)) Pack8 {
  TC v[8];
};
template <typename TC>
__global__ __launch_bounds__(NTB) void k_assemble_C(const float *Ys, int nsplit,
                                                    long split_stride, const float *Wu,
                                                    const float *Q, const float *a, const float *b,
                                                    const float *Wub, const float *Va, int M,
                                                    long ld, TC *Cm, long gs = 0) {
  __shared__ float ct[64][65];
  if (gs) {
    const long o = goff(gs);
    Ys = gsh(Ys, o); Wu = gsh(Wu, o); Q = gsh(Q, o); a = gsh(a, o); b = gsh(b, o);
    Wub = gsh(Wub, o); Va = gsh(Va, o); Cm = gsh(Cm, o);
  }
  const int t = blockIdx.x;
  int I = (int)((sqrtf(8.0f * t + 1.0f) - 1.0f) * 0.5f);
  while ((I + 1) * (I + 2) / 2 <= t) ++I;
  while (I * (I + 1) / 2 > t) --I;
  const int J = t - I * (I + 1) / 2;
  const int m0 = I * 64, n0 = J * 64;
  float cv[2][8];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int ch = threadIdx.x + k * NTB, r = ch / 8, c = (ch % 8) * 8;
    const int gi = m0 + r, gj = n0 + c;
    const long ij = (long)gi * ld + gj;
    f32x4 y0 = *(const f32x4 *)(Ys + ij), y1 = *(const f32x4 *)(Ys + ij + 4);
#pragma unroll 4
    for (int s = 1; s < nsplit; ++s) {
      y0 += *(const f32x4 *)(Ys + s * split_stride + ij);
      y1 += *(const f32x4 *)(Ys + s * split_stride + ij + 4);
    }
    const f32x4 wu0 = *(const f32x4 *)(Wu + ij), wu1 = *(const f32x4 *)(Wu + ij + 4);
    const f32x4 q0 = *(const f32x4 *)(Q + ij), q1 = *(const f32x4 *)(Q + ij + 4);
    const f32x4 a0 = *(const f32x4 *)(a + gj), a1 = *(const f32x4 *)(a + gj + 4);
    const f32x4 b0 = *(const f32x4 *)(b + gj), b1 = *(const f32x4 *)(b + gj + 4);
    const f32x4 w0 = *(const f32x4 *)(Wub + gj), w1 = *(const f32x4 *)(Wub + gj + 4);
    const f32x4 v0 = *(const f32x4 *)(Va + gj), v1 = *(const f32x4 *)(Va + gj + 4);
    const float ai = a[gi], bi = b[gi], wi = Wub[gi], vi = Va[gi];
    Pack8<TC> out;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const float ys = u < 4 ? y0[u] : y1[u - 4], wu = u < 4 ? wu0[u] : wu1[u - 4];
      const float q = u < 4 ? q0[u] : q1[u - 4], aj = u < 4 ? a0[u] : a1[u - 4];
      const float bj = u < 4 ? b0[u] : b1[u - 4], wj = u < 4 ? w0[u] : w1[u - 4];
      const float vj = u < 4 ? v0[u] : v1[u - 4];
      const float x = -0.5f * (vi * aj + ai * vj) - ys -
                      0.5f * (wu + (gi == gj + u ? 1.f : 0.f) - wi * aj - ai * wj) +
                      0.5f * (q - bi * bj);
      cv[k][u] = (gi < M && gj + u < M) ? x : 0.f;
      out.v[u] = from_f32<TC>(cv[k][u]);
      ct[r][c + u] = cv[k][u];
    }
    *(Pack8<TC> *)(Cm + ij) = out;
  }
  if (I == J) return;
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int ch = threadIdx.x + k * NTB, c = ch / 8, r = (ch % 8) * 8;
    Pack8<TC> out;
#pragma unroll
    for (int u = 0; u < 8; ++u) out.v[u] = from_f32<TC>(ct[r + u][c]);
    *(Pack8<TC> *)(Cm + (long)(n0 + c) * ld + m0 + r) = out;
  }
}

// rpw (1..VA_ROWS) rows of the operand-type V per workgroup (its four waves
// split the rows, each alpha / sqnb chunk loaded once for all of them):
// (V alpha)_i and the scaled copy Vs[i][n] = V[i][n] sqnb[n] over the whole
// padded row, the operand of the batch product (V D)(V D)^T.  alpha and sqnb
// are zero for n >= B (set by the likelihood kernel), so padded entries
// contribute nothing and Vs is zero there.  Launch with cdiv(M, rpw)
// workgroups.  With nlik > 0 one more workgroup (the last) forms F from the
// likelihood kernel's nlik block partials (lik_final), when that kernel
// deferred it: the kernel boundary orders the partials, so no arrival fence
// is needed.  Several rows per workgroup save re-reads of alpha and sqnb when
// there are rows enough to fill the chip regardless (va_rows).
constexpr int VA_ROWS = 4;
__host__ __device__ inline int va_rows(int M) { return M >= 2048 ? VA_ROWS : 1; }
template <typename T>
__global__ __launch_bounds__(NTB) void k_valpha(const T *V, long ld, int M, int Bp,
                                                const float *alpha, const float *sqnb, T *Vs,
                                                float *out, long gs, LikArgs la, int nlik,
                                                int rpw) {
  __shared__ float shw[VA_ROWS][NTB / 64];
  __shared__ double shl[7 * (NTB / 64)];
  if (gs) {
    const long o = goff(gs);
    V = gsh(V, o); alpha = gsh(alpha, o); sqnb = gsh(sqnb, o); Vs = gsh(Vs, o);
    out = gsh(out, o);
    if (nlik) la.shift(o);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nrb = (M + rpw - 1) / rpw, rb = blockIdx.x;
  if (rb >= nrb) {  // uniform across the workgroup
    if (nlik && rb == nrb) lik_final<NTB>(la, nlik, shl);
    return;
  }
  const int r0 = rb * rpw, nr = min(rpw, M - r0);
  constexpr int KPL = 16 / (int)sizeof(T);
  float s[VA_ROWS];
#pragma unroll
  for (int r = 0; r < VA_ROWS; ++r) s[r] = 0.f;
  for (int n = (int)threadIdx.x * KPL; n < Bp; n += NTB * KPL) {  // Bp is a multiple of KPL
    float al[KPL], sq[KPL];
#pragma unroll
    for (int q = 0; q < KPL; q += 4) {
      const f32x4 a4 = *(const f32x4 *)(alpha + n + q), s4 = *(const f32x4 *)(sqnb + n + q);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        al[q + u] = a4[u];
        sq[q + u] = s4[u];
      }
    }
    uint4 raw[VA_ROWS];
#pragma unroll
    for (int r = 0; r < VA_ROWS; ++r)
      if (r < nr) raw[r] = *(const uint4 *)(V + (long)(r0 + r) * ld + n);
#pragma unroll
    for (int r = 0; r < VA_ROWS; ++r) {
      if (r >= nr) break;
      const T *e = (const T *)&raw[r];
      uint4 sraw;
      T *se = (T *)&sraw;
#pragma unroll
      for (int q = 0; q < KPL; ++q) {
        const float x = to_f32(e[q]);
        s[r] = fmaf(x, al[q], s[r]);
        se[q] = from_f32<T>(x * sq[q]);
      }
      *(uint4 *)(Vs + (long)(r0 + r) * ld + n) = sraw;
    }
  }
#pragma unroll
  for (int r = 0; r < VA_ROWS; ++r) {
    const float w = wave_sum(s[r]);
    if (lane == 0) shw[r][wave] = w;
  }
  __syncthreads();
  if ((int)threadIdx.x < nr) {
    float t = 0.f;
#pragma unroll
    for (int w = 0; w < NTB / 64; ++w) t += shw[threadIdx.x][w];
    out[r0 + threadIdx.x] = t;
  }
}

// All gradient reductions in one launch, with blocks of three roles:
//  * [0, rb): rows of Z.  For thread (i, d): r_uf = sum of H_uf row sums,
//    hx = sum_n H_uf,in xs_nd, r_uu, hz likewise for H_uu over their per-tile
//    slots; dF/dZ_id = -(1/ell_d) [(zs r_uf - hx) + 2 (zs r_uu - hz)] and the
//    block partial of the lengthscale sums in scaled coordinates
//      sum_i r_uf zs^2 - 2 zs hx + 2 (r_uu zs^2 - zs hz);
//  * [rb, rb + cb): data columns: c_n = sum_i H_uf,in, partial sum_n c_n xs_nd^2;
//  * [rb + cb, rb + cb + rq): t2 = Q (V alpha - Wu b), one wave per row (the
//    inducing-mean gradient is L t2, formed by the next launch).
// The last workgroup forms dF/dell_d = (1/ell_d) sum of partials,
// dF/dsf2 = (sum H_uu + sum H_uf)/sf2 + sum beta and dF/dnoise = c sum dE/dnoise.
struct GradArgs {
  int M, B, D;
  const CallArgs *ca;  // N / B, grad_scale and the gradient outputs
  const float *Zs, *Xs, *inv_ell, *sfn;
  // per-tile partials (element type P of k_grad: fp64 in the fp32 form, else fp32)
  const void *hrow, *hx; int n_uf_nt;            // [n_uf_nt][M], [n_uf_nt][M][D]
  const void *hzrow, *hz; int nb;                // [nb][M], [nb][M][D]
  const void *hcol; int n_uf_mt; long ldc;       // [n_uf_mt][ldc]
  const double *uf_part; int n_uf_tiles;
  const double *uu_part; int n_uu_tiles;
  const double *lik_part; int n_lik;
  const float *Q, *Va, *Wub; long ld; float *t2;
  double *ell_part;  // [D][rb + cb]
  int rb, cb;
  // gradient with respect to s~ (skipped without g_s)
  const float *gdiag, *pdiag; long ldpd;  // diag(G_uu); [nb][ldpd] partials of diag(P)
  const float *Lb, *s_in;
  long gs;  // grouped launch: bytes between the problems' workspaces
  IFS_DEV void shift(long o) {
    ca = gsh(ca, o); Zs = gsh(Zs, o); Xs = gsh(Xs, o); inv_ell = gsh(inv_ell, o);
    sfn = gsh(sfn, o); hrow = gsh(hrow, o); hx = gsh(hx, o); hzrow = gsh(hzrow, o);
    hz = gsh(hz, o); hcol = gsh(hcol, o); uf_part = gsh(uf_part, o);
    uu_part = gsh(uu_part, o); lik_part = gsh(lik_part, o); Q = gsh(Q, o); Va = gsh(Va, o);
    Wub = gsh(Wub, o); t2 = gsh(t2, o); ell_part = gsh(ell_part, o); gdiag = gsh(gdiag, o);
    pdiag = gsh(pdiag, o); Lb = gsh(Lb, o); s_in = gsh(s_in, o);
  }
};

// Z-row blocks of k_grad: GRAD_SLOT_GROUPS threads per (row, d) split the
// tile slots, grad_zrows(D) rows per block.
constexpr int GRAD_SLOT_GROUPS = 4;
__host__ __device__ inline int grad_zrows(int D) { return NTB / (GRAD_SLOT_GROUPS * D); }

// Gradient reductions:
//  * blocks [0, rb): dF/dZ rows (grad_zrows(D) rows of D per block) from the
//    per-tile partials of H_uf and H_uu, and lengthscale partials;
//  * blocks [rb, rb + cb): lengthscale partials of the data side (column sums
//    of H_uf against Xs^2);
//  * the remaining blocks: t2 = Q (V alpha - Wu b), one wave per row.
template <typename P>
__global__ __launch_bounds__(NTB) void k_grad(GradArgs g) {
  __shared__ double sh[NTB];
  __shared__ double sx[GRAD_SLOT_GROUPS * NTB];
  if (g.gs) g.shift(goff(g.gs));
  const int blk = blockIdx.x, t = threadIdx.x;
  const int R = NTB / g.D;
  if (blk < g.rb) {
    // GRAD_SLOT_GROUPS threads per (row, d), each summing every
    // GRAD_SLOT_GROUPS-th tile slot, combined in a fixed order
    constexpr int G = GRAD_SLOT_GROUPS;
    const int Rz = grad_zrows(g.D), per = Rz * g.D;
    const int grp = t / per, rem = t % per, r = rem / g.D, d = rem % g.D;
    const int i = blk * Rz + r;
    const CallArgs &ca = *g.ca;
    const double scale = ca.grad_scale ? *ca.grad_scale : 1.0;
    double ruf = 0.0, ruu = 0.0, hx = 0.0, hz = 0.0;
    if (grp < G && i < g.M) {
      const long e = (long)i * g.D + d, MD = (long)g.M * g.D;
      // slots grp, grp + G, ... (a group with no slot keeps slot 0's address,
      // whose values slot_sum2 reads but discards)
      const int nuf = g.n_uf_nt > grp ? (g.n_uf_nt - grp + G - 1) / G : 0;
      const int nuu = g.nb > grp ? (g.nb - grp + G - 1) / G : 0;
      const long ouf = nuf ? (long)grp : 0, ouu = nuu ? (long)grp : 0;
      const P *hrow = (const P *)g.hrow, *hzrow = (const P *)g.hzrow;
      const P *hxp = (const P *)g.hx, *hzp = (const P *)g.hz;
      slot_sum2<double, P>(hrow + i + ouf * g.M, nuf, (long)G * g.M,
                           hzrow + i + ouu * g.M, nuu, (long)G * g.M, ruf, ruu);
      slot_sum2<double, P>(hxp + e + ouf * MD, nuf, G * MD, hzp + e + ouu * MD, nuu, G * MD,
                           hx, hz);
    }
    sx[t] = ruf;
    sx[NTB + t] = ruu;
    sx[2 * NTB + t] = hx;
    sx[3 * NTB + t] = hz;
    __syncthreads();
    double contrib = 0.0;
    if (t < per && i < g.M) {
      for (int q = 1; q < G; ++q) {
        ruf += sx[q * per + t];
        ruu += sx[NTB + q * per + t];
        hx += sx[2 * NTB + q * per + t];
        hz += sx[3 * NTB + q * per + t];
      }
      const long e = (long)i * g.D + d;
      const double zs = g.Zs[e];
      const double gz = -(double)g.inv_ell[d] * ((zs * ruf - hx) + 2.0 * (zs * ruu - hz));
      if (ca.g_Z) ca.g_Z[e] = (float)(scale * gz);
      contrib = ruf * zs * zs - 2.0 * zs * hx + 2.0 * (ruu * zs * zs - zs * hz);
    }
    sh[t] = contrib;
    __syncthreads();
    if (t < g.D) {
      double s = 0.0;
      for (int q = 0; q < Rz; ++q) s += sh[q * g.D + t];
      g.ell_part[(long)t * (g.rb + g.cb) + blk] = s;
    }
  } else if (blk < g.rb + g.cb) {
    const int r = t / g.D, d = t % g.D;
    const int n = (blk - g.rb) * R + r;
    double contrib = 0.0;
    if (r < R && n < g.B) {
      const double cn = slot_sum<8, P, double>((const P *)g.hcol + n, g.n_uf_mt, g.ldc);
      const double xs = g.Xs[(long)n * g.D + d];
      contrib = cn * xs * xs;
    }
    sh[t] = contrib;
    __syncthreads();
    if (t < g.D) {
      double s = 0.0;
      for (int q = 0; q < R; ++q) s += sh[q * g.D + t];
      g.ell_part[(long)t * (g.rb + g.cb) + blk] = s;
    }
  } else {
    const int row = (blk - g.rb - g.cb) * (NTB / 64) + (t >> 6);
    if (row < g.M) {
      const float s = row_dot(g.Q + (long)row * g.ld, g.Va, g.Wub, g.M);
      if ((t & 63) == 0) g.t2[row] = s;
    }
  }
}

// Tail of the gradient: blocks [0, rows) form dF/dm~ = scale * L t2 and
// dF/ds~ (one wave per row, each when requested):
//   dF/ds~_i = diag(G_Kt)_i + 1/(2 s~_i),
//   diag(G_Kt) = diag(G_uu) - diag(P)/2 + (L b)_i^2 / 2,
// diag(P) summed from the per-tile partials of L Q with J <= i/64; blocks
// [rows, rows + D) form dF/dell_d = (1/ell_d) sum of the partials of d; the
// last block dF/dsf2 = (sum H_uu + sum H_uf)/sf2 + sum beta and
// dF/dnoise = c sum dE/dnoise.  Launch with rows + D + 1 blocks.
__global__ void k_grad_tail(GradArgs g, const float *L, int rows) {
  __shared__ double sh[NTB];
  if (g.gs) {
    const long o = goff(g.gs);
    g.shift(o);
    L = gsh(L, o);
  }
  const int t = threadIdx.x;
  const CallArgs &ca = *g.ca;
  const double scale = ca.grad_scale ? *ca.grad_scale : 1.0;
  if ((int)blockIdx.x < rows) {
    const int row = blockIdx.x * (NTB / 64) + (t >> 6), lane = t & 63;
    if (row < g.M) {
      if (ca.g_m) {
        const float s = row_dot(L + (long)row * g.ld, g.t2, nullptr, row + 1);
        if (lane == 0) ca.g_m[row] = (float)(scale * s);
      }
      if (ca.g_s) {
        float pd = 0.f;
        for (int J = lane; J <= row / 64; J += 64) pd += g.pdiag[(long)J * g.ldpd + row];
        pd = wave_sum(pd);
        if (lane == 0) {
          const double lb = g.Lb[row];
          const double gs = (double)g.gdiag[row] - 0.5 * (double)pd + 0.5 * lb * lb +
                            0.5 / (double)g.s_in[row];
          ca.g_s[row] = (float)(scale * gs);
        }
      }
    }
    return;
  }
  const int nparts = g.rb + g.cb;
  const int blk = (int)blockIdx.x - rows;
  if (blk < g.D) {
    // dF/dell_d = (1/ell_d) sum of the block partials of d
    const int d = blk;
    const double *pp = g.ell_part + (long)d * nparts;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int p = t;
    for (; p + 3 * NTB < nparts; p += 4 * NTB) {
      s0 += pp[p];
      s1 += pp[p + NTB];
      s2 += pp[p + 2 * NTB];
      s3 += pp[p + 3 * NTB];
    }
    for (; p < nparts; p += NTB) s0 += pp[p];
    const double sd = block_sum<NTB>((s0 + s1) + (s2 + s3), sh);
    if (t == 0 && ca.g_ell) ca.g_ell[d] = (float)(scale * sd * g.inv_ell[d]);
    return;
  }
  // the last block: dF/dsf2 and dF/dnoise
  double huf = 0.0, huu = 0.0, dn = 0.0, bs = 0.0;
  for (int i = t; i < g.n_uf_tiles; i += NTB) huf += g.uf_part[i];
  for (int i = t; i < g.n_uu_tiles; i += NTB) huu += g.uu_part[i];
  for (int i = t; i < g.n_lik; i += NTB) {
    dn += g.lik_part[4 * i + 2];
    bs += g.lik_part[4 * i + 3];
  }
  double v4[4] = {huf, huu, dn, bs};
  block_sums<NTB, 4>(v4, sh);
  huf = v4[0]; huu = v4[1]; dn = v4[2]; bs = v4[3];
  if (t == 0) {
    if (ca.g_sf2) *ca.g_sf2 = (float)(scale * ((huf + huu) / (double)g.sfn[0] + bs));
    if (ca.g_noise) *ca.g_noise = (float)(scale * ca.c * dn);
  }
}

// ---------------------------------------------------------------- adaptive NG
// Stopping rule of an adaptive NG loop, one block, before the update of step
// `step`, from per-tile partial sums s:
//   rule 0 (eq. stopping_frobenius): r = sqrt(s / M) = ||W - I||_F / sqrt(M),
//          stop when r < tol;
//   rule 1 (Prop. 3, Gaussian likelihood): r = G = s / sigma^2 with
//          s = sum_n ||(I - K~ T) k_n||^2, stop when G <= 2 sigma_obs^2 tol.
// Once it stops the flag is set and the remaining products of the loop skip
// their k-loops (the updates then pass L through).  Step 0 clears the flag.
// out_resid[step] receives r, or the stopping value once the loop has
// stopped; *out_steps the updates applied so far.
__global__ void k_ng_check(const double *gram_part, int n_gram, int M, int step, int *flag,
                           double *scal, const CallArgs *ca, int rule) {
  __shared__ double sh[NTB / 64];
  __shared__ int stopped;
  if (threadIdx.x == 0) {
    if (step == 0) *flag = 0;
    stopped = step > 0 && *flag;
  }
  __syncthreads();
  if (stopped) {
    if (threadIdx.x == 0 && ca->out_resid) ca->out_resid[step] = scal[S_RESID];
    return;
  }
  double s = 0.0;
  for (int i = threadIdx.x; i < n_gram; i += NTB) s += gram_part[i];
  s = block_sum<NTB>(s, sh);
  if (threadIdx.x == 0) {
    const double r = rule == 0 ? sqrt(s / M) : s / (double)ca->gap_sigma2;
    const bool stop = rule == 0 ? r < (double)ca->ng_tol
                                : r <= 2.0 * (double)*ca->noise * (double)ca->ng_tol;
    scal[S_RESID] = r;
    if (ca->out_resid) ca->out_resid[step] = r;
    if (stop) {
      *flag = 1;
      if (ca->out_steps) *ca->out_steps = step;
    } else if (ca->out_steps) {
      *ca->out_steps = step + 1;
    }
  }
}

// ---------------------------------------------------------------- optimiser
// One Adam step (Kingma and Ba's algorithm with bias correction) on n fp32
// parameters: g' = sign g, m = b1 m + (1 - b1) g', v = b2 v + (1 - b2) g'^2,
// p -= lr (m / bc1) / (sqrt(v / bc2) + eps), with bc1 = 1 - b1^t and
// bc2 = 1 - b2^t of step t (from the host, in fp64); sign = -1 ascends.
__global__ void k_adam(float *p, const float *g, float *m, float *v, long n, float lr, float b1,
                       float b2, float eps, float inv_bc1, float inv_bc2, float sign) {
  for (long i = blockIdx.x * (long)NTB + threadIdx.x; i < n; i += (long)gridDim.x * NTB) {
    const float gi = sign * g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi * inv_bc1) / (sqrtf(vi * inv_bc2) + eps);
  }
}

// ---------------------------------------------------------------- multi-output
// Q outputs sharing Z, the kernel, S~ and so T = L L^T, each with its own m~_q
// and targets (Section 4's multi-output layers with S~ tied across outputs).
// Per-output vectors are rows of [Q][ld] fp32 arrays, zero beyond M.
constexpr int MO_QMAX = 16;

__global__ void k_fill(float *p, int n, float v) {
  const int i = blockIdx.x * NTB + threadIdx.x;
  if (i < n) p[i] = v;
}

// the caller's [Q][M] rows into a zero-padded [Q][ld] array
__global__ void k_mo_pack(const float *src, int M, long ld, float *dst) {
  const int q = blockIdx.y;
  for (int i = blockIdx.x * NTB + threadIdx.x; i < ld; i += gridDim.x * NTB)
    dst[q * ld + i] = i < M ? src[(long)q * M + i] : 0.f;
}

// Y[q] = scale * A X[q] over j < Cn (lower: j <= i), one wave per row, grid.y = q
__global__ void k_mo_gemv(const float *A, long lda, int R, int Cn, const float *X, long ldx,
                          int lower, const double *scale, float *Y, long ldy) {
  const int q = blockIdx.y;
  const int row = blockIdx.x * (NTB / 64) + (threadIdx.x >> 6);
  if (row >= R) return;
  const float s = row_dot(A + (long)row * lda, X + q * ldx, nullptr,
                          lower ? min(Cn, row + 1) : Cn);
  if ((threadIdx.x & 63) == 0) Y[q * ldy + row] = scale ? (float)(*scale * (double)s) : s;
}

// mu[q][n] = b_q^T V_n = k_n^T P m~_q (V_n: row n of the operand-type Vt,
// zero-padded to cols, a multiple of 16 bytes of it), one wave per batch
// point, 16-byte loads
template <typename T>
__global__ void k_mo_mu(const T *Vt, long ld, int cols, int B, const float *Bh, long ldb, int Q,
                        float *mu, long ldm) {
  constexpr int KPL = 16 / (int)sizeof(T);
  const int n = blockIdx.x * (NTB / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (n >= B) return;
  float acc[MO_QMAX];
#pragma unroll
  for (int q = 0; q < MO_QMAX; ++q) acc[q] = 0.f;
  const T *v = Vt + (long)n * ld;
  for (int i = lane * KPL; i < cols; i += 64 * KPL) {
    const uint4 raw = *(const uint4 *)(v + i);
    const T *e = (const T *)&raw;
    float x[KPL];
#pragma unroll
    for (int u = 0; u < KPL; ++u) x[u] = to_f32(e[u]);
#pragma unroll
    for (int q = 0; q < MO_QMAX; ++q)
      if (q < Q) {
        const float *b = Bh + q * ldb + i;
#pragma unroll
        for (int u = 0; u < KPL; u += 4) {
          const f32x4 b4 = *(const f32x4 *)(b + u);
          acc[q] = fmaf(x[u], b4[0], acc[q]);
          acc[q] = fmaf(x[u + 1], b4[1], acc[q]);
          acc[q] = fmaf(x[u + 2], b4[2], acc[q]);
          acc[q] = fmaf(x[u + 3], b4[3], acc[q]);
        }
      }
  }
#pragma unroll
  for (int q = 0; q < MO_QMAX; ++q)
    if (q < Q) {
      const float s = wave_sum(acc[q]);
      if (lane == 0) mu[q * ldm + n] = s;
    }
}

// x_q = V alpha_q - Wu b_q, one workgroup per row of the operand-type V
// ([Mp][Bp]; alpha_q zero for n >= B), its waves splitting the row, 16-byte
// loads.  Launch with M workgroups.
template <typename T>
__global__ __launch_bounds__(NTB) void k_mo_x(const T *V, long ld, int M, int Bp,
                                              const float *al, long lda, int Q,
                                              const float *Wub, long ldw, float *Xq) {
  constexpr int KPL = 16 / (int)sizeof(T);
  __shared__ float shq[MO_QMAX][NTB / 64];
  const int i = blockIdx.x;
  if (i >= M) return;  // uniform across the workgroup
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  float acc[MO_QMAX];
#pragma unroll
  for (int q = 0; q < MO_QMAX; ++q) acc[q] = 0.f;
  const T *v = V + (long)i * ld;
  for (int n = (int)threadIdx.x * KPL; n < Bp; n += NTB * KPL) {  // Bp is a multiple of KPL
    const uint4 raw = *(const uint4 *)(v + n);
    const T *e = (const T *)&raw;
    float x[KPL];
#pragma unroll
    for (int u = 0; u < KPL; ++u) x[u] = to_f32(e[u]);
#pragma unroll
    for (int q = 0; q < MO_QMAX; ++q)
      if (q < Q) {
        const float *a = al + q * lda + n;
#pragma unroll
        for (int u = 0; u < KPL; u += 4) {
          const f32x4 a4 = *(const f32x4 *)(a + u);
          acc[q] = fmaf(x[u], a4[0], acc[q]);
          acc[q] = fmaf(x[u + 1], a4[1], acc[q]);
          acc[q] = fmaf(x[u + 2], a4[2], acc[q]);
          acc[q] = fmaf(x[u + 3], a4[3], acc[q]);
        }
      }
  }
#pragma unroll
  for (int q = 0; q < MO_QMAX; ++q)
    if (q < Q) {
      const float s = wave_sum(acc[q]);
      if (lane == 0) shq[q][wave] = s;
    }
  __syncthreads();
  if ((int)threadIdx.x < Q) {
    const int q = threadIdx.x;
    float t = 0.f;
#pragma unroll
    for (int w = 0; w < NTB / 64; ++w) t += shq[q][w];
    Xq[q * ldw + i] = t - Wub[q * ldw + i];
  }
}

// Rows n < B of Ut become sum_q b_q alpha_qn - 2 beta_n U_n, so that L times
// them is G_uf = sum_q (P m~_q) alpha_q^T - 2 P K_uf diag(beta) directly.
// 16 bytes of a row per thread (rows padded to ld, a multiple of that; U and
// b_q are zero beyond M, so the padding stays zero).  grid.x covers
// ceil(M / KPL) chunks, grid.y the rows.
template <typename T>
__global__ void k_mo_u3(T *Ut, long ld, int M, int B, const float *Bh, long ldb,
                        const float *al, long lda, int Q, const float *beta) {
  constexpr int KPL = 16 / (int)sizeof(T);
  const int chunks = (M + KPL - 1) / KPL;
  for (int n = blockIdx.y; n < B; n += gridDim.y) {
    const float bn = -2.f * beta[n];
    for (int c = blockIdx.x * NTB + threadIdx.x; c < chunks; c += gridDim.x * NTB) {
      const int i = c * KPL;
      T *p = Ut + (long)n * ld + i;
      uint4 raw = *(const uint4 *)p;
      T *e = (T *)&raw;
      float v[KPL];
#pragma unroll
      for (int u = 0; u < KPL; ++u) v[u] = bn * to_f32(e[u]);
      for (int q = 0; q < Q; ++q) {
        const float a = al[q * lda + n];
        const float *b = Bh + q * ldb + i;
#pragma unroll
        for (int u = 0; u < KPL; u += 4) {
          const f32x4 b4 = *(const f32x4 *)(b + u);
          v[u] = fmaf(b4[0], a, v[u]);
          v[u + 1] = fmaf(b4[1], a, v[u + 1]);
          v[u + 2] = fmaf(b4[2], a, v[u + 2]);
          v[u + 3] = fmaf(b4[3], a, v[u + 3]);
        }
      }
#pragma unroll
      for (int u = 0; u < KPL; ++u) e[u] = from_f32<T>(v[u]);
      *(uint4 *)p = raw;
    }
  }
}

// C = sum_q [-1/2 (x_q a_q^T + a_q x_q^T) - 1/2 b_q b_q^T] + V diag(beta) V^T
//     + Q [-1/2 (Wu + I) + 1/2 Q],  V diag(beta) V^T = -sum_s Ys[s]
// (the single-output C with each output's vector terms summed and the trace
// part, which every output's KL carries, counted Q times)
template <typename TC>
__global__ __launch_bounds__(NTB) void k_assemble_C_mo(const float *Ys, int nsplit,
                                                       long split_stride, const float *Wu,
                                                       const float *Qm, const float *A,
                                                       const float *Bh, const float *Xq,
                                                       long ldv, int Q, int M, long ld,
                                                       TC *Cm) {
  const int cpr = (M + 3) / 4;
  const long n = (long)M * cpr;
  for (long e = blockIdx.x * (long)NTB + threadIdx.x; e < n; e += (long)gridDim.x * NTB) {
    const int i = (int)(e / cpr), j0 = (int)(e % cpr) * 4;
    const long ij = (long)i * ld + j0;
    f32x4 ys = *(const f32x4 *)(Ys + ij);
    for (int s = 1; s < nsplit; ++s) ys += *(const f32x4 *)(Ys + s * split_stride + ij);
    const f32x4 wu = *(const f32x4 *)(Wu + ij), qm = *(const f32x4 *)(Qm + ij);
    f32x4 vec = {0.f, 0.f, 0.f, 0.f};
    for (int q = 0; q < Q; ++q) {
      const float *a = A + q * ldv, *b = Bh + q * ldv, *x = Xq + q * ldv;
      const f32x4 aj = *(const f32x4 *)(a + j0), bj = *(const f32x4 *)(b + j0),
                  xj = *(const f32x4 *)(x + j0);
      const float ai = a[i], bi = b[i], xi = x[i];
#pragma unroll
      for (int u = 0; u < 4; ++u) vec[u] -= 0.5f * (xi * aj[u] + ai * xj[u] + bi * bj[u]);
    }
    TC out[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const float tr = -0.5f * (wu[u] + (i == j0 + u ? 1.f : 0.f)) + 0.5f * qm[u];
      out[u] = from_f32<TC>(vec[u] - ys[u] + (float)Q * tr);
    }
    if constexpr (sizeof(TC) == 4) {
      *(f32x4 *)(Cm + ij) = f32x4{(float)out[0], (float)out[1], (float)out[2], (float)out[3]};
    } else {
      uint2 raw;
      __builtin_memcpy(&raw, out, 8);
      *(uint2 *)(Cm + ij) = raw;
    }
  }
}

// Likelihood of the Q outputs: per batch point the shared sigma_n^2 (from the
// U epilogue's partials), per output E_qn and dF/dmu_qn = c dE/dmu; beta_n =
// c sum_q dE/dsigma^2 (sigma^2 is shared) with sqrt(-beta_n) for the batch
// product; the last workgroup forms F = c sum E - KL with
//   KL = Q/2 (-tr(Q Wu) + tr W - M - log|T| - sum log s~) + 1/2 sum_q b_q^T Wu b_q.
struct LikMoArgs {
  const float *var_part; int n_var; long ldp;
  const CallArgs *ca;
  const float *Y; int Q;  // targets [B][Q]
  int B, Bp;
  const float *sfn; int lik; const double *gh; int ngh;
  const float *mu; float *al; long ldm;  // [Q][ldm]
  float *alpha, *beta, *sqnb;
  double *part;
  const double *gram_part; int n_gram;
  const float *Bh, *Wub; long ldv;
  const float *L; long ldl; int M;
  double *scal; int *flag; int *counter;
};

__global__ __launch_bounds__(NTB) void k_lik_mo(LikMoArgs a) {
  __shared__ double sh[7 * (NTB / 64)];
  __shared__ int s_last;
  const int n = blockIdx.x * NTB + threadIdx.x;
  double e = 0.0, vs = 0.0, dn = 0.0, bs = 0.0;
  if (n < a.B) {
    const double var = (double)a.sfn[0] - (double)slot_sum(a.var_part + n, a.n_var, a.ldp);
    const double c = a.ca->c;
    double dvs = 0.0;
    for (int q = 0; q < a.Q; ++q) {
      const double mu = a.mu[q * a.ldm + n], y = a.Y[(long)n * a.Q + q];
      double E, dmu, dv;
      if (a.lik == 0) {
        const double s2 = a.sfn[1];
        const double r = y - mu;
        E = -0.5 * log(2.0 * M_PI * s2) - (r * r + var) / (2.0 * s2);
        dmu = r / s2;
        dv = -0.5 / s2;
        dn += -0.5 / s2 + (r * r + var) / (2.0 * s2 * s2);
      } else {
        probit_terms(y, mu, var, a.gh, a.ngh, E, dmu, dv);
      }
      a.al[q * a.ldm + n] = (float)(c * dmu);
      e += E;
      dvs += dv;
    }
    a.alpha[n] = 0.f;
    a.beta[n] = (float)(c * dvs);
    a.sqnb[n] = (float)sqrt(fmax(0.0, -c * dvs));
    vs = var;
    bs = c * dvs;
  } else if (n < a.Bp) {
    a.alpha[n] = 0.f;
    a.beta[n] = 0.f;
    a.sqnb[n] = 0.f;
    for (int q = 0; q < a.Q; ++q) a.al[q * a.ldm + n] = 0.f;
  }
  double v[4] = {e, vs, dn, bs};
  block_sums<NTB, 4>(v, sh);
  if (threadIdx.x == 0) {
    double *p = a.part + 4 * blockIdx.x;
    p[0] = v[0]; p[1] = v[1]; p[2] = v[2]; p[3] = v[3];
  }
  if (!arrive_last(a.counter, &s_last)) return;
  double w[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < (int)gridDim.x; i += NTB) {
    w[0] += a.part[4 * i];
    w[1] += a.part[4 * i + 1];
  }
  for (int i = threadIdx.x; i < a.n_gram; i += NTB) {
    w[2] += a.gram_part[3 * i];
    w[3] += a.gram_part[3 * i + 1];
    w[4] += a.gram_part[3 * i + 2];
  }
  for (int q = 0; q < a.Q; ++q)
    for (int i = threadIdx.x; i < a.M; i += NTB)
      w[5] += (double)a.Bh[q * a.ldv + i] * (double)a.Wub[q * a.ldv + i];
  for (int i = threadIdx.x; i < a.M; i += NTB) w[6] += log(fabs((double)a.L[(long)i * a.ldl + i]));
  block_sums<NTB, 7>(w, sh);
  if (threadIdx.x == 0) {
    const double trw = w[2], qwu = w[3], r2 = w[4], quad = w[5], logdet = 2.0 * w[6];
    const double sls = a.scal[S_SUMLOGS];
    a.scal[S_QUAD] = quad;
    a.scal[S_LOGDET] = logdet;
    const double KL = 0.5 * ((double)a.Q * (-qwu + trw - (double)a.M - logdet - sls) + quad);
    const double data = a.ca->c * w[0];
    const double F = data - KL;
    if (!isfinite(F)) atomicOr(a.flag, FLAG_NONFINITE);
    if (a.ca->out_bound) *a.ca->out_bound = F;
    if (a.ca->out_terms) {
      double *o = a.ca->out_terms;
      o[0] = data; o[1] = KL; o[2] = w[1]; o[3] = sqrt(r2 / a.M);
      o[4] = trw; o[5] = qwu; o[6] = quad; o[7] = logdet;
    }
  }
}
