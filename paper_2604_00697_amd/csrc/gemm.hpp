// Tiled MFMA GEMM for gfx950 in "NT" form:
//     C[i][j] = sum_k A[i][k] * Bt[j][k]
// with both operands stored k-contiguous in the MFMA operand type, in
// zero-padded buffers (rows padded to the tile, k padded to the k-step), so
// every global load is an unconditional 16-byte vector.  Producers write
// their outputs in the layout the next product consumes (plain or
// transposed), which removes all transposes from the inner loops.
//
// Data path per workgroup (NT = 64 * WGM * WGN threads):
//   global (16 B per lane, 8 lanes per 128-byte k-row) --> registers
//   (optional per-k scaling) --> LDS, double buffered, rows padded by 16 B
//   --> 16x16 MFMA (fp32: 4 x 16x16x4, bf16/fp16: 16x16x32), fp32 accumulators
//   --> fp32 tile staged in LDS --> epilogue functor (stores, fused reductions).
// Triangular operands skip their zero k-blocks through the tile schedule.
#pragma once
#include "common.hpp"

// P_: k-tiles whose global loads are in flight while one tile is computed
// (register sets of prefetched operands).
template <int BM_, int BN_, int WGM_, int WGN_, typename T_, int P_ = 2>
struct Cfg {
  using T = T_;
  static constexpr int BM = BM_, BN = BN_, WGM = WGM_, WGN = WGN_, P = P_;
  static constexpr int NT = 64 * WGM * WGN;
  static constexpr int WM = BM / WGM, WN = BN / WGN;
  static constexpr int TM = WM / 16, TN = WN / 16;
  static constexpr int KPL = 16 / (int)sizeof(T);  // operand elements per 16 bytes
  static constexpr int BK = 8 * KPL;               // k per stage: 128 bytes per row
  static constexpr int LDK = BK + KPL;             // padded LDS row (elements): 144 bytes
  static constexpr int RPP = NT / 8;               // rows covered by one load pass
  static constexpr int PA = BM / RPP, PB = BN / RPP;
  static constexpr int LDC = BN + 1;               // epilogue staging row, floats
  static constexpr int SMEM_MAIN = 2 * (BM + BN) * LDK * (int)sizeof(T);
  // epilogue: staged tile + 16*NT bytes of reduction scratch (+ extra per epilogue)
  static constexpr int SMEM_EPI = (BM * LDC + 4 * NT) * (int)sizeof(float);
  static constexpr int smem(int extra) {
    return SMEM_MAIN > SMEM_EPI + extra ? SMEM_MAIN : SMEM_EPI + extra;
  }
  static_assert(WM % 16 == 0 && WN % 16 == 0, "wave tile must be a multiple of 16");
  static_assert(BM % RPP == 0 && BN % RPP == 0, "tile rows per load pass");
};

// One operand: k-contiguous rows of length >= the padded k extent.
// scale (optional, when the kernel's SA/SB flag is set): multiply element k by scale[k].
template <typename T>
struct Opnd {
  const T *p;
  long ld;
  const float *scale;
};

// ------------------------------------------------------------------ schedule
enum : int { K_LO_M0 = 1, K_LO_N0 = 2, K_HI_M1 = 4, K_HI_N1 = 8 };

// Maps blockIdx.x to an output tile and its k-range.
//   sym = 0: rectangular grid of mt x nt tiles;
//   sym = 1: lower-triangular tiles (I >= J) of an mt x mt grid.
// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2), so block b is renumbered to run consecutive tiles on one XCD; for
// rectangular grids consecutive tiles share a column block (I fastest), so an
// XCD streams one slice of the B operand against the whole A operand.
// rule: K_* bounds (k >= m0, k >= n0, k < m0+BM, k < n0+BN) skipping blocks of
// a triangular operand known to be zero.  nsplit > 1 splits the k-range into
// BK-aligned pieces (split-K) selected by blockIdx.y.
struct Sched {
  int mt, nt, sym, nsplit, K, rule;
  template <class C>
  IFS_DEV void tile(int &m0, int &n0, int &kb, int &ke, int &ti) const {
    const int ntile = sym ? mt * (mt + 1) / 2 : mt * nt;
    const int b = blockIdx.x;
    // XCD-contiguous renumbering: blocks b, b+8, b+16, ... share XCD b % 8
    const int per = (ntile + 7) / 8, rem = ntile % 8;
    const int x = b % 8, q = b / 8;
    int t;
    if (rem == 0 || x < rem) t = x * per + q;
    else t = rem * per + (x - rem) * (per - 1) + q;
    int I, J;
    if (sym) {
      I = (int)((sqrtf(8.0f * t + 1.0f) - 1.0f) * 0.5f);
      while ((I + 1) * (I + 2) / 2 <= t) ++I;
      while (I * (I + 1) / 2 > t) --I;
      J = t - I * (I + 1) / 2;
    } else {
      J = t / mt;
      I = t - J * mt;
    }
    ti = t;
    m0 = I * C::BM;
    n0 = J * C::BN;
    int lo = 0, hi = K;
    if (rule & K_LO_M0) lo = max(lo, m0);
    if (rule & K_LO_N0) lo = max(lo, n0);
    if (rule & K_HI_M1) hi = min(hi, m0 + C::BM);
    if (rule & K_HI_N1) hi = min(hi, n0 + C::BN);
    lo = (lo / C::BK) * C::BK;
    if (nsplit > 1) {
      const int nkt = hi > lo ? (hi - lo + C::BK - 1) / C::BK : 0;
      const int per_s = (nkt + nsplit - 1) / nsplit;
      const int s = blockIdx.y;
      kb = lo + s * per_s * C::BK;
      ke = min(hi, lo + (s + 1) * per_s * C::BK);
    } else {
      kb = lo;
      ke = hi;
    }
  }
};

struct TileInfo {
  int m0, n0, ti, split;
};

// 16 bytes of operands, optionally scaled element-wise by s[k .. k+KPL).
template <typename T, bool SCALE>
IFS_DEV uint4 load_chunk(const T *p, const float *s) {
  uint4 v = *(const uint4 *)p;
  if constexpr (SCALE) {
    if constexpr (sizeof(T) == 4) {
      float *f = (float *)&v;
      const f32x4 sc = *(const f32x4 *)s;
#pragma unroll
      for (int j = 0; j < 4; ++j) f[j] *= sc[j];
    } else {
      T *h = (T *)&v;
      const f32x4 s0 = *(const f32x4 *)s, s1 = *(const f32x4 *)(s + 4);
#pragma unroll
      for (int j = 0; j < 4; ++j) h[j] = from_f32<T>(to_f32(h[j]) * s0[j]);
#pragma unroll
      for (int j = 0; j < 4; ++j) h[4 + j] = from_f32<T>(to_f32(h[4 + j]) * s1[j]);
    }
  }
  return v;
}

// ------------------------------------------------------------------ kernel
template <class C, bool SA, bool SB, class EPI>
__global__ __launch_bounds__(C::NT) void gemm_kernel(Opnd<typename C::T> A,
                                                     Opnd<typename C::T> Bt, Sched sc, EPI epi) {
  using T = typename C::T;
  using V = typename Vec16<T>::type;
  constexpr int BM = C::BM, BN = C::BN, BK = C::BK, LDK = C::LDK, KPL = C::KPL;

  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  T *As = (T *)smem_raw;          // [2][BM][LDK]
  T *Bs = As + 2 * BM * LDK;      // [2][BN][LDK]

  int m0, n0, kb, ke, ti;
  sc.tile<C>(m0, n0, kb, ke, ti);
  const int nk = ke > kb ? (ke - kb + BK - 1) / BK : 0;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave / C::WGN, wn = wave % C::WGN;
  const int lr = lane & 15, kq = lane >> 4;
  const int lrow = tid >> 3, lch = (tid & 7) * KPL;  // load row within a pass, k offset

  f32x4 acc[C::TM][C::TN];
#pragma unroll
  for (int i = 0; i < C::TM; ++i)
#pragma unroll
    for (int j = 0; j < C::TN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  const T *pa = A.p + (long)(m0 + lrow) * A.ld + lch;
  const T *pb = Bt.p + (long)(n0 + lrow) * Bt.ld + lch;
  constexpr int P = C::P;
  uint4 ra[P][C::PA], rb[P][C::PB];  // P register sets of prefetched k-tiles

  auto fetch = [&](int set, int k0) {
#pragma unroll
    for (int p = 0; p < C::PA; ++p)
      ra[set][p] = load_chunk<T, SA>(pa + (long)p * C::RPP * A.ld + k0,
                                     SA ? A.scale + k0 + lch : nullptr);
#pragma unroll
    for (int p = 0; p < C::PB; ++p)
      rb[set][p] = load_chunk<T, SB>(pb + (long)p * C::RPP * Bt.ld + k0,
                                     SB ? Bt.scale + k0 + lch : nullptr);
  };
  auto stash = [&](int set, int buf) {
    T *a = As + buf * BM * LDK + lrow * LDK + lch;
    T *b = Bs + buf * BN * LDK + lrow * LDK + lch;
#pragma unroll
    for (int p = 0; p < C::PA; ++p) *(uint4 *)(a + p * C::RPP * LDK) = ra[set][p];
#pragma unroll
    for (int p = 0; p < C::PB; ++p) *(uint4 *)(b + p * C::RPP * LDK) = rb[set][p];
  };
  auto compute = [&](int buf) {
    const T *a = As + buf * BM * LDK + (wm * C::WM + lr) * LDK;
    const T *b = Bs + buf * BN * LDK + (wn * C::WN + lr) * LDK;
    // all fragments of the k-tile are read before the first MFMA
    V av[2][C::TM], bv[2][C::TN];
#pragma unroll
    for (int kc = 0; kc < 2; ++kc) {
      const int koff = kc * 4 * KPL + kq * KPL;
#pragma unroll
      for (int i = 0; i < C::TM; ++i) av[kc][i] = *(const V *)(a + i * 16 * LDK + koff);
#pragma unroll
      for (int j = 0; j < C::TN; ++j) bv[kc][j] = *(const V *)(b + j * 16 * LDK + koff);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int kc = 0; kc < 2; ++kc)
#pragma unroll
      for (int i = 0; i < C::TM; ++i)
#pragma unroll
        for (int j = 0; j < C::TN; ++j) acc[i][j] = mfma16(av[kc][i], bv[kc][j], acc[i][j]);
  };

  // k-tile `it` lives in register set it % P and LDS buffer it % 2.  Fetch
  // addresses are clamped to the last k-tile (a harmless re-read), so the
  // steady-state loop has no branches and the accumulators stay in place.
  static_assert(P == 2, "the main loop is unrolled for two register sets");
  auto kclamp = [&](int it) { return kb + min(it, nk - 1) * BK; };
  if (nk > 0) {
    fetch(0, kclamp(0));
    fetch(1, kclamp(1));
    int it = 0;
    // scheduling fences keep each fetch ahead of the compute that hides it
    for (; it + 2 <= nk; it += 2) {
      stash(0, 0);
      __syncthreads();
      fetch(0, kclamp(it + 2));
      __builtin_amdgcn_sched_barrier(0);
      compute(0);
      __builtin_amdgcn_sched_barrier(0);
      stash(1, 1);
      __syncthreads();
      fetch(1, kclamp(it + 3));
      __builtin_amdgcn_sched_barrier(0);
      compute(1);
      __builtin_amdgcn_sched_barrier(0);
    }
    if (it < nk) {
      stash(0, 0);
      __syncthreads();
      compute(0);
    }
  }
  __syncthreads();
  // stage the fp32 accumulator tile in LDS: Cs[r][c], r < BM, c < BN
  float *Cs = (float *)smem_raw;
#pragma unroll
  for (int i = 0; i < C::TM; ++i)
#pragma unroll
    for (int j = 0; j < C::TN; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        Cs[(wm * C::WM + i * 16 + 4 * kq + q) * C::LDC + wn * C::WN + j * 16 + lr] = acc[i][j][q];
  __syncthreads();
  TileInfo t{m0, n0, ti, (int)blockIdx.y};
  epi.template run<C>(Cs, t);
}

// Host-side launch helper.  extra: LDS bytes the epilogue needs beyond the
// staged tile and its scratch.
template <class C, bool SA, bool SB, class EPI>
static inline hipError_t launch_gemm(hipStream_t st, const Opnd<typename C::T> &A,
                                     const Opnd<typename C::T> &Bt, const Sched &sc,
                                     const EPI &epi, int extra = 0) {
  const int ntile = sc.sym ? sc.mt * (sc.mt + 1) / 2 : sc.mt * sc.nt;
  if (ntile <= 0) return hipSuccess;
  dim3 grid(ntile, sc.nsplit > 1 ? sc.nsplit : 1);
  auto kern = gemm_kernel<C, SA, SB, EPI>;
  const int smem = C::smem(extra);
  static int attr_bytes = 0;
  if (smem > attr_bytes) {
    hipError_t e = hipFuncSetAttribute((const void *)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, smem);
    if (e != hipSuccess) return e;
    attr_bytes = smem;
  }
  hipLaunchKernelGGL(kern, grid, dim3(C::NT), smem, st, A, Bt, sc, epi);
  return hipGetLastError();
}
