// Tiled MFMA GEMM for gfx950 with pluggable operand loaders, tile schedules
// and epilogues.  C[m][n] = sum_k A(m,k) B(k,n) over a k-range chosen per tile
// (triangular operands skip their zero blocks).
//
// Data path per workgroup (NT = 64 * WGM * WGN threads):
//   global --(loader: bounds, triangular mask, scaling, fp32 -> operand type)-->
//   registers --> LDS (double buffered, k-contiguous rows, 16-byte padding) -->
//   16x16 MFMA tiles (fp32: 16x16x4, bf16/fp16: 16x16x32) with fp32 accumulators
//   --> fp32 tile staged in LDS --> epilogue functor (stores, fused reductions).
#pragma once
#include "common.hpp"

template <int BM_, int BN_, int WGM_, int WGN_, int KCH_, typename T_>
struct Cfg {
  using T = T_;
  static constexpr int BM = BM_, BN = BN_, WGM = WGM_, WGN = WGN_, KCH = KCH_;
  static constexpr int NT = 64 * WGM * WGN;
  static constexpr int WM = BM / WGM, WN = BN / WGN;
  static constexpr int TM = WM / 16, TN = WN / 16;
  static constexpr int KPL = 16 / (int)sizeof(T);  // operand elements per 16 bytes
  static constexpr int BK = 4 * KPL * KCH;         // k per LDS tile
  static constexpr int LDK = BK + KPL;             // padded LDS row, elements
  static constexpr int LDC = BN + 1;               // epilogue staging row, floats
  static constexpr int SMEM_MAIN = 2 * (BM + BN) * LDK * (int)sizeof(T);
  // epilogue: staged tile + 16*NT bytes of reduction scratch (+ extra per epilogue)
  static constexpr int SMEM_EPI = (BM * LDC + 4 * NT) * (int)sizeof(float);
  static constexpr int smem(int extra) {
    return SMEM_MAIN > SMEM_EPI + extra ? SMEM_MAIN : SMEM_EPI + extra;
  }
  static_assert(WM % 16 == 0 && WN % 16 == 0, "wave tile must be a multiple of 16");
  static_assert(BM % 4 == 0 && BN % 4 == 0 && BK % 4 == 0, "4x4 load chunks");
};

// ------------------------------------------------------------------ transforms
// Applied to element (a, b) of the stored source matrix after loading.
struct XfNone {
  IFS_DEV float operator()(float v, int, int) const { return v; }
};
struct XfLower {  // keep the lower triangle (a >= b)
  IFS_DEV float operator()(float v, int a, int b) const { return a >= b ? v : 0.f; }
};
struct XfLowerScaleRow {  // diag(s) L : lower triangle times s[a]
  const float *s;
  IFS_DEV float operator()(float v, int a, int b) const { return a >= b ? v * s[a] : 0.f; }
};
struct XfScaleCol {  // A diag(s)
  const float *s;
  IFS_DEV float operator()(float v, int, int b) const { return v * s[b]; }
};
// Natural-gradient middle factor from the lower triangle of W = L^T A L:
// tril(W) - (I + diag(W))/2, i.e. W_ab below the diagonal, (W_aa - 1)/2 on it.
struct XfNatgrad {
  IFS_DEV float operator()(float v, int a, int b) const {
    return a > b ? v : (a == b ? 0.5f * (v - 1.0f) : 0.f);
  }
};

// ------------------------------------------------------------------ loaders
// Logical operand element (r, k): r is the row of A (m) or the column of B (n).
// The stored matrix p (leading dimension ld) holds it at source coordinates
// (a, b) = KC ? (r, k) : (k, r).  Rows a < AR and columns b < BC are valid;
// everything else reads as zero.  load4 returns 4 consecutive elements along
// the contiguous source dimension starting at (r, k).
template <typename S, bool KC_, class Xf>
struct Ld {
  static constexpr bool KC = KC_;
  const S *p;
  long ld;
  int AR, BC;
  int vec;  // 1 if ld and p allow aligned 4-element vector loads
  Xf xf;
  IFS_DEV void load4(int r, int k, float v[4]) const {
    const int a = KC ? r : k, b = KC ? k : r;
    const bool rowok = a < AR;
    const S *q = p + (long)a * ld + b;
    if (rowok && vec && b + 3 < BC) {
      if constexpr (sizeof(S) == 4) {
        const f32x4 t = *(const f32x4 *)q;
        v[0] = t[0]; v[1] = t[1]; v[2] = t[2]; v[3] = t[3];
      } else {
        typedef S s4 __attribute__((ext_vector_type(4)));
        const s4 t = *(const s4 *)q;
        v[0] = to_f32(t[0]); v[1] = to_f32(t[1]); v[2] = to_f32(t[2]); v[3] = to_f32(t[3]);
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) v[j] = xf(v[j], a, b + j);
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j)
        v[j] = (rowok && b + j < BC) ? xf(to_f32(q[j]), a, b + j) : 0.f;
    }
  }
};

// ------------------------------------------------------------------ schedule
enum : int { K_LO_M0 = 1, K_LO_N0 = 2, K_HI_M1 = 4, K_HI_N1 = 8 };

// Maps blockIdx.x to an output tile and its k-range.
//   sym = 0: rectangular grid mt x nt (row-major over tiles);
//   sym = 1: lower-triangular tiles (I >= J) of an mt x mt grid.
// rule: bitmask of K_* bounds (k >= m0, k >= n0, k < m0+BM, k < n0+BN) that
// skip blocks of a triangular operand known to be zero.  nsplit > 1 splits
// the k-range into BK-aligned pieces (split-K); blockIdx.y selects the piece.
struct Sched {
  int mt, nt, sym, nsplit, K, rule;
  template <class C>
  IFS_DEV bool tile(int &m0, int &n0, int &kb, int &ke, int &ti) const {
    int I, J;
    const int t = blockIdx.x;
    if (sym) {
      I = (int)((sqrtf(8.0f * t + 1.0f) - 1.0f) * 0.5f);
      while ((I + 1) * (I + 2) / 2 <= t) ++I;
      while (I * (I + 1) / 2 > t) --I;
      J = t - I * (I + 1) / 2;
    } else {
      I = t / nt;
      J = t - I * nt;
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
      const int per = (nkt + nsplit - 1) / nsplit;
      const int s = blockIdx.y;
      kb = lo + s * per * C::BK;
      ke = min(hi, lo + (s + 1) * per * C::BK);
    } else {
      kb = lo;
      ke = hi;
    }
    return true;
  }
};

struct TileInfo {
  int m0, n0, ti, split;
};

// ------------------------------------------------------------------ kernel
template <class C, class LA, class LB, class EPI>
__global__ __launch_bounds__(C::NT) void gemm_kernel(LA la, LB lb, Sched sc, EPI epi) {
  using T = typename C::T;
  using V = typename Vec16<T>::type;
  constexpr int NT = C::NT, BM = C::BM, BN = C::BN, BK = C::BK, LDK = C::LDK;
  constexpr int CA = (BM / 4) * (BK / 4), CB = (BN / 4) * (BK / 4);
  constexpr int PA = (CA + NT - 1) / NT, PB = (CB + NT - 1) / NT;

  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  T *As = (T *)smem_raw;                 // [2][BM][LDK]
  T *Bs = As + 2 * BM * LDK;             // [2][BN][LDK]

  int m0, n0, kb, ke, ti;
  sc.tile<C>(m0, n0, kb, ke, ti);
  const int nk = ke > kb ? (ke - kb + BK - 1) / BK : 0;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave / C::WGN, wn = wave % C::WGN;
  const int lr = lane & 15, kq = lane >> 4;

  f32x4 acc[C::TM][C::TN];
#pragma unroll
  for (int i = 0; i < C::TM; ++i)
#pragma unroll
    for (int j = 0; j < C::TN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  T ra[PA][4][4], rb[PB][4][4];

  auto chunk_rk = [](int c, bool kc, int R, int &cr, int &ck) {
    if (kc) { cr = c / (BK / 4); ck = c % (BK / 4); }
    else    { ck = c / (R / 4); cr = c % (R / 4); }
  };
  auto fetch = [&](int k0) {
#pragma unroll
    for (int i = 0; i < PA; ++i) {
      const int c = tid + i * NT;
      if (CA % NT == 0 || c < CA) {
        int cr, ck;
        chunk_rk(c, LA::KC, BM, cr, ck);
        float v[4][4];
        if (LA::KC) {
#pragma unroll
          for (int rr = 0; rr < 4; ++rr) la.load4(m0 + 4 * cr + rr, k0 + 4 * ck, v[rr]);
        } else {
          float w[4][4];
#pragma unroll
          for (int kk = 0; kk < 4; ++kk) la.load4(m0 + 4 * cr, k0 + 4 * ck + kk, w[kk]);
#pragma unroll
          for (int rr = 0; rr < 4; ++rr)
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) v[rr][kk] = w[kk][rr];
        }
#pragma unroll
        for (int rr = 0; rr < 4; ++rr)
#pragma unroll
          for (int kk = 0; kk < 4; ++kk) ra[i][rr][kk] = from_f32<T>(v[rr][kk]);
      }
    }
#pragma unroll
    for (int i = 0; i < PB; ++i) {
      const int c = tid + i * NT;
      if (CB % NT == 0 || c < CB) {
        int cr, ck;
        chunk_rk(c, LB::KC, BN, cr, ck);
        float v[4][4];
        if (LB::KC) {
#pragma unroll
          for (int rr = 0; rr < 4; ++rr) lb.load4(n0 + 4 * cr + rr, k0 + 4 * ck, v[rr]);
        } else {
          float w[4][4];
#pragma unroll
          for (int kk = 0; kk < 4; ++kk) lb.load4(n0 + 4 * cr, k0 + 4 * ck + kk, w[kk]);
#pragma unroll
          for (int rr = 0; rr < 4; ++rr)
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) v[rr][kk] = w[kk][rr];
        }
#pragma unroll
        for (int rr = 0; rr < 4; ++rr)
#pragma unroll
          for (int kk = 0; kk < 4; ++kk) rb[i][rr][kk] = from_f32<T>(v[rr][kk]);
      }
    }
  };
  auto stash = [&](int buf) {
    T *A = As + buf * BM * LDK;
    T *Bq = Bs + buf * BN * LDK;
#pragma unroll
    for (int i = 0; i < PA; ++i) {
      const int c = tid + i * NT;
      if (CA % NT == 0 || c < CA) {
        int cr, ck;
        chunk_rk(c, LA::KC, BM, cr, ck);
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
          T *dst = A + (4 * cr + rr) * LDK + 4 * ck;
#pragma unroll
          for (int kk = 0; kk < 4; ++kk) dst[kk] = ra[i][rr][kk];
        }
      }
    }
#pragma unroll
    for (int i = 0; i < PB; ++i) {
      const int c = tid + i * NT;
      if (CB % NT == 0 || c < CB) {
        int cr, ck;
        chunk_rk(c, LB::KC, BN, cr, ck);
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
          T *dst = Bq + (4 * cr + rr) * LDK + 4 * ck;
#pragma unroll
          for (int kk = 0; kk < 4; ++kk) dst[kk] = rb[i][rr][kk];
        }
      }
    }
  };

  if (nk > 0) fetch(kb);
  for (int it = 0; it < nk; ++it) {
    const int buf = it & 1;
    stash(buf);
    __syncthreads();
    if (it + 1 < nk) fetch(kb + (it + 1) * BK);
    const T *A = As + buf * BM * LDK + (wm * C::WM + lr) * LDK;
    const T *Bq = Bs + buf * BN * LDK + (wn * C::WN + lr) * LDK;
#pragma unroll
    for (int kc = 0; kc < C::KCH; ++kc) {
      const int koff = kc * 4 * C::KPL + kq * C::KPL;
      V a[C::TM], b[C::TN];
#pragma unroll
      for (int i = 0; i < C::TM; ++i) a[i] = *(const V *)(A + i * 16 * LDK + koff);
#pragma unroll
      for (int j = 0; j < C::TN; ++j) b[j] = *(const V *)(Bq + j * 16 * LDK + koff);
#pragma unroll
      for (int i = 0; i < C::TM; ++i)
#pragma unroll
        for (int j = 0; j < C::TN; ++j) acc[i][j] = mfma16(a[i], b[j], acc[i][j]);
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

// Host-side launch helper.
// extra: LDS bytes the epilogue needs beyond the staged tile and scratch.
template <class C, class LA, class LB, class EPI>
static inline hipError_t launch_gemm(hipStream_t st, const LA &la, const LB &lb,
                                     const Sched &sc, const EPI &epi, int extra = 0) {
  const int ntile = sc.sym ? sc.mt * (sc.mt + 1) / 2 : sc.mt * sc.nt;
  if (ntile <= 0) return hipSuccess;
  dim3 grid(ntile, sc.nsplit > 1 ? sc.nsplit : 1);
  auto kern = gemm_kernel<C, LA, LB, EPI>;
  const int smem = C::smem(extra);
  static int attr_bytes = 0;
  if (smem > attr_bytes) {
    hipError_t e = hipFuncSetAttribute((const void *)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, smem);
    if (e != hipSuccess) return e;
    attr_bytes = smem;
  }
  hipLaunchKernelGGL(kern, grid, dim3(C::NT), smem, st, la, lb, sc, epi);
  return hipGetLastError();
}
