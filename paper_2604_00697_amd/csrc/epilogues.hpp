// GEMM epilogues of the inverse-free SVGP iteration.  Each runs with the whole
// workgroup after the fp32 accumulator tile Cs[BM][LDC] has been staged in LDS;
// 16*NT bytes of scratch LDS follow the tile, then any epilogue-specific LDS.
// Outputs are written in the layout their consumer's NT product reads:
// "T" suffixes below mark transposed stores (out[j][i] = C[i][j]).
#pragma once
#include "gemm.hpp"

// Each thread owns chunks of VEC consecutive elements of the tile:
//   row chunk    (r, c .. c+VEC)   -- one 16/32-byte access of a row-major array
//   column chunk (r .. r+VEC, c)   -- one access of a transposed array
// Workspace buffers are padded to whole tiles, so every chunk access is in
// bounds and unconditional; elements outside the logical extent are written
// as zeros, which keeps the padding of every operand zero.
constexpr int VEC = 8;

template <typename T>
struct alignas(VEC * sizeof(T)) Pack {
  T v[VEC];
};

template <typename T>
IFS_DEV void ld_pack(const T *p, float (&x)[VEC]) {
  const Pack<T> v = *(const Pack<T> *)p;
#pragma unroll
  for (int q = 0; q < VEC; ++q) x[q] = to_f32(v.v[q]);
}
template <typename T>
IFS_DEV void st_pack(T *p, const float (&x)[VEC]) {
  Pack<T> v;
#pragma unroll
  for (int q = 0; q < VEC; ++q) v.v[q] = from_f32<T>(x[q]);
  *(Pack<T> *)p = v;
}

template <class C>
struct Chunks {
  static constexpr int RPR = C::BN / VEC;                  // row chunks per tile row
  static constexpr int CPC = C::BM / VEC;                  // column chunks per tile column
  static constexpr int N = C::BM * C::BN / (VEC * C::NT);  // chunks per thread
  static_assert((C::BM * C::BN) % (VEC * C::NT) == 0, "tile / chunk mismatch");
  static_assert(C::NT % RPR == 0, "a thread's row chunks share their columns");
  // row chunk k of this thread; c is the same for every k
  static IFS_DEV void row(int k, int &r, int &c) {
    const int ch = threadIdx.x + k * C::NT;
    r = ch / RPR;
    c = (ch % RPR) * VEC;
  }
  static IFS_DEV void col(int k, int &r, int &c) {
    const int ch = threadIdx.x + k * C::NT;
    c = ch / CPC;
    r = (ch % CPC) * VEC;
  }
};

#define CS(r, c) Cs[(r) * C::LDC + (c)]

// A chunk of VEC staged values along a row (cs_row: columns c..c+VEC-1 of row
// r) or down a column (cs_col: rows r..r+VEC-1 of column c).  The staged tile
// always spans the whole BM x BN block, so the reads are unconditional (and
// stay in flight together); values outside the valid region (ok false, or
// index q >= nq along the chunk) are replaced by zero afterwards.
// pin: an empty asm statement that takes v in a register and hands it back,
// so a value loaded before it cannot be re-read later inside the branch of a
// select.  Guarded uses of staged values load every value first (plain LDS
// reads, all in flight together), pin them, then select.
IFS_DEV void pin(float &v) { asm volatile("" : "+v"(v)); }
#define CSV(r, c) Cs[(r) * C::LDC + (c)]

template <class C>
IFS_DEV void cs_row(const float *Cs, int r, int c, bool ok, int nq, float (&x)[VEC]) {
  float v[VEC];
#pragma unroll
  for (int q = 0; q < VEC; ++q) v[q] = CSV(r, c + q);
#pragma unroll
  for (int q = 0; q < VEC; ++q) pin(v[q]);
#pragma unroll
  for (int q = 0; q < VEC; ++q) x[q] = (ok && q < nq) ? v[q] : 0.f;
}
template <class C>
IFS_DEV void cs_col(const float *Cs, int r, int c, bool ok, int nq, float (&x)[VEC]) {
  float v[VEC];
#pragma unroll
  for (int q = 0; q < VEC; ++q) v[q] = CSV(r + q, c);
#pragma unroll
  for (int q = 0; q < VEC; ++q) pin(v[q]);
#pragma unroll
  for (int q = 0; q < VEC; ++q) x[q] = (ok && q < nq) ? v[q] : 0.f;
}

// Sum of one double per thread over the workgroup, result in thread 0.
template <class C>
IFS_DEV double tile_sum(double v, const float *Cs) {
  double *sh = (double *)(Cs + C::BM * C::LDC);
  return block_sum<C::NT>(v, sh);
}

// Column sums of the staged tile over its BM rows (NT / BN threads per column,
// partials combined in the scratch LDS), accumulated in A.  Valid for threads
// with g == 0, where c = threadIdx.x % BN.
template <class C, typename A = float>
IFS_DEV A tile_colsum(const float *Cs) {
  constexpr int RG = C::NT / C::BN;
  static_assert(C::NT % C::BN == 0, "column partial layout");
  A *sh = (A *)(Cs + C::BM * C::LDC);
  const int c = threadIdx.x % C::BN, g = threadIdx.x / C::BN;
  A s0 = 0, s1 = 0, s2 = 0, s3 = 0;
#pragma unroll 4
  for (int r = g; r < C::BM; r += 4 * RG) {
    s0 += (A)CS(r, c);
    s1 += (A)CS(r + RG, c);
    s2 += (A)CS(r + 2 * RG, c);
    s3 += (A)CS(r + 3 * RG, c);
  }
  A s = (s0 + s1) + (s2 + s3);
  sh[threadIdx.x] = s;
  __syncthreads();
  if (g == 0)
    for (int k = 1; k < RG; ++k) s += sh[k * C::BN + c];
  __syncthreads();
  return s;
}

// Small MFMA product of LDS operands, used for the D-wide reductions of the
// gradient epilogues:  Out[i][d] = sum_k A[i][k] Z[k][d],  i < R, d < DP,
// with A = H (row-major, stride ldh) or, TRANS, A = H^T.  Z is row-major
// [K][ldz].  R = 16 * TI * NW (each wave owns TI row tiles), K a multiple of 4,
// DP a multiple of 16 (d tiles two at a time, then a last single one).  Each
// output element goes to sink(i, d, value) from the lane that holds it.
// F64: the fp32 operands are widened and contracted on the fp64 matrix cores
// (exact products, fp64 sums), for the fp32 form, whose gradient sums cancel;
// otherwise fp32 MFMA.
template <bool F64>
struct RedMfma {
  using Acc = typename std::conditional<F64, f64x4, f32x4>::type;
  static IFS_DEV Acc op(float a, float b, Acc c) {
    if constexpr (F64) return __builtin_amdgcn_mfma_f64_16x16x4f64((double)a, (double)b, c, 0, 0, 0);
    else return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // row of the 16 x 16 output block that accumulator slot q of lane group l4
  // holds (the fp64 form interleaves the rows across the lane groups)
  static IFS_DEV int row(int l4, int q) { return F64 ? 4 * q + l4 : 4 * l4 + q; }
};

template <int NW, int TI, bool TRANS, bool F64 = false, class F>
IFS_DEV void lds_mfma(const float *H, int ldh, int K, const float *Z, int ldz, int DP,
                      F &&sink) {
  using R = RedMfma<F64>;
  using Acc = typename R::Acc;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l16 = lane & 15, l4 = lane >> 4;
  const int ib = wave * TI * 16;
  auto a_at = [&](int r, int k) { return TRANS ? H[k * ldh + r] : H[r * ldh + k]; };
  int d0 = 0;
  for (; d0 + 32 <= DP; d0 += 32) {
    Acc acc[TI][2];
#pragma unroll
    for (int i = 0; i < TI; ++i) acc[i][0] = acc[i][1] = Acc{0, 0, 0, 0};
#pragma unroll 4
    for (int k0 = 0; k0 < K; k0 += 4) {
      const float b0 = Z[(k0 + l4) * ldz + d0 + l16], b1 = Z[(k0 + l4) * ldz + d0 + 16 + l16];
#pragma unroll
      for (int i = 0; i < TI; ++i) {
        const float a = a_at(ib + 16 * i + l16, k0 + l4);
        acc[i][0] = R::op(a, b0, acc[i][0]);
        acc[i][1] = R::op(a, b1, acc[i][1]);
      }
    }
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int q = 0; q < 4; ++q) sink(ib + 16 * i + R::row(l4, q), d0 + 16 * h + l16, acc[i][h][q]);
  }
  if (d0 < DP) {
    Acc acc[TI];
#pragma unroll
    for (int i = 0; i < TI; ++i) acc[i] = Acc{0, 0, 0, 0};
#pragma unroll 4
    for (int k0 = 0; k0 < K; k0 += 4) {
      const float b0 = Z[(k0 + l4) * ldz + d0 + l16];
#pragma unroll
      for (int i = 0; i < TI; ++i) acc[i] = R::op(a_at(ib + 16 * i + l16, k0 + l4), b0, acc[i]);
    }
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
      for (int q = 0; q < 4; ++q) sink(ib + 16 * i + R::row(l4, q), d0 + l16, acc[i][q]);
  }
}

// The same product on the bf16 matrix cores (the reduced-precision forms):
// both fp32 operands are split into bf16 hi + lo parts as their fragments are
// read, and each 16 x 16 x 32 block takes hi hi + hi lo + lo hi (products to
// about 16 significant bits, fp32 sums: far below the bf16 / fp16 rounding of
// the GEMM operands that produced H), three instructions where the fp32
// instruction needs eight.  K a multiple of 32, DP a multiple of 16 up to 64;
// each of the workgroup's waves owns TI row tiles of 16; Out to
// sink(i, d, value).
IFS_DEV void split_bf16(const float (&x)[8], bf16x8 &hi, bf16x8 &lo) {
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const __bf16 h = (__bf16)x[j];
    hi[j] = h;
    lo[j] = (__bf16)(x[j] - (float)h);
  }
}
template <int TI, class F>
IFS_DEV void lds_mfma_split(const float *H, int ldh, int K, const float *Z, int ldz, int DP,
                            F &&sink) {
  constexpr int MAXDT = 4;  // d tiles of 16 (DP <= 64)
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l16 = lane & 15, l4 = lane >> 4;
  const int ib = wave * TI * 16;
  f32x4 acc[TI][MAXDT];
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int t = 0; t < MAXDT; ++t) acc[i][t] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += 32) {
    // A fragments: row ib + 16 i + l16, k = k0 + 8 l4 + j; each is read and
    // split once for all d tiles
    float ha[TI][8];
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
      for (int j = 0; j < 8; ++j) ha[i][j] = H[(ib + 16 * i + l16) * ldh + k0 + 8 * l4 + j];
    bf16x8 ah[TI], al[TI];
#pragma unroll
    for (int i = 0; i < TI; ++i) split_bf16(ha[i], ah[i], al[i]);
#pragma unroll
    for (int t = 0; t < MAXDT; ++t) {
      if (16 * t >= DP) break;
      // B fragment: column 16 t + l16, k = k0 + 8 l4 + j
      float zb[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) zb[j] = Z[(k0 + 8 * l4 + j) * ldz + 16 * t + l16];
      bf16x8 bh, bl;
      split_bf16(zb, bh, bl);
#pragma unroll
      for (int i = 0; i < TI; ++i) {
        acc[i][t] = mfma16(ah[i], bh, acc[i][t]);
        acc[i][t] = mfma16(ah[i], bl, acc[i][t]);
        acc[i][t] = mfma16(al[i], bh, acc[i][t]);
      }
    }
  }
#pragma unroll
  for (int t = 0; t < MAXDT; ++t) {
    if (16 * t >= DP) break;
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
      for (int q = 0; q < 4; ++q) sink(ib + 16 * i + 4 * l4 + q, 16 * t + l16, (double)acc[i][t][q]);
  }
}

// Row sums of the staged tile over its BN columns (NT / BM threads per row,
// partials combined in the scratch LDS), accumulated in A.  Valid for threads
// with threadIdx.x < BM, where the row is threadIdx.x.
template <class C, typename A = float>
IFS_DEV A tile_rowsum(const float *Cs) {
  constexpr int CG = C::NT / C::BM;  // column groups per row
  static_assert(C::NT % C::BM == 0 && C::BN % (4 * CG) == 0, "row partial layout");
  A *sh = (A *)(Cs + C::BM * C::LDC);
  const int r = threadIdx.x % C::BM, g = threadIdx.x / C::BM;
  constexpr int W = C::BN / CG;  // columns per group
  A s0 = 0, s1 = 0, s2 = 0, s3 = 0;
#pragma unroll 4
  for (int c = g * W; c < (g + 1) * W; c += 4) {
    s0 += (A)CS(r, c);
    s1 += (A)CS(r, c + 1);
    s2 += (A)CS(r, c + 2);
    s3 += (A)CS(r, c + 3);
  }
  A s = (s0 + s1) + (s2 + s3);
  sh[threadIdx.x] = s;
  __syncthreads();
  if (g == 0)
    for (int k = 1; k < CG; ++k) s += sh[k * C::BM + r];
  __syncthreads();
  return s;
}

// ---------------------------------------------------------------- plain stores
// out[gi][gj] = acc for rows < R, cols < N (zeros elsewhere in the tile);
// optional transposed mirror for off-diagonal tiles of a symmetric lower-tile
// schedule; split-K piece s writes to out + s * split_stride.
template <typename TO>
struct EpiStore {
  TO *out;
  long ld;
  int R, N, mirror;
  long split_stride;
  // grouped launches: every workspace pointer moved by o bytes
  IFS_DEV void shift(long o) {
    out = gsh(out, o);
  }
  template <class C>
  IFS_DEV void run(const float *Cs, const TileInfo &t) const {
    using K = Chunks<C>;
    TO *o = out + (long)t.split * split_stride;
#pragma unroll
    for (int k = 0; k < K::N; ++k) {
      int r, c;
      K::row(k, r, c);
      const int gi = t.m0 + r, gj = t.n0 + c;
      float x[VEC];
      cs_row<C>(Cs, r, c, gi < R, N - gj, x);
      st_pack(o + (long)gi * ld + gj, x);
    }
    if (mirror && t.m0 != t.n0) {
#pragma unroll
      for (int k = 0; k < K::N; ++k) {
        int r, c;
        K::col(k, r, c);
        const int gi = t.m0 + r, gj = t.n0 + c;
        float x[VEC];
        cs_col<C>(Cs, r, c, gj < N, R - gi, x);
        st_pack(o + (long)gj * ld + gi, x);
      }
    }
  }
};

// out[gj][gi] = acc (transposed store).
template <typename TO>
struct EpiStoreT {
  TO *out;
  long ld;
  int R, N;
  // grouped launches: every workspace pointer moved by o bytes
  IFS_DEV void shift(long o) {
    out = gsh(out, o);
  }
  template <class C>
  IFS_DEV void run(const float *Cs, const TileInfo &t) const {
    using K = Chunks<C>;
#pragma unroll
    for (int k = 0; k < K::N; ++k) {
      int r, c;
      K::col(k, r, c);
      const int gi = t.m0 + r, gj = t.n0 + c;
      float x[VEC];
      cs_col<C>(Cs, r, c, gj < N, R - gi, x);
      st_pack(out + (long)gj * ld + gi, x);
    }
  }
};

// ---------------------------------------------------------------- NG gram
// W = L^T K~ L on lower tiles.  Writes the natural-gradient middle factor
// X = tril(W) - (I + diag W)/2 transposed (Xt[j][i] = X[i][j], the operand
// layout of L X), and the partial of ||W - I||_F^2 (off-diagonal elements
// count twice).
template <typename T>
struct EpiNgGram {
  T *Xt;
  long ld;
  int M;
  double *part;  // [ntiles]
  // grouped launches: every workspace pointer moved by o bytes
  IFS_DEV void shift(long o) {
    Xt = gsh(Xt, o);
    part = gsh(part, o);
  }
  template <class C>
  IFS_DEV void run(const float *Cs, const TileInfo &t) const {
    using K = Chunks<C>;
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < K::N; ++k) {
      int r, c;
      K::col(k, r, c);
      const int gi0 = t.m0 + r, gj = t.n0 + c;
      float x[VEC];
#pragma unroll
      for (int q = 0; q < VEC; ++q) {
        const int gi = gi0 + q;
        const float w = CS(r + q, c);
        x[q] = 0.f;
        if (gi < M && gj < M) {
          if (gi > gj) {
            x[q] = w;
            s += 2.0 * (double)w * (double)w;
          } else if (gi == gj) {
            x[q] = 0.5f * (w - 1.0f);
            s += ((double)w - 1.0) * ((double)w - 1.0);
          }
        }
      }
      st_pack(Xt + (long)gj * ld + gi0, x);
    }
    s = tile_sum<C>(s, Cs);
    if (threadIdx.x == 0) part[t.ti] = s;
  }
};

// ---------------------------------------------------------------- variance gap
// R = Y V with Y = K~ L and V = L^T K_uf, i.e. K~ T K_uf: per-tile partial sums
// of (K_uf - R)^2 over the valid entries (Prop. 3's gap before the division by
// sigma^2), with K_uf read from its transposed operand copy Kft[n][i].
template <typename T>
struct EpiGap {
  const T *Kft;
  long ldk;
  int M, B;
  double *part;  // [ntiles]
  // grouped launches: every workspace pointer moved by o bytes
  IFS_DEV void shift(long o) {
    Kft = gsh(Kft, o);
    part = gsh(part, o);
  }
  template <class C>
  IFS_DEV void run(const float *Cs, const TileInfo &t) const {
    using K = Chunks<C>;
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < K::N; ++k) {
      int r, c;
      K::col(k, r, c);
      const int gi0 = t.m0 + r, gj = t.n0 + c;
      float kv[VEC];
      ld_pack(Kft + (long)gj * ldk + gi0, kv);
#pragma unroll
      for (int q = 0; q < VEC; ++q) {
        const double d = (double)kv[q] - (double)CS(r + q, c);
        if (gi0 + q < M && gj < B) s += d * d;
      }
    }
    s = tile_sum<C>(s, Cs);
    if (threadIdx.x == 0) part[t.ti] = s;
  }
};

// ---------------------------------------------------------------- NG update
// Lnew = L - gamma * (L X) on lower tiles (strict upper inside diagonal tiles
// written as 0; upper tiles are never touched and stay zero).  Writes the fp32
// master, the operand copy, the operand-type and fp32 transposes, the
// transpose scaled by s~ along k, and, on the last step of a call, the
// caller's L (lower triangle only).  Tile 0 also
// turns the gram partials of this step into the residual ||W - I||_F/sqrt(M).
template <typename T>
struct EpiNgUpdate {
  const float *L;
  float *Ln, *Lnt32;  // Lnt32 aliases LntT when T is float
  T *LnT, *LntT;      // LnT aliases Ln when T is float
  const float *sP;    // s~, zero-padded
  T *LnsT;            // LnsT[j][i] = Lnew[i][j] s~_i
  long ld;
  int M;
  const CallArgs *ca;  // step size gammas[gidx]; the caller's L (leading
                       // dimension M) when write_out; out_resid[step] if given
  int gidx, step, write_out;
  int resid_here;      // form this step's residual here (else a check kernel did)
  const double *gram_part;
  int n_gram;
  double *scal;
  // grouped launches: every workspace pointer moved by o bytes
  IFS_DEV void shift(long o) {
    L = gsh(L, o);
    Ln = gsh(Ln, o);
    Lnt32 = gsh(Lnt32, o);
    LnT = gsh(LnT, o);
    LntT = gsh(LntT, o);
    sP = gsh(sP, o);
    LnsT = gsh(LnsT, o);
    ca = gsh(ca, o);
    gram_part = gsh(gram_part, o);
    scal = gsh(scal, o);
  }
  template <class C>
  IFS_DEV void run(float *Cs, const TileInfo &t) const {
    using K = Chunks<C>;
    const float gamma = ca->gammas[gidx];
    float *Lout = write_out ? ca->L : nullptr;
    float lv[K::N][VEC];
#pragma unroll
    for (int k = 0; k < K::N; ++k) {
      int r, c;
      K::row(k, r, c);
      ld_pack(L + (long)(t.m0 + r) * ld + t.n0 + c, lv[k]);
    }
#pragma unroll
    for (int k = 0; k < K::N; ++k) {
      int r, c;
      K::row(k, r, c);
      const int gi = t.m0 + r, gj0 = t.n0 + c;
      float v[VEC], xs[VEC];
#pragma unroll
      for (int q = 0; q < VEC; ++q) xs[q] = CSV(r, c + q);
#pragma unroll
      for (int q = 0; q < VEC; ++q) pin(xs[q]);
#pragma unroll
      for (int q = 0; q < VEC; ++q) {
        const int gj = gj0 + q;
        v[q] = (gi < M && gj < M && gi >= gj) ? lv[k][q] - gamma * xs[q] : 0.f;
      }
      st_pack(Ln + (long)gi * ld + gj0, v);
      if constexpr (!std::is_same<T, float>::value) st_pack(LnT + (long)gi * ld + gj0, v);
      if (Lout && gi < M) {
#pragma unroll
        for (int q = 0; q < VEC; ++q)
          if (gj0 + q <= gi) Lout[(long)gi * M + gj0 + q] = v[q];
      }
#pragma unroll
      for (int q = 0; q < VEC; ++q) Cs[r * C::LDC + c + q] = v[q];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K::N; ++k) {
      int r, c;
      K::col(k, r, c);
      const int gi0 = t.m0 + r, gj = t.n0 + c;
      float x[VEC];
#pragma unroll
      for (int q = 0; q < VEC; ++q) x[q] = CS(r + q, c);
      st_pack(LntT + (long)gj * ld + gi0, x);
      if constexpr (!std::is_same<T, float>::value) st_pack(Lnt32 + (long)gj * ld + gi0, x);
      float sv[VEC];
      ld_pack(sP + gi0, sv);
#pragma unroll
      for (int q = 0; q < VEC; ++q) x[q] *= sv[q];
      st_pack(LnsT + (long)gj * ld + gi0, x);
    }
    if (t.ti == 0 && resid_here) {
      double s = 0.0;
      for (int i = threadIdx.x; i < n_gram; i += C::NT) s += gram_part[i];
      s = tile_sum<C>(s, Cs);
      if (threadIdx.x == 0) {
        const double r = sqrt(s / M);
        scal[S_RESID] = r;
        if (ca->out_resid) ca->out_resid[step] = r;
      }
    }
  }
};

// ---------------------------------------------------------------- bound gram
// Tile of E = L^T S~ L with W = L^T K~ L already stored (lower tiles) in W.
// Writes Q = 2I - W and Wu = W - E (fp32, symmetric, mirrored), Q in the
// operand type (mirrored), and per-tile partials [tr W, sum Q o Wu, ||W - I||^2].
// Only lower-triangle elements are used; the upper triangle is their mirror.
// Needs one extra staged tile of LDS (BM * LDC floats).
template <typename T>
struct EpiBoundGram {
  const float *W;
  float *Q, *Wu;
  T *QT;
  long ld;
  int M;
  double *part;  // [ntiles][3]
  // grouped launches: every workspace pointer moved by o bytes
  IFS_DEV void shift(long o) {
    W = gsh(W, o);
    Q = gsh(Q, o);
    Wu = gsh(Wu, o);
    QT = gsh(QT, o);
    part = gsh(part, o);
  }
  template <class C>
  IFS_DEV void run(float *Cs, const TileInfo &t) const {
    using K = Chunks<C>;
    float *S2 = Cs + C::BM * C::LDC + 4 * C::NT;  // staged Wu tile
    float wv[K::N][VEC];
#pragma unroll
    for (int k = 0; k < K::N; ++k) {
      int r, c;
      K::row(k, r, c);
      ld_pack(W + (long)(t.m0 + r) * ld + t.n0 + c, wv[k]);
    }
    double trw = 0.0, qwu = 0.0, r2 = 0.0;
#pragma unroll
    for (int k = 0; k < K::N; ++k) {
      int r, c;
      K::row(k, r, c);
      const int gi = t.m0 + r;
      float es[VEC];
#pragma unroll
      for (int q = 0; q < VEC; ++q) es[q] = CSV(r, c + q);
#pragma unroll
      for (int q = 0; q < VEC; ++q) pin(es[q]);
#pragma unroll
      for (int q = 0; q < VEC; ++q) {
        const int gj = t.n0 + c + q;
        const bool in = gi < M && gj < M;
        const float w = wv[k][q];
        const float qv = in ? (gi == gj ? 2.f : 0.f) - w : 0.f;
        const float e = es[q];
        const float wu = in ? w - e : 0.f;
        if (in && gi >= gj) {
          const double mult = gi == gj ? 1.0 : 2.0;
          if (gi == gj) trw += w;
          qwu += mult * (double)qv * (double)wu;
          const double d = (double)w - (gi == gj ? 1.0 : 0.0);
          r2 += mult * d * d;
        }
        Cs[r * C::LDC + c + q] = qv;
        S2[r * C::LDC + c + q] = wu;
      }
    }
    __syncthreads();
    const bool diag = t.m0 == t.n0;
#pragma unroll
    for (int k = 0; k < K::N; ++k) {
      int r, c;
      K::row(k, r, c);
      const int gi = t.m0 + r, gj = t.n0 + c;
      float xq[VEC], xw[VEC];
#pragma unroll
      for (int q = 0; q < VEC; ++q) {
        const bool up = diag && r < c + q;  // upper triangle of a diagonal tile: mirror
        const int rr = up ? c + q : r, cc = up ? r : c + q;
        xq[q] = Cs[rr * C::LDC + cc];
        xw[q] = S2[rr * C::LDC + cc];
      }
      st_pack(Q + (long)gi * ld + gj, xq);
      st_pack(QT + (long)gi * ld + gj, xq);
      st_pack(Wu + (long)gi * ld + gj, xw);
    }
    if (!diag) {
#pragma unroll
      for (int k = 0; k < K::N; ++k) {
        int r, c;
        K::col(k, r, c);
        const int gi0 = t.m0 + r, gj = t.n0 + c;
        float xq[VEC], xw[VEC];
#pragma unroll
        for (int q = 0; q < VEC; ++q) {
          xq[q] = Cs[(r + q) * C::LDC + c];
          xw[q] = S2[(r + q) * C::LDC + c];
        }
        st_pack(Q + (long)gj * ld + gi0, xq);
        st_pack(QT + (long)gj * ld + gi0, xq);
        st_pack(Wu + (long)gj * ld + gi0, xw);
      }
    }
    trw = tile_sum<C>(trw, Cs);
    qwu = tile_sum<C>(qwu, Cs);
    r2 = tile_sum<C>(r2, Cs);
    if (threadIdx.x == 0) {
      part[3 * t.ti + 0] = trw;
      part[3 * t.ti + 1] = qwu;
      part[3 * t.ti + 2] = r2;
    }
  }
};

// ---------------------------------------------------------------- V = L^T K_uf
// V[i][n] and its transpose Vt[n][i] in the operand type.  Columns n >= B of
// the last tile are written as zeros, so padding read by the split-K batch
// product never carries values of an earlier, larger batch.
template <typename T>
struct EpiV {
  T *V, *Vt;
  long ldv, ldt;
  int M, B;
  // grouped launches: every workspace pointer moved by o bytes
  IFS_DEV void shift(long o) {
    V = gsh(V, o);
    Vt = gsh(Vt, o);
  }
  template <class C>
  IFS_DEV void run(const float *Cs, const TileInfo &t) const {
    using K = Chunks<C>;
#pragma unroll
    for (int k = 0; k < K::N; ++k) {
      int r, c;
      K::row(k, r, c);
      const int gi = t.m0 + r, gj = t.n0 + c;
      float x[VEC];
      cs_row<C>(Cs, r, c, gi < M, B - gj, x);
      st_pack(V + (long)gi * ldv + gj, x);
    }
#pragma unroll
    for (int k = 0; k < K::N; ++k) {
      int r, c;
      K::col(k, r, c);
      const int gi = t.m0 + r, gj = t.n0 + c;
      float x[VEC];
      cs_col<C>(Cs, r, c, gj < B, M - gi, x);
      st_pack(Vt + (long)gj * ldt + gi, x);
    }
  }
};

// ---------------------------------------------------------------- U = Q V
// Ut[n][i] = U[i][n], and over the tile's rows the partials of
// sigma^2: sum_i V_in U_in and of the mean mu_n = (K_fu L b)_n = sum_i V_in b_i
// = sum_i U_in a_i (b = Q a with Q symmetric), formed from the U tile so that
// U does not wait for b.
template <typename T>
struct EpiU {
  T *Ut;
  const T *V;
  const float *a;   // L^T m~, zero-padded to Mp
  long ldv, ldt;
  int M, B;
  float *var_part;  // [m-tiles][ldp]
  float *mu_part;   // [m-tiles][ldp]
  long ldp;
  // grouped launches: every workspace pointer moved by o bytes
  IFS_DEV void shift(long o) {
    Ut = gsh(Ut, o);
    V = gsh(V, o);
    a = gsh(a, o);
    var_part = gsh(var_part, o);
    mu_part = gsh(mu_part, o);
  }
  template <class C>
  IFS_DEV void run(float *Cs, const TileInfo &t) const {
    using K = Chunks<C>;
    float vv[K::N][VEC];  // the V tile, loaded before anything waits on it
    float av[K::N];
#pragma unroll
    for (int k = 0; k < K::N; ++k) {
      int r, c;
      K::row(k, r, c);
      ld_pack(V + (long)(t.m0 + r) * ldv + t.n0 + c, vv[k]);
      av[k] = a[t.m0 + r];
    }
#pragma unroll
    for (int k = 0; k < K::N; ++k) {
      int r, c;
      K::col(k, r, c);
      const int gi = t.m0 + r, gj = t.n0 + c;
      float x[VEC];
      cs_col<C>(Cs, r, c, gj < B, M - gi, x);
      st_pack(Ut + (long)gj * ldt + gi, x);
    }
    __syncthreads();
    // V o U in place (V padding is zero), column sums; then diag(a) U the
    // same way (a padding is zero), from registers
    float ua[K::N][VEC];
#pragma unroll
    for (int k = 0; k < K::N; ++k) {
      int r, c;
      K::row(k, r, c);
#pragma unroll
      for (int q = 0; q < VEC; ++q) {
        const float u = CS(r, c + q);
        ua[k][q] = u * av[k];
        Cs[r * C::LDC + c + q] = vv[k][q] * u;
      }
    }
    __syncthreads();
    const int c = threadIdx.x % C::BN, gj = t.n0 + c;
    const long slot = (long)(t.m0 / C::BM) * ldp + gj;
    {
      const float s = tile_colsum<C>(Cs);
      if (threadIdx.x < C::BN && gj < B) var_part[slot] = s;
    }
#pragma unroll
    for (int k = 0; k < K::N; ++k) {
      int r, cc;
      K::row(k, r, cc);
#pragma unroll
      for (int q = 0; q < VEC; ++q) Cs[r * C::LDC + cc + q] = ua[k][q];
    }
    __syncthreads();
    {
      const float s = tile_colsum<C>(Cs);
      if (threadIdx.x < C::BN && gj < B) mu_part[slot] = s;
    }
  }
};

// Staged inputs for the D-wide MFMA reductions: D4 = D rounded up to 4
// columns (the cross term's contraction length), DP = D rounded up to 16 (the
// reduction product's output width), rows of stride DP + 1.
__host__ __device__ inline int d4of(int D) { return (D + 3) & ~3; }
__host__ __device__ inline int dpof(int D) { return (D + 15) / 16 * 16; }

// ---------------------------------------------------------------- backward K_uf side
// Tile of R = L U, taken straight from the accumulators.  Forms
// G_uf = (L b) alpha^T - 2 R diag(beta), recomputes the K_uf tile (norms plus
// an fp32 MFMA cross term, as in the forward), and reduces
// H = G_uf o K_uf to
//   hrow[i]    = sum_n H_in                 (per n-tile partial)
//   hcol[n]    = sum_i H_in                 (per m-tile partial)
//   hx[i][d]   = sum_n H_in Xs_nd           (per n-tile partial)
//   sum H                                   (per tile partial)
// hx comes from an fp32 MFMA product H Xs, the row and column sums from LDS.
// Extra LDS: graduf_extra(BM, BN, D) bytes (the Zs rows' region stays in the
// budget when the tile is generated and Zs is not staged: at one workgroup per
// CU R's launches are shorter beside the main stream's backward chain than at
// two, with the same step time).
__host__ __device__ inline int graduf_extra(int BM, int BN, int D) {
  const int D4 = d4of(D), LDX = dpof(D) + 1;
  return (BM * (D4 + 1) + BN * LDX + 2 * BM + 3 * BN) * 4;
}
//
// KW > 0 (bf16 / fp16 forms): the K_uf tile comes from the set-up's split
// inputs exactly as the forward generates it (KufGen: hi/lo bf16 cross term
// on the matrix cores, accumulator started at the norm terms, one exp2), read
// straight into registers; Zs is then not staged.  KW = 0: norms and an
// fp32-MFMA cross term, or (fp32 form) differences and the accurate exp.
template <int KW>
struct EpiGradUf {
  const float *Lb, *alpha, *beta;
  const float *Zs, *Xs;  // [M][D], [B][D]  (inputs / lengthscales)
  const float *sf2;
  int M, B, D;
  // per-tile partials, fp64 in the fp32 form and fp32 in the others (whose
  // tile reductions run in fp32)
  void *hrow;    // [n-tiles][M]
  void *hcol;    // [m-tiles][ldc]
  long ldc;
  void *hx;      // [n-tiles][M][D]
  double *part;  // [ntiles]
  const void *Zh, *Zl, *Xh, *Xl;  // generator inputs (KW > 0)
  const float *zc, *xr;
  static constexpr bool kRegs = true;  // takes the accumulators in registers
  // grouped launches: every workspace pointer moved by o bytes
  IFS_DEV void shift(long o) {
    Lb = gsh(Lb, o);
    alpha = gsh(alpha, o);
    beta = gsh(beta, o);
    Zs = gsh(Zs, o);
    Xs = gsh(Xs, o);
    sf2 = gsh(sf2, o);
    hrow = gsh(hrow, o);
    hcol = gsh(hcol, o);
    hx = gsh(hx, o);
    part = gsh(part, o);
    Zh = gsh(Zh, o); Zl = gsh(Zl, o); Xh = gsh(Xh, o); Xl = gsh(Xl, o);
    zc = gsh(zc, o); xr = gsh(xr, o);
  }
  // acc: fp32 or (C::A64) fp64 accumulators; the lane's rows are
  // 16 ii + 4 (lane/16) + q for fp32 and 16 ii + 4 q + lane/16 for fp64
  template <class C, class Acc>
  IFS_DEV void run_regs(const Acc (&acc)[C::TM][C::TN], float *Cs, const TileInfo &t) const {
    constexpr int BM = C::BM, BN = C::BN, NT = C::NT;
    const int D4 = d4of(D), DP = dpof(D), LDZ = D4 + 1, LDX = DP + 1;
    float *zs = Cs + BM * C::LDC + 4 * NT;  // [BM][LDZ]
    float *xs = zs + BM * LDZ;              // [BN][LDX]
    float *zn = xs + BN * LDX;              // [BM]
    float *lb = zn + BM;                    // [BM]
    float *xn = lb + BM;                    // [BN]
    float *al = xn + BN;                    // [BN]
    float *be = al + BN;                    // [BN]
    constexpr bool F32 = std::is_same<typename C::T, float>::value;
    constexpr bool GEN = !F32 && KW > 0;
    const int tid = threadIdx.x;
    for (int i = tid; i < BM; i += NT) lb[i] = Lb[t.m0 + i];    // padded to Mp
    for (int i = tid; i < BN; i += NT) {
      al[i] = alpha[t.n0 + i];                                   // padded to Bp
      be[i] = beta[t.n0 + i];
    }
    if constexpr (!GEN) stage_rows<NT>(zs, LDZ, Zs, t.m0, BM, M, D, -1);
    stage_rows<NT>(xs, LDX, Xs, t.n0, BN, B, D, -1);
    __syncthreads();
    if constexpr (!GEN) {
      for (int i = tid; i < BM + BN; i += NT) {
        const float *row = i < BM ? zs + i * LDZ : xs + (i - BM) * LDX;
        float s = 0.f;
        for (int d = 0; d < D4; ++d) s = fmaf(row[d], row[d], s);
        (i < BM ? zn : xn)[i < BM ? i : i - BM] = s;
      }
      __syncthreads();
    }
    const float s2f = *sf2;
    double hs = 0.0;
    {
      // wave (wm, wn) owns the WM x WN sub-block it accumulated in the product;
      // the cross term lands in the accumulators' lane layout
      const int lane = tid & 63, wave = tid >> 6, l16 = lane & 15, l4 = lane >> 4;
      const int ib = (wave / C::WGN) * C::WM, jb = (wave % C::WGN) * C::WN;
      // this lane's rows (16 ii + r(q)) and columns (16 jj + l16): their
      // staged values in registers, read once and unconditionally
      auto r_of = [&](int q) { return C::A64 ? 4 * q + l4 : 4 * l4 + q; };
      float zr[C::TM][4], lr[C::TM][4], xc[C::TN], ac[C::TN], bc[C::TN];
      bool rok[C::TM][4], cok[C::TN];
#pragma unroll
      for (int ii = 0; ii < C::TM; ++ii)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int i = ib + 16 * ii + r_of(q);
          zr[ii][q] = GEN ? 0.f : zn[i];
          lr[ii][q] = lb[i];
          rok[ii][q] = t.m0 + i < M;
        }
#pragma unroll
      for (int jj = 0; jj < C::TN; ++jj) {
        const int n = jb + 16 * jj + l16;
        xc[jj] = GEN ? 0.f : xn[n];
        ac[jj] = al[n];
        bc[jj] = be[n];
        cok[jj] = t.n0 + n < B;
      }
#pragma unroll
      for (int ii = 0; ii < C::TM; ++ii)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          pin(zr[ii][q]);
          pin(lr[ii][q]);
        }
#pragma unroll
      for (int jj = 0; jj < C::TN; ++jj) {
        pin(xc[jj]);
        pin(ac[jj]);
        pin(bc[jj]);
      }
      // the fp32 form recomputes K_uf from differences with the accurate exp
      // (as its forward does); the others as their forward generates it
      f32x4 c[C::TM][C::TN];
      if constexpr (GEN) {
        using KO = KufOp<(KW > 0 ? KW : 16)>;
        using Op = typename KO::type;
        constexpr int NC = KO::NC, RW = 4 * NC;
        const Op *zh = (const Op *)Zh, *zl = (const Op *)Zl;
        const Op *xh = (const Op *)Xh, *xl = (const Op *)Xl;
#pragma unroll
        for (int ii = 0; ii < C::TM; ++ii) {
          const f32x4 zcv = *(const f32x4 *)(zc + t.m0 + ib + 16 * ii + 4 * l4);
#pragma unroll
          for (int jj = 0; jj < C::TN; ++jj) {
            const float xrv = xr[t.n0 + jb + 16 * jj + l16];
#pragma unroll
            for (int q = 0; q < 4; ++q) c[ii][jj][q] = zcv[q] + xrv;
          }
        }
#pragma unroll
        for (int cc = 0; cc < NC; ++cc) {
          Op a_h[C::TM], a_l[C::TM], b_h[C::TN], b_l[C::TN];
#pragma unroll
          for (int ii = 0; ii < C::TM; ++ii) {
            const long r = (long)(t.m0 + ib + 16 * ii + l16) * RW + 4 * cc + l4;
            a_h[ii] = zh[r];
            a_l[ii] = zl[r];
          }
#pragma unroll
          for (int jj = 0; jj < C::TN; ++jj) {
            const long r = (long)(t.n0 + jb + 16 * jj + l16) * RW + 4 * cc + l4;
            b_h[jj] = xh[r];
            b_l[jj] = xl[r];
          }
#pragma unroll
          for (int ii = 0; ii < C::TM; ++ii)
#pragma unroll
            for (int jj = 0; jj < C::TN; ++jj) {
              c[ii][jj] = KO::mma(a_h[ii], b_h[jj], c[ii][jj]);
              c[ii][jj] = KO::mma(a_h[ii], b_l[jj], c[ii][jj]);
              c[ii][jj] = KO::mma(a_l[ii], b_h[jj], c[ii][jj]);
            }
        }
      } else if constexpr (!F32) {
        cross_block<C::TM, C::TN, C::A64>(zs + ib * LDZ, LDZ, xs + jb * LDX, LDX, D4, c);
      }
#pragma unroll
      for (int ii = 0; ii < C::TM; ++ii)
#pragma unroll
        for (int jj = 0; jj < C::TN; ++jj) {
          const int n = jb + 16 * jj + l16;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int i = ib + 16 * ii + r_of(q);
            float kuf;
            if constexpr (F32)
              kuf = s2f * kexp<true>(-0.5f * sqdist(zs + i * LDZ, xs + n * LDX, D));
            else if constexpr (GEN)
              kuf = __builtin_amdgcn_exp2f(c[ii][jj][q]);
            else
              kuf = kern_se(s2f, zr[ii][q], xc[jj], c[ii][jj][q]);
            const float g = lr[ii][q] * ac[jj] - 2.f * (float)acc[ii][jj][q] * bc[jj];
            const float h = (rok[ii][q] && cok[jj]) ? g * kuf : 0.f;
            hs += h;
            Cs[i * C::LDC + n] = h;
          }
        }
    }
    __syncthreads();
    hs = tile_sum<C>(hs, Cs);
    if (tid == 0) part[t.ti] = hs;
    const int nti = t.n0 / BN, mti = t.m0 / BM;
    // the fp32 form sums on the fp64 matrix cores (the gradient's sums of
    // these partials cancel) and keeps fp64 partials; the others sum in fp32
    // (H Xs from split-bf16 products) and keep fp32 partials
    constexpr bool F64 = std::is_same<typename C::T, float>::value;
    using P = typename std::conditional<F64, double, float>::type;
    {
      const double s = tile_colsum<C, double>(Cs);
      const int cl = tid % BN, gj = t.n0 + cl;
      if (tid < BN && gj < B) ((P *)hcol)[(long)mti * ldc + gj] = (P)s;
    }
    {
      const double s = tile_rowsum<C, double>(Cs);
      const int gi = t.m0 + tid % BM;
      if (tid < BM && gi < M) ((P *)hrow)[(long)nti * M + gi] = (P)s;
    }
    const int D_ = D, M_ = M;
    P *hx_ = (P *)hx + (long)nti * M * D;
    auto sink = [&](int i, int d, double v) {
      const int gi = t.m0 + i;
      if (gi < M_ && d < D_) hx_[(long)gi * D_ + d] = (P)v;
    };
    if constexpr (F64)
      lds_mfma<NT / 64, BM / (NT / 4), false, true>(Cs, C::LDC, BN, xs, LDX, DP, sink);
    else
      lds_mfma_split<BM / (NT / 4)>(Cs, C::LDC, BN, xs, LDX, DP, sink);
  }
};

// ---------------------------------------------------------------- backward K_uu side
// Tile (I >= J) of G_uu = Y2 L^T.  H = G_uu o K_uu with K_uu = K~ - diag(s~).
// For rows of block I (slot J): hz[i][d] = sum_j H_ij Zs_jd and hzrow[i] = sum_j H_ij;
// for an off-diagonal tile also rows of block J (slot I) through H^T.  The
// products with Zs run on fp32 MFMA; the row / column sums come from LDS.
// P: the partials' type, which the form sets (not the product's operand
// type: the fp16 form runs this product with fp32 operands): fp64 partials
// and fp64-MFMA reductions in the fp32 form, fp32 in the others.
// Extra LDS: 2 * BM * (DP + 1) floats (DP: dpof).
template <typename P>
struct EpiGradUu {
  const float *Kt, *s, *Zs;
  long ld;
  int M, D;
  void *hz;       // [nb][M][D]  (fp64 in the fp32 form, else fp32)
  void *hzrow;    // [nb][M]
  double *part;  // [ntiles]
  float *gdiag;  // [M]: diagonal of G_uu from the diagonal tiles, or null
  // grouped launches: every workspace pointer moved by o bytes
  IFS_DEV void shift(long o) {
    Kt = gsh(Kt, o);
    s = gsh(s, o);
    Zs = gsh(Zs, o);
    hz = gsh(hz, o);
    hzrow = gsh(hzrow, o);
    part = gsh(part, o);
    gdiag = gsh(gdiag, o);
  }
  template <class C>
  IFS_DEV void run(float *Cs, const TileInfo &t) const {
    using K = Chunks<C>;
    constexpr int BM = C::BM, BN = C::BN, NT = C::NT;
    static_assert(BM == BN, "symmetric tiles");
    const int DP = dpof(D), LDZ = DP + 1, LDC_ = C::LDC;
    float *zi = Cs + BM * C::LDC + 4 * NT;  // rows of block I  [BM][LDZ]
    float *zj = zi + BM * LDZ;              // rows of block J  [BN][LDZ]
    float kv[K::N][VEC];
#pragma unroll
    for (int k = 0; k < K::N; ++k) {
      int r, c;
      K::row(k, r, c);
      ld_pack(Kt + (long)(t.m0 + r) * ld + t.n0 + c, kv[k]);
    }
    float sv[K::N];
#pragma unroll
    for (int k = 0; k < K::N; ++k) {
      int r, c;
      K::row(k, r, c);
      sv[k] = ld_or0(s, t.m0 + r, t.m0 + r < M);
    }
    stage_rows<NT>(zi, LDZ, Zs, t.m0, BM, M, D, -1);
    stage_rows<NT>(zj, LDZ, Zs, t.n0, BN, M, D, -1);
    double hs = 0.0;
    const bool off = t.m0 != t.n0;
#pragma unroll
    for (int k = 0; k < K::N; ++k) {
      int r, c;
      K::row(k, r, c);
      const int gi = t.m0 + r;
#pragma unroll
      for (int q = 0; q < VEC; ++q) {
        const int gj = t.n0 + c + q;
        float h = 0.f;
        if (gi < M && gj < M) {
          const float kk = kv[k][q] - (gi == gj ? sv[k] : 0.f);
          if (gdiag && gi == gj) gdiag[gi] = CS(r, c + q);
          h = CS(r, c + q) * kk;
          hs += (off ? 2.0 : 1.0) * h;
        }
        Cs[r * C::LDC + c + q] = h;
      }
    }
    __syncthreads();
    hs = tile_sum<C>(hs, Cs);
    if (threadIdx.x == 0) part[t.ti] = hs;
    const int I = t.m0 / BM, J = t.n0 / BN, D_ = D, M_ = M;
    constexpr bool F64 = std::is_same<P, double>::value;
    {
      // rows of block I (slot J): row sums and H Zs_J
      const double rs = tile_rowsum<C, double>(Cs);
      const int gi = t.m0 + threadIdx.x % BM;
      if (threadIdx.x < BM && gi < M) ((P *)hzrow)[(long)J * M + gi] = (P)rs;
      P *hz_ = (P *)hz + (long)J * M * D;
      const int base = t.m0;
      lds_mfma<NT / 64, BM / (NT / 4), false, F64>(Cs, LDC_, BN, zj, LDZ, DP,
                                                   [&](int i, int d, double v) {
        const int g = base + i;
        if (g < M_ && d < D_) hz_[(long)g * D_ + d] = (P)v;
      });
    }
    if (!off) return;
    {
      // rows of block J (slot I) through H^T: column sums and H^T Zs_I
      const double cs = tile_colsum<C, double>(Cs);
      const int gj = t.n0 + threadIdx.x % BN;
      if (threadIdx.x < BN && gj < M) ((P *)hzrow)[(long)I * M + gj] = (P)cs;
      P *hz_ = (P *)hz + (long)I * M * D;
      const int base = t.n0;
      lds_mfma<NT / 64, BN / (NT / 4), true, F64>(Cs, LDC_, BM, zi, LDZ, DP,
                                                  [&](int i, int d, double v) {
        const int g = base + i;
        if (g < M_ && d < D_) hz_[(long)g * D_ + d] = (P)v;
      });
    }
  }
};

// ---------------------------------------------------------------- diag(L Q L^T)
// Tile (I >= J) of L Q.  part[J][i] = sum_{j in tile} (L Q)_ij L_ij, the
// tile's share of diag(L Q L^T) = diag(P); tiles with J > I would only meet
// L_ij = 0.  Used by the gradient with respect to s~.
struct EpiRowDotL {
  const float *L;  // fp32 master [Mp][Mp]
  long ld;
  int M;
  float *part;     // [nb][ldp]
  long ldp;
  // grouped launches: every workspace pointer moved by o bytes
  IFS_DEV void shift(long o) {
    L = gsh(L, o);
    part = gsh(part, o);
  }
  template <class C>
  IFS_DEV void run(float *Cs, const TileInfo &t) const {
    using K = Chunks<C>;
    float lv[K::N][VEC];
#pragma unroll
    for (int k = 0; k < K::N; ++k) {
      int r, c;
      K::row(k, r, c);
      ld_pack(L + (long)(t.m0 + r) * ld + t.n0 + c, lv[k]);
    }
#pragma unroll
    for (int k = 0; k < K::N; ++k) {
      int r, c;
      K::row(k, r, c);
#pragma unroll
      for (int q = 0; q < VEC; ++q) Cs[r * C::LDC + c + q] = CS(r, c + q) * lv[k][q];
    }
    __syncthreads();
    for (int r = threadIdx.x; r < C::BM; r += C::NT) {
      const int gi = t.m0 + r;
      float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
      for (int c = 0; c < C::BN; c += 4) {
        a0 += CS(r, c);
        a1 += CS(r, c + 1);
        a2 += CS(r, c + 2);
        a3 += CS(r, c + 3);
      }
      if (gi < M) part[(long)(t.n0 / C::BN) * ldp + gi] = (a0 + a1) + (a2 + a3);
    }
  }
};
