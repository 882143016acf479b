// GEMM epilogues of the inverse-free SVGP iteration.  Each runs with the whole
// workgroup after the fp32 accumulator tile Cs[BM][LDC] has been staged in LDS;
// 16*NT bytes of scratch LDS follow the tile, then any epilogue-specific LDS.
// Outputs are written in the layout their consumer's NT product reads:
// "T" suffixes below mark transposed stores (out[j][i] = C[i][j]).
#pragma once
#include "gemm.hpp"

// Row-major element loop over the tile (coalesced along columns).
#define TILE_LOOP(C, r, c)                                                    \
  for (int _i = threadIdx.x; _i < C::BM * C::BN; _i += C::NT)                 \
    if (const int r = _i / C::BN, c = _i % C::BN; true)

// Column-major element loop (coalesced along rows, for transposed stores).
#define TILE_LOOP_T(C, r, c)                                                  \
  for (int _i = threadIdx.x; _i < C::BM * C::BN; _i += C::NT)                 \
    if (const int c = _i / C::BM, r = _i % C::BM; true)

#define CS(r, c) Cs[(r) * C::LDC + (c)]

// Sum of one double per thread over the workgroup, result in thread 0.
template <class C>
IFS_DEV double tile_sum(double v, const float *Cs) {
  double *sh = (double *)(Cs + C::BM * C::LDC);
  return block_sum<C::NT>(v, sh);
}

// ---------------------------------------------------------------- plain stores
// out[gi][gj] = acc for rows < R, cols < N; optional transposed mirror for
// off-diagonal tiles of a symmetric lower-tile schedule; split-K piece s
// writes to out + s * split_stride.
template <typename TO>
struct EpiStore {
  TO *out;
  long ld;
  int R, N, mirror;
  long split_stride;
  template <class C>
  IFS_DEV void run(const float *Cs, const TileInfo &t) const {
    TO *o = out + (long)t.split * split_stride;
    TILE_LOOP(C, r, c) {
      const int gi = t.m0 + r, gj = t.n0 + c;
      if (gi < R && gj < N) o[(long)gi * ld + gj] = from_f32<TO>(CS(r, c));
    }
    if (mirror && t.m0 != t.n0) {
      TILE_LOOP_T(C, r, c) {
        const int gi = t.m0 + r, gj = t.n0 + c;
        if (gi < R && gj < N) o[(long)gj * ld + gi] = from_f32<TO>(CS(r, c));
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
  template <class C>
  IFS_DEV void run(const float *Cs, const TileInfo &t) const {
    TILE_LOOP_T(C, r, c) {
      const int gi = t.m0 + r, gj = t.n0 + c;
      if (gi < R && gj < N) out[(long)gj * ld + gi] = from_f32<TO>(CS(r, c));
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
  template <class C>
  IFS_DEV void run(const float *Cs, const TileInfo &t) const {
    double s = 0.0;
    TILE_LOOP_T(C, r, c) {
      const int gi = t.m0 + r, gj = t.n0 + c;
      if (gi < M && gj < M) {
        const float w = CS(r, c);
        float x = 0.f;
        if (gi > gj) {
          x = w;
          s += 2.0 * (double)w * (double)w;
        } else if (gi == gj) {
          x = 0.5f * (w - 1.0f);
          s += ((double)w - 1.0) * ((double)w - 1.0);
        }
        Xt[(long)gj * ld + gi] = from_f32<T>(x);
      }
    }
    s = tile_sum<C>(s, Cs);
    if (threadIdx.x == 0) part[t.ti] = s;
  }
};

// ---------------------------------------------------------------- NG update
// Lnew = L - gamma * (L X) on lower tiles (strict upper inside diagonal tiles
// written as 0; upper tiles are never touched and stay zero).  Writes the fp32
// master, the operand copy, the operand-type and fp32 transposes, and, on the
// last step of a call, the caller's L (lower triangle only).  Tile 0 also
// turns the gram partials of this step into the residual ||W - I||_F/sqrt(M).
template <typename T>
struct EpiNgUpdate {
  const float *L;
  float *Ln, *Lnt32;  // Lnt32 aliases LntT when T is float
  T *LnT, *LntT;      // LnT aliases Ln when T is float
  long ld;
  int M;
  float gamma;
  float *Lout;        // caller's L (leading dimension M) or null
  const double *gram_part;
  int n_gram;
  double *resid_out, *scal;
  template <class C>
  IFS_DEV void run(float *Cs, const TileInfo &t) const {
    TILE_LOOP(C, r, c) {
      const int gi = t.m0 + r, gj = t.n0 + c;
      float v = 0.f;
      if (gi < M && gj < M) {
        v = gi >= gj ? L[(long)gi * ld + gj] - gamma * CS(r, c) : 0.f;
        Ln[(long)gi * ld + gj] = v;
        if constexpr (!std::is_same<T, float>::value) LnT[(long)gi * ld + gj] = from_f32<T>(v);
        if (Lout && gi >= gj) Lout[(long)gi * M + gj] = v;
      }
      Cs[r * C::LDC + c] = v;
    }
    __syncthreads();
    TILE_LOOP_T(C, r, c) {
      const int gi = t.m0 + r, gj = t.n0 + c;
      if (gi < M && gj < M) {
        const float v = CS(r, c);
        LntT[(long)gj * ld + gi] = from_f32<T>(v);
        if constexpr (!std::is_same<T, float>::value) Lnt32[(long)gj * ld + gi] = v;
      }
    }
    if (t.ti == 0) {
      double s = 0.0;
      for (int i = threadIdx.x; i < n_gram; i += C::NT) s += gram_part[i];
      s = tile_sum<C>(s, Cs);
      if (threadIdx.x == 0) {
        const double r = sqrt(s / M);
        scal[S_RESID] = r;
        if (resid_out) *resid_out = r;
      }
    }
  }
};

// ---------------------------------------------------------------- bound gram
// Tile of E = L^T S~ L with W = L^T K~ L already stored (lower tiles) in W.
// Writes Q = 2I - W and Wu = W - E (fp32, symmetric, mirrored), Q in the
// operand type (mirrored), and per-tile partials [tr W, sum Q o Wu, ||W - I||^2].
template <typename T>
struct EpiBoundGram {
  const float *W;
  float *Q, *Wu;
  T *QT;
  long ld;
  int M;
  double *part;  // [ntiles][3]
  template <class C>
  IFS_DEV void run(const float *Cs, const TileInfo &t) const {
    double trw = 0.0, qwu = 0.0, r2 = 0.0;
    TILE_LOOP(C, r, c) {
      const int gi = t.m0 + r, gj = t.n0 + c;
      if (gi < M && gj < M && gi >= gj) {
        const float w = W[(long)gi * ld + gj];
        const float e = CS(r, c);
        const float q = (gi == gj ? 2.f : 0.f) - w;
        const float wu = w - e;
        Q[(long)gi * ld + gj] = q;
        QT[(long)gi * ld + gj] = from_f32<T>(q);
        Wu[(long)gi * ld + gj] = wu;
        const double mult = gi == gj ? 1.0 : 2.0;
        if (gi == gj) trw += w;
        qwu += mult * (double)q * (double)wu;
        const double d = (double)w - (gi == gj ? 1.0 : 0.0);
        r2 += mult * d * d;
      }
    }
    TILE_LOOP_T(C, r, c) {
      const int gi = t.m0 + r, gj = t.n0 + c;
      if (gi < M && gj < M && gi > gj) {
        const float w = W[(long)gi * ld + gj];
        Q[(long)gj * ld + gi] = -w;
        QT[(long)gj * ld + gi] = from_f32<T>(-w);
        Wu[(long)gj * ld + gi] = w - CS(r, c);
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
  template <class C>
  IFS_DEV void run(const float *Cs, const TileInfo &t) const {
    TILE_LOOP(C, r, c) {
      const int gi = t.m0 + r, gj = t.n0 + c;
      if (gi < M) V[(long)gi * ldv + gj] = from_f32<T>(gj < B ? CS(r, c) : 0.f);
    }
    TILE_LOOP_T(C, r, c) {
      const int gi = t.m0 + r, gj = t.n0 + c;
      if (gi < M) Vt[(long)gj * ldt + gi] = from_f32<T>(gj < B ? CS(r, c) : 0.f);
    }
  }
};

// ---------------------------------------------------------------- U = Q V
// Ut[n][i] = U[i][n] and the partial sum_i V_in U_in over the tile's rows.
template <typename T>
struct EpiU {
  T *Ut;
  const T *V;
  long ldv, ldt;
  int M, B;
  float *var_part;  // [m-tiles][ldp]
  long ldp;
  template <class C>
  IFS_DEV void run(float *Cs, const TileInfo &t) const {
    TILE_LOOP_T(C, r, c) {
      const int gi = t.m0 + r, gj = t.n0 + c;
      if (gi < M && gj < B) Ut[(long)gj * ldt + gi] = from_f32<T>(CS(r, c));
    }
    __syncthreads();
    // V o U in place (independent, coalesced loads of the V tile), then column sums in LDS
    TILE_LOOP(C, r, c) {
      const int gi = t.m0 + r, gj = t.n0 + c;
      const float v = (gi < M && gj < B) ? to_f32(V[(long)gi * ldv + gj]) : 0.f;
      Cs[r * C::LDC + c] = v * CS(r, c);
    }
    __syncthreads();
    float *sh = Cs + C::BM * C::LDC;
    constexpr int RG = C::NT / C::BN;  // row groups per column
    static_assert(C::NT % C::BN == 0, "column partial layout");
    const int c = threadIdx.x % C::BN, g = threadIdx.x / C::BN;
    const int gj = t.n0 + c;
    float s = 0.f;
    for (int r = g; r < C::BM; r += RG) s += CS(r, c);
    sh[threadIdx.x] = s;
    __syncthreads();
    if (g == 0 && gj < B) {
      for (int k = 1; k < RG; ++k) s += sh[k * C::BN + c];
      var_part[(long)(t.m0 / C::BM) * ldp + gj] = s;
    }
  }
};

// ---------------------------------------------------------------- backward K_uf side
// Tile of R = L U.  Forms G_uf = (L b) alpha^T - 2 R diag(beta), recomputes the
// K_uf tile from the scaled inputs staged in LDS, and reduces H = G_uf o K_uf to
//   hrow[i]    = sum_n H_in                 (per n-tile partial)
//   hcol[n]    = sum_i H_in                 (per m-tile partial)
//   hx[i][d]   = sum_n H_in Xs_nd           (per n-tile partial)
//   sum H                                   (per tile partial)
struct EpiGradUf {
  const float *Lb, *alpha, *beta;
  const float *Zs, *Xs;  // [M][D], [B][D]  (inputs / lengthscales)
  const float *sf2;
  int M, B, D;
  float *hrow;  // [n-tiles][M]
  float *hcol;  // [m-tiles][ldc]
  long ldc;
  float *hx;    // [n-tiles][M][D]
  double *part; // [ntiles]
  template <class C>
  IFS_DEV void run(float *Cs, const TileInfo &t) const {
    constexpr int BM = C::BM, BN = C::BN, NT = C::NT;
    const int D4 = (D + 3) & ~3;
    float *zs = Cs + BM * C::LDC + 4 * NT;  // [BM][D4]
    float *xs = zs + BM * D4;               // [BN][D4]
    for (int i = threadIdx.x; i < BM * D4; i += NT) {
      const int r = i / D4, d = i % D4, gi = t.m0 + r;
      zs[i] = (gi < M && d < D) ? Zs[(long)gi * D + d] : 0.f;
    }
    for (int i = threadIdx.x; i < BN * D4; i += NT) {
      const int c = i / D4, d = i % D4, gj = t.n0 + c;
      xs[i] = (gj < B && d < D) ? Xs[(long)gj * D + d] : 0.f;
    }
    __syncthreads();
    const float s2f = *sf2;
    double hs = 0.0;
    TILE_LOOP(C, r, c) {
      const int gi = t.m0 + r, gj = t.n0 + c;
      float h = 0.f;
      if (gi < M && gj < B) {
        float d2 = 0.f;
        for (int d = 0; d < D; ++d) {
          const float df = zs[r * D4 + d] - xs[c * D4 + d];
          d2 = fmaf(df, df, d2);
        }
        const float kuf = s2f * __expf(-0.5f * d2);
        const float g = Lb[gi] * alpha[gj] - 2.f * CS(r, c) * beta[gj];
        h = g * kuf;
        hs += h;
      }
      Cs[r * C::LDC + c] = h;
    }
    __syncthreads();
    hs = tile_sum<C>(hs, Cs);
    if (threadIdx.x == 0) part[t.ti] = hs;
    const int nti = t.n0 / BN, mti = t.m0 / BM;
    for (int c = threadIdx.x; c < BN; c += NT) {
      const int gj = t.n0 + c;
      if (gj < B) {
        float s = 0.f;
        for (int r = 0; r < BM; ++r) s += CS(r, c);
        hcol[(long)mti * ldc + gj] = s;
      }
    }
    for (int r = threadIdx.x; r < BM; r += NT) {
      const int gi = t.m0 + r;
      if (gi < M) {
        float s = 0.f;
        for (int c = 0; c < BN; ++c) s += CS(r, c);
        hrow[(long)nti * M + gi] = s;
      }
    }
    // hx = H Xs over the tile's columns, 4 x 4 register blocks of (r, d)
    const int nd4 = D4 / 4;
    for (int b = threadIdx.x; b < (BM / 4) * nd4; b += NT) {
      const int r4 = (b / nd4) * 4, d4 = (b % nd4) * 4;
      float a[4][4] = {};
      for (int c = 0; c < BN; ++c) {
        float hv[4], xv[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) hv[i] = CS(r4 + i, c);
#pragma unroll
        for (int j = 0; j < 4; ++j) xv[j] = xs[c * D4 + d4 + j];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) a[i][j] = fmaf(hv[i], xv[j], a[i][j]);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int gi = t.m0 + r4 + i;
        if (gi < M)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            if (d4 + j < D) hx[((long)nti * M + gi) * D + d4 + j] = a[i][j];
      }
    }
  }
};

// ---------------------------------------------------------------- backward K_uu side
// Tile (I >= J) of G_uu = Y2 L^T.  H = G_uu o K_uu with K_uu = K~ - diag(s~).
// For rows of block I (slot J): hz[i][d] = sum_j H_ij Zs_jd and hzrow[i] = sum_j H_ij;
// for an off-diagonal tile also rows of block J (slot I) through H^T.
struct EpiGradUu {
  const float *Kt, *s, *Zs;
  long ld;
  int M, D;
  float *hz;     // [nb][M][D]
  float *hzrow;  // [nb][M]
  double *part;  // [ntiles]
  template <class C>
  IFS_DEV void run(float *Cs, const TileInfo &t) const {
    constexpr int BM = C::BM, BN = C::BN, NT = C::NT;
    static_assert(BM == BN, "symmetric tiles");
    const int D4 = (D + 3) & ~3;
    float *zi = Cs + BM * C::LDC + 4 * NT;  // rows of block I  [BM][D4]
    float *zj = zi + BM * D4;               // rows of block J  [BN][D4]
    for (int i = threadIdx.x; i < BM * D4; i += NT) {
      const int r = i / D4, d = i % D4;
      const int gi = t.m0 + r, gj = t.n0 + r;
      zi[i] = (gi < M && d < D) ? Zs[(long)gi * D + d] : 0.f;
      zj[i] = (gj < M && d < D) ? Zs[(long)gj * D + d] : 0.f;
    }
    double hs = 0.0;
    const bool off = t.m0 != t.n0;
    TILE_LOOP(C, r, c) {
      const int gi = t.m0 + r, gj = t.n0 + c;
      float h = 0.f;
      if (gi < M && gj < M) {
        const float k = Kt[(long)gi * ld + gj] - (gi == gj ? s[gi] : 0.f);
        h = CS(r, c) * k;
        hs += (off ? 2.0 : 1.0) * h;
      }
      Cs[r * C::LDC + c] = h;
    }
    __syncthreads();
    hs = tile_sum<C>(hs, Cs);
    if (threadIdx.x == 0) part[t.ti] = hs;
    const int I = t.m0 / BM, J = t.n0 / BN;
    const int nd4 = D4 / 4;
    for (int r = threadIdx.x; r < BM; r += NT) {
      const int gi = t.m0 + r;
      if (gi < M) {
        float s_ = 0.f;
        for (int c = 0; c < BN; ++c) s_ += CS(r, c);
        hzrow[(long)J * M + gi] = s_;
      }
    }
    for (int b = threadIdx.x; b < (BM / 4) * nd4; b += NT) {
      const int r4 = (b / nd4) * 4, d4 = (b % nd4) * 4;
      float a[4][4] = {};
      for (int c = 0; c < BN; ++c) {
        float hv[4], zv[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) hv[i] = CS(r4 + i, c);
#pragma unroll
        for (int j = 0; j < 4; ++j) zv[j] = zj[c * D4 + d4 + j];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) a[i][j] = fmaf(hv[i], zv[j], a[i][j]);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int gi = t.m0 + r4 + i;
        if (gi < M)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            if (d4 + j < D) hz[((long)J * M + gi) * D + d4 + j] = a[i][j];
      }
    }
    if (!off) return;
    for (int c = threadIdx.x; c < BN; c += NT) {
      const int gj = t.n0 + c;
      if (gj < M) {
        float s_ = 0.f;
        for (int r = 0; r < BM; ++r) s_ += CS(r, c);
        hzrow[(long)I * M + gj] = s_;
      }
    }
    for (int b = threadIdx.x; b < (BN / 4) * nd4; b += NT) {
      const int c4 = (b / nd4) * 4, d4 = (b % nd4) * 4;
      float a[4][4] = {};
      for (int r = 0; r < BM; ++r) {
        float hv[4], zv[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) hv[i] = CS(r, c4 + i);
#pragma unroll
        for (int j = 0; j < 4; ++j) zv[j] = zi[r * D4 + d4 + j];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) a[i][j] = fmaf(hv[i], zv[j], a[i][j]);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int gj = t.n0 + c4 + i;
        if (gj < M)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            if (d4 + j < D) hz[((long)I * M + gj) * D + d4 + j] = a[i][j];
      }
    }
  }
};
