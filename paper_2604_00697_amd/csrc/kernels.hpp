// Non-GEMM kernels of the iteration: input scaling, kernel-matrix generation,
// matrix-vector products, likelihood expectations, fp64 finalisation.
#pragma once
#include "common.hpp"

#define NTB 256  // threads per block of the elementwise kernels

// Scalar slots of the context's fp64 buffer.
enum : int {
  S_SUMLOGS = 0,   // sum_i log s~_i
  S_LOGDET = 1,    // log|T| = 2 sum log|L_ii|
  S_QUAD = 2,      // b^T Wu b   (= m~^T P K_uu P m~)
  S_RESID = 3,     // residual of the last NG step
  S_NSLOT = 8
};

// ---------------------------------------------------------------- validation
// Domain checks, 1/ell and sum log s~ (one block).
__global__ void k_prep(const float *ell, const float *sf2, const float *noise, const float *s,
                       int M, int D, int need_noise, float *inv_ell, double *scal, int *flag) {
  __shared__ double sh[NTB / 64];
  int bad = 0;
  for (int d = threadIdx.x; d < D; d += NTB) {
    const float l = ell[d];
    if (!(l > 0.f) || !isfinite(l)) bad = 1;
    inv_ell[d] = 1.0f / l;
  }
  if (threadIdx.x == 0) {
    const float v = *sf2;
    if (!(v > 0.f) || !isfinite(v)) bad = 1;
    if (need_noise) {
      const float n = *noise;
      if (!(n > 0.f) || !isfinite(n)) bad = 1;
    }
  }
  double acc = 0.0;
  for (int i = threadIdx.x; i < M; i += NTB) {
    const float v = s[i];
    if (!(v > 0.f) || !isfinite(v)) bad = 1;
    acc += log((double)v);
  }
  acc = block_sum<NTB>(acc, sh);
  if (threadIdx.x == 0) scal[S_SUMLOGS] = acc;
  if (bad) atomicOr(flag, FLAG_DOMAIN);
}

// out[i][d] = A[i][d] / ell_d
__global__ void k_scale_rows(const float *A, int R, int D, const float *inv_ell, float *out) {
  const long n = (long)R * D;
  for (long i = blockIdx.x * (long)NTB + threadIdx.x; i < n; i += (long)gridDim.x * NTB)
    out[i] = A[i] * inv_ell[i % D];
}

// ---------------------------------------------------------------- kernel matrices
// K~[i][j] = sf2 exp(-1/2 |zs_i - zs_j|^2) + delta_ij s~_i, full square matrix.
// 16 x 16 threads per block, each block a 16 x 16 tile; scaled rows in LDS.
template <int MAXD>
__global__ void k_kuu(const float *Zs, int M, int D, const float *sf2, const float *s,
                      float *Kt, long ld) {
  __shared__ float zi[16][MAXD + 1], zj[16][MAXD + 1];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int i0 = blockIdx.y * 16, j0 = blockIdx.x * 16;
  for (int e = threadIdx.x; e < 16 * D; e += NTB) {
    const int r = e / D, d = e % D;
    zi[r][d] = (i0 + r < M) ? Zs[(long)(i0 + r) * D + d] : 0.f;
    zj[r][d] = (j0 + r < M) ? Zs[(long)(j0 + r) * D + d] : 0.f;
  }
  __syncthreads();
  const int i = i0 + ty, j = j0 + tx;
  if (i < M && j < M) {
    float d2 = 0.f;
    for (int d = 0; d < D; ++d) {
      const float df = zi[ty][d] - zj[tx][d];
      d2 = fmaf(df, df, d2);
    }
    float v = (*sf2) * __expf(-0.5f * d2);
    if (i == j) v += s[i];
    Kt[(long)i * ld + j] = v;
  }
}

// K_uf[k][n] = sf2 exp(-1/2 |zs_k - xs_n|^2) in the operand type, plus the
// partial mean mu_part[k-tile][n] = sum_{k in tile} K_uf[k][n] Lb[k] (fp32 values).
// Block: 64 (k) x 64 (n) tile, thread (ty, tx) owns rows ty+16i, cols tx+16j.
template <int MAXD, typename T>
__global__ void k_kuf(const float *Zs, const float *Xs, int M, int B, int D, const float *sf2,
                      const float *Lb, T *out, long ld, float *mu_part, long ldp) {
  __shared__ float zk[64][MAXD + 1], xn[64][MAXD + 1];
  __shared__ float red[16][65];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int k0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  for (int e = threadIdx.x; e < 64 * D; e += NTB) {
    const int r = e / D, d = e % D;
    zk[r][d] = (k0 + r < M) ? Zs[(long)(k0 + r) * D + d] : 0.f;
    xn[r][d] = (n0 + r < B) ? Xs[(long)(n0 + r) * D + d] : 0.f;
  }
  __syncthreads();
  const float s2 = *sf2;
  float mu[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r = ty + 16 * i, k = k0 + r;
    const float lb = k < M ? Lb[k] : 0.f;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = tx + 16 * j, n = n0 + c;
      float d2 = 0.f;
      for (int d = 0; d < D; ++d) {
        const float df = zk[r][d] - xn[c][d];
        d2 = fmaf(df, df, d2);
      }
      const float v = s2 * __expf(-0.5f * d2);
      if (k < M && n < B) {
        out[(long)k * ld + n] = from_f32<T>(v);
        mu[j] = fmaf(v, lb, mu[j]);
      }
    }
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) red[ty][tx + 16 * j] = mu[j];
  __syncthreads();
  if (threadIdx.x < 64) {
    const int n = n0 + threadIdx.x;
    float s = 0.f;
    for (int r = 0; r < 16; ++r) s += red[r][threadIdx.x];
    if (n < B) mu_part[(long)blockIdx.y * ldp + n] = s;
  }
}

// ---------------------------------------------------------------- copies
// dst = lower triangle of src (strict upper of dst set to 0).
__global__ void k_copy_lower(const float *src, long lds, float *dst, long ldd, int M) {
  const long n = (long)M * M;
  for (long e = blockIdx.x * (long)NTB + threadIdx.x; e < n; e += (long)gridDim.x * NTB) {
    const int i = (int)(e / M), j = (int)(e % M);
    dst[(long)i * ldd + j] = i >= j ? src[(long)i * lds + j] : 0.f;
  }
}
// dst lower triangle = src lower triangle; dst strict upper untouched.
__global__ void k_store_lower(const float *src, long lds, float *dst, long ldd, int M) {
  const long n = (long)M * M;
  for (long e = blockIdx.x * (long)NTB + threadIdx.x; e < n; e += (long)gridDim.x * NTB) {
    const int i = (int)(e / M), j = (int)(e % M);
    if (i >= j) dst[(long)i * ldd + j] = src[(long)i * lds + j];
  }
}

// ---------------------------------------------------------------- matrix-vector
// y[i] = alpha * sum_j A[i][j] x[j] + beta * z[i]; one wave per row; lower:
// restrict to j <= i.  A is fp32 or the operand type.
template <typename S>
__global__ void k_gemv_rows(const S *A, long ld, int R, int Cn, const float *x, int lower,
                            float alpha, const float *z, float beta, float *y) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * (NTB / 64) + (threadIdx.x >> 6);
  if (row >= R) return;
  const int cend = lower ? min(Cn, row + 1) : Cn;
  const S *a = A + (long)row * ld;
  float s = 0.f;
  for (int j = lane; j < cend; j += 64) s = fmaf(to_f32(a[j]), x[j], s);
  s = wave_sum(s);
  if (lane == 0) y[row] = alpha * s + (z ? beta * z[row] : 0.f);
}

// Partial column products: part[chunk][j] = sum_{i in chunk} A[i][j] x[i]
// (lower: i >= j only).  Grid: (ceil(Cn/NTB), nchunk); chunk = 64 rows.
__global__ void k_gemv_cols_part(const float *A, long ld, int R, int Cn, const float *x,
                                 int lower, float *part, long ldp) {
  const int j = blockIdx.x * NTB + threadIdx.x;
  const int i0 = blockIdx.y * 64;
  if (j >= Cn) return;
  float s = 0.f;
  const int iend = min(R, i0 + 64);
  for (int i = lower ? max(i0, j) : i0; i < iend; ++i) s = fmaf(A[(long)i * ld + j], x[i], s);
  part[(long)blockIdx.y * ldp + j] = s;
}
// y[j] = sum_c part[c][j]
__global__ void k_sum_parts(const float *part, long ldp, int nchunk, int n, float *y) {
  const int j = blockIdx.x * NTB + threadIdx.x;
  if (j >= n) return;
  float s = 0.f;
  for (int c = 0; c < nchunk; ++c) s += part[(long)c * ldp + j];
  y[j] = s;
}

// ---------------------------------------------------------------- scalars of the KL
// quad = b^T Wub, logdet = 2 sum log|L_ii| (one block).
__global__ void k_kl_scalars(const float *b, const float *Wub, const float *L, long ld, int M,
                             double *scal, int *flag) {
  __shared__ double sh[NTB / 64];
  double q = 0.0, ldt = 0.0;
  int bad = 0;
  for (int i = threadIdx.x; i < M; i += NTB) {
    q += (double)b[i] * (double)Wub[i];
    const float d = L[(long)i * ld + i];
    if (d == 0.f || !isfinite(d)) bad = 1;
    ldt += log(fabs((double)d));
  }
  q = block_sum<NTB>(q, sh);
  ldt = block_sum<NTB>(ldt, sh);
  if (threadIdx.x == 0) {
    scal[S_QUAD] = q;
    scal[S_LOGDET] = 2.0 * ldt;
  }
  if (bad) atomicOr(flag, FLAG_DOMAIN);
}

// ---------------------------------------------------------------- likelihood
// Per datum: mu = sum of mean partials, var = sf2 - sum of variance partials,
// E_n and alpha_n = c dE/dmu, beta_n = c dE/dvar (c = N/B); block partials of
// [sum E, sum var, sum dE/dnoise, sum beta] in fp64.
struct LikArgs {
  const float *mu_part; int n_mu; const float *var_part; int n_var; long ldp;
  const float *y; int B; const float *sf2; const float *noise; double c;
  int lik; const double *gh; int ngh;  // gh: nodes[ngh] then weights[ngh]
  float *mu, *var, *alpha, *beta, *sqnb;  // sqnb = sqrt(max(0, -beta))
  double *part;  // [nblocks][4]
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
      const double ec = erfc(u);
      logPhi = log1p(-0.5 * erfc(-u));
      lam = sq2_over_pi * exp(-u * u) / ec;
    }
    E += w * logPhi;
    dmu += w * lam * y;
    dsd += w * lam * y * sq2 * t;  // d/dsd
  }
  dv = sd > 0.0 ? dsd / (2.0 * sd) : 0.0;
}

__global__ void k_lik(LikArgs a) {
  __shared__ double sh[NTB / 64];
  const int n = blockIdx.x * NTB + threadIdx.x;
  double e = 0.0, vs = 0.0, dn = 0.0, bs = 0.0;
  if (n < a.B) {
    float m = 0.f, vp = 0.f;
    for (int k = 0; k < a.n_mu; ++k) m += a.mu_part[(long)k * a.ldp + n];
    for (int k = 0; k < a.n_var; ++k) vp += a.var_part[(long)k * a.ldp + n];
    const double mu = m, var = (double)(*a.sf2) - (double)vp;
    const double y = a.y[n];
    double E, dmu, dv;
    if (a.lik == 0) {
      const double s2 = *a.noise;
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
    a.alpha[n] = (float)(a.c * dmu);
    a.beta[n] = (float)(a.c * dv);
    a.sqnb[n] = (float)sqrt(fmax(0.0, -a.c * dv));
    e = E;
    vs = var;
    bs = a.c * dv;
  }
  e = block_sum<NTB>(e, sh);
  vs = block_sum<NTB>(vs, sh);
  dn = block_sum<NTB>(dn, sh);
  bs = block_sum<NTB>(bs, sh);
  if (threadIdx.x == 0) {
    double *p = a.part + 4 * blockIdx.x;
    p[0] = e; p[1] = vs; p[2] = dn; p[3] = bs;
  }
}

// ---------------------------------------------------------------- finalisation
// Residual of one NG step from the gram partials: sqrt(sum / M).
__global__ void k_resid(const double *part, int n, int M, double *out, double *scal) {
  __shared__ double sh[NTB / 64];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += NTB) s += part[i];
  s = block_sum<NTB>(s, sh);
  if (threadIdx.x == 0) {
    const double r = sqrt(s / M);
    scal[S_RESID] = r;
    if (out) *out = r;
  }
}

// F = c sum E - KL with
// KL = 1/2 (-tr(Q Wu) + tr W - M + quad - log|T| - sum log s~).
__global__ void k_finalize_bound(const double *gram_part, int n_gram, const double *lik_part,
                                 int n_lik, const double *scal, int M, double c,
                                 double *out_bound, double *out_terms, int *flag) {
  __shared__ double sh[NTB / 64];
  double trw = 0.0, qwu = 0.0, r2 = 0.0, e = 0.0, vs = 0.0;
  for (int i = threadIdx.x; i < n_gram; i += NTB) {
    trw += gram_part[3 * i];
    qwu += gram_part[3 * i + 1];
    r2 += gram_part[3 * i + 2];
  }
  for (int i = threadIdx.x; i < n_lik; i += NTB) {
    e += lik_part[4 * i];
    vs += lik_part[4 * i + 1];
  }
  trw = block_sum<NTB>(trw, sh);
  qwu = block_sum<NTB>(qwu, sh);
  r2 = block_sum<NTB>(r2, sh);
  e = block_sum<NTB>(e, sh);
  vs = block_sum<NTB>(vs, sh);
  if (threadIdx.x == 0) {
    const double quad = scal[S_QUAD], logdet = scal[S_LOGDET], sls = scal[S_SUMLOGS];
    const double KL = 0.5 * (-qwu + trw - (double)M + quad - logdet - sls);
    const double data = c * e;
    const double F = data - KL;
    if (!isfinite(F)) atomicOr(flag, FLAG_NONFINITE);
    if (out_bound) *out_bound = F;
    if (out_terms) {
      out_terms[0] = data;
      out_terms[1] = KL;
      out_terms[2] = vs;
      out_terms[3] = sqrt(r2 / M);
      out_terms[4] = trw;
      out_terms[5] = qwu;
      out_terms[6] = quad;
      out_terms[7] = logdet;
    }
  }
}

// ---------------------------------------------------------------- backward
// C = -sym((V alpha) a^T) + V diag(beta) V^T - 1/2 (Wu + I - Wub a^T - a Wub^T)
//     + 1/2 (Q - b b^T), with V diag(beta) V^T = -sum_s Ys[s] (split-K pieces of
// (V D)(V D)^T, D = diag(sqrt(-beta))).  Ys holds lower tiles only; read (max, min).
__global__ void k_assemble_C(const float *Ys, int nsplit, long split_stride, const float *Wu,
                             const float *Q, const float *a, const float *b, const float *Wub,
                             const float *Va, int M, long ld, float *Cm) {
  const long n = (long)M * M;
  for (long e = blockIdx.x * (long)NTB + threadIdx.x; e < n; e += (long)gridDim.x * NTB) {
    const int i = (int)(e / M), j = (int)(e % M);
    const int hi = max(i, j), lo = min(i, j);
    float ys = 0.f;
    for (int s = 0; s < nsplit; ++s) ys += Ys[s * split_stride + (long)hi * ld + lo];
    const long ij = (long)i * ld + j;
    const float c = -0.5f * (Va[i] * a[j] + a[i] * Va[j]) - ys -
                    0.5f * (Wu[ij] + (i == j ? 1.f : 0.f) - Wub[i] * a[j] - a[i] * Wub[j]) +
                    0.5f * (Q[ij] - b[i] * b[j]);
    Cm[ij] = c;
  }
}

// V alpha over the operand-type V (one wave per row).
template <typename T>
__global__ void k_valpha(const T *V, long ld, int M, int B, const float *alpha, float *out) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * (NTB / 64) + (threadIdx.x >> 6);
  if (row >= M) return;
  const T *v = V + (long)row * ld;
  float s = 0.f;
  for (int n = lane; n < B; n += 64) s = fmaf(to_f32(v[n]), alpha[n], s);
  s = wave_sum(s);
  if (lane == 0) out[row] = s;
}

struct GradArgs {
  int M, B, D;
  const float *Zs, *Xs, *inv_ell, *sf2;
  const float *hrow; int n_uf_nt;       // [n_uf_nt][M]
  const float *hx;                      // [n_uf_nt][M][D]
  const float *hcol; int n_uf_mt; long ldc;  // [n_uf_mt][ldc]
  const float *hzrow; const float *hz; int nb;  // [nb][M], [nb][M][D]
  const double *uf_part; int n_uf_tiles;
  const double *uu_part; int n_uu_tiles;
  const double *lik_part; int n_lik;
  double c;
  const double *grad_scale;
  float *g_Z, *g_ell, *g_sf2, *g_noise;
  double *ell_part;  // [nblk_rows + nblk_cols][D]
};

// Per inducing row i: reduce the partials, write dF/dZ_i, and accumulate the
// row part of dF/dell_d (scaled coordinates, divided by ell_d at the end):
//   sum_i r_uf_i zs_id^2 - 2 zs_id hx_id + 2 (r_uu_i zs_id^2 - zs_id hz_id)
__global__ void k_grad_rows(GradArgs g) {
  __shared__ double sh[64][65];
  const int i = blockIdx.x * 64 + (threadIdx.x & 63);
  const int dgrp = threadIdx.x >> 6;  // 4 groups of d
  const double scale = g.grad_scale ? *g.grad_scale : 1.0;
  float ruf = 0.f, ruu = 0.f;
  if (i < g.M) {
    for (int k = 0; k < g.n_uf_nt; ++k) ruf += g.hrow[(long)k * g.M + i];
    for (int k = 0; k < g.nb; ++k) ruu += g.hzrow[(long)k * g.M + i];
  }
  for (int d0 = 0; d0 < g.D; d0 += 64) {
    for (int dd = dgrp; dd < 64; dd += 4) {
      const int d = d0 + dd;
      double contrib = 0.0;
      if (i < g.M && d < g.D) {
        float hx = 0.f, hz = 0.f;
        for (int k = 0; k < g.n_uf_nt; ++k) hx += g.hx[((long)k * g.M + i) * g.D + d];
        for (int k = 0; k < g.nb; ++k) hz += g.hz[((long)k * g.M + i) * g.D + d];
        const double zs = g.Zs[(long)i * g.D + d];
        const double il = g.inv_ell[d];
        // dF/dZ_id = -(1/ell_d) [ (zs r_uf - hx) + 2 (zs r_uu - hz) ]
        const double gz = -il * ((zs * ruf - hx) + 2.0 * (zs * ruu - hz));
        if (g.g_Z) g.g_Z[(long)i * g.D + d] = (float)(scale * gz);
        contrib = ruf * zs * zs - 2.0 * zs * hx + 2.0 * (ruu * zs * zs - zs * hz);
      }
      sh[dd][threadIdx.x & 63] = contrib;
    }
    __syncthreads();
    for (int dd = threadIdx.x; dd < 64; dd += NTB) {
      double s = 0.0;
      for (int r = 0; r < 64; ++r) s += sh[dd][r];
      if (d0 + dd < g.D) g.ell_part[(long)blockIdx.x * g.D + d0 + dd] = s;
    }
    __syncthreads();
  }
}

// Per datum n: c_n = sum_i H_in; accumulate sum_n c_n xs_nd^2 into ell_part.
__global__ void k_grad_cols(GradArgs g, int row_blocks) {
  __shared__ double sh[64][65];
  const int n = blockIdx.x * 64 + (threadIdx.x & 63);
  const int dgrp = threadIdx.x >> 6;
  float cn = 0.f;
  if (n < g.B)
    for (int k = 0; k < g.n_uf_mt; ++k) cn += g.hcol[(long)k * g.ldc + n];
  for (int d0 = 0; d0 < g.D; d0 += 64) {
    for (int dd = dgrp; dd < 64; dd += 4) {
      const int d = d0 + dd;
      double contrib = 0.0;
      if (n < g.B && d < g.D) {
        const double xs = g.Xs[(long)n * g.D + d];
        contrib = cn * xs * xs;
      }
      sh[dd][threadIdx.x & 63] = contrib;
    }
    __syncthreads();
    for (int dd = threadIdx.x; dd < 64; dd += NTB) {
      double s = 0.0;
      for (int r = 0; r < 64; ++r) s += sh[dd][r];
      if (d0 + dd < g.D) g.ell_part[(long)(row_blocks + blockIdx.x) * g.D + d0 + dd] = s;
    }
    __syncthreads();
  }
}

// dF/dell_d = (1/ell_d) sum of partials; dF/dsf2 = (sum H_uu + sum H_uf)/sf2 + sum beta;
// dF/dnoise = c sum dE/dnoise.  One block.
__global__ void k_grad_final(GradArgs g, int nparts) {
  __shared__ double sh[NTB / 64];
  const double scale = g.grad_scale ? *g.grad_scale : 1.0;
  for (int d = threadIdx.x; d < g.D; d += NTB) {
    double s = 0.0;
    for (int p = 0; p < nparts; ++p) s += g.ell_part[(long)p * g.D + d];
    if (g.g_ell) g.g_ell[d] = (float)(scale * s * g.inv_ell[d]);
  }
  double huf = 0.0, huu = 0.0, dn = 0.0, bs = 0.0;
  for (int i = threadIdx.x; i < g.n_uf_tiles; i += NTB) huf += g.uf_part[i];
  for (int i = threadIdx.x; i < g.n_uu_tiles; i += NTB) huu += g.uu_part[i];
  for (int i = threadIdx.x; i < g.n_lik; i += NTB) {
    dn += g.lik_part[4 * i + 2];
    bs += g.lik_part[4 * i + 3];
  }
  huf = block_sum<NTB>(huf, sh);
  huu = block_sum<NTB>(huu, sh);
  dn = block_sum<NTB>(dn, sh);
  bs = block_sum<NTB>(bs, sh);
  if (threadIdx.x == 0) {
    if (g.g_sf2) *g.g_sf2 = (float)(scale * ((huf + huu) / (double)(*g.sf2) + bs));
    if (g.g_noise) *g.g_noise = (float)(scale * g.c * dn);
  }
}

// out = scale * x (optional scale pointer).
__global__ void k_scale_vec(const float *x, int n, const double *scale, float *out) {
  const int i = blockIdx.x * NTB + threadIdx.x;
  if (i < n) out[i] = (float)((scale ? *scale : 1.0) * x[i]);
}
// out = x - y
__global__ void k_sub_vec(const float *x, const float *y, int n, float *out) {
  const int i = blockIdx.x * NTB + threadIdx.x;
  if (i < n) out[i] = x[i] - y[i];
}
