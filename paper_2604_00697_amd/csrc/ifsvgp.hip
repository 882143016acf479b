// C ABI of the inverse-free SVGP training iteration (host orchestration).
// Declarations and the contract of every entry point: include/ifsvgp.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <type_traits>
#include <vector>

#include "../../include/ifsvgp.h"
#include "epilogues.hpp"
#include "kernels.hpp"

#define IFSVGP_VERSION 100

static constexpr int MAXD = 64;  // input dimension limit of the LDS-staged kernels

// ------------------------------------------------------------------ kernel kinds
enum KernelKind : int {
  KK_PREP = 0, KK_KUU, KK_COPYL, KK_NG_Y, KK_NG_W, KK_NG_L, KK_RESID,
  KK_GR_Y, KK_GR_W, KK_GR_E, KK_VEC, KK_KUF, KK_V, KK_U, KK_LIK, KK_FIN,
  KK_R, KK_VALPHA, KK_SYRK, KK_ASM, KK_Y2, KK_GUU, KK_GRAD, KK_STOREL, KK_N
};
static const char *KK_NAMES[KK_N] = {
    "prep", "kuu", "copy_L", "ng_KL", "ng_gram", "ng_update", "ng_resid",
    "bound_KL", "bound_gram", "bound_gram_E", "matvec", "kuf", "gemm_V", "gemm_U", "likelihood",
    "finalize", "gemm_R_grad_uf", "valpha", "syrk", "assemble_C", "gemm_LC", "gemm_G_grad_uu",
    "grad_final", "store_L"};

struct TimingRec {
  int kind;
  hipEvent_t a, b;
};

struct ifsvgp_ctx {
  int M, Bmax, D, prec, lik, ngh;
  int Mp, Bp;
  int nb64, nb128m, nb128n;  // tile counts
  int nsplit;
  hipStream_t st;
  // buffers
  float *Kt, *Lw[2], *Y, *Wn, *Q, *Wu, *Cm, *Y2, *Ys;
  void *Kuf, *V, *U;
  float *Zs, *Xs, *inv_ell;
  float *va, *vb, *vLb, *vWub, *vVa, *vt1, *vt2, *vpart;
  float *mu_part, *var_part, *mu, *var, *alpha, *beta, *sqnb;
  float *hrow, *hcol, *hx, *hzrow, *hz;
  double *scal, *tp_ng, *tp_gram, *tp_uf, *tp_uu, *lik_part, *ell_part;
  double *gh;
  int *flag;
  // last forward state for the backward
  int fwd_valid, fwd_B;
  int cur_L;  // which Lw holds the bound's L
  // timing
  long long timing;  // bit mask of timed kernel kinds
  std::vector<TimingRec> recs;
  std::vector<hipEvent_t> pool;
  double t_ms[KK_N];
  long t_cnt[KK_N];
  std::vector<void *> allocs;
};

// ------------------------------------------------------------------ helpers
static inline int rup(int x, int m) { return (x + m - 1) / m * m; }
static inline int cdiv(long x, long m) { return (int)((x + m - 1) / m); }

#define HIPCK(x)                                      \
  do {                                                \
    hipError_t _e = (x);                              \
    if (_e != hipSuccess) return IFSVGP_EHIP;         \
  } while (0)

struct Timed {
  ifsvgp_ctx *c;
  int kind;
  hipEvent_t b;
  Timed(ifsvgp_ctx *c_, int k) : c(c_), kind(k), b(nullptr) {
    if (!((c->timing >> kind) & 1)) return;
    hipEvent_t a = get();
    b = get();
    hipEventRecord(a, c->st);
    c->recs.push_back({kind, a, b});
  }
  ~Timed() {
    if (b) hipEventRecord(b, c->st);
  }
  hipEvent_t get() {
    if (!c->pool.empty()) {
      hipEvent_t e = c->pool.back();
      c->pool.pop_back();
      return e;
    }
    hipEvent_t e;
    hipEventCreate(&e);
    return e;
  }
};

template <typename T>
static hipError_t dmalloc(ifsvgp_ctx *c, T **p, size_t n) {
  void *q = nullptr;
  hipError_t e = hipMalloc(&q, std::max<size_t>(n, 1) * sizeof(T));
  if (e != hipSuccess) return e;
  e = hipMemset(q, 0, std::max<size_t>(n, 1) * sizeof(T));
  c->allocs.push_back(q);
  *p = (T *)q;
  return e;
}

static size_t op_size(int prec) { return prec == IFSVGP_PREC_FP32 ? 4 : 2; }

// ------------------------------------------------------------------ GH rule (host)
// Physicists' Hermite polynomials by the three-term recurrence
//   H_{k+1}(t) = 2 t H_k(t) - 2 k H_{k-1}(t),
// roots by Newton's method from asymptotic initial guesses, weights
// w_k = 2^{n-1} n! sqrt(pi) / (n^2 H_{n-1}(t_k)^2), evaluated with the
// normalised recurrence to avoid overflow.
extern "C" int ifsvgp_gh_rule(int n, double *nodes, double *weights) {
  if (n < 1 || n > 64 || !nodes || !weights) return IFSVGP_EINVAL;
  const double pim4 = 0.7511255444649425;  // pi^{-1/4}
  const int m = (n + 1) / 2;
  double z = 0.0;
  for (int i = 0; i < m; ++i) {
    // initial guesses for the largest roots first
    if (i == 0) z = std::sqrt(2.0 * n + 1) - 1.85575 * std::pow(2.0 * n + 1, -0.16667);
    else if (i == 1) z -= 1.14 * std::pow((double)n, 0.426) / z;
    else if (i == 2) z = 1.86 * z - 0.86 * nodes[0];
    else if (i == 3) z = 1.91 * z - 0.91 * nodes[1];
    else z = 2.0 * z - nodes[i - 2];
    double pp = 0.0;
    for (int it = 0; it < 100; ++it) {
      // orthonormal recurrence: p_{k} = sqrt(2/k) t p_{k-1} - sqrt((k-1)/k) p_{k-2}
      double p1 = pim4, p2 = 0.0;
      for (int k = 1; k <= n; ++k) {
        const double p3 = p2;
        p2 = p1;
        p1 = z * std::sqrt(2.0 / k) * p2 - std::sqrt((k - 1.0) / k) * p3;
      }
      pp = std::sqrt(2.0 * n) * p2;  // derivative of the orthonormal p_n
      const double z1 = z;
      z = z1 - p1 / pp;
      if (std::fabs(z - z1) <= 1e-15 * std::max(1.0, std::fabs(z))) break;
    }
    nodes[i] = z;
    nodes[n - 1 - i] = -z;
    weights[i] = 2.0 / (pp * pp);
    weights[n - 1 - i] = weights[i];
  }
  if (n % 2 == 1) nodes[m - 1] = 0.0;  // exact middle root
  // return ascending order
  for (int i = 0; i < n / 2; ++i) {
    std::swap(nodes[i], nodes[n - 1 - i]);
    std::swap(weights[i], weights[n - 1 - i]);
  }
  return IFSVGP_OK;
}

// ------------------------------------------------------------------ API: misc
extern "C" int ifsvgp_version(void) { return IFSVGP_VERSION; }

extern "C" const char *ifsvgp_strerror(int code) {
  switch (code) {
    case IFSVGP_OK: return "ok";
    case IFSVGP_EINVAL: return "invalid argument";
    case IFSVGP_EDOMAIN: return "domain error: non-positive ell, sf2, noise_var or s_tilde, or zero L_ii";
    case IFSVGP_EHIP: return "HIP runtime error";
    case IFSVGP_ENONFINITE: return "non-finite bound or factor";
    case IFSVGP_ENOMEM: return "out of device memory";
    case IFSVGP_ESTATE: return "backward without a matching forward on this context";
    default: return "unknown status code";
  }
}

extern "C" void ifsvgp_destroy(ifsvgp_ctx *c) {
  if (!c) return;
  for (void *p : c->allocs) hipFree(p);
  for (auto &r : c->recs) {
    hipEventDestroy(r.a);
    hipEventDestroy(r.b);
  }
  for (auto e : c->pool) hipEventDestroy(e);
  delete c;
}

extern "C" int ifsvgp_create(ifsvgp_ctx **out, int M, int B_max, int D, int prec, int lik,
                             int n_gh) {
  if (!out || M < 1 || B_max < 1 || D < 1 || D > MAXD) return IFSVGP_EINVAL;
  if (prec < 0 || prec > 2 || lik < 0 || lik > 1) return IFSVGP_EINVAL;
  if (lik == IFSVGP_LIK_PROBIT && (n_gh < 1 || n_gh > 64)) return IFSVGP_EINVAL;
  if ((long)M * M > (1L << 30) || (long)M * B_max > (1L << 31)) return IFSVGP_EINVAL;
  ifsvgp_ctx *c = new (std::nothrow) ifsvgp_ctx();
  if (!c) return IFSVGP_ENOMEM;
  c->M = M; c->Bmax = B_max; c->D = D; c->prec = prec; c->lik = lik;
  c->ngh = lik == IFSVGP_LIK_PROBIT ? n_gh : 0;
  c->Mp = rup(M, 64);
  c->Bp = rup(B_max, 64);
  c->nb64 = cdiv(M, 64);
  c->nb128m = cdiv(M, 128);
  c->nb128n = cdiv(B_max, 128);
  c->nsplit = std::max(1, std::min(16, cdiv(B_max, 512)));
  c->st = nullptr;
  const size_t MM = (size_t)M * c->Mp, MB = (size_t)M * c->Bp;
  const size_t os = op_size(prec);
  const int nt_sym64 = c->nb64 * (c->nb64 + 1) / 2;
  const int nt_rect = c->nb128m * c->nb128n;
  hipError_t e = hipSuccess;
#define ALLOC(p, n) if (e == hipSuccess) e = dmalloc(c, &(p), (n))
  ALLOC(c->Kt, MM);
  ALLOC(c->Lw[0], MM);
  ALLOC(c->Lw[1], MM);
  ALLOC(c->Y, MM);
  ALLOC(c->Wn, MM);
  ALLOC(c->Q, MM);
  ALLOC(c->Wu, MM);
  ALLOC(c->Cm, MM);
  ALLOC(c->Y2, MM);
  ALLOC(c->Ys, MM * c->nsplit);
  {
    unsigned char *k = nullptr, *v = nullptr, *u = nullptr;
    ALLOC(k, MB * os);
    ALLOC(v, MB * os);
    ALLOC(u, MB * os);
    c->Kuf = k; c->V = v; c->U = u;
  }
  ALLOC(c->Zs, (size_t)M * D);
  ALLOC(c->Xs, (size_t)B_max * D);
  ALLOC(c->inv_ell, (size_t)D);
  ALLOC(c->va, (size_t)c->Mp);
  ALLOC(c->vb, (size_t)c->Mp);
  ALLOC(c->vLb, (size_t)c->Mp);
  ALLOC(c->vWub, (size_t)c->Mp);
  ALLOC(c->vVa, (size_t)c->Mp);
  ALLOC(c->vt1, (size_t)c->Mp);
  ALLOC(c->vt2, (size_t)c->Mp);
  ALLOC(c->vpart, (size_t)c->nb64 * c->Mp);
  ALLOC(c->mu_part, (size_t)c->nb64 * c->Bp);
  ALLOC(c->var_part, (size_t)c->nb128m * c->Bp);
  ALLOC(c->mu, (size_t)c->Bp);
  ALLOC(c->var, (size_t)c->Bp);
  ALLOC(c->alpha, (size_t)c->Bp);
  ALLOC(c->beta, (size_t)c->Bp);
  ALLOC(c->sqnb, (size_t)c->Bp);
  ALLOC(c->hrow, (size_t)c->nb128n * M);
  ALLOC(c->hcol, (size_t)c->nb128m * c->Bp);
  ALLOC(c->hx, (size_t)c->nb128n * M * D);
  ALLOC(c->hzrow, (size_t)c->nb64 * M);
  ALLOC(c->hz, (size_t)c->nb64 * M * D);
  ALLOC(c->scal, (size_t)S_NSLOT);
  ALLOC(c->tp_ng, (size_t)nt_sym64);
  ALLOC(c->tp_gram, (size_t)3 * nt_sym64);
  ALLOC(c->tp_uf, (size_t)nt_rect);
  ALLOC(c->tp_uu, (size_t)nt_sym64);
  ALLOC(c->lik_part, (size_t)4 * cdiv(B_max, NTB));
  ALLOC(c->ell_part, (size_t)(cdiv(M, 64) + cdiv(B_max, 64)) * D);
  ALLOC(c->gh, (size_t)2 * std::max(1, c->ngh));
  ALLOC(c->flag, (size_t)1);
#undef ALLOC
  if (e == hipSuccess && c->ngh > 0) {
    std::vector<double> g(2 * c->ngh);
    ifsvgp_gh_rule(c->ngh, g.data(), g.data() + c->ngh);
    e = hipMemcpy(c->gh, g.data(), g.size() * sizeof(double), hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) {
    const int code = e == hipErrorOutOfMemory ? IFSVGP_ENOMEM : IFSVGP_EHIP;
    ifsvgp_destroy(c);
    return code;
  }
  c->fwd_valid = 0;
  c->cur_L = 0;
  c->timing = 0;
  for (int k = 0; k < KK_N; ++k) { c->t_ms[k] = 0.0; c->t_cnt[k] = 0; }
  *out = c;
  return IFSVGP_OK;
}

extern "C" int ifsvgp_set_stream(ifsvgp_ctx *c, void *s) {
  if (!c) return IFSVGP_EINVAL;
  c->st = (hipStream_t)s;
  return IFSVGP_OK;
}

extern "C" int ifsvgp_status(ifsvgp_ctx *c) {
  if (!c) return IFSVGP_EINVAL;
  HIPCK(hipStreamSynchronize(c->st));
  int f = 0;
  HIPCK(hipMemcpy(&f, c->flag, sizeof(int), hipMemcpyDeviceToHost));
  int z = 0;
  HIPCK(hipMemcpy(c->flag, &z, sizeof(int), hipMemcpyHostToDevice));
  if (f & FLAG_DOMAIN) return IFSVGP_EDOMAIN;
  if (f & FLAG_NONFINITE) return IFSVGP_ENONFINITE;
  return IFSVGP_OK;
}

extern "C" int ifsvgp_timing_enable(ifsvgp_ctx *c, long long kind_mask) {
  if (!c) return IFSVGP_EINVAL;
  c->timing = kind_mask;
  return IFSVGP_OK;
}

extern "C" int ifsvgp_timing_read(ifsvgp_ctx *c, int cap, double *total_ms, int *count,
                                  const char **names) {
  if (!c) return IFSVGP_EINVAL;
  HIPCK(hipStreamSynchronize(c->st));
  for (auto &r : c->recs) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      c->t_ms[r.kind] += ms;
      c->t_cnt[r.kind] += 1;
    }
    c->pool.push_back(r.a);
    c->pool.push_back(r.b);
  }
  c->recs.clear();
  for (int k = 0; k < KK_N && k < cap; ++k) {
    if (total_ms) total_ms[k] = c->t_ms[k];
    if (count) count[k] = (int)c->t_cnt[k];
    if (names) names[k] = KK_NAMES[k];
    c->t_ms[k] = 0.0;
    c->t_cnt[k] = 0;
  }
  return KK_N;
}

// Algorithmic flops per launch (structure-aware: triangular factors at their
// nonzero density, symmetric outputs counted once).
extern "C" int ifsvgp_kernel_flops(ifsvgp_ctx *c, int B, int cap, double *flops,
                                   const char **names) {
  if (!c || !flops) return IFSVGP_EINVAL;
  const double M = c->M, Bd = B, D = c->D;
  double f[KK_N] = {0};
  f[KK_NG_Y] = 2.0 * M * M * M / 3.0;   // lower part of K~ L, sum_{l>=j} over k>=j
  f[KK_NG_W] = M * M * M / 3.0;         // lower part of L^T Y
  f[KK_NG_L] = M * M * M / 3.0;         // L X, both lower triangular
  f[KK_GR_Y] = 2.0 * M * M * M / 3.0;
  f[KK_GR_W] = M * M * M / 3.0;
  f[KK_GR_E] = M * M * M / 3.0;
  f[KK_V] = M * M * Bd;                 // L^T K_uf, triangular
  f[KK_U] = 2.0 * M * M * Bd;           // Q V
  f[KK_R] = M * M * Bd + 2.0 * M * Bd * D;  // L U (+ H X)
  f[KK_SYRK] = M * M * Bd;              // lower half of V diag(beta) V^T
  f[KK_Y2] = M * M * M;                 // L C
  f[KK_GUU] = M * M * M / 3.0 + 2.0 * M * M * D;  // lower half of Y2 L^T (+ H Z)
  f[KK_KUF] = 3.0 * M * Bd * D;
  f[KK_KUU] = 3.0 * M * M * D;
  for (int k = 0; k < KK_N && k < cap; ++k) {
    flops[k] = f[k];
    if (names) names[k] = KK_NAMES[k];
  }
  return KK_N;
}

// ------------------------------------------------------------------ GEMM wrappers
template <typename T>
struct Ops {
  using CS = Cfg<64, 64, 2, 2, 2, T>;    // M x M products
  using CR = Cfg<128, 128, 2, 2, 2, T>;  // M x B products
  // The two products with the backward matrix C (whose entries grow like
  // B / noise_var) need fp32's exponent range: fp16 operands would overflow,
  // so the fp16 form runs them on bf16 MFMA.
  using TW = typename std::conditional<std::is_same<T, _Float16>::value, __bf16, T>::type;
  using CSW = Cfg<64, 64, 2, 2, 2, TW>;

  // Y = K~ L (lower tiles), k >= n0
  static hipError_t ng_Y(ifsvgp_ctx *c, const float *L, float *Y) {
    const int M = c->M;
    Ld<float, true, XfNone> la{c->Kt, c->Mp, M, M, 1, {}};
    Ld<float, false, XfLower> lb{L, c->Mp, M, M, 1, {}};
    Sched sc{c->nb64, c->nb64, 1, 1, M, K_LO_N0};
    EpiStore<float> e{Y, c->Mp, M, M, 0, 0};
    return launch_gemm<CS>(c->st, la, lb, sc, e);
  }
  // W = L^T Y (lower tiles), k >= m0, with residual partials
  static hipError_t ng_W(ifsvgp_ctx *c, const float *L) {
    const int M = c->M;
    Ld<float, false, XfLower> la{L, c->Mp, M, M, 1, {}};
    Ld<float, false, XfNone> lb{c->Y, c->Mp, M, M, 1, {}};
    Sched sc{c->nb64, c->nb64, 1, 1, M, K_LO_M0};
    EpiNgGram e{c->Wn, c->Mp, M, c->tp_ng};
    return launch_gemm<CS>(c->st, la, lb, sc, e);
  }
  // Lnew = L - gamma L X(W), lower tiles, n0 <= k < m0+BM
  static hipError_t ng_L(ifsvgp_ctx *c, const float *L, float *Ln, float gamma) {
    const int M = c->M;
    Ld<float, true, XfLower> la{L, c->Mp, M, M, 1, {}};
    Ld<float, false, XfNatgrad> lb{c->Wn, c->Mp, M, M, 1, {}};
    Sched sc{c->nb64, c->nb64, 1, 1, M, K_LO_N0 | K_HI_M1};
    EpiNgUpdate e{L, c->Mp, Ln, c->Mp, M, gamma};
    return launch_gemm<CS>(c->st, la, lb, sc, e);
  }
  // W' = L^T Y (lower tiles, plain store)
  static hipError_t gr_W(ifsvgp_ctx *c, const float *L) {
    const int M = c->M;
    Ld<float, false, XfLower> la{L, c->Mp, M, M, 1, {}};
    Ld<float, false, XfNone> lb{c->Y, c->Mp, M, M, 1, {}};
    Sched sc{c->nb64, c->nb64, 1, 1, M, K_LO_M0};
    EpiStore<float> e{c->Wn, c->Mp, M, M, 0, 0};
    return launch_gemm<CS>(c->st, la, lb, sc, e);
  }
  // E' = L^T diag(s) L (lower tiles) -> Q, Wu, gram partials
  static hipError_t gr_E(ifsvgp_ctx *c, const float *L, const float *s) {
    const int M = c->M;
    Ld<float, false, XfLower> la{L, c->Mp, M, M, 1, {}};
    Ld<float, false, XfLowerScaleRow> lb{L, c->Mp, M, M, 1, {s}};
    Sched sc{c->nb64, c->nb64, 1, 1, M, K_LO_M0};
    EpiBoundGram e{c->Wn, c->Q, c->Wu, c->Mp, M, c->tp_gram};
    return launch_gemm<CS>(c->st, la, lb, sc, e);
  }
  // V = L^T K_uf, k >= m0
  static hipError_t gemm_V(ifsvgp_ctx *c, const float *L, int B) {
    const int M = c->M;
    Ld<float, false, XfLower> la{L, c->Mp, M, M, 1, {}};
    Ld<T, false, XfNone> lb{(const T *)c->Kuf, c->Bp, M, B, 1, {}};
    Sched sc{cdiv(M, 128), cdiv(B, 128), 0, 1, M, K_LO_M0};
    EpiStore<T> e{(T *)c->V, c->Bp, M, B, 0, 0};
    return launch_gemm<CR>(c->st, la, lb, sc, e);
  }
  // U = Q V, sigma^2 partials
  static hipError_t gemm_U(ifsvgp_ctx *c, int B) {
    const int M = c->M;
    Ld<float, true, XfNone> la{c->Q, c->Mp, M, M, 1, {}};
    Ld<T, false, XfNone> lb{(const T *)c->V, c->Bp, M, B, 1, {}};
    Sched sc{cdiv(M, 128), cdiv(B, 128), 0, 1, M, 0};
    EpiU<T> e{(T *)c->U, (const T *)c->V, c->Bp, M, B, c->var_part, c->Bp};
    return launch_gemm<CR>(c->st, la, lb, sc, e);
  }
  // R = L U -> H_uf reductions
  static hipError_t gemm_R(ifsvgp_ctx *c, const float *L, int B, const float *sf2) {
    const int M = c->M, D = c->D;
    Ld<float, true, XfLower> la{L, c->Mp, M, M, 1, {}};
    Ld<T, false, XfNone> lb{(const T *)c->U, c->Bp, M, B, 1, {}};
    Sched sc{cdiv(M, 128), cdiv(B, 128), 0, 1, M, K_HI_M1};
    EpiGradUf e{c->vLb, c->alpha, c->beta, c->Zs, c->Xs, sf2, M, B, D,
                c->hrow, c->hcol, (long)c->Bp, c->hx, c->tp_uf};
    const int D4 = (D + 3) & ~3;
    return launch_gemm<CR>(c->st, la, lb, sc, e, (CR::BM + CR::BN) * D4 * 4);
  }
  // Ys[s] = (V_s D)(V_s D)^T with D = diag(sqrt(-beta)), i.e. -V diag(beta) V^T
  // (lower tiles, split-K over the batch).  beta <= 0 for log-concave
  // likelihoods (Gaussian, probit), so the split keeps both operands at the
  // scale sqrt(|beta|) |V| instead of |beta| |V|.
  static hipError_t syrk(ifsvgp_ctx *c, int B) {
    const int M = c->M;
    Ld<T, true, XfScaleCol> la{(const T *)c->V, c->Bp, M, B, 1, {c->sqnb}};
    Ld<T, true, XfScaleCol> lb{(const T *)c->V, c->Bp, M, B, 1, {c->sqnb}};
    const int ns = std::max(1, std::min(c->nsplit, cdiv(B, CS::BK)));
    Sched sc{c->nb64, c->nb64, 1, ns, B, 0};
    EpiStore<float> e{c->Ys, c->Mp, M, M, 0, (long)M * c->Mp};
    return launch_gemm<CS>(c->st, la, lb, sc, e);
  }
  // Y2 = L C, k < m0+BM
  static hipError_t gemm_Y2(ifsvgp_ctx *c, const float *L) {
    const int M = c->M;
    Ld<float, true, XfLower> la{L, c->Mp, M, M, 1, {}};
    Ld<float, false, XfNone> lb{c->Cm, c->Mp, M, M, 1, {}};
    Sched sc{c->nb64, c->nb64, 0, 1, M, K_HI_M1};
    EpiStore<float> e{c->Y2, c->Mp, M, M, 0, 0};
    return launch_gemm<CSW>(c->st, la, lb, sc, e);
  }
  // G_uu = Y2 L^T (lower tiles), k < n0+BN -> H_uu reductions
  static hipError_t gemm_Guu(ifsvgp_ctx *c, const float *L, const float *s) {
    const int M = c->M, D = c->D;
    Ld<float, true, XfNone> la{c->Y2, c->Mp, M, M, 1, {}};
    Ld<float, true, XfLower> lb{L, c->Mp, M, M, 1, {}};
    Sched sc{c->nb64, c->nb64, 1, 1, M, K_HI_N1};
    EpiGradUu e{c->Kt, s, c->Zs, c->Mp, M, D, c->hz, c->hzrow, c->tp_uu};
    const int D4 = (D + 3) & ~3;
    return launch_gemm<CSW>(c->st, la, lb, sc, e, 2 * CSW::BM * D4 * 4);
  }
};

// ------------------------------------------------------------------ stages
static int grid1(long n) { return (int)std::min<long>(std::max<long>(1, (n + NTB - 1) / NTB), 65536); }

static int stage_kernel_blocks(ifsvgp_ctx *c, const float *Z, const float *ell, const float *sf2,
                               const float *noise, const float *s, int need_noise) {
  const int M = c->M, D = c->D;
  {
    Timed t(c, KK_PREP);
    hipLaunchKernelGGL(k_prep, dim3(1), dim3(NTB), 0, c->st, ell, sf2, noise, s, M, D,
                       need_noise, c->inv_ell, c->scal, c->flag);
    hipLaunchKernelGGL(k_scale_rows, dim3(grid1((long)M * D)), dim3(NTB), 0, c->st, Z, M, D,
                       (const float *)c->inv_ell, c->Zs);
  }
  {
    Timed t(c, KK_KUU);
    hipLaunchKernelGGL(k_kuu<MAXD>, dim3(cdiv(M, 16), cdiv(M, 16)), dim3(NTB), 0, c->st,
                       (const float *)c->Zs, M, D, sf2, s, c->Kt, (long)c->Mp);
  }
  HIPCK(hipGetLastError());
  return IFSVGP_OK;
}

template <typename T>
static int stage_natgrad(ifsvgp_ctx *c, const float *L_in, const float *gammas, int n_ng,
                         double *out_resid) {
  const int M = c->M;
  {
    Timed t(c, KK_COPYL);
    hipLaunchKernelGGL(k_copy_lower, dim3(grid1((long)M * M)), dim3(NTB), 0, c->st, L_in,
                       (long)M, c->Lw[0], (long)c->Mp, M);
  }
  int cur = 0;
  const int nt = c->nb64 * (c->nb64 + 1) / 2;
  for (int s = 0; s < n_ng; ++s) {
    { Timed t(c, KK_NG_Y); HIPCK(Ops<T>::ng_Y(c, c->Lw[cur], c->Y)); }
    { Timed t(c, KK_NG_W); HIPCK(Ops<T>::ng_W(c, c->Lw[cur])); }
    { Timed t(c, KK_NG_L); HIPCK(Ops<T>::ng_L(c, c->Lw[cur], c->Lw[1 - cur], gammas[s])); }
    {
      Timed t(c, KK_RESID);
      hipLaunchKernelGGL(k_resid, dim3(1), dim3(NTB), 0, c->st, (const double *)c->tp_ng, nt, M,
                         out_resid ? out_resid + s : (double *)nullptr, c->scal);
    }
    cur = 1 - cur;
  }
  c->cur_L = cur;
  HIPCK(hipGetLastError());
  return IFSVGP_OK;
}

template <typename T>
static int stage_bound(ifsvgp_ctx *c, const float *X, const float *y, int B, double N,
                       const float *sf2, const float *noise, const float *m, const float *s,
                       double *out_bound, double *out_terms) {
  const int M = c->M, D = c->D;
  const float *L = c->Lw[c->cur_L];
  const long Mp = c->Mp;
  { Timed t(c, KK_GR_Y); HIPCK(Ops<T>::ng_Y(c, L, c->Y)); }
  { Timed t(c, KK_GR_W); HIPCK(Ops<T>::gr_W(c, L)); }
  { Timed t(c, KK_GR_E); HIPCK(Ops<T>::gr_E(c, L, s)); }
  {
    Timed t(c, KK_VEC);
    const int nch = cdiv(M, 64);
    // a = L^T m~
    hipLaunchKernelGGL(k_gemv_cols_part, dim3(cdiv(M, NTB), nch), dim3(NTB), 0, c->st, L, Mp, M,
                       M, m, 1, c->vpart, Mp);
    hipLaunchKernelGGL(k_sum_parts, dim3(cdiv(M, NTB)), dim3(NTB), 0, c->st,
                       (const float *)c->vpart, Mp, nch, M, c->va);
    // b = Q a
    hipLaunchKernelGGL(k_gemv_rows<float>, dim3(cdiv(M, NTB / 64)), dim3(NTB), 0, c->st,
                       (const float *)c->Q, Mp, M, M, (const float *)c->va, 0, 1.f,
                       (const float *)nullptr, 0.f, c->vb);
    // Lb = L b
    hipLaunchKernelGGL(k_gemv_rows<float>, dim3(cdiv(M, NTB / 64)), dim3(NTB), 0, c->st, L, Mp, M,
                       M, (const float *)c->vb, 1, 1.f, (const float *)nullptr, 0.f, c->vLb);
    // Wub = Wu b
    hipLaunchKernelGGL(k_gemv_rows<float>, dim3(cdiv(M, NTB / 64)), dim3(NTB), 0, c->st,
                       (const float *)c->Wu, Mp, M, M, (const float *)c->vb, 0, 1.f,
                       (const float *)nullptr, 0.f, c->vWub);
    hipLaunchKernelGGL(k_kl_scalars, dim3(1), dim3(NTB), 0, c->st, (const float *)c->vb,
                       (const float *)c->vWub, L, Mp, M, c->scal, c->flag);
  }
  {
    Timed t(c, KK_KUF);
    hipLaunchKernelGGL(k_scale_rows, dim3(grid1((long)B * D)), dim3(NTB), 0, c->st, X, B, D,
                       (const float *)c->inv_ell, c->Xs);
    hipLaunchKernelGGL((k_kuf<MAXD, T>), dim3(cdiv(B, 64), cdiv(M, 64)), dim3(NTB), 0, c->st,
                       (const float *)c->Zs, (const float *)c->Xs, M, B, D, sf2,
                       (const float *)c->vLb, (T *)c->Kuf, (long)c->Bp, c->mu_part,
                       (long)c->Bp);
  }
  { Timed t(c, KK_V); HIPCK(Ops<T>::gemm_V(c, L, B)); }
  { Timed t(c, KK_U); HIPCK(Ops<T>::gemm_U(c, B)); }
  const int nlik = cdiv(B, NTB);
  {
    Timed t(c, KK_LIK);
    LikArgs a{c->mu_part, cdiv(M, 64), c->var_part, cdiv(M, 128), (long)c->Bp,
              y, B, sf2, noise, N / (double)B, c->lik, c->gh, c->ngh,
              c->mu, c->var, c->alpha, c->beta, c->sqnb, c->lik_part};
    hipLaunchKernelGGL(k_lik, dim3(nlik), dim3(NTB), 0, c->st, a);
  }
  {
    Timed t(c, KK_FIN);
    const int nt = c->nb64 * (c->nb64 + 1) / 2;
    hipLaunchKernelGGL(k_finalize_bound, dim3(1), dim3(NTB), 0, c->st,
                       (const double *)c->tp_gram, nt, (const double *)c->lik_part, nlik,
                       (const double *)c->scal, M, N / (double)B, out_bound, out_terms, c->flag);
  }
  HIPCK(hipGetLastError());
  c->fwd_valid = 1;
  c->fwd_B = B;
  return IFSVGP_OK;
}

template <typename T>
static int stage_backward(ifsvgp_ctx *c, int B, double N, const float *sf2, const float *s,
                          const double *grad_scale, float *g_ell, float *g_sf2, float *g_noise,
                          float *g_Z, float *g_m) {
  const int M = c->M, D = c->D;
  const float *L = c->Lw[c->cur_L];
  const long Mp = c->Mp;
  { Timed t(c, KK_R); HIPCK(Ops<T>::gemm_R(c, L, B, sf2)); }
  {
    Timed t(c, KK_VALPHA);
    hipLaunchKernelGGL(k_valpha<T>, dim3(cdiv(M, NTB / 64)), dim3(NTB), 0, c->st,
                       (const T *)c->V, (long)c->Bp, M, B, (const float *)c->alpha, c->vVa);
  }
  { Timed t(c, KK_SYRK); HIPCK(Ops<T>::syrk(c, B)); }
  {
    Timed t(c, KK_ASM);
    const int ns = std::max(1, std::min(c->nsplit, cdiv(B, Ops<T>::CS::BK)));
    hipLaunchKernelGGL(k_assemble_C, dim3(grid1((long)M * M)), dim3(NTB), 0, c->st,
                       (const float *)c->Ys, ns, (long)M * Mp, (const float *)c->Wu,
                       (const float *)c->Q, (const float *)c->va, (const float *)c->vb,
                       (const float *)c->vWub, (const float *)c->vVa, M, Mp, c->Cm);
  }
  { Timed t(c, KK_Y2); HIPCK(Ops<T>::gemm_Y2(c, L)); }
  { Timed t(c, KK_GUU); HIPCK(Ops<T>::gemm_Guu(c, L, s)); }
  {
    Timed t(c, KK_GRAD);
    const int rb = cdiv(M, 64), cb = cdiv(B, 64);
    GradArgs g{M, B, D, c->Zs, c->Xs, c->inv_ell, sf2,
               c->hrow, cdiv(B, 128), c->hx, c->hcol, cdiv(M, 128), (long)c->Bp,
               c->hzrow, c->hz, c->nb64,
               c->tp_uf, cdiv(M, 128) * cdiv(B, 128), c->tp_uu, c->nb64 * (c->nb64 + 1) / 2,
               c->lik_part, cdiv(B, NTB), N / (double)B, grad_scale,
               g_Z, g_ell, g_sf2, g_noise, c->ell_part};
    hipLaunchKernelGGL(k_grad_rows, dim3(rb), dim3(NTB), 0, c->st, g);
    hipLaunchKernelGGL(k_grad_cols, dim3(cb), dim3(NTB), 0, c->st, g, rb);
    hipLaunchKernelGGL(k_grad_final, dim3(1), dim3(NTB), 0, c->st, g, rb + cb);
    if (g_m) {
      // dF/dm~ = L Q (V alpha - Wu b)
      hipLaunchKernelGGL(k_sub_vec, dim3(cdiv(M, NTB)), dim3(NTB), 0, c->st,
                         (const float *)c->vVa, (const float *)c->vWub, M, c->vt1);
      hipLaunchKernelGGL(k_gemv_rows<float>, dim3(cdiv(M, NTB / 64)), dim3(NTB), 0, c->st,
                         (const float *)c->Q, Mp, M, M, (const float *)c->vt1, 0, 1.f,
                         (const float *)nullptr, 0.f, c->vt2);
      hipLaunchKernelGGL(k_gemv_rows<float>, dim3(cdiv(M, NTB / 64)), dim3(NTB), 0, c->st, L,
                         Mp, M, M, (const float *)c->vt2, 1, 1.f, (const float *)nullptr, 0.f,
                         c->vt1);
      hipLaunchKernelGGL(k_scale_vec, dim3(cdiv(M, NTB)), dim3(NTB), 0, c->st,
                         (const float *)c->vt1, M, grad_scale, g_m);
    }
  }
  HIPCK(hipGetLastError());
  return IFSVGP_OK;
}

// ------------------------------------------------------------------ API: compute
static bool bad_common(ifsvgp_ctx *c, const float *ell, const float *sf2, const float *Z,
                       const float *s, const float *L) {
  return !c || !ell || !sf2 || !Z || !s || !L;
}

template <typename T>
static int do_natgrad(ifsvgp_ctx *c, const float *Z, const float *ell, const float *sf2,
                      const float *s, float *L, const float *gammas, int n_ng, double *out_resid) {
  int r = stage_kernel_blocks(c, Z, ell, sf2, nullptr, s, 0);
  if (r) return r;
  r = stage_natgrad<T>(c, L, gammas, n_ng, out_resid);
  if (r) return r;
  Timed t(c, KK_STOREL);
  hipLaunchKernelGGL(k_store_lower, dim3(grid1((long)c->M * c->M)), dim3(NTB), 0, c->st,
                     (const float *)c->Lw[c->cur_L], (long)c->Mp, L, (long)c->M, c->M);
  HIPCK(hipGetLastError());
  c->fwd_valid = 0;
  return IFSVGP_OK;
}

extern "C" int ifsvgp_natgrad(ifsvgp_ctx *c, const float *Z, const float *ell, const float *sf2,
                              const float *s_tilde, float *L, const float *gammas, int n_ng,
                              double *out_resid) {
  if (bad_common(c, ell, sf2, Z, s_tilde, L) || !gammas || n_ng < 1) return IFSVGP_EINVAL;
  switch (c->prec) {
    case IFSVGP_PREC_FP32: return do_natgrad<float>(c, Z, ell, sf2, s_tilde, L, gammas, n_ng, out_resid);
    case IFSVGP_PREC_BF16: return do_natgrad<__bf16>(c, Z, ell, sf2, s_tilde, L, gammas, n_ng, out_resid);
    default: return do_natgrad<_Float16>(c, Z, ell, sf2, s_tilde, L, gammas, n_ng, out_resid);
  }
}

static int check_bound_args(ifsvgp_ctx *c, const float *X, const float *y, int B, double N,
                            const float *ell, const float *sf2, const float *noise,
                            const float *Z, const float *m, const float *s, const float *L) {
  if (bad_common(c, ell, sf2, Z, s, L) || !X || !y || !m) return IFSVGP_EINVAL;
  if (B < 1 || B > c->Bmax || !(N > 0.0)) return IFSVGP_EINVAL;
  if (c->lik == IFSVGP_LIK_GAUSSIAN && !noise) return IFSVGP_EINVAL;
  return IFSVGP_OK;
}

template <typename T>
static int do_step(ifsvgp_ctx *c, const float *X, const float *y, int B, double N,
                   const float *ell, const float *sf2, const float *noise, const float *Z,
                   const float *m, const float *s, float *L, const float *gammas, int n_ng,
                   double *out_bound, double *out_terms, double *out_resid, bool fwd, bool bwd,
                   const double *grad_scale, float *g_ell, float *g_sf2, float *g_noise,
                   float *g_Z, float *g_m) {
  const int need_noise = c->lik == IFSVGP_LIK_GAUSSIAN;
  int r;
  if (fwd) {
    r = stage_kernel_blocks(c, Z, ell, sf2, noise, s, need_noise);
    if (r) return r;
    r = stage_natgrad<T>(c, L, gammas, n_ng, out_resid);
    if (r) return r;
    r = stage_bound<T>(c, X, y, B, N, sf2, noise, m, s, out_bound, out_terms);
    if (r) return r;
  }
  if (bwd) {
    if (!c->fwd_valid || c->fwd_B != B) return IFSVGP_ESTATE;
    r = stage_backward<T>(c, B, N, sf2, s, grad_scale, g_ell, g_sf2, g_noise, g_Z, g_m);
    if (r) return r;
  }
  if (fwd && n_ng > 0) {
    Timed t(c, KK_STOREL);
    hipLaunchKernelGGL(k_store_lower, dim3(grid1((long)c->M * c->M)), dim3(NTB), 0, c->st,
                       (const float *)c->Lw[c->cur_L], (long)c->Mp, L, (long)c->M, c->M);
    HIPCK(hipGetLastError());
  }
  return IFSVGP_OK;
}

template <typename T>
static int bound_impl(ifsvgp_ctx *c, const float *X, const float *y, int B, double N,
                      const float *ell, const float *sf2, const float *noise, const float *Z,
                      const float *m, const float *s, const float *L, double *out_bound,
                      double *out_terms) {
  return do_step<T>(c, X, y, B, N, ell, sf2, noise, Z, m, s, (float *)L, nullptr, 0, out_bound,
                    out_terms, nullptr, true, false, nullptr, nullptr, nullptr, nullptr, nullptr,
                    nullptr);
}

extern "C" int ifsvgp_bound(ifsvgp_ctx *c, const float *X, const float *y, int B, double N,
                            const float *ell, const float *sf2, const float *noise,
                            const float *Z, const float *m, const float *s, const float *L,
                            double *out_bound, double *out_terms) {
  int r = check_bound_args(c, X, y, B, N, ell, sf2, noise, Z, m, s, L);
  if (r) return r;
  if (!out_bound) return IFSVGP_EINVAL;
  switch (c->prec) {
    case IFSVGP_PREC_FP32: return bound_impl<float>(c, X, y, B, N, ell, sf2, noise, Z, m, s, L, out_bound, out_terms);
    case IFSVGP_PREC_BF16: return bound_impl<__bf16>(c, X, y, B, N, ell, sf2, noise, Z, m, s, L, out_bound, out_terms);
    default: return bound_impl<_Float16>(c, X, y, B, N, ell, sf2, noise, Z, m, s, L, out_bound, out_terms);
  }
}

extern "C" int ifsvgp_bound_bwd(ifsvgp_ctx *c, const float *X, const float *y, int B, double N,
                                const float *ell, const float *sf2, const float *noise,
                                const float *Z, const float *m, const float *s, const float *L,
                                const double *grad_scale, float *g_ell, float *g_sf2,
                                float *g_noise, float *g_Z, float *g_m, float *g_s) {
  int r = check_bound_args(c, X, y, B, N, ell, sf2, noise, Z, m, s, L);
  if (r) return r;
  if (g_s) return IFSVGP_EINVAL;  // gradient w.r.t. s~ not provided by this build
  switch (c->prec) {
    case IFSVGP_PREC_FP32:
      return do_step<float>(c, X, y, B, N, ell, sf2, noise, Z, m, s, (float *)L, nullptr, 0,
                            nullptr, nullptr, nullptr, false, true, grad_scale, g_ell, g_sf2,
                            g_noise, g_Z, g_m);
    case IFSVGP_PREC_BF16:
      return do_step<__bf16>(c, X, y, B, N, ell, sf2, noise, Z, m, s, (float *)L, nullptr, 0,
                             nullptr, nullptr, nullptr, false, true, grad_scale, g_ell, g_sf2,
                             g_noise, g_Z, g_m);
    default:
      return do_step<_Float16>(c, X, y, B, N, ell, sf2, noise, Z, m, s, (float *)L, nullptr, 0,
                               nullptr, nullptr, nullptr, false, true, grad_scale, g_ell, g_sf2,
                               g_noise, g_Z, g_m);
  }
}

extern "C" int ifsvgp_step(ifsvgp_ctx *c, const float *X, const float *y, int B, double N,
                           const float *ell, const float *sf2, const float *noise,
                           const float *Z, const float *m, const float *s, float *L,
                           const float *gammas, int n_ng, double *out_bound, double *out_terms,
                           double *out_resid, float *g_ell, float *g_sf2, float *g_noise,
                           float *g_Z, float *g_m, float *g_s) {
  int r = check_bound_args(c, X, y, B, N, ell, sf2, noise, Z, m, s, L);
  if (r) return r;
  if (n_ng < 0 || (n_ng > 0 && !gammas) || !out_bound) return IFSVGP_EINVAL;
  if (g_s) return IFSVGP_EINVAL;
  switch (c->prec) {
    case IFSVGP_PREC_FP32:
      return do_step<float>(c, X, y, B, N, ell, sf2, noise, Z, m, s, L, gammas, n_ng, out_bound,
                            out_terms, out_resid, true, true, nullptr, g_ell, g_sf2, g_noise,
                            g_Z, g_m);
    case IFSVGP_PREC_BF16:
      return do_step<__bf16>(c, X, y, B, N, ell, sf2, noise, Z, m, s, L, gammas, n_ng,
                             out_bound, out_terms, out_resid, true, true, nullptr, g_ell, g_sf2,
                             g_noise, g_Z, g_m);
    default:
      return do_step<_Float16>(c, X, y, B, N, ell, sf2, noise, Z, m, s, L, gammas, n_ng,
                               out_bound, out_terms, out_resid, true, true, nullptr, g_ell,
                               g_sf2, g_noise, g_Z, g_m);
  }
}
