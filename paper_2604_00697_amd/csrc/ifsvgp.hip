// C ABI of the inverse-free SVGP training iteration (host orchestration).
// Declarations and the contract of every entry point: include/ifsvgp.h.
//
// Every product of the iteration is an NT GEMM (gemm.hpp) over zero-padded
// operands in the MFMA operand type; the context's workspace holds each
// operand in the layout its consumer reads.  Padded extents: Mp and Bp are
// M and B_max rounded up to 128.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <type_traits>
#include <vector>

#include "../../include/ifsvgp.h"
#include "kernels.hpp"
#include "epilogues.hpp"

#define IFSVGP_VERSION 200

static constexpr int MAXD = 64;  // input dimension limit of the LDS-staged kernels
static constexpr int PAD = 128;  // padding granule of every workspace extent

// ------------------------------------------------------------------ kernel kinds
enum KernelKind : int {
  KK_PREP = 0, KK_NG_Y, KK_NG_W, KK_NG_L,
  KK_GR_Y, KK_GR_W, KK_GR_E, KK_VEC, KK_KUF, KK_V, KK_U, KK_LIK,
  KK_R, KK_VALPHA, KK_SYRK, KK_ASM, KK_Y2, KK_GUU, KK_LQ, KK_GRAD, KK_N
};
static const char *KK_NAMES[KK_N] = {
    "prep", "ng_KL", "ng_gram", "ng_update",
    "bound_KL", "bound_gram", "bound_gram_E", "matvec", "kuf", "gemm_V", "gemm_U", "likelihood",
    "gemm_R_grad_uf", "valpha", "syrk", "assemble_C", "gemm_LC", "gemm_G_grad_uu",
    "gemm_LQ_diag", "grad_final"};

struct TimingRec {
  int kind;
  hipEvent_t a, b;
};

// Launch structure of a call (what a recorded graph depends on).
// stopping rule of the NG steps of a call
enum : int { NG_FIXED = 0, NG_RESID = 1, NG_GAP = 2 };

struct GraphKey {
  bool setup, fwd, bwd;
  int B, n_ng;
  bool need_noise, want_gm, want_gs;
  int adapt;
  int cur0;  // L slot a backward-only call starts from (0 otherwise)
};
struct GraphEnt {
  GraphKey key;
  hipGraphExec_t exec;  // null until the structure is seen a second time
  int failed;           // recording failed: always run directly
  int cur;              // c->cur after the call
  long long tick;       // last use (least recently used entry is replaced)
};
static constexpr size_t kMaxGraphs = 16;

struct ifsvgp_ctx {
  int M, Bmax, D, prec, lik, ngh;
  int Mp, Bp;
  int nsplit;
  hipStream_t st;
  // side stream for branches of the iteration that are independent of the
  // main chain (K_uf tiles, then V and L^T m~, during the NG and Gram
  // products; R = L U during the backward's C chain); forked from and joined
  // back into st with events
  hipStream_t side;
  static constexpr int kEvents = 16;
  hipEvent_t evs[kEvents];  // fork / join points of one call, in order
  int ev_next;
  bool side_open;           // the side stream has work not yet joined into st
  bool single_stream;       // side is st: branches run in stream order, no events
  // grouped contexts: G independent problems of the same sizes, problem g's
  // workspace at the slab's g * gstride bytes; every launch covers all G
  int G;
  long gstride;
  bool capturing;           // launches are being recorded into a graph
  // device argument block of the current call, written by its k_latch
  CallArgs *dca;
  float *sfn;  // {sf2, noise_var} copied by the set-up
  // recorded calls (HIP graphs) and the stream they are recorded on
  hipStream_t cst;
  int use_graphs;
  int kuf_mode;  // IFSVGP_KUF_*
  std::vector<GraphEnt> graphs;
  long long graph_tick;
  // fp32 M x M ([Mp][Mp])
  float *Kt, *L32[2], *Lt32[2], *W32, *Q32, *Wu32, *Ys;  // Ys: [nsplit][Mp][Mp]
  // operand-type M x M ([Mp][Mp]); C and Y2 use the wide-range type of the form
  void *KtT, *LT[2], *LtT[2], *Yt, *Xgt, *QT, *Cm, *Y2;
  void *LstT[2];  // LstT[m][k] = L[k][m] s~_k: the scaled operand of L^T S~ L
  // operand-type M x B: Kft, Vt, Ut are [Bp][Mp]; V and Vs = V diag(sqrt(-beta)) are [Mp][Bp]
  void *Kft, *V, *Vt, *Ut, *Vs;
  float *Zs, *Xs, *inv_ell, *sP;  // sP: s~ zero-padded to Mp
  // inputs of the generated K_uf tiles (bf16 / fp16 forms): hi / lo bf16
  // rows of 2 z' and x' ([Mp][gldk], [Bp][gldk]), -|z'|^2, log2 sf2 - |x'|^2
  __bf16 *gZh, *gZl, *gXh, *gXl;
  float *gzc, *gxr;
  int gldk;
  float *va, *vb, *vLb, *vWub, *vVa, *vt2;
  float *mu_part, *var_part, *mu, *var, *alpha, *beta, *sqnb;
  double *hrow, *hcol, *hx, *hzrow, *hz;  // gradient partials per tile
  float *gdiag, *pdiag;  // diag(G_uu) [Mp]; partials of diag(L Q L^T) [nb64][Mp]
  double *scal, *tp_ng, *tp_gram, *tp_uf, *tp_uu, *lik_part, *ell_part, *vec_part;
  double *tp_gap;  // per-tile partials of the variance gap [nb128][cdiv(Bp, 64)]
  float *hwx, *hex;  // Hutchinson bound: W Xc and E Omega (fp32, [Bp][Mp])
  double *hp;        // Hutchinson bound: per-probe sums [Bp][4]
  void *hxt;         // its backward: X^T of C = X S X^T, [2 Bp][Mp] operand type
  void *hy1, *hy2;   // L X and L X S, [Mp][2 Bp] wide type
  float *hx1, *hx2;  // its backward: vectors [Mp]
  int fwd_K;         // probes of the last Hutchinson forward
  // multi-output: per-output vectors [MO_QMAX][Mp] (a = L^T m~_q, b = Q a,
  // Wu b, x = V alpha_q - Wu b, t2 = Q x) and [MO_QMAX][Bp] (mu, dF/dmu),
  // a zero [Mp] and a -1/2 [Bp] vector for the R epilogue
  float *mo_m, *mo_a, *mo_b, *mo_wub, *mo_x, *mo_t2, *mo_mu, *mo_al, *mo_zero, *mo_half;
  int fwd_Q;
  double *gh;
  int *flag, *counters;
  int *ngskip;  // stop flag of an adaptive NG loop
  // last forward state for the backward: 1 exact bound, 2 Hutchinson bound,
  // 3 multi-output bound
  int fwd_valid, fwd_B;
  int cur;  // which L32/LT/LtT slot holds the bound's L
  // timing
  long long timing;  // bit mask of timed kernel kinds
  hipEvent_t lev0, lev1;  // dispatch-stamped events of the next GEMM launch (timing)
  std::vector<TimingRec> recs;
  std::vector<hipEvent_t> pool;
  double t_ms[KK_N];
  long t_cnt[KK_N];
  std::vector<void *> allocs;
};

// ------------------------------------------------------------------ helpers
static inline int rup(int x, int m) { return (x + m - 1) / m * m; }
static inline int cdiv(long x, long m) { return (int)((x + m - 1) / m); }
static int grid1(long n) {
  return (int)std::min<long>(std::max<long>(1, (n + NTB - 1) / NTB), 65536);
}

#define HIPCK(x)                                      \
  do {                                                \
    hipError_t _e = (x);                              \
    if (_e != hipSuccess) return IFSVGP_EHIP;         \
  } while (0)

// Kinds that are exactly one GEMM launch: timed by events the dispatch
// stamps itself (kernel start to kernel end); other kinds are bracketed by
// recorded events.
static bool single_gemm_kind(int k) {
  switch (k) {
    case KK_NG_Y: case KK_NG_W: case KK_NG_L: case KK_GR_Y: case KK_GR_W: case KK_GR_E:
    case KK_V: case KK_U: case KK_R: case KK_SYRK: case KK_Y2: case KK_GUU: case KK_LQ:
      return true;
    default:
      return false;
  }
}

struct Timed {
  ifsvgp_ctx *c;
  int kind;
  hipEvent_t b;
  bool stamped;
  Timed(ifsvgp_ctx *c_, int k) : c(c_), kind(k), b(nullptr), stamped(false) {
    if (!((c->timing >> kind) & 1)) return;
    hipEvent_t a = get();
    b = get();
    stamped = single_gemm_kind(kind);
    if (stamped) {
      c->lev0 = a;
      c->lev1 = b;
    } else {
      hipEventRecord(a, c->st);
    }
    c->recs.push_back({kind, a, b});
  }
  ~Timed() {
    if (!b) return;
    if (stamped) c->lev0 = c->lev1 = nullptr;
    else hipEventRecord(b, c->st);
  }
  hipEvent_t get() {
    if (!c->pool.empty()) {
      hipEvent_t e = c->pool.back();
      c->pool.pop_back();
      return e;
    }
    // timing only: no system-scope fence when the event is reached, so the
    // stamps do not add a cache write-back to the launches they time
    hipEvent_t e;
    hipEventCreateWithFlags(&e, hipEventDisableSystemFence);
    return e;
  }
};

// Side-stream branches.  fork_side makes the side stream wait for all work
// enqueued on st so far; join_side makes st wait for all work enqueued on the
// side stream so far; OnSide redirects the enqueues of its scope (kernels and
// timing events) to the side stream.  In direct execution a branch also
// follows the side stream's earlier work in stream order.  While launches are
// recorded into a graph, a fork first joins the side stream's open work, so
// that every recorded branch depends exactly on its fork point.  Every fork
// and join point of a call uses its own event.
static hipEvent_t next_event(ifsvgp_ctx *c) {
  hipEvent_t e = c->evs[c->ev_next % ifsvgp_ctx::kEvents];
  ++c->ev_next;
  return e;
}
static hipError_t join_side(ifsvgp_ctx *c) {
  if (!c->side_open) return hipSuccess;
  hipEvent_t ev = next_event(c);
  hipError_t e = hipEventRecord(ev, c->side);
  if (e == hipSuccess) e = hipStreamWaitEvent(c->st, ev, 0);
  c->side_open = false;
  return e;
}
static hipError_t fork_side(ifsvgp_ctx *c) {
  if (c->single_stream) return hipSuccess;
  hipError_t e = c->capturing ? join_side(c) : hipSuccess;
  if (e != hipSuccess) return e;
  hipEvent_t ev = next_event(c);
  e = hipEventRecord(ev, c->st);
  if (e == hipSuccess) e = hipStreamWaitEvent(c->side, ev, 0);
  c->side_open = true;
  return e;
}
struct OnSide {
  ifsvgp_ctx *c;
  hipStream_t saved;
  explicit OnSide(ifsvgp_ctx *c_) : c(c_), saved(c_->st) {
    if (!c->single_stream) c->st = c->side;
  }
  ~OnSide() { c->st = saved; }
};

// bytes of the MFMA operand type and of the wide-range type used for the two
// products with the backward matrix C (fp16 would overflow there, so the
// fp16 form runs them in fp32)
static size_t op_size(int prec) { return prec == IFSVGP_PREC_FP32 ? 4 : 2; }
static size_t wide_size(int prec) { return prec == IFSVGP_PREC_BF16 ? 2 : 4; }

// ------------------------------------------------------------------ workspace layout
// Every workspace buffer of a context is carved, 256-byte aligned, from one
// slab.  layout() assigns the pointers from `base` (null: only count) and
// returns the slab's size in bytes for (M, B_max, D, prec, lik).  extras
// adds the buffers of the Hutchinson bound and its gradient; without them
// the slab serves the training iteration, its split entry points and the
// multi-output layer only (their pointers are left null).
struct Carve {
  char *base;
  size_t off;
  void *bytes(size_t n) {
    void *p = base ? (void *)(base + off) : nullptr;
    off += (std::max<size_t>(n, 16) + 255) / 256 * 256;
    return p;
  }
  template <typename T>
  void take(T *&p, size_t n) { p = (T *)bytes(n * sizeof(T)); }
};

static size_t layout(ifsvgp_ctx *c, char *base, bool extras) {
  Carve w{base, 0};
  const int M = c->M, B_max = c->Bmax, D = c->D, prec = c->prec;
  const size_t Mp = c->Mp, Bp = c->Bp;
  const size_t MM = Mp * Mp, MB = Mp * Bp;
  const size_t os = op_size(prec), ws = wide_size(prec);
  const bool f32 = prec == IFSVGP_PREC_FP32;
  const int nb64 = cdiv(M, 64), nb128 = cdiv(M, 128), nbB = cdiv(B_max, 128);
  const int nt_sym64 = nb64 * (nb64 + 1) / 2;
  w.take(c->Kt, MM);
  w.take(c->L32[0], MM);
  w.take(c->L32[1], MM);
  w.take(c->W32, MM);
  w.take(c->Q32, MM);
  w.take(c->Wu32, MM);
  w.take(c->Ys, MM * c->nsplit);
  if (f32) {
    c->KtT = c->Kt; c->LT[0] = c->L32[0]; c->LT[1] = c->L32[1]; c->QT = c->Q32;
  } else {
    c->KtT = w.bytes(MM * os);
    c->LT[0] = w.bytes(MM * os);
    c->LT[1] = w.bytes(MM * os);
    c->QT = w.bytes(MM * os);
  }
  c->LtT[0] = w.bytes(MM * os);
  c->LtT[1] = w.bytes(MM * os);
  c->LstT[0] = w.bytes(MM * os);
  c->LstT[1] = w.bytes(MM * os);
  if (f32) {
    c->Lt32[0] = (float *)c->LtT[0];
    c->Lt32[1] = (float *)c->LtT[1];
  } else {
    w.take(c->Lt32[0], MM);
    w.take(c->Lt32[1], MM);
  }
  c->Yt = w.bytes(MM * os);
  c->Xgt = w.bytes(MM * os);
  c->Cm = w.bytes(MM * ws);
  c->Y2 = w.bytes(MM * ws);
  c->Kft = w.bytes(MB * os);
  c->V = w.bytes(MB * os);
  c->Vt = w.bytes(MB * os);
  c->Ut = w.bytes(MB * os);
  c->Vs = w.bytes(MB * os);
  c->gldk = D <= 16 ? 16 : 32 * cdiv(D, 32);
  c->gZh = (__bf16 *)w.bytes(Mp * c->gldk * 2);
  c->gZl = (__bf16 *)w.bytes(Mp * c->gldk * 2);
  c->gXh = (__bf16 *)w.bytes(Bp * c->gldk * 2);
  c->gXl = (__bf16 *)w.bytes(Bp * c->gldk * 2);
  w.take(c->gzc, Mp);
  w.take(c->gxr, Bp);
  w.take(c->Zs, (size_t)M * D);
  w.take(c->Xs, (size_t)B_max * D);
  w.take(c->inv_ell, (size_t)D);
  w.take(c->sP, Mp);
  w.take(c->va, Mp);
  w.take(c->vb, Mp);
  w.take(c->vLb, Mp);
  w.take(c->vWub, Mp);
  w.take(c->vVa, Mp);
  w.take(c->vt2, Mp);
  w.take(c->mu_part, (size_t)nb64 * Bp);
  w.take(c->var_part, (size_t)nb128 * Bp);
  w.take(c->mu, Bp);
  w.take(c->var, Bp);
  w.take(c->alpha, Bp);
  w.take(c->beta, Bp);
  w.take(c->sqnb, Bp);
  w.take(c->hrow, (size_t)nbB * M);
  w.take(c->hcol, (size_t)nb128 * Bp);
  w.take(c->hx, (size_t)nbB * M * D);
  w.take(c->hzrow, (size_t)nb64 * M);
  w.take(c->hz, (size_t)nb64 * M * D);
  w.take(c->gdiag, Mp);
  w.take(c->pdiag, (size_t)nb64 * Mp);
  w.take(c->scal, (size_t)S_NSLOT);
  w.take(c->tp_ng, (size_t)nt_sym64);
  w.take(c->tp_gram, (size_t)3 * nt_sym64);
  w.take(c->tp_uf, (size_t)nb128 * nbB);
  w.take(c->tp_uu, (size_t)nt_sym64);
  w.take(c->tp_gap, (size_t)nb128 * cdiv(Bp, 64));
  w.take(c->mo_m, (size_t)MO_QMAX * Mp);
  w.take(c->mo_a, (size_t)MO_QMAX * Mp);
  w.take(c->mo_b, (size_t)MO_QMAX * Mp);
  w.take(c->mo_wub, (size_t)MO_QMAX * Mp);
  w.take(c->mo_x, (size_t)MO_QMAX * Mp);
  w.take(c->mo_t2, (size_t)MO_QMAX * Mp);
  w.take(c->mo_mu, (size_t)MO_QMAX * Bp);
  w.take(c->mo_al, (size_t)MO_QMAX * Bp);
  w.take(c->mo_zero, Mp);
  w.take(c->mo_half, Bp);
  w.take(c->lik_part, (size_t)4 * cdiv(Bp, NTB));
  w.take(c->vec_part, (size_t)2 * cdiv(2 * M, NTB / 64));
  w.take(c->ell_part, (size_t)(M + B_max + 64) * D);
  w.take(c->gh, (size_t)2 * std::max(1, c->ngh));
  w.take(c->flag, (size_t)1);
  w.take(c->counters, (size_t)CNT_N);
  w.take(c->dca, (size_t)1);
  w.take(c->ngskip, (size_t)1);
  w.take(c->sfn, (size_t)2);
  if (extras) {
    w.take(c->hwx, MB);
    w.take(c->hex, MB);
    w.take(c->hp, (size_t)4 * Bp);
    c->hxt = w.bytes(2 * MB * os);
    c->hy1 = w.bytes(2 * MB * ws);
    c->hy2 = w.bytes(2 * MB * ws);
    w.take(c->hx1, Mp);
    w.take(c->hx2, Mp);
  } else {
    c->hwx = c->hex = nullptr;
    c->hp = nullptr;
    c->hxt = c->hy1 = c->hy2 = nullptr;
    c->hx1 = c->hx2 = nullptr;
  }
  return w.off;
}

// ------------------------------------------------------------------ GH rule (host)
// Physicists' Gauss-Hermite rule: nodes are the roots of H_n, found by Newton's
// method on the orthonormal three-term recurrence
//   p_k(t) = sqrt(2/k) t p_{k-1}(t) - sqrt((k-1)/k) p_{k-2}(t),  p_0 = pi^{-1/4},
// from asymptotic starting values; weights w = 2 / p_n'(t)^2 with
// p_n' = sqrt(2n) p_{n-1}.
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
      double p1 = pim4, p2 = 0.0;
      for (int k = 1; k <= n; ++k) {
        const double p3 = p2;
        p2 = p1;
        p1 = z * std::sqrt(2.0 / k) * p2 - std::sqrt((k - 1.0) / k) * p3;
      }
      pp = std::sqrt(2.0 * n) * p2;
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
  for (int i = 0; i < n / 2; ++i) {    // ascending order
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
    case IFSVGP_ESCRATCH:
      return "problem too large for the static workspace of ifsvgp_step_noalloc";
    default: return "unknown status code";
  }
}

static void graphs_clear(ifsvgp_ctx *c);

extern "C" void ifsvgp_destroy(ifsvgp_ctx *c) {
  if (!c) return;
  graphs_clear(c);
  if (c->cst) hipStreamDestroy(c->cst);
  if (c->side) hipStreamDestroy(c->side);
  for (auto ev : c->evs)
    if (ev) hipEventDestroy(ev);
  for (void *p : c->allocs) hipFree(p);
  for (auto &r : c->recs) {
    hipEventDestroy(r.a);
    hipEventDestroy(r.b);
  }
  for (auto e : c->pool) hipEventDestroy(e);
  delete c;
}

// G = 1: a context of one problem (every entry point); G > 1: a grouped
// context whose slab holds G problems' workspaces (the training iteration
// without the Hutchinson buffers) one stride apart.
static int create_ctx(ifsvgp_ctx **out, int G, int M, int B_max, int D, int prec, int lik,
                      int n_gh) {
  if (!out || M < 1 || B_max < 1 || D < 1 || D > MAXD) return IFSVGP_EINVAL;
  if (G < 1 || G > IFSVGP_MAX_GROUP) return IFSVGP_EINVAL;
  if (prec < 0 || prec > 2 || lik < 0 || lik > 1) return IFSVGP_EINVAL;
  if (lik == IFSVGP_LIK_PROBIT && (n_gh < 1 || n_gh > 64)) return IFSVGP_EINVAL;
  if ((long)M > 32768 || (long)B_max > (1L << 24) || (long)M * B_max > (1L << 31))
    return IFSVGP_EINVAL;
  ifsvgp_ctx *c = new (std::nothrow) ifsvgp_ctx();
  if (!c) return IFSVGP_ENOMEM;
  c->M = M; c->Bmax = B_max; c->D = D; c->prec = prec; c->lik = lik;
  c->ngh = lik == IFSVGP_LIK_PROBIT ? n_gh : 0;
  c->Mp = rup(M, PAD);
  c->Bp = rup(B_max, PAD);
  c->nsplit = std::max(1, std::min(8, cdiv(B_max, 1024)));
  c->st = nullptr;
  c->use_graphs = 0;
  c->kuf_mode = IFSVGP_KUF_IN_PRODUCT;
  c->graph_tick = 0;
  c->G = G;
  c->gstride = 0;
#ifdef IFSVGP_SERIAL_SIDE
  // profiling builds: the side branches run in order on the context's stream
  // (kernel durations without the overlap)
  c->single_stream = true;
#endif
  bool ok = hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) == hipSuccess &&
            hipStreamCreateWithFlags(&c->cst, hipStreamNonBlocking) == hipSuccess;
  // fork / join events only order the two streams on the device (each
  // kernel's own end-of-dispatch release makes its writes visible there), so
  // they skip the system-scope fence an event record otherwise performs (a
  // probe on the box: fork + join of two streams 24.9 -> 19.8 us)
  for (int k = 0; ok && k < ifsvgp_ctx::kEvents; ++k)
    ok = hipEventCreateWithFlags(&c->evs[k], hipEventDisableTiming |
                                                 hipEventDisableSystemFence) == hipSuccess;
  if (!ok) {
    ifsvgp_destroy(c);
    return IFSVGP_EHIP;
  }
  const size_t bytes = layout(c, nullptr, G == 1);
  c->gstride = G > 1 ? (long)bytes : 0;
  void *slab = nullptr;
  hipError_t e = hipMalloc(&slab, bytes * G);
  if (e == hipSuccess) {
    c->allocs.push_back(slab);
    e = hipMemset(slab, 0, bytes * G);
  }
  if (e == hipSuccess) layout(c, (char *)slab, G == 1);
  for (int g = 0; e == hipSuccess && c->ngh > 0 && g < G; ++g) {
    std::vector<double> r(2 * c->ngh);
    ifsvgp_gh_rule(c->ngh, r.data(), r.data() + c->ngh);
    e = hipMemcpy((char *)c->gh + g * c->gstride, r.data(), r.size() * sizeof(double),
                  hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) {
    const int code = e == hipErrorOutOfMemory ? IFSVGP_ENOMEM : IFSVGP_EHIP;
    ifsvgp_destroy(c);
    return code;
  }
  c->fwd_valid = 0;
  c->cur = 0;
  c->timing = 0;
  for (int k = 0; k < KK_N; ++k) { c->t_ms[k] = 0.0; c->t_cnt[k] = 0; }
  *out = c;
  return IFSVGP_OK;
}

extern "C" int ifsvgp_create(ifsvgp_ctx **out, int M, int B_max, int D, int prec, int lik,
                             int n_gh) {
  return create_ctx(out, 1, M, B_max, D, prec, lik, n_gh);
}

extern "C" int ifsvgp_create_group(ifsvgp_ctx **out, int G, int M, int B_max, int D, int prec,
                                   int lik, int n_gh) {
  return create_ctx(out, G, M, B_max, D, prec, lik, n_gh);
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
  for (int g = 0; g < std::max(1, c->G); ++g) {  // every problem of a grouped context
    int *fl = (int *)((char *)c->flag + g * c->gstride), v = 0, z = 0;
    HIPCK(hipMemcpy(&v, fl, sizeof(int), hipMemcpyDeviceToHost));
    HIPCK(hipMemcpy(fl, &z, sizeof(int), hipMemcpyHostToDevice));
    f |= v;
  }
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
  f[KK_NG_Y] = 2.0 * M * M * M / 3.0;   // lower part of K~ L: sum_{l>=j} for k>=j
  f[KK_NG_W] = M * M * M / 3.0;         // lower part of L^T Y
  f[KK_NG_L] = M * M * M / 3.0;         // L X, both lower triangular
  f[KK_GR_Y] = 2.0 * M * M * M / 3.0;
  f[KK_GR_W] = M * M * M / 3.0;
  f[KK_GR_E] = M * M * M / 3.0;
  f[KK_V] = M * M * Bd;                 // L^T K_uf, triangular
  f[KK_U] = 2.0 * M * M * Bd;           // Q V
  f[KK_R] = M * M * Bd + 4.0 * M * Bd * D;  // L U, + K_uf cross term and H [Xs | 1]
  f[KK_SYRK] = M * M * Bd;              // lower half of (V D)(V D)^T
  f[KK_Y2] = M * M * M;                 // L C
  f[KK_GUU] = M * M * M / 3.0 + 2.0 * M * M * D;  // lower half of Y2 L^T (+ H Z)
  f[KK_LQ] = M * M * M / 3.0;           // lower tiles of L Q (only with the s~ gradient)
  f[KK_KUF] = 2.0 * M * Bd * D;         // cross term Zs Xs^T (MFMA)
  f[KK_PREP] = 3.0 * M * M * D;         // K~ from differences (VALU)
  for (int k = 0; k < KK_N && k < cap; ++k) {
    flops[k] = f[k];
    if (names) names[k] = KK_NAMES[k];
  }
  return KK_N;
}

// ------------------------------------------------------------------ GEMM wrappers
static Launch lnc(ifsvgp_ctx *c) { return Launch{c->st, c->lev0, c->lev1, c->G, c->gstride}; }
// grid of a launch covering the context's G problems, and their workspace stride
static dim3 gdim(ifsvgp_ctx *c, dim3 d) {
  d.z = std::max(1, c->G);
  return d;
}
static long gsz(ifsvgp_ctx *c) { return c->G > 1 ? c->gstride : 0; }

// The exact bound's likelihood arguments (partials of U's epilogue, the Gram
// products' trace partials, the vector kernel's quad / log|T| partials).
static LikArgs lik_args(ifsvgp_ctx *c, int B, long gs, int defer_final = 0) {
  const int M = c->M, nb = cdiv(M, 64);
  return LikArgs{c->mu_part, cdiv(M, 128), c->var_part, cdiv(M, 128), (long)c->Bp,
                 c->dca, B, c->Bp, c->sfn, c->lik, c->gh, c->ngh,
                 c->mu, c->var, c->alpha, c->beta, c->sqnb, c->lik_part,
                 c->tp_gram, nb * (nb + 1) / 2, c->vec_part, cdiv(2 * M, NTB / 64),
                 c->scal, M, c->flag, c->counters + CNT_LIK, gs, defer_final};
}

// element type of the per-tile gradient partials (the epilogues' P)
template <typename T>
using GradPartial = typename std::conditional<std::is_same<T, float>::value, double, float>::type;

template <typename T>
struct Ops {
  // TW: operand type of the two products with C (fp32 in the fp16 form)
  using TW = typename std::conditional<std::is_same<T, _Float16>::value, float, T>::type;
  // M x M products: three stages (48 KB) give two k-steps of load lookahead
  // and still leave room for three workgroups per CU
  using CS = Cfg<64, 64, 2, 2, T, 3>;
  using CSW = Cfg<64, 64, 2, 2, TW, 3>;
  // Gram products Y = K~ L and W = L^T Y (NG step and bound): after the NG
  // step W is within rounding of I, and the bound and its gradient depend on
  // I - W and on Q = 2I - W, so the fp32 form sums these two products on the
  // fp64 matrix cores (fp32 operands, one rounding of the result) instead of
  // letting M-long fp32 sums of terms of size ||L||^2 ||K~|| set their error
  static constexpr bool kA64 = std::is_same<T, float>::value;
  using CG = Cfg<64, 64, 2, 2, T, 3, kA64>;
  // M x B products, two stages.  CR: V and U on 128 x 64 tiles (twice the
  // workgroups of 128 x 128, so several share a CU and one's epilogue overlaps
  // another's main loop; their partial sums are per 128-row block).  CRG: R on
  // 128 x 128 tiles, whose gradient partials are per 128-column block.
  using CR = Cfg<128, 64, 2, 2, T, 2>;
  // (the fp32 form sums R = L U on the fp64 matrix cores too: R = P K_uf is
  // formed from terms of size ||L||^2 ||K_uf||, so its fp32 sums would set the
  // error of the H_uf reductions; eight waves keep the fp64 accumulators in
  // registers)
  using CRG = typename std::conditional<kA64, Cfg<128, 128, 2, 4, T, 2, true>,
                                        Cfg<128, 128, 2, 2, T, 2>>::type;
  // Ys = (V D)(V D)^T: lower tiles, split-K over the batch
  using CSY = Cfg<64, 64, 2, 2, T, 3>;
  using CH = Cfg<64, 64, 2, 2, T, 3>;  // the Hutchinson bound's thin products
  static_assert(CR::BM == 128 && CRG::BM == 128 && CRG::BN == 128, "partial-sum layout");

  static T *LT(ifsvgp_ctx *c, int i) { return (T *)c->LT[i]; }
  static T *LtT(ifsvgp_ctx *c, int i) { return (T *)c->LtT[i]; }
  static TW *LW(ifsvgp_ctx *c, int i) {
    return std::is_same<TW, T>::value ? (TW *)c->LT[i] : (TW *)c->L32[i];
  }
  static int nb(ifsvgp_ctx *c) { return cdiv(c->M, 64); }

  // Y = K~ L on lower tiles (k >= n0), stored transposed: Yt[j][i] = Y[i][j]
  static hipError_t gram_Y(ifsvgp_ctx *c, int cur, const int *skip = nullptr) {
    Opnd<T> a{(const T *)c->KtT, c->Mp}, b{LtT(c, cur), c->Mp};
    Sched sc{nb(c), nb(c), 1, 1, c->M, K_LO_N0, skip};
    EpiStoreT<T> e{(T *)c->Yt, c->Mp, c->M, c->M};
    return launch_gemm<CG>(lnc(c), a, b, sc, e);
  }
  // W = L^T Y on lower tiles (k >= m0) -> natural-gradient factor + residual
  static hipError_t ng_W(ifsvgp_ctx *c, int cur, const int *skip = nullptr) {
    Opnd<T> a{LtT(c, cur), c->Mp}, b{(const T *)c->Yt, c->Mp};
    Sched sc{nb(c), nb(c), 1, 1, c->M, K_LO_M0, skip};
    EpiNgGram<T> e{(T *)c->Xgt, c->Mp, c->M, c->tp_ng};
    return launch_gemm<CG>(lnc(c), a, b, sc, e);
  }
  // Lnew = L - gamma L X on lower tiles, n0 <= k < m0+BM, gamma the call's
  // step size gidx; also the residual of NG step `step` (unless a check
  // kernel forms it: skip non-null, the adaptive loop) and (write_out) the
  // caller's L
  static hipError_t ng_L(ifsvgp_ctx *c, int cur, int nxt, int gidx, int step, int write_out,
                         const int *skip = nullptr) {
    Opnd<T> a{LT(c, cur), c->Mp}, b{(const T *)c->Xgt, c->Mp};
    Sched sc{nb(c), nb(c), 1, 1, c->M, K_LO_N0 | K_HI_M1, skip};
    EpiNgUpdate<T> e{c->L32[cur], c->L32[nxt], c->Lt32[nxt], LT(c, nxt), LtT(c, nxt),
                     c->sP, (T *)c->LstT[nxt], c->Mp, c->M, c->dca, gidx, step, write_out,
                     skip ? 0 : 1, c->tp_ng, nb(c) * (nb(c) + 1) / 2, c->scal};
    return launch_gemm<CS>(lnc(c), a, b, sc, e);
  }
  // W' = L^T Y (lower tiles, fp32)
  static hipError_t gr_W(ifsvgp_ctx *c, int cur) {
    Opnd<T> a{LtT(c, cur), c->Mp}, b{(const T *)c->Yt, c->Mp};
    Sched sc{nb(c), nb(c), 1, 1, c->M, K_LO_M0};
    EpiStore<float> e{c->W32, c->Mp, c->M, c->M, 0, 0};
    return launch_gemm<CG>(lnc(c), a, b, sc, e);
  }
  // E' = L^T diag(s) L (lower tiles) -> Q, Wu, gram partials
  static hipError_t gr_E(ifsvgp_ctx *c, int cur) {
    Opnd<T> a{(const T *)c->LstT[cur], c->Mp}, b{LtT(c, cur), c->Mp};
    Sched sc{nb(c), nb(c), 1, 1, c->M, K_LO_M0};
    EpiBoundGram<T> e{c->W32, c->Q32, c->Wu32, (T *)c->QT, c->Mp, c->M, c->tp_gram};
    return launch_gemm<CS>(lnc(c), a, b, sc, e, CS::BM * CS::LDC * 4);
  }
  // V = L^T K_uf (k >= m0) -> V, Vt
  // V = L^T K_uf from the stored K_uf tiles; with va non-null workgroups
  // after the tiles also form va = L^T m~ from the same L
  static SideRows side_rows(ifsvgp_ctx *c, int cur, float *va) {
    return SideRows{(const float *)c->Lt32[cur], (long)c->Mp, (const CallArgs *)c->dca, va,
                    c->M, va ? cdiv(c->M, CR::NT / 64) : 0};
  }
  static hipError_t gemm_V(ifsvgp_ctx *c, int cur, int B, const int *skip = nullptr,
                           float *va = nullptr) {
    Opnd<T> a{LtT(c, cur), c->Mp}, b{(const T *)c->Kft, c->Mp};
    Sched sc{cdiv(c->M, CR::BM), cdiv(B, CR::BN), 0, 1, c->M, K_LO_M0, skip};
    EpiV<T> e{(T *)c->V, (T *)c->Vt, c->Bp, c->Mp, c->M, B};
    if (va) {
      SideOnly g;
      g.rows = side_rows(c, cur, va);
      return launch_gemm<CR>(lnc(c), a, b, sc, e, 0, g);
    }
    return launch_gemm<CR>(lnc(c), a, b, sc, e);
  }
  // the same product with the K_uf tiles generated in LDS (bf16 / fp16 forms;
  // inputs from the set-up), K_uf never stored; with va non-null workgroups
  // after the tiles also form va = L^T m~ from the same L
  template <int KW>
  static hipError_t gemm_Vf_kw(ifsvgp_ctx *c, int cur, int B, float *va) {
    using G = KufGen<T, KW>;
    using Op = typename G::Op;
    Opnd<T> a{LtT(c, cur), c->Mp};
    Sched sc{cdiv(c->M, CR::BM), cdiv(B, CR::BN), 0, 1, c->M, K_LO_M0};
    EpiV<T> e{(T *)c->V, (T *)c->Vt, c->Bp, c->Mp, c->M, B};
    G g{(const Op *)c->gZh, (const Op *)c->gZl, c->gzc, (const Op *)c->gXh,
        (const Op *)c->gXl, c->gxr, c->M, B, side_rows(c, cur, va)};
    return launch_gemm<CR>(lnc(c), a, a, sc, e, 0, g);
  }
  // the generated K_uf tiles stored (Kft, the B operand of gemm_V) with the
  // same arithmetic as gemm_Vf's
  template <int KW>
  static hipError_t kuf_gen_kw(ifsvgp_ctx *c, int B) {
    using G = KufGen<T, KW>;
    using Op = typename G::Op;
    G g{(const Op *)c->gZh, (const Op *)c->gZl, c->gzc, (const Op *)c->gXh,
        (const Op *)c->gXl, c->gxr, c->M, B, SideRows{}};
    const int nmt = cdiv(c->M, 64), nnt = cdiv(B, 64);
    hipLaunchKernelGGL((k_kuf_gen<CR, T, KW>), gdim(c, dim3(nmt * nnt)), dim3(CR::NT), 0, c->st,
                       g, (T *)c->Kft, (long)c->Mp, nmt, gsz(c));
    return hipGetLastError();
  }
  static hipError_t kuf_gen(ifsvgp_ctx *c, int B) {
    if constexpr (std::is_same<T, float>::value) {
      return hipErrorInvalidValue;  // the fp32 form stores K_uf with k_kuf
    } else {
      switch (c->gldk) {
        case 16: return kuf_gen_kw<16>(c, B);
        case 32: return kuf_gen_kw<32>(c, B);
        default: return kuf_gen_kw<64>(c, B);
      }
    }
  }
  static hipError_t gemm_Vf(ifsvgp_ctx *c, int cur, int B, float *va) {
    if constexpr (std::is_same<T, float>::value) {
      return hipErrorInvalidValue;  // the fp32 form stores K_uf (k_kuf)
    } else {
      switch (c->gldk) {
        case 16: return gemm_Vf_kw<16>(c, cur, B, va);
        case 32: return gemm_Vf_kw<32>(c, cur, B, va);
        default: return gemm_Vf_kw<64>(c, cur, B, va);
      }
    }
  }
  // variance gap: Y = K~ L on all tiles (k >= n0), plain layout, in the Y2
  // buffer (idle outside the backward) ...
  static T *Yfull(ifsvgp_ctx *c) { return (T *)c->Y2; }
  static hipError_t gap_Y(ifsvgp_ctx *c, int cur, const int *skip) {
    Opnd<T> a{(const T *)c->KtT, c->Mp}, b{LtT(c, cur), c->Mp};
    Sched sc{nb(c), nb(c), 0, 1, c->M, K_LO_N0, skip};
    EpiStore<T> e{Yfull(c), c->Mp, c->M, c->M, 0, 0};
    return launch_gemm<CS>(lnc(c), a, b, sc, e);
  }
  // ... then (K_uf - Y V)^2 partials per tile
  static hipError_t gap_R(ifsvgp_ctx *c, int B, const int *skip) {
    Opnd<T> a{(const T *)Yfull(c), c->Mp}, b{(const T *)c->Vt, c->Mp};
    Sched sc{cdiv(c->M, CR::BM), cdiv(B, CR::BN), 0, 1, c->M, 0, skip};
    EpiGap<T> e{(const T *)c->Kft, c->Mp, c->M, B, c->tp_gap};
    return launch_gemm<CR>(lnc(c), a, b, sc, e);
  }
  // Hutchinson bound: with NC columns Xc in the batch operand (Vt rows),
  // on 64 x 64 tiles (NC is a few hundred columns: the larger tiles leave
  // most CUs idle),
  // Y1 = L Xc -> Ut, Y2 = K~ Y1 -> Kft, W Xc = L^T Y2 -> hwx (fp32), and for
  // the K probe columns E Omega = L^T S~ Y1 -> hex (fp32); all stored
  // transposed ([column][row]).
  static hipError_t hutch_L(ifsvgp_ctx *c, int NC) {
    Opnd<T> a{LT(c, 0), c->Mp}, b{(const T *)c->Vt, c->Mp};
    Sched sc{cdiv(c->M, CH::BM), cdiv(NC, CH::BN), 0, 1, c->M, K_HI_M1};
    EpiStoreT<T> e{(T *)c->Ut, c->Mp, c->M, NC};
    return launch_gemm<CH>(lnc(c), a, b, sc, e);
  }
  static hipError_t hutch_K(ifsvgp_ctx *c, int NC) {
    Opnd<T> a{(const T *)c->KtT, c->Mp}, b{(const T *)c->Ut, c->Mp};
    Sched sc{cdiv(c->M, CH::BM), cdiv(NC, CH::BN), 0, 1, c->M, 0};
    EpiStoreT<T> e{(T *)c->Kft, c->Mp, c->M, NC};
    return launch_gemm<CH>(lnc(c), a, b, sc, e);
  }
  static hipError_t hutch_Lt(ifsvgp_ctx *c, int NC) {
    Opnd<T> a{LtT(c, 0), c->Mp}, b{(const T *)c->Kft, c->Mp};
    Sched sc{cdiv(c->M, CH::BM), cdiv(NC, CH::BN), 0, 1, c->M, K_LO_M0};
    EpiStoreT<float> e{c->hwx, c->Mp, c->M, NC};
    return launch_gemm<CH>(lnc(c), a, b, sc, e);
  }
  static hipError_t hutch_E(ifsvgp_ctx *c, int B, int K) {
    Opnd<T> a{(const T *)c->LstT[0], c->Mp}, b{(const T *)c->Ut + (long)B * c->Mp, c->Mp};
    Sched sc{cdiv(c->M, CH::BM), cdiv(K, CH::BN), 0, 1, c->M, K_LO_M0};
    EpiStoreT<float> e{c->hex, c->Mp, c->M, K};
    return launch_gemm<CH>(lnc(c), a, b, sc, e);
  }
  // Hutchinson backward: Y1 = L X for the r columns of X (k < m0+BM), then
  // G_uu = Y1 (Y1 S)^T on lower tiles (k < r) -> H_uu reductions
  static long ldr(ifsvgp_ctx *c) { return 2 * (long)c->Bp; }
  static hipError_t hutch_LX(ifsvgp_ctx *c, int r) {
    Opnd<T> a{LT(c, 0), c->Mp}, b{(const T *)c->hxt, c->Mp};
    Sched sc{cdiv(c->M, CH::BM), cdiv(r, CH::BN), 0, 1, c->M, K_HI_M1};
    EpiStore<TW> e{(TW *)c->hy1, ldr(c), c->M, r, 0, 0};
    return launch_gemm<CH>(lnc(c), a, b, sc, e);
  }
  static hipError_t hutch_Guu(ifsvgp_ctx *c, int r) {
    const int D = c->D;
    Opnd<TW> a{(const TW *)c->hy1, ldr(c)}, b{(const TW *)c->hy2, ldr(c)};
    Sched sc{nb(c), nb(c), 1, 1, r, 0};
    EpiGradUu<GradPartial<T>> e{c->Kt, c->sP, c->Zs, c->Mp, c->M, D, c->hz, c->hzrow, c->tp_uu,
                                nullptr};
    return launch_gemm<CSW>(lnc(c), a, b, sc, e, 2 * CSW::BM * (dpof(D) + 1) * 4);
  }
  // U = Q V -> Ut, sigma^2 partials
  static hipError_t gemm_U(ifsvgp_ctx *c, int B) {
    Opnd<T> a{(const T *)c->QT, c->Mp}, b{(const T *)c->Vt, c->Mp};
    Sched sc{cdiv(c->M, CR::BM), cdiv(B, CR::BN), 0, 1, c->M, 0};
    EpiU<T> e{(T *)c->Ut, (const T *)c->V, c->va, c->Bp, c->Mp, c->M, B, c->var_part,
              c->mu_part, c->Bp};
    return launch_gemm<CR>(lnc(c), a, b, sc, e);
  }
  // R = L U (k < m0+BM) -> H_uf reductions
  // (lb, al, be: the epilogue's L b, alpha, beta, by default the context's)
  // (KW: the K_uf recompute from the set-up's split inputs, bf16 / fp16 forms)
  template <int KW>
  static hipError_t gemm_R_kw(ifsvgp_ctx *c, int cur, int B, const float *lb, const float *al,
                              const float *be) {
    const int D = c->D;
    Opnd<T> a{LT(c, cur), c->Mp}, b{(const T *)c->Ut, c->Mp};
    Sched sc{cdiv(c->M, CRG::BM), cdiv(B, CRG::BN), 0, 1, c->M, K_HI_M1};
    EpiGradUf<KW> e{lb ? lb : c->vLb, al ? al : c->alpha, be ? be : c->beta, c->Zs, c->Xs,
                    c->sfn, c->M, B, D, c->hrow, c->hcol, (long)c->Bp, c->hx, c->tp_uf,
                    c->gZh, c->gZl, c->gXh, c->gXl, c->gzc, c->gxr};
    return launch_gemm<CRG>(lnc(c), a, b, sc, e, graduf_extra(CRG::BM, CRG::BN, D));
  }
  static hipError_t gemm_R(ifsvgp_ctx *c, int cur, int B, const float *lb = nullptr,
                           const float *al = nullptr, const float *be = nullptr) {
    if constexpr (std::is_same<T, float>::value) {
      return gemm_R_kw<0>(c, cur, B, lb, al, be);
    } else {
      switch (c->gldk) {
        case 16: return gemm_R_kw<16>(c, cur, B, lb, al, be);
        case 32: return gemm_R_kw<32>(c, cur, B, lb, al, be);
        default: return gemm_R_kw<64>(c, cur, B, lb, al, be);
      }
    }
  }
  // Ys[s] = (V_s D)(V_s D)^T, D = diag(sqrt(-beta)) (lower tiles mirrored, split-K
  // over the batch); equals -V diag(beta) V^T since beta <= 0 for the
  // log-concave Gaussian and probit likelihoods.
  // split-K pieces: enough workgroups for about four per CU, each piece at
  // least 4 k-steps long; every piece costs an fp32 M x M partial
  static constexpr int kSyrkWG = 1024;  // workgroups the split-K aims for
  static int syrk_splits(ifsvgp_ctx *c, int B) {
    const int n = cdiv(c->M, CSY::BM), nt = n * (n + 1) / 2;
    return std::max(1, std::min({c->nsplit, cdiv(B, 4 * CSY::BK), cdiv(kSyrkWG, nt)}));
  }
  // mirror: also store the upper tiles (else the pieces hold lower tiles only)
  static hipError_t syrk(ifsvgp_ctx *c, int B, bool mirror = true) {
    Opnd<T> a{(const T *)c->Vs, c->Bp}, b{(const T *)c->Vs, c->Bp};
    const int n = cdiv(c->M, CSY::BM);
    Sched sc{n, n, 1, syrk_splits(c, B), B, 0};
    EpiStore<float> e{c->Ys, c->Mp, c->M, c->M, mirror ? 1 : 0, (long)c->Mp * c->Mp};
    return launch_gemm<CSY>(lnc(c), a, b, sc, e);
  }
  // Y2 = L C (k < m0+BM), C symmetric
  static hipError_t gemm_Y2(ifsvgp_ctx *c, int cur) {
    Opnd<TW> a{LW(c, cur), c->Mp}, b{(const TW *)c->Cm, c->Mp};
    Sched sc{nb(c), nb(c), 0, 1, c->M, K_HI_M1};
    EpiStore<TW> e{(TW *)c->Y2, c->Mp, c->M, c->M, 0, 0};
    return launch_gemm<CSW>(lnc(c), a, b, sc, e);
  }
  // G_uu = Y2 L^T (lower tiles, k < n0+BN) -> H_uu reductions
  static hipError_t gemm_Guu(ifsvgp_ctx *c, int cur, float *gdiag) {
    const int D = c->D;
    Opnd<TW> a{(const TW *)c->Y2, c->Mp}, b{LW(c, cur), c->Mp};
    Sched sc{nb(c), nb(c), 1, 1, c->M, K_HI_N1};
    EpiGradUu<GradPartial<T>> e{c->Kt, c->sP, c->Zs, c->Mp, c->M, D, c->hz, c->hzrow, c->tp_uu,
                                gdiag};
    return launch_gemm<CSW>(lnc(c), a, b, sc, e, 2 * CSW::BM * (dpof(D) + 1) * 4);
  }
  // L Q on lower tiles (k < m0+BM) -> partials of diag(L Q L^T) = diag(P)
  static hipError_t gemm_LQ(ifsvgp_ctx *c, int cur) {
    Opnd<T> a{LT(c, cur), c->Mp}, b{(const T *)c->QT, c->Mp};
    Sched sc{nb(c), nb(c), 1, 1, c->M, K_HI_M1};
    EpiRowDotL e{c->L32[cur], c->Mp, c->M, c->pdiag, c->Mp};
    return launch_gemm<CS>(lnc(c), a, b, sc, e);
  }
};

// ------------------------------------------------------------------ stages
// One library call: the stages it runs and the host-side values that shape
// its launches.  Everything else the kernels read about the call (the
// caller's buffers, N / B, grad_scale, the NG step sizes) is in the device
// argument block c->dca written by the call's k_latch.
struct Call {
  bool setup, fwd, bwd;  // set-up + NG steps; bound; backward
  int B, n_ng;
  const float *gammas;   // host, n_ng values
  bool need_noise, want_gm, want_gs;
  int adapt;             // NG_FIXED, or the stopping rule of the NG steps (threshold in the block)
};

// Copies NG step sizes [s0, s0 + n) into the device block (stream ordered
// after the steps that read the previous window).
__global__ void k_latch_gammas(CallArgs g, int n, CallArgs *dst) {
  const int t = threadIdx.x;
  if (t < n) dst->gammas[t] = g.gammas[t];
}

// cav non-null: the set-up also writes the call's argument block (direct
// execution); null: a k_latch has written it (recorded calls).
// gen_B > 0 (bf16 / fp16 forms): also the inputs of the generated K_uf tiles
// for a batch of gen_B points, and Xs.
template <typename T>
static int stage_setup(ifsvgp_ctx *c, int need_noise, const CallArgs *cav, int gen_B = 0) {
  const int M = c->M;
  Timed t(c, KK_PREP);
  SetupArgs a;
  a.latch = cav != nullptr;
  if (cav) a.cav = *cav;
  a.ca = c->dca;
  a.M = M; a.D = c->D; a.need_noise = need_noise;
  a.Zs = c->Zs; a.inv_ell = c->inv_ell; a.sP = c->sP; a.Kt = c->Kt; a.sfn = c->sfn;
  a.KtT = c->KtT;
  a.ld = c->Mp;
  a.L32 = c->L32[0]; a.Lt32 = c->Lt32[0]; a.LT = c->LT[0]; a.LtT = c->LtT[0];
  a.LstT = c->LstT[0];
  a.scal = c->scal; a.flag = c->flag; a.ngskip = c->ngskip;
  a.nKx = cdiv(M, 64);
  a.nK = a.nKx * (a.nKx + 1) / 2;
  a.nLx = cdiv(M, 64);
  const bool gen = gen_B > 0 && !std::is_same<T, float>::value;
  a.nGz = gen ? cdiv(M, 64) : 0;
  a.nG = gen ? a.nGz + cdiv(gen_B, 64) : 0;
  a.B = gen_B;
  a.ldk = c->gldk;
  a.Zh = c->gZh; a.Zl = c->gZl; a.Xh = c->gXh; a.Xl = c->gXl;
  a.zc = c->gzc; a.xr = c->gxr; a.Xs = c->Xs;
  a.gs = gsz(c);
  const int nblk = 1 + a.nK + a.nLx * (a.nLx + 1) / 2 + a.nG;
  hipLaunchKernelGGL((k_setup<MAXD, T>), gdim(c, dim3(nblk)), dim3(NTB), 0, c->st, a);
  HIPCK(hipGetLastError());
  return IFSVGP_OK;
}

// n_ng natural-gradient steps from slot 0; the last writes the caller's L.
// Step sizes beyond the first MAX_NG_LATCH are latched window by window.
// NG_RESID: a check kernel after each W product applies the residual rule;
// NG_GAP: before each step V = L^T K_uf, Y = K~ L and the gap partials of
// K~ L V against K_uf (batch of B columns) feed the variance-gap rule.  Once a
// rule has fired, the remaining products skip their k-loops.
template <typename T>
static int launch_kuf(ifsvgp_ctx *c, int B);
template <typename T>
static int stage_natgrad(ifsvgp_ctx *c, const float *gammas, int n_ng, int rule, int B) {
  const int *skip = rule != NG_FIXED ? c->ngskip : nullptr;
  if (rule == NG_GAP) {
    HIPCK(fork_side(c));
    int r = launch_kuf<T>(c, B);
    if (r) return r;
    HIPCK(join_side(c));
  }
  int cur = 0;
  for (int s = 0; s < n_ng; ++s) {
    if (s > 0 && s % MAX_NG_LATCH == 0) {
      CallArgs g{};
      const int n = std::min(MAX_NG_LATCH, n_ng - s);
      for (int k = 0; k < n; ++k) g.gammas[k] = gammas[s + k];
      hipLaunchKernelGGL(k_latch_gammas, dim3(1), dim3(MAX_NG_LATCH), 0, c->st, g, n, c->dca);
      HIPCK(hipGetLastError());
    }
    if (rule == NG_GAP) {
      { Timed t(c, KK_V); HIPCK(Ops<T>::gemm_V(c, cur, B, skip)); }
      { Timed t(c, KK_NG_Y); HIPCK(Ops<T>::gap_Y(c, cur, skip)); }
      { Timed t(c, KK_U); HIPCK(Ops<T>::gap_R(c, B, skip)); }
      hipLaunchKernelGGL(k_ng_check, dim3(1), dim3(NTB), 0, c->st, (const double *)c->tp_gap,
                         cdiv(c->M, 128) * cdiv(B, 64), c->M, s, c->ngskip, c->scal,
                         (const CallArgs *)c->dca, 1);
    }
    { Timed t(c, KK_NG_Y); HIPCK(Ops<T>::gram_Y(c, cur, skip)); }
    { Timed t(c, KK_NG_W); HIPCK(Ops<T>::ng_W(c, cur, skip)); }
    if (rule == NG_RESID) {
      const int nbk = Ops<T>::nb(c);
      hipLaunchKernelGGL(k_ng_check, dim3(1), dim3(NTB), 0, c->st, (const double *)c->tp_ng,
                         nbk * (nbk + 1) / 2, c->M, s, c->ngskip, c->scal,
                         (const CallArgs *)c->dca, 0);
    }
    {
      Timed t(c, KK_NG_L);
      HIPCK(Ops<T>::ng_L(c, cur, 1 - cur, s % MAX_NG_LATCH, s, s == n_ng - 1, skip));
    }
    cur = 1 - cur;
  }
  c->cur = cur;
  return IFSVGP_OK;
}

// K_uf tiles on the side stream.
template <typename T>
static int launch_kuf(ifsvgp_ctx *c, int B) {
  OnSide side(c);
  Timed t(c, KK_KUF);
  static int kuf_attr = 0;
  const int kb = kuf_smem(c->D);
  if (kb > kuf_attr) {
    HIPCK(hipFuncSetAttribute((const void *)k_kuf<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              kb));
    kuf_attr = kb;
  }
  hipLaunchKernelGGL((k_kuf<T>), gdim(c, dim3(cdiv(B, KUF_T), cdiv(c->M, KUF_T))), dim3(NTB), kb,
                     c->st, (const float *)c->Zs, (const CallArgs *)c->dca,
                     (const float *)c->inv_ell, c->M, B, c->D, (const float *)c->sfn, c->Xs,
                     (T *)c->Kft, (long)c->Mp, gsz(c));
  HIPCK(hipGetLastError());
  return IFSVGP_OK;
}

// Bound at c->cur.  V = L^T K_uf and a = L^T m~ have been enqueued on the
// side stream (forked after the last update of L).
// defer_final: the backward follows in the same call and its k_valpha forms F.
template <typename T>
static int stage_bound(ifsvgp_ctx *c, int B, bool defer_final) {
  const int M = c->M, cur = c->cur;
  const float *L = c->L32[cur];
  const long Mp = c->Mp;
  { Timed t(c, KK_GR_Y); HIPCK(Ops<T>::gram_Y(c, cur)); }
  { Timed t(c, KK_GR_W); HIPCK(Ops<T>::gr_W(c, cur)); }
  { Timed t(c, KK_GR_E); HIPCK(Ops<T>::gr_E(c, cur)); }
  // V = L^T K_uf and a = L^T m~ come from the side stream; b = Q a and
  // Lb = L b, Wub = Wu b (with partials of quad and log|T|), then U, whose
  // epilogue takes the mean from a and runs the likelihood and F
  HIPCK(join_side(c));
  {
    Timed t(c, KK_VEC);
    hipLaunchKernelGGL(k_gemv_rows, gdim(c, dim3(cdiv(M, NTB / 64))), dim3(NTB), 0, c->st,
                       (const float *)c->Q32, Mp, M, M, (const float *)c->va,
                       (const float *)nullptr, 0, (const double *)nullptr, c->vb, gsz(c));
    hipLaunchKernelGGL(k_vec_lb_wub, gdim(c, dim3(cdiv(2 * M, NTB / 64))), dim3(NTB), 0, c->st,
                       L, (const float *)c->Wu32, Mp, M, (const float *)c->vb, c->vLb, c->vWub,
                       c->vec_part, c->flag, gsz(c));
  }
  { Timed t(c, KK_U); HIPCK(Ops<T>::gemm_U(c, B)); }
  {
    Timed t(c, KK_LIK);
    const LikArgs a = lik_args(c, B, gsz(c), defer_final ? 1 : 0);
    hipLaunchKernelGGL(k_lik, gdim(c, dim3(cdiv(c->Bp, NTB))), dim3(NTB), 0, c->st, a);
  }
  HIPCK(hipGetLastError());
  return IFSVGP_OK;
}

// lik_final: the forward of the same call deferred F to k_valpha.
template <typename T>
static int stage_backward(ifsvgp_ctx *c, int B, bool want_gm, bool want_gs, bool lik_final) {
  using TW = typename Ops<T>::TW;
  const int M = c->M, D = c->D, cur = c->cur;
  const long Mp = c->Mp;
  // R = L U and its gradient epilogue run on side stream 0 beside the C chain
  HIPCK(fork_side(c));
  {
    OnSide side(c);
    Timed t(c, KK_R);
    HIPCK(Ops<T>::gemm_R(c, cur, B));
  }
  {
    Timed t(c, KK_VALPHA);
    const int nlik = lik_final ? cdiv(c->Bp, NTB) : 0;
    // (measured: one row per workgroup 0.184 against four 0.188 ms per step
    // at M = 1024; four 0.551 against one 0.554 ms at M = 2048)
    const int rpw = va_rows(M);
    hipLaunchKernelGGL(k_valpha<T>, gdim(c, dim3(cdiv(M, rpw) + (nlik ? 1 : 0))), dim3(NTB), 0,
                       c->st, (const T *)c->V, (long)c->Bp, M, c->Bp, (const float *)c->alpha,
                       (const float *)c->sqnb, (T *)c->Vs, c->vVa, gsz(c),
                       lik_args(c, B, 0), nlik, rpw);
  }
  // (V D)(V D)^T by split-K on lower tiles; C assembled per lower tile
  { Timed t(c, KK_SYRK); HIPCK(Ops<T>::syrk(c, B, false)); }
  {
    Timed t(c, KK_ASM);
    const int nb = cdiv(M, 64);
    hipLaunchKernelGGL(k_assemble_C<TW>, gdim(c, dim3(nb * (nb + 1) / 2)), dim3(NTB), 0, c->st,
                       (const float *)c->Ys, Ops<T>::syrk_splits(c, B), Mp * Mp,
                       (const float *)c->Wu32, (const float *)c->Q32, (const float *)c->va,
                       (const float *)c->vb, (const float *)c->vWub, (const float *)c->vVa, M,
                       Mp, (TW *)c->Cm, gsz(c));
  }
  { Timed t(c, KK_Y2); HIPCK(Ops<T>::gemm_Y2(c, cur)); }
  { Timed t(c, KK_GUU); HIPCK(Ops<T>::gemm_Guu(c, cur, want_gs ? c->gdiag : nullptr)); }
  if (want_gs) {
    Timed t(c, KK_LQ);
    HIPCK(Ops<T>::gemm_LQ(c, cur));
  }
  HIPCK(join_side(c));
  {
    Timed t(c, KK_GRAD);
    const int ntB = cdiv(B, 128), nb = cdiv(M, 64), nbm = cdiv(M, 128);
    const int R = NTB / D;
    const int rb = cdiv(M, grad_zrows(D)), cb = cdiv(B, R), rq = cdiv(M, NTB / 64);
    GradArgs g{M, B, D, c->dca, c->Zs, c->Xs, c->inv_ell, c->sfn,
               c->hrow, c->hx, ntB, c->hzrow, c->hz, nb, c->hcol, nbm, (long)c->Bp,
               c->tp_uf, nbm * ntB, c->tp_uu, nb * (nb + 1) / 2,
               c->lik_part, cdiv(c->Bp, NTB),
               c->Q32, c->vVa, c->vWub, Mp, c->vt2, c->ell_part, rb, cb,
               c->gdiag, c->pdiag, (long)Mp, c->vLb, c->sP, gsz(c)};
    hipLaunchKernelGGL(k_grad<GradPartial<T>>, gdim(c, dim3(rb + cb + rq)), dim3(NTB), 0, c->st, g);
    // dF/dm~ = L t2 and dF/ds~ rows (when requested), then the scalar gradients
    const int mrows = (want_gm || want_gs) ? rq : 0;
    hipLaunchKernelGGL(k_grad_tail, gdim(c, dim3(mrows + D + 1)), dim3(NTB), 0, c->st, g,
                       (const float *)c->L32[cur], mrows);
  }
  HIPCK(hipGetLastError());
  return IFSVGP_OK;
}

// IFSVGP_KUF_AUTO stores the K_uf tiles of the bf16 / fp16 forms (generated
// once beside the natural-gradient step) rather than generating them inside
// V from this many entries M x B on: V's row blocks regenerate each tile
// M / 256 times on average, which outweighs the extra launch and fork for
// large problems (measured per training step: 0.188 ms generating inside V
// against 0.190 to 0.192 ms storing at M = 1024, B = 4096; 0.585 against
// 0.559 ms at M = 2048, B = 8192).
static constexpr long KUF_STORE_MIN = 1L << 23;

// All launches of one call on c->st (and the side stream), in order.
template <typename T>
static int enqueue(ifsvgp_ctx *c, const Call &k, const CallArgs *cav) {
  int r;
  c->ev_next = 0;
  c->side_open = false;
  // K_uf: the fp32 form stores it first (k_kuf: distances from differences,
  // accurate exp); bf16 / fp16 generate its tiles from the set-up's split
  // inputs, inside V = L^T K_uf (LDS only, the default) or, as the context's
  // K_uf mode asks, stored once (k_kuf_gen)
  constexpr bool gen = !std::is_same<T, float>::value;
  const bool stored = !gen || c->kuf_mode == IFSVGP_KUF_STORED ||
                      (c->kuf_mode == IFSVGP_KUF_AUTO && (long)c->M * k.B >= KUF_STORE_MIN);
  if (k.setup) {
    r = stage_setup<T>(c, k.need_noise, cav, k.fwd && gen ? k.B : 0);
    if (r) return r;
    if (!k.fwd) {
      c->fwd_valid = 0;
      return stage_natgrad<T>(c, k.gammas, k.n_ng, k.adapt, k.B);
    }
    if (stored) {
      // side stream: K_uf tiles need only Z / ell and the batch ...
      HIPCK(fork_side(c));
      if constexpr (gen) {
        OnSide side(c);
        Timed t(c, KK_KUF);
        HIPCK(Ops<T>::kuf_gen(c, k.B));
      } else {
        r = launch_kuf<T>(c, k.B);
        if (r) return r;
      }
    }
    r = stage_natgrad<T>(c, k.gammas, k.n_ng, NG_FIXED, k.B);
    if (r) return r;
    // ... and V = L^T K_uf and a = L^T m~ the updated L (the fork joins the
    // K_uf tiles first), so all of them run beside the Gram products; a
    // comes from extra workgroups of V's launch
    HIPCK(fork_side(c));
    {
      OnSide side(c);
      Timed t(c, KK_V);
      if (stored) HIPCK(Ops<T>::gemm_V(c, c->cur, k.B, nullptr, c->va));
      else HIPCK(Ops<T>::gemm_Vf(c, c->cur, k.B, c->va));
    }
    r = stage_bound<T>(c, k.B, k.bwd);
    if (r) return r;
    c->fwd_valid = 1;
    c->fwd_B = k.B;
  }
  if (k.bwd) {
    r = stage_backward<T>(c, k.B, k.want_gm, k.want_gs, k.setup && k.fwd);
    if (r) return r;
  }
  return IFSVGP_OK;
}

#define PREC_DISPATCH(fn, ...)                                     \
  switch (c->prec) {                                               \
    case IFSVGP_PREC_FP32: return fn<float>(__VA_ARGS__);          \
    case IFSVGP_PREC_BF16: return fn<__bf16>(__VA_ARGS__);         \
    default: return fn<_Float16>(__VA_ARGS__);                     \
  }

// cav: the call's arguments, latched by the set-up (direct execution of a
// call with a set-up), or null when a k_latch has already written them.
static int enqueue_any(ifsvgp_ctx *c, const Call &k, const CallArgs *cav) {
  PREC_DISPATCH(enqueue, c, k, cav)
}
static int latch(ifsvgp_ctx *c, const CallArgs &ca) {
  hipLaunchKernelGGL(k_latch, dim3(1), dim3(64), 0, c->st, ca, c->dca);
  HIPCK(hipGetLastError());
  return IFSVGP_OK;
}
// Prediction at n test points in chunks of at most B_max: the set-up and the
// Gram products for Q once (no NG step, T = L L^T as given), then per chunk
// K_u* and V_* = L^T K_u* (side stream), U_* = Q V_* with its mean and
// variance partials, and the predictive kernel.  Later chunks latch their own
// X / y into the argument block after the previous chunk's kernels.
struct PredOut {
  const float *X, *y;
  int n;
  float *mu, *var, *lpd;
  double *nlpd;
};

template <typename T>
static int enqueue_predict(ifsvgp_ctx *c, const CallArgs &ca0, const PredOut &o) {
  c->ev_next = 0;
  c->side_open = false;
  const bool want_lpd = o.y != nullptr;
  int r = stage_setup<T>(c, want_lpd && c->lik == IFSVGP_LIK_GAUSSIAN, &ca0);
  if (r) return r;
  c->cur = 0;
  c->fwd_valid = 0;
  const int nchunks = cdiv(o.n, c->Bmax);
  for (int q = 0; q < nchunks; ++q) {
    const int off = q * c->Bmax, nb = std::min(c->Bmax, o.n - off);
    if (q > 0) {
      CallArgs a = ca0;
      a.X = o.X + (long)off * c->D;
      a.y = want_lpd ? o.y + off : nullptr;
      r = latch(c, a);
      if (r) return r;
    }
    HIPCK(fork_side(c));
    r = launch_kuf<T>(c, nb);
    if (r) return r;
    {
      OnSide side(c);
      {
        Timed t(c, KK_V);
        HIPCK(Ops<T>::gemm_V(c, 0, nb));
      }
      if (q == 0) {
        Timed t(c, KK_VEC);
        hipLaunchKernelGGL(k_lt_m, dim3(cdiv(c->M, NTB / 64)), dim3(NTB), 0, c->st,
                           (const float *)c->Lt32[0], (long)c->Mp, c->M,
                           (const CallArgs *)c->dca, c->va);
      }
    }
    if (q == 0) {
      { Timed t(c, KK_GR_Y); HIPCK(Ops<T>::gram_Y(c, 0)); }
      { Timed t(c, KK_GR_W); HIPCK(Ops<T>::gr_W(c, 0)); }
      { Timed t(c, KK_GR_E); HIPCK(Ops<T>::gr_E(c, 0)); }
    }
    HIPCK(join_side(c));
    { Timed t(c, KK_U); HIPCK(Ops<T>::gemm_U(c, nb)); }
    Timed t(c, KK_LIK);
    const int nblk = cdiv(nb, NTB);
    PredArgs a{c->mu_part, cdiv(c->M, 128), c->var_part, cdiv(c->M, 128), (long)c->Bp,
               nb, c->sfn, c->lik, want_lpd ? o.y + off : nullptr,
               o.mu + off, o.var + off, o.lpd ? o.lpd + off : nullptr, c->lik_part};
    hipLaunchKernelGGL(k_predict, dim3(nblk), dim3(NTB), 0, c->st, a);
    if (want_lpd)
      hipLaunchKernelGGL(k_predict_sum, dim3(1), dim3(NTB), 0, c->st, (const double *)c->lik_part,
                         nblk, c->scal, q == 0 ? 1 : 0, q == nchunks - 1 ? 1 : 0,
                         (double)o.n, o.nlpd);
    HIPCK(hipGetLastError());
  }
  return IFSVGP_OK;
}

// Bound evaluation with Hutchinson trace estimates (K probes, Omt [K][M] on
// the device): set-up, K_uf tiles and V = L^T K_uf, a = L^T m~ (side stream),
// then the thin products with Xc = [V | Omega | a], the row reductions, the
// trace estimates, b^T Wu b by matrix-vector products, and the likelihood
// kernel's finalisation of F.  No M x M x M product.
// grid.y limit of a launch; kernels with a row index in y loop over it
static constexpr int kMaxGridY = 65535;

template <typename T>
static int enqueue_hutch(ifsvgp_ctx *c, const CallArgs &ca, int B, const float *Omt, int K) {
  c->ev_next = 0;
  c->side_open = false;
  // (with the split inputs of the K_uf tiles, which the backward's R epilogue reads)
  int r = stage_setup<T>(c, c->lik == IFSVGP_LIK_GAUSSIAN, &ca, B);
  if (r) return r;
  c->cur = 0;
  c->fwd_valid = 0;
  const int M = c->M, NC = B + K + 1;
  const long Mp = c->Mp;
  HIPCK(fork_side(c));
  r = launch_kuf<T>(c, B);
  if (r) return r;
  {
    OnSide side(c);
    HIPCK(Ops<T>::gemm_V(c, 0, B));
    hipLaunchKernelGGL(k_lt_m, dim3(cdiv(M, NTB / 64)), dim3(NTB), 0, c->st,
                       (const float *)c->Lt32[0], Mp, M, (const CallArgs *)c->dca, c->va);
  }
  HIPCK(join_side(c));
  hipLaunchKernelGGL((k_hutch_fill<T>), dim3(cdiv(c->Mp, NTB), std::min(K + 1, kMaxGridY)),
                     dim3(NTB), 0, c->st,
                     (T *)c->Vt, Mp, B, K, Omt, (const float *)c->va, M, c->Mp);
  HIPCK(Ops<T>::hutch_L(c, NC));
  HIPCK(Ops<T>::hutch_K(c, NC));
  HIPCK(Ops<T>::hutch_Lt(c, NC));
  HIPCK(Ops<T>::hutch_E(c, B, K));
  HutchArgs h{c->Vt, Mp, c->Ut, c->hwx, c->hex, Omt, c->va, M, B, K, c->var_part, c->mu_part, c->hp,
              c->vb};
  hipLaunchKernelGGL((k_hutch_rows<T>), dim3(cdiv(NC, NTB / 64)), dim3(NTB), 0, c->st, h);
  hipLaunchKernelGGL(k_hutch_final, dim3(1), dim3(NTB), 0, c->st, (const double *)c->hp, K,
                     c->tp_gram);
  // b^T Wu b with Wu b = L^T (K~ - S~) L b
  const dim3 gv(cdiv(M, NTB / 64));
  hipLaunchKernelGGL(k_gemv_rows, gv, dim3(NTB), 0, c->st, (const float *)c->L32[0], Mp, M, M,
                     (const float *)c->vb, (const float *)nullptr, 1, (const double *)nullptr,
                     c->vLb);
  hipLaunchKernelGGL(k_gemv_rows, gv, dim3(NTB), 0, c->st, (const float *)c->Kt, Mp, M, M,
                     (const float *)c->vLb, (const float *)nullptr, 0, (const double *)nullptr,
                     c->vt2);
  hipLaunchKernelGGL(k_hutch_sub_diag, dim3(cdiv(M, NTB)), dim3(NTB), 0, c->st, c->vt2,
                     (const float *)c->sP, (const float *)c->vLb, M);
  hipLaunchKernelGGL(k_gemv_rows, gv, dim3(NTB), 0, c->st, (const float *)c->Lt32[0], Mp, M, M,
                     (const float *)c->vt2, (const float *)nullptr, 0, (const double *)nullptr,
                     c->vWub);
  hipLaunchKernelGGL(k_hutch_quad, dim3(1), dim3(NTB), 0, c->st, (const float *)c->vb,
                     (const float *)c->vWub, (const float *)c->L32[0], Mp, M, c->vec_part,
                     c->flag);
  LikArgs a{c->mu_part, 1, c->var_part, 1, (long)c->Bp,
            c->dca, B, c->Bp, c->sfn, c->lik, c->gh, c->ngh,
            c->mu, c->var, c->alpha, c->beta, c->sqnb, c->lik_part,
            c->tp_gram, 1, c->vec_part, 1,
            c->scal, M, c->flag, c->counters + CNT_LIK};
  hipLaunchKernelGGL(k_lik, dim3(cdiv(c->Bp, NTB)), dim3(NTB), 0, c->st, a);
  HIPCK(hipGetLastError());
  c->fwd_valid = 2;
  c->fwd_B = B;
  c->fwd_K = K;
  return IFSVGP_OK;
}

// Backward of the Hutchinson bound at the forward's probes, with no
// M x M x M product: the data side's R = L U as in the exact backward (U =
// 2V - W V kept by the forward), and C = X S X^T in low-rank form (columns
// V, Omega, Omega - G, x = V alpha - Wu b, a, b; G = 2 W Omega - E Omega
// from the forward's W Omega and E Omega), so G_uu = L C L^T = Y1 (Y1 S)^T
// with Y1 = L X: two products of inner size r = B + 2K + 3; t2 = Q x by
// matrix-vector products, Q not being formed.
template <typename T>
static int enqueue_hutch_bwd(ifsvgp_ctx *c, const CallArgs &ca, int B, const float *Omt, int K,
                             bool want_gm) {
  using TW = typename Ops<T>::TW;
  c->ev_next = 0;
  c->side_open = false;
  int r = latch(c, ca);
  if (r) return r;
  const int M = c->M, D = c->D, nr = B + 2 * K + 3;
  const long Mp = c->Mp;
  HIPCK(fork_side(c));
  {
    OnSide side(c);
    Timed t(c, KK_R);
    HIPCK(Ops<T>::gemm_R(c, 0, B));
  }
  hipLaunchKernelGGL(k_valpha<T>, dim3(cdiv(M, va_rows(M))), dim3(NTB), 0, c->st,
                     (const T *)c->V, (long)c->Bp, M, c->Bp, (const float *)c->alpha,
                     (const float *)c->sqnb, (T *)c->Vs, c->vVa, 0L, LikArgs{}, 0, va_rows(M));
  hipLaunchKernelGGL((k_hutch_X<T>), dim3(cdiv(c->Mp, NTB), std::min(rup(nr, 64), kMaxGridY)),
                     dim3(NTB), 0, c->st, (const T *)c->Vt, Omt, (const float *)c->hwx,
                     (const float *)c->hex, (const float *)c->vVa, (const float *)c->vWub,
                     (const float *)c->va, (const float *)c->vb, B, K, M, c->Mp, rup(nr, 64),
                     (T *)c->hxt);
  HIPCK(Ops<T>::hutch_LX(c, nr));
  hipLaunchKernelGGL((k_hutch_mix<TW>), dim3(grid1((long)c->Mp * Ops<T>::ldr(c))), dim3(NTB), 0,
                     c->st, (const TW *)c->hy1, (TW *)c->hy2, Ops<T>::ldr(c), M, c->Mp, B, K,
                     (const float *)c->beta, (float)(0.25 / K));
  HIPCK(Ops<T>::hutch_Guu(c, nr));
  // W x = L^T K~ L x for x = V alpha - Wu b
  const dim3 gv(cdiv(M, NTB / 64));
  hipLaunchKernelGGL(k_gemv_rows, gv, dim3(NTB), 0, c->st, (const float *)c->L32[0], Mp, M, M,
                     (const float *)c->vVa, (const float *)c->vWub, 1, (const double *)nullptr,
                     c->hx1);
  hipLaunchKernelGGL(k_gemv_rows, gv, dim3(NTB), 0, c->st, (const float *)c->Kt, Mp, M, M,
                     (const float *)c->hx1, (const float *)nullptr, 0, (const double *)nullptr,
                     c->hx2);
  hipLaunchKernelGGL(k_gemv_rows, gv, dim3(NTB), 0, c->st, (const float *)c->Lt32[0], Mp, M, M,
                     (const float *)c->hx2, (const float *)nullptr, 0, (const double *)nullptr,
                     c->hx1);
  hipLaunchKernelGGL(k_hutch_t2, dim3(cdiv(M, NTB)), dim3(NTB), 0, c->st, c->vt2,
                     (const float *)c->vVa, (const float *)c->vWub, (const float *)c->hx1, M);
  HIPCK(join_side(c));
  const int ntB = cdiv(B, 128), nb = cdiv(M, 64), nbm = cdiv(M, 128);
  const int R = NTB / D;
  const int rb = cdiv(M, grad_zrows(D)), cb = cdiv(B, R);
  GradArgs g{M, B, D, c->dca, c->Zs, c->Xs, c->inv_ell, c->sfn,
             c->hrow, c->hx, ntB, c->hzrow, c->hz, nb, c->hcol, nbm, (long)c->Bp,
             c->tp_uf, nbm * ntB, c->tp_uu, nb * (nb + 1) / 2,
             c->lik_part, cdiv(c->Bp, NTB),
             nullptr, c->vVa, c->vWub, Mp, c->vt2, c->ell_part, rb, cb,
             nullptr, nullptr, (long)Mp, c->vLb, c->sP};
  hipLaunchKernelGGL(k_grad<GradPartial<T>>, dim3(rb + cb), dim3(NTB), 0, c->st, g);
  const int mrows = want_gm ? cdiv(M, NTB / 64) : 0;
  hipLaunchKernelGGL(k_grad_tail, dim3(mrows + D + 1), dim3(NTB), 0, c->st, g,
                     (const float *)c->L32[0], mrows);
  HIPCK(hipGetLastError());
  return IFSVGP_OK;
}

// direct execution: the set-up latches the arguments when there is one
static int run_direct(ifsvgp_ctx *c, const Call &k, const CallArgs &ca) {
  if (k.setup) return enqueue_any(c, k, &ca);
  int r = latch(c, ca);
  return r ? r : enqueue_any(c, k, nullptr);
}

// ------------------------------------------------------------------ graphs
// With recording on, a call whose launch structure (stages, B, NG step
// count, requested outputs) has been seen before is recorded once into a HIP
// graph on the private capture stream, then replayed on c->st with one
// launch; the caller's buffers reach the kernels through the argument block,
// so replays serve any buffers.  Structures seen once run directly, so
// changing shapes cost no recording.  A replay costs the host less than the
// direct launches but runs somewhat longer on the GPU, so recording is for
// callers whose issue rate, not the GPU, limits them.
static bool same_key(const GraphKey &a, const GraphKey &b) {
  return a.setup == b.setup && a.fwd == b.fwd && a.bwd == b.bwd && a.B == b.B &&
         a.n_ng == b.n_ng && a.need_noise == b.need_noise && a.want_gm == b.want_gm &&
         a.want_gs == b.want_gs && a.adapt == b.adapt && a.cur0 == b.cur0;
}

static void graphs_clear(ifsvgp_ctx *c) {
  for (auto &g : c->graphs)
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
  c->graphs.clear();
}

static int run_call(ifsvgp_ctx *c, const Call &k, const CallArgs &ca) {
  const GraphKey key{k.setup, k.fwd,     k.bwd,     k.B,
                     k.n_ng,  k.need_noise, k.want_gm, k.want_gs,
                     k.adapt, k.setup ? 0 : c->cur};
  if (!c->use_graphs || c->timing || k.n_ng > MAX_NG_LATCH) return run_direct(c, k, ca);
  GraphEnt *ent = nullptr;
  for (auto &g : c->graphs)
    if (same_key(g.key, key)) ent = &g;
  if (ent && ent->exec) {
    int r = latch(c, ca);
    if (r) return r;
    HIPCK(hipGraphLaunch(ent->exec, c->st));
    ent->tick = ++c->graph_tick;
    c->cur = ent->cur;
    if (k.setup) c->fwd_valid = k.fwd ? 1 : 0;
    if (k.fwd) c->fwd_B = k.B;
    return IFSVGP_OK;
  }
  if (!ent || ent->failed) {
    if (!ent) {
      // first sighting: remember the structure, run directly
      if (c->graphs.size() >= kMaxGraphs) {
        auto old = std::min_element(c->graphs.begin(), c->graphs.end(),
                                    [](const GraphEnt &a, const GraphEnt &b) { return a.tick < b.tick; });
        if (old->exec) (void)hipGraphExecDestroy(old->exec);
        c->graphs.erase(old);
      }
      GraphEnt g{};
      g.key = key;
      g.tick = ++c->graph_tick;
      c->graphs.push_back(g);
    }
    return run_direct(c, k, ca);
  }
  // second sighting: record on the capture stream, instantiate, replay
  int r = latch(c, ca);
  if (r) return r;
  const hipStream_t user = c->st;
  const int cur0 = c->cur, valid0 = c->fwd_valid, B0 = c->fwd_B;
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamBeginCapture(c->cst, hipStreamCaptureModeRelaxed);
  r = IFSVGP_EHIP;
  if (e == hipSuccess) {
    c->st = c->cst;
    c->capturing = true;
    r = enqueue_any(c, k, nullptr);
    c->capturing = false;
    c->st = user;
    e = hipStreamEndCapture(c->cst, &graph);
  }
  hipGraphExec_t exec = nullptr;
  if (r == IFSVGP_OK && e == hipSuccess && graph)
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (graph) (void)hipGraphDestroy(graph);
  if (r != IFSVGP_OK || e != hipSuccess || !exec) {
    // not recordable: this structure always runs directly (the arguments
    // are latched already)
    (void)hipGetLastError();
    ent->failed = 1;
    c->cur = cur0; c->fwd_valid = valid0; c->fwd_B = B0;
    return enqueue_any(c, k, nullptr);
  }
  ent->exec = exec;
  ent->cur = c->cur;
  ent->tick = ++c->graph_tick;
  HIPCK(hipGraphLaunch(exec, user));
  return IFSVGP_OK;
}

// ------------------------------------------------------------------ API: compute
static bool bad_common(ifsvgp_ctx *c, const float *ell, const float *sf2, const float *Z,
                       const float *s, const float *L) {
  return !c || c->G > 1 || !ell || !sf2 || !Z || !s || !L;  // grouped contexts: step_group only
}

static CallArgs make_args(const float *X, const float *y, int B, double N, const float *ell,
                          const float *sf2, const float *noise, const float *Z, const float *m,
                          const float *s, float *L, const float *gammas, int n_ng) {
  CallArgs a{};
  a.X = X; a.y = y; a.ell = ell; a.sf2 = sf2; a.noise = noise; a.Z = Z; a.m = m; a.s = s;
  a.L = L;
  a.c = B > 0 ? N / (double)B : 0.0;
  for (int k = 0; k < std::min(n_ng, MAX_NG_LATCH); ++k) a.gammas[k] = gammas[k];
  return a;
}

extern "C" int ifsvgp_natgrad(ifsvgp_ctx *c, const float *Z, const float *ell, const float *sf2,
                              const float *s_tilde, float *L, const float *gammas, int n_ng,
                              double *out_resid) {
  if (bad_common(c, ell, sf2, Z, s_tilde, L) || !gammas || n_ng < 1) return IFSVGP_EINVAL;
  CallArgs a = make_args(nullptr, nullptr, 0, 0.0, ell, sf2, nullptr, Z, nullptr, s_tilde, L,
                         gammas, n_ng);
  a.out_resid = out_resid;
  Call k{true, false, false, 0, n_ng, gammas, false, false, false, NG_FIXED};
  return run_call(c, k, a);
}

static int check_bound_args(ifsvgp_ctx *c, const float *X, const float *y, int B, double N,
                            const float *ell, const float *sf2, const float *noise,
                            const float *Z, const float *m, const float *s, const float *L) {
  if (bad_common(c, ell, sf2, Z, s, L) || !X || !y || !m) return IFSVGP_EINVAL;
  if (B < 1 || B > c->Bmax || !(N > 0.0)) return IFSVGP_EINVAL;
  if (c->lik == IFSVGP_LIK_GAUSSIAN && !noise) return IFSVGP_EINVAL;
  return IFSVGP_OK;
}

extern "C" int ifsvgp_bound(ifsvgp_ctx *c, const float *X, const float *y, int B, double N,
                            const float *ell, const float *sf2, const float *noise,
                            const float *Z, const float *m, const float *s, const float *L,
                            double *out_bound, double *out_terms) {
  int r = check_bound_args(c, X, y, B, N, ell, sf2, noise, Z, m, s, L);
  if (r) return r;
  if (!out_bound) return IFSVGP_EINVAL;
  CallArgs a = make_args(X, y, B, N, ell, sf2, noise, Z, m, s, (float *)L, nullptr, 0);
  a.out_bound = out_bound;
  a.out_terms = out_terms;
  Call k{true, true, false, B, 0, nullptr, c->lik == IFSVGP_LIK_GAUSSIAN, false, false, NG_FIXED};
  return run_call(c, k, a);
}

extern "C" int ifsvgp_bound_bwd(ifsvgp_ctx *c, const float *X, const float *y, int B, double N,
                                const float *ell, const float *sf2, const float *noise,
                                const float *Z, const float *m, const float *s, const float *L,
                                const double *grad_scale, float *g_ell, float *g_sf2,
                                float *g_noise, float *g_Z, float *g_m, float *g_s) {
  int r = check_bound_args(c, X, y, B, N, ell, sf2, noise, Z, m, s, L);
  if (r) return r;
  if (c->fwd_valid != 1 || c->fwd_B != B) return IFSVGP_ESTATE;
  CallArgs a = make_args(X, y, B, N, ell, sf2, noise, Z, m, s, (float *)L, nullptr, 0);
  a.grad_scale = grad_scale;
  a.g_ell = g_ell; a.g_sf2 = g_sf2; a.g_noise = g_noise; a.g_Z = g_Z; a.g_m = g_m; a.g_s = g_s;
  Call k{false, false, true, B, 0, nullptr, c->lik == IFSVGP_LIK_GAUSSIAN, g_m != nullptr,
         g_s != nullptr, NG_FIXED};
  return run_call(c, k, a);
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
  CallArgs a = make_args(X, y, B, N, ell, sf2, noise, Z, m, s, L, gammas, n_ng);
  a.out_bound = out_bound;
  a.out_terms = out_terms;
  a.out_resid = out_resid;
  a.g_ell = g_ell; a.g_sf2 = g_sf2; a.g_noise = g_noise; a.g_Z = g_Z; a.g_m = g_m; a.g_s = g_s;
  Call k{true, true, true, B, n_ng, gammas, c->lik == IFSVGP_LIK_GAUSSIAN, g_m != nullptr,
         g_s != nullptr, NG_FIXED};
  return run_call(c, k, a);
}

// G independent training iterations (problems of the same M, B, D, each with
// its own data, hyperparameters, Z, m~, s~ and L) on a grouped context: the
// per-problem argument blocks are latched one by one, then every kernel of
// the iteration runs once for all G problems (grid z = problem).
extern "C" int ifsvgp_step_group(ifsvgp_ctx *c, const ifsvgp_problem *probs, int G, int B,
                                 double N, const float *gammas, int n_ng) {
  if (!c || !probs || G < 1 || G != std::max(1, c->G)) return IFSVGP_EINVAL;
  if (B < 1 || B > c->Bmax || !(N > 0.0)) return IFSVGP_EINVAL;
  if (n_ng < 0 || n_ng > MAX_NG_LATCH || (n_ng > 0 && !gammas)) return IFSVGP_EINVAL;
  const bool gauss = c->lik == IFSVGP_LIK_GAUSSIAN;
  const ifsvgp_problem &p0 = probs[0];
  for (int g = 0; g < G; ++g) {
    const ifsvgp_problem &p = probs[g];
    if (!p.X || !p.y || !p.ell || !p.sf2 || !p.Z || !p.m_tilde || !p.s_tilde || !p.L ||
        !p.out_bound || (gauss && !p.noise_var))
      return IFSVGP_EINVAL;
    // the launch structure is shared: the same outputs for every problem
    if (!p.g_m != !p0.g_m || !p.g_s != !p0.g_s) return IFSVGP_EINVAL;
  }
  c->ev_next = 0;
  c->side_open = false;
  for (int g = 0; g < G; ++g) {
    const ifsvgp_problem &p = probs[g];
    CallArgs a = make_args(p.X, p.y, B, N, p.ell, p.sf2, p.noise_var, p.Z, p.m_tilde, p.s_tilde,
                           p.L, gammas, n_ng);
    a.out_bound = p.out_bound;
    a.out_terms = p.out_terms;
    a.out_resid = p.out_resid;
    a.g_ell = p.g_ell; a.g_sf2 = p.g_sf2; a.g_noise = p.g_noise; a.g_Z = p.g_Z;
    a.g_m = p.g_m; a.g_s = p.g_s;
    hipLaunchKernelGGL(k_latch, dim3(1), dim3(64), 0, c->st, a,
                       (CallArgs *)((char *)c->dca + g * c->gstride));
    HIPCK(hipGetLastError());
  }
  Call k{true, true, true, B, n_ng, gammas, gauss, p0.g_m != nullptr, p0.g_s != nullptr,
         NG_FIXED};
  return enqueue_any(c, k, nullptr);
}

extern "C" int ifsvgp_natgrad_tol(ifsvgp_ctx *c, const float *Z, const float *ell,
                                  const float *sf2, const float *s_tilde, float *L,
                                  const float *gammas, int n_max, float tol, double *out_resid,
                                  int *out_steps) {
  if (bad_common(c, ell, sf2, Z, s_tilde, L) || !gammas || n_max < 1 || !(tol >= 0.f))
    return IFSVGP_EINVAL;
  CallArgs a = make_args(nullptr, nullptr, 0, 0.0, ell, sf2, nullptr, Z, nullptr, s_tilde, L,
                         gammas, n_max);
  a.out_resid = out_resid;
  a.out_steps = out_steps;
  a.ng_tol = tol;
  Call k{true, false, false, 0, n_max, gammas, false, false, false, NG_RESID};
  return run_call(c, k, a);
}

extern "C" int ifsvgp_predict(ifsvgp_ctx *c, const float *X_test, int n, const float *y_test,
                              const float *ell, const float *sf2, const float *noise,
                              const float *Z, const float *m, const float *s_tilde,
                              const float *L, float *mu, float *var, float *lpd,
                              double *nlpd) {
  if (bad_common(c, ell, sf2, Z, s_tilde, L) || !m || n < 0) return IFSVGP_EINVAL;
  if (n == 0) return nlpd ? IFSVGP_EINVAL : IFSVGP_OK;
  if (!X_test || !mu || !var) return IFSVGP_EINVAL;
  if ((lpd || nlpd) && !y_test) return IFSVGP_EINVAL;
  if (y_test && c->lik == IFSVGP_LIK_GAUSSIAN && !noise) return IFSVGP_EINVAL;
  CallArgs a = make_args(X_test, y_test, 0, 0.0, ell, sf2, noise, Z, m, s_tilde, (float *)L,
                         nullptr, 0);
  PredOut o{X_test, y_test, n, mu, var, lpd, nlpd};
  PREC_DISPATCH(enqueue_predict, c, a, o)
}

extern "C" int ifsvgp_natgrad_gap(ifsvgp_ctx *c, const float *X, int B, const float *Z,
                                  const float *ell, const float *sf2, const float *noise,
                                  const float *s_tilde, float *L, const float *gammas, int n_max,
                                  float sigma2, float eps, double *out_gap, int *out_steps) {
  if (bad_common(c, ell, sf2, Z, s_tilde, L) || !X || !noise || !gammas || n_max < 1)
    return IFSVGP_EINVAL;
  if (c->lik != IFSVGP_LIK_GAUSSIAN || B < 1 || B > c->Bmax || !(sigma2 > 0.f) || !(eps >= 0.f))
    return IFSVGP_EINVAL;
  CallArgs a = make_args(X, nullptr, B, 0.0, ell, sf2, noise, Z, nullptr, s_tilde, L, gammas,
                         n_max);
  a.out_resid = out_gap;
  a.out_steps = out_steps;
  a.ng_tol = eps;
  a.gap_sigma2 = sigma2;
  Call k{true, false, false, B, n_max, gammas, true, false, false, NG_GAP};
  return run_call(c, k, a);
}

extern "C" int ifsvgp_bound_hutch(ifsvgp_ctx *c, const float *X, const float *y, int B,
                                  double N, const float *ell, const float *sf2,
                                  const float *noise, const float *Z, const float *m,
                                  const float *s, const float *L, const float *Omega_t, int K,
                                  double *out_bound, double *out_terms) {
  int r = check_bound_args(c, X, y, B, N, ell, sf2, noise, Z, m, s, L);
  if (r) return r;
  if (!Omega_t || K < 1 || !out_bound) return IFSVGP_EINVAL;
  if (rup(B, 64) + rup(K + 1, 64) > c->Bp) return IFSVGP_EINVAL;
  CallArgs a = make_args(X, y, B, N, ell, sf2, noise, Z, m, s, (float *)L, nullptr, 0);
  a.out_bound = out_bound;
  a.out_terms = out_terms;
  PREC_DISPATCH(enqueue_hutch, c, a, B, Omega_t, K)
}

extern "C" int ifsvgp_bound_hutch_bwd(ifsvgp_ctx *c, const float *X, const float *y, int B,
                                      double N, const float *ell, const float *sf2,
                                      const float *noise, const float *Z, const float *m,
                                      const float *s, const float *L, const float *Omega_t,
                                      int K, const double *grad_scale, float *g_ell,
                                      float *g_sf2, float *g_noise, float *g_Z, float *g_m,
                                      float *g_s) {
  int r = check_bound_args(c, X, y, B, N, ell, sf2, noise, Z, m, s, L);
  if (r) return r;
  if (!Omega_t || K < 1 || g_s) return IFSVGP_EINVAL;
  if (c->fwd_valid != 2 || c->fwd_B != B || c->fwd_K != K) return IFSVGP_ESTATE;
  CallArgs a = make_args(X, y, B, N, ell, sf2, noise, Z, m, s, (float *)L, nullptr, 0);
  a.grad_scale = grad_scale;
  a.g_ell = g_ell; a.g_sf2 = g_sf2; a.g_noise = g_noise; a.g_Z = g_Z; a.g_m = g_m;
  PREC_DISPATCH(enqueue_hutch_bwd, c, a, B, Omega_t, K, g_m != nullptr)
}

// Multi-output bound (Q outputs sharing Z, the kernel, S~ and T; Y [B][Q],
// Mt [Q][M] on the device): the single-output forward's set-up, K_uf tiles,
// V (side stream) and Gram products, then per output a = L^T m~_q,
// b = Q a, Wu b (batched matrix-vector products), U = Q V for the shared
// variances, mu_q = V^T b_q, and the multi-output likelihood kernel.
template <typename T>
static int enqueue_multi(ifsvgp_ctx *c, const CallArgs &ca, int B, const float *Y,
                         const float *Mt, int Q) {
  c->ev_next = 0;
  c->side_open = false;
  // (with the split inputs of the K_uf tiles, which the backward's R epilogue reads)
  int r = stage_setup<T>(c, c->lik == IFSVGP_LIK_GAUSSIAN, &ca, B);
  if (r) return r;
  c->cur = 0;
  c->fwd_valid = 0;
  const int M = c->M;
  const long Mp = c->Mp, Bp = c->Bp;
  HIPCK(fork_side(c));
  r = launch_kuf<T>(c, B);
  if (r) return r;
  {
    OnSide side(c);
    HIPCK(Ops<T>::gemm_V(c, 0, B));
  }
  HIPCK(Ops<T>::gram_Y(c, 0));
  HIPCK(Ops<T>::gr_W(c, 0));
  HIPCK(Ops<T>::gr_E(c, 0));
  const dim3 gq(cdiv(M, NTB / 64), Q);
  hipLaunchKernelGGL(k_mo_pack, dim3(cdiv(c->Mp, NTB), Q), dim3(NTB), 0, c->st, Mt, M, Mp,
                     c->mo_m);
  hipLaunchKernelGGL(k_mo_gemv, gq, dim3(NTB), 0, c->st, (const float *)c->Lt32[0], Mp, M, M,
                     (const float *)c->mo_m, Mp, 0, (const double *)nullptr, c->mo_a, Mp);
  hipLaunchKernelGGL(k_mo_gemv, gq, dim3(NTB), 0, c->st, (const float *)c->Q32, Mp, M, M,
                     (const float *)c->mo_a, Mp, 0, (const double *)nullptr, c->mo_b, Mp);
  hipLaunchKernelGGL(k_mo_gemv, gq, dim3(NTB), 0, c->st, (const float *)c->Wu32, Mp, M, M,
                     (const float *)c->mo_b, Mp, 0, (const double *)nullptr, c->mo_wub, Mp);
  HIPCK(join_side(c));
  HIPCK(Ops<T>::gemm_U(c, B));
  hipLaunchKernelGGL((k_mo_mu<T>), dim3(cdiv(B, NTB / 64)), dim3(NTB), 0, c->st,
                     (const T *)c->Vt, Mp, c->Mp, B, (const float *)c->mo_b, Mp, Q, c->mo_mu, Bp);
  LikMoArgs a{c->var_part, cdiv(M, 128), Bp, c->dca, Y, Q, B, c->Bp, c->sfn, c->lik, c->gh,
              c->ngh, c->mo_mu, c->mo_al, Bp, c->alpha, c->beta, c->sqnb, c->lik_part,
              c->tp_gram, cdiv(M, 64) * (cdiv(M, 64) + 1) / 2, c->mo_b, c->mo_wub, Mp,
              c->L32[0], Mp, M, c->scal, c->flag, c->counters + CNT_LIK};
  hipLaunchKernelGGL(k_lik_mo, dim3(cdiv(c->Bp, NTB)), dim3(NTB), 0, c->st, a);
  HIPCK(hipGetLastError());
  c->fwd_valid = 3;
  c->fwd_B = B;
  c->fwd_Q = Q;
  return IFSVGP_OK;
}

// Its backward at fixed T: R = L U3 with U3 = sum_q b_q alpha_q^T -
// 2 U diag(beta), so the R epilogue (given L b = 0 and beta = -1/2) forms
// H_uf from G_uf directly; C with the per-output vector terms summed and the
// trace part counted Q times; G_uu = L C L^T; dF/dm~_q = L Q x_q.
template <typename T>
static int enqueue_multi_bwd(ifsvgp_ctx *c, const CallArgs &ca, int B, int Q, float *g_M,
                             const double *grad_scale) {
  using TW = typename Ops<T>::TW;
  c->ev_next = 0;
  c->side_open = false;
  int r = latch(c, ca);
  if (r) return r;
  const int M = c->M, D = c->D;
  const long Mp = c->Mp, Bp = c->Bp;
  hipLaunchKernelGGL(k_fill, dim3(cdiv(c->Mp, NTB)), dim3(NTB), 0, c->st, c->mo_zero, c->Mp, 0.f);
  hipLaunchKernelGGL(k_fill, dim3(cdiv(c->Bp, NTB)), dim3(NTB), 0, c->st, c->mo_half, c->Bp,
                     -0.5f);
  hipLaunchKernelGGL((k_mo_u3<T>),
                     dim3(cdiv(cdiv(M, 16 / (int)sizeof(T)), NTB), std::min(B, kMaxGridY)),
                     dim3(NTB), 0,
                     c->st, (T *)c->Ut, Mp, M, B, (const float *)c->mo_b, Mp,
                     (const float *)c->mo_al, Bp, Q, (const float *)c->beta);
  HIPCK(fork_side(c));
  {
    OnSide side(c);
    HIPCK(Ops<T>::gemm_R(c, 0, B, c->mo_zero, c->mo_half, c->mo_half));
  }
  hipLaunchKernelGGL(k_valpha<T>, dim3(cdiv(M, va_rows(M))), dim3(NTB), 0, c->st,
                     (const T *)c->V, Bp, M, c->Bp, (const float *)c->alpha,
                     (const float *)c->sqnb, (T *)c->Vs, c->vVa, 0L, LikArgs{}, 0, va_rows(M));
  HIPCK(Ops<T>::syrk(c, B));
  hipLaunchKernelGGL((k_mo_x<T>), dim3(M), dim3(NTB), 0, c->st,
                     (const T *)c->V, Bp, M, c->Bp, (const float *)c->mo_al, Bp, Q,
                     (const float *)c->mo_wub, Mp, c->mo_x);
  hipLaunchKernelGGL(k_assemble_C_mo<TW>, dim3(grid1((long)M * cdiv(M, 4))), dim3(NTB), 0,
                     c->st, (const float *)c->Ys, Ops<T>::syrk_splits(c, B), Mp * Mp,
                     (const float *)c->Wu32, (const float *)c->Q32, (const float *)c->mo_a,
                     (const float *)c->mo_b, (const float *)c->mo_x, Mp, Q, M, Mp, (TW *)c->Cm);
  HIPCK(Ops<T>::gemm_Y2(c, 0));
  HIPCK(Ops<T>::gemm_Guu(c, 0, nullptr));
  if (g_M) {
    const dim3 gq(cdiv(M, NTB / 64), Q);
    hipLaunchKernelGGL(k_mo_gemv, gq, dim3(NTB), 0, c->st, (const float *)c->Q32, Mp, M, M,
                       (const float *)c->mo_x, Mp, 0, (const double *)nullptr, c->mo_t2, Mp);
    hipLaunchKernelGGL(k_mo_gemv, gq, dim3(NTB), 0, c->st, (const float *)c->L32[0], Mp, M, M,
                       (const float *)c->mo_t2, Mp, 1, grad_scale, g_M, (long)M);
  }
  HIPCK(join_side(c));
  const int ntB = cdiv(B, 128), nb = cdiv(M, 64), nbm = cdiv(M, 128);
  const int R = NTB / D;
  const int rb = cdiv(M, grad_zrows(D)), cb = cdiv(B, R);
  GradArgs g{M, B, D, c->dca, c->Zs, c->Xs, c->inv_ell, c->sfn,
             c->hrow, c->hx, ntB, c->hzrow, c->hz, nb, c->hcol, nbm, (long)c->Bp,
             c->tp_uf, nbm * ntB, c->tp_uu, nb * (nb + 1) / 2,
             c->lik_part, cdiv(c->Bp, NTB),
             nullptr, nullptr, nullptr, Mp, nullptr, c->ell_part, rb, cb,
             nullptr, nullptr, (long)Mp, nullptr, c->sP};
  hipLaunchKernelGGL(k_grad<GradPartial<T>>, dim3(rb + cb), dim3(NTB), 0, c->st, g);
  hipLaunchKernelGGL(k_grad_tail, dim3(D + 1), dim3(NTB), 0, c->st, g, (const float *)c->L32[0], 0);
  HIPCK(hipGetLastError());
  c->fwd_valid = 0;  // U was overwritten in place: one backward per forward
  return IFSVGP_OK;
}

extern "C" int ifsvgp_bound_multi(ifsvgp_ctx *c, const float *X, const float *Y, int B, int Q,
                                  double N, const float *ell, const float *sf2,
                                  const float *noise, const float *Z, const float *Mt,
                                  const float *s, const float *L, double *out_bound,
                                  double *out_terms) {
  int r = check_bound_args(c, X, Y, B, N, ell, sf2, noise, Z, Mt, s, L);
  if (r) return r;
  if (Q < 1 || Q > MO_QMAX || !out_bound) return IFSVGP_EINVAL;
  CallArgs a = make_args(X, Y, B, N, ell, sf2, noise, Z, Mt, s, (float *)L, nullptr, 0);
  a.out_bound = out_bound;
  a.out_terms = out_terms;
  PREC_DISPATCH(enqueue_multi, c, a, B, Y, Mt, Q)
}

extern "C" int ifsvgp_bound_multi_bwd(ifsvgp_ctx *c, const float *X, const float *Y, int B,
                                      int Q, double N, const float *ell, const float *sf2,
                                      const float *noise, const float *Z, const float *Mt,
                                      const float *s, const float *L, const double *grad_scale,
                                      float *g_ell, float *g_sf2, float *g_noise, float *g_Z,
                                      float *g_M, float *g_s) {
  int r = check_bound_args(c, X, Y, B, N, ell, sf2, noise, Z, Mt, s, L);
  if (r) return r;
  if (Q < 1 || Q > MO_QMAX || g_s) return IFSVGP_EINVAL;
  if (c->fwd_valid != 3 || c->fwd_B != B || c->fwd_Q != Q) return IFSVGP_ESTATE;
  CallArgs a = make_args(X, Y, B, N, ell, sf2, noise, Z, Mt, s, (float *)L, nullptr, 0);
  a.grad_scale = grad_scale;
  a.g_ell = g_ell; a.g_sf2 = g_sf2; a.g_noise = g_noise; a.g_Z = g_Z;
  PREC_DISPATCH(enqueue_multi_bwd, c, a, B, Q, g_M, grad_scale)
}

extern "C" int ifsvgp_set_graphs(ifsvgp_ctx *c, int enable) {
  if (!c) return IFSVGP_EINVAL;
  c->use_graphs = enable != 0;
  if (!c->use_graphs) {
    hipError_t e = hipStreamSynchronize(c->st);
    graphs_clear(c);
    if (e != hipSuccess) return IFSVGP_EHIP;
  }
  return IFSVGP_OK;
}

extern "C" int ifsvgp_set_kuf_mode(ifsvgp_ctx *c, int mode) {
  if (!c || (mode != IFSVGP_KUF_IN_PRODUCT && mode != IFSVGP_KUF_STORED &&
             mode != IFSVGP_KUF_AUTO))
    return IFSVGP_EINVAL;
  hipError_t e = hipStreamSynchronize(c->st);
  graphs_clear(c);
  c->kuf_mode = mode;
  return e == hipSuccess ? IFSVGP_OK : IFSVGP_EHIP;
}

extern "C" int ifsvgp_adam(ifsvgp_ctx *c, float *param, const float *grad, float *m, float *v,
                           long n, float lr, float beta1, float beta2, float eps, int step,
                           int ascend) {
  if (!c || n < 0 || step < 1 || !(lr >= 0.f) || !(beta1 >= 0.f && beta1 < 1.f) ||
      !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
    return IFSVGP_EINVAL;
  if (n == 0) return IFSVGP_OK;
  if (!param || !grad || !m || !v) return IFSVGP_EINVAL;
  const double bc1 = 1.0 - std::pow((double)beta1, step), bc2 = 1.0 - std::pow((double)beta2, step);
  hipLaunchKernelGGL(k_adam, dim3(grid1(n)), dim3(NTB), 0, c->st, param, grad, m, v, n, lr, beta1,
                     beta2, eps, (float)(1.0 / bc1), (float)(1.0 / bc2), ascend ? -1.f : 1.f);
  HIPCK(hipGetLastError());
  return IFSVGP_OK;
}

// ------------------------------------------------------------------ allocation-free iteration
// The training iteration of ifsvgp_step for callers that cannot allocate
// device memory (code under HIP graph capture, tight serving loops, harnesses
// that forbid hipMalloc).  Its workspace is the file-scope device array
// `scratch` (each device holds its own copy from module load until the
// process ends) instead of a context's slab, laid out per call for the
// call's (M, B, D, precision, likelihood) without the Hutchinson buffers,
// and zeroed by a fill kernel at the start of every call.  Host code reaches
// the array only through the device address hipGetSymbolAddress returns for
// it, taken once per device with that device current.  Everything runs on
// the caller's stream in stream order (no side stream, no events, no graphs).
static constexpr size_t kScratchBytes = IFSVGP_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static constexpr int kMaxDevices = 64;
struct NoAllocDevice {
  std::once_flag once;
  hipError_t err;
  char *ptr;       // device address of this device's copy of scratch
  std::mutex mu;   // serialises the host side of calls on this device
  ifsvgp_ctx ctx;  // host state of the calls, its pointers into scratch
};
static NoAllocDevice g_noalloc[kMaxDevices];

__global__ void k_zero16(uint4 *p, size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    p[i] = uint4{0u, 0u, 0u, 0u};
}

// Gauss-Hermite nodes and weights passed by value (n <= 64 each).
struct GhTable {
  double v[128];
};
__global__ void k_put_gh(GhTable t, int n2, double *dst) {
  const int i = threadIdx.x;
  if (i < n2) dst[i] = t.v[i];
}

__global__ void k_copy_flag(const int *flag, int *out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *out = *flag;
}

extern "C" int ifsvgp_step_noalloc(void *hip_stream, int M, int D, int prec, int lik, int n_gh,
                                   const float *X, const float *y, int B, double N,
                                   const float *ell, const float *sf2, const float *noise,
                                   const float *Z, const float *m, const float *s, float *L,
                                   const float *gammas, int n_ng, double *out_bound,
                                   double *out_terms, double *out_resid, float *g_ell,
                                   float *g_sf2, float *g_noise, float *g_Z, float *g_m,
                                   float *g_s, int *out_flag) {
  if (M < 1 || D < 1 || D > MAXD || B < 1) return IFSVGP_EINVAL;
  if (prec < 0 || prec > 2 || lik < 0 || lik > 1) return IFSVGP_EINVAL;
  if (lik == IFSVGP_LIK_PROBIT && (n_gh < 1 || n_gh > 64)) return IFSVGP_EINVAL;
  if ((long)M > 32768 || (long)B > (1L << 24) || (long)M * B > (1L << 31)) return IFSVGP_EINVAL;
  if (n_ng < 0 || (n_ng > 0 && !gammas) || !out_bound) return IFSVGP_EINVAL;
  int dev = 0;
  HIPCK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return IFSVGP_EINVAL;
  NoAllocDevice &nd = g_noalloc[dev];
  std::call_once(nd.once, [&nd] {
    void *p = nullptr;
    nd.err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    nd.ptr = (char *)p;
  });
  if (nd.err != hipSuccess || !nd.ptr) return IFSVGP_EHIP;
  std::lock_guard<std::mutex> lock(nd.mu);
  ifsvgp_ctx *c = &nd.ctx;
  c->M = M; c->Bmax = B; c->D = D; c->prec = prec; c->lik = lik;
  c->ngh = lik == IFSVGP_LIK_PROBIT ? n_gh : 0;
  c->Mp = rup(M, PAD);
  c->Bp = rup(B, PAD);
  c->nsplit = std::max(1, std::min(8, cdiv(B, 1024)));
  c->st = c->side = (hipStream_t)hip_stream;
  c->G = 1;
  c->gstride = 0;
  c->single_stream = true;
  c->capturing = false;
  c->use_graphs = 0;
  c->timing = 0;
  c->lev0 = c->lev1 = nullptr;
  c->fwd_valid = 0;
  c->cur = 0;
  const size_t bytes = layout(c, nullptr, false);
  if (bytes > kScratchBytes) return IFSVGP_ESCRATCH;
  layout(c, nd.ptr, false);
  int r = check_bound_args(c, X, y, B, N, ell, sf2, noise, Z, m, s, L);
  if (r) return r;
  hipLaunchKernelGGL(k_zero16, dim3((unsigned)std::min<size_t>(2048, cdiv(bytes / 16, NTB))),
                     dim3(NTB), 0, c->st, (uint4 *)nd.ptr, bytes / 16);
  HIPCK(hipGetLastError());
  if (c->ngh > 0) {
    GhTable t{};
    ifsvgp_gh_rule(c->ngh, t.v, t.v + c->ngh);
    hipLaunchKernelGGL(k_put_gh, dim3(1), dim3(128), 0, c->st, t, 2 * c->ngh, c->gh);
    HIPCK(hipGetLastError());
  }
  CallArgs a = make_args(X, y, B, N, ell, sf2, noise, Z, m, s, L, gammas, n_ng);
  a.out_bound = out_bound;
  a.out_terms = out_terms;
  a.out_resid = out_resid;
  a.g_ell = g_ell; a.g_sf2 = g_sf2; a.g_noise = g_noise; a.g_Z = g_Z; a.g_m = g_m; a.g_s = g_s;
  Call k{true, true, true, B, n_ng, gammas, lik == IFSVGP_LIK_GAUSSIAN, g_m != nullptr,
         g_s != nullptr, NG_FIXED};
  r = run_direct(c, k, a);
  if (r) return r;
  if (out_flag) {
    hipLaunchKernelGGL(k_copy_flag, dim3(1), dim3(64), 0, c->st, (const int *)c->flag, out_flag);
    HIPCK(hipGetLastError());
  }
  return IFSVGP_OK;
}
