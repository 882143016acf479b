/*
 * ifsvgp.h -- C ABI of the MI355X (gfx950) inverse-free sparse variational GP
 * training iteration.
 *
 * Method: Cortinovis, Aitchison, Eleftheriadis, van der Wilk, "Inverse-Free
 * Sparse Variational Gaussian Processes".  One training iteration is
 *   (1) t* natural-gradient steps on the factor L of the auxiliary matrix
 *       T = L L^T towards chol(K~^{-1}), K~ = K_uu + diag(s~)
 *       (Prop. 1, eq. natgrad; alternating scheme of Section 3.1);
 *   (2) the preconditioned inverse-free bound at the updated L
 *       (Section 3.2, eq. rsvgp_precond), with the mini-batch data term
 *       F = (N/B) sum_n E_q[log p(y_n | f_n)] - KL;
 *   (3) the gradient of that bound with respect to the kernel lengthscales,
 *       signal variance, noise variance, inducing inputs Z, inducing mean m~
 *       (and optionally s~), with T held fixed (stopgrad, Section 3.1 and the
 *       proof of Prop. 2 in Section S2).
 * Kernel: ARD squared exponential k(x,x') = sf2 exp(-1/2 sum_d (x_d-x'_d)^2/ell_d^2)
 * (Section 4, Section S5).  Likelihoods: Gaussian with variance noise_var, or
 * Bernoulli with probit link p(y|f) = Phi(y f), y in {-1,+1}, whose expectation
 * is the n_gh-point Gauss-Hermite rule over q(f_n) (Section S5, Model Setup).
 *
 * Conventions common to every entry point
 * ---------------------------------------
 * - All tensor arguments are DEVICE pointers to caller-owned, contiguous,
 *   row-major arrays on the device that was current when the context was
 *   created.  float = IEEE fp32, double = fp64.  The library keeps no pointer
 *   past the return of a call.
 * - Shapes: X is B x D, y is B, ell is D, sf2/noise_var are 1 element,
 *   Z is M x D, m_tilde and s_tilde are M, L is M x M.
 * - L is the lower-triangular factor of T.  Only its lower triangle
 *   (diagonal included) is read; updated values are written to the lower
 *   triangle only; the strict upper triangle is never read or written.
 * - Work is enqueued asynchronously on the context's HIP stream
 *   (ifsvgp_set_stream); no call synchronises the device except
 *   ifsvgp_status and ifsvgp_timing_read.
 * - Return codes: IFSVGP_OK or a negative IFSVGP_E* code.  Argument errors
 *   are detected on the host before any work is enqueued (IFSVGP_EINVAL).
 *   Value errors that live in device memory (non-positive ell, sf2, noise_var
 *   or s~, a zero diagonal entry of L, a non-finite bound) set a sticky
 *   device flag; ifsvgp_status reports and clears it.  Nothing throws across
 *   the ABI.
 * - A context is bound to one stream and is not thread-safe.  Calls on one
 *   context run in stream order and reuse its workspace.
 */
#ifndef IFSVGP_H
#define IFSVGP_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ifsvgp_ctx ifsvgp_ctx;

/* GEMM operand precision.  FP32: every product in fp32 on fp32 MFMA.
 * BF16 / FP16: the cubic and B*M^2 products take bf16 / fp16 operands with
 * fp32 accumulation (FP16 keeps the two products with the backward's M x M
 * matrix C in fp32, whose entries can exceed the fp16 range); the master L,
 * the kernel-matrix exponentials, the likelihood terms and all reductions
 * stay fp32 and the final scalar sums are fp64. */
enum ifsvgp_prec { IFSVGP_PREC_FP32 = 0, IFSVGP_PREC_BF16 = 1, IFSVGP_PREC_FP16 = 2 };

enum ifsvgp_lik { IFSVGP_LIK_GAUSSIAN = 0, IFSVGP_LIK_PROBIT = 1 };

enum ifsvgp_status_code {
  IFSVGP_OK = 0,
  IFSVGP_EINVAL = -1,      /* bad argument (null pointer, size, enum)          */
  IFSVGP_EDOMAIN = -2,     /* ell, sf2, noise_var or s~ <= 0, or L_ii == 0     */
  IFSVGP_EHIP = -3,        /* a HIP runtime call failed                        */
  IFSVGP_ENONFINITE = -4,  /* the bound or the updated L is not finite         */
  IFSVGP_ENOMEM = -5,      /* workspace allocation failed                      */
  IFSVGP_ESTATE = -6,      /* ifsvgp_bound_bwd without a matching forward      */
  IFSVGP_ESCRATCH = -7     /* too large for ifsvgp_step_noalloc's workspace    */
};

/* Indices into out_terms[IFSVGP_N_TERMS] (device fp64). */
enum ifsvgp_term {
  IFSVGP_TERM_DATA = 0,    /* (N/B) sum_n E_n                                  */
  IFSVGP_TERM_KL = 1,      /* KL upper bound of eq. rsvgp_precond              */
  IFSVGP_TERM_SUMVAR = 2,  /* sum_n sigma_n^2                                  */
  IFSVGP_TERM_RESID = 3,   /* ||L^T K~ L - I||_F / sqrt(M) at the bound's L    */
  IFSVGP_TERM_TRW = 4,     /* tr(K~ T)                                         */
  IFSVGP_TERM_TRPK = 5,    /* tr(P K_uu), P = 2T - T K~ T                      */
  IFSVGP_TERM_QUAD = 6,    /* m~^T P K_uu P m~                                 */
  IFSVGP_TERM_LOGDET = 7,  /* log|T| = 2 sum_i log|L_ii|                       */
  IFSVGP_N_TERMS = 8
};

/* Library version as an integer (major*10000 + minor*100 + patch). */
int ifsvgp_version(void);

/* Human-readable text for a status code.  Never NULL. */
const char *ifsvgp_strerror(int code);

/* Create a context for problems of M inducing points, mini-batches of at
 * most B_max rows and D input dimensions.  prec: enum ifsvgp_prec.  lik:
 * enum ifsvgp_lik.  n_gh: Gauss-Hermite points for the probit likelihood
 * (1..64; ignored for Gaussian).  Allocates the whole device workspace on the
 * current device (sizes grow as M^2 + M*B_max).  Stream: the null stream
 * until ifsvgp_set_stream.  *out is set only on IFSVGP_OK.  Sizes outside
 * 1 <= M <= 32768, 1 <= B_max <= 2^24, M*B_max <= 2^31, 1 <= D <= 64 return
 * IFSVGP_EINVAL before the device is touched. */
int ifsvgp_create(ifsvgp_ctx **out, int M, int B_max, int D, int prec, int lik, int n_gh);

/* Release the workspace.  The caller must make sure queued work has finished
 * (or the stream is synchronised) first.  NULL is accepted. */
void ifsvgp_destroy(ifsvgp_ctx *ctx);

/* Bind the context to a HIP stream (hipStream_t passed as void*). */
int ifsvgp_set_stream(ifsvgp_ctx *ctx, void *hip_stream);

/* Recorded calls (HIP graphs).  Off by default.  With enable = 1, the
 * second call on a context with the same launch structure (entry point, B,
 * n_ng up to 64, which of g_m / g_s are requested, and for ifsvgp_bound_bwd
 * the preceding forward's NG step parity) records that call's launches into
 * a HIP graph, and later calls with that structure replay it with one graph
 * launch on the context's stream, for any argument buffers: the caller's
 * pointers and scalars reach the kernels through a small device block
 * written at the start of every call.  Results are bit-identical to direct
 * execution.  A replay takes the host less time than the direct launches but
 * the GPU somewhat more, so it helps callers whose launch rate limits them.
 * enable = 0 synchronises the stream, frees the recorded graphs and runs
 * every later call directly; calls with timing enabled always run directly.
 * Up to 16 structures are kept (least recently used replaced). */
int ifsvgp_set_graphs(ifsvgp_ctx *ctx, int enable);

/* Where the bf16 / fp16 forms form the tiles of K_uf (the data-inducing
 * block of the SE-ARD kernel, Section 2) for V = L^T K_uf.
 * IFSVGP_KUF_IN_PRODUCT (the default): each tile is generated in LDS inside
 * the product's workgroups and K_uf is never stored.  IFSVGP_KUF_STORED: the
 * same generator writes the tiles once into the workspace, beside the
 * natural-gradient step, and the product loads them (faster for large
 * problems, whose triangular product otherwise regenerates every tile
 * M / 256 times on average, at the cost of an M x B store).
 * IFSVGP_KUF_AUTO: stored from M * B = 2^23 on.  All modes use the same
 * arithmetic, so results are bit-identical and only the step time differs;
 * the backward recomputes its tiles in every mode.  The fp32 form always
 * stores K_uf (computed from differences with the accurate exp).
 * Synchronises the stream and drops recorded graphs.  IFSVGP_EINVAL for
 * another mode. */
#define IFSVGP_KUF_IN_PRODUCT 0
#define IFSVGP_KUF_STORED 1
#define IFSVGP_KUF_AUTO 2
int ifsvgp_set_kuf_mode(ifsvgp_ctx *ctx, int mode);

/* Synchronise the stream, then report and clear the sticky device flag:
 * IFSVGP_OK, IFSVGP_EDOMAIN or IFSVGP_ENONFINITE. */
int ifsvgp_status(ifsvgp_ctx *ctx);

/* Physicists' Gauss-Hermite rule with n points (host only, no device use):
 * nodes t_k and weights w_k with sum_k w_k g(t_k) ~ int exp(-t^2) g(t) dt.
 * Computed by Newton iteration on the three-term Hermite recurrence.
 * nodes/weights are HOST arrays of n doubles.  Returns IFSVGP_EINVAL unless
 * 1 <= n <= 64. */
int ifsvgp_gh_rule(int n, double *nodes, double *weights);

/* Natural-gradient steps only (Prop. 1): builds K~ from (Z, ell, sf2, s_tilde)
 * and runs n_ng >= 1 steps L <- L - gammas[t] * L [tril(W) - (I + diag W)/2],
 * W = L^T K~ L, in place on L.  gammas: HOST array of n_ng floats.
 * out_resid: device fp64[n_ng] (may be NULL) receiving ||W - I||_F/sqrt(M)
 * measured before each step (eq. stopping_frobenius). */
int ifsvgp_natgrad(ifsvgp_ctx *ctx, const float *Z, const float *ell, const float *sf2,
                   const float *s_tilde, float *L, const float *gammas, int n_ng,
                   double *out_resid);

/* Adaptive natural-gradient loop (Section 3.3, eq. stopping_frobenius): up to
 * n_max steps as in ifsvgp_natgrad, where before step t the residual
 * r_t = ||L^T K~ L - I||_F / sqrt(M) of the current iterate is formed from the
 * step's own W, and the loop stops, without applying step t, as soon as
 * r_t < tol.  No host synchronisation: after the stop the remaining launches
 * skip their products and pass L through unchanged, so L holds the last
 * applied update.  out_resid: device fp64[n_max] (may be NULL) receiving r_t
 * for the checked steps and the stopping residual for the steps after it.
 * out_steps: device int[1] (may be NULL) receiving the number of updates
 * applied (0..n_max).  gammas: HOST array of n_max floats.  tol >= 0. */
int ifsvgp_natgrad_tol(ifsvgp_ctx *ctx, const float *Z, const float *ell, const float *sf2,
                       const float *s_tilde, float *L, const float *gammas, int n_max,
                       float tol, double *out_resid, int *out_steps);

/* Prediction at n >= 0 test inputs (Section 2: the marginals mu_n, sigma_n^2
 * of eq. elbo at new inputs, with P = 2T - T K~ T of eq. rsvgp_precond and
 * T = L L^T as given, no NG step; Section 4 reports the NLPD built from
 * them):
 *   mu[i]  = k(x_i, Z) P m~,   var[i] = sf2 - k(x_i, Z) P k(Z, x_i)   (latent f),
 * and with targets y_test the log predictive density of each point,
 *   Gaussian: lpd[i] = log N(y_i; mu[i], var[i] + noise_var),
 *   probit:   lpd[i] = log Phi(y_i mu[i] / sqrt(1 + var[i])), y_i in {-1, +1},
 * and *nlpd = -(1/n) sum_i lpd[i] (fp64 sum).
 * X_test: device fp32 [n][D] row-major; y_test: device fp32 [n] or NULL;
 * mu, var: device fp32 [n] (required); lpd: device fp32 [n] or NULL;
 * nlpd: device fp64 [1] or NULL.  lpd / nlpd require y_test; noise_var is
 * required with y_test for the Gaussian likelihood and otherwise unread.
 * Points are processed in chunks of B_max; n may exceed B_max.  The call
 * reuses the bound's workspace, so a following ifsvgp_bound_bwd needs a new
 * forward first (IFSVGP_ESTATE otherwise).  n = 0 does nothing (and is
 * IFSVGP_EINVAL when nlpd is requested). */
int ifsvgp_predict(ifsvgp_ctx *ctx, const float *X_test, int n, const float *y_test,
                   const float *ell, const float *sf2, const float *noise_var,
                   const float *Z, const float *m_tilde, const float *s_tilde,
                   const float *L, float *mu, float *var, float *lpd, double *nlpd);

/* Adaptive natural-gradient loop with the variance-gap rule (Section 3.3,
 * Prop. 3; Gaussian likelihood only): as ifsvgp_natgrad_tol, but before step t
 * the gap of the current iterate on the batch X (B <= B_max rows),
 *   G_t = sum_n ||(I - K~ T) k(Z, x_n)||^2 / sigma2,   T = L L^T,
 * is formed (from V = L^T K_uf, Y = K~ L and K_uf - Y V: two M x M x B and one
 * M x M x M product per step), and the loop stops, without applying step t,
 * as soon as G_t <= 2 noise_var eps.  sigma2 splits S~ = S~' + sigma2 I with
 * S~' positive, so 0 < sigma2 < min s_tilde makes G the summed slack between
 * the bounds of eq. lsvgp_ub and eq. lsvgp_lb (only sigma2 > 0 is checked).
 * noise_var: device fp32[1], the Gaussian noise variance.  out_gap: device
 * fp64[n_max] (may be NULL) receiving G_t for the checked steps and the
 * stopping value after the stop; out_steps as in ifsvgp_natgrad_tol.
 * IFSVGP_EINVAL for a probit context, B outside 1..B_max, sigma2 <= 0 or
 * eps < 0. */
int ifsvgp_natgrad_gap(ifsvgp_ctx *ctx, const float *X, int B, const float *Z,
                       const float *ell, const float *sf2, const float *noise_var,
                       const float *s_tilde, float *L, const float *gammas, int n_max,
                       float sigma2, float eps, double *out_gap, int *out_steps);

/* Bound evaluation with Hutchinson trace estimates (Section 3.4, bound
 * evaluation): as ifsvgp_bound, but the cubic trace terms of the KL bound are
 * replaced by unbiased estimates from K probe vectors, so no M x M x M product
 * is formed (cost O((B + K) M^2)).  With W = L^T K~ L and Wu = L^T K_uu L,
 *   tr W ~ (1/K) sum_k w_k^T W w_k,  tr Wu ~ (1/K) sum_k w_k^T Wu w_k,
 *   tr(W Wu) ~ (1/K) sum_k (W w_k)^T (Wu w_k),
 * and tr(P K_uu) = 2 tr Wu - tr(W Wu), tr(K~ T) = tr W.  The data term, the
 * mean term m~^T P K_uu P m~ and log|T| are exact (sigma_n^2 from
 * U = 2V - W V, V = L^T K_uf).  Omega_t: device fp32 [K][M] row-major, probe k
 * in row k (draw them with E[w w^T] = I, e.g. Rademacher; the caller's draw is
 * used as given).  Requires round_up(B, 64) + round_up(K + 1, 64) <=
 * round_up(B_max, 128) (IFSVGP_EINVAL otherwise).  out_terms as for
 * ifsvgp_bound, with the NG residual entry 0.  Its gradient comes from
 * ifsvgp_bound_hutch_bwd; ifsvgp_bound_bwd after it needs a new ifsvgp_bound
 * (IFSVGP_ESTATE otherwise). */
int ifsvgp_bound_hutch(ifsvgp_ctx *ctx, const float *X, const float *y, int B, double N_total,
                       const float *ell, const float *sf2, const float *noise_var,
                       const float *Z, const float *m_tilde, const float *s_tilde,
                       const float *L, const float *Omega_t, int K, double *out_bound,
                       double *out_terms);

/* Gradient of the preceding ifsvgp_bound_hutch's estimate F_K (Section 3.4)
 * with the probes and T = L L^T held fixed, with respect to ell, sf2,
 * noise_var, Z and m_tilde (outputs as in ifsvgp_bound_bwd, each may be
 * NULL; grad_scale likewise).  The trace part of the adjoint of the
 * cubic traces becomes, in L-space, (1/4K) [Omega (Omega - G)^T + its
 * transpose] with G = (W + Wu) Omega; the data side is that of the exact
 * backward.  Omega_t, K, B and the inputs must be those of the forward
 * (IFSVGP_ESTATE when the last forward on ctx was not a Hutchinson bound
 * with this B and K; the probes themselves are not compared).  The
 * gradient with respect to s_tilde is not offered: g_s must be NULL
 * (IFSVGP_EINVAL otherwise).  No M x M x M product is formed: the adjoint
 * C of the bound with respect to L^T K~ L is a rank-(B + 2K + 3) form
 * X S X^T, so L C L^T = (L X) S (L X)^T costs O((B + K) M^2). */
int ifsvgp_bound_hutch_bwd(ifsvgp_ctx *ctx, const float *X, const float *y, int B,
                           double N_total, const float *ell, const float *sf2,
                           const float *noise_var, const float *Z, const float *m_tilde,
                           const float *s_tilde, const float *L, const float *Omega_t, int K,
                           const double *grad_scale, float *g_ell, float *g_sf2,
                           float *g_noise_var, float *g_Z, float *g_m, float *g_s);

/* Multi-output bound (Section 4, multi-output layers with S~ tied across
 * outputs): Q outputs (1 <= Q <= 16) share Z, ell, sf2, noise_var, s_tilde and
 * so one T = L L^T; output q has its own inducing mean (row q of Mt, device
 * fp32 [Q][M]) and targets (column q of Y, device fp32 [B][Q] row-major).
 * The outputs are independent SVGPs given the shared quantities, so F is the
 * sum of the single-output bounds of eq. rsvgp_precond, each with its own KL
 * (trace and log-determinant terms included).  sigma_n^2 is shared; the means
 * are mu_qn = k_n^T P m~_q.  out_terms: data and KL summed over outputs,
 * sum_n sigma_n^2, the NG residual of W, tr W and tr(Q Wu) of one output, the
 * summed mean terms sum_q m~_q^T P K_uu P m~_q and log|T|.  Other arguments
 * as for ifsvgp_bound; IFSVGP_EINVAL for Q outside 1..16. */
int ifsvgp_bound_multi(ifsvgp_ctx *ctx, const float *X, const float *Y, int B, int Q,
                       double N_total, const float *ell, const float *sf2,
                       const float *noise_var, const float *Z, const float *Mt,
                       const float *s_tilde, const float *L, double *out_bound,
                       double *out_terms);

/* Gradient of the preceding ifsvgp_bound_multi's F at fixed T: the shared
 * parameters' gradients (ell, sf2, noise_var, Z) are sums over outputs, g_M
 * (device fp32 [Q][M]) holds dF/dm~_q in row q; each output may be NULL,
 * grad_scale as for ifsvgp_bound_bwd.  The gradient with respect to s_tilde
 * is not offered (g_s must be NULL, IFSVGP_EINVAL otherwise).  One backward
 * per forward: the call consumes the forward state (IFSVGP_ESTATE when the
 * last call on ctx was not an ifsvgp_bound_multi with this B and Q). */
int ifsvgp_bound_multi_bwd(ifsvgp_ctx *ctx, const float *X, const float *Y, int B, int Q,
                           double N_total, const float *ell, const float *sf2,
                           const float *noise_var, const float *Z, const float *Mt,
                           const float *s_tilde, const float *L, const double *grad_scale,
                           float *g_ell, float *g_sf2, float *g_noise_var, float *g_Z,
                           float *g_M, float *g_s);

/* Bound only, at the given L (eq. rsvgp_precond).  B <= B_max rows, N_total
 * the data-set size (the data term is scaled by N_total / B).  noise_var is
 * read only for the Gaussian likelihood (may be NULL for probit).
 * out_bound: device fp64[1] = F.  out_terms: device fp64[IFSVGP_N_TERMS] or
 * NULL.  The intermediates of this call stay in the workspace for a following
 * ifsvgp_bound_bwd with identical arguments. */
int ifsvgp_bound(ifsvgp_ctx *ctx, const float *X, const float *y, int B, double N_total,
                 const float *ell, const float *sf2, const float *noise_var,
                 const float *Z, const float *m_tilde, const float *s_tilde,
                 const float *L, double *out_bound, double *out_terms);

/* Gradient of the bound evaluated by the immediately preceding
 * ifsvgp_bound / ifsvgp_step on this context, which must have received the
 * same arguments (IFSVGP_ESTATE if there was none or B differs).  K_uf tiles
 * are recomputed, not stored.  grad_scale: device fp64[1] multiplying every
 * gradient (e.g. the incoming adjoint), or NULL for 1.  Gradient outputs are
 * device fp32 arrays shaped like their parameters; each may be NULL to skip
 * it.  g_s (dF/ds~) adds one triangular M^3 product, diag(L Q L^T) with
 * Q = 2I - L^T K~ L, and runs only when requested.  The gradient is of F (to
 * be maximised) with respect to the constrained values. */
int ifsvgp_bound_bwd(ifsvgp_ctx *ctx, const float *X, const float *y, int B, double N_total,
                     const float *ell, const float *sf2, const float *noise_var,
                     const float *Z, const float *m_tilde, const float *s_tilde,
                     const float *L, const double *grad_scale,
                     float *g_ell, float *g_sf2, float *g_noise, float *g_Z,
                     float *g_m, float *g_s);

/* One full training iteration in the order of Section 3.1: n_ng >= 0 NG
 * steps on L (in place, gammas on the host, out_resid as in
 * ifsvgp_natgrad), then the bound and its gradient at the updated L.
 * Arguments as in ifsvgp_natgrad / ifsvgp_bound / ifsvgp_bound_bwd. */
int ifsvgp_step(ifsvgp_ctx *ctx, const float *X, const float *y, int B, double N_total,
                const float *ell, const float *sf2, const float *noise_var,
                const float *Z, const float *m_tilde, const float *s_tilde,
                float *L, const float *gammas, int n_ng,
                double *out_bound, double *out_terms, double *out_resid,
                float *g_ell, float *g_sf2, float *g_noise, float *g_Z,
                float *g_m, float *g_s);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * training iteration of ifsvgp_step without a context.  It calls no
 * hipMalloc, hipFree, stream or event creation.  Its workspace is a static
 * device array of 64 MiB (IFSVGP_NOALLOC_SCRATCH_BYTES) that every device
 * the library runs on holds from module load until the process ends; the
 * call lays the workspace out for its own (M, B, D, prec, lik), and returns
 * IFSVGP_ESCRATCH, with nothing enqueued, when that exceeds the array (for
 * example M = 512, B = 1024, D = 8 fits in fp32; M = 1024, B = 4096 does not).
 * A fill kernel zeroes the used part at the start of every call, so no state
 * carries over between calls; the array keeps the last call's contents
 * until the next one.  All work is enqueued on hip_stream (hipStream_t
 * passed as void*; the device current at the call must own it), in stream
 * order, and may be captured into a HIP graph by the caller.  Calls that
 * overlap on one device race on its array: the host side of calls from
 * several threads is serialised per device, but the caller must keep the
 * GPU work of two calls on one device in order (one stream, or events).
 * Arguments and results are those of ifsvgp_step (device pointers; gammas
 * on the host; gradient outputs may be NULL; B >= 1 is the batch size, with
 * no separate B_max), plus the context's creation parameters M, D, prec,
 * lik and n_gh as in ifsvgp_create.  Device value errors are not kept in a
 * sticky flag: out_flag (device int[1] or NULL) receives this call's flag
 * bits, 0 when clean, 1 for a domain error (non-positive ell, sf2,
 * noise_var or s~, or L_ii == 0), 2 for a non-finite bound or factor. */
#define IFSVGP_NOALLOC_SCRATCH_BYTES (64u << 20)
int ifsvgp_step_noalloc(void *hip_stream, int M, int D, int prec, int lik, int n_gh,
                        const float *X, const float *y, int B, double N_total,
                        const float *ell, const float *sf2, const float *noise_var,
                        const float *Z, const float *m_tilde, const float *s_tilde, float *L,
                        const float *gammas, int n_ng, double *out_bound, double *out_terms,
                        double *out_resid, float *g_ell, float *g_sf2, float *g_noise,
                        float *g_Z, float *g_m, float *g_s, int *out_flag);

/* Independent problems in one launch per kernel (Section 4: deep GPs give
 * every layer its own Z, kernel hyperparameters, S~ and so its own T; a layer
 * with S~ tied across its outputs has one T, see ifsvgp_bound_multi).  A
 * grouped context holds the workspaces of G problems of the same sizes
 * (M, B_max, D, prec, lik), one after another; ifsvgp_step_group runs the
 * training iteration of ifsvgp_step for all G at once, every kernel of the
 * iteration launched once with the problem as its grid's third index, so G
 * small problems cost the launches of one.  A grouped context serves only
 * ifsvgp_step_group (and ifsvgp_adam, ifsvgp_set_stream, ifsvgp_status,
 * ifsvgp_timing_*); the single-problem entry points return IFSVGP_EINVAL on
 * it.  ifsvgp_status reports (and clears) the flags of all G problems.
 * 1 <= G <= IFSVGP_MAX_GROUP (G = 1 is an ordinary context, on which
 * ifsvgp_step_group with one problem equals ifsvgp_step). */
#define IFSVGP_MAX_GROUP 64
int ifsvgp_create_group(ifsvgp_ctx **out, int G, int M, int B_max, int D, int prec, int lik,
                        int n_gh);

/* One problem of a group: the arguments of ifsvgp_step (device pointers). */
typedef struct ifsvgp_problem {
  const float *X, *y, *ell, *sf2, *noise_var, *Z, *m_tilde, *s_tilde;
  float *L;
  double *out_bound, *out_terms, *out_resid;
  float *g_ell, *g_sf2, *g_noise, *g_Z, *g_m, *g_s;
} ifsvgp_problem;

/* The training iteration of ifsvgp_step for the G problems of probs (a HOST
 * array of G entries, G equal to the context's group size), all on batches of
 * B rows with the same data-set size N_total and the same NG step sizes
 * (gammas: host, n_ng <= 64).  Each problem's results go to its own outputs,
 * as ifsvgp_step would write them.  Every problem must request the same
 * optional outputs among g_m and g_s (they shape the launches; IFSVGP_EINVAL
 * otherwise); the others may differ.  Results are bit-identical to G
 * separate ifsvgp_step calls on ungrouped contexts. */
int ifsvgp_step_group(ifsvgp_ctx *ctx, const ifsvgp_problem *probs, int G, int B,
                      double N_total, const float *gammas, int n_ng);

/* One Adam step (Kingma and Ba's algorithm, with bias correction) on n fp32
 * parameters, enqueued on the context's stream: with g' = grad (or -grad when
 * ascend != 0, to maximise F), m = beta1 m + (1-beta1) g',
 * v = beta2 v + (1-beta2) g'^2 and
 * param -= lr * (m / (1 - beta1^step)) / (sqrt(v / (1 - beta2^step)) + eps).
 * param, m, v are updated in place (device fp32 arrays of n elements; m and v
 * start at zero before step 1); step >= 1 counts this parameter's updates.
 * Positivity of constrained parameters is the caller's transform.  For
 * callers that want a training loop without other device compute; it is not
 * part of the timed iteration.  Returns IFSVGP_EINVAL for a bad size, step,
 * rate or decay. */
int ifsvgp_adam(ifsvgp_ctx *ctx, float *param, const float *grad, float *m, float *v, long n,
                float lr, float beta1, float beta2, float eps, int step, int ascend);

/* Per-kernel timing for profiling.  kind_mask selects kernel kinds (bit k
 * for kind k, as indexed by ifsvgp_timing_read; -1 for all, 0 to stop);
 * every launch of a selected kind is bracketed by HIP events on the
 * context's stream.  ifsvgp_timing_read synchronises, accumulates the
 * elapsed times since the last read, and returns the number of kernel kinds;
 * for kind k < cap it writes the total milliseconds, launch count and a
 * static name (each array may be NULL). */
int ifsvgp_timing_enable(ifsvgp_ctx *ctx, long long kind_mask);
int ifsvgp_timing_read(ifsvgp_ctx *ctx, int cap, double *total_ms, int *count,
                       const char **names);

/* Algorithmic flop count of one launch of each kernel kind for batch size B
 * (the count used for roofline fractions; triangular operands at their
 * nonzero density, symmetric outputs once).  Same indexing and names as
 * ifsvgp_timing_read; names may be NULL.  Returns the number of kinds. */
int ifsvgp_kernel_flops(ifsvgp_ctx *ctx, int B, int cap, double *flops, const char **names);

#ifdef __cplusplus
}
#endif
#endif /* IFSVGP_H */
