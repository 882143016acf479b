"""Inverse-free SVGP (R-SVGP with inducing-mean preconditioning) in float64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Notation follows the paper:
  K_uu = k(Z, Z), K_uf = k(Z, X_b), k_nn = sigma_f^2          (Section 2, M-SVGP)
  K~ = K_uu + S~,  S~ = diag(s~)                               (Section 2, L-SVGP)
  T = L L^T, L lower triangular                                (Section 3.1)
  P = 2 T - T K~ T                                             (Section 3.2)
  mu_n = k_nu P m~,  sigma_n^2 = k_nn - k_nu P k_un             (eq. rsvgp_precond)
  KL <= 1/2 ( -tr(P K_uu) + tr(K~ T) - M + m~^T P K_uu P m~
              - log|T| - log|S~| )                             (eq. rsvgp_precond)
  F = (N / B) sum_{n in batch} E_n - KL                        (eq. elbo, mini-batch)
  at test inputs: the same mu_*, sigma_*^2, and the log predictive
  density whose negated mean is the NLPD (Section 4)           (predict)

Natural-gradient step on L (Prop. 1, eq. natgrad; alternating scheme of
Section 3.1):
  W = L^T K~ L,  L <- L - gamma L [ tril(W) - 1/2 (I + diag(W)) ],
with tril keeping the diagonal, and the stopping residual of eq.
stopping_frobenius:  r = ||W - I||_F / sqrt(M).

The gradient of F with respect to xi = {lengthscales, sigma_f^2, noise
variance, Z, m~, s~} holds T fixed (stopgrad, Section 3.1 and the proof of
Prop. 2 in Section S2).  It is written here as the adjoint of the literal
formulas above (explicit P, T), not in any factored form.
"""
import numpy as np
from scipy.special import log_ndtr

from .quadrature import expectation


# ----------------------------------------------------------------------------
# Covariance (ARD RBF kernel, Section 4 and Section S5)
# ----------------------------------------------------------------------------
def sq_dist_scaled(A, Bm, ell):
    """sum_d (a_d - b_d)^2 / ell_d^2 for every pair of rows, chunked over A."""
    A = np.asarray(A, np.float64) / ell
    Bm = np.asarray(Bm, np.float64) / ell
    out = np.empty((A.shape[0], Bm.shape[0]))
    step = max(1, int(2**24 // max(1, Bm.shape[0] * A.shape[1])))
    for i0 in range(0, A.shape[0], step):
        diff = A[i0:i0 + step, None, :] - Bm[None, :, :]
        out[i0:i0 + step] = np.sum(diff * diff, axis=-1)
    return out


def se_ard(A, Bm, ell, sf2):
    """k(a, b) = sigma_f^2 exp(-1/2 sum_d (a_d - b_d)^2 / ell_d^2)."""
    return sf2 * np.exp(-0.5 * sq_dist_scaled(A, Bm, ell))


def ktilde(Z, ell, sf2, s):
    """K~ = K_uu + diag(s~) (Section 2, L-SVGP)."""
    return se_ard(Z, Z, ell, sf2) + np.diag(np.asarray(s, np.float64))


# ----------------------------------------------------------------------------
# Natural gradient for T = L L^T (Prop. 1, Section 3.1)
# ----------------------------------------------------------------------------
def natgrad_direction(L, A):
    """L [tril(L^T A L) - 1/2 (I + diag(L^T A L))]  (eq. natgrad)."""
    L = np.asarray(L, np.float64)
    W = L.T @ A @ L
    M = L.shape[0]
    X = np.tril(W) - 0.5 * (np.eye(M) + np.diag(np.diag(W)))
    return L @ X


def ng_residual(L, A):
    """||L^T A L - I||_F / sqrt(M)  (eq. stopping_frobenius)."""
    L = np.asarray(L, np.float64)
    M = L.shape[0]
    return np.linalg.norm(L.T @ A @ L - np.eye(M), "fro") / np.sqrt(M)


def ng_steps(L, A, gammas):
    """Run len(gammas) NG steps L <- L - gamma_t * natgrad; returns (L, residuals).

    residuals[t] is measured at the iterate *before* step t, from the same
    W = L^T A L that the step uses.
    """
    L = np.array(L, np.float64)
    res = []
    for g in gammas:
        res.append(ng_residual(L, A))
        L = L - g * natgrad_direction(L, A)
    return L, np.array(res)


def ng_steps_adaptive(L, A, gammas, tol):
    """NG steps stopped by the residual (Section 3.3, eq. stopping_frobenius).

    Before step t the residual r_t of the current iterate is measured from the
    same W = L^T A L that the step would use; the loop stops, without applying
    step t, as soon as r_t < tol, and otherwise applies step t with gammas[t].
    At most len(gammas) steps.  Returns (L, residuals measured, steps applied).
    """
    L = np.array(L, np.float64)
    res = []
    for g in gammas:
        r = ng_residual(L, A)
        res.append(r)
        if r < tol:
            break
        L = L - g * natgrad_direction(L, A)
    applied = len(res) - (1 if res and res[-1] < tol else 0)
    return L, np.array(res), applied


def variance_gap(L, A, Kuf, sigma2):
    """G = sum_n ||(I - K~ T) k_un||^2 / sigma^2 with T = L L^T and A = K~
    (Prop. 3 and the text after it): the summed slack between the upper
    bound U_n of eq. lsvgp_ub and the lower bound L_n of eq. lsvgp_lb, where
    sigma^2 splits S~ = S~' + sigma^2 I (0 < sigma^2 < min s~)."""
    L, A, Kuf = _as64(L, A, Kuf)
    T = L @ L.T
    R = Kuf - A @ (T @ Kuf)
    return float(np.sum(R * R)) / float(sigma2)


def ng_steps_gap(L, A, Kuf, gammas, sigma2, noise_obs, eps):
    """NG steps stopped by the variance gap (Section 3.3, Gaussian likelihood):
    before step t the gap G_t of the current iterate is measured, and the loop
    stops, without applying step t, as soon as G_t <= 2 sigma_obs^2 eps;
    otherwise it applies step t with gammas[t].  At most len(gammas) steps.
    Returns (L, gaps measured, steps applied)."""
    L = np.array(L, np.float64)
    thr = 2.0 * float(noise_obs) * float(eps)
    gaps = []
    for g in gammas:
        G = variance_gap(L, A, Kuf, sigma2)
        gaps.append(G)
        if G <= thr:
            break
        L = L - g * natgrad_direction(L, A)
    applied = len(gaps) - (1 if gaps and gaps[-1] <= thr else 0)
    return L, np.array(gaps), applied


def loglinear_gammas(n, g0=1e-5, g1=1.0, ramp=10, start=0):
    """Log-linear step-size schedule of Section 3.4: g0 -> g1 over `ramp` steps.

    Step t (counting from the start of training) uses
    10^(log10 g0 + (log10 g1 - log10 g0) * min(t, ramp-1)/(ramp-1)).
    """
    out = []
    for t in range(start, start + n):
        f = min(t, ramp - 1) / (ramp - 1)
        out.append(10.0 ** (np.log10(g0) + (np.log10(g1) - np.log10(g0)) * f))
    return np.array(out)


# ----------------------------------------------------------------------------
# The preconditioned R-SVGP bound (eq. rsvgp_precond)
# ----------------------------------------------------------------------------
def _as64(*xs):
    return [np.asarray(x, np.float64) for x in xs]


def _perturbed(K, perturb, key):
    """K * (1 + perturb[key]) when a relative perturbation is supplied.

    Used only to measure how much rounding of the formed kernel matrices moves
    the results (tests set their tolerances from it); None leaves K exact."""
    if perturb is None or key not in perturb:
        return K
    return K * (1.0 + perturb[key])


def rsvgp_bound(X, y, N, ell, sf2, noise_var, Z, m, s, L, lik="gaussian",
                n_gh=20, return_parts=False, perturb=None):
    """Evaluate F = (N/B) sum_n E_n - KL at T = L L^T, literally.

    Returns a dict with F, data (the scaled expected log likelihood), KL,
    sum_var (sum_n sigma_n^2), mu (B), var (B), and the per-datum E_n.
    perturb: optional dict of relative perturbations of the formed K_uu
    ('Kuu', M x M) and K_uf ('Kuf', M x B).
    """
    X, y, ell, Z, m, s, L = _as64(X, y, ell, Z, m, s, L)
    sf2 = float(sf2)
    B = X.shape[0]
    M = Z.shape[0]
    Kuu = _perturbed(se_ard(Z, Z, ell, sf2), perturb, "Kuu")
    Kuf = _perturbed(se_ard(Z, X, ell, sf2), perturb, "Kuf")
    Kt = Kuu + np.diag(s)
    T = L @ L.T
    P = 2.0 * T - T @ Kt @ T
    mu = Kuf.T @ (P @ m)
    var = sf2 - np.sum(Kuf * (P @ Kuf), axis=0)
    E, _, _, _ = expectation(lik, y, mu, var, noise_var, n_gh)
    data = (N / B) * np.sum(E)
    logdetT = 2.0 * np.sum(np.log(np.abs(np.diag(L))))
    KL = 0.5 * (-np.trace(P @ Kuu) + np.trace(Kt @ T) - M
                + m @ P @ Kuu @ P @ m - logdetT - np.sum(np.log(s)))
    out = dict(F=data - KL, data=data, KL=KL, sum_var=np.sum(var),
               mu=mu, var=var, E=E)
    if return_parts:
        out.update(Kuu=Kuu, Kuf=Kuf, Kt=Kt, T=T, P=P)
    return out


def rsvgp_bound_hutchinson(X, y, N, ell, sf2, noise_var, Z, m, s, L, Omega,
                           lik="gaussian", n_gh=20, perturb=None):
    """The bound with its cubic trace terms replaced by Hutchinson estimates
    (Section 3.4, bound evaluation), literally.

    Omega: M x K probe matrix (its columns are the probes, E[w w^T] = I).  The
    traces are those of the L-space products
        W = L^T K~ L   (tr W = tr(K~ T))  and  Wu = L^T K_uu L,
    with tr(P K_uu) = 2 tr(Wu) - tr(W Wu), each estimated as
    tr(A) ~ (1/K) sum_k w_k^T A w_k (for W Wu: (W w_k)^T (Wu w_k)).  The data
    term, m~^T P K_uu P m~, log|T| and log|S~| are exact.  Returns the dict of
    rsvgp_bound (F, data, KL, sum_var, mu, var, E) plus the estimated traces
    trW, trWu, trWWu.  perturb: as in rsvgp_bound."""
    X, y, ell, Z, m, s, L, Omega = _as64(X, y, ell, Z, m, s, L, Omega)
    sf2 = float(sf2)
    B = X.shape[0]
    M, K = Omega.shape
    Kuu = _perturbed(se_ard(Z, Z, ell, sf2), perturb, "Kuu")
    Kuf = _perturbed(se_ard(Z, X, ell, sf2), perturb, "Kuf")
    Kt = Kuu + np.diag(s)
    T = L @ L.T
    P = T @ (2.0 * np.eye(M) - Kt @ T)
    Pm = P @ m
    mu = Kuf.T @ Pm
    var = sf2 - np.einsum("in,in->n", Kuf, P @ Kuf)
    E, _, _, _ = expectation(lik, y, mu, var, noise_var, n_gh)
    data = N / B * E.sum()
    W = L.T @ Kt @ L
    Wu = L.T @ Kuu @ L
    WO, WuO = W @ Omega, Wu @ Omega
    trW = np.sum(Omega * WO) / K
    trWu = np.sum(Omega * WuO) / K
    trWWu = np.sum(WO * WuO) / K
    trPK = 2.0 * trWu - trWWu
    quad = Pm @ Kuu @ Pm
    logdet = 2.0 * np.log(np.abs(np.diag(L))).sum()
    KL = 0.5 * (trW - trPK - M + quad - logdet - np.log(s).sum())
    return dict(F=data - KL, data=data, KL=KL, sum_var=np.sum(var), mu=mu, var=var, E=E,
                trW=trW, trWu=trWu, trWWu=trWWu)


def rsvgp_bound_grad(X, y, N, ell, sf2, noise_var, Z, m, s, L, lik="gaussian",
                     n_gh=20, perturb=None, Omega=None):
    """Gradient of rsvgp_bound w.r.t. xi at fixed T (adjoint of the literal form).

    Returns dict: ell (D), sf2, noise_var (Gaussian only, else 0), Z (MxD),
    m (M), s (M), plus the bound dict under key 'bound'.  perturb: as in
    rsvgp_bound.  Omega (M x K probes, optional): the gradient of the
    Hutchinson-estimated bound of rsvgp_bound_hutchinson instead, at fixed
    probes.
    """
    X, y, ell, Z, m, s, L = _as64(X, y, ell, Z, m, s, L)
    sf2 = float(sf2)
    B, D = X.shape
    c = N / B
    bd = rsvgp_bound(X, y, N, ell, sf2, noise_var, Z, m, s, L, lik, n_gh,
                     return_parts=True, perturb=perturb)
    Kuu, Kuf, T, P = bd["Kuu"], bd["Kuf"], bd["T"], bd["P"]
    mu, var = bd["mu"], bd["var"]
    _, dmu, dv, ds2 = expectation(lik, y, mu, var, noise_var, n_gh)
    alpha = c * dmu            # dF/dmu_n
    beta = c * dv              # dF/dsigma_n^2

    Pm = P @ m
    # Coefficient of dP in dF (symmetrised), collecting:
    #   data:  sum_n alpha_n k_n^T dP m~  -  sum_n beta_n k_n^T dP k_n
    #   -KL:   +1/2 tr(dP K_uu)  -  1/2 d(m~^T P K_uu P m~)|_P
    Ka = Kuf @ alpha
    G_P = 0.5 * (np.outer(Ka, m) + np.outer(m, Ka))
    G_P -= (Kuf * beta[None, :]) @ Kuf.T
    if Omega is None:
        G_P += 0.5 * Kuu
    KPm = Kuu @ Pm
    G_P -= 0.5 * (np.outer(KPm, m) + np.outer(m, KPm))
    if Omega is None:
        # dP = -T dK~ T (T fixed); plus -KL's -1/2 tr(T dK~)
        G_Kt = -T @ G_P @ T - 0.5 * T
        # direct K_uu dependence of -KL: +1/2 tr(P dK_uu) - 1/2 (Pm)^T dK_uu (Pm)
        G_Kuu = 0.5 * P - 0.5 * np.outer(Pm, Pm) + G_Kt
    else:
        # the estimated traces, with T_Om = L (Omega Omega^T / K) L^T:
        # -KL's trace part = tr(K_uu T_Om) - 1/2 tr(K~ T K_uu T_Om) - 1/2 tr(K~ T_Om)
        Om = np.asarray(Omega, np.float64)
        TO = L @ (Om @ Om.T / Om.shape[1]) @ L.T
        A1 = T @ Kuu @ TO     # d/dK~ of tr(K~ T K_uu T_Om) is A1^T (symmetrised below)
        A2 = T @ bd["Kt"] @ TO  # d/dK_uu (direct) of the same trace is A2
        G_Kt = -T @ G_P @ T - 0.25 * (A1 + A1.T) - 0.5 * TO
        G_Kuu = TO - 0.25 * (A2 + A2.T) - 0.5 * np.outer(Pm, Pm) + G_Kt
        bd = dict(bd, **{k: v for k, v in rsvgp_bound_hutchinson(
            X, y, N, ell, sf2, noise_var, Z, m, s, L, Om, lik, n_gh, perturb).items()
            if k in ("F", "data", "KL")})
    # K_uf: alpha_n (P m~)^T dk_n  - 2 beta_n (P k_n)^T dk_n
    G_Kuf = np.outer(Pm, alpha) - 2.0 * (P @ Kuf) * beta[None, :]
    # m~: sum_n alpha_n k_n^T P dm~  - (P K_uu P m~)^T dm~
    g_m = P @ Ka - P @ KPm
    # s~: through K~ (diagonal) and -KL's +1/2 sum log s~
    g_s = np.diag(G_Kt) + 0.5 / s

    # SE-ARD chain rule.  dK/dsf2 = K/sf2; dK/dell_d = K (a_d-b_d)^2/ell_d^3;
    # dK_ab/da_d = -K (a_d - b_d)/ell_d^2.
    Huu = G_Kuu * Kuu
    Huf = G_Kuf * Kuf
    g_sf2 = (np.sum(Huu) + np.sum(Huf)) / sf2 + np.sum(beta)
    g_ell = np.zeros(D)
    g_Z = np.zeros_like(Z)
    # the same sums over absolute values of their terms: the scale against
    # which any floating-point evaluation of these sums must be judged
    a_ell = np.zeros(D)
    a_Z = np.zeros_like(Z)
    for d in range(D):
        dzz = Z[:, d][:, None] - Z[:, d][None, :]
        dzx = Z[:, d][:, None] - X[:, d][None, :]
        g_ell[d] = (np.sum(Huu * dzz**2) + np.sum(Huf * dzx**2)) / ell[d]**3
        a_ell[d] = (np.sum(np.abs(Huu) * dzz**2) + np.sum(np.abs(Huf) * dzx**2)) / ell[d]**3
        # K_uu[i,j] depends on Z_i through row i and column i
        g_Z[:, d] = -(np.sum((Huu + Huu.T) * dzz, axis=1)
                      + np.sum(Huf * dzx, axis=1)) / ell[d]**2
        a_Z[:, d] = (np.sum(np.abs(Huu + Huu.T) * np.abs(dzz), axis=1)
                     + np.sum(np.abs(Huf * dzx), axis=1)) / ell[d]**2
    a_sf2 = (np.sum(np.abs(Huu)) + np.sum(np.abs(Huf))) / sf2 + np.sum(np.abs(beta))
    # s~: diag(G_Kt) = diag(G_Kuu) - diag(P)/2 + (P m~)^2/2, each term's size
    a_s = np.abs(np.diag(G_Kuu)) + 0.5 * np.abs(np.diag(P)) + 0.5 * Pm**2 + 0.5 / s
    g_noise = c * np.sum(ds2) if ds2 is not None else 0.0
    return dict(ell=g_ell, sf2=g_sf2, noise_var=g_noise, Z=g_Z, m=g_m, s=g_s,
                bound=bd, alpha=alpha, beta=beta,
                abs_terms=dict(ell=a_ell, Z=a_Z, sf2=a_sf2, s=a_s))


def predict(Xt, ell, sf2, Z, m, s, L, y=None, noise_var=None, lik="gaussian",
            perturb=None):
    """Predictive marginals at test inputs, literally (Section 2, eq. elbo's
    mu_n and sigma_n^2, with P of eq. rsvgp_precond):
        mu_* = k_*u P m~,  sigma_*^2 = k_** - k_*u P k_u*,  P = 2T - T K~ T,
    for the latent f.  With targets y, the log predictive density per point
    (its negated mean is the NLPD of Section 4's UCI experiments):
        Gaussian:  log N(y; mu_*, sigma_*^2 + noise_var),
        probit:    log Phi(y mu_* / sqrt(1 + sigma_*^2)),  y in {-1, +1}.
    Returns (mu, var, lpd); lpd is None without y.
    perturb: optional relative perturbations of the formed K_uu ('Kuu') and
    K_u* ('Kus'), as in rsvgp_bound."""
    Xt, ell, Z, m, s, L = _as64(Xt, ell, Z, m, s, L)
    sf2 = float(sf2)
    Kus = _perturbed(se_ard(Z, Xt, ell, sf2), perturb, "Kus")
    Kt = _perturbed(se_ard(Z, Z, ell, sf2), perturb, "Kuu") + np.diag(s)
    T = L @ L.T
    P = 2.0 * T - T @ (Kt @ T)
    mu = Kus.T @ (P @ m)
    var = sf2 - np.sum(Kus * (P @ Kus), axis=0)
    if y is None:
        return mu, var, None
    y = np.asarray(y, np.float64)
    if lik == "gaussian":
        vy = var + float(noise_var)
        lpd = -0.5 * np.log(2.0 * np.pi * vy) - (y - mu) ** 2 / (2.0 * vy)
    elif lik == "probit":
        lpd = log_ndtr(y * mu / np.sqrt(1.0 + var))
    else:
        raise ValueError(f"unknown likelihood {lik!r}")
    return mu, var, lpd


def training_iteration(X, y, N, ell, sf2, noise_var, Z, m, s, L, gammas,
                       lik="gaussian", n_gh=20, with_grad=True, perturb=None):
    """One iteration in the order of Section 3.1: NG steps on L with K~(xi),
    then bound (and gradient) at the updated L.  Returns (L_new, res, out).
    perturb: as in rsvgp_bound (applied to K_uu in the NG steps as well)."""
    Kuu = _perturbed(se_ard(Z, Z, ell, sf2), perturb, "Kuu")
    Kt = Kuu + np.diag(np.asarray(s, np.float64))
    L_new, res = ng_steps(L, Kt, gammas)
    if with_grad:
        out = rsvgp_bound_grad(X, y, N, ell, sf2, noise_var, Z, m, s, L_new,
                               lik, n_gh, perturb=perturb)
    else:
        out = dict(bound=rsvgp_bound(X, y, N, ell, sf2, noise_var, Z, m, s,
                                     L_new, lik, n_gh, perturb=perturb))
    return L_new, res, out


def multi_output_bound(X, Y, N, ell, sf2, noise_var, Z, Mt, s, L, lik="gaussian", n_gh=20,
                       perturb=None):
    """Q outputs sharing Z, the kernel hyperparameters and one S~, hence one
    T = L L^T (Section 4, multi-output layers with S~ tied across outputs);
    output q has its own inducing mean m~_q (row q of Mt, Q x M) and targets
    Y[:, q] (Y is B x Q).  The outputs are independent SVGPs given these
    shared quantities, so the bound is the sum over q of eq. rsvgp_precond's
    bound, each with its whole KL.  Returns F, data, KL (sums over outputs),
    sum_var (sum_n sigma_n^2, the same for every output) and mu (Q x B)."""
    Y = np.asarray(Y, np.float64).reshape(np.shape(X)[0], -1)
    Mt = np.atleast_2d(np.asarray(Mt, np.float64))
    parts = [rsvgp_bound(X, Y[:, q], N, ell, sf2, noise_var, Z, Mt[q], s, L, lik, n_gh,
                         perturb=perturb) for q in range(Mt.shape[0])]
    return dict(F=sum(p["F"] for p in parts), data=sum(p["data"] for p in parts),
                KL=sum(p["KL"] for p in parts), sum_var=parts[0]["sum_var"],
                mu=np.stack([p["mu"] for p in parts]), var=parts[0]["var"])


def multi_output_bound_grad(X, Y, N, ell, sf2, noise_var, Z, Mt, s, L, lik="gaussian",
                            n_gh=20, perturb=None):
    """Gradient of multi_output_bound at fixed T: for the shared parameters
    (ell, sf2, noise_var, Z, s~) the sum of the per-output gradients, for m~_q
    output q's own (m: Q x M).  abs_terms: the per-output absolute term sums
    added up (a bound on the scale of the combined sums)."""
    Y = np.asarray(Y, np.float64).reshape(np.shape(X)[0], -1)
    Mt = np.atleast_2d(np.asarray(Mt, np.float64))
    gs = [rsvgp_bound_grad(X, Y[:, q], N, ell, sf2, noise_var, Z, Mt[q], s, L, lik, n_gh,
                           perturb=perturb) for q in range(Mt.shape[0])]
    out = {k: sum(g[k] for g in gs) for k in ("ell", "sf2", "noise_var", "Z", "s")}
    out["m"] = np.stack([g["m"] for g in gs])
    out["abs_terms"] = {k: sum(g["abs_terms"][k] for g in gs) for k in gs[0]["abs_terms"]}
    out["bound"] = multi_output_bound(X, Y, N, ell, sf2, noise_var, Z, Mt, s, L, lik, n_gh,
                                      perturb=perturb)
    return out
