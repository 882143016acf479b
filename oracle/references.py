"""Independent reference quantities that pin the oracle (float64, CPU).

TEST INFRASTRUCTURE ONLY (see the package docstring).

None of these evaluate the inverse-free bound itself; they compute what the
paper says the bound must agree with or stay below:

* ``cholesky_elbo``        -- the standard (M-SVGP, Section 2) ELBO of an
                              explicit Gaussian q(u) = N(m, S), via Cholesky
                              solves; the R-SVGP bound equals it at T = K~^{-1}
                              (Section 2, R-SVGP paragraph and Section 3.2) and
                              is a valid ELBO below it for any T.
* ``cholesky_predict``     -- M-SVGP predictive marginals of an explicit q(u)
                              at new inputs, via Cholesky solves.
* ``induced_q``            -- the q(u) that a given T induces when substituted
                              into M-SVGP (Section 3.2, text before eq.
                              rsvgp_precond): m = K_uu P m~, S = K_uu - K_uu P K_uu.
* ``log_marginal_likelihood`` -- exact GP evidence (Gaussian, full batch).
* ``lsvgp_precond_bound``  -- preconditioned L-SVGP bound with the exact
                              inverse P = K~^{-1} (Section S2, eq.
                              kl_lsvgp_app); Prop. 2 equates its gradient with
                              the R-SVGP one at T = stopgrad(K~^{-1}).
* ``rsvgp_bound_unpreconditioned`` -- the earlier bound of eq. kl_rsvgp
                              (mean m = K_uu m~), maximised over T at K~^{-1}.
* ``fisher_natgrad``       -- textbook Fisher natural gradient of
                              KL[N(0, L L^T) || N(0, A^{-1})] on the
                              lower-triangular coordinates of L, built from the
                              Gaussian Fisher 1/2 tr(S^-1 dS S^-1 dS) and a
                              finite-difference gradient (Prop. 1 brute force).
* ``central_fd``           -- central finite differences.
"""
import numpy as np
from scipy.linalg import cho_factor, cho_solve

from .svgp import se_ard
from .quadrature import expectation


def _logdet_chol(A):
    c, low = cho_factor(A, lower=True)
    return 2.0 * np.sum(np.log(np.diag(c))), (c, low)


def gauss_kl(m, S, K):
    """KL[N(m, S) || N(0, K)] via Cholesky factorisations."""
    M = K.shape[0]
    ldK, cK = _logdet_chol(K)
    ldS, _ = _logdet_chol(S)
    return 0.5 * (np.trace(cho_solve(cK, S)) + m @ cho_solve(cK, m) - M
                  + ldK - ldS)


def cholesky_elbo(X, y, N, ell, sf2, noise_var, Z, qm, qS, lik="gaussian",
                  n_gh=20):
    """M-SVGP ELBO (Section 2) of q(u) = N(qm, qS) on a mini-batch."""
    X, y, ell, Z, qm, qS = [np.asarray(a, np.float64)
                            for a in (X, y, ell, Z, qm, qS)]
    B = X.shape[0]
    Kuu = se_ard(Z, Z, ell, sf2)
    Kuf = se_ard(Z, X, ell, sf2)
    _, cK = _logdet_chol(Kuu)
    A = cho_solve(cK, Kuf)                      # K_uu^{-1} k_un
    mu = A.T @ qm
    var = sf2 - np.sum(Kuf * A, axis=0) + np.sum(A * (qS @ A), axis=0)
    E, _, _, _ = expectation(lik, y, mu, var, noise_var, n_gh)
    KL = gauss_kl(qm, qS, Kuu)
    return dict(F=(N / B) * np.sum(E) - KL, KL=KL, mu=mu, var=var)


def cholesky_predict(Xt, ell, sf2, Z, qm, qS):
    """M-SVGP predictive marginals of q(u) = N(qm, qS) at test inputs
    (Section 2, M-SVGP): mu = k_*u K_uu^{-1} qm and
    sigma^2 = k_** - k_*u K_uu^{-1} k_u* + k_*u K_uu^{-1} qS K_uu^{-1} k_u*,
    via Cholesky solves."""
    Xt, ell, Z, qm, qS = [np.asarray(a, np.float64) for a in (Xt, ell, Z, qm, qS)]
    Kuu = se_ard(Z, Z, ell, sf2)
    Kus = se_ard(Z, Xt, ell, sf2)
    _, cK = _logdet_chol(Kuu)
    A = cho_solve(cK, Kus)
    mu = A.T @ qm
    var = sf2 - np.sum(Kus * A, axis=0) + np.sum(A * (qS @ A), axis=0)
    return mu, var


def induced_q(ell, sf2, Z, m, s, L):
    """q(u) = N(K_uu P m~, K_uu - K_uu P K_uu), P = 2T - T K~ T, T = L L^T."""
    Z, m, s, L = [np.asarray(a, np.float64) for a in (Z, m, s, L)]
    Kuu = se_ard(Z, Z, ell, sf2)
    Kt = Kuu + np.diag(s)
    T = L @ L.T
    P = 2.0 * T - T @ Kt @ T
    return Kuu @ P @ m, Kuu - Kuu @ P @ Kuu


def lsvgp_q(ell, sf2, Z, m, s):
    """L-SVGP q(u) with mean preconditioning: m = K_uu K~^{-1} m~,
    S = (K_uu^{-1} + S~^{-1})^{-1} (Woodbury form, Section 2 L-SVGP)."""
    Z, m, s = [np.asarray(a, np.float64) for a in (Z, m, s)]
    Kuu = se_ard(Z, Z, ell, sf2)
    Kt = Kuu + np.diag(s)
    qm = Kuu @ np.linalg.solve(Kt, m)
    qS = np.linalg.inv(np.linalg.inv(Kuu) + np.diag(1.0 / s))
    return qm, 0.5 * (qS + qS.T)


def log_marginal_likelihood(X, y, ell, sf2, noise_var):
    """log N(y | 0, K_ff + sigma^2 I) by Cholesky."""
    X, y = np.asarray(X, np.float64), np.asarray(y, np.float64)
    K = se_ard(X, X, ell, sf2) + noise_var * np.eye(X.shape[0])
    ld, c = _logdet_chol(K)
    return -0.5 * (y @ cho_solve(c, y) + ld + X.shape[0] * np.log(2 * np.pi))


def lsvgp_precond_bound(X, y, N, ell, sf2, noise_var, Z, m, s, lik="gaussian",
                        n_gh=20):
    """Preconditioned L-SVGP bound with P = K~^{-1} (Section S2)."""
    X, y, ell, Z, m, s = [np.asarray(a, np.float64)
                          for a in (X, y, ell, Z, m, s)]
    B, M = X.shape[0], Z.shape[0]
    Kuu = se_ard(Z, Z, ell, sf2)
    Kuf = se_ard(Z, X, ell, sf2)
    Kt = Kuu + np.diag(s)
    ldKt, c = _logdet_chol(Kt)
    P = cho_solve(c, np.eye(M))
    mu = Kuf.T @ (P @ m)
    var = sf2 - np.sum(Kuf * (P @ Kuf), axis=0)
    E, _, _, _ = expectation(lik, y, mu, var, noise_var, n_gh)
    KL = 0.5 * (-np.trace(P @ Kuu) + m @ P @ Kuu @ P @ m + ldKt
                - np.sum(np.log(s)))
    return (N / B) * np.sum(E) - KL


def rsvgp_bound_unpreconditioned(X, y, N, ell, sf2, noise_var, Z, m, s, L,
                                 lik="gaussian", n_gh=20):
    """Bound of eq. kl_rsvgp with the L-SVGP mean m = K_uu m~ (no preconditioner)."""
    X, y, ell, Z, m, s, L = [np.asarray(a, np.float64)
                             for a in (X, y, ell, Z, m, s, L)]
    B, M = X.shape[0], Z.shape[0]
    Kuu = se_ard(Z, Z, ell, sf2)
    Kuf = se_ard(Z, X, ell, sf2)
    Kt = Kuu + np.diag(s)
    T = L @ L.T
    P = 2.0 * T - T @ Kt @ T
    mu = Kuf.T @ m
    var = sf2 - np.sum(Kuf * (P @ Kuf), axis=0)
    E, _, _, _ = expectation(lik, y, mu, var, noise_var, n_gh)
    logdetT = 2.0 * np.sum(np.log(np.abs(np.diag(L))))
    KL = 0.5 * (-np.trace(P @ Kuu) - M + m @ Kuu @ m + np.trace(Kt @ T)
                - logdetT - np.sum(np.log(s)))
    return (N / B) * np.sum(E) - KL


def central_fd(f, x, idx, h):
    """Central differences of scalar f at array x along flat indices idx."""
    x = np.array(x, np.float64)
    g = np.empty(len(idx))
    for k, i in enumerate(idx):
        xp = x.copy()
        xm = x.copy()
        xp.flat[i] += h
        xm.flat[i] -= h
        g[k] = (f(xp) - f(xm)) / (2.0 * h)
    return g


def _gauss_kl_zero_mean(Sigma, A):
    """KL[N(0, Sigma) || N(0, A^{-1})] = 1/2 (tr(A Sigma) - M - log|A| - log|Sigma|)."""
    M = Sigma.shape[0]
    return 0.5 * (np.trace(A @ Sigma) - M - np.linalg.slogdet(A)[1]
                  - np.linalg.slogdet(Sigma)[1])


def fisher_natgrad(L, A, h=1e-6):
    """F^{-1} g on the lower-triangular coordinates of L (brute force, tiny M).

    F_ab = 1/2 tr(S^{-1} dS_a S^{-1} dS_b) with S = L L^T and
    dS_a = E_a L^T + L E_a^T (the textbook Fisher information of a zero-mean
    Gaussian); g = central finite differences of the KL objective.
    """
    L = np.array(L, np.float64)
    M = L.shape[0]
    coords = [(i, j) for i in range(M) for j in range(i + 1)]
    S = L @ L.T
    Si = np.linalg.inv(S)
    dS = []
    for (i, j) in coords:
        E = np.zeros((M, M))
        E[i, j] = 1.0
        dS.append(E @ L.T + L @ E.T)
    n = len(coords)
    Fm = np.empty((n, n))
    for a in range(n):
        for b in range(n):
            Fm[a, b] = 0.5 * np.trace(Si @ dS[a] @ Si @ dS[b])

    def loss(Lv):
        return _gauss_kl_zero_mean(Lv @ Lv.T, A)

    g = np.empty(n)
    for a, (i, j) in enumerate(coords):
        Lp = L.copy()
        Lm = L.copy()
        Lp[i, j] += h
        Lm[i, j] -= h
        g[a] = (loss(Lp) - loss(Lm)) / (2 * h)
    x = np.linalg.solve(Fm, g)
    G = np.zeros((M, M))
    for a, (i, j) in enumerate(coords):
        G[i, j] = x[a]
    return G
