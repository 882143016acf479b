"""Pins of the float64 oracle against what the paper and the mathematics fix.

No test here re-types an oracle formula and compares it with itself.  Each
one checks the oracle against an independent quantity: a Cholesky-based ELBO,
the exact GP evidence, a textbook Fisher natural gradient built by brute
force, adaptive quadrature, finite differences, or an identity the paper
proves (equality at T = K~^{-1}, bound validity, Newton-Schulz error
squaring, Prop. 2, Prop. 3).
"""
import numpy as np
import pytest
from scipy import integrate
from scipy.special import gamma as gamma_fn, log_ndtr

from oracle import svgp, references as ref, quadrature as quad


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def small_problem(seed=0, M=6, B=9, D=2, N=40.0, lik="gaussian"):
    g = _rng(seed)
    X = g.standard_normal((B, D))
    if lik == "gaussian":
        y = np.sin(X.sum(1)) + 0.1 * g.standard_normal(B)
    else:
        y = np.where(g.standard_normal(B) > 0, 1.0, -1.0)
    Z = g.standard_normal((M, D))
    ell = g.uniform(0.7, 1.5, D)
    sf2 = g.uniform(0.6, 1.6)
    noise = g.uniform(0.05, 0.4)
    m = g.standard_normal(M)
    s = g.uniform(0.05, 0.5, M)
    return dict(X=X, y=y, N=N, ell=ell, sf2=sf2, noise_var=noise, Z=Z, m=m,
                s=s, lik=lik)


def chol_Kinv(p):
    Kt = svgp.ktilde(p["Z"], p["ell"], p["sf2"], p["s"])
    return np.linalg.cholesky(np.linalg.inv(Kt))


def random_L(M, seed, scale=0.5):
    g = _rng(seed)
    L = np.tril(scale * g.standard_normal((M, M)), -1)
    L += np.diag(g.uniform(0.2, 1.5, M))
    return L


def bound(p, L):
    return svgp.rsvgp_bound(p["X"], p["y"], p["N"], p["ell"], p["sf2"],
                            p["noise_var"], p["Z"], p["m"], p["s"], L,
                            lik=p["lik"])


# ---------------------------------------------------------------- covariance
def test_se_ard_closed_form_values():
    # k(0, 1) with ell=1, sf2=2 is 2 exp(-1/2); k(x, x) = sf2
    K = svgp.se_ard(np.array([[0.0]]), np.array([[1.0], [0.0]]), np.array([1.0]), 2.0)
    assert np.allclose(K, [[2.0 * np.exp(-0.5), 2.0]], rtol=0, atol=1e-15)
    # ARD: distance along d is measured in units of ell_d
    K = svgp.se_ard(np.array([[0.0, 0.0]]), np.array([[3.0, 4.0]]),
                    np.array([3.0, 2.0]), 1.0)
    assert np.isclose(K[0, 0], np.exp(-0.5 * (1.0 + 4.0)), rtol=1e-15)
    # an infinitely long lengthscale removes that input dimension
    g = _rng(1)
    A, Bm = g.standard_normal((5, 2)), g.standard_normal((4, 2))
    K2 = svgp.se_ard(A, Bm, np.array([0.8, 1e12]), 1.3)
    K1 = svgp.se_ard(A[:, :1], Bm[:, :1], np.array([0.8]), 1.3)
    assert np.allclose(K2, K1, rtol=1e-12)


def test_se_ard_symmetric_psd():
    g = _rng(2)
    Z = g.standard_normal((12, 3))
    K = svgp.se_ard(Z, Z, np.array([0.5, 1.0, 2.0]), 1.7)
    assert np.allclose(K, K.T, atol=0)
    assert np.allclose(np.diag(K), 1.7, atol=1e-15)
    assert np.linalg.eigvalsh(K).min() > -1e-12


# ---------------------------------------------------------------- expectations
def test_gaussian_expectation_vs_adaptive_quadrature():
    for (y, mu, v, s2) in [(0.3, -0.2, 0.5, 0.1), (2.0, 1.0, 0.01, 1.0),
                           (-1.0, 0.5, 2.0, 0.3)]:
        def integrand(f):
            logp = -0.5 * np.log(2 * np.pi * s2) - (y - f) ** 2 / (2 * s2)
            return logp * np.exp(-(f - mu) ** 2 / (2 * v)) / np.sqrt(2 * np.pi * v)
        val, _ = integrate.quad(integrand, -np.inf, np.inf, epsabs=1e-13, epsrel=1e-13)
        E, _, _, _ = quad.gaussian_expectation(np.array([y]), np.array([mu]),
                                               np.array([v]), s2)
        assert np.isclose(E[0], val, rtol=1e-10, atol=1e-12)


def test_gh_rule_integrates_polynomials_exactly():
    t, w = quad.gh_rule(20)
    for j in range(20):  # degree 2j <= 38 < 40
        assert np.isclose(np.sum(w * t ** (2 * j)), gamma_fn(j + 0.5), rtol=1e-11)
        assert abs(np.sum(w * t ** (2 * j + 1))) < 1e-8 * gamma_fn(j + 1.0)


def test_probit_expectation_vs_adaptive_quadrature():
    # 20-point Gauss-Hermite vs adaptive quadrature of E[log Phi(y f)]
    for (y, mu, v) in [(1.0, 0.3, 0.2), (-1.0, 0.3, 0.2), (1.0, -2.0, 0.05),
                       (1.0, 1.5, 1.0), (-1.0, 0.0, 0.5)]:
        def integrand(f):
            return log_ndtr(y * f) * np.exp(-(f - mu) ** 2 / (2 * v)) / np.sqrt(2 * np.pi * v)
        val, _ = integrate.quad(integrand, mu - 40 * np.sqrt(v), mu + 40 * np.sqrt(v),
                                epsabs=1e-13, epsrel=1e-12, limit=200)
        E, _, _ = quad.probit_expectation(np.array([y]), np.array([mu]), np.array([v]))
        assert np.isclose(E[0], val, rtol=2e-6, atol=1e-8)


def test_probit_partials_match_finite_differences_of_gh_sum():
    g = _rng(3)
    y = np.where(g.standard_normal(7) > 0, 1.0, -1.0)
    mu = g.standard_normal(7)
    v = g.uniform(0.05, 2.0, 7)
    E, dmu, dv = quad.probit_expectation(y, mu, v)
    h = 1e-6
    Ep, _, _ = quad.probit_expectation(y, mu + h, v)
    Em, _, _ = quad.probit_expectation(y, mu - h, v)
    assert np.allclose(dmu, (Ep - Em) / (2 * h), rtol=1e-6, atol=1e-9)
    Ep, _, _ = quad.probit_expectation(y, mu, v + h)
    Em, _, _ = quad.probit_expectation(y, mu, v - h)
    assert np.allclose(dv, (Ep - Em) / (2 * h), rtol=1e-6, atol=1e-9)


def test_gh_on_gaussian_loglik_reproduces_closed_form():
    # GH is exact for the quadratic Gaussian log-density
    t, w = quad.gh_rule(20)
    y, mu, v, s2 = 0.7, -0.4, 0.3, 0.2
    f = mu + np.sqrt(2 * v) * t
    gh = np.sum(w * (-0.5 * np.log(2 * np.pi * s2) - (y - f) ** 2 / (2 * s2))) / np.sqrt(np.pi)
    E, _, _, _ = quad.gaussian_expectation(np.array([y]), np.array([mu]), np.array([v]), s2)
    assert np.isclose(gh, E[0], rtol=1e-13)


# ---------------------------------------------------------------- the bound
@pytest.mark.parametrize("lik", ["gaussian", "probit"])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_bound_equals_cholesky_elbo_at_Ktilde_inverse(lik, seed):
    """At T = K~^{-1} the bound is the L-SVGP (preconditioned) ELBO, i.e. the
    Cholesky ELBO of q(u) = N(K_uu K~^{-1} m~, (K_uu^{-1} + S~^{-1})^{-1})."""
    p = small_problem(seed, lik=lik)
    out = bound(p, chol_Kinv(p))
    qm, qS = ref.lsvgp_q(p["ell"], p["sf2"], p["Z"], p["m"], p["s"])
    ch = ref.cholesky_elbo(p["X"], p["y"], p["N"], p["ell"], p["sf2"],
                           p["noise_var"], p["Z"], qm, qS, lik=lik)
    assert np.isclose(out["F"], ch["F"], rtol=1e-10, atol=1e-10)
    assert np.isclose(out["KL"], ch["KL"], rtol=1e-9, atol=1e-10)
    assert np.allclose(out["var"], ch["var"], rtol=1e-9, atol=1e-12)
    assert np.allclose(out["mu"], ch["mu"], rtol=1e-9, atol=1e-12)


@pytest.mark.parametrize("lik", ["gaussian", "probit"])
def test_bound_never_exceeds_elbo_of_induced_q(lik):
    """Validity (Section 2, R-SVGP): for any T the bound is an ELBO of the
    q(u) it induces, so it never exceeds that q's exact Cholesky ELBO."""
    p = small_problem(4, lik=lik)
    worst = -np.inf
    for k in range(150):
        L = random_L(6, 100 + k, scale=0.6)
        out = bound(p, L)
        qm, qS = ref.induced_q(p["ell"], p["sf2"], p["Z"], p["m"], p["s"], L)
        ch = ref.cholesky_elbo(p["X"], p["y"], p["N"], p["ell"], p["sf2"],
                               p["noise_var"], p["Z"], qm, qS, lik=lik)
        # same predictive marginals: the variance bound is attained by this q
        assert np.allclose(out["var"], ch["var"], rtol=1e-8, atol=1e-10)
        worst = max(worst, out["F"] - ch["F"])
    assert worst <= 1e-9


def test_bound_below_log_marginal_likelihood_full_batch():
    g = _rng(5)
    X = g.standard_normal((10, 2))
    y = np.cos(X[:, 0]) + 0.2 * g.standard_normal(10)
    Z = g.standard_normal((5, 2))
    ell, sf2, noise = np.array([0.9, 1.2]), 1.1, 0.15
    lml = ref.log_marginal_likelihood(X, y, ell, sf2, noise)
    for k in range(100):
        L = random_L(5, 300 + k, 0.5)
        m = g.standard_normal(5)
        s = g.uniform(0.01, 1.0, 5)
        F = svgp.rsvgp_bound(X, y, 10, ell, sf2, noise, Z, m, s, L)["F"]
        assert F <= lml + 1e-9


def test_unpreconditioned_bound_is_maximised_over_T_at_Ktilde_inverse():
    p = small_problem(6)
    args = (p["X"], p["y"], p["N"], p["ell"], p["sf2"], p["noise_var"], p["Z"],
            p["m"], p["s"])
    Fstar = ref.rsvgp_bound_unpreconditioned(*args, chol_Kinv(p))
    for k in range(100):
        assert ref.rsvgp_bound_unpreconditioned(*args, random_L(6, 500 + k)) <= Fstar + 1e-9


def test_preconditioner_is_one_newton_schulz_step():
    """P = 2T - T K~ T satisfies I - K~ P = (I - K~ T)^2 (error squaring)."""
    p = small_problem(7)
    L = random_L(6, 7, 0.3)
    out = svgp.rsvgp_bound(p["X"], p["y"], p["N"], p["ell"], p["sf2"],
                           p["noise_var"], p["Z"], p["m"], p["s"], L,
                           return_parts=True)
    I = np.eye(6)
    E = I - out["Kt"] @ (L @ L.T)
    assert np.allclose(I - out["Kt"] @ out["P"], E @ E, atol=1e-10)
    assert np.allclose(out["P"], out["P"].T, atol=1e-12)


def test_prop3_variance_sandwich():
    """L_n <= sigma_n^2(L-SVGP) <= U_n = oracle variance, and
    U_n - L_n = ||(I - K~ T) k_n||^2 / sigma^2 (Prop. 3, Section S3)."""
    p = small_problem(8)
    L = random_L(6, 8, 0.4)
    out = svgp.rsvgp_bound(p["X"], p["y"], p["N"], p["ell"], p["sf2"],
                           p["noise_var"], p["Z"], p["m"], p["s"], L,
                           return_parts=True)
    Kt, T, Kuf = out["Kt"], out["T"], out["Kuf"]
    sig2 = 0.5 * p["s"].min()               # S~ = S~' + sig2 I with S~' PD
    Ktm = Kt - sig2 * np.eye(6)
    var_L = p["sf2"] - np.sum(Kuf * np.linalg.solve(Kt, Kuf), axis=0)
    Ln = p["sf2"] - (np.sum(Kuf * Kuf, 0) - 2 * np.sum(Kuf * (T @ Ktm @ Kuf), 0)
                     + np.sum(Kuf * (T @ Ktm @ Kt @ T @ Kuf), 0)) / sig2
    assert np.all(Ln <= var_L + 1e-10)
    assert np.all(var_L <= out["var"] + 1e-10)
    R = (np.eye(6) - Kt @ T) @ Kuf
    assert np.allclose(out["var"] - Ln, np.sum(R * R, 0) / sig2, rtol=1e-8, atol=1e-10)


def test_logdet_T_from_cholesky_diagonal():
    L = random_L(7, 9)
    L[2, 2] *= -1.0                          # sign flips keep T = L L^T
    assert np.isclose(2 * np.sum(np.log(np.abs(np.diag(L)))),
                      np.linalg.slogdet(L @ L.T)[1], rtol=1e-12)


# ---------------------------------------------------------------- natural gradient
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_natgrad_equals_textbook_fisher_natural_gradient(seed):
    g = _rng(10 + seed)
    M = 4
    R = g.standard_normal((M, M))
    A = R @ R.T + 0.5 * np.eye(M)
    L = random_L(M, 20 + seed, 0.4)
    G = svgp.natgrad_direction(L, A)
    Gb = ref.fisher_natgrad(L, A)
    assert np.allclose(np.triu(G, 1), 0.0)
    assert np.allclose(G, Gb, rtol=1e-6, atol=1e-7)


def test_natgrad_fixed_point_and_quadratic_convergence():
    p = small_problem(11, M=8)
    Kt = svgp.ktilde(p["Z"], p["ell"], p["sf2"], p["s"])
    Ls = np.linalg.cholesky(np.linalg.inv(Kt))
    assert np.abs(svgp.natgrad_direction(Ls, Kt)).max() < 1e-10
    assert svgp.ng_residual(Ls, Kt) < 1e-12
    # from a nearby start, unit steps converge quadratically to chol(K~^{-1})
    L = Ls + 0.02 * np.tril(_rng(12).standard_normal((8, 8)))
    _, res = svgp.ng_steps(L, Kt, [1.0] * 5)
    assert res[0] > 1e-3
    for a, b in zip(res[:-1], res[1:]):
        if a > 1e-7:
            assert b < 10.0 * a * a
    Ln, _ = svgp.ng_steps(L, Kt, [1.0] * 8)
    assert np.allclose(Ln @ Ln.T, np.linalg.inv(Kt), rtol=1e-9, atol=1e-9)


@pytest.mark.parametrize("M", [1, 4, 9, 37])
def test_ng_residual_closed_forms(M):
    """eq. stopping_frobenius divides the Frobenius norm by sqrt(M): with
    A = I and L = c I every diagonal entry of W - I is c^2 - 1, so the
    residual is |c^2 - 1| at every M; with L = sqrt(2) chol(A^{-1}) for a
    random SPD A, W = 2 I and the residual is exactly 1."""
    for c in (0.5, 1.0, 1.7):
        assert np.isclose(svgp.ng_residual(c * np.eye(M), np.eye(M)), abs(c * c - 1.0),
                          rtol=1e-12, atol=1e-15)
    g = _rng(40 + M)
    R = g.standard_normal((M, M))
    A = R @ R.T + M * np.eye(M)
    L = np.sqrt(2.0) * np.linalg.cholesky(np.linalg.inv(A))
    assert np.isclose(svgp.ng_residual(L, A), 1.0, rtol=1e-10)
    # one symmetric off-diagonal perturbation e of W = I: ||.||_F = sqrt(2) e
    if M > 1:
        e = 1e-3
        W = np.eye(M)
        W[1, 0] = W[0, 1] = e
        Lw = np.linalg.cholesky(np.linalg.inv(A))
        Aw = np.linalg.inv(Lw.T) @ W @ np.linalg.inv(Lw)
        assert np.isclose(svgp.ng_residual(Lw, Aw), np.sqrt(2.0) * e / np.sqrt(M), rtol=1e-6)


def test_loglinear_schedule_endpoints():
    gm = svgp.loglinear_gammas(12)
    assert np.isclose(gm[0], 1e-5) and np.isclose(gm[9], 1.0) and np.isclose(gm[11], 1.0)
    assert np.all(np.diff(np.log10(gm[:10])) > 0)


def test_schedule_converges_from_identity_on_snelson_like_grid():
    """From T0 = I/sf2 the unit step diverges when lambda_max(K~) is large;
    the log-linear schedule converges (Section 3.4)."""
    x = np.linspace(0.0, 6.0, 16)[:, None]
    Kt = svgp.ktilde(x, np.array([1.0]), 1.0, np.full(16, 1e-4))
    _, res_unit = svgp.ng_steps(np.eye(16), Kt, [1.0] * 6)
    assert res_unit[-1] > 1e2
    Lc, res = svgp.ng_steps(np.eye(16), Kt, svgp.loglinear_gammas(60))
    assert res[-1] < 1e-8
    assert np.allclose(Lc @ Lc.T @ Kt, np.eye(16), atol=1e-6)


# ---------------------------------------------------------------- gradient
def _flat_fd(p, L, key, idx, h=1e-5):
    def f(v):
        q = dict(p)
        q[key] = v if np.ndim(p[key]) else float(v.reshape(()))
        return bound(q, L)["F"]
    return ref.central_fd(f, np.asarray(p[key], np.float64), idx, h)


@pytest.mark.parametrize("lik", ["gaussian", "probit"])
def test_gradient_matches_central_differences(lik):
    p = small_problem(13, M=7, B=11, D=3, lik=lik)
    L = random_L(7, 14, 0.3)
    gr = svgp.rsvgp_bound_grad(p["X"], p["y"], p["N"], p["ell"], p["sf2"],
                               p["noise_var"], p["Z"], p["m"], p["s"], L, lik=lik)
    for key in ["ell", "Z", "m", "s"]:
        n = np.size(p[key])
        fd = _flat_fd(p, L, key, list(range(n)))
        an = np.ravel(gr[key])
        assert np.allclose(an, fd, rtol=1e-6, atol=1e-6 * np.abs(fd).max()), key
    fd = _flat_fd(p, L, "sf2", [0])
    assert np.isclose(gr["sf2"], fd[0], rtol=1e-6)
    if lik == "gaussian":
        fd = _flat_fd(p, L, "noise_var", [0], h=1e-6)
        assert np.isclose(gr["noise_var"], fd[0], rtol=1e-6)


def test_prop2_gradient_equals_lsvgp_gradient_at_stopgrad_inverse():
    """Prop. 2: with T = stopgrad(K~^{-1}) the R-SVGP gradient w.r.t. xi equals
    the gradient of the preconditioned L-SVGP bound (exact inverse inside)."""
    p = small_problem(15, M=6, B=8, D=2)
    L = chol_Kinv(p)
    gr = svgp.rsvgp_bound_grad(p["X"], p["y"], p["N"], p["ell"], p["sf2"],
                               p["noise_var"], p["Z"], p["m"], p["s"], L)

    def lsvgp(q):
        return ref.lsvgp_precond_bound(q["X"], q["y"], q["N"], q["ell"], q["sf2"],
                                       q["noise_var"], q["Z"], q["m"], q["s"])
    for key in ["ell", "Z", "m", "s", "sf2"]:
        x0 = np.atleast_1d(np.asarray(p[key], np.float64))

        def f(v, key=key):
            q = dict(p)
            q[key] = v if np.ndim(p[key]) else float(v[0])
            return lsvgp(q)
        fd = ref.central_fd(f, x0, list(range(x0.size)), 1e-5)
        assert np.allclose(np.ravel(gr[key]), fd, rtol=1e-6,
                           atol=1e-6 * np.abs(fd).max()), key


def test_minibatch_scaling_of_data_term():
    """F = (N/B) sum_batch E_n - KL: doubling N doubles the data term only."""
    p = small_problem(16)
    L = random_L(6, 16)
    a = bound(p, L)
    q = dict(p)
    q["N"] = 2 * p["N"]
    b = bound(q, L)
    assert np.isclose(b["data"], 2 * a["data"], rtol=1e-14)
    assert np.isclose(b["KL"], a["KL"], rtol=1e-14)


# ---------------------------------------------------------------------------
# adaptive NG loop (Section 3.3, eq. stopping_frobenius)
def _ng_problem(M=24, seed=5):
    g = np.random.Generator(np.random.PCG64(seed))
    Z = g.standard_normal((M, 3))
    A = svgp.ktilde(Z, np.array([1.2, 0.8, 1.0]), 1.3, g.uniform(1e-2, 5e-2, M))
    return A, np.eye(M) / np.sqrt(1.3)


def test_adaptive_ng_tol_zero_is_the_fixed_loop():
    A, L0 = _ng_problem()
    gam = svgp.loglinear_gammas(15)
    La, ra, na = svgp.ng_steps_adaptive(L0, A, gam, 0.0)
    Lf, rf = svgp.ng_steps(L0, A, gam)
    assert na == 15
    np.testing.assert_array_equal(La, Lf)
    np.testing.assert_array_equal(ra, rf)


def test_adaptive_ng_large_tol_applies_nothing():
    A, L0 = _ng_problem()
    r0 = svgp.ng_residual(L0, A)
    La, ra, na = svgp.ng_steps_adaptive(L0, A, [1.0] * 4, 2.0 * r0)
    assert na == 0 and len(ra) == 1 and ra[0] == r0
    np.testing.assert_array_equal(La, L0)


def test_adaptive_ng_is_the_fixed_loop_cut_at_the_first_small_residual():
    A, L0 = _ng_problem()
    gam = svgp.loglinear_gammas(25)
    _, rf = svgp.ng_steps(L0, A, gam)
    tol = 1e-6
    first = int(np.argmax(rf < tol))           # first step whose residual is below tol
    assert rf[first] < tol and np.all(rf[:first] >= tol) and 0 < first < 25
    La, ra, na = svgp.ng_steps_adaptive(L0, A, gam, tol)
    Lc, rc = svgp.ng_steps(L0, A, gam[:first])
    assert na == first
    np.testing.assert_array_equal(La, Lc)
    np.testing.assert_array_equal(ra, rf[:first + 1])
    assert ra[-1] < tol


# ---------------------------------------------------------------- prediction
def _test_inputs(seed, n, D):
    return 1.2 * _rng(seed).standard_normal((n, D))


@pytest.mark.parametrize("seed", [0, 1])
def test_predict_equals_cholesky_predictive_of_induced_q(seed):
    """For any T, mu_* and sigma_*^2 are the M-SVGP predictive marginals of
    the q(u) that T induces (Section 2, R-SVGP paragraph), computed here by
    Cholesky solves of K_uu at inputs away from the training batch."""
    p = small_problem(seed)
    Xt = _test_inputs(50 + seed, 11, 2)
    for k in range(5):
        L = random_L(6, 300 + 10 * seed + k, scale=0.6)
        mu, var, _ = svgp.predict(Xt, p["ell"], p["sf2"], p["Z"], p["m"], p["s"], L)
        qm, qS = ref.induced_q(p["ell"], p["sf2"], p["Z"], p["m"], p["s"], L)
        cm, cv = ref.cholesky_predict(Xt, p["ell"], p["sf2"], p["Z"], qm, qS)
        assert np.allclose(mu, cm, rtol=1e-8, atol=1e-10)
        assert np.allclose(var, cv, rtol=1e-8, atol=1e-10)


def test_predict_variance_bounds_lsvgp_variance_with_equality_at_inverse():
    """eq. lsvgp_ub: sigma_*^2 >= k_** - k_*u K~^{-1} k_u* (eq. pv) for every
    T, with equality (and mu_* = k_*u K~^{-1} m~) at T = K~^{-1}."""
    p = small_problem(3)
    Xt = _test_inputs(7, 13, 2)
    Kus = svgp.se_ard(p["Z"], Xt, p["ell"], p["sf2"])
    Kt = svgp.ktilde(p["Z"], p["ell"], p["sf2"], p["s"])
    var_l = p["sf2"] - np.sum(Kus * np.linalg.solve(Kt, Kus), axis=0)
    mu_l = Kus.T @ np.linalg.solve(Kt, p["m"])
    mu, var, _ = svgp.predict(Xt, p["ell"], p["sf2"], p["Z"], p["m"], p["s"], chol_Kinv(p))
    assert np.allclose(var, var_l, rtol=1e-9, atol=1e-12)
    assert np.allclose(mu, mu_l, rtol=1e-9, atol=1e-12)
    for k in range(20):
        _, v, _ = svgp.predict(Xt, p["ell"], p["sf2"], p["Z"], p["m"], p["s"],
                               random_L(6, 400 + k, scale=0.6))
        assert np.all(v >= var_l - 1e-12)


@pytest.mark.parametrize("lik", ["gaussian", "probit"])
def test_predict_on_the_batch_gives_the_bound_marginals(lik):
    """At the training inputs the predictive marginals are the bound's mu_n,
    sigma_n^2 (eq. elbo)."""
    p = small_problem(5, lik=lik)
    L = random_L(6, 77)
    mu, var, _ = svgp.predict(p["X"], p["ell"], p["sf2"], p["Z"], p["m"], p["s"], L)
    bd = bound(p, L)
    assert np.allclose(mu, bd["mu"], rtol=1e-12, atol=1e-13)
    assert np.allclose(var, bd["var"], rtol=1e-12, atol=1e-13)


def test_gaussian_log_predictive_density_is_the_normal_log_density():
    """Gaussian likelihood: p(y_* | x_*) = N(y_*; mu_*, sigma_*^2 + noise)."""
    from scipy.stats import norm
    p = small_problem(6)
    Xt = _test_inputs(8, 9, 2)
    yt = np.sin(Xt.sum(1))
    L = random_L(6, 88)
    mu, var, lpd = svgp.predict(Xt, p["ell"], p["sf2"], p["Z"], p["m"], p["s"], L,
                                y=yt, noise_var=p["noise_var"])
    assert np.allclose(lpd, norm.logpdf(yt, mu, np.sqrt(var + p["noise_var"])),
                       rtol=1e-12, atol=1e-12)


def test_probit_log_predictive_density_is_the_integrated_probit():
    """Probit likelihood: p(y_* | x_*) = integral of Phi(y_* f) N(f; mu_*,
    sigma_*^2) df, checked by adaptive quadrature."""
    p = small_problem(7, lik="probit")
    Xt = _test_inputs(9, 6, 2)
    yt = np.array([1.0, -1.0, 1.0, -1.0, 1.0, -1.0])
    L = random_L(6, 99)
    mu, var, lpd = svgp.predict(Xt, p["ell"], p["sf2"], p["Z"], p["m"], p["s"], L,
                                y=yt, lik="probit")
    for n in range(6):
        sd = np.sqrt(var[n])
        f = lambda t: np.exp(log_ndtr(yt[n] * t)) * np.exp(-0.5 * ((t - mu[n]) / sd) ** 2) \
            / (sd * np.sqrt(2 * np.pi))
        val, _ = integrate.quad(f, mu[n] - 12 * sd, mu[n] + 12 * sd, epsabs=1e-13, epsrel=1e-12)
        assert np.isclose(lpd[n], np.log(val), rtol=1e-9, atol=1e-11)


# ---------------------------------------------------------------- variance gap
def test_variance_gap_is_the_sum_of_prop3_bound_differences():
    """G = sum_n (U_n - L_n), with U_n from eq. lsvgp_ub (the bound's own
    variance) and L_n from eq. lsvgp_lb written out with K~_- = K~ - sigma^2 I,
    for random T and two splits sigma^2 of S~; both bounds sandwich the exact
    L-SVGP variance of eq. pv."""
    p = small_problem(12)
    for k in range(6):
        L = random_L(6, 500 + k, 0.5)
        out = svgp.rsvgp_bound(p["X"], p["y"], p["N"], p["ell"], p["sf2"], p["noise_var"],
                               p["Z"], p["m"], p["s"], L, return_parts=True)
        Kt, T, Kuf = out["Kt"], out["T"], out["Kuf"]
        var_L = p["sf2"] - np.sum(Kuf * np.linalg.solve(Kt, Kuf), axis=0)
        for frac in (0.3, 0.9):
            sig2 = frac * p["s"].min()
            Km = Kt - sig2 * np.eye(6)
            Ln = p["sf2"] - (np.sum(Kuf * Kuf, 0) - 2 * np.sum(Kuf * (T @ Km @ Kuf), 0)
                             + np.sum(Kuf * (T @ Km @ Kt @ T @ Kuf), 0)) / sig2
            assert np.all(Ln <= var_L + 1e-10) and np.all(var_L <= out["var"] + 1e-10)
            G = svgp.variance_gap(L, Kt, Kuf, sig2)
            assert np.isclose(G, np.sum(out["var"] - Ln), rtol=1e-9, atol=1e-12)


def test_variance_gap_vanishes_at_Ktilde_inverse_and_scales_with_split():
    p = small_problem(13)
    Kt = svgp.ktilde(p["Z"], p["ell"], p["sf2"], p["s"])
    Kuf = svgp.se_ard(p["Z"], p["X"], p["ell"], p["sf2"])
    assert svgp.variance_gap(chol_Kinv(p), Kt, Kuf, 0.01) < 1e-20
    L = random_L(6, 9)
    assert np.isclose(svgp.variance_gap(L, Kt, Kuf, 0.01),
                      2.0 * svgp.variance_gap(L, Kt, Kuf, 0.02), rtol=1e-13)


def _gap_problem():
    p = small_problem(14)
    Kt = svgp.ktilde(p["Z"], p["ell"], p["sf2"], p["s"])
    Kuf = svgp.se_ard(p["Z"], p["X"], p["ell"], p["sf2"])
    L0 = chol_Kinv(p) * (1.0 + 0.05 * np.tril(_rng(15).standard_normal((6, 6))))
    return p, Kt, Kuf, L0


def test_gap_loop_with_eps_zero_is_the_fixed_loop_until_exact():
    p, Kt, Kuf, L0 = _gap_problem()
    gam = [1.0] * 4
    Lf, _ = svgp.ng_steps(L0, Kt, gam)
    La, gaps, applied = svgp.ng_steps_gap(L0, Kt, Kuf, gam, 0.5 * p["s"].min(), 0.1, 0.0)
    assert applied == 4 and len(gaps) == 4
    assert np.allclose(La, Lf, rtol=0, atol=0)
    # each gap is the one of the fixed loop's iterate before that step
    L = L0.copy()
    for t in range(4):
        assert np.isclose(gaps[t], svgp.variance_gap(L, Kt, Kuf, 0.5 * p["s"].min()), rtol=1e-14)
        L = L - natgrad_step(L, Kt)


def natgrad_step(L, Kt):
    return svgp.natgrad_direction(L, Kt)


def test_gap_loop_cut_at_the_first_small_gap():
    """The loop stops before the first step whose gap is <= 2 sigma_obs^2 eps
    (the gap decreases along the converging NG sequence here)."""
    p, Kt, Kuf, L0 = _gap_problem()
    gam = [1.0] * 5
    sig2, nobs = 0.5 * p["s"].min(), 0.1
    _, gaps, applied = svgp.ng_steps_gap(L0, Kt, Kuf, gam, sig2, nobs, 0.0)
    assert np.all(np.diff(gaps) < 0)
    for k in (0, 1, 2):
        eps = gaps[k] / (2 * nobs) * 1.0000001   # G_k <= threshold < G_{k-1}
        Lk, gk, ak = svgp.ng_steps_gap(L0, Kt, Kuf, gam, sig2, nobs, eps)
        Lf, _ = svgp.ng_steps(L0, Kt, gam[:k])
        assert ak == k and len(gk) == k + 1
        assert np.allclose(Lk, Lf, rtol=0, atol=0)


# ---------------------------------------------------------------- Hutchinson
def _hutch(p, L, Omega):
    return svgp.rsvgp_bound_hutchinson(p["X"], p["y"], p["N"], p["ell"], p["sf2"],
                                       p["noise_var"], p["Z"], p["m"], p["s"], L, Omega,
                                       lik=p["lik"])


@pytest.mark.parametrize("lik", ["gaussian", "probit"])
def test_hutchinson_with_scaled_unit_probes_is_the_exact_bound(lik):
    """With the M probes sqrt(M) e_i every trace estimate is exact, so the
    estimated bound is the bound of eq. rsvgp_precond."""
    p = small_problem(20, lik=lik)
    for k in range(3):
        L = random_L(6, 600 + k)
        h = _hutch(p, L, np.sqrt(6.0) * np.eye(6))
        b = bound(p, L)
        assert np.isclose(h["F"], b["F"], rtol=1e-12, atol=1e-12)
        assert np.isclose(h["KL"], b["KL"], rtol=1e-12, atol=1e-12)
        assert np.allclose(h["var"], b["var"], rtol=1e-12, atol=1e-14)


def test_hutchinson_estimate_is_unbiased():
    """Rademacher probes: the mean of the estimated bound over many
    independent single-probe draws is the exact bound (within 4 standard
    errors), and its spread matches the Hutchinson variance
    Var(w^T A w) = 2 (||A||_F^2 - sum_i A_ii^2) of the estimated combination."""
    p = small_problem(21)
    L = random_L(6, 77, 0.4)
    exact = bound(p, L)["F"]
    g = _rng(5)
    vals = []
    for _ in range(4000):
        w = g.choice([-1.0, 1.0], size=(6, 1))
        vals.append(_hutch(p, L, w)["F"])
    vals = np.array(vals)
    se = vals.std(ddof=1) / np.sqrt(len(vals))
    assert abs(vals.mean() - exact) <= 4.0 * se
    # the estimated part of -KL is -1/2 (w^T A w) with the symmetric matrix
    # A = W - 2 Wu + sym(W Wu) (from tr W - tr(P K_uu)), so Var F = Var(w^T A w) / 4
    Kt = svgp.ktilde(p["Z"], p["ell"], p["sf2"], p["s"])
    Kuu = Kt - np.diag(p["s"])
    W, Wu = L.T @ Kt @ L, L.T @ Kuu @ L
    A = W - 2.0 * Wu + 0.5 * (W @ Wu + Wu @ W)
    var_th = 2.0 * (np.sum(A * A) - np.sum(np.diag(A) ** 2)) / 4.0
    assert np.isclose(vals.var(ddof=1), var_th, rtol=0.1)


@pytest.mark.parametrize("lik", ["gaussian", "probit"])
def test_hutchinson_gradient_matches_central_differences(lik):
    """The gradient of the estimated bound (fixed probes, fixed T) against
    central differences of rsvgp_bound_hutchinson in every coordinate."""
    p = small_problem(22, M=5, B=7, D=2, lik=lik)
    L = random_L(5, 44, 0.4)
    Om = _rng(6).choice([-1.0, 1.0], size=(5, 3))
    g = svgp.rsvgp_bound_grad(p["X"], p["y"], p["N"], p["ell"], p["sf2"], p["noise_var"],
                              p["Z"], p["m"], p["s"], L, lik=lik, Omega=Om)

    def F_of(key, x):
        q = dict(p)
        q[key] = x
        return _hutch(q, L, Om)["F"]
    for key in ("ell", "Z", "m", "s"):
        x0 = np.asarray(p[key], np.float64)
        fd = ref.central_fd(lambda x: F_of(key, x.reshape(x0.shape)), x0.ravel(),
                            list(range(x0.size)), 1e-6)
        assert np.allclose(np.ravel(g[key]), fd, rtol=1e-6, atol=1e-7), key
    for key in ("sf2",) + (("noise_var",) if lik == "gaussian" else ()):
        fd = (F_of(key, p[key] + 1e-6) - F_of(key, p[key] - 1e-6)) / 2e-6
        assert np.isclose(g[key], fd, rtol=1e-6, atol=1e-7), key
    assert np.isclose(g["bound"]["F"], _hutch(p, L, Om)["F"], rtol=1e-14)


def test_hutchinson_gradient_with_scaled_unit_probes_is_the_exact_gradient():
    p = small_problem(23)
    L = random_L(6, 45)
    ge = svgp.rsvgp_bound_grad(p["X"], p["y"], p["N"], p["ell"], p["sf2"], p["noise_var"],
                               p["Z"], p["m"], p["s"], L)
    gh = svgp.rsvgp_bound_grad(p["X"], p["y"], p["N"], p["ell"], p["sf2"], p["noise_var"],
                               p["Z"], p["m"], p["s"], L, Omega=np.sqrt(6.0) * np.eye(6))
    for k in ("ell", "sf2", "noise_var", "Z", "m", "s"):
        assert np.allclose(gh[k], ge[k], rtol=1e-10, atol=1e-12), k


# ---------------------------------------------------------------- multi-output
def _multi_problem(seed, Q=3, lik="gaussian"):
    p = small_problem(seed, lik=lik)
    g = _rng(seed + 100)
    B, M = p["X"].shape[0], p["Z"].shape[0]
    if lik == "gaussian":
        Y = np.sin(p["X"] @ g.standard_normal((p["X"].shape[1], Q))) + 0.1 * g.standard_normal((B, Q))
    else:
        Y = np.where(g.standard_normal((B, Q)) > 0, 1.0, -1.0)
    return p, Y, g.standard_normal((Q, M))


@pytest.mark.parametrize("lik", ["gaussian", "probit"])
def test_multi_output_bound_at_Ktilde_inverse_is_sum_of_cholesky_elbos(lik):
    """With S~ tied across outputs and T = K~^{-1}, each output's bound is the
    Cholesky ELBO of its own q_q(u) = N(K_uu K~^{-1} m~_q, (K_uu^{-1} + S~^{-1})^{-1});
    the outputs being independent given the shared parameters, the bound is
    the sum of those ELBOs."""
    p, Y, Mt = _multi_problem(31, lik=lik)
    out = svgp.multi_output_bound(p["X"], Y, p["N"], p["ell"], p["sf2"], p["noise_var"],
                                  p["Z"], Mt, p["s"], chol_Kinv(p), lik=lik)
    tot = kl = 0.0
    for q in range(Mt.shape[0]):
        qm, qS = ref.lsvgp_q(p["ell"], p["sf2"], p["Z"], Mt[q], p["s"])
        ch = ref.cholesky_elbo(p["X"], Y[:, q], p["N"], p["ell"], p["sf2"], p["noise_var"],
                               p["Z"], qm, qS, lik=lik)
        tot += ch["F"]
        kl += ch["KL"]
        assert np.allclose(out["mu"][q], ch["mu"], rtol=1e-9, atol=1e-12)
    assert np.isclose(out["F"], tot, rtol=1e-10, atol=1e-10)
    assert np.isclose(out["KL"], kl, rtol=1e-9, atol=1e-10)


@pytest.mark.parametrize("lik", ["gaussian", "probit"])
def test_multi_output_gradient_matches_central_differences(lik):
    """The multi-output gradient (shared parameters summed over outputs, m~_q
    per output) against central differences of multi_output_bound in every
    coordinate: a gradient routed to the wrong output or a KL counted once
    instead of per output fails here."""
    p, Y, Mt = _multi_problem(32, lik=lik)
    L = random_L(6, 47, 0.4)
    args = lambda q: (p["X"], Y, p["N"], q["ell"], q["sf2"], q["noise_var"], q["Z"], q["Mt"],
                      q["s"], L)
    base = dict(p, Mt=Mt)
    g = svgp.multi_output_bound_grad(*args(base), lik=lik)

    def F_of(key, x):
        q = dict(base)
        q[key] = x
        return svgp.multi_output_bound(*args(q), lik=lik)["F"]
    for key, gk in (("ell", "ell"), ("Z", "Z"), ("Mt", "m"), ("s", "s")):
        x0 = np.asarray(base[key], np.float64)
        fd = ref.central_fd(lambda x: F_of(key, x.reshape(x0.shape)), x0.ravel(),
                            list(range(x0.size)), 1e-6)
        assert np.allclose(np.ravel(g[gk]), fd, rtol=1e-6, atol=1e-7), key
    for key in ("sf2",) + (("noise_var",) if lik == "gaussian" else ()):
        fd = (F_of(key, p[key] + 1e-6) - F_of(key, p[key] - 1e-6)) / 2e-6
        assert np.isclose(g[key], fd, rtol=1e-6, atol=1e-7), key


def test_multi_output_with_one_output_is_the_single_output_bound():
    p = small_problem(33)
    L = random_L(6, 48)
    one = svgp.multi_output_bound_grad(p["X"], p["y"][:, None], p["N"], p["ell"], p["sf2"],
                                       p["noise_var"], p["Z"], p["m"][None, :], p["s"], L)
    sg = svgp.rsvgp_bound_grad(p["X"], p["y"], p["N"], p["ell"], p["sf2"], p["noise_var"],
                               p["Z"], p["m"], p["s"], L)
    assert np.isclose(one["bound"]["F"], sg["bound"]["F"], rtol=1e-14)
    for k in ("ell", "sf2", "noise_var", "Z", "s"):
        assert np.allclose(one[k], sg[k], rtol=1e-14, atol=0), k
    assert np.allclose(one["m"][0], sg["m"], rtol=1e-14, atol=0)
