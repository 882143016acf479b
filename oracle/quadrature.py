"""Variational expectations E_{N(f; mu, v)}[log p(y | f)] and their partials.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The ELBO (Section 2, eq. elbo) needs, per datum, the expectation of the log
likelihood under the marginal q(f_n) = N(mu_n, sigma_n^2).  Section S5
(Model Setup) uses a Gaussian likelihood for regression and a Bernoulli
likelihood for binary classification.

* Gaussian, noise variance s2: closed form
      E = -1/2 log(2 pi s2) - ((y - mu)^2 + v) / (2 s2).
* Bernoulli with the probit link, labels y in {-1, +1}: p(y | f) = Phi(y f).
  The expectation has no closed form; it is defined here as the n-point
  Gauss-Hermite rule (n = 20 by default) applied to the marginal:
      E = pi^{-1/2} sum_k w_k log Phi(y (mu + sqrt(2 v) t_k)),
  with (t_k, w_k) the physicists' Hermite nodes/weights from
  ``numpy.polynomial.hermite.hermgauss`` (Golub-Welsch).  The partials are the
  exact derivatives of that finite sum.
"""
import numpy as np
from numpy.polynomial.hermite import hermgauss
from scipy.special import log_ndtr

LOG_2PI = np.log(2.0 * np.pi)


def gh_rule(n=20):
    """Physicists' Gauss-Hermite nodes and weights (library routine)."""
    t, w = hermgauss(n)
    return np.asarray(t, np.float64), np.asarray(w, np.float64)


def gaussian_expectation(y, mu, v, s2):
    """Closed-form Gaussian expectation, and dE/dmu, dE/dv, dE/ds2 per datum."""
    y = np.asarray(y, np.float64)
    r = y - mu
    E = -0.5 * LOG_2PI - 0.5 * np.log(s2) - (r * r + v) / (2.0 * s2)
    dmu = r / s2
    dv = np.full_like(E, -0.5 / s2)
    ds2 = -0.5 / s2 + (r * r + v) / (2.0 * s2 * s2)
    return E, dmu, dv, ds2


def _inv_mills(z):
    """phi(z) / Phi(z), evaluated in log space to stay finite for z << 0."""
    log_phi = -0.5 * z * z - 0.5 * LOG_2PI
    return np.exp(log_phi - log_ndtr(z))


def probit_expectation(y, mu, v, n_gh=20):
    """Gauss-Hermite probit expectation and its exact partials dE/dmu, dE/dv.

    ``y`` must hold labels in {-1, +1}.  ``v`` must be positive.
    """
    y = np.asarray(y, np.float64)
    t, w = gh_rule(n_gh)
    sd = np.sqrt(v)
    z = y[:, None] * (mu[:, None] + np.sqrt(2.0) * sd[:, None] * t[None, :])
    wk = w[None, :] / np.sqrt(np.pi)
    E = np.sum(wk * log_ndtr(z), axis=1)
    lam = _inv_mills(z)
    dmu = np.sum(wk * lam, axis=1) * y
    # d z_k / d v = y sqrt(2) t_k / (2 sqrt(v)) = y t_k / sqrt(2 v)
    dv = np.sum(wk * lam * t[None, :], axis=1) * y / np.sqrt(2.0 * v)
    return E, dmu, dv


def expectation(lik, y, mu, v, noise_var=None, n_gh=20):
    """Dispatch on the likelihood name: returns (E, dE/dmu, dE/dv, dE/ds2|None)."""
    if lik == "gaussian":
        return gaussian_expectation(y, mu, v, noise_var)
    if lik == "probit":
        E, dmu, dv = probit_expectation(y, mu, v, n_gh)
        return E, dmu, dv, None
    raise ValueError(f"unknown likelihood {lik!r}")
