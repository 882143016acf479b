"""FP64 CPU oracle for the inverse-free sparse variational GP training iteration.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library, its
Python binding, the autograd wrapper) may import, call or link anything under
this directory.  It is imported by ``tests/``, by ``__graft_entry__.smoke()``
and by the ``cpu_baseline`` leg of ``bench.py``, nothing else.

Every quantity is computed in float64 with plain NumPy/SciPy, directly from
the paper's definitions (Cortinovis, Aitchison, Eleftheriadis, van der Wilk,
"Inverse-Free Sparse Variational Gaussian Processes"):

* ``svgp``        -- SE-ARD kernel, the natural-gradient step of Prop. 1, the
                     preconditioned R-SVGP bound (eq. rsvgp_precond) written
                     literally with P = 2T - T K~ T, and its gradient with
                     respect to xi = {theta, Z, m~, S~} at fixed T.
* ``quadrature``  -- Gaussian and Bernoulli-probit variational expectations.
* ``references``  -- independent quantities the oracle is pinned against:
                     Cholesky-based SVGP ELBO of an explicit q(u), the exact
                     log marginal likelihood, the textbook Fisher natural
                     gradient, the L-SVGP bound, central finite differences.

No function here shares code with the GPU path: no kernels, tables, constants
or helpers are common to both.
"""
from . import svgp, quadrature, references  # noqa: F401
