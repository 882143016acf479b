"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws random numbers and builds arrays.  It holds none of
the method's arithmetic (no kernel matrices, no bound, no natural gradient),
so it can feed both the HIP path and the float64 oracle with identical inputs.

The paper trains on snelson, banana, UCI elevators/kin40k and mnist
(Section S5, Datasets).  None of them is used here; the generators below stand
in for them with the shapes and value ranges of the paper's regression and
classification workloads:

* ``snelson1d``  -- 1-D regression, x ~ U[0, 6], y = sin 2x + 0.3 cos 5x +
                    N(0, 0.1^2), M inducing points on a grid (toy regression of
                    Section 4.1, M on a uniform grid as in Section S5).
* ``rff_regression`` -- x ~ N(0, I_D), y = f(x) + N(0, noise_sd^2) where f is a
                    random-Fourier-feature draw (1024 features) approximating a
                    GP with a unit-variance, unit-lengthscale SE kernel.
* ``rff_classification`` -- labels sign(f(x)) in {-1, +1}, each flipped with
                    probability 0.05.

Rows are i.i.d., so a mini-batch is drawn as B fresh rows; that has the same
distribution as sampling B rows of a fixed data set of N rows, and N enters
the method only through the N/B scale of the data term.
"""
from dataclasses import dataclass, field

import numpy as np

SEED_DATA = 0
SEED_Z = 1
SEED_BATCH = 2
SEED_PERTURB = 3
SEED_FD = 4


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


@dataclass
class RFF:
    """f(x) = sqrt(2/F) sum_j w_j cos(omega_j . x + phi_j), omega ~ N(0, I/ls^2)."""
    omega: np.ndarray
    phi: np.ndarray
    w: np.ndarray

    @classmethod
    def draw(cls, D, n_features=1024, lengthscale=1.0, seed=SEED_DATA):
        g = rng(seed)
        omega = g.standard_normal((n_features, D)) / lengthscale
        phi = g.uniform(0.0, 2.0 * np.pi, n_features)
        w = g.standard_normal(n_features)
        return cls(omega, phi, w)

    def __call__(self, X):
        F = self.w.shape[0]
        return np.sqrt(2.0 / F) * (np.cos(X @ self.omega.T + self.phi) @ self.w)


@dataclass
class Workload:
    """One configuration: sizes, likelihood, and the data generator."""
    name: str
    D: int
    N: int
    B: int
    M: int
    lik: str = "gaussian"          # "gaussian" | "probit"
    noise_sd: float = 0.05
    flip: float = 0.05
    kind: str = "rff"              # "rff" | "snelson"
    _f: object = field(default=None, repr=False)

    def f(self):
        if self._f is None:
            self._f = RFF.draw(self.D, seed=SEED_DATA)
        return self._f

    def inputs(self, n, seed):
        g = rng(seed)
        if self.kind == "snelson":
            return g.uniform(0.0, 6.0, (n, 1))
        return g.standard_normal((n, self.D))

    def targets(self, X, seed):
        g = rng(seed)
        if self.kind == "snelson":
            x = X[:, 0]
            return np.sin(2 * x) + 0.3 * np.cos(5 * x) + 0.1 * g.standard_normal(len(x))
        fx = self.f()(X)
        if self.lik == "probit":
            y = np.where(fx >= 0.0, 1.0, -1.0)
            flip = g.uniform(size=len(y)) < self.flip
            return np.where(flip, -y, y)
        return fx + self.noise_sd * g.standard_normal(len(fx))

    def batch(self, it=0, B=None):
        """Mini-batch number `it` (rows and targets), float64."""
        B = self.B if B is None else B
        if self.kind == "snelson":
            # full batch: the whole data set every iteration
            X = self.inputs(self.N, SEED_DATA)
            return X, self.targets(X, SEED_DATA + 100)
        s = SEED_BATCH * 1_000_003 + it
        X = self.inputs(B, s)
        return X, self.targets(X, s + 7919)

    def inducing(self):
        if self.kind == "snelson":
            X = self.inputs(self.N, SEED_DATA)
            return np.linspace(X.min(), X.max(), self.M)[:, None]
        return self.inputs(self.M, SEED_Z)


def workload(name):
    """The five configurations (C1..C5)."""
    if name == "C1":
        return Workload("C1", D=1, N=200, B=200, M=16, kind="snelson")
    if name == "C2":
        return Workload("C2", D=8, N=100_000, B=1024, M=512)
    if name == "C3":
        return Workload("C3", D=16, N=1_000_000, B=4096, M=1024)
    if name == "C4":
        return Workload("C4", D=32, N=1_000_000, B=8192, M=2048)
    if name == "C5":
        return Workload("C5", D=20, N=500_000, B=4096, M=1024, lik="probit")
    raise KeyError(name)


@dataclass
class Params:
    """xi = {lengthscales, sigma_f^2, noise variance, Z, m~, s~} and L."""
    ell: np.ndarray
    sf2: float
    noise_var: float
    Z: np.ndarray
    m: np.ndarray
    s: np.ndarray
    L: np.ndarray


def params_s0(w):
    """Literal initial state: ell=1, sf2=1, noise 1, m~=0, s~=1e-4, L=I/sf."""
    M, D = w.M, w.D
    sf2 = 1.0
    return Params(ell=np.ones(D), sf2=sf2, noise_var=1.0, Z=w.inducing(),
                  m=np.zeros(M), s=np.full(M, 1e-4),
                  L=np.eye(M) / np.sqrt(sf2))


def params_s1(w):
    """Informative state: ell = sqrt(D)/2 (ell=0.5 for the 1-D toy), noise
    0.05^2, m~ = f(Z) + small noise (the L-SVGP optimum has m~ close to the
    targets at the inducing inputs), s~ ~ U[1e-4, 1e-2], L = I/sf (callers
    move L towards chol(K~^{-1}) with natural-gradient steps)."""
    M, D = w.M, w.D
    g = rng(SEED_PERTURB)
    Z = w.inducing()
    if w.kind == "snelson":
        ell = np.full(D, 0.5)
        m = np.sin(2 * Z[:, 0]) + 0.3 * np.cos(5 * Z[:, 0])
    else:
        ell = np.full(D, np.sqrt(D) / 2.0)
        fz = w.f()(Z)
        m = np.where(fz >= 0, 1.0, -1.0) if w.lik == "probit" else fz
    m = m + 0.05 * g.standard_normal(M)
    return Params(ell=ell, sf2=1.0, noise_var=0.05**2, Z=Z, m=m,
                  s=g.uniform(1e-4, 1e-2, M), L=np.eye(M))


def lower_perturbation(M, scale, seed=SEED_PERTURB):
    """A random strictly-lower-triangular + diagonal perturbation matrix."""
    g = rng(seed + 17)
    return np.tril(scale * g.standard_normal((M, M)))
