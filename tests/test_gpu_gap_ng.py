"""GPU parity of the NG loop stopped by the variance gap (ifsvgp_natgrad_gap,
Prop. 3) against the float64 oracle (oracle.svgp.ng_steps_gap): the number
of updates applied, the updated L and the gaps of the checked steps.

The threshold 2 sigma_obs^2 eps is placed at the geometric mean of two
consecutive gaps of the oracle's sequence at least a factor 16 apart (the NG
loop converges quadratically at gamma = 1, and the gap is quadratic in the
residual), so both sides take the same stopping decision.  Gates: L within
max(base, mult * spread) relative (norm-wise), base 3e-4 / 2e-2 and mult 30 / 4
for fp32 / bf16, spread being the oracle's own change of the updated L when
K~ (elementwise) and L0 carry independent rounding of the operand precision,
as in test_gpu_parity.py; each
gap measured before the stop within 1e-3 (fp32) / 0.1 (bf16) relative, plus
an absolute floor of the threshold / 10 (the gap is a difference of nearly
equal K_uf and K~ T K_uf, so its own rounding floor scales with ||K_uf||^2 /
sigma^2 times the operand precision squared)."""
import numpy as np
import pytest

from oracle import svgp

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def gap_problem(M, B, D, seed, pert):
    g = np.random.Generator(np.random.PCG64(seed))
    Z = g.standard_normal((M, D)).astype(np.float32)
    X = g.standard_normal((B, D)).astype(np.float32)
    ell = np.full(D, 0.35 * np.sqrt(D), np.float32)   # well-conditioned K~
    s = g.uniform(5e-2, 1e-1, M).astype(np.float32)
    sf2 = np.float32(1.3)
    noise = np.float32(0.05)
    Kt = svgp.ktilde(Z, ell, sf2, s)
    Kuf = svgp.se_ard(Z, X, ell, sf2)
    L0 = np.linalg.cholesky(np.linalg.inv(Kt))
    L0 = (L0 * (1.0 + pert * np.tril(g.standard_normal((M, M))))).astype(np.float32)
    sigma2 = float(np.float32(0.5 * s.min()))
    return dict(Z=Z, X=X, ell=ell, s=s, sf2=sf2, noise=noise, Kt=Kt, Kuf=Kuf, L0=L0,
                sigma2=sigma2)


def l_spread(p, Lr, k, eps, nsamp=3, seed=9):
    g = np.random.Generator(np.random.PCG64(seed))
    M = p["Kt"].shape[0]
    worst = 0.0
    for _ in range(nsamp):
        du = eps * g.standard_normal((M, M))
        Ktp = p["Kt"] * (1.0 + np.tril(du) + np.tril(du, -1).T)
        L0p = p["L0"].astype(np.float64) * (1.0 + eps * g.standard_normal((M, M)))
        Lp, _ = svgp.ng_steps(L0p, Ktp, [1.0] * k)
        worst = max(worst, np.linalg.norm(Lp - Lr) / np.linalg.norm(Lr))
    return worst


@pytest.mark.parametrize("prec,M,B,D,seed,k,pert", [("fp32", 130, 300, 3, 1, 1, 0.02),
                                                    ("fp32", 200, 96, 4, 2, 2, 0.05),
                                                    ("bf16", 160, 256, 3, 3, 1, 0.05)])
def test_gap_ng_parity(prec, M, B, D, seed, k, pert):
    from paper_2604_00697_amd.lib import Context
    dev = torch.device("cuda", 0)
    p = gap_problem(M, B, D, seed, pert)
    n_max = 5
    gam = [1.0] * n_max
    L64 = p["L0"].astype(np.float64)
    _, Gf, _ = svgp.ng_steps_gap(L64, p["Kt"], p["Kuf"], gam, p["sigma2"], p["noise"], 0.0)
    assert Gf[k] < Gf[k - 1] / 16.0
    thr = float(np.sqrt(Gf[k - 1] * Gf[k]))
    eps = thr / (2.0 * float(p["noise"]))
    Lr, Gr, nr = svgp.ng_steps_gap(L64, p["Kt"], p["Kuf"], gam, p["sigma2"], p["noise"], eps)
    assert nr == k
    t = lambda a: torch.from_numpy(np.ascontiguousarray(np.atleast_1d(np.asarray(a, np.float32)))).to(dev)
    print(f"GAP case prec={prec} M={M} B={B} k={k} thr={thr:.3e}", flush=True)
    ctx = Context(M, max(B, 8), D, prec)
    L = t(p["L0"])
    gaps, steps = ctx.natgrad_gap(t(p["X"]), t(p["Z"]), t(p["ell"]), t([p["sf2"]]),
                                  t([p["noise"]]), t(p["s"]), L, gam, p["sigma2"], eps)
    torch.cuda.synchronize()
    assert ctx.status() == 0
    g = gaps.cpu().numpy()
    print(f"GAP oracle steps {nr} gpu steps {int(steps.item())} oracle {Gr} gpu {g[:k + 1]}", flush=True)
    assert int(steps.item()) == nr
    rtol = 1e-3 if prec == "fp32" else 0.1
    for j in range(k + 1):
        assert abs(g[j] - Gr[j]) <= rtol * Gr[j] + thr / 10.0, (j, g[j], Gr[j])
    # after the stop every entry holds the stopping value
    assert np.all(g[k + 1:] == g[k])
    Lg = L.cpu().numpy().astype(np.float64)
    err = np.linalg.norm(Lg - Lr) / np.linalg.norm(Lr)
    sp = l_spread(p, Lr, k, 2.0 ** -24 if prec == "fp32" else 2.0 ** -9)
    tol = max(3e-4, 30.0 * sp) if prec == "fp32" else max(2e-2, 4.0 * sp)
    print(f"GAP L relerr {err:.3e} tol {tol:.3e} spread {sp:.3e}", flush=True)
    assert err <= tol


def test_gap_ng_argument_errors(require_gpu):
    from paper_2604_00697_amd import lib
    from paper_2604_00697_amd.lib import Context
    dev = torch.device("cuda", 0)
    p = gap_problem(40, 32, 2, 5, 0.02)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(np.atleast_1d(np.asarray(a, np.float32)))).to(dev)
    X, Z, ell, sf2, noise, s, L = (t(p["X"]), t(p["Z"]), t(p["ell"]), t([p["sf2"]]),
                                   t([p["noise"]]), t(p["s"]), t(p["L0"]))
    g = np.ones(3, np.float32)
    ptr = lambda a: a.data_ptr()
    ctx = Context(40, 32, 2, "fp32")
    f = ctx._lib.ifsvgp_natgrad_gap
    args = lambda B=32, noise_p=ptr(noise), sig=0.01, eps=1e-3: (
        ctx._h, ptr(X), B, ptr(Z), ptr(ell), ptr(sf2), noise_p, ptr(s), ptr(L), g.ctypes.data, 3,
        sig, eps, None, None)
    assert f(*args(B=0)) == lib.EINVAL
    assert f(*args(B=33)) == lib.EINVAL
    assert f(*args(noise_p=None)) == lib.EINVAL
    assert f(*args(sig=0.0)) == lib.EINVAL
    assert f(*args(eps=-1.0)) == lib.EINVAL
    cp = Context(40, 32, 2, "fp32", "probit")
    assert cp._lib.ifsvgp_natgrad_gap(cp._h, *args()[1:]) == lib.EINVAL
    torch.cuda.synchronize()
    assert ctx.status() == 0
