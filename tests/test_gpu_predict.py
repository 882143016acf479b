"""GPU parity of ifsvgp_predict against the float64 oracle (oracle.svgp.predict):
predictive mean and variance of f at test inputs, the per-point log
predictive density and the NLPD, for both likelihoods, with more test points
than the context's B_max (several chunks and a ragged last one).

Gate, per output q (mu, var, lpd, nlpd), element by element:

    max_i |gpu_i - ref_i| / max_i |ref_i|  <=  max(base, mult * spread(q))

where spread(q) is the oracle's own change, in the same measure, when its
inputs and the kernel matrices it forms (K_uu, K_u*) carry independent
relative rounding of the GPU form's operand precision (as in
test_gpu_parity.py): fp32 base 1e-5, mult 30; bf16 base 1e-2, mult 4.
The mean is the sensitive output: mu_* = k_*u P m~ with P close to K~^{-1}
applies K~^{-1} to m~, so elementwise rounding of K~ moves it by about
eps * cond(K~) relative (a plain float32 evaluation of the same L-space
algorithm on the CPU shows errors of 1e-4 at cond(K~) ~ 1e4).  The bf16 case
therefore uses a better-conditioned K~ (s~ in [0.3, 1])."""
import zlib

import numpy as np
import pytest

from oracle import svgp
from test_gpu_parity import make_case

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

EPS = {"fp32": 2.0 ** -24, "bf16": 2.0 ** -9}
BASE = {"fp32": 1e-5, "bf16": 1e-2}
MULT = {"fp32": 30.0, "bf16": 4.0}


def _test_points(n, D, lik, seed):
    g = np.random.Generator(np.random.PCG64(seed))
    X = g.standard_normal((n, D))
    f = np.sin(X @ g.standard_normal(D) / np.sqrt(D))
    y = np.where(f + 0.3 * g.standard_normal(n) > 0, 1.0, -1.0) if lik == "probit" \
        else f + 0.05 * g.standard_normal(n)
    return X.astype(np.float32), y.astype(np.float32)


def _oracle(c, Xt, yt, lik, perturb=None):
    mu, var, lpd = svgp.predict(Xt, c["ell"], float(c["sf2"]), c["Z"], c["m"], c["s"], c["L"],
                                y=yt, noise_var=float(c["noise"]), lik=lik, perturb=perturb)
    return dict(mu=mu, var=var, lpd=lpd, nlpd=np.array([-np.mean(lpd)]))


def _rel(a, b):
    a, b = np.asarray(a, np.float64).ravel(), np.asarray(b, np.float64).ravel()
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _spread(c, Xt, yt, lik, eps, nsamp=3, seed=5):
    base = _oracle(c, Xt, yt, lik)
    g = np.random.Generator(np.random.PCG64(seed))
    sp = {k: 0.0 for k in base}
    for _ in range(nsamp):
        p = dict(c)
        for k in ("Z", "ell", "m", "s", "L"):
            a = np.asarray(c[k], np.float64)
            p[k] = a * (1.0 + eps * g.standard_normal(a.shape))
        p["sf2"] = float(c["sf2"]) * (1.0 + eps * g.standard_normal())
        p["noise"] = float(c["noise"]) * (1.0 + eps * g.standard_normal())
        Xp = np.asarray(Xt, np.float64) * (1.0 + eps * g.standard_normal(Xt.shape))
        M = c["Z"].shape[0]
        du = eps * g.standard_normal((M, M))
        pert = dict(Kuu=np.tril(du) + np.tril(du, -1).T,
                    Kus=eps * g.standard_normal((M, Xt.shape[0])))
        out = _oracle(p, Xp, yt, lik, pert)
        for k in base:
            sp[k] = max(sp[k], _rel(out[k], base[k]))
    return base, sp


CASES = {
    # name: (prec, lik, M, B_max, D, n, range of s~)
    "fp32_gauss_M130_n250": ("fp32", "gaussian", 130, 96, 3, 250, (1e-4, 1e-2)),
    "fp32_probit_M64_n300": ("fp32", "probit", 64, 128, 2, 300, (1e-4, 1e-2)),
    "fp32_gauss_M257_n64": ("fp32", "gaussian", 257, 64, 5, 64, (1e-4, 1e-2)),
    "fp32_gauss_wellcond_M96_n200": ("fp32", "gaussian", 96, 128, 3, 200, (5e-2, 1e-1)),
    "bf16_gauss_M200_n356": ("bf16", "gaussian", 200, 256, 4, 356, (0.3, 1.0)),
}


@pytest.mark.parametrize("name", list(CASES))
def test_predict_parity(require_gpu, name):
    from paper_2604_00697_amd.lib import Context
    prec, lik, M, Bmax, D, n, s_range = CASES[name]
    seed = zlib.crc32(name.encode()) % 1000
    c = make_case(M, 8, D, seed=seed, lik=lik, s_range=s_range)
    Xt, yt = _test_points(n, D, lik, seed + 1)
    dev = torch.device("cuda", 0)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(np.atleast_1d(np.asarray(a, np.float32)))).to(dev)
    print(f"PREDICT case {name} prec={prec} lik={lik} M={M} B_max={Bmax} n={n}", flush=True)
    ctx = Context(M, Bmax, D, prec, lik)
    mu, var, lpd, nlpd = ctx.predict(t(Xt), t(c["ell"]), t([c["sf2"]]), t(c["Z"]), t(c["m"]),
                                     t(c["s"]), t(c["L"]), y=t(yt),
                                     noise=t([c["noise"]]) if lik == "gaussian" else None)
    # the same call without targets gives the same marginals
    mu2, var2, lpd2, nlpd2 = ctx.predict(t(Xt), t(c["ell"]), t([c["sf2"]]), t(c["Z"]), t(c["m"]),
                                         t(c["s"]), t(c["L"]))
    torch.cuda.synchronize()
    assert ctx.status() == 0
    assert lpd2 is None and nlpd2 is None
    assert torch.equal(mu, mu2) and torch.equal(var, var2)
    ref, sp = _spread(c, Xt, yt, lik, EPS[prec], nsamp=2 if M > 200 else 3)
    gpu = dict(mu=mu.cpu().numpy(), var=var.cpu().numpy(), lpd=lpd.cpu().numpy(),
               nlpd=nlpd.cpu().numpy())
    for q in ("mu", "var", "lpd", "nlpd"):
        assert np.all(np.isfinite(gpu[q])), q
        err = _rel(gpu[q], ref[q])
        tol = max(BASE[prec], MULT[prec] * sp[q])
        print(f"PARITY {name} {q} {err:.3e} tol {tol:.3e} spread {sp[q]:.3e}", flush=True)
        assert err <= tol, (q, err, tol)


def test_predict_argument_errors_and_state(require_gpu):
    from paper_2604_00697_amd import lib
    from paper_2604_00697_amd.lib import Context, IFSVGPError
    M, D, B = 40, 2, 32
    c = make_case(M, B, D, seed=11)
    dev = torch.device("cuda", 0)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(np.atleast_1d(np.asarray(a, np.float32)))).to(dev)
    ctx = Context(M, B, D, "fp32")
    h, L = ctx._h, ctx._lib
    Xt, yt = t(c["X"][:5]), t(c["y"][:5])
    ptr = lambda a: a.data_ptr()
    ell, sf2, noise, Z, m, s, Lm = (t(c["ell"]), t([c["sf2"]]), t([c["noise"]]), t(c["Z"]),
                                    t(c["m"]), t(c["s"]), t(c["L"]))
    mu = torch.empty(5, device=dev)
    var = torch.empty(5, device=dev)
    lpd = torch.empty(5, device=dev)
    nl = torch.empty(1, dtype=torch.float64, device=dev)
    common = (ptr(ell), ptr(sf2), ptr(noise), ptr(Z), ptr(m), ptr(s), ptr(Lm))
    # n = 0: nothing to do, unless the NLPD (a mean over no points) is asked for
    assert L.ifsvgp_predict(h, None, 0, None, *common, None, None, None, None) == lib.OK
    assert L.ifsvgp_predict(h, None, 0, ptr(yt), *common, None, None, None, ptr(nl)) == lib.EINVAL
    assert L.ifsvgp_predict(h, ptr(Xt), -1, None, *common, ptr(mu), ptr(var), None, None) == lib.EINVAL
    # lpd / nlpd without targets, missing outputs, Gaussian targets without noise
    assert L.ifsvgp_predict(h, ptr(Xt), 5, None, *common, ptr(mu), ptr(var), ptr(lpd), None) == lib.EINVAL
    assert L.ifsvgp_predict(h, ptr(Xt), 5, None, *common, ptr(mu), ptr(var), None, ptr(nl)) == lib.EINVAL
    assert L.ifsvgp_predict(h, ptr(Xt), 5, None, *common, None, ptr(var), None, None) == lib.EINVAL
    bad = (ptr(ell), ptr(sf2), None, ptr(Z), ptr(m), ptr(s), ptr(Lm))
    assert L.ifsvgp_predict(h, ptr(Xt), 5, ptr(yt), *bad, ptr(mu), ptr(var), None, None) == lib.EINVAL
    # a prediction replaces the forward state: a gradient needs a new forward
    X, y = t(c["X"]), t(c["y"])
    ctx.bound(X, y, 1000.0, ell, sf2, noise, Z, m, s, Lm)
    ctx.predict(Xt, ell, sf2, Z, m, s, Lm)
    with pytest.raises(IFSVGPError) as e:
        ctx.bound_bwd(X, y, 1000.0, ell, sf2, noise, Z, m, s, Lm)
    assert e.value.code == lib.ESTATE
    torch.cuda.synchronize()
    assert ctx.status() == 0


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_predict_full_size_sampled(require_gpu, prec):
    """The iteration's largest single-batch shape (M = 1024, B_max = 4096,
    D = 16) with 4 B + 77 test points (five chunks, a ragged last one), as the
    benchmark's prediction row runs it; the oracle checks 64 sampled points
    (chunk edges included) one by one, under the gates above."""
    from paper_2604_00697_amd.lib import Context
    M, Bmax, D = 1024, 4096, 16
    n = 4 * Bmax + 77
    c = make_case(M, 8, D, seed=1024, s_range=(5e-2, 1e-1))
    Xt, yt = _test_points(n, D, "gaussian", 1025)
    dev = torch.device("cuda", 0)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(np.atleast_1d(np.asarray(a, np.float32)))).to(dev)
    print(f"PREDICT full size prec={prec} M={M} B_max={Bmax} n={n}", flush=True)
    ctx = Context(M, Bmax, D, prec, "gaussian")
    mu, var, lpd, nlpd = ctx.predict(t(Xt), t(c["ell"]), t([c["sf2"]]), t(c["Z"]), t(c["m"]),
                                     t(c["s"]), t(c["L"]), y=t(yt), noise=t([c["noise"]]))
    torch.cuda.synchronize()
    assert ctx.status() == 0
    g = np.random.Generator(np.random.PCG64(7))
    edges = [0, Bmax - 1, Bmax, 2 * Bmax, 4 * Bmax - 1, 4 * Bmax, n - 1]
    idx = np.unique(np.concatenate([edges, g.choice(n, 64 - len(edges), replace=False)]))
    ref, sp = _spread(c, Xt[idx], yt[idx], "gaussian", EPS[prec], nsamp=2)
    gpu = dict(mu=mu.cpu().numpy()[idx], var=var.cpu().numpy()[idx],
               lpd=lpd.cpu().numpy()[idx])
    for q in ("mu", "var", "lpd"):
        assert np.all(np.isfinite(gpu[q])), q
        err = _rel(gpu[q], ref[q])
        tol = max(BASE[prec], MULT[prec] * sp[q])
        print(f"PARITY predict_full_{prec} {q} {err:.3e} tol {tol:.3e} spread {sp[q]:.3e}", flush=True)
        assert err <= tol, (q, err, tol)
    # the NLPD is the mean of all n log densities
    l_all = lpd.double().cpu().numpy()
    assert np.isfinite(nlpd.item())
    assert abs(nlpd.item() + l_all.mean()) <= 1e-6 * max(1.0, abs(nlpd.item()))
    ctx.close()
