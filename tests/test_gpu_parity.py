"""GPU parity: the HIP library (through its C ABI) against the float64 oracle.

Both sides receive the same seeded float32 inputs.  The gate for every
quantity q (the updated L, the NG residuals, F, each term, each gradient
block) is

    tol(q) = max(base(q), mult * spread(q))

for the norm-wise relative error ||gpu - ref|| / ||ref||, and the same with
the spread taken in the element-wise measure for the element-wise error
max_i |gpu_i - ref_i| / max_i |ref_i| (every coordinate of a gradient block is
checked against the block's scale, so a wrong small coordinate such as one
lengthscale fails even when the norm hides it).

spread(q) is the oracle's own relative change when its inputs (X, y, Z, ell,
sf2, noise, m~, s~, L) and the kernel matrices it forms (K_uu, K_uf) carry
independent relative rounding of the size of the GPU form's operand precision
(eps = 2^-24 fp32, 2^-9 bf16, 2^-12 fp16; worst of 3 seeded perturbations,
1 at the largest sizes): what rounding the inputs of the computation to that
precision alone does to the result.  W = L^T K~ L and P = L(2I - W)L^T amplify
it by about kappa = ||L||^2 ||K~||, so ill-conditioned cases gate above base.

  fp32:      base 1e-5 for everything, mult 30
  bf16/fp16: base 1e-3 (F), 1e-2 (terms), 2e-2 (L, gradients), mult 4
A quantity whose gate would exceed 0.5 (rounding of the inputs to the form's
precision alone moves it by more than 50 % / mult) is reported as unresolved
and not gated: no evaluation in that precision resolves it.
Each check prints "PARITY <case> <quantity> <err> tol <tol> el <elementwise err>
spread <spread> cond <summation condition of the oracle's gradient sums>".
"""
import zlib

import numpy as np
import pytest

from oracle import svgp

pytestmark = pytest.mark.gpu

EPS = {"fp32": 2.0 ** -24, "bf16": 2.0 ** -9, "fp16": 2.0 ** -12}
BASE = {"fp32": dict(F=1e-5, term=1e-5, L=1e-5, grad=1e-5),
        "bf16": dict(F=1e-3, term=1e-2, L=2e-2, grad=2e-2),
        "fp16": dict(F=1e-3, term=1e-2, L=2e-2, grad=2e-2)}
MULT = {"fp32": 30.0, "bf16": 4.0, "fp16": 4.0}
EL = "@el"  # spread key suffix: the spread in the element-wise measure
GRADS = ("ell", "sf2", "Z", "m", "noise_var", "s")


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def make_case(M, B, D, seed=0, lik="gaussian", state="s1", N=None, snelson=False,
              s_range=(1e-4, 1e-2)):
    """float32 inputs.  s1: informative state, L near chol(K~^{-1}) (fp64 Cholesky
    of the inverse plus a small lower-triangular perturbation); s0: literal
    initial state, L = I / sf."""
    g = _rng(seed)
    if snelson:
        X = g.uniform(0, 6, (B, 1))
        y = np.sin(2 * X[:, 0]) + 0.3 * np.cos(5 * X[:, 0]) + 0.1 * g.standard_normal(B)
        Z = np.linspace(X.min(), X.max(), M)[:, None]
        ell = np.array([0.8])
    else:
        X = g.standard_normal((B, D))
        f = np.sin(X @ g.standard_normal(D) / np.sqrt(D))
        y = np.where(f + 0.3 * g.standard_normal(B) > 0, 1.0, -1.0) if lik == "probit" \
            else f + 0.05 * g.standard_normal(B)
        Z = g.standard_normal((M, D))
        ell = np.full(D, np.sqrt(D) / 2.0) if state == "s1" else np.ones(D)
    sf2 = 1.3
    noise = 0.05 ** 2 if state == "s1" else 1.0
    m = 0.5 * g.standard_normal(M) if state == "s1" else np.zeros(M)
    s = g.uniform(*s_range, M) if state == "s1" else np.full(M, 1e-4)
    f32 = lambda a: np.asarray(a, np.float32)
    X, y, Z, ell, m, s = map(f32, (X, y, Z, ell, m, s))
    if state == "s1":
        Kt = svgp.ktilde(Z, ell, np.float32(sf2), s)
        L = np.linalg.cholesky(np.linalg.inv(Kt))
        L = L + np.tril(0.01 * np.abs(L).max() * g.standard_normal((M, M)) / np.sqrt(M))
    else:
        L = np.eye(M) / np.sqrt(sf2)
    return dict(X=X, y=y, N=float(N or 10 * B), ell=ell, sf2=np.float32(sf2),
                noise=np.float32(noise), Z=Z, m=m, s=s, L=f32(L), lik=lik)


def to_dev(c):
    import torch
    dev = torch.device("cuda")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(np.atleast_1d(a))).to(dev)
    return dict(X=t(c["X"]), y=t(c["y"]), ell=t(c["ell"]), sf2=t(np.array([c["sf2"]])),
                noise=t(np.array([c["noise"]])) if c["lik"] == "gaussian" else None,
                Z=t(c["Z"]), m=t(c["m"]), s=t(c["s"]), L=t(c["L"]))


def relerr(a, b, floor=0.0):
    a, b = np.ravel(np.asarray(a, np.float64)), np.ravel(np.asarray(b, np.float64))
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), floor, 1e-300))


def klass(q):
    if q == "F":
        return "F"
    if q == "L_after_ng":
        return "L"
    return "grad" if q.startswith("grad_") else "term"


def oracle_outputs(c, gammas, perturb=None):
    Lr, res, out = svgp.training_iteration(
        c["X"], c["y"], c["N"], c["ell"], float(c["sf2"]), float(c["noise"]), c["Z"], c["m"],
        c["s"], c["L"], list(gammas), lik=c["lik"], perturb=perturb)
    bd = out["bound"]
    q = dict(L_after_ng=Lr, F=bd["F"], data=bd["data"], KL=bd["KL"], sum_var=bd["sum_var"])
    if len(gammas):
        q["resid"] = res
    for k in GRADS:
        if k != "noise_var" or c["lik"] == "gaussian":
            q["grad_" + k] = out[k]
    # summation condition of the gradient sums: ||sum of |terms||| / ||sum||
    cond = {"grad_" + k: np.linalg.norm(np.ravel(v)) / max(np.linalg.norm(np.ravel(out[k])), 1e-300)
            for k, v in out["abs_terms"].items()}
    return q, cond


def sensitivity(c, gammas, eps, nsamp=3, seed=99):
    """Oracle outputs, their worst relative change when the inputs and the
    formed K_uu, K_uf carry independent relative rounding of size eps, and
    the summation condition of each gradient block."""
    base, cond = oracle_outputs(c, gammas)
    spread = {k: 0.0 for k in base}
    g = _rng(seed)
    M, B = c["Z"].shape[0], c["X"].shape[0]
    for _ in range(nsamp):
        p = dict(c)
        keys = ("X", "Z", "ell", "m", "s", "L") + (("y",) if c["lik"] == "gaussian" else ())
        for k in keys:
            a = np.asarray(c[k], np.float64)
            p[k] = a * (1.0 + eps * g.standard_normal(a.shape))
        p["sf2"] = float(c["sf2"]) * (1.0 + eps * g.standard_normal())
        p["noise"] = float(c["noise"]) * (1.0 + eps * g.standard_normal())
        du = eps * g.standard_normal((M, M))
        pert = dict(Kuu=np.tril(du) + np.tril(du, -1).T, Kuf=eps * g.standard_normal((M, B)))
        out, _ = oracle_outputs(p, gammas, pert)
        for k in base:
            spread[k] = max(spread[k], relerr(out[k], base[k], 1.0 if k == "KL" else 0.0))
            if np.size(base[k]) > 1:
                spread[k + EL] = max(spread.get(k + EL, 0.0), elerr(out[k], base[k]))
    return base, spread, cond


def elerr(a, b):
    """max_i |a_i - b_i| / max_i |b_i| (element-wise error on the block's scale)."""
    a, b = np.ravel(np.asarray(a, np.float64)), np.ravel(np.asarray(b, np.float64))
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def gate(case, prec, gpu, ref, spread, cond, base=None):
    """tol = max(base, mult * spread); the norm-wise and the element-wise
    errors must both stay within it.  Reports every quantity, then asserts.
    base: optional per-class override.  A quantity that rounding of the
    inputs to this precision alone moves by more than 0.5 / mult (its gate
    would exceed 50 %) is reported as unresolved and not gated; fp32 gates
    every quantity."""
    bad = []
    for q in ref:
        if prec != "fp32" and MULT[prec] * spread[q] > 0.5:
            print(f"PARITY {case} {q} {relerr(gpu[q], ref[q]):.3e} unresolved spread "
                  f"{spread[q]:.2e}", flush=True)
            continue
        b = (base or BASE[prec])[klass(q)]
        tol = max(b, MULT[prec] * spread[q])
        tol_el = max(b, MULT[prec] * spread.get(q + EL, spread[q]))
        err = relerr(gpu[q], ref[q], 1.0 if q == "KL" else 0.0)
        el = elerr(gpu[q], ref[q]) if np.size(ref[q]) > 1 else err
        print(f"PARITY {case} {q} {err:.3e} tol {tol:.2e} el {el:.3e} tol_el {tol_el:.2e} "
              f"spread {spread[q]:.2e} cond {cond.get(q, 1.0):.1f}", flush=True)
        if not err <= tol:
            bad.append(f"{q}: {err:.3e} > {tol:.2e}")
        if not el <= tol_el:
            bad.append(f"{q} element-wise: {el:.3e} > {tol_el:.2e}")
    assert not bad, f"{case}: " + "; ".join(bad)


def run_gpu(c, prec="fp32", gammas=(1.0,)):
    from paper_2604_00697_amd.lib import Context
    import torch
    M, D = c["Z"].shape
    B = c["X"].shape[0]
    ctx = Context(M, B, D, prec, c["lik"])
    d = to_dev(c)
    F, terms, resid, g = ctx.step(d["X"], d["y"], c["N"], d["ell"], d["sf2"], d["noise"], d["Z"],
                                  d["m"], d["s"], d["L"], list(gammas), want=GRADS)
    torch.cuda.synchronize()
    code = ctx.status()
    t = terms.cpu().numpy()
    out = dict(L_after_ng=d["L"].cpu().numpy(), F=F.item(), data=t[0], KL=t[1], sum_var=t[2])
    if len(gammas):
        out["resid"] = resid.cpu().numpy()
    for k, v in g.items():
        out["grad_" + k] = v.cpu().numpy()
    ctx.close()
    return out, code


def compare(case, c, prec="fp32", gammas=(1.0,), nsamp=3, base=None):
    gpu, code = run_gpu(c, prec, gammas)
    assert code == 0, f"device status {code}"
    ref, spread, cond = sensitivity(c, gammas, EPS[prec], nsamp=nsamp)
    gate(case, prec, gpu, ref, spread, cond, base)


CASES_FP32 = {
    # name: (M, B, D, kwargs)
    "snelson_M16_B200": (16, 200, 1, dict(snelson=True)),
    "ragged_M100_B300_D3": (100, 300, 3, {}),
    "ragged_M200_B333_D5_s0": (200, 333, 5, dict(state="s0")),
    "wellcond_M300_B520_D4": (300, 520, 4, dict(s_range=(0.2, 0.5))),
    "C2_M512_B1024_D8": (512, 1024, 8, {}),
    "C2_M512_B1024_D8_s0": (512, 1024, 8, dict(state="s0")),
    "M1_B1": (1, 1, 2, {}),
    "maxD_M96_B200_D64": (96, 200, 64, {}),
}

# The paper's largest UCI configuration (M = 4000 inducing points, batch 100),
# fp32, against the oracle with one spread sample (the oracle iteration takes
# ~10 s); s~ in [0.05, 0.1] keeps cond(K~) near 1e5.  Every product here is a
# 4000-long fp32 dot product, so the accumulation error that the base and
# summation-condition terms cover at the smaller sizes grows: a plain float32
# evaluation of the same L-space algorithm (NumPy, blocked BLAS sums) is off
# by 6.2e-6 on F at this case, and the GPU's sequential MFMA accumulation over
# k = 4000 by about three times that; the F / term / gradient base is
# therefore 3e-5 (dF/dnoise is a sum of the same data-term quantities) and
# the summation allowance doubles (acc 256, sums of ~64K terms).  The bf16
# form is not checked at this size: with 4000 inducing points in 8 dimensions
# its spread-based gates exceed 100 % on the gradients, i.e. bf16 operands
# cannot resolve this K~.
def test_uci_size_M4000_B100_fp32(require_gpu):
    c = make_case(4000, 100, 8, seed=4000, s_range=(0.05, 0.1))
    base = dict(BASE["fp32"], F=3e-5, term=3e-5, grad=3e-5)
    compare("uci_M4000_B100_D8_fp32", c, "fp32", (1.0,), nsamp=1, base=base)


@pytest.mark.parametrize("name", list(CASES_FP32))
def test_fp32_iteration_parity(require_gpu, name):
    M, B, D, kw = CASES_FP32[name]
    gam = (1.0,) if kw.get("state") != "s0" else (1e-3,)
    compare(name, make_case(M, B, D, seed=zlib.crc32(name.encode()) % 1000, **kw), "fp32", gam)


def test_fp32_probit_parity(require_gpu):
    compare("probit_M130_B260_D4", make_case(130, 260, 4, seed=7, lik="probit"), "fp32")


def test_fp32_multi_step_schedule(require_gpu):
    c = make_case(96, 128, 2, seed=3, state="s0")
    compare("schedule12_M96", c, "fp32", list(svgp.loglinear_gammas(12)))


def test_bound_only_and_split_backward_match_step(require_gpu):
    import torch
    from paper_2604_00697_amd.lib import Context
    c = make_case(150, 400, 3, seed=11, s_range=(0.05, 0.2))
    ctx = Context(150, 400, 3, "fp32", "gaussian")
    d = to_dev(c)
    F1, t1 = ctx.bound(d["X"], d["y"], c["N"], d["ell"], d["sf2"], d["noise"], d["Z"], d["m"],
                       d["s"], d["L"])
    scale = torch.tensor([-2.0], dtype=torch.float64, device="cuda")
    g1 = ctx.bound_bwd(d["X"], d["y"], c["N"], d["ell"], d["sf2"], d["noise"], d["Z"], d["m"],
                       d["s"], d["L"], grad_scale=scale, want=GRADS)
    F2, t2, _, g2 = ctx.step(d["X"], d["y"], c["N"], d["ell"], d["sf2"], d["noise"], d["Z"],
                             d["m"], d["s"], d["L"], [], want=GRADS)
    torch.cuda.synchronize()
    assert ctx.status() == 0
    assert F1.item() == F2.item()
    for k in g1:
        assert torch.equal(g1[k], -2.0 * g2[k]), k
    ref, spread, cond = sensitivity(c, [], EPS["fp32"])
    gpu = dict(L_after_ng=c["L"], F=F1.item(), data=t1[0].item(), KL=t1[1].item(),
               sum_var=t1[2].item(), **{"grad_" + k: v.cpu().numpy() for k, v in g2.items()})
    gate("bound_only_M150", "fp32", gpu, ref, spread, cond)
    ctx.close()


def test_autograd_function_matches_oracle(require_gpu):
    from paper_2604_00697_amd.lib import Context
    from paper_2604_00697_amd.autograd import ifsvgp_bound
    c = make_case(70, 90, 2, seed=5, s_range=(0.05, 0.2))
    ctx = Context(70, 90, 2, "fp32", "gaussian")
    d = to_dev(c)
    leaves = {k: d[k].clone().requires_grad_(True)
              for k in ("ell", "sf2", "noise", "Z", "m", "s")}
    F, terms = ifsvgp_bound(ctx, d["X"], d["y"], c["N"], leaves["ell"], leaves["sf2"],
                            leaves["noise"], leaves["Z"], leaves["m"], leaves["s"], d["L"])
    (-F).backward()
    ref, spread, cond = sensitivity(c, [], EPS["fp32"])
    names = {"ell": "ell", "sf2": "sf2", "noise": "noise_var", "Z": "Z", "m": "m", "s": "s"}
    gpu = dict(L_after_ng=c["L"], F=F.item(), data=terms[0].item(), KL=terms[1].item(),
               sum_var=terms[2].item(),
               **{"grad_" + names[k]: -v.grad.cpu().numpy() for k, v in leaves.items()})
    gate("autograd_M70", "fp32", gpu, ref, spread, cond)
    ctx.close()


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_low_precision_parity(require_gpu, prec):
    # bf16 at s~ in [1e-4, 1e-2] leaves the NG residual unresolved (input
    # rounding alone moves it by 15 %); s~ in [0.01, 0.05] keeps it resolvable
    sr = (1e-2, 5e-2) if prec == "bf16" else (1e-4, 1e-2)
    compare(f"{prec}_M256_B512_D8", make_case(256, 512, 8, seed=21, s_range=sr), prec)


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_low_precision_parity_wellcond(require_gpu, prec):
    c = make_case(256, 512, 8, seed=22, s_range=(0.2, 0.5))
    compare(f"{prec}_wellcond_M256_B512_D8", c, prec)


def test_bf16_probit_parity(require_gpu):
    # at s~ in [1e-4, 1e-2] bf16 rounding of the inputs alone moves this
    # case's dF/dZ by 350 % (K~ is not resolvable in bf16); s~ in [0.2, 0.5]
    # keeps every quantity resolvable
    compare("bf16_probit_M200", make_case(200, 300, 6, seed=23, lik="probit",
                                          s_range=(0.2, 0.5)), "bf16")


def test_argument_errors_and_domain_flag(require_gpu):
    import torch
    from paper_2604_00697_amd.lib import (Context, IFSVGPError, EINVAL, EDOMAIN, ESTATE,
                                          ENONFINITE)
    c = make_case(20, 30, 2, seed=1)
    ctx = Context(20, 30, 2, "fp32", "gaussian")
    d = to_dev(c)
    big = torch.zeros(31, 2, device="cuda")
    with pytest.raises(IFSVGPError) as e:
        ctx.bound(big, torch.zeros(31, device="cuda"), 100.0, d["ell"], d["sf2"], d["noise"],
                  d["Z"], d["m"], d["s"], d["L"])
    assert e.value.code == EINVAL
    with pytest.raises(IFSVGPError) as e:   # backward before any forward
        Context(20, 30, 2).bound_bwd(d["X"], d["y"], c["N"], d["ell"], d["sf2"], d["noise"],
                                     d["Z"], d["m"], d["s"], d["L"])
    assert e.value.code == ESTATE
    s_bad = d["s"].clone()
    s_bad[3] = -1.0
    ctx.bound(d["X"], d["y"], c["N"], d["ell"], d["sf2"], d["noise"], d["Z"], d["m"], s_bad,
              d["L"])
    assert ctx.status() == EDOMAIN
    assert ctx.status() == 0          # the flag is cleared by the read
    # a zero on the diagonal of L (log|T| undefined) and a non-positive
    # lengthscale are domain errors; a NaN target gives a non-finite bound
    L_bad = d["L"].clone()
    L_bad[5, 5] = 0.0
    ctx.bound(d["X"], d["y"], c["N"], d["ell"], d["sf2"], d["noise"], d["Z"], d["m"], d["s"],
              L_bad)
    assert ctx.status() == EDOMAIN
    ell_bad = d["ell"].clone()
    ell_bad[0] = 0.0
    ctx.bound(d["X"], d["y"], c["N"], ell_bad, d["sf2"], d["noise"], d["Z"], d["m"], d["s"],
              d["L"])
    assert ctx.status() == EDOMAIN
    y_nan = d["y"].clone()
    y_nan[7] = float("nan")
    F, _ = ctx.bound(d["X"], y_nan, c["N"], d["ell"], d["sf2"], d["noise"], d["Z"], d["m"],
                     d["s"], d["L"])
    torch.cuda.synchronize()
    assert not torch.isfinite(F).all()
    assert ctx.status() == ENONFINITE
    # a clean call afterwards is unaffected
    F, _ = ctx.bound(d["X"], d["y"], c["N"], d["ell"], d["sf2"], d["noise"], d["Z"], d["m"],
                     d["s"], d["L"])
    torch.cuda.synchronize()
    assert torch.isfinite(F).all() and ctx.status() == 0
    ctx.close()


# ---------------------------------------------------------------- full sizes
# The benchmark workloads at their full sizes (inputs from the shared seeded
# generator, the same library call the benchmark times), against the oracle.
# L starts near the natural-gradient fixed point: the fp64 Cholesky factor of
# K~^{-1} plus a small lower-triangular perturbation, so the gamma = 1 step is
# the converged-regime step the benchmark runs.
def full_size_case(name):
    from paper_2604_00697_amd import synth
    w = synth.workload(name)
    p = synth.params_s1(w)
    X, y = w.batch(0)
    f32 = lambda a: np.asarray(a, np.float32)
    X, y, Z, ell, m, s = map(f32, (X, y, p.Z, p.ell, p.m, p.s))
    Kt = svgp.ktilde(Z, ell, np.float32(p.sf2), s)
    L = np.linalg.cholesky(np.linalg.inv(Kt))
    L = L + 0.01 * np.abs(L).max() * synth.lower_perturbation(w.M, 1.0) / np.sqrt(w.M)
    return dict(X=X, y=y, N=float(w.N), ell=ell, sf2=np.float32(p.sf2),
                noise=np.float32(p.noise_var), Z=Z, m=m, s=s, L=f32(L), lik=w.lik)


@pytest.mark.parametrize("name,prec", [("C3", "bf16"), ("C3", "fp32"), ("C3", "fp16"),
                                       ("C5", "bf16"), ("C4", "bf16"), ("C4", "fp32")])
def test_full_size_workloads(require_gpu, name, prec):
    c = full_size_case(name)
    compare(f"full_{name}_{prec}", c, prec, nsamp=1 if name == "C4" else 3)
