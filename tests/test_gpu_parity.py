"""GPU parity: the HIP library (through its C ABI) against the float64 oracle.

Both sides receive the same seeded float32 inputs.  Tolerances (relative):
  fp32       F, every term, L after the NG steps, gradients (norm-wise): 1e-5
             (gradient blocks whose own magnitude is tiny relative to the
             others are compared norm-wise against their own scale)
  bf16/fp16  F 1e-3, terms 1e-2, gradients 2e-2 norm-wise
Each check prints "PARITY <case> <quantity> <relative error>".
"""
import zlib

import numpy as np
import pytest

from oracle import svgp

pytestmark = pytest.mark.gpu

TOL = {
    "fp32": dict(F=1e-5, term=1e-5, L=1e-5, grad=1e-5),
    "bf16": dict(F=1e-3, term=1e-2, L=2e-2, grad=2e-2),
    "fp16": dict(F=1e-3, term=1e-2, L=2e-2, grad=2e-2),
}


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def make_case(M, B, D, seed=0, lik="gaussian", state="s1", N=None, snelson=False):
    """float32 inputs; L near chol(K~^{-1}) (fp64 Cholesky of the inverse plus a
    small lower-triangular perturbation) unless state == 's0' (L = I/sf)."""
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
    s = g.uniform(1e-4, 1e-2, M) if state == "s1" else np.full(M, 1e-4)
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


def rel(a, b):
    a, b = np.ravel(np.asarray(a, np.float64)), np.ravel(np.asarray(b, np.float64))
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def report(case, what, err, tol):
    print(f"PARITY {case} {what} {err:.3e} (tol {tol:.0e})", flush=True)
    assert err <= tol, f"{case} {what}: {err:.3e} > {tol:.0e}"


def run_gpu(c, prec="fp32", gammas=(1.0,), grads=True):
    from paper_2604_00697_amd.lib import Context
    import torch
    M, D = c["Z"].shape
    B = c["X"].shape[0]
    ctx = Context(M, B, D, prec, c["lik"])
    d = to_dev(c)
    F, terms, resid, g = ctx.step(d["X"], d["y"], c["N"], d["ell"], d["sf2"], d["noise"], d["Z"],
                                  d["m"], d["s"], d["L"], list(gammas))
    torch.cuda.synchronize()
    code = ctx.status()
    out = dict(F=F.item(), terms=terms.cpu().numpy(), L=d["L"].cpu().numpy(),
               resid=resid.cpu().numpy() if resid is not None else None,
               grads={k: v.cpu().numpy() for k, v in g.items()}, status=code)
    ctx.close()
    return out


def run_oracle(c, gammas=(1.0,)):
    Lr, res, out = svgp.training_iteration(
        c["X"], c["y"], c["N"], c["ell"], float(c["sf2"]), float(c["noise"]), c["Z"], c["m"],
        c["s"], c["L"], list(gammas), lik=c["lik"])
    return Lr, res, out


def compare(case, c, prec="fp32", gammas=(1.0,)):
    tol = TOL[prec]
    gp = run_gpu(c, prec, gammas)
    assert gp["status"] == 0, gp["status"]
    Lr, res, out = run_oracle(c, gammas)
    bd = out["bound"]
    report(case, "L_after_ng", rel(gp["L"], Lr), tol["L"])
    if len(gammas):
        report(case, "resid", rel(gp["resid"], res), tol["term"])
    report(case, "F", abs(gp["F"] - bd["F"]) / abs(bd["F"]), tol["F"])
    report(case, "data", abs(gp["terms"][0] - bd["data"]) / abs(bd["data"]), tol["term"])
    report(case, "KL", abs(gp["terms"][1] - bd["KL"]) / max(abs(bd["KL"]), 1.0), tol["term"])
    report(case, "sum_var", abs(gp["terms"][2] - bd["sum_var"]) / abs(bd["sum_var"]), tol["term"])
    for k in ("ell", "sf2", "Z", "m") + (("noise_var",) if c["lik"] == "gaussian" else ()):
        report(case, f"grad_{k}", rel(gp["grads"][k], out[k]), tol["grad"])
    return gp, out


CASES_FP32 = {
    # name: (M, B, D, kwargs)
    "snelson_M16_B200": (16, 200, 1, dict(snelson=True)),
    "ragged_M100_B300_D3": (100, 300, 3, {}),
    "ragged_M200_B333_D5_s0": (200, 333, 5, dict(state="s0")),
    "C2_M512_B1024_D8": (512, 1024, 8, {}),
    "C2_M512_B1024_D8_s0": (512, 1024, 8, dict(state="s0")),
    "M1_B1": (1, 1, 2, {}),
}


@pytest.mark.parametrize("name", list(CASES_FP32))
def test_fp32_iteration_parity(require_gpu, name):
    M, B, D, kw = CASES_FP32[name]
    gam = (1.0,) if kw.get("state") != "s0" else (1e-3,)
    compare(name, make_case(M, B, D, seed=zlib.crc32(name.encode()) % 1000, **kw), "fp32", gam)


def test_fp32_probit_parity(require_gpu):
    c = make_case(130, 260, 4, seed=7, lik="probit")
    compare("probit_M130_B260_D4", c, "fp32")


def test_fp32_multi_step_schedule(require_gpu):
    c = make_case(96, 128, 2, seed=3, state="s0")
    gam = list(svgp.loglinear_gammas(12))
    compare("schedule12_M96", c, "fp32", gam)


def test_bound_only_and_split_backward_match_step(require_gpu):
    import torch
    from paper_2604_00697_amd.lib import Context
    c = make_case(150, 400, 3, seed=11)
    ctx = Context(150, 400, 3, "fp32", "gaussian")
    d = to_dev(c)
    F1, t1 = ctx.bound(d["X"], d["y"], c["N"], d["ell"], d["sf2"], d["noise"], d["Z"], d["m"],
                       d["s"], d["L"])
    scale = torch.tensor([-2.0], dtype=torch.float64, device="cuda")
    g1 = ctx.bound_bwd(d["X"], d["y"], c["N"], d["ell"], d["sf2"], d["noise"], d["Z"], d["m"],
                       d["s"], d["L"], grad_scale=scale)
    F2, t2, _, g2 = ctx.step(d["X"], d["y"], c["N"], d["ell"], d["sf2"], d["noise"], d["Z"],
                             d["m"], d["s"], d["L"], [])
    torch.cuda.synchronize()
    assert ctx.status() == 0
    assert F1.item() == F2.item()
    for k in g1:
        assert torch.equal(g1[k], -2.0 * g2[k]), k
    # oracle at the same (unchanged) L
    out = svgp.rsvgp_bound_grad(c["X"], c["y"], c["N"], c["ell"], float(c["sf2"]),
                                float(c["noise"]), c["Z"], c["m"], c["s"], c["L"])
    report("bound_only_M150", "F", abs(F1.item() - out["bound"]["F"]) / abs(out["bound"]["F"]), 1e-5)
    ctx.close()


def test_autograd_function_matches_library_backward(require_gpu):
    import torch
    from paper_2604_00697_amd.lib import Context
    from paper_2604_00697_amd.autograd import ifsvgp_bound
    c = make_case(70, 90, 2, seed=5)
    ctx = Context(70, 90, 2, "fp32", "gaussian")
    d = to_dev(c)
    leaves = {k: d[k].clone().requires_grad_(True) for k in ("ell", "sf2", "noise", "Z", "m")}
    F, terms = ifsvgp_bound(ctx, d["X"], d["y"], c["N"], leaves["ell"], leaves["sf2"],
                            leaves["noise"], leaves["Z"], leaves["m"], d["s"], d["L"])
    (-F).backward()
    out = svgp.rsvgp_bound_grad(c["X"], c["y"], c["N"], c["ell"], float(c["sf2"]),
                                float(c["noise"]), c["Z"], c["m"], c["s"], c["L"])
    names = {"ell": "ell", "sf2": "sf2", "noise": "noise_var", "Z": "Z", "m": "m"}
    for k, v in leaves.items():
        report("autograd_M70", f"grad_{k}", rel(-v.grad.cpu().numpy(), out[names[k]]), 1e-5)
    ctx.close()


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_low_precision_parity(require_gpu, prec):
    c = make_case(256, 512, 8, seed=21)
    compare(f"{prec}_M256_B512_D8", c, prec)


def test_bf16_probit_parity(require_gpu):
    c = make_case(200, 300, 6, seed=23, lik="probit")
    compare("bf16_probit_M200", c, "bf16")


def test_argument_errors_and_domain_flag(require_gpu):
    import torch
    from paper_2604_00697_amd.lib import Context, IFSVGPError, EINVAL, EDOMAIN
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
    s_bad = d["s"].clone()
    s_bad[3] = -1.0
    ctx.bound(d["X"], d["y"], c["N"], d["ell"], d["sf2"], d["noise"], d["Z"], d["m"], s_bad,
              d["L"])
    assert ctx.status() == EDOMAIN
    assert ctx.status() == 0          # the flag is cleared by the read
    ctx.close()
