"""The allocation-free training iteration (ifsvgp_step_noalloc) against the
context entry point ifsvgp_step on the same inputs, through the C ABI.

Both run the same kernels in the same order (the allocation-free call on one
stream, the context's with a side stream), so their results agree to the
fp32 bar of the parity tests (1e-5 relative) and in practice bit for bit.
Two calls in a row, the second on a smaller problem, check that nothing of
the first call's workspace leaks into the second; a problem beyond the
static workspace is refused before any work is enqueued.
"""
import numpy as np
import pytest

from paper_2604_00697_amd import lib
from paper_2604_00697_amd.lib import Context, IFSVGPError, step_noalloc

from test_gpu_parity import make_case, to_dev

pytestmark = pytest.mark.gpu

GRADS = ("ell", "sf2", "noise_var", "Z", "m", "s")


def _rel(a, b):
    a = np.ravel(np.asarray(a, np.float64))
    b = np.ravel(np.asarray(b, np.float64))
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _both(c, prec, gammas):
    import torch
    M, D = c["Z"].shape
    B = c["X"].shape[0]
    d1, d2 = to_dev(c), to_dev(c)
    ctx = Context(M, B, D, prec, c["lik"])
    want = tuple(k for k in GRADS if not (k == "noise_var" and c["lik"] != "gaussian"))
    F1, t1, r1, g1 = ctx.step(d1["X"], d1["y"], c["N"], d1["ell"], d1["sf2"], d1["noise"],
                              d1["Z"], d1["m"], d1["s"], d1["L"], list(gammas), want=want)
    torch.cuda.synchronize()
    assert ctx.status() == 0
    ctx.close()
    F2, t2, r2, g2, flag = step_noalloc(d2["X"], d2["y"], c["N"], d2["ell"], d2["sf2"],
                                        d2["noise"], d2["Z"], d2["m"], d2["s"], d2["L"],
                                        list(gammas), prec=prec, lik=c["lik"], want=want)
    torch.cuda.synchronize()
    assert int(flag.item()) == 0
    pairs = dict(F=(F2, F1), terms=(t2, t1), L=(d2["L"], d1["L"]))
    if len(gammas):
        pairs["resid"] = (r2, r1)
    for k in g1:
        pairs["grad_" + k] = (g2[k], g1[k])
    worst = 0.0
    for q, (a, b) in pairs.items():
        a, b = a.cpu().numpy(), b.cpu().numpy()
        e = _rel(a, b)
        same = np.array_equal(a, b)
        print(f"NOALLOC {prec} M={M} B={B} {q} rel {e:.2e} bitwise {same}", flush=True)
        worst = max(worst, e)
        assert e <= 1e-5, (q, e)
    return worst


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_noalloc_matches_step_twice_second_smaller(require_gpu, prec):
    # first a larger problem, then a smaller one: the second call's workspace
    # layout overlaps the first's stale contents
    big = make_case(300, 520, 4, seed=5)
    small = make_case(100, 200, 3, seed=6)
    _both(big, prec, (1.0,))
    _both(small, prec, (0.5, 1.0))


def test_noalloc_probit_and_no_ng(require_gpu):
    c = make_case(200, 333, 5, seed=7, lik="probit")
    _both(c, "fp32", ())


def test_noalloc_refuses_problems_beyond_its_workspace(require_gpu):
    import torch
    c = make_case(64, 64, 4, seed=8)
    d = to_dev(c)
    M, B = 1024, 4096
    big = dict(X=torch.zeros((B, 4), device="cuda"), y=torch.zeros(B, device="cuda"),
               Z=torch.zeros((M, 4), device="cuda"), m=torch.zeros(M, device="cuda"),
               s=torch.ones(M, device="cuda"), L=torch.eye(M, device="cuda"))
    with pytest.raises(IFSVGPError) as ei:
        step_noalloc(big["X"], big["y"], 1e6, d["ell"], d["sf2"], d["noise"], big["Z"],
                     big["m"], big["s"], big["L"], [1.0], prec="bf16")
    assert ei.value.code == lib.ESCRATCH


def test_noalloc_reports_a_domain_error_in_its_flag(require_gpu):
    import torch
    c = make_case(64, 96, 3, seed=9)
    d = to_dev(c)
    d["ell"][0] = 0.0
    _, _, _, _, flag = step_noalloc(d["X"], d["y"], c["N"], d["ell"], d["sf2"], d["noise"],
                                    d["Z"], d["m"], d["s"], d["L"], [1.0])
    torch.cuda.synchronize()
    assert int(flag.item()) & 1
    # a clean call afterwards starts from a cleared flag
    c2 = make_case(64, 96, 3, seed=10)
    _both(c2, "fp32", (1.0,))
