"""GPU parity of the adaptive NG loop (ifsvgp_natgrad_tol) against the float64
oracle (oracle.svgp.ng_steps_adaptive): the number of updates applied, the
updated L and the residuals of the checked steps.

The tolerance is taken from the oracle's own residual sequence, at the
geometric mean of two consecutive residuals at least a factor 4 apart (the
loop converges quadratically at gamma = 1), so both sides take the same
stopping decision; the gates on L
and on the residuals are those of the NG parity cases in test_gpu_parity.py's
spirit: fp32 relative 1e-5 on L (plus the conditioning-driven floor there),
bf16 2e-2."""
import numpy as np
import pytest

from oracle import svgp

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _problem(M, D, seed, pert=0.01):
    g = np.random.Generator(np.random.PCG64(seed))
    Z = g.standard_normal((M, D)).astype(np.float32)
    ell = np.full(D, 0.35 * np.sqrt(D), np.float32)   # well-conditioned K~
    s = g.uniform(5e-2, 1e-1, M).astype(np.float32)
    sf2 = np.float32(1.3)
    Kt = svgp.ktilde(Z, ell, sf2, s)
    # start from a perturbed Cholesky factor of K~^{-1} (converging regime)
    L0 = np.linalg.cholesky(np.linalg.inv(Kt))
    L0 = (L0 * (1.0 + pert * np.tril(g.standard_normal((M, M))))).astype(np.float32)
    return Z, ell, sf2, s, Kt, L0


# bf16 starts farther from the fixed point, so that its tolerance lies well
# above the residual floor that bf16 operands put under W (about 1e-2 here)
@pytest.mark.parametrize("prec,M,D,seed,k,pert", [("fp32", 130, 3, 1, 2, 0.01),
                                                  ("fp32", 257, 5, 2, 1, 0.01),
                                                  ("bf16", 200, 4, 3, 1, 0.04),
                                                  # the largest configuration's M and D
                                                  ("fp32", 2048, 32, 6, 1, 0.01)])
def test_adaptive_ng_parity(prec, M, D, seed, k, pert):
    from paper_2604_00697_amd.lib import Context
    dev = torch.device("cuda", 0)
    Z, ell, sf2, s, Kt, L0 = _problem(M, D, seed, pert)
    n_max = 6
    gam = [1.0] * n_max
    _, rf = svgp.ng_steps(L0.astype(np.float64), Kt, gam)
    # a tolerance between residuals k-1 and k (a factor of 4 or more apart:
    # each at least a factor of 2 from it), so both sides apply exactly k updates
    assert rf[k] < 0.25 * rf[k - 1]
    tol = float(np.sqrt(rf[k - 1] * rf[k]))
    Lr, rr, nr = svgp.ng_steps_adaptive(L0.astype(np.float64), Kt, gam, tol)
    ctx = Context(M, 8, D, prec)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(np.asarray(a, np.float32))).to(dev)
    L = t(L0)
    resid, steps = ctx.natgrad_tol(t(Z), t(ell), t([sf2]), t(s), L, gam, tol)
    torch.cuda.synchronize()
    print(f"ADAPTIVE prec={prec} M={M} tol={tol:.3e} oracle steps {nr} gpu steps {int(steps.item())}",
          flush=True)
    assert ctx.status() == 0
    assert nr == k and int(steps.item()) == nr
    Lg = L.double().cpu().numpy()
    tolL = 1e-5 if prec == "fp32" else 2e-2
    # fp32: the residual amplification of W = L^T K~ L (cond(K~) here is small)
    errL = np.linalg.norm(np.tril(Lg) - Lr) / np.linalg.norm(Lr)
    assert errL <= tolL * 30 if prec == "fp32" else errL <= tolL, errL
    rg = resid.cpu().numpy()
    nchk = len(rr)
    # the GPU's W = L^T K~ L carries the rounding of its operands, a floor
    # under the residual: about 5e-5 in fp32 and 1e-2 in bf16 at these sizes
    np.testing.assert_allclose(rg[:nchk], rr, rtol=(1e-3 if prec == "fp32" else 0.15),
                               atol=(5e-5 if prec == "fp32" else 1.5e-2))
    # after the stop every later entry repeats the stopping residual
    if nr < n_max:
        np.testing.assert_array_equal(rg[nchk:], np.full(n_max - nchk, rg[nchk - 1]))
    ctx.close()


def test_adaptive_calls_in_a_row_are_independent(require_gpu):
    """A loop that stopped early leaves its stop flag set; the next adaptive
    call on the same context must start from its own first step regardless
    (same inputs twice -> identical residuals, steps and L)."""
    from paper_2604_00697_amd.lib import Context
    dev = torch.device("cuda", 0)
    Z, ell, sf2, s, Kt, L0 = _problem(100, 3, 4, 0.02)
    gam = [1.0] * 6
    _, rf = svgp.ng_steps(L0.astype(np.float64), Kt, gam)
    tol = float(np.sqrt(rf[1] * rf[2]))
    ctx = Context(100, 8, 3, "fp32")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(np.asarray(a, np.float32))).to(dev)
    outs = []
    for _ in range(2):
        L = t(L0)
        r, k = ctx.natgrad_tol(t(Z), t(ell), t([sf2]), t(s), L, gam, tol)
        outs.append((r.clone(), k.clone(), L))
    torch.cuda.synchronize()
    assert ctx.status() == 0
    assert int(outs[0][1].item()) == 2
    for a, b in zip(outs[0], outs[1]):
        assert torch.equal(a, b)
