"""The bf16 / fp16 forms form K_uf's tiles either inside V's launch (the
default, K_uf never stored) or once into memory beside the natural-gradient
step (ifsvgp_set_kuf_mode).  Both ways run the same arithmetic on the same
split inputs, so every output of a training iteration (F, its terms, the NG
residual, the updated L and every gradient) must be bit-identical between
them; the automatic choice is one of the two.  Ragged sizes (partial tiles in
both M and B), Gaussian and probit; the parity tests cover the default way
against the oracle at every size, so the stored way inherits them through
this identity."""
import numpy as np
import pytest

from test_gpu_parity import make_case, to_dev, GRADS

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _run(c, prec, mode, gammas=(1.0,)):
    from paper_2604_00697_amd.lib import Context
    M, D = c["Z"].shape
    B = c["X"].shape[0]
    lik = c["lik"]
    want = tuple(k for k in GRADS if k != "noise_var" or lik == "gaussian")
    ctx = Context(M, B, D, prec, lik)
    if mode is not None:
        ctx.set_kuf_mode(mode)
    d = to_dev(c)
    F, t, r, g = ctx.step(d["X"], d["y"], c["N"], d["ell"], d["sf2"], d["noise"], d["Z"],
                          d["m"], d["s"], d["L"], list(gammas), want=want)
    torch.cuda.synchronize()
    assert ctx.status() == 0
    out = dict(F=F.item(), terms=t.cpu().numpy(), resid=r.cpu().numpy(), L=d["L"].cpu().numpy())
    for k, v in g.items():
        out["grad_" + k] = v.cpu().numpy()
    ctx.close()
    return out


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
@pytest.mark.parametrize("lik", ["gaussian", "probit"])
def test_stored_and_generated_kuf_bit_identical(require_gpu, prec, lik):
    c = make_case(200, 333, 5, seed=41, lik=lik, s_range=(0.05, 0.2))
    _compare(c, prec, lik)


# the generator's three split widths: D <= 16, <= 32, <= 64
@pytest.mark.parametrize("D", [20, 40])
def test_stored_and_generated_kuf_bit_identical_wide_inputs(require_gpu, D):
    c = make_case(150, 260, D, seed=43, s_range=(0.05, 0.2))
    _compare(c, "bf16", "gaussian")


def test_auto_mode_above_its_threshold(require_gpu):
    """M B of at least 2^23 entries, where the automatic choice stores the
    tiles; ragged M and B (partial tiles in both)."""
    c = make_case(1030, 8200, 8, seed=47, s_range=(0.05, 0.2))
    assert 1030 * 8200 >= 1 << 23
    _compare(c, "bf16", "gaussian")


def test_stored_and_generated_kuf_bit_identical_grouped(require_gpu):
    """Two problems in one grouped context (the store kernel's grouped launch
    with per-problem workspaces)."""
    from paper_2604_00697_amd.lib import GroupContext
    cases = [make_case(130, 200, 3, seed=50 + q, s_range=(0.05, 0.2)) for q in range(2)]
    outs = {}
    for mode in ("in_product", "stored"):
        g = GroupContext(2, 130, 200, 3, "bf16")
        g.set_kuf_mode(mode)
        devs = [to_dev(c) for c in cases]
        res = g.step_group([dict(d) for d in devs], cases[0]["N"], [1.0])
        torch.cuda.synchronize()
        assert g.status() == 0
        outs[mode] = [(F.item(), t.cpu().numpy(), d["L"].cpu().numpy(),
                       {k: v.cpu().numpy() for k, v in gr.items()})
                      for (F, t, r, gr), d in zip(res, devs)]
        g.close()
    for q in range(2):
        a, b = outs["in_product"][q], outs["stored"][q]
        assert a[0] == b[0]
        assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
        for k in a[3]:
            assert np.array_equal(a[3][k], b[3][k]), (q, k)


def _compare(c, prec, lik):
    a = _run(c, prec, "in_product")
    b = _run(c, prec, "stored")
    auto = _run(c, prec, "auto")
    default = _run(c, prec, None)
    for k in a:
        same = np.array_equal(np.asarray(a[k]), np.asarray(b[k]))
        print(f"KUF {prec} {lik} {k} in_product == stored: {same}", flush=True)
        assert same, k
        assert np.array_equal(np.asarray(a[k]), np.asarray(auto[k])), k
        assert np.array_equal(np.asarray(a[k]), np.asarray(default[k])), k
    assert np.isfinite(a["F"])


def test_kuf_mode_argument_errors(require_gpu):
    from paper_2604_00697_amd import lib
    from paper_2604_00697_amd.lib import Context
    ctx = Context(40, 50, 2, "bf16")
    with pytest.raises(ValueError):
        ctx.set_kuf_mode("sometimes")
    assert ctx._lib.ifsvgp_set_kuf_mode(ctx._h, 3) == lib.EINVAL
    assert ctx._lib.ifsvgp_set_kuf_mode(ctx._h, -1) == lib.EINVAL
    assert ctx._lib.ifsvgp_set_kuf_mode(None, 0) == lib.EINVAL
    ctx.close()
