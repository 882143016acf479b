"""Recorded calls (HIP graphs) against direct execution.

The library records a call's launches into a HIP graph when it meets the
same launch structure a second time and replays that graph afterwards, with
the caller's buffers passed through a device argument block.  Every kernel
reduces in a fixed order (no floating-point atomics), so a replay must give
bit-identical results to direct execution of the same call.  These tests run
two contexts side by side, one with recording disabled, through several
calls with changing mini-batch buffers, with the program's own eager work
and synchronisations between the calls, and compare every output bitwise.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _inputs(M, B, D, nbatch, seed):
    g = np.random.Generator(np.random.PCG64(seed))
    dev = torch.device("cuda", 0)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(np.asarray(a, np.float32))).to(dev)
    batches = []
    for _ in range(nbatch):
        X = g.standard_normal((B, D))
        y = np.sin(X.sum(1)) + 0.05 * g.standard_normal(B)
        batches.append((t(X), t(y)))
    Z = g.standard_normal((M, D))
    # short lengthscales keep K~ well conditioned, so the bf16 NG iteration
    # stays finite over the repeated calls (equality is checked bitwise)
    ell = np.full(D, 0.25 * np.sqrt(D))
    s = g.uniform(1e-2, 5e-2, M)
    par = dict(ell=t(ell), sf2=t([1.3]), noise=t([0.01]), Z=t(Z),
               m=t(0.5 * g.standard_normal(M)), s=t(s))
    # a stable starting factor: the Cholesky factor of K~^{-1} (float64 numpy)
    zs = Z / ell
    d2 = (zs ** 2).sum(1)[:, None] + (zs ** 2).sum(1)[None, :] - 2 * zs @ zs.T
    Kt = 1.3 * np.exp(-0.5 * np.maximum(d2, 0.0)) + np.diag(s)
    L0 = t(np.linalg.cholesky(np.linalg.inv(Kt)))
    return batches, par, L0


def _eager_noise(dev, k):
    # the program's own work between calls
    a = torch.randn(257 + k, 129, device=dev)
    b = (a @ a.T).sum()
    if k % 2 == 0:
        torch.cuda.synchronize()
    return b


@pytest.mark.parametrize("prec,shape", [("bf16", (200, 300, 5)), ("fp32", (130, 257, 3)),
                                        ("bf16", (1024, 4096, 16))])
def test_step_replays_match_direct(prec, shape):
    from paper_2604_00697_amd.lib import Context
    M, B, D = shape
    dev = torch.device("cuda", 0)
    batches, par, L0 = _inputs(M, B, D, 3, seed=M + B)
    ctxs = {"direct": Context(M, B, D, prec), "graph": Context(M, B, D, prec)}
    ctxs["direct"].set_graphs(False)
    ctxs["graph"].set_graphs(True)
    L = {k: L0.clone() for k in ctxs}
    want = ("ell", "sf2", "noise_var", "Z", "m", "s")
    for it in range(6):
        X, y = batches[it % 3]
        outs = {}
        for k, ctx in ctxs.items():
            gam = [1.0] if it < 4 else [0.5, 1.0]   # a second structure from it = 4
            F, terms, resid, g = ctx.step(X, y, 1e5, par["ell"], par["sf2"], par["noise"],
                                          par["Z"], par["m"], par["s"], L[k], gam, want=want)
            outs[k] = (F, terms, resid, g)
        _eager_noise(dev, it)
        torch.cuda.synchronize()
        print(f"GRAPH step prec={prec} shape={shape} it={it}", flush=True)
        d, r = outs["direct"], outs["graph"]
        assert torch.isfinite(d[0]).all() and torch.isfinite(L["direct"]).all(), it
        assert torch.equal(d[0], r[0]), (it, d[0].item(), r[0].item())
        assert torch.equal(d[1], r[1]), it
        assert torch.equal(d[2], r[2]), it
        for name in d[3]:
            assert torch.equal(d[3][name], r[3][name]), (it, name)
        assert torch.equal(L["direct"], L["graph"]), it
    for ctx in ctxs.values():
        assert ctx.status() == 0
        ctx.close()


def test_split_calls_replay_match_direct():
    """bound, then bound_bwd (the autograd path), and natgrad-only calls."""
    from paper_2604_00697_amd.lib import Context
    M, B, D = 300, 500, 4
    dev = torch.device("cuda", 0)
    batches, par, L0 = _inputs(M, B, D, 2, seed=7)
    ctxs = {"direct": Context(M, B, D, "bf16"), "graph": Context(M, B, D, "bf16")}
    ctxs["direct"].set_graphs(False)
    ctxs["graph"].set_graphs(True)
    L = {k: L0.clone() for k in ctxs}
    scale = torch.tensor([0.75], dtype=torch.float64, device=dev)
    for it in range(5):
        X, y = batches[it % 2]
        outs = {}
        for k, ctx in ctxs.items():
            r = ctx.natgrad(par["Z"], par["ell"], par["sf2"], par["s"], L[k], [1.0])
            F, terms = ctx.bound(X, y, 1e4, par["ell"], par["sf2"], par["noise"], par["Z"],
                                 par["m"], par["s"], L[k])
            g = ctx.bound_bwd(X, y, 1e4, par["ell"], par["sf2"], par["noise"], par["Z"],
                              par["m"], par["s"], L[k], grad_scale=scale,
                              want=("ell", "Z", "m", "noise_var"))
            outs[k] = (r, F, terms, g)
        _eager_noise(dev, it + 1)
        torch.cuda.synchronize()
        print(f"GRAPH split it={it}", flush=True)
        d, q = outs["direct"], outs["graph"]
        assert torch.isfinite(d[1]).all() and torch.isfinite(L["direct"]).all(), it
        for a, b in zip(d[:3], q[:3]):
            assert torch.equal(a, b), it
        for name in d[3]:
            assert torch.equal(d[3][name], q[3][name]), (it, name)
        assert torch.equal(L["direct"], L["graph"]), it
    for ctx in ctxs.values():
        assert ctx.status() == 0
        ctx.close()


def test_adaptive_loop_replays_match_direct():
    """The adaptive NG loops (residual rule and variance-gap rule) replayed
    from recorded graphs, with the stopping threshold changing between calls
    (it reaches the kernels through the argument block), so the replays stop
    at different steps; residuals, steps applied and L compared bitwise."""
    from paper_2604_00697_amd.lib import Context
    M, B, D = 160, 256, 3
    dev = torch.device("cuda", 0)
    batches, par, L0 = _inputs(M, B, D, 2, seed=11)
    # start away from the fixed point so the loops take several steps
    g = np.random.Generator(np.random.PCG64(5))
    pert = torch.from_numpy(np.tril(0.05 * g.standard_normal((M, M))).astype(np.float32)).to(dev)
    L0 = L0 * (1.0 + pert)
    ctxs = {"direct": Context(M, B, D, "fp32"), "graph": Context(M, B, D, "fp32")}
    ctxs["direct"].set_graphs(False)
    ctxs["graph"].set_graphs(True)
    sig2 = 0.5 * float(par["s"].min().item())
    tols = [1e-3, 1e-1, 1e-5, 3e-2, 1e-3]
    first = {}
    for it, tol in enumerate(tols):
        X, _ = batches[it % 2]
        outs = {}
        for k, ctx in ctxs.items():
            La, Lb = L0.clone(), L0.clone()
            r1, s1 = ctx.natgrad_tol(par["Z"], par["ell"], par["sf2"], par["s"], La, [1.0] * 5, tol)
            r2, s2 = ctx.natgrad_gap(X, par["Z"], par["ell"], par["sf2"], par["noise"], par["s"],
                                     Lb, [1.0] * 5, sig2, tol)
            outs[k] = (r1, s1, La, r2, s2, Lb)
        _eager_noise(dev, it)
        torch.cuda.synchronize()
        d, q = outs["direct"], outs["graph"]
        print(f"GRAPH adaptive it={it} tol={tol} steps {d[1].item()} / {d[4].item()} "
              f"resid {d[0].cpu().numpy()} gaps {d[3].cpu().numpy()}", flush=True)
        assert torch.isfinite(d[2]).all() and torch.isfinite(d[5]).all(), it
        for a, b in zip(d, q):
            assert torch.equal(a, b), it
        # every call starts from the same L0: the measure before the first step
        # does not depend on where earlier calls stopped
        first.setdefault("r", d[0][:1].clone())
        assert torch.equal(d[0][:1], first["r"]), it
        if it == 4:
            assert torch.equal(d[2], first["L_tol3"]) and torch.equal(d[1], first["s_tol3"])
        if it == 0:
            first["L_tol3"], first["s_tol3"] = d[2].clone(), d[1].clone()
    for ctx in ctxs.values():
        assert ctx.status() == 0
        ctx.close()
