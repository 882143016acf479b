"""Grouped training iterations (ifsvgp_step_group): G independent problems,
each with its own data, hyperparameters, Z, m~, s~ and L (one T per problem,
as the layers of a deep GP have; Section 4), advanced by one launch per
kernel for the whole group.

Each problem's results must be bit-identical to an ifsvgp_step call on an
ungrouped context with the same inputs (the kernels and their order are the
same; only the grid's third index selects the problem), and every problem is
checked against the float64 oracle with the parity gate of
test_gpu_parity.py.  Cases: G = 1 and G = 3 at ragged sizes (fp32, Gaussian),
G = 3 probit, and G = 3 problems of the M = 1024, B = 4096, D = 16 workload's
size in bf16."""
import zlib

import numpy as np
import pytest

from test_gpu_parity import make_case, to_dev, sensitivity, gate, EPS, GRADS

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _gpu_out(F, terms, resid, g, L):
    t = terms.cpu().numpy()
    out = dict(L_after_ng=L.cpu().numpy(), F=F.item(), data=t[0], KL=t[1], sum_var=t[2])
    if resid is not None and resid.numel():
        out["resid"] = resid.cpu().numpy()
    for k, v in g.items():
        out["grad_" + k] = v.cpu().numpy()
    return out


def run_group(cases, prec, gammas, oracle=True, nsamp=2):
    from paper_2604_00697_amd.lib import Context, GroupContext
    G = len(cases)
    M, D = cases[0]["Z"].shape
    B = cases[0]["X"].shape[0]
    lik = cases[0]["lik"]
    want = tuple(k for k in GRADS if k != "noise_var" or lik == "gaussian")
    devs = [to_dev(c) for c in cases]
    gctx = GroupContext(G, M, B, D, prec, lik)
    outs = gctx.step_group([dict(d) for d in devs], cases[0]["N"], list(gammas), want=want)
    torch.cuda.synchronize()
    assert gctx.status() == 0
    gpu = [_gpu_out(F, t, r, g, d["L"]) for (F, t, r, g), d in zip(outs, devs)]
    gctx.close()
    # the same problems one by one on an ungrouped context
    ctx = Context(M, B, D, prec, lik)
    for q, c in enumerate(cases):
        d = to_dev(c)
        F, t, r, g = ctx.step(d["X"], d["y"], c["N"], d["ell"], d["sf2"], d["noise"], d["Z"],
                              d["m"], d["s"], d["L"], list(gammas), want=want)
        torch.cuda.synchronize()
        one = _gpu_out(F, t, r, g, d["L"])
        for k in one:
            same = np.array_equal(np.asarray(one[k]), np.asarray(gpu[q][k]))
            print(f"GROUP G={G} problem {q} {k} bitwise {same}", flush=True)
            assert same, (q, k)
    assert ctx.status() == 0
    ctx.close()
    if oracle:
        for q, c in enumerate(cases):
            ref, spread, cond = sensitivity(c, list(gammas), EPS[prec], nsamp=nsamp)
            gate(f"group{G}_{prec}_p{q}", prec, gpu[q], ref, spread, cond)


@pytest.mark.parametrize("G", [1, 3])
def test_group_fp32_ragged(require_gpu, G):
    cases = [make_case(130, 260, 3, seed=100 + q, s_range=(0.05, 0.2)) for q in range(G)]
    # different hyperparameters per problem (each layer has its own)
    for q, c in enumerate(cases):
        c["ell"] = (c["ell"] * (1.0 + 0.1 * q)).astype(np.float32)
        c["sf2"] = np.float32(1.3 + 0.2 * q)
    run_group(cases, "fp32", (1.0,))


def test_group_fp32_probit_two_ng_steps(require_gpu):
    cases = [make_case(96, 150, 4, seed=200 + q, lik="probit", s_range=(0.05, 0.2))
             for q in range(3)]
    run_group(cases, "fp32", (0.5, 1.0))


def test_group_of_three_workload_sized_problems_bf16(require_gpu):
    from test_gpu_parity import full_size_case
    from oracle import svgp
    from paper_2604_00697_amd import synth
    base = full_size_case("C3")
    w = synth.workload("C3")
    g = np.random.Generator(np.random.PCG64(303))
    cases = []
    for q in range(3):
        # each problem its own batch, inducing mean and signal variance, with L
        # near the fixed point of its own K~ (as the workload cases are)
        c = dict(base)
        X, y = w.batch(q)
        c["X"], c["y"] = X.astype(np.float32), y.astype(np.float32)
        c["m"] = (base["m"] + 0.1 * g.standard_normal(base["m"].shape)).astype(np.float32)
        c["sf2"] = np.float32(base["sf2"] * (1.0 + 0.1 * q))
        Kt = svgp.ktilde(c["Z"], c["ell"], np.float32(c["sf2"]), c["s"])
        L = np.linalg.cholesky(np.linalg.inv(Kt))
        M = L.shape[0]
        L = L + np.tril(0.01 * np.abs(L).max() * g.standard_normal((M, M)) / np.sqrt(M))
        c["L"] = L.astype(np.float32)
        cases.append(c)
    run_group(cases, "bf16", (1.0,), nsamp=1)


def test_group_argument_errors(require_gpu):
    from paper_2604_00697_amd import lib
    from paper_2604_00697_amd.lib import GroupContext, IFSVGPError
    c = make_case(40, 50, 2, seed=7)
    d = to_dev(c)
    gctx = GroupContext(2, 40, 50, 2, "fp32")
    with pytest.raises(ValueError):              # the binding checks the count
        gctx.step_group([dict(d)], c["N"], [1.0])
    # the library too: G must be the context's group size
    arr = (lib.Problem * 1)()
    rc = gctx._lib.ifsvgp_step_group(gctx._h, lib.ctypes.cast(arr, lib._P), 1, 50, c["N"],
                                     None, 0)
    assert rc == lib.EINVAL
    with pytest.raises(IFSVGPError) as e:        # single-problem entry points refuse
        gctx.bound(d["X"], d["y"], c["N"], d["ell"], d["sf2"], d["noise"], d["Z"], d["m"], d["s"],
                   d["L"])
    assert e.value.code == lib.EINVAL
    gctx.close()
