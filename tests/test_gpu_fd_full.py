"""Central finite differences (float64 oracle bound, h = 1e-4) against the
GPU gradient at the M = 2048, B = 8192, D = 32 workload, fp32 and bf16 forms.

Per coordinate: tests/golden/fd_C4.npz holds the float64 oracle's central
differences on 64 stratified coordinates (8 lengthscales, sf2, the noise
variance, 30 entries of Z, 24 of m~), written by
tests/golden/make_fd_C4.py (about 15 s of oracle work per coordinate at this
size, so they are not recomputed here).  Each coordinate is gated as

    |g_i - fd_i| <= tol * (||g_block||_inf + |fd_i|)

with ||g_block||_inf the largest magnitude of the GPU's own gradient block
the coordinate belongs to; tol = 1e-5 (fp32, the per-coordinate criterion
1e-5 ||g||_inf + 1e-5 |g_i| with the block's scale) and 0.1 (bf16).

Directional:

The bound is F(xi) at fixed T (Section 3.1), so the GPU gradient comes from
ifsvgp_bound + ifsvgp_bound_bwd at the given L.  Each check is a directional
derivative along a sparse random direction over 64 random coordinates of
xi = (lengthscales, sigma_f^2, noise variance, Z, m~), so one pair of oracle
evaluations (about 5 s each at this size) covers all 64 coordinates:

    | (F(xi + h v) - F(xi - h v)) / (2h) - g_gpu . v |  <=  tol * sum_k |g_k v_k|

tol = 1e-4 (fp32) and 0.1 (bf16; the per-block gradient errors of the bf16
form at this size are 4-9 %, see test_gpu_parity.py's full-size cases)."""
import numpy as np
import pytest

from oracle import svgp
from test_gpu_parity import full_size_case, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

KEYS = ("ell", "sf2", "noise", "Z", "m")
GKEY = {"ell": "ell", "sf2": "sf2", "noise": "noise_var", "Z": "Z", "m": "m"}


def _direction(c, n, seed):
    """v: a dict of arrays shaped like the parameters, nonzero (+-1) on n
    random coordinates of the concatenated parameter vector."""
    sizes = [np.size(c[k]) for k in KEYS]
    g = np.random.Generator(np.random.PCG64(seed))
    idx = g.choice(sum(sizes), size=n, replace=False)
    flat = np.zeros(sum(sizes))
    flat[idx] = g.choice([-1.0, 1.0], size=n)
    v, o = {}, 0
    for k, sz in zip(KEYS, sizes):
        v[k] = flat[o:o + sz].reshape(np.shape(c[k]))
        o += sz
    return v


def _F(c, v, h):
    q = {k: np.asarray(c[k], np.float64) + h * v[k] for k in KEYS}
    return svgp.rsvgp_bound(c["X"], c["y"], c["N"], q["ell"], float(q["sf2"]),
                            float(q["noise"]), q["Z"], q["m"], c["s"], c["L"], lik=c["lik"])["F"]


def _gpu_grad(prec, c):
    from paper_2604_00697_amd.lib import Context
    M, D = c["Z"].shape
    B = c["X"].shape[0]
    ctx = Context(M, B, D, prec, c["lik"])
    d = to_dev(c)
    ctx.bound(d["X"], d["y"], c["N"], d["ell"], d["sf2"], d["noise"], d["Z"], d["m"], d["s"], d["L"])
    g = ctx.bound_bwd(d["X"], d["y"], c["N"], d["ell"], d["sf2"], d["noise"], d["Z"], d["m"],
                      d["s"], d["L"], want=tuple(GKEY.values()))
    torch.cuda.synchronize()
    assert ctx.status() == 0
    ctx.close()
    return {k: g[GKEY[k]].double().cpu().numpy().reshape(np.shape(c[k])) for k in KEYS}


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_fd_per_coordinate_M2048(require_gpu, prec):
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fd_C4.npz")
    with np.load(path, allow_pickle=False) as z:
        keys, idxs, fds = [str(k) for k in z["key"]], z["idx"], z["fd"]
    c = full_size_case("C4")
    print(f"FD per-coordinate case C4 prec={prec}", flush=True)
    gg = _gpu_grad(prec, c)
    tol = 1e-5 if prec == "fp32" else 0.1
    bad, worst = [], 0.0
    for k, i, fd in zip(keys, idxs, fds):
        g = float(np.ravel(gg[k])[i])
        scale = float(np.max(np.abs(gg[k]))) + abs(fd)
        r = abs(g - fd) / scale
        worst = max(worst, r)
        print(f"FDC {prec} {k}[{i}] gpu {g:.9e} fd {fd:.9e} err/scale {r:.2e}", flush=True)
        if not r <= tol:
            bad.append(f"{k}[{i}]: {r:.2e}")
    print(f"FDC {prec} worst {worst:.2e} tol {tol}", flush=True)
    assert not bad, bad


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_fd_directional_derivative_M2048(require_gpu, prec):
    from paper_2604_00697_amd.lib import Context
    c = full_size_case("C4")
    M, D = c["Z"].shape
    B = c["X"].shape[0]
    print(f"FD case C4 prec={prec} M={M} B={B} D={D}", flush=True)
    ctx = Context(M, B, D, prec, c["lik"])
    d = to_dev(c)
    ctx.bound(d["X"], d["y"], c["N"], d["ell"], d["sf2"], d["noise"], d["Z"], d["m"], d["s"], d["L"])
    g = ctx.bound_bwd(d["X"], d["y"], c["N"], d["ell"], d["sf2"], d["noise"], d["Z"], d["m"],
                      d["s"], d["L"], want=tuple(GKEY.values()))
    torch.cuda.synchronize()
    assert ctx.status() == 0
    gg = {k: g[GKEY[k]].double().cpu().numpy().reshape(np.shape(c[k])) for k in KEYS}
    v = _direction(c, 64, seed=2048 + (prec == "bf16"))
    h = 1e-4
    fd = (_F(c, v, h) - _F(c, v, -h)) / (2.0 * h)
    gv = sum(float(np.sum(gg[k] * v[k])) for k in KEYS)
    scale = sum(float(np.sum(np.abs(gg[k] * v[k]))) for k in KEYS)
    tol = 1e-4 if prec == "fp32" else 0.1
    print(f"FD prec={prec} fd {fd:.6e} gpu {gv:.6e} diff {abs(fd - gv):.3e} "
          f"scale {scale:.3e} rel {abs(fd - gv) / scale:.3e} tol {tol}", flush=True)
    assert abs(fd - gv) <= tol * scale
