"""Writes tests/golden/fd_C4.npz: central finite differences of the float64
oracle's bound at the M = 2048, B = 8192, D = 32 workload (the state of the
full-size parity cases: L near chol(K~^{-1}), fixed T) on 64 stratified
coordinates of xi: 8 lengthscales, sf2, the noise variance, 30 entries of Z
and 24 of m~ (seeded).  Step h = 1e-4, relative to the value for the three
positive hyperparameter kinds (the noise variance is 2.5e-3 here) and
absolute for Z and m~.  It calls only oracle/ and the seeded generators.

Usage:  python tests/golden/make_fd_C4.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
for p in (ROOT, os.path.dirname(HERE)):
    if p not in sys.path:
        sys.path.insert(0, p)

from oracle import svgp                    # noqa: E402
from test_gpu_parity import full_size_case  # noqa: E402

H = 1e-4
COUNTS = (("ell", 8), ("sf2", 1), ("noise", 1), ("Z", 30), ("m", 24))


def coordinates(c, seed=4):
    """(key, flat index) pairs, stratified over the parameter kinds."""
    g = np.random.Generator(np.random.PCG64(seed))
    out = []
    for k, n in COUNTS:
        size = np.size(c[k])
        for i in sorted(g.choice(size, size=min(n, size), replace=False)):
            out.append((k, int(i)))
    return out


def bound(c, key, idx, delta):
    q = {k: np.array(c[k], np.float64) for k in ("ell", "sf2", "noise", "Z", "m")}
    a = q[key].reshape(-1)
    a[idx] += delta
    q[key] = a.reshape(np.shape(q[key]))
    return svgp.rsvgp_bound(c["X"], c["y"], c["N"], q["ell"], float(q["sf2"]),
                            float(q["noise"]), q["Z"], q["m"], c["s"], c["L"], lik=c["lik"])["F"]


if __name__ == "__main__":
    c = full_size_case("C4")
    coords = coordinates(c)
    keys, idxs, steps, fd = [], [], [], []
    t0 = time.perf_counter()
    for k, i in coords:
        x = float(np.asarray(c[k], np.float64).reshape(-1)[i])
        h = H * abs(x) if k in ("ell", "sf2", "noise") else H
        v = (bound(c, k, i, h) - bound(c, k, i, -h)) / (2.0 * h)
        keys.append(k)
        idxs.append(i)
        steps.append(h)
        fd.append(v)
        print(f"{k}[{i}] h={h:.3e} fd={v:.12e} ({time.perf_counter() - t0:.0f} s)", flush=True)
    np.savez_compressed(os.path.join(HERE, "fd_C4.npz"), key=np.array(keys), idx=np.array(idxs),
                        h=np.array(steps), fd=np.array(fd))
