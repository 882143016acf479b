"""Writes tests/golden/training_<C>.npz: the float64 oracle's training
trajectory at workload C under the protocol of tests/training_protocol.py
(one natural-gradient step per iteration with the log-linear schedule, Adam
on xi with the Section 3.4 treatment of Z).  It calls only oracle/ and the
seeded input generators; nothing here comes from the HIP library.

Usage:  python tests/golden/make_training_trajectories.py C3 C5
Recorded per iteration t: the bound F_t and its data and KL terms at the
post-NG factor L_t (before the Adam step), the NG residual, ||L_t||_F and
L_t at fixed lower-triangular entries, and after the Adam step the
log-hyperparameters and fixed entries of m~, s~ and Z.
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

from oracle import svgp                     # noqa: E402
from oracle.optim import adam_step          # noqa: E402
import training_protocol as tp              # noqa: E402


def trajectory(name, verbose=True, callback=None):
    """callback(t, L): called with the post-NG factor of every iteration."""
    from paper_2604_00697_amd import synth
    wname, _ = tp.CONFIGS[name]
    w = synth.workload(wname)
    st, batch = tp.initial_state(w)
    M, D = w.M, w.D
    gauss = w.lik == "gaussian"
    sp = tp.sample_positions(M, D)
    f64 = lambda a: np.asarray(a, np.float64)
    phi = np.concatenate([np.log(f64(st["ell"])), [np.log(float(st["sf2"]))]]
                         + ([[np.log(float(st["noise"]))]] if gauss else []))
    ls, m, Z, L = np.log(f64(st["s"])), f64(st["m"]), f64(st["Z"]), f64(st["L"])
    mom = {k: (np.zeros_like(v), np.zeros_like(v)) for k, v in
           (("phi", phi), ("ls", ls), ("m", m), ("Z", Z))}
    gam = svgp.loglinear_gammas(tp.ITERS, ramp=tp.NG_RAMP)
    rec = {k: [] for k in ("F", "data", "KL", "resid", "Lnorm", "Ls", "phi", "m", "s", "Z")}
    t0 = time.perf_counter()
    for t in range(tp.ITERS):
        X, y = batch(t)
        ell, sf2 = np.exp(phi[:D]), float(np.exp(phi[D]))
        noise = float(np.exp(phi[D + 1])) if gauss else 1.0
        s = np.exp(ls)
        L, res, out = svgp.training_iteration(X, y, float(w.N), ell, sf2, noise, Z, m, s, L,
                                              [gam[t]], lik=w.lik)
        bd = out["bound"]
        rec["F"].append(bd["F"])
        rec["data"].append(bd["data"])
        rec["KL"].append(bd["KL"])
        rec["resid"].append(res[0])
        rec["Lnorm"].append(np.linalg.norm(L))
        rec["Ls"].append(L[sp["Li"], sp["Lj"]])
        if callback is not None:
            callback(t, L)
        g_phi = np.concatenate([out["ell"] * ell, [out["sf2"] * sf2]]
                               + ([[out["noise_var"] * noise]] if gauss else []))
        phi, *mom["phi"] = adam_step(phi, g_phi, *mom["phi"], t + 1, lr=tp.LR, ascend=True)
        ls, *mom["ls"] = adam_step(ls, out["s"] * s, *mom["ls"], t + 1, lr=tp.LR, ascend=True)
        m, *mom["m"] = adam_step(m, out["m"], *mom["m"], t + 1, lr=tp.LR, ascend=True)
        if t >= tp.Z_FREEZE:
            Z, *mom["Z"] = adam_step(Z, out["Z"], *mom["Z"], t - tp.Z_FREEZE + 1, lr=tp.Z_LR,
                                     beta1=tp.Z_BETA1, ascend=True)
        rec["phi"].append(phi.copy())
        rec["m"].append(m[sp["v"]])
        rec["s"].append(np.exp(ls)[sp["v"]])
        rec["Z"].append(Z[sp["Zi"], sp["Zd"]])
        if verbose:
            print(f"{name} t={t} F={bd['F']:.10e} resid={res[0]:.3e} "
                  f"({time.perf_counter() - t0:.0f} s)", flush=True)
    return {k: np.asarray(v, np.float64) for k, v in rec.items()}


if __name__ == "__main__":
    for name in sys.argv[1:] or ["C3", "C5"]:
        out = trajectory(name)
        np.savez_compressed(os.path.join(HERE, f"training_{name}.npz"), **out)
