"""Settings of the training-loop checks at the benchmark workloads (shared by
the float64 trajectory generator in tests/golden/ and the GPU test).  Holds
no arithmetic of the method: sizes, learning rates, the schedule's
parameters, the fp32 initial state and which entries are recorded.

Protocol (Section 3.4, Step Size Scheduling, and Section S5, Training):
  * one natural-gradient step on L per iteration with the log-linear step
    size schedule from 1e-5 to 1 over the first 10 steps, then 1;
  * Adam (bias-corrected) on xi each iteration, maximising the bound:
    log-lengthscales, log signal variance, log noise variance (Gaussian),
    log s~ and m~ at learning rate 5e-3 (beta1 0.9);
  * the inducing inputs Z regularised as the paper recommends when runtime
    matters: frozen for the first Z_FREEZE iterations, then trained with
    their own Adam (learning rate 1e-3, beta1 0.99) whose step count starts
    when Z starts moving;
  * mini-batch t is the workload's batch t; the initial state is the
    informative state S1 with T0 = I / sf2 (L0 = I / sf).
"""
import numpy as np

ITERS = 100
LR = 5e-3
Z_FREEZE = 10
Z_LR = 1e-3
Z_BETA1 = 0.99
NG_RAMP = 10          # log-linear from 1e-5 to 1 over this many NG steps
N_SAMPLES = 512       # recorded entries of the lower triangle of L
N_VEC_SAMPLES = 64    # recorded entries of m~, s~ and Z

CONFIGS = {
    # name: (workload, precision of the GPU run)
    "C2": ("C2", "fp32"),
    "C3": ("C3", "bf16"),
    "C5": ("C5", "bf16"),
}


def initial_state(w):
    """fp32 initial state (the values both sides start from) and the batch
    function returning fp32 mini-batch t."""
    from paper_2604_00697_amd import synth
    p = synth.params_s1(w)
    f32 = lambda a: np.asarray(a, np.float32)
    st = dict(ell=f32(p.ell), sf2=np.float32(p.sf2), noise=np.float32(p.noise_var),
              Z=f32(p.Z), m=f32(p.m), s=f32(p.s),
              L=f32(np.eye(w.M) / np.sqrt(p.sf2)))

    def batch(t):
        X, y = w.batch(t)
        return f32(X), f32(y)
    return st, batch


def sample_positions(M, D, seed=2604):
    """Fixed recorded entries: lower-triangular (i, j) of L, indices of m~ /
    s~, and (i, d) of Z."""
    g = np.random.Generator(np.random.PCG64(seed))
    i = g.integers(0, M, N_SAMPLES)
    j = (g.uniform(size=N_SAMPLES) * (i + 1)).astype(np.int64)
    idx = g.choice(M, size=min(M, N_VEC_SAMPLES), replace=False)
    zi = g.integers(0, M, N_VEC_SAMPLES)
    zd = g.integers(0, D, N_VEC_SAMPLES)
    return dict(Li=i, Lj=j, v=idx, Zi=zi, Zd=zd)
