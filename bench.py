#!/usr/bin/env python3
"""Throughput of the inverse-free SVGP training iteration on one MI355X.

One step = one pass of the whole hot path on one mini-batch resident in HBM:
a natural-gradient step on L (gamma = 1), the preconditioned bound at the
updated L, and its hand-written backward (gradients for the lengthscales,
signal and noise variance, Z and m~), all in the HIP library.  The workload
is the paper-shaped regression configuration with D = 16, N = 1e6,
B = 4096, M = 1024 (synthetic data, seeded; see paper_2604_00697_amd.synth).

Prints one JSON line.  `value` is iterations per second of the bf16 form
(bf16 MFMA operands, fp32 accumulation, fp32 master L, fp64 final sums);
the fp32 form is timed on the same inputs and reported under "fp32".
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "train iters/sec (bound+backward+T natgrad) M=1024,B=4096, BF16 vs FP32; MFMA %"
PEAK_TFLOPS = {"bf16": 2500.0, "fp16": 2500.0, "fp32": 157.3}
N_BATCHES = 8
REPEATS = 5


# MFMA products of one step (the flop count of the MFMA percentage); the s~
# gradient's extra product is not requested by the step timed here.
STEP_GEMMS = ("ng_KL", "ng_gram", "ng_update", "bound_KL", "bound_gram", "bound_gram_E",
              "gemm_V", "gemm_U", "gemm_R_grad_uf", "syrk", "gemm_LC", "gemm_G_grad_uu")
# Sources whose change invalidates a stored HBM traffic measurement.
KERNEL_SOURCES = ("paper_2604_00697_amd/csrc/gemm.hpp", "paper_2604_00697_amd/csrc/epilogues.hpp",
                  "paper_2604_00697_amd/csrc/common.hpp", "paper_2604_00697_amd/csrc/ifsvgp.hip")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_sources_digest():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def kernel_traffic(kernel, workload, prec):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, each scaled by the counter's reading
    for a plain copy of known size), or None when there is none for this
    workload or the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_{prec}_hbm_traffic.md")
    try:
        with open(path) as fh:
            kv = dict(line.strip()[2:].split(": ", 1) for line in fh
                      if line.startswith("- ") and ": " in line)
        if kv.get("sources_digest") != kernel_sources_digest():
            return None
        return int(float(kv["traffic_bytes_per_launch"]))
    except (OSError, KeyError, ValueError):
        return None


def make_inputs(wname, dev):
    import numpy as np
    import torch
    from paper_2604_00697_amd import synth
    w = synth.workload(wname)
    p = synth.params_s1(w)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(np.asarray(a, np.float32))).to(dev)
    batches = []
    for it in range(N_BATCHES):
        X, y = w.batch(it)
        batches.append((t(X), t(y)))
    par = dict(ell=t(p.ell), sf2=t([p.sf2]), noise=t([p.noise_var]), Z=t(p.Z), m=t(p.m),
               s=t(p.s), L=t(p.L))
    return w, p, batches, par


def schedule(n, g0=1e-5, g1=1.0, ramp=10):
    """Log-linear NG step sizes g0 -> g1 over `ramp` steps, then constant."""
    import math
    out = []
    for t in range(n):
        f = min(t, ramp - 1) / (ramp - 1)
        out.append(10.0 ** (math.log10(g0) + (math.log10(g1) - math.log10(g0)) * f))
    return out


def time_form(prec, w, batches, par, L0, steps, warmup, kinds, dev, graphs=False, kuf_mode=None):
    import torch
    from paper_2604_00697_amd.lib import Context
    ctx = Context(w.M, w.B, w.D, prec, w.lik)
    ctx.set_graphs(graphs)
    if kuf_mode:
        ctx.set_kuf_mode(kuf_mode)
    L = L0.clone()
    F = torch.empty(1, dtype=torch.float64, device=dev)
    terms = torch.empty(8, dtype=torch.float64, device=dev)
    resid = torch.empty(1, dtype=torch.float64, device=dev)
    grads = ctx._grad_buffers(("ell", "sf2", "noise_var", "Z", "m"))

    def step(i):
        X, y = batches[i % len(batches)]
        ctx.step(X, y, w.N, par["ell"], par["sf2"], par["noise"], par["Z"], par["m"],
                 par["s"], L, [1.0], out=F, terms=terms, resid=resid, grads=grads)

    for i in range(warmup):
        step(i)
    torch.cuda.synchronize()
    if ctx.status() != 0:
        raise RuntimeError(f"{prec}: device status flag set during warmup")
    ctx.timing(list(kinds))
    ctx.timing_read()
    # REPEATS equal chunks of the timed steps, split by events on the stream
    # (no synchronisation inside the timed region)
    bounds = [round(k * steps / REPEATS) for k in range(REPEATS + 1)]
    evs = [torch.cuda.Event(enable_timing=True) for _ in bounds]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs[0].record()
    for k in range(REPEATS):
        for i in range(bounds[k], bounds[k + 1]):
            step(warmup + i)
        evs[k + 1].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    chunks = sorted(evs[k].elapsed_time(evs[k + 1]) / max(1, bounds[k + 1] - bounds[k])
                    for k in range(REPEATS))
    ctx.timing(False)
    kt = ctx.timing_read()
    status = ctx.status()
    flops = ctx.kernel_flops(w.B)
    per_launch = {k: kt[k][0] / max(kt[k][1], 1) for k in kinds}
    res = dict(ms_per_step=1e3 * (t1 - t0) / steps, iters_per_s=steps / (t1 - t0),
               repeats=dict(n=REPEATS, median_ms=round(chunks[REPEATS // 2], 4),
                            p10_ms=round(chunks[0], 4), p90_ms=round(chunks[-1], 4)),
               launch_ms=per_launch, flops=flops, status=status,
               F=F.item(), resid=terms[3].item())
    ctx.close()
    return res


def one_step(prec, w, batches, par, L0):
    """One iteration (NG step gamma = 1, bound, gradient) of the `prec` form
    from L0 on the first batch; host float64 copies of its outputs."""
    import torch
    from paper_2604_00697_amd.lib import Context
    ctx = Context(w.M, w.B, w.D, prec, w.lik)
    L = L0.clone()
    X, y = batches[0]
    F, terms, _, g = ctx.step(X, y, w.N, par["ell"], par["sf2"], par["noise"], par["Z"],
                              par["m"], par["s"], L, [1.0])
    torch.cuda.synchronize()
    out = dict(F=F.item(), data=terms[0].item(), KL=terms[1].item(),
               L=L.double().cpu().numpy(), status=ctx.status())
    out.update({k: v.double().cpu().numpy() for k, v in g.items()})
    ctx.close()
    return out


def accuracy(w, par, batches, L0, gpu):
    """Relative error of each form's F, terms, updated L and gradient blocks
    against one float64 oracle iteration from the same state and batch."""
    import numpy as np
    from oracle import svgp
    h = lambda t: t.double().cpu().numpy()
    X, y = batches[0]
    L_ref, _, ref = svgp.training_iteration(
        h(X), h(y), w.N, h(par["ell"]), h(par["sf2"])[0], h(par["noise"])[0], h(par["Z"]),
        h(par["m"]), h(par["s"]), h(L0), [1.0], lik=w.lik)
    b = ref["bound"]
    rel = lambda a, r: float(np.linalg.norm(np.ravel(a) - np.ravel(r)) /
                             max(np.linalg.norm(np.ravel(r)), 1e-300))
    out = {"reference": "float64 oracle, one iteration from the timed state on batch 0"}
    for prec, o in gpu.items():
        e = {"F": rel(o["F"], b["F"]), "data": rel(o["data"], b["data"]),
             "KL": rel(o["KL"], b["KL"]), "L": rel(o["L"], L_ref)}
        for k in ("ell", "sf2", "noise_var", "Z", "m"):
            if k in o:
                e["grad_" + k] = rel(o[k], ref[k])
        out[prec] = {k: float(f"{v:.3g}") for k, v in e.items()}
    return out


def kernel_breakdown(prec, w, batches, par, L0, steps, dev):
    """Per-kernel mean durations (all kinds timed; a separate, untimed pass)."""
    import torch
    from paper_2604_00697_amd.lib import Context
    ctx = Context(w.M, w.B, w.D, prec, w.lik)
    L = L0.clone()
    for i in range(3):
        X, y = batches[i % len(batches)]
        ctx.step(X, y, w.N, par["ell"], par["sf2"], par["noise"], par["Z"], par["m"], par["s"],
                 L, [1.0])
    ctx.timing(True)
    ctx.timing_read()
    for i in range(steps):
        X, y = batches[i % len(batches)]
        ctx.step(X, y, w.N, par["ell"], par["sf2"], par["noise"], par["Z"], par["m"], par["s"],
                 L, [1.0])
    kt = ctx.timing_read()
    ctx.close()
    return {k: round(ms / steps * 1e3, 2) for k, (ms, c) in kt.items() if c}


def next_rows(prec, w, batches, par, L0, dev, reps=5):
    """Timing of the entry points beside the iteration, on the same workload
    (median over `reps` calls, each bracketed by events on the stream):
    prediction at 4 B test points with their log densities and NLPD, the
    adaptive NG loop with the residual rule (4 checked steps, none stopped),
    the NG loop with the variance-gap rule (3 checked steps on one batch),
    the Hutchinson bound, the multi-output bound with its gradient, grouped
    iterations of independent problems against separate calls, and one Adam
    step on Z."""
    import torch
    from paper_2604_00697_amd.lib import Context
    ctx = Context(w.M, w.B, w.D, prec, w.lik)
    Xt = torch.cat([b[0] for b in batches[:4]])
    yt = torch.cat([b[1] for b in batches[:4]])
    noise = par["noise"] if w.lik == "gaussian" else None

    def timed(fn, setup=None):
        ts = []
        for _ in range(reps + 1):
            a = setup() if setup else None
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record()
            fn(a)
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        ts = sorted(ts[1:])
        return ts[len(ts) // 2]

    out = {}
    ms = timed(lambda _: ctx.predict(Xt, par["ell"], par["sf2"], par["Z"], par["m"], par["s"],
                                     L0, y=yt, noise=noise))
    out["predict"] = {"points": int(Xt.shape[0]), "ms": round(ms, 4),
                      "points_per_s": round(Xt.shape[0] / (ms * 1e-3), 1)}
    ms_fix = timed(lambda L: ctx.natgrad(par["Z"], par["ell"], par["sf2"], par["s"], L,
                                         [1.0] * 4), setup=L0.clone)
    ms_tol = timed(lambda L: ctx.natgrad_tol(par["Z"], par["ell"], par["sf2"], par["s"], L,
                                             [1.0] * 4, 0.0), setup=L0.clone)
    out["natgrad_residual_rule"] = {"steps": 4, "ms_per_step": round(ms_tol / 4, 4),
                                    "fixed_loop_ms_per_step": round(ms_fix / 4, 4)}
    if w.lik == "gaussian":
        sig2 = 0.5 * float(par["s"].min().item())
        ms_gap = timed(lambda L: ctx.natgrad_gap(batches[0][0], par["Z"], par["ell"], par["sf2"],
                                                 par["noise"], par["s"], L, [1.0] * 3, sig2, 0.0),
                       setup=L0.clone)
        out["natgrad_gap_rule"] = {"steps": 3, "B": w.B, "ms_per_step": round(ms_gap / 3, 4)}
    # the paper's Hutchinson setting (Appendix on approximate bound evaluation):
    # B = 100, K = 256 probes; exact bound vs the estimate on the same inputs,
    # alone and with the gradient
    # (D = 8 synthetic regression data), at the paper's M = 2000 and at
    # M = 8192, where the cubic traces outweigh the launches
    if w.lik == "gaussian":
        import numpy as np
        from paper_2604_00697_amd import synth
        out["hutchinson_bound"] = []
        for Mh in (2000, 8192):
            wu = synth.Workload(f"M{Mh}_B100_D8", D=8, N=40_000, B=100, M=Mh)
            pu = synth.params_s1(wu)
            tt = lambda a: torch.from_numpy(np.ascontiguousarray(np.asarray(a, np.float32))).to(dev)
            Xu, yu = wu.batch(0)
            du = dict(X=tt(Xu), y=tt(yu), ell=tt(pu.ell), sf2=tt([pu.sf2]),
                      noise=tt([pu.noise_var]), Z=tt(pu.Z), m=tt(pu.m), s=tt(pu.s), L=tt(pu.L))
            Kp = 256
            om = tt(synth.rng(synth.SEED_PERTURB + 29).choice([-1.0, 1.0], size=(Kp, wu.M)))
            cu = Context(wu.M, 448, wu.D, prec, "gaussian")
            args = (du["X"], du["y"], wu.N, du["ell"], du["sf2"], du["noise"], du["Z"], du["m"],
                    du["s"], du["L"])
            ms_ex = timed(lambda _: cu.bound(*args))
            ms_hu = timed(lambda _: cu.bound_hutch(*args, om))
            # bound and gradient (ell, sf2, noise, Z, m~) at fixed L
            ms_exg = timed(lambda _: (cu.bound(*args), cu.bound_bwd(*args)))
            ms_hug = timed(lambda _: (cu.bound_hutch(*args, om), cu.bound_hutch_bwd(*args, om)))
            out["hutchinson_bound"].append(
                {"M": wu.M, "B": wu.B, "K": Kp, "exact_ms": round(ms_ex, 4),
                 "hutchinson_ms": round(ms_hu, 4), "speedup": round(ms_ex / ms_hu, 3),
                 "exact_with_grad_ms": round(ms_exg, 4),
                 "hutchinson_with_grad_ms": round(ms_hug, 4),
                 "speedup_with_grad": round(ms_exg / ms_hug, 3)})
            torch.cuda.synchronize()
            if cu.status() != 0:
                raise RuntimeError("device status flag set in the Hutchinson timing")
            cu.close()
            del cu, du, om
            torch.cuda.empty_cache()
    # multi-output (Q outputs sharing Z, the kernel, S~ and T) at the workload's
    # shapes: bound and gradient for Q = 8 outputs in one call, against Q
    # single-output bound + gradient calls on the same inputs
    import numpy as np
    Qm = 8
    gq = np.random.Generator(np.random.PCG64(8))
    Xb, yb = batches[0]
    if w.lik == "gaussian":
        Yq = yb[:, None] + 0.1 * torch.from_numpy(gq.standard_normal((w.B, Qm)).astype(np.float32)).to(dev)
    else:
        Yq = yb[:, None].repeat(1, Qm)
    Yq = Yq.contiguous()
    Mq = (par["m"][None, :] + 0.1 * torch.from_numpy(gq.standard_normal((Qm, w.M)).astype(np.float32)).to(dev)).contiguous()
    margs = (Xb, Yq, w.N, par["ell"], par["sf2"], noise, par["Z"], Mq, par["s"], L0)
    ms_multi = timed(lambda _: (ctx.bound_multi(*margs), ctx.bound_multi_bwd(*margs)))
    ycols = [Yq[:, q].contiguous() for q in range(Qm)]

    def singles(_):
        for q in range(Qm):
            a1 = (Xb, ycols[q], w.N, par["ell"], par["sf2"], noise, par["Z"], Mq[q], par["s"], L0)
            ctx.bound(*a1)
            ctx.bound_bwd(*a1)
    ms_single = timed(singles)
    out["multi_output"] = {"Q": Qm, "B": w.B, "with_grad_ms": round(ms_multi, 4),
                           "single_output_calls_ms": round(ms_single, 4),
                           "speedup": round(ms_single / ms_multi, 3)}
    # independent problems (one T each, as the layers of a deep GP): G
    # iterations in one grouped call against G ifsvgp_step calls, at the
    # workload's shapes (G = 4) and for small layers (M = 256, B = 1024, D = 8,
    # G = 8), where the launches dominate
    from paper_2604_00697_amd.lib import GroupContext
    out["group"] = []
    for G, (Mg, Bg, Dg) in ((4, (w.M, w.B, w.D)), (8, (256, 1024, 8))):
        from paper_2604_00697_amd import synth
        wg = w if (Mg, Bg, Dg) == (w.M, w.B, w.D) else synth.Workload(
            f"M{Mg}_B{Bg}_D{Dg}", D=Dg, N=100_000, B=Bg, M=Mg, lik=w.lik)
        pg = synth.params_s1(wg)
        tg = lambda a: torch.from_numpy(np.ascontiguousarray(np.asarray(a, np.float32))).to(dev)
        probs = []
        for q in range(G):
            Xq, yq = wg.batch(q)
            probs.append(dict(X=tg(Xq), y=tg(yq), ell=tg(pg.ell), sf2=tg([pg.sf2]),
                              noise=tg([pg.noise_var]) if wg.lik == "gaussian" else None,
                              Z=tg(pg.Z), m=tg(pg.m), s=tg(pg.s),
                              L=tg(np.eye(wg.M))))
        gctx = GroupContext(G, wg.M, wg.B, wg.D, prec, wg.lik)
        sctx = Context(wg.M, wg.B, wg.D, prec, wg.lik)
        ms_grp = timed(lambda _: gctx.step_group(probs, wg.N, [1e-3]))

        def seq(_):
            for p_ in probs:
                sctx.step(p_["X"], p_["y"], wg.N, p_["ell"], p_["sf2"], p_["noise"], p_["Z"],
                          p_["m"], p_["s"], p_["L"], [1e-3])
        ms_seq = timed(seq)
        torch.cuda.synchronize()
        if gctx.status() != 0 or sctx.status() != 0:
            raise RuntimeError("device status flag set in the grouped timing")
        out["group"].append({"G": G, "M": wg.M, "B": wg.B, "D": wg.D,
                             "grouped_ms": round(ms_grp, 4), "sequential_steps_ms": round(ms_seq, 4),
                             "speedup": round(ms_seq / ms_grp, 3)})
        gctx.close()
        sctx.close()
    g = torch.zeros_like(par["Z"]) + 1e-3

    def adam_setup():
        return (par["Z"].clone(), torch.zeros_like(par["Z"]), torch.zeros_like(par["Z"]))
    ms_adam = timed(lambda a: ctx.adam(a[0], g, a[1], a[2], 1, ascend=True), setup=adam_setup)
    out["adam_Z"] = {"params": int(par["Z"].numel()), "us": round(ms_adam * 1e3, 2)}
    torch.cuda.synchronize()
    if ctx.status() != 0:
        raise RuntimeError("device status flag set in the entry-point timings")
    ctx.close()
    return out


def cpu_baseline(w, p, budget_s=20.0):
    """The float64 oracle (as it stands) on the host cores: iterations per second
    on the same workload, timed over a bounded number of full iterations."""
    import numpy as np
    from oracle import svgp
    try:
        from threadpoolctl import threadpool_info
        threads = max(i.get("num_threads", 1) for i in threadpool_info()) or 1
    except Exception:
        threads = os.cpu_count()
    X, y = w.batch(0)
    Kt = svgp.ktilde(p.Z, p.ell, p.sf2, p.s)
    L, _ = svgp.ng_steps(np.eye(w.M), Kt, schedule(20))
    n, t0 = 0, time.perf_counter()
    while True:
        X, y = w.batch(n % N_BATCHES)
        L, _, _ = svgp.training_iteration(X, y, w.N, p.ell, p.sf2, p.noise_var, p.Z, p.m, p.s,
                                          L, [1.0])
        n += 1
        el = time.perf_counter() - t0
        if el >= budget_s or n >= 20:
            break
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((l.split(":", 1)[1].strip() for l in fh if l.startswith("model name")), "")
    except OSError:
        pass
    aff = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return dict(value=round(n / el, 4), unit="iters/s", cores=int(threads), kind="oracle",
                sample=f"{n} full iterations (NG step + bound + gradient) of the same "
                       f"workload in float64 NumPy, {el:.1f} s, BLAS threads {threads}, "
                       f"{aff} cores in the affinity mask, {model}")


def c4_leg(args, dev, dominant, second):
    """The M = 2048, B = 8192, D = 32 workload (the MFMA target's workload), timed
    like the headline one for the bf16 form (and fp32 unless --no-fp32), with the
    roofline of its dominant kernel; no oracle work."""
    import torch
    from paper_2604_00697_amd.lib import Context
    log("bench: C4 leg: building inputs")
    w, _, batches, par = make_inputs("C4", dev)
    c32 = Context(w.M, w.B, w.D, "fp32", w.lik)
    L0 = par["L"].clone()
    c32.natgrad(par["Z"], par["ell"], par["sf2"], par["s"], L0, schedule(30))
    torch.cuda.synchronize()
    c32.close()
    out = {"workload": f"C4: SE-ARD regression, D={w.D}, N={w.N}, B={w.B}, M={w.M}, "
                       f"gaussian likelihood; same step as the headline"}
    forms = ["bf16"] + ([] if args.no_fp32 else ["fp32"])
    for prec in forms:
        steps, warm = args.c4_steps, args.c4_steps
        if prec == "fp32":
            steps, warm = max(20, steps // 5), max(20, warm // 5)
        log(f"bench: C4 {prec}: {warm} warmup + {steps} steps")
        r = time_form(prec, w, batches, par, L0, steps, warm, (dominant,), dev,
                      graphs=args.graphs)
        f_iter = sum(r["flops"][k] for k in STEP_GEMMS)
        peak = PEAK_TFLOPS[prec]
        ms = r["launch_ms"][dominant]
        tf = r["flops"][dominant] / (ms * 1e-3) / 1e12
        out[prec] = {"value": round(r["iters_per_s"], 3), "ms_per_step": round(r["ms_per_step"], 4),
                     "repeats": r["repeats"], "flops_per_step": f_iter,
                     "mfma_pct": round(100.0 * f_iter / (r["ms_per_step"] * 1e-3) / (peak * 1e12), 3),
                     "roofline": {"bound": "mfma", "kernel": dominant, "achieved": round(tf, 3),
                                  "peak": peak, "unit": "TFLOP/s", "frac": round(tf / peak, 4),
                                  "traffic": kernel_traffic(dominant, "C4", prec),
                                  "flops_per_launch": r["flops"][dominant],
                                  "avg_launch_us": round(ms * 1e3, 3)},
                     "status": r["status"]}
        if prec == "bf16":
            # the same step with K_uf's tiles stored once beside the NG step
            # instead of generated inside V's launch (bit-identical results)
            log(f"bench: C4 bf16, K_uf stored: {warm} warmup + {steps} steps")
            rs = time_form(prec, w, batches, par, L0, steps, warm, (dominant,), dev,
                           graphs=args.graphs, kuf_mode="stored")
            out["bf16_kuf_stored"] = {"value": round(rs["iters_per_s"], 3),
                                      "ms_per_step": round(rs["ms_per_step"], 4),
                                      "repeats": rs["repeats"], "status": rs["status"]}
        log(f"bench: C4 {prec} {r['ms_per_step']:.3f} ms/step")
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    # enough untimed steps (about half a second at M=1024) for the GPU clocks
    # to settle before the timed region
    ap.add_argument("--warmup", type=int, default=2000)
    ap.add_argument("--workload", default="C3")
    ap.add_argument("--prec", default="bf16", choices=["bf16", "fp16", "fp32"])
    ap.add_argument("--no-fp32", action="store_true", help="skip the fp32 comparison form")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle cpu_baseline")
    ap.add_argument("--breakdown", action="store_true", help="add per-kernel mean durations")
    ap.add_argument("--no-next", action="store_true",
                    help="skip the timings of prediction, the adaptive NG loops and Adam")
    ap.add_argument("--no-c4", action="store_true",
                    help="skip the M=2048, B=8192, D=32 leg (the target workload of the MFMA goal)")
    ap.add_argument("--c4-steps", type=int, default=300)
    ap.add_argument("--graphs", action="store_true",
                    help="replay recorded HIP graphs instead of direct calls (the dominant "
                         "kernel's timing then runs the timed steps directly anyway)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="also run one plain device-to-device copy of BYTES bytes (the "
                         "reference dispatch for scaling HBM byte counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: the library runs on one GPU only (the iteration's multi-GPU "
              "sharding is a design, not implemented); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2604_00697_amd.lib import Context
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    log(f"bench: workload {args.workload}, building inputs")
    w, p, batches, par = make_inputs(args.workload, dev)

    # converge L towards chol(K~^{-1}) before timing (gamma = 1 from here on)
    c32 = Context(w.M, w.B, w.D, "fp32", w.lik)
    L0 = par["L"].clone()
    r = c32.natgrad(par["Z"], par["ell"], par["sf2"], par["s"], L0, schedule(30))
    torch.cuda.synchronize()
    log(f"bench: NG schedule residuals first/last {r[0].item():.3e} / {r[-1].item():.3e}")
    c32.close()

    # the kernel with the longest launches in the profiles of both workloads
    # (R = L U and its gradient epilogue, on the side stream), and the forward's
    # largest product for comparison
    dominant, second = "gemm_R_grad_uf", "gemm_U"
    forms = [args.prec] + ([] if args.no_fp32 or args.prec == "fp32" else ["fp32"])
    # the fp16-operand variant of the precision form, beside bf16
    if args.prec == "bf16" and not args.no_fp32 and w.lik == "gaussian":
        forms.append("fp16")
    res = {}
    for prec in forms:
        log(f"bench: timing {prec}: {args.warmup} warmup + {args.steps} steps")
        res[prec] = time_form(prec, w, batches, par, L0, args.steps, args.warmup,
                              (dominant,), dev,
                              graphs=args.graphs)
        log(f"bench: {prec} {res[prec]['ms_per_step']:.3f} ms/step, {dominant} "
            f"{res[prec]['launch_ms'][dominant] * 1e3:.1f} us, status {res[prec]['status']}")
    main_r = res[args.prec]
    # the comparison kernel's launches, timed in a short run of their own so
    # that the timed region above stamps events on one kind only
    log(f"bench: {args.prec} {second} launches")
    sec = time_form(args.prec, w, batches, par, L0, 200, 50, (second,), dev, graphs=args.graphs)
    main_r["launch_ms"][second] = sec["launch_ms"][second]
    flops = main_r["flops"]
    f_iter = sum(flops[k] for k in STEP_GEMMS)
    peak = PEAK_TFLOPS[args.prec]

    def roofline(kernel):
        ms = main_r["launch_ms"][kernel]
        tf = flops[kernel] / (ms * 1e-3) / 1e12
        return {"bound": "mfma", "kernel": kernel, "achieved": round(tf, 3), "peak": peak,
                "unit": "TFLOP/s", "frac": round(tf / peak, 4),
                "traffic": kernel_traffic(kernel, args.workload, args.prec),
                "flops_per_launch": flops[kernel], "avg_launch_us": round(ms * 1e3, 3)}
    out = {
        "metric": METRIC,
        "value": round(main_r["iters_per_s"], 3),
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_r["ms_per_step"], 4),
        "repeats": main_r["repeats"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.prec,
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: SE-ARD "
                               f"{'regression' if w.lik == 'gaussian' else 'classification'}, "
                               f"D={w.D}, N={w.N}, B={w.B}, M={w.M}, {w.lik} likelihood; step = "
                               f"1 NG step (gamma=1) + bound + backward",
                   "M": w.M, "B": w.B, "D": w.D, "N": w.N, "state": "S1"},
        "mfma_pct": round(100.0 * f_iter / (main_r["ms_per_step"] * 1e-3) / (peak * 1e12), 3),
        "flops_per_step": f_iter,
        "roofline": roofline(dominant),
        "roofline_" + second: roofline(second),
    }
    if "fp32" in res and args.prec != "fp32":
        r32 = res["fp32"]
        out["fp32"] = {"value": round(r32["iters_per_s"], 3),
                       "ms_per_step": round(r32["ms_per_step"], 4),
                       "mfma_pct": round(100.0 * f_iter / (r32["ms_per_step"] * 1e-3) /
                                         (PEAK_TFLOPS["fp32"] * 1e12), 3),
                       "F": r32["F"]}
        out["F"] = main_r["F"]
    if "fp16" in res and args.prec != "fp16":
        r16 = res["fp16"]
        out["fp16"] = {"value": round(r16["iters_per_s"], 3),
                       "ms_per_step": round(r16["ms_per_step"], 4),
                       "mfma_pct": round(100.0 * f_iter / (r16["ms_per_step"] * 1e-3) /
                                         (PEAK_TFLOPS["fp16"] * 1e12), 3),
                       "F": r16["F"]}
    if args.workload == "C3" and not args.no_c4:
        out["c4"] = c4_leg(args, dev, dominant, second)
    if not args.no_next:
        log("bench: prediction, adaptive NG loops, Adam")
        out["entry_points"] = next_rows(args.prec, w, batches, par, L0, dev)
    if args.breakdown:
        out["kernel_us"] = kernel_breakdown(args.prec, w, batches, par, L0, 20, dev)
    if not args.no_cpu:
        log("bench: cpu_baseline (oracle on host cores)")
        out["cpu_baseline"] = cpu_baseline(w, p)
        try:
            from threadpoolctl import threadpool_limits
            log("bench: cpu_baseline on one thread")
            with threadpool_limits(limits=1):
                one = cpu_baseline(w, p, budget_s=10.0)
            out["cpu_baseline_1thread"] = {k: one[k] for k in ("value", "unit", "sample")}
        except ImportError:
            pass
        log("bench: accuracy of each form against one oracle iteration")
        gpu = {f: one_step(f, w, batches, par, L0) for f in forms}
        out["accuracy"] = accuracy(w, par, batches, L0, gpu)
    if args.copy_calibration > 0:
        n = args.copy_calibration // 4
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"bench: copy calibration {4 * n} bytes")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
