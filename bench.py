"""Benchmark: Crank-Nicolson steps per second at 255^3, mixed precision vs
float64, on one MI355X.

Workload (3D non-symmetric): (alpha, beta, gamma) = (0.4, 0.6, 0.8),
k+ = (1.0, 0.8, 1.2), k- = (0.5, 1.0, 0.3), 255^3 interior unknowns, 16 CN
steps to T = 1, f = 8 seeded Gaussian bumps, u0 = 0, left-preconditioned
GMRES(20) with the sine-transform preconditioner from u^{m-1}.  Both solvers
run at the paper's tolerance 1e-9 (workloads.HEADLINE_SOLVER), which keeps
u^M within 1e-8 of a tightly solved float64 trajectory in the 2-norm and the
max-norm; the figures at the configuration's literal tol 1e-8 are reported
beside them.

A step is one fsd_cn_step: right-hand side, then the solve.  The headline
value is the mixed-precision solver (float32 inner GMRES, float64 defect
correction with the float64 stopping test), against the float64 solver.
Timed steps come only from steps 2..16 of the workload: each timed pass
restarts from u0, runs step 1 untimed and times `--steps` steps (past step
16 it restarts again, step 1 untimed); `value` is the median over
`--repeats` passes, with the interquartile range beside it.

    python bench.py [--steps K] [--warmup W] [--repeats R] [--gpus 1] [--no-cpu]

Prints one JSON line (rank 0).  Inputs are generated on the host and copied
to the GPU before timing.  The timed passes run without per-kernel events;
the per-kernel figures (`roofline`, `roofline_kernels`) come from one more
pass over the same steps with the library's hipEvents around each launch on
its stream.  `hbm_peak` is a measured stream copy (fsd_hbm_copy);
`cpu_baseline` times the float64 oracle on this host for a bounded sample,
normalised per GMRES iteration.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

# Hardware queues per process (read when the HIP runtime starts, so before
# torch is imported).  HIP's default of 4 leaves the batched executor's lanes
# sharing queues: at 8 the 64-instance workload runs 1,767 against 1,446
# instance-steps/s (16 gives no more).  Values below 8 are raised to 8; a
# larger value set by the caller is kept.
try:
    _hwq = int(os.environ.get("GPU_MAX_HW_QUEUES", "4"))
except ValueError:
    _hwq = 4
if _hwq < 8:
    os.environ["GPU_MAX_HW_QUEUES"] = "8"

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
METRIC = "CN steps/s at 255^3, mixed vs FP64 (rel err 1e-8); Toeplitz matvec HBM GB/s"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


class Trajectory:
    """The headline workload's CN trajectory u^0 = u0, u^1, ..., u^M.  A step
    past u^M starts the trajectory again from u0 (the step after is step 1
    again), so no step ever runs past T."""

    def __init__(self, prob, u0, F, M):
        self.prob, self.u0, self.F, self.M = prob, u0, F, M
        self.u = u0.clone()
        self.m = 0            # steps taken since u0

    def restart(self):
        self.u = self.u0.clone()
        self.m = 0
        self.prob.reset_history()

    def step(self):
        if self.m == self.M:
            self.restart()
        self.u, st = self.prob.cn_step(self.u, self.F, out=self.u)
        self.m += 1
        return st


def timed_steps(traj, K):
    """Time K steps of the trajectory taken only from steps 2..M: step 1 of
    each pass (after the restart from u0) runs untimed.  Each run of
    consecutive timed steps is bracketed by torch.cuda.synchronize(); the
    time is their sum.  Returns (seconds, iterations, outer steps) of the
    timed steps."""
    import torch
    total, its, outer = 0.0, [], []
    done = 0
    while done < K:
        if traj.m in (0, traj.M):
            if traj.m == traj.M:
                traj.restart()
            traj.step()                      # step 1: untimed
        seg = min(K - done, traj.M - traj.m)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(seg):
            st = traj.step()
            its.append(st["iters"])
            outer.append(st["outer_iters"])
        torch.cuda.synchronize()
        total += time.perf_counter() - t0
        done += seg
    return total, its, outer


def repeat_timing(prob, u0, F, M, steps, warmup, repeats, profile=False):
    """W warm-up steps, then `repeats` timed passes of `steps` steps, each
    from u0 with step 1 untimed (the same steps 2..steps+1 every time: the
    solves are deterministic).  With `profile`, one more pass with the
    library's per-launch hipEvents on its stream gives the per-kernel
    figures (the timed passes run without events: an event pair around every
    launch adds about 10% to the wall time at 255^3).  Returns a dict with
    the per-pass CN steps/s, their median and interquartile range, the
    iterations of the timed steps and the profile."""
    traj = Trajectory(prob, u0, F, M)
    for _ in range(warmup):
        traj.step()
    rates, its, outer = [], None, None
    for _ in range(repeats):
        traj.restart()
        t, it, ou = timed_steps(traj, steps)
        rates.append(steps / t)
        if its is None:
            its, outer = it, ou
        elif it != its:
            log(f"note: iteration counts differ between repeats: {it} vs {its}")
    prof = None
    if profile:
        traj.restart()
        traj.step()
        prob.profile(True)
        prob.profile_read()
        _, it, _ = timed_steps(traj, steps)
        prof = prob.profile_read()
        prob.profile(False)
    q = np.percentile(rates, [25, 50, 75])
    return {"steps_per_s": float(q[1]), "iqr": [float(q[0]), float(q[2])],
            "per_repeat": [round(r, 3) for r in rates], "iters": its, "outer": outer,
            "prof": prof}


def final_state(prob, u0, F, M):
    """u^M of the whole trajectory (untimed), for the error figures."""
    prob.reset_history()
    u = u0.clone()
    for _ in range(M):
        u, _ = prob.cn_step(u, F)
    return u


def errors(u, uref):
    import torch
    return {"rel_2norm": float(torch.linalg.vector_norm(u - uref) / torch.linalg.vector_norm(uref)),
            "rel_maxnorm": float((u - uref).abs().max() / uref.abs().max())}


def cpu_baseline(w, gpu_mean_iters, iters=10):
    """Float64 oracle on this host, normalised per GMRES iteration: one
    right-hand side and the first `iters` GMRES iterations of step 1 are
    timed, and the rate is given for a step of the mean iteration count of
    the GPU's timed steps (steps 2..M, float64 solver at the same
    tolerance; the oracle's counts agree within one)."""
    from oracle import cn, operators as op
    prob = op.Problem(3, w.n, w.delta, w.kplus, w.kminus, T=w.T, M=w.M)
    t0 = time.perf_counter()
    op.apply_rhs(prob, w.u0, w.F)
    t_rhs = time.perf_counter() - t0
    t0 = time.perf_counter()
    cn.run(prob, w.u0, lambda m: w.F, tol=1e-30, x0_mode="prev", solver="gmres", steps=1,
           maxit=iters)
    t_run = time.perf_counter() - t0
    t_iter = max(t_run - t_rhs, 0.0) / iters
    t_step = t_rhs + gpu_mean_iters * t_iter
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count()
    return {"value": round(1.0 / t_step, 5), "unit": "CN steps/s", "cores": cores, "kind": "oracle",
            "sample": f"float64 NumPy/SciPy oracle on {cpu_model()}: one right-hand side "
                      f"({t_rhs:.2f} s) and {iters} GMRES iterations of step 1 "
                      f"({t_iter:.2f} s each) of the same workload, scaled to a step of "
                      f"{gpu_mean_iters:.2f} iterations (the mean over steps 2..16 of the GPU "
                      f"float64 solver at the same tolerance): {t_step:.1f} s per CN step"}


def hbm_peak(nbytes=1 << 30, reps=20):
    """Measured HBM peak: fsd_hbm_copy of nbytes (read nbytes, write nbytes),
    median over reps calls timed with hipEvents on the current stream."""
    import torch
    from paper_2511_21198_amd.solver import hbm_copy
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda").fill_(1)
    b = torch.empty_like(a)
    st = torch.cuda.current_stream()
    for _ in range(3):
        hbm_copy(a, b, st)
    ms = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        hbm_copy(a, b, st)
        e1.record(st)
        e1.synchronize()
        ms.append(e0.elapsed_time(e1))
    med = float(np.median(ms))
    del a, b
    return {"kernel": "fsd_hbm_copy (k_stream_copy)", "bytes_per_call": 2 * nbytes,
            "median_ms": round(med, 4), "gbps": round(2 * nbytes / (med * 1e-3) / 1e9, 1)}


TRAFFIC_JSON = os.path.join(ROOT, "profiles", "hbm_traffic_3d_nonsym_255.json")


def counter_traffic(kind):
    """HBM bytes per launch of a kernel kind from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary, or None when there is none or when the
    kernel sources changed after it was taken."""
    try:
        with open(TRAFFIC_JSON) as f:
            doc = json.load(f)
    except (OSError, ValueError):
        return None
    from paper_2511_21198_amd.rocprof_summary import source_hash
    e = doc.get("kinds", {}).get(kind, {})
    if e.get("source_hash") != source_hash(kind):
        return None
    return e.get("hbm_bytes_per_dispatch")


def operator_bench(w, peak, reps=100):
    """The operators at the workload's size, each called `reps` times: the
    float64 and float32 Toeplitz matvec (fsd_apply_A, fsd_apply_A32) and the
    float64 and float32 preconditioner (fsd_apply_Pinv, fsd_apply_Pinv32).
    Per call (hipEvents on the library's stream around each call, median):
    (i) algorithmic GB/s, 2 N b / t with b the bytes of the operator's
    arithmetic type (read x, write y); (ii) pass-level GB/s, the bytes every
    line pass must read and write over the summed pass durations (library
    profiler, hipEvents per launch).  The calls also pack and unpack the
    dense float64 ABI layout, which (i) includes and (ii) does not."""
    import torch
    from paper_2511_21198_amd.solver import Problem
    N = int(np.prod(w.n))
    p = Problem(3, w.n, w.delta, w.kplus, w.kminus, M=w.M, T=w.T, solver="gmres", precision="mixed")
    x = torch.from_numpy(w.F).cuda()
    y = torch.empty_like(x)
    out = {}
    for name, fn, b in (("apply_A_fp64", p.apply_A, 8), ("apply_A_fp32", p.apply_A32, 4),
                        ("apply_Pinv_fp64", p.apply_Pinv, 8), ("apply_Pinv_fp32", p.apply_Pinv32, 4)):
        for _ in range(5):
            fn(x, out=y)
        st = p.stream
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(reps)]
        for e0, e1 in ev:
            e0.record(st)
            fn(x, out=y)
            e1.record(st)
        torch.cuda.synchronize()
        ms = float(np.median([e0.elapsed_time(e1) for e0, e1 in ev]))
        p.profile(True)
        p.profile_read()
        for _ in range(reps):
            fn(x, out=y)
        prof = p.profile_read()
        p.profile(False)
        pass_ms = sum(v["total_ms"] for v in prof.values()) / reps
        pass_bytes = sum(v["bytes"] for v in prof.values()) / reps
        alg = 2 * N * b / (ms * 1e-3) / 1e9
        pl = pass_bytes / (pass_ms * 1e-3) / 1e9
        out[name] = {"median_ms": round(ms, 4), "algorithmic_gbps": round(alg, 1),
                     "passes_ms": round(pass_ms, 4), "pass_level_gbps": round(pl, 1),
                     "pass_level_frac_datasheet": round(pl / HBM_PEAK_GBPS, 3),
                     "pass_level_frac_measured": round(pl / peak, 3) if peak else None,
                     "passes": {k: {"avg_ms": round(v["avg_ms"], 4), "gbps": round(v["gbps"], 1)}
                                for k, v in prof.items()}}
        log(f"operator {name}: {out[name]['median_ms']} ms, pass level {out[name]['pass_level_gbps']} GB/s")
    del p
    out["note"] = (f"{reps} calls each at {w.n[0]}^3; (i) algorithmic and (ii) pass-level GB/s as "
                   "defined in the function docstring; (iii) DRAM bytes from rocprofv3 counters "
                   "are in profiles/")
    return out


WEIGHTS = os.path.join(ROOT, "paper_2511_21198_amd", "weights", "warmstart_3d_sym.npy")


def learned_workload(a, seed=10001, n=255, M=200):
    """Learned warm start workload (3D symmetric, orders drawn for the
    evaluation seed, moving bumps, M steps to T = 1, tol 1e-8): plain float64
    PCG from u^{m-1} against the same solver from the network's guess (with
    the residual guard), float64 and mixed precision, and linear
    extrapolation in time (the network's base guess).  All sources F^{m-1/2} are generated on the GPU
    before timing; a step includes the network inference when it is used."""
    import torch
    import workloads
    from paper_2511_21198_amd.solver import Problem
    w = workloads.config_learned(seed, n=n, M=M)
    dev = torch.device("cuda:0")
    dt = w.T / w.M
    Fs = [workloads.bumps_source_torch([n] * 3, w.bumps["c0"] + w.bumps["v"] * ((m - 0.5) * dt),
                                       w.bumps["width"], dev) for m in range(1, M + 1)]
    u0 = torch.zeros((n, n, n), dtype=torch.float64, device=dev)
    common = dict(dim=3, n=[n] * 3, delta=w.delta, kplus=w.kplus, kminus=w.kminus, M=w.M, T=w.T,
                  solver="pcg", tol=w.tol)
    params = None
    net = None
    if os.path.exists(WEIGHTS):
        from paper_2511_21198_amd import warmstart
        params = torch.from_numpy(np.load(WEIGHTS)).to(dev)
        net = warmstart.Net(n, n, n)
    out = {"workload": f"3D symmetric {n}^3, (alpha,beta,gamma)={np.round(w.delta, 3).tolist()} "
                       f"(seed {seed}), k=1, {M} CN steps to T=1, 8 moving seeded bumps, u0=0, "
                       "PCG, tol 1e-8",
           "weights": os.path.relpath(WEIGHTS, ROOT) if net else None}
    variants = [("fp64_prev", "fp64", "prev"), ("fp64_extrap", "fp64", "extrap"),
                ("mixed_prev", "mixed", "prev"), ("mixed_extrap", "mixed", "extrap")]
    if net:
        variants += [("fp64_net", "fp64", "guarded"), ("mixed_net", "mixed", "guarded")]
    finals = {}
    for name, prec, x0 in variants:
        p = Problem(**common, precision=prec, inner_tol=1e-4, x0=x0)
        p.autotune()
        eta = [p.coefficients(i)[2] for i in range(3)]
        u = u0.clone()
        un = torch.empty_like(u)
        up = torch.empty_like(u)
        guess = torch.empty_like(u) if x0 == "guarded" else None
        its, fb = [], 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for m in range(M):
            if m == 1:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
            if guess is not None:
                net.predict(params, u, Fs[m], dt, eta, u_prev=up if m > 0 else None,
                            F_prev=Fs[m - 1] if m > 0 else None, out=guess)
            un, st = p.cn_step(u, Fs[m], guess=guess, out=un)
            its.append(st["iters"])
            fb += st["x0_fallback"]
            up, u, un = u, un, up
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        finals[name] = u.clone()
        out[name] = {"steps_per_s": round((M - 1) / t, 2), "mean_iters": round(float(np.mean(its)), 3),
                     "iters_first10": its[:10]}
        if x0 == "guarded":
            out[name]["fallbacks"] = fb
        log(f"learned {name}: {out[name]}")
        del p
    pref = Problem(**{**common, "tol": 1e-12}, precision="fp64", x0="prev")
    u = u0.clone()
    for m in range(M):
        u, _ = pref.cn_step(u, Fs[m])
    nrm = torch.linalg.vector_norm(u)
    for name in finals:
        out[name]["rel_err_vs_tight_fp64"] = float(torch.linalg.vector_norm(finals[name] - u) / nrm)
    base = out["fp64_prev"]["steps_per_s"]
    for name in finals:
        out[name]["speedup_vs_fp64_prev"] = round(out[name]["steps_per_s"] / base, 3)
    return out


def batched_workload(a, streams=8, steps=8):
    """64 independent instances (32 2D with n per axis in {127, 255, 511,
    1023}, 32 3D with n in {63, 95, 127}; orders U(0.1, 0.9), k+- U(0.5, 2),
    k+ = k- (PCG) for even instances, PGMRES otherwise; 8 bumps; u0 = 0;
    mixed precision, tol 1e-8), `steps` CN steps each, through the batched
    executor: one lane (problems one after the other on one stream) against
    the autotuned lane count and launch mode (direct launches or launch
    graphs of the Krylov iteration chunks)."""
    import torch
    import workloads
    from paper_2511_21198_amd.batch import Batch
    ws = workloads.config_batched()
    probs = [dict(dim=w.dim, n=w.n, delta=w.delta, kplus=w.kplus, kminus=w.kminus, M=w.M, T=w.T,
                  solver=w.solver, precision="mixed", inner_tol=1e-4, tol=w.tol, x0="prev")
             for w in ws]
    Fs = [torch.from_numpy(w.F).cuda() for w in ws]
    u0 = [torch.zeros_like(F) for F in Fs]
    unknowns = sum(int(np.prod(w.n)) for w in ws)
    b = Batch(probs, streams=streams)
    out = {"workload": f"{len(ws)} instances (32 2D n in {{127,255,511,1023}}^2, 32 3D n in "
                       f"{{63,95,127}}^3, half PCG / half PGMRES), {steps} CN steps each, mixed "
                       "precision, tol 1e-8", "unknowns": unknowns, "streams": streams}

    def run(label):
        u = [x.clone() for x in u0]
        its = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            u, st = b.cn_step(u, Fs)
            its.append(sum(x["iters"] for x in st))
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        out[label] = {"lanes": b.lanes, "instance_steps_per_s": round(len(ws) * steps / t, 1),
                      "unknown_steps_per_s": float(f"{unknowns * steps / t:.4g}"),
                      "ms_per_batch_step": round(1e3 * t / steps, 2),
                      "total_iters_per_step": its}
        log(f"batched {label}: {out[label]}")
        return u

    b.set_lanes(1)
    run("one_lane")
    lanes, ms = b.autotune(u0, Fs)
    out["autotune_ms"] = {f"lanes={l},graphs={int(g)}": round(v, 2) for (l, g), v in ms.items()}
    out["autotuned_config"] = {"lanes": lanes, "graphs": b.graphs}
    # engines (tile shapes) the autotuner chose: how many problems run each
    # (pass, precision, length) on each engine
    from collections import Counter
    chosen = Counter()
    for i in range(len(ws)):
        for item in b.engines(i).split(","):
            chosen[item] += 1
    out["autotuned_engines"] = dict(sorted(chosen.items()))
    run("autotuned")
    out["speedup_vs_one_lane"] = round(out["autotuned"]["instance_steps_per_s"] /
                                       out["one_lane"]["instance_steps_per_s"], 3)
    return out


def two_sided(w, F, u0, steps, warmup, tol):
    """GMRES(20) on the two-sided system P^{-1/2} A P^{-1/2} v = P^{-1/2} b
    (the system Theorem 3.2 bounds) on the headline workload and tolerance,
    float64 and mixed precision, with the Theorem 3.2 rate omega of the
    workload; steps 2..steps+1 timed (median of 3 passes)."""
    import math
    from paper_2511_21198_amd.solver import Problem
    common = dict(dim=3, n=w.n, delta=w.delta, kplus=w.kplus, kminus=w.kminus, M=w.M, T=w.T,
                  solver="gmres2", restart=20, tol=tol, x0="prev")
    vs = 1.5 * max(math.tan(w.delta[i] * math.pi / 2) * abs(w.kplus[i] - w.kminus[i])
                   / (w.kplus[i] + w.kminus[i]) for i in range(3))
    out = {"solver": "GMRES(20) on P^{-1/2} A P^{-1/2}, two half-preconditioner applications "
                     "per iteration", "tol": tol, "varsigma": round(vs, 4),
           "omega": round(math.sqrt((2 + 4 * vs ** 2) / (3 + 4 * vs ** 2)), 4)}
    for name, kw in (("fp64", dict(precision="fp64")),
                     ("mixed", dict(precision="mixed", inner_tol=1e-3, max_outer=8))):
        p = Problem(**common, **kw)
        p.autotune()
        r = repeat_timing(p, u0, F, w.M, steps, warmup, 3)
        out[name] = {"steps_per_s": round(r["steps_per_s"], 3), "iters": r["iters"],
                     "outer": r["outer"]}
        del p
    return out


def comparators(w, F, u0):
    """The comparator preconditioners of Section 4 on the headline workload
    (float64 left GMRES(20) from u^{m-1}): CN steps/s and iterations, 2 timed
    steps after 1, against the sine-transform preconditioner; and one
    application of P^{-1} (100 calls, library hipEvents per pass)."""
    import torch
    from paper_2511_21198_amd.solver import Problem
    common = dict(dim=3, n=w.n, delta=w.delta, kplus=w.kplus, kminus=w.kminus, M=w.M, T=w.T,
                  solver="gmres", restart=20, tol=w.tol, x0="prev", precision="fp64")
    out = {"solver": "float64 left GMRES(20), x0 = u^{m-1}, tol 1e-8; steps 2 and 3 timed"}
    r = torch.from_numpy(w.F).cuda()
    for kind in ("tau", "tchan", "strang", "none"):
        log(f"comparator {kind} ...")
        p = Problem(**common, precond=kind, maxit=4000)
        rt = repeat_timing(p, u0, F, w.M, 2, 0, 1)
        e = {"steps_per_s": round(rt["steps_per_s"], 3), "iters": rt["iters"]}
        z = torch.empty_like(r)
        for _ in range(3):
            p.apply_Pinv(r, z)
        torch.cuda.synchronize()
        p.profile(True)
        t0 = time.perf_counter()
        for _ in range(100):
            p.apply_Pinv(r, z)
        torch.cuda.synchronize()
        e["apply_Pinv_ms"] = round((time.perf_counter() - t0) * 10.0, 4)
        prof = p.profile_read()
        p.profile(False)
        e["passes"] = {k: {"avg_ms": round(v["avg_ms"], 4), "gbps": round(v["gbps"], 1)}
                       for k, v in prof.items() if v["launches"]}
        out[kind] = e
        del p
    return out


def secondary_symmetric(a):
    """3D symmetric 127^3, (0.3, 0.5, 0.7), k = 1, 8 bumps, tol 1e-10: float64
    PCG vs float32-inner / float64-outer PCG, steps 2..9 timed (median of 3
    passes); errors of u^9 against a tol-1e-13 float64 run."""
    import torch
    import workloads
    from paper_2511_21198_amd.solver import Problem
    w = workloads.config_3d_symmetric(seed=0, n=127, M=32)
    F = torch.from_numpy(w.F).cuda()
    u0 = torch.zeros_like(F)
    common = dict(dim=3, n=w.n, delta=w.delta, kplus=w.kplus, kminus=w.kminus, M=w.M, T=w.T,
                  solver="pcg", tol=w.tol, x0="prev")
    out = {"workload": "3D symmetric 127^3, (alpha,beta,gamma)=(0.3,0.5,0.7), k=1, 32 CN steps "
                       "to T=1, 8 seeded bumps, u0=0, PCG, tol 1e-10"}
    us = {}
    for name, kw in (("fp64", dict(precision="fp64")),
                     ("mixed", dict(precision="mixed", inner_tol=1e-5))):
        p = Problem(**common, **kw)
        engines = p.autotune()
        r = repeat_timing(p, u0, F, w.M, 8, 2, 3)
        us[name] = final_state(p, u0, F, 9)
        out[name] = {"steps_per_s": round(r["steps_per_s"], 2), "iqr": r["iqr"], "iters": r["iters"],
                     "outer": r["outer"], "engines": engines}
        del p
    pref = Problem(**{**common, "tol": 1e-13}, precision="fp64")
    uref = final_state(pref, u0, F, 9)
    for name in us:
        out[name]["rel_err_vs_tight_fp64"] = float(torch.linalg.vector_norm(us[name] - uref)
                                                   / torch.linalg.vector_norm(uref))
    out["speedup"] = round(out["mixed"]["steps_per_s"] / out["fp64"]["steps_per_s"], 3)
    return out


LINE_PASSES = ("toep_", "dst_", "dsts_")


def kernel_table(prof, peak):
    """Per kernel kind of a profiled pass: launches, average hipEvent
    duration, algorithmic bytes per launch and GB/s, and the fraction of the
    datasheet and of the measured HBM peak."""
    out = {}
    for k, v in sorted(prof.items(), key=lambda kv: -kv[1]["total_ms"]):
        per = v["bytes"] / max(v["launches"], 1)
        out[k] = {"launches": v["launches"], "avg_ms": round(v["avg_ms"], 5),
                  "total_ms": round(v["total_ms"], 3), "bytes_per_launch": per,
                  "gbps": round(v["gbps"], 1), "frac_datasheet": round(v["gbps"] / HBM_PEAK_GBPS, 3),
                  "frac_measured": round(v["gbps"] / peak, 3) if peak else None}
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=15,
                    help="timed CN steps per repeat, taken from steps 2..16 of the workload "
                         "(a pass restarts from u0 with step 1 untimed)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--repeats", type=int, default=5)
    ap.add_argument("--n", type=int, default=255)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle timing")
    ap.add_argument("--only", choices=["mixed", "fp64", "both"], default="both")
    ap.add_argument("--inner-tol", type=float, default=None,
                    help="mixed-precision inner tolerance (default: the headline setting)")
    ap.add_argument("--dst-mfma", action="store_true",
                    help="mixed solver: float32 DST-I as bf16 matrix-core products (the "
                         "measured alternative to the FFT passes)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the built-in line-pass engines (no fsd_autotune at setup), e.g. "
                         "for a profiled run whose per-kernel figures should not include the "
                         "autotuner's timing launches")
    ap.add_argument("--no-warm", action="store_true",
                    help="skip the mixed solver run from the extrapolated warm start")
    ap.add_argument("--no-ref", action="store_true",
                    help="skip the tight float64 reference run used for the error figures")
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the tol-1e-8 figures, two-sided GMRES, comparators, operators "
                         "and the 127^3 symmetric PCG comparison")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned warm start workload (255^3, 200 steps)")
    ap.add_argument("--only-learned", action="store_true",
                    help="run only the learned warm start workload and print its JSON")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the 64-instance batched workload")
    ap.add_argument("--only-batched", action="store_true",
                    help="run only the batched workload and print its JSON")
    ap.add_argument("--only-comparators", action="store_true",
                    help="run only the comparator preconditioners and print their JSON")
    ap.add_argument("--only-operators", action="store_true",
                    help="run only the operator timings and print their JSON")
    a = ap.parse_args(argv)
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print(json.dumps({"error": "this solver runs on one GPU; multi-GPU runs are not "
                                   "supported (use --gpus 1)", "n_gpus": a.gpus}))
        return 2

    import torch
    import workloads
    from paper_2511_21198_amd.solver import Problem

    if a.only_learned:
        print(json.dumps(learned_workload(a)), flush=True)
        return 0
    if a.only_batched:
        print(json.dumps(batched_workload(a)), flush=True)
        return 0
    w = workloads.config_3d_nonsymmetric(seed=0, n=a.n, M=16)
    if a.only_comparators:
        F = torch.from_numpy(w.F).cuda()
        print(json.dumps(comparators(w, F, torch.zeros_like(F))), flush=True)
        return 0
    log("hbm peak (stream copy) ...")
    peak = hbm_peak()
    if a.only_operators:
        print(json.dumps({"hbm_peak": peak, "operators": operator_bench(w, peak["gbps"])}),
              flush=True)
        return 0
    S = dict(workloads.HEADLINE_SOLVER)
    tol = S.pop("tol")
    inner_tol = S.pop("inner_tol") if a.inner_tol is None else a.inner_tol
    S.pop("inner_tol", None)
    max_outer = S.pop("max_outer")
    dev = torch.device("cuda:0")
    F = torch.from_numpy(w.F).to(dev)
    u0 = torch.zeros_like(F)
    common = dict(dim=3, n=w.n, delta=w.delta, kplus=w.kplus, kminus=w.kminus, M=w.M, T=w.T,
                  solver="gmres", **S)
    mixed_kw = dict(precision="mixed", inner_tol=inner_tol, max_outer=max_outer)

    def leg(name, t, kw, profile=False, repeats=None, x0=None):
        log(f"{name} (tol {t:g}) ...")
        c = dict(common)
        if x0:
            c["x0"] = x0
        p = Problem(**c, tol=t, **kw)
        # tile shapes per pass, chosen at setup (untimed)
        engines = p.engines() if a.no_autotune else p.autotune()
        r = repeat_timing(p, u0, F, w.M, a.steps, a.warmup, repeats or a.repeats, profile)
        r["engines"] = engines
        r["u_final"] = final_state(p, u0, F, w.M) if not a.no_ref else None
        del p
        log(f"  {r['steps_per_s']:.3f} CN steps/s (IQR {r['iqr'][0]:.3f}..{r['iqr'][1]:.3f})")
        return r

    res = {}
    if a.only in ("fp64", "both"):
        res["fp64"] = leg("fp64 solver", tol, dict(precision="fp64"), profile=True)
    if a.only in ("mixed", "both"):
        res["mixed"] = leg("mixed solver", tol, dict(mixed_kw, dst_mfma=a.dst_mfma), profile=True)
        if not a.no_warm:
            res["mixed_extrap"] = leg("mixed solver, extrapolated warm start", tol, mixed_kw,
                                      x0="extrap", repeats=3)
    if not a.no_secondary:
        res["fp64_tol_1e-8"] = leg("fp64 solver", 1e-8, dict(precision="fp64"), repeats=3)
        res["mixed_tol_1e-8"] = leg("mixed solver", 1e-8, mixed_kw, repeats=3)
    errs = {}
    if not a.no_ref:
        log("tight float64 reference (tol 1e-12, untimed) ...")
        pref = Problem(**{**common, "tol": 1e-12}, precision="fp64")
        uref = final_state(pref, u0, F, w.M)
        del pref
        for k, r in res.items():
            errs[k] = errors(r["u_final"], uref)
    head = "mixed" if "mixed" in res else "fp64"
    H = res[head]
    value = H["steps_per_s"]
    ms_per_step = 1e3 / value
    ktab = kernel_table(H["prof"], peak["gbps"])
    lp = [k for k in ktab if k.startswith(LINE_PASSES)]
    dom = lp[0] if lp else next(iter(ktab))
    d = ktab[dom]
    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "CN steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if head == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": f"3D non-symmetric {a.n}^3, (alpha,beta,gamma)=(0.4,0.6,0.8), "
                               "k+=(1.0,0.8,1.2), k-=(0.5,1.0,0.3), 16 CN steps to T=1, "
                               "8 seeded Gaussian bumps, u0=0, PGMRES(20) + sine-transform "
                               f"preconditioner from u^(m-1), tol {tol:g}; timed steps are taken "
                               "from steps 2..16 only (a pass restarts from u0, step 1 untimed); "
                               f"value = median over {a.repeats} passes; line-pass engines from "
                               "the library's autotuner at setup (untimed)",
                   "solver": f"{head}: " + (f"float32 inner GMRES (inner tol {inner_tol:g}) in "
                                             "float64 defect correction, float64 outer test"
                                             if head == "mixed" else "float64 GMRES"),
                   "tol": tol, "n": a.n, "unknowns": a.n ** 3},
        "iqr_steps_per_s": [round(v, 3) for v in H["iqr"]],
        "engines": H.get("engines"),
        "per_repeat_steps_per_s": H["per_repeat"],
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": d["gbps"], "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": d["frac_datasheet"],
                     "traffic": counter_traffic(dom) if a.n == 255 else None,
                     "avg_launch_ms": d["avg_ms"], "algorithmic_bytes_per_launch": d["bytes_per_launch"],
                     "measured_peak_gbps": peak["gbps"], "frac_measured_peak": d["frac_measured"],
                     "note": "the line pass (Toeplitz matvec or DST preconditioner pass) with the "
                             "largest total time in the timed mixed-precision steps; every kernel "
                             "kind is in roofline_kernels"},
        "hbm_peak": peak,
    }
    if "fp64" in res:
        out["fp64_steps_per_s"] = round(res["fp64"]["steps_per_s"], 3)
        out["fp64_iqr_steps_per_s"] = [round(v, 3) for v in res["fp64"]["iqr"]]
        out["iters_fp64"] = res["fp64"]["iters"]
    if "mixed" in res:
        out["iters_mixed_inner"] = res["mixed"]["iters"]
        out["outer_mixed"] = res["mixed"]["outer"]
    if "mixed" in res and "fp64" in res:
        out["speedup_vs_fp64"] = round(value / res["fp64"]["steps_per_s"], 3)
    if errs:
        out["rel_err_vs_tight_fp64"] = errs
        if "mixed" in res and "fp64" in res:
            out["rel_diff_mixed_vs_fp64"] = errors(res["mixed"]["u_final"], res["fp64"]["u_final"])
    if "mixed_extrap" in res:
        wx = res["mixed_extrap"]
        out["mixed_extrap"] = {"steps_per_s": round(wx["steps_per_s"], 3), "iters_inner": wx["iters"],
                               "outer": wx["outer"]}
        if "fp64" in res:
            out["mixed_extrap"]["speedup_vs_fp64_prev"] = round(
                wx["steps_per_s"] / res["fp64"]["steps_per_s"], 3)
    if "mixed_tol_1e-8" in res:
        m8, f8 = res["mixed_tol_1e-8"], res["fp64_tol_1e-8"]
        out["tol_1e-8"] = {"note": "both solvers at the configuration's literal tol 1e-8: u^M "
                                   "misses the 1e-8 error target (rel_err_vs_tight_fp64)",
                           "mixed_steps_per_s": round(m8["steps_per_s"], 3),
                           "fp64_steps_per_s": round(f8["steps_per_s"], 3),
                           "speedup": round(m8["steps_per_s"] / f8["steps_per_s"], 3),
                           "iters_mixed_inner": m8["iters"], "iters_fp64": f8["iters"]}
    out["roofline_kernels"] = {"mixed": ktab}
    if "fp64" in res:
        out["roofline_kernels"]["fp64"] = kernel_table(res["fp64"]["prof"], peak["gbps"])
    if not a.no_secondary:
        log("two-sided GMRES ...")
        out["two_sided"] = two_sided(w, F, u0, min(a.steps, 8), a.warmup, tol)
        out["comparators"] = comparators(w, F, u0)
        out["operators"] = operator_bench(w, peak["gbps"])
        out["secondary"] = secondary_symmetric(a)
    if not a.no_learned:
        out["learned"] = learned_workload(a)
    if not a.no_batched:
        out["batched"] = batched_workload(a)
    if not a.no_cpu and "fp64" in res:
        log("cpu baseline (oracle, per-iteration sample) ...")
        wc = workloads.config_3d_nonsymmetric(seed=0, n=a.n, M=16)
        its = res["fp64"]["iters"][:15]
        out["cpu_baseline"] = cpu_baseline(wc, float(np.mean(its)))
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
