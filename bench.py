"""Benchmark of the CIA right-hand side inside RK4 on one MI355X.

Workload: Kuramoto on the N = 1e6 planted power-law community graph
(sizes ~ s^-2 on [100, 5000], p_in 0.95, mean inter degree 5, Cauchy(0, 0.5)
frequencies, K = 3, RK4 dt 0.01), synthetic and seeded.

One bench step = one RK4 step = four RHS evaluations (E1 + E2 + combine),
fused with the stage updates, plus the FP64 order parameter r(t).
value = N * 4 * steps / seconds (RHS node-updates per second).  The direct
O(|E|) method is timed the same way on the same data; the FP64 CPU oracle
is timed on a bounded sample.

Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3   # published FP32 vector peak (256 CUs at 2.4 GHz)
FLOPS_PER_PAIR = 22        # flock pair evaluation, see bench_flock


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def profiled_traffic(workload, summary="phase_stage_kernel_kuramoto_n1e6.md"):
    """HBM bytes per stage-kernel launch from a committed rocprofv3 counter
    summary, valid only for the workload it was measured on and while the
    kernel sources are the ones profiled."""
    import hashlib
    prof = os.path.join(ROOT, "profiles", summary)
    srcs = [os.path.join(ROOT, "paper_2203_16657_amd", "csrc", f) for f in ("cia_phase.hip", "plan.h", "fastmath.h", "wave.h")]
    try:
        text = open(prof).read()
        h = hashlib.sha256(b"".join(open(f, "rb").read() for f in srcs)).hexdigest()
    except OSError:
        return None
    keys = ("traffic_bytes_per_launch: ", "source_sha256: ", "workload: ")
    vals = dict(line.split(": ", 1) for line in text.splitlines() if line.startswith(keys))
    if vals.get("source_sha256", "").strip() != h or vals.get("workload", "").strip() != workload:
        return None
    return float(vals["traffic_bytes_per_launch"])


def time_integrate(plan, torch, theta0, dt, steps, warmup, with_r=True, timing_every=0, reps=5):
    """Warm up with `warmup` steps, then time `reps` calls of exactly `steps`
    steps, each from the same initial state and bracketed by HIP events on
    the launch stream after a device synchronisation.  Returns the median
    call's milliseconds, the library's kernel timing over all timed calls,
    the last call's r(t) and every call's milliseconds."""
    import numpy as np
    tdt = torch.float64 if plan.precision == 1 else torch.float32
    th0 = torch.as_tensor(theta0, dtype=tdt, device="cuda")
    th = th0.clone()
    # the warm-up passes the timed calls' trace, so the library sizes its
    # device trace buffer before the timed region
    count = len(getattr(plan, "offsets", (0, 0))) - 1   # instances of a batched plan
    r = np.zeros(count * (steps + 1)) if with_r else None
    if warmup:
        plan.integrate(th, dt, warmup, r)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    # kernel durations: HIP events around one stage launch in `timing_every`
    # (17: coprime with the 4 stages, so every stage is sampled), on the
    # launch stream, inside the timed region
    plan.set_timing(timing_every)
    plan.timing(reset=True)
    times = []
    for _ in range(reps):
        th.copy_(th0)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        plan.integrate(th, dt, steps, r, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    t = plan.timing(reset=True)
    return float(np.median(times)), t, r, times


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="large", choices=["large", "small", "flock", "ensemble", "triadic", "structured", "poly", "general"],
                    help="large: the N = 1e6 Kuramoto bench line; flock, ensemble and triadic: the "
                         "Cucker-Smale, batched-ensemble and higher-order workloads (measurement modes, "
                         "not the bench line)")
    ap.add_argument("--triadic-n", type=int, default=6000, help="triadic: network size (sizes U[200, 2000])")
    ap.add_argument("--train-iters", type=int, default=3000, help="flock: optimiser steps of the basis")
    ap.add_argument("--ensemble-nmax", type=float, default=2e5, help="ensemble: largest instance size")
    ap.add_argument("--ensemble-oracle-share", type=float, default=0.25,
                    help="ensemble: share of every instance's rows the CPU oracle evaluates")
    ap.add_argument("--no-sequential", action="store_true",
                    help="ensemble: skip the 256 single-network plans")
    ap.add_argument("--reps", type=int, default=5,
                    help="timed calls of --steps steps each; the median call is reported")
    ap.add_argument("--direct-steps", type=int, default=100,
                    help="RK4 steps timed for the direct method")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-timing", action="store_true", help="no per-kernel events")
    ap.add_argument("--timing-every", type=int, default=17,
                    help="HIP events around one stage launch in this many (1 = every launch)")
    ap.add_argument("--autotune", action="store_true",
                    help="let the library's autotuner pick the unit and block size before timing")
    ap.add_argument("--unit-work", type=int, default=0)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 256 MiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(communities would shard across GPUs with one halo exchange of z per RK stage)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2203_16657_amd as cia
    import workloads as W

    if not os.path.exists(cia.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    cia.load()
    assert torch.cuda.is_available(), "bench.py needs a GPU"

    if args.calibrate_copy:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE per dispatch
        # calibrate the byte counters of the stage kernel
        src = torch.empty(64 << 20, dtype=torch.float32, device="cuda").uniform_()
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 5 x %d bytes" % (src.numel() * 4))
        del src, dst

    if args.workload == "flock":
        return bench_flock(args, cia, W, torch, np)
    if args.workload == "ensemble":
        return bench_ensemble(args, cia, W, torch, np)
    if args.workload == "general":
        return bench_general(args, cia, W, torch, np)
    if args.workload == "poly":
        return bench_poly(args, cia, W, torch, np)
    if args.workload == "structured":
        return bench_structured(args, cia, W, torch, np)
    if args.workload == "triadic":
        return bench_triadic(args, cia, W, torch, np)

    t0 = time.time()
    P = W.kuramoto_large() if args.workload == "large" else W.kuramoto_small()
    g = P.graph
    log("workload %s: n=%d nnz=%d communities=%d (%.1fs)" % (P.name, g.n, g.nnz, g.ncomm, time.time() - t0))

    every = 0 if args.no_timing else max(1, args.timing_every)
    # the N = 1000 network is run in FP64, as specified for it
    prec = cia.CIA_F64 if args.workload == "small" else cia.CIA_F32
    t0 = time.time()
    plan = cia.Plan.phase(g.n, g.row_ptr, g.col, g.labels, P.omega, K=P.K, precision=prec,
                          unit_work=args.unit_work, block=args.block)
    tune = None
    if args.autotune and not args.unit_work and not args.block:
        rep = plan.autotune()
        tune = {"unit_work": rep.unit_work, "block": rep.block, "candidates": rep.candidates,
                "best_us": round(rep.best_us, 2), "default_us": round(rep.default_us, 2)}
        log("autotune: unit_work %d block %d (%.2f us vs %.2f us default, %d candidates)" % (
            rep.unit_work, rep.block, rep.best_us, rep.default_us, rep.candidates))
    info = plan.info()
    log("cia plan: units=%d ncomm=%d nnz_neg=%d nnz_pos=%d unassigned=%d merged_slices=%d bytes/stage=%.3e (%.1fs)" % (
        info.nunits, info.ncomm, info.nnz_neg, info.nnz_pos, info.n_unassigned, info.merged_slices,
        info.bytes_per_stage, time.time() - t0))
    ms, tim, r, calls = time_integrate(plan, torch, P.theta0, P.dt, args.steps, args.warmup, timing_every=every,
                                       reps=args.reps)
    n = g.n
    rhs_per_step = 4
    value = n * rhs_per_step * args.steps / (ms / 1e3)
    log("cia: %.3f ms/step, %.3e RHS node-updates/s" % (ms / args.steps, value))
    stage_avg_ms = tim.stage_ms / max(tim.stage_launches, 1) if tim.stage_launches else None
    roof = None
    if stage_avg_ms:
        achieved = info.bytes_per_stage / (stage_avg_ms / 1e3) / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": profiled_traffic(P.name),
                "kernel": "phase_stage_kernel", "avg_launch_us": round(stage_avg_ms * 1e3, 2),
                "algorithmic_bytes_per_launch": info.bytes_per_stage, "timed_launches": tim.stage_launches}
        log("stage kernel avg %.2f us, %.1f GB/s algorithmic (%.1f%% of 8 TB/s)" % (
            stage_avg_ms * 1e3, achieved, 100 * achieved / HBM_PEAK_GBS))
    plan.close()

    # direct method, same data layout and stepper
    t0 = time.time()
    dplan = cia.Plan.phase(g.n, g.row_ptr, g.col, g.labels, P.omega, K=P.K, method=cia.CIA_METHOD_DIRECT,
                           precision=prec)
    dinfo = dplan.info()
    log("direct plan: units=%d nnz=%d (%.1fs)" % (dinfo.nunits, dinfo.nnz_pos, time.time() - t0))
    dsteps = min(args.direct_steps, args.steps)
    dms, dtim, _, dcalls = time_integrate(dplan, torch, P.theta0, P.dt, dsteps, min(args.warmup, 5),
                                          timing_every=0 if args.no_timing else 1, reps=args.reps)
    dvalue = n * rhs_per_step * dsteps / (dms / 1e3)
    d_stage_ms = dtim.stage_ms / max(dtim.stage_launches, 1) if dtim.stage_launches else None
    log("direct: %.3f ms/step, %.3e RHS node-updates/s" % (dms / dsteps, dvalue))
    direct = {"value": dvalue, "ms_per_step": dms / dsteps, "steps": dsteps,
              "ms_per_call": [round(x, 4) for x in dcalls]}
    if d_stage_ms:
        dach = dinfo.bytes_per_stage / (d_stage_ms / 1e3) / 1e9
        direct.update(avg_launch_us=round(d_stage_ms * 1e3, 2), achieved_gbs=round(dach, 1),
                      frac=round(dach / HBM_PEAK_GBS, 4))
    dplan.close()

    cpu = None
    if not args.no_cpu:
        import oracle
        th = P.theta0.astype(np.float64)
        csteps = 2 if args.workload == "large" else 20
        t0 = time.time()
        oracle.phase_integrate(g.n, g.row_ptr, g.col, P.omega, P.K, [0, 1], [0, 0], th, P.dt, csteps,
                               trace=False)
        ct = time.time() - t0
        cpu = {"value": n * rhs_per_step * csteps / ct, "unit": "RHS node-updates/s",
               "cores": oracle.num_threads(), "kind": "oracle",
               "sample": "%d FP64 RK4 step(s) (%d RHS evaluations) of the full workload, %.1f s" % (
                   csteps, rhs_per_step * csteps, ct)}
        log("cpu oracle: %.3e RHS node-updates/s on %d threads" % (cpu["value"], cpu["cores"]))
        # the same oracle on one thread, over a sample of rows of one RHS
        nt = oracle.num_threads()
        oracle.set_num_threads(1)
        try:
            rows = np.sort(np.random.default_rng(0).choice(n, min(n, 50000), replace=False)).astype(np.int64)
            t0 = time.time()
            oracle.phase_rhs(g.n, g.row_ptr, g.col, P.omega, P.K, [0, 1], [0, 0], th, rows=rows)
            c1 = time.time() - t0
        finally:
            oracle.set_num_threads(nt)
        cpu["single_thread"] = {"value": len(rows) / c1, "unit": "RHS node-updates/s", "cores": 1,
                                "sample": "%d sampled rows of one FP64 right-hand side, %.1f s" % (len(rows), c1)}
        log("cpu oracle, one thread: %.3e RHS node-updates/s" % cpu["single_thread"]["value"])

    res = {
        "metric": "RHS node-updates/s, CIA vs direct, 1 MI355X, N=1e6, <=1e-5 rel err vs FP64",
        "value": value,
        "unit": "RHS node-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "timed_calls": {"count": len(calls), "statistic": "median",
                        "ms_per_call": [round(x, 4) for x in calls]},
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == cia.CIA_F64 else "f32",
        "data": "synthetic",
        "config": {"workload": P.name, "n": n, "communities": info.ncomm, "nnz_graph": info.nnz_graph,
                   "nnz_neg": info.nnz_neg, "nnz_pos": info.nnz_pos, "stepper": "rk4", "dt": P.dt,
                   "rhs_per_step": rhs_per_step, "parallelism": "single-gpu", "units": info.nunits,
                   "autotune": tune},
        "direct": direct,
        "speedup_vs_direct": value / dvalue,
        "roofline": roof,
        "cpu_baseline": cpu,
        "r_final": float(r[-1]) if r is not None else None,
    }
    print(json.dumps(res), flush=True)


def oracle_baseline(args, fn, n, what, target_s=8.0):
    """The oracle timed on the host on a bounded sample: fn(rows) evaluates
    the FP64 right-hand side of the sampled rows of the workload; the sample
    grows until it takes about target_s / 4 .. target_s seconds."""
    if args.no_cpu:
        return None
    import numpy as np
    import oracle
    rng = np.random.default_rng(0)
    k = 64
    while True:
        rows = np.sort(rng.choice(n, min(k, n), replace=False)).astype(np.int64)
        t0 = time.time()
        fn(rows)
        ct = time.time() - t0
        if ct >= target_s / 4 or k >= n:
            break
        k = int(min(n, k * max(2.0, target_s / max(ct, 1e-3))))
    out = {"value": len(rows) / ct, "unit": "RHS node-updates/s", "cores": oracle.num_threads(), "kind": "oracle",
           "sample": "%s: %d sampled rows of one FP64 right-hand side, %.1f s" % (what, len(rows), ct)}
    log("cpu oracle (%s): %.3e RHS node-updates/s on %d threads" % (what, out["value"], out["cores"]))
    return out


def timed(torch, fn):
    s = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(s)
    fn(s)
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def bench_flock(args, cia, W, torch, np):
    """Cucker-Smale on 400 communities of 500 (N = 2e5): the learned rank-32
    basis (trained on the GPU, judged per community), the exact community
    path, the Fourier basis and the direct method; single-RHS errors against
    the FP64 oracle on sampled rows and RK4 throughput."""
    import oracle
    F = W.flock()
    g = F.graph
    n = g.n
    log("flock workload: n=%d nnz=%d communities=%d" % (n, g.nnz, g.ncomm))
    st = torch.as_tensor(np.concatenate([F.x0, F.v0]).astype(np.float32), device="cuda").contiguous()
    s64 = st.cpu().numpy().astype(np.float64)
    rows = np.random.default_rng(1).choice(n, 2000, replace=False)
    _, vref = oracle.cs_rhs(n, g.row_ptr, g.col, F.K, F.sigma, F.beta, s64[:3], s64[3:], rows=rows)

    def rhs_err(plan):
        out = torch.empty_like(st)
        plan.rhs(st, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy().astype(np.float64)[3:, rows]
        return float(np.abs(got - vref).max() / np.abs(vref).max())

    def make(basis, **kw):
        return cia.Plan.flock(n, g.row_ptr, g.col, g.labels, K=F.K, sigma=F.sigma, beta=F.beta, basis=basis, **kw)

    steps = min(args.steps, 50)
    res = {}
    # learned basis: train, then time steps with the judge
    learned = make(cia.CIA_BASIS_LEARNED, rank=32)
    lt = np.zeros(args.train_iters)
    train_ms = timed(torch, lambda s: learned.basis_train(st, args.train_iters, seed=11, loss_trace=lt, stream=s))
    params, lo, hi = learned.basis_get_params(cia.cia_basis_param_count(32))
    free = make(cia.CIA_BASIS_LEARNED, rank=32, flags=cia.CIA_FLAG_NO_JUDGE)
    free.basis_set_params(params, lo, hi)
    fourier = make(cia.CIA_BASIS_FOURIER, p=1, flags=cia.CIA_FLAG_NO_JUDGE)
    exact = make(cia.CIA_BASIS_EXACT)
    direct = make(cia.CIA_BASIS_EXACT, method=cia.CIA_METHOD_DIRECT)
    errs = {"learned_no_judge": rhs_err(free), "learned_judged": rhs_err(learned), "fourier_p1": rhs_err(fourier),
            "exact": rhs_err(exact), "direct": rhs_err(direct)}
    fallbacks = learned.info().judge_fallbacks
    for name, plan in (("learned_judged", learned), ("learned_no_judge", free), ("exact", exact),
                       ("direct", direct)):
        y = st.clone()
        plan.integrate(y, F.dt, 2)
        y = st.clone()
        plan.set_timing(17)
        plan.timing(reset=True)
        ms = timed(torch, lambda s: plan.integrate(y, F.dt, steps, stream=s))
        t = plan.timing(reset=True)
        res[name] = {"value": n * 4 * steps / (ms / 1e3), "ms_per_step": ms / steps,
                     "stage_us": round(1e3 * t.stage_ms / max(t.stage_launches, 1), 2),
                     "prep_us": round(1e3 * t.prep_ms / max(t.prep_launches, 1), 2)}
        log("%-17s %.3f ms/step, %.3e node-updates/s" % (name, ms / steps, res[name]["value"]))
    out = {
        "metric": "flock RHS node-updates/s (learned rank-32 basis, judged), 1 MI355X, N=2e5",
        "value": res["learned_judged"]["value"], "unit": "RHS node-updates/s", "n_gpus": 1, "steps": steps,
        "warmup": 2, "ms_per_step": res["learned_judged"]["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+bf16", "data": "synthetic",
        "config": {"workload": "flock_n200000", "n": n, "communities": g.ncomm, "rank": 32, "judge_tol": 1e-3,
                   "stepper": "rk4", "dt": F.dt},
        "methods": res, "rhs_rel_err": errs, "judge_fallbacks": fallbacks,
        "train": {"iters": args.train_iters, "ms": train_ms, "loss_first": float(lt[:10].mean()),
                  "loss_last": float(lt[-100:].mean())},
        "gain_vs_fourier": errs["fourier_p1"] / errs["learned_no_judge"],
    }
    # roofline of the line's dominant kernel, flock_stage_kernel.  A community
    # on the exact path evaluates w(|x_j - x_i|)(v_j - v_i) on all of its
    # lambda (lambda - 1) ordered pairs, and every row its S-neg and S-pos
    # entries: FLOPS_PER_PAIR FP32 operations each (3 differences, |d|^2 in 5,
    # s^2 + r^2, log2, scale, exp2, times K, 3 differences and 3 FMAs of the
    # velocity sum; a transcendental counts as one).  Those pair evaluations,
    # not the 4-byte index streams, bound the kernel.
    info = learned.info()
    sizes = np.bincount(g.labels[g.labels >= 0])
    fb_pairs = float((sizes * (sizes - 1)).sum()) * min(1.0, fallbacks / max(g.ncomm, 1))
    pairs = fb_pairs + float(info.nnz_neg + info.nnz_pos)
    st_us = res["learned_judged"]["stage_us"]
    if st_us > 0:
        tflops = pairs * FLOPS_PER_PAIR / (st_us * 1e-6) / 1e12
        gbs = info.bytes_per_stage / (st_us * 1e-6) / 1e9
        out["roofline"] = {"bound": "alu", "achieved": round(tflops, 2), "peak": FP32_PEAK_TFLOPS,
                           "unit": "TFLOP/s", "frac": round(tflops / FP32_PEAK_TFLOPS, 4), "traffic": None,
                           "kernel": "flock_stage_kernel", "avg_launch_us": st_us,
                           "pairs_per_launch": pairs, "flops_per_pair": FLOPS_PER_PAIR,
                           "algorithmic_bytes_per_launch": info.bytes_per_stage,
                           "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}
        log("flock stage kernel %.1f us: %.2f TFLOP/s (%.1f%% of FP32 vector peak), %.1f GB/s algorithmic" % (
            st_us, tflops, 100 * tflops / FP32_PEAK_TFLOPS, gbs))
    else:
        out["roofline"] = None
    out["cpu_baseline"] = oracle_baseline(args, lambda r_: oracle.cs_rhs(
        n, g.row_ptr, g.col, F.K, F.sigma, F.beta, s64[:3], s64[3:], rows=r_), n, "flock_n200000 exact sum")
    print(json.dumps(out), flush=True)


def bench_ensemble(args, cia, W, torch, np):
    """The 256-instance ensemble: N log-uniform in [1e3, --ensemble-nmax]
    (default 2e5, about 9.6e6 nodes in total), 4..500 communities, p_in in
    [0.7, 0.95], p_out log-uniform in [1e-4, 1e-2], K swept over [0, 6].

    Instances are generated one at a time and added to an incremental batch
    build, so host memory holds one instance's adjacency at a time.  While an
    instance's graph is in hand, the FP64 oracle evaluates a sample of its rows
    (the cpu_baseline, and the reference of a sampled-row parity check of the
    batched plan) and, unless --no-sequential, a single-network plan of it is
    built, warmed up, timed over the same steps with HIP events and destroyed;
    the sum of those 256 timings is the sequential comparison."""
    import oracle
    count = 256
    steps = max(1, min(args.steps, 100))
    share = args.ensemble_oracle_share
    bb = cia.BatchBuilder(flags=cia.CIA_FLAG_AUTOTUNE)
    rng = np.random.default_rng(23)
    th_parts = []
    seq_ms, cpu_s, cpu_rows, nnz = 0.0, 0.0, 0, 0
    t0 = time.time()
    for b in range(count):
        P = W.ensemble_member(b, n_hi=args.ensemble_nmax, count=count)
        g = P.graph
        nnz += g.nnz
        th32 = P.theta0.astype(np.float32)
        bb.add(g.n, g.row_ptr, g.col, g.labels, P.omega, P.K)
        if not args.no_cpu:
            rows = np.sort(rng.choice(g.n, max(1, int(round(g.n * share))), replace=False)).astype(np.int64)
            tc = time.time()
            oracle.phase_rhs(g.n, g.row_ptr, g.col, P.omega, P.K, [0, 1], [0, 0], th32.astype(np.float64),
                             rows=rows)
            cpu_s += time.time() - tc
            cpu_rows += len(rows)
        if not args.no_sequential:
            pl = cia.Plan.phase(g.n, g.row_ptr, g.col, g.labels, P.omega, K=P.K,
                                flags=cia.CIA_FLAG_NO_VALIDATE)
            t = torch.as_tensor(th32, device="cuda")
            rr = np.zeros(steps + 1)
            pl.integrate(t, 0.01, 2, rr[:3])
            t.copy_(torch.as_tensor(th32, device="cuda"))
            seq_ms += timed(torch, lambda st: pl.integrate(t, 0.01, steps, rr, stream=st))
            pl.close()
            del t
        th_parts.append(th32)
        del P, g
        if b % 32 == 31:
            log("ensemble: %d instances added, N %d, nnz %d (%.0f s)" % (b + 1, bb.n, nnz, time.time() - t0))
    tb = time.time()
    plan = bb.finish()
    info = plan.info()
    off = plan.offsets
    ntot = int(off[-1])
    log("ensemble plan: N %d nnz %d units %d nnz_neg %d nnz_pos %d merged_slices %d bytes/stage %.3e "
        "(finish %.0f s, all %.0f s)" % (ntot, info.nnz_graph, info.nunits, info.nnz_neg, info.nnz_pos,
                                         info.merged_slices, info.bytes_per_stage, time.time() - tb, time.time() - t0))
    th0 = np.concatenate(th_parts)
    del th_parts
    every = 0 if args.no_timing else max(1, args.timing_every)
    ms, tim, r, calls = time_integrate(plan, torch, th0, 0.01, steps, 2, timing_every=every, reps=args.reps)
    value = ntot * 4 * steps / (ms / 1e3)
    log("batched: %.3f ms/step, %.3e RHS node-updates/s" % (ms / steps, value))
    roof = None
    stage_avg_ms = tim.stage_ms / max(tim.stage_launches, 1) if tim.stage_launches else None
    if stage_avg_ms:
        achieved = info.bytes_per_stage / (stage_avg_ms / 1e3) / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": profiled_traffic("ensemble_256" if args.ensemble_nmax == 2e5 else "other",
                                            "ensemble_batched_256.md"),
                "kernel": "phase_stage_kernel",
                "avg_launch_us": round(stage_avg_ms * 1e3, 2),
                "algorithmic_bytes_per_launch": info.bytes_per_stage, "timed_launches": tim.stage_launches}
        log("ensemble stage kernel avg %.2f us, %.1f GB/s algorithmic (%.1f%% of 8 TB/s)" % (
            stage_avg_ms * 1e3, achieved, 100 * achieved / HBM_PEAK_GBS))
    res = {"batched": {"value": value, "ms_per_step": ms / steps, "units": info.nunits,
                       "ms_per_call": [round(x, 4) for x in calls]}}
    if not args.no_sequential:
        res["sequential"] = {"value": ntot * 4 * steps / (seq_ms / 1e3), "ms_per_step": seq_ms / steps,
                             "how": "sum over the 256 instances of one timed cia_integrate call each"}
        log("sequential: %.3f ms/step" % (seq_ms / steps))
    plan.close()
    out = {
        "metric": "ensemble RHS node-updates/s (256 instances, one batched plan), 1 MI355X",
        "value": value, "unit": "RHS node-updates/s", "n_gpus": 1, "steps": steps, "warmup": 2,
        "ms_per_step": ms / steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "ensemble_256", "n_total": ntot, "n_max": args.ensemble_nmax,
                   "nnz_graph": int(info.nnz_graph), "nnz_neg": int(info.nnz_neg), "nnz_pos": int(info.nnz_pos),
                   "stepper": "rk4", "dt": 0.01, "units": info.nunits},
        "methods": res,
        "speedup_vs_sequential": (res["batched"]["value"] / res["sequential"]["value"]
                                  if "sequential" in res else None),
        "roofline": roof,
        "cpu_baseline": None if args.no_cpu else {
            "value": cpu_rows / cpu_s, "unit": "RHS node-updates/s", "cores": oracle.num_threads(),
            "kind": "oracle", "sample": "%.1f%% of the rows of every instance (%d rows), one FP64 right-hand "
            "side, %.1f s" % (100 * share, cpu_rows, cpu_s)},
    }
    print(json.dumps(out), flush=True)


def bench_triadic(args, cia, W, torch, np):
    """Higher-order Kuramoto with the config-3 community sizes (U[200, 2000],
    pairwise p_in 0.9, intra triples with p = 0.9, 3 cross triples per node):
    CIA (stored missing pairs) against the direct method (present triples
    enumerated on the GPU), FP32, RK4."""
    T = W.triadic(seed=3, n=args.triadic_n)
    g = T.graph
    n = g.n
    log("triadic workload: n=%d communities=%d pairwise nnz=%d cross triples=%d" % (
        n, g.ncomm, g.nnz, len(T.cross_tri)))
    steps = min(args.steps, 20)
    res = {}
    for name, method in (("cia", cia.CIA_METHOD_CIA), ("direct", cia.CIA_METHOD_DIRECT)):
        t0 = time.time()
        plan = cia.Plan.triadic(n, g.row_ptr, g.col, g.labels, T.omega, K1=T.K1, K2=T.K2, tri_seed=T.tri_seed,
                                p_tri=T.p_tri, cross_tri=T.cross_tri, method=method)
        build_s = time.time() - t0
        info = plan.info()
        th = torch.as_tensor(T.theta0.astype(np.float32), device="cuda")
        plan.integrate(th, T.dt, 1)
        th = torch.as_tensor(T.theta0.astype(np.float32), device="cuda")
        plan.set_timing(1)
        plan.timing(reset=True)
        ms = timed(torch, lambda s: plan.integrate(th, T.dt, steps, stream=s))
        t = plan.timing(reset=True)
        res[name] = {"value": n * 4 * steps / (ms / 1e3), "ms_per_step": ms / steps,
                     "stage_us": round(1e3 * t.stage_ms / max(t.stage_launches, 1), 2),
                     "aux_us": round(1e3 * t.aux_ms / max(t.aux_launches, 1), 2),
                     "build_s": round(build_s, 2), "pair_entries": info.nnz_extra,
                     "bytes_per_stage": info.bytes_per_stage, "bytes_aux": info.bytes_aux}
        log("%-7s %.3f ms/step (build %.1f s, %d stored pairs)" % (name, ms / steps, build_s, info.nnz_extra))
        plan.close()
    out = {
        "metric": "triadic RHS node-updates/s (CIA), 1 MI355X, config-3 community sizes",
        "value": res["cia"]["value"], "unit": "RHS node-updates/s", "n_gpus": 1, "steps": steps, "warmup": 1,
        "ms_per_step": res["cia"]["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "triadic_n%d" % n, "n": n, "communities": g.ncomm, "stepper": "rk4", "dt": T.dt},
        "methods": res, "speedup_vs_direct": res["cia"]["value"] / res["direct"]["value"],
    }
    import oracle
    th64 = T.theta0.astype(np.float32).astype(np.float64)
    out["cpu_baseline"] = oracle_baseline(args, lambda rows: oracle.triadic_rhs(
        n, g.row_ptr, g.col, g.labels, T.tri_seed, T.p_tri, T.cross_tri, None, T.K1, T.K2, th64, rows=rows),
        n, "triadic_n%d" % n)
    aux_us = res["cia"]["aux_us"]
    if aux_us > 0 and res["cia"]["bytes_aux"] > 0:
        # the missing-pair sum launch streams the stored lists once per stage
        achieved = res["cia"]["bytes_aux"] / (aux_us * 1e-6) / 1e9
        out["roofline"] = {"kernel": "tri_missing_kernel", "bound": "hbm", "achieved": round(achieved, 1),
                           "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                           "traffic": None}
    print(json.dumps(out), flush=True)


def bench_general(args, cia, W, torch, np):
    """A general (non-difference) phase coupling, the real 2-D Fourier series
    of App. A.2 with p = 2 and seeded coefficients, on the N = 1e6 power-law
    community graph of the phase bench, FP32, RK4: CIA against the direct
    method on the same GPU."""
    P = W.kuramoto_large()
    g = P.graph
    n = g.n
    rng = np.random.default_rng(23)
    cs = [rng.normal(size=(3, 3)) / 3.0 for _ in range(4)]
    log("general-coupling workload: n=%d nnz=%d communities=%d p=2" % (n, g.nnz, g.ncomm))
    th0 = P.theta0.astype(np.float32)
    res = {}
    for name, method, steps in (("cia", cia.CIA_METHOD_CIA, 50), ("direct", cia.CIA_METHOD_DIRECT, 5)):
        plan = cia.Plan.phase(n, g.row_ptr, g.col, g.labels, P.omega, K=P.K, gen=cs, method=method,
                              flags=cia.CIA_FLAG_NO_VALIDATE)
        info = plan.info()
        th = torch.as_tensor(th0, device="cuda")
        plan.integrate(th, P.dt, 2)
        plan.set_timing(1)
        plan.timing(reset=True)
        ms = timed(torch, lambda s: plan.integrate(th, P.dt, steps, stream=s))
        t = plan.timing(reset=True)
        stage_us = 1e3 * t.stage_ms / max(t.stage_launches, 1)
        res[name] = {"ms_per_step": ms / steps, "value": n * 4 * steps / (ms / 1e3), "stage_us": round(stage_us, 2),
                     "bytes_per_stage": info.bytes_per_stage,
                     "achieved_gbs": round(info.bytes_per_stage / (stage_us * 1e-6) / 1e9, 1)}
        log("%-7s %.4f ms/step, stage %.2f us, %.1f GB/s" % (name, ms / steps, stage_us, res[name]["achieved_gbs"]))
        plan.close()
    c = res["cia"]
    line = {
        "metric": "general-coupling RHS node-updates/s (CIA), 1 MI355X, N=1e6 community graph",
        "value": c["value"], "unit": "RHS node-updates/s", "n_gpus": 1, "steps": 50, "warmup": 2,
        "ms_per_step": c["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "general_p2_n1e6", "n": n, "stepper": "rk4", "dt": P.dt},
        "roofline": {"kernel": "phase_stage_kernel (general)", "bound": "hbm", "achieved": c["achieved_gbs"],
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(c["achieved_gbs"] / HBM_PEAK_GBS, 4),
                     "traffic": None},
        "methods": res, "speedup_vs_direct": res["direct"]["ms_per_step"] / c["ms_per_step"],
    }
    import oracle
    th64 = th0.astype(np.float64)
    line["cpu_baseline"] = oracle_baseline(args, lambda rows: oracle.phase_rhs_general(
        n, g.row_ptr, g.col, P.omega, P.K, *cs, th64, rows=rows), n, "general_p2_n1e6")
    print(json.dumps(line), flush=True)


def bench_poly(args, cia, W, torch, np):
    """Desai-Zwanzig dynamics (App. A.5: h(x) = x, f = x - x^3), a cubic
    difference coupling and coupled van der Pol oscillators (two components,
    Table 1) on the N = 1e6 power-law community graph of the phase bench,
    FP32, RK4: CIA against the direct method on the same GPU."""
    P = W.kuramoto_large()
    g = P.graph
    n = g.n
    log("poly workload: n=%d nnz=%d communities=%d" % (n, g.nnz, g.ncomm))
    x0 = np.random.default_rng(17).uniform(-1.5, 1.5, n).astype(np.float32)
    res = {}
    for name, h in (("dz", [0.0, 1.0]), ("cubic", [0.0, 1.0, 0.0, -0.2])):
        for method in (cia.CIA_METHOD_CIA, cia.CIA_METHOD_DIRECT):
            plan = cia.Plan.poly(n, g.row_ptr, g.col, g.labels, None, K=3.0, h=h, f=[0.0, 1.0, 0.0, -1.0],
                                 method=method, flags=cia.CIA_FLAG_NO_VALIDATE)
            info = plan.info()
            steps = 50 if method == cia.CIA_METHOD_CIA else 5
            x = torch.as_tensor(x0, device="cuda")
            plan.integrate(x, 0.01, 2)
            plan.set_timing(1)
            plan.timing(reset=True)
            ms = timed(torch, lambda s: plan.integrate(x, 0.01, steps, stream=s))
            t = plan.timing(reset=True)
            stage_us = 1e3 * t.stage_ms / max(t.stage_launches, 1)
            key = "%s_%s" % (name, "cia" if method == cia.CIA_METHOD_CIA else "direct")
            res[key] = {"ms_per_step": ms / steps, "value": n * 4 * steps / (ms / 1e3), "stage_us": round(stage_us, 2),
                        "bytes_per_stage": info.bytes_per_stage,
                        "achieved_gbs": round(info.bytes_per_stage / (stage_us * 1e-6) / 1e9, 1)}
            log("%-12s %.4f ms/step, stage %.2f us, %.1f GB/s" % (key, ms / steps, stage_us,
                                                                  res[key]["achieved_gbs"]))
            plan.close()
    # coupled van der Pol oscillators (two components, Table 1 with eps = 0.3)
    F = np.zeros((2, 4, 4))
    F[0, 0, 1], F[0, 3, 0], F[0, 1, 0], F[1, 1, 0] = 1.0, -1.0 / 3.0, 1.0, -0.3
    xv0 = np.random.default_rng(18).uniform(-1.5, 1.5, (2, n)).astype(np.float32)
    for method in (cia.CIA_METHOD_CIA, cia.CIA_METHOD_DIRECT):
        plan = cia.Plan.poly(n, g.row_ptr, g.col, g.labels, None, K=3.0, h=[0.0, 1.0], dim=2, f2=F,
                             method=method, flags=cia.CIA_FLAG_NO_VALIDATE)
        info = plan.info()
        steps = 50 if method == cia.CIA_METHOD_CIA else 5
        x = torch.as_tensor(xv0, device="cuda")
        plan.integrate(x, 0.01, 2)
        plan.set_timing(1)
        plan.timing(reset=True)
        ms = timed(torch, lambda s: plan.integrate(x, 0.01, steps, stream=s))
        t = plan.timing(reset=True)
        stage_us = 1e3 * t.stage_ms / max(t.stage_launches, 1)
        key = "vdp_%s" % ("cia" if method == cia.CIA_METHOD_CIA else "direct")
        res[key] = {"ms_per_step": ms / steps, "value": n * 4 * steps / (ms / 1e3), "stage_us": round(stage_us, 2),
                    "bytes_per_stage": info.bytes_per_stage,
                    "achieved_gbs": round(info.bytes_per_stage / (stage_us * 1e-6) / 1e9, 1)}
        log("%-12s %.4f ms/step, stage %.2f us, %.1f GB/s" % (key, ms / steps, stage_us, res[key]["achieved_gbs"]))
        plan.close()
    dz = res["dz_cia"]
    line = {
        "metric": "Desai-Zwanzig RHS node-updates/s (CIA), 1 MI355X, N=1e6 community graph",
        "value": dz["value"], "unit": "RHS node-updates/s", "n_gpus": 1, "steps": 50, "warmup": 2,
        "ms_per_step": dz["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "poly_dz_n1e6", "n": n, "stepper": "rk4", "dt": 0.01},
        "roofline": {"kernel": "poly_stage_kernel", "bound": "hbm", "achieved": dz["achieved_gbs"],
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(dz["achieved_gbs"] / HBM_PEAK_GBS, 4),
                     "traffic": None},
        "methods": res,
        "speedup_vs_direct": {k: res[k + "_direct"]["ms_per_step"] / res[k + "_cia"]["ms_per_step"]
                              for k in ("dz", "cubic", "vdp")},
    }
    import oracle
    x64 = x0.astype(np.float64)
    line["cpu_baseline"] = oracle_baseline(args, lambda rows: oracle.poly_rhs(
        n, g.row_ptr, g.col, None, 3.0, [0.0, 1.0], [0.0, 1.0, 0.0, -1.0], x64, rows=rows), n, "poly_dz_n1e6")
    print(json.dumps(line), flush=True)


def bench_structured(args, cia, W, torch, np):
    """Phase model on the structured adjacencies of App. B, FP32, RK4: rank-one
    coupling and the k-nearest-neighbour ring with k = N/10 at N = 1e7 (E1
    only: O(N) per stage for any k), then CIA against the direct method at
    N = 1e5 (ring k = 1e4; rank one, O(N^2) direct)."""
    rng = np.random.default_rng(31)

    def make(n, kind, k, method):
        om = rng.standard_normal(n)
        kw = dict(alpha=rng.uniform(0.5, 1.5, n), beta=rng.uniform(0.5, 1.5, n)) if kind == "rank1" else dict(ring_k=k)
        return cia.Plan.structured(n, kind, om, K=2.0, method=method, **kw)

    def run(n, kind, k, method, steps):
        plan = make(n, kind, k, method)
        info = plan.info()
        th0 = rng.uniform(0, 2 * np.pi, n).astype(np.float32)
        # median of args.reps calls; HIP events around one launch in 17 of
        # each kind (stage, scan), inside the timed region
        ms, t, _, _ = time_integrate(plan, torch, th0, 0.01, steps, 2, with_r=False, timing_every=17,
                                     reps=args.reps)
        stage_us = 1e3 * t.stage_ms / max(t.stage_launches, 1)
        res = {"n": n, "kind": kind, "k": k, "method": "cia" if method == 0 else "direct", "steps": steps,
               "ms_per_step": ms / steps, "value": n * 4 * steps / (ms / 1e3), "stage_us": round(stage_us, 2),
               "scan_us": round(1e3 * t.aux_ms / max(t.aux_launches, 1), 2),
               "bytes_per_stage": info.bytes_per_stage}
        if method == 0:
            gbs = info.bytes_per_stage / (stage_us * 1e-6) / 1e9
            res["roofline"] = {"kernel": "struct_stage_kernel", "bound": "hbm", "achieved": round(gbs, 1),
                               "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                               "traffic": None}
        log("%-6s %-6s n=%d k=%d: %.4f ms/step, stage %.2f us, scan %.2f us" % (
            kind, res["method"], n, k, res["ms_per_step"], stage_us, res["scan_us"]))
        plan.close()
        return res

    big = int(1e7)
    out = {"rank1": run(big, "rank1", 0, 0, 50), "ring": run(big, "ring", big // 10, 0, 50)}
    small = int(1e5)
    cmp = {}
    for kind, k in (("rank1", 0), ("ring", small // 10)):
        a = run(small, kind, k, 0, 50)
        b = run(small, kind, k, 1, 3)
        cmp[kind] = {"cia": a, "direct": b, "speedup": b["ms_per_step"] / a["ms_per_step"]}
    line = {
        "metric": "structured-adjacency RHS node-updates/s (ring, k = N/10), 1 MI355X",
        "value": out["ring"]["value"], "unit": "RHS node-updates/s", "n_gpus": 1, "steps": 50, "warmup": 2,
        "ms_per_step": out["ring"]["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "structured_ring_n1e7_k1e6", "n": big, "stepper": "rk4", "dt": 0.01},
        "roofline": out["ring"]["roofline"], "large": out, "vs_direct_n1e5": cmp,
    }
    import oracle
    th64 = rng.uniform(0, 2 * np.pi, big)
    line["cpu_baseline"] = oracle_baseline(args, lambda rows: oracle.structured_rhs(
        "ring", big, None, 2.0, [0.0, 1.0], [0.0, 0.0], th64, k=big // 10, rows=rows), big, "structured_ring_n1e7_k1e6")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
