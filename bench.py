"""Benchmark: fused harmonic summing + detection on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-variants]
                    [--batched-fops N] [--copy-calibration] [--launch JSON]
    python bench.py --traffic-summary FETCH_CSV WRITE_CSV --launch JSON --traffic-cmds C1 C2

Workload: one filter-output plane of 85 templates x 2^21 bins of fp32 power
(Exp(1) noise, 50 injected harmonic signals, seed 2), 8 harmonic planes,
thresholds T_k = k + 6 sqrt(k), full candidate list.  A step is one
hs_detect call (counter clear + detection kernel) over the plane, which is
resident in HBM before the timed region starts.

The launch configuration is the autotuner's choice for the plane (every
candidate timed on the resident input before the timed region; the planner's
defaults stay unless another candidate is faster by more than 2 %); the line
reports it with its margins under `autotuned`.

Prints one JSON line.  `value` is FOP points per second (every point taken
through all 8 planes and the threshold test).  `roofline` refers to the
detection kernel the chosen plan launches: algorithmic bytes (one read of
the FOP + 8 bytes per candidate + the counters) over the average duration
of one hs_detect call (the counter clear, the detection kernel and the
per-plane counting pass), measured with HIP events on the launch stream.
`cold_start` times the process's first 60 launches.  `traffic` comes from
rocprofv3 FETCH_SIZE / WRITE_SIZE counters recorded in profiles/ for that
kernel and its current sources (null otherwise).  `read_ceiling` times one
streaming read of the plane (hs_stream_read), the bound the detection
kernel is compared against.  `cpu_baseline` times the CPU oracle on a
bounded sample of the same plane.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
CSRC = "paper_1805_12258_amd/csrc/"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "ska_detect_f32_traffic.json")
CTYPE = {"f32": "float", "f16": "_Float16", "bf16": "bf16"}


def log(msg):
    """Progress on stderr (the JSON line alone goes to stdout)."""
    print("bench: " + msg, file=sys.stderr, flush=True)


def detection_kernel(plan, dtype="f32"):
    """Name of the detection kernel the plan launches and the sources it is
    built from (the tile kernel, the strip walk at V bins per lane or the
    fractional-mapping kernel)."""
    info, H = plan.info, plan.n_hp
    g = (H - 1) // 4
    if info["detector"] == 1:
        v = info["bins_per_lane"]
        return ("k_walk<%s,%d,%d>" % (CTYPE[dtype], H, v),
                [CSRC + "hs_walk_impl.h", CSRC + "hs_walk_inst.h",
                 CSRC + "hs_walk_%s_v%d_g%d.hip" % (dtype, v, g), CSRC + "hs_internal.h"])
    if info["detector"] == 2:
        return ("k_frac<%s,detect>" % CTYPE[dtype], [CSRC + "hs_frac.hip", CSRC + "hs_internal.h"])
    return ("k_fused<%s,%d,detect>" % (CTYPE[dtype], H),
            [CSRC + "hs_fused_impl.h", CSRC + "hs_fused_inst.h",
             CSRC + "hs_fused_%s_g%d.hip" % (dtype, g), CSRC + "hs_internal.h"])


def kernel_source_hash(sources):
    h = hashlib.sha256()
    for f in sources:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def stored_traffic(kernel, sources):
    """Per-launch HBM bytes of the detection kernel from the committed
    counter summary, or None when it was taken on another kernel or on
    different kernel sources."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    d = json.load(open(TRAFFIC_FILE))
    if d.get("kernel") != kernel or d.get("source_hash") != kernel_source_hash(sources):
        return None
    return d


def tuned_plan(T, N, H, store, ta, dtype="f32", input_scale=1.0, reps=20, launch=None):
    """The autotuner's choice for this plane (every candidate timed on the
    resident input), and a summary: the configuration, its time, the
    planner's default time and the margin over the runner-up.  A given
    `launch` configuration is taken as it is (no tuning)."""
    import paper_1805_12258_amd as hs
    from paper_1805_12258_amd import autotune
    if launch is not None:
        plan = hs.Plan(T, N, H, dtype=dtype, input_scale=input_scale, **launch)
        return plan, {"config": launch, "tuned": False, "kernel": detection_kernel(plan, dtype)[0]}
    t0 = time.perf_counter()
    best, ms, tried = autotune.tune(T, N, H, dtype=dtype, input_scale=input_scale, fops=store, ta=ta,
                                    reps=reps, cache=None)
    sm = autotune.summary(best, ms, tried)
    sm["tuning_s"] = time.perf_counter() - t0
    plan = hs.Plan(T, N, H, dtype=dtype, input_scale=input_scale, **best)
    sm["kernel"] = detection_kernel(plan, dtype)[0]
    return plan, sm


def time_detect(plan, fop, ta, capacity, steps, warmup):
    import paper_1805_12258_amd as hs
    dev = fop.device
    out = torch.empty((capacity, 2), dtype=torch.int32, device=dev)
    counts = torch.empty(plan.n_hp + 1, dtype=torch.int64, device=dev)
    ld = fop.stride(0)
    for _ in range(warmup):
        hs.hs_detect(plan.handle, fop, ld, ta, out, capacity, counts)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t0.record()
    for i in range(steps):
        ev[i][0].record()
        hs.hs_detect(plan.handle, fop, ld, ta, out, capacity, counts)
        ev[i][1].record()
    t1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    total_ms = t0.elapsed_time(t1)
    per_launch = [a.elapsed_time(b) for a, b in ev]
    return dict(ms_per_step=total_ms / steps, launch_ms=float(np.mean(per_launch)),
                launch_ms_min=float(np.min(per_launch)), wall_s=wall,
                counts=counts.cpu().numpy().tolist())


def host_threads():
    """Threads for host work: the CPUs this process may run on, at most 16
    (the host share of one GPU on the machines this runs on)."""
    return max(1, min(16, len(os.sched_getaffinity(0))))


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(fop_cpu, H, ta_np, max_bins, seconds_per_run=4.0, runs=3):
    """The oracle (Algorithm 1 order, fp32, with detection) on the first
    `max_bins` bins of the plane (a prefix of bins is self-contained: every
    source bin floor(j/m) <= j): three timed runs of about 4 s each (a
    bounded sample of the workload), the median reported, on host_threads()
    threads; plus one single-thread pass on an eighth of the sample."""
    import oracle
    sample = np.ascontiguousarray(fop_cpu[:, :max_bins].numpy())
    threads = host_threads()
    cap = 1 << 22
    oracle.detect_f32(sample[:, :1024], H, ta_np, cap=cap, nthreads=threads)     # load + warm
    rates = []
    total_pts = 0
    for _ in range(runs):
        reps = 0
        t = time.perf_counter()
        while True:
            oracle.detect_f32(sample, H, ta_np, cap=cap, nthreads=threads)
            reps += 1
            dt = time.perf_counter() - t
            if dt >= seconds_per_run:
                break
        pts = sample.shape[0] * sample.shape[1] * reps
        total_pts += pts
        rates.append(pts / dt)
    t1 = time.perf_counter()
    one = np.ascontiguousarray(sample[:, :max_bins // 8])
    oracle.detect_f32(one, H, ta_np, cap=cap, nthreads=1)
    dt1 = time.perf_counter() - t1
    return {"value": float(np.median(rates)), "unit": "points/s", "cores": threads, "kind": "oracle",
            "nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)), "cpu_model": cpu_model(),
            "runs_points_per_s": rates,
            "sample": "first %d bins x %d templates of the same plane (%.1f M points in all), median of %d "
                      "runs of about %.0f s on %d threads (the CPU share of one GPU: at most 16 of the "
                      "%d CPUs); 1 thread on %d bins: %.3g points/s"
                      % (max_bins, sample.shape[0], total_pts / 1e6, runs, seconds_per_run, threads,
                         os.cpu_count() or 0, max_bins // 8, one.size / dt1)}


def candidate_words(out, counts):
    """Sorted int64 CL1 words of a detect output (first counts[-1] rows)."""
    n = int(counts[-1].item())
    w = out[:n, 0].to(torch.int64) & 0xffffffff
    return torch.sort(w).values


def precision_recall(words, ref_words):
    """Candidate-set agreement of a reduced-precision run with the fp32 run
    (which equals the oracle bitwise)."""
    if len(words) == 0 or len(ref_words) == 0:
        return 1.0 if len(words) == len(ref_words) else 0.0, 0.0
    common = int(torch.isin(words, ref_words).sum().item())
    return common / len(words), common / len(ref_words)


def batched_leg(n_fops, steps, warmup, dev, launch=None):
    """The batched workload: n_fops FOPs of 85 templates and 2^19, 2^20 or
    2^21 bins (seeded), 16 planes, in one persistent launch replayed from a
    captured HIP graph, against one hs_detect launch per FOP."""
    import paper_1805_12258_amd as hs
    import synth
    cfg = synth.BATCHED
    T, H = cfg["n_temp"], cfg["n_hp"]
    lens = synth.batched_lengths(n_fops)
    fops = []
    for f, n in enumerate(lens):
        fops.append(synth.make_batched_fop(f, n, device=dev))
        if (f + 1) % 128 == 0:
            log("batched: %d FOPs drawn" % (f + 1))
    ta = torch.from_numpy(synth.thresholds(H, T)).to(dev)
    # room for twice the expected noise candidates of 16 planes
    caps = [int(2 * 180000 * n / (1 << 20)) + 4096 for n in lens]
    offs = np.concatenate([[0], np.cumsum(caps)[:-1]]).astype(np.int64)
    out = torch.empty((int(np.sum(caps)), 2), dtype=torch.int32, device=dev)
    counts = torch.empty((n_fops, H + 1), dtype=torch.int64, device=dev)
    fop_ptrs = torch.tensor([x.data_ptr() for x in fops], dtype=torch.int64, device=dev)
    lds = torch.tensor([x.stride(0) for x in fops], dtype=torch.int64, device=dev)
    offs_d = torch.from_numpy(offs).to(dev)
    caps_d = torch.tensor(caps, dtype=torch.int64, device=dev)
    # launch configuration from the autotuner, timed on the first 64 FOPs
    from paper_1805_12258_amd import autotune
    t_tune = time.perf_counter()
    sub = min(64, n_fops)
    if launch is None:
        tuned, tuned_ms, tried = autotune.tune(T, 0, H, n_chans=lens[:sub], fops=fops[:sub], ta=ta, reps=3,
                                               cache=None)
        summary = autotune.summary(tuned, tuned_ms, tried)
    else:
        tuned, summary = launch, {"config": launch, "tuned": False}
    t_tune = time.perf_counter() - t_tune
    plan = hs.Plan(T, 0, H, n_chans=lens, **tuned)
    args = (plan.handle, fop_ptrs, lds, ta, out, offs_d, caps_d, counts)
    hs.hs_detect_batched(*args)                 # eager call: uploads the plan tables
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=stream):
        hs.hs_detect_batched(*args, stream=stream)
    for _ in range(warmup):
        graph.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        graph.replay()
    e1.record()
    torch.cuda.synchronize()
    batched_ms = e0.elapsed_time(e1) / steps
    batched_counts = counts.clone()

    plans = {n: hs.Plan(T, n, H) for n in sorted(set(lens))}
    single_counts = torch.empty_like(counts)
    out_single = torch.empty_like(out)

    def per_fop():
        for f, x in enumerate(fops):
            hs.hs_detect(plans[lens[f]].handle, x, x.stride(0), ta, out_single[offs[f]:], caps[f],
                         single_counts[f])

    for _ in range(max(1, warmup // 2)):
        per_fop()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        per_fop()
    e1.record()
    torch.cuda.synchronize()
    single_ms = e0.elapsed_time(e1) / steps
    if not torch.equal(single_counts, batched_counts):
        raise RuntimeError("batched and per-FOP candidate counts differ")
    # the candidate lists themselves, FOP by FOP: (row, plane, bin, power
    # bits), sorted; the batched word takes its bin field from the longest
    # FOP, a per-FOP word from its own length
    graph.replay()
    torch.cuda.synchronize()

    def canonical(o, n, info):
        w = o[:n, 0].to(torch.int64) & 0xffffffff
        kb = info["s_row"] - info["s_bin"]
        r = w >> info["s_row"]
        k = (w >> info["s_bin"]) & ((1 << kb) - 1)
        j = w & ((1 << info["s_bin"]) - 1)
        c = (r << 40) | (k << 32) | j
        order = torch.argsort(c)
        return c[order], o[:n, 1][order]

    for f in range(n_fops):
        n = int(batched_counts[f, -1].item())
        if n > caps[f]:
            continue                     # which entries are stored past the capacity is unspecified
        ca, pa = canonical(out[offs[f]:], n, plan.info)
        cb, pb = canonical(out_single[offs[f]:], n, plans[lens[f]].info)
        if not (torch.equal(ca, cb) and torch.equal(pa, pb)):
            raise RuntimeError("batched and per-FOP candidate lists differ (FOP %d)" % f)
    points = T * int(np.sum(lens))
    fop_bytes = 4 * points
    del fops, out, out_single
    return {"n_fops": n_fops, "points": points, "fop_gb": fop_bytes / 1e9,
            "value": points / (batched_ms * 1e-3), "unit": "points/s",
            "ms_per_step": batched_ms, "hbm_gbs": fop_bytes / (batched_ms * 1e-3) / 1e9,
            "per_fop_launches_ms": single_ms, "vs_per_fop": single_ms / batched_ms,
            "candidates": int(batched_counts[:, -1].sum().item()),
            "lists_equal_per_fop": True,
            "launch": "one persistent kernel replayed from a captured HIP graph",
            "autotuned": dict(summary, on_fops=sub, tuning_s=t_tune)}


def precision_leg(n_fops, dev, threads):
    """The precision workload: fp16 and bf16 storage of power x 1/8 for the
    first n_fops FOPs of 85 x 2^21 fp32 (50 signals each, seeds 4*10^6 + f),
    8 planes.  Per storage type, over every point of every plane of those
    FOPs: the error of the 16-bit path's planes (hs_sum) against the fp64
    oracle's planes of the fp32 FOP, as the largest relative error where the
    fp64 sum is >= 1 and the largest absolute error, and the closed-form
    bound |S - S64| <= (u_in + (k-1) 2^-24) S64 + k d_sub checked at every
    point (all terms are >= 0; u_in = 2^-11 for fp16, 2^-8 for bf16; d_sub =
    8 2^-25 for fp16 subnormals of x/8, 0 for bf16); and per plane the
    precision and recall of the 16-bit candidate lists against the fp32
    oracle's.  The FOPs are drawn on the GPU and copied to the host for the
    oracle."""
    import oracle
    import paper_1805_12258_amd as hs
    import synth
    cfg = synth.PRECISION
    T, N, H, scale = cfg["n_temp"], cfg["n_chan"], cfg["n_hp"], cfg["input_scale"]
    ta_np = synth.thresholds(H, T)
    ta = torch.from_numpy(ta_np).to(dev)
    kinds = {"f16": (torch.float16, 2.0 ** -11, 8 * 2.0 ** -25), "bf16": (torch.bfloat16, 2.0 ** -8, 0.0)}
    plans = {name: hs.Plan(T, N, H, dtype=name, input_scale=scale) for name in kinds}
    res = {name: {"max_rel_err": 0.0, "max_abs_err": 0.0, "bound_held": True, "max_err_over_bound": 0.0,
                  "tp": [0] * H, "fp": [0] * H, "fn": [0] * H} for name in kinds}
    t0 = time.perf_counter()
    for f in range(n_fops):
        x = synth.make_precision_fop(f, device=dev)
        xc = x.cpu().numpy()
        ref = torch.from_numpy(oracle.sum_f64(xc, H, nthreads=threads)).to(dev)
        iw, _, ic = oracle.detect_f32(xc, H, ta_np, nthreads=threads)
        want = torch.from_numpy(iw.astype(np.int64)).to(dev)
        for name, (dt, u_in, d_sub) in kinds.items():
            r = res[name]
            store = synth.quantize(x, dt, scale)
            plan = plans[name]
            hp = plan.sum(store)
            for k in range(1, H + 1):
                s64 = ref[k - 1]
                err = (hp[k - 1].double() - s64).abs()
                big = s64 >= 1.0
                if bool(big.any()):
                    r["max_rel_err"] = max(r["max_rel_err"], float((err[big] / s64[big]).max()))
                r["max_abs_err"] = max(r["max_abs_err"], float(err.max()))
                bound = (u_in + (k - 1) * 2.0 ** -24) * s64 + k * d_sub
                r["bound_held"] = r["bound_held"] and bool((err <= bound * (1 + 1e-12)).all())
                pos = bound > 0
                r["max_err_over_bound"] = max(r["max_err_over_bound"], float((err[pos] / bound[pos]).max()))
                del err, big, bound, pos
            del hp
            out, cnt = plan.detect(store, ta, capacity=1 << 22)
            got = candidate_words(out, cnt)
            kmask = (1 << plan.info["s_k"]) - 1
            for k in range(1, H + 1):
                g = got[((got >> plan.info["s_bin"]) & kmask) == k - 1]
                w = want[((want >> plan.info["s_bin"]) & kmask) == k - 1]
                common = int(torch.isin(g, w).sum().item())
                r["tp"][k - 1] += common
                r["fp"][k - 1] += len(g) - common
                r["fn"][k - 1] += len(w) - common
            del store, out
        del x, ref, want
        torch.cuda.empty_cache()
        log("precision: FOP %d of %d done" % (f + 1, n_fops))
    out = {"fops": n_fops, "of": cfg["n_fops"], "n_temp": T, "n_chan": N, "n_hp": H, "input_scale": scale,
           "seconds": time.perf_counter() - t0}
    for name, r in res.items():
        prec = [r["tp"][k] / max(1, r["tp"][k] + r["fp"][k]) for k in range(H)]
        rec = [r["tp"][k] / max(1, r["tp"][k] + r["fn"][k]) for k in range(H)]
        out[name] = {"max_rel_err_s_ge_1": r["max_rel_err"], "max_abs_err": r["max_abs_err"],
                     "p10_bound_held_every_point": r["bound_held"],
                     "max_err_over_bound": r["max_err_over_bound"],
                     "precision_per_k": prec, "recall_per_k": rec,
                     "candidates_vs_fp32_oracle": {"common": sum(r["tp"]), "extra": sum(r["fp"]),
                                                   "missed": sum(r["fn"])}}
    return out


def diff_leg(n_fops, steps, warmup, dev):
    """The differentiation workload: n_fops FOPs of 85 x 2^20 fp32, 8 planes,
    tau = 0.5.  Forward: lse of every plane (hs_lse_forward, fused: no plane
    is stored); backward: the
    gradient of L = sum_k tau * lse_k with respect to the FOP
    (hs_lse_backward, which forms the planes again, turns them into softmax
    weights and takes them through the transpose).  Timed separately."""
    import paper_1805_12258_amd as hs
    import synth
    cfg = synth.DIFF
    T, N, H, tau = cfg["n_temp"], cfg["n_chan"], cfg["n_hp"], cfg["tau"]
    fops = [synth.make_diff_fop(f, device=dev) for f in range(n_fops)]
    plan = hs.Plan(T, N, H)
    work = torch.empty(hs.hs_lse_workspace_bytes(plan.handle), dtype=torch.uint8, device=dev)
    lse = torch.empty((n_fops, H), dtype=torch.float64, device=dev)
    dfop = torch.empty((T, N), dtype=torch.float32, device=dev)

    def fwd():
        for f, x in enumerate(fops):
            hs.hs_lse_forward(plan.handle, x, x.stride(0), tau, lse[f], None, work)

    def bwd():
        for f, x in enumerate(fops):
            hs.hs_lse_backward(plan.handle, x, x.stride(0), lse[f], tau, None, dfop, work)

    out = {}
    for name, fn in (("forward", fwd), ("backward", bwd)):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        out[name + "_ms"] = e0.elapsed_time(e1) / steps
    points = n_fops * T * N
    total = out["forward_ms"] + out["backward_ms"]
    # per-point bytes that any such pass must move: the forward reads the
    # FOP once (4); the backward reads the FOP and writes the gradient (8).
    # The kernels move more (counters: 5.3 and 18.5 B per point, with the
    # staged source re-reads, the tile partials and the second pass's
    # read-modify-write of the touched quarter of the gradient)
    fb, bb = 4, 8
    out.update({"n_fops": n_fops, "points": points, "value": points / (total * 1e-3),
                "unit": "points/s (forward + backward)",
                "forward_gbs": fb * points / (out["forward_ms"] * 1e-3) / 1e9,
                "backward_gbs": bb * points / (out["backward_ms"] * 1e-3) / 1e9,
                "bytes_per_point": {"forward": fb, "backward": bb},
                "loss": float(tau * lse.sum().item())})
    del fops, work
    return out


def cold_start(T, N, H, fop, ta, n=60):
    """Launch durations of the first n detection launches of the process
    (HIP events per launch, the planner's defaults), before anything else
    has run on the GPU: the clocks ramp up over the first launches, which
    is why the timed region follows a warm-up."""
    import paper_1805_12258_amd as hs
    plan = hs.Plan(T, N, H)
    out = torch.empty((1 << 22, 2), dtype=torch.int32, device=fop.device)
    counts = torch.empty(H + 1, dtype=torch.int64, device=fop.device)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
    for a, b in ev:
        a.record()
        hs.hs_detect(plan.handle, fop, fop.stride(0), ta, out, 1 << 22, counts)
        b.record()
    torch.cuda.synchronize()
    us = [a.elapsed_time(b) * 1e3 for a, b in ev]
    return {"launches": n, "first_us": us[0], "us_2_5": float(np.mean(us[1:5])),
            "us_6_20": float(np.mean(us[5:20])), "us_21_%d" % n: float(np.mean(us[20:]))}


def read_ceiling(fop, reps=20):
    """The streaming-read ceiling for the plane: hs_stream_read of the whole
    resident FOP at several grid sizes, median launch time of each (HIP
    events on the launch stream), the best grid reported."""
    import paper_1805_12258_amd as hs
    nbytes = fop.numel() * fop.element_size()
    sink = torch.empty(8192, dtype=torch.float32, device=fop.device)
    res = {}
    for g in (2048, 4096, 8192):
        for _ in range(3):
            hs.hs_stream_read(fop, nbytes, sink, g)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for a, b in ev:
            a.record()
            hs.hs_stream_read(fop, nbytes, sink, g)
            b.record()
        torch.cuda.synchronize()
        res[g] = float(np.median([a.elapsed_time(b) for a, b in ev]))
    g = min(res, key=res.get)
    us = res[g] * 1e3
    return {"kernel": "k_stream_read", "bytes": nbytes, "grid": g, "us_median": us,
            "gbs": nbytes / (us * 1e-6) / 1e9, "frac": nbytes / (us * 1e-6) / 1e9 / HBM_PEAK_GBS,
            "us_by_grid": {str(k): v * 1e3 for k, v in res.items()}}


def traffic_summary(fetch_csv, write_csv, launch, cmds):
    """Writes the committed traffic figures of the detection kernel from two
    rocprofv3 counter runs of `bench.py --copy-calibration --launch ...`
    (FETCH_SIZE, then WRITE_SIZE): per-dispatch medians, each scaled by what
    the same counter reads for torch's copy of the plane (713031680 bytes
    each way)."""
    import csv
    import statistics
    import paper_1805_12258_amd as hs
    import synth
    cfg = synth.SKA
    T, N, H = cfg["n_temp"], cfg["n_chan"], cfg["n_hp"]
    plan = hs.Plan(T, N, H, **launch)
    kname, ksrc = detection_kernel(plan)
    base = kname.split("<")[0]
    targs = kname[kname.index("<") + 1:-1].split(",")
    if base == "k_fused":
        targs[-1] = "0"                                    # Mode: detect
    match = "%s<%s>" % (base, ", ".join(targs))
    plane = T * N * 4

    def medians(path, counter):
        k, c = [], []
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != counter:
                continue
            if match in r["Kernel_Name"]:
                k.append(float(r["Counter_Value"]))
            elif "copy" in r["Kernel_Name"].lower():
                c.append(float(r["Counter_Value"]))
        if not k or not c:
            raise SystemExit("%s: no %s dispatches of %s or of the copy kernel" % (path, counter, match))
        c = [v for v in c if v >= 0.5 * max(c)]          # the plane copies, not small transfers
        return statistics.median(k), statistics.median(c), len(k)

    fk, fc, nf = medians(fetch_csv, "FETCH_SIZE")
    wk, wc, nw = medians(write_csv, "WRITE_SIZE")
    fscale, wscale = plane / (fc * 1024), plane / (wc * 1024)
    d = {"source_hash": kernel_source_hash(ksrc), "kernel": kname, "launch": launch,
         "workload": "85 x 2^21 fp32, H=8, thresholds k+6*sqrt(k)",
         "fetch_kib_raw": fk, "write_kib_raw": wk, "dispatches": [nf, nw],
         "copy_bytes": plane, "copy_fetch_kib": fc, "copy_write_kib": wc,
         "fetch_scale": fscale, "write_scale": wscale,
         "fetch_bytes": fk * 1024 * fscale, "write_bytes": wk * 1024 * wscale,
         "fetch_cmd": cmds[0], "write_cmd": cmds[1]}
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(d, f, indent=1)
        f.write("\n")
    md = ["# HBM-side traffic of the detection kernel %s (85 x 2^21 fp32, H=8)" % kname, "",
          "Launch configuration %s.  Commands (repository root, TMPDIR=/tmp), one counter per run:" %
          json.dumps(launch), "", "    " + cmds[0], "    " + cmds[1], "",
          "Calibration: torch's copy of the plane (%d B each way) reads FETCH_SIZE %.1f KiB and "
          "WRITE_SIZE %.1f KiB, so FETCH_SIZE is scaled by %.4f and WRITE_SIZE by %.4f." %
          (plane, fc, wc, fscale, wscale), "",
          "| per launch (median of %d / %d dispatches) | raw KiB | scaled bytes | vs one read of the plane |" %
          (nf, nw), "|---|---|---|---|",
          "| FETCH_SIZE | %.1f | %.4g | %.3f |" % (fk, d["fetch_bytes"], d["fetch_bytes"] / plane),
          "| WRITE_SIZE | %.1f | %.4g | %.4f |" % (wk, d["write_bytes"], d["write_bytes"] / plane), "",
          "Kernel source hash %s: bench.py reports these bytes as roofline.traffic only while the "
          "plan launches this kernel and its sources hash to this value." % d["source_hash"], ""]
    with open(TRAFFIC_FILE[:-5] + ".md", "w") as f:
        f.write("\n".join(md))
    print(json.dumps(d, indent=1))


def profile_detect(spec, launches=6):
    """Six hs_detect launches of one configuration on the synthetic plane
    (for rocprofv3 counter passes); prints the candidate count."""
    import paper_1805_12258_amd as hs
    import synth
    dt, H, V = spec.split(",")
    H, V = int(H), int(V)
    cfg = synth.SKA
    T, N = cfg["n_temp"], cfg["n_chan"]
    fop = synth.make_ska(device=torch.device("cuda:0"))
    scale = 1.0
    if dt != "f32":
        scale = synth.PRECISION["input_scale"]
        fop = synth.quantize(fop, {"f16": torch.float16, "bf16": torch.bfloat16}[dt], scale)
    ta = torch.from_numpy(synth.thresholds(H, T)).cuda()
    kw = {"schedule": 4, "bins_per_lane": V} if V > 0 else {}
    plan = hs.Plan(T, N, H, dtype=dt, input_scale=scale, **kw)
    cap = 1 << 23
    out = torch.empty((cap, 2), dtype=torch.int32, device=fop.device)
    counts = torch.empty(H + 1, dtype=torch.int64, device=fop.device)
    for _ in range(launches):
        hs.hs_detect(plan.handle, fop, fop.stride(0), ta, out, cap, counts)
    torch.cuda.synchronize()
    print(json.dumps({"profile_detect": spec, "kernel": detection_kernel(plan, dt)[0],
                      "candidates": int(counts[-1].item())}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--cpu-bins", type=int, default=1 << 21)
    ap.add_argument("--batched-fops", type=int, default=512,
                    help="FOPs of the batched leg (0 skips it)")
    ap.add_argument("--singlehp-steps", type=int, default=10,
                    help="timed steps of the SingleHP baseline (0 skips it)")
    ap.add_argument("--diff-fops", type=int, default=16,
                    help="FOPs of the differentiation leg (0 skips it)")
    ap.add_argument("--precision-fops", type=int, default=8,
                    help="FOPs of the precision leg taken through the fp64 oracle (0 skips it)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain device copy of the FOP's size (counter scale)")
    ap.add_argument("--launch", default="{}",
                    help='launch configurations as JSON, {"f32": {...}, "f16": {...}, "bf16": {...}, '
                         '"batched": {...}} of Plan keyword arguments; a leg not named takes the '
                         "autotuner's choice")
    ap.add_argument("--no-read-ceiling", action="store_true")
    ap.add_argument("--traffic-summary", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the traffic figures under profiles/ from two counter runs "
                         "(with --launch and --traffic-cmds) and exit; runs on the CPU")
    ap.add_argument("--traffic-cmds", nargs=2, default=["", ""])
    ap.add_argument("--profile-detect", default=None, metavar="DTYPE,H,V",
                    help="only six hs_detect launches on the 85 x 2^21 plane stored as DTYPE with H planes "
                         "(V > 0: strip walk with V bins per lane; 0: the planner's choice), for counter runs")
    args = ap.parse_args()
    if args.profile_detect:
        profile_detect(args.profile_detect)
        return
    launch = json.loads(args.launch)
    if args.traffic_summary:
        traffic_summary(args.traffic_summary[0], args.traffic_summary[1],
                        launch.get("f32", {"schedule": 0}), args.traffic_cmds)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the harmonic-summing path here runs on a single "
              "MI355X (--gpus %d is not supported)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import paper_1805_12258_amd as hs
    import synth

    cfg = synth.SKA
    T, N, H = cfg["n_temp"], cfg["n_chan"], cfg["n_hp"]
    dev = torch.device("cuda:0")
    fop = synth.make_ska(device=dev)
    ta_np = synth.thresholds(H, T)
    ta = torch.from_numpy(ta_np).to(dev)
    capacity = 1 << 22
    cold = cold_start(T, N, H, fop, ta)
    log("cold start: %s" % cold)
    plan, tuned = tuned_plan(T, N, H, fop, ta, launch=launch.get("f32"))
    kname, ksrc = detection_kernel(plan)
    log("autotuned: %s" % tuned)
    torch.cuda.synchronize()

    if args.copy_calibration:
        dst = torch.empty_like(fop)
        for _ in range(3):
            dst.copy_(fop)
        torch.cuda.synchronize()
        del dst

    r = time_detect(plan, fop, ta, capacity, args.steps, args.warmup)
    log("headline: %.4f ms per step" % r["ms_per_step"])
    ref_out, ref_counts = plan.detect(fop, ta, capacity=capacity)
    ref_words = candidate_words(ref_out, ref_counts)
    points = T * N
    n_cand = int(r["counts"][-1])
    alg_bytes = points * 4 + 8 * n_cand + 8 * (H + 1)
    achieved = alg_bytes / (r["launch_ms"] * 1e-3) / 1e9
    tr = stored_traffic(kname, ksrc)
    traffic = None
    fetch_ideal = None
    if tr is not None:
        traffic = tr["fetch_bytes"] + tr["write_bytes"]
        fetch_ideal = tr["fetch_bytes"] / (points * 4)

    line = {
        "metric": "harmonic-summed FOP points/s + achieved HBM GB/s; batched/FP16 vs plain fp32",
        "value": points / (r["ms_per_step"] * 1e-3),
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic: Exp(1) noise + 50 injected harmonic signals, seed 2",
        "config": {"workload": "ska-plain", "n_temp": T, "n_chan": N, "n_hp": H,
                   "thresholds": "k+6*sqrt(k)", "candidates": n_cand, "launch": tuned["config"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": kname, "launch_ms": r["launch_ms"],
                     "launch": "one hs_detect call: k_zero_i64 + %s + k_plane_counts" % kname,
                     "algorithmic_bytes": alg_bytes, "fetch_over_ideal": fetch_ideal},
        "seeds": {"ska": synth.SKA["seed"], "batched": synth.BATCHED["seed"],
                  "precision": synth.PRECISION["seed"], "differentiation": synth.DIFF["seed"]},
        "autotuned": tuned,
        "cold_start": cold,
        "hbm_gbs": achieved,
        "plane_points_per_s": H * points / (r["ms_per_step"] * 1e-3),
    }

    if not args.no_read_ceiling:
        rc = read_ceiling(fop)
        rc["detection_vs_ceiling"] = rc["us_median"] / (r["launch_ms"] * 1e3)
        line["read_ceiling"] = rc
        log("read ceiling: %.1f us (%.0f GB/s)" % (rc["us_median"], rc["gbs"]))

    # materialised planes (hs_sum): 4 B read + 4H B written per point
    hp = torch.empty((H, T, N), dtype=torch.float32, device=dev)
    ld = fop.stride(0)
    hs.hs_sum(plan.handle, fop, ld, hp)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        hs.hs_sum(plan.handle, fop, ld, hp)
    e1.record()
    torch.cuda.synchronize()
    sum_ms = e0.elapsed_time(e1) / 10
    sum_bytes = (4 + 4 * H) * points
    log("hs_sum: %.3f ms" % sum_ms)
    line["sum"] = {"ms": sum_ms, "bytes_per_point": 4 + 4 * H,
                   "gbs": sum_bytes / (sum_ms * 1e-3) / 1e9,
                   "frac": sum_bytes / (sum_ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
    del hp

    # canonical order of the full candidate list (hs_sort_candidates)
    n_all = int(ref_counts[-1].item())
    srt = ref_out[:n_all].clone()
    srt_work = torch.empty(max(hs.hs_sort_workspace_bytes(n_all), 1), dtype=torch.uint8, device=dev)
    copies = [srt.clone() for _ in range(6)]
    hs.hs_sort_candidates(copies.pop(), n_all, srt_work)          # warm-up (first use loads the kernels)
    torch.cuda.synchronize()
    e0.record()
    for c in copies:
        hs.hs_sort_candidates(c, n_all, srt_work)
    e1.record()
    torch.cuda.synchronize()
    line["sort"] = {"candidates": n_all, "ms": e0.elapsed_time(e1) / len(copies)}
    del srt, srt_work, copies

    # per-plane capped lists (N_cand = 200, Sec. III) from the full candidate
    # list, under each policy (bounded selection)
    n_all = int(ref_counts[-1].item())
    sel_out = torch.empty((H, 200, 2), dtype=torch.int32, device=dev)
    sel_cnt = torch.empty(H, dtype=torch.int64, device=dev)
    sel_work = torch.empty(max(hs.hs_select_workspace_bytes(plan.handle, n_all), 1), dtype=torch.uint8,
                           device=dev)
    capped = {"n_cand": 200, "candidates_in": n_all}
    for pname, pol in (("top", hs.HS_SELECT_TOP), ("last_alg2", hs.HS_SELECT_LAST_ALG2),
                       ("last_alg1", hs.HS_SELECT_LAST_ALG1)):
        hs.hs_select(plan.handle, ref_out, n_all, 200, pol, sel_out, sel_cnt, sel_work)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(20):
            hs.hs_select(plan.handle, ref_out, n_all, 200, pol, sel_out, sel_cnt, sel_work)
        e1.record()
        torch.cuda.synchronize()
        capped[pname + "_ms"] = e0.elapsed_time(e1) / 20
    capped["kept"] = int(sel_cnt.sum().item())
    line["capped"] = capped
    log("capped lists: %s" % capped)
    del sel_work

    if args.singlehp_steps > 0:
        # the paper's SingleHP method (planes through memory) on the same GPU,
        # with one launch per plane and with a single launch (Sec. V-A)
        out1 = torch.empty((capacity, 2), dtype=torch.int32, device=dev)
        cnt1 = torch.empty(H + 1, dtype=torch.int64, device=dev)
        work1 = torch.empty(hs.hs_singlehp_workspace_bytes(plan.handle), dtype=torch.uint8, device=dev)
        ld = fop.stride(0)
        # bytes per point: FOP read and HP_1 written, then per further plane
        # HP_{k-1} read, the stretched FOP value, HP_k written
        sb = 8 + 12 * (H - 1)
        line["singlehp"] = {"bytes_per_point": sb}
        for lname, fn in (("multiple_launch", hs.hs_detect_singlehp), ("single_launch", hs.hs_detect_singlehp_one)):
            for _ in range(2):
                fn(plan.handle, fop, ld, ta, out1, capacity, cnt1, work1)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(args.singlehp_steps):
                fn(plan.handle, fop, ld, ta, out1, capacity, cnt1, work1)
            e1.record()
            torch.cuda.synchronize()
            sh_ms = e0.elapsed_time(e1) / args.singlehp_steps
            if not torch.equal(cnt1.cpu(), ref_counts.cpu()):
                raise RuntimeError("SingleHP and fused candidate counts differ")
            line["singlehp"][lname] = {"ms_per_step": sh_ms, "value": points / (sh_ms * 1e-3),
                                       "unit": "points/s", "fused_speedup": sh_ms / r["ms_per_step"],
                                       "gbs": sb * points / (sh_ms * 1e-3) / 1e9}
        log("singlehp: %s" % line["singlehp"])
        del out1, work1

    if not args.no_variants:
        var = {}
        for name, dt in (("f16", torch.float16), ("bf16", torch.bfloat16)):
            scale = synth.PRECISION["input_scale"]
            store = synth.quantize(fop, dt, scale)
            p2, t2 = tuned_plan(T, N, H, store, ta, dtype=name, input_scale=scale, launch=launch.get(name))
            r2 = time_detect(p2, store, ta, capacity, max(20, args.steps // 2), 5)
            o2, c2 = p2.detect(store, ta, capacity=capacity)
            prec, rec = precision_recall(candidate_words(o2, c2), ref_words)
            ab = points * 2 + 8 * int(r2["counts"][-1]) + 8 * (H + 1)
            var[name] = {"value": points / (r2["ms_per_step"] * 1e-3),
                         "ms_per_step": r2["ms_per_step"], "launch_ms": r2["launch_ms"],
                         "hbm_gbs": ab / (r2["launch_ms"] * 1e-3) / 1e9,
                         "vs_f32": r["ms_per_step"] / r2["ms_per_step"],
                         "kernel": t2["kernel"], "autotuned": t2,
                         "candidates": int(r2["counts"][-1]),
                         "precision_vs_f32": prec, "recall_vs_f32": rec,
                         "storage": "%s of power x %g, fp32 sums" % (name, scale)}
            del store
        line["variants"] = var
        log("variants done")

    if not args.no_variants:
        # the fractional m/k mapping on the same plane (k source points per
        # point of plane k, 36 at H = 8)
        pf = hs.Plan(T, N, H, mapping="fractional")
        rf = time_detect(pf, fop, ta, capacity, max(10, args.steps // 10), 3)
        abf = points * 4 + 8 * int(rf["counts"][-1]) + 8 * (H + 1)
        line["fractional"] = {"ms_per_step": rf["ms_per_step"], "launch_ms": rf["launch_ms"],
                              "value": points / (rf["ms_per_step"] * 1e-3), "unit": "points/s",
                              "gathers_per_point": H * (H + 1) // 2, "candidates": int(rf["counts"][-1]),
                              "hbm_gbs": abf / (rf["launch_ms"] * 1e-3) / 1e9,
                              "kernel": detection_kernel(pf)[0]}
        log("fractional: %.3f ms" % rf["ms_per_step"])

    if args.batched_fops > 0:
        del fop, ref_out
        torch.cuda.empty_cache()
        line["batched"] = batched_leg(args.batched_fops, max(3, args.steps // 40),
                                      2, dev, launch=launch.get("batched"))
        log("batched: %.3f ms" % line["batched"]["ms_per_step"])
        fop = synth.make_ska(device=dev)

    if args.diff_fops > 0:
        line["differentiation"] = diff_leg(args.diff_fops, 3, 1, dev)
        log("differentiation done")
        torch.cuda.empty_cache()

    if args.precision_fops > 0:
        line["precision"] = precision_leg(args.precision_fops, dev, host_threads())
        log("precision done")
        torch.cuda.empty_cache()

    if not args.no_cpu:
        fop_cpu = fop[:, :args.cpu_bins].cpu()
        line["cpu_baseline"] = cpu_baseline(fop_cpu, H, ta_np, args.cpu_bins)
        log("cpu baseline done")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
