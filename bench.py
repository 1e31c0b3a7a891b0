#!/usr/bin/env python3
"""Benchmark of the PID hot path on one MI355X.

Default (headline) workload: the 2D soft-mask ensemble, N = 256 members on a
512 x 512 grid (M = 262,144 points), FP32 masks.  One step = the whole hot
path on that batch: all-pairs PID (FP16 MFMA Gram numerators, FP64 masses,
ratios, depths, ranks) plus PID-mean (its numerators are the Gram row sums of
the same pass; depths, ranks), one pid_both call.  The streaming PID-mean
kernel of pid_mean is measured in GB/s on the large 3D workload (extras).
``value`` = N^2 * M / (seconds per step), pair*points/s, inputs resident in
HBM.  The line also carries the roofline of the dominant kernel measured with
HIP events inside the timed region (on every 4th launch), the FP64 CPU oracle timed on the host, the
measured depth errors, and side measurements of the other workloads (FP32
comparator, BF16 split, fused scalar-field extraction with its binary INT8
variant, large 3D PID-mean in GB/s, 2D FP64).

``--mode serve`` runs the serving workload instead (Poisson arrivals of mixed
requests) and prints p50/p99 latency and requests/s; ``--mode sweep`` times
PID-mean on the shapes of the paper's scalability study; ``--mode largen`` runs
only the large-N leg (all-pairs depths with and without the matrix).
"""
from __future__ import annotations

import argparse
import gc
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "all-pairs PID pair·points/s (MFMA vs FP32) at ≤1e-4 err; PID-mean GB/s; p99 ms"
HBM_PEAK_GBPS = 8000.0
TIME_EVERY = 4   # the Gram kernel is bracketed by events on every 4th timed launch
ROTATE = 4       # resident copies of the headline batch the timed steps cycle over
KERNEL_SOURCES = ["paper_2512_15187_amd/csrc/gram_kernel.h", "paper_2512_15187_amd/csrc/device_common.h",
                  "paper_2512_15187_amd/csrc/k_gram.hip", "paper_2512_15187_amd/csrc/k_gram_f32.hip"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "gram_f16_2d_n256_m262144_traffic.txt")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic():
    """HBM bytes per launch of the gram kernel from the committed rocprofv3
    counter summary, if it was taken on the current kernel sources."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    for line in open(TRAFFIC_FILE):
        if "=" in line and not line.lstrip().startswith("#"):
            k, v = line.split("=", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_sources_sha256_16") != kernel_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def timed(fn, steps, warmup, torch, pid=None):
    """Seconds per call of fn over `steps` calls after `warmup` untimed ones.
    With `pid`, the library's kernel events are switched on (totals cleared)
    after the warm-up, so that the per-kernel averages leave out the first
    launches (which load the kernels)."""
    gc.collect()   # the previous legs' garbage is collected here, before the warm-up calls
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    if pid is not None:
        pid.pid_timing_enable(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def kernel_ms(pid, name):
    ms, n = pid.pid_timing_get(name)
    return (ms / n if n else float("nan")), n


def host_cpu():
    """(os.cpu_count(), CPU model name, BLAS libraries with their thread counts)."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    blas = []
    try:
        from threadpoolctl import threadpool_info
        blas = [dict(api=d.get("internal_api"), threads=d.get("num_threads")) for d in threadpool_info()]
    except Exception:
        pass
    return os.cpu_count(), model, blas


def cpu_baseline(U_host, budget_s=12.0):
    """The FP64 oracle (untuned) on the same step: all-pairs PID + PID-mean,
    with the BLAS threads it gets by default and with one thread."""
    import numpy as np
    import oracle
    ncpu, model, blas = host_cpu()
    threads = max([b["threads"] or 1 for b in blas] or [1])
    U64 = U_host.astype(np.float64)
    n, m = U64.shape
    reps, t_tot = 0, 0.0
    ref = refm = None
    while reps == 0 or (t_tot < budget_s and reps < 20):
        t0 = time.perf_counter()
        ref = oracle.pid(U64)
        refm = oracle.pid_mean(U64)
        t_tot += time.perf_counter() - t0
        reps += 1
    t = t_tot / reps
    t1 = None
    try:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            oracle.pid(U64)
            oracle.pid_mean(U64)
            t1 = time.perf_counter() - t0
    except Exception:
        pass
    return dict(value=n * n * m / t, unit="pair*points/s", cores=int(threads), kind="oracle",
                sample=f"the full workload ({n} x {m} FP64), all-pairs PID + PID-mean, mean of {reps} runs",
                value_1thread=(n * n * m / t1) if t1 else None, os_cpu_count=ncpu, cpu_model=model,
                blas=blas, seconds_per_step=t), ref, refm


def ranks_outside_ties(rank_gpu, depth_ref, tol):
    """Ranks agree with the oracle's up to permutations inside tie groups
    (oracle depths within 2*tol of each other, transitive closure)."""
    import numpy as np
    from oracle import rank_order
    rr, _ = rank_order(depth_ref)
    d = np.asarray(depth_ref)
    order = np.argsort(-d, kind="stable")
    groups, cur = [], [order[0]]
    for a, b in zip(order[:-1], order[1:]):
        if abs(d[a] - d[b]) <= 2 * tol:
            cur.append(b)
        else:
            groups.append(cur)
            cur = [b]
    groups.append(cur)
    return all(sorted(rank_gpu[g].tolist()) == sorted(rr[g].tolist()) for g in groups)


def headline(args):
    import numpy as np
    import torch

    import paper_2512_15187_amd as pid
    import synth

    dev = "cuda:0"
    log("generating the 2D soft-mask ensemble N=256 on 512x512 (FP32)")
    U, _ = synth.config1(device=dev)
    n, m = U.shape
    # The timed steps cycle over ROTATE resident copies of the batch (1.07 GB
    # in all, four times the 256 MB Infinity Cache), so that every step reads
    # its masks from HBM, as a stream of different batches would; one call
    # computes both depth kinds (PID-mean from the Gram row sums of the pass).
    copies = [U] + [U.clone() for _ in range(ROTATE - 1)]
    calls = [pid.PreparedCall("both", c, gemm="f16", inclusion=True) for c in copies]
    both = calls[0]
    k_step = [0]

    def step():
        calls[k_step[0] % ROTATE].run()
        k_step[0] += 1

    def same():
        both.run()

    log("timing the step")
    gc.collect()
    for _ in range(max(args.warmup, ROTATE)):
        step()
    torch.cuda.synchronize()
    # timed region: events bracket the dominant kernel only, on every
    # TIME_EVERY-th launch (an event pair costs several microseconds of a
    # step that is itself tens of microseconds)
    pid.pid_timing_select("gram")
    pid.pid_timing_sample(TIME_EVERY)
    pid.pid_timing_enable(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t_step = (time.perf_counter() - t0) / args.steps
    kt = {"gram": kernel_ms(pid, "gram")}
    pid.pid_timing_enable(False)
    pid.pid_timing_select(None)
    pid.pid_timing_sample(1)
    # per-kernel breakdown, outside the timed region
    pid.pid_timing_enable(True)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    breakdown = {k: kernel_ms(pid, k) for k in ("gram", "gram_reduce", "pairs_finish", "pidmean",
                                                 "pidmean_finalize", "rank")
                 if kernel_ms(pid, k)[1] > 0}
    pid.pid_timing_enable(False)
    # for context, outside the timed region: the same steps with no events,
    # and the step repeated on one batch (most of which then stays in the
    # Infinity Cache between steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t_plain = (time.perf_counter() - t1) / args.steps
    pid.pid_timing_select("gram")
    pid.pid_timing_enable(True)
    t2 = time.perf_counter()
    for _ in range(args.steps):
        same()
    torch.cuda.synchronize()
    t_same = (time.perf_counter() - t2) / args.steps
    warm = kernel_ms(pid, "gram")
    pid.pid_timing_enable(False)
    pid.pid_timing_select(None)
    log(f"step {t_step * 1e3:.3f} ms ({t_plain * 1e3:.3f} ms without kernel events); gram "
        f"{kt['gram'][0] * 1e3:.1f} us in the timed region; breakdown " +
        ", ".join(f"{k} {v[0] * 1e3:.1f} us" for k, v in breakdown.items()) +
        f"; one batch repeated: step {t_same * 1e3:.3f} ms, gram {warm[0] * 1e3:.1f} us")

    gram_ms = kt["gram"][0]
    algo_bytes = n * m * 4
    achieved = algo_bytes / (gram_ms * 1e-3) / 1e9
    roof = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBPS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBPS, 4), traffic=read_traffic(), kernel="gram (FP16 MFMA)",
                kernel_avg_us=round(gram_ms * 1e3, 2), algorithmic_bytes=algo_bytes,
                kernel_timed_launches=kt["gram"][1],
                timed_as=f"HIP events on every {TIME_EVERY}th launch of the timed steps, which cycle over "
                         f"{ROTATE} resident copies of the batch (no Infinity Cache reuse)")

    res_pairs = {k: v.clone() for k, v in both.out.items()}
    res_mean = {k: v.clone() for k, v in both.out_mean.items()}
    U_host = U.cpu().numpy()

    extra = {"kernel_us": {k: round(v[0] * 1e3, 2) for k, v in breakdown.items()},
             "step_us_without_kernel_events": round(t_plain * 1e6, 2),
             "one_batch_repeated_step_us": round(t_same * 1e6, 2),
             "one_batch_repeated_gram_us": round(warm[0] * 1e3, 2),
             "one_batch_repeated_gram_frac_hbm": round(algo_bytes / (warm[0] * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4)}
    cpu = None
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on the host")
        cpu, ref, refm = cpu_baseline(U_host)
        extra["depth_err_pairs_f16"] = float(np.max(np.abs(res_pairs["depth"].cpu().numpy() - ref["depth"])))
        extra["in_err_pairs_f16"] = float(max(np.max(np.abs(res_pairs["in_in"].cpu().numpy() - ref["in_in"])),
                                              np.max(np.abs(res_pairs["in_out"].cpu().numpy() - ref["in_out"]))))
        extra["inclusion_err_pairs_f16"] = float(np.max(np.abs(res_pairs["inclusion"].cpu().numpy() - ref["inclusion"])))
        extra["depth_err_mean"] = float(np.max(np.abs(res_mean["depth"].cpu().numpy() - refm["depth"])))
        from oracle import rank_order
        extra["ranks_equal_pairs"] = bool((res_pairs["rank"].cpu().numpy() == rank_order(ref["depth"])[0]).all())
        extra["ranks_equal_mean"] = bool((res_mean["rank"].cpu().numpy() == rank_order(refm["depth"])[0]).all())
        extra["ranks_equal_outside_ties_pairs"] = ranks_outside_ties(res_pairs["rank"].cpu().numpy(), ref["depth"], 1e-4)
        extra["ranks_equal_outside_ties_mean"] = ranks_outside_ties(res_mean["rank"].cpu().numpy(), refm["depth"], 1e-4)
        cpu.pop("seconds_per_step", None)

    if not args.no_extras:
        extra.update(side_measurements(pid, torch, np, synth, U, args, ref if cpu else None))
        extra["serving"] = serving_leg(pid, torch, synth, args.serve_requests)
        extra["sweep_sec52"] = sweep_rows(pid, torch, synth, SWEEP_SHAPES)

    line = {
        "metric": METRIC, "value": n * n * m / t_step, "unit": "pair*points/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": t_step * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f16", "data": "synthetic",
        "config": {"workload": "2D soft masks, N=256 on 512x512 (M=262144), FP32 masks; all-pairs PID "
                               "(FP16 MFMA Gram, FP64 normalisation) and PID-mean (from the Gram row sums) "
                               "from one call (pid_both: one pass over the masks), with both rankings; steps "
                               "cycle over 4 resident copies of the batch so that each reads HBM",
                   "n": n, "m": m, "scheme": "f16", "parallelism": "single GPU"},
        "roofline": roof, "cpu_baseline": cpu, "extra": extra,
    }
    print(json.dumps(line), flush=True)


def side_measurements(pid, torch, np, synth, U, args, ref):
    out = {}
    dev = "cuda:0"
    n, m = U.shape
    k = max(3, args.steps // 4)
    # FP32 comparator and BF16 split on the same ensemble
    for scheme in ("f32", "bf16_split", "bf16"):
        call = pid.PreparedCall("pairs", U, gemm=scheme)
        t = timed(call.run, k, 2, torch, pid)
        g, _ = kernel_ms(pid, "gram")
        pid.pid_timing_enable(False)
        out[f"pairs_{scheme}_pp_per_s"] = n * n * m / t
        out[f"gram_{scheme}_us"] = g * 1e3
        if ref is not None:
            out[f"depth_err_pairs_{scheme}"] = float(np.max(np.abs(call.out["depth"].cpu().numpy() - ref["depth"])))
    pf16 = pid.PreparedCall("pairs", U, gemm="f16")
    t16 = timed(pf16.run, k, 2, torch, pid)
    g16, _ = kernel_ms(pid, "gram")
    pid.pid_timing_enable(False)
    out["pairs_f16_pp_per_s"] = n * n * m / t16
    out["gram_f16_us"] = g16 * 1e3
    out["mfma_f16_vs_fp32_call"] = out["pairs_f16_pp_per_s"] / out["pairs_f32_pp_per_s"]
    out["mfma_f16_vs_fp32_gram"] = out["gram_f32_us"] / out["gram_f16_us"]
    out["mfma_bf16split_vs_fp32_gram"] = out["gram_f32_us"] / out["gram_bf16_split_us"]
    # issued MFMA utilisation of the split scheme (3 products per unique MAC on the upper sub-tiles)
    nbt = (n + 31) // 32
    sub_macs = nbt * (nbt + 1) // 2 * 1024 * m
    out["bf16_split_issued_tflops"] = 3 * 2 * sub_macs / (out["gram_bf16_split_us"] * 1e-6) / 1e12
    out["bf16_split_issued_frac_of_2500"] = out["bf16_split_issued_tflops"] / 2500.0
    out["f16_issued_tflops"] = 2 * sub_macs / (out["gram_f16_us"] * 1e-6) / 1e12

    # 3D PID-mean, N=64 FP16 on 256^3 with weights (HBM streaming)
    log("3D PID-mean workload N=64 on 256^3 (FP16 + FP32 weights)")
    U3, w3 = synth.config3(device=dev)
    n3, m3 = U3.shape
    call = pid.PreparedCall("mean", U3, w3)
    t = timed(call.run, max(5, args.steps // 2), 2, torch, pid)
    km, _ = kernel_ms(pid, "pidmean")
    pid.pid_timing_enable(False)
    b3 = n3 * m3 * 2 + m3 * 4
    out["mean3d_call_ms"] = t * 1e3
    out["mean3d_kernel_us"] = km * 1e3
    out["mean3d_GBps"] = b3 / (km * 1e-3) / 1e9
    out["mean3d_frac_hbm"] = out["mean3d_GBps"] / HBM_PEAK_GBPS
    out["mean3d_call_GBps"] = b3 / t / 1e9
    callu = pid.PreparedCall("mean", U3)
    timed(callu.run, max(5, args.steps // 2), 2, torch, pid)
    kmu, _ = kernel_ms(pid, "pidmean")
    pid.pid_timing_enable(False)
    out["mean3d_unweighted_GBps"] = n3 * m3 * 2 / (kmu * 1e-3) / 1e9
    # against a reliability-weighted mean contour: two streaming passes
    r3 = torch.linspace(0.5, 1.5, n3, dtype=torch.float64, device=dev)
    callw = pid.PreparedCall("weighted", U3, w3, member_weights=r3)
    tw = timed(callw.run, max(5, args.steps // 2), 2, torch)
    out["mean3d_reliability_weighted_call_ms"] = tw * 1e3
    out["mean3d_reliability_weighted_GBps_2_reads"] = 2 * b3 / tw / 1e9
    del U3, w3, call, callu, callw

    # scalar fields -> fuzzy contours, N=128 on 128^3, fused extraction
    log("scalar-field workload N=128 on 128^3 (FP32 fields, fused Phi)")
    F, iso = synth.config2(device=dev)
    nf, mf = F.shape
    giso = dict(kind="gaussian", c=iso["c"], sigma=iso["sigma"], side=iso["side"])
    siso = dict(kind="step", c=iso["c"], side=iso["side"])
    for name, call in (("fields_pairs_f16", pid.PreparedCall("pairs", F, iso=giso, gemm="f16")),
                       ("fields_pairs_i8", pid.PreparedCall("pairs", F, iso=siso, gemm="i8")),
                       ("fields_mean", pid.PreparedCall("mean", F, iso=giso)),
                       ("fields_mean_binary", pid.PreparedCall("mean", F, iso=siso))):
        t = timed(call.run, k, 2, torch, pid)
        # the kernels that read the fields: the Gram, the PID-mean pass, or
        # for the sharp isovalue the bit path's first pass (threshold, pack
        # and count; its row pass reads only the packed bits)
        binary_mean = name == "fields_mean_binary"
        kn = "gram" if "pairs" in name else ("pidmean_colsum" if binary_mean else "pidmean")
        kk, _ = kernel_ms(pid, kn)
        pid.pid_timing_enable(False)
        out[f"{name}_call_ms"] = t * 1e3
        gbps = nf * mf * 4 / (kk * 1e-3) / 1e9
        out[f"{name}_first_pass_GBps" if binary_mean else f"{name}_kernel_GBps"] = gbps
        out[f"{name}_frac_hbm"] = round(gbps / HBM_PEAK_GBPS, 4)
        if "pairs" in name:
            out[f"{name}_pp_per_s"] = nf * nf * mf / t
    # the further probability models on the same fields: ramp (uniform
    # isovalue), tent (level-centred map), normalised density; PID-mean and
    # the FP16 all-pairs call
    fmax = pid.pid_field_max(F).item()
    models = {"ramp": dict(kind="ramp", c=iso["c"], width=iso["sigma"] * 3 ** 0.5, side=iso["side"]),
              "tent": dict(kind="tent", c=iso["c"], width=2 * iso["sigma"]),
              "density": dict(kind="density", c=fmax)}
    for mname, miso in models.items():
        for variant, kn in (("mean", "pidmean"), ("pairs", "gram")):
            call = pid.PreparedCall(variant, F, iso=miso, gemm="f16")
            t = timed(call.run, k, 2, torch, pid)
            kk, _ = kernel_ms(pid, kn)
            pid.pid_timing_enable(False)
            out[f"fields_{variant}_{mname}_call_ms"] = t * 1e3
            gbps = nf * mf * 4 / (kk * 1e-3) / 1e9
            out[f"fields_{variant}_{mname}_kernel_GBps"] = gbps
            out[f"fields_{variant}_{mname}_frac_hbm"] = round(gbps / HBM_PEAK_GBPS, 4)
    del F

    out.update(large_n(pid, torch, synth, dev, k))

    # contour-boxplot bands on the headline ensemble: median, 50 % and 100 %
    # groups of its all-pairs ranking (reads the 256 rows once, writes M bytes)
    order = pid.pid_all_pairs(U, gemm="f16")["order"]
    t = timed(lambda: pid.pid_bands(U, order, n // 2, n, 0.5), k, 2, torch)
    pid.pid_timing_enable(True)          # after the warm-up (the first launch loads the kernel)
    timed(lambda: pid.pid_bands(U, order, n // 2, n, 0.5), k, 0, torch)
    kb, _ = kernel_ms(pid, "bands")
    pid.pid_timing_enable(False)
    out["bands_n256_m262144_call_us"] = t * 1e6
    out["bands_kernel_us"] = kb * 1e3
    out["bands_kernel_GBps"] = (n * m * 4 + m) / (kb * 1e-3) / 1e9

    # 2D FP64 plain PID, N=50 on 128x128
    U0, _ = synth.config0(device=dev)
    p0 = pid.PreparedCall("pairs", U0, gemm="f64")
    m0 = pid.PreparedCall("mean", U0)
    t = timed(lambda: (p0.run(), m0.run()), k, 2, torch)
    out["fp64_2d_n50_step_ms"] = t * 1e3
    return out


def percentile(xs, q):
    import numpy as np
    return float(np.percentile(np.asarray(xs), q)) if len(xs) else float("nan")


def run_server(pid, torch, pool, reqs, slots, arena_bytes):
    """Submit ``reqs`` at their arrival times to a server with ``slots``
    execution slots.  Latency = completion - arrival, both on the server's
    clock (a submitter that falls behind its arrivals counts against the
    server).  Returns latency percentiles (ms), requests/s over the span from
    the first arrival to the last completion, and the mean number of requests
    on the device at once (from the per-request device timestamps)."""
    srv = pid.PidServer(arena_bytes, max_slots=slots)
    torch.cuda.synchronize()
    tickets = []
    t0 = time.perf_counter()
    t0s = srv.pid_server_clock()
    for r in reqs:
        now = time.perf_counter() - t0
        if r.arrival_s > now:
            time.sleep(r.arrival_s - now)
        U = pool[(r.kind, r.side)][: r.n]
        t, _ = srv.pid_submit(U, variant=r.variant)
        tickets.append((r, t))
    lat, done, dev = [], [], []
    for r, t in tickets:
        st = srv.pid_wait(t)
        if st != pid.PID_OK:
            raise RuntimeError(f"request {r} failed: {srv.last_error()}")
        _, _, td = srv.pid_request_times(t)
        lat.append((td - (t0s + r.arrival_s)) * 1e3)
        done.append(td)
        dev.append(srv.pid_request_device_times(t))
        srv.release(t)
    srv.pid_server_destroy()
    n = len(lat)
    span = max(done) - (t0s + min(r.arrival_s for r in reqs))
    busy = sum(e - s for s, e in dev)
    dev_span = max(e for _, e in dev) - min(s for s, _ in dev)
    return dict(requests=n, slots=slots, p50_ms=percentile(lat, 50), p90_ms=percentile(lat, 90),
                p99_ms=percentile(lat, 99), mean_ms=float(sum(lat) / max(1, n)), max_ms=float(max(lat)),
                req_per_s=n / max(1e-9, span), mean_requests_on_device=busy / max(1e-9, dev_span))


def serving_pool_for(synth, torch, reqs, dev):
    keys = {}
    for r in reqs:
        keys[(r.kind, r.side)] = max(keys.get((r.kind, r.side), 0), r.n)
    pool = {k: synth.serving_pool(k[0], k[1], n_max, device=dev) for k, n_max in sorted(keys.items())}
    torch.cuda.synchronize()
    return pool


def serving_leg(pid, torch, synth, n_requests, rates=(200.0, None), slot_counts=(4, 1)):
    """Serving workload: Poisson arrivals of mixed requests (60 % 2D, N 32..512,
    128^2..1024^2; 40 % 3D, N 16..128, 64^3..192^3; FP16 soft masks; all-pairs
    or PID-mean 50/50), masks resident on the device, at each rate (req/s;
    None = every request arrives at once, the saturating case), with 4 slots
    (continuous batching) and 1 slot (one request at a time)."""
    dev = "cuda:0"
    base = synth.serving_requests(n_requests)
    log(f"serving: generating the request pool for {n_requests} requests")
    pool = serving_pool_for(synth, torch, base, dev)
    # every kernel variant of the mix runs once before anything is timed
    for r in base:
        U = pool[(r.kind, r.side)][: r.n]
        (pid.pid_all_pairs(U, inclusion=False) if r.variant == "pairs" else pid.pid_mean(U))
    torch.cuda.synchronize()
    arena = 4 << 30
    out = {}
    for rate in rates:
        reqs = synth.serving_requests(n_requests, rate_hz=rate) if rate else \
            [type(r)(r.rid, 0.0, r.kind, r.n, r.side, r.variant) for r in base]
        name = f"poisson_{int(rate)}_per_s" if rate else "burst"
        for slots in slot_counts:
            res = run_server(pid, torch, pool, reqs, slots, arena)
            log(f"serving {name}, {slots} slot(s): p50 {res['p50_ms']:.3f} ms, p99 {res['p99_ms']:.3f} ms, "
                f"{res['req_per_s']:.0f} req/s, {res['mean_requests_on_device']:.2f} requests on the device")
            out[f"{name}_slots{slots}"] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in res.items()}
    del pool
    torch.cuda.empty_cache()
    return out


def serve(args):
    import torch

    import paper_2512_15187_amd as pid
    import synth

    res = serving_leg(pid, torch, synth, args.requests, rates=(200.0, 1000.0, None))
    line = {
        "metric": METRIC, "value": res["poisson_200_per_s_slots4"]["p99_ms"], "unit": "ms (p99 latency)",
        "n_gpus": 1, "steps": args.requests, "warmup": 0,
        "ms_per_step": res["poisson_200_per_s_slots4"]["mean_ms"], "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f16", "data": "synthetic",
        "config": {"workload": "serving: Poisson 200 req/s (and 1000 req/s, and all at once); 60% 2D "
                               "(N 32..512, 128^2..1024^2), 40% 3D (N 16..128, 64^3..192^3), FP16 soft masks, "
                               "all-pairs / PID-mean 50/50; latency from arrival", "slots": 4},
        "serving": res,
    }
    print(json.dumps(line), flush=True)


def copy_calibration(args):
    """A plain device-to-device copy of 1 GiB (reads 1 GiB, writes 1 GiB), used
    to scale the FETCH_SIZE / WRITE_SIZE counters of rocprofv3 into bytes."""
    import torch
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    t = timed(lambda: dst.copy_(src), max(3, args.steps), 2, torch)
    print(json.dumps({"copy_bytes_read": 1 << 30, "copy_bytes_written": 1 << 30,
                      "copy_GBps_read_plus_write": 2 * (1 << 30) / t / 1e9}), flush=True)


# The paper's own GPU PID-mean timings on the same shapes (RTX 4080 Super; the
# paper does not say what they include), seconds, Sec. 5.2.
PAPER_SWEEP_GPU_S = {(10000, 50): 1.23, (20000, 50): 2.00, (50, 256): 2.36, (50, 352): 5.50}


def sweep_rows(pid, torch, synth, shapes, reps=5):
    """PID-mean of binary 3D ellipsoid ensembles (Sec. 5.2: 80 % normal, 20 %
    outlying members) as U8 masks and bit-packed (one bit per voxel), inputs
    resident in HBM; the results of the two layouts are compared bit for bit."""
    rows = []
    for n, res in shapes:
        U = synth.ellipsoids_3d(n, res, synth.BASE_SEED + 7 + n + res, device="cuda:0")
        m = res ** 3
        row = {"n": n, "res": res}
        for layout in ("u8", "packed"):
            if layout == "packed":
                P = pid.pid_pack_bits(U)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                pid.pid_pack_bits(U, out=P.words)
                torch.cuda.synchronize()
                row["pack_ms"] = round((time.perf_counter() - t0) * 1e3, 4)
                src = P
            else:
                src = U
            call = pid.PreparedCall("mean", src)
            t = timed(call.run, reps, 2, torch)
            pid.pid_timing_enable(True)
            timed(call.run, reps, 0, torch)
            kern = sum(kernel_ms(pid, k)[0] if kernel_ms(pid, k)[1] else 0.0
                       for k in ("pidmean_colsum", "pidmean", "pidmean_finalize"))
            pid.pid_timing_enable(False)
            nbytes = n * m if layout == "u8" else n * ((m + 31) // 32) * 4
            row[layout] = {"call_ms": round(t * 1e3, 4), "kernels_ms": round(kern, 4),
                           "member_voxels_per_s": n * m / t, "mask_GBps": nbytes / t / 1e9}
            row[layout + "_depth"] = call.out["depth"].clone()
            del call
        row["bitwise_equal"] = bool(torch.equal(row.pop("u8_depth"), row.pop("packed_depth")))
        if (n, res) in PAPER_SWEEP_GPU_S:
            row["paper_gpu_s"] = PAPER_SWEEP_GPU_S[(n, res)]
        log(f"sweep N={n} {res}^3: U8 {row['u8']['call_ms']:.3f} ms, packed {row['packed']['call_ms']:.3f} ms "
            f"(pack {row['pack_ms']:.3f} ms), equal={row['bitwise_equal']}")
        rows.append(row)
        del U, P, src
        torch.cuda.empty_cache()
    return rows


def large_n(pid, torch, synth, dev, k):
    """All-pairs depths without the matrix (streaming passes over the masks)
    against the FP16 Gram at a large N, where the Gram's N^2 M work
    dominates: N = 2048 on 256^2, FP16 masks."""
    log("large-N all-pairs depths: N=2048 on 256x256 (FP16 masks), Gram vs O(N M)")
    out = {}
    UL = synth.config1(device=dev, res=256, n=2048)[0].to(torch.float16)
    nl, ml = UL.shape
    gl = pid.PreparedCall("pairs", UL, gemm="f16")
    dl = pid.PreparedCall("depths", UL)
    tg = timed(gl.run, k, 2, torch)
    td = timed(dl.run, k, 2, torch)
    out["largeN_n2048_m65536_gram_f16_call_ms"] = tg * 1e3
    out["largeN_n2048_m65536_linear_call_ms"] = td * 1e3
    out["largeN_linear_speedup"] = tg / td
    # four reads of the masks: column sums and row sums (masses, IN_in), then
    # the column sums of u_j / m_j and the row sums against them
    out["largeN_linear_GBps_4_reads"] = 4 * nl * ml * 2 / td / 1e9
    out["largeN_max_depth_diff_linear_vs_gram"] = float((gl.out["depth"] - dl.out["depth"]).abs().max())
    del UL, gl, dl
    return out


def large_n_main(args):
    """The large-N leg alone (for a kernel trace of it); one JSON line."""
    import torch
    import paper_2512_15187_amd as pid
    import synth
    res = large_n(pid, torch, synth, "cuda:0", max(3, args.steps // 4))
    print(json.dumps({"metric": "all-pairs depths, N=2048 on 256^2 FP16 masks", "unit": "ms per call",
                      "data": "synthetic", **res}), flush=True)


SWEEP_SHAPES = [(n, 50) for n in (100, 1000, 10000, 20000, 40000)] + \
               [(50, r) for r in (128, 192, 256, 352, 512)]


def sweep(args):
    """The shapes of the paper's scalability study (Sec. 5.2): N from 100 to
    40,000 at 50^3 voxels, and 128^3 to 512^3 voxels at N = 50; one JSON line."""
    import torch
    import paper_2512_15187_amd as pid
    import synth
    rows = sweep_rows(pid, torch, synth, SWEEP_SHAPES)
    print(json.dumps({"metric": "PID-mean on binary 3D ellipsoid ensembles (Sec. 5.2 shapes)",
                      "unit": "ms per call", "dtype": "u8 / packed bits", "data": "synthetic", "rows": rows}),
          flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--mode", choices=["headline", "serve", "copycal", "sweep", "largen"], default="headline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--requests", type=int, default=2000, help="serve mode: requests per run")
    ap.add_argument("--serve-requests", type=int, default=400, help="requests per run of the serving leg")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the PID hot path is built and timed on a single "
              "MI355X; run it with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.mode == "serve":
        serve(args)
    elif args.mode == "copycal":
        copy_calibration(args)
    elif args.mode == "sweep":
        sweep(args)
    elif args.mode == "largen":
        large_n_main(args)
    else:
        headline(args)


if __name__ == "__main__":
    main()
