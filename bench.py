#!/usr/bin/env python3
"""Benchmark of the dual-quaternion Julia ray-march hot path on one MI355X.

One step = one pass of the whole path (march, bisection, normal, shade, write) over
the 1024x1024 workload: 3 seeded Julia constants, max_iter 24, 512 march steps,
10 bisection steps, all three frames in one persistent launch replayed from a HIP
graph. Inputs (parameters) are resident on the device before timing starts.

value = Julia iterations per second = I_alg / t, where I_alg is the number of
dual-quaternion updates the method runs for the three frames as counted by the
FP64 oracle (tests/golden/ialg_plain_1024.json), and t the wall time per step.
Each update is priced at 52 FP32 flops (37 for z^2 + c, 15 for the 8-square norm)
for the roofline against the FP32 vector peak.

Prints ONE JSON line. ``--gpus N`` with N > 1 exits: the benchmark runs on one GPU.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Julia iters/sec & % FP32 VALU peak; p50/p99 frame latency served vs plain"
FLOPS_PER_UPDATE = 52
FP32_PEAK_TFLOPS = 157.3          # MI355X FP32 vector peak
# Measured issue ceiling of v_fmac_f32 with vector-register operands on this GPU (no packed
# FP32): 2.87 clocks per wave64 instruction at the nominal 2.4 GHz, i.e. 128 flops per
# 1.196 ns per SIMD x 1024 SIMDs (profiles/gfx950_valu_issue.md).
FP32_FMAC_ISSUE_TFLOPS = 109.6

# HBM bytes per launch of the timed kernels, from rocprofv3 FETCH_SIZE and WRITE_SIZE runs
# (mean per dispatch), each scaled by what the counter reads for a 256 MiB device copy
# (profiles/render_refill_plain_1024.md, profiles/classify_grid_voxel_1024.md). A record
# belongs to the kernel sources it was measured on: bench.py reports it only while their
# hash is unchanged, else null.
TRAFFIC_RECORDS = {
    "plain": {
        "sources": ["paper_2303_14827_amd/csrc/render_refill.hip", "paper_2303_14827_amd/csrc/persist.h",
                    "paper_2303_14827_amd/csrc/qform.h",
                    "paper_2303_14827_amd/csrc/dq_device.h", "paper_2303_14827_amd/csrc/kparams.h",
                    "paper_2303_14827_amd/csrc/launch.h", "paper_2303_14827_amd/csrc/refill.h",
                    "paper_2303_14827_amd/csrc/tile_order.h",
                    "paper_2303_14827_amd/csrc/runtime_internal.h", "paper_2303_14827_amd/build.py",
                    "include/dqj.h"],
        "sources_sha256": "55664e1d07ba53540131593ecf89f7e0d9402b80ff34752ddccdbae8f57f532d",
        "fetch_kib": 100.23, "fetch_factor": 2.0, "write_kib": 38250.9, "write_factor": 1.0,
    },
    "voxel": {
        "sources": ["paper_2303_14827_amd/csrc/voxel.hip", "paper_2303_14827_amd/csrc/persist.h",
                    "paper_2303_14827_amd/csrc/qform.h",
                    "paper_2303_14827_amd/csrc/dq_device.h", "paper_2303_14827_amd/csrc/kparams.h",
                    "paper_2303_14827_amd/csrc/runtime_internal.h", "paper_2303_14827_amd/build.py",
                    "include/dqj.h"],
        "sources_sha256": "cd9e1af443f3142322565516528a323878029304a00b17a22d2c6d59e3dbf92a",
        "fetch_kib": 622.02, "fetch_factor": 2.0, "write_kib": 1336996.35, "write_factor": 1.0,
    },
}


def sources_sha256(which="plain"):
    import hashlib
    h = hashlib.sha256()
    for rel in TRAFFIC_RECORDS[which]["sources"]:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(rel.encode() + b"\0" + f.read())
    return h.hexdigest()


def recorded_traffic(which="plain"):
    """Bytes per launch of the timed kernel, or None if its sources changed since."""
    r = TRAFFIC_RECORDS[which]
    if sources_sha256(which) != r["sources_sha256"]:
        return None
    return (r["fetch_kib"] * r["fetch_factor"] + r["write_kib"] * r["write_factor"]) * 1024.0


def cpu_threads():
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        return int(env)
    return len(os.sched_getaffinity(0))


def cpu_baseline(ps, target_s):
    """The FP64 oracle on a bounded random sample of the same frames' pixels."""
    import numpy as np
    import oracle
    nthreads = cpu_threads()
    rng = np.random.default_rng(12345)
    # calibrate on a small sample, then size the sample to about target_s seconds
    pilot = [np.sort(rng.choice(p.width * p.height, 600, replace=False)) for p in ps]
    t = time.perf_counter()
    it = sum(oracle.render(p, pixels=pix, nthreads=nthreads)["total_iters"] for p, pix in zip(ps, pilot))
    rate_px = 600 * len(ps) / max(time.perf_counter() - t, 1e-6)
    per_frame = int(min(max(target_s * rate_px / len(ps), 1000), ps[0].width * ps[0].height))
    sample = [np.sort(rng.choice(p.width * p.height, per_frame, replace=False)) for p in ps]
    t = time.perf_counter()
    it = sum(oracle.render(p, pixels=pix, nthreads=nthreads)["total_iters"] for p, pix in zip(ps, sample))
    dt = time.perf_counter() - t
    return {"value": it / dt, "unit": "Julia iters/s", "cores": nthreads, "kind": "oracle",
            "sample": f"{per_frame} uniformly sampled pixels of each of the {len(ps)} frames "
                      f"({per_frame * len(ps)} rays, {it} updates, {dt:.1f} s, FP64)",
            "seconds": round(dt, 2)}


def cpu_one_thread_c1():
    """The FP64 oracle on one thread over the whole 128x128 plain frame (seed 0: max_iter 12,
    128 march steps, 8 bisection steps), the small configuration it finishes in a second."""
    import oracle
    import workloads
    p = workloads.plain_128(0)[0]
    t = time.perf_counter()
    it = oracle.render(p, nthreads=1)["total_iters"]
    dt = time.perf_counter() - t
    return {"value": it / dt, "unit": "Julia iters/s", "cores": 1, "kind": "oracle",
            "sample": f"the whole plain_128 frame, seed 0 ({p.pixels} rays, {it} updates, {dt:.2f} s, FP64)",
            "seconds": round(dt, 3)}


def with_clock(line, dqj):
    """Add the engine clock measured after the timed region (dqj_measure_engine_clock) and
    the fraction of the FP32 vector peak at that clock: 256 flop/clk per CU x CUs x clock.
    The headline `frac` stays against the nominal 157.3 TFLOP/s."""
    r = line.get("roofline")
    if not r or r.get("unit") != "TFLOP/s":
        return line
    try:
        mhz = dqj.measure_engine_clock(0.2)
    except Exception as e:   # the headline does not depend on it
        r["sclk_mhz_measured"] = None
        r["sclk_error"] = str(e)
        return line
    cus = dqj.device_info()["compute_units"]
    peak = 256.0 * cus * mhz * 1e-6
    r["sclk_mhz_measured"] = mhz
    r["peak_at_measured_sclk"] = peak
    r["frac_of_clock_adjusted_peak"] = r["achieved"] / peak
    return line


def progress(msg):
    """A progress line on stderr (stdout carries only the result line)."""
    print(f"bench.py: {msg}", file=sys.stderr, flush=True)


def _pct(xs, q):
    import numpy as np
    return float(np.quantile(np.asarray(xs), q)) if len(xs) else None


def _tail(recs, keys, q=0.99):
    """p50/p99 of the latency and, for the requests at or above the p99 latency, the mean
    of each latency component (ms) and their sizes."""
    import numpy as np
    lat = np.asarray([r["lat"] for r in recs])
    thr = float(np.quantile(lat, q))
    tail = [r for r in recs if r["lat"] >= thr]
    out = {"p50_ms": 1e3 * float(np.quantile(lat, 0.5)), "p99_ms": 1e3 * thr,
           "max_ms": 1e3 * float(lat.max()), "tail_requests": len(tail)}
    out["tail_mean_ms"] = {k: 1e3 * float(np.mean([r[k] for r in tail])) for k in ("lat",) + keys}
    sides = {}
    for r in tail:
        sides[r["side"]] = sides.get(r["side"], 0) + 1
    out["tail_sides"] = {str(k): v for k, v in sorted(sides.items())}
    out["tail_max_iter_mean"] = float(np.mean([r["max_iter"] for r in tail]))
    return out


def serve_bench(duration_s, rate_hz, capacity_n, dqj, workloads, torch, policy=None, slots=0,
                epoch_work=0.0):
    """The request stream replayed against the server (continuous batching; split
    precision, the stream's own, and FP32) and against the plain path (one FP32 dqj_render
    at a time, FIFO).

    Open loop: requests are submitted at their scheduled (Poisson) arrival times;
    latency = completion seen by the host - scheduled arrival. Served latency splits into
    admit wait (arrival to admission), first-launch wait (admission to the first epoch
    holding one of its tiles) and run (first launch to completion); plain latency into
    queue wait (arrival to the start of its render) and render. The p99 tail is reported
    with the mean of each component. Closed loop ("capacity"): the first capacity_n
    requests submitted back to back; throughput = requests, pixels and GPU-counted DQ
    updates over the makespan. The latency streams run without the update counter, as a
    production server would (the counting kernels are slower); the capacity runs count.
    """
    import threading
    import queue as q

    stream = workloads.serve_stream(duration_s=duration_s, rate_hz=rate_hz)
    policy = dqj.SERVE_FAIR if policy is None else policy

    def served(arrivals, open_loop, precision=workloads.PREC_SPLIT, count=False):
        srv = dqj.Server(precision=precision, count_iters=count, policy=policy, slots=slots,
                         epoch_work=epoch_work)
        pend = q.Queue()
        t0 = time.monotonic() + 0.05

        def submitter():
            cur = torch.cuda.current_stream()
            for a in arrivals:
                if open_loop:
                    dt = t0 + a.t - time.monotonic()
                    if dt > 0:
                        time.sleep(dt)
                out = dqj.alloc_outputs(a.params.width, a.params.height, extras=False)
                if count:
                    cur.synchronize()   # the zeroed work counter must be in place before the server adds to it
                else:
                    del out["iters"]
                p = a.params.replace(precision=precision)
                tk = srv.submit(p, out)
                pend.put((tk, (t0 + a.t) if open_loop else time.monotonic(), out, p))
            pend.put(None)

        th = threading.Thread(target=submitter)
        start = time.monotonic()
        th.start()
        recs, counters, pixels, n = [], [], 0, 0
        while True:
            item = pend.get()
            if item is None:
                break
            tk, t_arr, out, p = item
            r = srv.wait(tk)
            assert r["status"] == dqj.OK, r
            recs.append({"lat": r["t_done"] - t_arr, "admit_wait": r["t_admit"] - t_arr,
                         "first_launch_wait": r["t_first_launch"] - r["t_admit"],
                         "run": r["t_done"] - r["t_first_launch"], "side": p.width,
                         "max_iter": p.max_iter})
            if len(recs) % 2000 == 0:
                progress(f"served ({'split' if precision == workloads.PREC_SPLIT else 'FP32'}): "
                         f"{len(recs)} of {len(arrivals)} requests done")
            if count:
                counters.append(out["iters"])   # summed once at the end, off the critical path
            pixels += p.pixels
            n += 1
        th.join()
        end = time.monotonic()
        iters = int(torch.stack(counters).sum().item()) if count else None
        st = srv.stats()
        srv.close()
        return recs, iters, pixels, n, end - start, st

    def plain(arrivals, open_loop, count=False):
        s = torch.cuda.current_stream()
        t0 = time.monotonic() + 0.05
        recs, counters, pixels = [], [], 0
        start = time.monotonic()
        for a in arrivals:
            p = a.params.replace(precision=workloads.PREC_FP32)
            if open_loop:
                dt = t0 + a.t - time.monotonic()
                if dt > 0:
                    time.sleep(dt)
                t_arr = t0 + a.t
            else:
                t_arr = time.monotonic()
            out = dqj.alloc_outputs(p.width, p.height, extras=False)
            if not count:
                del out["iters"]
            t_start = time.monotonic()
            dqj.render(p, out=out, stream=s)
            s.synchronize()
            t_end = time.monotonic()
            recs.append({"lat": t_end - t_arr, "queue_wait": t_start - t_arr, "render": t_end - t_start,
                         "side": p.width, "max_iter": p.max_iter})
            if len(recs) % 2000 == 0:
                progress(f"plain: {len(recs)} of {len(arrivals)} requests done")
            if count:
                counters.append(out["iters"])
            pixels += p.pixels
        dur = time.monotonic() - start
        return recs, int(torch.stack(counters).sum().item()) if count else None, pixels, len(arrivals), dur

    served_keys = ("admit_wait", "first_launch_wait", "run")
    res = {"stream": f"Poisson {rate_hz:g} req/s for {duration_s:g} s ({len(stream)} requests), "
                     "side uniform over {128,256,512,1024,2048}, max_iter U[8,64], "
                     "march steps 16*max_iter, 10 bisection steps",
           "requests": len(stream),
           "policy": "oldest first" if policy == dqj.SERVE_OLDEST else "fair share",
           "slots": slots or 3, "epoch_work": epoch_work or 8e9,
           "latency_runs": "without the update counter; capacity runs count"}
    progress(f"serve stream of {len(stream)} requests: split server, FP32 server, plain")
    sr, si, sp, sn, sdur, sst = served(stream, True)
    res["served"] = {"precision": "split (FP16 march, FP32 re-check and bisection, FP64 re-bisection)",
                     **_tail(sr, served_keys), "epochs": sst["epochs"]}
    fr, fi, fp, fn, fdur, fst = served(stream, True, workloads.PREC_FP32)
    res["served_fp32"] = {"precision": "FP32 (the plain path's kernels, continuously batched)",
                          **_tail(fr, served_keys), "epochs": fst["epochs"]}
    pr, pi, pp, pn, pdur = plain(stream, True)
    res["plain"] = {"precision": "FP32, one request at a time, FIFO",
                    **_tail(pr, ("queue_wait", "render"))}
    progress(f"capacity: {capacity_n} requests back to back, each way")
    cap = stream[:capacity_n]
    cl, ci, cp, cn, cdur, _ = served(cap, False, count=True)
    gl, gi, gp, gn, gdur, _ = served(cap, False, workloads.PREC_FP32, count=True)
    ql, qi, qp, qn, qdur = plain(cap, False, count=True)
    res["capacity"] = {
        "requests": cn,
        "served": {"req_per_s": cn / cdur, "mpix_per_s": cp / cdur / 1e6,
                   "iters_per_s": ci / cdur, "makespan_s": cdur},
        "served_fp32": {"req_per_s": gn / gdur, "mpix_per_s": gp / gdur / 1e6,
                        "iters_per_s": gi / gdur, "makespan_s": gdur},
        "plain": {"req_per_s": qn / qdur, "mpix_per_s": qp / qdur / 1e6,
                  "iters_per_s": qi / qdur, "makespan_s": qdur},
        "note": "iters = DQ updates counted on the GPU (split: FP16 march through the first "
                "inside sample + FP32 re-check/bisection/normal + FP64 re-bisection; plain: "
                "the method's count in FP32)"}
    return res


def frame_error(p, g, pixels, oracle_mod):
    """Error of one GPU frame against the FP64 oracle on the listed pixels."""
    import numpy as np
    import workloads
    o = oracle_mod.render(p, pixels=pixels)
    gm = g["mask"].reshape(-1)[pixels].astype(bool)
    om = o["mask"].astype(bool)
    gd = g["depth"].reshape(-1)[pixels].astype(np.float64)
    gs = g["shade"].reshape(-1)[pixels].astype(np.float64)
    E = workloads.scene_extent(p)
    both = gm & om
    dd = np.zeros(len(pixels))
    dd[both] = np.abs(gd[both] - o["depth"][both])   # (misses hold +inf)
    agree = (~gm & ~om) | (both & (dd <= 1e-4 * E))
    ok = both & agree
    ds = np.abs(gs - o["shade"])[ok]
    return {"pixels": int(len(pixels)), "mask_agree": float(agree.mean()),
            "mask_disagree_pixels": int((gm != om).sum()),
            "hits_gpu": int(gm.sum()), "hits_oracle": int(om.sum()),
            "depth_err_max_E": float(dd[ok].max() / E) if ok.any() else 0.0,
            "depth_err_mean_E": float(dd[ok].mean() / E) if ok.any() else 0.0,
            "shade_err_max": float(ds.max()) if ok.any() else 0.0,
            "shade_within_1_255": float((ds <= 1 / 255).mean()) if ok.any() else 1.0}


def timed_plan(dqj, torch, ps, outs, steps, warmup, schedule=None):
    stream = torch.cuda.current_stream()
    plan = dqj.BatchPlan(ps, outs, schedule=schedule)
    for _ in range(warmup):
        plan.launch(stream)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    times = []
    for _ in range(steps):
        e0.record(stream)
        plan.launch(stream)
        e1.record(stream)
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    plan.close()
    return times


def bench_split(args, dqj, workloads, torch):
    import numpy as np
    import oracle
    ps = workloads.split_1080p()
    outs = [dqj.alloc_outputs(p.width, p.height, extras=True) for p in ps]
    # work counters from one counting launch outside the timing
    cplan = dqj.BatchPlan(ps, outs)
    cplan.launch()
    torch.cuda.synchronize()
    split_iters = sum(int(o["iters"].item()) for o in outs)
    cplan.close()
    timed = [{k: v for k, v in o.items() if k != "iters"} for o in outs]
    t_split = timed_plan(dqj, torch, ps, timed, args.steps, args.warmup)
    fp64_rays = [int(((o["flags"] & dqj.FLAG_FP64) != 0).sum().item()) for o in outs]
    hits = [int(o["mask"].sum().item()) for o in outs]
    # the FP32 path on the same frames
    ps32 = [p.replace(precision=workloads.PREC_FP32) for p in ps]
    outs32 = [dqj.alloc_outputs(p.width, p.height, extras=False) for p in ps32]
    c32 = dqj.BatchPlan(ps32, outs32)
    c32.launch()
    torch.cuda.synchronize()
    fp32_iters = sum(int(o["iters"].item()) for o in outs32)
    c32.close()
    t_fp32 = timed_plan(dqj, torch, ps32, [{k: v for k, v in o.items() if k != "iters"} for o in outs32],
                        args.steps, args.warmup)
    # error of every frame against the FP64 oracle on sampled pixels (uniform + GPU hits),
    # for the split form and for the FP32 path on the same pixels
    rng = np.random.default_rng(7)
    errors, errors32 = [], []
    for p, o, o32 in zip(ps, outs, outs32):
        g = {k: v.cpu().numpy() for k, v in o.items()}
        g32 = {k: v.cpu().numpy() for k, v in o32.items()}
        pix = rng.choice(p.pixels, args.error_pixels, replace=False)
        h = np.nonzero(g["mask"].reshape(-1))[0]
        if h.size:
            pix = np.union1d(pix, rng.choice(h, min(h.size, args.error_pixels // 2), replace=False))
        pix = np.sort(pix)
        errors.append(frame_error(p, g, pix, oracle))
        errors32.append(frame_error(p, g32, pix, oracle))
    ms_split = float(np.median(t_split))
    ms_fp32 = float(np.median(t_fp32))
    # the FP32 path's count is the method's update count (its FP32 classification)
    return {
        "metric": METRIC, "value": fp32_iters / (ms_split * 1e-3), "unit": "Julia iters/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_split,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f16/f32/f64",
        "data": "synthetic",
        "config": {"workload": "split_1080p: 8 seeded c, 1920x1080, max_iter 32, packed-FP16 "
                               "512-step march, FP32 12-step bisection, FP64 re-bisection of rays "
                               "whose FP32 window (+-2 samples) flips; one graph-replayed launch",
                   "frames": 8},
        "value_note": "method updates (FP32 path's count) per second of the split launch",
        "split": {"ms_per_step": ms_split, "gpu_counted_updates": split_iters,
                  "fp64_rays_per_frame": fp64_rays, "hits_per_frame": hits},
        "fp32_same_frames": {"ms_per_step": ms_fp32, "updates": fp32_iters,
                             "iters_per_s": fp32_iters / (ms_fp32 * 1e-3)},
        "speedup_vs_fp32": ms_fp32 / ms_split,
        "pct_fp32_peak_equiv": 100.0 * FLOPS_PER_UPDATE * fp32_iters / (ms_split * 1e-3) / 1e12 / FP32_PEAK_TFLOPS,
        "error_vs_fp64_oracle": errors,
        "fp32_error_vs_fp64_oracle": errors32,
    }


def bench_sweep(args, dqj, workloads, torch):
    import numpy as np
    import oracle
    n = args.sweep_frames
    ps = workloads.sweep_256(n)
    outs = [dqj.alloc_outputs(p.width, p.height, extras=False) for p in ps]
    tune_n = min(64, n)
    best = dqj.autotune(ps[:tune_n], outs[:tune_n])
    for o in outs[:tune_n]:
        o["iters"].zero_()           # the tuning launches counted into these
    torch.cuda.synchronize()
    sched = {"tile_w": best.tile_w, "tile_h": best.tile_h, "waves_per_block": best.waves_per_block,
             "blocks_per_cu": best.blocks_per_cu}
    cplan = dqj.BatchPlan(ps, outs)          # uses the autotuned schedule
    cplan.launch()
    torch.cuda.synchronize()
    counts = torch.stack([o["iters"] for o in outs]).cpu().numpy().reshape(-1)
    iters = int(counts.sum())
    cplan.close()
    timed = [{k: v for k, v in o.items() if k != "iters"} for o in outs]
    t = timed_plan(dqj, torch, ps, timed, args.steps, args.warmup)
    ms = float(np.median(t))
    # cross-check of the GPU-counted work with the oracle on the first frames
    k = min(args.sweep_oracle_frames, n)
    t0 = time.perf_counter()
    ora = [oracle.render(p, nthreads=cpu_threads())["total_iters"] for p in ps[:k]]
    cpu_s = time.perf_counter() - t0
    achieved = FLOPS_PER_UPDATE * iters / (ms * 1e-3) / 1e12
    return {
        "metric": METRIC, "value": iters / (ms * 1e-3), "unit": "Julia iters/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"sweep_256: {n} seeded c (real comps U[-0.8,0.8]), each 256x256, "
                               "max_iter 16, 256 march steps, 8 bisection steps, one persistent "
                               "graph-replayed launch, autotuned schedule", "frames": n,
                   "schedule": sched},
        "pct_fp32_peak": 100.0 * achieved / FP32_PEAK_TFLOPS,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP32_PEAK_TFLOPS, "traffic": None},
        "ialg_source": "GPU-counted method updates (FP32 classification)",
        "oracle_check": {"frames": k, "gpu_counted": int(counts[:k].sum()), "oracle": int(sum(ora)),
                         "rel_diff": abs(int(counts[:k].sum()) - sum(ora)) / max(1, sum(ora))},
        "cpu_baseline": {"value": sum(ora) / cpu_s, "unit": "Julia iters/s", "cores": cpu_threads(),
                         "kind": "oracle", "sample": f"the first {k} frames in full "
                         f"({sum(ora)} updates, {cpu_s:.1f} s, FP64)"},
    }


def bench_de(args, dqj, workloads, torch):
    """plain_1024's three frames marched by distance estimates (FP32): one graph-replayed
    launch per step of the one-thread-per-pixel kernel over the three frames, against the
    FP64 oracle's count of the updates that march runs (tests/golden/ialg_de_1024.json).
    Each DE update also carries the derivative norm: 2 more flops than the fixed march's
    52. The per-frame launches of the three DE kernels are timed beside it."""
    ps = workloads.de_1024()
    with open(os.path.join(ROOT, "tests", "golden", "ialg_de_1024.json")) as f:
        ialg = json.load(f)["total_iters"]
    stream = torch.cuda.current_stream()
    outs = [dqj.alloc_outputs(p.width, p.height, extras=False) for p in ps]
    count_plan = dqj.BatchPlan(ps, outs)
    count_plan.launch(stream)
    torch.cuda.synchronize()
    counted = sum(int(o["iters"].item()) for o in outs)
    count_plan.close()
    timed = [{k: v for k, v in o.items() if k != "iters"} for o in outs]

    def run(step, steps, warmup):
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        for _ in range(steps):
            step()
        e1.record(stream)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / steps, e0.elapsed_time(e1) / steps

    def per_frame(kernel):
        sched = dqj.make_schedule(kernel=kernel)

        def step():
            for p, o in zip(ps, timed):
                dqj.render(p, out=o, stream=stream, schedule=sched)
        return step

    others = {}
    for name, kern in [("render_de_kernel, one dqj_render per frame", dqj.KERNEL_DIRECT),
                       ("render_de_refill_kernel, one dqj_render per frame", dqj.KERNEL_REFILL),
                       ("render_de_lockstep_kernel, one dqj_render per frame", dqj.KERNEL_LOCKSTEP)]:
        oms, oev = run(per_frame(kern), max(1, args.steps // 4), 2)
        others[name] = {"ms_per_step": oms, "kernel_ms_per_step": oev, "value": ialg / (oms * 1e-3)}
    plan = dqj.BatchPlan(ps, timed)
    ms, ev_ms = run(lambda: plan.launch(stream), args.steps, args.warmup)
    plan.close()
    flops = FLOPS_PER_UPDATE + 2
    achieved = flops * ialg / (ev_ms * 1e-3) / 1e12
    line = {
        "metric": METRIC, "value": ialg / (ms * 1e-3), "unit": "Julia iters/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "de_1024: plain_1024's 3 frames marched by distance estimates "
                               "(at most 512 steps, hit below 1e-4, steps in [1e-4, 0.25], "
                               "10 bisection steps), one graph-replayed launch per step",
                   "frames": 3, "width": 1024, "height": 1024, "max_iter": 24},
        "pct_fp32_peak": 100.0 * achieved / FP32_PEAK_TFLOPS,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP32_PEAK_TFLOPS, "traffic": None,
                     "kernel": "render_de_batch_kernel", "kernel_ms_per_step": ev_ms,
                     "flops_per_update": flops,
                     "frac_of_measured_fmac_issue": achieved / FP32_FMAC_ISSUE_TFLOPS},
        "other_kernels": others,
        "ialg_per_step": ialg, "ialg_source": "FP64 oracle, tests/golden/ialg_de_1024.json",
        "gpu_counted_iters_per_step": counted,
        "hits_per_frame": [int(o["mask"].sum().item()) for o in outs],
    }
    if not args.no_cpu:
        progress("CPU baseline: the FP64 oracle on the host cores")
        line["cpu_baseline"] = cpu_baseline(ps, args.cpu_seconds)
    return line


def bench_project(args, dqj, workloads, torch):
    """Projection ("shadow") rendering: three 512x512 frames of the paper's constants,
    each point's fibre sampled by 16 offsets, as one graph-replayed batch launch (the
    frames' blocks interleaved; 4 lanes per pixel), against the FP64 oracle's count of the
    updates the render runs (tests/golden/ialg_project_512.json). The three frames as
    single dqj_render launches are timed beside it."""
    ps = workloads.project_512()
    with open(os.path.join(ROOT, "tests", "golden", "ialg_project_512.json")) as f:
        ialg = json.load(f)["total_iters"]
    stream = torch.cuda.current_stream()
    outs = [dqj.alloc_outputs(p.width, p.height, extras=False) for p in ps]
    cplan = dqj.BatchPlan(ps, outs)
    cplan.launch()
    torch.cuda.synchronize()
    cplan.close()
    counted = sum(int(o["iters"].item()) for o in outs)
    timed = [{k: v for k, v in o.items() if k != "iters"} for o in outs]
    plan = dqj.BatchPlan(ps, timed)

    def timed_loop(step, steps, warmup):
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        for _ in range(steps):
            step()
        e1.record(stream)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / steps, e0.elapsed_time(e1) / steps

    ms, ev_ms = timed_loop(lambda: plan.launch(stream), args.steps, args.warmup)

    def singles():
        for p, o in zip(ps, timed):
            dqj.render(p, out=o, stream=stream)
    single_ms, _ = timed_loop(singles, max(1, args.steps // 4), 2)
    plan.close()
    achieved = FLOPS_PER_UPDATE * ialg / (ev_ms * 1e-3) / 1e12
    line = {
        "metric": METRIC, "value": ialg / (ms * 1e-3), "unit": "Julia iters/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "project_512: 3 frames of 512x512, the shadows of the sets of "
                               "the paper's constants PAPER_C[7], [0], [4] (max_iter 15, 256 "
                               "march steps, 10 bisection steps), each fibre sampled by 16 "
                               "offsets; one graph-replayed batch launch per step",
                   "frames": 3, "width": 512, "height": 512, "max_iter": 15, "fibers": 16,
                   "single_launches_ms_per_step": single_ms},
        "pct_fp32_peak": 100.0 * achieved / FP32_PEAK_TFLOPS,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP32_PEAK_TFLOPS, "traffic": None,
                     "kernel": "render_project_batch_kernel", "kernel_ms_per_step": ev_ms,
                     "flops_per_update": FLOPS_PER_UPDATE,
                     "frac_of_measured_fmac_issue": achieved / FP32_FMAC_ISSUE_TFLOPS},
        "ialg_per_step": ialg, "ialg_source": "FP64 oracle, tests/golden/ialg_project_512.json",
        "gpu_counted_iters_per_step": counted,
        "hits_per_frame": [int(o["mask"].sum().item()) for o in outs],
    }
    if not args.no_cpu:
        progress("CPU baseline: the FP64 oracle on the host cores")
        line["cpu_baseline"] = cpu_baseline(ps, args.cpu_seconds)
    return line


def bench_voxel(args, dqj, workloads, torch):
    """Dense voxel-grid classification (dqj_classify_grid): the 1024^3 voxel centres of
    the box for the paper's high-detail constant (max_iter 15), against the FP64 oracle's
    count of the updates classification runs (tests/golden/ialg_voxel_1024.json)."""
    import numpy as np
    p, dims = workloads.voxel_1024()
    with open(os.path.join(ROOT, "tests", "golden", "ialg_voxel_1024.json")) as f:
        gold = json.load(f)
    assert [round(x, 7) for x in gold["c"]] == [round(x, 7) for x in p.c], "golden/c mismatch"
    ialg = int(gold["total_iters"])
    nvox = int(np.prod(dims))
    stream = torch.cuda.current_stream()
    mask = torch.empty(dims[::-1], dtype=torch.uint8, device="cuda")
    iters = torch.zeros((1,), dtype=torch.int64, device="cuda")
    dqj.classify_grid(p, *dims, mask=mask, iters=iters, stream=stream)
    torch.cuda.synchronize()
    counted = int(iters.item())
    inside = int(mask.sum().item())
    for _ in range(args.warmup):
        dqj.classify_grid(p, *dims, mask=mask, stream=stream)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        dqj.classify_grid(p, *dims, mask=mask, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    ev_ms = e0.elapsed_time(e1) / args.steps
    achieved = FLOPS_PER_UPDATE * ialg / (ev_ms * 1e-3) / 1e12
    line = {
        "metric": METRIC, "value": ialg / (ms * 1e-3), "unit": "Julia iters/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "voxel_1024: the 1024^3 voxel centres of the box [-1.5, 1.5]^3, "
                               "identity slice, the paper's high-detail constant, max_iter 15, "
                               "one dqj_classify_grid per step",
                   "nx": dims[0], "ny": dims[1], "nz": dims[2], "max_iter": p.max_iter},
        "voxels_per_s": nvox / (ms * 1e-3),
        "pct_fp32_peak": 100.0 * achieved / FP32_PEAK_TFLOPS,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP32_PEAK_TFLOPS,
                     "traffic": recorded_traffic("voxel"),
                     "kernel": "classify_grid_kernel", "kernel_ms_per_step": ev_ms,
                     "flops_per_update": FLOPS_PER_UPDATE,
                     "algorithmic_bytes_per_launch": nvox,
                     "frac_of_measured_fmac_issue": achieved / FP32_FMAC_ISSUE_TFLOPS},
        "ialg_per_step": ialg, "ialg_source": "FP64 oracle, tests/golden/ialg_voxel_1024.json",
        "gpu_counted_iters_per_step": counted, "inside_voxels": inside,
        "inside_voxels_oracle": int(gold["inside"]),
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline_grid(p, dims, args.cpu_seconds)
    return line


def cpu_baseline_grid(p, dims, target_s):
    """The FP64 oracle on a bounded random sample of the grid's voxels."""
    import numpy as np
    import oracle
    nthreads = cpu_threads()
    rng = np.random.default_rng(12345)
    n = int(np.prod(dims))
    pilot = np.sort(rng.integers(0, n, 200000))
    t = time.perf_counter()
    oracle.classify_grid(p, *dims, voxels=pilot, nthreads=nthreads)
    rate = pilot.size / max(time.perf_counter() - t, 1e-6)
    k = int(min(max(target_s * rate, 100000), 64 * 1024 * 1024))
    sample = np.sort(rng.integers(0, n, k))
    t = time.perf_counter()
    it = oracle.classify_grid(p, *dims, voxels=sample, nthreads=nthreads)["total_iters"]
    dt = time.perf_counter() - t
    return {"value": it / dt, "unit": "Julia iters/s", "cores": nthreads, "kind": "oracle",
            "sample": f"{k} uniformly sampled voxels of the {dims[0]}x{dims[1]}x{dims[2]} grid "
                      f"({it} updates, {dt:.1f} s, FP64)", "seconds": round(dt, 2)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--kernel", choices=["refill", "direct"], default="refill")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="length of the served request stream (0: skip)")
    ap.add_argument("--serve-policy", choices=["fair", "oldest"], default="fair")
    ap.add_argument("--serve-slots", type=int, default=0, help="epoch slots (0: the library default)")
    ap.add_argument("--serve-epoch-work", type=float, default=0.0,
                    help="estimated DQ updates per epoch (0: the library default, 8e9)")
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--capacity-requests", type=int, default=300)
    ap.add_argument("--workload", choices=["plain_1024", "split_1080p", "sweep_256", "de_1024",
                                           "voxel_1024", "project_512"],
                    default="plain_1024")
    ap.add_argument("--error-pixels", type=int, default=4000)
    ap.add_argument("--sweep-frames", type=int, default=4096)
    ap.add_argument("--sweep-oracle-frames", type=int, default=16)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first run one device copy of this many MiB (a known-size kernel that "
                         "calibrates hardware byte counters under a profiler)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU; --gpus {args.gpus} is not supported "
              "(every pixel, frame and request is independent: see the sharding design)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2303_14827_amd as dqj
    import workloads

    if args.copy_probe_mib > 0:
        src = torch.ones(args.copy_probe_mib << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    if args.workload != "plain_1024":
        torch.cuda.set_device(0)
        fn = {"split_1080p": bench_split, "sweep_256": bench_sweep, "de_1024": bench_de,
              "voxel_1024": bench_voxel, "project_512": bench_project}[args.workload]
        print(json.dumps(with_clock(fn(args, dqj, workloads, torch), dqj)), flush=True)
        return

    ps = workloads.plain_1024()
    golden_path = os.path.join(ROOT, "tests", "golden", "ialg_plain_1024.json")
    with open(golden_path) as f:
        golden = json.load(f)
    for fr, p in zip(golden["frames"], ps):
        assert [round(x, 7) for x in fr["c"]] == [round(x, 7) for x in p.c], "golden/c mismatch"
    ialg = int(golden["total_iters"])

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    info = dqj.device_info(0)
    stream = torch.cuda.current_stream()
    outs = [dqj.alloc_outputs(p.width, p.height, extras=False) for p in ps]
    # The work counter is a diagnostic output: timed launches leave it off (the kernel
    # variant without the per-sample add), one extra launch outside the timing fills it.
    # The timed launches write buffers of their own, compared bit for bit with the
    # counting launch's after the timing.
    timed_outs = [{k: v for k, v in dqj.alloc_outputs(p.width, p.height, extras=False).items()
                   if k != "iters"} for p in ps]

    if args.kernel == "refill":
        count_plan = dqj.BatchPlan(ps, outs)
        count_plan.launch(stream)
        torch.cuda.synchronize()
        exec_iters = sum(int(o["iters"].item()) for o in outs)
        count_plan.close()
        plan = dqj.BatchPlan(ps, timed_outs)

        def step():
            plan.launch(stream)
    else:
        sched = dqj.make_schedule(kernel=dqj.KERNEL_DIRECT)

        for p, o in zip(ps, outs):
            dqj.render(p, out=o, stream=stream, schedule=sched)
        torch.cuda.synchronize()
        exec_iters = sum(int(o["iters"].item()) for o in outs)

        def step():
            for p, o in zip(ps, timed_outs):
                dqj.render(p, out=o, stream=stream, schedule=sched)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = e0.elapsed_time(e1) / args.steps
    ms_per_step = wall * 1e3 / args.steps
    hits = [int(o["mask"].sum().item()) for o in outs]
    for f, (t, o) in enumerate(zip(timed_outs, outs)):
        for k in ("mask", "depth", "shade"):
            if not torch.equal(t[k], o[k]):
                raise SystemExit(f"bench.py: timed output {k} of frame {f} differs from the "
                                 "counting launch's")

    value = ialg / (ms_per_step * 1e-3)
    achieved_tf = FLOPS_PER_UPDATE * ialg / (ev_ms * 1e-3) / 1e12
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "Julia iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "plain_1024: 3 seeded c (seeds 0,1,2; real comps U[-0.6,0.6], "
                               "dual U[-0.5,0.5]), 1024x1024, max_iter 24, escape radius 4, "
                               "512 march steps, 10 bisection steps, one graph-replayed "
                               "persistent launch per step",
                   "frames": 3, "width": 1024, "height": 1024, "max_iter": 24,
                   "march_steps": 512, "bisect_steps": 10, "kernel": args.kernel},
        "pct_fp32_peak": 100.0 * achieved_tf / FP32_PEAK_TFLOPS,
        "roofline": {"bound": "alu", "achieved": achieved_tf, "peak": FP32_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved_tf / FP32_PEAK_TFLOPS,
                     "traffic": recorded_traffic() if args.kernel == "refill" else None,
                     "kernel": "render_refill_batch_kernel" if args.kernel == "refill" else
                               "render_direct_kernel",
                     "kernel_ms_per_launch": ev_ms,
                     "flops_per_launch": FLOPS_PER_UPDATE * ialg,
                     "frac_of_measured_fmac_issue": achieved_tf / FP32_FMAC_ISSUE_TFLOPS},
        "ialg_per_step": ialg,
        "ialg_source": "FP64 oracle, tests/golden/ialg_plain_1024.json",
        "gpu_counted_iters_per_step": exec_iters,
        "hits_per_frame": hits,
        "device": {"arch": info["arch"], "cus": info["compute_units"],
                   "clock_mhz": info["clock_khz"] / 1000.0},
    }
    if args.serve_seconds > 0:
        line["serve"] = serve_bench(args.serve_seconds, args.serve_rate, args.capacity_requests,
                                    dqj, workloads, torch,
                                    dqj.SERVE_OLDEST if args.serve_policy == "oldest" else dqj.SERVE_FAIR,
                                    args.serve_slots, args.serve_epoch_work)
    if not args.no_cpu:
        progress("CPU baseline: the FP64 oracle on the host cores")
        line["cpu_baseline"] = cpu_baseline(ps, args.cpu_seconds)
        line["cpu_baseline"]["one_thread_plain_128"] = cpu_one_thread_c1()
    if args.kernel == "refill":
        plan.close()
    print(json.dumps(with_clock(line, dqj)), flush=True)


if __name__ == "__main__":
    main()
