"""Throughput bench of the register-state dataflow analysis on one MI355X.

One step = the whole hot path over one batch: decode and checks, leaders,
block numbering, edges and predecessor lists, reverse postorder, fixpoint,
extraction and dense compaction, on 65,536 seeded synthetic GCN kernels with
lengths log-uniform on [200, 2000] (51.2M instructions, 820 MB of records)
already resident in HBM.  Prints one JSON line.

Beside the headline figure it reports the plain form (each kernel analysed
by its own launch sequence) on a sample, and the request server at Poisson
arrivals (latency percentiles, served rate, the same requests offline).

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-serving] [--copy-calibration]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
# the request server runs one lane per HIP hardware queue (one queue per
# lane keeps a long batch from holding up another lane's); must be set before
# the HIP runtime starts
os.environ["GPU_MAX_HW_QUEUES"] = "16"

METRIC = "instructions analysed/sec to fixpoint (bit-exact) + HBM GB/s fraction; p99 latency"
HBM_PEAK_GBS = 8000.0
PROFILE = os.path.join(ROOT, "profiles", "k_fixpoint_c2_65536_kernels.md")
FIXPOINT_SRC = os.path.join(ROOT, "paper_2107_07809_amd", "csrc", "dc_fixpoint.hip")


def measured_traffic():
    """HBM bytes per launch of the fixpoint kernel from the committed rocprofv3
    summary (FETCH_SIZE + WRITE_SIZE, calibrated by a 1 GiB copy), or None when
    the kernel source has changed since the counters were taken."""
    import hashlib
    try:
        text = open(PROFILE).read()
        src = hashlib.sha256(open(FIXPOINT_SRC, "rb").read()).hexdigest()
    except OSError:
        return None
    fields = dict(line.split(": ", 1) for line in text.splitlines()
                  if line.startswith(("traffic_bytes_per_launch: ", "measured_source_sha256: ")))
    if fields.get("measured_source_sha256", "").strip() != src:
        return None
    return float(fields["traffic_bytes_per_launch"])


def log(msg):
    print("bench: " + msg, file=sys.stderr, flush=True)


def cpu_baseline(cfg, n_kernels, target_core_seconds=15.0):
    """The oracle as it stands, one worker process per available core, on a
    bounded sample (a prefix of the same workload)."""
    import dcgen
    from concurrent.futures import ProcessPoolExecutor
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from gpu_common import _oracle_chunk
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    cores = max(1, min(cores, 16))
    # size the sample from a quick single-core probe
    probe = dcgen.generate(cfg, 256, threads=1)
    t = time.perf_counter()
    _oracle_chunk((cfg, 0, 256))
    rate1 = probe.n_instr / (time.perf_counter() - t)
    mean_len = probe.n_instr / 256
    n = int(min(n_kernels, max(256, target_core_seconds * rate1 / mean_len)))
    step = max(1, n // (cores * 8))
    jobs = [(cfg, i, min(step, n - i)) for i in range(0, n, step)]
    lens, _ = dcgen.sizes(cfg, 0, n)
    n_instr = int(lens.sum())
    with ProcessPoolExecutor(cores) as ex:
        list(ex.map(_oracle_chunk, [(cfg, 0, 16)] * cores))   # start the workers
        t = time.perf_counter()
        list(ex.map(_oracle_chunk, jobs))
        dt = time.perf_counter() - t
    return {"value": n_instr / dt, "unit": "instructions/s", "cores": cores, "kind": "oracle",
            "sample": f"first {n} of the {n_kernels} kernels ({n_instr} instructions, regenerated per worker "
                      f"shard, generation inside the timed span); single-core rate {rate1:.4g} instructions/s",
            "seconds": dt}


def plain_per_kernel(ctx, b, dev, stream, n_sample):
    """The plain form for comparison: every kernel analysed by its own
    sequence of launches (its own batch of one), one after another, on the
    first n_sample kernels of the same workload.  Planning and allocation
    happen before the timed region, as for the batched form."""
    import torch
    from paper_2107_07809_amd import dc
    batches = []
    n_instr = 0
    for k in range(n_sample):
        d = b.kernels[k:k + 1].copy()
        ab, na = int(d["arg_begin"][0]), int(d["n_args"][0])
        d["arg_begin"] = 0
        batches.append(ctx.analyze(d, dev, b.n_instr, b.args[ab:ab + na], stream=stream))
        n_instr += int(d["n_instr"][0])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for bt in batches:
        bt.run(stream=stream)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    for bt in batches:
        bt.free()
    return {"value": n_instr / dt, "unit": "instructions/s", "sample": f"first {n_sample} kernels of the same "
            f"workload ({n_instr} instructions), one launch sequence per kernel", "seconds": dt}


def serving(ctx, rate, seconds, warm_seconds=0.3, offline=True, **server_opts):
    """The request server at Poisson arrivals (log-normal lengths, median
    1,000 instructions, sigma 1, cap 100k): offered and served rates, latency
    from submission to result on the host, and the same requests analysed
    as one offline batch."""
    import dcgen
    from paper_2107_07809_amd import dc
    n_warm = int(rate * warm_seconds)
    n = int(rate * seconds)
    b = dcgen.generate(5, n_warm + n)
    reqs = dc.requests(b.kernels, b.instrs, b.args)
    due = np.cumsum(np.random.default_rng(0xD1C5A11E).exponential(1.0 / rate, n_warm + n))
    srv = dc.Server(ctx, **server_opts)
    stride = dc.REQUEST_DTYPE.itemsize
    base = reqs.ctypes.data
    done = []
    t0 = time.perf_counter()
    i = 0
    while i < n_warm + n:
        now = time.perf_counter() - t0
        while i < n_warm + n and due[i] <= now:
            srv.submit_raw(base + i * stride)
            i += 1
        res, _ = srv.poll(8192, records=False)
        if len(res):
            done.append(res)
    deadline = time.perf_counter() + 60
    while sum(len(x) for x in done) < n_warm + n and time.perf_counter() < deadline:
        res, _ = srv.poll(8192, records=False)
        if len(res):
            done.append(res)
        else:
            time.sleep(0.0002)
    st = srv.stats()
    srv.close()
    res = np.concatenate(done)
    res = res[res["tag"] >= n_warm]           # measured window: after the warm-up arrivals
    lat = (res["t_done_ns"] - res["t_submit_ns"]) / 1e6
    instr = int(b.kernels["n_instr"][n_warm:].sum())
    span = (res["t_done_ns"].max() - res["t_submit_ns"].min()) / 1e9
    offered = len(res) / ((res["t_submit_ns"].max() - res["t_submit_ns"].min()) / 1e9)
    failed = int((res["summary"]["status"] != 0).sum())

    def med(x):
        return float(np.percentile(x.astype(np.float64), 50) / 1e6)
    out = {}
    if offline:
        out["offline_batch_instructions_per_s"] = offline_rate(ctx, b.subset(np.arange(n_warm, n_warm + n)))
    return {"requests": int(len(res)), "completed_all": bool(len(res) == n), "failed": failed,
            "offered_per_s": offered, "offered_target_per_s": rate,
            "instructions": instr, "served_instructions_per_s": instr / span,
            "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                           "max": float(lat.max())},
            "stage_ms_p50": {"wait": med(res["t_admit_ns"] - res["t_submit_ns"]),
                             "pack": med(res["t_enqueued_ns"] - res["t_admit_ns"]),
                             "device": med(res["t_device_ns"] - res["t_enqueued_ns"]),
                             "copy_back": med(res["t_done_ns"] - res["t_device_ns"])},
            "batches": int(len(np.unique(res["batch"]))), "mean_batch": float(res["batch_kernels"].mean()),
            "lanes": st["lanes"], **out,
            "workload": f"{n} log-normal requests (median 1,000 instructions, sigma 1, cap 100k) at Poisson "
                        f"arrivals after {n_warm} warm-up arrivals"}


def offline_rate(ctx, off):
    """Instructions/s of one dc_analyze_batch run over the same requests."""
    import torch
    from paper_2107_07809_amd import dc
    dev = dc.to_device(off.instrs)
    stream = torch.cuda.current_stream()
    bt = ctx.analyze(off.kernels, dev, off.n_instr, off.args, stream=stream)
    bt.wait()
    torch.cuda.synchronize()
    t = time.perf_counter()
    bt.run(stream=stream)
    torch.cuda.synchronize()
    off_rate = off.n_instr / (time.perf_counter() - t)
    bt.free()
    del dev
    return off_rate


def timed_batch(ctx, b, stream, reps=1):
    """Plan once (untimed, with its first run), then time `reps` whole runs
    with the records resident in HBM."""
    import torch
    from paper_2107_07809_amd import dc
    dev = dc.to_device(b.instrs)
    bt = ctx.analyze(b.kernels, dev, b.n_instr, b.args, flags=dc.OPT_TIMING, stream=stream)
    bt.wait()
    res = bt.results()
    st = bt.stats()
    bt.timing_reset()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        bt.run(stream=stream)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / reps
    tm = bt.timing()
    bt.free()
    del dev
    torch.cuda.empty_cache()
    return dt, tm["ms_fixpoint"] / max(1, tm["runs"]), res, st


def other_workloads(ctx, stream, c3_slices=8):
    """The other configurations, each timed as whole-path runs with its
    records in HBM: the 16 kernels of 1-4M instructions; the 1,048,576-kernel
    Zipf workload in slices of 131,072 kernels (one plan per slice, the
    slices' run times summed); the 32-kernel workload batched and as one
    launch sequence per kernel."""
    import dcgen
    out = {}
    b = dcgen.generate(4, 16)
    dt, fix, res, st = timed_batch(ctx, b, stream)
    out["c4_16_kernels_1M_to_4M"] = {"instructions": int(b.n_instr), "seconds": dt, "instructions_per_s": b.n_instr / dt,
                                     "sweeps_max": st["sweeps_max"], "blocks_max": int(res["n_blocks"].max()),
                                     "failed": int((res["status"] != 0).sum()),
                                     "form": "one wavefront per kernel (overflow pass)"}
    log("workloads: 16 huge kernels done")
    per = 1048576 // c3_slices
    tot_s = tot_i = fail = 0
    for k in range(c3_slices):
        b = dcgen.generate(3, per, i0=k * per)
        dt, fix, res, st = timed_batch(ctx, b, stream)
        tot_s += dt
        tot_i += int(b.n_instr)
        fail += int((res["status"] != 0).sum())
        log(f"workloads: Zipf slice {k + 1}/{c3_slices}: {b.n_instr} instructions in {dt * 1e3:.1f} ms")
    out["c3_zipf_1048576_kernels"] = {"instructions": tot_i, "seconds": tot_s, "instructions_per_s": tot_i / tot_s,
                                      "failed": fail, "form": f"{c3_slices} slices of {per} kernels, batched persistent"}
    b = dcgen.generate(1, 32)
    dt, fix, res, st = timed_batch(ctx, b, stream, reps=20)
    plain = plain_per_kernel(ctx, b, dc_dev(b), stream, 32)
    out["c1_32_kernels"] = {"instructions": int(b.n_instr), "batched_instructions_per_s": b.n_instr / dt,
                            "plain_instructions_per_s": plain["value"], "batched_ms": dt * 1e3}
    return out


def dc_dev(b):
    from paper_2107_07809_amd import dc
    return dc.to_device(b.instrs)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--kernels", type=int, default=65536)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one 1 GiB device copy first (a known-size reference for HBM counters)")
    ap.add_argument("--waves-per-group", type=int, default=0)
    ap.add_argument("--groups-per-cu", type=int, default=0)
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the library's default launch shape instead of dc_autotune's (also when a shape is given)")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serve-rate", type=float, default=50000.0)
    ap.add_argument("--serve-seconds", type=float, default=2.0)
    ap.add_argument("--plain-sample", type=int, default=256)
    ap.add_argument("--workloads", action="store_true",
                    help="also time the 16 huge kernels, the 1,048,576-kernel Zipf workload and the 32-kernel one")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    import torch
    import dcgen
    from paper_2107_07809_amd import dc

    cfg = 2
    t = time.perf_counter()
    b = dcgen.generate(cfg, args.kernels)
    log(f"generated {b.n_kernels} kernels, {b.n_instr} instructions in {time.perf_counter() - t:.2f}s")
    dev = dc.to_device(b.instrs)
    stream = torch.cuda.current_stream()
    if args.copy_calibration:
        src = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("copy calibration: 1 GiB device-to-device copy done")
    ctx = dc.Context(0)
    shape = {"waves_per_group": args.waves_per_group, "groups_per_cu": args.groups_per_cu}
    tuned = False
    if not args.no_autotune and not (args.waves_per_group or args.groups_per_cu):
        # launch shape from the autotuner on a sample (outside the timed region)
        shape, tune_ms = ctx.autotune(b.kernels, dev, b.n_instr, b.args, sample=8192, stream=stream)
        tuned = True
        log(f"autotune: {shape} ({tune_ms:.2f} ms per run of the sample)")
    batch = ctx.analyze(b.kernels, dev, b.n_instr, b.args, flags=dc.OPT_TIMING, stream=stream, **shape)
    for _ in range(max(0, args.warmup - 1)):
        batch.run(stream=stream)
    batch.wait()
    res = batch.results()
    n_failed = int((res["status"] != 0).sum())
    n_acc, n_sys = int(res["n_access"].sum()), int(res["n_sysval"].sum())
    st = batch.stats()
    log(f"warmup done: failed={n_failed} sweeps max={st['sweeps_max']} overflow={st['n_overflow']}")

    # timed region: K steps, each one whole pass of the hot path
    batch.timing_reset()
    step_ms = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        batch.run(stream=stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tm = batch.timing()
    elapsed = t1 - t0
    # per-step device time from the events of each run (for latency percentiles)
    ms_per_step = elapsed * 1e3 / args.steps
    value = b.n_instr * args.steps / elapsed
    fix_ms = tm["ms_fixpoint"] / max(1, tm["runs"])
    total_ms = tm["ms_total"] / max(1, tm["runs"])
    # algorithmic bytes of the fixpoint kernel per launch: every record read
    # once, descriptors, the access/system-value records and results written
    alg_bytes = 16 * b.n_instr + 32 * b.n_kernels + 16 * n_acc + 8 * n_sys + 32 * b.n_kernels
    achieved = alg_bytes / (fix_ms * 1e-3) / 1e9
    traffic_bytes = measured_traffic()
    traffic = traffic_bytes / (fix_ms * 1e-3) / 1e9 if traffic_bytes else None
    # per-run latencies from a second, short pass with one sync per step
    lat = []
    for _ in range(min(args.steps, 20)):
        t = time.perf_counter()
        batch.run(stream=stream)
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - t) * 1e3)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "instructions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "65,536 seeded synthetic GCN kernels, lengths log-uniform on [200, 2000], nested "
                               "exec-mask if/else and counted loops to depth 3, ~18% float ALU",
                   "kernels": b.n_kernels, "instructions": b.n_instr, "record_bytes": 16 * b.n_instr,
                   "form": "batched persistent (one wavefront per kernel)",
                   "launch": {**shape, "autotuned": tuned}},
        "roofline": {"bound": "hbm", "kernel": "k_fixpoint", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "alg_bytes_per_launch": alg_bytes, "traffic_bytes_per_launch": traffic_bytes,
                     "avg_launch_ms": fix_ms},
        "stages_ms": {"total": total_ms, "decode": tm["ms_decode"] / max(1, tm["runs"]),
                      "cfg": tm["ms_cfg"] / max(1, tm["runs"]), "fixpoint": fix_ms,
                      "compact": tm["ms_compact"] / max(1, tm["runs"])},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
        "sweeps": {"max": st["sweeps_max"], "mean": st["sweeps_sum"] / max(1, b.n_kernels - n_failed)},
        "failed_kernels": n_failed,
    }
    batch.free()
    if args.plain_sample:
        log(f"plain form: {args.plain_sample} kernels, one launch sequence each")
        out["plain_per_kernel"] = plain_per_kernel(ctx, b, dev, stream, args.plain_sample)
        out["plain_per_kernel"]["batched_speedup"] = value / out["plain_per_kernel"]["value"]
    del dev
    if args.workloads:
        out["workloads"] = other_workloads(ctx, stream)
    if not args.no_serving:
        log(f"serving: {args.serve_rate:.0f} requests/s for {args.serve_seconds} s")
        out["serving"] = serving(ctx, args.serve_rate, args.serve_seconds)
    ctx.close()
    if not args.no_cpu:
        log("timing the CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(cfg, args.kernels)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
