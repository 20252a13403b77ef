"""Throughput bench of the register-state dataflow analysis on one MI355X.

One step = the whole hot path over one batch: decode and checks, leaders,
block numbering, record regions, edges and predecessor lists, reverse
postorder, fixpoint, extraction and dense compaction.  The headline workload
is 1,048,576 seeded synthetic GCN kernels with Zipf(1.2) lengths on
[20, 20000] (1.74e9 instructions, 27.8 GB of records) in one persistent
launch, records resident in HBM.  Prints one JSON line.

Beside the headline figure it reports: the 65,536-kernel log-uniform
workload; the 16 kernels of 1-4M instructions (sweeps and GB/s); the
32-kernel workload batched and in the plain form (each kernel analysed by its
own launch sequence); the request server at Poisson arrivals (latency
percentiles, served rate, the same requests offline); and the CPU oracle on
a length-stratified sample of the headline workload, whose results also
check the timed run's results for the sampled kernels.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-serving] [--no-extra] [--copy-calibration]
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "instructions analysed/sec to fixpoint (bit-exact) + HBM GB/s fraction; p99 latency"
HBM_PEAK_GBS = 8000.0
N_CU = 256
CLOCK_GHZ = 2.4
PROFILE = os.path.join(ROOT, "profiles", "k_fixpoint_zipf_1048576_kernels.md")
# the fixpoint kernel's source: the per-kernel core and the persistent kernel
FIXPOINT_SRC = [os.path.join(ROOT, "paper_2107_07809_amd", "csrc", f) for f in ("dc_fixpoint_core.h", "dc_fixpoint.hip")]
WORKLOADS = {
    3: ("1,048,576 seeded synthetic GCN kernels, Zipf(s=1.2) lengths on [20, 20000], nested exec-mask if/else "
        "and counted loops to depth 3, ~18% float ALU", 1048576),
    2: ("65,536 seeded synthetic GCN kernels, lengths log-uniform on [200, 2000], nested exec-mask if/else and "
        "counted loops to depth 3, ~18% float ALU", 65536),
}


def log(msg):
    print("bench: " + msg, file=sys.stderr, flush=True)


def profile_fields():
    """Per-launch counter figures of the fixpoint kernel from the committed
    rocprofv3 summary, or {} when the kernel source has changed since the
    counters were taken."""
    try:
        text = open(PROFILE).read()
        src = hashlib.sha256(b"".join(open(f, "rb").read() for f in FIXPOINT_SRC)).hexdigest()
    except OSError:
        return {}
    fields = dict(line.split(": ", 1) for line in text.splitlines() if ": " in line and line[:1].islower())
    if fields.get("measured_source_sha256", "").strip() != src:
        return {}
    out = {}
    for k, v in fields.items():
        try:
            out[k] = float(v)
        except ValueError:
            pass
    return out


# ---------------------------------------------------------------- CPU leg

def _oracle_job(job):
    """One worker's share of the sample: generate its kernels (untimed), then
    time the oracle over them."""
    import dcgen
    import oracle
    cfg, idx = job
    b = dcgen.concat([dcgen.generate(cfg, 1, i0=int(i), threads=1).kernel(0) for i in idx])
    t = time.perf_counter()
    summ, acc, sysv = oracle.analyze_batch(b)
    dt = time.perf_counter() - t
    return dt, int(b.n_instr), summ, acc, sysv


def stratified_sample(cfg, n_kernels, fraction):
    """Every (1/fraction)-th kernel in order of length: a length-stratified
    sample of the workload's kernel indices, ascending."""
    import dcgen
    lens, _ = dcgen.sizes(cfg, 0, n_kernels)
    order = np.argsort(lens, kind="stable")
    step = max(1, int(round(1.0 / fraction)))
    return np.sort(order[step // 2::step]), lens


def cpu_baseline(cfg, n_kernels, idx, lens):
    """The oracle as it stands, one single-threaded worker process per core of
    this process's CPU share, on the sampled kernels; every worker gets an
    equal share of each length stratum and is timed on the oracle alone."""
    from concurrent.futures import ProcessPoolExecutor
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    # a one-GPU host grants that GPU's process 16 cores, whatever the machine shows
    cores = max(1, min(avail, 16))
    jobs = [(cfg, idx[w::cores]) for w in range(cores)]
    with ProcessPoolExecutor(cores) as ex:
        parts = list(ex.map(_oracle_job, jobs))
    secs = [p[0] for p in parts]
    n_instr = sum(p[1] for p in parts)
    total_instr = int(lens.sum(dtype=np.uint64))
    value = n_instr / max(secs)
    per_core = n_instr / sum(secs)
    # results back in sample order (worker w holds idx[w::cores])
    by_kernel = {}
    for w, p in enumerate(parts):
        summ, acc, sysv = p[2], p[3], p[4]
        ia = isy = 0
        for j, k in enumerate(idx[w::cores]):
            na, ns = int(summ[j]["n_acc"]), int(summ[j]["n_sys"])
            by_kernel[int(k)] = (summ[j], acc[ia:ia + na], sysv[isy:isy + ns])
            ia += na
            isy += ns
    out = {"value": value, "unit": "instructions/s", "cores": cores, "kind": "oracle",
           "sample": f"{len(idx)} of the {n_kernels} kernels, every {n_kernels // max(1, len(idx))}th in order of "
                     f"length ({n_instr} instructions, {100.0 * n_instr / total_instr:.2f}% of the workload's "
                     f"{total_instr}); value = sample instructions / the longest worker's oracle seconds "
                     f"(generation untimed); the whole workload would take {total_instr / value:.0f} s",
           "per_core_value": per_core, "seconds": max(secs), "host_cpus": os.cpu_count(), "cpu_share": avail}
    return out, by_kernel


def verify_sample(gpu, by_kernel):
    """The timed run's results of the sampled kernels against the oracle:
    status, blocks, sweeps, record counts and every record byte."""
    bad = 0
    for k, (s, acc, sysv) in by_kernel.items():
        r = gpu["results"][k]
        ok = (int(r["status"]), int(r["n_blocks"]), int(r["sweeps"]), int(r["n_access"]), int(r["n_sysval"])) == \
            (int(s["status"]), int(s["n_blocks"]), int(s["sweeps"]), int(s["n_acc"]), int(s["n_sys"]))
        ga, gs = gpu["records"][k]
        ok = ok and ga.tobytes() == acc.tobytes() and gs.tobytes() == sysv.tobytes()
        bad += 0 if ok else 1
    return {"kernels": len(by_kernel), "mismatches": bad}


# ---------------------------------------------------------------- GPU legs

def timed_run(ctx, b, stream, steps, warmup, shape, sample_idx=None, lat_steps=5, what="batch"):
    """Plan once (with its first run, untimed), `warmup` more runs, then time
    `steps` whole-path runs with the records resident in HBM.  Returns the
    figures, the per-kernel results and, for sample_idx, those kernels'
    records."""
    import torch
    from paper_2107_07809_amd import dc
    t = time.perf_counter()
    dev = dc.to_device(b.instrs)
    torch.cuda.synchronize()
    log(f"{what}: records uploaded in {time.perf_counter() - t:.1f}s")
    t = time.perf_counter()
    bt = ctx.analyze(b.kernels, dev, b.n_instr, b.args, flags=dc.OPT_TIMING, stream=stream, **shape)
    bt.wait()
    log(f"{what}: planned and first run in {time.perf_counter() - t:.1f}s")
    for _ in range(warmup):
        bt.run(stream=stream)
    bt.wait()
    res = bt.results()
    st = bt.stats()
    bt.timing_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        bt.run(stream=stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    tm = bt.timing()
    runs = max(1, tm["runs"])
    lat = []
    for _ in range(lat_steps):
        t = time.perf_counter()
        bt.run(stream=stream)
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - t) * 1e3)
    res_after = bt.results()
    records = {}
    if sample_idx is not None:
        for k in sample_idx:
            records[int(k)] = (bt.accesses(int(k)), bt.sysvals(int(k)))
    bt.free()
    del dev
    torch.cuda.empty_cache()
    n_failed = int((res["status"] != 0).sum())
    n_acc, n_sys = int(res["n_access"].sum()), int(res["n_sysval"].sum())
    fix_ms = tm["ms_fixpoint"] / runs
    alg_bytes = 16 * b.n_instr + 32 * b.n_kernels + 16 * n_acc + 8 * n_sys + 32 * b.n_kernels
    return {
        "elapsed": elapsed, "value": b.n_instr * steps / elapsed, "ms_per_step": elapsed * 1e3 / steps,
        "fix_ms": fix_ms, "alg_bytes": alg_bytes,
        "stages_ms": {"total": tm["ms_total"] / runs, "decode": tm["ms_decode"] / runs, "cfg": tm["ms_cfg"] / runs,
                      "fixpoint": fix_ms, "compact": tm["ms_compact"] / runs},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))} if lat else None,
        "sweeps": {"max": st["sweeps_max"], "mean": st["sweeps_sum"] / max(1, b.n_kernels - n_failed)},
        "failed": n_failed, "overflow_kernels": st["n_overflow"],
        "rerun_identical": bool(res_after.tobytes() == res.tobytes()),
        "results": res, "records": records,
    }


def plain_per_kernel(ctx, b, stream, n_sample, reps=3):
    """The plain form for comparison (DC_OPT_PLAIN): one launch per kernel, in
    which one workgroup runs every stage of that kernel, one launch after
    another, on the first n_sample kernels.  Planning happens before the
    timed region."""
    import torch
    from paper_2107_07809_amd import dc
    sub = b.subset(np.arange(n_sample))
    dev = dc.to_device(sub.instrs)
    bt = ctx.analyze(sub.kernels, dev, sub.n_instr, sub.args, flags=dc.OPT_PLAIN, stream=stream)
    bt.wait()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        bt.run(stream=stream)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    failed = int((bt.results()["status"] != 0).sum())
    bt.free()
    return {"value": sub.n_instr / dt, "unit": "instructions/s", "kernels": n_sample, "instructions": int(sub.n_instr),
            "seconds": dt, "failed": failed, "form": "one launch per kernel (DC_OPT_PLAIN)"}


def graph_replay_ms(ctx, b, stream, reps=50):
    """Milliseconds per run of the batch when its stages replay as one captured
    HIP graph (DC_OPT_GRAPH), beside the eager runs: on a small batch the
    launches are a visible share of a run."""
    import torch
    from paper_2107_07809_amd import dc
    dev = dc.to_device(b.instrs)
    bt = ctx.analyze(b.kernels, dev, b.n_instr, b.args, flags=dc.OPT_GRAPH, stream=stream)
    bt.run(stream=stream)
    bt.wait()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        bt.run(stream=stream)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t) * 1e3 / reps
    bt.free()
    return ms


def stage_roofline(alg_bytes, ms, kernel):
    """HBM roofline of one stage: its algorithmic bytes over its time by the
    HIP events, against MI355X's 8 TB/s."""
    if not ms:
        return None
    gbs = alg_bytes / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": kernel, "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": gbs / HBM_PEAK_GBS}


def ssa_workload(ctx, b, stream, steps=5, cpu_kernels=2048):
    """Register versions (dc_build_ssa) of a workload: whole runs (the graph
    stages, then the version stages) with the records in HBM; the version
    stages' time from HIP events on the same stream; the oracle's versions on
    one core over the first cpu_kernels kernels."""
    import torch
    import oracle
    from paper_2107_07809_amd import dc
    dev = dc.to_device(b.instrs)
    # the digests of one run are checked against the oracle on a sample; the
    # timed object computes none (as a caller that wants the versions would)
    s = ctx.build_ssa(b.kernels, dev, b.n_instr, digest=True, stream=stream)
    dig = s.results()
    s.free()
    s = ctx.build_ssa(b.kernels, dev, b.n_instr, timing=True, digest=False, stream=stream)
    s.run()
    s.wait()
    res0 = s.results()
    s.timing_reset()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        s.run()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / steps
    tm = s.timing()
    res = s.results()
    s.free()
    ok = res["status"] == 0
    ssa_ms = tm["ms_fixpoint"] / max(1, tm["runs"])
    alg = (16 * b.n_instr + b.n_instr + 4 * int(res["n_operands"].sum()) + 12 * int(res["n_phi"].sum()) +
           4 * int(res["n_phi_args"].sum()) + 4 * int(res["n_blocks"].sum()) + 32 * b.n_kernels)
    sub = b.subset(np.arange(min(cpu_kernels, b.n_kernels)))
    t = time.perf_counter()
    osum = oracle.ssa_batch(sub)
    cpu_dt = time.perf_counter() - t
    return {"instructions_per_s": b.n_instr / dt, "ms_per_step": dt * 1e3, "ssa_stages_ms": ssa_ms,
            "graph_stages_ms": (tm["ms_decode"] + tm["ms_cfg"]) / max(1, tm["runs"]),
            "merges": int(res["n_phi"].sum()), "merge_args": int(res["n_phi_args"].sum()),
            "operand_versions": int(res["n_operands"].sum()), "failed": int((~ok).sum()),
            "rerun_identical": bool(res.tobytes() == res0.tobytes()),
            "sample_matches_oracle": bool(dig[:sub.n_kernels]["digest"].tobytes() == osum["digest"].tobytes()),
            "counts_match_digest_run": bool(np.array_equal(dig["n_operands"], res["n_operands"]) and
                                            np.array_equal(dig["n_phi"], res["n_phi"])),
            "alg_bytes": alg, "ssa_stages_GBps": alg / (ssa_ms * 1e-3) / 1e9 if ssa_ms else None,
            "roofline": stage_roofline(alg, ssa_ms, "k_ssa_graph + k_ssa_emit"),
            "cpu_oracle": {"instructions_per_s": sub.n_instr / cpu_dt, "cores": 1, "kernels": sub.n_kernels}}


def types_workload(ctx, b, stream, steps=5, cpu_kernels=2048):
    """Variables and types over the register versions (dc_build_types) of a
    workload: whole runs (graph stages, version stages, type stage) with the
    records in HBM; the type stage's time from HIP events on the same stream;
    the oracle on one core over the first cpu_kernels kernels."""
    import torch
    import oracle
    from paper_2107_07809_amd import dc
    dev = dc.to_device(b.instrs)
    t = ctx.build_types(b.kernels, dev, b.n_instr, b.args, digest=True, stream=stream)
    dig = t.types()
    t.free()
    t = ctx.build_types(b.kernels, dev, b.n_instr, b.args, timing=True, digest=False, stream=stream)
    t.run()
    t.wait()
    res0 = t.types()
    t.timing_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        t.run()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    tm = t.timing()
    res = t.types()
    sres = t.results()
    t.free()
    ok = res["status"] == 0
    runs = max(1, tm["runs"])
    ty_ms = tm["ms_compact"] / runs
    nodes = int(res["n_nodes"].sum())
    # the type stage reads the records, operand versions, merges and their
    # arguments, and writes 16 B per node
    alg = (16 * b.n_instr + 4 * int(sres["n_operands"].sum()) + 16 * int(sres["n_phi"].sum()) +
           4 * int(sres["n_phi_args"].sum()) + 16 * nodes + 32 * b.n_kernels)
    sub = b.subset(np.arange(min(cpu_kernels, b.n_kernels)))
    t0 = time.perf_counter()
    osum = oracle.types_batch(sub)
    cpu_dt = time.perf_counter() - t0
    return {"instructions_per_s": b.n_instr / dt, "ms_per_step": dt * 1e3, "type_stage_ms": ty_ms,
            "version_stages_ms": tm["ms_fixpoint"] / runs,
            "graph_stages_ms": (tm["ms_decode"] + tm["ms_cfg"]) / runs,
            "nodes": nodes, "variables": int(res["n_vars"].sum()), "type_classes": int(res["n_tclasses"].sum()),
            "live_merges": int(res["n_live_merges"].sum()), "ternaries": int(res["n_ternary"].sum()),
            "failed": int((~ok).sum()), "rerun_identical": bool(res.tobytes() == res0.tobytes()),
            "sample_matches_oracle": bool(dig[:sub.n_kernels]["digest"].tobytes() == osum["digest"].tobytes()),
            "counts_match_digest_run": bool(np.array_equal(dig["n_vars"], res["n_vars"]) and
                                            np.array_equal(dig["n_live_merges"], res["n_live_merges"])),
            "alg_bytes": alg, "type_stage_GBps": alg / (ty_ms * 1e-3) / 1e9 if ty_ms else None,
            "roofline": stage_roofline(alg, ty_ms, "k_types"),
            "cpu_oracle": {"instructions_per_s": sub.n_instr / cpu_dt, "cores": 1, "kernels": sub.n_kernels}}


def text_workload(ctx, b, stream, steps=5, cpu_kernels=2048):
    """The text front end (dc_parse_text) on a workload rendered as one
    listing: whole runs (line starts, kinds, per-kernel counts, labels and
    records) with the text in HBM, stage times from HIP events; the oracle's
    parser on one core over the listing of the first cpu_kernels kernels."""
    import torch
    import dcgen
    import oracle
    from paper_2107_07809_amd import dc
    text = dcgen.render(b)
    dev = dc.text_to_device(text)
    t = ctx.parse_text(dev, len(text), timing=True, stream=stream)
    t.run()
    t.wait()
    t.timing_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        t.run()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    tm = t.timing()
    c = t.counts()
    ok = bool(t.kernels().tobytes() == b.kernels.tobytes() and t.args().tobytes() == b.args.tobytes())
    t.free()
    runs = max(1, tm["runs"])
    alg = len(text) + 16 * c["n_instr"] + 8 * c["n_args"] + 32 * c["n_kernels"]
    sub = dcgen.render(b.subset(np.arange(min(cpu_kernels, b.n_kernels))))
    t0 = time.perf_counter()
    oracle.parse_text(sub)
    cpu_dt = time.perf_counter() - t0
    return {"text_bytes": len(text), "lines": c["n_lines"], "instructions": c["n_instr"],
            "instructions_per_s": c["n_instr"] / dt, "GB_per_s": len(text) / dt / 1e9, "ms_per_step": dt * 1e3,
            "stage_ms": {"lines_and_kinds": tm["ms_decode"] / runs, "counts": tm["ms_cfg"] / runs,
                         "records": tm["ms_fixpoint"] / runs},
            "descriptors_and_args_match": ok, "alg_bytes": alg,
            "alg_GBps": alg / (tm["ms_total"] / runs * 1e-3) / 1e9 if tm["ms_total"] else None,
            "roofline": stage_roofline(alg, tm["ms_total"] / runs, "k_tx_* (whole front end)"),
            "cpu_oracle": {"bytes_per_s": len(sub) / cpu_dt, "cores": 1, "kernels": min(cpu_kernels, b.n_kernels)}}


def struct_workload(ctx, b, stream, steps=5, cpu_kernels=2048):
    """Region-graph structuring (dc_structure) of a workload: whole runs (the
    graph stages, then one search per kernel) with the records in HBM, the
    structuring's own time from HIP events; the oracle on one core over the
    first cpu_kernels kernels."""
    import torch
    import oracle
    from paper_2107_07809_amd import dc
    dev = dc.to_device(b.instrs)
    s = ctx.structure(b.kernels, dev, b.n_instr, timing=True, stream=stream)
    s.run()
    s.wait()
    res0 = s.results()
    s.timing_reset()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        s.run()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / steps
    tm = s.timing()
    res = s.results()
    s.free()
    sub = b.subset(np.arange(min(cpu_kernels, b.n_kernels)))
    t = time.perf_counter()
    osum = oracle.structure_batch(sub)
    cpu_dt = time.perf_counter() - t
    st_ms = tm["ms_fixpoint"] / max(1, tm["runs"])
    # the search reads 16 B of graph per block and the kernel's status, writes
    # 24 B per merge and a 32 B result per kernel
    alg = 16 * int(res["n_blocks"].sum()) + 24 * int(res["n_merges"].sum()) + 36 * b.n_kernels
    return {"instructions_per_s": b.n_instr / dt, "ms_per_step": dt * 1e3,
            "struct_ms": st_ms, "alg_bytes": alg, "roofline": stage_roofline(alg, st_ms, "k_struct"),
            "graph_stages_ms": (tm["ms_decode"] + tm["ms_cfg"]) / max(1, tm["runs"]),
            "merges": int(res["n_merges"].sum()), "kernels_reduced_to_one_region": int((res["n_left"] == 1).sum()),
            "failed": int((res["status"] != 0).sum()), "rerun_identical": bool(res.tobytes() == res0.tobytes()),
            "sample_matches_oracle": bool(res[:sub.n_kernels]["digest"].tobytes() == osum["digest"].tobytes()),
            "cpu_oracle": {"instructions_per_s": sub.n_instr / cpu_dt, "cores": 1, "kernels": sub.n_kernels}}


def extra_workloads(ctx, stream):
    """The other configurations, each timed as whole-path runs with its
    records in HBM."""
    import dcgen
    out = {}
    b = dcgen.generate(2, 65536)
    r = timed_run(ctx, b, stream, steps=10, warmup=2, shape={}, lat_steps=0, what="65,536 kernels")
    plain = plain_per_kernel(ctx, b, stream, 2048)
    out["loguniform_65536_kernels"] = {"instructions": int(b.n_instr), "instructions_per_s": r["value"],
                                       "ms_per_step": r["ms_per_step"], "fixpoint_ms": r["fix_ms"],
                                       "sweeps_max": r["sweeps"]["max"], "failed": r["failed"],
                                       "plain": plain, "batched_speedup": r["value"] / plain["value"]}
    log("65,536 kernels: register versions")
    out["loguniform_65536_kernels"]["ssa"] = ssa_workload(ctx, b, stream)
    log("65,536 kernels: variables and types")
    out["loguniform_65536_kernels"]["types"] = types_workload(ctx, b, stream)
    log("65,536 kernels: structuring")
    out["loguniform_65536_kernels"]["structure"] = struct_workload(ctx, b, stream)
    log("65,536 kernels: text front end")
    out["loguniform_65536_kernels"]["text"] = text_workload(ctx, b, stream)
    b = dcgen.generate(4, 16)
    r = timed_run(ctx, b, stream, steps=2, warmup=0, shape={}, lat_steps=0, what="16 huge kernels")
    out["huge_16_kernels_1M_to_4M"] = {
        "instructions": int(b.n_instr), "instructions_per_s": r["value"], "ms_per_step": r["ms_per_step"],
        "sweeps_max": r["sweeps"]["max"], "blocks_max": int(r["results"]["n_blocks"].max()),
        "alg_GBps": r["alg_bytes"] / (r["fix_ms"] * 1e-3) / 1e9, "failed": r["failed"]}
    b = dcgen.generate(1, 32)
    r = timed_run(ctx, b, stream, steps=50, warmup=2, shape={}, lat_steps=0, what="32 kernels")
    plain = plain_per_kernel(ctx, b, stream, 32)
    out["small_32_kernels"] = {"instructions": int(b.n_instr), "batched_instructions_per_s": r["value"],
                               "batched_ms": r["ms_per_step"], "graph_replay_ms": graph_replay_ms(ctx, b, stream),
                               "plain_instructions_per_s": plain["value"],
                               "plain_ms_per_kernel": plain["seconds"] * 1e3 / 32,
                               "batched_speedup": r["value"] / plain["value"]}
    return out


def serving(ctx, rate, seconds, warm_seconds=1.0, offline=True, **server_opts):
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
            "lanes": st["lanes"], "hw_queues": os.environ.get("GPU_MAX_HW_QUEUES", "HIP default"), **out,
            "workload": f"{n} log-normal requests (median 1,000 instructions, sigma 1, cap 100k) at Poisson "
                        f"arrivals in {seconds:g} s after {n_warm} warm-up arrivals ({warm_seconds:g} s)"}


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


def roofline(r, prof):
    """HBM roofline of the fixpoint kernel (algorithmic bytes per launch over
    its HIP-event launch time) and, from the committed counters of the same
    source, the measured HBM traffic and the issue rate against the chip's
    instruction-issue limits."""
    achieved = r["alg_bytes"] / (r["fix_ms"] * 1e-3) / 1e9
    tb = prof.get("traffic_bytes_per_launch")
    out = {"bound": "hbm", "kernel": "k_fixpoint", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": achieved / HBM_PEAK_GBS, "traffic": tb / (r["fix_ms"] * 1e-3) / 1e9 if tb else None,
           "alg_bytes_per_launch": r["alg_bytes"], "traffic_bytes_per_launch": tb, "avg_launch_ms": r["fix_ms"]}
    if "wave_instructions_per_launch" in prof:
        # one instruction of each kind per cycle per CU at most for wave64
        # work (four SIMDs, each issuing to a unit every fourth cycle): the
        # kernel's busiest kind is compared with that
        cyc = r["fix_ms"] * 1e-3 * CLOCK_GHZ * 1e9 * N_CU
        kinds = {k: prof[k + "_per_launch"] for k in ("valu", "salu", "lds", "smem", "branch", "vmem")
                 if k + "_per_launch" in prof}
        busiest = max(kinds, key=kinds.get)
        out["issue"] = {"bound": "issue", "kind": busiest, "achieved": kinds[busiest] / cyc,
                        "peak": 1.0, "unit": "wave-instructions/cycle/CU", "frac": kinds[busiest] / cyc,
                        "all_kinds_per_cycle_per_cu": prof["wave_instructions_per_launch"] / cyc,
                        "all_kinds_peak": 5.0,
                        "lds_bank_conflict_cycles_per_lds_cycle": prof.get("lds_conflict_frac")}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", type=int, default=3, choices=sorted(WORKLOADS),
                    help="3: 1,048,576 Zipf kernels (the headline); 2: 65,536 log-uniform kernels")
    ap.add_argument("--kernels", type=int, default=0, help="first N kernels of the workload (0 = all)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-fraction", type=float, default=0.01)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one 1 GiB device copy first (a known-size reference for HBM counters)")
    ap.add_argument("--waves-per-group", type=int, default=0)
    ap.add_argument("--groups-per-cu", type=int, default=0)
    ap.add_argument("--longest-first", action="store_true", help="kernels longest first (with an explicit shape)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the library's default launch shape instead of dc_autotune's")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serve-rate", type=float, default=50000.0)
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--no-extra", action="store_true", help="skip the other workloads")
    ap.add_argument("--only-struct", action="store_true",
                    help="time only the structuring (dc_structure) of the workload")
    ap.add_argument("--only-text", action="store_true",
                    help="time only the text front end (dc_parse_text) on the workload rendered as one listing")
    ap.add_argument("--only-types", action="store_true",
                    help="time only the variables and types (dc_build_types) of the workload")
    ap.add_argument("--only-ssa", action="store_true",
                    help="time only the register versions (dc_build_ssa) of the workload and print their figures")
    ap.add_argument("--lat-steps", type=int, default=5, help="runs timed one by one for the latency percentiles")
    ap.add_argument("--tune-sample", type=int, default=65536,
                    help="kernels in the autotuner's sample (every stride-th kernel; enough work to fill the GPU)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    import torch
    import dcgen
    from paper_2107_07809_amd import dc

    cfg = args.workload
    desc, n_all = WORKLOADS[cfg]
    n_k = args.kernels or n_all
    t = time.perf_counter()
    b = dcgen.generate(cfg, n_k)
    log(f"generated {b.n_kernels} kernels, {b.n_instr} instructions in {time.perf_counter() - t:.1f}s")
    stream = torch.cuda.current_stream()
    if args.only_struct:
        ctx = dc.Context(0)
        r = struct_workload(ctx, b, stream, steps=args.steps)
        ctx.close()
        print(json.dumps({"workload": desc, "kernels": b.n_kernels, "instructions": b.n_instr, "structure": r}),
              flush=True)
        return
    if args.only_text:
        ctx = dc.Context(0)
        r = text_workload(ctx, b, stream, steps=args.steps)
        ctx.close()
        print(json.dumps({"workload": desc, "kernels": b.n_kernels, "instructions": b.n_instr, "text": r}), flush=True)
        return
    if args.only_types:
        ctx = dc.Context(0)
        r = types_workload(ctx, b, stream, steps=args.steps)
        ctx.close()
        print(json.dumps({"workload": desc, "kernels": b.n_kernels, "instructions": b.n_instr, "types": r}),
              flush=True)
        return
    if args.only_ssa:
        ctx = dc.Context(0)
        r = ssa_workload(ctx, b, stream, steps=args.steps)
        ctx.close()
        print(json.dumps({"workload": desc, "kernels": b.n_kernels, "instructions": b.n_instr, "ssa": r}), flush=True)
        return
    if args.copy_calibration:
        src = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("copy calibration: 1 GiB device-to-device copy done")
    ctx = dc.Context(0)
    shape = {"waves_per_group": args.waves_per_group, "groups_per_cu": args.groups_per_cu,
             "longest_first": args.longest_first}
    tuned = False
    if not args.no_autotune and not (args.waves_per_group or args.groups_per_cu):
        # launch shape from the autotuner on a sample of every stride-th
        # kernel (outside the timed region)
        sub = b.subset(np.arange(0, b.n_kernels, max(1, b.n_kernels // args.tune_sample)))
        dev = dc.to_device(sub.instrs)
        shape, tune_ms = ctx.autotune(sub.kernels, dev, sub.n_instr, sub.args, sample=sub.n_kernels, stream=stream)
        del dev, sub
        torch.cuda.empty_cache()
        tuned = True
        log(f"autotune: {shape} ({tune_ms:.2f} ms per run of the sample)")
    sample_idx = lens = None
    if not args.no_cpu:
        sample_idx, lens = stratified_sample(cfg, n_k, args.cpu_fraction)
    r = timed_run(ctx, b, stream, args.steps, args.warmup, shape, sample_idx=sample_idx, lat_steps=args.lat_steps,
                  what="headline")
    log(f"headline: {r['value']:.4g} instructions/s, {r['ms_per_step']:.1f} ms per step, failed {r['failed']}")
    prof = profile_fields()
    out = {
        "metric": METRIC,
        "value": r["value"],
        "unit": "instructions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": desc if n_k == n_all else f"first {n_k} of: {desc}",
                   "kernels": b.n_kernels, "instructions": b.n_instr, "record_bytes": 16 * b.n_instr,
                   "form": "batched persistent (one wavefront per kernel), one plan for the whole batch",
                   "launch": {**shape, "autotuned": tuned}},
        "roofline": roofline(r, prof),
        "stages_ms": r["stages_ms"],
        "latency_ms": r["latency_ms"],
        "sweeps": r["sweeps"],
        "failed_kernels": r["failed"],
        "overflow_kernels": r["overflow_kernels"],
        "rerun_identical": r["rerun_identical"],
    }
    del b
    if not args.no_extra:
        out["workloads"] = extra_workloads(ctx, stream)
    if not args.no_serving:
        log(f"serving: {args.serve_rate:.0f} requests/s for {args.serve_seconds} s")
        out["serving"] = serving(ctx, args.serve_rate, args.serve_seconds)
    ctx.close()
    if not args.no_cpu:
        log("timing the CPU oracle baseline on the stratified sample")
        out["cpu_baseline"], by_kernel = cpu_baseline(cfg, n_k, sample_idx, lens)
        out["verified_sample"] = verify_sample(r, by_kernel)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
