"""Helpers shared by the GPU parity tests (test infrastructure)."""
import os
from concurrent.futures import ProcessPoolExecutor

import numpy as np

import dcgen
import oracle


def _oracle_chunk(args):
    cfg, i0, n = args
    b = dcgen.generate(cfg, n, i0=i0, threads=1)
    return oracle.analyze_batch(b)


class OracleRun:
    """Oracle summaries and dense records for kernels [0, n) of a config,
    computed in parallel worker processes (each regenerates its shard); the
    workers start at construction, so the caller can run the GPU meanwhile."""

    def __init__(self, cfg: int, n: int, procs: int = 0, jobs_per_proc: int = 4):
        procs = procs or min(16, os.cpu_count() or 1)
        step = max(1, (n + procs * jobs_per_proc - 1) // (procs * jobs_per_proc))
        self.ex = ProcessPoolExecutor(procs)
        self.futs = [self.ex.submit(_oracle_chunk, (cfg, i, min(step, n - i))) for i in range(0, n, step)]

    def result(self):
        parts = [f.result() for f in self.futs]
        self.ex.shutdown()
        summ = np.concatenate([p[0] for p in parts])
        acc = np.concatenate([p[1] for p in parts])
        sys = np.concatenate([p[2] for p in parts])
        return summ, acc, sys


def oracle_config(cfg: int, n: int, procs: int = 0):
    """Oracle summaries and dense records for kernels [0, n) of a config."""
    return OracleRun(cfg, n, procs).result()


def compare_summaries(gpu_res, summ, digest: bool = True):
    """Per-kernel status, block count, sweeps, counts and (unless the run did
    not ask for it) the state digest."""
    assert len(gpu_res) == len(summ)
    for f_gpu, f_or in [("status", "status"), ("n_blocks", "n_blocks"), ("sweeps", "sweeps"),
                        ("n_access", "n_acc"), ("n_sysval", "n_sys")]:
        bad = np.nonzero(gpu_res[f_gpu] != summ[f_or])[0]
        assert len(bad) == 0, (f_gpu, bad[:10], gpu_res[f_gpu][bad[:10]], summ[f_or][bad[:10]])
    if digest:
        bad = np.nonzero(gpu_res["digest"] != summ["digest"])[0]
        assert len(bad) == 0, ("digest", bad[:10])


def _oracle_ssa_chunk(args):
    cfg, i0, n = args
    b = dcgen.generate(cfg, n, i0=i0, threads=1)
    return oracle.ssa_batch(b)


class OracleSsaRun:
    """Oracle version summaries for kernels [0, n) of a config, in parallel
    worker processes started at construction."""

    def __init__(self, cfg: int, n: int, procs: int = 0, jobs_per_proc: int = 4):
        procs = procs or min(16, os.cpu_count() or 1)
        step = max(1, (n + procs * jobs_per_proc - 1) // (procs * jobs_per_proc))
        self.ex = ProcessPoolExecutor(procs)
        self.futs = [self.ex.submit(_oracle_ssa_chunk, (cfg, i, min(step, n - i))) for i in range(0, n, step)]

    def result(self):
        parts = [f.result() for f in self.futs]
        self.ex.shutdown()
        return np.concatenate(parts)


def compare_ssa_summaries(gpu_res, summ):
    """Per-kernel status, blocks, merges, merge arguments, operand count and
    digest of the versions."""
    assert len(gpu_res) == len(summ)
    for f_gpu, f_or in [("status", "status"), ("n_blocks", "n_blocks"), ("n_phi", "n_phi"),
                        ("n_phi_args", "n_args"), ("n_operands", "n_operands"), ("digest", "digest")]:
        bad = np.nonzero(gpu_res[f_gpu] != summ[f_or])[0]
        assert len(bad) == 0, (f_gpu, bad[:10], gpu_res[f_gpu][bad[:10]], summ[f_or][bad[:10]])


def _oracle_struct_chunk(args):
    cfg, i0, n = args
    b = dcgen.generate(cfg, n, i0=i0, threads=1)
    return oracle.structure_batch(b)


class OracleStructRun:
    """Oracle structuring summaries for kernels [0, n) of a config, in
    parallel worker processes started at construction."""

    def __init__(self, cfg: int, n: int, procs: int = 0, jobs_per_proc: int = 4):
        procs = procs or min(16, os.cpu_count() or 1)
        step = max(1, (n + procs * jobs_per_proc - 1) // (procs * jobs_per_proc))
        self.ex = ProcessPoolExecutor(procs)
        self.futs = [self.ex.submit(_oracle_struct_chunk, (cfg, i, min(step, n - i))) for i in range(0, n, step)]

    def result(self):
        parts = [f.result() for f in self.futs]
        self.ex.shutdown()
        return np.concatenate(parts)


def compare_struct_summaries(gpu_res, summ):
    assert len(gpu_res) == len(summ)
    for f in ("status", "n_blocks", "n_merges", "n_left", "root", "digest"):
        bad = np.nonzero(gpu_res[f] != summ[f])[0]
        assert len(bad) == 0, (f, bad[:10], gpu_res[f][bad[:10]], summ[f][bad[:10]])


def _oracle_types_chunk(args):
    cfg, i0, n = args
    b = dcgen.generate(cfg, n, i0=i0, threads=1)
    return oracle.types_batch(b)


class OracleTypesRun:
    """Oracle variable and type summaries for kernels [0, n) of a config, in
    parallel worker processes started at construction."""

    def __init__(self, cfg: int, n: int, procs: int = 0, jobs_per_proc: int = 4):
        procs = procs or min(16, os.cpu_count() or 1)
        step = max(1, (n + procs * jobs_per_proc - 1) // (procs * jobs_per_proc))
        self.ex = ProcessPoolExecutor(procs)
        self.futs = [self.ex.submit(_oracle_types_chunk, (cfg, i, min(step, n - i))) for i in range(0, n, step)]

    def result(self):
        parts = [f.result() for f in self.futs]
        self.ex.shutdown()
        return np.concatenate(parts)


def compare_types_summaries(gpu_res, summ, digest: bool = True):
    """Per-kernel status, node, variable, type-class, live-merge and ternary
    counts and the digest over every node."""
    assert len(gpu_res) == len(summ)
    fields = ["status", "n_nodes", "n_vars", "n_tclasses", "n_live_merges", "n_ternary"] + (["digest"] if digest else [])
    for f in fields:
        bad = np.nonzero(gpu_res[f] != summ[f])[0]
        assert len(bad) == 0, (f, bad[:10], gpu_res[f][bad[:10]], summ[f][bad[:10]])
