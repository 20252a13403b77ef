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


def fuzz_listing(text: bytes, seed: int, rate: float = 0.15) -> bytes:
    """A listing with seeded random edits on a fraction of its lines: characters
    deleted, inserted (from the characters the grammar gives meaning to, and
    others), replaced or case-swapped, lines cut short, duplicated, joined or
    dropped; no line is made longer than a few hundred bytes."""
    rng = np.random.default_rng(seed)
    alphabet = b" \t,:;[]/.-+_0123456789abcdefxsvABCDEFXSV\"*#@\r"
    out = []
    for line in text.split(b"\n"):
        if rng.random() >= rate:
            out.append(line)
            continue
        op = int(rng.integers(0, 8))
        b = bytearray(line)
        if op == 0 and b:
            del b[int(rng.integers(0, len(b)))]
        elif op == 1:
            b.insert(int(rng.integers(0, len(b) + 1)), alphabet[int(rng.integers(0, len(alphabet)))])
        elif op == 2 and b:
            b[int(rng.integers(0, len(b)))] = alphabet[int(rng.integers(0, len(alphabet)))]
        elif op == 3:
            b = bytearray(bytes(b).swapcase())
        elif op == 4 and b:
            b = b[:int(rng.integers(0, len(b)))]
        elif op == 5:
            out.append(bytes(b))
        elif op == 6:
            b += b" " + bytes(b)
        elif op == 7:
            continue
        out.append(bytes(b[:400]))
    return b"\n".join(out)
