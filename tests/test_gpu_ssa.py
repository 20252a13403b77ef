"""GPU parity of the register versions (minimal SSA form): the HIP path
through the C ABI (dc_build_ssa) against the CPU oracle, bit-exact: every
immediate dominator, merge, merge argument and the version of every use and
definition, and at full size the per-kernel digest over all of them."""
import sys
import time

import numpy as np
import pytest

import asmtext
import dcgen
import hand_kernels as hk
import oracle
from gpu_common import OracleSsaRun, compare_ssa_summaries

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2107_07809_amd import dc  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = dc.Context(0)
    yield c
    c.close()


def compare_kernel(s, res, k, recs, desc):
    r = oracle.ssa(recs, desc)
    g = res[k]
    assert g["status"] == r["status"], k
    if r["status"] != 0:
        assert g["n_blocks"] == 0 and g["digest"] == 0 and len(s.phis(k)) == 0, k
        u, d = s.versions(k)
        assert (u == dc.SSA_NONE).all() and (d == dc.SSA_NONE).all(), k
        return
    assert g["n_blocks"] == r["n_blocks"], k
    assert s.idom(k).tobytes() == r["idom"].tobytes(), k
    ph = s.phis(k)
    assert ph.tobytes() == r["phis"].tobytes(), (k, ph[:5], r["phis"][:5])
    assert s.phi_args(k).tobytes() == r["phi_arg"].tobytes(), k
    u, d = s.versions(k)
    if u.tobytes() != r["use_ver"].tobytes():
        i, q = np.argwhere(u != r["use_ver"])[0]
        raise AssertionError(f"kernel {k} instruction {i} use {q}: gpu {u[i, q]} oracle {r['use_ver'][i, q]}")
    if d.tobytes() != r["def_ver"].tobytes():
        i, q = np.argwhere(d != r["def_ver"])[0]
        raise AssertionError(f"kernel {k} instruction {i} def {q}: gpu {d[i, q]} oracle {r['def_ver'][i, q]}")
    assert g["digest"] == r["digest"], k
    assert (g["n_phi"], g["n_phi_args"]) == (len(r["phis"]), len(r["phi_arg"])), k


def full_compare(ctx, b, label):
    say(f"ssa {label}: {b.n_kernels} kernels, {b.n_instr} instructions")
    dev = dc.to_device(b.instrs)
    s = ctx.build_ssa(b.kernels, dev, b.n_instr)
    res = s.results()
    for k in range(b.n_kernels):
        compare_kernel(s, res, k, *b.kernel(k)[:2])
    s.free()
    return res


def test_ssa_small_and_hand_written(ctx):
    """The small workload, a sample of the 200-2,000-instruction workload with
    loops, the hand-written rule kernels (entry-block loops, unreachable code,
    exec-mask diamonds), and kernels that fail their checks."""
    good = dcgen.generate(2, 6)
    r, d, a = good.kernel(0)
    bad_op = r.copy()
    bad_op[5]["op"] = 200
    d_unsup = d.copy()
    d_unsup["useargs"] = 0
    parts = [dcgen.generate(1, 32).kernel(k) for k in range(32)] + \
        [dcgen.generate(2, 150, i0=3000).kernel(k) for k in range(150)] + \
        [k for _, k in hk.all_kernels()] + \
        [(bad_op, d, a), (r, d_unsup, a), (r[:-1].copy(), d, a)]
    res = full_compare(ctx, dcgen.concat(parts), "small")
    assert (res["status"] < 0).sum() == 3 and (res["n_phi"] > 0).sum() > 100


def test_ssa_paper_diamond(ctx):
    """v5 set on both arms of an exec-mask if/else: one merge at the join,
    arguments from each arm, read by the add after the join."""
    src = """
      v_cmp_gt_u32 vcc, v0, 3
      s_and_saveexec_b64 s[20:21], vcc
      s_cbranch_execz ELSE
      v_mov_b32 v5, 1
      s_branch END
    ELSE:
      v_mov_b32 v5, 2
    END:
      s_or_b64 exec, exec, s[20:21]
      v_add_u32 v6, v5, v0
      s_endpgm
    """
    recs = asmtext.assemble(src)
    b = dcgen.concat([(recs, dcgen.descriptor(len(recs)), np.zeros(0, dcgen.ARG_DTYPE))])
    dev = dc.to_device(b.instrs)
    s = ctx.build_ssa(b.kernels, dev, b.n_instr)
    ph = s.phis(0)
    v5 = [p for p in ph if p["slot"] == 112 + 5]
    assert len(v5) == 1 and v5[0]["block"] == 3 and v5[0]["version"] == 3
    u, _ = s.versions(0)
    assert u[7][0] == 3 and u[7][1] == 0
    s.free()


def test_ssa_many_blocks(ctx):
    """Kernels of 1,600-2,600 blocks (graph in global memory, loops and ifs
    nested to depth 5) beside short ones (graph in LDS), in one batch."""
    b6 = dcgen.generate(6, 12)
    parts = [b6.kernel(k) for k in (0, 5, 9)] + [dcgen.generate(3, 40, i0=77).kernel(k) for k in range(40)]
    res = full_compare(ctx, dcgen.concat(parts), "many blocks")
    assert (res["n_blocks"] > 256).sum() >= 3


def test_ssa_c2_full_digest(ctx):
    """All 65,536 kernels of the 51.2M-instruction workload: per-kernel
    status, blocks, merges, arguments, operand count and digest; then a second
    run of the same object (no allocation) gives the same bytes."""
    n = 65536
    orc = OracleSsaRun(2, n)
    b = dcgen.generate(2, n)
    dev = dc.to_device(b.instrs)
    t = time.time()
    s = ctx.build_ssa(b.kernels, dev, b.n_instr)
    res = s.results()
    say(f"ssa c2: gpu done in {time.time() - t:.1f}s")
    s.run()
    assert s.results().tobytes() == res.tobytes()
    s.free()
    compare_ssa_summaries(res, orc.result())


def test_ssa_c4_very_large(ctx):
    """The 16 kernels of 1-4M instructions (up to ~17k blocks)."""
    orc = OracleSsaRun(4, 16, procs=16, jobs_per_proc=1)
    b = dcgen.generate(4, 16)
    dev = dc.to_device(b.instrs)
    s = ctx.build_ssa(b.kernels, dev, b.n_instr)
    res = s.results()
    s.free()
    say(f"ssa c4: gpu done, blocks max {int(res['n_blocks'].max())}")
    compare_ssa_summaries(res, orc.result())


def _nops_like(b):
    """Records of the same layout: every instruction a s_nop, the last of
    each kernel s_endpgm (one block per kernel, no definitions)."""
    r = b.instrs.copy()
    nop, end = dcgen.opcode("s_nop"), dcgen.opcode("s_endpgm")
    r["op"] = nop
    r["r0"] = r["r1"] = r["r2"] = 0xFFFF
    r["imm"] = 0
    r["target"] = -1
    last = b.kernels["instr_begin"] + b.kernels["n_instr"] - 1
    r["op"][last] = end
    return r


def test_ssa_rerun_on_other_records(ctx):
    """dc_ssa_run on a new record pointer: the object was sized for records
    with one block per kernel and no definitions; the new records of the same
    layout have loops and thousands of blocks, and the run sizes the tables
    and outputs again.  Both against the oracle, then back on the first."""
    b = dcgen.concat([dcgen.generate(2, 300, i0=40).kernel(k) for k in range(300)] +
                     [dcgen.generate(6, 2).kernel(k) for k in range(2)])
    sparse_h = _nops_like(b)
    sparse = dc.to_device(sparse_h)
    dense = dc.to_device(b.instrs)
    s = ctx.build_ssa(b.kernels, sparse, b.n_instr)
    res = s.results()
    assert (res["status"] == 0).all() and (res["n_blocks"] == 1).all() and (res["n_phi"] == 0).all()
    nb = dcgen.Batch(sparse_h, b.kernels, b.args)
    compare_ssa_summaries(res, oracle.ssa_batch(nb))
    s.run(dense)
    compare_ssa_summaries(s.results(), oracle.ssa_batch(b))
    compare_kernel(s, s.results(), 301, *b.kernel(301)[:2])
    s.run(sparse)
    assert s.results().tobytes() == res.tobytes()
    s.free()


def test_ssa_empty_batch(ctx):
    kern = np.zeros(0, dc.KERNEL_DTYPE)
    dev = dc.to_device(np.zeros(1, dc.INSTR_DTYPE))
    s = ctx.build_ssa(kern, dev, 1)
    assert len(s.results()) == 0
    s.free()


def test_ssa_c3_zipf_full(ctx):
    """All 1,048,576 kernels of the Zipf(1.2) 20-20,000 workload (1.74e9
    instructions) in one object: per-kernel status, blocks, merges,
    arguments, operand count and digest against the oracle (worker
    processes, started first)."""
    n = 1048576
    orc = OracleSsaRun(3, n, jobs_per_proc=16)
    b = dcgen.generate(3, n)
    dev = dc.to_device(b.instrs)
    torch.cuda.synchronize()
    t = time.time()
    s = ctx.build_ssa(b.kernels, dev, b.n_instr)
    res = s.results()
    say(f"ssa c3: gpu done in {time.time() - t:.1f}s, merges {int(res['n_phi'].sum())}")
    s.free()
    del dev
    torch.cuda.empty_cache()
    compare_ssa_summaries(res, orc.result())
