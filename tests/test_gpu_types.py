"""GPU parity of the variables and types over the register versions: the
HIP path through the C ABI (dc_build_types) against the CPU oracle,
bit-exact: every node's slot, version, variable, type class, type bits and
flags, and at full size the per-kernel counts and the digest over all of
them."""
import sys
import time

import numpy as np
import pytest

import asmtext
import dcgen
import hand_kernels as hk
import oracle
from gpu_common import OracleTypesRun, compare_types_summaries

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


def compare_kernel(t, res, k, recs, desc, args):
    r = oracle.types(recs, desc, args)
    g = res[k]
    assert g["status"] == r["status"], k
    v = t.vars(k)
    if r["status"] != 0:
        assert g["n_nodes"] == 0 and g["digest"] == 0 and len(v) == 0, k
        return
    if v.tobytes() != r["nodes"].tobytes():
        bad = np.nonzero(v != r["nodes"])[0]
        raise AssertionError(f"kernel {k}: {len(bad)} nodes differ, first {bad[0]}: gpu {v[bad[0]]} "
                             f"oracle {r['nodes'][bad[0]]}")
    for f in ("n_vars", "n_tclasses", "n_live_merges", "n_ternary", "digest"):
        assert g[f] == r[f], (k, f, g[f], r[f])
    assert g["n_nodes"] == len(r["nodes"]), k


def full_compare(ctx, b, label):
    say(f"types {label}: {b.n_kernels} kernels, {b.n_instr} instructions")
    dev = dc.to_device(b.instrs)
    t = ctx.build_types(b.kernels, dev, b.n_instr, b.args)
    res = t.types()
    for k in range(b.n_kernels):
        compare_kernel(t, res, k, *b.kernel(k))
    t.free()
    return res


PINNED = [
    ("s_add_u32 s0, s4, s0\ns_endpgm", 1, None),
    ("v_cvt_f32_u32 v1, v0\nv_cvt_f64_f32 v[2:3], v1\nv_cvt_u32_f32 v4, v1\nv_fma_f32 v5, v6, v7, v8\ns_endpgm", 1, None),
    ("v_mov_b32 v1, v0\nv_add_f32 v2, v1, v1\ns_mov_b64 s[8:9], s[2:3]\ns_add_u32 s10, s8, 1\n"
     "s_mul_i32 s11, s9, 3\ns_endpgm", 1, None),
    ("v_cmp_gt_u32 vcc, v0, 4\nv_cndmask_b32 v3, v1, v2, vcc\nv_mul_f32 v4, v3, 2.0\ns_endpgm", 3, None),
    ("s_branch END\nv_cndmask_b32 v3, v1, v2, vcc\nv_mul_f32 v4, v3, 2.0\nEND:\ns_endpgm", 3, None),
    ("""v_cmp_gt_u32 vcc, v0, 4
        s_and_saveexec_b64 s[20:21], vcc
        s_cbranch_execz ELSE
        v_mov_b32 v5, 1
        s_branch END
      ELSE:
        v_mov_b32 v5, 2
      END:
        s_or_b64 exec, exec, s[20:21]
        v_cvt_f32_u32 v6, v5
        s_endpgm""", 1, None),
    ("""s_mov_b32 s20, 0
      HEAD:
        s_cmp_eq_u32 s22, 0
        s_cbranch_scc1 SKIP
        s_mov_b32 s20, 7
      SKIP:
        s_cmp_lt_u32 s23, 9
        s_cbranch_scc1 HEAD
        s_add_u32 s24, s20, 1
        s_endpgm""", 1, None),
    ("""s_load_dwordx2 s[8:9], s[4:5], 0x30
        s_load_dword s10, s[4:5], 0x38
        s_load_dword s11, s[4:5], 0x0
        s_load_dword s12, s[4:5], 0x18
        s_load_dword s13, s[4:5], 0x40
        s_load_dword s15, s[4:5], 0x20010
        s_mov_b32 s4, 0
        s_load_dword s14, s[4:5], 0x38
        s_endpgm""", 1, "copy"),
    ("""global_load_dword v1, v[2:3], off
        global_store_dword v[4:5], v1, s[8:9]
        flat_store_dword v[6:7], v1
        ds_write_b32 v8, v1
        ds_read_b32 v9, v10
        s_endpgm""", 1, None),
]


def copy_args():
    a = np.zeros(2, dcgen.ARG_DTYPE)
    a[0] = (0x30, 8, dcgen.T_PTR, dcgen.T_INT)
    a[1] = (0x38, 4, dcgen.T_INT, 0)
    return a


def test_types_pinned_and_hand_written(ctx):
    """The kernels the oracle's pins work out by hand, every hand-written rule
    kernel (argument tables, hidden slots, clobbered s4, loops, unreachable
    code), a small generated sample and kernels that fail their checks."""
    parts = []
    for src, dims, args in PINNED:
        recs = asmtext.assemble(src)
        a = copy_args() if args == "copy" else np.zeros(0, dcgen.ARG_DTYPE)
        parts.append((recs, dcgen.descriptor(len(recs), dims, (64, 1, 1), 1, len(a)), a))
    parts += [k for _, k in hk.all_kernels()]
    good = dcgen.generate(2, 6)
    r, d, a = good.kernel(0)
    bad_op = r.copy()
    bad_op[5]["op"] = 200
    d_unsup = d.copy()
    d_unsup["useargs"] = 0
    parts += [dcgen.generate(1, 32).kernel(k) for k in range(32)] + \
        [dcgen.generate(2, 100, i0=3000).kernel(k) for k in range(100)] + \
        [(bad_op, d, a), (r, d_unsup, a), (r[:-1].copy(), d, a)]
    res = full_compare(ctx, dcgen.concat(parts), "pinned and hand-written")
    assert (res["status"] < 0).sum() == 3 and (res["n_live_merges"] > 0).sum() > 50


def test_types_many_nodes(ctx):
    """Kernels with thousands of blocks and more nodes than the LDS holds
    (forests in global memory) beside short ones."""
    b6 = dcgen.generate(6, 12)
    parts = [b6.kernel(k) for k in (0, 5, 9)] + [dcgen.generate(3, 40, i0=77).kernel(k) for k in range(40)]
    res = full_compare(ctx, dcgen.concat(parts), "many nodes")
    assert (res["n_nodes"] > 2048).sum() >= 3 and (res["n_nodes"] <= 2048).sum() >= 10


def test_types_c2_full_digest(ctx):
    """All 65,536 kernels of the 51.2M-instruction workload: per-kernel counts
    and digest; a second run of the same object gives the same bytes."""
    n = 65536
    orc = OracleTypesRun(2, n)
    b = dcgen.generate(2, n)
    dev = dc.to_device(b.instrs)
    t0 = time.time()
    t = ctx.build_types(b.kernels, dev, b.n_instr, b.args)
    res = t.types()
    say(f"types c2: gpu done in {time.time() - t0:.1f}s, nodes {int(res['n_nodes'].sum())}")
    t.run()
    assert t.types().tobytes() == res.tobytes()
    t.free()
    compare_types_summaries(res, orc.result())


def test_types_c4_very_large(ctx):
    """The 16 kernels of 1-4M instructions."""
    orc = OracleTypesRun(4, 16, procs=16, jobs_per_proc=1)
    b = dcgen.generate(4, 16)
    dev = dc.to_device(b.instrs)
    t = ctx.build_types(b.kernels, dev, b.n_instr, b.args)
    res = t.types()
    t.free()
    say(f"types c4: gpu done, nodes max {int(res['n_nodes'].max())}")
    compare_types_summaries(res, orc.result())


def test_types_c3_zipf_full(ctx):
    """All 1,048,576 kernels of the Zipf(1.2) 20-20,000 workload (1.74e9
    instructions) in one object: per-kernel counts and digest against the
    oracle (worker processes, started first)."""
    n = 1048576
    orc = OracleTypesRun(3, n, jobs_per_proc=16)
    b = dcgen.generate(3, n)
    dev = dc.to_device(b.instrs)
    torch.cuda.synchronize()
    t0 = time.time()
    t = ctx.build_types(b.kernels, dev, b.n_instr, b.args)
    res = t.types()
    say(f"types c3: gpu done in {time.time() - t0:.1f}s, nodes {int(res['n_nodes'].sum())}")
    t.free()
    del dev
    torch.cuda.empty_cache()
    compare_types_summaries(res, orc.result())


def test_types_need_a_types_object(ctx):
    b = dcgen.generate(1, 4)
    dev = dc.to_device(b.instrs)
    s = ctx.build_ssa(b.kernels, dev, b.n_instr)
    with pytest.raises(dc.DCError):
        s.types()
    s.free()
    t = ctx.build_types(np.zeros(0, dc.KERNEL_DTYPE), dev, b.n_instr)
    assert len(t.types()) == 0
    t.free()
