"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

The bar is bit-exact: every output of the analysis is integer or bit-set
work, so per-kernel status, block count, sweep count, access and system-value
records and the fixpoint IN state of every block must match byte for byte
(at full size through a digest of the states plus every record)."""
import glob
import os
import sys
import time

import numpy as np
import pytest

import asmtext
import dcgen
import oracle
from gpu_common import OracleRun, compare_summaries, oracle_config

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2107_07809_amd import dc  # noqa: E402

GOLDEN = sorted(glob.glob(os.path.join(os.path.dirname(__file__), "golden", "*.txt")))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = dc.Context(0)
    yield c
    c.close()


def run(ctx, b, **kw):
    dev = dc.to_device(b.instrs)
    batch = ctx.analyze(b.kernels, dev, b.n_instr, b.args, **kw)
    return batch, dev


def full_compare(ctx, b, **kw):
    """Byte-exact comparison of everything, states included."""
    say(f"full_compare: {b.n_kernels} kernels, {b.n_instr} instructions, {kw}")
    batch, dev = run(ctx, b, flags=dc.OPT_EXPORT_STATES | dc.OPT_DIGEST, **kw)
    res = batch.results()
    for k in range(b.n_kernels):
        r = oracle.analyze(*b.kernel(k))
        g = res[k]
        assert (g["status"], g["n_blocks"], g["sweeps"]) == (r["status"], r["n_blocks"], r["sweeps"]), k
        assert g["digest"] == r["digest"], k
        assert batch.accesses(k).tobytes() == r["accesses"].tobytes(), k
        assert batch.sysvals(k).tobytes() == r["sysvals"].tobytes(), k
        for blk in range(r["n_blocks"]):
            st, reached = batch.block_state(k, blk)
            assert reached == r["reached"][blk], (k, blk)
            if st.tobytes() != r["in_states"][blk].tobytes():
                diff = np.nonzero(st.view(np.uint8).reshape(368, 16) != r["in_states"][blk].view(np.uint8).reshape(
                    368, 16))[0]
                slot = int(diff[0])
                raise AssertionError(f"kernel {k} block {blk} slot {slot}: gpu {st[slot]} oracle "
                                     f"{r['in_states'][blk][slot]} ({oracle.decode(st[slot]['val'])} vs "
                                     f"{oracle.decode(r['in_states'][blk][slot]['val'])})")
    batch.free()
    return res


def test_c1_full(ctx):
    """All 32 kernels of the small configuration, every output byte."""
    full_compare(ctx, dcgen.generate(1, 32))


def test_golden_fixtures(ctx):
    """The paper's worked statements, analysed on the GPU in one batch."""
    import test_oracle_golden as tg
    fxs = [asmtext.Fixture(p) for p in GOLDEN]
    b = dcgen.concat([fx.kernel() for fx in fxs])
    batch, dev = run(ctx, b, flags=dc.OPT_EXPORT_STATES | dc.OPT_DIGEST)
    res = batch.results()
    for k, fx in enumerate(fxs):
        r = oracle.analyze(*fx.kernel())
        g = dict(status=int(res[k]["status"]), n_blocks=int(res[k]["n_blocks"]), sweeps=int(res[k]["sweeps"]),
                 accesses=batch.accesses(k), sysvals=batch.sysvals(k))
        g["in_states"] = [batch.block_state(k, i)[0] for i in range(g["n_blocks"])] if g["status"] == 0 else []
        tg.check_fixture(fx, g, None, None, where="gpu")
        assert g["accesses"].tobytes() == r["accesses"].tobytes(), fx.path
        assert g["sysvals"].tobytes() == r["sysvals"].tobytes(), fx.path
        assert int(res[k]["digest"]) == r["digest"], fx.path
    batch.free()



def test_hand_written_kernels(ctx):
    """Every hand-written rule kernel of the oracle's CPU pins (folding with
    edge and random constants, 64-bit shifts up to 63, inline floats, the
    argument-area table with hidden slots, mid-argument and spanning loads
    and a clobbered s4, index and pointer rules, uninitialised sources, the
    second dimension, loops and an entry-block back edge), in one batch:
    every state byte, record and digest against the oracle."""
    import hand_kernels as hk
    ks = hk.all_kernels()
    say(f"hand-written kernels: {len(ks)}")
    b = dcgen.concat([k for _, k in ks])
    res = full_compare(ctx, b)
    assert (res["status"] == 0).all(), [ks[i][0] for i in np.nonzero(res["status"])[0]]

def test_c2_subset_states(ctx):
    """Ragged lengths 200-2000 with loops: 600 kernels, states byte-exact
    (including kernels that use the full register range)."""
    b = dcgen.generate(2, 600)
    full_compare(ctx, b)


def test_c3_and_c5_shapes(ctx):
    """Zipf and log-normal lengths (short kernels of 20 instructions, long
    ones with hundreds of blocks)."""
    full_compare(ctx, dcgen.generate(3, 300))
    full_compare(ctx, dcgen.generate(5, 100))


def test_dense_cfg_main_and_overflow(ctx):
    """Kernels of 6,000-12,000 instructions with 1,300-2,400 blocks: states
    byte-exact through the overflow pass (default block cap), then with the
    largest block cap, where kernels up to 2,048 blocks take the main pass and
    the rest the overflow pass."""
    b = dcgen.generate(6, 12)
    full_compare(ctx, b)
    full_compare(ctx, b, block_cap=2048)


def test_c2_full_digest(ctx):
    """All 65,536 kernels of the 51.2M-instruction workload: every record and
    every kernel's state digest; then the run as the bench makes it (no
    digest, no exported states, so the IN states of chained blocks are never
    stored) in the launch shape the autotuner picks for it, again every
    record, status, block count and sweep count."""
    n = 65536
    orc = OracleRun(2, n)
    b = dcgen.generate(2, n)
    say("c2 full: generated", b.n_instr)
    dev = dc.to_device(b.instrs)
    sub = b.subset(np.arange(0, n, 8))
    sdev = dc.to_device(sub.instrs)
    shape, ms = ctx.autotune(sub.kernels, sdev, sub.n_instr, sub.args, sample=sub.n_kernels)
    say(f"c2 full: autotuned shape {shape} ({ms:.2f} ms per run of the sample)")
    summ, oacc, osys = orc.result()
    say("c2 full: oracle done")
    for flags, digest, kw in ((dc.OPT_DIGEST, True, {}), (dc.OPT_TIMING, False, shape)):
        batch = ctx.analyze(b.kernels, dev, b.n_instr, b.args, flags=flags, **kw)
        batch.run()
        res = batch.results()
        acc, _ = batch.all_accesses()
        sysv, _ = batch.all_sysvals()
        say(f"c2 full: gpu done (flags {flags}, {kw})")
        compare_summaries(res, summ, digest=digest)
        assert acc.tobytes() == oacc.tobytes()
        assert sysv.tobytes() == osys.tobytes()
        batch.free()


def test_c3_zipf_full(ctx):
    """All 1,048,576 kernels of the Zipf(1.2) 20-20,000 workload (1.74e9
    instructions) in one plan, as the bench analyses them: every status,
    block count, sweep count, record count, state digest and record byte
    against the oracle (run in worker processes meanwhile); then the run
    without the digest in the launch shape and kernel order the autotuner
    picks for it (on the bench's sample of every 16th kernel), every record
    again."""
    n = 1048576
    t = time.time()
    orc = OracleRun(3, n, jobs_per_proc=16)
    b = dcgen.generate(3, n)
    say(f"c3 full: generated {b.n_instr} instructions in {time.time() - t:.1f}s")
    dev = dc.to_device(b.instrs)
    torch.cuda.synchronize()
    say(f"c3 full: uploaded ({time.time() - t:.1f}s)")
    sub = b.subset(np.arange(0, n, 16))
    sdev = dc.to_device(sub.instrs)
    shape, ms = ctx.autotune(sub.kernels, sdev, sub.n_instr, sub.args, sample=sub.n_kernels)
    del sdev, sub
    say(f"c3 full: autotuned {shape} ({ms:.1f} ms per run of the sample)")
    runs = []
    for flags, kw in ((dc.OPT_DIGEST, {}), (dc.OPT_TIMING, shape)):
        batch = ctx.analyze(b.kernels, dev, b.n_instr, b.args, flags=flags, **kw)
        batch.run()
        res = batch.results()
        acc, _ = batch.all_accesses()
        sysv, _ = batch.all_sysvals()
        runs.append((flags, res, acc, sysv))
        batch.free()
        say(f"c3 full: gpu done (flags {flags}, {kw}; {time.time() - t:.1f}s)")
    del dev
    torch.cuda.empty_cache()
    summ, oacc, osys = orc.result()
    say(f"c3 full: oracle done ({time.time() - t:.1f}s)")
    for flags, res, acc, sysv in runs:
        compare_summaries(res, summ, digest=flags == dc.OPT_DIGEST)
        assert acc.tobytes() == oacc.tobytes()
        assert sysv.tobytes() == osys.tobytes()


def _records_and_summaries(ctx, b, summ, oacc, osys, flags, digest, tag):
    dev = dc.to_device(b.instrs)
    batch = ctx.analyze(b.kernels, dev, b.n_instr, b.args, flags=flags)
    batch.run()
    res = batch.results()
    acc, _ = batch.all_accesses()
    sysv, _ = batch.all_sysvals()
    say(f"{tag}: gpu done (flags {flags})")
    compare_summaries(res, summ, digest=digest)
    assert acc.tobytes() == oacc.tobytes()
    assert sysv.tobytes() == osys.tobytes()
    batch.free()
    return res


def test_c5_lognormal_65536(ctx):
    """The first 65,536 kernels of the log-normal workload (median 1,000
    instructions, cap 100k; about 108M instructions), with the main-pass
    arenas sized on the first run: every record, status, sweep count and
    digest."""
    n = 65536
    b = dcgen.generate(5, n)
    say("c5 65536: generated", b.n_instr)
    summ, oacc, osys = oracle_config(5, n)
    say("c5 65536: oracle done")
    _records_and_summaries(ctx, b, summ, oacc, osys, dc.OPT_DIGEST, True, "c5 65536")


def test_c4_very_large(ctx):
    """All 16 kernels of 1-4M instructions (up to ~17k blocks, which take
    the overflow pass with global-memory bitmaps), alone and interleaved with
    short kernels that take the main pass, in one batch."""
    b4 = dcgen.generate(4, 16)
    say("c4: generated", b4.n_instr)
    summ, oacc, osys = oracle_config(4, 16)
    say("c4: oracle done", int(summ["n_blocks"].max()))
    res = _records_and_summaries(ctx, b4, summ, oacc, osys, dc.OPT_DIGEST, True, "c4")
    assert (res["n_blocks"] > 2048).any()
    b2 = dcgen.generate(2, 48, i0=5000)
    order = [(4, k) for k in range(16)] + [(2, k) for k in range(48)]
    rng = np.random.default_rng(11)
    rng.shuffle(order)
    mix = dcgen.concat([(b4 if c == 4 else b2).kernel(k) for c, k in order])
    ms, ma, my = oracle.analyze_batch(mix)
    _records_and_summaries(ctx, mix, ms, ma, my, dc.OPT_DIGEST, True, "c4 mix")


def test_cfg_parity(ctx):
    b = dcgen.generate(2, 300)
    dev = dc.to_device(b.instrs)
    cfg = ctx.build_cfg(b.kernels, dev, b.n_instr)
    for k in range(b.n_kernels):
        v = cfg.view(k)
        r = oracle.analyze(*b.kernel(k), states=False)
        assert v["status"] == r["status"]
        for key in ("block_start", "succ", "pred_off", "pred", "rpo"):
            assert np.array_equal(v[key], r[key]), (k, key)
        assert v["n_reach"] == r["n_reach"]
    cfg.free()


def _rec(name, r0=0xFFFF, r1=0xFFFF, r2=0xFFFF, imm=0, target=-1):
    x = np.zeros(1, dcgen.INSTR_DTYPE)
    x[0] = (dcgen.opcode(name), r0, r1, r2, imm, target)
    return x


ENTRY_LOOPS = [
    # the entry block jumps to itself
    """
    L0:
      s_add_u32 s20, s20, 1
      s_branch L0
      s_endpgm
    """,
    # a cycle through the entry block of blocks with one predecessor each
    """
    L0:
      s_add_u32 s20, s20, 1
      s_branch L2
      s_endpgm
    L2:
      s_add_u32 s21, s21, s20
      s_branch L0
      s_endpgm
    """,
    # the taken edge returns to the entry, the fall-through has two predecessors
    """
    L0:
      s_add_u32 s20, s20, 1
      s_cmp_lt_u32 s20, 10
      s_cbranch_scc0 L0
    L1:
      s_add_u32 s22, s22, s20
      s_cmp_lt_u32 s22, 5
      s_cbranch_scc1 L3
      s_endpgm
    L3:
      s_branch L1
    """,
]


def test_entry_block_loops(ctx):
    """Kernels whose entry block is its own or a chain's only predecessor: the
    entry block's IN state joins the entry state with the back edge, so it is
    never run as a continuation of another block's visit."""
    ks = []
    for src in ENTRY_LOOPS:
        recs = asmtext.assemble(src)
        ks.append((recs, dcgen.descriptor(len(recs)), np.zeros(0, dcgen.ARG_DTYPE)))
    b = dcgen.concat(ks + [dcgen.generate(2, 3).kernel(k) for k in range(3)])
    res = full_compare(ctx, b)
    assert (res["status"] == 0).all()


MOVE_CHAINS = """
  s_load_dwordx4 s[8:11], s[4:5], 0x30
  s_load_dwordx2 s[2:3], s[4:5], 0x0
  s_mul_i32 s0, s6, 64
  v_add_co_u32 v1, vcc, s0, v0
  s_mov_b64 s[20:21], s[8:9]
  s_mov_b64 s[22:23], s[20:21]
  s_mov_b32 s24, s23
  s_mov_b32 s25, s22
  s_mov_b64 s[26:27], s[24:25]
  s_mov_b64 s[28:29], s[10:11]
  s_mov_b32 s30, 5
  s_mov_b32 s31, s30
  v_mov_b32 v2, v1
  v_mov_b32 v3, v2
  v_mov_b32 v4, 0
  v_mov_b32 v5, v4
  v_lshlrev_b64 v[6:7], 2, v[3:4]
  v_mov_b32 v8, v6
  v_mov_b32 v9, v7
  v_add_co_u32 v10, vcc, s22, v8
  v_mov_b32 v20, s26
  v_mov_b32 v12, v20
  v_addc_co_u32 v11, vcc, v12, v9, vcc
  global_load_dword v14, v[10:11], off
  v_mov_b32 v15, v10
  v_mov_b32 v16, v11
  global_store_dword v[15:16], v14, off
  s_mov_b64 s[32:33], s[2:3]
  s_mov_b32 s34, s32
  v_mov_b32 v17, s34
  v_add_co_u32 v18, vcc, v17, v1
  v_mov_b32 v19, v18
  s_endpgm
"""


def test_move_chains(ctx):
    """Chains of moves: of pairs whose halves come from different
    definitions, of wide SMEM dwords, of constants, of moves of moves, and
    the same chains split across 64-instruction chunks."""
    recs = asmtext.assemble(MOVE_CHAINS)
    pad = asmtext.assemble("\n".join(["  s_nop"] * 40 + ["  s_endpgm"]))[:-1]
    ks = [(recs, dcgen.descriptor(len(recs), n_args=2), None)]
    for cut in (5, 13, 17, 25):
        r2 = np.concatenate([recs[:cut], pad, recs[cut:]])
        ks.append((r2, dcgen.descriptor(len(r2), n_args=2), None))
    args = np.zeros(2, dcgen.ARG_DTYPE)
    args["offset"] = [0x30, 0x38]
    args["size"] = 8
    args["type"] = 16
    args["flags"] = [4, 2]
    b = dcgen.concat([(r, d, args) for r, d, _ in ks])
    res = full_compare(ctx, b)
    assert (res["status"] == 0).all()
    assert (res["n_access"] == 2).all()


def test_errors_do_not_poison_batch(ctx):
    """Bad records, bad descriptors and empty kernels mixed with good ones:
    each kernel gets its own status and the good ones are unaffected."""
    good = dcgen.generate(2, 6)
    parts = [good.kernel(k) for k in range(6)]
    end = _rec("s_endpgm")
    r, d, a = good.kernel(0)
    bad_op = r.copy(); bad_op[5]["op"] = 200
    bad_reg = r.copy(); bad_reg[7]["r0"] = 111
    bad_tgt = r.copy(); bad_tgt[3]["target"] = 5
    no_end = r[:-1].copy()
    d_unsup = d.copy(); d_unsup["useargs"] = 0
    d_dims = d.copy(); d_dims["dims"] = 4
    empty = np.zeros(0, dcgen.INSTR_DTYPE)
    mixed = [parts[0], (bad_op, d, a), parts[1], (bad_reg, d, a), (bad_tgt, d, a), parts[2], (no_end, d, a),
             (r, d_unsup, a), (r, d_dims, a), (empty, dcgen.descriptor(0), np.zeros(0, dcgen.ARG_DTYPE)),
             (end, dcgen.descriptor(1), np.zeros(0, dcgen.ARG_DTYPE)), parts[3], parts[4], parts[5]]
    b = dcgen.concat(mixed)
    res = full_compare(ctx, b)
    want = [0, -10, 0, -11, -12, 0, -13, -14, -14, -13, 0, 0, 0, 0]
    assert list(res["status"]) == want



def test_many_tiny_kernels_per_tile(ctx):
    """Thousands of one- to three-instruction kernels (and empty ones) among a
    few generated kernels: a 4,096-position lookup tile then holds more kernel
    starts than its LDS cache (the per-position search in global memory) and
    more kernels than the decode stage gathers slot marks for in LDS."""
    rng = np.random.default_rng(5)
    gen = dcgen.generate(2, 4, i0=300)
    empty_args = np.zeros(0, dcgen.ARG_DTYPE)
    end = _rec("s_endpgm")
    smov = np.concatenate([_rec("s_mov_b32", r0=8, r1=4), end])
    vmov = np.concatenate([_rec("v_mov_b32", r0=113, r1=112), _rec("s_mov_b32", r0=9, r1=6), end])
    parts = []
    for i in range(6000):
        c = int(rng.integers(0, 10))
        if c < 5:
            parts.append((end, dcgen.descriptor(1), empty_args))
        elif c < 8:
            parts.append((smov, dcgen.descriptor(1), empty_args))
        elif c < 9:
            parts.append((vmov, dcgen.descriptor(2), empty_args))
        else:
            parts.append((np.zeros(0, dcgen.INSTR_DTYPE), dcgen.descriptor(0), empty_args))
        if i % 1500 == 0:
            parts.append(gen.kernel(i // 1500))
    b = dcgen.concat(parts)
    say(f"tiny kernels: {b.n_kernels} kernels, {b.n_instr} instructions")
    assert b.n_kernels / max(1, b.n_instr) > 1026 / 4096
    batch, dev = run(ctx, b, flags=dc.OPT_DIGEST)
    res = batch.results()
    acc, _ = batch.all_accesses()
    sysv, _ = batch.all_sysvals()
    s, oacc, osys = oracle.analyze_batch(b)
    compare_summaries(res, s)
    assert acc.tobytes() == oacc.tobytes() and sysv.tobytes() == osys.tobytes()
    batch.free()


def _nops_like(b):
    """Records of the same layout as b's (every kernel as long as b's) but
    each kernel one straight block of s_nop closed by s_endpgm: one block and
    no records per kernel."""
    recs = np.zeros(b.n_instr, dcgen.INSTR_DTYPE)
    recs["op"] = dcgen.opcode("s_nop")
    recs["r0"] = recs["r1"] = recs["r2"] = dcgen.NONE
    recs["target"] = -1
    ends = (b.kernels["instr_begin"] + b.kernels["n_instr"] - 1).astype(np.int64)
    recs["op"][ends[b.kernels["n_instr"] > 0]] = dcgen.opcode("s_endpgm")
    return recs


def test_rerun_on_other_records_plans_again(ctx):
    """dc_batch_run on a new record pointer: the batch was planned for
    records with one block and no records per kernel; the new records of the
    same layout have loops, hundreds of blocks and thousands of records, and
    the run plans again for them (block arrays, record regions, arenas).
    Every result against the oracle, then back on the first records."""
    b = dcgen.concat([dcgen.generate(2, 300, i0=40).kernel(k) for k in range(300)] +
                     [dcgen.generate(6, 2).kernel(k) for k in range(2)])
    dense = dc.to_device(b.instrs)
    sparse = dc.to_device(_nops_like(b))
    batch = ctx.analyze(b.kernels, sparse, b.n_instr, b.args, flags=dc.OPT_DIGEST)
    res = batch.results()
    assert (res["status"] == 0).all() and (res["n_blocks"] == 1).all() and (res["n_access"] == 0).all()
    s, oacc, osys = oracle.analyze_batch(b)
    batch.run(dense)
    compare_summaries(batch.results(), s)
    assert batch.all_accesses()[0].tobytes() == oacc.tobytes()
    assert batch.all_sysvals()[0].tobytes() == osys.tobytes()
    batch.run(sparse)
    assert batch.results().tobytes() == res.tobytes()
    batch.free()


def test_records_changed_in_place_fail_with_capacity(ctx):
    """Records overwritten in place after planning (the caller's error) with
    more blocks and records than planned: every kernel reports DC_E_CAPACITY
    and no records, nothing is written outside the plan; the same records
    under a new pointer are analysed normally."""
    b = dcgen.generate(2, 200, i0=900)
    buf = dc.to_device(_nops_like(b))
    batch = ctx.analyze(b.kernels, buf, b.n_instr, b.args, flags=dc.OPT_DIGEST)
    assert (batch.results()["status"] == 0).all()
    buf.copy_(dc.to_device(b.instrs))
    torch.cuda.synchronize()
    batch.run()
    res = batch.results()
    assert (res["status"] == -16).all()
    assert len(batch.all_accesses()[0]) == 0 and len(batch.all_sysvals()[0]) == 0
    batch.run(dc.to_device(b.instrs))
    s, oacc, osys = oracle.analyze_batch(b)
    compare_summaries(batch.results(), s)
    assert batch.all_accesses()[0].tobytes() == oacc.tobytes()
    batch.free()

def test_plain_form(ctx):
    """The plain form (one launch per kernel, one workgroup doing every stage):
    the small workload, a sample with loops, kernels of 1,600 to 2,600 blocks
    (bitmaps in global memory past 2,048), malformed and
    unsupported kernels and the hand-written rule kernels, every record,
    status, sweep count and state digest against the oracle, and the same
    bytes as the batched form."""
    import hand_kernels as hk
    good = dcgen.generate(2, 6)
    r, d, a = good.kernel(0)
    bad_op = r.copy()
    bad_op[5]["op"] = 200
    d_unsup = d.copy()
    d_unsup["useargs"] = 0
    parts = [dcgen.generate(1, 32).kernel(k) for k in range(32)] + \
        [dcgen.generate(2, 120, i0=2000).kernel(k) for k in range(120)] + \
        [dcgen.generate(6, 12).kernel(k) for k in (0, 5, 9)] + \
        [(bad_op, d, a), (r, d_unsup, a), (r[:-1].copy(), d, a)] + [k for _, k in hk.all_kernels()]
    b = dcgen.concat(parts)
    dev = dc.to_device(b.instrs)
    s, oacc, osys = oracle.analyze_batch(b)
    plain = ctx.analyze(b.kernels, dev, b.n_instr, b.args, flags=dc.OPT_DIGEST | dc.OPT_PLAIN)
    res = plain.results()
    compare_summaries(res, s)
    assert plain.all_accesses()[0].tobytes() == oacc.tobytes()
    assert plain.all_sysvals()[0].tobytes() == osys.tobytes()
    assert (res["n_blocks"] > 2048).any() and (res["status"] < 0).sum() == 3
    batched = ctx.analyze(b.kernels, dev, b.n_instr, b.args, flags=dc.OPT_DIGEST)
    assert batched.results().tobytes() == res.tobytes()
    plain.run()
    assert plain.results().tobytes() == res.tobytes()
    plain.free()
    batched.free()


def test_nofix_cap(ctx):
    b = dcgen.generate(2, 200)
    s, _, _ = oracle.analyze_batch(b)
    for cap in (1, 2, 3):
        batch, dev = run(ctx, b, sweep_cap=cap, flags=dc.OPT_DIGEST)
        res = batch.results()
        s2, _, _ = oracle.analyze_batch(b, sweep_cap=cap)
        compare_summaries(res, s2)
        assert np.any(res["status"] == -15)
        batch.free()


def test_empty_batch(ctx):
    b = dcgen.concat([])
    dev = torch.zeros(16, dtype=torch.uint8, device="cuda")
    batch = ctx.analyze(b.kernels, dev, 0, b.args)
    assert len(batch.results()) == 0
    acc, off = batch.all_accesses()
    assert len(acc) == 0 and list(off) == [0]
    batch.free()


def test_launch_shapes_invariant(ctx):
    """Batching invariance: waves per group, resident groups and the
    overflow pass (tiny block cap) leave every byte unchanged."""
    b = dcgen.generate(2, 400, i0=1000)
    ref = None
    for kw in [dict(), dict(waves_per_group=1), dict(waves_per_group=2, groups_per_cu=1),
               dict(block_cap=8), dict(block_cap=1, waves_per_group=3)]:
        batch, dev = run(ctx, b, flags=dc.OPT_DIGEST, **kw)
        res = batch.results()
        acc, _ = batch.all_accesses()
        sysv, _ = batch.all_sysvals()
        cur = (res.tobytes(), acc.tobytes(), sysv.tobytes())
        if ref is None:
            ref = cur
            s, oacc, osys = oracle.analyze_batch(b)
            compare_summaries(res, s)
            assert acc.tobytes() == oacc.tobytes() and sysv.tobytes() == osys.tobytes()
        assert cur == ref, kw
        batch.free()


def test_rerun_identical(ctx):
    b = dcgen.generate(2, 300, i0=7)
    batch, dev = run(ctx, b, flags=dc.OPT_DIGEST | dc.OPT_TIMING)
    r1 = batch.results().tobytes()
    a1 = batch.all_accesses()[0].tobytes()
    for _ in range(3):
        batch.run()
        assert batch.results().tobytes() == r1
        assert batch.all_accesses()[0].tobytes() == a1
    st = batch.stats()
    assert st["ms_total"] > 0 and st["n_failed"] == 0
    batch.free()


def test_single_and_alone_vs_batch(ctx):
    """A kernel analysed alone gives the same bytes as inside a batch."""
    b = dcgen.generate(2, 50, i0=321)
    batch, dev = run(ctx, b, flags=dc.OPT_DIGEST)
    res = batch.results()
    for k in (0, 17, 49):
        sub = dcgen.concat([b.kernel(k)])
        b1, d1 = run(ctx, sub, flags=dc.OPT_DIGEST)
        r1 = b1.results()
        assert r1.tobytes() == res[k:k + 1].tobytes()
        assert b1.accesses(0).tobytes() == batch.accesses(k).tobytes()
        b1.free()
    batch.free()


def test_graph_replays_match_eager(ctx):
    """DC_OPT_GRAPH: the stages captured once and replayed give the eager
    results on every replay, with eager work on the same stream between the
    replays (a second batch's runs and a torch operation)."""
    b = dcgen.generate(2, 1500, i0=3000)
    dev = dc.to_device(b.instrs)
    stream = torch.cuda.Stream()
    eager = ctx.analyze(b.kernels, dev, b.n_instr, b.args, flags=dc.OPT_DIGEST, stream=stream)
    ref = (eager.results(), eager.all_accesses()[0], eager.all_sysvals()[0])
    g = ctx.analyze(b.kernels, dev, b.n_instr, b.args, flags=dc.OPT_DIGEST | dc.OPT_GRAPH, stream=stream)
    x = torch.ones(1 << 20, device="cuda")
    for rep in range(5):
        g.run(stream=stream)
        got = (g.results(), g.all_accesses()[0], g.all_sysvals()[0])
        assert got[0].tobytes() == ref[0].tobytes(), rep
        assert got[1].tobytes() == ref[1].tobytes(), rep
        assert got[2].tobytes() == ref[2].tobytes(), rep
        eager.run(stream=stream)
        with torch.cuda.stream(stream):
            x.mul_(1.0001)
        eager.wait()
    # small batches are launch-bound: replaying the graph saves the launches
    s1 = dcgen.generate(1, 32)
    dev1 = dc.to_device(s1.instrs)
    times = {}
    for name, fl in (("eager", 0), ("graph", dc.OPT_GRAPH)):
        bt = ctx.analyze(s1.kernels, dev1, s1.n_instr, s1.args, flags=fl, stream=stream)
        bt.run(stream=stream)
        bt.wait()
        t = time.perf_counter()
        for _ in range(50):
            bt.run(stream=stream)
        bt.wait()
        times[name] = (time.perf_counter() - t) / 50 * 1e3
        bt.free()
    say(f"32-kernel batch: eager {times['eager']:.3f} ms, graph {times['graph']:.3f} ms per run")
    g.free()
    eager.free()


def test_autotune_shape_gives_same_results(ctx):
    """The autotuner's launch shape for a Zipf sample is a valid shape and
    gives byte-identical results to the default shape."""
    b = dcgen.generate(3, 20000, i0=7000)
    dev = dc.to_device(b.instrs)
    shape, ms = ctx.autotune(b.kernels, dev, b.n_instr, b.args, flags=dc.OPT_DIGEST, sample=4096)
    say(f"autotune: {shape}, {ms:.3f} ms per run of the sample")
    assert 1 <= shape["waves_per_group"] <= 4 and shape["groups_per_cu"] >= 1 and ms > 0
    t = time.time()
    again, ms2 = ctx.autotune(b.kernels, dev, b.n_instr, b.args, flags=dc.OPT_DIGEST, sample=4096)
    assert again == shape and ms2 == ms and time.time() - t < 0.5   # the cached choice
    ref = ctx.analyze(b.kernels, dev, b.n_instr, b.args, flags=dc.OPT_DIGEST)
    tuned = ctx.analyze(b.kernels, dev, b.n_instr, b.args, flags=dc.OPT_DIGEST, **shape)
    assert tuned.results().tobytes() == ref.results().tobytes()
    assert tuned.all_accesses()[0].tobytes() == ref.all_accesses()[0].tobytes()
    assert tuned.all_sysvals()[0].tobytes() == ref.all_sysvals()[0].tobytes()
    tuned.free()
    ref.free()
