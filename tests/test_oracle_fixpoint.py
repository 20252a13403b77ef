"""Oracle pins for the fixpoint machinery.

* Meet over all paths (Kildall; Kam & Ullman): for the distributive tiers
  (provenance and type bit sets, unions of inputs plus constant gens) the
  maximal fixpoint equals the union over every entry-to-block path of the
  path's transfer applied to the entry state.  Checked by brute-force path
  enumeration on acyclic graphs, and on small looped graphs by enumerating
  paths with a growing bound until the union stops changing.
* For the payload (a flat lattice, monotone but not distributive) the
  fixpoint is at least as general as the path union: slot by slot it agrees
  or is TOP.
* The least fixpoint is unique, so FIFO and randomly ordered worklists give
  the same bytes as the round-robin reference.
* The sweep cap turns an unconverged iteration into DC_E_NOFIX exactly at
  the pass count the reference schedule needs.
"""
import numpy as np
import pytest

import asmtext
import hand_kernels as hk
import dcgen
import oracle

SL = oracle.SLOT_DTYPE


def union_states(states):
    out = states[0].copy()
    for s in states[1:]:
        out["prov"] |= s["prov"]
        out["type"] |= s["type"]
        out["val"] = np.where(out["val"] == s["val"], out["val"], np.uint64(oracle.TOP))
    return out


def path_union(recs, d, a, res, max_len):
    """Join over all block paths from block 0 with at most max_len blocks
    (the endpoint excluded) of the state reaching each block."""
    nb = res["n_blocks"]
    succ = res["succ"].reshape(nb, 2)
    entry = oracle.entry_state(d)
    acc = {0: [entry]}

    def walk(b, st, depth):
        out = oracle.apply_blocks(recs, d, a, st, [b])
        if depth == max_len:
            return
        for s in succ[b]:
            if s < 0:
                continue
            acc.setdefault(int(s), []).append(out)
            walk(int(s), out, depth + 1)
    walk(0, entry, 1)
    return {b: union_states(v) for b, v in acc.items()}


def check_mop(res, mop, exact_payload=False):
    for b in range(res["n_blocks"]):
        mfp = res["in_states"][b]
        if b not in mop:
            assert res["reached"][b] == 0
            continue
        m = mop[b]
        assert np.array_equal(mfp["prov"], m["prov"]), b
        assert np.array_equal(mfp["type"], m["type"]), b
        same = mfp["val"] == m["val"]
        assert np.all(same | (mfp["val"] == np.uint64(oracle.TOP))), b
        if exact_payload:
            assert np.all(same)


def test_mop_acyclic_c1():
    b = dcgen.generate(1, 32)
    for k in range(32):
        recs, d, a = b.kernel(k)
        res = oracle.analyze(recs, d, a)
        mop = path_union(recs, d, a, res, max_len=res["n_blocks"] + 1)
        check_mop(res, mop)


LOOPS = hk.LOOPS


@pytest.mark.parametrize("src", LOOPS)
def test_mop_cyclic_bounded(src):
    recs = asmtext.assemble(src)
    d = dcgen.descriptor(len(recs), dims=2, cws=(64, 4, 1))
    a = np.zeros(0, dcgen.ARG_DTYPE)
    res = oracle.analyze(recs, d, a)
    assert res["status"] == 0 and res["sweeps"] >= 2
    prev = None
    for L in range(res["n_blocks"], 6 * res["n_blocks"] + 1, res["n_blocks"]):
        mop = path_union(recs, d, a, res, L)
        key = {b: (m["prov"].tobytes(), m["type"].tobytes()) for b, m in mop.items()}
        if key == prev:
            break
        prev = key
    check_mop(res, mop)


def test_schedule_independence():
    """FIFO and random worklist orders reach the same fixpoint bytes."""
    b = dcgen.generate(2, 60)
    for k in range(60):
        recs, d, a = b.kernel(k)
        ref = oracle.analyze(recs, d, a, schedule=0)
        assert ref["status"] == 0
        for sched, seed in [(1, 0), (2, 1), (2, 2), (2, 12345)]:
            r = oracle.analyze(recs, d, a, schedule=sched, seed=seed)
            assert r["status"] == 0
            assert r["in_states"].tobytes() == ref["in_states"].tobytes()
            assert r["reached"].tobytes() == ref["reached"].tobytes()
            assert r["accesses"].tobytes() == ref["accesses"].tobytes()
            assert r["sysvals"].tobytes() == ref["sysvals"].tobytes()
            assert r["digest"] == ref["digest"]


def test_sweep_cap_nofix():
    b = dcgen.generate(2, 300)
    seen = 0
    for k in range(300):
        recs, d, a = b.kernel(k)
        ref = oracle.analyze(recs, d, a, states=False)
        s = ref["sweeps"]
        if s < 2:
            continue
        seen += 1
        assert oracle.analyze(recs, d, a, sweep_cap=s, states=False)["status"] == 0
        r = oracle.analyze(recs, d, a, sweep_cap=s - 1, states=False)
        assert r["status"] == oracle.E_NOFIX
        assert len(r["accesses"]) == 0 and len(r["sysvals"]) == 0 and r["n_blocks"] == 0
        if seen > 20:
            break
    assert seen > 5


def test_acyclic_converges_in_one_sweep():
    """Reverse postorder visits every predecessor first on a DAG."""
    b = dcgen.generate(1, 32)
    s, _, _ = oracle.analyze_batch(b)
    assert np.all(s["status"] == 0) and np.all(s["sweeps"] == 1)


def test_straight_line_is_sequential():
    """One block: IN[0] is the entry state and the extraction walks the
    records in order (sequential evaluation)."""
    recs = asmtext.assemble(hk.STRAIGHT_GLOBAL_ID)
    d = dcgen.descriptor(len(recs))
    res = oracle.analyze(recs, d, np.zeros(0, dcgen.ARG_DTYPE))
    assert res["n_blocks"] == 1
    assert res["in_states"][0].tobytes() == oracle.entry_state(d).tobytes()
    assert [(int(x["instr"]), int(x["slot"]), int(x["kind"])) for x in res["sysvals"]] == \
        [(0, 2, 2), (1, 0, 6), (2, 113, 1), (3, 113, 0), (4, 121, 0)]


def test_batch_matches_single():
    b = dcgen.generate(2, 40)
    s, acc, sys = oracle.analyze_batch(b)
    ia = isy = 0
    for k in range(40):
        r = oracle.analyze(*b.kernel(k))
        assert (s[k]["status"], s[k]["n_blocks"], s[k]["sweeps"], s[k]["digest"]) == \
            (r["status"], r["n_blocks"], r["sweeps"], r["digest"])
        assert acc[ia:ia + len(r["accesses"])].tobytes() == r["accesses"].tobytes()
        assert sys[isy:isy + len(r["sysvals"])].tobytes() == r["sysvals"].tobytes()
        ia += len(r["accesses"])
        isy += len(r["sysvals"])
    assert ia == len(acc) and isy == len(sys)
