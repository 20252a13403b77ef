"""Pins of the oracle's variables and types over the register versions.

Section "Data type recovery": types come from the .arg lines of a kernel's
configuration (Listing 3) and from instruction suffixes, and a suffix types
the operands as well as the result (the paper's example: an unsigned add of
two registers is the sum of two unsigned 32-bit integers).  Section "Search
for control structures": a register whose value at a join depends on the
path becomes a variable when it is used later; the ternary operator is one
instruction.  The hand-written kernels below have their answers worked out
by hand from those statements; the generated kernels check the partitions
against connected components computed by scipy and the live flags against a
breadth-first search, both from the version form alone.
"""
import numpy as np
import pytest
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components

import asmtext
import dcgen
import hand_kernels as hk
import oracle

INT, UINT, FLOAT, DOUBLE, PTR = 1, 2, 4, 8, 16
V = 112   # first vector register slot
VCC, EXEC, SCC = 104, 106, 108


def run(src, dims=1, args=hk.NOARGS):
    recs = asmtext.assemble(src)
    r = oracle.types(recs, dcgen.descriptor(len(recs), dims, (64, 1, 1), 1, len(args)), args)
    assert r["status"] == 0
    nodes = r["nodes"]
    idx = {(int(x["slot"]), int(x["version"])): i for i, x in enumerate(nodes)}
    return r, nodes, idx


def ty(nodes, idx, slot, ver):
    return int(nodes[idx[(slot, ver)]]["type"])


def test_unsigned_add_types_both_operands_and_the_result():
    """The paper's suffix statement, on the one-instruction body it prints."""
    r, nodes, idx = run("s_add_u32 s0, s4, s0\ns_endpgm")
    # nodes: the named slots 0 and 4 and vcc, exec, scc, slots ascending, then versions
    assert [(int(x["slot"]), int(x["version"])) for x in nodes] == \
        [(0, 0), (0, 1), (4, 0), (104, 0), (105, 0), (106, 0), (107, 0), (108, 0), (108, 1)]
    assert ty(nodes, idx, 0, 0) == UINT and ty(nodes, idx, 4, 0) == UINT   # both addends
    assert ty(nodes, idx, 0, 1) == UINT                                     # the sum
    assert ty(nodes, idx, SCC, 1) == 0                                      # the carry is no typed value
    assert nodes[idx[(0, 0)]]["flags"] == oracle.VF_LIVE and nodes[idx[(0, 1)]]["flags"] == 0
    assert r["n_live_merges"] == 0 and r["n_ternary"] == 0


def test_first_suffix_types_the_result_last_suffix_the_source():
    r, nodes, idx = run("""
      v_cvt_f32_u32 v1, v0
      v_cvt_f64_f32 v[2:3], v1
      v_cvt_u32_f32 v4, v1
      v_fma_f32 v5, v6, v7, v8
      s_endpgm""")
    assert ty(nodes, idx, V + 0, 0) == UINT
    assert ty(nodes, idx, V + 1, 1) == FLOAT
    assert ty(nodes, idx, V + 2, 1) == DOUBLE and ty(nodes, idx, V + 3, 1) == DOUBLE
    assert ty(nodes, idx, V + 4, 1) == UINT
    assert all(ty(nodes, idx, V + j, 0) == FLOAT for j in (6, 7, 8))      # the third source too


def test_copies_carry_types_back_but_make_no_variable():
    r, nodes, idx = run("""
      v_mov_b32 v1, v0
      v_add_f32 v2, v1, v1
      s_mov_b64 s[8:9], s[2:3]
      s_add_u32 s10, s8, 1
      s_mul_i32 s11, s9, 3
      s_endpgm""")
    a, b = nodes[idx[(V, 0)]], nodes[idx[(V + 1, 1)]]
    assert int(a["type"]) == FLOAT and int(b["type"]) == FLOAT            # backward through the move
    assert a["tclass"] == b["tclass"] and a["var"] != b["var"]
    # a 64-bit move copies dword by dword: s8 <- s2 (unsigned), s9 <- s3 (signed)
    assert ty(nodes, idx, 2, 0) == UINT and ty(nodes, idx, 3, 0) == INT
    assert ty(nodes, idx, 8, 1) == UINT and ty(nodes, idx, 9, 1) == INT


def test_ternary_is_one_instruction_joining_its_two_values():
    r, nodes, idx = run("""
      v_cmp_gt_u32 vcc, v0, 4
      v_cndmask_b32 v3, v1, v2, vcc
      v_mul_f32 v4, v3, 2.0
      s_endpgm""", dims=3)
    assert r["n_ternary"] == 1
    c = {int(nodes[idx[k]]["tclass"]) for k in [(V + 1, 0), (V + 2, 0), (V + 3, 1)]}
    assert len(c) == 1
    assert ty(nodes, idx, V + 1, 0) == FLOAT and ty(nodes, idx, V + 2, 0) == FLOAT and ty(nodes, idx, V + 3, 1) == FLOAT
    assert ty(nodes, idx, V, 0) == UINT                                    # the compared value
    assert nodes[idx[(VCC, 1)]]["flags"] == oracle.VF_LIVE                 # the condition is read


def test_unreachable_code_types_nothing():
    """Records no path reaches make no versions: they type nothing, read
    nothing and count no ternary."""
    r, nodes, idx = run("""
      s_branch END
      v_cndmask_b32 v3, v1, v2, vcc
      v_mul_f32 v4, v3, 2.0
    END:
      s_endpgm""", dims=3)
    assert r["n_ternary"] == 0
    assert (V + 3, 1) not in idx and (V + 4, 1) not in idx
    assert all(int(x["type"]) == 0 and int(x["flags"]) == 0 for x in nodes)


DIAMOND = """
      v_cmp_gt_u32 vcc, v0, 4
      s_and_saveexec_b64 s[20:21], vcc
      s_cbranch_execz ELSE
      v_mov_b32 v5, 1
      s_branch END
    ELSE:
      v_mov_b32 v5, 2
    END:
      s_or_b64 exec, exec, s[20:21]
{use}
      s_endpgm
"""


def test_join_makes_a_variable_when_the_value_is_used_later():
    """v5 set on both arms reaches the join from two definitions; used after
    it, the merge is a variable of both arms' values and the use's type
    reaches both definitions."""
    r, nodes, idx = run(DIAMOND.format(use="      v_cvt_f32_u32 v6, v5"))
    m, a, b = nodes[idx[(V + 5, 3)]], nodes[idx[(V + 5, 1)]], nodes[idx[(V + 5, 2)]]
    assert m["flags"] == oracle.VF_MERGE | oracle.VF_LIVE
    assert a["flags"] == oracle.VF_LIVE and b["flags"] == oracle.VF_LIVE
    assert m["var"] == a["var"] == b["var"] == idx[(V + 5, 1)]              # the first node of the class
    assert int(m["type"]) == int(a["type"]) == int(b["type"]) == UINT
    assert r["n_live_merges"] == 1
    # without the later use the merge makes no variable and nothing is typed
    r, nodes, idx = run(DIAMOND.format(use=""))
    m = nodes[idx[(V + 5, 3)]]
    assert m["flags"] == oracle.VF_MERGE and int(m["type"]) == 0 and r["n_live_merges"] == 0
    assert m["var"] == idx[(V + 5, 1)]                                      # still one class


LOOP = """
      s_mov_b32 s20, 0
    HEAD:
      s_cmp_eq_u32 s22, 0
      s_cbranch_scc1 SKIP
      s_mov_b32 s20, 7
    SKIP:
      s_cmp_lt_u32 s23, 9
      s_cbranch_scc1 HEAD
      s_add_u32 s24, s20, 1
      s_endpgm
"""


def test_liveness_runs_back_through_chained_merges():
    """Only the exit reads s20, and it reads the inner join's merge; the loop
    header's merge is an argument of it, so it is live as well, and so are
    the definitions feeding both.  scc merges at the header too, but the
    compare there overwrites it before any read: that merge stays dead."""
    r, nodes, idx = run(LOOP)
    head, skip = nodes[idx[(20, 2)]], nodes[idx[(20, 4)]]
    assert head["flags"] == oracle.VF_MERGE | oracle.VF_LIVE and skip["flags"] == oracle.VF_MERGE | oracle.VF_LIVE
    for v in (1, 3):
        assert nodes[idx[(20, v)]]["flags"] == oracle.VF_LIVE
    assert {int(nodes[idx[(20, v)]]["var"]) for v in range(1, 5)} == {idx[(20, 1)]}
    assert {int(nodes[idx[(20, v)]]["type"]) for v in range(1, 5)} == {UINT}
    scc_merges = [x for x in nodes if x["slot"] == SCC and x["flags"] & oracle.VF_MERGE]
    assert len(scc_merges) == 1 and not scc_merges[0]["flags"] & oracle.VF_LIVE
    assert r["n_live_merges"] == 2


def copy_args():
    a = np.zeros(2, dcgen.ARG_DTYPE)
    a[0] = (0x30, 8, PTR, INT)     # int *data
    a[1] = (0x38, 4, INT, 0)       # int x
    return a


def test_argument_loads_take_the_config_types():
    """Listing 3's copy(int *data, int x): the two argument loads take the
    .arg types; the global offset is unsigned, the printf slot untyped; once
    s4 is overwritten the load no longer reads the argument area."""
    r, nodes, idx = run("""
      s_load_dwordx2 s[8:9], s[4:5], 0x30
      s_load_dword s10, s[4:5], 0x38
      s_load_dword s11, s[4:5], 0x0
      s_load_dword s12, s[4:5], 0x18
      s_load_dword s13, s[4:5], 0x40
      s_load_dword s15, s[4:5], 0x20010
      s_mov_b32 s4, 0
      s_load_dword s14, s[4:5], 0x38
      s_endpgm""", args=copy_args())
    assert ty(nodes, idx, 8, 1) == PTR and ty(nodes, idx, 9, 1) == PTR
    assert ty(nodes, idx, 10, 1) == INT
    assert ty(nodes, idx, 11, 1) == UINT and ty(nodes, idx, 15, 1) == UINT
    assert ty(nodes, idx, 12, 1) == 0 and ty(nodes, idx, 13, 1) == 0
    assert ty(nodes, idx, 14, 1) == 0
    assert ty(nodes, idx, 4, 0) == PTR and ty(nodes, idx, 5, 0) == PTR and ty(nodes, idx, 4, 1) == PTR


def test_memory_addresses():
    r, nodes, idx = run("""
      global_load_dword v1, v[2:3], off
      global_store_dword v[4:5], v1, s[8:9]
      flat_store_dword v[6:7], v1
      ds_write_b32 v8, v1
      ds_read_b32 v9, v10
      s_endpgm""")
    assert ty(nodes, idx, V + 2, 0) == PTR and ty(nodes, idx, V + 3, 0) == PTR
    assert ty(nodes, idx, V + 4, 0) == UINT and ty(nodes, idx, V + 5, 0) == UINT   # an offset beside saddr
    assert ty(nodes, idx, 8, 0) == PTR and ty(nodes, idx, 9, 0) == PTR
    assert ty(nodes, idx, V + 6, 0) == PTR and ty(nodes, idx, V + 7, 0) == PTR
    assert ty(nodes, idx, V + 8, 0) == UINT and ty(nodes, idx, V + 10, 0) == UINT
    assert ty(nodes, idx, V + 1, 1) == 0 and ty(nodes, idx, V + 9, 1) == 0         # loaded and stored data


def test_failed_kernel_has_no_nodes():
    recs = asmtext.assemble("v_mov_b32 v1, v0")
    r = oracle.types(recs, dcgen.descriptor(len(recs)), hk.NOARGS)
    assert r["status"] == oracle.E_NOEND and len(r["nodes"]) == 0 and r["digest"] == 0


# ---------------------------------------------------------------- generated kernels

MOVES = {"s_mov_b32", "s_mov_b64", "v_mov_b32"}
NAMES = oracle.op_names()


def components(n, edges):
    """Class representative (the smallest member) of every node."""
    if not edges:
        return np.arange(n)
    e = np.array(edges, np.int64)
    g = coo_matrix((np.ones(len(e)), (e[:, 0], e[:, 1])), shape=(n, n))
    _, lab = connected_components(g, directed=False)
    first = np.full(lab.max() + 1, n)
    np.minimum.at(first, lab, np.arange(n))
    return first[lab]


def check_kernel(recs, d, args):
    r = oracle.types(recs, d, args)
    s = oracle.ssa(recs, d)
    assert r["status"] == s["status"]
    if r["status"] != 0:
        return 0
    nodes = r["nodes"]
    n = len(nodes)
    idx = {(int(x["slot"]), int(x["version"])): i for i, x in enumerate(nodes)}
    # every version of every node's slot is a node, in slot then version order
    assert all(int(nodes[i]["version"]) < int(s["n_ver"][int(nodes[i]["slot"])]) for i in range(n))
    assert sorted(idx) == list(idx)
    merge_edges, copy_edges, read = [], [], set()
    merges = set()
    for p, ph in enumerate(s["phis"]):
        m = idx[(int(ph["slot"]), int(ph["version"]))]
        merges.add(m)
        for a in s["phi_arg"][s["phi_arg_off"][p]:s["phi_arg_off"][p + 1]]:
            merge_edges.append((m, idx[(int(ph["slot"]), int(a))]))
    for i, rec in enumerate(recs):
        us, ds = oracle.ssa_operands(rec)
        if (len(us) and s["use_ver"][i][0] == oracle.SSA_NONE) or (len(ds) and s["def_ver"][i][0] == oracle.SSA_NONE):
            continue
        u = [idx[(sl, int(s["use_ver"][i][q]))] for q, sl in enumerate(us)]
        read.update(u)
        name = NAMES[int(rec["op"])]
        if name in MOVES and int(rec["r1"]) < oracle.NSLOT:
            w = 2 if name == "s_mov_b64" else 1
            for j in range(w):
                copy_edges.append((idx[(ds[j], int(s["def_ver"][i][j]))], u[j]))
        if name == "v_cndmask_b32":
            dst = idx[(ds[0], int(s["def_ver"][i][0]))]
            q = 0
            for f in ("r1", "r2"):
                if int(rec[f]) < oracle.NSLOT:
                    copy_edges.append((dst, u[q]))
                    q += 1
    assert (nodes["var"] == components(n, merge_edges)).all()
    assert (nodes["tclass"] == components(n, merge_edges + copy_edges)).all()
    # one type per type class
    for c in np.unique(nodes["tclass"]):
        assert len(set(nodes["type"][nodes["tclass"] == c].tolist())) == 1
    # live: the nodes read, closed under merge -> argument
    live = set(read)
    stack = [m for m in live if m in merges]
    adj = {}
    for m, a in merge_edges:
        adj.setdefault(m, []).append(a)
    while stack:
        m = stack.pop()
        for a in adj.get(m, []):
            if a not in live:
                live.add(a)
                if a in merges:
                    stack.append(a)
    want = np.array([(oracle.VF_MERGE if i in merges else 0) | (oracle.VF_LIVE if i in live else 0)
                     for i in range(n)], np.uint8)
    assert (nodes["flags"] == want).all()
    assert r["n_live_merges"] == sum(1 for m in merges if m in live)
    return n


@pytest.mark.parametrize("cfg,count", [(1, 24), (2, 40), (3, 30)])
def test_generated_kernels_partitions_and_liveness(cfg, count):
    b = dcgen.generate(cfg, count, i0=5)
    total = 0
    for k in range(count):
        recs, d, args = b.kernel(k)
        if int(d["n_instr"]) > 3000:
            continue
        total += check_kernel(recs, d, args)
    assert total > 0


def test_hand_kernels_partitions_and_liveness():
    for name, (recs, d, args) in hk.all_kernels(n_random=2):
        check_kernel(recs, d, args)


def test_batch_matches_single_kernels():
    b = dcgen.generate(2, 12, i0=40)
    summ = oracle.types_batch(b)
    for k in range(12):
        recs, d, args = b.kernel(k)
        r = oracle.types(recs, d, args)
        assert summ[k]["status"] == r["status"] and summ[k]["digest"] == r["digest"]
        assert summ[k]["n_nodes"] == len(r["nodes"]) and summ[k]["n_ternary"] == r["n_ternary"]
