"""Pins of the oracle's structuring (Section "Search for control
structures"): the paper's worked trace of Fig. 3 merge by merge, each
template on a hand-written kernel with its expected merges, the search
order, an irreducible graph, and invariants of the region tree on generated
kernels (every reachable block in exactly one leaf, every region merged at
most once, member counts per kind)."""
import numpy as np
import pytest

import asmtext
import dcgen
import oracle

NONE = 0xFFFFFFFF
LIN, IF, IFELSE, WHILE, LOOP = oracle.RG_LINEAR, oracle.RG_IF, oracle.RG_IFELSE, oracle.RG_WHILE, oracle.RG_LOOP


def run(src):
    recs = asmtext.assemble(src)
    r = oracle.structure(recs, dcgen.descriptor(len(recs)))
    assert r["status"] == 0
    return r


def merges(r):
    return [(int(m["region"]), int(m["kind"]), [int(x) for x in m["member"][:m["n"]]]) for m in r["merges"]]


# Fig. 3's region graph: 1 -> 2, 6; 2 -> 3, 6; 3 -> 4; 4 -> 5, 6; 5 -> 6
# (regions #1..#6 are blocks 0..5 here; new regions #7.. are 6..)
FIG3 = """
  s_cmp_eq_u32 s0, 0
  s_cbranch_scc1 B6
  s_cmp_eq_u32 s1, 0
  s_cbranch_scc1 B6
  s_add_u32 s2, s2, 1
  s_branch B4
B4:
  s_cmp_eq_u32 s3, 0
  s_cbranch_scc1 B6
  v_mov_b32 v1, v0
B6:
  s_endpgm
"""


def test_fig3_trace():
    """Section "Search for control structures", the trace of Fig. 3: #4 with
    #5 and #6 is an if template but #6 has other predecessors, so #4 and #5
    merge into #7; #3 and #7 form a linear region #8; #2, #8 (and #6, again
    connected elsewhere) give #9; #1, #9 and #6 give #10, the single
    region."""
    r = run(FIG3)
    assert r["n_blocks"] == 6
    assert merges(r) == [(6, IF, [3, 4]), (7, LIN, [2, 6]), (8, IF, [1, 7]), (9, IF, [0, 8, 5])]
    assert r["n_left"] == 1 and r["root"] == 9


def test_if_else_standard_form():
    """The standard if-else form (a diamond): one merge of header, both arms
    and the join."""
    r = run("""
      s_cmp_eq_u32 s0, 0
      s_cbranch_scc1 ELSE
      s_mov_b32 s1, 1
      s_branch END
    ELSE:
      s_mov_b32 s1, 2
    END:
      s_endpgm
    """)
    assert merges(r) == [(4, IFELSE, [0, 1, 2, 3])] and r["root"] == 4


def test_exec_mask_if_else_reduces_as_two_ifs():
    """The exec-mask if/else the compiler emits (then-arm falls into the else
    test): two if templates, the inner one first."""
    r = run("""
      v_cmp_gt_u32 vcc, v0, 3
      s_and_saveexec_b64 s[20:21], vcc
      s_cbranch_execz ELSE
      v_mov_b32 v5, 1
    ELSE:
      s_or_saveexec_b64 s[20:21], s[20:21]
      s_cbranch_execz END
      v_mov_b32 v5, 2
    END:
      s_or_b64 exec, exec, s[20:21]
      s_endpgm
    """)
    assert merges(r) == [(5, IF, [0, 1, 2]), (6, IF, [5, 3, 4])]


def test_loops():
    """A counted loop whose body is its header (an edge to itself): a loop
    merge; a top-tested loop (header -> body -> header, header -> exit): a
    while merge; a bottom-tested loop over two blocks: a linear merge that
    closes the loop, then a loop merge."""
    r = run("""
      s_mov_b32 s20, 0
    HEAD:
      s_add_u32 s20, s20, 1
      s_cmp_lt_u32 s20, 10
      s_cbranch_scc1 HEAD
      s_endpgm
    """)
    assert merges(r) == [(3, LOOP, [1]), (4, LIN, [0, 3]), (5, LIN, [4, 2])]
    r = run("""
    HEAD:
      s_cmp_lt_u32 s20, 10
      s_cbranch_scc0 EXIT
      s_add_u32 s20, s20, 1
      s_branch HEAD
    EXIT:
      s_endpgm
    """)
    assert merges(r) == [(3, WHILE, [0, 1]), (4, LIN, [3, 2])]
    r = run("""
      s_mov_b32 s20, 0
    TOP:
      s_add_u32 s20, s20, 1
      s_branch NEXT
    NEXT:
      s_cmp_lt_u32 s20, 10
      s_cbranch_scc1 TOP
      s_endpgm
    """)
    assert merges(r) == [(4, LIN, [1, 2]), (5, LOOP, [4]), (6, LIN, [0, 5]), (7, LIN, [6, 3])]


def test_search_order_is_preorder_fall_through_first():
    """Two if templates on the two arms of a branch: the one on the
    fall-through arm is merged first."""
    r = run("""
      s_cmp_eq_u32 s0, 0
      s_cbranch_scc1 RIGHT
      s_cmp_eq_u32 s1, 0
      s_cbranch_scc1 L2
      s_mov_b32 s2, 1
    L2:
      s_branch END
    RIGHT:
      s_cmp_eq_u32 s3, 0
      s_cbranch_scc1 R2
      s_mov_b32 s4, 1
    R2:
      s_nop 0
    END:
      s_endpgm
    """)
    m = merges(r)
    assert m[0][1] == IF and m[0][2][0] == 1 and m[1][1] == IF and m[1][2][0] == 4
    assert r["n_left"] == 1


def test_irreducible_graph_stays_unreduced():
    """Two entries into a cycle (1 <-> 2, each entered from block 0): no
    template applies at the end; several regions are left and there is no
    root."""
    r = run("""
      s_cmp_eq_u32 s0, 0
      s_cbranch_scc1 B2
    B1:
      s_cmp_eq_u32 s1, 0
      s_cbranch_scc1 EXIT
    B2:
      s_cmp_eq_u32 s2, 0
      s_cbranch_scc1 B1
    EXIT:
      s_endpgm
    """)
    assert r["n_left"] > 1 and r["root"] == NONE


def test_unreachable_blocks_take_no_part():
    r = run("""
      s_branch END
      s_mov_b32 s0, 1
    END:
      s_endpgm
    """)
    assert merges(r) == [(3, LIN, [0, 2])] and r["n_left"] == 1


def tree_check(r, reach):
    """Every region is merged at most once, every reachable block ends up in
    exactly one leaf of the root's tree, member counts fit the kinds."""
    nb = r["n_blocks"]
    used = set()
    counts = {LIN: (2,), IF: (2, 3), IFELSE: (3, 4), WHILE: (2,), LOOP: (1,)}
    children = {}
    for reg, kind, mem in merges(r):
        assert len(mem) in counts[kind]
        for x in mem:
            assert x not in used
            used.add(x)
        children[reg] = mem
    if r["n_left"] == 1:
        leaves, stack = [], [r["root"]]
        while stack:
            x = stack.pop()
            if x < nb:
                leaves.append(x)
            else:
                stack.extend(children[x])
        assert sorted(leaves) == sorted(reach)


@pytest.mark.parametrize("cfg,n", [(1, 32), (2, 300), (3, 300), (6, 3)])
def test_generated_kernels_reduce_to_one_region(cfg, n):
    b = dcgen.generate(cfg, n, i0=5)
    s = oracle.structure_batch(b)
    assert (s["status"] == 0).all() and (s["n_left"] == 1).all()
    for k in range(0, n, max(1, n // 40)):
        recs, d, a = b.kernel(k)
        r = oracle.structure(recs, d)
        g = oracle.analyze(recs, d, a, states=False)
        tree_check(r, [int(x) for x in g["rpo"]])
        assert r["digest"] == s[k]["digest"]


def test_if_on_the_taken_edge():
    """An if whose then-arm is the taken successor, placed after the join:
    header, arm and join merge (the join's only predecessors are the two)."""
    r = run("""
      s_cmp_eq_u32 s0, 0
      s_cbranch_scc1 THEN
    JOIN:
      s_endpgm
    THEN:
      s_mov_b32 s1, 1
      s_branch JOIN
    """)
    assert merges(r) == [(3, IF, [0, 2, 1])] and r["root"] == 3


def test_entry_is_never_an_inner_region():
    """A back edge into block 0 from its only successor: the start counts as
    one more predecessor of block 0, so block 1 does not take block 0 as the
    body of a loop; block 0 heads a linear merge that closes the loop."""
    r = run("""
    TOP:
      s_add_u32 s20, s20, 1
      s_branch B1
    B1:
      s_cmp_lt_u32 s20, 10
      s_cbranch_scc1 TOP
      s_endpgm
    """)
    assert merges(r) == [(3, LIN, [0, 1]), (4, LOOP, [3]), (5, LIN, [4, 2])]


def test_entry_is_not_a_loop_body():
    """Block 0 jumps to block 1, which branches back to block 0 or on to
    block 2, which branches back to block 1 or to the end: block 1 has two
    predecessors, so block 0 heads nothing; with the start counted, block 0
    has two predecessors and block 1 cannot take it as the body of a while
    loop.  No template applies anywhere: four regions are left."""
    r = run("""
    E:
      s_nop 0
      s_branch H
    H:
      s_cmp_eq_u32 s0, 0
      s_cbranch_scc1 E
      s_cmp_eq_u32 s1, 0
      s_cbranch_scc1 H
      s_endpgm
    """)
    assert merges(r) == [] and r["n_left"] == 4
