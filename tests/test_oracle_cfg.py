"""Oracle CFG pins: the textbook basic-block definition, checked by
properties rather than by re-deriving the oracle's own loops.

A partition of the instructions into blocks is the textbook one iff
  (1) block 0 starts at instruction 0 and blocks tile [0, n) in order;
  (2) inside a block no instruction except the last transfers control, and
      no instruction except the first is a branch target (entry only at the
      top, exit only at the bottom);
  (3) each block boundary is forced: the first instruction of a block is a
      branch target or follows a branch/terminator (maximality).
Edges: fall-through to the next block unless the block ends in s_branch or
s_endpgm; a branch adds its target's block; duplicate edges collapse.
Predecessor lists are exactly the transpose of the successor lists, sorted.
The reverse postorder is that of a depth-first search from block 0 that
takes the fall-through edge first."""
import sys

import numpy as np
import pytest

import dcgen
import oracle

NAMES = dcgen.op_names()
BRANCH = {i for i, n in enumerate(NAMES) if n == "s_branch" or n.startswith("s_cbranch")}
UNCOND = {dcgen.opcode("s_branch"), dcgen.opcode("s_endpgm")}
ENDS = BRANCH | {dcgen.opcode("s_endpgm")}


def check_cfg(recs, res):
    n = len(recs)
    ops = recs["op"]
    tg = recs["target"]
    bs = res["block_start"]
    nb = res["n_blocks"]
    targets = {int(tg[i]) for i in range(n) if ops[i] in BRANCH}
    # (1) tiling
    assert bs[0] == 0 and bs[-1] == n and np.all(np.diff(bs) > 0) and len(bs) == nb + 1
    for b in range(nb):
        lo, hi = int(bs[b]), int(bs[b + 1])
        # (2) entry only at the top, exit only at the bottom
        for i in range(lo, hi - 1):
            assert ops[i] not in ENDS
        for i in range(lo + 1, hi):
            assert i not in targets
        # (3) the boundary is forced
        if lo > 0:
            assert lo in targets or ops[lo - 1] in ENDS
    block_of = np.searchsorted(bs, np.arange(n), side="right") - 1
    succ = res["succ"].reshape(nb, 2)
    for b in range(nb):
        last = int(bs[b + 1]) - 1
        want = []
        if ops[last] not in UNCOND and b + 1 < nb:
            want.append(b + 1)
        if ops[last] in BRANCH:
            t = int(block_of[tg[last]])
            if t not in want:
                want.append(t)
        got = [int(s) for s in succ[b] if s >= 0]
        assert got == want, (b, got, want)
        # fall-through slot holds the next block or -1
        assert succ[b][0] in (-1, b + 1)
    # predecessors are the transpose, ascending
    po, pred = res["pred_off"], res["pred"]
    for b in range(nb):
        ps = list(pred[po[b]:po[b + 1]])
        want = [p for p in range(nb) if b in succ[p]]
        assert ps == want
    # reverse postorder of a fall-through-first DFS from block 0
    sys.setrecursionlimit(100000)
    seen, post = set(), []

    def dfs(u):
        seen.add(u)
        for s in succ[u]:
            if s >= 0 and int(s) not in seen:
                dfs(int(s))
        post.append(u)
    dfs(0)
    assert list(res["rpo"]) == post[::-1]
    # every reachable block is reached; nothing else is
    reach = set(post)
    assert set(np.nonzero(res["reached"])[0].tolist()) == reach


@pytest.mark.parametrize("cfg,n", [(1, 32), (2, 120), (3, 200)])
def test_cfg_textbook(cfg, n):
    b = dcgen.generate(cfg, n)
    for k in range(n):
        recs, d, a = b.kernel(k)
        res = oracle.analyze(recs, d, a, states=False)
        assert res["status"] == 0
        check_cfg(recs, res)


def test_c1_shape():
    """C1 kernels: at most 8 blocks, no back edges (acyclic)."""
    b = dcgen.generate(1, 32)
    for k in range(32):
        recs, d, a = b.kernel(k)
        res = oracle.analyze(recs, d, a, states=False)
        assert res["n_blocks"] <= 8
        pos = {int(x): i for i, x in enumerate(res["rpo"])}
        succ = res["succ"].reshape(-1, 2)
        for u in range(res["n_blocks"]):
            for s in succ[u]:
                if s >= 0:
                    assert pos[int(s)] > pos[u]


def test_branch_to_entry_and_unreachable():
    """A back edge into block 0 and code after s_endpgm that nothing targets."""
    import asmtext
    import hand_kernels as hk
    recs = asmtext.assemble(hk.ENTRY_AND_UNREACHABLE)
    d = dcgen.descriptor(len(recs))
    res = oracle.analyze(recs, d, np.zeros(0, dcgen.ARG_DTYPE))
    assert res["status"] == 0
    check_cfg(recs, res)
    assert list(res["reached"]) == [1, 1, 0]
    assert res["in_states"][2].tobytes() == bytes(368 * 16)
    # block 0 is its own predecessor; IN[0] joins the entry with the back edge
    assert list(res["pred"][res["pred_off"][0]:res["pred_off"][1]]) == [0]
    assert res["in_states"][0][20]["val"] == oracle.TOP
