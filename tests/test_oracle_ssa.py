"""Pins of the oracle's register versions (minimal SSA form).

Each pin recomputes a textbook definition independently of the oracle's
algorithm, on the oracle's own control flow graph:
  * dominators by reachability with one block removed (d dominates b when b
    cannot be reached from the entry without d), the immediate dominator as
    the strict dominator closest to b;
  * merge (phi) sites as the iterated join set of the defining blocks plus a
    virtual start before block 0: a block is in J(X) when two non-empty paths
    from different members of X reach it and share no block but it (the
    characterisation of minimal SSA by Cytron et al.), by path enumeration on
    small graphs;
  * versions by walking every path from the start: each use must name the
    version the last definition or merge on that path produced, and each
    merge argument the version live at the end of its edge's source;
  * the numbering as defined: per slot, 1, 2, 3, ... over the merges and
    definitions in a preorder walk of the dominator tree (children by
    ascending index), merges first, then instructions in order.
Section "Search for control structures" (a register at a block with several
predecessors can hold the values of different definitions, and the paper
then creates a variable); the version field of the paper's Register record
(Section "Search for memory accesses")."""
import itertools

import numpy as np
import pytest

import asmtext
import dcgen
import hand_kernels as hk
import oracle

NONE = oracle.SSA_NONE


def graph(recs, d, args=None):
    """The oracle's graph of a kernel (states not needed; a kernel's
    argument table is passed when it has one)."""
    if args is None:
        args = np.zeros(int(np.asarray(d)["n_args"]), dcgen.ARG_DTYPE)
    a = oracle.analyze(recs, d, args, states=False)
    nb = a["n_blocks"]
    succ = [[int(s) for s in a["succ"][2 * b:2 * b + 2] if s >= 0] for b in range(nb)]
    return a, nb, succ


def reachable(nb, succ, removed=None):
    seen = set()
    if removed == 0:
        return seen
    stack = [0]
    while stack:
        u = stack.pop()
        if u in seen:
            continue
        seen.add(u)
        stack.extend(v for v in succ[u] if v != removed and v not in seen)
    return seen


def brute_idom(nb, succ):
    reach = reachable(nb, succ)
    dom = {b: {d for d in reach if d == b or b not in reachable(nb, succ, removed=d)} for b in reach}
    idom = [NONE] * nb
    for b in reach:
        if b == 0:
            idom[b] = 0
            continue
        strict = dom[b] - {b}
        # the strict dominator that every other strict dominator dominates
        idom[b] = next(d for d in strict if all(e in dom[d] for e in strict))
    return idom


def kernels_small():
    out = []
    b = dcgen.generate(1, 32)
    out += [b.kernel(k) for k in range(32)]
    b = dcgen.generate(2, 200, i0=300)
    out += [b.kernel(k) for k in range(200) if 0 < b.kernels[k]["n_instr"] <= 600]
    out += [k for _, k in hk.all_kernels() if True]
    return out


def test_dominators_brute_force():
    n = 0
    for recs, d, a in kernels_small():
        _, nb, succ = graph(recs, d)
        if nb > 40:
            continue
        r = oracle.ssa(recs, d)
        assert r["status"] == 0
        assert list(r["idom"]) == brute_idom(nb, succ)
        n += 1
    assert n > 50


def simple_paths(succ, src, dst, start_edge):
    """Non-empty simple paths src ->+ dst (node lists) in the graph with the
    virtual start S (-1) whose only edge is S -> 0."""
    out = []

    def nxt(u):
        return [0] if u == -1 else succ[u]

    def go(u, path):
        for v in nxt(u):
            if v == dst:
                out.append(path + [v])
            elif v not in path and v != -1:
                go(v, path + [v])
    go(src, [src])
    return out


def join_set(succ, X, nb):
    """J(X): blocks y reached by two non-empty paths from different members of
    X that share no block but y."""
    J = set()
    for y in range(nb):
        paths = {x: simple_paths(succ, x, y, True) for x in X}
        found = False
        for x1, x2 in itertools.combinations(sorted(X), 2):
            for p1 in paths[x1]:
                for p2 in paths[x2]:
                    if not (set(p1[:-1]) & set(p2[:-1])):
                        found = True
                        break
                if found:
                    break
            if found:
                break
        if found:
            J.add(y)
    return J


def iterated_join(succ, X, nb):
    J = set()
    while True:
        nj = join_set(succ, set(X) | J, nb)
        if nj == J:
            return J
        J = nj


def defined_blocks(recs, a, nb, reach):
    dfn = {}
    for b in range(nb):
        if b not in reach:
            continue
        for i in range(int(a["block_start"][b]), int(a["block_start"][b + 1])):
            for v in oracle.ssa_operands(recs[i])[1]:
                dfn.setdefault(v, set()).add(b)
    return dfn


def test_phi_sites_are_the_iterated_join_set():
    """Cytron et al.: minimal SSA merges a slot exactly at J+(its defining
    blocks and the start).  Brute force on graphs of at most 9 blocks."""
    n = 0
    for recs, d, _ in kernels_small():
        a, nb, succ = graph(recs, d)
        if nb > 9:
            continue
        reach = reachable(nb, succ)
        r = oracle.ssa(recs, d)
        dfn = defined_blocks(recs, a, nb, reach)
        got = {}
        for p in r["phis"]:
            got.setdefault(int(p["slot"]), set()).add(int(p["block"]))
        for v in set(dfn) | set(got):
            want = iterated_join(succ, dfn.get(v, set()) | {-1}, nb)
            assert got.get(v, set()) == want, (v, got.get(v), want)
        n += 1
    assert n > 20


def walk_paths(succ, nb, max_blocks):
    """Block paths from block 0 with at most max_blocks blocks (all of them on
    acyclic graphs; bounded on loops)."""
    out = []

    def go(path):
        out.append(path)
        if len(path) >= max_blocks:
            return
        for v in succ[path[-1]]:
            go(path + [v])
    go([0])
    return out


def check_paths(recs, d, max_blocks):
    a, nb, succ = graph(recs, d)
    r = oracle.ssa(recs, d)
    phi_at = {(int(p["block"]), int(p["slot"])): i for i, p in enumerate(r["phis"])}
    preds = [[p for p in range(nb) if b in succ[p] and p in reachable(nb, succ)] for b in range(nb)]
    for path in walk_paths(succ, nb, max_blocks):
        cur = {}   # slot -> version live; absent = 0 (the entry value)
        prev = None
        for b in path:
            # merges of b take their argument for the edge from prev
            k_of = ([-1] if b == 0 else []) + preds[b]
            k = k_of.index(prev if prev is not None else -1)
            for (bb, v), i in phi_at.items():
                if bb != b:
                    continue
                arg = r["phi_arg"][r["phi_arg_off"][i] + k]
                assert arg == cur.get(v, 0), (path, b, v)
            for (bb, v), i in phi_at.items():
                if bb == b:
                    cur[v] = int(r["phis"][i]["version"])
            for i in range(int(a["block_start"][b]), int(a["block_start"][b + 1])):
                uses, defs = oracle.ssa_operands(recs[i])
                for q, v in enumerate(uses):
                    assert r["use_ver"][i][q] == cur.get(v, 0), (path, i, v)
                for q, v in enumerate(defs):
                    cur[v] = int(r["def_ver"][i][q])
            prev = b


def test_versions_on_every_path():
    n = 0
    for recs, d, _ in kernels_small():
        a, nb, succ = graph(recs, d)
        if nb > 12:
            continue
        check_paths(recs, d, max_blocks=nb + 3)
        n += 1
    assert n > 20


def test_numbering_is_dominator_tree_preorder():
    """Per slot the merges and definitions are numbered 1, 2, ... in a preorder
    walk of the dominator tree (children ascending), merges before the
    instructions of their block; version 0 is the entry value; n_ver counts
    them all."""
    for recs, d, _ in kernels_small()[:120]:
        a, nb, succ = graph(recs, d)
        r = oracle.ssa(recs, d)
        idom = r["idom"]
        children = {b: sorted(c for c in range(1, nb) if idom[c] == b and idom[c] != NONE) for b in range(nb)}
        order, stack = [], [0]
        while stack:
            b = stack.pop()
            order.append(b)
            stack.extend(reversed(children[b]))
        seen = {}
        phis_of = {}
        for p in r["phis"]:
            phis_of.setdefault(int(p["block"]), []).append(p)
        for b in order:
            for p in sorted(phis_of.get(b, []), key=lambda x: int(x["slot"])):
                v = int(p["slot"])
                seen[v] = seen.get(v, 0) + 1
                assert int(p["version"]) == seen[v]
            for i in range(int(a["block_start"][b]), int(a["block_start"][b + 1])):
                for q, v in enumerate(oracle.ssa_operands(recs[i])[1]):
                    seen[v] = seen.get(v, 0) + 1
                    assert int(r["def_ver"][i][q]) == seen[v]
        for v in range(oracle.NSLOT):
            assert int(r["n_ver"][v]) == 1 + seen.get(v, 0)


DIAMOND = """
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


def test_diamond_and_loop_merges():
    """The paper's case: v5 set on both arms of an if/else reaches the join
    from two definitions, so a merge (a new variable) is made there; v0, set
    only by the ABI, is not merged.  In a loop the counter merges at the
    header, from the entry value and from the latch."""
    recs = asmtext.assemble(DIAMOND)
    r = oracle.ssa(recs, dcgen.descriptor(len(recs)))
    # blocks: 0 (compare, saveexec, branch), 1 (then), 2 (else), 3 (join)
    v5 = 112 + 5
    phis = {(int(p["block"]), int(p["slot"])): i for i, p in enumerate(r["phis"])}
    assert (3, v5) in phis and (3, 112) not in phis
    i = phis[(3, v5)]
    assert list(r["phi_arg"][r["phi_arg_off"][i]:r["phi_arg_off"][i + 1]]) == [1, 2]   # from block 1, from block 2
    assert int(r["phis"][i]["version"]) == 3
    assert r["use_ver"][7][0] == 3 and r["use_ver"][7][1] == 0                          # v_add_u32 reads v5.3, v0.0
    loop = asmtext.assemble("""
      s_mov_b32 s20, 0
    HEAD:
      s_add_u32 s20, s20, 1
      s_cmp_lt_u32 s20, 10
      s_cbranch_scc1 HEAD
      s_endpgm
    """)
    r = oracle.ssa(loop, dcgen.descriptor(len(loop)))
    phis = {(int(p["block"]), int(p["slot"])): i for i, p in enumerate(r["phis"])}
    i = phis[(1, 20)]
    assert list(r["phi_arg"][r["phi_arg_off"][i]:r["phi_arg_off"][i + 1]]) == [1, 3]   # entry edge s20.1, back edge s20.3
    assert int(r["phis"][i]["version"]) == 2 and r["use_ver"][1][0] == 2 and r["def_ver"][1][0] == 3


def test_entry_block_with_a_back_edge_merges_the_entry_value():
    """A back edge into block 0 makes block 0 a join of the start and the
    latch: its merge takes version 0 on the entry edge."""
    recs = asmtext.assemble(hk.ENTRY_AND_UNREACHABLE)
    r = oracle.ssa(recs, dcgen.descriptor(len(recs)))
    phis = {(int(p["block"]), int(p["slot"])): i for i, p in enumerate(r["phis"])}
    i = phis[(0, 20)]
    assert list(r["phi_arg"][r["phi_arg_off"][i]:r["phi_arg_off"][i + 1]]) == [0, 2]
    assert r["idom"][2] == NONE   # the unreachable block
    assert (r["use_ver"][4] == NONE).all() and (r["def_ver"][4] == NONE).all()


def test_failed_kernel_has_no_versions():
    recs = asmtext.assemble("v_mov_b32 v1, v0")
    r = oracle.ssa(recs, dcgen.descriptor(len(recs)))
    assert r["status"] == oracle.E_NOEND and r["n_blocks"] == 0 and len(r["phis"]) == 0


@pytest.mark.parametrize("cfg", [2, 3])
def test_larger_kernels_consistent(cfg):
    """Every use on a bounded set of paths of larger kernels (loops to depth 3)."""
    b = dcgen.generate(cfg, 40, i0=17)
    n = 0
    for k in range(40):
        recs, d, _ = b.kernel(k)
        a, nb, succ = graph(recs, d)
        if nb > 25:
            continue
        check_paths(recs, d, max_blocks=min(nb + 4, 14))
        n += 1
    assert n > 5
