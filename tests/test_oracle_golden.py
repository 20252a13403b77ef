"""Oracle pins from the paper's worked statements (tests/golden/*.txt).

Each fixture cites the passage it encodes.  `after i r` checks the state
after instruction i of a straight-line prefix (sequential application from
the entry state), `in b r` the fixpoint IN state of block b, `entry r` the
ABI entry state."""
import glob
import os

import numpy as np
import pytest

import asmtext
import oracle

GOLDEN = sorted(glob.glob(os.path.join(os.path.dirname(__file__), "golden", "*.txt")))


def _slot(tok):
    return asmtext.reg(tok)


def check_fixture(fx, res, entry, after_state, where="oracle"):
    """Check expectation lines against an analysis result dict (oracle or GPU)."""
    for line in fx.expect:
        key, *rest = line.split()
        if key == "status":
            assert res["status"] == asmtext.STATUS[rest[0]], (where, line)
        elif key == "nblocks":
            assert res["n_blocks"] == int(rest[0]), (where, line)
        elif key == "sweeps":
            assert res["sweeps"] == int(rest[0]), (where, line)
        elif key in ("after", "in", "entry"):
            if key == "entry":
                if entry is None:
                    continue
                st, slot, fields = entry, _slot(rest[0]), rest[1:]
            elif key == "after":
                if after_state is None:
                    continue
                st, slot, fields = after_state(int(rest[0])), _slot(rest[1]), rest[2:]
            else:
                st, slot, fields = res["in_states"][int(rest[0])], _slot(rest[1]), rest[2:]
            for f in fields:
                k, v = f.split("=", 1)
                if k == "val":
                    assert int(st[slot]["val"]) == asmtext.parse_val(v), \
                        (where, line, oracle.decode(st[slot]["val"]))
                elif k == "prov":
                    assert int(st[slot]["prov"]) == asmtext.parse_bits(v, asmtext.PROV_BITS), (where, line,
                                                                                            hex(st[slot]["prov"]))
                elif k == "type":
                    assert int(st[slot]["type"]) == asmtext.parse_bits(v, asmtext.TYPE_BITS), (where, line,
                                                                                            st[slot]["type"])
        elif key == "sysval":
            i, r, kind, dim = int(rest[0]), _slot(rest[1]), asmtext.SVKIND[rest[2]], int(rest[3])
            sv = res["sysvals"]
            hit = (sv["instr"] == i) & (sv["slot"] == r) & (sv["kind"] == kind) & (sv["dim"] == dim)
            assert hit.sum() == 1, (where, line, sv)
        elif key == "sysvals":
            assert len(res["sysvals"]) == int(rest[0]), (where, line, res["sysvals"])
        elif key == "access":
            i = int(rest[0])
            kind = {"LOAD": 0, "STORE": 1}[rest[1]]
            space = {"GLOBAL": 0, "FLAT": 1, "LDS": 2}[rest[2]]
            width = int(rest[3])
            dtype = asmtext.parse_bits(rest[4], asmtext.TYPE_BITS)
            addr = asmtext.parse_val(rest[5])
            a = res["accesses"]
            row = a[a["instr"] == i]
            assert len(row) == 1, (where, line)
            assert (row["kind"][0], row["space"][0], row["width"][0], row["dtype"][0]) == \
                (kind, space, width, dtype), (where, line, row)
            assert int(row["addr"][0]) == addr, (where, line, oracle.decode(row["addr"][0]))
        elif key == "accesses":
            assert len(res["accesses"]) == int(rest[0]), (where, line)
        else:
            raise AssertionError("unknown expectation " + line)


def oracle_after(recs, desc, args):
    st0 = oracle.entry_state(desc)
    cache = {}

    def after(i):
        if i not in cache:
            st = st0
            for j in range(i + 1):
                st = oracle.transfer(desc, args, recs[j], st)
            cache[i] = st
        return cache[i]
    return after


@pytest.mark.parametrize("path", GOLDEN, ids=[os.path.basename(p) for p in GOLDEN])
def test_golden_oracle(path):
    fx = asmtext.Fixture(path)
    assert fx.cite, "fixture must cite the passage it encodes"
    recs, desc, args = fx.kernel()
    res = oracle.analyze(recs, desc, args)
    assert res["status"] != -99
    check_fixture(fx, res, oracle.entry_state(desc), oracle_after(recs, desc, args))
    # straight-line prefix states agree with the fixpoint machinery on block 0's end
    if res["status"] == 0 and res["n_blocks"] == 1:
        st = oracle_after(recs, desc, args)(len(recs) - 1)
        assert res["in_states"][0].tobytes() == oracle.entry_state(desc).tobytes()
