"""Tiny text assembler and fixture reader for hand-written test kernels.

Test infrastructure: turns GCN-style assembly text (the syntax of the
paper's examples, e.g. ``s_load_dwordx2 s[2:3], s[4:5], 0x0``) into the
16-byte records, and reads the golden fixture files under tests/golden/.
Operand placement follows the record encoding (destination in r0, sources in
r1/r2, a third source's operand id in imm, byte offsets in imm).
"""
from __future__ import annotations

import re
import struct

import numpy as np

import dcgen

SPECIAL = {"vcc": 104, "vcc_lo": 104, "vcc_hi": 105, "exec": 106, "exec_lo": 106, "exec_hi": 107,
           "scc": 108, "m0": 109}
TYPES = {"int": dcgen.T_INT, "uint": dcgen.T_UINT, "float": dcgen.T_FLOAT, "double": dcgen.T_DOUBLE,
         "ptr": dcgen.T_PTR}


def reg(tok: str):
    """Register operand id, or None if `tok` is not a register."""
    t = tok.strip().lower()
    if t in SPECIAL:
        return SPECIAL[t]
    m = re.fullmatch(r"([sv])\[(\d+):(\d+)\]", t) or re.fullmatch(r"([sv])(\d+)", t)
    if not m:
        return None
    n = int(m.group(2))
    return n if m.group(1) == "s" else 112 + n


def operand(tok: str):
    """(operand id, literal or None)."""
    r = reg(tok)
    if r is not None:
        return r, None
    t = tok.strip().lower()
    try:
        x = float(t)
        if x in dcgen.FCONST_VALUES and ("." in t):
            return dcgen.fconst(x), None
    except ValueError:
        pass
    v = int(t, 0)
    if v >= 2 ** 31:
        v -= 2 ** 32
    if -16 <= v <= 64:
        return dcgen.iconst(v), None
    return dcgen.LIT, v


SRC2 = {"v_mad_u32_u24", "v_mad_f32", "v_fma_f32", "v_fma_f64"}
CARRY_OUT = {"v_add_co_u32", "v_addc_co_u32", "v_sub_co_u32"}


def assemble(text: str):
    """Assemble text; returns the record array. Labels end with ':'."""
    lines = []
    labels = {}
    for raw in text.splitlines():
        s = raw.split("//")[0].split(";")[0].strip()
        if not s:
            continue
        if s.endswith(":"):
            labels[s[:-1]] = len(lines)
            continue
        lines.append(s)
    recs = np.zeros(len(lines), dcgen.INSTR_DTYPE)
    for i, s in enumerate(lines):
        parts = s.split(None, 1)
        name = parts[0].lower()
        ops = [o.strip() for o in parts[1].split(",")] if len(parts) > 1 else []
        r0 = r1 = r2 = dcgen.NONE
        imm, target = 0, -1
        lit = None

        def src(tok):
            nonlocal lit
            o, l = operand(tok)
            if l is not None:
                lit = l
            return o

        if name.startswith("s_load_"):
            r0, r1, imm = reg(ops[0]), reg(ops[1]), int(ops[2], 0)
        elif name.startswith("s_cbranch") or name == "s_branch":
            target = labels_ref(ops[0], labels)
        elif name in ("s_waitcnt", "s_barrier", "s_nop", "s_endpgm"):
            pass
        elif name.startswith("s_cmp"):
            r1, r2 = src(ops[0]), src(ops[1])
        elif name.startswith("v_cmp"):
            r1, r2 = src(ops[1]), src(ops[2])       # first operand is vcc
        elif name.startswith(("global_load", "flat_load")):
            r0, r1 = reg(ops[0]), reg(ops[1].split()[0])
            r2 = dcgen.NONE if len(ops) < 3 or ops[2].split()[0] == "off" else reg(ops[2].split()[0])
            imm = _offset(s)
        elif name.startswith(("global_store", "flat_store")):
            r1, r0 = reg(ops[0]), reg(ops[1].split()[0])
            r2 = dcgen.NONE if len(ops) < 3 or ops[2].split()[0] == "off" else reg(ops[2].split()[0])
            imm = _offset(s)
        elif name == "ds_read_b32":
            r0, r1 = reg(ops[0]), reg(ops[1].split()[0])
            imm = _offset(s)
        elif name == "ds_write_b32":
            r1, r0 = reg(ops[0]), reg(ops[1].split()[0])
            imm = _offset(s)
        elif name in CARRY_OUT:
            r0, r1, r2 = reg(ops[0]), src(ops[2]), src(ops[3])    # ops[1] is the carry-out vcc
        elif name == "v_cndmask_b32":
            r0, r1, r2 = reg(ops[0]), src(ops[1]), src(ops[2])
        elif name in SRC2:
            r0, r1, r2 = reg(ops[0]), src(ops[1]), src(ops[2])
            imm = operand(ops[3])[0]
        elif len(ops) == 2:
            r0, r1 = reg(ops[0]), src(ops[1])
        else:
            r0, r1, r2 = reg(ops[0]), src(ops[1]), src(ops[2])
        if lit is not None:
            imm = lit
        recs[i] = (dcgen.opcode(name), r0, r1, r2, imm, target)
    return recs


def labels_ref(tok, labels):
    tok = tok.strip()
    if tok in labels:
        return labels[tok]
    return int(tok, 0)


def _offset(s):
    m = re.search(r"offset:(-?\w+)", s)
    return int(m.group(1), 0) if m else 0


# ---------------------------------------------------------------- fixtures

PROV_BITS = {**{f"LID{d}": d for d in range(3)}, **{f"WGID{d}": 3 + d for d in range(3)},
             **{f"GOFF{d}": 6 + d for d in range(3)}, **{f"GSIZE{d}": 9 + d for d in range(3)},
             "WORKDIM": 12, "SYSPTR": 13, "CONST": 14, "LOAD_GLOBAL": 15, "LOAD_LDS": 16, "UNINIT": 17,
             "MASK": 18, "HIDDEN": 19, **{f"KARG{k}": 20 + k for k in range(12)}}
TYPE_BITS = {"INT": 1, "UINT": 2, "FLOAT": 4, "DOUBLE": 8, "PTR": 16}
TAG = {"CONST": 0, "SYSPTR": 1, "KARG": 2, "WGID": 3, "IDX": 4, "SHL": 5, "PTR": 6, "SYS": 7, "UNINIT": 8}
INTEG = {"": 0, "low": 1, "high": 2}
MASK = {"WG": 1, "LID": 2, "GOFF": 4}
SYSKIND = {"GOFF_HI": 0, "GSIZE": 1, "NUMGROUPS": 2, "WORKDIM": 3, "HIDDEN": 4}
SVKIND = {"GLOBAL_ID": 0, "GLOBAL_ID_MINUS_OFFSET": 1, "GLOBAL_OFFSET": 2, "GLOBAL_SIZE": 3,
          "NUM_GROUPS": 4, "WORK_DIM": 5, "GROUP_BASE": 6, "LOCAL_ID": 7, "GROUP_ID": 8}
STATUS = {"OK": 0, "BADOP": -10, "BADREG": -11, "BADTARGET": -12, "NOEND": -13, "UNSUPPORTED": -14,
          "NOFIX": -15}
TOP = 0xFFFFFFFFFFFFFFFF


def parse_val(s: str) -> int:
    """Payload text: TOP | UNINIT | CONST(c) | TAG[.low|.high](k=v,...)."""
    s = s.strip()
    if s == "TOP":
        return TOP
    m = re.fullmatch(r"(\w+)(?:\.(low|high))?(?:\((.*)\))?", s)
    tag, integ, body = m.group(1), m.group(2) or "", m.group(3) or ""
    f = dict(tag=TAG[tag], integ=INTEG[integ], dim=0, aux=0, shift=0, arg=0, c=0)
    if tag == "CONST" and body and "=" not in body:
        f["c"] = int(body, 0) & 0xFFFFFFFF
        body = ""
    for kv in filter(None, (x.strip() for x in body.split(","))):
        k, v = kv.split("=")
        if k == "m":
            f["aux"] = sum(MASK[t] for t in v.split("|")) if not v.isdigit() else int(v)
        elif k == "kind":
            f["aux"] = SYSKIND[v]
        elif k == "d":
            f["dim"] = int(v)
        elif k == "s":
            f["shift"] = int(v)
        elif k == "k":
            f["arg"] = int(v)
        elif k == "c":
            f["c"] = int(v, 0) & 0xFFFFFFFF
    return (f["tag"] << 60) | (f["integ"] << 58) | (f["dim"] << 56) | (f["aux"] << 52) | (f["shift"] << 48) | \
        (f["arg"] << 40) | f["c"]


def parse_bits(s: str, table) -> int:
    s = s.strip()
    if s in ("{}", ""):
        return 0
    return sum(1 << table[t] if table is PROV_BITS else table[t] for t in s.strip("{}").split("|"))


class Fixture:
    def __init__(self, path):
        self.path = path
        self.cite = []
        self.dims, self.cws, self.useargs = 1, (64, 1, 1), 1
        self.args = []
        code, expect = [], []
        mode = None
        for raw in open(path):
            line = raw.rstrip("\n")
            if line.startswith("#"):
                self.cite.append(line[1:].strip())
                continue
            s = line.strip()
            if not s:
                continue
            if s in ("code", "expect"):
                mode = s
                continue
            if mode == "code":
                code.append(s)
            elif mode == "expect":
                expect.append(s)
            else:
                key, *v = s.split()
                if key == "dims":
                    self.dims = int(v[0])
                elif key == "cws":
                    self.cws = tuple(int(x) for x in v)
                elif key == "useargs":
                    self.useargs = int(v[0])
                elif key == "arg":
                    off, size, ty = int(v[0], 0), int(v[1]), TYPES[v[2]]
                    pointee = TYPES[v[3]] if len(v) > 3 else 0
                    self.args.append((off, size, ty, pointee))
        self.records = assemble("\n".join(code))
        self.expect = expect

    def kernel(self):
        d = dcgen.descriptor(len(self.records), self.dims, self.cws, self.useargs, len(self.args))
        a = np.zeros(len(self.args), dcgen.ARG_DTYPE)
        for i, (off, size, ty, pointee) in enumerate(self.args):
            a[i] = (off, size, ty, pointee)
        return self.records, d, a
