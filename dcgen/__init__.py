"""Seeded synthetic GCN kernel generator (input synthesis only).

Shared by the oracle's tests and the GPU path's tests and bench.  It knows the
16-byte record encoding and a grammar of compiler-like kernels; it holds none
of the analysis.  The C source is ``dcgen.c``; ``build()`` compiles it.

Records, descriptors and argument tables come back as numpy structured arrays
whose byte layouts are the wire formats:

* record (16 B):   op u16, r0 u16, r1 u16, r2 u16, imm i32, target i32
* kernel (32 B):   instr_begin u64, n_instr u32, dims u8, useargs u8,
                   n_args u16, cws[3] u32, arg_begin u32
* arg (8 B):       offset u32, size u16, type u8, flags u8
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdcgen.so")

INSTR_DTYPE = np.dtype([("op", "<u2"), ("r0", "<u2"), ("r1", "<u2"), ("r2", "<u2"),
                        ("imm", "<i4"), ("target", "<i4")])
KERNEL_DTYPE = np.dtype([("instr_begin", "<u8"), ("n_instr", "<u4"), ("dims", "u1"),
                         ("useargs", "u1"), ("n_args", "<u2"), ("cws", "<u4", (3,)),
                         ("arg_begin", "<u4")])
ARG_DTYPE = np.dtype([("offset", "<u4"), ("size", "<u2"), ("type", "u1"), ("flags", "u1")])
assert INSTR_DTYPE.itemsize == 16 and KERNEL_DTYPE.itemsize == 32 and ARG_DTYPE.itemsize == 8

# operand ids of the record encoding
VCC, EXEC, SCC, M0 = 104, 106, 108, 109
NONE, LIT = 0xFFFF, 0xFFFE
# type-tier bits (argument table `type`, pointee type in `flags`)
T_INT, T_UINT, T_FLOAT, T_DOUBLE, T_PTR = 1, 2, 4, 8, 16


def sreg(n: int) -> int:
    return n


def vreg(n: int) -> int:
    return 112 + n


def iconst(v: int) -> int:
    """Inline integer constant v in [-16, 64]."""
    assert -16 <= v <= 64
    return 0x8000 + v + 16


FCONST_VALUES = (0.5, -0.5, 1.0, -1.0, 2.0, -2.0, 4.0, -4.0)


def fconst(x: float) -> int:
    return 0x8060 + FCONST_VALUES.index(x)


_lib = None


def build(force: bool = False) -> str:
    if force or not os.path.exists(LIB_PATH) or \
            os.path.getmtime(LIB_PATH) < os.path.getmtime(os.path.join(HERE, "dcgen.c")):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-Wall", "-o", tmp,
                               os.path.join(HERE, "dcgen.c"), "-lm", "-lpthread"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        L.dcgen_n_ops.restype = ctypes.c_int
        L.dcgen_op_name.restype = ctypes.c_char_p
        L.dcgen_op_name.argtypes = [ctypes.c_int]
        L.dcgen_sizes.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_uint32,
                                  ctypes.c_void_p, ctypes.c_void_p]
        L.dcgen_generate.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_uint32,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
        L.dcgen_render.restype = ctypes.c_void_p
        L.dcgen_render.argtypes = [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.POINTER(ctypes.c_uint64)]
        L.dcgen_free.argtypes = [ctypes.c_void_p]
        _lib = L
    return _lib


def op_names() -> list[str]:
    L = lib()
    return [L.dcgen_op_name(i).decode() for i in range(L.dcgen_n_ops())]


OPS = None


def opcode(name: str) -> int:
    global OPS
    if OPS is None:
        OPS = {n: i for i, n in enumerate(op_names())}
    return OPS[name]


class Batch:
    """A batch of kernels: records, descriptors, argument table."""

    def __init__(self, instrs, kernels, args):
        self.instrs = instrs
        self.kernels = kernels
        self.args = args

    @property
    def n_kernels(self) -> int:
        return len(self.kernels)

    @property
    def n_instr(self) -> int:
        return len(self.instrs)

    def kernel(self, k: int):
        """(records, descriptor with instr_begin=0/arg_begin=0, args) of kernel k."""
        d = self.kernels[k].copy()
        ib, n, ab, na = int(d["instr_begin"]), int(d["n_instr"]), int(d["arg_begin"]), int(d["n_args"])
        d["instr_begin"] = 0
        d["arg_begin"] = 0
        return self.instrs[ib:ib + n].copy(), d, self.args[ab:ab + na].copy()

    def subset(self, idx) -> "Batch":
        return concat([self.kernel(int(k)) for k in idx])


def sizes(cfg: int, i0: int, n: int):
    ln = np.zeros(n, np.uint32)
    na = np.zeros(n, np.uint32)
    lib().dcgen_sizes(cfg, i0, n, ln.ctypes.data, na.ctypes.data)
    return ln, na


def generate(cfg: int, n: int, i0: int = 0, threads: int | None = None) -> Batch:
    """Kernels [i0, i0+n) of config `cfg` (1..5; 6 is a dense-control-flow test
    shape), packed densely in index order."""
    ln, na = sizes(cfg, i0, n)
    ioff = np.zeros(n, np.uint64)
    aoff = np.zeros(n, np.uint32)
    if n:
        ioff[1:] = np.cumsum(ln[:-1], dtype=np.uint64)
        aoff[1:] = np.cumsum(na[:-1], dtype=np.uint64).astype(np.uint32)
    instrs = np.zeros(int(ln.sum(dtype=np.uint64)), INSTR_DTYPE)
    kernels = np.zeros(n, KERNEL_DTYPE)
    args = np.zeros(int(na.sum(dtype=np.uint64)), ARG_DTYPE)
    if threads is None:
        threads = min(16, os.cpu_count() or 1)
    if n:
        lib().dcgen_generate(cfg, i0, n, ioff.ctypes.data, aoff.ctypes.data, instrs.ctypes.data,
                             kernels.ctypes.data, args.ctypes.data, threads)
    return Batch(instrs, kernels, args)


def concat(parts) -> Batch:
    """Pack (records, descriptor, args) triples into one batch."""
    recs, descs, argl = [], [], []
    ib = ab = 0
    for r, d, a in parts:
        d = np.array(d, KERNEL_DTYPE).reshape(())
        d = d.copy()
        d["instr_begin"] = ib
        d["arg_begin"] = ab
        d["n_instr"] = len(r)
        d["n_args"] = len(a)
        recs.append(np.asarray(r, INSTR_DTYPE))
        descs.append(d)
        argl.append(np.asarray(a, ARG_DTYPE))
        ib += len(r)
        ab += len(a)
    instrs = np.concatenate(recs) if recs else np.zeros(0, INSTR_DTYPE)
    kernels = np.array(descs, KERNEL_DTYPE) if descs else np.zeros(0, KERNEL_DTYPE)
    args = np.concatenate(argl) if argl else np.zeros(0, ARG_DTYPE)
    return Batch(instrs, kernels, args)


def render(batch: Batch) -> bytes:
    """The batch as listing text (the format of the paper's Listings 1 and 3:
    .kernel / .config / .text sections, .dims, .cws, .useargs, .arg lines,
    labels, one instruction per line), with comments, blank lines and tabs
    sprinkled in deterministically."""
    n = ctypes.c_uint64(0)
    kernels = np.ascontiguousarray(batch.kernels)
    instrs = np.ascontiguousarray(batch.instrs)
    args = np.ascontiguousarray(batch.args)
    p = lib().dcgen_render(kernels.ctypes.data if len(kernels) else None, len(kernels),
                           instrs.ctypes.data if len(instrs) else None, args.ctypes.data if len(args) else None,
                           ctypes.byref(n))
    try:
        return ctypes.string_at(p, n.value)
    finally:
        lib().dcgen_free(p)


def descriptor(n_instr: int, dims: int = 1, cws=(64, 1, 1), useargs: int = 1, n_args: int = 0):
    d = np.zeros((), KERNEL_DTYPE)
    d["n_instr"] = n_instr
    d["dims"] = dims
    d["useargs"] = useargs
    d["n_args"] = n_args
    d["cws"] = cws
    return d


def assemble(lines):
    """Tiny assembler for hand-written cases: each line is
    (mnemonic, r0, r1, r2, imm, target) with missing trailing fields
    defaulting to NONE/0/-1; operands are already operand ids."""
    out = np.zeros(len(lines), INSTR_DTYPE)
    for i, ln in enumerate(lines):
        name, *rest = ln
        r = list(rest) + [None] * (5 - len(rest))
        out[i]["op"] = opcode(name)
        out[i]["r0"] = NONE if r[0] is None else r[0]
        out[i]["r1"] = NONE if r[1] is None else r[1]
        out[i]["r2"] = NONE if r[2] is None else r[2]
        out[i]["imm"] = 0 if r[3] is None else r[3]
        out[i]["target"] = -1 if r[4] is None else r[4]
    return out
