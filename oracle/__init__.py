"""CPU oracle for the register-state dataflow analysis -- TEST INFRASTRUCTURE.

Only tests/, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and
its binding) never does.  The oracle is plain C (``dc_oracle.c``), compiled
with gcc, and shares no code with the GPU path; this module is its ctypes
wrapper.

Parity: pinned by tests/test_oracle_*.py (the paper's worked statements,
textbook basic blocks, meet-over-all-paths for the distributive tiers,
schedule independence, lattice laws; register versions against brute-force
dominators, join sets and path walks; variables and their types against the paper's
suffix statement and hand-derived cases; the text front end against the
paper's Listings 1 and 3 written out by hand and the generator's renderer).  The payload tier beyond the paper's
printed cases is "parity unpinned": only invariants pin it (monotone rules,
meet over all paths below the fixpoint, schedule independence, constant
folding in closed form), since the paper prints no further values.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("DC_ORACLE_LIB") or os.path.join(HERE, "libdcoracle.so")
SRC = os.path.join(HERE, "dc_oracle.c")

NSLOT = 368
SLOT_DTYPE = np.dtype([("prov", "<u4"), ("type", "u1"), ("flags", "u1"), ("pad0", "u1"), ("pad1", "u1"),
                       ("val", "<u8")])
ACCESS_DTYPE = np.dtype([("instr", "<u4"), ("kind", "u1"), ("space", "u1"), ("width", "u1"), ("dtype", "u1"),
                         ("addr", "<u8")])
SYSVAL_DTYPE = np.dtype([("instr", "<u4"), ("slot", "<u2"), ("kind", "u1"), ("dim", "u1")])
SUMMARY_DTYPE = np.dtype([("status", "<i4"), ("n_blocks", "<u4"), ("sweeps", "<u4"), ("n_acc", "<u4"),
                          ("n_sys", "<u4"), ("pad", "<u4"), ("digest", "<u8")])
assert SLOT_DTYPE.itemsize == 16 and ACCESS_DTYPE.itemsize == 16 and SYSVAL_DTYPE.itemsize == 8
assert SUMMARY_DTYPE.itemsize == 32

OK, E_BADOP, E_BADREG, E_BADTARGET, E_NOEND, E_UNSUPPORTED, E_NOFIX = 0, -10, -11, -12, -13, -14, -15
TOP = 0xFFFFFFFFFFFFFFFF


class _Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("n_blocks", ctypes.c_uint32), ("n_reach", ctypes.c_uint32),
                ("sweeps", ctypes.c_uint32), ("n_acc", ctypes.c_uint32), ("n_sys", ctypes.c_uint32),
                ("n_pred", ctypes.c_uint32), ("digest", ctypes.c_uint64),
                ("block_start", ctypes.c_void_p), ("succ", ctypes.c_void_p), ("pred_off", ctypes.c_void_p),
                ("pred", ctypes.c_void_p), ("rpo", ctypes.c_void_p), ("in_states", ctypes.c_void_p),
                ("reached", ctypes.c_void_p), ("acc", ctypes.c_void_p), ("sys", ctypes.c_void_p)]


_lib = None


def build(force: bool = False, extra=()) -> str:
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-Wall", *extra, "-o", tmp, SRC])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        L.or_n_ops.restype = ctypes.c_int
        L.or_op_name.restype = ctypes.c_char_p
        L.or_op_name.argtypes = [ctypes.c_int]
        L.or_kernel_status.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        L.or_kernel_status.restype = ctypes.c_int
        L.or_analyze.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_int,
                                 ctypes.c_uint64, ctypes.POINTER(_Result)]
        L.or_analyze.restype = ctypes.c_int
        L.or_ssa.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.or_ssa.restype = ctypes.c_int
        L.or_ssa_free.argtypes = [ctypes.c_void_p]
        L.or_ssa_batch.argtypes = [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p]
        L.or_ssa_batch.restype = ctypes.c_int
        L.or_structure.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.or_structure.restype = ctypes.c_int
        L.or_structure_free.argtypes = [ctypes.c_void_p]
        L.or_structure_batch.argtypes = [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p]
        L.or_structure_batch.restype = ctypes.c_int
        L.or_types.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.or_types.restype = ctypes.c_int
        L.or_types_free.argtypes = [ctypes.c_void_p]
        L.or_types_batch.argtypes = [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p]
        L.or_types_batch.restype = ctypes.c_int
        L.or_parse_text.argtypes = [ctypes.c_char_p, ctypes.c_uint64, ctypes.c_void_p]
        L.or_parse_text.restype = ctypes.c_int
        L.or_text_free.argtypes = [ctypes.c_void_p]
        L.or_ssa_uses.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        L.or_ssa_uses.restype = ctypes.c_int
        L.or_ssa_defs.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        L.or_ssa_defs.restype = ctypes.c_int
        L.or_analyze_batch.argtypes = [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64)]
        L.or_apply_path.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_uint32, ctypes.c_void_p]
        L.or_apply_path.restype = ctypes.c_int
        L.or_apply_path_from.argtypes = L.or_apply_path.argtypes
        L.or_apply_path_from.restype = ctypes.c_int
        L.or_check_record.argtypes = [ctypes.c_void_p, ctypes.c_uint32]
        L.or_check_record.restype = ctypes.c_int
        L.or_entry_state.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        L.or_transfer.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.or_join.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        _lib = L
    return _lib


def op_names():
    L = lib()
    return [L.or_op_name(i).decode() for i in range(L.or_n_ops())]


def _ptr(a):
    return a.ctypes.data if a is not None and a.size else None


def _desc(desc):
    from dcgen import KERNEL_DTYPE
    d = np.array(desc, KERNEL_DTYPE).reshape(1).copy()
    return d


def kernel_status(recs, desc) -> int:
    d = _desc(desc)
    recs = np.ascontiguousarray(recs)
    return lib().or_kernel_status(d.ctypes.data, _ptr(recs))


def analyze(recs, desc, args, sweep_cap: int = 0, schedule: int = 0, seed: int = 0, states: bool = True) -> dict:
    """Analyse one kernel. Returns a dict of numpy arrays (CFG, IN states,
    accesses, system values) plus status, sweeps and digest."""
    d = _desc(desc)
    n = int(d[0]["n_instr"])
    recs = np.ascontiguousarray(recs)
    args = np.ascontiguousarray(args)
    cap = max(n, 1)
    bs = np.zeros(cap + 1, np.uint32)
    succ = np.zeros(2 * cap, np.int32)
    po = np.zeros(cap + 1, np.uint32)
    pred = np.zeros(2 * cap, np.uint32)
    rpo = np.zeros(cap, np.uint32)
    st = np.zeros(cap * NSLOT if states else 0, SLOT_DTYPE)
    reached = np.zeros(cap, np.uint8)
    acc = np.zeros(cap, ACCESS_DTYPE)
    sys = np.zeros(4 * cap, SYSVAL_DTYPE)
    R = _Result()
    R.block_start, R.succ, R.pred_off, R.pred, R.rpo = bs.ctypes.data, succ.ctypes.data, po.ctypes.data, \
        pred.ctypes.data, rpo.ctypes.data
    R.in_states = st.ctypes.data if states else None
    R.reached, R.acc, R.sys = reached.ctypes.data, acc.ctypes.data, sys.ctypes.data
    lib().or_analyze(d.ctypes.data, _ptr(recs), _ptr(args), sweep_cap, schedule, seed, ctypes.byref(R))
    nb = R.n_blocks
    out = dict(status=R.status, n_blocks=nb, n_reach=R.n_reach, sweeps=R.sweeps, digest=R.digest,
               block_start=bs[:nb + 1] if nb else np.zeros(0, np.uint32), succ=succ[:2 * nb],
               pred_off=po[:nb + 1] if nb else np.zeros(0, np.uint32), pred=pred[:R.n_pred],
               rpo=rpo[:R.n_reach], reached=reached[:nb], accesses=acc[:R.n_acc], sysvals=sys[:R.n_sys])
    if states:
        out["in_states"] = st[:nb * NSLOT].reshape(nb, NSLOT)
    return out


PHI_DTYPE = np.dtype([("block", "<u4"), ("slot", "<u2"), ("pad", "<u2"), ("version", "<u4")])
SSA_NU, SSA_ND, SSA_NONE = 13, 9, 0xFFFFFFFF


class _SsaOut(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("n_blocks", ctypes.c_uint32), ("n_phi", ctypes.c_uint32),
                ("n_args", ctypes.c_uint32), ("idom", ctypes.c_void_p), ("phi", ctypes.c_void_p),
                ("phi_arg_off", ctypes.c_void_p), ("phi_arg", ctypes.c_void_p), ("use_ver", ctypes.c_void_p),
                ("def_ver", ctypes.c_void_p), ("n_ver", ctypes.c_uint32 * NSLOT), ("digest", ctypes.c_uint64)]


def _copy(ptr, n, dt):
    if not n:
        return np.zeros(0, dt)
    return np.ctypeslib.as_array(ctypes.cast(ptr, ctypes.POINTER(ctypes.c_uint8)), shape=(n * np.dtype(dt).itemsize,)) \
        .view(dt).copy()


def ssa(recs, desc) -> dict:
    """Register versions of one kernel (minimal SSA form): immediate
    dominators, phis with their arguments, the version every use reads and
    every definition makes, the versions per slot, and a digest."""
    d = _desc(desc)
    n = int(d[0]["n_instr"])
    recs = np.ascontiguousarray(recs)
    R = _SsaOut()
    L = lib()
    L.or_ssa(d.ctypes.data, _ptr(recs), ctypes.byref(R))
    nb = R.n_blocks
    out = dict(status=R.status, n_blocks=nb, idom=_copy(R.idom, nb, np.uint32), phis=_copy(R.phi, R.n_phi, PHI_DTYPE),
               phi_arg_off=_copy(R.phi_arg_off, R.n_phi + 1, np.uint32), phi_arg=_copy(R.phi_arg, R.n_args, np.uint32),
               use_ver=_copy(R.use_ver, SSA_NU * n, np.uint32).reshape(n, SSA_NU),
               def_ver=_copy(R.def_ver, SSA_ND * n, np.uint32).reshape(n, SSA_ND),
               n_ver=np.array(R.n_ver[:], np.uint32), digest=R.digest)
    L.or_ssa_free(ctypes.byref(R))
    return out


MERGE_DTYPE = np.dtype([("region", "<u4"), ("kind", "u1"), ("n", "u1"), ("pad", "<u2"), ("member", "<u4", (4,))])
RG_LINEAR, RG_IF, RG_IFELSE, RG_WHILE, RG_LOOP = 1, 2, 3, 4, 5
STRUCT_SUMMARY_DTYPE = np.dtype([("status", "<i4"), ("n_blocks", "<u4"), ("n_merges", "<u4"), ("n_left", "<u4"),
                                 ("root", "<u4"), ("pad", "<u4"), ("digest", "<u8")])


class _StructOut(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("n_blocks", ctypes.c_uint32), ("n_merges", ctypes.c_uint32),
                ("n_left", ctypes.c_uint32), ("root", ctypes.c_uint32), ("pad", ctypes.c_uint32),
                ("digest", ctypes.c_uint64), ("merges", ctypes.c_void_p)]


def structure(recs, desc) -> dict:
    """Region-graph structuring of one kernel: the merges in the order they
    were made (new region, kind, members; blocks are regions 0..n_blocks-1),
    the regions left, the root when one is left, and a digest."""
    d = _desc(desc)
    recs = np.ascontiguousarray(recs)
    R = _StructOut()
    L = lib()
    L.or_structure(d.ctypes.data, _ptr(recs), ctypes.byref(R))
    out = dict(status=R.status, n_blocks=R.n_blocks, n_left=R.n_left, root=R.root, digest=R.digest,
               merges=_copy(R.merges, R.n_merges, MERGE_DTYPE))
    L.or_structure_free(ctypes.byref(R))
    return out


def structure_batch(batch):
    summ = np.zeros(batch.n_kernels, STRUCT_SUMMARY_DTYPE)
    lib().or_structure_batch(_ptr(batch.kernels), batch.n_kernels, _ptr(batch.instrs), _ptr(summ))
    return summ


VAR_DTYPE = np.dtype([("slot", "<u2"), ("type", "u1"), ("flags", "u1"), ("version", "<u4"), ("var", "<u4"),
                      ("tclass", "<u4")])
VF_MERGE, VF_LIVE = 1, 2
TYPES_SUMMARY_DTYPE = np.dtype([("status", "<i4"), ("n_nodes", "<u4"), ("n_vars", "<u4"), ("n_tclasses", "<u4"),
                                ("n_live_merges", "<u4"), ("n_ternary", "<u4"), ("digest", "<u8")])
assert VAR_DTYPE.itemsize == 16 and TYPES_SUMMARY_DTYPE.itemsize == 32


class _TypesOut(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("n_nodes", ctypes.c_uint32), ("n_vars", ctypes.c_uint32),
                ("n_tclasses", ctypes.c_uint32), ("n_live_merges", ctypes.c_uint32), ("n_ternary", ctypes.c_uint32),
                ("digest", ctypes.c_uint64), ("nodes", ctypes.c_void_p)]


def types(recs, desc, args) -> dict:
    """Variables and types over the register versions of one kernel: one
    entry per (slot, version) node with its variable (merges joined with
    their arguments), type class (also joined through copies and
    v_cndmask_b32), the class's type bits and the merge / live flags."""
    d = _desc(desc)
    recs = np.ascontiguousarray(recs)
    args = np.ascontiguousarray(args)
    R = _TypesOut()
    L = lib()
    L.or_types(d.ctypes.data, _ptr(recs), _ptr(args), ctypes.byref(R))
    out = dict(status=R.status, n_vars=R.n_vars, n_tclasses=R.n_tclasses, n_live_merges=R.n_live_merges,
               n_ternary=R.n_ternary, digest=R.digest, nodes=_copy(R.nodes, R.n_nodes, VAR_DTYPE))
    L.or_types_free(ctypes.byref(R))
    return out


def types_batch(batch):
    summ = np.zeros(batch.n_kernels, TYPES_SUMMARY_DTYPE)
    lib().or_types_batch(_ptr(batch.kernels), batch.n_kernels, _ptr(batch.instrs), _ptr(batch.args), _ptr(summ))
    return summ


class _TextOut(ctypes.Structure):
    _fields_ = [("n_kernels", ctypes.c_uint32), ("n_instr", ctypes.c_uint64), ("n_args", ctypes.c_uint64),
                ("kernels", ctypes.c_void_p), ("instrs", ctypes.c_void_p), ("args", ctypes.c_void_p),
                ("name_off", ctypes.c_void_p), ("name_len", ctypes.c_void_p)]


def parse_text(text: bytes) -> dict:
    """The text front end: a listing (Listings 1-3 format) to descriptors,
    records and argument tables, plus each kernel's name."""
    from dcgen import ARG_DTYPE, INSTR_DTYPE, KERNEL_DTYPE
    R = _TextOut()
    L = lib()
    L.or_parse_text(text, len(text), ctypes.byref(R))
    k = _copy(R.kernels, R.n_kernels, KERNEL_DTYPE)
    out = dict(kernels=k, instrs=_copy(R.instrs, R.n_instr, INSTR_DTYPE), args=_copy(R.args, R.n_args, ARG_DTYPE))
    off = _copy(R.name_off, R.n_kernels, np.uint64)
    ln = _copy(R.name_len, R.n_kernels, np.uint32)
    out["names"] = [bytes(text[int(o):int(o) + int(n)]) for o, n in zip(off, ln)]
    out["name_off"], out["name_len"] = off, ln
    L.or_text_free(ctypes.byref(R))
    return out


def ssa_operands(rec):
    """(use slots, def slots) of one record in the order the versions are
    reported."""
    u = (ctypes.c_uint * SSA_NU)()
    dd = (ctypes.c_uint * SSA_ND)()
    rec = np.ascontiguousarray(np.asarray(rec).reshape(1))
    nu = lib().or_ssa_uses(_ptr(rec), u)
    nd = lib().or_ssa_defs(_ptr(rec), dd)
    return list(u[:nu]), list(dd[:nd])


SSA_SUMMARY_DTYPE = np.dtype([("status", "<i4"), ("n_blocks", "<u4"), ("n_phi", "<u4"), ("n_args", "<u4"),
                              ("n_operands", "<u4"), ("pad", "<u4"), ("digest", "<u8")])


def ssa_batch(batch):
    """Per-kernel version summaries (status, blocks, merges, merge
    arguments, stored operand versions, digest) for a dcgen.Batch."""
    summ = np.zeros(batch.n_kernels, SSA_SUMMARY_DTYPE)
    lib().or_ssa_batch(_ptr(batch.kernels), batch.n_kernels, _ptr(batch.instrs), _ptr(summ))
    return summ


def analyze_batch(batch, sweep_cap: int = 0):
    """Per-kernel summaries plus dense access/sysval arrays for a dcgen.Batch."""
    n = batch.n_kernels
    N = max(batch.n_instr, 1)
    summ = np.zeros(n, SUMMARY_DTYPE)
    acc = np.zeros(N, ACCESS_DTYPE)
    sys = np.zeros(4 * N, SYSVAL_DTYPE)
    na, ns = ctypes.c_uint64(0), ctypes.c_uint64(0)
    lib().or_analyze_batch(_ptr(batch.kernels), n, _ptr(batch.instrs), _ptr(batch.args), sweep_cap,
                           _ptr(summ), acc.ctypes.data, sys.ctypes.data, ctypes.byref(na), ctypes.byref(ns))
    return summ, acc[:na.value], sys[:ns.value]


def entry_state(desc):
    d = _desc(desc)
    st = np.zeros(NSLOT, SLOT_DTYPE)
    lib().or_entry_state(d.ctypes.data, st.ctypes.data)
    return st


def transfer(desc, args, rec, state):
    """Apply one record to a copy of `state`."""
    d = _desc(desc)
    st = np.array(state, SLOT_DTYPE).copy()
    r = np.ascontiguousarray(np.array(rec).reshape(1))
    args = np.ascontiguousarray(args)
    lib().or_transfer(d.ctypes.data, _ptr(args), r.ctypes.data, st.ctypes.data)
    return st


def join(a, b):
    out = np.array(a, SLOT_DTYPE).copy()
    bb = np.ascontiguousarray(np.array(b, SLOT_DTYPE))
    lib().or_join(out.ctypes.data, bb.ctypes.data)
    return out


def apply_path(recs, desc, args, path):
    d = _desc(desc)
    p = np.array(path, np.uint32)
    out = np.zeros(NSLOT, SLOT_DTYPE)
    recs = np.ascontiguousarray(recs)
    args = np.ascontiguousarray(args)
    rc = lib().or_apply_path(d.ctypes.data, _ptr(recs), _ptr(args), _ptr(p), len(p), out.ctypes.data)
    assert rc == 0
    return out


def apply_blocks(recs, desc, args, state, path):
    """Apply the blocks in `path` to a copy of `state`."""
    d = _desc(desc)
    p = np.array(path, np.uint32)
    st = np.array(state, SLOT_DTYPE).copy()
    recs = np.ascontiguousarray(recs)
    args = np.ascontiguousarray(args)
    rc = lib().or_apply_path_from(d.ctypes.data, _ptr(recs), _ptr(args), _ptr(p), len(p), st.ctypes.data)
    assert rc == 0
    return st


def check_record(rec, n: int) -> int:
    r = np.ascontiguousarray(np.array(rec).reshape(1))
    return lib().or_check_record(r.ctypes.data, n)


# ---- payload encoding helpers (for reading results in tests) ----
TAGS = {0: "CONST", 1: "SYSPTR", 2: "KARG", 3: "WGID", 4: "IDX", 5: "SHL", 6: "PTR", 7: "SYS", 8: "UNINIT",
        15: "TOP"}


def val(tag, integ=0, dim=0, aux=0, shift=0, arg=0, c=0) -> int:
    return (tag << 60) | (integ << 58) | (dim << 56) | (aux << 52) | (shift << 48) | (arg << 40) | (c & 0xFFFFFFFF)


def decode(v: int) -> str:
    v = int(v)
    if v == TOP:
        return "TOP"
    t = v >> 60
    return "%s(integ=%d,d=%d,aux=%d,s=%d,arg=%d,c=%d)" % (TAGS.get(t, t), (v >> 58) & 3, (v >> 56) & 3,
                                                          (v >> 52) & 15, (v >> 48) & 15, (v >> 40) & 255,
                                                          v & 0xFFFFFFFF)
