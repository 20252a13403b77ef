"""Python binding of libdc (include/dc.h): argument marshalling only.

Every step of the analysis runs in the HIP kernels of libdc.so; this module
converts numpy/torch buffers to pointers and results back to numpy arrays.
It fails loudly when libdc.so is missing: there is no fallback path.
Device memory and streams come from torch (ROCm).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdc.so")

DC_OK = 0
STATUS = {0: "OK", -1: "INVAL", -2: "HIP", -3: "OOM", -4: "NOTREADY", -10: "BADOP", -11: "BADREG",
          -12: "BADTARGET", -13: "NOEND", -14: "UNSUPPORTED", -15: "NOFIX", -16: "CAPACITY"}
OPT_EXPORT_STATES, OPT_DIGEST, OPT_TIMING, OPT_GRAPH, OPT_LONGEST_FIRST, OPT_PLAIN = 1, 2, 4, 8, 16, 32
NOALLOC_MAX_KERNELS, NOALLOC_MAX_INSTR = 4096, 262144   # DC_NOALLOC_MAX_KERNELS, DC_NOALLOC_MAX_INSTR
NSLOT = 368

INSTR_DTYPE = np.dtype([("op", "<u2"), ("r0", "<u2"), ("r1", "<u2"), ("r2", "<u2"), ("imm", "<i4"),
                        ("target", "<i4")])
KERNEL_DTYPE = np.dtype([("instr_begin", "<u8"), ("n_instr", "<u4"), ("dims", "u1"), ("useargs", "u1"),
                         ("n_args", "<u2"), ("cws", "<u4", (3,)), ("arg_begin", "<u4")])
ARG_DTYPE = np.dtype([("offset", "<u4"), ("size", "<u2"), ("type", "u1"), ("flags", "u1")])
REG_DTYPE = np.dtype([("prov", "<u4"), ("type", "u1"), ("flags", "u1"), ("pad0", "u1"), ("pad1", "u1"),
                      ("val", "<u8")])
ACCESS_DTYPE = np.dtype([("instr", "<u4"), ("kind", "u1"), ("space", "u1"), ("width", "u1"), ("dtype", "u1"),
                         ("addr", "<u8")])
SYSVAL_DTYPE = np.dtype([("instr", "<u4"), ("slot", "<u2"), ("kind", "u1"), ("dim", "u1")])
RESULT_DTYPE = np.dtype([("status", "<i4"), ("n_blocks", "<u4"), ("sweeps", "<u4"), ("n_access", "<u4"),
                         ("n_sysval", "<u4"), ("pad", "<u4"), ("digest", "<u8")])
# register versions (dc_build_ssa)
SSA_NU, SSA_ND, SSA_NONE = 13, 9, 0xFFFFFFFF
PHI_DTYPE = np.dtype([("block", "<u4"), ("slot", "<u2"), ("pad", "<u2"), ("version", "<u4")])
SSA_RESULT_DTYPE = np.dtype([("status", "<i4"), ("n_blocks", "<u4"), ("n_phi", "<u4"), ("n_phi_args", "<u4"),
                             ("n_operands", "<u4"), ("pad", "<u4"), ("digest", "<u8")])
# variables and types (dc_build_types)
VF_MERGE, VF_LIVE = 1, 2
VAR_DTYPE = np.dtype([("slot", "<u2"), ("type", "u1"), ("flags", "u1"), ("version", "<u4"), ("var", "<u4"),
                      ("tclass", "<u4")])
TYPES_RESULT_DTYPE = np.dtype([("status", "<i4"), ("n_nodes", "<u4"), ("n_vars", "<u4"), ("n_tclasses", "<u4"),
                               ("n_live_merges", "<u4"), ("n_ternary", "<u4"), ("digest", "<u8")])
# structuring (dc_structure)
RG_LINEAR, RG_IF, RG_IFELSE, RG_WHILE, RG_LOOP = 1, 2, 3, 4, 5
MERGE_DTYPE = np.dtype([("region", "<u4"), ("kind", "u1"), ("n", "u1"), ("pad", "<u2"), ("member", "<u4", (4,))])
STRUCT_RESULT_DTYPE = np.dtype([("status", "<i4"), ("n_blocks", "<u4"), ("n_merges", "<u4"), ("n_left", "<u4"),
                                ("root", "<u4"), ("pad", "<u4"), ("digest", "<u8")])
# dc_request_t and dc_result_t of the request server
REQUEST_DTYPE = np.dtype([("kernel", KERNEL_DTYPE), ("instrs", "<u8"), ("args", "<u8"), ("tag", "<u8")])
SERVER_RESULT_DTYPE = np.dtype([("ticket", "<u8"), ("tag", "<u8"), ("summary", RESULT_DTYPE), ("accesses", "<u8"),
                                ("sysvals", "<u8"), ("t_submit_ns", "<u8"), ("t_admit_ns", "<u8"),
                                ("t_enqueued_ns", "<u8"), ("t_device_ns", "<u8"), ("t_done_ns", "<u8"), ("batch", "<u8"), ("batch_kernels", "<u4"), ("lane", "<u4")])


class Options(ctypes.Structure):
    _fields_ = [("flags", ctypes.c_uint32), ("sweep_cap", ctypes.c_uint32), ("waves_per_group", ctypes.c_uint32),
                ("groups_per_cu", ctypes.c_uint32), ("block_cap", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32 * 3)]


class Stats(ctypes.Structure):
    _fields_ = [("n_kernels", ctypes.c_uint64), ("n_instr", ctypes.c_uint64), ("n_blocks", ctypes.c_uint64),
                ("n_unreached", ctypes.c_uint64), ("sweeps_sum", ctypes.c_uint64), ("n_access", ctypes.c_uint64),
                ("n_sysval", ctypes.c_uint64), ("bytes_alg", ctypes.c_uint64), ("sweeps_max", ctypes.c_uint32),
                ("n_failed", ctypes.c_uint32), ("n_overflow", ctypes.c_uint32), ("pad", ctypes.c_uint32),
                ("ms_total", ctypes.c_float), ("ms_decode", ctypes.c_float), ("ms_cfg", ctypes.c_float),
                ("ms_fixpoint", ctypes.c_float), ("ms_compact", ctypes.c_float), ("ms_pad", ctypes.c_float)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k not in ("pad", "ms_pad")}


class ServerOpts(ctypes.Structure):
    _fields_ = [("pool_bytes", ctypes.c_uint64), ("lanes", ctypes.c_uint32), ("max_request_instr", ctypes.c_uint32),
                ("max_batch_kernels", ctypes.c_uint32), ("long_instr", ctypes.c_uint32), ("flags", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32 * 3)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("waiting", ctypes.c_uint64),
                ("batches", ctypes.c_uint64), ("max_batch_kernels", ctypes.c_uint64),
                ("device_bytes", ctypes.c_uint64), ("lane_instr", ctypes.c_uint64), ("lanes", ctypes.c_uint32),
                ("pad", ctypes.c_uint32)]


class Timing(ctypes.Structure):
    _fields_ = [("runs", ctypes.c_uint32), ("pad", ctypes.c_uint32), ("ms_total", ctypes.c_float),
                ("ms_decode", ctypes.c_float), ("ms_cfg", ctypes.c_float), ("ms_fixpoint", ctypes.c_float),
                ("ms_compact", ctypes.c_float), ("ms_pad", ctypes.c_float)]


class TextCounts(ctypes.Structure):
    _fields_ = [("n_kernels", ctypes.c_uint32), ("fail", ctypes.c_uint32), ("n_lines", ctypes.c_uint64),
                ("n_instr", ctypes.c_uint64), ("n_args", ctypes.c_uint64)]


class CfgView(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("n_blocks", ctypes.c_uint32), ("n_reach", ctypes.c_uint32),
                ("n_pred", ctypes.c_uint32), ("block_start", ctypes.POINTER(ctypes.c_uint32)),
                ("succ", ctypes.POINTER(ctypes.c_int32)), ("pred_off", ctypes.POINTER(ctypes.c_uint32)),
                ("pred", ctypes.POINTER(ctypes.c_uint32)), ("rpo", ctypes.POINTER(ctypes.c_uint32))]


VP = ctypes.c_void_p
U32, U64, I32 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32

# (name, restype, argtypes): every symbol include/dc.h declares
SIGNATURES = [
    ("dc_ctx_create", I32, [ctypes.c_int, ctypes.POINTER(VP)]),
    ("dc_ctx_destroy", None, [VP]),
    ("dc_build_cfg", I32, [VP, VP, U32, VP, U64, VP, ctypes.POINTER(VP)]),
    ("dc_cfg_view", I32, [VP, U32, ctypes.POINTER(CfgView)]),
    ("dc_cfg_free", None, [VP]),
    ("dc_analyze_batch", I32, [VP, VP, U32, VP, U64, VP, U64, ctypes.POINTER(Options), VP, ctypes.POINTER(VP)]),
    ("dc_batch_run", I32, [VP, VP, VP]),
    ("dc_autotune", I32, [VP, VP, U32, VP, U64, VP, U64, ctypes.POINTER(Options), U32, VP, ctypes.POINTER(Options),
                          ctypes.POINTER(ctypes.c_float)]),
    ("dc_batch_wait", I32, [VP]),
    ("dc_get_kernel_status", I32, [VP, U32, ctypes.POINTER(I32)]),
    ("dc_get_kernel_result", I32, [VP, U32, VP]),
    ("dc_get_results", I32, [VP, VP, U32]),
    ("dc_get_accesses", I32, [VP, U32, VP, U32, ctypes.POINTER(U32)]),
    ("dc_get_sysvals", I32, [VP, U32, VP, U32, ctypes.POINTER(U32)]),
    ("dc_get_all_accesses", I32, [VP, VP, U64, ctypes.POINTER(U64), VP]),
    ("dc_get_all_sysvals", I32, [VP, VP, U64, ctypes.POINTER(U64), VP]),
    ("dc_get_block_state", I32, [VP, U32, U32, VP, ctypes.POINTER(ctypes.c_uint8)]),
    ("dc_get_stats", I32, [VP, ctypes.POINTER(Stats)]),
    ("dc_get_timing", I32, [VP, ctypes.POINTER(Timing)]),
    ("dc_timing_reset", I32, [VP]),
    ("dc_batch_free", None, [VP]),
    ("dc_analyze_noalloc", I32, [VP, VP, U32, U32, VP, U64, VP, U64, U32, VP, VP, U32, VP, VP, U32, VP, VP]),
    ("dc_parse_text", I32, [VP, VP, U64, ctypes.POINTER(Options), VP, ctypes.POINTER(VP)]),
    ("dc_text_run", I32, [VP, VP, U64]),
    ("dc_text_wait", I32, [VP]),
    ("dc_text_get_counts", I32, [VP, ctypes.POINTER(TextCounts)]),
    ("dc_text_device_arrays", I32, [VP, ctypes.POINTER(VP), ctypes.POINTER(VP), ctypes.POINTER(VP)]),
    ("dc_text_get_kernels", I32, [VP, VP, U32, ctypes.POINTER(U32)]),
    ("dc_text_get_records", I32, [VP, VP, U64, ctypes.POINTER(U64)]),
    ("dc_text_get_args", I32, [VP, VP, U64, ctypes.POINTER(U64)]),
    ("dc_text_get_names", I32, [VP, VP, VP, U32, ctypes.POINTER(U32)]),
    ("dc_text_get_timing", I32, [VP, ctypes.POINTER(Timing)]),
    ("dc_text_timing_reset", I32, [VP]),
    ("dc_text_free", None, [VP]),
    ("dc_structure", I32, [VP, VP, U32, VP, U64, ctypes.POINTER(Options), VP, ctypes.POINTER(VP)]),
    ("dc_struct_run", I32, [VP, VP]),
    ("dc_struct_wait", I32, [VP]),
    ("dc_struct_get_results", I32, [VP, VP, U32]),
    ("dc_struct_get_merges", I32, [VP, U32, VP, U32, ctypes.POINTER(U32)]),
    ("dc_struct_get_timing", I32, [VP, ctypes.POINTER(Timing)]),
    ("dc_struct_timing_reset", I32, [VP]),
    ("dc_struct_free", None, [VP]),
    ("dc_build_ssa", I32, [VP, VP, U32, VP, U64, ctypes.POINTER(Options), VP, ctypes.POINTER(VP)]),
    ("dc_ssa_run", I32, [VP, VP]),
    ("dc_ssa_wait", I32, [VP]),
    ("dc_ssa_get_results", I32, [VP, VP, U32]),
    ("dc_ssa_get_idom", I32, [VP, U32, VP, U32, ctypes.POINTER(U32)]),
    ("dc_ssa_get_phis", I32, [VP, U32, VP, U32, ctypes.POINTER(U32)]),
    ("dc_ssa_get_phi_args", I32, [VP, U32, VP, U32, ctypes.POINTER(U32)]),
    ("dc_ssa_get_versions", I32, [VP, U32, VP, VP, U32, ctypes.POINTER(U32)]),
    ("dc_ssa_get_timing", I32, [VP, ctypes.POINTER(Timing)]),
    ("dc_ssa_timing_reset", I32, [VP]),
    ("dc_ssa_free", None, [VP]),
    ("dc_build_types", I32, [VP, VP, U32, VP, U64, VP, U64, ctypes.POINTER(Options), VP, ctypes.POINTER(VP)]),
    ("dc_types_get_results", I32, [VP, VP, U32]),
    ("dc_types_get_vars", I32, [VP, U32, VP, U32, ctypes.POINTER(U32)]),
    ("dc_server_create", I32, [VP, ctypes.POINTER(ServerOpts), ctypes.POINTER(VP)]),
    ("dc_server_submit", I32, [VP, VP, ctypes.POINTER(U64)]),
    ("dc_server_poll", I32, [VP, VP, U32, ctypes.POINTER(U32)]),
    ("dc_server_get_stats", I32, [VP, ctypes.POINTER(ServerStats)]),
    ("dc_server_destroy", None, [VP]),
    ("dc_status_str", ctypes.c_char_p, [I32]),
    ("dc_opcode_count", ctypes.c_int, []),
    ("dc_opcode_name", ctypes.c_char_p, [ctypes.c_int]),
]

_lib = None


class DCError(RuntimeError):
    def __init__(self, where, code):
        super().__init__(f"{where}: {STATUS.get(code, code)} ({code})")
        self.code = code


def lib():
    """Load libdc.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(where, code):
    if code != DC_OK:
        raise DCError(where, code)


def opcode_names():
    L = lib()
    return [L.dc_opcode_name(i).decode() for i in range(L.dc_opcode_count())]


def status_str(code: int) -> str:
    return lib().dc_status_str(code).decode()


def _np_ptr(a):
    return a.ctypes.data if a is not None and a.size else None


class DevicePtr:
    """A raw device address owned elsewhere (e.g. a library object's output
    array), usable wherever a device tensor is taken."""

    def __init__(self, addr: int, owner=None):
        self.addr = addr
        self.owner = owner      # keeps the owning object alive

    def data_ptr(self) -> int:
        return self.addr

    def numel(self) -> int:
        return 1 if self.addr else 0


def _dev_ptr(t):
    return t.data_ptr() if t is not None and t.numel() else None


def _stream_ptr(stream):
    if stream is None:
        return None
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def text_to_device(text: bytes, device="cuda:0"):
    """A listing's bytes as a uint8 tensor on the device (at least one byte)."""
    import torch
    buf = np.frombuffer(text, np.uint8) if text else np.zeros(1, np.uint8)
    return torch.from_numpy(buf.copy()).to(device)


def to_device(records: np.ndarray, device="cuda:0"):
    """Records (numpy, INSTR_DTYPE) -> a torch uint8 tensor on the GPU."""
    import torch
    raw = np.ascontiguousarray(records).view(np.uint8).reshape(-1)
    return torch.from_numpy(raw).to(device)


class Context:
    def __init__(self, device: int = 0):
        h = VP()
        check("dc_ctx_create", lib().dc_ctx_create(device, ctypes.byref(h)))
        self.h = h
        self.device = device

    def close(self):
        if self.h:
            lib().dc_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def analyze(self, kernels, instrs_dev, n_records, args=None, flags=0, sweep_cap=0, waves_per_group=0,
                groups_per_cu=0, block_cap=0, stream=None, longest_first=False) -> "Batch":
        flags |= OPT_LONGEST_FIRST if longest_first else 0
        kernels = np.ascontiguousarray(np.asarray(kernels, KERNEL_DTYPE))
        args = np.ascontiguousarray(np.asarray(args if args is not None else np.zeros(0, ARG_DTYPE), ARG_DTYPE))
        o = Options(flags, sweep_cap, waves_per_group, groups_per_cu, block_cap)
        h = VP()
        check("dc_analyze_batch", lib().dc_analyze_batch(self.h, _np_ptr(kernels), len(kernels), _dev_ptr(instrs_dev),
                                                         n_records, _np_ptr(args), len(args), ctypes.byref(o),
                                                         _stream_ptr(stream), ctypes.byref(h)))
        return Batch(h, len(kernels), instrs_dev, stream)

    def autotune(self, kernels, instrs_dev, n_records, args=None, flags=0, sample=0, stream=None):
        """Fastest fixpoint launch shape and kernel order on a sample of the
        batch: (dict of options for analyze(), ms per run of the sample)."""
        kernels = np.ascontiguousarray(np.asarray(kernels, KERNEL_DTYPE))
        args = np.ascontiguousarray(np.asarray(args if args is not None else np.zeros(0, ARG_DTYPE), ARG_DTYPE))
        base = Options(flags, 0, 0, 0, 0)
        best = Options()
        ms = ctypes.c_float()
        check("dc_autotune", lib().dc_autotune(self.h, _np_ptr(kernels), len(kernels), _dev_ptr(instrs_dev), n_records,
                                               _np_ptr(args), len(args), ctypes.byref(base), sample,
                                               _stream_ptr(stream), ctypes.byref(best), ctypes.byref(ms)))
        return {"waves_per_group": best.waves_per_group, "groups_per_cu": best.groups_per_cu,
                "longest_first": bool(best.flags & OPT_LONGEST_FIRST)}, ms.value

    def analyze_noalloc(self, kernels_dev, n_kernels, n_instr_total, instrs_dev, n_records, args_dev, n_args_total,
                        results_dev, acc_dev, acc_cap, acc_off_dev, sys_dev, sys_cap, sys_off_dev, flags=0,
                        stream=None):
        """dc_analyze_noalloc: every argument a device tensor (or a count);
        enqueues the analysis and returns (the outputs are filled when the
        stream reaches the work)."""
        check("dc_analyze_noalloc", lib().dc_analyze_noalloc(
            self.h, _dev_ptr(kernels_dev), n_kernels, n_instr_total, _dev_ptr(instrs_dev), n_records,
            _dev_ptr(args_dev), n_args_total, flags, _dev_ptr(results_dev), _dev_ptr(acc_dev), acc_cap,
            _dev_ptr(acc_off_dev), _dev_ptr(sys_dev), sys_cap, _dev_ptr(sys_off_dev), _stream_ptr(stream)))

    def build_cfg(self, kernels, instrs_dev, n_records, stream=None) -> "Cfg":
        kernels = np.ascontiguousarray(np.asarray(kernels, KERNEL_DTYPE))
        h = VP()
        check("dc_build_cfg", lib().dc_build_cfg(self.h, _np_ptr(kernels), len(kernels), _dev_ptr(instrs_dev),
                                                 n_records, _stream_ptr(stream), ctypes.byref(h)))
        return Cfg(h, len(kernels))

    def parse_text(self, text_dev, n_bytes, timing=False, stream=None) -> "Text":
        """The text front end on a listing already in device memory (a uint8
        tensor, see text_to_device)."""
        o = Options()
        o.flags = OPT_TIMING if timing else 0
        h = VP()
        check("dc_parse_text", lib().dc_parse_text(self.h, _dev_ptr(text_dev), n_bytes, ctypes.byref(o),
                                                   _stream_ptr(stream), ctypes.byref(h)))
        return Text(h, text_dev, n_bytes)

    def structure(self, kernels, instrs_dev, n_records, timing=False, stream=None) -> "Struct":
        kernels = np.ascontiguousarray(np.asarray(kernels, KERNEL_DTYPE))
        o = Options()
        o.flags = OPT_TIMING if timing else 0
        h = VP()
        check("dc_structure", lib().dc_structure(self.h, _np_ptr(kernels), len(kernels), _dev_ptr(instrs_dev),
                                                 n_records, ctypes.byref(o), _stream_ptr(stream), ctypes.byref(h)))
        return Struct(h, kernels, instrs_dev)

    def build_ssa(self, kernels, instrs_dev, n_records, timing=False, digest=True, stream=None) -> "Ssa":
        kernels = np.ascontiguousarray(np.asarray(kernels, KERNEL_DTYPE))
        o = Options()
        o.flags = (OPT_TIMING if timing else 0) | (OPT_DIGEST if digest else 0)
        h = VP()
        check("dc_build_ssa", lib().dc_build_ssa(self.h, _np_ptr(kernels), len(kernels), _dev_ptr(instrs_dev),
                                                 n_records, ctypes.byref(o), _stream_ptr(stream), ctypes.byref(h)))
        return Ssa(h, kernels, instrs_dev)

    def build_types(self, kernels, instrs_dev, n_records, args=None, timing=False, digest=True,
                    stream=None) -> "Ssa":
        """Versions plus variables and types (dc_build_types); the object's
        types() and vars(k) read the latter."""
        kernels = np.ascontiguousarray(np.asarray(kernels, KERNEL_DTYPE))
        args = np.ascontiguousarray(np.asarray(args if args is not None else np.zeros(0, ARG_DTYPE), ARG_DTYPE))
        o = Options()
        o.flags = (OPT_TIMING if timing else 0) | (OPT_DIGEST if digest else 0)
        h = VP()
        check("dc_build_types", lib().dc_build_types(self.h, _np_ptr(kernels), len(kernels), _dev_ptr(instrs_dev),
                                                     n_records, _np_ptr(args), len(args), ctypes.byref(o),
                                                     _stream_ptr(stream), ctypes.byref(h)))
        return Ssa(h, kernels, instrs_dev)


class Batch:
    def __init__(self, h, n_kernels, instrs_dev, stream):
        self.h = h
        self.n_kernels = n_kernels
        self._keep = instrs_dev     # caller memory must outlive the run
        self.stream = stream

    def run(self, instrs_dev=None, stream=None):
        if instrs_dev is not None:
            self._keep = instrs_dev
        check("dc_batch_run", lib().dc_batch_run(self.h, _dev_ptr(instrs_dev) if instrs_dev is not None else None,
                                                 _stream_ptr(stream if stream is not None else self.stream)))

    def wait(self):
        check("dc_batch_wait", lib().dc_batch_wait(self.h))

    def results(self) -> np.ndarray:
        out = np.zeros(self.n_kernels, RESULT_DTYPE)
        check("dc_get_results", lib().dc_get_results(self.h, _np_ptr(out), self.n_kernels))
        return out

    def status(self, k: int) -> int:
        s = I32()
        check("dc_get_kernel_status", lib().dc_get_kernel_status(self.h, k, ctypes.byref(s)))
        return s.value

    def accesses(self, k: int) -> np.ndarray:
        n = U32()
        check("dc_get_accesses", lib().dc_get_accesses(self.h, k, None, 0, ctypes.byref(n)))
        out = np.zeros(n.value, ACCESS_DTYPE)
        check("dc_get_accesses", lib().dc_get_accesses(self.h, k, _np_ptr(out), n.value, ctypes.byref(n)))
        return out

    def sysvals(self, k: int) -> np.ndarray:
        n = U32()
        check("dc_get_sysvals", lib().dc_get_sysvals(self.h, k, None, 0, ctypes.byref(n)))
        out = np.zeros(n.value, SYSVAL_DTYPE)
        check("dc_get_sysvals", lib().dc_get_sysvals(self.h, k, _np_ptr(out), n.value, ctypes.byref(n)))
        return out

    def all_accesses(self):
        n = U64()
        check("dc_get_all_accesses", lib().dc_get_all_accesses(self.h, None, 0, ctypes.byref(n), None))
        out = np.zeros(n.value, ACCESS_DTYPE)
        off = np.zeros(self.n_kernels + 1, np.uint64)
        check("dc_get_all_accesses", lib().dc_get_all_accesses(self.h, _np_ptr(out), n.value, ctypes.byref(n),
                                                               off.ctypes.data))
        return out, off

    def all_sysvals(self):
        n = U64()
        check("dc_get_all_sysvals", lib().dc_get_all_sysvals(self.h, None, 0, ctypes.byref(n), None))
        out = np.zeros(n.value, SYSVAL_DTYPE)
        off = np.zeros(self.n_kernels + 1, np.uint64)
        check("dc_get_all_sysvals", lib().dc_get_all_sysvals(self.h, _np_ptr(out), n.value, ctypes.byref(n),
                                                             off.ctypes.data))
        return out, off

    def block_state(self, k: int, b: int):
        out = np.zeros(NSLOT, REG_DTYPE)
        r = ctypes.c_uint8()
        check("dc_get_block_state", lib().dc_get_block_state(self.h, k, b, out.ctypes.data, ctypes.byref(r)))
        return out, r.value

    def stats(self) -> dict:
        s = Stats()
        check("dc_get_stats", lib().dc_get_stats(self.h, ctypes.byref(s)))
        return s.as_dict()

    def timing(self) -> dict:
        t = Timing()
        check("dc_get_timing", lib().dc_get_timing(self.h, ctypes.byref(t)))
        return {k: getattr(t, k) for k, _ in t._fields_ if k not in ("pad", "ms_pad")}

    def timing_reset(self):
        check("dc_timing_reset", lib().dc_timing_reset(self.h))

    def free(self):
        if self.h:
            lib().dc_batch_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Cfg:
    def __init__(self, h, n_kernels):
        self.h = h
        self.n_kernels = n_kernels

    def view(self, k: int) -> dict:
        v = CfgView()
        check("dc_cfg_view", lib().dc_cfg_view(self.h, k, ctypes.byref(v)))
        nb = v.n_blocks

        def arr(p, n, dt):
            return np.ctypeslib.as_array(p, shape=(n,)).astype(dt).copy() if n else np.zeros(0, dt)
        if v.status != DC_OK:
            return dict(status=v.status, n_blocks=0)
        return dict(status=v.status, n_blocks=nb, n_reach=v.n_reach,
                    block_start=arr(v.block_start, nb + 1, np.uint32), succ=arr(v.succ, 2 * nb, np.int32),
                    pred_off=arr(v.pred_off, nb + 1, np.uint32), pred=arr(v.pred, v.n_pred, np.uint32),
                    rpo=arr(v.rpo, v.n_reach, np.uint32))

    def free(self):
        if self.h:
            lib().dc_cfg_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def requests(kernels, instrs, args=None, tags=None) -> np.ndarray:
    """dc_request_t array for kernels[k] of a packed batch: pointers into
    `instrs` and `args`, which must stay alive until the requests are
    submitted (dc_server_submit copies them)."""
    kernels = np.asarray(kernels, KERNEL_DTYPE)
    out = np.zeros(len(kernels), REQUEST_DTYPE)
    out["kernel"] = kernels
    out["kernel"]["instr_begin"] = 0
    out["kernel"]["arg_begin"] = 0
    ib = instrs.ctypes.data if instrs.size else 0
    ab = args.ctypes.data if args is not None and args.size else 0
    out["instrs"] = ib + kernels["instr_begin"].astype(np.uint64) * np.uint64(INSTR_DTYPE.itemsize)
    out["args"] = ab + kernels["arg_begin"].astype(np.uint64) * np.uint64(ARG_DTYPE.itemsize)
    out["tag"] = np.arange(len(kernels), dtype=np.uint64) if tags is None else tags
    return out


class Server:
    """dc_server_*: continuous batching of single-kernel requests."""

    def __init__(self, ctx: Context, pool_bytes=0, lanes=0, max_request_instr=0, max_batch_kernels=0,
                 long_instr=0, flags=0):
        o = ServerOpts(pool_bytes, lanes, max_request_instr, max_batch_kernels, long_instr, flags)
        h = VP()
        check("dc_server_create", lib().dc_server_create(ctx.h, ctypes.byref(o), ctypes.byref(h)))
        self.h = h
        self._ticket = U64()
        self._buf = np.zeros(0, SERVER_RESULT_DTYPE)

    def submit_raw(self, req_addr: int) -> int:
        """Submit the dc_request_t at host address req_addr; returns its ticket."""
        check("dc_server_submit", lib().dc_server_submit(self.h, req_addr, ctypes.byref(self._ticket)))
        return self._ticket.value

    def submit(self, reqs: np.ndarray, i: int) -> int:
        return self.submit_raw(reqs.ctypes.data + i * REQUEST_DTYPE.itemsize)

    def poll(self, max_results: int = 4096, records: bool = True):
        """Completed results as a SERVER_RESULT_DTYPE array and, with
        records=True, a list of (accesses, sysvals) copies per result."""
        if len(self._buf) < max_results:
            self._buf = np.zeros(max_results, SERVER_RESULT_DTYPE)
        n = U32()
        check("dc_server_poll", lib().dc_server_poll(self.h, self._buf.ctypes.data, max_results, ctypes.byref(n)))
        res = self._buf[:n.value].copy()
        if not records:
            return res, None
        recs = []
        for r in res:
            na, ns = int(r["summary"]["n_access"]), int(r["summary"]["n_sysval"])
            acc = np.zeros(na, ACCESS_DTYPE)
            sysv = np.zeros(ns, SYSVAL_DTYPE)
            if na:
                ctypes.memmove(acc.ctypes.data, int(r["accesses"]), na * ACCESS_DTYPE.itemsize)
            if ns:
                ctypes.memmove(sysv.ctypes.data, int(r["sysvals"]), ns * SYSVAL_DTYPE.itemsize)
            recs.append((acc, sysv))
        return res, recs

    def stats(self) -> dict:
        st = ServerStats()
        check("dc_server_get_stats", lib().dc_server_get_stats(self.h, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in st._fields_ if k != "pad"}

    def close(self):
        if self.h:
            lib().dc_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Ssa:
    """Register versions of a batch (dc_build_ssa): merges, their arguments,
    the version of every use and definition."""

    def __init__(self, h, kernels, instrs_dev):
        self.h = h
        self.kernels = kernels
        self.n_kernels = len(kernels)
        self._keep = instrs_dev

    def run(self, instrs_dev=None):
        if instrs_dev is not None:
            self._keep = instrs_dev
        check("dc_ssa_run", lib().dc_ssa_run(self.h, _dev_ptr(self._keep)))

    def wait(self):
        check("dc_ssa_wait", lib().dc_ssa_wait(self.h))

    def results(self) -> np.ndarray:
        out = np.zeros(self.n_kernels, SSA_RESULT_DTYPE)
        check("dc_ssa_get_results", lib().dc_ssa_get_results(self.h, _np_ptr(out), self.n_kernels))
        return out

    def _get(self, name, k, dtype):
        n = U32()
        f = getattr(lib(), name)
        check(name, f(self.h, k, None, 0, ctypes.byref(n)))
        out = np.zeros(n.value, dtype)
        if n.value:
            check(name, f(self.h, k, _np_ptr(out), n.value, ctypes.byref(n)))
        return out

    def idom(self, k: int) -> np.ndarray:
        return self._get("dc_ssa_get_idom", k, np.uint32)

    def phis(self, k: int) -> np.ndarray:
        return self._get("dc_ssa_get_phis", k, PHI_DTYPE)

    def phi_args(self, k: int) -> np.ndarray:
        return self._get("dc_ssa_get_phi_args", k, np.uint32)

    def versions(self, k: int):
        n = int(self.kernels[k]["n_instr"])
        use = np.zeros((n, SSA_NU), np.uint32)
        dfn = np.zeros((n, SSA_ND), np.uint32)
        m = U32()
        check("dc_ssa_get_versions", lib().dc_ssa_get_versions(self.h, k, _np_ptr(use), _np_ptr(dfn), n,
                                                               ctypes.byref(m)))
        return use, dfn

    def types(self) -> np.ndarray:
        out = np.zeros(self.n_kernels, TYPES_RESULT_DTYPE)
        check("dc_types_get_results", lib().dc_types_get_results(self.h, _np_ptr(out), self.n_kernels))
        return out

    def vars(self, k: int) -> np.ndarray:
        return self._get("dc_types_get_vars", k, VAR_DTYPE)

    def timing(self) -> dict:
        """Stage times; ms_compact is the variable and type stage."""
        t = Timing()
        check("dc_ssa_get_timing", lib().dc_ssa_get_timing(self.h, ctypes.byref(t)))
        return {k: getattr(t, k) for k, _ in t._fields_ if k not in ("pad", "ms_pad")}

    def timing_reset(self):
        check("dc_ssa_timing_reset", lib().dc_ssa_timing_reset(self.h))

    def free(self):
        if self.h:
            lib().dc_ssa_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Text:
    """A text front end run (dc_parse_text): descriptors, records, argument
    tables and kernel names of a listing."""

    def __init__(self, h, text_dev, n_bytes):
        self.h = h
        self._keep = text_dev
        self.n_bytes = n_bytes

    def run(self, text_dev=None, n_bytes=None):
        if text_dev is not None:
            self._keep = text_dev
            self.n_bytes = n_bytes
        check("dc_text_run", lib().dc_text_run(self.h, _dev_ptr(self._keep), self.n_bytes))

    def wait(self):
        check("dc_text_wait", lib().dc_text_wait(self.h))

    def counts(self) -> dict:
        c = TextCounts()
        check("dc_text_get_counts", lib().dc_text_get_counts(self.h, ctypes.byref(c)))
        return {k: getattr(c, k) for k, _ in c._fields_}

    def device_arrays(self):
        """(descriptors, records, arguments) as DevicePtr to the object's
        device arrays (valid until free)."""
        k, i, a = VP(), VP(), VP()
        check("dc_text_device_arrays", lib().dc_text_device_arrays(self.h, ctypes.byref(k), ctypes.byref(i),
                                                                   ctypes.byref(a)))
        return DevicePtr(k.value or 0, self), DevicePtr(i.value or 0, self), DevicePtr(a.value or 0, self)

    def kernels(self) -> np.ndarray:
        n = U32()
        check("dc_text_get_kernels", lib().dc_text_get_kernels(self.h, None, 0, ctypes.byref(n)))
        out = np.zeros(n.value, KERNEL_DTYPE)
        check("dc_text_get_kernels", lib().dc_text_get_kernels(self.h, _np_ptr(out), n.value, ctypes.byref(n)))
        return out

    def records(self) -> np.ndarray:
        n = U64()
        check("dc_text_get_records", lib().dc_text_get_records(self.h, None, 0, ctypes.byref(n)))
        out = np.zeros(n.value, INSTR_DTYPE)
        check("dc_text_get_records", lib().dc_text_get_records(self.h, _np_ptr(out), n.value, ctypes.byref(n)))
        return out

    def args(self) -> np.ndarray:
        n = U64()
        check("dc_text_get_args", lib().dc_text_get_args(self.h, None, 0, ctypes.byref(n)))
        out = np.zeros(n.value, ARG_DTYPE)
        check("dc_text_get_args", lib().dc_text_get_args(self.h, _np_ptr(out), n.value, ctypes.byref(n)))
        return out

    def names(self):
        """(byte offsets, lengths) of the kernels' names in the text."""
        n = U32()
        check("dc_text_get_names", lib().dc_text_get_names(self.h, None, None, 0, ctypes.byref(n)))
        off = np.zeros(n.value, np.uint64)
        ln = np.zeros(n.value, np.uint32)
        check("dc_text_get_names", lib().dc_text_get_names(self.h, _np_ptr(off), _np_ptr(ln), n.value,
                                                           ctypes.byref(n)))
        return off, ln

    def timing(self) -> dict:
        t = Timing()
        check("dc_text_get_timing", lib().dc_text_get_timing(self.h, ctypes.byref(t)))
        return {k: getattr(t, k) for k, _ in t._fields_ if k not in ("pad", "ms_pad", "ms_compact")}

    def timing_reset(self):
        check("dc_text_timing_reset", lib().dc_text_timing_reset(self.h))

    def free(self):
        if self.h:
            lib().dc_text_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Struct:
    """Region-graph structuring of a batch (dc_structure): per kernel the
    merges in the order made, the regions left and the root."""

    def __init__(self, h, kernels, instrs_dev):
        self.h = h
        self.kernels = kernels
        self.n_kernels = len(kernels)
        self._keep = instrs_dev

    def run(self, instrs_dev=None):
        if instrs_dev is not None:
            self._keep = instrs_dev
        check("dc_struct_run", lib().dc_struct_run(self.h, _dev_ptr(self._keep)))

    def wait(self):
        check("dc_struct_wait", lib().dc_struct_wait(self.h))

    def results(self) -> np.ndarray:
        out = np.zeros(self.n_kernels, STRUCT_RESULT_DTYPE)
        check("dc_struct_get_results", lib().dc_struct_get_results(self.h, _np_ptr(out), self.n_kernels))
        return out

    def merges(self, k: int) -> np.ndarray:
        n = U32()
        check("dc_struct_get_merges", lib().dc_struct_get_merges(self.h, k, None, 0, ctypes.byref(n)))
        out = np.zeros(n.value, MERGE_DTYPE)
        if n.value:
            check("dc_struct_get_merges", lib().dc_struct_get_merges(self.h, k, _np_ptr(out), n.value,
                                                                     ctypes.byref(n)))
        return out

    def timing(self) -> dict:
        t = Timing()
        check("dc_struct_get_timing", lib().dc_struct_get_timing(self.h, ctypes.byref(t)))
        return {k: getattr(t, k) for k, _ in t._fields_ if k not in ("pad", "ms_pad", "ms_compact")}

    def timing_reset(self):
        check("dc_struct_timing_reset", lib().dc_struct_timing_reset(self.h))

    def free(self):
        if self.h:
            lib().dc_struct_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass
