"""Host-side checks of the C ABI that need no GPU: the library loads, it
exports every function include/dc.h declares, the binding covers them, and
calls that cannot reach a device fail with a status instead of crashing."""
import ctypes
import os
import re

import pytest

import dcgen
import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def dc():
    from paper_2107_07809_amd import _build, dc as mod
    if not os.path.exists(_build.LIB):
        _build.build()
    return mod


def declared_functions():
    text = open(os.path.join(ROOT, "include", "dc.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dc_[a-z0-9_]+)\s*\(", text)))


def test_exports_every_declared_symbol(dc):
    names = declared_functions()
    assert len(names) >= 20
    L = ctypes.CDLL(dc.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n
    bound = {s[0] for s in dc.SIGNATURES}
    assert set(names) == bound


def test_opcode_numbering_agrees(dc):
    """The record encoding: the library, the generator and the oracle name
    every opcode id the same way."""
    assert dc.opcode_names() == dcgen.op_names() == oracle.op_names()


def test_status_strings(dc):
    for code in (0, -1, -2, -3, -4, -10, -11, -12, -13, -14, -15, -16):
        assert dc.status_str(code) != "unknown status"
    assert dc.status_str(-99) == "unknown status"


def test_no_device_is_an_error_not_a_crash(dc):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(dc.DCError) as e:
        dc.Context(0)
    assert e.value.code == -2


def test_null_arguments(dc):
    L = dc.lib()
    assert L.dc_ctx_create(0, None) == -1
    assert L.dc_analyze_batch(None, None, 0, None, 0, None, 0, None, None, None) == -1
    h = ctypes.c_void_p()
    assert L.dc_analyze_batch(None, None, 0, None, 0, None, 0, None, None, ctypes.byref(h)) == -1
    assert L.dc_build_cfg(None, None, 0, None, 0, None, ctypes.byref(h)) == -1
    assert L.dc_batch_wait(None) == -1
    assert L.dc_get_stats(None, None) == -1
    L.dc_batch_free(None)
    L.dc_cfg_free(None)
    L.dc_ctx_destroy(None)
    assert L.dc_server_create(None, None, ctypes.byref(h)) == -1
    t = ctypes.c_uint64()
    n = ctypes.c_uint32()
    assert L.dc_server_submit(None, None, ctypes.byref(t)) == -1
    assert L.dc_server_poll(None, None, 0, ctypes.byref(n)) == -1
    assert L.dc_server_get_stats(None, None) == -1
    L.dc_server_destroy(None)
    best = dc.Options()
    ms = ctypes.c_float()
    assert L.dc_autotune(None, None, 0, None, 0, None, 0, None, 0, None, ctypes.byref(best), ctypes.byref(ms)) == -1
    assert L.dc_autotune(None, None, 0, None, 0, None, 0, None, 0, None, None, None) == -1


def test_struct_sizes(dc):
    assert dc.INSTR_DTYPE.itemsize == 16 and dc.KERNEL_DTYPE.itemsize == 32 and dc.ARG_DTYPE.itemsize == 8
    assert dc.REG_DTYPE.itemsize == 16 and dc.ACCESS_DTYPE.itemsize == 16 and dc.SYSVAL_DTYPE.itemsize == 8
    assert dc.RESULT_DTYPE.itemsize == 32 and ctypes.sizeof(dc.Options) == 32
    assert dc.INSTR_DTYPE == dcgen.INSTR_DTYPE and dc.KERNEL_DTYPE == dcgen.KERNEL_DTYPE
    assert dc.REQUEST_DTYPE.itemsize == 56 and dc.SERVER_RESULT_DTYPE.itemsize == 120
    assert ctypes.sizeof(dc.ServerOpts) == 40 and ctypes.sizeof(dc.ServerStats) == 64


def test_request_pointers(dc):
    """dc_request_t entries point at each kernel's own records and arguments."""
    import numpy as np
    b = dcgen.generate(1, 5)
    reqs = dc.requests(b.kernels, b.instrs, b.args)
    for k in range(5):
        d = b.kernels[k]
        assert reqs["instrs"][k] == b.instrs.ctypes.data + 16 * int(d["instr_begin"])
        assert reqs["args"][k] == b.args.ctypes.data + 8 * int(d["arg_begin"])
        assert reqs["kernel"][k]["instr_begin"] == 0 and reqs["kernel"][k]["n_instr"] == d["n_instr"]
    assert (reqs["tag"] == np.arange(5)).all()


def test_bench_refuses_several_gpus():
    """The bench measures one GPU; asking for more prints why and exits 2."""
    import json
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]
