"""Build of libdc.so (hipcc, gfx950)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libdc.so")
SOURCES = [os.path.join(CSRC, "dc_kernels.hip"), os.path.join(CSRC, "dc_fixpoint.hip"),
           os.path.join(CSRC, "dc_noalloc.hip"), os.path.join(CSRC, "dc_plain.hip"),
           os.path.join(CSRC, "dc_ssa.hip"), os.path.join(CSRC, "dc_types.hip"),
           os.path.join(CSRC, "dc_text.hip"),
           os.path.join(CSRC, "dc_struct.hip"), os.path.join(CSRC, "dc_api.cpp"), os.path.join(CSRC, "dc_text_api.cpp"), os.path.join(CSRC, "dc_server.cpp")]
HEADERS = [os.path.join(CSRC, "dc_internal.h"), os.path.join(CSRC, "dc_fixpoint_core.h"), os.path.join(CSRC, "dc_records.h"), os.path.join(CSRC, "dc_opnames.h"), os.path.join(CSRC, "dc_ssa_ops.h"), os.path.join(CSRC, "dc_host.h"), os.path.join(CSRC, "dc_isa.h"),
           os.path.join(CSRC, "dc_device.h"), os.path.join(ROOT, "include", "dc.h")]

FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         # no packed fp32 instructions anywhere in the library
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument"]


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp"
    cmd = [hipcc, *FLAGS, "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-o", tmp, *SOURCES, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + r.stderr[-4000:])
    if verbose:
        print(r.stderr)
    os.replace(tmp, LIB)
    return LIB


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(f) > t for f in SOURCES + HEADERS)
