"""The plain C parts -- the oracle and the input generator -- built with
AddressSanitizer and UndefinedBehaviorSanitizer and run on every entry point
the tests use: generated kernels of every shape (analysis, versions,
variables and types, structuring, the rendered listing through the text
front end), the hand-written rule kernels, and malformed listings.  Any
out-of-bounds access, use after free or undefined operation stops the run.
CPU only (gcc); the GPU library's device code is not involved."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import sys
ROOT, GEN = sys.argv[1], sys.argv[2]
sys.path.insert(0, ROOT)
sys.path.insert(0, ROOT + "/tests")
import dcgen
dcgen.LIB_PATH = GEN
import oracle
import hand_kernels as hk
for cfg, n in ((1, 32), (2, 24), (3, 48), (5, 12), (6, 1)):
    b = dcgen.generate(cfg, n, threads=2)
    oracle.analyze_batch(b)
    oracle.ssa_batch(b)
    oracle.types_batch(b)
    oracle.structure_batch(b)
    oracle.parse_text(dcgen.render(b))
for name, (recs, d, args) in hk.all_kernels(n_random=2):
    oracle.analyze(recs, d, args)
    oracle.types(recs, d, args)
    oracle.structure(recs, d)
for text in (b".kernel a\n .text\n s_add_u32 s0,\n v_mov_b32 v1 v0 v2 v3 v4\n L:\n s_branch NOWHERE\n",
             b".kernel\n.config\n .arg x, \"int\"\n .cws 1,2,3,4\n.text\n\n", b"", b"\n\n\r\n", b".text\n s_endpgm",
             b".kernel k\n .config\n .dims xyzw\n .arg p, \"float*\", float*, global\n .text\n global_load_dword v1, v[2:3], off offset:0x\n"):
    oracle.parse_text(text)
from gpu_common import fuzz_listing
base = dcgen.render(dcgen.concat([dcgen.generate(2, 12, i0=900, threads=2).kernel(k) for k in range(12)]))
for seed in range(12):
    oracle.parse_text(fuzz_listing(base, seed))
print("SANITIZED RUN OK")
"""


def _lib(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def test_oracle_and_generator_under_asan_and_ubsan(tmp_path):
    asan = _lib("libasan.so")
    if asan is None or _lib("libubsan.so") is None:
        pytest.skip("gcc's sanitizer runtimes are not installed")
    flags = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
             "-fPIC", "-shared"]
    orc = str(tmp_path / "liboracle_san.so")
    gen = str(tmp_path / "libdcgen_san.so")
    subprocess.check_call(["gcc", *flags, "-o", orc, os.path.join(ROOT, "oracle", "dc_oracle.c")])
    subprocess.check_call(["gcc", *flags, "-o", gen, os.path.join(ROOT, "dcgen", "dcgen.c"), "-lm", "-lpthread"])
    env = dict(os.environ, LD_PRELOAD=asan, DC_ORACLE_LIB=orc,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:exitcode=23",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=24")
    r = subprocess.run([sys.executable, "-c", SCRIPT, ROOT, gen], env=env, capture_output=True, text=True,
                       timeout=900)
    assert r.returncode == 0 and "SANITIZED RUN OK" in r.stdout, (r.returncode, r.stderr[-3000:])
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-3000:]
