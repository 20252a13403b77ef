"""GPU parity of the text front end (Section "The body extraction"): the HIP
parser through the C ABI (dc_parse_text) against the oracle's parser,
bit-exact on descriptors, records, argument tables and kernel names; then the
parsed records, straight from the parser's device arrays, through the
analysis, against the oracle's analysis of the oracle's parse."""
import sys

import numpy as np
import pytest

import dcgen
import hand_kernels as hk
import oracle
from gpu_common import compare_summaries, fuzz_listing

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2107_07809_amd import dc  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = dc.Context(0)
    yield c
    c.close()


def compare(ctx, text: bytes, label: str):
    say(f"text {label}: {len(text)} bytes")
    o = oracle.parse_text(text)
    dev = dc.text_to_device(text)
    t = ctx.parse_text(dev, len(text))
    k = t.kernels()
    assert k.tobytes() == o["kernels"].tobytes(), label
    r = t.records()
    if r.tobytes() != o["instrs"].tobytes():
        i = int(np.nonzero(r != o["instrs"])[0][0])
        raise AssertionError(f"{label}: record {i}: gpu {r[i]} oracle {o['instrs'][i]}")
    assert t.args().tobytes() == o["args"].tobytes(), label
    off, ln = t.names()
    assert off.tobytes() == o["name_off"].tobytes() and ln.tobytes() == o["name_len"].tobytes(), label
    c = t.counts()
    assert (c["n_kernels"], c["n_instr"], c["n_args"], c["fail"]) == (len(k), len(r), len(o["args"]), 0)
    return t, dev, o


def test_paper_listings_and_syntax_cases(ctx):
    """Listing 3 with the paper's printed instructions, and every syntax case
    of the oracle's pins (states, operands, malformed lines, alignment)."""
    from test_oracle_text import ALL_TEXTS
    for i, text in enumerate(ALL_TEXTS):
        t, _, _ = compare(ctx, text, f"case {i}")
        t.free()


def test_edge_texts(ctx):
    """Empty text, text without kernels, no trailing newline, a kernel with no
    body, CRLF endings, a very long line, labels defined twice, numeric
    branch targets."""
    long_line = b"  v_add_u32 v1, v2, v3" + b" " * 5000 + b"// tail\n"
    texts = [b"", b"\n\n", b"just text\n", b".kernel a\n.config\n.dims x\n.text\ns_endpgm",
             b".kernel a\r\n.config\r\n.cws 8\r\n.text\r\nL:\r\ns_branch L\r\n",
             b".kernel a\n.text\n" + long_line + b"s_endpgm\n",
             b".kernel a\n.text\nX:\ns_nop 0\nX:\ns_branch X\ns_branch 1\ns_branch -1\ns_endpgm\n",
             b".kernel\n.text\ns_endpgm\n.kernel b c\n.config\n.text\n"]
    for i, text in enumerate(texts):
        t, _, _ = compare(ctx, text, f"edge {i}")
        t.free()


def test_operand_word_edge_cases(ctx):
    """The operand text split into words and fields: empty fields, trailing
    and doubled commas, tabs, extra words inside a field, modifiers alone or
    between operands, offsets in hex, negative or malformed, comments after
    operands, blank-separated operands with a modifier."""
    body = [
        "v_add_u32 v1, , v3",
        "v_add_u32 v1,v2,v3,",
        "v_add_u32 v1,, v2, v3",
        "v_add_u32\tv1,\tv2 ,\t v3",
        "v_add_u32 v1 extra, v2 more words, v3",
        "global_load_dword v1, v[2:3], off offset:0x10",
        "global_load_dword v1, v[2:3], off offset:-4",
        "global_load_dword v1, v[2:3], off offset:abc",
        "global_load_dword v1, v[2:3], off offset:",
        "global_load_dword v1, v[2:3], off glc offset:8 slc",
        "global_store_dword v[2:3], v1, off offset:4 // comment, with a comma",
        "s_load_dwordx2 s[2:3] s[4:5] 0x0",
        "s_load_dwordx2 s[2:3] s[4:5] 0x8 ; trailing",
        "ds_read_b32 v1, v2 offset:16",
        "ds_write_b32 v2, v1 offset:65536",
        "v_mov_b32 v1 , v0",
        "v_mov_b32 , v0",
        "v_mov_b32",
        "s_mov_b32 s0, 0x7fffffff",
        "s_mov_b32 s0, -17",
        "s_mov_b32 s0, 64",
        "s_mov_b32 s0, 65",
        "v_mad_u32_u24 v1, v2, v3, v4",
        "v_add_co_u32 v1, vcc, v2, v3",
        "s_endpgm",
    ]
    text = (".kernel k\n.config\n.dims x\n.cws 64, 1, 1\n.arg _.global_offset_0, \"size_t\", long\n"
            ".arg a, \"int*\", int*\n.text\n" + "\n".join("  " + x for x in body) + "\n").encode()
    t, _, _ = compare(ctx, text, "operand words")
    t.free()


def test_rendered_workloads(ctx):
    """The small workload, a log-uniform sample, Zipf kernels with long ones,
    the dense control-flow shape (thousands of labels per kernel) and the
    hand-written kernels, rendered to listings."""
    for label, b in (("c1", dcgen.generate(1, 32)), ("c2", dcgen.generate(2, 2000, i0=7)),
                     ("c3", dcgen.generate(3, 3000, i0=99)), ("c6", dcgen.generate(6, 4)),
                     ("hand", dcgen.concat([k for _, k in hk.all_kernels()]))):
        t, _, _ = compare(ctx, dcgen.render(b), label)
        t.free()


def test_text_to_analysis(ctx):
    """Parse on the GPU and analyse the parsed records where they lie (the
    parser's device arrays): every summary and record against the oracle's
    analysis of the oracle's parse of the same text."""
    b = dcgen.generate(2, 400, i0=123)
    text = dcgen.render(b)
    t, dev, o = compare(ctx, text, "to analysis")
    _, rec_dev, _ = t.device_arrays()
    batch = ctx.analyze(t.kernels(), rec_dev, len(o["instrs"]), t.args(), flags=dc.OPT_DIGEST)
    ob = dcgen.Batch(o["instrs"], o["kernels"], o["args"])
    s, oacc, osys = oracle.analyze_batch(ob)
    compare_summaries(batch.results(), s)
    assert batch.all_accesses()[0].tobytes() == oacc.tobytes()
    assert batch.all_sysvals()[0].tobytes() == osys.tobytes()
    batch.free()
    t.free()


def test_rerun_and_other_text(ctx):
    """dc_text_run on the same text gives the same bytes without planning
    again; on another text it plans again."""
    b1 = dcgen.generate(1, 32)
    b2 = dcgen.generate(3, 500, i0=3)
    t1, d1 = dcgen.render(b1), dcgen.render(b2)
    t, dev1, o1 = compare(ctx, t1, "first")
    r1 = t.records()
    t.run()
    assert t.records().tobytes() == r1.tobytes()
    dev2 = dc.text_to_device(d1)
    t.run(dev2, len(d1))
    o2 = oracle.parse_text(d1)
    assert t.records().tobytes() == o2["instrs"].tobytes()
    assert t.kernels().tobytes() == o2["kernels"].tobytes()
    t.run(dev1, len(t1))
    assert t.records().tobytes() == r1.tobytes()
    t.free()


def test_c2_full_text(ctx):
    """All 65,536 kernels of the log-uniform workload as one listing (~1.5 GB
    of text): every descriptor, record and argument against the batch the
    text was rendered from (the round trip the oracle is pinned to), and every
    64th kernel's listing against the oracle's parse of it alone."""
    from test_oracle_text import canonical
    b = dcgen.generate(2, 65536)
    text = dcgen.render(b)
    say(f"text c2 full: {len(text)} bytes")
    dev = dc.text_to_device(text)
    t = ctx.parse_text(dev, len(text))
    k = t.kernels()
    assert k.tobytes() == b.kernels.tobytes()
    assert t.args().tobytes() == b.args.tobytes()
    r = t.records()
    assert r.tobytes() == canonical(b).tobytes()
    off, ln = t.names()
    starts = [text.rfind(b".kernel", 0, int(o)) for o in off]
    for i in range(0, 65536, 64):
        end = starts[i + 1] if i + 1 < len(starts) else len(text)
        o = oracle.parse_text(text[starts[i]:end])
        ki = k[i]
        mine = r[int(ki["instr_begin"]):int(ki["instr_begin"]) + int(ki["n_instr"])]
        assert mine.tobytes() == o["instrs"].tobytes(), i
        assert o["kernels"][0]["n_args"] == ki["n_args"] and o["kernels"][0]["dims"] == ki["dims"], i
    t.free()


def test_fuzzed_listings(ctx):
    """Rendered listings with seeded random edits on 15% of their lines
    (malformed mnemonics, operands, labels, configuration lines, cut and
    joined lines): the parser and the oracle's agree on every byte."""
    base = dcgen.render(dcgen.concat([dcgen.generate(2, 40, i0=900).kernel(k) for k in range(40)] +
                                     [k for _, k in hk.all_kernels(n_random=2)]))
    for seed in range(12):
        compare(ctx, fuzz_listing(base, seed), f"fuzz {seed}")
