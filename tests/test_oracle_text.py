"""Pins of the oracle's text front end (Section "The body extraction",
Listings 1-3): the listing format to kernel descriptors, records and argument
tables.  Expected values are written out by hand from the paper's listings
and from the record layout; the round trip runs the generator's own renderer
(input synthesis, independent of the oracle) over seeded batches."""
import numpy as np

import dcgen
import hand_kernels as hk
import oracle

OP = dcgen.opcode
NONE, LIT, BAD = 0xFFFF, 0xFFFE, 0xFFFD


def rec(name, r0=NONE, r1=NONE, r2=NONE, imm=0, target=-1):
    return (OP(name), r0, r1, r2, imm, target)


# Section "Data type recovery", Listing 3 (the configuration of
# void copy(__global int *data, int x)), with a body made of the paper's
# printed instructions: the get_global_offset(0) load of Section "Search for
# memory accesses" (first step, printed without commas) and the s_add_u32 of
# Section "Data type recovery".
LISTING3 = b""".kernel copy
 .config
  .dims x
  .cws 64, 1, 1
  .sgprsnum 13
  .vgprsnum 3
  .floatmode 0xc0
  .pgmrsrc1 0x00ac0040
  .pgmrsrc2 0x0000008c
  .dx10clamp
  .ieeemode
  .useargs
  .priority 0
  .arg _.global_offset_0, "size_t", long
  .arg _.global_offset_1, "size_t", long
  .arg _.global_offset_2, "size_t", long
  .arg _.printf_buffer, "size_t", void*, global, , rdonly
  .arg _.vqueue_pointer,"size_t", long
  .arg _.aqlwrap_pointer,"size_t", long
  .arg data, "int*", int*, global,
  .arg x, "int", int
 .text
  s_load_dwordx2 s[2:3] s[4:5] 0x0
  s_add_u32 s0, s4, s0
  s_endpgm
"""


ALIGN_TEXT = b""".kernel a
 .config
  .dims x
  .cws 64, 1, 1
  .useargs
  .arg _.global_offset_0, "size_t", long
  .arg n, "int", int
  .arg p, "float*", float*, global,
  .arg q, "uint", uint
  .arg c, "char", char
  .arg h, "ushort", ushort
  .arg d, "double", double
  .arg v, "void*", void*, global, , rdonly
 .text
  s_endpgm
"""

LISTING1_TEXT = b""".kernel k1
    .config
        dims xyz
        .cws 8, 8, 2
            .sgprsnum 16
    .text
        v_mov_b32 v3, v0
        s_endpgm <- end of program
"""

STATES_TEXT = b"""garbage before
s_nop 0
.kernel a
  s_nop 0
  .config
    .dims xy
    .cws 16, 4
  .text
    s_nop 0
  .config
    .useargs
  .text
  s_endpgm
.kernel b
  .config
    .dims x
.kernel c extra words
  .text
L:
    s_branch L
"""

SYNTAX_TEXT = b""".kernel t
.config
  .dims x
  .cws 64, 1, 1
  .useargs
.text
TOP:
  s_mov_b32 s7, -16            // inline -16
  s_mov_b32 s7, 64 ; inline 64
  s_mov_b32 s7, 65
  s_mov_b32 s7, -17
  s_mov_b32 s7, 0xffffffff\r
  v_mul_f32 v1, -4.0, v2
  v_mul_f32 v1, 0.5, v255
  s_and_saveexec_b64 s[20:21], vcc
  s_mov_b64 exec, s[20:21]
  v_mov_b32 v1, vcc_hi
  v_mov_b32 v1, exec_lo
  v_mov_b32 v1, m0
  v_add_co_u32 v4, vcc, s12, v2
  v_addc_co_u32 v5, vcc, v5, v3, vcc
  v_cndmask_b32 v6, v1, v2, vcc
  v_mad_u32_u24 v7, v1, v2, v3
  v_cmp_gt_u32 vcc, v0, 3
  s_cmp_lt_u32 s20, 10
  global_load_dword v30, v[4:5], off offset:16
  global_store_dword v[4:5], v30, s[8:9]
  flat_load_dword v1, v[2:3] offset:-8
  ds_write_b32 v6, v7 offset:4
  ds_read_b32 v8, v6
  s_load_dword s16, s[4:5], 0x40
  s_cbranch_scc1 TOP
  s_branch END
END:
; a whole-line comment
  // another
  s_endpgm
"""

MALFORMED_TEXT = b""".kernel e
.config
  .dims x
.text
  s_frobnicate s0, s1
  s_mov_b32 s104, s1
  v_mov_b32 v256, v1
  v_mov_b32 v1, v[4:3]
  s_add_u32 s0, s1
  ds_read_b32 v1, v2 offset:zz
  s_branch NOWHERE
  v_mul_f32 v1, 3.0, v2
  s_endpgm
"""


def test_listing3_configuration_and_arguments():
    r = oracle.parse_text(LISTING3)
    assert r["names"] == [b"copy"]
    k = r["kernels"][0]
    assert (k["dims"], list(k["cws"]), k["useargs"], k["n_args"], k["n_instr"]) == (1, [64, 1, 1], 1, 2, 3)
    # the six hidden slots take 0x00-0x2f; data is a pointer to int at 0x30,
    # x an int at 0x38
    assert r["args"].tolist() == [(0x30, 8, dcgen.T_PTR, dcgen.T_INT), (0x38, 4, dcgen.T_INT, 0)]
    assert r["instrs"].tolist() == [rec("s_load_dwordx2", 2, 4, NONE, 0), rec("s_add_u32", 0, 4, 0),
                                    rec("s_endpgm")]


def test_argument_layout_alignment():
    """User arguments follow the six hidden 8-byte slots from 0x30, each at
    the next multiple of its size: an int at 0x30 puts the next pointer at
    0x38; a char then a short then a double go to 0x3c, 0x3e, 0x40; unsigned
    and float types give their bits; void* points to nothing."""
    text = ALIGN_TEXT
    r = oracle.parse_text(text)
    T = dcgen
    assert r["args"].tolist() == [(0x30, 4, T.T_INT, 0), (0x38, 8, T.T_PTR, T.T_FLOAT), (0x40, 4, T.T_UINT, 0),
                                  (0x44, 1, T.T_INT, 0), (0x46, 2, T.T_UINT, 0), (0x48, 8, T.T_DOUBLE, 0),
                                  (0x50, 8, T.T_PTR, 0)]


def test_listing1_structure():
    """Listing 1: dims xyz (printed without the dot) and .cws 8, 8, 2 mean a
    3-D range of 8x8x2 work-groups; other configuration lines are skipped;
    the body ends at s_endpgm (whose trailing words are not operands)."""
    text = LISTING1_TEXT
    r = oracle.parse_text(text)
    k = r["kernels"][0]
    assert (k["dims"], list(k["cws"]), k["useargs"], k["n_args"], k["n_instr"]) == (3, [8, 8, 2], 0, 0, 2)
    assert r["instrs"].tolist() == [rec("v_mov_b32", 112 + 3, 112 + 0), rec("s_endpgm")]


def test_extraction_states():
    """Listing 2's loop: lines before the first .kernel and between .kernel
    and .config are skipped; .config and .text switch the state (again and
    again); a kernel without .text has no body; kernels follow one another."""
    text = STATES_TEXT
    r = oracle.parse_text(text)
    assert r["names"] == [b"a", b"b", b"c"]
    ka, kb, kc = r["kernels"]
    assert (ka["dims"], list(ka["cws"]), ka["useargs"], ka["n_instr"]) == (2, [16, 4, 1], 1, 2)
    assert (kb["dims"], list(kb["cws"]), kb["n_instr"], kb["instr_begin"]) == (1, [0, 0, 0], 0, 2)
    assert (kc["dims"], kc["n_instr"], kc["instr_begin"]) == (0, 1, 2)
    assert r["instrs"].tolist() == [rec("s_nop"), rec("s_endpgm"), rec("s_branch", target=0)]


def test_operand_syntax():
    """Registers, specials, ranges, inline integers and floats, literals in
    decimal and hex, saddr off, offsets, labels, blank-separated operands,
    comments and carriage returns."""
    text = SYNTAX_TEXT
    r = oracle.parse_text(text)
    V = lambda n: 112 + n  # noqa: E731
    I = lambda v: 0x8000 + v + 16  # noqa: E731
    want = [rec("s_mov_b32", 7, I(-16)), rec("s_mov_b32", 7, I(64)), rec("s_mov_b32", 7, LIT, imm=65),
            rec("s_mov_b32", 7, LIT, imm=-17), rec("s_mov_b32", 7, LIT, imm=-1),
            rec("v_mul_f32", V(1), 0x8067, V(2)), rec("v_mul_f32", V(1), 0x8060, V(255)),
            rec("s_and_saveexec_b64", 20, 104), rec("s_mov_b64", 106, 20), rec("v_mov_b32", V(1), 105),
            rec("v_mov_b32", V(1), 106), rec("v_mov_b32", V(1), 109),
            rec("v_add_co_u32", V(4), 12, V(2)), rec("v_addc_co_u32", V(5), V(5), V(3)),
            rec("v_cndmask_b32", V(6), V(1), V(2)), rec("v_mad_u32_u24", V(7), V(1), V(2), imm=V(3)),
            rec("v_cmp_gt_u32", NONE, V(0), I(3)), rec("s_cmp_lt_u32", NONE, 20, I(10)),
            rec("global_load_dword", V(30), V(4), NONE, 16), rec("global_store_dword", V(30), V(4), 8),
            rec("flat_load_dword", V(1), V(2), NONE, -8), rec("ds_write_b32", V(7), V(6), NONE, 4),
            rec("ds_read_b32", V(8), V(6)), rec("s_load_dword", 16, 4, NONE, 0x40),
            rec("s_cbranch_scc1", target=0), rec("s_branch", target=26), rec("s_endpgm")]
    got = r["instrs"].tolist()
    assert len(got) == len(want)
    for i, (g, w) in enumerate(zip(got, want)):
        assert g == w, (i, g, w)


def test_malformed_lines_become_failing_records():
    """Each malformed line still yields one record, which the record checks
    of the analysis then reject: an unknown mnemonic (opcode 0xFFFF), a
    register out of range or a reversed range (operand 0xFFFD), a missing
    operand (0xFFFD), a malformed offset (opcode 0xFFFF), an unknown label
    (target 0x7FFFFFFF), a float other than the eight inline ones."""
    text = MALFORMED_TEXT
    r = oracle.parse_text(text)
    got = r["instrs"].tolist()
    assert got[0][0] == NONE
    assert got[1][:3] == (OP("s_mov_b32"), BAD, 1)
    assert got[2][:3] == (OP("v_mov_b32"), BAD, 113)
    assert got[3][:3] == (OP("v_mov_b32"), 113, BAD)
    assert got[4][:4] == (OP("s_add_u32"), 0, 1, BAD)
    assert got[5][0] == NONE
    assert got[6] == rec("s_branch", target=0x7FFFFFFF)
    assert got[7][:4] == (OP("v_mul_f32"), 113, BAD, 114)
    # the analysis reports them
    assert oracle.kernel_status(r["instrs"][:1], dcgen.descriptor(1)) == oracle.E_BADOP
    for i in (1, 2, 3, 4, 7):
        one = np.concatenate([r["instrs"][i:i + 1], r["instrs"][-1:]])
        assert oracle.kernel_status(one, dcgen.descriptor(2)) == oracle.E_BADREG, i
    one = np.concatenate([r["instrs"][6:7], r["instrs"][-1:]])
    assert oracle.kernel_status(one, dcgen.descriptor(2)) == oracle.E_BADTARGET


def canonical(b):
    """Records as text can carry them: a literal operand whose value is in the
    inline range [-16, 64] reads back as that inline constant (imm 0)."""
    r = b.instrs.copy()
    names = dcgen.op_names()
    noimm = np.array([n.startswith(("s_load", "global_", "flat_", "ds_"))
                      or n in ("v_mad_u32_u24", "v_mad_f32", "v_fma_f32", "v_fma_f64") for n in names] + [True] * 65536)
    imm = r["imm"].astype(np.int64)
    hit = ~noimm[r["op"]] & (imm >= -16) & (imm <= 64) & ((r["r1"] == LIT) | (r["r2"] == LIT))
    inline = (0x8000 + imm + 16).astype(np.uint16)
    for f in ("r1", "r2"):
        m = hit & (r[f] == LIT)
        r[f][m] = inline[m]
    r["imm"][hit] = 0
    return r


def test_round_trip_generated_batches():
    """parse(render(batch)) gives the batch back: descriptors, argument
    tables and (canonical) records, for the small, log-uniform, Zipf and
    dense-control-flow shapes and the hand-written kernels (whose argument
    tables are not all laid out naturally, which a listing cannot express:
    their offsets are not compared)."""
    parts = [k for _, k in hk.all_kernels()]
    for b, natural in ((dcgen.generate(1, 32), True), (dcgen.generate(2, 200, i0=11), True),
                       (dcgen.generate(3, 300, i0=5), True), (dcgen.generate(6, 2), True),
                       (dcgen.concat(parts), False)):
        r = oracle.parse_text(dcgen.render(b))
        assert r["kernels"].tobytes() == b.kernels.tobytes()
        if natural:
            assert r["args"].tobytes() == b.args.tobytes()
        else:
            for f in ("size", "type", "flags"):
                assert np.array_equal(r["args"][f], b.args[f]), f
        assert r["instrs"].tobytes() == canonical(b).tobytes()
        assert r["names"] == [f"k{k}".encode() for k in range(b.n_kernels)]


# every hand-written listing above, for the GPU parser's parity test
ALL_TEXTS = [LISTING3, ALIGN_TEXT, LISTING1_TEXT, STATES_TEXT, SYNTAX_TEXT, MALFORMED_TEXT]
