"""Hand-written rule kernels shared by the oracle's CPU pins and the GPU
parity test (test infrastructure).

Each entry is straight-line assembly (or a small loop) that exercises one
family of transfer rules: constant folding, inline float constants, the
argument-area table of scalar loads through s[4:5] (Listing 3's layout:
global offsets, hidden slots, user arguments, loads landing inside an
argument, a clobbered s4), index and pointer formation, 64-bit shifts,
uninitialised sources, and the second dimension's work-group size.  The CPU
tests check the oracle's results against closed forms; the GPU test runs the
same kernels through the C ABI and compares every state byte with the
oracle.  For the GPU a straight-line body is closed by a jump to a final
block, so the body's OUT state becomes that block's IN state (the states the
library exports are IN states).
"""
from __future__ import annotations

import numpy as np

import asmtext
import dcgen


def fold_scalar_src(x: int, y: int) -> str:
    return f"""
      s_mov_b32 s1, {x:#x}
      s_mov_b32 s2, {y:#x}
      s_add_u32 s3, s1, s2
      s_sub_u32 s10, s1, s2
      s_mul_i32 s11, s1, s2
      s_and_b32 s12, s1, s2
      s_or_b32 s13, s1, s2
      s_lshl_b32 s14, s1, s2
      s_lshr_b32 s15, s1, s2
      v_xor_b32 v3, s1, s2
      v_mul_u32_u24 v4, s1, s2
      v_lshlrev_b32 v5, s2, s1
      v_lshrrev_b32 v6, s2, s1
      v_ashrrev_i32 v7, s2, s1
      v_mad_u32_u24 v8, s1, s2, s1
      s_endpgm
    """


def fold_64_src(a: int, b: int, c: int, d: int, sh: int) -> str:
    return f"""
      s_mov_b32 s10, {a:#x}
      s_mov_b32 s11, {b:#x}
      s_mov_b32 s12, {c:#x}
      s_mov_b32 s13, {d:#x}
      s_and_b64 s[20:21], s[10:11], s[12:13]
      s_or_b64 s[22:23], s[10:11], s[12:13]
      s_xor_b64 s[24:25], s[10:11], s[12:13]
      s_andn2_b64 s[26:27], s[10:11], s[12:13]
      v_mov_b32 v10, s10
      v_mov_b32 v11, s11
      v_lshlrev_b64 v[20:21], {sh}, v[10:11]
      s_endpgm
    """


INLINE_CONSTANTS = """
      s_mov_b32 s1, 0.5
      s_mov_b32 s2, -4.0
      v_mov_b32 v1, 1.0
      s_mov_b64 s[10:11], 2.0
      s_mov_b64 s[12:13], -16
      s_mov_b64 s[14:15], 64
      s_mov_b64 s[16:17], -70000
      s_mov_b32 s18, 100000
      s_endpgm
"""

FLOAT_OPS = """
      v_mov_b32 v1, 1.0
      v_add_f32 v2, v1, v1
      v_mad_f32 v3, v1, v1, v1
      v_cvt_f32_u32 v4, v0
      v_cvt_u32_f32 v5, v1
      v_cvt_f64_f32 v[6:7], v1
      v_add_f64 v[8:9], v[6:7], v[6:7]
      v_mul_hi_u32 v10, v0, 7
      s_endpgm
"""

# exact (offset, width) entries, then per-dword resolution: global offsets as
# x2 and x4 loads, an x2 load straddling two arguments, a load inside an
# argument, a load past the last argument, a load not through s[4:5], and the
# high dword of a hidden pointer slot
SMEM_TABLE = """
      s_load_dwordx2 s[10:11], s[4:5], 0x8
      s_load_dwordx2 s[12:13], s[4:5], 0x10
      s_load_dwordx4 s[16:19], s[4:5], 0x0
      s_load_dword s20, s[4:5], 0x3c
      s_load_dword s21, s[4:5], 0x34
      s_load_dwordx2 s[22:23], s[4:5], 0x34
      s_load_dword s24, s[2:3], 0x30
      s_load_dword s25, s[4:5], 0x2c
      s_endpgm
"""


def smem_table_args():
    args = np.zeros(2, dcgen.ARG_DTYPE)
    args[0] = (0x30, 8, dcgen.T_PTR, dcgen.T_FLOAT)
    args[1] = (0x38, 4, dcgen.T_UINT, 0)
    return args


# every hidden slot dword (0x18..0x2c), an x4 load spanning the hidden area
# and the first argument, a dword in the middle of an 8-byte argument, and
# the work-dimension offset as printed
SMEM_HIDDEN = """
      s_load_dword s10, s[4:5], 0x18
      s_load_dword s11, s[4:5], 0x1c
      s_load_dword s12, s[4:5], 0x20
      s_load_dword s13, s[4:5], 0x24
      s_load_dword s14, s[4:5], 0x28
      s_load_dwordx2 s[16:17], s[4:5], 0x28
      s_load_dwordx4 s[20:23], s[4:5], 0x28
      s_load_dword s24, s[4:5], 0x42
      s_load_dword s25, s[4:5], 0x20010
      s_load_dword s26, s[4:5], 0x4
      s_endpgm
"""


def smem_hidden_args():
    args = np.zeros(2, dcgen.ARG_DTYPE)
    args[0] = (0x30, 8, dcgen.T_PTR, dcgen.T_INT)
    args[1] = (0x40, 8, dcgen.T_PTR, dcgen.T_DOUBLE)
    return args


# a clobbered s4 keeps the load's syntactic provenance and type, not its payload
SMEM_CLOBBERED = """
      s_mov_b32 s4, 0
      s_load_dword s10, s[4:5], 0xc
      s_endpgm
"""

INDEX_RULES = """
      s_lshl_b32 s0, s6, 6
      s_lshl_b32 s1, s6, 5
      s_mul_i32 s2, 64, s6
      v_add_co_u32 v1, vcc, s0, v0
      v_add_u32 v2, v1, 12
      v_mul_lo_u32 v3, v1, 8
      v_lshlrev_b32 v4, 0, v1
      v_lshlrev_b32 v5, 16, v1
      v_add_co_u32 v6, vcc, v3, 5
      v_ashrrev_i32 v7, 31, v1
      v_add_co_u32 v8, vcc, v1, v1
      v_mad_u32_u24 v9, v1, 4, 3
      v_mul_lo_u32 v10, v1, 12
      v_add_co_u32 v11, vcc, v3, v3
      v_add_co_u32 v12, vcc, v0, v7
      s_endpgm
"""

MAD_RULES = """
      v_mad_u32_u24 v9, v0, 4, 3
      v_mad_u32_u24 v10, s6, 64, v0
      s_endpgm
"""

POINTER_RULES = """
      s_load_dwordx2 s[8:9], s[4:5], 0x30
      s_add_u32 s10, s8, 16
      s_addc_u32 s11, s9, 0
      s_add_u32 s12, s10, 4
      v_mov_b32 v2, v0
      v_ashrrev_i32 v3, 31, v2
      v_lshlrev_b64 v[2:3], 3, v[2:3]
      v_add_co_u32 v4, vcc, s10, v2
      v_addc_co_u32 v5, vcc, s11, v3, vcc
      v_add_co_u32 v6, vcc, s12, v2
      s_addc_u32 s13, s9, 1
      s_addc_u32 s14, 3, 4
      global_load_dword v7, v[4:5], off offset:8
      ds_read_b32 v8, v2 offset:4
      s_endpgm
"""


def pointer_rules_args():
    args = np.zeros(1, dcgen.ARG_DTYPE)
    args[0] = (0x30, 8, dcgen.T_PTR, dcgen.T_INT)
    return args


UNINIT_TOP = """
      v_mov_b32 v3, v9
      v_add_u32 v4, v9, 1
      s_mov_b32 s30, exec_lo
      s_endpgm
"""

SECOND_DIM = """
      s_load_dword s10, s[4:5], 0x10
      s_lshr_b32 s11, s10, 2
      s_lshr_b32 s12, s10, 6
      s_mul_i32 s13, s7, 4
      s_mul_i32 s14, s7, 64
      v_add_co_u32 v3, vcc, s13, v1
      s_endpgm
"""

STRAIGHT_GLOBAL_ID = """
      s_load_dwordx2 s[2:3], s[4:5], 0x0
      s_mul_i32 s0, s6, 64
      v_add_co_u32 v1, vcc, s0, v0
      v_add_co_u32 v1, vcc, s2, v1
      v_mov_b32 v9, v1
      s_endpgm
"""

LOOPS = [
    # a loop around a diamond; values flow around the back edge
    """
      s_mov_b32 s20, 0
      v_mov_b32 v5, 0
    HEAD:
      v_cmp_gt_u32 vcc, v0, s20
      s_and_saveexec_b64 s[24:25], vcc
      s_cbranch_execz ELSE
      v_add_co_u32 v5, vcc, v5, v0
      v_mov_b32 v7, s6
      s_branch END
    ELSE:
      v_mov_b32 v6, v5
      s_load_dword s12, s[4:5], 0xc
    END:
      s_or_b64 exec, exec, s[24:25]
      v_mov_b32 v8, v6
      s_add_u32 s20, s20, 1
      s_cmp_lt_u32 s20, 16
      s_cbranch_scc1 HEAD
      global_store_dword v[2:3], v8, off
      s_endpgm
    """,
    # nested loops with a rotating chain of copies (bits need several trips)
    """
      s_mov_b32 s21, 0
    OUTER:
      s_mov_b32 s20, 0
    INNER:
      v_mov_b32 v9, v8
      v_mov_b32 v8, v7
      v_mov_b32 v7, v6
      v_mov_b32 v6, v0
      s_add_u32 s20, s20, 1
      s_cmp_lt_u32 s20, 4
      s_cbranch_scc1 INNER
      s_mov_b32 s13, s7
      s_add_u32 s21, s21, 1
      s_cmp_lt_u32 s21, 4
      s_cbranch_scc1 OUTER
      s_endpgm
    """,
]

# a back edge into block 0 and code after s_endpgm that nothing targets
ENTRY_AND_UNREACHABLE = """
    L0:
      s_add_u32 s20, s20, 1
      s_cmp_lt_u32 s20, 10
      s_cbranch_scc1 L0
      s_endpgm
      v_mov_b32 v3, 1
      s_endpgm
"""

NOARGS = np.zeros(0, dcgen.ARG_DTYPE)


def closed(src: str) -> str:
    """The body with its final s_endpgm replaced by a jump to a last block:
    the body's OUT state is then that block's IN state."""
    lines = [x for x in src.strip().splitlines() if x.strip()]
    assert lines[-1].strip() == "s_endpgm"
    return "\n".join(lines[:-1] + ["      s_branch ZZEND", "    ZZEND:", "      s_endpgm"])


def kernel(src: str, dims=1, cws=(64, 1, 1), args=NOARGS):
    recs = asmtext.assemble(src)
    return recs, dcgen.descriptor(len(recs), dims, cws, 1, len(args)), args


def all_kernels(seed: int = 20210716, n_random: int = 24):
    """(name, (records, descriptor, args)) of every hand-written kernel, the
    randomised folding kernels drawn from a fixed seed; straight-line bodies
    closed by a final block."""
    rng = np.random.default_rng(seed)
    out = []
    edge = [0, 1, 2, 31, 32, 63, 0x7FFFFFFF, 0x80000000, 0xFFFFFFFF, 0xFFFFFF, 0x1000000]
    pairs = [(x, y) for x in edge[:6] for y in edge[6:]] + \
        [tuple(int(v) for v in rng.integers(0, 2 ** 32, 2)) for _ in range(n_random)]
    for x, y in pairs:
        out.append((f"fold_scalar({x:#x},{y:#x})", kernel(closed(fold_scalar_src(x, y)))))
    for sh in list(range(0, 64, 7)) + [63]:
        a, b, c, d = (int(v) for v in rng.integers(0, 2 ** 32, 4))
        out.append((f"fold_64(sh={sh})", kernel(closed(fold_64_src(a, b, c, d, sh)))))
    straight = [
        ("inline_constants", INLINE_CONSTANTS, {}),
        ("float_ops", FLOAT_OPS, {}),
        ("smem_table", SMEM_TABLE, dict(dims=3, cws=(8, 8, 2), args=smem_table_args())),
        ("smem_hidden", SMEM_HIDDEN, dict(dims=2, cws=(64, 2, 1), args=smem_hidden_args())),
        ("smem_clobbered", SMEM_CLOBBERED, {}),
        ("index_rules", INDEX_RULES, {}),
        ("mad_rules", MAD_RULES, {}),
        ("pointer_rules", POINTER_RULES, dict(args=pointer_rules_args())),
        ("uninit_top", UNINIT_TOP, {}),
        ("second_dim", SECOND_DIM, dict(dims=2, cws=(64, 4, 1))),
        ("straight_global_id", STRAIGHT_GLOBAL_ID, {}),
    ]
    for name, src, kw in straight:
        out.append((name, kernel(closed(src), **kw)))
    for i, src in enumerate(LOOPS):
        out.append((f"loop{i}", kernel(src, dims=2, cws=(64, 4, 1))))
    out.append(("entry_and_unreachable", kernel(ENTRY_AND_UNREACHABLE)))
    return out
