"""Oracle pins for the per-instruction rules and the record checks.

Constant folding is compared with plain numpy integer arithmetic (a closed
form independent of the oracle), inline float constants with numpy's IEEE-754
bit patterns, and the lattice laws (join commutative, associative,
idempotent; every transfer monotone) are property-tested on random states."""
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import asmtext
import dcgen
import hand_kernels as hk
import oracle

TOP = oracle.TOP
NOARGS = np.zeros(0, dcgen.ARG_DTYPE)


def run_after(src, dims=1, cws=(64, 1, 1), args=NOARGS):
    recs = asmtext.assemble(src)
    d = dcgen.descriptor(len(recs), dims, cws, 1, len(args))
    stt = oracle.entry_state(d)
    for r in recs:
        stt = oracle.transfer(d, args, r, stt)
    return stt


def cval(v):
    return oracle.val(0, c=int(v) & 0xFFFFFFFF)


U32 = st.integers(0, 2 ** 32 - 1)


@settings(max_examples=60, deadline=None)
@given(U32, U32)
def test_fold_scalar(x, y):
    s = run_after(hk.fold_scalar_src(x, y))
    X, Y = np.uint64(x), np.uint64(y)
    m = np.uint64(0xFFFFFFFF)
    sh = int(y) & 31
    want = {
        3: (X + Y) & m, 10: (X - Y) & m, 11: (X * Y) & m, 12: X & Y, 13: X | Y,
        14: (X << np.uint64(sh)) & m, 15: X >> np.uint64(sh),
        112 + 3: X ^ Y, 112 + 4: ((X & np.uint64(0xFFFFFF)) * (Y & np.uint64(0xFFFFFF))) & m,
        112 + 5: (X << np.uint64(sh)) & m, 112 + 6: X >> np.uint64(sh),
        112 + 7: np.uint64(int(np.int32(np.uint32(x)) >> np.int32(sh)) & 0xFFFFFFFF),
        112 + 8: (((X & np.uint64(0xFFFFFF)) * (Y & np.uint64(0xFFFFFF))) + X) & m,
    }
    for slot, w in want.items():
        assert int(s[slot]["val"]) == cval(w), (slot, oracle.decode(s[slot]["val"]), int(w))


@settings(max_examples=40, deadline=None)
@given(U32, U32, U32, U32, st.integers(0, 63))
def test_fold_64(a, b, c, d, sh):
    s = run_after(hk.fold_64_src(a, b, c, d, sh))
    A = (b << 32) | a
    C = (d << 32) | c
    M = 2 ** 64 - 1
    for base, w in [(20, A & C), (22, A | C), (24, A ^ C), (26, A & (~C & M))]:
        assert int(s[base]["val"]) == cval(w & 0xFFFFFFFF)
        assert int(s[base + 1]["val"]) == cval(w >> 32)
    w = (A << sh) & M
    assert int(s[112 + 20]["val"]) == cval(w & 0xFFFFFFFF)
    assert int(s[112 + 21]["val"]) == cval(w >> 32)


def test_inline_constants():
    s = run_after(hk.INLINE_CONSTANTS)
    f32 = lambda x: int(np.float32(x).view(np.uint32))
    f64 = lambda x: int(np.float64(x).view(np.uint64))
    assert int(s[1]["val"]) == cval(f32(0.5))
    assert int(s[2]["val"]) == cval(f32(-4.0))
    assert int(s[113]["val"]) == cval(f32(1.0))
    assert (int(s[10]["val"]), int(s[11]["val"])) == (cval(f64(2.0) & 0xFFFFFFFF), cval(f64(2.0) >> 32))
    assert (int(s[12]["val"]), int(s[13]["val"])) == (cval(-16), cval(-1))
    assert (int(s[14]["val"]), int(s[15]["val"])) == (cval(64), cval(0))
    assert (int(s[16]["val"]), int(s[17]["val"])) == (cval(-70000), cval(-1))
    assert int(s[18]["val"]) == cval(100000)
    assert int(s[1]["prov"]) == 1 << 14 and int(s[1]["type"]) == 0


def test_float_ops_are_typed_not_folded():
    s = run_after(hk.FLOAT_OPS)
    for slot, ty in [(114, 4), (115, 4), (116, 4), (117, 2), (118, 8), (119, 8), (120, 8), (121, 8), (122, 2)]:
        assert int(s[slot]["val"]) == TOP and int(s[slot]["type"]) == ty, slot


def test_smem_table():
    """Exact (offset, width) entries, then per-dword resolution (Listing 3
    layout: offsets 0..2 at 0x0/0x8/0x10, hidden slots to 0x30, args)."""
    args = np.zeros(2, dcgen.ARG_DTYPE)
    args[0] = (0x30, 8, dcgen.T_PTR, dcgen.T_FLOAT)
    args[1] = (0x38, 4, dcgen.T_UINT, 0)
    s = run_after(hk.SMEM_TABLE, dims=3, cws=(8, 8, 2), args=args)
    v = oracle.val
    IDX, SYS, KARG = 4, 7, 2
    assert int(s[10]["val"]) == v(IDX, 1, 1, 4) and int(s[11]["val"]) == v(SYS, 2, 1, 0)
    assert int(s[12]["val"]) == v(IDX, 1, 2, 4) and int(s[13]["val"]) == v(SYS, 2, 2, 0)
    assert [int(s[16 + j]["val"]) for j in range(4)] == [v(IDX, 1, 0, 4), v(SYS, 2, 0, 0), v(IDX, 1, 1, 4),
                                                       v(SYS, 2, 1, 0)]
    assert int(s[16]["prov"]) == 1 << 6 and int(s[18]["prov"]) == 1 << 7
    # past the last argument: a plain global load
    assert int(s[20]["val"]) == TOP and int(s[20]["prov"]) == 1 << 15 and int(s[20]["type"]) == 0
    assert int(s[21]["val"]) == v(KARG, 2, arg=0) and int(s[21]["type"]) == dcgen.T_PTR
    assert int(s[22]["val"]) == v(KARG, 2, arg=0) and int(s[23]["val"]) == v(KARG, 0, arg=1)
    assert int(s[23]["prov"]) == 1 << 21 and int(s[23]["type"]) == dcgen.T_UINT
    # not through s[4:5]
    assert int(s[24]["val"]) == TOP and int(s[24]["prov"]) == 1 << 15
    # hidden slot, high half of the aqlwrap pointer
    assert int(s[25]["val"]) == v(SYS, 2, 2, 4) and int(s[25]["prov"]) == 1 << 19
    # a clobbered s4 keeps the syntactic type/provenance but loses the payload
    t = run_after(hk.SMEM_CLOBBERED)
    assert int(t[10]["val"]) == TOP and int(t[10]["prov"]) == 1 << 9 and int(t[10]["type"]) == dcgen.T_UINT



def test_smem_hidden_slots_and_mid_argument():
    """Listing 3's argument area dword by dword: the three hidden 8-byte
    pointer slots after the global offsets (printf buffer, vqueue, aqlwrap;
    low then high dword), an x2 and an x4 load starting in the last hidden
    slot (the x4 runs into the first user argument), a load in the middle of
    an 8-byte argument (its provenance and type, no payload), the work
    dimension at its printed offset, and the high dword of the first global
    offset read on its own."""
    s = run_after(hk.SMEM_HIDDEN, dims=2, cws=(64, 2, 1), args=hk.smem_hidden_args())
    v = oracle.val
    KARG, SYS = 2, 7
    HIDDEN, GOFF_HI, WORKDIM = 4, 0, 3
    P_HIDDEN = 1 << 19
    for slot, q, hi in [(10, 0, 0), (11, 0, 1), (12, 1, 0), (13, 1, 1), (14, 2, 0)]:
        assert int(s[slot]["val"]) == v(SYS, 2 if hi else 1, q, HIDDEN), slot
        assert int(s[slot]["prov"]) == P_HIDDEN and int(s[slot]["type"]) == 0, slot
    assert int(s[16]["val"]) == v(SYS, 1, 2, HIDDEN) and int(s[17]["val"]) == v(SYS, 2, 2, HIDDEN)
    assert [int(s[20 + j]["val"]) for j in range(4)] == [v(SYS, 1, 2, HIDDEN), v(SYS, 2, 2, HIDDEN),
                                                       v(KARG, 1, arg=0), v(KARG, 2, arg=0)]
    assert [int(s[20 + j]["prov"]) for j in range(4)] == [P_HIDDEN, P_HIDDEN, 1 << 20, 1 << 20]
    assert [int(s[20 + j]["type"]) for j in range(4)] == [0, 0, dcgen.T_PTR, dcgen.T_PTR]
    assert int(s[24]["val"]) == TOP and int(s[24]["prov"]) == 1 << 21 and int(s[24]["type"]) == dcgen.T_PTR
    assert int(s[25]["val"]) == v(SYS, 0, 0, WORKDIM) and int(s[25]["prov"]) == 1 << 12
    assert int(s[25]["type"]) == dcgen.T_UINT
    assert int(s[26]["val"]) == v(SYS, 2, 0, GOFF_HI) and int(s[26]["prov"]) == 1 << 6
    assert int(s[26]["type"]) == dcgen.T_UINT

def test_index_rules():
    s = run_after(hk.INDEX_RULES)
    v = oracle.val
    IDX, SHL = 4, 5
    assert int(s[0]["val"]) == v(IDX, 0, 0, 1)                 # WGID << log2(cws) -> group base
    assert int(s[1]["val"]) == TOP
    assert int(s[2]["val"]) == v(IDX, 0, 0, 1)                 # either operand order
    assert int(s[113]["val"]) == v(IDX, 0, 0, 3)
    assert int(s[114]["val"]) == v(IDX, 0, 0, 3, c=12)
    assert int(s[115]["val"]) == v(SHL, 0, 0, 3, 3)
    assert int(s[116]["val"]) == v(IDX, 0, 0, 3)               # shift by zero keeps the index
    assert int(s[117]["val"]) == TOP                            # shifts above 15 are not tracked
    assert int(s[118]["val"]) == v(SHL, 0, 0, 3, 3, c=5)
    assert int(s[119]["val"]) == v(IDX, 2, 0, 3)               # sign word of an index
    assert int(s[120]["val"]) == TOP                            # overlapping terms
    assert int(s[121]["val"]) == v(SHL, 0, 0, 3, 2, c=3)
    assert int(s[122]["val"]) == TOP                            # not a power of two
    assert int(s[123]["val"]) == TOP                            # SHL + SHL
    assert int(s[124]["val"]) == TOP                            # IDX + IDX.high


def test_mad_is_add_of_mul():
    s = run_after(hk.MAD_RULES)
    v = oracle.val
    assert int(s[121]["val"]) == v(5, 0, 0, 2, 2, c=3)
    assert int(s[122]["val"]) == v(4, 0, 0, 3)


def test_pointer_rules():
    args = np.zeros(1, dcgen.ARG_DTYPE)
    args[0] = (0x30, 8, dcgen.T_PTR, dcgen.T_INT)
    s = run_after(hk.POINTER_RULES, args=args)
    v = oracle.val
    PTR, SHL = 6, 5
    assert int(s[10]["val"]) == v(PTR, 1, arg=0, c=16)
    assert int(s[11]["val"]) == v(PTR, 2, arg=0)
    assert int(s[12]["val"]) == v(PTR, 1, arg=0, c=20)
    assert int(s[114]["val"]) == v(SHL, 1, 0, 2, 3) and int(s[115]["val"]) == v(SHL, 2, 0, 2, 3)
    assert int(s[116]["val"]) == v(PTR, 1, 0, 2, 3, arg=0, c=16)
    assert int(s[117]["val"]) == v(PTR, 2, arg=0)
    assert int(s[118]["val"]) == v(PTR, 1, 0, 2, 3, arg=0, c=20)
    assert int(s[13]["val"]) == TOP and int(s[14]["val"]) == TOP     # carries are not modelled
    assert int(s[116]["type"]) == dcgen.T_UINT | dcgen.T_PTR


def test_uninit_and_top():
    s = run_after(hk.UNINIT_TOP)
    assert int(s[115]["val"]) == oracle.val(8) and int(s[115]["prov"]) == 1 << 17
    assert int(s[116]["val"]) == TOP and int(s[116]["prov"]) == (1 << 17) | (1 << 14)
    assert int(s[30]["val"]) == TOP and int(s[30]["prov"]) == 1 << 18


# ------------------------------------------------------------------ checks

def status_of(src=None, recs=None, **kw):
    if recs is None:
        recs = asmtext.assemble(src)
    d = dcgen.descriptor(len(recs), **kw)
    return oracle.kernel_status(recs, d)


def rec(name, r0=0xFFFF, r1=0xFFFF, r2=0xFFFF, imm=0, target=-1):
    x = np.zeros(1, dcgen.INSTR_DTYPE)
    x[0] = (dcgen.opcode(name), r0, r1, r2, imm, target)
    return x


END = rec("s_endpgm")


@pytest.mark.parametrize("bad", [
    rec("s_mov_b64", 1, 2),                       # odd scalar pair
    rec("s_mov_b32", 112, 2),                     # vector dst on a scalar op
    rec("v_mov_b32", 3, 112),                     # scalar dst on a vector op
    rec("s_load_dwordx4", 2, 4, imm=0),           # x4 destination not 4-aligned
    rec("s_load_dword", 2, 5, imm=0),             # odd sbase
    rec("s_mov_b32", 110, 1),                     # reserved id
    rec("s_mov_b32", 108, 1),                     # SCC is never an explicit operand
    rec("s_endpgm", 3),                           # unused field not none
    rec("global_store_dword", 0x8000 + 17, 114),  # store data must be a VGPR
    rec("v_mad_u32_u24", 113, 0xFFFE, 114, imm=114),   # literal where imm holds src2
    rec("v_mad_u32_u24", 113, 114, 115, imm=0x10072),  # src2 id out of range
    rec("v_lshlrev_b64", 367, 0x8012, 114),       # pair runs past v255
    rec("v_mov_b32", 113, 0x8051),                # inline id between ints and floats
    rec("global_load_dword", 113, 114, 3),        # odd saddr
])
def test_badreg(bad):
    recs = np.concatenate([bad, END])
    assert status_of(recs=recs) == oracle.E_BADREG


def test_status_order():
    assert status_of(recs=np.concatenate([rec("s_endpgm"), END]).copy()) == 0
    badop = END.copy()
    badop[0]["op"] = dcgen.lib().dcgen_n_ops()
    assert status_of(recs=np.concatenate([badop, END])) == oracle.E_BADOP
    assert status_of(recs=np.concatenate([rec("s_branch", target=2), END])) == oracle.E_BADTARGET
    assert status_of(recs=np.concatenate([rec("s_branch", target=-3), END])) == oracle.E_BADTARGET
    assert status_of(recs=np.concatenate([rec("s_nop", target=1), END])) == oracle.E_BADTARGET
    # the first bad record decides; within a record, operands before target
    assert status_of(recs=np.concatenate([rec("s_branch", 3, target=9), rec("s_mov_b64", 1, 2), END])) == \
        oracle.E_BADREG
    assert status_of(recs=np.concatenate([rec("s_nop", target=0), rec("s_mov_b64", 1, 2), END])) == \
        oracle.E_BADTARGET
    # control must not fall off the end
    assert status_of(recs=rec("v_mov_b32", 113, 112)) == oracle.E_NOEND
    assert status_of(recs=np.concatenate([END, rec("s_cbranch_scc0", target=0)])) == oracle.E_NOEND
    assert status_of(recs=np.concatenate([END, rec("s_branch", target=0)])) == 0
    assert status_of(recs=np.zeros(0, dcgen.INSTR_DTYPE)) == oracle.E_NOEND
    # descriptor: only the useargs ABI with 1..3 dims and nonzero sizes
    assert status_of(recs=END, useargs=0) == oracle.E_UNSUPPORTED
    assert status_of(recs=END, dims=0) == oracle.E_UNSUPPORTED
    assert status_of(recs=END, dims=4) == oracle.E_UNSUPPORTED
    assert status_of(recs=END, dims=2, cws=(64, 0, 1)) == oracle.E_UNSUPPORTED
    assert status_of(recs=END, dims=1, cws=(64, 0, 0)) == 0
    assert status_of(recs=END, n_args=256) == oracle.E_UNSUPPORTED


def test_generated_records_valid():
    for cfg in (1, 2, 3, 5):
        b = dcgen.generate(cfg, 300)
        s, _, _ = oracle.analyze_batch(b)
        assert np.all(s["status"] == 0), cfg


# ------------------------------------------------------------------ lattice laws

def random_slot_vals(rng, n):
    """A mix of payloads: TOP, UNINIT, constants and random tagged values
    (with the unused bits [39:32] zero)."""
    kinds = rng.integers(0, 4, n)
    out = np.empty(n, np.uint64)
    for i, k in enumerate(kinds):
        if k == 0:
            out[i] = TOP
        elif k == 1:
            out[i] = oracle.val(8)
        elif k == 2:
            out[i] = oracle.val(0, c=int(rng.integers(0, 2 ** 32)))
        else:
            out[i] = oracle.val(int(rng.integers(0, 8)), int(rng.integers(0, 3)), int(rng.integers(0, 3)),
                                int(rng.integers(0, 8)), int(rng.integers(0, 16)), int(rng.integers(0, 4)),
                                int(rng.integers(0, 256)))
    return out


def random_state(rng, base=None):
    s = np.zeros(368, oracle.SLOT_DTYPE)
    s["prov"] = rng.integers(0, 2 ** 32, 368, dtype=np.uint64).astype(np.uint32) & rng.integers(
        0, 2 ** 32, 368, dtype=np.uint64).astype(np.uint32)
    s["type"] = rng.integers(0, 32, 368).astype(np.uint8)
    s["val"] = random_slot_vals(rng, 368)
    if base is not None:   # keep s4/s5 plausibly a system pointer sometimes
        s[4], s[5] = base[4], base[5]
    return s


def leq(a, b):
    return bool(np.all((a["prov"] & ~b["prov"]) == 0) and np.all((a["type"] & ~b["type"]) == 0) and
                np.all((a["val"] == b["val"]) | (b["val"] == np.uint64(TOP))))


@settings(max_examples=40, deadline=None)
@given(st.integers(0, 2 ** 32 - 1))
def test_join_laws(seed):
    rng = np.random.default_rng(seed)
    a, b, c = random_state(rng), random_state(rng), random_state(rng)
    ab = oracle.join(a, b)
    assert ab.tobytes() == oracle.join(b, a).tobytes()
    assert oracle.join(ab, c).tobytes() == oracle.join(a, oracle.join(b, c)).tobytes()
    assert oracle.join(a, a).tobytes() == a.tobytes()
    assert leq(a, ab) and leq(b, ab)


_POOL = dcgen.generate(2, 40)


@settings(max_examples=60, deadline=None)
@given(st.integers(0, 2 ** 32 - 1))
def test_transfer_monotone(seed):
    rng = np.random.default_rng(seed)
    k = int(rng.integers(0, _POOL.n_kernels))
    recs, d, a = _POOL.kernel(k)
    entry = oracle.entry_state(d)
    x = random_state(rng, entry if rng.integers(0, 2) else None)
    y = oracle.join(x, random_state(rng))
    for i in rng.integers(0, len(recs), 12):
        fx = oracle.transfer(d, a, recs[i], x)
        fy = oracle.transfer(d, a, recs[i], y)
        assert leq(fx, fy), (dcgen.op_names()[recs[i]["op"]], i)
        # no stray bits in the packed fields
        assert np.all(fx["flags"] == 0) and np.all(fx["pad0"] == 0) and np.all(fx["type"] < 32)


def test_second_dimension_uses_its_own_size():
    """get_num_groups(1) and the group-base term of dimension 1 divide or
    multiply by the second .cws entry, not the first."""
    s = run_after(hk.SECOND_DIM, dims=2, cws=(64, 4, 1))
    v = oracle.val
    assert int(s[11]["val"]) == v(7, 0, 1, 2)
    assert int(s[12]["val"]) == TOP
    assert int(s[13]["val"]) == v(4, 0, 1, 1)
    assert int(s[14]["val"]) == TOP
    assert int(s[115]["val"]) == v(4, 0, 1, 3)


def test_hand_kernels_valid():
    """The shared hand-written kernels are well formed (the GPU parity test
    runs the same list)."""
    for name, (recs, d, a) in hk.all_kernels():
        assert oracle.kernel_status(recs, d) == 0, name
        r = oracle.analyze(recs, d, a)
        assert r["status"] == 0 and r["n_blocks"] >= 2, name
