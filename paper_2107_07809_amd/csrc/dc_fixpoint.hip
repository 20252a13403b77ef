/*
 * dc_fixpoint.hip -- steps a5-a9 on gfx950: the register-state fixpoint of
 * every kernel of a batch (Section "Register state analysis" of the paper:
 * a forward pass over the control flow graph that tracks, per register, where
 * its value came from and what type it carries), and the extraction of memory
 * accesses (Section "The body extraction") and work-item built-ins (Section
 * "Work-item built-in functions").
 *
 * Layout of the work.  A persistent grid; one wavefront takes one kernel at a
 * time from an atomic counter.  Per kernel:
 *
 *   1. Compact slots.  The lanes mark every register slot the kernel's records
 *      name (plus vcc, exec, scc and the argument pointer s[4:5]); a ballot
 *      prefix numbers them.  A slot no record names keeps its ABI entry value
 *      on every path, so only the U named slots are carried (U <= 368).
 *   2. Register-resident state.  The working state of a block lives in VGPRs:
 *      compact slot c is lane c % 64 of row c / 64, three words per slot
 *      (provenance bits; payload low word; payload high word with the type bits
 *      in its low byte).  Two rows hold up to 128 slots, six rows any kernel.
 *   3. Chunks.  A block's records are staged 64 at a time, one per lane:
 *      descriptor lookup, compact operand indices and constant operand values
 *      are computed lane-parallel.  A wave-uniform loop then applies the
 *      transfer of each instruction in order, reading sources with readlane
 *      and writing definitions with a lane select.
 *   4. Emission on every visit.  Access and built-in records of a visit are
 *      written into the block's own region of the sparse outputs (one slot per
 *      instruction, four per instruction for built-ins) with the block's counts;
 *      a block's last visit runs on its fixpoint IN state, so the last write
 *      is the result and no extraction walk is needed.
 *   5. Joins.  The OUT state is joined lane-parallel into each successor's IN
 *      state in an HBM arena; a ballot detects change and marks the successor
 *      dirty in a bitmap over reverse-postorder positions.  Passes sweep that
 *      bitmap in order (the round-robin schedule).
 *
 * Control flow in the wave-uniform parts depends only on uniform values
 * (readlane / readfirstlane results and loop counters).  Lane-dependent
 * choices are selects: a store that only some lanes should make is a store by
 * every lane whose address is the real one or a per-lane scratch word.  A
 * lane-predicated branch around uniform code lets the optimiser thread the
 * predicate across a loop back edge and split the wave.
 */
#include "dc_device.h"

namespace dc {

constexpr int32_t ST_OK_FIX = 0;
constexpr uint32_t CX_NONE = 0x1FFu;       /* compact index of a non-register operand */
constexpr uint32_t HTOP = 0xFFFFFF00u;     /* payload high word of TOP, type bits cleared */
constexpr uint32_t ROW_DW = FIX_ROW_DWORDS;   /* arena dwords of one state row: 3 words x 64 lanes */
constexpr int RMAX = (int)FIX_MAX_ROWS;       /* rows for any kernel: 6 x 64 >= NSLOT */
constexpr uint32_t USLOT_N = RMAX * 64;
constexpr uint32_t MAIN_MAX_BLOCKS = 2048; /* register bitmap: 64 lanes x 32 bits */

/* per-wavefront LDS */
struct WaveLds {
    uint16_t umap[USLOT_N];         /* slot -> compact index; entries >= NSLOT unused */
    uint16_t uslot[USLOT_N + 64];   /* compact index -> slot; 64-entry scratch tail */
    uint8_t umark[USLOT_N + 64];    /* slot marks; entries >= NSLOT are scratch */
    uint32_t tail[64];              /* scratch words for single-lane bitmap stores */
};
static_assert(sizeof(WaveLds) % 16 == 0, "LDS layout");

/* ------------------------------------------------------------------ */
/* abstract values                                                      */
/* ------------------------------------------------------------------ */
struct SV {
    uint32_t prov, type;
    uint64_t val;
};

struct KCtx {
    uint32_t cws0, cws1, cws2, n_args;
    const dc_arg_t *args;
    __device__ __forceinline__ uint32_t cws(uint32_t d) const { return d == 0 ? cws0 : d == 1 ? cws1 : cws2; }
};

__device__ __forceinline__ bool is_c(uint64_t v) { return v != VTOP && v_tag(v) == T_CONST; }
__device__ __forceinline__ uint64_t C32(uint32_t c) { return (uint64_t)c; }
__device__ __forceinline__ bool idx_lo(uint64_t v) { return v != VTOP && v_tag(v) == T_IDX && v_ig(v) <= IG_LO; }
__device__ __forceinline__ int lg2(uint32_t x) {
    /* exact base-2 logarithm, -1 when x is not a power of two */
    return (x != 0 && (x & (x - 1)) == 0) ? (int)__builtin_ctz(x) : -1;
}

/* ---- payload rules (Section "Register state analysis": index arithmetic,
 *      pointer formation from an argument base plus a scaled index) ---- */
__device__ uint64_t r_add1(uint64_t a, uint64_t b) {
    const uint32_t ta = v_tag(a), tb = v_tag(b);
    if (is_c(a) && is_c(b)) return C32(v_c(a) + v_c(b));
    if (idx_lo(a) && idx_lo(b) && v_dim(a) == v_dim(b) && (v_aux(a) & v_aux(b)) == 0)
        return pv(T_IDX, IG_ENT, v_dim(a), v_aux(a) | v_aux(b), 0, 0, v_c(a) + v_c(b));
    if (idx_lo(a) && is_c(b)) return pv(T_IDX, IG_ENT, v_dim(a), v_aux(a), 0, 0, v_c(a) + v_c(b));
    if (ta == T_SHL && v_ig(a) == IG_ENT && is_c(b)) return pv(T_SHL, IG_ENT, v_dim(a), v_aux(a), v_sh(a), 0, v_c(a) + v_c(b));
    if (ta == T_KARG && v_ig(a) == IG_LO) {
        if (tb == T_SHL && v_ig(b) == IG_LO) return pv(T_PTR, IG_LO, v_dim(b), v_aux(b), v_sh(b), v_arg(a), v_c(b));
        if (is_c(b)) return pv(T_PTR, IG_LO, 0, 0, 0, v_arg(a), v_c(b));
    }
    if (ta == T_PTR && v_ig(a) == IG_LO) {
        if (is_c(b)) return pv(T_PTR, IG_LO, v_dim(a), v_aux(a), v_sh(a), v_arg(a), v_c(a) + v_c(b));
        if (tb == T_SHL && v_ig(b) == IG_LO && v_dim(a) == 0 && v_aux(a) == 0 && v_sh(a) == 0)
            return pv(T_PTR, IG_LO, v_dim(b), v_aux(b), v_sh(b), v_arg(a), v_c(a) + v_c(b));
    }
    return VTOP;
}
__device__ __forceinline__ uint64_t r_add(uint64_t a, uint64_t b) {
    if (a == VTOP || b == VTOP) return VTOP;
    const uint64_t r = r_add1(a, b);
    return r != VTOP ? r : r_add1(b, a);
}
__device__ __forceinline__ bool ptr_hi(uint64_t v) {
    return v != VTOP && (v_tag(v) == T_KARG || v_tag(v) == T_PTR) && v_ig(v) == IG_HI;
}
__device__ __forceinline__ bool ext_hi(uint64_t v) {
    return v != VTOP && (((v_tag(v) == T_SHL || v_tag(v) == T_IDX) && v_ig(v) == IG_HI) || (is_c(v) && v_c(v) == 0));
}
__device__ __forceinline__ uint64_t r_addc(uint64_t a, uint64_t b) {
    if (ptr_hi(a) && ext_hi(b)) return pv(T_PTR, IG_HI, 0, 0, 0, v_arg(a), 0);
    if (ptr_hi(b) && ext_hi(a)) return pv(T_PTR, IG_HI, 0, 0, 0, v_arg(b), 0);
    return VTOP;
}
/* IDX shifted left by s */
__device__ __forceinline__ uint64_t idx_shl(uint64_t a, uint32_t s) {
    if (s == 0) return pv(T_IDX, IG_ENT, v_dim(a), v_aux(a), 0, 0, v_c(a));
    if (s > 15) return VTOP;
    return pv(T_SHL, IG_ENT, v_dim(a), v_aux(a), s, 0, v_c(a) << s);
}
__device__ uint64_t r_mul1(const KCtx &K, uint64_t a, uint64_t b) {
    if (is_c(a) && is_c(b)) return C32(v_c(a) * v_c(b));
    if (!is_c(b)) return VTOP;
    if (a != VTOP && v_tag(a) == T_WGID) {
        const uint32_t d = v_dim(a);
        return (K.cws(d) != 0 && v_c(b) == K.cws(d)) ? pv(T_IDX, IG_ENT, d, M_WG, 0, 0, 0) : VTOP;
    }
    if (idx_lo(a)) {
        const int s = lg2(v_c(b));
        if (s >= 0) return idx_shl(a, (uint32_t)s);
    }
    return VTOP;
}
__device__ __forceinline__ uint64_t r_mul(const KCtx &K, uint64_t a, uint64_t b) {
    if (a == VTOP || b == VTOP) return VTOP;
    const uint64_t r = r_mul1(K, a, b);
    return r != VTOP ? r : r_mul1(K, b, a);
}
__device__ __forceinline__ uint64_t low24(uint64_t v) { return is_c(v) ? C32(v_c(v) & 0xFFFFFFu) : v; }
__device__ uint64_t r_shl(const KCtx &K, uint64_t x, uint64_t amt) {
    if (x == VTOP || !is_c(amt)) return VTOP;
    const uint32_t s = v_c(amt) & 31u;
    if (is_c(x)) return C32(v_c(x) << s);
    if (idx_lo(x)) return idx_shl(x, s);
    if (v_tag(x) == T_WGID && lg2(K.cws(v_dim(x))) == (int)s) return pv(T_IDX, IG_ENT, v_dim(x), M_WG, 0, 0, 0);
    return VTOP;
}
__device__ uint64_t r_lshr(const KCtx &K, uint64_t x, uint64_t amt) {
    if (x == VTOP || !is_c(amt)) return VTOP;
    const uint32_t s = v_c(amt) & 31u;
    if (is_c(x)) return C32(v_c(x) >> s);
    if (v_tag(x) == T_SYS && v_aux(x) == K_GSIZE && v_ig(x) == IG_ENT && lg2(K.cws(v_dim(x))) == (int)s)
        return pv(T_SYS, IG_ENT, v_dim(x), K_NUMGROUPS, 0, 0, 0);
    return VTOP;
}
__device__ uint64_t r_ashr(uint64_t x, uint64_t amt) {
    if (x == VTOP || !is_c(amt)) return VTOP;
    const uint32_t s = v_c(amt) & 31u;
    if (is_c(x)) return C32((uint32_t)((int32_t)v_c(x) >> s));
    if (idx_lo(x) && s == 31) return pv(T_IDX, IG_HI, v_dim(x), v_aux(x), 0, 0, 0);
    return VTOP;
}

/* one dword of the kernel-argument area addressed by s[4:5] (Listing 3 of
 * the paper: hidden offsets first, user arguments at their .arg offsets) */
__device__ __forceinline__ void arg_dword(const KCtx &K, uint32_t o, uint32_t &prov, uint32_t &type, uint64_t &val) {
    if ((o & 3u) == 0 && o < 0x30u) {
        const uint32_t q = o >> 3, hi = (o >> 2) & 1u;
        if (o < 0x18u) {   /* global offsets x, y, z */
            prov = 1u << (PB_GOFF + q);
            type = TY_U;
            val = hi ? pv(T_SYS, IG_HI, q, K_GOFFHI, 0, 0, 0) : pv(T_IDX, IG_LO, q, M_GOFF, 0, 0, 0);
        } else {           /* printf buffer, vqueue, aqlwrap */
            prov = 1u << PB_HIDDEN;
            type = 0;
            val = pv(T_SYS, hi ? IG_HI : IG_LO, q - 3, K_HIDDEN, 0, 0, 0);
        }
        return;
    }
    if (o == 0x20010u) {
        prov = 1u << PB_WORKDIM;
        type = TY_U;
        val = pv(T_SYS, IG_ENT, 0, K_WORKDIM, 0, 0, 0);
        return;
    }
    for (uint32_t k = 0; k < K.n_args; k++) {
        const uint32_t off = rfl(K.args[k].offset), sz = rfl(K.args[k].size);
        if (o >= off && (uint64_t)o < (uint64_t)off + sz) {
            prov = 1u << (PB_KARG + (k < 11 ? k : 11));
            type = rfl(K.args[k].type);
            if (sz == 4 && o == off) val = pv(T_KARG, IG_ENT, 0, 0, 0, k, 0);
            else if (sz == 8 && o == off) val = pv(T_KARG, IG_LO, 0, 0, 0, k, 0);
            else if (sz == 8 && o == off + 4) val = pv(T_KARG, IG_HI, 0, 0, 0, k, 0);
            else val = VTOP;
            return;
        }
    }
    prov = 1u << PB_LOADG;
    type = 0;
    val = VTOP;
}

/* recognised work-item built-ins (Section "Work-item built-in functions");
 * returns the DC_SV_* kind or -1 */
__device__ __forceinline__ int builtin_kind(uint64_t v, uint32_t &dim) {
    if (v == VTOP) return -1;
    const uint32_t t = v_tag(v), ig = v_ig(v), m = v_aux(v);
    dim = v_dim(v);
    if (t == T_IDX && v_c(v) == 0) {
        if (ig == IG_ENT && m == (M_WG | M_LID | M_GOFF)) return DC_SV_GLOBAL_ID;
        if (ig == IG_ENT && m == (M_WG | M_LID)) return DC_SV_GLOBAL_ID_MINUS_OFFSET;
        if (ig == IG_LO && m == M_GOFF) return DC_SV_GLOBAL_OFFSET;
        if (ig == IG_ENT && m == M_WG) return DC_SV_GROUP_BASE;
        if (ig == IG_ENT && m == M_LID) return DC_SV_LOCAL_ID;
        return -1;
    }
    if (t == T_SYS && ig == IG_ENT) {
        if (m == K_GSIZE) return DC_SV_GLOBAL_SIZE;
        if (m == K_NUMGROUPS) return DC_SV_NUM_GROUPS;
        if (m == K_WORKDIM) { dim = 0; return DC_SV_WORK_DIM; }
        return -1;
    }
    if (t == T_WGID) return DC_SV_GROUP_ID;
    return -1;
}

/* ABI entry state of slot j (Section "Register state analysis": s[4:5] the
 * argument pointer, s6.. group ids, v0.. local ids, exec the launch mask,
 * every other register uninitialised), as (prov, type, payload lo, hi) */
__device__ __forceinline__ uint4 entry_slot(uint32_t j, uint32_t dims) {
    uint32_t prov = 1u << PB_UNINIT, type = 0;
    uint64_t val = pv(T_UNINIT, 0, 0, 0, 0, 0, 0);
    if (j == 4u || j == 5u) {
        prov = 1u << PB_SYSPTR;
        val = pv(T_SYSPTR, j == 4u ? IG_LO : IG_HI, 0, 0, 0, 0, 0);
    } else if (j >= 6u && j < 6u + dims) {
        prov = 1u << (PB_WGID + (j - 6u));
        type = TY_U;
        val = pv(T_WGID, IG_ENT, j - 6u, 0, 0, 0, 0);
    } else if (j >= 112u && j < 112u + dims) {
        prov = 1u << (PB_LID + (j - 112u));
        type = TY_U;
        val = pv(T_IDX, IG_ENT, j - 112u, M_LID, 0, 0, 0);
    } else if (j == 106u || j == 107u) {
        prov = 1u << PB_MASK;
        val = VTOP;
    }
    return make_uint4(prov, type, (uint32_t)val, (uint32_t)(val >> 32));
}

/* in-register form of a payload: high word with the type bits in its low
 * byte (payload bits 39:32 are always zero; TOP's become HTOP) */
__device__ __forceinline__ uint32_t pack_hi(uint64_t val, uint32_t type) {
    return ((uint32_t)(val >> 32) & 0xFFFFFF00u) | type;
}
__device__ __forceinline__ uint64_t unpack_val(uint32_t lo, uint32_t hi) {
    return hi >= HTOP ? VTOP : (((uint64_t)(hi & 0xFFFFFF00u) << 32) | lo);
}

/* ------------------------------------------------------------------ */
/* register-resident state                                              */
/* ------------------------------------------------------------------ */
template <int R>
struct St {
    uint32_t p[R], lo[R], hi[R];
};

template <int R>
__device__ __forceinline__ uint32_t rdc(const uint32_t (&a)[R], uint32_t c) {
    const uint32_t ln = c & 63u, row = c >> 6;
    uint32_t x = rdl(a[0], ln);
#pragma unroll
    for (int r = 1; r < R; r++) x = row == (uint32_t)r ? rdl(a[r], ln) : x;
    return x;
}
template <int R>
__device__ __forceinline__ SV get(const St<R> &S, uint32_t c) {
    SV v;
    v.prov = rdc(S.p, c);
    const uint32_t lo = rdc(S.lo, c), hi = rdc(S.hi, c);
    v.type = hi & 0xFFu;
    v.val = unpack_val(lo, hi);
    return v;
}
template <int R>
__device__ __forceinline__ uint32_t get_prov(const St<R> &S, uint32_t c) { return rdc(S.p, c); }
template <int R>
__device__ __forceinline__ uint32_t get_type(const St<R> &S, uint32_t c) { return rdc(S.hi, c) & 0xFFu; }

template <int R>
__device__ __forceinline__ void put(St<R> &S, uint32_t c, uint32_t prov, uint32_t type, uint64_t val) {
    const uint32_t lo = (uint32_t)val, hi = pack_hi(val, type);
    const uint32_t row = c >> 6;
    const bool me = lane_id() == (c & 63u);
#pragma unroll
    for (int r = 0; r < R; r++) {
        const bool sel = me && row == (uint32_t)r;
        S.p[r] = sel ? prov : S.p[r];
        S.lo[r] = sel ? lo : S.lo[r];
        S.hi[r] = sel ? hi : S.hi[r];
    }
}

template <int R>
__device__ __forceinline__ void st_load(St<R> &S, const uint32_t *a) {
    const uint32_t l = lane_id();
#pragma unroll
    for (int r = 0; r < R; r++) {
        S.p[r] = a[r * ROW_DW + l];
        S.lo[r] = a[r * ROW_DW + 64 + l];
        S.hi[r] = a[r * ROW_DW + 128 + l];
    }
}
template <int R>
__device__ __forceinline__ void st_store(const St<R> &S, uint32_t *a) {
    const uint32_t l = lane_id();
#pragma unroll
    for (int r = 0; r < R; r++) {
        a[r * ROW_DW + l] = S.p[r];
        a[r * ROW_DW + 64 + l] = S.lo[r];
        a[r * ROW_DW + 128 + l] = S.hi[r];
    }
}
/* a := a join S (provenance and type bits unite; payloads that differ go to
 * TOP); true when a changed */
template <int R>
__device__ __forceinline__ bool st_join(const St<R> &S, uint32_t *a) {
    const uint32_t l = lane_id();
    St<R> J;
    bool ch = false;
#pragma unroll
    for (int r = 0; r < R; r++) {
        const uint32_t pa = a[r * ROW_DW + l], la = a[r * ROW_DW + 64 + l], ha = a[r * ROW_DW + 128 + l];
        const uint32_t pb = S.p[r], lb = S.lo[r], hb = S.hi[r];
        const bool same = la == lb && (ha & 0xFFFFFF00u) == (hb & 0xFFFFFF00u);
        const uint32_t ty = (ha | hb) & 0xFFu;
        J.p[r] = pa | pb;
        J.lo[r] = same ? la : 0xFFFFFFFFu;
        J.hi[r] = (same ? (ha & 0xFFFFFF00u) : HTOP) | ty;
        ch = ch || J.p[r] != pa || J.lo[r] != la || J.hi[r] != ha;
    }
    const bool any = ballot(ch) != 0;
    if (any) st_store(J, a);
    return any;
}

/* ------------------------------------------------------------------ */
/* block bitmaps                                                        */
/* ------------------------------------------------------------------ */
/* up to 2048 bits in one VGPR: lane w holds bits [32w, 32w + 32) */
struct RegBits {
    uint32_t w;
    __device__ __forceinline__ void init(uint32_t) { w = 0; }
    __device__ __forceinline__ bool get(uint32_t i) const { return (rdl(w, i >> 5) >> (i & 31)) & 1u; }
    __device__ __forceinline__ bool get_lane(uint32_t i) const {   /* i differs per lane, i < 2048 */
        return (__shfl(w, (int)(i >> 5), 64) >> (i & 31)) & 1u;
    }
    __device__ __forceinline__ void set(uint32_t i) { w = lane_id() == (i >> 5) ? w | (1u << (i & 31)) : w; }
    __device__ __forceinline__ void clr(uint32_t i) { w = lane_id() == (i >> 5) ? w & ~(1u << (i & 31)) : w; }
    /* first set bit >= from, or n if none (bits >= n are never set) */
    __device__ __forceinline__ uint32_t next(uint32_t from, uint32_t n) const {
        const uint32_t l = lane_id(), fw = from >> 5;
        uint32_t x = l < fw ? 0u : w;
        x = l == fw ? x & (~0u << (from & 31)) : x;
        x = from >= n ? 0u : x;
        const uint64_t m = ballot(x != 0);
        if (m == 0) return n;
        const uint32_t fl = (uint32_t)__builtin_ctzll(m);
        return (fl << 5) + (uint32_t)__builtin_ctz(rdl(x, fl));
    }
};
/* any size, in global memory; lanes other than 0 store into a scratch tail */
struct MemBits {
    uint32_t *bm, *tail;
    __device__ __forceinline__ void init(uint32_t n) {
        const uint32_t words = (n + 31) >> 5;
        for (uint32_t i = lane_id(); i < words; i += 64) bm[i] = 0;
        /* other lanes read these words through lane 0 */
        __threadfence_block();
        __builtin_amdgcn_wave_barrier();
    }
    __device__ __forceinline__ bool get(uint32_t i) const { return (rfl(bm[i >> 5]) >> (i & 31)) & 1u; }
    __device__ __forceinline__ bool get_lane(uint32_t i) const { return (bm[i >> 5] >> (i & 31)) & 1u; }
    __device__ __forceinline__ void set(uint32_t i) {
        const uint32_t v = rfl(bm[i >> 5]) | (1u << (i & 31));
        *(lane_id() == 0 ? &bm[i >> 5] : &tail[lane_id()]) = v;
    }
    __device__ __forceinline__ void clr(uint32_t i) {
        const uint32_t v = rfl(bm[i >> 5]) & ~(1u << (i & 31));
        *(lane_id() == 0 ? &bm[i >> 5] : &tail[lane_id()]) = v;
    }
    __device__ __forceinline__ uint32_t next(uint32_t from, uint32_t n) const {
        const uint32_t l = lane_id();
        for (uint32_t w0 = from >> 5; (w0 << 5) < n; w0 += 64) {
            const uint32_t wi = w0 + l;
            uint32_t x = bm[(wi << 5) < n ? wi : w0];
            x = (wi << 5) < n ? x : 0u;
            x = wi == (from >> 5) ? x & (~0u << (from & 31)) : x;
            const uint64_t m = ballot(x != 0);
            if (m) {
                const uint32_t fl = (uint32_t)__builtin_ctzll(m);
                return ((w0 + fl) << 5) + (uint32_t)__builtin_ctz(rdl(x, fl));
            }
        }
        return n;
    }
};

/* ------------------------------------------------------------------ */
/* staged chunk: one instruction per lane                                */
/* ------------------------------------------------------------------ */
struct Stage {
    uint32_t x, y, z;          /* record words: op | r0 << 16, r1 | r2 << 16, imm */
    uint32_t elo, ehi;         /* opcode descriptor */
    uint32_t cx;               /* compact indices: r0 [8:0], r1 [17:9], r2 [26:18] */
    uint32_t cc;               /* compact index of the third source [8:0] */
    uint32_t ka0, ka1, kb0, kb1, kc0;  /* dwords of non-register sources */
};

/* dword j of a non-register source id of width w (inline integer, inline
 * float, or the record's literal) */
__device__ __forceinline__ uint32_t const_dword(uint32_t id, uint32_t j, uint32_t w, int32_t lit) {
    if (id <= 0x8050u) {
        const int32_t k = (int32_t)(id - 0x8000u) - 16;
        return j == 0 ? (uint32_t)k : (k < 0 ? 0xFFFFFFFFu : 0u);
    }
    if (id >= 0x8060u && id <= 0x8067u) {
        /* +-0.5, +-1, +-2, +-4: sign in bit 0 of the index, magnitude 2^(q/2-1) */
        const uint32_t q = id - 0x8060u, neg = q & 1u, m = q >> 1;
        if (w == 1) return (neg << 31) | ((126u + m) << 23);
        return j == 0 ? 0u : (neg << 31) | ((1022u + m) << 20);
    }
    return j == 0 ? (uint32_t)lit : (lit < 0 ? 0xFFFFFFFFu : 0u);
}

__device__ __forceinline__ uint32_t cmap(const WaveLds &L, uint32_t id) {
    return id < (uint32_t)NSLOT ? (uint32_t)L.umap[id] : CX_NONE;
}

/* records of positions [g0, g0 + cnt) of the kernel starting at pos0 */
__device__ __forceinline__ Stage stage_chunk(const Plan *__restrict__ P, const WaveLds &L, uint64_t rb, uint32_t pos0,
                                             uint32_t g0, uint32_t cnt) {
    const uint32_t l = lane_id();
    const uint32_t li = l < cnt ? l : cnt - 1;   /* spare lanes repeat the last record */
    const uint4 r = reinterpret_cast<const uint4 *>(P->instrs)[rb + (g0 + li - pos0)];
    const uint64_t e = OPTAB[r.x & 0xFFFFu];
    Stage T;
    T.x = r.x;
    T.y = r.y;
    T.z = r.z;
    T.elo = (uint32_t)e;
    T.ehi = (uint32_t)(e >> 32);
    const uint32_t r0 = r.x >> 16, r1 = r.y & 0xFFFFu, r2 = r.y >> 16;
    const int32_t imm = (int32_t)r.z;
    T.cx = cmap(L, r0) | cmap(L, r1) << 9 | cmap(L, r2) << 18;
    const bool third = e_role(e, 3) != RO_NO;
    T.cc = third ? cmap(L, (uint32_t)imm) : CX_NONE;
    const uint32_t w1 = e_width(e, 1), w2 = e_width(e, 2), w3 = e_width(e, 3);
    T.ka0 = const_dword(r1, 0, w1, imm);
    T.ka1 = const_dword(r1, 1, w1, imm);
    T.kb0 = const_dword(r2, 0, w2, imm);
    T.kb1 = const_dword(r2, 1, w2, imm);
    T.kc0 = const_dword((uint32_t)imm, 0, w3, 0);
    return T;
}

/* ------------------------------------------------------------------ */
/* record buffers (one record per lane, flushed lane-parallel)          */
/* ------------------------------------------------------------------ */
struct Emit {
    uint32_t a0, a1, a2, a3;   /* access: instr, kind|space<<8|width<<16|dtype<<24, addr lo, hi */
    uint32_t s0, s1;           /* built-in: instr, slot|kind<<16|dim<<24 */
    uint32_t na, ns;           /* buffered counts (uniform) */
    uint32_t ta, ts;           /* records already written for this visit (uniform) */
};

__device__ __forceinline__ void flush_acc(const Plan *__restrict__ P, Emit &E, uint32_t g_lo, uint4 *dummy) {
    if (E.na == 0) return;
    const uint32_t l = lane_id();
    uint4 *dst = l < E.na ? reinterpret_cast<uint4 *>(P->acc_sparse) + g_lo + E.ta + l : dummy + l;
    *dst = make_uint4(E.a0, E.a1, E.a2, E.a3);
    E.ta += E.na;
    E.na = 0;
}
__device__ __forceinline__ void flush_sys(const Plan *__restrict__ P, Emit &E, uint32_t g_lo, uint4 *dummy) {
    if (E.ns == 0) return;
    const uint32_t l = lane_id();
    uint2 *dst = l < E.ns ? reinterpret_cast<uint2 *>(P->sys_sparse) + 4ull * g_lo + E.ts + l
                          : reinterpret_cast<uint2 *>(dummy + l);
    *dst = make_uint2(E.s0, E.s1);
    E.ts += E.ns;
    E.ns = 0;
}

/* ------------------------------------------------------------------ */
/* one instruction                                                      */
/* ------------------------------------------------------------------ */
struct KConst {
    uint32_t cv;      /* compact index of vcc (exec = cv + 2, scc = cv + 4) */
};

template <int R>
__device__ __forceinline__ SV src(const St<R> &S, uint32_t c, uint32_t j, uint32_t k) {
    if (c != CX_NONE) return get(S, c + j);
    SV v;
    v.prov = 1u << PB_CONST;
    v.type = 0;
    v.val = C32(k);
    return v;
}

/* the access record of a memory instruction from the pre-state */
template <int R>
__device__ __forceinline__ void emit_access(const St<R> &S, const KCtx &K, uint64_t e, uint32_t cx, uint32_t y,
                                            int32_t imm, uint32_t instr, Emit &E) {
    const uint32_t cls = e_cls(e), w0 = e_width(e, 0);
    const uint32_t cd = cx & 0x1FFu, ca = (cx >> 9) & 0x1FFu;
    uint32_t kind, space, width;
    uint64_t addr = VTOP;
    if (cls == C_GLD || cls == C_FLD || cls == C_GST || cls == C_FST) {
        kind = (cls == C_GLD || cls == C_FLD) ? 0 : 1;
        space = (cls == C_GLD || cls == C_GST) ? 0 : 1;
        width = 4 * w0;
        if ((y >> 16) == 0xFFFFu && ca != CX_NONE) {
            const uint64_t lo = get(S, ca).val, hi = get(S, ca + 1).val;
            if (lo != VTOP && hi != VTOP && v_ig(lo) == IG_LO && v_ig(hi) == IG_HI && v_arg(lo) == v_arg(hi)) {
                if (v_tag(lo) == T_PTR && v_tag(hi) == T_PTR)
                    addr = pv(T_PTR, IG_ENT, v_dim(lo), v_aux(lo), v_sh(lo), v_arg(lo), v_c(lo) + (uint32_t)imm);
                else if (v_tag(lo) == T_KARG && v_tag(hi) == T_KARG)
                    addr = pv(T_PTR, IG_ENT, 0, 0, 0, v_arg(lo), (uint32_t)imm);
            }
        }
    } else {   /* C_DSR, C_DSW */
        kind = cls == C_DSR ? 0 : 1;
        space = 2;
        width = 4;
        if (ca != CX_NONE) {
            const uint64_t v = get(S, ca).val;
            if (v != VTOP) {
                const uint32_t c = v_c(v) + (uint32_t)imm;
                if (v_tag(v) == T_SHL && v_ig(v) == IG_ENT) addr = pv(T_SHL, IG_ENT, v_dim(v), v_aux(v), v_sh(v), 0, c);
                else if (idx_lo(v)) addr = pv(T_IDX, IG_ENT, v_dim(v), v_aux(v), 0, 0, c);
                else if (is_c(v)) addr = C32(c);
            }
        }
    }
    uint32_t dt = 0;
    if (kind == 1) {
        for (uint32_t j = 0; j < w0; j++) dt |= get_type(S, cd + j);
    } else if (addr != VTOP && v_tag(addr) == T_PTR && v_arg(addr) < K.n_args) {
        dt = rfl(K.args[v_arg(addr)].flags) & 31u;
    }
    const bool me = lane_id() == E.na;
    E.a0 = me ? instr : E.a0;
    E.a1 = me ? (kind | space << 8 | width << 16 | dt << 24) : E.a1;
    E.a2 = me ? (uint32_t)addr : E.a2;
    E.a3 = me ? (uint32_t)(addr >> 32) : E.a3;
    E.na++;
}

__device__ __forceinline__ void emit_sysval(uint64_t v, uint32_t slot, uint32_t instr, Emit &E) {
    uint32_t dim;
    const int kind = builtin_kind(v, dim);
    if (kind < 0) return;
    const bool me = lane_id() == E.ns;
    E.s0 = me ? instr : E.s0;
    E.s1 = me ? (slot | (uint32_t)kind << 16 | dim << 24) : E.s1;
    E.ns++;
}

/* transfer of instruction i of the staged chunk, with emission */
template <int R>
__device__ __forceinline__ void step(St<R> &S, const KCtx &K, const KConst &KC, const Stage &T, uint32_t i,
                                     uint32_t instr, Emit &E) {
    const uint32_t x = rdl(T.x, i), y = rdl(T.y, i);
    const int32_t imm = (int32_t)rdl(T.z, i);
    const uint64_t e = ((uint64_t)rdl(T.ehi, i) << 32) | rdl(T.elo, i);
    const uint32_t cx = rdl(T.cx, i);
    const uint32_t cls = e_cls(e);
    const uint32_t cd = cx & 0x1FFu, ca = (cx >> 9) & 0x1FFu, cb = cx >> 18;
    const uint32_t r0 = x >> 16;

    if (cls >= C_GLD) emit_access(S, K, e, cx, y, imm, instr, E);

    uint64_t dv[4] = {VTOP, VTOP, VTOP, VTOP};
    uint32_t nd = 0;
    if (cls == C_SMEM) {
        const uint32_t w = e_width(e, 0);
        const bool via = (y & 0xFFFFu) == 4u;
        const bool ok = via && get(S, ca).val == pv(T_SYSPTR, IG_LO, 0, 0, 0, 0, 0) &&
                        get(S, ca + 1).val == pv(T_SYSPTR, IG_HI, 0, 0, 0, 0, 0);
        const uint32_t off = (uint32_t)imm;
        uint32_t pr[4], ty[4];
        uint64_t va[4];
#pragma unroll
        for (uint32_t j = 0; j < 4; j++) {
            pr[j] = 1u << PB_LOADG;
            ty[j] = 0;
            va[j] = VTOP;
            if (via && j < w) arg_dword(K, off + 4u * j, pr[j], ty[j], va[j]);
        }
        if (via && w == 2 && (off == 0u || off == 8u || off == 16u)) {
            const uint32_t d = off >> 3;
            pr[0] = pr[1] = 1u << (PB_GOFF + d);
            ty[0] = ty[1] = TY_U;
            va[0] = pv(T_IDX, IG_LO, d, M_GOFF, 0, 0, 0);
            va[1] = pv(T_SYS, IG_HI, d, K_GOFFHI, 0, 0, 0);
        } else if (via && w == 1 && (off == 0xCu || off == 0x10u || off == 0x14u)) {
            const uint32_t d = (off - 0xCu) >> 2;
            pr[0] = 1u << (PB_GSIZE + d);
            ty[0] = TY_U;
            va[0] = pv(T_SYS, IG_ENT, d, K_GSIZE, 0, 0, 0);
        } else if (via && w == 1 && off == 0x20010u) {
            pr[0] = 1u << PB_WORKDIM;
            ty[0] = TY_U;
            va[0] = pv(T_SYS, IG_ENT, 0, K_WORKDIM, 0, 0, 0);
        }
#pragma unroll
        for (uint32_t j = 0; j < 4; j++) {
            dv[j] = ok ? va[j] : VTOP;
            if (j < w) put(S, cd + j, pr[j], ty[j], dv[j]);
        }
        nd = w;
    } else if (cls == C_GLD || cls == C_FLD || cls == C_DSR) {
        const uint32_t w = e_width(e, 0);
        const uint32_t pr = cls == C_DSR ? 1u << PB_LOADL : 1u << PB_LOADG;
#pragma unroll
        for (uint32_t j = 0; j < 4; j++)
            if (j < w) put(S, cd + j, pr, 0, VTOP);
        nd = w;
    } else if (cls == C_SALU || cls == C_SCMP || cls == C_VALU || cls == C_VCMP) {
        const uint32_t w1 = e_role(e, 1) != RO_NO ? e_width(e, 1) : 0;
        const uint32_t w2 = e_role(e, 2) != RO_NO ? e_width(e, 2) : 0;
        const uint32_t w3 = e_role(e, 3) != RO_NO ? e_width(e, 3) : 0;
        SV a0 = {0, 0, VTOP}, a1 = {0, 0, VTOP}, b0 = {0, 0, VTOP}, b1 = {0, 0, VTOP}, c0 = {0, 0, VTOP};
        uint32_t rp = 0;
        if (w1) { a0 = src(S, ca, 0, rdl(T.ka0, i)); rp |= a0.prov; }
        if (w1 == 2) { a1 = src(S, ca, 1, rdl(T.ka1, i)); rp |= a1.prov; }
        if (w2) { b0 = src(S, cb, 0, rdl(T.kb0, i)); rp |= b0.prov; }
        if (w2 == 2) { b1 = src(S, cb, 1, rdl(T.kb1, i)); rp |= b1.prov; }
        if (w3) {
            const uint32_t cc = rdl(T.cc, i);
            c0 = src(S, cc, 0, rdl(T.kc0, i));
            rp |= c0.prov;
            if (w3 == 2) rp |= cc != CX_NONE ? get_prov(S, cc + 1) : (1u << PB_CONST);
        }
        const uint32_t iu = e_iuse(e);
        if (iu & IM_VCC) rp |= get_prov(S, KC.cv) | get_prov(S, KC.cv + 1);
        if (iu & IM_EXEC) rp |= get_prov(S, KC.cv + 2) | get_prov(S, KC.cv + 3);
        if (iu & IM_SCC) rp |= get_prov(S, KC.cv + 4);

        const uint32_t rrole = e_role(e, 0);
        if (rrole == RO_SD || rrole == RO_VD) {
            const uint32_t w0 = e_width(e, 0);
            uint32_t ty0 = 0, ty1 = 0;
            switch (e_trule(e)) {
            case TR_SUF: ty0 = ty1 = e_suffix(e); break;
            case TR_ADD: ty0 = ty1 = e_suffix(e) | ((a0.type | a1.type | b0.type | b1.type) & TY_P); break;
            case TR_B: {
                const uint32_t vs = e_vsrc(e);
                uint32_t t = 0;
                if (vs & 1u) t |= a0.type | a1.type;
                if (vs & 2u) t |= b0.type | b1.type;
                ty0 = ty1 = t;
                break;
            }
            case TR_MOVE: ty0 = a0.type; ty1 = a1.type; break;
            default: break;
            }
            uint64_t v0 = VTOP, v1 = VTOP;
            const bool val_is_r1 = e_vsrc(e) == 1u;   /* shift forms: which operand is shifted */
            switch (e_prule(e)) {
            case PR_MOV: v0 = a0.val; v1 = a1.val; break;
            case PR_ADD: v0 = r_add(a0.val, b0.val); break;
            case PR_ADDC: v0 = r_addc(a0.val, b0.val); break;
            case PR_SUB: if (is_c(a0.val) && is_c(b0.val)) v0 = C32(v_c(a0.val) - v_c(b0.val)); break;
            case PR_AND: if (is_c(a0.val) && is_c(b0.val)) v0 = C32(v_c(a0.val) & v_c(b0.val)); break;
            case PR_OR: if (is_c(a0.val) && is_c(b0.val)) v0 = C32(v_c(a0.val) | v_c(b0.val)); break;
            case PR_XOR: if (is_c(a0.val) && is_c(b0.val)) v0 = C32(v_c(a0.val) ^ v_c(b0.val)); break;
            case PR_MUL: v0 = r_mul(K, a0.val, b0.val); break;
            case PR_MUL24: v0 = r_mul(K, low24(a0.val), low24(b0.val)); break;
            case PR_MAD24: v0 = r_add(r_mul(K, low24(a0.val), low24(b0.val)), c0.val); break;
            case PR_SHL: v0 = val_is_r1 ? r_shl(K, a0.val, b0.val) : r_shl(K, b0.val, a0.val); break;
            case PR_LSHR: v0 = val_is_r1 ? r_lshr(K, a0.val, b0.val) : r_lshr(K, b0.val, a0.val); break;
            case PR_ASHR: v0 = val_is_r1 ? r_ashr(a0.val, b0.val) : r_ashr(b0.val, a0.val); break;
            case PR_SEL: v0 = a0.val == b0.val ? a0.val : VTOP; break;
            case PR_AND64: case PR_OR64: case PR_XOR64: case PR_ANDN264:
                if (is_c(a0.val) && is_c(a1.val) && is_c(b0.val) && is_c(b1.val)) {
                    const uint32_t pr = e_prule(e);
                    const uint32_t x0 = v_c(a0.val), x1 = v_c(a1.val), y0 = v_c(b0.val), y1 = v_c(b1.val);
                    if (pr == PR_AND64) { v0 = C32(x0 & y0); v1 = C32(x1 & y1); }
                    else if (pr == PR_OR64) { v0 = C32(x0 | y0); v1 = C32(x1 | y1); }
                    else if (pr == PR_XOR64) { v0 = C32(x0 ^ y0); v1 = C32(x1 ^ y1); }
                    else { v0 = C32(x0 & ~y0); v1 = C32(x1 & ~y1); }
                }
                break;
            case PR_SHL64: {
                const uint64_t amt = a0.val, lo = b0.val, hi = b1.val;
                if (!is_c(amt) || lo == VTOP || hi == VTOP) break;
                const uint32_t s = v_c(amt) & 63u;
                if (is_c(lo) && is_c(hi)) {
                    const uint64_t xx = (((uint64_t)v_c(hi) << 32) | v_c(lo)) << s;
                    v0 = C32((uint32_t)xx);
                    v1 = C32((uint32_t)(xx >> 32));
                } else if (idx_lo(lo) && ((is_c(hi) && v_c(hi) == 0) ||
                                          (v_tag(hi) == T_IDX && v_ig(hi) == IG_HI && v_dim(hi) == v_dim(lo) &&
                                           v_aux(hi) == v_aux(lo)))) {
                    if (s == 0) { v0 = lo; v1 = hi; }
                    else if (s <= 15) {
                        v0 = pv(T_SHL, IG_LO, v_dim(lo), v_aux(lo), s, 0, v_c(lo) << s);
                        v1 = pv(T_SHL, IG_HI, v_dim(lo), v_aux(lo), s, 0, 0);
                    }
                }
                break;
            }
            default: break;
            }
            const uint32_t prov = rp | (e_maskdef(e) ? 1u << PB_MASK : 0u);
            dv[0] = v0;
            dv[1] = v1;
            put(S, cd, prov, ty0, v0);
            if (w0 == 2) put(S, cd + 1, prov, ty1, v1);
            nd = w0;
        }
        const uint32_t idf = e_idef(e);
        const uint32_t ip = rp | (1u << PB_MASK);
        if (idf & IM_VCC) { put(S, KC.cv, ip, 0, VTOP); put(S, KC.cv + 1, ip, 0, VTOP); }
        if (idf & IM_EXEC) { put(S, KC.cv + 2, ip, 0, VTOP); put(S, KC.cv + 3, ip, 0, VTOP); }
        if (idf & IM_SCC) put(S, KC.cv + 4, ip, 0, VTOP);
        /* built-ins among the explicit definitions (an implicit definition of
         * the same slot overwrote the value with TOP) */
#pragma unroll
        for (uint32_t j = 0; j < 2; j++) {
            const uint32_t slot = r0 + j;
            const bool covered = ((idf & IM_VCC) && (slot == 104u || slot == 105u)) ||
                                 ((idf & IM_EXEC) && (slot == 106u || slot == 107u)) ||
                                 ((idf & IM_SCC) && slot == 108u);
            if (j < nd && !covered) emit_sysval(dv[j], slot, instr, E);
        }
        return;
    }
#pragma unroll
    for (uint32_t j = 0; j < 4; j++)
        if (j < nd) emit_sysval(dv[j], r0 + j, instr, E);
}

/* ------------------------------------------------------------------ */
/* one kernel                                                           */
/* ------------------------------------------------------------------ */
/* mark the slots the kernel names and number them; returns U */
__device__ __forceinline__ uint32_t build_compact(const Plan *__restrict__ P, WaveLds &L, uint64_t rb, uint32_t n) {
    const uint32_t l = lane_id();
    uint32_t *mk = reinterpret_cast<uint32_t *>(L.umark);
    for (uint32_t j = 0; j < (USLOT_N + 64) / 4; j += 64) mk[(j + l) < (USLOT_N + 64) / 4 ? j + l : l] = 0;
    /* LDS is in order within a wavefront; the barriers only order the lanes
     * of emulated builds and keep the compiler from moving code across */
    __builtin_amdgcn_wave_barrier();
    const uint4 *recs = reinterpret_cast<const uint4 *>(P->instrs) + rb;
    const uint32_t junk = USLOT_N + l;
    for (uint32_t g0 = 0; g0 < n; g0 += 64) {
        const uint32_t gi = g0 + l < n ? g0 + l : n - 1;
        const uint4 r = recs[gi];
        const uint64_t e = OPTAB[r.x & 0xFFFFu];
        const uint32_t id[4] = {r.x >> 16, r.y & 0xFFFFu, r.y >> 16, r.z};
#pragma unroll
        for (int o = 0; o < 4; o++) {
            const uint32_t w = e_role(e, o) != RO_NO ? e_width(e, o) : 0;
#pragma unroll
            for (uint32_t j = 0; j < 4; j++) {
                const uint32_t s = id[o] + j;
                L.umark[(j < w && id[o] < (uint32_t)NSLOT && s < (uint32_t)NSLOT) ? s : junk] = 1;
            }
        }
    }
    /* vcc, exec, scc (implicit operands) and the argument pointer */
    L.umark[l < 5 ? 104 + l : (l < 7 ? l - 1 : junk)] = 1;
    __builtin_amdgcn_wave_barrier();
    uint32_t base = 0;
#pragma unroll
    for (uint32_t grp = 0; grp < RMAX; grp++) {
        const uint32_t s = grp * 64 + l;
        const bool f = s < (uint32_t)NSLOT && L.umark[s] != 0;
        const uint64_t m = ballot(f);
        const uint32_t c = base + lanes_below(m);
        L.umap[s] = (uint16_t)(f ? c : CX_NONE);
        L.uslot[f ? c : USLOT_N + l] = (uint16_t)s;
        base += (uint32_t)__builtin_popcountll(m);
    }
    __builtin_amdgcn_wave_barrier();
    return base;
}

/* per-wave arena, bitmaps and scratch */
struct WaveMem {
    uint32_t *arena;
    uint4 *dummy;
};

template <int R, class Bits>
__device__ __forceinline__ void analyze(const Plan *__restrict__ P, uint32_t k, WaveLds &L, Bits &reached,
                                        Bits &dirty, const WaveMem &M, uint32_t nu) {
    const uint32_t l = lane_id();
    const dc_kernel_t *D = &P->kernels[k];
    const uint32_t nb = rfl(P->n_blocks[k]), fb = rfl(P->first_block[k]), nr = rfl(P->n_reach[k]);
    const uint32_t pos0 = rfl(P->pos_begin[k]);
    KCtx K;
    K.cws0 = rfl(D->cws[0]);
    K.cws1 = rfl(D->cws[1]);
    K.cws2 = rfl(D->cws[2]);
    K.n_args = rfl(D->n_args);
    K.args = P->args + rfl(D->arg_begin);
    const uint64_t rb = ((uint64_t)rfl((uint32_t)(D->instr_begin >> 32)) << 32) | rfl((uint32_t)D->instr_begin);
    const uint32_t dims = rfl(D->dims);
    KConst KC;
    KC.cv = L.umap[104];
    KC.cv = rfl(KC.cv);
    const uint32_t blk_dw = (uint32_t)R * ROW_DW;

    reached.init(nb);
    dirty.init(nr);
    /* IN[0] = the ABI entry state on the compact slots */
    {
        St<R> S;
#pragma unroll
        for (int r = 0; r < R; r++) {
            const uint32_t c = (uint32_t)r * 64 + l;
            const uint4 v = c < nu ? entry_slot(L.uslot[c], dims) : make_uint4(0, 0, 0, 0);
            S.p[r] = v.x;
            S.lo[r] = v.z;
            S.hi[r] = (v.w & 0xFFFFFF00u) | v.y;
        }
        st_store(S, M.arena);
    }
    reached.set(0);
    dirty.set(0);   /* block 0 is first in reverse postorder */
    const uint32_t sweep_cap = P->sweep_cap ? P->sweep_cap : 64u + 2u * nb;
    uint32_t sweeps = 0, pos = nr;
    int32_t status = ST_OK_FIX;
    for (;;) {
        uint32_t p = dirty.next(pos, nr);
        if (p >= nr) {
            p = dirty.next(0, nr);
            if (p >= nr) break;
            if (++sweeps > sweep_cap) {
                status = DC_E_NOFIX;
                break;
            }
        }
        dirty.clr(p);
        pos = p + 1;
        const uint32_t b = rfl(P->rpo[fb + p]);
        St<R> S;
        st_load(S, M.arena + (uint64_t)b * blk_dw);
        const uint32_t g_lo = rfl(P->block_start[fb + b]), g_hi = rfl(P->block_start[fb + b + 1]);
        Emit E;
        E.a0 = E.a1 = E.a2 = E.a3 = E.s0 = E.s1 = 0;
        E.na = E.ns = E.ta = E.ts = 0;
        for (uint32_t g0 = g_lo; g0 < g_hi; g0 += 64) {
            const uint32_t cnt = min(64u, g_hi - g0);
            const Stage T = stage_chunk(P, L, rb, pos0, g0, cnt);
            for (uint32_t i = 0; i < cnt; i++) {
                if (E.ns > 60) flush_sys(P, E, g_lo, M.dummy);
                step(S, K, KC, T, i, g0 + i - pos0, E);
            }
            flush_acc(P, E, g_lo, M.dummy);
        }
        flush_sys(P, E, g_lo, M.dummy);
        P->blk_acc[fb + b] = E.ta;
        P->blk_sys[fb + b] = E.ts;
        for (int ed = 0; ed < 2; ed++) {
            const int32_t s = (int32_t)rfl((uint32_t)P->succ[2 * (uint64_t)(fb + b) + ed]);
            if (s < 0) continue;
            uint32_t *dst = M.arena + (uint64_t)s * blk_dw;
            bool changed;
            if (!reached.get((uint32_t)s)) {
                st_store(S, dst);
                reached.set((uint32_t)s);
                changed = true;
            } else {
                changed = st_join(S, dst);
            }
            if (changed) dirty.set(rfl((uint32_t)P->rpo_pos[fb + (uint32_t)s]));
        }
    }

    /* counts of blocks without a valid last visit are zero */
    const bool ok = status == ST_OK_FIX;
    for (uint32_t b0 = 0; b0 < nb; b0 += 64) {
        const uint32_t b = b0 + l;
        const bool rch = reached.get_lane(b < nb ? b : 0);   /* every lane takes part in the exchange */
        const bool keep = ok && b < nb && rch;
        uint32_t *pa = keep || b >= nb ? reinterpret_cast<uint32_t *>(M.dummy + l) : P->blk_acc + fb + b;
        uint32_t *ps = keep || b >= nb ? reinterpret_cast<uint32_t *>(M.dummy + l) + 1 : P->blk_sys + fb + b;
        *pa = 0;
        *ps = 0;
    }

    dc_kernel_result_t res = {status, 0, 0, 0, 0, 0, 0};
    if (ok) {
        uint64_t dig = 0;
        const bool want_dig = (P->flags & DC_OPT_DIGEST) != 0, want_ex = (P->flags & DC_OPT_EXPORT_STATES) != 0;
        if (want_dig || want_ex) {
            /* the lanes read state words other lanes stored */
            __threadfence_block();
            __builtin_amdgcn_wave_barrier();
            for (uint32_t b = 0; b < nb; b++) {
                const bool rb_ = reached.get(b);
                const uint32_t *a = M.arena + (uint64_t)b * blk_dw;
                uint64_t h = 0;
                for (uint32_t j0 = 0; j0 < USLOT_N; j0 += 64) {
                    const uint32_t j = j0 + l;
                    const uint32_t c = j < (uint32_t)NSLOT ? L.umap[j] : CX_NONE;
                    uint32_t prov, type;
                    uint64_t val;
                    if (c != CX_NONE) {
                        const uint32_t o = (c >> 6) * ROW_DW + (c & 63u);
                        prov = a[o];
                        const uint32_t lo = a[o + 64], hi = a[o + 128];
                        type = hi & 0xFFu;
                        val = unpack_val(lo, hi);
                    } else {
                        const uint4 v = entry_slot(j, dims);
                        prov = v.x;
                        type = v.y;
                        val = ((uint64_t)v.w << 32) | v.z;
                    }
                    if (want_ex) {
                        uint4 *ex = reinterpret_cast<uint4 *>(P->export_states) + (uint64_t)(fb + b) * NSLOT;
                        const uint4 xv = rb_ ? make_uint4(prov, type, (uint32_t)val, (uint32_t)(val >> 32))
                                             : make_uint4(0, 0, 0, 0);
                        *(j < (uint32_t)NSLOT ? ex + j : M.dummy + l) = xv;
                    }
                    const uint64_t z = mix64(val + 0x9E3779B97F4A7C15ull * ((uint64_t)b * NSLOT + j + 1));
                    h += j < (uint32_t)NSLOT ? mix64(z ^ ((uint64_t)prov | ((uint64_t)(type & 0xFFu) << 32))) : 0ull;
                }
                if (want_ex) {
                    uint8_t *er = P->export_reached + fb + b;
                    *(l == 0 ? er : reinterpret_cast<uint8_t *>(M.dummy + l)) = rb_ ? 1 : 0;
                }
                if (!rb_ || !want_dig) continue;
                for (int d = 32; d >= 1; d >>= 1) {
                    const uint32_t lo = (uint32_t)h, hi = (uint32_t)(h >> 32);
                    h += ((uint64_t)__shfl_xor(hi, d, 64) << 32) | __shfl_xor(lo, d, 64);
                }
                dig += h + mix64(0xB10C0000ull + b);
            }
        }
        res.n_blocks = nb;
        res.sweeps = sweeps;
        res.digest = dig;
    } else if (P->flags & DC_OPT_EXPORT_STATES) {
        for (uint32_t b = 0; b < nb; b++) {
            uint4 *ex = reinterpret_cast<uint4 *>(P->export_states) + (uint64_t)(fb + b) * NSLOT;
            for (uint32_t j0 = 0; j0 < USLOT_N; j0 += 64) {
                const uint32_t j = j0 + l;
                *(j < (uint32_t)NSLOT ? ex + j : M.dummy + l) = make_uint4(0, 0, 0, 0);
            }
            uint8_t *er = P->export_reached + fb + b;
            *(l == 0 ? er : reinterpret_cast<uint8_t *>(M.dummy + l)) = 0;
        }
    }
    /* n_access / n_sysval are filled from the block counts after the launch */
    P->results[k] = res;
}

/* a kernel that fails before the fixpoint: status only, no records */
__device__ __forceinline__ void fail_kernel(const Plan *__restrict__ P, uint32_t k, int32_t status, const WaveMem &M) {
    const uint32_t l = lane_id();
    const uint32_t nb = rfl(P->n_blocks[k]), fb = rfl(P->first_block[k]);
    for (uint32_t b0 = 0; b0 < nb; b0 += 64) {
        const uint32_t b = b0 + l;
        *(b < nb ? P->blk_acc + fb + b : reinterpret_cast<uint32_t *>(M.dummy + l)) = 0;
        *(b < nb ? P->blk_sys + fb + b : reinterpret_cast<uint32_t *>(M.dummy + l) + 1) = 0;
    }
    if (P->flags & DC_OPT_EXPORT_STATES) {
        for (uint32_t b = 0; b < nb; b++) {
            uint4 *ex = reinterpret_cast<uint4 *>(P->export_states) + (uint64_t)(fb + b) * NSLOT;
            for (uint32_t j0 = 0; j0 < USLOT_N; j0 += 64) {
                const uint32_t j = j0 + l;
                *(j < (uint32_t)NSLOT ? ex + j : M.dummy + l) = make_uint4(0, 0, 0, 0);
            }
            uint8_t *er = P->export_reached + fb + b;
            *(l == 0 ? er : reinterpret_cast<uint8_t *>(M.dummy + l)) = 0;
        }
    }
    dc_kernel_result_t res = {status, 0, 0, 0, 0, 0, 0};
    P->results[k] = res;
}

/* rows of state for U compact slots */
__device__ __forceinline__ uint32_t rows_for(uint32_t nu) { return nu <= 128u ? 2u : (uint32_t)RMAX; }

/* Persistent grid.  Main pass: kernels whose blocks fit the register bitmap
 * and whose IN states fit the wave's arena; the others are queued for the
 * overflow pass, which keeps its bitmaps in HBM and has a larger arena. */
template <bool OVF>
__global__ __launch_bounds__(256) void k_fixpoint(const Plan *__restrict__ P, uint32_t wpg) {
    extern __shared__ uint4 smem[];
    const uint32_t w = rfl(threadIdx.x >> 6), l = lane_id();
    WaveLds &L = reinterpret_cast<WaveLds *>(smem)[w];
    const uint32_t gw = blockIdx.x * wpg + w;
    WaveMem M;
    uint32_t cap_rows;
    if (!OVF) {
        cap_rows = P->arena_rows;
        M.arena = P->arena + (uint64_t)gw * cap_rows * ROW_DW;
        M.dummy = P->dummy + (uint64_t)gw * 64;
    } else {
        cap_rows = P->ovf_rows;
        M.arena = P->ovf_arena + (uint64_t)gw * cap_rows * ROW_DW;
        M.dummy = P->dummy + ((uint64_t)P->main_waves + gw) * 64;
    }
    for (;;) {
        /* branch-free: every lane takes part, only lane 0 adds 1 */
        const uint32_t idx = rfl(atomicAdd(&P->counters[OVF ? 2 : 0], l == 0 ? 1u : 0u));
        const uint32_t limit = OVF ? rfl(P->counters[1]) : P->n_kernels;
        if (idx >= limit) break;
        const uint32_t k = OVF ? rfl(P->ovf_list[idx]) : idx;
        const int32_t status = (int32_t)rfl((uint32_t)P->status[k]);
        if (status != ST_OK_FIX) {
            fail_kernel(P, k, status, M);
            continue;
        }
        const uint32_t nb = rfl(P->n_blocks[k]), n = rfl(P->pos_begin[k + 1]) - rfl(P->pos_begin[k]);
        const dc_kernel_t *D = &P->kernels[k];
        const uint64_t rb = ((uint64_t)rfl((uint32_t)(D->instr_begin >> 32)) << 32) | rfl((uint32_t)D->instr_begin);
        const uint32_t nu = rfl(build_compact(P, L, rb, n));
        const uint32_t R = rows_for(nu);
        if (!OVF) {
            if (nb > MAIN_MAX_BLOCKS || (uint64_t)nb * R > cap_rows) {
                const uint32_t slot = rfl(atomicAdd(&P->counters[1], l == 0 ? 1u : 0u));
                *(l == 0 ? &P->ovf_list[slot] : reinterpret_cast<uint32_t *>(M.dummy + l)) = k;
                continue;
            }
            RegBits reached, dirty;
            if (R == 2) analyze<2>(P, k, L, reached, dirty, M, nu);
            else analyze<RMAX>(P, k, L, reached, dirty, M, nu);
        } else {
            if ((uint64_t)nb * R > cap_rows) {
                fail_kernel(P, k, DC_E_UNSUPPORTED, M);
                continue;
            }
            const uint32_t words = (P->ovf_block_cap + 31) >> 5;
            uint32_t *bm = P->ovf_bitmaps + (uint64_t)gw * (2 * words + 64);
            MemBits reached{bm, bm + 2 * words}, dirty{bm + words, bm + 2 * words};
            if (R == 2) analyze<2>(P, k, L, reached, dirty, M, nu);
            else analyze<RMAX>(P, k, L, reached, dirty, M, nu);
        }
    }
}

uint32_t fixpoint_groups_per_cu(uint32_t wpg) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_fixpoint<false>, (int)(64 * wpg), wpg * sizeof(WaveLds)) !=
            hipSuccess ||
        n < 1)
        n = 1;
    return (uint32_t)n;
}

hipError_t launch_fixpoint(const Plan &P, const Plan *dP, const FixCfg &c, hipStream_t s, hipEvent_t before,
                           hipEvent_t after) {
    hipError_t e = launch_fill_u32(P.counters, 4, 0u, s);
    if (e != hipSuccess) return e;
    if (before && (e = hipEventRecord(before, s)) != hipSuccess) return e;
    if (P.n_kernels == 0) return after ? hipEventRecord(after, s) : hipSuccess;
    const uint32_t wpg = (uint32_t)c.waves_per_group;
    hipLaunchKernelGGL(k_fixpoint<false>, dim3(c.groups), dim3(64 * wpg), wpg * sizeof(WaveLds), s, dP, wpg);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (after && (e = hipEventRecord(after, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_fixpoint<true>, dim3(P.ovf_waves), dim3(64), sizeof(WaveLds), s, dP, 1u);
    return hipGetLastError();
}

}  // namespace dc
