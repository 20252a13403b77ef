/* dc_fixpoint_core.h -- the per-kernel fixpoint and extraction on one
 * wavefront (compact slots, chunk pipeline, joins, the pass schedule), shared
 * by the persistent batch kernel (dc_fixpoint.hip) and the one-launch-per-
 * kernel form (dc_plain.hip).  The design is described in dc_fixpoint.hip. */
#pragma once
#include "dc_device.h"

namespace dc {

constexpr int32_t ST_OK_FIX = 0;
constexpr uint32_t CX_NONE = 0x1FFu;          /* compact index of a non-register operand */
constexpr uint32_t HTOP = 0xFFFFFF00u;        /* arena: payload high word of TOP, type bits cleared */
constexpr uint32_t ROW_DW = FIX_ROW_DWORDS;   /* arena dwords of 64 slots: 3 words each */
constexpr int RMAX = (int)FIX_MAX_ROWS;       /* 6 x 64 >= NSLOT */
constexpr uint32_t USLOT_N = RMAX * 64;
constexpr uint32_t MAIN_MAX_BLOCKS = 2048;    /* register bitmap: 64 lanes x 32 bits */

/* LDS value tables: [0, 384) the block state by compact slot; [IX_DEF + 64 k
 * + i) definition k of the chunk's instruction i (k < 4 the explicit dwords,
 * k = 4 the implicit registers); IX_CONST an inline or literal source; IX_ZERO
 * no source. */
constexpr uint32_t IX_DEF = USLOT_N;
constexpr uint32_t K_IMP = 4;
constexpr uint32_t IX_CONST = IX_DEF + 5 * 64;
constexpr uint32_t IX_ZERO = IX_CONST + 1;
constexpr uint32_t IX_SCR = IX_ZERO + 1;      /* 64 per-lane scratch entries */
constexpr uint32_t TBL_N = IX_SCR + 64 + 6;
/* fpt entry: provenance bits | (type bits [4:0], T [5], N [6]) << 32, where T:
 * the payload may be other than TOP, N: other than TOP and uninitialised */
constexpr uint32_t FT_T = 1u << 5, FT_N = 1u << 6;

/* per-wavefront LDS */
struct WaveLds {
    uint64_t fpt[TBL_N];
    uint64_t fv[TBL_N];             /* payloads */
    uint64_t dm[USLOT_N + 64];      /* per compact slot: the chunk's lanes that define it; tail scratch */
    uint64_t junk[64];              /* per-lane scratch stores */
    uint32_t lcd[64];               /* per lane: compact index of r0 | implicit definitions << 16 */
    uint64_t optab[80];             /* opcode descriptors */
    uint16_t umap[USLOT_N];         /* slot -> compact index; entries >= NSLOT unused */
    uint16_t uslot[USLOT_N + 64];   /* compact index -> slot; 64-entry scratch tail */
    uint32_t tail[64];              /* scratch words for single-lane bitmap stores */
    uint8_t argf[64];               /* pointee type bits of the kernel's first 64 arguments */
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

/* ---- payload rules (Section "Search for memory accesses": the global id
 *      composed from group id, work-group size, local id and offset; array
 *      accesses as an argument base plus a scaled index) ---- */
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
        const uint32_t off = K.args[k].offset, sz = K.args[k].size;
        if (o >= off && (uint64_t)o < (uint64_t)off + sz) {
            prov = 1u << (PB_KARG + (k < 11 ? k : 11));
            type = K.args[k].type;
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

/* recognised work-item built-ins (the list in Section "Search for memory
 * accesses");
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

/* ABI entry state of slot j (Section "Search for memory accesses": s[4:5] the
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
/* table entries                                                        */
/* ------------------------------------------------------------------ */
__device__ __forceinline__ uint64_t fpt_pack(uint32_t prov, uint32_t type, uint32_t live) {
    return (uint64_t)prov | ((uint64_t)(type | live) << 32);
}
__device__ __forceinline__ uint32_t fpt_prov(uint64_t x) { return (uint32_t)x; }
__device__ __forceinline__ uint32_t fpt_type(uint64_t x) { return (uint32_t)(x >> 32) & 31u; }
__device__ __forceinline__ bool fpt_t(uint64_t x) { return ((x >> 32) & FT_T) != 0; }
__device__ __forceinline__ bool fpt_n(uint64_t x) { return ((x >> 32) & FT_N) != 0; }
/* liveness bits of a known payload */
__device__ __forceinline__ uint32_t live_bits(uint64_t v) {
    return v == VTOP ? 0u : (v_tag(v) == T_UNINIT ? FT_T : FT_T | FT_N);
}

/* the arena keeps three words per slot: provenance, payload low word, payload
 * high word with the type bits in its low byte (payload bits 39:32 are always
 * zero; TOP's high word becomes HTOP) */
__device__ __forceinline__ uint32_t pack_hi(uint64_t val, uint32_t type) {
    return ((uint32_t)(val >> 32) & 0xFFFFFF00u) | type;
}
__device__ __forceinline__ uint64_t unpack_val(uint32_t lo, uint32_t hi) {
    return hi >= HTOP ? VTOP : (((uint64_t)(hi & 0xFFFFFF00u) << 32) | lo);
}

/* IN state of a block (arena, nu_pad slots per field) -> LDS state; all
 * rows' loads are issued before the first LDS write */
__device__ __forceinline__ void state_load(WaveLds &L, const uint32_t *a, uint32_t nu_pad) {
    const uint32_t l = lane_id();
    uint32_t p[RMAX], lo[RMAX], hi[RMAX];
#pragma unroll
    for (int r = 0; r < RMAX; r++) {
        if ((uint32_t)r * 64 < nu_pad) {   /* uniform */
            const uint32_t c = (uint32_t)r * 64 + l;
            p[r] = a[c];
            lo[r] = a[nu_pad + c];
            hi[r] = a[2 * nu_pad + c];
        }
    }
#pragma unroll
    for (int r = 0; r < RMAX; r++) {
        if ((uint32_t)r * 64 < nu_pad) {
            const uint32_t c = (uint32_t)r * 64 + l;
            const uint64_t v = unpack_val(lo[r], hi[r]);
            L.fpt[c] = fpt_pack(p[r], hi[r] & 0xFFu, live_bits(v));
            L.fv[c] = v;
        }
    }
}

/* a := a join OUT for one slot per lane (provenance and type bits unite;
 * payloads that differ go to TOP), or a := OUT when first.  Only the words
 * that change are stored (the others go to the lane's scratch words), so a
 * join that changes nothing writes nothing to the arena. */
__device__ __forceinline__ bool join_slot(uint32_t *a, uint32_t nu_pad, uint32_t c, bool first, uint32_t pb, uint32_t lb,
                                          uint32_t hb, uint32_t *scr) {
    uint32_t pn = pb, ln = lb, hn = hb;
    bool cp = true, cl = true, chh = true;
    if (!first) {   /* uniform */
        const uint32_t pa = a[c], la = a[nu_pad + c], ha = a[2 * nu_pad + c];
        const bool same = la == lb && (ha & 0xFFFFFF00u) == (hb & 0xFFFFFF00u);
        pn = pa | pb;
        ln = same ? la : 0xFFFFFFFFu;
        hn = (same ? (ha & 0xFFFFFF00u) : HTOP) | ((ha | hb) & 0xFFu);
        cp = pn != pa;
        cl = ln != la;
        chh = hn != ha;
    }
    *(cp ? &a[c] : scr) = pn;
    *(cl ? &a[nu_pad + c] : scr + 1) = ln;
    *(chh ? &a[2 * nu_pad + c] : scr + 2) = hn;
    return cp || cl || chh;
}
/* OUT state into the IN states of up to two successors (null when absent);
 * returns the per-successor change bits (bit 0, bit 1) */
__device__ __forceinline__ uint32_t state_join2(const WaveLds &L, uint32_t *a0, bool first0, uint32_t *a1, bool first1,
                                                uint32_t nu_pad, uint32_t *scr) {
    const uint32_t l = lane_id();
    bool ch0 = false, ch1 = false;
#pragma unroll
    for (int r = 0; r < RMAX; r++) {
        if ((uint32_t)r * 64 < nu_pad) {   /* uniform */
            const uint32_t c = (uint32_t)r * 64 + l;
            const uint64_t x = L.fpt[c], v = L.fv[c];
            const uint32_t pb = fpt_prov(x), lb = (uint32_t)v, hb = pack_hi(v, fpt_type(x));
            if (a0) ch0 = join_slot(a0, nu_pad, c, first0, pb, lb, hb, scr) || ch0;
            if (a1) ch1 = join_slot(a1, nu_pad, c, first1, pb, lb, hb, scr) || ch1;
        }
    }
    return (ballot(ch0) != 0 ? 1u : 0u) | (ballot(ch1) != 0 ? 2u : 0u);
}

/* ------------------------------------------------------------------ */
/* staged chunk: one instruction per lane                                */
/* ------------------------------------------------------------------ */
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

__device__ __forceinline__ bool imp_covers(uint32_t idf, uint32_t s, uint32_t cv) {
    return ((idf & IM_VCC) && (s == cv || s == cv + 1)) || ((idf & IM_EXEC) && (s == cv + 2 || s == cv + 3)) ||
           ((idf & IM_SCC) && s == cv + 4);
}

/* table index of compact slot s read by this lane's instruction: the latest
 * earlier definition in the chunk, else the block state */
__device__ __forceinline__ uint32_t src_ix(const WaveLds &L, uint32_t s, uint32_t cv) {
    const uint32_t l = lane_id();
    const uint64_t m = L.dm[s < USLOT_N ? s : USLOT_N + l] & ((1ull << l) - 1ull);
    const uint32_t p = 63u - (uint32_t)__builtin_clzll(m | 1ull);
    const uint32_t lc = L.lcd[p];
    const uint32_t k = imp_covers((lc >> 16) & 7u, s, cv) ? K_IMP : s - (lc & 0x1FFu);
    return m ? IX_DEF + k * 64 + p : s;
}

/* per-lane staged instruction */
struct Ins {
    uint32_t x, y, imm;        /* record words: op | r0 << 16, r1 | r2 << 16, imm */
    uint32_t elo, ehi;         /* descriptor; a no-op for lanes past the chunk */
    uint32_t cd, ndef;         /* compact index of r0, explicit definition dwords */
    uint32_t ia, ib, ic;       /* table indices A0 | A1 << 16, B0 | B1 << 16, C0 | C1 << 16 */
    uint32_t iv, ie, isd;      /* VCC0 | VCC1 << 16, EXEC0 | EXEC1 << 16, SCC | D0 << 16 */
    uint32_t id1;              /* D1 (second dword of store data) */
    uint32_t ka0, ka1, kb0, kb1, kc0;   /* dwords of constant sources */
};

struct KCtx2 {
    KCtx K;
    uint32_t cv, dims;
};

/* ------------------------------------------------------------------ */
/* payload rule of one instruction (wave-uniform)                        */
/* ------------------------------------------------------------------ */
__device__ __forceinline__ void eval_rule(const KCtx &K, uint32_t prule, bool val_is_r1, uint64_t a0, uint64_t a1,
                                          uint64_t b0, uint64_t b1, uint64_t c0, uint64_t &v0, uint64_t &v1) {
    v0 = VTOP;
    v1 = VTOP;
    switch (prule) {
    case PR_MOV: v0 = a0; v1 = a1; break;
    case PR_ADD: v0 = r_add(a0, b0); break;
    case PR_ADDC: v0 = r_addc(a0, b0); break;
    case PR_SUB: if (is_c(a0) && is_c(b0)) v0 = C32(v_c(a0) - v_c(b0)); break;
    case PR_AND: if (is_c(a0) && is_c(b0)) v0 = C32(v_c(a0) & v_c(b0)); break;
    case PR_OR: if (is_c(a0) && is_c(b0)) v0 = C32(v_c(a0) | v_c(b0)); break;
    case PR_XOR: if (is_c(a0) && is_c(b0)) v0 = C32(v_c(a0) ^ v_c(b0)); break;
    case PR_MUL: v0 = r_mul(K, a0, b0); break;
    case PR_MUL24: v0 = r_mul(K, low24(a0), low24(b0)); break;
    case PR_MAD24: v0 = r_add(r_mul(K, low24(a0), low24(b0)), c0); break;
    case PR_SHL: v0 = val_is_r1 ? r_shl(K, a0, b0) : r_shl(K, b0, a0); break;
    case PR_LSHR: v0 = val_is_r1 ? r_lshr(K, a0, b0) : r_lshr(K, b0, a0); break;
    case PR_ASHR: v0 = val_is_r1 ? r_ashr(a0, b0) : r_ashr(b0, a0); break;
    case PR_SEL: v0 = a0 == b0 ? a0 : VTOP; break;
    case PR_AND64: case PR_OR64: case PR_XOR64: case PR_ANDN264:
        if (is_c(a0) && is_c(a1) && is_c(b0) && is_c(b1)) {
            const uint32_t x0 = v_c(a0), x1 = v_c(a1), y0 = v_c(b0), y1 = v_c(b1);
            if (prule == PR_AND64) { v0 = C32(x0 & y0); v1 = C32(x1 & y1); }
            else if (prule == PR_OR64) { v0 = C32(x0 | y0); v1 = C32(x1 | y1); }
            else if (prule == PR_XOR64) { v0 = C32(x0 ^ y0); v1 = C32(x1 ^ y1); }
            else { v0 = C32(x0 & ~y0); v1 = C32(x1 & ~y1); }
        }
        break;
    case PR_SHL64: {
        const uint64_t amt = a0, lo = b0, hi = b1;
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
}

/* the SMEM loads of the argument area (Listing 3): provenance, type and
 * payload of definition dword j (payload before the base-register check) */
__device__ __forceinline__ void smem_dword(const KCtx &K, uint32_t w, uint32_t off, uint32_t j, uint32_t &pr,
                                          uint32_t &ty, uint64_t &va) {
    pr = 1u << PB_LOADG;
    ty = 0;
    va = VTOP;
    arg_dword(K, off + 4u * j, pr, ty, va);
    if (w == 2 && (off == 0u || off == 8u || off == 16u)) {
        const uint32_t d = off >> 3;
        pr = 1u << (PB_GOFF + d);
        ty = TY_U;
        va = j == 0 ? pv(T_IDX, IG_LO, d, M_GOFF, 0, 0, 0) : pv(T_SYS, IG_HI, d, K_GOFFHI, 0, 0, 0);
    } else if (w == 1 && (off == 0xCu || off == 0x10u || off == 0x14u)) {
        const uint32_t d = (off - 0xCu) >> 2;
        pr = 1u << (PB_GSIZE + d);
        ty = TY_U;
        va = pv(T_SYS, IG_ENT, d, K_GSIZE, 0, 0, 0);
    } else if (w == 1 && off == 0x20010u) {
        pr = 1u << PB_WORKDIM;
        ty = TY_U;
        va = pv(T_SYS, IG_ENT, 0, K_WORKDIM, 0, 0, 0);
    }
}

__device__ __forceinline__ uint64_t lds_val(const WaveLds &L, uint32_t ix) {
    const uint64_t v = L.fv[ix];
    return ((uint64_t)rfl((uint32_t)(v >> 32)) << 32) | rfl((uint32_t)v);
}
/* lane 0 stores a uniform value; the other lanes store into scratch */
__device__ __forceinline__ void lds_put_u64(WaveLds &L, uint64_t *dst, uint64_t v) {
    const uint32_t l = lane_id();
    *(l == 0 ? dst : &L.junk[l]) = v;
}

/* ------------------------------------------------------------------ */
/* record output                                                        */
/* ------------------------------------------------------------------ */
struct Emit {
    uint32_t ta, ts;       /* records emitted in this visit (uniform) */
    uint32_t ab, acap;     /* the block's access-record region: first slot, capacity */
    uint32_t sb, scap;     /* its built-in-record region */
};

__device__ __forceinline__ uint32_t wave_excl_scan(uint32_t x, uint32_t &total) {
    const uint32_t l = lane_id();
    uint32_t inc = x;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(inc, d, 64);
        inc += l >= (uint32_t)d ? y : 0u;
    }
    total = __shfl(inc, 63, 64);
    return inc - x;
}

/* ------------------------------------------------------------------ */
/* one chunk                                                            */
/* ------------------------------------------------------------------ */
/* records of positions [g0, g0 + cnt) of the kernel starting at pos0, one per
 * lane (spare lanes repeat the last one) */
__device__ __forceinline__ uint4 load_chunk(const Plan *__restrict__ P, uint64_t rb, uint32_t pos0, uint32_t g0,
                                            uint32_t cnt) {
    const uint32_t l = lane_id();
    const uint32_t li = l < cnt ? l : cnt - 1;
    return reinterpret_cast<const uint4 *>(P->instrs)[rb + (g0 + li - pos0)];
}

__device__ __forceinline__ void run_chunk(const Plan *__restrict__ P, WaveLds &L, const KCtx2 &KX, uint4 r,
                                          uint32_t pos0, uint32_t g0, uint32_t cnt, Emit &E,
                                          uint4 *dummy) {
    const uint32_t l = lane_id();
    const KCtx &K = KX.K;
    const uint32_t cv = KX.cv;
    const bool act = l < cnt;
    const uint64_t bit = 1ull << l;

    /* ---- stage ---- */
    Ins I;
    const uint32_t opc = r.x & 0xFFFFu;
    const uint64_t e = act ? L.optab[opc < (uint32_t)N_OPS ? opc : 0] : (uint64_t)C_NOP;
    I.x = r.x;
    I.y = r.y;
    I.imm = r.z;
    I.elo = (uint32_t)e;
    I.ehi = (uint32_t)(e >> 32);
    const uint32_t cls = e_cls(e);
    const uint32_t r0 = r.x >> 16, r1 = r.y & 0xFFFFu, r2 = r.y >> 16;
    const int32_t imm = (int32_t)r.z;
    const uint32_t c0 = cmap(L, r0), c1 = cmap(L, r1), c2 = cmap(L, r2);
    const uint32_t role0 = e_role(e, 0);
    const uint32_t w0 = e_width(e, 0);
    const bool alu = cls == C_SALU || cls == C_SCMP || cls == C_VALU || cls == C_VCMP;
    I.cd = c0;
    I.ndef = (role0 == RO_SD || role0 == RO_VD) ? w0 : 0u;
    const uint32_t idf = alu ? e_idef(e) : 0u;
    L.lcd[l] = c0 | idf << 16;
    const uint32_t junk = USLOT_N + l;   /* def-mask scratch entry */
    const uint32_t tscr = IX_SCR + l;     /* value-table scratch entry */
#pragma unroll
    for (uint32_t j = 0; j < 4; j++) atomicOr((unsigned long long *)&L.dm[j < I.ndef ? c0 + j : junk], bit);
    atomicOr((unsigned long long *)&L.dm[(idf & IM_VCC) ? cv : junk], bit);
    atomicOr((unsigned long long *)&L.dm[(idf & IM_VCC) ? cv + 1 : junk], bit);
    atomicOr((unsigned long long *)&L.dm[(idf & IM_EXEC) ? cv + 2 : junk], bit);
    atomicOr((unsigned long long *)&L.dm[(idf & IM_EXEC) ? cv + 3 : junk], bit);
    atomicOr((unsigned long long *)&L.dm[(idf & IM_SCC) ? cv + 4 : junk], bit);
    __builtin_amdgcn_wave_barrier();

    const uint32_t w1 = e_role(e, 1) != RO_NO ? e_width(e, 1) : 0;
    const uint32_t w2 = e_role(e, 2) != RO_NO ? e_width(e, 2) : 0;
    const uint32_t w3 = e_role(e, 3) != RO_NO ? e_width(e, 3) : 0;
    const uint32_t c3 = w3 ? cmap(L, (uint32_t)imm) : CX_NONE;
    /* source roles: A0 A1 B0 B1 C0 C1 (explicit operands), V0 V1 E0 E1 S
     * (implicit vcc, exec, scc), D0 D1 (store data).  All lookups are issued
     * together: def masks first, then the producers' descriptors. */
    constexpr int NR = 13;
    const uint32_t iu = alu ? e_iuse(e) : 0u;
    const bool store = cls == C_GST || cls == C_FST || cls == C_DSW;
    uint32_t rs[NR], rk[NR];   /* compact slot (CX_NONE if none); index used when it is not a register */
    auto role = [&](int q, uint32_t c, uint32_t w, uint32_t j) {
        rs[q] = j < w && c != CX_NONE ? c + j : CX_NONE;
        rk[q] = j < w ? IX_CONST : IX_ZERO;
    };
    role(0, c1, w1, 0);
    role(1, c1, w1, 1);
    role(2, c2, w2, 0);
    role(3, c2, w2, 1);
    role(4, c3, w3, 0);
    role(5, c3, w3, 1);
#pragma unroll
    for (int q = 0; q < 5; q++) {
        const uint32_t m = q < 2 ? IM_VCC : (q < 4 ? IM_EXEC : IM_SCC);
        rs[6 + q] = (iu & m) ? cv + (uint32_t)q : CX_NONE;
        rk[6 + q] = IX_ZERO;
    }
    rs[11] = store && c0 != CX_NONE ? c0 : CX_NONE;
    rs[12] = store && c0 != CX_NONE && w0 == 2 ? c0 + 1 : CX_NONE;
    rk[11] = rk[12] = IX_ZERO;
    uint64_t dmq[NR];
    const uint64_t below = bit - 1ull;
#pragma unroll
    for (int q = 0; q < NR; q++) dmq[q] = L.dm[rs[q] != CX_NONE ? rs[q] : junk] & below;
    uint32_t lcq[NR];
#pragma unroll
    for (int q = 0; q < NR; q++) lcq[q] = L.lcd[63u - (uint32_t)__builtin_clzll(dmq[q] | 1ull)];
    uint32_t ix[NR];
#pragma unroll
    for (int q = 0; q < NR; q++) {
        const uint32_t p = 63u - (uint32_t)__builtin_clzll(dmq[q] | 1ull);
        const uint32_t k = imp_covers((lcq[q] >> 16) & 7u, rs[q], cv) ? K_IMP : rs[q] - (lcq[q] & 0x1FFu);
        ix[q] = dmq[q] ? IX_DEF + k * 64 + p : (rs[q] != CX_NONE ? rs[q] : rk[q]);
    }
    I.ia = ix[0] | ix[1] << 16;
    I.ib = ix[2] | ix[3] << 16;
    I.ic = ix[4] | ix[5] << 16;
    I.iv = ix[6] | ix[7] << 16;
    I.ie = ix[8] | ix[9] << 16;
    I.isd = ix[10] | ix[11] << 16;
    I.id1 = ix[12];
    I.ka0 = const_dword(r1, 0, w1, imm);
    I.ka1 = const_dword(r1, 1, w1, imm);
    I.kb0 = const_dword(r2, 0, w2, imm);
    I.kb1 = const_dword(r2, 1, w2, imm);
    I.kc0 = const_dword((uint32_t)imm, 0, w3, 0);

    /* static definitions: SMEM (argument area), loads; payloads start as TOP */
    const bool via = cls == C_SMEM && r1 == 4u;
#pragma unroll
    for (uint32_t k = 0; k < 5; k++) L.fv[IX_DEF + k * 64 + l] = VTOP;
#pragma unroll
    for (uint32_t k = 0; k < 4; k++) {
        uint64_t x = fpt_pack(0, 0, FT_T | FT_N);
        if (cls == C_SMEM) {
            uint32_t pr = 1u << PB_LOADG, ty = 0;
            uint64_t va = VTOP;
            if (via) smem_dword(K, w0, (uint32_t)imm, k, pr, ty, va);
            x = fpt_pack(pr, ty, via ? FT_T | FT_N : 0u);
        } else if (cls == C_GLD || cls == C_FLD || cls == C_DSR) {
            x = fpt_pack(cls == C_DSR ? 1u << PB_LOADL : 1u << PB_LOADG, 0, 0);
        }
        L.fpt[IX_DEF + k * 64 + l] = x;
    }
    L.fpt[IX_DEF + K_IMP * 64 + l] = fpt_pack(0, 0, 0);
    /* constant and absent sources */
    L.fpt[l == 0 ? IX_CONST : (l == 1 ? IX_ZERO : tscr)] =
        l == 0 ? fpt_pack(1u << PB_CONST, 0, FT_T | FT_N) : fpt_pack(0, 0, FT_T | FT_N);
    L.fv[l == 1 ? IX_ZERO : tscr] = VTOP;
    __builtin_amdgcn_wave_barrier();

    /* ---- provenance, types, liveness: passes to the solution ---- */
    const uint32_t prule = alu && I.ndef ? e_prule(e) : PR_TOP;
    const uint32_t trule = e_trule(e), suffix = e_suffix(e), vsrc = e_vsrc(e);
    const uint32_t mbit = e_maskdef(e) ? 1u << PB_MASK : 0u;
    /* Each lane's type and liveness rules as masks, so that the passes are
     * straight-line code.  Types: the union of the A and/or B source types,
     * masked, plus the suffix type (a move copies each dword's type).
     * Liveness: the result may be other than TOP (T) and other than TOP and
     * uninitialised (N) when the sources in needT carry T and those in needN
     * carry N (bits: A0 1, A1 2, B0 4, B1 8, C0 16; 32 = never); a move copies
     * its source's bits; `both` gives dword 1 the same liveness. */
    const bool tadd = trule == TR_ADD, tbu = trule == TR_B, tmove = trule == TR_MOVE;
    const bool selA = tadd || (tbu && (vsrc & 1u)), selB = tadd || (tbu && (vsrc & 2u));
    const uint32_t tmask = tadd ? TY_P : (tbu ? 31u : 0u);
    const uint32_t tsuf = (trule == TR_SUF || tadd) ? suffix : 0u;
    uint32_t needT = 32u, needN = 0u;
    bool both = false;
    switch (prule) {
    case PR_SEL: needT = 5u; break;
    case PR_ADD: case PR_ADDC: case PR_SUB: case PR_AND: case PR_OR: case PR_XOR: case PR_MUL: case PR_MUL24:
    case PR_SHL: case PR_LSHR: case PR_ASHR:
        needT = 0u; needN = 5u;
        break;
    case PR_MAD24: needT = 0u; needN = 21u; break;
    case PR_AND64: case PR_OR64: case PR_XOR64: case PR_ANDN264: needT = 0u; needN = 15u; both = true; break;
    case PR_SHL64: needT = 0u; needN = 13u; both = true; break;
    default: break;
    }
    const bool lmov = prule == PR_MOV;
    uint64_t o0 = fpt_pack(0, 0, FT_T | FT_N), o1 = o0, o4 = fpt_pack(0, 0, 0);
    for (;;) {
        const uint64_t xa0 = L.fpt[I.ia & 0xFFFFu], xa1 = L.fpt[I.ia >> 16];
        const uint64_t xb0 = L.fpt[I.ib & 0xFFFFu], xb1 = L.fpt[I.ib >> 16];
        const uint64_t xc0 = L.fpt[I.ic & 0xFFFFu], xc1 = L.fpt[I.ic >> 16];
        const uint64_t xv0 = L.fpt[I.iv & 0xFFFFu], xv1 = L.fpt[I.iv >> 16];
        const uint64_t xe0 = L.fpt[I.ie & 0xFFFFu], xe1 = L.fpt[I.ie >> 16];
        const uint64_t xs = L.fpt[I.isd & 0xFFFFu];
        const uint32_t rp = fpt_prov(xa0) | fpt_prov(xa1) | fpt_prov(xb0) | fpt_prov(xb1) | fpt_prov(xc0) |
                            fpt_prov(xc1) | fpt_prov(xv0) | fpt_prov(xv1) | fpt_prov(xe0) | fpt_prov(xe1) | fpt_prov(xs);
        const uint32_t ha0 = (uint32_t)(xa0 >> 32), ha1 = (uint32_t)(xa1 >> 32);
        const uint32_t hb0 = (uint32_t)(xb0 >> 32), hb1 = (uint32_t)(xb1 >> 32), hc0 = (uint32_t)(xc0 >> 32);
        const uint32_t ta0 = ha0 & 31u, ta1 = ha1 & 31u, tb0 = hb0 & 31u, tb1 = hb1 & 31u;
        const uint32_t un = (selA ? ta0 | ta1 : 0u) | (selB ? tb0 | tb1 : 0u);
        const uint32_t tyc = tsuf | (un & tmask);
        const uint32_t ty0 = tmove ? ta0 : tyc, ty1 = tmove ? ta1 : tyc;
        /* liveness of the payload rule's result (TOP in, TOP out) */
        const uint32_t tbits = ((ha0 & FT_T) >> 5) | ((ha1 & FT_T) >> 4) | ((hb0 & FT_T) >> 3) | ((hb1 & FT_T) >> 2) |
                               ((hc0 & FT_T) >> 1);
        const uint32_t nbits = ((ha0 & FT_N) >> 6) | ((ha1 & FT_N) >> 5) | ((hb0 & FT_N) >> 4) | ((hb1 & FT_N) >> 3) |
                               ((hc0 & FT_N) >> 2);
        const uint32_t lvx = ((tbits & needT) == needT && (nbits & needN) == needN) ? FT_T | FT_N : 0u;
        const uint32_t lv0 = lmov ? (ha0 & (FT_T | FT_N)) : lvx;
        const uint32_t lv1 = lmov ? (ha1 & (FT_T | FT_N)) : (both ? lvx : 0u);
        const uint32_t pe = rp | mbit;
        const uint64_t n0 = fpt_pack(pe, ty0, lv0), n1 = fpt_pack(pe, ty1, lv1), n4 = fpt_pack(rp | (1u << PB_MASK), 0, 0);
        L.fpt[alu && I.ndef >= 1 ? IX_DEF + l : tscr] = n0;
        L.fpt[alu && I.ndef >= 2 ? IX_DEF + 64 + l : tscr] = n1;
        L.fpt[idf ? IX_DEF + K_IMP * 64 + l : tscr] = n4;
        const bool ch = alu && (n0 != o0 || n1 != o1 || n4 != o4);
        o0 = n0;
        o1 = n1;
        o4 = n4;
        if (ballot(ch) == 0) break;
    }
    __builtin_amdgcn_wave_barrier();

    /* ---- payloads of the instructions whose result may be other than TOP ---- */
    /* Payload sources A0 A1 B0 B1 C0 of each lane: a definition of an earlier
     * lane of the chunk is read from the value table once that lane's level
     * has run; anything else (block state, constant, TOP) is gathered first
     * into sv. */
    const bool live = (alu && prule != PR_TOP && prule != PR_NONE && ((o0 >> 32) & FT_T)) ||
                      (alu && prule != PR_TOP && prule != PR_NONE && I.ndef == 2 && ((o1 >> 32) & FT_T)) || via;
    uint32_t dv0lo = 0xFFFFFFFFu, dv0hi = 0xFFFFFFFFu, dv1lo = 0xFFFFFFFFu, dv1hi = 0xFFFFFFFFu;
    if (ballot(live)) {
        const uint32_t xq[5] = {I.ia & 0xFFFFu, I.ia >> 16, I.ib & 0xFFFFu, I.ib >> 16, I.ic & 0xFFFFu};
        const uint32_t kq[5] = {I.ka0, I.ka1, I.kb0, I.kb1, I.kc0};
        uint32_t svlo[5], svhi[5], sd[5];
#pragma unroll
        for (int q = 0; q < 5; q++) {
            const uint32_t x = xq[q];
            const uint64_t v = L.fv[x < IX_DEF ? x : IX_ZERO];
            const bool def = x >= IX_DEF && x < IX_CONST;
            const uint32_t k = (x - IX_DEF) >> 6, pl = (x - IX_DEF) & 63u;
            const uint64_t sv = x == IX_CONST ? C32(kq[q]) : (x < IX_DEF ? v : VTOP);
            svlo[q] = (uint32_t)sv;
            svhi[q] = (uint32_t)(sv >> 32);
            /* source mode: 0 sv, 1 definition dword k (0 or 1, in bit 7) of lane pl, 2 table entry x */
            sd[q] = def && k < 2 ? (1u << 16) | pl | k << 7 : (def && k < 4 ? (2u << 16) | x : 0u);
        }
        /* A move whose source dwords are not definitions of this chunk
         * (block state, constant) takes its payload now, before the levels.
         * Each lane also records which sources its rule reads (bit q of the
         * mask for source q), so the levels fetch only those. */
        const uint32_t m0 = sd[0] >> 16, m1 = sd[1] >> 16;
        const bool wide = I.ndef >= 2;
        const bool mv = live && prule == PR_MOV && m0 == 0u && (!wide || m1 == 0u);
        dv0lo = mv ? svlo[0] : dv0lo;
        dv0hi = mv ? svhi[0] : dv0hi;
        dv1lo = mv && wide ? svlo[1] : dv1lo;
        dv1hi = mv && wide ? svhi[1] : dv1hi;
        const uint32_t rr = cls == C_SMEM ? PR_SMEM : prule;
        const uint32_t need = rr == PR_MOV || rr == PR_SMEM ? 0x03u
                              : rr == PR_MAD24 ? 0x15u
                              : (rr == PR_AND64 || rr == PR_OR64 || rr == PR_XOR64 || rr == PR_ANDN264) ? 0x0Fu
                              : rr == PR_SHL64 ? 0x0Du : 0x05u;
        sd[0] |= need << 18;
        const uint32_t nq = need;
        /* Levels: a lane whose rule still has to run sits one level above the
         * highest lane whose definition it reads (always an earlier lane), so
         * the lanes of one level read only results of lower levels.  The
         * levels run in order, each one lane-parallel; a result goes to the
         * lane's own entries of the value table, where the next levels read
         * it. */
        const bool ev = live && !mv;
        uint32_t lev = ev ? 1u : 0u;
        for (;;) {
            uint32_t nl = ev ? 1u : 0u;
#pragma unroll
            for (int q = 0; q < 5; q++) {
                const uint32_t d = sd[q], mode = (d >> 16) & 3u;
                const uint32_t pl = mode == 1u ? (d & 63u) : (((d & 0xFFFFu) - IX_DEF) & 63u);
                const uint32_t lp = __shfl(lev, (int)pl, 64);
                nl = (ev && ((nq >> q) & 1u) && mode != 0u) ? max(nl, lp + 1u) : nl;
            }
            const bool ch = nl != lev;
            lev = nl;
            if (ballot(ch) == 0) break;
        }
        uint32_t top = lev;
#pragma unroll
        for (int dd = 32; dd >= 1; dd >>= 1) top = max(top, (uint32_t)__shfl_xor(top, dd, 64));
        top = rfl(top);
        L.fv[IX_DEF + l] = ((uint64_t)dv0hi << 32) | dv0lo;
        L.fv[IX_DEF + 64 + l] = ((uint64_t)dv1hi << 32) | dv1lo;
        __builtin_amdgcn_wave_barrier();
        const uint64_t ei = e;
        const uint32_t wi = e_width(ei, 0);
        for (uint32_t lv = 1; lv <= top; lv++) {
            uint64_t vq[5];
#pragma unroll
            for (int q = 0; q < 5; q++) {
                const uint32_t d = sd[q], mode = (d >> 16) & 3u;
                const uint32_t x = mode == 1u ? IX_DEF + ((d >> 7) & 1u) * 64u + (d & 63u)
                                              : (mode == 2u ? (d & 0xFFFFu) : IX_ZERO);
                const uint64_t tv = L.fv[x];
                const uint64_t sv = ((uint64_t)svhi[q] << 32) | svlo[q];
                vq[q] = ((nq >> q) & 1u) ? (mode != 0u ? tv : sv) : VTOP;
            }
            if (lev == lv) {
                uint64_t v0 = VTOP, v1 = VTOP;
                if (cls == C_SMEM) {
                    const uint32_t off = I.imm;
                    const bool ok = vq[0] == pv(T_SYSPTR, IG_LO, 0, 0, 0, 0, 0) &&
                                    vq[1] == pv(T_SYSPTR, IG_HI, 0, 0, 0, 0, 0);
                    for (uint32_t j = 0; j < wi; j++) {
                        uint32_t pr, ty;
                        uint64_t va;
                        smem_dword(K, wi, off, j, pr, ty, va);
                        va = ok ? va : VTOP;
                        if (j == 0) v0 = va;
                        else if (j == 1) v1 = va;
                        else L.fv[IX_DEF + j * 64 + l] = va;
                    }
                } else {
                    eval_rule(K, e_prule(ei), e_vsrc(ei) == 1u, vq[0], vq[1], vq[2], vq[3], vq[4], v0, v1);
                }
                L.fv[IX_DEF + l] = v0;
                if (wi >= 2) L.fv[IX_DEF + 64 + l] = v1;
            }
            __builtin_amdgcn_wave_barrier();
        }
    }
    __builtin_amdgcn_wave_barrier();

    /* ---- records: accesses from the pre-state, built-ins among definitions ---- */
    {
        const bool mem = cls >= C_GLD;
        /* address dwords and store-data types, read by every lane */
        const uint32_t xa0 = I.ia & 0xFFFFu, xa1 = I.ia >> 16;
        const uint64_t lo = L.fv[xa0 < IX_CONST ? xa0 : IX_ZERO], hi = L.fv[xa1 < IX_CONST ? xa1 : IX_ZERO];
        const uint32_t tdat = fpt_type(L.fpt[I.isd >> 16]) | fpt_type(L.fpt[I.id1]);
        uint32_t kind = 0, space = 0, width = 0, dt = 0;
        uint64_t addr = VTOP;
        if (cls == C_GLD || cls == C_FLD || cls == C_GST || cls == C_FST) {
            kind = (cls == C_GLD || cls == C_FLD) ? 0 : 1;
            space = (cls == C_GLD || cls == C_GST) ? 0 : 1;
            width = 4 * w0;
            if (r2 == 0xFFFFu && (I.ia & 0xFFFFu) < IX_CONST) {
                if (lo != VTOP && hi != VTOP && v_ig(lo) == IG_LO && v_ig(hi) == IG_HI && v_arg(lo) == v_arg(hi)) {
                    if (v_tag(lo) == T_PTR && v_tag(hi) == T_PTR)
                        addr = pv(T_PTR, IG_ENT, v_dim(lo), v_aux(lo), v_sh(lo), v_arg(lo), v_c(lo) + (uint32_t)imm);
                    else if (v_tag(lo) == T_KARG && v_tag(hi) == T_KARG)
                        addr = pv(T_PTR, IG_ENT, 0, 0, 0, v_arg(lo), (uint32_t)imm);
                }
            }
        } else if (cls == C_DSR || cls == C_DSW) {
            kind = cls == C_DSR ? 0 : 1;
            space = 2;
            width = 4;
            if ((I.ia & 0xFFFFu) < IX_CONST) {
                const uint64_t v = lo;
                if (v != VTOP) {
                    const uint32_t c = v_c(v) + (uint32_t)imm;
                    if (v_tag(v) == T_SHL && v_ig(v) == IG_ENT) addr = pv(T_SHL, IG_ENT, v_dim(v), v_aux(v), v_sh(v), 0, c);
                    else if (idx_lo(v)) addr = pv(T_IDX, IG_ENT, v_dim(v), v_aux(v), 0, 0, c);
                    else if (is_c(v)) addr = C32(c);
                }
            }
        }
        if (kind == 1) {
            dt = tdat;
        } else if (mem && addr != VTOP && v_tag(addr) == T_PTR && v_arg(addr) < K.n_args) {
            dt = (v_arg(addr) < 64 ? L.argf[v_arg(addr)] : K.args[v_arg(addr)].flags) & 31u;
        }
        const uint64_t am = ballot(mem);
        if (am) {   /* wave-uniform */
            const uint32_t apos = E.ta + lanes_below(am);
            /* a region holds every record its block can emit; the bound only
             * keeps a wrong capacity from writing outside it */
            uint4 *adst = mem && apos < E.acap ? reinterpret_cast<uint4 *>(P->acc_sparse) + E.ab + apos : dummy + l;
            *adst = make_uint4(g0 + l - pos0, kind | space << 8 | width << 16 | dt << 24, (uint32_t)addr,
                               (uint32_t)(addr >> 32));
            E.ta += (uint32_t)__builtin_popcountll(am);
        }

        /* built-ins: explicit definitions not overwritten by an implicit one */
        auto sys_kind = [&](uint32_t j, uint32_t &dim) -> int {
            const uint32_t slot = r0 + j;
            const bool covered = ((idf & IM_VCC) && (slot == 104u || slot == 105u)) ||
                                 ((idf & IM_EXEC) && (slot == 106u || slot == 107u)) ||
                                 ((idf & IM_SCC) && slot == 108u);
            return j < I.ndef && !covered ? builtin_kind(L.fv[IX_DEF + j * 64 + l], dim) : -1;
        };
        uint32_t skd[4], ns = 0;   /* kind | dim << 8 of each definition dword, 0xFF none */
#pragma unroll
        for (uint32_t j = 0; j < 4; j++) {
            uint32_t dim = 0;
            const int kd = sys_kind(j, dim);
            skd[j] = kd >= 0 ? (uint32_t)kd | dim << 8 : 0xFFu;
            ns += kd >= 0 ? 1u : 0u;
        }
        if (ballot(ns != 0)) {   /* wave-uniform: most chunks define no built-in */
            uint32_t tot;
            uint32_t spos = E.ts + wave_excl_scan(ns, tot);
#pragma unroll
            for (uint32_t j = 0; j < 4; j++) {
                const bool has = skd[j] != 0xFFu;
                uint2 *sdst = has && spos < E.scap ? reinterpret_cast<uint2 *>(P->sys_sparse) + E.sb + spos
                                  : reinterpret_cast<uint2 *>(dummy + l);
                *sdst = make_uint2(g0 + l - pos0,
                                   (r0 + j) | (has ? (skd[j] & 0xFFu) : 0u) << 16 | (has ? skd[j] >> 8 : 0u) << 24);
                spos += has ? 1u : 0u;
            }
            E.ts += tot;
        }
    }
    __builtin_amdgcn_wave_barrier();

    /* ---- last definitions back to the block state; clear the def masks ---- */
    /* definition j < 4: explicit dword j; j >= 4: implicit vcc, vcc hi, exec,
     * exec hi, scc.  An explicit dword that an implicit definition of the same
     * instruction covers is written back through the implicit entry. */
    auto def_slot = [&](uint32_t j) -> uint32_t {
        if (j < 4) return j < I.ndef && !imp_covers(idf, c0 + j, cv) ? c0 + j : junk;
        const uint32_t m = j < 6 ? IM_VCC : (j < 8 ? IM_EXEC : IM_SCC);
        return (idf & m) ? cv + (j - 4) : junk;
    };
    uint64_t wx[5], wv[5];
#pragma unroll
    for (uint32_t k = 0; k < 5; k++) {
        wx[k] = L.fpt[IX_DEF + k * 64 + l];
        wv[k] = L.fv[IX_DEF + k * 64 + l];
    }
    uint64_t wm[9];
#pragma unroll
    for (uint32_t j = 0; j < 9; j++) wm[j] = L.dm[def_slot(j)];
#pragma unroll
    for (uint32_t j = 0; j < 9; j++) {
        const uint32_t s = def_slot(j);
        const bool last = s != junk && (63u - (uint32_t)__builtin_clzll(wm[j] | 1ull)) == l;
        const uint32_t dst = last ? s : tscr;
        L.fpt[dst] = wx[j < 4 ? j : K_IMP];
        L.fv[dst] = wv[j < 4 ? j : K_IMP];
    }
    __builtin_amdgcn_wave_barrier();
    /* the explicit definitions' own slots, including those an implicit
     * definition covers, leave the def masks too */
    for (uint32_t j = 0; j < 4; j++) L.dm[j < I.ndef ? c0 + j : junk] = 0;
    for (uint32_t j = 4; j < 9; j++) L.dm[def_slot(j)] = 0;
    __builtin_amdgcn_wave_barrier();
}
/* ------------------------------------------------------------------ */
/* one kernel                                                           */
/* ------------------------------------------------------------------ */
/* number the slots kernel k names (the decode stage's per-kernel bitmap)
 * plus vcc, exec, scc and the argument pointer s[4:5]; returns U */
__device__ __forceinline__ uint32_t build_compact(const Plan *__restrict__ P, WaveLds &L, uint32_t k) {
    const uint32_t l = lane_id();
    const uint32_t *ks = P->kslots + (uint64_t)k * KSLOT_WORDS;
    uint32_t base = 0;
#pragma unroll
    for (uint32_t grp = 0; grp < RMAX; grp++) {
        const uint32_t s = grp * 64 + l;
        const bool imp = (s >= 104u && s <= 108u) || s == 4u || s == 5u;
        const bool f = s < (uint32_t)NSLOT && (((ks[s >> 5] >> (s & 31u)) & 1u) != 0 || imp);
        const uint64_t m = ballot(f);
        const uint32_t c = base + lanes_below(m);
        L.umap[s] = (uint16_t)(f ? c : CX_NONE);
        L.uslot[f ? c : USLOT_N + l] = (uint16_t)s;
        base += (uint32_t)__builtin_popcountll(m);
    }
    __builtin_amdgcn_wave_barrier();
    return base;
}

/* per-wave arena and scratch */
struct WaveMem {
    uint32_t *arena;
    uint4 *dummy;
};

template <class Bits>
__device__ __forceinline__ void analyze(const Plan *__restrict__ P, uint32_t k, WaveLds &L, Bits &reached,
                                        Bits &dirty, const WaveMem &M, uint32_t nu) {
    const uint32_t l = lane_id();
    const dc_kernel_t *D = &P->kernels[k];
    const uint32_t nb = rfl(P->n_blocks[k]), fb = rfl(P->first_block[k]), nr = rfl(P->n_reach[k]);
    const uint32_t pos0 = rfl(P->pos_begin[k]);
    KCtx2 KX;
    KX.K.cws0 = rfl(D->cws[0]);
    KX.K.cws1 = rfl(D->cws[1]);
    KX.K.cws2 = rfl(D->cws[2]);
    KX.K.n_args = rfl(D->n_args);
    KX.K.args = P->args + rfl(D->arg_begin);
    const uint64_t rb = ((uint64_t)rfl((uint32_t)(D->instr_begin >> 32)) << 32) | rfl((uint32_t)D->instr_begin);
    const uint32_t dims = rfl(D->dims);
    KX.dims = dims;
    KX.cv = rfl(L.umap[104]);
    const uint32_t nu_pad = (nu + 63u) & ~63u;
    const uint32_t bs = 3 * nu_pad;   /* arena dwords per block */
    const bool keep_states = (P->flags & (DC_OPT_DIGEST | DC_OPT_EXPORT_STATES)) != 0;

    reached.init(nr);   /* both bitmaps are indexed by reverse-postorder position */
    dirty.init(nr);
    {
        const uint32_t na = KX.K.n_args;
        L.argf[l] = l < na ? KX.K.args[l < na ? l : 0].flags : 0;
    }
    for (uint32_t c0 = 0; c0 < USLOT_N + 64; c0 += 64) L.dm[c0 + l] = 0;
    /* IN[0] = the ABI entry state on the compact slots */
    for (uint32_t c0 = 0; c0 < nu_pad; c0 += 64) {
        const uint32_t c = c0 + l;
        const uint4 v = c < nu ? entry_slot(L.uslot[c], dims) : make_uint4(0, 0, 0, 0);
        M.arena[c] = v.x;
        M.arena[nu_pad + c] = v.z;
        M.arena[2 * nu_pad + c] = (v.w & 0xFFFFFF00u) | v.y;
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
        /* the block record and the IN state (arena slot = RPO position) load together */
        const uint4 *bi = P->binfo + 2 * ((uint64_t)fb + p);
        uint4 i0 = bi[0], i1 = bi[1];
        state_load(L, M.arena + (uint64_t)p * bs, nu_pad);
        /* the block, then the chain of successors whose only predecessor is the
         * block before them: their IN state is that block's OUT state, already
         * in LDS.  Running a chained block right after its predecessor instead
         * of at its own RPO position changes no pass's result: nothing between
         * the two positions feeds it or is fed by it. */
        for (;;) {
            const uint32_t b = rfl(i0.x), g_lo = rfl(i0.y), g_hi = rfl(i0.z);
            const int32_t ps0 = (int32_t)rfl(i1.x), ps1 = (int32_t)rfl(i1.y);
            const uint32_t chain = rfl(i1.z);
            const int32_t pc = chain == 0 ? ps0 : (chain == 1 ? ps1 : -1);
            /* a chained successor's IN state is stored only when states are
             * exported or digested */
            const bool join0 = ps0 >= 0 && (ps0 != pc || keep_states);
            const bool join1 = ps1 >= 0 && (ps1 != pc || keep_states);
            const bool first0 = ps0 >= 0 && !reached.get((uint32_t)(ps0 >= 0 ? ps0 : 0));
            const bool first1 = ps1 >= 0 && !reached.get((uint32_t)(ps1 >= 0 ? ps1 : 0));
            uint32_t *const a0 = join0 ? M.arena + (uint64_t)ps0 * bs : nullptr;
            uint32_t *const a1 = join1 ? M.arena + (uint64_t)ps1 * bs : nullptr;
            uint4 n0 = i0, n1 = i1;
            if (pc >= 0) {
                const uint4 *bn = P->binfo + 2 * ((uint64_t)fb + (uint32_t)pc);
                n0 = bn[0];
                n1 = bn[1];
            }
            __builtin_amdgcn_wave_barrier();
            Emit E;
            E.ta = E.ts = 0;
            E.ab = rfl(P->blk_acc_base[fb + b]);
            E.acap = rfl(P->blk_acc_base[fb + b + 1]) - E.ab;
            E.sb = rfl(P->blk_sys_base[fb + b]);
            E.scap = rfl(P->blk_sys_base[fb + b + 1]) - E.sb;
            /* records of the next chunk are in flight while a chunk runs */
            uint4 rnext = load_chunk(P, rb, pos0, g_lo, min(64u, g_hi - g_lo));
            for (uint32_t g0 = g_lo; g0 < g_hi; g0 += 64) {
                const uint4 r = rnext;
                if (g0 + 64 < g_hi) rnext = load_chunk(P, rb, pos0, g0 + 64, min(64u, g_hi - g0 - 64));
                run_chunk(P, L, KX, r, pos0, g0, min(64u, g_hi - g0), E, M.dummy);
            }
            P->blk_acc[fb + b] = min(E.ta, E.acap);
            P->blk_sys[fb + b] = min(E.ts, E.scap);
            const uint32_t chg = state_join2(L, a0, first0, a1, first1, nu_pad,
                                             reinterpret_cast<uint32_t *>(M.dummy + l));
            if (first0) reached.set((uint32_t)ps0);
            if (first1) reached.set((uint32_t)ps1);
            if ((chg & 1u) && ps0 != pc) dirty.set((uint32_t)ps0);
            if ((chg & 2u) && ps1 != pc) dirty.set((uint32_t)ps1);
            if (pc < 0) break;
            i0 = n0;
            i1 = n1;
        }
    }

    /* counts of blocks without a valid last visit are zero */
    const bool ok = status == ST_OK_FIX;
    for (uint32_t b0 = 0; b0 < nb; b0 += 64) {
        const uint32_t b = b0 + l;
        const int32_t pb = b < nb ? P->rpo_pos[fb + b] : -1;
        const bool rch = reached.get_lane(pb >= 0 ? (uint32_t)pb : 0u) && pb >= 0;   /* every lane takes part */
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
                const int32_t pb = (int32_t)rfl((uint32_t)P->rpo_pos[fb + b]);
                const bool rb_ = reached.get(pb >= 0 ? (uint32_t)pb : 0u) && pb >= 0;
                const uint32_t *a = M.arena + (uint64_t)(pb >= 0 ? pb : 0) * bs;
                uint64_t h = 0;
                for (uint32_t j0 = 0; j0 < USLOT_N; j0 += 64) {
                    const uint32_t j = j0 + l;
                    const uint32_t c = j < (uint32_t)NSLOT ? L.umap[j] : CX_NONE;
                    uint32_t prov, type;
                    uint64_t val;
                    if (c != CX_NONE) {
                        prov = a[c];
                        const uint32_t lo = a[nu_pad + c], hi = a[2 * nu_pad + c];
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

}  // namespace dc
