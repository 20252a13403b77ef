/*
 * dc_text.hip -- the text front end (Section "The body extraction"): listings
 * in the format of the paper's Listings 1-3 to kernel descriptors, 16-byte
 * records and argument tables, for many kernels at once.
 *
 * The extraction loop the paper gives walks the lines one by one: a ".kernel"
 * line opens a kernel (its second word is the name), ".config" and ".text"
 * switch between collecting configuration lines and instruction lines.  Here
 * every line is looked at by its own thread, and the loop's state at a line
 * -- the last .config or .text marker since its kernel's .kernel line -- is a
 * max-scan over the lines of that kernel.  Grammar (the paper fixes none;
 * identical to the reading documented with dc_parse_text): comments from "//"
 * or ";", blanks are space, tab and carriage return; ".dims"/"dims" x|xy|xyz;
 * ".cws" up to three integers; ".useargs"; ".arg name, "ctype", type" with
 * the six "_."-named hidden slots skipped and user arguments laid out from
 * 0x30 at their natural alignment; "NAME:" lines are labels; every other
 * line of the body is one instruction.
 *
 * Stages:
 *   k_tx_count    per 4 KiB tile of text: its line ends
 *   k_tx_scan     exclusive scans of per-tile or per-kernel counts
 *   k_tx_lines    per tile: the start of every line
 *   k_tx_classify per line: blank, .kernel, .config, .text, label, user
 *                 argument, other (after removing comment and blanks)
 *   k_tx_kcount / k_tx_klist  the .kernel lines (kernel starts)
 *   k_tx_kernel1  one workgroup per kernel: extraction state of each line,
 *                 counts of instructions, labels and user arguments
 *   k_tx_kernel2  one workgroup per kernel: labels into the kernel's hash
 *                 table, the configuration and argument table, one record
 *                 per instruction line, the descriptor
 */
#include "dc_device.h"
#include "dc_opnames.h"

namespace dc {

constexpr uint32_t TX_TILE = 4096;       /* bytes (or lines) per tile */
constexpr uint32_t TX_T = 256;           /* threads of the per-kernel workgroups */
constexpr uint32_t TX_STAGE = 16384;     /* bytes of a chunk of lines staged in LDS */
constexpr uint16_t TX_BAD = 0xFFFD, TX_NONE = 0xFFFF, TX_LIT = 0xFFFE;
enum : uint8_t { K_EMPTY, K_KERNEL, K_CONFIG, K_TEXT, K_LABEL, K_ARG, K_OTHER };

static __constant__ char OPN[N_OPS][24] = {DC_OPNAME_LIST};

/* ------------------------------------------------------------------ */
/* spans of the text                                                     */
/* ------------------------------------------------------------------ */
struct Sp {
    const uint8_t *p;
    uint32_t n;
};
__device__ __forceinline__ bool blank(uint8_t c) { return c == ' ' || c == '\t' || c == '\r'; }
__device__ __forceinline__ uint8_t lower(uint8_t c) { return (c >= 'A' && c <= 'Z') ? (uint8_t)(c - 'A' + 'a') : c; }
__device__ Sp trim(Sp s) {
    while (s.n && blank(s.p[s.n - 1])) s.n--;
    while (s.n && blank(s.p[0])) {
        s.p++;
        s.n--;
    }
    return s;
}
/* the line without its comment and surrounding blanks */
__device__ Sp clean(const uint8_t *p, uint32_t n) {
    for (uint32_t i = 0; i < n; i++)
        if (p[i] == ';' || (p[i] == '/' && i + 1 < n && p[i + 1] == '/')) {
            n = i;
            break;
        }
    return trim(Sp{p, n});
}
__device__ Sp word(Sp s, Sp *rest) {
    uint32_t i = 0;
    while (i < s.n && !blank(s.p[i])) i++;
    if (rest) *rest = trim(Sp{s.p + i, s.n - i});
    return Sp{s.p, i};
}
__device__ Sp field(Sp s, int k) {
    uint32_t a = 0;
    for (int f = 0;; f++) {
        uint32_t b = a;
        while (b < s.n && s.p[b] != ',') b++;
        if (f == k) return trim(Sp{s.p + a, b - a});
        if (b >= s.n) return Sp{s.p, 0};
        a = b + 1;
    }
}
__device__ bool eq(Sp s, const char *lit) {
    uint32_t i = 0;
    for (; lit[i]; i++)
        if (i >= s.n || s.p[i] != (uint8_t)lit[i]) return false;
    return i == s.n;
}
__device__ bool ieq(Sp s, const char *lit) {
    uint32_t i = 0;
    for (; lit[i]; i++)
        if (i >= s.n || lower(s.p[i]) != (uint8_t)lit[i]) return false;
    return i == s.n;
}
__device__ bool same(Sp a, Sp b) {
    if (a.n != b.n) return false;
    for (uint32_t i = 0; i < a.n; i++)
        if (a.p[i] != b.p[i]) return false;
    return true;
}
/* integer: optional '-', then 0x hex digits or decimal digits */
__device__ bool to_int(Sp s, int64_t *v) {
    uint32_t i = 0;
    bool neg = false;
    if (i < s.n && s.p[i] == '-') {
        neg = true;
        i++;
    }
    if (i >= s.n) return false;
    uint64_t x = 0;
    if (i + 1 < s.n && s.p[i] == '0' && (s.p[i + 1] == 'x' || s.p[i + 1] == 'X')) {
        i += 2;
        if (i >= s.n) return false;
        for (; i < s.n; i++) {
            const uint8_t c = s.p[i];
            const int d = c >= '0' && c <= '9' ? c - '0' : c >= 'a' && c <= 'f' ? c - 'a' + 10
                        : c >= 'A' && c <= 'F' ? c - 'A' + 10 : -1;
            if (d < 0 || (x >> 60)) return false;
            x = x * 16 + (uint64_t)d;
        }
    } else {
        for (; i < s.n; i++) {
            const uint8_t c = s.p[i];
            if (c < '0' || c > '9' || x > 100000000000000000ull) return false;
            x = x * 10 + (uint64_t)(c - '0');
        }
    }
    *v = neg ? -(int64_t)x : (int64_t)x;
    return true;
}
__device__ uint64_t fnv(Sp s) {
    uint64_t h = 0xcbf29ce484222325ull;
    for (uint32_t i = 0; i < s.n; i++) h = (h ^ s.p[i]) * 0x100000001b3ull;
    return h ? h : 1ull;
}

/* line j of the text (without its '\n'), cleaned; empty when the line
 * table does not describe the text (it changed after planning) */
__device__ Sp line_clean(const TextPlan &T, uint64_t j) {
    const uint64_t s = T.line_start[j], e1 = T.line_start[j + 1];
    if (e1 < s + 1 || e1 > T.n_bytes + 1) return Sp{T.text, 0};
    return clean(T.text + s, (uint32_t)(e1 - 1 - s));
}
/* line j, not cleaned, from a copy of text bytes [cs, ce) (in LDS) when the
 * line lies in it, else from the text; empty as above */
__device__ Sp line_staged(const TextPlan &T, uint64_t j, const uint8_t *stage, uint64_t cs, uint64_t ce) {
    const uint64_t s = T.line_start[j], e1 = T.line_start[j + 1];
    if (e1 < s + 1 || e1 > T.n_bytes + 1) return Sp{T.text, 0};
    if (stage && s >= cs && e1 - 1 <= ce) return Sp{stage + (s - cs), (uint32_t)(e1 - 1 - s)};
    return Sp{T.text + s, (uint32_t)(e1 - 1 - s)};
}

/* ------------------------------------------------------------------ */
/* operands and records                                                  */
/* ------------------------------------------------------------------ */
__device__ uint16_t operand(Sp t, bool *has_lit, int32_t *lit) {
    if (ieq(t, "vcc") || ieq(t, "vcc_lo")) return 104;
    if (ieq(t, "vcc_hi")) return 105;
    if (ieq(t, "exec") || ieq(t, "exec_lo")) return 106;
    if (ieq(t, "exec_hi")) return 107;
    if (ieq(t, "scc")) return 108;
    if (ieq(t, "m0")) return 109;
    if (ieq(t, "off")) return TX_NONE;
    if (t.n >= 2 && (lower(t.p[0]) == 's' || lower(t.p[0]) == 'v')) {
        const bool vec = lower(t.p[0]) == 'v';
        const int64_t lim = vec ? 255 : 103;
        int64_t a, b;
        if (t.p[1] == '[') {
            uint32_t c = 2;
            while (c < t.n && t.p[c] != ':') c++;
            if (c >= t.n || t.p[t.n - 1] != ']') return TX_BAD;
            const Sp x{t.p + 2, c - 2}, y{t.p + c + 1, t.n - c - 2};
            if (!to_int(x, &a) || !to_int(y, &b) || a < 0 || b < a || b > lim || x.p[0] == '-') return TX_BAD;
        } else {
            const Sp x{t.p + 1, t.n - 1};
            if (x.p[0] == '-' || !to_int(x, &a) || a < 0 || a > lim) return TX_BAD;
        }
        return (uint16_t)(vec ? 112 + a : a);
    }
    if (eq(t, "0.5")) return 0x8060;
    if (eq(t, "-0.5")) return 0x8061;
    if (eq(t, "1.0")) return 0x8062;
    if (eq(t, "-1.0")) return 0x8063;
    if (eq(t, "2.0")) return 0x8064;
    if (eq(t, "-2.0")) return 0x8065;
    if (eq(t, "4.0")) return 0x8066;
    if (eq(t, "-4.0")) return 0x8067;
    int64_t v;
    if (!to_int(t, &v)) return TX_BAD;
    if (v >= -16 && v <= 64) return (uint16_t)(0x8000 + (v + 16));
    *has_lit = true;
    *lit = (int32_t)(uint32_t)(uint64_t)v;
    return TX_LIT;
}

/* the kernel's label table: open addressing on the name's hash */
struct Labels {
    unsigned long long *key;
    uint32_t *idx;
    uint32_t *line;       /* line of the definition, relative to the kernel's first line */
    uint32_t cap;         /* power of two, or 0 */
    const uint8_t *text;  /* the listing and its line table (held here, not */
    const uint64_t *line_start;   /* through the kernel argument, whose address */
    uint64_t n_bytes;     /* would put a copy of it in scratch memory) */
    uint64_t l0, l1;
};
__device__ Sp label_name(const Labels &L, uint32_t rel) {
    if (L.l0 + rel >= L.l1) return Sp{L.text, 0};
    const uint64_t j = L.l0 + rel, s = L.line_start[j], e1 = L.line_start[j + 1];
    if (e1 < s + 1 || e1 > L.n_bytes + 1) return Sp{L.text, 0};
    Sp c = clean(L.text + s, (uint32_t)(e1 - 1 - s));
    if (c.n) c.n--;   /* drop the ':' */
    return c;
}
__device__ bool label_find(const Labels &L, Sp name, uint32_t *index) {
    if (!L.cap) return false;
    const uint64_t h = fnv(name);
    for (uint32_t slot = (uint32_t)h & (L.cap - 1), n = 0; n < L.cap; slot = (slot + 1) & (L.cap - 1), n++) {
        const unsigned long long k = __hip_atomic_load(&L.key[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (k == 0) return false;
        if (k == h) {
            const uint32_t rel = __hip_atomic_load(&L.line[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (!same(label_name(L, rel), name)) return false;
            *index = __hip_atomic_load(&L.idx[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return true;
        }
    }
    return false;
}

/* Mnemonic lookup: an open-addressing table of OP_TAB slots in LDS, keyed by
 * a 32-bit FNV-1a hash of the lower-case mnemonic, holding op + 1 (0 empty);
 * a hit is confirmed by comparing the names. */
constexpr uint32_t OP_TAB = 256;
__device__ __forceinline__ uint32_t op_hash(const uint8_t *p, uint32_t n) {
    uint32_t h = 2166136261u;
    for (uint32_t i = 0; i < n; i++) h = (h ^ lower(p[i])) * 16777619u;
    return h;
}
/* every thread of the group calls it; thread t inserts op t */
__device__ void op_table_build(uint32_t *tab, const char (*names)[24]) {
    const uint32_t t = threadIdx.x;
    for (uint32_t i = t; i < OP_TAB; i += blockDim.x) tab[i] = 0;
    __syncthreads();
    for (uint32_t op = t; op < (uint32_t)N_OPS; op += blockDim.x) {
        uint32_t n = 0;
        while (names[op][n]) n++;
        for (uint32_t slot = op_hash((const uint8_t *)names[op], n) & (OP_TAB - 1), m = 0; m < OP_TAB;
             slot = (slot + 1) & (OP_TAB - 1), m++)
            if (atomicCAS(&tab[slot], 0u, op + 1u) == 0u) break;
    }
    __syncthreads();
}
__device__ int find_op(Sp w, const char (*names)[24], const uint32_t *tab) {
    for (uint32_t slot = op_hash(w.p, w.n) & (OP_TAB - 1), m = 0; m < OP_TAB; slot = (slot + 1) & (OP_TAB - 1), m++) {
        const uint32_t e = tab[slot];
        if (e == 0) return -1;
        const char *nm = names[e - 1];
        uint32_t i = 0;
        for (; nm[i]; i++)
            if (i >= w.n || lower(w.p[i]) != (uint8_t)nm[i]) break;
        if (!nm[i] && i == w.n) return (int)e - 1;
    }
    return -1;
}

/* A raw line (without its '\n') as its mnemonic and the trimmed rest, in one
 * pass: the same spans as cleaning the line (cut at ';' or '//', trim) and
 * then splitting off its first word; has_comma: the rest holds a comma. */
__device__ void split_line(const uint8_t *p, uint32_t n, Sp *w, Sp *rest, bool *has_comma) {
    constexpr uint32_t NONE = 0xFFFFFFFFu;
    uint32_t st = NONE, last = 0, mend = NONE, rs = NONE, lastc = NONE;
    for (uint32_t i = 0; i < n; i++) {
        const uint8_t c = p[i];
        if (c == ';' || (c == '/' && i + 1 < n && p[i + 1] == '/')) break;
        if (!blank(c)) {
            st = st == NONE ? i : st;
            rs = (mend != NONE && rs == NONE) ? i : rs;
            last = i + 1;
            lastc = c == ',' ? i : lastc;
        } else if (st != NONE && mend == NONE) {
            mend = i;
        }
    }
    if (st == NONE) {
        *w = *rest = Sp{p, 0};
        *has_comma = false;
        return;
    }
    const uint32_t we = (mend != NONE && mend < last) ? mend : last;
    *w = Sp{p + st, we - st};
    *rest = rs != NONE ? Sp{p + rs, last - rs} : Sp{p + last, 0};
    *has_comma = rs != NONE && lastc != NONE && lastc >= rs;
}

/* one instruction line (its mnemonic and operand text) -> record */
__device__ __forceinline__ dc_instr_t parse_instr(Sp w, Sp rest, bool has_comma, const Labels &L, const char (*names)[24],
                                 const uint32_t *optab) {
    dc_instr_t r;
    r.op = TX_NONE;
    r.r0 = r.r1 = r.r2 = TX_NONE;
    r.imm = 0;
    r.target = -1;
    const int op = find_op(w, names, optab);
    if (op < 0) return r;
    r.op = (uint16_t)op;
    const uint64_t e = OPTAB[op];
    /* operand words (a comma-separated field's first word; without commas
     * every word) and modifiers (key:value words without '['; offset:N), in
     * one pass: a word is a run of characters other than blanks and commas,
     * a field ends at a comma or at the end */
    bool bad_num = false;
    int nf = 0;
    /* operand words 0..3 (no template uses more), as separate scalars: a
     * select between whole spans would put them in scratch memory */
    const uint8_t *p0 = rest.p, *p1 = rest.p, *p2 = rest.p, *p3 = rest.p;
    uint32_t n0 = 0, n1 = 0, n2 = 0, n3 = 0;
    auto put = [&](Sp v) {
        p0 = nf == 0 ? v.p : p0;
        n0 = nf == 0 ? v.n : n0;
        p1 = nf == 1 ? v.p : p1;
        n1 = nf == 1 ? v.n : n1;
        p2 = nf == 2 ? v.p : p2;
        n2 = nf == 2 ? v.n : n2;
        p3 = nf == 3 ? v.p : p3;
        n3 = nf == 3 ? v.n : n3;
    };
    bool first = true;   /* the current field has no operand word yet */
    for (uint32_t i = 0;;) {
        while (i < rest.n && blank(rest.p[i])) i++;
        if (i >= rest.n || rest.p[i] == ',') {
            if (has_comma && first) {
                put(Sp{rest.p, 0});
                nf++;
            }
            if (i >= rest.n) break;
            i++;
            first = true;
            continue;
        }
        const uint32_t a = i;
        bool colon = false, bracket = false;
        for (; i < rest.n; i++) {
            const uint8_t c = rest.p[i];
            if (blank(c) || c == ',') break;
            colon |= c == ':';
            bracket |= c == '[';
        }
        const Sp mw{rest.p + a, i - a};
        if (colon && !bracket) {
            if (mw.n > 7 && eq(Sp{mw.p, 7}, "offset:")) {
                int64_t v;
                if (to_int(Sp{mw.p + 7, mw.n - 7}, &v)) r.imm = (int32_t)(uint32_t)(uint64_t)v;
                else bad_num = true;
            }
        } else if (first || !has_comma) {
            put(mw);
            nf++;
            first = false;
        }
    }
    if (nf > 8) nf = 8;
    bool has_lit = false;
    int32_t lit = 0;
    /* which operand word goes where: 4 bits per word 0..3 (0 r0, 1 r1, 2 r2,
     * 3 imm, 15 unused); the words are parsed in order, so the last literal
     * among them is the one kept */
    const uint32_t cls = e_cls(e);
    uint32_t map = 0xFFFFu;
    switch (cls) {
    case C_SMEM: map = 0xFF10u; break;
    case C_SCMP: map = 0xFF21u; break;
    case C_VCMP: map = 0xF21Fu; break;
    case C_GLD: map = 0xF210u; break;
    case C_FLD: case C_DSR: map = 0xFF10u; break;
    case C_GST: map = 0xF201u; break;
    case C_FST: case C_DSW: map = 0xFF01u; break;
    case C_BR: case C_CBR: case C_NOP: case C_END: break;
    default:
        if (cls == C_VALU && (e_idef(e) & IM_VCC)) map = 0x21F0u;      /* dst, vcc, src0, src1 */
        else if (e_role(e, 3) != RO_NO) map = 0x3210u;                 /* dst, src0, src1, src2 */
        else if (e_role(e, 2) == RO_NO) map = 0xFF10u;                 /* dst, src */
        else map = 0xF210u;                                            /* dst, src0, src1 */
    }
    for (int k = 0; k < 4; k++) {
        const uint32_t d = (map >> (4 * k)) & 15u;
        if (d == 15u) continue;
        const Sp fk{k == 0 ? p0 : (k == 1 ? p1 : (k == 2 ? p2 : p3)), k == 0 ? n0 : (k == 1 ? n1 : (k == 2 ? n2 : n3))};
        const uint16_t v = (k < nf && fk.n) ? operand(fk, &has_lit, &lit) : TX_BAD;
        if (d == 0) r.r0 = v;
        else if (d == 1) r.r1 = v;
        else if (d == 2) r.r2 = v;
        else r.imm = (int32_t)v;
    }
    if (cls == C_SMEM) {
        int64_t v;
        if (nf > 2 && to_int(Sp{p2, n2}, &v)) r.imm = (int32_t)(uint32_t)(uint64_t)v;
        else bad_num = true;
    } else if (cls == C_BR || cls == C_CBR) {
        r.target = 0x7FFFFFFF;
        if (nf > 0) {
            uint32_t idx;
            int64_t v;
            if (label_find(L, Sp{p0, n0}, &idx)) r.target = (int32_t)idx;
            else if (to_int(Sp{p0, n0}, &v) && v >= 0 && v < 0x7FFFFFFF) r.target = (int32_t)v;
        }
    }
    if (has_lit && !e_immoff(e) && e_role(e, 3) == RO_NO) r.imm = lit;
    if (bad_num) r.op = TX_NONE;
    return r;
}

static __constant__ char TY_NAME[12][8] = {"char", "uchar", "short", "ushort", "int", "uint",
                                            "long", "ulong", "float", "double", "size_t", "void"};
static __constant__ uint8_t TY_BITS[12] = {1, 2, 1, 2, 1, 2, 1, 2, 4, 8, 2, 0};
static __constant__ uint16_t TY_SIZE[12] = {1, 1, 2, 2, 4, 4, 8, 8, 4, 8, 8, 4};

/* .arg type: size, type bits, pointee bits */
__device__ void arg_type(Sp t, uint16_t *size, uint8_t *type, uint8_t *flags) {
    bool ptr = false;
    if (t.n && t.p[t.n - 1] == '*') {
        ptr = true;
        t.n--;
        t = trim(t);
    }
    uint8_t b = 0;
    uint16_t sz = 4;
    for (int i = 0; i < 12; i++)
        if (eq(t, TY_NAME[i])) {
            b = TY_BITS[i];
            sz = TY_SIZE[i];
            break;
        }
    if (ptr) {
        *size = 8;
        *type = 16;
        *flags = b;
    } else {
        *size = sz;
        *type = b;
        *flags = 0;
    }
}

/* ------------------------------------------------------------------ */
/* block-wide scans (TX_T threads)                                       */
/* ------------------------------------------------------------------ */
__device__ uint32_t block_excl_sum(uint32_t x, uint32_t *total, uint32_t *wsum) {
    const uint32_t t = threadIdx.x, w = t >> 6, l = lane_id();
    uint32_t y = x;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t z = __shfl_up(y, d, 64);
        if (l >= (uint32_t)d) y += z;
    }
    if (l == 63) wsum[w] = y;
    __syncthreads();
    uint32_t before = 0, tot = 0;
    for (uint32_t i = 0; i < TX_T / 64; i++) {
        before += i < w ? wsum[i] : 0u;
        tot += wsum[i];
    }
    __syncthreads();
    *total = tot;
    return before + y - x;
}
__device__ uint32_t block_incl_max(uint32_t x, uint32_t *all_max, uint32_t *wsum) {
    const uint32_t t = threadIdx.x, w = t >> 6, l = lane_id();
    uint32_t y = x;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t z = __shfl_up(y, d, 64);
        if (l >= (uint32_t)d) y = max(y, z);
    }
    if (l == 63) wsum[w] = y;
    __syncthreads();
    uint32_t before = 0, tot = 0;
    for (uint32_t i = 0; i < TX_T / 64; i++) {
        before = i < w ? max(before, wsum[i]) : before;
        tot = max(tot, wsum[i]);
    }
    __syncthreads();
    *all_max = tot;
    return max(before, y);
}

/* ------------------------------------------------------------------ */
/* lines                                                                 */
/* ------------------------------------------------------------------ */
/* bit 7 of each byte of w that is a '\n' (exact: no carries between bytes) */
__device__ __forceinline__ uint32_t nl_bytes(uint32_t w) {
    const uint32_t x = w ^ 0x0A0A0A0Au;
    return ~(((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x) & 0x80808080u;
}
/* the 16 text bytes of a thread from byte t0 as four words: one 16-byte load
 * when they lie in the text and the text is 16-byte aligned, else bytes
 * (bytes past the end read as 0) */
__device__ __forceinline__ uint4 text16(const TextPlan &T, uint64_t t0) {
    if (t0 + 16 <= T.n_bytes && (reinterpret_cast<uintptr_t>(T.text) & 15u) == 0)
        return *reinterpret_cast<const uint4 *>(T.text + t0);
    uint32_t w[4] = {0, 0, 0, 0};
    for (uint32_t i = 0; i < 16; i++)
        if (t0 + i < T.n_bytes) w[i >> 2] |= (uint32_t)T.text[t0 + i] << (8 * (i & 3));
    return make_uint4(w[0], w[1], w[2], w[3]);
}

/* text bytes [cs, ce) (cs 16-byte aligned) into LDS by the workgroup: 16 bytes
 * per load when the text is aligned and the last 16-byte unit lies in it */
__device__ __forceinline__ void stage_text(const TextPlan &T, uint8_t *stage, uint64_t cs, uint64_t ce) {
    if ((reinterpret_cast<uintptr_t>(T.text) & 15u) == 0 && ((ce + 15) & ~15ull) <= T.n_bytes) {
        const uint4 *src = reinterpret_cast<const uint4 *>(T.text + cs);
        for (uint64_t q = threadIdx.x; 16 * q < ce - cs; q += blockDim.x) reinterpret_cast<uint4 *>(stage)[q] = src[q];
    } else {
        for (uint64_t i = threadIdx.x; i < ce - cs; i += blockDim.x) stage[i] = T.text[cs + i];
    }
}

__global__ __launch_bounds__(256) void k_tx_count(TextPlan T) {
    __shared__ uint32_t ws[4];
    const uint4 v = text16(T, (uint64_t)blockIdx.x * TX_TILE + (uint64_t)threadIdx.x * 16);
    const uint32_t c = __popc(nl_bytes(v.x)) + __popc(nl_bytes(v.y)) + __popc(nl_bytes(v.z)) + __popc(nl_bytes(v.w));
    uint32_t tot;
    block_excl_sum(c, &tot, ws);
    if (threadIdx.x == 0) T.tile_cnt[blockIdx.x] = tot;
}

/* exclusive scan of n counts into n + 1 offsets (one workgroup) */
__global__ __launch_bounds__(1024) void k_tx_scan(const uint32_t *in, uint64_t *out, uint64_t n) {
    const uint32_t t = threadIdx.x, w = t >> 6, l = lane_id();
    __shared__ uint64_t wsum[16], carry;
    if (t == 0) carry = 0;
    __syncthreads();
    for (uint64_t c = 0; c < n; c += 1024) {
        const uint64_t i = c + t;
        const uint64_t x = i < n ? in[i] : 0;
        uint64_t y = x;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint64_t z = __shfl_up(y, d, 64);
            if (l >= (uint32_t)d) y += z;
        }
        if (l == 63) wsum[w] = y;
        __syncthreads();
        uint64_t before = carry;
        for (uint32_t j = 0; j < w; j++) before += wsum[j];
        if (i < n) out[i] = before + y - x;
        __syncthreads();
        if (t == 1023) carry = before + y;
        __syncthreads();
    }
    if (t == 0) out[n] = carry;
}

__global__ __launch_bounds__(256) void k_tx_lines(TextPlan T) {
    __shared__ uint32_t ws[4];
    const uint64_t t0 = (uint64_t)blockIdx.x * TX_TILE + (uint64_t)threadIdx.x * 16;
    const uint4 v = text16(T, t0);
    const uint32_t m[4] = {nl_bytes(v.x), nl_bytes(v.y), nl_bytes(v.z), nl_bytes(v.w)};
    const uint32_t c = __popc(m[0]) + __popc(m[1]) + __popc(m[2]) + __popc(m[3]);
    uint32_t tot;
    const uint32_t ex = block_excl_sum(c, &tot, ws);
    uint64_t o = T.tile_off[blockIdx.x] + ex + 1;
#pragma unroll
    for (uint32_t q = 0; q < 4; q++)
        for (uint32_t b = m[q]; b; b &= b - 1) {
            const uint64_t g = t0 + 4 * q + (uint32_t)(__builtin_ctz(b) >> 3);
            if (o < T.n_lines) T.line_start[o] = g + 1;   /* more line ends than planned: flagged below */
            o++;
        }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        T.line_start[0] = 0;
        T.line_start[T.n_lines] = T.n_bytes + 1;
    }
}

/* kinds of lines; each workgroup's 256 consecutive lines are staged in LDS
 * with 16-byte loads when their text fits */
__global__ __launch_bounds__(256) void k_tx_classify(TextPlan T) {
    __shared__ __align__(16) uint8_t s_txt[TX_STAGE];
    for (uint64_t c0 = (uint64_t)blockIdx.x * 256; c0 < T.n_lines; c0 += (uint64_t)gridDim.x * 256) {
        const uint64_t j = c0 + threadIdx.x;
        const uint64_t cend = c0 + 256 < T.n_lines ? c0 + 256 : T.n_lines;
        const uint64_t cs = T.line_start[c0] & ~15ull;
        uint64_t ce = T.line_start[cend];
        if (ce > T.n_bytes) ce = T.n_bytes;
        const bool staged = ce >= cs && ce - cs <= TX_STAGE;
        __syncthreads();   /* the previous chunk's lines are done */
        if (staged) stage_text(T, s_txt, cs, ce);
        __syncthreads();
        if (j >= T.n_lines) continue;
        const Sp raw = line_staged(T, j, staged ? s_txt : nullptr, cs, ce);
        const Sp c = clean(raw.p, raw.n);
        uint8_t kd = K_EMPTY;
        if (c.n) {
            Sp rest;
            const Sp w = word(c, &rest);
            if (eq(w, ".kernel")) kd = K_KERNEL;
            else if (eq(c, ".config")) kd = K_CONFIG;
            else if (eq(c, ".text")) kd = K_TEXT;
            else if (c.p[c.n - 1] == ':' && rest.n == 0) kd = K_LABEL;
            else if (eq(w, ".arg")) {
                const Sp nm = field(rest, 0);
                kd = (nm.n >= 2 && nm.p[0] == '_' && nm.p[1] == '.') ? K_OTHER : K_ARG;
            } else kd = K_OTHER;
        }
        T.kind[j] = kd;
    }
}

/* .kernel lines: count per tile of lines, then their indices */
__global__ __launch_bounds__(256) void k_tx_kcount(TextPlan T) {
    __shared__ uint32_t ws[4];
    const uint64_t t0 = (uint64_t)blockIdx.x * TX_TILE;
    uint32_t c = 0;
    for (uint32_t i = threadIdx.x; i < TX_TILE; i += 256) {
        const uint64_t j = t0 + i;
        c += (j < T.n_lines && T.kind[j] == K_KERNEL) ? 1u : 0u;
    }
    uint32_t tot;
    block_excl_sum(c, &tot, ws);
    if (threadIdx.x == 0) T.ltile_cnt[blockIdx.x] = tot;
}
__global__ __launch_bounds__(256) void k_tx_klist(TextPlan T) {
    __shared__ uint32_t ws[4];
    const uint64_t t0 = (uint64_t)blockIdx.x * TX_TILE + (uint64_t)threadIdx.x * 16;
    uint32_t c = 0;
    for (uint32_t i = 0; i < 16; i++) {
        const uint64_t j = t0 + i;
        c += (j < T.n_lines && T.kind[j] == K_KERNEL) ? 1u : 0u;
    }
    uint32_t tot;
    const uint32_t ex = block_excl_sum(c, &tot, ws);
    uint64_t o = T.ltile_off[blockIdx.x] + ex;
    for (uint32_t i = 0; i < 16; i++) {
        const uint64_t j = t0 + i;
        if (j < T.n_lines && T.kind[j] == K_KERNEL) {
            if (o < T.k_cap) T.kline[o] = j;
            o++;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && T.n_kernels <= T.k_cap) T.kline[T.n_kernels] = T.n_lines;
}

/* the text has the line and kernel counts it was planned for (else every
 * later stage stops and the run reports DC_E_CAPACITY) */
__global__ void k_tx_check(TextPlan T) {
    if (threadIdx.x == 0 && (T.tile_off[T.n_tiles] + 1 != T.n_lines || T.ltile_off[T.n_ltiles] != T.n_kernels))
        atomicOr(T.fail, 1u);
}

/* the extraction state of a chunk of a kernel's lines: 1 config, 2 text,
 * 0 before either (marker = (relative line + 1) << 2 | state) */
__device__ uint32_t chunk_state(uint8_t kd, uint32_t rel, uint32_t *carry, uint32_t *ws) {
    const uint32_t m = kd == K_CONFIG ? ((rel + 1) << 2 | 1u) : kd == K_TEXT ? ((rel + 1) << 2 | 2u) : 0u;
    uint32_t all;
    const uint32_t mm = block_incl_max(m, &all, ws);
    const uint32_t st = mm ? (mm & 3u) : *carry;
    __syncthreads();
    if (all) *carry = all & 3u;
    return st;
}

__global__ __launch_bounds__(TX_T) void k_tx_kernel1(TextPlan T) {
    __shared__ uint32_t ws[4];
    const uint32_t k = blockIdx.x, K = T.n_kernels;
    if (k >= K || K > T.k_cap || *T.fail) return;
    const uint64_t l0 = T.kline[k] + 1, l1 = T.kline[k + 1];
    uint32_t carry = 0, ni = 0, nl = 0, na = 0;
    for (uint64_t c = l0; c < l1; c += TX_T) {
        const uint64_t j = c + threadIdx.x;
        const bool act = j < l1;
        const uint8_t kd = act ? T.kind[j] : K_EMPTY;
        const uint32_t st = chunk_state(kd, (uint32_t)(j - l0), &carry, ws);
        const uint32_t is_i = act && st == 2 && (kd == K_OTHER || kd == K_ARG);
        const uint32_t is_l = act && st == 2 && kd == K_LABEL;
        const uint32_t is_a = act && st == 1 && kd == K_ARG;
        uint32_t a, b, d;
        block_excl_sum(is_i, &a, ws);
        block_excl_sum(is_l, &b, ws);
        block_excl_sum(is_a, &d, ws);
        ni += a;
        nl += b;
        na += d;
    }
    if (threadIdx.x == 0) {
        T.kcounts[k] = ni;
        uint32_t cap = 0;
        if (nl) {
            cap = 2;
            while (cap < 2 * nl) cap <<= 1;
        }
        T.kcounts[(uint64_t)K + k] = cap;
        T.kcounts[2ull * K + k] = na;
    }
}

/* at least four waves per SIMD: the parser's registers are capped at 128 */
__global__ __launch_bounds__(TX_T, 4) void k_tx_kernel2(TextPlan T) {
    __shared__ uint32_t ws[4];
    __shared__ char names[N_OPS][24];
    __shared__ uint32_t s_optab[OP_TAB];
    __shared__ uint32_t s_dims, s_cws, s_use;
    __shared__ __align__(16) uint8_t s_txt[TX_STAGE];
    const uint32_t k = blockIdx.x, K = T.n_kernels, t = threadIdx.x;
    if (k >= K || K > T.k_cap || *T.fail) return;
    for (uint32_t i = t; i < N_OPS * 24; i += TX_T) (&names[0][0])[i] = (&OPN[0][0])[i];
    __syncthreads();
    op_table_build(s_optab, names);
    if (t == 0) {
        s_dims = s_cws = s_use = 0;
    }
    const uint64_t l0 = T.kline[k] + 1, l1 = T.kline[k + 1];
    const uint64_t ib = T.koffs[k], lb = T.koffs[(uint64_t)(K + 1) + k], ab = T.koffs[2ull * (K + 1) + k];
    const uint32_t ni = T.kcounts[k], cap = T.kcounts[(uint64_t)K + k], na = T.kcounts[2ull * K + k];
    const bool fits = ib + ni <= T.instr_cap && lb + cap <= T.lab_cap && ab + na <= T.arg_cap;
    if (!fits) {
        if (t == 0) atomicOr(T.fail, 1u);
        return;
    }
    Labels L{T.lab_key + lb, T.lab_idx + lb, T.lab_line + lb, cap, T.text, T.line_start, T.n_bytes, l0, l1};
    __syncthreads();
    /* labels, configuration lines, argument order */
    uint32_t carry = 0, icount = 0, acount = 0;
    for (uint64_t c = l0; c < l1; c += TX_T) {
        const uint64_t j = c + t;
        const bool act = j < l1;
        const uint8_t kd = act ? T.kind[j] : K_EMPTY;
        const uint32_t rel = (uint32_t)(j - l0);
        const uint32_t st = chunk_state(kd, rel, &carry, ws);
        const uint32_t is_i = act && st == 2 && (kd == K_OTHER || kd == K_ARG);
        const uint32_t is_a = act && st == 1 && kd == K_ARG;
        uint32_t ti, ta;
        const uint32_t xi = block_excl_sum(is_i, &ti, ws);
        const uint32_t xa = block_excl_sum(is_a, &ta, ws);
        if (act && st == 2 && kd == K_LABEL) {
            const Sp nm = label_name(L, rel);
            const uint64_t h = fnv(nm);
            for (uint32_t slot = (uint32_t)h & (cap - 1), n = 0; n < cap; slot = (slot + 1) & (cap - 1), n++) {
                const unsigned long long old = atomicCAS(&L.key[slot], 0ull, (unsigned long long)h);
                if (old == 0 || old == h) {
                    atomicMin(&L.idx[slot], icount + xi);
                    atomicMin(&L.line[slot], rel);
                    break;
                }
            }
        }
        if (act && st == 1 && kd == K_OTHER) {
            const Sp w = word(line_clean(T, j), nullptr);
            if (eq(w, ".dims") || eq(w, "dims")) atomicMax(&s_dims, rel + 1);
            else if (eq(w, ".cws")) atomicMax(&s_cws, rel + 1);
            else if (eq(w, ".useargs")) atomicOr(&s_use, 1u);
        }
        if (is_a && acount + xa < na) T.args[ab + acount + xa].offset = rel;   /* the line, until the layout pass */
        icount += ti;
        acount += ta;
    }
    __threadfence();
    __syncthreads();
    /* records: each chunk's text is staged in LDS with coalesced loads when
     * it fits, and its lines are parsed from there */
    carry = 0;
    icount = 0;
    for (uint64_t c = l0; c < l1; c += TX_T) {
        const uint64_t j = c + t;
        const bool act = j < l1;
        const uint8_t kd = act ? T.kind[j] : K_EMPTY;
        const uint32_t st = chunk_state(kd, (uint32_t)(j - l0), &carry, ws);
        const uint32_t is_i = act && st == 2 && (kd == K_OTHER || kd == K_ARG);
        uint32_t ti;
        const uint32_t xi = block_excl_sum(is_i, &ti, ws);
        const uint64_t cend = c + TX_T < l1 ? c + TX_T : l1;
        const uint64_t cs = T.line_start[c] & ~15ull;   /* 16-byte aligned start of the chunk's text */
        uint64_t ce = T.line_start[cend];
        if (ce > T.n_bytes) ce = T.n_bytes;
        const bool staged = ce >= cs && ce - cs <= TX_STAGE;
        if (staged) stage_text(T, s_txt, cs, ce);
        __syncthreads();
        if (is_i && icount + xi < ni) {
            const Sp ln = line_staged(T, j, staged ? s_txt : nullptr, cs, ce);
            Sp w, rest;
            bool has_comma;
            split_line(ln.p, ln.n, &w, &rest, &has_comma);
            T.instrs[ib + icount + xi] = parse_instr(w, rest, has_comma, L, names, s_optab);
        }
        __syncthreads();
        icount += ti;
    }
    __syncthreads();
    if (t != 0) return;
    /* configuration, argument layout, descriptor, name (one thread) */
    dc_kernel_t D;
    D.instr_begin = ib;
    D.n_instr = ni;
    D.dims = 0;
    D.useargs = (uint8_t)s_use;
    D.n_args = (uint16_t)na;
    D.cws[0] = D.cws[1] = D.cws[2] = 0;
    D.arg_begin = (uint32_t)ab;
    auto line_at = [&](uint32_t rel) { return l0 + rel < l1 ? line_clean(T, l0 + rel) : Sp{T.text, 0}; };
    if (s_dims) {
        Sp rest;
        word(line_at(s_dims - 1), &rest);
        const Sp d = word(rest, nullptr);
        D.dims = eq(d, "x") ? 1 : eq(d, "xy") ? 2 : eq(d, "xyz") ? 3 : 0;
    }
    if (s_cws) {
        Sp rest;
        word(line_at(s_cws - 1), &rest);
        for (int d = 0; d < 3; d++) {
            const Sp v = field(rest, d);
            int64_t x;
            D.cws[d] = v.n == 0 ? 1u : (to_int(v, &x) && x >= 0 && x <= 0xFFFFFFFFll ? (uint32_t)x : 0u);
        }
    }
    uint32_t cursor = 0x30;
    for (uint32_t a = 0; a < na; a++) {
        dc_arg_t *A = &T.args[ab + a];
        Sp rest;
        word(line_at(A->offset), &rest);
        dc_arg_t out;
        arg_type(field(rest, 2), &out.size, &out.type, &out.flags);
        cursor = (cursor + out.size - 1) / out.size * out.size;
        out.offset = cursor;
        cursor += out.size;
        *A = out;
    }
    T.kernels[k] = D;
    {
        Sp rest;
        word(line_clean(T, l0 - 1), &rest);
        const Sp nm = word(rest, nullptr);
        T.name_off[k] = (uint64_t)(nm.p - T.text);
        T.name_len[k] = nm.n;
    }
}

/* ------------------------------------------------------------------ */
/* launchers                                                             */
/* ------------------------------------------------------------------ */
static uint32_t tx_grid(uint64_t n) {
    const uint64_t g = (n + 255) / 256;
    return g < 1 ? 1u : g > (1u << 20) ? (1u << 20) : (uint32_t)g;
}

hipError_t launch_text_lines(const TextPlan &T, hipStream_t s) {
    hipLaunchKernelGGL(k_tx_count, dim3(T.n_tiles), dim3(256), 0, s, T);
    hipLaunchKernelGGL(k_tx_scan, dim3(1), dim3(1024), 0, s, T.tile_cnt, T.tile_off, (uint64_t)T.n_tiles);
    return hipGetLastError();
}
hipError_t launch_text_classify(const TextPlan &T, hipStream_t s) {
    hipLaunchKernelGGL(k_tx_lines, dim3(T.n_tiles), dim3(256), 0, s, T);
    hipLaunchKernelGGL(k_tx_classify, dim3(tx_grid(T.n_lines)), dim3(256), 0, s, T);
    hipLaunchKernelGGL(k_tx_kcount, dim3(T.n_ltiles), dim3(256), 0, s, T);
    hipLaunchKernelGGL(k_tx_scan, dim3(1), dim3(1024), 0, s, T.ltile_cnt, T.ltile_off, (uint64_t)T.n_ltiles);
    return hipGetLastError();
}
hipError_t launch_text_kernels1(const TextPlan &T, hipStream_t s) {
    hipLaunchKernelGGL(k_tx_check, dim3(1), dim3(64), 0, s, T);
    hipLaunchKernelGGL(k_tx_klist, dim3(T.n_ltiles), dim3(256), 0, s, T);
    if (T.n_kernels) {
        hipLaunchKernelGGL(k_tx_kernel1, dim3(T.n_kernels), dim3(TX_T), 0, s, T);
        for (int a = 0; a < 3; a++)
            hipLaunchKernelGGL(k_tx_scan, dim3(1), dim3(1024), 0, s, T.kcounts + (uint64_t)a * T.n_kernels,
                               T.koffs + (uint64_t)a * (T.n_kernels + 1), (uint64_t)T.n_kernels);
    }
    return hipGetLastError();
}
hipError_t launch_text_kernels2(const TextPlan &T, hipStream_t s) {
    if (!T.n_kernels) return hipSuccess;
    hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t *>(T.lab_key), 2 * T.lab_cap, 0u, s);
    if (e == hipSuccess) e = launch_fill_u32(T.lab_idx, T.lab_cap, 0xFFFFFFFFu, s);
    if (e == hipSuccess) e = launch_fill_u32(T.lab_line, T.lab_cap, 0xFFFFFFFFu, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_tx_kernel2, dim3(T.n_kernels), dim3(TX_T), 0, s, T);
    return hipGetLastError();
}

}  // namespace dc
