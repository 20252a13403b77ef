/*
 * dcgen.c -- seeded synthetic GCN kernel generator.
 *
 * Input synthesis only: this file knows the 16-byte record encoding and a
 * grammar of plausible compiler output, and nothing of the analysis.  It is
 * shared by the CPU oracle's tests and by the GPU path's tests and bench.
 *
 * Grammar (modelled on what the paper says compiled OpenCL kernels contain):
 *   - prologue: kernel-argument loads through s[4:5] (get_global_offset at
 *     0x0, Section "Search for memory accesses"; user arguments after the six
 *     hidden 8-byte slots of the Listing 3 layout), an optional get_global_size
 *     load (offset 0xc), and the global-id idiom
 *       s_mul_i32 s0, s6, cws0 ; v_add_co_u32 v1, vcc, s0, v0 ;
 *       v_add_co_u32 v1, vcc, s2, v1
 *     (work-group id times work-group size plus local id plus offset);
 *   - body: scalar/vector integer ALU, float ALU, array-element address
 *     idioms feeding global loads/stores, LDS traffic, exec-mask if/else
 *     diamonds (two exit shapes) and scalar counted loops;
 *   - s_endpgm.
 * Every kernel has exactly the sampled length.  Kernel i of config c draws
 * all of its randomness from splitmix64 (Steele, Lea & Flood, 2014) seeded
 * with 0xD1C00000 + (c << 32) + i, so any kernel can be regenerated alone.
 */
#include <math.h>
#include <pthread.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct { uint16_t op, r0, r1, r2; int32_t imm, target; } gen_instr;   /* 16 B */
typedef struct {
    uint64_t instr_begin; uint32_t n_instr; uint8_t dims, useargs; uint16_t n_args;
    uint32_t cws[3]; uint32_t arg_begin;
} gen_kernel;                                                                   /* 32 B */
typedef struct { uint32_t offset; uint16_t size; uint8_t type, flags; } gen_arg; /* 8 B */

_Static_assert(sizeof(gen_instr) == 16, "record");
_Static_assert(sizeof(gen_kernel) == 32, "descriptor");
_Static_assert(sizeof(gen_arg) == 8, "arg");

/* ---- the record encoding: opcode numbering (dense, in this order) ---- */
static const char *const OP_NAMES[] = {
    "s_load_dword", "s_load_dwordx2", "s_load_dwordx4", "s_mov_b32", "s_mov_b64",
    "s_and_saveexec_b64", "s_or_saveexec_b64", "s_add_u32", "s_add_i32", "s_addc_u32",
    "s_sub_u32", "s_mul_i32", "s_lshl_b32", "s_lshr_b32", "s_and_b32",
    "s_or_b32", "s_and_b64", "s_or_b64", "s_xor_b64", "s_andn2_b64",
    "s_cmp_eq_u32", "s_cmp_lt_u32", "s_cmp_gt_u32", "s_cmp_lt_i32", "s_branch",
    "s_cbranch_scc0", "s_cbranch_scc1", "s_cbranch_vccz", "s_cbranch_vccnz", "s_cbranch_execz",
    "s_cbranch_execnz", "s_waitcnt", "s_barrier", "s_nop", "s_endpgm",
    "v_mov_b32", "v_cvt_f32_u32", "v_cvt_u32_f32", "v_cvt_f64_f32", "v_add_co_u32",
    "v_addc_co_u32", "v_sub_co_u32", "v_add_u32", "v_mul_lo_u32", "v_mul_u32_u24",
    "v_mul_hi_u32", "v_mad_u32_u24", "v_lshlrev_b32", "v_lshrrev_b32", "v_ashrrev_i32",
    "v_and_b32", "v_or_b32", "v_xor_b32", "v_lshlrev_b64", "v_cndmask_b32",
    "v_add_f32", "v_sub_f32", "v_mul_f32", "v_max_f32", "v_mad_f32",
    "v_fma_f32", "v_add_f64", "v_mul_f64", "v_fma_f64", "v_cmp_eq_u32",
    "v_cmp_gt_u32", "v_cmp_lt_u32", "v_cmp_lt_i32", "v_cmp_gt_f32", "global_load_dword",
    "global_load_dwordx2", "flat_load_dword", "global_store_dword", "global_store_dwordx2", "flat_store_dword",
    "ds_read_b32", "ds_write_b32",
};
enum {
    S_LOAD_DWORD, S_LOAD_DWORDX2, S_LOAD_DWORDX4, S_MOV_B32, S_MOV_B64,
    S_AND_SAVEEXEC_B64, S_OR_SAVEEXEC_B64, S_ADD_U32, S_ADD_I32, S_ADDC_U32,
    S_SUB_U32, S_MUL_I32, S_LSHL_B32, S_LSHR_B32, S_AND_B32,
    S_OR_B32, S_AND_B64, S_OR_B64, S_XOR_B64, S_ANDN2_B64,
    S_CMP_EQ_U32, S_CMP_LT_U32, S_CMP_GT_U32, S_CMP_LT_I32, S_BRANCH,
    S_CBRANCH_SCC0, S_CBRANCH_SCC1, S_CBRANCH_VCCZ, S_CBRANCH_VCCNZ, S_CBRANCH_EXECZ,
    S_CBRANCH_EXECNZ, S_WAITCNT, S_BARRIER, S_NOP, S_ENDPGM,
    V_MOV_B32, V_CVT_F32_U32, V_CVT_U32_F32, V_CVT_F64_F32, V_ADD_CO_U32,
    V_ADDC_CO_U32, V_SUB_CO_U32, V_ADD_U32, V_MUL_LO_U32, V_MUL_U32_U24,
    V_MUL_HI_U32, V_MAD_U32_U24, V_LSHLREV_B32, V_LSHRREV_B32, V_ASHRREV_I32,
    V_AND_B32, V_OR_B32, V_XOR_B32, V_LSHLREV_B64, V_CNDMASK_B32,
    V_ADD_F32, V_SUB_F32, V_MUL_F32, V_MAX_F32, V_MAD_F32,
    V_FMA_F32, V_ADD_F64, V_MUL_F64, V_FMA_F64, V_CMP_EQ_U32,
    V_CMP_GT_U32, V_CMP_LT_U32, V_CMP_LT_I32, V_CMP_GT_F32, GLOBAL_LOAD_DWORD,
    GLOBAL_LOAD_DWORDX2, FLAT_LOAD_DWORD, GLOBAL_STORE_DWORD, GLOBAL_STORE_DWORDX2, FLAT_STORE_DWORD,
    DS_READ_B32, DS_WRITE_B32, N_OPS
};
_Static_assert(sizeof(OP_NAMES) / sizeof(OP_NAMES[0]) == N_OPS, "op names");

/* operand ids: 0..103 s, 104/105 vcc, 106/107 exec, 108 scc, 109 m0,
 * 112..367 v0..v255, 0x8000+k inline int k-16 (k<=80), 0x8060.. inline
 * floats, 0xFFFE literal (value in imm), 0xFFFF none */
#define SG(n) ((uint16_t)(n))
#define VG(n) ((uint16_t)(112 + (n)))
#define VCC 104
#define EXEC 106
#define ICONST(v) ((uint16_t)(0x8000 + ((v) + 16)))
#define FCONST(k) ((uint16_t)(0x8060 + (k)))
#define LIT 0xFFFE
#define NONE 0xFFFF

/* type-tier bits carried in the argument table */
#define T_INT 1
#define T_UINT 2
#define T_FLOAT 4
#define T_DOUBLE 8
#define T_PTR 16

/* ---- splitmix64 ---- */
static inline uint64_t sm64(uint64_t *s) {
    uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
static inline double u01(uint64_t *s) { return (double)(sm64(s) >> 11) * (1.0 / 9007199254740992.0); }
static inline uint32_t below(uint64_t *s, uint32_t n) { return n ? (uint32_t)(((sm64(s) >> 32) * (uint64_t)n) >> 32) : 0; }
static inline int chance(uint64_t *s, double p) { return u01(s) < p; }

/* ---- Zipf(s=1.2) on [20, 20000]: inverse CDF over the integer support ---- */
#define ZMIN 20
#define ZMAX 20000
static double *zipf_cdf;
static pthread_once_t zipf_once = PTHREAD_ONCE_INIT;
static void zipf_init(void) {
    int n = ZMAX - ZMIN + 1;
    double *c = (double *)malloc(sizeof(double) * n), acc = 0;
    for (int i = 0; i < n; i++) { acc += pow((double)(ZMIN + i), -1.2); c[i] = acc; }
    for (int i = 0; i < n; i++) c[i] /= acc;
    zipf_cdf = c;
}
static uint32_t zipf_len(uint64_t *s) {
    pthread_once(&zipf_once, zipf_init);
    double u = u01(s);
    int lo = 0, hi = ZMAX - ZMIN;
    while (lo < hi) { int m = (lo + hi) / 2; if (zipf_cdf[m] < u) lo = m + 1; else hi = m; }
    return (uint32_t)(ZMIN + lo);
}

/* ---- per-kernel header: everything decided before the body ---- */
typedef struct {
    uint64_t rng;
    uint32_t len;
    int dims, full_range, has_int_arg, has_gsize, shift_form;
    uint32_t cws[3];
    uint8_t pointee[2];
} header;

static uint64_t kernel_seed(int cfg, uint64_t index) {
    return 0xD1C00000ull + ((uint64_t)cfg << 32) + index;
}

static void make_header(int cfg, uint64_t index, header *h) {
    memset(h, 0, sizeof(*h));
    h->rng = kernel_seed(cfg, index);
    uint64_t *r = &h->rng;
    switch (cfg) {
    case 1: h->len = 50 + below(r, 251); break;
    case 2: h->len = (uint32_t)floor(200.0 * pow(10.0, u01(r))); if (h->len > 2000) h->len = 2000; break;
    case 3: h->len = zipf_len(r); break;
    case 4: h->len = 1000000 + below(r, 3000001); break;
    case 5: {
        double u1 = u01(r), u2 = u01(r);
        if (u1 < 1e-300) u1 = 1e-300;
        double z = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
        double l = floor(exp(log(1000.0) + z));
        if (l < 20) l = 20;
        if (l > 100000) l = 100000;
        h->len = (uint32_t)l;
        break;
    }
    case 6: h->len = 6000 + below(r, 6001); break;   /* dense control flow (test shape) */
    default: h->len = 64; break;
    }
    h->dims = 1 + (int)below(r, 3);
    static const uint32_t cw0[3] = {64, 128, 256};
    h->cws[0] = cw0[below(r, 3)];
    h->cws[1] = h->dims >= 2 ? (uint32_t)(1u << below(r, 3)) : 1;
    h->cws[2] = h->dims >= 3 ? 1 : 1;
    h->full_range = (cfg == 2) ? (index % 10 == 0) : chance(r, 0.1);
    h->has_int_arg = chance(r, 0.5);
    h->has_gsize = chance(r, 0.2);
    h->shift_form = chance(r, 0.3);
    h->pointee[0] = chance(r, 0.5) ? T_FLOAT : T_INT;
    h->pointee[1] = chance(r, 0.5) ? T_FLOAT : T_UINT;
}

/* ---- body generation ---- */
typedef struct {
    header h;
    int cfg;
    gen_instr *out;
    uint32_t n;
    int s_lo, s_hi, v_lo, v_hi;       /* random-def pools */
    uint16_t vrec[8], srec[8];        /* recent definitions */
    int nvrec, nsrec;
    int loop_depth_max, if_depth_max;
    double p_struct;
} G;

static void emit(G *g, uint16_t op, uint16_t r0, uint16_t r1, uint16_t r2, int32_t imm) {
    gen_instr *x = &g->out[g->n++];
    x->op = op; x->r0 = r0; x->r1 = r1; x->r2 = r2; x->imm = imm; x->target = -1;
}
static uint32_t emit_branch(G *g, uint16_t op) {
    gen_instr *x = &g->out[g->n];
    x->op = op; x->r0 = x->r1 = x->r2 = NONE; x->imm = 0; x->target = -1;
    return g->n++;
}

static void note_v(G *g, uint16_t r) { g->vrec[g->nvrec++ & 7] = r; }
static void note_s(G *g, uint16_t r) { g->srec[g->nsrec++ & 7] = r; }

static uint16_t pick_vdst(G *g) { return VG(g->v_lo + (int)below(&g->h.rng, (uint32_t)(g->v_hi - g->v_lo + 1))); }
static uint16_t pick_sdst(G *g) { return SG(g->s_lo + (int)below(&g->h.rng, (uint32_t)(g->s_hi - g->s_lo + 1))); }

static uint16_t pick_const(G *g, int32_t *lit) {
    uint64_t *r = &g->h.rng;
    if (chance(r, 0.05)) { *lit = (int32_t)(sm64(r) & 0xFFFF) - 4096; return LIT; }
    return ICONST(-16 + (int)below(r, 81));
}

/* a vector-ALU source: recent def, pool register, special id value, or constant */
static uint16_t pick_vsrc(G *g, int32_t *lit, int allow_const) {
    uint64_t *r = &g->h.rng;
    if (g->nvrec && chance(r, 0.7)) return g->vrec[below(r, g->nvrec < 8 ? (uint32_t)g->nvrec : 8u)];
    double u = u01(r);
    if (allow_const && u < 0.2) return pick_const(g, lit);
    if (u < 0.3) return VG(below(r, (uint32_t)g->h.dims));   /* local id */
    if (u < 0.35) return VG(1);                                /* global id */
    if (u < 0.45) return SG(below(r, 2) ? 6 : 0);              /* group id / group base */
    return pick_vdst(g);
}
/* a vector register only (store data must live in a VGPR) */
static uint16_t pick_vreg(G *g) {
    uint64_t *r = &g->h.rng;
    if (g->nvrec && chance(r, 0.7)) return g->vrec[below(r, g->nvrec < 8 ? (uint32_t)g->nvrec : 8u)];
    return chance(r, 0.2) ? VG(1) : pick_vdst(g);
}
static uint16_t pick_ssrc(G *g, int32_t *lit, int allow_const) {
    uint64_t *r = &g->h.rng;
    if (g->nsrec && chance(r, 0.7)) return g->srec[below(r, g->nsrec < 8 ? (uint32_t)g->nsrec : 8u)];
    double u = u01(r);
    if (allow_const && u < 0.3) return pick_const(g, lit);
    if (u < 0.4) return SG(6 + below(r, (uint32_t)g->h.dims));
    if (u < 0.45 && g->h.has_int_arg) return SG(16);
    if (u < 0.5 && g->h.has_gsize) return SG(17);
    return pick_sdst(g);
}

static void scalar_alu(G *g) {
    static const uint16_t ops[] = {S_ADD_U32, S_MUL_I32, S_LSHL_B32, S_AND_B32, S_ADD_I32, S_SUB_U32, S_OR_B32, S_LSHR_B32};
    uint64_t *r = &g->h.rng;
    uint16_t op = ops[below(r, 8)];
    int32_t lit = 0;
    uint16_t a = pick_ssrc(g, &lit, 0);
    uint16_t b = pick_ssrc(g, &lit, 1);
    if (op == S_LSHL_B32 || op == S_LSHR_B32) b = ICONST((int)below(r, 8));
    uint16_t d = pick_sdst(g);
    emit(g, op, d, a, b, b == LIT ? lit : 0);
    note_s(g, d);
}

static void vector_alu(G *g) {
    static const uint16_t ops[] = {V_ADD_CO_U32, V_MUL_LO_U32, V_LSHLREV_B32, V_AND_B32, V_CNDMASK_B32, V_ADD_U32,
                                   V_MUL_U32_U24, V_MAD_U32_U24, V_OR_B32, V_XOR_B32, V_SUB_CO_U32, V_LSHRREV_B32,
                                   V_ASHRREV_I32, V_MOV_B32, V_MUL_HI_U32};
    uint64_t *r = &g->h.rng;
    uint16_t op = ops[below(r, 15)];
    int32_t lit = 0;
    uint16_t d = pick_vdst(g);
    if (op == V_MOV_B32) {
        uint16_t a = chance(r, 0.3) ? pick_ssrc(g, &lit, 1) : pick_vsrc(g, &lit, 1);
        emit(g, op, d, a, NONE, a == LIT ? lit : 0);
    } else if (op == V_LSHLREV_B32 || op == V_LSHRREV_B32 || op == V_ASHRREV_I32) {
        uint16_t v = pick_vsrc(g, &lit, 0);
        emit(g, op, d, ICONST((int)below(r, 6)), v, 0);
    } else if (op == V_MAD_U32_U24) {
        uint16_t a = pick_vsrc(g, &lit, 0), b = pick_vsrc(g, &lit, 0);
        uint16_t c = chance(r, 0.3) ? ICONST((int)below(r, 64)) : pick_vsrc(g, &lit, 0);
        emit(g, op, d, a, b, (int32_t)c);
    } else {
        uint16_t a = pick_vsrc(g, &lit, 0);
        uint16_t b = chance(r, 0.3) ? pick_ssrc(g, &lit, 1) : pick_vsrc(g, &lit, 1);
        emit(g, op, d, a, b, b == LIT ? lit : 0);
    }
    note_v(g, d);
}

static void float_alu(G *g) {
    uint64_t *r = &g->h.rng;
    int32_t lit = 0;
    double u = u01(r);
    if (u < 0.08) {   /* a few doubles on an even-aligned scratch pair */
        uint16_t d = VG(g->v_lo + 2 * (int)below(r, (uint32_t)((g->v_hi - g->v_lo) / 2)));
        uint16_t a = VG(g->v_lo + 2 * (int)below(r, (uint32_t)((g->v_hi - g->v_lo) / 2)));
        uint16_t op = below(r, 2) ? V_ADD_F64 : V_MUL_F64;
        emit(g, op, d, a, chance(r, 0.3) ? FCONST(below(r, 8)) : d, 0);
        return;
    }
    if (u < 0.15) {
        uint16_t d = pick_vdst(g);
        emit(g, below(r, 2) ? V_CVT_F32_U32 : V_CVT_U32_F32, d, pick_vsrc(g, &lit, 0), NONE, 0);
        note_v(g, d);
        return;
    }
    static const uint16_t ops[] = {V_ADD_F32, V_MUL_F32, V_MAD_F32, V_SUB_F32, V_MAX_F32, V_FMA_F32};
    uint16_t op = ops[below(r, 6)];
    uint16_t d = pick_vdst(g);
    uint16_t a = pick_vsrc(g, &lit, 0);
    uint16_t b = chance(r, 0.25) ? FCONST(below(r, 8)) : pick_vsrc(g, &lit, 0);
    if (op == V_MAD_F32 || op == V_FMA_F32) emit(g, op, d, a, b, (int32_t)pick_vsrc(g, &lit, 0));
    else emit(g, op, d, a, b, 0);
    note_v(g, d);
}

/* array element access through a pointer argument: 7 instructions */
static void global_access(G *g) {
    uint64_t *r = &g->h.rng;
    int32_t lit = 0;
    uint16_t idx = chance(r, 0.75) ? VG(1) : pick_vsrc(g, &lit, 0);
    int arg = (int)below(r, 2);
    int shift = chance(r, 0.85) ? 2 : 3;
    emit(g, V_MOV_B32, VG(2), idx, NONE, 0);
    if (chance(r, 0.5)) emit(g, V_MOV_B32, VG(3), ICONST(0), NONE, 0);
    else emit(g, V_ASHRREV_I32, VG(3), ICONST(31), VG(2), 0);
    emit(g, V_LSHLREV_B64, VG(2), ICONST(shift), VG(2), 0);
    emit(g, V_ADD_CO_U32, VG(4), SG(12 + 2 * arg), VG(2), 0);
    emit(g, V_MOV_B32, VG(5), SG(13 + 2 * arg), NONE, 0);
    emit(g, V_ADDC_CO_U32, VG(5), VG(5), VG(3), 0);
    int32_t off = chance(r, 0.8) ? 0 : 4 * (int)below(r, 16);
    if (chance(r, 0.55)) {
        uint16_t d = pick_vdst(g);
        emit(g, chance(r, 0.9) ? GLOBAL_LOAD_DWORD : FLAT_LOAD_DWORD, d, VG(4), NONE, off);
        note_v(g, d);
    } else {
        emit(g, chance(r, 0.9) ? GLOBAL_STORE_DWORD : FLAT_STORE_DWORD, pick_vreg(g), VG(4), NONE, off);
    }
}

/* local-memory traffic indexed by local id: 2 instructions */
static void lds_access(G *g) {
    uint64_t *r = &g->h.rng;
    int32_t lit = 0;
    emit(g, V_LSHLREV_B32, VG(6), ICONST(2), chance(r, 0.7) ? VG(below(r, (uint32_t)g->h.dims)) : pick_vsrc(g, &lit, 0), 0);
    int32_t off = 4 * (int)below(r, 64);
    if (chance(r, 0.5)) {
        emit(g, DS_WRITE_B32, pick_vreg(g), VG(6), NONE, off);
    } else {
        uint16_t d = pick_vdst(g);
        emit(g, DS_READ_B32, d, VG(6), NONE, off);
        note_v(g, d);
    }
}

/* one straight-line item; returns its size (<= budget) */
static uint32_t item(G *g, uint32_t budget) {
    uint64_t *r = &g->h.rng;
    double u = u01(r);
    if (u < 0.26) { scalar_alu(g); return 1; }
    if (u < 0.52) { vector_alu(g); return 1; }
    if (u < 0.82) { float_alu(g); return 1; }
    if (u < 0.91 && budget >= 7) { global_access(g); return 7; }
    if (budget >= 2) { lds_access(g); return 2; }
    vector_alu(g);
    return 1;
}

static void straight(G *g, uint32_t budget) {
    while (budget > 0) budget -= item(g, budget);
}

static void region(G *g, uint32_t budget, int if_depth, int loop_depth);

static void patch(G *g, uint32_t at, uint32_t target) { g->out[at].target = (int32_t)target; }

/* exec-mask if/else.  Shape A closes the then part with a second exec test
 * (s_or_saveexec / s_xor exec / s_cbranch_execz), shape B with an
 * unconditional jump to the join; both restore exec with s_or_b64 at the join. */
static void diamond_shape(G *g, uint32_t budget, int shape_a, int if_depth, int loop_depth) {
    uint64_t *r = &g->h.rng;
    uint32_t fixed = shape_a ? 7 : 5;
    uint32_t body = budget - fixed;
    uint32_t then_n = 1 + below(r, body - 1);
    uint32_t else_n = body - then_n;
    uint16_t pair = SG(24 + 2 * if_depth);
    static const uint16_t cmps[] = {V_CMP_GT_U32, V_CMP_LT_U32, V_CMP_EQ_U32, V_CMP_LT_I32, V_CMP_GT_F32};
    int32_t lit = 0;
    uint16_t a = pick_vsrc(g, &lit, 0), b = pick_vsrc(g, &lit, 0);
    emit(g, cmps[below(r, 5)], NONE, a, b, 0);
    emit(g, S_AND_SAVEEXEC_B64, pair, VCC, NONE, 0);
    uint32_t j_else = emit_branch(g, S_CBRANCH_EXECZ);
    region(g, then_n, if_depth + 1, loop_depth);
    if (shape_a) {
        patch(g, j_else, g->n);
        emit(g, S_OR_SAVEEXEC_B64, pair, pair, NONE, 0);
        emit(g, S_XOR_B64, EXEC, EXEC, pair, 0);
        uint32_t j_end = emit_branch(g, S_CBRANCH_EXECZ);
        region(g, else_n, if_depth + 1, loop_depth);
        patch(g, j_end, g->n);
    } else {
        uint32_t j_end = emit_branch(g, S_BRANCH);
        patch(g, j_else, g->n);
        region(g, else_n, if_depth + 1, loop_depth);
        patch(g, j_end, g->n);
    }
    emit(g, S_OR_B64, EXEC, EXEC, pair, 0);
}

static void diamond(G *g, uint32_t budget, int if_depth, int loop_depth) {
    int shape_a = budget >= 9 && chance(&g->h.rng, 0.5);
    diamond_shape(g, budget, shape_a, if_depth, loop_depth);
}

/* counted scalar loop with a back edge: s_mov / body / s_add, s_cmp, s_cbranch_scc1 */
static void loop(G *g, uint32_t budget, int if_depth, int loop_depth) {
    uint64_t *r = &g->h.rng;
    uint16_t ctr = SG(18 + loop_depth);
    emit(g, S_MOV_B32, ctr, ICONST(0), NONE, 0);
    uint32_t head = g->n;
    region(g, budget - 4, if_depth, loop_depth + 1);
    emit(g, S_ADD_U32, ctr, ctr, ICONST(1), 0);
    emit(g, S_CMP_LT_U32, NONE, ctr, ICONST(2 + (int)below(r, 60)), 0);
    uint32_t j = emit_branch(g, S_CBRANCH_SCC1);
    patch(g, j, head);
}

static void region(G *g, uint32_t budget, int if_depth, int loop_depth) {
    uint64_t *r = &g->h.rng;
    while (budget > 0) {
        int can_if = if_depth < g->if_depth_max && budget >= 8;
        int can_loop = loop_depth < g->loop_depth_max && budget >= 6;
        if ((can_if || can_loop) && chance(r, g->p_struct)) {
            uint32_t hi = budget < 400 ? budget : 400;
            uint32_t sz = 8 + below(r, hi - 7);
            if (sz > budget) sz = budget;
            if (can_if && (!can_loop || chance(r, 0.6)) && sz >= 8) diamond(g, sz, if_depth, loop_depth);
            else if (can_loop && sz >= 6) loop(g, sz, if_depth, loop_depth);
            else { budget -= item(g, budget); continue; }
            budget -= sz;
        } else {
            budget -= item(g, budget);
        }
    }
}

/* C1: 0-2 top-level diamonds, at most one of shape A, no loops: <= 8 blocks */
static void body_c1(G *g, uint32_t budget) {
    uint64_t *r = &g->h.rng;
    int nd = budget < 40 ? 0 : (int)below(r, 3);
    uint32_t dsz[2] = {0, 0}, seg[3] = {0, 0, 0};
    for (int i = 0; i < nd; i++) dsz[i] = 9 + below(r, budget / 4 - 8);
    uint32_t rest = budget - dsz[0] - dsz[1];
    for (int i = 0; i < nd; i++) { seg[i] = below(r, rest + 1); rest -= seg[i]; }
    seg[nd] = rest;
    int used_a = 0;
    int saved = g->if_depth_max;
    g->if_depth_max = 0;   /* no nesting inside the diamonds */
    for (int i = 0; i <= nd; i++) {
        straight(g, seg[i]);
        if (i < nd) {
            int shape_a = !used_a && chance(r, 0.5);
            used_a |= shape_a;
            diamond_shape(g, dsz[i], shape_a, 0, 0);
        }
    }
    g->if_depth_max = saved;
}

static void gen_body(G *g) {
    header *h = &g->h;
    uint32_t L = h->len;
    /* prologue */
    emit(g, S_LOAD_DWORDX2, SG(2), SG(4), NONE, 0x0);
    emit(g, S_LOAD_DWORDX4, SG(12), SG(4), NONE, 0x30);
    if (h->has_int_arg) emit(g, S_LOAD_DWORD, SG(16), SG(4), NONE, 0x40);
    if (h->has_gsize) emit(g, S_LOAD_DWORD, SG(17), SG(4), NONE, 0xc);
    emit(g, S_WAITCNT, NONE, NONE, NONE, 0);
    if (h->shift_form) {
        int lg = 0;
        while ((1u << lg) < h->cws[0]) lg++;
        emit(g, S_LSHL_B32, SG(0), SG(6), ICONST(lg), 0);
    } else {
        emit(g, S_MUL_I32, SG(0), SG(6), h->cws[0] <= 64 ? ICONST((int)h->cws[0]) : LIT, (int32_t)h->cws[0]);
        if (h->cws[0] <= 64) g->out[g->n - 1].imm = 0;
    }
    emit(g, V_ADD_CO_U32, VG(1), SG(0), VG(0), 0);
    emit(g, V_ADD_CO_U32, VG(1), SG(2), VG(1), 0);
    uint32_t pro = g->n;
    if (h->has_gsize && L >= pro + 2 + 8) {
        int lg = 0;
        while ((1u << lg) < h->cws[0]) lg++;
        emit(g, S_LSHR_B32, SG(11), SG(17), ICONST(lg), 0);
        pro++;
    }
    note_v(g, VG(1));
    note_s(g, SG(0));
    uint32_t budget = L - pro - 1;
    if (g->cfg == 1) body_c1(g, budget);
    else region(g, budget, 0, 0);
    emit(g, S_ENDPGM, NONE, NONE, NONE, 0);
}

static uint32_t n_args_of(const header *h) { return 2u + (h->has_int_arg ? 1u : 0u); }

static void fill_args(const header *h, gen_arg *a) {
    a[0].offset = 0x30; a[0].size = 8; a[0].type = T_PTR; a[0].flags = h->pointee[0];
    a[1].offset = 0x38; a[1].size = 8; a[1].type = T_PTR; a[1].flags = h->pointee[1];
    if (h->has_int_arg) { a[2].offset = 0x40; a[2].size = 4; a[2].type = T_INT; a[2].flags = 0; }
}

static void gen_one(int cfg, uint64_t index, gen_instr *out) {
    G g;
    memset(&g, 0, sizeof(g));
    make_header(cfg, index, &g.h);
    g.cfg = cfg;
    g.out = out;
    g.s_lo = 34; g.s_hi = g.h.full_range ? 103 : 63;
    g.v_lo = 8; g.v_hi = g.h.full_range ? 255 : 63;
    g.if_depth_max = cfg == 1 ? 1 : (cfg == 4 || cfg == 6) ? 5 : 3;
    g.loop_depth_max = cfg == 1 ? 0 : (cfg == 4 || cfg == 6) ? 5 : 3;
    g.p_struct = cfg == 4 ? 0.0025 : cfg == 6 ? 0.3 : 0.012;
    gen_body(&g);
}

/* ---------------- exported API ---------------- */
int dcgen_n_ops(void) { return N_OPS; }
const char *dcgen_op_name(int id) { return (id >= 0 && id < N_OPS) ? OP_NAMES[id] : 0; }

/* lengths and argument counts of kernels [i0, i0+n) of config cfg */
void dcgen_sizes(int cfg, uint64_t i0, uint32_t n, uint32_t *len, uint32_t *nargs) {
    for (uint32_t i = 0; i < n; i++) {
        header h;
        make_header(cfg, i0 + i, &h);
        len[i] = h.len;
        nargs[i] = n_args_of(&h);
    }
}

typedef struct {
    int cfg; uint64_t i0; uint32_t lo, hi;
    gen_instr *instrs; gen_kernel *kernels; gen_arg *args;
    const uint64_t *ioff; const uint32_t *aoff;
} job;

static void *worker(void *p) {
    job *j = (job *)p;
    for (uint32_t i = j->lo; i < j->hi; i++) {
        header h;
        make_header(j->cfg, j->i0 + i, &h);
        gen_kernel *k = &j->kernels[i];
        k->instr_begin = j->ioff[i];
        k->n_instr = h.len;
        k->dims = (uint8_t)h.dims;
        k->useargs = 1;
        k->n_args = (uint16_t)n_args_of(&h);
        k->cws[0] = h.cws[0]; k->cws[1] = h.cws[1]; k->cws[2] = h.cws[2];
        k->arg_begin = j->aoff[i];
        fill_args(&h, &j->args[j->aoff[i]]);
        gen_one(j->cfg, j->i0 + i, &j->instrs[j->ioff[i]]);
    }
    return 0;
}

/* Generate kernels [i0, i0+n) of config cfg into caller buffers sized from
 * dcgen_sizes: instrs (sum of lengths), kernels (n), args (sum of nargs).
 * ioff/aoff are the exclusive prefix sums of the lengths / argument counts. */
int dcgen_generate(int cfg, uint64_t i0, uint32_t n, const uint64_t *ioff, const uint32_t *aoff,
                   gen_instr *instrs, gen_kernel *kernels, gen_arg *args, int threads) {
    if (threads < 1) threads = 1;
    if (threads > 64) threads = 64;
    if ((uint32_t)threads > n) threads = n ? (int)n : 1;
    pthread_once(&zipf_once, zipf_init);
    pthread_t th[64];
    job jobs[64];
    for (int t = 0; t < threads; t++) {
        jobs[t] = (job){cfg, i0, (uint32_t)((uint64_t)n * t / threads), (uint32_t)((uint64_t)n * (t + 1) / threads),
                        instrs, kernels, args, ioff, aoff};
        if (threads > 1) pthread_create(&th[t], 0, worker, &jobs[t]);
    }
    if (threads == 1) worker(&jobs[0]);
    else for (int t = 0; t < threads; t++) pthread_join(th[t], 0);
    return 0;
}

/* ---- text rendering: the listing format of the paper's Listings 1 and 3 ----
 * Each kernel becomes
 *   .kernel k<index>
 *     .config
 *       .dims x|xy|xyz
 *       .cws a, b, c
 *       <ignored directives>, .useargs, six hidden .arg lines, user .arg lines
 *     .text
 *   L<i>:              (before every branch target i)
 *       <mnemonic> <operands>
 * with comment lines, trailing comments, blank lines and tabs sprinkled in
 * deterministically, so that a reader must cope with them.  The operand
 * syntax per opcode is the one of the tests' assembler. */
typedef struct { char *p; uint64_t n, cap; } sbuf;

static void sb_grow(sbuf *b, uint64_t more) {
    if (b->n + more + 1 <= b->cap) return;
    uint64_t c = b->cap ? b->cap : 4096;
    while (c < b->n + more + 1) c *= 2;
    b->p = (char *)realloc(b->p, c);
    b->cap = c;
}
static void sb_str(sbuf *b, const char *s) {
    const size_t l = strlen(s);
    sb_grow(b, l);
    memcpy(b->p + b->n, s, l);
    b->n += l;
}
static void sb_fmt(sbuf *b, const char *fmt, ...) {
    char tmp[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(tmp, sizeof tmp, fmt, ap);
    va_end(ap);
    sb_str(b, tmp);
}

/* register width of operand slot o (0 r0, 1 r1, 2 r2, 3 src2) of op, for
 * the register-range syntax only */
static int op_width(int op, int o) {
    switch (op) {
    case S_LOAD_DWORD: return o == 0 ? 1 : 2;
    case S_LOAD_DWORDX2: return 2;
    case S_LOAD_DWORDX4: return o == 0 ? 4 : 2;
    case S_MOV_B64: case S_AND_SAVEEXEC_B64: case S_OR_SAVEEXEC_B64: case S_AND_B64: case S_OR_B64:
    case S_XOR_B64: case S_ANDN2_B64: case V_ADD_F64: case V_MUL_F64: case V_FMA_F64:
        return 2;
    case V_CVT_F64_F32: return o == 0 ? 2 : 1;
    case V_LSHLREV_B64: return o == 1 ? 1 : 2;
    case GLOBAL_LOAD_DWORD: case GLOBAL_STORE_DWORD: return o == 0 ? 1 : 2;
    case FLAT_LOAD_DWORD: case FLAT_STORE_DWORD: return o == 0 ? 1 : 2;
    case GLOBAL_LOAD_DWORDX2: case GLOBAL_STORE_DWORDX2: return 2;
    default: return 1;
    }
}

static const char *const FLOAT_TEXT[8] = {"0.5", "-0.5", "1.0", "-1.0", "2.0", "-2.0", "4.0", "-4.0"};

static void operand_text(sbuf *b, uint16_t id, int w, int32_t imm, uint64_t salt) {
    if (id >= 0x8000 && id <= 0x8050) { sb_fmt(b, "%d", (int)id - 0x8000 - 16); return; }
    if (id >= 0x8060 && id <= 0x8067) { sb_str(b, FLOAT_TEXT[id - 0x8060]); return; }
    if (id == LIT) {
        if (imm < 0 || (salt & 1)) sb_fmt(b, "%d", imm);
        else sb_fmt(b, "0x%x", (uint32_t)imm);
        return;
    }
    if (id == NONE) { sb_str(b, "off"); return; }
    if (id == 104) { sb_str(b, w == 2 ? "vcc" : "vcc_lo"); return; }
    if (id == 105) { sb_str(b, "vcc_hi"); return; }
    if (id == 106) { sb_str(b, w == 2 ? "exec" : "exec_lo"); return; }
    if (id == 107) { sb_str(b, "exec_hi"); return; }
    if (id == 108) { sb_str(b, "scc"); return; }
    if (id == 109) { sb_str(b, "m0"); return; }
    const char c = id >= 112 ? 'v' : 's';
    const int n = id >= 112 ? id - 112 : id;
    if (w == 1) sb_fmt(b, "%c%d", c, n);
    else sb_fmt(b, "%c[%d:%d]", c, n, n + w - 1);
}

static const char *type_name(uint8_t t) {
    switch (t) {
    case T_INT: return "int";
    case T_UINT: return "uint";
    case T_FLOAT: return "float";
    case T_DOUBLE: return "double";
    default: return "void";
    }
}

static void render_kernel(sbuf *b, uint64_t index, const gen_kernel *k, const gen_instr *ins, const gen_arg *args) {
    uint64_t salt = 0x5EED0000u + index;
    sb_fmt(b, ".kernel k%llu\n  .config\n", (unsigned long long)index);
    static const char *const DIMS[4] = {"", "x", "xy", "xyz"};
    sb_fmt(b, "    .dims %s\n", k->dims <= 3 ? DIMS[k->dims] : "xyzw");
    sb_fmt(b, "    .cws %u, %u, %u\n", k->cws[0], k->cws[1], k->cws[2]);
    sb_str(b, "    .sgprsnum 104\n    .vgprsnum 256\n    .floatmode 0xc0\n");
    if (k->useargs) sb_str(b, "    .useargs\n");
    sb_str(b, "    .priority 0\n"
              "    .arg _.global_offset_0, \"size_t\", long\n"
              "    .arg _.global_offset_1, \"size_t\", long\n"
              "    .arg _.global_offset_2, \"size_t\", long\n"
              "    .arg _.printf_buffer, \"size_t\", void*, global, , rdonly\n"
              "    .arg _.vqueue_pointer,\"size_t\", long\n"
              "    .arg _.aqlwrap_pointer,\"size_t\", long\n");
    for (uint32_t a = 0; a < k->n_args; a++) {
        const gen_arg *g = &args[a];
        if (g->type == T_PTR) {
            const char *t = type_name(g->flags);
            sb_fmt(b, "    .arg a%u, \"%s*\", %s*, global,\n", a, t, t);
        } else {
            const char *t = type_name(g->type);
            sb_fmt(b, "    .arg a%u, \"%s\", %s\n", a, t, t);
        }
    }
    sb_str(b, "  .text\n");
    const uint32_t n = k->n_instr;
    uint8_t *tgt = (uint8_t *)calloc(n ? n : 1, 1);
    for (uint32_t i = 0; i < n; i++)
        if (ins[i].target >= 0 && (uint32_t)ins[i].target < n) tgt[ins[i].target] = 1;
    for (uint32_t i = 0; i < n; i++) {
        const gen_instr *x = &ins[i];
        salt = salt * 6364136223846793005ull + 1442695040888963407ull;
        if (tgt[i]) sb_fmt(b, "L%u:\n", i);
        if ((salt >> 59) == 0) sb_str(b, "\n");
        if ((salt >> 58) == 3) sb_str(b, "    // note\n");
        sb_str(b, (salt >> 40) & 1 ? "\t" : "    ");
        const int op = x->op;
        if (op >= N_OPS) { sb_fmt(b, "op%d\n", op); continue; }
        sb_str(b, OP_NAMES[op]);
        const uint64_t s2 = salt >> 20;
#define OPND(id, o) operand_text(b, (id), op_width(op, (o)), x->imm, s2)
        switch (op) {
        case S_LOAD_DWORD: case S_LOAD_DWORDX2: case S_LOAD_DWORDX4:
            sb_str(b, " "); OPND(x->r0, 0); sb_str(b, ", "); OPND(x->r1, 1); sb_fmt(b, ", 0x%x", (uint32_t)x->imm);
            break;
        case S_BRANCH: case S_CBRANCH_SCC0: case S_CBRANCH_SCC1: case S_CBRANCH_VCCZ: case S_CBRANCH_VCCNZ:
        case S_CBRANCH_EXECZ: case S_CBRANCH_EXECNZ:
            sb_fmt(b, " L%d", x->target);
            break;
        case S_WAITCNT: sb_str(b, " lgkmcnt(0)"); break;
        case S_BARRIER: case S_ENDPGM: break;
        case S_NOP: sb_str(b, " 0"); break;
        case S_CMP_EQ_U32: case S_CMP_LT_U32: case S_CMP_GT_U32: case S_CMP_LT_I32:
            sb_str(b, " "); OPND(x->r1, 1); sb_str(b, ", "); OPND(x->r2, 2);
            break;
        case V_CMP_EQ_U32: case V_CMP_GT_U32: case V_CMP_LT_U32: case V_CMP_LT_I32: case V_CMP_GT_F32:
            sb_str(b, " vcc, "); OPND(x->r1, 1); sb_str(b, ", "); OPND(x->r2, 2);
            break;
        case GLOBAL_LOAD_DWORD: case GLOBAL_LOAD_DWORDX2:
            sb_str(b, " "); OPND(x->r0, 0); sb_str(b, ", "); OPND(x->r1, 1); sb_str(b, ", "); OPND(x->r2, 2);
            if (x->imm) sb_fmt(b, " offset:%d", x->imm);
            break;
        case FLAT_LOAD_DWORD: case DS_READ_B32:
            sb_str(b, " "); OPND(x->r0, 0); sb_str(b, ", "); OPND(x->r1, 1);
            if (x->imm) sb_fmt(b, " offset:%d", x->imm);
            break;
        case GLOBAL_STORE_DWORD: case GLOBAL_STORE_DWORDX2:
            sb_str(b, " "); OPND(x->r1, 1); sb_str(b, ", "); OPND(x->r0, 0); sb_str(b, ", "); OPND(x->r2, 2);
            if (x->imm) sb_fmt(b, " offset:%d", x->imm);
            break;
        case FLAT_STORE_DWORD: case DS_WRITE_B32:
            sb_str(b, " "); OPND(x->r1, 1); sb_str(b, ", "); OPND(x->r0, 0);
            if (x->imm) sb_fmt(b, " offset:%d", x->imm);
            break;
        case V_ADD_CO_U32: case V_SUB_CO_U32: case V_ADDC_CO_U32:
            sb_str(b, " "); OPND(x->r0, 0); sb_str(b, ", vcc, "); OPND(x->r1, 1); sb_str(b, ", "); OPND(x->r2, 2);
            if (op == V_ADDC_CO_U32) sb_str(b, ", vcc");
            break;
        case V_CNDMASK_B32:
            sb_str(b, " "); OPND(x->r0, 0); sb_str(b, ", "); OPND(x->r1, 1); sb_str(b, ", "); OPND(x->r2, 2);
            sb_str(b, ", vcc");
            break;
        case V_MAD_U32_U24: case V_MAD_F32: case V_FMA_F32: case V_FMA_F64:
            sb_str(b, " "); OPND(x->r0, 0); sb_str(b, ", "); OPND(x->r1, 1); sb_str(b, ", "); OPND(x->r2, 2);
            sb_str(b, ", "); operand_text(b, (uint16_t)x->imm, op_width(op, 3), 0, s2);
            break;
        case S_MOV_B32: case S_MOV_B64: case S_AND_SAVEEXEC_B64: case S_OR_SAVEEXEC_B64: case V_MOV_B32:
        case V_CVT_F32_U32: case V_CVT_U32_F32: case V_CVT_F64_F32:
            sb_str(b, " "); OPND(x->r0, 0); sb_str(b, ", "); OPND(x->r1, 1);
            break;
        default:
            sb_str(b, " "); OPND(x->r0, 0); sb_str(b, ", "); OPND(x->r1, 1); sb_str(b, ", "); OPND(x->r2, 2);
        }
#undef OPND
        if ((salt >> 56) == 7) sb_str(b, "   ; trailing");
        sb_str(b, (salt >> 30) % 13 == 0 ? " \r\n" : "\n");
    }
    free(tgt);
}

/* Render n kernels (records relative to instrs, args relative to args) into
 * a malloc'ed buffer; *out_len = its length.  Free it with dcgen_free. */
char *dcgen_render(const gen_kernel *kernels, uint32_t n, const gen_instr *instrs, const gen_arg *args,
                   uint64_t *out_len) {
    sbuf b = {0, 0, 0};
    sb_str(&b, "// seeded synthetic kernels\n");
    for (uint32_t k = 0; k < n; k++)
        render_kernel(&b, k, &kernels[k], instrs + kernels[k].instr_begin, args + kernels[k].arg_begin);
    sb_grow(&b, 0);
    b.p[b.n] = 0;
    *out_len = b.n;
    return b.p;
}
void dcgen_free(void *p) { free(p); }
