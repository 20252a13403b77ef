/*
 * dc_oracle.c -- plain CPU oracle for the register-state dataflow analysis.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the bench's
 * CPU-baseline leg may load this.  It shares no code with the GPU path.
 *
 * What it computes: the least fixpoint (Kildall 1973; Kam & Ullman 1977) of
 * a forward dataflow problem over each GCN kernel's control flow graph, whose
 * lattice value per register is the triple (provenance bits, type bits,
 * payload).  This is the analysis behind the paper's "search for memory
 * accesses" and "data type recovery" steps (Section "Statement of the
 * problem", method steps 2 and 3):
 *   - the entry state is the ABI's register initialisation (Section "Search
 *     for memory accesses": s[4:5] holds the kernel-argument pointer, v0..v2
 *     the local ids, s6..s8 the work-group ids when "useargs" is set);
 *   - a load from s[4:5] at a known offset is a call of a work-item built-in
 *     or the value of a kernel argument (same section; Listing 3 layout);
 *   - work-group id times the work-group size from .cws, plus local id, plus
 *     global offset, is get_global_id (same section, steps 4-5);
 *   - types come from instruction suffixes and from the .arg table (Section
 *     "Data type recovery");
 *   - at a block with several predecessors a register whose incoming values
 *     differ becomes ambiguous (Section "Search for control structures",
 *     paragraph on vertices with several ancestors): the payload joins to TOP.
 * The rule tables below make these passages exact.  Where the paper leaves a
 * choice open (record format, argument-area offsets, the order of id terms,
 * carries, float results) they take one reading throughout; the tests under
 * tests/ pin each one.
 *
 * Everything here is deliberately simple: full 368-slot states, plain loops,
 * no blocking.  The reference schedule is round-robin in reverse postorder
 * (pull form, IN[b] = join of the OUT of reached predecessors); a FIFO and a
 * randomly ordered worklist are provided so tests can check that the result
 * does not depend on the schedule.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* wire formats                                                         */
/* ------------------------------------------------------------------ */
typedef struct { uint16_t op, r0, r1, r2; int32_t imm, target; } or_instr;
typedef struct {
    uint64_t instr_begin; uint32_t n_instr; uint8_t dims, useargs; uint16_t n_args;
    uint32_t cws[3]; uint32_t arg_begin;
} or_kernel;
typedef struct { uint32_t offset; uint16_t size; uint8_t type, flags; } or_arg;
typedef struct { uint32_t prov; uint8_t type, flags, pad0, pad1; uint64_t val; } or_slot;
typedef struct { uint32_t instr; uint8_t kind, space, width, dtype; uint64_t addr; } or_access;
typedef struct { uint32_t instr; uint16_t slot; uint8_t kind, dim; } or_sysval;

_Static_assert(sizeof(or_instr) == 16, "instr");
_Static_assert(sizeof(or_kernel) == 32, "kernel");
_Static_assert(sizeof(or_arg) == 8, "arg");
_Static_assert(sizeof(or_slot) == 16, "slot");
_Static_assert(sizeof(or_access) == 16, "access");
_Static_assert(sizeof(or_sysval) == 8, "sysval");

#define NSLOT 368

/* status codes */
enum {
    OK = 0, E_BADOP = -10, E_BADREG = -11, E_BADTARGET = -12, E_NOEND = -13,
    E_UNSUPPORTED = -14, E_NOFIX = -15
};

/* provenance bits */
#define P_LID(d) (1u << (0 + (d)))
#define P_WGID(d) (1u << (3 + (d)))
#define P_GOFF(d) (1u << (6 + (d)))
#define P_GSIZE(d) (1u << (9 + (d)))
#define P_WORKDIM (1u << 12)
#define P_SYSPTR (1u << 13)
#define P_CONST (1u << 14)
#define P_LOADG (1u << 15)
#define P_LOADL (1u << 16)
#define P_UNINIT (1u << 17)
#define P_MASK (1u << 18)
#define P_HIDDEN (1u << 19)
static uint32_t P_KARG(unsigned k) { return 1u << (20 + (k < 11 ? k : 11)); }

/* type bits */
#define TY_INT 1
#define TY_UINT 2
#define TY_FLOAT 4
#define TY_DOUBLE 8
#define TY_PTR 16

/* payload tags and fields */
enum { CONSTV = 0, SYSPTR = 1, KARG = 2, WGID = 3, IDX = 4, SHL = 5, PTR = 6, SYS = 7, UNINIT = 8, TOPTAG = 15 };
enum { ENTIRE = 0, LOW = 1, HIGH = 2 };
enum { SYS_GOFF_HI = 0, SYS_GSIZE = 1, SYS_NUMGROUPS = 2, SYS_WORKDIM = 3, SYS_HIDDEN = 4 };
#define M_WG 1
#define M_LID 2
#define M_GOFF 4
#define TOP 0xFFFFFFFFFFFFFFFFull

static uint64_t mk(unsigned tag, unsigned integ, unsigned dim, unsigned aux, unsigned shift, unsigned arg, uint32_t c) {
    return ((uint64_t)tag << 60) | ((uint64_t)integ << 58) | ((uint64_t)dim << 56) | ((uint64_t)aux << 52) |
           ((uint64_t)shift << 48) | ((uint64_t)arg << 40) | (uint64_t)c;
}
static unsigned tag_of(uint64_t v) { return (unsigned)(v >> 60); }
static unsigned integ_of(uint64_t v) { return (unsigned)(v >> 58) & 3; }
static unsigned dim_of(uint64_t v) { return (unsigned)(v >> 56) & 3; }
static unsigned aux_of(uint64_t v) { return (unsigned)(v >> 52) & 15; }
static unsigned shift_of(uint64_t v) { return (unsigned)(v >> 48) & 15; }
static unsigned arg_of(uint64_t v) { return (unsigned)(v >> 40) & 255; }
static uint32_t c_of(uint64_t v) { return (uint32_t)v; }
static uint64_t CONST32(uint32_t c) { return mk(CONSTV, ENTIRE, 0, 0, 0, 0, c); }
static int is_const(uint64_t v) { return v != TOP && tag_of(v) == CONSTV; }

/* sysval kinds, access kinds/spaces */
enum { SV_GLOBAL_ID, SV_GLOBAL_ID_MINUS_OFFSET, SV_GLOBAL_OFFSET, SV_GLOBAL_SIZE, SV_NUM_GROUPS,
       SV_WORK_DIM, SV_GROUP_BASE, SV_LOCAL_ID, SV_GROUP_ID };
enum { AK_LOAD = 0, AK_STORE = 1 };
enum { SP_GLOBAL = 0, SP_FLAT = 1, SP_LDS = 2 };

/* ------------------------------------------------------------------ */
/* the instruction subset                                               */
/* ------------------------------------------------------------------ */
/* Operand roles.  A role names what a field holds and how wide it is.    */
enum role {
    NO,      /* field must be none (0xFFFF) */
    SD,      /* scalar register def */
    SU,      /* scalar register use (no constants) */
    SC,      /* scalar register use or constant */
    VD,      /* vector register def */
    VU,      /* vector register use (no constants) */
    VC,      /* vector or scalar register use, or constant */
    SADDR    /* scalar pair use, or none */
};
/* type rules (Section "Data type recovery"; mnemonic suffixes) */
enum trule { T_NONE, T_SUF, T_ADD, T_B, T_MOVE, T_SMEM };
/* payload rules */
enum prule { R_TOP, R_SMEM, R_MOV, R_ADD, R_ADDC, R_SUB, R_MUL, R_MUL24, R_MAD24, R_SHL32, R_LSHR32,
             R_ASHR, R_AND, R_OR, R_XOR, R_FOLD64_AND, R_FOLD64_OR, R_FOLD64_XOR, R_FOLD64_ANDN2,
             R_SHL64, R_SEL, R_NOEFFECT };
/* classes */
enum cls { C_SMEM, C_SALU, C_SCMP, C_BRANCH, C_CBRANCH, C_NOP, C_END, C_VALU, C_VCMP, C_GLOAD, C_GSTORE,
           C_FLOAD, C_FSTORE, C_DSREAD, C_DSWRITE };
/* implicit register sets */
#define I_VCC 1
#define I_SCC 2
#define I_EXEC 4

typedef struct {
    const char *name;
    enum cls cls;
    enum role r0, r1, r2, src2;   /* src2 lives in imm's low 16 bits */
    int w0, w1, w2, w_src2;       /* dword widths */
    int imm_is_offset;
    int imp_use, imp_def;
    enum trule trule;
    int suffix;                   /* type bits of the first suffix */
    enum prule prule;
    int value_srcs;               /* bitmask of which of r1/r2/src2 are value sources for T_B (1,2,4) */
    int mask_def;                 /* explicit defs also get MASK (exec-mask ops) */
} opinfo;

#define SMEM(n, w) {n, C_SMEM, SD, SU, NO, NO, w, 2, 0, 0, 1, 0, 0, T_SMEM, 0, R_SMEM, 0, 0}
#define SALU2(n, imp_u, imp_d, tr, suf, pr, vs) {n, C_SALU, SD, SC, SC, NO, 1, 1, 1, 0, 0, imp_u, imp_d, tr, suf, pr, vs, 0}
#define SALU64(n, pr) {n, C_SALU, SD, SC, SC, NO, 2, 2, 2, 0, 0, 0, I_SCC, T_B, 0, pr, 3, 0}
#define SCMP(n) {n, C_SCMP, NO, SC, SC, NO, 0, 1, 1, 0, 0, 0, I_SCC, T_NONE, 0, R_NOEFFECT, 0, 0}
#define CBR(n, imp) {n, C_CBRANCH, NO, NO, NO, NO, 0, 0, 0, 0, 0, imp, 0, T_NONE, 0, R_NOEFFECT, 0, 0}
#define PLAIN(n, c) {n, c, NO, NO, NO, NO, 0, 0, 0, 0, 0, 0, 0, T_NONE, 0, R_NOEFFECT, 0, 0}
#define VALU2(n, wd, ws, imp_u, imp_d, tr, suf, pr, vs) {n, C_VALU, VD, VC, VC, NO, wd, ws, ws, 0, 0, imp_u, imp_d, tr, suf, pr, vs, 0}
#define VALU3(n, wd, ws, tr, suf, pr) {n, C_VALU, VD, VC, VC, VC, wd, ws, ws, ws, 0, 0, 0, tr, suf, pr, 0, 0}
#define VCMP(n) {n, C_VCMP, NO, VC, VC, NO, 0, 1, 1, 0, 0, 0, I_VCC, T_NONE, 0, R_NOEFFECT, 0, 0}

static const opinfo OPS[] = {
    SMEM("s_load_dword", 1),
    SMEM("s_load_dwordx2", 2),
    SMEM("s_load_dwordx4", 4),
    {"s_mov_b32", C_SALU, SD, SC, NO, NO, 1, 1, 0, 0, 0, 0, 0, T_MOVE, 0, R_MOV, 1, 0},
    {"s_mov_b64", C_SALU, SD, SC, NO, NO, 2, 2, 0, 0, 0, 0, 0, T_MOVE, 0, R_MOV, 1, 0},
    {"s_and_saveexec_b64", C_SALU, SD, SC, NO, NO, 2, 2, 0, 0, 0, I_EXEC, I_EXEC | I_SCC, T_NONE, 0, R_TOP, 0, 1},
    {"s_or_saveexec_b64", C_SALU, SD, SC, NO, NO, 2, 2, 0, 0, 0, I_EXEC, I_EXEC | I_SCC, T_NONE, 0, R_TOP, 0, 1},
    SALU2("s_add_u32", 0, I_SCC, T_ADD, TY_UINT, R_ADD, 3),
    SALU2("s_add_i32", 0, I_SCC, T_ADD, TY_INT, R_ADD, 3),
    SALU2("s_addc_u32", I_SCC, I_SCC, T_ADD, TY_UINT, R_ADDC, 3),
    SALU2("s_sub_u32", 0, I_SCC, T_SUF, TY_UINT, R_SUB, 3),
    SALU2("s_mul_i32", 0, 0, T_SUF, TY_INT, R_MUL, 3),
    SALU2("s_lshl_b32", 0, I_SCC, T_B, 0, R_SHL32, 1),    /* value r1, amount r2 */
    SALU2("s_lshr_b32", 0, I_SCC, T_B, 0, R_LSHR32, 1),
    SALU2("s_and_b32", 0, I_SCC, T_B, 0, R_AND, 3),
    SALU2("s_or_b32", 0, I_SCC, T_B, 0, R_OR, 3),
    SALU64("s_and_b64", R_FOLD64_AND),
    SALU64("s_or_b64", R_FOLD64_OR),
    SALU64("s_xor_b64", R_FOLD64_XOR),
    SALU64("s_andn2_b64", R_FOLD64_ANDN2),
    SCMP("s_cmp_eq_u32"),
    SCMP("s_cmp_lt_u32"),
    SCMP("s_cmp_gt_u32"),
    SCMP("s_cmp_lt_i32"),
    PLAIN("s_branch", C_BRANCH),
    CBR("s_cbranch_scc0", I_SCC),
    CBR("s_cbranch_scc1", I_SCC),
    CBR("s_cbranch_vccz", I_VCC),
    CBR("s_cbranch_vccnz", I_VCC),
    CBR("s_cbranch_execz", I_EXEC),
    CBR("s_cbranch_execnz", I_EXEC),
    PLAIN("s_waitcnt", C_NOP),
    PLAIN("s_barrier", C_NOP),
    PLAIN("s_nop", C_NOP),
    PLAIN("s_endpgm", C_END),
    {"v_mov_b32", C_VALU, VD, VC, NO, NO, 1, 1, 0, 0, 0, 0, 0, T_MOVE, 0, R_MOV, 1, 0},
    {"v_cvt_f32_u32", C_VALU, VD, VC, NO, NO, 1, 1, 0, 0, 0, 0, 0, T_SUF, TY_FLOAT, R_TOP, 0, 0},
    {"v_cvt_u32_f32", C_VALU, VD, VC, NO, NO, 1, 1, 0, 0, 0, 0, 0, T_SUF, TY_UINT, R_TOP, 0, 0},
    {"v_cvt_f64_f32", C_VALU, VD, VC, NO, NO, 2, 1, 0, 0, 0, 0, 0, T_SUF, TY_DOUBLE, R_TOP, 0, 0},
    VALU2("v_add_co_u32", 1, 1, 0, I_VCC, T_ADD, TY_UINT, R_ADD, 3),
    VALU2("v_addc_co_u32", 1, 1, I_VCC, I_VCC, T_ADD, TY_UINT, R_ADDC, 3),
    VALU2("v_sub_co_u32", 1, 1, 0, I_VCC, T_SUF, TY_UINT, R_SUB, 3),
    VALU2("v_add_u32", 1, 1, 0, 0, T_ADD, TY_UINT, R_ADD, 3),
    VALU2("v_mul_lo_u32", 1, 1, 0, 0, T_SUF, TY_UINT, R_MUL, 3),
    VALU2("v_mul_u32_u24", 1, 1, 0, 0, T_SUF, TY_UINT, R_MUL24, 3),
    VALU2("v_mul_hi_u32", 1, 1, 0, 0, T_SUF, TY_UINT, R_TOP, 3),
    VALU3("v_mad_u32_u24", 1, 1, T_SUF, TY_UINT, R_MAD24),
    VALU2("v_lshlrev_b32", 1, 1, 0, 0, T_B, 0, R_SHL32, 2),   /* amount r1, value r2 */
    VALU2("v_lshrrev_b32", 1, 1, 0, 0, T_B, 0, R_LSHR32, 2),
    VALU2("v_ashrrev_i32", 1, 1, 0, 0, T_SUF, TY_INT, R_ASHR, 2),
    VALU2("v_and_b32", 1, 1, 0, 0, T_B, 0, R_AND, 3),
    VALU2("v_or_b32", 1, 1, 0, 0, T_B, 0, R_OR, 3),
    VALU2("v_xor_b32", 1, 1, 0, 0, T_B, 0, R_XOR, 3),
    {"v_lshlrev_b64", C_VALU, VD, VC, VC, NO, 2, 1, 2, 0, 0, 0, 0, T_B, 0, R_SHL64, 2, 0},
    VALU2("v_cndmask_b32", 1, 1, I_VCC, 0, T_B, 0, R_SEL, 3),
    VALU2("v_add_f32", 1, 1, 0, 0, T_SUF, TY_FLOAT, R_TOP, 3),
    VALU2("v_sub_f32", 1, 1, 0, 0, T_SUF, TY_FLOAT, R_TOP, 3),
    VALU2("v_mul_f32", 1, 1, 0, 0, T_SUF, TY_FLOAT, R_TOP, 3),
    VALU2("v_max_f32", 1, 1, 0, 0, T_SUF, TY_FLOAT, R_TOP, 3),
    VALU3("v_mad_f32", 1, 1, T_SUF, TY_FLOAT, R_TOP),
    VALU3("v_fma_f32", 1, 1, T_SUF, TY_FLOAT, R_TOP),
    VALU2("v_add_f64", 2, 2, 0, 0, T_SUF, TY_DOUBLE, R_TOP, 3),
    VALU2("v_mul_f64", 2, 2, 0, 0, T_SUF, TY_DOUBLE, R_TOP, 3),
    VALU3("v_fma_f64", 2, 2, T_SUF, TY_DOUBLE, R_TOP),
    VCMP("v_cmp_eq_u32"),
    VCMP("v_cmp_gt_u32"),
    VCMP("v_cmp_lt_u32"),
    VCMP("v_cmp_lt_i32"),
    VCMP("v_cmp_gt_f32"),
    {"global_load_dword", C_GLOAD, VD, VU, SADDR, NO, 1, 2, 2, 0, 1, 0, 0, T_NONE, 0, R_TOP, 0, 0},
    {"global_load_dwordx2", C_GLOAD, VD, VU, SADDR, NO, 2, 2, 2, 0, 1, 0, 0, T_NONE, 0, R_TOP, 0, 0},
    {"flat_load_dword", C_FLOAD, VD, VU, NO, NO, 1, 2, 0, 0, 1, 0, 0, T_NONE, 0, R_TOP, 0, 0},
    {"global_store_dword", C_GSTORE, VU, VU, SADDR, NO, 1, 2, 2, 0, 1, 0, 0, T_NONE, 0, R_NOEFFECT, 0, 0},
    {"global_store_dwordx2", C_GSTORE, VU, VU, SADDR, NO, 2, 2, 2, 0, 1, 0, 0, T_NONE, 0, R_NOEFFECT, 0, 0},
    {"flat_store_dword", C_FSTORE, VU, VU, NO, NO, 1, 2, 0, 0, 1, 0, 0, T_NONE, 0, R_NOEFFECT, 0, 0},
    {"ds_read_b32", C_DSREAD, VD, VU, NO, NO, 1, 1, 0, 0, 1, 0, 0, T_NONE, 0, R_TOP, 0, 0},
    {"ds_write_b32", C_DSWRITE, VU, VU, NO, NO, 1, 1, 0, 0, 1, 0, 0, T_NONE, 0, R_NOEFFECT, 0, 0},
};
#define N_OPS ((int)(sizeof(OPS) / sizeof(OPS[0])))

int or_n_ops(void) { return N_OPS; }
const char *or_op_name(int id) { return (id >= 0 && id < N_OPS) ? OPS[id].name : 0; }

/* ------------------------------------------------------------------ */
/* validation                                                            */
/* ------------------------------------------------------------------ */
#define NONE_ID 0xFFFF
#define LIT_ID 0xFFFE

static int is_inline_const(unsigned id) { return (id >= 0x8000 && id <= 0x8050) || (id >= 0x8060 && id <= 0x8067); }

/* a scalar register operand of width w starting at id */
static int scalar_reg_ok(unsigned id, int w) {
    if (w == 1) return id <= 107 || id == 109;
    if (w == 2) return (id % 2 == 0) && (id <= 102 || id == 104 || id == 106);
    if (w == 4) return (id % 4 == 0) && id <= 100;
    return 0;
}
static int vector_reg_ok(unsigned id, int w) { return id >= 112 && id + (unsigned)w - 1 <= 367; }

static int field_ok(enum role r, unsigned id, int w, int lit_ok) {
    switch (r) {
    case NO: return id == NONE_ID;
    case SD: return scalar_reg_ok(id, w);
    case SU: return scalar_reg_ok(id, w);
    case SC: return scalar_reg_ok(id, w) || is_inline_const(id) || (lit_ok && id == LIT_ID);
    case VD: return vector_reg_ok(id, w);
    case VU: return vector_reg_ok(id, w);
    case VC: return vector_reg_ok(id, w) || scalar_reg_ok(id, w) || is_inline_const(id) || (lit_ok && id == LIT_ID);
    case SADDR: return id == NONE_ID || (scalar_reg_ok(id, 2) && id <= 102);
    }
    return 0;
}

/* status of one record at index i of a kernel with n records */
static int check_record(const or_instr *I, uint32_t n) {
    if (I->op >= N_OPS) return E_BADOP;
    const opinfo *o = &OPS[I->op];
    int imm_free = !o->imm_is_offset && o->src2 == NO;
    /* s_load destinations are plain SGPRs; sbase is an SGPR pair */
    if (o->cls == C_SMEM) {
        if (!(scalar_reg_ok(I->r0, o->w0) && I->r0 + (unsigned)o->w0 - 1 <= 103)) return E_BADREG;
        if (!(scalar_reg_ok(I->r1, 2) && I->r1 <= 102)) return E_BADREG;
        if (I->r2 != NONE_ID) return E_BADREG;
    } else {
        if (!field_ok(o->r0, I->r0, o->w0, 0)) return E_BADREG;
        if (!field_ok(o->r1, I->r1, o->w1, imm_free)) return E_BADREG;
        if (!field_ok(o->r2, I->r2, o->w2, imm_free)) return E_BADREG;
        if (o->src2 != NO) {
            if (I->imm < 0 || I->imm > 0xFFFF) return E_BADREG;
            if (!field_ok(o->src2, (unsigned)I->imm, o->w_src2, 0)) return E_BADREG;
        }
    }
    if (o->cls == C_BRANCH || o->cls == C_CBRANCH) {
        if (I->target < 0 || (uint32_t)I->target >= n) return E_BADTARGET;
    } else if (I->target != -1) {
        return E_BADTARGET;
    }
    return OK;
}

int or_check_record(const or_instr *I, uint32_t n) { return check_record(I, n); }

static int descriptor_status(const or_kernel *K) {
    if (K->useargs != 1) return E_UNSUPPORTED;          /* only the useargs ABI is described */
    if (K->dims < 1 || K->dims > 3) return E_UNSUPPORTED;
    for (int d = 0; d < K->dims; d++)
        if (K->cws[d] == 0) return E_UNSUPPORTED;
    if (K->n_args > 255) return E_UNSUPPORTED;
    return OK;
}

static int is_terminator(uint16_t op) {
    return op < N_OPS && (OPS[op].cls == C_BRANCH || OPS[op].cls == C_END);
}
static int ends_block(uint16_t op) {
    return op < N_OPS && (OPS[op].cls == C_BRANCH || OPS[op].cls == C_CBRANCH || OPS[op].cls == C_END);
}

/* status before the fixpoint: descriptor, then records in order, then end */
int or_kernel_status(const or_kernel *K, const or_instr *I) {
    int st = descriptor_status(K);
    if (st != OK) return st;
    for (uint32_t i = 0; i < K->n_instr; i++) {
        st = check_record(&I[i], K->n_instr);
        if (st != OK) return st;
    }
    if (K->n_instr == 0 || !is_terminator(I[K->n_instr - 1].op)) return E_NOEND;
    return OK;
}

/* ------------------------------------------------------------------ */
/* control flow graph (textbook basic blocks)                           */
/* ------------------------------------------------------------------ */
typedef struct {
    uint32_t n_blocks;
    uint32_t *block_start;   /* n_blocks + 1 */
    uint32_t *block_of;      /* per instruction */
    int32_t *succ;           /* 2 per block: fall-through, taken (or -1) */
    uint32_t *pred_off;      /* n_blocks + 1 */
    uint32_t *pred;          /* ascending per block */
    uint32_t *rpo;           /* reachable blocks in reverse postorder */
    uint32_t n_reach;
} cfg_t;

static void dfs_post(const cfg_t *G, uint32_t b, uint8_t *seen, uint32_t *post, uint32_t *np) {
    seen[b] = 1;
    for (int e = 0; e < 2; e++) {
        int32_t s = G->succ[2 * b + e];
        if (s >= 0 && !seen[s]) dfs_post(G, (uint32_t)s, seen, post, np);
    }
    post[(*np)++] = b;
}

static void build_cfg(const or_instr *I, uint32_t n, cfg_t *G) {
    uint8_t *leader = (uint8_t *)calloc(n + 1, 1);
    leader[0] = 1;
    for (uint32_t i = 0; i < n; i++) {
        if (OPS[I[i].op].cls == C_BRANCH || OPS[I[i].op].cls == C_CBRANCH) leader[I[i].target] = 1;
        if (ends_block(I[i].op) && i + 1 < n) leader[i + 1] = 1;
    }
    uint32_t nb = 0;
    for (uint32_t i = 0; i < n; i++) nb += leader[i];
    G->n_blocks = nb;
    G->block_start = (uint32_t *)malloc(sizeof(uint32_t) * (nb + 1));
    G->block_of = (uint32_t *)malloc(sizeof(uint32_t) * n);
    uint32_t b = 0;
    for (uint32_t i = 0; i < n; i++) {
        if (leader[i]) G->block_start[b++] = i;
        G->block_of[i] = b - 1;
    }
    G->block_start[nb] = n;
    G->succ = (int32_t *)malloc(sizeof(int32_t) * 2 * nb);
    for (b = 0; b < nb; b++) {
        uint32_t last = G->block_start[b + 1] - 1;
        const or_instr *L = &I[last];
        enum cls c = OPS[L->op].cls;
        int32_t fall = -1, taken = -1;
        if (c == C_END) {
        } else if (c == C_BRANCH) {
            taken = (int32_t)G->block_of[L->target];
        } else {
            if (b + 1 < nb) fall = (int32_t)(b + 1);
            if (c == C_CBRANCH) taken = (int32_t)G->block_of[L->target];
        }
        if (taken == fall) taken = -1;
        G->succ[2 * b] = fall;
        G->succ[2 * b + 1] = taken;
    }
    /* predecessors: for each block, every block that names it, ascending */
    G->pred_off = (uint32_t *)calloc(nb + 1, sizeof(uint32_t));
    for (b = 0; b < nb; b++)
        for (int e = 0; e < 2; e++)
            if (G->succ[2 * b + e] >= 0) G->pred_off[G->succ[2 * b + e] + 1]++;
    for (b = 0; b < nb; b++) G->pred_off[b + 1] += G->pred_off[b];
    G->pred = (uint32_t *)malloc(sizeof(uint32_t) * (G->pred_off[nb] + 1));
    uint32_t *fill = (uint32_t *)calloc(nb + 1, sizeof(uint32_t));
    for (uint32_t s = 0; s < nb; s++)           /* ascending scan over p gives ascending lists */
        for (uint32_t p = 0; p < nb; p++)
            if (G->succ[2 * p] == (int32_t)s || G->succ[2 * p + 1] == (int32_t)s)
                G->pred[G->pred_off[s] + fill[s]++] = p;
    free(fill);
    /* reverse postorder of a depth-first search from block 0, fall-through first */
    uint8_t *seen = (uint8_t *)calloc(nb, 1);
    uint32_t *post = (uint32_t *)malloc(sizeof(uint32_t) * nb);
    uint32_t np = 0;
    dfs_post(G, 0, seen, post, &np);
    G->rpo = (uint32_t *)malloc(sizeof(uint32_t) * (nb ? nb : 1));
    for (uint32_t i = 0; i < np; i++) G->rpo[i] = post[np - 1 - i];
    G->n_reach = np;
    free(seen);
    free(post);
    free(leader);
}

static void free_cfg(cfg_t *G) {
    free(G->block_start); free(G->block_of); free(G->succ); free(G->pred_off); free(G->pred); free(G->rpo);
}

/* ------------------------------------------------------------------ */
/* entry state (ABI initialisation)                                     */
/* ------------------------------------------------------------------ */
void or_entry_state(const or_kernel *K, or_slot *st) {
    memset(st, 0, sizeof(or_slot) * NSLOT);
    for (int s = 0; s < NSLOT; s++) {
        st[s].prov = P_UNINIT;
        st[s].val = mk(UNINIT, 0, 0, 0, 0, 0, 0);
    }
    /* s[4:5]: pointer to the kernel settings / arguments */
    st[4].prov = P_SYSPTR; st[4].type = 0; st[4].val = mk(SYSPTR, LOW, 0, 0, 0, 0, 0);
    st[5].prov = P_SYSPTR; st[5].type = 0; st[5].val = mk(SYSPTR, HIGH, 0, 0, 0, 0, 0);
    for (int d = 0; d < K->dims; d++) {
        /* s6.. : work-group ids; v0.. : local ids */
        st[6 + d].prov = P_WGID(d); st[6 + d].type = TY_UINT; st[6 + d].val = mk(WGID, ENTIRE, (unsigned)d, 0, 0, 0, 0);
        st[112 + d].prov = P_LID(d); st[112 + d].type = TY_UINT; st[112 + d].val = mk(IDX, ENTIRE, (unsigned)d, M_LID, 0, 0, 0);
    }
    st[106].prov = P_MASK; st[106].type = 0; st[106].val = TOP;
    st[107].prov = P_MASK; st[107].type = 0; st[107].val = TOP;
}

/* ------------------------------------------------------------------ */
/* operand reads                                                         */
/* ------------------------------------------------------------------ */
static const uint32_t FLOAT_BITS[8] = {0x3F000000u, 0xBF000000u, 0x3F800000u, 0xBF800000u,
                                       0x40000000u, 0xC0000000u, 0x40800000u, 0xC0800000u};
static const uint32_t DOUBLE_HI_BITS[8] = {0x3FE00000u, 0xBFE00000u, 0x3FF00000u, 0xBFF00000u,
                                           0x40000000u, 0xC0000000u, 0x40100000u, 0xC0100000u};

/* dword j of operand `id` used as a w-dword source */
static or_slot read_op(const or_slot *st, unsigned id, int j, int w, int32_t imm) {
    or_slot s;
    memset(&s, 0, sizeof(s));
    if (id < NSLOT) return st[id + (unsigned)j];
    s.prov = P_CONST;
    s.type = 0;
    if (id >= 0x8000 && id <= 0x8050) {
        int32_t v = (int32_t)(id - 0x8000) - 16;
        s.val = CONST32(j == 0 ? (uint32_t)v : (v < 0 ? 0xFFFFFFFFu : 0u));
    } else if (id >= 0x8060 && id <= 0x8067) {
        unsigned q = id - 0x8060;
        if (w == 1) s.val = CONST32(FLOAT_BITS[q]);
        else s.val = CONST32(j == 0 ? 0u : DOUBLE_HI_BITS[q]);
    } else { /* literal */
        s.val = CONST32(j == 0 ? (uint32_t)imm : (imm < 0 ? 0xFFFFFFFFu : 0u));
    }
    return s;
}

/* ------------------------------------------------------------------ */
/* payload rules                                                         */
/* ------------------------------------------------------------------ */
static int idx_lowish(uint64_t v) { return v != TOP && tag_of(v) == IDX && (integ_of(v) == ENTIRE || integ_of(v) == LOW); }

static uint64_t add_once(uint64_t a, uint64_t b) {
    /* patterns tried with a on the left; add_rule tries both orders */
    if (is_const(a) && is_const(b)) return CONST32(c_of(a) + c_of(b));
    if (idx_lowish(a) && idx_lowish(b) && dim_of(a) == dim_of(b) && (aux_of(a) & aux_of(b)) == 0)
        return mk(IDX, ENTIRE, dim_of(a), aux_of(a) | aux_of(b), 0, 0, c_of(a) + c_of(b));
    if (idx_lowish(a) && is_const(b)) return mk(IDX, ENTIRE, dim_of(a), aux_of(a), 0, 0, c_of(a) + c_of(b));
    if (tag_of(a) == SHL && integ_of(a) == ENTIRE && is_const(b))
        return mk(SHL, ENTIRE, dim_of(a), aux_of(a), shift_of(a), 0, c_of(a) + c_of(b));
    if (tag_of(a) == KARG && integ_of(a) == LOW && tag_of(b) == SHL && integ_of(b) == LOW)
        return mk(PTR, LOW, dim_of(b), aux_of(b), shift_of(b), arg_of(a), c_of(b));
    if (tag_of(a) == KARG && integ_of(a) == LOW && is_const(b)) return mk(PTR, LOW, 0, 0, 0, arg_of(a), c_of(b));
    if (tag_of(a) == PTR && integ_of(a) == LOW && is_const(b))
        return mk(PTR, LOW, dim_of(a), aux_of(a), shift_of(a), arg_of(a), c_of(a) + c_of(b));
    if (tag_of(a) == PTR && integ_of(a) == LOW && dim_of(a) == 0 && aux_of(a) == 0 && shift_of(a) == 0 &&
        tag_of(b) == SHL && integ_of(b) == LOW)
        return mk(PTR, LOW, dim_of(b), aux_of(b), shift_of(b), arg_of(a), c_of(a) + c_of(b));
    return TOP;
}
static uint64_t add_rule(uint64_t a, uint64_t b) {
    if (a == TOP || b == TOP) return TOP;
    uint64_t r = add_once(a, b);
    return r != TOP ? r : add_once(b, a);
}

static uint64_t addc_rule(uint64_t a, uint64_t b) {
    if (a == TOP || b == TOP) return TOP;
    for (int k = 0; k < 2; k++) {
        uint64_t p = k ? b : a, q = k ? a : b;
        int ptr_hi = (tag_of(p) == KARG || tag_of(p) == PTR) && integ_of(p) == HIGH;
        int ext_hi = (tag_of(q) == SHL && integ_of(q) == HIGH) || (tag_of(q) == IDX && integ_of(q) == HIGH) ||
                     (is_const(q) && c_of(q) == 0);
        if (ptr_hi && ext_hi) return mk(PTR, HIGH, 0, 0, 0, arg_of(p), 0);
    }
    return TOP;
}

static int log2_exact(uint32_t x, unsigned *s) {
    if (x == 0 || (x & (x - 1))) return 0;
    unsigned k = 0;
    while ((1u << k) != x) k++;
    *s = k;
    return 1;
}

/* IDX(d,m,c) shifted left by s (s already reduced) */
static uint64_t idx_shift(uint64_t a, unsigned s) {
    if (s == 0) return mk(IDX, ENTIRE, dim_of(a), aux_of(a), 0, 0, c_of(a));
    if (s > 15) return TOP;
    return mk(SHL, ENTIRE, dim_of(a), aux_of(a), s, 0, c_of(a) << s);
}

static uint64_t mul_once(const or_kernel *K, uint64_t a, uint64_t b) {
    if (is_const(a) && is_const(b)) return CONST32(c_of(a) * c_of(b));
    if (tag_of(a) == WGID && is_const(b)) {
        unsigned d = dim_of(a);
        if (K->cws[d] > 0 && c_of(b) == K->cws[d]) return mk(IDX, ENTIRE, d, M_WG, 0, 0, 0);
        return TOP;
    }
    if (idx_lowish(a) && is_const(b)) {
        unsigned s;
        if (log2_exact(c_of(b), &s)) return idx_shift(a, s);
    }
    return TOP;
}
static uint64_t mul_rule(const or_kernel *K, uint64_t a, uint64_t b) {
    if (a == TOP || b == TOP) return TOP;
    uint64_t r = mul_once(K, a, b);
    return r != TOP ? r : mul_once(K, b, a);
}
static uint64_t mask24(uint64_t v) { return is_const(v) ? CONST32(c_of(v) & 0xFFFFFFu) : v; }

static uint64_t shl32_rule(const or_kernel *K, uint64_t val, uint64_t amt) {
    if (val == TOP || amt == TOP || !is_const(amt)) return TOP;
    unsigned s = c_of(amt) & 31;
    if (is_const(val)) return CONST32(c_of(val) << s);
    if (idx_lowish(val)) return idx_shift(val, s);
    if (tag_of(val) == WGID) {
        unsigned d = dim_of(val), lg;
        if (log2_exact(K->cws[d], &lg) && lg == s) return mk(IDX, ENTIRE, d, M_WG, 0, 0, 0);
    }
    return TOP;
}

static uint64_t lshr32_rule(const or_kernel *K, uint64_t val, uint64_t amt) {
    if (val == TOP || amt == TOP || !is_const(amt)) return TOP;
    unsigned s = c_of(amt) & 31;
    if (is_const(val)) return CONST32(c_of(val) >> s);
    if (tag_of(val) == SYS && aux_of(val) == SYS_GSIZE && integ_of(val) == ENTIRE) {
        unsigned d = dim_of(val), lg;
        if (log2_exact(K->cws[d], &lg) && lg == s) return mk(SYS, ENTIRE, d, SYS_NUMGROUPS, 0, 0, 0);
    }
    return TOP;
}

static uint64_t ashr_rule(uint64_t val, uint64_t amt) {
    if (val == TOP || amt == TOP || !is_const(amt)) return TOP;
    unsigned s = c_of(amt) & 31;
    if (is_const(val)) return CONST32((uint32_t)((int32_t)c_of(val) >> s));
    if (idx_lowish(val) && s == 31) return mk(IDX, HIGH, dim_of(val), aux_of(val), 0, 0, 0);
    return TOP;
}

static uint64_t fold_rule(enum prule r, uint64_t a, uint64_t b) {
    if (!is_const(a) || !is_const(b)) return TOP;
    uint32_t x = c_of(a), y = c_of(b);
    switch (r) {
    case R_SUB: return CONST32(x - y);
    case R_AND: return CONST32(x & y);
    case R_OR: return CONST32(x | y);
    case R_XOR: return CONST32(x ^ y);
    default: return TOP;
    }
}

/* ------------------------------------------------------------------ */
/* s_load resolution against the kernel-argument area                   */
/* ------------------------------------------------------------------ */
typedef struct { uint32_t prov; uint8_t type; uint64_t val; } dword_info;

static dword_info resolve_dword(const or_kernel *K, const or_arg *args, uint32_t o) {
    dword_info r = {P_LOADG, 0, TOP};
    if (o < 0x18 && o % 4 == 0) {                 /* global offsets 0..2, 8 bytes each */
        unsigned g = o / 8, half = (o / 4) & 1;
        r.prov = P_GOFF(g); r.type = TY_UINT;
        r.val = half == 0 ? mk(IDX, LOW, g, M_GOFF, 0, 0, 0) : mk(SYS, HIGH, g, SYS_GOFF_HI, 0, 0, 0);
        return r;
    }
    if (o >= 0x18 && o < 0x30 && o % 4 == 0) {    /* printf buffer, vqueue, aqlwrap */
        unsigned h = (o - 0x18) / 8, half = (o / 4) & 1;
        r.prov = P_HIDDEN; r.type = 0;
        r.val = mk(SYS, half == 0 ? LOW : HIGH, h, SYS_HIDDEN, 0, 0, 0);
        return r;
    }
    if (o == 0x20010) {
        r.prov = P_WORKDIM; r.type = TY_UINT; r.val = mk(SYS, ENTIRE, 0, SYS_WORKDIM, 0, 0, 0);
        return r;
    }
    for (unsigned k = 0; k < K->n_args; k++) {
        const or_arg *a = &args[k];
        if ((uint64_t)a->offset <= o && (uint64_t)o < (uint64_t)a->offset + a->size) {
            r.prov = P_KARG(k);
            r.type = a->type;
            if (a->size == 4 && o == a->offset) r.val = mk(KARG, ENTIRE, 0, 0, 0, k, 0);
            else if (a->size == 8 && o == a->offset) r.val = mk(KARG, LOW, 0, 0, 0, k, 0);
            else if (a->size == 8 && o == a->offset + 4) r.val = mk(KARG, HIGH, 0, 0, 0, k, 0);
            else r.val = TOP;
            return r;
        }
    }
    return r;
}

/* ------------------------------------------------------------------ */
/* one instruction                                                       */
/* ------------------------------------------------------------------ */
typedef struct { unsigned slot; or_slot v; } def_t;

/* Computes the defs of instruction I from state st (which it does not
 * modify).  Returns the number of defs; explicit defs come first, then
 * implicit ones, so writing them in order lets implicit defs win. */
static int compute_defs(const or_kernel *K, const or_arg *args, const or_instr *I, const or_slot *st, def_t *defs) {
    const opinfo *o = &OPS[I->op];
    int nd = 0;
    if (o->cls == C_BRANCH || o->cls == C_CBRANCH || o->cls == C_NOP || o->cls == C_END ||
        o->cls == C_GSTORE || o->cls == C_FSTORE || o->cls == C_DSWRITE)
        return 0;

    if (o->cls == C_SMEM) {
        int w = o->w0;
        int via_ptr = I->r1 == 4;
        int ptr_ok = st[4].val == mk(SYSPTR, LOW, 0, 0, 0, 0, 0) && st[5].val == mk(SYSPTR, HIGH, 0, 0, 0, 0, 0);
        uint32_t off = (uint32_t)I->imm;
        dword_info di[4];
        for (int j = 0; j < w; j++) {
            if (via_ptr) di[j] = resolve_dword(K, args, off + 4u * (uint32_t)j);
            else { di[j].prov = P_LOADG; di[j].type = 0; di[j].val = TOP; }
        }
        if (via_ptr) {   /* exact (offset, width) matches take precedence */
            if (w == 2 && (off == 0x0 || off == 0x8 || off == 0x10)) {
                unsigned d = off / 8;
                di[0].prov = di[1].prov = P_GOFF(d);
                di[0].type = di[1].type = TY_UINT;
                di[0].val = mk(IDX, LOW, d, M_GOFF, 0, 0, 0);
                di[1].val = mk(SYS, HIGH, d, SYS_GOFF_HI, 0, 0, 0);
            }
            if (w == 1 && (off == 0xc || off == 0x10 || off == 0x14)) {
                unsigned d = (off - 0xc) / 4;
                di[0].prov = P_GSIZE(d); di[0].type = TY_UINT; di[0].val = mk(SYS, ENTIRE, d, SYS_GSIZE, 0, 0, 0);
            }
            if (w == 1 && off == 0x20010) {
                di[0].prov = P_WORKDIM; di[0].type = TY_UINT; di[0].val = mk(SYS, ENTIRE, 0, SYS_WORKDIM, 0, 0, 0);
            }
        }
        for (int j = 0; j < w; j++) {
            defs[nd].slot = I->r0 + (unsigned)j;
            memset(&defs[nd].v, 0, sizeof(or_slot));
            defs[nd].v.prov = di[j].prov;
            defs[nd].v.type = di[j].type;
            defs[nd].v.val = (via_ptr && ptr_ok) ? di[j].val : TOP;
            nd++;
        }
        return nd;
    }

    if (o->cls == C_GLOAD || o->cls == C_FLOAD || o->cls == C_DSREAD) {
        for (int j = 0; j < o->w0; j++) {
            defs[nd].slot = I->r0 + (unsigned)j;
            memset(&defs[nd].v, 0, sizeof(or_slot));
            defs[nd].v.prov = o->cls == C_DSREAD ? P_LOADL : P_LOADG;
            defs[nd].v.val = TOP;
            nd++;
        }
        return nd;
    }

    /* ALU and compares: gather every source dword first */
    or_slot s1[2], s2[2], s3[2];
    int n1 = 0, n2 = 0, n3 = 0;
    uint32_t rp = 0;
    if (o->r1 != NO) { n1 = o->w1; for (int j = 0; j < n1; j++) s1[j] = read_op(st, I->r1, j, o->w1, I->imm); }
    if (o->r2 != NO) { n2 = o->w2; for (int j = 0; j < n2; j++) s2[j] = read_op(st, I->r2, j, o->w2, I->imm); }
    if (o->src2 != NO) { n3 = o->w_src2; for (int j = 0; j < n3; j++) s3[j] = read_op(st, (unsigned)I->imm, j, o->w_src2, 0); }
    for (int j = 0; j < n1; j++) rp |= s1[j].prov;
    for (int j = 0; j < n2; j++) rp |= s2[j].prov;
    for (int j = 0; j < n3; j++) rp |= s3[j].prov;
    if (o->imp_use & I_VCC) rp |= st[104].prov | st[105].prov;
    if (o->imp_use & I_EXEC) rp |= st[106].prov | st[107].prov;
    if (o->imp_use & I_SCC) rp |= st[108].prov;

    if (o->r0 == SD || o->r0 == VD) {
        int w = o->w0;
        uint8_t ty[2] = {0, 0};
        uint8_t src_types = 0;
        for (int j = 0; j < n1; j++) if (o->value_srcs & 1) src_types |= s1[j].type;
        for (int j = 0; j < n2; j++) if (o->value_srcs & 2) src_types |= s2[j].type;
        switch (o->trule) {
        case T_NONE: break;
        case T_SUF: ty[0] = ty[1] = (uint8_t)o->suffix; break;
        case T_ADD: {
            uint8_t u = 0;
            for (int j = 0; j < n1; j++) u |= s1[j].type;
            for (int j = 0; j < n2; j++) u |= s2[j].type;
            ty[0] = ty[1] = (uint8_t)(o->suffix | (u & TY_PTR));
            break;
        }
        case T_B: ty[0] = ty[1] = src_types; break;
        case T_MOVE: ty[0] = s1[0].type; ty[1] = w == 2 ? s1[1].type : 0; break;
        case T_SMEM: break;
        }
        uint64_t v[2] = {TOP, TOP};
        uint64_t a = n1 ? s1[0].val : TOP, b = n2 ? s2[0].val : TOP;
        switch (o->prule) {
        case R_TOP: case R_NOEFFECT: case R_SMEM: break;
        case R_MOV: v[0] = s1[0].val; v[1] = w == 2 ? s1[1].val : TOP; break;
        case R_ADD: v[0] = add_rule(a, b); break;
        case R_ADDC: v[0] = addc_rule(a, b); break;
        case R_SUB: case R_AND: case R_OR: case R_XOR: v[0] = fold_rule(o->prule, a, b); break;
        case R_MUL: v[0] = mul_rule(K, a, b); break;
        case R_MUL24: v[0] = mul_rule(K, mask24(a), mask24(b)); break;
        case R_MAD24: v[0] = add_rule(mul_rule(K, mask24(a), mask24(b)), s3[0].val); break;
        /* shifts: the value is r1 in the scalar forms, r2 in the vector "rev" forms */
        case R_SHL32: v[0] = o->value_srcs == 1 ? shl32_rule(K, a, b) : shl32_rule(K, b, a); break;
        case R_LSHR32: v[0] = o->value_srcs == 1 ? lshr32_rule(K, a, b) : lshr32_rule(K, b, a); break;
        case R_ASHR: v[0] = o->value_srcs == 1 ? ashr_rule(a, b) : ashr_rule(b, a); break;
        case R_SEL: v[0] = (a == b) ? a : TOP; break;
        case R_FOLD64_AND: case R_FOLD64_OR: case R_FOLD64_XOR: case R_FOLD64_ANDN2: {
            if (is_const(s1[0].val) && is_const(s1[1].val) && is_const(s2[0].val) && is_const(s2[1].val)) {
                for (int j = 0; j < 2; j++) {
                    uint32_t x = c_of(s1[j].val), y = c_of(s2[j].val), z;
                    if (o->prule == R_FOLD64_AND) z = x & y;
                    else if (o->prule == R_FOLD64_OR) z = x | y;
                    else if (o->prule == R_FOLD64_XOR) z = x ^ y;
                    else z = x & ~y;
                    v[j] = CONST32(z);
                }
            }
            break;
        }
        case R_SHL64: {
            uint64_t amt = s1[0].val, lo = s2[0].val, hi = s2[1].val;
            if (amt == TOP || lo == TOP || hi == TOP || !is_const(amt)) break;
            unsigned s = c_of(amt) & 63;
            if (is_const(lo) && is_const(hi)) {
                uint64_t x = ((uint64_t)c_of(hi) << 32 | c_of(lo)) << s;
                v[0] = CONST32((uint32_t)x);
                v[1] = CONST32((uint32_t)(x >> 32));
            } else if (idx_lowish(lo) &&
                       ((is_const(hi) && c_of(hi) == 0) ||
                        (tag_of(hi) == IDX && integ_of(hi) == HIGH && dim_of(hi) == dim_of(lo) && aux_of(hi) == aux_of(lo)))) {
                if (s == 0) { v[0] = lo; v[1] = hi; }
                else if (s <= 15) {
                    v[0] = mk(SHL, LOW, dim_of(lo), aux_of(lo), s, 0, c_of(lo) << s);
                    v[1] = mk(SHL, HIGH, dim_of(lo), aux_of(lo), s, 0, 0);
                }
            }
            break;
        }
        }
        for (int j = 0; j < w; j++) {
            defs[nd].slot = I->r0 + (unsigned)j;
            memset(&defs[nd].v, 0, sizeof(or_slot));
            defs[nd].v.prov = rp | (o->mask_def ? P_MASK : 0);
            defs[nd].v.type = ty[j];
            defs[nd].v.val = v[j];
            nd++;
        }
    }
    /* implicit defs: masks and condition codes carry no value */
    unsigned imp[5];
    int ni = 0;
    if (o->imp_def & I_VCC) { imp[ni++] = 104; imp[ni++] = 105; }
    if (o->imp_def & I_EXEC) { imp[ni++] = 106; imp[ni++] = 107; }
    if (o->imp_def & I_SCC) imp[ni++] = 108;
    for (int j = 0; j < ni; j++) {
        defs[nd].slot = imp[j];
        memset(&defs[nd].v, 0, sizeof(or_slot));
        defs[nd].v.prov = rp | P_MASK;
        defs[nd].v.type = 0;
        defs[nd].v.val = TOP;
        nd++;
    }
    return nd;
}

static void apply(const or_kernel *K, const or_arg *args, const or_instr *I, or_slot *st) {
    def_t defs[16];
    int nd = compute_defs(K, args, I, st, defs);
    for (int j = 0; j < nd; j++) st[defs[j].slot] = defs[j].v;
}

/* exported for property tests: apply one instruction in place */
void or_transfer(const or_kernel *K, const or_arg *args, const or_instr *I, or_slot *st) { apply(K, args, I, st); }

/* ------------------------------------------------------------------ */
/* join                                                                  */
/* ------------------------------------------------------------------ */
static void join_into(or_slot *dst, const or_slot *src) {
    for (int s = 0; s < NSLOT; s++) {
        dst[s].prov |= src[s].prov;
        dst[s].type |= src[s].type;
        if (dst[s].val != src[s].val) dst[s].val = TOP;
    }
}
void or_join(or_slot *dst, const or_slot *src) { join_into(dst, src); }

static int state_eq(const or_slot *a, const or_slot *b) { return memcmp(a, b, sizeof(or_slot) * NSLOT) == 0; }

/* ------------------------------------------------------------------ */
/* extraction                                                            */
/* ------------------------------------------------------------------ */
static int sysval_kind(uint64_t v, unsigned *kind, unsigned *dim) {
    if (v == TOP) return 0;
    unsigned t = tag_of(v), ig = integ_of(v), m = aux_of(v), d = dim_of(v);
    *dim = d;
    if (t == IDX && c_of(v) == 0) {
        if (ig == ENTIRE && m == (M_WG | M_LID | M_GOFF)) { *kind = SV_GLOBAL_ID; return 1; }
        if (ig == ENTIRE && m == (M_WG | M_LID)) { *kind = SV_GLOBAL_ID_MINUS_OFFSET; return 1; }
        if (ig == LOW && m == M_GOFF) { *kind = SV_GLOBAL_OFFSET; return 1; }
        if (ig == ENTIRE && m == M_WG) { *kind = SV_GROUP_BASE; return 1; }
        if (ig == ENTIRE && m == M_LID) { *kind = SV_LOCAL_ID; return 1; }
    }
    if (t == SYS && ig == ENTIRE) {
        if (m == SYS_GSIZE) { *kind = SV_GLOBAL_SIZE; return 1; }
        if (m == SYS_NUMGROUPS) { *kind = SV_NUM_GROUPS; return 1; }
        if (m == SYS_WORKDIM) { *kind = SV_WORK_DIM; *dim = 0; return 1; }
    }
    if (t == WGID) { *kind = SV_GROUP_ID; return 1; }
    return 0;
}

static uint64_t global_address(const or_instr *I, const or_slot *st) {
    if (I->r2 != NONE_ID) return TOP;
    uint64_t lo = st[I->r1].val, hi = st[I->r1 + 1].val;
    if (lo == TOP || hi == TOP) return TOP;
    if (tag_of(lo) == PTR && integ_of(lo) == LOW && tag_of(hi) == PTR && integ_of(hi) == HIGH && arg_of(lo) == arg_of(hi))
        return mk(PTR, ENTIRE, dim_of(lo), aux_of(lo), shift_of(lo), arg_of(lo), c_of(lo) + (uint32_t)I->imm);
    if (tag_of(lo) == KARG && integ_of(lo) == LOW && tag_of(hi) == KARG && integ_of(hi) == HIGH && arg_of(lo) == arg_of(hi))
        return mk(PTR, ENTIRE, 0, 0, 0, arg_of(lo), (uint32_t)I->imm);
    return TOP;
}

static uint64_t lds_address(const or_instr *I, const or_slot *st) {
    uint64_t v = st[I->r1].val;
    if (v == TOP) return TOP;
    uint32_t c = c_of(v) + (uint32_t)I->imm;
    if (tag_of(v) == SHL && integ_of(v) == ENTIRE) return mk(SHL, ENTIRE, dim_of(v), aux_of(v), shift_of(v), 0, c);
    if (idx_lowish(v)) return mk(IDX, ENTIRE, dim_of(v), aux_of(v), 0, 0, c);
    if (is_const(v)) return CONST32(c);
    return TOP;
}

/* emit the access record of a memory instruction at pre-state st */
static int make_access(const or_kernel *K, const or_arg *args, const or_instr *I, uint32_t idx, const or_slot *st, or_access *out) {
    const opinfo *o = &OPS[I->op];
    memset(out, 0, sizeof(*out));
    out->instr = idx;
    switch (o->cls) {
    case C_GLOAD: case C_FLOAD: case C_GSTORE: case C_FSTORE:
        out->kind = (o->cls == C_GLOAD || o->cls == C_FLOAD) ? AK_LOAD : AK_STORE;
        out->space = (o->cls == C_GLOAD || o->cls == C_GSTORE) ? SP_GLOBAL : SP_FLAT;
        out->width = (uint8_t)(4 * o->w0);
        out->addr = global_address(I, st);
        break;
    case C_DSREAD: case C_DSWRITE:
        out->kind = o->cls == C_DSREAD ? AK_LOAD : AK_STORE;
        out->space = SP_LDS;
        out->width = 4;
        out->addr = lds_address(I, st);
        break;
    default:
        return 0;
    }
    if (out->kind == AK_STORE) {
        uint8_t t = 0;
        for (int j = 0; j < o->w0; j++) t |= st[I->r0 + (unsigned)j].type;
        out->dtype = t;
    } else if (out->addr != TOP && tag_of(out->addr) == PTR && arg_of(out->addr) < K->n_args) {
        out->dtype = (uint8_t)(args[arg_of(out->addr)].flags & 31);
    }
    return 1;
}

/* ------------------------------------------------------------------ */
/* digest of the fixpoint states                                         */
/* ------------------------------------------------------------------ */
static uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
static uint64_t states_digest(uint32_t nb, const or_slot *IN, const uint8_t *reached) {
    uint64_t h = 0;
    for (uint32_t b = 0; b < nb; b++) {
        if (!reached[b]) continue;
        h += mix64(0xB10C0000ull + b);
        for (uint32_t s = 0; s < NSLOT; s++) {
            const or_slot *x = &IN[(size_t)b * NSLOT + s];
            uint64_t z = mix64(x->val + 0x9E3779B97F4A7C15ull * ((uint64_t)b * NSLOT + s + 1));
            h += mix64(z ^ ((uint64_t)x->prov | ((uint64_t)x->type << 32)));
        }
    }
    return h;
}

/* ------------------------------------------------------------------ */
/* the analysis of one kernel                                           */
/* ------------------------------------------------------------------ */
typedef struct {
    int32_t status;
    uint32_t n_blocks, n_reach, sweeps, n_acc, n_sys, n_pred;
    uint64_t digest;
    /* caller buffers (capacities: n_instr+1, 2*(n_instr), n_instr+1, 2*n_instr, n_instr,
     * n_instr*368 slots or NULL, n_instr, n_instr, 4*n_instr) */
    uint32_t *block_start;
    int32_t *succ;
    uint32_t *pred_off;
    uint32_t *pred;
    uint32_t *rpo;
    or_slot *in_states;
    uint8_t *reached;
    or_access *acc;
    or_sysval *sys;
} or_result;

static void apply_block(const or_kernel *K, const or_arg *args, const or_instr *I, const cfg_t *G, uint32_t b, or_slot *st) {
    for (uint32_t i = G->block_start[b]; i < G->block_start[b + 1]; i++) apply(K, args, &I[i], st);
}

/* next-state pseudo-random generator for worklist shuffles (splitmix64) */
static uint64_t sm_next(uint64_t *s) {
    uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
    return mix64(z);
}

/*
 * schedule 0: round-robin passes over the reverse postorder, IN[b] pulled
 *             from the reached predecessors (the reference; defines `sweeps`:
 *             the number of passes in which some block's IN changed).
 * schedule 1: FIFO worklist, IN[s] joined as each predecessor finishes.
 * schedule 2: worklist that pops a uniformly random queued block (seeded).
 */
int or_analyze(const or_kernel *K, const or_instr *I, const or_arg *args, uint32_t sweep_cap, int schedule,
               uint64_t seed, or_result *R) {
    R->status = or_kernel_status(K, I);
    R->n_blocks = R->n_reach = R->sweeps = R->n_acc = R->n_sys = R->n_pred = 0;
    R->digest = 0;
    if (R->status != OK) return R->status;
    uint32_t n = K->n_instr;
    cfg_t G;
    build_cfg(I, n, &G);
    uint32_t nb = G.n_blocks;
    or_slot *IN = (or_slot *)calloc((size_t)nb * NSLOT, sizeof(or_slot));
    or_slot *OUT = (or_slot *)calloc((size_t)nb * NSLOT, sizeof(or_slot));
    uint8_t *reached = (uint8_t *)calloc(nb, 1);
    or_slot entry[NSLOT], tmp[NSLOT];
    or_entry_state(K, entry);
    uint32_t cap = sweep_cap ? sweep_cap : 64 + 2 * nb;
    uint32_t sweeps = 0;
    int status = OK;

    if (schedule == 0) {
        for (;;) {
            int changed = 0;
            for (uint32_t r = 0; r < G.n_reach; r++) {
                uint32_t b = G.rpo[r];
                int any = 0;
                if (b == 0) { memcpy(tmp, entry, sizeof(tmp)); any = 1; }
                for (uint32_t q = G.pred_off[b]; q < G.pred_off[b + 1]; q++) {
                    uint32_t p = G.pred[q];
                    if (!reached[p]) continue;
                    if (!any) { memcpy(tmp, &OUT[(size_t)p * NSLOT], sizeof(tmp)); any = 1; }
                    else join_into(tmp, &OUT[(size_t)p * NSLOT]);
                }
                if (!any) continue;
                if (!reached[b] || !state_eq(tmp, &IN[(size_t)b * NSLOT])) {
                    memcpy(&IN[(size_t)b * NSLOT], tmp, sizeof(tmp));
                    reached[b] = 1;
                    changed = 1;
                    memcpy(&OUT[(size_t)b * NSLOT], tmp, sizeof(tmp));
                    apply_block(K, args, I, &G, b, &OUT[(size_t)b * NSLOT]);
                }
            }
            if (!changed) break;
            sweeps++;
            if (sweeps > cap) { status = E_NOFIX; break; }
        }
    } else {
        /* worklist: IN[0] = entry; push-style joins */
        uint32_t *queue = (uint32_t *)malloc(sizeof(uint32_t) * (nb + 1));
        uint8_t *queued = (uint8_t *)calloc(nb, 1);
        uint32_t qh = 0, qn = 0;   /* circular FIFO of at most nb entries */
        uint64_t rs = seed;
        uint64_t visits = 0, visit_cap = (uint64_t)(cap + 1) * nb * 64 + 1024;
        memcpy(&IN[0], entry, sizeof(entry));
        reached[0] = 1;
        queue[0] = 0; qn = 1; queued[0] = 1;
        while (qn) {
            uint32_t b;
            if (schedule == 2) {
                uint32_t k = (uint32_t)(sm_next(&rs) % qn);
                uint32_t pos = (qh + k) % nb;
                b = queue[pos];
                queue[pos] = queue[qh];
            } else {
                b = queue[qh];
            }
            qh = (qh + 1) % nb;
            qn--;
            queued[b] = 0;
            if (++visits > visit_cap) { status = E_NOFIX; break; }
            memcpy(&OUT[(size_t)b * NSLOT], &IN[(size_t)b * NSLOT], sizeof(tmp));
            apply_block(K, args, I, &G, b, &OUT[(size_t)b * NSLOT]);
            for (int e = 0; e < 2; e++) {
                int32_t s = G.succ[2 * b + e];
                if (s < 0) continue;
                or_slot *dst = &IN[(size_t)s * NSLOT];
                int upd;
                if (!reached[s]) {
                    memcpy(dst, &OUT[(size_t)b * NSLOT], sizeof(tmp));
                    if (s == 0) join_into(dst, entry);
                    reached[s] = 1;
                    upd = 1;
                } else {
                    memcpy(tmp, dst, sizeof(tmp));
                    join_into(dst, &OUT[(size_t)b * NSLOT]);
                    upd = !state_eq(tmp, dst);
                }
                if (upd && !queued[s]) {
                    queue[(qh + qn) % nb] = (uint32_t)s;
                    qn++;
                    queued[s] = 1;
                }
            }
        }
        free(queue);
        free(queued);
        sweeps = 0;   /* not defined for worklist schedules */
    }

    if (status == OK) {
        /* fixpoint check: each reached IN equals the join of its inputs */
        for (uint32_t b = 0; b < nb; b++) {
            if (!reached[b]) continue;
            int any = 0;
            if (b == 0) { memcpy(tmp, entry, sizeof(tmp)); any = 1; }
            for (uint32_t q = G.pred_off[b]; q < G.pred_off[b + 1]; q++) {
                uint32_t p = G.pred[q];
                if (!reached[p]) continue;
                or_slot o2[NSLOT];
                memcpy(o2, &IN[(size_t)p * NSLOT], sizeof(o2));
                apply_block(K, args, I, &G, p, o2);
                if (!any) { memcpy(tmp, o2, sizeof(tmp)); any = 1; }
                else join_into(tmp, o2);
            }
            if (!any || !state_eq(tmp, &IN[(size_t)b * NSLOT])) { status = -99; break; }
        }
    }

    R->status = status;
    if (status == OK) {
        R->n_blocks = nb;
        R->n_reach = G.n_reach;
        R->sweeps = sweeps;
        R->n_pred = G.pred_off[nb];
        if (R->block_start) memcpy(R->block_start, G.block_start, sizeof(uint32_t) * (nb + 1));
        if (R->succ) memcpy(R->succ, G.succ, sizeof(int32_t) * 2 * nb);
        if (R->pred_off) memcpy(R->pred_off, G.pred_off, sizeof(uint32_t) * (nb + 1));
        if (R->pred) memcpy(R->pred, G.pred, sizeof(uint32_t) * G.pred_off[nb]);
        if (R->rpo) memcpy(R->rpo, G.rpo, sizeof(uint32_t) * G.n_reach);
        if (R->reached) memcpy(R->reached, reached, nb);
        for (uint32_t b = 0; b < nb; b++)
            if (!reached[b]) memset(&IN[(size_t)b * NSLOT], 0, sizeof(or_slot) * NSLOT);
        if (R->in_states) memcpy(R->in_states, IN, sizeof(or_slot) * NSLOT * nb);
        R->digest = states_digest(nb, IN, reached);
        /* extraction: reached blocks in index order, from their IN states */
        uint32_t na = 0, ns = 0;
        for (uint32_t b = 0; b < nb; b++) {
            if (!reached[b]) continue;
            memcpy(tmp, &IN[(size_t)b * NSLOT], sizeof(tmp));
            for (uint32_t i = G.block_start[b]; i < G.block_start[b + 1]; i++) {
                or_access a;
                if (make_access(K, args, &I[i], i, tmp, &a)) { if (R->acc) R->acc[na] = a; na++; }
                def_t defs[16];
                int nd = compute_defs(K, args, &I[i], tmp, defs);
                for (int j = 0; j < nd; j++) tmp[defs[j].slot] = defs[j].v;
                /* distinct def slots, ascending */
                unsigned slots[16];
                int nslots = 0;
                for (int j = 0; j < nd; j++) {
                    int dup = 0;
                    for (int q = 0; q < nslots; q++) if (slots[q] == defs[j].slot) dup = 1;
                    if (!dup) slots[nslots++] = defs[j].slot;
                }
                for (int x = 1; x < nslots; x++)
                    for (int y = x; y > 0 && slots[y - 1] > slots[y]; y--) { unsigned t = slots[y]; slots[y] = slots[y - 1]; slots[y - 1] = t; }
                for (int q = 0; q < nslots; q++) {
                    unsigned kind, dim;
                    if (sysval_kind(tmp[slots[q]].val, &kind, &dim)) {
                        if (R->sys) {
                            R->sys[ns].instr = i;
                            R->sys[ns].slot = (uint16_t)slots[q];
                            R->sys[ns].kind = (uint8_t)kind;
                            R->sys[ns].dim = (uint8_t)dim;
                        }
                        ns++;
                    }
                }
            }
        }
        R->n_acc = na;
        R->n_sys = ns;
    }
    free(IN); free(OUT); free(reached);
    free_cfg(&G);
    return R->status;
}

/* Apply the blocks of `path` in order starting from the entry state
 * (used by the meet-over-all-paths test). */
int or_apply_path(const or_kernel *K, const or_instr *I, const or_arg *args, const uint32_t *path, uint32_t len, or_slot *out) {
    if (or_kernel_status(K, I) != OK) return -1;
    cfg_t G;
    build_cfg(I, K->n_instr, &G);
    or_entry_state(K, out);
    for (uint32_t j = 0; j < len; j++) {
        if (path[j] >= G.n_blocks) { free_cfg(&G); return -1; }
        apply_block(K, args, I, &G, path[j], out);
    }
    free_cfg(&G);
    return 0;
}

/* Apply the blocks of `path` in order to the state in `st` (in place). */
int or_apply_path_from(const or_kernel *K, const or_instr *I, const or_arg *args, const uint32_t *path, uint32_t len,
                       or_slot *st) {
    if (or_kernel_status(K, I) != OK) return -1;
    cfg_t G;
    build_cfg(I, K->n_instr, &G);
    for (uint32_t j = 0; j < len; j++) {
        if (path[j] >= G.n_blocks) { free_cfg(&G); return -1; }
        apply_block(K, args, I, &G, path[j], st);
    }
    free_cfg(&G);
    return 0;
}

/* ------------------------------------------------------------------ */
/* register versions (SSA form)                                         */
/* ------------------------------------------------------------------ */
/* Section "Search for control structures": at a block with several
 * predecessors a register may hold the value of different definitions, and
 * the paper then creates a variable; the Register record of Section "Search
 * for memory accesses" carries a version.  The reading: minimal SSA form of
 * the kernel's control flow graph (Cytron, Ferrante, Rosen, Wegman & Zadeck
 * 1991).  Every register slot is a variable; a virtual start node before
 * block 0 defines version 0 of every slot (the ABI entry value); each
 * definition of an instruction (explicit destination dwords, then the
 * implicit vcc, exec and scc definitions) makes a new version; a merge (phi)
 * of a slot sits at every block of the iterated dominance frontier of the
 * blocks defining it.  Dominators: the iterative algorithm of Cooper, Harvey
 * & Kennedy (2001) over reverse postorder.  Versions are numbered per slot in
 * a preorder walk of the dominator tree (children by ascending block
 * index), phis of a block first (by slot), then the instructions in order.
 * Only reachable blocks take part. */
#define SSA_NU 13   /* register uses of one instruction, at most */
#define SSA_ND 9    /* register definitions of one instruction, at most */
#define SSA_NONE 0xFFFFFFFFu

/* register slots instruction I reads, in a fixed order: r1, r2, src2 and a
 * stored r0, dword by dword, then the implicit vcc, exec and scc uses */
static int ssa_uses(const or_instr *I, unsigned *out) {
    const opinfo *o = &OPS[I->op];
    int n = 0;
    const enum role roles[4] = {o->r1, o->r2, o->src2, o->r0};
    const unsigned ids[4] = {I->r1, I->r2, (unsigned)I->imm & 0xFFFFu, I->r0};
    const int ws[4] = {o->w1, o->w2, o->w_src2, o->w0};
    for (int q = 0; q < 4; q++) {
        const enum role r = roles[q];
        if (r == NO || r == SD || r == VD) continue;
        if (q == 2 && o->src2 == NO) continue;
        for (int j = 0; j < ws[q]; j++)
            if (ids[q] < NSLOT && ids[q] + (unsigned)j < NSLOT) out[n++] = ids[q] + (unsigned)j;
    }
    if (o->imp_use & I_VCC) { out[n++] = 104; out[n++] = 105; }
    if (o->imp_use & I_EXEC) { out[n++] = 106; out[n++] = 107; }
    if (o->imp_use & I_SCC) out[n++] = 108;
    return n;
}

/* register slots instruction I defines: the destination dwords, then the
 * implicit vcc, exec and scc definitions */
static int ssa_defs(const or_instr *I, unsigned *out) {
    const opinfo *o = &OPS[I->op];
    int n = 0;
    if (o->r0 == SD || o->r0 == VD)
        for (int j = 0; j < o->w0; j++) out[n++] = I->r0 + (unsigned)j;
    if (o->imp_def & I_VCC) { out[n++] = 104; out[n++] = 105; }
    if (o->imp_def & I_EXEC) { out[n++] = 106; out[n++] = 107; }
    if (o->imp_def & I_SCC) out[n++] = 108;
    return n;
}

typedef struct { uint32_t block; uint16_t slot, pad; uint32_t version; } or_phi;
typedef struct {
    int32_t status;
    uint32_t n_blocks, n_phi, n_args;
    uint32_t *idom;          /* n_blocks: immediate dominator; block 0 -> 0; unreachable -> SSA_NONE */
    or_phi *phi;             /* n_phi, ascending (block, slot) */
    uint32_t *phi_arg_off;   /* n_phi + 1 */
    uint32_t *phi_arg;       /* per phi, one version per incoming edge: block 0's entry edge first, then the
                                predecessors in ascending order */
    uint32_t *use_ver;       /* SSA_NU per instruction, in ssa_uses order; SSA_NONE past the uses */
    uint32_t *def_ver;       /* SSA_ND per instruction, in ssa_defs order; SSA_NONE past the definitions */
    uint32_t n_ver[NSLOT];   /* versions of each slot, version 0 included */
    uint64_t digest;
} or_ssa_out;

/* walk up the dominator tree from a and b to their nearest common dominator
 * (positions in reverse postorder decrease towards the root) */
static uint32_t dom_meet(const uint32_t *idom, const int32_t *po, uint32_t a, uint32_t b) {
    while (a != b) {
        while (po[a] > po[b]) a = idom[a];
        while (po[b] > po[a]) b = idom[b];
    }
    return a;
}

/* the digest: a sum over (kind, index, value) items, so its value does not
 * depend on the order the items are produced in */
static uint64_t ssa_item(uint64_t kind, uint64_t index, uint64_t value) {
    return mix64(mix64(kind * 0x9E3779B97F4A7C15ull + index) ^ value);
}

int or_ssa_uses(const or_instr *I, unsigned *out) { return ssa_uses(I, out); }
int or_ssa_defs(const or_instr *I, unsigned *out) { return ssa_defs(I, out); }

void or_ssa_free(or_ssa_out *R) {
    free(R->idom); free(R->phi); free(R->phi_arg_off); free(R->phi_arg); free(R->use_ver); free(R->def_ver);
    memset(R, 0, sizeof(*R));
}

int or_ssa(const or_kernel *K, const or_instr *I, or_ssa_out *R) {
    memset(R, 0, sizeof(*R));
    const uint32_t n = K->n_instr;
    R->use_ver = (uint32_t *)malloc(sizeof(uint32_t) * SSA_NU * (n ? n : 1));
    R->def_ver = (uint32_t *)malloc(sizeof(uint32_t) * SSA_ND * (n ? n : 1));
    for (uint64_t i = 0; i < (uint64_t)SSA_NU * n; i++) R->use_ver[i] = SSA_NONE;
    for (uint64_t i = 0; i < (uint64_t)SSA_ND * n; i++) R->def_ver[i] = SSA_NONE;
    R->phi_arg_off = (uint32_t *)calloc(1, sizeof(uint32_t));
    R->status = or_kernel_status(K, I);
    if (R->status != OK) return R->status;
    cfg_t G;
    build_cfg(I, n, &G);
    const uint32_t nb = G.n_blocks;
    R->n_blocks = nb;
    /* reverse postorder positions; -1 unreachable */
    int32_t *po = (int32_t *)malloc(sizeof(int32_t) * nb);
    for (uint32_t b = 0; b < nb; b++) po[b] = -1;
    for (uint32_t i = 0; i < G.n_reach; i++) po[G.rpo[i]] = (int32_t)i;
    /* dominators */
    uint32_t *idom = (uint32_t *)malloc(sizeof(uint32_t) * nb);
    for (uint32_t b = 0; b < nb; b++) idom[b] = SSA_NONE;
    idom[0] = 0;
    for (int changed = 1; changed;) {
        changed = 0;
        for (uint32_t i = 1; i < G.n_reach; i++) {
            const uint32_t b = G.rpo[i];
            uint32_t nd = SSA_NONE;
            for (uint32_t j = G.pred_off[b]; j < G.pred_off[b + 1]; j++) {
                const uint32_t p = G.pred[j];
                if (po[p] < 0 || idom[p] == SSA_NONE) continue;
                nd = nd == SSA_NONE ? p : dom_meet(idom, po, p, nd);
            }
            if (nd != idom[b]) { idom[b] = nd; changed = 1; }
        }
    }
    R->idom = idom;
    /* dominance frontiers (lists per block); the virtual start dominates
     * block 0, so a predecessor of block 0 climbs to block 0 inclusive */
    uint32_t *df_n = (uint32_t *)calloc(nb, sizeof(uint32_t)), *df_cap = (uint32_t *)calloc(nb, sizeof(uint32_t));
    uint32_t **df = (uint32_t **)calloc(nb, sizeof(uint32_t *));
    uint32_t *mark = (uint32_t *)malloc(sizeof(uint32_t) * nb);
    for (uint32_t b = 0; b < nb; b++) mark[b] = SSA_NONE;
    for (uint32_t b = 0; b < nb; b++) {
        if (po[b] < 0) continue;
        for (uint32_t j = G.pred_off[b]; j < G.pred_off[b + 1]; j++) {
            uint32_t r = G.pred[j];
            if (po[r] < 0) continue;
            for (;;) {
                if (b != 0 && r == idom[b]) break;
                if (mark[r] != b) {
                    mark[r] = b;
                    if (df_n[r] == df_cap[r]) {
                        df_cap[r] = df_cap[r] ? 2 * df_cap[r] : 4;
                        df[r] = (uint32_t *)realloc(df[r], sizeof(uint32_t) * df_cap[r]);
                    }
                    df[r][df_n[r]++] = b;
                }
                if (r == 0) break;   /* above block 0 is the virtual start */
                r = idom[r];
            }
        }
    }
    /* phi placement: per slot, the iterated dominance frontier of its
     * defining blocks (worklist) */
    uint8_t *defines = (uint8_t *)calloc((size_t)nb * NSLOT, 1);
    for (uint32_t b = 0; b < nb; b++) {
        if (po[b] < 0) continue;
        for (uint32_t i = G.block_start[b]; i < G.block_start[b + 1]; i++) {
            unsigned d[SSA_ND];
            const int nd = ssa_defs(&I[i], d);
            for (int q = 0; q < nd; q++) defines[(size_t)b * NSLOT + d[q]] = 1;
        }
    }
    uint8_t *has_phi = (uint8_t *)calloc((size_t)nb * NSLOT, 1);
    uint32_t *work = (uint32_t *)malloc(sizeof(uint32_t) * (nb + 1)), *inw = (uint32_t *)malloc(sizeof(uint32_t) * nb);
    for (unsigned v = 0; v < NSLOT; v++) {
        uint32_t nw = 0;
        for (uint32_t b = 0; b < nb; b++) {
            inw[b] = 0;
            if (defines[(size_t)b * NSLOT + v]) { work[nw++] = b; inw[b] = 1; }
        }
        while (nw) {
            const uint32_t x = work[--nw];
            for (uint32_t j = 0; j < df_n[x]; j++) {
                const uint32_t y = df[x][j];
                if (has_phi[(size_t)y * NSLOT + v]) continue;
                has_phi[(size_t)y * NSLOT + v] = 1;
                if (!inw[y]) { inw[y] = 1; work[nw++] = y; }
            }
        }
    }
    uint32_t n_phi = 0;
    for (size_t i = 0; i < (size_t)nb * NSLOT; i++) n_phi += has_phi[i];
    R->n_phi = n_phi;
    R->phi = (or_phi *)malloc(sizeof(or_phi) * (n_phi ? n_phi : 1));
    uint32_t *phi_at = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)nb * NSLOT);   /* phi index or SSA_NONE */
    R->phi_arg_off = (uint32_t *)realloc(R->phi_arg_off, sizeof(uint32_t) * (n_phi + 1));
    uint32_t np = 0, na = 0;
    for (uint32_t b = 0; b < nb; b++) {
        uint32_t inc = 0;   /* incoming edges: reachable predecessors, plus the entry edge of block 0 */
        for (uint32_t j = G.pred_off[b]; j < G.pred_off[b + 1]; j++) inc += po[G.pred[j]] >= 0;
        if (b == 0) inc++;
        for (unsigned v = 0; v < NSLOT; v++) {
            phi_at[(size_t)b * NSLOT + v] = SSA_NONE;
            if (!has_phi[(size_t)b * NSLOT + v]) continue;
            R->phi[np].block = b;
            R->phi[np].slot = (uint16_t)v;
            R->phi[np].pad = 0;
            R->phi[np].version = SSA_NONE;
            R->phi_arg_off[np] = na;
            phi_at[(size_t)b * NSLOT + v] = np++;
            na += inc;
        }
    }
    R->phi_arg_off[np] = na;
    R->n_args = na;
    R->phi_arg = (uint32_t *)malloc(sizeof(uint32_t) * (na ? na : 1));
    for (uint32_t i = 0; i < na; i++) R->phi_arg[i] = SSA_NONE;
    /* block 0's entry edge carries version 0 */
    for (unsigned v = 0; v < NSLOT; v++)
        if (phi_at[v] != SSA_NONE) R->phi_arg[R->phi_arg_off[phi_at[v]]] = 0;
    /* dominator-tree children, ascending */
    uint32_t *ch_off = (uint32_t *)calloc(nb + 1, sizeof(uint32_t)), *ch = (uint32_t *)malloc(sizeof(uint32_t) * (nb ? nb : 1));
    for (uint32_t b = 1; b < nb; b++) if (po[b] >= 0) ch_off[idom[b] + 1]++;
    for (uint32_t b = 0; b < nb; b++) ch_off[b + 1] += ch_off[b];
    uint32_t *chf = (uint32_t *)calloc(nb + 1, sizeof(uint32_t));
    for (uint32_t b = 1; b < nb; b++) if (po[b] >= 0) ch[ch_off[idom[b]] + chf[idom[b]]++] = b;
    free(chf);
    /* renaming: a stack of versions per slot; an explicit walk stack of
     * (block, next child) with the count of versions each visit pushed */
    uint32_t counter[NSLOT], *vstk[NSLOT], vsp[NSLOT], vcap[NSLOT];
    for (unsigned v = 0; v < NSLOT; v++) {
        counter[v] = 1;
        vcap[v] = 16;
        vstk[v] = (uint32_t *)malloc(sizeof(uint32_t) * vcap[v]);
        vstk[v][0] = 0;
        vsp[v] = 1;
    }
#define SSA_PUSH(v, x) do { if (vsp[v] == vcap[v]) { vcap[v] *= 2; vstk[v] = (uint32_t *)realloc(vstk[v], sizeof(uint32_t) * vcap[v]); } vstk[v][vsp[v]++] = (x); } while (0)
    typedef struct { uint32_t b, next; uint32_t pushed_lo; } frame_t;
    frame_t *fs = (frame_t *)malloc(sizeof(frame_t) * (nb + 1));
    uint32_t *pushlog = (uint32_t *)malloc(sizeof(uint32_t) * ((size_t)SSA_ND * n + (size_t)nb * NSLOT + 1));
    uint32_t pl = 0, fsp = 0;
    if (nb) { fs[0].b = 0; fs[0].next = SSA_NONE; fs[0].pushed_lo = 0; fsp = 1; }
    while (fsp) {
        frame_t *f = &fs[fsp - 1];
        const uint32_t b = f->b;
        if (f->next == SSA_NONE) {   /* enter b */
            f->pushed_lo = pl;
            for (unsigned v = 0; v < NSLOT; v++) {
                const uint32_t pi = phi_at[(size_t)b * NSLOT + v];
                if (pi == SSA_NONE) continue;
                R->phi[pi].version = counter[v];
                SSA_PUSH(v, counter[v]);
                counter[v]++;
                pushlog[pl++] = v;
            }
            for (uint32_t i = G.block_start[b]; i < G.block_start[b + 1]; i++) {
                unsigned u[SSA_NU], d[SSA_ND];
                const int nu = ssa_uses(&I[i], u), nd = ssa_defs(&I[i], d);
                for (int q = 0; q < nu; q++) R->use_ver[(size_t)i * SSA_NU + q] = vstk[u[q]][vsp[u[q]] - 1];
                for (int q = 0; q < nd; q++) {
                    R->def_ver[(size_t)i * SSA_ND + q] = counter[d[q]];
                    SSA_PUSH(d[q], counter[d[q]]);
                    counter[d[q]]++;
                    pushlog[pl++] = d[q];
                }
            }
            /* arguments of the successors' phis for the edge from b */
            for (int e = 0; e < 2; e++) {
                const int32_t s = G.succ[2 * b + e];
                if (s < 0) continue;
                uint32_t k = (s == 0) ? 1 : 0;   /* incoming-edge index of b at s */
                for (uint32_t j = G.pred_off[s]; j < G.pred_off[s + 1] && G.pred[j] != b; j++) k += po[G.pred[j]] >= 0;
                for (unsigned v = 0; v < NSLOT; v++) {
                    const uint32_t pi = phi_at[(size_t)s * NSLOT + v];
                    if (pi != SSA_NONE) R->phi_arg[R->phi_arg_off[pi] + k] = vstk[v][vsp[v] - 1];
                }
            }
            f->next = ch_off[b];
        }
        if (f->next < ch_off[b + 1]) {
            const uint32_t c = ch[f->next++];
            fs[fsp].b = c;
            fs[fsp].next = SSA_NONE;
            fs[fsp].pushed_lo = 0;
            fsp++;
        } else {   /* leave b: pop what it pushed */
            while (pl > f->pushed_lo) vsp[pushlog[--pl]]--;
            fsp--;
        }
    }
#undef SSA_PUSH
    for (unsigned v = 0; v < NSLOT; v++) { R->n_ver[v] = counter[v]; free(vstk[v]); }
    /* digest over idom, phis, arguments and every use and definition version */
    uint64_t h = 0;
    for (uint32_t b = 0; b < nb; b++) h += ssa_item(1, b, idom[b]);
    for (uint32_t i = 0; i < n_phi; i++)
        h += ssa_item(2, ((uint64_t)R->phi[i].block << 16) | R->phi[i].slot, R->phi[i].version);
    for (uint32_t i = 0; i < n_phi; i++)
        for (uint32_t k = R->phi_arg_off[i]; k < R->phi_arg_off[i + 1]; k++)
            h += ssa_item(3, ((uint64_t)R->phi[i].block << 24) | ((uint64_t)R->phi[i].slot << 12) | (k - R->phi_arg_off[i]),
                          R->phi_arg[k]);
    for (uint64_t i = 0; i < (uint64_t)SSA_NU * n; i++) h += ssa_item(4, i, R->use_ver[i]);
    for (uint64_t i = 0; i < (uint64_t)SSA_ND * n; i++) h += ssa_item(5, i, R->def_ver[i]);
    R->digest = h;
    for (uint32_t b = 0; b < nb; b++) free(df[b]);
    free(df); free(df_n); free(df_cap); free(mark); free(defines); free(has_phi); free(work); free(inw);
    free(phi_at); free(ch_off); free(ch); free(fs); free(pushlog); free(po);
    free_cfg(&G);
    return OK;
}

/* Batch driver of the versions: per kernel status, block count, merges,
 * merge arguments, stored operand versions (the uses and definitions of
 * every instruction of a kernel that passed its checks) and the digest. */
typedef struct { int32_t status; uint32_t n_blocks, n_phi, n_args, n_operands, pad; uint64_t digest; } or_ssa_summary;

int or_ssa_batch(const or_kernel *kernels, uint32_t n_kernels, const or_instr *instrs, or_ssa_summary *sum) {
    for (uint32_t k = 0; k < n_kernels; k++) {
        const or_kernel *K = &kernels[k];
        const or_instr *I = instrs + K->instr_begin;
        or_ssa_out R;
        or_ssa(K, I, &R);
        memset(&sum[k], 0, sizeof(sum[k]));
        sum[k].status = R.status;
        if (R.status == OK) {
            sum[k].n_blocks = R.n_blocks;
            sum[k].n_phi = R.n_phi;
            sum[k].n_args = R.n_args;
            for (uint32_t i = 0; i < K->n_instr; i++) {
                unsigned u[SSA_NU], d[SSA_ND];
                sum[k].n_operands += (uint32_t)(ssa_uses(&I[i], u) + ssa_defs(&I[i], d));
            }
            sum[k].digest = R.digest;
        }
        or_ssa_free(&R);
    }
    return 0;
}

/*
 * Batch driver: per kernel summary (status, n_blocks, sweeps, counts, digest)
 * and the accesses and system values packed densely in kernel order.
 * acc/sys capacities are the batch's instruction count and 4x that.
 */
typedef struct { int32_t status; uint32_t n_blocks, sweeps, n_acc, n_sys, pad; uint64_t digest; } or_summary;

int or_analyze_batch(const or_kernel *kernels, uint32_t n_kernels, const or_instr *instrs, const or_arg *args,
                     uint32_t sweep_cap, or_summary *sum, or_access *acc, or_sysval *sys, uint64_t *n_acc_total,
                     uint64_t *n_sys_total) {
    uint64_t na = 0, ns = 0;
    for (uint32_t k = 0; k < n_kernels; k++) {
        const or_kernel *K = &kernels[k];
        or_result R;
        memset(&R, 0, sizeof(R));
        R.acc = acc ? acc + na : 0;
        R.sys = sys ? sys + ns : 0;
        or_analyze(K, instrs + K->instr_begin, args + K->arg_begin, sweep_cap, 0, 0, &R);
        sum[k].status = R.status;
        sum[k].n_blocks = R.n_blocks;
        sum[k].sweeps = R.sweeps;
        sum[k].n_acc = R.n_acc;
        sum[k].n_sys = R.n_sys;
        sum[k].pad = 0;
        sum[k].digest = R.digest;
        na += R.n_acc;
        ns += R.n_sys;
    }
    if (n_acc_total) *n_acc_total = na;
    if (n_sys_total) *n_sys_total = ns;
    return 0;
}

/* ------------------------------------------------------------------ */
/* text front end (Section "The body extraction")                       */
/* ------------------------------------------------------------------ */
/* Listing 2's extraction loop over the lines of a listing: a line holding
 * ".kernel" opens a kernel whose name is its second word; a line ".config"
 * switches to the configuration state and ".text" to the instruction state;
 * lines in those states are collected into the kernel's configuration and
 * body; anything else is skipped.  Each kernel is then processed: the
 * configuration gives .dims, .cws, .useargs and the .arg lines of Listing 3;
 * the body gives one record per instruction line, labels (a line "NAME:")
 * naming the index of the next instruction.  Readings (the paper fixes no
 * grammar): comments run from "//" or ";" to the end of the line; blanks
 * are spaces, tabs and carriage returns; ".dims" (or "dims", as Listing 1
 * prints it) takes x, xy or xyz; ".cws" takes up to three integers (a
 * missing later one is 1; without .cws every size is 0); args whose names
 * begin with "_." are the six hidden slots of Listing 3 and take no entry;
 * user args are laid out from byte 0x30, each aligned to its size.  An
 * unknown mnemonic gives opcode 0xFFFF, an operand that is not a register,
 * inline constant or integer gives operand id 0xFFFD, a malformed offset
 * gives opcode 0xFFFF, and an unknown branch label gives target 0x7FFFFFFF,
 * so the record checks of the analysis report each of them. */
#define TX_BAD 0xFFFDu
#define TX_NONE 0xFFFFu
#define TX_LIT 0xFFFEu

typedef struct { const char *p; uint32_t n; } tx_span;

static int tx_blank(char c) { return c == ' ' || c == '\t' || c == '\r'; }

/* the line without its comment and surrounding blanks */
static tx_span tx_clean(const char *p, uint32_t n) {
    for (uint32_t i = 0; i < n; i++)
        if (p[i] == ';' || (p[i] == '/' && i + 1 < n && p[i + 1] == '/')) { n = i; break; }
    while (n && tx_blank(p[n - 1])) n--;
    while (n && tx_blank(p[0])) { p++; n--; }
    tx_span s = {p, n};
    return s;
}
static tx_span tx_trim(tx_span s) { return tx_clean(s.p, s.n); }
static int tx_eq(tx_span s, const char *lit) { return strlen(lit) == s.n && memcmp(s.p, lit, s.n) == 0; }
/* first blank-separated word of s; *rest = what follows it */
static tx_span tx_word(tx_span s, tx_span *rest) {
    uint32_t i = 0;
    while (i < s.n && !tx_blank(s.p[i])) i++;
    tx_span w = {s.p, i};
    if (rest) { tx_span r = {s.p + i, s.n - i}; *rest = tx_trim(r); }
    return w;
}
/* field k of a comma-separated list (trimmed); n = 0 when absent */
static tx_span tx_field(tx_span s, int k) {
    uint32_t a = 0;
    for (int f = 0; f <= k; f++) {
        uint32_t b = a;
        while (b < s.n && s.p[b] != ',') b++;
        if (f == k) { tx_span r = {s.p + a, b - a}; return tx_trim(r); }
        if (b >= s.n) { tx_span z = {s.p, 0}; return z; }
        a = b + 1;
    }
    tx_span z = {s.p, 0};
    return z;
}
static int tx_nfields(tx_span s) {
    if (!s.n) return 0;
    int n = 1;
    for (uint32_t i = 0; i < s.n; i++) n += s.p[i] == ',';
    return n;
}
/* integer: optional '-', then 0x hex digits or decimal digits; 0 on error */
static int tx_int(tx_span s, int64_t *v) {
    uint32_t i = 0;
    int neg = 0;
    if (i < s.n && s.p[i] == '-') { neg = 1; i++; }
    if (i >= s.n) return 0;
    uint64_t x = 0;
    if (i + 1 < s.n && s.p[i] == '0' && (s.p[i + 1] == 'x' || s.p[i + 1] == 'X')) {
        i += 2;
        if (i >= s.n) return 0;
        for (; i < s.n; i++) {
            const char c = s.p[i];
            int d = c >= '0' && c <= '9' ? c - '0' : c >= 'a' && c <= 'f' ? c - 'a' + 10 : c >= 'A' && c <= 'F' ? c - 'A' + 10 : -1;
            if (d < 0 || x >> 60) return 0;
            x = x * 16 + (uint64_t)d;
        }
    } else {
        for (; i < s.n; i++) {
            const char c = s.p[i];
            if (c < '0' || c > '9' || x > 100000000000000000ull) return 0;
            x = x * 10 + (uint64_t)(c - '0');
        }
    }
    *v = neg ? -(int64_t)x : (int64_t)x;
    return 1;
}
static unsigned tx_lower(char c) { return (c >= 'A' && c <= 'Z') ? (unsigned)(c - 'A' + 'a') : (unsigned)(unsigned char)c; }
static int tx_ieq(tx_span s, const char *lit) {
    if (strlen(lit) != s.n) return 0;
    for (uint32_t i = 0; i < s.n; i++)
        if (tx_lower(s.p[i]) != (unsigned char)lit[i]) return 0;
    return 1;
}

/* a register, inline constant or literal; *lit set for a literal */
static unsigned tx_operand(tx_span t, int *has_lit, int32_t *lit) {
    static const char *const special[] = {"vcc", "vcc_lo", "vcc_hi", "exec", "exec_lo", "exec_hi", "scc", "m0", "off"};
    static const unsigned special_id[] = {104, 104, 105, 106, 106, 107, 108, 109, TX_NONE};
    for (int i = 0; i < 9; i++)
        if (tx_ieq(t, special[i])) return special_id[i];
    if (t.n >= 2 && (tx_lower(t.p[0]) == 's' || tx_lower(t.p[0]) == 'v')) {
        const int vec = tx_lower(t.p[0]) == 'v';
        const int64_t lim = vec ? 255 : 103;
        int64_t a, b;
        if (t.p[1] == '[') {
            uint32_t c = 2;
            while (c < t.n && t.p[c] != ':') c++;
            if (c >= t.n || t.p[t.n - 1] != ']') return TX_BAD;
            tx_span x = {t.p + 2, c - 2}, y = {t.p + c + 1, t.n - c - 2};
            if (!tx_int(x, &a) || !tx_int(y, &b) || a < 0 || b < a || b > lim || x.p[0] == '-') return TX_BAD;
        } else {
            tx_span x = {t.p + 1, t.n - 1};
            if (x.p[0] == '-' || !tx_int(x, &a) || a < 0 || a > lim) return TX_BAD;
        }
        return vec ? 112u + (unsigned)a : (unsigned)a;
    }
    static const char *const floats[8] = {"0.5", "-0.5", "1.0", "-1.0", "2.0", "-2.0", "4.0", "-4.0"};
    for (int i = 0; i < 8; i++)
        if (tx_eq(t, floats[i])) return 0x8060u + (unsigned)i;
    int64_t v;
    if (!tx_int(t, &v)) return TX_BAD;
    if (v >= -16 && v <= 64) return 0x8000u + (unsigned)(v + 16);
    *has_lit = 1;
    *lit = (int32_t)(uint32_t)(uint64_t)v;
    return TX_LIT;
}

typedef struct { tx_span name; uint32_t index; } tx_label;

static int tx_find_op(tx_span w) {
    for (int op = 0; op < N_OPS; op++)
        if (tx_ieq(w, OPS[op].name)) return op;
    return -1;
}

/* one instruction line -> record */
static or_instr tx_instr(tx_span line, const tx_label *labels, uint32_t n_labels) {
    or_instr r = {TX_NONE, TX_NONE, TX_NONE, TX_NONE, 0, -1};
    tx_span rest;
    const tx_span w = tx_word(line, &rest);
    const int op = tx_find_op(w);
    if (op < 0) { r.op = TX_NONE; return r; }
    r.op = (uint16_t)op;
    const opinfo *o = &OPS[op];
    /* operands: comma-separated fields, each an operand word followed by
     * modifier words; without any comma (as the paper prints
     * "s_load_dwordx2 s[2:3] s[4:5] 0x0") every blank-separated word is an
     * operand, except modifiers.  A modifier is a word with ':' and no '['
     * (key:value); only offset:N is read. */
    int bad_num = 0;
    int nf = 0;
    tx_span f[8];
    int has_comma = 0;
    for (uint32_t i = 0; i < rest.n; i++) has_comma |= rest.p[i] == ',';
    const int nfields = has_comma ? tx_nfields(rest) : 1;
    for (int k = 0; k < nfields; k++) {
        tx_span words = has_comma ? tx_field(rest, k) : rest;
        int first = 1;
        while (words.n) {
            tx_span more;
            const tx_span mw = tx_word(words, &more);
            int colon = 0, bracket = 0;
            for (uint32_t i = 0; i < mw.n; i++) { colon |= mw.p[i] == ':'; bracket |= mw.p[i] == '['; }
            if (colon && !bracket) {
                if (mw.n > 7 && memcmp(mw.p, "offset:", 7) == 0) {
                    tx_span num = {mw.p + 7, mw.n - 7};
                    int64_t v;
                    if (tx_int(num, &v)) r.imm = (int32_t)(uint32_t)(uint64_t)v;
                    else bad_num = 1;
                }
            } else if (first || !has_comma) {
                if (nf < 8) f[nf] = mw;
                nf++;
                first = 0;
            }
            words = more;
        }
        if (has_comma && first) {   /* an empty field still counts */
            if (nf < 8) f[nf].p = rest.p, f[nf].n = 0;
            nf++;
        }
    }
    if (nf > 8) nf = 8;
    int has_lit = 0;
    int32_t lit = 0;
#define OPD(k) ((k) < nf && f[k].n ? (uint16_t)tx_operand(f[k], &has_lit, &lit) : (uint16_t)TX_BAD)
    switch (o->cls) {
    case C_SMEM: {
        r.r0 = OPD(0);
        r.r1 = OPD(1);
        int64_t v;
        if (nf > 2 && tx_int(f[2], &v)) r.imm = (int32_t)(uint32_t)(uint64_t)v;
        else bad_num = 1;
        break;
    }
    case C_BRANCH:
    case C_CBRANCH: {
        r.target = 0x7FFFFFFF;
        if (nf > 0) {
            int found = 0;
            for (uint32_t j = 0; j < n_labels && !found; j++)
                if (labels[j].name.n == f[0].n && memcmp(labels[j].name.p, f[0].p, f[0].n) == 0) {
                    r.target = (int32_t)labels[j].index;
                    found = 1;
                }
            int64_t v;
            if (!found && tx_int(f[0], &v) && v >= 0 && v < 0x7FFFFFFF) r.target = (int32_t)v;
        }
        break;
    }
    case C_NOP:
    case C_END: break;
    case C_SCMP: r.r1 = OPD(0); r.r2 = OPD(1); break;
    case C_VCMP: r.r1 = OPD(1); r.r2 = OPD(2); break;
    case C_GLOAD: r.r0 = OPD(0); r.r1 = OPD(1); r.r2 = OPD(2); break;
    case C_FLOAD:
    case C_DSREAD: r.r0 = OPD(0); r.r1 = OPD(1); break;
    case C_GSTORE: r.r1 = OPD(0); r.r0 = OPD(1); r.r2 = OPD(2); break;
    case C_FSTORE:
    case C_DSWRITE: r.r1 = OPD(0); r.r0 = OPD(1); break;
    default:
        if (o->cls == C_VALU && (o->imp_def & I_VCC)) {   /* dst, vcc, src0, src1 */
            r.r0 = OPD(0); r.r1 = OPD(2); r.r2 = OPD(3);
        } else if (o->src2 != NO) {                        /* dst, src0, src1, src2 */
            r.r0 = OPD(0); r.r1 = OPD(1); r.r2 = OPD(2);
            r.imm = (int32_t)OPD(3);
        } else if (o->r2 == NO) {                          /* dst, src */
            r.r0 = OPD(0); r.r1 = OPD(1);
        } else {                                           /* dst, src0, src1 */
            r.r0 = OPD(0); r.r1 = OPD(1); r.r2 = OPD(2);
        }
    }
#undef OPD
    if (has_lit && !o->imm_is_offset && o->src2 == NO) r.imm = lit;
    if (bad_num) r.op = TX_NONE;
    return r;
}

/* Listing 3's .arg type: size, type bits, pointee bits */
static void tx_argtype(tx_span t, uint16_t *size, uint8_t *type, uint8_t *flags) {
    int ptr = 0;
    if (t.n && t.p[t.n - 1] == '*') {
        ptr = 1;
        t.n--;
        t = tx_trim(t);
    }
    static const char *const names[] = {"char", "uchar", "short", "ushort", "int", "uint", "long", "ulong",
                                        "float", "double", "size_t", "void"};
    static const uint8_t bits[] = {1, 2, 1, 2, 1, 2, 1, 2, 4, 8, 2, 0};
    static const uint16_t sizes[] = {1, 1, 2, 2, 4, 4, 8, 8, 4, 8, 8, 4};
    uint8_t b = 0;
    uint16_t sz = 4;
    for (int i = 0; i < 12; i++)
        if (tx_eq(t, names[i])) { b = bits[i]; sz = sizes[i]; break; }
    if (ptr) { *size = 8; *type = 16; *flags = b; }
    else { *size = sz; *type = b; *flags = 0; }
}

typedef struct {
    uint32_t n_kernels;
    uint64_t n_instr, n_args;
    or_kernel *kernels;
    or_instr *instrs;
    or_arg *args;
    uint64_t *name_off;      /* per kernel: byte offset of its name in the text */
    uint32_t *name_len;
} or_text_out;

typedef struct { uint64_t *off; uint32_t *len; uint32_t n, cap; } tx_lines;
static void tx_push(tx_lines *L, uint64_t off, uint32_t len) {
    if (L->n == L->cap) {
        L->cap = L->cap ? 2 * L->cap : 64;
        L->off = (uint64_t *)realloc(L->off, sizeof(uint64_t) * L->cap);
        L->len = (uint32_t *)realloc(L->len, sizeof(uint32_t) * L->cap);
    }
    L->off[L->n] = off;
    L->len[L->n] = len;
    L->n++;
}

/* process_data of Listing 2: one kernel's configuration and body */
static void tx_process(const char *text, uint64_t name_off, uint32_t name_len, const tx_lines *cfg,
                       const tx_lines *body, or_text_out *O) {
    or_kernel K;
    memset(&K, 0, sizeof(K));
    K.instr_begin = O->n_instr;
    K.arg_begin = (uint32_t)O->n_args;
    uint32_t cursor = 0x30;
    for (uint32_t j = 0; j < cfg->n; j++) {
        tx_span line = {text + cfg->off[j], cfg->len[j]}, rest;
        const tx_span w = tx_word(line, &rest);
        if (tx_eq(w, ".dims") || tx_eq(w, "dims")) {
            const tx_span d = tx_word(rest, 0);
            K.dims = tx_eq(d, "x") ? 1 : tx_eq(d, "xy") ? 2 : tx_eq(d, "xyz") ? 3 : 0;
        } else if (tx_eq(w, ".cws")) {
            for (int d = 0; d < 3; d++) {
                const tx_span v = tx_field(rest, d);
                int64_t x;
                K.cws[d] = v.n == 0 ? 1u : (tx_int(v, &x) && x >= 0 && x <= 0xFFFFFFFFll ? (uint32_t)x : 0u);
            }
        } else if (tx_eq(w, ".useargs")) {
            K.useargs = 1;
        } else if (tx_eq(w, ".arg")) {
            const tx_span name = tx_field(rest, 0);
            if (name.n >= 2 && name.p[0] == '_' && name.p[1] == '.') continue;
            or_arg a;
            tx_argtype(tx_field(rest, 2), &a.size, &a.type, &a.flags);
            cursor = (cursor + a.size - 1) / a.size * a.size;
            a.offset = cursor;
            cursor += a.size;
            O->args = (or_arg *)realloc(O->args, sizeof(or_arg) * (O->n_args + 1));
            O->args[O->n_args++] = a;
            K.n_args++;
        }
    }
    /* labels: the index of the next instruction line */
    tx_label *labels = (tx_label *)malloc(sizeof(tx_label) * (body->n ? body->n : 1));
    uint32_t n_labels = 0, n_ins = 0;
    for (uint32_t j = 0; j < body->n; j++) {
        tx_span line = {text + body->off[j], body->len[j]};
        tx_span rest;
        tx_word(line, &rest);
        if (line.p[line.n - 1] == ':' && rest.n == 0) {
            tx_span nm = {line.p, line.n - 1};
            int seen = 0;
            for (uint32_t q = 0; q < n_labels; q++)
                if (labels[q].name.n == nm.n && memcmp(labels[q].name.p, nm.p, nm.n) == 0) seen = 1;
            if (!seen) { labels[n_labels].name = nm; labels[n_labels].index = n_ins; n_labels++; }
        } else {
            n_ins++;
        }
    }
    O->instrs = (or_instr *)realloc(O->instrs, sizeof(or_instr) * (O->n_instr + n_ins + 1));
    for (uint32_t j = 0; j < body->n; j++) {
        tx_span line = {text + body->off[j], body->len[j]};
        tx_span rest;
        tx_word(line, &rest);
        if (line.p[line.n - 1] == ':' && rest.n == 0) continue;
        O->instrs[O->n_instr++] = tx_instr(line, labels, n_labels);
    }
    free(labels);
    K.n_instr = n_ins;
    O->kernels = (or_kernel *)realloc(O->kernels, sizeof(or_kernel) * (O->n_kernels + 1));
    O->name_off = (uint64_t *)realloc(O->name_off, sizeof(uint64_t) * (O->n_kernels + 1));
    O->name_len = (uint32_t *)realloc(O->name_len, sizeof(uint32_t) * (O->n_kernels + 1));
    O->kernels[O->n_kernels] = K;
    O->name_off[O->n_kernels] = name_off;
    O->name_len[O->n_kernels] = name_len;
    O->n_kernels++;
}

int or_parse_text(const char *text, uint64_t len, or_text_out *O) {
    memset(O, 0, sizeof(*O));
    enum { S_START, S_KERNEL, S_CONFIG, S_TEXT } state = S_START;
    tx_lines cfg = {0, 0, 0, 0}, body = {0, 0, 0, 0};
    int open = 0;
    uint64_t name_off = 0;
    uint32_t name_len = 0;
    uint64_t a = 0;
    while (a <= len) {
        uint64_t b = a;
        while (b < len && text[b] != '\n') b++;
        const tx_span line = tx_clean(text + a, (uint32_t)(b - a));
        if (line.n) {
            tx_span rest;
            const tx_span w = tx_word(line, &rest);
            if (tx_eq(w, ".kernel")) {
                if (open) tx_process(text, name_off, name_len, &cfg, &body, O);
                cfg.n = body.n = 0;
                open = 1;
                const tx_span nm = tx_word(rest, 0);
                name_off = (uint64_t)(nm.p - text);
                name_len = nm.n;
                state = S_KERNEL;
            } else if (open && tx_eq(line, ".config")) {
                state = S_CONFIG;
            } else if (open && tx_eq(line, ".text")) {
                state = S_TEXT;
            } else if (state == S_CONFIG) {
                tx_push(&cfg, (uint64_t)(line.p - text), line.n);
            } else if (state == S_TEXT) {
                tx_push(&body, (uint64_t)(line.p - text), line.n);
            }
        }
        a = b + 1;
    }
    if (open) tx_process(text, name_off, name_len, &cfg, &body, O);
    free(cfg.off); free(cfg.len); free(body.off); free(body.len);
    return 0;
}

void or_text_free(or_text_out *O) {
    free(O->kernels); free(O->instrs); free(O->args); free(O->name_off); free(O->name_len);
    memset(O, 0, sizeof(*O));
}

/* ------------------------------------------------------------------ */
/* structuring (Section "Search for control structures")                */
/* ------------------------------------------------------------------ */
/* The region graph starts as the reachable blocks of the control flow graph
 * (consecutive instructions of a block form one region).  A depth-first
 * search from the entry region visits the regions in preorder (fall-through
 * successor first); the first region that heads a known template has the
 * template's regions merged into a new region; the search starts again until
 * one region is left or no region heads a template.  Templates, checked in
 * this order at a header H:
 *   if-else  H's two successors A, B each have H as their only predecessor
 *            and one common single successor J (not H, A, B); J joins the
 *            merge when A and B are its only predecessors;
 *   if       (Fig. 2) of H's two successors, T has H as only predecessor and
 *            the other, F, as only successor; F joins the merge when H and T
 *            are its only predecessors, else the merge is H and T (the two
 *            cases of the Fig. 3 trace);
 *   while    one successor B of H has H as only predecessor and H as only
 *            successor: H and B merge, the back edge disappears;
 *   linear   H's only successor S is not H, has H as only predecessor and at
 *            most one successor of its own, or H among its successors (which
 *            closes a loop: the merge has an edge to itself);
 *   loop     H has an edge to itself: it disappears.
 * The entry counts one predecessor more (the start), so it is never the
 * inner region of a template.  The paper names the if and linear templates
 * and several exec-mask forms of if-else whose figures are missing; if-else
 * is read as the standard diamond, and while / loop are this reading's
 * additions so that counted loops reduce. */
enum { RG_LINEAR = 1, RG_IF = 2, RG_IFELSE = 3, RG_WHILE = 4, RG_LOOP = 5 };
typedef struct { uint32_t region; uint8_t kind, n; uint16_t pad; uint32_t member[4]; } or_merge;   /* 24 B */
typedef struct {
    int32_t status;
    uint32_t n_blocks, n_merges, n_left, root, pad;
    uint64_t digest;
    or_merge *merges;
} or_struct_out;

typedef struct {
    uint32_t cap, entry, next;
    int32_t *succ;      /* 2 per region, -1 none */
    uint32_t *npred;    /* edges in (+1 for the entry) */
    uint8_t *alive;
} rg_t;

static int rg_nsucc(const rg_t *g, uint32_t x) { return (g->succ[2 * x] >= 0) + (g->succ[2 * x + 1] >= 0); }
static int32_t rg_only(const rg_t *g, uint32_t x) {   /* the single successor, or -1 */
    if (rg_nsucc(g, x) != 1) return -1;
    return g->succ[2 * x] >= 0 ? g->succ[2 * x] : g->succ[2 * x + 1];
}
static int rg_has(const rg_t *g, uint32_t x, uint32_t y) {
    return g->succ[2 * x] == (int32_t)y || g->succ[2 * x + 1] == (int32_t)y;
}

/* merge members m[0..n) (m[0] the header) into a new region */
static uint32_t rg_merge(rg_t *g, const uint32_t *m, int n, int kind) {
    const uint32_t H = m[0], R = g->next++;
    int32_t out[2] = {-1, -1};
    int no = 0, self = 0;
    uint32_t into_h = 0;   /* edges from members into H */
    for (int i = 0; i < n; i++)
        for (int e = 0; e < 2; e++) {
            const int32_t y = g->succ[2 * m[i] + e];
            if (y < 0) continue;
            int inside = 0;
            for (int j = 0; j < n; j++) inside |= (uint32_t)y == m[j];
            if ((uint32_t)y == H) {
                into_h++;
                if (kind != RG_WHILE && kind != RG_LOOP && !self) {
                    self = 1;
                    if (no < 2) out[no++] = (int32_t)R;
                }
                continue;
            }
            if (inside) continue;
            g->npred[y]--;
            int dup = 0;
            for (int k = 0; k < no; k++) dup |= out[k] == y;
            if (!dup) {
                g->npred[y]++;
                if (no < 2) out[no++] = y;
            }
        }
    g->succ[2 * R] = out[0];
    g->succ[2 * R + 1] = out[1];
    g->npred[R] = g->npred[H] - into_h + (uint32_t)self;
    /* edges from outside into H now enter R (no other member has any) */
    for (uint32_t x = 0; x < g->next - 1; x++) {
        if (!g->alive[x]) continue;
        int mem = 0;
        for (int j = 0; j < n; j++) mem |= x == m[j];
        if (mem) continue;
        for (int e = 0; e < 2; e++)
            if (g->succ[2 * x + e] == (int32_t)H) g->succ[2 * x + e] = (int32_t)R;
    }
    for (int i = 0; i < n; i++) g->alive[m[i]] = 0;
    g->alive[R] = 1;
    if (g->entry == H) g->entry = R;
    return R;
}

/* the template headed by x: members into m, returns the kind (0 none) */
static int rg_match(const rg_t *g, uint32_t x, uint32_t *m, int *n) {
    const int32_t a = g->succ[2 * x], b = g->succ[2 * x + 1];
    if (a >= 0 && b >= 0 && a != (int32_t)x && b != (int32_t)x) {
        const int32_t ja = rg_only(g, (uint32_t)a), jb = rg_only(g, (uint32_t)b);
        if (g->npred[a] == 1 && g->npred[b] == 1 && ja >= 0 && ja == jb && ja != (int32_t)x && ja != a && ja != b) {
            m[0] = x; m[1] = (uint32_t)a; m[2] = (uint32_t)b; *n = 3;
            if (g->npred[ja] == 2) { m[3] = (uint32_t)ja; *n = 4; }
            return RG_IFELSE;
        }
        for (int k = 0; k < 2; k++) {
            const int32_t t = k == 0 ? a : b, f = k == 0 ? b : a;
            if (g->npred[t] == 1 && rg_only(g, (uint32_t)t) == f) {
                m[0] = x; m[1] = (uint32_t)t; *n = 2;
                if (g->npred[f] == 2) { m[2] = (uint32_t)f; *n = 3; }
                return RG_IF;
            }
        }
        for (int k = 0; k < 2; k++) {
            const int32_t t = k == 0 ? a : b;
            if (g->npred[t] == 1 && rg_only(g, (uint32_t)t) == (int32_t)x) {
                m[0] = x; m[1] = (uint32_t)t; *n = 2;
                return RG_WHILE;
            }
        }
    }
    const int32_t s = rg_only(g, x);
    if (s >= 0 && s != (int32_t)x && g->npred[s] == 1 && (rg_nsucc(g, (uint32_t)s) <= 1 || rg_has(g, (uint32_t)s, x))) {
        m[0] = x; m[1] = (uint32_t)s; *n = 2;
        return RG_LINEAR;
    }
    if (rg_has(g, x, x)) {
        m[0] = x; *n = 1;
        return RG_LOOP;
    }
    return 0;
}

int or_structure(const or_kernel *K, const or_instr *I, or_struct_out *R) {
    memset(R, 0, sizeof(*R));
    R->root = 0xFFFFFFFFu;   /* no region is left of a kernel that fails its checks */
    R->status = or_kernel_status(K, I);
    if (R->status != OK) return R->status;
    cfg_t G;
    build_cfg(I, K->n_instr, &G);
    const uint32_t nb = G.n_blocks;
    R->n_blocks = nb;
    rg_t g;
    g.cap = 4 * nb + 2;   /* ids: blocks, at most nb - 1 joining merges, one loop merge per edge to itself */
    g.entry = 0;
    g.next = nb;
    g.succ = (int32_t *)malloc(sizeof(int32_t) * 2 * g.cap);
    g.npred = (uint32_t *)calloc(g.cap, sizeof(uint32_t));
    g.alive = (uint8_t *)calloc(g.cap, 1);
    for (uint32_t i = 0; i < 2 * g.cap; i++) g.succ[i] = -1;
    for (uint32_t i = 0; i < G.n_reach; i++) g.alive[G.rpo[i]] = 1;
    for (uint32_t b = 0; b < nb; b++) {
        if (!g.alive[b]) continue;
        g.succ[2 * b] = G.succ[2 * b];
        g.succ[2 * b + 1] = G.succ[2 * b + 1];
        for (int e = 0; e < 2; e++)
            if (G.succ[2 * b + e] >= 0) g.npred[G.succ[2 * b + e]]++;
    }
    g.npred[0]++;   /* the start */
    R->merges = (or_merge *)malloc(sizeof(or_merge) * (g.cap + 1));
    uint32_t *order = (uint32_t *)malloc(sizeof(uint32_t) * g.cap), *stack = (uint32_t *)malloc(sizeof(uint32_t) * 2 * g.cap);
    uint8_t *seen = (uint8_t *)malloc(g.cap);
    uint32_t n_alive = G.n_reach;
    while (n_alive > 1) {
        /* preorder from the entry, fall-through successor first */
        memset(seen, 0, g.cap);
        uint32_t no = 0, sp = 0;
        stack[sp++] = g.entry;
        while (sp) {
            const uint32_t x = stack[--sp];
            if (seen[x]) continue;
            seen[x] = 1;
            order[no++] = x;
            for (int e = 1; e >= 0; e--) {
                const int32_t y = g.succ[2 * x + e];
                if (y >= 0 && !seen[y]) stack[sp++] = (uint32_t)y;
            }
        }
        int done = 0;
        for (uint32_t i = 0; i < no && !done; i++) {
            uint32_t m[4];
            int n = 0;
            const int kind = rg_match(&g, order[i], m, &n);
            if (!kind) continue;
            const uint32_t r = rg_merge(&g, m, n, kind);
            or_merge *M = &R->merges[R->n_merges++];
            memset(M, 0, sizeof(*M));
            M->region = r;
            M->kind = (uint8_t)kind;
            M->n = (uint8_t)n;
            for (int j = 0; j < 4; j++) M->member[j] = j < n ? m[j] : 0xFFFFFFFFu;
            n_alive -= (uint32_t)n - 1;
            done = 1;
        }
        if (!done) break;
    }
    R->n_left = n_alive;
    R->root = n_alive == 1 ? g.entry : 0xFFFFFFFFu;
    uint64_t h = 0;
    for (uint32_t j = 0; j < R->n_merges; j++) {
        const or_merge *M = &R->merges[j];
        uint64_t v = ((uint64_t)M->kind << 56) ^ ((uint64_t)M->n << 48) ^ M->region;
        for (int k = 0; k < 4; k++) v = mix64(v + M->member[k] + 0x9E3779B97F4A7C15ull * (uint64_t)(k + 1));
        h += mix64(mix64(0x5354ull * 0x9E3779B97F4A7C15ull + j) ^ v);
    }
    R->digest = h;
    free(order); free(stack); free(seen);
    free(g.succ); free(g.npred); free(g.alive);
    free_cfg(&G);
    return OK;
}

void or_structure_free(or_struct_out *R) { free(R->merges); R->merges = 0; }

/* Batch driver of the structuring: per kernel status, blocks, merges,
 * regions left, root and digest. */
typedef struct { int32_t status; uint32_t n_blocks, n_merges, n_left, root, pad; uint64_t digest; } or_struct_summary;

int or_structure_batch(const or_kernel *kernels, uint32_t n_kernels, const or_instr *instrs, or_struct_summary *sum) {
    for (uint32_t k = 0; k < n_kernels; k++) {
        or_struct_out R;
        or_structure(&kernels[k], instrs + kernels[k].instr_begin, &R);
        sum[k].status = R.status;
        sum[k].n_blocks = R.n_blocks;
        sum[k].n_merges = R.n_merges;
        sum[k].n_left = R.n_left;
        sum[k].root = R.root;
        sum[k].pad = 0;
        sum[k].digest = R.digest;
        or_structure_free(&R);
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* variables and their types over the register versions                 */
/* ------------------------------------------------------------------ */
/* Section "Search for control structures": a register whose value at a
 * block with several predecessors depends on the path taken becomes a
 * variable when it is used later.  Section "Data type recovery": types come
 * from the .arg lines of the configuration and from instruction suffixes,
 * and a suffix types the values an instruction reads as well as the one it
 * writes (an unsigned add adds two unsigned integers).  The ternary operator
 * (the same section) is one instruction, v_cndmask_b32.  Readings, over the
 * versions of or_ssa:
 *   nodes: every version 0 .. n_ver - 1 of every register slot that some
 *     record of the kernel names as an operand, and of vcc, exec and scc;
 *     ordered by slot, then version;
 *   variable: a merge and each of its arguments are one variable (the
 *     variable made at the join); the classes of that relation;
 *   type class: the same, plus a move's destination dword with the source
 *     dword it copies, and v_cndmask_b32's result with each of its two values;
 *   the representative of a class is its first node;
 *   type of a node: the union over its type class of the type each
 *     definition gives its destination dwords and each use gives the
 *     registers it reads:
 *       definition: the first type suffix of the mnemonic (i -> INT, u ->
 *       UINT, f32 -> FLOAT, f64 -> DOUBLE; b and no suffix: none); a scalar
 *       load through the kernel-argument pointer (s4 and s5 both at version
 *       0) at dword offset o: UINT for the global offsets (o < 0x18) and the
 *       work dimension (0x20010), none for the other hidden slots
 *       (0x18 <= o < 0x30), else the type of the .arg covering o (none when
 *       no argument does);
 *       use: a mnemonic whose last suffix is typed gives that type to every
 *       register it reads as an explicit source; a global or flat access's
 *       address registers are pointers (the saddr pair when the record has
 *       one, its vaddr then being an unsigned offset); an LDS address and an
 *       s_load base are unsigned and pointer respectively;
 *   live: a node a reachable instruction reads, or an argument of a live
 *     merge; a live merge is a variable the method creates.
 */
typedef struct { uint16_t slot; uint8_t type, flags; uint32_t version, var, tclass; } or_var;
#define VF_MERGE 1
#define VF_LIVE 2

static int suffix_type(const char *tok, int n) {
    if (n < 2 || !(tok[0] == 'i' || tok[0] == 'u' || tok[0] == 'f' || tok[0] == 'b')) return -1;
    for (int j = 1; j < n; j++)
        if (tok[j] < '0' || tok[j] > '9') return -1;
    if (tok[0] == 'i') return TY_INT;
    if (tok[0] == 'u') return TY_UINT;
    if (tok[0] == 'f') return (n == 3 && tok[1] == '6' && tok[2] == '4') ? TY_DOUBLE : TY_FLOAT;
    return 0;   /* b: bits, no type */
}

/* the first and last type suffix of a mnemonic ("v_cvt_f32_u32": FLOAT, UINT) */
static void mnemonic_types(const char *name, int *first, int *last) {
    *first = *last = -1;
    const char *p = name;
    while (*p) {
        const char *q = p;
        while (*q && *q != '_') q++;
        const int t = suffix_type(p, (int)(q - p));
        if (t >= 0) {
            if (*first < 0) *first = t;
            *last = t;
        }
        p = *q ? q + 1 : q;
    }
    if (*first < 0) *first = 0;
    if (*last < 0) *last = 0;
}

static uint32_t uf_find(uint32_t *par, uint32_t x) {
    while (par[x] != x) x = par[x];
    return x;
}
static void uf_union(uint32_t *par, uint32_t a, uint32_t b) {
    a = uf_find(par, a);
    b = uf_find(par, b);
    if (a < b) par[b] = a;
    else if (b < a) par[a] = b;
}

static uint8_t smem_arg_type(const or_kernel *K, const or_arg *args, uint32_t o) {
    if (o < 0x18) return TY_UINT;
    if (o < 0x30) return 0;
    if (o == 0x20010) return TY_UINT;
    for (unsigned k = 0; k < K->n_args; k++)
        if ((uint64_t)args[k].offset <= o && (uint64_t)o < (uint64_t)args[k].offset + args[k].size) return args[k].type;
    return 0;
}

typedef struct {
    int32_t status;
    uint32_t n_nodes, n_vars, n_tclasses, n_live_merges, n_ternary;
    uint64_t digest;
    or_var *nodes;
} or_types_out;

int or_types(const or_kernel *K, const or_instr *I, const or_arg *args, or_types_out *R) {
    memset(R, 0, sizeof(*R));
    or_ssa_out S;
    or_ssa(K, I, &S);
    R->status = S.status;
    if (S.status != OK) {
        or_ssa_free(&S);
        return R->status;
    }
    const uint32_t n = K->n_instr;
    /* the slots the records name, plus vcc, exec and scc */
    uint8_t named[NSLOT];
    memset(named, 0, sizeof(named));
    for (unsigned v = 104; v <= 108; v++) named[v] = 1;
    for (uint32_t i = 0; i < n; i++) {
        const opinfo *o = &OPS[I[i].op];
        const enum role roles[4] = {o->r0, o->r1, o->r2, o->src2};
        const unsigned ids[4] = {I[i].r0, I[i].r1, I[i].r2, (unsigned)I[i].imm};
        const int ws[4] = {o->w0, o->w1, o->w2, o->w_src2};
        for (int q = 0; q < 4; q++) {
            if (roles[q] == NO) continue;
            for (int j = 0; j < ws[q]; j++)
                if (ids[q] < NSLOT && ids[q] + (unsigned)j < NSLOT) named[ids[q] + (unsigned)j] = 1;
        }
    }
    uint32_t base[NSLOT], N = 0;
    for (unsigned v = 0; v < NSLOT; v++) {
        base[v] = N;
        if (named[v]) N += S.n_ver[v];
    }
    R->n_nodes = N;
    R->nodes = (or_var *)calloc(N ? N : 1, sizeof(or_var));
    uint32_t *pv = (uint32_t *)malloc(sizeof(uint32_t) * (N ? N : 1));   /* variable classes */
    uint32_t *pt = (uint32_t *)malloc(sizeof(uint32_t) * (N ? N : 1));   /* type classes */
    uint8_t *ty = (uint8_t *)calloc(N ? N : 1, 1);
    uint8_t *live = (uint8_t *)calloc(N ? N : 1, 1);
    for (unsigned v = 0; v < NSLOT; v++)
        if (named[v])
            for (uint32_t x = 0; x < S.n_ver[v]; x++) {
                R->nodes[base[v] + x].slot = (uint16_t)v;
                R->nodes[base[v] + x].version = x;
            }
    for (uint32_t x = 0; x < N; x++) pv[x] = pt[x] = x;

    /* merges: one variable with each argument */
    for (uint32_t p = 0; p < S.n_phi; p++) {
        const uint32_t m = base[S.phi[p].slot] + S.phi[p].version;
        R->nodes[m].flags |= VF_MERGE;
        for (uint32_t a = S.phi_arg_off[p]; a < S.phi_arg_off[p + 1]; a++) {
            const uint32_t y = base[S.phi[p].slot] + S.phi_arg[a];
            uf_union(pv, m, y);
            uf_union(pt, m, y);
        }
    }
    /* instructions: types of definitions and uses, copies, ternaries */
    for (uint32_t i = 0; i < n; i++) {
        const or_instr *X = &I[i];
        const opinfo *o = &OPS[X->op];
        unsigned us[SSA_NU], ds[SSA_ND];
        const int nu = ssa_uses(X, us), nd = ssa_defs(X, ds);
        const uint32_t *uv = S.use_ver + (uint64_t)i * SSA_NU, *dv = S.def_ver + (uint64_t)i * SSA_ND;
        if (nd > 0 && dv[0] == SSA_NONE) continue;   /* unreachable */
        if (nu > 0 && uv[0] == SSA_NONE) continue;
        int tfirst, tlast;
        mnemonic_types(o->name, &tfirst, &tlast);
        /* the type each use gives: walk the explicit sources as ssa_uses does */
        const enum role roles[4] = {o->r1, o->r2, o->src2, o->r0};
        const unsigned ids[4] = {X->r1, X->r2, (unsigned)X->imm & 0xFFFFu, X->r0};
        const int ws[4] = {o->w1, o->w2, o->w_src2, o->w0};
        const int has_saddr = o->r2 == SADDR && X->r2 < NSLOT;
        int q = 0;
        int first_use[4] = {-1, -1, -1, -1};   /* use index of each operand's first dword */
        for (int f = 0; f < 4; f++) {
            const enum role r = roles[f];
            if (r == NO || r == SD || r == VD) continue;
            if (f == 2 && o->src2 == NO) continue;
            for (int j = 0; j < ws[f]; j++) {
                if (!(ids[f] < NSLOT && ids[f] + (unsigned)j < NSLOT)) continue;
                if (j == 0) first_use[f] = q;
                uint8_t t = 0;
                if (o->cls == C_GLOAD || o->cls == C_GSTORE || o->cls == C_FLOAD || o->cls == C_FSTORE) {
                    if (f == 0) t = has_saddr ? TY_UINT : TY_PTR;   /* vaddr */
                    else if (f == 1) t = TY_PTR;                     /* saddr */
                } else if (o->cls == C_DSREAD || o->cls == C_DSWRITE) {
                    if (f == 0) t = TY_UINT;
                } else if (o->cls == C_SMEM) {
                    t = TY_PTR;
                } else if (f != 3) {
                    t = (uint8_t)tlast;
                }
                const uint32_t node = base[us[q]] + uv[q];
                ty[node] |= t;
                live[node] = 1;
                q++;
            }
        }
        for (; q < nu; q++) live[base[us[q]] + uv[q]] = 1;   /* implicit uses */
        /* the type each definition gives its destination dwords */
        const int nexp = (o->r0 == SD || o->r0 == VD) ? o->w0 : 0;
        for (int j = 0; j < nexp; j++) {
            const uint32_t node = base[ds[j]] + dv[j];
            uint8_t t = (uint8_t)tfirst;
            if (o->cls == C_SMEM) {
                t = 0;
                if (X->r1 == 4 && uv[0] == 0 && uv[1] == 0)
                    t = smem_arg_type(K, args, (uint32_t)X->imm + 4u * (uint32_t)j);
            }
            ty[node] |= t;
        }
        /* copies and the ternary */
        if (o->trule == T_MOVE && first_use[0] >= 0)
            for (int j = 0; j < nexp && j < o->w1; j++)
                uf_union(pt, base[ds[j]] + dv[j], base[us[first_use[0] + j]] + uv[first_use[0] + j]);
        if (o->prule == R_SEL) {
            R->n_ternary++;
            for (int f = 0; f < 2; f++)
                if (first_use[f] >= 0) uf_union(pt, base[ds[0]] + dv[0], base[us[first_use[f]]] + uv[first_use[f]]);
        }
    }
    /* live merges: repeat until no argument of a live merge turns live */
    for (int changed = 1; changed;) {
        changed = 0;
        for (uint32_t p = 0; p < S.n_phi; p++) {
            const uint32_t m = base[S.phi[p].slot] + S.phi[p].version;
            if (!live[m]) continue;
            for (uint32_t a = S.phi_arg_off[p]; a < S.phi_arg_off[p + 1]; a++) {
                const uint32_t y = base[S.phi[p].slot] + S.phi_arg[a];
                if (!live[y]) { live[y] = 1; changed = 1; }
            }
        }
    }
    /* the type of a class is the union over its members */
    uint8_t *cty = (uint8_t *)calloc(N ? N : 1, 1);
    for (uint32_t x = 0; x < N; x++) cty[uf_find(pt, x)] |= ty[x];
    uint64_t h = 0;
    for (uint32_t x = 0; x < N; x++) {
        or_var *V = &R->nodes[x];
        V->var = uf_find(pv, x);
        V->tclass = uf_find(pt, x);
        V->type = cty[V->tclass];
        if (live[x]) V->flags |= VF_LIVE;
        R->n_vars += V->var == x;
        R->n_tclasses += V->tclass == x;
        R->n_live_merges += (V->flags & (VF_MERGE | VF_LIVE)) == (VF_MERGE | VF_LIVE);
        h += ssa_item(6, x, ((uint64_t)V->var << 32) | V->tclass);
        h += ssa_item(7, x, ((uint64_t)V->slot << 48) | ((uint64_t)V->version << 16) | ((uint64_t)V->type << 8) | V->flags);
    }
    R->digest = h;
    free(pv); free(pt); free(ty); free(live); free(cty);
    or_ssa_free(&S);
    return OK;
}

void or_types_free(or_types_out *R) { free(R->nodes); R->nodes = 0; }

/* Batch driver: per kernel status, nodes, variables, type classes, live
 * merges, ternaries and digest. */
typedef struct {
    int32_t status;
    uint32_t n_nodes, n_vars, n_tclasses, n_live_merges, n_ternary;
    uint64_t digest;
} or_types_summary;

int or_types_batch(const or_kernel *kernels, uint32_t n_kernels, const or_instr *instrs, const or_arg *args,
                   or_types_summary *sum) {
    for (uint32_t k = 0; k < n_kernels; k++) {
        or_types_out R;
        or_types(&kernels[k], instrs + kernels[k].instr_begin, args + kernels[k].arg_begin, &R);
        memset(&sum[k], 0, sizeof(sum[k]));
        sum[k].status = R.status;
        if (R.status == OK) {
            sum[k].n_nodes = R.n_nodes;
            sum[k].n_vars = R.n_vars;
            sum[k].n_tclasses = R.n_tclasses;
            sum[k].n_live_merges = R.n_live_merges;
            sum[k].n_ternary = R.n_ternary;
            sum[k].digest = R.digest;
        }
        or_types_free(&R);
    }
    return 0;
}
