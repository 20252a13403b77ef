/* dc_isa.h -- the instruction subset as the GPU path sees it: one packed
 * 64-bit descriptor per opcode (class, operand roles and widths, implicit
 * registers, type rule, payload rule), plus the payload encoding.
 *
 * Mnemonic decomposition follows Section "The body extraction": a prefix
 * (s, v, ds, flat/global) selects the unit, the type suffix (i, u, f, b with
 * a size) gives the result type (Section "Data type recovery"). */
#pragma once
#include <stdint.h>

namespace dc {

/* instruction classes */
enum : uint32_t { C_SMEM, C_SALU, C_SCMP, C_BR, C_CBR, C_NOP, C_END, C_VALU, C_VCMP, C_GLD, C_GST, C_FLD, C_FST,
                  C_DSR, C_DSW };
/* operand roles */
enum : uint32_t { RO_NO, RO_SD, RO_SU, RO_SC, RO_VD, RO_VU, RO_VC, RO_SADDR };
/* type rules */
enum : uint32_t { TR_NONE, TR_SUF, TR_ADD, TR_B, TR_MOVE, TR_SMEM };
/* payload rules */
enum : uint32_t { PR_TOP, PR_SMEM, PR_MOV, PR_ADD, PR_ADDC, PR_SUB, PR_MUL, PR_MUL24, PR_MAD24, PR_SHL, PR_LSHR,
                  PR_ASHR, PR_AND, PR_OR, PR_XOR, PR_AND64, PR_OR64, PR_XOR64, PR_ANDN264, PR_SHL64, PR_SEL,
                  PR_NONE };
/* implicit register sets */
enum : uint32_t { IM_VCC = 1, IM_SCC = 2, IM_EXEC = 4 };
/* type bits */
enum : uint32_t { TY_I = 1, TY_U = 2, TY_F = 4, TY_D = 8, TY_P = 16 };

/* bit layout of a descriptor:
 *   [3:0] class  [6:4] role r0  [9:7] role r1  [12:10] role r2  [15:13] role src2
 *   [17:16] [19:18] [21:20] [23:22] width codes of r0 r1 r2 src2 (0,1,2 dwords; 3 = 4 dwords)
 *   [24] imm is a byte offset  [27:25] implicit uses  [30:28] implicit defs
 *   [33:31] type rule  [38:34] suffix type bits  [43:39] payload rule
 *   [45:44] value sources for bitwise types (1 = r1, 2 = r2, 3 = both)
 *   [46] explicit defs are exec masks */
constexpr uint64_t wcode(uint32_t w) { return w == 4 ? 3 : w; }
constexpr uint64_t OPE(uint32_t cls, uint32_t a, uint32_t b, uint32_t c, uint32_t d, uint32_t w0, uint32_t w1,
                       uint32_t w2, uint32_t w3, uint32_t immoff, uint32_t iu, uint32_t idf, uint32_t tr,
                       uint32_t suf, uint32_t pr, uint32_t vs, uint32_t md) {
    return (uint64_t)cls | (uint64_t)a << 4 | (uint64_t)b << 7 | (uint64_t)c << 10 | (uint64_t)d << 13 |
           wcode(w0) << 16 | wcode(w1) << 18 | wcode(w2) << 20 | wcode(w3) << 22 | (uint64_t)immoff << 24 |
           (uint64_t)iu << 25 | (uint64_t)idf << 28 | (uint64_t)tr << 31 | (uint64_t)suf << 34 |
           (uint64_t)pr << 39 | (uint64_t)vs << 44 | (uint64_t)md << 46;
}

#define DC_SLOAD(w) OPE(C_SMEM, RO_SD, RO_SU, RO_NO, RO_NO, w, 2, 0, 0, 1, 0, 0, TR_SMEM, 0, PR_SMEM, 0, 0)
#define DC_S2(idf, iu, tr, suf, pr, vs) OPE(C_SALU, RO_SD, RO_SC, RO_SC, RO_NO, 1, 1, 1, 0, 0, iu, idf, tr, suf, pr, vs, 0)
#define DC_S64(pr) OPE(C_SALU, RO_SD, RO_SC, RO_SC, RO_NO, 2, 2, 2, 0, 0, 0, IM_SCC, TR_B, 0, pr, 3, 0)
#define DC_SCMP OPE(C_SCMP, RO_NO, RO_SC, RO_SC, RO_NO, 0, 1, 1, 0, 0, 0, IM_SCC, TR_NONE, 0, PR_NONE, 0, 0)
#define DC_CTL(c, iu) OPE(c, RO_NO, RO_NO, RO_NO, RO_NO, 0, 0, 0, 0, 0, iu, 0, TR_NONE, 0, PR_NONE, 0, 0)
#define DC_V2(w, idf, iu, tr, suf, pr, vs) OPE(C_VALU, RO_VD, RO_VC, RO_VC, RO_NO, w, w, w, 0, 0, iu, idf, tr, suf, pr, vs, 0)
#define DC_V3(w, tr, suf, pr) OPE(C_VALU, RO_VD, RO_VC, RO_VC, RO_VC, w, w, w, w, 0, 0, 0, tr, suf, pr, 0, 0)
#define DC_V1(wd, ws, tr, suf, pr, vs) OPE(C_VALU, RO_VD, RO_VC, RO_NO, RO_NO, wd, ws, 0, 0, 0, 0, 0, tr, suf, pr, vs, 0)
#define DC_VCMP OPE(C_VCMP, RO_NO, RO_VC, RO_VC, RO_NO, 0, 1, 1, 0, 0, 0, IM_VCC, TR_NONE, 0, PR_NONE, 0, 0)

/* opcode ids are the record encoding's numbering (dc_opcode_name) */
#define DC_OPTAB_INIT                                                                                  \
    {                                                                                                  \
        DC_SLOAD(1), DC_SLOAD(2), DC_SLOAD(4),                                                        \
        OPE(C_SALU, RO_SD, RO_SC, RO_NO, RO_NO, 1, 1, 0, 0, 0, 0, 0, TR_MOVE, 0, PR_MOV, 1, 0),       \
        OPE(C_SALU, RO_SD, RO_SC, RO_NO, RO_NO, 2, 2, 0, 0, 0, 0, 0, TR_MOVE, 0, PR_MOV, 1, 0),       \
        OPE(C_SALU, RO_SD, RO_SC, RO_NO, RO_NO, 2, 2, 0, 0, 0, IM_EXEC, IM_EXEC | IM_SCC, TR_NONE, 0, PR_TOP, 0, 1), \
        OPE(C_SALU, RO_SD, RO_SC, RO_NO, RO_NO, 2, 2, 0, 0, 0, IM_EXEC, IM_EXEC | IM_SCC, TR_NONE, 0, PR_TOP, 0, 1), \
        DC_S2(IM_SCC, 0, TR_ADD, TY_U, PR_ADD, 3),      /* s_add_u32 */                                \
        DC_S2(IM_SCC, 0, TR_ADD, TY_I, PR_ADD, 3),      /* s_add_i32 */                                \
        DC_S2(IM_SCC, IM_SCC, TR_ADD, TY_U, PR_ADDC, 3), /* s_addc_u32 */                              \
        DC_S2(IM_SCC, 0, TR_SUF, TY_U, PR_SUB, 3),      /* s_sub_u32 */                                \
        DC_S2(0, 0, TR_SUF, TY_I, PR_MUL, 3),           /* s_mul_i32 */                                \
        DC_S2(IM_SCC, 0, TR_B, 0, PR_SHL, 1),           /* s_lshl_b32: value r1, amount r2 */          \
        DC_S2(IM_SCC, 0, TR_B, 0, PR_LSHR, 1),          /* s_lshr_b32 */                               \
        DC_S2(IM_SCC, 0, TR_B, 0, PR_AND, 3),                                                          \
        DC_S2(IM_SCC, 0, TR_B, 0, PR_OR, 3),                                                           \
        DC_S64(PR_AND64), DC_S64(PR_OR64), DC_S64(PR_XOR64), DC_S64(PR_ANDN264),                       \
        DC_SCMP, DC_SCMP, DC_SCMP, DC_SCMP,                                                            \
        DC_CTL(C_BR, 0), DC_CTL(C_CBR, IM_SCC), DC_CTL(C_CBR, IM_SCC), DC_CTL(C_CBR, IM_VCC),          \
        DC_CTL(C_CBR, IM_VCC), DC_CTL(C_CBR, IM_EXEC), DC_CTL(C_CBR, IM_EXEC),                         \
        DC_CTL(C_NOP, 0), DC_CTL(C_NOP, 0), DC_CTL(C_NOP, 0), DC_CTL(C_END, 0),                        \
        DC_V1(1, 1, TR_MOVE, 0, PR_MOV, 1),             /* v_mov_b32 */                                \
        DC_V1(1, 1, TR_SUF, TY_F, PR_TOP, 0),           /* v_cvt_f32_u32 */                            \
        DC_V1(1, 1, TR_SUF, TY_U, PR_TOP, 0),           /* v_cvt_u32_f32 */                            \
        DC_V1(2, 1, TR_SUF, TY_D, PR_TOP, 0),           /* v_cvt_f64_f32 */                            \
        DC_V2(1, IM_VCC, 0, TR_ADD, TY_U, PR_ADD, 3),   /* v_add_co_u32 */                             \
        DC_V2(1, IM_VCC, IM_VCC, TR_ADD, TY_U, PR_ADDC, 3),                                            \
        DC_V2(1, IM_VCC, 0, TR_SUF, TY_U, PR_SUB, 3),                                                  \
        DC_V2(1, 0, 0, TR_ADD, TY_U, PR_ADD, 3),        /* v_add_u32 */                                \
        DC_V2(1, 0, 0, TR_SUF, TY_U, PR_MUL, 3),        /* v_mul_lo_u32 */                             \
        DC_V2(1, 0, 0, TR_SUF, TY_U, PR_MUL24, 3),      /* v_mul_u32_u24 */                            \
        DC_V2(1, 0, 0, TR_SUF, TY_U, PR_TOP, 3),        /* v_mul_hi_u32 */                             \
        DC_V3(1, TR_SUF, TY_U, PR_MAD24),               /* v_mad_u32_u24 */                            \
        DC_V2(1, 0, 0, TR_B, 0, PR_SHL, 2),             /* v_lshlrev_b32: amount r1, value r2 */       \
        DC_V2(1, 0, 0, TR_B, 0, PR_LSHR, 2),                                                           \
        DC_V2(1, 0, 0, TR_SUF, TY_I, PR_ASHR, 2),                                                      \
        DC_V2(1, 0, 0, TR_B, 0, PR_AND, 3), DC_V2(1, 0, 0, TR_B, 0, PR_OR, 3),                         \
        DC_V2(1, 0, 0, TR_B, 0, PR_XOR, 3),                                                            \
        OPE(C_VALU, RO_VD, RO_VC, RO_VC, RO_NO, 2, 1, 2, 0, 0, 0, 0, TR_B, 0, PR_SHL64, 2, 0),        \
        DC_V2(1, 0, IM_VCC, TR_B, 0, PR_SEL, 3),        /* v_cndmask_b32 */                            \
        DC_V2(1, 0, 0, TR_SUF, TY_F, PR_TOP, 3), DC_V2(1, 0, 0, TR_SUF, TY_F, PR_TOP, 3),              \
        DC_V2(1, 0, 0, TR_SUF, TY_F, PR_TOP, 3), DC_V2(1, 0, 0, TR_SUF, TY_F, PR_TOP, 3),              \
        DC_V3(1, TR_SUF, TY_F, PR_TOP), DC_V3(1, TR_SUF, TY_F, PR_TOP),                                \
        DC_V2(2, 0, 0, TR_SUF, TY_D, PR_TOP, 3), DC_V2(2, 0, 0, TR_SUF, TY_D, PR_TOP, 3),              \
        DC_V3(2, TR_SUF, TY_D, PR_TOP),                                                                \
        DC_VCMP, DC_VCMP, DC_VCMP, DC_VCMP, DC_VCMP,                                                   \
        OPE(C_GLD, RO_VD, RO_VU, RO_SADDR, RO_NO, 1, 2, 2, 0, 1, 0, 0, TR_NONE, 0, PR_TOP, 0, 0),     \
        OPE(C_GLD, RO_VD, RO_VU, RO_SADDR, RO_NO, 2, 2, 2, 0, 1, 0, 0, TR_NONE, 0, PR_TOP, 0, 0),     \
        OPE(C_FLD, RO_VD, RO_VU, RO_NO, RO_NO, 1, 2, 0, 0, 1, 0, 0, TR_NONE, 0, PR_TOP, 0, 0),        \
        OPE(C_GST, RO_VU, RO_VU, RO_SADDR, RO_NO, 1, 2, 2, 0, 1, 0, 0, TR_NONE, 0, PR_NONE, 0, 0),    \
        OPE(C_GST, RO_VU, RO_VU, RO_SADDR, RO_NO, 2, 2, 2, 0, 1, 0, 0, TR_NONE, 0, PR_NONE, 0, 0),    \
        OPE(C_FST, RO_VU, RO_VU, RO_NO, RO_NO, 1, 2, 0, 0, 1, 0, 0, TR_NONE, 0, PR_NONE, 0, 0),       \
        OPE(C_DSR, RO_VD, RO_VU, RO_NO, RO_NO, 1, 1, 0, 0, 1, 0, 0, TR_NONE, 0, PR_TOP, 0, 0),        \
        OPE(C_DSW, RO_VU, RO_VU, RO_NO, RO_NO, 1, 1, 0, 0, 1, 0, 0, TR_NONE, 0, PR_NONE, 0, 0),       \
    }

/* field accessors */
__host__ __device__ constexpr uint32_t e_cls(uint64_t e) { return (uint32_t)(e & 15); }
__host__ __device__ constexpr uint32_t e_role(uint64_t e, int i) { return (uint32_t)(e >> (4 + 3 * i)) & 7; }
__host__ __device__ constexpr uint32_t e_width(uint64_t e, int i) {
    return ((uint32_t)(e >> (16 + 2 * i)) & 3) == 3 ? 4u : ((uint32_t)(e >> (16 + 2 * i)) & 3);
}
__host__ __device__ constexpr uint32_t e_immoff(uint64_t e) { return (uint32_t)(e >> 24) & 1; }
__host__ __device__ constexpr uint32_t e_iuse(uint64_t e) { return (uint32_t)(e >> 25) & 7; }
__host__ __device__ constexpr uint32_t e_idef(uint64_t e) { return (uint32_t)(e >> 28) & 7; }
__host__ __device__ constexpr uint32_t e_trule(uint64_t e) { return (uint32_t)(e >> 31) & 7; }
__host__ __device__ constexpr uint32_t e_suffix(uint64_t e) { return (uint32_t)(e >> 34) & 31; }
__host__ __device__ constexpr uint32_t e_prule(uint64_t e) { return (uint32_t)(e >> 39) & 31; }
__host__ __device__ constexpr uint32_t e_vsrc(uint64_t e) { return (uint32_t)(e >> 44) & 3; }
__host__ __device__ constexpr uint32_t e_maskdef(uint64_t e) { return (uint32_t)(e >> 46) & 1; }

/* ---- payload encoding ----
 * [63:60] tag  [59:58] integrity  [57:56] dim  [55:52] aux  [51:48] shift
 * [47:40] argument slot  [39:32] zero  [31:0] c */
enum : uint32_t { T_CONST = 0, T_SYSPTR = 1, T_KARG = 2, T_WGID = 3, T_IDX = 4, T_SHL = 5, T_PTR = 6, T_SYS = 7,
                  T_UNINIT = 8 };
enum : uint32_t { IG_ENT = 0, IG_LO = 1, IG_HI = 2 };
enum : uint32_t { K_GOFFHI = 0, K_GSIZE = 1, K_NUMGROUPS = 2, K_WORKDIM = 3, K_HIDDEN = 4 };
enum : uint32_t { M_WG = 1, M_LID = 2, M_GOFF = 4 };
constexpr uint64_t VTOP = ~0ull;

__host__ __device__ constexpr uint64_t pv(uint32_t tag, uint32_t ig, uint32_t d, uint32_t aux, uint32_t sh,
                                          uint32_t arg, uint32_t c) {
    return (uint64_t)tag << 60 | (uint64_t)ig << 58 | (uint64_t)d << 56 | (uint64_t)aux << 52 |
           (uint64_t)sh << 48 | (uint64_t)arg << 40 | (uint64_t)c;
}
__host__ __device__ constexpr uint32_t v_tag(uint64_t v) { return (uint32_t)(v >> 60); }
__host__ __device__ constexpr uint32_t v_ig(uint64_t v) { return (uint32_t)(v >> 58) & 3; }
__host__ __device__ constexpr uint32_t v_dim(uint64_t v) { return (uint32_t)(v >> 56) & 3; }
__host__ __device__ constexpr uint32_t v_aux(uint64_t v) { return (uint32_t)(v >> 52) & 15; }
__host__ __device__ constexpr uint32_t v_sh(uint64_t v) { return (uint32_t)(v >> 48) & 15; }
__host__ __device__ constexpr uint32_t v_arg(uint64_t v) { return (uint32_t)(v >> 40) & 255; }
__host__ __device__ constexpr uint32_t v_c(uint64_t v) { return (uint32_t)v; }

/* provenance bits */
enum : uint32_t {
    PB_LID = 0, PB_WGID = 3, PB_GOFF = 6, PB_GSIZE = 9, PB_WORKDIM = 12, PB_SYSPTR = 13, PB_CONST = 14,
    PB_LOADG = 15, PB_LOADL = 16, PB_UNINIT = 17, PB_MASK = 18, PB_HIDDEN = 19, PB_KARG = 20
};

}  // namespace dc
