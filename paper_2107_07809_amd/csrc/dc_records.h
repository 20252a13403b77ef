/* dc_records.h -- per-record device checks shared by the batch stages
 * (dc_kernels.hip) and the one-launch-per-kernel form (dc_plain.hip): operand
 * validity for each role, the record check with its status code, block ends,
 * and the record capacity of an instruction. */
#pragma once
#include "dc_device.h"

namespace dc {

/* ------------------------------------------------------------------ */
/* record checks (per thread)                                           */
/* ------------------------------------------------------------------ */
__device__ inline bool sreg_ok(uint32_t id, uint32_t w) {
    switch (w) {
    case 1: return id <= 107u || id == 109u;
    case 2: return (id & 1u) == 0 && (id <= 102u || id == 104u || id == 106u);
    case 4: return (id & 3u) == 0 && id <= 100u;
    }
    return false;
}
__device__ inline bool vreg_ok(uint32_t id, uint32_t w) { return id >= 112u && id + w <= 368u; }
__device__ inline bool inl_ok(uint32_t id) {
    return (id >= 0x8000u && id <= 0x8050u) || (id >= 0x8060u && id <= 0x8067u);
}
__device__ inline bool role_ok(uint32_t role, uint32_t id, uint32_t w, bool lit) {
    switch (role) {
    case RO_NO: return id == 0xFFFFu;
    case RO_SD:
    case RO_SU: return sreg_ok(id, w);
    case RO_SC: return sreg_ok(id, w) || inl_ok(id) || (lit && id == 0xFFFEu);
    case RO_VD:
    case RO_VU: return vreg_ok(id, w);
    case RO_VC: return vreg_ok(id, w) || sreg_ok(id, w) || inl_ok(id) || (lit && id == 0xFFFEu);
    case RO_SADDR: return id == 0xFFFFu || (sreg_ok(id, 2) && id <= 102u);
    }
    return false;
}
/* 0 ok, 1 bad opcode, 2 bad operand, 3 bad target */
__device__ inline uint32_t check_record(uint32_t op, uint32_t r0, uint32_t r1, uint32_t r2, int32_t imm, int32_t target,
                                 uint32_t n) {
    if (op >= (uint32_t)N_OPS) return 1;
    const uint64_t e = OPTAB[op];
    const uint32_t cls = e_cls(e);
    if (cls == C_SMEM) {
        const uint32_t w = e_width(e, 0);
        if (!(sreg_ok(r0, w) && r0 + w <= 104u)) return 2;
        if (!(sreg_ok(r1, 2) && r1 <= 102u)) return 2;
        if (r2 != 0xFFFFu) return 2;
    } else {
        const bool lit = !e_immoff(e) && e_role(e, 3) == RO_NO;
        if (!role_ok(e_role(e, 0), r0, e_width(e, 0), false)) return 2;
        if (!role_ok(e_role(e, 1), r1, e_width(e, 1), lit)) return 2;
        if (!role_ok(e_role(e, 2), r2, e_width(e, 2), lit)) return 2;
        if (e_role(e, 3) != RO_NO) {
            if (imm < 0 || imm > 0xFFFF) return 2;
            if (!role_ok(e_role(e, 3), (uint32_t)imm, e_width(e, 3), false)) return 2;
        }
    }
    if (cls == C_BR || cls == C_CBR) {
        if (target < 0 || (uint32_t)target >= n) return 3;
    } else if (target != -1) {
        return 3;
    }
    return 0;
}
__device__ inline bool ends_block(uint32_t cls) { return cls == C_BR || cls == C_CBR || cls == C_END; }

/* Record capacity of one instruction: one access record for a memory
 * instruction; one built-in record per explicit definition dword of a rule
 * that can yield a work-item built-in (moves, selects, adds, multiplies,
 * shifts, argument loads).  The other rules yield only constants, pointer
 * halves, sign words or unknowns, none of which is a built-in.  Packed as
 * bit 0 (access) and bits 3:1 (built-ins). */
__device__ inline uint32_t rec_cap(uint64_t e) {
    const uint32_t cls = e_cls(e), pr = e_prule(e), r0 = e_role(e, 0);
    const uint32_t acc = cls >= C_GLD ? 1u : 0u;
    const bool alu = cls == C_SALU || cls == C_VALU;
    const bool can = cls == C_SMEM || (alu && (pr == PR_MOV || pr == PR_SEL || pr == PR_ADD || pr == PR_MUL ||
                                               pr == PR_MUL24 || pr == PR_MAD24 || pr == PR_SHL || pr == PR_LSHR ||
                                               pr == PR_SHL64));
    const uint32_t sys = can && (r0 == RO_SD || r0 == RO_VD) ? e_width(e, 0) : 0u;
    return acc | sys << 1;
}

}  // namespace dc
