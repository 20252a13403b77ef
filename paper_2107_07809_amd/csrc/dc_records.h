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
/* Written as selects over all the conditions rather than as branches: the
 * lanes of a wavefront check different records, and branching on each lane's
 * role and width costs more in exec-mask work than evaluating everything. */
__device__ __forceinline__ bool sreg_ok(uint32_t id, uint32_t w) {
    const bool w1 = (id <= 107u) | (id == 109u);
    const bool w2 = ((id & 1u) == 0) & ((id <= 102u) | (id == 104u) | (id == 106u));
    const bool w4 = ((id & 3u) == 0) & (id <= 100u);
    return ((w == 1u) & w1) | ((w == 2u) & w2) | ((w == 4u) & w4);
}
__device__ __forceinline__ bool vreg_ok(uint32_t id, uint32_t w) { return (id >= 112u) & (id + w <= 368u); }
__device__ __forceinline__ bool inl_ok(uint32_t id) {
    return ((id >= 0x8000u) & (id <= 0x8050u)) | ((id >= 0x8060u) & (id <= 0x8067u));
}
__device__ __forceinline__ bool role_ok(uint32_t role, uint32_t id, uint32_t w, bool lit) {
    const bool none = id == 0xFFFFu, s = sreg_ok(id, w), v = vreg_ok(id, w), c = inl_ok(id) | (lit & (id == 0xFFFEu));
    const bool saddr = none | (sreg_ok(id, 2) & (id <= 102u));
    bool ok = false;
    ok = role == RO_NO ? none : ok;
    ok = (role == RO_SD) | (role == RO_SU) ? s : ok;
    ok = role == RO_SC ? s | c : ok;
    ok = (role == RO_VD) | (role == RO_VU) ? v : ok;
    ok = role == RO_VC ? v | s | c : ok;
    ok = role == RO_SADDR ? saddr : ok;
    return ok;
}
/* 0 ok, 1 bad opcode, 2 bad operand, 3 bad target (the first that applies) */
__device__ __forceinline__ uint32_t check_record(uint32_t op, uint32_t r0, uint32_t r1, uint32_t r2, int32_t imm,
                                                 int32_t target, uint32_t n) {
    const bool bad_op = op >= (uint32_t)N_OPS;
    const uint64_t e = OPTAB[bad_op ? 0u : op];
    const uint32_t cls = e_cls(e);
    const uint32_t w0 = e_width(e, 0);
    const bool smem_ok = sreg_ok(r0, w0) & (r0 + w0 <= 104u) & sreg_ok(r1, 2) & (r1 <= 102u) & (r2 == 0xFFFFu);
    const bool lit = !e_immoff(e) && e_role(e, 3) == RO_NO;
    const bool has3 = e_role(e, 3) != RO_NO;
    const bool ok3 = !has3 | ((imm >= 0) & (imm <= 0xFFFF) &
                              role_ok(e_role(e, 3), (uint32_t)imm & 0xFFFFu, e_width(e, 3), false));
    const bool gen_ok = role_ok(e_role(e, 0), r0, w0, false) & role_ok(e_role(e, 1), r1, e_width(e, 1), lit) &
                        role_ok(e_role(e, 2), r2, e_width(e, 2), lit) & ok3;
    const bool opd_ok = cls == C_SMEM ? smem_ok : gen_ok;
    const bool br = (cls == C_BR) | (cls == C_CBR);
    const bool tgt_ok = br ? (target >= 0) & ((uint32_t)target < n) : target == -1;
    return bad_op ? 1u : (!opd_ok ? 2u : (!tgt_ok ? 3u : 0u));
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
