/* dc_ssa_ops.h -- the operands of a record as the version stages read
 * them (uses and definitions in their fixed order) and the wavefront sums
 * they share. */
#pragma once
#include "dc_device.h"

namespace dc {

/* ------------------------------------------------------------------ */
/* operands                                                              */
/* ------------------------------------------------------------------ */
struct Rec {
    uint64_t e;
    uint32_t id[4];   /* r0, r1, r2, third source */
};
__device__ __forceinline__ Rec load_rec(const Plan &P, const dc_kernel_t &D, uint32_t i) {
    const uint4 r = reinterpret_cast<const uint4 *>(P.instrs)[D.instr_begin + i];
    Rec x;
    x.e = OPTAB[r.x & 0xFFFFu];
    x.id[0] = r.x >> 16;
    x.id[1] = r.y & 0xFFFFu;
    x.id[2] = r.y >> 16;
    x.id[3] = r.z & 0xFFFFu;
    return x;
}

/* f(q, slot) for each register slot the instruction reads: the dwords of
 * r1, r2, the third source and a stored r0 that name slots, then the
 * implicit vcc, exec, scc uses */
template <typename F>
__device__ __forceinline__ uint32_t for_uses(const Rec &x, F f) {
    uint32_t q = 0;
    const int order[4] = {1, 2, 3, 0};
#pragma unroll
    for (int t = 0; t < 4; t++) {
        const int o = order[t];
        const uint32_t role = e_role(x.e, o);
        if (role == RO_NO || role == RO_SD || role == RO_VD) continue;
        const uint32_t w = e_width(x.e, o), v = x.id[o];
#pragma unroll
        for (uint32_t j = 0; j < 4; j++)
            if (j < w && v + j < (uint32_t)NSLOT) f(q++, v + j);
    }
    const uint32_t iu = e_iuse(x.e);
    if (iu & IM_VCC) {
        f(q++, 104u);
        f(q++, 105u);
    }
    if (iu & IM_EXEC) {
        f(q++, 106u);
        f(q++, 107u);
    }
    if (iu & IM_SCC) f(q++, 108u);
    return q;
}

/* f(q, slot, again) for each definition: the destination dwords, then the
 * implicit vcc, exec, scc; again = 1 when the destination already wrote the
 * slot in this instruction (an implicit pair that the destination names) */
template <typename F>
__device__ __forceinline__ uint32_t for_defs(const Rec &x, F f) {
    uint32_t q = 0;
    const uint32_t r0 = e_role(x.e, 0);
    const bool ex = r0 == RO_SD || r0 == RO_VD;
    const uint32_t w0 = ex ? e_width(x.e, 0) : 0u, v0 = x.id[0];
#pragma unroll
    for (uint32_t j = 0; j < 4; j++)
        if (j < w0) f(q++, v0 + j, 0u);
    auto again = [&](uint32_t v) { return (ex && v >= v0 && v < v0 + w0) ? 1u : 0u; };
    const uint32_t idf = e_idef(x.e);
    if (idf & IM_VCC) {
        f(q++, 104u, again(104u));
        f(q++, 105u, again(105u));
    }
    if (idf & IM_EXEC) {
        f(q++, 106u, again(106u));
        f(q++, 107u, again(107u));
    }
    if (idf & IM_SCC) f(q++, 108u, again(108u));
    return q;
}
__device__ __forceinline__ uint32_t n_uses(const Rec &x) {
    return for_uses(x, [](uint32_t, uint32_t) {});
}
__device__ __forceinline__ uint32_t n_defs(const Rec &x) {
    return for_defs(x, [](uint32_t, uint32_t, uint32_t) {});
}

/* ------------------------------------------------------------------ */
/* wavefront helpers                                                     */
/* ------------------------------------------------------------------ */
__device__ __forceinline__ uint64_t ssa_item(uint64_t kind, uint64_t index, uint64_t value) {
    return mix64(mix64(kind * 0x9E3779B97F4A7C15ull + index) ^ value);
}
__device__ __forceinline__ uint64_t wave_sum64(uint64_t x) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
    return x;
}
__device__ __forceinline__ uint32_t wave_sum32(uint32_t x) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
    return x;
}
/* exclusive prefix over the lanes; *total = the sum over all lanes */
__device__ __forceinline__ uint32_t wave_excl(uint32_t x, uint32_t *total) {
    const uint32_t l = lane_id();
    uint32_t y = x;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t t = __shfl_up(y, d, 64);
        if (l >= (uint32_t)d) y += t;
    }
    *total = __shfl(y, 63, 64);
    return y - x;
}

}  // namespace dc
