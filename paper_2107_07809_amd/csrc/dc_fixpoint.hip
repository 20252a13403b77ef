/*
 * dc_fixpoint.hip -- the analysis proper on gfx950: the register-state fixpoint of
 * every kernel of a batch (Section "Statement of the problem", steps 2 and 3:
 * registers initialised from the ABI, then instruction processing over the
 * control flow graph that determines, per register, where its value came from
 * and what type it carries), and the extraction of memory accesses and
 * work-item built-ins (Section "Search for memory accesses") with the types of
 * Section "Data type recovery".
 *
 * Layout of the work.  A persistent grid; one wavefront takes one kernel at a
 * time from an atomic counter.  Per kernel:
 *
 *   1. Compact slots.  The lanes mark every register slot the kernel's records
 *      name (plus vcc, exec, scc and the argument pointer s[4:5]); a ballot
 *      prefix numbers them.  A slot no record names keeps its ABI entry value
 *      on every path, so only the U named slots are carried (U <= 368).
 *   2. Block state in LDS.  A visit loads the block's IN state from the HBM
 *      arena into LDS tables (provenance and type bits; payload).
 *   3. Chunks of 64 instructions, one per lane.  Each lane finds, for every
 *      source dword of its instruction, the latest earlier definition in the
 *      chunk (a per-slot bit mask of defining lanes) or else the block state.
 *      Provenance, type bits and two liveness bits of every definition (can
 *      the payload be other than TOP; other than TOP and uninitialised) then
 *      follow from a few lane-parallel passes over that def-use graph: the
 *      graph is acyclic, so the passes reach its unique solution after as many
 *      passes as the longest def-use chain.
 *   4. Payloads.  Only instructions whose result can be other than TOP run
 *      their payload rule; every rule gives TOP when one of its inputs is TOP
 *      (and, except the move and select rules, when one is uninitialised), so
 *      the others are TOP without evaluation.  The rules run lane-parallel by
 *      levels of the chunk's def-use graph: a lane runs once every lane whose
 *      definition it reads has run.
 *   5. Emission on every visit.  The lanes build the chunk's access and
 *      built-in records and write them compacted (ballot prefix) into the
 *      block's region of the sparse outputs; a block's last visit runs on its
 *      fixpoint IN state, so the last write is the result and no extraction
 *      walk is needed.  The last definition of each slot goes back to the block
 *      state.
 *   6. Joins.  The OUT state is joined lane-parallel into each successor's IN
 *      state in the arena; a ballot detects change and marks the successor
 *      dirty in a bitmap over reverse-postorder positions.  Passes sweep that
 *      bitmap in order (the round-robin schedule).
 *
 * Control flow in the wave-uniform parts depends only on uniform values
 * (readlane / readfirstlane results and loop counters).  Lane-dependent
 * choices are selects: a store that only some lanes should make is a store by
 * every lane whose address is the real one or a per-lane scratch word.  A
 * lane-predicated branch around uniform code lets the optimiser thread the
 * predicate across a loop back edge and split the wave.  LDS accesses of one
 * wavefront execute in order, which orders the lanes' table writes and reads;
 * the wave barriers mark those points (they emit no instruction).
 */
#include "dc_fixpoint_core.h"

namespace dc {

/* Persistent grid.  Main pass: kernels whose blocks fit the register bitmap
 * and whose IN states fit the wave's arena; the others are queued for the
 * overflow pass, which keeps its bitmaps in HBM and has a larger arena. */
template <bool OVF>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_fixpoint(const Plan *__restrict__ P, uint32_t wpg) {
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
    L.optab[l] = OPTAB[l < (uint32_t)N_OPS ? l : 0];
    L.optab[l < 16 ? 64 + l : l] = OPTAB[l < 16 && 64 + l < (uint32_t)N_OPS ? 64 + l : (l < (uint32_t)N_OPS ? l : 0)];
    __builtin_amdgcn_wave_barrier();
    for (;;) {
        /* branch-free: every lane takes part, only lane 0 adds 1 */
        const uint32_t idx = rfl(atomicAdd(&P->counters[OVF ? 2 : 0], l == 0 ? 1u : 0u));
        const uint32_t limit = OVF ? rfl(P->counters[1]) : P->n_kernels;
        if (idx >= limit) break;
        const uint32_t k = OVF ? rfl(P->ovf_list[idx]) : (P->work_order ? rfl(P->work_order[idx]) : idx);
        const int32_t status = (int32_t)rfl((uint32_t)P->status[k]);
        if (status != ST_OK_FIX) {
            fail_kernel(P, k, status, M);
            continue;
        }
        const uint32_t nb = rfl(P->n_blocks[k]);
        const uint32_t nu = rfl(build_compact(P, L, k));
        const uint64_t rows = (uint64_t)nb * ((nu + 63u) >> 6);
        if (!OVF) {
            if (nb > MAIN_MAX_BLOCKS || rows > cap_rows) {
                const uint32_t slot = rfl(atomicAdd(&P->counters[1], l == 0 ? 1u : 0u));
                *(l == 0 ? &P->ovf_list[slot] : reinterpret_cast<uint32_t *>(M.dummy + l)) = k;
                continue;
            }
            RegBits reached, dirty;
            analyze(P, k, L, reached, dirty, M, nu);
        } else {
            if (nb > P->ovf_block_cap || rows > cap_rows) {   /* more blocks than the pass was planned for */
                fail_kernel(P, k, DC_E_CAPACITY, M);
                continue;
            }
            const uint32_t words = (P->ovf_block_cap + 31) >> 5;
            uint32_t *bm = P->ovf_bitmaps + (uint64_t)gw * (2 * words + 64);
            MemBits reached{bm, bm + 2 * words}, dirty{bm + words, bm + 2 * words};
            analyze(P, k, L, reached, dirty, M, nu);
        }
    }
}

size_t fixpoint_lds_per_wave() { return sizeof(WaveLds); }

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
    hipLaunchKernelGGL(k_fixpoint<true>, dim3(P.ovf_waves), dim3(64), sizeof(WaveLds), s, dP, 1u);
    e = hipGetLastError();
    if (e == hipSuccess && after) e = hipEventRecord(after, s);
    return e;
}

}  // namespace dc
