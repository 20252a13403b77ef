/*
 * dc_plain.hip -- the plain form of the analysis: one launch per analysed
 * kernel, in which one workgroup runs every stage for that kernel (records
 * checked and decoded, leaders, block numbering and record regions, edges,
 * predecessor lists, reverse postorder, the fixpoint with extraction on its
 * first wavefront, dense output).  It is the form a batch of one would take
 * without batching, kept as the comparison point for the batched persistent
 * form (DC_OPT_PLAIN of dc_analyze_batch).
 *
 * The launches of a batch run one after another on its stream and share one
 * scratch plan sized for the batch's longest kernel (block arrays for one
 * block per instruction, regions for one access and four built-in records
 * per instruction, an arena for six state rows per block).  Each launch
 * appends its kernel's records to the batch's dense outputs at the running
 * totals the previous launch left in counters[4] and counters[5], so the
 * per-kernel offsets are exact without a scan over the batch.
 */
#include "dc_fixpoint_core.h"
#include "dc_records.h"

namespace dc {

constexpr uint32_t PL_T = 256;   /* threads of the plain workgroup */

/* exclusive scan of x across the workgroup; *total = the sum */
__device__ __forceinline__ uint32_t pl_scan(uint32_t x, uint32_t *total, uint32_t *wsum) {
    const uint32_t w = threadIdx.x >> 6, l = lane_id();
    uint32_t inc = x;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(inc, d, 64);
        inc += l >= (uint32_t)d ? y : 0u;
    }
    if (l == 63) wsum[w] = inc;
    __syncthreads();
    uint32_t base = 0, tot = 0;
    for (uint32_t j = 0; j < PL_T / 64; j++) {
        base += j < w ? wsum[j] : 0u;
        tot += wsum[j];
    }
    __syncthreads();
    *total = tot;
    return base + inc - x;
}

__global__ __launch_bounds__(PL_T) void k_plain(const Plan *__restrict__ P, uint32_t k) {
    extern __shared__ uint4 smem[];
    WaveLds &L = *reinterpret_cast<WaveLds *>(smem);
    __shared__ uint32_t s_bad, s_km[KSLOT_WORDS], s_wsum[PL_T / 64], s_nreach;
    const uint32_t tid = threadIdx.x;
    const dc_kernel_t D = P->kernels[k];
    const uint32_t n = D.n_instr, pos0 = P->pos_begin[k];
    const uint4 *recs = reinterpret_cast<const uint4 *>(P->instrs) + D.instr_begin;
    const uint32_t out_a = P->counters[4], out_s = P->counters[5];

    /* decode, record checks, leaders, capacities, named slots */
    for (uint32_t i = tid; i < n; i += PL_T) P->leader[i] = 0;
    if (tid == 0) s_bad = 0xFFFFFFFFu;
    if (tid < KSLOT_WORDS) s_km[tid] = 0;
    __syncthreads();
    for (uint32_t i = tid; i < n; i += PL_T) {
        const uint4 r = recs[i];
        const uint32_t op = r.x & 0xFFFFu, r0 = r.x >> 16, r1 = r.y & 0xFFFFu, r2 = r.y >> 16;
        const int32_t imm = (int32_t)r.z, target = (int32_t)r.w;
        const uint32_t bad = check_record(op, r0, r1, r2, imm, target, n);
        if (i == 0) P->leader[0] = 1;
        if (bad) {
            P->pcap[i] = 0;
            atomicMin(&s_bad, (i << 2) | bad);
            continue;
        }
        const uint64_t e = OPTAB[op];
        const uint32_t cls = e_cls(e);
        P->pcap[i] = (uint8_t)rec_cap(e);
        if (ends_block(cls) && i + 1 < n) P->leader[i + 1] = 1;
        if (cls == C_BR || cls == C_CBR) P->leader[(uint32_t)target] = 1;
        const uint32_t id[4] = {r0, r1, r2, (uint32_t)imm};
#pragma unroll
        for (int o = 0; o < 4; o++) {
            const uint32_t w = e_role(e, o) != RO_NO ? e_width(e, o) : 0u;
            if (w == 0 || id[o] >= (uint32_t)NSLOT) continue;
            const uint32_t first = id[o], last = min(id[o] + w, (uint32_t)NSLOT) - 1u;
            const uint32_t wa = first >> 5, wb = last >> 5;
            const uint32_t hi_a = wa == wb ? (last & 31u) : 31u;
            atomicOr(&s_km[wa], (0xFFFFFFFFu >> (31u - hi_a)) & (0xFFFFFFFFu << (first & 31u)));
            if (wb != wa) atomicOr(&s_km[wb], 0xFFFFFFFFu >> (31u - (last & 31u)));
        }
    }
    __syncthreads();
    int32_t st = P->desc_status[k];
    if (st == DC_OK) {
        if (s_bad != 0xFFFFFFFFu) {
            const uint32_t code = s_bad & 3u;
            st = code == 1 ? DC_E_BADOP : code == 2 ? DC_E_BADREG : DC_E_BADTARGET;
        } else if (n == 0) {
            st = DC_E_NOEND;
        } else {
            const uint32_t cls = e_cls(OPTAB[recs[n - 1].x & 0xFFFFu]);
            if (!(cls == C_BR || cls == C_END)) st = DC_E_NOEND;
        }
    }

    /* block numbering and record regions: one scan of (leader, access
     * capacity, built-in capacity) packed in 9, 10 and 12 bits */
    uint32_t nb = 0, ta = 0, ts = 0;
    if (st == DC_OK) {
        for (uint32_t c = 0; c < n; c += PL_T) {
            const uint32_t i = c + tid;
            const uint32_t ld = i < n ? P->leader[i] : 0u, cp = i < n ? P->pcap[i] : 0u;
            const uint32_t x = ld | (cp & 1u) << 9 | (cp >> 1) << 19;
            uint32_t tot;
            const uint32_t ex = pl_scan(x, &tot, s_wsum);
            const uint32_t id = nb + (ex & 0x1FFu) + ld - 1u;
            if (i < n) P->block_id[i] = id;
            if (i < n && ld) {
                P->block_start[id] = i;
                P->blk_acc_base[id] = ta + ((ex >> 9) & 0x3FFu);
                P->blk_sys_base[id] = ts + (ex >> 19);
            }
            nb += tot & 0x1FFu;
            ta += (tot >> 9) & 0x3FFu;
            ts += tot >> 19;
        }
        if (tid == 0) {
            P->block_start[nb] = n;
            P->blk_acc_base[nb] = ta;
            P->blk_sys_base[nb] = ts;
        }
        for (uint32_t b = tid; b <= nb; b += PL_T) {
            P->pred_cnt[b] = 0;
            P->pred_fill[b] = 0;
        }
        __syncthreads();

        /* successors (fall-through first) and predecessor counts */
        for (uint32_t b = tid; b < nb; b += PL_T) {
            const uint4 r = recs[P->block_start[b + 1] - 1];
            const uint32_t cls = e_cls(OPTAB[r.x & 0xFFFFu]);
            int32_t s0 = -1, s1 = -1;
            if (cls != C_BR && cls != C_END && b + 1 < nb) s0 = (int32_t)(b + 1);
            if (cls == C_BR || cls == C_CBR) s1 = (int32_t)P->block_id[(uint32_t)(int32_t)r.w];
            if (s1 == s0) s1 = -1;
            P->succ[2 * b] = s0;
            P->succ[2 * b + 1] = s1;
            if (s0 >= 0) atomicAdd(&P->pred_cnt[s0], 1u);
            if (s1 >= 0) atomicAdd(&P->pred_cnt[s1], 1u);
        }
        __syncthreads();
        uint32_t run = 0;
        for (uint32_t c = 0; c <= nb; c += PL_T) {
            const uint32_t b = c + tid;
            const uint32_t x = b <= nb ? P->pred_cnt[b] : 0u;
            uint32_t tot;
            const uint32_t ex = pl_scan(x, &tot, s_wsum);
            if (b <= nb) P->pred_cnt[b] = run + ex;
            run += tot;
        }
        __syncthreads();
        for (uint32_t b = tid; b < nb; b += PL_T) {
            for (int e = 0; e < 2; e++) {
                const int32_t s = P->succ[2 * b + e];
                if (s < 0) continue;
                const uint32_t slot = atomicAdd(&P->pred_fill[s], 1u);
                P->pred[P->pred_cnt[s] + slot] = b;
            }
        }
        __syncthreads();
        /* predecessor lists ascending */
        for (uint32_t b = tid; b < nb; b += PL_T) {
            const uint32_t lo = P->pred_cnt[b], hi = P->pred_cnt[b + 1];
            for (uint32_t i = lo + 1; i < hi; i++) {
                const uint32_t x = P->pred[i];
                uint32_t j = i;
                while (j > lo && P->pred[j - 1] > x) {
                    P->pred[j] = P->pred[j - 1];
                    j--;
                }
                P->pred[j] = x;
            }
            P->dfs_seen[b] = 0;
            P->rpo_pos[b] = -1;
        }
        __syncthreads();
        /* reverse postorder of a DFS from block 0 taking the fall-through edge
         * first (one thread; the stack entries carry the next edge in bits
         * 31:30) */
        if (tid == 0) {
            uint32_t *stk = P->dfs_stack, *post = P->rpo;
            uint32_t sp = 0, np = 0;
            stk[sp++] = 0;
            P->dfs_seen[0] = 1;
            while (sp) {
                const uint32_t top = stk[sp - 1];
                const uint32_t u = top & 0x3FFFFFFFu, e = top >> 30;
                if (e < 2) {
                    stk[sp - 1] = u | ((e + 1) << 30);
                    const int32_t s = P->succ[2 * u + e];
                    if (s >= 0 && !P->dfs_seen[s]) {
                        P->dfs_seen[s] = 1;
                        stk[sp++] = (uint32_t)s;
                    }
                } else {
                    sp--;
                    post[np++] = u;
                }
            }
            for (uint32_t i = 0; i < np / 2; i++) {
                const uint32_t t = post[i];
                post[i] = post[np - 1 - i];
                post[np - 1 - i] = t;
            }
            for (uint32_t i = 0; i < np; i++) P->rpo_pos[post[i]] = (int32_t)i;
            s_nreach = np;
        }
        __syncthreads();
        /* the fixpoint's block records by RPO position (see k_blockinfo) */
        for (uint32_t b = tid; b < nb; b += PL_T) {
            const int32_t p = P->rpo_pos[b];
            if (p < 0) continue;
            const int32_t s0 = P->succ[2 * b], s1 = P->succ[2 * b + 1];
            const int32_t ps0 = s0 >= 0 ? P->rpo_pos[s0] : -1, ps1 = s1 >= 0 ? P->rpo_pos[s1] : -1;
            auto single = [&](int32_t sb) { return sb > 0 && P->pred_cnt[sb + 1] - P->pred_cnt[sb] == 1; };
            const uint32_t chain = single(s0) ? 0u : (single(s1) ? 1u : 2u);
            P->binfo[2 * p] = make_uint4(b, pos0 + P->block_start[b], pos0 + P->block_start[b + 1], 0u);
            P->binfo[2 * p + 1] = make_uint4((uint32_t)ps0, (uint32_t)ps1, chain, 0u);
        }
        if (tid == 0) {
            P->n_blocks[k] = nb;
            P->first_block[k] = 0;
            P->n_reach[k] = s_nreach;
            P->status[k] = DC_OK;
        }
        if (tid < KSLOT_WORDS) P->kslots[(uint64_t)k * KSLOT_WORDS + tid] = s_km[tid];
        __syncthreads();

        /* the fixpoint and extraction on the first wavefront */
        if (tid < 64) {
            const uint32_t l = lane_id();
            L.optab[l] = OPTAB[l < (uint32_t)N_OPS ? l : 0];
            L.optab[l < 16 ? 64 + l : l] =
                OPTAB[l < 16 && 64 + l < (uint32_t)N_OPS ? 64 + l : (l < (uint32_t)N_OPS ? l : 0)];
            __builtin_amdgcn_wave_barrier();
            WaveMem M;
            M.arena = P->arena;
            M.dummy = P->dummy;
            const uint32_t nu = rfl(build_compact(P, L, k));
            if (nb <= MAIN_MAX_BLOCKS) {
                RegBits reached, dirty;
                analyze(P, k, L, reached, dirty, M, nu);
            } else {
                const uint32_t words = (nb + 31) >> 5;
                MemBits reached{P->ovf_bitmaps, P->ovf_bitmaps + 2 * words},
                    dirty{P->ovf_bitmaps + words, P->ovf_bitmaps + 2 * words};
                analyze(P, k, L, reached, dirty, M, nu);
            }
        }
        __syncthreads();
    } else if (tid == 0) {
        dc_kernel_result_t res = {st, 0, 0, 0, 0, 0, 0};
        P->results[k] = res;
        P->status[k] = st;
    }

    /* dense output: the kernel's records after the batch's running totals */
    uint32_t na = 0, ns = 0;
    if (st == DC_OK) {
        for (uint32_t c = 0; c < nb; c += PL_T) {
            const uint32_t b = c + tid;
            const uint32_t xa = b < nb ? P->blk_acc[b] : 0u, xs = b < nb ? P->blk_sys[b] : 0u;
            uint32_t tota, tots;
            const uint32_t ea = pl_scan(xa, &tota, s_wsum), es = pl_scan(xs, &tots, s_wsum);
            if (b < nb) {
                const uint4 *sa = reinterpret_cast<const uint4 *>(P->acc_sparse) + P->blk_acc_base[b];
                uint4 *da = reinterpret_cast<uint4 *>(P->acc_dense) + out_a + na + ea;
                for (uint32_t i = 0; i < xa; i++) da[i] = sa[i];
                const uint2 *ss = reinterpret_cast<const uint2 *>(P->sys_sparse) + P->blk_sys_base[b];
                uint2 *ds = reinterpret_cast<uint2 *>(P->sys_dense) + out_s + ns + es;
                for (uint32_t i = 0; i < xs; i++) ds[i] = ss[i];
            }
            na += tota;
            ns += tots;
        }
    }
    __syncthreads();
    if (tid == 0) {
        P->results[k].n_access = na;
        P->results[k].n_sysval = ns;
        P->acc_count[k] = out_a;
        P->sys_count[k] = out_s;
        P->acc_count[k + 1] = out_a + na;
        P->sys_count[k + 1] = out_s + ns;
        P->counters[4] = out_a + na;
        P->counters[5] = out_s + ns;
    }
}

hipError_t launch_plain(const Plan &P, const Plan *dP, hipStream_t s, hipEvent_t before, hipEvent_t after) {
    hipError_t e = launch_fill_u32(P.counters, 8, 0u, s);
    if (e != hipSuccess) return e;
    if (before && (e = hipEventRecord(before, s)) != hipSuccess) return e;
    if (P.n_kernels == 0) {
        e = launch_fill_u32(P.acc_count, 1, 0u, s);
        if (e == hipSuccess) e = launch_fill_u32(P.sys_count, 1, 0u, s);
    }
    for (uint32_t k = 0; k < P.n_kernels && e == hipSuccess; k++) {
        hipLaunchKernelGGL(k_plain, dim3(1), dim3(PL_T), sizeof(WaveLds), s, dP, k);
        e = hipGetLastError();
    }
    if (e == hipSuccess && after) e = hipEventRecord(after, s);
    return e;
}

}  // namespace dc
