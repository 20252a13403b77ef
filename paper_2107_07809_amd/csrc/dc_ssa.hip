/*
 * dc_ssa.hip -- register versions (minimal SSA form) of every kernel of a
 * batch whose control flow graphs the graph stages have built.
 *
 * Section "Search for control structures": where a block has several
 * predecessors a register can hold the values of different definitions, and
 * the method then introduces a variable; the Register record of Section
 * "Search for memory accesses" carries a version.  Read as the minimal SSA
 * form (Cytron, Ferrante, Rosen, Wegman & Zadeck 1991) over the register
 * slots: a virtual start before block 0 defines version 0 of every slot;
 * every definition makes a new version; a merge of a slot sits at each block
 * of the iterated dominance frontier of its defining blocks; versions are
 * numbered per slot along a preorder walk of the dominator tree (children by
 * ascending block index), a block's merges before its instructions.
 *
 * One workgroup of one wavefront per kernel:
 *   k_ssa_size   per kernel, the size of its (block x slot) tables
 *   k_ssa_graph  immediate dominators (the iterative method of Cooper, Harvey
 *                & Kennedy 2001 over reverse postorder); the dominator-tree
 *                preorder (subtree sizes, then sibling offsets, then
 *                positions); per block and slot the number of definitions;
 *                merge placement; per slot the numbering along the preorder
 *                and the version live at each block's end; output counts
 *   k_ssa_scan   exclusive scans of the per-kernel counts (offsets)
 *   k_ssa_emit   the merges with their arguments, every operand's version,
 *                the digest (when asked for)
 *
 * Merge placement without frontier lists: a join block b has the slot's
 * merge when some block on one of b's frontier walks (from each reachable
 * predecessor up the dominator tree to b's immediate dominator, exclusive;
 * from a predecessor of block 0 up to block 0 inclusive, the start being
 * its immediate dominator) defines the slot or merges it.  The blocks on b's
 * walks are exactly those whose dominance frontier holds b, so the least
 * solution of this rule, reached by repeating passes over the join blocks
 * until none changes, is the iterated dominance frontier.  The walks do not
 * depend on the slot: one walk serves all slots, lane l holding slots l,
 * l + 64, ... of the kernel's table.
 *
 * Versions: with base(b, s) = 1 + the number of definitions and merges of
 * slot s in the blocks before b in the preorder, a merge of s at b has
 * version base(b, s), the j-th definition of s in b (0-based) has
 * base(b, s) + merge(b, s) + j, and a use of s in b after j > 0 definitions
 * in b reads the last of them, else the version live at b's entry: its
 * merge's, or the one live at the end of its immediate dominator (version 0
 * at block 0).
 *
 * A kernel's graph sits in LDS when it has at most SB_LDS blocks, else in
 * global memory; the same code reads both through generic pointers.
 */
#include "dc_ssa_ops.h"

namespace dc {

constexpr uint32_t SSA_NONE = DC_SSA_NONE;
constexpr uint32_t SB_LDS = 256;                      /* blocks of a kernel whose graph is staged in LDS */
constexpr uint32_t SLOTS_MAX = KSLOT_WORDS * 32;      /* 384 >= DC_NSLOT */
constexpr uint32_t SSA_G = (SLOTS_MAX + 63) / 64;     /* table columns per lane, at most */
constexpr uint32_t PHI_BIT = 0x80000000u;

/* The kernel's register slots (those its records name, plus vcc, exec and
 * scc) in ascending order: rank[slot] = table column; slot[column] when
 * asked for.  Returns their number. */
__device__ uint32_t slot_columns(const uint32_t *ks, uint16_t *rank, uint16_t *slot) {
    const uint32_t l = lane_id();
    uint32_t run = 0;
    for (uint32_t v0 = 0; v0 < SLOTS_MAX; v0 += 64) {
        const uint32_t v = v0 + l;
        uint32_t w = ks[v >> 5];
        if ((v >> 5) == 3) w |= 0x1F00u;   /* slots 104..108 */
        const bool set = v < (uint32_t)NSLOT && ((w >> (v & 31)) & 1u);
        const uint64_t m = ballot(set);
        const uint32_t r = run + lanes_below(m);
        if (set) {
            rank[v] = (uint16_t)r;
            if (slot) slot[r] = (uint16_t)v;
        }
        run += (uint32_t)__popcll(m);
    }
    __syncthreads();
    return run;
}
__device__ __forceinline__ uint32_t slot_count(const uint32_t *ks) {
    uint32_t n = 0;
    for (uint32_t w = 0; w < KSLOT_WORDS; w++) n += __popc(ks[w] | (w == 3 ? 0x1F00u : 0u));
    return n;
}

/* offsets of count array a (0 table words, 1 merges, 2 merge arguments, 3 operands; with the types 4
 * register columns, 5 nodes, 6 nodes of kernels over TY_LDS_NODES) */
__device__ __forceinline__ uint64_t soff(const SsaPlan &S, uint32_t K, uint32_t a, uint32_t k) {
    return S.offs[(uint64_t)a * (K + 1) + k];
}

/* ------------------------------------------------------------------ */
/* k_ssa_size                                                            */
/* ------------------------------------------------------------------ */
__global__ __launch_bounds__(256) void k_ssa_size(Plan P, SsaPlan S) {
    const uint32_t k = blockIdx.x * 256 + threadIdx.x;
    if (k >= P.n_kernels) return;
    const uint32_t U = P.status[k] == DC_OK ? slot_count(P.kslots + (uint64_t)k * KSLOT_WORDS) : 0u;
    S.counts[k] = P.n_blocks[k] * U;
    if (S.nver) S.counts[4ull * P.n_kernels + k] = U;
}

/* ------------------------------------------------------------------ */
/* k_ssa_scan: exclusive scans, one workgroup per count array            */
/* ------------------------------------------------------------------ */
__global__ __launch_bounds__(1024) void k_ssa_scan(SsaPlan S, uint32_t K, uint32_t a0) {
    const uint32_t a = a0 + blockIdx.x, t = threadIdx.x, w = t >> 6, l = lane_id();
    const uint32_t *in = S.counts + (uint64_t)a * K;
    uint64_t *out = S.offs + (uint64_t)a * (K + 1);
    __shared__ uint64_t wsum[16], carry;
    if (t == 0) carry = 0;
    __syncthreads();
    for (uint32_t c = 0; c < K; c += 1024) {
        const uint32_t i = c + t;
        const uint64_t x = i < K ? in[i] : 0;
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
        if (i < K) out[i] = before + y - x;
        __syncthreads();
        if (t == 1023) carry = before + y;
        __syncthreads();
    }
    if (t == 0) out[K] = carry;
}

/* walk up the dominator tree from a and b to their nearest common dominator
 * (positions in reverse postorder decrease towards block 0) */
__device__ __forceinline__ uint32_t dom_meet(const uint32_t *idom, const int32_t *pos, uint32_t a, uint32_t b) {
    while (a != b) {
        while (pos[a] > pos[b]) a = idom[a];
        while (pos[b] > pos[a]) b = idom[b];
    }
    return a;
}

/* ------------------------------------------------------------------ */
/* k_ssa_graph                                                           */
/* ------------------------------------------------------------------ */
/* The sequential parts (dominators, preorder) run on every lane with the
 * same values: each lane reads back only what it stored itself. */
/* the work of k_ssa_graph on one kernel's graph arrays (rpo, pos, poff,
 * pred, idom and the preorder scratch), called with the arrays staged in LDS
 * or with the global ones, so that each copy uses the memory instructions of
 * its own address space */
struct GraphOut {
    uint32_t nphi, nargs, nops, nnodes;
};
__device__ __forceinline__ GraphOut ssa_graph_body(const Plan &P, const SsaPlan &S, uint32_t k, uint32_t nb,
                                                   uint32_t fb, uint32_t nreach, uint32_t pb, uint32_t n,
                                                   const dc_kernel_t &D, uint32_t U, const uint16_t *s_rank,
                                                   uint32_t *s_cnt, const uint32_t *rpo, const int32_t *pos,
                                                   const uint32_t *poff, const uint32_t *pred, uint32_t *idom,
                                                   uint32_t *t1, uint32_t *t2, uint32_t *pinv) {
    const uint32_t l = lane_id(), K = P.n_kernels;
    const uint64_t tab0 = soff(S, K, 0, k);
    for (uint32_t b = l; b < nb; b += 64) {
        idom[b] = b == 0 ? 0u : SSA_NONE;
        t1[b] = 1;
        t2[b] = 0;
    }
    __syncthreads();

    /* immediate dominators: passes over reverse postorder until none changes */
    for (bool changed = true; changed;) {
        changed = false;
        for (uint32_t j = 1; j < nreach; j++) {
            const uint32_t b = rpo[j];
            uint32_t nd = SSA_NONE;
            for (uint32_t e = poff[b]; e < poff[b + 1]; e++) {
                const uint32_t p = pred[e];
                if (pos[p] < 0 || idom[p] == SSA_NONE) continue;
                nd = nd == SSA_NONE ? p : dom_meet(idom, pos, p, nd);
            }
            if (nd != idom[b]) {
                idom[b] = nd;
                changed = true;
            }
        }
    }
    /* preorder of the dominator tree, children ascending: subtree sizes
     * (children after parents in reverse postorder), then each child's
     * offset among its siblings (t1), then positions (t2) */
    for (uint32_t j = nreach; j-- > 1;) {
        const uint32_t b = rpo[j];
        t1[idom[b]] += t1[b];
    }
    for (uint32_t b = 1; b < nb; b++) {
        if (pos[b] < 0) continue;
        const uint32_t p = idom[b], s = t1[b];
        t1[b] = t2[p];
        t2[p] += s;
    }
    t2[0] = 0;
    pinv[0] = 0;
    for (uint32_t j = 1; j < nreach; j++) {
        const uint32_t b = rpo[j];
        const uint32_t pr = t2[idom[b]] + 1 + t1[b];
        t2[b] = pr;
        pinv[pr] = b;
    }
    __syncthreads();

    /* definitions of each slot in each reachable block */
    uint32_t *A = S.tab_a + tab0, *Bt = S.tab_b + tab0;
    for (uint32_t b = 0; b < nb; b++) {
        if (pos[b] < 0) continue;
        for (uint32_t u = l; u < U; u += 64) s_cnt[u] = 0;
        __syncthreads();
        const uint32_t s0 = P.block_start[fb + b] - pb, s1 = P.block_start[fb + b + 1] - pb;
        for (uint32_t i = s0 + l; i < s1; i += 64) {
            const Rec x = load_rec(P, D, i);
            for_defs(x, [&](uint32_t, uint32_t v, uint32_t) { atomicAdd(&s_cnt[s_rank[v]], 1u); });
        }
        __syncthreads();
        for (uint32_t u = l; u < U; u += 64) A[(uint64_t)b * U + u] = s_cnt[u];
        __syncthreads();
    }

    /* merges: the least solution of "a join block merges a slot when a block
     * on one of its frontier walks defines or merges it" */
    const uint32_t G = (U + 63) / 64;
    for (bool again = true; again;) {
        uint32_t grew = 0;
        for (uint32_t j = 0; j < nreach; j++) {
            const uint32_t b = rpo[j];
            uint32_t inc = b == 0 ? 1u : 0u;
            for (uint32_t e = poff[b]; e < poff[b + 1]; e++) inc += pos[pred[e]] >= 0 ? 1u : 0u;
            if (inc < 2) continue;
            const uint64_t row = (uint64_t)b * U;
            uint32_t need = 0;
#pragma unroll
            for (uint32_t g = 0; g < SSA_G; g++) {
                const uint32_t u = l + 64 * g;
                if (g < G && u < U && !(A[row + u] & PHI_BIT)) need |= 1u << g;
            }
            if (ballot(need != 0) == 0) continue;
            uint32_t got = 0;
            const uint32_t stop = b == 0 ? SSA_NONE : idom[b];
            for (uint32_t e = poff[b]; e < poff[b + 1]; e++) {
                uint32_t r = pred[e];
                if (pos[r] < 0) continue;
                while (r != stop) {
                    const uint64_t rr = (uint64_t)r * U;
#pragma unroll
                    for (uint32_t g = 0; g < SSA_G; g++)
                        if (((need >> g) & 1u) && A[rr + l + 64 * g] != 0) {
                            got |= 1u << g;
                            need &= ~(1u << g);
                        }
                    if (r == 0) break;
                    r = idom[r];
                }
            }
#pragma unroll
            for (uint32_t g = 0; g < SSA_G; g++)
                if ((got >> g) & 1u) A[row + l + 64 * g] |= PHI_BIT;
            grew |= got;
        }
        again = ballot(grew != 0) != 0;
    }

    /* numbering along the preorder: A <- first version of the block | merge
     * flag, Bt <- the version live at the block's end */
    uint32_t run[SSA_G];
#pragma unroll
    for (uint32_t g = 0; g < SSA_G; g++) run[g] = 1;
    uint32_t nphi = 0, nargs = 0;
    for (uint32_t j = 0; j < nreach; j++) {
        const uint32_t b = pinv[j];
        uint32_t inc = b == 0 ? 1u : 0u;
        for (uint32_t e = poff[b]; e < poff[b + 1]; e++) inc += pos[pred[e]] >= 0 ? 1u : 0u;
        const uint64_t row = (uint64_t)b * U, prow = (uint64_t)(b == 0 ? 0u : idom[b]) * U;
#pragma unroll
        for (uint32_t g = 0; g < SSA_G; g++) {
            const uint32_t u = l + 64 * g;
            if (g < G && u < U) {
                const uint32_t a = A[row + u], d = a & ~PHI_BIT, ph = a >> 31, base = run[g];
                run[g] += d + ph;
                const uint32_t in = ph ? base : (b == 0 ? 0u : Bt[prow + u]);
                A[row + u] = base | (ph << 31);
                Bt[row + u] = d ? base + ph + d - 1 : in;
                nphi += ph;
                nargs += ph * inc;
            }
        }
    }
    /* versions per column (version 0 included), for the types */
    uint32_t nnodes = 0;
    if (S.nver) {
        uint32_t *nv = S.nver + soff(S, K, 4, k);
#pragma unroll
        for (uint32_t g = 0; g < SSA_G; g++) {
            const uint32_t u = l + 64 * g;
            if (g < G && u < U) {
                nv[u] = run[g];
                nnodes += run[g];
            }
        }
        nnodes = wave_sum32(nnodes);
    }
    uint32_t nops = 0;
    for (uint32_t i = l; i < n; i += 64) {
        const Rec x = load_rec(P, D, i);
        nops += n_uses(x) + n_defs(x);
    }
    nphi = wave_sum32(nphi);
    nargs = wave_sum32(nargs);
    nops = wave_sum32(nops);
    return GraphOut{nphi, nargs, nops, nnodes};
}

__global__ __launch_bounds__(64) void k_ssa_graph(Plan P, SsaPlan S) {
    __shared__ uint32_t l_rpo[SB_LDS], l_idom[SB_LDS], l_poff[SB_LDS + 1], l_pred[2 * SB_LDS], l_t1[SB_LDS],
        l_t2[SB_LDS], l_pinv[SB_LDS];
    __shared__ int32_t l_pos[SB_LDS];
    __shared__ uint16_t s_rank[SLOTS_MAX];
    __shared__ uint32_t s_cnt[SLOTS_MAX];
    const uint32_t k = blockIdx.x, l = lane_id(), K = P.n_kernels;
    int32_t st = P.status[k];
    if (st == DC_OK && soff(S, K, 0, k + 1) > S.tab_cap) st = DC_E_CAPACITY;
    if (st == DC_OK && S.nver && soff(S, K, 4, k + 1) > S.col_cap) st = DC_E_CAPACITY;
    if (st != DC_OK) {
        S.status[k] = st;
        S.counts[(uint64_t)K + k] = 0;
        S.counts[2ull * K + k] = 0;
        S.counts[3ull * K + k] = 0;
        if (S.nver) {
            S.counts[5ull * K + k] = 0;
            S.counts[6ull * K + k] = 0;
        }
        return;
    }
    const uint32_t nb = P.n_blocks[k], fb = P.first_block[k], nreach = P.n_reach[k], pb = P.pos_begin[k];
    const uint32_t n = P.pos_begin[k + 1] - pb;
    const dc_kernel_t D = P.kernels[k];
    const uint32_t U = slot_columns(P.kslots + (uint64_t)k * KSLOT_WORDS, s_rank, nullptr);

    /* the graph: staged in LDS when small */
    const uint32_t pred0 = P.pred_cnt[fb], npred = P.pred_cnt[fb + nb] - pred0;
    const bool lds = nb <= SB_LDS && npred <= 2 * SB_LDS;
    if (lds) {
        for (uint32_t b = l; b <= nb; b += 64) {
            l_poff[b] = P.pred_cnt[fb + b] - pred0;
            if (b < nb) {
                l_rpo[b] = P.rpo[fb + b];
                l_pos[b] = P.rpo_pos[fb + b];
            }
        }
        for (uint32_t j = l; j < npred; j += 64) l_pred[j] = P.pred[pred0 + j];
    }
    const uint64_t cap = P.blk_cap;
    GraphOut o;
    if (lds)   /* uniform */
        o = ssa_graph_body(P, S, k, nb, fb, nreach, pb, n, D, U, s_rank, s_cnt, l_rpo, l_pos, l_poff, l_pred, l_idom,
                           l_t1, l_t2, l_pinv);
    else
        o = ssa_graph_body(P, S, k, nb, fb, nreach, pb, n, D, U, s_rank, s_cnt, P.rpo + fb, P.rpo_pos + fb,
                           P.pred_cnt + fb, P.pred, S.idom + fb, S.scr + fb, S.scr + cap + fb, S.scr + 2 * cap + fb);
    const uint32_t nphi = o.nphi, nargs = o.nargs, nops = o.nops, nnodes = o.nnodes;
    if (lds)
        for (uint32_t b = l; b < nb; b += 64) S.idom[fb + b] = l_idom[b];
    S.status[k] = DC_OK;
    S.counts[(uint64_t)K + k] = nphi;
    S.counts[2ull * K + k] = nargs;
    S.counts[3ull * K + k] = nops;
    if (S.nver) {
        S.counts[5ull * K + k] = nnodes;
        S.counts[6ull * K + k] = nnodes > TY_LDS_NODES ? nnodes : 0u;
    }
}

/* ------------------------------------------------------------------ */
/* k_ssa_emit                                                            */
/* ------------------------------------------------------------------ */
template <bool DIGEST>
__global__ __launch_bounds__(64) void k_ssa_emit(Plan P, SsaPlan S) {
    __shared__ uint16_t s_rank[SLOTS_MAX], s_slot[SLOTS_MAX];
    __shared__ uint32_t s_cnt[SLOTS_MAX];
    __shared__ unsigned long long s_m1[SLOTS_MAX], s_m2[SLOTS_MAX];
    const uint32_t k = blockIdx.x, l = lane_id(), K = P.n_kernels;
    int32_t st = S.status[k];
    const uint64_t po = soff(S, K, 1, k), ao = soff(S, K, 2, k), oo = soff(S, K, 3, k);
    if (st == DC_OK && (soff(S, K, 1, k + 1) > S.phi_cap || soff(S, K, 2, k + 1) > S.arg_cap ||
                        soff(S, K, 3, k + 1) > S.ops_cap))
        st = DC_E_CAPACITY;
    dc_ssa_result_t res = {st, 0, 0, 0, 0, 0, 0};
    if (st != DC_OK) {
        S.res[k] = res;
        return;
    }
    const uint32_t nb = P.n_blocks[k], fb = P.first_block[k], pb = P.pos_begin[k];
    const dc_kernel_t D = P.kernels[k];
    const uint32_t U = slot_columns(P.kslots + (uint64_t)k * KSLOT_WORDS, s_rank, s_slot);
    const uint32_t G = (U + 63) / 64;
    const uint32_t *A = S.tab_a + soff(S, K, 0, k), *Bt = S.tab_b + soff(S, K, 0, k);
    const uint32_t *idom = S.idom + fb, *poff = P.pred_cnt + fb;
    const int32_t *pos = P.rpo_pos + fb;
    uint64_t h = 0;
    if (DIGEST)
        for (uint32_t b = l; b < nb; b += 64) h += ssa_item(1, b, idom[b]);

    /* merges (ascending block, then slot) and their arguments.  Blocks go in
     * groups of 64: lane l first finds whether block b0 + l is reachable and
     * how many arguments its merges take (its reachable predecessors, plus the
     * entry for block 0); the blocks of the group then run in order, each
     * loading its table row (all columns at once) before emitting. */
    uint32_t np = 0, na = 0;
    for (uint32_t b0 = 0; b0 < nb; b0 += 64) {
        const uint32_t bl = b0 + l;
        const bool rl = bl < nb && pos[bl < nb ? bl : 0] >= 0;
        uint32_t incl = bl == 0 ? 1u : 0u;
        if (rl)
            for (uint32_t e = poff[bl]; e < poff[bl + 1]; e++) incl += pos[P.pred[e]] >= 0 ? 1u : 0u;
        const uint64_t rm = ballot(rl);
        const uint32_t bend = nb - b0 < 64u ? nb : b0 + 64u;
        for (uint32_t b = b0; b < bend; b++) {
            if (!((rm >> (b - b0)) & 1ull)) continue;
            const uint32_t inc = (uint32_t)__shfl((int)incl, (int)(b - b0), 64);
            const uint64_t row = (uint64_t)b * U;
            const uint32_t np_b = np;
            uint32_t av[SSA_G];
#pragma unroll
            for (uint32_t g = 0; g < SSA_G; g++) {
                const uint32_t u = l + 64 * g;
                av[g] = g < G && u < U ? A[row + u] : 0u;
            }
#pragma unroll
            for (uint32_t g = 0; g < SSA_G; g++) {
                if (g >= G) break;
                const uint32_t u = l + 64 * g;
                const uint32_t a = av[g];
                const bool ph = u < U && (a & PHI_BIT);
                const uint64_t m = ballot(ph);
                if (ph) {
                    const uint32_t idx = np + lanes_below(m), v = s_slot[u], ver = a & ~PHI_BIT;
                    dc_phi_t f;
                    f.block = b;
                    f.slot = (uint16_t)v;
                    f.pad = 0;
                    f.version = ver;
                    S.phis[po + idx] = f;
                    if (DIGEST) h += ssa_item(2, ((uint64_t)b << 16) | v, ver);
                    uint32_t *arg = S.phi_args + ao + na + (uint64_t)(idx - np_b) * inc;
                    uint32_t kk = 0;
                    if (b == 0) {
                        arg[0] = 0;
                        if (DIGEST) h += ssa_item(3, ((uint64_t)b << 24) | ((uint64_t)v << 12), 0);
                        kk = 1;
                    }
                    for (uint32_t e = poff[b]; e < poff[b + 1]; e++) {
                        const uint32_t p = P.pred[e];
                        if (pos[p] < 0) continue;
                        const uint32_t x = Bt[(uint64_t)p * U + u];
                        arg[kk] = x;
                        if (DIGEST) h += ssa_item(3, ((uint64_t)b << 24) | ((uint64_t)v << 12) | kk, x);
                        kk++;
                    }
                }
                np += (uint32_t)__popcll(m);
            }
            na += (np - np_b) * inc;
        }
    }

    /* every operand's version, block by block in index order */
    for (uint32_t u = l; u < SLOTS_MAX; u += 64) {
        s_m1[u] = 0;
        s_m2[u] = 0;
    }
    uint32_t opos = 0;
    for (uint32_t b = 0; b < nb; b++) {
        const bool reach = pos[b] >= 0;
        const uint32_t s0 = P.block_start[fb + b] - pb, s1 = P.block_start[fb + b + 1] - pb;
        const uint64_t row = (uint64_t)b * U, prow = (uint64_t)(reach && b != 0 ? idom[b] : 0u) * U;
        for (uint32_t u = l; u < U; u += 64) s_cnt[u] = 0;
        __syncthreads();
        for (uint32_t c0 = s0; c0 < s1; c0 += 64) {
            const uint32_t i = c0 + l;
            const bool act = i < s1;
            Rec x;
            x.e = OPTAB[0];
            x.id[0] = x.id[1] = x.id[2] = x.id[3] = 0xFFFFu;
            uint32_t nu = 0, nd = 0;
            if (act) {
                x = load_rec(P, D, i);
                nu = n_uses(x);
                nd = n_defs(x);
            }
            uint32_t tot;
            const uint32_t off = wave_excl(nu + nd, &tot);
            if (act && reach)
                for_defs(x, [&](uint32_t, uint32_t v, uint32_t again) {
                    atomicOr(again ? &s_m2[s_rank[v]] : &s_m1[s_rank[v]], 1ull << l);
                });
            __syncthreads();
            if (act) {
                const uint64_t below = (1ull << l) - 1ull;
                uint32_t *out = S.vers + oo + opos + off;
                if (reach) {
                    for_uses(x, [&](uint32_t q, uint32_t v) {
                        const uint32_t r = s_rank[v], a = A[row + r], base = a & ~PHI_BIT, ph = a >> 31;
                        const uint32_t c = s_cnt[r] + (uint32_t)__popcll(s_m1[r] & below) +
                                           (uint32_t)__popcll(s_m2[r] & below);
                        const uint32_t ver = c ? base + ph + c - 1 : (ph ? base : (b == 0 ? 0u : Bt[prow + r]));
                        out[q] = ver;
                        if (DIGEST) h += ssa_item(4, (uint64_t)i * DC_SSA_NU + q, ver);
                    });
                    for_defs(x, [&](uint32_t q, uint32_t v, uint32_t again) {
                        const uint32_t r = s_rank[v], a = A[row + r], base = a & ~PHI_BIT, ph = a >> 31;
                        const uint32_t c = s_cnt[r] + (uint32_t)__popcll(s_m1[r] & below) +
                                           (uint32_t)__popcll(s_m2[r] & below) + again;
                        const uint32_t ver = base + ph + c;
                        out[nu + q] = ver;
                        if (DIGEST) h += ssa_item(5, (uint64_t)i * DC_SSA_ND + q, ver);
                    });
                } else {
                    for (uint32_t q = 0; q < nu; q++) {
                        out[q] = SSA_NONE;
                        if (DIGEST) h += ssa_item(4, (uint64_t)i * DC_SSA_NU + q, SSA_NONE);
                    }
                    for (uint32_t q = 0; q < nd; q++) {
                        out[nu + q] = SSA_NONE;
                        if (DIGEST) h += ssa_item(5, (uint64_t)i * DC_SSA_ND + q, SSA_NONE);
                    }
                }
                if (DIGEST) {
                    for (uint32_t q = nu; q < DC_SSA_NU; q++) h += ssa_item(4, (uint64_t)i * DC_SSA_NU + q, SSA_NONE);
                    for (uint32_t q = nd; q < DC_SSA_ND; q++) h += ssa_item(5, (uint64_t)i * DC_SSA_ND + q, SSA_NONE);
                }
                S.opn[pb + i] = (uint8_t)(nu | nd << 4);
            }
            __syncthreads();
            if (act && reach)
                for_defs(x, [&](uint32_t, uint32_t v, uint32_t) {
                    const uint32_t r = s_rank[v];
                    atomicAdd(&s_cnt[r], 1u);
                    s_m1[r] = 0;
                    s_m2[r] = 0;
                });
            __syncthreads();
            opos += tot;
        }
    }
    if (DIGEST) h = wave_sum64(h);
    res.n_blocks = nb;
    res.n_phi = np;
    res.n_phi_args = na;
    res.n_operands = opos;
    res.digest = h;
    S.res[k] = res;
}

/* ------------------------------------------------------------------ */
/* launchers                                                             */
/* ------------------------------------------------------------------ */
hipError_t launch_ssa_size(const Plan &P, const SsaPlan &S, hipStream_t s) {
    const uint32_t K = P.n_kernels;
    if (!K) return hipSuccess;
    hipLaunchKernelGGL(k_ssa_size, dim3((K + 255) / 256), dim3(256), 0, s, P, S);
    hipLaunchKernelGGL(k_ssa_scan, dim3(1), dim3(1024), 0, s, S, K, 0u);
    if (S.nver) hipLaunchKernelGGL(k_ssa_scan, dim3(1), dim3(1024), 0, s, S, K, 4u);
    return hipGetLastError();
}
hipError_t launch_ssa_graph(const Plan &P, const SsaPlan &S, hipStream_t s) {
    const uint32_t K = P.n_kernels;
    if (!K) return hipSuccess;
    hipLaunchKernelGGL(k_ssa_graph, dim3(K), dim3(64), 0, s, P, S);
    hipLaunchKernelGGL(k_ssa_scan, dim3(3), dim3(1024), 0, s, S, K, 1u);
    if (S.nver) hipLaunchKernelGGL(k_ssa_scan, dim3(2), dim3(1024), 0, s, S, K, 5u);
    return hipGetLastError();
}
hipError_t launch_ssa_emit(const Plan &P, const SsaPlan &S, hipStream_t s) {
    const uint32_t K = P.n_kernels;
    if (!K) return hipSuccess;
    if (S.digest) hipLaunchKernelGGL(k_ssa_emit<true>, dim3(K), dim3(64), 0, s, P, S);
    else hipLaunchKernelGGL(k_ssa_emit<false>, dim3(K), dim3(64), 0, s, P, S);
    return hipGetLastError();
}

}  // namespace dc
