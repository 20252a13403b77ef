/*
 * dc_types.hip -- variables and types over the register versions of every
 * kernel of a batch (Section "Data type recovery": types from the .arg
 * table and from instruction suffixes, a suffix typing what an instruction
 * reads as well as what it writes; Section "Search for control structures":
 * a register ambiguous at a join and used later becomes a variable, and the
 * ternary operator is one instruction).
 *
 * Nodes are the versions of each register column of a kernel (version 0
 * included), columns ascending, node = vbase[column] + version.  One
 * workgroup of 256 threads per kernel:
 *   1. column ranks from the kernel's slot bitmap, column bases by a scan of
 *      the per-column version counts the graph stage wrote;
 *   2. merges, in chunks: each merge's first argument (a scan of the
 *      incoming-edge counts of the merges' blocks), the merge flag, and the
 *      merge joined with each argument in both partitions;
 *   3. instructions, in chunks: each one's operand versions (a scan of the
 *      operand counts), the type each definition and each use gives, the
 *      live flag of every read node, copies and v_cndmask_b32 joined in the
 *      type partition;
 *   4. liveness back through the merges: passes until no argument of a live
 *      merge turns live;
 *   5. each node's type bits ORed into its type class's root;
 *   6. the output per node and the per-kernel counts (and digest).
 * The partitions are union-find forests whose roots are hooked under the
 * smaller root with a compare-and-swap, so the root of a class is its
 * smallest node whatever the order of the joins; finds halve paths.  A
 * kernel's forests and flags sit in LDS up to TY_LDS_NODES nodes, else in
 * global scratch; all accesses are atomics through generic pointers, so the
 * same code serves both and no thread reads a stale cached word.
 */
#include "dc_ssa_ops.h"

namespace dc {

constexpr uint32_t TY_THREADS = 256;
constexpr uint32_t TY_WAVES = TY_THREADS / 64;
constexpr uint32_t TY_COLS = KSLOT_WORDS * 32;
constexpr uint32_t TF_MERGE = DC_VF_MERGE << 8, TF_LIVE = DC_VF_LIVE << 8;
constexpr uint32_t NO_Q = 0xFFu;

/* per opcode: the first suffix's type (given to the destination), the last
 * suffix's type (given to every register read as an explicit source), and
 * whether the record copies (moves) or selects (v_cndmask_b32) a value */
enum : uint32_t { TK_COPY = 1, TK_SELECT = 2 };
constexpr uint16_t tyop(uint32_t def, uint32_t use, uint32_t kind) {
    return (uint16_t)(def | use << 5 | kind << 10);
}
constexpr uint16_t UU = tyop(TY_U, TY_U, 0), II = tyop(TY_I, TY_I, 0), FF = tyop(TY_F, TY_F, 0),
                   DD = tyop(TY_D, TY_D, 0);
static __constant__ uint16_t TYOP[N_OPS] = {
    0, 0, 0,                                    /* s_load_dword, _dwordx2, _dwordx4: the argument table */
    tyop(0, 0, TK_COPY), tyop(0, 0, TK_COPY),   /* s_mov_b32, s_mov_b64 */
    0, 0,                                       /* s_and_saveexec_b64, s_or_saveexec_b64 */
    UU, II, UU, UU, II,                         /* s_add_u32, s_add_i32, s_addc_u32, s_sub_u32, s_mul_i32 */
    0, 0, 0, 0, 0, 0, 0, 0,                     /* s_lshl_b32 .. s_andn2_b64 */
    UU, UU, UU, II,                             /* s_cmp_eq_u32, _lt_u32, _gt_u32, _lt_i32 */
    0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0,            /* branches, s_waitcnt, s_barrier, s_nop, s_endpgm */
    tyop(0, 0, TK_COPY),                        /* v_mov_b32 */
    tyop(TY_F, TY_U, 0),                        /* v_cvt_f32_u32 */
    tyop(TY_U, TY_F, 0),                        /* v_cvt_u32_f32 */
    tyop(TY_D, TY_F, 0),                        /* v_cvt_f64_f32 */
    UU, UU, UU, UU, UU, UU, UU, UU,             /* v_add_co_u32 .. v_mad_u32_u24 */
    0, 0,                                       /* v_lshlrev_b32, v_lshrrev_b32 */
    II,                                         /* v_ashrrev_i32 */
    0, 0, 0, 0,                                 /* v_and_b32, v_or_b32, v_xor_b32, v_lshlrev_b64 */
    tyop(0, 0, TK_SELECT),                      /* v_cndmask_b32 */
    FF, FF, FF, FF, FF, FF,                     /* v_add_f32 .. v_fma_f32 */
    DD, DD, DD,                                 /* v_add_f64, v_mul_f64, v_fma_f64 */
    UU, UU, UU, II, FF,                         /* v_cmp_eq_u32, _gt_u32, _lt_u32, _lt_i32, _gt_f32 */
    0, 0, 0, 0, 0, 0, 0, 0,                     /* memory: address rules by class */
};

__device__ __forceinline__ uint64_t toff(const SsaPlan &S, uint32_t K, uint32_t a, uint32_t k) {
    return S.offs[(uint64_t)a * (K + 1) + k];
}
__device__ __forceinline__ uint32_t ald(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void ast(uint32_t *p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void aor(uint32_t *p, uint32_t v) {
    __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t uf_find(uint32_t *par, uint32_t x) {
    for (;;) {
        const uint32_t p = ald(par + x);
        if (p == x) return x;
        const uint32_t g = ald(par + p);
        if (g != p) ast(par + x, g);   /* x is no root: any ancestor is a valid parent */
        x = g;
    }
}
__device__ void uf_union(uint32_t *par, uint32_t a, uint32_t b) {
    for (;;) {
        a = uf_find(par, a);
        b = uf_find(par, b);
        if (a == b) return;
        if (a < b) {
            const uint32_t t = a;
            a = b;
            b = t;
        }
        uint32_t expect = a;   /* hook the larger root under the smaller one, if it is still a root */
        if (__hip_atomic_compare_exchange_strong(par + a, &expect, b, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT))
            return;
    }
}

/* exclusive prefix over the workgroup; *total = the sum (all threads call) */
__device__ uint32_t block_excl(uint32_t x, uint32_t *total, uint32_t *s_w) {
    const uint32_t w = threadIdx.x >> 6;
    uint32_t wt;
    const uint32_t ex = wave_excl(x, &wt);
    if (lane_id() == 0) s_w[w] = wt;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (uint32_t j = 0; j < TY_WAVES; j++) {
        before += j < w ? s_w[j] : 0u;
        all += s_w[j];
    }
    __syncthreads();
    *total = all;
    return before + ex;
}

__device__ __forceinline__ uint32_t slot_word(const uint32_t *ks, uint32_t w) {
    return ks[w] | (w == 3 ? 0x1F00u : 0u);   /* vcc, exec, scc: slots 104..108 */
}

/* the .arg type of the argument covering dword offset o of the argument area */
__device__ uint32_t smem_type(const Plan &P, const dc_kernel_t &D, uint32_t o) {
    if (o < 0x18) return TY_U;       /* global offsets */
    if (o < 0x30) return 0;          /* printf buffer, vqueue, aqlwrap */
    if (o == 0x20010) return TY_U;   /* work dimension */
    for (uint32_t a = 0; a < D.n_args; a++) {
        const dc_arg_t A = P.args[D.arg_begin + a];
        if ((uint64_t)A.offset <= o && (uint64_t)o < (uint64_t)A.offset + A.size) return A.type;
    }
    return 0;
}

/* steps 2-6 of one kernel on forests and flags at pv, pt, fl: called with
 * the LDS arrays or with global scratch, so that each copy uses the memory
 * instructions of its own address space */
struct TyShared {
    const uint16_t *rank, *slot;
    const uint32_t *vb;
    uint32_t *w, *flag, *tern;
    uint32_t (*red)[3];
    unsigned long long *h;
};
template <bool DIGEST>
__device__ __forceinline__ void types_body(const Plan &P, const SsaPlan &S, const dc_ssa_result_t &sr, uint32_t k,
                                           const dc_kernel_t &D, uint32_t fb, uint32_t n, uint32_t U, uint32_t N,
                                           uint64_t n0, uint32_t *pv, uint32_t *pt, uint32_t *fl, const TyShared &H) {
    const uint32_t t = threadIdx.x, l = lane_id(), K = P.n_kernels;
    const uint16_t *s_rank = H.rank, *s_slot = H.slot;
    const uint32_t *s_vb = H.vb;
    uint32_t *s_w = H.w;
    uint32_t &s_flag = *H.flag, &s_tern = *H.tern;
    uint32_t (*s_red)[3] = H.red;
    unsigned long long *s_h = H.h;
    for (uint32_t x = t; x < N; x += TY_THREADS) {
        ast(pv + x, x);
        ast(pt + x, x);
        ast(fl + x, 0u);
    }
    if (t == 0) s_tern = 0;
    __syncthreads();
    auto node = [&](uint32_t slot, uint32_t ver) { return s_vb[s_rank[slot]] + ver; };

    /* 2. merges */
    const uint64_t po = toff(S, K, 1, k), ao = toff(S, K, 2, k);
    const uint32_t np = sr.n_phi;
    uint32_t acarry = 0;
    for (uint32_t c = 0; c < np; c += TY_THREADS) {
        const uint32_t j = c + t;
        dc_phi_t f{};
        uint32_t inc = 0;
        if (j < np) {
            f = S.phis[po + j];
            const uint32_t b = f.block;
            inc = b == 0 ? 1u : 0u;
            for (uint32_t e = P.pred_cnt[fb + b]; e < P.pred_cnt[fb + b + 1]; e++)
                inc += P.rpo_pos[fb + P.pred[e]] >= 0 ? 1u : 0u;
        }
        uint32_t tot;
        const uint32_t a0 = acarry + block_excl(inc, &tot, s_w);
        acarry += tot;
        if (j < np) {
            S.aoff[po + j] = a0;
            const uint32_t m = node(f.slot, f.version);
            aor(fl + m, TF_MERGE);
            for (uint32_t e = 0; e < inc; e++) {
                const uint32_t y = node(f.slot, S.phi_args[ao + a0 + e]);
                uf_union(pv, m, y);
                uf_union(pt, m, y);
            }
        }
    }

    /* 3. instructions */
    const uint64_t oo = toff(S, K, 3, k);
    uint32_t ocarry = 0, tern = 0;
    for (uint32_t c = 0; c < n; c += TY_THREADS) {
        const uint32_t i = c + t;
        Rec x;
        uint32_t nu = 0, nd = 0, opc = 0, imm = 0;
        if (i < n) {
            const uint4 r = reinterpret_cast<const uint4 *>(P.instrs)[D.instr_begin + i];
            opc = r.x & 0xFFFFu;
            imm = r.z;
            x = load_rec(P, D, i);
            nu = n_uses(x);
            nd = n_defs(x);
        }
        uint32_t tot;
        const uint64_t o = oo + ocarry + block_excl(nu + nd, &tot, s_w);
        ocarry += tot;
        if (i >= n) continue;
        const uint32_t *ver = S.vers + o;
        if ((nu && ver[0] == DC_SSA_NONE) || (nd && ver[nu] == DC_SSA_NONE)) continue;   /* unreachable */
        const uint64_t e = x.e;
        const uint32_t cls = e_cls(e), ty = TYOP[opc];
        const bool mem = cls == C_GLD || cls == C_GST || cls == C_FLD || cls == C_FST;
        const bool saddr = e_role(e, 2) == RO_SADDR && x.id[2] < (uint32_t)NSLOT;
        /* uses: explicit sources in the order r1, r2, third source, stored r0 */
        uint32_t q = 0, first[4] = {NO_Q, NO_Q, NO_Q, NO_Q};
        const int order[4] = {1, 2, 3, 0};
#pragma unroll
        for (int f = 0; f < 4; f++) {
            const int op = order[f];
            const uint32_t role = e_role(e, op);
            if (role == RO_NO || role == RO_SD || role == RO_VD) continue;
            const uint32_t w = e_width(e, op), v = x.id[op];
            for (uint32_t j = 0; j < w; j++) {
                if (v + j >= (uint32_t)NSLOT) continue;
                if (j == 0) first[f] = q;
                uint32_t tt = 0;
                if (mem) tt = f == 0 ? (saddr ? TY_U : TY_P) : (f == 1 ? TY_P : 0u);
                else if (cls == C_DSR || cls == C_DSW) tt = f == 0 ? TY_U : 0u;
                else if (cls == C_SMEM) tt = TY_P;
                else if (f != 3) tt = (ty >> 5) & 31u;
                aor(fl + node(v + j, ver[q]), TF_LIVE | tt);
                q++;
            }
        }
        /* implicit uses (vcc, exec, scc): read, untyped */
        if (q < nu)
            for_uses(x, [&](uint32_t qq, uint32_t slot) {
                if (qq >= q) aor(fl + node(slot, ver[qq]), TF_LIVE);
            });
        /* definitions: the destination dwords */
        const uint32_t r0 = e_role(e, 0);
        const uint32_t w0 = (r0 == RO_SD || r0 == RO_VD) ? e_width(e, 0) : 0u;
        const bool argp = cls == C_SMEM && x.id[1] == 4u && nu >= 2 && ver[0] == 0u && ver[1] == 0u;
        for (uint32_t j = 0; j < w0; j++) {
            uint32_t tt = ty & 31u;
            if (cls == C_SMEM) tt = argp ? smem_type(P, D, imm + 4u * j) : 0u;
            if (tt) aor(fl + node(x.id[0] + j, ver[nu + j]), tt);
        }
        /* copies and the ternary */
        const uint32_t kind = ty >> 10;
        if (kind == TK_COPY && first[0] != NO_Q) {
            const uint32_t w1 = e_width(e, 1);
            for (uint32_t j = 0; j < w0 && j < w1; j++)
                uf_union(pt, node(x.id[0] + j, ver[nu + j]), node(x.id[1] + j, ver[first[0] + j]));
        }
        if (kind == TK_SELECT) {
            tern++;
            const uint32_t d = node(x.id[0], ver[nu]);
            if (first[0] != NO_Q) uf_union(pt, d, node(x.id[1], ver[first[0]]));
            if (first[1] != NO_Q) uf_union(pt, d, node(x.id[2], ver[first[1]]));
        }
    }
    tern = wave_sum32(tern);
    if (l == 0 && tern) atomicAdd(&s_tern, tern);
    __syncthreads();

    /* 4. liveness back through the merges */
    const uint32_t na = sr.n_phi_args;
    for (;;) {
        if (t == 0) s_flag = 0;
        __syncthreads();
        bool grew = false;
        for (uint32_t j = t; j < np; j += TY_THREADS) {
            const dc_phi_t f = S.phis[po + j];
            if (!(ald(fl + node(f.slot, f.version)) & TF_LIVE)) continue;
            const uint32_t a0 = S.aoff[po + j], a1 = j + 1 < np ? S.aoff[po + j + 1] : na;
            for (uint32_t a = a0; a < a1; a++) {
                const uint32_t y = node(f.slot, S.phi_args[ao + a]);
                if (!(ald(fl + y) & TF_LIVE)) {
                    aor(fl + y, TF_LIVE);
                    grew = true;
                }
            }
        }
        if (grew) s_flag = 1;
        __syncthreads();
        const bool again = s_flag != 0;
        __syncthreads();
        if (!again) break;
    }

    /* 5. type bits to the type classes' roots */
    for (uint32_t x = t; x < N; x += TY_THREADS) {
        const uint32_t tt = ald(fl + x) & 0xFFu, r = uf_find(pt, x);
        if (tt && r != x) aor(fl + r, tt);
    }
    __syncthreads();

    /* 6. output */
    uint32_t cv = 0, ct = 0, cm = 0;
    uint64_t h = 0;
    for (uint32_t x = t; x < N; x += TY_THREADS) {
        uint32_t lo = 0, hi = U;   /* the column: the last base <= x */
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (s_vb[mid] <= x) lo = mid;
            else hi = mid;
        }
        dc_var_t V;
        V.slot = s_slot[lo];
        V.version = x - s_vb[lo];
        V.var = uf_find(pv, x);
        V.tclass = uf_find(pt, x);
        V.type = (uint8_t)(ald(fl + V.tclass) & 0xFFu);
        V.flags = (uint8_t)((ald(fl + x) >> 8) & 3u);
        S.vars[n0 + x] = V;
        cv += V.var == x;
        ct += V.tclass == x;
        cm += V.flags == (DC_VF_MERGE | DC_VF_LIVE);
        if (DIGEST) {
            h += ssa_item(6, x, ((uint64_t)V.var << 32) | V.tclass);
            h += ssa_item(7, x, ((uint64_t)V.slot << 48) | ((uint64_t)V.version << 16) | ((uint64_t)V.type << 8) |
                                    V.flags);
        }
    }
    cv = wave_sum32(cv);
    ct = wave_sum32(ct);
    cm = wave_sum32(cm);
    if (DIGEST) h = wave_sum64(h);
    const uint32_t w = t >> 6;
    if (l == 0) {
        s_red[w][0] = cv;
        s_red[w][1] = ct;
        s_red[w][2] = cm;
        s_h[w] = h;
    }
    __syncthreads();
    if (t == 0) {
        dc_types_result_t R{DC_OK, N, 0, 0, 0, s_tern, 0};
        for (uint32_t j = 0; j < TY_WAVES; j++) {
            R.n_vars += s_red[j][0];
            R.n_tclasses += s_red[j][1];
            R.n_live_merges += s_red[j][2];
            R.digest += s_h[j];
        }
        S.tres[k] = R;
    }
}

template <bool DIGEST>
__global__ __launch_bounds__(TY_THREADS) void k_types(Plan P, SsaPlan S) {
    __shared__ uint16_t s_rank[TY_COLS], s_slot[TY_COLS];
    __shared__ uint32_t s_vb[TY_COLS + 1];
    __shared__ uint32_t l_pv[TY_LDS_NODES], l_pt[TY_LDS_NODES], l_fl[TY_LDS_NODES];
    __shared__ uint32_t s_w[TY_WAVES], s_flag, s_tern;
    __shared__ uint32_t s_red[TY_WAVES][3];
    __shared__ unsigned long long s_h[TY_WAVES];
    const uint32_t k = blockIdx.x, t = threadIdx.x, l = lane_id(), K = P.n_kernels;
    const dc_ssa_result_t sr = S.res[k];
    int32_t st = sr.status;
    const uint64_t n0 = toff(S, K, 5, k), c0 = toff(S, K, 6, k);
    if (st == DC_OK && (toff(S, K, 5, k + 1) > S.node_cap || toff(S, K, 6, k + 1) > S.scr_cap)) st = DC_E_CAPACITY;
    if (st != DC_OK) {
        if (t == 0) S.tres[k] = dc_types_result_t{st, 0, 0, 0, 0, 0, 0};
        return;
    }
    const dc_kernel_t D = P.kernels[k];
    const uint32_t fb = P.first_block[k], pb = P.pos_begin[k], n = P.pos_begin[k + 1] - pb;

    /* 1. columns and their node bases */
    const uint32_t *ks = P.kslots + (uint64_t)k * KSLOT_WORDS;
    uint32_t U = 0;
    for (uint32_t w = 0; w < KSLOT_WORDS; w++) U += __popc(slot_word(ks, w));
    for (uint32_t v = t; v < (uint32_t)NSLOT; v += TY_THREADS) {
        uint32_t below = 0;
        for (uint32_t w = 0; w < (v >> 5); w++) below += __popc(slot_word(ks, w));
        const uint32_t word = slot_word(ks, v >> 5), bit = v & 31u;
        if ((word >> bit) & 1u) {
            const uint32_t r = below + __popc(word & ((1u << bit) - 1u));
            s_rank[v] = (uint16_t)r;
            s_slot[r] = (uint16_t)v;
        }
    }
    if (t < 64) {
        const uint32_t *nv = S.nver + toff(S, K, 4, k);
        uint32_t run = 0;
        for (uint32_t c = 0; c < U; c += 64) {
            const uint32_t u = c + l;
            uint32_t tot;
            const uint32_t ex = wave_excl(u < U ? nv[u] : 0u, &tot);
            if (u < U) s_vb[u] = run + ex;
            run += tot;
        }
        if (l == 0) s_vb[U] = run;
    }
    __syncthreads();
    const uint32_t N = s_vb[U];
    const TyShared H{s_rank, s_slot, s_vb, s_w, &s_flag, &s_tern, s_red, s_h};
    if (N <= TY_LDS_NODES)   /* uniform over the workgroup */
        types_body<DIGEST>(P, S, sr, k, D, fb, n, U, N, n0, l_pv, l_pt, l_fl, H);
    else
        types_body<DIGEST>(P, S, sr, k, D, fb, n, U, N, n0, S.tscr + 3 * c0, S.tscr + 3 * c0 + N,
                           S.tscr + 3 * c0 + 2 * (uint64_t)N, H);
}

hipError_t launch_types(const Plan &P, const SsaPlan &S, hipStream_t s) {
    const uint32_t K = P.n_kernels;
    if (!K) return hipSuccess;
    if (S.digest) hipLaunchKernelGGL(k_types<true>, dim3(K), dim3(TY_THREADS), 0, s, P, S);
    else hipLaunchKernelGGL(k_types<false>, dim3(K), dim3(TY_THREADS), 0, s, P, S);
    return hipGetLastError();
}

}  // namespace dc
