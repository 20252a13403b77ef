/*
 * dc_kernels.hip -- HIP kernels for gfx950 (CDNA4) of the register-state
 * dataflow analysis.
 *
 * Stages (all integer work; no MFMA):
 *   a1+a2  k_decode       one thread per instruction: coalesced 16-byte
 *                         record loads, opcode-table lookup, record checks,
 *                         leader flags (textbook basic-block leaders)
 *   a3     k_scan_*       reduce-then-scan of the leader flags over the whole
 *                         batch: global block ids, block_start
 *   a4     k_kernel_info, k_edges, k_pred_*, k_order
 *                         successors, predecessor CSR (count, scan, scatter,
 *                         sort), reverse postorder, per-kernel status
 *   a5-a9  k_fixpoint     persistent grid, one wavefront per analysed kernel:
 *                         ABI entry state, round-robin passes over the reverse
 *                         postorder driven by a dirty bitmap, per-instruction
 *                         transfer on a 368-slot working state in LDS, joins
 *                         into per-block IN states in an HBM arena (change
 *                         detection by ballot), then the extraction walk
 *   out    k_compact      dense output records
 */
#include <hip/hip_runtime.h>

#include "dc_internal.h"
#include "dc_isa.h"

namespace dc {

__constant__ uint64_t OPTAB[N_OPS] = DC_OPTAB_INIT;

/* ------------------------------------------------------------------ */
/* small helpers                                                        */
/* ------------------------------------------------------------------ */
__device__ __forceinline__ uint32_t rfl(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ uint32_t rdl(uint32_t x, uint32_t l) { return __builtin_amdgcn_readlane(x, l); }
__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }
__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & 63; }

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    /* splitmix64 finaliser (Steele, Lea & Flood 2014) */
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* ------------------------------------------------------------------ */
/* record checks (per thread)                                           */
/* ------------------------------------------------------------------ */
__device__ __forceinline__ bool sreg_ok(uint32_t id, uint32_t w) {
    switch (w) {
    case 1: return id <= 107u || id == 109u;
    case 2: return (id & 1u) == 0 && (id <= 102u || id == 104u || id == 106u);
    case 4: return (id & 3u) == 0 && id <= 100u;
    }
    return false;
}
__device__ __forceinline__ bool vreg_ok(uint32_t id, uint32_t w) { return id >= 112u && id + w <= 368u; }
__device__ __forceinline__ bool inl_ok(uint32_t id) {
    return (id >= 0x8000u && id <= 0x8050u) || (id >= 0x8060u && id <= 0x8067u);
}
__device__ bool role_ok(uint32_t role, uint32_t id, uint32_t w, bool lit) {
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
__device__ uint32_t check_record(uint32_t op, uint32_t r0, uint32_t r1, uint32_t r2, int32_t imm, int32_t target,
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
__device__ __forceinline__ bool ends_block(uint32_t cls) { return cls == C_BR || cls == C_CBR || cls == C_END; }

/* ------------------------------------------------------------------ */
/* fills                                                                 */
/* ------------------------------------------------------------------ */
__global__ void k_fill_u32(uint32_t *p, uint64_t n, uint32_t v) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_fill_u8(uint8_t *p, uint64_t n, uint8_t v) {
    /* 16 bytes per thread where aligned, bytes at the tail */
    uint64_t n16 = n / 16;
    uint4 w;
    uint32_t b = v * 0x01010101u;
    w.x = w.y = w.z = w.w = b;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += (uint64_t)gridDim.x * blockDim.x)
        reinterpret_cast<uint4 *>(p)[i] = w;
    for (uint64_t i = n16 * 16 + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
static uint32_t grid_for(uint64_t n, uint32_t per_block) {
    uint64_t g = (n + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > 65536ull * 16) g = 65536ull * 16;
    return (uint32_t)g;
}
hipError_t launch_fill_u32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t s) {
    if (!n) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, 256 * 8)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}
hipError_t launch_fill_u8(uint8_t *p, uint64_t n, uint8_t v, hipStream_t s) {
    if (!n) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u8, dim3(grid_for(n / 16 + 1, 256 * 8)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

/* ------------------------------------------------------------------ */
/* position -> kernel lookup for a tile of positions                     */
/* ------------------------------------------------------------------ */
constexpr int TILE_LK = 1024;          /* positions per lookup tile */
constexpr int LK_CAP = TILE_LK + 2;    /* kernel starts cached in LDS */

/* last k in [lo, hi] with pos_begin[k] <= g (global memory) */
__device__ uint32_t kernel_of_global(const uint32_t *pos_begin, uint32_t lo, uint32_t hi, uint32_t g) {
    while (lo < hi) {
        uint32_t mid = lo + (hi - lo + 1) / 2;
        if (pos_begin[mid] <= g) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

/* Cooperative setup for a tile [t0, t1): caches the starts of the kernels
 * that overlap it.  Returns k0 and the count (0 if they do not fit). */
__device__ void lookup_setup(const uint32_t *pos_begin, uint32_t K, uint32_t t0, uint32_t t1, uint32_t *lk,
                             uint32_t *k0_out, uint32_t *cnt_out) {
    __shared__ uint32_t s_k0, s_k1;
    if (threadIdx.x == 0) {
        s_k0 = kernel_of_global(pos_begin, 0, K - 1, t0);
        s_k1 = kernel_of_global(pos_begin, s_k0, K - 1, t1 - 1);
    }
    __syncthreads();
    uint32_t k0 = s_k0, cnt = s_k1 - s_k0 + 1;
    if (cnt <= (uint32_t)LK_CAP) {
        for (uint32_t i = threadIdx.x; i < cnt; i += blockDim.x) lk[i] = pos_begin[k0 + i];
    } else {
        cnt = 0;
    }
    __syncthreads();
    *k0_out = k0;
    *cnt_out = cnt;
}
__device__ __forceinline__ uint32_t lookup(const uint32_t *pos_begin, uint32_t K, const uint32_t *lk, uint32_t k0,
                                           uint32_t cnt, uint32_t g) {
    if (cnt == 0) return kernel_of_global(pos_begin, k0, K - 1, g);
    uint32_t lo = 0, hi = cnt - 1;
    while (lo < hi) {
        uint32_t mid = lo + (hi - lo + 1) / 2;
        if (lk[mid] <= g) lo = mid;
        else hi = mid - 1;
    }
    return k0 + lo;
}

/* ------------------------------------------------------------------ */
/* a1 + a2: decode, check, leader flags                                  */
/* ------------------------------------------------------------------ */
__global__ __launch_bounds__(256) void k_decode(Plan P) {
    __shared__ uint32_t lk[LK_CAP];
    const uint32_t t0 = blockIdx.x * TILE_LK;
    if (t0 >= P.n_pos) return;
    const uint32_t t1 = min(P.n_pos, t0 + TILE_LK);
    uint32_t k0, cnt;
    lookup_setup(P.pos_begin, P.n_kernels, t0, t1, lk, &k0, &cnt);
    for (uint32_t g = t0 + threadIdx.x; g < t1; g += blockDim.x) {
        const uint32_t k = lookup(P.pos_begin, P.n_kernels, lk, k0, cnt, g);
        const uint32_t pb = P.pos_begin[k];
        const uint32_t n = P.pos_begin[k + 1] - pb;
        const uint32_t i = g - pb;
        const dc_kernel_t *D = &P.kernels[k];
        const uint4 r = reinterpret_cast<const uint4 *>(P.instrs)[D->instr_begin + i];
        const uint32_t op = r.x & 0xFFFFu, r0 = r.x >> 16, r1 = r.y & 0xFFFFu, r2 = r.y >> 16;
        const int32_t imm = (int32_t)r.z, target = (int32_t)r.w;
        const uint32_t bad = check_record(op, r0, r1, r2, imm, target, n);
        if (i == 0) P.leader[g] = 1;
        if (bad) {
            atomicMin(&P.kbad[k], (i << 2) | bad);
            continue;
        }
        const uint32_t cls = e_cls(OPTAB[op]);
        if (ends_block(cls) && i + 1 < n) P.leader[g + 1] = 1;
        if (cls == C_BR || cls == C_CBR) P.leader[pb + (uint32_t)target] = 1;
    }
}
hipError_t launch_decode(const Plan &P, hipStream_t s) {
    if (!P.n_pos) return hipSuccess;
    uint32_t tiles = (P.n_pos + TILE_LK - 1) / TILE_LK;
    hipLaunchKernelGGL(k_decode, dim3(tiles), dim3(256), 0, s, P);
    return hipGetLastError();
}

/* ------------------------------------------------------------------ */
/* block-wide scan helpers (256 threads)                                 */
/* ------------------------------------------------------------------ */
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
    const uint32_t l = lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t y = __shfl_up(x, d, 64);
        if (l >= (uint32_t)d) x += y;
    }
    return x;
}
/* exclusive scan across the 256 threads of a block; returns the block total */
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t x, uint32_t *out_excl) {
    __shared__ uint32_t wsum[4];
    const uint32_t w = threadIdx.x >> 6, l = lane_id();
    uint32_t inc = wave_incl_scan(x);
    if (l == 63) wsum[w] = inc;
    __syncthreads();
    uint32_t base = 0, total = 0;
    for (uint32_t j = 0; j < 4; j++) {
        if (j < w) base += wsum[j];
        total += wsum[j];
    }
    __syncthreads();
    *out_excl = base + inc - x;
    return total;
}

constexpr int SCAN_ITEMS = 16;
constexpr int SCAN_TILE = 256 * SCAN_ITEMS;   /* 4096 elements per tile */

template <typename T>
__device__ __forceinline__ void load_items(const T *in, uint64_t n, uint64_t base, uint32_t v[SCAN_ITEMS]) {
    const uint64_t s = base + (uint64_t)threadIdx.x * SCAN_ITEMS;
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; j++) v[j] = (s + j < n) ? (uint32_t)in[s + j] : 0u;
}

template <typename T>
__global__ __launch_bounds__(256) void k_scan_reduce(const T *in, uint64_t n, uint32_t *tile_sums) {
    uint32_t v[SCAN_ITEMS];
    load_items(in, n, (uint64_t)blockIdx.x * SCAN_TILE, v);
    uint32_t s = 0;
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; j++) s += v[j];
    uint32_t excl;
    uint32_t tot = block_excl_scan(s, &excl);
    if (threadIdx.x == 0) tile_sums[blockIdx.x] = tot;
}

/* exclusive scan with per-tile offsets; out may alias in (T == uint32_t) */
template <typename T>
__global__ __launch_bounds__(256) void k_scan_apply(const T *in, uint64_t n, const uint32_t *tile_offs,
                                                     uint32_t *out, uint32_t *total_out) {
    uint32_t v[SCAN_ITEMS];
    const uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE;
    load_items(in, n, base, v);
    uint32_t s = 0;
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; j++) s += v[j];
    uint32_t excl;
    uint32_t tot = block_excl_scan(s, &excl);
    uint32_t run = tile_offs[blockIdx.x] + excl;
    const uint64_t st = base + (uint64_t)threadIdx.x * SCAN_ITEMS;
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; j++) {
        if (st + j < n) out[st + j] = run;
        run += v[j];
    }
    if (total_out && blockIdx.x == gridDim.x - 1 && threadIdx.x == 255) *total_out = tile_offs[blockIdx.x] + tot;
}

uint64_t scan_tmp_words_needed(uint64_t n) {
    uint64_t words = 0;
    while (true) {
        uint64_t tiles = (n + SCAN_TILE - 1) / SCAN_TILE;
        if (tiles < 1) tiles = 1;
        words += tiles + 1;
        if (tiles == 1) break;
        n = tiles;
    }
    return words + 16;
}

/* exclusive scan of in[0..n) into out (u32); *total_out (device) = sum */
template <typename T>
hipError_t scan_excl(const T *in, uint64_t n, uint32_t *out, uint32_t *total_out, uint32_t *tmp, hipStream_t s) {
    if (n == 0) {
        if (total_out) hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, total_out, (uint64_t)1, 0u);
        return hipGetLastError();
    }
    uint64_t tiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (tiles == 1) {
        hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, tmp, (uint64_t)1, 0u);
        hipLaunchKernelGGL(k_scan_apply<T>, dim3(1), dim3(256), 0, s, in, n, tmp, out, total_out);
        return hipGetLastError();
    }
    uint32_t *sums = tmp;
    hipLaunchKernelGGL(k_scan_reduce<T>, dim3((uint32_t)tiles), dim3(256), 0, s, in, n, sums);
    hipError_t e = scan_excl<uint32_t>(sums, tiles, sums, nullptr, tmp + tiles + 1, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scan_apply<T>, dim3((uint32_t)tiles), dim3(256), 0, s, in, n, sums, out, total_out);
    return hipGetLastError();
}

/* ------------------------------------------------------------------ */
/* a3: block numbering                                                   */
/* ------------------------------------------------------------------ */
/* block_id[g] = (exclusive leader count at g) + leader[g] - 1, and for every
 * leader g: block_start[id] = g, block_kernel[id] = kernel of g */
__global__ __launch_bounds__(256) void k_number(Plan P, const uint32_t *excl) {
    __shared__ uint32_t lk[LK_CAP];
    const uint32_t t0 = blockIdx.x * TILE_LK;
    if (t0 >= P.n_pos) return;
    const uint32_t t1 = min(P.n_pos, t0 + TILE_LK);
    uint32_t k0, cnt;
    lookup_setup(P.pos_begin, P.n_kernels, t0, t1, lk, &k0, &cnt);
    for (uint32_t g = t0 + threadIdx.x; g < t1; g += blockDim.x) {
        const uint32_t l = P.leader[g];
        const uint32_t id = excl[g] + l - 1;
        P.block_id[g] = id;
        if (l) {
            P.block_start[id] = g;
            P.block_kernel[id] = lookup(P.pos_begin, P.n_kernels, lk, k0, cnt, g);
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) P.block_start[*P.total_blocks] = P.n_pos;
}

hipError_t launch_number_blocks(const Plan &P, hipStream_t s) {
    if (!P.n_pos) {
        hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, P.total_blocks, (uint64_t)1, 0u);
        hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, P.block_start, (uint64_t)1, 0u);
        return hipGetLastError();
    }
    /* the exclusive leader counts go to block_id first, then k_number rewrites
     * block_id in place (each position reads its own entry before writing) */
    hipError_t e = scan_excl<uint8_t>(P.leader, P.n_pos, P.block_id, P.total_blocks, P.scan_tmp, s);
    if (e != hipSuccess) return e;
    uint32_t tiles = (P.n_pos + TILE_LK - 1) / TILE_LK;
    hipLaunchKernelGGL(k_number, dim3(tiles), dim3(256), 0, s, P, P.block_id);
    return hipGetLastError();
}

/* ------------------------------------------------------------------ */
/* a4: per-kernel info, edges, predecessors, reverse postorder          */
/* ------------------------------------------------------------------ */
constexpr int32_t ST_OK = 0;

__global__ void k_kernel_info(Plan P) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= P.n_kernels) return;
    const uint32_t pb = P.pos_begin[k], n = P.pos_begin[k + 1] - pb;
    int32_t st = P.desc_status[k];
    if (st == ST_OK) {
        const uint32_t bad = P.kbad[k];
        if (bad != 0xFFFFFFFFu) {
            const uint32_t code = bad & 3u;
            st = code == 1 ? DC_E_BADOP : code == 2 ? DC_E_BADREG : DC_E_BADTARGET;
        } else if (n == 0) {
            st = DC_E_NOEND;
        } else {
            const dc_kernel_t *D = &P.kernels[k];
            const uint32_t op = P.instrs[D->instr_begin + n - 1].op;
            const uint32_t cls = e_cls(OPTAB[op]);
            if (!(cls == C_BR || cls == C_END)) st = DC_E_NOEND;
        }
    }
    P.status[k] = st;
    uint32_t fb = 0, nb = 0;
    if (n) {
        fb = P.block_id[pb];
        nb = P.block_id[pb + n - 1] - fb + 1;
    }
    P.first_block[k] = fb;
    P.n_blocks[k] = nb;
}

__global__ void k_edges(Plan P) {
    const uint32_t total = *P.total_blocks;
    for (uint32_t b = blockIdx.x * blockDim.x + threadIdx.x; b < total; b += gridDim.x * blockDim.x) {
        const uint32_t k = P.block_kernel[b];
        int32_t s0 = -1, s1 = -1;
        if (P.status[k] == ST_OK) {
            const uint32_t fb = P.first_block[k], nb = P.n_blocks[k], pb = P.pos_begin[k];
            const uint32_t last = P.block_start[b + 1] - 1;
            const dc_instr_t R = P.instrs[P.kernels[k].instr_begin + (last - pb)];
            const uint32_t cls = e_cls(OPTAB[R.op]);
            const uint32_t lb = b - fb;
            if (cls != C_BR && cls != C_END && lb + 1 < nb) s0 = (int32_t)(lb + 1);
            if (cls == C_BR || cls == C_CBR) s1 = (int32_t)(P.block_id[pb + (uint32_t)R.target] - fb);
            if (s1 == s0) s1 = -1;
            if (s0 >= 0) atomicAdd(&P.pred_cnt[fb + (uint32_t)s0], 1u);
            if (s1 >= 0) atomicAdd(&P.pred_cnt[fb + (uint32_t)s1], 1u);
        }
        P.succ[2 * (uint64_t)b] = s0;
        P.succ[2 * (uint64_t)b + 1] = s1;
    }
}

__global__ void k_pred_scatter(Plan P) {
    const uint32_t total = *P.total_blocks;
    for (uint32_t b = blockIdx.x * blockDim.x + threadIdx.x; b < total; b += gridDim.x * blockDim.x) {
        const uint32_t k = P.block_kernel[b];
        const uint32_t fb = P.first_block[k];
        for (int e = 0; e < 2; e++) {
            const int32_t s = P.succ[2 * (uint64_t)b + e];
            if (s < 0) continue;
            const uint32_t t = fb + (uint32_t)s;
            const uint32_t slot = atomicAdd(&P.pred_fill[t], 1u);
            P.pred[P.pred_cnt[t] + slot] = b - fb;
        }
    }
}

/* one thread per kernel: sort each block's predecessor list and compute the
 * reverse postorder of a DFS from block 0 that takes the fall-through edge
 * first (iterative; the stack holds block ids with the next edge in bit 31) */
__global__ void k_order(Plan P) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= P.n_kernels) return;
    const uint32_t fb = P.first_block[k], nb = P.n_blocks[k];
    if (P.status[k] != ST_OK || nb == 0) {
        P.n_reach[k] = 0;
        return;
    }
    for (uint32_t b = 0; b < nb; b++) {
        uint32_t lo = P.pred_cnt[fb + b], hi = P.pred_cnt[fb + b + 1];
        for (uint32_t i = lo + 1; i < hi; i++) {
            uint32_t x = P.pred[i], j = i;
            while (j > lo && P.pred[j - 1] > x) {
                P.pred[j] = P.pred[j - 1];
                j--;
            }
            P.pred[j] = x;
        }
        P.dfs_seen[fb + b] = 0;
        P.rpo_pos[fb + b] = -1;
    }
    /* explicit-stack emulation of the recursive DFS: an entry holds a block
     * id and, in bits 31:30, the index of the next out-edge to examine */
    uint32_t *stk = P.dfs_stack + fb;
    uint32_t *post = P.rpo + fb;   /* postorder first, reversed below */
    uint32_t sp = 0, np = 0;
    stk[sp++] = 0;
    P.dfs_seen[fb] = 1;
    while (sp) {
        const uint32_t top = stk[sp - 1];
        const uint32_t u = top & 0x3FFFFFFFu, e = top >> 30;
        if (e < 2) {
            stk[sp - 1] = u | ((e + 1) << 30);
            const int32_t s = P.succ[2 * (uint64_t)(fb + u) + e];
            if (s >= 0 && !P.dfs_seen[fb + (uint32_t)s]) {
                P.dfs_seen[fb + (uint32_t)s] = 1;
                stk[sp++] = (uint32_t)s;
            }
        } else {
            sp--;
            post[np++] = u;
        }
    }
    for (uint32_t i = 0; i < np / 2; i++) {
        uint32_t t = post[i];
        post[i] = post[np - 1 - i];
        post[np - 1 - i] = t;
    }
    for (uint32_t i = 0; i < np; i++) P.rpo_pos[fb + post[i]] = (int32_t)i;
    P.n_reach[k] = np;
}

hipError_t launch_edges(const Plan &P, hipStream_t s) {
    const uint32_t K = P.n_kernels;
    if (K) hipLaunchKernelGGL(k_kernel_info, dim3((K + 255) / 256), dim3(256), 0, s, P);
    hipError_t e = launch_fill_u32(P.pred_cnt, (uint64_t)P.n_pos + 1, 0u, s);
    if (e != hipSuccess) return e;
    e = launch_fill_u32(P.pred_fill, (uint64_t)P.n_pos, 0u, s);
    if (e != hipSuccess) return e;
    const uint32_t grid = grid_for(P.n_pos ? P.n_pos : 1, 256 * 4);
    hipLaunchKernelGGL(k_edges, dim3(grid), dim3(256), 0, s, P);
    e = scan_excl<uint32_t>(P.pred_cnt, (uint64_t)P.n_pos + 1, P.pred_cnt, nullptr, P.scan_tmp, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_pred_scatter, dim3(grid), dim3(256), 0, s, P);
    if (K) hipLaunchKernelGGL(k_order, dim3((K + 63) / 64), dim3(64), 0, s, P);
    return hipGetLastError();
}


/* ------------------------------------------------------------------ */
/* a5-a9: fixpoint and extraction                                        */
/* ------------------------------------------------------------------ */
/* One wavefront analyses one kernel.  Control flow in this section is
 * wave-uniform: every lane runs the same scalar code on values read from
 * LDS with a broadcast and made uniform with readfirstlane.  Lane-parallel
 * work (state copies, joins, bitmap scans, record staging) uses all 64 lanes.
 *
 * No branch here depends on the lane id.  A "lane 0 only" store is written
 * as a store by every lane, lane 0 to the real address and the other lanes
 * to a private 64-entry scratch tail; values that one lane computes (the
 * work counter) come from branch-free atomics read with readfirstlane.  A
 * lane-predicated branch lets the optimiser thread the predicate across the
 * loop back edge, splitting the wave so that lanes 1..63 re-enter the loop
 * without lane 0 (which is how a readlane of lane 0's work index can see a
 * stale value and never reach the loop exit). */

struct SV {
    uint32_t prov, type;
    uint64_t val;
};

struct KCtx {
    uint32_t cws0, cws1, cws2, n_args;
    const dc_arg_t *args;
    __device__ __forceinline__ uint32_t cws(uint32_t d) const { return d == 0 ? cws0 : d == 1 ? cws1 : cws2; }
};

__device__ __forceinline__ SV lds_get(const uint4 *st, uint32_t s) {
    const uint4 v = st[s];
    SV r;
    r.prov = rfl(v.x);
    r.type = rfl(v.y);
    r.val = ((uint64_t)rfl(v.w) << 32) | rfl(v.z);
    return r;
}
/* st points at NSLOT state slots followed by a 64-slot scratch tail */
__device__ __forceinline__ void lds_put(uint4 *st, uint32_t s, uint32_t prov, uint32_t type, uint64_t val) {
    const uint32_t l = lane_id();
    st[l == 0 ? s : (uint32_t)NSLOT + l] = make_uint4(prov, type, (uint32_t)val, (uint32_t)(val >> 32));
}

__device__ __forceinline__ bool is_c(uint64_t v) { return v != VTOP && v_tag(v) == T_CONST; }
__device__ __forceinline__ uint64_t C32(uint32_t c) { return (uint64_t)c; }
__device__ __forceinline__ bool idx_lo(uint64_t v) {
    return v != VTOP && v_tag(v) == T_IDX && v_ig(v) <= IG_LO;
}
__device__ __forceinline__ int lg2(uint32_t x) {
    /* exact base-2 logarithm, -1 when x is not a power of two */
    return (x != 0 && (x & (x - 1)) == 0) ? (int)__builtin_ctz(x) : -1;
}

/* dword j of operand id as a source of width w */
__device__ __forceinline__ SV src_operand(const uint4 *st, uint32_t id, uint32_t j, uint32_t w, int32_t imm) {
    if (id < (uint32_t)NSLOT) return lds_get(st, id + j);
    SV r;
    r.prov = 1u << PB_CONST;
    r.type = 0;
    if (id <= 0x8050u) {
        const int32_t k = (int32_t)(id - 0x8000u) - 16;
        r.val = j == 0 ? C32((uint32_t)k) : C32(k < 0 ? 0xFFFFFFFFu : 0u);
    } else if (id >= 0x8060u && id <= 0x8067u) {
        /* +-0.5, +-1, +-2, +-4: sign in bit 0 of the index, magnitude 2^(q/2-1) */
        const uint32_t q = id - 0x8060u, neg = q & 1u, m = q >> 1;
        if (w == 1) r.val = C32((neg << 31) | ((126u + m) << 23));
        else r.val = j == 0 ? 0 : C32((neg << 31) | ((1022u + m) << 20));
    } else {
        r.val = j == 0 ? C32((uint32_t)imm) : C32(imm < 0 ? 0xFFFFFFFFu : 0u);
    }
    return r;
}

/* ---- payload rules ---- */
__device__ uint64_t r_add1(uint64_t a, uint64_t b) {
    const uint32_t ta = v_tag(a), tb = v_tag(b);
    if (is_c(a) && is_c(b)) return C32(v_c(a) + v_c(b));
    if (idx_lo(a) && idx_lo(b) && v_dim(a) == v_dim(b) && (v_aux(a) & v_aux(b)) == 0)
        return pv(T_IDX, IG_ENT, v_dim(a), v_aux(a) | v_aux(b), 0, 0, v_c(a) + v_c(b));
    if (idx_lo(a) && is_c(b)) return pv(T_IDX, IG_ENT, v_dim(a), v_aux(a), 0, 0, v_c(a) + v_c(b));
    if (ta == T_SHL && v_ig(a) == IG_ENT && is_c(b))
        return pv(T_SHL, IG_ENT, v_dim(a), v_aux(a), v_sh(a), 0, v_c(a) + v_c(b));
    if (ta == T_KARG && v_ig(a) == IG_LO) {
        if (tb == T_SHL && v_ig(b) == IG_LO) return pv(T_PTR, IG_LO, v_dim(b), v_aux(b), v_sh(b), v_arg(a), v_c(b));
        if (is_c(b)) return pv(T_PTR, IG_LO, 0, 0, 0, v_arg(a), v_c(b));
    }
    if (ta == T_PTR && v_ig(a) == IG_LO) {
        if (is_c(b)) return pv(T_PTR, IG_LO, v_dim(a), v_aux(a), v_sh(a), v_arg(a), v_c(a) + v_c(b));
        if (tb == T_SHL && v_ig(b) == IG_LO && v_dim(a) == 0 && v_aux(a) == 0 && v_sh(a) == 0)
            return pv(T_PTR, IG_LO, v_dim(b), v_aux(b), v_sh(b), v_arg(a), v_c(a) + v_c(b));
    }
    return VTOP;
}
__device__ __forceinline__ uint64_t r_add(uint64_t a, uint64_t b) {
    if (a == VTOP || b == VTOP) return VTOP;
    const uint64_t r = r_add1(a, b);
    return r != VTOP ? r : r_add1(b, a);
}
__device__ __forceinline__ bool ptr_hi(uint64_t v) {
    return v != VTOP && (v_tag(v) == T_KARG || v_tag(v) == T_PTR) && v_ig(v) == IG_HI;
}
__device__ __forceinline__ bool ext_hi(uint64_t v) {
    return v != VTOP && (((v_tag(v) == T_SHL || v_tag(v) == T_IDX) && v_ig(v) == IG_HI) || (is_c(v) && v_c(v) == 0));
}
__device__ __forceinline__ uint64_t r_addc(uint64_t a, uint64_t b) {
    if (ptr_hi(a) && ext_hi(b)) return pv(T_PTR, IG_HI, 0, 0, 0, v_arg(a), 0);
    if (ptr_hi(b) && ext_hi(a)) return pv(T_PTR, IG_HI, 0, 0, 0, v_arg(b), 0);
    return VTOP;
}
/* IDX shifted left by s */
__device__ __forceinline__ uint64_t idx_shl(uint64_t a, uint32_t s) {
    if (s == 0) return pv(T_IDX, IG_ENT, v_dim(a), v_aux(a), 0, 0, v_c(a));
    if (s > 15) return VTOP;
    return pv(T_SHL, IG_ENT, v_dim(a), v_aux(a), s, 0, v_c(a) << s);
}
__device__ uint64_t r_mul1(const KCtx &K, uint64_t a, uint64_t b) {
    if (is_c(a) && is_c(b)) return C32(v_c(a) * v_c(b));
    if (!is_c(b)) return VTOP;
    if (a != VTOP && v_tag(a) == T_WGID) {
        const uint32_t d = v_dim(a);
        return (K.cws(d) != 0 && v_c(b) == K.cws(d)) ? pv(T_IDX, IG_ENT, d, M_WG, 0, 0, 0) : VTOP;
    }
    if (idx_lo(a)) {
        const int s = lg2(v_c(b));
        if (s >= 0) return idx_shl(a, (uint32_t)s);
    }
    return VTOP;
}
__device__ __forceinline__ uint64_t r_mul(const KCtx &K, uint64_t a, uint64_t b) {
    if (a == VTOP || b == VTOP) return VTOP;
    const uint64_t r = r_mul1(K, a, b);
    return r != VTOP ? r : r_mul1(K, b, a);
}
__device__ __forceinline__ uint64_t low24(uint64_t v) { return is_c(v) ? C32(v_c(v) & 0xFFFFFFu) : v; }

__device__ uint64_t r_shl(const KCtx &K, uint64_t x, uint64_t amt) {
    if (x == VTOP || !is_c(amt)) return VTOP;
    const uint32_t s = v_c(amt) & 31u;
    if (is_c(x)) return C32(v_c(x) << s);
    if (idx_lo(x)) return idx_shl(x, s);
    if (v_tag(x) == T_WGID && lg2(K.cws(v_dim(x))) == (int)s) return pv(T_IDX, IG_ENT, v_dim(x), M_WG, 0, 0, 0);
    return VTOP;
}
__device__ uint64_t r_lshr(const KCtx &K, uint64_t x, uint64_t amt) {
    if (x == VTOP || !is_c(amt)) return VTOP;
    const uint32_t s = v_c(amt) & 31u;
    if (is_c(x)) return C32(v_c(x) >> s);
    if (v_tag(x) == T_SYS && v_aux(x) == K_GSIZE && v_ig(x) == IG_ENT && lg2(K.cws(v_dim(x))) == (int)s)
        return pv(T_SYS, IG_ENT, v_dim(x), K_NUMGROUPS, 0, 0, 0);
    return VTOP;
}
__device__ uint64_t r_ashr(uint64_t x, uint64_t amt) {
    if (x == VTOP || !is_c(amt)) return VTOP;
    const uint32_t s = v_c(amt) & 31u;
    if (is_c(x)) return C32((uint32_t)((int32_t)v_c(x) >> s));
    if (idx_lo(x) && s == 31) return pv(T_IDX, IG_HI, v_dim(x), v_aux(x), 0, 0, 0);
    return VTOP;
}

/* resolution of one dword of the kernel-argument area addressed by s[4:5] */
__device__ __forceinline__ void arg_dword(const KCtx &K, uint32_t o, uint32_t &prov, uint32_t &type, uint64_t &val) {
    if ((o & 3u) == 0 && o < 0x30u) {
        const uint32_t q = o >> 3, hi = (o >> 2) & 1u;
        if (o < 0x18u) {   /* global offsets x, y, z */
            prov = 1u << (PB_GOFF + q);
            type = TY_U;
            val = hi ? pv(T_SYS, IG_HI, q, K_GOFFHI, 0, 0, 0) : pv(T_IDX, IG_LO, q, M_GOFF, 0, 0, 0);
        } else {           /* printf buffer, vqueue, aqlwrap */
            prov = 1u << PB_HIDDEN;
            type = 0;
            val = pv(T_SYS, hi ? IG_HI : IG_LO, q - 3, K_HIDDEN, 0, 0, 0);
        }
        return;
    }
    if (o == 0x20010u) {
        prov = 1u << PB_WORKDIM;
        type = TY_U;
        val = pv(T_SYS, IG_ENT, 0, K_WORKDIM, 0, 0, 0);
        return;
    }
    for (uint32_t k = 0; k < K.n_args; k++) {
        const uint32_t off = K.args[k].offset, sz = K.args[k].size;
        if (o >= off && (uint64_t)o < (uint64_t)off + sz) {
            prov = 1u << (PB_KARG + (k < 11 ? k : 11));
            type = K.args[k].type;
            if (sz == 4 && o == off) val = pv(T_KARG, IG_ENT, 0, 0, 0, k, 0);
            else if (sz == 8 && o == off) val = pv(T_KARG, IG_LO, 0, 0, 0, k, 0);
            else if (sz == 8 && o == off + 4) val = pv(T_KARG, IG_HI, 0, 0, 0, k, 0);
            else val = VTOP;
            return;
        }
    }
    prov = 1u << PB_LOADG;
    type = 0;
    val = VTOP;
}

struct Defs {
    uint32_t n;        /* explicit def dwords written */
    uint32_t slot0;
    uint32_t imp;      /* implicit def set */
    uint64_t v[4];     /* their payloads */
};

/* Apply one instruction to the LDS working state (sources read first). */
__device__ __forceinline__ Defs apply(uint4 *st, const KCtx &K, uint32_t op, uint32_t r0, uint32_t r1, uint32_t r2, int32_t imm,
                      uint64_t e) {
    Defs D;
    D.n = 0;
    D.slot0 = r0;
    D.imp = 0;
    D.v[0] = D.v[1] = D.v[2] = D.v[3] = VTOP;
    const uint32_t cls = e_cls(e);
    if (cls == C_SMEM) {
        const uint32_t w = e_width(e, 0);
        const bool via = r1 == 4u;
        const bool ok = via && lds_get(st, 4).val == pv(T_SYSPTR, IG_LO, 0, 0, 0, 0, 0) &&
                        lds_get(st, 5).val == pv(T_SYSPTR, IG_HI, 0, 0, 0, 0, 0);
        const uint32_t off = (uint32_t)imm;
        uint32_t pr[4], ty[4];
        uint64_t va[4];
#pragma unroll
        for (uint32_t j = 0; j < 4; j++) {
            pr[j] = 1u << PB_LOADG;
            ty[j] = 0;
            va[j] = VTOP;
            if (via && j < w) arg_dword(K, off + 4u * j, pr[j], ty[j], va[j]);
        }
        if (via && w == 2 && (off == 0u || off == 8u || off == 16u)) {
            const uint32_t d = off >> 3;
            pr[0] = pr[1] = 1u << (PB_GOFF + d);
            ty[0] = ty[1] = TY_U;
            va[0] = pv(T_IDX, IG_LO, d, M_GOFF, 0, 0, 0);
            va[1] = pv(T_SYS, IG_HI, d, K_GOFFHI, 0, 0, 0);
        } else if (via && w == 1 && (off == 0xCu || off == 0x10u || off == 0x14u)) {
            const uint32_t d = (off - 0xCu) >> 2;
            pr[0] = 1u << (PB_GSIZE + d);
            ty[0] = TY_U;
            va[0] = pv(T_SYS, IG_ENT, d, K_GSIZE, 0, 0, 0);
        } else if (via && w == 1 && off == 0x20010u) {
            pr[0] = 1u << PB_WORKDIM;
            ty[0] = TY_U;
            va[0] = pv(T_SYS, IG_ENT, 0, K_WORKDIM, 0, 0, 0);
        }
#pragma unroll
        for (uint32_t j = 0; j < 4; j++) {
            D.v[j] = ok ? va[j] : VTOP;
            if (j < w) lds_put(st, r0 + j, pr[j], ty[j], D.v[j]);
        }
        D.n = w;
        return D;
    }
    if (cls == C_GLD || cls == C_FLD || cls == C_DSR) {
        const uint32_t w = e_width(e, 0);
        const uint32_t pr = cls == C_DSR ? 1u << PB_LOADL : 1u << PB_LOADG;
#pragma unroll
        for (uint32_t j = 0; j < 4; j++) {
            D.v[j] = VTOP;
            if (j < w) lds_put(st, r0 + j, pr, 0, VTOP);
        }
        D.n = w;
        return D;
    }
    if (cls != C_SALU && cls != C_SCMP && cls != C_VALU && cls != C_VCMP) return D;

    /* gather sources */
    const uint32_t w1 = e_role(e, 1) != RO_NO ? e_width(e, 1) : 0;
    const uint32_t w2 = e_role(e, 2) != RO_NO ? e_width(e, 2) : 0;
    const uint32_t w3 = e_role(e, 3) != RO_NO ? e_width(e, 3) : 0;
    SV a0 = {0, 0, VTOP}, a1 = {0, 0, VTOP}, b0 = {0, 0, VTOP}, b1 = {0, 0, VTOP}, c0 = {0, 0, VTOP};
    uint32_t rp = 0;
    if (w1) { a0 = src_operand(st, r1, 0, w1, imm); rp |= a0.prov; }
    if (w1 == 2) { a1 = src_operand(st, r1, 1, w1, imm); rp |= a1.prov; }
    if (w2) { b0 = src_operand(st, r2, 0, w2, imm); rp |= b0.prov; }
    if (w2 == 2) { b1 = src_operand(st, r2, 1, w2, imm); rp |= b1.prov; }
    if (w3) {
        c0 = src_operand(st, (uint32_t)imm, 0, w3, 0);
        rp |= c0.prov;
        if (w3 == 2) rp |= src_operand(st, (uint32_t)imm, 1, w3, 0).prov;
    }
    const uint32_t iu = e_iuse(e);
    if (iu & IM_VCC) rp |= lds_get(st, 104).prov | lds_get(st, 105).prov;
    if (iu & IM_EXEC) rp |= lds_get(st, 106).prov | lds_get(st, 107).prov;
    if (iu & IM_SCC) rp |= lds_get(st, 108).prov;

    const uint32_t rrole = e_role(e, 0);
    if (rrole == RO_SD || rrole == RO_VD) {
        const uint32_t w0 = e_width(e, 0);
        uint32_t ty0 = 0, ty1 = 0;
        switch (e_trule(e)) {
        case TR_SUF: ty0 = ty1 = e_suffix(e); break;
        case TR_ADD: ty0 = ty1 = e_suffix(e) | ((a0.type | a1.type | b0.type | b1.type) & TY_P); break;
        case TR_B: {
            const uint32_t vs = e_vsrc(e);
            uint32_t t = 0;
            if (vs & 1u) t |= a0.type | a1.type;
            if (vs & 2u) t |= b0.type | b1.type;
            ty0 = ty1 = t;
            break;
        }
        case TR_MOVE: ty0 = a0.type; ty1 = a1.type; break;
        default: break;
        }
        uint64_t v0 = VTOP, v1 = VTOP;
        const bool val_is_r1 = e_vsrc(e) == 1u;   /* shift forms: which operand is shifted */
        switch (e_prule(e)) {
        case PR_MOV: v0 = a0.val; v1 = a1.val; break;
        case PR_ADD: v0 = r_add(a0.val, b0.val); break;
        case PR_ADDC: v0 = r_addc(a0.val, b0.val); break;
        case PR_SUB: if (is_c(a0.val) && is_c(b0.val)) v0 = C32(v_c(a0.val) - v_c(b0.val)); break;
        case PR_AND: if (is_c(a0.val) && is_c(b0.val)) v0 = C32(v_c(a0.val) & v_c(b0.val)); break;
        case PR_OR: if (is_c(a0.val) && is_c(b0.val)) v0 = C32(v_c(a0.val) | v_c(b0.val)); break;
        case PR_XOR: if (is_c(a0.val) && is_c(b0.val)) v0 = C32(v_c(a0.val) ^ v_c(b0.val)); break;
        case PR_MUL: v0 = r_mul(K, a0.val, b0.val); break;
        case PR_MUL24: v0 = r_mul(K, low24(a0.val), low24(b0.val)); break;
        case PR_MAD24: v0 = r_add(r_mul(K, low24(a0.val), low24(b0.val)), c0.val); break;
        case PR_SHL: v0 = val_is_r1 ? r_shl(K, a0.val, b0.val) : r_shl(K, b0.val, a0.val); break;
        case PR_LSHR: v0 = val_is_r1 ? r_lshr(K, a0.val, b0.val) : r_lshr(K, b0.val, a0.val); break;
        case PR_ASHR: v0 = val_is_r1 ? r_ashr(a0.val, b0.val) : r_ashr(b0.val, a0.val); break;
        case PR_SEL: v0 = a0.val == b0.val ? a0.val : VTOP; break;
        case PR_AND64: case PR_OR64: case PR_XOR64: case PR_ANDN264:
            if (is_c(a0.val) && is_c(a1.val) && is_c(b0.val) && is_c(b1.val)) {
                const uint32_t pr = e_prule(e);
                const uint32_t x0 = v_c(a0.val), x1 = v_c(a1.val), y0 = v_c(b0.val), y1 = v_c(b1.val);
                if (pr == PR_AND64) { v0 = C32(x0 & y0); v1 = C32(x1 & y1); }
                else if (pr == PR_OR64) { v0 = C32(x0 | y0); v1 = C32(x1 | y1); }
                else if (pr == PR_XOR64) { v0 = C32(x0 ^ y0); v1 = C32(x1 ^ y1); }
                else { v0 = C32(x0 & ~y0); v1 = C32(x1 & ~y1); }
            }
            break;
        case PR_SHL64: {
            const uint64_t amt = a0.val, lo = b0.val, hi = b1.val;
            if (!is_c(amt) || lo == VTOP || hi == VTOP) break;
            const uint32_t s = v_c(amt) & 63u;
            if (is_c(lo) && is_c(hi)) {
                const uint64_t x = (((uint64_t)v_c(hi) << 32) | v_c(lo)) << s;
                v0 = C32((uint32_t)x);
                v1 = C32((uint32_t)(x >> 32));
            } else if (idx_lo(lo) && ((is_c(hi) && v_c(hi) == 0) ||
                                      (v_tag(hi) == T_IDX && v_ig(hi) == IG_HI && v_dim(hi) == v_dim(lo) &&
                                       v_aux(hi) == v_aux(lo)))) {
                if (s == 0) { v0 = lo; v1 = hi; }
                else if (s <= 15) {
                    v0 = pv(T_SHL, IG_LO, v_dim(lo), v_aux(lo), s, 0, v_c(lo) << s);
                    v1 = pv(T_SHL, IG_HI, v_dim(lo), v_aux(lo), s, 0, 0);
                }
            }
            break;
        }
        default: break;
        }
        const uint32_t prov = rp | (e_maskdef(e) ? 1u << PB_MASK : 0u);
        D.v[0] = v0;
        D.v[1] = v1;
        lds_put(st, r0, prov, ty0, v0);
        if (w0 == 2) lds_put(st, r0 + 1, prov, ty1, v1);
        D.n = w0;
    }
    const uint32_t idf = e_idef(e);
    D.imp = idf;
    const uint32_t ip = rp | (1u << PB_MASK);
    if (idf & IM_VCC) { lds_put(st, 104, ip, 0, VTOP); lds_put(st, 105, ip, 0, VTOP); }
    if (idf & IM_EXEC) { lds_put(st, 106, ip, 0, VTOP); lds_put(st, 107, ip, 0, VTOP); }
    if (idf & IM_SCC) lds_put(st, 108, ip, 0, VTOP);
    return D;
}

__device__ __forceinline__ bool implicit_covers(uint32_t imp, uint32_t slot) {
    return ((imp & IM_VCC) && (slot == 104u || slot == 105u)) || ((imp & IM_EXEC) && (slot == 106u || slot == 107u)) ||
           ((imp & IM_SCC) && slot == 108u);
}

/* recognised work-item built-ins; returns kind or -1 */
__device__ __forceinline__ int builtin_kind(uint64_t v, uint32_t &dim) {
    if (v == VTOP) return -1;
    const uint32_t t = v_tag(v), ig = v_ig(v), m = v_aux(v);
    dim = v_dim(v);
    if (t == T_IDX && v_c(v) == 0) {
        if (ig == IG_ENT && m == (M_WG | M_LID | M_GOFF)) return DC_SV_GLOBAL_ID;
        if (ig == IG_ENT && m == (M_WG | M_LID)) return DC_SV_GLOBAL_ID_MINUS_OFFSET;
        if (ig == IG_LO && m == M_GOFF) return DC_SV_GLOBAL_OFFSET;
        if (ig == IG_ENT && m == M_WG) return DC_SV_GROUP_BASE;
        if (ig == IG_ENT && m == M_LID) return DC_SV_LOCAL_ID;
        return -1;
    }
    if (t == T_SYS && ig == IG_ENT) {
        if (m == K_GSIZE) return DC_SV_GLOBAL_SIZE;
        if (m == K_NUMGROUPS) return DC_SV_NUM_GROUPS;
        if (m == K_WORKDIM) { dim = 0; return DC_SV_WORK_DIM; }
        return -1;
    }
    if (t == T_WGID) return DC_SV_GROUP_ID;
    return -1;
}

/* access record of a memory instruction from the pre-state */
__device__ __forceinline__ bool make_access(const uint4 *st, const KCtx &K, uint32_t cls, uint32_t w0, uint32_t r0, uint32_t r1,
                            uint32_t r2, int32_t imm, uint32_t instr, dc_access_t &A) {
    A.instr = instr;
    if (cls == C_GLD || cls == C_FLD || cls == C_GST || cls == C_FST) {
        A.kind = (cls == C_GLD || cls == C_FLD) ? 0 : 1;
        A.space = (cls == C_GLD || cls == C_GST) ? 0 : 1;
        A.width = (uint8_t)(4 * w0);
        uint64_t addr = VTOP;
        if (r2 == 0xFFFFu) {
            const uint64_t lo = lds_get(st, r1).val, hi = lds_get(st, r1 + 1).val;
            if (lo != VTOP && hi != VTOP && v_ig(lo) == IG_LO && v_ig(hi) == IG_HI && v_arg(lo) == v_arg(hi)) {
                if (v_tag(lo) == T_PTR && v_tag(hi) == T_PTR)
                    addr = pv(T_PTR, IG_ENT, v_dim(lo), v_aux(lo), v_sh(lo), v_arg(lo), v_c(lo) + (uint32_t)imm);
                else if (v_tag(lo) == T_KARG && v_tag(hi) == T_KARG)
                    addr = pv(T_PTR, IG_ENT, 0, 0, 0, v_arg(lo), (uint32_t)imm);
            }
        }
        A.addr = addr;
    } else if (cls == C_DSR || cls == C_DSW) {
        A.kind = cls == C_DSR ? 0 : 1;
        A.space = 2;
        A.width = 4;
        const uint64_t v = lds_get(st, r1).val;
        uint64_t addr = VTOP;
        if (v != VTOP) {
            const uint32_t c = v_c(v) + (uint32_t)imm;
            if (v_tag(v) == T_SHL && v_ig(v) == IG_ENT) addr = pv(T_SHL, IG_ENT, v_dim(v), v_aux(v), v_sh(v), 0, c);
            else if (idx_lo(v)) addr = pv(T_IDX, IG_ENT, v_dim(v), v_aux(v), 0, 0, c);
            else if (is_c(v)) addr = C32(c);
        }
        A.addr = addr;
    } else {
        return false;
    }
    uint32_t dt = 0;
    if (A.kind == 1) {
        for (uint32_t j = 0; j < w0; j++) dt |= lds_get(st, r0 + j).type;
    } else if (A.addr != VTOP && v_tag(A.addr) == T_PTR && v_arg(A.addr) < K.n_args) {
        dt = K.args[v_arg(A.addr)].flags & 31u;
    }
    A.dtype = (uint8_t)dt;
    return true;
}

/* entry state for slot j (ABI initialisation) */
__device__ __forceinline__ uint4 entry_slot(uint32_t j, uint32_t dims) {
    uint32_t prov = 1u << PB_UNINIT, type = 0;
    uint64_t val = pv(T_UNINIT, 0, 0, 0, 0, 0, 0);
    if (j == 4u || j == 5u) {
        prov = 1u << PB_SYSPTR;
        val = pv(T_SYSPTR, j == 4u ? IG_LO : IG_HI, 0, 0, 0, 0, 0);
    } else if (j >= 6u && j < 6u + dims) {
        prov = 1u << (PB_WGID + (j - 6u));
        type = TY_U;
        val = pv(T_WGID, IG_ENT, j - 6u, 0, 0, 0, 0);
    } else if (j >= 112u && j < 112u + dims) {
        prov = 1u << (PB_LID + (j - 112u));
        type = TY_U;
        val = pv(T_IDX, IG_ENT, j - 112u, M_LID, 0, 0, 0);
    } else if (j == 106u || j == 107u) {
        prov = 1u << PB_MASK;
        val = VTOP;
    }
    return make_uint4(prov, type, (uint32_t)val, (uint32_t)(val >> 32));
}

/* bitmap helpers: bits live in LDS (main pass) or global memory (overflow) */
__device__ __forceinline__ bool bit_get(const uint32_t *bm, uint32_t i) { return (bm[i >> 5] >> (i & 31)) & 1u; }
/* read-modify-write of one bitmap word; lanes other than 0 write the same
 * value into their own word of the 64-word scratch `tail` */
__device__ __forceinline__ void bit_set(uint32_t *bm, uint32_t i, uint32_t *tail) {
    const uint32_t l = lane_id();
    const uint32_t w = bm[i >> 5] | (1u << (i & 31));
    *(l == 0 ? &bm[i >> 5] : &tail[l]) = w;
}
__device__ __forceinline__ void bit_clr(uint32_t *bm, uint32_t i, uint32_t *tail) {
    const uint32_t l = lane_id();
    const uint32_t w = bm[i >> 5] & ~(1u << (i & 31));
    *(l == 0 ? &bm[i >> 5] : &tail[l]) = w;
}
/* first set bit >= from among [0, n); n if none */
__device__ __forceinline__ uint32_t next_set(const uint32_t *bm, uint32_t from, uint32_t n) {
    const uint32_t l = lane_id();
    for (uint32_t w0 = from >> 5; (w0 << 5) < n; w0 += 64) {
        const uint32_t wi = w0 + l;
        uint32_t x = (wi << 5) < n ? bm[wi] : 0u;
        if (wi == (from >> 5)) x &= ~0u << (from & 31);
        const uint64_t m = ballot(x != 0);
        if (m) {
            const uint32_t fl = (uint32_t)__builtin_ctzll(m);
            const uint32_t word = rdl(x, fl);
            return ((w0 + fl) << 5) + (uint32_t)__builtin_ctz(word);
        }
    }
    return n;
}


/* transfer of one block, or (emit) the extraction walk over it */
__device__ __forceinline__ void run_block(const Plan *__restrict__ P, uint4 *st, const KCtx &K, uint64_t rb, uint32_t pos0, uint32_t g_lo,
                          uint32_t g_hi, bool emit, uint32_t &na, uint32_t &ns) {
    const uint32_t l = lane_id();
    const uint4 *recs = reinterpret_cast<const uint4 *>(P->instrs);
    for (uint32_t g0 = g_lo; g0 < g_hi; g0 += 64) {
        const uint32_t cnt = min(64u, g_hi - g0);
        uint4 r = make_uint4(0, 0, 0, 0);
        uint64_t e = 0;
        if (l < cnt) {
            r = recs[rb + (g0 + l - pos0)];
            e = OPTAB[r.x & 0xFFFFu];
        }
        const uint32_t elo = (uint32_t)e, ehi = (uint32_t)(e >> 32);
        for (uint32_t i = 0; i < cnt; i++) {
            const uint32_t x0 = rdl(r.x, i), x1 = rdl(r.y, i);
            const int32_t imm = (int32_t)rdl(r.z, i);
            const uint64_t ei = ((uint64_t)rdl(ehi, i) << 32) | rdl(elo, i);
            const uint32_t op = x0 & 0xFFFFu, r0 = x0 >> 16, r1 = x1 & 0xFFFFu, r2 = x1 >> 16;
            const uint32_t instr = g0 + i - pos0;
            if (emit) {
                dc_access_t A;
                if (make_access(st, K, e_cls(ei), e_width(ei, 0), r0, r1, r2, imm, instr, A)) {
                    P->acc_sparse[pos0 + na] = A;   /* every lane, same record */
                    na++;
                }
            }
            const Defs D = apply(st, K, op, r0, r1, r2, imm, ei);
            if (emit) {
#pragma unroll
                for (uint32_t j = 0; j < 4; j++) {
                    const uint32_t slot = D.slot0 + j;
                    if (j >= D.n || implicit_covers(D.imp, slot)) continue;
                    uint32_t dim;
                    const int kind = builtin_kind(D.v[j], dim);
                    if (kind >= 0) {
                        dc_sysval_t S;
                        S.instr = instr;
                        S.slot = (uint16_t)slot;
                        S.kind = (uint8_t)kind;
                        S.dim = (uint8_t)dim;
                        P->sys_sparse[4ull * pos0 + ns] = S;   /* every lane, same record */
                        ns++;
                    }
                }
            }
        }
    }
}

__device__ __forceinline__ void analyze_kernel(const Plan *__restrict__ P, uint32_t k, uint4 *st, uint32_t *reached, uint32_t *dirty,
                               uint32_t *tail, uint4 *arena, uint32_t cap_blocks, bool overflow) {
    const uint32_t l = lane_id();
    const dc_kernel_t *D = &P->kernels[k];
    int32_t status = P->status[k];
    const uint32_t nb = P->n_blocks[k], fb = P->first_block[k], nr = P->n_reach[k], pos0 = P->pos_begin[k];
    dc_kernel_result_t res = {status, 0, 0, 0, 0, 0, 0};
    if (status != ST_OK) {
        P->results[k] = res;
        return;
    }
    if (nb > cap_blocks) {
        if (!overflow) {
            const uint32_t slot = rfl(atomicAdd(&P->counters[1], l == 0 ? 1u : 0u));
            P->ovf_list[slot] = k;
        } else {
            res.status = DC_E_UNSUPPORTED;
            P->results[k] = res;
        }
        return;
    }
    KCtx K;
    K.cws0 = D->cws[0];
    K.cws1 = D->cws[1];
    K.cws2 = D->cws[2];
    K.n_args = D->n_args;
    K.args = P->args + D->arg_begin;
    const uint64_t rb = D->instr_begin;
    const uint32_t dims = D->dims;
    const uint32_t words = (nb + 31) >> 5;
    for (uint32_t i = l; i < words; i += 64) {
        reached[i] = 0;
        dirty[i] = 0;
    }
    /* IN[0] = entry state */
    _Pragma("unroll 2") for (uint32_t j = l; j < (uint32_t)NSLOT; j += 64) arena[j] = entry_slot(j, dims);
    bit_set(reached, 0, tail);
    bit_set(dirty, 0, tail);   /* block 0 is first in reverse postorder */
    const uint32_t sweep_cap = P->sweep_cap ? P->sweep_cap : 64u + 2u * nb;
    uint32_t sweeps = 0, pos = nr, na = 0, ns = 0;
    for (;;) {
        uint32_t p = next_set(dirty, pos, nr);
        if (p >= nr) {
            p = next_set(dirty, 0, nr);
            if (p >= nr) break;
            if (++sweeps > sweep_cap) {
                status = DC_E_NOFIX;
                break;
            }
        }
        bit_clr(dirty, p, tail);
        pos = p + 1;
        const uint32_t b = P->rpo[fb + p];
        const uint4 *in = arena + (uint64_t)b * NSLOT;
        _Pragma("unroll 2") for (uint32_t j = l; j < (uint32_t)NSLOT; j += 64) st[j] = in[j];
        run_block(P, st, K, rb, pos0, P->block_start[fb + b], P->block_start[fb + b + 1], false, na, ns);
        for (int ed = 0; ed < 2; ed++) {
            const int32_t s = P->succ[2 * (uint64_t)(fb + b) + ed];
            if (s < 0) continue;
            uint4 *dst = arena + (uint64_t)s * NSLOT;
            bool changed;
            if (!bit_get(reached, (uint32_t)s)) {
                _Pragma("unroll 2") for (uint32_t j = l; j < (uint32_t)NSLOT; j += 64) dst[j] = st[j];
                bit_set(reached, (uint32_t)s, tail);
                changed = true;
            } else {
                bool ch = false;
                _Pragma("unroll 2") for (uint32_t j = l; j < (uint32_t)NSLOT; j += 64) {
                    const uint4 a = dst[j], o = st[j];
                    uint4 n;
                    n.x = a.x | o.x;
                    n.y = a.y | o.y;
                    const bool same = a.z == o.z && a.w == o.w;
                    n.z = same ? a.z : 0xFFFFFFFFu;
                    n.w = same ? a.w : 0xFFFFFFFFu;
                    if (n.x != a.x || n.y != a.y || n.z != a.z || n.w != a.w) {
                        dst[j] = n;
                        ch = true;
                    }
                }
                changed = ballot(ch) != 0;
            }
            if (changed) bit_set(dirty, (uint32_t)P->rpo_pos[fb + (uint32_t)s], tail);
        }
    }
    if (status == ST_OK) {
        uint64_t dig = 0;
        for (uint32_t b = 0; b < nb; b++) {
            const bool rb_ = bit_get(reached, b);
            const uint4 *in = arena + (uint64_t)b * NSLOT;
            if (P->flags & DC_OPT_EXPORT_STATES) {
                uint4 *ex = reinterpret_cast<uint4 *>(P->export_states) + (uint64_t)(fb + b) * NSLOT;
                _Pragma("unroll 2") for (uint32_t j = l; j < (uint32_t)NSLOT; j += 64) ex[j] = rb_ ? in[j] : make_uint4(0, 0, 0, 0);
                P->export_reached[fb + b] = rb_ ? 1 : 0;
            }
            if (!rb_) continue;
            if (P->flags & DC_OPT_DIGEST) {
                uint64_t h = 0;
                _Pragma("unroll 2") for (uint32_t j = l; j < (uint32_t)NSLOT; j += 64) {
                    const uint4 x = in[j];
                    const uint64_t val = ((uint64_t)x.w << 32) | x.z;
                    const uint64_t z = mix64(val + 0x9E3779B97F4A7C15ull * ((uint64_t)b * NSLOT + j + 1));
                    h += mix64(z ^ ((uint64_t)x.x | ((uint64_t)(x.y & 0xFFu) << 32)));
                }
                for (int d = 32; d >= 1; d >>= 1) {
                    const uint32_t lo = (uint32_t)h, hi = (uint32_t)(h >> 32);
                    h += ((uint64_t)__shfl_xor(hi, d, 64) << 32) | __shfl_xor(lo, d, 64);
                }
                dig += h + mix64(0xB10C0000ull + b);
            }
            _Pragma("unroll 2") for (uint32_t j = l; j < (uint32_t)NSLOT; j += 64) st[j] = in[j];
            run_block(P, st, K, rb, pos0, P->block_start[fb + b], P->block_start[fb + b + 1], true, na, ns);
        }
        res.n_blocks = nb;
        res.sweeps = sweeps;
        res.n_access = na;
        res.n_sysval = ns;
        res.digest = dig;
    } else {
        res.status = status;
        if (P->flags & DC_OPT_EXPORT_STATES) {
            for (uint32_t b = 0; b < nb; b++) {
                uint4 *ex = reinterpret_cast<uint4 *>(P->export_states) + (uint64_t)(fb + b) * NSLOT;
                _Pragma("unroll 2") for (uint32_t j = l; j < (uint32_t)NSLOT; j += 64) ex[j] = make_uint4(0, 0, 0, 0);
                P->export_reached[fb + b] = 0;
            }
        }
    }
    P->results[k] = res;
}

constexpr uint32_t MAIN_BM_WORDS = 64;   /* LDS bitmaps: up to 2048 blocks in the main pass */

/* LDS per wavefront: NSLOT + 64 state slots (working state, scratch tail);
 * main pass also: reached bitmap, dirty bitmap, 64-word scratch tail */
constexpr uint32_t ST_SLOTS = NSLOT + 64;
constexpr uint32_t BM_WORDS_PER_WAVE = 2 * MAIN_BM_WORDS + 64;

template <bool OVF>
__global__ __launch_bounds__(256) void k_fixpoint(const Plan *__restrict__ P, uint32_t wpg) {
    extern __shared__ uint4 smem[];
    const uint32_t w = rfl(threadIdx.x >> 6), l = lane_id();
    uint4 *st = smem + (uint64_t)w * ST_SLOTS;
    const uint32_t gw = blockIdx.x * wpg + w;
    uint32_t *reached, *dirty, *tail;
    uint4 *arena;
    uint32_t cap;
    if (!OVF) {
        uint32_t *bm = reinterpret_cast<uint32_t *>(smem + (uint64_t)wpg * ST_SLOTS) + w * BM_WORDS_PER_WAVE;
        reached = bm;
        dirty = bm + MAIN_BM_WORDS;
        tail = bm + 2 * MAIN_BM_WORDS;
        cap = P->block_cap;
        arena = P->arena + (uint64_t)gw * cap * NSLOT;
    } else {
        const uint32_t words = (P->ovf_block_cap + 31) >> 5;
        reached = P->ovf_bitmaps + (uint64_t)gw * (2 * words + 64);
        dirty = reached + words;
        tail = reached + 2 * words;
        cap = P->ovf_block_cap;
        arena = P->ovf_arena + (uint64_t)gw * cap * NSLOT;
    }
    for (;;) {
        /* branch-free: every lane takes part, only lane 0 adds 1 */
        const uint32_t idx = rfl(atomicAdd(&P->counters[OVF ? 2 : 0], l == 0 ? 1u : 0u));
        const uint32_t limit = OVF ? P->counters[1] : P->n_kernels;
        if (idx >= limit) break;
        const uint32_t k = OVF ? P->ovf_list[idx] : idx;
        analyze_kernel(P, k, st, reached, dirty, tail, arena, cap, OVF);
    }
}

hipError_t launch_fixpoint(const Plan &P, const Plan *dP, const FixCfg &c, hipStream_t s, hipEvent_t before,
                           hipEvent_t after) {
    hipError_t e = launch_fill_u32(P.counters, 4, 0u, s);
    if (e != hipSuccess) return e;
    if (before && (e = hipEventRecord(before, s)) != hipSuccess) return e;
    if (P.n_kernels == 0) return after ? hipEventRecord(after, s) : hipSuccess;
    const uint32_t wpg = (uint32_t)c.waves_per_group;
    const size_t lds = (size_t)wpg * ST_SLOTS * sizeof(uint4) + (size_t)wpg * BM_WORDS_PER_WAVE * sizeof(uint32_t);
    hipLaunchKernelGGL(k_fixpoint<false>, dim3(c.groups), dim3(64 * wpg), lds, s, dP, wpg);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (after && (e = hipEventRecord(after, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_fixpoint<true>, dim3(P.ovf_waves), dim3(64), (size_t)ST_SLOTS * sizeof(uint4), s, dP, 1u);
    return hipGetLastError();
}

/* ------------------------------------------------------------------ */
/* dense outputs                                                         */
/* ------------------------------------------------------------------ */
__global__ void k_counts(Plan P) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k > P.n_kernels) return;
    P.acc_count[k] = k < P.n_kernels ? P.results[k].n_access : 0u;
    P.sys_count[k] = k < P.n_kernels ? P.results[k].n_sysval : 0u;
}
/* one wavefront per kernel copies its records */
__global__ void k_compact(Plan P) {
    const uint32_t k = (blockIdx.x * blockDim.x + threadIdx.x) >> 6, l = lane_id();
    if (k >= P.n_kernels) return;
    const uint32_t pos0 = P.pos_begin[k];
    const uint32_t na = P.acc_count[k + 1] - P.acc_count[k], ns = P.sys_count[k + 1] - P.sys_count[k];
    for (uint32_t i = l; i < na; i += 64) P.acc_dense[P.acc_count[k] + i] = P.acc_sparse[pos0 + i];
    for (uint32_t i = l; i < ns; i += 64) P.sys_dense[P.sys_count[k] + i] = P.sys_sparse[4ull * pos0 + i];
}
hipError_t launch_compact(const Plan &P, hipStream_t s) {
    const uint32_t K = P.n_kernels;
    hipLaunchKernelGGL(k_counts, dim3((K + 1 + 255) / 256), dim3(256), 0, s, P);
    hipError_t e = scan_excl<uint32_t>(P.acc_count, (uint64_t)K + 1, P.acc_count, nullptr, P.scan_tmp, s);
    if (e != hipSuccess) return e;
    e = scan_excl<uint32_t>(P.sys_count, (uint64_t)K + 1, P.sys_count, nullptr, P.scan_tmp, s);
    if (e != hipSuccess) return e;
    if (K) hipLaunchKernelGGL(k_compact, dim3((K + 3) / 4), dim3(256), 0, s, P);
    return hipGetLastError();
}

}  // namespace dc
