/*
 * dc_kernels.hip -- HIP kernels for gfx950 (CDNA4) of the register-state
 * dataflow analysis.
 *
 * Stages (all integer work; no MFMA):
 *   decode   k_decode     one thread per instruction: coalesced 16-byte
 *                         record loads, opcode-table lookup, record checks,
 *                         leader flags (textbook basic-block leaders), record
 *                         capacities (access and built-in records the
 *                         instruction can emit)
 *   number   k_scan_*     reduce-then-scan of the leader flags over the whole
 *                         batch: global block ids, block_start
 *            k_cap_*      scan of the capacities: each block's record region
 *   graph    k_kernel_info, k_edges, k_pred_*, k_order
 *                         successors, predecessor CSR (count, scan, scatter,
 *                         sort), reverse postorder, per-kernel status
 *   fixpoint k_fixpoint   in dc_fixpoint.hip
 *   out      k_finish, k_compact
 *                         scans of the per-block record counts, per-kernel
 *                         totals, dense output records in instruction order
 *
 * Block-indexed arrays hold P.blk_cap blocks (the count the batch was planned
 * for); every kernel bounds its block indices by it, and a batch whose
 * records have more blocks or record capacity than planned fails every kernel
 * with DC_E_CAPACITY instead of writing past an array.
 */
#include "dc_device.h"
#include "dc_records.h"

namespace dc {

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
constexpr int TILE_LK = 4096;          /* positions per lookup tile (one workgroup of 256 threads) */
constexpr int LK_CAP = 1026;           /* kernel starts cached in LDS (more: searched in global memory) */
constexpr int LK_PER = 4;              /* positions a thread handles together (256 apart) */
constexpr int LK_ROUNDS = TILE_LK / (256 * LK_PER);

/* last k in [lo, hi] with pos_begin[k] <= g (global memory) */
__device__ uint32_t kernel_of_global(const uint32_t *pos_begin, uint32_t lo, uint32_t hi, uint32_t g) {
    while (lo < hi) {
        uint32_t mid = lo + (hi - lo + 1) / 2;
        if (pos_begin[mid] <= g) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

/* last k in [lo, hi] with pos_begin[k] <= g, given pos_begin[lo] <= g: steps
 * of doubling length from lo, then a binary search in the last one (few
 * loads when the answer is near lo) */
__device__ uint32_t kernel_of_gallop(const uint32_t *pos_begin, uint32_t lo, uint32_t hi, uint32_t g) {
    uint32_t step = 1;
    while (lo < hi) {
        const uint32_t nx = hi - lo < step ? hi : lo + step;
        if (pos_begin[nx] <= g) {
            lo = nx;
            step <<= 1;
        } else {
            hi = nx - 1;
            break;
        }
    }
    return kernel_of_global(pos_begin, lo, hi, g);
}

/* Cooperative setup for a tile [t0, t1): caches the starts of the kernels
 * that overlap it.  Returns k0 and the count (0 if they do not fit). */
__device__ void lookup_setup(const uint32_t *pos_begin, uint32_t K, uint32_t t0, uint32_t t1, uint32_t *lk,
                             uint32_t *k0_out, uint32_t *cnt_out) {
    __shared__ uint32_t s_k0, s_k1;
    if (threadIdx.x == 0) {
        s_k0 = kernel_of_global(pos_begin, 0, K - 1, t0);
        s_k1 = kernel_of_gallop(pos_begin, s_k0, K - 1, t1 - 1);
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
/* decode, check, leader flags                                          */
/* ------------------------------------------------------------------ */
constexpr uint32_t KM_KERNELS = 128;   /* kernels of a tile whose slot bitmaps are gathered in LDS */

__global__ __launch_bounds__(256) void k_decode(Plan P) {
    __shared__ uint32_t lk[LK_CAP];
    __shared__ uint32_t km[KM_KERNELS * KSLOT_WORDS];
    const uint32_t t0 = blockIdx.x * TILE_LK;
    if (t0 >= P.n_pos) return;
    const uint32_t t1 = min(P.n_pos, t0 + TILE_LK);
    uint32_t k0, cnt;
    lookup_setup(P.pos_begin, P.n_kernels, t0, t1, lk, &k0, &cnt);
    for (uint32_t i = threadIdx.x; i < KM_KERNELS * KSLOT_WORDS; i += blockDim.x) km[i] = 0;
    __syncthreads();
    /* slot bitmaps gathered in LDS when the tile's kernels all have a copy
     * there, else ORed straight into global memory */
    const bool lds_marks = cnt != 0 && cnt <= KM_KERNELS;
    /* a thread's positions in rounds of LK_PER (256 apart): their kernels,
     * then the kernels' ranges, then the records, each step's loads issued
     * together */
    for (int q = 0; q < LK_ROUNDS; q++) {
        const uint32_t tr = t0 + 256u * LK_PER * q;
        uint32_t kk[LK_PER], pbk[LK_PER], nkr[LK_PER];
        uint64_t ibk[LK_PER];
        uint4 rr[LK_PER];
#pragma unroll
        for (int j = 0; j < LK_PER; j++) {
            const uint32_t g = tr + threadIdx.x + 256u * j;
            kk[j] = g < t1 ? lookup(P.pos_begin, P.n_kernels, lk, k0, cnt, g) : k0;
        }
#pragma unroll
        for (int j = 0; j < LK_PER; j++) {
            pbk[j] = P.pos_begin[kk[j]];
            nkr[j] = P.pos_begin[kk[j] + 1] - pbk[j];
            ibk[j] = P.kernels[kk[j]].instr_begin;
        }
#pragma unroll
        for (int j = 0; j < LK_PER; j++) {
            const uint32_t g = tr + threadIdx.x + 256u * j, i = g - pbk[j];
            rr[j] = g < t1 && i < nkr[j] ? reinterpret_cast<const uint4 *>(P.instrs)[ibk[j] + i] : make_uint4(0, 0, 0, 0);
        }
#pragma unroll
        for (int j = 0; j < LK_PER; j++) {
            const uint32_t g = tr + threadIdx.x + 256u * j;
            if (g >= t1) continue;
            const uint32_t k = kk[j], pb = pbk[j], n = nkr[j];
            const uint32_t i = g - pb;
            if (i >= n) {   /* a position no kernel owns (a call whose descriptors failed their checks) */
                P.pcap[g] = 0;
                continue;
            }
            const uint4 r = rr[j];
            const uint32_t op = r.x & 0xFFFFu, r0 = r.x >> 16, r1 = r.y & 0xFFFFu, r2 = r.y >> 16;
            const int32_t imm = (int32_t)r.z, target = (int32_t)r.w;
            const uint32_t bad = check_record(op, r0, r1, r2, imm, target, n);
            if (i == 0) P.leader[g] = 1;
            if (bad) {
                P.pcap[g] = 0;
                atomicMin(&P.kbad[k], (i << 2) | bad);
                continue;
            }
            const uint64_t e = OPTAB[op];
            const uint32_t cls = e_cls(e);
            P.pcap[g] = (uint8_t)rec_cap(e);
            if (ends_block(cls) && i + 1 < n) P.leader[g + 1] = 1;
            if (cls == C_BR || cls == C_CBR) P.leader[pb + (uint32_t)target] = 1;
            if (!P.kslots) continue;
            /* the register slots the record names: each operand covers a run of
             * at most four slots, in one or two bitmap words (masks computed with
             * selects; an operand that names no slot gives empty masks) */
            const uint32_t id[4] = {r0, r1, r2, (uint32_t)imm};
#pragma unroll
            for (int o = 0; o < 4; o++) {
                const uint32_t w = e_role(e, o) != RO_NO ? e_width(e, o) : 0u;
                const bool named = (w != 0) & (id[o] < (uint32_t)NSLOT);
                const uint32_t first = named ? id[o] : 0u, last = named ? min(id[o] + w, (uint32_t)NSLOT) - 1u : 0u;
                const uint32_t wa = first >> 5, wb = last >> 5;
                const uint32_t hi_a = wa == wb ? (last & 31u) : 31u;
                const uint32_t ma = named ? (0xFFFFFFFFu >> (31u - hi_a)) & (0xFFFFFFFFu << (first & 31u)) : 0u;
                const uint32_t mb = named && wb != wa ? 0xFFFFFFFFu >> (31u - (last & 31u)) : 0u;
                if (lds_marks) {   /* wave-uniform */
                    uint32_t *km_k = km + (k - k0) * KSLOT_WORDS;
                    if (ma) atomicOr(&km_k[wa], ma);
                    if (mb) atomicOr(&km_k[wb], mb);
                } else {
                    uint32_t *ks_k = P.kslots + (uint64_t)k * KSLOT_WORDS;
                    if (ma) atomicOr(&ks_k[wa], ma);
                    if (mb) atomicOr(&ks_k[wb], mb);
                }
            }
        }
    }
    if (!P.kslots || !cnt) return;
    __syncthreads();
    const uint32_t nk = min(cnt, KM_KERNELS);
    for (uint32_t t = threadIdx.x; t < nk * KSLOT_WORDS; t += blockDim.x)
        if (km[t]) atomicOr(&P.kslots[(uint64_t)(k0 + t / KSLOT_WORDS) * KSLOT_WORDS + t % KSLOT_WORDS], km[t]);
}
hipError_t launch_decode(const Plan &P, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, P.totals, (uint64_t)4, 0u);
    if (P.kslots && P.n_kernels) {
        const hipError_t e = launch_fill_u32(P.kslots, (uint64_t)P.n_kernels * KSLOT_WORDS, 0u, s);
        if (e != hipSuccess) return e;
    }
    if (!P.n_pos) return hipGetLastError();
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

/* effective length: n, or *n_dev when given (device-side count <= n) */
__device__ __forceinline__ uint64_t eff_n(uint64_t n, const uint32_t *n_dev) {
    return n_dev ? min(n, (uint64_t)*n_dev) : n;
}

/* a thread's SCAN_ITEMS consecutive items; a full tile of a 16-byte aligned
 * array is read with 16-byte loads (one per 16 bytes of items) */
template <typename T>
__device__ __forceinline__ void load_items(const T *in, uint64_t n, uint64_t base, uint32_t v[SCAN_ITEMS]) {
    const uint64_t s = base + (uint64_t)threadIdx.x * SCAN_ITEMS;
    const bool vec = base + SCAN_TILE <= n && (reinterpret_cast<uintptr_t>(in) & 15u) == 0;   /* uniform */
    if (vec) {
        constexpr int PER = 16 / (int)sizeof(T);   /* items per 16-byte load */
        const uint4 *q = reinterpret_cast<const uint4 *>(in + s);
#pragma unroll
        for (int c = 0; c < SCAN_ITEMS / PER; c++) {
            const uint4 x = q[c];
            const uint32_t wds[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
            for (int j = 0; j < PER; j++) {
                const uint32_t wd = wds[j * (int)sizeof(T) / 4];
                v[c * PER + j] = sizeof(T) == 4 ? wd : (wd >> (8 * ((j * (int)sizeof(T)) & 3))) & ((1u << (8 * sizeof(T))) - 1u);
            }
        }
        return;
    }
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; j++) v[j] = (s + j < n) ? (uint32_t)in[s + j] : 0u;
}

template <typename T>
__global__ __launch_bounds__(256) void k_scan_reduce(const T *in, uint64_t n, const uint32_t *n_dev,
                                                      uint32_t *tile_sums) {
    n = eff_n(n, n_dev);
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
__global__ __launch_bounds__(256) void k_scan_apply(const T *in, uint64_t n, const uint32_t *n_dev,
                                                     const uint32_t *tile_offs, uint32_t *out, uint32_t *total_out) {
    n = eff_n(n, n_dev);
    uint32_t v[SCAN_ITEMS];
    const uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE;
    load_items(in, n, base, v);
    uint32_t s = 0;
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; j++) s += v[j];
    uint32_t excl;
    uint32_t tot = block_excl_scan(s, &excl);
    uint32_t run = tile_offs[blockIdx.x] + excl;
    /* the results go through LDS (17 words per thread's 16, against bank
     * conflicts) so that each store instruction writes 256 consecutive words */
    __shared__ uint32_t stage[256 * (SCAN_ITEMS + 1)];
    const uint32_t t = threadIdx.x;
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; j++) {
        stage[t * (SCAN_ITEMS + 1) + j] = run;
        run += v[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; j++) {
        const uint32_t q = (uint32_t)j * 256 + t;   /* item of the tile */
        if (base + q < n) out[base + q] = stage[(q / SCAN_ITEMS) * (SCAN_ITEMS + 1) + q % SCAN_ITEMS];
    }
    if (total_out && blockIdx.x == gridDim.x - 1 && threadIdx.x == 255) *total_out = tile_offs[blockIdx.x] + tot;
}

/* words after scan_tmp_words_needed(n) that the capacity scan of n positions
 * uses for its two tile-sum arrays */
uint64_t cap_scan_words(uint64_t n) { return 2 * ((n + SCAN_TILE - 1) / SCAN_TILE + 1) + 16; }

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

/* exclusive scan of in[0..n) into out (u32); *total_out (device) = sum.
 * With n_dev, only the first min(n, *n_dev) elements are read and written
 * (the rest count as zero). */
template <typename T>
hipError_t scan_excl(const T *in, uint64_t n, uint32_t *out, uint32_t *total_out, uint32_t *tmp, hipStream_t s,
                     const uint32_t *n_dev = nullptr) {
    if (n == 0) {
        if (total_out) hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, total_out, (uint64_t)1, 0u);
        return hipGetLastError();
    }
    uint64_t tiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (tiles == 1) {
        hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, tmp, (uint64_t)1, 0u);
        hipLaunchKernelGGL(k_scan_apply<T>, dim3(1), dim3(256), 0, s, in, n, n_dev, tmp, out, total_out);
        return hipGetLastError();
    }
    uint32_t *sums = tmp;
    hipLaunchKernelGGL(k_scan_reduce<T>, dim3((uint32_t)tiles), dim3(256), 0, s, in, n, n_dev, sums);
    hipError_t e = scan_excl<uint32_t>(sums, tiles, sums, nullptr, tmp + tiles + 1, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scan_apply<T>, dim3((uint32_t)tiles), dim3(256), 0, s, in, n, n_dev, sums, out, total_out);
    return hipGetLastError();
}

/* ------------------------------------------------------------------ */
/* block numbering                                                       */
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
    /* a thread's positions in rounds of LK_PER (256 apart), each round's
     * loads issued together (block_id may be excl itself: each position
     * reads its entry first) */
    for (int q = 0; q < LK_ROUNDS; q++) {
        const uint32_t tr = t0 + 256u * LK_PER * q;
        uint32_t lv[LK_PER], xv[LK_PER];
#pragma unroll
        for (int j = 0; j < LK_PER; j++) {
            const uint32_t g = tr + threadIdx.x + 256u * j;
            lv[j] = g < t1 ? P.leader[g] : 0u;
            xv[j] = g < t1 ? excl[g] : 0u;
        }
#pragma unroll
        for (int j = 0; j < LK_PER; j++) {
            const uint32_t g = tr + threadIdx.x + 256u * j;
            if (g >= t1) continue;
            const uint32_t l = lv[j];
            const uint32_t id = xv[j] + l - 1;
            P.block_id[g] = id;
            if (l && id < P.blk_cap) {
                P.block_start[id] = g;
                P.block_kernel[id] = lookup(P.pos_begin, P.n_kernels, lk, k0, cnt, g);
            }
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && P.totals[0] <= P.blk_cap) P.block_start[P.totals[0]] = P.n_pos;
}

/* Record regions.  Each block's access (built-in) records go to a region of
 * the sparse output as long as the access (built-in) capacity of its
 * instructions; the region starts at the exclusive prefix sum of the
 * capacities at the block's first position.  The two capacity fields of a
 * tile are summed as one word (access count in bits 15:0, built-ins in
 * 31:16: a tile of 4096 positions holds at most 4096 and 16384). */
__device__ __forceinline__ uint32_t cap_pack(uint32_t c) { return (c & 1u) | (c >> 1) << 16; }

__global__ __launch_bounds__(256) void k_cap_reduce(Plan P, uint32_t *sums_a, uint32_t *sums_s) {
    uint32_t c[SCAN_ITEMS];
    load_items<uint8_t>(P.pcap, P.n_pos, (uint64_t)blockIdx.x * SCAN_TILE, c);
    uint32_t x = 0;
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; j++) x += cap_pack(c[j]);
    uint32_t excl;
    const uint32_t tot = block_excl_scan(x, &excl);
    if (threadIdx.x == 0) {
        sums_a[blockIdx.x] = tot & 0xFFFFu;
        sums_s[blockIdx.x] = tot >> 16;
    }
}

/* offs_a/offs_s: exclusive tile offsets */
__global__ __launch_bounds__(256) void k_cap_apply(Plan P, const uint32_t *offs_a, const uint32_t *offs_s) {
    const uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE + (uint64_t)threadIdx.x * SCAN_ITEMS;
    uint32_t c[SCAN_ITEMS], ld[SCAN_ITEMS];
    load_items<uint8_t>(P.pcap, P.n_pos, (uint64_t)blockIdx.x * SCAN_TILE, c);
    load_items<uint8_t>(P.leader, P.n_pos, (uint64_t)blockIdx.x * SCAN_TILE, ld);
    uint32_t x = 0;
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; j++) {
        c[j] = cap_pack(c[j]);
        x += c[j];
    }
    uint32_t excl;
    block_excl_scan(x, &excl);
    uint32_t ra = offs_a[blockIdx.x] + (excl & 0xFFFFu), rs = offs_s[blockIdx.x] + (excl >> 16);
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; j++) {
        if (base + j < P.n_pos && ld[j]) {
            const uint32_t id = P.block_id[base + j];
            if (id < P.blk_cap) {
                P.blk_acc_base[id] = ra;
                P.blk_sys_base[id] = rs;
            }
        }
        ra += c[j] & 0xFFFFu;
        rs += c[j] >> 16;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && P.totals[0] <= P.blk_cap) {
        P.blk_acc_base[P.totals[0]] = P.totals[1];
        P.blk_sys_base[P.totals[0]] = P.totals[2];
    }
}

/* tile sums of the capacity scan, after the scan scratch */
__host__ __device__ inline uint32_t *cap_sums(const Plan &P) { return P.scan_tmp + P.scan_tmp_words; }

hipError_t launch_leader_scan(const Plan &P, hipStream_t s) {
    if (!P.n_pos) return hipSuccess;   /* the totals are zero from the decode stage */
    /* the exclusive leader counts go to block_id first; k_number rewrites
     * block_id in place (each position reads its own entry before writing) */
    hipError_t e = scan_excl<uint8_t>(P.leader, P.n_pos, P.block_id, P.totals, P.scan_tmp, s);
    if (e != hipSuccess || !P.with_records) return e;
    /* the capacity scan's tile offsets and the batch's capacity totals
     * (totals[1], totals[2]); the regions are written after numbering */
    const uint64_t ct = ((uint64_t)P.n_pos + SCAN_TILE - 1) / SCAN_TILE;
    uint32_t *sums_a = cap_sums(P), *sums_s = sums_a + ct + 1;
    hipLaunchKernelGGL(k_cap_reduce, dim3((uint32_t)ct), dim3(256), 0, s, P, sums_a, sums_s);
    e = scan_excl<uint32_t>(sums_a, ct, sums_a, P.totals + 1, P.scan_tmp, s);
    if (e == hipSuccess) e = scan_excl<uint32_t>(sums_s, ct, sums_s, P.totals + 2, P.scan_tmp, s);
    return e;
}

hipError_t launch_number_blocks(const Plan &P, hipStream_t s) {
    if (!P.n_pos) {
        if (P.blk_cap) {
            hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, P.block_start, (uint64_t)1, 0u);
            if (P.blk_acc_base) {
                hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, P.blk_acc_base, (uint64_t)1, 0u);
                hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, P.blk_sys_base, (uint64_t)1, 0u);
            }
        }
        return hipGetLastError();
    }
    const uint32_t tiles = (P.n_pos + TILE_LK - 1) / TILE_LK;
    hipLaunchKernelGGL(k_number, dim3(tiles), dim3(256), 0, s, P, P.block_id);
    if (!P.blk_acc_base) return hipGetLastError();   /* graph only: no record regions */
    /* the tile offsets left by launch_leader_scan */
    const uint64_t ct = ((uint64_t)P.n_pos + SCAN_TILE - 1) / SCAN_TILE;
    uint32_t *sums_a = cap_sums(P), *sums_s = sums_a + ct + 1;
    hipLaunchKernelGGL(k_cap_apply, dim3((uint32_t)ct), dim3(256), 0, s, P, sums_a, sums_s);
    return hipGetLastError();
}

/* ------------------------------------------------------------------ */
/* per-kernel info, edges, predecessors, reverse postorder              */
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
    uint32_t fb = 0, nb = 0;
    if (n) {
        fb = P.block_id[pb];
        nb = P.block_id[pb + n - 1] - fb + 1;
    }
    /* records changed since the batch was planned: more blocks or record
     * capacity than its arrays hold */
    const bool over = P.totals[0] > P.blk_cap ||
                      (P.acc_sparse && (P.totals[1] > P.acc_cap || P.totals[2] > P.sys_cap));
    if (over) {
        st = DC_E_CAPACITY;
        nb = 0;
    }
    P.status[k] = st;
    P.first_block[k] = fb;
    P.n_blocks[k] = nb;
}

__global__ void k_edges(Plan P) {
    const uint32_t total = min(P.totals[0], P.blk_cap);
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
    const uint32_t total = min(P.totals[0], P.blk_cap);
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
    /* predecessor lists sorted (insertion sort; most have one or two
     * entries), eight blocks' list bounds loaded together */
    for (uint32_t b0 = 0; b0 < nb; b0 += 8) {
        uint32_t pc[9];
#pragma unroll
        for (uint32_t j = 0; j < 9; j++) pc[j] = P.pred_cnt[fb + min(b0 + j, nb)];
#pragma unroll
        for (uint32_t j = 0; j < 8; j++) {
            if (b0 + j >= nb) break;
            const uint32_t lo = pc[j], hi = pc[j + 1];
            for (uint32_t i = lo + 1; i < hi; i++) {
                uint32_t x = P.pred[i], q = i;
                while (q > lo && P.pred[q - 1] > x) {
                    P.pred[q] = P.pred[q - 1];
                    q--;
                }
                P.pred[q] = x;
            }
            P.dfs_seen[fb + b0 + j] = 0;
            P.rpo_pos[fb + b0 + j] = -1;
        }
    }
    /* Explicit-stack emulation of the recursive DFS.  The top entry lives in
     * registers (block u, next out-edge e, its successor pair); an entry below
     * it is stored as u | e << 30 and its successors are loaded again when it
     * becomes the top.  The postorder fills rpo from the end, so that its
     * last np entries are the reverse postorder. */
    uint32_t *stk = P.dfs_stack + fb;
    uint32_t *rpo = P.rpo + fb;
    const int2 *succ = reinterpret_cast<const int2 *>(P.succ) + fb;
    uint32_t sp = 1, np = 0, u = 0, e = 0;
    int2 sc = succ[0];
    P.dfs_seen[fb] = 1;
    for (;;) {
        if (e < 2) {
            const int32_t x = e == 0 ? sc.x : sc.y;
            e++;
            if (x >= 0 && !P.dfs_seen[fb + (uint32_t)x]) {
                P.dfs_seen[fb + (uint32_t)x] = 1;
                stk[sp - 1] = u | (e << 30);
                sp++;
                u = (uint32_t)x;
                e = 0;
                sc = succ[u];
            }
        } else {
            rpo[nb - 1 - np] = u;
            np++;
            if (--sp == 0) break;
            const uint32_t top = stk[sp - 1];
            u = top & 0x3FFFFFFFu;
            e = top >> 30;
            if (e < 2) sc = succ[u];
        }
    }
    if (np < nb)
        for (uint32_t i = 0; i < np; i++) rpo[i] = rpo[nb - np + i];
    for (uint32_t i = 0; i < np; i++) P.rpo_pos[fb + rpo[i]] = (int32_t)i;
    P.n_reach[k] = np;
}

/* one thread per global block: the fixpoint's per-visit block record, stored
 * at the block's reverse-postorder position (local id, instruction range,
 * RPO positions of the successors, -1 when absent, and which successor, if
 * any, has this block as its only predecessor) */
__global__ void k_blockinfo(Plan P) {
    const uint32_t total = min(P.totals[0], P.blk_cap);
    for (uint32_t gb = blockIdx.x * blockDim.x + threadIdx.x; gb < total; gb += gridDim.x * blockDim.x) {
        const uint32_t k = P.block_kernel[gb];
        if (P.status[k] != ST_OK) continue;
        const int32_t p = P.rpo_pos[gb];
        if (p < 0) continue;
        const uint32_t fb = P.first_block[k];
        const int32_t s0 = P.succ[2 * (uint64_t)gb], s1 = P.succ[2 * (uint64_t)gb + 1];
        const int32_t ps0 = s0 >= 0 ? P.rpo_pos[fb + (uint32_t)s0] : -1;
        const int32_t ps1 = s1 >= 0 ? P.rpo_pos[fb + (uint32_t)s1] : -1;
        /* a successor whose only predecessor is this block continues this
         * block's visit (its IN state is this block's OUT state).  The entry
         * block never does: its IN state also holds the entry state, and a
         * jump back to it would chain forever. */
        auto single = [&](int32_t sb) {
            return sb > 0 && P.pred_cnt[fb + (uint32_t)sb + 1] - P.pred_cnt[fb + (uint32_t)sb] == 1;
        };
        const uint32_t chain = single(s0) ? 0u : (single(s1) ? 1u : 2u);
        uint4 *dst = P.binfo + 2 * ((uint64_t)fb + (uint32_t)p);
        dst[0] = make_uint4(gb - fb, P.block_start[gb], P.block_start[gb + 1], 0u);
        dst[1] = make_uint4((uint32_t)ps0, (uint32_t)ps1, chain, 0u);
    }
}

hipError_t launch_edges(const Plan &P, hipStream_t s) {
    const uint32_t K = P.n_kernels;
    if (K) hipLaunchKernelGGL(k_kernel_info, dim3((K + 255) / 256), dim3(256), 0, s, P);
    hipError_t e = launch_fill_u32(P.pred_cnt, (uint64_t)P.blk_cap + 1, 0u, s);
    if (e != hipSuccess) return e;
    e = launch_fill_u32(P.pred_fill, (uint64_t)P.blk_cap, 0u, s);
    if (e != hipSuccess) return e;
    const uint32_t grid = grid_for(P.blk_cap ? P.blk_cap : 1, 256 * 4);
    hipLaunchKernelGGL(k_edges, dim3(grid), dim3(256), 0, s, P);
    e = scan_excl<uint32_t>(P.pred_cnt, (uint64_t)P.blk_cap + 1, P.pred_cnt, nullptr, P.scan_tmp, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_pred_scatter, dim3(grid), dim3(256), 0, s, P);
    if (K) hipLaunchKernelGGL(k_order, dim3((K + 63) / 64), dim3(64), 0, s, P);
    if (P.binfo) hipLaunchKernelGGL(k_blockinfo, dim3(grid), dim3(256), 0, s, P);
    return hipGetLastError();
}


/* ------------------------------------------------------------------ */
/* dense outputs                                                         */
/* ------------------------------------------------------------------ */
/* The fixpoint leaves, per global block, the number of access and built-in
 * records of the block's last visit (zero for unreached blocks and failed
 * kernels) and the records themselves in the block's regions.  Blocks are
 * numbered in position order, so exclusive scans of the counts are the dense
 * offsets directly. */
__global__ void k_finish(Plan P) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= P.n_kernels) return;
    const uint32_t fb = P.first_block[k], nb = P.n_blocks[k];
    uint32_t na = 0, ns = 0;
    if (nb && fb + nb <= P.blk_cap) {
        const uint32_t lb = fb + nb - 1;
        na = P.blk_acc_off[lb] + P.blk_acc[lb] - P.blk_acc_off[fb];
        ns = P.blk_sys_off[lb] + P.blk_sys[lb] - P.blk_sys_off[fb];
    }
    P.results[k].n_access = na;
    P.results[k].n_sysval = ns;
    P.acc_count[k] = na;
    P.sys_count[k] = ns;
}
__global__ void k_count_tail(Plan P) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        P.acc_count[P.n_kernels] = 0;
        P.sys_count[P.n_kernels] = 0;
    }
}
/* the records of global blocks, from their regions of the sparse outputs to
 * their dense offsets: a wavefront takes 64 blocks (one per lane for the
 * counts and offsets), then copies each block's records with its 64 lanes
 * (consecutive records on consecutive lanes) */
__global__ __launch_bounds__(256) void k_compact(Plan P) {
    /* records that outgrew the plan: every kernel failed, nothing to copy
     * (the counts of the blocks are stale) */
    if (P.totals[0] > P.blk_cap || P.totals[1] > P.acc_cap || P.totals[2] > P.sys_cap) return;
    const uint32_t total = P.totals[0];
    const uint32_t l = lane_id();
    const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6, nwaves = (gridDim.x * blockDim.x) >> 6;
    const uint4 *acc_src = reinterpret_cast<const uint4 *>(P.acc_sparse);
    uint4 *acc_dst = reinterpret_cast<uint4 *>(P.acc_dense);
    const uint2 *sys_src = reinterpret_cast<const uint2 *>(P.sys_sparse);
    uint2 *sys_dst = reinterpret_cast<uint2 *>(P.sys_dense);
    for (uint32_t b0 = wave * 64; b0 < total; b0 += nwaves * 64) {   /* wave-uniform */
        const uint32_t b = b0 + l;
        uint32_t na = 0, ns = 0, sa = 0, da = 0, ss = 0, ds = 0;
        if (b < total) {
            na = P.blk_acc[b];
            ns = P.blk_sys[b];
            sa = P.blk_acc_base[b];
            da = P.blk_acc_off[b];
            ss = P.blk_sys_base[b];
            ds = P.blk_sys_off[b];
            na = sa + na <= P.acc_cap && da + na <= P.acc_cap ? na : 0u;
            ns = ss + ns <= P.sys_cap && ds + ns <= P.sys_cap ? ns : 0u;
        }
        for (uint64_t m = __ballot(na != 0); m; m &= m - 1) {
            const int j = (int)__builtin_ctzll(m);
            const uint32_t n = __shfl(na, j, 64), src = __shfl(sa, j, 64), dst = __shfl(da, j, 64);
            for (uint32_t i = l; i < n; i += 64) acc_dst[(uint64_t)dst + i] = acc_src[(uint64_t)src + i];
        }
        for (uint64_t m = __ballot(ns != 0); m; m &= m - 1) {
            const int j = (int)__builtin_ctzll(m);
            const uint32_t n = __shfl(ns, j, 64), src = __shfl(ss, j, 64), dst = __shfl(ds, j, 64);
            for (uint32_t i = l; i < n; i += 64) sys_dst[(uint64_t)dst + i] = sys_src[(uint64_t)src + i];
        }
    }
}
hipError_t launch_compact(const Plan &P, hipStream_t s) {
    const uint32_t K = P.n_kernels;
    hipError_t e = scan_excl<uint32_t>(P.blk_acc, (uint64_t)P.blk_cap, P.blk_acc_off, nullptr, P.scan_tmp, s,
                                       P.totals);
    if (e != hipSuccess) return e;
    e = scan_excl<uint32_t>(P.blk_sys, (uint64_t)P.blk_cap, P.blk_sys_off, nullptr, P.scan_tmp, s, P.totals);
    if (e != hipSuccess) return e;
    if (K) hipLaunchKernelGGL(k_finish, dim3((K + 255) / 256), dim3(256), 0, s, P);
    hipLaunchKernelGGL(k_count_tail, dim3(1), dim3(64), 0, s, P);
    e = scan_excl<uint32_t>(P.acc_count, (uint64_t)K + 1, P.acc_count, nullptr, P.scan_tmp, s);
    if (e != hipSuccess) return e;
    e = scan_excl<uint32_t>(P.sys_count, (uint64_t)K + 1, P.sys_count, nullptr, P.scan_tmp, s);
    if (e != hipSuccess) return e;
    if (P.blk_cap) hipLaunchKernelGGL(k_compact, dim3(grid_for(P.blk_cap, 256 * 2)), dim3(256), 0, s, P);
    return hipGetLastError();
}

}  // namespace dc
