/*
 * dc_noalloc.hip -- dc_analyze_noalloc: the whole analysis of a batch with
 * every intermediate array in one static device array of the library
 * (`scratch`), for callers that cannot allocate device memory.
 *
 * The array is carved at fixed offsets for the limits in dc.h
 * (DC_NOALLOC_MAX_KERNELS kernels, DC_NOALLOC_MAX_INSTR instructions): the
 * per-kernel and per-position arrays, the block-indexed arrays for one block
 * per instruction, the sparse record regions for one access and four
 * built-in records per instruction, a fixed fixpoint grid with its arenas and
 * a small overflow pass, the scan scratch and the device copy of the plan.
 * Descriptors are device memory: a one-workgroup kernel checks them and
 * numbers their positions, so nothing is copied from the host.  The results
 * go to the caller's device buffers.
 *
 * Host code never uses the array's name as an address: at set-up each device
 * resolves the symbol once (hipGetSymbolAddress, with the device current) and
 * the kernels receive pointers derived from that address.  Every call on one
 * device shares the array, so calls that overlap on one device race; each
 * call clears what must start at zero.
 */
#include <mutex>

#include "dc_device.h"
#include "dc_host.h"

namespace dc {

/* ---- layout ---- */
constexpr uint64_t NA_K = DC_NOALLOC_MAX_KERNELS;
constexpr uint64_t NA_N = DC_NOALLOC_MAX_INSTR;
constexpr uint32_t NA_WPG = 2;                  /* fixpoint waves per workgroup */
constexpr uint32_t NA_GROUPS = 32;              /* persistent main-pass workgroups */
constexpr uint64_t NA_WAVES = (uint64_t)NA_WPG * NA_GROUPS;
constexpr uint32_t NA_ROWS = 512;               /* main-pass arena rows per wave (256 blocks of two rows) */
constexpr uint32_t NA_OVF_WAVES = 4;
constexpr uint32_t NA_OVF_BLOCKS = 1024;        /* blocks of a kernel in the overflow pass */
constexpr uint32_t NA_OVF_ROWS = NA_OVF_BLOCKS * FIX_MAX_ROWS;
constexpr uint64_t NA_BM_WORDS = 2 * ((NA_OVF_BLOCKS + 31) / 32) + 64;

constexpr uint64_t al(uint64_t x) { return (x + 255) & ~255ull; }

struct Layout {
    uint64_t kernels, pos_begin, desc_status, kbad, status, first_block, n_blocks, n_reach, ovf_list, kslots;
    uint64_t leader, pcap, block_id, totals, counters;
    uint64_t block_start, block_kernel, succ, pred_cnt, pred_fill, pred, rpo, rpo_pos, dfs_stack, dfs_seen;
    uint64_t binfo, acc_base, sys_base, blk_acc, blk_sys, blk_acc_off, blk_sys_off;
    uint64_t acc_sparse, sys_sparse, arena, ovf_arena, ovf_bitmaps, dummy, scan_tmp, plan, end;
};

constexpr uint64_t SCAN_WORDS_MAX = 2 * ((NA_N + 1) / 4096 + 2) + 64;   /* >= scan_tmp_words_needed(NA_N + 1) */
constexpr uint64_t CAP_WORDS_MAX = 2 * (NA_N / 4096 + 2) + 16;        /* >= cap_scan_words(NA_N) */

constexpr Layout make_layout() {
    Layout L{};
    uint64_t o = 0;
    auto take = [&](uint64_t bytes) {
        const uint64_t at = o;
        o += al(bytes);
        return at;
    };
    L.kernels = take(NA_K * sizeof(dc_kernel_t));
    L.pos_begin = take((NA_K + 1) * 4);
    L.desc_status = take(NA_K * 4);
    L.kbad = take(NA_K * 4);
    L.status = take(NA_K * 4);
    L.first_block = take(NA_K * 4);
    L.n_blocks = take(NA_K * 4);
    L.n_reach = take(NA_K * 4);
    L.ovf_list = take(NA_K * 4);
    L.kslots = take(NA_K * KSLOT_WORDS * 4);
    L.leader = take(NA_N + 16);
    L.pcap = take(NA_N + 16);
    L.block_id = take(NA_N * 4);
    L.totals = take(16);
    L.counters = take(16);
    L.block_start = take((NA_N + 1) * 4);
    L.block_kernel = take(NA_N * 4);
    L.succ = take(NA_N * 8);
    L.pred_cnt = take((NA_N + 1) * 4);
    L.pred_fill = take(NA_N * 4);
    L.pred = take(NA_N * 8);
    L.rpo = take(NA_N * 4);
    L.rpo_pos = take(NA_N * 4);
    L.dfs_stack = take(NA_N * 4);
    L.dfs_seen = take(NA_N);
    L.binfo = take(NA_N * 32);
    L.acc_base = take((NA_N + 1) * 4);
    L.sys_base = take((NA_N + 1) * 4);
    L.blk_acc = take(NA_N * 4);
    L.blk_sys = take(NA_N * 4);
    L.blk_acc_off = take(NA_N * 4);
    L.blk_sys_off = take(NA_N * 4);
    L.acc_sparse = take(NA_N * sizeof(dc_access_t));
    L.sys_sparse = take(4 * NA_N * sizeof(dc_sysval_t));
    L.arena = take(NA_WAVES * NA_ROWS * FIX_ROW_DWORDS * 4);
    L.ovf_arena = take((uint64_t)NA_OVF_WAVES * NA_OVF_ROWS * FIX_ROW_DWORDS * 4);
    L.ovf_bitmaps = take(NA_OVF_WAVES * NA_BM_WORDS * 4);
    L.dummy = take((NA_WAVES + NA_OVF_WAVES) * 64 * 16);
    L.scan_tmp = take((SCAN_WORDS_MAX + CAP_WORDS_MAX) * 4);
    L.plan = take(sizeof(Plan));
    L.end = o;
    return L;
}
constexpr Layout LAYOUT = make_layout();
static_assert(LAYOUT.end <= DC_NOALLOC_SCRATCH_BYTES, "the scratch array holds the layout");

/* the scratch array; host code uses only the address resolved per device */
static __device__ __align__(256) unsigned char scratch[DC_NOALLOC_SCRATCH_BYTES];

/* ---- device set-up ---- */
static std::mutex g_mu;
static void *g_scratch[256];

/* the device address of `scratch` on the current device `dev`, resolved once
 * per device; null when the lookup fails */
void *noalloc_setup(int dev) {
    if (dev < 0 || dev >= 256) return nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
        g_scratch[dev] = p;
    }
    return g_scratch[dev];
}

/* ---- descriptor checks and positions (one workgroup of 256) ---- */
__device__ __forceinline__ int32_t desc_status_dev(const dc_kernel_t &k) {
    if (k.useargs != 1 || k.dims < 1 || k.dims > 3) return DC_E_UNSUPPORTED;
    for (int d = 0; d < k.dims; d++)
        if (k.cws[d] == 0) return DC_E_UNSUPPORTED;
    return k.n_args > 255 ? DC_E_UNSUPPORTED : DC_OK;
}

__device__ __forceinline__ uint32_t wg_excl_scan(uint32_t x, uint32_t *total) {
    __shared__ uint32_t wsum[4];
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
    for (uint32_t j = 0; j < 4; j++) {
        base += j < w ? wsum[j] : 0u;
        tot += wsum[j];
    }
    __syncthreads();
    *total = tot;
    return base + inc - x;
}

/* A descriptor whose records or arguments lie outside the arrays fails with
 * DC_E_INVAL and owns no positions.  Kernels whose positions would run past
 * max_pos fail with DC_E_CAPACITY and own none (those that fit are a prefix
 * of the list).  When the positions owned differ from the caller's
 * instruction total, every kernel fails with DC_E_INVAL and owns none. */
__global__ __launch_bounds__(256) void k_na_prep(dc_kernel_t *kout, uint32_t *pos_begin, int32_t *desc_status,
                                                 const dc_kernel_t *kin, uint32_t K, uint64_t n_records,
                                                 uint64_t n_args_total, uint32_t max_pos, uint32_t n_pos) {
    __shared__ uint32_t s_fit;
    uint32_t carry = 0, fit = 0;
    /* pass 1: the positions the fitting kernels own */
    for (uint32_t c = 0; c < K; c += 256) {
        const uint32_t k = c + threadIdx.x;
        const dc_kernel_t d = kin[k < K ? k : 0];
        const bool ok = k < K && d.instr_begin <= n_records && d.n_instr <= n_records - d.instr_begin &&
                        (desc_status_dev(d) != DC_OK || (uint64_t)d.arg_begin + d.n_args <= n_args_total);
        /* lengths above max_pos never fit; clamped, a chunk's sum stays in 32 bits */
        const uint32_t n = ok ? (d.n_instr <= max_pos ? d.n_instr : max_pos + 1) : 0u;
        uint32_t tot;
        const uint32_t ex = carry + wg_excl_scan(n, &tot);
        const bool fits = (uint64_t)ex + n <= max_pos;
        if (threadIdx.x == 0) s_fit = 0;
        __syncthreads();
        if (k < K && fits && n) atomicMax(&s_fit, ex + n);
        __syncthreads();
        fit = s_fit > fit ? s_fit : fit;
        carry = (uint64_t)carry + tot > 0xFFFFFFF0ull ? 0xFFFFFFF0u : carry + tot;
        __syncthreads();
    }
    const bool agree = fit == n_pos;
    /* pass 2: the sanitised copy, positions and descriptor statuses */
    carry = 0;
    for (uint32_t c = 0; c < K; c += 256) {
        const uint32_t k = c + threadIdx.x;
        dc_kernel_t d = kin[k < K ? k : 0];
        int32_t st = desc_status_dev(d);
        const bool ok = k < K && d.instr_begin <= n_records && d.n_instr <= n_records - d.instr_begin &&
                        (st != DC_OK || (uint64_t)d.arg_begin + d.n_args <= n_args_total);
        uint32_t n = ok ? (d.n_instr <= max_pos ? d.n_instr : max_pos + 1) : 0u;
        uint32_t tot;
        const uint32_t ex = carry + wg_excl_scan(n, &tot);
        if (!ok) st = DC_E_INVAL;
        if ((uint64_t)ex + n > max_pos) {
            st = DC_E_CAPACITY;
            n = 0;
        }
        if (!agree) {
            st = DC_E_INVAL;
            n = 0;
        }
        d.n_instr = n;
        if (k < K) {
            kout[k] = d;
            pos_begin[k] = agree ? (ex < fit ? ex : fit) : 0u;
            desc_status[k] = st;
        }
        carry = (uint64_t)carry + tot > 0xFFFFFFF0ull ? 0xFFFFFFF0u : carry + tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) pos_begin[K] = agree ? fit : 0u;
}

__global__ void k_na_store_plan(Plan P, Plan *dst) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *dst = P;
}

}  // namespace dc

using namespace dc;

extern "C" dc_status_t dc_analyze_noalloc(dc_ctx_t *ctx, const dc_kernel_t *kernels, uint32_t n_kernels,
                                          uint32_t n_instr_total, const dc_instr_t *instrs, uint64_t n_records,
                                          const dc_arg_t *args, uint64_t n_args_total, uint32_t flags,
                                          dc_kernel_result_t *results, dc_access_t *accesses, uint32_t acc_cap,
                                          uint32_t *acc_off, dc_sysval_t *sysvals, uint32_t sys_cap,
                                          uint32_t *sys_off, void *stream) {
    if (!ctx || (n_kernels && (!kernels || !results)) || !acc_off || !sys_off || (n_records && !instrs) ||
        (n_args_total && !args) || (acc_cap && !accesses) || (sys_cap && !sysvals))
        return DC_E_INVAL;
    if (n_kernels > DC_NOALLOC_MAX_KERNELS || n_instr_total > DC_NOALLOC_MAX_INSTR || (flags & ~DC_OPT_DIGEST) ||
        (n_kernels == 0 && n_instr_total != 0))
        return DC_E_INVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return DC_E_HIP;
    unsigned char *base = static_cast<unsigned char *>(noalloc_setup(ctx->device));
    if (!base) return DC_E_HIP;
    if (NA_WPG * fixpoint_lds_per_wave() > ctx->lds_per_group) return DC_E_HIP;
    hipStream_t s = (hipStream_t)stream;
    const Layout &L = LAYOUT;
    auto at = [&](uint64_t off) { return static_cast<void *>(base + off); };
    Plan P{};
    dc_kernel_t *ks = static_cast<dc_kernel_t *>(at(L.kernels));
    uint32_t *pb = static_cast<uint32_t *>(at(L.pos_begin));
    int32_t *ds = static_cast<int32_t *>(at(L.desc_status));
    P.instrs = instrs;
    P.kernels = ks;
    P.args = args;
    P.pos_begin = pb;
    P.desc_status = ds;
    P.work_order = nullptr;
    P.n_kernels = n_kernels;
    P.n_pos = n_instr_total;
    P.n_records = n_records;
    P.n_args = n_args_total;
    P.leader = static_cast<uint8_t *>(at(L.leader));
    P.pcap = static_cast<uint8_t *>(at(L.pcap));
    P.block_id = static_cast<uint32_t *>(at(L.block_id));
    P.totals = static_cast<uint32_t *>(at(L.totals));
    P.kslots = static_cast<uint32_t *>(at(L.kslots));
    P.with_records = 1;
    P.blk_cap = (uint32_t)NA_N;
    P.block_start = static_cast<uint32_t *>(at(L.block_start));
    P.block_kernel = static_cast<uint32_t *>(at(L.block_kernel));
    P.succ = static_cast<int32_t *>(at(L.succ));
    P.pred_cnt = static_cast<uint32_t *>(at(L.pred_cnt));
    P.pred_fill = static_cast<uint32_t *>(at(L.pred_fill));
    P.pred = static_cast<uint32_t *>(at(L.pred));
    P.rpo = static_cast<uint32_t *>(at(L.rpo));
    P.rpo_pos = static_cast<int32_t *>(at(L.rpo_pos));
    P.dfs_stack = static_cast<uint32_t *>(at(L.dfs_stack));
    P.dfs_seen = static_cast<uint8_t *>(at(L.dfs_seen));
    P.blk_acc_base = static_cast<uint32_t *>(at(L.acc_base));
    P.blk_sys_base = static_cast<uint32_t *>(at(L.sys_base));
    P.kbad = static_cast<uint32_t *>(at(L.kbad));
    P.status = static_cast<int32_t *>(at(L.status));
    P.first_block = static_cast<uint32_t *>(at(L.first_block));
    P.n_blocks = static_cast<uint32_t *>(at(L.n_blocks));
    P.n_reach = static_cast<uint32_t *>(at(L.n_reach));
    P.binfo = static_cast<uint4 *>(at(L.binfo));
    P.arena = static_cast<uint32_t *>(at(L.arena));
    P.arena_rows = NA_ROWS;
    P.main_waves = (uint32_t)NA_WAVES;
    P.ovf_arena = static_cast<uint32_t *>(at(L.ovf_arena));
    P.ovf_rows = NA_OVF_ROWS;
    P.ovf_bitmaps = static_cast<uint32_t *>(at(L.ovf_bitmaps));
    P.ovf_block_cap = NA_OVF_BLOCKS;
    P.ovf_waves = NA_OVF_WAVES;
    P.ovf_list = static_cast<uint32_t *>(at(L.ovf_list));
    P.dummy = static_cast<uint4 *>(at(L.dummy));
    P.counters = static_cast<uint32_t *>(at(L.counters));
    P.sweep_cap = 0;
    P.flags = flags;
    /* the dense outputs are the caller's: a region must fit both */
    P.acc_cap = acc_cap < (uint32_t)NA_N ? acc_cap : (uint32_t)NA_N;
    P.sys_cap = sys_cap < (uint32_t)(4 * NA_N) ? sys_cap : (uint32_t)(4 * NA_N);
    P.acc_sparse = static_cast<dc_access_t *>(at(L.acc_sparse));
    P.sys_sparse = static_cast<dc_sysval_t *>(at(L.sys_sparse));
    P.blk_acc = static_cast<uint32_t *>(at(L.blk_acc));
    P.blk_sys = static_cast<uint32_t *>(at(L.blk_sys));
    P.results = results;
    P.export_states = nullptr;
    P.export_reached = nullptr;
    P.blk_acc_off = static_cast<uint32_t *>(at(L.blk_acc_off));
    P.blk_sys_off = static_cast<uint32_t *>(at(L.blk_sys_off));
    P.acc_count = acc_off;
    P.sys_count = sys_off;
    P.acc_dense = accesses;
    P.sys_dense = sysvals;
    P.scan_tmp = static_cast<uint32_t *>(at(L.scan_tmp));
    P.scan_tmp_words = scan_tmp_words_needed((uint64_t)NA_N + 1);
    if (P.scan_tmp_words + cap_scan_words(NA_N) > SCAN_WORDS_MAX + CAP_WORDS_MAX) return DC_E_HIP;
    Plan *dP = static_cast<Plan *>(at(L.plan));

    hipError_t e = hipSuccess;
#define TRY(x)                                  \
    do {                                        \
        e = (x);                                \
        if (e != hipSuccess) return DC_E_HIP;   \
    } while (0)
    if (n_kernels)
        hipLaunchKernelGGL(k_na_prep, dim3(1), dim3(256), 0, s, ks, pb, ds, kernels, n_kernels, n_records,
                           n_args_total, (uint32_t)NA_N, n_instr_total);
    else
        TRY(launch_fill_u32(pb, 1, 0u, s));
    TRY(hipGetLastError());
    /* what this call reads before writing: leaders, first bad records and
     * the per-block record counts (a previous call's are still there) */
    TRY(launch_fill_u8(P.leader, n_instr_total, 0, s));
    TRY(launch_fill_u32(P.kbad, n_kernels, 0xFFFFFFFFu, s));
    TRY(launch_fill_u32(P.blk_acc, NA_N, 0u, s));
    TRY(launch_fill_u32(P.blk_sys, NA_N, 0u, s));
    TRY(launch_decode(P, s));
    TRY(launch_leader_scan(P, s));
    TRY(launch_number_blocks(P, s));
    TRY(launch_edges(P, s));
    hipLaunchKernelGGL(k_na_store_plan, dim3(1), dim3(64), 0, s, P, dP);
    TRY(hipGetLastError());
    FixCfg fc;
    fc.waves_per_group = (int)NA_WPG;
    fc.groups = (int)NA_GROUPS;
    TRY(launch_fixpoint(P, dP, fc, s, nullptr, nullptr));
    TRY(launch_compact(P, s));
#undef TRY
    return DC_OK;
}
