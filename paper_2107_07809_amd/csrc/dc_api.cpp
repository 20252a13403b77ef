/*
 * dc_api.cpp -- the C ABI of libdc (declared in include/dc.h): batch
 * planning and checks on the host, device allocation, stage enqueue on the
 * caller's stream, and result getters.
 */
#include <hip/hip_runtime_api.h>
#include <stdlib.h>
#include <string.h>

#include <stdio.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

#include "dc.h"
#include "dc_host.h"
#include "dc_internal.h"
#include "dc_opnames.h"

using namespace dc;

static const char *const OPCODE_NAMES[N_OPS] = {DC_OPNAME_LIST};

/* HIP events per run: start, after decoding, after the graph, right before and
 * right after the main fixpoint launch, end */
enum { EV_START, EV_DECODE, EV_CFG, EV_FIXB, EV_FIX, EV_END, N_EV };
constexpr int TIMING_RING = 64;

struct dc_batch {
    dc_ctx *ctx = nullptr;
    hipStream_t stream = nullptr;
    bool cfg_only = false;
    dc_options_t opts{};
    uint32_t K = 0;
    uint64_t N = 0;
    uint64_t n_records = 0, n_args_total = 0;
    DevMem mem;    /* arrays sized by kernels and positions, the arenas */
    DevMem bmem;   /* block-indexed arrays and record regions, sized from the records' totals */
    Plan P{};
    Plan *dP = nullptr;
    FixCfg fc{};
    std::vector<dc_kernel_t> kernels;
    std::vector<uint32_t> pos_begin;
    hipEvent_t ev[TIMING_RING][N_EV] = {};
    bool have_events = false;
    uint64_t runs = 0, runs_at_reset = 0;   /* enqueued runs; ring slot = run % TIMING_RING */
    uint64_t export_blocks = 0;
    bool blocks_planned = false;   /* bmem sized from the totals of the first run on these records */
    bool ovf_planned = false;   /* the overflow pass is sized from the first run's block counts */
    bool auto_arena = false;    /* no block cap given: the main arena grows to the largest kernel */
    hipGraphExec_t graph = nullptr;   /* DC_OPT_GRAPH: the stages captured on the second run */
    /* host copies, filled on first use after a run */
    bool host_valid = false;
    std::vector<dc_kernel_result_t> results;
    std::vector<uint32_t> acc_off, sys_off;
    std::vector<dc_access_t> acc;
    std::vector<dc_sysval_t> sys;
    std::vector<uint32_t> first_block;
    std::vector<dc_reg_state_t> states;
    std::vector<uint8_t> reached;
    /* CFG view copies */
    std::vector<int32_t> k_status;
    std::vector<uint32_t> k_nblocks, k_nreach, h_block_start, h_pred_off, h_pred, h_rpo;
    std::vector<int32_t> h_succ;
    std::vector<uint32_t> v_block_start, v_pred_off;   /* scratch for one view */
    /* a run on this graph whose stages follow the graph's (versions, structuring) */
    dc_status_t (*after_graph)(void *) = nullptr;
    void *after_graph_arg = nullptr;
    dc_status_t (*after_fix)(void *) = nullptr;   /* a graph-only batch's last stage, timed as ms_compact */
};
struct dc_cfg {
    dc_batch b;
};

static dc_status_t hip_fail(hipError_t e) { return e == hipErrorOutOfMemory ? DC_E_OOM : DC_E_HIP; }

extern "C" const char *dc_status_str(dc_status_t st) {
    switch (st) {
    case DC_OK: return "ok";
    case DC_E_INVAL: return "invalid argument";
    case DC_E_HIP: return "HIP runtime error";
    case DC_E_OOM: return "out of memory";
    case DC_E_NOTREADY: return "result not available";
    case DC_E_BADOP: return "opcode outside the instruction subset";
    case DC_E_BADREG: return "operand invalid for its role";
    case DC_E_BADTARGET: return "branch target out of range";
    case DC_E_NOEND: return "control falls off the end";
    case DC_E_UNSUPPORTED: return "unsupported kernel descriptor";
    case DC_E_NOFIX: return "no fixpoint within the sweep cap";
    case DC_E_CAPACITY: return "records changed after planning: more blocks or records than planned";
    }
    return "unknown status";
}

extern "C" int dc_opcode_count(void) { return N_OPS; }
extern "C" const char *dc_opcode_name(int id) { return (id >= 0 && id < N_OPS) ? OPCODE_NAMES[id] : nullptr; }

extern "C" dc_status_t dc_ctx_create(int hip_device, dc_ctx_t **out) {
    if (!out) return DC_E_INVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || hip_device < 0 || hip_device >= n) return DC_E_HIP;
    if (hipSetDevice(hip_device) != hipSuccess) return DC_E_HIP;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, hip_device) != hipSuccess) return DC_E_HIP;
    dc_ctx *c = new (std::nothrow) dc_ctx;
    if (!c) return DC_E_OOM;
    c->device = hip_device;
    c->n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 1;
    c->lds_per_cu = prop.maxSharedMemoryPerMultiProcessor ? prop.maxSharedMemoryPerMultiProcessor : 65536;
    c->lds_per_group = prop.sharedMemPerBlock ? prop.sharedMemPerBlock : 65536;
    /* set-up of dc_analyze_noalloc on this device: resolve its scratch array */
    if (!noalloc_setup(hip_device)) {
        delete c;
        return DC_E_HIP;
    }
    *out = c;
    return DC_OK;
}

extern "C" void dc_ctx_destroy(dc_ctx_t *ctx) { delete ctx; }

PlanInputs dc::alloc_plan(DevMem &M, Plan &P, const PlanDims &d) {
    const uint64_t N = d.N, K = d.K;
    PlanInputs in;
    in.kernels = M.alloc<dc_kernel_t>(K);
    in.args = M.alloc<dc_arg_t>(d.A);
    in.pos_begin = M.alloc<uint32_t>(K + 1);
    in.desc_status = M.alloc<int32_t>(K);
    P.kernels = in.kernels;
    P.args = in.args;
    P.pos_begin = in.pos_begin;
    P.desc_status = in.desc_status;
    P.leader = M.alloc<uint8_t>(N + 16);
    P.pcap = M.alloc<uint8_t>(N + 16);
    P.block_id = M.alloc<uint32_t>(N);
    P.totals = M.alloc<uint32_t>(4);
    P.kbad = M.alloc<uint32_t>(K);
    P.status = M.alloc<int32_t>(K);
    P.first_block = M.alloc<uint32_t>(K);
    P.n_blocks = M.alloc<uint32_t>(K);
    P.n_reach = M.alloc<uint32_t>(K);
    P.scan_tmp_words = scan_tmp_words_needed(std::max<uint64_t>(N + 1, K + 1));
    P.scan_tmp = M.alloc<uint32_t>(P.scan_tmp_words + (d.cfg_only ? 0 : cap_scan_words(N)));
    P.blk_cap = 0;
    in.work_order = nullptr;
    P.work_order = nullptr;
    P.kslots = nullptr;
    P.with_records = d.cfg_only ? 0u : 1u;
    if (d.cfg_only) return in;
    in.work_order = M.alloc<uint32_t>(K);
    P.work_order = in.work_order;
    P.kslots = M.alloc<uint32_t>(K * KSLOT_WORDS);
    P.arena_rows = d.arena_rows;
    P.main_waves = (uint32_t)d.waves;
    P.arena = M.alloc<uint32_t>(d.waves * d.arena_rows * FIX_ROW_DWORDS);
    P.ovf_block_cap = 0;
    P.ovf_rows = 0;
    P.ovf_waves = 0;
    P.ovf_arena = nullptr;
    P.ovf_bitmaps = nullptr;
    P.dummy = M.alloc<uint4>((d.waves + OVF_MAX_WAVES) * 64);
    P.ovf_list = M.alloc<uint32_t>(K);
    P.counters = M.alloc<uint32_t>(8);
    P.results = M.alloc<dc_kernel_result_t>(K);
    P.acc_count = M.alloc<uint32_t>(K + 1);
    P.sys_count = M.alloc<uint32_t>(K + 1);
    P.export_states = nullptr;
    P.export_reached = nullptr;
    return in;
}

void dc::alloc_blocks(DevMem &M, Plan &P, uint64_t blocks, uint64_t acc, uint64_t sys, bool cfg_only) {
    const uint64_t B = blocks;
    P.blk_cap = (uint32_t)B;
    P.block_start = M.alloc<uint32_t>(B + 1);
    P.block_kernel = M.alloc<uint32_t>(B);
    P.succ = M.alloc<int32_t>(2 * B);
    P.pred_cnt = M.alloc<uint32_t>(B + 1);
    P.pred_fill = M.alloc<uint32_t>(B);
    P.pred = M.alloc<uint32_t>(2 * B);
    P.rpo = M.alloc<uint32_t>(B);
    P.rpo_pos = M.alloc<int32_t>(B);
    P.dfs_stack = M.alloc<uint32_t>(B);
    P.dfs_seen = M.alloc<uint8_t>(B);
    if (cfg_only) {
        P.binfo = nullptr;
        P.blk_acc_base = P.blk_sys_base = nullptr;
        return;
    }
    P.binfo = M.alloc<uint4>(2 * B);
    P.blk_acc_base = M.alloc<uint32_t>(B + 1);
    P.blk_sys_base = M.alloc<uint32_t>(B + 1);
    P.blk_acc = M.alloc<uint32_t>(B);
    P.blk_sys = M.alloc<uint32_t>(B);
    P.blk_acc_off = M.alloc<uint32_t>(B);
    P.blk_sys_off = M.alloc<uint32_t>(B);
    P.acc_cap = (uint32_t)acc;
    P.sys_cap = (uint32_t)sys;
    P.acc_sparse = M.alloc<dc_access_t>(acc);
    P.acc_dense = M.alloc<dc_access_t>(acc);
    P.sys_sparse = M.alloc<dc_sysval_t>(sys);
    P.sys_dense = M.alloc<dc_sysval_t>(sys);
}

static dc_status_t plan_batch(dc_batch *B, dc_ctx *ctx, const dc_kernel_t *kernels, uint32_t n_kernels,
                              const dc_instr_t *instrs, uint64_t n_records, const dc_arg_t *args, uint64_t n_args_total,
                              const dc_options_t *opts, void *stream, bool cfg_only) {
    if (!ctx || (n_kernels && !kernels) || (n_records && !instrs) || (n_args_total && !args)) return DC_E_INVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return DC_E_HIP;
    B->ctx = ctx;
    B->stream = (hipStream_t)stream;
    B->cfg_only = cfg_only;
    if (opts) B->opts = *opts;
    if (B->opts.flags & ~(DC_OPT_EXPORT_STATES | DC_OPT_DIGEST | DC_OPT_TIMING | DC_OPT_GRAPH | DC_OPT_LONGEST_FIRST |
                          DC_OPT_PLAIN))
        return DC_E_INVAL;
    if ((B->opts.flags & DC_OPT_PLAIN) && (cfg_only || (B->opts.flags & (DC_OPT_EXPORT_STATES | DC_OPT_GRAPH))))
        return DC_E_INVAL;
    if ((B->opts.flags & DC_OPT_GRAPH) && (B->opts.flags & (DC_OPT_EXPORT_STATES | DC_OPT_TIMING))) return DC_E_INVAL;
    /* waves per group: the fixpoint kernel's LDS per wave must fit a group */
    const size_t lds_wave = fixpoint_lds_per_wave();
    if (B->opts.waves_per_group == 0)
        B->opts.waves_per_group = (uint32_t)std::max<size_t>(1, std::min<size_t>(4, ctx->lds_per_group / lds_wave));
    if (B->opts.waves_per_group > 4 || B->opts.waves_per_group * lds_wave > ctx->lds_per_group) return DC_E_INVAL;
    B->auto_arena = B->opts.block_cap == 0;
    if (B->opts.block_cap == 0) B->opts.block_cap = 256;
    if (B->opts.block_cap > 2048) return DC_E_INVAL;   /* the main pass keeps its bitmaps in one VGPR */
    B->K = n_kernels;
    B->n_records = n_records;
    B->n_args_total = n_args_total;
    B->kernels.assign(kernels, kernels + n_kernels);
    B->pos_begin.resize((size_t)n_kernels + 1);
    std::vector<int32_t> dstat(n_kernels);
    uint64_t pos = 0;
    for (uint32_t k = 0; k < n_kernels; k++) {
        const dc_kernel_t &d = kernels[k];
        if (d.instr_begin > n_records || d.n_instr > n_records - d.instr_begin) return DC_E_INVAL;
        dstat[k] = descriptor_status(d);
        if (dstat[k] == DC_OK && ((uint64_t)d.arg_begin + d.n_args > n_args_total)) return DC_E_INVAL;
        B->pos_begin[k] = (uint32_t)pos;
        pos += d.n_instr;
        if (pos >= 0xFFFFFFF0ull) return DC_E_INVAL;   /* positions are 32-bit */
    }
    B->pos_begin[n_kernels] = (uint32_t)pos;
    B->N = pos;
    const uint64_t N = pos, K = n_kernels;
    DevMem &M = B->mem;
    Plan &P = B->P;
    P.instrs = instrs;
    P.n_kernels = n_kernels;
    P.n_pos = (uint32_t)N;
    P.n_records = n_records;
    P.n_args = n_args_total;
    const bool plain = (B->opts.flags & DC_OPT_PLAIN) != 0;
    uint64_t n_max = 0;
    for (uint32_t k = 0; k < n_kernels; k++) n_max = std::max<uint64_t>(n_max, kernels[k].n_instr);
    PlanDims dims{N, K, n_args_total, cfg_only, 0, 0};
    if (plain) {
        /* one scratch plan for the longest kernel: the launches run in turn */
        dims.N = n_max;
        dims.waves = 1;
        dims.arena_rows = (uint32_t)(FIX_MAX_ROWS * std::max<uint64_t>(n_max, 1));
        B->fc.waves_per_group = 1;
        B->fc.groups = 1;
    } else if (!cfg_only) {
        const uint32_t wpg = B->opts.waves_per_group;
        /* persistent grid: as many groups per CU as the fixpoint kernel's
         * registers and LDS allow */
        uint32_t per_cu = B->opts.groups_per_cu;
        if (per_cu == 0) per_cu = fixpoint_groups_per_cu(wpg);
        B->fc.waves_per_group = (int)wpg;
        B->fc.groups = (int)std::max<uint64_t>(1, std::min<uint64_t>((uint64_t)ctx->n_cu * per_cu, (K + wpg - 1) / wpg));
        dims.waves = (uint64_t)B->fc.groups * wpg;
        /* main pass arena: block_cap blocks of two state rows (kernels with up
         * to 128 named register slots), or fewer blocks of six rows */
        dims.arena_rows = 2 * B->opts.block_cap;
    }
    const PlanInputs in = alloc_plan(M, P, dims);
    dc_kernel_t *d_k = in.kernels;
    dc_arg_t *d_a = in.args;
    uint32_t *d_pb = in.pos_begin;
    int32_t *d_ds = in.desc_status;
    if (!cfg_only) {
        P.sweep_cap = B->opts.sweep_cap;
        P.flags = B->opts.flags;
    }
    if (plain) {
        /* block arrays and regions for the longest kernel; dense outputs for
         * the batch (one access and four built-in records per instruction) */
        P.n_pos = (uint32_t)n_max;
        alloc_blocks(B->bmem, P, n_max, n_max, 4 * n_max, false);
        P.acc_dense = M.alloc<dc_access_t>(N);
        P.sys_dense = M.alloc<dc_sysval_t>(4 * N);
        P.ovf_bitmaps = M.alloc<uint32_t>(2 * ((n_max + 31) / 32) + 64);
        P.ovf_block_cap = (uint32_t)n_max;
        B->blocks_planned = B->ovf_planned = true;
    }
    B->dP = M.alloc<Plan>(1);
    if (M.failed) return DC_E_OOM;
    hipStream_t s = B->stream;
    hipError_t e = hipSuccess;
    if (K) e = hipMemcpyAsync(d_k, kernels, K * sizeof(dc_kernel_t), hipMemcpyHostToDevice, s);
    if (e == hipSuccess && n_args_total)
        e = hipMemcpyAsync(d_a, args, n_args_total * sizeof(dc_arg_t), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_pb, B->pos_begin.data(), (K + 1) * sizeof(uint32_t), hipMemcpyHostToDevice, s);
    if (e == hipSuccess && K) e = hipMemcpyAsync(d_ds, dstat.data(), K * sizeof(int32_t), hipMemcpyHostToDevice, s);
    /* DC_OPT_LONGEST_FIRST: the fixpoint takes the longest kernels first, so
     * that no long kernel starts last and holds up the end of the launch (it
     * also runs the longest kernels side by side, whose larger arenas compete
     * for the caches; the autotuner measures which order is faster) */
    std::vector<uint32_t> order;
    if (!cfg_only && !(B->opts.flags & DC_OPT_LONGEST_FIRST)) P.work_order = nullptr;
    if (!cfg_only && K && (B->opts.flags & DC_OPT_LONGEST_FIRST)) {
        order.resize(K);
        for (uint32_t k = 0; k < K; k++) order[k] = k;
        std::stable_sort(order.begin(), order.end(),
                         [&](uint32_t a, uint32_t b) { return kernels[a].n_instr > kernels[b].n_instr; });
        if (e == hipSuccess)
            e = hipMemcpyAsync(in.work_order, order.data(), K * sizeof(uint32_t), hipMemcpyHostToDevice, s);
    }
    if (e == hipSuccess) e = hipMemcpyAsync(B->dP, &P, sizeof(Plan), hipMemcpyHostToDevice, s);
    /* the host vectors above are stack/batch owned: make the copies complete */
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e);
    if (B->opts.flags & DC_OPT_TIMING) {
        for (int r = 0; r < TIMING_RING; r++)
            for (int i = 0; i < N_EV; i++)
                if (hipEventCreate(&B->ev[r][i]) != hipSuccess) return DC_E_HIP;
        B->have_events = true;
    }
    return DC_OK;
}

/* Arena sizing from the block counts of the CFG stage just enqueued (waits
 * for the stream).  A kernel whose state width is not known yet may need up
 * to FIX_MAX_ROWS rows per block.  Without an explicit block cap the main
 * pass's arenas grow to hold the largest kernel it can take (at most 2048
 * blocks), within ARENA_BUDGET and a quarter of the free device memory; the
 * kernels that still do not fit go to the overflow pass, which gets up to
 * OVF_MAX_WAVES waves within the same budget.  A later run on the same
 * records has the same block counts; a run on other records plans again. */
static hipError_t plan_overflow(dc_batch *B, hipStream_t s) {
    Plan &P = B->P;
    std::vector<uint32_t> nb(B->K);
    hipError_t e = hipSuccess;
    if (B->K) e = hipMemcpyAsync(nb.data(), P.n_blocks, B->K * sizeof(uint32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    const uint64_t row_bytes = FIX_ROW_DWORDS * 4ull;
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) free_b = 0;
    const uint64_t budget = std::min<uint64_t>(ARENA_BUDGET, free_b / 4);
    if (B->auto_arena) {
        uint64_t need = 0;
        for (uint32_t x : nb)
            if (x <= 2048) need = std::max<uint64_t>(need, (uint64_t)x * FIX_MAX_ROWS);
        const uint64_t rows = std::min<uint64_t>(need, budget / ((uint64_t)P.main_waves * row_bytes));
        if (rows > P.arena_rows) {
            B->mem.release(P.arena);
            P.arena = B->mem.alloc<uint32_t>((uint64_t)P.main_waves * rows * FIX_ROW_DWORDS);
            if (B->mem.failed) return hipErrorOutOfMemory;
            P.arena_rows = (uint32_t)rows;
        }
    }
    uint64_t cap = 1, n_ovf = 0;
    for (uint32_t x : nb) {
        if (x > 2048 || (uint64_t)x * FIX_MAX_ROWS > P.arena_rows) {
            n_ovf++;
            cap = std::max<uint64_t>(cap, x);
        }
    }
    const uint64_t fit = budget / (cap * FIX_MAX_ROWS * row_bytes);
    const uint64_t waves = std::max<uint64_t>(1, std::min<uint64_t>({(uint64_t)OVF_MAX_WAVES, n_ovf, fit}));
    P.ovf_block_cap = (uint32_t)cap;
    P.ovf_rows = (uint32_t)(cap * FIX_MAX_ROWS);
    P.ovf_waves = (uint32_t)waves;
    if (P.ovf_arena) B->mem.release(P.ovf_arena);
    if (P.ovf_bitmaps) B->mem.release(P.ovf_bitmaps);
    P.ovf_arena = B->mem.alloc<uint32_t>(waves * P.ovf_rows * FIX_ROW_DWORDS);
    P.ovf_bitmaps = B->mem.alloc<uint32_t>(waves * (2 * ((cap + 31) / 32) + 64));
    if (B->mem.failed) return hipErrorOutOfMemory;
    B->ovf_planned = true;
    return hipSuccess;
}

/* Size the block-indexed arrays and the record regions from the totals of
 * the decode and leader-scan stages just enqueued (waits for the stream):
 * the block count, the access and the built-in record capacity. */
static hipError_t plan_blocks(dc_batch *B, hipStream_t s) {
    Plan &P = B->P;
    uint32_t t[4] = {0, 0, 0, 0};
    hipError_t e = hipMemcpyAsync(t, P.totals, sizeof(t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    B->bmem.reset();
    alloc_blocks(B->bmem, P, t[0], t[1], t[2], B->cfg_only);
    if (B->bmem.failed) return hipErrorOutOfMemory;
    B->blocks_planned = true;
    return hipSuccess;
}

/* every stage of an analysis run, enqueued on s (no host synchronisation) */
static hipError_t enqueue_stages(dc_batch *B, hipStream_t s) {
    const Plan &P = B->P;
    hipError_t e = launch_fill_u8(P.leader, B->N, 0, s);
    if (e == hipSuccess) e = launch_fill_u32(P.kbad, B->K, 0xFFFFFFFFu, s);
    if (e == hipSuccess) e = launch_decode(P, s);
    if (e == hipSuccess) e = launch_leader_scan(P, s);
    if (e == hipSuccess) e = launch_number_blocks(P, s);
    if (e == hipSuccess) e = launch_edges(P, s);
    if (e == hipSuccess) e = launch_fixpoint(P, B->dP, B->fc, s, nullptr, nullptr);
    if (e == hipSuccess) e = launch_compact(P, s);
    return e;
}

/* DC_OPT_GRAPH runs after the first: capture the stages once, replay */
static dc_status_t enqueue_graph(dc_batch *B) {
    hipStream_t s = B->stream;
    if (!B->graph) {
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(e);
        const hipError_t es = enqueue_stages(B, s);
        e = hipStreamEndCapture(s, &g);
        if (es != hipSuccess || e != hipSuccess) {
            if (g) hipGraphDestroy(g);
            return hip_fail(es != hipSuccess ? es : e);
        }
        e = hipGraphInstantiate(&B->graph, g, nullptr, nullptr, 0);
        hipGraphDestroy(g);
        if (e != hipSuccess) {
            B->graph = nullptr;
            return hip_fail(e);
        }
    }
    const hipError_t e = hipGraphLaunch(B->graph, s);
    if (e != hipSuccess) return hip_fail(e);
    B->runs++;
    return DC_OK;
}

static dc_status_t enqueue(dc_batch *B) {
    Plan &P = B->P;
    hipStream_t s = B->stream;
    hipError_t e = hipSuccess;
    B->host_valid = false;
    if ((B->opts.flags & DC_OPT_GRAPH) && B->ovf_planned && !B->cfg_only && s) return enqueue_graph(B);
    hipEvent_t *ev = B->ev[B->runs % TIMING_RING];
#define TRY(x)                                  \
    do {                                        \
        e = (x);                                \
        if (e != hipSuccess) return hip_fail(e); \
    } while (0)
    if (B->have_events) TRY(hipEventRecord(ev[EV_START], s));
    if (B->opts.flags & DC_OPT_PLAIN) {
        if (B->have_events) {
            TRY(hipEventRecord(ev[EV_DECODE], s));
            TRY(hipEventRecord(ev[EV_CFG], s));
        }
        TRY(launch_plain(P, B->dP, s, B->have_events ? ev[EV_FIXB] : nullptr, B->have_events ? ev[EV_FIX] : nullptr));
        if (B->have_events) TRY(hipEventRecord(ev[EV_END], s));
        B->runs++;
        return DC_OK;
    }
    TRY(launch_fill_u8(P.leader, B->N, 0, s));
    TRY(launch_fill_u32(P.kbad, B->K, 0xFFFFFFFFu, s));
    TRY(launch_decode(P, s));
    if (B->have_events) TRY(hipEventRecord(ev[EV_DECODE], s));
    TRY(launch_leader_scan(P, s));
    bool plan_changed = false;
    if (!B->blocks_planned) {
        e = plan_blocks(B, s);
        if (e == hipErrorOutOfMemory) return DC_E_OOM;
        if (e != hipSuccess) return hip_fail(e);
        plan_changed = true;
    }
    TRY(launch_number_blocks(P, s));
    TRY(launch_edges(P, s));
    if (B->have_events) TRY(hipEventRecord(ev[EV_CFG], s));
    if (B->cfg_only) {
        if (B->have_events) TRY(hipEventRecord(ev[EV_FIXB], s));
        if (B->after_graph) {
            const dc_status_t st = B->after_graph(B->after_graph_arg);
            if (st != DC_OK) return st;
        }
        if (B->have_events) TRY(hipEventRecord(ev[EV_FIX], s));
        if (B->after_fix) {
            const dc_status_t st = B->after_fix(B->after_graph_arg);
            if (st != DC_OK) return st;
        }
        if (B->have_events) TRY(hipEventRecord(ev[EV_END], s));
        B->runs++;
        return DC_OK;
    }
    if (!B->ovf_planned) {
        e = plan_overflow(B, s);
        if (e == hipErrorOutOfMemory) return DC_E_OOM;
        if (e != hipSuccess) return hip_fail(e);
        plan_changed = true;
    }
    if (B->opts.flags & DC_OPT_EXPORT_STATES) {
        /* size the state export from the block count */
        uint32_t total = 0;
        TRY(hipMemcpyAsync(&total, P.totals, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        TRY(hipStreamSynchronize(s));
        if (total > B->export_blocks || !P.export_states) {
            if (P.export_states) B->mem.release(P.export_states);
            if (P.export_reached) B->mem.release(P.export_reached);
            P.export_states = B->mem.alloc<dc_reg_state_t>((uint64_t)std::max<uint32_t>(total, 1) * NSLOT);
            P.export_reached = B->mem.alloc<uint8_t>(std::max<uint32_t>(total, 1));
            if (B->mem.failed) return DC_E_OOM;
            B->export_blocks = total;
        }
        plan_changed = true;
    }
    if (plan_changed) {
        TRY(hipMemcpyAsync(B->dP, &P, sizeof(Plan), hipMemcpyHostToDevice, s));
        TRY(hipStreamSynchronize(s));
    }
    TRY(launch_fixpoint(P, B->dP, B->fc, s, B->have_events ? ev[EV_FIXB] : nullptr,
                        B->have_events ? ev[EV_FIX] : nullptr));
    TRY(launch_compact(P, s));
    if (B->have_events) TRY(hipEventRecord(ev[EV_END], s));
    B->runs++;
#undef TRY
    return DC_OK;
}

extern "C" dc_status_t dc_analyze_batch(dc_ctx_t *ctx, const dc_kernel_t *kernels, uint32_t n_kernels,
                                        const dc_instr_t *instrs, uint64_t n_records, const dc_arg_t *args,
                                        uint64_t n_args_total, const dc_options_t *opts, void *stream,
                                        dc_batch_t **out) {
    if (!out) return DC_E_INVAL;
    *out = nullptr;
    dc_batch *B = new (std::nothrow) dc_batch;
    if (!B) return DC_E_OOM;
    dc_status_t st = plan_batch(B, ctx, kernels, n_kernels, instrs, n_records, args, n_args_total, opts, stream, false);
    if (st == DC_OK) st = enqueue(B);
    if (st != DC_OK) {
        hipStreamSynchronize(B->stream);
        delete B;
        return st;
    }
    *out = B;
    return DC_OK;
}

/* Autotuner cache: the choice for a batch of this size bucket on a device of
 * this many CUs (in the process; in the file named by DC_TUNE_CACHE when
 * set, one entry per line: cus len_bucket k_bucket flags waves groups order ms) */
struct TuneKey {
    int cus;
    uint32_t len_bucket, k_bucket, flags;
    bool operator<(const TuneKey &o) const {
        return std::tie(cus, len_bucket, k_bucket, flags) < std::tie(o.cus, o.len_bucket, o.k_bucket, o.flags);
    }
};
struct TuneVal {
    uint32_t waves, groups, order;
    float ms;
};
static std::mutex g_tune_mu;
static std::map<TuneKey, TuneVal> g_tune;
static bool g_tune_loaded = false;

static uint32_t log2_bucket(uint64_t x) {
    uint32_t b = 0;
    while (x > 1) {
        x >>= 1;
        b++;
    }
    return b;
}

static void tune_load_locked() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char *path = getenv("DC_TUNE_CACHE");
    if (!path) return;
    FILE *f = fopen(path, "r");
    if (!f) return;
    TuneKey k;
    TuneVal v;
    while (fscanf(f, "%d %u %u %u %u %u %u %f", &k.cus, &k.len_bucket, &k.k_bucket, &k.flags, &v.waves, &v.groups,
                  &v.order, &v.ms) == 8)
        g_tune[k] = v;
    fclose(f);
}

static void tune_store_locked(const TuneKey &k, const TuneVal &v) {
    g_tune[k] = v;
    const char *path = getenv("DC_TUNE_CACHE");
    if (!path) return;
    FILE *f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "%d %u %u %u %u %u %u %.4f\n", k.cus, k.len_bucket, k.k_bucket, k.flags, v.waves, v.groups, v.order,
            v.ms);
    fclose(f);
}

extern "C" dc_status_t dc_autotune(dc_ctx_t *ctx, const dc_kernel_t *kernels, uint32_t n_kernels,
                                   const dc_instr_t *instrs, uint64_t n_records, const dc_arg_t *args,
                                   uint64_t n_args_total, const dc_options_t *base, uint32_t sample, void *stream,
                                   dc_options_t *best, float *best_ms) {
    if (!ctx || !best || !best_ms || (n_kernels && !kernels)) return DC_E_INVAL;
    if (base && (base->flags & DC_OPT_GRAPH)) return DC_E_INVAL;
    if (sample == 0) sample = 8192;
    const uint32_t stride = std::max<uint32_t>(1, (n_kernels + sample - 1) / sample);
    std::vector<dc_kernel_t> ks;
    uint64_t n_sum = 0;
    for (uint32_t k = 0; k < n_kernels; k += stride) {
        ks.push_back(kernels[k]);
        n_sum += kernels[k].n_instr;
    }
    const uint32_t keep = base ? base->flags & (DC_OPT_DIGEST | DC_OPT_EXPORT_STATES) : 0u;
    const TuneKey key{ctx->n_cu, log2_bucket(ks.empty() ? 0 : n_sum / ks.size()), log2_bucket(n_kernels), keep};
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_load_locked();
        auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            *best = base ? *base : dc_options_t{};
            best->waves_per_group = it->second.waves;
            best->groups_per_cu = it->second.groups;
            best->flags = (best->flags & ~DC_OPT_LONGEST_FIRST) | it->second.order;
            *best_ms = it->second.ms;
            return DC_OK;
        }
    }
    const size_t lds_wave = fixpoint_lds_per_wave();
    const uint32_t wmax = (uint32_t)std::max<size_t>(1, std::min<size_t>(4, ctx->lds_per_group / lds_wave));
    std::vector<std::pair<uint32_t, uint32_t>> shapes;
    for (uint32_t w : {1u, 2u, wmax}) {
        if (w > wmax || std::find_if(shapes.begin(), shapes.end(), [&](auto &x) { return x.first == w; }) != shapes.end())
            continue;
        const uint32_t pc = fixpoint_groups_per_cu(w);
        shapes.push_back({w, pc});
        if ((pc * 3 + 3) / 4 != pc) shapes.push_back({w, (pc * 3 + 3) / 4});
    }
    dc_options_t o{};
    if (base) o = *base;
    o.flags = (o.flags & ~(DC_OPT_EXPORT_STATES | DC_OPT_LONGEST_FIRST)) | DC_OPT_TIMING;
    float best_t = -1.0f;
    TuneVal bv{};
    for (uint32_t order : {0u, DC_OPT_LONGEST_FIRST}) {
        for (auto [w, pc] : shapes) {
            o.waves_per_group = w;
            o.groups_per_cu = pc;
            const uint32_t f0 = o.flags;
            o.flags = f0 | order;
            dc_batch_t *B = nullptr;
            dc_status_t st = dc_analyze_batch(ctx, ks.data(), (uint32_t)ks.size(), instrs, n_records, args,
                                              n_args_total, &o, stream, &B);
            o.flags = f0;
            if (st != DC_OK) return st;
            dc_timing_t t{};
            st = dc_batch_wait(B);
            if (st == DC_OK) st = dc_timing_reset(B);
            for (int r = 0; r < 3 && st == DC_OK; r++) st = dc_batch_run(B, nullptr, stream);
            if (st == DC_OK) st = dc_get_timing(B, &t);
            dc_batch_free(B);
            if (st != DC_OK) return st;
            const float ms = t.runs ? t.ms_total / t.runs : 0.0f;
            if (best_t < 0.0f || ms < best_t) {
                best_t = ms;
                bv = TuneVal{w, pc, order, ms};
            }
        }
    }
    *best = base ? *base : dc_options_t{};
    best->waves_per_group = bv.waves;
    best->groups_per_cu = bv.groups;
    best->flags = (best->flags & ~DC_OPT_LONGEST_FIRST) | bv.order;
    *best_ms = best_t;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_store_locked(key, bv);
    return DC_OK;
}

extern "C" dc_status_t dc_batch_run(dc_batch_t *B, const dc_instr_t *instrs, void *stream) {
    if (!B || B->cfg_only) return DC_E_INVAL;
    if (hipSetDevice(B->ctx->device) != hipSuccess) return DC_E_HIP;
    B->stream = (hipStream_t)stream;
    if (instrs && instrs != B->P.instrs) {
        /* other records: their block counts and record capacities may differ,
         * so the block-indexed arrays, the regions and the arenas are planned
         * again on this run */
        if (hipStreamSynchronize(B->stream) != hipSuccess) return DC_E_HIP;
        B->P.instrs = instrs;
        if (B->graph) {   /* the captured launches hold the old plan */
            hipGraphExecDestroy(B->graph);
            B->graph = nullptr;
        }
        B->blocks_planned = false;
        B->ovf_planned = false;
    }
    return enqueue(B);
}

extern "C" dc_status_t dc_batch_wait(dc_batch_t *B) {
    if (!B) return DC_E_INVAL;
    if (hipSetDevice(B->ctx->device) != hipSuccess) return DC_E_HIP;
    hipError_t e = hipStreamSynchronize(B->stream);
    return e == hipSuccess ? DC_OK : hip_fail(e);
}

/* copy results to the host once per run */
static dc_status_t fetch(dc_batch *B) {
    if (B->host_valid) return DC_OK;
    dc_status_t st = dc_batch_wait(B);
    if (st != DC_OK) return st;
    const Plan &P = B->P;
    const uint32_t K = B->K;
    hipError_t e = hipSuccess;
    B->results.resize(K);
    B->acc_off.resize((size_t)K + 1);
    B->sys_off.resize((size_t)K + 1);
    if (K) e = hipMemcpy(B->results.data(), P.results, K * sizeof(dc_kernel_result_t), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(B->acc_off.data(), P.acc_count, (K + 1) * sizeof(uint32_t), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(B->sys_off.data(), P.sys_count, (K + 1) * sizeof(uint32_t), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e);
    const uint64_t na = B->acc_off[K], ns = B->sys_off[K];
    B->acc.resize(na);
    B->sys.resize(ns);
    if (na) e = hipMemcpy(B->acc.data(), P.acc_dense, na * sizeof(dc_access_t), hipMemcpyDeviceToHost);
    if (e == hipSuccess && ns) e = hipMemcpy(B->sys.data(), P.sys_dense, ns * sizeof(dc_sysval_t), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e);
    if (B->opts.flags & DC_OPT_EXPORT_STATES) {
        B->first_block.resize(K);
        B->states.resize(B->export_blocks * NSLOT);
        B->reached.resize(B->export_blocks);
        if (K) e = hipMemcpy(B->first_block.data(), P.first_block, K * sizeof(uint32_t), hipMemcpyDeviceToHost);
        if (e == hipSuccess && B->export_blocks)
            e = hipMemcpy(B->states.data(), P.export_states, B->export_blocks * NSLOT * sizeof(dc_reg_state_t),
                          hipMemcpyDeviceToHost);
        if (e == hipSuccess && B->export_blocks)
            e = hipMemcpy(B->reached.data(), P.export_reached, B->export_blocks, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e);
    }
    B->host_valid = true;
    return DC_OK;
}

extern "C" dc_status_t dc_get_kernel_result(const dc_batch_t *cb, uint32_t k, dc_kernel_result_t *out) {
    dc_batch *B = const_cast<dc_batch *>(cb);
    if (!B || !out || B->cfg_only || k >= B->K) return DC_E_INVAL;
    dc_status_t st = fetch(B);
    if (st != DC_OK) return st;
    *out = B->results[k];
    return DC_OK;
}

extern "C" dc_status_t dc_get_kernel_status(const dc_batch_t *cb, uint32_t k, dc_status_t *out) {
    dc_kernel_result_t r;
    if (!out) return DC_E_INVAL;
    dc_status_t st = dc_get_kernel_result(cb, k, &r);
    if (st == DC_OK) *out = r.status;
    return st;
}

extern "C" dc_status_t dc_get_results(const dc_batch_t *cb, dc_kernel_result_t *out, uint32_t cap) {
    dc_batch *B = const_cast<dc_batch *>(cb);
    if (!B || (cap && !out) || B->cfg_only) return DC_E_INVAL;
    dc_status_t st = fetch(B);
    if (st != DC_OK) return st;
    if (std::min<uint64_t>(cap, B->K)) memcpy(out, B->results.data(), sizeof(dc_kernel_result_t) * std::min<uint64_t>(cap, B->K));
    return DC_OK;
}

template <typename T>
static dc_status_t get_records(dc_batch *B, const std::vector<T> &all, const std::vector<uint32_t> &off, uint32_t k,
                               T *buf, uint32_t cap, uint32_t *n_total) {
    if (!n_total || (cap && !buf) || k >= B->K) return DC_E_INVAL;
    const uint32_t n = off[k + 1] - off[k];
    *n_total = n;
    if (std::min(cap, n)) memcpy(buf, all.data() + off[k], sizeof(T) * std::min(cap, n));
    return DC_OK;
}

extern "C" dc_status_t dc_get_accesses(const dc_batch_t *cb, uint32_t k, dc_access_t *buf, uint32_t cap,
                                       uint32_t *n_total) {
    dc_batch *B = const_cast<dc_batch *>(cb);
    if (!B || B->cfg_only) return DC_E_INVAL;
    dc_status_t st = fetch(B);
    if (st != DC_OK) return st;
    return get_records(B, B->acc, B->acc_off, k, buf, cap, n_total);
}

extern "C" dc_status_t dc_get_sysvals(const dc_batch_t *cb, uint32_t k, dc_sysval_t *buf, uint32_t cap,
                                      uint32_t *n_total) {
    dc_batch *B = const_cast<dc_batch *>(cb);
    if (!B || B->cfg_only) return DC_E_INVAL;
    dc_status_t st = fetch(B);
    if (st != DC_OK) return st;
    return get_records(B, B->sys, B->sys_off, k, buf, cap, n_total);
}

template <typename T>
static dc_status_t get_all(dc_batch *B, const std::vector<T> &all, const std::vector<uint32_t> &off, T *buf,
                           uint64_t cap, uint64_t *n_total, uint64_t *offsets) {
    if (!n_total || (cap && !buf)) return DC_E_INVAL;
    *n_total = all.size();
    if (std::min<uint64_t>(cap, all.size())) memcpy(buf, all.data(), sizeof(T) * std::min<uint64_t>(cap, all.size()));
    if (offsets)
        for (uint32_t k = 0; k <= B->K; k++) offsets[k] = off[k];
    return DC_OK;
}

extern "C" dc_status_t dc_get_all_accesses(const dc_batch_t *cb, dc_access_t *buf, uint64_t cap, uint64_t *n_total,
                                           uint64_t *offsets) {
    dc_batch *B = const_cast<dc_batch *>(cb);
    if (!B || B->cfg_only) return DC_E_INVAL;
    dc_status_t st = fetch(B);
    if (st != DC_OK) return st;
    return get_all(B, B->acc, B->acc_off, buf, cap, n_total, offsets);
}

extern "C" dc_status_t dc_get_all_sysvals(const dc_batch_t *cb, dc_sysval_t *buf, uint64_t cap, uint64_t *n_total,
                                          uint64_t *offsets) {
    dc_batch *B = const_cast<dc_batch *>(cb);
    if (!B || B->cfg_only) return DC_E_INVAL;
    dc_status_t st = fetch(B);
    if (st != DC_OK) return st;
    return get_all(B, B->sys, B->sys_off, buf, cap, n_total, offsets);
}

extern "C" dc_status_t dc_get_block_state(const dc_batch_t *cb, uint32_t k, uint32_t block, dc_reg_state_t *out368,
                                          uint8_t *reached) {
    dc_batch *B = const_cast<dc_batch *>(cb);
    if (!B || !out368 || B->cfg_only || k >= B->K) return DC_E_INVAL;
    if (!(B->opts.flags & DC_OPT_EXPORT_STATES)) return DC_E_NOTREADY;
    dc_status_t st = fetch(B);
    if (st != DC_OK) return st;
    const dc_kernel_result_t &r = B->results[k];
    if (r.status != DC_OK || block >= r.n_blocks) return DC_E_INVAL;
    const uint64_t g = (uint64_t)B->first_block[k] + block;
    memcpy(out368, B->states.data() + g * NSLOT, sizeof(dc_reg_state_t) * NSLOT);
    if (reached) *reached = B->reached[g];
    return DC_OK;
}

extern "C" dc_status_t dc_get_stats(const dc_batch_t *cb, dc_stats_t *out) {
    dc_batch *B = const_cast<dc_batch *>(cb);
    if (!B || !out || B->cfg_only) return DC_E_INVAL;
    dc_status_t st = fetch(B);
    if (st != DC_OK) return st;
    memset(out, 0, sizeof(*out));
    out->n_kernels = B->K;
    out->n_instr = B->N;
    uint32_t ovf = 0;
    for (const dc_kernel_result_t &r : B->results) {
        if (r.status != DC_OK) {
            out->n_failed++;
            continue;
        }
        out->n_blocks += r.n_blocks;
        out->sweeps_sum += r.sweeps;
        out->sweeps_max = std::max(out->sweeps_max, r.sweeps);
        out->n_access += r.n_access;
        out->n_sysval += r.n_sysval;
    }
    if (hipMemcpy(&ovf, B->P.counters + 1, sizeof(uint32_t), hipMemcpyDeviceToHost) == hipSuccess)
        out->n_overflow = ovf;
    /* records read once, descriptors, outputs written once, per-kernel results */
    out->bytes_alg = 16ull * B->N + 32ull * B->K + 16ull * out->n_access + 8ull * out->n_sysval + 32ull * B->K;
    if (B->have_events && B->runs) {
        dc_timing_t t;
        if (dc_get_timing(B, &t) == DC_OK && t.runs) {
            out->ms_total = t.ms_total / t.runs;
            out->ms_decode = t.ms_decode / t.runs;
            out->ms_cfg = t.ms_cfg / t.runs;
            out->ms_fixpoint = t.ms_fixpoint / t.runs;
            out->ms_compact = t.ms_compact / t.runs;
        }
    }
    return DC_OK;
}

extern "C" dc_status_t dc_timing_reset(dc_batch_t *B) {
    if (!B) return DC_E_INVAL;
    B->runs_at_reset = B->runs;
    return DC_OK;
}

extern "C" dc_status_t dc_get_timing(const dc_batch_t *cb, dc_timing_t *out) {
    dc_batch *B = const_cast<dc_batch *>(cb);
    if (!B || !out) return DC_E_INVAL;
    memset(out, 0, sizeof(*out));
    if (!B->have_events) return DC_E_NOTREADY;
    dc_status_t st = dc_batch_wait(B);
    if (st != DC_OK) return st;
    uint64_t first = B->runs_at_reset;
    if (B->runs - first > (uint64_t)TIMING_RING) first = B->runs - TIMING_RING;
    for (uint64_t r = first; r < B->runs; r++) {
        hipEvent_t *ev = B->ev[r % TIMING_RING];
        float a = 0, b = 0, c = 0, d = 0, e = 0;
        if (hipEventElapsedTime(&a, ev[EV_START], ev[EV_END]) != hipSuccess ||
            hipEventElapsedTime(&b, ev[EV_START], ev[EV_DECODE]) != hipSuccess ||
            hipEventElapsedTime(&c, ev[EV_DECODE], ev[EV_CFG]) != hipSuccess ||
            hipEventElapsedTime(&d, ev[EV_FIXB], ev[EV_FIX]) != hipSuccess ||
            hipEventElapsedTime(&e, ev[EV_FIX], ev[EV_END]) != hipSuccess)
            return DC_E_HIP;
        out->ms_total += a;
        out->ms_decode += b;
        out->ms_cfg += c;
        out->ms_fixpoint += d;
        out->ms_compact += e;
        out->runs++;
    }
    return DC_OK;
}

extern "C" void dc_batch_free(dc_batch_t *B) {
    if (!B) return;
    hipSetDevice(B->ctx->device);
    hipStreamSynchronize(B->stream);
    if (B->have_events)
        for (int r = 0; r < TIMING_RING; r++)
            for (int i = 0; i < N_EV; i++) hipEventDestroy(B->ev[r][i]);
    if (B->graph) hipGraphExecDestroy(B->graph);
    delete B;
}

/* ---------------------------------------------------------------- CFG only */
extern "C" dc_status_t dc_build_cfg(dc_ctx_t *ctx, const dc_kernel_t *kernels, uint32_t n_kernels,
                                    const dc_instr_t *instrs, uint64_t n_records, void *stream, dc_cfg_t **out) {
    if (!out) return DC_E_INVAL;
    *out = nullptr;
    dc_cfg *C = new (std::nothrow) dc_cfg;
    if (!C) return DC_E_OOM;
    dc_batch *B = &C->b;
    /* argument tables play no part in the graph: plan without them, then
     * restore the descriptor verdicts of the real descriptors */
    std::vector<dc_kernel_t> ks_noargs(kernels, kernels + (kernels ? n_kernels : 0));
    for (auto &k : ks_noargs) {
        k.n_args = 0;
        k.arg_begin = 0;
    }
    dc_status_t st = plan_batch(B, ctx, kernels ? ks_noargs.data() : nullptr, n_kernels, instrs, n_records, nullptr, 0,
                                nullptr, stream, true);
    if (st == DC_OK) {
        std::vector<int32_t> ds(n_kernels);
        for (uint32_t k = 0; k < n_kernels; k++) ds[k] = descriptor_status(kernels[k]);
        if (n_kernels &&
            hipMemcpy((void *)B->P.desc_status, ds.data(), n_kernels * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess)
            st = DC_E_HIP;
    }
    if (st == DC_OK) st = enqueue(B);
    if (st != DC_OK) {
        hipStreamSynchronize(B->stream);
        delete C;
        return st;
    }
    *out = C;
    return DC_OK;
}

static dc_status_t fetch_cfg(dc_batch *B) {
    if (B->host_valid) return DC_OK;
    if (hipStreamSynchronize(B->stream) != hipSuccess) return DC_E_HIP;
    const Plan &P = B->P;
    const uint32_t K = B->K;
    uint32_t total = 0;
    hipError_t e = hipMemcpy(&total, P.totals, sizeof(uint32_t), hipMemcpyDeviceToHost);
    B->k_status.resize(K);
    B->k_nblocks.resize(K);
    B->k_nreach.resize(K);
    B->first_block.resize(K);
    B->h_block_start.resize((size_t)total + 1);
    B->h_succ.resize(2 * (size_t)total);
    B->h_pred_off.resize((size_t)total + 1);
    B->h_rpo.resize(total);
    if (e == hipSuccess && K) e = hipMemcpy(B->k_status.data(), P.status, K * 4, hipMemcpyDeviceToHost);
    if (e == hipSuccess && K) e = hipMemcpy(B->k_nblocks.data(), P.n_blocks, K * 4, hipMemcpyDeviceToHost);
    if (e == hipSuccess && K) e = hipMemcpy(B->k_nreach.data(), P.n_reach, K * 4, hipMemcpyDeviceToHost);
    if (e == hipSuccess && K) e = hipMemcpy(B->first_block.data(), P.first_block, K * 4, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(B->h_block_start.data(), P.block_start, ((size_t)total + 1) * 4, hipMemcpyDeviceToHost);
    if (e == hipSuccess && total) e = hipMemcpy(B->h_succ.data(), P.succ, (size_t)total * 8, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(B->h_pred_off.data(), P.pred_cnt, ((size_t)total + 1) * 4, hipMemcpyDeviceToHost);
    if (e == hipSuccess && total) e = hipMemcpy(B->h_rpo.data(), P.rpo, (size_t)total * 4, hipMemcpyDeviceToHost);
    const uint32_t npred = total ? B->h_pred_off[total] : 0;
    B->h_pred.resize(npred);
    if (e == hipSuccess && npred) e = hipMemcpy(B->h_pred.data(), P.pred, (size_t)npred * 4, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e);
    B->host_valid = true;
    return DC_OK;
}

extern "C" dc_status_t dc_cfg_view(dc_cfg_t *C, uint32_t k, dc_cfg_view_t *v) {
    if (!C || !v || k >= C->b.K) return DC_E_INVAL;
    dc_batch *B = &C->b;
    dc_status_t st = fetch_cfg(B);
    if (st != DC_OK) return st;
    memset(v, 0, sizeof(*v));
    v->status = B->k_status[k];
    if (v->status != DC_OK) return DC_OK;
    const uint32_t fb = B->first_block[k], nb = B->k_nblocks[k], pb = B->pos_begin[k];
    B->v_block_start.resize((size_t)nb + 1);
    B->v_pred_off.resize((size_t)nb + 1);
    for (uint32_t b = 0; b <= nb; b++) {
        B->v_block_start[b] = B->h_block_start[fb + b] - pb;
        B->v_pred_off[b] = B->h_pred_off[fb + b] - B->h_pred_off[fb];
    }
    v->n_blocks = nb;
    v->n_reach = B->k_nreach[k];
    v->n_pred = B->v_pred_off[nb];
    v->block_start = B->v_block_start.data();
    v->succ = B->h_succ.data() + 2 * (size_t)fb;
    v->pred_off = B->v_pred_off.data();
    v->pred = B->h_pred.data() + B->h_pred_off[fb];
    v->rpo = B->h_rpo.data() + fb;
    return DC_OK;
}

extern "C" void dc_cfg_free(dc_cfg_t *C) {
    if (!C) return;
    hipSetDevice(C->b.ctx->device);
    hipStreamSynchronize(C->b.stream);
    delete C;
}

/* ---------------------------------------------------------------- register versions */
struct dc_ssa {
    dc_cfg c;
    DevMem smem;   /* per-block arrays, tables and outputs, sized by the first run on these records */
    SsaPlan S{};
    bool types = false;          /* made by dc_build_types: the variable and type stage follows */
    bool sized = false;
    bool host_valid = false;     /* results, offsets and first blocks copied since the last run */
    bool arrays_valid = false;   /* dominators, merges, arguments and versions copied since the last run */
    std::vector<dc_ssa_result_t> res;
    std::vector<uint64_t> offs;
    std::vector<uint32_t> first_block, idom, args, vers;
    std::vector<dc_phi_t> phis;
    std::vector<uint8_t> opn;
};

/* Enqueue the version stages after the graph stages.  The first run on a
 * set of records sizes the tables and then the outputs from the counts it
 * reads back (two waits for the stream); later runs reuse them. */
static dc_status_t enqueue_ssa_stages(void *arg) {
    dc_ssa *X = static_cast<dc_ssa *>(arg);
    dc_batch *B = &X->c.b;
    const Plan &P = B->P;
    SsaPlan &S = X->S;
    hipStream_t s = B->stream;
    const uint32_t K = B->K;
    X->host_valid = false;
    hipError_t e = hipSuccess;
    auto total = [&](uint32_t a, uint64_t *out) {
        if (e == hipSuccess)
            e = hipMemcpyAsync(out, S.offs + (uint64_t)a * (K + 1) + K, sizeof(uint64_t), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
    };
    if (!X->sized) {
        X->smem.reset();
        const uint64_t blocks = std::max<uint32_t>(P.blk_cap, 1);
        S.idom = X->smem.alloc<uint32_t>(blocks);
        S.scr = X->smem.alloc<uint32_t>(3 * blocks);
        S.opn = X->smem.alloc<uint8_t>(std::max<uint64_t>(B->N, 1));
        S.tab_a = S.tab_b = nullptr;
        S.phis = nullptr;
        S.phi_args = S.vers = nullptr;
        S.tab_cap = S.phi_cap = S.arg_cap = S.ops_cap = 0;
        S.aoff = S.tscr = nullptr;
        S.vars = nullptr;
        S.col_cap = S.node_cap = S.scr_cap = 0;
        /* non-null marks the type stages in the graph stage (sized below) */
        S.nver = X->types ? X->smem.alloc<uint32_t>(1) : nullptr;
        if (X->smem.failed) return DC_E_OOM;
        e = launch_ssa_size(P, S, s);
        uint64_t words = 0, cols = 0;
        if (K) total(0, &words);
        if (K && X->types) total(4, &cols);
        if (e != hipSuccess) return hip_fail(e);
        S.tab_a = X->smem.alloc<uint32_t>(words);
        S.tab_b = X->smem.alloc<uint32_t>(words);
        S.tab_cap = words;
        if (X->types) {
            S.nver = X->smem.alloc<uint32_t>(cols);
            S.col_cap = cols;
        }
        if (X->smem.failed) return DC_E_OOM;
        e = launch_ssa_graph(P, S, s);
        uint64_t t[6] = {0, 0, 0, 0, 0, 0};
        for (uint32_t a = 1; a <= (X->types ? 6u : 3u) && K; a++)
            if (a != 4) total(a, &t[a - 1]);
        if (e != hipSuccess) return hip_fail(e);
        S.phis = X->smem.alloc<dc_phi_t>(t[0]);
        S.phi_args = X->smem.alloc<uint32_t>(t[1]);
        S.vers = X->smem.alloc<uint32_t>(t[2]);
        S.phi_cap = t[0];
        S.arg_cap = t[1];
        S.ops_cap = t[2];
        if (X->types) {
            S.aoff = X->smem.alloc<uint32_t>(t[0]);
            S.vars = X->smem.alloc<dc_var_t>(t[4]);
            S.tscr = X->smem.alloc<uint32_t>(3 * t[5]);
            S.node_cap = t[4];
            S.scr_cap = t[5];
        }
        if (X->smem.failed) return DC_E_OOM;
        X->sized = true;
    } else {
        e = launch_ssa_size(P, S, s);
        if (e == hipSuccess) e = launch_ssa_graph(P, S, s);
        if (e != hipSuccess) return hip_fail(e);
    }
    e = launch_ssa_emit(P, S, s);
    return e == hipSuccess ? DC_OK : hip_fail(e);
}

/* the variable and type stage, after the versions */
static dc_status_t enqueue_types_stage(void *arg) {
    dc_ssa *X = static_cast<dc_ssa *>(arg);
    const hipError_t e = launch_types(X->c.b.P, X->S, X->c.b.stream);
    return e == hipSuccess ? DC_OK : hip_fail(e);
}

static dc_status_t build_ssa(dc_ctx_t *ctx, const dc_kernel_t *kernels, uint32_t n_kernels, const dc_instr_t *instrs,
                             uint64_t n_records, const dc_arg_t *args, uint64_t n_args, const dc_options_t *opts,
                             void *stream, bool types, dc_ssa_t **out) {
    if (!out) return DC_E_INVAL;
    *out = nullptr;
    if (opts && (opts->flags & ~(DC_OPT_TIMING | DC_OPT_DIGEST))) return DC_E_INVAL;
    dc_ssa *X = new (std::nothrow) dc_ssa;
    if (!X) return DC_E_OOM;
    X->S.digest = opts && (opts->flags & DC_OPT_DIGEST) ? 1u : 0u;
    X->types = types;
    dc_batch *B = &X->c.b;
    /* the graph plan, as dc_build_cfg makes it, plus the per-kernel bitmaps of
     * the register slots the records name and the per-kernel version arrays;
     * the argument tables only where the types read them */
    std::vector<dc_kernel_t> ks_noargs(kernels, kernels + (kernels ? n_kernels : 0));
    if (!types)
        for (auto &k : ks_noargs) {
            k.n_args = 0;
            k.arg_begin = 0;
        }
    dc_options_t o{};
    if (opts) o.flags = opts->flags & DC_OPT_TIMING;
    dc_status_t st = plan_batch(B, ctx, kernels ? ks_noargs.data() : nullptr, n_kernels, instrs, n_records,
                                types ? args : nullptr, types ? n_args : 0, &o, stream, true);
    if (st == DC_OK) {
        const uint64_t K = n_kernels;
        B->P.kslots = B->mem.alloc<uint32_t>(std::max<uint64_t>(K, 1) * KSLOT_WORDS);
        X->S.counts = B->mem.alloc<uint32_t>(SSA_ARRAYS * std::max<uint64_t>(K, 1));
        X->S.offs = B->mem.alloc<uint64_t>(SSA_ARRAYS * (K + 1));
        X->S.status = B->mem.alloc<int32_t>(std::max<uint64_t>(K, 1));
        X->S.res = B->mem.alloc<dc_ssa_result_t>(std::max<uint64_t>(K, 1));
        if (types) X->S.tres = B->mem.alloc<dc_types_result_t>(std::max<uint64_t>(K, 1));
        if (B->mem.failed) st = DC_E_OOM;
    }
    if (st == DC_OK) {
        std::vector<int32_t> ds(n_kernels);
        for (uint32_t k = 0; k < n_kernels; k++) ds[k] = descriptor_status(kernels[k]);
        if (n_kernels &&
            hipMemcpy((void *)B->P.desc_status, ds.data(), n_kernels * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess)
            st = DC_E_HIP;
        if (st == DC_OK && hipMemcpy(B->dP, &B->P, sizeof(Plan), hipMemcpyHostToDevice) != hipSuccess) st = DC_E_HIP;
    }
    if (st == DC_OK) {
        B->after_graph = enqueue_ssa_stages;
        B->after_graph_arg = X;
        if (types) B->after_fix = enqueue_types_stage;
        st = enqueue(B);
    }
    if (st != DC_OK) {
        hipStreamSynchronize(B->stream);
        delete X;
        return st;
    }
    *out = X;
    return DC_OK;
}

extern "C" dc_status_t dc_build_ssa(dc_ctx_t *ctx, const dc_kernel_t *kernels, uint32_t n_kernels,
                                    const dc_instr_t *instrs, uint64_t n_records, const dc_options_t *opts,
                                    void *stream, dc_ssa_t **out) {
    return build_ssa(ctx, kernels, n_kernels, instrs, n_records, nullptr, 0, opts, stream, false, out);
}

extern "C" dc_status_t dc_build_types(dc_ctx_t *ctx, const dc_kernel_t *kernels, uint32_t n_kernels,
                                      const dc_instr_t *instrs, uint64_t n_records, const dc_arg_t *args,
                                      uint64_t n_args, const dc_options_t *opts, void *stream, dc_ssa_t **out) {
    return build_ssa(ctx, kernels, n_kernels, instrs, n_records, args, n_args, opts, stream, true, out);
}

extern "C" dc_status_t dc_ssa_run(dc_ssa_t *X, const dc_instr_t *instrs) {
    if (!X || (X->c.b.n_records && !instrs)) return DC_E_INVAL;
    dc_batch *B = &X->c.b;
    if (hipSetDevice(B->ctx->device) != hipSuccess) return DC_E_HIP;
    if (instrs != B->P.instrs) {
        /* other records: plan the blocks and the version arrays again */
        if (hipStreamSynchronize(B->stream) != hipSuccess) return DC_E_HIP;
        B->P.instrs = instrs;
        B->blocks_planned = false;
        X->sized = false;
    }
    return enqueue(B);
}

extern "C" dc_status_t dc_ssa_wait(dc_ssa_t *X) {
    if (!X) return DC_E_INVAL;
    return dc_batch_wait(&X->c.b);
}

static dc_status_t fetch_ssa(dc_ssa *X) {
    if (X->host_valid) return DC_OK;
    dc_batch *B = &X->c.b;
    dc_status_t st = dc_batch_wait(B);
    if (st != DC_OK) return st;
    const uint32_t K = B->K;
    const SsaPlan &S = X->S;
    X->res.resize(K);
    X->offs.resize(SSA_ARRAYS * ((size_t)K + 1));
    X->first_block.resize(K);
    hipError_t e = hipSuccess;
    if (K) e = hipMemcpy(X->res.data(), S.res, K * sizeof(dc_ssa_result_t), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(X->offs.data(), S.offs, X->offs.size() * sizeof(uint64_t), hipMemcpyDeviceToHost);
    if (e == hipSuccess && K)
        e = hipMemcpy(X->first_block.data(), B->P.first_block, K * sizeof(uint32_t), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e);
    X->host_valid = true;
    X->arrays_valid = false;
    return DC_OK;
}

/* the graph's dominators, the merges, their arguments and the operand
 * versions, copied on first use after a run */
static dc_status_t fetch_ssa_arrays(dc_ssa *X) {
    dc_status_t st = fetch_ssa(X);
    if (st != DC_OK || X->arrays_valid) return st;
    dc_batch *B = &X->c.b;
    const uint32_t K = B->K;
    const SsaPlan &S = X->S;
    hipError_t e = hipSuccess;
    const uint64_t nblk = B->P.blk_cap, np = X->offs[2 * ((size_t)K + 1) - 1], na = X->offs[3 * ((size_t)K + 1) - 1],
                   no = X->offs[4 * ((size_t)K + 1) - 1];
    X->idom.resize(nblk);
    X->phis.resize(std::min<uint64_t>(np, S.phi_cap));
    X->args.resize(std::min<uint64_t>(na, S.arg_cap));
    X->vers.resize(std::min<uint64_t>(no, S.ops_cap));
    X->opn.resize(B->N);
    if (nblk) e = hipMemcpy(X->idom.data(), S.idom, nblk * sizeof(uint32_t), hipMemcpyDeviceToHost);
    if (e == hipSuccess && !X->phis.empty())
        e = hipMemcpy(X->phis.data(), S.phis, X->phis.size() * sizeof(dc_phi_t), hipMemcpyDeviceToHost);
    if (e == hipSuccess && !X->args.empty())
        e = hipMemcpy(X->args.data(), S.phi_args, X->args.size() * sizeof(uint32_t), hipMemcpyDeviceToHost);
    if (e == hipSuccess && !X->vers.empty())
        e = hipMemcpy(X->vers.data(), S.vers, X->vers.size() * sizeof(uint32_t), hipMemcpyDeviceToHost);
    if (e == hipSuccess && B->N) e = hipMemcpy(X->opn.data(), S.opn, B->N, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e);
    X->arrays_valid = true;
    return DC_OK;
}

extern "C" dc_status_t dc_ssa_get_results(dc_ssa_t *X, dc_ssa_result_t *out, uint32_t cap) {
    if (!X || (cap && !out)) return DC_E_INVAL;
    dc_status_t st = fetch_ssa(X);
    if (st != DC_OK) return st;
    const uint32_t n = std::min<uint32_t>(cap, X->c.b.K);
    if (n) memcpy(out, X->res.data(), n * sizeof(dc_ssa_result_t));
    return DC_OK;
}

/* kernel k's slice [lo, hi) of count array a, when the kernel succeeded */
static bool ssa_slice(dc_ssa *X, uint32_t k, uint32_t a, uint64_t *lo, uint64_t *hi) {
    const uint32_t K = X->c.b.K;
    *lo = *hi = 0;
    if (X->res[k].status != DC_OK) return false;
    *lo = X->offs[(size_t)a * (K + 1) + k];
    *hi = X->offs[(size_t)a * (K + 1) + k + 1];
    return true;
}

extern "C" dc_status_t dc_ssa_get_idom(dc_ssa_t *X, uint32_t k, uint32_t *buf, uint32_t cap, uint32_t *n_total) {
    if (!X || !n_total || (cap && !buf) || k >= X->c.b.K) return DC_E_INVAL;
    dc_status_t st = fetch_ssa_arrays(X);
    if (st != DC_OK) return st;
    const uint32_t nb = X->res[k].status == DC_OK ? X->res[k].n_blocks : 0;
    *n_total = nb;
    if (std::min(cap, nb)) memcpy(buf, X->idom.data() + X->first_block[k], std::min(cap, nb) * sizeof(uint32_t));
    return DC_OK;
}

extern "C" dc_status_t dc_ssa_get_phis(dc_ssa_t *X, uint32_t k, dc_phi_t *buf, uint32_t cap, uint32_t *n_total) {
    if (!X || !n_total || (cap && !buf) || k >= X->c.b.K) return DC_E_INVAL;
    dc_status_t st = fetch_ssa_arrays(X);
    if (st != DC_OK) return st;
    uint64_t lo, hi;
    ssa_slice(X, k, 1, &lo, &hi);
    *n_total = (uint32_t)(hi - lo);
    if (std::min<uint64_t>(cap, hi - lo)) memcpy(buf, X->phis.data() + lo, std::min<uint64_t>(cap, hi - lo) * sizeof(dc_phi_t));
    return DC_OK;
}

extern "C" dc_status_t dc_ssa_get_phi_args(dc_ssa_t *X, uint32_t k, uint32_t *buf, uint32_t cap, uint32_t *n_total) {
    if (!X || !n_total || (cap && !buf) || k >= X->c.b.K) return DC_E_INVAL;
    dc_status_t st = fetch_ssa_arrays(X);
    if (st != DC_OK) return st;
    uint64_t lo, hi;
    ssa_slice(X, k, 2, &lo, &hi);
    *n_total = (uint32_t)(hi - lo);
    if (std::min<uint64_t>(cap, hi - lo)) memcpy(buf, X->args.data() + lo, std::min<uint64_t>(cap, hi - lo) * sizeof(uint32_t));
    return DC_OK;
}

extern "C" dc_status_t dc_ssa_get_versions(dc_ssa_t *X, uint32_t k, uint32_t *use_ver, uint32_t *def_ver,
                                           uint32_t cap_instr, uint32_t *n_instr) {
    if (!X || !n_instr || k >= X->c.b.K) return DC_E_INVAL;
    dc_status_t st = fetch_ssa_arrays(X);
    if (st != DC_OK) return st;
    dc_batch *B = &X->c.b;
    const uint32_t n = B->kernels[k].n_instr, m = std::min(cap_instr, n);
    *n_instr = n;
    if (use_ver)
        for (uint64_t i = 0; i < (uint64_t)m * DC_SSA_NU; i++) use_ver[i] = DC_SSA_NONE;
    if (def_ver)
        for (uint64_t i = 0; i < (uint64_t)m * DC_SSA_ND; i++) def_ver[i] = DC_SSA_NONE;
    uint64_t lo, hi;
    if (!ssa_slice(X, k, 3, &lo, &hi)) return DC_OK;
    const uint32_t pb = B->pos_begin[k];
    uint64_t o = lo;
    for (uint32_t i = 0; i < m; i++) {
        const uint32_t nu = X->opn[pb + i] & 15u, nd = X->opn[pb + i] >> 4;
        if (o + nu + nd > hi || nu > DC_SSA_NU || nd > DC_SSA_ND) return DC_E_HIP;
        for (uint32_t q = 0; q < nu; q++)
            if (use_ver) use_ver[(uint64_t)i * DC_SSA_NU + q] = X->vers[o + q];
        for (uint32_t q = 0; q < nd; q++)
            if (def_ver) def_ver[(uint64_t)i * DC_SSA_ND + q] = X->vers[o + nu + q];
        o += nu + nd;
    }
    return DC_OK;
}

extern "C" dc_status_t dc_ssa_get_timing(dc_ssa_t *X, dc_timing_t *out) {
    if (!X) return DC_E_INVAL;
    dc_status_t st = dc_get_timing(&X->c.b, out);
    if (st == DC_OK && !X->types) out->ms_compact = 0;
    return st;
}

extern "C" dc_status_t dc_types_get_results(dc_ssa_t *X, dc_types_result_t *out, uint32_t cap) {
    if (!X || !X->types || (cap && !out)) return DC_E_INVAL;
    dc_batch *B = &X->c.b;
    dc_status_t st = dc_batch_wait(B);
    if (st != DC_OK) return st;
    const uint32_t n = std::min<uint32_t>(cap, B->K);
    if (n && hipMemcpy(out, X->S.tres, n * sizeof(dc_types_result_t), hipMemcpyDeviceToHost) != hipSuccess)
        return DC_E_HIP;
    return DC_OK;
}

extern "C" dc_status_t dc_types_get_vars(dc_ssa_t *X, uint32_t k, dc_var_t *buf, uint32_t cap, uint32_t *n_total) {
    if (!X || !X->types || !n_total || (cap && !buf) || k >= X->c.b.K) return DC_E_INVAL;
    dc_status_t st = fetch_ssa(X);
    if (st != DC_OK) return st;
    dc_types_result_t r;
    if (hipMemcpy(&r, X->S.tres + k, sizeof(r), hipMemcpyDeviceToHost) != hipSuccess) return DC_E_HIP;
    const uint32_t K = X->c.b.K;
    const uint32_t nn = r.status == DC_OK ? r.n_nodes : 0;
    *n_total = nn;
    const uint32_t m = std::min(cap, nn);
    if (m && hipMemcpy(buf, X->S.vars + X->offs[5 * ((size_t)K + 1) + k], m * sizeof(dc_var_t),
                       hipMemcpyDeviceToHost) != hipSuccess)
        return DC_E_HIP;
    return DC_OK;
}

extern "C" dc_status_t dc_ssa_timing_reset(dc_ssa_t *X) {
    if (!X) return DC_E_INVAL;
    return dc_timing_reset(&X->c.b);
}

extern "C" void dc_ssa_free(dc_ssa_t *X) {
    if (!X) return;
    hipSetDevice(X->c.b.ctx->device);
    hipStreamSynchronize(X->c.b.stream);
    dc_batch *B = &X->c.b;
    if (B->have_events)
        for (int r = 0; r < TIMING_RING; r++)
            for (int i = 0; i < N_EV; i++) hipEventDestroy(B->ev[r][i]);
    delete X;
}

/* ---------------------------------------------------------------- structuring */
struct dc_struct {
    dc_cfg c;
    DevMem smem;   /* region arrays, sized by the block count of the first run on these records */
    StructPlan S{};
    bool sized = false;
    bool host_valid = false, merges_valid = false;
    std::vector<dc_struct_result_t> res;
    std::vector<dc_merge_t> merges;
    std::vector<uint32_t> first_block;
};

static dc_status_t enqueue_struct_stages(void *arg) {
    dc_struct *X = static_cast<dc_struct *>(arg);
    dc_batch *B = &X->c.b;
    const Plan &P = B->P;
    StructPlan &S = X->S;
    X->host_valid = false;
    if (!X->sized) {
        X->smem.reset();
        const uint64_t slots = 4ull * std::max<uint32_t>(P.blk_cap, 1) + 2ull * B->K;
        S.succ = X->smem.alloc<int32_t>(2 * slots);
        S.npred = X->smem.alloc<uint32_t>(slots);
        S.fwd = X->smem.alloc<uint32_t>(slots);
        S.mark = X->smem.alloc<uint32_t>(slots);
        S.stack = X->smem.alloc<uint32_t>(2 * slots);
        S.merges = X->smem.alloc<dc_merge_t>(slots);
        if (X->smem.failed) return DC_E_OOM;
        X->sized = true;
    }
    const hipError_t e = launch_struct(P, S, B->stream);
    return e == hipSuccess ? DC_OK : hip_fail(e);
}

extern "C" dc_status_t dc_structure(dc_ctx_t *ctx, const dc_kernel_t *kernels, uint32_t n_kernels,
                                    const dc_instr_t *instrs, uint64_t n_records, const dc_options_t *opts,
                                    void *stream, dc_struct_t **out) {
    if (!out) return DC_E_INVAL;
    *out = nullptr;
    if (opts && (opts->flags & ~DC_OPT_TIMING)) return DC_E_INVAL;
    dc_struct *X = new (std::nothrow) dc_struct;
    if (!X) return DC_E_OOM;
    dc_batch *B = &X->c.b;
    std::vector<dc_kernel_t> ks_noargs(kernels, kernels + (kernels ? n_kernels : 0));
    for (auto &k : ks_noargs) {
        k.n_args = 0;
        k.arg_begin = 0;
    }
    dc_options_t o{};
    if (opts) o.flags = opts->flags;
    dc_status_t st = plan_batch(B, ctx, kernels ? ks_noargs.data() : nullptr, n_kernels, instrs, n_records, nullptr, 0,
                                &o, stream, true);
    if (st == DC_OK) {
        X->S.res = B->mem.alloc<dc_struct_result_t>(std::max<uint64_t>(n_kernels, 1));
        if (B->mem.failed) st = DC_E_OOM;
    }
    if (st == DC_OK) {
        std::vector<int32_t> ds(n_kernels);
        for (uint32_t k = 0; k < n_kernels; k++) ds[k] = descriptor_status(kernels[k]);
        if (n_kernels &&
            hipMemcpy((void *)B->P.desc_status, ds.data(), n_kernels * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess)
            st = DC_E_HIP;
    }
    if (st == DC_OK) {
        B->after_graph = enqueue_struct_stages;
        B->after_graph_arg = X;
        st = enqueue(B);
    }
    if (st != DC_OK) {
        hipStreamSynchronize(B->stream);
        delete X;
        return st;
    }
    *out = X;
    return DC_OK;
}

extern "C" dc_status_t dc_struct_run(dc_struct_t *X, const dc_instr_t *instrs) {
    if (!X || (X->c.b.n_records && !instrs)) return DC_E_INVAL;
    dc_batch *B = &X->c.b;
    if (hipSetDevice(B->ctx->device) != hipSuccess) return DC_E_HIP;
    if (instrs != B->P.instrs) {
        if (hipStreamSynchronize(B->stream) != hipSuccess) return DC_E_HIP;
        B->P.instrs = instrs;
        B->blocks_planned = false;
        X->sized = false;
    }
    return enqueue(B);
}

extern "C" dc_status_t dc_struct_wait(dc_struct_t *X) {
    if (!X) return DC_E_INVAL;
    return dc_batch_wait(&X->c.b);
}

static dc_status_t fetch_struct(dc_struct *X) {
    if (X->host_valid) return DC_OK;
    dc_batch *B = &X->c.b;
    dc_status_t st = dc_batch_wait(B);
    if (st != DC_OK) return st;
    const uint32_t K = B->K;
    X->res.resize(K);
    X->first_block.resize(K);
    hipError_t e = hipSuccess;
    if (K) e = hipMemcpy(X->res.data(), X->S.res, K * sizeof(dc_struct_result_t), hipMemcpyDeviceToHost);
    if (e == hipSuccess && K)
        e = hipMemcpy(X->first_block.data(), B->P.first_block, K * sizeof(uint32_t), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e);
    X->host_valid = true;
    X->merges_valid = false;
    return DC_OK;
}

/* the merge records, copied on first use after a run */
static dc_status_t fetch_struct_merges(dc_struct *X) {
    dc_status_t st = fetch_struct(X);
    if (st != DC_OK || X->merges_valid) return st;
    const uint64_t slots = 4ull * std::max<uint32_t>(X->c.b.P.blk_cap, 1) + 2ull * X->c.b.K;
    X->merges.resize(slots);
    if (X->S.merges &&
        hipMemcpy(X->merges.data(), X->S.merges, slots * sizeof(dc_merge_t), hipMemcpyDeviceToHost) != hipSuccess)
        return DC_E_HIP;
    X->merges_valid = true;
    return DC_OK;
}

extern "C" dc_status_t dc_struct_get_results(dc_struct_t *X, dc_struct_result_t *out, uint32_t cap) {
    if (!X || (cap && !out)) return DC_E_INVAL;
    dc_status_t st = fetch_struct(X);
    if (st != DC_OK) return st;
    const uint32_t n = std::min<uint32_t>(cap, X->c.b.K);
    if (n) memcpy(out, X->res.data(), n * sizeof(dc_struct_result_t));
    return DC_OK;
}

extern "C" dc_status_t dc_struct_get_merges(dc_struct_t *X, uint32_t k, dc_merge_t *buf, uint32_t cap,
                                            uint32_t *n_total) {
    if (!X || !n_total || (cap && !buf) || k >= X->c.b.K) return DC_E_INVAL;
    dc_status_t st = fetch_struct_merges(X);
    if (st != DC_OK) return st;
    const dc_struct_result_t &r = X->res[k];
    *n_total = r.status == DC_OK ? r.n_merges : 0;
    const uint64_t base = 4ull * X->first_block[k] + 2ull * k;
    const uint32_t n = std::min(cap, *n_total);
    if (n) memcpy(buf, X->merges.data() + base, n * sizeof(dc_merge_t));
    return DC_OK;
}

extern "C" dc_status_t dc_struct_get_timing(dc_struct_t *X, dc_timing_t *out) {
    if (!X) return DC_E_INVAL;
    dc_status_t st = dc_get_timing(&X->c.b, out);
    if (st == DC_OK) out->ms_compact = 0;
    return st;
}

extern "C" dc_status_t dc_struct_timing_reset(dc_struct_t *X) {
    if (!X) return DC_E_INVAL;
    return dc_timing_reset(&X->c.b);
}

extern "C" void dc_struct_free(dc_struct_t *X) {
    if (!X) return;
    hipSetDevice(X->c.b.ctx->device);
    hipStreamSynchronize(X->c.b.stream);
    dc_batch *B = &X->c.b;
    if (B->have_events)
        for (int r = 0; r < TIMING_RING; r++)
            for (int i = 0; i < N_EV; i++) hipEventDestroy(B->ev[r][i]);
    delete X;
}
