/*
 * dc_server.cpp -- the request server of libdc (dc_server_* in include/dc.h):
 * continuous batching of single-kernel analysis requests.
 *
 * Requests are copied at submission into host queues.  A service thread
 * owns the lanes: each lane is a plan preallocated for a batch of up to
 * lane_instr instructions (device arrays, fixpoint arenas, pinned staging)
 * with its own stream.  The thread loops over three steps:
 *   1. a lane whose analysis event has fired gets its record counts; the
 *      exact record ranges are copied back behind a second event;
 *   2. a lane whose second event has fired publishes one result per request
 *      and becomes free;
 *   3. a free lane takes waiting requests of one length class (the class
 *      whose oldest request has waited longest, within the class's share of
 *      the lanes), packs them into its pinned staging and enqueues the copies
 *      and every stage of the analysis on its stream.
 * A batch returns when its longest kernel is done, and one kernel runs on
 * one wavefront, so requests are batched with others of similar length.
 * Lanes run concurrently on the device: a batch admitted while others run
 * overlaps with them.  Nothing is allocated per request on the device.
 */
#include <hip/hip_runtime_api.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "dc.h"
#include "dc_host.h"
#include "dc_internal.h"

using namespace dc;

namespace {

uint64_t now_ns() {
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct Req {
    uint64_t ticket = 0, tag = 0;
    dc_kernel_t kd{};
    std::vector<dc_instr_t> instrs;
    std::vector<dc_arg_t> args;
    uint64_t t_submit = 0, t_admit = 0;
};

struct Done {
    dc_result_t r{};
    std::vector<dc_access_t> acc;
    std::vector<dc_sysval_t> sys;
};

/* pinned host buffer; grown only while no copy into or out of it is pending */
template <typename T>
struct Pinned {
    T *p = nullptr;
    uint64_t cap = 0;
    hipError_t reserve(uint64_t n) {
        if (n <= cap && p) return hipSuccess;
        const uint64_t c = std::max<uint64_t>({n, cap * 2, 1});
        void *q = nullptr;
        hipError_t e = hipHostMalloc(&q, c * sizeof(T), hipHostMallocDefault);
        if (e != hipSuccess) return e;
        if (p) hipHostFree(p);
        p = static_cast<T *>(q);
        cap = c;
        return hipSuccess;
    }
    Pinned() = default;
    Pinned(const Pinned &) = delete;
    Pinned &operator=(const Pinned &) = delete;
    ~Pinned() {
        if (p) hipHostFree(p);
    }
};

enum LaneState { L_FREE, L_RUN, L_FETCH };

struct Lane {
    uint32_t id = 0;
    hipStream_t s = nullptr;
    DevMem mem;
    Plan P{};
    Plan *dP = nullptr;
    FixCfg fc{};
    PlanInputs in{};
    uint32_t groups_cap = 0;
    Pinned<dc_instr_t> h_instrs;
    Pinned<dc_kernel_t> h_k;
    Pinned<dc_arg_t> h_a;
    Pinned<uint32_t> h_pb;
    Pinned<int32_t> h_ds;
    Pinned<uint32_t> h_order;
    Pinned<Plan> h_plan;
    Pinned<dc_kernel_result_t> h_res;
    Pinned<uint32_t> h_acc_off, h_sys_off;
    Pinned<dc_access_t> h_acc;
    Pinned<dc_sysval_t> h_sys;
    hipEvent_t ev_run = nullptr, ev_fetch = nullptr;
    LaneState st = L_FREE;
    int cls = -1;   /* length class of the batch in flight */
    std::vector<std::unique_ptr<Req>> reqs;
    uint64_t batch = 0;
    uint64_t t_enqueued = 0, t_device = 0;
};

constexpr int N_CLASS = 4;   /* length classes: < L/16, < L/4, < L, the rest (L = long_instr) */
constexpr uint32_t LANE_ARENA_ROWS = 512;            /* main-pass rows per wave (256 blocks of two rows) */
constexpr uint64_t LANE_INSTR_MAX = 4ull << 20;      /* largest lane, in instructions */
constexpr uint64_t OVF_BUDGET_BYTES = 1ull << 30;    /* overflow arenas per lane */
constexpr uint64_t ROW_BYTES = FIX_ROW_DWORDS * 4ull;
/* device bytes per instruction of a lane's arrays: records, the
 * per-position arrays (leader, capacity, block id), the block-indexed arrays
 * for one block per instruction, one access and four built-in record slots
 * per instruction (alloc_plan, alloc_blocks), the capacity scan */
constexpr uint64_t BYTES_PER_INSTR = 16 + 1 + 1 + 4 + BLOCK_BYTES + ACC_SLOT_BYTES + 4 * SYS_SLOT_BYTES + 8;
constexpr uint64_t BYTES_PER_KERNEL = 32 + 255 * 8 + 4 + 4 + 4 + 4 + 4 + 4 + 4 + 4 + 32 + 4 + 4 + 8;

static_assert(sizeof(dc_request_t) == 56 && sizeof(dc_result_t) == 120, "server ABI layout");

}  // namespace

struct dc_server {
    dc_ctx *ctx = nullptr;
    dc_server_opts_t o{};
    uint64_t lane_instr = 0, lane_kernels = 0, lane_args = 0, ovf_rows_budget = 0, device_bytes = 0;
    uint32_t wpg = 1;
    std::vector<std::unique_ptr<Lane>> lanes;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<std::unique_ptr<Req>> q[N_CLASS];
    uint32_t class_lanes[N_CLASS] = {};   /* lanes a class may hold at once */
    std::deque<std::unique_ptr<Done>> done;
    std::vector<std::unique_ptr<Done>> delivered;
    uint64_t next_ticket = 1, next_batch = 1;
    uint64_t n_submitted = 0, n_completed = 0, n_batches = 0, max_batch = 0;
    bool stop = false;
    dc_status_t fault = DC_OK;
    std::thread th;
};

namespace {

int length_class(const dc_server *S, uint32_t n_instr) {
    const uint32_t L = S->o.long_instr;
    return n_instr < L / 16 ? 0 : n_instr < L / 4 ? 1 : n_instr < L ? 2 : 3;
}

/* the class whose oldest request waited longest among those below their
 * share of the lanes; -1 if none */
int pick_class(dc_server *S) {
    uint32_t busy[N_CLASS] = {};
    for (auto &L : S->lanes)
        if (L->st != L_FREE && L->cls >= 0) busy[L->cls]++;
    int best = -1;
    for (int c = 0; c < N_CLASS; c++) {
        if (S->q[c].empty() || busy[c] >= S->class_lanes[c]) continue;
        if (best < 0 || S->q[c].front()->t_submit < S->q[best].front()->t_submit) best = c;
    }
    return best;
}

uint64_t waiting(const dc_server *S) {
    uint64_t n = 0;
    for (const auto &q : S->q) n += q.size();
    return n;
}

void take_requests(dc_server *S, std::deque<std::unique_ptr<Req>> &q, std::vector<std::unique_ptr<Req>> &take) {
    uint64_t n = 0, a = 0;
    while (!q.empty() && take.size() < S->lane_kernels) {
        const Req &r = *q.front();
        if (!take.empty() && (n + r.kd.n_instr > S->lane_instr || a + r.args.size() > S->lane_args)) break;
        n += r.kd.n_instr;
        a += r.args.size();
        take.push_back(std::move(q.front()));
        q.pop_front();
    }
}

#define TRYH(x)                          \
    do {                                 \
        hipError_t e_ = (x);             \
        if (e_ != hipSuccess) return e_; \
    } while (0)

/* pack the requests into the lane and enqueue copies, stages and the first
 * copy-back */
hipError_t launch(dc_server *S, Lane &L) {
    const uint64_t t = now_ns();
    const uint32_t K = (uint32_t)L.reqs.size();
    uint64_t N = 0, A = 0;
    uint32_t maxlen = 1;
    for (uint32_t k = 0; k < K; k++) {
        Req &r = *L.reqs[k];
        r.t_admit = t;
        dc_kernel_t d = r.kd;
        d.instr_begin = N;
        d.arg_begin = (uint32_t)A;
        L.h_k.p[k] = d;
        L.h_pb.p[k] = (uint32_t)N;
        L.h_ds.p[k] = descriptor_status(d);
        if (r.instrs.size()) memcpy(L.h_instrs.p + N, r.instrs.data(), r.instrs.size() * sizeof(dc_instr_t));
        if (r.args.size()) memcpy(L.h_a.p + A, r.args.data(), r.args.size() * sizeof(dc_arg_t));
        N += r.instrs.size();
        A += r.args.size();
        maxlen = std::max<uint32_t>(maxlen, d.n_instr);
    }
    L.h_pb.p[K] = (uint32_t)N;
    /* the fixpoint takes the longest requests first */
    for (uint32_t k = 0; k < K; k++) L.h_order.p[k] = k;
    std::stable_sort(L.h_order.p, L.h_order.p + K,
                     [&](uint32_t a, uint32_t b) { return L.h_k.p[a].n_instr > L.h_k.p[b].n_instr; });
    Plan &P = L.P;
    P.n_kernels = K;
    P.n_pos = (uint32_t)N;
    P.n_records = N;
    P.n_args = A;
    /* overflow pass of this batch: a kernel has at most one block per
     * instruction, so the longest request bounds every block count */
    P.ovf_block_cap = maxlen;
    P.ovf_rows = maxlen * FIX_MAX_ROWS;
    P.ovf_waves = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(OVF_MAX_WAVES, S->ovf_rows_budget / P.ovf_rows));
    L.fc.waves_per_group = (int)S->wpg;
    L.fc.groups = (int)std::max<uint64_t>(1, std::min<uint64_t>(L.groups_cap, (K + S->wpg - 1) / S->wpg));
    *L.h_plan.p = P;
    hipStream_t s = L.s;
    if (N) TRYH(hipMemcpyAsync(const_cast<dc_instr_t *>(P.instrs), L.h_instrs.p, N * sizeof(dc_instr_t),
                               hipMemcpyHostToDevice, s));
    TRYH(hipMemcpyAsync(L.in.kernels, L.h_k.p, K * sizeof(dc_kernel_t), hipMemcpyHostToDevice, s));
    if (A) TRYH(hipMemcpyAsync(L.in.args, L.h_a.p, A * sizeof(dc_arg_t), hipMemcpyHostToDevice, s));
    TRYH(hipMemcpyAsync(L.in.pos_begin, L.h_pb.p, (K + 1) * sizeof(uint32_t), hipMemcpyHostToDevice, s));
    TRYH(hipMemcpyAsync(L.in.desc_status, L.h_ds.p, K * sizeof(int32_t), hipMemcpyHostToDevice, s));
    TRYH(hipMemcpyAsync(L.in.work_order, L.h_order.p, K * sizeof(uint32_t), hipMemcpyHostToDevice, s));
    TRYH(hipMemcpyAsync(L.dP, L.h_plan.p, sizeof(Plan), hipMemcpyHostToDevice, s));
    TRYH(launch_fill_u8(P.leader, N, 0, s));
    TRYH(launch_fill_u32(P.kbad, K, 0xFFFFFFFFu, s));
    TRYH(launch_decode(P, s));
    TRYH(launch_leader_scan(P, s));
    TRYH(launch_number_blocks(P, s));
    TRYH(launch_edges(P, s));
    TRYH(launch_fixpoint(P, L.dP, L.fc, s, nullptr, nullptr));
    TRYH(launch_compact(P, s));
    TRYH(hipMemcpyAsync(L.h_res.p, P.results, K * sizeof(dc_kernel_result_t), hipMemcpyDeviceToHost, s));
    TRYH(hipMemcpyAsync(L.h_acc_off.p, P.acc_count, (K + 1) * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    TRYH(hipMemcpyAsync(L.h_sys_off.p, P.sys_count, (K + 1) * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    TRYH(hipEventRecord(L.ev_run, s));
    L.st = L_RUN;
    L.t_enqueued = now_ns();
    return hipSuccess;
}

/* the record counts are on the host: copy exactly the records back */
hipError_t fetch_records(Lane &L) {
    L.t_device = now_ns();
    const uint32_t K = (uint32_t)L.reqs.size();
    const uint64_t na = L.h_acc_off.p[K], ns = L.h_sys_off.p[K];
    TRYH(L.h_acc.reserve(na));
    TRYH(L.h_sys.reserve(ns));
    if (na) TRYH(hipMemcpyAsync(L.h_acc.p, L.P.acc_dense, na * sizeof(dc_access_t), hipMemcpyDeviceToHost, L.s));
    if (ns) TRYH(hipMemcpyAsync(L.h_sys.p, L.P.sys_dense, ns * sizeof(dc_sysval_t), hipMemcpyDeviceToHost, L.s));
    TRYH(hipEventRecord(L.ev_fetch, L.s));
    L.st = L_FETCH;
    return hipSuccess;
}
#undef TRYH

/* one result per request of the lane; `failed` marks them DC_E_HIP */
void publish(dc_server *S, Lane &L, bool failed) {
    const uint64_t t = now_ns();
    const uint32_t K = (uint32_t)L.reqs.size();
    std::vector<std::unique_ptr<Done>> out;
    out.reserve(K);
    for (uint32_t k = 0; k < K; k++) {
        const Req &q = *L.reqs[k];
        std::unique_ptr<Done> d(new Done);
        d->r.ticket = q.ticket;
        d->r.tag = q.tag;
        d->r.t_submit_ns = q.t_submit;
        d->r.t_admit_ns = q.t_admit;
        d->r.t_enqueued_ns = L.t_enqueued;
        d->r.t_device_ns = L.t_device;
        d->r.t_done_ns = t;
        d->r.batch = L.batch;
        d->r.batch_kernels = K;
        d->r.lane = L.id;
        if (failed) {
            d->r.summary.status = DC_E_HIP;
        } else {
            d->r.summary = L.h_res.p[k];
            const uint32_t a0 = L.h_acc_off.p[k], a1 = L.h_acc_off.p[k + 1];
            const uint32_t s0 = L.h_sys_off.p[k], s1 = L.h_sys_off.p[k + 1];
            d->acc.assign(L.h_acc.p + a0, L.h_acc.p + a1);
            d->sys.assign(L.h_sys.p + s0, L.h_sys.p + s1);
        }
        out.push_back(std::move(d));
    }
    {
        std::lock_guard<std::mutex> g(S->mu);
        for (auto &d : out) S->done.push_back(std::move(d));
        S->n_completed += K;
    }
    L.reqs.clear();
    L.st = L_FREE;
    L.cls = -1;
}

/* a HIP error: every request in flight or waiting fails, no more admission */
void fail_all(dc_server *S) {
    for (auto &L : S->lanes) {
        if (L->st == L_FREE) continue;
        hipStreamSynchronize(L->s);
        publish(S, *L, true);
    }
    std::lock_guard<std::mutex> g(S->mu);
    S->fault = DC_E_HIP;
    const uint64_t t = now_ns();
    for (auto *q = S->q; q != S->q + N_CLASS; q++) {
        while (!q->empty()) {
            std::unique_ptr<Done> d(new Done);
            d->r.ticket = q->front()->ticket;
            d->r.tag = q->front()->tag;
            d->r.t_submit_ns = q->front()->t_submit;
            d->r.t_done_ns = t;
            d->r.summary.status = DC_E_HIP;
            S->done.push_back(std::move(d));
            S->n_completed++;
            q->pop_front();
        }
    }
}

void service(dc_server *S) {
    hipSetDevice(S->ctx->device);
    for (;;) {
        bool progress = false, error = false;
        for (auto &L : S->lanes) {
            if (L->st == L_RUN) {
                const hipError_t q = hipEventQuery(L->ev_run);
                if (q == hipErrorNotReady) continue;
                if (q != hipSuccess || fetch_records(*L) != hipSuccess) {
                    error = true;
                    break;
                }
                progress = true;
            }
            if (L->st == L_FETCH) {
                const hipError_t q = hipEventQuery(L->ev_fetch);
                if (q == hipErrorNotReady) continue;
                if (q != hipSuccess) {
                    error = true;
                    break;
                }
                publish(S, *L, false);
                progress = true;
            }
        }
        if (error) {
            fail_all(S);
            progress = true;
        }
        for (auto &L : S->lanes) {
            if (L->st != L_FREE) continue;
            {
                std::lock_guard<std::mutex> g(S->mu);
                if (S->stop || S->fault != DC_OK) break;
                const int c = pick_class(S);
                if (c < 0) break;
                take_requests(S, S->q[c], L->reqs);
                L->cls = c;
                L->batch = S->next_batch++;
                S->n_batches++;
                S->max_batch = std::max<uint64_t>(S->max_batch, L->reqs.size());
            }
            if (launch(S, *L) != hipSuccess) {
                /* the lane's requests fail with the rest */
                hipStreamSynchronize(L->s);
                publish(S, *L, true);
                fail_all(S);
                break;
            }
            progress = true;
        }
        bool busy = false;
        for (auto &L : S->lanes) busy |= L->st != L_FREE;
        std::unique_lock<std::mutex> g(S->mu);
        if (S->stop && !busy) break;
        if (progress) continue;
        if (busy) {
            g.unlock();
            std::this_thread::yield();
        } else {
            S->cv.wait_for(g, std::chrono::milliseconds(2),
                           [&] { return S->stop || (S->fault == DC_OK && waiting(S) > 0); });
        }
    }
}

void destroy_lanes(dc_server *S) {
    for (auto &L : S->lanes) {
        if (L->s) hipStreamSynchronize(L->s);
        if (L->ev_run) hipEventDestroy(L->ev_run);
        if (L->ev_fetch) hipEventDestroy(L->ev_fetch);
        if (L->s) hipStreamDestroy(L->s);
    }
    S->lanes.clear();
}

}  // namespace

extern "C" dc_status_t dc_server_create(dc_ctx_t *ctx, const dc_server_opts_t *opts, dc_server_t **out) {
    if (!ctx || !out) return DC_E_INVAL;
    *out = nullptr;
    dc_server_opts_t o{};
    if (opts) o = *opts;
    if (o.lanes == 0) {
        /* lanes that share a hardware queue run in order, so one lane per
         * queue of the process, leaving one for the caller's own stream */
        const char *q = getenv("GPU_MAX_HW_QUEUES");
        const int hwq = std::max(2, q ? atoi(q) : 4);
        o.lanes = (uint32_t)std::min(8, hwq - 1);
    }
    if (o.max_request_instr == 0) o.max_request_instr = 100000;
    if (o.max_batch_kernels == 0) o.max_batch_kernels = 2048;
    if (o.long_instr == 0) o.long_instr = 16384;
    if (o.lanes > 16 || o.max_batch_kernels > 65536 || o.max_request_instr > LANE_INSTR_MAX ||
        (o.flags & ~DC_OPT_DIGEST))
        return DC_E_INVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return DC_E_HIP;
    std::unique_ptr<dc_server> S(new (std::nothrow) dc_server);
    if (!S) return DC_E_OOM;
    S->ctx = ctx;
    S->o = o;
    const size_t lds_wave = fixpoint_lds_per_wave();
    S->wpg = (uint32_t)std::max<size_t>(1, std::min<size_t>(4, ctx->lds_per_group / lds_wave));
    const uint64_t per_cu = fixpoint_groups_per_cu(S->wpg);
    const uint64_t groups_cap =
        std::max<uint64_t>(1, std::min<uint64_t>((uint64_t)ctx->n_cu * per_cu, (o.max_batch_kernels + S->wpg - 1) / S->wpg));
    const uint64_t waves = groups_cap * S->wpg;
    S->lane_kernels = o.max_batch_kernels;
    /* the two shorter classes may use every lane, the longer ones half and a
     * quarter of them (at least one) */
    S->class_lanes[0] = S->class_lanes[1] = o.lanes;
    S->class_lanes[2] = std::max<uint32_t>(1, o.lanes / 2);
    S->class_lanes[3] = std::max<uint32_t>(1, o.lanes / 4);
    S->lane_args = (uint64_t)o.max_batch_kernels * 255;
    /* overflow arenas: up to a quarter of a lane's share of the pool, and
     * at least one wave's worth for the longest request */
    uint64_t ovf_bytes = OVF_BUDGET_BYTES;
    if (o.pool_bytes) ovf_bytes = std::min<uint64_t>(ovf_bytes, o.pool_bytes / o.lanes / 4);
    S->ovf_rows_budget = std::max<uint64_t>((uint64_t)o.max_request_instr * FIX_MAX_ROWS, ovf_bytes / ROW_BYTES);
    const uint64_t bitmap_words = OVF_MAX_WAVES * (2 * ((o.max_request_instr + 31) / 32) + 64);
    const uint64_t fixed = waves * LANE_ARENA_ROWS * ROW_BYTES + S->ovf_rows_budget * ROW_BYTES + bitmap_words * 4 +
                           (waves + OVF_MAX_WAVES) * 64 * 16 + S->lane_kernels * BYTES_PER_KERNEL + (1u << 20);
    uint64_t lane_instr = LANE_INSTR_MAX;
    if (o.pool_bytes) {
        const uint64_t per_lane = o.pool_bytes / o.lanes;
        if (per_lane <= fixed) return DC_E_INVAL;
        lane_instr = std::min<uint64_t>(lane_instr, (per_lane - fixed) / BYTES_PER_INSTR);
        if (lane_instr < o.max_request_instr) return DC_E_INVAL;
    }
    S->lane_instr = lane_instr;
    for (uint32_t i = 0; i < o.lanes; i++) {
        std::unique_ptr<Lane> L(new (std::nothrow) Lane);
        if (!L) return DC_E_OOM;
        L->id = i;
        L->groups_cap = (uint32_t)groups_cap;
        if (hipStreamCreateWithFlags(&L->s, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&L->ev_run, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&L->ev_fetch, hipEventDisableTiming) != hipSuccess) {
            S->lanes.push_back(std::move(L));
            destroy_lanes(S.get());
            return DC_E_HIP;
        }
        PlanDims d{lane_instr, S->lane_kernels, S->lane_args, false, waves, LANE_ARENA_ROWS};
        Plan &P = L->P;
        L->in = alloc_plan(L->mem, P, d);
        /* a lane plans for its worst case: one block, one access and four
         * built-in records per instruction */
        alloc_blocks(L->mem, P, lane_instr, lane_instr, 4 * lane_instr, false);
        P.instrs = L->mem.alloc<dc_instr_t>(lane_instr);
        P.ovf_arena = L->mem.alloc<uint32_t>(S->ovf_rows_budget * FIX_ROW_DWORDS);
        P.ovf_bitmaps = L->mem.alloc<uint32_t>(bitmap_words);
        P.sweep_cap = 0;
        P.flags = o.flags;
        L->dP = L->mem.alloc<Plan>(1);
        const bool pin_ok = L->h_instrs.reserve(lane_instr) == hipSuccess && L->h_k.reserve(S->lane_kernels) == hipSuccess &&
                            L->h_a.reserve(S->lane_args) == hipSuccess &&
                            L->h_pb.reserve(S->lane_kernels + 1) == hipSuccess &&
                            L->h_ds.reserve(S->lane_kernels) == hipSuccess && L->h_plan.reserve(1) == hipSuccess &&
                            L->h_order.reserve(S->lane_kernels) == hipSuccess &&
                            L->h_res.reserve(S->lane_kernels) == hipSuccess &&
                            L->h_acc_off.reserve(S->lane_kernels + 1) == hipSuccess &&
                            L->h_sys_off.reserve(S->lane_kernels + 1) == hipSuccess &&
                            L->h_acc.reserve(lane_instr / 8) == hipSuccess && L->h_sys.reserve(lane_instr / 8) == hipSuccess;
        const bool failed = L->mem.failed || !pin_ok;
        S->device_bytes += L->mem.bytes_total;
        S->lanes.push_back(std::move(L));
        if (failed) {
            destroy_lanes(S.get());
            return DC_E_OOM;
        }
    }
    try {
        S->th = std::thread(service, S.get());
    } catch (...) {
        destroy_lanes(S.get());
        return DC_E_OOM;
    }
    *out = S.release();
    return DC_OK;
}

extern "C" dc_status_t dc_server_submit(dc_server_t *S, const dc_request_t *req, uint64_t *ticket) {
    if (!S || !req || !ticket) return DC_E_INVAL;
    const dc_kernel_t &k = req->kernel;
    if (k.n_instr > S->o.max_request_instr || (k.n_instr && !req->instrs)) return DC_E_INVAL;
    /* a descriptor with too many arguments fails per request; its table is not read */
    const uint32_t n_args = k.n_args <= 255 ? k.n_args : 0;
    if (n_args && !req->args) return DC_E_INVAL;
    std::unique_ptr<Req> r(new (std::nothrow) Req);
    if (!r) return DC_E_OOM;
    try {
        r->instrs.assign(req->instrs, req->instrs + k.n_instr);
        r->args.assign(req->args, req->args + n_args);
    } catch (...) {
        return DC_E_OOM;
    }
    r->kd = k;
    r->tag = req->tag;
    r->t_submit = now_ns();
    {
        std::lock_guard<std::mutex> g(S->mu);
        if (S->fault != DC_OK) return S->fault;
        r->ticket = S->next_ticket++;
        *ticket = r->ticket;
        S->q[length_class(S, k.n_instr)].push_back(std::move(r));
        S->n_submitted++;
    }
    S->cv.notify_one();
    return DC_OK;
}

extern "C" dc_status_t dc_server_poll(dc_server_t *S, dc_result_t *out, uint32_t max, uint32_t *n) {
    if (!S || !n || (max && !out)) return DC_E_INVAL;
    std::lock_guard<std::mutex> g(S->mu);
    S->delivered.clear();
    uint32_t c = 0;
    while (c < max && !S->done.empty()) {
        std::unique_ptr<Done> d = std::move(S->done.front());
        S->done.pop_front();
        d->r.accesses = d->acc.data();
        d->r.sysvals = d->sys.data();
        out[c++] = d->r;
        S->delivered.push_back(std::move(d));
    }
    *n = c;
    return DC_OK;
}

extern "C" dc_status_t dc_server_get_stats(dc_server_t *S, dc_server_stats_t *out) {
    if (!S || !out) return DC_E_INVAL;
    std::lock_guard<std::mutex> g(S->mu);
    memset(out, 0, sizeof(*out));
    out->submitted = S->n_submitted;
    out->completed = S->n_completed;
    out->waiting = waiting(S);
    out->batches = S->n_batches;
    out->max_batch_kernels = S->max_batch;
    out->device_bytes = S->device_bytes;
    out->lane_instr = S->lane_instr;
    out->lanes = (uint32_t)S->lanes.size();
    return DC_OK;
}

extern "C" void dc_server_destroy(dc_server_t *S) {
    if (!S) return;
    {
        std::lock_guard<std::mutex> g(S->mu);
        S->stop = true;
    }
    S->cv.notify_one();
    if (S->th.joinable()) S->th.join();
    hipSetDevice(S->ctx->device);
    destroy_lanes(S);
    delete S;
}
