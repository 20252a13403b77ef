/*
 * dc_text_api.cpp -- C ABI of the text front end (include/dc.h,
 * dc_parse_text and friends): planning from the counts of the first run,
 * stage enqueue on the caller's stream, getters.
 */
#include <hip/hip_runtime_api.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "dc.h"
#include "dc_host.h"
#include "dc_internal.h"

using namespace dc;

namespace {
enum { TE_START, TE_LINES, TE_COUNTS, TE_END, TE_N };
constexpr int TE_RING = 64;
}  // namespace

struct dc_text {
    dc_ctx *ctx = nullptr;
    hipStream_t stream = nullptr;
    DevMem mem;                 /* the fail flag */
    DevMem lmem;                /* arrays sized by the text: tiles, lines, kernels, outputs */
    TextPlan T{};
    bool planned = false;
    bool have_events = false;
    hipEvent_t ev[TE_RING][TE_N] = {};
    uint64_t runs = 0, runs_at_reset = 0;
    bool host_valid = false;
    uint32_t fail = 0;
    std::vector<dc_kernel_t> kernels;
    std::vector<dc_instr_t> instrs;
    std::vector<dc_arg_t> args;
    std::vector<uint64_t> name_off;
    std::vector<uint32_t> name_len;
};

static dc_status_t tx_fail(hipError_t e) { return e == hipErrorOutOfMemory ? DC_E_OOM : DC_E_HIP; }

/* read one u64 back from the device (waits for the stream) */
static hipError_t read_u64(const uint64_t *p, uint64_t *out, hipStream_t s) {
    hipError_t e = hipMemcpyAsync(out, p, sizeof(uint64_t), hipMemcpyDeviceToHost, s);
    return e == hipSuccess ? hipStreamSynchronize(s) : e;
}

/* every stage; the first run on a text sizes the arrays from the counts (three waits) */
static dc_status_t tx_enqueue(dc_text *X) {
    TextPlan &T = X->T;
    hipStream_t s = X->stream;
    hipError_t e = hipSuccess;
    X->host_valid = false;
    hipEvent_t *ev = X->ev[X->runs % TE_RING];
#define TRY(x)                                  \
    do {                                        \
        e = (x);                                \
        if (e != hipSuccess) return tx_fail(e); \
    } while (0)
    if (X->have_events) TRY(hipEventRecord(ev[TE_START], s));
    TRY(launch_fill_u32(T.fail, 1, 0u, s));
    if (!X->planned) {
        X->lmem.reset();
        T.n_tiles = (uint32_t)std::max<uint64_t>(1, (T.n_bytes + 4095) / 4096);
        T.tile_cnt = X->lmem.alloc<uint32_t>(T.n_tiles);
        T.tile_off = X->lmem.alloc<uint64_t>((uint64_t)T.n_tiles + 1);
        if (X->lmem.failed) return DC_E_OOM;
        TRY(launch_text_lines(T, s));
        uint64_t nl = 0;
        TRY(read_u64(T.tile_off + T.n_tiles, &nl, s));
        T.n_lines = nl + 1;
        T.line_start = X->lmem.alloc<uint64_t>(T.n_lines + 1);
        T.kind = X->lmem.alloc<uint8_t>(T.n_lines);
        T.n_ltiles = (uint32_t)((T.n_lines + 4095) / 4096);
        T.ltile_cnt = X->lmem.alloc<uint32_t>(T.n_ltiles);
        T.ltile_off = X->lmem.alloc<uint64_t>((uint64_t)T.n_ltiles + 1);
        if (X->lmem.failed) return DC_E_OOM;
        TRY(launch_text_classify(T, s));
        uint64_t nk = 0;
        TRY(read_u64(T.ltile_off + T.n_ltiles, &nk, s));
        if (nk > 0xFFFFFFF0ull) return DC_E_INVAL;
        T.n_kernels = T.k_cap = (uint32_t)nk;
        const uint64_t K = nk;
        T.kline = X->lmem.alloc<uint64_t>(K + 1);
        T.kcounts = X->lmem.alloc<uint32_t>(3 * std::max<uint64_t>(K, 1));
        T.koffs = X->lmem.alloc<uint64_t>(3 * (K + 1));
        T.kernels = X->lmem.alloc<dc_kernel_t>(K);
        T.name_off = X->lmem.alloc<uint64_t>(K);
        T.name_len = X->lmem.alloc<uint32_t>(K);
        T.lab_key = nullptr;
        T.lab_idx = T.lab_line = nullptr;
        T.instrs = nullptr;
        T.args = nullptr;
        T.lab_cap = T.instr_cap = T.arg_cap = 0;
        if (X->lmem.failed) return DC_E_OOM;
        if (X->have_events) TRY(hipEventRecord(ev[TE_LINES], s));
        TRY(launch_text_kernels1(T, s));
        uint64_t tot[3] = {0, 0, 0};
        for (int a = 0; a < 3 && K; a++) TRY(read_u64(T.koffs + (uint64_t)a * (K + 1) + K, &tot[a], s));
        T.instrs = X->lmem.alloc<dc_instr_t>(tot[0]);
        T.lab_key = X->lmem.alloc<unsigned long long>(tot[1]);
        T.lab_idx = X->lmem.alloc<uint32_t>(tot[1]);
        T.lab_line = X->lmem.alloc<uint32_t>(tot[1]);
        T.args = X->lmem.alloc<dc_arg_t>(tot[2]);
        T.instr_cap = tot[0];
        T.lab_cap = tot[1];
        T.arg_cap = tot[2];
        if (X->lmem.failed) return DC_E_OOM;
        X->planned = true;
    } else {
        TRY(launch_text_lines(T, s));
        TRY(launch_text_classify(T, s));
        if (X->have_events) TRY(hipEventRecord(ev[TE_LINES], s));
        TRY(launch_text_kernels1(T, s));
    }
    if (X->have_events) TRY(hipEventRecord(ev[TE_COUNTS], s));
    TRY(launch_text_kernels2(T, s));
    if (X->have_events) TRY(hipEventRecord(ev[TE_END], s));
#undef TRY
    X->runs++;
    return DC_OK;
}

extern "C" dc_status_t dc_parse_text(dc_ctx_t *ctx, const char *text, uint64_t n_bytes, const dc_options_t *opts,
                                     void *stream, dc_text_t **out) {
    if (!out) return DC_E_INVAL;
    *out = nullptr;
    if (!ctx || (n_bytes && !text) || (opts && (opts->flags & ~DC_OPT_TIMING))) return DC_E_INVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return DC_E_HIP;
    dc_text *X = new (std::nothrow) dc_text;
    if (!X) return DC_E_OOM;
    X->ctx = ctx;
    X->stream = (hipStream_t)stream;
    X->T.text = reinterpret_cast<const uint8_t *>(text);
    X->T.n_bytes = n_bytes;
    X->T.fail = X->mem.alloc<uint32_t>(1);
    dc_status_t st = X->mem.failed ? DC_E_OOM : DC_OK;
    if (st == DC_OK && opts && (opts->flags & DC_OPT_TIMING)) {
        for (int r = 0; r < TE_RING && st == DC_OK; r++)
            for (int i = 0; i < TE_N; i++)
                if (hipEventCreate(&X->ev[r][i]) != hipSuccess) st = DC_E_HIP;
        X->have_events = st == DC_OK;
    }
    if (st == DC_OK) st = tx_enqueue(X);
    if (st != DC_OK) {
        hipStreamSynchronize(X->stream);
        dc_text_free(X);
        return st;
    }
    *out = X;
    return DC_OK;
}

extern "C" dc_status_t dc_text_run(dc_text_t *X, const char *text, uint64_t n_bytes) {
    if (!X || (n_bytes && !text)) return DC_E_INVAL;
    if (hipSetDevice(X->ctx->device) != hipSuccess) return DC_E_HIP;
    if (reinterpret_cast<const uint8_t *>(text) != X->T.text || n_bytes != X->T.n_bytes) {
        if (hipStreamSynchronize(X->stream) != hipSuccess) return DC_E_HIP;
        X->T.text = reinterpret_cast<const uint8_t *>(text);
        X->T.n_bytes = n_bytes;
        X->planned = false;
    }
    return tx_enqueue(X);
}

extern "C" dc_status_t dc_text_wait(dc_text_t *X) {
    if (!X) return DC_E_INVAL;
    if (hipSetDevice(X->ctx->device) != hipSuccess) return DC_E_HIP;
    return hipStreamSynchronize(X->stream) == hipSuccess ? DC_OK : DC_E_HIP;
}

static dc_status_t tx_fetch(dc_text *X) {
    if (X->host_valid) return X->fail ? DC_E_CAPACITY : DC_OK;
    dc_status_t st = dc_text_wait(X);
    if (st != DC_OK) return st;
    const TextPlan &T = X->T;
    hipError_t e = hipMemcpy(&X->fail, T.fail, sizeof(uint32_t), hipMemcpyDeviceToHost);
    X->kernels.resize(T.n_kernels);
    X->instrs.resize(T.instr_cap);
    X->args.resize(T.arg_cap);
    X->name_off.resize(T.n_kernels);
    X->name_len.resize(T.n_kernels);
    if (e == hipSuccess && T.n_kernels)
        e = hipMemcpy(X->kernels.data(), T.kernels, T.n_kernels * sizeof(dc_kernel_t), hipMemcpyDeviceToHost);
    if (e == hipSuccess && T.instr_cap)
        e = hipMemcpy(X->instrs.data(), T.instrs, T.instr_cap * sizeof(dc_instr_t), hipMemcpyDeviceToHost);
    if (e == hipSuccess && T.arg_cap)
        e = hipMemcpy(X->args.data(), T.args, T.arg_cap * sizeof(dc_arg_t), hipMemcpyDeviceToHost);
    if (e == hipSuccess && T.n_kernels)
        e = hipMemcpy(X->name_off.data(), T.name_off, T.n_kernels * sizeof(uint64_t), hipMemcpyDeviceToHost);
    if (e == hipSuccess && T.n_kernels)
        e = hipMemcpy(X->name_len.data(), T.name_len, T.n_kernels * sizeof(uint32_t), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return tx_fail(e);
    X->host_valid = true;
    return X->fail ? DC_E_CAPACITY : DC_OK;
}

extern "C" dc_status_t dc_text_get_counts(dc_text_t *X, dc_text_counts_t *out) {
    if (!X || !out) return DC_E_INVAL;
    dc_status_t st = dc_text_wait(X);
    if (st != DC_OK) return st;
    uint32_t fail = 0;
    if (hipMemcpy(&fail, X->T.fail, sizeof(uint32_t), hipMemcpyDeviceToHost) != hipSuccess) return DC_E_HIP;
    memset(out, 0, sizeof(*out));
    out->n_kernels = X->T.n_kernels;
    out->n_lines = X->T.n_lines;
    out->n_instr = X->T.instr_cap;
    out->n_args = X->T.arg_cap;
    out->fail = fail;
    return fail ? DC_E_CAPACITY : DC_OK;
}

extern "C" dc_status_t dc_text_device_arrays(dc_text_t *X, const dc_kernel_t **kernels, const dc_instr_t **instrs,
                                             const dc_arg_t **args) {
    if (!X) return DC_E_INVAL;
    if (kernels) *kernels = X->T.kernels;
    if (instrs) *instrs = X->T.instrs;
    if (args) *args = X->T.args;
    return DC_OK;
}

extern "C" dc_status_t dc_text_get_kernels(dc_text_t *X, dc_kernel_t *buf, uint32_t cap, uint32_t *n_total) {
    if (!X || !n_total || (cap && !buf)) return DC_E_INVAL;
    dc_status_t st = tx_fetch(X);
    if (st != DC_OK) return st;
    *n_total = (uint32_t)X->kernels.size();
    const uint32_t n = std::min<uint32_t>(cap, *n_total);
    if (n) memcpy(buf, X->kernels.data(), n * sizeof(dc_kernel_t));
    return DC_OK;
}

extern "C" dc_status_t dc_text_get_records(dc_text_t *X, dc_instr_t *buf, uint64_t cap, uint64_t *n_total) {
    if (!X || !n_total || (cap && !buf)) return DC_E_INVAL;
    dc_status_t st = tx_fetch(X);
    if (st != DC_OK) return st;
    *n_total = X->instrs.size();
    const uint64_t n = std::min<uint64_t>(cap, *n_total);
    if (n) memcpy(buf, X->instrs.data(), n * sizeof(dc_instr_t));
    return DC_OK;
}

extern "C" dc_status_t dc_text_get_args(dc_text_t *X, dc_arg_t *buf, uint64_t cap, uint64_t *n_total) {
    if (!X || !n_total || (cap && !buf)) return DC_E_INVAL;
    dc_status_t st = tx_fetch(X);
    if (st != DC_OK) return st;
    *n_total = X->args.size();
    const uint64_t n = std::min<uint64_t>(cap, *n_total);
    if (n) memcpy(buf, X->args.data(), n * sizeof(dc_arg_t));
    return DC_OK;
}

extern "C" dc_status_t dc_text_get_names(dc_text_t *X, uint64_t *name_off, uint32_t *name_len, uint32_t cap,
                                         uint32_t *n_total) {
    if (!X || !n_total || (cap && (!name_off || !name_len))) return DC_E_INVAL;
    dc_status_t st = tx_fetch(X);
    if (st != DC_OK) return st;
    *n_total = (uint32_t)X->name_off.size();
    const uint32_t n = std::min<uint32_t>(cap, *n_total);
    if (n) {
        memcpy(name_off, X->name_off.data(), n * sizeof(uint64_t));
        memcpy(name_len, X->name_len.data(), n * sizeof(uint32_t));
    }
    return DC_OK;
}

extern "C" dc_status_t dc_text_get_timing(dc_text_t *X, dc_timing_t *out) {
    if (!X || !out) return DC_E_INVAL;
    memset(out, 0, sizeof(*out));
    if (!X->have_events) return DC_E_NOTREADY;
    dc_status_t st = dc_text_wait(X);
    if (st != DC_OK) return st;
    uint64_t first = X->runs_at_reset;
    if (X->runs - first > (uint64_t)TE_RING) first = X->runs - TE_RING;
    for (uint64_t r = first; r < X->runs; r++) {
        hipEvent_t *ev = X->ev[r % TE_RING];
        float a = 0, b = 0, c = 0, d = 0;
        if (hipEventElapsedTime(&a, ev[TE_START], ev[TE_END]) != hipSuccess ||
            hipEventElapsedTime(&b, ev[TE_START], ev[TE_LINES]) != hipSuccess ||
            hipEventElapsedTime(&c, ev[TE_LINES], ev[TE_COUNTS]) != hipSuccess ||
            hipEventElapsedTime(&d, ev[TE_COUNTS], ev[TE_END]) != hipSuccess)
            return DC_E_HIP;
        out->ms_total += a;
        out->ms_decode += b;
        out->ms_cfg += c;
        out->ms_fixpoint += d;
        out->runs++;
    }
    return DC_OK;
}

extern "C" dc_status_t dc_text_timing_reset(dc_text_t *X) {
    if (!X) return DC_E_INVAL;
    X->runs_at_reset = X->runs;
    return DC_OK;
}

extern "C" void dc_text_free(dc_text_t *X) {
    if (!X) return;
    hipSetDevice(X->ctx->device);
    hipStreamSynchronize(X->stream);
    for (int r = 0; r < TE_RING; r++)
        for (int i = 0; i < TE_N; i++)
            if (X->ev[r][i]) hipEventDestroy(X->ev[r][i]);
    delete X;
}
