/* dc_host.h -- host-side pieces shared by the batch API (dc_api.cpp) and the
 * request server (dc_server.cpp): the context, device allocation lists, the
 * descriptor checks and the allocation of a plan's device arrays. */
#pragma once
#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include <stdlib.h>

#include <algorithm>
#include <vector>

#include "dc.h"
#include "dc_internal.h"

struct dc_ctx {
    int device;
    int n_cu;
    size_t lds_per_cu;
    size_t lds_per_group;
};

namespace dc {

/* Failure injection for tests: with DC_FAULT_ALLOC=n in the environment the
 * n-th device allocation of every allocation list fails as if the device
 * were out of memory (0 or unset: none). */
inline uint64_t fault_alloc_nth() {
    const char *e = getenv("DC_FAULT_ALLOC");
    return e ? strtoull(e, nullptr, 10) : 0;
}

/* one device allocation list per object, freed together */
struct DevMem {
    std::vector<void *> ptrs;
    bool failed = false;
    uint64_t bytes_total = 0;
    uint64_t n_allocs = 0;
    template <typename T>
    T *alloc(uint64_t count) {
        void *p = nullptr;
        uint64_t bytes = count * sizeof(T);
        if (bytes == 0) bytes = 16;
        bytes = (bytes + 255) & ~255ull;
        const uint64_t nth = fault_alloc_nth();
        if (++n_allocs == nth || hipMalloc(&p, bytes) != hipSuccess) {
            failed = true;
            return nullptr;
        }
        ptrs.push_back(p);
        bytes_total += bytes;
        return static_cast<T *>(p);
    }
    void reset() {
        for (void *p : ptrs) hipFree(p);
        ptrs.clear();
        failed = false;
        bytes_total = 0;
    }
    void release(void *p) {
        auto it = std::find(ptrs.begin(), ptrs.end(), p);
        if (it != ptrs.end()) {
            hipFree(p);
            ptrs.erase(it);
        }
    }
    DevMem() = default;
    DevMem(const DevMem &) = delete;
    DevMem &operator=(const DevMem &) = delete;
    ~DevMem() {
        for (void *p : ptrs) hipFree(p);
    }
};

/* descriptor checks that need no records (per kernel) */
inline int32_t descriptor_status(const dc_kernel_t &k) {
    if (k.useargs != 1) return DC_E_UNSUPPORTED;
    if (k.dims < 1 || k.dims > 3) return DC_E_UNSUPPORTED;
    for (int d = 0; d < k.dims; d++)
        if (k.cws[d] == 0) return DC_E_UNSUPPORTED;
    if (k.n_args > 255) return DC_E_UNSUPPORTED;
    return DC_OK;
}

/* Sizes a plan's device arrays are allocated for: positions, kernels,
 * argument entries; for an analysis (not CFG-only) also the main-pass waves
 * and their arena rows. */
struct PlanDims {
    uint64_t N, K, A;
    bool cfg_only;
    uint64_t waves;
    uint32_t arena_rows;
};

/* device bytes per block and per record slot of alloc_blocks */
constexpr uint64_t BLOCK_BYTES_CFG = 4 + 4 + 8 + 4 + 4 + 8 + 4 + 4 + 4 + 1;
constexpr uint64_t BLOCK_BYTES = BLOCK_BYTES_CFG + 32 + 4 * 2 + 4 * 4;
constexpr uint64_t ACC_SLOT_BYTES = 2 * 16, SYS_SLOT_BYTES = 2 * 8;

/* Device input tables of a plan (the Plan holds them as const pointers). */
struct PlanInputs {
    dc_kernel_t *kernels;
    dc_arg_t *args;
    uint32_t *pos_begin;
    int32_t *desc_status;
    uint32_t *work_order;   /* analysis plans only */
};

/* Allocate the per-kernel and per-position device arrays of P for dims d
 * (and, for an analysis, the main-pass arena) from M (M.failed on error).
 * The block-indexed arrays, the overflow arena, the state export and the
 * counts in P are left to the caller. */
PlanInputs alloc_plan(DevMem &M, Plan &P, const PlanDims &d);
/* Allocate the block-indexed arrays of P for `blocks` global blocks and,
 * for an analysis, the record regions for `acc` access and `sys` built-in
 * record slots. */
void alloc_blocks(DevMem &M, Plan &P, uint64_t blocks, uint64_t acc, uint64_t sys, bool cfg_only);

}  // namespace dc
