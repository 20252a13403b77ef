/* dc_device.h -- device helpers shared by the HIP translation units of
 * libdc: wavefront primitives, the opcode descriptor table, the digest mix. */
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dc_internal.h"
#include "dc_isa.h"

namespace dc {

/* one copy per translation unit (constant memory, 616 bytes) */
static __constant__ uint64_t OPTAB[N_OPS] = DC_OPTAB_INIT;

__device__ __forceinline__ uint32_t rfl(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ uint32_t rdl(uint32_t x, uint32_t l) { return __builtin_amdgcn_readlane(x, l); }
__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }
__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & 63; }
/* lanes below this one in a 64-bit lane mask */
__device__ __forceinline__ uint32_t lanes_below(uint64_t m) {
    return (uint32_t)__builtin_popcountll(m & ((1ull << lane_id()) - 1ull));
}

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    /* splitmix64 finaliser (Steele, Lea & Flood 2014) */
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

}  // namespace dc
