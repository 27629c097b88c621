// Raw buffer memory operations shared by the temporally blocked kernels.
//
// Every lattice access of those kernels goes through a buffer resource (base
// address + size) with a 32-bit byte offset.  An offset at or beyond the
// resource's size returns 0 on a load and drops a store, so an operand a lane
// does not need is given the offset kNone instead of a branch, and no index
// mistake can reach memory outside the buffer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace stn {

using rsrc_t = __amdgpu_buffer_rsrc_t;

// Byte offset beyond every buffer the kernels touch (each is based so that
// it spans less than 2^31 bytes).
constexpr uint32_t kNone = 0x80000000u;

// Cache policy bits of buffer operations on gfx950: SC1 makes a load or a
// store coherent across the whole device (the two-level XCD caches included),
// which is what relaxed agent-scope atomics compile to; bit 31 marks a load
// volatile, so a polling loop re-issues it.
constexpr int kSC1 = 16;
constexpr int kVolatile = int(1u << 31);

__device__ __forceinline__ rsrc_t make_rsrc(const void* p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ float bload(rsrc_t r, uint32_t voff, uint32_t soff) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
__device__ __forceinline__ void bstore(rsrc_t r, float v, uint32_t voff, uint32_t soff) {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, voff, soff, 0);
}
// coefficient loads: FP32 as stored, BF16 expanded exactly (the 16 stored
// bits become the high half of the FP32 pattern)
__device__ __forceinline__ float cload(const float*, rsrc_t r, uint32_t voff, uint32_t soff) {
    return bload(r, voff, soff);
}
__device__ __forceinline__ float cload(const uint16_t*, rsrc_t r, uint32_t voff, uint32_t soff) {
    return __uint_as_float(static_cast<uint32_t>(__builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0))
                           << 16);
}

}  // namespace stn
