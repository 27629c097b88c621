// Host-side interface of the blocked (diamond/wavefront) row kernel.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace stn {

// One row of diamonds: reads the old frontier pair, writes the new one.  The
// boundary shell (width R) is read from the old frontier top and must be the
// same in every frontier buffer.
struct blocked_row_args {
    const float* ftop_o;  // old frontier: newest level per point
    const float* fsub_o;  // old frontier: the level below it
    float* ftop_n;        // new frontier (distinct buffers)
    float* fsub_n;
    const void* coef;
    int64_t sk;
    dims d;
    host_weights wt;
    int64_t t0, nt;
    int first_centre, n_diamonds;
    int dw;       // diamond width
    int xo;       // output x extent per workgroup
    int gx;       // x tiles
    int zchunk;   // planes per z-chunk
    int gz;       // z-chunks
    uint64_t field_bytes;  // bytes of one field from its padded origin
    uint64_t coef_bytes;   // bytes of one coefficient array from its padded origin
    // (a workgroup addresses a window of zchunk + 2R(L+1) + 1 planes from a
    // base of its own with 32-bit offsets: the window must stay below 2^31 bytes)
    // If set, launch_blocked_row launches nothing and stores the number of
    // workgroups of the kernel it would launch that the device holds at once.
    long long* slots_out = nullptr;
    // BF16 coefficients whose arrays all start on 4-byte boundaries, with even
    // sk and sz: the level update then reads each element's word at a
    // per-column offset (ignored for FP32)
    bool coef_aligned = false;
};

// Device memory of the allocation-free blocked run (stencil_run_noalloc): a
// file-scope device array of kScratchBytes, one copy per GPU, held from the
// library's load to the end of the process.
constexpr size_t kScratchBytes = size_t(128) << 20;
// Device address of that array on the current device (looked up once per
// device with hipGetSymbolAddress, then cached).  Host code must use this
// address, never the array's name.
hipError_t blocked_scratch(void** ptr);

bool blocked_supported(int kind, int dw);
int blocked_default_dw(int kind);
int blocked_max_xo(int kind, int dw);
hipError_t launch_blocked_row(int kind, bool bf16, const blocked_row_args& a, hipStream_t s);

}  // namespace stn
