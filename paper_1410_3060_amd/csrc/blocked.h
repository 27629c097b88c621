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

// Multi-workgroup diamonds for the radius-4 kinds (mwd.hip): one launch per
// diamond row; teams of workgroups share a diamond, one x-slice of xs = 16 or
// 32 columns each (0 = the default for the width), exchanging x-halos through
// `xbuf` (cleared to zero before the first row of a run; `tag` 1 .. 4095
// differs between consecutive launches).  A halo that never arrives sets
// *err to non-zero.
struct mwd_row_args {
    const float* ftop_o;
    const float* fsub_o;
    float* ftop_n;
    float* fsub_n;
    const void* coef;
    int64_t sk;
    dims d;
    host_weights wt;
    int64_t t0, nt;
    int first_centre, n_diamonds;
    int dw;
    int xs = 0;      // slice width (columns per workgroup), 0 = default
    int zchunk = 0;  // planes per z-chunk, 0 = chosen from the team count
    uint64_t field_bytes, coef_bytes;
    // BF16 arrays on 4-byte boundaries with even sk and sz: word loads
    bool coef_aligned = false;
    void* xbuf;
    size_t xbuf_bytes;
    int* err;
    uint32_t tag;
};
bool mwd_supported(int kind, int dw, int xs);
// workgroups sharing one diamond (x-slices) for nx columns, 0 if not provided
int mwd_slices(int kind, int dw, int xs, int nx);
// bytes of exchange buffer the launches of (kind, dw, xs) need on this device for nx
hipError_t mwd_workspace(int kind, bool bf16, int dw, int xs, int nx, size_t* xbytes);
hipError_t launch_mwd_row(int kind, bool bf16, const mwd_row_args& a, hipStream_t s);
hipError_t launch_fill_u32(void* p, size_t words, uint32_t v, hipStream_t s);

bool blocked_supported(int kind, int dw, int xs = 0);
// the diamond width used when none is given, for a grid of `points` interior
// points and FP32 or BF16 coefficients
int blocked_default_dw(int kind, int64_t points, bool bf16);
int blocked_max_xo(int kind, int dw);
hipError_t launch_blocked_row(int kind, bool bf16, const blocked_row_args& a, hipStream_t s);

}  // namespace stn
