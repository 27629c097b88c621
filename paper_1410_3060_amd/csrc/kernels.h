// Host-side launchers of the HIP kernels (internal to libstencil.so).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace stn {

// Geometry of one call: interior sizes, boundary width, element strides.
struct dims {
    int nx, ny, nz, h;
    int64_t sy, sz;
    // element offset of interior (0,0,0) from the padded origin
    int64_t org() const { return (int64_t)h * sz + (int64_t)h * sy + h; }
};

struct host_weights {
    float w[5];
    float alpha;
    float lres;  // w0 + 6 (w1 + w2 + w3 + w4), formed in double (see op_lap8)
};

// One naive time step (Sect. 4.1).  Jacobi kinds: out <- A(cur).  Leapfrog
// kinds: out <- 2 cur - prev + alpha L8(cur); out may equal prev.  Pointers
// address padded origins.  coef_bf16 selects uint16 BF16 coefficient storage.
hipError_t launch_naive_step(int kind, bool coef_bf16, const float* cur, const float* prev,
                             float* out, const void* coef, int64_t sk, const dims& d,
                             const host_weights& wt, int zchunk, hipStream_t s);
// (zchunk <= 0: planes per z-chunk chosen from the kernel's occupancy)

// Workgroups of `kernel` (with `threads` threads) resident on the current
// device at once: its occupancy per compute unit times the compute units.
long long device_slots(const void* kernel, int threads);

// Planes per z-chunk for a streaming kernel with txy workgroups per z-chunk
// and stencil radius R, given `slots` resident workgroups: the chunk count
// minimises (rounds of resident workgroups) x (planes a workgroup streams,
// its chunk plus the 2R planes that prime its register queues) -- the time of
// a bandwidth-bound launch whose workgroups stream equal chunks.
int pick_zchunk(int nz, long long txy, long long slots, int R);

// Copy the boundary shell of width r (every point of [-r, n+r)^3 outside the
// interior) from src to dst; interior points of dst are not touched.
hipError_t launch_copy_shell(float* dst, const float* src, const dims& d, int r, hipStream_t s);

}  // namespace stn
