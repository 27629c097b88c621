// Naive scheme (Sect. 4.1): one full sweep of the lattice per time step.
//
// GPU mapping.  A workgroup of 4 waves owns a 64 x TY tile of (x, y) columns
// and streams along z through a chunk of planes (the 2.5D form of the
// spatial blocking of Sect. 3.3: every value of the input level is read from
// HBM once per sweep).  Each lane keeps, for each of its RPT columns, the
// 2R+1 values u(z-R..z+R) in registers; the current plane with its x/y halo
// of width R is staged in LDS (double buffered, one barrier per plane) for the
// in-plane neighbours.  x is the lane index, so every global access of a wave
// is one contiguous 256-byte row.  Coefficients are read once per point.
#include <algorithm>
#include <mutex>
#include <vector>

#include "common.h"
#include "kernels.h"
#include "point_ops.h"

namespace stn {

namespace {

template <int KIND, typename CT, int RPT, int NW>
__global__ __launch_bounds__(NW * 64) void naive_step_kernel(
    const float* __restrict__ cur, const float* prev, float* out, const CT* __restrict__ coef,
    int64_t sk, int nx, int ny, int nz, int64_t sy, int64_t sz, int64_t org, weights wt,
    int zchunk, int gx, int gy, int ntiles) {
    constexpr int R = kind_traits<KIND>::R;
    constexpr int K = kind_traits<KIND>::K;
    constexpr int Q = 2 * R + 1;
    constexpr int TY = NW * RPT;
    constexpr int LW = 64 + 2 * R;
    constexpr int LH = TY + 2 * R;
    __shared__ float lds[2][LH][LW];

    const int tile = xcd_remap(blockIdx.x, ntiles);
    const int bx = tile % gx;
    const int by = (tile / gx) % gy;
    const int bz = tile / (gx * gy);
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int x0 = bx * 64, y0 = by * TY;
    const int z0 = bz * zchunk;
    const int z1 = min(nz, z0 + zchunk);
    const int x = x0 + lane;

    // interior-origin based pointers: element (x, y, z) at p + z*sz + y*sy + x
    const float* C = cur + org;
    const float* P = prev ? prev + org : nullptr;
    float* O = out + org;
    const CT* W = coef ? coef + org : nullptr;

    // columns of this lane: y = y0 + wv + NW*i
    int64_t colo[RPT];
    bool ld_ok[RPT], st_ok[RPT];
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
        const int y = y0 + wv + NW * i;
        colo[i] = (int64_t)y * sy + x;
        ld_ok[i] = (x < nx + R) && (y < ny + R);
        st_ok[i] = (x < nx) && (y < ny);
    }

    // y-halo rows handled by this wave: hr = wv + NW*j over [0, 2R)
    constexpr int HYJ = (2 * R + NW - 1) / NW;
    int64_t hyo[HYJ];
    bool hy_ok[HYJ];
    int hy_row[HYJ];
#pragma unroll
    for (int j = 0; j < HYJ; ++j) {
        const int hr = wv + NW * j;
        const int ly = hr < R ? hr - R : TY + (hr - R);  // local row in [-R,0) or [TY,TY+R)
        const int y = y0 + ly;
        hy_row[j] = ly + R;
        hyo[j] = (int64_t)y * sy + x;
        hy_ok[j] = (hr < 2 * R) && (x < nx + R) && (y < ny + R);
    }
    // x-halo columns: thread id < 2R*TY loads one value per plane
    const int hxi = threadIdx.x;
    const bool hx_any = hxi < 2 * R * TY;
    int hx_lx = 0, hx_ly = 0;
    int64_t hxo = 0;
    bool hx_ok = false;
    if (hx_any) {
        const int col = hxi % (2 * R), row = hxi / (2 * R);
        const int gxp = col < R ? x0 - R + col : x0 + 64 + (col - R);
        const int y = y0 + row;
        hx_lx = (col < R ? col : 64 + R + (col - R));
        hx_ly = row + R;
        hxo = (int64_t)y * sy + gxp;
        hx_ok = (gxp < nx + R) && (y < ny + R);
    }

    // register queues: q[i][k] = u(column i, plane z - R + k)
    float q[RPT][Q];
    float nxt[RPT];
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
#pragma unroll
        for (int k = 1; k < Q; ++k)
            q[i][k] = ld_ok[i] ? C[(int64_t)(z0 - R - 1 + k) * sz + colo[i]] : 0.0f;
        nxt[i] = ld_ok[i] ? C[(int64_t)(z0 + R) * sz + colo[i]] : 0.0f;
    }
    float hy[HYJ], hx = 0.0f;
#pragma unroll
    for (int j = 0; j < HYJ; ++j) hy[j] = hy_ok[j] ? C[(int64_t)z0 * sz + hyo[j]] : 0.0f;
    if (hx_ok) hx = C[(int64_t)z0 * sz + hxo];

    for (int z = z0; z < z1; ++z) {
        const int b = (z - z0) & 1;
        const int64_t zo = (int64_t)z * sz;
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
#pragma unroll
            for (int k = 0; k < Q - 1; ++k) q[i][k] = q[i][k + 1];
            q[i][Q - 1] = nxt[i];
            lds[b][R + wv + NW * i][R + lane] = q[i][R];
        }
#pragma unroll
        for (int j = 0; j < HYJ; ++j)
            if (wv + NW * j < 2 * R) lds[b][hy_row[j]][R + lane] = hy[j];
        if (hx_any) lds[b][hx_ly][hx_lx] = hx;

        // prefetch the next plane while this one is computed
        if (z + 1 < z1) {
            const int64_t zn = (int64_t)(z + 1 + R) * sz, z1o = (int64_t)(z + 1) * sz;
#pragma unroll
            for (int i = 0; i < RPT; ++i)
                if (ld_ok[i]) nxt[i] = C[zn + colo[i]];
#pragma unroll
            for (int j = 0; j < HYJ; ++j)
                if (hy_ok[j]) hy[j] = C[z1o + hyo[j]];
            if (hx_ok) hx = C[z1o + hxo];
        }
        // coefficients and the older level for this plane
        float Wv[RPT][kslots<KIND>];
        float pv[RPT];
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            pv[i] = 0.0f;
#pragma unroll
            for (int k = 0; k < kslots<KIND>; ++k) Wv[i][k] = 0.0f;
            if (st_ok[i]) {
                if constexpr (K > 0) {
#pragma unroll
                    for (int k = 0; k < K; ++k) Wv[i][k] = load_coef(W, k * sk + zo + colo[i]);
                }
                if constexpr (kind_traits<KIND>::leapfrog) pv[i] = P[zo + colo[i]];
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            const int ly = R + wv + NW * i, lx = R + lane;
            nbhd<R> n;
            n.c = q[i][R];
#pragma unroll
            for (int r = 1; r <= R; ++r) {
                n.pair[0][r - 1] = lds[b][ly][lx - r] + lds[b][ly][lx + r];
                n.pair[1][r - 1] = lds[b][ly - r][lx] + lds[b][ly + r][lx];
                n.pair[2][r - 1] = q[i][R - r] + q[i][R + r];
            }
            n.m1[0] = lds[b][ly][lx - 1];
            n.p1[0] = lds[b][ly][lx + 1];
            n.m1[1] = lds[b][ly - 1][lx];
            n.p1[1] = lds[b][ly + 1][lx];
            n.m1[2] = q[i][R - 1];
            n.p1[2] = q[i][R + 1];
            const float v = update<KIND>(wt, Wv[i], n, pv[i]);
            if (st_ok[i]) O[zo + colo[i]] = v;
        }
    }
}

// Rows per lane and waves per workgroup (tile 64 x NW*RPT), measured per kind:
// the radius-4 kinds take 8 or 16 waves (taller tiles re-read fewer halo rows);
// the 7-point stencil with BF16 coefficients takes one row per lane and 8
// waves (216 GLUP/s at 512^3 against 148 with the FP32 shape).
template <int KIND, typename CT>
constexpr int naive_rpt() {
    if (KIND == 2 && sizeof(CT) == 2) return 1;
    return KIND == 1 || KIND == 2 ? 8 : (KIND == 4 ? 4 : 1);
}
template <int KIND, typename CT>
constexpr int naive_nw() {
    if (KIND == 2 && sizeof(CT) == 2) return 8;
    return KIND == 1 || KIND == 2 ? 4 : (KIND == 4 ? 8 : 16);
}
// planes per z-chunk from the occupancy of the instance that runs
template <int KIND, typename CT>
int zchunk_for(const dims& d) {
    constexpr int RPT = naive_rpt<KIND, CT>(), NW = naive_nw<KIND, CT>(), TY = NW * RPT;
    const long long txy = (long long)((d.nx + 63) / 64) * ((d.ny + TY - 1) / TY);
    const void* k = reinterpret_cast<const void*>(&naive_step_kernel<KIND, CT, RPT, NW>);
    return pick_zchunk(d.nz, txy, device_slots(k, NW * 64), kind_traits<KIND>::R);
}

template <int KIND, typename CT>
hipError_t launch_kind(const float* cur, const float* prev, float* out, const void* coef,
                       int64_t sk, const dims& d, const host_weights& hw, int zchunk,
                       hipStream_t s) {
    constexpr int RPT = naive_rpt<KIND, CT>();
    constexpr int NW = naive_nw<KIND, CT>();
    constexpr int TY = NW * RPT;
    if (zchunk <= 0) zchunk = zchunk_for<KIND, CT>(d);
    const int gx = (d.nx + 63) / 64, gy = (d.ny + TY - 1) / TY;
    const int gz = (d.nz + zchunk - 1) / zchunk;
    const long long ntiles = (long long)gx * gy * gz;
    if (ntiles <= 0) return hipSuccess;
    if (ntiles > 0x7fffffffLL) return hipErrorInvalidValue;
    weights wt;
    for (int i = 0; i < 5; ++i) wt.w[i] = hw.w[i];
    wt.alpha = hw.alpha;
    wt.lres = hw.lres;
    hipLaunchKernelGGL((naive_step_kernel<KIND, CT, RPT, NW>), dim3((unsigned)ntiles), dim3(NW * 64),
                       0, s,
                       cur, prev, out, static_cast<const CT*>(coef), sk, d.nx, d.ny, d.nz, d.sy,
                       d.sz, d.org(), wt, zchunk, gx, gy, (int)ntiles);
    return hipGetLastError();
}

// Boundary shell copy in two launches.  Rows that lie in the shell (y or z
// outside the interior) are copied whole, one workgroup per row; interior rows
// contribute their 2r boundary points, one thread per point.
__global__ void copy_shell_rows_kernel(float* dst, const float* src, int nx, int ny, int nz,
                                       int r, int64_t sy, int64_t sz, int64_t org) {
    const int rows_y = ny + 2 * r;
    int b = (int)blockIdx.x, y, z;
    if (b < 2 * r * rows_y) {  // the 2r shell planes, every row
        const int zi = b / rows_y;
        z = zi < r ? zi - r : nz + zi - r;
        y = b % rows_y - r;
    } else {  // interior planes, the 2r shell rows
        b -= 2 * r * rows_y;
        z = b / (2 * r);
        const int yi = b % (2 * r);
        y = yi < r ? yi - r : ny + yi - r;
    }
    const int64_t o = org + (int64_t)z * sz + (int64_t)y * sy;
    for (int x = (int)threadIdx.x - r; x < nx + r; x += blockDim.x) dst[o + x] = src[o + x];
}

__global__ void copy_shell_cols_kernel(float* dst, const float* src, int nx, int ny, int nz,
                                       int r, int64_t sy, int64_t sz, int64_t org) {
    const int64_t n = (int64_t)ny * nz * 2 * r;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t row = i / (2 * r);
        const int c = (int)(i % (2 * r));
        const int64_t y = row % ny, z = row / ny;
        const int x = c < r ? c - r : nx + c - r;
        const int64_t o = org + z * sz + y * sy + x;
        dst[o] = src[o];
    }
}

}  // namespace

hipError_t launch_copy_shell(float* dst, const float* src, const dims& d, int r, hipStream_t s) {
    if (d.nx <= 0 || d.ny <= 0 || d.nz <= 0) return hipSuccess;
    if (r > 32) return hipErrorInvalidValue;
    const long long rows = 2LL * r * (d.ny + 2 * r) + 2LL * r * d.nz;
    if (rows > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(copy_shell_rows_kernel, dim3((unsigned)rows), dim3(256), 0, s, dst, src,
                       d.nx, d.ny, d.nz, r, d.sy, d.sz, d.org());
    const long long pts = (long long)d.ny * d.nz * 2 * r;
    const long long blocks = std::min<long long>((pts + 255) / 256, 8192);
    hipLaunchKernelGGL(copy_shell_cols_kernel, dim3((unsigned)blocks), dim3(256), 0, s, dst, src,
                       d.nx, d.ny, d.nz, r, d.sy, d.sz, d.org());
    return hipGetLastError();
}

long long device_slots(const void* kernel, int threads) {
    // cached per (kernel, device): occupancy queries cost host time per launch
    struct entry {
        const void* k;
        int dev, threads;
        long long slots;
    };
    static std::mutex mu;
    static std::vector<entry> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    {
        std::lock_guard<std::mutex> lk(mu);
        for (const entry& e : cache)
            if (e.k == kernel && e.dev == dev && e.threads == threads) return e.slots;
    }
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    const long long slots = (long long)(per_cu > 0 ? per_cu : 1) * (cus > 0 ? cus : 1);
    std::lock_guard<std::mutex> lk(mu);
    cache.push_back({kernel, dev, threads, slots});
    return slots;
}

int pick_zchunk(int nz, long long txy, long long slots, int R) {
    if (nz <= 0) return 1;
    if (txy <= 0 || slots <= 0) return nz;
    int best = nz;
    long long best_cost = -1;
    for (int gz = 1; gz <= nz; ++gz) {
        const int zc = (nz + gz - 1) / gz;
        const long long wgs = txy * ((nz + zc - 1) / zc);
        if (wgs > 0x7fffffffLL) break;
        const long long rounds = (wgs + slots - 1) / slots;
        const long long cost = rounds * (zc + 2 * R);
        if (best_cost < 0 || cost < best_cost) {
            best_cost = cost;
            best = zc;
        }
        if (zc == 1) break;
    }
    return best;
}

hipError_t launch_naive_step(int kind, bool bf16, const float* cur, const float* prev, float* out,
                             const void* coef, int64_t sk, const dims& d, const host_weights& wt,
                             int zchunk, hipStream_t s) {
    switch (kind) {
    case 1: return launch_kind<1, float>(cur, prev, out, coef, sk, d, wt, zchunk, s);
    case 2:
        return bf16 ? launch_kind<2, uint16_t>(cur, prev, out, coef, sk, d, wt, zchunk, s)
                    : launch_kind<2, float>(cur, prev, out, coef, sk, d, wt, zchunk, s);
    case 3:
        return bf16 ? launch_kind<3, uint16_t>(cur, prev, out, coef, sk, d, wt, zchunk, s)
                    : launch_kind<3, float>(cur, prev, out, coef, sk, d, wt, zchunk, s);
    case 4: return launch_kind<4, float>(cur, prev, out, coef, sk, d, wt, zchunk, s);
    case 5:
        return bf16 ? launch_kind<5, uint16_t>(cur, prev, out, coef, sk, d, wt, zchunk, s)
                    : launch_kind<5, float>(cur, prev, out, coef, sk, d, wt, zchunk, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace stn
