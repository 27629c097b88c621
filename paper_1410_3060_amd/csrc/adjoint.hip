// Adjoint (reverse time stepping) of the leapfrog with a domain-sized
// coefficient (Fig. 1e with alpha = c(x)).  The paper has no adjoint; the
// recurrence below is the transpose of the forward one.
//
// Forward:  u_{n+1} = M u_n - u_{n-1},   M = 2I + diag(c) L8.
// Reverse:  lambda_n = 2 lambda_{n+1} - lambda_{n+2} + L8(c * lambda_{n+1})
//           g_c     += lambda_{n+1} * L8(u_n)          (accumulated in FP64)
// with L8 symmetric on the interior (zero outside for the adjoint fields).
//
// One launch performs one reverse step for all points, fused: a 2.5D stream
// along z like the naive sweep, with two stencil operands (v = c * lambda_{n+1}
// and u_n), each held as a register z-queue plus an LDS plane.  lambda_n
// overwrites lambda_{n+2} in place (each point reads its own old value
// first), so two lambda buffers suffice.  The gradient term uses an FP64
// evaluation of L8(u_n) from the FP32 values, so that the cancellation inside
// the stencil sum does not cost FP32 digits in the coefficient gradient.
#include "adjoint.h"
#include "common.h"
#include "point_ops.h"

namespace stn {

namespace {

constexpr int NT = 256;
constexpr int NW = 4;
constexpr int R = 4;
constexpr int Q = 2 * R + 1;

struct w64 {
    double w[5];
};

template <typename CT, int RPT>
__global__ __launch_bounds__(NT) void adjoint_step_kernel(
    const float* __restrict__ lam1, float* lam2, const CT* __restrict__ coef,
    const float* __restrict__ us, double* __restrict__ g, int nx, int ny, int nz, int64_t sy,
    int64_t sz, int64_t org, weights wt, w64 wd, int zchunk, int gx, int gy, int ntiles) {
    constexpr int TY = NW * RPT;
    constexpr int LW = 64 + 2 * R;
    constexpr int LH = TY + 2 * R;
    __shared__ float ldv[2][LH][LW];
    __shared__ float ldu[2][LH][LW];

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

    const float* L1 = lam1 + org;
    float* L2 = lam2 + org;
    const CT* C = coef + org;
    const float* U = us + org;
    double* G = g + org;

    // v = c * lambda on the interior, 0 on the boundary shell
    auto vload = [&](int64_t zo, int64_t co, int xx, int yy, int zz) -> float {
        const bool in = xx >= 0 && xx < nx && yy >= 0 && yy < ny && zz >= 0 && zz < nz;
        return in ? load_coef(C, zo + co) * L1[zo + co] : 0.0f;
    };

    int64_t colo[RPT];
    int ys[RPT];
    bool ld_ok[RPT], st_ok[RPT];
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
        const int y = y0 + wv + NW * i;
        ys[i] = y;
        colo[i] = (int64_t)y * sy + x;
        ld_ok[i] = (x < nx + R) && (y < ny + R);
        st_ok[i] = (x < nx) && (y < ny);
    }
    constexpr int HYJ = (2 * R + NW - 1) / NW;
    int64_t hyo[HYJ];
    int hy_y[HYJ], hy_row[HYJ];
    bool hy_ok[HYJ];
#pragma unroll
    for (int j = 0; j < HYJ; ++j) {
        const int hr = wv + NW * j;
        const int ly = hr < R ? hr - R : TY + (hr - R);
        const int y = y0 + ly;
        hy_row[j] = ly + R;
        hy_y[j] = y;
        hyo[j] = (int64_t)y * sy + x;
        hy_ok[j] = (hr < 2 * R) && (x < nx + R) && (y < ny + R);
    }
    const int hxi = threadIdx.x;
    const bool hx_any = hxi < 2 * R * TY;
    int hx_lx = 0, hx_ly = 0, hx_x = 0, hx_y = 0;
    int64_t hxo = 0;
    bool hx_ok = false;
    if (hx_any) {
        const int col = hxi % (2 * R), row = hxi / (2 * R);
        hx_x = col < R ? x0 - R + col : x0 + 64 + (col - R);
        hx_y = y0 + row;
        hx_lx = (col < R ? col : 64 + R + (col - R));
        hx_ly = row + R;
        hxo = (int64_t)hx_y * sy + hx_x;
        hx_ok = (hx_x < nx + R) && (hx_y < ny + R);
    }

    float qv[RPT][Q], qu[RPT][Q];
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
#pragma unroll
        for (int k = 1; k < Q; ++k) {
            const int zz = z0 - R - 1 + k;
            const int64_t zo = (int64_t)zz * sz;
            qv[i][k] = ld_ok[i] ? vload(zo, colo[i], x, ys[i], zz) : 0.0f;
            qu[i][k] = ld_ok[i] ? U[zo + colo[i]] : 0.0f;
        }
        qv[i][0] = qu[i][0] = 0.0f;
    }

    for (int z = z0; z < z1; ++z) {
        const int b = (z - z0) & 1;
        const int64_t zo = (int64_t)z * sz;
        const int zn = z + R;
        const int64_t zno = (int64_t)zn * sz;
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
#pragma unroll
            for (int k = 0; k < Q - 1; ++k) {
                qv[i][k] = qv[i][k + 1];
                qu[i][k] = qu[i][k + 1];
            }
            qv[i][Q - 1] = ld_ok[i] ? vload(zno, colo[i], x, ys[i], zn) : 0.0f;
            qu[i][Q - 1] = ld_ok[i] ? U[zno + colo[i]] : 0.0f;
            ldv[b][R + wv + NW * i][R + lane] = qv[i][R];
            ldu[b][R + wv + NW * i][R + lane] = qu[i][R];
        }
#pragma unroll
        for (int j = 0; j < HYJ; ++j)
            if (wv + NW * j < 2 * R) {
                ldv[b][hy_row[j]][R + lane] = hy_ok[j] ? vload(zo, hyo[j], x, hy_y[j], z) : 0.0f;
                ldu[b][hy_row[j]][R + lane] = hy_ok[j] ? U[zo + hyo[j]] : 0.0f;
            }
        if (hx_any) {
            ldv[b][hx_ly][hx_lx] = hx_ok ? vload(zo, hxo, hx_x, hx_y, z) : 0.0f;
            ldu[b][hx_ly][hx_lx] = hx_ok ? U[zo + hxo] : 0.0f;
        }
        float l1c[RPT], l2c[RPT];
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            l1c[i] = st_ok[i] ? L1[zo + colo[i]] : 0.0f;
            l2c[i] = st_ok[i] ? L2[zo + colo[i]] : 0.0f;
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            const int ly = R + wv + NW * i, lx = R + lane;
            nbhd<R> nv;
            nv.c = qv[i][R];
            double lu = wd.w[0] * (double)qu[i][R];
#pragma unroll
            for (int r = 1; r <= R; ++r) {
                nv.pair[0][r - 1] = ldv[b][ly][lx - r] + ldv[b][ly][lx + r];
                nv.pair[1][r - 1] = ldv[b][ly - r][lx] + ldv[b][ly + r][lx];
                nv.pair[2][r - 1] = qv[i][R - r] + qv[i][R + r];
                const double px = (double)ldu[b][ly][lx - r] + (double)ldu[b][ly][lx + r];
                const double py = (double)ldu[b][ly - r][lx] + (double)ldu[b][ly + r][lx];
                const double pz = (double)qu[i][R - r] + (double)qu[i][R + r];
                lu = __builtin_fma(wd.w[r], (px + py) + pz, lu);
            }
            const float lv = op_lap8(wt, nv);
            const float lam_n = op_leapfrog(1.0f, lv, l1c[i], l2c[i]);
            if (st_ok[i]) {
                L2[zo + colo[i]] = lam_n;
                G[zo + colo[i]] += (double)l1c[i] * lu;
            }
        }
    }
}

// dst = a * src on the interior (a = 1 or -1), dst shell untouched.
__global__ void scale_copy_kernel(float* dst, const float* src, float a, int nx, int ny, int nz,
                                  int64_t sy, int64_t sz, int64_t org) {
    const int64_t n = (int64_t)nx * ny * nz;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t x = i % nx, y = (i / nx) % ny, z = i / ((int64_t)nx * ny);
        const int64_t o = org + z * sz + y * sy + x;
        dst[o] = a * src[o];
    }
}

template <typename T>
__global__ void zero_kernel(T* dst, int nx, int ny, int nz, int64_t sy, int64_t sz, int64_t org) {
    const int64_t n = (int64_t)nx * ny * nz;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t x = i % nx, y = (i / nx) % ny, z = i / ((int64_t)nx * ny);
        dst[org + z * sz + y * sy + x] = T(0);
    }
}

__global__ void zero_span_kernel(float* dst, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        dst[i] = 0.0f;
}

int util_blocks(const dims& d) {
    const long long n = (long long)d.nx * d.ny * d.nz;
    long long b = (n + 255) / 256;
    return (int)(b > 8192 ? 8192 : (b < 1 ? 1 : b));
}

constexpr int ADJ_RPT = 4;

}  // namespace

hipError_t launch_adjoint_step(bool bf16, const float* lam1, float* lam2, const void* coef,
                               const float* us, double* g, const dims& d, const double* w,
                               int zchunk, hipStream_t s) {
    constexpr int TY = NW * ADJ_RPT;
    const int gx = (d.nx + 63) / 64, gy = (d.ny + TY - 1) / TY;
    if (zchunk <= 0) {
        const long long txy = (long long)gx * gy;
        long long nzc = (2048 + txy - 1) / txy;
        zchunk = (int)((d.nz + nzc - 1) / nzc);
        if (zchunk < 4 * R) zchunk = 4 * R;
        if (zchunk > d.nz) zchunk = d.nz;
    }
    const int gz = (d.nz + zchunk - 1) / zchunk;
    const long long ntiles = (long long)gx * gy * gz;
    if (ntiles <= 0) return hipSuccess;
    weights wt;
    w64 wd;
    for (int i = 0; i < 5; ++i) {
        wt.w[i] = (float)w[i];
        wd.w[i] = w[i];
    }
    wt.alpha = 1.0f;
    if (bf16)
        hipLaunchKernelGGL((adjoint_step_kernel<uint16_t, ADJ_RPT>), dim3((unsigned)ntiles), dim3(NT),
                           0, s, lam1, lam2, static_cast<const uint16_t*>(coef), us, g, d.nx, d.ny,
                           d.nz, d.sy, d.sz, d.org(), wt, wd, zchunk, gx, gy, (int)ntiles);
    else
        hipLaunchKernelGGL((adjoint_step_kernel<float, ADJ_RPT>), dim3((unsigned)ntiles), dim3(NT), 0,
                           s, lam1, lam2, static_cast<const float*>(coef), us, g, d.nx, d.ny, d.nz,
                           d.sy, d.sz, d.org(), wt, wd, zchunk, gx, gy, (int)ntiles);
    return hipGetLastError();
}

hipError_t launch_scale_copy(float* dst, const float* src, float a, const dims& d, hipStream_t s) {
    hipLaunchKernelGGL(scale_copy_kernel, dim3(util_blocks(d)), dim3(256), 0, s, dst, src, a, d.nx,
                       d.ny, d.nz, d.sy, d.sz, d.org());
    return hipGetLastError();
}

hipError_t launch_zero_f32(float* dst, const dims& d, hipStream_t s) {
    hipLaunchKernelGGL(zero_kernel<float>, dim3(util_blocks(d)), dim3(256), 0, s, dst, d.nx, d.ny,
                       d.nz, d.sy, d.sz, d.org());
    return hipGetLastError();
}

hipError_t launch_zero_f64(double* dst, const dims& d, hipStream_t s) {
    hipLaunchKernelGGL(zero_kernel<double>, dim3(util_blocks(d)), dim3(256), 0, s, dst, d.nx, d.ny,
                       d.nz, d.sy, d.sz, d.org());
    return hipGetLastError();
}

hipError_t launch_zero_span(float* dst, size_t n, hipStream_t s) {
    size_t b = (n + 255) / 256;
    if (b > 8192) b = 8192;
    if (b < 1) b = 1;
    hipLaunchKernelGGL(zero_span_kernel, dim3((unsigned)b), dim3(256), 0, s, dst, n);
    return hipGetLastError();
}

}  // namespace stn
