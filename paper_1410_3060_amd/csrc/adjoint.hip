// Adjoint (reverse time stepping) of the leapfrog with a domain-sized
// coefficient (Fig. 1e with alpha = c(x)).  The paper has no adjoint; the
// recurrence below is the transpose of the forward one.
//
// Forward:  u_{n+1} = M u_n - u_{n-1},   M = 2I + diag(c) L8.
// Reverse:  lambda_n = 2 lambda_{n+1} - lambda_{n+2} + L8(c * lambda_{n+1})
//           g_c     += lambda_{n+1} * L8(u_n)          (accumulated in FP64)
// with L8 symmetric on the interior (zero outside for the adjoint fields).
//
// One launch performs one reverse step m for all points: a 2.5D stream along
// z like the naive sweep, with the stencil operand v = c * lambda_{m+1} held
// as a register z-queue plus an LDS plane, every operand of the next plane
// loaded while the current one is computed.  lambda_m overwrites
// lambda_{m+2} in place (each point reads its own old value first), so two
// lambda buffers suffice.
//
// The gradient update is the costly part of a step in memory traffic (an
// FP64 read and write per point), so a launch may fold in the gradient terms
// of up to three consecutive steps and the steps around it carry none.  At
// step m the launch knows lambda_{m+2}, lambda_{m+1} and lambda_m, which are
// the multipliers of the terms of steps m+1, m and m-1:
//     g += lambda_{m+2} L8(u_{m+1}) + lambda_{m+1} L8(u_m) + lambda_m L8(u_{m-1})
// (TERMS selects which are present).  Each L8(u) is formed in FP32 from
// per-neighbour differences (u(p+r) - u(p)) + (u(p-r) - u(p)), which are exact
// or nearly so for nearby values, so that the cancellation inside the stencil
// sum costs no FP32 digits; the products and their sum are FP64.
//
// Scaled form (MU).  Where c has no zero, mu = c * lambda obeys
//     mu_m = 2 mu_{m+1} - mu_{m+2} + c L8(mu_{m+1}),
// the forward leapfrog itself, so a step needs no product at every stencil
// load and a step without gradient terms is the forward kernel.  The
// gradient is then accumulated as sum mu_{n+1} L8(u_n) and divided by c once
// at the end, as are lambda_0 = mu_0 / c and lambda_1 = mu_1 / c.
#include <type_traits>

#include "adjoint.h"
#include "common.h"
#include "point_ops.h"

namespace stn {

namespace {

constexpr int R = 4;
constexpr int Q = 2 * R + 1;

// TERMS: bit 0 the term of step m+1, bit 1 of step m, bit 2 of step m-1.
template <typename CT, int NW, int RPT, int TERMS, bool MU>
__global__ __launch_bounds__(NW * 64) void adjoint_step_kernel(
    const float* __restrict__ lam1, float* lam2, const CT* __restrict__ coef,
    const float* u_p, const float* u_c, const float* u_n, double* __restrict__ g, int nx, int ny,
    int nz, int64_t sy, int64_t sz, int64_t org, weights wt, int zchunk, int gx, int gy,
    int ntiles) {
    constexpr int NU = (TERMS & 1) + ((TERMS >> 1) & 1) + ((TERMS >> 2) & 1);
    constexpr int NUA = NU > 0 ? NU : 1;
    constexpr int F = 1 + NU;  // LDS planes: v, then the u fields
    constexpr int TY = NW * RPT;
    constexpr int LW = 64 + 2 * R;
    constexpr int LH = TY + 2 * R;
    constexpr int HYJ = (2 * R + NW - 1) / NW;
    __shared__ float ldv[2][LH][LW];
    __shared__ float ldu[NUA][2][LH][LW];

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
    double* G = g + org;
    const float* U[NUA];
    {
        int f = 0;
        if constexpr ((TERMS & 1) != 0) U[f++] = u_p + org;
        if constexpr ((TERMS & 2) != 0) U[f++] = u_c + org;
        if constexpr ((TERMS & 4) != 0) U[f++] = u_n + org;
        if constexpr (NU == 0) U[0] = nullptr;
    }

    // Points a lane loads: its RPT columns, its share of the 2R y-halo rows
    // and (first 2R*TY threads) one x-halo point.  Loads that are not needed
    // read the interior origin instead, so that no load sits in a branch.
    int64_t co[RPT];
    bool cin[RPT], cld[RPT], cst[RPT];
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
        const int y = y0 + wv + NW * i;
        co[i] = (int64_t)y * sy + x;
        cin[i] = x < nx && y < ny;
        cld[i] = x < nx + R && y < ny + R;
        cst[i] = cin[i];
    }
    int64_t ho[HYJ];
    bool hin[HYJ], hld[HYJ];
    int hrow[HYJ];
#pragma unroll
    for (int j = 0; j < HYJ; ++j) {
        const int hr = wv + NW * j;
        const int ly = hr < R ? hr - R : TY + (hr - R);
        const int y = y0 + ly;
        hrow[j] = ly + R;
        ho[j] = (int64_t)y * sy + x;
        hld[j] = hr < 2 * R && x < nx + R && y < ny + R;
        hin[j] = hld[j] && x < nx && y >= 0 && y < ny;
    }
    const bool hx_any = threadIdx.x < 2 * R * TY;
    int hx_lx = 0, hx_ly = 0;
    int64_t hxo = 0;
    bool hx_in = false, hx_ld = false;
    if (hx_any) {
        const int col = threadIdx.x % (2 * R), row = threadIdx.x / (2 * R);
        const int xx = col < R ? x0 - R + col : x0 + 64 + (col - R);
        const int yy = y0 + row;
        hx_lx = col < R ? col : 64 + R + (col - R);
        hx_ly = row + R;
        hxo = (int64_t)yy * sy + xx;
        hx_ld = xx < nx + R && yy < ny + R;
        hx_in = hx_ld && xx >= 0 && xx < nx && yy < ny;
    }

    // v = c * lambda_{m+1} on the interior, 0 elsewhere
    auto vload = [&](int64_t o, bool in) -> float {
        const int64_t a = in ? o : 0;
        const float l = L1[a];
        const float c = load_coef(C, a);
        return in ? c * l : 0.0f;
    };
    auto uload = [&](int f, int64_t o, bool ok) -> float {
        const float v = U[f][ok ? o : 0];
        return ok ? v : 0.0f;
    };
    auto uload1 = [&](const float* P, int64_t o, bool ok) -> float {
        const float v = P[ok ? o : 0];
        return ok ? v : 0.0f;
    };
    auto zok = [&](int z) { return z >= 0 && z < nz; };

    // register queues: qv[i][k] = v at plane z - R + k; qr = lambda_{m+1} at z .. z + R
    float qv[RPT][Q], qr[RPT][R + 1], qu[NUA][RPT][Q];
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
        qv[i][0] = qr[i][0] = 0.0f;
#pragma unroll
        for (int f = 0; f < NUA; ++f) qu[f][i][0] = 0.0f;
#pragma unroll
        for (int k = 1; k < Q; ++k) {
            const int zz = z0 - R - 1 + k;
            const int64_t o = (int64_t)zz * sz + co[i];
            if constexpr (MU) {
                qv[i][k] = uload1(L1, o, cld[i]);
            } else {
                const bool in = cin[i] && zok(zz);
                const int64_t a = in ? o : 0;
                const float l = L1[a];
                const float c = load_coef(C, a);
                qv[i][k] = in ? c * l : 0.0f;
                if (k >= R) qr[i][k - R] = l;
            }
#pragma unroll
            for (int f = 0; f < NU; ++f) qu[f][i][k] = uload(f, o, cld[i]);
        }
    }
    // operands of plane z (prefetched one plane ahead)
    float nv[RPT], nr[RPT], ncp[RPT], nu[NUA][RPT], l2n[RPT];
    double gn[RPT];
    float hv[HYJ], hu[NUA][HYJ], xv = 0.0f, xu[NUA];
    auto fetch = [&](int z) {
        const int64_t zh = (int64_t)(z + R) * sz, zo = (int64_t)z * sz;
        const bool hin_z = zok(z + R), in_z = zok(z);
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            if constexpr (MU) {
                // mu fields carry a zero boundary shell
                const float l = L1[cld[i] ? zh + co[i] : 0];
                nv[i] = cld[i] ? l : 0.0f;
                nr[i] = 0.0f;
                ncp[i] = load_coef(C, cst[i] ? zo + co[i] : 0);
            } else {
                const bool in = cin[i] && hin_z;
                const int64_t a = in ? zh + co[i] : 0;
                const float l = L1[a];
                const float c = load_coef(C, a);
                nr[i] = l;
                nv[i] = in ? c * l : 0.0f;
            }
#pragma unroll
            for (int f = 0; f < NU; ++f) nu[f][i] = uload(f, zh + co[i], cld[i]);
            l2n[i] = L2[cst[i] ? zo + co[i] : 0];
            if constexpr (NU > 0) gn[i] = G[cst[i] ? zo + co[i] : 0];
        }
#pragma unroll
        for (int j = 0; j < HYJ; ++j) {
            if constexpr (MU)
                hv[j] = uload1(L1, zo + ho[j], hld[j]);
            else
                hv[j] = vload(zo + ho[j], hin[j] && in_z);
#pragma unroll
            for (int f = 0; f < NU; ++f) hu[f][j] = uload(f, zo + ho[j], hld[j]);
        }
        if constexpr (MU)
            xv = uload1(L1, zo + hxo, hx_ld);
        else
            xv = vload(zo + hxo, hx_in && in_z);
#pragma unroll
        for (int f = 0; f < NU; ++f) xu[f] = uload(f, zo + hxo, hx_ld);
    };
    fetch(z0);

    for (int z = z0; z < z1; ++z) {
        const int b = (z - z0) & 1;
        const int64_t zo = (int64_t)z * sz;
        float l2c[RPT], cpt[RPT];
        double gc[RPT];
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
#pragma unroll
            for (int k = 0; k < Q - 1; ++k) qv[i][k] = qv[i][k + 1];
            qv[i][Q - 1] = nv[i];
#pragma unroll
            for (int k = 0; k < R; ++k) qr[i][k] = qr[i][k + 1];
            qr[i][R] = nr[i];
#pragma unroll
            for (int f = 0; f < NU; ++f) {
#pragma unroll
                for (int k = 0; k < Q - 1; ++k) qu[f][i][k] = qu[f][i][k + 1];
                qu[f][i][Q - 1] = nu[f][i];
            }
            l2c[i] = l2n[i];
            cpt[i] = MU ? ncp[i] : 0.0f;
            gc[i] = NU > 0 ? gn[i] : 0.0;
            ldv[b][R + wv + NW * i][R + lane] = qv[i][R];
#pragma unroll
            for (int f = 0; f < NU; ++f) ldu[f][b][R + wv + NW * i][R + lane] = qu[f][i][R];
        }
#pragma unroll
        for (int j = 0; j < HYJ; ++j)
            if (wv + NW * j < 2 * R) {
                ldv[b][hrow[j]][R + lane] = hv[j];
#pragma unroll
                for (int f = 0; f < NU; ++f) ldu[f][b][hrow[j]][R + lane] = hu[f][j];
            }
        if (hx_any) {
            ldv[b][hx_ly][hx_lx] = xv;
#pragma unroll
            for (int f = 0; f < NU; ++f) ldu[f][b][hx_ly][hx_lx] = xu[f];
        }
        if (z + 1 < z1) fetch(z + 1);
        __syncthreads();
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            const int ly = R + wv + NW * i, lx = R + lane;
            nbhd<R> n;
            n.c = qv[i][R];
#pragma unroll
            for (int r = 1; r <= R; ++r) {
                n.pair[0][r - 1] = ldv[b][ly][lx - r] + ldv[b][ly][lx + r];
                n.pair[1][r - 1] = ldv[b][ly - r][lx] + ldv[b][ly + r][lx];
                n.pair[2][r - 1] = qv[i][R - r] + qv[i][R + r];
            }
            const float lam1c = MU ? qv[i][R] : qr[i][0];
            const float lam_m = op_leapfrog(MU ? cpt[i] : 1.0f, op_lap8(wt, n), lam1c, l2c[i]);
            if constexpr (NU > 0) {
                // multipliers of the u fields, in the order they were bound
                float mul[NUA];
                {
                    int f = 0;
                    if constexpr ((TERMS & 1) != 0) mul[f++] = l2c[i];
                    if constexpr ((TERMS & 2) != 0) mul[f++] = lam1c;
                    if constexpr ((TERMS & 4) != 0) mul[f++] = lam_m;
                }
                // L8(u) from per-neighbour differences, which are exact or
                // nearly so for nearby values: the cancellation inside the
                // stencil sum costs no FP32 digits and the value carries about
                // one FP32 rounding; the products and their sum in FP64
                double sum = 0.0;
#pragma unroll
                for (int f = 0; f < NU; ++f) {
                    const float c = qu[f][i][R];
                    float lu = wt.lres * c;
#pragma unroll
                    for (int r = 1; r <= R; ++r) {
                        const float dx = (ldu[f][b][ly][lx - r] - c) + (ldu[f][b][ly][lx + r] - c);
                        const float dy = (ldu[f][b][ly - r][lx] - c) + (ldu[f][b][ly + r][lx] - c);
                        const float dz = (qu[f][i][R - r] - c) + (qu[f][i][R + r] - c);
                        lu = __builtin_fmaf(wt.w[r], (dx + dy) + dz, lu);
                    }
                    sum = f == 0 ? (double)mul[f] * (double)lu
                                 : __builtin_fma((double)mul[f], (double)lu, sum);
                }
                if (cst[i]) G[zo + co[i]] = gc[i] + sum;
            }
            if (cst[i]) L2[zo + co[i]] = lam_m;
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

// Scaled form: dst = c * src on the interior.
template <typename CT>
__global__ void mul_coef_kernel(float* dst, const float* src, const CT* coef, int nx, int ny,
                                int nz, int64_t sy, int64_t sz, int64_t org) {
    const int64_t n = (int64_t)nx * ny * nz;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t x = i % nx, y = (i / nx) % ny, z = i / ((int64_t)nx * ny);
        const int64_t o = org + z * sz + y * sy + x;
        dst[o] = load_coef(coef, o) * src[o];
    }
}

// Scaled form, last pass: g /= c, g_u0 = mu_0 / c, g_um1 = -mu_1 / c.
template <typename CT>
__global__ void finish_mu_kernel(double* g, float* g_u0, float* g_um1, const float* mu0,
                                 const float* mu1, const CT* coef, int nx, int ny, int nz,
                                 int64_t sy, int64_t sz, int64_t org) {
    const int64_t n = (int64_t)nx * ny * nz;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t x = i % nx, y = (i / nx) % ny, z = i / ((int64_t)nx * ny);
        const int64_t o = org + z * sz + y * sy + x;
        const float c = load_coef(coef, o);
        g[o] = g[o] / (double)c;
        g_u0[o] = mu0[o] / c;
        g_um1[o] = -(mu1[o] / c);
    }
}

// flag <- 1 if some interior coefficient is zero, tiny (|c| < 2^-60) or not
// finite: the scaled form cannot be divided back there.  Only 1 is ever
// written, so the order of the stores does not matter.
template <typename CT>
__global__ void coef_check_kernel(int* flag, const CT* coef, int nx, int ny, int nz, int64_t sy,
                                  int64_t sz, int64_t org) {
    const int64_t n = (int64_t)nx * ny * nz;
    bool bad = false;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t x = i % nx, y = (i / nx) % ny, z = i / ((int64_t)nx * ny);
        const float c = fabsf(load_coef(coef, org + z * sz + y * sy + x));
        bad |= !(c >= 0x1p-60f && c <= 3.0e38f);
    }
    if (bad) *flag = 1;
}

__global__ void set_int_kernel(int* p, int v) { *p = v; }

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

}  // namespace

namespace {

template <typename CT, int NW, int RPT, int TERMS, bool MU>
hipError_t launch_terms(const float* lam1, float* lam2, const CT* coef, const float* up,
                        const float* uc, const float* un, double* g, const dims& d,
                        const weights& wt, int zchunk, hipStream_t s) {
    constexpr int TY = NW * RPT;
    const int gx = (d.nx + 63) / 64, gy = (d.ny + TY - 1) / TY;
    if (zchunk <= 0) {
        const long long slots = device_slots(
            reinterpret_cast<const void*>(&adjoint_step_kernel<CT, NW, RPT, TERMS, MU>), NW * 64);
        zchunk = pick_zchunk(d.nz, (long long)gx * gy, slots, R);
    }
    const int gz = (d.nz + zchunk - 1) / zchunk;
    const long long ntiles = (long long)gx * gy * gz;
    if (ntiles <= 0) return hipSuccess;
    if (ntiles > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL((adjoint_step_kernel<CT, NW, RPT, TERMS, MU>), dim3((unsigned)ntiles),
                       dim3(NW * 64), 0,
                       s, lam1, lam2, coef, up, uc, un, g, d.nx, d.ny, d.nz, d.sy, d.sz, d.org(),
                       wt, zchunk, gx, gy, (int)ntiles);
    return hipGetLastError();
}

template <typename CT, bool MU>
hipError_t launch_ct(const float* lam1, float* lam2, const CT* coef, const float* up,
                     const float* uc, const float* un, double* g, const dims& d, const weights& wt,
                     int zchunk, hipStream_t s) {
    const int terms = (up ? 1 : 0) | (uc ? 2 : 0) | (un ? 4 : 0);
#define STN_ADJ_CASE(T, NW, RPT)                                                               \
    case T:                                                                                    \
        return launch_terms<CT, NW, RPT, T, MU>(lam1, lam2, coef, up, uc, un, g, d, wt, zchunk, s)
    // waves per workgroup and rows per lane by term set (registers: one
    // 2R+1 queue per stencil field and row); measured on the 256^3 leapfrog:
    // 4 x 2 ahead of 8 x 1, 8 x 2 and 16 x 1
    switch (terms) {
        STN_ADJ_CASE(0, 4, 4);
        STN_ADJ_CASE(1, 4, 2);
        STN_ADJ_CASE(2, 4, 2);
        STN_ADJ_CASE(3, 4, 2);
        STN_ADJ_CASE(4, 4, 2);
        STN_ADJ_CASE(6, 4, 2);
        STN_ADJ_CASE(7, 4, 2);
    default: return hipErrorInvalidValue;
    }
#undef STN_ADJ_CASE
}

}  // namespace

hipError_t launch_adjoint_step(bool bf16, bool mu, const float* lam1, float* lam2,
                               const void* coef, const float* u_p, const float* u_c,
                               const float* u_n, double* g, const dims& d, const double* w,
                               int zchunk, hipStream_t s) {
    if ((u_p || u_c || u_n) && !g) return hipErrorInvalidValue;
    weights wt;
    for (int i = 0; i < 5; ++i) wt.w[i] = (float)w[i];
    wt.alpha = 1.0f;
    wt.lres = (float)(w[0] + 6.0 * (w[1] + w[2] + w[3] + w[4]));
    const auto* c16 = static_cast<const uint16_t*>(coef);
    const auto* c32 = static_cast<const float*>(coef);
    if (mu)
        return bf16 ? launch_ct<uint16_t, true>(lam1, lam2, c16, u_p, u_c, u_n, g, d, wt, zchunk, s)
                    : launch_ct<float, true>(lam1, lam2, c32, u_p, u_c, u_n, g, d, wt, zchunk, s);
    return bf16 ? launch_ct<uint16_t, false>(lam1, lam2, c16, u_p, u_c, u_n, g, d, wt, zchunk, s)
                : launch_ct<float, false>(lam1, lam2, c32, u_p, u_c, u_n, g, d, wt, zchunk, s);
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

hipError_t launch_mul_coef(float* dst, const float* src, bool bf16, const void* coef,
                           const dims& d, hipStream_t s) {
    if (bf16)
        hipLaunchKernelGGL(mul_coef_kernel<uint16_t>, dim3(util_blocks(d)), dim3(256), 0, s, dst,
                           src, static_cast<const uint16_t*>(coef), d.nx, d.ny, d.nz, d.sy, d.sz,
                           d.org());
    else
        hipLaunchKernelGGL(mul_coef_kernel<float>, dim3(util_blocks(d)), dim3(256), 0, s, dst, src,
                           static_cast<const float*>(coef), d.nx, d.ny, d.nz, d.sy, d.sz, d.org());
    return hipGetLastError();
}

hipError_t launch_finish_mu(double* g, float* g_u0, float* g_um1, const float* mu0,
                            const float* mu1, bool bf16, const void* coef, const dims& d,
                            hipStream_t s) {
    if (bf16)
        hipLaunchKernelGGL(finish_mu_kernel<uint16_t>, dim3(util_blocks(d)), dim3(256), 0, s, g,
                           g_u0, g_um1, mu0, mu1, static_cast<const uint16_t*>(coef), d.nx, d.ny,
                           d.nz, d.sy, d.sz, d.org());
    else
        hipLaunchKernelGGL(finish_mu_kernel<float>, dim3(util_blocks(d)), dim3(256), 0, s, g, g_u0,
                           g_um1, mu0, mu1, static_cast<const float*>(coef), d.nx, d.ny, d.nz,
                           d.sy, d.sz, d.org());
    return hipGetLastError();
}

hipError_t launch_coef_check(int* flag, bool bf16, const void* coef, const dims& d,
                             hipStream_t s) {
    hipLaunchKernelGGL(set_int_kernel, dim3(1), dim3(1), 0, s, flag, 0);
    if (bf16)
        hipLaunchKernelGGL(coef_check_kernel<uint16_t>, dim3(util_blocks(d)), dim3(256), 0, s, flag,
                           static_cast<const uint16_t*>(coef), d.nx, d.ny, d.nz, d.sy, d.sz,
                           d.org());
    else
        hipLaunchKernelGGL(coef_check_kernel<float>, dim3(util_blocks(d)), dim3(256), 0, s, flag,
                           static_cast<const float*>(coef), d.nx, d.ny, d.nz, d.sy, d.sz, d.org());
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
