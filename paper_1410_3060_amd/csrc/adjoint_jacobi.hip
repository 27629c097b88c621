// Adjoint (reverse time stepping) of the first-order variable-coefficient
// stencils of Fig. 1c (7 points, K = 7) and Fig. 1d (25 points, K = 13).  The
// paper treats only the forward updates; the kernels below evaluate the
// transposed operator and the coefficient gradients.
//
// Forward:  u_{t+1} = A(W) u_t on the interior, boundary shell fixed.
// Reverse:  lambda_t = A^T lambda_{t+1}  (lambda_nt = the seed),
//           dJ/dW_k(p) = sum_t lambda_{t+1}(p) * (the value W_k multiplies at p
//           in step t),  dJ/du_0 = lambda_0.
//
// 7 points.  A^T is again an operator of the Fig. 1c form: the neighbour
// x-1 of q is the point whose x+1 tap reaches q, so
//     W'_0(q) = W_0(q),
//     W'_1(q) = W_2(q - e_x),  W'_2(q) = W_1(q + e_x),
//     W'_3(q) = W_4(q - e_y),  W'_4(q) = W_3(q + e_y),
//     W'_5(q) = W_6(q - e_z),  W'_6(q) = W_5(q + e_z),
// each zero where the shifted point lies outside the interior.  These arrays
// are built once per adjoint call (transpose7_kernel) and a reverse step is
// the forward Fig. 1c sweep applied to lambda, whose boundary shell is zero.
//
// 25 points.  A^T gives every neighbour its own coefficient,
//     (A^T l)(q) = W_0(q) l(q) + sum_{r,a} [P_ra(q - r e_a) + P_ra(q + r e_a)],
// with the products P_ra = W_ra * l on the interior (0 outside).
// adj25_step_kernel streams along z like the naive sweep: the z products sit
// in register queues, the x and y products of the current plane (with their
// halos) in LDS, so every coefficient and lambda value is read from HBM once
// per step.
//
// Gradients.  jacobi_grad_kernel adds the terms of G consecutive steps in
// one pass: for each point it reads u_s and lambda_{s+1} of the G steps and
// reads and writes the K FP64 gradient arrays once, accumulating in FP64
// registers; the FP64 read-modify-write, the largest part of the traffic, is
// thereby shared by G steps.
#include "adjoint.h"
#include "common.h"
#include "point_ops.h"

namespace stn {

namespace {

// W' of the 7-point transpose on the interior; dst arrays at element stride dk.
template <typename CT>
__global__ void transpose7_kernel(CT* __restrict__ dst, int64_t dk, const CT* __restrict__ src,
                                 int64_t sk, int nx, int ny, int nz, int64_t sy, int64_t sz,
                                 int64_t org) {
    const int64_t n = (int64_t)nx * ny * nz;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(i % nx), y = (int)((i / nx) % ny), z = (int)(i / ((int64_t)nx * ny));
        const int64_t o = org + (int64_t)z * sz + (int64_t)y * sy + x;
        const CT zero = CT(0);
        dst[o] = src[o];
        dst[1 * dk + o] = x > 0 ? src[2 * sk + o - 1] : zero;
        dst[2 * dk + o] = x < nx - 1 ? src[1 * sk + o + 1] : zero;
        dst[3 * dk + o] = y > 0 ? src[4 * sk + o - sy] : zero;
        dst[4 * dk + o] = y < ny - 1 ? src[3 * sk + o + sy] : zero;
        dst[5 * dk + o] = z > 0 ? src[6 * sk + o - sz] : zero;
        dst[6 * dk + o] = z < nz - 1 ? src[5 * sk + o + sz] : zero;
    }
}

// One reverse step of the 25-point stencil: lam0 <- A^T lam1 on the interior.
// A workgroup of NW waves owns a 64 x NW tile of columns (one row per wave)
// and streams through a chunk of planes.  Loads that a lane does not need
// address the interior origin and are discarded, so no load sits in a branch.
template <typename CT, int NW>
__global__ __launch_bounds__(NW * 64) void adj25_step_kernel(
    const float* __restrict__ lam1, float* __restrict__ lam0, const CT* __restrict__ coef,
    int64_t sk, int nx, int ny, int nz, int64_t sy, int64_t sz, int64_t org, int zchunk, int gx,
    int gy, int ntiles) {
    constexpr int R = 4, Q = 2 * R + 1, TY = NW;
    constexpr int LW = 64 + 2 * R, LH = TY + 2 * R;
    constexpr int HYJ = (2 * R + NW - 1) / NW;
    // x products with their x halo, y products with their y halo
    __shared__ float lpx[2][R][TY][LW];
    __shared__ float lpy[2][R][LH][64];

    const int tile = xcd_remap(blockIdx.x, ntiles);
    const int bx = tile % gx;
    const int by = (tile / gx) % gy;
    const int bz = tile / (gx * gy);
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int x0 = bx * 64, y0 = by * TY;
    const int z0 = bz * zchunk;
    const int z1 = min(nz, z0 + zchunk);
    const int x = x0 + lane, y = y0 + wv;

    const float* L1 = lam1 + org;
    float* L0 = lam0 + org;
    const CT* C = coef + org;

    const int64_t co = (int64_t)y * sy + x;
    const bool cin = x < nx && y < ny;
    int64_t ho[HYJ];
    bool hin[HYJ];
    int hrow[HYJ];
#pragma unroll
    for (int j = 0; j < HYJ; ++j) {
        const int hr = wv + NW * j;
        const int ly = hr < R ? hr - R : TY + (hr - R);
        const int yy = y0 + ly;
        hrow[j] = ly + R;
        ho[j] = (int64_t)yy * sy + x;
        hin[j] = hr < 2 * R && x < nx && yy >= 0 && yy < ny;
    }
    const bool hx_any = threadIdx.x < 2 * R * TY;
    int hx_lx = 0, hx_ly = 0;
    int64_t hxo = 0;
    bool hx_in = false;
    if (hx_any) {
        const int col = threadIdx.x % (2 * R), row = threadIdx.x / (2 * R);
        const int xx = col < R ? x0 - R + col : x0 + 64 + (col - R);
        const int yy = y0 + row;
        hx_lx = col < R ? col : 64 + R + (col - R);
        hx_ly = row;
        hxo = (int64_t)yy * sy + xx;
        hx_in = xx >= 0 && xx < nx && yy < ny;
    }

    // coefficient k and lambda at offset o, zero where `ok` is false
    auto cf = [&](int k, int64_t o, bool ok) -> float {
        const float v = load_coef(C, (int64_t)k * sk + (ok ? o : 0));
        return ok ? v : 0.0f;
    };
    auto lf = [&](int64_t o, bool ok) -> float {
        const float v = L1[ok ? o : 0];
        return ok ? v : 0.0f;
    };

    // qz[r-1][k]: z product of radius r at plane z - R + k; ql[k]: lambda at z + k
    float qz[R][Q], ql[R + 1];
#pragma unroll
    for (int r = 0; r < R; ++r) qz[r][0] = 0.0f;
    ql[0] = 0.0f;
#pragma unroll
    for (int k = 1; k < Q; ++k) {
        const int zz = z0 - R - 1 + k;
        const bool in = cin && zz >= 0 && zz < nz;
        const int64_t o = (int64_t)zz * sz + co;
        const float l = lf(o, in);
#pragma unroll
        for (int r = 1; r <= R; ++r) qz[r - 1][k] = cf(3 * r, o, in) * l;
        if (k >= R) ql[k - R] = l;
    }

    // operands of plane z, loaded one plane ahead
    float nl, nzc[R], nw0, nwx[R], nwy[R], hl[HYJ], hwy[HYJ][R], xl, xw[R];
    auto fetch = [&](int z) {
        const int64_t zl = (int64_t)(z + R) * sz + co, zo = (int64_t)z * sz;
        const bool inl = cin && z + R < nz;
        nl = lf(zl, inl);
#pragma unroll
        for (int r = 1; r <= R; ++r) nzc[r - 1] = cf(3 * r, zl, inl);
        nw0 = cf(0, zo + co, cin);
#pragma unroll
        for (int r = 1; r <= R; ++r) {
            nwx[r - 1] = cf(3 * r - 2, zo + co, cin);
            nwy[r - 1] = cf(3 * r - 1, zo + co, cin);
        }
#pragma unroll
        for (int j = 0; j < HYJ; ++j) {
            hl[j] = lf(zo + ho[j], hin[j]);
#pragma unroll
            for (int r = 1; r <= R; ++r) hwy[j][r - 1] = cf(3 * r - 1, zo + ho[j], hin[j]);
        }
        xl = lf(zo + hxo, hx_in);
#pragma unroll
        for (int r = 1; r <= R; ++r) xw[r - 1] = cf(3 * r - 2, zo + hxo, hx_in);
    };
    fetch(z0);

    for (int z = z0; z < z1; ++z) {
        const int b = (z - z0) & 1;
        const int64_t zo = (int64_t)z * sz;
#pragma unroll
        for (int r = 0; r < R; ++r) {
#pragma unroll
            for (int k = 0; k < Q - 1; ++k) qz[r][k] = qz[r][k + 1];
            qz[r][Q - 1] = nzc[r] * nl;
        }
#pragma unroll
        for (int k = 0; k < R; ++k) ql[k] = ql[k + 1];
        ql[R] = nl;
        const float lc = ql[0];
        const float p0 = nw0 * lc;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            lpx[b][r][wv][R + lane] = nwx[r] * lc;
            lpy[b][r][R + wv][lane] = nwy[r] * lc;
        }
#pragma unroll
        for (int j = 0; j < HYJ; ++j)
            if (wv + NW * j < 2 * R) {
#pragma unroll
                for (int r = 0; r < R; ++r) lpy[b][r][hrow[j]][lane] = hwy[j][r] * hl[j];
            }
        if (hx_any) {
#pragma unroll
            for (int r = 0; r < R; ++r) lpx[b][r][hx_ly][hx_lx] = xw[r] * xl;
        }
        if (z + 1 < z1) fetch(z + 1);
        __syncthreads();
        float acc = p0;
#pragma unroll
        for (int r = 1; r <= R; ++r) {
            acc += lpx[b][r - 1][wv][R + lane - r] + lpx[b][r - 1][wv][R + lane + r];
            acc += lpy[b][r - 1][R + wv - r][lane] + lpy[b][r - 1][R + wv + r][lane];
            acc += qz[r - 1][R - r] + qz[r - 1][R + r];
        }
        if (cin) L0[zo + co] = acc;
    }
}

// Fields of one gradient group: u_s and lambda_{s+1} for G consecutive steps.
struct grad_fields {
    const float* u[kGradGroupMax];
    const float* l[kGradGroupMax];
};

// g_k += sum over the G steps s of lambda_{s+1} * tap_k(u_s), FP64.
// Taps: kind 2, u(p + o_k) for o = 0, -x, +x, -y, +y, -z, +z; kind 3, u(p) for
// W_0 and u(p - r e_a) + u(p + r e_a) for W_{3(r-1)+1+a}.  The u fields carry
// the boundary shell, which the taps of boundary points read.
template <int KIND, int G, int NW>
__global__ __launch_bounds__(NW * 64) void jacobi_grad_kernel(
    grad_fields fs, double* __restrict__ g, int64_t sk, int nx, int ny, int nz, int64_t sy,
    int64_t sz, int64_t org, int zchunk, int gx, int gy, int ntiles) {
    constexpr int R = kind_traits<KIND>::R, K = kind_traits<KIND>::K;
    constexpr int Q = 2 * R + 1, TY = NW;
    constexpr int LW = 64 + 2 * R, LH = TY + 2 * R;
    constexpr int HYJ = (2 * R + NW - 1) / NW;
    __shared__ float ldu[2][G][LH][LW];

    const int tile = xcd_remap(blockIdx.x, ntiles);
    const int bx = tile % gx;
    const int by = (tile / gx) % gy;
    const int bz = tile / (gx * gy);
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int x0 = bx * 64, y0 = by * TY;
    const int z0 = bz * zchunk;
    const int z1 = min(nz, z0 + zchunk);
    const int x = x0 + lane, y = y0 + wv;

    const float* U[G];
    const float* L[G];
#pragma unroll
    for (int s = 0; s < G; ++s) {
        U[s] = fs.u[s] + org;
        L[s] = fs.l[s] + org;
    }
    double* Gp = g + org;

    const int64_t co = (int64_t)y * sy + x;
    const bool cin = x < nx && y < ny;
    const bool cld = x < nx + R && y < ny + R;  // inside the padded box
    int64_t ho[HYJ];
    bool hld[HYJ];
    int hrow[HYJ];
#pragma unroll
    for (int j = 0; j < HYJ; ++j) {
        const int hr = wv + NW * j;
        const int ly = hr < R ? hr - R : TY + (hr - R);
        const int yy = y0 + ly;
        hrow[j] = ly + R;
        ho[j] = (int64_t)yy * sy + x;
        hld[j] = hr < 2 * R && x < nx + R && yy < ny + R;
    }
    const bool hx_any = threadIdx.x < 2 * R * TY;
    int hx_lx = 0, hx_ly = 0;
    int64_t hxo = 0;
    bool hx_ld = false;
    if (hx_any) {
        const int col = threadIdx.x % (2 * R), row = threadIdx.x / (2 * R);
        const int xx = col < R ? x0 - R + col : x0 + 64 + (col - R);
        const int yy = y0 + row;
        hx_lx = col < R ? col : 64 + R + (col - R);
        hx_ly = row + R;
        hxo = (int64_t)yy * sy + xx;
        hx_ld = xx < nx + R && yy < ny + R;
    }
    auto ld = [&](const float* P, int64_t o, bool ok) -> float {
        const float v = P[ok ? o : 0];
        return ok ? v : 0.0f;
    };

    float qu[G][Q];
#pragma unroll
    for (int s = 0; s < G; ++s) {
        qu[s][0] = 0.0f;
#pragma unroll
        for (int k = 1; k < Q; ++k) qu[s][k] = ld(U[s], (int64_t)(z0 - R - 1 + k) * sz + co, cld);
    }
    float nu[G], nl[G], hu[G][HYJ], xu[G];
    double gn[K];
    auto fetch = [&](int z) {
        const int64_t zo = (int64_t)z * sz, zl = (int64_t)(z + R) * sz + co;
#pragma unroll
        for (int s = 0; s < G; ++s) {
            nu[s] = ld(U[s], zl, cld);
            nl[s] = ld(L[s], zo + co, cin);
#pragma unroll
            for (int j = 0; j < HYJ; ++j) hu[s][j] = ld(U[s], zo + ho[j], hld[j]);
            xu[s] = ld(U[s], zo + hxo, hx_ld);
        }
#pragma unroll
        for (int k = 0; k < K; ++k) gn[k] = Gp[(int64_t)k * sk + (cin ? zo + co : 0)];
    };
    fetch(z0);

    for (int z = z0; z < z1; ++z) {
        const int b = (z - z0) & 1;
        const int64_t zo = (int64_t)z * sz;
        double acc[K];
        float lc[G];
#pragma unroll
        for (int s = 0; s < G; ++s) {
#pragma unroll
            for (int k = 0; k < Q - 1; ++k) qu[s][k] = qu[s][k + 1];
            qu[s][Q - 1] = nu[s];
            lc[s] = nl[s];
            ldu[b][s][R + wv][R + lane] = qu[s][R];
#pragma unroll
            for (int j = 0; j < HYJ; ++j)
                if (wv + NW * j < 2 * R) ldu[b][s][hrow[j]][R + lane] = hu[s][j];
            if (hx_any) ldu[b][s][hx_ly][hx_lx] = xu[s];
        }
#pragma unroll
        for (int k = 0; k < K; ++k) acc[k] = gn[k];
        if (z + 1 < z1) fetch(z + 1);
        __syncthreads();
        const int ly = R + wv, lx = R + lane;
#pragma unroll
        for (int s = 0; s < G; ++s) {
            const double l = (double)lc[s];
            if constexpr (KIND == 2) {
                const float t[7] = {qu[s][R],
                                    ldu[b][s][ly][lx - 1], ldu[b][s][ly][lx + 1],
                                    ldu[b][s][ly - 1][lx], ldu[b][s][ly + 1][lx],
                                    qu[s][R - 1],          qu[s][R + 1]};
#pragma unroll
                for (int k = 0; k < 7; ++k) acc[k] = __builtin_fma(l, (double)t[k], acc[k]);
            } else {
                acc[0] = __builtin_fma(l, (double)qu[s][R], acc[0]);
#pragma unroll
                for (int r = 1; r <= R; ++r) {
                    const double px = (double)ldu[b][s][ly][lx - r] + (double)ldu[b][s][ly][lx + r];
                    const double py = (double)ldu[b][s][ly - r][lx] + (double)ldu[b][s][ly + r][lx];
                    const double pz = (double)qu[s][R - r] + (double)qu[s][R + r];
                    acc[3 * r - 2] = __builtin_fma(l, px, acc[3 * r - 2]);
                    acc[3 * r - 1] = __builtin_fma(l, py, acc[3 * r - 1]);
                    acc[3 * r] = __builtin_fma(l, pz, acc[3 * r]);
                }
            }
        }
        if (cin) {
#pragma unroll
            for (int k = 0; k < K; ++k) Gp[(int64_t)k * sk + zo + co] = acc[k];
        }
    }
}

int util_grid(const dims& d) {
    const long long n = (long long)d.nx * d.ny * d.nz;
    long long b = (n + 255) / 256;
    return (int)(b > 8192 ? 8192 : (b < 1 ? 1 : b));
}

constexpr int kAdjNW = 16;   // waves per workgroup of the 25-point reverse step
constexpr int kGradNW = 8;   // waves per workgroup of the gradient kernel (2 per SIMD: 256 VGPRs)

// Launch geometry of a z-streaming kernel over 64 x TY column tiles.
struct stream_grid {
    int gx, gy, gz, zchunk;
    long long ntiles;
};

stream_grid make_grid(const void* kernel, int threads, int TY, int R, const dims& d, int zchunk) {
    stream_grid sgr;
    sgr.gx = (d.nx + 63) / 64;
    sgr.gy = (d.ny + TY - 1) / TY;
    if (zchunk <= 0)
        zchunk = pick_zchunk(d.nz, (long long)sgr.gx * sgr.gy, device_slots(kernel, threads), R);
    sgr.zchunk = zchunk;
    sgr.gz = (d.nz + zchunk - 1) / zchunk;
    sgr.ntiles = (long long)sgr.gx * sgr.gy * sgr.gz;
    return sgr;
}

template <typename CT>
hipError_t launch_adj25(const float* lam1, float* lam0, const CT* coef, int64_t sk, const dims& d,
                        int zchunk, hipStream_t s) {
    auto* kern = &adj25_step_kernel<CT, kAdjNW>;
    const stream_grid sgr =
        make_grid(reinterpret_cast<const void*>(kern), kAdjNW * 64, kAdjNW, 4, d, zchunk);
    if (sgr.ntiles <= 0) return hipSuccess;
    if (sgr.ntiles > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(kern, dim3((unsigned)sgr.ntiles), dim3(kAdjNW * 64), 0, s, lam1, lam0, coef,
                       sk, d.nx, d.ny, d.nz, d.sy, d.sz, d.org(), sgr.zchunk, sgr.gx, sgr.gy,
                       (int)sgr.ntiles);
    return hipGetLastError();
}

template <int KIND, int G>
hipError_t launch_grad_g(const grad_fields& fs, double* g, int64_t sk, const dims& d, int zchunk,
                         hipStream_t s) {
    auto* kern = &jacobi_grad_kernel<KIND, G, kGradNW>;
    const stream_grid sgr = make_grid(reinterpret_cast<const void*>(kern), kGradNW * 64, kGradNW,
                                      kind_traits<KIND>::R, d, zchunk);
    if (sgr.ntiles <= 0) return hipSuccess;
    if (sgr.ntiles > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(kern, dim3((unsigned)sgr.ntiles), dim3(kGradNW * 64), 0, s, fs, g, sk, d.nx,
                       d.ny, d.nz, d.sy, d.sz, d.org(), sgr.zchunk, sgr.gx, sgr.gy,
                       (int)sgr.ntiles);
    return hipGetLastError();
}

template <int KIND>
hipError_t launch_grad_kind(int n, const grad_fields& fs, double* g, int64_t sk, const dims& d,
                            int zchunk, hipStream_t s) {
    switch (n) {
    case 1: return launch_grad_g<KIND, 1>(fs, g, sk, d, zchunk, s);
    case 2: return launch_grad_g<KIND, 2>(fs, g, sk, d, zchunk, s);
    case 3: return launch_grad_g<KIND, 3>(fs, g, sk, d, zchunk, s);
    case 4: return launch_grad_g<KIND, 4>(fs, g, sk, d, zchunk, s);
    case 5: return launch_grad_g<KIND, 5>(fs, g, sk, d, zchunk, s);
    case 6: return launch_grad_g<KIND, 6>(fs, g, sk, d, zchunk, s);
    default:
        if constexpr (grad_group_max(KIND) > 6) {
            if (n == 7) return launch_grad_g<KIND, 7>(fs, g, sk, d, zchunk, s);
            if (n == 8) return launch_grad_g<KIND, 8>(fs, g, sk, d, zchunk, s);
        }
        return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_transpose7(void* dst, int64_t dk, const void* src, int64_t sk, bool bf16,
                             const dims& d, hipStream_t s) {
    if (bf16)
        hipLaunchKernelGGL(transpose7_kernel<uint16_t>, dim3(util_grid(d)), dim3(256), 0, s,
                           static_cast<uint16_t*>(dst), dk, static_cast<const uint16_t*>(src), sk,
                           d.nx, d.ny, d.nz, d.sy, d.sz, d.org());
    else
        hipLaunchKernelGGL(transpose7_kernel<float>, dim3(util_grid(d)), dim3(256), 0, s,
                           static_cast<float*>(dst), dk, static_cast<const float*>(src), sk, d.nx,
                           d.ny, d.nz, d.sy, d.sz, d.org());
    return hipGetLastError();
}

hipError_t launch_adj25_step(bool bf16, const float* lam1, float* lam0, const void* coef,
                             int64_t sk, const dims& d, int zchunk, hipStream_t s) {
    return bf16 ? launch_adj25<uint16_t>(lam1, lam0, static_cast<const uint16_t*>(coef), sk, d,
                                         zchunk, s)
                : launch_adj25<float>(lam1, lam0, static_cast<const float*>(coef), sk, d, zchunk,
                                      s);
}

hipError_t launch_jacobi_grad(int kind, int n, const float* const* u, const float* const* lam,
                              double* g, int64_t sk, const dims& d, int zchunk, hipStream_t s) {
    if (n < 1 || n > grad_group_max(kind)) return hipErrorInvalidValue;
    grad_fields fs{};
    for (int i = 0; i < n; ++i) {
        fs.u[i] = u[i];
        fs.l[i] = lam[i];
    }
    if (kind == 2) return launch_grad_kind<2>(n, fs, g, sk, d, zchunk, s);
    if (kind == 3) return launch_grad_kind<3>(n, fs, g, sk, d, zchunk, s);
    return hipErrorInvalidValue;
}

}  // namespace stn
