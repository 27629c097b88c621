// Temporally blocked scheme: diamond tiles along y, a wavefront streaming
// along z inside each diamond (Sect. 4.1-4.3: the "CATS2"/1WD form of
// wavefront diamond blocking; Sect. 5.1: several workers share one diamond).
//
// One launch processes one row of diamonds (the rows of Sect. 4.2 are
// independent inside, dependent across: the launch boundary is the global
// synchronisation between rows).  A workgroup owns one diamond, one x-tile and
// one z-chunk and plays the role of the paper's thread group: its waves split
// every time level of the frontline among themselves (Sect. 5.1) and meet at a
// barrier after each level (Sect. 4.1, multi-thread wavefront).
//
// Inside a workgroup.  Level j (time t0 + j, j = 1 .. 2H-1) of the diamond is
// produced at plane z_j = s - (j-1)R at stream step s: the frontline slope is
// -1/R as in Sect. 4.1, since level j at plane z needs level j-1 at planes
// z-R .. z+R and level j-1 has just produced plane z+R.  Every level keeps the
// last 2R+1 planes of its values in registers (a z-queue per column); the
// centre plane of the level below is staged in LDS for the in-plane
// neighbours.  So all intermediate levels stay on chip and HBM sees, per
// diamond, the lower edge it reads and the upper edge it writes.
//
// Frontier storage.  Between rows the state is the "frontier": for every
// point the two newest levels computed so far (top and the one below).  Row r
// reads the old frontier and writes a new one into a separate pair of
// buffers, so that workgroups that overlap in x or z (they recompute a halo of
// R per remaining level, redundant work instead of communication) never read
// what another workgroup of the same launch writes.  The two pairs alternate
// between rows; one pair is the caller's two time-level buffers.
//
// Boundary values (the shell of width halo) are always read from the caller's
// buffer that holds that time level in the two-buffer convention.
#include <algorithm>
#include <type_traits>

#include "blocked.h"
#include "common.h"
#include "point_ops.h"

namespace stn {

namespace {

template <int KIND, typename CT, int H, int NWV, int XCH, bool G0, bool CRING, int CG, int PD>
__global__ __launch_bounds__(NWV * 64) void blocked_row_kernel(
    const float* ftop_o, const float* fsub_o, float* ftop_n, float* fsub_n,
    const float* __restrict__ hb0, const float* __restrict__ hb1, const CT* __restrict__ coef,
    int64_t sk, int nx, int ny, int nz, int64_t sy, int64_t sz, int64_t org, weights wt, int t0,
    int nt, int first_centre, int XO, int gx, int zchunk, int gz, int ntiles) {
    constexpr int R = kind_traits<KIND>::R;
    constexpr int K = kind_traits<KIND>::K;
    constexpr bool LF = kind_traits<KIND>::leapfrog;
    constexpr int L = 2 * H - 1;
    constexpr int Q = 2 * R + 1;
    constexpr int DW = 2 * R * H;
    constexpr int YT = DW + 2 * R;
    constexpr int XT = 64 * XCH;
    constexpr int NCOL = YT * XCH;
    constexpr int CPT = (NCOL + NWV - 1) / NWV;
    __shared__ float lds[2][L][YT * XT];

    const int tile = xcd_remap(blockIdx.x, ntiles);
    const int g = tile % gx;
    const int zc = (tile / gx) % gz;
    const int di = tile / (gx * gz);
    const int yc = first_centre + di * DW;
    const int x0 = g * XO;
    const int z0 = zc * zchunk;
    const int z1 = min(nz, z0 + zchunk);
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;

    // All addressing is relative to the tile corner (x0 - RL, y_c - RH - R, 0),
    // so a column offset fits in 32 bits.
    const int ybase = yc - R * H - R;
    const int xbase = x0 - R * L;
    const int64_t cb = org + (int64_t)ybase * sy + xbase;
    const float* FT = ftop_o + cb;
    const float* FS = fsub_o + cb;
    float* NT_ = ftop_n + cb;
    float* NS = fsub_n + cb;
    const float* B0 = hb0 + cb;
    const float* B1 = hb1 + cb;
    const CT* W = coef ? coef + cb : nullptr;
    // An always-valid element (the interior origin) for loads whose value is
    // not needed: every load below is issued unconditionally so that no
    // memory operation sits in divergent control flow, which keeps the
    // hardware load counter exact and lets prefetches stay in flight.
    const int64_t safe = -((int64_t)ybase * sy + xbase);

    // ---- per-column geometry, packed (fixed for the whole stream) -----------
    // off: yl*sy + xl.  info bits: [0,8) jold+64, [8,16) jnew+64, [16,24)
    // jxmax+64, 24 needed (exists, within R of the interior), 25 interior in
    // x and y, 26 new frontier written here.  jold/jnew are the levels (t - t0)
    // of the old and new frontier tops; jxmax the last level whose x-range
    // [x0 - R(L-j), x0 + XO + R(L-j)) contains the column.
    int off[CPT];
    uint32_t info[CPT];
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        const int q = wv + NWV * c;
        const int yl = q / XCH;
        const int xl = (q % XCH) * 64 + lane;
        const int y = ybase + yl;
        const int x = xbase + xl;
        off[c] = yl * (int)sy + xl;
        const bool col = q < NCOL;
        const bool yneed = y >= -R && y < ny + R;
        const bool xneed = x >= -R && x < nx + R;
        const bool inr = x >= 0 && x < nx && y >= 0 && y < ny;
        const int xr = max(max(x0 - x, x - (x0 + XO - 1)), 0);
        const int jx = max(L - (xr + R - 1) / R, -1);
        const int d = y - yc;
        int k = d >= 0 ? d / R : (-d - 1) / R;
        const bool own = k <= H - 1;
        if (!own) k = 2 * H - 1 - k;  // flank rows belong to a neighbour of this row
        const int to = min(max(t0 + k, 0), nt);
        const int tn = own ? max(to, min(t0 + 2 * H - 1 - k, nt)) : to;
        const bool outc = col && own && inr && x >= x0 && x < x0 + XO;
        info[c] = (uint32_t)(to - t0 + 64) | ((uint32_t)(tn - t0 + 64) << 8) |
                  ((uint32_t)(jx + 64) << 16) | ((col && yneed && xneed) ? (1u << 24) : 0u) |
                  (inr ? (1u << 25) : 0u) | (outc ? (1u << 26) : 0u);
    }

    auto lds_index = [&](int c) {
        const int q = wv + NWV * c;
        return (q / XCH) * XT + (q % XCH) * 64 + lane;
    };
    // What level j holds at column c and plane z: 0 not needed here, 1
    // boundary value, 2 old frontier top, 3 old frontier level below it,
    // 4 computed by this workgroup.
    auto classify = [&](int c, int j, bool zact, bool zin) -> int {
        const uint32_t f = info[c];
        const int jold = (int)(f & 255u) - 64;
        const int jnew = (int)((f >> 8) & 255u) - 64;
        const int jxm = (int)((f >> 16) & 255u) - 64;
        if (!(zact && (f & (1u << 24)) && j <= jxm)) return 0;
        if (!((f & (1u << 25)) && zin)) return 1;
        if (j == jold) return 2;
        if (j == jold - 1) return 3;
        if (j > jold && j <= jnew) return 4;
        return 0;
    };
    auto level_active = [&](int j, int z) {
        const int t = t0 + j;
        return z >= max(z0 - R * (L - j), -R) && z < min(z1 + R * (L - j), nz + R) && t >= -1 &&
               t <= nt;
    };
    auto halo_src = [&](int j) {
        const int t = t0 + j;
        return LF ? (((t + 1) & 1) ? B1 : B0) : ((t & 1) ? B1 : B0);
    };

    // Value of level j at column c, plane z when it is held in memory (old
    // frontier or boundary); 0 otherwise.
    auto load_sel = [&](int code, int j, int64_t o) -> float {
        const float* src = code == 1 ? halo_src(j) : (code == 3 ? FS : FT);
        const bool mem = code >= 1 && code <= 3;
        const float v = src[mem ? o : safe];
        return mem ? v : 0.0f;
    };
    auto load_level = [&](int c, int j, int z) -> float {
        const int code = classify(c, j, level_active(j, z), z >= 0 && z < nz);
        return load_sel(code, j, (int64_t)z * sz + off[c]);
    };

    // ---- register z-queues: qv[j][c][i] = level j at plane z_j - 2R + i ------
    // With G0 level 0 (never computed here) has no queue: level 1 reads it
    // from memory (cache) and its in-plane plane is prefetched.
    float qv[L][CPT][Q];
#pragma unroll
    for (int j = 0; j < L; ++j)
#pragma unroll
        for (int c = 0; c < CPT; ++c)
#pragma unroll
            for (int i = 0; i < Q; ++i) qv[j][c][i] = 0.0f;

    // ---- coefficient ring (CRING): the coefficients of plane z serve level j
    // at step z + (j-1)R, so each column keeps the last NR = (L-1)R + 1 planes:
    // cr[c][i][k] = coefficient k at plane s - i.  Loaded once per diamond,
    // one step ahead (cp).  Without the ring, level j loads its coefficients
    // from memory (cache) when it computes.
    constexpr int NR = CRING ? (L - 1) * R + 1 : 1;
    constexpr int KR = CRING ? kslots<KIND> : 1;
    float cr[CPT][NR][KR];
    // PD = prefetch depth in steps (1 or 2): the number of prefetch slots
    float cp[PD][CPT][KR];
#pragma unroll
    for (int c = 0; c < CPT; ++c)
#pragma unroll
        for (int k = 0; k < KR; ++k) {
#pragma unroll
            for (int d = 0; d < PD; ++d) cp[d][c][k] = 0.0f;
#pragma unroll
            for (int i = 0; i < NR; ++i) cr[c][i][k] = 0.0f;
        }
    // a column needs coefficients if it computes some level of this diamond
    // and lies in level 1's x-range; planes of level 1's range, interior only
    auto ring_load = [&](int s, auto slot) {
        constexpr int SL = decltype(slot)::value;
        if constexpr (CRING) {
            const bool zok = s >= 0 && s < nz && s >= z0 - R * (L - 1) && s < z1 + R * (L - 1);
#pragma unroll
            for (int c = 0; c < CPT; ++c) {
                const uint32_t f = info[c];
                const int jold = (int)(f & 255u) - 64;
                const int jnew = (int)((f >> 8) & 255u) - 64;
                const int jxm = (int)((f >> 16) & 255u) - 64;
                const bool need = zok && (f & (1u << 24)) && (f & (1u << 25)) && jnew > jold &&
                                  jxm >= 1;
#pragma unroll
                for (int k = 0; k < KR; ++k) {
                    const float v = load_coef(W, need ? k * sk + (int64_t)s * sz + off[c] : safe);
                    cp[SL][c][k] = need ? v : 0.0f;
                }
            }
        }
    };

    // Values every level reads from memory (frontier or boundary) are loaded
    // two stream steps ahead, into slot s % 2: pf[slot][j][c], and for the
    // leapfrog pp[slot][c] = u_{t0-1} under level 1.  The stream loop is
    // unrolled by two so that the slots stay registers.
    float pf[PD][L + 1][CPT];
    float pp[PD][CPT];
    auto prefetch = [&](int s, auto slot) {
        constexpr int SL = decltype(slot)::value;
#pragma unroll
        for (int c = 0; c < CPT; ++c) asm volatile("" : "+v"(info[c]));
#pragma unroll
        for (int j = 0; j <= L; ++j) {
            // with G0, level 0 is prefetched at the plane level 1 reads in-plane
            const int z = (G0 && j == 0) ? s : s - (j - 1) * R;
            const bool za = level_active(j, z);
            const bool zin = z >= 0 && z < nz;
            const int64_t zo = (int64_t)z * sz;
#pragma unroll
            for (int c = 0; c < CPT; ++c) {
                const int code = classify(c, j, za, zin);
                pf[SL][j][c] = load_sel(code, j, zo + off[c]);
                if (LF && j == 1) {
                    const float v = FS[code == 4 ? zo + off[c] : safe];
                    pp[SL][c] = code == 4 ? v : 0.0f;
                }
            }
        }
        ring_load(s, slot);
    };

    const int s_begin = z0 - R * (L + 1);
    const int s_end = z1 + R * (L - 1);
    prefetch(s_begin, std::integral_constant<int, 0>{});
    if (PD == 2 && s_begin + 1 < s_end) prefetch(s_begin + 1, std::integral_constant<int, PD - 1>{});
    auto step = [&](int s, auto par) {
        constexpr int set = decltype(par)::value;  // LDS set read by step s: parity of s - s_begin
        constexpr int SL = PD == 2 ? set : 0;      // prefetch slot holding step s
        float cur[L + 1][CPT];
        float curp[CPT];
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            curp[c] = pp[SL][c];
#pragma unroll
            for (int j = 0; j <= L; ++j) cur[j][c] = pf[SL][j][c];
            if constexpr (CRING) {
#pragma unroll
                for (int i = NR - 1; i > 0; --i)
#pragma unroll
                    for (int k = 0; k < KR; ++k) cr[c][i][k] = cr[c][i - 1][k];
#pragma unroll
                for (int k = 0; k < KR; ++k) cr[c][0][k] = cp[SL][c][k];
            }
        }
        if constexpr (PD == 2) {
            if (s + 2 < s_end) prefetch(s + 2, std::integral_constant<int, SL>{});
        } else {
            if (s + 1 < s_end) prefetch(s + 1, std::integral_constant<int, 0>{});
        }
#pragma unroll
        for (int c = 0; c < CPT; ++c) asm volatile("" : "+v"(info[c]));
#pragma unroll
        for (int j = 0; j <= L; ++j) {
            const int z = s - (j - 1) * R;
            const bool za = level_active(j, z);
            const bool zin = z >= 0 && z < nz;
            const bool zout = z >= z0 && z < z1;
            const int64_t zo = (int64_t)z * sz;
            const int jp = j >= 1 ? j - 1 : 0;
            const float* P = lds[set][jp];
            int code[CPT];
#pragma unroll
            for (int c = 0; c < CPT; ++c) code[c] = classify(c, j, za, zin);
            // Columns are processed in groups of CG: phase 1 issues every memory
            // read of the group's updates, phase 2 consumes them, so one memory
            // round trip serves CG columns while only CG columns' operands are live.
#pragma unroll
            for (int g0 = 0; g0 < CPT; g0 += CG) {
            // phase 1: every memory read of this level for the group, before any use
            float Wv[CG][kslots<KIND>];
            float zq[CG][Q];
            float pv[CG];
#pragma unroll
            for (int cc = 0; cc < CG; ++cc) {
                const int c = g0 + cc < CPT ? g0 + cc : CPT - 1;
#pragma unroll
                for (int k = 0; k < kslots<KIND>; ++k) Wv[cc][k] = 0.0f;
                pv[cc] = 0.0f;
                const bool cmp = g0 + cc < CPT && j >= 1 && code[c] == 4;
                if constexpr (K > 0 && !CRING) {
                    if (j >= 1) {
#pragma unroll
                        for (int k = 0; k < K; ++k)
                            Wv[cc][k] = load_coef(W, cmp ? k * sk + zo + off[c] : safe);
                    }
                }
                if (cmp) {
                    if constexpr (K > 0 && CRING) {
#pragma unroll
                        for (int k = 0; k < K; ++k) Wv[cc][k] = cr[c][(j >= 1 ? j - 1 : 0) * R][k];
                    }
                    if constexpr (LF) {
                        if (j == 1)
                            pv[cc] = curp[c];
                        else if (!(G0 && j == 2))
                            pv[cc] = qv[j >= 2 ? j - 2 : 0][c][0];
                    }
                }
                // level 0 operands from memory (G0): issued for every column
                if constexpr (G0 && LF) {
                    if (j == 2) {
                        const float v = load_level(c, 0, z);
                        if (cmp) pv[cc] = v;
                    }
                }
                if (G0 && j == 1) {
#pragma unroll
                    for (int i = 0; i < Q; ++i) zq[cc][i] = load_level(c, 0, z - R + i);
                }
                if (!(G0 && j == 1)) {
#pragma unroll
                    for (int i = 0; i < Q; ++i) zq[cc][i] = qv[jp][c][i];
                }
            }
            // phase 2: compute, push, write back
#pragma unroll
            for (int cc = 0; cc < CG; ++cc) {
                const int c = g0 + cc < CPT ? g0 + cc : CPT - 1;
                if (g0 + cc >= CPT) continue;
                // with G0, cur[0] holds level 0 at the in-plane plane, not at z
                float v = (G0 && j == 0) ? 0.0f : cur[j][c];
                if (j >= 1 && code[c] == 4) {
                    const int li = lds_index(c);
                    nbhd<R> n;
                    n.c = zq[cc][R];
#pragma unroll
                    for (int r = 1; r <= R; ++r) {
                        n.pair[0][r - 1] = P[li - r] + P[li + r];
                        n.pair[1][r - 1] = P[li - r * XT] + P[li + r * XT];
                        n.pair[2][r - 1] = zq[cc][R - r] + zq[cc][R + r];
                    }
                    n.m1[0] = P[li - 1];
                    n.p1[0] = P[li + 1];
                    n.m1[1] = P[li - XT];
                    n.p1[1] = P[li + XT];
                    n.m1[2] = zq[cc][R - 1];
                    n.p1[2] = zq[cc][R + 1];
                    v = update<KIND>(wt, Wv[cc], n, pv[cc]);
                }
                if (j < L && !(G0 && j == 0)) {
                    const int jq = j < L ? j : 0;
#pragma unroll
                    for (int i = 0; i < Q - 1; ++i) qv[jq][c][i] = qv[jq][c][i + 1];
                    qv[jq][c][Q - 1] = v;
                }
                if (G0 && j == 0) v = load_level(c, 0, z);  // only written back, rarely
                if (za && zout && (info[c] & (1u << 26))) {
                    const int jnew = (int)((info[c] >> 8) & 255u) - 64;
                    if (j == jnew)
                        NT_[zo + off[c]] = v;
                    else if (j == jnew - 1)
                        NS[zo + off[c]] = v;
                }
            }
            // keep the next group's loads from being hoisted above this one
            if constexpr (CG < CPT) __builtin_amdgcn_sched_barrier(0);
            }
        }
        // Stage the planes the next step reads in-plane: level j-1 at plane
        // z_j(s+1) sits at queue index R+1 now (it is R steps old).
#pragma unroll
        for (int j = 1; j <= L; ++j)
#pragma unroll
            for (int c = 0; c < CPT; ++c)
                if (wv + NWV * c < NCOL)
                    lds[set ^ 1][j - 1][lds_index(c)] =
                        (G0 && j == 1) ? pf[PD == 2 ? SL ^ 1 : 0][0][c] : qv[j - 1][c][R + 1];
        __syncthreads();
    };
    for (int s = s_begin; s < s_end; s += 2) {
        step(s, std::integral_constant<int, 0>{});
        if (s + 1 < s_end) step(s + 1, std::integral_constant<int, 1>{});
    }
}

// Register and LDS budget per (R, H): workgroup shape and columns per lane.
template <int KIND, typename CT, int H, int NWV, int XCH, bool G0 = false, bool CRING = false,
          int CG = 8, int PD = 2>
hipError_t launch_cfg(const blocked_row_args& a, hipStream_t s) {
    constexpr int R = kind_traits<KIND>::R;
    const int ntiles = a.n_diamonds * a.gx * a.gz;
    if (ntiles <= 0) return hipSuccess;
    weights wt;
    for (int i = 0; i < 5; ++i) wt.w[i] = a.wt.w[i];
    wt.alpha = a.wt.alpha;
    (void)R;
    hipLaunchKernelGGL((blocked_row_kernel<KIND, CT, H, NWV, XCH, G0, CRING, CG, PD>), dim3(ntiles), dim3(NWV * 64), 0,
                       s, a.ftop_o, a.fsub_o, a.ftop_n, a.fsub_n, a.hb0, a.hb1,
                       static_cast<const CT*>(a.coef), a.sk, a.d.nx, a.d.ny, a.d.nz, a.d.sy,
                       a.d.sz, a.d.org(), wt, (int)a.t0, (int)a.nt, a.first_centre, a.xo, a.gx,
                       a.zchunk, a.gz, ntiles);
    return hipGetLastError();
}

// Workgroup shape per (kind, H): waves, 64-lane x chunks, level 0 read from
// cache (G0), coefficient ring in registers (CRING).  Register budget per
// column: L z-queues of 2R+1 values, plus (L-1)R+1 coefficient planes of K
// values with the ring.
template <int KIND, typename CT>
hipError_t launch_kind(const blocked_row_args& a, hipStream_t s) {
    constexpr int R = kind_traits<KIND>::R;
    const int H = a.dw / (2 * R);
    if constexpr (KIND == 1) {
        if (H == 2) return launch_cfg<KIND, CT, 2, 6, 2>(a, s);
        if (H == 4) return launch_cfg<KIND, CT, 4, 10, 2>(a, s);
        if (H == 6) return launch_cfg<KIND, CT, 6, 7, 2>(a, s);
    } else if constexpr (KIND == 2) {
        if (H == 2) return launch_cfg<KIND, CT, 2, 6, 2, false, true>(a, s);
        if (H == 4) return launch_cfg<KIND, CT, 4, 10, 1, false, true>(a, s);
        if (H == 6) return launch_cfg<KIND, CT, 6, 7, 2>(a, s);
    } else if constexpr (KIND == 5) {
        if (H == 2) return launch_cfg<KIND, CT, 2, 12, 2, true, false, 1, 1>(a, s);
    } else {
        if (H == 2) return launch_cfg<KIND, CT, 2, 12, 2, true, false, 1, 1>(a, s);
    }
    return hipErrorInvalidValue;
}

// x chunks of the configuration above (host side)
int cfg_xch(int kind, int H) { return (kind == 2 && H == 4) ? 1 : 2; }

}  // namespace

bool blocked_supported(int kind, int dw) {
    const int R = (kind == 1 || kind == 2) ? 1 : 4;
    if (dw % (2 * R) != 0) return false;
    const int H = dw / (2 * R);
    return R == 1 ? (H == 2 || H == 4 || H == 6) : (H == 2);
}

int blocked_default_dw(int kind) { return (kind == 1 || kind == 2) ? 8 : 16; }

int blocked_max_xo(int kind, int dw) {
    const int R = (kind == 1 || kind == 2) ? 1 : 4;
    const int H = dw / (2 * R);
    const int L = 2 * H - 1;
    return 64 * cfg_xch(kind, H) - 2 * R * L;
}

hipError_t launch_blocked_row(int kind, bool bf16, const blocked_row_args& a, hipStream_t s) {
    switch (kind) {
    case 1: return launch_kind<1, float>(a, s);
    case 2: return bf16 ? launch_kind<2, uint16_t>(a, s) : launch_kind<2, float>(a, s);
    case 3: return bf16 ? launch_kind<3, uint16_t>(a, s) : launch_kind<3, float>(a, s);
    case 4: return launch_kind<4, float>(a, s);
    case 5: return bf16 ? launch_kind<5, uint16_t>(a, s) : launch_kind<5, float>(a, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace stn
