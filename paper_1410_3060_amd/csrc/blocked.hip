// Temporally blocked scheme for the radius-1 stencils (Fig. 1b, 1c): diamond
// tiles along y, a wavefront streaming along z inside each diamond
// (Sect. 4.1-4.3: the "CATS2"/1WD form of wavefront diamond blocking;
// Sect. 5.1: several workers share one diamond).  The radius-4 stencils take
// the multi-workgroup form in mwd.hip; the entry points below dispatch to it.
//
// One launch processes one row of diamonds (the rows of Sect. 4.2 are
// independent inside, dependent across: the launch boundary is the global
// synchronisation between rows).  A workgroup owns one diamond, one x-tile and
// one z-chunk and plays the role of the paper's thread group: its waves split
// every time level of the frontline among themselves (Sect. 5.1) and meet at a
// barrier once per stream step.
//
// Inside a workgroup.  Level j (time t0 + j, j = 1 .. 2H-1) of the diamond is
// produced at plane z_j = s - (j-1)R at stream step s: the frontline slope is
// -1/R as in Sect. 4.1, since level j at plane z needs level j-1 at planes
// z-R .. z+R and level j-1 has just produced plane z+R.  Every level keeps the
// last 2R+1 planes of its values in registers (a z-queue per column).  The
// in-plane neighbours of level j are those of level j-1 at plane z_j, which
// level j-1 produced R steps earlier: all LDS planes are therefore staged at
// the end of the previous step and one barrier per step suffices.
//
// Each wave owns whole rows (one y per column slot), so everything that
// depends on y -- where the row sits in the diamond, which levels it reads
// from the old frontier and which it computes -- is uniform across the wave
// and decided with scalar branches.  Per step a row reads from memory only
// the two old-frontier levels below the diamond and a shell value (prefetched
// ahead) and, where the registers allow (CRING), one plane of coefficients
// into a register ring that serves every level (a coefficient is then read
// once per diamond; otherwise once per level).  Levels are computed
// across the whole tile width; values near the x edges that depend on columns
// outside the tile are wrong but never stored and never read by a stored
// value (the overlapped-halo argument: level j is correct R*j columns inside
// the tile edge, and only columns x0 .. x0+XO-1 are written).
//
// Frontier storage.  Between rows the state is the "frontier": for every
// point the two newest levels computed so far (top and the one below).  Row r
// reads the old frontier and writes a new one into a separate pair of
// buffers, so that workgroups that overlap in x or z (they recompute a halo
// instead of communicating) never read what another workgroup of the same
// launch writes.  The boundary shell is time independent and both frontier
// buffers carry it, so boundary values are read like frontier values.
#include <algorithm>
#include <mutex>
#include <type_traits>

#include "blocked.h"
#include "common.h"
#include "point_ops.h"

namespace stn {

namespace {

template <int N>
using ic = std::integral_constant<int, N>;

using rsrc_t = __amdgpu_buffer_rsrc_t;

// Byte offset beyond every buffer the kernel touches (every buffer is sized
// below 2^31 bytes): a buffer load there returns 0 and a buffer store is
// dropped, so an operand a row does not need costs neither a branch nor a
// memory access.
constexpr uint32_t kNone = 0x80000000u;

__device__ __forceinline__ rsrc_t make_rsrc(const void* p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ float bload(rsrc_t r, uint32_t voff, uint32_t soff) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
__device__ __forceinline__ void bstore(rsrc_t r, float v, uint32_t voff, uint32_t soff) {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, voff, soff, 0);
}
// Coefficient array k as a buffer.  In a level's update BF16 arrays are read
// a 32-bit word at a time (the compiler waits for every 16-bit buffer load at
// once, which would serialise the level's K loads); the resource starts at the
// word-aligned address at or below the array and `mis` (0 or 2 bytes) is the
// array's offset from it.
struct coef_rsrc {
    rsrc_t r;
    uint32_t mis;
};
// coefficient loads: FP32, or BF16 expanded exactly to FP32 (as load_coef)
__device__ __forceinline__ float cload(const float*, const coef_rsrc& c, uint32_t voff,
                                       uint32_t soff) {
    return bload(c.r, voff, soff);
}
// Prefetched coefficients, read steps before their use, take 16-bit loads
// and stay raw (the stored bits) until cexpand where they enter the ring: an
// expansion next to the load would make the wave wait for the load there.
// Coefficients read in a level's update take the word loads below.
__device__ __forceinline__ float cload_raw(const float*, const coef_rsrc& c, uint32_t voff,
                                           uint32_t soff) {
    return bload(c.r, voff, soff);
}
__device__ __forceinline__ float cload_raw(const uint16_t*, const coef_rsrc& c, uint32_t voff,
                                           uint32_t soff) {
    const uint32_t vo = voff >= kNone ? voff : voff + c.mis;
    return __uint_as_float(static_cast<uint32_t>(__builtin_amdgcn_raw_buffer_load_b16(c.r, vo, soff, 0)));
}
__device__ __forceinline__ float cexpand(const float*, float raw) { return raw; }
__device__ __forceinline__ float cexpand(const uint16_t*, float raw) {
    return __uint_as_float(__float_as_uint(raw) << 16);
}
__device__ __forceinline__ float cload(const uint16_t*, const coef_rsrc& c, uint32_t voff,
                                       uint32_t soff) {
    // the value sits in the high half of the word 2 bytes below it when its
    // byte offset from the aligned base is 2 mod 4, else in the low half
    const uint32_t adj = (voff + soff + c.mis) & 2u;
    const uint32_t vo = voff >= kNone ? voff : voff + c.mis - adj;
    const uint32_t w = __builtin_amdgcn_raw_buffer_load_b32(c.r, vo, soff, 0);
    return __uint_as_float(adj ? (w & 0xffff0000u) : (w << 16));
}

// A copy of a wave-uniform value that the compiler cannot move out of a
// loop: a test against it stays a compare at its use instead of a lane mask
// kept (or spilled) across the loop.
__device__ __forceinline__ int opaque_s(int v) {
    int r;
    asm volatile("s_mov_b32 %0, %1" : "=s"(r) : "s"(v));
    return r;
}

template <int KIND, typename CT, int H, int NWV, int XCH, bool CRING, bool G0, int PD, bool WIN,
          bool ALN>
__global__ __launch_bounds__(NWV * 64) void blocked_row_kernel(
    const float* ftop_o, const float* fsub_o, float* ftop_n, float* fsub_n,
    const CT* __restrict__ coef, int64_t sk, int nx, int ny, int nz, int hh, int64_t sy,
    int64_t sz, std::conditional_t<WIN, uint64_t, uint32_t> field_bytes,
    std::conditional_t<WIN, uint64_t, uint32_t> coef_bytes, weights wt, int t0, int nt,
    int first_centre, int XO, int gx, int zchunk, int gz, int ntiles) {
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
    constexpr int NR = CRING ? (L - 1) * R + 1 : 1;  // coefficient planes in the ring
    constexpr int KR = CRING ? kslots<KIND> : 1;
    constexpr int NSH = L * R + 1;                   // planes in the shell ring
    constexpr uint32_t CB = sizeof(CT);
    // ALN: BF16 arrays word-aligned, strides even (the host checks), so an
    // element's half of its 32-bit word depends on its column only
    static_assert(!ALN || (CB == 2 && !CRING), "ALN is for BF16 loads in the level update");
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
    const int wvu = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));

    // Tile corner (x0 - RL, y_c - RH - R).  Offsets are bytes from the
    // buffers' bases: row part (y+h)*sy + (x+h), plane part (z-zw)*sz.  Fields
    // below 2 GiB are based at their padded origin (zw = -h); larger ones
    // (WIN) at plane zw of the workgroup's window, below every plane its
    // z-chunk touches (at most R(L+2) below z0), which the host keeps below
    // 2^31 bytes.
    const int ybase = yc - R * H - R;
    const int xbase = x0 - R * L;
    const int zw = WIN ? max(z0 - R * (L + 2), -hh) : -hh;
    // window start in bytes of a field and of a coefficient array (0 if !WIN)
    const uint64_t wfb = WIN ? (uint64_t)(zw + hh) * (uint64_t)sz * 4u : 0u;
    const uint64_t wcb = WIN ? (uint64_t)(zw + hh) * (uint64_t)sz * CB : 0u;
    // bytes from the window start to the end of the array, at most 2^31 - 1
    // (offsets at or beyond kNone stay outside)
    auto nrec = [](uint64_t total, uint64_t off) -> uint32_t {
        const uint64_t r = total > off ? total - off : 0u;
        return (uint32_t)(r < 0x7fffffffull ? r : 0x7fffffffull);
    };
    auto buf = [&](const void* p) -> rsrc_t {
        if constexpr (WIN)
            return make_rsrc(static_cast<const char*>(p) + wfb, nrec(field_bytes, wfb));
        else
            return make_rsrc(p, field_bytes);
    };
    const rsrc_t rFT = buf(ftop_o);
    const rsrc_t rFS = buf(fsub_o);
    const rsrc_t rNT = buf(ftop_n);
    const rsrc_t rNS = buf(fsub_n);
    const uint32_t sz4 = (uint32_t)(sz * 4);
    const uint32_t szc = (uint32_t)(sz * CB);
    // field / coefficient plane bytes
    auto pf = [&](int z) { return WIN ? (uint32_t)(z - zw) * sz4 : (uint32_t)(z + hh) * sz4; };
    auto pc_ = [&](int z) { return WIN ? (uint32_t)(z - zw) * szc : (uint32_t)(z + hh) * szc; };
    auto crs = [&](int k) -> coef_rsrc {
        const uint64_t nrc = WIN ? nrec(coef_bytes, wcb) : (uint64_t)coef_bytes;
        if constexpr (CB == 2) {
            const uintptr_t a = reinterpret_cast<uintptr_t>(coef + (int64_t)k * sk) + wcb;
            const uint32_t mis = (uint32_t)(a & 2u);
            // every word that holds an element of the window
            const uint64_t nr = nrc + mis + 2u;
            return {make_rsrc(reinterpret_cast<const void*>(a - mis),
                              (uint32_t)(nr < 0x7fffffffull ? nr : 0x7fffffffull)),
                    mis};
        } else if constexpr (WIN) {
            return {make_rsrc(reinterpret_cast<const char*>(coef + (int64_t)k * sk) + wcb,
                              (uint32_t)nrc),
                    0u};
        } else {
            return {make_rsrc(coef + (int64_t)k * sk, coef_bytes), 0u};
        }
    };
    // the tile reaches outside [0, nx) in x: boundary columns hold the shell
    const bool xb = xbase < 0 || xbase + XT > nx;

    // ---- rows (uniform per wave) and columns (per lane) ----------------------
    // rt: 0 row not needed, 1 boundary-shell row, 2 interior row.
    // jo, jn: levels (t - t0) of the old and new frontier tops of the row;
    // the diamond computes levels jo+1 .. jn of the row (none off the diamond).
    int rt[CPT], jo[CPT], jn[CPT];
    bool own[CPT];
    uint32_t vf[CPT], vc[CPT];  // byte offsets of the column's row in a field / coefficient plane
    uint32_t vw[CPT], vsel[CPT];  // ALN: the column's word offset, byte selector of its half
    int lidx[CPT];              // LDS index of the column
    bool xin[CPT], outx[CPT];
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        const int q = wvu + NWV * c;
        const int yl = q / XCH;
        const int xl = (q % XCH) * 64 + lane;
        const int y = ybase + yl;
        const int x = xbase + xl;
        const bool valid = q < NCOL;
        rt[c] = (!valid || y < -R || y >= ny + R) ? 0 : ((y < 0 || y >= ny) ? 1 : 2);
        const int d = y - yc;
        int k = d >= 0 ? d / R : (-d - 1) / R;
        own[c] = k <= H - 1;
        if (!own[c]) k = 2 * H - 1 - k;  // flank rows belong to a neighbour of this row
        const int to = min(max(t0 + k, 0), nt);
        const int tn = own[c] ? max(to, min(t0 + 2 * H - 1 - k, nt)) : to;
        jo[c] = to - t0;
        jn[c] = tn - t0;
        const int xc = min(max(x, -R), nx + R - 1);
        const uint32_t e = rt[c] != 0 ? (uint32_t)((int64_t)(y + hh) * sy + (xc + hh)) : 0u;
        vf[c] = e * 4u;
        vc[c] = e * CB;
        if constexpr (ALN) {
            vw[c] = vc[c] & ~3u;
            vsel[c] = (vc[c] & 2u) ? 0x03020c0cu : 0x01000c0cu;  // high / low half to bits 31..16
        }
        lidx[c] = valid ? yl * XT + xl : 0;
        xin[c] = x >= 0 && x < nx;
        outx[c] = x >= x0 && x < x0 + XO && x < nx;
    }

    auto level_active = [&](int j, int z) __attribute__((always_inline)) {
        const int t = t0 + j;
        return z >= max(z0 - R * (L - j), -R) && z < min(z1 + R * (L - j), nz + R) && t >= -1 &&
               t <= nt;
    };

    // Steps of the fast range (every level z_j = s - (j-1)R inside [0, nz)
    // and inside its active window, see run) read operands whose need
    // depends on the row alone: the lane offset of each such load (kNone
    // where the row does not need it) and its plane's offset from plane s
    // are fixed here, so a fast step forms a load's offset with one add.
    // An unneeded load keeps a valid plane, so kNone + offset stays below
    // 2^32 and beyond the buffer.
    uint32_t ft_v[CPT], fs_v[CPT], fh_v[CPT], fc_v[CPT];
    uint32_t ft_p[CPT], fs_p[CPT], fh_p[CPT], fl_p[CPT], f0_p[CPT], fp_p[CPT];
    uint32_t fl_v[CPT], f0_v[CPT], fp_v[CPT];
    bool f0_sub[CPT];
    const uint32_t pf0 = pf(0);
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        const bool intr = rt[c] == 2;
        // (the plane offset must stay uniform across the wave: it is the
        // load's scalar offset)
        auto off = [&](bool ok, int d, uint32_t& v, uint32_t& p) {
            v = ok ? vf[c] : kNone;
            p = ok ? pf0 + (uint32_t)d * sz4 : pf0;
        };
        off(intr && jo[c] <= L, (1 - jo[c]) * R, ft_v[c], ft_p[c]);
        off(intr && jo[c] >= 1 && jo[c] <= L + 1, (2 - jo[c]) * R, fs_v[c], fs_p[c]);
        fh_v[c] = (rt[c] == 1 || (intr && xb && !xin[c])) ? vf[c] : kNone;
        fh_p[c] = pf0 + (uint32_t)R * sz4;
        off(intr && jo[c] == 0 && jn[c] >= 1, 0, fl_v[c], fl_p[c]);
        off(rt[c] >= 1, 1, f0_v[c], f0_p[c]);
        off(intr && jo[c] == 1 && jn[c] >= 2, -R, fp_v[c], fp_p[c]);
        f0_sub[c] = intr && jo[c] == 1;
        fc_v[c] = (intr && own[c] && jn[c] > jo[c]) ? vc[c] : kNone;
    }

    // ---- register state -------------------------------------------------------
    // qv[j][c][i] = level j at plane z_j - 2R + i (level 0 has none with G0)
    float qv[L][CPT][Q];
    // coefficient ring: cr[c][i][k] = coefficient k at plane s - i
    float cr[CPT][NR][KR];
    // shell ring: sh[c][i] = old frontier top at plane s + R - i, i.e. the value
    // of level j at its plane is sh[c][jR] wherever that point is boundary
    // shell (time independent), and for rows whose top is level 0 it is level 0
    float sh[CPT][NSH];
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
#pragma unroll
        for (int j = 0; j < L; ++j)
#pragma unroll
            for (int i = 0; i < Q; ++i) qv[j][c][i] = 0.0f;
#pragma unroll
        for (int i = 0; i < NR; ++i)
#pragma unroll
            for (int k = 0; k < KR; ++k) cr[c][i][k] = 0.0f;
#pragma unroll
        for (int i = 0; i < NSH; ++i) sh[c][i] = 0.0f;
    }
    // Memory operands of step s, loaded PD steps ahead into slot (s - s_begin) % PD:
    // pt/ps = old frontier top/sub at their planes, pl = u_{t0-1} at plane s
    // (leapfrog rows that compute level 1), p0 = level 0 at plane s+1 (G0: the
    // in-plane plane of level 1 next step), pp = level 0 at plane s - R of rows
    // whose top is level 1 (G0 leapfrog: the older level of their level 2),
    // ph = the shell ring's input at plane s + R, pc = coefficients at plane s.
    float pt[PD][CPT], ps[PD][CPT], pl[PD][CPT], p0[PD][CPT], pp[PD][CPT], ph[PD][CPT];
    float pc[PD][CPT][KR];

    auto prefetch = [&](int s, auto slot) __attribute__((always_inline)) {
        constexpr int SL = decltype(slot)::value;
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            const bool intr = rt[c] == 2;
            const int zt = s - (jo[c] - 1) * R, zs = s - (jo[c] - 2) * R;
            const bool okt = intr && jo[c] <= L && zt >= 0 && zt < nz && level_active(jo[c], zt);
            const bool oks = intr && jo[c] >= 1 && zs >= 0 && zs < nz && level_active(jo[c] - 1, zs);
            pt[SL][c] = bload(rFT, okt ? vf[c] : kNone, okt ? pf(zt) : 0u);
            ps[SL][c] = bload(rFS, oks ? vf[c] : kNone, oks ? pf(zs) : 0u);
            if constexpr (LF) {
                const bool okl = intr && jo[c] == 0 && jn[c] >= 1 && s >= 0 && s < nz;
                pl[SL][c] = bload(rFS, okl ? vf[c] : kNone, okl ? pf(s) : 0u);
            }
            if constexpr (G0) {
                // level 0 at plane s+1 is the top (jo = 0) or the sub (jo = 1)
                // of the old frontier, or the shell off the interior
                const int zz = s + 1;
                const bool ok0 = rt[c] >= 1 && zz >= -R && zz < nz + R;
                const bool sub = rt[c] == 2 && jo[c] == 1 && zz >= 0 && zz < nz;
                p0[SL][c] = bload(sub ? rFS : rFT, ok0 ? vf[c] : kNone, ok0 ? pf(zz) : 0u);
                if constexpr (LF) {
                    const int zp = s - R;
                    const bool okp = intr && jo[c] == 1 && jn[c] >= 2 && zp >= 0 && zp < nz;
                    pp[SL][c] = bload(rFS, okp ? vf[c] : kNone, okp ? pf(zp) : 0u);
                }
            }
            {
                // the shell ring's input: needed on shell rows, on shell
                // planes, and in tiles that reach the x boundary
                const int zh = s + R;
                const bool inz = zh >= 0 && zh < nz;
                const bool okh = rt[c] != 0 && zh >= -R && zh < nz + R &&
                                 (rt[c] == 1 || !inz || (xb && !xin[c]));
                ph[SL][c] = bload(rFT, okh ? vf[c] : kNone, okh ? pf(zh) : 0u);
            }
            if constexpr (CRING) {
                const bool okc = intr && own[c] && jn[c] > jo[c] && s >= 0 && s < nz &&
                                 s >= z0 - R * (L - 1) && s < z1 + R * (L - 1);
#pragma unroll
                for (int k = 0; k < KR; ++k)
                    pc[SL][c][k] = cload_raw(coef, crs(k), okc ? vc[c] : kNone, okc ? pc_(s) : 0u);
            }
        }
    };
    // the same loads for a step s of the fast range
    const uint32_t pc0 = pc_(0);
    auto prefetch_fast = [&](int s, auto slot) __attribute__((always_inline)) {
        constexpr int SL = decltype(slot)::value;
        const uint32_t sf = (uint32_t)s * sz4;
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            pt[SL][c] = bload(rFT, ft_v[c], sf + ft_p[c]);
            ps[SL][c] = bload(rFS, fs_v[c], sf + fs_p[c]);
            if constexpr (LF) pl[SL][c] = bload(rFS, fl_v[c], sf + fl_p[c]);
            if constexpr (G0) {
                p0[SL][c] = bload(f0_sub[c] ? rFS : rFT, f0_v[c], sf + f0_p[c]);
                if constexpr (LF) pp[SL][c] = bload(rFS, fp_v[c], sf + fp_p[c]);
            }
            ph[SL][c] = bload(rFT, fh_v[c], sf + fh_p[c]);
            if constexpr (CRING) {
                const uint32_t so = pc0 + (uint32_t)s * szc;
#pragma unroll
                for (int k = 0; k < KR; ++k) pc[SL][c][k] = cload_raw(coef, crs(k), fc_v[c], so);
            }
        }
    };

    const int s_begin = z0 - R * (L + 1);
    const int s_end = z1 + R * (L - 1);

    // mode 0: interior tile; 1: tile reaching the x boundary; 2, 3: the same
    // at a step whose levels are all active and inside [0, nz) (no z logic)
    // and whose prefetched step is one too
    auto step = [&](int s, auto par, auto mode) __attribute__((always_inline)) {
        constexpr int set = decltype(par)::value;  // LDS set read by step s
        constexpr int SL = PD == 2 ? set : 0;      // prefetch slot holding step s
        constexpr bool XB = decltype(mode)::value % 2 == 1;
        constexpr bool FAST = decltype(mode)::value >= 2;
        float ft[CPT], fs[CPT], fl[CPT], f0n[CPT], fp[CPT];
        const int zh = s + R;
        const bool inzh = zh >= 0 && zh < nz;
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            ft[c] = pt[SL][c];
            fs[c] = ps[SL][c];
            fl[c] = LF ? pl[SL][c] : 0.0f;
            // G0: level 0 at plane s+1, staged at the end of this step
            f0n[c] = G0 ? p0[SL][c] : 0.0f;
            fp[c] = (G0 && LF) ? pp[SL][c] : 0.0f;
#pragma unroll
            for (int i = NSH - 1; i > 0; --i) sh[c][i] = sh[c][i - 1];
            // rows whose top is level 0 find it at plane s + R in ft
            sh[c][0] = (rt[c] == 2 && jo[c] == 0 && inzh) ? ft[c] : ph[SL][c];
            if constexpr (CRING) {
#pragma unroll
                for (int i = NR - 1; i > 0; --i)
#pragma unroll
                    for (int k = 0; k < KR; ++k) cr[c][i][k] = cr[c][i - 1][k];
#pragma unroll
                for (int k = 0; k < KR; ++k) cr[c][0][k] = cexpand(coef, pc[SL][c][k]);
            }
        }
        // level j of column slot c at plane z_j, computed from level j-1
        auto level_update = [&](int c, int j, const float* P) __attribute__((always_inline)) {
            const int jq = j >= 1 ? j - 1 : 0;
            float Wv[kslots<KIND>];
            Wv[0] = 0.0f;
            if constexpr (K > 0) {
                if constexpr (CRING) {
#pragma unroll
                    for (int k = 0; k < K; ++k) Wv[k] = cr[c][jq * R][k];
                } else {
                    const uint32_t so = pc_(s - (j - 1) * R);
                    if constexpr (ALN) {
                        uint32_t wv[K];
#pragma unroll
                        for (int k = 0; k < K; ++k)
                            wv[k] = __builtin_amdgcn_raw_buffer_load_b32(crs(k).r, vw[c], so, 0);
                        // keep the K loads in flight together (otherwise the
                        // words share a register and load one at a time)
                        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                        for (int k = 0; k < K; ++k)
                            Wv[k] = __uint_as_float(__builtin_amdgcn_perm(wv[k], wv[k], vsel[c]));
                    } else {
#pragma unroll
                        for (int k = 0; k < K; ++k) Wv[k] = cload(coef, crs(k), vc[c], so);
                    }
                }
            }
            float pv = 0.0f;
            if constexpr (LF) {
                if (j == 1)
                    pv = fl[c];
                else if (G0 && j == 2)
                    pv = jo[c] == 0 ? sh[c][2 * R] : fp[c];
                else
                    pv = qv[j >= 2 ? j - 2 : 0][c][0];
            }
            float zq[Q];
            if (G0 && j == 1) {
                // level 0 (the old frontier top here: jo = 0)
                // at planes z - R .. z + R, from the shell ring
#pragma unroll
                for (int i = 0; i < Q; ++i) zq[i] = sh[c][2 * R - i];
            } else {
#pragma unroll
                for (int i = 0; i < Q; ++i) zq[i] = qv[jq][c][i];
            }
            const int li = lidx[c];
            nbhd<R> n;
            n.c = zq[R];
#pragma unroll
            for (int r = 1; r <= R; ++r) {
                n.pair[0][r - 1] = P[li - r] + P[li + r];
                n.pair[1][r - 1] = P[li - r * XT] + P[li + r * XT];
                n.pair[2][r - 1] = zq[R - r] + zq[R + r];
            }
            n.m1[0] = P[li - 1];
            n.p1[0] = P[li + 1];
            n.m1[1] = P[li - XT];
            n.p1[1] = P[li + XT];
            n.m1[2] = zq[R - 1];
            n.p1[2] = zq[R + 1];
            return update<KIND>(wt, Wv, n, pv);
        };
        auto push = [&](int c, int j, float v) __attribute__((always_inline)) {
            if (j < L && !(G0 && j == 0)) {
                const int jw = j < L ? j : 0;
#pragma unroll
                for (int i = 0; i < Q - 1; ++i) qv[jw][c][i] = qv[jw][c][i + 1];
                qv[jw][c][Q - 1] = v;
            }
        };
        float vt[CPT], vs[CPT];
        if constexpr (FAST) {
            // Every level is active and inside [0, nz): an interior row holds
            // the old sub and top at levels jo-1 and jo, computes jo+1 .. jn
            // in order, and no row reads its levels below jo-1 or above jn
            // (those take any value); a shell row holds the shell at every
            // level.  The row's type and levels are re-read each step
            // (opaque_s) so that each test is one compare where it is used.
#pragma unroll
            for (int c = 0; c < CPT; ++c) {
                const int rq = opaque_s(rt[c]), joq = opaque_s(jo[c]), jnq = opaque_s(jn[c]);
                float top = ft[c], sub = fs[c];
                if (rq == 2) {
#pragma unroll
                    for (int j = 0; j <= L; ++j) {
                        // (jo >= 0: level 0 is never computed)
                        float v;
                        if (j == 0 || j <= joq) {
                            v = j == joq ? ft[c] : fs[c];
                            if constexpr (XB) v = xin[c] ? v : sh[c][j * R];
                        } else if (j <= jnq) {
                            v = level_update(c, j, lds[set][j >= 1 ? j - 1 : 0]);
                            // columns outside [0, nx) hold the shell at every level
                            if constexpr (XB) v = xin[c] ? v : sh[c][j * R];
                            sub = top;
                            top = v;
                        } else {
                            v = 0.0f;
                        }
                        push(c, j, v);
                    }
                } else {
#pragma unroll
                    for (int j = 0; j <= L; ++j) push(c, j, rq == 1 ? sh[c][j * R] : 0.0f);
                }
                vt[c] = top;
                vs[c] = sub;
            }
        } else {
#pragma unroll
            for (int c = 0; c < CPT; ++c) vt[c] = vs[c] = 0.0f;
#pragma unroll
            for (int j = 0; j <= L; ++j) {
                const int z = s - (j - 1) * R;
                const bool act = level_active(j, z);
                const bool zin = z >= 0 && z < nz;
#pragma unroll
                for (int c = 0; c < CPT; ++c) {
                    float v = 0.0f;
                    if (rt[c] != 0 && act) {
                        const float shv = sh[c][j * R];
                        if (rt[c] == 1 || !zin) {
                            // boundary shell (time independent)
                            v = shv;
                        } else {
                            v = (j == jo[c]) ? ft[c] : ((j == jo[c] - 1) ? fs[c] : 0.0f);
                            if (j >= 1 && j > jo[c] && j <= jn[c])
                                v = level_update(c, j, lds[set][j >= 1 ? j - 1 : 0]);
                            if constexpr (XB) {
                                // columns outside [0, nx) hold the shell at every level
                                v = xin[c] ? v : shv;
                            }
                        }
                    }
                    if (j == jn[c]) vt[c] = v;
                    if (j == jn[c] - 1) vs[c] = v;
                    push(c, j, v);
                }
            }
        }
        // new frontier: the top two levels of the row, at their planes
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            const bool row = rt[c] == 2 && own[c];
            const int zt = s - (jn[c] - 1) * R, zs = s - (jn[c] - 2) * R;
            const bool okt = row && zt >= z0 && zt < z1;
            const bool oks = row && zs >= z0 && zs < z1;
            bstore(rNT, vt[c], (okt && outx[c]) ? vf[c] : kNone, okt ? pf(zt) : 0u);
            bstore(rNS, vs[c], (oks && outx[c]) ? vf[c] : kNone, oks ? pf(zs) : 0u);
        }
        // stage the planes read in-plane next step: level j-1 at plane
        // z_j(s+1), which is queue index R+1 of level j-1 now (R steps old)
#pragma unroll
        for (int j = 1; j <= L; ++j)
#pragma unroll
            for (int c = 0; c < CPT; ++c)
                if (wvu + NWV * c < NCOL)
                    lds[set ^ 1][j - 1][lidx[c]] = (G0 && j == 1) ? f0n[c] : qv[j - 1][c][R + 1];
        // operands of a later step, issued after this step's work so that no
        // wait inside it covers them
        if constexpr (FAST) {
            prefetch_fast(s + PD, ic<PD == 2 ? SL : 0>{});
        } else if constexpr (PD == 2) {
            if (s + 2 < s_end) prefetch(s + 2, ic<SL>{});
        } else {
            if (s + 1 < s_end) prefetch(s + 1, ic<0>{});
        }
        __syncthreads();
    };

    auto run = [&](auto mode) __attribute__((always_inline)) {
        constexpr int M = decltype(mode)::value;
        prefetch(s_begin, ic<0>{});
        if (PD == 2 && s_begin + 1 < s_end) prefetch(s_begin + 1, ic<PD - 1>{});
        int s = s_begin;
        // steps in [f_lo, f_hi) put every level z_j = s - (j-1)R, j = 0 .. L,
        // inside [0, nz) and inside its active window; they run in pairs that
        // keep the LDS and prefetch parity of the stream, the last pair ending
        // two steps before s_b so that the steps they prefetch (at most s + 3)
        // lie in the range too
        const int f_lo = max(z0, 0) + (L - 1) * R;
        const int f_hi = min(s_end, nz - R);
        const int s_a = s_begin + 2 * ((max(f_lo - s_begin, 0) + 1) / 2);
        const int s_b = s_a + 2 * (max(f_hi - s_a, 0) / 2);
        for (; s < s_a && s < s_end; s += 2) {
            step(s, ic<0>{}, mode);
            if (s + 1 < s_end) step(s + 1, ic<1>{}, mode);
        }
        for (; s + 2 < s_b; s += 2) {
            step(s, ic<0>{}, ic<M + 2>{});
            step(s + 1, ic<1>{}, ic<M + 2>{});
        }
        for (; s < s_end; s += 2) {
            step(s, ic<0>{}, mode);
            if (s + 1 < s_end) step(s + 1, ic<1>{}, mode);
        }
    };
    if (xb)
        run(ic<1>{});
    else
        run(ic<0>{});
}

template <int KIND, typename CT, int H, int NWV, int XCH, bool CRING, bool G0, int PD, bool WIN,
          bool ALN>
hipError_t launch_inst(const blocked_row_args& a, hipStream_t s) {
    auto kern = blocked_row_kernel<KIND, CT, H, NWV, XCH, CRING, G0, PD, WIN, ALN>;
    if (a.slots_out) {
        *a.slots_out = device_slots(reinterpret_cast<const void*>(kern), NWV * 64);
        return hipSuccess;
    }
    const int ntiles = a.n_diamonds * a.gx * a.gz;
    if (ntiles <= 0) return hipSuccess;
    weights wt;
    for (int i = 0; i < 5; ++i) wt.w[i] = a.wt.w[i];
    wt.alpha = a.wt.alpha;
    wt.lres = a.wt.lres;
    using bytes_t = std::conditional_t<WIN, uint64_t, uint32_t>;
    hipLaunchKernelGGL(kern, dim3(ntiles), dim3(NWV * 64), 0, s, a.ftop_o, a.fsub_o, a.ftop_n,
                       a.fsub_n, static_cast<const CT*>(a.coef), a.sk, a.d.nx, a.d.ny, a.d.nz, a.d.h,
                       a.d.sy, a.d.sz, (bytes_t)a.field_bytes, (bytes_t)a.coef_bytes, wt, (int)a.t0,
                       (int)a.nt, a.first_centre, a.xo, a.gx, a.zchunk, a.gz, ntiles);
    return hipGetLastError();
}

template <int KIND, typename CT, int H, int NWV, int XCH, bool CRING = false, bool G0 = false,
          int PD = 2>
hipError_t launch_cfg(const blocked_row_args& a, hipStream_t s) {
    // per-workgroup address windows only where a buffer reaches 2 GiB
    const bool win = a.field_bytes >= 0x80000000ull || a.coef_bytes >= 0x80000000ull;
    if constexpr (std::is_same<CT, uint16_t>::value && !CRING) {
        if (a.coef_aligned)
            return win ? launch_inst<KIND, CT, H, NWV, XCH, CRING, G0, PD, true, true>(a, s)
                       : launch_inst<KIND, CT, H, NWV, XCH, CRING, G0, PD, false, true>(a, s);
    }
    return win ? launch_inst<KIND, CT, H, NWV, XCH, CRING, G0, PD, true, false>(a, s)
               : launch_inst<KIND, CT, H, NWV, XCH, CRING, G0, PD, false, false>(a, s);
}

// Workgroup shape per (kind, H): waves, 64-lane x chunks, coefficient ring,
// level 0 from the shell ring (G0), prefetch depth.  Register budget per
// column: L z-queues of 2R+1 values, the shell ring of LR+1 values, and with
// the coefficient ring (L-1)R+1 planes of K values.
template <int KIND, typename CT>
hipError_t launch_kind(const blocked_row_args& a, hipStream_t s) {
    constexpr int R = kind_traits<KIND>::R;
    const int H = a.dw / (2 * R);
    if constexpr (KIND == 1) {
        if (H == 2) return launch_cfg<KIND, CT, 2, 6, 2>(a, s);
        if (H == 3) return launch_cfg<KIND, CT, 3, 8, 2>(a, s);
        if (H == 4) return launch_cfg<KIND, CT, 4, 10, 2>(a, s);
        if (H == 5) return launch_cfg<KIND, CT, 5, 12, 2>(a, s);
        if (H == 6) return launch_cfg<KIND, CT, 6, 14, 2>(a, s);
    } else if constexpr (KIND == 2) {
        if (H == 2) return launch_cfg<KIND, CT, 2, 6, 1, true>(a, s);
        if (H == 3) return launch_cfg<KIND, CT, 3, 8, 1, true, true, 2>(a, s);
        if (H == 4) return launch_cfg<KIND, CT, 4, 10, 1, true>(a, s);
        if (H == 5) return launch_cfg<KIND, CT, 5, 12, 1, true, true, 2>(a, s);
        if (H == 6) return launch_cfg<KIND, CT, 6, 14, 1, true, false, 1>(a, s);
    }
    return hipErrorInvalidValue;
}

// x chunks of the configuration above (host side)
int cfg_xch(int kind, int H) {
    (void)H;
    return kind == 1 ? 2 : 1;
}

}  // namespace

// Scratch of the allocation-free entry point.  The name is a host-side
// stand-in in host code: only the address from hipGetSymbolAddress, taken
// with the device current, may reach a kernel or a copy.
static __device__ __align__(256) float scratch[kScratchBytes / sizeof(float)];

hipError_t blocked_scratch(void** ptr) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void* addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    return hipSuccess;
}

bool blocked_supported(int kind, int dw, int xs) {
    if (kind >= 3) return mwd_supported(kind, dw, xs);
    if (dw % 2 != 0) return false;
    const int H = dw / 2;
    return H >= 2 && H <= 6;
}

// Measured on MI355X (cubes of 64 .. 512, 100 steps): 6 for the 7-point
// constant stencil; for the 7-point variable one 10 from 256^3 points on with
// FP32 coefficients and from 300^3 with BF16 ones, where 12 waves share a
// diamond's nine levels (FP32: equal at 256^3, 1.17-1.25x the rate of 6 at
// 320^3 .. 512^3; BF16: 0.87x at 256^3, 1.01-1.16x at 320^3 .. 512^3), else 6.
// On the benchmark grids 16 for the 25-point variable stencil and the
// variable leapfrog (32-column slices, two workgroups per compute unit), 32
// for the constant leapfrog.
int blocked_default_dw(int kind, int64_t points, bool bf16) {
    switch (kind) {
    case 2: return points >= (bf16 ? 300LL * 300 * 300 : 256LL * 256 * 256) ? 10 : 6;
    case 3: return 16;
    case 4: return 32;
    case 5: return 16;
    default: return 6;
    }
}

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
    default: return hipErrorInvalidValue;
    }
}

}  // namespace stn
