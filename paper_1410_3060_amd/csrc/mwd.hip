// Temporally blocked scheme for the radius-4 stencils (Fig. 1d, 1e): diamond
// tiles along y, a wavefront along z, and several workgroups sharing one
// diamond -- the multi-thread-group form of wavefront diamond blocking
// (Sect. 4.1-4.3, 5.1).
//
// Why several workgroups per diamond.  A diamond of half-height H keeps 2H-1
// time levels in flight, and a point's coefficients are used by its first
// level and again (2H-2)R stream steps later by its last one.  For the
// 25-point variable-coefficient stencil (13 arrays) the coefficient planes in
// flight for a diamond of width 24 are about 11 KB per x column: one compute
// unit holds them for 16 columns, not for a whole row of the lattice.  The
// paper meets the same wall with its cache (Sect. 5.3, 6.1) and answers it
// with thread groups sharing a diamond; here a "team" of workgroups shares a
// diamond, each workgroup owning a 16-column x-slice of every level, so that
// no column is computed twice.  Neighbouring slices exchange the R columns of
// each level that the other needs, through device memory.
//
// Inside a workgroup.  Level j (j = 1 .. L = 2H-1, time t0 + j) is produced
// at plane z_j = s - (j-1)R at stream step s (slope -1/R, Sect. 4.1).  A wave
// owns one band of R = 4 rows of the diamond (rows whose distance from the
// centre lies in [B R, (B+1) R)) and 16 columns; band B computes the levels
// B+1 .. 2H-1-B, each band in its own specialised loop.  A wave keeps per
// column the last 2R+1 planes of each level it reads (z-queues in registers)
// and, where the registers allow, the coefficient planes its levels still
// need (a register ring; for band 0 of the 13-array stencil the ring is in
// LDS).  The in-plane neighbours of level j are level j-1 at plane z_j, which
// was produced R steps earlier: at the end of each step every wave writes the
// planes the next step reads into a double-buffered LDS tile per level (its
// own values, the x-halo columns from the neighbouring slices or the
// lattice), and the workgroup meets at one barrier per step.
//
// Exchange.  A value of level l produced at step s by one slice is read by
// its neighbour at that neighbour's step s + R - 1, so neighbours may drift
// R - 1 steps apart without waiting.  Each exchanged value travels with a
// stamp (launch tag, step number) in one 8-byte device-coherent store; the
// reader compares the stamp and polls again until it matches (a bounded
// number of times, after which an error flag is raised and the run is
// reported as failed at the next synchronisation).  Every workgroup of the
// launch is resident at once (cooperative launch), so every awaited value is
// eventually written.  Slices of one team are placed on one XCD when the XCD
// holds a whole team, so the exchange stays in that XCD's L2.
//
// Rows and launches.  One launch per diamond row; a team processes the
// row's diamonds (and z-chunks) one after another.  Rows at the start and the
// end of the run are clipped to levels 1 .. nt: each band computes the
// levels jo+1 .. jn of its rows, jo and jn from t0 and nt (the same for every
// item of a launch), with jo = B and jn = 2H-1-B in the interior rows.
#include <algorithm>
#include <type_traits>

#include "blocked.h"
#include "bufops.h"
#include "common.h"
#include "point_ops.h"

namespace stn {

namespace {

template <int N>
using ic = std::integral_constant<int, N>;
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

constexpr int kR = 4;
constexpr int kSlots = 16;       // exchange ring depth (steps), a power of two
constexpr int kPolls = 1 << 16;  // polls of a late halo (tens of ms) before the error flag

struct mwd_kargs {
    const float* ftop_o;
    const float* fsub_o;
    float* ftop_n;
    float* fsub_n;
    const void* coef;
    int64_t sk;
    int nx, ny, nz, hh;
    int64_t sy, sz;
    uint64_t field_bytes;  // bytes of one field from its padded origin
    uint64_t coef_bytes;   // bytes of one coefficient array from its padded origin
    weights wt;
    int t0, nt;
    int first_centre;
    int zchunk, gz, n_items;
    int k;         // workgroups (x-slices) per team
    int teams;
    int xcd_teams; // teams per XCD when every team sits on one XCD, else 0
    uint32_t* xbuf;
    uint32_t xbuf_bytes;
    int* err;
    uint32_t tag;  // launch tag 1 .. 4095 (stamps of this launch)
};

// Exchanged levels per band: band B exchanges levels B+1 .. 2H-2-B.
template <int H>
constexpr int nex(int B) {
    return 2 * H - 2 - 2 * B > 0 ? 2 * H - 2 - 2 * B : 0;
}
template <int H>
constexpr int exoff(int B) {
    int o = 0;
    for (int b = 0; b < B; ++b) o += nex<H>(b);
    return o;
}

template <int KIND, typename CT, int H, int NXW, bool LRING, bool ALN, int CG>
__global__ __launch_bounds__(2 * H * NXW * 64) void mwd_row_kernel(mwd_kargs a) {
    constexpr int R = kR;
    constexpr int K = kind_traits<KIND>::K;
    constexpr int KS = kslots<KIND>;
    constexpr bool LF = kind_traits<KIND>::leapfrog;
    constexpr int L = 2 * H - 1;
    constexpr int Q = 2 * R + 1;
    constexpr int DW = 2 * R * H;
    constexpr int XS = 16 * NXW;
    constexpr int XT = XS + 2 * R;
    constexpr int YT = DW + 2 * R;
    constexpr int NR0 = (L - 1) * R + 1;  // coefficient planes of band 0
    constexpr int NEXT = exoff<H>(H);     // exchanged (band, level) pairs per side
    constexpr uint32_t RECB = 2u * 2u * NEXT * 16u * 8u;  // bytes per workgroup and slot
    constexpr uint32_t CB = sizeof(CT);
    constexpr int KG = K > 0 ? K : 1;
    static_assert(!LRING || K > 1, "the LDS ring is for the 13-array stencil");
    static_assert(!ALN || CB == 2, "word loads are for BF16 arrays");

    __shared__ float tile[2][L][YT][XT];
    __shared__ float spare[2 * H * NXW][64];  // target of lanes with nothing to stage
    using RT = std::conditional_t<std::is_same<CT, float>::value, float, uint16_t>;
    __shared__ RT ring0[LRING ? NR0 : 1][LRING ? K : 1][LRING ? 2 * NXW : 1][64];

    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int band = w / (2 * NXW);
    const int side = (w / NXW) & 1;
    const int xw = w % NXW;
    const int cx = lane & 15, rr = lane >> 4;

    // team and slice of this workgroup
    int team, member;
    {
        const int id = blockIdx.x;
        if (a.xcd_teams > 0) {
            const int xcd = id & 7, slot = id >> 3;
            member = slot % a.k;
            team = (slot / a.k) * 8 + xcd;
        } else {
            member = id % a.k;
            team = id / a.k;
        }
    }
    const int x0 = member * XS;
    const int xl = xw * 16 + cx;  // slice-local column of the lane
    const int x = x0 + xl;
    const bool has_left = member > 0, has_right = member < a.k - 1;
    // halo lanes: lanes 0..31 of the slice's edge waves carry the R columns
    // beyond the slice (left for xw = 0, right for xw = NXW-1), rows rr
    const int hside = (lane >> 4) & 1, hr = (lane >> 2) & 3, hc = lane & 3;
    const bool hlane = lane < 32 && (hside == 0 ? xw == 0 : xw == NXW - 1);
    const int xh = hside ? x0 + XS + hc : x0 - R + hc;
    const bool hx_nb = hside ? has_right : has_left;  // halo from a neighbour slice
    // edge lanes that publish the slice's outer R columns
    const int eedge = (xw == 0 && cx < 4) ? 0 : ((xw == NXW - 1 && cx >= 12) ? 1 : -1);
    const int ecol = eedge == 0 ? cx : cx - 12;

    const rsrc_t rX = make_rsrc(a.xbuf, a.xbuf_bytes);
    const uint32_t my_rec = (uint32_t)(team * a.k + member) * kSlots * RECB;
    const uint32_t nb_rec = (uint32_t)(team * a.k + member + (hside ? 1 : -1)) * kSlots * RECB;

    uint32_t seq = 0;  // steps done by this workgroup in this launch
    auto stamp = [&](uint32_t q) { return (a.tag << 20) | (q & 0xfffffu); };

    const int t0 = a.t0, nt = a.nt;
    auto clampt = [&](int t) { return t < 0 ? 0 : (t > nt ? nt : t); };
    const uint32_t sz4 = (uint32_t)(a.sz * 4), szc = (uint32_t)(a.sz * CB);
    auto nrec = [](uint64_t total, uint64_t off) -> uint32_t {
        const uint64_t r = total > off ? total - off : 0u;
        return (uint32_t)(r < 0x7fffffffull ? r : 0x7fffffffull);
    };

    for (int it = team; it < a.n_items; it += a.teams) {
        const int di = it / a.gz, zc = it % a.gz;
        const int yc = a.first_centre + di * DW;
        const int z0 = zc * a.zchunk;
        const int z1 = min(a.nz, z0 + a.zchunk);
        // Level j is needed at planes [z0 - R(L-j), z1 + R(L-j)) (clipped to
        // [-R, nz+R)): the chunk's outputs at level L depend on nothing wider.
        // Every level is computed at every step; values outside a level's
        // window are never read by values inside the windows, so they need no
        // test.  Level 1 starts at its window, after 2R steps that fill the
        // z-queue of the old top.
        const int s_begin = max(z0 - R * (L - 1), -R) - 2 * R;
        const int s_end = z1 + (L - 1) * R;
        // Buffers are based at plane zw, below every plane the item reads, so
        // that 32-bit offsets cover the item's window.  A lane's offset is its
        // row and column plus the plane; it advances by one plane per step.
        // Planes below zw give offsets above 2^31 and planes beyond a buffer
        // offsets beyond its size: both read 0 and store nothing.
        const int zw = max(z0 - R * (L + 2), -a.hh);
        const uint64_t fwb = (uint64_t)(zw + a.hh) * (uint64_t)a.sz * 4u;
        const uint64_t cwb = (uint64_t)(zw + a.hh) * (uint64_t)a.sz * CB;
        const uint32_t fnr = nrec(a.field_bytes, fwb);
        const rsrc_t rFT = make_rsrc(reinterpret_cast<const char*>(a.ftop_o) + fwb, fnr);
        const rsrc_t rFS = make_rsrc(reinterpret_cast<const char*>(a.fsub_o) + fwb, fnr);
        const rsrc_t rNT = make_rsrc(reinterpret_cast<const char*>(a.ftop_n) + fwb, fnr);
        const rsrc_t rNS = make_rsrc(reinterpret_cast<const char*>(a.fsub_n) + fwb, fnr);
        // Coefficient arrays: groups of CG arrays share one resource based at
        // the first array's window and spanning the group (the range check
        // covers the scalar offset too); array k is reached with the scalar
        // offset (k mod CG) * sk bytes, the lane's offset in the vector offset.
        const uint32_t cnr = nrec(a.coef_bytes, cwb);
        const uint32_t skb = (uint32_t)((uint64_t)a.sk * CB);
        constexpr int NG = (KG + CG - 1) / CG;
        rsrc_t rC[NG];
#pragma unroll
        for (int g = 0; g < NG; ++g) {
            const int ng = min(CG, KG - g * CG);
            const uint64_t span = (uint64_t)(ng - 1) * skb + cnr;
            rC[g] = __builtin_amdgcn_make_buffer_rsrc(
                const_cast<char*>(static_cast<const char*>(a.coef) + (uint64_t)(g * CG) * (uint64_t)a.sk * CB + cwb),
                (short)0, (int)(uint32_t)(span < 0xffffffffull ? span : 0xffffffffull), 0x00020000);
        }
        auto crs = [&](int kk) { return rC[kk / CG]; };
        auto csoff = [&](int kk) { return (uint32_t)(kk % CG) * skb; };
        auto plane_off = [&](int z, uint32_t stride) { return (uint32_t)(z - zw) * stride; };

        auto run_band = [&](auto Bc, auto JOc, auto JNc) __attribute__((always_inline)) {
            constexpr int B = decltype(Bc)::value;
            constexpr int JO = decltype(JOc)::value;  // old top level: B, or H in the first row
            constexpr int JN = decltype(JNc)::value;  // new top level if known (> 0)
            constexpr int J0 = B + 1, J1 = 2 * H - 1 - B;
            constexpr int NL = J1 - J0 + 1;
            constexpr bool RL = LRING && B == 0;  // coefficient ring in LDS
            constexpr int NR = RL ? 1 : (K > 0 ? (NL - 1) * R + 1 : 1);
            constexpr int KR = (K > 0 && !RL) ? K : 1;
            constexpr int NSH = (J1 - B) * R + 1;
            constexpr int NX = nex<H>(B) > 0 ? nex<H>(B) : 1;
            constexpr int QS = R + 2;

            constexpr int jo = JO;
            const int jn = JN > 0 ? JN : max(jo, clampt(t0 + J1) - t0);
            // rows of the band-side, flank rows beyond band H-1
            const int ybase = side ? yc + B * R : yc - (B + 1) * R;
            const int y = ybase + rr;
            const int ylt = side ? (H + 1) * R + B * R + rr : (H - B) * R + rr;  // tile row
            const int xt = R + xl;                                                 // tile column
            const bool need = x >= -R && x < a.nx + R && y >= -R && y < a.ny + R;
            const bool intr = x >= 0 && x < a.nx && y >= 0 && y < a.ny;
            const uint32_t rc = (uint32_t)((int64_t)(y + a.hh) * a.sy + (x + a.hh));  // element
            const int yh = ybase + hr;
            const bool hneed = hlane && xh >= -R && xh < a.nx + R && yh >= -R && yh < a.ny + R;
            const uint32_t rch = (uint32_t)((int64_t)(yh + a.hh) * a.sy + (xh + a.hh));
            const int htc = hside ? R + XS + hc : hc;  // tile column of the halo lane
            const int hty = side ? (H + 1) * R + B * R + hr : (H - B) * R + hr;
            // flank rows (band H-1 waves): the neighbour diamonds' rows next to this one
            const int yf = side ? yc + H * R + rr : yc - (H + 1) * R + rr;
            const int ylf = side ? (2 * H + 1) * R + rr : rr;
            const bool fneed = B == H - 1 && x >= -R && x < a.nx + R && yf >= -R && yf < a.ny + R;
            const uint32_t rcf = (uint32_t)((int64_t)(yf + a.hh) * a.sy + (x + a.hh));
            const int jf = clampt(t0 + H - 1) - t0;
            const bool flank_on = B == H - 1 && jo == H - 1 && jn >= H && jf == H - 1;
            // exchange record offsets of this band-side (edge e, level l)
            auto xoff = [&](int e, int l) {
                return (uint32_t)(((e * 2 + side) * NEXT + exoff<H>(B) + (l - J0)) * 128);
            };

            // Per-lane running offsets of the prefetched streams, for the step
            // the next prefetch is for.  Every offset advances by one plane per
            // step; a lane that needs nothing starts at kNone and stays at or
            // above 2^31 (an item's window spans less than 2^31 bytes).
            const int sp = s_begin;  // first prefetched step
            uint32_t o_ot = need ? rc * 4u + plane_off(sp - (jo - 1) * R, sz4) : kNone;
            uint32_t o_ht = (hneed && jn > jo) ? rch * 4u + plane_off(sp + 1 - jo * R, sz4) : kNone;
            uint32_t o_fl = (fneed && flank_on) ? rcf * 4u + plane_off(sp + 1 - (H - 1) * R, sz4) : kNone;
            // coefficients of interior points only
            const int cz0 = RL ? sp : sp - B * R;
            uint32_t o_c = (need && intr) ? rc * CB + plane_off(cz0, szc) : kNone;
            // BF16 word loads: the element's half of its 32-bit word is fixed
            // per lane (even strides, word-aligned arrays)
            const uint32_t csel = (o_c & 2u) ? 0x03020c0cu : 0x01000c0cu;
            // band 0's LDS ring slot of the plane it loads at step s
            int rslot = ((s_begin % NR0) + NR0) % NR0;

            // ---- register state ------------------------------------------
            float q[NL][Q];      // q[i][.]: level B+i at planes z_{B+i+1} - R .. + R
            float qt[R];         // level J1, last R steps (qt[0] newest)
            float qs[QS];        // old sub, last R+2 steps (qs[0] newest)
            float sh[NSH];       // old-top loads, last NSH steps (sh[0] newest)
            float cr[NR][KR];    // coefficient ring: cr[i] = plane s - B R - i
#pragma unroll
            for (int i = 0; i < NL; ++i)
#pragma unroll
                for (int m = 0; m < Q; ++m) q[i][m] = 0.0f;
#pragma unroll
            for (int m = 0; m < R; ++m) qt[m] = 0.0f;
#pragma unroll
            for (int m = 0; m < QS; ++m) qs[m] = 0.0f;
#pragma unroll
            for (int m = 0; m < NSH; ++m) sh[m] = 0.0f;
#pragma unroll
            for (int i = 0; i < NR; ++i)
#pragma unroll
                for (int kk = 0; kk < KR; ++kk) cr[i][kk] = 0.0f;

            // prefetched operands, two slots
            float p_ot[2], p_qs[2], p_ht[2], p_fl[2];
            float p_c[2][KG];
            uint32_t x_v[NX], x_s[NX];

            const int ringw = w;  // band 0 waves are w = 0 .. 2 NXW - 1
            auto prefetch = [&](auto slot) __attribute__((always_inline)) {
                constexpr int SL = decltype(slot)::value;
                p_ot[SL] = bload(rFT, o_ot, 0u);
                // the old sub one plane above the old top's
                p_qs[SL] = (LF || JO >= 1) ? bload(rFS, o_ot + sz4, 0u) : 0.0f;
                p_ht[SL] = bload(rFT, o_ht, 0u);
                p_fl[SL] = (B == H - 1) ? bload(rFT, o_fl, 0u) : 0.0f;
                o_ot += sz4;
                o_ht += sz4;
                o_fl += sz4;
                if constexpr (K > 0) {
                    if constexpr (ALN) {
                        uint32_t wv[K];
#pragma unroll
                        for (int kk = 0; kk < K; ++kk)
                            wv[kk] = __builtin_amdgcn_raw_buffer_load_b32(crs(kk), o_c & ~3u, csoff(kk), 0);
#pragma unroll
                        for (int kk = 0; kk < K; ++kk)
                            p_c[SL][kk] = __uint_as_float(__builtin_amdgcn_perm(wv[kk], wv[kk], csel));
                    } else {
#pragma unroll
                        for (int kk = 0; kk < K; ++kk)
                            p_c[SL][kk] = cload(static_cast<const CT*>(nullptr), crs(kk), o_c, csoff(kk));
                    }
                    o_c += szc;
                }
            };
            // halos of the computed levels jo+1 .. jn-1 that the staging at the
            // end of step s writes: produced by the neighbours at step s+1-R,
            // loaded at the start of step s (two steps of slack)
            auto xload = [&]() __attribute__((always_inline)) {
                const uint32_t slotb = ((seq + 1 - R) & (kSlots - 1)) * RECB;
                const uint32_t want = stamp(seq + 1 - R);
#pragma unroll
                for (int e = 0; e < NX; ++e) {
                    const int l = J0 + e;
                    x_v[e] = 0u;
                    x_s[e] = want;
                    if (nex<H>(B) > 0 && l > jo && l < jn) {
                        // from the neighbour slice, or the shell beyond the
                        // lattice (plane s + 1 - l R) for an edge slice
                        const uint32_t rec = nb_rec + slotb + xoff(hside ? 0 : 1, l) + (uint32_t)(hr * 4 + hc) * 8u;
                        const auto v = __builtin_amdgcn_raw_buffer_load_b64(rX, (hlane && hx_nb) ? rec : kNone, 0, kSC1);
                        // o_ht is at plane s + 3 - jo R (two steps ahead)
                        const uint32_t sv = __builtin_amdgcn_raw_buffer_load_b32(
                            rFT, (hlane && !hx_nb) ? o_ht - (uint32_t)(2 + (l - jo) * R) * sz4 : kNone, 0u, 0);
                        x_v[e] = hx_nb ? v[0] : sv;
                        x_s[e] = hx_nb ? v[1] : want;
                    }
                }
            };

            auto step = [&](int s, auto par) __attribute__((always_inline)) {
                constexpr int P = decltype(par)::value;
                xload();
                const float ot = p_ot[P];
                // rings
#pragma unroll
                for (int m = NSH - 1; m > 0; --m) sh[m] = sh[m - 1];
                sh[0] = ot;
#pragma unroll
                for (int m = QS - 1; m > 0; --m) qs[m] = qs[m - 1];
                qs[0] = p_qs[P];
                if constexpr (K > 0) {
                    if constexpr (RL) {
#pragma unroll
                        for (int kk = 0; kk < K; ++kk) {
                            if constexpr (std::is_same<RT, float>::value)
                                ring0[rslot][kk][ringw][lane] = p_c[P][kk];
                            else
                                ring0[rslot][kk][ringw][lane] = (uint16_t)(__float_as_uint(p_c[P][kk]) >> 16);
                        }
                    } else {
#pragma unroll
                        for (int i = NR - 1; i > 0; --i)
#pragma unroll
                            for (int kk = 0; kk < K; ++kk) cr[i][kk] = cr[i - 1][kk];
#pragma unroll
                        for (int kk = 0; kk < K; ++kk) cr[0][kk] = p_c[P][kk];
                    }
                }
                // the old top enters the queue of level jo (or the top queue)
                if constexpr (JO < J1) {
#pragma unroll
                    for (int m = 0; m < Q - 1; ++m) q[JO - B][m] = q[JO - B][m + 1];
                    q[JO - B][Q - 1] = ot;
                }
                if constexpr (JO == J1) {
#pragma unroll
                    for (int m = R - 1; m > 0; --m) qt[m] = qt[m - 1];
                    qt[0] = ot;
                }
                const float(*Pt)[YT][XT] = tile[P];
                float vtop = ot, vsub = (jn == jo) ? qs[0] : ot;
#pragma unroll
                for (int jj = 0; jj < NL; ++jj) {
                    const int j = J0 + jj;
                    if (j > JO && j <= jn) {
                        const int z = s - (j - 1) * R;
                        float v;
                        {
                            float Wv[KS];
                            Wv[0] = 0.0f;
                            if constexpr (K > 0) {
                                if constexpr (RL) {
                                    int slot = rslot - (j - 1) * R;
                                    slot = slot < 0 ? slot + NR0 : slot;
#pragma unroll
                                    for (int kk = 0; kk < K; ++kk) {
                                        if constexpr (std::is_same<RT, float>::value)
                                            Wv[kk] = ring0[slot][kk][ringw][lane];
                                        else
                                            Wv[kk] = __uint_as_float((uint32_t)ring0[slot][kk][ringw][lane] << 16);
                                    }
                                } else {
#pragma unroll
                                    for (int kk = 0; kk < K; ++kk) Wv[kk] = cr[(j - J0) * R][kk];
                                }
                            }
                            // level j-1: z-queue (registers) and in-plane tile (LDS)
                            const float* zq = q[j - 1 - B >= 0 ? j - 1 - B : 0];
                            const float(*T)[XT] = Pt[j - 1];
                            nbhd<R> n;
                            n.c = zq[R];
#pragma unroll
                            for (int r = 1; r <= R; ++r) {
                                n.pair[0][r - 1] = T[ylt][xt - r] + T[ylt][xt + r];
                                n.pair[1][r - 1] = T[ylt - r][xt] + T[ylt + r][xt];
                                n.pair[2][r - 1] = zq[R - r] + zq[R + r];
                            }
                            n.m1[0] = T[ylt][xt - 1];
                            n.p1[0] = T[ylt][xt + 1];
                            n.m1[1] = T[ylt - 1][xt];
                            n.p1[1] = T[ylt + 1][xt];
                            n.m1[2] = zq[R - 1];
                            n.p1[2] = zq[R + 1];
                            float pv = 0.0f;
                            if constexpr (LF) {
                                // level j-2 at plane z: the old sub for j = jo+1,
                                // else the oldest entry of level j-2's queue
                                if (j == JO + 1)
                                    pv = qs[R + 1];
                                else
                                    pv = q[j - 2 - B >= 0 ? j - 2 - B : 0][0];
                            }
                            v = update<KIND>(a.wt, Wv, n, pv);
                            // boundary shell: time independent, from the old-top ring
                            const bool zin = z >= 0 && z < a.nz;
                            v = (intr && zin) ? v : sh[(j > JO ? j - JO : 0) * R];
                        }
                        // queue of level j (input of level j+1) or the top queue
                        if (j < J1) {
                            const int qi = jj + 1 < NL ? jj + 1 : 0;
#pragma unroll
                            for (int m = 0; m < Q - 1; ++m) q[qi][m] = q[qi][m + 1];
                            q[qi][Q - 1] = v;
                        } else {
#pragma unroll
                            for (int m = R - 1; m > 0; --m) qt[m] = qt[m - 1];
                            qt[0] = v;
                        }
                        if (j == jn) vtop = v;
                        if (j == jn - 1) vsub = v;
                        // the slice's edge columns for the neighbours
                        if (j < jn && nex<H>(B) > 0) {
                            const uint32_t rec = my_rec + (seq & (kSlots - 1)) * RECB +
                                                 xoff(eedge > 0 ? 1 : 0, j) + (uint32_t)(rr * 4 + ecol) * 8u;
                            u32x2 pk;
                            pk.x = __float_as_uint(v);
                            pk.y = stamp(seq);
                            __builtin_amdgcn_raw_buffer_store_b64(pk, rX, eedge >= 0 ? rec : kNone, 0, kSC1);
                        }
                    }
                }
                // new frontier: levels jn and jn-1 of the band's rows, at their planes
                {
                    // o_ot is at plane s + 2 - (jo - 1) R (two steps ahead)
                    const int zt = s - (jn - 1) * R;
                    const int zs = jn > jo ? s - (jn - 2) * R : s + 1 - (jo - 1) * R;
                    const uint32_t ot_s = o_ot - 2u * sz4;  // plane s - (jo - 1) R
                    const uint32_t st = ot_s - (uint32_t)((jn - jo) * R) * sz4;
                    const uint32_t ss = jn > jo ? ot_s - (uint32_t)((jn - 1 - jo) * R) * sz4 : ot_s + sz4;
                    bstore(rNT, vtop, (intr && zt >= z0 && zt < z1) ? st : kNone, 0u);
                    bstore(rNS, vsub, (intr && zs >= z0 && zs < z1) ? ss : kNone, 0u);
                }
                // stage the planes the next step reads in-plane: level l at
                // plane z_{l+1}(s+1) = s + 1 - l R
                float(*Pn)[YT][XT] = tile[P ^ 1];
                if constexpr (JO >= 1) Pn[JO - 1][ylt][xt] = qs[0];
                if constexpr (JO <= L - 1) {
                    if constexpr (JO < J1)
                        Pn[JO][ylt][xt] = q[JO - B][R + 1];
                    else
                        Pn[JO][ylt][xt] = qt[R - 1];
                }
#pragma unroll
                for (int jj = 0; jj < NL; ++jj) {
                    const int l = J0 + jj;
                    if (l > JO && l <= jn && l <= L - 1) {
                        if (l < J1)
                            Pn[l][ylt][xt] = q[jj + 1 < NL ? jj + 1 : 0][R + 1];
                        else
                            Pn[l][ylt][xt] = qt[R - 1];
                    }
                }
                // halo columns: halo lanes write the tile, the others a spare slot
                {
                    if (jn > JO) *(hlane ? &Pn[JO][hty][htc] : &spare[w][lane]) = p_ht[P];
                    const bool xon = seq + 1 >= (uint32_t)R;
                    const uint32_t want = stamp(seq + 1 - R);
#pragma unroll
                    for (int e = 0; e < NX; ++e) {
                        const int l = J0 + e;
                        if (nex<H>(B) > 0 && l > jo && l < jn) {
                            uint32_t v = x_v[e];
                            if (__ballot(hlane && xon && x_s[e] != want)) {
                                // late: poll, coherent across the device, until
                                // the neighbour's value arrives
                                const uint32_t rec = nb_rec + ((seq + 1 - R) & (kSlots - 1)) * RECB +
                                                     xoff(hside ? 0 : 1, l) + (uint32_t)(hr * 4 + hc) * 8u;
                                uint32_t got = (hlane && xon) ? x_s[e] : want;
                                // after one failure the run is invalid: do not wait again
                                int polls = __hip_atomic_load(a.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                                ? kPolls
                                                : 0;
                                while (__ballot(got != want) && polls < kPolls) {
                                    __builtin_amdgcn_s_sleep(1);
                                    if (got != want) {
                                        const auto r2 = __builtin_amdgcn_raw_buffer_load_b64(rX, rec, 0, kSC1 | kVolatile);
                                        v = r2[0];
                                        got = r2[1];
                                    }
                                    ++polls;
                                }
                                if (got != want) atomicOr(a.err, 1);
                            }
                            *(hlane ? &Pn[l][hty][htc] : &spare[w][lane]) = __uint_as_float(v);
                        }
                    }
                }
                if (B == H - 1 && flank_on) Pn[H - 1][ylf][xt] = p_fl[P];
                rslot = rslot + 1 == NR0 ? 0 : rslot + 1;
                ++seq;
            };

            // prefetches run two steps ahead, also past the last step (their
            // loads are then unused), so that every running offset is two
            // steps ahead of the step in progress
            prefetch(ic<0>{});
            prefetch(ic<1>{});
            for (int s = s_begin; s < s_end; s += 2) {
                step(s, ic<0>{});
                prefetch(ic<0>{});
                __syncthreads();
                if (s + 1 < s_end) {
                    step(s + 1, ic<1>{});
                    prefetch(ic<1>{});
                    __syncthreads();
                }
            }
        };

        // a band-side whose rows are already at level nt before this row (the
        // last rows of a run): nothing is computed and no neighbour reads it;
        // its frontier pair is copied to the new buffers
        auto copy_band = [&](int B) __attribute__((always_inline)) {
            const int jo = clampt(t0 + B) - t0;
            const int y = (side ? yc + B * R : yc - (B + 1) * R) + rr;
            const bool intr = x >= 0 && x < a.nx && y >= 0 && y < a.ny;
            const uint32_t rc4 = (uint32_t)((int64_t)(y + a.hh) * a.sy + (x + a.hh)) * 4u;
            for (int s = s_begin; s < s_end; ++s) {
                const int zt = s - (jo - 1) * R, zs = s + 1 - (jo - 1) * R;
                const bool okt = intr && zt >= z0 && zt < z1;
                const bool oks = intr && zs >= z0 && zs < z1;
                const uint32_t ot_ = okt ? rc4 + plane_off(zt, sz4) : kNone;
                const uint32_t os_ = oks ? rc4 + plane_off(zs, sz4) : kNone;
                bstore(rNT, bload(rFT, ot_, 0u), ot_, 0u);
                bstore(rNS, bload(rFS, os_, 0u), os_, 0u);
                ++seq;
                __syncthreads();
            }
        };
        auto dispatch = [&](auto Bc) __attribute__((always_inline)) {
            constexpr int B = decltype(Bc)::value;
            const int jo = clampt(t0 + B) - t0;
            constexpr int J1 = 2 * H - 1 - B;
            if (jo == B) {
                if (t0 + J1 <= nt)
                    run_band(Bc, ic<B>{}, ic<J1>{});  // every row but the first and last
                else
                    run_band(Bc, ic<B>{}, ic<0>{});
            } else if (jo == H) {
                run_band(Bc, ic<H>{}, ic<0>{});
            } else {
                copy_band(B);
            }
        };
        if constexpr (H >= 1) if (band == 0) dispatch(ic<0>{});
        if constexpr (H >= 2) if (band == 1) dispatch(ic<1>{});
        if constexpr (H >= 3) if (band == 2) dispatch(ic<2>{});
        if constexpr (H >= 4) if (band == 3) dispatch(ic<3>{});
    }
}

__global__ void fill_u32_kernel(uint32_t* p, uint64_t n, uint32_t v) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

template <int KIND, typename CT, int H, int NXW, bool LRING, bool ALN, int CG>
struct mwd_inst {
    static constexpr int threads = 2 * H * NXW * 64;
    static constexpr int XS = 16 * NXW;
    static constexpr uint32_t recb = 2u * 2u * exoff<H>(H) * 16u * 8u;
    static const void* kernel() {
        return reinterpret_cast<const void*>(mwd_row_kernel<KIND, CT, H, NXW, LRING, ALN, CG>);
    }
};

// Team layout of a launch: k slices per team, as many teams as the device
// holds resident (every workgroup of a cooperative launch is resident), on
// one XCD each when an XCD holds a whole team.
struct team_layout {
    int k = 0, teams = 0, xcd_teams = 0, threads = 0, xs = 0;
    uint32_t recb = 0;
    const void* kernel = nullptr;
};

template <typename I>
hipError_t layout_of(int nx, team_layout* t) {
    t->kernel = I::kernel();
    t->threads = I::threads;
    t->xs = I::XS;
    t->recb = I::recb;
    t->k = (nx + I::XS - 1) / I::XS;
    if (t->k < 1) t->k = 1;
    const long long slots = device_slots(t->kernel, I::threads);
    if (slots < t->k) return hipErrorInvalidConfiguration;
    const long long per_xcd = slots / 8;
    if (per_xcd >= t->k) {
        t->xcd_teams = (int)(per_xcd / t->k);
        t->teams = 8 * t->xcd_teams;
    } else {
        t->xcd_teams = 0;
        t->teams = (int)(slots / t->k);
    }
    return hipSuccess;
}

template <int KIND, typename CT, bool ALN, int CG>
hipError_t pick_cg(int dw, int nx, team_layout* t) {
    constexpr int R = kR;
    const int H = dw / (2 * R);
    if constexpr (KIND == 3) {
        if (H == 2) return layout_of<mwd_inst<KIND, CT, 2, 1, false, ALN, CG>>(nx, t);
        if (H == 3) return layout_of<mwd_inst<KIND, CT, 3, 1, true, ALN, CG>>(nx, t);
    } else {
        if (H == 2) return layout_of<mwd_inst<KIND, CT, 2, 1, false, ALN, CG>>(nx, t);
        if (H == 3) return layout_of<mwd_inst<KIND, CT, 3, 1, false, ALN, CG>>(nx, t);
        if (H == 4) return layout_of<mwd_inst<KIND, CT, 4, 1, false, ALN, CG>>(nx, t);
    }
    return hipErrorInvalidValue;
}

// Coefficient arrays per buffer resource: the 13 arrays of the 25-point
// stencil in one or two resources when (group - 1) sk + one array's bytes
// stays below 2^32 (the offsets are 32-bit), else one per array.
int coef_group(int kind, bool bf16, int64_t sk, uint64_t coef_bytes) {
    if (kind != 3) return 1;
    const uint64_t skb = (uint64_t)sk * (bf16 ? 2u : 4u);
    const uint64_t span = std::min<uint64_t>(coef_bytes, 0x7fffffffull);
    auto fits = [&](int g) { return (uint64_t)(g - 1) * skb + span <= 0xffffffffull; };
    if (fits(13)) return 13;
    if (fits(7)) return 7;
    return 1;
}

template <int KIND, typename CT, bool ALN>
hipError_t pick_aln(int dw, int nx, int cg, team_layout* t) {
    if constexpr (KIND == 3) {
        if (cg == 13) return pick_cg<KIND, CT, ALN, 13>(dw, nx, t);
        if (cg == 7) return pick_cg<KIND, CT, ALN, 7>(dw, nx, t);
    }
    return pick_cg<KIND, CT, ALN, 1>(dw, nx, t);
}

template <int KIND, typename CT>
hipError_t pick(int dw, int nx, bool aln, int cg, team_layout* t) {
    if constexpr (std::is_same<CT, uint16_t>::value) {
        if (aln) return pick_aln<KIND, CT, true>(dw, nx, cg, t);
    }
    return pick_aln<KIND, CT, false>(dw, nx, cg, t);
}

hipError_t pick_any(int kind, bool bf16, int dw, int nx, bool aln, int cg, team_layout* t) {
    switch (kind) {
    case 3: return bf16 ? pick<3, uint16_t>(dw, nx, aln, cg, t) : pick<3, float>(dw, nx, aln, cg, t);
    case 4: return pick<4, float>(dw, nx, false, 1, t);
    case 5: return bf16 ? pick<5, uint16_t>(dw, nx, aln, 1, t) : pick<5, float>(dw, nx, aln, 1, t);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

bool mwd_supported(int kind, int dw) {
    if (kind < 3 || kind > 5 || dw % (2 * kR) != 0) return false;
    const int H = dw / (2 * kR);
    return kind == 3 ? (H == 2 || H == 3) : (H >= 2 && H <= 4);
}

hipError_t mwd_workspace(int kind, bool bf16, int dw, int nx, size_t* xbytes) {
    team_layout t;
    hipError_t e = pick_any(kind, bf16, dw, nx, false, 1, &t);
    if (e != hipSuccess) return e;
    *xbytes = (size_t)t.teams * t.k * kSlots * t.recb;
    return hipSuccess;
}

hipError_t launch_fill_u32(void* p, size_t words, uint32_t v, hipStream_t s) {
    if (words == 0) return hipSuccess;
    const int blocks = (int)std::min<size_t>((words + 255) / 256, 4096);
    hipLaunchKernelGGL(fill_u32_kernel, dim3(blocks), dim3(256), 0, s, static_cast<uint32_t*>(p),
                       (uint64_t)words, v);
    return hipGetLastError();
}

hipError_t launch_mwd_row(int kind, bool bf16, const mwd_row_args& r, hipStream_t s) {
    team_layout t;
    hipError_t e = pick_any(kind, bf16, r.dw, r.d.nx, r.coef_aligned,
                            coef_group(kind, bf16, r.sk, r.coef_bytes), &t);
    if (e != hipSuccess) return e;
    const int R = kR;
    const int H = r.dw / (2 * R);
    const int L = 2 * H - 1;
    if (r.n_diamonds <= 0) return hipSuccess;
    const size_t need = (size_t)t.teams * t.k * kSlots * t.recb;
    if (need > r.xbuf_bytes || need >= 0x80000000ull) return hipErrorInvalidValue;
    // z-chunks: the count that minimises rounds of teams x steps per item
    // (its planes plus the 2RL steps that fill and drain the wavefront),
    // with every item's address window below 2 GiB
    const int nz = r.d.nz;
    const uint64_t plane = (uint64_t)r.d.sz * 4u;
    const int64_t maxw = (int64_t)(0x7fffffffull / plane) - 2 * R * (L + 2) - 2;
    int zchunk = r.zchunk;
    if (zchunk <= 0) {
        double best = 0.0;
        for (int gz = 1; gz <= 32; ++gz) {
            const int c = (nz + gz - 1) / gz;
            const long long items = (long long)r.n_diamonds * gz;
            const long long rounds = (items + t.teams - 1) / t.teams;
            const double cost = (double)rounds * (c + 2 * R * L);
            if (zchunk <= 0 || cost < best) {
                best = cost;
                zchunk = c;
            }
        }
    }
    if (maxw < 1) return hipErrorInvalidValue;
    zchunk = (int)std::min<int64_t>(std::max(zchunk, 1), maxw);
    const int gz = (nz + zchunk - 1) / zchunk;
    mwd_kargs a;
    a.ftop_o = r.ftop_o;
    a.fsub_o = r.fsub_o;
    a.ftop_n = r.ftop_n;
    a.fsub_n = r.fsub_n;
    a.coef = r.coef;
    a.sk = r.sk;
    a.nx = r.d.nx;
    a.ny = r.d.ny;
    a.nz = r.d.nz;
    a.hh = r.d.h;
    a.sy = r.d.sy;
    a.sz = r.d.sz;
    a.field_bytes = r.field_bytes;
    a.coef_bytes = r.coef_bytes;
    for (int i = 0; i < 5; ++i) a.wt.w[i] = r.wt.w[i];
    a.wt.alpha = r.wt.alpha;
    a.wt.lres = r.wt.lres;
    a.t0 = (int)r.t0;
    a.nt = (int)r.nt;
    a.first_centre = r.first_centre;
    a.zchunk = zchunk;
    a.gz = gz;
    a.n_items = r.n_diamonds * gz;
    a.k = t.k;
    a.teams = t.teams;
    a.xcd_teams = t.xcd_teams;
    a.xbuf = static_cast<uint32_t*>(r.xbuf);
    a.xbuf_bytes = (uint32_t)need;
    a.err = r.err;
    a.tag = r.tag;
    void* args[] = {&a};
    return hipLaunchCooperativeKernel(t.kernel, dim3(t.teams * t.k), dim3(t.threads), args, 0, s);
}

}  // namespace stn
