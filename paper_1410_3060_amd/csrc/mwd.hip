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
// unit holds them for 16 or 32 columns, not for a whole row of the lattice.
// The paper meets the same wall with its cache (Sect. 5.3, 6.1) and answers it
// with thread groups sharing a diamond; here a "team" of workgroups shares a
// diamond, each workgroup owning an x-slice of 16 or 32 columns of every
// level, so that no column is computed twice.  Neighbouring slices exchange
// the R columns of each level that the other needs, through device memory.
//
// Inside a workgroup.  Level j (j = 1 .. L = 2H-1, time t0 + j) is produced
// at plane z_j = s - (j-1)R at stream step s (slope -1/R, Sect. 4.1).  A wave
// owns one band of R = 4 rows of the diamond (rows whose distance from the
// centre lies in [B R, (B+1) R)) and 16 columns; band B computes the levels
// B+1 .. 2H-1-B, each band in its own specialised loop, and each wave runs
// one or two bands (four waves per 16 columns).  A wave keeps per
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
// holds a whole team, so the exchange stays in that XCD's L2; larger teams
// span XCDs and rely on the device-coherent path.
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

// Compile-time configuration of one kernel instance.
template <int KIND_, typename CT_, int H_, int NXW_, bool LRING_, bool ALN_, int CG_>
struct mwd_cfg {
    static constexpr int KIND = KIND_, H = H_, NXW = NXW_, CG = CG_;
    using CT = CT_;
    static constexpr bool LRING = LRING_, ALN = ALN_;
    static constexpr int R = kR;
    static constexpr int K = kind_traits<KIND>::K;
    static constexpr int KS = kslots<KIND>;
    static constexpr int KG = K > 0 ? K : 1;
    static constexpr int NG = (KG + CG - 1) / CG;  // coefficient buffer resources
    static constexpr bool LF = kind_traits<KIND>::leapfrog;
    static constexpr int L = 2 * H - 1;
    static constexpr int Q = 2 * R + 1;
    static constexpr int DW = 2 * R * H;
    static constexpr int XS = 16 * NXW;
    static constexpr int XT = XS + 2 * R;
    static constexpr int YT = DW + 2 * R;
    // LDS tile of level l: the rows level l+1 reads, [trlo(l), trlo(l) +
    // trows(l)) of the YT rows around the diamond, with a pitch of XP floats.
    // A wave reads 4 rows of 16 columns at a time; XP = 16 (mod 32) puts
    // them in 4 disjoint 16-bank groups.
    static constexpr int XP = XT <= 16 ? 16 : ((XT - 16 + 31) / 32) * 32 + 16;
    static constexpr int tm(int l) { return l < 2 * H - 2 - l ? l : 2 * H - 2 - l; }
    static constexpr int trlo(int l) { return (H - 1 - tm(l)) * R; }
    static constexpr int trows(int l) { return (2 * tm(l) + 4) * R; }
    static constexpr int tbase(int l) {
        int b = 0;
        for (int i = 0; i < l; ++i) b += trows(i);
        return b;
    }
    static constexpr int TR = tbase(L);  // rows of all levels
    // lanes with nothing to stage write a padding column instead (never
    // read): SPL lanes per row, rows counted across both buffers
    static constexpr int SPL = XP - XT >= 16 ? 16 : 8;
    static_assert(XP - XT >= SPL && 4 * NXW_ * 64 / SPL <= 2 * TR, "no room for the staging sink");
    // flat row of tile row y of level l
    static constexpr int trow(int l, int y) { return tbase(l) - trlo(l) + y; }
    static constexpr int NR0 = (L - 1) * R + 1;  // coefficient planes of band 0
    static constexpr int NEXT = exoff<H>(H);     // exchanged (band, level) pairs per side
    static constexpr uint32_t RECB = 2u * 2u * NEXT * 16u * 8u;  // bytes per workgroup and slot
    static constexpr uint32_t CB = sizeof(CT);
    static constexpr int NW = 4 * NXW;  // waves: two band groups x two sides x NXW
    using RT = std::conditional_t<std::is_same<CT, float>::value, float, uint16_t>;
    static_assert(!LRING || K > 1, "the LDS ring is for the 13-array stencil");
    static_assert(!ALN || CB == 2, "word loads are for BF16 arrays");
};

// Bands per wave group, chosen so that both groups compute about the same
// number of levels per step (band B computes 2H-1-2B levels):
// H = 2: {0}, {1};  H = 3: {0}, {1, 2};  H = 4: {0, 3}, {1, 2}.
template <int H>
constexpr int gband(int g, int i) {
    if (H == 2) return i == 0 ? g : -1;
    if (H == 3) return g == 0 ? (i == 0 ? 0 : -1) : (i == 0 ? 1 : 2);
    return g == 0 ? (i == 0 ? 0 : 3) : (i == 0 ? 1 : 2);
}

// What one wave knows about the item and the lanes it runs (shared by the
// bands of the wave).
template <class C>
struct mwd_item {
    const mwd_kargs* a;
    float (*tile)[C::TR][C::XP];
    typename C::RT (*ring0)[C::LRING ? C::K : 1][C::LRING ? 2 * C::NXW : 1][64];
    float* spare;  // this lane's sink for lanes with nothing to stage (tile padding)
    rsrc_t rFT, rFS, rNT, rNS, rX;
    rsrc_t rC[C::NG];
    uint32_t skb, sz4, szc;
    int yc, z0, z1, zw, s_begin, s_end, t0, nt;
    // lanes
    int lane, side, xw, ringw, cx, rr, x, xl;
    int hside, hr, hc, xh, eedge, ecol;
    bool hlane, hx_nb;
    uint32_t my_rec, nb_rec;

    __device__ __forceinline__ uint32_t stamp(uint32_t q) const { return (a->tag << 20) | (q & 0xfffffu); }
    __device__ __forceinline__ int clampt(int t) const { return t < 0 ? 0 : (t > nt ? nt : t); }
    __device__ __forceinline__ uint32_t plane_off(int z, uint32_t stride) const {
        return (uint32_t)(z - zw) * stride;
    }
    __device__ __forceinline__ rsrc_t crs(int kk) const { return rC[kk / C::CG]; }
    __device__ __forceinline__ uint32_t csoff(int kk) const { return (uint32_t)(kk % C::CG) * skb; }
};

// One band-side of a diamond, run by one wave: old top level JO (B, or H in
// the first row of a run), new top level JN (2H-1-B; 0 = computed at run
// time for the first and last rows).
template <class C, int B, int JO, int JN>
struct mwd_band {
    static constexpr int R = C::R, K = C::K, Q = C::Q, L = C::L, H = C::H;
    static constexpr int XS = C::XS, XT = C::XT, YT = C::YT, NR0 = C::NR0;
    static constexpr int J0 = B + 1, J1 = 2 * H - 1 - B;
    static constexpr int NL = J1 - J0 + 1;
    static constexpr bool RL = C::LRING && B == 0;  // coefficient ring in LDS
    static constexpr int NR = RL ? 1 : (K > 0 ? (NL - 1) * R + 1 : 1);
    static constexpr int KR = (K > 0 && !RL) ? K : 1;
    static constexpr int NX = nex<H>(B) > 0 ? nex<H>(B) : 1;
    static constexpr int QS = R + 2;
    static constexpr int jo = JO;

    int jn;
    int ylt, xt, hty, htc, ylf;
    bool intr, flank_on;
    uint32_t o_ot, o_ht, o_fl, o_c, csel;
    int rslot;
    float q[NL][Q];    // q[i][.]: level B+i at planes z_{B+i+1} - R .. + R
    float qt[R];       // level J1, last R steps (qt[0] newest)
    float qs[QS];      // old sub, last R+2 steps (qs[0] newest)
    float cr[NR][KR];  // coefficient ring: cr[i] = plane s - B R - i
    float p_ot[2], p_qs[2], p_ht[2], p_fl[2];
    float p_c[2][C::KG];
    uint32_t x_v[NX], x_s[NX], x_sh[NX];  // exchange loads in flight

    __device__ __forceinline__ uint32_t xoff(const mwd_item<C>& I, int e, int l) const {
        return (uint32_t)(((e * 2 + I.side) * C::NEXT + exoff<H>(B) + (l - J0)) * 128);
    }

    __device__ __forceinline__ void init(const mwd_item<C>& I) {
        const mwd_kargs& a = *I.a;
        // new top: 2H-1-B clipped to nt; a band already at nt copies its pair
        if (JN > 0) {
            jn = JN;
        } else {
            jn = I.t0 + B > I.nt ? JO : max(JO, I.clampt(I.t0 + J1) - I.t0);
        }
        const int ybase = I.side ? I.yc + B * R : I.yc - (B + 1) * R;
        const int y = ybase + I.rr;
        ylt = I.side ? (H + 1) * R + B * R + I.rr : (H - B) * R + I.rr;  // tile row
        xt = R + I.xl;                                                     // tile column
        const bool need = I.x >= -R && I.x < a.nx + R && y >= -R && y < a.ny + R;
        intr = I.x >= 0 && I.x < a.nx && y >= 0 && y < a.ny;
        const uint32_t rc = (uint32_t)((int64_t)(y + a.hh) * a.sy + (I.x + a.hh));  // element
        const int yh = ybase + I.hr;
        const bool hneed = I.hlane && I.xh >= -R && I.xh < a.nx + R && yh >= -R && yh < a.ny + R;
        const uint32_t rch = (uint32_t)((int64_t)(yh + a.hh) * a.sy + (I.xh + a.hh));
        htc = I.hside ? R + XS + I.hc : I.hc;  // tile column of the halo lane
        hty = I.side ? (H + 1) * R + B * R + I.hr : (H - B) * R + I.hr;
        // flank rows (band H-1): the neighbour diamonds' rows next to this one
        const int yf = I.side ? I.yc + H * R + I.rr : I.yc - (H + 1) * R + I.rr;
        ylf = I.side ? (2 * H + 1) * R + I.rr : I.rr;
        const bool fneed = B == H - 1 && I.x >= -R && I.x < a.nx + R && yf >= -R && yf < a.ny + R;
        const uint32_t rcf = (uint32_t)((int64_t)(yf + a.hh) * a.sy + (I.x + a.hh));
        const int jf = I.clampt(I.t0 + H - 1) - I.t0;
        flank_on = B == H - 1 && JO == H - 1 && jn >= H && jf == H - 1;
        // Per-lane running offsets of the prefetched streams, for the step
        // the next prefetch is for.  Every offset advances by one plane per
        // step; a lane that needs nothing starts at kNone and stays at or
        // above 2^31 (an item's window spans less than 2^31 bytes).
        const int sp = I.s_begin;  // first prefetched step
        o_ot = need ? rc * 4u + I.plane_off(sp - (JO - 1) * R, I.sz4) : kNone;
        o_ht = (hneed && jn > JO) ? rch * 4u + I.plane_off(sp + 1 - JO * R, I.sz4) : kNone;
        o_fl = (fneed && flank_on) ? rcf * 4u + I.plane_off(sp + 1 - (H - 1) * R, I.sz4) : kNone;
        // coefficients of interior points only
        const int cz0 = RL ? sp : sp - B * R;
        o_c = (need && intr) ? rc * C::CB + I.plane_off(cz0, I.szc) : kNone;
        // BF16 word loads: the element's half of its 32-bit word is fixed
        // per lane (even strides, word-aligned arrays)
        csel = (o_c & 2u) ? 0x03020c0cu : 0x01000c0cu;
        rslot = ((I.s_begin % NR0) + NR0) % NR0;
#pragma unroll
        for (int i = 0; i < NL; ++i)
#pragma unroll
            for (int m = 0; m < Q; ++m) q[i][m] = 0.0f;
#pragma unroll
        for (int m = 0; m < R; ++m) qt[m] = 0.0f;
#pragma unroll
        for (int m = 0; m < QS; ++m) qs[m] = 0.0f;
#pragma unroll
        for (int i = 0; i < NR; ++i)
#pragma unroll
            for (int kk = 0; kk < KR; ++kk) cr[i][kk] = 0.0f;
    }

    template <int SL>
    __device__ __forceinline__ void prefetch(const mwd_item<C>& I) {
        p_ot[SL] = bload(I.rFT, o_ot, 0u);
        // the old sub one plane above the old top's
        p_qs[SL] = (C::LF || JO >= 1) ? bload(I.rFS, o_ot + I.sz4, 0u) : 0.0f;
        p_ht[SL] = bload(I.rFT, o_ht, 0u);
        p_fl[SL] = (B == H - 1) ? bload(I.rFT, o_fl, 0u) : 0.0f;
        o_ot += I.sz4;
        o_ht += I.sz4;
        o_fl += I.sz4;
        if constexpr (K > 0) {
            // The band with the LDS ring keeps them as loaded (FP32 values,
            // BF16 words or halfwords) until they enter the ring two steps
            // later (cbits): expanding them beside the loads makes the wave
            // wait for the loads here.  The register-ring bands expand them
            // at once (cexp): raw values held beside the ring cost them more
            // registers than the wait.
#pragma unroll
            for (int kk = 0; kk < K; ++kk) {
                float raw;
                if constexpr (C::ALN)
                    raw = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(I.crs(kk), o_c & ~3u, I.csoff(kk), 0));
                else if constexpr (std::is_same<typename C::CT, float>::value)
                    raw = bload(I.crs(kk), o_c, I.csoff(kk));
                else
                    raw = __uint_as_float(
                        static_cast<uint32_t>(__builtin_amdgcn_raw_buffer_load_b16(I.crs(kk), o_c, I.csoff(kk), 0)));
                p_c[SL][kk] = RL ? raw : cexp(raw);
            }
            o_c += I.szc;
        }
    }

    // a loaded coefficient as its FP32 value (BF16 expanded exactly)
    __device__ __forceinline__ float cexp(float raw) const {
        if constexpr (std::is_same<typename C::CT, float>::value)
            return raw;
        else if constexpr (C::ALN)
            return __uint_as_float(__builtin_amdgcn_perm(__float_as_uint(raw), __float_as_uint(raw), csel));
        else
            return __uint_as_float(__float_as_uint(raw) << 16);
    }
    // a loaded BF16 coefficient's 16 stored bits (from the raw load)
    __device__ __forceinline__ uint16_t cbits(float raw) const {
        if constexpr (C::ALN)
            return (uint16_t)(__float_as_uint(cexp(raw)) >> 16);
        else
            return (uint16_t)__float_as_uint(raw);
    }

    // halos of the computed levels jo+1 .. jn-1 that the staging at the end
    // of step s writes: produced by the neighbours at step s+1-R, loaded at
    // the start of step s (two steps of slack).  Only the loads are issued
    // here; stage() resolves them, so that their latency overlaps the step's
    // computation.
    __device__ __forceinline__ void xload(const mwd_item<C>& I, uint32_t seq) {
        const uint32_t slotb = ((seq + 1 - R) & (kSlots - 1)) * C::RECB;
#pragma unroll
        for (int e = 0; e < NX; ++e) {
            const int l = J0 + e;
            if (nex<H>(B) > 0 && l > jo && l < jn) {
                // from the neighbour slice (value and stamp), or the shell
                // beyond the lattice (plane s + 1 - l R; o_ht is two steps
                // ahead) for an edge slice
                const uint32_t rec = I.nb_rec + slotb + xoff(I, I.hside ? 0 : 1, l) + (uint32_t)(I.hr * 4 + I.hc) * 8u;
                const auto v = __builtin_amdgcn_raw_buffer_load_b64(I.rX, (I.hlane && I.hx_nb) ? rec : kNone, 0, kSC1);
                x_v[e] = v[0];
                x_s[e] = v[1];
                x_sh[e] = __builtin_amdgcn_raw_buffer_load_b32(
                    I.rFT, (I.hlane && !I.hx_nb) ? o_ht - (uint32_t)(2 + (l - jo) * R) * I.sz4 : kNone, 0u, 0);
            }
        }
    }

    // the levels of step s, the new frontier, the slice's edge columns
    template <int P>
    __device__ __forceinline__ void compute(const mwd_item<C>& I, int s, uint32_t seq) {
        const mwd_kargs& a = *I.a;
        const float ot = p_ot[P];
#pragma unroll
        for (int m = QS - 1; m > 0; --m) qs[m] = qs[m - 1];
        qs[0] = p_qs[P];
        if constexpr (K > 0) {
            if constexpr (RL) {
#pragma unroll
                for (int kk = 0; kk < K; ++kk) {
                    if constexpr (std::is_same<typename C::RT, float>::value)
                        I.ring0[rslot][kk][I.ringw][I.lane] = p_c[P][kk];
                    else
                        I.ring0[rslot][kk][I.ringw][I.lane] = cbits(p_c[P][kk]);
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
        const float(*Pt)[C::XP] = I.tile[P];
        float vtop = ot, vsub = (jn == jo) ? qs[0] : ot;
#pragma unroll
        for (int jj = 0; jj < NL; ++jj) {
            const int j = J0 + jj;
            if (j > JO && j <= jn) {
                const int z = s - (j - 1) * R;
                float v;
                {
                    float Wv[C::KS];
                    Wv[0] = 0.0f;
                    if constexpr (K > 0) {
                        if constexpr (RL) {
                            int slot = rslot - (j - 1) * R;
                            slot = slot < 0 ? slot + NR0 : slot;
#pragma unroll
                            for (int kk = 0; kk < K; ++kk) {
                                if constexpr (std::is_same<typename C::RT, float>::value)
                                    Wv[kk] = I.ring0[slot][kk][I.ringw][I.lane];
                                else
                                    Wv[kk] = __uint_as_float((uint32_t)I.ring0[slot][kk][I.ringw][I.lane] << 16);
                            }
                        } else {
#pragma unroll
                            for (int kk = 0; kk < K; ++kk) Wv[kk] = cr[(j - J0) * R][kk];
                        }
                    }
                    // level j-1: z-queue (registers) and in-plane tile (LDS)
                    const float* zq = q[j - 1 - B >= 0 ? j - 1 - B : 0];
                    const float* T = &Pt[C::trow(j - 1, ylt)][xt];  // the lane's point
                    constexpr int XP = C::XP;
                    nbhd<R> n;
                    n.c = zq[R];
#pragma unroll
                    for (int r = 1; r <= R; ++r) {
                        n.pair[0][r - 1] = T[-r] + T[r];
                        n.pair[1][r - 1] = T[-r * XP] + T[r * XP];
                        n.pair[2][r - 1] = zq[R - r] + zq[R + r];
                    }
                    n.m1[0] = T[-1];
                    n.p1[0] = T[1];
                    n.m1[1] = T[-XP];
                    n.p1[1] = T[XP];
                    n.m1[2] = zq[R - 1];
                    n.p1[2] = zq[R + 1];
                    float pv = 0.0f;
                    if constexpr (C::LF) {
                        // level j-2 at plane z: the old sub for j = jo+1, else
                        // the oldest entry of level j-2's queue
                        if (j == JO + 1)
                            pv = qs[R + 1];
                        else
                            pv = q[j - 2 - B >= 0 ? j - 2 - B : 0][0];
                    }
                    v = update<C::KIND>(a.wt, Wv, n, pv);
                    // boundary shell: time independent, so a shell point of
                    // level j keeps the value it has at level j-1 (which is,
                    // level by level, the value the old top was loaded with)
                    const bool zin = z >= 0 && z < a.nz;
                    v = (intr && zin) ? v : n.c;
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
                    const uint32_t rec = I.my_rec + (seq & (kSlots - 1)) * C::RECB +
                                         xoff(I, I.eedge > 0 ? 1 : 0, j) + (uint32_t)(I.rr * 4 + I.ecol) * 8u;
                    u32x2 pk;
                    pk.x = __float_as_uint(v);
                    pk.y = I.stamp(seq);
                    __builtin_amdgcn_raw_buffer_store_b64(pk, I.rX, I.eedge >= 0 ? rec : kNone, 0, kSC1);
                }
            }
        }
        // new frontier: levels jn and jn-1 of the band's rows, at their planes
        // (o_ot is at plane s + 2 - (jo - 1) R: two steps ahead)
        {
            const int zt = s - (jn - 1) * R;
            const int zs = jn > jo ? s - (jn - 2) * R : s + 1 - (jo - 1) * R;
            const uint32_t ot_s = o_ot - 2u * I.sz4;  // plane s - (jo - 1) R
            const uint32_t st = ot_s - (uint32_t)((jn - jo) * R) * I.sz4;
            const uint32_t ss = jn > jo ? ot_s - (uint32_t)((jn - 1 - jo) * R) * I.sz4 : ot_s + I.sz4;
            bstore(I.rNT, vtop, (intr && zt >= I.z0 && zt < I.z1) ? st : kNone, 0u);
            bstore(I.rNS, vsub, (intr && zs >= I.z0 && zs < I.z1) ? ss : kNone, 0u);
        }
    }

    // stage the planes the next step reads in-plane: level l at plane
    // z_{l+1}(s+1) = s + 1 - l R, the halo columns, the flank rows
    template <int P>
    __device__ __forceinline__ void stage(const mwd_item<C>& I, uint32_t seq) {
        const mwd_kargs& a = *I.a;
        float(*Pn)[C::XP] = I.tile[P ^ 1];
        if constexpr (JO >= 1) Pn[C::trow(JO - 1, ylt)][xt] = qs[0];
        if constexpr (JO <= L - 1) {
            if constexpr (JO < J1)
                Pn[C::trow(JO, ylt)][xt] = q[JO - B][R + 1];
            else
                Pn[C::trow(JO, ylt)][xt] = qt[R - 1];
        }
#pragma unroll
        for (int jj = 0; jj < NL; ++jj) {
            const int l = J0 + jj;
            if (l > JO && l <= jn && l <= L - 1) {
                if (l < J1)
                    Pn[C::trow(l, ylt)][xt] = q[jj + 1 < NL ? jj + 1 : 0][R + 1];
                else
                    Pn[C::trow(l, ylt)][xt] = qt[R - 1];
            }
        }
        // halo columns: halo lanes write the tile, the others a spare slot
        if (jn > JO) *(I.hlane ? &Pn[C::trow(JO, hty)][htc] : I.spare) = p_ht[P];
        const bool xon = seq + 1 >= (uint32_t)R;
        const uint32_t want = I.stamp(seq + 1 - R);
#pragma unroll
        for (int e = 0; e < NX; ++e) {
            const int l = J0 + e;
            if (nex<H>(B) > 0 && l > jo && l < jn) {
                uint32_t v = I.hx_nb ? x_v[e] : x_sh[e];
                const bool nb = I.hlane && I.hx_nb && xon;
                if (__ballot(nb && x_s[e] != want)) {
                    // late: poll, coherent across the device, until the
                    // neighbour's value arrives
                    const uint32_t rec = I.nb_rec + ((seq + 1 - R) & (kSlots - 1)) * C::RECB +
                                         xoff(I, I.hside ? 0 : 1, l) + (uint32_t)(I.hr * 4 + I.hc) * 8u;
                    uint32_t got = nb ? x_s[e] : want;
                    // after one failure the run is invalid: do not wait again
                    int polls = __hip_atomic_load(a.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ? kPolls : 0;
                    while (__ballot(got != want) && polls < kPolls) {
                        __builtin_amdgcn_s_sleep(1);
                        if (got != want) {
                            const auto r2 = __builtin_amdgcn_raw_buffer_load_b64(I.rX, rec, 0, kSC1 | kVolatile);
                            v = r2[0];
                            got = r2[1];
                        }
                        ++polls;
                    }
                    if (got != want) atomicOr(a.err, 1);
                }
                *(I.hlane ? &Pn[C::trow(l, hty)][htc] : I.spare) = __uint_as_float(v);
            }
        }
        if (B == H - 1 && flank_on) Pn[C::trow(H - 1, ylf)][xt] = p_fl[P];
        rslot = rslot + 1 == NR0 ? 0 : rslot + 1;
    }
};

// The stream of one wave over one item: its one or two bands step together,
// one barrier per step.
template <class C, int BA, int BB, int JOA, int JOB, int JNA, int JNB>
__device__ __forceinline__ void mwd_run(mwd_item<C>& I, uint32_t& seq) {
    mwd_band<C, BA, JOA, JNA> A;
    A.init(I);
    constexpr int BBv = BB >= 0 ? BB : BA;  // (unused when BB < 0)
    mwd_band<C, BBv, JOB, JNB> Bd;
    if constexpr (BB >= 0) Bd.init(I);
    // prefetches run two steps ahead, also past the last step (their loads
    // are then unused), so that every running offset is two steps ahead of
    // the step in progress
    A.template prefetch<0>(I);
    if constexpr (BB >= 0) Bd.template prefetch<0>(I);
    A.template prefetch<1>(I);
    if constexpr (BB >= 0) Bd.template prefetch<1>(I);
    auto one = [&](int s, auto par) __attribute__((always_inline)) {
        constexpr int P = decltype(par)::value;
        A.xload(I, seq);
        if constexpr (BB >= 0) Bd.xload(I, seq);
        A.template compute<P>(I, s, seq);
        if constexpr (BB >= 0) Bd.template compute<P>(I, s, seq);
        A.template stage<P>(I, seq);
        if constexpr (BB >= 0) Bd.template stage<P>(I, seq);
        A.template prefetch<P>(I);
        if constexpr (BB >= 0) Bd.template prefetch<P>(I);
        ++seq;
        __syncthreads();
    };
    for (int s = I.s_begin; s < I.s_end; s += 2) {
        one(s, ic<0>{});
        if (s + 1 < I.s_end) one(s + 1, ic<1>{});
    }
}

template <class C, int BA, int BB>
__device__ __forceinline__ void mwd_dispatch(mwd_item<C>& I, uint32_t& seq) {
    constexpr int H = C::H;
    constexpr int JA = 2 * H - 1 - BA, JB = BB >= 0 ? 2 * H - 1 - BB : 0;
    if (I.t0 == -H) {
        // first row: level 0 is the old top of every row, levels 1 .. 2H-1-B
        // clipped to nt are computed
        mwd_run<C, BA, BB, H, H, 0, 0>(I, seq);
    } else if (I.t0 + 2 * H - 1 <= I.nt) {
        // the rows in between: every level of the diamond
        mwd_run<C, BA, BB, BA, (BB >= 0 ? BB : BA), JA, JB>(I, seq);
    } else {
        // last rows: levels clipped to nt; a band already at nt copies its pair
        mwd_run<C, BA, BB, BA, (BB >= 0 ? BB : BA), 0, 0>(I, seq);
    }
}

template <class C>
constexpr int mwd_lds_bytes() {
    return 2 * C::TR * C::XP * 4 + (C::LRING ? C::NR0 * C::K * 2 * C::NXW * 64 * (int)sizeof(typename C::RT) : 0);
}
// Waves per SIMD the registers are sized for: two workgroups per compute unit
// where the LDS allows it.  At H = 2 with 32-column slices that is 4 (128
// registers; a few spill to scratch, measured faster: BF16 25-point variable
// stencil 127 -> 149 GLUP/s, variable leapfrog 198 at dw 16); elsewhere 2
// (H <= 3) or 1.
template <class C>
constexpr int mwd_waves_per_eu() {
    if (mwd_lds_bytes<C>() > 80 * 1024) return 1;
    if (C::H == 2 && C::NXW == 2) return 4;
    return C::H <= 3 ? 2 : 1;
}

template <int KIND, typename CT, int H, int NXW, bool LRING, bool ALN, int CG>
__global__ __launch_bounds__(4 * NXW * 64)
__attribute__((amdgpu_waves_per_eu(mwd_waves_per_eu<mwd_cfg<KIND, CT, H, NXW, LRING, ALN, CG>>())))
void mwd_row_kernel(mwd_kargs a) {
    using C = mwd_cfg<KIND, CT, H, NXW, LRING, ALN, CG>;
    constexpr int R = C::R;
    __shared__ float tile[2][C::TR][C::XP];
    __shared__ typename C::RT ring0[LRING ? C::NR0 : 1][LRING ? C::K : 1][LRING ? 2 * NXW : 1][64];

    mwd_item<C> I;
    I.a = &a;
    I.tile = tile;
    I.ring0 = ring0;
    I.lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int group = w / (2 * NXW);
    I.side = (w / NXW) & 1;
    I.xw = w % NXW;
    I.ringw = w % (2 * NXW);  // the band-0 waves are group 0
    {
        const int sr = (w * 64 + I.lane) / C::SPL;  // sink row across both buffers
        I.spare = &tile[sr / C::TR][sr % C::TR][C::XT + I.lane % C::SPL];
    }
    I.cx = I.lane & 15;
    I.rr = I.lane >> 4;
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
    const int x0 = member * C::XS;
    I.xl = I.xw * 16 + I.cx;  // slice-local column of the lane
    I.x = x0 + I.xl;
    // halo lanes: lanes 0..31 of the slice's edge waves carry the R columns
    // beyond the slice (left for xw = 0, right for xw = NXW-1), rows rr
    I.hside = (I.lane >> 4) & 1;
    I.hr = (I.lane >> 2) & 3;
    I.hc = I.lane & 3;
    I.hlane = I.lane < 32 && (I.hside == 0 ? I.xw == 0 : I.xw == NXW - 1);
    I.xh = I.hside ? x0 + C::XS + I.hc : x0 - R + I.hc;
    I.hx_nb = I.hside ? member < a.k - 1 : member > 0;  // halo from a neighbour slice
    // edge lanes that publish the slice's outer R columns
    I.eedge = (I.xw == 0 && I.cx < 4) ? 0 : ((I.xw == NXW - 1 && I.cx >= 12) ? 1 : -1);
    I.ecol = I.eedge == 0 ? I.cx : I.cx - 12;
    I.rX = make_rsrc(a.xbuf, a.xbuf_bytes);
    I.my_rec = (uint32_t)(team * a.k + member) * kSlots * C::RECB;
    I.nb_rec = (uint32_t)(team * a.k + member + (I.hside ? 1 : -1)) * kSlots * C::RECB;
    I.t0 = a.t0;
    I.nt = a.nt;
    I.sz4 = (uint32_t)(a.sz * 4);
    I.szc = (uint32_t)(a.sz * C::CB);
    I.skb = (uint32_t)((uint64_t)a.sk * C::CB);
    auto nrec = [](uint64_t total, uint64_t off) -> uint32_t {
        const uint64_t r = total > off ? total - off : 0u;
        return (uint32_t)(r < 0x7fffffffull ? r : 0x7fffffffull);
    };

    uint32_t seq = 0;  // steps done by this workgroup in this launch
    for (int it = team; it < a.n_items; it += a.teams) {
        const int di = it / a.gz, zc = it % a.gz;
        I.yc = a.first_centre + di * C::DW;
        I.z0 = zc * a.zchunk;
        I.z1 = min(a.nz, I.z0 + a.zchunk);
        // Level j is needed at planes [z0 - R(L-j), z1 + R(L-j)) (clipped to
        // [-R, nz+R)): the chunk's outputs at level L depend on nothing wider.
        // Every level is computed at every step; values outside a level's
        // window are never read by values inside the windows, so they need no
        // test.  Level 1 starts at its window, after 2R steps that fill the
        // z-queue of the old top.
        I.s_begin = max(I.z0 - R * (C::L - 1), -R) - 2 * R;
        I.s_end = I.z1 + (C::L - 1) * R;
        // Buffers are based at plane zw, below every plane the item reads, so
        // that 32-bit offsets cover the item's window.  A lane's offset is its
        // row and column plus the plane; it advances by one plane per step.
        // Planes below zw give offsets above 2^31 and planes beyond a buffer
        // offsets beyond its size: both read 0 and store nothing.
        I.zw = max(I.z0 - R * (C::L + 2), -a.hh);
        const uint64_t fwb = (uint64_t)(I.zw + a.hh) * (uint64_t)a.sz * 4u;
        const uint64_t cwb = (uint64_t)(I.zw + a.hh) * (uint64_t)a.sz * C::CB;
        const uint32_t fnr = nrec(a.field_bytes, fwb);
        I.rFT = make_rsrc(reinterpret_cast<const char*>(a.ftop_o) + fwb, fnr);
        I.rFS = make_rsrc(reinterpret_cast<const char*>(a.fsub_o) + fwb, fnr);
        I.rNT = make_rsrc(reinterpret_cast<const char*>(a.ftop_n) + fwb, fnr);
        I.rNS = make_rsrc(reinterpret_cast<const char*>(a.fsub_n) + fwb, fnr);
        // Coefficient arrays: groups of CG arrays share one resource based at
        // the first array's window and spanning the group (the range check
        // covers the scalar offset too); array k is reached with the scalar
        // offset (k mod CG) * sk bytes, the lane's offset in the vector offset.
        const uint32_t cnr = nrec(a.coef_bytes, cwb);
#pragma unroll
        for (int g = 0; g < C::NG; ++g) {
            const int ng = min(C::CG, C::KG - g * C::CG);
            const uint64_t span = (uint64_t)(ng - 1) * I.skb + cnr;
            I.rC[g] = __builtin_amdgcn_make_buffer_rsrc(
                const_cast<char*>(static_cast<const char*>(a.coef) + (uint64_t)(g * C::CG) * (uint64_t)a.sk * C::CB + cwb),
                (short)0, (int)(uint32_t)(span < 0xffffffffull ? span : 0xffffffffull), 0x00020000);
        }
        if (group == 0)
            mwd_dispatch<C, gband<H>(0, 0), gband<H>(0, 1)>(I, seq);
        else
            mwd_dispatch<C, gband<H>(1, 0), gband<H>(1, 1)>(I, seq);
    }
}

__global__ void fill_u32_kernel(uint32_t* p, uint64_t n, uint32_t v) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

template <int KIND, typename CT, int H, int NXW, bool LRING, bool ALN, int CG>
struct mwd_inst {
    static constexpr int threads = 4 * NXW * 64;
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

// Slice width xs (0 = the default for the width): 32 columns at H = 2, and at
// H = 3, 4 of the leapfrogs; 16 columns at H = 3 of the 25-point variable
// stencil, whose LDS coefficient ring for 32 columns would not fit beside the
// tiles (xs = 32 is not provided there).
template <int KIND, typename CT, bool ALN, int CG>
hipError_t pick_cg(int dw, int nx, int xs, team_layout* t) {
    constexpr int R = kR;
    const int H = dw / (2 * R);
    if constexpr (KIND == 3) {
        if (H == 2) {
            if (xs == 16) return layout_of<mwd_inst<KIND, CT, 2, 1, true, ALN, CG>>(nx, t);
            return layout_of<mwd_inst<KIND, CT, 2, 2, true, ALN, CG>>(nx, t);
        }
        if (H == 3 && xs != 32) return layout_of<mwd_inst<KIND, CT, 3, 1, true, ALN, CG>>(nx, t);
    } else {
        if (xs == 16) {
            if (H == 2) return layout_of<mwd_inst<KIND, CT, 2, 1, false, ALN, CG>>(nx, t);
            if (H == 3) return layout_of<mwd_inst<KIND, CT, 3, 1, false, ALN, CG>>(nx, t);
            if (H == 4) return layout_of<mwd_inst<KIND, CT, 4, 1, false, ALN, CG>>(nx, t);
        } else {
            if (H == 2) return layout_of<mwd_inst<KIND, CT, 2, 2, false, ALN, CG>>(nx, t);
            if (H == 3) return layout_of<mwd_inst<KIND, CT, 3, 2, false, ALN, CG>>(nx, t);
            if (H == 4) return layout_of<mwd_inst<KIND, CT, 4, 2, false, ALN, CG>>(nx, t);
        }
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
hipError_t pick_aln(int dw, int nx, int xs, int cg, team_layout* t) {
    if constexpr (KIND == 3) {
        if (cg == 13) return pick_cg<KIND, CT, ALN, 13>(dw, nx, xs, t);
        if (cg == 7) return pick_cg<KIND, CT, ALN, 7>(dw, nx, xs, t);
    }
    return pick_cg<KIND, CT, ALN, 1>(dw, nx, xs, t);
}

template <int KIND, typename CT>
hipError_t pick(int dw, int nx, int xs, bool aln, int cg, team_layout* t) {
    if constexpr (std::is_same<CT, uint16_t>::value) {
        if (aln) return pick_aln<KIND, CT, true>(dw, nx, xs, cg, t);
    }
    return pick_aln<KIND, CT, false>(dw, nx, xs, cg, t);
}

hipError_t pick_any(int kind, bool bf16, int dw, int nx, int xs, bool aln, int cg,
                    team_layout* t) {
    switch (kind) {
    case 3:
        return bf16 ? pick<3, uint16_t>(dw, nx, xs, aln, cg, t)
                    : pick<3, float>(dw, nx, xs, aln, cg, t);
    case 4: return pick<4, float>(dw, nx, xs, false, 1, t);
    case 5:
        return bf16 ? pick<5, uint16_t>(dw, nx, xs, aln, 1, t)
                    : pick<5, float>(dw, nx, xs, aln, 1, t);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

bool mwd_supported(int kind, int dw, int xs) {
    if (kind < 3 || kind > 5 || dw % (2 * kR) != 0) return false;
    if (xs != 0 && xs != 16 && xs != 32) return false;
    const int H = dw / (2 * kR);
    if (kind == 3) return H == 2 || (H == 3 && xs != 32);
    return H >= 2 && H <= 4;
}

int mwd_slices(int kind, int dw, int xs, int nx) {
    if (!mwd_supported(kind, dw, xs)) return 0;
    const int H = dw / (2 * kR);
    const int w = xs ? xs : ((kind == 3 && H == 3) ? 16 : 32);
    return nx < 1 ? 1 : (nx + w - 1) / w;
}

hipError_t mwd_workspace(int kind, bool bf16, int dw, int xs, int nx, size_t* xbytes) {
    team_layout t;
    hipError_t e = pick_any(kind, bf16, dw, nx, xs, false, 1, &t);
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
    hipError_t e = pick_any(kind, bf16, r.dw, r.d.nx, r.xs, r.coef_aligned,
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
