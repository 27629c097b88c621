// C ABI of libstencil.so: argument validation, contexts, workspace and the
// host-side time loop.  Every argument is checked before the first HIP call,
// so every error path can be exercised on a machine without a GPU.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/stencil.h"
#include "adjoint.h"
#include "blocked.h"
#include "kernels.h"
#include "plan.h"

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int dev_fail(hipError_t e, const char* what) {
    return fail(STENCIL_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

int kind_radius(int kind) { return (kind == 1 || kind == 2) ? 1 : 4; }
int kind_ncoef(int kind) {
    switch (kind) {
    case 2: return 7;
    case 3: return 13;
    case 5: return 1;
    default: return 0;
    }
}
bool kind_leapfrog(int kind) { return kind == 4 || kind == 5; }

}  // namespace

struct stencil_ctx {
    stencil_scheme scheme;
    stencil_tuning tuning;
    hipStream_t stream;
    int device;
    // workspace: a list of device allocations owned by the context
    std::vector<std::pair<void*, size_t>> bufs;
    size_t ws_bytes = 0;
    // blocked scheme frontier buffers (two pairs of fields)
    void* frontier = nullptr;
    size_t frontier_bytes = 0;
    // radius-4 blocked scheme: halo exchange buffer of the workgroup teams
    // (the error flag follows it), and the flag the last run used
    void* xchg = nullptr;
    size_t xchg_bytes = 0;
    int* err_dev = nullptr;
    uint32_t tag = 0;  // launch tag of the last row launch (1 .. 4095)
    // checkpoints recorded by stencil_run for stencil_adjoint (kinds 2, 3, 5)
    struct recording {
        bool valid = false;
        int kind = 0;
        int nx = 0, ny = 0, nz = 0, halo = 0;
        int64_t sy = 0, sz = 0, nt = 0, sk = 0;
        int every = 0;            // checkpoint interval k
        const void* coef = nullptr;
        int dtype = 0;
        void* buf = nullptr;      // kind 5: 2n fields (u_{qk-1}, u_{qk}); kinds 2, 3: n
                                  // fields u_{qk}; q = 0 .. n-1
        size_t bytes = 0;         // allocated size of buf
        size_t lead = 0, stride = 0;  // placement of the fields (elements)
        int n = 0;
        const float* field(size_t i) const {
            return static_cast<const float*>(buf) + lead + i * stride;
        }
    } rec;
};

namespace {

// Allocate (or reuse) a device workspace region tracked by the context.
int ws_alloc(stencil_ctx* ctx, size_t bytes, void** out) {
    if (ctx->tuning.workspace_limit > 0 &&
        ctx->ws_bytes + bytes > (size_t)ctx->tuning.workspace_limit)
        return fail(STENCIL_ERR_NOMEM,
                    "workspace of %zu bytes exceeds the tuning limit of %lld bytes",
                    ctx->ws_bytes + bytes, (long long)ctx->tuning.workspace_limit);
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(STENCIL_ERR_NOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
    }
    ctx->bufs.push_back({p, bytes});
    ctx->ws_bytes += bytes;
    *out = p;
    return STENCIL_OK;
}

void ws_free(stencil_ctx* ctx, void* p) {
    for (size_t i = 0; i < ctx->bufs.size(); ++i)
        if (ctx->bufs[i].first == p) {
            (void)hipFree(p);
            ctx->ws_bytes -= ctx->bufs[i].second;
            ctx->bufs.erase(ctx->bufs.begin() + (long)i);
            return;
        }
}

// Elements spanned by one padded field (from the origin to the last element).
int64_t field_span(const stencil_grid* g) {
    const int64_t h = g->halo;
    return (g->nz + 2 * h - 1) * g->sz + (g->ny + 2 * h - 1) * g->sy + (g->nx + 2 * h);
}

// Placement of workspace fields.  Field i of a workspace region starts `lead`
// elements into the region plus i strides of a multiple of 64 elements, so
// that its rows sit on the same 256-byte boundaries as those of the caller's
// u[0] (hipMalloc regions are 256-byte aligned); a misaligned copy would
// split every 256-byte row access of a wave over three cache lines.
struct field_layout {
    size_t lead = 0, stride = 0, span = 0;  // elements
    size_t bytes(size_t n) const { return (lead + n * stride) * sizeof(float) + 256; }
    float* at(void* base, size_t i) const { return static_cast<float*>(base) + lead + i * stride; }
};

field_layout layout_of(const stencil_grid* g) {
    field_layout L;
    L.span = (size_t)field_span(g);
    L.stride = (L.span + 63) / 64 * 64;
    L.lead = (size_t)((reinterpret_cast<uintptr_t>(g->u[0]) / sizeof(float)) % 64);
    return L;
}

int validate_grid(int kind, const stencil_grid* g) {
    if (!g) return fail(STENCIL_ERR_INVALID, "grid is NULL");
    if (g->nx < 0 || g->ny < 0 || g->nz < 0)
        return fail(STENCIL_ERR_INVALID, "negative grid size (%d, %d, %d)", g->nx, g->ny, g->nz);
    const int R = kind_radius(kind);
    if (g->halo < R)
        return fail(STENCIL_ERR_INVALID, "halo %d is smaller than the stencil radius %d", g->halo, R);
    if (g->halo > 64) return fail(STENCIL_ERR_INVALID, "halo %d is larger than 64", g->halo);
    const int64_t px = (int64_t)g->nx + 2 * g->halo, py = (int64_t)g->ny + 2 * g->halo;
    if (g->sy < px)
        return fail(STENCIL_ERR_INVALID, "row stride sy=%lld < nx + 2*halo = %lld",
                    (long long)g->sy, (long long)px);
    if (g->sz < g->sy * py)
        return fail(STENCIL_ERR_INVALID, "plane stride sz=%lld < sy*(ny + 2*halo) = %lld",
                    (long long)g->sz, (long long)(g->sy * py));
    if ((int64_t)g->nx + 2 * g->halo > (1 << 30) || (int64_t)g->ny + 2 * g->halo > (1 << 30) ||
        (int64_t)g->nz + 2 * g->halo > (1 << 30))
        return fail(STENCIL_ERR_INVALID, "grid dimension too large");
    if (!g->u[0] || !g->u[1]) return fail(STENCIL_ERR_INVALID, "grid field pointer is NULL");
    if (g->u[0] == g->u[1]) return fail(STENCIL_ERR_INVALID, "u[0] and u[1] must be distinct");
    return STENCIL_OK;
}

int validate_coeffs(int kind, const stencil_grid* g, const stencil_coeffs* c) {
    if (!c) return fail(STENCIL_ERR_INVALID, "coeffs is NULL");
    if (c->dtype != STENCIL_F32 && c->dtype != STENCIL_BF16)
        return fail(STENCIL_ERR_INVALID, "unknown coefficient dtype %d", (int)c->dtype);
    const int K = kind_ncoef(kind);
    if (K == 0) {
        if (c->dtype != STENCIL_F32)
            return fail(STENCIL_ERR_UNSUPPORTED,
                        "BF16 coefficient storage needs a variable-coefficient kind (2, 3, 5)");
    } else {
        if (!c->arrays) return fail(STENCIL_ERR_INVALID, "kind %d needs %d coefficient arrays", kind, K);
        if (K > 1 && c->sk < field_span(g))
            return fail(STENCIL_ERR_INVALID, "coefficient stride sk=%lld overlaps the arrays (need >= %lld)",
                        (long long)c->sk, (long long)field_span(g));
    }
    for (int i = 0; i < 5; ++i)
        if (!std::isfinite(c->w[i])) return fail(STENCIL_ERR_INVALID, "w[%d] is not finite", i);
    if (!std::isfinite(c->alpha)) return fail(STENCIL_ERR_INVALID, "alpha is not finite");
    return STENCIL_OK;
}

stn::dims to_dims(const stencil_grid* g) {
    stn::dims d;
    d.nx = g->nx; d.ny = g->ny; d.nz = g->nz; d.h = g->halo; d.sy = g->sy; d.sz = g->sz;
    return d;
}

stn::host_weights to_weights(const stencil_coeffs* c) {
    stn::host_weights w;
    for (int i = 0; i < 5; ++i) w.w[i] = (float)c->w[i];
    w.alpha = (float)c->alpha;
    w.lres = (float)(c->w[0] + 6.0 * (c->w[1] + c->w[2] + c->w[3] + c->w[4]));
    return w;
}

bool empty(const stencil_grid* g) { return g->nx == 0 || g->ny == 0 || g->nz == 0; }

// The context binds to the device that is current at its first device call.
int set_device(stencil_ctx* ctx) {
    if (ctx->device < 0) {
        int dev = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return dev_fail(e, "hipGetDevice");
        ctx->device = dev;
        return STENCIL_OK;
    }
    // switch only when needed: a run captured into a HIP graph then makes
    // no call besides its launches and copies
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e == hipSuccess && cur == ctx->device) return STENCIL_OK;
    e = hipSetDevice(ctx->device);
    return e == hipSuccess ? STENCIL_OK : dev_fail(e, "hipSetDevice");
}

// Naive time loop: nt launches, two-buffer storage.  The boundary is time
// independent: before the first step the level-0 buffer's shell is copied
// into the other buffer, which the odd steps read.
int run_naive(stencil_ctx* ctx, int kind, const stencil_grid* g, const stencil_coeffs* c,
              int64_t nt) {
    const stn::dims d = to_dims(g);
    const stn::host_weights w = to_weights(c);
    const bool bf16 = c->dtype == STENCIL_BF16;
    float* u0 = static_cast<float*>(g->u[0]);
    float* u1 = static_cast<float*>(g->u[1]);
    if (nt >= 1) {
        const bool lf = kind_leapfrog(kind);
        hipError_t e = stn::launch_copy_shell(lf ? u0 : u1, lf ? u1 : u0, d, kind_radius(kind),
                                              ctx->stream);
        if (e != hipSuccess) return dev_fail(e, "shell copy");
    }
    for (int64_t t = 0; t < nt; ++t) {
        hipError_t e;
        if (kind_leapfrog(kind)) {
            // level t lives in u[(t+1)%2]; level t+1 overwrites level t-1
            float* cur = (t % 2 == 0) ? u1 : u0;
            float* old = (t % 2 == 0) ? u0 : u1;
            e = stn::launch_naive_step(kind, bf16, cur, old, old, c->arrays, c->sk, d, w,
                                       ctx->tuning.zchunk, ctx->stream);
        } else {
            const float* cur = (t % 2 == 0) ? u0 : u1;
            float* nxt = (t % 2 == 0) ? u1 : u0;
            e = stn::launch_naive_step(kind, bf16, cur, nullptr, nxt, c->arrays, c->sk, d, w,
                                       ctx->tuning.zchunk, ctx->stream);
        }
        if (e != hipSuccess) return dev_fail(e, "naive step launch");
    }
    return STENCIL_OK;
}


// Device workspace for the blocked scheme's second frontier pair.
int ensure_frontier(stencil_ctx* ctx, size_t bytes) {
    if (ctx->frontier && ctx->frontier_bytes >= bytes) return STENCIL_OK;
    if (ctx->frontier) {
        ws_free(ctx, ctx->frontier);
        ctx->frontier = nullptr;
        ctx->frontier_bytes = 0;
    }
    void* p = nullptr;
    int rc = ws_alloc(ctx, bytes, &p);
    if (rc) return rc;
    ctx->frontier = p;
    ctx->frontier_bytes = bytes;
    return STENCIL_OK;
}

// Device workspace for the exchange buffer of the radius-4 blocked scheme.
int ensure_exchange(stencil_ctx* ctx, size_t bytes) {
    if (ctx->xchg && ctx->xchg_bytes >= bytes) return STENCIL_OK;
    if (ctx->xchg) {
        ws_free(ctx, ctx->xchg);
        ctx->xchg = nullptr;
        ctx->xchg_bytes = 0;
    }
    void* p = nullptr;
    int rc = ws_alloc(ctx, bytes, &p);
    if (rc) return rc;
    ctx->xchg = p;
    ctx->xchg_bytes = bytes;
    return STENCIL_OK;
}

// The context's frontier workspace for a blocked run on grid g (none for
// the naive scheme).
int ensure_frontier_for(stencil_ctx* ctx, const stencil_grid* g) {
    if (ctx->scheme != STENCIL_BLOCKED) return STENCIL_OK;
    return ensure_frontier(ctx, layout_of(g).bytes(2));
}

// Planes per z-chunk of the blocked kernel whose address window (the chunk
// plus 2R(L+1) + 1 planes, from a base of the workgroup's own) stays below
// 2^31 bytes, so that 32-bit offsets reach it; < 1 if none does.
int64_t blocked_max_zchunk(int kind, int dw, const stencil_grid* g) {
    const int R = kind_radius(kind);
    const int L = 2 * (dw / (2 * R)) - 1;
    const int64_t plane = g->sz * (int64_t)sizeof(float);
    return (int64_t)0x7fffffff / plane - 2LL * R * (L + 1) - 1;
}

// Diamond width of a blocked run: the context's, else the library's choice
// for the grid's size and the coefficients' storage.
int blocked_dw(const stencil_ctx* ctx, int kind, const stencil_grid* g, const stencil_coeffs* c) {
    if (ctx->tuning.dw) return ctx->tuning.dw;
    const bool bf16 = c && c->dtype == STENCIL_BF16;
    return stn::blocked_default_dw(kind, (int64_t)g->nx * g->ny * g->nz, bf16);
}

// Limits of the blocked scheme, checked with the other arguments before any
// HIP call: a provided diamond width, and an address window of one z-chunk
// plane below 2^31 bytes (planes below about 2^31 / (2R(L+1) + 2) bytes).
int check_blocked(const stencil_ctx* ctx, int kind, const stencil_grid* g,
                  const stencil_coeffs* c) {
    const int dw = blocked_dw(ctx, kind, g, c);
    const int xs = kind_radius(kind) == 4 ? ctx->tuning.xtile : 0;
    if (!stn::blocked_supported(kind, dw, xs))
        return fail(STENCIL_ERR_UNSUPPORTED,
                    "blocked scheme: dw=%d with xtile=%d is not provided for kind %d", dw, xs,
                    kind);
    if (blocked_max_zchunk(kind, dw, g) < 1)
        return fail(STENCIL_ERR_UNSUPPORTED,
                    "blocked scheme: a plane of %lld bytes is too large for the 2 GiB address "
                    "window of a z-chunk",
                    (long long)(g->sz * (int64_t)sizeof(float)));
    return STENCIL_OK;
}

// Blocked time loop (diamond rows of plan.h, one launch per row).  The
// frontier pair alternates between the caller's buffers and a workspace pair;
// when the number of rows is odd the initial state is first copied to the
// workspace so that the last row writes the caller's buffers, with level nt in
// the slot the two-buffer convention prescribes.
// `frontier` is the second frontier pair (FL.bytes(2) bytes): the context's
// workspace, or the library's scratch for the allocation-free entry point.
// The radius-4 kinds also need the teams' exchange buffer: `xchg` (xcap
// bytes) or, if NULL, the context's workspace.
int run_blocked(stencil_ctx* ctx, int kind, const stencil_grid* g, const stencil_coeffs* c,
                int64_t nt, void* frontier, void* xchg = nullptr, size_t xcap = 0) {
    const int R = kind_radius(kind);
    const int dw = blocked_dw(ctx, kind, g, c);
    const int H = dw / (2 * R);
    const int L = 2 * H - 1;
    const stn::dims d = to_dims(g);
    const stn::diamond_plan plan = stn::make_plan(R, dw, g->ny, nt);
    const field_layout FL = layout_of(g);
    const size_t fbytes = FL.span * sizeof(float);
    float* w0 = FL.at(frontier, 0);
    float* w1 = FL.at(frontier, 1);
    float* u0 = static_cast<float*>(g->u[0]);
    float* u1 = static_cast<float*>(g->u[1]);
    const bool lf = kind_leapfrog(kind);
    const int slot = lf ? (int)((nt + 1) % 2) : (int)(nt % 2);
    float* fin_top = slot ? u1 : u0;
    float* fin_sub = slot ? u0 : u1;
    const float* rt = lf ? u1 : u0;  // level 0
    const float* rs = lf ? u0 : u1;  // level -1 (leapfrog) / unused (Jacobi)
    // The blocked kernel reads boundary values from whichever frontier buffer
    // holds the newest level, so every buffer it reads carries the shell of
    // the level-0 buffer (the boundary is time independent).
    const float* shell = rt;
    float* other = const_cast<float*>(rs);
    hipError_t e = stn::launch_copy_shell(other, shell, d, R, ctx->stream);
    if (e != hipSuccess) return dev_fail(e, "shell copy");
    bool reading_caller = true;
    if (plan.rows.size() % 2 == 1) {
        e = hipMemcpyAsync(w0, rt, fbytes, hipMemcpyDeviceToDevice, ctx->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(w1, rs, fbytes, hipMemcpyDeviceToDevice, ctx->stream);
        if (e != hipSuccess) return dev_fail(e, "frontier copy");
        rt = w0;
        rs = w1;
        reading_caller = false;
    } else {
        e = stn::launch_copy_shell(w0, shell, d, R, ctx->stream);
        if (e == hipSuccess) e = stn::launch_copy_shell(w1, shell, d, R, ctx->stream);
        if (e != hipSuccess) return dev_fail(e, "shell copy");
    }
    const bool bf16 = c->dtype == STENCIL_BF16;
    const int xs = ctx->tuning.xtile;
    if (stn::mwd_supported(kind, dw, xs)) {
        size_t xbytes = 0;
        e = stn::mwd_workspace(kind, bf16, dw, xs, g->nx, &xbytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(STENCIL_ERR_UNSUPPORTED,
                        "blocked scheme: no team of workgroups for nx=%d fits the device (%s)",
                        g->nx, hipGetErrorString(e));
        }
        const size_t need = xbytes + 256;  // the error flag follows the buffer
        if (!xchg) {
            int rc = ensure_exchange(ctx, need);
            if (rc) return rc;
            xchg = ctx->xchg;
        } else if (need > xcap) {
            return fail(STENCIL_ERR_UNSUPPORTED,
                        "stencil_run_noalloc: the frontier pair and the %zu-byte halo exchange "
                        "buffer exceed the library's %zu-byte scratch",
                        need, stn::kScratchBytes);
        }
        int* err = reinterpret_cast<int*>(static_cast<char*>(xchg) + xbytes);
        ctx->err_dev = err;
        e = stn::launch_fill_u32(xchg, need / 4, 0u, ctx->stream);
        if (e != hipSuccess) return dev_fail(e, "exchange clear");
        for (const stn::diamond_row& row : plan.rows) {
            stn::mwd_row_args a;
            a.ftop_o = rt;
            a.fsub_o = rs;
            a.ftop_n = reading_caller ? w0 : fin_top;
            a.fsub_n = reading_caller ? w1 : fin_sub;
            a.coef = c->arrays;
            a.sk = c->sk;
            a.d = d;
            a.wt = to_weights(c);
            a.t0 = row.t0;
            a.nt = nt;
            a.first_centre = row.first_centre;
            a.n_diamonds = row.n_diamonds;
            a.dw = dw;
            a.xs = xs;
            a.zchunk = ctx->tuning.zchunk;
            a.field_bytes = fbytes;
            a.coef_bytes = FL.span * (bf16 ? 2 : 4);
            a.xbuf = xchg;
            a.xbuf_bytes = xbytes;
            a.coef_aligned = bf16 && (reinterpret_cast<uintptr_t>(c->arrays) & 3u) == 0 &&
                             c->sk % 2 == 0 && g->sz % 2 == 0;
            a.err = err;
            // stamps differ between consecutive launches; after 4095 launches
            // the tags repeat and the buffer is cleared again
            if (ctx->tag >= 4095) {
                ctx->tag = 0;
                e = stn::launch_fill_u32(xchg, xbytes / 4, 0u, ctx->stream);
                if (e != hipSuccess) return dev_fail(e, "exchange clear");
            }
            a.tag = ++ctx->tag;
            e = stn::launch_mwd_row(kind, bf16, a, ctx->stream);
            if (e != hipSuccess) return dev_fail(e, "blocked row launch");
            rt = a.ftop_n;
            rs = a.fsub_n;
            reading_caller = !reading_caller;
        }
        return STENCIL_OK;
    }
    const int64_t zmax = blocked_max_zchunk(kind, dw, g);
    const int xomax = stn::blocked_max_xo(kind, dw);
    const int gx = (g->nx + xomax - 1) / xomax;
    const int xo = (g->nx + gx - 1) / gx;
    const bool coef_aligned = bf16 && (reinterpret_cast<uintptr_t>(c->arrays) & 3u) == 0 &&
                              c->sk % 2 == 0 && g->sz % 2 == 0;
    // workgroups of the row kernel the device holds at once, for the z-chunk
    long long slots = 0;
    if (ctx->tuning.zchunk <= 0) {
        stn::blocked_row_args q;
        q.dw = dw;
        q.field_bytes = fbytes;
        q.coef_bytes = FL.span * (bf16 ? 2 : 4);
        q.slots_out = &slots;
        q.coef_aligned = coef_aligned;
        e = stn::launch_blocked_row(kind, bf16, q, ctx->stream);
        if (e != hipSuccess) return dev_fail(e, "blocked occupancy query");
    }
    for (const stn::diamond_row& row : plan.rows) {
        stn::blocked_row_args a;
        a.ftop_o = rt;
        a.fsub_o = rs;
        a.ftop_n = reading_caller ? w0 : fin_top;
        a.fsub_n = reading_caller ? w1 : fin_sub;
        a.coef = c->arrays;
        a.sk = c->sk;
        a.d = d;
        a.wt = to_weights(c);
        a.t0 = row.t0;
        a.nt = nt;
        a.first_centre = row.first_centre;
        a.n_diamonds = row.n_diamonds;
        a.dw = dw;
        a.field_bytes = fbytes;
        a.coef_bytes = FL.span * (bf16 ? 2 : 4);
        a.xo = xo;
        a.coef_aligned = coef_aligned;
        a.gx = gx;
        int zc = ctx->tuning.zchunk;
        if (zc <= 0) {
            // the chunk count that minimises rounds of resident workgroups x
            // steps per workgroup (its chunk plus the 2RL steps that fill and
            // drain the wavefront)
            zc = stn::pick_zchunk(g->nz, (long long)row.n_diamonds * gx, slots, R * L);
        }
        zc = (int)std::min<int64_t>(zc, zmax);
        a.zchunk = zc;
        a.gz = (g->nz + zc - 1) / zc;
        if ((long long)a.n_diamonds * a.gx * a.gz > 0x7fffffffLL)
            return fail(STENCIL_ERR_INVALID, "grid too large for one launch");
        e = stn::launch_blocked_row(kind, bf16, a, ctx->stream);
        if (e != hipSuccess) return dev_fail(e, "blocked row launch");
        rt = a.ftop_n;
        rs = a.fsub_n;
        reading_caller = !reading_caller;
    }
    return STENCIL_OK;
}

// Forward run in segments of k steps, copying the state at t = q k into
// checkpoint q before segment q: (u_{t-1}, u_t) for the leapfrog, u_t for the
// Jacobi kinds.  A segment runs on a grid whose u[0], u[1] are the buffers
// holding (u_{t-1}, u_t) (leapfrog) or (u_t, the other buffer) (Jacobi), so
// the two-buffer convention is the same as in one long run.  Jacobi
// checkpoints get the boundary shell of u[0], the level-0 buffer.  With k = 1
// (every level recorded) a Jacobi forward writes each level straight into
// its checkpoint, so recording costs no extra pass over the lattice.
int run_recorded(stencil_ctx* ctx, int kind, const stencil_grid* g, const stencil_coeffs* c,
                 int64_t nt, int k, stencil_ctx::recording* rec) {
    const field_layout FL = layout_of(g);
    const size_t span = FL.span;
    const bool lf = kind_leapfrog(kind);
    const size_t nf = lf ? 2 : 1;
    const int n = (int)((nt + k - 1) / k);
    // leapfrog with k = 1: one field per level u_{-1} .. u_{nt-1}
    const bool lf_all = lf && k == 1;
    const size_t need = FL.bytes(lf_all ? (size_t)nt + 1 : nf * (size_t)n);
    if (!rec->buf || rec->bytes < need) {
        if (rec->buf) ws_free(ctx, rec->buf);
        rec->buf = nullptr;
        rec->bytes = 0;
        rec->valid = false;
        void* p = nullptr;
        int rc = ws_alloc(ctx, need, &p);
        if (rc) return rc;
        rec->buf = p;
        rec->bytes = need;
    }
    rec->valid = false;
    rec->lead = FL.lead;
    rec->stride = FL.stride;
    rec->n = n;
    if (!lf && k == 1) {
        // every level is a checkpoint: the sweeps write straight into the
        // recording (level-0 shell on every field), the last into the buffer
        // that holds level nt
        const stn::dims d = to_dims(g);
        const stn::host_weights wt = to_weights(c);
        const bool bf16 = c->dtype == STENCIL_BF16;
        const float* u0 = static_cast<const float*>(g->u[0]);
        hipError_t e = hipMemcpyAsync(FL.at(rec->buf, 0), u0, span * sizeof(float),
                                      hipMemcpyDeviceToDevice, ctx->stream);
        for (int i = 1; i < n && e == hipSuccess; ++i)
            e = stn::launch_copy_shell(FL.at(rec->buf, (size_t)i), u0, d, kind_radius(kind),
                                       ctx->stream);
        for (int64_t t = 0; t < nt && e == hipSuccess; ++t) {
            float* out = t + 1 < nt ? FL.at(rec->buf, (size_t)(t + 1))
                                    : static_cast<float*>(g->u[nt % 2]);
            e = stn::launch_naive_step(kind, bf16, FL.at(rec->buf, (size_t)t), nullptr, out,
                                       c->arrays, c->sk, d, wt, ctx->tuning.zchunk, ctx->stream);
        }
        if (e != hipSuccess) return dev_fail(e, "recorded forward");
    } else if (lf_all) {
        // every level recorded, field i = u_{i-1}: the sweeps write each level
        // into its own field (level-0 shell on every field), the last into
        // the caller's buffer for level nt, and u_{nt-1} is copied into the
        // other buffer, as the two-buffer convention asks
        const stn::dims d = to_dims(g);
        const stn::host_weights wt = to_weights(c);
        const bool bf16 = c->dtype == STENCIL_BF16;
        const float* u0 = static_cast<const float*>(g->u[1]);
        hipError_t e = hipMemcpyAsync(FL.at(rec->buf, 0), g->u[0], span * sizeof(float),
                                      hipMemcpyDeviceToDevice, ctx->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(FL.at(rec->buf, 1), u0, span * sizeof(float),
                               hipMemcpyDeviceToDevice, ctx->stream);
        for (int64_t i = 2; i <= nt && e == hipSuccess; ++i)
            e = stn::launch_copy_shell(FL.at(rec->buf, (size_t)i), u0, d, kind_radius(kind),
                                       ctx->stream);
        for (int64_t t = 0; t < nt && e == hipSuccess; ++t) {
            float* out = t + 1 < nt ? FL.at(rec->buf, (size_t)(t + 2))
                                    : static_cast<float*>(g->u[(nt + 1) % 2]);
            e = stn::launch_naive_step(kind, bf16, FL.at(rec->buf, (size_t)(t + 1)),
                                       FL.at(rec->buf, (size_t)t), out, c->arrays, c->sk, d, wt,
                                       ctx->tuning.zchunk, ctx->stream);
        }
        if (e == hipSuccess)
            e = hipMemcpyAsync(g->u[nt % 2], FL.at(rec->buf, (size_t)nt), span * sizeof(float),
                               hipMemcpyDeviceToDevice, ctx->stream);
        if (e != hipSuccess) return dev_fail(e, "recorded forward");
    } else {
        for (int q = 0; q < n; ++q) {
            const int64_t t = (int64_t)q * k;
            const int64_t steps = std::min<int64_t>(k, nt - t);
            stencil_grid sub = *g;
            sub.u[0] = g->u[t % 2];        // leapfrog: u_{t-1}; Jacobi: u_t
            sub.u[1] = g->u[(t + 1) % 2];  // leapfrog: u_t
            hipError_t e = hipMemcpyAsync(FL.at(rec->buf, nf * (size_t)q), sub.u[0],
                                          span * sizeof(float), hipMemcpyDeviceToDevice,
                                          ctx->stream);
            if (e == hipSuccess && lf)
                e = hipMemcpyAsync(FL.at(rec->buf, 2 * (size_t)q + 1), sub.u[1],
                                   span * sizeof(float), hipMemcpyDeviceToDevice, ctx->stream);
            if (e == hipSuccess && !lf && t % 2 == 1)
                e = stn::launch_copy_shell(FL.at(rec->buf, (size_t)q),
                                           static_cast<const float*>(g->u[0]), to_dims(g),
                                           kind_radius(kind), ctx->stream);
            if (e != hipSuccess) return dev_fail(e, "checkpoint copy");
            int rc = ensure_frontier_for(ctx, &sub);
            if (rc == STENCIL_OK)
                rc = ctx->scheme == STENCIL_NAIVE
                         ? run_naive(ctx, kind, &sub, c, steps)
                         : run_blocked(ctx, kind, &sub, c, steps, ctx->frontier);
            if (rc) return rc;
        }
    }
    rec->valid = true;
    rec->kind = kind;
    rec->sk = c->sk;
    rec->nx = g->nx; rec->ny = g->ny; rec->nz = g->nz; rec->halo = g->halo;
    rec->sy = g->sy; rec->sz = g->sz; rec->nt = nt; rec->every = k;
    rec->coef = c->arrays;
    rec->dtype = (int)c->dtype;
    return STENCIL_OK;
}

bool recording_matches(const stencil_ctx::recording& r, int kind, const stencil_grid* g,
                       const stencil_coeffs* c, int64_t nt) {
    return r.valid && r.kind == kind && r.sk == c->sk && r.nx == g->nx && r.ny == g->ny &&
           r.nz == g->nz && r.halo == g->halo && r.sy == g->sy && r.sz == g->sz && r.nt == nt && r.coef == c->arrays &&
           r.dtype == (int)c->dtype;
}

int default_ckpt(int64_t nt) {
    const int k = (int)std::lround(std::sqrt((double)nt));
    return k < 1 ? 1 : k;
}

// Reverse time stepping of kind 5 from the recorded checkpoints: segments in
// reverse order; each restores (u_{a-1}, u_a), recomputes u_{a+1} .. u_{b-1}
// with the naive step (bit-identical to the forward), then runs the reverse
// steps s = b-1 .. a.
int run_adjoint(stencil_ctx* ctx, const stencil_grid* g, const stencil_coeffs* c, int64_t nt,
                const float* seed, float* g_u0, float* g_um1, double* g_c) {
    const stn::dims d = to_dims(g);
    const hipStream_t st = ctx->stream;
    const bool bf16 = c->dtype == STENCIL_BF16;
    hipError_t e;
    if (nt == 0) {
        e = stn::launch_scale_copy(g_u0, seed, 1.0f, d, st);
        if (e == hipSuccess) e = stn::launch_zero_f32(g_um1, d, st);
        if (e == hipSuccess) e = stn::launch_zero_f64(g_c, d, st);
        return e == hipSuccess ? STENCIL_OK : dev_fail(e, "adjoint (nt = 0)");
    }
    stencil_ctx::recording& rec = ctx->rec;
    const field_layout FL = layout_of(g);
    const size_t span = FL.span;
    int rc;
    if (!recording_matches(rec, 5, g, c, nt)) {
        // no usable recording: rerun the forward from the initial state held by
        // the caller's buffers, on workspace copies
        void* p = nullptr;
        rc = ws_alloc(ctx, FL.bytes(2), &p);
        if (rc) return rc;
        float* w0 = FL.at(p, 0);
        float* w1 = FL.at(p, 1);
        e = hipMemcpyAsync(w0, g->u[0], span * sizeof(float), hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(w1, g->u[1], span * sizeof(float), hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return dev_fail(e, "adjoint forward copy");
        stencil_grid wg = *g;
        wg.u[0] = w0;
        wg.u[1] = w1;
        const int k = ctx->tuning.ckpt_every > 0 ? ctx->tuning.ckpt_every : default_ckpt(nt);
        rc = run_recorded(ctx, 5, &wg, c, nt, k, &rec);
        // the recording describes the caller's grid (same sizes and strides)
        e = hipStreamSynchronize(st);
        ws_free(ctx, p);
        if (rc) return rc;
        if (e != hipSuccess) return dev_fail(e, "adjoint forward");
    }
    const int k = rec.every;
    // workspace: segment slots for levels a+1 .. a+k-1 (levels a-1 and a are
    // read from the checkpoint itself), two adjoint fields and a flag
    void* p = nullptr;
    const size_t nslot = (size_t)(k > 1 ? k - 1 : 0);
    rc = ws_alloc(ctx, FL.bytes(nslot + 3), &p);
    if (rc) return rc;
    float* lam_a = FL.at(p, nslot);
    float* lam_b = FL.at(p, nslot + 1);
    int* flag = reinterpret_cast<int*>(FL.at(p, nslot + 2));
    const float* seg0 = nullptr;  // checkpoint of the current segment: u_{a-1}, u_a
    const float* seg1 = nullptr;
    auto slot = [&](int i) -> float* {
        if (i == 0) return const_cast<float*>(seg0);
        if (i == 1) return const_cast<float*>(seg1);
        return FL.at(p, (size_t)(i - 2));
    };
    auto done = [&](hipError_t err, const char* what) {
        const hipError_t es = hipStreamSynchronize(st);
        ws_free(ctx, p);
        if (err == hipSuccess) err = es;
        return err == hipSuccess ? STENCIL_OK : dev_fail(err, what);
    };
    // Scaled form (mu = c lambda) unless some coefficient is zero, tiny or
    // not finite there.
    int bad = 0;
    e = stn::launch_coef_check(flag, bf16, c->arrays, d, st);
    if (e == hipSuccess) e = hipMemcpyAsync(&bad, flag, sizeof(int), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return done(e, "adjoint coefficient check");
    const bool mu = bad == 0;
    // the boundary shell is taken as time independent: every slot gets the
    // stencil-deep shell of the buffer holding level 0 (its interior is
    // written by the recomputation before it is read)
    for (size_t i = 0; i < nslot && e == hipSuccess; ++i)
        e = stn::launch_copy_shell(FL.at(p, i), static_cast<const float*>(g->u[1]), d,
                                   kind_radius(5), st);
    if (e == hipSuccess) e = stn::launch_zero_span(lam_a, span, st);
    if (e == hipSuccess) e = stn::launch_zero_span(lam_b, span, st);
    if (e == hipSuccess)
        e = mu ? stn::launch_mul_coef(lam_a, seed, bf16, c->arrays, d, st)
               : stn::launch_scale_copy(lam_a, seed, 1.0f, d, st);
    if (e == hipSuccess) e = stn::launch_zero_f64(g_c, d, st);
    if (e != hipSuccess) return done(e, "adjoint setup");
    float* cur = lam_a;  // lambda_{m+1} (or mu_{m+1})
    float* nxt = lam_b;  // lambda_{m+2}, becomes lambda_m
    const stn::host_weights wt = to_weights(c);
    const double* w = c->w;
    // one reverse step m; up/uc/un: u_{m+1}, u_m, u_{m-1} for its gradient terms
    auto step = [&](const float* up, const float* uc, const float* un) {
        hipError_t r;
        if (mu && !up && !uc && !un)
            r = stn::launch_naive_step(5, bf16, cur, nxt, nxt, c->arrays, c->sk, d, wt, 0, st);
        else
            r = stn::launch_adjoint_step(bf16, mu, cur, nxt, c->arrays, up, uc, un, g_c, d, w, 0,
                                         st);
        std::swap(cur, nxt);
        return r;
    };
    // k = 1: every level is recorded (field i = u_{i-1}), so the whole run is
    // one segment and nothing is recomputed
    const bool all = k == 1;
    for (int q = all ? 0 : rec.n - 1; q >= 0 && e == hipSuccess; --q) {
        const int64_t a = all ? 0 : (int64_t)q * k;
        const int64_t b = all ? nt : std::min<int64_t>(a + k, nt);
        if (!all) {
            seg0 = rec.field(2 * (size_t)q);
            seg1 = rec.field(2 * (size_t)q + 1);
        }
        // slot i holds u_{a-1+i}
        for (int64_t i = 1; !all && i + a < b && e == hipSuccess; ++i)
            e = stn::launch_naive_step(5, bf16, slot((int)i), slot((int)i - 1), slot((int)i + 1),
                                       c->arrays, c->sk, d, wt, 0, st);
        // reverse steps b-1 .. a in groups of three: the middle step of a
        // group also adds the gradient terms of its two neighbours, so the
        // FP64 gradient is read and written once per group
        auto U = [&](int64_t n) -> const float* {
            return all ? rec.field((size_t)(n + 1)) : slot((int)(n - a + 1));
        };
        for (int64_t s = b - 1; s >= a && e == hipSuccess;) {
            const int64_t left = s - a + 1;
            if (left >= 3) {
                e = step(nullptr, nullptr, nullptr);
                if (e == hipSuccess) e = step(U(s), U(s - 1), U(s - 2));
                if (e == hipSuccess) e = step(nullptr, nullptr, nullptr);
                s -= 3;
            } else if (left == 2) {
                e = step(nullptr, nullptr, nullptr);
                if (e == hipSuccess) e = step(U(s), U(s - 1), nullptr);
                s -= 2;
            } else {
                e = step(nullptr, U(s), nullptr);
                s -= 1;
            }
        }
    }
    if (e == hipSuccess) {
        if (mu) {
            e = stn::launch_finish_mu(g_c, g_u0, g_um1, cur, nxt, bf16, c->arrays, d, st);
        } else {
            e = stn::launch_scale_copy(g_u0, cur, 1.0f, d, st);
            if (e == hipSuccess) e = stn::launch_scale_copy(g_um1, nxt, -1.0f, d, st);
        }
    }
    return done(e, "adjoint");
}

// Reverse time stepping of the Jacobi kinds 2 and 3 (lambda_t = A^T
// lambda_{t+1}, lambda_nt = seed) from the recorded checkpoints u_{qk}:
// segments in reverse order; each recomputes u_{a+1} .. u_{b-1} from its
// checkpoint with the naive step (bit-identical to the forward), runs the
// reverse steps b-1 .. a into a ring of k + 1 lambda fields, and then adds
// the gradient terms of the segment's steps in groups of up to
// stn::grad_group_max(kind) steps per pass over the FP64 arrays.
int run_adjoint_jacobi(stencil_ctx* ctx, int kind, const stencil_grid* g,
                       const stencil_coeffs* c, int64_t nt, const float* seed, float* g_u0,
                       double* g_c) {
    const stn::dims d = to_dims(g);
    const hipStream_t st = ctx->stream;
    const bool bf16 = c->dtype == STENCIL_BF16;
    const int K = kind_ncoef(kind);
    hipError_t e = stn::launch_scale_copy(g_u0, seed, 1.0f, d, st);
    for (int k = 0; k < K && e == hipSuccess; ++k) e = stn::launch_zero_f64(g_c + k * c->sk, d, st);
    if (e != hipSuccess) return dev_fail(e, "adjoint setup");
    if (nt == 0) return STENCIL_OK;
    stencil_ctx::recording& rec = ctx->rec;
    const field_layout FL = layout_of(g);
    const size_t span = FL.span;
    int rc;
    if (!recording_matches(rec, kind, g, c, nt)) {
        // no usable recording: rerun the forward from the initial state u[0]
        // on workspace copies (both with the level-0 shell)
        void* p = nullptr;
        rc = ws_alloc(ctx, FL.bytes(2), &p);
        if (rc) return rc;
        float* w0 = FL.at(p, 0);
        float* w1 = FL.at(p, 1);
        e = hipMemcpyAsync(w0, g->u[0], span * sizeof(float), hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(w1, g->u[0], span * sizeof(float), hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) {
            (void)hipStreamSynchronize(st);
            ws_free(ctx, p);
            return dev_fail(e, "adjoint forward copy");
        }
        stencil_grid wg = *g;
        wg.u[0] = w0;
        wg.u[1] = w1;
        const int k = ctx->tuning.ckpt_every > 0 ? ctx->tuning.ckpt_every : default_ckpt(nt);
        rc = run_recorded(ctx, kind, &wg, c, nt, k, &rec);
        e = hipStreamSynchronize(st);
        ws_free(ctx, p);
        if (rc) return rc;
        if (e != hipSuccess) return dev_fail(e, "adjoint forward");
    }
    const int k = rec.every;
    const int gmax = stn::grad_group_max(kind);
    // workspace: k - 1 state slots (u_{a+1} .. u_{a+k-1}; u_a is the
    // checkpoint itself), a ring of lambda fields (the one being computed and
    // those the pending gradient group still reads), and for kind 2 the seven
    // transposed coefficient arrays
    const size_t nslot = (size_t)(k - 1), nlam = (size_t)std::max(k, gmax) + 1;
    void* p = nullptr;
    rc = ws_alloc(ctx, FL.bytes(nslot + nlam), &p);
    if (rc) return rc;
    void* pc = nullptr;
    const size_t csize = bf16 ? sizeof(uint16_t) : sizeof(float);
    if (kind == 2) {
        rc = ws_alloc(ctx, (FL.lead + 7 * FL.stride) * csize + 256, &pc);
        if (rc) {
            ws_free(ctx, p);
            return rc;
        }
    }
    auto done = [&](hipError_t err, const char* what) {
        const hipError_t es = hipStreamSynchronize(st);
        ws_free(ctx, p);
        if (pc) ws_free(ctx, pc);
        if (err == hipSuccess) err = es;
        return err == hipSuccess ? STENCIL_OK : dev_fail(err, what);
    };
    void* coefT = pc ? static_cast<char*>(pc) + FL.lead * csize : nullptr;
    std::vector<float*> lam(nlam);
    for (size_t i = 0; i < nlam; ++i) lam[i] = FL.at(p, nslot + i);
    // state slots carry the stencil-deep level-0 shell (their interiors are
    // recomputed before they are read); lambda fields a zero shell
    for (size_t i = 0; i < nslot && e == hipSuccess; ++i)
        e = stn::launch_copy_shell(FL.at(p, i), static_cast<const float*>(g->u[0]), d,
                                   kind_radius(kind), st);
    for (size_t i = 0; i < nlam && e == hipSuccess; ++i) e = stn::launch_zero_span(lam[i], span, st);
    // lambda_s lives in lam[(nt - s) % nlam]
    auto lam_at = [&](int64_t s) { return lam[(size_t)((nt - s) % (int64_t)nlam)]; };
    if (e == hipSuccess) e = stn::launch_scale_copy(lam_at(nt), seed, 1.0f, d, st);
    if (e == hipSuccess && kind == 2)
        e = stn::launch_transpose7(coefT, (int64_t)FL.stride, c->arrays, c->sk, bf16, d, st);
    if (e != hipSuccess) return done(e, "adjoint setup");
    const stn::host_weights wt = to_weights(c);
    // pending gradient group: (u_s, lambda_{s+1}) for the most recent steps;
    // it is flushed when full and, when the states are segment slots that the
    // next segment overwrites (k > 1), at the end of every segment
    std::vector<const float*> PU, PL, U(k);
    auto flush = [&]() {
        hipError_t r = hipSuccess;
        if (!PU.empty())
            r = stn::launch_jacobi_grad(kind, (int)PU.size(), PU.data(), PL.data(), g_c, c->sk, d,
                                        0, st);
        PU.clear();
        PL.clear();
        return r;
    };
    for (int q = rec.n - 1; q >= 0 && e == hipSuccess; --q) {
        const int64_t a = (int64_t)q * k;
        const int m = (int)(std::min<int64_t>(a + k, nt) - a);
        // U[i] = u_{a+i}: the checkpoint, then the recomputed slots
        U[0] = rec.field((size_t)q);
        for (int i = 1; i < m; ++i) U[i] = FL.at(p, (size_t)(i - 1));
        for (int i = 1; i < m && e == hipSuccess; ++i)
            e = stn::launch_naive_step(kind, bf16, U[i - 1], nullptr, const_cast<float*>(U[i]),
                                       c->arrays, c->sk, d, wt, 0, st);
        for (int64_t s = a + m - 1; s >= a && e == hipSuccess; --s) {
            e = kind == 2 ? stn::launch_naive_step(2, bf16, lam_at(s + 1), nullptr, lam_at(s),
                                                   coefT, (int64_t)FL.stride, d, wt, 0, st)
                          : stn::launch_adj25_step(bf16, lam_at(s + 1), lam_at(s), c->arrays,
                                                   c->sk, d, 0, st);
            PU.push_back(U[s - a]);
            PL.push_back(lam_at(s + 1));
            if (e == hipSuccess && (int)PU.size() == gmax) e = flush();
        }
        if (e == hipSuccess && k > 1) e = flush();
    }
    if (e == hipSuccess) e = flush();
    if (e == hipSuccess) e = stn::launch_scale_copy(g_u0, lam_at(0), 1.0f, d, st);
    return done(e, "adjoint");
}

}  // namespace

extern "C" {

const char* stencil_last_error(void) { return g_err.c_str(); }

int stencil_create(stencil_ctx** out, stencil_scheme scheme, const stencil_tuning* tuning,
                   void* hip_stream) {
    if (!out) return fail(STENCIL_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (scheme != STENCIL_NAIVE && scheme != STENCIL_BLOCKED)
        return fail(STENCIL_ERR_INVALID, "unknown scheme %d", (int)scheme);
    stencil_tuning t{};
    if (tuning) t = *tuning;
    if (t.dw < 0 || t.zchunk < 0 || t.ckpt_every < 0 || t.workspace_limit < 0 || t.xtile < 0)
        return fail(STENCIL_ERR_INVALID, "negative tuning value");
    if (t.dw != 0 && (t.dw % 2 != 0 || t.dw < 4))
        return fail(STENCIL_ERR_INVALID, "dw=%d must be even and >= 4", t.dw);
    if (t.xtile != 0 && t.xtile != 16 && t.xtile != 32)
        return fail(STENCIL_ERR_INVALID, "xtile=%d must be 0, 16 or 32", t.xtile);
    stencil_ctx* ctx = new (std::nothrow) stencil_ctx();
    if (!ctx) return fail(STENCIL_ERR_NOMEM, "context allocation failed");
    ctx->scheme = scheme;
    ctx->tuning = t;
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    ctx->device = -1;  // bound at the first device call
    *out = ctx;
    return STENCIL_OK;
}

int stencil_run(stencil_ctx* ctx, stencil_kind kind, const stencil_grid* grid,
                const stencil_coeffs* coeffs, int64_t nt, int* result_slot) {
    if (!ctx) return fail(STENCIL_ERR_INVALID, "ctx is NULL");
    const int k = (int)kind;
    if (k < 1 || k > 5) return fail(STENCIL_ERR_INVALID, "unknown stencil kind %d", k);
    int rc = validate_grid(k, grid);
    if (rc) return rc;
    rc = validate_coeffs(k, grid, coeffs);
    if (rc) return rc;
    if (nt < 0) return fail(STENCIL_ERR_INVALID, "nt=%lld is negative", (long long)nt);
    if (ctx->scheme == STENCIL_BLOCKED && ctx->tuning.dw != 0 &&
        ctx->tuning.dw % (2 * kind_radius(k)) != 0)
        return fail(STENCIL_ERR_INVALID, "dw=%d is not a multiple of 2R=%d", ctx->tuning.dw,
                    2 * kind_radius(k));
    if (ctx->tuning.ckpt_every > 0 && k != 2 && k != 3 && k != 5)
        return fail(STENCIL_ERR_UNSUPPORTED,
                    "checkpoint recording is provided for kinds 2, 3 and 5 (those with an adjoint)");
    const int slot = kind_leapfrog(k) ? (int)((nt + 1) % 2) : (int)(nt % 2);
    if (nt == 0 || empty(grid)) {
        if (result_slot) *result_slot = slot;
        return STENCIL_OK;
    }
    if (ctx->scheme == STENCIL_BLOCKED) {
        rc = check_blocked(ctx, k, grid, coeffs);
        if (rc) return rc;
    }
    rc = set_device(ctx);
    if (rc) return rc;
    if (ctx->tuning.ckpt_every > 0) {
        rc = run_recorded(ctx, k, grid, coeffs, nt, ctx->tuning.ckpt_every, &ctx->rec);
    } else if (ctx->scheme == STENCIL_NAIVE) {
        rc = run_naive(ctx, k, grid, coeffs, nt);
    } else {
        rc = ensure_frontier_for(ctx, grid);
        if (rc == STENCIL_OK) rc = run_blocked(ctx, k, grid, coeffs, nt, ctx->frontier);
    }
    if (rc) return rc;
    if (result_slot) *result_slot = slot;
    return STENCIL_OK;
}

int stencil_run_noalloc(stencil_ctx* ctx, stencil_kind kind, const stencil_grid* grid,
                        const stencil_coeffs* coeffs, int64_t nt, int* result_slot) {
    if (!ctx) return fail(STENCIL_ERR_INVALID, "ctx is NULL");
    const int k = (int)kind;
    if (k < 1 || k > 5) return fail(STENCIL_ERR_INVALID, "unknown stencil kind %d", k);
    int rc = validate_grid(k, grid);
    if (rc) return rc;
    rc = validate_coeffs(k, grid, coeffs);
    if (rc) return rc;
    if (nt < 0) return fail(STENCIL_ERR_INVALID, "nt=%lld is negative", (long long)nt);
    if (ctx->scheme != STENCIL_BLOCKED)
        return fail(STENCIL_ERR_UNSUPPORTED,
                    "stencil_run_noalloc runs the blocked scheme (the naive one allocates "
                    "nothing: use stencil_run)");
    if (ctx->tuning.dw != 0 && ctx->tuning.dw % (2 * kind_radius(k)) != 0)
        return fail(STENCIL_ERR_INVALID, "dw=%d is not a multiple of 2R=%d", ctx->tuning.dw,
                    2 * kind_radius(k));
    if (ctx->tuning.ckpt_every > 0)
        return fail(STENCIL_ERR_UNSUPPORTED,
                    "stencil_run_noalloc does not record checkpoints (ckpt_every must be 0)");
    const int slot = kind_leapfrog(k) ? (int)((nt + 1) % 2) : (int)(nt % 2);
    if (nt == 0 || empty(grid)) {
        if (result_slot) *result_slot = slot;
        return STENCIL_OK;
    }
    rc = check_blocked(ctx, k, grid, coeffs);
    if (rc) return rc;
    const size_t need = layout_of(grid).bytes(2);
    if (need > stn::kScratchBytes)
        return fail(STENCIL_ERR_UNSUPPORTED,
                    "stencil_run_noalloc: the grid needs %zu bytes of frontier storage; the "
                    "library's scratch holds %zu (two fields of at most about %zu elements)",
                    need, stn::kScratchBytes, (stn::kScratchBytes - 256) / 8);
    rc = set_device(ctx);
    if (rc) return rc;
    void* scratch = nullptr;
    hipError_t e = stn::blocked_scratch(&scratch);
    if (e != hipSuccess) return dev_fail(e, "hipGetSymbolAddress(scratch)");
    const size_t fpair = (need + 255) / 256 * 256;
    rc = run_blocked(ctx, k, grid, coeffs, nt, scratch, static_cast<char*>(scratch) + fpair,
                     stn::kScratchBytes - fpair);
    if (rc) return rc;
    if (result_slot) *result_slot = slot;
    return STENCIL_OK;
}

int stencil_adjoint(stencil_ctx* ctx, stencil_kind kind, const stencil_grid* grid,
                    const stencil_coeffs* coeffs, int64_t nt, const float* seed, float* grad_u0,
                    float* grad_um1, double* grad_c) {
    if (!ctx) return fail(STENCIL_ERR_INVALID, "ctx is NULL");
    const int k = (int)kind;
    if (k != 2 && k != 3 && k != 5)
        return fail(STENCIL_ERR_UNSUPPORTED,
                    "the adjoint is provided for kinds 2, 3 (Jacobi, variable coefficients) and 5");
    int rc = validate_grid(k, grid);
    if (rc) return rc;
    rc = validate_coeffs(k, grid, coeffs);
    if (rc) return rc;
    if (nt < 0) return fail(STENCIL_ERR_INVALID, "nt=%lld is negative", (long long)nt);
    if (!seed || !grad_u0 || !grad_c)
        return fail(STENCIL_ERR_INVALID, "adjoint field pointer is NULL");
    if (k == 5 && !grad_um1) return fail(STENCIL_ERR_INVALID, "grad_um1 is NULL");
    if (k != 5 && grad_um1)
        return fail(STENCIL_ERR_INVALID, "grad_um1 must be NULL for the Jacobi kinds (one initial level)");
    if (empty(grid)) return STENCIL_OK;
    if (ctx->scheme == STENCIL_BLOCKED) {
        // a missing recording is rebuilt with the context's (blocked) forward
        rc = check_blocked(ctx, k, grid, coeffs);
        if (rc) return rc;
    }
    rc = set_device(ctx);
    if (rc) return rc;
    if (k != 5) return run_adjoint_jacobi(ctx, k, grid, coeffs, nt, seed, grad_u0, grad_c);
    return run_adjoint(ctx, grid, coeffs, nt, seed, grad_u0, grad_um1, grad_c);
}

int stencil_sync(stencil_ctx* ctx) {
    if (!ctx) return fail(STENCIL_ERR_INVALID, "ctx is NULL");
    if (ctx->device < 0) return STENCIL_OK;  // nothing was ever launched
    int rc = set_device(ctx);
    if (rc) return rc;
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return dev_fail(e, "hipStreamSynchronize");
    if (ctx->err_dev) {
        // a halo of the radius-4 blocked scheme that never arrived
        int flag = 0;
        e = hipMemcpy(&flag, ctx->err_dev, sizeof flag, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return dev_fail(e, "error flag read");
        if (flag) {
            const int zero = 0;
            (void)hipMemcpy(ctx->err_dev, &zero, sizeof zero, hipMemcpyHostToDevice);
            return fail(STENCIL_ERR_DEVICE,
                        "blocked scheme: a workgroup waited in vain for a neighbour's halo; the "
                        "results of the run are invalid");
        }
    }
    return STENCIL_OK;
}

void stencil_destroy(stencil_ctx* ctx) {
    if (!ctx) return;
    if (ctx->device >= 0 && hipSetDevice(ctx->device) == hipSuccess) {
        (void)hipStreamSynchronize(ctx->stream);
        for (auto& b : ctx->bufs) (void)hipFree(b.first);
    }
    delete ctx;
}

int32_t stencil_default_dw(stencil_kind kind, int32_t nx, int32_t ny, int32_t nz,
                           stencil_dtype coef_dtype) {
    const int k = (int)kind;
    if (k < 1 || k > 5) {
        fail(STENCIL_ERR_INVALID, "unknown stencil kind %d", k);
        return 0;
    }
    if (nx < 0 || ny < 0 || nz < 0 || (coef_dtype != STENCIL_F32 && coef_dtype != STENCIL_BF16)) {
        fail(STENCIL_ERR_INVALID, "bad grid size or coefficient storage");
        return 0;
    }
    return stn::blocked_default_dw(k, (int64_t)nx * ny * nz, coef_dtype == STENCIL_BF16);
}

int32_t stencil_blocked_slices(stencil_kind kind, int32_t dw, int32_t xtile, int32_t nx) {
    const int k = (int)kind;
    if (k < 1 || k > 5 || nx < 1) return 0;
    if (kind_radius(k) != 4) return 1;  // one workgroup per diamond and x-tile
    if (dw == 0) dw = stn::blocked_default_dw(k, 0, false);  // radius 4: independent of both
    return stn::mwd_slices(k, dw, xtile, nx);
}

int stencil_plan_rows(stencil_kind kind, int32_t dw, int32_t ny, int64_t nt, int64_t* out,
                      int32_t cap) {
    const int k = (int)kind;
    if (k < 1 || k > 5 || ny < 0 || nt < 0 || cap < 0 || (cap > 0 && !out)) return -1;
    const int R = kind_radius(k);
    if (dw % (2 * R) != 0 || dw < 4 * R) return -1;
    stn::diamond_plan p = stn::make_plan(R, dw, ny, nt);
    const int n = (int)p.rows.size();
    for (int i = 0; i < n && i < cap; ++i) {
        out[4 * i + 0] = p.rows[i].r;
        out[4 * i + 1] = p.rows[i].t0;
        out[4 * i + 2] = p.rows[i].n_diamonds;
        out[4 * i + 3] = p.rows[i].first_centre;
    }
    return n;
}

}  // extern "C"
