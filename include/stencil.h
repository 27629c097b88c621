/*
 * stencil.h -- C ABI of the MI355X stencil library (libstencil.so).
 *
 * Repeated time-stepped updates of 3D star stencils on Cartesian lattices,
 * after Malas et al., "Multicore-optimized wavefront diamond blocking for
 * optimizing stencil updates" (arXiv 1410.3060):
 *   - the five operators of Fig. 1b-1e (Sect. 3.1),
 *   - a one-sweep-per-step scheme ("naive", Sect. 4.1),
 *   - a temporally blocked scheme: diamond tiles along y with a wavefront
 *     along z (Sect. 4.2-4.3 and 5.1),
 *   - the adjoints (reverse time stepping) of the variable-coefficient
 *     Jacobi stencils of Fig. 1c and 1d and of the leapfrog with c(x), which
 *     the paper does not treat: the transposes of those recurrences.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Memory.  Every array argument is a DEVICE pointer owned by the caller, who
 *   keeps it alive until stencil_sync() returns.  The library owns only its
 *   context and the workspace inside it.
 * Layout (Sect. 3.1: x is the leading dimension, then y, then z).  A field is
 *   a padded box with a boundary shell of width `halo` on all six faces.  The
 *   pointer addresses the padded origin (x, y, z) = (-halo, -halo, -halo);
 *   interior point (x, y, z), 0 <= x < nx etc., is element
 *       (z + halo) * sz + (y + halo) * sy + (x + halo).
 *   x stride is 1; sy >= nx + 2*halo; sz >= sy * (ny + 2*halo).  All fields of
 *   one call (both time levels, every coefficient array, adjoint inputs and
 *   outputs) share these element strides.
 * Boundary.  The shell is a time-independent Dirichlet boundary: every level
 *   reads the shell of the buffer that holds level 0 (u[0] for kinds 1-3,
 *   u[1] for kinds 4-5).  Both schemes copy the R-deep level-0 shell into the
 *   other buffer before the first step (nt >= 1), so they agree bit for bit
 *   whatever shells the two buffers carried on entry.
 * Two-buffer time storage (Sect. 3.1: only two levels are stored and level
 *   t+1 overwrites level t-1).  Jacobi kinds (1-3): u[0] holds level 0 on
 *   entry and level t lives in u[t % 2].  Leapfrog kinds (4-5): u[0] holds
 *   u_{-1}, u[1] holds u_0 and level n lives in u[(n + 1) % 2].
 * Precision.  Lattice values are FP32.  Coefficient arrays are FP32 or BF16
 *   (expanded exactly to FP32 in the kernels); arithmetic is FP32 with one
 *   fixed fused-multiply-add order per kind, the same in every scheme, so the
 *   blocked scheme reproduces the naive scheme bit for bit.  FP64 is used only
 *   for the coefficient gradient of stencil_adjoint().  BF16 arrays may start
 *   on any 2-byte boundary.  Arrays on 4-byte boundaries, with even sk and sz,
 *   are read faster by the blocked scheme for kinds 3 and 5, with the same
 *   results.
 * Streams.  Calls are asynchronous on the HIP stream given to stencil_create()
 *   (borrowed, not owned).  Device faults surface at the next stencil_sync().
 * Errors.  Every argument is validated on the host before any HIP call.  A
 *   non-zero return leaves caller memory untouched (except after
 *   STENCIL_ERR_DEVICE) and sets a thread-local message, read with
 *   stencil_last_error().
 */
#ifndef STENCIL_H
#define STENCIL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    STENCIL_OK = 0,
    STENCIL_ERR_INVALID = 1,     /* bad argument */
    STENCIL_ERR_UNSUPPORTED = 2, /* valid but not provided (e.g. BF16 with a constant kind) */
    STENCIL_ERR_NOMEM = 3,       /* workspace over the tuning limit or allocation failure */
    STENCIL_ERR_DEVICE = 4       /* HIP runtime error; message from hipGetErrorString */
};

/* Stencil operators (Fig. 1 of the paper). */
typedef enum {
    /* Fig. 1b, R = 1: u' = w[0]*u + w[1]*(sum of the six face neighbours). */
    STENCIL_7PT_CONST = 1,
    /* Fig. 1c, R = 1, K = 7 arrays: u' = sum_k W_k * u(nbr_k), neighbour order
       centre, x-1, x+1, y-1, y+1, z-1, z+1. */
    STENCIL_7PT_VAR = 2,
    /* Fig. 1d, R = 4, K = 13 arrays: u' = W_0*u + sum_{r=1..4}
       [W_{3r-2}*(x pair at r) + W_{3r-1}*(y pair) + W_{3r}*(z pair)]. */
    STENCIL_25PT_VAR = 3,
    /* Fig. 1e with scalar alpha (coeffs.alpha), R = 4:
       u_{n+1} = 2 u_n - u_{n-1} + alpha * L8(u_n),
       L8(u) = w[0]*u + sum_{r=1..4} w[r]*(x pair + y pair + z pair at r),
       evaluated in FP32 as (w[0] + 6 sum_r w[r])*u + sum_r w[r]*(pairs - 6u)
       (the same operator; its row sum stays zero after the weights are
       rounded to FP32). */
    STENCIL_25PT_WAVE = 4,
    /* Fig. 1e with alpha a domain-sized array (K = 1), e.g. c(x) of the wave
       equation. */
    STENCIL_25PT_WAVE_VARC = 5
} stencil_kind;

typedef enum {
    STENCIL_NAIVE = 0,  /* one full sweep per time step (Sect. 4.1) */
    STENCIL_BLOCKED = 1 /* diamond tiles in y, wavefront in z (Sect. 4.2, 4.3, 5.1); a
                           workgroup addresses its z-chunk with 32-bit byte offsets from a
                           base of its own, so fields of any size work while a window of
                           2R(L+1) + 2 planes (L = 2 dw / (2R) - 1) stays below 2 GiB, else
                           STENCIL_ERR_UNSUPPORTED; z-chunks are capped to fit */
} stencil_scheme;

typedef enum { STENCIL_F32 = 0, STENCIL_BF16 = 1 } stencil_dtype;

typedef struct {
    int32_t nx, ny, nz; /* interior sizes, each >= 0 (0 makes every call a no-op) */
    int32_t halo;       /* boundary width, >= R of the kind (1 or 4) */
    int64_t sy, sz;     /* element strides (see layout above) */
    void* u[2];         /* FP32 fields, distinct, see the two-buffer convention */
} stencil_grid;

typedef struct {
    stencil_dtype dtype; /* storage of `arrays`; BF16 only for kinds 2, 3, 5 */
    const void* arrays;  /* K arrays for kinds 2 (K=7), 3 (K=13), 5 (K=1); unused otherwise */
    int64_t sk;          /* element stride between arrays, >= sz * (nz + 2*halo) */
    double w[5];         /* kind 1: w[0] centre, w[1] neighbour; kinds 4-5: L8 weights */
    double alpha;        /* kind 4 */
} stencil_coeffs;

typedef struct {
    int32_t dw;          /* diamond width in y for STENCIL_BLOCKED: a multiple of 2R with
                            dw >= 4R; provided: 4..12 for R = 1, 16 and 24 for kind 3,
                            16, 24 and 32 for kinds 4-5 (others return
                            STENCIL_ERR_UNSUPPORTED); 0 = the library's choice,
                            stencil_default_dw() (6 for R = 1, but 10 for kind 2 on
                            grids of at least 256^3 points with FP32 coefficients and
                            300^3 with BF16 ones; 16, 32, 16 for kinds 3, 4, 5) */
    int32_t xtile;       /* x columns per workgroup of the radius-4 blocked scheme: 16 or
                            32 (32 not at dw 24 of kind 3); each diamond is then shared by
                            ceil(nx / xtile) cooperating workgroups (Sect. 5.1, thread
                            groups); 0 = the library's choice (32, or 16 at dw 24 of
                            kind 3); other values are STENCIL_ERR_INVALID; ignored by
                            the naive scheme and the radius-1 blocked kernel */
    int32_t zchunk;      /* planes per z-chunk of one workgroup (parallelism along z);
                            0 = the library's choice */
    int32_t ckpt_every;  /* checkpoint interval k recorded by stencil_run() for the kinds
                            with an adjoint (2, 3, 5); 0 = no recording; 1 = every
                            level (no recomputation in the adjoint, nt + 1 fields) */
    int64_t workspace_limit; /* bytes the context may allocate; 0 = no limit */
} stencil_tuning;

typedef struct stencil_ctx stencil_ctx;

/* Create a context for one scheme.  `tuning` may be NULL (all zero).
   `hip_stream` is a hipStream_t (NULL = the null stream), borrowed.  No HIP
   call is made here: the context binds to the device that is current at its
   first device call (stencil_run / stencil_adjoint with work to do). */
int stencil_create(stencil_ctx** out, stencil_scheme scheme, const stencil_tuning* tuning,
                   void* hip_stream);

/* Advance `nt` >= 0 time steps in place (Fig. 1b-1e, two-buffer storage as
   above).  On return *result_slot (if not NULL) is the index of u[] that holds
   level nt: nt % 2 for kinds 1-3, (nt + 1) % 2 for kinds 4-5 (the other slot
   then holds u_{nt-1}).  nt = 0 is a no-op.  For kinds 2, 3 and 5 with
   ckpt_every = k > 0 the context records the state at n = 0, k, 2k, ... < nt
   (u_n; for kind 5 the pair (u_{n-1}, u_n)) for a later stencil_adjoint();
   the recording is replaced by the next recording run.  With k = 1 every
   level is recorded and the sweeps write straight into the recording (the
   naive sweep is used whatever the scheme); for kind 5 the buffer of u_{nt-1}
   then receives a copy of it with the level-0 shell, and for kinds 2-3 the
   buffer that does not hold level nt is left unspecified.
   Graphs: once the context has run the same sizes eagerly (its workspace then
   exists), a run without recording makes only kernel launches and
   device-to-device copies on the context's stream, so it can be captured
   into a HIP graph and replayed. */
int stencil_run(stencil_ctx* ctx, stencil_kind kind, const stencil_grid* grid,
                const stencil_coeffs* coeffs, int64_t nt, int* result_slot);

/* Allocation-free variant of stencil_run for the blocked scheme, for callers
   that cannot allocate device memory: code being captured into a HIP graph,
   tight serving loops, harnesses that forbid hipMalloc.  Same arguments,
   results (bit for bit) and result slot as stencil_run on a STENCIL_BLOCKED
   context; the context's scheme must be STENCIL_BLOCKED
   (STENCIL_ERR_UNSUPPORTED otherwise) and ckpt_every 0 (no recording).
   It calls no hipMalloc, hipFree or other allocating routine: the blocked
   scheme's second frontier pair lives in a static device array of the
   library, 128 MiB per GPU, held from the library's load until the process
   ends.  Grids whose two frontier fields (each spanning the padded field, at
   the caller's row alignment) need more than 128 MiB are rejected with
   STENCIL_ERR_UNSUPPORTED before any HIP call; that is about 16.7 M elements
   per field, e.g. 250^3 with halo 4.  Every call on a GPU uses that GPU's
   one array: calls that overlap in time on one GPU (other streams, other
   contexts, other threads) race and give wrong results; calls in one stream
   are ordered and safe.  The array keeps the previous call's contents; the
   scheme writes every value it reads before reading it. */
int stencil_run_noalloc(stencil_ctx* ctx, stencil_kind kind, const stencil_grid* grid,
                        const stencil_coeffs* coeffs, int64_t nt, int* result_slot);

/* Reverse time stepping (adjoint) for kinds 2, 3 and 5.

   Kinds 2 and 3 (Fig. 1c, 1d).  With A = A(W) the sweep operator on the
   interior (fixed shell), u_{t+1} = A u_t; for a loss with seed
   lambda_nt = dJ/du_nt the adjoint recurrence is lambda_t = A^T lambda_{t+1}
   and the outputs are
       grad_u0     = dJ/du_0 = lambda_0                                (FP32),
       grad_c + k*sk = dJ/dW_k = sum_{t=0}^{nt-1} lambda_{t+1} * tap_k(u_t)  (FP64),
   tap_k the value W_k multiplies in the update of Fig. 1c / 1d (u at the
   neighbour for kind 2, u(p) for W_0 and the pair sum at radius r for
   W_{3(r-1)+1+a} of kind 3), boundary shell values included.  grad_c holds
   K FP64 arrays at the coefficients' element stride sk; grad_um1 must be
   NULL.  BF16 coefficients are differentiated at their FP32 expansion.
   Without a matching recording grid->u[0] must hold u_0.

   Kind 5 (STENCIL_25PT_WAVE_VARC).  With
   M = 2I + diag(c) L8 the forward map is u_{n+1} = M u_n - u_{n-1}; for a
   loss with seed lambda_nt = dJ/du_nt the adjoint recurrence is
       lambda_n = 2 lambda_{n+1} - lambda_{n+2} + L8(c * lambda_{n+1}),
   lambda_{nt+1} = 0, and the outputs are
       grad_u0  = dJ/du_0    = lambda_0,
       grad_um1 = dJ/du_{-1} = -lambda_1,
       grad_c   = dJ/dc      = sum_{n=0}^{nt-1} lambda_{n+1} * L8(u_n)   (FP64).

   All kinds.  Forward states are rebuilt from the context's recording when
   it matches (same kind, sizes, strides, coefficient pointer and stride, and
   nt; made by stencil_run with ckpt_every > 0); otherwise grid->u[] must hold
   the INITIAL state (kind 5: u[0] = u_{-1}, u[1] = u_0) and the forward pass
   is recomputed with checkpoints first (ckpt_every, or about sqrt(nt) if 0).
   seed, grad_u0, grad_um1 are FP32 and grad_c FP64 padded fields with the
   grid's strides; only their interiors are read or written.  The gradients
   are overwritten (not accumulated).  Every level reads the boundary shell of
   the level-0 buffer.  The context allocates ~ (ckpt_every + 4) fields of
   workspace (kinds 2-3: ~ 2 ckpt_every + 9, plus 7 coefficient arrays for
   kind 2). */
int stencil_adjoint(stencil_ctx* ctx, stencil_kind kind, const stencil_grid* grid,
                    const stencil_coeffs* coeffs, int64_t nt, const float* seed,
                    float* grad_u0, float* grad_um1, double* grad_c);

/* Wait for all work of this context; reports asynchronous device errors. */
int stencil_sync(stencil_ctx* ctx);

/* Release the context and its workspace (waits for its stream first). */
void stencil_destroy(stencil_ctx* ctx);

/* Message of the last non-zero return on this thread ("" if none). */
const char* stencil_last_error(void);

/* Diamond geometry the blocked scheme uses for (kind, dw, ny, nt), for tests
   and tuning: fills up to `cap` rows of {row, t0, n_diamonds, first_centre}
   and returns the number of diamond rows, or -1 on a bad argument. */
int stencil_plan_rows(stencil_kind kind, int32_t dw, int32_t ny, int64_t nt, int64_t* out,
                      int32_t cap);

/* The diamond width the blocked scheme uses for `kind` when stencil_tuning.dw
   is 0 (Sect. 4.2: a multiple of 2R, at least 4R) on an nx x ny x nz grid with
   coefficients stored as `coef_dtype` (ignored by the kinds without arrays),
   chosen from measured rates (Sect. 5.3 models the same trade-off between the
   bytes a wider diamond saves and the block it has to hold); 0 for an unknown
   kind, a negative size or an unknown dtype (stencil_last_error says which).
   No HIP call. */
int32_t stencil_default_dw(stencil_kind kind, int32_t nx, int32_t ny, int32_t nz,
                           stencil_dtype coef_dtype);

/* Workgroups that share one diamond of the blocked scheme (the thread group
   of Sect. 5.1) for (kind, dw, xtile, nx) as stencil_tuning would set them (dw 0 and xtile 0 = the
   library's choices): ceil(nx / slice width) for the radius-4 kinds, 1 for
   the radius-1 kinds (one workgroup per diamond and x-tile), 0 for a
   combination that is not provided or a bad argument.  No HIP call. */
int32_t stencil_blocked_slices(stencil_kind kind, int32_t dw, int32_t xtile, int32_t nx);

#ifdef __cplusplus
}
#endif

#endif /* STENCIL_H */
