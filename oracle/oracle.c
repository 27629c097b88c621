/*
 * FP64 CPU oracle for time-stepped 3D star stencils.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: it exists so that tests, the smoke check and the CPU
 * baseline leg of the benchmark can compare the GPU library against a plain,
 * slow, obviously correct implementation of the paper's definitions.
 *
 * Paper: Malas, Hager, Ltaief, Stengel, Wellein, Keyes, "Multicore-optimized
 * wavefront diamond blocking for optimizing stencil updates" (arXiv 1410.3060).
 *
 * What it computes (Sect. 3.1, Fig. 1b-1e): nt Jacobi-style sweeps, one full
 * sweep per time step, each sweep reading only the previous level(s) and
 * writing a new one.  No temporal blocking, no tiling, no fusion: the
 * temporally blocked schemes of Sect. 4-5 reorder exactly these updates, so
 * their result is this result up to floating-point rounding order.
 *
 * Storage (Sect. 3.1): a field is [z][y][x] with x fastest.  Every array here
 * is a padded box of (nx+2h) x (ny+2h) x (nz+2h) doubles, contiguous; the
 * interior point (x,y,z), 0 <= x < nx etc., sits at padded (x+h, y+h, z+h).
 * The h-wide shell is the boundary: it is read by the stencil and never
 * written (fixed Dirichlet values, the same at every time level).
 *
 * Kinds (numbering is the oracle's own):
 *   1  7-point constant, Fig. 1b:  u' = w0*u + w1*(sum of the 6 face neighbours)
 *   2  7-point variable, Fig. 1c:  u' = sum_k W_k * u(nbr_k),
 *                                  nbr order: centre, x-1, x+1, y-1, y+1, z-1, z+1
 *   3  25-point variable axis-symmetric, Fig. 1d:
 *                                  u' = W_0*u + sum_{r=1..4} [ W_{3r-2}*(x-pair at r)
 *                                       + W_{3r-1}*(y-pair at r) + W_{3r}*(z-pair at r) ]
 *   4  25-point leapfrog, Fig. 1e, scalar alpha:
 *                                  u_{n+1} = 2 u_n - u_{n-1} + alpha * L8(u_n)
 *   5  same with alpha a domain-sized array (c(x) in the wave equation)
 *   where L8(u) = w0*u + sum_{r=1..4} w_r * (x-pair + y-pair + z-pair at r).
 *
 * The adjoint (reverse time stepping for kind 5) is not in the paper; its
 * definition is the transpose of the linear recurrence of Fig. 1e and is
 * written out above oracle_adjoint_wave_varc().
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fPIC -shared (no FMA contraction,
 * so every line below is evaluated exactly as written).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { OK_7C = 1, OK_7V = 2, OK_25V = 3, OK_WAVE = 4, OK_WAVE_VARC = 5 };

typedef struct {
    int64_t nx, ny, nz, h;  /* interior sizes and boundary width */
    int64_t px, py, pz;     /* padded sizes */
} box;

static box mkbox(int64_t nx, int64_t ny, int64_t nz, int64_t h) {
    box b = {nx, ny, nz, h, nx + 2 * h, ny + 2 * h, nz + 2 * h};
    return b;
}

/* linear index of interior coordinate (x, y, z); the boundary shell is at
 * coordinates -h..-1 and n..n+h-1 */
static inline int64_t at(const box* b, int64_t x, int64_t y, int64_t z) {
    return ((z + b->h) * b->py + (y + b->h)) * b->px + (x + b->h);
}

static int64_t box_size(const box* b) { return b->px * b->py * b->pz; }

static int radius_of(int kind) { return (kind == OK_7C || kind == OK_7V) ? 1 : 4; }

static int ncoef_of(int kind) {
    switch (kind) {
    case OK_7V: return 7;
    case OK_25V: return 13;
    case OK_WAVE_VARC: return 1;
    default: return 0;
    }
}

/* L8(u) at one point: w[0]*u + sum_r w[r]*(x-pair + y-pair + z-pair). */
static inline double lap8(const box* b, const double* u, const double* w,
                          int64_t x, int64_t y, int64_t z) {
    double s = w[0] * u[at(b, x, y, z)];
    for (int r = 1; r <= 4; ++r) {
        double xp = u[at(b, x - r, y, z)] + u[at(b, x + r, y, z)];
        double yp = u[at(b, x, y - r, z)] + u[at(b, x, y + r, z)];
        double zp = u[at(b, x, y, z - r)] + u[at(b, x, y, z + r)];
        s += w[r] * (xp + yp + zp);
    }
    return s;
}

/* One Jacobi sweep of kinds 1-3 (Fig. 1b, 1c, 1d): out <- A(in), interior only. */
static void sweep_jacobi(int kind, const box* b, const double* in, double* out,
                         const double* coef, const double* w) {
    const int64_t n = box_size(b);
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < b->nz; ++z) {
        for (int64_t y = 0; y < b->ny; ++y) {
            for (int64_t x = 0; x < b->nx; ++x) {
                const int64_t p = at(b, x, y, z);
                double v;
                if (kind == OK_7C) {
                    v = w[0] * in[p]
                      + w[1] * (in[at(b, x - 1, y, z)] + in[at(b, x + 1, y, z)])
                      + w[1] * (in[at(b, x, y - 1, z)] + in[at(b, x, y + 1, z)])
                      + w[1] * (in[at(b, x, y, z - 1)] + in[at(b, x, y, z + 1)]);
                } else if (kind == OK_7V) {
                    const double* W = coef;
                    v = W[0 * n + p] * in[p]
                      + W[1 * n + p] * in[at(b, x - 1, y, z)]
                      + W[2 * n + p] * in[at(b, x + 1, y, z)]
                      + W[3 * n + p] * in[at(b, x, y - 1, z)]
                      + W[4 * n + p] * in[at(b, x, y + 1, z)]
                      + W[5 * n + p] * in[at(b, x, y, z - 1)]
                      + W[6 * n + p] * in[at(b, x, y, z + 1)];
                } else { /* OK_25V */
                    const double* W = coef;
                    v = W[0 * n + p] * in[p];
                    for (int r = 1; r <= 4; ++r) {
                        const int64_t kx = 3 * (r - 1) + 1, ky = kx + 1, kz = kx + 2;
                        v += W[kx * n + p] * (in[at(b, x - r, y, z)] + in[at(b, x + r, y, z)]);
                        v += W[ky * n + p] * (in[at(b, x, y - r, z)] + in[at(b, x, y + r, z)]);
                        v += W[kz * n + p] * (in[at(b, x, y, z - r)] + in[at(b, x, y, z + r)]);
                    }
                }
                out[p] = v;
            }
        }
    }
}

/* One leapfrog step (Fig. 1e), in place on the older level:
 * prev <- 2*cur - prev + alpha * L8(cur).  Each point reads its own old value
 * of prev before writing it and no point reads prev at any other position, so
 * the in-place update is the two-level storage the paper describes. */
static void sweep_wave(int kind, const box* b, const double* cur, double* prev,
                       const double* alpha_arr, double alpha, const double* w) {
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < b->nz; ++z) {
        for (int64_t y = 0; y < b->ny; ++y) {
            for (int64_t x = 0; x < b->nx; ++x) {
                const int64_t p = at(b, x, y, z);
                const double a = (kind == OK_WAVE_VARC) ? alpha_arr[p] : alpha;
                prev[p] = 2.0 * cur[p] - prev[p] + a * lap8(b, cur, w, x, y, z);
            }
        }
    }
}

static void set_threads(int nthreads) {
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

/* Number of OpenMP threads a parallel region would use now. */
int oracle_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * Run nt time steps.
 *   kind 1-3: u holds level 0 on entry and level nt on return (u_prev unused).
 *   kind 4-5: (u_prev, u) hold (u_{-1}, u_0) on entry and (u_{nt-1}, u_nt) on
 *             return.
 *   coef: K padded fields back to back (K = 7, 13 or 1 for kinds 2, 3, 5).
 *   w: kind 1 uses w[0] (centre), w[1] (neighbour); kinds 4-5 use w[0..4].
 *   alpha: kind 4 only.
 *   seconds (optional): wall time of the time-step loop alone.
 * Returns 0, or -1 on a bad argument / allocation failure.
 */
int oracle_run(int kind, int64_t nx, int64_t ny, int64_t nz, int64_t h,
               double* u_prev, double* u, const double* coef, const double* w,
               double alpha, int64_t nt, int nthreads, double* seconds) {
    if (kind < OK_7C || kind > OK_WAVE_VARC || nx < 0 || ny < 0 || nz < 0 || nt < 0)
        return -1;
    if (h < radius_of(kind) || !u || !w) return -1;
    if (ncoef_of(kind) > 0 && !coef) return -1;
    if (kind >= OK_WAVE && !u_prev) return -1;
    set_threads(nthreads);
    box b = mkbox(nx, ny, nz, h);
    const int64_t n = box_size(&b);
    struct timespec t0, t1;

    if (kind <= OK_25V) {
        double* tmp = (double*)malloc((size_t)n * sizeof(double));
        if (!tmp) return -1;
        memcpy(tmp, u, (size_t)n * sizeof(double)); /* same boundary shell */
        double *cur = u, *nxt = tmp;
        clock_gettime(CLOCK_MONOTONIC, &t0);
        for (int64_t t = 0; t < nt; ++t) {
            sweep_jacobi(kind, &b, cur, nxt, coef, w);
            double* s = cur; cur = nxt; nxt = s;
        }
        clock_gettime(CLOCK_MONOTONIC, &t1);
        if (cur != u) memcpy(u, cur, (size_t)n * sizeof(double));
        free(tmp);
    } else {
        double *cur = u, *prev = u_prev;
        clock_gettime(CLOCK_MONOTONIC, &t0);
        for (int64_t t = 0; t < nt; ++t) {
            sweep_wave(kind, &b, cur, prev, coef, alpha, w);
            double* s = cur; cur = prev; prev = s; /* prev now holds u_{t+1} */
        }
        clock_gettime(CLOCK_MONOTONIC, &t1);
        if (cur != u) { /* odd nt: the two buffers hold the pair swapped */
            for (int64_t i = 0; i < n; ++i) {
                double s = u[i]; u[i] = u_prev[i]; u_prev[i] = s;
            }
        }
    }
    if (seconds)
        *seconds = (double)(t1.tv_sec - t0.tv_sec) + 1e-9 * (double)(t1.tv_nsec - t0.tv_nsec);
    return 0;
}

/*
 * Adjoint of kind 5 (reverse time stepping).
 *
 * Forward recurrence (Fig. 1e with alpha = c):  u_{n+1} = M u_n - u_{n-1},
 * M = 2I + diag(c) L, n = 0..nt-1, L the 25-point operator on the interior
 * with the boundary held fixed.  For a scalar loss J(u_nt) with seed
 * lambda_nt = dJ/du_nt, the reverse recurrence is
 *     lambda_n = M^T lambda_{n+1} - lambda_{n+2},   lambda_{nt+1} = 0,
 *     M^T      = 2I + L diag(c)        (L is symmetric on the interior),
 * and the gradients are
 *     dJ/du_0     = lambda_0,
 *     dJ/du_{-1}  = -lambda_1,
 *     dJ/dc       = sum_{n=0}^{nt-1} lambda_{n+1} (.) L(u_n).
 * Inputs and outputs are padded boxes; adjoint fields carry a zero shell.
 * Every forward level u_0..u_{nt-1} is stored (no checkpointing): meant for
 * small grids.  Returns 0 or -1.
 */
int oracle_adjoint_wave_varc(int64_t nx, int64_t ny, int64_t nz, int64_t h,
                             const double* um1, const double* u0, const double* c,
                             const double* w, int64_t nt, const double* seed,
                             double* g_um1, double* g_u0, double* g_c, int nthreads) {
    if (nx < 0 || ny < 0 || nz < 0 || h < 4 || nt < 0) return -1;
    if (!um1 || !u0 || !c || !w || !seed || !g_um1 || !g_u0 || !g_c) return -1;
    set_threads(nthreads);
    box b = mkbox(nx, ny, nz, h);
    const int64_t n = box_size(&b);

    /* forward, keeping u_{-1} .. u_{nt-1} */
    double* hist = (double*)malloc((size_t)(nt + 1) * (size_t)n * sizeof(double));
    double* lam = (double*)calloc((size_t)3 * (size_t)n, sizeof(double));
    double* cl = (double*)calloc((size_t)n, sizeof(double));
    if (!hist || !lam || !cl) { free(hist); free(lam); free(cl); return -1; }
    /* hist slot k holds u_{k-1} */
    memcpy(hist, um1, (size_t)n * sizeof(double));
    if (nt >= 1) memcpy(hist + n, u0, (size_t)n * sizeof(double));
    for (int64_t k = 2; k <= nt; ++k) {
        /* u_{k-1} = 2 u_{k-2} - u_{k-3} + c L8(u_{k-2}) */
        double* dst = hist + k * n;
        const double* cur = hist + (k - 1) * n;
        memcpy(dst, hist + (k - 2) * n, (size_t)n * sizeof(double));
        sweep_wave(OK_WAVE_VARC, &b, cur, dst, c, 0.0, w);
    }

    memset(g_c, 0, (size_t)n * sizeof(double));
    /* lambda buffers: a = lambda_{n+1}, bb = lambda_{n+2}, nw = lambda_n */
    double* la = lam;         /* lambda_{n+1} */
    double* lb = lam + n;     /* lambda_{n+2} */
    double* ln = lam + 2 * n; /* lambda_n     */
    for (int64_t z = 0; z < nz; ++z)
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t x = 0; x < nx; ++x) la[at(&b, x, y, z)] = seed[at(&b, x, y, z)];
    /* lb = lambda_{nt+1} = 0 already */
    for (int64_t s = nt - 1; s >= 0; --s) {
        const double* us = hist + (s + 1) * n; /* u_s */
        /* cl = c (.) lambda_{s+1} on the interior, zero shell */
        for (int64_t z = 0; z < nz; ++z)
            for (int64_t y = 0; y < ny; ++y)
                for (int64_t x = 0; x < nx; ++x) {
                    const int64_t p = at(&b, x, y, z);
                    cl[p] = c[p] * la[p];
                }
#pragma omp parallel for schedule(static)
        for (int64_t z = 0; z < nz; ++z)
            for (int64_t y = 0; y < ny; ++y)
                for (int64_t x = 0; x < nx; ++x) {
                    const int64_t p = at(&b, x, y, z);
                    g_c[p] += la[p] * lap8(&b, us, w, x, y, z);
                    ln[p] = 2.0 * la[p] - lb[p] + lap8(&b, cl, w, x, y, z);
                }
        double* t = lb; lb = la; la = ln; ln = t; /* la = lambda_s, lb = lambda_{s+1} */
    }
    /* now la = lambda_0, lb = lambda_1 (for nt = 0: la = seed, lb = 0) */
    memset(g_u0, 0, (size_t)n * sizeof(double));
    memset(g_um1, 0, (size_t)n * sizeof(double));
    for (int64_t z = 0; z < nz; ++z)
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t x = 0; x < nx; ++x) {
                const int64_t p = at(&b, x, y, z);
                g_u0[p] = la[p];
                g_um1[p] = -lb[p];
            }
    free(hist); free(lam); free(cl);
    return 0;
}

/*
 * Adjoint of the first-order variable-coefficient kinds 2 and 3 (Fig. 1c,
 * 1d).  Not in the paper: with A the sweep operator of Fig. 1c/1d for fixed
 * coefficients (zero Dirichlet boundary), u_{t+1} = A u_t, and a loss J with
 * dJ/du_nt = seed, the adjoint fields are lambda_nt = seed,
 * lambda_t = A^T lambda_{t+1}, and dJ/du_0 = lambda_0.  Written as a gather,
 * A^T lambda at interior q sums, over the taps of the stencil, the weight a
 * point p = q - offset gives u(q), times lambda(p), for interior p only:
 *   kind 2:  (A^T l)(q) = sum_k W_k(q - o_k) l(q - o_k),  o_k = 0, -x, +x, -y, +y, -z, +z
 *   kind 3:  (A^T l)(q) = W_0(q) l(q) + sum_{r,a} [ W_{ra}(q + r e_a) l(q + r e_a)
 *                                                + W_{ra}(q - r e_a) l(q - r e_a) ]
 * The coefficient gradients are dJ/dW_k(p) = sum_t lambda_{t+1}(p) * (the
 * value W_k multiplies at p in step t): u_t(p + o_k) for kind 2, u_t(p) for
 * W_0 and the pair u_t(p - r e_a) + u_t(p + r e_a) for W_{ra} of kind 3.
 * g_coef holds K arrays of the box size (same layout as coef).  All levels of
 * the forward run are kept (small grids only).
 */
static int inside(const box* b, int64_t x, int64_t y, int64_t z) {
    return x >= 0 && y >= 0 && z >= 0 && x < b->nx && y < b->ny && z < b->nz;
}

int oracle_adjoint_jacobi_var(int kind, int64_t nx, int64_t ny, int64_t nz, int64_t h,
                              const double* u0, const double* coef, int64_t nt,
                              const double* seed, double* g_u0, double* g_coef, int nthreads) {
    if ((kind != OK_7V && kind != OK_25V) || nx < 0 || ny < 0 || nz < 0 || nt < 0) return -1;
    if (h < radius_of(kind) || !u0 || !coef || !seed || !g_u0 || !g_coef) return -1;
    set_threads(nthreads);
    box b = mkbox(nx, ny, nz, h);
    const int64_t n = box_size(&b);
    const int K = ncoef_of(kind);
    double* hist = (double*)malloc((size_t)(nt > 0 ? nt : 1) * (size_t)n * sizeof(double));
    double* la = (double*)calloc((size_t)n, sizeof(double));
    double* ln = (double*)calloc((size_t)n, sizeof(double));
    if (!hist || !la || !ln) { free(hist); free(la); free(ln); return -1; }
    /* forward: hist slot t holds u_t, t = 0 .. nt-1 (shell included) */
    if (nt >= 1) memcpy(hist, u0, (size_t)n * sizeof(double));
    for (int64_t t = 1; t < nt; ++t) {
        memcpy(hist + t * n, hist + (t - 1) * n, (size_t)n * sizeof(double)); /* the shell */
        sweep_jacobi(kind, &b, hist + (t - 1) * n, hist + t * n, coef, NULL);
    }
    memset(g_coef, 0, (size_t)K * (size_t)n * sizeof(double));
    for (int64_t z = 0; z < nz; ++z)
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t x = 0; x < nx; ++x) la[at(&b, x, y, z)] = seed[at(&b, x, y, z)];
    static const int ox[7] = {0, -1, 1, 0, 0, 0, 0};
    static const int oy[7] = {0, 0, 0, -1, 1, 0, 0};
    static const int oz[7] = {0, 0, 0, 0, 0, -1, 1};
    const double* W = coef;
    for (int64_t t = nt - 1; t >= 0; --t) {
        const double* u = hist + t * n; /* u_t; la = lambda_{t+1} */
#pragma omp parallel for schedule(static)
        for (int64_t z = 0; z < nz; ++z)
            for (int64_t y = 0; y < ny; ++y)
                for (int64_t x = 0; x < nx; ++x) {
                    const int64_t q = at(&b, x, y, z);
                    /* gradient terms of step t at p = q */
                    if (kind == OK_7V) {
                        for (int k = 0; k < 7; ++k)
                            g_coef[k * n + q] += la[q] * u[at(&b, x + ox[k], y + oy[k], z + oz[k])];
                    } else {
                        g_coef[q] += la[q] * u[q];
                        for (int r = 1; r <= 4; ++r) {
                            const int64_t kx = 3 * (r - 1) + 1;
                            g_coef[kx * n + q] += la[q] * (u[at(&b, x - r, y, z)] + u[at(&b, x + r, y, z)]);
                            g_coef[(kx + 1) * n + q] += la[q] * (u[at(&b, x, y - r, z)] + u[at(&b, x, y + r, z)]);
                            g_coef[(kx + 2) * n + q] += la[q] * (u[at(&b, x, y, z - r)] + u[at(&b, x, y, z + r)]);
                        }
                    }
                    /* lambda_t(q) = (A^T lambda_{t+1})(q) */
                    double v = 0.0;
                    if (kind == OK_7V) {
                        for (int k = 0; k < 7; ++k) {
                            const int64_t px = x - ox[k], py = y - oy[k], pz = z - oz[k];
                            if (inside(&b, px, py, pz)) {
                                const int64_t pp = at(&b, px, py, pz);
                                v += W[k * n + pp] * la[pp];
                            }
                        }
                    } else {
                        v = W[q] * la[q];
                        for (int r = 1; r <= 4; ++r) {
                            const int64_t kx = 3 * (r - 1) + 1;
                            const int64_t nb[6][3] = {{x + r, y, z}, {x - r, y, z}, {x, y + r, z},
                                                      {x, y - r, z}, {x, y, z + r}, {x, y, z - r}};
                            for (int i = 0; i < 6; ++i) {
                                if (!inside(&b, nb[i][0], nb[i][1], nb[i][2])) continue;
                                const int64_t pp = at(&b, nb[i][0], nb[i][1], nb[i][2]);
                                v += W[(kx + i / 2) * n + pp] * la[pp];
                            }
                        }
                    }
                    ln[q] = v;
                }
        double* tmp = la; la = ln; ln = tmp;
    }
    memset(g_u0, 0, (size_t)n * sizeof(double));
    for (int64_t z = 0; z < nz; ++z)
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t x = 0; x < nx; ++x) g_u0[at(&b, x, y, z)] = la[at(&b, x, y, z)];
    free(hist); free(la); free(ln);
    return 0;
}

/*
 * One update (Fig. 1b-1e) evaluated at a list of interior points, for
 * checking single sweeps of very large grids on sampled outputs.  pts holds
 * npts triples (x, y, z); out[i] receives the new value at point i (for the
 * leapfrog kinds: 2 u - u_prev + alpha L8(u)).  Returns 0 or -1.
 */
int oracle_step_points(int kind, int64_t nx, int64_t ny, int64_t nz, int64_t h,
                       const double* u_prev, const double* u, const double* coef,
                       const double* w, double alpha, int64_t npts, const int64_t* pts,
                       double* out) {
    if (kind < OK_7C || kind > OK_WAVE_VARC || h < radius_of(kind) || !u || !w || !pts || !out)
        return -1;
    if (ncoef_of(kind) > 0 && !coef) return -1;
    if (kind >= OK_WAVE && !u_prev) return -1;
    box b = mkbox(nx, ny, nz, h);
    const int64_t n = box_size(&b);
    for (int64_t i = 0; i < npts; ++i) {
        const int64_t x = pts[3 * i], y = pts[3 * i + 1], z = pts[3 * i + 2];
        if (x < 0 || y < 0 || z < 0 || x >= nx || y >= ny || z >= nz) return -1;
        const int64_t p = at(&b, x, y, z);
        double v;
        if (kind == OK_7C) {
            v = w[0] * u[p]
              + w[1] * (u[at(&b, x - 1, y, z)] + u[at(&b, x + 1, y, z)])
              + w[1] * (u[at(&b, x, y - 1, z)] + u[at(&b, x, y + 1, z)])
              + w[1] * (u[at(&b, x, y, z - 1)] + u[at(&b, x, y, z + 1)]);
        } else if (kind == OK_7V) {
            const double* W = coef;
            v = W[0 * n + p] * u[p]
              + W[1 * n + p] * u[at(&b, x - 1, y, z)]
              + W[2 * n + p] * u[at(&b, x + 1, y, z)]
              + W[3 * n + p] * u[at(&b, x, y - 1, z)]
              + W[4 * n + p] * u[at(&b, x, y + 1, z)]
              + W[5 * n + p] * u[at(&b, x, y, z - 1)]
              + W[6 * n + p] * u[at(&b, x, y, z + 1)];
        } else if (kind == OK_25V) {
            const double* W = coef;
            v = W[0 * n + p] * u[p];
            for (int r = 1; r <= 4; ++r) {
                const int64_t kx = 3 * (r - 1) + 1, ky = kx + 1, kz = kx + 2;
                v += W[kx * n + p] * (u[at(&b, x - r, y, z)] + u[at(&b, x + r, y, z)]);
                v += W[ky * n + p] * (u[at(&b, x, y - r, z)] + u[at(&b, x, y + r, z)]);
                v += W[kz * n + p] * (u[at(&b, x, y, z - r)] + u[at(&b, x, y, z + r)]);
            }
        } else {
            const double a = (kind == OK_WAVE_VARC) ? coef[p] : alpha;
            v = 2.0 * u[p] - u_prev[p] + a * lap8(&b, u, w, x, y, z);
        }
        out[i] = v;
    }
    return 0;
}
