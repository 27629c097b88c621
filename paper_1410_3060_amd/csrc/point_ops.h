// Per-point stencil operators of Fig. 1b-1e (Sect. 3.1), one fixed FP32
// evaluation order per kind.  Every kernel of the library (naive sweep,
// temporally blocked wavefront, adjoint) evaluates a lattice update through
// these functions, so all schemes round identically and the blocked result
// equals the naive one bit for bit.  Translation units that include this
// header are compiled with -ffp-contract=off: the only fused operations are
// the explicit __builtin_fmaf calls below.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace stn {

// Stencil radius R and number of domain-sized coefficient arrays K per kind
// (kind numbering of include/stencil.h).
template <int KIND> struct kind_traits;
template <> struct kind_traits<1> { static constexpr int R = 1, K = 0; static constexpr bool leapfrog = false; };
template <> struct kind_traits<2> { static constexpr int R = 1, K = 7; static constexpr bool leapfrog = false; };
template <> struct kind_traits<3> { static constexpr int R = 4, K = 13; static constexpr bool leapfrog = false; };
template <> struct kind_traits<4> { static constexpr int R = 4, K = 0; static constexpr bool leapfrog = true; };
template <> struct kind_traits<5> { static constexpr int R = 4, K = 1; static constexpr bool leapfrog = true; };

// Coefficient loads: FP32 as is, BF16 expanded exactly (the 16 stored bits
// become the high half of the FP32 pattern).
__device__ __forceinline__ float load_coef(const float* p, int64_t i) { return p[i]; }
__device__ __forceinline__ float load_coef(const uint16_t* p, int64_t i) {
    return __uint_as_float(static_cast<uint32_t>(p[i]) << 16);
}

// Scalar weights passed by value to the kernels.  lres is the centre
// weight that L8 keeps after its neighbour terms are written as differences
// from the centre: w0 + 6 (w1 + w2 + w3 + w4), rounded once from double on
// the host (zero for the 8th-order weights).
struct weights {
    float w[5];
    float alpha;
    float lres;
};

// Neighbourhood of one point: centre value, the six axis pairs per radius
// already summed, and the individual face neighbours at radius 1 (needed by
// the unsymmetric Fig. 1c operator).  pair[a][r-1] = u(p - r e_a) + u(p + r e_a),
// a = 0 (x), 1 (y), 2 (z).
template <int R>
struct nbhd {
    float c;
    float pair[3][R];
    float m1[3], p1[3];  // u(p - e_a), u(p + e_a)
};

// Fig. 1b: w0*u + w1*((x pair + y pair) + z pair)
__device__ __forceinline__ float op_7pt_const(const weights& wt, const nbhd<1>& n) {
    const float s = (n.pair[0][0] + n.pair[1][0]) + n.pair[2][0];
    return __builtin_fmaf(wt.w[1], s, wt.w[0] * n.c);
}

// Fig. 1c: W0*u, then W1..W6 in the order x-1, x+1, y-1, y+1, z-1, z+1.
__device__ __forceinline__ float op_7pt_var(const float (&W)[7], const nbhd<1>& n) {
    float a = W[0] * n.c;
    a = __builtin_fmaf(W[1], n.m1[0], a);
    a = __builtin_fmaf(W[2], n.p1[0], a);
    a = __builtin_fmaf(W[3], n.m1[1], a);
    a = __builtin_fmaf(W[4], n.p1[1], a);
    a = __builtin_fmaf(W[5], n.m1[2], a);
    a = __builtin_fmaf(W[6], n.p1[2], a);
    return a;
}

// Fig. 1d: W0*u, then for r = 1..4 the x, y, z pairs with W_{3(r-1)+1+axis}.
__device__ __forceinline__ float op_25pt_var(const float (&W)[13], const nbhd<4>& n) {
    float a = W[0] * n.c;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        a = __builtin_fmaf(W[3 * r + 1], n.pair[0][r], a);
        a = __builtin_fmaf(W[3 * r + 2], n.pair[1][r], a);
        a = __builtin_fmaf(W[3 * r + 3], n.pair[2][r], a);
    }
    return a;
}

// L8 of Fig. 1e, w0*u + sum_r w_r * (x pair + y pair + z pair), evaluated as
//   lres*u + sum_{r=1..4} w_r * (((x pair + y pair) + z pair) - 6u),
// lres = w0 + 6 sum_r w_r: the same operator, but each difference is exactly
// zero on a constant field, so the FP32-rounded weights keep the operator's
// zero row sum.  With w0 * u first the rounded weights leave a row sum of
// about 1e-7 * |w0|, an extra alpha*eps*u term per leapfrog step whose effect
// grows like nt^2: 3.4e-5 relative after 100 steps of the 512^3 constant-
// coefficient workload, against 5e-7 in this form.
__device__ __forceinline__ float op_lap8(const weights& wt, const nbhd<4>& n) {
    const float six = 6.0f * n.c;
    float a = wt.lres * n.c;
#pragma unroll
    for (int r = 0; r < 4; ++r)
        a = __builtin_fmaf(wt.w[r + 1], ((n.pair[0][r] + n.pair[1][r]) + n.pair[2][r]) - six, a);
    return a;
}

// Leapfrog update of Fig. 1e: (2u - u_prev) + alpha * L8(u).
__device__ __forceinline__ float op_leapfrog(float alpha, float lap, float c, float prev) {
    return __builtin_fmaf(alpha, lap, __builtin_fmaf(2.0f, c, -prev));
}

// Number of coefficient slots a kernel carries per point (at least one).
template <int KIND>
constexpr int kslots = kind_traits<KIND>::K > 0 ? kind_traits<KIND>::K : 1;

// One lattice-site update of kind KIND.  W holds the K coefficient values at
// the point (for kind 5, W[0] is alpha(p)); prev is u_{n-1}(p) for the
// leapfrog kinds and ignored otherwise.
template <int KIND>
__device__ __forceinline__ float update(const weights& wt, const float (&W)[kslots<KIND>],
                                        const nbhd<kind_traits<KIND>::R>& n, float prev) {
    if constexpr (KIND == 1) {
        return op_7pt_const(wt, n);
    } else if constexpr (KIND == 2) {
        return op_7pt_var(W, n);
    } else if constexpr (KIND == 3) {
        return op_25pt_var(W, n);
    } else if constexpr (KIND == 4) {
        return op_leapfrog(wt.alpha, op_lap8(wt, n), n.c, prev);
    } else {
        return op_leapfrog(W[0], op_lap8(wt, n), n.c, prev);
    }
}

}  // namespace stn
