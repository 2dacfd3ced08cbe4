// Per-element uniform samples on the device (sec. 4.1 step 3).
//
// Sample j of target element t is a pure function of (seed, stream, t, j):
// Philox4x32-10 at counter (j, t, stream, blk) with key (seed_lo, seed_hi).
//  * triangles: xi from words (0,1), eta from words (2,3) of block 0; the
//    area-uniform barycentric weights of Osada et al. (2002),
//    lambda = (1 - sqrt(xi), sqrt(xi)(1 - eta), sqrt(xi) eta);
//  * tetrahedra: u1, u2 from block 0, u3 from words (0,1) of block 1; sorted,
//    the spacings (s1, s2 - s1, s3 - s2, 1 - s3) are uniform on the simplex.
// lambda_k belongs to vertex k of the element in connectivity order; the
// physical point is sum_k lambda_k x_{v_k}.
#pragma once

#include "common.h"

namespace ft {

struct SampleKey {
    uint32_t k0, k1, stream;
};

// Square root of a in [2^-53, 1]: the hardware reciprocal-square-root estimate,
// one Goldschmidt step (g -> sqrt(a), h -> 1 / (2 sqrt(a))) and two Newton
// corrections of g (Markstein's scheme).  The argument range needs none of the
// general routine's rescaling or special cases.
__device__ __forceinline__ double sqrt_unit(double a) {
    const double y = __builtin_amdgcn_rsq(a);
    double g = a * y, h = 0.5 * y;
    const double r = fma(-h, g, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    double d = fma(-g, g, a);
    g = fma(d, h, g);
    d = fma(-g, g, a);
    return fma(d, h, g);
}

template <int D>
__device__ __forceinline__ void sample_lambda(uint32_t t, uint32_t j, const SampleKey& key, double (&lam)[D + 1]) {
    const u32x4 w = philox4x32_10(u32x4{j, t, key.stream, 0u}, key.k0, key.k1);
    if constexpr (D == 2) {
        const double xi = uniform53(w.x, w.y);
        const double eta = uniform53(w.z, w.w);
        const double r = sqrt_unit(xi);
        lam[0] = 1.0 - r;
        lam[1] = r * (1.0 - eta);
        lam[2] = r * eta;
    } else {
        const u32x4 w1 = philox4x32_10(u32x4{j, t, key.stream, 1u}, key.k0, key.k1);
        double a = uniform53(w.x, w.y), b = uniform53(w.z, w.w), c = uniform53(w1.x, w1.y);
        // three-comparator sorting network
        double lo = fmin(a, b), hi = fmax(a, b);
        a = lo; b = hi;
        lo = fmin(b, c); hi = fmax(b, c);
        b = lo; c = hi;
        lo = fmin(a, b); hi = fmax(a, b);
        a = lo; b = hi;
        lam[0] = a;
        lam[1] = b - a;
        lam[2] = c - b;
        lam[3] = 1.0 - c;
    }
}

// Single-precision form: the same counters, 24-bit uniforms (2 (m >> 29) + 1) 2^-24
// from the same 52-bit m, arithmetic in binary32.
template <int D>
__device__ __forceinline__ void sample_lambda_f32(uint32_t t, uint32_t j, const SampleKey& key, float (&lam)[D + 1]) {
    const u32x4 w = philox4x32_10(u32x4{j, t, key.stream, 0u}, key.k0, key.k1);
    if constexpr (D == 2) {
        const float xi = uniform24(w.x);
        const float eta = uniform24(w.z);
        const float r = sqrtf(xi);
        lam[0] = 1.0f - r;
        lam[1] = r * (1.0f - eta);
        lam[2] = r * eta;
    } else {
        const u32x4 w1 = philox4x32_10(u32x4{j, t, key.stream, 1u}, key.k0, key.k1);
        float a = uniform24(w.x), b = uniform24(w.z), c = uniform24(w1.x);
        float lo = fminf(a, b), hi = fmaxf(a, b);
        a = lo; b = hi;
        lo = fminf(b, c); hi = fmaxf(b, c);
        b = lo; c = hi;
        lo = fminf(a, b); hi = fmaxf(a, b);
        a = lo; b = hi;
        lam[0] = a;
        lam[1] = b - a;
        lam[2] = c - b;
        lam[3] = 1.0f - c;
    }
}

}  // namespace ft
