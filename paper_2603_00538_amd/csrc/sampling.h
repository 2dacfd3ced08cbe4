// Per-element uniform samples on the device (sec. 4.1 step 3).
//
// Sample j of target element t is a pure function of (seed, stream, t, j):
// Philox4x32-10 at counter (j, t, stream, blk) with key (seed_lo, seed_hi).
//  * triangles: xi from words (0,1), eta from words (2,3) of block 0; the
//    area-uniform barycentric weights of Osada et al. (2002),
//    lambda = (1 - sqrt(xi), sqrt(xi)(1 - eta), sqrt(xi) eta);
//  * tetrahedra: u1, u2 from block 0, u3 from words (0,1) of block 1; sorted,
//    the spacings (s1, s2 - s1, s3 - s2, 1 - s3) are uniform on the simplex;
//  * d-simplices, d = 4..6: the same with d uniforms, u_(i+1) from block i/2,
//    words (0,1) for even i and (2,3) for odd i, sorted by a compare-exchange
//    network (the sorted values, so the spacings are those of any sort).
// lambda_k belongs to vertex k of the element in connectivity order; the
// physical point is sum_k lambda_k x_{v_k}.
// Stratified samples (FT_SAMPLING_STRATIFIED): with m = floor(N^(1/d')) cells
// per axis of the d' = d uniforms, sample j < m^d' takes the cell given by the
// base-m digits of j, lowest first (j mod m, (j / m) mod m, ...), and its uniforms become
// min((cell_i + u_i) (1/m), 1 - 2^-53) (binary32: 1/m and 1 - 2^-24 in binary32)
// before the same maps; the other samples stay plain.  Each cell maps onto an
// equal-volume part of the simplex, so every sample stays uniform on its part
// and the estimate unbiased.
#pragma once

#include "common.h"

namespace ft {

struct SampleKey {
    uint32_t k0, k1, stream;
    uint32_t strat_n;   // samples j < strat_n are stratified (m^d' of them); 0: plain sampling
    FastDiv m_div;      // division by m, the cells per axis
    double inv_m;       // 1/m rounded to binary64
    float inv_m_f;      // 1/m rounded to binary32
};

// Key of a transfer's samples: Philox key and counter word 2, and the strata.
inline SampleKey make_sample_key(const ft_sample_cfg& c, int dim) {
    SampleKey k{};
    k.k0 = uint32_t(c.seed & 0xFFFFFFFFu);
    k.k1 = uint32_t(c.seed >> 32);
    k.stream = c.stream_id;
    k.strat_n = 0;
    k.m_div = make_fastdiv(1);
    k.inv_m = 1.0;
    k.inv_m_f = 1.0f;
    if (c.sampling == FT_SAMPLING_STRATIFIED && c.samples_per_elem > 0) {
        const int dp = dim;   // uniforms per sample
        const uint64_t N = uint64_t(c.samples_per_elem);
        uint64_t m = 1;
        auto pw = [dp](uint64_t x) {
            uint64_t r = 1;
            for (int i = 0; i < dp; ++i) r *= x;
            return r;
        };
        while (pw(m + 1) <= N) ++m;
        k.strat_n = uint32_t(pw(m));
        k.m_div = make_fastdiv(uint32_t(m));
        k.inv_m = 1.0 / double(m);
        k.inv_m_f = 1.0f / float(m);
    }
    return k;
}

constexpr double kBelowOne = 0x1.fffffffffffffp-1;   // 1 - 2^-53
constexpr float kBelowOneF = 0x1.fffffep-1f;         // 1 - 2^-24

// The stratum of sample j < strat_n: its cell per axis, the base-m digits
// of j, lowest first.
template <int DP>
__device__ __forceinline__ void sample_cell(uint32_t j, const SampleKey& key, uint32_t (&cell)[DP]) {
    uint32_t q = j;
#pragma unroll
    for (int i = 0; i + 1 < DP; ++i) {
        const uint32_t qn = fast_div(q, key.m_div);
        cell[i] = q - qn * key.m_div.d;
        q = qn;
    }
    cell[DP - 1] = q;
}

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

// Ascending order of n values (uniforms in (0, 1), never NaN) by odd-even
// transposition (n rounds of compare-exchanges): fixed, branch-free, exact
// (min and max only).
template <int NV, typename T>
__device__ __forceinline__ void sort_network(T (&u)[NV]) {
#pragma unroll
    for (int r = 0; r < NV; ++r)
#pragma unroll
        for (int i = r & 1; i + 1 < NV; i += 2) {
            const T lo = fmin(u[i], u[i + 1]);
            const T hi = fmax(u[i], u[i + 1]);
            u[i] = lo;
            u[i + 1] = hi;
        }
}

template <int D>
__device__ __forceinline__ void sample_lambda(uint32_t t, uint32_t j, const SampleKey& key, double (&lam)[D + 1]) {
    const u32x4 w = philox4x32_10(u32x4{j, t, key.stream, 0u}, key.k0, key.k1);
    if constexpr (D == 2) {
        double xi = uniform53(w.x, w.y);
        double eta = uniform53(w.z, w.w);
        if (j < key.strat_n) {
            uint32_t cell[2];
            sample_cell<2>(j, key, cell);
            xi = fmin((double(cell[0]) + xi) * key.inv_m, kBelowOne);
            eta = fmin((double(cell[1]) + eta) * key.inv_m, kBelowOne);
        }
        const double r = sqrt_unit(xi);
        lam[0] = 1.0 - r;
        lam[1] = r * (1.0 - eta);
        lam[2] = r * eta;
    } else if constexpr (D >= 4) {
        double u[D];
        u[0] = uniform53(w.x, w.y);
        u[1] = uniform53(w.z, w.w);
#pragma unroll
        for (int b = 1; b < (D + 1) / 2; ++b) {
            const u32x4 wb = philox4x32_10(u32x4{j, t, key.stream, uint32_t(b)}, key.k0, key.k1);
            u[2 * b] = uniform53(wb.x, wb.y);
            if (2 * b + 1 < D) u[2 * b + 1] = uniform53(wb.z, wb.w);
        }
        if (j < key.strat_n) {
            uint32_t cell[D];
            sample_cell<D>(j, key, cell);
#pragma unroll
            for (int i = 0; i < D; ++i) u[i] = fmin((double(cell[i]) + u[i]) * key.inv_m, kBelowOne);
        }
        sort_network<D>(u);
        lam[0] = u[0];
#pragma unroll
        for (int k = 1; k < D; ++k) lam[k] = u[k] - u[k - 1];
        lam[D] = 1.0 - u[D - 1];
    } else {
        const u32x4 w1 = philox4x32_10(u32x4{j, t, key.stream, 1u}, key.k0, key.k1);
        double a = uniform53(w.x, w.y), b = uniform53(w.z, w.w), c = uniform53(w1.x, w1.y);
        if (j < key.strat_n) {
            uint32_t cell[3];
            sample_cell<3>(j, key, cell);
            a = fmin((double(cell[0]) + a) * key.inv_m, kBelowOne);
            b = fmin((double(cell[1]) + b) * key.inv_m, kBelowOne);
            c = fmin((double(cell[2]) + c) * key.inv_m, kBelowOne);
        }
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
        float xi = uniform24(w.x);
        float eta = uniform24(w.z);
        if (j < key.strat_n) {
            uint32_t cell[2];
            sample_cell<2>(j, key, cell);
            xi = fminf((float(cell[0]) + xi) * key.inv_m_f, kBelowOneF);
            eta = fminf((float(cell[1]) + eta) * key.inv_m_f, kBelowOneF);
        }
        const float r = sqrtf(xi);
        lam[0] = 1.0f - r;
        lam[1] = r * (1.0f - eta);
        lam[2] = r * eta;
    } else if constexpr (D >= 4) {
        float u[D];
        u[0] = uniform24(w.x);
        u[1] = uniform24(w.z);
#pragma unroll
        for (int b = 1; b < (D + 1) / 2; ++b) {
            const u32x4 wb = philox4x32_10(u32x4{j, t, key.stream, uint32_t(b)}, key.k0, key.k1);
            u[2 * b] = uniform24(wb.x);
            if (2 * b + 1 < D) u[2 * b + 1] = uniform24(wb.z);
        }
        if (j < key.strat_n) {
            uint32_t cell[D];
            sample_cell<D>(j, key, cell);
#pragma unroll
            for (int i = 0; i < D; ++i) u[i] = fminf((float(cell[i]) + u[i]) * key.inv_m_f, kBelowOneF);
        }
        sort_network<D>(u);
        lam[0] = u[0];
#pragma unroll
        for (int k = 1; k < D; ++k) lam[k] = u[k] - u[k - 1];
        lam[D] = 1.0f - u[D - 1];
    } else {
        const u32x4 w1 = philox4x32_10(u32x4{j, t, key.stream, 1u}, key.k0, key.k1);
        float a = uniform24(w.x), b = uniform24(w.z), c = uniform24(w1.x);
        if (j < key.strat_n) {
            uint32_t cell[3];
            sample_cell<3>(j, key, cell);
            a = fminf((float(cell[0]) + a) * key.inv_m_f, kBelowOneF);
            b = fminf((float(cell[1]) + b) * key.inv_m_f, kBelowOneF);
            c = fminf((float(cell[2]) + c) * key.inv_m_f, kBelowOneF);
        }
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
