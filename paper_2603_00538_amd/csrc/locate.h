// Device side of the mesh-backed P1 source: bin grid, barycentric records and
// the wave-cooperative localization (shared by the evaluation kernel and the
// fused sample-evaluate-consume kernel).
//
// Localization rule: the element maximizing min_k mu_k(x) (mu: barycentric
// coordinates); exact ties -> lowest element id; a best min mu below -1e-10
// is out of the domain (counted, extrapolated from that element).  A point
// whose best element has min mu > 1e-12 is strictly inside it, and no other
// element can tie or win, so the search stops there.
//
// The 64 points of a wave are usually samples of one target element, so they
// share a handful of bins.  The wave computes its own bounding box, culls each
// bin's candidates 64 at a time against it (one candidate per lane, a
// ballot), and then every lane tests its point against each surviving
// candidate, whose record is wave-uniform (scalar loads).  Waves whose points
// span many bins (scattered input) fall back to one bin per lane.
#pragma once

#include <cfloat>

#include "common.h"

namespace ft {

constexpr double kInsideTau = 1e-12;
constexpr double kOutTol = -1e-10;

template <int D>
struct RecSize { static constexpr int value = D == 2 ? 8 : 16; };

__device__ __forceinline__ float f32_down(double x) {
    float f = (float)x;
    if ((double)f > x) f = nextafterf(f, -INFINITY);
    return f;
}
__device__ __forceinline__ float f32_up(double x) {
    float f = (float)x;
    if ((double)f < x) f = nextafterf(f, INFINITY);
    return f;
}

struct GridView {
    int32_t nb[3];
    double lo[3];
    double inv_h[3];
};

// Bin index along axis c; monotone in x, so a point inside a box always maps
// into the box's bin range.  NaN maps to bin 0.
__device__ __forceinline__ int bin_of(double x, int c, const GridView& g) {
    double u = (x - g.lo[c]) * g.inv_h[c];
    u = fmin(fmax(u, 0.0), double(g.nb[c] - 1));
    return int(u);
}

// ---------------------------------------------------------------- evaluation
struct SrcView {
    const double* rec;
    const float* box;
    const int32_t* conn;
    const double* values;
    const int64_t* bin_ptr;
    const int32_t* bin_elems;
    int64_t n;
    int F;
    GridView g;
};

// Barycentric coordinates of p in element e (record r): mu_{k+1} = A[k] . (p - x0),
// mu_0 = 1 - sum.  Returns min_k mu_k.
template <int D>
__device__ __forceinline__ double barycentric(const double* __restrict__ r, const double (&p)[D],
                                              double (&mu)[D + 1]) {
    double d[D];
#pragma unroll
    for (int c = 0; c < D; ++c) d[c] = p[c] - r[c];
    mu[0] = 1.0;
    double mn = INFINITY;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        double s = 0.0;
#pragma unroll
        for (int c = 0; c < D; ++c) s = fma(r[D + k * D + c], d[c], s);
        mu[k + 1] = s;
        mu[0] -= s;
        mn = fmin(mn, s);
    }
    return fmin(mn, mu[0]);
}

template <int D>
__device__ __forceinline__ void test_candidate(const double* __restrict__ r, int e, const double (&p)[D], double& best,
                                               int& bid) {
    double mu[D + 1];
    const double mn = barycentric<D>(r, p, mu);
    if ((mn > best) || (mn == best && e < bid)) {
        best = mn;
        bid = e;
    }
}

// Rule winner for each of this lane's P points among the candidates of the
// bins the wave's points touch (see the file comment).  Every lane of the
// wave must call it (points a lane does not own pass active = false).
// Returns best = max min-barycentric and bid = its element id (INT_MAX if no
// candidate was found) per point; barycentric() recomputes mu for the winner.
template <int D, int P>
__device__ __forceinline__ void locate_wave(const SrcView& S, const double (&p)[P][D], const bool (&active)[P],
                                            double (&best)[P], int (&bid)[P]) {
    constexpr int RS = RecSize<D>::value;
    constexpr int MAX_SPAN = D == 2 ? 9 : 12;
    const int lane = threadIdx.x & 63;
    double wlo[D], whi[D];
    int b0[3] = {0, 0, 0}, b1[3] = {0, 0, 0};
    int span = 1;
#pragma unroll
    for (int c = 0; c < D; ++c) {
        double lo = INFINITY, hi = -INFINITY;
#pragma unroll
        for (int q = 0; q < P; ++q)
            if (active[q]) {
                lo = fmin(lo, p[q][c]);
                hi = fmax(hi, p[q][c]);
            }
        wlo[c] = wave_min(lo);
        whi[c] = wave_max(hi);
        b0[c] = uniform_int(bin_of(wlo[c], c, S.g));
        b1[c] = uniform_int(bin_of(whi[c], c, S.g));
        span *= b1[c] - b0[c] + 1;
    }
#pragma unroll
    for (int q = 0; q < P; ++q) {
        best[q] = -DBL_MAX;
        bid[q] = INT_MAX;
    }

    if (span <= MAX_SPAN) {
        float flo[D], fhi[D];
#pragma unroll
        for (int c = 0; c < D; ++c) {
            flo[c] = f32_down(wlo[c]);
            fhi[c] = f32_up(whi[c]);
        }
        bool finished = false;
        for (int bz = b0[2]; bz <= b1[2] && !finished; ++bz)
            for (int by = b0[1]; by <= b1[1] && !finished; ++by)
                for (int bx = b0[0]; bx <= b1[0] && !finished; ++bx) {
                    const int64_t b = (int64_t(bz) * S.g.nb[1] + by) * S.g.nb[0] + bx;
                    const int64_t start = S.bin_ptr[b], end = S.bin_ptr[b + 1];
                    for (int64_t c0 = start; c0 < end && !finished; c0 += 64) {
                        int cid = -1;
                        bool ov = false;
                        if (c0 + lane < end) {
                            cid = S.bin_elems[c0 + lane];
                            const float* bx_ = S.box + int64_t(cid) * 2 * D;
                            ov = true;
#pragma unroll
                            for (int c = 0; c < D; ++c) ov &= (bx_[c] <= fhi[c]) & (bx_[D + c] >= flo[c]);
                        }
                        uint64_t mask = __ballot(ov);
                        while (mask) {
                            const int l = __ffsll((unsigned long long)mask) - 1;
                            mask &= mask - 1;
                            const int e = read_lane(cid, l);
                            const double* r = S.rec + int64_t(e) * RS;
                            bool done = true;
#pragma unroll
                            for (int q = 0; q < P; ++q) {
                                test_candidate<D>(r, e, p[q], best[q], bid[q]);
                                done &= !active[q] || best[q] > kInsideTau;
                            }
                            if (__all(done)) {
                                finished = true;
                                break;
                            }
                        }
                    }
                }
    } else {
#pragma unroll
        for (int q = 0; q < P; ++q) {
            if (!active[q]) continue;
            int bc[3] = {0, 0, 0};
#pragma unroll
            for (int c = 0; c < D; ++c) bc[c] = bin_of(p[q][c], c, S.g);
            const int64_t b = (int64_t(bc[2]) * S.g.nb[1] + bc[1]) * S.g.nb[0] + bc[0];
            const int64_t start = S.bin_ptr[b], end = S.bin_ptr[b + 1];
            for (int64_t c = start; c < end; ++c) {
                const int e = S.bin_elems[c];
                test_candidate<D>(S.rec + int64_t(e) * RS, e, p[q], best[q], bid[q]);
                if (best[q] > kInsideTau) break;
            }
        }
    }
}

// Barycentric coordinates of p in the located element (zeros if none).
template <int D>
__device__ __forceinline__ void winner_mu(const SrcView& S, int bid, const double (&p)[D], double (&mu)[D + 1]) {
    if (bid == INT_MAX) {
#pragma unroll
        for (int k = 0; k <= D; ++k) mu[k] = 0.0;
        return;
    }
    (void)barycentric<D>(S.rec + int64_t(bid) * RecSize<D>::value, p, mu);
}

// P1 value of field f at a located point (0 if no element was found).
template <int D>
__device__ __forceinline__ double p1_value(const SrcView& S, int bid, const double (&bmu)[D + 1], int f) {
    if (bid == INT_MAX) return 0.0;
    const double* Fv = S.values + int64_t(f) * S.n;
    double y = 0.0;
#pragma unroll
    for (int k = 0; k <= D; ++k) y = fma(bmu[k], Fv[S.conn[int64_t(bid) * (D + 1) + k]], y);
    return y;
}

}  // namespace ft
