// Device side of the mesh-backed P1 source: bin grid, barycentric records and
// the wave-cooperative localization (shared by the evaluation kernel and the
// fused sample-evaluate-consume kernel).
//
// Localization rule: the element maximizing min_k mu_k(x) (mu: barycentric
// coordinates); exact ties -> lowest element id; a best min mu below -1e-10
// is out of the domain (counted, extrapolated from that element).  A point
// whose best element has min mu > 1e-12 is strictly inside it: no other
// element can tie or win, and rounding (far below 1e-12) cannot change that.
//
// Search.  Every element is registered once, in the bin holding the centre
// of its box; with hx the largest half-extent of an element box per axis, the
// elements that can meet a region [lo, hi] are registered in the bins of
// [lo - hx, hi + hx].  The points of a wave (64 lanes x P points)
// are usually samples of one target element, so they share a handful of bins.
// The wave forms its points' bounding box and their ranges along a few more
// directions (x±y in 2D, x-y, y-z, x-z in 3D) and the bins that can hold candidates; lanes load
// those bins' ranges and a wave scan turns them into one flat candidate
// sequence (no element appears twice), culled 64 at a time, one per lane: the
// element's box and direction ranges must meet the wave's.  Only the
// survivors fetch the element's absolute affine barycentric form, and park it
// in the wave's LDS; every lane then tests its points against each survivor
// in lane order (broadcast LDS reads).  The selection test accepts an element
// once mu_1..mu_D and mu_0 = 1 - their sum all exceed the source's margin tau
// (1e-9, or more for meshes whose affine forms carry large terms: tau bounds
// the rounding of the form at any point of any element's box), so an
// accepted element truly contains the point and is the unique winner; a wave
// stops when all its points are accepted.  Points never accepted (within tau
// of a face, or outside) are re-searched alone with the full rule over the
// bins that can hold their elements; a point those bins leave outside the
// domain (or without any candidate) takes the full rule over every element,
// so the extrapolating element is the rule's winner however far out the
// point lies.  The barycentrics used to interpolate are always recomputed
// from the element origin.  Waves whose points need more than 64 bins
// (scattered input) search point by point.  Each wave brings its own LDS
// slots (kWaveSlots<D> doubles).
#pragma once

#include <cfloat>

#include "common.h"

namespace ft {

constexpr double kInsideTau = 1e-12;   // strictly inside (rule winner is unique)
constexpr double kFastTau = 1e-9;      // smallest margin of the fast selection test (absolute affine form)
// The margin a source uses: kFastTau, or kFastTauUlps units of rounding of the
// largest |c_k| + sum_c |g_kc x_c| over its elements' boxes when that is larger
// (the form's value at a point is off by at most a few such units).
constexpr double kFastTauUlps = 64.0 * 0x1p-53;
constexpr double kOutTol = -1e-10;

// Record of element e, rec[e*RS ...] (doubles; 128 B in 2D, 256 B in 3D):
//   [0, D)                    constants c_k of mu_k(x) = c_k + g_k . x, k = 1..D
//   [D, D + D*D)              gradients g_k (D each), k = 1..D: the rows of the
//                             inverse of J = [x1-x0 | ... | xd-x0]
//   [X0, X0 + D)              origin x0 (vertex 0), X0 = D + D*D
//   [VAL, VAL + D + 1)        vertex values of a one-field source (else zero)
// The first D(D+1) doubles, the absolute affine form of mu_1..mu_D, are what
// the cull parks in LDS (one aligned contiguous block; mu_0 = 1 - the others);
// the origin form mu_{k+1} = g_{k+1} . (x - x0) gives the barycentrics used to
// interpolate, and for one field the vertex values sit in the same record.
template <int D>
struct RecSize { static constexpr int value = D == 2 ? 16 : 32; };
template <int D>
struct RecForm { static constexpr int value = D * (D + 1); };   // parked doubles
template <int D>
struct RecX0 { static constexpr int value = D + D * D; };
template <int D>
struct RecValues { static constexpr int value = D + D * D + D; };
static_assert(RecValues<2>::value + 3 <= RecSize<2>::value, "2D record overflow");
static_assert(RecValues<3>::value + 4 <= RecSize<3>::value, "3D record overflow");

// Extra directions of the element and wave boxes: x+y and x-y in 2D (with the
// axes an octagon); x-y, y-z and x-z in 3D (the planes that split a hex into
// its six Kuhn tetrahedra).
template <int D>
struct Dirs {
    static constexpr int n = D == 2 ? 2 : 3;
    static __host__ __device__ __forceinline__ double proj(int k, const double* x) {
        if (D == 2) return k == 0 ? x[0] + x[1] : x[0] - x[1];
        return k == 0 ? x[0] - x[1] : (k == 1 ? x[1] - x[2] : x[0] - x[2]);
    }
};

// floats per element in the box array, outward-rounded:
// [min per axis | max per axis | min per direction | max per direction]
template <int D>
struct BoxSize { static constexpr int value = 2 * D + 2 * Dirs<D>::n; };

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
    double hx[3];   // largest half-extent of an element's box, per axis (slightly enlarged)
};

// Bin index along axis c; monotone in x, so a point inside a box always maps
// into the box's bin range.  NaN maps to bin 0.
__device__ __forceinline__ int bin_of(double x, int c, const GridView& g) {
    double u = (x - g.lo[c]) * g.inv_h[c];
    u = fmin(fmax(u, 0.0), double(g.nb[c] - 1));
    return int(u);
}

struct SrcView {
    const double* rec;
    const float* box;
    const int32_t* conn;
    const double* values;      // [F][n]
    const double* values_nm;   // [n][F] (F > 1)
    const int64_t* bin_ptr;
    const int32_t* bin_elems;
    int64_t n;
    int F;
    GridView g;
    int64_t E;        // elements (the whole-mesh search for points outside the domain)
    double tau;       // margin of the fast selection test (>= kFastTau)
    int32_t rec_values;   // 1: the (one) field's vertex values sit in the element records
};

// Barycentric coordinates of p in the element of record r (origin x0 and the
// inverse Jacobian A): mu_{k+1} = A[k] . (p - x0), mu_0 = 1 - sum.  Returns min mu.
template <int D>
__device__ __forceinline__ double barycentric(const double* __restrict__ r, const double (&p)[D],
                                              double (&mu)[D + 1]) {
    double d[D];
#pragma unroll
    for (int c = 0; c < D; ++c) d[c] = p[c] - r[RecX0<D>::value + c];
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

// Full rule (max of min mu, ties to the lowest id), absolute coordinates.
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

// Fast selection test from a parked form in LDS (wave-uniform address: a
// broadcast read).  The form holds the constants of mu_1..mu_D, then their
// gradients (mu_0 = 1 - sum of the others): true when every mu_k exceeds
// tau at p, i.e. p lies inside the element with that margin.
template <int D>
__device__ __forceinline__ bool inside_lds(const double* af, const double (&p)[D], double tau) {
    bool in = true;
    double s;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        double l = af[k];
#pragma unroll
        for (int c = 0; c < D; ++c) l = fma(af[D + k * D + c], p[c], l);
        in &= l > tau;
        s = k == 0 ? l : s + l;
    }
    return in & (s < 1.0 - tau);
}

// Own-bin search of one point with the full rule (absolute coordinates).
template <int D>
__device__ __forceinline__ void locate_point(const SrcView& S, const double (&p)[D], double& best, int& bid) {
    constexpr int RS = RecSize<D>::value;
    int hi[3] = {0, 0, 0}, lo[3] = {0, 0, 0};
#pragma unroll
    for (int c = 0; c < D; ++c) {
        lo[c] = bin_of(p[c] - S.g.hx[c], c, S.g);
        hi[c] = bin_of(p[c] + S.g.hx[c], c, S.g);
    }
    best = -DBL_MAX;
    bid = INT_MAX;
    // an element whose box holds p has its box centre within hx of p
    for (int bz = lo[2]; bz <= hi[2]; ++bz)
        for (int by = lo[1]; by <= hi[1]; ++by)
            for (int bx = lo[0]; bx <= hi[0]; ++bx) {
                const int64_t b = (int64_t(bz) * S.g.nb[1] + by) * S.g.nb[0] + bx;
                const int64_t start = S.bin_ptr[b], end = S.bin_ptr[b + 1];
                for (int64_t c = start; c < end; ++c) {
                    const int e = S.bin_elems[c];
                    test_candidate<D>(S.rec + int64_t(e) * RS, e, p, best, bid);
                    if (best > kInsideTau) return;   // strictly inside: the unique winner
                }
            }
    // outside the domain, or no candidate at all: the bins near p need not hold
    // the rule's winner (for a point outside the mesh the maximizer of min mu
    // can be any element), so every element is tested, in id order
    if (bid == INT_MAX || best < kOutTol) {
        best = -DBL_MAX;
        bid = INT_MAX;
        for (int64_t e = 0; e < S.E; ++e) test_candidate<D>(S.rec + e * RS, int(e), p, best, bid);
    }
}

// LDS slots for the candidates' parked forms: 64 per wave, D(D+1) doubles
// each, then 64 ints of slot marks (see locate_wave).  Every kernel that
// localizes declares its block's slots (waves per block x kWaveSlots<D>
// doubles) and hands each wave its own part.
template <int D>
constexpr int kWaveSlots = 64 * D * (D + 1) + 32;

// Inclusive prefix sum over the 64 lanes of the wave: a scan inside each row
// of 16 lanes on the DPP crossbar (shifts by 1, 2, 4, 8; lanes shifted in
// from outside the row read zero), then the totals of the rows below.
template <int CTRL>
__device__ __forceinline__ int dpp_shr_zero(int x) {
    return __builtin_amdgcn_update_dpp(0, x, CTRL, 0xF, 0xF, true);
}

// Inclusive prefix maximum over the 64 lanes of non-negative values (same
// row-then-rows structure as the scan below).
__device__ __forceinline__ int wave_prefix_max(int x);

__device__ __forceinline__ int wave_scan_incl(int x) {
    const int lane = threadIdx.x & 63;
    x += dpp_shr_zero<0x111>(x);   // row_shr:1
    x += dpp_shr_zero<0x112>(x);   // row_shr:2
    x += dpp_shr_zero<0x114>(x);   // row_shr:4
    x += dpp_shr_zero<0x118>(x);   // row_shr:8
    const int r0 = __builtin_amdgcn_readlane(x, 15), r1 = __builtin_amdgcn_readlane(x, 31),
              r2 = __builtin_amdgcn_readlane(x, 47);
    return x + (lane >= 16 ? r0 : 0) + (lane >= 32 ? r1 : 0) + (lane >= 48 ? r2 : 0);
}

__device__ __forceinline__ int wave_prefix_max(int x) {
    const int lane = threadIdx.x & 63;
    x = max(x, dpp_shr_zero<0x111>(x));   // lanes shifted in from outside the row read zero
    x = max(x, dpp_shr_zero<0x112>(x));
    x = max(x, dpp_shr_zero<0x114>(x));
    x = max(x, dpp_shr_zero<0x118>(x));
    const int r0 = __builtin_amdgcn_readlane(x, 15), r1 = __builtin_amdgcn_readlane(x, 31),
              r2 = __builtin_amdgcn_readlane(x, 47);
    int c = lane >= 16 ? r0 : 0;
    c = lane >= 32 ? max(c, r1) : c;
    c = lane >= 48 ? max(c, r2) : c;
    return max(x, c);
}

// Rule winner for each of this lane's P points (see the file comment).  Every
// lane of the wave must call it (points a lane does not own pass
// active = false).  Returns bid = the winner's element id (INT_MAX only for
// inactive points) and best: 1 for points the fast test accepted (inside
// their element with margin S.tau), the full rule's max min-barycentric for
// the others.
template <int D, int P>
__device__ __forceinline__ void locate_wave(const SrcView& S, const double (&p)[P][D], const bool (&active)[P],
                                            double (&best)[P], int (&bid)[P], double* __restrict__ c_af) {
    constexpr int RS = RecSize<D>::value;
    constexpr int BS = BoxSize<D>::value;
    constexpr int MAX_SPAN = 64;   // bins a wave searches as one flat sequence (one per lane)
    const int lane = threadIdx.x & 63;
    // the wave's box, rounded outward to binary32 (DPP reductions, no LDS)
    double wlo[D], whi[D];
    float flo[D], fhi[D];
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
        flo[c] = wave_min_f32(f32_down(lo));
        fhi[c] = wave_max_f32(f32_up(hi));
        wlo[c] = flo[c];
        whi[c] = fhi[c];
        // elements meeting the wave's box have their box centre within hx of it
        b0[c] = uniform_int(bin_of(wlo[c] - S.g.hx[c], c, S.g));
        b1[c] = uniform_int(bin_of(whi[c] + S.g.hx[c], c, S.g));
        span *= b1[c] - b0[c] + 1;
    }
#pragma unroll
    for (int q = 0; q < P; ++q) {
        best[q] = -DBL_MAX;
        bid[q] = INT_MAX;
    }

    if (span <= MAX_SPAN) {
        // during the fast search bid[q] != INT_MAX marks an accepted point; inactive
        // points start marked (-1), so the wave's exit test needs no activity mask
#pragma unroll
        for (int q = 0; q < P; ++q) bid[q] = active[q] ? INT_MAX : -1;
        constexpr int ND = Dirs<D>::n;
        float fdlo[ND], fdhi[ND];   // wave ranges along the extra directions
#pragma unroll
        for (int k = 0; k < ND; ++k) {
            double lo = INFINITY, hi = -INFINITY;
#pragma unroll
            for (int q = 0; q < P; ++q)
                if (active[q]) {
                    const double u = Dirs<D>::proj(k, p[q]);
                    lo = fmin(lo, u);
                    hi = fmax(hi, u);
                }
            fdlo[k] = wave_min_f32(f32_down(lo));
            fdhi[k] = wave_max_f32(f32_up(hi));
        }
        // Lane i < span describes bin i of the wave's bin box (x fastest): its
        // coordinates, first registration and count.  The candidate slots of all
        // these bins are then culled 64 at a time in one flat sequence.
        constexpr int AL = RecForm<D>::value;   // parked form: constants of mu_1..mu_D, then D x D gradients
        const int wx = b1[0] - b0[0] + 1, wy = b1[1] - b0[1] + 1;
        int64_t bstart = 0;
        int bcnt = 0;
        if (lane < span) {
            const int cx = b0[0] + lane % wx, cy = b0[1] + (lane / wx) % wy, cz = b0[2] + lane / (wx * wy);
            const int64_t b = (int64_t(cz) * S.g.nb[1] + cy) * S.g.nb[0] + cx;
            bstart = S.bin_ptr[b];
            bcnt = int(S.bin_ptr[b + 1] - bstart);
        }
        const int incl = wave_scan_incl(bcnt);
        const int excl = incl - bcnt;
        const int total = __builtin_amdgcn_readlane(incl, span - 1);
        int* mark = reinterpret_cast<int*>(c_af + 64 * AL);   // 64 slot marks
        bool finished = false;
        for (int c0 = 0; c0 < total && !finished; c0 += 64) {
            const int sl = c0 + lane;
            // bin of slot sl: every non-empty bin marks (lane + 1) the first slot
            // of this chunk it fills, the bin running in from the previous chunk
            // marks slot 0, and a prefix maximum carries the marks forward
            mark[lane] = 0;
            __builtin_amdgcn_wave_barrier();
            if (lane < span && bcnt > 0 && excl >= c0 && excl < c0 + 64) mark[excl - c0] = lane + 1;
            const uint64_t run_in = __builtin_amdgcn_ballot_w64(lane < span && excl < c0 && incl > c0);
            // lanes read marks other lanes wrote: the wavefront-scope fences keep the
            // compiler from forwarding a lane's own store of 0 to its load
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            int m = mark[lane];
            if (lane == 0 && run_in) m = max(m, int(__ffsll((unsigned long long)run_in)));
            m = wave_prefix_max(m);
            const int i = m > 0 ? m - 1 : 0;
            const int excl_i = __shfl(excl, i, 64);
            const int cnt_i = __shfl(bcnt, i, 64);
            const int64_t st_i = __shfl((long long)bstart, i, 64);
            int cid = -1;
            bool ov = false;
            // (the slot lies in its bin's range by construction; the range test only
            // guards the load)
            if (sl < total && unsigned(sl - excl_i) < unsigned(cnt_i)) {
                cid = S.bin_elems[st_i + (sl - excl_i)];
                const float* bx_ = S.box + int64_t(cid) * BS;
                ov = true;
#pragma unroll
                for (int c = 0; c < D; ++c) ov &= (bx_[c] <= fhi[c]) & (bx_[D + c] >= flo[c]);
#pragma unroll
                for (int k = 0; k < ND; ++k) ov &= (bx_[2 * D + k] <= fdhi[k]) & (bx_[2 * D + ND + k] >= fdlo[k]);
            }
            // only the survivors (a small fraction of the slots) fetch their affine
            // form (mu_1..mu_D) and park it in their own LDS slot; they are then
            // read back in lane order
            if (ov) {
                const double* r = S.rec + int64_t(cid) * RS;
#pragma unroll
                for (int m = 0; m < AL; ++m) c_af[lane * AL + m] = r[m];
            }
            uint64_t mask = __ballot(ov);
            __builtin_amdgcn_wave_barrier();
            while (mask) {
                const int l1 = __ffsll((unsigned long long)mask) - 1;
                mask &= mask - 1;
                const int e1 = read_lane(cid, l1);
                const double* a1 = &c_af[l1 * AL];
                uint64_t pending = 0;   // lanes with a point not yet accepted
#pragma unroll
                for (int q = 0; q < P; ++q) {
                    const bool in = inside_lds<D>(a1, p[q], S.tau);
                    bid[q] = in ? e1 : bid[q];
                    pending |= __builtin_amdgcn_ballot_w64(bid[q] == INT_MAX);
                }
                if (pending == 0) {
                    finished = true;
                    break;
                }
            }
            __builtin_amdgcn_wave_barrier();
        }
        // accepted points lie inside their element with margin tau; the others
        // (near a face, or outside) take the full rule over the bins that can hold
        // their elements
#pragma unroll
        for (int q = 0; q < P; ++q) {
            if (!active[q]) bid[q] = INT_MAX;
            else if (bid[q] != INT_MAX) best[q] = 1.0;
            else locate_point<D>(S, p[q], best[q], bid[q]);
        }
    } else {
#pragma unroll
        for (int q = 0; q < P; ++q)
            if (active[q]) locate_point<D>(S, p[q], best[q], bid[q]);
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
    double y = 0.0;
    if (S.rec_values) {   // vertex values in the element's record
        const double* rv = S.rec + int64_t(bid) * RecSize<D>::value + RecValues<D>::value;
#pragma unroll
        for (int k = 0; k <= D; ++k) y = fma(bmu[k], rv[k], y);
        return y;
    }
    const double* Fv = S.values + int64_t(f) * S.n;
#pragma unroll
    for (int k = 0; k <= D; ++k) y = fma(bmu[k], Fv[S.conn[int64_t(bid) * (D + 1) + k]], y);
    return y;
}

// Localize and evaluate the points [base, min(base + 64P, lim)) of a (d, ld)
// point array: lane l takes points base + q*64 + l.  Writes values (and ids
// if non-null) and returns this lane's count of out-of-domain points.
// ROUND (binary64 points and values): the points are rounded to binary32
// before the search and the values to binary32 when stored, as the binary32
// form's query list holds them.
template <int D, int P, bool IN_F32, bool OUT_F32, bool ROUND = false>
__device__ __forceinline__ unsigned eval_wave(const SrcView& S, int64_t base, int64_t lim,
                                              const void* __restrict__ pts_, int64_t ld, void* __restrict__ out_,
                                              int64_t ld_out, int32_t* __restrict__ ids, double* __restrict__ c_af) {
    const int lane = threadIdx.x & 63;
    double p[P][D];
    bool active[P];
#pragma unroll
    for (int q = 0; q < P; ++q) {
        const int64_t i = base + q * 64 + lane;
        active[q] = i < lim;
#pragma unroll
        for (int c = 0; c < D; ++c) {
            if (IN_F32)
                p[q][c] = active[q] ? double(static_cast<const float*>(pts_)[c * ld + i]) : 0.0;
            else if (ROUND)
                p[q][c] = active[q] ? double(float(static_cast<const double*>(pts_)[c * ld + i])) : 0.0;
            else
                p[q][c] = active[q] ? static_cast<const double*>(pts_)[c * ld + i] : 0.0;
        }
    }
    double best[P];
    int bid[P];
    locate_wave<D, P>(S, p, active, best, bid, c_af);
    unsigned int nood = 0;
#pragma unroll
    for (int q = 0; q < P; ++q) {
        if (!active[q]) continue;
        const int64_t i = base + q * 64 + lane;
        const bool found = bid[q] != INT_MAX;
        nood += !found || best[q] < kOutTol;
        if (ids) ids[i] = found ? bid[q] : -1;
        if (!out_) continue;   // localization only
        double mu[D + 1];
        winner_mu<D>(S, bid[q], p[q], mu);
        if (S.F == 1) {
            double y = p1_value<D>(S, bid[q], mu, 0);
            if (ROUND) y = double(float(y));
            if (OUT_F32)
                static_cast<float*>(out_)[i] = float(y);
            else
                static_cast<double*>(out_)[i] = y;
            continue;
        }
        // several fields (the evaluation kernel hands these to its lanes-over-fields
        // variant): the element's vertices once, then one gather per vertex and field
        int vk[D + 1];
#pragma unroll
        for (int k = 0; k <= D; ++k) vk[k] = found ? S.conn[int64_t(bid[q]) * (D + 1) + k] : 0;
#pragma unroll 4
        for (int f = 0; f < S.F; ++f) {
            const double* Fv = S.values + int64_t(f) * S.n;
            double y = 0.0;
            if (found)
#pragma unroll
                for (int k = 0; k <= D; ++k) y = fma(mu[k], Fv[vk[k]], y);
            if (ROUND) y = double(float(y));
            if (OUT_F32)
                static_cast<float*>(out_)[int64_t(f) * ld_out + i] = float(y);
            else
                static_cast<double*>(out_)[int64_t(f) * ld_out + i] = y;
        }
    }
    return nood;
}

}  // namespace ft
