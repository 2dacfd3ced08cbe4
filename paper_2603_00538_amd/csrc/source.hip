// Built-in P1 source: uniform-grid point localization and P1 evaluation.
//
// Benchmarks need a source that can only be queried at points (sec. 2, the
// black-box setting); here it is a P1 field on a source mesh, localized with
// a uniform grid of bins as in sec. 5.3 (int(L sqrt(#elements)) cells per
// axis by default).
//
// Localization rule and search: see locate.h.
//
// Layout: every source element e has a record rec[e*RS ...] holding its
// barycentric map (absolute affine form of mu_1..mu_D, whose gradients are the
// rows of the inverse of J = [x1-x0 | ... | xd-x0]), its origin and, for one
// field, its vertex values (see locate.h); plus outward-rounded binary32
// ranges along the axes and a few extra directions (its box).  Each element
// is registered once, in the bin holding the centre of its box (CSR, ascending
// ids per bin); the largest half-extent of a box tells a search how far
// around a region to look.  A source of several fields also keeps a
// node-major copy of its nodal values for the many-field evaluation.

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstring>
#include <type_traits>
#include <vector>

#include "locate.h"
#include "solve_common.h"

namespace ft {

template <int D>
__global__ void k_src_geom(const double* __restrict__ X, int64_t n, const int32_t* __restrict__ conn, int64_t E,
                           const double* __restrict__ values, int F, double* __restrict__ rec,
                           float* __restrict__ box, unsigned long long* __restrict__ flags) {
    constexpr int RS = RecSize<D>::value;
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= E) return;
    int v[D + 1];
    bool bad = false;
#pragma unroll
    for (int k = 0; k <= D; ++k) {
        v[k] = conn[e * (D + 1) + k];
        bad |= (v[k] < 0) | (int64_t(v[k]) >= n);
    }
    if (bad) {
        atomicAdd(&flags[0], 1ull);
        return;
    }
    double x[D + 1][D];
#pragma unroll
    for (int k = 0; k <= D; ++k)
#pragma unroll
        for (int c = 0; c < D; ++c) x[k][c] = X[c * n + v[k]];
    double J[D][D];   // J[c][k] = x_{k+1,c} - x_{0,c}
#pragma unroll
    for (int c = 0; c < D; ++c)
#pragma unroll
        for (int k = 0; k < D; ++k) J[c][k] = x[k + 1][c] - x[0][c];
    double A[D][D], det;
    if constexpr (D == 2) {
        det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
        A[0][0] = J[1][1] / det;
        A[0][1] = -J[0][1] / det;
        A[1][0] = -J[1][0] / det;
        A[1][1] = J[0][0] / det;
    } else {
        const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
        const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
        const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
        det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
        // inverse = adjugate / det (rows of A index the barycentric coordinate)
        A[0][0] = c00 / det;
        A[1][0] = c01 / det;
        A[2][0] = c02 / det;
        A[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
        A[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
        A[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
        A[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
        A[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
        A[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
    }
    double h2 = 0.0;
#pragma unroll
    for (int a = 0; a <= D; ++a)
#pragma unroll
        for (int b = a + 1; b <= D; ++b) {
            double s = 0.0;
#pragma unroll
            for (int c = 0; c < D; ++c) s += (x[b][c] - x[a][c]) * (x[b][c] - x[a][c]);
            h2 = fmax(h2, s);
        }
    const double hd = D == 2 ? h2 : h2 * sqrt(h2);
    if (!(fabs(det) > 1e-12 * hd)) atomicAdd(&flags[1], 1ull);
    double* r = rec + e * RS;
#pragma unroll
    for (int i = 0; i < RS; ++i) r[i] = 0.0;
#pragma unroll
    for (int c = 0; c < D; ++c) r[RecX0<D>::value + c] = x[0][c];
    // absolute affine form of mu_1..mu_D: g_{k+1} = A[k], c_{k+1} = -A[k] . x0
#pragma unroll
    for (int k = 0; k < D; ++k) {
        double ck = 0.0;
#pragma unroll
        for (int c = 0; c < D; ++c) {
            ck = fma(-A[k][c], x[0][c], ck);
            r[D + k * D + c] = A[k][c];
        }
        r[k] = ck;
    }
    if (F == 1)
#pragma unroll
        for (int k = 0; k <= D; ++k) r[RecValues<D>::value + k] = values[v[k]];
    constexpr int BS = BoxSize<D>::value;
    double xmax[D];   // largest |x_c| over the element's box
#pragma unroll
    for (int c = 0; c < D; ++c) {
        double lo = x[0][c], hi = x[0][c];
#pragma unroll
        for (int k = 1; k <= D; ++k) {
            lo = fmin(lo, x[k][c]);
            hi = fmax(hi, x[k][c]);
        }
        box[e * BS + c] = f32_down(lo);
        box[e * BS + D + c] = f32_up(hi);
        xmax[c] = fmax(fabs(lo), fabs(hi));
    }
    // largest term magnitude |c_k| + sum_c |g_kc x_c| of the absolute affine form
    // over the box: it scales the rounding of the fast selection test
    double mag = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        double m = fabs(r[k]);
#pragma unroll
        for (int c = 0; c < D; ++c) m = fma(fabs(r[D + k * D + c]), xmax[c], m);
        mag = fmax(mag, m);
    }
    atomicMax(&flags[2], (unsigned long long)__double_as_longlong(mag));
    constexpr int ND = Dirs<D>::n;
#pragma unroll
    for (int k = 0; k < ND; ++k) {
        double lo = INFINITY, hi = -INFINITY;
#pragma unroll
        for (int j = 0; j <= D; ++j) {
            const double u = Dirs<D>::proj(k, x[j]);
            lo = fmin(lo, u);
            hi = fmax(hi, u);
        }
        box[e * BS + 2 * D + k] = f32_down(lo);
        box[e * BS + 2 * D + ND + k] = f32_up(hi);
    }
}

// Each element is registered once, in the bin of its box centre; the count
// pass also records the largest half-extent of a box per axis (as the bits of
// a non-negative double, whose integer order is the numeric order).
template <int D, bool FILL>
__global__ void k_src_register(const double* __restrict__ X, int64_t n, const int32_t* __restrict__ conn, int64_t E,
                               GridView g, int32_t* __restrict__ cnt, const int64_t* __restrict__ ptr,
                               int32_t* __restrict__ elems, unsigned long long* __restrict__ hx) {
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= E) return;
    int bc[3] = {0, 0, 0};
#pragma unroll
    for (int c = 0; c < D; ++c) {
        double lo = INFINITY, hi = -INFINITY;
#pragma unroll
        for (int k = 0; k <= D; ++k) {
            const double xv = X[c * n + conn[e * (D + 1) + k]];
            lo = fmin(lo, xv);
            hi = fmax(hi, xv);
        }
        bc[c] = bin_of(0.5 * (lo + hi), c, g);
        if (!FILL) atomicMax(&hx[c], __double_as_longlong(0.5 * (hi - lo)));
    }
    const int64_t b = (int64_t(bc[2]) * g.nb[1] + bc[1]) * g.nb[0] + bc[0];
    if (!FILL) {
        atomicAdd(&cnt[b], 1);
    } else {
        const int pos = atomicAdd(&cnt[b], 1);
        elems[ptr[b] + pos] = int32_t(e);
    }
}

__global__ void k_minmax(const double* __restrict__ X, int64_t n, int dim, double* __restrict__ out) {
    // out[(blockIdx.x * dim + c) * 2 + {0,1}] = block min / max of coordinate c
    __shared__ double smin[256], smax[256];
    for (int c = 0; c < dim; ++c) {
        double lo = INFINITY, hi = -INFINITY;
        for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
            lo = fmin(lo, X[c * n + i]);
            hi = fmax(hi, X[c * n + i]);
        }
        smin[threadIdx.x] = lo;
        smax[threadIdx.x] = hi;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if (threadIdx.x < o) {
                smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + o]);
                smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + o]);
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            out[(blockIdx.x * dim + c) * 2 + 0] = smin[0];
            out[(blockIdx.x * dim + c) * 2 + 1] = smax[0];
        }
        __syncthreads();
    }
}

__global__ void k_sort_bins(const int64_t* __restrict__ ptr, int64_t nseg, int32_t* __restrict__ data) {
    const int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (s >= nseg) return;
    int32_t* a = data + ptr[s];
    const int64_t len = ptr[s + 1] - ptr[s];
    for (int64_t i = 1; i < len; ++i) {
        const int32_t x = a[i];
        int64_t j = i - 1;
        while (j >= 0 && a[j] > x) {
            a[j + 1] = a[j];
            --j;
        }
        a[j + 1] = x;
    }
}

// Each wave owns 64*P consecutive points; lane l holds points base + q*64 + l.
// WPB waves per block, each with its own LDS candidate slots: small blocks
// release their slots as soon as their waves end (waves of a block finish at
// very different times: early exit, fallback searches).
template <int D, int P, bool IN_F32, bool OUT_F32, int WPB>
__global__ __launch_bounds__(64 * WPB) void k_src_eval(SrcView S, int64_t head, int64_t npts,
                                                       const void* __restrict__ pts_, int64_t ld,
                                                       void* __restrict__ out_, int64_t ld_out,
                                                       int32_t* __restrict__ ids,
                                                       unsigned long long* __restrict__ n_ood) {
    __shared__ double lds[WPB * kWaveSlots<D>];
    const int wv = WPB == 1 ? 0 : int(threadIdx.x >> 6);
    // two segments, [0, head) and [head, npts), each starting on a wavefront boundary
    constexpr int64_t WP = 64 * P;
    const int64_t wave = int64_t(blockIdx.x) * WPB + wv;
    const int64_t wh = (head + WP - 1) / WP;
    const int64_t base = wave < wh ? wave * WP : head + (wave - wh) * WP;
    const int64_t lim = wave < wh ? head : npts;
    if (base >= lim) return;   // wave-uniform
    const unsigned nood =
        eval_wave<D, P, IN_F32, OUT_F32>(S, base, lim, pts_, ld, out_, ld_out, ids, lds + wv * kWaveSlots<D>);
    if (nood) atomicAdd(n_ood, (unsigned long long)nood);
}

// Node-major copy of the nodal values: out[v * F + f] = values[f * n + v].
__global__ void k_node_major(const double* __restrict__ values, int64_t n, int F, double* __restrict__ out) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n * F; i += int64_t(gridDim.x) * blockDim.x) {
        const int64_t v = i / F;
        const int f = int(i - v * F);
        out[i] = values[int64_t(f) * n + v];
    }
}

// Many fields (F > 1): localization as k_src_eval, then the interpolation with
// the lanes over fields.  Each lane parks its points' winner barycentrics and
// vertices in LDS; for a block of 16 fields, four points at a time are
// evaluated by 16 lanes each (lane = field), reading a vertex's 16 field
// values as one 128-byte row of the node-major copy; the values collect in an
// LDS tile [16 fields][64 points] and leave as 16 coalesced row stores.
constexpr int kManyFB = 16;   // fields per block
constexpr int kManyU = 8;     // points per lane whose gathers are issued together

template <int D, int P, bool OUT_F32>
struct ManyLds {
    using T = typename std::conditional<OUT_F32, float, double>::type;
    static constexpr int kStashBytes = 64 * P * (D + 1) * 12;   // (mu double, vertex int) per point and vertex
    static constexpr int kSlotBytes = kWaveSlots<D> * 8;
    static constexpr int kRegionA = kStashBytes > kSlotBytes ? kStashBytes : kSlotBytes;
    static constexpr int kTileBytes = kManyFB * 65 * int(sizeof(T));
    static constexpr int kBytes = kRegionA + kTileBytes;
};

template <int D, int P, bool IN_F32, bool OUT_F32>
__global__ __launch_bounds__(64) void k_src_eval_many(SrcView S, int64_t head, int64_t npts,
                                                      const void* __restrict__ pts_, int64_t ld,
                                                      void* __restrict__ out_, ValueLayout VL,
                                                      int32_t* __restrict__ ids,
                                                      unsigned long long* __restrict__ n_ood) {
    using L = ManyLds<D, P, OUT_F32>;
    using T = typename L::T;
    __shared__ __align__(16) unsigned char lds[L::kBytes];
    double* c_af = reinterpret_cast<double*>(lds);
    double* st_mu = reinterpret_cast<double*>(lds);                                  // [64P][D+1]
    int* st_v = reinterpret_cast<int*>(lds + 64 * P * (D + 1) * 8);                   // [64P][D+1]
    T* tile = reinterpret_cast<T*>(lds + L::kRegionA);                                 // [16][65]
    constexpr int64_t WP = 64 * P;
    const int lane = int(threadIdx.x & 63);
    const int64_t wave = int64_t(blockIdx.x);
    const int64_t wh = (head + WP - 1) / WP;
    const int64_t base = wave < wh ? wave * WP : head + (wave - wh) * WP;
    const int64_t lim = wave < wh ? head : npts;
    if (base >= lim) return;   // wave-uniform
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
            else
                p[q][c] = active[q] ? static_cast<const double*>(pts_)[c * ld + i] : 0.0;
        }
    }
    double best[P];
    int bid[P];
    locate_wave<D, P>(S, p, active, best, bid, c_af);
    unsigned nood = 0;
    __builtin_amdgcn_wave_barrier();   // the candidate slots become the stash
#pragma unroll
    for (int q = 0; q < P; ++q) {
        const int64_t i = base + q * 64 + lane;
        const bool found = active[q] && bid[q] != INT_MAX;
        if (active[q]) {
            nood += !found || best[q] < kOutTol;
            if (ids) ids[i] = found ? bid[q] : -1;
        }
        double mu[D + 1];
        winner_mu<D>(S, found ? bid[q] : INT_MAX, p[q], mu);
        const int slot = q * 64 + lane;
#pragma unroll
        for (int k = 0; k <= D; ++k) {
            st_mu[slot * (D + 1) + k] = mu[k];   // zero weights for missing / inactive points
            st_v[slot * (D + 1) + k] = found ? S.conn[int64_t(bid[q]) * (D + 1) + k] : 0;
        }
    }
    __builtin_amdgcn_wave_barrier();
    const int fl = lane & (kManyFB - 1);   // field within the block
    const int pg = lane >> 4;              // point within a group of four
    for (int q = 0; q < P; ++q) {
        const int64_t i0 = base + q * 64;
        // this lane's point in the output: field 0 at a_base, fields a_fs apart
        const int64_t iq = i0 + lane;
        int64_t a_base = iq, a_fs = VL.node_ld;
        if (iq >= head) {
            const int64_t sq = iq - head;
            int64_t te = sq, je = 0;
            if (VL.ndiv.d != 1) {
                te = int64_t(fast_div(uint32_t(sq), VL.ndiv));
                je = sq - te * int64_t(VL.ndiv.d);
            }
            a_base = VL.samp0 + te * VL.samp_elem + je;
            a_fs = VL.samp_fld;
        }
        for (int f0 = 0; f0 < S.F; f0 += kManyFB) {
            // a field past F reads field 0 (a valid address); its values are never stored
            const int f = f0 + fl < S.F ? f0 + fl : 0;
            // eight points' vertex values in flight before the first is used: the
            // gathers hit the caches, and their latency, not their bytes, sets the pace
            for (int h = 0; h < 16; h += kManyU) {
                double v[kManyU][D + 1];
#pragma unroll
                for (int u = 0; u < kManyU; ++u) {
                    const int slot = q * 64 + (h + u) * 4 + pg;
#pragma unroll
                    for (int k = 0; k <= D; ++k)
                        v[u][k] = S.values_nm[int64_t(st_v[slot * (D + 1) + k]) * S.F + f];
                }
#pragma unroll
                for (int u = 0; u < kManyU; ++u) {
                    const int j = (h + u) * 4 + pg;   // point of this slot
                    const int slot = q * 64 + j;
                    double y = 0.0;
#pragma unroll
                    for (int k = 0; k <= D; ++k) y = fma(st_mu[slot * (D + 1) + k], v[u][k], y);
                    tile[fl * 65 + j] = T(y);
                }
            }
            __builtin_amdgcn_wave_barrier();
            const int64_t i = i0 + lane;
            if (i < lim) {
                for (int r = 0; r < kManyFB && f0 + r < S.F; ++r)
                    // streamed past the caches: the values are read by a later launch,
                    // and the vertex rows of the gathers keep the level-2 cache
                    __builtin_nontemporal_store(tile[r * 65 + lane], static_cast<T*>(out_) + a_base + int64_t(f0 + r) * a_fs);
            }
            __builtin_amdgcn_wave_barrier();
        }
    }
    if (nood) atomicAdd(n_ood, (unsigned long long)nood);
}

// ---------------------------------------------------------------- host side
// (Re)build the bin grid: nb[c] > 0 fixes the cells on axis c; otherwise the
// longest axis gets `per_axis` cells and the others proportionally fewer.
template <int D>
static ft_status build_bins(ft_source* S, const int32_t (&nb_in)[3], double per_axis, hipStream_t s) {
    constexpr int B = 256;
    const int64_t n = S->n, E = S->E;
    dev_free(S->bin_ptr);
    dev_free(S->bin_elems);
    S->bin_ptr = nullptr;
    S->bin_elems = nullptr;
    double ext_max = 0.0;
    for (int c = 0; c < D; ++c) ext_max = std::fmax(ext_max, S->dom_hi[c] - S->dom_lo[c]);
    int64_t nbins = 1;
    for (int c = 0; c < 3; ++c) {
        S->nb[c] = 1;
        S->lo[c] = 0.0;
        S->inv_h[c] = 0.0;
    }
    for (int c = 0; c < D; ++c) {
        const double ext = S->dom_hi[c] - S->dom_lo[c];
        int32_t nb = nb_in[c];
        if (nb <= 0) nb = int32_t(std::max(1.0, std::ceil(per_axis * (ext_max > 0 ? ext / ext_max : 1.0) - 1e-9)));
        S->nb[c] = nb;
        S->lo[c] = S->dom_lo[c];
        S->inv_h[c] = ext > 0 ? double(nb) / ext : 0.0;
        nbins *= nb;
    }
    if (nbins > (int64_t(1) << 30)) {
        set_error("bin grid of %lld cells is too large", (long long)nbins);
        return FT_E_ARG;
    }
    GridView g{};
    for (int c = 0; c < 3; ++c) {
        g.nb[c] = S->nb[c];
        g.lo[c] = S->lo[c];
        g.inv_h[c] = S->inv_h[c];
    }
    int32_t* cnt = nullptr;
    unsigned long long* hxb = nullptr;
    int64_t* tmp = nullptr;
    ScratchGuard guard;
    guard.add((void**)&cnt);
    guard.add((void**)&hxb);
    guard.add((void**)&tmp);
    FT_TRY(dev_alloc_n(&cnt, size_t(nbins)));
    FT_TRY(dev_alloc_n(&tmp, size_t(scan_tmp_elems(nbins))));
    FT_TRY(dev_alloc_n(&S->bin_ptr, size_t(nbins + 1)));
    FT_TRY_HIP(hipMemsetAsync(cnt, 0, sizeof(int32_t) * nbins, s));
    FT_TRY(dev_alloc_n(&hxb, 3));
    FT_TRY_HIP(hipMemsetAsync(hxb, 0, sizeof(unsigned long long) * 3, s));
    k_src_register<D, false><<<grid_for(E, B), B, 0, s>>>(S->coords, n, S->conn, E, g, cnt, nullptr, nullptr, hxb);
    FT_TRY(exclusive_scan(cnt, S->bin_ptr, nbins, tmp, s));
    int64_t nreg = 0;
    unsigned long long hbits[3] = {0, 0, 0};
    FT_TRY_HIP(hipMemcpyAsync(&nreg, S->bin_ptr + nbins, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    FT_TRY_HIP(hipMemcpyAsync(hbits, hxb, sizeof(hbits), hipMemcpyDeviceToHost, s));
    FT_TRY_HIP(hipStreamSynchronize(s));
    S->n_reg = nreg;
    for (int c = 0; c < 3; ++c) {
        double h = 0.0;
        std::memcpy(&h, &hbits[c], sizeof(h));
        // enlarged so that rounding of box centres and of the search bounds cannot drop an element
        S->hx[c] = c < D ? h * (1.0 + 1e-9) + 1e-300 : 0.0;
    }
    FT_TRY(dev_alloc_n(&S->bin_elems, size_t(nreg)));
    FT_TRY_HIP(hipMemsetAsync(cnt, 0, sizeof(int32_t) * nbins, s));
    k_src_register<D, true><<<grid_for(E, B), B, 0, s>>>(S->coords, n, S->conn, E, g, cnt, S->bin_ptr, S->bin_elems,
                                                          nullptr);
    k_sort_bins<<<grid_for(nbins, B), B, 0, s>>>(S->bin_ptr, nbins, S->bin_elems);
    FT_TRY_HIP(hipGetLastError());
    FT_TRY_HIP(hipStreamSynchronize(s));
    return FT_OK;
}


template <int D>
static ft_status build(ft_source* S, const double* coords, const int32_t* conn, const double* values,
                       const int32_t* bins, hipStream_t s) {
    constexpr int RS = RecSize<D>::value;
    const int64_t n = S->n, E = S->E;
    constexpr int B = 256;
    FT_TRY(dev_alloc_n(&S->coords, size_t(D) * n));
    FT_TRY(dev_alloc_n(&S->conn, size_t(E) * (D + 1)));
    FT_TRY(dev_alloc_n(&S->values, size_t(S->F) * n));
    FT_TRY(dev_alloc_n(&S->rec, size_t(E) * RS));
    FT_TRY(dev_alloc_n(&S->box, size_t(E) * BoxSize<D>::value));
    FT_TRY(dev_alloc_n(&S->counters, 4));
    FT_TRY_HIP(hipHostMalloc((void**)&S->h_counters, 4 * sizeof(unsigned long long), hipHostMallocDefault));
    FT_TRY_HIP(hipMemcpyAsync(S->coords, coords, sizeof(double) * D * n, hipMemcpyDeviceToDevice, s));
    FT_TRY_HIP(hipMemcpyAsync(S->conn, conn, sizeof(int32_t) * (D + 1) * E, hipMemcpyDeviceToDevice, s));
    FT_TRY_HIP(hipMemcpyAsync(S->values, values, sizeof(double) * S->F * n, hipMemcpyDeviceToDevice, s));
    FT_TRY_HIP(hipMemsetAsync(S->counters, 0, 4 * sizeof(unsigned long long), s));
    if (S->F > 1) {
        FT_TRY(dev_alloc_n(&S->values_nm, size_t(S->F) * n));
        k_node_major<<<grid_for(n * S->F, B), B, 0, s>>>(S->values, n, S->F, S->values_nm);
    }

    unsigned long long* flags = nullptr;
    double* mm = nullptr;
    ScratchGuard guard;
    guard.add((void**)&flags);
    guard.add((void**)&mm);
    FT_TRY(dev_alloc_n(&flags, 4));
    FT_TRY_HIP(hipMemsetAsync(flags, 0, 4 * sizeof(unsigned long long), s));
    k_src_geom<D><<<grid_for(E, B), B, 0, s>>>(S->coords, n, S->conn, E, S->values, S->F, S->rec, S->box, flags);
    const int mmb = 256;
    FT_TRY(dev_alloc_n(&mm, size_t(mmb) * D * 2));
    k_minmax<<<mmb, 256, 0, s>>>(S->coords, n, D, mm);
    FT_TRY_HIP(hipGetLastError());
    unsigned long long hf[4];
    std::vector<double> hmm(size_t(mmb) * D * 2);
    FT_TRY_HIP(hipMemcpyAsync(hf, flags, sizeof(hf), hipMemcpyDeviceToHost, s));
    FT_TRY_HIP(hipMemcpyAsync(hmm.data(), mm, sizeof(double) * hmm.size(), hipMemcpyDeviceToHost, s));
    FT_TRY_HIP(hipStreamSynchronize(s));
    if (hf[0]) {
        set_error("%llu source element(s) reference a node id outside [0, %lld)", hf[0], (long long)n);
        return FT_E_MESH;
    }
    if (hf[1]) {
        set_error("%llu degenerate source element(s): |det J| <= 1e-12 h^d", hf[1]);
        return FT_E_MESH;
    }
    double mag = 0.0;
    std::memcpy(&mag, &hf[2], sizeof(mag));
    S->fast_tau = std::fmax(kFastTau, kFastTauUlps * mag);
    for (int c = 0; c < D; ++c) {
        S->dom_lo[c] = INFINITY;
        S->dom_hi[c] = -INFINITY;
        for (int b = 0; b < mmb; ++b) {
            S->dom_lo[c] = std::fmin(S->dom_lo[c], hmm[(b * D + c) * 2]);
            S->dom_hi[c] = std::fmax(S->dom_hi[c], hmm[(b * D + c) * 2 + 1]);
        }
    }
    int32_t nb[3] = {0, 0, 0};
    for (int c = 0; c < D; ++c) nb[c] = bins && bins[c] > 0 ? bins[c] : 0;
    // default cells along the longest axis: int(sqrt(E)) in 2D (sec. 5.3); in 3D
    // about 0.75 of the cube-root of E/6 (a Kuhn-split hex per 0.4 bins): with
    // centre registration the region a wavefront searches must stay within 64 bins
    const double per_axis = D == 2 ? std::floor(std::sqrt(double(E)))
                                   : std::max(1.0, std::round(0.75 * std::cbrt(double(E) / 6.0)));
    return build_bins<D>(S, nb, per_axis, s);
}

ft_status source_setup(ft_source* S, const double* coords, const int32_t* conn, const double* values,
                       const int32_t* bins, hipStream_t s) {
    return S->dim == 2 ? build<2>(S, coords, conn, values, bins, s) : build<3>(S, coords, conn, values, bins, s);
}

SrcView source_view(const ft_source* S) {
    SrcView v;
    std::memset(&v, 0, sizeof(v));   // padding too: batches compare views bytewise
    v.rec = S->rec;
    v.box = S->box;
    v.conn = S->conn;
    v.values = S->values;
    v.values_nm = S->values_nm;
    v.bin_ptr = S->bin_ptr;
    v.bin_elems = S->bin_elems;
    v.n = S->n;
    v.F = S->F;
    v.E = S->E;
    v.tau = S->fast_tau;
    v.rec_values = S->F == 1 ? 1 : 0;
    for (int c = 0; c < 3; ++c) {
        v.g.nb[c] = S->nb[c];
        v.g.hx[c] = S->hx[c];
        v.g.lo[c] = S->lo[c];
        v.g.inv_h[c] = S->inv_h[c];
    }
    return v;
}

constexpr int kEvalWavesPerBlock = 1;

template <int D>
static ft_status launch_eval(ft_source* S, int64_t head, int64_t npts, const void* pts, int64_t ld, int prec,
                             void* out, int64_t ld_out, int32_t* ids, unsigned long long* ood, hipStream_t s,
                             const ValueLayout* tiles = nullptr) {
    // points per lane: a wave covers 256 consecutive points in 2D, 128 in 3D
    // (one target element's samples at N = 256 / 128; fewer registers in 3D)
    constexpr int P = D == 2 ? 4 : 2;
    constexpr int64_t WP = 64 * P;
    const SrcView v = source_view(S);
    constexpr int WPB = kEvalWavesPerBlock;
    const int64_t waves = (head + WP - 1) / WP + (npts - head + WP - 1) / WP;
    const unsigned grid = unsigned((waves + WPB - 1) / WPB);
    if (S->F > 1 && out) {   // many fields: the lanes interpolate over fields
        const unsigned gw = unsigned(waves);
        const ValueLayout L = tiles ? *tiles : field_major_layout(ld_out, head, 1);
        if (prec == FT_F64)
            k_src_eval_many<D, P, false, false><<<gw, 64, 0, s>>>(v, head, npts, pts, ld, out, L, ids, ood);
        else
            k_src_eval_many<D, P, true, true><<<gw, 64, 0, s>>>(v, head, npts, pts, ld, out, L, ids, ood);
    } else if (prec == FT_F64) {
        k_src_eval<D, P, false, false, WPB><<<grid, 64 * WPB, 0, s>>>(v, head, npts, pts, ld, out, ld_out, ids, ood);
    } else {
        k_src_eval<D, P, true, true, WPB><<<grid, 64 * WPB, 0, s>>>(v, head, npts, pts, ld, out, ld_out, ids, ood);
    }
    FT_TRY_HIP(hipGetLastError());
    return FT_OK;
}

// Bin-grid autotuner: for each candidate resolution, rebuild the bins and time
// the evaluation of a sample of the real queries (two timed launches after a
// warm-up); keep the fastest.  The tuning launches' out-of-domain counts are
// discarded.
template <int D>
static ft_status autotune_impl(ft_source* S, int64_t head, int64_t npts, const void* pts, int64_t ld, int prec,
                              int ncand, const int32_t* cand, hipStream_t s) {
    const size_t esz = prec == FT_F64 ? 8 : 4;
    unsigned char* out = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ScratchGuard guard;
    guard.add((void**)&out);
    FT_TRY(dev_alloc_n(&out, size_t(S->F) * size_t(npts) * esz));
    FT_TRY_HIP(hipEventCreate(&e0));
    FT_TRY_HIP(hipEventCreate(&e1));
    float best_ms = INFINITY;
    int best = cand[0];
    ft_status st = FT_OK;
    const int32_t none[3] = {0, 0, 0};
    for (int c = 0; c < ncand && st == FT_OK; ++c) {
        st = build_bins<D>(S, none, double(cand[c]), s);
        if (st != FT_OK) break;
        st = launch_eval<D>(S, head, npts, pts, ld, prec, out, npts, nullptr, S->counters, s);
        if (hipEventRecord(e0, s) != hipSuccess) st = FT_E_DEVICE;
        for (int r = 0; r < 2 && st == FT_OK; ++r)
            st = launch_eval<D>(S, head, npts, pts, ld, prec, out, npts, nullptr, S->counters, s);
        float ms = 0.0f;
        if (st == FT_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                            hipEventElapsedTime(&ms, e0, e1) != hipSuccess)) {
            set_error("event timing failed while tuning the bin grid");
            st = FT_E_DEVICE;
        }
        if (st == FT_OK && ms < best_ms) {
            best_ms = ms;
            best = cand[c];
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != FT_OK) return st;
    FT_TRY(build_bins<D>(S, none, double(best), s));
    FT_TRY_HIP(hipMemsetAsync(S->counters, 0, sizeof(unsigned long long), s));
    FT_TRY_HIP(hipStreamSynchronize(s));
    return FT_OK;
}

ft_status source_autotune(ft_source* S, int64_t head, int64_t npts, const void* pts, int64_t ld, int prec, int ncand,
                          const int32_t* cand, hipStream_t s) {
    return S->dim == 2 ? autotune_impl<2>(S, head, npts, pts, ld, prec, ncand, cand, s)
                       : autotune_impl<3>(S, head, npts, pts, ld, prec, ncand, cand, s);
}

// Out-of-domain points are counted into `ood` (the source's own counter when null).
ft_status source_eval(ft_source* S, int64_t head, int64_t npts, const void* pts, int64_t ld, int prec, void* out,
                      int64_t ld_out, int32_t* ids, hipStream_t s, unsigned long long* ood) {
    if (npts == 0) return FT_OK;
    if (!ood) ood = S->counters;
    return S->dim == 2 ? launch_eval<2>(S, head, npts, pts, ld, prec, out, ld_out, ids, ood, s)
                       : launch_eval<3>(S, head, npts, pts, ld, prec, out, ld_out, ids, ood, s);
}

// A query list (n_nodes nodes, then n_elems x N samples) with the values
// written as element tiles: [F][n_nodes], then an F x N tile per element.
// With one field the tiles are the field-major list.
ft_status source_eval_tiles(ft_source* S, int64_t n_nodes, int64_t n_elems, int N, const void* pts, int64_t ld,
                            int prec, void* out, int32_t* ids, hipStream_t s) {
    const int64_t npts = n_nodes + n_elems * int64_t(N);
    if (npts == 0) return FT_OK;
    const ValueLayout L = element_tile_layout(n_nodes, N, S->F);
    return S->dim == 2 ? launch_eval<2>(S, n_nodes, npts, pts, ld, prec, out, npts, ids, S->counters, s, &L)
                       : launch_eval<3>(S, n_nodes, npts, pts, ld, prec, out, npts, ids, S->counters, s, &L);
}

// Exact integral of each P1 field over the source mesh (sec. 2, Eq.
// conservation: the quantity a conservative transfer preserves):
//   int f = sum_e |Omega_e| (sum of e's vertex values) / (d + 1),
// |Omega_e| = |det J_e| / d!.  Compensated sums per block, pairs [F][nb][2].
template <int D>
__global__ __launch_bounds__(RB) void k_src_integral(const double* __restrict__ X, int64_t n,
                                                     const int32_t* __restrict__ conn, int64_t E,
                                                     const double* __restrict__ values, int F,
                                                     double* __restrict__ part) {
    for (int f = 0; f < F; ++f) {
        double s = 0.0, c = 0.0;
        for (int64_t e = int64_t(blockIdx.x) * RB + threadIdx.x; e < E; e += int64_t(gridDim.x) * RB) {
            int v[D + 1];
            double x[D + 1][D], vs = 0.0;
#pragma unroll
            for (int k = 0; k <= D; ++k) {
                v[k] = conn[e * (D + 1) + k];
                vs += values[int64_t(f) * n + v[k]];
#pragma unroll
                for (int cc = 0; cc < D; ++cc) x[k][cc] = X[cc * n + v[k]];
            }
            double det;
            if constexpr (D == 2) {
                det = (x[1][0] - x[0][0]) * (x[2][1] - x[0][1]) - (x[2][0] - x[0][0]) * (x[1][1] - x[0][1]);
            } else {
                double J[3][3];
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int b = 0; b < 3; ++b) J[a][b] = x[b + 1][a] - x[0][a];
                det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                      J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                      J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
            }
            const double vol = fabs(det) / (D == 2 ? 2.0 : 6.0);
            comp_add(s, c, vol * vs / double(D + 1));
        }
        block_total_comp(s, c);
        if (threadIdx.x == 0) {
            part[(int64_t(f) * gridDim.x + blockIdx.x) * 2] = s;
            part[(int64_t(f) * gridDim.x + blockIdx.x) * 2 + 1] = c;
        }
    }
}

ft_status source_integral(ft_source* S, double* out, hipStream_t s) {
    const int nb = int(std::min<int64_t>(256, (S->E + RB - 1) / RB));
    double* part = nullptr;
    ScratchGuard guard;
    guard.add((void**)&part);
    FT_TRY(dev_alloc_n(&part, size_t(S->F) * nb * 2));
    if (S->dim == 2)
        k_src_integral<2><<<nb, RB, 0, s>>>(S->coords, S->n, S->conn, S->E, S->values, S->F, part);
    else
        k_src_integral<3><<<nb, RB, 0, s>>>(S->coords, S->n, S->conn, S->E, S->values, S->F, part);
    FT_TRY_HIP(hipGetLastError());
    std::vector<double> h(size_t(S->F) * nb * 2);
    FT_TRY_HIP(hipMemcpyAsync(h.data(), part, sizeof(double) * h.size(), hipMemcpyDeviceToHost, s));
    FT_TRY_HIP(hipStreamSynchronize(s));
    for (int f = 0; f < S->F; ++f) {
        // the block pairs, added with the same compensation on the host
        double sum = 0.0, c = 0.0;
        for (int b = 0; b < nb; ++b) {
            const double x = h[(size_t(f) * nb + b) * 2];
            const double t = sum + x;
            const double bp = t - sum;
            c += (sum - (t - bp)) + (x - bp);
            sum = t;
            c += h[(size_t(f) * nb + b) * 2 + 1];
        }
        out[f] = sum + c;
    }
    return FT_OK;
}

// Rebuild the bins with per_axis cells along the longest axis (the others
// proportionally fewer); the current count along the longest axis.
ft_status source_rebin(ft_source* S, int32_t per_axis, hipStream_t s) {
    const int32_t none[3] = {0, 0, 0};
    return S->dim == 2 ? build_bins<2>(S, none, double(per_axis), s) : build_bins<3>(S, none, double(per_axis), s);
}

// The default cells along the longest axis (sec. 5.3: int(sqrt(E)) in 2D;
// round(0.75 cbrt(E / 6)) in 3D).
int32_t source_default_cells(const ft_source* S) {
    const double E = double(S->E);
    return int32_t(S->dim == 2 ? std::floor(std::sqrt(E)) : std::max(1.0, std::round(0.75 * std::cbrt(E / 6.0))));
}

int32_t source_cells_longest(const ft_source* S) {
    int32_t m = 1;
    for (int c = 0; c < S->dim; ++c) m = std::max(m, S->nb[c]);
    return m;
}

ft_status source_release(ft_source* S) {
    dev_free(S->coords);
    dev_free(S->conn);
    dev_free(S->values);
    dev_free(S->values_nm);
    dev_free(S->rec);
    dev_free(S->box);
    dev_free(S->bin_ptr);
    dev_free(S->bin_elems);
    dev_free(S->counters);
    if (S->h_counters) (void)hipHostFree(S->h_counters);
    return FT_OK;
}

}  // namespace ft
