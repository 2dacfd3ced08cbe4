// Target setup: element measures, node -> element incidence, mass matrix.
//
// Sec. 2: M_ki = int psi_k psi_i, assembled element by element.  On a
// straight-sided simplex the element matrix is |Omega_t| times a reference
// matrix of integrals of products of the basis polynomials in the
// barycentric coordinates: for P1 in closed form,
//   M^t_kl = |Omega_t| (1 + delta_kl) / ((d+1)(d+2)),
// for P2 (vertex functions l_k (2 l_k - 1), edge functions 4 l_a l_b) from
// the exact simplex moments int l^a = d! a_0! ... a_d! |T| / (d + |a|)!.
// |Omega_t| = |det J_t| / d!.
//
// Everything is built on the device and is deterministic: incidence lists
// are sorted by (element, local vertex), CSR rows by column, and every
// floating-point sum runs in ascending element order.
#include <cstring>

#include "common.h"

namespace ft {

// The element mass matrix divided by |Omega_t| and its row sums (the
// integrals of the basis functions over a unit-measure element).
struct RefMass {
    double m[10][10];
    double rs[10];
};

static double simplex_moment(int d, const int* a) {   // int l^a over a unit-measure simplex
    double num = 1.0, den = 1.0;
    int s = 0;
    for (int k = 0; k <= d; ++k) {
        for (int i = 2; i <= a[k]; ++i) num *= i;
        s += a[k];
    }
    for (int i = 2; i <= d; ++i) num *= i;
    for (int i = 2; i <= d + s; ++i) den *= i;
    return num / den;
}

static RefMass reference_mass(int d, int order) {
    RefMass R{};
    const int nb = order == 1 ? d + 1 : (d + 1) * (d + 2) / 2;
    if (order == 1) {
        const double c = 1.0 / ((d + 1) * (d + 2));
        for (int k = 0; k < nb; ++k)
            for (int l = 0; l < nb; ++l) R.m[k][l] = k == l ? 2.0 * c : c;
    } else {
        // basis polynomials: up to two terms (coefficient, exponents)
        double cf[10][2];
        int ex[10][2][4];
        int nt[10];
        std::memset(ex, 0, sizeof(ex));
        for (int k = 0; k <= d; ++k) {
            nt[k] = 2;
            cf[k][0] = 2.0;
            ex[k][0][k] = 2;
            cf[k][1] = -1.0;
            ex[k][1][k] = 1;
        }
        for (int e = 0; e < nb - d - 1; ++e) {
            nt[d + 1 + e] = 1;
            cf[d + 1 + e][0] = 4.0;
            ex[d + 1 + e][0][p2_edge(d, e, 0)] = 1;
            ex[d + 1 + e][0][p2_edge(d, e, 1)] = 1;
        }
        for (int i = 0; i < nb; ++i)
            for (int j = 0; j < nb; ++j) {
                double v = 0.0;
                for (int p = 0; p < nt[i]; ++p)
                    for (int q = 0; q < nt[j]; ++q) {
                        int a[4];
                        for (int k = 0; k < 4; ++k) a[k] = ex[i][p][k] + ex[j][q][k];
                        v += cf[i][p] * cf[j][q] * simplex_moment(d, a);
                    }
                R.m[i][j] = v;
            }
    }
    for (int k = 0; k < nb; ++k) {
        double r = 0.0;
        for (int l = 0; l < nb; ++l) r += R.m[k][l];
        R.rs[k] = r;
    }
    return R;
}

template <int D>
__global__ __launch_bounds__(256) void k_elem_geom(const double* __restrict__ X, int64_t n, const int32_t* __restrict__ conn, int64_t E,
                            double* __restrict__ vol, unsigned long long* __restrict__ flags) {
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= E) return;
    int v[D + 1];
    bool bad = false;
#pragma unroll
    for (int k = 0; k <= D; ++k) {
        v[k] = conn[t * (D + 1) + k];
        bad |= (v[k] < 0) | (int64_t(v[k]) >= n);
    }
    if (bad) {
        atomicAdd(&flags[0], 1ull);
        vol[t] = 0.0;
        return;
    }
    double e[D][D];   // e[k][c] = x_{k+1,c} - x_{0,c}
#pragma unroll
    for (int k = 0; k < D; ++k)
#pragma unroll
        for (int c = 0; c < D; ++c) e[k][c] = X[c * n + v[k + 1]] - X[c * n + v[0]];
    double det, fact;
    if constexpr (D == 2) {
        det = e[0][0] * e[1][1] - e[0][1] * e[1][0];
        fact = 2.0;
    } else if constexpr (D == 3) {
        det = e[0][0] * (e[1][1] * e[2][2] - e[1][2] * e[2][1]) - e[0][1] * (e[1][0] * e[2][2] - e[1][2] * e[2][0]) +
              e[0][2] * (e[1][0] * e[2][1] - e[1][1] * e[2][0]);
        fact = 6.0;
    } else {
        // Gaussian elimination with partial pivoting, det = sign * product of
        // pivots; the pivot row is brought up by conditional swaps with each
        // lower row in turn (static indices: the matrix stays in registers)
        det = 1.0;
        fact = 1.0;
#pragma unroll
        for (int i = 2; i <= D; ++i) fact *= double(i);
#pragma unroll
        for (int c = 0; c < D; ++c) {
#pragma unroll
            for (int r = c + 1; r < D; ++r) {
                const bool sw = fabs(e[r][c]) > fabs(e[c][c]);
                det = sw ? -det : det;
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    const double a = e[c][k], b = e[r][k];
                    e[c][k] = sw ? b : a;
                    e[r][k] = sw ? a : b;
                }
            }
            const double piv = e[c][c];
            det *= piv;
            if (piv != 0.0) {
#pragma unroll
                for (int r = c + 1; r < D; ++r) {
                    const double m = e[r][c] / piv;
#pragma unroll
                    for (int k = c; k < D; ++k) e[r][k] = fma(-m, e[c][k], e[r][k]);
                }
            }
        }
    }
    // longest edge
    double h2 = 0.0;
#pragma unroll
    for (int a = 0; a <= D; ++a)
#pragma unroll
        for (int b = a + 1; b <= D; ++b) {
            double s = 0.0;
#pragma unroll
            for (int c = 0; c < D; ++c) {
                const double d = X[c * n + v[b]] - X[c * n + v[a]];
                s += d * d;
            }
            h2 = fmax(h2, s);
        }
    const double hd = D == 2 ? h2 : (D == 3 ? h2 * sqrt(h2) : pow(h2, 0.5 * D));
    if (!(fabs(det) > 1e-12 * hd)) atomicAdd(&flags[1], 1ull);
    if (det < 0.0) atomicAdd(&flags[2], 1ull);
    vol[t] = fabs(det) / fact;
}

__global__ void k_count_incidence(const int32_t* __restrict__ dofs, int64_t NI, int32_t* __restrict__ cnt) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= NI) return;
    atomicAdd(&cnt[dofs[i]], 1);
}

__global__ void k_fill_incidence(const int32_t* __restrict__ dofs, int64_t NI, const int64_t* __restrict__ ptr,
                                 int32_t* __restrict__ slot, int32_t* __restrict__ inc) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= NI) return;
    const int v = dofs[i];
    const int pos = atomicAdd(&slot[v], 1);
    inc[ptr[v] + pos] = int32_t(i);   // i = t*nb + k
}

// P2: the vertex ids of each element (its first d+1 nodes); every node id in
// range and every edge node at the midpoint of its edge (straight-sided
// elements), else flags[0] / flags[4].
template <int D>
__global__ void k_p2_vertices(const double* __restrict__ X, int64_t n, const int32_t* __restrict__ dofs, int64_t E,
                              int32_t* __restrict__ conn, unsigned long long* __restrict__ flags) {
    constexpr int NB = (D + 1) * (D + 2) / 2;
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= E) return;
    int v[NB];
    bool bad = false;
#pragma unroll
    for (int k = 0; k < NB; ++k) {
        v[k] = dofs[t * NB + k];
        bad |= (v[k] < 0) | (int64_t(v[k]) >= n);
    }
#pragma unroll
    for (int k = 0; k <= D; ++k) conn[t * (D + 1) + k] = bad ? 0 : v[k];
    if (bad) {
        atomicAdd(&flags[0], 1ull);
        return;
    }
    bool off = false;
#pragma unroll
    for (int e = 0; e < NB - D - 1; ++e) {
        const int a = v[p2_edge(D, e, 0)];
        const int b = v[p2_edge(D, e, 1)];
        double len2 = 0.0, dev2 = 0.0;
#pragma unroll
        for (int c = 0; c < D; ++c) {
            const double xa = X[c * n + a], xb = X[c * n + b], xm = X[c * n + v[D + 1 + e]];
            len2 += (xb - xa) * (xb - xa);
            const double dm = xm - 0.5 * (xa + xb);
            dev2 += dm * dm;
        }
        off |= !(dev2 <= 1e-20 * len2);
    }
    if (off) atomicAdd(&flags[4], 1ull);
}

__global__ void k_count_unused(const int32_t* __restrict__ cnt, int64_t n, unsigned long long* __restrict__ flag) {
    const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (v < n && cnt[v] == 0) atomicAdd(flag, 1ull);
}

__device__ void insertion_sort(int32_t* a, int64_t len) {
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

// In-place heapsort: n log n for the long incidence lists of d-simplex meshes
// (5040 entries per vertex in 6D), where insertion sort would take n^2 / 4 moves.
__device__ void heap_sort(int32_t* a, int64_t len) {
    auto sift = [a](int64_t root, int64_t end) {
        while (true) {
            int64_t c = 2 * root + 1;
            if (c >= end) return;
            if (c + 1 < end && a[c + 1] > a[c]) ++c;
            if (a[root] >= a[c]) return;
            const int32_t tmp = a[root];
            a[root] = a[c];
            a[c] = tmp;
            root = c;
        }
    };
    for (int64_t i = len / 2 - 1; i >= 0; --i) sift(i, len);
    for (int64_t end = len - 1; end > 0; --end) {
        const int32_t tmp = a[0];
        a[0] = a[end];
        a[end] = tmp;
        sift(0, end);
    }
}

// Each node's incidence entries ascending (they are distinct, so any sort gives
// the same order).
__global__ void k_sort_segments(const int64_t* __restrict__ ptr, int64_t nseg, int32_t* __restrict__ data) {
    const int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (s >= nseg) return;
    const int64_t len = ptr[s + 1] - ptr[s];
    if (len <= 32) insertion_sort(data + ptr[s], len);
    else heap_sort(data + ptr[s], len);
}

// Columns of row v: the nodes of the elements touching v, sorted and unique,
// written to cand[nb*inc_ptr[v] ...] (room for every candidate), their count
// to rowlen[v].  Each candidate is looked up by binary search in the columns
// found so far and inserted if new: the work grows with the candidates times
// log of the row length, not with the square of the candidates (a 6-simplex
// vertex of a Kuhn mesh has 5040 elements, 35280 candidates, 127 columns).
__global__ void k_row_candidates(const int32_t* __restrict__ dofs, int nb, const int64_t* __restrict__ inc_ptr,
                                 const int32_t* __restrict__ inc, int64_t n, int32_t* __restrict__ cand,
                                 int32_t* __restrict__ rowlen) {
    const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int64_t b = inc_ptr[v], e = inc_ptr[v + 1];
    int32_t* seg = cand + nb * b;
    int64_t u = 0;
    for (int64_t i = b; i < e; ++i) {
        const int t = inc[i] / nb;
        for (int l = 0; l < nb; ++l) {
            const int32_t c = dofs[int64_t(t) * nb + l];
            int64_t lo = 0, hi = u;
            while (lo < hi) {
                const int64_t mid = (lo + hi) >> 1;
                if (seg[mid] < c) lo = mid + 1; else hi = mid;
            }
            if (lo < u && seg[lo] == c) continue;
            for (int64_t k = u; k > lo; --k) seg[k] = seg[k - 1];
            seg[lo] = c;
            ++u;
        }
    }
    rowlen[v] = int32_t(u);
}

// Row v of M: for every (element t, local node k) at v, vol_t * R.m[k][l]
// added at column dofs[t][l], in ascending (t, k) order.  The row sum (the
// lumped mass m_v = int psi_v) is vol_t / (d+1) per element for P1, and
// vol_t * R.rs[k] for P2.
template <int D>
__global__ void k_fill_csr(const int32_t* __restrict__ dofs, int nb, int order, RefMass R,
                           const double* __restrict__ vol,
                           const int64_t* __restrict__ inc_ptr, const int32_t* __restrict__ inc,
                           const int32_t* __restrict__ cand, int64_t n, const int64_t* __restrict__ rowptr,
                           int32_t* __restrict__ col, double* __restrict__ val, double* __restrict__ diag,
                           double* __restrict__ lumped) {
    const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int64_t b = inc_ptr[v], e = inc_ptr[v + 1];
    const int32_t* seg = cand + nb * b;   // the row's sorted unique columns
    const int64_t r0 = rowptr[v], r1 = rowptr[v + 1];
    for (int64_t w = r0; w < r1; ++w) {
        col[w] = seg[w - r0];
        val[w] = 0.0;
    }
    double m = 0.0;
    for (int64_t i = b; i < e; ++i) {
        const int64_t t = inc[i] / nb;
        const int kv = int(inc[i] - t * nb);
        const double vt = vol[t];
        m += order == 1 ? vt / (D + 1) : vt * R.rs[kv];
        for (int l = 0; l < nb; ++l) {
            const int32_t cw = dofs[t * nb + l];
            int64_t lo = r0, hi = r1 - 1;   // binary search in the sorted row
            while (lo < hi) {
                const int64_t mid = (lo + hi) >> 1;
                if (col[mid] < cw) lo = mid + 1; else hi = mid;
            }
            val[lo] += vt * R.m[kv][l];
        }
    }
    for (int64_t i = r0; i < r1; ++i)
        if (col[i] == v) diag[v] = val[i];
    lumped[v] = m;
}

template <int D>
static ft_status build(ft_target* T, const double* coords_in, const int32_t* conn_in, hipStream_t s) {
    const int nb = T->order == 1 ? D + 1 : (D + 1) * (D + 2) / 2;
    T->nb = nb;
    const int64_t n = T->n, E = T->E, NI = E * nb;
    constexpr int B = 256;
    FT_TRY(dev_alloc_n(&T->coords, size_t(D) * n));
    FT_TRY(dev_alloc_n(&T->conn, size_t(E) * (D + 1)));
    FT_TRY(dev_alloc_n(&T->vol, size_t(E)));
    FT_TRY_HIP(hipMemcpyAsync(T->coords, coords_in, sizeof(double) * D * n, hipMemcpyDeviceToDevice, s));

    // scratch: flags, counters, scan temp
    unsigned long long* flags = nullptr;
    int32_t *cnt = nullptr, *rowlen = nullptr, *cand = nullptr;
    int64_t* tmp = nullptr;
    ScratchGuard guard;
    guard.add((void**)&flags);
    guard.add((void**)&cnt);
    guard.add((void**)&rowlen);
    guard.add((void**)&cand);
    guard.add((void**)&tmp);
    FT_TRY(dev_alloc_n(&flags, 5));
    FT_TRY(dev_alloc_n(&cnt, size_t(n)));
    FT_TRY(dev_alloc_n(&rowlen, size_t(n)));
    FT_TRY(dev_alloc_n(&tmp, size_t(scan_tmp_elems(n))));
    FT_TRY_HIP(hipMemsetAsync(flags, 0, 5 * sizeof(unsigned long long), s));

    if (T->order == 1) {
        FT_TRY_HIP(hipMemcpyAsync(T->conn, conn_in, sizeof(int32_t) * NI, hipMemcpyDeviceToDevice, s));
        T->dofs = T->conn;
    } else if constexpr (D <= 3) {
        FT_TRY(dev_alloc_n(&T->dofs, size_t(NI)));
        FT_TRY_HIP(hipMemcpyAsync(T->dofs, conn_in, sizeof(int32_t) * NI, hipMemcpyDeviceToDevice, s));
        k_p2_vertices<D><<<grid_for(E, B), B, 0, s>>>(T->coords, n, T->dofs, E, T->conn, flags);
        FT_TRY_HIP(hipGetLastError());
    } else {
        set_error("P2 targets are triangles and tetrahedra");
        return FT_E_UNSUPPORTED;
    }
    k_elem_geom<D><<<grid_for(E, B), B, 0, s>>>(T->coords, n, T->conn, E, T->vol, flags);
    FT_TRY_HIP(hipGetLastError());
    unsigned long long hf[5];
    FT_TRY_HIP(hipMemcpyAsync(hf, flags, sizeof(hf), hipMemcpyDeviceToHost, s));
    FT_TRY_HIP(hipStreamSynchronize(s));
    if (hf[0]) {
        set_error("%llu element(s) reference a node id outside [0, %lld)", hf[0], (long long)n);
        return FT_E_MESH;
    }
    if (hf[1]) {
        set_error("%llu degenerate element(s): |det J| <= 1e-12 h^d", hf[1]);
        return FT_E_MESH;
    }
    if (hf[4]) {
        set_error("%llu element(s) have an edge node off the midpoint of its edge (straight-sided P2 only)", hf[4]);
        return FT_E_MESH;
    }
    T->n_inverted = (int64_t)hf[2];

    // incidence CSR, entries t*nb+k sorted ascending per node
    FT_TRY(dev_alloc_n(&T->inc_ptr, size_t(n + 1)));
    FT_TRY(dev_alloc_n(&T->inc, size_t(NI)));
    FT_TRY_HIP(hipMemsetAsync(cnt, 0, sizeof(int32_t) * n, s));
    k_count_incidence<<<grid_for(NI, B), B, 0, s>>>(T->dofs, NI, cnt);
    k_count_unused<<<grid_for(n, B), B, 0, s>>>(cnt, n, flags + 3);
    FT_TRY(exclusive_scan(cnt, T->inc_ptr, n, tmp, s));
    FT_TRY_HIP(hipMemsetAsync(cnt, 0, sizeof(int32_t) * n, s));
    k_fill_incidence<<<grid_for(NI, B), B, 0, s>>>(T->dofs, NI, T->inc_ptr, cnt, T->inc);
    k_sort_segments<<<grid_for(n, B), B, 0, s>>>(T->inc_ptr, n, T->inc);
    FT_TRY_HIP(hipGetLastError());

    // CSR pattern and values
    FT_TRY(dev_alloc_n(&cand, size_t(NI) * nb));
    k_row_candidates<<<grid_for(n, B), B, 0, s>>>(T->dofs, nb, T->inc_ptr, T->inc, n, cand, rowlen);
    FT_TRY(dev_alloc_n(&T->rowptr, size_t(n + 1)));
    FT_TRY(exclusive_scan(rowlen, T->rowptr, n, tmp, s));
    int64_t nnz = 0;
    FT_TRY_HIP(hipMemcpyAsync(&nnz, T->rowptr + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    FT_TRY_HIP(hipMemcpyAsync(hf, flags, sizeof(hf), hipMemcpyDeviceToHost, s));
    FT_TRY_HIP(hipStreamSynchronize(s));
    if (hf[3]) {
        set_error("%llu node(s) belong to no element (the mass matrix would be singular)", hf[3]);
        return FT_E_MESH;
    }
    T->nnz = nnz;
    FT_TRY(dev_alloc_n(&T->col, size_t(nnz)));
    FT_TRY(dev_alloc_n(&T->val, size_t(nnz)));
    FT_TRY(dev_alloc_n(&T->diag, size_t(n)));
    FT_TRY(dev_alloc_n(&T->lumped, size_t(n)));
    k_fill_csr<D><<<grid_for(n, B), B, 0, s>>>(T->dofs, nb, T->order, reference_mass(D, T->order), T->vol, T->inc_ptr,
                                              T->inc, cand, n, T->rowptr, T->col, T->val, T->diag, T->lumped);
    FT_TRY_HIP(hipGetLastError());
    FT_TRY_HIP(hipStreamSynchronize(s));
    return FT_OK;
}

ft_status target_setup(ft_target* T, const double* coords, const int32_t* conn, hipStream_t s) {
    switch (T->dim) {
        case 2: return build<2>(T, coords, conn, s);
        case 3: return build<3>(T, coords, conn, s);
        case 4: return build<4>(T, coords, conn, s);
        case 5: return build<5>(T, coords, conn, s);
        case 6: return build<6>(T, coords, conn, s);
        default: set_error("dim must lie in [2, 6] (got %d)", T->dim); return FT_E_ARG;
    }
}

}  // namespace ft
