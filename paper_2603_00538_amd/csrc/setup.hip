// Target setup: element measures, node -> element incidence, P1 mass matrix.
//
// Sec. 2: M_ki = int psi_k psi_i, assembled element by element.  For P1
// simplices the element matrix is exact in closed form,
//   M^t_kl = |Omega_t| (1 + delta_kl) / ((d+1)(d+2)),
// which a degree-2 Gauss rule reproduces exactly.  |Omega_t| = |det J_t| / d!.
//
// Everything is built on the device and is deterministic: incidence lists
// are sorted by (element, local vertex), CSR rows by column, and every
// floating-point sum runs in ascending element order.
#include "common.h"

namespace ft {

template <int D>
__global__ void k_elem_geom(const double* __restrict__ X, int64_t n, const int32_t* __restrict__ conn, int64_t E,
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
    } else {
        det = e[0][0] * (e[1][1] * e[2][2] - e[1][2] * e[2][1]) - e[0][1] * (e[1][0] * e[2][2] - e[1][2] * e[2][0]) +
              e[0][2] * (e[1][0] * e[2][1] - e[1][1] * e[2][0]);
        fact = 6.0;
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
    const double hd = D == 2 ? h2 : h2 * sqrt(h2);
    if (!(fabs(det) > 1e-12 * hd)) atomicAdd(&flags[1], 1ull);
    if (det < 0.0) atomicAdd(&flags[2], 1ull);
    vol[t] = fabs(det) / fact;
}

template <int D>
__global__ void k_count_incidence(const int32_t* __restrict__ conn, int64_t E, int32_t* __restrict__ cnt) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= E * (D + 1)) return;
    atomicAdd(&cnt[conn[i]], 1);
}

template <int D>
__global__ void k_fill_incidence(const int32_t* __restrict__ conn, int64_t E, const int64_t* __restrict__ ptr,
                                 int32_t* __restrict__ slot, int32_t* __restrict__ inc) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= E * (D + 1)) return;
    const int v = conn[i];
    const int pos = atomicAdd(&slot[v], 1);
    inc[ptr[v] + pos] = int32_t(i);   // i = t*(D+1) + k
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

__global__ void k_sort_segments(const int64_t* __restrict__ ptr, int64_t nseg, int32_t* __restrict__ data) {
    const int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (s >= nseg) return;
    insertion_sort(data + ptr[s], ptr[s + 1] - ptr[s]);
}

// Candidate columns of row v: every vertex of every element touching v.
// Written to cand[(D+1)*inc_ptr[v] ...], sorted, unique count -> rowlen[v].
template <int D>
__global__ void k_row_candidates(const int32_t* __restrict__ conn, const int64_t* __restrict__ inc_ptr,
                                 const int32_t* __restrict__ inc, int64_t n, int32_t* __restrict__ cand,
                                 int32_t* __restrict__ rowlen) {
    const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int64_t b = inc_ptr[v], e = inc_ptr[v + 1];
    int32_t* seg = cand + (D + 1) * b;
    for (int64_t i = b; i < e; ++i) {
        const int t = inc[i] / (D + 1);
#pragma unroll
        for (int l = 0; l <= D; ++l) seg[(D + 1) * (i - b) + l] = conn[int64_t(t) * (D + 1) + l];
    }
    const int64_t len = (D + 1) * (e - b);
    insertion_sort(seg, len);
    int32_t u = len > 0 ? 1 : 0;
    for (int64_t i = 1; i < len; ++i) u += seg[i] != seg[i - 1];
    rowlen[v] = u;
}

template <int D>
__global__ void k_fill_csr(const int32_t* __restrict__ conn, const double* __restrict__ vol,
                           const int64_t* __restrict__ inc_ptr, const int32_t* __restrict__ inc,
                           const int32_t* __restrict__ cand, int64_t n, const int64_t* __restrict__ rowptr,
                           int32_t* __restrict__ col, double* __restrict__ val, double* __restrict__ diag,
                           double* __restrict__ lumped) {
    const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int64_t b = inc_ptr[v], e = inc_ptr[v + 1];
    const int32_t* seg = cand + (D + 1) * b;
    const int64_t len = (D + 1) * (e - b);
    const int64_t r0 = rowptr[v];
    int64_t w = r0;
    for (int64_t i = 0; i < len; ++i)
        if (i == 0 || seg[i] != seg[i - 1]) {
            col[w] = seg[i];
            val[w] = 0.0;
            ++w;
        }
    const int64_t r1 = w;
    const double c = 1.0 / ((D + 1) * (D + 2));
    double m = 0.0;
    for (int64_t i = b; i < e; ++i) {
        const int64_t t = inc[i] / (D + 1);
        const double vt = vol[t];
        m += vt / (D + 1);
#pragma unroll
        for (int l = 0; l <= D; ++l) {
            const int32_t cw = conn[t * (D + 1) + l];
            int64_t lo = r0, hi = r1 - 1;   // binary search in the sorted row
            while (lo < hi) {
                const int64_t mid = (lo + hi) >> 1;
                if (col[mid] < cw) lo = mid + 1; else hi = mid;
            }
            val[lo] += (cw == v ? 2.0 : 1.0) * vt * c;
        }
    }
    for (int64_t i = r0; i < r1; ++i)
        if (col[i] == v) diag[v] = val[i];
    lumped[v] = m;
}

template <int D>
static ft_status build(ft_target* T, const double* coords_in, const int32_t* conn_in, hipStream_t s) {
    const int64_t n = T->n, E = T->E, NI = E * (D + 1);
    constexpr int B = 256;
    FT_TRY(dev_alloc_n(&T->coords, size_t(D) * n));
    FT_TRY(dev_alloc_n(&T->conn, size_t(NI)));
    FT_TRY(dev_alloc_n(&T->vol, size_t(E)));
    FT_TRY_HIP(hipMemcpyAsync(T->coords, coords_in, sizeof(double) * D * n, hipMemcpyDeviceToDevice, s));
    FT_TRY_HIP(hipMemcpyAsync(T->conn, conn_in, sizeof(int32_t) * NI, hipMemcpyDeviceToDevice, s));

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
    FT_TRY(dev_alloc_n(&flags, 4));
    FT_TRY(dev_alloc_n(&cnt, size_t(n)));
    FT_TRY(dev_alloc_n(&rowlen, size_t(n)));
    FT_TRY(dev_alloc_n(&tmp, size_t(scan_tmp_elems(n))));
    FT_TRY_HIP(hipMemsetAsync(flags, 0, 4 * sizeof(unsigned long long), s));

    k_elem_geom<D><<<grid_for(E, B), B, 0, s>>>(T->coords, n, T->conn, E, T->vol, flags);
    FT_TRY_HIP(hipGetLastError());
    unsigned long long hf[4];
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
    T->n_inverted = (int64_t)hf[2];

    // incidence CSR, entries t*(D+1)+k sorted ascending per node
    FT_TRY(dev_alloc_n(&T->inc_ptr, size_t(n + 1)));
    FT_TRY(dev_alloc_n(&T->inc, size_t(NI)));
    FT_TRY_HIP(hipMemsetAsync(cnt, 0, sizeof(int32_t) * n, s));
    k_count_incidence<D><<<grid_for(NI, B), B, 0, s>>>(T->conn, E, cnt);
    k_count_unused<<<grid_for(n, B), B, 0, s>>>(cnt, n, flags + 3);
    FT_TRY(exclusive_scan(cnt, T->inc_ptr, n, tmp, s));
    FT_TRY_HIP(hipMemsetAsync(cnt, 0, sizeof(int32_t) * n, s));
    k_fill_incidence<D><<<grid_for(NI, B), B, 0, s>>>(T->conn, E, T->inc_ptr, cnt, T->inc);
    k_sort_segments<<<grid_for(n, B), B, 0, s>>>(T->inc_ptr, n, T->inc);
    FT_TRY_HIP(hipGetLastError());

    // CSR pattern and values
    FT_TRY(dev_alloc_n(&cand, size_t(NI) * (D + 1)));
    k_row_candidates<D><<<grid_for(n, B), B, 0, s>>>(T->conn, T->inc_ptr, T->inc, n, cand, rowlen);
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
    k_fill_csr<D><<<grid_for(n, B), B, 0, s>>>(T->conn, T->vol, T->inc_ptr, T->inc, cand, n, T->rowptr, T->col,
                                              T->val, T->diag, T->lumped);
    FT_TRY_HIP(hipGetLastError());
    FT_TRY_HIP(hipStreamSynchronize(s));
    return FT_OK;
}

ft_status target_setup(ft_target* T, const double* coords, const int32_t* conn, hipStream_t s) {
    return T->dim == 2 ? build<2>(T, coords, conn, s) : build<3>(T, coords, conn, s);
}

}  // namespace ft
