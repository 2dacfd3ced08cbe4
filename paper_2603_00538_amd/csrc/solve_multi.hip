// Batched Jacobi-PCG for several fields that share one mass matrix (sec. 4.1
// step 7 for F right-hand sides at once).
//
// Internal vectors are stored row-major over fields, v[i * Fp + f], with Fp the
// field count rounded up to a power of two (<= 64).  A wavefront covers
// 64 / Fp consecutive rows, one lane per (row, field): a row's matrix entries
// are shared by its Fp lanes and the products read Fp consecutive doubles per
// column (coalesced), so the matrix is read once for all fields.  Every field
// keeps its own CG scalars and convergence flag; a converged field stops
// updating while the others continue.
//
// Reductions without atomics: each block writes one partial per field (its
// lanes of that field, in a fixed order); a kernel with one block per field
// adds that field's partials in block order and updates its CG scalars.  One
// iteration is five launches: (direction p = z + beta p_old), (q = M p,
// partial p.q), (alpha), (update y, r, z, partial r.z, r.r), (stopping test,
// beta for the next direction).  Forming p in its own pass halves the rows
// the product gathers (one vector instead of two).
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"

namespace ft {

constexpr int MB = 256;               // threads per block
constexpr int MAX_MBLOCKS = 4096;   // enough waves to cover the gather latency at 64 fields

enum { PM_BB = 0, PM_SB, PM_RZ, PM_RR, PM_PQ, PM_TRR, PM_MX, PM_COUNT };
enum { SC_RHO = 0, SC_ALPHA, SC_BETA, SC_TOL2, SC_DONE, SC_ITERS, SC_BB, SC_SUMB, SC_INTX, SC_TRR, SC_COUNT };

struct MView {
    const int64_t* rowptr;
    const int32_t* col;
    const double* val;
    const double* diag;
    const double* lumped;
    int64_t n;
    int F, Fp, shift;   // Fp = 1 << shift
};

#define FOR_ROWS(A, i, f)                                                                        \
    const int f = int(threadIdx.x) & (A.Fp - 1);                                                 \
    const int64_t row0 = (int64_t(blockIdx.x) * MB + threadIdx.x) >> A.shift;                    \
    const int64_t rstride = (int64_t(gridDim.x) * MB) >> A.shift;                                \
    for (int64_t i = row0; i < A.n; i += rstride)

__device__ __forceinline__ double row_dot(const MView& A, int64_t i, const double* __restrict__ v, int f) {
    double s = 0.0;
    for (int64_t k = A.rowptr[i]; k < A.rowptr[i + 1]; ++k) s = fma(A.val[k], v[int64_t(A.col[k]) * A.Fp + f], s);
    return s;
}

// part[(slot * Fp + f) * nb + block] = sum over this block's lanes of field f (fixed order)
template <int NV>
__device__ __forceinline__ void field_partials(const MView& A, const double (&v)[NV], const int (&slot)[NV],
                                               double* __restrict__ part) {
    __shared__ double sm[NV][MB];
#pragma unroll
    for (int k = 0; k < NV; ++k) sm[k][threadIdx.x] = v[k];
    __syncthreads();
    if (threadIdx.x < unsigned(A.Fp)) {
        const int f = threadIdx.x;
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double s = 0.0;
            for (int r = f; r < MB; r += A.Fp) s += sm[k][r];
            part[(int64_t(slot[k]) * A.Fp + f) * gridDim.x + blockIdx.x] = s;
        }
    }
}

__global__ __launch_bounds__(MB) void k_m_transpose_in(const double* __restrict__ src, int64_t n, int F, int Fp,
                                                       double* __restrict__ dst) {
    const int64_t idx = int64_t(blockIdx.x) * MB + threadIdx.x;   // dst[i*Fp + f] = src[f*n + i]
    if (idx >= n * Fp) return;
    const int64_t i = idx / Fp;
    const int f = int(idx - i * Fp);
    dst[idx] = f < F ? src[int64_t(f) * n + i] : 0.0;
}

// dst[i*Fp + f] = src[i*F + f] (fields-inner source), zero padding
__global__ __launch_bounds__(MB) void k_m_pad_in(const double* __restrict__ src, int64_t n, int F, int Fp,
                                                 double* __restrict__ dst) {
    const int64_t idx = int64_t(blockIdx.x) * MB + threadIdx.x;
    if (idx >= n * Fp) return;
    const int64_t i = idx / Fp;
    const int f = int(idx - i * Fp);
    dst[idx] = f < F ? src[i * F + f] : 0.0;
}

__global__ __launch_bounds__(MB) void k_m_transpose_out(const double* __restrict__ src, int64_t n, int F, int Fp,
                                                        double* __restrict__ dst) {
    const int64_t idx = int64_t(blockIdx.x) * MB + threadIdx.x;   // dst[f*n + i] = src[i*Fp + f]
    if (idx >= n * F) return;
    const int f = int(idx / n);
    const int64_t i = idx - int64_t(f) * n;
    dst[idx] = src[i * Fp + f];
}

// B = alpha M G + R (R holds b_res); partials of ||b||^2 and sum b.
__global__ __launch_bounds__(MB) void k_m_rhs(MView A, const double* __restrict__ G, double alpha,
                                              const double* __restrict__ Bres, double* __restrict__ B,
                                              double* __restrict__ part) {
    double v[2] = {0.0, 0.0};
    FOR_ROWS(A, i, f) {
        const double bi = alpha * row_dot(A, i, G, f) + Bres[i * A.Fp + f];
        B[i * A.Fp + f] = bi;
        v[0] = fma(bi, bi, v[0]);
        v[1] += bi;
    }
    const int slot[2] = {PM_BB, PM_SB};
    field_partials<2>(A, v, slot, part);
}

// Y = 0, Z = D^-1 R, P_old = 0; partials of r.z and r.r.
__global__ __launch_bounds__(MB) void k_m_init(MView A, double* __restrict__ Y, const double* __restrict__ R,
                                               double* __restrict__ Z, double* __restrict__ P,
                                               double* __restrict__ part) {
    double v[2] = {0.0, 0.0};
    FOR_ROWS(A, i, f) {
        const int64_t o = i * A.Fp + f;
        const double ri = R[o];
        const double zi = ri / A.diag[i];
        Y[o] = 0.0;
        Z[o] = zi;
        P[o] = 0.0;
        v[0] = fma(ri, zi, v[0]);
        v[1] = fma(ri, ri, v[1]);
    }
    const int slot[2] = {PM_RZ, PM_RR};
    field_partials<2>(A, v, slot, part);
}

// Sum of one field's nb block partials of a slot, in block order (every
// thread of the block returns it).
__device__ __forceinline__ double field_block_total(const MView& A, const double* __restrict__ part, int slot, int f,
                                                    int nb) {
    __shared__ double sm[MB / 64];
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += MB) s += part[(int64_t(slot) * A.Fp + f) * nb + b];
    s = wave_sum_xor(s, 64);
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = s;
    __syncthreads();
    double t = sm[0];
    for (int w = 1; w < MB / 64; ++w) t += sm[w];
    __syncthreads();
    return t;
}

// Per-field scalar updates from the partials (one block per field).
//   mode 0: after k_m_rhs   -> ||b||^2, sum b, threshold, reset
//   mode 1: after r.z, r.r  -> stopping test, beta = rz / rho (0 at k = 0), rho = rz
//   mode 2: after p.q       -> alpha = rho / pq
//   mode 3: after k_m_report -> true residual, m^T x
__global__ __launch_bounds__(MB) void k_m_scalars(MView A, int mode, int k, int nb, double rtol2,
                                                  const double* __restrict__ part, double* __restrict__ sc) {
    const int f = blockIdx.x;
    const int Fp = A.Fp;
    if (mode == 0) {
        const double bb = field_block_total(A, part, PM_BB, f, nb);
        const double sb = field_block_total(A, part, PM_SB, f, nb);
        if (threadIdx.x == 0) {
            sc[SC_BB * Fp + f] = bb;
            sc[SC_SUMB * Fp + f] = sb;
            sc[SC_TOL2 * Fp + f] = rtol2 * bb;
            sc[SC_DONE * Fp + f] = 0.0;
            sc[SC_ITERS * Fp + f] = 0.0;
            sc[SC_BETA * Fp + f] = 0.0;
            sc[SC_ALPHA * Fp + f] = 0.0;
        }
    } else if (mode == 1) {
        if (sc[SC_DONE * Fp + f] != 0.0) return;   // block-uniform
        const double rz = field_block_total(A, part, PM_RZ, f, nb);
        const double rr = field_block_total(A, part, PM_RR, f, nb);
        if (threadIdx.x == 0) {
            sc[SC_ITERS * Fp + f] = double(k);
            if (rr <= sc[SC_TOL2 * Fp + f] || !isfinite(rr)) {
                sc[SC_DONE * Fp + f] = 1.0;
            } else {
                sc[SC_BETA * Fp + f] = k == 0 ? 0.0 : rz / sc[SC_RHO * Fp + f];
                sc[SC_RHO * Fp + f] = rz;
            }
        }
    } else if (mode == 2) {
        if (sc[SC_DONE * Fp + f] != 0.0) return;
        const double pq = field_block_total(A, part, PM_PQ, f, nb);
        if (threadIdx.x == 0) sc[SC_ALPHA * Fp + f] = sc[SC_RHO * Fp + f] / pq;
    } else {
        const double trr = field_block_total(A, part, PM_TRR, f, nb);
        const double mx = field_block_total(A, part, PM_MX, f, nb);
        if (threadIdx.x == 0) {
            sc[SC_TRR * Fp + f] = trr;
            sc[SC_INTX * Fp + f] = mx;
        }
    }
}

// true when every field has converged (wave-uniform scalar loads)
__device__ __forceinline__ bool all_done(const MView& A, const double* __restrict__ sc) {
    for (int f = 0; f < A.F; ++f)
        if (sc[SC_DONE * A.Fp + f] == 0.0) return false;
    return true;
}

// New direction P_new = Z + beta P_old (elementwise; a converged field keeps
// beta = 0, its lanes' values are not used again).
__global__ __launch_bounds__(MB) void k_m_dir(MView A, const double* __restrict__ Z, const double* __restrict__ Pold,
                                              double* __restrict__ Pnew, const double* __restrict__ sc) {
    if (all_done(A, sc)) return;
    FOR_ROWS(A, i, f) {
        const bool live = f < A.F && sc[SC_DONE * A.Fp + f] == 0.0;
        const double bt = live ? sc[SC_BETA * A.Fp + f] : 0.0;
        const int64_t o = i * A.Fp + f;
        Pnew[o] = fma(bt, Pold[o], Z[o]);
    }
}

// Q = M P over this thread's rows; returns the partial of p.q.  WAVE_ROW (64
// fields): a wavefront owns one row, so the row index and its matrix entries
// are wave-uniform and load through the scalar cache, and each product reads
// one 512-byte row of P per matrix entry.
template <bool WAVE_ROW>
__device__ __forceinline__ double spmv_rows(const MView& A, const int64_t* __restrict__ rowptr,
                                            const int32_t* __restrict__ colidx, const double* __restrict__ val,
                                            const double* __restrict__ P, double* __restrict__ Qv,
                                            const double* __restrict__ sc) {
    const int f = int(threadIdx.x) & (A.Fp - 1);
    int64_t row0 = (int64_t(blockIdx.x) * MB + threadIdx.x) >> A.shift;
    if (WAVE_ROW) row0 = uniform_int(int(row0));
    const int64_t rstride = (int64_t(gridDim.x) * MB) >> A.shift;
    const bool live = f < A.F && sc[SC_DONE * A.Fp + f] == 0.0;
    double pq = 0.0;
    for (int64_t i = row0; i < A.n; i += rstride) {
        double qi = 0.0;
        const int64_t k0 = rowptr[i], k1 = rowptr[i + 1];
#pragma unroll 4
        for (int64_t kk = k0; kk < k1; ++kk) qi = fma(val[kk], P[int64_t(colidx[kk]) * A.Fp + f], qi);
        const int64_t o = i * A.Fp + f;
        Qv[o] = qi;
        if (live) pq = fma(P[o], qi, pq);
    }
    return pq;
}

// (the matrix arrays are separate no-alias parameters so that uniform loads
// of them may use the scalar cache)
__global__ __launch_bounds__(MB) void k_m_spmv(MView A, const int64_t* __restrict__ rowptr,
                                               const int32_t* __restrict__ colidx, const double* __restrict__ val,
                                               const double* __restrict__ P, double* __restrict__ Qv,
                                               const double* __restrict__ sc, double* __restrict__ part) {
    if (all_done(A, sc)) return;
    double v[1];
    v[0] = A.Fp == 64 ? spmv_rows<true>(A, rowptr, colidx, val, P, Qv, sc)
                      : spmv_rows<false>(A, rowptr, colidx, val, P, Qv, sc);
    const int slot[1] = {PM_PQ};
    field_partials<1>(A, v, slot, part);
}

__global__ __launch_bounds__(MB) void k_m_update(MView A, const double* __restrict__ P, const double* __restrict__ Qv,
                                                 double* __restrict__ Y, double* __restrict__ R, double* __restrict__ Z,
                                                 const double* __restrict__ sc, double* __restrict__ part) {
    if (all_done(A, sc)) return;
    double v[2] = {0.0, 0.0};
    {
        FOR_ROWS(A, i, f) {
            if (f >= A.F || sc[SC_DONE * A.Fp + f] != 0.0) continue;
            const double a = sc[SC_ALPHA * A.Fp + f];
            const int64_t o = i * A.Fp + f;
            Y[o] = fma(a, P[o], Y[o]);
            const double ri = fma(-a, Qv[o], R[o]);
            const double zi = ri / A.diag[i];
            R[o] = ri;
            Z[o] = zi;
            v[0] = fma(ri, zi, v[0]);
            v[1] = fma(ri, ri, v[1]);
        }
    }
    const int slot[2] = {PM_RZ, PM_RR};
    field_partials<2>(A, v, slot, part);
}

// X = alpha G + Y (in place into Y)
__global__ __launch_bounds__(MB) void k_m_solution(MView A, const double* __restrict__ G, double alpha,
                                                   double* __restrict__ Y) {
    FOR_ROWS(A, i, f) {
        const int64_t o = i * A.Fp + f;
        Y[o] = fma(alpha, G[o], Y[o]);
    }
}

__global__ __launch_bounds__(MB) void k_m_report(MView A, const double* __restrict__ B, const double* __restrict__ X,
                                                 double* __restrict__ part) {
    double v[2] = {0.0, 0.0};
    FOR_ROWS(A, i, f) {
        const int64_t o = i * A.Fp + f;
        const double ri = B[o] - row_dot(A, i, X, f);
        v[0] = fma(ri, ri, v[0]);
        v[1] = fma(A.lumped[i], X[o], v[1]);
    }
    const int slot[2] = {PM_TRR, PM_MX};
    field_partials<2>(A, v, slot, part);
}

ft_status project_multi(ft_target* T, const ft_solve_cfg* cfg, double* x, double* b_out, ft_report* rep,
                        hipStream_t s) {
    const int F = T->consumed_cfg.n_fields;
    int shift = 0;
    while ((1 << shift) < F) ++shift;
    const int Fp = 1 << shift;
    if (Fp > 64) {
        set_error("the batched solver handles at most 64 fields per call (got %d)", F);
        return FT_E_UNSUPPORTED;
    }
    const int64_t n = T->n;
    const double alpha = T->consumed_cfg.alpha;
    const int nb = int(std::max<int64_t>(1, std::min<int64_t>(MAX_MBLOCKS, (n * Fp + MB - 1) / MB)));
    MView A{T->rowptr, T->col, T->val, T->diag, T->lumped, n, F, Fp, shift};

    // work arrays: kept by the target and reused by later solves (grown when
    // a solve needs more fields)
    if (T->mf_Fp < Fp) {
        dev_free(T->mf_vec);
        dev_free(T->mf_sc);
        dev_free(T->mf_part);
        T->mf_vec = T->mf_sc = T->mf_part = nullptr;
        T->mf_Fp = 0;
        FT_TRY(dev_alloc_n(&T->mf_vec, size_t(8) * n * Fp));
        FT_TRY(dev_alloc_n(&T->mf_sc, size_t(SC_COUNT) * 64));
        FT_TRY(dev_alloc_n(&T->mf_part, size_t(PM_COUNT) * 64 * MAX_MBLOCKS));
        T->mf_Fp = Fp;
    }
    const size_t vn = size_t(n) * Fp;
    double* G = T->mf_vec;
    double* B = G + vn;
    double* Y = B + vn;
    double* R = Y + vn;
    double* Z = R + vn;
    double* Qv = Z + vn;
    double* P = Qv + vn;   // two direction buffers, alternating
    double* sc = T->mf_sc;
    double* part = T->mf_part;
    std::vector<double> h(size_t(SC_COUNT) * Fp);

    unsigned long long cnt[2] = {0, 0};   // non-finite values, out-of-domain queries
    FT_TRY_HIP(hipMemcpyAsync(cnt, T->counters, sizeof(cnt), hipMemcpyDeviceToHost, s));
    const unsigned gt = grid_for(n * Fp, MB);
    if (T->fields_inner) {   // the control and residual loads are already node-major
        k_m_pad_in<<<gt, MB, 0, s>>>(T->g, n, F, Fp, G);
        k_m_pad_in<<<gt, MB, 0, s>>>(T->bres, n, F, Fp, R);
    } else {
        k_m_transpose_in<<<gt, MB, 0, s>>>(T->g, n, F, Fp, G);
        k_m_transpose_in<<<gt, MB, 0, s>>>(T->bres, n, F, Fp, R);
    }
    k_m_rhs<<<nb, MB, 0, s>>>(A, G, alpha, R, B, part);
    k_m_scalars<<<F, MB, 0, s>>>(A, 0, 0, nb, cfg->rtol * cfg->rtol, part, sc);
    k_m_init<<<nb, MB, 0, s>>>(A, Y, R, Z, P, part);
    k_m_scalars<<<F, MB, 0, s>>>(A, 1, 0, nb, 0.0, part, sc);
    FT_TRY_HIP(hipGetLastError());
    int launched = 0, chunk = first_chunk(T->cg_hint[2]);
    while (launched < cfg->max_iter) {
        const int k = std::min(chunk, cfg->max_iter - launched);
        for (int it = 0; it < k; ++it) {
            const int kk = launched + it;
            double* Pold = P + ((kk & 1) ? n * Fp : 0);
            double* Pnew = P + ((kk & 1) ? 0 : n * Fp);
            k_m_dir<<<nb, MB, 0, s>>>(A, Z, Pold, Pnew, sc);
            k_m_spmv<<<nb, MB, 0, s>>>(A, A.rowptr, A.col, A.val, Pnew, Qv, sc, part);
            k_m_scalars<<<F, MB, 0, s>>>(A, 2, kk, nb, 0.0, part, sc);
            k_m_update<<<nb, MB, 0, s>>>(A, Pnew, Qv, Y, R, Z, sc, part);
            k_m_scalars<<<F, MB, 0, s>>>(A, 1, kk + 1, nb, 0.0, part, sc);
        }
        launched += k;
        FT_TRY_HIP(hipGetLastError());
        FT_TRY_HIP(hipMemcpyAsync(h.data(), sc, sizeof(double) * h.size(), hipMemcpyDeviceToHost, s));
        FT_TRY_HIP(hipStreamSynchronize(s));
        bool done_all = true;
        for (int f = 0; f < F; ++f) done_all &= h[SC_DONE * Fp + f] != 0.0;
        if (done_all) break;
        chunk = 4;
    }
    k_m_solution<<<nb, MB, 0, s>>>(A, G, alpha, Y);
    k_m_report<<<nb, MB, 0, s>>>(A, B, Y, part);
    k_m_scalars<<<F, MB, 0, s>>>(A, 3, 0, nb, 0.0, part, sc);
    const unsigned go = grid_for(n * F, MB);
    k_m_transpose_out<<<go, MB, 0, s>>>(Y, n, F, Fp, x);
    if (b_out) k_m_transpose_out<<<go, MB, 0, s>>>(B, n, F, Fp, b_out);
    FT_TRY_HIP(hipGetLastError());
    FT_TRY_HIP(hipMemcpyAsync(h.data(), sc, sizeof(double) * h.size(), hipMemcpyDeviceToHost, s));
    FT_TRY_HIP(hipStreamSynchronize(s));
    ft_status worst = FT_OK;
    T->cg_hint[2] = 0;
    for (int f = 0; f < F; ++f) {
        ft_report& Rp = rep[f];
        const double bb = h[SC_BB * Fp + f], sb = h[SC_SUMB * Fp + f];
        Rp.sum_b = sb;
        Rp.int_x = h[SC_INTX * Fp + f];
        Rp.cons_defect = sb != 0.0 ? std::fabs(Rp.int_x - sb) / std::fabs(sb) : std::fabs(Rp.int_x);
        Rp.rel_resid = bb > 0.0 ? std::sqrt(h[SC_TRR * Fp + f] / bb) : std::sqrt(h[SC_TRR * Fp + f]);
        Rp.iters = int32_t(h[SC_ITERS * Fp + f]);
        T->cg_hint[2] = std::max(T->cg_hint[2], int(Rp.iters));
        Rp.n_nonfinite = int64_t(cnt[0]);
        Rp.n_out_of_domain = report_ood(T, cnt);
        Rp.status = cnt[0] ? FT_E_NONFINITE : (h[SC_DONE * Fp + f] != 0.0 ? FT_OK : FT_E_NOCONV);
        if (Rp.status != FT_OK && (worst == FT_OK || Rp.status == FT_E_NONFINITE)) worst = ft_status(Rp.status);
    }
    if (worst == FT_E_NONFINITE) set_error("%llu non-finite query value(s) were consumed", cnt[0]);
    else if (worst == FT_E_NOCONV) set_error("CG did not reach rtol=%g within %d iterations", cfg->rtol, cfg->max_iter);
    return worst;
}

}  // namespace ft
