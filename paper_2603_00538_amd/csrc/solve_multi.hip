// Batched Jacobi-PCG for several fields that share one mass matrix (sec. 4.1
// step 7 for F right-hand sides at once).
//
// Internal vectors are stored row-major over fields, v[i * Fp + f], with Fp the
// field count rounded up to a power of two (<= 64).  A wavefront covers
// 64 / Fp consecutive rows, one lane per (row, field): a row's matrix entries
// are shared by its Fp lanes and the products read Fp consecutive doubles per
// column (coalesced), so the matrix is read once for all fields.  Every field
// keeps its own CG scalars and convergence flag; a converged field stops
// updating while the others continue.  Reductions are deterministic: each lane
// sums its own field over a fixed set of rows, blocks add their waves in a
// fixed order, and the last block adds block partials in block order.
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"

namespace ft {

constexpr int MB = 256;               // threads per block
constexpr int MAX_MBLOCKS = 1024;

enum { SC_RHO = 0, SC_ALPHA, SC_BETA, SC_RR, SC_BB, SC_DONE, SC_ITERS, SC_TOL2, SC_SUMB, SC_INTX, SC_TRR, SC_ALL,
       SC_COUNT };

struct MView {
    const int64_t* rowptr;
    const int32_t* col;
    const double* val;
    const double* diag;
    const double* lumped;
    int64_t n;
    int F, Fp, shift;   // Fp = 1 << shift
};

__device__ __forceinline__ double row_dot(const MView& A, int64_t i, const double* __restrict__ v, int f) {
    double s = 0.0;
    for (int64_t k = A.rowptr[i]; k < A.rowptr[i + 1]; ++k) s = fma(A.val[k], v[int64_t(A.col[k]) * A.Fp + f], s);
    return s;
}

// Sum each lane's NV values per field over the block (fixed order), then over
// blocks in the last block; fin(f, totals) runs once per field there.
template <int NV, class Fin>
__device__ __forceinline__ void field_reduce(const MView& A, double (&v)[NV], double* __restrict__ partials,
                                             unsigned int* ticket, Fin fin) {
    __shared__ double sm[NV][MB];
    __shared__ bool last;
#pragma unroll
    for (int k = 0; k < NV; ++k) sm[k][threadIdx.x] = v[k];
    __syncthreads();
    // lanes with the same field: threadIdx % Fp; rows in a fixed order
    if (threadIdx.x < unsigned(A.Fp)) {
        const int f = threadIdx.x;
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double s = 0.0;
            for (int r = f; r < MB; r += A.Fp) s += sm[k][r];
            partials[(int64_t(k) * A.Fp + f) * gridDim.x + blockIdx.x] = s;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        last = atomicAdd(ticket, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (!last) return;
    __threadfence();
    if (threadIdx.x < unsigned(A.Fp)) {
        const int f = threadIdx.x;
        double t[NV];
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double s = 0.0;
            for (unsigned int b = 0; b < gridDim.x; ++b) s += partials[(int64_t(k) * A.Fp + f) * gridDim.x + b];
            t[k] = s;
        }
        if (f < A.F) fin(f, t);
    }
    __syncthreads();
    if (threadIdx.x == 0) *ticket = 0u;
}

#define FOR_ROWS(A, i, f)                                                                        \
    const int f = int(threadIdx.x) & (A.Fp - 1);                                                 \
    const int64_t row0 = (int64_t(blockIdx.x) * MB + threadIdx.x) >> A.shift;                    \
    const int64_t rstride = (int64_t(gridDim.x) * MB) >> A.shift;                                \
    for (int64_t i = row0; i < A.n; i += rstride)

__global__ __launch_bounds__(MB) void k_m_transpose_in(const double* __restrict__ src, int64_t n, int F, int Fp,
                                                       double* __restrict__ dst) {
    // dst[i*Fp + f] = src[f*n + i] (0 for padded fields)
    const int64_t idx = int64_t(blockIdx.x) * MB + threadIdx.x;
    if (idx >= n * Fp) return;
    const int64_t i = idx / Fp;
    const int f = int(idx - i * Fp);
    dst[idx] = f < F ? src[int64_t(f) * n + i] : 0.0;
}

__global__ __launch_bounds__(MB) void k_m_transpose_out(const double* __restrict__ src, int64_t n, int F, int Fp,
                                                        double* __restrict__ dst) {
    // dst[f*n + i] = src[i*Fp + f]
    const int64_t idx = int64_t(blockIdx.x) * MB + threadIdx.x;
    if (idx >= n * F) return;
    const int f = int(idx / n);
    const int64_t i = idx - int64_t(f) * n;
    dst[idx] = src[i * Fp + f];
}

// B = alpha M G + R (R holds b_res on entry); sums ||b||^2 and sum b per field.
__global__ __launch_bounds__(MB) void k_m_rhs(MView A, const double* __restrict__ G, double alpha,
                                              const double* __restrict__ Bres, double* __restrict__ B,
                                              double* __restrict__ sc, double* __restrict__ partials,
                                              unsigned int* ticket) {
    double v[2] = {0.0, 0.0};
    FOR_ROWS(A, i, f) {
        const double bi = alpha * row_dot(A, i, G, f) + Bres[i * A.Fp + f];
        B[i * A.Fp + f] = bi;
        v[0] = fma(bi, bi, v[0]);
        v[1] += bi;
    }
    field_reduce<2>(A, v, partials, ticket, [&](int ff, double (&t)[2]) {
        sc[SC_BB * A.Fp + ff] = t[0];
        sc[SC_SUMB * A.Fp + ff] = t[1];
    });
}

__global__ __launch_bounds__(MB) void k_m_init(MView A, double rtol2, double* __restrict__ Y, double* __restrict__ R,
                                               double* __restrict__ Z, double* __restrict__ P, double* __restrict__ sc,
                                               double* __restrict__ partials, unsigned int* ticket) {
    double v[2] = {0.0, 0.0};
    FOR_ROWS(A, i, f) {
        const int64_t o = i * A.Fp + f;
        const double ri = R[o];   // b_res
        const double zi = ri / A.diag[i];
        Y[o] = 0.0;
        Z[o] = zi;
        P[o] = zi;
        v[0] = fma(ri, zi, v[0]);
        v[1] = fma(ri, ri, v[1]);
    }
    field_reduce<2>(A, v, partials, ticket, [&](int ff, double (&t)[2]) {
        const double tol2 = rtol2 * sc[SC_BB * A.Fp + ff];
        sc[SC_RHO * A.Fp + ff] = t[0];
        sc[SC_RR * A.Fp + ff] = t[1];
        sc[SC_TOL2 * A.Fp + ff] = tol2;
        sc[SC_ITERS * A.Fp + ff] = 0.0;
        sc[SC_DONE * A.Fp + ff] = (t[1] <= tol2 || !isfinite(t[1]) || !isfinite(tol2)) ? 1.0 : 0.0;
        sc[SC_ALPHA * A.Fp + ff] = 0.0;
        sc[SC_BETA * A.Fp + ff] = 0.0;
    });
}

// all-fields-done flag: computed by one small kernel after every update
__global__ void k_m_all_done(int F, int Fp, double* __restrict__ sc) {
    if (threadIdx.x == 0) {
        double all = 1.0;
        for (int f = 0; f < F; ++f) all = sc[SC_DONE * Fp + f] != 0.0 ? all : 0.0;
        sc[SC_ALL * Fp] = all;
    }
}

__global__ __launch_bounds__(MB) void k_m_spmv(MView A, const double* __restrict__ P, double* __restrict__ Qv,
                                               double* __restrict__ sc, double* __restrict__ partials,
                                               unsigned int* ticket) {
    if (sc[SC_ALL * A.Fp] != 0.0) return;
    double v[1] = {0.0};
    FOR_ROWS(A, i, f) {
        const double qi = row_dot(A, i, P, f);
        Qv[i * A.Fp + f] = qi;
        v[0] = fma(P[i * A.Fp + f], qi, v[0]);
    }
    field_reduce<1>(A, v, partials, ticket, [&](int ff, double (&t)[1]) {
        const bool done = sc[SC_DONE * A.Fp + ff] != 0.0;
        sc[SC_ALPHA * A.Fp + ff] = done ? 0.0 : sc[SC_RHO * A.Fp + ff] / t[0];
    });
}

__global__ __launch_bounds__(MB) void k_m_update(MView A, const double* __restrict__ P, const double* __restrict__ Qv,
                                                 double* __restrict__ Y, double* __restrict__ R, double* __restrict__ Z,
                                                 double* __restrict__ sc, double* __restrict__ partials,
                                                 unsigned int* ticket) {
    if (sc[SC_ALL * A.Fp] != 0.0) return;
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
    field_reduce<2>(A, v, partials, ticket, [&](int ff, double (&t)[2]) {
        if (sc[SC_DONE * A.Fp + ff] != 0.0) return;
        sc[SC_BETA * A.Fp + ff] = t[0] / sc[SC_RHO * A.Fp + ff];
        sc[SC_RHO * A.Fp + ff] = t[0];
        sc[SC_RR * A.Fp + ff] = t[1];
        sc[SC_ITERS * A.Fp + ff] += 1.0;
        if (t[1] <= sc[SC_TOL2 * A.Fp + ff]) sc[SC_DONE * A.Fp + ff] = 1.0;
    });
}

__global__ __launch_bounds__(MB) void k_m_direction(MView A, const double* __restrict__ Z, double* __restrict__ P,
                                                    const double* __restrict__ sc) {
    if (sc[SC_ALL * A.Fp] != 0.0) return;
    FOR_ROWS(A, i, f) {
        if (f >= A.F || sc[SC_DONE * A.Fp + f] != 0.0) continue;
        const int64_t o = i * A.Fp + f;
        P[o] = fma(sc[SC_BETA * A.Fp + f], P[o], Z[o]);
    }
}

// X = alpha G + Y (in place into Y), then true residual and m^T x per field
__global__ __launch_bounds__(MB) void k_m_solution(MView A, const double* __restrict__ G, double alpha,
                                                   double* __restrict__ Y) {
    FOR_ROWS(A, i, f) {
        const int64_t o = i * A.Fp + f;
        Y[o] = fma(alpha, G[o], Y[o]);
    }
}

__global__ __launch_bounds__(MB) void k_m_report(MView A, const double* __restrict__ B, const double* __restrict__ X,
                                                 double* __restrict__ sc, double* __restrict__ partials,
                                                 unsigned int* ticket) {
    double v[2] = {0.0, 0.0};
    FOR_ROWS(A, i, f) {
        const int64_t o = i * A.Fp + f;
        const double ri = B[o] - row_dot(A, i, X, f);
        v[0] = fma(ri, ri, v[0]);
        v[1] = fma(A.lumped[i], X[o], v[1]);
    }
    field_reduce<2>(A, v, partials, ticket, [&](int ff, double (&t)[2]) {
        sc[SC_TRR * A.Fp + ff] = t[0];
        sc[SC_INTX * A.Fp + ff] = t[1];
    });
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
    const int nb = int(std::min<int64_t>(MAX_MBLOCKS, (n * Fp + MB - 1) / MB));
    MView A{T->rowptr, T->col, T->val, T->diag, T->lumped, n, F, Fp, shift};

    // work arrays (freed on return; the solve is synchronous)
    double *G = nullptr, *B = nullptr, *Y = nullptr, *R = nullptr, *Z = nullptr, *P = nullptr, *Qv = nullptr;
    double *sc = nullptr, *partials = nullptr;
    unsigned int* ticket = nullptr;
    ScratchGuard guard;
    for (double** p : {&G, &B, &Y, &R, &Z, &P, &Qv}) {
        guard.add((void**)p);
        FT_TRY(dev_alloc_n(p, size_t(n) * Fp));
    }
    guard.add((void**)&sc);
    guard.add((void**)&partials);
    guard.add((void**)&ticket);
    FT_TRY(dev_alloc_n(&sc, size_t(SC_COUNT) * Fp));
    FT_TRY(dev_alloc_n(&partials, size_t(2) * Fp * nb));
    FT_TRY(dev_alloc_n(&ticket, 4));
    std::vector<double> h(size_t(SC_COUNT) * Fp);
    FT_TRY_HIP(hipMemsetAsync(ticket, 0, 4 * sizeof(unsigned int), s));
    FT_TRY_HIP(hipMemsetAsync(sc, 0, sizeof(double) * SC_COUNT * Fp, s));

    unsigned long long nonfinite = 0;
    FT_TRY_HIP(hipMemcpyAsync(&nonfinite, T->counters, sizeof(nonfinite), hipMemcpyDeviceToHost, s));
    const unsigned gt = grid_for(n * Fp, MB);
    k_m_transpose_in<<<gt, MB, 0, s>>>(T->g, n, F, Fp, G);
    k_m_transpose_in<<<gt, MB, 0, s>>>(T->bres, n, F, Fp, R);
    k_m_rhs<<<nb, MB, 0, s>>>(A, G, alpha, R, B, sc, partials, ticket);
    k_m_init<<<nb, MB, 0, s>>>(A, cfg->rtol * cfg->rtol, Y, R, Z, P, sc, partials, ticket);
    k_m_all_done<<<1, 64, 0, s>>>(F, Fp, sc);
    FT_TRY_HIP(hipGetLastError());
    int launched = 0, chunk = 8;
    bool all_done = false;
    while (launched < cfg->max_iter) {
        const int k = std::min(chunk, cfg->max_iter - launched);
        for (int it = 0; it < k; ++it) {
            k_m_spmv<<<nb, MB, 0, s>>>(A, P, Qv, sc, partials, ticket);
            k_m_update<<<nb, MB, 0, s>>>(A, P, Qv, Y, R, Z, sc, partials, ticket);
            k_m_all_done<<<1, 64, 0, s>>>(F, Fp, sc);
            k_m_direction<<<nb, MB, 0, s>>>(A, Z, P, sc);
        }
        launched += k;
        FT_TRY_HIP(hipGetLastError());
        FT_TRY_HIP(hipMemcpyAsync(h.data(), sc, sizeof(double) * h.size(), hipMemcpyDeviceToHost, s));
        FT_TRY_HIP(hipStreamSynchronize(s));
        if (h[SC_ALL * Fp] != 0.0) {
            all_done = true;
            break;
        }
        chunk = 4;
    }
    (void)all_done;
    k_m_solution<<<nb, MB, 0, s>>>(A, G, alpha, Y);
    k_m_report<<<nb, MB, 0, s>>>(A, B, Y, sc, partials, ticket);
    const unsigned go = grid_for(n * F, MB);
    k_m_transpose_out<<<go, MB, 0, s>>>(Y, n, F, Fp, x);
    if (b_out) k_m_transpose_out<<<go, MB, 0, s>>>(B, n, F, Fp, b_out);
    FT_TRY_HIP(hipGetLastError());
    FT_TRY_HIP(hipMemcpyAsync(h.data(), sc, sizeof(double) * h.size(), hipMemcpyDeviceToHost, s));
    FT_TRY_HIP(hipStreamSynchronize(s));
    ft_status worst = FT_OK;
    for (int f = 0; f < F; ++f) {
        ft_report& Rp = rep[f];
        const double bb = h[SC_BB * Fp + f], sb = h[SC_SUMB * Fp + f];
        Rp.sum_b = sb;
        Rp.int_x = h[SC_INTX * Fp + f];
        Rp.cons_defect = sb != 0.0 ? std::fabs(Rp.int_x - sb) / std::fabs(sb) : std::fabs(Rp.int_x);
        Rp.rel_resid = bb > 0.0 ? std::sqrt(h[SC_TRR * Fp + f] / bb) : std::sqrt(h[SC_TRR * Fp + f]);
        Rp.iters = int32_t(h[SC_ITERS * Fp + f]);
        Rp.n_nonfinite = int64_t(nonfinite);
        Rp.status = nonfinite ? FT_E_NONFINITE : (h[SC_DONE * Fp + f] != 0.0 ? FT_OK : FT_E_NOCONV);
        if (Rp.status != FT_OK && (worst == FT_OK || Rp.status == FT_E_NONFINITE)) worst = ft_status(Rp.status);
    }
    if (worst == FT_E_NONFINITE) set_error("%llu non-finite query value(s) were consumed", nonfinite);
    else if (worst == FT_E_NOCONV) set_error("CG did not reach rtol=%g within %d iterations", cfg->rtol, cfg->max_iter);
    return worst;
}

}  // namespace ft
