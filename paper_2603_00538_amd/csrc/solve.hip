// Control load, mass solve and conservation report (sec. 4.1 steps 2, 6, 7).
//
// Step 2: the control part of the load vector, integral alpha g psi_i, is
// exactly alpha (M g)_i for P1 g (degree-2 quadrature is exact), so
// b = alpha M g + b_res is one CSR product.
// Step 7: M x = b.  Since M (alpha g) = alpha M g, the residual of the start
// x0 = alpha g is exactly b_res; Jacobi-PCG therefore runs on M y = b_res from
// y = 0 and x = alpha g + y, stopping when ||b_res - M y|| <= rtol ||b||
// (which is ||b - M x|| <= rtol ||b||).  The Jacobi-scaled P1 mass matrix has
// eigenvalues in [1/2, 2] (triangles) or [1/2, 5/2] (tetrahedra), so CG
// converges in a few tens of iterations.
// Conservation (sec. 2 Eq. conservation; App. B with w_h = 1): with m = M 1,
// m^T x = sum_i b_i up to the solver tolerance.
//
// Every reduction is two-level and deterministic: per-thread sums over a
// fixed grid-stride set of rows, a fixed block tree, and the last block to
// finish (atomic ticket) adds the block partials in block order.
#include <algorithm>
#include <cmath>

#include "common.h"

namespace ft {

constexpr int RB = 256;             // threads per block in the solver kernels
constexpr int MAX_RBLOCKS = 1024;   // grid size cap (grid-stride loops beyond it)

// device scalar slots
enum {
    S_RHO = 0, S_ALPHA, S_BETA, S_RR, S_BB, S_DONE, S_ITERS, S_TOL2, S_SUMB, S_INTX, S_TRR, S_ACOEF, S_COUNT
};

template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV]) {
    __shared__ double sm[NV][RB / 64];
    const int w = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = wave_sum_xor(v[i], 64);
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int i = 0; i < NV; ++i) sm[i][w] = v[i];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            double s = sm[i][0];
            for (int k = 1; k < RB / 64; ++k) s += sm[i][k];
            v[i] = s;
        }
    __syncthreads();
}

// Combine per-block sums; the last block to arrive calls fin(total) on thread 0.
template <int NV, class Fin>
__device__ __forceinline__ void grid_reduce(double (&v)[NV], double* __restrict__ partials, unsigned int* ticket,
                                            Fin fin) {
    block_sum<NV>(v);
    __shared__ bool last;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i) partials[i * gridDim.x + blockIdx.x] = v[i];
        __threadfence();
        const unsigned int prev = atomicAdd(ticket, 1u);
        last = prev == gridDim.x - 1;
    }
    __syncthreads();
    if (!last) return;
    __threadfence();
    double acc[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        acc[i] = 0.0;
        for (unsigned int b = threadIdx.x; b < gridDim.x; b += RB) acc[i] += partials[i * gridDim.x + b];
    }
    block_sum<NV>(acc);
    if (threadIdx.x == 0) {
        fin(acc);
        *ticket = 0u;
    }
}

__device__ __forceinline__ double csr_row(const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                                          const double* __restrict__ val, const double* __restrict__ x, int64_t i) {
    double s = 0.0;
    for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) s = fma(val[k], x[col[k]], s);
    return s;
}

struct Mat {
    const int64_t* rowptr;
    const int32_t* col;
    const double* val;
    const double* diag;
    const double* lumped;
    int64_t n;
};

// b = alpha M g + b_res; sums: ||b||^2 and sum b.
__global__ __launch_bounds__(RB) void k_rhs(Mat A, const double* __restrict__ g, const double* __restrict__ bres,
                                            double alpha, double* __restrict__ b, double* __restrict__ scal,
                                            double* __restrict__ partials, unsigned int* ticket) {
    double v[2] = {0.0, 0.0};
    for (int64_t i = int64_t(blockIdx.x) * RB + threadIdx.x; i < A.n; i += int64_t(gridDim.x) * RB) {
        const double bi = alpha * csr_row(A.rowptr, A.col, A.val, g, i) + bres[i];
        b[i] = bi;
        v[0] = fma(bi, bi, v[0]);
        v[1] += bi;
    }
    grid_reduce<2>(v, partials, ticket, [&](double (&t)[2]) {
        scal[S_BB] = t[0];
        scal[S_SUMB] = t[1];
    });
}

__global__ __launch_bounds__(RB) void k_cg_init(Mat A, const double* __restrict__ bres, double rtol2,
                                                double* __restrict__ y, double* __restrict__ r, double* __restrict__ z,
                                                double* __restrict__ p, double* __restrict__ scal,
                                                double* __restrict__ partials, unsigned int* ticket) {
    double v[2] = {0.0, 0.0};
    for (int64_t i = int64_t(blockIdx.x) * RB + threadIdx.x; i < A.n; i += int64_t(gridDim.x) * RB) {
        const double ri = bres[i];
        const double zi = ri / A.diag[i];
        y[i] = 0.0;
        r[i] = ri;
        z[i] = zi;
        p[i] = zi;
        v[0] = fma(ri, zi, v[0]);
        v[1] = fma(ri, ri, v[1]);
    }
    grid_reduce<2>(v, partials, ticket, [&](double (&t)[2]) {
        const double tol2 = rtol2 * scal[S_BB];
        scal[S_RHO] = t[0];
        scal[S_RR] = t[1];
        scal[S_TOL2] = tol2;
        scal[S_ITERS] = 0.0;
        // a non-finite right-hand side cannot converge: stop at once (reported as non-finite)
        scal[S_DONE] = (t[1] <= tol2 || !isfinite(t[1]) || !isfinite(tol2)) ? 1.0 : 0.0;
    });
}

// q = M p, alpha = rho / (p . q)
__global__ __launch_bounds__(RB) void k_cg_spmv(Mat A, const double* __restrict__ p, double* __restrict__ q,
                                                double* __restrict__ scal, double* __restrict__ partials,
                                                unsigned int* ticket) {
    if (scal[S_DONE] != 0.0) return;
    double v[1] = {0.0};
    for (int64_t i = int64_t(blockIdx.x) * RB + threadIdx.x; i < A.n; i += int64_t(gridDim.x) * RB) {
        const double qi = csr_row(A.rowptr, A.col, A.val, p, i);
        q[i] = qi;
        v[0] = fma(p[i], qi, v[0]);
    }
    grid_reduce<1>(v, partials, ticket, [&](double (&t)[1]) { scal[S_ALPHA] = scal[S_RHO] / t[0]; });
}

// y += alpha p; r -= alpha q; z = D^-1 r; beta = (r.z)_new / (r.z)_old; convergence test on ||r||
__global__ __launch_bounds__(RB) void k_cg_update(Mat A, const double* __restrict__ p, const double* __restrict__ q,
                                                  double* __restrict__ y, double* __restrict__ r,
                                                  double* __restrict__ z, double* __restrict__ scal,
                                                  double* __restrict__ partials, unsigned int* ticket) {
    if (scal[S_DONE] != 0.0) return;
    const double a = scal[S_ALPHA];
    double v[2] = {0.0, 0.0};
    for (int64_t i = int64_t(blockIdx.x) * RB + threadIdx.x; i < A.n; i += int64_t(gridDim.x) * RB) {
        y[i] = fma(a, p[i], y[i]);
        const double ri = fma(-a, q[i], r[i]);
        const double zi = ri / A.diag[i];
        r[i] = ri;
        z[i] = zi;
        v[0] = fma(ri, zi, v[0]);
        v[1] = fma(ri, ri, v[1]);
    }
    grid_reduce<2>(v, partials, ticket, [&](double (&t)[2]) {
        scal[S_BETA] = t[0] / scal[S_RHO];
        scal[S_RHO] = t[0];
        scal[S_RR] = t[1];
        scal[S_ITERS] += 1.0;
        if (t[1] <= scal[S_TOL2]) scal[S_DONE] = 1.0;
    });
}

__global__ __launch_bounds__(RB) void k_cg_direction(int64_t n, const double* __restrict__ z, double* __restrict__ p,
                                                     const double* __restrict__ scal) {
    if (scal[S_DONE] != 0.0) return;
    const double bt = scal[S_BETA];
    for (int64_t i = int64_t(blockIdx.x) * RB + threadIdx.x; i < n; i += int64_t(gridDim.x) * RB)
        p[i] = fma(bt, p[i], z[i]);
}

__global__ __launch_bounds__(RB) void k_solution(int64_t n, const double* __restrict__ g, const double* __restrict__ y,
                                                 double alpha, double* __restrict__ x) {
    for (int64_t i = int64_t(blockIdx.x) * RB + threadIdx.x; i < n; i += int64_t(gridDim.x) * RB)
        x[i] = fma(alpha, g[i], y[i]);
}

// true residual ||b - M x||^2 and m^T x
__global__ __launch_bounds__(RB) void k_report(Mat A, const double* __restrict__ b, const double* __restrict__ x,
                                               double* __restrict__ scal, double* __restrict__ partials,
                                               unsigned int* ticket) {
    double v[2] = {0.0, 0.0};
    for (int64_t i = int64_t(blockIdx.x) * RB + threadIdx.x; i < A.n; i += int64_t(gridDim.x) * RB) {
        const double ri = b[i] - csr_row(A.rowptr, A.col, A.val, x, i);
        v[0] = fma(ri, ri, v[0]);
        v[1] = fma(A.lumped[i], x[i], v[1]);
    }
    grid_reduce<2>(v, partials, ticket, [&](double (&t)[2]) {
        scal[S_TRR] = t[0];
        scal[S_INTX] = t[1];
    });
}

ft_status solver_alloc(ft_target* T, hipStream_t s) {
    const int64_t n = T->n;
    T->reduce_blocks = int(std::min<int64_t>(MAX_RBLOCKS, (n + RB - 1) / RB));
    if (T->reduce_blocks < 1) T->reduce_blocks = 1;
    FT_TRY(dev_alloc_n(&T->r, size_t(n)));
    FT_TRY(dev_alloc_n(&T->z, size_t(n)));
    FT_TRY(dev_alloc_n(&T->p, size_t(n)));
    FT_TRY(dev_alloc_n(&T->q, size_t(n)));
    FT_TRY(dev_alloc_n(&T->y, size_t(n)));
    FT_TRY(dev_alloc_n(&T->b, size_t(n)));
    FT_TRY(dev_alloc_n(&T->scal, S_COUNT));
    FT_TRY(dev_alloc_n(&T->partials, size_t(T->reduce_blocks) * 4));
    FT_TRY(dev_alloc_n(&T->ticket, 4));
    FT_TRY(dev_alloc_n(&T->counters, 4));
    FT_TRY_HIP(hipMemsetAsync(T->ticket, 0, 4 * sizeof(unsigned int), s));
    FT_TRY_HIP(hipMemsetAsync(T->counters, 0, 4 * sizeof(unsigned long long), s));
    FT_TRY_HIP(hipMemsetAsync(T->scal, 0, S_COUNT * sizeof(double), s));
    FT_TRY_HIP(hipHostMalloc((void**)&T->h_scal, S_COUNT * sizeof(double), hipHostMallocDefault));
    return FT_OK;
}

ft_status project_multi(ft_target* T, const ft_solve_cfg* cfg, double* x, double* b_out, ft_report* rep,
                        hipStream_t s);

ft_status project(ft_target* T, const ft_solve_cfg* cfg, double* x, double* b_out, ft_report* rep, hipStream_t s) {
    const int F = T->consumed_cfg.n_fields;
    if (F > 1) return project_multi(T, cfg, x, b_out, rep, s);
    const double alpha = T->consumed_cfg.alpha;
    const int64_t n = T->n;
    const unsigned nb = unsigned(T->reduce_blocks);
    Mat A{T->rowptr, T->col, T->val, T->diag, T->lumped, n};
    const double rtol2 = cfg->rtol * cfg->rtol;
    // non-finite values seen by the last consume
    unsigned long long nonfinite = 0;
    FT_TRY_HIP(hipMemcpyAsync(&nonfinite, T->counters, sizeof(nonfinite), hipMemcpyDeviceToHost, s));
    ft_status worst = FT_OK;
    for (int f = 0; f < F; ++f) {
        const double* gf = T->g + int64_t(f) * n;
        const double* bresf = T->bres + int64_t(f) * n;
        double* bf = b_out ? b_out + int64_t(f) * n : T->b;
        double* xf = x + int64_t(f) * n;
        k_rhs<<<nb, RB, 0, s>>>(A, gf, bresf, alpha, bf, T->scal, T->partials, T->ticket);
        k_cg_init<<<nb, RB, 0, s>>>(A, bresf, rtol2, T->y, T->r, T->z, T->p, T->scal, T->partials, T->ticket);
        FT_TRY_HIP(hipGetLastError());
        int launched = 0;
        int chunk = 8;
        bool done = false;
        while (launched < cfg->max_iter) {
            const int k = std::min(chunk, cfg->max_iter - launched);
            for (int it = 0; it < k; ++it) {
                k_cg_spmv<<<nb, RB, 0, s>>>(A, T->p, T->q, T->scal, T->partials, T->ticket);
                k_cg_update<<<nb, RB, 0, s>>>(A, T->p, T->q, T->y, T->r, T->z, T->scal, T->partials, T->ticket);
                k_cg_direction<<<nb, RB, 0, s>>>(n, T->z, T->p, T->scal);
            }
            launched += k;
            FT_TRY_HIP(hipGetLastError());
            FT_TRY_HIP(hipMemcpyAsync(T->h_scal, T->scal, S_COUNT * sizeof(double), hipMemcpyDeviceToHost, s));
            FT_TRY_HIP(hipStreamSynchronize(s));
            if (T->h_scal[S_DONE] != 0.0) {
                done = true;
                break;
            }
            chunk = 4;
        }
        if (!done) {
            FT_TRY_HIP(hipMemcpyAsync(T->h_scal, T->scal, S_COUNT * sizeof(double), hipMemcpyDeviceToHost, s));
            FT_TRY_HIP(hipStreamSynchronize(s));
            done = T->h_scal[S_DONE] != 0.0;
        }
        k_solution<<<nb, RB, 0, s>>>(n, gf, T->y, alpha, xf);
        k_report<<<nb, RB, 0, s>>>(A, bf, xf, T->scal, T->partials, T->ticket);
        FT_TRY_HIP(hipGetLastError());
        FT_TRY_HIP(hipMemcpyAsync(T->h_scal, T->scal, S_COUNT * sizeof(double), hipMemcpyDeviceToHost, s));
        FT_TRY_HIP(hipStreamSynchronize(s));
        const double* h = T->h_scal;
        ft_report& R = rep[f];
        R.sum_b = h[S_SUMB];
        R.int_x = h[S_INTX];
        R.cons_defect = h[S_SUMB] != 0.0 ? std::fabs(h[S_INTX] - h[S_SUMB]) / std::fabs(h[S_SUMB])
                                         : std::fabs(h[S_INTX]);
        R.rel_resid = h[S_BB] > 0.0 ? std::sqrt(h[S_TRR] / h[S_BB]) : std::sqrt(h[S_TRR]);
        R.iters = int32_t(h[S_ITERS]);
        R.n_nonfinite = int64_t(nonfinite);
        R.status = FT_OK;
        if (nonfinite) R.status = FT_E_NONFINITE;
        else if (!done) R.status = FT_E_NOCONV;
        if (R.status != FT_OK && (worst == FT_OK || R.status == FT_E_NONFINITE)) worst = ft_status(R.status);
    }
    if (worst == FT_E_NONFINITE) set_error("%llu non-finite query value(s) were consumed", nonfinite);
    else if (worst == FT_E_NOCONV) set_error("CG did not reach rtol=%g within %d iterations", cfg->rtol, cfg->max_iter);
    return worst;
}

}  // namespace ft
