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
// Reductions without atomics: every kernel writes one partial sum per block
// (fixed grid-stride rows, fixed block tree), and the kernel that needs the
// total has each of its blocks add the partials in block order.  The totals
// are therefore bitwise identical in every block and from run to run, and no
// counter or memset is involved (the sequence can be captured in a graph).
// Each CG iteration is two kernels: (direction + product + p.q) and
// (update + r.z + r.r); the direction p = z + beta p_old is formed on the fly
// from two alternating buffers.
#include <algorithm>
#include <cmath>

#include "common.h"

namespace ft {

constexpr int RB = 256;            // threads per block in the solver kernels
constexpr int MAX_RBLOCKS = 512;   // grid size cap (grid-stride loops beyond it)

// partial-sum slots (each nb doubles) and device scalar slots
enum { P_BB = 0, P_SB, P_RZ, P_RR, P_PQ, P_TRR, P_MX, P_COUNT };
enum { S_RHO0 = 0, S_RHO1, S_TOL2, S_DONE, S_ITERS, S_BB, S_SUMB, S_TRR, S_INTX, S_COUNT };

__device__ __forceinline__ double block_total(double v) {
    __shared__ double sm[RB / 64];
    __shared__ double tot;
    v = wave_sum_xor(v, 64);
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = sm[0];
        for (int k = 1; k < RB / 64; ++k) s += sm[k];
        tot = s;
    }
    __syncthreads();
    const double t = tot;
    __syncthreads();
    return t;
}

// Sum of the nb partials of one slot, in block order (same value in every block).
__device__ __forceinline__ double partial_total(const double* __restrict__ part, int slot, int nb) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += RB) s += part[slot * nb + b];
    return block_total(s);
}

__device__ __forceinline__ void write_partial(double* __restrict__ part, int slot, double v) {
    const double t = block_total(v);
    if (threadIdx.x == 0) part[slot * gridDim.x + blockIdx.x] = t;
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

#define FOR_ROW(i) for (int64_t i = int64_t(blockIdx.x) * RB + threadIdx.x; i < A.n; i += int64_t(gridDim.x) * RB)

// b = alpha M g + b_res; partials of ||b||^2 and sum b.
__global__ __launch_bounds__(RB) void k_rhs(Mat A, const double* __restrict__ g, const double* __restrict__ bres,
                                            double alpha, double* __restrict__ b, double* __restrict__ part) {
    double bb = 0.0, sb = 0.0;
    FOR_ROW(i) {
        const double bi = alpha * csr_row(A.rowptr, A.col, A.val, g, i) + bres[i];
        b[i] = bi;
        bb = fma(bi, bi, bb);
        sb += bi;
    }
    write_partial(part, P_BB, bb);
    write_partial(part, P_SB, sb);
}

// y = 0, r = b_res, z = D^-1 r, p_old = 0 (beta = 0 makes the first direction z);
// partials of r.z and r.r; block 0 records the stopping threshold.
__global__ __launch_bounds__(RB) void k_cg_init(Mat A, const double* __restrict__ bres, double rtol2,
                                                double* __restrict__ y, double* __restrict__ r, double* __restrict__ z,
                                                double* __restrict__ p_old, double* __restrict__ part,
                                                double* __restrict__ scal) {
    double rz = 0.0, rr = 0.0;
    FOR_ROW(i) {
        const double ri = bres[i];
        const double zi = ri / A.diag[i];
        y[i] = 0.0;
        r[i] = ri;
        z[i] = zi;
        p_old[i] = 0.0;
        rz = fma(ri, zi, rz);
        rr = fma(ri, ri, rr);
    }
    const double bb = partial_total(part, P_BB, gridDim.x);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        scal[S_TOL2] = rtol2 * bb;
        scal[S_DONE] = 0.0;
        scal[S_ITERS] = 0.0;
    }
    write_partial(part, P_RZ, rz);
    write_partial(part, P_RR, rr);
}

// Iteration k, first half: convergence test on ||r_k||; beta = rz_k / rz_{k-1};
// p = z + beta p_old (own rows into p_new), q = M p (p formed on the fly at the
// neighbours), partials of p.q.  A non-finite residual also stops (reported as
// non-finite by the caller).
__global__ __launch_bounds__(RB) void k_cg_spmv(Mat A, int k, const double* __restrict__ z,
                                                const double* __restrict__ p_old, double* __restrict__ p_new,
                                                double* __restrict__ q, double* __restrict__ part,
                                                double* __restrict__ scal) {
    if (scal[S_DONE] != 0.0) return;
    const double rz = partial_total(part, P_RZ, gridDim.x);
    const double rr = partial_total(part, P_RR, gridDim.x);
    if (rr <= scal[S_TOL2] || !isfinite(rr)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            scal[S_DONE] = 1.0;
            scal[S_ITERS] = double(k);
        }
        return;
    }
    const double bt = k == 0 ? 0.0 : rz / scal[S_RHO0 + ((k - 1) & 1)];
    if (blockIdx.x == 0 && threadIdx.x == 0) scal[S_RHO0 + (k & 1)] = rz;
    double pq = 0.0;
    FOR_ROW(i) {
        double qi = 0.0;
        for (int64_t kk = A.rowptr[i]; kk < A.rowptr[i + 1]; ++kk) {
            const int32_t j = A.col[kk];
            qi = fma(A.val[kk], fma(bt, p_old[j], z[j]), qi);
        }
        const double pi = fma(bt, p_old[i], z[i]);
        p_new[i] = pi;
        q[i] = qi;
        pq = fma(pi, qi, pq);
    }
    write_partial(part, P_PQ, pq);
}

// Iteration k, second half: alpha = rz_k / (p.q); y += alpha p; r -= alpha q;
// z = D^-1 r; partials of r.z and r.r for iteration k+1.
__global__ __launch_bounds__(RB) void k_cg_update(Mat A, int k, const double* __restrict__ p,
                                                  const double* __restrict__ q, double* __restrict__ y,
                                                  double* __restrict__ r, double* __restrict__ z,
                                                  double* __restrict__ part, double* __restrict__ scal) {
    if (scal[S_DONE] != 0.0) return;
    const double a = scal[S_RHO0 + (k & 1)] / partial_total(part, P_PQ, gridDim.x);
    double rz = 0.0, rr = 0.0;
    FOR_ROW(i) {
        y[i] = fma(a, p[i], y[i]);
        const double ri = fma(-a, q[i], r[i]);
        const double zi = ri / A.diag[i];
        r[i] = ri;
        z[i] = zi;
        rz = fma(ri, zi, rz);
        rr = fma(ri, ri, rr);
    }
    write_partial(part, P_RZ, rz);
    write_partial(part, P_RR, rr);
}

// After the last launched iteration: the stopping test for the final residual.
__global__ __launch_bounds__(RB) void k_cg_check(int k, int nb, const double* __restrict__ part,
                                                 double* __restrict__ scal) {
    if (scal[S_DONE] != 0.0) return;
    const double rr = partial_total(part, P_RR, nb);
    if (threadIdx.x == 0) {
        scal[S_ITERS] = double(k);
        if (rr <= scal[S_TOL2] || !isfinite(rr)) scal[S_DONE] = 1.0;
    }
}

__global__ __launch_bounds__(RB) void k_solution(int64_t n, const double* __restrict__ g, const double* __restrict__ y,
                                                 double alpha, double* __restrict__ x) {
    for (int64_t i = int64_t(blockIdx.x) * RB + threadIdx.x; i < n; i += int64_t(gridDim.x) * RB)
        x[i] = fma(alpha, g[i], y[i]);
}

// partials of the true residual ||b - M x||^2 and of m^T x
__global__ __launch_bounds__(RB) void k_report(Mat A, const double* __restrict__ b, const double* __restrict__ x,
                                               double* __restrict__ part) {
    double trr = 0.0, mx = 0.0;
    FOR_ROW(i) {
        const double ri = b[i] - csr_row(A.rowptr, A.col, A.val, x, i);
        trr = fma(ri, ri, trr);
        mx = fma(A.lumped[i], x[i], mx);
    }
    write_partial(part, P_TRR, trr);
    write_partial(part, P_MX, mx);
}

__global__ __launch_bounds__(RB) void k_report_totals(int nb, const double* __restrict__ part,
                                                      double* __restrict__ scal) {
    const double bb = partial_total(part, P_BB, nb);
    const double sb = partial_total(part, P_SB, nb);
    const double trr = partial_total(part, P_TRR, nb);
    const double mx = partial_total(part, P_MX, nb);
    if (threadIdx.x == 0) {
        scal[S_BB] = bb;
        scal[S_SUMB] = sb;
        scal[S_TRR] = trr;
        scal[S_INTX] = mx;
    }
}

ft_status solver_alloc(ft_target* T, hipStream_t s) {
    const int64_t n = T->n;
    T->reduce_blocks = int(std::min<int64_t>(MAX_RBLOCKS, (n + RB - 1) / RB));
    if (T->reduce_blocks < 1) T->reduce_blocks = 1;
    FT_TRY(dev_alloc_n(&T->r, size_t(n)));
    FT_TRY(dev_alloc_n(&T->z, size_t(n)));
    FT_TRY(dev_alloc_n(&T->p, size_t(2 * n)));   // two direction buffers, alternating
    FT_TRY(dev_alloc_n(&T->q, size_t(n)));
    FT_TRY(dev_alloc_n(&T->y, size_t(n)));
    FT_TRY(dev_alloc_n(&T->b, size_t(n)));
    FT_TRY(dev_alloc_n(&T->scal, S_COUNT));
    FT_TRY(dev_alloc_n(&T->partials, size_t(T->reduce_blocks) * P_COUNT));
    FT_TRY(dev_alloc_n(&T->counters, 4));
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
    const int nb = T->reduce_blocks;
    Mat A{T->rowptr, T->col, T->val, T->diag, T->lumped, n};
    const double rtol2 = cfg->rtol * cfg->rtol;
    // non-finite values seen by the last consume
    unsigned long long nonfinite = 0;
    FT_TRY_HIP(hipMemcpyAsync(&nonfinite, T->counters, sizeof(nonfinite), hipMemcpyDeviceToHost, s));
    const double* gf = T->g;
    const double* bresf = T->bres;
    double* bf = b_out ? b_out : T->b;
    k_rhs<<<nb, RB, 0, s>>>(A, gf, bresf, alpha, bf, T->partials);
    k_cg_init<<<nb, RB, 0, s>>>(A, bresf, rtol2, T->y, T->r, T->z, T->p, T->partials, T->scal);
    FT_TRY_HIP(hipGetLastError());
    int launched = 0;
    int chunk = 8;
    bool done = false;
    while (true) {
        const int k = std::min(chunk, cfg->max_iter - launched);
        for (int it = 0; it < k; ++it) {
            const int kk = launched + it;
            double* p_old = T->p + ((kk & 1) ? n : 0);
            double* p_new = T->p + ((kk & 1) ? 0 : n);
            k_cg_spmv<<<nb, RB, 0, s>>>(A, kk, T->z, p_old, p_new, T->q, T->partials, T->scal);
            k_cg_update<<<nb, RB, 0, s>>>(A, kk, p_new, T->q, T->y, T->r, T->z, T->partials, T->scal);
        }
        launched += k;
        k_cg_check<<<1, RB, 0, s>>>(launched, nb, T->partials, T->scal);
        FT_TRY_HIP(hipGetLastError());
        FT_TRY_HIP(hipMemcpyAsync(T->h_scal, T->scal, S_COUNT * sizeof(double), hipMemcpyDeviceToHost, s));
        FT_TRY_HIP(hipStreamSynchronize(s));
        if (T->h_scal[S_DONE] != 0.0) {
            done = true;
            break;
        }
        if (launched >= cfg->max_iter) break;
        chunk = 4;
    }
    k_solution<<<nb, RB, 0, s>>>(n, gf, T->y, alpha, x);
    k_report<<<nb, RB, 0, s>>>(A, bf, x, T->partials);
    k_report_totals<<<1, RB, 0, s>>>(nb, T->partials, T->scal);
    FT_TRY_HIP(hipGetLastError());
    FT_TRY_HIP(hipMemcpyAsync(T->h_scal, T->scal, S_COUNT * sizeof(double), hipMemcpyDeviceToHost, s));
    FT_TRY_HIP(hipStreamSynchronize(s));
    const double* h = T->h_scal;
    ft_report& R = rep[0];
    R.sum_b = h[S_SUMB];
    R.int_x = h[S_INTX];
    R.cons_defect = h[S_SUMB] != 0.0 ? std::fabs(h[S_INTX] - h[S_SUMB]) / std::fabs(h[S_SUMB]) : std::fabs(h[S_INTX]);
    R.rel_resid = h[S_BB] > 0.0 ? std::sqrt(h[S_TRR] / h[S_BB]) : std::sqrt(h[S_TRR]);
    R.iters = int32_t(h[S_ITERS]);
    R.n_nonfinite = int64_t(nonfinite);
    R.status = FT_OK;
    if (nonfinite) R.status = FT_E_NONFINITE;
    else if (!done) R.status = FT_E_NOCONV;
    if (R.status == FT_E_NONFINITE) set_error("%llu non-finite query value(s) were consumed", nonfinite);
    else if (R.status == FT_E_NOCONV) set_error("CG did not reach rtol=%g within %d iterations", cfg->rtol, cfg->max_iter);
    return ft_status(R.status);
}

}  // namespace ft
