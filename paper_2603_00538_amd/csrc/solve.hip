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

#include "solve_common.h"

namespace ft {

// b = alpha M g + b_res; partials of ||b||^2 and of sum b (compensated).
__global__ __launch_bounds__(RB) void k_rhs(Mat A, const double* __restrict__ g, const double* __restrict__ bres,
                                            double alpha, double* __restrict__ b, double* __restrict__ part) {
    double bb = 0.0, sb = 0.0, sbc = 0.0;
    FOR_ROW(i) {
        const double bi = alpha * csr_row(A.rowptr, A.col, A.val, g, i) + bres[i];
        b[i] = bi;
        bb = fma(bi, bi, bb);
        comp_add(sb, sbc, bi);
    }
    write_partial(part, P_BB, bb);
    write_partial_comp(part, P_SB, sb, sbc);
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
template <int NT>
__global__ __launch_bounds__(NT) void k_cg_spmv(Mat A, int k, const double* __restrict__ z,
                                                const double* __restrict__ p_old, double* __restrict__ p_new,
                                                double* __restrict__ q, double* __restrict__ part,
                                                double* __restrict__ scal) {
    if (scal[S_DONE] != 0.0) return;
    const double rz = partial_total<NT>(part, P_RZ, gridDim.x);
    const double rr = partial_total<NT>(part, P_RR, gridDim.x);
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
    FOR_ROW_NT(i, NT) {
        const double qi = row_dot4(A.col, A.val, A.rowptr[i], A.rowptr[i + 1],
                                   [&](int32_t j) { return fma(bt, p_old[j], z[j]); });
        const double pi = fma(bt, p_old[i], z[i]);
        p_new[i] = pi;
        q[i] = qi;
        pq = fma(pi, qi, pq);
    }
    write_partial<NT>(part, P_PQ, pq);
}

// The same iteration for matrices with long rows (P2 tetrahedra: about 30
// entries a row): L lanes per row walk its entries together (consecutive
// entries, so each load of the matrix is a contiguous run) and add their
// parts with a butterfly; a block takes RB / L rows per pass.
template <int L, int NT>
__global__ __launch_bounds__(NT) void k_cg_spmv_rows(Mat A, int k, const double* __restrict__ z,
                                                     const double* __restrict__ p_old, double* __restrict__ p_new,
                                                     double* __restrict__ q, double* __restrict__ part,
                                                     double* __restrict__ scal) {
    if (scal[S_DONE] != 0.0) return;
    const double rz = partial_total<NT>(part, P_RZ, gridDim.x);
    const double rr = partial_total<NT>(part, P_RR, gridDim.x);
    if (rr <= scal[S_TOL2] || !isfinite(rr)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            scal[S_DONE] = 1.0;
            scal[S_ITERS] = double(k);
        }
        return;
    }
    const double bt = k == 0 ? 0.0 : rz / scal[S_RHO0 + ((k - 1) & 1)];
    if (blockIdx.x == 0 && threadIdx.x == 0) scal[S_RHO0 + (k & 1)] = rz;
    const int sub = int(threadIdx.x) & (L - 1);
    double pq = 0.0;
    for (int64_t i0 = int64_t(blockIdx.x) * (NT / L); i0 < A.n; i0 += int64_t(gridDim.x) * (NT / L)) {
        const int64_t i = i0 + int(threadIdx.x) / L;
        double qi = 0.0;
        if (i < A.n) {
            const int64_t k1 = A.rowptr[i + 1];
            for (int64_t kk = A.rowptr[i] + sub; kk < k1; kk += L) {
                const int32_t j = A.col[kk];
                qi = fma(A.val[kk], fma(bt, p_old[j], z[j]), qi);
            }
        }
#pragma unroll
        for (int o = L / 2; o > 0; o >>= 1) qi += __shfl_xor(qi, o, L);
        if (i < A.n && sub == 0) {
            const double pi = fma(bt, p_old[i], z[i]);
            p_new[i] = pi;
            q[i] = qi;
            pq = fma(pi, qi, pq);
        }
    }
    write_partial<NT>(part, P_PQ, pq);
}

// Rows this long or longer on average take the lanes-per-row product.
constexpr int kLongRows = 24;

// Threads per block of the CG iteration kernels for long rows.  Their grid is
// capped by the number of block partials (at most MAX_RBLOCKS, which every
// block of the next kernel adds up), so wide blocks are what keeps enough
// loads in flight: with 256 threads the P2 tetrahedral product ran two waves
// per SIMD at 1.9 TB/s, with 1024 eight.  (The P1 matrices ran slower with
// wide blocks and keep RB.)
constexpr int kCgWide = 1024;

// Iteration k, second half: alpha = rz_k / (p.q); y += alpha p; r -= alpha q;
// z = D^-1 r; partials of r.z and r.r for iteration k+1.
template <int NT>
__global__ __launch_bounds__(NT) void k_cg_update(Mat A, int k, const double* __restrict__ p,
                                                  const double* __restrict__ q, double* __restrict__ y,
                                                  double* __restrict__ r, double* __restrict__ z,
                                                  double* __restrict__ part, double* __restrict__ scal) {
    if (scal[S_DONE] != 0.0) return;
    const double a = scal[S_RHO0 + (k & 1)] / partial_total<NT>(part, P_PQ, gridDim.x);
    double rz = 0.0, rr = 0.0;
    FOR_ROW_NT(i, NT) {
        y[i] = fma(a, p[i], y[i]);
        const double ri = fma(-a, q[i], r[i]);
        const double zi = ri / A.diag[i];
        r[i] = ri;
        z[i] = zi;
        rz = fma(ri, zi, rz);
        rr = fma(ri, ri, rr);
    }
    write_partial<NT>(part, P_RZ, rz);
    write_partial<NT>(part, P_RR, rr);
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

// partials of the true residual ||b - M x||^2 and of m^T x (compensated: each
// product m_i x_i is split exactly into its rounded value and error by an FMA)
__global__ __launch_bounds__(RB) void k_report(Mat A, const double* __restrict__ b, const double* __restrict__ x,
                                               double* __restrict__ part) {
    double trr = 0.0, mx = 0.0, mxc = 0.0;
    FOR_ROW(i) {
        const double ri = b[i] - csr_row(A.rowptr, A.col, A.val, x, i);
        trr = fma(ri, ri, trr);
        const double pr = A.lumped[i] * x[i];
        mxc += fma(A.lumped[i], x[i], -pr);
        comp_add(mx, mxc, pr);
    }
    write_partial(part, P_TRR, trr);
    write_partial_comp(part, P_MX, mx, mxc);
}

__global__ __launch_bounds__(RB) void k_report_totals(int nb, const double* __restrict__ part,
                                                      double* __restrict__ scal) {
    const double bb = partial_total(part, P_BB, nb);
    const double sb = partial_total_comp(part, P_SB, nb);
    const double trr = partial_total(part, P_TRR, nb);
    const double mx = partial_total_comp(part, P_MX, nb);
    if (threadIdx.x == 0) {
        scal[S_BB] = bb;
        scal[S_SUMB] = sb;
        scal[S_TRR] = trr;
        scal[S_INTX] = mx;
    }
}

// ---- the standard error of sum b (App. B, Eq. cv_global_integral_estimator:
// the element totals are independent, so the variance of sum b is the sum of
// the element variances).  Per field: block partials over contiguous element
// ranges, then their total in block order; compensated throughout.
__global__ __launch_bounds__(RB) void k_var_partials(const double* __restrict__ var_el, int64_t E,
                                                     double* __restrict__ part) {
    const int f = blockIdx.y;
    const int64_t chunk = (E + kVarBlocks - 1) / kVarBlocks;
    const int64_t b0 = int64_t(blockIdx.x) * chunk, b1 = b0 + chunk < E ? b0 + chunk : E;
    double s = 0.0, c = 0.0;
    for (int64_t i = b0 + threadIdx.x; i < b1; i += RB) comp_add(s, c, var_el[int64_t(f) * E + i]);
    block_total_comp(s, c);
    if (threadIdx.x == 0) {
        part[(int64_t(f) * kVarBlocks + blockIdx.x) * 2] = s;
        part[(int64_t(f) * kVarBlocks + blockIdx.x) * 2 + 1] = c;
    }
}

__global__ __launch_bounds__(RB) void k_var_total(const double* __restrict__ part, double* __restrict__ tot) {
    const int f = blockIdx.x;
    double s = 0.0, c = 0.0;
    if (threadIdx.x < kVarBlocks) {
        s = part[(int64_t(f) * kVarBlocks + threadIdx.x) * 2];
        c = part[(int64_t(f) * kVarBlocks + threadIdx.x) * 2 + 1];
    }
    block_total_comp(s, c);
    if (threadIdx.x == 0) tot[f] = s + c;
}

ft_status stderr_launch(ft_target* T, int F, hipStream_t s) {
    if (T->var_mode != VAR_ESTIMATED) return FT_OK;
    k_var_partials<<<dim3(kVarBlocks, unsigned(F)), RB, 0, s>>>(T->var_el, T->E, T->var_part);
    k_var_total<<<unsigned(F), RB, 0, s>>>(T->var_part, T->var_tot);
    FT_TRY_HIP(hipGetLastError());
    FT_TRY_HIP(hipMemcpyAsync(T->h_var, T->var_tot, size_t(F) * sizeof(double), hipMemcpyDeviceToHost, s));
    return FT_OK;
}

// after the stream has been synchronized
void stderr_fill(const ft_target* T, int F, ft_report* rep) {
    for (int f = 0; f < F; ++f)
        // (a sum that is not finite: some element had a single sample, or a value was not finite)
        rep[f].sum_b_stderr = T->var_mode == VAR_ESTIMATED ? (std::isfinite(T->h_var[f]) ? std::sqrt(T->h_var[f]) : -1.0)
                              : T->var_mode == VAR_EXACT   ? 0.0
                                                           : -1.0;
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

// ---------------------------------------------------------------- mixed precision
// Binary64 residual and iterative refinement around a binary32 inner solve
// (sec. 4.1 step 7 in the binary32 form).  Outer: r = b_res - M y in binary64;
// stop when ||r|| <= rtol ||b|| (the true residual of M x = b, x = alpha g + y).
// Inner: Jacobi-PCG on M d = r with binary32 matrix values and vectors and
// binary64 accumulation of every dot product, to ||r - M d|| <= 1e-6 ||r||
// (binary32 carries about seven digits and D^-1 M is well conditioned, so each
// step gains about six); then y += d.
constexpr double kInnerRtol = 1e-6;
enum { M_RHO0 = 0, M_RHO1, M_TOL2, M_DONE, M_ITERS, M_COUNT };

struct Mat32 {
    const int64_t* rowptr;
    const int32_t* col;
    const float* val;
    const float* diag;
    int64_t n;
};

__global__ void k_to_f32(const double* __restrict__ src, int64_t n, float* __restrict__ dst) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
        dst[i] = float(src[i]);
}

// y = 0, r = b_res; partial of ||r||^2
__global__ __launch_bounds__(RB) void k_mx_start(Mat A, const double* __restrict__ bres, double* __restrict__ y,
                                                 double* __restrict__ r, double* __restrict__ part) {
    double rr = 0.0;
    FOR_ROW(i) {
        const double ri = bres[i];
        y[i] = 0.0;
        r[i] = ri;
        rr = fma(ri, ri, rr);
    }
    write_partial(part, P_RR, rr);
}

// outer residual r = b_res - M y (binary64); partial of ||r||^2
__global__ __launch_bounds__(RB) void k_mx_resid(Mat A, const double* __restrict__ bres, const double* __restrict__ y,
                                                 double* __restrict__ r, double* __restrict__ part) {
    double rr = 0.0;
    FOR_ROW(i) {
        const double ri = bres[i] - csr_row(A.rowptr, A.col, A.val, y, i);
        r[i] = ri;
        rr = fma(ri, ri, rr);
    }
    write_partial(part, P_RR, rr);
}

// one block: the outer totals (mode 0: also ||b||^2, sum b and the threshold)
__global__ __launch_bounds__(RB) void k_mx_totals(int mode, int nb, double rtol2, const double* __restrict__ part,
                                                  double* __restrict__ scal) {
    const double rr = partial_total(part, P_RR, nb);
    if (mode == 0) {
        const double bb = partial_total(part, P_BB, nb);
        const double sb = partial_total_comp(part, P_SB, nb);
        if (threadIdx.x == 0) {
            scal[S_BB] = bb;
            scal[S_SUMB] = sb;
            scal[S_TOL2] = rtol2 * bb;
        }
    }
    if (threadIdx.x == 0) scal[S_TRR] = rr;
}

// inner start: r32 = r, z32 = D^-1 r32, d = 0, p_old = 0; partials of r.z, r.r
__global__ __launch_bounds__(RB) void k_m32_init(Mat32 A, const double* __restrict__ r64, float* __restrict__ r,
                                                 float* __restrict__ z, float* __restrict__ d,
                                                 float* __restrict__ p_old, double* __restrict__ part,
                                                 double* __restrict__ sc) {
    double rz = 0.0, rr = 0.0;
    FOR_ROW(i) {
        const float ri = float(r64[i]);
        const float zi = ri / A.diag[i];
        r[i] = ri;
        z[i] = zi;
        d[i] = 0.0f;
        p_old[i] = 0.0f;
        rz = fma(double(ri), double(zi), rz);
        rr = fma(double(ri), double(ri), rr);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc[M_DONE] = 0.0;
        sc[M_ITERS] = 0.0;
    }
    write_partial(part, P_RZ, rz);
    write_partial(part, P_RR, rr);
}

__global__ __launch_bounds__(RB) void k_m32_spmv(Mat32 A, int k, const float* __restrict__ z,
                                                 const float* __restrict__ p_old, float* __restrict__ p_new,
                                                 float* __restrict__ q, double* __restrict__ part,
                                                 double* __restrict__ sc) {
    if (sc[M_DONE] != 0.0) return;
    const double rz = partial_total(part, P_RZ, gridDim.x);
    const double rr = partial_total(part, P_RR, gridDim.x);
    const double tol2 = k == 0 ? kInnerRtol * kInnerRtol * rr : sc[M_TOL2];
    if (k == 0 && blockIdx.x == 0 && threadIdx.x == 0) sc[M_TOL2] = tol2;
    if (rr <= tol2 || !isfinite(rr)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            sc[M_DONE] = 1.0;
            sc[M_ITERS] = double(k);
        }
        return;
    }
    const float bt = k == 0 ? 0.0f : float(rz / sc[M_RHO0 + ((k - 1) & 1)]);
    if (blockIdx.x == 0 && threadIdx.x == 0) sc[M_RHO0 + (k & 1)] = rz;
    double pq = 0.0;
    FOR_ROW(i) {
        const float qi = row_dot4(A.col, A.val, A.rowptr[i], A.rowptr[i + 1],
                                  [&](int32_t j) { return fmaf(bt, p_old[j], z[j]); });
        const float pi = fmaf(bt, p_old[i], z[i]);
        p_new[i] = pi;
        q[i] = qi;
        pq = fma(double(pi), double(qi), pq);
    }
    write_partial(part, P_PQ, pq);
}

// The binary32 product for long rows: L lanes per row and NT-thread blocks,
// as k_cg_spmv_rows.
template <int L, int NT>
__global__ __launch_bounds__(NT) void k_m32_spmv_rows(Mat32 A, int k, const float* __restrict__ z,
                                                      const float* __restrict__ p_old, float* __restrict__ p_new,
                                                      float* __restrict__ q, double* __restrict__ part,
                                                      double* __restrict__ sc) {
    if (sc[M_DONE] != 0.0) return;
    const double rz = partial_total<NT>(part, P_RZ, gridDim.x);
    const double rr = partial_total<NT>(part, P_RR, gridDim.x);
    const double tol2 = k == 0 ? kInnerRtol * kInnerRtol * rr : sc[M_TOL2];
    if (k == 0 && blockIdx.x == 0 && threadIdx.x == 0) sc[M_TOL2] = tol2;
    if (rr <= tol2 || !isfinite(rr)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            sc[M_DONE] = 1.0;
            sc[M_ITERS] = double(k);
        }
        return;
    }
    const float bt = k == 0 ? 0.0f : float(rz / sc[M_RHO0 + ((k - 1) & 1)]);
    if (blockIdx.x == 0 && threadIdx.x == 0) sc[M_RHO0 + (k & 1)] = rz;
    const int sub = int(threadIdx.x) & (L - 1);
    double pq = 0.0;
    for (int64_t i0 = int64_t(blockIdx.x) * (NT / L); i0 < A.n; i0 += int64_t(gridDim.x) * (NT / L)) {
        const int64_t i = i0 + int(threadIdx.x) / L;
        float qi = 0.0f;
        if (i < A.n) {
            const int64_t k1 = A.rowptr[i + 1];
            for (int64_t kk = A.rowptr[i] + sub; kk < k1; kk += L) {
                const int32_t j = A.col[kk];
                qi = fmaf(A.val[kk], fmaf(bt, p_old[j], z[j]), qi);
            }
        }
#pragma unroll
        for (int o = L / 2; o > 0; o >>= 1) qi += __shfl_xor(qi, o, L);
        if (i < A.n && sub == 0) {
            const float pi = fmaf(bt, p_old[i], z[i]);
            p_new[i] = pi;
            q[i] = qi;
            pq = fma(double(pi), double(qi), pq);
        }
    }
    write_partial<NT>(part, P_PQ, pq);
}

template <int NT>
__global__ __launch_bounds__(NT) void k_m32_update(Mat32 A, int k, const float* __restrict__ p,
                                                   const float* __restrict__ q, float* __restrict__ d,
                                                   float* __restrict__ r, float* __restrict__ z,
                                                   double* __restrict__ part, const double* __restrict__ sc) {
    if (sc[M_DONE] != 0.0) return;
    const float a = float(sc[M_RHO0 + (k & 1)] / partial_total<NT>(part, P_PQ, gridDim.x));
    double rz = 0.0, rr = 0.0;
    FOR_ROW_NT(i, NT) {
        d[i] = fmaf(a, p[i], d[i]);
        const float ri = fmaf(-a, q[i], r[i]);
        const float zi = ri / A.diag[i];
        r[i] = ri;
        z[i] = zi;
        rz = fma(double(ri), double(zi), rz);
        rr = fma(double(ri), double(ri), rr);
    }
    write_partial<NT>(part, P_RZ, rz);
    write_partial<NT>(part, P_RR, rr);
}

__global__ __launch_bounds__(RB) void k_m32_check(int k, int nb, const double* __restrict__ part,
                                                  double* __restrict__ sc) {
    if (sc[M_DONE] != 0.0) return;
    const double rr = partial_total(part, P_RR, nb);
    if (threadIdx.x == 0) {
        sc[M_ITERS] = double(k);
        if (rr <= sc[M_TOL2] || !isfinite(rr)) sc[M_DONE] = 1.0;
    }
}

// y += d (binary32 correction into the binary64 iterate)
__global__ void k_mx_apply(int64_t n, const float* __restrict__ d, double* __restrict__ y) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
        y[i] += double(d[i]);
}

static ft_status mixed_alloc(ft_target* T, hipStream_t s) {
    if (T->val32) return FT_OK;
    FT_TRY(dev_alloc_n(&T->val32, size_t(T->nnz)));
    FT_TRY(dev_alloc_n(&T->diag32, size_t(T->n)));
    FT_TRY(dev_alloc_n(&T->w32, size_t(6) * T->n));
    FT_TRY(dev_alloc_n(&T->scal32, size_t(M_COUNT)));
    k_to_f32<<<grid_for(T->nnz, 256), 256, 0, s>>>(T->val, T->nnz, T->val32);
    k_to_f32<<<grid_for(T->n, 256), 256, 0, s>>>(T->diag, T->n, T->diag32);
    FT_TRY_HIP(hipGetLastError());
    return FT_OK;
}

static ft_status read_scalars(ft_target* T, const double* src, int count, hipStream_t s) {
    FT_TRY_HIP(hipMemcpyAsync(T->h_scal, src, sizeof(double) * count, hipMemcpyDeviceToHost, s));
    FT_TRY_HIP(hipStreamSynchronize(s));
    return FT_OK;
}

static ft_status project_mixed(ft_target* T, const ft_solve_cfg* cfg, double* x, double* b_out, ft_report* rep,
                               hipStream_t s) {
    FT_TRY(mixed_alloc(T, s));
    const double alpha = T->consumed_cfg.alpha;
    const int64_t n = T->n;
    const int nb = T->reduce_blocks;
    Mat A{T->rowptr, T->col, T->val, T->diag, T->lumped, n};
    Mat32 A32{T->rowptr, T->col, T->val32, T->diag32, n};
    float* r32 = T->w32;
    float* z32 = r32 + n;
    float* p32 = z32 + n;   // two buffers
    float* q32 = p32 + 2 * n;
    float* d32 = q32 + n;
    unsigned long long cnt[2] = {0, 0};   // non-finite values, out-of-domain queries
    FT_TRY_HIP(hipMemcpyAsync(cnt, T->counters, sizeof(cnt), hipMemcpyDeviceToHost, s));
    double* bf = b_out ? b_out : T->b;
    k_rhs<<<nb, RB, 0, s>>>(A, T->g, T->bres, alpha, bf, T->partials);
    k_mx_start<<<nb, RB, 0, s>>>(A, T->bres, T->y, T->r, T->partials);
    k_mx_totals<<<1, RB, 0, s>>>(0, nb, cfg->rtol * cfg->rtol, T->partials, T->scal);
    FT_TRY_HIP(hipGetLastError());
    FT_TRY(read_scalars(T, T->scal, S_COUNT, s));
    const double tol2 = T->h_scal[S_TOL2];
    double rr = T->h_scal[S_TRR];
    int iters = 0;
    bool done = rr <= tol2 || !std::isfinite(rr);
    const bool long_rows = T->nnz >= kLongRows * n;
    for (int step = 0; step < cfg->refine_steps && !done; ++step) {
        k_m32_init<<<nb, RB, 0, s>>>(A32, T->r, r32, z32, d32, p32, T->partials, T->scal32);
        int launched = 0, chunk = first_chunk(T->cg_hint[1]);
        while (launched < cfg->max_iter) {
            const int k = std::min(chunk, cfg->max_iter - launched);
            for (int it = 0; it < k; ++it) {
                const int kk = launched + it;
                float* p_old = p32 + ((kk & 1) ? n : 0);
                float* p_new = p32 + ((kk & 1) ? 0 : n);
                if (long_rows) {
                    k_m32_spmv_rows<8, kCgWide><<<nb, kCgWide, 0, s>>>(A32, kk, z32, p_old, p_new, q32,
                                                                      T->partials, T->scal32);
                    k_m32_update<kCgWide><<<nb, kCgWide, 0, s>>>(A32, kk, p_new, q32, d32, r32, z32, T->partials,
                                                                T->scal32);
                } else {
                    k_m32_spmv<<<nb, RB, 0, s>>>(A32, kk, z32, p_old, p_new, q32, T->partials, T->scal32);
                    k_m32_update<RB><<<nb, RB, 0, s>>>(A32, kk, p_new, q32, d32, r32, z32, T->partials, T->scal32);
                }
            }
            launched += k;
            k_m32_check<<<1, RB, 0, s>>>(launched, nb, T->partials, T->scal32);
            FT_TRY_HIP(hipGetLastError());
            FT_TRY(read_scalars(T, T->scal32, M_COUNT, s));
            if (T->h_scal[M_DONE] != 0.0) break;
            chunk = 4;
        }
        iters += int(T->h_scal[M_ITERS]);
        T->cg_hint[1] = int(T->h_scal[M_ITERS]);
        k_mx_apply<<<grid_for(n, 256), 256, 0, s>>>(n, d32, T->y);
        k_mx_resid<<<nb, RB, 0, s>>>(A, T->bres, T->y, T->r, T->partials);
        k_mx_totals<<<1, RB, 0, s>>>(1, nb, 0.0, T->partials, T->scal);
        FT_TRY_HIP(hipGetLastError());
        FT_TRY(read_scalars(T, T->scal, S_COUNT, s));
        rr = T->h_scal[S_TRR];
        done = rr <= tol2 || !std::isfinite(rr);
    }
    k_solution<<<nb, RB, 0, s>>>(n, T->g, T->y, alpha, x);
    k_report<<<nb, RB, 0, s>>>(A, bf, x, T->partials);
    k_report_totals<<<1, RB, 0, s>>>(nb, T->partials, T->scal);
    FT_TRY_HIP(hipGetLastError());
    FT_TRY(read_scalars(T, T->scal, S_COUNT, s));
    const double* h = T->h_scal;
    ft_report& R = rep[0];
    R.sum_b = h[S_SUMB];
    R.int_x = h[S_INTX];
    R.cons_defect = h[S_SUMB] != 0.0 ? std::fabs(h[S_INTX] - h[S_SUMB]) / std::fabs(h[S_SUMB]) : std::fabs(h[S_INTX]);
    R.rel_resid = h[S_BB] > 0.0 ? std::sqrt(h[S_TRR] / h[S_BB]) : std::sqrt(h[S_TRR]);
    R.iters = iters;
    R.n_nonfinite = int64_t(cnt[0]);
    R.n_out_of_domain = report_ood(T, cnt);
    R.status = cnt[0] ? FT_E_NONFINITE : (done ? FT_OK : FT_E_NOCONV);
    if (R.status == FT_E_NONFINITE) set_error("%llu non-finite query value(s) were consumed", cnt[0]);
    else if (R.status == FT_E_NOCONV)
        set_error("refinement did not reach rtol=%g within %d steps", cfg->rtol, cfg->refine_steps);
    return ft_status(R.status);
}

static ft_status project_one(ft_target* T, const ft_solve_cfg* cfg, double* x, double* b_out, ft_report* rep,
                             hipStream_t s) {
    const int F = T->consumed_cfg.n_fields;
    if (cfg->refine_steps > 0) {
        if (F > 1) {
            set_error("the mixed-precision solve (refine_steps > 0) handles one field per call");
            return FT_E_UNSUPPORTED;
        }
        return project_mixed(T, cfg, x, b_out, rep, s);
    }
    if (F > 1) return project_multi(T, cfg, x, b_out, rep, s);
    const double alpha = T->consumed_cfg.alpha;
    const int64_t n = T->n;
    const int nb = T->reduce_blocks;
    Mat A{T->rowptr, T->col, T->val, T->diag, T->lumped, n};
    const double rtol2 = cfg->rtol * cfg->rtol;
    // non-finite values seen by the last consume, out-of-domain queries of the last transfer
    unsigned long long cnt[2] = {0, 0};
    FT_TRY_HIP(hipMemcpyAsync(cnt, T->counters, sizeof(cnt), hipMemcpyDeviceToHost, s));
    const double* gf = T->g;
    const double* bresf = T->bres;
    double* bf = b_out ? b_out : T->b;
    k_rhs<<<nb, RB, 0, s>>>(A, gf, bresf, alpha, bf, T->partials);
    k_cg_init<<<nb, RB, 0, s>>>(A, bresf, rtol2, T->y, T->r, T->z, T->p, T->partials, T->scal);
    FT_TRY_HIP(hipGetLastError());
    int launched = 0;
    int chunk = first_chunk(T->cg_hint[0]);
    bool done = false;
    const bool long_rows = T->nnz >= kLongRows * n;
    while (true) {
        const int k = std::min(chunk, cfg->max_iter - launched);
        for (int it = 0; it < k; ++it) {
            const int kk = launched + it;
            double* p_old = T->p + ((kk & 1) ? n : 0);
            double* p_new = T->p + ((kk & 1) ? 0 : n);
            if (long_rows) {
                k_cg_spmv_rows<8, kCgWide><<<nb, kCgWide, 0, s>>>(A, kk, T->z, p_old, p_new, T->q, T->partials,
                                                                 T->scal);
                k_cg_update<kCgWide><<<nb, kCgWide, 0, s>>>(A, kk, p_new, T->q, T->y, T->r, T->z, T->partials,
                                                           T->scal);
            } else {
                k_cg_spmv<RB><<<nb, RB, 0, s>>>(A, kk, T->z, p_old, p_new, T->q, T->partials, T->scal);
                k_cg_update<RB><<<nb, RB, 0, s>>>(A, kk, p_new, T->q, T->y, T->r, T->z, T->partials, T->scal);
            }
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
    T->cg_hint[0] = R.iters;
    R.n_nonfinite = int64_t(cnt[0]);
    R.n_out_of_domain = report_ood(T, cnt);
    R.status = FT_OK;
    if (cnt[0]) R.status = FT_E_NONFINITE;
    else if (!done) R.status = FT_E_NOCONV;
    if (R.status == FT_E_NONFINITE) set_error("%llu non-finite query value(s) were consumed", cnt[0]);
    else if (R.status == FT_E_NOCONV) set_error("CG did not reach rtol=%g within %d iterations", cfg->rtol, cfg->max_iter);
    return ft_status(R.status);
}

// Every form of the solve, then the standard error of sum b per field (the
// element variances are summed on the stream before the solve; each form
// synchronizes before it fills its reports).
ft_status project(ft_target* T, const ft_solve_cfg* cfg, double* x, double* b_out, ft_report* rep, hipStream_t s) {
    const int F = T->consumed_cfg.n_fields;
    FT_TRY(stderr_launch(T, F, s));
    const ft_status st = project_one(T, cfg, x, b_out, rep, s);
    if (st == FT_OK || st == FT_E_NOCONV || st == FT_E_NONFINITE) stderr_fill(T, F, rep);
    return st;
}

}  // namespace ft
