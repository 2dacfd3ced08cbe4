// Variance-driven samples per element.
//
// The conservation error of the CV-MC load vector is the sampling error of
// sum b (App. B, Eq. conservation_residual_bound); with N_t independent
// samples in element t its variance is sum_t |Omega_t|^2 sigma_t^2 / N_t,
// sigma_t^2 the variance of the residual f^s - alpha g over the element
// (Eq. cv_global_integral_estimator).  Sec. 7 names better sampling as the
// way forward; for a total of B samples this variance is smallest with N_t
// proportional to a_t = |Omega_t| sigma_t (Neyman allocation: minimize
// sum a_t^2 / N_t subject to sum N_t = B, by a Lagrange multiplier), and then
// equals (sum a_t)^2 / B.
//
// A pilot transfer with N0 >= 2 samples per element has left its element
// variance terms v_t = |Omega_t|^2 s_t^2 / N0 in the target, so
// a_t = sqrt(N0 v_t) estimates |Omega_t| sigma_t.  The allocation is
//   W   = sum_t a_t                   (compensated, in a fixed order)
//   N_t = clamp(floor(B a_t / W + 1/2), n_min, n_max)
// (every N_t = n_min when W = 0), the element's samples occupy positions
// offs[t] .. offs[t+1] - 1 of the query list's sample block (exclusive prefix
// sums), and the prediction of the new standard error is
// sqrt(sum_t a_t^2 / N_t).  Non-finite or negative terms count as a_t = 0.
//
// Kernels: weight partials over kVarBlocks contiguous ranges; per block of
// kAllocChunk elements the count total and the predicted-variance partial;
// one block scans the block totals; then each block writes its offsets from
// the counts (recomputed, not stored) with a block scan.  Integer sums are
// exact and the floating-point ones taken in a fixed order, so the offsets
// are the same on every run.
#include "adaptive.h"
#include "solve_common.h"

namespace ft {

constexpr int kAllocItems = 8;                    // elements per thread per block
constexpr int kAllocChunk = RB * kAllocItems;     // elements per block

struct AllocArgs {
    const double* var;   // [E] variance terms of the chosen field
    int64_t E;
    double n0;           // the pilot's samples per element
    double budget;       // B
    double lo, hi;       // n_min, n_max
};

__device__ __forceinline__ double alloc_weight(const AllocArgs& a, int64_t t) {
    const double x = a.n0 * a.var[t];
    return (x > 0.0 && x < __builtin_huge_val()) ? sqrt(x) : 0.0;
}

__device__ __forceinline__ double alloc_count(const AllocArgs& a, double w, double W) {
    const double c = W > 0.0 ? floor(a.budget * w / W + 0.5) : a.lo;
    return fmin(fmax(c, a.lo), a.hi);
}

// exclusive prefix sum over the block (thread order) and the block's total
__device__ __forceinline__ int64_t block_excl_scan(int64_t x, int64_t& total) {
    __shared__ int64_t ws[RB / 64];
    const int lane = int(threadIdx.x & 63u), w = int(threadIdx.x >> 6);
    int64_t inc = x;
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t y = __shfl_up(inc, o, 64);
        if (lane >= o) inc += y;
    }
    if (lane == 63) ws[w] = inc;
    __syncthreads();
    int64_t before = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < RB / 64; ++k) {
        const int64_t s = ws[k];
        before += k < w ? s : 0;
        tot += s;
    }
    __syncthreads();
    total = tot;
    return before + inc - x;
}

__device__ __forceinline__ int64_t block_sum_i64(int64_t x) {
    int64_t tot;
    (void)block_excl_scan(x, tot);
    return tot;
}

// slot 0/1 of part: the compensated partial of sum a_t over a contiguous range
__global__ __launch_bounds__(RB) void k_alloc_weights(AllocArgs a, double* __restrict__ part) {
    const int64_t chunk = (a.E + kVarBlocks - 1) / kVarBlocks;
    const int64_t b0 = int64_t(blockIdx.x) * chunk, b1 = b0 + chunk < a.E ? b0 + chunk : a.E;
    double s = 0.0, c = 0.0;
    for (int64_t t = b0 + threadIdx.x; t < b1; t += RB) comp_add(s, c, alloc_weight(a, t));
    write_partial_comp(part, 0, s, c);
}

// per block: the total of its counts and the compensated partial of a_t^2 / N_t
__global__ __launch_bounds__(RB) void k_alloc_blocks(AllocArgs a, const double* __restrict__ wpart,
                                                     int64_t* __restrict__ bcnt, double* __restrict__ bvar) {
    const double W = partial_total_comp(wpart, 0, kVarBlocks);
    int64_t cnt = 0;
    double s = 0.0, c = 0.0;
    const int64_t base = int64_t(blockIdx.x) * kAllocChunk;
#pragma unroll
    for (int k = 0; k < kAllocItems; ++k) {
        const int64_t t = base + k * RB + threadIdx.x;
        if (t < a.E) {
            const double w = alloc_weight(a, t);
            const double nt = alloc_count(a, w, W);
            cnt += int64_t(nt);
            comp_add(s, c, w * w / nt);
        }
    }
    const int64_t tot = block_sum_i64(cnt);
    if (threadIdx.x == 0) bcnt[blockIdx.x] = tot;
    write_partial_comp(bvar, 0, s, c);
}

// one block: exclusive scan of the block totals; res = {W, predicted variance},
// offs[E] = the total
__global__ __launch_bounds__(RB) void k_alloc_scan(const double* __restrict__ wpart, const int64_t* __restrict__ bcnt,
                                                   const double* __restrict__ bvar, int nblk, int64_t E,
                                                   int64_t* __restrict__ bpre, double* __restrict__ res,
                                                   int64_t* __restrict__ offs) {
    int64_t carry = 0;
    for (int b0 = 0; b0 < nblk; b0 += RB) {
        const int b = b0 + int(threadIdx.x);
        const int64_t x = b < nblk ? bcnt[b] : 0;
        int64_t tot;
        const int64_t ex = block_excl_scan(x, tot);
        if (b < nblk) bpre[b] = carry + ex;
        carry += tot;
    }
    const double W = partial_total_comp(wpart, 0, kVarBlocks);
    const double pv = partial_total_comp(bvar, 0, nblk);
    if (threadIdx.x == 0) {
        res[0] = W;
        res[1] = pv;
        offs[E] = carry;
    }
}

__global__ __launch_bounds__(RB) void k_alloc_offsets(AllocArgs a, const double* __restrict__ wpart,
                                                      const int64_t* __restrict__ bpre, int64_t* __restrict__ offs) {
    const double W = partial_total_comp(wpart, 0, kVarBlocks);
    int64_t carry = bpre[blockIdx.x];
    const int64_t base = int64_t(blockIdx.x) * kAllocChunk;
    for (int k = 0; k < kAllocItems; ++k) {
        const int64_t t = base + k * RB + threadIdx.x;
        const int64_t nt = t < a.E ? int64_t(alloc_count(a, alloc_weight(a, t), W)) : 0;
        int64_t tot;
        const int64_t ex = block_excl_scan(nt, tot);
        if (t < a.E) offs[t] = carry + ex;
        carry += tot;
    }
}

// device scratch of an allocation over E elements
size_t alloc_scratch_bytes(int64_t E) {
    const int64_t nblk = (E + kAllocChunk - 1) / kAllocChunk;
    return sizeof(double) * size_t(2 * kVarBlocks + 4 * nblk + 4);
}

// var: [E] terms of one field; scratch of alloc_scratch_bytes(E); res_host
// receives {total, W, predicted variance} after the stream has synchronized.
ft_status allocate_samples(const double* var, int64_t E, int n0, int64_t budget, int n_min, int n_max,
                           int64_t* offs, void* scratch, int64_t* total, double* W, double* pred_var,
                           hipStream_t s) {
    const int nblk = int((E + kAllocChunk - 1) / kAllocChunk);
    double* wpart = static_cast<double*>(scratch);
    int64_t* bcnt = reinterpret_cast<int64_t*>(wpart + 2 * kVarBlocks);
    int64_t* bpre = bcnt + nblk;
    double* bvar = reinterpret_cast<double*>(bpre + nblk);
    double* res = bvar + 2 * nblk;
    const AllocArgs a{var, E, double(n0), double(budget), double(n_min), double(n_max)};
    k_alloc_weights<<<kVarBlocks, RB, 0, s>>>(a, wpart);
    k_alloc_blocks<<<nblk, RB, 0, s>>>(a, wpart, bcnt, bvar);
    k_alloc_scan<<<1, RB, 0, s>>>(wpart, bcnt, bvar, nblk, E, bpre, res, offs);
    k_alloc_offsets<<<nblk, RB, 0, s>>>(a, wpart, bpre, offs);
    FT_TRY_HIP(hipGetLastError());
    double h[2];
    FT_TRY_HIP(hipMemcpyAsync(h, res, sizeof h, hipMemcpyDeviceToHost, s));
    FT_TRY_HIP(hipMemcpyAsync(total, offs + E, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    FT_TRY_HIP(hipStreamSynchronize(s));
    *W = h[0];
    *pred_var = h[1];
    return FT_OK;
}

}  // namespace ft
