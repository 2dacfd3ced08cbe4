// Shared pieces of the mass-matrix solvers: block reductions without atomics
// (block partials added in block order by the consumer) and the CSR view.
#pragma once

#include "common.h"

namespace ft {

constexpr int RB = 256;            // threads per block in the solver kernels
constexpr int MAX_RBLOCKS = 512;   // grid size cap (grid-stride loops beyond it)

// partial-sum slots (each nb doubles) and device scalar slots
// (P_SB, P_SBC) and (P_MX, P_MXC) hold compensated sums: sum, then compensation
enum { P_BB = 0, P_SB, P_SBC, P_RZ, P_RR, P_PQ, P_TRR, P_MX, P_MXC, P_COUNT };
enum { S_RHO0 = 0, S_RHO1, S_TOL2, S_DONE, S_ITERS, S_BB, S_SUMB, S_TRR, S_INTX, S_COUNT };

// NT: threads of the block (a multiple of 64)
template <int NT = RB>
__device__ __forceinline__ double block_total(double v) {
    __shared__ double sm[NT / 64];
    __shared__ double tot;
    v = wave_sum_xor(v, 64);
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = sm[0];
        for (int k = 1; k < NT / 64; ++k) s += sm[k];
        tot = s;
    }
    __syncthreads();
    const double t = tot;
    __syncthreads();
    return t;
}

// Sum of the nb partials of one slot, in block order (same value in every block).
template <int NT = RB>
__device__ __forceinline__ double partial_total(const double* __restrict__ part, int slot, int nb) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += NT) s += part[slot * nb + b];
    return block_total<NT>(s);
}

template <int NT = RB>
__device__ __forceinline__ void write_partial(double* __restrict__ part, int slot, double v) {
    const double t = block_total<NT>(v);
    if (threadIdx.x == 0) part[slot * gridDim.x + blockIdx.x] = t;
}

// ---- compensated sums (the conservation report's sum b and m^T x)
// s + c carries a sum with the rounding error of every addition kept in c:
// Knuth's TwoSum gives the exact error of s + x, which is added to c
// (Neumaier's scheme; pairs combine the same way).
__device__ __forceinline__ void comp_add(double& s, double& c, double x) {
    const double t = s + x;
    const double bp = t - s;
    c += (s - (t - bp)) + (x - bp);
    s = t;
}

// block total of the pairs (s, c): fixed butterfly per wave, then the waves in order
__device__ __forceinline__ void block_total_comp(double& s, double& c) {
    __shared__ double sm[2][RB / 64];
    __shared__ double tot[2];
    for (int o = 32; o > 0; o >>= 1) {
        const double os = __shfl_xor(s, o, 64), oc = __shfl_xor(c, o, 64);
        comp_add(s, c, os);
        c += oc;
    }
    if ((threadIdx.x & 63) == 0) {
        sm[0][threadIdx.x >> 6] = s;
        sm[1][threadIdx.x >> 6] = c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double ts = sm[0][0], tc = sm[1][0];
        for (int k = 1; k < RB / 64; ++k) {
            comp_add(ts, tc, sm[0][k]);
            tc += sm[1][k];
        }
        tot[0] = ts;
        tot[1] = tc;
    }
    __syncthreads();
    s = tot[0];
    c = tot[1];
    __syncthreads();
}

// block partial of a compensated sum: slots `slot` (sum) and `slot + 1` (compensation)
__device__ __forceinline__ void write_partial_comp(double* __restrict__ part, int slot, double s, double c) {
    block_total_comp(s, c);
    if (threadIdx.x == 0) {
        part[slot * gridDim.x + blockIdx.x] = s;
        part[(slot + 1) * gridDim.x + blockIdx.x] = c;
    }
}

// total of the nb compensated partials of `slot`, rounded once at the end
__device__ __forceinline__ double partial_total_comp(const double* __restrict__ part, int slot, int nb) {
    double s = 0.0, c = 0.0;
    for (int b = threadIdx.x; b < nb; b += RB) {
        comp_add(s, c, part[slot * nb + b]);
        c += part[(slot + 1) * nb + b];
    }
    block_total_comp(s, c);
    return s + c;
}

__device__ __forceinline__ double csr_row(const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                                          const double* __restrict__ val, const double* __restrict__ x, int64_t i) {
    return row_dot4(col, val, rowptr[i], rowptr[i + 1], [&](int32_t j) { return x[j]; });
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
// the same for blocks of NT threads
#define FOR_ROW_NT(i, NT) \
    for (int64_t i = int64_t(blockIdx.x) * (NT) + threadIdx.x; i < A.n; i += int64_t(gridDim.x) * (NT))

}  // namespace ft
