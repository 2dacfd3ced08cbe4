// Shared pieces of the mass-matrix solvers: block reductions without atomics
// (block partials added in block order by the consumer) and the CSR view.
#pragma once

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

}  // namespace ft
