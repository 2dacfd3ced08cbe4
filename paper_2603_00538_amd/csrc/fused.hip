// Fused transfer from the built-in P1 source: sec. 4.1 steps 1 and 3-6 in one
// pass over the samples, with no point-query list in memory.
//
// For each target element t and sample j the kernel draws lambda from the
// Philox stream (same counters as the emission kernel), forms the physical
// point, localizes it in the source with the wave-cooperative bin search,
// interpolates f^s there, and accumulates the residual element load
//   beta_tk = |Omega_t| / N * sum_j (f^s(X_tj) - alpha g(X_tj)) lambda_k
// exactly as the consume kernel does.  The localization rule's winner does
// not depend on which points share a wave, so the two routes give the same
// element, the same barycentrics and the same values; the element sums run
// in the consume kernel's lane order for N >= 64 with G*P samples per round.
// Only the control g (f^s at the target nodes) and beta are written.
#include "adaptive.h"
#include "fused.h"

namespace ft {

// One field: register targets for four waves per SIMD in 2D and in the
// binary64 3D form with one element per wave and at most two samples per lane
// (128 registers, no spill), three for its binary32 form (which would spill
// at four), two for the other 3D variants (which would spill at three).  The
// unconstrained allocation leaves two waves per SIMD (2D: 21% slower).  P2
// targets (ORD = 2, more basis functions per element): two waves.
template <int D, int G, int P, int FC, bool F32, int ORD>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(FC != 1 || ORD != 1 ? (ORD != 1 ? 2 : 1)
                                                       : (D == 2 ? 4 : (G == 64 && P <= 2 ? (F32 ? 3 : 4) : 2)))))
void k_fused_p1(SrcView S, const double* __restrict__ X, int64_t n, const int32_t* __restrict__ conn,
                const int32_t* __restrict__ dofs, const double* __restrict__ vol, uint32_t E, uint32_t N,
                double alpha, SampleKey key, const double* __restrict__ g, double* __restrict__ beta,
                double* __restrict__ var_el, unsigned long long* __restrict__ nonfinite,
                unsigned long long* __restrict__ n_ood) {
    constexpr int WS = kWaveSlots<D> + kLamSlots<D, P>;
    __shared__ double lds[4 * WS];
    const uint32_t gid = blockIdx.x * 256u + threadIdx.x;
    unsigned nf = 0, nood = 0;
    fused_elements<D, G, P, FC, F32, ORD>(S, X, n, conn, vol, E, N, alpha, key, g, beta, gid / G,
                                          int(gid & (G - 1)), nf, nood, lds + (threadIdx.x >> 6) * WS, var_el,
                                          dofs);
    if (nf) atomicAdd(nonfinite, (unsigned long long)nf);
    if (nood) atomicAdd(n_ood, (unsigned long long)nood);
}

// Per-element counts (offsets from an allocation): one element per wave,
// element t's samples j < N_t = offs[t+1] - offs[t], from the same counters as
// the emission of their list, so the route reproduces the black-box
// consumption of that list.  An element whose range is invalid (see
// element_range) takes no samples: zero loads, undefined variance, one
// non-finite count.
template <int D, int P, int FC, bool F32, int ORD>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(FC != 1 || ORD != 1 ? (ORD != 1 ? 2 : 1) : (D == 2 ? 4 : (P <= 2 ? (F32 ? 3 : 4) : 2)))))
void k_fused_varn(SrcView S, const double* __restrict__ X, int64_t n, const int32_t* __restrict__ conn,
                  const int32_t* __restrict__ dofs, const double* __restrict__ vol, uint32_t E,
                  const int64_t* __restrict__ offs, int64_t total, double alpha, SampleKey key,
                  const double* __restrict__ g, double* __restrict__ beta, double* __restrict__ var_el,
                  unsigned long long* __restrict__ nonfinite, unsigned long long* __restrict__ n_ood) {
    constexpr int WS = kWaveSlots<D> + kLamSlots<D, P>;
    constexpr int NB = Basis<D, ORD>::n;
    __shared__ double lds[4 * WS];
    const uint32_t t = blockIdx.x * 4u + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (t >= E) return;   // the whole wave
    const int lane = int(threadIdx.x & 63u);
    int64_t o0;
    uint32_t N;
    unsigned nf = 0, nood = 0;
    if (element_range(offs, t, total, o0, N)) {
        fused_elements<D, 64, P, FC, F32, ORD, true>(S, X, n, conn, vol, E, N, alpha, key, g, beta, t, lane, nf,
                                                     nood, lds + (threadIdx.x >> 6) * WS, var_el, dofs);
    } else if (lane == 0) {
        for (int f = 0; f < S.F; ++f) {
#pragma unroll
            for (int k = 0; k < NB; ++k) beta[(int64_t(f) * E + t) * NB + k] = 0.0;
            var_el[int64_t(f) * E + t] = __builtin_nan("");
        }
        nf = 1;
    }
    if (nf) atomicAdd(nonfinite, (unsigned long long)nf);
    if (nood) atomicAdd(n_ood, (unsigned long long)nood);
}

SrcView source_view(const ft_source* S);
ft_status source_eval(ft_source* S, int64_t head, int64_t npts, const void* pts, int64_t ld, int prec, void* out,
                      int64_t ld_out, int32_t* ids, hipStream_t s, unsigned long long* ood);
ft_status assemble_residual(ft_target* T, int F, const void* values, int64_t ld, bool f32, hipStream_t s);
void zero_counters(unsigned long long* p, int n, hipStream_t s);

template <int D, int G, int P, int FC, int ORD = 1>
static void launch_fused(ft_target* T, ft_source* S, const ft_sample_cfg* cfg, hipStream_t s) {
    const SampleKey key = make_sample_key(*cfg, D);
    const unsigned grid = grid_for(T->E * G, 256);
    auto kern = cfg->precision == FT_F32 ? k_fused_p1<D, G, P, FC, true, ORD> : k_fused_p1<D, G, P, FC, false, ORD>;
    kern<<<grid, 256, 0, s>>>(source_view(S), T->coords, T->n, T->conn, T->dofs, T->vol, uint32_t(T->E),
                              uint32_t(cfg->samples_per_elem), cfg->alpha, key, T->g, T->beta, T->var_el,
                              T->counters, T->counters + 1);
}

// The control of the binary32 form: the source at the target nodes rounded to
// binary32, the values rounded to binary32 (as its query list holds them).
template <int D>
__global__ __launch_bounds__(64) void k_nodes_rounded(SrcView S, const double* __restrict__ X, int64_t n,
                                                      double* __restrict__ g, unsigned long long* __restrict__ n_ood) {
    constexpr int P = D == 2 ? 4 : 2;
    __shared__ double lds[kWaveSlots<D>];
    const int64_t base = int64_t(blockIdx.x) * 64 * P;
    if (base >= n) return;
    const unsigned nood = eval_wave<D, P, false, false, true>(S, base, n, X, n, g, n, nullptr, lds);
    if (nood) atomicAdd(n_ood, (unsigned long long)nood);
}

template <int D, int G, int P>
static void fused_fc(ft_target* T, ft_source* S, const ft_sample_cfg* cfg, hipStream_t s) {
    if (cfg->n_fields == 1) launch_fused<D, G, P, 1>(T, S, cfg, s);
    else launch_fused<D, G, P, 4>(T, S, cfg, s);
}

// lanes per element G and samples per lane per round P (P2 targets: one
// element per wave for N >= 64, else 16 lanes per element; one sample per
// lane per round)
template <int D>
static void fused_g(ft_target* T, ft_source* S, const ft_sample_cfg* cfg, hipStream_t s) {
    const int N = cfg->samples_per_elem;
    if (T->order == 2) {
        const bool one = cfg->n_fields == 1;
        if (N >= 64) {
            if (one) launch_fused<D, 64, 1, 1, 2>(T, S, cfg, s);
            else launch_fused<D, 64, 1, 4, 2>(T, S, cfg, s);
        } else {
            if (one) launch_fused<D, 16, 1, 1, 2>(T, S, cfg, s);
            else launch_fused<D, 16, 1, 4, 2>(T, S, cfg, s);
        }
        return;
    }
    if (N >= 256) fused_fc<D, 64, 4>(T, S, cfg, s);
    else if (N >= 128) fused_fc<D, 64, 2>(T, S, cfg, s);
    else if (N >= 64) fused_fc<D, 64, 1>(T, S, cfg, s);
    else if (N > 16) fused_fc<D, 32, 1>(T, S, cfg, s);
    else if (N > 8) fused_fc<D, 16, 1>(T, S, cfg, s);
    else if (N > 4) fused_fc<D, 8, 1>(T, S, cfg, s);
    else if (N > 2) fused_fc<D, 4, 1>(T, S, cfg, s);
    else if (N > 1) fused_fc<D, 2, 1>(T, S, cfg, s);
    else fused_fc<D, 1, 1>(T, S, cfg, s);
}

// Step 1: the control, f^s at the target nodes, straight into T->g (with the
// counters of this transfer's non-finite values and out-of-domain queries cleared).
static ft_status fused_control(ft_target* T, ft_source* S, const ft_sample_cfg* cfg, hipStream_t s) {
    zero_counters(T->counters, 2, s);
    T->ood_mode = 1;
    T->var_mode = VAR_NONE;
    if (cfg->precision == FT_F32) {
        const unsigned gw = grid_for(T->n, 64 * (T->dim == 2 ? 4 : 2));
        if (T->dim == 2) k_nodes_rounded<2><<<gw, 64, 0, s>>>(source_view(S), T->coords, T->n, T->g, T->counters + 1);
        else k_nodes_rounded<3><<<gw, 64, 0, s>>>(source_view(S), T->coords, T->n, T->g, T->counters + 1);
    } else {
        FT_TRY(source_eval(S, 0, T->n, T->coords, T->n, FT_F64, T->g, T->n, nullptr, s, T->counters + 1));
    }
    return FT_OK;
}

ft_status transfer_p1(ft_target* T, ft_source* S, const ft_sample_cfg* cfg, hipStream_t s) {
    FT_TRY(fused_control(T, S, cfg, s));
    if (T->dim == 2) fused_g<2>(T, S, cfg, s);
    else fused_g<3>(T, S, cfg, s);
    FT_TRY_HIP(hipGetLastError());
    T->var_mode = cfg->samples_per_elem >= 2 ? VAR_ESTIMATED : VAR_NONE;
    return assemble_residual(T, cfg->n_fields, nullptr, 0, false, s);
}

template <int D, int P, int FC, int ORD>
static void launch_fused_varn(ft_target* T, ft_source* S, const ft_sample_cfg* cfg, const int64_t* offs,
                              int64_t total, hipStream_t s) {
    const SampleKey key = make_sample_key(*cfg, D);   // plain samples (samples_per_elem is 0)
    const unsigned grid = grid_for(T->E, 4);
    auto kern = cfg->precision == FT_F32 ? k_fused_varn<D, P, FC, true, ORD> : k_fused_varn<D, P, FC, false, ORD>;
    kern<<<grid, 256, 0, s>>>(source_view(S), T->coords, T->n, T->conn, T->dofs, T->vol, uint32_t(T->E), offs, total,
                              cfg->alpha, key, T->g, T->beta, T->var_el, T->counters, T->counters + 1);
}

// Samples per lane per round from the mean count (P2 targets: one).
template <int D>
static void fused_varn_d(ft_target* T, ft_source* S, const ft_sample_cfg* cfg, const int64_t* offs, int64_t total,
                         hipStream_t s) {
    const bool one = cfg->n_fields == 1;
    if (T->order == 2) {
        if (one) launch_fused_varn<D, 1, 1, 2>(T, S, cfg, offs, total, s);
        else launch_fused_varn<D, 1, 4, 2>(T, S, cfg, offs, total, s);
        return;
    }
    const int64_t mean = total / T->E;
    if (mean >= 256) {
        if (one) launch_fused_varn<D, 4, 1, 1>(T, S, cfg, offs, total, s);
        else launch_fused_varn<D, 4, 4, 1>(T, S, cfg, offs, total, s);
    } else if (mean >= 128) {
        if (one) launch_fused_varn<D, 2, 1, 1>(T, S, cfg, offs, total, s);
        else launch_fused_varn<D, 2, 4, 1>(T, S, cfg, offs, total, s);
    } else {
        if (one) launch_fused_varn<D, 1, 1, 1>(T, S, cfg, offs, total, s);
        else launch_fused_varn<D, 1, 4, 1>(T, S, cfg, offs, total, s);
    }
}

ft_status transfer_p1_varn(ft_target* T, ft_source* S, const ft_sample_cfg* cfg, const int64_t* offs, int64_t total,
                           hipStream_t s) {
    FT_TRY(fused_control(T, S, cfg, s));
    if (T->dim == 2) fused_varn_d<2>(T, S, cfg, offs, total, s);
    else fused_varn_d<3>(T, S, cfg, offs, total, s);
    FT_TRY_HIP(hipGetLastError());
    T->var_mode = VAR_ESTIMATED;
    return assemble_residual(T, cfg->n_fields, nullptr, 0, false, s);
}

}  // namespace ft
