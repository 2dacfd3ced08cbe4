// Sample emission and consumption: the Monte Carlo part of the CV-MC load vector.
//
// Emission (sec. 4.1 step 1 and step 3) writes the point-query list: the n
// target nodes, then sample j of element t at position n + t*N + j.
//
// Consumption (sec. 4.1 steps 4-6) forms, for every element t and local
// vertex k, the residual element load of Eq. cv_element_load_residual_operator
// with the uniform density of Eq. mc_element_integral_operator_uniform:
//   beta_tk = |Omega_t| / N * sum_j (y_tj - alpha g(X_tj)) psi_k(X_tj),
// where psi_k(X_tj) = lambda_k of the sample (P1 basis = barycentric
// coordinates) and g(X_tj) = sum_l lambda_l g_{v_l} (the control, P1 on the
// target).  lambda is regenerated from the same Philox counters instead of
// being stored.  Then b_res,v = sum of beta_tk over the incidence list of v.
//
// Thread mapping of the consume kernel: a group of G lanes (G = smallest
// power of two >= N, at most 64) per element; lanes stride over the samples
// (coalesced reads of y), keep per-lane partial sums, and the group reduces
// them with a fixed butterfly.  No floating-point atomics anywhere, so results
// are bitwise reproducible run to run.
#include <type_traits>

#include "adaptive.h"
#include "sampling.h"

namespace ft {

// Sample j of element t (vertices v) written to query q of the list.
template <int D, bool F32>
__device__ __forceinline__ void emit_sample(const double* __restrict__ X, int64_t n, const int (&v)[D + 1],
                                            uint32_t t, uint32_t j, const SampleKey& key, void* __restrict__ out_,
                                            int64_t ld, int64_t q) {
    if constexpr (!F32) {
        double lam[D + 1];
        sample_lambda<D>(t, j, key, lam);
        double* out = static_cast<double*>(out_);
#pragma unroll
        for (int c = 0; c < D; ++c) {
            double x = lam[0] * X[c * n + v[0]];
#pragma unroll
            for (int k = 1; k <= D; ++k) x = fma(lam[k], X[c * n + v[k]], x);
            out[c * ld + q] = x;
        }
    } else {
        float lam[D + 1];
        sample_lambda_f32<D>(t, j, key, lam);
        float* out = static_cast<float*>(out_);
#pragma unroll
        for (int c = 0; c < D; ++c) {
            float x = lam[0] * float(X[c * n + v[0]]);
#pragma unroll
            for (int k = 1; k <= D; ++k) x = fmaf(lam[k], float(X[c * n + v[k]]), x);
            out[c * ld + q] = x;
        }
    }
}

// R == 0: one sample per lane, any N.  R > 0 (N a multiple of 64): every run
// of 64 consecutive samples belongs to one element, whose connectivity and
// vertex coordinates are then scalar loads, and each wave writes R runs.
template <int D, bool F32, int R>
__global__ __launch_bounds__(256) void k_emit(const double* __restrict__ X, int64_t n, const int32_t* __restrict__ conn,
                                              uint32_t total, uint32_t N, FastDiv divN, SampleKey key,
                                              void* __restrict__ out_, int64_t ld) {
    if constexpr (R == 0) {
        const uint32_t idx = blockIdx.x * 256u + threadIdx.x;
        if (idx >= total) return;
        const uint32_t t = fast_div(idx, divN);
        int v[D + 1];
#pragma unroll
        for (int k = 0; k <= D; ++k) v[k] = conn[int64_t(t) * (D + 1) + k];
        emit_sample<D, F32>(X, n, v, t, idx - t * N, key, out_, ld, n + int64_t(idx));
    } else {
        const uint32_t lane = threadIdx.x & 63u;
        const uint64_t wave = uint64_t(blockIdx.x) * 4u + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint64_t c0 = (wave * R + r) * 64u;   // first sample of the run (wave-uniform)
            if (c0 >= total) break;
            const uint32_t t = fast_div(uint32_t(c0), divN);
            int v[D + 1];
#pragma unroll
            for (int k = 0; k <= D; ++k) v[k] = conn[int64_t(t) * (D + 1) + k];
            emit_sample<D, F32>(X, n, v, t, uint32_t(c0) - t * N + lane, key, out_, ld, n + int64_t(c0) + lane);
        }
    }
}

// 64-sample runs per wave when N is a multiple of 64 (a tetrahedron sample
// draws two Philox blocks, so half as many runs)
template <int D>
constexpr int kEmitRuns = D == 2 ? 8 : 4;

// Samples per element from allocation offsets: element t's samples go to
// queries n + offs[t] + j, j < offs[t+1] - offs[t]; a wave takes kVarRuns
// consecutive elements, its lanes striding over each one's samples.  An
// element whose range is invalid (see element_range) writes nothing.
constexpr int kVarRuns = 4;

template <int D, bool F32>
__global__ __launch_bounds__(256) void k_emit_varn(const double* __restrict__ X, int64_t n,
                                                   const int32_t* __restrict__ conn, uint32_t E,
                                                   const int64_t* __restrict__ offs, int64_t total, SampleKey key,
                                                   void* __restrict__ out_, int64_t ld) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = blockIdx.x * 4u + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (int r = 0; r < kVarRuns; ++r) {
        const uint32_t t = wave * uint32_t(kVarRuns) + uint32_t(r);
        if (t >= E) break;
        int64_t o0;
        uint32_t N;
        if (!element_range(offs, t, total, o0, N)) continue;
        int v[D + 1];
#pragma unroll
        for (int k = 0; k <= D; ++k) v[k] = conn[int64_t(t) * (D + 1) + k];
        for (uint32_t j = lane; j < N; j += 64u) emit_sample<D, F32>(X, n, v, t, j, key, out_, ld, n + o0 + j);
    }
}

template <bool F32>
__global__ void k_emit_nodes(const double* __restrict__ X, int64_t n, int dim, void* __restrict__ out_, int64_t ld) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int c = 0; c < dim; ++c) {
        if (F32)
            static_cast<float*>(out_)[c * ld + i] = float(X[c * n + i]);
        else
            static_cast<double*>(out_)[c * ld + i] = X[c * n + i];
    }
}

// Element t's sums over its N samples (lanes stride over them, G lanes per
// element); returns the number of non-finite values seen by this lane.
// OWN: the element's own control coefficient (variance-minimizing, from its
// samples): with A_k = sum y l_k, B_k = sum g l_k, P = sum y g w, Q = sum g^2 w,
// w = sum_k l_k^2, alpha_t = (P/N - sum A_k B_k / N^2) / (Q/N - sum B_k^2 / N^2)
// clipped to [0, 2] (1 unless the denominator is positive), and the load
// carries the exact control part: beta_k = alpha_t (M_t g)_k + |Omega|/N (A_k - alpha_t B_k).
// var_el[f][t] (when non-null): the variance of the element's Monte Carlo
// total |Omega|/N sum_j r_j (sum_k l_k = 1), |Omega|^2 s^2 / N with s^2 the
// unbiased sample variance of the residuals r_j = y_j - alpha g(X_j); 0 for
// N < 2.  The moments are taken of residuals shifted by a constant of the
// element, which leaves s^2 unchanged and keeps the one-pass form free of
// cancellation: s = r - (1 - alpha) gbar for a fixed alpha (gbar: the mean of
// the element's vertex controls, so s = y - g at alpha = 1, y - gbar at 0);
// with the element's own alpha (not known until its sums are complete) the
// moments of d = y - g and u = g - gbar, and r - (1 - alpha) gbar = d + (1 - alpha) u.
// Only the squares and products need sums of their own: the plain sums follow
// from the element sums, since the weights of a sample add up to 1.
constexpr double kOwnAlphaLo = 0.0, kOwnAlphaHi = 2.0;


// P: degree of the target elements; dofs: the element's nodes, [E][nb].
// N: the element's samples, at queries qbase .. qbase + N - 1 of field 0.
// VN (samples per element from an allocation): the element variance of an
// element with one sample is undefined (NaN) rather than 0, so that a sum
// over elements says it cannot be estimated.
template <int D, int P, int G, int FC, bool F32, bool OWN, bool VN>
__device__ __forceinline__ unsigned int consume_element(uint32_t t, int lane, const void* __restrict__ values_,
                                                        const ValueLayout& L, int F, const int32_t* __restrict__ dofs,
                                                        const double* __restrict__ vol, int64_t n, uint32_t E,
                                                        uint32_t N, int64_t qbase, double alpha,
                                                        const SampleKey& key, double* __restrict__ beta,
                                                        double* __restrict__ var_el) {
    static_assert(P == 1 || !OWN, "each element's own coefficient: P1 targets");
    constexpr int NB = Basis<D, P>::n;
    int v[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k) v[k] = dofs[int64_t(t) * NB + k];
    const double scale = vol[t] / double(N);
    unsigned int nf = 0;
    constexpr int FO = OWN ? FC : 1;
    const double Nd = double(N);
    const double inv_n = 1.0 / Nd;
    const double inv_var = N > 1 ? inv_n / (Nd - 1.0) : (VN ? __builtin_nan("") : 0.0);
    for (int f0 = 0; f0 < F; f0 += FC) {
        double gk[FC][NB];
        double acc[FC][NB];       // sum r psi_k (fixed alpha) or sum y l_k (OWN)
        double accb[FO][NB];      // OWN: sum g l_k
        double pq[FO][2];         // OWN: sum y g w, sum g^2 w
        double vs[FC];            // sum s^2 (fixed alpha) or sum d^2 (OWN)
        double vm[FO][2];         // OWN: sum d u, sum u^2
        double gbar[FC], sh[FC];
#pragma unroll
        for (int f = 0; f < FC; ++f) {
            gbar[f] = 0.0;
            vs[f] = 0.0;
#pragma unroll
            for (int k = 0; k < NB; ++k) {
                acc[f][k] = 0.0;
                const int64_t off = int64_t(f0 + f < F ? f0 + f : 0) * L.node_ld + v[k];
                gk[f][k] = F32 ? double(static_cast<const float*>(values_)[off])
                               : static_cast<const double*>(values_)[off];
                gbar[f] += gk[f][k];
            }
            gbar[f] *= 1.0 / double(NB);
            sh[f] = (alpha - 1.0) * gbar[f];
        }
#pragma unroll
        for (int f = 0; f < FO; ++f) {
            pq[f][0] = pq[f][1] = 0.0;
            vm[f][0] = vm[f][1] = 0.0;
#pragma unroll
            for (int k = 0; k < NB; ++k) accb[f][k] = 0.0;
        }
        for (uint32_t j = lane; j < N; j += G) {
            double lam[D + 1];
            if constexpr (F32) {
                float lf[D + 1];
                sample_lambda_f32<D>(t, j, key, lf);
#pragma unroll
                for (int k = 0; k <= D; ++k) lam[k] = lf[k];
            } else {
                sample_lambda<D>(t, j, key, lam);
            }
            double psi[NB];
            basis_at<D, P>(lam, psi);
            double w = 0.0;
            if constexpr (OWN) {
#pragma unroll
                for (int k = 0; k < NB; ++k) w = fma(psi[k], psi[k], w);
            }
#pragma unroll
            for (int f = 0; f < FC; ++f) {
                if (f0 + f >= F) break;
                const int64_t off = int64_t(f0 + f) * L.samp_fld + qbase + j;
                const double y = F32 ? double(static_cast<const float*>(values_)[off])
                                     : static_cast<const double*>(values_)[off];
                nf += !isfinite(y);
                double gx = psi[0] * gk[f][0];
#pragma unroll
                for (int k = 1; k < NB; ++k) gx = fma(psi[k], gk[f][k], gx);
                if constexpr (OWN) {
#pragma unroll
                    for (int k = 0; k < NB; ++k) {
                        acc[f][k] = fma(y, psi[k], acc[f][k]);
                        accb[f][k] = fma(gx, psi[k], accb[f][k]);
                    }
                    pq[f][0] = fma(y * gx, w, pq[f][0]);
                    pq[f][1] = fma(gx * gx, w, pq[f][1]);
                    const double d = y - gx, u = gx - gbar[f];
                    vs[f] = fma(d, d, vs[f]);
                    vm[f][0] = fma(d, u, vm[f][0]);
                    vm[f][1] = fma(u, u, vm[f][1]);
                } else {
                    const double r = y - alpha * gx;
#pragma unroll
                    for (int k = 0; k < NB; ++k) acc[f][k] = fma(r, psi[k], acc[f][k]);
                    const double sv = r + sh[f];
                    vs[f] = fma(sv, sv, vs[f]);
                }
            }
        }
        // element totals: with one element per wave on the lane-swap / DPP
        // path, else butterflies over the element's G lanes
        constexpr int KA = FC * NB + FC;   // acc, vs
        constexpr int KO = NB + 4;         // OWN, per field: accb, pq, vm
        constexpr int K = OWN ? KA + FO * KO : KA;
        double red[K];
#pragma unroll
        for (int f = 0; f < FC; ++f) {
#pragma unroll
            for (int k = 0; k < NB; ++k) red[f * NB + k] = acc[f][k];
            red[FC * NB + f] = vs[f];
        }
        if constexpr (OWN) {
#pragma unroll
            for (int f = 0; f < FO; ++f) {
#pragma unroll
                for (int k = 0; k < NB; ++k) red[KA + f * KO + k] = accb[f][k];
                red[KA + f * KO + NB] = pq[f][0];
                red[KA + f * KO + NB + 1] = pq[f][1];
                red[KA + f * KO + NB + 2] = vm[f][0];
                red[KA + f * KO + NB + 3] = vm[f][1];
            }
        }
        if constexpr (G == 64) {
            wave_totals<K>(red);
        } else {
#pragma unroll
            for (int i = 0; i < K; ++i) red[i] = wave_sum_xor(red[i], G);
        }
#pragma unroll
        for (int f = 0; f < FC; ++f) {
#pragma unroll
            for (int k = 0; k < NB; ++k) acc[f][k] = red[f * NB + k];
            vs[f] = red[FC * NB + f];
        }
        if constexpr (OWN) {
#pragma unroll
            for (int f = 0; f < FO; ++f) {
#pragma unroll
                for (int k = 0; k < NB; ++k) accb[f][k] = red[KA + f * KO + k];
                pq[f][0] = red[KA + f * KO + NB];
                pq[f][1] = red[KA + f * KO + NB + 1];
                vm[f][0] = red[KA + f * KO + NB + 2];
                vm[f][1] = red[KA + f * KO + NB + 3];
            }
        }
        if (lane == 0) {
#pragma unroll
            for (int f = 0; f < FC; ++f) {
                if (f0 + f >= F) break;
                double* bt = beta + (int64_t(f0 + f) * E + t) * NB;
                double sa = 0.0;   // sum_k of the element sums: the plain sum over the samples
#pragma unroll
                for (int k = 0; k < NB; ++k) sa += acc[f][k];
                if constexpr (OWN) {
                    double ab = 0.0, bb = 0.0, gs = 0.0, sb = 0.0;
#pragma unroll
                    for (int k = 0; k <= D; ++k) {
                        ab = fma(acc[f][k], accb[f][k], ab);
                        bb = fma(accb[f][k], accb[f][k], bb);
                        gs += gk[f][k];
                        sb += accb[f][k];
                    }
                    const double num = pq[f][0] / Nd - ab / (Nd * Nd);
                    const double den = pq[f][1] / Nd - bb / (Nd * Nd);
                    double a = (isfinite(num) && isfinite(den) && den > 0.0) ? num / den : 1.0;
                    a = fmin(fmax(a, kOwnAlphaLo), kOwnAlphaHi);
#pragma unroll
                    for (int k = 0; k <= D; ++k) {
                        const double ctrl = vol[t] * (gs + gk[f][k]) / double((D + 1) * (D + 2));
                        bt[k] = a * ctrl + scale * (acc[f][k] - a * accb[f][k]);
                    }
                    if (var_el) {
                        // r - (1 - a) gbar = d + c u, c = 1 - a; sum d = sum y - sum g, sum u = sum g - N gbar
                        const double c = 1.0 - a;
                        const double s1 = (sa - sb) + c * fma(-Nd, gbar[f], sb);
                        const double s2 = fma(c * c, vm[f][1], fma(2.0 * c, vm[f][0], vs[f]));
                        var_el[int64_t(f0 + f) * E + t] = element_variance(vol[t], s1, s2, inv_n, inv_var);
                    }
                } else {
#pragma unroll
                    for (int k = 0; k < NB; ++k) bt[k] = acc[f][k] * scale;
                    // sum s = sum r + N (alpha - 1) gbar
                    if (var_el)
                        var_el[int64_t(f0 + f) * E + t] =
                            element_variance(vol[t], fma(Nd, sh[f], sa), vs[f], inv_n, inv_var);
                }
            }
        }
    }
    return nf;
}

// An element whose samples per element (VN) are out of range or whose queries
// leave [0, total): no loads are taken, its element loads are 0, its variance
// undefined, and it counts as one non-finite value.
template <int NB>
__device__ __forceinline__ unsigned int reject_element(uint32_t t, int lane, int F, uint32_t E,
                                                       double* __restrict__ beta, double* __restrict__ var_el) {
    if (lane != 0) return 0;
    for (int f = 0; f < F; ++f) {
#pragma unroll
        for (int k = 0; k < NB; ++k) beta[(int64_t(f) * E + t) * NB + k] = 0.0;
        if (var_el) var_el[int64_t(f) * E + t] = __builtin_nan("");
    }
    return 1;
}

// G lanes per element.  R > 1 (G == 64 only): each wave sums R consecutive
// elements in turn, with their element data in scalar registers.  VN (G == 64):
// element t has the samples offs[t] .. offs[t+1] - 1 of the list's sample block
// (total samples in all), N is not read.
template <int D, int P, int G, int FC, bool F32, int R, bool OWN, bool VN>
__global__ __launch_bounds__(256) void k_consume(const void* __restrict__ values_, ValueLayout L, int F,
                                                 const int32_t* __restrict__ dofs, const double* __restrict__ vol,
                                                 int64_t n, uint32_t E, uint32_t N, const int64_t* __restrict__ offs,
                                                 int64_t total, double alpha, SampleKey key,
                                                 double* __restrict__ beta, double* __restrict__ var_el,
                                                 unsigned long long* __restrict__ nonfinite) {
    static_assert(!VN || G == 64, "samples per element from offsets: one element per wave");
    constexpr int NB = Basis<D, P>::n;
    unsigned int nf = 0;
    if constexpr (R > 1) {
        static_assert(G == 64, "one element per wave");
        const uint32_t wave = blockIdx.x * 4u + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
        const int lane = int(threadIdx.x & 63u);
        for (int e = 0; e < R; ++e) {
            const uint32_t t = wave * uint32_t(R) + uint32_t(e);
            if (t >= E) break;
            uint32_t Nt = N;
            int64_t qbase = L.samp0 + int64_t(t) * L.samp_elem;
            if constexpr (VN) {
                int64_t o0;
                if (!element_range(offs, t, total, o0, Nt)) {
                    nf += reject_element<NB>(t, lane, F, E, beta, var_el);
                    continue;
                }
                qbase = L.samp0 + o0;
            }
            nf += consume_element<D, P, G, FC, F32, OWN, VN>(t, lane, values_, L, F, dofs, vol, n, E, Nt, qbase,
                                                             alpha, key, beta, var_el);
        }
    } else {
        const uint32_t gid = blockIdx.x * 256u + threadIdx.x;
        uint32_t t = gid / G;
        const int lane = int(gid & (G - 1));
        if (t >= E) return;   // the whole group leaves together
        if (G == 64) t = __builtin_amdgcn_readfirstlane(t);   // one element per wave: scalar element data
        uint32_t Nt = N;
        int64_t qbase = L.samp0 + int64_t(t) * L.samp_elem;
        bool ok = true;
        if constexpr (VN) {
            int64_t o0;
            ok = element_range(offs, t, total, o0, Nt);
            qbase = L.samp0 + o0;
        }
        nf = ok ? consume_element<D, P, G, FC, F32, OWN, VN>(t, lane, values_, L, F, dofs, vol, n, E, Nt, qbase,
                                                             alpha, key, beta, var_el)
                : reject_element<NB>(t, lane, F, E, beta, var_el);
    }
    if (nf) atomicAdd(nonfinite, (unsigned long long)nf);
}

// b_res,v = sum over the incidence list of v (ascending (t, k)) of beta; also
// keeps g_v = values[f][v] (the control at the nodes) for the solve, unless
// values is null (the fused route writes g itself).
template <int D, bool F32>
__global__ void k_assemble(const double* __restrict__ beta, int64_t E, int nb, const int64_t* __restrict__ inc_ptr,
                           const int32_t* __restrict__ inc, int64_t n, int F, const void* __restrict__ values_,
                           int64_t ld, double* __restrict__ bres, double* __restrict__ g,
                           unsigned long long* __restrict__ nonfinite) {
    const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int64_t b = inc_ptr[v], e = inc_ptr[v + 1];
    unsigned int nf = 0;
    for (int f = 0; f < F; ++f) {
        const double* bf = beta + int64_t(f) * E * nb;
        double s = 0.0;
        for (int64_t i = b; i < e; ++i) s += bf[inc[i]];
        bres[int64_t(f) * n + v] = s;
        if (values_) {
            const int64_t off = int64_t(f) * ld + v;
            const double gv = F32 ? double(static_cast<const float*>(values_)[off])
                                  : static_cast<const double*>(values_)[off];
            nf += !isfinite(gv);
            g[int64_t(f) * n + v] = gv;
        }
    }
    if (nf) atomicAdd(nonfinite, (unsigned long long)nf);
}

// The same with one wavefront per node, its lanes striding over the node's
// incidence list (then a fixed butterfly): for meshes whose nodes touch
// thousands of elements (d-simplices, d >= 4: 720 per vertex of a 5D Kuhn
// mesh, 5040 in 6D), where one lane per node would leave the GPU nearly idle.
template <bool F32>
__global__ __launch_bounds__(256) void k_assemble_wide(const double* __restrict__ beta, int64_t E, int nb,
                                                       const int64_t* __restrict__ inc_ptr,
                                                       const int32_t* __restrict__ inc, int64_t n, int F,
                                                       const void* __restrict__ values_, int64_t ld,
                                                       double* __restrict__ bres, double* __restrict__ g,
                                                       unsigned long long* __restrict__ nonfinite) {
    const int64_t v = int64_t(blockIdx.x) * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (v >= n) return;   // the whole wave
    const int lane = int(threadIdx.x & 63u);
    const int64_t b = inc_ptr[v], e = inc_ptr[v + 1];
    unsigned int nf = 0;
    for (int f = 0; f < F; ++f) {
        const double* bf = beta + int64_t(f) * E * nb;
        double s = 0.0;
        for (int64_t i = b + lane; i < e; i += 64) s += bf[inc[i]];
        s = wave_sum_xor(s, 64);
        if (lane == 0) {
            bres[int64_t(f) * n + v] = s;
            if (values_) {
                const int64_t off = int64_t(f) * ld + v;
                const double gv = F32 ? double(static_cast<const float*>(values_)[off])
                                      : static_cast<const double*>(values_)[off];
                nf += !isfinite(gv);
                g[int64_t(f) * n + v] = gv;
            }
        }
    }
    if (nf) atomicAdd(nonfinite, (unsigned long long)nf);
}

// Fields-inner node assembly (many fields, F <= 64): one wavefront per node,
// lane = field; each incidence entry adds one contiguous row beta[t][k][0..F)
// in ascending (element, vertex) order; bres[v][f] and g[v][f] come out as
// coalesced rows.
template <bool F32>
__global__ __launch_bounds__(256) void k_assemble_fi(const double* __restrict__ beta, const int64_t* __restrict__ inc_ptr,
                                                     const int32_t* __restrict__ inc, int64_t n, int F,
                                                     const void* __restrict__ values_, int64_t ld,
                                                     double* __restrict__ bres, double* __restrict__ g,
                                                     unsigned long long* __restrict__ nonfinite) {
    const int64_t v = __builtin_amdgcn_readfirstlane(int(blockIdx.x * 4u + (threadIdx.x >> 6)));
    const int f = int(threadIdx.x & 63);
    if (v >= n) return;   // wave-uniform
    const int64_t b = inc_ptr[v], e = inc_ptr[v + 1];
    double s = 0.0;
    if (f < F)
        for (int64_t i = b; i < e; ++i) s += beta[int64_t(inc[i]) * F + f];
    unsigned nf = 0;
    if (f < F) {
        bres[v * F + f] = s;
        const int64_t off = int64_t(f) * ld + v;
        const double gv = F32 ? double(static_cast<const float*>(values_)[off]) : static_cast<const double*>(values_)[off];
        nf = !isfinite(gv);
        g[v * F + f] = gv;
    }
    if (nf) atomicAdd(nonfinite, (unsigned long long)nf);
}

__global__ void k_zero_u64(unsigned long long* __restrict__ p, int n) {
    if (int(threadIdx.x) < n) p[threadIdx.x] = 0ull;
}

// ---------------------------------------------------------------- host side
static SampleKey make_key(const ft_target* T, const ft_sample_cfg* cfg) { return make_sample_key(*cfg, T->dim); }

template <int D>
static ft_status emit_impl(ft_target* T, const ft_sample_cfg* cfg, void* points, hipStream_t s) {
    const uint32_t N = uint32_t(cfg->samples_per_elem);
    const uint64_t total = uint64_t(T->E) * N;
    const int64_t ld = T->n + int64_t(total);
    const bool f32 = cfg->precision != FT_F64;
    if (f32)
        k_emit_nodes<true><<<grid_for(T->n, 256), 256, 0, s>>>(T->coords, T->n, D, points, ld);
    else
        k_emit_nodes<false><<<grid_for(T->n, 256), 256, 0, s>>>(T->coords, T->n, D, points, ld);
    if (total) {
        const FastDiv dv = make_fastdiv(N);
        const SampleKey key = make_key(T, cfg);
        const unsigned grid = grid_for(int64_t(total), 256);
        if (N % 64 == 0) {
            auto kern = f32 ? k_emit<D, true, kEmitRuns<D>> : k_emit<D, false, kEmitRuns<D>>;
            kern<<<grid_for(int64_t(total), 256 * kEmitRuns<D>), 256, 0, s>>>(T->coords, T->n, T->conn, uint32_t(total),
                                                                            N, dv, key, points, ld);
        } else {
            auto kern = f32 ? k_emit<D, true, 0> : k_emit<D, false, 0>;
            kern<<<grid, 256, 0, s>>>(T->coords, T->n, T->conn, uint32_t(total), N, dv, key, points, ld);
        }
    }
    FT_TRY_HIP(hipGetLastError());
    return FT_OK;
}

// Calls f with the target's dimension as a compile-time constant (2..6).
template <typename Fn>
static ft_status by_dim(int dim, Fn&& f) {
    switch (dim) {
        case 2: return f(std::integral_constant<int, 2>{});
        case 3: return f(std::integral_constant<int, 3>{});
        case 4: return f(std::integral_constant<int, 4>{});
        case 5: return f(std::integral_constant<int, 5>{});
        case 6: return f(std::integral_constant<int, 6>{});
        default: set_error("dim must lie in [2, 6] (got %d)", dim); return FT_E_ARG;
    }
}

ft_status emit_points(ft_target* T, const ft_sample_cfg* cfg, void* points, hipStream_t s) {
    return by_dim(T->dim, [&](auto d) { return emit_impl<decltype(d)::value>(T, cfg, points, s); });
}

// The query list of per-element counts: the nodes, then element t's samples
// at n + offs[t] + j (leading dimension n + total).
template <int D>
static ft_status emit_varn_impl(ft_target* T, const ft_sample_cfg* cfg, const int64_t* offs, int64_t total,
                                void* points, hipStream_t s) {
    const int64_t ld = T->n + total;
    const SampleKey key = make_key(T, cfg);   // plain samples
    if (cfg->precision != FT_F64) {
        k_emit_nodes<true><<<grid_for(T->n, 256), 256, 0, s>>>(T->coords, T->n, D, points, ld);
        k_emit_varn<D, true><<<grid_for(T->E, 4 * kVarRuns), 256, 0, s>>>(T->coords, T->n, T->conn, uint32_t(T->E),
                                                                          offs, total, key, points, ld);
    } else {
        k_emit_nodes<false><<<grid_for(T->n, 256), 256, 0, s>>>(T->coords, T->n, D, points, ld);
        k_emit_varn<D, false><<<grid_for(T->E, 4 * kVarRuns), 256, 0, s>>>(T->coords, T->n, T->conn, uint32_t(T->E),
                                                                           offs, total, key, points, ld);
    }
    FT_TRY_HIP(hipGetLastError());
    return FT_OK;
}

ft_status emit_points_varn(ft_target* T, const ft_sample_cfg* cfg, const int64_t* offs, int64_t total, void* points,
                           hipStream_t s) {
    return by_dim(T->dim, [&](auto d) { return emit_varn_impl<decltype(d)::value>(T, cfg, offs, total, points, s); });
}

constexpr int kConsumeRuns = 4;   // elements per wave when G == 64

// Per-element counts (offs non-null): ranges offs[t] .. offs[t+1] of total samples.
struct VarCounts {
    const int64_t* offs = nullptr;
    int64_t total = 0;
};

template <int D, int P, int G, int FC, bool F32, bool VN = false>
static void launch_consume(ft_target* T, const ft_sample_cfg* cfg, const void* values, const ValueLayout& L,
                           double* beta, hipStream_t s, const VarCounts& vc = VarCounts{}) {
    const SampleKey key = make_key(T, cfg);
    constexpr int R = G == 64 ? kConsumeRuns : 1;
    const unsigned grid = grid_for(T->E * G, 256 * R);
    auto kern = k_consume<D, P, G, FC, F32, R, false, VN>;
    if constexpr (P == 1)
        if (cfg->alpha_mode == FT_ALPHA_ELEMENT) kern = k_consume<D, P, G, FC, F32, R, true, VN>;
    kern<<<grid, 256, 0, s>>>(values, L, cfg->n_fields, T->dofs, T->vol, T->n, uint32_t(T->E),
                              uint32_t(cfg->samples_per_elem), vc.offs, vc.total, cfg->alpha, key, beta, T->var_el,
                              T->counters);
}

template <int D, int P, int G, bool F32, bool VN = false>
static void consume_fc(ft_target* T, const ft_sample_cfg* cfg, const void* values, const ValueLayout& L,
                       double* beta, hipStream_t s, const VarCounts& vc = VarCounts{}) {
    if (cfg->n_fields == 1)
        launch_consume<D, P, G, 1, F32, VN>(T, cfg, values, L, beta, s, vc);
    else
        launch_consume<D, P, G, 4, F32, VN>(T, cfg, values, L, beta, s, vc);
}

// Lanes per element G from N (P2 targets: one element per wave for N >= 64,
// else 16 lanes per element).
template <int D, bool F32>
static void consume_g(ft_target* T, const ft_sample_cfg* cfg, const void* values, const ValueLayout& L,
                      double* beta, hipStream_t s) {
    const int N = cfg->samples_per_elem;
    if constexpr (D >= 4) {   // d-simplices (P1): one element per wave
        consume_fc<D, 1, 64, F32>(T, cfg, values, L, beta, s);
    } else {
        if (T->order == 2) {
            if (N >= 64) consume_fc<D, 2, 64, F32>(T, cfg, values, L, beta, s);
            else consume_fc<D, 2, 16, F32>(T, cfg, values, L, beta, s);
            return;
        }
        if (N >= 64) consume_fc<D, 1, 64, F32>(T, cfg, values, L, beta, s);
        else if (N > 16) consume_fc<D, 1, 32, F32>(T, cfg, values, L, beta, s);
        else if (N > 8) consume_fc<D, 1, 16, F32>(T, cfg, values, L, beta, s);
        else if (N > 4) consume_fc<D, 1, 8, F32>(T, cfg, values, L, beta, s);
        else if (N > 2) consume_fc<D, 1, 4, F32>(T, cfg, values, L, beta, s);
        else if (N > 1) consume_fc<D, 1, 2, F32>(T, cfg, values, L, beta, s);
        else consume_fc<D, 1, 1, F32>(T, cfg, values, L, beta, s);
    }
}

// The layout of the caller's query values (ft_sample_cfg.values_layout).
ValueLayout query_layout(const ft_target* T, const ft_sample_cfg* cfg) {
    const int64_t N = cfg->samples_per_elem;
    return cfg->values_layout == FT_VALUES_ELEMENT_TILES ? element_tile_layout(T->n, N, cfg->n_fields)
                                                         : field_major_layout(T->n + T->E * N, T->n, N);
}

void zero_counter(unsigned long long* p, hipStream_t s) {
    k_zero_u64<<<1, 64, 0, s>>>(p, 1);   // a kernel, not a memset: safe inside captured graphs
}

void zero_counters(unsigned long long* p, int n, hipStream_t s) { k_zero_u64<<<1, 64, 0, s>>>(p, n); }

template <int D>
static void launch_assemble(ft_target* T, const double* beta, int F, const void* values, int64_t ld, bool f32,
                            hipStream_t s) {
    if constexpr (D >= 4) {
        auto kern = f32 ? k_assemble_wide<true> : k_assemble_wide<false>;
        kern<<<grid_for(T->n, 4), 256, 0, s>>>(beta, T->E, T->nb, T->inc_ptr, T->inc, T->n, F, values, ld, T->bres,
                                              T->g, T->counters);
        return;
    }
    if (f32)
        k_assemble<D, true><<<grid_for(T->n, 256), 256, 0, s>>>(beta, T->E, T->nb, T->inc_ptr, T->inc, T->n, F, values,
                                                               ld, T->bres, T->g, T->counters);
    else
        k_assemble<D, false><<<grid_for(T->n, 256), 256, 0, s>>>(beta, T->E, T->nb, T->inc_ptr, T->inc, T->n, F, values,
                                                                ld, T->bres, T->g, T->counters);
}

static ft_status assemble_from(ft_target* T, const double* beta, int F, const void* values, int64_t ld, bool f32,
                               hipStream_t s) {
    FT_TRY(by_dim(T->dim, [&](auto d) {
        launch_assemble<decltype(d)::value>(T, beta, F, values, ld, f32, s);
        return FT_OK;
    }));
    FT_TRY_HIP(hipGetLastError());
    return FT_OK;
}

ft_status assemble_residual(ft_target* T, int F, const void* values, int64_t ld, bool f32, hipStream_t s) {
    return assemble_from(T, T->beta, F, values, ld, f32, s);
}

static ft_status assemble_fields_inner(ft_target* T, const double* beta, int F, const void* values, int64_t ld,
                                       bool f32, hipStream_t s) {
    const unsigned grid = grid_for(T->n, 4);
    if (f32)
        k_assemble_fi<true><<<grid, 256, 0, s>>>(beta, T->inc_ptr, T->inc, T->n, F, values, ld, T->bres, T->g,
                                                 T->counters);
    else
        k_assemble_fi<false><<<grid, 256, 0, s>>>(beta, T->inc_ptr, T->inc, T->n, F, values, ld, T->bres, T->g,
                                                  T->counters);
    FT_TRY_HIP(hipGetLastError());
    return FT_OK;
}

ft_status consume_mfma(ft_target* T, const ft_sample_cfg* cfg, const void* values, const ValueLayout& L,
                       double* beta, hipStream_t s);
constexpr int kMfmaMaxSamples = 256;   // the matrix-core form stages <= 256 samples
constexpr int kMfmaMaxFields = 64;     // and <= 64 control values per vertex in LDS

template <int D>
static ft_status consume_impl(ft_target* T, const ft_sample_cfg* cfg, const void* values, double* beta,
                              hipStream_t s) {
    const ValueLayout L = query_layout(T, cfg);
    const bool f32 = cfg->precision != FT_F64;
    const bool split = cfg->precision == FT_SPLIT_F16 || cfg->precision == FT_SPLIT_BF16;
    zero_counter(T->counters, s);
    T->ood_mode = 0;   // the caller's black box evaluated the points
    T->var_mode = VAR_NONE;
    if (split && cfg->samples_per_elem <= kMfmaMaxSamples && cfg->n_fields <= kMfmaMaxFields) {
        FT_TRY(consume_mfma(T, cfg, values, L, beta, s));   // element loads fields-inner
        T->fields_inner = cfg->n_fields > 1;
        return assemble_fields_inner(T, beta, cfg->n_fields, values, L.node_ld, f32, s);
    }
    if (f32) consume_g<D, true>(T, cfg, values, L, beta, s);
    else consume_g<D, false>(T, cfg, values, L, beta, s);
    FT_TRY_HIP(hipGetLastError());
    T->var_mode = cfg->samples_per_elem >= 2 ? VAR_ESTIMATED : VAR_NONE;
    return assemble_from(T, beta, cfg->n_fields, values, L.node_ld, f32, s);
}

// The element loads go to `beta` ([F][E][d+1], or [E][d+1][F] on the
// many-field matrix-core route): the target's own buffer, or caller-provided
// scratch of at least F E (d+1) doubles.  Only the element kernel and the
// node assembly that follows it touch them.
ft_status consume_values(ft_target* T, const ft_sample_cfg* cfg, const void* values, double* beta, hipStream_t s) {
    return by_dim(T->dim, [&](auto d) { return consume_impl<decltype(d)::value>(T, cfg, values, beta, s); });
}

// Consumption of a list with per-element counts (field-major values, one
// element per wave): the element variances are estimated (an element with a
// single sample makes their sum undefined).
template <int D>
static ft_status consume_varn_impl(ft_target* T, const ft_sample_cfg* cfg, const int64_t* offs, int64_t total,
                                   const void* values, hipStream_t s) {
    const int64_t Q = T->n + total;
    const ValueLayout L{Q, T->n, Q, 0, make_fastdiv(1)};
    const bool f32 = cfg->precision != FT_F64;
    const VarCounts vc{offs, total};
    zero_counter(T->counters, s);
    T->ood_mode = 0;
    T->var_mode = VAR_NONE;
    if constexpr (D <= 3) {
        if (T->order == 2) {
            if (f32) consume_fc<D, 2, 64, true, true>(T, cfg, values, L, T->beta, s, vc);
            else consume_fc<D, 2, 64, false, true>(T, cfg, values, L, T->beta, s, vc);
        }
    }
    if (T->order != 2) {
        if (f32) consume_fc<D, 1, 64, true, true>(T, cfg, values, L, T->beta, s, vc);
        else consume_fc<D, 1, 64, false, true>(T, cfg, values, L, T->beta, s, vc);
    }
    FT_TRY_HIP(hipGetLastError());
    T->var_mode = VAR_ESTIMATED;
    return assemble_from(T, T->beta, cfg->n_fields, values, L.node_ld, f32, s);
}

ft_status consume_values_varn(ft_target* T, const ft_sample_cfg* cfg, const int64_t* offs, int64_t total,
                              const void* values, hipStream_t s) {
    return by_dim(T->dim, [&](auto d) { return consume_varn_impl<decltype(d)::value>(T, cfg, offs, total, values, s); });
}

}  // namespace ft
