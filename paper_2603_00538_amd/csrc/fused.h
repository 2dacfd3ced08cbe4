// Fused per-element work of the built-in-source route (sec. 4.1 steps 3-5):
// sample, localize, interpolate and accumulate the residual element loads of
// target element t, with G lanes per element and P samples per lane per
// round.  Shared by the single-transfer kernel and the batched kernel.
#pragma once

#include "locate.h"
#include "sampling.h"

namespace ft {

// Whether a round's barycentric weights wait in LDS while the wave localizes
// (P(D+1) doubles per lane) instead of being drawn again from their Philox
// counters afterwards.  Measured: 10% faster for the 2D fused kernel, 18%
// slower in 3D (registers and LDS per wave grow), so 3D draws them again.
template <int D, int P>
constexpr bool kStashLambda = D == 2;
template <int D, int P>
constexpr int kLamSlots = kStashLambda<D, P> ? 64 * P * (D + 1) : 0;

// lane: index within the element's lane group [0, G); t >= E marks an idle
// group (it still takes part in the wave-cooperative localization).  Adds the
// lane's non-finite and out-of-domain counts to nf / nood.  c_af: the wave's
// LDS candidate slots (kWaveSlots<D> doubles), followed by its weight stash
// (kLamSlots<D, P> doubles).
// F32: the binary32 form of the black-box route with the query list kept in
// registers: weights from the binary32 sampling, the point formed in binary32
// from binary32 vertex coordinates, the value rounded to binary32 (the
// control values g must hold binary32-rounded values too); sums in binary64.
// var_el (unless null): each element's variance term, as the consumption
// kernel writes it (sum and sum of squares of r - (1 - alpha) gbar).
// ORD: degree of the target elements; for P2 dofs lists each element's
// nodes ([E][nb]: vertices, then edge nodes), where g and the loads live.
// VN: N is this element's own count (per-element counts, G == 64); the
// variance of a single-sample element is undefined (NaN) rather than 0.
template <int D, int G, int P, int FC, bool F32 = false, int ORD = 1, bool VN = false>
__device__ __forceinline__ void fused_elements(const SrcView& S, const double* __restrict__ X, int64_t n,
                                               const int32_t* __restrict__ conn, const double* __restrict__ vol,
                                               uint32_t E, uint32_t N, double alpha, SampleKey key,
                                               const double* __restrict__ g, double* __restrict__ beta, uint32_t t,
                                               int lane, unsigned& nf, unsigned& nood, double* __restrict__ c_af,
                                               double* __restrict__ var_el = nullptr,
                                               const int32_t* __restrict__ dofs = nullptr) {
    constexpr int NB = Basis<D, ORD>::n;
    // with one element per wave, its connectivity, vertices and control values
    // are wave-uniform: scalar loads into scalar registers
    if (G == 64) t = __builtin_amdgcn_readfirstlane(t);
    const bool valid = t < E;
    const uint32_t tt = valid ? t : 0u;
    int v[D + 1];
#pragma unroll
    for (int k = 0; k <= D; ++k) v[k] = conn[int64_t(tt) * (D + 1) + k];
    double xv[D + 1][D];
#pragma unroll
    for (int k = 0; k <= D; ++k)
#pragma unroll
        for (int c = 0; c < D; ++c) xv[k][c] = X[c * n + v[k]];
    int gv[NB];   // the element's nodes
#pragma unroll
    for (int k = 0; k < NB; ++k) gv[k] = ORD == 1 ? v[k < D + 1 ? k : 0] : dofs[int64_t(tt) * NB + k];
    double gk[FC][NB], acc[FC][NB], vs[FC], sh[FC];
#pragma unroll
    for (int f = 0; f < FC; ++f) {
        vs[f] = 0.0;
        double gs = 0.0;   // summed in node order, as the consumption kernel does
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            acc[f][k] = 0.0;
            gk[f][k] = f < S.F ? g[int64_t(f) * n + gv[k]] : 0.0;
            gs += gk[f][k];
        }
        sh[f] = (alpha - 1.0) * (gs * (1.0 / double(NB)));   // (alpha - 1) gbar
    }
    // every lane runs the same number of rounds: the localization is wave-cooperative.
    // Round r, slot q of a lane holds sample j = r*G*P + q*G + lane.
    for (uint32_t j0 = 0; j0 < N; j0 += G * P) {
        double pt[P][D];
        bool act[P];
#pragma unroll
        for (int q = 0; q < P; ++q) {
            const uint32_t j = j0 + q * G + lane;
            act[q] = valid && j < N;
            double lam[D + 1];
            float lf[D + 1];
            if (act[q]) {
                if (F32) {
                    sample_lambda_f32<D>(tt, j, key, lf);
#pragma unroll
                    for (int k = 0; k <= D; ++k) lam[k] = lf[k];
                } else {
                    sample_lambda<D>(tt, j, key, lam);
                }
            } else {
#pragma unroll
                for (int k = 0; k <= D; ++k) {
                    lam[k] = 0.0;
                    lf[k] = 0.0f;
                }
            }
            if (kStashLambda<D, P>) {
                double* st = c_af + kWaveSlots<D> + (q * (D + 1)) * 64 + (threadIdx.x & 63);
#pragma unroll
                for (int k = 0; k <= D; ++k) st[k * 64] = lam[k];
            }
#pragma unroll
            for (int c = 0; c < D; ++c) {
                if (F32) {
                    float x = lf[0] * float(xv[0][c]);
#pragma unroll
                    for (int k = 1; k <= D; ++k) x = fmaf(lf[k], float(xv[k][c]), x);
                    pt[q][c] = x;
                } else {
                    double x = lam[0] * xv[0][c];
#pragma unroll
                    for (int k = 1; k <= D; ++k) x = fma(lam[k], xv[k][c], x);
                    pt[q][c] = x;
                }
            }
        }
        double best[P];
        int bid[P];
        locate_wave<D, P>(S, pt, act, best, bid, c_af);
#pragma unroll
        for (int q = 0; q < P; ++q) {
            if (!act[q]) continue;
            nood += (bid[q] == INT_MAX || best[q] < kOutTol);
            double mu[D + 1];
            winner_mu<D>(S, bid[q], pt[q], mu);
            // the weights from the LDS stash, or again from their counter: keeping
            // P of them live in registers through the localization would cost
            // occupancy
            double lam[D + 1];
            if (kStashLambda<D, P>) {
                const double* st = c_af + kWaveSlots<D> + (q * (D + 1)) * 64 + (threadIdx.x & 63);
#pragma unroll
                for (int k = 0; k <= D; ++k) lam[k] = st[k * 64];
            } else if (F32) {
                float lf[D + 1];
                sample_lambda_f32<D>(tt, j0 + q * G + lane, key, lf);
#pragma unroll
                for (int k = 0; k <= D; ++k) lam[k] = lf[k];
            } else {
                sample_lambda<D>(tt, j0 + q * G + lane, key, lam);
            }
            double psi[NB];
            basis_at<D, ORD>(lam, psi);
#pragma unroll
            for (int f = 0; f < FC; ++f) {
                if (f >= S.F) break;
                double y = p1_value<D>(S, bid[q], mu, f);
                if (F32) y = double(float(y));
                nf += !isfinite(y);
                double gx = psi[0] * gk[f][0];
#pragma unroll
                for (int k = 1; k < NB; ++k) gx = fma(psi[k], gk[f][k], gx);
                const double r = y - alpha * gx;
#pragma unroll
                for (int k = 0; k < NB; ++k) acc[f][k] = fma(r, psi[k], acc[f][k]);
                if (var_el) {
                    const double sv = r + sh[f];
                    vs[f] = fma(sv, sv, vs[f]);
                }
            }
        }
    }
    // element totals as the consumption kernel forms them (lane-swap / DPP
    // path with one element per wave, else butterflies over G lanes)
    constexpr int K = FC * (NB + 1);
    double red[K];
#pragma unroll
    for (int f = 0; f < FC; ++f) {
#pragma unroll
        for (int k = 0; k < NB; ++k) red[f * NB + k] = acc[f][k];
        red[FC * NB + f] = vs[f];
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
    if (valid && lane == 0) {
        const double scale = vol[t] / double(N);
        const double Nd = double(N);
        const double inv_n = 1.0 / Nd;
        const double inv_var = N > 1 ? inv_n / (Nd - 1.0) : (VN ? __builtin_nan("") : 0.0);
#pragma unroll
        for (int f = 0; f < FC; ++f) {
            if (f >= S.F) break;
#pragma unroll
            for (int k = 0; k < NB; ++k) beta[(int64_t(f) * E + t) * NB + k] = acc[f][k] * scale;
            if (var_el) {
                double sa = 0.0;   // the plain sum of the residuals (the weights add up to 1)
#pragma unroll
                for (int k = 0; k < NB; ++k) sa += acc[f][k];
                var_el[int64_t(f) * E + t] = element_variance(vol[t], fma(Nd, sh[f], sa), vs[f], inv_n, inv_var);
            }
        }
    }
}

}  // namespace ft
