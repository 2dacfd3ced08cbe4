// Setup/online split of a transfer from the built-in P1 source (the paper's
// amortization: localization belongs to the one-time initialization, and each
// later transfer between the same meshes only evaluates, accumulates and
// solves; sec. 5.3, initialization versus online cost).
//
// Setup (ft_plan_create): draw the samples of cfg and localize every target
// node and every sample in the source once, keeping the containing source
// element of each query (int32, [Q] in query-list order).
// Online (ft_plan_transfer): for new nodal values of the source field on the
// same source mesh, regenerate each sample from its Philox counter, take its
// cached element, recompute the barycentrics there (origin form) and
// interpolate the new values; then the residual element sums and the node
// assembly exactly as the fused route.  With the source's own values the
// result is bitwise that of ft_transfer_p1 (same points, same element, same
// arithmetic, same summation order).
#include "locate.h"
#include "sampling.h"

struct ft_plan;

namespace ft {

SrcView source_view(const ft_source* S);
ft_status source_eval(ft_source* S, int64_t head, int64_t npts, const void* pts, int64_t ld, int prec, void* out,
                      int64_t ld_out, int32_t* ids, hipStream_t s, unsigned long long* ood);
ft_status assemble_residual(ft_target* T, int F, const void* values, int64_t ld, bool f32, hipStream_t s);
void zero_counter(unsigned long long* p, hipStream_t s);
void zero_counters(unsigned long long* p, int n, hipStream_t s);
ft_status ensure_field_buffers(ft_target* T, int F, hipStream_t stream);

// setup: localize the samples of G-lane element groups, P per lane per round
template <int D, int G, int P>
__global__ __launch_bounds__(256) void k_plan_locate(SrcView S, const double* __restrict__ X, int64_t n,
                                                     const int32_t* __restrict__ conn, uint32_t E, uint32_t N,
                                                     SampleKey key, int32_t* __restrict__ ids,
                                                     unsigned long long* __restrict__ n_ood) {
    __shared__ double lds[4 * kWaveSlots<D>];
    double* c_af = lds + (threadIdx.x >> 6) * kWaveSlots<D>;
    const uint32_t gid = blockIdx.x * 256u + threadIdx.x;
    uint32_t t = gid / G;
    if (G == 64) t = __builtin_amdgcn_readfirstlane(t);   // one element per wave: scalar element data
    const int lane = int(gid & (G - 1));
    const bool valid = t < E;
    const uint32_t tt = valid ? t : 0u;
    double xv[D + 1][D];
#pragma unroll
    for (int k = 0; k <= D; ++k) {
        const int v = conn[int64_t(tt) * (D + 1) + k];
#pragma unroll
        for (int c = 0; c < D; ++c) xv[k][c] = X[c * n + v];
    }
    unsigned nood = 0;
    for (uint32_t j0 = 0; j0 < N; j0 += G * P) {
        double pt[P][D];
        bool act[P];
#pragma unroll
        for (int q = 0; q < P; ++q) {
            const uint32_t j = j0 + q * G + lane;
            act[q] = valid && j < N;
            double lam[D + 1];
            if (act[q]) {
                sample_lambda<D>(tt, j, key, lam);
            } else {
#pragma unroll
                for (int k = 0; k <= D; ++k) lam[k] = 0.0;
            }
#pragma unroll
            for (int c = 0; c < D; ++c) {
                double x = lam[0] * xv[0][c];
#pragma unroll
                for (int k = 1; k <= D; ++k) x = fma(lam[k], xv[k][c], x);
                pt[q][c] = x;
            }
        }
        double best[P];
        int bid[P];
        locate_wave<D, P>(S, pt, act, best, bid, c_af);
#pragma unroll
        for (int q = 0; q < P; ++q) {
            if (!act[q]) continue;
            nood += (bid[q] == INT_MAX || best[q] < kOutTol);
            ids[int64_t(tt) * N + j0 + q * G + lane] = bid[q] == INT_MAX ? -1 : bid[q];
        }
    }
    if (nood) atomicAdd(n_ood, (unsigned long long)nood);
}

// online, step 1: the control at the target nodes from their cached elements
template <int D>
__global__ void k_plan_nodes(const double* __restrict__ rec, const int32_t* __restrict__ sconn,
                             const double* __restrict__ vals, int64_t ns, int F, const double* __restrict__ X,
                             int64_t n, const int32_t* __restrict__ ids, double* __restrict__ g) {
    const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int id = ids[v];
    double p[D], mu[D + 1];
#pragma unroll
    for (int c = 0; c < D; ++c) p[c] = X[c * n + v];
    if (id >= 0) (void)barycentric<D>(rec + int64_t(id) * RecSize<D>::value, p, mu);
    for (int f = 0; f < F; ++f) {
        double y = 0.0;
        if (id >= 0)
#pragma unroll
            for (int k = 0; k <= D; ++k) y = fma(mu[k], vals[int64_t(f) * ns + sconn[int64_t(id) * (D + 1) + k]], y);
        g[int64_t(f) * n + v] = y;
    }
}

// online, steps 3-5: residual element sums with cached elements; G lanes per
// element, lane-stride sample order and butterfly as the fused route.  R > 1
// (G == 64 only): each wave sums R consecutive elements in turn.
template <int D, int G, int FC, int R>
__global__ __launch_bounds__(256) void k_plan_elements(const double* __restrict__ rec, const int32_t* __restrict__ sconn,
                                                       const double* __restrict__ vals, int64_t ns, int F,
                                                       const double* __restrict__ X, int64_t n,
                                                       const int32_t* __restrict__ conn, const double* __restrict__ vol,
                                                       uint32_t E, uint32_t N, double alpha, SampleKey key,
                                                       const int32_t* __restrict__ ids, const double* __restrict__ g,
                                                       double* __restrict__ beta, double* __restrict__ var_el,
                                                       unsigned long long* __restrict__ nonfinite) {
    static_assert(R == 1 || G == 64, "several elements per wave need one element per wave");
    const uint32_t gid = blockIdx.x * 256u + threadIdx.x;
    const int lane = int(gid & (G - 1));
    unsigned nf = 0;
    for (int e = 0; e < R; ++e) {
        uint32_t t = R > 1 ? (blockIdx.x * 4u + (threadIdx.x >> 6)) * uint32_t(R) + uint32_t(e) : gid / G;
        if (G == 64) t = __builtin_amdgcn_readfirstlane(t);   // one element per wave: scalar element data
        if (t >= E) break;   // the whole group leaves together
        int v[D + 1];
        double xv[D + 1][D];
#pragma unroll
        for (int k = 0; k <= D; ++k) {
            v[k] = conn[int64_t(t) * (D + 1) + k];
#pragma unroll
            for (int c = 0; c < D; ++c) xv[k][c] = X[c * n + v[k]];
        }
        for (int f0 = 0; f0 < F; f0 += FC) {
            // vs: sum and sum of squares of r - (1 - alpha) gbar (the element variance)
            double gk[FC][D + 1], acc[FC][D + 1], vs[FC], sh[FC];
#pragma unroll
            for (int f = 0; f < FC; ++f) {
                vs[f] = 0.0;
                double gs = 0.0;
#pragma unroll
                for (int k = 0; k <= D; ++k) {
                    acc[f][k] = 0.0;
                    gk[f][k] = g[int64_t(f0 + f < F ? f0 + f : 0) * n + v[k]];
                    gs += gk[f][k];
                }
                sh[f] = (alpha - 1.0) * (gs * (1.0 / double(D + 1)));
            }
            for (uint32_t j = lane; j < N; j += G) {
                double lam[D + 1], pt[D], mu[D + 1];
                sample_lambda<D>(t, j, key, lam);
#pragma unroll
                for (int c = 0; c < D; ++c) {
                    double x = lam[0] * xv[0][c];
#pragma unroll
                    for (int k = 1; k <= D; ++k) x = fma(lam[k], xv[k][c], x);
                    pt[c] = x;
                }
                const int id = ids[int64_t(t) * N + j];
                if (id >= 0) (void)barycentric<D>(rec + int64_t(id) * RecSize<D>::value, pt, mu);
#pragma unroll
                for (int f = 0; f < FC; ++f) {
                    if (f0 + f >= F) break;
                    double y = 0.0;
                    if (id >= 0)
#pragma unroll
                        for (int k = 0; k <= D; ++k)
                            y = fma(mu[k], vals[int64_t(f0 + f) * ns + sconn[int64_t(id) * (D + 1) + k]], y);
                    nf += !isfinite(y);
                    double gx = lam[0] * gk[f][0];
#pragma unroll
                    for (int k = 1; k <= D; ++k) gx = fma(lam[k], gk[f][k], gx);
                    const double r = y - alpha * gx;
#pragma unroll
                    for (int k = 0; k <= D; ++k) acc[f][k] = fma(r, lam[k], acc[f][k]);
                    const double sv = r + sh[f];
                    vs[f] = fma(sv, sv, vs[f]);
                }
            }
            // element totals in the fused route's order
            constexpr int K = FC * (D + 2);
            double red[K];
#pragma unroll
            for (int f = 0; f < FC; ++f) {
#pragma unroll
                for (int k = 0; k <= D; ++k) red[f * (D + 1) + k] = acc[f][k];
                red[FC * (D + 1) + f] = vs[f];
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
                for (int k = 0; k <= D; ++k) acc[f][k] = red[f * (D + 1) + k];
                vs[f] = red[FC * (D + 1) + f];
            }
            if (lane == 0) {
                const double scale = vol[t] / double(N);
                const double Nd = double(N);
                const double inv_n = 1.0 / Nd, inv_var = N > 1 ? inv_n / (Nd - 1.0) : 0.0;
#pragma unroll
                for (int f = 0; f < FC; ++f) {
                    if (f0 + f >= F) break;
#pragma unroll
                    for (int k = 0; k <= D; ++k) beta[(int64_t(f0 + f) * E + t) * (D + 1) + k] = acc[f][k] * scale;
                    double sa = 0.0;   // the plain sum of the residuals (the weights add up to 1)
#pragma unroll
                    for (int k = 0; k <= D; ++k) sa += acc[f][k];
                    var_el[int64_t(f0 + f) * E + t] =
                        element_variance(vol[t], fma(Nd, sh[f], sa), vs[f], inv_n, inv_var);
                }
            }
        }
    }
    if (nf) atomicAdd(nonfinite, (unsigned long long)nf);
}

}  // namespace ft

// ---------------------------------------------------------------- host side
struct ft_plan {
    ft_target* T = nullptr;
    ft_source* S = nullptr;
    ft_sample_cfg cfg{};
    int32_t* ids = nullptr;   // [n + E*N]
    unsigned long long* ood = nullptr;   // out-of-domain queries found at setup (device)
    int64_t n_ood = 0;                   // the same count on the host
};

namespace ft {

template <int D, int G, int P>
static void launch_locate(ft_plan* pl, hipStream_t s) {
    const ft_target* T = pl->T;
    const SampleKey key = make_sample_key(pl->cfg, D);
    k_plan_locate<D, G, P><<<grid_for(T->E * G, 256), 256, 0, s>>>(
        source_view(pl->S), T->coords, T->n, T->conn, uint32_t(T->E), uint32_t(pl->cfg.samples_per_elem), key,
        pl->ids + T->n, pl->ood);
}

template <int D>
static void locate_g(ft_plan* pl, hipStream_t s) {
    const int N = pl->cfg.samples_per_elem;
    if (N >= 256) launch_locate<D, 64, 4>(pl, s);
    else if (N >= 128) launch_locate<D, 64, 2>(pl, s);
    else if (N >= 64) launch_locate<D, 64, 1>(pl, s);
    else if (N > 16) launch_locate<D, 32, 1>(pl, s);
    else launch_locate<D, 16, 1>(pl, s);
}

ft_status plan_setup(ft_plan* pl, hipStream_t s) {
    ft_target* T = pl->T;
    const int64_t Q = T->n + T->E * int64_t(pl->cfg.samples_per_elem);
    FT_TRY(dev_alloc_n(&pl->ids, size_t(Q)));
    FT_TRY(dev_alloc_n(&pl->ood, 1));
    zero_counters(pl->ood, 1, s);
    FT_TRY(source_eval(pl->S, 0, T->n, T->coords, T->n, FT_F64, nullptr, T->n, pl->ids, s, pl->ood));
    if (T->dim == 2) locate_g<2>(pl, s);
    else locate_g<3>(pl, s);
    FT_TRY_HIP(hipGetLastError());
    unsigned long long h = 0;
    FT_TRY_HIP(hipMemcpyAsync(&h, pl->ood, sizeof(h), hipMemcpyDeviceToHost, s));
    FT_TRY_HIP(hipStreamSynchronize(s));
    pl->n_ood = int64_t(h);
    return FT_OK;
}

template <int D, int G>
static void launch_elements(ft_plan* pl, const double* vals, hipStream_t s) {
    ft_target* T = pl->T;
    const ft_source* S = pl->S;
    const SampleKey key = make_sample_key(pl->cfg, D);
    const int F = pl->cfg.n_fields;
    constexpr int R = G == 64 && D == 2 ? 4 : 1;   // elements per wave (measured no gain for tetrahedra)
    const unsigned grid = grid_for(T->E * G, 256 * R);
    const uint32_t N = uint32_t(pl->cfg.samples_per_elem);
    if (F == 1)
        k_plan_elements<D, G, 1, R><<<grid, 256, 0, s>>>(S->rec, S->conn, vals, S->n, F, T->coords, T->n, T->conn,
                                                      T->vol, uint32_t(T->E), N, pl->cfg.alpha, key, pl->ids + T->n,
                                                      T->g, T->beta, T->var_el, T->counters);
    else
        k_plan_elements<D, G, 4, R><<<grid, 256, 0, s>>>(S->rec, S->conn, vals, S->n, F, T->coords, T->n, T->conn,
                                                      T->vol, uint32_t(T->E), N, pl->cfg.alpha, key, pl->ids + T->n,
                                                      T->g, T->beta, T->var_el, T->counters);
}

template <int D>
static void elements_g(ft_plan* pl, const double* vals, hipStream_t s) {
    const int N = pl->cfg.samples_per_elem;
    if (N >= 64) launch_elements<D, 64>(pl, vals, s);
    else if (N > 16) launch_elements<D, 32>(pl, vals, s);
    else if (N > 8) launch_elements<D, 16>(pl, vals, s);
    else if (N > 4) launch_elements<D, 8>(pl, vals, s);
    else if (N > 2) launch_elements<D, 4>(pl, vals, s);
    else if (N > 1) launch_elements<D, 2>(pl, vals, s);
    else launch_elements<D, 1>(pl, vals, s);
}

ft_status plan_transfer(ft_plan* pl, const double* vals, hipStream_t s) {
    ft_target* T = pl->T;
    const ft_source* S = pl->S;
    const double* v = vals ? vals : S->values;
    const int F = pl->cfg.n_fields;
    zero_counter(T->counters, s);
    T->ood_mode = 2;   // the localization (and its out-of-domain count) was fixed at setup
    T->var_mode = VAR_NONE;
    T->ood_host = pl->n_ood;
    if (T->dim == 2) {
        k_plan_nodes<2><<<grid_for(T->n, 256), 256, 0, s>>>(S->rec, S->conn, v, S->n, F, T->coords, T->n, pl->ids,
                                                           T->g);
        elements_g<2>(pl, v, s);
    } else {
        k_plan_nodes<3><<<grid_for(T->n, 256), 256, 0, s>>>(S->rec, S->conn, v, S->n, F, T->coords, T->n, pl->ids,
                                                           T->g);
        elements_g<3>(pl, v, s);
    }
    FT_TRY_HIP(hipGetLastError());
    T->var_mode = pl->cfg.samples_per_elem >= 2 ? VAR_ESTIMATED : VAR_NONE;
    return assemble_residual(T, F, nullptr, 0, false, s);
}

ft_plan* plan_new(ft_target* T, ft_source* S, const ft_sample_cfg* cfg) {
    auto* p = new ft_plan();
    p->T = T;
    p->S = S;
    p->cfg = *cfg;
    return p;
}

ft_target* plan_target(ft_plan* p) { return p->T; }
const ft_sample_cfg* plan_cfg(const ft_plan* p) { return &p->cfg; }

void plan_delete(ft_plan* p) {
    if (!p) return;
    dev_free(p->ids);
    dev_free(p->ood);
    delete p;
}

}  // namespace ft
