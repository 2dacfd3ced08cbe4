// Exact intersection-based load vector on P1 triangles (sec. 3: the
// mesh-intersection route, the reference the stochastic estimate converges
// to and the paper's comparator).
//
// b_k = integral f^s psi_k over the target mesh splits over the non-empty
// intersections t cap s of target and source elements.  On each of them f^s
// (P1 on s) and psi_k (P1 on t) are linear, so f^s psi_k is quadratic and the
// degree-2 Gauss rule on a triangulation of the convex polygon t cap s is
// exact.  Per target element t (one lane each):
//   candidates  the source elements registered in the bins around t's box
//               (widened by the largest half-extent of a source box), kept
//               when their outward-rounded boxes meet t's box; every source
//               element that meets t is among them, none twice;
//   clip        t against the three edge half-planes of s, counter-clockwise
//               (Sutherland-Hodgman; at most six vertices);
//   integrate   the polygon fanned from its first vertex, each sub-triangle
//               with the three-point rule at barycentric (2/3, 1/6, 1/6) and
//               its permutations, weights 1/3; psi_k from t's inverse
//               Jacobian, f^s from s's barycentric record.
// The element loads go where the Monte Carlo element sums go (beta), and the
// node assembly and the solve follow unchanged with no control (alpha = 0).
// The paper finds the intersecting source elements by an adjacency walk from
// a seed element; here the source's uniform bin grid gives each lane its
// candidates directly, without a per-element queue.
#include "locate.h"

namespace ft {

SrcView source_view(const ft_source* S);
ft_status assemble_residual(ft_target* T, int F, const void* values, int64_t ld, bool f32, hipStream_t s);
void zero_counters(unsigned long long* p, int n, hipStream_t s);

constexpr int kPolyMax = 8;   // a triangle clipped by three half-planes has at most six vertices

// Keep the part of polygon (px, py)[0, n) left of the directed line a -> b.
__device__ __forceinline__ int clip_halfplane(const double (&px)[kPolyMax], const double (&py)[kPolyMax], int n,
                                              double ax, double ay, double bx, double by, double (&qx)[kPolyMax],
                                              double (&qy)[kPolyMax]) {
    int m = 0;
    const double ex = bx - ax, ey = by - ay;
    for (int i = 0; i < n; ++i) {
        const int j = i + 1 < n ? i + 1 : 0;
        const double sp = ex * (py[i] - ay) - ey * (px[i] - ax);
        const double sq = ex * (py[j] - ay) - ey * (px[j] - ax);
        if (sp >= 0.0 && m < kPolyMax) {
            qx[m] = px[i];
            qy[m] = py[i];
            ++m;
        }
        if ((sp >= 0.0) != (sq >= 0.0) && m < kPolyMax) {
            const double u = sp / (sp - sq);
            qx[m] = fma(u, px[j] - px[i], px[i]);
            qy[m] = fma(u, py[j] - py[i], py[i]);
            ++m;
        }
    }
    return m;
}

template <int FC>
__global__ __launch_bounds__(256) void k_supermesh2d(SrcView S, const double* __restrict__ sX,
                                                     const double* __restrict__ X, int64_t n,
                                                     const int32_t* __restrict__ conn, const double* __restrict__ vol,
                                                     int64_t E, double* __restrict__ beta,
                                                     double* __restrict__ area_out,
                                                     unsigned long long* __restrict__ n_partial) {
    constexpr int RS = RecSize<2>::value;
    constexpr int BS = BoxSize<2>::value;
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= E) return;
    double tx[3], ty[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int v = conn[t * 3 + k];
        tx[k] = X[v];
        ty[k] = X[n + v];
    }
    // target barycentrics psi_1, psi_2 = A (p - x0), psi_0 = 1 - psi_1 - psi_2
    const double j00 = tx[1] - tx[0], j01 = tx[2] - tx[0], j10 = ty[1] - ty[0], j11 = ty[2] - ty[0];
    const double det = j00 * j11 - j01 * j10;
    const double a00 = j11 / det, a01 = -j01 / det, a10 = -j10 / det, a11 = j00 / det;
    double lo[2] = {fmin(tx[0], fmin(tx[1], tx[2])), fmin(ty[0], fmin(ty[1], ty[2]))};
    double hi[2] = {fmax(tx[0], fmax(tx[1], tx[2])), fmax(ty[0], fmax(ty[1], ty[2]))};
    int b0[2], b1[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        b0[c] = bin_of(lo[c] - S.g.hx[c], c, S.g);
        b1[c] = bin_of(hi[c] + S.g.hx[c], c, S.g);
    }
    double acc[FC][3];
#pragma unroll
    for (int f = 0; f < FC; ++f)
#pragma unroll
        for (int k = 0; k < 3; ++k) acc[f][k] = 0.0;
    double area = 0.0;
    for (int by = b0[1]; by <= b1[1]; ++by)
        for (int bx = b0[0]; bx <= b1[0]; ++bx) {
            const int64_t b = int64_t(by) * S.g.nb[0] + bx;
            const int64_t c1 = S.bin_ptr[b + 1];
            for (int64_t c = S.bin_ptr[b]; c < c1; ++c) {
                const int e = S.bin_elems[c];
                const float* bx_ = S.box + int64_t(e) * BS;
                if (double(bx_[0]) > hi[0] || double(bx_[2]) < lo[0] || double(bx_[1]) > hi[1] ||
                    double(bx_[3]) < lo[1])
                    continue;
                int sv[3];
                double sx[3], sy[3];
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    sv[k] = S.conn[int64_t(e) * 3 + k];
                    sx[k] = sX[sv[k]];
                    sy[k] = sX[S.n + sv[k]];
                }
                // edges of s counter-clockwise
                const bool ccw = (sx[1] - sx[0]) * (sy[2] - sy[0]) - (sx[2] - sx[0]) * (sy[1] - sy[0]) > 0.0;
                // t, counter-clockwise (its sub-triangles then have positive area)
                double px[kPolyMax], py[kPolyMax], qx[kPolyMax], qy[kPolyMax];
                px[0] = tx[0];
                py[0] = ty[0];
                px[1] = det > 0.0 ? tx[1] : tx[2];
                py[1] = det > 0.0 ? ty[1] : ty[2];
                px[2] = det > 0.0 ? tx[2] : tx[1];
                py[2] = det > 0.0 ? ty[2] : ty[1];
                int m = 3;
                for (int k = 0; k < 3 && m > 0; ++k) {
                    const int ka = ccw ? k : (3 - k) % 3;
                    const int kb = ccw ? (k + 1) % 3 : (2 - k + 3) % 3;
                    m = clip_halfplane(px, py, m, sx[ka], sy[ka], sx[kb], sy[kb], qx, qy);
                    for (int i = 0; i < m; ++i) {
                        px[i] = qx[i];
                        py[i] = qy[i];
                    }
                }
                if (m < 3) continue;
                // source values at its vertices
                double fv[FC][3];
                const double* r = S.rec + int64_t(e) * RS;
#pragma unroll
                for (int f = 0; f < FC; ++f)
#pragma unroll
                    for (int k = 0; k < 3; ++k)
                        fv[f][k] = f >= S.F ? 0.0
                                            : (S.F == 1 ? r[RecValues<2>::value + k]
                                                        : S.values[int64_t(f) * S.n + sv[k]]);
                for (int i = 1; i + 1 < m; ++i) {
                    const double ar =
                        0.5 * ((px[i] - px[0]) * (py[i + 1] - py[0]) - (px[i + 1] - px[0]) * (py[i] - py[0]));
                    if (!(ar > 0.0)) continue;
                    area += ar;
                    const double w = ar / 3.0;
#pragma unroll
                    for (int qd = 0; qd < 3; ++qd) {
                        // quadrature point: 2/3 at sub-triangle vertex qd, 1/6 at the others
                        const double l0 = qd == 0 ? 2.0 / 3.0 : 1.0 / 6.0;
                        const double l1 = qd == 1 ? 2.0 / 3.0 : 1.0 / 6.0;
                        const double l2 = qd == 2 ? 2.0 / 3.0 : 1.0 / 6.0;
                        const double q[2] = {l0 * px[0] + l1 * px[i] + l2 * px[i + 1],
                                             l0 * py[0] + l1 * py[i] + l2 * py[i + 1]};
                        double mu[3];
                        (void)barycentric<2>(r, q, mu);
                        const double dx = q[0] - tx[0], dy = q[1] - ty[0];
                        const double psi1 = a00 * dx + a01 * dy, psi2 = a10 * dx + a11 * dy;
                        const double psi[3] = {1.0 - psi1 - psi2, psi1, psi2};
#pragma unroll
                        for (int f = 0; f < FC; ++f) {
                            const double fs = mu[0] * fv[f][0] + mu[1] * fv[f][1] + mu[2] * fv[f][2];
#pragma unroll
                            for (int k = 0; k < 3; ++k) acc[f][k] = fma(w * fs, psi[k], acc[f][k]);
                        }
                    }
                }
            }
        }
#pragma unroll
    for (int f = 0; f < FC; ++f) {
        if (f >= S.F) break;
#pragma unroll
        for (int k = 0; k < 3; ++k) beta[(int64_t(f) * E + t) * 3 + k] = acc[f][k];
    }
    if (area_out) area_out[t] = area;
    // target elements the source does not cover entirely
    if (area < vol[t] * (1.0 - 1e-12)) atomicAdd(n_partial, 1ull);
}

__global__ void k_fill_f64(double* __restrict__ p, int64_t n, double v) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
        p[i] = v;
}

ft_status transfer_supermesh(ft_target* T, ft_source* S, double* area, hipStream_t s) {
    const int F = S->F;
    zero_counters(T->counters, 2, s);
    T->ood_mode = 1;   // counters[1]: target elements not entirely inside the source
    // no control: g = 0 (the load vector is exact, alpha = 0 in the solve)
    k_fill_f64<<<grid_for(int64_t(F) * T->n, 256), 256, 0, s>>>(T->g, int64_t(F) * T->n, 0.0);
    const unsigned grid = grid_for(T->E, 256);
    if (F == 1)
        k_supermesh2d<1><<<grid, 256, 0, s>>>(source_view(S), S->coords, T->coords, T->n, T->conn, T->vol, T->E,
                                              T->beta, area, T->counters + 1);
    else
        k_supermesh2d<4><<<grid, 256, 0, s>>>(source_view(S), S->coords, T->coords, T->n, T->conn, T->vol, T->E,
                                              T->beta, area, T->counters + 1);
    FT_TRY_HIP(hipGetLastError());
    return assemble_residual(T, F, nullptr, 0, false, s);
}

}  // namespace ft
