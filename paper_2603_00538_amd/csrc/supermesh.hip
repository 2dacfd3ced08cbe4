// Exact intersection-based load vector on P1 triangles and tetrahedra (sec. 3: the
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
                                            : (S.rec_values ? r[RecValues<2>::value + k]
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

// ---- tetrahedra.  t cap s is t cut by the four face half-spaces mu_m >= 0
// of s (mu: the barycentric coordinates of s, from its record).  Cutting a
// tetrahedron by a half-space leaves nothing, the whole tetrahedron, a corner
// tetrahedron (one vertex inside) or a triangular prism (two or three
// vertices inside) that splits into three tetrahedra, so t cap s comes out as
// a set of tetrahedra, each integrated with the four-point degree-2 rule
// (barycentric a = (5 + 3 sqrt 5)/20 at one vertex, b = (5 - sqrt 5)/20 at the
// others, weights 1/4).  The pieces of the four cuts are walked depth first
// on a small stack: popping a piece at depth L pushes at most three at L + 1,
// so at most 1 + 2 * 4 entries are ever held.
constexpr int kTetStack = 9;

// Point at which the segment p -> q crosses the plane, from the plane values sp >= 0 > sq.
__device__ __forceinline__ void cut_point(const double (&p)[3], const double (&q)[3], double sp, double sq,
                                          double (&x)[3]) {
    const double u = sp / (sp - sq);
#pragma unroll
    for (int c = 0; c < 3; ++c) x[c] = fma(u, q[c] - p[c], p[c]);
}

__device__ __forceinline__ void copy3(double* __restrict__ dst, const double (&x)[3]) {
    dst[0] = x[0];
    dst[1] = x[1];
    dst[2] = x[2];
}

// Writes the tetrahedra of {x in P : s(x) >= 0} (s affine, sv its values at
// the vertices of P) to out[0..), 12 doubles each; returns their number.
__device__ __forceinline__ int cut_tet(const double (&P)[4][3], const double (&sv)[4], double* __restrict__ out) {
    int in[4], ou[4], ni = 0, no = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if (sv[i] >= 0.0) in[ni++] = i;
        else ou[no++] = i;
    }
    if (ni == 0) return 0;
    if (ni == 4) {
#pragma unroll
        for (int i = 0; i < 4; ++i) copy3(out + 3 * i, P[i]);
        return 1;
    }
    if (ni == 1) {   // corner (a, ab, ac, ad)
        const int a = in[0];
        copy3(out, P[a]);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            double x[3];
            cut_point(P[a], P[ou[k]], sv[a], sv[ou[k]], x);
            copy3(out + 3 * (k + 1), x);
        }
        return 1;
    }
    // a prism with triangles (p0, p1, p2) and (q0, q1, q2) and edges p_i - q_i:
    // tetrahedra (p0 p1 p2 q0), (p1 p2 q0 q1), (p2 q0 q1 q2)
    double pp[3][3], qq[3][3];
    if (ni == 3) {   // (a, b, c) and (ad, bd, cd)
        const int d = ou[0];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
#pragma unroll
            for (int c = 0; c < 3; ++c) pp[k][c] = P[in[k]][c];
            cut_point(P[in[k]], P[d], sv[in[k]], sv[d], qq[k]);
        }
    } else {         // two inside: (a, ac, ad) and (b, bc, bd)
        const int a = in[0], b = in[1], c0 = ou[0], d0 = ou[1];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            pp[0][c] = P[a][c];
            qq[0][c] = P[b][c];
        }
        cut_point(P[a], P[c0], sv[a], sv[c0], pp[1]);
        cut_point(P[a], P[d0], sv[a], sv[d0], pp[2]);
        cut_point(P[b], P[c0], sv[b], sv[c0], qq[1]);
        cut_point(P[b], P[d0], sv[b], sv[d0], qq[2]);
    }
    copy3(out + 0, pp[0]); copy3(out + 3, pp[1]); copy3(out + 6, pp[2]); copy3(out + 9, qq[0]);
    copy3(out + 12, pp[1]); copy3(out + 15, pp[2]); copy3(out + 18, qq[0]); copy3(out + 21, qq[1]);
    copy3(out + 24, pp[2]); copy3(out + 27, qq[0]); copy3(out + 30, qq[1]); copy3(out + 33, qq[2]);
    return 3;
}

template <int FC>
__global__ __launch_bounds__(256) void k_supermesh3d(SrcView S, const double* __restrict__ X, int64_t n,
                                                     const int32_t* __restrict__ conn, const double* __restrict__ vol,
                                                     int64_t E, double* __restrict__ beta,
                                                     double* __restrict__ vol_out,
                                                     unsigned long long* __restrict__ n_partial) {
    constexpr int RS = RecSize<3>::value;
    constexpr int BS = BoxSize<3>::value;
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= E) return;
    double tv[4][3];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int v = conn[t * 4 + k];
#pragma unroll
        for (int c = 0; c < 3; ++c) tv[k][c] = X[c * n + v];
    }
    // target barycentrics psi_{k+1} = A[k] . (p - tv0), A the inverse of J = [tv1-tv0 | tv2-tv0 | tv3-tv0]
    double J[3][3];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) J[r][c] = tv[c + 1][r] - tv[0][r];
    const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                       J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                       J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    const double id = 1.0 / det;
    double A[3][3];
    A[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) * id;
    A[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id;
    A[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
    A[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) * id;
    A[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
    A[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
    A[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) * id;
    A[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
    A[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
    double lo[3], hi[3], dlo[3], dhi[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        lo[c] = fmin(fmin(tv[0][c], tv[1][c]), fmin(tv[2][c], tv[3][c]));
        hi[c] = fmax(fmax(tv[0][c], tv[1][c]), fmax(tv[2][c], tv[3][c]));
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        dlo[k] = INFINITY;
        dhi[k] = -INFINITY;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const double pr = Dirs<3>::proj(k, tv[i]);
            dlo[k] = fmin(dlo[k], pr);
            dhi[k] = fmax(dhi[k], pr);
        }
    }
    int b0[3], b1[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        b0[c] = bin_of(lo[c] - S.g.hx[c], c, S.g);
        b1[c] = bin_of(hi[c] + S.g.hx[c], c, S.g);
    }
    const double qa = (5.0 + 3.0 * 2.2360679774997896964) / 20.0, qb = (5.0 - 2.2360679774997896964) / 20.0;
    double acc[FC][4];
#pragma unroll
    for (int f = 0; f < FC; ++f)
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[f][k] = 0.0;
    double vsum = 0.0;
    double stk[kTetStack * 12];
    int lvl[kTetStack];
    for (int bz = b0[2]; bz <= b1[2]; ++bz)
        for (int by = b0[1]; by <= b1[1]; ++by)
            for (int bx = b0[0]; bx <= b1[0]; ++bx) {
                const int64_t b = (int64_t(bz) * S.g.nb[1] + by) * S.g.nb[0] + bx;
                const int64_t c1 = S.bin_ptr[b + 1];
                for (int64_t cc = S.bin_ptr[b]; cc < c1; ++cc) {
                    const int e = S.bin_elems[cc];
                    const float* eb = S.box + int64_t(e) * BS;
                    bool miss = false;
#pragma unroll
                    for (int c = 0; c < 3; ++c) miss |= double(eb[c]) > hi[c] || double(eb[3 + c]) < lo[c];
#pragma unroll
                    for (int k = 0; k < 3; ++k) miss |= double(eb[6 + k]) > dhi[k] || double(eb[9 + k]) < dlo[k];
                    if (miss) continue;
                    const double* r = S.rec + int64_t(e) * RS;
                    double fv[FC][4];
#pragma unroll
                    for (int f = 0; f < FC; ++f)
#pragma unroll
                        for (int k = 0; k < 4; ++k)
                            fv[f][k] = f >= S.F ? 0.0
                                                : (S.rec_values ? r[RecValues<3>::value + k]
                                                            : S.values[int64_t(f) * S.n + S.conn[int64_t(e) * 4 + k]]);
                    // depth-first over the cuts by mu_0 .. mu_3 >= 0
#pragma unroll
                    for (int i = 0; i < 4; ++i)
#pragma unroll
                        for (int c = 0; c < 3; ++c) stk[3 * i + c] = tv[i][c];
                    lvl[0] = 0;
                    int top = 1;
                    while (top > 0) {
                        --top;
                        double P[4][3];
#pragma unroll
                        for (int i = 0; i < 4; ++i)
#pragma unroll
                            for (int c = 0; c < 3; ++c) P[i][c] = stk[top * 12 + 3 * i + c];
                        const int L = lvl[top];
                        if (L < 4) {
                            double sv[4];
#pragma unroll
                            for (int i = 0; i < 4; ++i) {
                                double mu[4];
                                (void)barycentric<3>(r, P[i], mu);
                                sv[i] = mu[L];
                            }
                            // popping a depth-3 piece leaves at most 2 + 2 + 2 entries, so
                            // three more always fit; the test only guards the buffer
                            if (top + 3 > kTetStack) continue;
                            const int m = cut_tet(P, sv, stk + top * 12);
                            for (int i = 0; i < m; ++i) lvl[top + i] = L + 1;
                            top += m;
                            continue;
                        }
                        // a piece of t cap s: the four-point rule
                        const double e1[3] = {P[1][0] - P[0][0], P[1][1] - P[0][1], P[1][2] - P[0][2]};
                        const double e2[3] = {P[2][0] - P[0][0], P[2][1] - P[0][1], P[2][2] - P[0][2]};
                        const double e3[3] = {P[3][0] - P[0][0], P[3][1] - P[0][1], P[3][2] - P[0][2]};
                        const double v6 = e1[0] * (e2[1] * e3[2] - e2[2] * e3[1]) -
                                          e1[1] * (e2[0] * e3[2] - e2[2] * e3[0]) +
                                          e1[2] * (e2[0] * e3[1] - e2[1] * e3[0]);
                        const double pv = fabs(v6) / 6.0;
                        if (!(pv > 0.0)) continue;
                        vsum += pv;
                        const double w = 0.25 * pv;
#pragma unroll
                        for (int qd = 0; qd < 4; ++qd) {
                            double q[3];
#pragma unroll
                            for (int c = 0; c < 3; ++c)
                                q[c] = (qd == 0 ? qa : qb) * P[0][c] + (qd == 1 ? qa : qb) * P[1][c] +
                                       (qd == 2 ? qa : qb) * P[2][c] + (qd == 3 ? qa : qb) * P[3][c];
                            double mu[4];
                            (void)barycentric<3>(r, q, mu);
                            const double dx[3] = {q[0] - tv[0][0], q[1] - tv[0][1], q[2] - tv[0][2]};
                            double psi[4];
                            psi[1] = A[0][0] * dx[0] + A[0][1] * dx[1] + A[0][2] * dx[2];
                            psi[2] = A[1][0] * dx[0] + A[1][1] * dx[1] + A[1][2] * dx[2];
                            psi[3] = A[2][0] * dx[0] + A[2][1] * dx[1] + A[2][2] * dx[2];
                            psi[0] = 1.0 - psi[1] - psi[2] - psi[3];
#pragma unroll
                            for (int f = 0; f < FC; ++f) {
                                const double fs = mu[0] * fv[f][0] + mu[1] * fv[f][1] + mu[2] * fv[f][2] +
                                                  mu[3] * fv[f][3];
#pragma unroll
                                for (int k = 0; k < 4; ++k) acc[f][k] = fma(w * fs, psi[k], acc[f][k]);
                            }
                        }
                    }
                }
            }
#pragma unroll
    for (int f = 0; f < FC; ++f) {
        if (f >= S.F) break;
#pragma unroll
        for (int k = 0; k < 4; ++k) beta[(int64_t(f) * E + t) * 4 + k] = acc[f][k];
    }
    if (vol_out) vol_out[t] = vsum;
    if (vsum < vol[t] * (1.0 - 1e-12)) atomicAdd(n_partial, 1ull);
}

__global__ void k_fill_f64(double* __restrict__ p, int64_t n, double v) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
        p[i] = v;
}

ft_status transfer_supermesh(ft_target* T, ft_source* S, double* area, hipStream_t s) {
    const int F = S->F;
    zero_counters(T->counters, 2, s);
    T->ood_mode = 1;   // counters[1]: target elements not entirely inside the source
    T->var_mode = VAR_EXACT;
    // no control: g = 0 (the load vector is exact, alpha = 0 in the solve)
    k_fill_f64<<<grid_for(int64_t(F) * T->n, 256), 256, 0, s>>>(T->g, int64_t(F) * T->n, 0.0);
    const unsigned grid = grid_for(T->E, 256);
    if (T->dim == 3) {
        if (F == 1)
            k_supermesh3d<1><<<grid, 256, 0, s>>>(source_view(S), T->coords, T->n, T->conn, T->vol, T->E, T->beta,
                                                  area, T->counters + 1);
        else
            k_supermesh3d<4><<<grid, 256, 0, s>>>(source_view(S), T->coords, T->n, T->conn, T->vol, T->E, T->beta,
                                                  area, T->counters + 1);
    } else if (F == 1) {
        k_supermesh2d<1><<<grid, 256, 0, s>>>(source_view(S), S->coords, T->coords, T->n, T->conn, T->vol, T->E,
                                              T->beta, area, T->counters + 1);
    } else {
        k_supermesh2d<4><<<grid, 256, 0, s>>>(source_view(S), S->coords, T->coords, T->n, T->conn, T->vol, T->E,
                                              T->beta, area, T->counters + 1);
    }
    FT_TRY_HIP(hipGetLastError());
    return assemble_residual(T, F, nullptr, 0, false, s);
}

}  // namespace ft
