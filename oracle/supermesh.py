"""Exact intersection-based (supermesh) load vector on small 2D meshes (oracle side).

Sec. 3: b_k = sum over target elements t of the integral of f^s psi_k over t,
and that integral splits over the non-empty intersections t cap s with the
source elements s.  On each intersection both the P1 source field and the P1
target basis are linear, so their product is quadratic and the degree-2 Gauss
rule on a fan triangulation of the convex intersection polygon is exact (the
intersection-integration procedure of sec. 3: clip, order counter-clockwise,
fan from an anchor vertex, quadrature per sub-triangle, sum).

Clipping is plain Sutherland-Hodgman of the target triangle against the three
half-planes of the (counter-clockwise) source triangle.

It also gives the exact error metrics of sec. 5.1 on the supermesh: the
relative L2 accuracy error (e = f^s - f^t is linear on each sub-triangle, so
integral e^2 = |T|/6 (sum e_k^2 + sum_{k<l} e_k e_l)) and the relative
conservation error.

Parity: pinned by the partition identity sum_s |t cap s| = |t|, the exact
integral sum_k b_k = integral f^s, and source == target giving b = M F.
"""
from __future__ import annotations

import numpy as np
from scipy.spatial import cKDTree

from . import geometry
from .source import barycentric_cramer


def _clip(poly, a, b):
    """Keep the part of polygon ``poly`` left of the directed line a -> b."""
    out = []
    n = len(poly)
    if n == 0:
        return out

    def side(p):
        return (b[0] - a[0]) * (p[1] - a[1]) - (b[1] - a[1]) * (p[0] - a[0])

    for i in range(n):
        p, q = poly[i], poly[(i + 1) % n]
        sp_, sq = side(p), side(q)
        if sp_ >= 0:
            out.append(p)
        if (sp_ >= 0) != (sq >= 0):
            t = sp_ / (sp_ - sq)
            out.append((p[0] + t * (q[0] - p[0]), p[1] + t * (q[1] - p[1])))
    return out


def intersect(tri_t: np.ndarray, tri_s: np.ndarray):
    """Convex polygon t cap s (list of vertices, counter-clockwise)."""
    poly = [tuple(v) for v in tri_t]
    for k in range(3):
        poly = _clip(poly, tri_s[k], tri_s[(k + 1) % 3])
        if not poly:
            break
    return poly


def _area(a, b, c):
    return 0.5 * ((b[0] - a[0]) * (c[1] - a[1]) - (c[0] - a[0]) * (b[1] - a[1]))


def _pairs(tc, tconn, sc, sconn):
    """Candidate (t, s) pairs whose circumscribing balls around the centroids overlap."""
    ct = tc[tconn].mean(axis=1)
    cs = sc[sconn].mean(axis=1)
    rt = np.linalg.norm(tc[tconn] - ct[:, None], axis=2).max()
    rs = np.linalg.norm(sc[sconn] - cs[:, None], axis=2).max()
    tree = cKDTree(cs)
    return ct, tree.query_ball_point(ct, rt + rs + 1e-12)


def fan(poly):
    """Sub-triangles (anchor = first vertex) of a convex polygon with positive area."""
    for i in range(1, len(poly) - 1):
        a, b, c = poly[0], poly[i], poly[i + 1]
        ar = _area(a, b, c)
        if ar > 0:
            yield np.array([a, b, c]), ar


def intersections(tc, tconn, sc, sconn):
    """Fan sub-triangles of every non-empty t cap s.

    Returns (t ids (K,), s ids (K,), vertices (K, 3, 2), areas (K,)).
    """
    tc = np.asarray(tc, dtype=np.float64)
    sc = np.asarray(sc, dtype=np.float64)
    ts, ss, vs, ars = [], [], [], []
    _, cand = _pairs(tc, tconn, sc, sconn)
    for t, slist in enumerate(cand):
        T = tc[tconn[t]]
        for s in slist:
            poly = intersect(T, sc[sconn[s]])
            if len(poly) < 3:
                continue
            for sub, ar in fan(poly):
                ts.append(t); ss.append(s); vs.append(sub); ars.append(ar)
    return np.array(ts), np.array(ss), np.array(vs).reshape(-1, 3, 2), np.array(ars)


def supermesh_projection(tc, tconn, sc, sconn, svals, x_target=None, pieces=None):
    """Exact b (F, n_t) and, if x_target (F, n_t) is given, exact error integrals.

    ``pieces`` may carry a precomputed ``intersections(...)`` result.
    Returns dict(b, area_sum (per target element), int_fs, and when x_target
    is given: int_e2, int_fs2, int_ft, E_L2, E_mass).
    """
    tc = np.asarray(tc, dtype=np.float64)
    sc = np.asarray(sc, dtype=np.float64)
    tconn = np.asarray(tconn)
    sconn = np.asarray(sconn)
    svals = np.atleast_2d(np.asarray(svals, dtype=np.float64))
    F = svals.shape[0]
    if pieces is None:
        pieces = intersections(tc, tconn, sc, sconn)
    ts, ss, vs, ar = pieces
    T = tc[tconn[ts]]                                   # (K, 3, 2) target element of each piece
    S = sc[sconn[ss]]                                   # (K, 3, 2) source element of each piece
    pts, w = geometry.quadrature_rule(2)
    q = np.einsum("qk,pkc->pqc", pts, vs)               # quadrature points (K, 3, 2)
    psi = barycentric_cramer(T[:, None], q)             # target basis at q (K, 3q, 3)
    mu = barycentric_cramer(S[:, None], q)              # source basis at q
    fs = np.einsum("pqk,fpk->fpq", mu, svals[:, sconn[ss]])     # f^s at q (F, K, 3q)
    loc = np.einsum("p,q,fpq,pqk->fpk", ar, w, fs, psi)         # (F, K, 3) local loads
    b = np.zeros((F, tc.shape[0]))
    for f in range(F):
        np.add.at(b[f], tconn[ts].ravel(), loc[f].ravel())
    area_sum = np.zeros(tconn.shape[0])
    np.add.at(area_sum, ts, ar)
    int_fs = np.einsum("p,q,fpq->f", ar, w, fs)
    out = {"b": b, "area_sum": area_sum, "int_fs": int_fs}
    if x_target is not None:
        xt = np.atleast_2d(x_target)
        psi_v = barycentric_cramer(T[:, None], vs)      # (K, 3 vertices, 3)
        mu_v = barycentric_cramer(S[:, None], vs)
        fs_v = np.einsum("pvk,fpk->fpv", mu_v, svals[:, sconn[ss]])
        ft_v = np.einsum("pvk,fpk->fpv", psi_v, xt[:, tconn[ts]])

        def lin_sq(e):   # exact integral of a squared linear function per piece
            return ar / 6.0 * ((e * e).sum(axis=-1) + e[..., 0] * e[..., 1]
                               + e[..., 0] * e[..., 2] + e[..., 1] * e[..., 2])
        int_e2 = lin_sq(fs_v - ft_v).sum(axis=1)
        int_fs2 = lin_sq(fs_v).sum(axis=1)
        int_ft = (ar * ft_v.mean(axis=-1)).sum(axis=1)
        out.update(int_e2=int_e2, int_fs2=int_fs2, int_ft=int_ft,
                   E_L2=np.sqrt(int_e2 / int_fs2),
                   E_mass=np.abs(int_fs - int_ft) / np.abs(int_fs))
    return out
