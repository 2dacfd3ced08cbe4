"""Exact intersection-based (supermesh) load vector on small tetrahedral meshes
(oracle side, test infrastructure).

Sec. 3: b_k = sum over target elements t of the integral of f^s psi_k over t,
split over the non-empty intersections t cap s with the source elements s.
On each intersection the P1 source field and the P1 target basis are linear,
so their product is quadratic, and the degree-2 four-point rule on any
tetrahedralization of the convex polyhedron t cap s integrates it exactly.

The polyhedron is found here by vertex enumeration, a method unrelated to the
clipping the library uses: t cap s is the set where the eight face
half-spaces of t and s all hold, and its vertices are the points where three
of the eight face planes meet and every half-space holds.  The convex hull of
those points is then split into tetrahedra by a Delaunay triangulation
(scipy's Qhull).  Degenerate intersections (a face, an edge or a point) have
zero volume and are dropped.

Parity: pinned by closed forms (a tetrahedron and its translate, and a
tetrahedron and its reflection through its centroid, whose intersection is an
octahedron of half its volume), the partition identity
sum_s |t cap s| = |t|, the exact integral sum_k b_k = integral f^s, a source
equal to the target giving b = M F, and an affine source reproduced exactly.
"""
from __future__ import annotations

import itertools

import numpy as np
from scipy.spatial import Delaunay, QhullError, cKDTree

from . import geometry
from .source import barycentric_cramer

_TRIPLES = np.array(list(itertools.combinations(range(8), 3)))


def face_planes(tet: np.ndarray):
    """(n (4, 3), c (4,)) with n_k . x + c_k >= 0 inside: face k is opposite
    vertex k, the normals have unit length."""
    n = np.empty((4, 3))
    c = np.empty(4)
    for k in range(4):
        a, b, d = (tet[i] for i in range(4) if i != k)
        nk = np.cross(b - a, d - a)
        nk /= np.linalg.norm(nk)
        ck = -nk @ a
        if nk @ tet[k] + ck < 0:
            nk, ck = -nk, -ck
        n[k], c[k] = nk, ck
    return n, c


def intersection_vertices(T: np.ndarray, S: np.ndarray, tol: float = 1e-12):
    """Vertices of the convex polyhedron T cap S (K, 3); K < 4 when it has no volume."""
    nt, ct = face_planes(T)
    ns, cs = face_planes(S)
    n = np.concatenate([nt, ns])
    c = np.concatenate([ct, cs])
    A = n[_TRIPLES]                                  # (56, 3, 3)
    rhs = -c[_TRIPLES]                               # (56, 3)
    ok = np.abs(np.linalg.det(A)) > 1e-12
    x = np.linalg.solve(A[ok], rhs[ok][..., None])[..., 0]
    scale = max(np.abs(T).max(), np.abs(S).max(), 1.0)
    inside = (x @ n.T + c >= -tol * scale).all(axis=1)
    x = x[inside]
    if len(x) == 0:
        return x
    # the same vertex from several triples of planes
    keep = []
    for i, p in enumerate(x):
        if all(np.linalg.norm(p - x[j]) > 1e-10 * scale for j in keep):
            keep.append(i)
    return x[keep]


def intersect(T: np.ndarray, S: np.ndarray):
    """Tetrahedra (m, 4, 3) and their volumes (m,) that fill T cap S."""
    v = intersection_vertices(T, S)
    if len(v) < 4:
        return np.empty((0, 4, 3)), np.empty(0)
    try:
        tets = v[Delaunay(v).simplices]
    except QhullError:          # flat: no volume
        return np.empty((0, 4, 3)), np.empty(0)
    vol = np.abs(np.linalg.det(tets[:, 1:] - tets[:, :1])) / 6.0
    big = vol > 1e-15 * np.abs(v).max() ** 3
    return tets[big], vol[big]


def intersections(tc, tconn, sc, sconn):
    """Sub-tetrahedra of every non-empty t cap s.

    Returns (t ids (K,), s ids (K,), vertices (K, 4, 3), volumes (K,)).
    """
    tc = np.asarray(tc, dtype=np.float64)
    sc = np.asarray(sc, dtype=np.float64)
    ct = tc[tconn].mean(axis=1)
    cs = sc[sconn].mean(axis=1)
    rt = np.linalg.norm(tc[tconn] - ct[:, None], axis=2).max()
    rs = np.linalg.norm(sc[sconn] - cs[:, None], axis=2).max()
    cand = cKDTree(cs).query_ball_point(ct, rt + rs + 1e-12)
    ts, ss, vs, vols = [], [], [], []
    for t, slist in enumerate(cand):
        T = tc[tconn[t]]
        for s in slist:
            sub, vol = intersect(T, sc[sconn[s]])
            for q in range(len(vol)):
                ts.append(t); ss.append(s); vs.append(sub[q]); vols.append(vol[q])
    return np.array(ts, dtype=np.int64), np.array(ss, dtype=np.int64), np.array(vs).reshape(-1, 4, 3), \
        np.array(vols)


def supermesh_projection(tc, tconn, sc, sconn, svals, pieces=None):
    """Exact b (F, n_t), the intersection volume per target element and the
    exact integral of f^s over the covered part of the target."""
    tc = np.asarray(tc, dtype=np.float64)
    sc = np.asarray(sc, dtype=np.float64)
    tconn = np.asarray(tconn)
    sconn = np.asarray(sconn)
    svals = np.atleast_2d(np.asarray(svals, dtype=np.float64))
    F = svals.shape[0]
    if pieces is None:
        pieces = intersections(tc, tconn, sc, sconn)
    ts, ss, vs, vol = pieces
    T = tc[tconn[ts]]                                   # (K, 4, 3)
    S = sc[sconn[ss]]
    pts, w = geometry.quadrature_rule(3)
    q = np.einsum("qk,pkc->pqc", pts, vs)               # (K, 4q, 3)
    psi = barycentric_cramer(T[:, None], q)             # (K, 4q, 4)
    mu = barycentric_cramer(S[:, None], q)
    fs = np.einsum("pqk,fpk->fpq", mu, svals[:, sconn[ss]])
    loc = np.einsum("p,q,fpq,pqk->fpk", vol, w, fs, psi)
    b = np.zeros((F, tc.shape[0]))
    for f in range(F):
        np.add.at(b[f], tconn[ts].ravel(), loc[f].ravel())
    vol_sum = np.zeros(tconn.shape[0])
    np.add.at(vol_sum, ts, vol)
    int_fs = np.einsum("p,q,fpq->f", vol, w, fs)
    return {"b": b, "vol_sum": vol_sum, "int_fs": int_fs}
