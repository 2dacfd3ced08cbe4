"""Mesh-backed P1 source: localization and evaluation (oracle side).

The method itself only needs point values f^s(x) (sec. 2: the source may be
known only through pointwise evaluations; algorithm step 1 and step 4 query
it).  For benchmarks the source is a P1 field on a source mesh (the test
functions of sec. 5.1 are nodal interpolants on the source mesh), evaluated at
a point by finding the containing source element and interpolating with its
barycentric coordinates mu.

Localization rule (reading; the paper is silent on ties): the source element
maximising min_k mu_k(x); among exact ties, the lowest element id.  A point
whose best min_k mu_k is below -1e-10 is out of the domain: it is counted and
evaluated by extrapolation from that best element.

This oracle finds the rule's winner exactly and independently of any bin grid:
an element can contain x only if its centroid lies within R_max of x, where
R_max is the largest centroid-to-vertex distance of the mesh, so all centroids
within R_max (a k-d tree query, widened until the k-th neighbour is farther)
are the complete candidate set; out-of-domain points fall back to brute force
over every element.  Barycentric coordinates use Cramer's rule (ratios of
signed simplex volumes).

Parity: pinned against brute force over all elements with barycentrics from a
dense linear solve, on small meshes.
"""
from __future__ import annotations

import numpy as np
from scipy.spatial import cKDTree

from . import geometry

OUT_OF_DOMAIN_TOL = -1e-10


def _det2(a, b):
    return a[..., 0] * b[..., 1] - a[..., 1] * b[..., 0]


def _det3(a, b, c):
    return (a[..., 0] * (b[..., 1] * c[..., 2] - b[..., 2] * c[..., 1])
            - a[..., 1] * (b[..., 0] * c[..., 2] - b[..., 2] * c[..., 0])
            + a[..., 2] * (b[..., 0] * c[..., 1] - b[..., 1] * c[..., 0]))


def barycentric_cramer(verts: np.ndarray, p: np.ndarray) -> np.ndarray:
    """mu of points p (..., d) in simplices verts (..., d+1, d) by Cramer's rule."""
    d = p.shape[-1]
    e = [verts[..., k, :] - verts[..., 0, :] for k in range(1, d + 1)]
    r = p - verts[..., 0, :]
    if d == 2:
        den = _det2(e[0], e[1])
        m1 = _det2(r, e[1]) / den
        m2 = _det2(e[0], r) / den
        return np.stack([1.0 - m1 - m2, m1, m2], axis=-1)
    den = _det3(e[0], e[1], e[2])
    m1 = _det3(r, e[1], e[2]) / den
    m2 = _det3(e[0], r, e[2]) / den
    m3 = _det3(e[0], e[1], r) / den
    return np.stack([1.0 - m1 - m2 - m3, m1, m2, m3], axis=-1)


class P1Source:
    """P1 field(s) on a simplex mesh; values has shape (F, n_nodes)."""

    def __init__(self, coords: np.ndarray, conn: np.ndarray, values: np.ndarray):
        self.coords = np.asarray(coords, dtype=np.float64)
        self.conn = np.asarray(conn, dtype=np.int64)
        v = np.asarray(values, dtype=np.float64)
        self.values = v[None, :] if v.ndim == 1 else v
        self.dim = self.coords.shape[1]
        verts = self.coords[self.conn]
        self.centroids = verts.mean(axis=1)
        self.r_max = float(np.linalg.norm(verts - self.centroids[:, None, :], axis=2).max()) * (1 + 1e-9)
        self.tree = cKDTree(self.centroids)
        self.vol = geometry.element_measures(self.coords, self.conn)
        self.heights = self._heights(verts)

    def _heights(self, verts):
        """h_k = d |Omega_s| / |face opposite k|: distance from vertex k to that face."""
        d = self.dim
        faces = []
        for k in range(d + 1):
            others = [verts[:, i, :] for i in range(d + 1) if i != k]
            if d == 2:
                faces.append(np.linalg.norm(others[1] - others[0], axis=1))
            else:
                faces.append(0.5 * np.linalg.norm(np.cross(others[1] - others[0], others[2] - others[0]), axis=1))
        return d * self.vol[:, None] / np.stack(faces, axis=1)

    # -- localization ---------------------------------------------------------
    def _best(self, cand: np.ndarray, p: np.ndarray):
        """Rule winner among candidate ids cand (n, K) for points p (n, d)."""
        mu = barycentric_cramer(self.coords[self.conn[cand]], p[:, None, :])   # (n, K, d+1)
        mn = mu.min(axis=2)
        best_val = mn.max(axis=1)
        # lowest id among the candidates that attain the maximum
        masked = np.where(mn == best_val[:, None], cand, np.iinfo(np.int64).max)
        best = masked.min(axis=1)
        sel = np.argmax(masked == best[:, None], axis=1)
        return best, mu[np.arange(len(p)), sel], best_val

    def locate(self, points: np.ndarray, chunk: int = 200_000):
        """Returns (elem ids (n,), mu (n, d+1), out_of_domain mask (n,))."""
        points = np.asarray(points, dtype=np.float64)
        n = points.shape[0]
        ids = np.empty(n, dtype=np.int64)
        mus = np.empty((n, self.dim + 1))
        E = self.conn.shape[0]
        for s in range(0, n, chunk):
            p = points[s:s + chunk]
            k = min(16, E)
            todo = np.arange(len(p))
            while todo.size:
                dist, cand = self.tree.query(p[todo], k=k)
                if k == 1:
                    dist, cand = dist[:, None], cand[:, None]
                complete = (dist[:, -1] > self.r_max) | (k >= E)
                done = todo[complete]
                if done.size:
                    b, mu, _ = self._best(cand[complete], p[done])
                    ids[s + done] = b
                    mus[s + done] = mu
                todo = todo[~complete]
                k = min(2 * k, E)
        out = mus.min(axis=1) < OUT_OF_DOMAIN_TOL
        for i in np.nonzero(out)[0]:
            b, mu, _ = self._best(np.arange(E)[None, :], points[i:i + 1])
            ids[i], mus[i] = b[0], mu[0]
        out = mus.min(axis=1) < OUT_OF_DOMAIN_TOL
        return ids, mus, out

    def face_distance(self, ids: np.ndarray, mu: np.ndarray) -> np.ndarray:
        """Signed distance from each point to the nearest face of its element."""
        return (mu * self.heights[ids]).min(axis=1)

    def evaluate_at(self, ids: np.ndarray, mu: np.ndarray) -> np.ndarray:
        """y_f = sum_k mu_k F_f[s_k]; returns (F, n)."""
        return np.einsum("nk,fnk->fn", mu, self.values[:, self.conn[ids]])

    def __call__(self, points: np.ndarray) -> np.ndarray:
        ids, mu, _ = self.locate(points)
        return self.evaluate_at(ids, mu)

    def integral(self) -> np.ndarray:
        """Exact integral of each field: sum_s |Omega_s| * mean of its vertex values."""
        return (self.values[:, self.conn].mean(axis=2) * self.vol[None, :]).sum(axis=1)
