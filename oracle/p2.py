"""Quadratic (P2) target elements for the CV-MC transfer (oracle side, test
infrastructure).

Sec. 2 states the Galerkin projection for any target finite-element space
V_t = span{psi_i}, and the error bounds of App. A are for degree p; the
control g = I_h f^s is the interpolant in V_t (sec. 4.1 step 1).  Here V_t
holds Lagrange elements of degree 2 on straight-sided triangles and
tetrahedra.  Degrees of freedom of an element: its d+1 vertices, then its
edge midpoints in the order of LOCAL_EDGES (vertex pairs a < b,
lexicographic).  In barycentric coordinates the basis functions are
    vertex k:    l_k (2 l_k - 1),
    edge (a, b): 4 l_a l_b;
they add up to 1, so sum_i b_i estimates the integral of f^s and
m^T x = sum_i b_i (m = M 1) as for P1.

The transfer follows sec. 4.1 with psi the P2 basis:
  step 1  g = f^s at every P2 node (vertices and midpoints);
  step 2  b_g = alpha M g (g is in V_t, so the control load is exact);
  step 3  N uniform samples per element, drawn exactly as for P1 from the
          element's vertices (``sampling``);
  step 4  f^s(X) by query; g(X) = sum_i g_i psi_i(X);
  step 5  beta_ti = |Omega_t|/N sum_j (f^s(X_tj) - alpha g(X_tj)) psi_i(X_tj);
  step 6  b = b_g + assembled beta;  step 7  solve M x = b.

The element mass matrix is |Omega_t| times a reference matrix whose entries
are integrals of products of the basis polynomials, taken monomial by
monomial with the Dirichlet formula.

Parity: pinned by the reference mass matrix against a collapsed
Gauss-Legendre rule (a different integration method), the nodal (Kronecker)
property and the partition of unity of the basis, exact reproduction of a
quadratic field (alpha = 1, any N), conservation of a constant for any
alpha, m^T x = sum b, and the unbiasedness of b against its exact value for
a cubic field (z-scores over realizations).
"""
from __future__ import annotations

import itertools
import math

import numpy as np
import scipy.sparse as sp

from . import cvmc, geometry, sampling

LOCAL_EDGES = {2: [(0, 1), (0, 2), (1, 2)], 3: [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]}


def n_basis(dim: int) -> int:
    return (dim + 1) * (dim + 2) // 2


def basis(lam: np.ndarray) -> np.ndarray:
    """P2 basis at barycentric points lam (..., d+1) -> (..., n_basis)."""
    dim = lam.shape[-1] - 1
    cols = [lam[..., k] * (2.0 * lam[..., k] - 1.0) for k in range(dim + 1)]
    cols += [4.0 * lam[..., a] * lam[..., b] for a, b in LOCAL_EDGES[dim]]
    return np.stack(cols, axis=-1)


def _polys(dim: int):
    """Basis functions as {exponent tuple: coefficient} in the barycentric coordinates."""
    out = []
    for k in range(dim + 1):
        e2 = tuple(2 if i == k else 0 for i in range(dim + 1))
        e1 = tuple(1 if i == k else 0 for i in range(dim + 1))
        out.append({e2: 2.0, e1: -1.0})
    for a, b in LOCAL_EDGES[dim]:
        out.append({tuple(1 if i in (a, b) else 0 for i in range(dim + 1)): 4.0})
    return out


def reference_mass(dim: int) -> np.ndarray:
    """M^t = |Omega_t| * reference_mass(dim): integrals of psi_i psi_j over a unit-measure simplex."""
    P = _polys(dim)
    nb = len(P)
    Mr = np.zeros((nb, nb))
    for i in range(nb):
        for j in range(nb):
            s = 0.0
            for ea, ca in P[i].items():
                for eb, cb in P[j].items():
                    s += ca * cb * geometry.dirichlet_monomial_integral(tuple(x + y for x, y in zip(ea, eb)), 1.0)
            Mr[i, j] = s
    return Mr


def vertex_conn(conn2: np.ndarray, dim: int) -> np.ndarray:
    return np.ascontiguousarray(conn2[:, : dim + 1])


def mass_matrix(coords: np.ndarray, conn2: np.ndarray) -> sp.csr_matrix:
    dim = coords.shape[1]
    nb = n_basis(dim)
    vol = geometry.element_measures(coords, vertex_conn(conn2, dim))
    Mr = reference_mass(dim)
    rows = np.repeat(conn2, nb, axis=1).ravel()
    cols = np.tile(conn2, (1, nb)).ravel()
    vals = (vol[:, None, None] * Mr[None]).reshape(len(vol), -1).ravel()
    n = coords.shape[0]
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


def element_loads(coords, conn2, g, y, lam, alpha, elems):
    """Step 5 with the P2 basis: beta (F, E', n_basis)."""
    dim = coords.shape[1]
    vol = geometry.element_measures(coords, vertex_conn(conn2, dim)[elems])
    psi = basis(lam)                                                 # (E', N, nb)
    g_at = np.einsum("tjk,ftk->ftj", psi, g[:, conn2[elems]])        # g(X_tj)
    r = y - alpha * g_at
    beta = cvmc.neumaier_sum(r[..., None] * psi[None], axis=2)
    return beta * (vol / lam.shape[1])[None, :, None], r


def transfer(coords, conn2, query, n_samples, alpha=1.0, seed=0, stream=0, chunk_elems=20_000, stratified=False):
    """Whole CV-MC transfer onto a P2 target (coords of every P2 node, conn2 (E, n_basis))."""
    coords = np.asarray(coords, dtype=np.float64)
    conn2 = np.asarray(conn2, dtype=np.int64)
    dim = coords.shape[1]
    n, E = coords.shape[0], conn2.shape[0]
    conn = vertex_conn(conn2, dim)
    M = mass_matrix(coords, conn2)
    g = np.atleast_2d(query(coords))                                  # step 1
    F = g.shape[0]
    b_g = alpha * np.stack([M @ gf for gf in g])                      # step 2
    beta = np.empty((F, E, n_basis(dim)))
    var_terms = np.empty((F, E))
    for s in range(0, E, chunk_elems):
        el = np.arange(s, min(E, s + chunk_elems))
        lam, X = cvmc.query_points(coords, conn, n_samples, seed, stream, el, stratified)   # step 3
        y = np.atleast_2d(query(X.reshape(-1, dim))).reshape(F, el.size, n_samples)       # step 4
        beta[:, el], r = element_loads(coords, conn2, g, y, lam, alpha, el)                # step 5
        var_terms[:, el] = cvmc.element_variance_terms(coords, conn, r, el)
    b_res = cvmc.assemble(conn2, beta, n)                             # step 6
    b = b_g + b_res
    x = cvmc.solve_mass(M, b, dim)                                    # step 7
    m = np.asarray(M.sum(axis=1)).ravel()
    report = cvmc.conservation_report(b, x, m)
    for f, rep in enumerate(report):
        rep["sum_b_stderr"] = math.sqrt(math.fsum(var_terms[f])) if n_samples >= 2 else -1.0
    return {"g": g, "b_g": b_g, "beta": beta, "b_res": b_res, "b": b, "x": x, "M": M, "m": m,
            "report": report, "var_terms": var_terms}


def exact_load(coords, conn2, f, order: int = 8):
    """b_i = integral f psi_i for a callable f (points (K, d) -> (F, K)), by a
    collapsed Gauss-Legendre rule of ``order`` points per direction on each
    element (exact for polynomials f up to degree 2 order - 3)."""
    coords = np.asarray(coords, dtype=np.float64)
    conn2 = np.asarray(conn2, dtype=np.int64)
    dim = coords.shape[1]
    lam, w = collapsed_rule(dim, order)
    conn = vertex_conn(conn2, dim)
    vol = geometry.element_measures(coords, conn)
    X = np.einsum("qk,tkc->tqc", lam, coords[conn])                   # (E, q, d)
    fv = np.atleast_2d(f(X.reshape(-1, dim))).reshape(-1, len(conn), len(w))
    psi = basis(lam)                                                  # (q, nb)
    loc = np.einsum("t,q,ftq,qi->fti", vol, w, fv, psi)
    return cvmc.assemble(conn2, loc, coords.shape[0])


def collapsed_rule(dim: int, order: int):
    """Barycentric points and weights (summing to 1) of the Duffy-collapsed
    tensor Gauss-Legendre rule on the reference simplex."""
    x, wx = np.polynomial.legendre.leggauss(order)
    u, wu = 0.5 * (x + 1.0), 0.5 * wx
    pts, ws = [], []
    if dim == 2:
        for (a, wa), (b, wb) in itertools.product(zip(u, wu), zip(u, wu)):
            px, py = a, b * (1.0 - a)
            pts.append((1.0 - px - py, px, py))
            ws.append(wa * wb * (1.0 - a) * 2.0)        # reference area 1/2
    else:
        for (a, wa), (b, wb), (c, wc) in itertools.product(zip(u, wu), zip(u, wu), zip(u, wu)):
            px, py, pz = a, b * (1.0 - a), c * (1.0 - a) * (1.0 - b)
            pts.append((1.0 - px - py - pz, px, py, pz))
            ws.append(wa * wb * wc * (1.0 - a) ** 2 * (1.0 - b) * 6.0)   # reference volume 1/6
    return np.array(pts), np.array(ws)
