"""Target-mesh geometry, P1 basis, mass matrix and quadrature (oracle side).

Sec. 2: M_ki = integral of psi_k psi_i over the domain (mass matrix), computed
exactly on the target mesh by Gaussian quadrature; the P1 hat function psi_i
equals the barycentric coordinate of vertex i inside each element it touches.
The element measure of a simplex is |det J| / d!, J = [x_1-x_0, ..., x_d-x_0]
(sec. 4.1 uses |Omega_t| in the uniform density and in the estimator).

Two independent routes to M are provided and must agree:
  * closed form of the P1 element matrix, |T| (1 + delta_kl) / ((d+1)(d+2));
  * a degree-2 rule (exact for the quadratic products psi_k psi_l): d+1
    points at barycentric (a, b, ..., b) and permutations, weights 1/(d+1),
    b = (d + 2 - sqrt(d + 2)) / ((d + 1)(d + 2)), a = 1 - d b (Stroud's
    T_n:2-1); triangle (2/3, 1/6, 1/6), tetrahedron a = (5 + 3 sqrt 5)/20,
    b = (5 - sqrt 5)/20.

Parity: pinned by the Dirichlet monomial formula (quadrature exactness up to
degree 2), sum(M) = |domain|, and closed form == quadrature.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp


def quadrature_rule(dim: int):
    """(barycentric points (q, d+1), weights (q,) summing to 1): degree-2 exact."""
    if dim == 2:
        a, b = 2.0 / 3.0, 1.0 / 6.0
    elif dim == 3:
        s5 = math.sqrt(5.0)
        a, b = (5.0 + 3.0 * s5) / 20.0, (5.0 - s5) / 20.0
    elif 4 <= dim <= 6:
        b = (dim + 2 - math.sqrt(dim + 2)) / ((dim + 1) * (dim + 2))
        a = 1.0 - dim * b
    else:
        raise ValueError("dim must lie in [2, 6]")
    pts = np.full((dim + 1, dim + 1), b)
    np.fill_diagonal(pts, a)
    w = np.full(dim + 1, 1.0 / (dim + 1))
    return pts, w


def signed_dets(coords: np.ndarray, conn: np.ndarray) -> np.ndarray:
    """det J_t for every element (positive for counter-clockwise / right-handed)."""
    x = coords[conn]
    jac = x[:, 1:, :] - x[:, :1, :]          # rows are edge vectors
    return np.linalg.det(jac)


def element_measures(coords: np.ndarray, conn: np.ndarray) -> np.ndarray:
    """|Omega_t| = |det J_t| / d!."""
    dim = coords.shape[1]
    return np.abs(signed_dets(coords, conn)) / math.factorial(dim)


def local_mass_closed_form(dim: int, vol: float) -> np.ndarray:
    return vol * (np.ones((dim + 1, dim + 1)) + np.eye(dim + 1)) / ((dim + 1) * (dim + 2))


def local_mass_quadrature(dim: int, vol: float) -> np.ndarray:
    pts, w = quadrature_rule(dim)
    # psi_k at quadrature point q is the barycentric coordinate pts[q, k]
    return vol * np.einsum("q,qk,ql->kl", w, pts, pts)


def mass_matrix(coords: np.ndarray, conn: np.ndarray, method: str = "closed") -> sp.csr_matrix:
    """Assembled P1 mass matrix as scipy CSR (sum of element matrices)."""
    dim = coords.shape[1]
    vol = element_measures(coords, conn)
    if method == "closed":
        ref = local_mass_closed_form(dim, 1.0)
    elif method == "quadrature":
        ref = local_mass_quadrature(dim, 1.0)
    else:
        raise ValueError(method)
    nl = dim + 1
    rows = np.repeat(conn, nl, axis=1).ravel()
    cols = np.tile(conn, (1, nl)).ravel()
    vals = (vol[:, None] * ref.ravel()[None, :]).ravel()
    n = coords.shape[0]
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


def lumped_mass(coords: np.ndarray, conn: np.ndarray) -> np.ndarray:
    """m_i = integral of psi_i = sum over elements touching i of |Omega_t| / (d+1)."""
    dim = coords.shape[1]
    vol = element_measures(coords, conn)
    m = np.zeros(coords.shape[0])
    np.add.at(m, conn.ravel(), np.repeat(vol / (dim + 1), dim + 1))
    return m


def dirichlet_monomial_integral(exps, vol: float) -> float:
    """Exact integral over a d-simplex of prod_k lambda_k^{a_k}: d! prod a_k! |T| / (d + sum a)!."""
    d = len(exps) - 1
    num = math.factorial(d) * math.prod(math.factorial(a) for a in exps)
    return num * vol / math.factorial(d + sum(exps))
