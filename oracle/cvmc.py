"""Control-variate Monte Carlo Galerkin projection (oracle side).

Follows sec. 4.1 step by step, in the paper's notation:

  step 1  g = I_h f^s: query the source at the target nodes (control).
  step 2  b_g,i = integral of alpha g psi_i, assembled element by element with
          the degree-2 Gauss rule (exact for the P1 x P1 product, so it equals
          alpha (M g)_i).
  step 3  N uniform samples X_tj per target element (see ``sampling``).
  step 4  f^s(X_tj) by point query; g(X_tj) = sum_k lambda_k g_{v_k} and
          psi_{v_k}(X_tj) = lambda_k because both live on the target element.
  step 5  b_res,i^t = |Omega_t|/N sum_j (f^s(X_tj) - alpha g(X_tj)) psi_i(X_tj)
          (the residual form of the control-variate element load).
  step 6  b_i = b_g,i + sum over elements of b_res,i^t.
  step 7  solve M f^t = b.

The sum over j in step 5 is compensated (Neumaier) so that the oracle's own
rounding stays far below the parity tolerance.  The solve is a sparse direct
factorisation (SuperLU) up to 2e5 nodes in 2D / 6e4 in 3D, else a plain
Jacobi-CG to 1e-15 (both pinned against each other).

The point-query layout shared with the library is: entries [0, n) are the n
target nodes (step 1), entries [n, n + E N) the samples, element-major
(n + t N + j).

Parity: pinned by special cases (affine source is reproduced exactly with
alpha = 1; constant source conserves sum(b) = c |domain| for every alpha;
source mesh == target mesh reproduces the nodal field), the discrete
conservation identity m^T x = sum(b), unbiasedness against the exact
supermesh load vector, and the N^-1/2 decay of the error.  The standard
error of sum b (App. B) is pinned by a closed-form residual variance (Dirichlet
moments of the barycentric weights), by the spread of sum b over independent
realizations, and by an affine source (zero residual, zero error).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import geometry, sampling


def neumaier_sum(terms: np.ndarray, axis: int) -> np.ndarray:
    """Compensated sum along ``axis`` (vectorised over the other axes)."""
    terms = np.moveaxis(terms, axis, 0)
    s = np.zeros(terms.shape[1:])
    c = np.zeros(terms.shape[1:])
    for term in terms:
        t = s + term
        c += np.where(np.abs(s) >= np.abs(term), (s - t) + term, (term - t) + s)
        s = t
    return s + c


def control_load(coords: np.ndarray, conn: np.ndarray, g: np.ndarray, alpha: float) -> np.ndarray:
    """Step 2: b_g (F, n) by degree-2 quadrature of alpha g psi_i per element."""
    dim = coords.shape[1]
    vol = geometry.element_measures(coords, conn)
    pts, w = geometry.quadrature_rule(dim)
    g_el = g[:, conn]                                   # (F, E, d+1) nodal values per element
    g_q = np.einsum("qk,fek->feq", pts, g_el)           # g at each quadrature point
    # local load: sum_q w_q |T| alpha g(q) psi_k(q)
    loc = alpha * np.einsum("q,e,feq,qk->fek", w, vol, g_q, pts)
    b = np.zeros((g.shape[0], coords.shape[0]))
    for f in range(g.shape[0]):
        np.add.at(b[f], conn.ravel(), loc[f].ravel())
    return b


def query_points(coords, conn, n_samples, seed, stream, elems=None, stratified=False):
    """Step 3: samples of the given elements as (E', N, d) physical points."""
    dim = coords.shape[1]
    lam = sampling.element_samples(dim, conn.shape[0], n_samples, seed, stream, elems, stratified)
    return lam, sampling.physical_points(coords, conn, lam, elems)


def element_loads(coords, conn, g, y, lam, alpha, elems=None):
    """Step 5 for elements ``elems``: beta (F, E', d+1).

    g: (F, n) control at target nodes; y: (F, E', N) source values at the
    samples; lam: (E', N, d+1) barycentric weights of the samples.
    """
    if elems is None:
        elems = np.arange(conn.shape[0])
    vol = geometry.element_measures(coords, conn[elems])
    n_samples = lam.shape[1]
    g_at = np.einsum("tjk,ftk->ftj", lam, g[:, conn[elems]])        # g(X_tj)
    r = y - alpha * g_at                                            # residual f^s - alpha g
    prod = r[..., None] * lam[None, ...]                            # (F, E', N, d+1)
    beta = neumaier_sum(prod, axis=2)                               # sum over j
    return beta * (vol / n_samples)[None, :, None]


ALPHA_ELEMENT_RANGE = (0.0, 2.0)


def element_loads_own_alpha(coords, conn, g, y, lam, elems=None):
    """Step 5 with each element's own control coefficient (reading: sec. 4.1
    leaves alpha free and sec. 5.1 shows the error depends on it; the
    coefficient that minimizes the sample variance of the residual terms
    (f^s - alpha g) psi_k summed over k is the classic control-variate one).

    With A_k = sum_j y_j l_jk, B_k = sum_j g_j l_jk, P = sum_j y_j g_j w_j,
    Q = sum_j g_j^2 w_j and w_j = sum_k l_jk^2 (g_j = g(X_tj)):
        alpha_t = (P/N - sum_k A_k B_k / N^2) / (Q/N - sum_k B_k^2 / N^2),
    clipped to ALPHA_ELEMENT_RANGE (1 when the denominator is not positive);
    then the element load includes its exact control part,
        beta_tk = alpha_t (M_t g_t)_k + |Omega_t| / N (A_k - alpha_t B_k),
    (M_t g_t)_k = |Omega_t| (sum_l g_l + g_k) / ((d+1)(d+2)).
    Returns (beta (F, E', d+1), alpha (F, E')).
    """
    if elems is None:
        elems = np.arange(conn.shape[0])
    dim = coords.shape[1]
    vol = geometry.element_measures(coords, conn[elems])
    N = lam.shape[1]
    gv = g[:, conn[elems]]                                           # (F, E', d+1) nodal control values
    g_at = np.einsum("tjk,ftk->ftj", lam, gv)                        # g(X_tj)
    w = (lam * lam).sum(axis=2)                                      # (E', N)
    A = neumaier_sum(y[..., None] * lam[None], axis=2)               # (F, E', d+1)
    B = neumaier_sum(g_at[..., None] * lam[None], axis=2)
    P = neumaier_sum(y * g_at * w[None], axis=2)                     # (F, E')
    Q = neumaier_sum(g_at * g_at * w[None], axis=2)
    num = P / N - (A * B).sum(axis=2) / N ** 2
    den = Q / N - (B * B).sum(axis=2) / N ** 2
    ok = np.isfinite(num) & np.isfinite(den) & (den > 0)
    alpha = np.where(ok, num / np.where(ok, den, 1.0), 1.0)
    alpha = np.clip(alpha, *ALPHA_ELEMENT_RANGE)
    control = vol[None, :, None] * (gv.sum(axis=2, keepdims=True) + gv) / ((dim + 1) * (dim + 2))
    beta = alpha[..., None] * control + (vol / N)[None, :, None] * (A - alpha[..., None] * B)
    return beta, alpha


def element_variance_terms(coords, conn, r, elems=None):
    """Variance of each element's Monte Carlo total |Omega_t|/N sum_j r_tj
    (the part of sum_k b^t_k the samples estimate; sum_k psi_k = 1), estimated
    from its own residuals: |Omega_t|^2 s_t^2 / N with s_t^2 the unbiased
    sample variance of r_tj over j.  r: (F, E', N).  Returns (F, E'), zeros
    for N < 2.  Summed over the elements (independent samples) it is the
    variance of the estimate of sum_i b_i = integral f^s (App. B,
    Eq. cv_global_integral_estimator; its expectation is the E[E_cons^2] that
    Eq. conservation_residual_bound bounds)."""
    if elems is None:
        elems = np.arange(conn.shape[0])
    vol = geometry.element_measures(coords, conn[elems])
    N = r.shape[2]
    if N < 2:
        return np.zeros(r.shape[:2])
    s2 = r.var(axis=2, ddof=1)
    return (vol ** 2)[None, :] * s2 / N


def samples_for_tolerance(stderr: float, sum_b: float, n_samples: int, rel_tol: float) -> int:
    """Samples per element for which the standard error of sum b, which falls
    as N^-1/2, reaches rel_tol |sum b|: ceil(N (stderr / (rel_tol |sum b|))^2)."""
    target = rel_tol * abs(sum_b)
    if target <= 0.0 or stderr <= 0.0:
        return 1
    return int(min(1 << 20, max(1, math.ceil(n_samples * (stderr / target) ** 2))))


def assemble(conn: np.ndarray, beta: np.ndarray, n_nodes: int) -> np.ndarray:
    """Step 6 (residual part): b_res,v = sum of beta over (element, local vertex) at v."""
    b = np.zeros((beta.shape[0], n_nodes))
    for f in range(beta.shape[0]):
        np.add.at(b[f], conn.ravel(), beta[f].ravel())
    return b


def solve_mass(M: sp.csr_matrix, b: np.ndarray, dim: int) -> np.ndarray:
    """Step 7: x = M^-1 b for each field row of b."""
    n = M.shape[0]
    if n <= (200_000 if dim == 2 else 60_000):
        lu = spla.splu(M.tocsc(), permc_spec="MMD_AT_PLUS_A")
        return np.stack([lu.solve(bf) for bf in b])
    return np.stack([jacobi_cg(M, bf, 1e-15) for bf in b])


def jacobi_cg(M: sp.csr_matrix, b: np.ndarray, rtol: float, max_iter: int = 500) -> np.ndarray:
    """Textbook Jacobi-preconditioned conjugate gradients from x = 0."""
    dinv = 1.0 / M.diagonal()
    x = np.zeros_like(b)
    r = b.copy()
    z = dinv * r
    p = z.copy()
    rz = math.fsum(r * z)
    bn = math.sqrt(math.fsum(b * b))
    for _ in range(max_iter):
        q = M @ p
        a = rz / math.fsum(p * q)
        x += a * p
        r -= a * q
        if math.sqrt(math.fsum(r * r)) <= rtol * bn:
            break
        z = dinv * r
        rz_new = math.fsum(r * z)
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x


def transfer(coords, conn, query, n_samples, alpha=1.0, seed=0, stream=0, chunk_elems=20_000, stratified=False,
             own_alpha=False):
    """Whole CV-MC transfer of a black-box ``query`` (points (n, d) -> values (F, n)).

    own_alpha: each element's own control coefficient (element_loads_own_alpha);
    the control part is then inside the element loads and b_g is zero.
    Returns a dict with g, b_g, b_res, b, x, the mass matrix, lumped mass, the
    conservation report (with sum_b_stderr: the standard error of sum b from
    the element variance terms, -1 for N = 1) and var_terms (F, E).
    """
    coords = np.asarray(coords, dtype=np.float64)
    conn = np.asarray(conn, dtype=np.int64)
    dim = coords.shape[1]
    n, E = coords.shape[0], conn.shape[0]
    g = np.atleast_2d(query(coords))                                 # step 1
    F = g.shape[0]
    b_g = control_load(coords, conn, g, 0.0 if own_alpha else alpha)   # step 2
    beta = np.empty((F, E, dim + 1))
    var_terms = np.empty((F, E))
    alphas = np.empty((F, E)) if own_alpha else None
    for s in range(0, E, chunk_elems):
        el = np.arange(s, min(E, s + chunk_elems))
        lam, X = query_points(coords, conn, n_samples, seed, stream, el, stratified)   # step 3
        y = np.atleast_2d(query(X.reshape(-1, dim))).reshape(F, el.size, n_samples)  # step 4
        if own_alpha:                                                                  # step 5
            beta[:, el], alphas[:, el] = element_loads_own_alpha(coords, conn, g, y, lam, el)
            a_el = alphas[:, el][..., None]
        else:
            beta[:, el] = element_loads(coords, conn, g, y, lam, alpha, el)
            a_el = alpha
        g_at = np.einsum("tjk,ftk->ftj", lam, g[:, conn[el]])
        var_terms[:, el] = element_variance_terms(coords, conn, y - a_el * g_at, el)
    b_res = assemble(conn, beta, n)                                  # step 6
    b = b_g + b_res
    M = geometry.mass_matrix(coords, conn)
    x = solve_mass(M, b, dim)                                        # step 7
    m = geometry.lumped_mass(coords, conn)
    report = conservation_report(b, x, m)
    for f, rep in enumerate(report):
        # no spread to estimate from a single sample per element
        rep["sum_b_stderr"] = math.sqrt(math.fsum(var_terms[f])) if n_samples >= 2 else -1.0
    return {
        "g": g, "b_g": b_g, "beta": beta, "b_res": b_res, "b": b, "x": x,
        "M": M, "m": m, "report": report, "alpha_elements": alphas, "var_terms": var_terms,
    }


def conservation_report(b: np.ndarray, x: np.ndarray, m: np.ndarray):
    """Sum of the load vector, integral m^T x of the solution, and their relative defect."""
    out = []
    for bf, xf in zip(np.atleast_2d(b), np.atleast_2d(x)):
        sb = math.fsum(bf)
        sx = math.fsum(m * xf)
        out.append({"sum_b": sb, "int_x": sx, "cons_defect": abs(sx - sb) / max(abs(sb), 1e-300)})
    return out


def rel_l2(a: np.ndarray, ref: np.ndarray) -> float:
    """Relative discrete l2 error ||a - ref|| / ||ref|| (the DoF metric of sec. 5.2)."""
    return float(np.linalg.norm(np.ravel(a) - np.ravel(ref)) / np.linalg.norm(np.ravel(ref)))
