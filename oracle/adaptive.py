"""Variance-driven samples per element (oracle side, test infrastructure).

App. B: with N_t independent samples in target element t the estimate of
sum b has variance sum_t |Omega_t|^2 sigma_t^2 / N_t (Eq.
cv_global_integral_estimator), sigma_t^2 the variance of the residual
f^s - alpha g over the element, and its square root bounds the conservation
error (Eq. conservation_residual_bound).  Sec. 7 names better sampling as the
way to improve the method.  For a total of B samples the variance is smallest
with N_t proportional to a_t = |Omega_t| sigma_t (Neyman allocation: minimize
sum a_t^2 / N_t subject to sum N_t = B), and is then (sum a_t)^2 / B.

A pilot transfer with N0 samples per element estimates a_t from its own
element variance terms v_t = |Omega_t|^2 s_t^2 / N0 as sqrt(N0 v_t) (a term
that is not finite, or negative, counts as 0).

allocate()              N_t = clamp(floor(B a_t / W + 1/2), n_min, n_max), W = sum a_t
allocation_summary()    W and the predicted standard error sqrt(sum a_t^2 / N_t)
budget_for_tolerance()  the B whose prediction W / sqrt(B) reaches rel_tol |sum b|
transfer()              the CV-MC transfer with N_t samples in element t: the
                        steps of cvmc.transfer (P1 targets, fixed alpha or each
                        element's own) or p2.transfer (P2 targets), element by
                        element with its own N_t; sample j of element t is drawn
                        from Philox counter (j, t) as with a fixed N, and the
                        query list holds element t's samples at n + offs[t] + j,
                        offs the exclusive prefix sums of the counts.

Parity: the allocation is pinned by its defining properties (the counts
before rounding are proportional to the weights and add up to the budget,
the clamps, equal weights giving equal counts), by brute force over all
integer allocations of a tiny budget (no allocation with the same total has
a smaller sum a_t^2 / N_t than the one rounded from the proportional one,
beyond rounding), and by the closed form (sum a_t)^2 / B of the prediction;
the transfer by the uniform case (N_t = N reproduces cvmc.transfer and
p2.transfer), unbiasedness of sum b and b against the exact load with very
uneven counts, and a smaller spread of sum b than uniform sampling at the
same total over realizations.
"""
from __future__ import annotations

import math

import numpy as np

from . import cvmc, geometry, p2


def weights(var_terms: np.ndarray, n0: int) -> np.ndarray:
    """a_t = sqrt(n0 v_t), 0 where n0 v_t is not finite and positive."""
    x = n0 * np.asarray(var_terms, dtype=np.float64)
    ok = np.isfinite(x) & (x > 0.0)
    return np.where(ok, np.sqrt(np.where(ok, x, 0.0)), 0.0)


def allocate(var_terms: np.ndarray, n0: int, budget: int, n_min: int, n_max: int) -> np.ndarray:
    """Counts N_t (int64) from one field's variance terms (E,) of a pilot with n0 samples per element."""
    a = weights(var_terms, n0)
    W = math.fsum(a)
    if W <= 0.0:
        return np.full(a.shape, n_min, dtype=np.int64)
    n = np.floor(float(budget) * a / W + 0.5)
    return np.clip(n, n_min, n_max).astype(np.int64)


def allocation_summary(var_terms: np.ndarray, n0: int, counts: np.ndarray):
    """(W, predicted standard error sqrt(sum a_t^2 / N_t)) of an allocation."""
    a = weights(var_terms, n0)
    return math.fsum(a), math.sqrt(math.fsum(a * a / np.asarray(counts, dtype=np.float64)))


def budget_for_tolerance(weight_sum: float, sum_b: float, rel_tol: float) -> int:
    target = rel_tol * abs(sum_b)
    if weight_sum == 0.0 or target <= 0.0:
        return 1
    return int(min(2 ** 40, max(1, math.ceil((weight_sum / target) ** 2))))


def offsets(counts: np.ndarray) -> np.ndarray:
    """(E+1,) exclusive prefix sums: element t's samples at positions offs[t] .. offs[t+1]-1."""
    return np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)


def query_points(coords, conn, counts, seed, stream):
    """The list's samples in order: (sum N_t, d) points and (sum N_t, d+1) barycentric weights."""
    coords = np.asarray(coords, dtype=np.float64)
    conn = np.asarray(conn, dtype=np.int64)
    counts = np.asarray(counts, dtype=np.int64)
    dim = coords.shape[1]
    off = offsets(counts)
    L = np.empty((off[-1], dim + 1))
    P = np.empty((off[-1], dim))
    for N in np.unique(counts):
        el = np.nonzero(counts == N)[0]
        lam, X = cvmc.query_points(coords, conn[:, : dim + 1], int(N), seed, stream, el)
        idx = (off[el][:, None] + np.arange(int(N))[None, :]).ravel()
        L[idx] = lam.reshape(-1, dim + 1)
        P[idx] = X.reshape(-1, dim)
    return P, L


def transfer(coords, conn, query, counts, alpha=1.0, seed=0, stream=0, own_alpha=False):
    """CV-MC transfer with counts[t] samples in element t.  conn (E, d+1) for P1
    targets, (E, (d+1)(d+2)/2) for P2 (vertices, then edge nodes)."""
    coords = np.asarray(coords, dtype=np.float64)
    conn = np.asarray(conn, dtype=np.int64)
    counts = np.asarray(counts, dtype=np.int64)
    dim = coords.shape[1]
    n, E = coords.shape[0], conn.shape[0]
    order = 1 if conn.shape[1] == dim + 1 else 2
    if order == 2 and own_alpha:
        raise ValueError("each element's own alpha: P1 targets")
    vconn = conn[:, : dim + 1]
    nb = conn.shape[1]
    g = np.atleast_2d(query(coords))                                       # step 1
    F = g.shape[0]
    if order == 1:
        M = geometry.mass_matrix(coords, conn)
        b_g = cvmc.control_load(coords, conn, g, 0.0 if own_alpha else alpha)   # step 2
        m = geometry.lumped_mass(coords, conn)
    else:
        M = p2.mass_matrix(coords, conn)
        b_g = alpha * np.stack([M @ gf for gf in g])
        m = np.asarray(M.sum(axis=1)).ravel()
    beta = np.empty((F, E, nb))
    var_terms = np.zeros((F, E))
    for N in np.unique(counts):                                            # steps 3-5, per count
        el = np.nonzero(counts == N)[0]
        lam, X = cvmc.query_points(coords, vconn, int(N), seed, stream, el)
        y = np.atleast_2d(query(X.reshape(-1, dim))).reshape(F, el.size, int(N))
        if order == 2:
            beta[:, el], r = p2.element_loads(coords, conn, g, y, lam, alpha, el)
        elif own_alpha:
            beta[:, el], a_el = cvmc.element_loads_own_alpha(coords, conn, g, y, lam, el)
            r = y - a_el[..., None] * np.einsum("tjk,ftk->ftj", lam, g[:, conn[el]])
        else:
            beta[:, el] = cvmc.element_loads(coords, conn, g, y, lam, alpha, el)
            r = y - alpha * np.einsum("tjk,ftk->ftj", lam, g[:, conn[el]])
        var_terms[:, el] = cvmc.element_variance_terms(coords, vconn, r, el)
    b = b_g + cvmc.assemble(conn, beta, n)                                 # step 6
    x = cvmc.solve_mass(M, b, dim)                                         # step 7
    report = cvmc.conservation_report(b, x, m)
    for f, rep in enumerate(report):
        # one sample in some element: its variance, and so the sum's, cannot be estimated
        rep["sum_b_stderr"] = math.sqrt(math.fsum(var_terms[f])) if counts.min() >= 2 else -1.0
    return {"g": g, "b": b, "x": x, "beta": beta, "report": report, "var_terms": var_terms,
            "offsets": offsets(counts)}
