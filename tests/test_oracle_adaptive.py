"""Pins of the oracle's variance-driven samples per element (oracle/adaptive.py).

The allocation is checked against what defines it (counts proportional to
|Omega_t| sigma_t before rounding, the clamps, the total, optimality by brute
force over every integer allocation of a small budget, the closed form of the
predicted variance); the transfer with per-element counts against the
fixed-N transfers it must reduce to, against the exact load vector
(unbiasedness with very uneven counts) and, over realizations, against its
own predicted standard error and the spread of uniform sampling at the same
total.
"""
import itertools
import math

import numpy as np
import pytest

from oracle import adaptive, cvmc, p2, sampling, supermesh
from oracle.source import P1Source
from workloads import fields, meshes


def _objective(a, counts):
    return float(np.sum(a * a / counts))


def test_counts_proportional_to_weights_and_clamped():
    rng = np.random.default_rng(1)
    v = rng.gamma(0.5, 1e-6, 400)
    n0, B = 8, 400 * 48
    c = adaptive.allocate(v, n0, B, 1, 1 << 20)
    a = np.sqrt(n0 * v)
    ideal = B * a / a.sum()
    big = ideal >= 0.5
    assert np.abs(c - ideal)[big].max() <= 0.5 + 1e-9     # nearest integer of the proportional count
    assert np.all(c[~big] == 1)                            # else the smallest count
    assert abs(int(c.sum()) - B) <= 400 // 2
    lo, hi = 6, 90
    cc = adaptive.allocate(v, n0, B, lo, hi)
    assert cc.min() >= lo and cc.max() <= hi
    inside = (ideal > lo + 0.5) & (ideal < hi - 0.5)
    assert np.array_equal(cc[inside], c[inside])
    assert np.all(cc[ideal >= hi] == hi) and np.all(cc[ideal < lo] == lo)
    # equal weights: equal counts; no weight at all (or only non-finite terms): n_min
    assert np.all(adaptive.allocate(np.full(10, 3e-5), 16, 640, 1, 1000) == 64)
    assert np.all(adaptive.allocate(np.zeros(10), 16, 640, 3, 1000) == 3)
    w = np.array([1e-4, np.nan, np.inf, -1.0, 1e-4])
    assert list(adaptive.allocate(w, 4, 100, 2, 1000)) == [50, 2, 2, 2, 50]


def test_allocation_is_optimal_by_brute_force():
    """For a tiny budget no integer allocation with the same total has a smaller
    sum a_t^2 / N_t than the Neyman counts (when they add up to the budget),
    and the continuous optimum (sum a_t)^2 / B is a lower bound on all of them.
    Counts proportional to a_t^2 (the variance) or uniform are clearly worse."""
    rng = np.random.default_rng(2)
    hits = 0
    for _ in range(40):
        a = rng.gamma(1.0, 1.0, 4)
        v = a * a / 4.0                                   # a pilot with n0 = 4
        B = int(rng.integers(12, 30))
        c = adaptive.allocate(v, 4, B, 1, B)
        best = min(_objective(a, np.array(k)) for k in itertools.product(range(1, B), repeat=4) if sum(k) == B)
        assert (a.sum() ** 2) / B <= best * (1 + 1e-12)
        if c.sum() == B:
            hits += 1
            assert _objective(a, c) <= best * 1.02
    assert hits >= 20
    a = np.array([4.0, 1.0, 1.0, 0.25])
    v = a * a / 4.0
    neyman = _objective(a, adaptive.allocate(v, 4, 64, 1, 64))
    var_prop = np.maximum(1, np.round(64 * a * a / np.sum(a * a)))
    assert neyman < 0.9 * _objective(a, var_prop)
    assert neyman < 0.75 * _objective(a, np.full(4, 16.0))


def test_prediction_closed_form_and_budget():
    """Counts exactly proportional to a_t give the predicted standard error
    W / sqrt(B); the budget for a tolerance meets it and one sample less does not."""
    a = np.array([1.0, 2.0, 3.0, 6.0])
    n0 = 16
    v = a * a / n0
    c = adaptive.allocate(v, n0, 1200, 1, 10_000)
    assert list(c) == [100, 200, 300, 600]
    W, se = adaptive.allocation_summary(v, n0, c)
    assert W == 12.0 and abs(se - 12.0 / math.sqrt(1200)) < 1e-15
    B = adaptive.budget_for_tolerance(W, 50.0, 1e-3)
    assert W / math.sqrt(B) <= 1e-3 * 50.0 < W / math.sqrt(B - 1)
    assert adaptive.budget_for_tolerance(0.0, 1.0, 1e-3) == 1


@pytest.mark.parametrize("dim", [2, 3])
def test_sample_j_of_element_t_does_not_depend_on_its_count(dim):
    """Element t's samples in a list with per-element counts are the first N_t
    samples of the list with a fixed N (Philox counter (j, t)), in element order."""
    m = meshes.delaunay_tri_mesh(5, 0.3, 3) if dim == 2 else meshes.kuhn_tet_mesh(2, 0.08, 3)
    E = m[1].shape[0]
    counts = np.random.default_rng(4).integers(1, 20, E)
    X, L = adaptive.query_points(*m, counts, 77, 5)
    lam = sampling.element_samples(dim, E, 20, 77, 5)
    _, Xf = cvmc.query_points(*m, 20, 77, 5)
    off = adaptive.offsets(counts)
    assert off[-1] == X.shape[0] == counts.sum()
    for t in range(E):
        np.testing.assert_array_equal(L[off[t]:off[t + 1]], lam[t, : counts[t]])
        np.testing.assert_array_equal(X[off[t]:off[t + 1]], Xf[t, : counts[t]])


def _pair(kind):
    if kind == "tri":
        return meshes.delaunay_tri_mesh(8, 0.3, 21), meshes.delaunay_tri_mesh(12, 0.3, 22)
    return meshes.kuhn_tet_mesh(3, 0.08, 23), meshes.kuhn_tet_mesh(4, 0.08, 24)


@pytest.mark.parametrize("kind,own", [("tri", False), ("tri", True), ("tet", False)])
def test_uniform_counts_reproduce_fixed_n(kind, own):
    tm, sm = _pair(kind)
    sv = fields.evaluate("front_2d" if kind == "tri" else "gaussian_bumps_3d", np, sm[0])
    src = P1Source(*sm, sv)
    ref = cvmc.transfer(*tm, src, 12, alpha=0.75, seed=5, stream=2, own_alpha=own)
    got = adaptive.transfer(*tm, src, np.full(tm[1].shape[0], 12), alpha=0.75, seed=5, stream=2, own_alpha=own)
    np.testing.assert_allclose(got["b"], ref["b"], rtol=0, atol=1e-15 * np.abs(ref["b"]).max())
    np.testing.assert_allclose(got["x"], ref["x"], rtol=0, atol=1e-13 * np.abs(ref["x"]).max())
    assert abs(got["report"][0]["sum_b_stderr"] - ref["report"][0]["sum_b_stderr"]) < 1e-15


def test_uniform_counts_reproduce_fixed_n_p2():
    c2, t2 = meshes.p2_mesh(*meshes.delaunay_tri_mesh(6, 0.3, 25))
    sm = meshes.delaunay_tri_mesh(9, 0.3, 26)
    src = P1Source(*sm, fields.evaluate("paper_f2", np, sm[0]))
    ref = p2.transfer(c2, t2, src, 9, alpha=0.5, seed=8, stream=1)
    got = adaptive.transfer(c2, t2, src, np.full(t2.shape[0], 9), alpha=0.5, seed=8, stream=1)
    np.testing.assert_allclose(got["b"], ref["b"], rtol=0, atol=1e-15 * np.abs(ref["b"]).max())
    assert abs(got["report"][0]["sum_b_stderr"] - ref["report"][0]["sum_b_stderr"]) < 1e-15


def test_single_sample_elements_leave_stderr_undefined_and_constants_conserved():
    tm, sm = _pair("tri")
    E = tm[1].shape[0]
    counts = np.random.default_rng(6).integers(1, 5, E)
    counts[0] = 1
    vol = cvmc.geometry.element_measures(*tm).sum()
    r = adaptive.transfer(*tm, lambda x: np.full((1, len(x)), 2.5), counts, alpha=0.3, seed=1)
    assert r["report"][0]["sum_b_stderr"] == -1.0
    assert abs(r["report"][0]["sum_b"] - 2.5 * vol) < 1e-13
    assert r["report"][0]["cons_defect"] < 1e-12


@pytest.fixture(scope="module")
def front_case():
    tm, sm = meshes.delaunay_tri_mesh(7, 0.3, 31), meshes.delaunay_tri_mesh(11, 0.3, 32)
    sv = fields.evaluate("front_2d", np, sm[0])
    src = P1Source(*sm, sv)
    pieces = supermesh.intersections(*tm, *sm)
    exact = supermesh.supermesh_projection(*tm, *sm, sv, pieces=pieces)["b"][0]
    return tm, src, exact


def test_unbiased_with_uneven_counts(front_case):
    """E[b] is the exact load vector whatever the counts: 300 realizations with
    counts from 2 to 40 (alpha = 1/2), z-scores at every node."""
    tm, src, exact = front_case
    counts = np.random.default_rng(7).integers(2, 41, tm[1].shape[0])
    R = 300
    bs = np.array([adaptive.transfer(*tm, src, counts, alpha=0.5, seed=900, stream=s)["b"][0] for s in range(R)])
    z = (bs.mean(axis=0) - exact) / (bs.std(axis=0, ddof=1) / math.sqrt(R))
    assert np.abs(z).max() < 4.5
    assert 0.6 < np.mean(z ** 2) < 1.5


def test_neyman_counts_beat_uniform_and_meet_their_prediction(front_case):
    """A pilot (N0 = 8, its own stream) sets the counts for a total of 16 per
    element; over 250 later realizations the spread of sum b is that of the
    prediction and below the spread of 16 uniform samples per element."""
    tm, src, exact = front_case
    E = tm[1].shape[0]
    pilot = cvmc.transfer(*tm, src, 8, alpha=0.5, seed=11, stream=10_000)
    counts = adaptive.allocate(pilot["var_terms"][0], 8, 16 * E, 2, 1 << 20)
    _, pred = adaptive.allocation_summary(pilot["var_terms"][0], 8, counts)
    R = 250
    ad = np.array([adaptive.transfer(*tm, src, counts, alpha=0.5, seed=12, stream=s)["report"][0]["sum_b"]
                   for s in range(R)])
    un = np.array([cvmc.transfer(*tm, src, 16, alpha=0.5, seed=12, stream=s)["report"][0]["sum_b"]
                   for s in range(R)])
    sa, su = ad.std(ddof=1), un.std(ddof=1)
    assert sa < 0.85 * su
    assert 0.75 < sa / pred < 1.3
    assert abs(ad.mean() - exact.sum()) < 4.0 * sa / math.sqrt(R)
