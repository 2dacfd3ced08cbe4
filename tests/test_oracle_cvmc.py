"""Pins of the oracle's control-variate Monte Carlo transfer and supermesh projection.

Each test checks the oracle against a fact fixed by the paper or by the
mathematics (special cases, identities, unbiasedness, convergence rates), so
that a dropped term, a wrong sign, a wrong vertex index or a transposed
operand anywhere in the pipeline fails at least one of them.
"""
import math

import numpy as np
import pytest

from oracle import cvmc, geometry, supermesh
from oracle.source import P1Source
from workloads import fields, meshes


def _pair(kind="2d", seeds=(1, 2)):
    if kind == "2d":
        return meshes.delaunay_tri_mesh(9, 0.3, seeds[0]), meshes.delaunay_tri_mesh(13, 0.3, seeds[1])
    return meshes.kuhn_tet_mesh(4, 0.08, seeds[0]), meshes.kuhn_tet_mesh(6, 0.08, seeds[1])


def _source(smesh, name):
    sc, sconn = smesh
    return P1Source(sc, sconn, fields.evaluate(name, np, sc))


# ---- building blocks ---------------------------------------------------------------------
def test_neumaier_sum_matches_fsum():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((300, 7)) * 10.0 ** rng.integers(-8, 8, (300, 7))
    s = cvmc.neumaier_sum(x, axis=0)
    ref = np.array([math.fsum(x[:, c]) for c in range(7)])
    assert np.array_equal(s, ref) or np.abs(s - ref).max() <= 1e-16 * np.abs(x).sum(axis=0).max()


@pytest.mark.parametrize("kind", ["2d", "3d"])
def test_control_load_is_alpha_M_g(kind):
    (tc, tconn), _ = _pair(kind)
    rng = np.random.default_rng(3)
    g = rng.standard_normal((2, tc.shape[0]))
    M = geometry.mass_matrix(tc, tconn)
    for alpha in (1.0, 0.3):
        bg = cvmc.control_load(tc, tconn, g, alpha)
        ref = alpha * (M @ g.T).T
        assert np.abs(bg - ref).max() <= 1e-15 * np.abs(ref).max() * 10


def test_assembly_scatters_to_connectivity():
    conn = np.array([[0, 1, 2], [2, 1, 3]])
    beta = np.arange(6, dtype=float).reshape(1, 2, 3) + 1.0
    b = cvmc.assemble(conn, beta, 4)
    assert b.tolist() == [[1.0, 2.0 + 5.0, 3.0 + 4.0, 6.0]]


def test_jacobi_cg_matches_direct():
    (tc, tconn), _ = _pair("3d")
    M = geometry.mass_matrix(tc, tconn)
    b = np.random.default_rng(1).standard_normal(tc.shape[0])
    x1 = cvmc.jacobi_cg(M, b, 1e-15)
    x2 = cvmc.solve_mass(M, b[None], 3)[0]
    assert cvmc.rel_l2(x1, x2) < 1e-13


# ---- special cases of the whole pipeline ----------------------------------------------
@pytest.mark.parametrize("kind", ["2d", "3d"])
@pytest.mark.parametrize("N", [1, 7, 64])
def test_affine_source_reproduced_with_alpha_one(kind, N):
    """f^s affine lies in V_t, g = f^s, the residual vanishes: x = f at the nodes."""
    tmesh, smesh = _pair(kind)
    src = _source(smesh, "affine")
    r = cvmc.transfer(*tmesh, src, N, alpha=1.0, seed=17, stream=2)
    assert cvmc.rel_l2(r["x"], fields.evaluate("affine", np, tmesh[0])) < 1e-13
    assert np.abs(r["b_res"]).max() < 1e-15


@pytest.mark.parametrize("alpha", [0.0, 0.4, 1.0])
def test_constant_source_conserved_for_any_alpha(alpha):
    """sum_k lambda_k = 1 makes sum(b) = c |domain| exactly, for any samples and alpha."""
    tmesh, smesh = _pair("2d")
    src = _source(smesh, "constant")
    r = cvmc.transfer(*tmesh, src, 5, alpha=alpha, seed=4, stream=0)
    assert abs(r["report"][0]["sum_b"] - 2.5) < 1e-13
    assert abs(r["report"][0]["int_x"] - 2.5) < 1e-13
    if alpha == 1.0:
        # the residual is identically zero, so the nodal values are exact too
        assert cvmc.rel_l2(r["x"], np.full(tmesh[0].shape[0], 2.5)) < 1e-12


@pytest.mark.parametrize("kind", ["2d", "3d"])
def test_identical_meshes_reproduce_nodal_field(kind):
    """Source mesh == target mesh, alpha = 1: f^s = g on every element, so x = F."""
    tmesh, _ = _pair(kind)
    name = "smooth_2d" if kind == "2d" else "gaussian_bumps_3d"
    src = _source(tmesh, name)
    r = cvmc.transfer(*tmesh, src, 9, alpha=1.0, seed=8, stream=1)
    assert cvmc.rel_l2(r["x"], src.values) < 1e-12


@pytest.mark.parametrize("alpha", [0.0, 1.0])
def test_discrete_conservation_identity(alpha):
    """Testing the Galerkin system with the constant function: m^T x = sum(b)."""
    tmesh, smesh = _pair("2d")
    r = cvmc.transfer(*tmesh, _source(smesh, "front_2d"), 11, alpha=alpha, seed=2, stream=0)
    assert r["report"][0]["cons_defect"] < 1e-13


# ---- supermesh (exact b) -----------------------------------------------------------------
@pytest.fixture(scope="module")
def sm_case():
    tmesh, smesh = _pair("2d")
    pieces = supermesh.intersections(*tmesh, *smesh)
    return tmesh, smesh, pieces


def test_supermesh_partition_identity(sm_case):
    tmesh, smesh, pieces = sm_case
    sv = fields.evaluate("smooth_2d", np, smesh[0])
    sm = supermesh.supermesh_projection(*tmesh, *smesh, sv, pieces=pieces)
    vol = geometry.element_measures(*tmesh)
    assert np.abs(sm["area_sum"] - vol).max() < 1e-16 * 20
    src = P1Source(*smesh, sv)
    assert abs(sm["b"].sum() - src.integral()[0]) < 1e-14
    assert abs(sm["int_fs"][0] - src.integral()[0]) < 1e-14


def test_supermesh_affine_source_gives_M_f(sm_case):
    """An affine f^s lies in V_t, so the exact load vector is M f(nodes) on any mesh pair."""
    tmesh, smesh, pieces = sm_case
    sv = fields.evaluate("affine", np, smesh[0])
    sm = supermesh.supermesh_projection(*tmesh, *smesh, sv, x_target=fields.evaluate("affine", np, tmesh[0]),
                                        pieces=pieces)
    M = geometry.mass_matrix(*tmesh)
    ref = M @ fields.evaluate("affine", np, tmesh[0])[0]
    assert np.abs(sm["b"][0] - ref).max() < 1e-15
    assert sm["E_L2"][0] < 1e-7        # sqrt of a rounding-level integral


def test_supermesh_identical_meshes_gives_MF():
    tmesh, _ = _pair("2d")
    sv = fields.evaluate("front_2d", np, tmesh[0])
    sm = supermesh.supermesh_projection(*tmesh, *tmesh, sv)
    ref = geometry.mass_matrix(*tmesh) @ sv[0]
    assert np.abs(sm["b"][0] - ref).max() < 1e-15


# ---- statistics: unbiasedness and N^-1/2 -------------------------------------------------
@pytest.mark.parametrize("alpha", [0.0, 0.5, 1.0])
def test_estimator_unbiased_against_supermesh(sm_case, alpha):
    """E[b_hat] = b: replicate means sit within sampling error of the exact b."""
    tmesh, smesh, pieces = sm_case
    sv = fields.evaluate("front_2d", np, smesh[0])
    exact = supermesh.supermesh_projection(*tmesh, *smesh, sv, pieces=pieces)["b"][0]
    src = P1Source(*smesh, sv)
    R = 300
    bs = np.array([cvmc.transfer(*tmesh, src, 6, alpha=alpha, seed=1000 + s, stream=3)["b"][0]
                   for s in range(R)])
    z = (bs.mean(axis=0) - exact) / (bs.std(axis=0, ddof=1) / math.sqrt(R))
    assert np.abs(z).max() < 4.5
    assert 0.6 < np.mean(z ** 2) < 1.5


def test_error_decays_as_inverse_sqrt_N(sm_case):
    tmesh, smesh, pieces = sm_case
    sv = fields.evaluate("front_2d", np, smesh[0])
    exact = supermesh.supermesh_projection(*tmesh, *smesh, sv, pieces=pieces)["b"][0]
    src = P1Source(*smesh, sv)
    Ns = [4, 16, 64, 256]
    rms = []
    for N in Ns:
        errs = [cvmc.transfer(*tmesh, src, N, alpha=0.5, seed=50 + s, stream=N)["b"][0] - exact
                for s in range(24)]
        rms.append(np.sqrt(np.mean(np.square(errs))))
    slope = np.polyfit(np.log(Ns), np.log(rms), 1)[0]
    assert abs(slope + 0.5) < 0.08


def test_error_decreases_as_alpha_goes_to_one(sm_case):
    tmesh, smesh, pieces = sm_case
    sv = fields.evaluate("paper_f3", np, smesh[0])
    exact = supermesh.supermesh_projection(*tmesh, *smesh, sv, pieces=pieces)["b"][0]
    src = P1Source(*smesh, sv)
    rms = []
    for alpha in (0.0, 0.5, 0.75, 1.0):
        errs = [cvmc.transfer(*tmesh, src, 20, alpha=alpha, seed=7 + s, stream=0)["b"][0] - exact
                for s in range(16)]
        rms.append(np.sqrt(np.mean(np.square(errs))))
    assert all(a > b for a, b in zip(rms, rms[1:]))
    assert rms[-1] < 0.1 * rms[0]


def test_h_convergence_rates():
    """alpha = 1, N = 20: E_L2 ~ h^2 and the RMS conservation error ~ h^3 (2D, P1)."""
    res = []
    for kt, ks in [(9, 13), (17, 25), (33, 49)]:
        tc, tconn = meshes.structured_tri_mesh(kt, 0.2, 21)
        sc, sconn = meshes.delaunay_tri_mesh(ks, 0.3, 22)
        sv = fields.evaluate("paper_f2", np, sc)
        src = P1Source(sc, sconn, sv)
        pieces = supermesh.intersections(tc, tconn, sc, sconn)
        el2, em = [], []
        for s in range(6):
            r = cvmc.transfer(tc, tconn, src, 20, 1.0, seed=s, stream=0)
            sm = supermesh.supermesh_projection(tc, tconn, sc, sconn, sv, r["x"], pieces=pieces)
            el2.append(sm["E_L2"][0])
            em.append(sm["E_mass"][0])
        res.append((1.0 / (kt - 1), np.mean(el2), np.sqrt(np.mean(np.square(em)))))
    res = np.array(res)
    s_l2 = np.polyfit(np.log(res[:, 0]), np.log(res[:, 1]), 1)[0]
    s_m = np.polyfit(np.log(res[:, 0]), np.log(res[:, 2]), 1)[0]
    assert 1.8 < s_l2 < 2.2
    assert 2.6 < s_m < 3.4


# ---- stratified sampling ---------------------------------------------------------------
@pytest.mark.parametrize("dim,N", [(2, 64), (2, 50), (3, 64), (3, 100), (4, 81), (5, 40), (6, 64)])
def test_stratified_samples_fill_every_cell_once(dim, N):
    """Each element's first m^d' samples put their uniforms one in each cell of
    the m^d' grid (m = floor(N^(1/d'))), the rest stay plain; the placed value
    is (cell + u) / m to the last bit or two."""
    from oracle import sampling

    dp = dim
    m = sampling.strata_per_axis(dim, N)
    assert m ** dp <= N < (m + 1) ** dp
    E = 40
    t = np.repeat(np.arange(E), N)
    j = np.tile(np.arange(N), E)
    u = sampling.uniforms(dim, t, j, 99, 2)
    v = sampling.stratify(dim, u, j, N)
    S = m ** dp
    strat = j < S
    assert np.array_equal(v[~strat], u[~strat])
    cells = np.stack([(j // m ** i) % m for i in range(dp)], axis=1)
    exact = (cells + u) / m
    assert np.abs(v[strat] - exact[strat]).max() <= 2 ** -51
    assert (v > 0).all() and (v < 1).all()
    # away from cell boundaries, floor(v m) recovers the cell; per element every cell once
    inner = np.abs(v * m - np.round(v * m)) > 1e-9
    rec = np.floor(v * m).astype(np.int64)
    ok = strat[:, None] & inner
    assert np.array_equal(rec[ok], cells[:, :][ok])
    key = (cells * (m ** np.arange(dp))).sum(axis=1)
    for e in range(E):
        sel = strat & (t == e)
        assert np.array_equal(np.sort(key[sel]), np.arange(S))


@pytest.mark.parametrize("dim", [2, 3])
def test_stratified_simplex_moments(dim):
    """Uniform on the simplex still: E[l_k] = 1/(d+1), E[l_k l_l] = (1 + delta_kl)/((d+1)(d+2))."""
    from oracle import sampling

    lam = sampling.element_samples(dim, 3000, 64, seed=321, stream=1, stratified=True).reshape(-1, dim + 1)
    d1 = dim + 1
    assert np.abs(lam.sum(axis=1) - 1.0).max() < 4e-16
    n = lam.shape[0]
    assert np.abs(lam.mean(axis=0) - 1.0 / d1).max() < 5 * lam.std(axis=0).max() / math.sqrt(n)
    second = lam.T @ lam / n
    expect = (np.ones((d1, d1)) + np.eye(d1)) / (d1 * (dim + 2))
    sd = np.sqrt(((lam[:, :, None] * lam[:, None, :]) ** 2).mean(axis=0) / n)
    assert np.all(np.abs(second - expect) < 6 * sd)


def test_stratified_estimator_unbiased_and_smaller_variance(sm_case):
    """Stratified samples keep E[b_hat] = b (replicate means within sampling
    error of the exact b) and, for a smooth field, cut the RMS error well
    below plain sampling with the same N; their error falls faster than
    N^-1/2 (about N^-1 for two stratified uniforms)."""
    tmesh, smesh, pieces = sm_case
    sv = fields.evaluate("paper_f2", np, smesh[0])
    exact = supermesh.supermesh_projection(*tmesh, *smesh, sv, pieces=pieces)["b"][0]
    src = P1Source(*smesh, sv)
    R = 120
    bs = np.array([cvmc.transfer(*tmesh, src, 16, alpha=0.5, seed=2000 + s, stream=1, stratified=True)["b"][0]
                   for s in range(R)])
    z = (bs.mean(axis=0) - exact) / (bs.std(axis=0, ddof=1) / math.sqrt(R))
    assert np.abs(z).max() < 4.5
    assert 0.5 < np.mean(z ** 2) < 1.6
    rms = {}
    for strat in (False, True):
        for N in (16, 64, 256):
            errs = [cvmc.transfer(*tmesh, src, N, alpha=0.5, seed=70 + s, stream=N, stratified=strat)["b"][0] - exact
                    for s in range(12)]
            rms[strat, N] = np.sqrt(np.mean(np.square(errs)))
    for N in (16, 64, 256):
        assert rms[True, N] < 0.7 * rms[False, N]
    slope = np.polyfit(np.log([16, 64, 256]), np.log([rms[True, N] for N in (16, 64, 256)]), 1)[0]
    assert slope < -0.8


# ---- each element's own control coefficient ---------------------------------------------
def _dirichlet_moment(a):
    """E[prod l_k^a_k] for the uniform distribution on the triangle: 2! prod a_k! / (2 + sum a)!."""
    return 2 * math.prod(math.factorial(x) for x in a) / math.factorial(2 + sum(a))


def test_own_alpha_estimates_closed_form_coefficient():
    """One reference triangle, f = x^2 (x = l_1), so g = l_1 and y = l_1^2.  The
    variance-minimizing coefficient sum_k Cov(y l_k, g l_k) / sum_k Var(g l_k)
    follows from the Dirichlet moments; the estimate from N = 200000 samples
    must agree to within its sampling error."""
    from oracle import sampling

    e = lambda *a: _dirichlet_moment(a)   # noqa: E731
    unit = [(1, 0, 0), (0, 1, 0), (0, 0, 1)]
    # E[y g l_k^2] summed over k, y g = l_1^3
    num = sum(e(*(u0 + 2 * uk for u0, uk in zip((0, 3, 0), u))) for u in unit)
    num -= sum(e(*(u0 + uk for u0, uk in zip((0, 2, 0), u))) * e(*(u0 + uk for u0, uk in zip((0, 1, 0), u)))
               for u in unit)
    den = sum(e(*(u0 + 2 * uk for u0, uk in zip((0, 2, 0), u))) for u in unit)
    den -= sum(e(*(u0 + uk for u0, uk in zip((0, 1, 0), u))) ** 2 for u in unit)
    alpha_star = num / den
    coords = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]])
    conn = np.array([[0, 1, 2]])
    N = 200_000
    lam = sampling.element_samples(2, 1, N, seed=77, stream=0)
    X = sampling.physical_points(coords, conn, lam)
    y = (X[..., 0] ** 2)[None]
    g = (coords[:, 0] ** 2)[None]
    _, alpha = cvmc.element_loads_own_alpha(coords, conn, g, y, lam)
    assert abs(alpha_star - 88 / 119) < 1e-15   # the same moments in exact rational arithmetic
    assert abs(alpha[0, 0] - alpha_star) < 0.01


@pytest.mark.parametrize("kind", ["2d", "3d"])
def test_own_alpha_reproduces_affine_and_conserves_constant(kind):
    """Affine f^s: y = g(X) exactly, so every element's coefficient is 1 and the
    target reproduces f; constant f^s: sum b = c |domain| for any coefficient."""
    tmesh, smesh = _pair(kind)
    r = cvmc.transfer(*tmesh, _source(smesh, "affine"), 8, seed=3, own_alpha=True)
    assert np.abs(r["alpha_elements"] - 1.0).max() < 1e-9
    assert np.abs(r["x"][0] - fields.evaluate("affine", np, tmesh[0])[0]).max() < 1e-12
    r = cvmc.transfer(*tmesh, _source(smesh, "constant"), 8, seed=4, own_alpha=True)
    assert abs(r["b"].sum() - 2.5) < 1e-13


def test_own_alpha_variance_no_larger_than_fixed(sm_case):
    """Per-element coefficients lower the replicate RMS error against the exact
    b below alpha = 1 and far below alpha = 0 (plain Monte Carlo), and the
    estimate stays centred on the exact b at this N (its bias, of order 1/N,
    is below the sampling error)."""
    tmesh, smesh, pieces = sm_case
    for name in ("paper_f2", "front_2d"):
        sv = fields.evaluate(name, np, smesh[0])
        exact = supermesh.supermesh_projection(*tmesh, *smesh, sv, pieces=pieces)["b"][0]
        src = P1Source(*smesh, sv)
        rms = {}
        for mode in ("zero", "one", "own"):
            bs = np.array([cvmc.transfer(*tmesh, src, 16, alpha=0.0 if mode == "zero" else 1.0, seed=500 + s,
                                         stream=2, own_alpha=mode == "own")["b"][0] for s in range(40)])
            rms[mode] = np.sqrt(np.mean(np.square(bs - exact)))
            if mode == "own":
                z = (bs.mean(axis=0) - exact) / (bs.std(axis=0, ddof=1) / math.sqrt(len(bs)))
                assert np.mean(z ** 2) < 1.6
        assert rms["own"] < rms["one"] < 0.2 * rms["zero"]


# ---- the standard error of sum b and the samples an error target needs --------------------
def test_variance_term_closed_form():
    """One reference triangle, f = x^2, alpha = 0: the residual is l_1^2 and its
    variance is E[l_1^4] - E[l_1^2]^2 = 1/15 - 1/36 = 7/180 (Dirichlet moments),
    so the variance term is |T|^2 (7/180) / N with |T| = 1/2."""
    from oracle import sampling

    coords = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]])
    conn = np.array([[0, 1, 2]])
    N = 200_000
    lam = sampling.element_samples(2, 1, N, seed=5, stream=0)
    X = sampling.physical_points(coords, conn, lam)
    r = (X[..., 0] ** 2)[None]
    v = cvmc.element_variance_terms(coords, conn, r)
    assert abs(v[0, 0] * N / 0.25 - 7.0 / 180.0) < 0.01 * 7.0 / 180.0
    # with three samples per element the sample variance is unbiased only with
    # the N - 1 divisor: averaged over many copies of the element it is still
    # 7/180 (the N divisor would give two thirds of it)
    Ec, n3 = 200_000, 3
    conn_c = np.tile(conn, (Ec, 1))
    lam = sampling.element_samples(2, Ec, n3, seed=6, stream=0)
    X = sampling.physical_points(coords, conn_c, lam)
    v = cvmc.element_variance_terms(coords, conn_c, (X[..., 0] ** 2)[None])
    assert abs(v.mean() * n3 / 0.25 - 7.0 / 180.0) < 0.02 * 7.0 / 180.0


def test_stderr_matches_replicate_spread(sm_case):
    """Over 200 realizations the spread of sum b matches the reported standard
    error, sum b centres on the exact integral of f^s (z-scores), an affine
    source has standard error 0, and samples_for_tolerance follows N^-1/2."""
    tmesh, smesh, pieces = sm_case
    sv = fields.evaluate("paper_f3", np, smesh[0])
    src = P1Source(*smesh, sv)
    exact = src.integral()[0]
    sums, errs = [], []
    for s in range(200):
        rep = cvmc.transfer(*tmesh, src, 8, alpha=0.5, seed=900 + s, stream=1)["report"][0]
        sums.append(rep["sum_b"])
        errs.append(rep["sum_b_stderr"])
    sums, errs = np.array(sums), np.array(errs)
    assert 0.85 < sums.std(ddof=1) / np.sqrt(np.mean(errs ** 2)) < 1.15
    z = (sums - exact) / errs
    assert 0.7 < np.mean(z ** 2) < 1.4
    aff = cvmc.transfer(*tmesh, _source(smesh, "affine"), 8, seed=3)["report"][0]
    assert aff["sum_b_stderr"] < 1e-15
    N2 = cvmc.samples_for_tolerance(errs[0], sums[0], 8, 0.25 * (1 + 1e-12) * errs[0] / abs(sums[0]))
    assert N2 == 8 * 16
    # one sample per element: no spread to estimate from
    assert cvmc.transfer(*tmesh, src, 1, alpha=0.5, seed=4)["report"][0]["sum_b_stderr"] == -1.0
