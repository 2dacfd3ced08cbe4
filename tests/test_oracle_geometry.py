"""Pins of the oracle's sampling maps, quadrature, element measures and mass matrix."""
import itertools
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import geometry, sampling
from workloads import meshes


# ---- sampling: uniform on the simplex -----------------------------------------------
@pytest.mark.parametrize("dim", [2, 3])
def test_simplex_moments(dim):
    """E[l_k] = 1/(d+1), E[l_k^2] = 2/((d+1)(d+2)), E[l_k l_l] = 1/((d+1)(d+2))."""
    n_el, N = 4000, 128
    lam = sampling.element_samples(dim, n_el, N, seed=123, stream=1).reshape(-1, dim + 1)
    n = lam.shape[0]
    assert np.all(lam > 0)
    assert np.abs(lam.sum(axis=1) - 1.0).max() < 4e-16
    d1 = dim + 1
    m1 = lam.mean(axis=0)
    assert np.abs(m1 - 1.0 / d1).max() < 5 * lam.std(axis=0).max() / math.sqrt(n)
    second = lam.T @ lam / n
    expect = (np.ones((d1, d1)) + np.eye(d1)) / (d1 * (dim + 2))
    sd = np.sqrt(((lam[:, :, None] * lam[:, None, :]) ** 2).mean(axis=0) / n)
    assert np.all(np.abs(second - expect) < 6 * sd)


@pytest.mark.parametrize("dim", [2, 3])
def test_simplex_chi2_equal_volume_cells(dim):
    """Midpoint subdivision: corner cells {l_k > 1/2} hold 2^-d of the volume each."""
    from scipy import stats

    lam = sampling.element_samples(dim, 2000, 200, seed=77, stream=0).reshape(-1, dim + 1)
    corner = np.argmax(lam > 0.5, axis=1)
    inner = ~(lam > 0.5).any(axis=1)
    counts = [np.sum((corner == k) & ~inner) for k in range(dim + 1)] + [inner.sum()]
    p_corner = 2.0 ** -dim
    probs = [p_corner] * (dim + 1) + [1.0 - (dim + 1) * p_corner]
    chi2 = stats.chisquare(counts, np.array(probs) * lam.shape[0])
    assert chi2.pvalue > 1e-4


def test_physical_points_inside_element():
    coords, conn = meshes.delaunay_tri_mesh(8, 0.3, 3)
    lam, = [sampling.element_samples(2, conn.shape[0], 16, 5, 0)]
    X = sampling.physical_points(coords, conn, lam)
    from oracle.source import barycentric_cramer
    mu = barycentric_cramer(coords[conn][:, None, :, :], X)
    assert np.abs(mu - lam).max() < 1e-12


def test_samples_are_pure_function_of_counter():
    a = sampling.element_samples(2, 50, 8, seed=9, stream=3, elems=np.array([7, 40]))
    b = sampling.element_samples(2, 50, 8, seed=9, stream=3)[[7, 40]]
    assert np.array_equal(a, b)
    c = sampling.element_samples(2, 50, 8, seed=9, stream=4, elems=np.array([7, 40]))
    assert not np.array_equal(a, c)


# ---- quadrature -----------------------------------------------------------------------
def _ref_simplex_integral(dim, fn):
    if dim == 2:
        return integrate.dblquad(lambda y, x: fn(x, y), 0, 1, 0, lambda x: 1 - x, epsabs=1e-13)[0]
    return integrate.tplquad(lambda z, y, x: fn(x, y, z), 0, 1, 0, lambda x: 1 - x,
                             0, lambda x, y: 1 - x - y, epsabs=1e-12)[0]


@pytest.mark.parametrize("dim", [2, 3])
def test_dirichlet_formula_vs_numerical_integration(dim):
    vol = 1.0 / math.factorial(dim)
    for exps in [(0,) * (dim + 1), (1,) + (0,) * dim, (2,) + (0,) * dim, (1, 1) + (0,) * (dim - 1),
                 (0, 2) + (0,) * (dim - 1), (1, 0, 2) + (0,) * (dim - 2)]:
        def fn(*x):
            lam = [1.0 - sum(x)] + list(x)
            return math.prod(l ** a for l, a in zip(lam, exps))
        ref = _ref_simplex_integral(dim, fn)
        assert abs(geometry.dirichlet_monomial_integral(exps, vol) - ref) < 1e-10


@pytest.mark.parametrize("dim", [2, 3])
def test_quadrature_exact_to_degree_two(dim):
    pts, w = geometry.quadrature_rule(dim)
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.abs(pts.sum(axis=1) - 1.0).max() < 1e-15
    for deg in range(3):
        for exps in itertools.product(range(deg + 1), repeat=dim + 1):
            if sum(exps) != deg:
                continue
            q = float(np.sum(w * np.prod(pts ** np.array(exps), axis=1)))
            exact = geometry.dirichlet_monomial_integral(exps, 1.0)
            assert abs(q - exact) < 1e-15, exps
    # and it is not exact for every cubic (it is a genuine degree-2 rule)
    cub = (3,) + (0,) * dim
    q = float(np.sum(w * pts[:, 0] ** 3))
    assert abs(q - geometry.dirichlet_monomial_integral(cub, 1.0)) > 1e-6


# ---- measures and mass matrix ---------------------------------------------------------
MESHES = {
    "delaunay": lambda: meshes.delaunay_tri_mesh(12, 0.3, 4),
    "structured": lambda: meshes.structured_tri_mesh(10, 0.2, 5),
    "kuhn": lambda: meshes.kuhn_tet_mesh(5, 0.08, 6),
}


@pytest.mark.parametrize("name", list(MESHES))
def test_measures_tile_the_unit_domain(name):
    coords, conn = MESHES[name]()
    vol = geometry.element_measures(coords, conn)
    assert np.all(geometry.signed_dets(coords, conn) > 0)
    assert abs(vol.sum() - 1.0) < 1e-13


@pytest.mark.parametrize("name", list(MESHES))
def test_mass_matrix_closed_form_equals_quadrature(name):
    coords, conn = MESHES[name]()
    dim = coords.shape[1]
    for v in (1.0, 0.37):
        a = geometry.local_mass_closed_form(dim, v)
        b = geometry.local_mass_quadrature(dim, v)
        assert np.abs(a - b).max() < 1e-16 * 10
    Mc = geometry.mass_matrix(coords, conn, "closed")
    Mq = geometry.mass_matrix(coords, conn, "quadrature")
    assert abs(Mc - Mq).max() < 1e-17 * 100
    # sum of all entries is the domain measure, row sums are the lumped mass
    assert abs(Mc.sum() - 1.0) < 1e-13
    assert np.abs(np.asarray(Mc.sum(axis=1)).ravel() - geometry.lumped_mass(coords, conn)).max() < 1e-16 * 10
    assert abs(Mc - Mc.T).max() <= 4e-16 * abs(Mc).max()


@pytest.mark.parametrize("name", list(MESHES))
def test_jacobi_scaled_mass_spectrum(name):
    """Eigenvalues of D^-1 M lie in [1/2, 2] (triangles) or [1/2, 5/2] (tets)."""
    coords, conn = MESHES[name]()
    dim = coords.shape[1]
    M = geometry.mass_matrix(coords, conn).toarray()
    d = np.sqrt(np.diag(M))
    ev = np.linalg.eigvalsh(M / d[:, None] / d[None, :])
    hi = 2.0 if dim == 2 else 2.5
    assert ev.min() >= 0.5 - 1e-12 and ev.max() <= hi + 1e-12
