"""Pins of the oracle's P1 source localization and evaluation (brute force, exactness)."""
import numpy as np
import pytest

from oracle.source import OUT_OF_DOMAIN_TOL, P1Source
from workloads import fields, meshes


def _brute_force(coords, conn, pts):
    """Rule winner over every element; barycentrics by a dense linear solve."""
    d = coords.shape[1]
    V = coords[conn]                                   # (E, d+1, d)
    A = np.ones((conn.shape[0], d + 1, d + 1))
    A[:, :d, :] = np.transpose(V, (0, 2, 1))           # columns are homogeneous vertices
    ids, mus = [], []
    for p in pts:
        rhs = np.append(p, 1.0)
        mu = np.linalg.solve(A, np.broadcast_to(rhs, (conn.shape[0], d + 1))[..., None])[..., 0]
        mn = mu.min(axis=1)
        best = np.flatnonzero(mn == mn.max()).min()
        ids.append(best)
        mus.append(mu[best])
    return np.array(ids), np.array(mus)


@pytest.mark.parametrize("kind", ["delaunay", "structured", "kuhn"])
def test_locate_matches_brute_force(kind):
    rng = np.random.default_rng(11)
    if kind == "delaunay":
        coords, conn = meshes.delaunay_tri_mesh(10, 0.3, 1)
    elif kind == "structured":
        coords, conn = meshes.structured_tri_mesh(9, 0.2, 2)
    else:
        coords, conn = meshes.kuhn_tet_mesh(4, 0.08, 3)
    d = coords.shape[1]
    pts = np.concatenate([rng.uniform(0, 1, (600, d)), coords[:40],          # vertices
                          0.5 * (coords[conn[:30, 0]] + coords[conn[:30, 1]])])  # edge midpoints
    src = P1Source(coords, conn, np.zeros(coords.shape[0]))
    ids, mu, out = src.locate(pts)
    bids, bmu = _brute_force(coords, conn, pts)
    fd = src.face_distance(ids, mu)
    away = fd > 1e-12
    assert away.sum() > 500
    assert np.array_equal(ids[away], bids[away])
    assert np.abs(mu[away] - bmu[away]).max() < 1e-12
    # the winner's min barycentric equals the brute-force maximum everywhere
    assert np.abs(mu.min(axis=1) - bmu.min(axis=1)).max() < 1e-12
    assert not out.any()


@pytest.mark.parametrize("kind", ["delaunay", "kuhn"])
def test_affine_field_is_reproduced(kind):
    rng = np.random.default_rng(5)
    if kind == "delaunay":
        coords, conn = meshes.delaunay_tri_mesh(11, 0.3, 7)
    else:
        coords, conn = meshes.kuhn_tet_mesh(5, 0.08, 8)
    d = coords.shape[1]
    vals = fields.evaluate("affine", np, coords)
    src = P1Source(coords, conn, vals)
    pts = rng.uniform(0, 1, (3000, d))
    assert np.abs(src(pts) - fields.evaluate("affine", np, pts)).max() < 1e-13
    # exact integral of an affine function over the unit square / cube
    c0, c = 1.25, (0.75, -2.0, 0.5)
    assert abs(src.integral()[0] - (c0 + 0.5 * sum(c[:d]))) < 1e-13


def test_out_of_domain_points_flagged_and_extrapolated():
    coords, conn = meshes.structured_tri_mesh(6, 0.0, 0)
    vals = fields.evaluate("affine", np, coords)
    src = P1Source(coords, conn, vals)
    pts = np.array([[1.2, 0.5], [-0.3, -0.1], [0.5, 0.5], [1.0 + 1e-12, 0.3]])
    ids, mu, out = src.locate(pts)
    assert out.tolist() == [True, True, False, False]
    assert mu[0].min() < OUT_OF_DOMAIN_TOL
    # extrapolation of an affine field from the best element is still exact
    assert np.abs(src.evaluate_at(ids, mu) - fields.evaluate("affine", np, pts)).max() < 1e-12


def test_multi_field_evaluation():
    coords, conn = meshes.kuhn_tet_mesh(4, 0.08, 9)
    modes = fields.fourier_modes(seed=3, n_fields=5, n_modes=4, kmax=2)
    vals = fields.fourier_fields_3d(np, coords[:, 0], coords[:, 1], coords[:, 2], modes)
    src = P1Source(coords, conn, vals)
    pts = coords[[3, 17, 40]]
    y = src(pts)
    assert y.shape == (5, 3)
    assert np.abs(y - vals[:, [3, 17, 40]]).max() < 1e-13


# ---------------------------------------------------------------- face distances
# Elements whose heights h_k (distance from vertex k to the opposite face) are
# known in closed form: the right triangle (0,0), (a,0), (0,b) has h_1 = a,
# h_2 = b and h_0 = ab / sqrt(a^2 + b^2); the right tetrahedron with legs a, b,
# c has h_1 = a, h_2 = b, h_3 = c and h_0 = 1 / sqrt(a^-2 + b^-2 + c^-2).  The
# legs differ, so a height taken from the wrong face, or scaled wrongly, is
# caught, and so is the exclusion decision at the 1e-12 cut of the element-id
# comparison (points within 1e-12 of a face are left out of it).
def _right_simplex(d, legs):
    coords = np.zeros((d + 1, d))
    for k in range(d):
        coords[k + 1, k] = legs[k]
    conn = np.arange(d + 1)[None, :]
    h0 = 1.0 / np.sqrt(np.sum(1.0 / np.asarray(legs, dtype=float) ** 2))
    return coords, conn, np.array([h0, *legs])


@pytest.mark.parametrize("d,legs", [(2, (0.7, 0.2)), (3, (0.5, 0.3, 0.9)), (3, (3e-6, 7e-6, 2e-6))])
def test_face_distance_closed_form(d, legs):
    coords, conn, h = _right_simplex(d, legs)
    src = P1Source(coords, conn, np.zeros(d + 1))
    assert np.allclose(src.heights[0], h, rtol=1e-14, atol=0)
    scale = min(legs)
    # a point well inside: every face distance is mu_k h_k; at the centroid mu_k = 1/(d+1)
    centroid = coords.mean(axis=0)
    ids, mu, _ = src.locate(centroid[None, :])
    assert np.isclose(src.face_distance(ids, mu)[0], h.min() / (d + 1), rtol=1e-13)
    for k in range(d + 1):
        # points at signed distance delta from face k (positive: inside), near
        # the middle of that face; for k >= 1 the face is the coordinate plane
        # x_{k-1} = 0, for k = 0 the hypotenuse face with outward normal n
        if k == 0:
            n = 1.0 / np.asarray(legs, dtype=float)
            n /= np.linalg.norm(n)
            on_face = coords[1:].mean(axis=0)
            direction = -n
        else:
            others = [i for i in range(d + 1) if i != k]
            on_face = coords[others].mean(axis=0)
            direction = np.zeros(d)
            direction[k - 1] = 1.0
        for rel, inside in ((1e-13, False), (1e-11, True), (-1e-11, False), (0.05, True)):
            delta = rel * (1.0 if rel < 1e-3 else scale)
            p = on_face + delta * direction
            ids, mu, _ = src.locate(p[None, :])
            fd = src.face_distance(ids, mu)[0]
            tol = 1e-15 * max(1.0, np.abs(p).max() / scale) + 1e-16 * abs(delta)
            assert abs(fd - delta) <= max(tol, 2e-12 * abs(delta)), (k, rel, fd, delta)
            assert (fd > 1e-12) == inside, (k, rel, fd)
