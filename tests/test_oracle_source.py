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
