"""Pins of the oracle's exact tetrahedral supermesh projection
(oracle/supermesh3d.py) against closed forms and identities."""
import numpy as np
import pytest

from oracle import cvmc, geometry, supermesh3d
from oracle.source import P1Source
from workloads import fields, meshes

UNIT = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])


def test_closed_form_intersections():
    """The unit right tetrahedron against (i) its translate by (1/2, 0, 0): the
    tetrahedron x >= 1/2 of volume (1/2)^3 / 6; (ii) its reflection through its
    centroid: {x, y, z <= 1/2, 1/2 <= x + y + z <= 1}, the half cube minus two
    corner tetrahedra, volume 1/8 - 2/48 = 1/12 (an octahedron, half the
    tetrahedron), centred at the centroid; (iii) a far translate and (iv) its
    mirror image across the face x = 0: nothing (a shared face has no volume)."""
    sub, vol = supermesh3d.intersect(UNIT, UNIT + np.array([0.5, 0.0, 0.0]))
    assert abs(vol.sum() - 1.0 / 48.0) < 1e-15
    refl = 2.0 * UNIT.mean(axis=0) - UNIT
    sub, vol = supermesh3d.intersect(UNIT, refl)
    assert abs(vol.sum() - 1.0 / 12.0) < 1e-15
    assert len(supermesh3d.intersection_vertices(UNIT, refl)) == 6
    centre = (vol[:, None] * sub.mean(axis=1)).sum(axis=0) / vol.sum()
    assert np.abs(centre - 0.25).max() < 1e-15
    # integral of x^2 over it by the degree-2 rule on its pieces, against the
    # closed form: the half cube C = [0,1/2]^3 gives (1/2)^2 (1/2)^3 / 3 = 1/96;
    # the corner A = {x+y+z <= 1/2} gives (1/2)^5 / 60 = 1/1920 (Dirichlet);
    # the far corner B is A mapped by x -> 1/2 - x, so int_B x^2 =
    # int_A (1/2 - x)^2 = |A|/4 - |A|/8 + 1/1920 with |A| = 1/48, centroid 1/8
    pts, w = geometry.quadrature_rule(3)
    q = np.einsum("qk,pkc->pqc", pts, sub)
    ix2 = float(np.einsum("p,q,pq->", vol, w, q[..., 0] ** 2))
    corner_far = (1.0 / 48.0) / 4.0 - (1.0 / 48.0) / 8.0 + 1.0 / 1920.0
    assert abs(ix2 - (1.0 / 96.0 - 1.0 / 1920.0 - corner_far)) < 1e-15
    assert len(supermesh3d.intersect(UNIT, UNIT + 5.0)[1]) == 0
    assert len(supermesh3d.intersect(UNIT, UNIT * np.array([-1.0, 1.0, 1.0]))[1]) == 0


@pytest.fixture(scope="module")
def tets_case():
    tm = meshes.kuhn_tet_mesh(4, 0.08, 201)
    sm = meshes.kuhn_tet_mesh(5, 0.08, 202)
    return tm, sm, supermesh3d.intersections(*tm, *sm)


def test_partition_identity(tets_case):
    tm, sm, pieces = tets_case
    vol_t = geometry.element_measures(tm[0], np.asarray(tm[1], dtype=np.int64))
    got = supermesh3d.supermesh_projection(*tm, *sm, fields.evaluate("gaussian_bumps_3d", np, sm[0]),
                                           pieces=pieces)
    assert np.abs(got["vol_sum"] - vol_t).max() < 1e-14
    # and the source elements: every one is covered exactly once
    vol_s = geometry.element_measures(sm[0], np.asarray(sm[1], dtype=np.int64))
    per_s = np.zeros(len(vol_s))
    np.add.at(per_s, pieces[1], pieces[3])
    assert np.abs(per_s - vol_s).max() < 1e-14


def test_sum_b_is_source_integral_and_affine_reproduced(tets_case):
    tm, sm, pieces = tets_case
    sv = fields.evaluate("gaussian_bumps_3d", np, sm[0])
    got = supermesh3d.supermesh_projection(*tm, *sm, sv, pieces=pieces)
    I = P1Source(*sm, sv).integral()[0]
    assert abs(got["b"].sum() - I) < 1e-14 * abs(I)
    assert abs(got["int_fs"][0] - I) < 1e-14 * abs(I)
    aff = fields.evaluate("affine", np, sm[0])
    b = supermesh3d.supermesh_projection(*tm, *sm, aff, pieces=pieces)["b"]
    M = geometry.mass_matrix(tm[0], np.asarray(tm[1], dtype=np.int64))
    x = cvmc.solve_mass(M, b, 3)
    assert np.abs(x - fields.evaluate("affine", np, tm[0])).max() < 1e-12


def test_identical_meshes_give_mass_times_values():
    tm = meshes.kuhn_tet_mesh(3, 0.08, 203)
    F = fields.evaluate("gaussian_bumps_3d", np, tm[0])
    b = supermesh3d.supermesh_projection(*tm, *tm, F)["b"]
    M = geometry.mass_matrix(tm[0], np.asarray(tm[1], dtype=np.int64))
    assert np.abs(b - (M @ F[0])[None]).max() < 1e-14 * np.abs(M @ F[0]).max()
