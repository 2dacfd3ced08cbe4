"""Pins of the oracle's quadratic (P2) target transfer (oracle/p2.py)."""
import math

import numpy as np
import pytest

from oracle import geometry, p2
from oracle.source import P1Source
from workloads import fields, meshes


@pytest.mark.parametrize("dim", [2, 3])
def test_reference_mass_against_collapsed_gauss(dim):
    """The Dirichlet-formula reference mass matrix equals the one from a
    collapsed (Duffy) tensor Gauss-Legendre rule, a different integration
    method; the triangle's is the textbook |T|/180 [6 -1 -1 0 0 -4; ...]."""
    Mr = p2.reference_mass(dim)
    lam, w = p2.collapsed_rule(dim, 6)
    assert abs(w.sum() - 1.0) < 1e-14
    psi = p2.basis(lam)
    assert np.abs(np.einsum("q,qi,qj->ij", w, psi, psi) - Mr).max() < 1e-15
    if dim == 2:
        ref = np.array([[6, -1, -1, 0, 0, -4], [-1, 6, -1, 0, -4, 0], [-1, -1, 6, -4, 0, 0],
                        [0, 0, -4, 32, 16, 16], [0, -4, 0, 16, 32, 16], [-4, 0, 0, 16, 16, 32]]) / 180.0
        assert np.abs(Mr - ref).max() < 1e-16
    # row sums: the integrals of the basis functions (0 at triangle vertices,
    # -1/20 at tetrahedron vertices; 1/3 and 1/5 at edges)
    rs = Mr.sum(axis=1)
    v, e = (0.0, 1.0 / 3.0) if dim == 2 else (-1.0 / 20.0, 1.0 / 5.0)
    assert np.abs(rs[: dim + 1] - v).max() < 1e-15 and np.abs(rs[dim + 1:] - e).max() < 1e-15


@pytest.mark.parametrize("dim", [2, 3])
def test_basis_is_nodal_and_sums_to_one(dim):
    nodes = np.eye(dim + 1)
    mids = np.array([(nodes[a] + nodes[b]) / 2 for a, b in p2.LOCAL_EDGES[dim]])
    psi = p2.basis(np.concatenate([nodes, mids]))
    assert np.abs(psi - np.eye(p2.n_basis(dim))).max() < 1e-15
    lam = np.random.default_rng(3).dirichlet(np.ones(dim + 1), 500)
    assert np.abs(p2.basis(lam).sum(axis=1) - 1.0).max() < 1e-14


def _p2(kind, k, seed):
    c, t = meshes.delaunay_tri_mesh(k, 0.3, seed) if kind == "tri" else meshes.kuhn_tet_mesh(k, 0.08, seed)
    return meshes.p2_mesh(c, t)


def _quadratic(x):
    if x.shape[1] == 2:
        return (1.0 + x[:, 0] - 2.0 * x[:, 1] + 3.0 * x[:, 0] * x[:, 1] - x[:, 0] ** 2 + 0.5 * x[:, 1] ** 2)[None]
    return (1.0 + x[:, 0] - x[:, 2] + 2.0 * x[:, 1] * x[:, 2] - x[:, 0] ** 2 + x[:, 0] * x[:, 1])[None]


@pytest.mark.parametrize("kind,k", [("tri", 7), ("tet", 4)])
def test_quadratic_field_reproduced_and_conservation(kind, k):
    """alpha = 1: g interpolates a quadratic exactly, the residual vanishes and
    x equals the field at every P2 node for any N; a constant is conserved for
    every alpha; m^T x = sum b."""
    c2, t2 = _p2(kind, k, 40 + k)
    r = p2.transfer(c2, t2, _quadratic, 3, alpha=1.0, seed=9)
    assert np.abs(r["x"] - _quadratic(c2)).max() < 1e-12
    vol = geometry.element_measures(c2, np.asarray(t2[:, : c2.shape[1] + 1], dtype=np.int64)).sum()
    for a in (0.0, 0.5, 1.0):
        rc = p2.transfer(c2, t2, lambda x: np.full((1, len(x)), 2.5), 5, alpha=a, seed=3)
        assert abs(rc["report"][0]["sum_b"] - 2.5 * vol) < 1e-13
        assert rc["report"][0]["cons_defect"] < 1e-12
    assert abs(r["report"][0]["cons_defect"]) < 1e-12


@pytest.mark.parametrize("kind,k", [("tri", 6), ("tet", 3)])
def test_unbiased_against_exact_load(kind, k):
    """E[b] is the exact integral of f psi_i (a cubic f, its exact load from the
    collapsed rule): the mean over 300 realizations lies within a few standard
    errors at every node, with alpha = 1/2 so the residual is not small."""
    c2, t2 = _p2(kind, k, 60 + k)

    def cubic(x):
        return (1.0 + x[:, 0] ** 3 - 2.0 * x[:, 1] ** 2 * x[:, 0] + x[:, -1])[None]

    exact = p2.exact_load(c2, t2, cubic)[0]
    bs = np.array([p2.transfer(c2, t2, cubic, 8, alpha=0.5, seed=77, stream=s)["b"][0] for s in range(300)])
    z = (bs.mean(axis=0) - exact) / (bs.std(axis=0, ddof=1) / math.sqrt(len(bs)))
    assert np.abs(z).max() < 5.0
    assert np.mean(z ** 2) < 1.5


def test_p1_source_transfer_runs_and_conserves():
    """A P1 source on another mesh (the benchmark's black box): sum b and
    m^T x agree, and the standard error of sum b bounds its distance from the
    exact source integral."""
    c2, t2 = _p2("tri", 9, 81)
    sm = meshes.delaunay_tri_mesh(13, 0.3, 82)
    sv = fields.evaluate("paper_f2", np, sm[0])
    src = P1Source(*sm, sv)
    r = p2.transfer(c2, t2, src, 16, alpha=1.0, seed=5)
    rep = r["report"][0]
    assert rep["cons_defect"] < 1e-12
    assert abs(rep["sum_b"] - src.integral()[0]) < 6.0 * rep["sum_b_stderr"]
