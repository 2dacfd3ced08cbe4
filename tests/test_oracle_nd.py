"""Pins of the oracle on d-simplices, d = 4..6 (sec. 2's formulation for any
dimension; sec. 7's 5D/6D transfers): the sampling map against Dirichlet
closed forms, the degree-2 rule and the mass matrix against the Dirichlet
monomial formula, and the transfer against an affine field (reproduced), a
constant (conserved), and the exact load vector of a quadratic field
(unbiasedness), on Kuhn meshes of the unit hypercube."""
import itertools
import math

import numpy as np
import pytest

from oracle import cvmc, geometry, sampling
from workloads import fields, meshes

DIMS = [4, 5, 6]


@pytest.mark.parametrize("dim", DIMS)
def test_sample_weights_are_dirichlet(dim):
    """E[l_k] = 1/(d+1), E[l_k^2] = 2/((d+1)(d+2)), E[l_k l_m] = 1/((d+1)(d+2)),
    P(l_k > 1/2) = 2^-d, and every weight vector sums to 1."""
    n = 200_000
    lam = sampling.element_samples(dim, 1, n, 0x5EED0000 + dim, 3)[0]
    assert np.abs(lam.sum(axis=1) - 1.0).max() < 1e-15 and lam.min() >= 0.0
    d1 = dim + 1
    m1, m2, mx = 1.0 / d1, 2.0 / (d1 * (dim + 2)), 1.0 / (d1 * (dim + 2))
    se = 5.0 / math.sqrt(n)
    assert np.abs(lam.mean(axis=0) - m1).max() < se * math.sqrt(m2)
    assert np.abs((lam ** 2).mean(axis=0) - m2).max() < se * 0.1
    cross = (lam[:, :, None] * lam[:, None, :]).mean(axis=0)
    off = cross[~np.eye(d1, dtype=bool)]
    assert np.abs(off - mx).max() < se * 0.05
    tail = (lam > 0.5).mean(axis=0)
    assert np.abs(tail - 2.0 ** -dim).max() < 5.0 * math.sqrt(2.0 ** -dim / n)


@pytest.mark.parametrize("dim", DIMS)
def test_uniforms_follow_the_block_layout(dim):
    """u_(i+1) of a sample is uniform53 of Philox block i/2, words (0,1) or (2,3)."""
    from oracle import philox

    t = np.array([3, 17], dtype=np.uint32)
    j = np.array([0, 5], dtype=np.uint32)
    u = sampling.uniforms(dim, t, j, 0x1234_5678_9ABC_DEF0, 7)
    k0, k1 = philox.key_from_seed(0x1234_5678_9ABC_DEF0)
    for i in range(dim):
        w = philox.philox4x32_10(j, t, np.uint32(7), np.uint32(i // 2), k0, k1)
        ref = philox.uniform53(w[2 * (i % 2)], w[2 * (i % 2) + 1])
        assert np.array_equal(u[:, i], ref)


@pytest.mark.parametrize("dim", DIMS)
def test_degree_two_rule_and_mass_matrix(dim):
    pts, w = geometry.quadrature_rule(dim)
    assert abs(w.sum() - 1.0) < 1e-15
    for exps in itertools.product(range(3), repeat=dim + 1):
        if sum(exps) > 2:
            continue
        q = float(np.sum(w * np.prod(pts ** np.array(exps)[None, :], axis=1)))
        assert abs(q - geometry.dirichlet_monomial_integral(exps, 1.0)) < 1e-15
    c, t = meshes.kuhn_mesh(dim, 3, 0.03, 40 + dim)
    Mc = geometry.mass_matrix(c, t, "closed")
    Mq = geometry.mass_matrix(c, t, "quadrature")
    assert abs(Mc - Mq).max() < 1e-16
    assert abs(Mc.sum() - 1.0) < 1e-13
    assert np.abs(np.asarray(Mc.sum(axis=1)).ravel() - geometry.lumped_mass(c, t)).max() < 1e-16


def _quadratic(dim):
    rng = np.random.default_rng(70 + dim)
    c0 = 0.7
    cl = rng.uniform(-1, 1, dim)
    Q = rng.uniform(-1, 1, (dim, dim))
    Q = 0.5 * (Q + Q.T)

    def f(x):
        return (c0 + x @ cl + np.einsum("na,ab,nb->n", x, Q, x))[None]

    return f, c0, cl, Q


def _exact_load_quadratic(coords, conn, c0, cl, Q):
    """b_i = integral of f psi_i for f = c0 + cl.x + x^T Q x, element by element
    from the Dirichlet formula: on element t, x = sum_k l_k X_k, so f psi_i is a
    cubic in the barycentric weights."""
    dim = coords.shape[1]
    d1 = dim + 1
    vol = geometry.element_measures(coords, conn)
    X = coords[conn]                                                  # (E, d+1, d)
    I1 = np.array([geometry.dirichlet_monomial_integral(tuple(int(m == i) for m in range(d1)), 1.0)
                   for i in range(d1)])
    I2 = np.empty((d1, d1))
    I3 = np.empty((d1, d1, d1))
    for i, k in itertools.product(range(d1), repeat=2):
        I2[i, k] = geometry.dirichlet_monomial_integral(
            tuple((m == i) + (m == k) for m in range(d1)), 1.0)
    for i, k, l in itertools.product(range(d1), repeat=3):
        I3[i, k, l] = geometry.dirichlet_monomial_integral(
            tuple((m == i) + (m == k) + (m == l) for m in range(d1)), 1.0)
    lin = X @ cl                                                      # (E, d+1): cl . X_k
    quad = np.einsum("eka,ab,elb->ekl", X, Q, X)                      # X_k^T Q X_l
    loc = c0 * I1[None, :] + lin @ I2.T + np.einsum("ekl,ikl->ei", quad, I3)
    loc *= vol[:, None]
    b = np.zeros(coords.shape[0])
    np.add.at(b, conn.ravel(), loc.ravel())
    return b


@pytest.mark.parametrize("dim", DIMS)
def test_affine_reproduced_and_constant_conserved(dim):
    c, t = meshes.kuhn_mesh(dim, 3, 0.03, 50 + dim)

    def aff(x):
        return (0.3 + x @ np.linspace(-1.0, 1.0, dim))[None]

    r = cvmc.transfer(c, t, aff, 5, alpha=1.0, seed=9)
    assert np.abs(r["x"] - aff(c)).max() < 1e-12
    for a in (0.0, 0.6):
        rc = cvmc.transfer(c, t, lambda x: np.full((1, len(x)), 1.5), 4, alpha=a, seed=2)
        assert abs(rc["report"][0]["sum_b"] - 1.5) < 1e-12
        assert rc["report"][0]["cons_defect"] < 1e-12


@pytest.mark.parametrize("dim,strat", [(4, False), (5, False), (4, True)])
def test_unbiased_against_exact_quadratic_load(dim, strat):
    """The exact load of a quadratic field (Dirichlet formula): the mean of b
    over 200 realizations (alpha = 1/2, N = 6) within a few standard errors at
    every node; the quadratic integrates exactly under the degree-2 rule, so
    sum b is also checked against it."""
    c, t = meshes.kuhn_mesh(dim, 3, 0.03, 60 + dim)
    f, c0, cl, Q = _quadratic(dim)
    exact = _exact_load_quadratic(c, t, c0, cl, Q)
    pts, w = geometry.quadrature_rule(dim)
    vol = geometry.element_measures(c, t)
    integral = float(np.sum(vol[:, None] * w[None, :] * f(np.einsum("qk,ekc->eqc", pts, c[t]).reshape(-1, dim))
                            .reshape(len(t), -1)))
    assert abs(exact.sum() - integral) < 1e-13
    R = 200
    N = 16 if strat else 6   # 16 = 2^4: every sample of a 4-simplex in its own cell
    bs = np.array([cvmc.transfer(c, t, f, N, alpha=0.5, seed=300, stream=s, stratified=strat)["b"][0]
                   for s in range(R)])
    z = (bs.mean(axis=0) - exact) / (bs.std(axis=0, ddof=1) / math.sqrt(R))
    assert np.abs(z).max() < 5.0
    assert 0.6 < np.mean(z ** 2) < 1.5


def test_phase_space_field_and_kuhn_meshes():
    """The 5D/6D workload inputs: Kuhn meshes cover the unit hypercube with
    positively oriented simplices (d! (k-1)^d of them); the field is positive."""
    for dim, k in ((5, 3), (6, 3)):
        c, t = meshes.kuhn_mesh(dim, k, 0.03, 7)
        assert t.shape == (math.factorial(dim) * (k - 1) ** dim, dim + 1)
        assert (geometry.signed_dets(c, t) > 0).all()
        assert abs(geometry.element_measures(c, t).sum() - 1.0) < 1e-12
        v = fields.evaluate("phase_space", np, c)
        assert v.shape == (1, c.shape[0]) and v.min() > 0.0


def test_phase_space_integral_against_direct_quadrature():
    """The exact integral of the 5D/6D workload field (one-dimensional
    quadrature after separating the other coordinates) against direct
    two- and three-dimensional adaptive quadrature of the field itself."""
    from scipy.integrate import dblquad, tplquad

    def f2(y, x):
        return float(fields.evaluate("phase_space", np, np.array([[x, y]]))[0, 0])

    def f3(z, y, x):
        return float(fields.evaluate("phase_space", np, np.array([[x, y, z]]))[0, 0])

    v2, _ = dblquad(f2, 0, 1, 0, 1, epsabs=1e-13, epsrel=1e-12)
    assert abs(v2 - fields.phase_space_integral(2)) < 1e-11
    v3, _ = tplquad(f3, 0, 1, 0, 1, 0, 1, epsabs=1e-10, epsrel=1e-9)
    assert abs(v3 - fields.phase_space_integral(3)) < 1e-8
