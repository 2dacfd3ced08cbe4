"""GPU parity on d-simplices, d = 4..6 (sec. 2's formulation for any
dimension; sec. 7's 5D/6D distribution-function transfers) against the FP64
oracle: emitted points, the load vector, the solution and the standard error
of sum b for the black-box route (binary64 and binary32 forms, fixed and
per-element alpha, several fields, per-element sample counts) with the
analytic phase-space field as the point-query black box, evaluated by torch at
the emitted points; an affine field reproduced exactly; the routes that need
a source mesh or the triangle/tetrahedron-only variants rejected; and at full
size (933k 5-simplices, 525k 6-simplices) the load vector at sampled nodes
against the oracle, conservation, and sum b against the exact integral."""
import math

import numpy as np
import pytest

from gpu_cases import log, rel_l2
from oracle import adaptive, cvmc, geometry, sampling
from paper_2603_00538_amd import ft
from workloads import configs, fields, meshes

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SEED = 0x0F7A5EED00000160


def _mesh(dim):
    k = {4: 4, 5: 3, 6: 3}[dim]
    return meshes.kuhn_mesh(dim, k, 0.03, 210 + dim)


def _query_np(F):
    def q(x):
        rows = [fields.evaluate("phase_space", np, x)[0]]
        if F > 1:
            rows.append(np.cos(3.0 * x[:, 0]) + x[:, -1] ** 2)
        if F > 2:
            rows.append(np.exp(-np.sum((x - 0.3) ** 2, axis=1)))
        return np.stack(rows[:F])
    return q


def _query_torch(pts, F):
    x = pts.double().t()
    rows = [fields.evaluate("phase_space", torch, x)[0]]
    if F > 1:
        rows.append(torch.cos(3.0 * x[:, 0]) + x[:, -1] ** 2)
    if F > 2:
        rows.append(torch.exp(-torch.sum((x - 0.3) ** 2, dim=1)))
    v = torch.stack(rows[:F]).contiguous()
    return v if pts.dtype == torch.float64 else v.float()


def _cfg(N, F=1, alpha=1.0, stream=0, prec=ft.FT_F64, own=False):
    c = ft.SampleCfg(N, F, alpha, SEED, stream, prec)
    c.alpha_mode = ft.FT_ALPHA_ELEMENT if own else ft.FT_ALPHA_FIXED
    return c


@pytest.mark.parametrize("dim,N", [(4, 7), (4, 64), (5, 33), (5, 128), (6, 5)])
def test_nd_points_match_oracle(dim, N):
    c, t = _mesh(dim)
    log(f"emission dim={dim} N={N} E={len(t)}")
    lam = sampling.element_samples(dim, t.shape[0], N, SEED, 4)
    X = sampling.physical_points(c, np.asarray(t, dtype=np.int64), lam)
    ref = np.concatenate([c, X.reshape(-1, dim)]).T
    T = ft.Target(c, t)
    assert T.info.n_inverted == 0 and T.info.dim == dim
    for prec in (ft.FT_F64, ft.FT_F32):
        pts = T.sample_points(_cfg(N, stream=4, prec=prec)).double().cpu().numpy()
        assert pts.shape == ref.shape
        err = np.abs(pts - ref)
        if prec == ft.FT_F64:
            assert np.array_equal(pts[:, : c.shape[0]], ref[:, : c.shape[0]])
            assert err.max() < 2e-15
        else:
            assert np.median(err) < 1e-7 and err.max() < 1e-6
    T.close()


def test_nd_setup_matches_oracle_mass_matrix():
    """M g, the lumped mass and the element measures through a transfer of the
    control alone (a field in the target space: N = 1, alpha = 1 makes every
    residual zero, so b = M g exactly)."""
    for dim in (4, 5, 6):
        c, t = _mesh(dim)

        def aff(x):
            return (0.3 + x @ np.linspace(-1.0, 1.0, dim))[None]

        T = ft.Target(c, t)
        assert T.info.nnz == geometry.mass_matrix(c, t).nnz
        cfg = _cfg(1)
        pts = T.sample_points(cfg)
        vals = torch.as_tensor(aff(pts.double().cpu().numpy().T), device="cuda").contiguous()
        T.consume(cfg, vals)
        r = T.project(1)
        M = geometry.mass_matrix(c, t)
        g = aff(c)[0]
        b = r.b.cpu().numpy()[0]
        assert np.abs(b - M @ g).max() < 1e-15 * np.abs(M @ g).max() * 10
        assert np.abs(r.x.cpu().numpy()[0] - g).max() < 1e-12
        assert r.reports[0]["cons_defect"] < 1e-13
        T.close()


@pytest.mark.parametrize("dim,N,F,alpha,own", [
    (4, 64, 1, 1.0, False), (4, 20, 2, 0.5, False), (5, 37, 1, 0.75, False), (5, 16, 3, 1.0, True),
    (6, 8, 1, 1.0, False), (6, 3, 2, 0.0, True)])
def test_nd_transfer_matches_oracle(dim, N, F, alpha, own):
    c, t = _mesh(dim)
    ref = cvmc.transfer(c, t, _query_np(F), N, alpha=alpha, seed=SEED, stream=5, own_alpha=own)
    log(f"transfer dim={dim} N={N} F={F} alpha={alpha} own={own} E={len(t)}")
    T = ft.Target(c, t)
    for prec in (ft.FT_F64, ft.FT_F32):
        cfg = _cfg(N, F, alpha, 5, prec, own)
        pts = T.sample_points(cfg)
        T.consume(cfg, _query_torch(pts, F))
        r = T.project(F)
        assert r.status == ft.FT_OK
        eb, ex = rel_l2(r.b.cpu().numpy(), ref["b"]), rel_l2(r.x.cpu().numpy(), ref["x"])
        tol = 1e-12 if prec == ft.FT_F64 else 2e-5
        assert eb < tol and ex < tol, (prec, eb, ex)
        for f in range(F):
            want = ref["report"][f]["sum_b_stderr"]
            got = r.reports[f]["sum_b_stderr"]
            assert abs(got - want) <= (1e-9 if prec == ft.FT_F64 else 2e-2) * want
            assert r.reports[f]["cons_defect"] < 1e-12
    T.close()


def test_nd_per_element_counts_match_oracle():
    """Neyman counts in 5D: a pilot, the allocation (against the oracle's,
    away from rounding ties) and the transfer with caller counts."""
    dim = 5
    c, t = _mesh(dim)
    E = t.shape[0]
    q = _query_np(1)
    pilot = cvmc.transfer(c, t, q, 16, alpha=1.0, seed=SEED, stream=20)
    T = ft.Target(c, t)
    cfg = _cfg(16, stream=20)
    pts = T.sample_points(cfg)
    T.consume(cfg, _query_torch(pts, 1))
    T.project(1)
    off, al = T.allocate_samples(40 * E, n_min=2)
    got = np.diff(off.cpu().numpy())
    want = adaptive.allocate(pilot["var_terms"][0], 16, 40 * E, 2, 1 << 20)
    a = adaptive.weights(pilot["var_terms"][0], 16)
    frac = (40 * E * a / a.sum() + 0.5) % 1.0
    tie = np.minimum(frac, 1.0 - frac) < 1e-9
    assert np.array_equal(got[~tie], want[~tie]) and np.all(np.abs(got[tie] - want[tie]) <= 1)
    counts = np.random.default_rng(5).integers(1, 90, E)
    ref = adaptive.transfer(c, t, q, counts, alpha=0.5, seed=SEED, stream=21)
    o = torch.as_tensor(adaptive.offsets(counts), device="cuda")
    total = int(counts.sum())
    c0 = _cfg(0, 1, 0.5, 21)
    pts = T.sample_points_adaptive(c0, o, total)
    T.consume_adaptive(c0, o, total, _query_torch(pts, 1))
    r = T.project(1)
    assert rel_l2(r.b.cpu().numpy(), ref["b"]) < 1e-12 and rel_l2(r.x.cpu().numpy(), ref["x"]) < 1e-12
    assert r.reports[0]["sum_b_stderr"] == -1.0   # some element has a single sample
    T.close()


@pytest.mark.parametrize("dim,N", [(4, 81), (5, 40), (6, 64)])
def test_nd_stratified_matches_oracle(dim, N):
    """Stratified samples on d-simplices: points (binary64 and binary32) and
    the transfer against the oracle."""
    c, t = _mesh(dim)
    lam = sampling.element_samples(dim, t.shape[0], N, SEED, 6, stratified=True)
    X = sampling.physical_points(c, np.asarray(t, dtype=np.int64), lam)
    ref_pts = np.concatenate([c, X.reshape(-1, dim)]).T
    ref = cvmc.transfer(c, t, _query_np(1), N, alpha=0.5, seed=SEED, stream=6, stratified=True)
    log(f"stratified dim={dim} N={N}")
    T = ft.Target(c, t)
    for prec in (ft.FT_F64, ft.FT_F32):
        cfg = _cfg(N, 1, 0.5, 6, prec)
        cfg.sampling = ft.FT_SAMPLING_STRATIFIED
        pts = T.sample_points(cfg)
        err = np.abs(pts.double().cpu().numpy() - ref_pts)
        T.consume(cfg, _query_torch(pts, 1))
        r = T.project(1)
        if prec == ft.FT_F64:
            assert err.max() < 2e-15
            assert rel_l2(r.b.cpu().numpy(), ref["b"]) < 1e-12 and rel_l2(r.x.cpu().numpy(), ref["x"]) < 1e-12
        else:
            assert np.median(err) < 1e-7 and err.max() < 1e-6
            assert rel_l2(r.b.cpu().numpy(), ref["b"]) < 2e-5
    T.close()


def test_nd_unsupported_variants():
    c, t = _mesh(5)
    T = ft.Target(c, t)
    for kw in ({"precision": ft.FT_SPLIT_F16}, {"precision": ft.FT_SPLIT_BF16}):
        cfg = _cfg(16)
        for k, v in kw.items():
            setattr(cfg, k, v)
        with pytest.raises(ft.FtError) as e:
            T.sample_points(cfg)
        assert e.value.status == ft.FT_E_UNSUPPORTED, kw
    tm, sm = meshes.kuhn_tet_mesh(3, 0.08, 1), meshes.kuhn_tet_mesh(4, 0.08, 2)
    S = ft.Source(*sm, fields.evaluate("gaussian_bumps_3d", np, sm[0]))
    with pytest.raises(ft.FtError) as e:        # no 5D source: dimensions differ
        T.transfer_from(S, _cfg(16))
    assert e.value.status == ft.FT_E_ARG
    with pytest.raises(ft.FtError) as e:
        ft.Batch([T], None, [_cfg(16)])
    assert e.value.status == ft.FT_E_UNSUPPORTED
    with pytest.raises(ft.FtError) as e:        # P2 targets: triangles and tetrahedra (rejected before any copy)
        ft.Target(np.zeros((20, 4)), np.arange(15, dtype=np.int32)[None, :], order=2)
    assert e.value.status == ft.FT_E_ARG
    bad = np.array([[0.0] * 7] * 8)
    with pytest.raises(ft.FtError) as e:        # 7 dimensions
        ft.Target(bad, np.arange(8, dtype=np.int32)[None, :])
    assert e.value.status == ft.FT_E_ARG
    T.close()
    S.close()


def _node_load_oracle(c, t, q, N, alpha, seed, stream, nodes):
    """b at the given nodes from the oracle, over their incident elements only."""
    dim = c.shape[1]
    t64 = np.asarray(t, dtype=np.int64)
    out = []
    g = q(c)
    for v in nodes:
        el = np.nonzero((t64 == v).any(axis=1))[0]
        lam, X = cvmc.query_points(c, t64, N, seed, stream, el)
        y = q(X.reshape(-1, dim)).reshape(g.shape[0], el.size, N)
        beta = cvmc.element_loads(c, t64, g, y, lam, alpha, el)
        vol = geometry.element_measures(c, t64[el])
        k = np.argmax(t64[el] == v, axis=1)
        res = beta[:, np.arange(el.size), k].sum(axis=1)
        ctrl = alpha * np.sum(vol[None, :] * (g[:, t64[el]].sum(axis=2) + g[:, [v]]), axis=1) / ((dim + 1) * (dim + 2))
        out.append(res + ctrl)
    return np.array(out).T


@pytest.mark.parametrize("name", ["kuhn5d_1m", "kuhn6d_500k"])
def test_nd_fullsize(name):
    w = configs.WORKLOADS[name]
    c, t = configs.target_mesh(w)
    N = w.samples_per_elem
    log(f"full-size {name}: E={len(t)}, n={len(c)}, N={N}")
    T = ft.Target(c, t)
    cfg = ft.SampleCfg(N, 1, w.alpha, w.philox_seed, 0, ft.FT_F64)
    pts = T.sample_points(cfg)
    vals = _query_torch(pts, 1)
    del pts
    T.consume(cfg, vals)
    r = T.project(1, rtol=w.rtol, max_iter=1000)
    rep = r.reports[0]
    I = configs.field_integral(w)
    log(f"  sum b {rep['sum_b']:.15e}, integral {I:.15e}, stderr {rep['sum_b_stderr']:.3e}, iters {rep['iters']}")
    assert r.status == ft.FT_OK and rep["cons_defect"] < 1e-12
    assert abs(rep["sum_b"] - I) < 6.0 * rep["sum_b_stderr"]
    rng = np.random.default_rng(3)
    interior = np.nonzero(np.all((c > 0.0) & (c < 1.0), axis=1))[0]
    nodes = np.concatenate([rng.choice(interior, 3, replace=False), [0, len(c) - 1]])
    ref = _node_load_oracle(c, t, _query_np(1), N, w.alpha, w.philox_seed, 0, nodes)
    got = r.b.cpu().numpy()[:, nodes]
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max(), (got, ref)
    T.close()
