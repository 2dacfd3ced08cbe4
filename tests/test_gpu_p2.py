"""GPU parity of quadratic (P2) targets (ft_target_create_p2) against the
oracle's P2 transfer (oracle/p2.py): the query list (every P2 node, then the
samples), the black-box consumption in binary64 and binary32 (several
fields, stratified samples, the element-tile layout, the no-allocation entry
point), the fused route, the standard error of sum b, exact reproduction of
a quadratic field, and the routes that do not take P2 targets."""
import numpy as np
import pytest

from gpu_cases import log, rel_l2
from oracle import p2, sampling
from oracle.source import P1Source
from paper_2603_00538_amd import ft
from workloads import fields, meshes

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SEED = 0x0F7A5EED00000130


def _case(dim, F=1):
    if dim == 2:
        tm, sm = meshes.delaunay_tri_mesh(9, 0.3, 241), meshes.delaunay_tri_mesh(14, 0.3, 242)
        names = ["front_2d", "paper_f2", "smooth_2d"]
        sv = np.stack([fields.evaluate(n_, np, sm[0])[0] for n_ in names[:F]])
    else:
        tm, sm = meshes.kuhn_tet_mesh(4, 0.08, 243), meshes.kuhn_tet_mesh(6, 0.08, 244)
        x = sm[0]
        sv = np.stack([fields.evaluate("gaussian_bumps_3d", np, x)[0], np.cos(3 * x[:, 0]) + x[:, 2],
                       np.sin(2 * x[:, 1])][:F])
    return meshes.p2_mesh(*tm), sm, np.ascontiguousarray(sv)


def _cfg(N, F=1, alpha=1.0, stream=0, prec=ft.FT_F64, strat=False, tiles=False):
    c = ft.SampleCfg(N, F, alpha, SEED, stream, prec)
    c.sampling = ft.FT_SAMPLING_STRATIFIED if strat else ft.FT_SAMPLING_PLAIN
    c.values_layout = ft.FT_VALUES_ELEMENT_TILES if tiles else ft.FT_VALUES_FIELD_MAJOR
    return c


@pytest.mark.parametrize("dim,N,F,alpha,strat,tiles", [
    (2, 64, 1, 1.0, False, False), (2, 20, 3, 0.5, True, False), (3, 37, 1, 1.0, False, False),
    (3, 128, 2, 0.75, False, True), (2, 5, 1, 0.0, False, False), (3, 64, 1, 1.0, True, False)])
def test_p2_black_box_matches_oracle(dim, N, F, alpha, strat, tiles):
    tm2, sm, sv = _case(dim, F)
    ref = p2.transfer(*tm2, P1Source(*sm, sv), N, alpha=alpha, seed=SEED, stream=3, stratified=strat)
    log(f"P2 black box dim={dim} N={N} F={F} alpha={alpha} stratified={strat} tiles={tiles}")
    T = ft.Target(*tm2, order=2)
    assert T.info.order == 2 and T.info.n_nodes == tm2[0].shape[0]
    S = ft.Source(*sm, sv)
    for prec, tol in ((ft.FT_F64, 1e-12), (ft.FT_F32, 1e-5)):
        cfg = _cfg(N, F, alpha, 3, prec, strat, tiles)
        pts = T.sample_points(cfg)
        if prec == ft.FT_F64:   # the query list: every P2 node, then the samples from the vertices
            lam = sampling.element_samples(dim, tm2[1].shape[0], N, SEED, 3, stratified=strat)
            X = sampling.physical_points(tm2[0], np.asarray(tm2[1][:, : dim + 1], dtype=np.int64), lam)
            want = np.concatenate([tm2[0], X.reshape(-1, dim)]).T
            assert np.abs(pts.cpu().numpy() - want).max() < 2e-15
        vals = S.eval_tiles(pts, T.n_nodes, T.n_elems, N) if tiles else S.eval_query_list(pts, T.n_nodes)
        T.consume(cfg, vals)
        r = T.project(F)
        assert r.status == ft.FT_OK
        assert rel_l2(r.b.cpu().numpy(), ref["b"]) < tol
        assert rel_l2(r.x.cpu().numpy(), ref["x"]) < tol
        for f in range(F):
            rep, rr = r.reports[f], ref["report"][f]
            assert abs(rep["sum_b"] - rr["sum_b"]) <= (1e-12 if prec == ft.FT_F64 else 1e-6) * abs(rr["sum_b"])
            assert rep["cons_defect"] < 1e-10
            if N >= 2:
                assert abs(rep["sum_b_stderr"] - rr["sum_b_stderr"]) <= \
                    (1e-9 if prec == ft.FT_F64 else 1e-2) * rr["sum_b_stderr"]
    T.close()
    S.close()


@pytest.mark.parametrize("dim,N,F", [(2, 64, 1), (2, 24, 3), (3, 128, 1), (3, 10, 2)])
def test_p2_fused_matches_black_box(dim, N, F):
    """ft_transfer_p1 on a P2 target: the same points, values and sums as the
    black-box route, binary64 and binary32."""
    tm2, sm, sv = _case(dim, F)
    T = ft.Target(*tm2, order=2)
    S = ft.Source(*sm, sv)
    log(f"P2 fused dim={dim} N={N} F={F}")
    for prec in (ft.FT_F64, ft.FT_F32):
        cfg = _cfg(N, F, 1.0, 4, prec)
        pts = T.sample_points(cfg)
        T.consume(cfg, S.eval_query_list(pts, T.n_nodes))
        rb = T.project(F)
        T.transfer_from(S, cfg)
        rf = T.project(F)
        assert rel_l2(rf.b.cpu().numpy(), rb.b.cpu().numpy()) < 1e-14
        assert rel_l2(rf.x.cpu().numpy(), rb.x.cpu().numpy()) < 1e-13
        for f in range(F):
            assert abs(rf.reports[f]["sum_b_stderr"] - rb.reports[f]["sum_b_stderr"]) <= \
                1e-12 * rb.reports[f]["sum_b_stderr"]
    T.close()
    S.close()


@pytest.mark.parametrize("dim", [2, 3])
def test_p2_reproduces_quadratic_black_box(dim):
    """A quadratic evaluated by the caller at the query points (alpha = 1): the
    residual vanishes, so x is the field at every P2 node, for any N."""
    tm2, _, _ = _case(dim)
    T = ft.Target(*tm2, order=2)
    cfg = _cfg(3)
    pts = T.sample_points(cfg)
    x = pts.double()
    if dim == 2:
        vals = 1.0 + x[0] - 2.0 * x[1] + 3.0 * x[0] * x[1] - x[0] ** 2 + 0.5 * x[1] ** 2
    else:
        vals = 1.0 + x[0] - x[2] + 2.0 * x[1] * x[2] - x[0] ** 2 + x[0] * x[1]
    T.consume(cfg, vals[None].contiguous())
    r = T.project(1)
    want = vals[: T.n_nodes].cpu().numpy()
    assert np.abs(r.x[0].cpu().numpy() - want).max() < 1e-12
    assert r.reports[0]["sum_b_stderr"] < 1e-12 * abs(r.reports[0]["sum_b"])
    T.close()


def test_p2_noalloc_and_unsupported_routes():
    tm2, sm, sv = _case(2)
    T = ft.Target(*tm2, order=2)
    S = ft.Source(*sm, sv)
    cfg = _cfg(32)
    pts = T.sample_points(cfg)
    vals = S.eval_query_list(pts, T.n_nodes)
    T.consume(cfg, vals)
    b1 = T.project(1).b.clone()
    T.consume(cfg, vals, noalloc=True)
    assert torch.equal(T.project(1).b, b1)
    own = _cfg(32)
    own.alpha_mode = ft.FT_ALPHA_ELEMENT
    calls = [lambda: T.consume(own, vals), lambda: T.transfer_supermesh(S), lambda: ft.Plan(T, S, cfg),
             lambda: ft.Batch([T], [S], [cfg])]
    c16 = _cfg(32, prec=ft.FT_SPLIT_F16)

    def split_form():
        pts16 = T.sample_points(c16)
        T.consume(c16, S.eval_query_list(pts16, T.n_nodes))

    calls.append(split_form)
    for call in calls:
        with pytest.raises(ft.FtError) as e:
            call()
        assert e.value.status == ft.FT_E_UNSUPPORTED
    T.close()
    S.close()
    # an edge node off its edge's midpoint
    c2, t2 = tm2
    bad = c2.copy()
    bad[t2[0, 3]] += 0.01
    with pytest.raises(ft.FtError) as e:
        ft.Target(bad, t2, order=2)
    assert e.value.status == ft.FT_E_MESH


@pytest.mark.parametrize("name,N", [("tri2d_1m_p2", 16), ("tet3d_2m_p2", 8)])
def test_p2_fullsize_quadratic_and_conservation(name, N):
    """At the full P2 workload sizes (2.0M and 2.9M nodes): a quadratic field
    evaluated by the caller at the query points is reproduced at every node
    (the P2 mass matrix, assembly and solve at scale), and for the workload's
    own source sum b lies within six standard errors of the exact integral."""
    from workloads import configs
    w = configs.WORKLOADS[name]
    c2, t2 = configs.target_mesh(w)
    log(f"full-size P2: {name}, N={N}")
    T = ft.Target(c2, t2, order=2)
    cfg = _cfg(N)
    pts = T.sample_points(cfg)
    x = pts
    if w.dim == 2:
        vals = 1.0 + x[0] - 2.0 * x[1] + 3.0 * x[0] * x[1] - x[0] ** 2 + 0.5 * x[1] ** 2
    else:
        vals = 1.0 + x[0] - x[2] + 2.0 * x[1] * x[2] - x[0] ** 2 + x[0] * x[1]
    T.consume(cfg, vals[None].contiguous())
    del vals
    r = T.project(1, rtol=1e-14, max_iter=1000)
    assert r.status == ft.FT_OK
    want = 1.0 + c2[:, 0] - 2.0 * c2[:, 1] + 3.0 * c2[:, 0] * c2[:, 1] - c2[:, 0] ** 2 + 0.5 * c2[:, 1] ** 2 \
        if w.dim == 2 else 1.0 + c2[:, 0] - c2[:, 2] + 2.0 * c2[:, 1] * c2[:, 2] - c2[:, 0] ** 2 + c2[:, 0] * c2[:, 1]
    assert np.abs(r.x[0].cpu().numpy() - want).max() < 1e-10
    sm = configs.build_mesh(w.source)
    S = ft.Source(*sm, configs.source_nodal_values(w, sm[0]), bins=w.bins[: w.dim] if any(w.bins) else None)
    T.transfer_from(S, _cfg(N))
    rep = T.project(1, rtol=1e-14, max_iter=1000).reports[0]
    I = S.integral()[0]
    log(f"  sum b {rep['sum_b']:.15e}, integral {I:.15e}, stderr {rep['sum_b_stderr']:.3e}, iters {rep['iters']}")
    assert rep["cons_defect"] < 1e-10
    assert abs(rep["sum_b"] - I) < 6.0 * rep["sum_b_stderr"]
    T.close()
    S.close()
