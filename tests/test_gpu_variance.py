"""GPU parity of the variance variants against the FP64 oracle: stratified
samples (every route that draws samples) and each element's own control
coefficient (the black-box consumption), and their statistics against the
exact load vector of the intersection route."""
import numpy as np
import pytest

from gpu_cases import log, rel_l2
from oracle import cvmc, sampling
from oracle.source import P1Source
from paper_2603_00538_amd import ft
from workloads import fields, meshes

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SEED = 0x0F7A5EED000000F0


def _pair(dim):
    if dim == 2:
        return meshes.delaunay_tri_mesh(11, 0.3, 141), meshes.delaunay_tri_mesh(15, 0.3, 142)
    return meshes.kuhn_tet_mesh(5, 0.08, 143), meshes.kuhn_tet_mesh(7, 0.08, 144)


def _field(dim, x):
    return fields.evaluate("front_2d" if dim == 2 else "gaussian_bumps_3d", np, x)


def _cfg(N, F=1, alpha=1.0, stream=0, prec=ft.FT_F64, strat=False, own=False):
    c = ft.SampleCfg(N, F, alpha, SEED, stream, prec)
    c.sampling = ft.FT_SAMPLING_STRATIFIED if strat else ft.FT_SAMPLING_PLAIN
    c.alpha_mode = ft.FT_ALPHA_ELEMENT if own else ft.FT_ALPHA_FIXED
    return c


@pytest.mark.parametrize("dim,N", [(2, 64), (2, 50), (2, 7), (3, 64), (3, 27), (3, 100)])
def test_stratified_points_match_oracle(dim, N):
    tm, _ = _pair(dim)
    tc, tconn = tm
    log(f"stratified emission dim={dim} N={N}")
    lam = sampling.element_samples(dim, tconn.shape[0], N, SEED, 2, stratified=True)
    X = sampling.physical_points(tc, np.asarray(tconn, dtype=np.int64), lam)
    ref = np.concatenate([tc, X.reshape(-1, dim)]).T
    T = ft.Target(*tm)
    for prec in (ft.FT_F64, ft.FT_F32):
        pts = T.sample_points(_cfg(N, stream=2, prec=prec, strat=True)).double().cpu().numpy()
        err = np.abs(pts - ref)
        if prec == ft.FT_F64:
            assert err.max() < 2e-15
        else:
            assert np.median(err) < 1e-7 and err.max() < 5e-5
    T.close()


@pytest.mark.parametrize("dim,N,alpha", [(2, 64, 1.0), (2, 20, 0.5), (3, 27, 1.0), (3, 64, 0.75)])
def test_stratified_transfer_matches_oracle_all_routes(dim, N, alpha):
    tm, sm = _pair(dim)
    sv = _field(dim, sm[0])
    ref = cvmc.transfer(*tm, P1Source(*sm, sv), N, alpha=alpha, seed=SEED, stream=3, stratified=True)
    log(f"stratified transfer dim={dim} N={N} alpha={alpha}")
    T = ft.Target(*tm)
    S = ft.Source(*sm, sv)
    cfg = _cfg(N, alpha=alpha, stream=3, strat=True)
    # black box
    pts = T.sample_points(cfg)
    T.consume(cfg, S.eval_query_list(pts, T.n_nodes))
    r = T.project(1)
    assert rel_l2(r.b.cpu().numpy(), ref["b"]) < 1e-12
    assert rel_l2(r.x.cpu().numpy(), ref["x"]) < 1e-12
    # fused route, plan and batch draw the same samples
    T.transfer_from(S, cfg)
    r2 = T.project(1)
    assert rel_l2(r2.b.cpu().numpy(), ref["b"]) < 1e-12
    plan = ft.Plan(T, S, cfg)
    plan.transfer()
    assert torch.equal(T.project(1).b, r2.b)
    plan.close()
    B = ft.Batch([T], [S], [cfg])
    _, bs, _, _, _ = B.run(rtol=1e-14, max_iter=80)
    assert rel_l2(bs[0].cpu().numpy(), ref["b"][0]) < 1e-12
    B.close()
    # consumption must use the sampling the points were drawn with
    with pytest.raises(ft.FtError) as e:
        T.consume(_cfg(N, alpha=alpha, stream=3), S.eval_query_list(pts, T.n_nodes))
    assert e.value.status == ft.FT_E_ORDER
    T.close()
    S.close()


@pytest.mark.parametrize("dim,N,F,strat", [(2, 64, 1, False), (2, 16, 3, False), (3, 32, 1, False),
                                           (2, 36, 1, True), (3, 64, 2, True)])
def test_own_alpha_matches_oracle(dim, N, F, strat):
    tm, sm = _pair(dim)
    if F == 1:
        sv = _field(dim, sm[0])
    else:
        names = ["front_2d", "paper_f2", "smooth_2d"] if dim == 2 else None
        sv = (np.stack([fields.evaluate(n_, np, sm[0])[0] for n_ in names[:F]]) if dim == 2 else
              np.stack([fields.evaluate("gaussian_bumps_3d", np, sm[0])[0], np.cos(3 * sm[0][:, 0]) + sm[0][:, 2]]))
    ref = cvmc.transfer(*tm, P1Source(*sm, sv), N, seed=SEED, stream=4, stratified=strat, own_alpha=True)
    log(f"own alpha dim={dim} N={N} F={F} stratified={strat}")
    T = ft.Target(*tm)
    S = ft.Source(*sm, np.ascontiguousarray(sv))
    for prec in (ft.FT_F64, ft.FT_F32):
        cfg = _cfg(N, F=F, stream=4, prec=prec, strat=strat, own=True)
        pts = T.sample_points(cfg)
        T.consume(cfg, S.eval_query_list(pts, T.n_nodes))
        r = T.project(F)
        eb, ex = rel_l2(r.b.cpu().numpy(), ref["b"]), rel_l2(r.x.cpu().numpy(), ref["x"])
        if prec == ft.FT_F64:
            assert eb < 1e-12 and ex < 1e-12
        else:
            assert eb < 1e-5 and ex < 1e-5
        for f in range(F):
            assert abs(r.reports[f]["sum_b"] - ref["report"][f]["sum_b"]) <= 1e-6 * abs(ref["report"][f]["sum_b"])
    T.close()
    S.close()


def test_own_alpha_unsupported_routes():
    tm, sm = _pair(2)
    T = ft.Target(*tm)
    S = ft.Source(*sm, _field(2, sm[0]))
    cfg = _cfg(16, own=True)
    for call in (lambda: T.transfer_from(S, cfg), lambda: ft.Plan(T, S, cfg), lambda: ft.Batch([T], [S], [cfg])):
        with pytest.raises(ft.FtError) as e:
            call()
        assert e.value.status == ft.FT_E_UNSUPPORTED
    c16 = _cfg(16, own=True, prec=ft.FT_SPLIT_F16)
    pts = T.sample_points(c16)
    with pytest.raises(ft.FtError) as e:
        T.consume(c16, S.eval_query_list(pts, T.n_nodes))
    assert e.value.status == ft.FT_E_UNSUPPORTED
    T.close()
    S.close()


def test_variants_reduce_error_against_exact():
    """Over 30 realizations the RMS error of b against the intersection route's
    exact b: stratified samples and each element's own coefficient are both
    below plain sampling with alpha = 1 (paper_f2 field, N = 16)."""
    tm, sm = meshes.delaunay_tri_mesh(12, 0.3, 145), meshes.delaunay_tri_mesh(18, 0.3, 146)
    sv = fields.evaluate("paper_f2", np, sm[0])
    T = ft.Target(*tm)
    S = ft.Source(*sm, sv)
    T.transfer_supermesh(S)
    exact = T.project(1).b[0].cpu().numpy()
    rms = {}
    for name, strat, own in (("plain", False, False), ("stratified", True, False), ("own", False, True)):
        errs = []
        for r in range(30):
            cfg = _cfg(16, stream=100 + r, strat=strat, own=own)
            pts = T.sample_points(cfg)
            T.consume(cfg, S.eval_query_list(pts, T.n_nodes))
            errs.append(T.project(1).b[0].cpu().numpy() - exact)
        rms[name] = float(np.sqrt(np.mean(np.square(errs))))
    log(f"RMS error against the exact b: {rms}")
    assert rms["stratified"] < 0.7 * rms["plain"]
    assert rms["own"] < rms["plain"]
    T.close()
    S.close()
