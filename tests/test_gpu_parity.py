"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle.

Tolerances: FP64 load vector and solution within 1e-12 relative L2; element
ids bit-exact for points farther than 1e-12 from every face of the oracle's
element; FP32 form within 1e-5 relative L2 with conservation parity 1e-6.
"""
import os

import numpy as np
import pytest

from gpu_cases import gpu_transfer, log, oracle_query_points, oracle_transfer, rel_l2
from oracle import geometry
from oracle.source import P1Source
from paper_2603_00538_amd import ft
from workloads import configs, fields, meshes

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _small_2d():
    return meshes.delaunay_tri_mesh(12, 0.3, 31), meshes.delaunay_tri_mesh(17, 0.3, 32)


def _small_3d():
    return meshes.kuhn_tet_mesh(6, 0.08, 33), meshes.kuhn_tet_mesh(8, 0.08, 34)


@pytest.fixture(scope="module")
def c1():
    w = configs.WORKLOADS["tri2d_4k"]
    tm = configs.build_mesh(w.target)
    sm = configs.build_mesh(w.source)
    return w, tm, sm, configs.source_nodal_values(w, sm[0])


# ---------------------------------------------------------------- emission
# N a multiple of 64 takes the several-runs-per-wave emission: 242 triangles
# x 64 or 192 and 750 tetrahedra x 64 samples leave partial last waves
@pytest.mark.parametrize("dim,N", [(2, 1), (2, 7), (2, 64), (2, 192), (3, 5), (3, 33), (3, 64)])
def test_emitted_points_match_oracle(dim, N):
    tm, _ = _small_2d() if dim == 2 else _small_3d()
    log(f"emit dim={dim} N={N}")
    T = ft.Target(*tm)
    ref = oracle_query_points(tm, N, seed=0x0F7A5EED00000001, stream=3)
    for prec in (ft.FT_F64, ft.FT_F32):
        cfg = ft.SampleCfg(N, 1, 1.0, 0x0F7A5EED00000001, 3, prec)
        pts = T.sample_points(cfg).double().cpu().numpy()
        assert pts.shape == ref.shape
        err = np.abs(pts - ref)
        if prec == ft.FT_F64:
            assert np.array_equal(pts[:, :tm[0].shape[0]], ref[:, :tm[0].shape[0]])
            assert err.max() < 2e-15
        else:
            # 24-bit uniforms differ from 53-bit ones by <= 2^-24; sqrt amplifies that near xi -> 0
            assert np.median(err) < 1e-7 and err.max() < 5e-5
    T.close()


# ---------------------------------------------------------------- source localization
def test_source_ids_and_values_match_oracle(c1):
    w, tm, sm, sv = c1
    log("source ids/values on tri2d_4k query list + extra points")
    rng = np.random.default_rng(5)
    ref_pts = oracle_query_points(tm, 16, w.philox_seed, 0)
    extra = np.concatenate([rng.uniform(0, 1, (5000, 2)), sm[0][:500], tm[0],
                            0.5 * (sm[0][sm[1][:300, 0]] + sm[0][sm[1][:300, 1]]),
                            [[0.0, 0.0], [1.0, 1.0], [1.0, 0.3], [0.3, 0.0]]])
    pts = np.concatenate([ref_pts.T, extra]).T.copy()
    S = ft.Source(*sm, sv)
    dp = torch.as_tensor(pts, device="cuda")
    ids = torch.empty(pts.shape[1], dtype=torch.int32, device="cuda")
    vals = S.eval(dp, ids=ids).cpu().numpy()
    ids = ids.cpu().numpy()
    assert S.take_out_of_domain() == 0
    o = P1Source(*sm, sv)
    oid, omu, ood = o.locate(pts.T)
    fd = o.face_distance(oid, omu)
    away = fd > 1e-12
    log(f"away-from-face points: {away.sum()} of {away.size}")
    assert away.sum() > 0.9 * away.size
    assert np.array_equal(ids[away], oid[away])
    ovals = o.evaluate_at(oid, omu)
    assert np.abs(vals - ovals).max() < 1e-13
    S.close()


def test_source_out_of_domain_counted():
    _, sm = _small_2d()
    sv = fields.evaluate("affine", np, sm[0])
    S = ft.Source(*sm, sv)
    pts = np.array([[0.5, 0.5], [1.5, 0.5], [-0.2, 0.9], [0.25, 1.0 + 1e-13], [0.7, 0.1]]).T.copy()
    out = S.eval(torch.as_tensor(pts, device="cuda")).cpu().numpy()
    assert S.take_out_of_domain() == 2
    assert S.take_out_of_domain() == 0
    inside = [0, 3, 4]
    assert np.abs(out[0, inside] - fields.evaluate("affine", np, pts.T[inside])[0]).max() < 1e-13
    S.close()


@pytest.mark.parametrize("dim,F,dtype", [(2, 5, "f64"), (3, 64, "f32"), (3, 17, "f64"), (2, 40, "f32")])
def test_many_field_eval_matches_oracle(dim, F, dtype):
    """Several fields per source (the lanes-over-fields evaluation): element ids,
    values and the out-of-domain count against the oracle, with a ragged last
    wave and points outside the domain."""
    tm, sm = _small_2d() if dim == 2 else _small_3d()
    rng = np.random.default_rng(40 + F)
    sv = rng.standard_normal((F, sm[0].shape[0]))
    inside = np.concatenate([oracle_query_points(tm, 7, 21, 0).T, rng.uniform(0, 1, (777, dim)), sm[0][:50]])
    outside = np.concatenate([rng.uniform(1.2, 1.5, (5, dim)), -rng.uniform(0.2, 0.4, (4, dim))])
    pts = np.concatenate([inside, outside]).T.copy()
    log(f"many-field eval dim={dim} F={F} {dtype}: {pts.shape[1]} points")
    S = ft.Source(*sm, sv)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    dp = torch.as_tensor(pts, device="cuda").to(tdt)
    ids = torch.empty(pts.shape[1], dtype=torch.int32, device="cuda")
    vals = S.eval(dp, ids=ids).double().cpu().numpy()
    ids = ids.cpu().numpy()
    assert vals.shape == (F, pts.shape[1])
    assert S.take_out_of_domain() == outside.shape[0]
    o = P1Source(*sm, sv)
    qp = dp.double().cpu().numpy().T   # the points the kernel saw (binary32 rounded for f32)
    oid, omu, ood = o.locate(qp)
    n_in = inside.shape[0]
    away = o.face_distance(oid[:n_in], omu[:n_in]) > 1e-12
    assert away.sum() > 0.9 * n_in
    assert np.array_equal(ids[:n_in][away], oid[:n_in][away])
    ovals = o.evaluate_at(oid[:n_in], omu[:n_in])
    tol = 1e-13 if dtype == "f64" else 1e-6
    scale = np.abs(ovals).max()
    assert np.abs(vals[:, :n_in] - ovals).max() <= tol * scale
    S.close()


@pytest.mark.parametrize("bins", [None, (7, 5), (64, 64)])
def test_source_bins_do_not_change_results(bins):
    tm, sm = _small_2d()
    sv = fields.evaluate("front_2d", np, sm[0])
    pts = oracle_query_points(tm, 9, 11, 0)
    S = ft.Source(*sm, sv, bins=bins)
    ids = torch.empty(pts.shape[1], dtype=torch.int32, device="cuda")
    vals = S.eval(torch.as_tensor(pts, device="cuda"), ids=ids).cpu().numpy()
    o = P1Source(*sm, sv)
    oid, omu, _ = o.locate(pts.T)
    away = o.face_distance(oid, omu) > 1e-12
    assert np.array_equal(ids.cpu().numpy()[away], oid[away])
    assert np.abs(vals - o.evaluate_at(oid, omu)).max() < 1e-13
    S.close()


# ---------------------------------------------------------------- whole transfer
def test_transfer_parity_tri2d_4k(c1):
    w, tm, sm, sv = c1
    log("transfer tri2d_4k FP64")
    g = gpu_transfer(tm, sm, sv, w.samples_per_elem, w.alpha, w.philox_seed, 0)
    o = oracle_transfer(tm, sm, sv, w.samples_per_elem, w.alpha, w.philox_seed, 0)
    log(f"oracle {o['seconds']:.1f}s; GPU iters {g['reports'][0]['iters']}")
    assert g["status"] == ft.FT_OK
    assert rel_l2(g["b"], o["b"]) < 1e-12
    assert rel_l2(g["x"], o["x"]) < 1e-12
    rep, orep = g["reports"][0], o["report"][0]
    assert abs(rep["sum_b"] - orep["sum_b"]) <= 1e-13 * abs(orep["sum_b"])
    assert abs(rep["int_x"] - orep["int_x"]) <= 1e-12 * abs(orep["int_x"])
    assert rep["cons_defect"] < 1e-13
    assert rep["rel_resid"] < 1e-13
    assert g["ood"] == 0


@pytest.mark.parametrize("N", [1, 3, 20, 64, 100])
def test_transfer_parity_group_sizes(N):
    tm, sm = _small_2d()
    sv = fields.evaluate("front_2d", np, sm[0])
    log(f"transfer 2D N={N}")
    g = gpu_transfer(tm, sm, sv, N, 1.0, 99, 5)
    o = oracle_transfer(tm, sm, sv, N, 1.0, 99, 5)
    assert rel_l2(g["b"], o["b"]) < 1e-12
    assert rel_l2(g["x"], o["x"]) < 1e-12


@pytest.mark.parametrize("alpha", [0.0, 0.5, 1.0])
def test_transfer_parity_alpha(alpha):
    tm, sm = _small_2d()
    sv = fields.evaluate("paper_f3", np, sm[0])
    g = gpu_transfer(tm, sm, sv, 20, alpha, 3, 1)
    o = oracle_transfer(tm, sm, sv, 20, alpha, 3, 1)
    assert rel_l2(g["b"], o["b"]) < 1e-12
    assert rel_l2(g["x"], o["x"]) < 1e-12


def test_transfer_parity_3d():
    tm, sm = _small_3d()
    sv = fields.evaluate("gaussian_bumps_3d", np, sm[0])
    log("transfer 3D FP64")
    g = gpu_transfer(tm, sm, sv, 16, 1.0, 21, 2)
    o = oracle_transfer(tm, sm, sv, 16, 1.0, 21, 2)
    assert rel_l2(g["b"], o["b"]) < 1e-12
    assert rel_l2(g["x"], o["x"]) < 1e-12
    assert g["reports"][0]["cons_defect"] < 1e-13


def test_transfer_parity_multi_field_3d():
    tm, sm = _small_3d()
    modes = fields.fourier_modes(seed=13, n_fields=5, n_modes=4, kmax=2)
    sv = fields.fourier_fields_3d(np, sm[0][:, 0], sm[0][:, 1], sm[0][:, 2], modes)
    g = gpu_transfer(tm, sm, sv, 12, 1.0, 8, 0)
    o = oracle_transfer(tm, sm, sv, 12, 1.0, 8, 0)
    assert g["x"].shape == (5, tm[0].shape[0])
    for f in range(5):
        assert rel_l2(g["b"][f], o["b"][f]) < 1e-12
        assert rel_l2(g["x"][f], o["x"][f]) < 1e-12


def test_transfer_black_box_analytic():
    """A point-query black box evaluated by torch on the device (a stand-in for a surrogate model)."""
    tm, _ = _small_2d()

    def bb(points):
        return fields.smooth_2d(torch, points[0], points[1])[None, :]

    g = gpu_transfer(tm, None, None, 32, 1.0, 17, 4, black_box=bb)
    o = oracle_transfer(tm, None, None, 32, 1.0, 17, 4, query=lambda p: fields.evaluate("smooth_2d", np, p))
    assert rel_l2(g["b"], o["b"]) < 1e-12
    assert rel_l2(g["x"], o["x"]) < 1e-12


def test_affine_source_reproduced_exactly():
    tm, sm = _small_3d()
    sv = fields.evaluate("affine", np, sm[0])
    g = gpu_transfer(tm, sm, sv, 8, 1.0, 1, 0)
    assert rel_l2(g["x"], fields.evaluate("affine", np, tm[0])) < 1e-13
    assert g["reports"][0]["iters"] == 0


def test_mass_matrix_product_matches_oracle():
    """alpha = 1 and values equal to the P1 interpolant of random nodal g: b = M g."""
    tm, _ = _small_2d()
    tc, tconn = tm
    rng = np.random.default_rng(4)
    gn = rng.standard_normal(tc.shape[0])
    N = 6
    T = ft.Target(tc, tconn)
    cfg = ft.SampleCfg(N, 1, 1.0, 12, 0, ft.FT_F64)
    pts = T.sample_points(cfg).cpu().numpy()
    n, E = tc.shape[0], tconn.shape[0]
    X = pts[:, n:].T.reshape(E, N, 2)
    from oracle.source import barycentric_cramer
    lam = barycentric_cramer(tc[tconn][:, None], X)            # (E, N, 3)
    y = np.concatenate([gn, np.einsum("ejk,ek->ej", lam, gn[tconn]).ravel()])
    T.consume(cfg, torch.as_tensor(y[None, :], device="cuda"))
    res = T.project(1)
    M = geometry.mass_matrix(tc, tconn)
    ref = M @ gn
    assert np.abs(res.b.cpu().numpy()[0] - ref).max() < 1e-14 * np.abs(ref).max() * 10
    assert T.info.nnz == M.nnz
    T.close()


def test_fp32_form_within_1e5(c1):
    w, tm, sm, sv = c1
    log("transfer tri2d_4k FP32 form")
    g = gpu_transfer(tm, sm, sv, w.samples_per_elem, w.alpha, w.philox_seed, 0, precision=ft.FT_F32)
    o = oracle_transfer(tm, sm, sv, w.samples_per_elem, w.alpha, w.philox_seed, 0)
    ex, eb = rel_l2(g["x"], o["x"]), rel_l2(g["b"], o["b"])
    log(f"FP32 form: rel l2 x {ex:.2e}, b {eb:.2e}")
    assert ex < 1e-5 and eb < 1e-5
    rep, orep = g["reports"][0], o["report"][0]
    assert abs(rep["sum_b"] - orep["sum_b"]) <= 1e-6 * abs(orep["sum_b"])
    assert abs(rep["int_x"] - orep["int_x"]) <= 1e-6 * abs(orep["int_x"])


def test_bitwise_deterministic(c1):
    w, tm, sm, sv = c1
    a = gpu_transfer(tm, sm, sv, 64, 1.0, 5, 0)
    b = gpu_transfer(tm, sm, sv, 64, 1.0, 5, 0)
    assert np.array_equal(a["x"], b["x"]) and np.array_equal(a["b"], b["b"])
    c = gpu_transfer(tm, sm, sv, 64, 1.0, 5, 1)
    assert not np.array_equal(a["x"], c["x"])


def test_solver_launch_hint_keeps_results(c1):
    """A target launches as many CG iterations as its previous solve of the same
    kind needed before its first host check; the launches after convergence
    must leave x, b and the iteration count as a fresh target computes them."""
    w, tm, sm, sv = c1
    T, T2, S = ft.Target(*tm), ft.Target(*tm), ft.Source(*sm, sv)
    cfg = ft.SampleCfg(64, 1, 1.0, 5, 0, ft.FT_F64)
    pts = T.sample_points(cfg)
    T2.sample_points(cfg)
    vals = S.eval_query_list(pts, tm[0].shape[0])
    T.consume(cfg, vals)
    T2.consume(cfg, vals)
    hard = T.project(1, rtol=1e-14)
    hx, hit = hard.x.clone(), hard.reports[0]["iters"]
    easy = T.project(1, rtol=1e-6)   # first launch chunk longer than this solve needs
    fresh = T2.project(1, rtol=1e-6)
    assert easy.reports[0]["iters"] == fresh.reports[0]["iters"] < hit
    assert torch.equal(easy.x, fresh.x) and torch.equal(easy.b, fresh.b)
    again = T.project(1, rtol=1e-14)
    assert torch.equal(again.x, hx) and again.reports[0]["iters"] == hit
    m1 = T.project(1, refine_steps=3).x.clone()   # binary32 inner solves, then with their hint
    m2 = T.project(1, refine_steps=3).x
    assert torch.equal(m1, m2)
    for h in (T, T2, S):
        h.close()


# ---------------------------------------------------------------- error paths
def test_call_order_and_status_errors():
    tm, sm = _small_2d()
    T = ft.Target(*tm)
    x = torch.empty((1, tm[0].shape[0]), dtype=torch.float64, device="cuda")
    with pytest.raises(ft.FtError) as e:
        ft.ft_project(T.handle, ft.SolveCfg(1e-14, 100), x.data_ptr(), None, 1, ft.current_stream())
    assert e.value.status == ft.FT_E_ORDER
    cfg = ft.SampleCfg(4, 1, 1.0, 1, 0, ft.FT_F64)
    vals = torch.zeros((1, T.query_count(4)), dtype=torch.float64, device="cuda")
    with pytest.raises(ft.FtError) as e:
        T.consume(cfg, vals)                       # no sample_points yet
    assert e.value.status == ft.FT_E_ORDER
    T.sample_points(cfg)
    bad = ft.SampleCfg(4, 1, 1.0, 2, 0, ft.FT_F64)  # different seed than the samples
    with pytest.raises(ft.FtError) as e:
        T.consume(bad, vals)
    assert e.value.status == ft.FT_E_ORDER
    # non-finite values are counted and reported
    vals[0, 100] = float("nan")
    vals[0, 7] = float("inf")
    T.consume(cfg, vals)
    res = T.project(1)
    assert res.status == ft.FT_E_NONFINITE and res.reports[0]["n_nonfinite"] == 2
    # non-convergence
    sv = fields.evaluate("front_2d", np, sm[0])
    S = ft.Source(*sm, sv)
    pts = T.sample_points(cfg)
    T.consume(cfg, S.eval(pts))
    res = T.project(1, max_iter=1)
    assert res.status == ft.FT_E_NOCONV and res.reports[0]["iters"] == 1
    res = T.project(1)
    assert res.status == ft.FT_OK
    T.close()
    S.close()


@pytest.mark.parametrize("dim,N", [(2, 5), (3, 3), (2, 300), (3, 64)])
def test_single_element_target(dim, N):
    """The smallest target (one element: grids of one block, one reduction
    block, a partial wave) through the black-box and the fused routes."""
    if dim == 2:
        tm = (np.array([[0.1, 0.1], [0.9, 0.2], [0.3, 0.8]]), np.array([[0, 1, 2]], dtype=np.int32))
        sm = _small_2d()[1]
        sv = fields.evaluate("front_2d", np, sm[0])
    else:
        tm = (np.array([[0.1, 0.1, 0.1], [0.9, 0.2, 0.1], [0.2, 0.8, 0.2], [0.2, 0.3, 0.9]]),
              np.array([[0, 1, 2, 3]], dtype=np.int32))
        sm = _small_3d()[1]
        sv = fields.evaluate("gaussian_bumps_3d", np, sm[0])
    g = gpu_transfer(tm, sm, sv, N, 1.0, 77, 0)
    o = oracle_transfer(tm, sm, sv, N, 1.0, 77, 0)
    assert g["status"] == ft.FT_OK
    assert rel_l2(g["b"], o["b"]) < 1e-12 and rel_l2(g["x"], o["x"]) < 1e-12
    T, S = ft.Target(*tm), ft.Source(*sm, sv)
    T.transfer_from(S, ft.SampleCfg(N, 1, 1.0, 77, 0, ft.FT_F64))
    r = T.project(1)
    assert rel_l2(r.x.cpu().numpy(), o["x"]) < 1e-12
    T.close()
    S.close()


def test_empty_point_ranges():
    """Evaluating no points is a no-op that leaves the output untouched."""
    tm, sm = _small_2d()
    S = ft.Source(*sm, fields.evaluate("smooth_2d", np, sm[0]))
    pts = torch.zeros((2, 10), dtype=torch.float64, device="cuda")
    out = torch.full((1, 10), 7.0, dtype=torch.float64, device="cuda")
    S.eval(pts, out=out, start=3, count=0)
    torch.cuda.synchronize()
    assert bool((out == 7.0).all())
    assert S.take_out_of_domain() == 0
    S.close()


def test_degenerate_and_out_of_range_meshes_rejected():
    tc = np.array([[0.0, 0.0], [1.0, 0.0], [2.0, 0.0], [0.0, 1.0]])
    with pytest.raises(ft.FtError) as e:
        ft.Target(tc, np.array([[0, 1, 2]], dtype=np.int32))      # collinear
    assert e.value.status == ft.FT_E_MESH
    with pytest.raises(ft.FtError) as e:
        ft.Target(tc, np.array([[0, 1, 9]], dtype=np.int32))      # id out of range
    assert e.value.status == ft.FT_E_MESH
    with pytest.raises(ft.FtError) as e:
        ft.Target(tc, np.array([[0, 1, 3]], dtype=np.int32))      # node 2 unused
    assert e.value.status == ft.FT_E_MESH
    inv = ft.Target(tc[[0, 1, 3]], np.array([[0, 2, 1]], dtype=np.int32))   # clockwise: accepted
    assert inv.info.n_inverted == 1
    inv.close()


def test_allocation_cap_reports_oom(monkeypatch):
    tm, _ = _small_2d()
    monkeypatch.setenv("FT_MAX_BYTES", "1000")
    with pytest.raises(ft.FtError) as e:
        ft.Target(*tm)
    assert e.value.status == ft.FT_E_OOM
    monkeypatch.delenv("FT_MAX_BYTES")
    T = ft.Target(*tm)
    T.close()


# ---------------------------------------------------------------- fused built-in route
@pytest.mark.parametrize("dim,N", [(2, 64), (2, 20), (3, 16), (2, 256)])
def test_fused_route_matches_unfused_and_oracle(dim, N):
    tm, sm = _small_2d() if dim == 2 else _small_3d()
    name = "front_2d" if dim == 2 else "gaussian_bumps_3d"
    sv = fields.evaluate(name, np, sm[0])
    log(f"fused route dim={dim} N={N}")
    ref = gpu_transfer(tm, sm, sv, N, 1.0, 77, 1)
    T = ft.Target(*tm)
    S = ft.Source(*sm, sv)
    cfg = ft.SampleCfg(N, 1, 1.0, 77, 1, ft.FT_F64)
    T.transfer_from(S, cfg)
    res = T.project(1)
    x, b = res.x.cpu().numpy(), res.b.cpu().numpy()
    assert rel_l2(x, ref["x"]) < 1e-14 and rel_l2(b, ref["b"]) < 1e-14
    o = oracle_transfer(tm, sm, sv, N, 1.0, 77, 1)
    assert rel_l2(b, o["b"]) < 1e-12 and rel_l2(x, o["x"]) < 1e-12
    assert S.take_out_of_domain() == 0
    with pytest.raises(ft.FtError) as e:   # the matrix-core forms have no fused route
        T.transfer_from(S, ft.SampleCfg(N, 1, 1.0, 77, 1, ft.FT_SPLIT_BF16))
    assert e.value.status == ft.FT_E_UNSUPPORTED
    T.close()
    S.close()


# ---------------------------------------------------------------- split matrix-core form
@pytest.mark.parametrize("prec", [ft.FT_SPLIT_F16, ft.FT_SPLIT_BF16])
@pytest.mark.parametrize("dim,F,N", [(3, 20, 16), (3, 64, 128), (2, 9, 40), (2, 33, 256), (3, 17, 200)])
def test_split_matrix_core_form_within_1e5(prec, dim, F, N):
    """Many fields at once through the split-product MFMA element sums."""
    tm, sm = _small_2d() if dim == 2 else _small_3d()
    modes = fields.fourier_modes(seed=13 + F, n_fields=F, n_modes=4, kmax=2)
    if dim == 3:
        sv = fields.fourier_fields_3d(np, sm[0][:, 0], sm[0][:, 1], sm[0][:, 2], modes)
    else:
        sv = fields.fourier_fields_3d(np, sm[0][:, 0], sm[0][:, 1], 0.25 + 0 * sm[0][:, 0], modes)
    log(f"split form prec={prec} dim={dim} F={F} N={N}")
    g = gpu_transfer(tm, sm, sv, N, 1.0, 40 + F, 1, precision=prec)
    o = oracle_transfer(tm, sm, sv, N, 1.0, 40 + F, 1)
    assert g["status"] == ft.FT_OK
    assert g["x"].shape == (F, tm[0].shape[0])
    ex = max(rel_l2(g["x"][f], o["x"][f]) for f in range(F))
    eb = max(rel_l2(g["b"][f], o["b"][f]) for f in range(F))
    log(f"worst field: rel l2 x {ex:.2e}, b {eb:.2e}")
    assert ex < 1e-5 and eb < 1e-5
    # Fourier fields have integrals near zero (sum b is a cancellation of O(1)
    # terms), so the conservation error is measured against sum |b|.
    for f in range(F):
        rep, orep = g["reports"][f], o["report"][f]
        mass = np.abs(o["b"][f]).sum()
        assert abs(rep["sum_b"] - orep["sum_b"]) <= 1e-6 * mass
        assert abs(rep["int_x"] - rep["sum_b"]) <= 1e-12 * mass


@pytest.mark.parametrize("dim,N", [(2, 256), (2, 37), (3, 128)])
def test_query_list_launch_matches_plain_eval(dim, N):
    """ft_source_eval_queries (node and sample blocks in separate wavefronts) gives
    bitwise the values and ids of ft_source_eval over the same points."""
    tm, sm = _small_2d() if dim == 2 else _small_3d()
    sv = fields.evaluate("front_2d" if dim == 2 else "gaussian_bumps_3d", np, sm[0])
    T = ft.Target(*tm)
    S = ft.Source(*sm, sv)
    cfg = ft.SampleCfg(N, 1, 1.0, 77, 0, ft.FT_F64)
    pts = T.sample_points(cfg)
    n = tm[0].shape[0]
    Q = pts.shape[1]
    ids_a = torch.full((Q,), -5, dtype=torch.int32, device="cuda")
    ids_b = torch.full((Q,), -6, dtype=torch.int32, device="cuda")
    a = S.eval_query_list(pts, n, ids=ids_a)
    b = S.eval(pts, ids=ids_b)
    for head in (0, 1, 255, 256, Q - 3, Q):
        c = S.eval_query_list(pts, head)
        assert torch.equal(c, b), head
    assert torch.equal(a, b) and torch.equal(ids_a, ids_b)
    assert int((ids_a < 0).sum()) == 0
    T.close()
    S.close()


# ---------------------------------------------------------------- mixed-precision solve
def test_refinement_solve_matches_binary64_solve(c1):
    """binary32 inner PCG + binary64 residual refinement reaches the binary64
    solution of the same M x = b (FP32-form load vector)."""
    w, tm, sm, sv = c1
    tc, tconn = tm
    T = ft.Target(tc, tconn)
    S = ft.Source(*sm, sv)
    cfg = ft.SampleCfg(w.samples_per_elem, 1, w.alpha, w.philox_seed, 0, ft.FT_F32)
    pts = T.sample_points(cfg)
    vals = S.eval_query_list(pts, tc.shape[0])
    T.consume(cfg, vals)
    ref = T.project(1, rtol=1e-14)
    mixed = T.project(1, rtol=1e-14, refine_steps=4)
    torch.cuda.synchronize()
    rep = mixed.reports[0]
    log(f"refinement: {rep['iters']} inner iterations, rel resid {rep['rel_resid']:.2e}")
    assert mixed.status == ft.FT_OK
    assert rep["rel_resid"] < 1e-13
    assert torch.equal(mixed.b, ref.b)
    assert rel_l2(mixed.x.cpu().numpy(), ref.x.cpu().numpy()) < 1e-13
    assert rep["cons_defect"] < 1e-13
    one = T.project(1, rtol=1e-14, refine_steps=1)
    assert one.status == ft.FT_E_NOCONV            # one binary32 step gains about six digits only
    assert one.reports[0]["rel_resid"] < 1e-4
    T.close()
    S.close()


def test_bin_autotune_keeps_results(c1):
    """The autotuner only changes the bin grid: values and ids stay those of the rule."""
    w, tm, sm, sv = c1
    S = ft.Source(*sm, sv)
    pts = torch.as_tensor(oracle_query_points(tm, 16, w.philox_seed, 0), device="cuda")
    n = tm[0].shape[0]
    ids0 = torch.empty(pts.shape[1], dtype=torch.int32, device="cuda")
    v0 = S.eval_query_list(pts, n, ids=ids0).clone()
    chosen = S.autotune(pts[:, : n + 4000].contiguous(), n, [8, 24, 48, 97, 160])
    log(f"autotune chose bins {chosen}")
    assert chosen[0] in (8, 24, 48, 97, 160) or chosen[1] in (8, 24, 48, 97, 160)
    assert list(S.info.bins)[:2] == chosen[:2]
    assert S.take_out_of_domain() == 0
    ids1 = torch.empty_like(ids0)
    v1 = S.eval_query_list(pts, n, ids=ids1)
    assert torch.equal(v0, v1) and torch.equal(ids0, ids1)
    S.close()
