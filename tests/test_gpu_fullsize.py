"""Parity at the benchmark's full size (1M target triangles, 4M source
triangles, 256 samples per element, 512x512 bins), in the launch
configuration bench.py times.

The oracle cannot redo 2.6e8 point queries in a test, so it checks sampled
outputs it can compute one by one (the samples of chosen elements, the load
vector at chosen nodes, with every element around them) plus properties that
hold at any size (the solve against the oracle's own mass matrix and CG, the
conservation identity, run-to-run determinism).
"""
import math

import numpy as np
import pytest

from gpu_cases import log
from oracle import cvmc, geometry
from oracle.source import P1Source
from paper_2603_00538_amd import ft
from workloads import configs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

W = configs.WORKLOADS["tri2d_1m"]


@pytest.fixture(scope="module")
def case():
    log("tri2d_1m: meshes")
    tm = configs.build_mesh(W.target)
    sm = configs.build_mesh(W.source)
    sv = configs.source_nodal_values(W, sm[0])
    log("tri2d_1m: oracle source (k-d tree over 4M centroids)")
    osrc = P1Source(*sm, sv)
    return tm, sm, sv, osrc


def _run(tm, sm, sv, precision):
    tc, tconn = tm
    T = ft.Target(tc, tconn)
    S = ft.Source(*sm, sv, bins=W.bins[:2])
    cfg = ft.SampleCfg(W.samples_per_elem, 1, W.alpha, W.philox_seed, 0, precision)
    pts = T.sample_points(cfg)
    ids = torch.empty(pts.shape[1], dtype=torch.int32, device="cuda")
    vals = S.eval_query_list(pts, tc.shape[0], ids=ids)
    T.consume(cfg, vals)
    res = T.project(1, rtol=W.rtol)
    torch.cuda.synchronize()
    return T, S, cfg, pts, vals, ids, res


def _sample_sets(tm):
    tc, tconn = tm
    rng = np.random.default_rng(2024)
    E, n = tconn.shape[0], tc.shape[0]
    elems = np.unique(np.concatenate([rng.choice(E, 250, replace=False), [0, 1, E - 2, E - 1]]))
    nodes = np.unique(np.concatenate([rng.choice(n, 150, replace=False), [0, n - 1, 707, n - 708]]))
    return elems, nodes


def _oracle_b_at(tm, osrc, g, nodes):
    """Oracle b at `nodes`: exact control part plus the MC residual of every element touching them."""
    tc, tconn = tm
    tconn64 = np.asarray(tconn, dtype=np.int64)
    b_g = cvmc.control_load(tc, tconn64, g, W.alpha)
    touching = np.unique(np.nonzero(np.isin(tconn64, nodes).any(axis=1))[0])
    lam, X = cvmc.query_points(tc, tconn64, W.samples_per_elem, W.philox_seed, 0, touching)
    y = osrc(X.reshape(-1, 2)).reshape(1, touching.size, W.samples_per_elem)
    beta = cvmc.element_loads(tc, tconn64, g, y, lam, W.alpha, touching)
    b_res = np.zeros(tc.shape[0])
    # assemble in ascending (element, local vertex) order, as step 6 does
    np.add.at(b_res, tconn64[touching].ravel(), beta[0].ravel())
    return (b_g[0] + b_res)[nodes]


@pytest.fixture(scope="module")
def fp64(case):
    tm, sm, sv, osrc = case
    log("tri2d_1m: GPU transfer FP64")
    T, S, cfg, pts, vals, ids, res = _run(tm, sm, sv, ft.FT_F64)
    yield T, S, cfg, pts, vals, ids, res
    T.close()
    S.close()


def test_fullsize_samples_and_source_values(case, fp64):
    tm, sm, sv, osrc = case
    T, S, cfg, pts, vals, ids, res = fp64
    tc, tconn = tm
    n, N = tc.shape[0], W.samples_per_elem
    elems, nodes = _sample_sets(tm)
    log(f"checking {elems.size} elements x {N} samples and {nodes.size} nodes")
    cols = np.concatenate([n + t * N + np.arange(N) for t in elems])
    gp = pts[:, torch.as_tensor(cols, device="cuda")].cpu().numpy().T
    lam, X = cvmc.query_points(tc, np.asarray(tconn, dtype=np.int64), N, W.philox_seed, 0, elems)
    X = X.reshape(-1, 2)
    assert np.abs(gp - X).max() < 2e-15
    qcols = np.concatenate([nodes, cols])
    qp = np.concatenate([tc[nodes], X])
    oid, omu, ood = osrc.locate(qp)
    gid = ids[torch.as_tensor(qcols, device="cuda")].cpu().numpy()
    gv = vals[0, torch.as_tensor(qcols, device="cuda")].cpu().numpy()
    away = osrc.face_distance(oid, omu) > 1e-12
    log(f"ids compared away from faces: {away.sum()} of {away.size}")
    assert away.sum() > 0.95 * away.size
    assert np.array_equal(gid[away], oid[away])
    assert np.abs(gv - osrc.evaluate_at(oid, omu)[0]).max() < 1e-13
    assert S.take_out_of_domain() == 0


def test_fullsize_load_vector_at_sampled_nodes(case, fp64):
    tm, sm, sv, osrc = case
    T, S, cfg, pts, vals, ids, res = fp64
    tc, _ = tm
    _, nodes = _sample_sets(tm)
    log("oracle control at all 501k target nodes")
    g = np.atleast_2d(osrc(tc))
    ref = _oracle_b_at(tm, osrc, g, nodes)
    got = res.b.cpu().numpy()[0, nodes]
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    log(f"sampled-node b rel l2 {err:.2e}")
    assert err < 1e-12


def test_fullsize_solution_and_conservation(case, fp64):
    tm, _, _, _ = case
    T, S, cfg, pts, vals, ids, res = fp64
    tc, tconn = tm
    b = res.b.cpu().numpy()[0]
    x = res.x.cpu().numpy()[0]
    M = geometry.mass_matrix(tc, tconn)
    rr = np.linalg.norm(b - M @ x) / np.linalg.norm(b)
    log(f"residual against the oracle's M: {rr:.2e}; CG iters {res.reports[0]['iters']}")
    assert rr < 1e-13
    x_or = cvmc.jacobi_cg(M, b, 1e-15)
    assert cvmc.rel_l2(x, x_or) < 1e-12
    m = geometry.lumped_mass(tc, tconn)
    rep = res.reports[0]
    assert abs(rep["sum_b"] - math.fsum(b)) <= 1e-13 * abs(math.fsum(b))
    assert abs(rep["int_x"] - math.fsum(m * x)) <= 1e-13 * abs(math.fsum(m * x))
    assert rep["cons_defect"] < 1e-13


def test_fullsize_rerun_is_bitwise_identical(case, fp64):
    T, S, cfg, pts, vals, ids, res = fp64
    x0 = res.x.clone()
    S.eval_query_list(pts, T.info.n_nodes, out=vals)
    T.consume(cfg, vals)
    again = T.project(1, rtol=W.rtol)
    assert torch.equal(again.x, x0)


def test_fullsize_fp32_form(case, fp64):
    """The binary32 form at full size: its load vector at the sampled nodes
    against the binary64 oracle; its binary64 PCG solution and its binary32
    PCG + binary64 refinement solution against the oracle's own CG solve of
    the same load vector; conservation."""
    tm, sm, sv, osrc = case
    tc, tconn = tm
    x64 = fp64[6].x.cpu().numpy()[0]
    log("tri2d_1m: GPU transfer FP32 form")
    T, S, cfg, pts, vals, ids, res = _run(tm, sm, sv, ft.FT_F32)
    x32 = res.x.cpu().numpy()[0]
    b32 = res.b.cpu().numpy()[0]
    mixed = T.project(1, rtol=W.rtol, refine_steps=4)
    torch.cuda.synchronize()
    xr = mixed.x.cpu().numpy()[0]
    assert mixed.status == ft.FT_OK and torch.equal(mixed.b, res.b)
    _, nodes = _sample_sets(tm)
    g = np.atleast_2d(osrc(tc))
    ref = _oracle_b_at(tm, osrc, g, nodes)
    eb = np.linalg.norm(b32[nodes] - ref) / np.linalg.norm(ref)
    M = geometry.mass_matrix(tc, tconn)
    x_or = cvmc.jacobi_cg(M, b32, 1e-15)
    es, er = cvmc.rel_l2(x32, x_or), cvmc.rel_l2(xr, x_or)
    log(f"FP32 form: sampled b rel l2 {eb:.2e}; x vs oracle CG of the same b {es:.2e} (refined {er:.2e}); "
        f"x vs binary64 route {cvmc.rel_l2(x32, x64):.2e}")
    assert eb < 1e-5
    assert es < 1e-12 and er < 1e-12
    assert cvmc.rel_l2(x32, x64) < 1e-5
    m = geometry.lumped_mass(tc, tconn)
    for r, x in ((res.reports[0], x32), (mixed.reports[0], xr)):
        assert abs(r["int_x"] - math.fsum(m * x)) <= 1e-13 * abs(r["int_x"])
        assert r["cons_defect"] < 1e-13
    r64 = fp64[6].reports[0]
    assert abs(res.reports[0]["sum_b"] - r64["sum_b"]) <= 1e-6 * abs(r64["sum_b"])
    T.close()
    S.close()
