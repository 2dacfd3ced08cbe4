"""Parity at the 3D workload's full size (2,058,000 target tetrahedra, 7,986,000
source tetrahedra, 128 samples per element, 108^3 bins: the grid the bin
autotuner picks for it), in the launch configuration bench.py times.

A whole-mesh oracle source over 8M tetrahedra takes minutes to build, so the
checks are regional: in three boxes of the domain the oracle source is built
on the source elements that can hold any sample of the target elements there
(every source element whose bounding box meets the box grown by the largest
target element), which leaves its localization exact for those samples.  It
checks the emitted samples, the element ids away from faces, the values, and
the load vector at the nodes whose incident elements all lie in the box.

The binary32 form (binary32 points and values, binary32 inner PCG with
binary64 refinement steps) is run on the same workload and checked against
the same binary64 oracle load vectors in the boxes (1e-5), and its whole
solution against the oracle's own CG solve of the same load vector.
"""
import numpy as np
import pytest

from gpu_cases import log
from oracle import cvmc, geometry
from oracle.source import P1Source
from paper_2603_00538_amd import ft
from workloads import configs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

W = configs.WORKLOADS["tet3d_2m"]
BINS = (108, 108, 108)
CENTERS = [(0.21, 0.33, 0.47), (0.52, 0.81, 0.18), (0.88, 0.12, 0.66)]
HALF = 0.035   # box half-width (a target element spans about 1/71): about 750 elements


@pytest.fixture(scope="module")
def run3d():
    log("tet3d_2m: meshes")
    tm = configs.build_mesh(W.target)
    sm = configs.build_mesh(W.source)
    sv = configs.source_nodal_values(W, sm[0])
    tc, tconn = tm
    log("tet3d_2m: GPU transfer FP64")
    T = ft.Target(tc, tconn)
    S = ft.Source(*sm, sv, bins=BINS)
    cfg = ft.SampleCfg(W.samples_per_elem, 1, W.alpha, W.philox_seed, 0, ft.FT_F64)
    pts = T.sample_points(cfg)
    ids = torch.empty(pts.shape[1], dtype=torch.int32, device="cuda")
    vals = S.eval_query_list(pts, tc.shape[0], ids=ids)
    T.consume(cfg, vals)
    res = T.project(1, rtol=W.rtol)
    torch.cuda.synchronize()
    assert S.take_out_of_domain() == 0
    yield tm, sm, sv, pts, vals, ids, res
    T.close()
    S.close()


def _region(tm, sm, sv, center):
    """Target elements with their centroid in the box, and an oracle source on
    every source element that can hold one of their samples."""
    tc, tconn = tm
    sc, sconn = sm
    c = np.asarray(center)
    tv = tc[tconn]
    elems = np.nonzero(np.all(np.abs(tv.mean(axis=1) - c) <= HALF, axis=1))[0]
    grow = HALF + float((tv.max(axis=1) - tv.min(axis=1)).max())
    sv_ = sc[sconn]
    near = np.nonzero(np.all((sv_.min(axis=1) <= c + grow) & (sv_.max(axis=1) >= c - grow), axis=1))[0]
    return elems, near, P1Source(sc, sconn[near], sv)


@pytest.fixture(scope="module")
def regions(run3d):
    """Per box: its target elements, the restricted oracle source, the oracle's
    samples (lambda, X) and their localization."""
    tm, sm, sv = run3d[:3]
    tc, tconn = tm
    out = []
    for k, c in enumerate(CENTERS):
        elems, near, osrc = _region(tm, sm, sv, c)
        lam, X = cvmc.query_points(tc, np.asarray(tconn, dtype=np.int64), W.samples_per_elem, W.philox_seed, 0,
                                   elems)
        X = X.reshape(-1, 3)
        oid, omu, ood = osrc.locate(X)
        log(f"box {k}: {elems.size} target elements, {near.size} source elements, {X.shape[0]} samples")
        out.append((elems, near, osrc, lam, X, oid, omu, ood))
    return out


@pytest.mark.parametrize("k", range(len(CENTERS)))
def test_fullsize_3d_samples_ids_values(run3d, regions, k):
    tm, sm, sv, pts, vals, ids, res = run3d
    elems, near, osrc, lam, X, oid, omu, ood = regions[k]
    tc, tconn = tm
    n, N = tc.shape[0], W.samples_per_elem
    assert elems.size > 200
    cols = (n + elems[:, None] * N + np.arange(N)[None, :]).ravel()
    gcols = torch.as_tensor(cols, device="cuda")
    gp = pts[:, gcols].cpu().numpy().T
    assert np.abs(gp - X).max() < 2e-15
    assert not ood.any()
    away = osrc.face_distance(oid, omu) > 1e-12
    log(f"box {k}: ids compared away from faces: {away.sum()} of {away.size}")
    assert away.sum() > 0.95 * away.size
    gid = ids[gcols].cpu().numpy()
    assert np.array_equal(gid[away], near[oid[away]])
    gv = vals[0, gcols].cpu().numpy()
    assert np.abs(gv - osrc.evaluate_at(oid, omu)[0]).max() < 1e-13


def _box_reference(tm, region):
    """Nodes whose incident elements all lie in the box, and the oracle's load
    vector there: exact control part plus the Monte Carlo residual loads."""
    elems, near, osrc, lam, X, oid, omu, ood = region
    tc, tconn = tm
    tconn64 = np.asarray(tconn, dtype=np.int64)
    # nodes whose incident elements are all among the box's elements
    inside = np.zeros(tconn64.shape[0], bool)
    inside[elems] = True
    bad = np.zeros(tc.shape[0], bool)
    bad[tconn64[~inside].ravel()] = True
    vnodes = np.unique(tconn64[elems].ravel())
    nodes = np.setdiff1d(vnodes, np.nonzero(bad)[0])
    assert nodes.size > 10
    # the control g at the box's nodes (they lie in the grown box, where the
    # restricted source is exact), its exact load, and the MC residual loads
    g = np.zeros((1, tc.shape[0]))
    g[0, vnodes] = osrc(tc[vnodes])[0]
    sub = tconn64[elems]
    b_g = cvmc.control_load(tc, sub, g, W.alpha)
    y = osrc.evaluate_at(oid, omu).reshape(1, elems.size, W.samples_per_elem)
    beta = cvmc.element_loads(tc, tconn64, g, y, lam, W.alpha, elems)
    b_res = np.zeros(tc.shape[0])
    np.add.at(b_res, sub.ravel(), beta[0].ravel())
    return nodes, (b_g[0] + b_res)[nodes]


@pytest.fixture(scope="module")
def box_refs(run3d, regions):
    return [_box_reference(run3d[0], r) for r in regions]


@pytest.mark.parametrize("k", range(len(CENTERS)))
def test_fullsize_3d_load_vector_in_box(run3d, box_refs, k):
    res = run3d[6]
    nodes, ref = box_refs[k]
    got = res.b.cpu().numpy()[0, nodes]
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    log(f"box {k}: b rel l2 {err:.2e} at {nodes.size} interior nodes")
    assert err < 1e-12


@pytest.fixture(scope="module")
def run3d_f32(run3d):
    """The binary32 form of the same transfer, solved by binary32 inner PCG
    with four binary64 refinement steps."""
    tm, sm, sv = run3d[:3]
    tc, tconn = tm
    log("tet3d_2m: GPU transfer, binary32 form, binary32 PCG + 4 refinement steps")
    T = ft.Target(tc, tconn)
    S = ft.Source(*sm, sv, bins=BINS)
    cfg = ft.SampleCfg(W.samples_per_elem, 1, W.alpha, W.philox_seed, 0, ft.FT_F32)
    pts = T.sample_points(cfg)
    vals = S.eval_query_list(pts, tc.shape[0])
    T.consume(cfg, vals)
    res = T.project(1, rtol=W.rtol, refine_steps=4)
    torch.cuda.synchronize()
    assert S.take_out_of_domain() == 0
    out = res.x.cpu().numpy()[0], res.b.cpu().numpy()[0], res.reports[0], res.status
    del pts, vals
    T.close()
    S.close()
    return out


@pytest.mark.parametrize("k", range(len(CENTERS)))
def test_fullsize_3d_f32_load_vector_in_box(run3d_f32, box_refs, k):
    x32, b32, rep, status = run3d_f32
    nodes, ref = box_refs[k]
    got = b32[nodes]
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    cons = abs(got.sum() - ref.sum()) / abs(ref.sum())
    log(f"box {k}: binary32 form b rel l2 {err:.2e}, box sum {cons:.2e}")
    assert err < 1e-5
    assert cons < 1e-6


def test_fullsize_3d_f32_solve_and_conservation(run3d, run3d_f32):
    """The refinement solve reaches the oracle's binary64 CG solution of the
    same load vector; conservation holds; the whole binary32-form solution
    stays within 1e-5 of the binary64 route's, whose load vector the boxes pin."""
    tm = run3d[0]
    tc, tconn = tm
    x32, b32, rep, status = run3d_f32
    assert status == ft.FT_OK
    log(f"binary32 form: {rep['iters']} inner iterations, rel resid {rep['rel_resid']:.2e}")
    assert rep["rel_resid"] < 1e-13 and rep["cons_defect"] < 1e-13
    M = geometry.mass_matrix(tc, tconn)
    x_or = cvmc.jacobi_cg(M, b32, 1e-15)
    es = cvmc.rel_l2(x32, x_or)
    log(f"refinement solve vs oracle CG of the same b: {es:.2e}")
    assert es < 1e-12
    m = geometry.lumped_mass(tc, tconn)
    assert abs(rep["int_x"] - float(np.dot(m, x32))) <= 1e-12 * abs(rep["int_x"])
    r64 = run3d[6].reports[0]
    assert abs(rep["sum_b"] - r64["sum_b"]) <= 1e-6 * abs(r64["sum_b"])
    assert cvmc.rel_l2(x32, run3d[6].x.cpu().numpy()[0]) < 1e-5
