"""Parity of the split many-field form at its full size (998,250 target
tetrahedra x 128 samples, 3,951,018 source tetrahedra, 64 fields, 110^3 bins:
the grid the bin autotuner picks), in the launch configuration bench.py
times: binary32 points and values, hi+lo binary16 matrix-core element sums,
batched binary64 PCG.

As for the 3D single-field workload, the oracle works in three boxes of the
domain, on the source elements that can hold the samples of the target
elements there.  Values are checked at the binary32 points the kernels saw
(to binary32 rounding); the load vector at the nodes whose elements all lie
in a box, against the oracle's binary64 samples, within the 1e-5 of the
split form (its samples use 24-bit uniforms).
"""
import numpy as np
import pytest

from gpu_cases import log
from oracle import cvmc
from oracle.source import P1Source
from paper_2603_00538_amd import ft
from workloads import configs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

W = configs.WORKLOADS["tet3d_1m_64f"]
BINS = (110, 110, 110)
CENTERS = [(0.27, 0.61, 0.44), (0.74, 0.22, 0.83)]
HALF = 0.04   # box half-width (a target element spans about 1/56)


def _region(tm, sm, sv, center):
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
def split_case():
    log("tet3d_1m_64f: meshes and fields")
    tm = configs.build_mesh(W.target)
    sm = configs.build_mesh(W.source)
    sv = configs.source_nodal_values(W, sm[0])
    tc, tconn = tm
    n, N, F = tc.shape[0], W.samples_per_elem, W.n_fields
    log("tet3d_1m_64f: GPU transfer, split f16")
    T = ft.Target(tc, tconn)
    S = ft.Source(*sm, sv, bins=BINS)
    cfg = ft.SampleCfg(N, F, W.alpha, W.philox_seed, 0, ft.FT_SPLIT_F16)
    pts = T.sample_points(cfg)
    ids = torch.empty(pts.shape[1], dtype=torch.int32, device="cuda")
    vals = S.eval_query_list(pts, n, ids=ids)
    T.consume(cfg, vals)
    res = T.project(F, rtol=W.rtol)
    torch.cuda.synchronize()
    assert res.status == ft.FT_OK
    assert S.take_out_of_domain() == 0
    boxes = []
    for k, c in enumerate(CENTERS):
        elems, near, osrc = _region(tm, sm, sv, c)
        cols = torch.as_tensor((n + elems[:, None] * N + np.arange(N)[None, :]).ravel(), device="cuda")
        boxes.append((elems, near, osrc, pts[:, cols].double().cpu().numpy().T, vals[:, cols].double().cpu().numpy(),
                      ids[cols].cpu().numpy()))
        log(f"box {k}: {elems.size} target elements, {near.size} source elements")
    b = res.b.cpu().numpy()
    del pts, vals, ids
    T.close()
    S.close()
    return tm, sv, boxes, b


@pytest.mark.parametrize("k", range(len(CENTERS)))
def test_fullsize_split_values(split_case, k):
    tm, sv, boxes, b = split_case
    elems, near, osrc, gp, gv, gid = boxes[k]
    oid, omu, ood = osrc.locate(gp)   # the binary32 points the kernels saw
    assert not ood.any()
    away = osrc.face_distance(oid, omu) > 1e-12
    log(f"box {k}: {gp.shape[0]} samples, ids compared away from faces: {away.sum()}")
    assert away.sum() > 0.95 * away.size
    assert np.array_equal(gid[away], near[oid[away]])
    ref = osrc.evaluate_at(oid, omu)   # (64, samples)
    scale = np.abs(ref).max()
    err = np.abs(gv[:, away] - ref[:, away]).max()
    log(f"box {k}: values max error {err / scale:.2e} of the largest value")
    assert err <= 1e-6 * scale


@pytest.mark.parametrize("k", range(len(CENTERS)))
def test_fullsize_split_load_vector_in_box(split_case, k):
    tm, sv, boxes, b = split_case
    elems, near, osrc, gp, gv, gid = boxes[k]
    tc, tconn = tm
    tconn64 = np.asarray(tconn, dtype=np.int64)
    F, N = W.n_fields, W.samples_per_elem
    inside = np.zeros(tconn64.shape[0], bool)
    inside[elems] = True
    bad = np.zeros(tc.shape[0], bool)
    bad[tconn64[~inside].ravel()] = True
    vnodes = np.unique(tconn64[elems].ravel())
    nodes = np.setdiff1d(vnodes, np.nonzero(bad)[0])
    log(f"box {k}: load vectors of {F} fields at {nodes.size} interior nodes")
    assert nodes.size > 10
    g = np.zeros((F, tc.shape[0]))
    g[:, vnodes] = osrc(tc[vnodes])
    sub = tconn64[elems]
    b_g = cvmc.control_load(tc, sub, g, W.alpha)
    lam, X = cvmc.query_points(tc, tconn64, N, W.philox_seed, 0, elems)
    y = osrc(X.reshape(-1, 3)).reshape(F, elems.size, N)
    beta = cvmc.element_loads(tc, tconn64, g, y, lam, W.alpha, elems)
    worst = 0.0
    for f in range(F):
        b_res = np.zeros(tc.shape[0])
        np.add.at(b_res, sub.ravel(), beta[f].ravel())
        ref = (b_g[f] + b_res)[nodes]
        worst = max(worst, np.linalg.norm(b[f, nodes] - ref) / np.linalg.norm(ref))
    log(f"box {k}: worst field b rel l2 {worst:.2e}")
    assert worst < 1e-5
