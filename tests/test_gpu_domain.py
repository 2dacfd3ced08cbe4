"""GPU parity at the edges of the source domain and of the localization's
arithmetic, against the FP64 oracle:

* points far outside the source mesh (beyond the largest element box): the
  localization rule's winner over all elements, and its extrapolated value;
* transfers whose target reaches outside the source: the out-of-domain count
  of every route in the report, and the load vector with extrapolated values;
* a mesh of small elements far from the origin: the fast selection test's
  margin grows with the affine forms' magnitude, so points near a shared
  face still get the element that strictly contains them;
* batches whose sources' bins or targets' field buffers were rebuilt between
  runs;
* the report's compensated sums against exactly rounded sums.
"""
import math

import numpy as np
import pytest

from gpu_cases import log, oracle_query_points, oracle_transfer, rel_l2
from oracle import geometry
from oracle.source import P1Source
from paper_2603_00538_amd import ft
from workloads import fields, meshes

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SEED = 0x0F7A5EED000000D0


def _mesh_pair(dim):
    if dim == 2:
        return meshes.delaunay_tri_mesh(12, 0.3, 81), meshes.delaunay_tri_mesh(16, 0.3, 82)
    return meshes.kuhn_tet_mesh(5, 0.08, 83), meshes.kuhn_tet_mesh(6, 0.08, 84)


def _field(dim, x):
    return fields.evaluate("smooth_2d" if dim == 2 else "gaussian_bumps_3d", np, x)


def _min_mu_all(o, p):
    """min_k mu_k of point p in every element of the oracle source (Cramer's rule)."""
    from oracle.source import barycentric_cramer
    mu = barycentric_cramer(o.coords[o.conn], np.broadcast_to(p, (o.conn.shape[0], p.shape[0])))
    return mu.min(axis=1)


@pytest.mark.parametrize("dim", [2, 3])
def test_far_outside_points_take_the_rule_winner(dim):
    _, sm = _mesh_pair(dim)
    sv = _field(dim, sm[0])
    o = P1Source(*sm, sv)
    rng = np.random.default_rng(90 + dim)
    # points 0.3 to 3 units outside the unit square / cube, in every direction
    cand = rng.uniform(-3.0, 4.0, (400, dim))
    far = cand[np.abs(cand - 0.5).max(axis=1) > 0.8]
    # keep the points whose winner is clear (the runner-up's min mu is lower by 1e-9)
    keep = []
    for p in far:
        m = np.sort(_min_mu_all(o, p))
        if m[-1] - m[-2] > 1e-9:
            keep.append(p)
    pts = np.array(keep[:120])
    log(f"far-outside points dim={dim}: {pts.shape[0]}")
    S = ft.Source(*sm, sv)
    dp = torch.as_tensor(np.ascontiguousarray(pts.T), device="cuda")
    ids = torch.empty(pts.shape[0], dtype=torch.int32, device="cuda")
    vals = S.eval(dp, ids=ids).cpu().numpy()[0]
    assert S.take_out_of_domain() == pts.shape[0]
    oid, omu, ood = o.locate(pts)
    assert ood.all()
    assert np.array_equal(ids.cpu().numpy(), oid)
    ov = o.evaluate_at(oid, omu)[0]
    assert np.abs(vals - ov).max() <= 1e-12 * max(1.0, np.abs(ov).max())
    S.close()


def _outside_target(dim):
    """A target on [-0.1, 1.15]^d: nodes and samples outside the unit source domain."""
    if dim == 2:
        tc, tconn = meshes.delaunay_tri_mesh(11, 0.3, 85)
    else:
        tc, tconn = meshes.kuhn_tet_mesh(5, 0.08, 86)
    return (tc * 1.25 - 0.1, tconn)


class _ValuesInOrder:
    """A black box for the oracle that answers with given values: cvmc.transfer
    queries the nodes, then the samples element by element, i.e. the query
    list in order, so each call takes the next block of values."""

    def __init__(self, values):
        self.values = values
        self.pos = 0

    def __call__(self, points):
        m = points.shape[0]
        out = self.values[:, self.pos:self.pos + m]
        self.pos += m
        return out


@pytest.mark.parametrize("dim,N", [(2, 64), (3, 32)])
def test_transfer_reports_out_of_domain(dim, N):
    """A target reaching outside the source.  Outside the mesh the rule's
    winner can be tied: the elements next to a straight boundary that share
    the vertex opposite it give that vertex the same barycentric coordinate,
    so different roundings may pick either (and extrapolate different
    values).  The GPU's element must attain the oracle's best min mu to
    1e-12, its value must be that element's extrapolation, and the rest of
    the transfer is checked against the oracle fed with the same values."""
    tm = _outside_target(dim)
    _, sm = _mesh_pair(dim)
    sv = _field(dim, sm[0])
    o = P1Source(*sm, sv)
    qp = oracle_query_points(tm, N, SEED, 1)
    oid, omu, ood = o.locate(qp.T)
    n_ood = int(ood.sum())
    log(f"out-of-domain transfer dim={dim} N={N}: {n_ood} of {qp.shape[1]} queries outside")
    assert n_ood > 100
    T = ft.Target(*tm)
    S = ft.Source(*sm, sv)
    cfg = ft.SampleCfg(N, 1, 1.0, SEED, 1, ft.FT_F64)
    # black-box route through the built-in source, with its element ids
    pts = T.sample_points(cfg)
    ids = torch.empty(pts.shape[1], dtype=torch.int32, device="cuda")
    vals = S.eval_query_list(pts, T.n_nodes, ids=ids)
    assert S.take_out_of_domain() == n_ood
    gid = ids.cpu().numpy().astype(np.int64)
    gval = vals.cpu().numpy()
    from oracle.source import barycentric_cramer
    gmu = barycentric_cramer(o.coords[o.conn[gid]], qp.T)
    best = omu.min(axis=1)
    assert (gmu.min(axis=1) >= best - 1e-12 * np.maximum(1.0, np.abs(best))).all()
    tied = gid != oid
    log(f"  {int(tied.sum())} queries took another element of a tied set")
    assert np.abs(gval - o.evaluate_at(gid, gmu)).max() <= 1e-12 * max(1.0, np.abs(gval).max())
    ref = oracle_transfer(tm, None, None, N, 1.0, SEED, 1, query=_ValuesInOrder(gval))
    T.consume(cfg, vals)
    r2 = T.project(1)
    assert r2.reports[0]["n_out_of_domain"] == -1   # the caller's black box evaluated the queries
    assert rel_l2(r2.b.cpu().numpy(), ref["b"]) < 1e-12
    assert rel_l2(r2.x.cpu().numpy(), ref["x"]) < 1e-12
    # fused route: the same localization, counted for the report
    T.transfer_from(S, cfg)
    r = T.project(1)
    assert r.reports[0]["n_out_of_domain"] == n_ood
    assert rel_l2(r.b.cpu().numpy(), ref["b"]) < 1e-12
    assert rel_l2(r.x.cpu().numpy(), ref["x"]) < 1e-12
    assert S.take_out_of_domain() == 0   # the transfer's count is the report's
    # plan: counted at setup, reported after every online transfer
    plan = ft.Plan(T, S, cfg)
    for _ in range(2):
        plan.transfer()
        r3 = T.project(1)
        assert r3.reports[0]["n_out_of_domain"] == n_ood
        assert torch.equal(r3.b, r.b)
    plan.close()
    # batch of one
    B = ft.Batch([T], [S], [cfg])
    _, bs, reps, _, st = B.run(rtol=1e-14, max_iter=80)
    assert reps[0]["n_out_of_domain"] == n_ood
    assert rel_l2(bs[0].cpu().numpy(), ref["b"][0]) < 1e-12
    B.close()
    T.close()
    S.close()


def test_fast_test_margin_scales_with_mesh():
    """Elements of size ~1e-5 around (1e4, -2e4): the absolute affine forms
    carry terms near 1e10, so their rounding (about 1e-6 in barycentric
    terms) dwarfs a fixed 1e-9 acceptance margin, and a point just outside
    an element could be taken as inside it.  Points placed 5e-8
    (barycentric) from shared edges, on both sides, must get the oracle's
    element wherever the oracle finds them strictly inside one."""
    sc, sconn = meshes.delaunay_tri_mesh(14, 0.3, 87)
    shift = np.array([1.0e4, -2.0e4])
    sv = fields.evaluate("smooth_2d", np, sc)
    sc = sc * 1e-4 + shift
    o = P1Source(sc, sconn, sv)
    edges = {}
    for e, tri in enumerate(sconn):
        for k in range(3):
            key = tuple(sorted((tri[(k + 1) % 3], tri[(k + 2) % 3])))
            edges.setdefault(key, []).append((e, k))
    pts = []
    rng = np.random.default_rng(7)
    for owners in edges.values():
        if len(owners) != 2:
            continue
        for e, k in owners:
            lam = np.empty(3)
            lam[k] = 5e-8
            s = rng.uniform(0.2, 0.8)
            lam[(k + 1) % 3] = (1 - 5e-8) * s
            lam[(k + 2) % 3] = (1 - 5e-8) * (1 - s)
            pts.append(lam @ sc[sconn[e]])
    pts = np.array(pts)
    oid, omu, ood = o.locate(pts)
    assert not ood.any()
    inside = omu.min(axis=1) > 1e-12   # a unique winner
    assert inside.sum() > 0.8 * pts.shape[0]
    S = ft.Source(sc, sconn, sv)
    ids = torch.empty(pts.shape[0], dtype=torch.int32, device="cuda")
    vals = S.eval(torch.as_tensor(np.ascontiguousarray(pts.T), device="cuda"), ids=ids).cpu().numpy()[0]
    ids = ids.cpu().numpy()
    log(f"fast-test margin: {pts.shape[0]} points next to shared edges, {int(inside.sum())} strictly inside")
    assert np.array_equal(ids[inside], oid[inside])
    assert np.abs(vals - o.evaluate_at(oid, omu)[0]).max() < 1e-9
    assert S.take_out_of_domain() == 0
    S.close()


def test_batch_follows_rebuilt_bins_and_field_buffers():
    """A batch keeps working after its source's bins are rebuilt (autotune)
    and its target's field buffers are reallocated by a transfer of more
    fields: the next run reads the live descriptors, graph replays too."""
    items = [(meshes.delaunay_tri_mesh(12, 0.3, 91), meshes.delaunay_tri_mesh(17, 0.3, 92), 64),
             (meshes.kuhn_tet_mesh(5, 0.08, 93), meshes.kuhn_tet_mesh(7, 0.08, 94), 32)]
    targets, sources, cfgs = [], [], []
    for k, (tm, sm, N) in enumerate(items):
        dim = tm[0].shape[1]
        targets.append(ft.Target(*tm))
        sources.append(ft.Source(*sm, _field(dim, sm[0])))
        cfgs.append(ft.SampleCfg(N, 1, 1.0, SEED, 10 + k, ft.FT_F64))
    B = ft.Batch(targets, sources, cfgs, graph=True)
    _, b0, _, _, _ = B.run(rtol=1e-14, max_iter=80)
    ref = [b.clone() for b in b0]
    # rebuild the bins of both sources on their own query lists
    for T, S, c in zip(targets, sources, cfgs):
        pts = T.sample_points(c)
        S.autotune(pts, T.n_nodes, [5, 9, 13])
    # grow the first target's field buffers with a two-field black-box transfer
    T0 = targets[0]
    c2 = ft.SampleCfg(16, 2, 1.0, SEED, 3, ft.FT_F64)
    p2 = T0.sample_points(c2)
    T0.consume(c2, torch.stack([p2[0], p2[1]]).contiguous())
    T0.project(2)
    log("batch after autotune and field-buffer growth")
    for _ in range(2):
        _, b1, reps, _, st = B.run(rtol=1e-14, max_iter=80)
        assert st == ft.FT_OK
        for k in range(len(items)):
            assert torch.equal(b1[k], ref[k])
    for T, S, c, b in zip(targets, sources, cfgs, ref):
        T.transfer_from(S, c)
        r = T.project(1)
        assert rel_l2(r.b[0].cpu().numpy(), b.cpu().numpy()) < 1e-15
    B.close()
    for o in targets + sources:
        o.close()


@pytest.mark.parametrize("dim", [2, 3])
def test_report_sums_are_compensated(dim):
    tm, sm = _mesh_pair(dim)
    sv = _field(dim, sm[0])
    res = None
    T = ft.Target(*tm)
    S = ft.Source(*sm, sv)
    T.transfer_from(S, ft.SampleCfg(48, 1, 1.0, SEED, 4, ft.FT_F64))
    res = T.project(1)
    b = res.b[0].cpu().numpy()
    x = res.x[0].cpu().numpy()
    rep = res.reports[0]
    exact_b = math.fsum(b)
    assert abs(rep["sum_b"] - exact_b) <= 2 * math.ulp(abs(exact_b))
    m = geometry.lumped_mass(np.asarray(tm[0], dtype=np.float64), np.asarray(tm[1], dtype=np.int64))
    exact_x = math.fsum((m * x).tolist())
    assert abs(rep["int_x"] - exact_x) <= 1e-15 * abs(exact_x)
    T.close()
    S.close()


@pytest.mark.parametrize("dim,F", [(2, 1), (3, 1), (3, 5)])
def test_source_integral_matches_oracle(dim, F):
    """ft_source_integral against the oracle's exact integral, and against
    the closed form for an affine field (c0 + c . x over the unit square /
    cube integrates to c0 + sum(c) / 2)."""
    _, sm = _mesh_pair(dim)
    if F == 1:
        sv = _field(dim, sm[0])
    else:
        modes = fields.fourier_modes(seed=5, n_fields=F, n_modes=3, kmax=2)
        sv = fields.fourier_fields_3d(np, sm[0][:, 0], sm[0][:, 1], sm[0][:, 2], modes) + 1.0
    S = ft.Source(*sm, np.ascontiguousarray(sv))
    got = np.array(S.integral())
    ref = P1Source(*sm, sv).integral()
    assert np.abs(got - ref).max() <= 1e-14 * np.abs(ref).max()
    S.close()
    va = fields.evaluate("affine", np, sm[0])
    S = ft.Source(*sm, va)
    c0, c = 1.25, (0.75, -2.0, 0.5)
    assert abs(S.integral()[0] - (c0 + 0.5 * sum(c[:dim]))) < 1e-14
    S.close()
