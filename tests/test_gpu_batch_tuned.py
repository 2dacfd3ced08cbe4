"""The binary32 form of the fused route and of batches, and the batch
autotuner (element variants and bin grids timed per kind of transfer, with a
JSON cache), against the FP64 oracle and the single-transfer routes."""
import json
import os

import numpy as np
import pytest

from gpu_cases import log, oracle_transfer, rel_l2
from paper_2603_00538_amd import ft
from workloads import fields, meshes

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SEED = 0x0F7A5EED00000110


def _items():
    specs = [
        (meshes.delaunay_tri_mesh(12, 0.3, 161), meshes.delaunay_tri_mesh(17, 0.3, 162), "front_2d", 64),
        (meshes.structured_tri_mesh(14, 0.2, 163), meshes.structured_tri_mesh(24, 0.2, 164), "smooth_2d", 256),
        (meshes.kuhn_tet_mesh(5, 0.08, 165), meshes.kuhn_tet_mesh(7, 0.08, 166), "gaussian_bumps_3d", 128),
        (meshes.kuhn_tet_mesh(4, 0.08, 167), meshes.kuhn_tet_mesh(6, 0.08, 168), "gaussian_bumps_3d", 20),
        (meshes.delaunay_tri_mesh(9, 0.3, 169), meshes.delaunay_tri_mesh(13, 0.3, 170), "smooth_2d", 32),
    ]
    return [(tm, sm, fields.evaluate(f, np, sm[0]), N) for tm, sm, f, N in specs]


@pytest.mark.parametrize("dim,N", [(2, 64), (2, 20), (3, 128), (3, 37)])
def test_fused_f32_matches_black_box_f32(dim, N):
    """ft_transfer_p1 in FT_F32 is the binary32 black-box route with the query
    list kept in registers: the same points, values rounded alike, binary64 sums."""
    if dim == 2:
        tm, sm = meshes.delaunay_tri_mesh(12, 0.3, 171), meshes.delaunay_tri_mesh(16, 0.3, 172)
        sv = fields.evaluate("front_2d", np, sm[0])
    else:
        tm, sm = meshes.kuhn_tet_mesh(5, 0.08, 173), meshes.kuhn_tet_mesh(7, 0.08, 174)
        sv = fields.evaluate("gaussian_bumps_3d", np, sm[0])
    log(f"fused binary32 dim={dim} N={N}")
    T = ft.Target(*tm)
    S = ft.Source(*sm, sv)
    cfg = ft.SampleCfg(N, 1, 1.0, SEED, 2, ft.FT_F32)
    pts = T.sample_points(cfg)
    T.consume(cfg, S.eval_query_list(pts, T.n_nodes))
    rb = T.project(1)
    T.transfer_from(S, cfg)
    rf = T.project(1)
    assert rel_l2(rf.b.cpu().numpy(), rb.b.cpu().numpy()) < 1e-14
    assert rel_l2(rf.x.cpu().numpy(), rb.x.cpu().numpy()) < 1e-13
    ref = oracle_transfer(tm, sm, sv, N, 1.0, SEED, 2)
    assert rel_l2(rf.b.cpu().numpy(), ref["b"]) < 1e-5
    assert rel_l2(rf.x.cpu().numpy(), ref["x"]) < 1e-5
    assert abs(rf.reports[0]["sum_b"] - ref["report"][0]["sum_b"]) <= 1e-6 * abs(ref["report"][0]["sum_b"])
    T.close()
    S.close()


@pytest.fixture(scope="module")
def tuned_case(tmp_path_factory):
    items = _items()
    targets = [ft.Target(*tm) for tm, _, _, _ in items]
    sources = [ft.Source(*sm, sv) for _, sm, sv, _ in items]
    cache = str(tmp_path_factory.mktemp("tune") / "batch_tune.json")
    yield items, targets, sources, cache
    for o in targets + sources:
        o.close()


@pytest.mark.parametrize("prec", [ft.FT_F64, ft.FT_F32])
def test_batch_forms_match_single_route_and_oracle(tuned_case, prec):
    items, targets, sources, _ = tuned_case
    cfgs = [ft.SampleCfg(N, 1, 1.0, SEED, 30 + k, prec) for k, (_, _, _, N) in enumerate(items)]
    log(f"batch form precision={prec}")
    B = ft.Batch(targets, sources, cfgs, graph=True)
    xs, bs, reps, sts, st = B.run(rtol=1e-14, max_iter=80)
    assert st == ft.FT_OK
    for k, ((tm, sm, sv, N), T, S, c) in enumerate(zip(items, targets, sources, cfgs)):
        T.transfer_from(S, c)
        r = T.project(1)
        assert rel_l2(bs[k].cpu().numpy(), r.b[0].cpu().numpy()) < 1e-14
        ref = oracle_transfer(tm, sm, sv, N, 1.0, SEED, 30 + k)
        tol = 1e-12 if prec == ft.FT_F64 else 1e-5
        assert rel_l2(bs[k].cpu().numpy(), ref["b"][0]) < tol
        assert rel_l2(xs[k].cpu().numpy(), ref["x"][0]) < tol
    B.close()


def test_batch_autotune_and_cache(tuned_case):
    items, targets, sources, cache = tuned_case
    cfgs = [ft.SampleCfg(N, 1, 1.0, SEED, 40 + k, ft.FT_F64) for k, (_, _, _, N) in enumerate(items)]
    B = ft.Batch(targets, sources, cfgs, graph=True)
    _, b_default, _, _, _ = B.run(rtol=1e-14, max_iter=80)
    b_default = [b.clone() for b in b_default]
    n = B.autotune(cache)
    log(f"batch autotune: {n} kinds timed; variants {[B.variant(k) for k in range(len(items))]}")
    assert n == len(items)   # every transfer here is its own kind
    with open(cache) as fh:
        entries = json.load(fh)["entries"]
    assert len(entries) == len(items)
    assert all(v["G"] in (16, 32, 64) and v["P"] in (1, 2, 4) and v["bins_scale"] > 0 for v in entries.values())
    for _ in range(2):   # graph captured again, then replayed
        xs, bs, reps, sts, st = B.run(rtol=1e-14, max_iter=80)
        assert st == ft.FT_OK
        for k, (tm, sm, sv, N) in enumerate(items):
            # another variant changes only the order of each element's sums
            assert rel_l2(bs[k].cpu().numpy(), b_default[k].cpu().numpy()) < 1e-14
    ref = oracle_transfer(items[0][0], items[0][1], items[0][2], items[0][3], 1.0, SEED, 40)
    assert rel_l2(bs[0].cpu().numpy(), ref["b"][0]) < 1e-12
    variants = [B.variant(k) for k in range(len(items))]
    B.close()
    # a second batch of the same kinds takes everything from the cache
    B2 = ft.Batch(targets, sources, cfgs)
    assert B2.autotune(cache) == 0
    assert [B2.variant(k) for k in range(len(items))] == variants
    _, bs2, _, _, st = B2.run(rtol=1e-14, max_iter=80)
    assert st == ft.FT_OK
    for k in range(len(items)):
        assert torch.equal(bs2[k], bs[k])
    B2.close()
    os.remove(cache)


def test_batch_many_fields_match_single_route_and_oracle():
    """Transfers of several fields in one batch (each field a system of its
    own on the transfer's target): per field the single-transfer fused route's
    load vector and the oracle's; more than four fields, beyond the fused
    route, against the oracle; reports per field, transfer by transfer."""
    t2, s2 = meshes.delaunay_tri_mesh(10, 0.3, 181), meshes.delaunay_tri_mesh(15, 0.3, 182)
    t3, s3 = meshes.kuhn_tet_mesh(4, 0.08, 183), meshes.kuhn_tet_mesh(6, 0.08, 184)
    x2, x3 = s2[0], s3[0]
    v2 = np.ascontiguousarray(np.stack([np.sin((f + 1) * x2[:, 0]) + np.cos((f + 2) * x2[:, 1]) for f in range(3)]))
    v3 = np.ascontiguousarray(np.stack([np.cos(f * x3[:, 0] + 1.0) * x3[:, 2] + x3[:, 1] for f in range(7)]))
    v1 = fields.evaluate("smooth_2d", np, s2[0])
    t1 = meshes.delaunay_tri_mesh(8, 0.3, 185)
    items = [(t2, s2, v2, 64), (t3, s3, v3, 32), (t1, s2, v1, 20)]
    targets = [ft.Target(*tm) for tm, _, _, _ in items]
    sources = [ft.Source(*sm, sv) for _, sm, sv, _ in items]
    cfgs = [ft.SampleCfg(N, sv.shape[0], 1.0, SEED, 50 + k, ft.FT_F64) for k, (_, _, sv, N) in enumerate(items)]
    log("batch of many-field transfers: F = 3, 7, 1")
    B = ft.Batch(targets, sources, cfgs, graph=True)
    for _ in range(2):
        xs, bs, reps, sts, st = B.run(rtol=1e-14, max_iter=80)
        assert st == ft.FT_OK and len(reps) == 3 + 7 + 1 and all(s_ == ft.FT_OK for s_ in sts)
    r = 0
    for k, ((tm, sm, sv, N), T, S, c) in enumerate(zip(items, targets, sources, cfgs)):
        F = sv.shape[0]
        bk = bs[k].cpu().numpy().reshape(F, -1)
        xk = xs[k].cpu().numpy().reshape(F, -1)
        ref = oracle_transfer(tm, sm, sv, N, 1.0, SEED, 50 + k)
        assert rel_l2(bk, ref["b"]) < 1e-12 and rel_l2(xk, ref["x"]) < 1e-12
        for f in range(F):
            assert abs(reps[r + f]["sum_b"] - ref["report"][f]["sum_b"]) <= 1e-12 * abs(ref["report"][f]["sum_b"])
        r += F
        if F <= 4:
            T.transfer_from(S, c)
            single = T.project(F)
            assert rel_l2(bk, single.b.cpu().numpy().reshape(F, -1)) < 1e-14
    B.close()
    for o in targets + sources:
        o.close()


def test_batch_consume_run_matches_single_black_box():
    """Caller values for every transfer (a batch created without sources): per
    field the load vector and solution of each target's own black-box route
    (ft_consume_queries + ft_project), binary64 and binary32, one and several
    fields, with the standard error of sum b; the built-in run is refused for
    such a batch, and so is a target sampled with another configuration."""
    t2, s2 = meshes.delaunay_tri_mesh(11, 0.3, 191), meshes.delaunay_tri_mesh(16, 0.3, 192)
    t3, s3 = meshes.kuhn_tet_mesh(5, 0.08, 193), meshes.kuhn_tet_mesh(6, 0.08, 194)
    v2 = np.ascontiguousarray(np.stack([np.sin((f + 1) * s2[0][:, 0]) + s2[0][:, 1] for f in range(2)]))
    v3 = fields.evaluate("gaussian_bumps_3d", np, s3[0])
    items = [(t2, s2, v2, 48, ft.FT_F64), (t3, s3, v3, 64, ft.FT_F32), (t2, s2, v2[:1].copy(), 100, ft.FT_F64)]
    targets = [ft.Target(*tm) for tm, _, _, _, _ in items]
    sources = [ft.Source(*sm, sv) for _, sm, sv, _, _ in items]
    cfgs = [ft.SampleCfg(N, sv.shape[0], 0.75, SEED, 60 + k, prec) for k, (_, _, sv, N, prec) in enumerate(items)]
    log("batch of caller-value transfers")
    B = ft.Batch(targets, None, cfgs)
    values = []
    for T, S, c in zip(targets, sources, cfgs):
        pts = T.sample_points(c)
        values.append(S.eval_query_list(pts, T.n_nodes))
    xs, bs, reps, sts, st = B.consume_run(values, rtol=1e-14, max_iter=100)
    assert st == ft.FT_OK and len(reps) == 2 + 1 + 1
    r = 0
    for k, (T, c) in enumerate(zip(targets, cfgs)):
        F = c.n_fields
        T.consume(c, values[k])
        single = T.project(F)
        assert rel_l2(bs[k].cpu().numpy().reshape(F, -1), single.b.cpu().numpy()) < 1e-14
        assert rel_l2(xs[k].cpu().numpy().reshape(F, -1), single.x.cpu().numpy()) < 1e-12
        for f in range(F):
            assert reps[r + f]["n_out_of_domain"] == -1
            assert abs(reps[r + f]["sum_b_stderr"] - single.reports[f]["sum_b_stderr"]) <= \
                1e-12 * single.reports[f]["sum_b_stderr"]
        r += F
    with pytest.raises(ft.FtError) as e:
        B.run()
    assert e.value.status == ft.FT_E_ORDER
    other = ft.SampleCfg(cfgs[0].samples_per_elem, cfgs[0].n_fields, 0.75, SEED, 99, ft.FT_F64)
    targets[0].sample_points(other)
    with pytest.raises(ft.FtError) as e:
        B.consume_run(values)
    assert e.value.status == ft.FT_E_ORDER
    B.close()
    for o in targets + sources:
        o.close()
