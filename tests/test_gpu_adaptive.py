"""GPU parity of variance-driven samples per element against the FP64 oracle
(oracle/adaptive.py): the allocation from a pilot's element variances
(ft_allocate_samples: counts, W, predicted standard error), the query list
of per-element counts (ft_sample_points_adaptive) and its consumption
(ft_consume_queries_adaptive: b, x, the standard error of sum b) with fixed
and per-element alpha, several fields, binary32 and P2 targets; uniform counts
against the fixed-N route bit for bit; invalid ranges and single-sample
elements; the pilot -> allocation -> transfer sequence at 1M triangles."""
import math

import numpy as np
import pytest

from gpu_cases import log, rel_l2
from oracle import adaptive, cvmc, p2, sampling
from oracle.source import P1Source
from paper_2603_00538_amd import ft
from workloads import configs, fields, meshes

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SEED = 0x0F7A5EED00000140


def _pair(dim):
    if dim == 2:
        return meshes.delaunay_tri_mesh(11, 0.3, 191), meshes.delaunay_tri_mesh(15, 0.3, 192)
    return meshes.kuhn_tet_mesh(5, 0.08, 193), meshes.kuhn_tet_mesh(7, 0.08, 194)


def _values(dim, x, F):
    if dim == 2:
        names = ["front_2d", "paper_f2", "smooth_2d"]
        return np.ascontiguousarray(np.stack([fields.evaluate(n_, np, x)[0] for n_ in names[:F]]))
    rows = [fields.evaluate("gaussian_bumps_3d", np, x)[0], np.cos(3 * x[:, 0]) + x[:, 2], np.sin(2 * x[:, 1])]
    return np.ascontiguousarray(np.stack(rows[:F]))


def _cfg(N, F=1, alpha=1.0, stream=0, prec=ft.FT_F64, own=False):
    c = ft.SampleCfg(N, F, alpha, SEED, stream, prec)
    c.alpha_mode = ft.FT_ALPHA_ELEMENT if own else ft.FT_ALPHA_FIXED
    return c


def _offsets(counts):
    return torch.as_tensor(adaptive.offsets(counts), dtype=torch.int64, device="cuda")


def _counts(E, lo, hi, seed):
    """Uneven counts spanning partial waves, full waves and several waves per element."""
    c = np.random.default_rng(seed).integers(lo, hi + 1, E)
    c[: min(E, 4)] = [lo, hi, 64, 128][: min(E, 4)]
    return np.clip(c, lo, hi)


@pytest.mark.parametrize("dim", [2, 3])
def test_adaptive_points_match_oracle(dim):
    tm, _ = _pair(dim)
    tc, tconn = tm
    counts = _counts(tconn.shape[0], 1, 150, 11 + dim)
    off = _offsets(counts)
    total = int(counts.sum())
    X, _ = adaptive.query_points(tc, tconn, counts, SEED, 3)
    ref = np.concatenate([tc, X]).T
    log(f"adaptive emission dim={dim} E={tconn.shape[0]} total={total}")
    T = ft.Target(*tm)
    for prec in (ft.FT_F64, ft.FT_F32):
        pts = T.sample_points_adaptive(_cfg(0, stream=3, prec=prec), off, total).double().cpu().numpy()
        assert pts.shape == ref.shape
        err = np.abs(pts - ref)
        if prec == ft.FT_F64:
            assert np.array_equal(pts[:, : tc.shape[0]], ref[:, : tc.shape[0]])
            assert err.max() < 2e-15
        else:
            assert np.median(err) < 1e-7 and err.max() < 5e-5
    # N_t = N everywhere: the fixed-N list, bit for bit
    c64 = np.full(tconn.shape[0], 64)
    a = T.sample_points_adaptive(_cfg(0, stream=3), _offsets(c64), int(c64.sum()))
    b = T.sample_points(_cfg(64, stream=3))
    assert torch.equal(a, b)
    T.close()


@pytest.mark.parametrize("dim,F,alpha,own,lo,hi", [
    (2, 1, 1.0, False, 2, 150), (2, 1, 0.5, False, 1, 90), (3, 1, 0.75, False, 2, 130),
    (2, 3, 1.0, False, 2, 70), (2, 1, 1.0, True, 2, 100), (3, 2, 1.0, True, 3, 80)])
def test_adaptive_transfer_matches_oracle(dim, F, alpha, own, lo, hi):
    tm, sm = _pair(dim)
    sv = _values(dim, sm[0], F)
    counts = _counts(tm[1].shape[0], lo, hi, 21 + dim + F)
    ref = adaptive.transfer(*tm, P1Source(*sm, sv), counts, alpha=alpha, seed=SEED, stream=5, own_alpha=own)
    log(f"adaptive transfer dim={dim} F={F} alpha={alpha} own={own} counts {lo}..{hi}")
    T = ft.Target(*tm)
    S = ft.Source(*sm, sv)
    off = _offsets(counts)
    total = int(counts.sum())
    for prec in (ft.FT_F64, ft.FT_F32):
        cfg = _cfg(0, F, alpha, 5, prec, own)
        pts = T.sample_points_adaptive(cfg, off, total)
        T.consume_adaptive(cfg, off, total, S.eval_query_list(pts, T.n_nodes))
        r = T.project(F)
        assert r.status == ft.FT_OK
        eb, ex = rel_l2(r.b.cpu().numpy(), ref["b"]), rel_l2(r.x.cpu().numpy(), ref["x"])
        tol = 1e-12 if prec == ft.FT_F64 else 1e-5
        assert eb < tol and ex < tol, (prec, eb, ex)
        for f in range(F):
            rep, want = r.reports[f], ref["report"][f]
            assert rep["cons_defect"] < 1e-12
            if lo >= 2:
                assert abs(rep["sum_b_stderr"] - want["sum_b_stderr"]) <= (1e-9 if prec == ft.FT_F64 else 1e-2) * \
                    want["sum_b_stderr"]
            else:
                assert rep["sum_b_stderr"] == -1.0 and want["sum_b_stderr"] == -1.0
    T.close()
    S.close()


@pytest.mark.parametrize("dim", [2, 3])
def test_adaptive_p2_matches_oracle(dim):
    c, t = meshes.delaunay_tri_mesh(7, 0.3, 195) if dim == 2 else meshes.kuhn_tet_mesh(3, 0.08, 196)
    c2, t2 = meshes.p2_mesh(c, t)
    sm = meshes.delaunay_tri_mesh(12, 0.3, 197) if dim == 2 else meshes.kuhn_tet_mesh(5, 0.08, 198)
    sv = _values(dim, sm[0], 1)
    counts = _counts(t2.shape[0], 2, 100, 31 + dim)
    ref = adaptive.transfer(c2, t2, P1Source(*sm, sv), counts, alpha=0.5, seed=SEED, stream=6)
    log(f"adaptive P2 dim={dim}")
    T = ft.Target(c2, t2, order=2)
    S = ft.Source(*sm, sv)
    off = _offsets(counts)
    total = int(counts.sum())
    cfg = _cfg(0, 1, 0.5, 6)
    pts = T.sample_points_adaptive(cfg, off, total)
    T.consume_adaptive(cfg, off, total, S.eval_query_list(pts, T.n_nodes))
    r = T.project(1)
    assert rel_l2(r.b.cpu().numpy(), ref["b"]) < 1e-12 and rel_l2(r.x.cpu().numpy(), ref["x"]) < 1e-11
    assert abs(r.reports[0]["sum_b_stderr"] - ref["report"][0]["sum_b_stderr"]) < 1e-9 * ref["report"][0]["sum_b_stderr"]
    T.close()
    S.close()


@pytest.mark.parametrize("N", [64, 128])
def test_uniform_counts_equal_fixed_n_bitwise(N):
    """One element per wave on both routes (N >= 64): the same sums in the same order."""
    tm, sm = _pair(2)
    sv = _values(2, sm[0], 1)
    T = ft.Target(*tm)
    S = ft.Source(*sm, sv)
    cfg = _cfg(N, 1, 0.5, 7)
    pts = T.sample_points(cfg)
    T.consume(cfg, S.eval_query_list(pts, T.n_nodes))
    r0 = T.project(1)
    c = np.full(tm[1].shape[0], N)
    off = _offsets(c)
    ca = _cfg(0, 1, 0.5, 7)
    pa = T.sample_points_adaptive(ca, off, int(c.sum()))
    T.consume_adaptive(ca, off, int(c.sum()), S.eval_query_list(pa, T.n_nodes))
    r1 = T.project(1)
    assert torch.equal(r0.b, r1.b) and torch.equal(r0.x, r1.x)
    assert r0.reports[0]["sum_b_stderr"] == r1.reports[0]["sum_b_stderr"]
    T.close()
    S.close()


@pytest.mark.parametrize("dim,F,order", [(2, 1, 1), (3, 1, 1), (2, 3, 1), (2, 1, 2), (3, 1, 2)])
def test_fused_adaptive_matches_black_box_and_oracle(dim, F, order):
    """ft_transfer_p1_adaptive draws the same samples as the list of per-element
    counts and sums them in the same lane order: the black-box route's loads
    (both forms) and the oracle's (binary64)."""
    if order == 1:
        tm, sm = _pair(dim)
    else:
        c, t = meshes.delaunay_tri_mesh(7, 0.3, 199) if dim == 2 else meshes.kuhn_tet_mesh(3, 0.08, 200)
        tm = meshes.p2_mesh(c, t)
        sm = meshes.delaunay_tri_mesh(12, 0.3, 201) if dim == 2 else meshes.kuhn_tet_mesh(5, 0.08, 202)
    sv = _values(dim, sm[0], F)
    counts = _counts(tm[1].shape[0], 2, 300, 41 + dim + F + order)
    ref = adaptive.transfer(*tm, P1Source(*sm, sv), counts, alpha=0.75, seed=SEED, stream=12)
    log(f"fused adaptive dim={dim} F={F} order={order}")
    T = ft.Target(*tm, order=order)
    S = ft.Source(*sm, sv)
    off = _offsets(counts)
    total = int(counts.sum())
    for prec in (ft.FT_F64, ft.FT_F32):
        cfg = _cfg(0, F, 0.75, 12, prec)
        T.transfer_from_adaptive(S, cfg, off, total)
        rf = T.project(F)
        pts = T.sample_points_adaptive(cfg, off, total)
        T.consume_adaptive(cfg, off, total, S.eval_query_list(pts, T.n_nodes))
        rb = T.project(F)
        assert rf.status == ft.FT_OK and rb.status == ft.FT_OK
        assert rel_l2(rf.b.cpu().numpy(), rb.b.cpu().numpy()) < 1e-13
        tol = 1e-12 if prec == ft.FT_F64 else 1e-5
        assert rel_l2(rf.b.cpu().numpy(), ref["b"]) < tol and rel_l2(rf.x.cpu().numpy(), ref["x"]) < 10 * tol
        for f in range(F):
            a_, b_ = rf.reports[f]["sum_b_stderr"], rb.reports[f]["sum_b_stderr"]
            assert abs(a_ - b_) <= 1e-12 * b_
            assert abs(a_ - ref["report"][f]["sum_b_stderr"]) <= (1e-9 if prec == ft.FT_F64 else 1e-2) * a_
    T.close()
    S.close()


def test_fused_adaptive_errors_and_invalid_ranges():
    tm, sm = _pair(2)
    sv = _values(2, sm[0], 1)
    E = tm[1].shape[0]
    T = ft.Target(*tm)
    S = ft.Source(*sm, sv)
    counts = np.full(E, 12)
    off = _offsets(counts)
    total = int(counts.sum())
    for kw, st in (({"alpha_mode": ft.FT_ALPHA_ELEMENT}, ft.FT_E_UNSUPPORTED),
                   ({"sampling": ft.FT_SAMPLING_STRATIFIED}, ft.FT_E_UNSUPPORTED),
                   ({"samples_per_elem": 12}, ft.FT_E_ARG), ({"n_fields": 2}, ft.FT_E_ARG)):
        c = _cfg(0)
        for k, v in kw.items():
            setattr(c, k, v)
        with pytest.raises(ft.FtError) as e:
            T.transfer_from_adaptive(S, c, off, total)
        assert e.value.status == st, kw
    bad = adaptive.offsets(counts)
    bad[3] = bad[2]          # element 2 empty
    bad[E] = total + 1       # the last element runs past total
    T.transfer_from_adaptive(S, _cfg(0), torch.as_tensor(bad, device="cuda"), total)
    r = T.project(1)
    assert r.status == ft.FT_E_NONFINITE and r.reports[0]["n_nonfinite"] == 2
    T.close()
    S.close()


def test_allocation_matches_oracle():
    """A pilot (N0 = 16) on both sides; the GPU counts equal the oracle's except
    where the proportional count lies within 1e-9 of a rounding tie (the two
    element variances differ by rounding); W and the predicted standard error
    to 1e-9; the clamps and the total."""
    tm, sm = _pair(2)
    sv = _values(2, sm[0], 2)
    E = tm[1].shape[0]
    pilot = cvmc.transfer(*tm, P1Source(*sm, sv), 16, alpha=0.5, seed=SEED, stream=8)
    T = ft.Target(*tm)
    S = ft.Source(*sm, sv)
    cfg = _cfg(16, 2, 0.5, 8)
    pts = T.sample_points(cfg)
    T.consume(cfg, S.eval_query_list(pts, T.n_nodes))
    T.project(2)
    for field, budget, lo, hi in ((0, 48 * E, 2, 1 << 20), (1, 48 * E, 2, 1 << 20), (0, 30 * E, 8, 100),
                                  (1, 7, 1, 5), (0, 1, 1, 1)):
        off, al = T.allocate_samples(budget, field=field, n_min=lo, n_max=hi)
        got = np.diff(off.cpu().numpy())
        v = pilot["var_terms"][field]
        want = adaptive.allocate(v, 16, budget, lo, hi)
        a = adaptive.weights(v, 16)
        frac = (budget * a / a.sum() + 0.5) % 1.0
        tie = np.minimum(frac, 1.0 - frac) < 1e-9
        log(f"allocation field={field} budget={budget} [{lo}, {hi}]: total {al.total}, near ties {tie.sum()}")
        assert np.array_equal(got[~tie], want[~tie])
        assert np.all(np.abs(got[tie] - want[tie]) <= 1)
        assert off[0].item() == 0 and al.total == off[-1].item() == got.sum()
        assert got.min() >= lo and got.max() <= hi
        W, se = adaptive.allocation_summary(v, 16, got)
        assert abs(al.weight_sum - W) <= 1e-9 * W and abs(al.predicted_stderr - se) <= 1e-9 * se
    T.close()
    S.close()


def test_allocation_argument_and_order_errors():
    tm, sm = _pair(2)
    sv = _values(2, sm[0], 1)
    T = ft.Target(*tm)
    S = ft.Source(*sm, sv)
    with pytest.raises(ft.FtError) as e:                      # no pilot yet
        T.allocate_samples(100)
    assert e.value.status == ft.FT_E_ORDER
    c1 = _cfg(1)
    pts = T.sample_points(c1)
    T.consume(c1, S.eval_query_list(pts, T.n_nodes))
    with pytest.raises(ft.FtError) as e:                      # N0 = 1 estimates no variance
        T.allocate_samples(100)
    assert e.value.status == ft.FT_E_ORDER
    T.transfer_supermesh(S)
    with pytest.raises(ft.FtError) as e:                      # exact b: nothing to allocate from
        T.allocate_samples(100)
    assert e.value.status == ft.FT_E_ORDER
    T.transfer_from(S, _cfg(8))
    for kw in ({"field": 1}, {"n_min": 0}, {"n_min": 5, "n_max": 4}, {"n_max": (1 << 20) + 1}):
        with pytest.raises(ft.FtError) as e:
            T.allocate_samples(100, **kw)
        assert e.value.status == ft.FT_E_ARG, kw
    with pytest.raises(ft.FtError) as e:
        T.allocate_samples(0)
    assert e.value.status == ft.FT_E_ARG
    off, al = T.allocate_samples(8 * T.n_elems)                # the fused route is a pilot too
    total = al.total
    # the adaptive entries: samples_per_elem must be 0, plain samples, field-major, binary64/32
    with pytest.raises(ft.FtError) as e:
        T.sample_points_adaptive(_cfg(4), off, total)
    assert e.value.status == ft.FT_E_ARG
    for mod in ({"sampling": ft.FT_SAMPLING_STRATIFIED}, {"values_layout": ft.FT_VALUES_ELEMENT_TILES},
                {"precision": ft.FT_SPLIT_F16}):
        c = _cfg(0)
        for k, v in mod.items():
            setattr(c, k, v)
        with pytest.raises(ft.FtError) as e:
            T.sample_points_adaptive(c, off, total)
        assert e.value.status == ft.FT_E_UNSUPPORTED, mod
    with pytest.raises(ft.FtError) as e:                      # total below one sample per element
        T.sample_points_adaptive(_cfg(0), off, T.n_elems - 1)
    assert e.value.status == ft.FT_E_ARG
    pts = T.sample_points_adaptive(_cfg(0), off, total)
    vals = S.eval_query_list(pts, T.n_nodes)
    with pytest.raises(ft.FtError) as e:                      # another stream than the points
        T.consume_adaptive(_cfg(0, stream=9), off, total, vals)
    assert e.value.status == ft.FT_E_ORDER
    with pytest.raises(ft.FtError) as e:                      # fixed-N consumption of this list
        ft.ft_consume_queries(T.handle, _cfg(8), vals.data_ptr(), ft.current_stream())
    assert e.value.status == ft.FT_E_ORDER
    T.consume_adaptive(_cfg(0), off, total, vals)
    assert T.project(1).status == ft.FT_OK
    T.close()
    S.close()


def test_invalid_ranges_and_single_samples():
    """Elements whose ranges are empty, decreasing or past total take no loads,
    count as non-finite values (FT_E_NONFINITE, one per element) and contribute
    zero; a single-sample element leaves the standard error undefined (-1)."""
    tm, sm = _pair(2)
    sv = _values(2, sm[0], 1)
    E = tm[1].shape[0]
    T = ft.Target(*tm)
    S = ft.Source(*sm, sv)
    counts = np.full(E, 10)
    off_np = adaptive.offsets(counts)
    total = int(off_np[-1])
    bad = off_np.copy()
    bad[5] = bad[4]              # element 4 empty (element 5 then has 20: still valid)
    bad[E] = total + 7           # the last element runs past total
    bad_t = torch.as_tensor(bad, device="cuda")
    cfg = _cfg(0, 1, 1.0, 4)
    # the invalid elements' samples are not written: start from zeros
    pts = torch.zeros((2, T.n_nodes + total), dtype=torch.float64, device="cuda")
    T.sample_points_adaptive(cfg, bad_t, total, out=pts)
    vals = S.eval_query_list(pts, T.n_nodes)
    T.consume_adaptive(cfg, bad_t, total, vals)
    r = T.project(1)
    assert r.status == ft.FT_E_NONFINITE and r.reports[0]["n_nonfinite"] == 2
    # single-sample elements: estimable loads, undefined standard error
    c1 = np.full(E, 6)
    c1[::7] = 1
    off1 = _offsets(c1)
    pts = T.sample_points_adaptive(cfg, off1, int(c1.sum()))
    T.consume_adaptive(cfg, off1, int(c1.sum()), S.eval_query_list(pts, T.n_nodes))
    r = T.project(1)
    ref = adaptive.transfer(*tm, P1Source(*sm, sv), c1, alpha=1.0, seed=SEED, stream=4)
    assert r.status == ft.FT_OK and r.reports[0]["sum_b_stderr"] == -1.0
    assert rel_l2(r.b.cpu().numpy(), ref["b"]) < 1e-12
    T.close()
    S.close()


def test_fullsize_pilot_allocation_transfer():
    """tri2d_1m (1M triangles): a pilot with N0 = 16 (fused route, its own
    stream), Neyman counts for 64 samples per element in all, then the
    black-box transfer with those counts (and the fused route with them: the
    same sum b).  Its standard error is below that of
    64 uniform samples and within 15% of the allocation's prediction, sum b lies
    within six standard errors of the exact source integral, and the
    conservation identity holds."""
    w = configs.WORKLOADS["tri2d_1m"]
    tm = configs.build_mesh(w.target)
    sm = configs.build_mesh(w.source)
    sv = configs.source_nodal_values(w, sm[0])
    log("full-size adaptive: tri2d_1m")
    T = ft.Target(*tm)
    S = ft.Source(*sm, sv, bins=w.bins[:2])
    E = T.n_elems
    pilot = ft.SampleCfg(16, 1, w.alpha, w.philox_seed, 1000, ft.FT_F64)
    T.transfer_from(S, pilot)
    T.project(1)
    off, al = T.allocate_samples(64 * E, n_min=2)
    log(f"  total {al.total} (budget {64 * E}), W {al.weight_sum:.6e}, predicted stderr {al.predicted_stderr:.3e}")
    cfg = ft.SampleCfg(0, 1, w.alpha, w.philox_seed, 0, ft.FT_F64)
    pts = T.sample_points_adaptive(cfg, off, al.total)
    T.consume_adaptive(cfg, off, al.total, S.eval_query_list(pts, T.n_nodes))
    del pts
    ra = T.project(1).reports[0]
    T.transfer_from_adaptive(S, cfg, off, al.total)
    rf = T.project(1).reports[0]
    assert abs(rf["sum_b"] - ra["sum_b"]) <= 1e-13 * abs(ra["sum_b"])
    assert abs(rf["sum_b_stderr"] - ra["sum_b_stderr"]) <= 1e-12 * ra["sum_b_stderr"]
    T.transfer_from(S, ft.SampleCfg(64, 1, w.alpha, w.philox_seed, 0, ft.FT_F64))
    ru = T.project(1).reports[0]
    I = S.integral()[0]
    log(f"  adaptive stderr {ra['sum_b_stderr']:.3e}, uniform {ru['sum_b_stderr']:.3e}, "
        f"|sum b - I| {abs(ra['sum_b'] - I):.3e}")
    assert abs(al.total - 64 * E) <= E // 2 + 2 * E // 64
    assert 0.0 < ra["sum_b_stderr"] < ru["sum_b_stderr"]
    assert abs(ra["sum_b_stderr"] / al.predicted_stderr - 1.0) < 0.15
    assert abs(ra["sum_b"] - I) < 6.0 * ra["sum_b_stderr"]
    assert ra["cons_defect"] < 1e-12
    T.close()
    S.close()
