"""GPU parity of the intersection-based (supermesh) load vector,
ft_transfer_supermesh, against the oracle's exact supermesh projection
(oracle/supermesh.py: Sutherland-Hodgman clip, fan, degree-2 rule per
sub-triangle; oracle/supermesh3d.py: vertex enumeration and a Delaunay split
of each tetrahedral intersection), and its identities: the intersection areas of a target element
add up to its area, sum b = integral f^s, an identical source gives b = M F,
an affine source gives x = f.  It is also the exact reference the Monte Carlo
estimate converges to: at small size the mean over realizations, at the
1M-triangle size the error of one realization against the spread between
two."""
import numpy as np
import pytest

from gpu_cases import log, rel_l2
from oracle import cvmc, geometry, supermesh, supermesh3d
from paper_2603_00538_amd import ft
from workloads import configs, fields, meshes

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SEED = 0x0F7A5EED000000E0


def _gpu_supermesh(tm, sm, sv, area=True):
    T = ft.Target(*tm)
    S = ft.Source(*sm, np.ascontiguousarray(sv))
    a = T.transfer_supermesh(S, area=area)
    r = T.project(S.n_fields, rtol=1e-14, max_iter=500)
    torch.cuda.synchronize()
    out = {"b": r.b.cpu().numpy(), "x": r.x.cpu().numpy(), "reports": r.reports, "status": r.status,
           "area": a.cpu().numpy() if a is not None else None, "integral": np.array(S.integral())}
    T.close()
    S.close()
    return out


@pytest.mark.parametrize("kt,ks,kind,F", [(8, 11, "delaunay", 1), (10, 7, "delaunay", 1), (9, 13, "delaunay", 3),
                                          (6, 12, "structured", 1)])
def test_supermesh_matches_oracle(kt, ks, kind, F):
    """Random meshes both ways round (finer and coarser source), several fields,
    and structured meshes whose edges and vertices coincide (a target edge lies
    on source edges: intersections touch along edges)."""
    if kind == "delaunay":
        tm, sm = meshes.delaunay_tri_mesh(kt, 0.3, 110 + kt), meshes.delaunay_tri_mesh(ks, 0.3, 120 + ks)
    else:
        tm, sm = meshes.structured_tri_mesh(kt, 0.0, 0), meshes.structured_tri_mesh(ks, 0.0, 0)
    if F == 1:
        sv = fields.evaluate("paper_f1", np, sm[0])
    else:
        sv = np.stack([fields.evaluate(n_, np, sm[0])[0] for n_ in ("paper_f1", "paper_f2", "smooth_2d")])
    log(f"supermesh {kind} target {kt} source {ks} F={F}")
    got = _gpu_supermesh(tm, sm, sv)
    ref = supermesh.supermesh_projection(*tm, *sm, sv)
    assert got["status"] == ft.FT_OK
    assert rel_l2(got["b"], ref["b"]) < 1e-12
    vol = geometry.element_measures(np.asarray(tm[0]), np.asarray(tm[1], dtype=np.int64))
    assert np.abs(got["area"] - vol).max() <= 1e-13 * vol.max()
    assert np.abs(ref["area_sum"] - vol).max() <= 1e-13 * vol.max()
    M = geometry.mass_matrix(np.asarray(tm[0]), np.asarray(tm[1], dtype=np.int64))
    x_ref = cvmc.solve_mass(M, ref["b"], 2)
    assert rel_l2(got["x"], x_ref) < 1e-12
    # sum of b is the exact integral of the source field
    for f in range(F):
        assert abs(got["b"][f].sum() - got["integral"][f]) <= 1e-13 * max(1.0, abs(got["integral"][f]))
        assert got["reports"][f]["n_out_of_domain"] == 0


def test_supermesh_identities():
    tm = meshes.delaunay_tri_mesh(10, 0.3, 131)
    # identical source: b = M F, so x = F
    F = fields.evaluate("paper_f3", np, tm[0])
    got = _gpu_supermesh(tm, tm, F)
    assert rel_l2(got["x"], F) < 1e-12
    # affine source on another mesh: the target reproduces it exactly
    sm = meshes.delaunay_tri_mesh(14, 0.3, 132)
    got = _gpu_supermesh(tm, sm, fields.evaluate("affine", np, sm[0]))
    assert np.abs(got["x"] - fields.evaluate("affine", np, tm[0])).max() < 1e-12


def test_supermesh_partial_cover():
    """A target reaching outside the source: the covered part of each element
    is integrated (as the oracle does), and the elements not entirely covered
    are counted."""
    tc, tconn = meshes.delaunay_tri_mesh(9, 0.3, 133)
    tm = (tc * 1.2 - 0.1, tconn)
    sm = meshes.delaunay_tri_mesh(12, 0.3, 134)
    sv = fields.evaluate("smooth_2d", np, sm[0])
    got = _gpu_supermesh(tm, sm, sv)
    ref = supermesh.supermesh_projection(*tm, *sm, sv)
    assert rel_l2(got["b"], ref["b"]) < 1e-12
    assert np.abs(got["area"] - ref["area_sum"]).max() < 1e-14
    vol = geometry.element_measures(tm[0], np.asarray(tconn, dtype=np.int64))
    partial = int((ref["area_sum"] < vol * (1 - 1e-12)).sum())
    assert partial > 0 and got["reports"][0]["n_out_of_domain"] == partial
    # more than four fields are not supported by the intersection route
    S5 = ft.Source(*sm, np.ascontiguousarray(np.stack([sv[0]] * 5)))
    T = ft.Target(*tm)
    with pytest.raises(ft.FtError) as e:
        T.transfer_supermesh(S5)
    assert e.value.status == ft.FT_E_UNSUPPORTED
    T.close()
    S5.close()


# ---- tetrahedra: against the oracle's vertex-enumeration supermesh -------------------------
@pytest.mark.parametrize("kt,ks,F,jt,js", [(4, 5, 1, 0.08, 0.08), (5, 3, 1, 0.08, 0.08), (4, 5, 3, 0.08, 0.05),
                                           (3, 5, 1, 0.0, 0.0)])
def test_supermesh3d_matches_oracle(kt, ks, F, jt, js):
    """Perturbed Kuhn meshes both ways round (finer and coarser source), several
    fields, and unperturbed meshes whose faces lie in common planes (pieces
    touch along faces and edges)."""
    tm, sm = meshes.kuhn_tet_mesh(kt, jt, 210 + kt), meshes.kuhn_tet_mesh(ks, js, 220 + ks)
    rows = [fields.evaluate("gaussian_bumps_3d", np, sm[0])[0], np.cos(3 * sm[0][:, 0]) + sm[0][:, 2],
            np.sin(2 * sm[0][:, 1]) * sm[0][:, 0]]
    sv = np.ascontiguousarray(np.stack(rows[:F]))
    log(f"supermesh 3D target {kt} source {ks} F={F}")
    got = _gpu_supermesh(tm, sm, sv)
    ref = supermesh3d.supermesh_projection(*tm, *sm, sv)
    assert got["status"] == ft.FT_OK
    assert rel_l2(got["b"], ref["b"]) < 1e-12
    vol = geometry.element_measures(np.asarray(tm[0]), np.asarray(tm[1], dtype=np.int64))
    assert np.abs(got["area"] - vol).max() <= 1e-13 * vol.max()
    M = geometry.mass_matrix(np.asarray(tm[0]), np.asarray(tm[1], dtype=np.int64))
    assert rel_l2(got["x"], cvmc.solve_mass(M, ref["b"], 3)) < 1e-12
    for f in range(F):
        assert abs(got["b"][f].sum() - got["integral"][f]) <= 1e-13 * max(1.0, abs(got["integral"][f]))
        assert got["reports"][f]["n_out_of_domain"] == 0
        assert got["reports"][f]["sum_b_stderr"] == 0.0


def test_supermesh3d_identities_and_partial_cover():
    tm = meshes.kuhn_tet_mesh(4, 0.08, 230)
    F = fields.evaluate("gaussian_bumps_3d", np, tm[0])
    got = _gpu_supermesh(tm, tm, F)           # identical source: b = M F
    assert rel_l2(got["x"], F) < 1e-12
    sm = meshes.kuhn_tet_mesh(6, 0.08, 231)   # affine source: reproduced exactly
    got = _gpu_supermesh(tm, sm, fields.evaluate("affine", np, sm[0]))
    assert np.abs(got["x"] - fields.evaluate("affine", np, tm[0])).max() < 1e-12
    # a target reaching outside the source
    tc, tconn = meshes.kuhn_tet_mesh(4, 0.08, 232)
    tm2 = (tc * 1.2 - 0.1, tconn)
    sm = meshes.kuhn_tet_mesh(5, 0.08, 235)
    sv = fields.evaluate("gaussian_bumps_3d", np, sm[0])
    got = _gpu_supermesh(tm2, sm, sv)
    ref = supermesh3d.supermesh_projection(*tm2, *sm, sv)
    assert rel_l2(got["b"], ref["b"]) < 1e-12
    assert np.abs(got["area"] - ref["vol_sum"]).max() < 1e-14
    vol = geometry.element_measures(tm2[0], np.asarray(tconn, dtype=np.int64))
    partial = int((ref["vol_sum"] < vol * (1 - 1e-12)).sum())
    assert partial > 0 and got["reports"][0]["n_out_of_domain"] == partial


def test_monte_carlo_mean_converges_to_supermesh3d():
    """The tetrahedral CV-MC load vector is unbiased: its mean over R
    realizations approaches the exact b within a few standard errors."""
    tm, sm = meshes.kuhn_tet_mesh(4, 0.08, 233), meshes.kuhn_tet_mesh(5, 0.08, 234)
    sv = fields.evaluate("gaussian_bumps_3d", np, sm[0])
    exact = _gpu_supermesh(tm, sm, sv)["b"][0]
    T = ft.Target(*tm)
    S = ft.Source(*sm, sv)
    bs = []
    for r in range(200):
        T.transfer_from(S, ft.SampleCfg(16, 1, 0.5, SEED, 300 + r, ft.FT_F64))
        bs.append(T.project(1).b[0].cpu().numpy())
    bs = np.array(bs)
    z = np.abs(bs.mean(axis=0) - exact) / (bs.std(axis=0, ddof=1) / np.sqrt(len(bs)))
    log(f"3D MC mean vs supermesh: max z {z.max():.2f} over {z.size} nodes")
    assert z.max() < 5.0
    assert np.mean(z ** 2) < 1.5
    T.close()
    S.close()


def test_monte_carlo_mean_converges_to_supermesh():
    """The CV-MC load vector is unbiased: over R independent realizations its
    mean approaches the exact b within a few standard errors at every node
    (alpha = 0.5, so the residual has spread), and the error of the mean
    shrinks like 1/sqrt(R)."""
    tm, sm = meshes.delaunay_tri_mesh(8, 0.3, 136), meshes.delaunay_tri_mesh(11, 0.3, 137)
    sv = fields.evaluate("paper_f2", np, sm[0])
    exact = _gpu_supermesh(tm, sm, sv)["b"][0]
    T = ft.Target(*tm)
    S = ft.Source(*sm, sv)
    R = 200
    bs = []
    for r in range(R):
        T.transfer_from(S, ft.SampleCfg(16, 1, 0.5, SEED, r, ft.FT_F64))
        bs.append(T.project(1).b[0].cpu().numpy())
    bs = np.array(bs)
    mean, sd = bs.mean(axis=0), bs.std(axis=0, ddof=1)
    z = np.abs(mean - exact) / (sd / np.sqrt(R))
    log(f"MC mean vs supermesh: max z {z.max():.2f} over {z.size} nodes")
    assert z.max() < 5.0
    assert np.mean(z ** 2) < 1.5   # about 1 for an unbiased estimator
    T.close()
    S.close()


def test_fullsize_supermesh_reference():
    """tri2d_1m: the exact b of the 1M-triangle target from the 4M-triangle
    source; the Monte Carlo b of one realization deviates from it by as much
    as two realizations deviate from each other divided by sqrt 2 (no bias),
    and sum b equals the source integral."""
    w = configs.WORKLOADS["tri2d_1m"]
    tm = configs.build_mesh(w.target)
    sm = configs.build_mesh(w.source)
    sv = configs.source_nodal_values(w, sm[0])
    log("full-size supermesh: tri2d_1m")
    T = ft.Target(*tm)
    S = ft.Source(*sm, sv, bins=w.bins[:2])
    area = T.transfer_supermesh(S, area=True)
    r = T.project(1)
    exact = r.b[0].cpu().numpy()
    vol = geometry.element_measures(tm[0], np.asarray(tm[1], dtype=np.int64))
    assert np.abs(area.cpu().numpy() - vol).max() <= 1e-12 * vol.max()
    assert r.reports[0]["n_out_of_domain"] == 0
    I = S.integral()[0]
    assert abs(exact.sum() - I) <= 1e-12 * abs(I)
    bs = []
    for stream in (0, 1):
        T.transfer_from(S, ft.SampleCfg(w.samples_per_elem, 1, w.alpha, w.philox_seed, stream, ft.FT_F64))
        bs.append(T.project(1).b[0].cpu().numpy())
    err = np.linalg.norm(bs[0] - exact)
    spread = np.linalg.norm(bs[0] - bs[1]) / np.sqrt(2.0)
    log(f"  |b_MC - b_exact| {err:.3e}, spread/sqrt2 {spread:.3e}, rel {err / np.linalg.norm(exact):.3e}")
    assert 0.9 < err / spread < 1.1
    T.close()
    S.close()
