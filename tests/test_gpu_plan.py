"""GPU parity of the setup/online split (ft_plan_create / ft_plan_transfer)
and of repeated round trips between two meshes built on it."""
import numpy as np
import pytest

from gpu_cases import log, oracle_transfer, rel_l2
from oracle import geometry
from oracle.source import P1Source
from paper_2603_00538_amd import ft
from workloads import fields, meshes

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SEED = 0x0F7A5EED000000C0


@pytest.mark.parametrize("dim,N", [(2, 64), (2, 20), (3, 16), (3, 128)])
def test_plan_equals_fused_route(dim, N):
    """With the source's own values the online half is bitwise ft_transfer_p1."""
    if dim == 2:
        tm, sm = meshes.delaunay_tri_mesh(12, 0.3, 61), meshes.delaunay_tri_mesh(17, 0.3, 62)
        sv = fields.evaluate("front_2d", np, sm[0])
    else:
        tm, sm = meshes.kuhn_tet_mesh(6, 0.08, 63), meshes.kuhn_tet_mesh(8, 0.08, 64)
        sv = fields.evaluate("gaussian_bumps_3d", np, sm[0])
    T = ft.Target(*tm)
    S = ft.Source(*sm, sv)
    cfg = ft.SampleCfg(N, 1, 1.0, SEED, 2, ft.FT_F64)
    T.transfer_from(S, cfg)
    ref = T.project(1)
    plan = ft.Plan(T, S, cfg)
    for _ in range(2):
        plan.transfer()
        got = T.project(1)
        assert torch.equal(got.b, ref.b)
        assert torch.equal(got.x, ref.x)
    plan.close()
    T.close()
    S.close()


def test_plan_new_values_match_oracle():
    """New nodal values on the same source mesh: the online half against the oracle."""
    tm, sm = meshes.delaunay_tri_mesh(14, 0.3, 65), meshes.delaunay_tri_mesh(20, 0.3, 66)
    sv1 = fields.evaluate("front_2d", np, sm[0])
    sv2 = fields.evaluate("smooth_2d", np, sm[0])
    T = ft.Target(*tm)
    S = ft.Source(*sm, sv1)
    cfg = ft.SampleCfg(48, 1, 1.0, SEED, 3, ft.FT_F64)
    plan = ft.Plan(T, S, cfg)
    for sv in (sv2, sv1, sv2):
        plan.transfer(torch.as_tensor(np.ascontiguousarray(sv), device="cuda"))
        got = T.project(1)
        o = oracle_transfer(tm, sm, sv, 48, 1.0, SEED, 3)
        assert rel_l2(got.b.cpu().numpy(), o["b"]) < 1e-12
        assert rel_l2(got.x.cpu().numpy(), o["x"]) < 1e-12
    plan.close()
    T.close()
    S.close()


def test_round_trips_match_oracle_and_conserve():
    """Mesh A -> B -> A, twice (sec. 5.2's repeated transfer between two meshes),
    each leg with its own fixed samples, against the oracle doing the same legs."""
    mA, mB = meshes.delaunay_tri_mesh(13, 0.3, 67), meshes.delaunay_tri_mesh(18, 0.3, 68)
    fA = fields.evaluate("smooth_2d", np, mA[0])
    TA, TB = ft.Target(*mA), ft.Target(*mB)
    SA, SB = ft.Source(*mA, fA), ft.Source(*mB, np.zeros((1, mB[0].shape[0])))
    cab = ft.SampleCfg(32, 1, 1.0, SEED, 10, ft.FT_F64)
    cba = ft.SampleCfg(32, 1, 1.0, SEED, 11, ft.FT_F64)
    pab, pba = ft.Plan(TB, SA, cab), ft.Plan(TA, SB, cba)
    mass_A = geometry.lumped_mass(*mA)
    cur_gpu = torch.as_tensor(np.ascontiguousarray(fA), device="cuda")
    cur_or = np.atleast_2d(fA)
    for trip in range(2):
        pab.transfer(cur_gpu)
        rB = TB.project(1)
        oB = oracle_transfer(mB, None, None, 32, 1.0, SEED, 10, query=P1Source(*mA, cur_or))
        eB = rel_l2(rB.x.cpu().numpy(), oB["x"])
        pba.transfer(rB.x.contiguous())
        rA = TA.project(1)
        oA = oracle_transfer(mA, None, None, 32, 1.0, SEED, 11, query=P1Source(*mB, oB["x"]))
        eA = rel_l2(rA.x.cpu().numpy(), oA["x"])
        log(f"round trip {trip + 1}: x_B rel l2 {eB:.2e}, x_A rel l2 {eA:.2e}")
        assert eB < 1e-12 and eA < 1e-12
        for r in (rB, rA):
            assert r.reports[0]["cons_defect"] < 1e-13
        # the integral after the trip stays within the Monte Carlo error of the start
        i0 = float(mass_A @ np.atleast_2d(fA)[0])
        i1 = float(mass_A @ rA.x.cpu().numpy()[0])
        assert abs(i1 - i0) < 1e-2 * abs(i0)
        cur_gpu = rA.x.contiguous()
        cur_or = oA["x"]
    for h in (pab, pba, TA, TB, SA, SB):
        h.close()
