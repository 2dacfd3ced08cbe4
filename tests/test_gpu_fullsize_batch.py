"""The batch at its full size (batch256: 256 built-in-source transfers, mixed 2D
and 3D, 1e3-4.5e5 elements each, N in {32, 64, 128, 256}), in the launch
configuration bench.py times (one HIP graph per ft_batch_run).

Every transfer of the batch is checked against the conservation identity, and
a spread of them (the largest 2D and 3D ones, the smallest, and every 37th)
against the single-transfer route (ft_transfer_p1 + ft_project), whose
parity with the oracle the other GPU tests establish: the load vectors agree
to rounding (the element sums are bitwise those of the fused route) and the
solutions to the solver tolerance.
"""
import numpy as np
import pytest

from gpu_cases import log, rel_l2
from paper_2603_00538_amd import ft
from workloads import configs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def batch_full():
    items = configs.batch_items()
    log(f"batch256: building {len(items)} mesh pairs")
    host = []
    for it in items:
        tc, tconn = it.target.build()
        sc, sconn = it.source.build()
        host.append((tc, tconn, sc, sconn, np.ascontiguousarray(it.field(np, sc))))
    targets = [ft.Target(tc, tconn) for tc, tconn, _, _, _ in host]
    sources = [ft.Source(sc, sconn, sv) for _, _, sc, sconn, sv in host]
    cfgs = [ft.SampleCfg(it.samples_per_elem, 1, 1.0, configs.BATCH_PHILOX_SEED, it.stream_id, ft.FT_F64)
            for it in items]
    log("batch256: graph run")
    B = ft.Batch(targets, sources, cfgs, graph=True)
    xs = [torch.empty(t.n_nodes, dtype=torch.float64, device="cuda") for t in targets]
    bs = [torch.empty(t.n_nodes, dtype=torch.float64, device="cuda") for t in targets]
    _, _, reps, sts, st = B.run(rtol=1e-14, max_iter=60, xs=xs, bs=bs)
    torch.cuda.synchronize()
    yield items, targets, sources, cfgs, xs, bs, reps, sts, st
    B.close()
    for h in targets + sources:
        h.close()


def test_fullsize_batch_status_and_conservation(batch_full):
    items, targets, sources, cfgs, xs, bs, reps, sts, st = batch_full
    assert st == ft.FT_OK and all(s == ft.FT_OK for s in sts)
    worst = max(r["cons_defect"] for r in reps)
    log(f"batch256: worst conservation defect {worst:.2e}")
    assert worst < 1e-12


def test_fullsize_batch_matches_single_route(batch_full):
    items, targets, sources, cfgs, xs, bs, reps, sts, st = batch_full
    E = np.array([t.n_elems for t in targets])
    D = np.array([t.dim for t in targets])
    picks = sorted({int(np.argmax(np.where(D == 2, E, 0))), int(np.argmax(np.where(D == 3, E, 0))),
                    int(np.argmin(E)), *range(0, len(targets), 37)})
    for k in picks:
        T, S, cfg = targets[k], sources[k], cfgs[k]
        T.transfer_from(S, cfg)
        r = T.project(1, rtol=1e-14)
        eb = rel_l2(bs[k].cpu().numpy(), r.b[0].cpu().numpy())
        ex = rel_l2(xs[k].cpu().numpy(), r.x[0].cpu().numpy())
        log(f"transfer {k}: dim {T.dim}, {T.n_elems} elements, N={cfg.samples_per_elem}: b {eb:.1e}, x {ex:.1e}")
        assert eb < 1e-15 and ex < 1e-13
