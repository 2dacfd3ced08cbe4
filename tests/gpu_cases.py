"""Shared helpers of the GPU parity tests: run a transfer through the C ABI and
the same transfer through the oracle, on the same seeded inputs."""
from __future__ import annotations

import sys
import time

import numpy as np

from oracle import cvmc, sampling
from oracle.source import P1Source
from paper_2603_00538_amd import ft


def log(msg):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


def gpu_transfer(tmesh, smesh, svals, N, alpha=1.0, seed=7, stream=0, precision=ft.FT_F64, bins=None,
                 rtol=1e-14, max_iter=500, black_box=None, refine_steps=0):
    """Whole transfer through libft.  black_box: optional callable on the (d, Q)
    device points returning (F, Q) device values (replaces the built-in source).
    refine_steps > 0 solves with binary32 inner PCG and that many binary64
    refinement steps."""
    import torch

    tc, tconn = tmesh
    T = ft.Target(tc, tconn)
    S = None
    F = 1
    cfg = None
    if black_box is None:
        sc, sconn = smesh
        S = ft.Source(sc, sconn, svals, bins=bins)
        F = S.n_fields
    cfg = ft.SampleCfg(N, F, alpha, seed, stream, precision)
    pts = T.sample_points(cfg)
    ids = torch.full((pts.shape[1],), -7, dtype=torch.int32, device=pts.device)
    if black_box is None:
        vals = S.eval_query_list(pts, tc.shape[0], ids=ids)
    else:
        vals = black_box(pts)
        F = vals.shape[0]
        cfg.n_fields = F
    T.consume(cfg, vals)
    res = T.project(F, rtol=rtol, max_iter=max_iter, refine_steps=refine_steps)
    torch.cuda.synchronize()
    out = {
        "points": pts.double().cpu().numpy(), "values": vals.double().cpu().numpy(), "ids": ids.cpu().numpy(),
        "x": res.x.cpu().numpy(), "b": res.b.cpu().numpy(), "reports": res.reports, "status": res.status,
        "info": T.info, "ood": S.take_out_of_domain() if S is not None else 0,
    }
    T.close()
    if S is not None:
        S.close()
    return out


def oracle_transfer(tmesh, smesh, svals, N, alpha=1.0, seed=7, stream=0, query=None):
    tc, tconn = tmesh
    if query is None:
        sc, sconn = smesh
        query = P1Source(sc, sconn, svals)
    t0 = time.time()
    r = cvmc.transfer(tc, tconn, query, N, alpha=alpha, seed=seed, stream=stream)
    r["seconds"] = time.time() - t0
    return r


def oracle_query_points(tmesh, N, seed, stream):
    """The oracle's point-query list (d, Q): nodes, then samples element-major."""
    tc, tconn = tmesh
    dim = tc.shape[1]
    lam = sampling.element_samples(dim, tconn.shape[0], N, seed, stream)
    X = sampling.physical_points(tc, np.asarray(tconn, dtype=np.int64), lam)
    return np.ascontiguousarray(np.concatenate([tc, X.reshape(-1, dim)], axis=0).T)


def rel_l2(a, b):
    return cvmc.rel_l2(a, b)
