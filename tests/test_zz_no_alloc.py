"""The entry point that allocates nothing, ft_consume_queries_noalloc, against
ft_consume_queries: on the same target and the same query values both must
give bitwise the same load vector and solution (the same kernels in the same
order; only where the element loads wait between the element kernel and the
node assembly differs).  Each case makes two no-allocation calls in a row,
the second on a smaller input, so the second runs on what the first left in
the shared scratch array."""
import ctypes

import numpy as np
import pytest

from gpu_cases import log
from paper_2603_00538_amd import ft
from workloads import fields, meshes

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _transfer(T, S, cfg, noalloc):
    pts = T.sample_points(cfg)
    vals = S.eval_query_list(pts, T.n_nodes)
    T.consume(cfg, vals, noalloc=noalloc)
    res = T.project(cfg.n_fields, rtol=1e-14, max_iter=500)
    torch.cuda.synchronize()
    return res.x.cpu().numpy(), res.b.cpu().numpy(), res.reports, res.status


def _pair(dim, kt, ks, seed):
    if dim == 2:
        return meshes.delaunay_tri_mesh(kt, 0.3, seed), meshes.delaunay_tri_mesh(ks, 0.3, seed + 1)
    return meshes.kuhn_tet_mesh(kt, 0.08, seed), meshes.kuhn_tet_mesh(ks, 0.08, seed + 1)


def _values(dim, sc, F):
    if F == 1:
        return fields.evaluate("front_2d" if dim == 2 else "gaussian_bumps_3d", np, sc)
    vals = fields.fourier_fields_3d(np, sc[:, 0], sc[:, 1], sc[:, 2], fields.fourier_modes(n_fields=F))
    return np.ascontiguousarray(vals)


# (dim, target size, source size, N, fields, precision): large call, then a smaller one
CASES = [
    ("2d-f64", [(2, 40, 55, 64, 1, ft.FT_F64), (2, 14, 20, 37, 1, ft.FT_F64)]),
    ("3d-f32", [(3, 9, 12, 128, 1, ft.FT_F32), (3, 5, 7, 16, 1, ft.FT_F32)]),
    ("3d-split", [(3, 7, 9, 128, 8, ft.FT_SPLIT_F16), (3, 5, 7, 40, 8, ft.FT_SPLIT_BF16)]),
]


@pytest.mark.parametrize("name,calls", CASES, ids=[c[0] for c in CASES])
def test_noalloc_consume_matches_consume(name, calls):
    for i, (dim, kt, ks, N, F, prec) in enumerate(calls):
        log(f"no-alloc consume {name} call {i + 1}: dim={dim} target k={kt} N={N} F={F} precision={prec}")
        tm, sm = _pair(dim, kt, ks, 400 + 10 * i)
        sv = _values(dim, sm[0], F)
        S = ft.Source(*sm, sv)
        cfg = ft.SampleCfg(N, F, 1.0, 0x0F7A5EED000000A0 + i, 5, prec)
        # the no-allocation call first, on a new target (one field provisioned
        # at creation); many fields need one ordinary consume to size the buffers
        T1 = ft.Target(*tm)
        if F > 1:
            _transfer(T1, S, cfg, noalloc=False)
        x1, b1, r1, s1 = _transfer(T1, S, cfg, noalloc=True)
        T2 = ft.Target(*tm)
        x2, b2, r2, s2 = _transfer(T2, S, cfg, noalloc=False)
        assert s1 == s2 == ft.FT_OK
        assert np.array_equal(b1, b2), f"load vectors differ by {np.abs(b1 - b2).max():.3e}"
        assert np.array_equal(x1, x2)
        for a, b in zip(r1, r2):
            assert a["iters"] == b["iters"] and a["sum_b"] == b["sum_b"] and a["n_nonfinite"] == 0
        T1.close()
        T2.close()
        S.close()


def test_noalloc_consume_rejections():
    tm, sm = _pair(3, 10, 12, 470)
    log(f"no-alloc consume rejections: {tm[1].shape[0]} tetrahedra")
    T = ft.Target(*tm)
    lib = ft.load()
    stream = ft.current_stream()
    dummy = torch.zeros(8, dtype=torch.float64, device="cuda")
    # no samples drawn yet: out of order
    cfg = ft.SampleCfg(16, 1, 1.0, 9, 0, ft.FT_F64)
    st = lib.ft_consume_queries_noalloc(T.handle, ctypes.byref(cfg), ctypes.c_void_p(dummy.data_ptr()), stream)
    assert st == ft.FT_E_ORDER
    T.sample_points(cfg)
    # element loads beyond the 64 MiB array: F fields x E tetrahedra x 4 vertices x 8 B
    E = tm[1].shape[0]
    F_big = (64 << 20) // (E * 4 * 8) + 1
    big = ft.SampleCfg(16, F_big, 1.0, 9, 0, ft.FT_F64)
    st = lib.ft_consume_queries_noalloc(T.handle, ctypes.byref(big), ctypes.c_void_p(dummy.data_ptr()), stream)
    assert st == ft.FT_E_ARG and b"scratch" in lib.ft_last_error()
    # more fields than the target's buffers (one at creation)
    two = ft.SampleCfg(16, 2, 1.0, 9, 0, ft.FT_F64)
    st = lib.ft_consume_queries_noalloc(T.handle, ctypes.byref(two), ctypes.c_void_p(dummy.data_ptr()), stream)
    assert st == ft.FT_E_ARG and b"field" in lib.ft_last_error()
    torch.cuda.synchronize()
    T.close()
