"""The element-tile layout of the query values (FT_VALUES_ELEMENT_TILES):
ft_source_eval_tiles writes exactly the values of ft_source_eval_queries in
the tile order, and ft_consume_queries on tiles gives bitwise the results of
the field-major list, in every consumption form (binary64, binary32, the
matrix-core split forms, each element's own coefficient, the no-allocation
entry point)."""
import numpy as np
import pytest

from gpu_cases import log
from paper_2603_00538_amd import ft
from workloads import fields, meshes

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SEED = 0x0F7A5EED00000100


def _case(dim, F):
    if dim == 2:
        tm, sm = meshes.delaunay_tri_mesh(10, 0.3, 151), meshes.delaunay_tri_mesh(14, 0.3, 152)
        sc = sm[0]
        sv = np.stack([np.sin((f + 1) * sc[:, 0]) + np.cos((f + 2) * sc[:, 1]) for f in range(F)])
    else:
        tm, sm = meshes.kuhn_tet_mesh(5, 0.08, 153), meshes.kuhn_tet_mesh(7, 0.08, 154)
        sv = fields.fourier_fields_3d(np, sm[0][:, 0], sm[0][:, 1], sm[0][:, 2],
                                      fields.fourier_modes(seed=9, n_fields=F, n_modes=4, kmax=3))
    return tm, sm, np.ascontiguousarray(sv)


def _to_tiles(vals, n, E, N):
    """Field-major (F, Q) values -> the element-tile order (flat)."""
    F = vals.shape[0]
    nodes = vals[:, :n].reshape(-1)
    samples = vals[:, n:].reshape(F, E, N).transpose(1, 0, 2).reshape(-1)
    return np.concatenate([nodes, samples])


@pytest.mark.parametrize("dim,F,N,dtype", [(2, 5, 64, "f64"), (2, 17, 37, "f32"), (3, 64, 128, "f32"),
                                           (3, 3, 20, "f64"), (2, 1, 16, "f64")])
def test_eval_tiles_is_the_query_list_in_tile_order(dim, F, N, dtype):
    tm, sm, sv = _case(dim, F)
    T = ft.Target(*tm)
    S = ft.Source(*sm, sv)
    prec = ft.FT_F64 if dtype == "f64" else ft.FT_F32
    cfg = ft.SampleCfg(N, F, 1.0, SEED, 0, prec)
    pts = T.sample_points(cfg)
    log(f"eval tiles dim={dim} F={F} N={N} {dtype}")
    ids_a = torch.empty(pts.shape[1], dtype=torch.int32, device="cuda")
    ids_b = torch.empty_like(ids_a)
    fm = S.eval_query_list(pts, T.n_nodes, ids=ids_a).cpu().numpy()
    tl = S.eval_tiles(pts, T.n_nodes, T.n_elems, N, ids=ids_b).cpu().numpy()
    assert np.array_equal(tl, _to_tiles(fm, T.n_nodes, T.n_elems, N))
    assert torch.equal(ids_a, ids_b)
    T.close()
    S.close()


@pytest.mark.parametrize("dim,F,N,prec,own", [(2, 3, 64, ft.FT_F64, False), (3, 5, 37, ft.FT_F32, False),
                                              (3, 64, 128, ft.FT_SPLIT_F16, False),
                                              (2, 40, 100, ft.FT_SPLIT_BF16, False),
                                              (2, 4, 48, ft.FT_F64, True), (3, 2, 64, ft.FT_F32, True)])
def test_consume_tiles_equals_field_major(dim, F, N, prec, own):
    tm, sm, sv = _case(dim, F)
    S = ft.Source(*sm, sv)
    log(f"consume tiles dim={dim} F={F} N={N} precision={prec} own alpha={own}")
    out = {}
    for layout in (ft.FT_VALUES_FIELD_MAJOR, ft.FT_VALUES_ELEMENT_TILES):
        for noalloc in (False, True):
            T = ft.Target(*tm)
            cfg = ft.SampleCfg(N, F, 1.0, SEED, 1, prec)
            cfg.alpha_mode = ft.FT_ALPHA_ELEMENT if own else ft.FT_ALPHA_FIXED
            cfg.values_layout = layout
            pts = T.sample_points(cfg)
            if layout == ft.FT_VALUES_ELEMENT_TILES:
                vals = S.eval_tiles(pts, T.n_nodes, T.n_elems, N)
            else:
                vals = S.eval_query_list(pts, T.n_nodes)
            if noalloc:
                if F > 1:
                    T.consume(cfg, vals)   # sizes the target's field buffers
                T.consume(cfg, vals, noalloc=True)
            else:
                T.consume(cfg, vals)
            r = T.project(F)
            out[layout, noalloc] = (r.b.cpu().numpy(), r.x.cpu().numpy(), r.status)
            T.close()
    ref = out[ft.FT_VALUES_FIELD_MAJOR, False]
    assert ref[2] == ft.FT_OK
    for k, v in out.items():
        assert np.array_equal(v[0], ref[0]), k
        assert np.array_equal(v[1], ref[1]), k
    S.close()
