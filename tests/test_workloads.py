"""The seeded input generators (shared by the oracle tests and the GPU path)."""
import numpy as np

from workloads import configs, meshes


def test_batch_items_follow_the_recipe():
    a = configs.batch_items()
    b = configs.batch_items()
    assert a == b                                    # seeded: identical on every call
    assert len(a) == 256
    E = np.array([2 * (i.target.k - 1) ** 2 if i.dim == 2 else 6 * (i.target.k - 1) ** 3 for i in a])
    Es = np.array([2 * (i.source.k - 1) ** 2 if i.dim == 2 else 6 * (i.source.k - 1) ** 3 for i in a])
    assert E.min() >= 500 and E.max() <= 6e5
    ratio = Es / E
    assert ratio.min() > 1.4 and ratio.max() < 5.2   # sources 2-4x finer, up to grid rounding (small 3D grids)
    # log-uniform sizes: the median of log E sits near the middle of [ln 1e3, ln 5e5]
    mid = 0.5 * (np.log(1e3) + np.log(5e5))
    assert abs(np.median(np.log(E)) - mid) < 0.6
    assert 90 < sum(i.dim == 2 for i in a) < 166
    assert {i.samples_per_elem for i in a} == {32, 64, 128, 256}
    assert [i.stream_id for i in a] == list(range(256))
    for i in a:
        assert all(any(k) for k in i.kvec) and len(i.kvec) == 4


def test_batch_field_has_unit_mean():
    """Every mode has a nonzero integer wave vector, so the field integrates to 1."""
    it = configs.batch_items()[3]
    tc, tconn = meshes.make_mesh(it.target.kind, 40 if it.dim == 2 else 14, 0.0, 1)
    rng = np.random.default_rng(0)
    X = rng.uniform(0.0, 1.0, size=(400000, it.dim))
    v = it.field(np, X)[0]
    assert abs(v.mean() - 1.0) < 4 * v.std() / np.sqrt(X.shape[0])
