"""Pins of the oracle's Philox4x32-10 and its uniform conversions."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import philox, sampling

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand/rocrand_kernel.h"):
        pytest.skip("hipcc or rocRAND headers not available")
    exe = tmp_path_factory.mktemp("rr") / "philox_words"
    src = os.path.join(HERE, "rocrand_philox_words.cpp")
    # host-only program: rocRAND's engine is host-callable; the device part is empty
    subprocess.run([hipcc, "-O1", "-x", "hip", "--offload-arch=gfx950", src, "-o", str(exe)],
                   check=True, capture_output=True, timeout=300)
    return str(exe)


def test_philox_matches_rocrand_engine(rocrand_ref):
    rng = np.random.default_rng(0)
    seeds = [0, 1, 0xFFFFFFFFFFFFFFFF, 0x0F7A5EED00000002] + [int(s) for s in rng.integers(0, 2**63, 4)]
    cases = []
    for s in seeds:
        for sub in (0, 1, 0x500000003, 0xFFFFFFFFFFFFFFFF, int(rng.integers(0, 2**63))):
            for blk in (0, 3, 0x100000002, int(rng.integers(0, 2**62))):
                cases.append((s, sub, blk))
    inp = "".join(f"{s} {sub} {4 * blk}\n" for s, sub, blk in cases)
    out = subprocess.run([rocrand_ref], input=inp, capture_output=True, text=True, check=True, timeout=60)
    ref = [[int(w, 16) for w in line.split()] for line in out.stdout.strip().splitlines()]
    assert len(ref) == len(cases)
    for (s, sub, blk), r in zip(cases, ref):
        k0, k1 = philox.key_from_seed(s)
        w = philox.philox4x32_10(blk & 0xFFFFFFFF, blk >> 32, sub & 0xFFFFFFFF, sub >> 32, k0, k1)
        assert [int(v) for v in w] == r, (s, sub, blk)


def test_uniform53_exact_open_interval():
    a = np.array([0, 0, 0xFFFFFFFF, 0x80000000, 0x12345678], dtype=np.uint32)
    b = np.array([0, 0xFFF, 0xFFFFFFFF, 0, 0x9ABCDEF0], dtype=np.uint32)
    u = philox.uniform53(a, b)
    m = ((a.astype(object) << 32) | b.astype(object)) >> 12
    for ui, mi in zip(u, m):
        # (2m+1) 2^-53 is exactly representable: reconstruct the integer exactly
        assert float(ui) * 2.0 ** 53 == float(2 * mi + 1)
    assert u.min() == 2.0 ** -53 and u.max() == 1.0 - 2.0 ** -53
    assert np.all((u > 0) & (u < 1))


def test_uniform24_consistent_with_uniform53():
    rng = np.random.default_rng(1)
    a = rng.integers(0, 2**32, 10000, dtype=np.uint64).astype(np.uint32)
    b = rng.integers(0, 2**32, 10000, dtype=np.uint64).astype(np.uint32)
    u53 = philox.uniform53(a, b)
    u24 = philox.uniform24(a, b)
    assert u24.dtype == np.float32
    assert np.all((u24 > 0) & (u24 < 1))
    assert np.abs(u24.astype(np.float64) - u53).max() <= 2.0 ** -24


def test_uniforms_distribution_ks():
    """Kolmogorov-Smirnov test of every uniform stream used by the sampler."""
    from scipy import stats

    t = np.repeat(np.arange(2000), 100)
    j = np.tile(np.arange(100), 2000)
    u = sampling.uniforms(3, t, j, seed=0x0F7A5EED00000001, stream=7)
    for c in range(3):
        assert stats.kstest(u[:, c], "uniform").pvalue > 1e-4
    # the three coordinates are uncorrelated
    cc = np.corrcoef(u.T)
    assert np.abs(cc - np.eye(3)).max() < 5.0 / np.sqrt(u.shape[0])
