"""Per-element uniform samples (oracle side).

Follows sec. 4.1: uniform density p_t = 1/|Omega_t| on each target element,
N independent samples per element (uniform-density estimator), drawn per
algorithm step 3 as two independent U(0,1) scalars mapped to area-uniform
barycentric weights by the map of Osada et al. (2002) and then mapped to the
physical element by the affine element map.

Reading for tetrahedra (the paper gives no 3D rule): three independent U(0,1)
scalars are sorted, s1 <= s2 <= s3, and the spacings
(s1, s2-s1, s3-s2, 1-s3) are the barycentric weights; uniform spacings are
Dirichlet(1,1,1,1), i.e. uniform on the tetrahedron.

Reading for d-simplices, d = 4..6 (sec. 2 states the formulation for any
dimension and sec. 7 names 5D/6D transfers): the same sorted-spacings map
with d uniforms, (s1, s2-s1, ..., sd-s(d-1), 1-sd) ~ Dirichlet(1, ..., 1).

Counter layout (one Philox4x32-10 block per 2D sample, two per 3D sample,
ceil(d/2) per d-simplex sample): counter = (j, t, stream, blk), key =
(seed_lo, seed_hi), where t is the target element index, j the sample index
within the element.
  2D: blk 0 words (0,1) -> xi, words (2,3) -> eta;
      lambda = (1 - sqrt(xi), sqrt(xi) (1 - eta), sqrt(xi) eta).
  d >= 3: uniform u_(i+1) from blk i/2, words (0,1) for even i and (2,3) for
      odd i (3D: blk 0 words (0,1) -> u1, (2,3) -> u2; blk 1 words (0,1) -> u3).
lambda_k multiplies vertex k of the element in connectivity order.

Stratified (jittered) variant, a reading of the paper's suggestion of
better sampling schemes (sec. 7): the d' = d uniforms of a sample are
stratified over the unit cube before the same maps.  With m = floor(N^(1/d')) cells per axis, sample j < m^d' of an
element takes cell j (digits c_i = floor(j / m^i) mod m, lowest first) and
u_i <- min((c_i + u_i) * (1/m), 1 - 2^-53), the same Philox uniform u_i
placed in that cell; samples j >= m^d' stay plain.  Both maps are
measure-preserving from the unit cube onto the simplex (the spacings map is
6-to-1), so each sample is uniform on the image of its cell, the cells have
equal volume, and the estimator stays unbiased; each element's first m^d'
samples cover all cells once.  1/m is rounded once and the clamp keeps the
result in (0, 1): the GPU computes the same expression in the same order.

Parity: pinned by closed-form simplex moments and an equal-volume chi-square
test (uniformity), plus exactness of the affine identity sum(lambda) = 1;
the stratified variant by its one-sample-per-cell structure (exact), the
same moments, unbiased estimates and a smaller variance than plain sampling.
"""
from __future__ import annotations

import numpy as np

from . import philox


def uniforms(dim: int, t: np.ndarray, j: np.ndarray, seed: int, stream: int):
    """The d open-interval doubles of sample (t, j); returns (n, d)."""
    k0, k1 = philox.key_from_seed(seed)
    t = np.asarray(t, dtype=np.uint32)
    j = np.asarray(j, dtype=np.uint32)
    s = np.uint32(stream)
    u = []
    for blk in range((dim + 1) // 2):
        w = philox.philox4x32_10(j, t, s, np.uint32(blk), k0, k1)
        u.append(philox.uniform53(w[0], w[1]))
        if len(u) < dim:
            u.append(philox.uniform53(w[2], w[3]))
    return np.stack(u, axis=1)


def strata_per_axis(dim: int, n_samples: int) -> int:
    """m = floor(N^(1/d')) with d' = dim uniforms per sample, exactly."""
    dp = dim
    m = max(1, int(round(n_samples ** (1.0 / dp))))
    while m ** dp > n_samples:
        m -= 1
    while (m + 1) ** dp <= n_samples:
        m += 1
    return m


def stratify(dim: int, u: np.ndarray, j: np.ndarray, n_samples: int) -> np.ndarray:
    """Place the uniforms of samples j < m^d' in their cells (see the module text)."""
    m = strata_per_axis(dim, n_samples)
    dp = u.shape[1]
    inv_m = 1.0 / m
    j = np.asarray(j, dtype=np.int64)
    out = u.copy()
    strat = j < m ** dp
    for i in range(dp):
        cell = (j // m ** i) % m
        v = np.minimum((cell.astype(np.float64) + u[:, i]) * inv_m, 1.0 - 2.0 ** -53)
        out[:, i] = np.where(strat, v, u[:, i])
    return out


def barycentric_from_uniforms(dim: int, u: np.ndarray) -> np.ndarray:
    """Map d uniforms to d+1 barycentric weights, uniform on the simplex."""
    if dim == 2:
        # Osada et al. (2002): area-uniform point from (xi, eta)
        xi, eta = u[:, 0], u[:, 1]
        r = np.sqrt(xi)
        return np.stack([1.0 - r, r * (1.0 - eta), r * eta], axis=1)
    if 3 <= dim <= 6:
        s = np.sort(u, axis=1)
        cols = [s[:, 0]] + [s[:, k] - s[:, k - 1] for k in range(1, dim)] + [1.0 - s[:, dim - 1]]
        return np.stack(cols, axis=1)
    raise ValueError("dim must lie in [2, 6]")


def element_samples(dim: int, n_elems: int, n_samples: int, seed: int, stream: int,
                    elems: np.ndarray | None = None, stratified: bool = False) -> np.ndarray:
    """Barycentric weights of every sample of the given elements, shape (len(elems), N, d+1)."""
    if elems is None:
        elems = np.arange(n_elems)
    elems = np.asarray(elems)
    t = np.repeat(elems, n_samples)
    j = np.tile(np.arange(n_samples), elems.size)
    u = uniforms(dim, t, j, seed, stream)
    if stratified:
        u = stratify(dim, u, j, n_samples)
    lam = barycentric_from_uniforms(dim, u)
    return lam.reshape(elems.size, n_samples, dim + 1)


def physical_points(coords: np.ndarray, conn: np.ndarray, lam: np.ndarray,
                    elems: np.ndarray | None = None) -> np.ndarray:
    """Affine element map X = sum_k lambda_k x_{v_k}; lam is (E', N, d+1) -> (E', N, d)."""
    if elems is None:
        elems = np.arange(conn.shape[0])
    verts = coords[conn[elems]]                      # (E', d+1, d)
    return np.einsum("tjk,tkc->tjc", lam, verts)
