"""Named synthetic transfer workloads.

Each workload is a seeded (target mesh, source mesh, source field, sampling)
tuple.  The paper's gmsh/LTX/WEST meshes are unavailable; these stand in with
the same element types and the size range the paper times (1e3 to 2.3e6
elements).  Sizes:

======================  ===  ==================  =========  ===================  ==========  ====  ==
name                    dim  target             E          source               E_s         N     F
======================  ===  ==================  =========  ===================  ==========  ====  ==
tri2d_4k                2    Delaunay 45^2       3,872      Delaunay 70^2        9,522       64    1
tri2d_1m                2    structured 708^2    999,698    structured 1415^2    3,998,792   256   1
tet3d_2m                3    Kuhn 71^3 nodes     2,058,000  Kuhn 111^3 nodes     7,986,000   128   1
tet3d_1m_64f            3    Kuhn 56^3 nodes     998,250    Kuhn 88^3 nodes      3,951,018   128   64
tri2d_1m_p2             2    as tri2d_1m, P2     999,698    as tri2d_1m          3,998,792   256   1
tet3d_2m_p2             3    as tet3d_2m, P2     2,058,000  as tet3d_2m          7,986,000   128   1
kuhn5d_1m               5    Kuhn 7^5 nodes      933,120    analytic black box   -           64    1
kuhn6d_500k             6    Kuhn 4^6 nodes      524,880    analytic black box   -           64    1
======================  ===  ==================  =========  ===================  ==========  ====  ==

The 5D and 6D workloads (distribution-function-like transfers, sec. 7) have
no source mesh: the field ``phase_space`` is the point-query black box
itself, evaluated at the query points.

Seeds: target jitter 11, source jitter 12, field parameters 13, Philox key
``0x0F7A5EED00000000 + index``.

Batch workload (``batch_items``): 256 transfers whose target sizes are
log-uniform in [1e3, 5e5] elements, 2D (structured triangles) or 3D (Kuhn
tetrahedra) by a fair coin, each with its own source mesh 2-4 times finer
(element count), its own smooth field 1 + 0.5 sum_q a_q cos(2 pi k_q.x + phi_q)
(4 modes, k_q in {0,1,2}^d without 0, a_q ~ N(0,1), phi_q ~ U[0, 2 pi)) and N
drawn from {32, 64, 128, 256}.  Seed 14; Philox key base + 5, stream id =
transfer index.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from functools import lru_cache

import numpy as np

from . import fields as _fields
from . import meshes as _meshes

PHILOX_SEED_BASE = 0x0F7A5EED00000000


@dataclass(frozen=True)
class MeshSpec:
    kind: str          # structured_tri | delaunay_tri | kuhn_tet | kuhn<d>d
    k: int             # nodes per axis
    jitter: float      # fraction of the grid spacing
    seed: int

    def build(self):
        return _meshes.make_mesh(self.kind, self.k, self.jitter, self.seed)


@dataclass(frozen=True)
class Workload:
    name: str
    dim: int
    target: MeshSpec
    source: MeshSpec | None     # None: the field itself is the black box
    field: str
    samples_per_elem: int
    n_fields: int = 1
    alpha: float = 1.0
    index: int = 0
    bins: tuple = (0, 0, 0)      # 0 = library default
    rtol: float = 1e-14
    order: int = 1               # target elements: 1 (P1) or 2 (P2, midpoints added by meshes.p2_mesh)

    @property
    def philox_seed(self) -> int:
        return PHILOX_SEED_BASE + self.index


WORKLOADS = {
    "tri2d_4k": Workload(
        "tri2d_4k", 2,
        MeshSpec("delaunay_tri", 45, 0.3, 11), MeshSpec("delaunay_tri", 70, 0.3, 12),
        "smooth_2d", 64, index=1),
    "tri2d_1m": Workload(
        "tri2d_1m", 2,
        MeshSpec("structured_tri", 708, 0.2, 11), MeshSpec("structured_tri", 1415, 0.2, 12),
        "front_2d", 256, index=2, bins=(512, 512, 0)),
    "tet3d_2m": Workload(
        "tet3d_2m", 3,
        MeshSpec("kuhn_tet", 71, 0.08, 11), MeshSpec("kuhn_tet", 111, 0.08, 12),
        "gaussian_bumps_3d", 128, index=3),
    "tet3d_1m_64f": Workload(
        "tet3d_1m_64f", 3,
        MeshSpec("kuhn_tet", 56, 0.08, 11), MeshSpec("kuhn_tet", 88, 0.08, 12),
        "fourier_fields_3d", 128, n_fields=64, index=4),
    # the same meshes with quadratic target elements
    "tri2d_1m_p2": Workload(
        "tri2d_1m_p2", 2,
        MeshSpec("structured_tri", 708, 0.2, 11), MeshSpec("structured_tri", 1415, 0.2, 12),
        "front_2d", 256, index=6, bins=(512, 512, 0), order=2),
    "tet3d_2m_p2": Workload(
        "tet3d_2m_p2", 3,
        MeshSpec("kuhn_tet", 71, 0.08, 11), MeshSpec("kuhn_tet", 111, 0.08, 12),
        "gaussian_bumps_3d", 128, index=7, order=2),
    # phase-space transfers: d-simplices of the unit hypercube, an analytic black box
    "kuhn5d_1m": Workload(
        "kuhn5d_1m", 5, MeshSpec("kuhn5d", 7, 0.03, 11), None, "phase_space", 64, index=8),
    "kuhn6d_500k": Workload(
        "kuhn6d_500k", 6, MeshSpec("kuhn6d", 4, 0.03, 11), None, "phase_space", 64, index=9),
}


def target_mesh(w: Workload):
    """The workload's target mesh: P1 as built, or with edge nodes for P2."""
    coords, conn = build_mesh(w.target)
    if w.order == 1:
        return coords, conn
    return _meshes.p2_mesh(coords, conn)


@lru_cache(maxsize=8)
def build_mesh(spec: MeshSpec):
    coords, conn = spec.build()
    coords.setflags(write=False)
    conn.setflags(write=False)
    return coords, conn


def field_integral(w: Workload):
    """The exact integral of an analytic black-box field over the unit hypercube
    (None where no closed form is coded)."""
    if w.field == "phase_space":
        return _fields.phase_space_integral(w.dim)
    return None


def source_nodal_values(w: Workload, src_coords: np.ndarray) -> np.ndarray:
    """(F, n_s) nodal values of the workload's field on its source mesh."""
    return np.ascontiguousarray(_fields.evaluate(w.field, np, src_coords), dtype=np.float64)


def scaled(w: Workload, target_k: int, source_k: int, samples_per_elem: int | None = None,
           name: str | None = None) -> Workload:
    """Same recipe at a different size (for tests that need a smaller instance)."""
    return Workload(
        name or f"{w.name}@{target_k}/{source_k}", w.dim,
        MeshSpec(w.target.kind, target_k, w.target.jitter, w.target.seed),
        MeshSpec(w.source.kind, source_k, w.source.jitter, w.source.seed),
        w.field, samples_per_elem or w.samples_per_elem, w.n_fields, w.alpha, w.index,
        (0, 0, 0), w.rtol)


@dataclass(frozen=True)
class BatchItem:
    dim: int
    target: MeshSpec
    source: MeshSpec
    kvec: tuple          # (4, dim) integer wave vectors
    amp: tuple           # (4,)
    phase: tuple         # (4,)
    samples_per_elem: int
    stream_id: int

    def field(self, xp, coords):
        """Nodal values (1, n) of this transfer's field at coords (n, dim)."""
        out = 1.0 + 0.0 * coords[:, 0]
        for q in range(len(self.amp)):
            arg = 2.0 * np.pi * sum(self.kvec[q][c] * coords[:, c] for c in range(self.dim)) + self.phase[q]
            out = out + 0.5 * self.amp[q] * xp.cos(arg)
        return out[None, :]


BATCH_PHILOX_SEED = PHILOX_SEED_BASE + 5


def batch_items(count: int = 256, seed: int = 14, e_min: float = 1e3, e_max: float = 5e5):
    """The uneven batch: see the module docstring."""
    rng = np.random.default_rng(seed)
    items = []
    for k in range(count):
        E = float(np.exp(rng.uniform(np.log(e_min), np.log(e_max))))
        dim = 2 if rng.random() < 0.5 else 3
        ratio = int(rng.integers(2, 5))
        N = int(rng.choice([32, 64, 128, 256]))
        kv = []
        while len(kv) < 4:
            v = tuple(int(c) for c in rng.integers(0, 3, size=dim))
            if any(v):
                kv.append(v)
        amp = tuple(float(a) for a in rng.standard_normal(4))
        phase = tuple(float(f) for f in rng.uniform(0.0, 2.0 * np.pi, 4))
        if dim == 2:
            kt = max(3, int(round(np.sqrt(E / 2.0))) + 1)
            ks = max(3, int(round(np.sqrt(ratio * E / 2.0))) + 1)
            tgt = MeshSpec("structured_tri", kt, 0.2, 1000 + k)
            src = MeshSpec("structured_tri", ks, 0.2, 2000 + k)
        else:
            kt = max(3, int(round((E / 6.0) ** (1.0 / 3.0))) + 1)
            ks = max(3, int(round((ratio * E / 6.0) ** (1.0 / 3.0))) + 1)
            tgt = MeshSpec("kuhn_tet", kt, 0.08, 1000 + k)
            src = MeshSpec("kuhn_tet", ks, 0.08, 2000 + k)
        items.append(BatchItem(dim, tgt, src, tuple(kv), amp, phase, N, k))
    return items
