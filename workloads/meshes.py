"""Seeded synthetic P1 meshes of the unit square / unit cube.

Input generators only: these build node coordinates and element connectivity
and hold none of the transfer method's arithmetic.  Both the CPU oracle and the
GPU path consume the same arrays.

Conventions
-----------
* ``coords`` is ``(n_nodes, dim)`` float64, ``conn`` is ``(n_elems, dim+1)``
  int32, every element positively oriented (counter-clockwise triangles,
  right-handed tetrahedra).
* "k-grid" means k nodes per axis, i.e. (k-1) cells per axis.
* Jitter moves every node by a uniform offset in ``[-a*h, a*h]`` per axis, but
  a coordinate that sits exactly on the domain boundary (0 or 1) is not moved,
  so boundary nodes slide tangentially, corners stay fixed, and the mesh covers
  exactly ``[0,1]^dim``.

The paper's meshes (gmsh square meshes from 1k to 2.3M triangles, the LTX and
WEST reactor meshes) are not available; these generators stand in for them
with the same element type, dimension and size range.
"""
from __future__ import annotations

import itertools

import numpy as np


def _grid_points(k: int, dim: int) -> np.ndarray:
    g = np.linspace(0.0, 1.0, k)
    axes = np.meshgrid(*([g] * dim), indexing="ij")
    # node id = i + j*k (+ l*k*k): the x index varies fastest
    return np.stack([a.transpose(tuple(reversed(range(dim)))).ravel() for a in axes], axis=1)


def jittered_grid_points(k: int, dim: int, jitter: float, seed: int) -> np.ndarray:
    """k^dim grid nodes on [0,1]^dim with tangential-only boundary jitter."""
    p = _grid_points(k, dim)
    h = 1.0 / (k - 1)
    rng = np.random.default_rng(seed)
    d = rng.uniform(-jitter * h, jitter * h, size=p.shape)
    d[(p == 0.0) | (p == 1.0)] = 0.0
    return np.ascontiguousarray(p + d)


def _orient(coords: np.ndarray, conn: np.ndarray) -> np.ndarray:
    """Swap the last two vertices of negatively oriented simplices."""
    x0 = coords[conn[:, 0]]
    e = [coords[conn[:, i]] - x0 for i in range(1, conn.shape[1])]
    if conn.shape[1] > 4:
        det = np.linalg.det(np.stack(e, axis=1))
    elif conn.shape[1] == 3:
        det = e[0][:, 0] * e[1][:, 1] - e[0][:, 1] * e[1][:, 0]
    else:
        det = (e[0][:, 0] * (e[1][:, 1] * e[2][:, 2] - e[1][:, 2] * e[2][:, 1])
               - e[0][:, 1] * (e[1][:, 0] * e[2][:, 2] - e[1][:, 2] * e[2][:, 0])
               + e[0][:, 2] * (e[1][:, 0] * e[2][:, 1] - e[1][:, 1] * e[2][:, 0]))
    flip = det < 0
    conn = conn.copy()
    conn[flip, -2], conn[flip, -1] = conn[flip, -1].copy(), conn[flip, -2].copy()
    return conn


def structured_tri_mesh(k: int, jitter: float, seed: int):
    """Jittered k x k node grid, every cell split along its (i,j)-(i+1,j+1) diagonal.

    2*(k-1)^2 triangles.  Any jitter below h/4 keeps every area positive.
    """
    coords = jittered_grid_points(k, 2, jitter, seed)
    i, j = np.meshgrid(np.arange(k - 1), np.arange(k - 1), indexing="xy")
    i = i.ravel(); j = j.ravel()
    a = i + j * k
    b = a + 1
    c = a + k + 1
    d = a + k
    conn = np.empty((2 * a.size, 3), dtype=np.int64)
    conn[0::2] = np.stack([a, b, c], 1)
    conn[1::2] = np.stack([a, c, d], 1)
    conn = _orient(coords, conn)
    return coords, conn.astype(np.int32)


def delaunay_tri_mesh(k: int, jitter: float, seed: int):
    """Delaunay triangulation of a jittered k x k point grid (2n - 2 - #hull triangles)."""
    from scipy.spatial import Delaunay

    coords = jittered_grid_points(k, 2, jitter, seed)
    tri = Delaunay(coords)
    if len(tri.coplanar):
        raise RuntimeError("Delaunay dropped points")
    conn = _orient(coords, tri.simplices.astype(np.int64))
    return coords, conn.astype(np.int32)


# the six monotone lattice paths from corner (0,0,0) to (1,1,1) of a cube
_KUHN_PATHS = list(itertools.permutations(range(3)))


def kuhn_tet_mesh(k: int, jitter: float, seed: int):
    """Perturbed Kuhn (Freudenthal) split of a (k-1)^3 hex grid: 6*(k-1)^3 tets.

    Jitter up to about 0.09h keeps every volume positive; the default 0.08h
    is used for the 3D workloads.
    """
    coords = jittered_grid_points(k, 3, jitter, seed)
    c = k - 1
    ii, jj, ll = np.meshgrid(np.arange(c), np.arange(c), np.arange(c), indexing="ij")
    base = (ii + jj * k + ll * k * k).transpose(2, 1, 0).ravel()
    stride = np.array([1, k, k * k])
    tets = []
    for perm in _KUHN_PATHS:
        v0 = base
        v1 = v0 + stride[perm[0]]
        v2 = v1 + stride[perm[1]]
        v3 = v0 + stride.sum()
        tets.append(np.stack([v0, v1, v2, v3], 1))
    conn = np.stack(tets, 1).reshape(-1, 4)
    conn = _orient(coords, conn)
    return coords, conn.astype(np.int32)


def kuhn_mesh(dim: int, k: int, jitter: float, seed: int):
    """Perturbed Kuhn (Freudenthal) split of a (k-1)^dim hypercube grid of
    [0,1]^dim into dim! (k-1)^dim simplices: one per monotone lattice path
    from a cell's lowest corner to its highest (the vertices after 0, 1, ...,
    dim unit steps along the axes in the path's order).  dim = 3 gives the
    same tetrahedra as kuhn_tet_mesh.  Jitter up to about 0.05h keeps every
    volume positive in 6D (the default here is 0.03h)."""
    coords = jittered_grid_points(k, dim, jitter, seed)
    c = k - 1
    idx = np.meshgrid(*([np.arange(c)] * dim), indexing="ij")
    stride = np.array([k ** a for a in range(dim)], dtype=np.int64)
    # cells with the x index fastest, as the node numbering
    base = sum(idx[a].transpose(tuple(reversed(range(dim)))).ravel() * stride[a] for a in range(dim))
    simp = []
    for perm in itertools.permutations(range(dim)):
        verts = [base]
        for a in perm:
            verts.append(verts[-1] + stride[a])
        simp.append(np.stack(verts, 1))
    conn = np.stack(simp, 1).reshape(-1, dim + 1)
    conn = _orient(coords, conn)
    return coords, conn.astype(np.int32)


def make_mesh(kind: str, k: int, jitter: float, seed: int):
    if kind == "structured_tri":
        return structured_tri_mesh(k, jitter, seed)
    if kind == "delaunay_tri":
        return delaunay_tri_mesh(k, jitter, seed)
    if kind == "kuhn_tet":
        return kuhn_tet_mesh(k, jitter, seed)
    if kind.startswith("kuhn") and kind.endswith("d") and kind[4:-1].isdigit():
        return kuhn_mesh(int(kind[4:-1]), k, jitter, seed)
    raise ValueError(f"unknown mesh kind {kind!r}")


# local edges of a P2 element, vertex pairs a < b in lexicographic order
P2_LOCAL_EDGES = {2: ((0, 1), (0, 2), (1, 2)), 3: ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3))}


def p2_mesh(coords: np.ndarray, conn: np.ndarray):
    """Straight-sided P2 mesh on a P1 mesh: the vertices keep their ids, the
    edge midpoints follow them, numbered in ascending (lower, higher vertex
    id) order; each element lists its d+1 vertices, then its edge nodes in
    the order of P2_LOCAL_EDGES.  Returns (coords2, conn2)."""
    coords = np.asarray(coords, dtype=np.float64)
    conn = np.asarray(conn, dtype=np.int64)
    dim = coords.shape[1]
    n = coords.shape[0]
    pairs = np.stack([np.sort(conn[:, [a, b]], axis=1) for a, b in P2_LOCAL_EDGES[dim]], axis=1)  # (E, ne, 2)
    keys = pairs[..., 0] * n + pairs[..., 1]
    uniq, inv = np.unique(keys.ravel(), return_inverse=True)
    lo, hi = uniq // n, uniq % n
    mid = 0.5 * (coords[lo] + coords[hi])
    coords2 = np.concatenate([coords, mid])
    conn2 = np.concatenate([conn, n + inv.reshape(keys.shape)], axis=1)
    return coords2, conn2.astype(np.int32)
