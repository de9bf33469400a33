"""Seeded synthetic triangle meshes shaped like the paper's benchmark plates.

The paper meshes its plates with Gmsh (Sec. 2.3, Sec. 3); those meshes are not
available, so structured grids of squares split into two linear triangles,
with seeded node jitter, optional per-cell random diagonals and circular holes,
stand in for them.  This module only builds geometry and index arrays: it holds
none of the fracture method's arithmetic, so both the CPU oracle and the GPU
path may take their inputs from it.

Random numbers come from NumPy's PCG64 via ``default_rng([seed, stream, ...])``
with fixed stream numbers: 0 jitter, 1 diagonals, 2 holes, 3 fracture-energy
draws, 4 mesh sizes.
"""
from __future__ import annotations

import numpy as np

STREAM_JITTER = 0
STREAM_DIAG = 1
STREAM_HOLES = 2
STREAM_GC = 3
STREAM_SIZES = 4


def rng(seed: int, stream: int, *sub: int) -> np.random.Generator:
    return np.random.default_rng([int(seed), int(stream), *[int(s) for s in sub]])


def grid_nodes(nx: int, ny: int, h: float) -> tuple[np.ndarray, np.ndarray]:
    """Unjittered node positions and their (i, j) grid indices.

    Node (i, j) has index j*(nx+1) + i and sits at (i*h, j*h).
    """
    j, i = np.meshgrid(np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
    ij = np.stack([i.ravel(), j.ravel()], axis=1).astype(np.int32)
    xy = ij.astype(np.float64) * h
    return xy, ij


def jitter_nodes(xy: np.ndarray, ij: np.ndarray, nx: int, ny: int, h: float,
                 amp: float, gen: np.random.Generator) -> np.ndarray:
    """Move every coordinate by an independent U[-amp*h, +amp*h] draw.

    Nodes on a vertical edge keep their x, nodes on a horizontal edge keep
    their y (so boundary nodes slide along the boundary); the four corners
    therefore stay put.
    """
    delta = gen.uniform(-amp * h, amp * h, size=xy.shape)
    on_v = (ij[:, 0] == 0) | (ij[:, 0] == nx)
    on_h = (ij[:, 1] == 0) | (ij[:, 1] == ny)
    delta[on_v, 0] = 0.0
    delta[on_h, 1] = 0.0
    return xy + delta


def grid_triangles(nx: int, ny: int, flip: np.ndarray | None = None) -> np.ndarray:
    """Two counter-clockwise triangles per grid cell.

    By default every cell is cut along (i,j)-(i+1,j+1); where ``flip`` (shape
    (ny, nx), bool) is set the cell is cut along (i+1,j)-(i,j+1) instead.
    Cells are visited row by row; each cell contributes its lower triangle
    first.
    """
    jj, ii = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    n00 = (jj * (nx + 1) + ii).ravel()
    n10 = n00 + 1
    n01 = n00 + nx + 1
    n11 = n01 + 1
    t_main = np.stack([np.stack([n00, n10, n11], 1), np.stack([n00, n11, n01], 1)], 1)
    t_anti = np.stack([np.stack([n00, n10, n01], 1), np.stack([n10, n11, n01], 1)], 1)
    if flip is None:
        tri = t_main
    else:
        f = flip.ravel()[:, None, None]
        tri = np.where(f, t_anti, t_main)
    return tri.reshape(-1, 3).astype(np.int32)


def _seg_dist(p: np.ndarray, a: np.ndarray, b: np.ndarray) -> float:
    ab = b - a
    t = np.clip(np.dot(p - a, ab) / np.dot(ab, ab), 0.0, 1.0)
    return float(np.linalg.norm(p - (a + t * ab)))


def hole_centres(n_holes: int, radius: float, width: float, height: float, h: float,
                 notch_a: np.ndarray, notch_b: np.ndarray,
                 gen: np.random.Generator, max_tries: int = 100000) -> np.ndarray:
    """Rejection-sample hole centres in [10h, W-10h] x [10h, H-10h].

    Accepted holes keep a gap of at least 4h between circles and an edge at
    least 12h away from the notch segment [notch_a, notch_b].
    """
    centres: list[np.ndarray] = []
    tries = 0
    while len(centres) < n_holes:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("hole placement failed")
        c = np.array([gen.uniform(10 * h, width - 10 * h), gen.uniform(10 * h, height - 10 * h)])
        if _seg_dist(c, notch_a, notch_b) < radius + 12 * h:
            continue
        if any(np.linalg.norm(c - o) < 2 * radius + 4 * h for o in centres):
            continue
        centres.append(c)
    return np.array(centres).reshape(-1, 2)


def plate_mesh(nx: int, ny: int, h: float, jitter: float, seed: int, *,
               random_diag: bool = False, n_holes: int = 0, hole_radius_cells: float = 8.0,
               sub: tuple[int, ...] = ()) -> dict:
    """Jittered structured plate, optionally perforated.

    Returns a dict with ``xy`` (N,2) float64, ``tri`` (Ne,3) int32 (CCW on the
    unjittered grid), ``ij`` (N,2) int32 grid indices of each kept node, and the
    sizes used.  Holes remove every triangle whose (jittered) centroid lies
    inside a circle; nodes left without a triangle are dropped and the rest
    renumbered in their original order.
    """
    xy0, ij = grid_nodes(nx, ny, h)
    xy = jitter_nodes(xy0, ij, nx, ny, h, jitter, rng(seed, STREAM_JITTER, *sub)) if jitter > 0 else xy0
    flip = None
    if random_diag:
        flip = rng(seed, STREAM_DIAG, *sub).random((ny, nx)) < 0.5
    tri = grid_triangles(nx, ny, flip)
    centres = np.zeros((0, 2))
    radius = hole_radius_cells * h
    if n_holes > 0:
        notch_a = np.array([0.0, (ny // 2) * h])
        notch_b = np.array([(nx // 2) * h, (ny // 2) * h])
        centres = hole_centres(n_holes, radius, nx * h, ny * h, h, notch_a, notch_b,
                               rng(seed, STREAM_HOLES, *sub))
        cen = xy[tri].mean(axis=1)
        keep = np.ones(len(tri), dtype=bool)
        for c in centres:
            keep &= np.hypot(cen[:, 0] - c[0], cen[:, 1] - c[1]) >= radius
        tri = tri[keep]
        used = np.zeros(len(xy), dtype=bool)
        used[tri.ravel()] = True
        new_id = np.cumsum(used) - 1
        tri = new_id[tri].astype(np.int32)
        xy = xy[used]
        ij = ij[used]
    return {"xy": np.ascontiguousarray(xy), "tri": np.ascontiguousarray(tri, dtype=np.int32),
            "ij": np.ascontiguousarray(ij), "nx": nx, "ny": ny, "h": h,
            "hole_centres": centres, "hole_radius": radius}
