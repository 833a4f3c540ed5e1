"""Seeded synthetic triangle meshes (test and benchmark inputs only).

Every mesh has fixed connectivity, as the paper's dynamic meshes do (Sec. II:
a sequence of static meshes that share one vertex/face structure).  Nothing here
computes any part of the compression method; the Laplacian, covariance and the
rest are built separately by the oracle and by the HIP library.

Returned arrays:
  verts  float64 [n][3]
  tris   int32   [n_tris][3]  (vertex indices, counter-clockwise seen from outside)
"""
from __future__ import annotations

import numpy as np


def icosphere(level: int):
    """Icosahedron subdivided `level` times by edge midpoints, on the unit sphere.

    n = 10*4**level + 2 vertices, 20*4**level triangles.
    """
    if level < 0:
        raise ValueError("level must be >= 0")
    g = (1.0 + 5.0 ** 0.5) / 2.0
    v = [(-1, g, 0), (1, g, 0), (-1, -g, 0), (1, -g, 0),
         (0, -1, g), (0, 1, g), (0, -1, -g), (0, 1, -g),
         (g, 0, -1), (g, 0, 1), (-g, 0, -1), (-g, 0, 1)]
    f = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
         (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
         (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
         (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    verts = [np.array(p, dtype=np.float64) / np.linalg.norm(p) for p in v]
    faces = list(f)
    for _ in range(level):
        cache: dict[tuple[int, int], int] = {}

        def mid(a: int, b: int) -> int:
            key = (a, b) if a < b else (b, a)
            idx = cache.get(key)
            if idx is None:
                p = verts[a] + verts[b]
                verts.append(p / np.linalg.norm(p))
                idx = len(verts) - 1
                cache[key] = idx
            return idx

        nf = []
        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
    return np.asarray(verts, dtype=np.float64), np.asarray(faces, dtype=np.int32)


def _quad_grid_tris(a: int, b: int, wrap_i: bool, wrap_j: bool) -> np.ndarray:
    """Triangles of an a x b vertex lattice, vertex (i, j) -> i*b + j.

    Every quad is split along the same diagonal, so on a fully periodic lattice
    every vertex has exactly six neighbours.
    """
    ii = np.arange(a if wrap_i else a - 1)
    jj = np.arange(b if wrap_j else b - 1)
    I, J = np.meshgrid(ii, jj, indexing="ij")
    I1 = (I + 1) % a
    J1 = (J + 1) % b
    v00 = I * b + J
    v10 = I1 * b + J
    v11 = I1 * b + J1
    v01 = I * b + J1
    t1 = np.stack([v00, v10, v11], axis=-1).reshape(-1, 3)
    t2 = np.stack([v00, v11, v01], axis=-1).reshape(-1, 3)
    return np.concatenate([t1, t2], axis=0).astype(np.int32)


def torus(a: int, b: int, major: float = 1.0, minor: float = 0.3):
    """Closed a x b torus lattice (major radius 1, tube radius 0.3 by default)."""
    if a < 3 or b < 3:
        raise ValueError("torus needs a, b >= 3")
    u = 2.0 * np.pi * np.arange(a) / a
    w = 2.0 * np.pi * np.arange(b) / b
    U, W = np.meshgrid(u, w, indexing="ij")
    rr = major + minor * np.cos(W)
    verts = np.stack([rr * np.cos(U), rr * np.sin(U), minor * np.sin(W)], axis=-1)
    return verts.reshape(-1, 3).astype(np.float64), _quad_grid_tris(a, b, True, True)


def grid(a: int, b: int):
    """Planar a x b grid on the unit square (has a boundary; corner/edge vertices
    have degree 2..4)."""
    if a < 2 or b < 2:
        raise ValueError("grid needs a, b >= 2")
    x = np.linspace(0.0, 1.0, a)
    y = np.linspace(0.0, 1.0, b)
    X, Y = np.meshgrid(x, y, indexing="ij")
    verts = np.stack([X, Y, np.zeros_like(X)], axis=-1).reshape(-1, 3)
    return verts.astype(np.float64), _quad_grid_tris(a, b, False, False)


def disjoint_union(*meshes):
    """Several meshes as one vertex/face set with no edges between the parts
    (used to build an input with more than one connected component)."""
    vs, ts, off = [], [], 0
    for v, t in meshes:
        vs.append(v)
        ts.append(t + off)
        off += v.shape[0]
    return np.concatenate(vs, axis=0), np.concatenate(ts, axis=0).astype(np.int32)
