"""Objects of other shapes: triangle-mesh integration surfaces and sound-speed fields.

The paper divides the object's boundary into surface elements, segments in
2D and triangles in 3D, each with its centre, normal and area (Sec. "Wave-
particle interaction and interpolation"), and says the approach applies to
objects of any shape (Conclusions).  This module lays out such inputs for
the C descriptor (surf_xyz = element centres, surf_normal, surf_area, and a
per-cell c_field); like the rest of this package it holds none of the
method's arithmetic.

* icosphere(level): the icosahedron with every triangle split in four,
  `level` times, vertices pushed onto the unit sphere (20 * 4**level faces).
* ellipsoid_surface: the integration surface around an ellipsoid with
  semi-axes (a, b, c): the icosphere mapped onto the ellipsoid, every vertex
  moved `offset` cells outward along the ellipsoid's normal (by default two
  cells, in the fluid, as for the sphere), one element per triangle.
* ellipsoid_c_field: the density-matched object's sound speed generalising
  eq. sound_speed_object with the ellipsoid's level function:
    c = c0 - ((c0 - c_p)/2) (1 - tanh((q - 1) R_e^2 / d)),
    q = sum_i (x_i - x0_i)^2 / a_i^2,  R_e = (a b c)^(1/3),
  which for a = b = c = R is exactly (|r - r0|^2 - R^2)/d.
"""
from __future__ import annotations

import math

import numpy as np


def icosphere(level: int):
    """Unit-sphere triangle mesh: (vertices (V, 3), faces (F, 3), counter-clockwise outside)."""
    t = (1.0 + math.sqrt(5.0)) / 2.0
    V = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t), (0, -1, -t),
         (0, 1, -t), (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    F = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4),
         (11, 10, 2), (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8),
         (3, 8, 9), (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    verts = [np.array(v, dtype=np.float64) / np.linalg.norm(v) for v in V]
    faces = list(F)
    for _ in range(level):
        mid = {}

        def middle(i, j):
            key = (min(i, j), max(i, j))
            if key not in mid:
                m = verts[i] + verts[j]
                verts.append(m / np.linalg.norm(m))
                mid[key] = len(verts) - 1
            return mid[key]

        nf = []
        for a, b, c in faces:
            ab, bc, ca = middle(a, b), middle(b, c), middle(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
    return np.array(verts), np.array(faces, dtype=np.int64)


def mesh_elements(vertices, faces):
    """One surface element per triangle: centroid, unit normal (right-hand order), area."""
    P = np.asarray(vertices, dtype=np.float64)[np.asarray(faces)]
    cen = P.mean(axis=1)
    cr = np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0])
    area = 0.5 * np.linalg.norm(cr, axis=1)
    nrm = cr / (2.0 * area[:, None])
    return cen, nrm, area


def ellipsoid_surface(center, axes, level: int = 4, offset: float = 2.0):
    """Integration surface `offset` cells outside the ellipsoid (element centres, normals, areas)."""
    U, F = icosphere(level)
    ax = np.asarray(axes, dtype=np.float64)
    P = U * ax                      # on the ellipsoid
    n = P / ax ** 2                 # outward normal direction of the level set
    n /= np.linalg.norm(n, axis=1)[:, None]
    return mesh_elements(np.asarray(center, dtype=np.float64) + P + offset * n, F)


def ellipsoid_c_field(shape_zyx, center, axes, c0: float, cp: float, d: float = 4.0):
    """Per-cell sound speed (z, y, x order, flattened) of a density-matched ellipsoid."""
    nz, ny, nx = shape_zyx
    ax = np.asarray(axes, dtype=np.float64)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    q = (((x - center[0]) / ax[0]) ** 2 + ((y - center[1]) / ax[1]) ** 2
         + ((z - center[2]) / ax[2]) ** 2)
    Re2 = float(np.prod(ax)) ** (2.0 / 3.0)
    c = c0 - ((c0 - cp) / 2.0) * (1.0 - np.tanh((q - 1.0) * Re2 / d))
    return c.reshape(-1)


def ellipsoid_problem(base: dict, axes, level: int = 4, offset: float = 2.0):
    """A copy of a 3D sphere problem (same box, drive and centre) with an ellipsoid instead."""
    p = dict(base)
    xyz, nrm, area = ellipsoid_surface(p["center"], axes, level, offset)
    p["surf_xyz"], p["surf_normal"], p["surf_area"] = xyz, nrm, area
    p["c_field"] = ellipsoid_c_field((p["nz"], p["ny"], p["nx"]), p["center"], axes, p["c0"],
                                     p["cp"], p["d"])
    p["axes"] = tuple(float(a) for a in axes)
    return p
