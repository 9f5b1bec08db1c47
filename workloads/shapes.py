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
* Any closed triangle mesh (mesh_problem): c(x) from the signed distance s
  to the mesh (negative inside),
    c = c0 - ((c0 - c_p)/2) (1 - tanh(s (s + 2 R_e) / d)),
  with R_e the radius of the sphere of equal volume; for a sphere
  s (s + 2 R) = |r - r0|^2 - R^2, so this is again eq. sound_speed_object.
  The distance is the smallest point-to-triangle distance; the sign comes
  from the generalised winding number (the sum of the triangles' solid
  angles by the formula of Van Oosterom and Strackee, over 4 pi: 1 inside,
  0 outside).  The integration surface is the mesh moved `offset` cells
  outward along its area-weighted vertex normals.  radial_mesh builds
  star-shaped test objects r = r(u) on the icosphere, e.g. the non-convex
  peanut r = R (1 + eps P4(u_x)).
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


# ---------------------------------------------------------------------------
# Any closed triangle mesh
# ---------------------------------------------------------------------------

def radial_mesh(radius_fn, level: int = 3):
    """The icosphere with every vertex u moved to radius_fn(u) u (a star-shaped closed mesh)."""
    U, F = icosphere(level)
    return U * np.asarray(radius_fn(U), dtype=np.float64)[:, None], F


def peanut(R: float, eps: float = 0.3, level: int = 3):
    """r(u) = R (1 + eps P4(u_x)): lobes along x and around the waist, pinched between them."""
    def r(U):
        t = U[:, 0]
        return R * (1.0 + eps * (35.0 * t ** 4 - 30.0 * t ** 2 + 3.0) / 8.0)
    return radial_mesh(r, level)


def mesh_volume(vertices, faces) -> float:
    """Enclosed volume of a closed, outward-oriented mesh (divergence theorem)."""
    P = np.asarray(vertices, dtype=np.float64)[np.asarray(faces)]
    return float(np.einsum("ij,ij->i", P[:, 0], np.cross(P[:, 1], P[:, 2])).sum() / 6.0)


def vertex_normals(vertices, faces):
    """Area-weighted unit normals at the vertices."""
    V = np.asarray(vertices, dtype=np.float64)
    F = np.asarray(faces)
    P = V[F]
    cr = np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0])
    n = np.zeros_like(V)
    for k in range(3):
        np.add.at(n, F[:, k], cr)
    return n / np.linalg.norm(n, axis=1)[:, None]


def _seg2(px, py, pz, ax, ay, az, ex, ey, ez, ee):
    # squared distance from points p to the segments a + t e, t in [0, 1] (ee = |e|^2)
    t = np.clip(((px - ax) * ex + (py - ay) * ey + (pz - az) * ez) / ee, 0.0, 1.0)
    dx, dy, dz = px - ax - t * ex, py - ay - t * ey, pz - az - t * ez
    return dx * dx + dy * dy + dz * dz


def _triangle_distance2(P, T):
    """Squared distances (points x triangles) from P (n, 3) to the triangles T (m, 3, 3)."""
    px, py, pz = (P[:, k][:, None] for k in range(3))
    ax, ay, az = (T[None, :, 0, k] for k in range(3))
    bx, by, bz = (T[None, :, 1, k] for k in range(3))
    cx, cy, cz = (T[None, :, 2, k] for k in range(3))
    abx, aby, abz = bx - ax, by - ay, bz - az
    bcx, bcy, bcz = cx - bx, cy - by, cz - bz
    cax, cay, caz = ax - cx, ay - cy, az - cz
    nx = aby * (cz - az) - abz * (cy - ay)             # n = (b - a) x (c - a)
    ny = abz * (cx - ax) - abx * (cz - az)
    nz = abx * (cy - ay) - aby * (cx - ax)
    qax, qay, qaz = px - ax, py - ay, pz - az
    qbx, qby, qbz = px - bx, py - by, pz - bz
    qcx, qcy, qcz = px - cx, py - cy, pz - cz
    # the foot of the perpendicular lies inside when (e x (p - v)) . n >= 0 for the three edges
    inside = (((aby * qaz - abz * qay) * nx + (abz * qax - abx * qaz) * ny
               + (abx * qay - aby * qax) * nz >= 0)
              & ((bcy * qbz - bcz * qby) * nx + (bcz * qbx - bcx * qbz) * ny
                 + (bcx * qby - bcy * qbx) * nz >= 0)
              & ((cay * qcz - caz * qcy) * nx + (caz * qcx - cax * qcz) * ny
                 + (cax * qcy - cay * qcx) * nz >= 0))
    hn = qax * nx + qay * ny + qaz * nz                  # (p - a) . n
    d_plane = hn * hn / (nx * nx + ny * ny + nz * nz)
    d_edge = np.minimum(np.minimum(
        _seg2(px, py, pz, ax, ay, az, abx, aby, abz, abx * abx + aby * aby + abz * abz),
        _seg2(px, py, pz, bx, by, bz, bcx, bcy, bcz, bcx * bcx + bcy * bcy + bcz * bcz)),
        _seg2(px, py, pz, cx, cy, cz, cax, cay, caz, cax * cax + cay * cay + caz * caz))
    return np.where(inside, d_plane, d_edge)


def _row_crossings(T, y, z):
    """x where the line (., y, z) crosses each triangle of T (m, 3, 3); NaN where it misses."""
    ay, az, by, bz, cy, cz = (T[:, 0, 1], T[:, 0, 2], T[:, 1, 1], T[:, 1, 2], T[:, 2, 1],
                              T[:, 2, 2])
    det = (by - ay) * (cz - az) - (bz - az) * (cy - ay)
    with np.errstate(divide="ignore", invalid="ignore"):
        u = ((y - ay) * (cz - az) - (z - az) * (cy - ay)) / det   # barycentric weight of b
        v = ((by - ay) * (z - az) - (bz - az) * (y - ay)) / det   # barycentric weight of c
        hit = (u >= 0) & (v >= 0) & (u + v <= 1) & (det != 0)
        x = T[:, 0, 0] + u * (T[:, 1, 0] - T[:, 0, 0]) + v * (T[:, 2, 0] - T[:, 0, 0])
    return np.where(hit, x, np.nan)


def mesh_signed_distance_grid(vertices, faces, lo, hi, cutoff: float):
    """Signed distance (negative inside) from every node of the box lo..hi (x, y, z inclusive)
    to a closed mesh, as an array (z, y, x); magnitudes beyond `cutoff` are clipped to it.

    The sign comes from the parity of the mesh crossings of each x row to the right of the
    node (the row is moved by 1e-7 cells in y and z so that it misses edges and vertices); the
    distance is the smallest point-to-triangle distance over the triangles that reach within
    `cutoff` of the node's z plane."""
    V = np.asarray(vertices, dtype=np.float64)
    T = V[np.asarray(faces)]
    xs = np.arange(lo[0], hi[0] + 1, dtype=np.float64)
    ys = np.arange(lo[1], hi[1] + 1, dtype=np.float64)
    zs = np.arange(lo[2], hi[2] + 1, dtype=np.float64)
    out = np.empty((len(zs), len(ys), len(xs)))
    tz_lo, tz_hi = T[:, :, 2].min(axis=1), T[:, :, 2].max(axis=1)
    yy, xx = np.meshgrid(ys, xs, indexing="ij")
    for iz, z in enumerate(zs):
        sel = (tz_lo <= z + cutoff) & (tz_hi >= z - cutoff)
        dist = np.full(yy.size, cutoff)
        if sel.any():
            P = np.stack([xx.ravel(), yy.ravel(), np.full(yy.size, z)], axis=1)
            Ts = T[sel]
            d2 = np.full(len(P), cutoff * cutoff)
            for p0 in range(0, len(P), 256):
                d2[p0:p0 + 256] = np.minimum(d2[p0:p0 + 256],
                                             _triangle_distance2(P[p0:p0 + 256], Ts).min(axis=1))
            dist = np.sqrt(d2)
        inside = np.zeros((len(ys), len(xs)), dtype=bool)
        for iy, y in enumerate(ys):
            xc = _row_crossings(T, y + 1.1e-7, z + 0.7e-7)
            xc = np.sort(xc[~np.isnan(xc)])
            inside[iy] = (len(xc) - np.searchsorted(xc, xs, side="right")) % 2 == 1
        out[iz] = np.where(inside.ravel(), -dist, dist).reshape(len(ys), len(xs))
    return out


def mesh_signed_distance(vertices, faces, points, chunk: int = 256):
    """Signed distance from arbitrary points to a closed, outward-oriented mesh (negative
    inside): the point-to-triangle distance, signed by the generalised winding number (the
    triangles' solid angles, formula of Van Oosterom and Strackee, summed over 4 pi)."""
    V = np.asarray(vertices, dtype=np.float64)
    T = V[np.asarray(faces)]
    X = np.asarray(points, dtype=np.float64).reshape(-1, 3)
    out = np.empty(len(X))
    for p0 in range(0, len(X), chunk):
        P = X[p0:p0 + chunk]
        dist = np.sqrt(_triangle_distance2(P, T).min(axis=1))
        a, b, c = (T[None, :, k, :] - P[:, None, :] for k in range(3))
        la, lb, lc = (np.linalg.norm(w, axis=2) for w in (a, b, c))
        num = np.einsum("ijk,ijk->ij", a, np.cross(b, c))
        den = (la * lb * lc + np.einsum("ijk,ijk->ij", a, b) * lc
               + np.einsum("ijk,ijk->ij", a, c) * lb + np.einsum("ijk,ijk->ij", b, c) * la)
        wind = (2.0 * np.arctan2(num, den)).sum(axis=1) / (4.0 * math.pi)
        out[p0:p0 + chunk] = np.where(wind > 0.5, -dist, dist)
    return out


def mesh_c_field(shape_zyx, vertices, faces, c0: float, cp: float, d: float = 4.0):
    """Per-cell sound speed (z, y, x order, flattened) of a density-matched object bounded by a
    closed mesh (vertices in lattice coordinates x, y, z)."""
    nz, ny, nx = shape_zyx
    V = np.asarray(vertices, dtype=np.float64)
    Re = (3.0 * mesh_volume(V, faces) / (4.0 * math.pi)) ** (1.0 / 3.0)
    # beyond s (s + 2 Re) = 20 d the profile equals c0 in FP64 (1 - tanh 20 < 1e-17)
    cut = -Re + math.sqrt(Re * Re + 20.0 * d)
    lo = np.maximum(np.floor(V.min(axis=0) - cut - 1), 0).astype(int)
    hi = np.minimum(np.ceil(V.max(axis=0) + cut + 1), [nx - 1, ny - 1, nz - 1]).astype(int)
    c = np.full((nz, ny, nx), float(c0))
    sd = mesh_signed_distance_grid(V, faces, lo, hi, cut + 1.0)
    box = c0 - ((c0 - cp) / 2.0) * (1.0 - np.tanh(sd * (sd + 2.0 * Re) / d))
    c[lo[2]:hi[2] + 1, lo[1]:hi[1] + 1, lo[0]:hi[0] + 1] = box
    return c.reshape(-1)


def mesh_problem(base: dict, vertices, faces, offset: float = 2.0, surface_level_faces=None):
    """A copy of a 3D sphere problem (same box, drive and centre) with the object bounded by a
    closed mesh given around the origin; the integration surface is the mesh moved `offset`
    cells outward (or `surface_level_faces` = (vertices, faces) of a finer copy of it)."""
    p = dict(base)
    cen = np.asarray(p["center"], dtype=np.float64)
    V = np.asarray(vertices, dtype=np.float64) + cen
    sv, sf = (vertices, faces) if surface_level_faces is None else surface_level_faces
    SV = np.asarray(sv, dtype=np.float64) + cen
    xyz, nrm, area = mesh_elements(SV + offset * vertex_normals(SV, sf), sf)
    p["surf_xyz"], p["surf_normal"], p["surf_area"] = xyz, nrm, area
    p["c_field"] = mesh_c_field((p["nz"], p["ny"], p["nx"]), V, faces, p["c0"], p["cp"], p["d"])
    p["volume"] = mesh_volume(vertices, faces)
    return p
