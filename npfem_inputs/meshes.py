"""Seeded, synthetic cell meshes: the geometry both the oracle and the library consume.

This module holds input data only (vertex positions and triangle lists). It contains
none of the solver's arithmetic: no rest frames, stencils, masses or system matrices.

Cell shapes follow the paper's Results section (normal biconcave red blood cells and
nearly rigid oblate-ellipsoid platelets) and its parameter table (258 surface vertices
for a red blood cell, 66 for a platelet). The paper does not give a shape formula, so the
red-cell profile is the published Evans-Fung (1972) biconcave curve; the platelet is an
oblate ellipsoid of 3.6 um diameter and 0.9 um thickness.

Mesh topology is a UV sphere: two poles plus ``rings`` latitude rings of ``segments``
vertices each. Vertex 0 is the +z pole, vertices 1 .. rings*segments are the rings from +z
to -z (ring k, segment j at index 1 + k*segments + j), and the last vertex is the -z pole.
Triangles are counter-clockwise seen from outside, so the enclosed signed volume is
positive.
"""
from __future__ import annotations

import numpy as np

# Evans-Fung biconcave profile constants (um); z = +-(R0/2) sqrt(1-s) (C0 + C2 s + C4 s^2),
# with s = (r/R0)^2.
EF_R0 = 3.91
EF_C0 = 0.207161
EF_C2 = 2.002558
EF_C4 = -1.122762

RBC_DIAMETER = 7.82      # um, nominal red-cell diameter (2 * EF_R0)
PLT_DIAMETER = 3.6       # um
PLT_THICKNESS = 0.9      # um


def uv_sphere_topology(rings: int, segments: int) -> np.ndarray:
    """Triangle list (int32 [m][3]) of a UV sphere with the vertex order described above.

    m = 2*segments (pole caps) + 2*segments*(rings-1) (bands).
    """
    if rings < 1 or segments < 3:
        raise ValueError("need rings >= 1 and segments >= 3")
    north = 0
    south = 1 + rings * segments

    def ring(k: int, j: int) -> int:
        return 1 + k * segments + (j % segments)

    tris = []
    for j in range(segments):
        tris.append((north, ring(0, j), ring(0, j + 1)))
    for k in range(rings - 1):
        for j in range(segments):
            a, b = ring(k, j), ring(k, j + 1)
            c, d = ring(k + 1, j), ring(k + 1, j + 1)
            tris.append((a, c, d))
            tris.append((a, d, b))
    for j in range(segments):
        tris.append((south, ring(rings - 1, j + 1), ring(rings - 1, j)))
    return np.asarray(tris, dtype=np.int32)


def _uv_angles(rings: int, segments: int):
    theta = np.pi * np.arange(1, rings + 1) / (rings + 1)          # polar angle of each ring
    phi = 2.0 * np.pi * np.arange(segments) / segments              # azimuth of each segment
    return theta, phi


def evans_fung_z(sin_theta: np.ndarray, cos_theta: np.ndarray) -> np.ndarray:
    """Height of the biconcave surface above the mid-plane at radius R0*sin(theta).

    With s = sin^2(theta), sqrt(1 - s) = |cos(theta)|, so the signed height is
    (R0/2) cos(theta) (C0 + C2 s + C4 s^2).
    """
    s = sin_theta ** 2
    return 0.5 * EF_R0 * cos_theta * (EF_C0 + EF_C2 * s + EF_C4 * s * s)


def rbc_mesh(rings: int = 16, segments: int = 16):
    """Biconcave red blood cell: (rest_xyz float64 [n][3], tri int32 [m][3]).

    Default 16 x 16 UV sphere: n = 258 vertices, m = 512 triangles.
    """
    theta, phi = _uv_angles(rings, segments)
    st, ct = np.sin(theta), np.cos(theta)
    pts = [(0.0, 0.0, float(evans_fung_z(np.array(0.0), np.array(1.0))))]
    for k in range(rings):
        r = EF_R0 * st[k]
        z = float(evans_fung_z(st[k], ct[k]))
        for j in range(segments):
            pts.append((r * np.cos(phi[j]), r * np.sin(phi[j]), z))
    pts.append((0.0, 0.0, float(evans_fung_z(np.array(0.0), np.array(-1.0)))))
    return np.asarray(pts, dtype=np.float64), uv_sphere_topology(rings, segments)


def platelet_mesh(rings: int = 8, segments: int = 8,
                  diameter: float = PLT_DIAMETER, thickness: float = PLT_THICKNESS):
    """Oblate-ellipsoid platelet: (rest_xyz float64 [n][3], tri int32 [m][3]).

    Default 8 x 8 UV sphere: n = 66 vertices, m = 128 triangles.
    """
    a, c = 0.5 * diameter, 0.5 * thickness
    theta, phi = _uv_angles(rings, segments)
    pts = [(0.0, 0.0, c)]
    for k in range(rings):
        for j in range(segments):
            pts.append((a * np.sin(theta[k]) * np.cos(phi[j]),
                        a * np.sin(theta[k]) * np.sin(phi[j]),
                        c * np.cos(theta[k])))
    pts.append((0.0, 0.0, -c))
    return np.asarray(pts, dtype=np.float64), uv_sphere_topology(rings, segments)


def tetrahedron():
    """Regular-ish tetrahedron (4 vertices), outward CCW triangles."""
    x = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])
    t = np.array([[0, 2, 1], [0, 1, 3], [0, 3, 2], [1, 2, 3]], dtype=np.int32)
    return x, t


def octahedron(scale: float = 1.0):
    x = scale * np.array([[0, 0, 1], [1, 0, 0], [0, 1, 0], [-1, 0, 0], [0, -1, 0], [0, 0, -1]],
                         dtype=np.float64)
    t = np.array([[0, 1, 2], [0, 2, 3], [0, 3, 4], [0, 4, 1],
                  [5, 2, 1], [5, 3, 2], [5, 4, 3], [5, 1, 4]], dtype=np.int32)
    return x, t


def icosahedron(scale: float = 1.0):
    p = (1.0 + 5.0 ** 0.5) / 2.0
    x = np.array([[-1, p, 0], [1, p, 0], [-1, -p, 0], [1, -p, 0],
                  [0, -1, p], [0, 1, p], [0, -1, -p], [0, 1, -p],
                  [p, 0, -1], [p, 0, 1], [-p, 0, -1], [-p, 0, 1]], dtype=np.float64)
    x *= scale / np.linalg.norm(x[0])
    t = np.array([[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
                  [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
                  [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
                  [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]], dtype=np.int32)
    return x, t


def bipyramid(k: int, height: float = 1.0):
    """Two apexes over a regular k-gon (k + 2 vertices): apexes of degree k, equator vertices
    of degree 4; outward CCW triangles."""
    ang = 2.0 * np.pi * np.arange(k) / k
    x = np.concatenate([[[0.0, 0.0, height]], np.stack([np.cos(ang), np.sin(ang), 0 * ang], 1),
                        [[0.0, 0.0, -height]]])
    t = []
    for i in range(k):
        a, b = 1 + i, 1 + (i + 1) % k
        t.append((0, a, b))
        t.append((k + 1, b, a))
    return x, np.asarray(t, dtype=np.int32)


def mesh_summary(x: np.ndarray, tri: np.ndarray) -> dict:
    """Plain geometric summary used to pin the generated geometry (not solver arithmetic)."""
    a, b, c = x[tri[:, 0]], x[tri[:, 1]], x[tri[:, 2]]
    vol = float(np.sum(np.einsum("ij,ij->i", a, np.cross(b, c))) / 6.0)
    area = float(np.sum(0.5 * np.linalg.norm(np.cross(b - a, c - a), axis=1)))
    edges = set()
    for t in tri:
        for k in range(3):
            i, j = int(t[k]), int(t[(k + 1) % 3])
            edges.add((min(i, j), max(i, j)))
    e = np.array(sorted(edges))
    lens = np.linalg.norm(x[e[:, 0]] - x[e[:, 1]], axis=1)
    return {
        "n_vertices": int(x.shape[0]), "n_triangles": int(tri.shape[0]), "n_edges": int(len(e)),
        "volume": vol, "area": area,
        "edge_mean": float(lens.mean()), "edge_min": float(lens.min()), "edge_max": float(lens.max()),
        "span_x": float(x[:, 0].max() - x[:, 0].min()),
        "span_z": float(x[:, 2].max() - x[:, 2].min()),
    }
