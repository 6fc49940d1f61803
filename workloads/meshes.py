"""Closed triangulated surfaces for the deforming-body workloads (synthetic geometry inputs).

Every function returns float64 vertex positions ``verts`` [nv, 3], int32 triangles ``tris``
[nt, 3] (vertex indices, counter-clockwise seen from outside) and, where the surface moves,
vertex velocities ``vels`` [nv, 3].  None of the lattice Boltzmann arithmetic lives here; both
the GPU library and the oracle receive the same arrays.

* ``box_mesh``        -- axis-aligned box, 12 triangles.
* ``octahedron_mesh`` -- |x-c|_1 = r, 8 triangles (integer vertices put rays through edges and
                         vertices: the tie cases of the inside test).
* ``icosphere_mesh``  -- sphere of radius r from a subdivided icosahedron (vertices on the sphere).
* ``swimmer_mesh``    -- the anguilliform swimmer of Sec. IV.C: elliptical cross sections with
                         the half axes w(s), h(s) of the paper along a centre line that undulates
                         laterally as y(s, t) = 0.125 beta(t) L (s/L + 0.03125)/1.03125
                         sin(2 pi (s/L - t/T)) with the ramp beta(t) of eq. fish_ramping;
                         vertex velocities by central differences in time.
"""
from __future__ import annotations

import math

import numpy as np


def box_mesh(lo, hi):
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    v = np.array([[lo[0] if i & 1 == 0 else hi[0], lo[1] if i & 2 == 0 else hi[1], lo[2] if i & 4 == 0 else hi[2]]
                  for i in range(8)])
    # faces as quads (listed clockwise seen from outside), split along one diagonal
    quads = [(0, 2, 6, 4), (1, 5, 7, 3),   # x = lo, x = hi
             (0, 4, 5, 1), (2, 3, 7, 6),   # y = lo, y = hi
             (0, 1, 3, 2), (4, 6, 7, 5)]   # z = lo, z = hi
    t = []
    for a, b, c, d in quads:
        t += [(a, c, b), (a, d, c)]
    return v, np.array(t, dtype=np.int32)


def octahedron_mesh(center, r):
    c = np.asarray(center, float)
    v = np.array([c + [r, 0, 0], c - [r, 0, 0], c + [0, r, 0], c - [0, r, 0], c + [0, 0, r], c - [0, 0, r]])
    t = []
    for sx, ix in ((1, 0), (-1, 1)):
        for sy, iy in ((1, 2), (-1, 3)):
            for sz, iz in ((1, 4), (-1, 5)):
                tri = (ix, iy, iz)
                if sx * sy * sz < 0:
                    tri = (ix, iz, iy)
                t.append(tri)
    return v, np.array(t, dtype=np.int32)


def icosphere_mesh(center, r, level: int):
    p = (1.0 + math.sqrt(5.0)) / 2.0
    v = [(-1, p, 0), (1, p, 0), (-1, -p, 0), (1, -p, 0), (0, -1, p), (0, 1, p), (0, -1, -p), (0, 1, -p),
         (p, 0, -1), (p, 0, 1), (-p, 0, -1), (-p, 0, 1)]
    v = [np.array(a, float) / np.linalg.norm(a) for a in v]
    f = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6),
         (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9), (4, 9, 5), (2, 4, 11), (6, 2, 10),
         (8, 6, 7), (9, 8, 1)]
    for _ in range(level):
        mid = {}

        def m(a, b):
            key = (min(a, b), max(a, b))
            if key not in mid:
                w = v[a] + v[b]
                v.append(w / np.linalg.norm(w))
                mid[key] = len(v) - 1
            return mid[key]
        nf = []
        for a, b, c in f:
            ab, bc, ca = m(a, b), m(b, c), m(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        f = nf
    verts = np.asarray(center, float) + r * np.array(v)
    return verts, np.array(f, dtype=np.int32)


# ----------------------------------------------------------------------------- swimmer (Sec. IV.C)
def swimmer_halfwidth(s, L):
    """w(s): half width of the cross section at arc length s (w_h = s_b = 0.04 L, s_t = 0.95 L,
    w_t = 0.01 L)."""
    s = np.asarray(s, float)
    wh = sb = 0.04 * L
    st, wt = 0.95 * L, 0.01 * L
    head = np.sqrt(np.clip(2.0 * wh * s - s * s, 0.0, None))
    body = wh - (wh - wt) * ((s - sb) / (st - sb)) ** 2
    tail = wt * (L - s) / (L - st)
    return np.where(s < sb, head, np.where(s < st, body, tail))


def swimmer_halfheight(s, L):
    """h(s) = b sqrt(1 - ((s - a)/a)^2), a = 0.51 L, b = 0.08 L."""
    s = np.asarray(s, float)
    a, b = 0.51 * L, 0.08 * L
    return b * np.sqrt(np.clip(1.0 - ((s - a) / a) ** 2, 0.0, None))


def swimmer_ramp(t, T):
    """beta(t) of eq. fish_ramping: (1 - cos(pi t/T))/2 for t <= T, then 1."""
    return 0.5 * (1.0 - math.cos(math.pi * t / T)) if t <= T else 1.0


def swimmer_lateral(s, t, L, T):
    return 0.125 * swimmer_ramp(t, T) * L * (s / L + 0.03125) / 1.03125 * np.sin(2.0 * math.pi * (s / L - t / T))


def _swimmer_points(head, L, T, t, n_seg, n_theta):
    s = np.arange(1, n_seg) * (L / n_seg)
    w = swimmer_halfwidth(s, L)
    h = swimmer_halfheight(s, L)
    y = swimmer_lateral(s, t, L, T)
    th = 2.0 * math.pi * np.arange(n_theta) / n_theta
    ring = np.empty((n_seg - 1, n_theta, 3))
    ring[:, :, 0] = head[0] + s[:, None]
    ring[:, :, 1] = head[1] + y[:, None] + w[:, None] * np.cos(th)[None, :]
    ring[:, :, 2] = head[2] + h[:, None] * np.sin(th)[None, :]
    nose = np.array([head[0], head[1] + swimmer_lateral(0.0, t, L, T), head[2]])
    tail = np.array([head[0] + L, head[1] + swimmer_lateral(L, t, L, T), head[2]])
    return np.vstack([nose[None, :], ring.reshape(-1, 3), tail[None, :]])


def swimmer_mesh(head, L: float, T: float, t: float, n_seg: int = 150, n_theta: int = 16, dt: float = 1e-3):
    """Swimmer surface at time t: head (nose) at ``head`` (its centre line along +x, undulating in
    y), n_seg segments along the centre line (150 in the paper), n_theta points per cross section,
    closed by the nose and the tail point.  Returns (verts, tris, vels)."""
    head = np.asarray(head, float)
    X = _swimmer_points(head, L, T, t, n_seg, n_theta)
    V = (_swimmer_points(head, L, T, t + dt, n_seg, n_theta) - _swimmer_points(head, L, T, t - dt, n_seg, n_theta)) \
        / (2.0 * dt)
    K = n_theta
    nr = n_seg - 1
    last = 1 + nr * K

    def vid(j, k):
        return 1 + j * K + (k % K)
    tris = []
    for k in range(K):
        tris.append((0, vid(0, k + 1), vid(0, k)))
    for j in range(nr - 1):
        for k in range(K):
            a, b, c, d = vid(j, k), vid(j, k + 1), vid(j + 1, k + 1), vid(j + 1, k)
            tris += [(a, b, c), (a, c, d)]
    for k in range(K):
        tris.append((last, vid(nr - 1, k), vid(nr - 1, k + 1)))
    return X, np.array(tris, dtype=np.int32), V


def mesh_volume(verts, tris):
    """Enclosed volume by the divergence theorem (positive for outward orientation)."""
    a, b, c = verts[tris[:, 0]], verts[tris[:, 1]], verts[tris[:, 2]]
    return float(np.einsum("ij,ij->i", a, np.cross(b, c)).sum() / 6.0)


def edge_use_counts(tris):
    """Number of triangles using each undirected edge (2 everywhere for a closed surface), and
    whether every directed edge appears once (consistent orientation)."""
    und = {}
    directed = set()
    ok = True
    for t in tris:
        for a, b in ((t[0], t[1]), (t[1], t[2]), (t[2], t[0])):
            key = (min(a, b), max(a, b))
            und[key] = und.get(key, 0) + 1
            if (a, b) in directed:
                ok = False
            directed.add((a, b))
    return und, ok
