"""Seeded surface meshes for the scattering workloads.

Every mesh is returned as ``(verts, tris)``: ``verts`` float64 (nv, 3) and
``tris`` int32 (F, 3), triangles counter-clockwise seen from outside so that
the right-hand normal points into the exterior medium (the orientation the
PMCHWT formulation assumes for n_m, Section 2).

Workloads (Sections 4 and 5 of the paper describe the physical set-ups these
stand in for; the meshes are synthetic):
  * icosphere(level)      -- dielectric sphere of radius 1 (Mie-checkable)
  * hex_prism(s, a)       -- hexagonal ice column, diameter 1, length 2.5
  * aggregate(...)        -- several rotated prisms, disjoint (Section 5 stand-in)
  * three_cubes(k_e)      -- the three-cube array of Section 4
"""

import numpy as np


def _orient_outward(verts, tris, center=None):
    """Flip triangles whose right-hand normal points towards ``center``.

    Only valid for star-shaped bodies about ``center`` (all meshes here are
    convex per component).
    """
    if center is None:
        center = verts.mean(axis=0)
    a, b, c = verts[tris[:, 0]], verts[tris[:, 1]], verts[tris[:, 2]]
    n = np.cross(b - a, c - a)
    g = (a + b + c) / 3.0 - center
    flip = np.einsum("ij,ij->i", n, g) < 0
    out = tris.copy()
    out[flip] = out[flip][:, [0, 2, 1]]
    return out


def icosphere(level, radius=1.0):
    """Icosahedron refined ``level`` times by edge midpoints projected to the sphere.

    level 2: F = 320, E = 480; level 4: F = 5120, E = 7680.
    """
    p = (1.0 + 5.0 ** 0.5) / 2.0
    v = np.array([[-1, p, 0], [1, p, 0], [-1, -p, 0], [1, -p, 0],
                  [0, -1, p], [0, 1, p], [0, -1, -p], [0, 1, -p],
                  [p, 0, -1], [p, 0, 1], [-p, 0, -1], [-p, 0, 1]], dtype=np.float64)
    v /= np.linalg.norm(v, axis=1)[:, None]
    f = [[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
         [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
         [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
         [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]]
    verts = [tuple(x) for x in v]
    tris = [tuple(t) for t in f]
    for _ in range(level):
        cache = {}

        def mid(i, j):
            key = (min(i, j), max(i, j))
            if key not in cache:
                m = np.add(verts[i], verts[j]) / 2.0
                m /= np.linalg.norm(m)
                cache[key] = len(verts)
                verts.append(tuple(m))
            return cache[key]

        new = []
        for (a, b, c) in tris:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            new += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        tris = new
    verts = np.array(verts, dtype=np.float64) * radius
    tris = np.array(tris, dtype=np.int32)
    return verts, _orient_outward(verts, tris, np.zeros(3))


class _VertexPool:
    """Merges coincident vertices (structured meshes built face by face)."""

    def __init__(self, tol=1e-9):
        self.tol = tol
        self.index = {}
        self.pts = []

    def add(self, x):
        key = tuple(np.round(np.asarray(x) / self.tol).astype(np.int64))
        if key not in self.index:
            self.index[key] = len(self.pts)
            self.pts.append(np.asarray(x, dtype=np.float64))
        return self.index[key]


def hex_prism(s, a, diameter=1.0, length=2.5):
    """Hexagonal column along z, circumscribed ``diameter``, ``length`` long.

    ``s`` divisions per hexagon side, ``a`` axial divisions:
    F = 12*s*a + 12*s*s (side quads split in two, caps of 6*s*s triangles each).
    """
    R = diameter / 2.0
    corners = [np.array([R * np.cos(np.pi / 3 * j), R * np.sin(np.pi / 3 * j)]) for j in range(6)]
    ring = []
    for j in range(6):
        c0, c1 = corners[j], corners[(j + 1) % 6]
        for i in range(s):
            ring.append(c0 + (c1 - c0) * (i / s))
    nr = len(ring)
    pool = _VertexPool()
    zs = np.linspace(-length / 2.0, length / 2.0, a + 1)
    ids = [[pool.add([ring[i][0], ring[i][1], z]) for i in range(nr)] for z in zs]
    tris = []
    for l in range(a):
        for i in range(nr):
            i2 = (i + 1) % nr
            p00, p01 = ids[l][i], ids[l][i2]
            p10, p11 = ids[l + 1][i], ids[l + 1][i2]
            tris += [(p00, p01, p11), (p00, p11, p10)]
    for z in (zs[0], zs[-1]):
        center = np.array([0.0, 0.0])
        for j in range(6):
            c0, c1 = corners[j], corners[(j + 1) % 6]

            def lat(u, v):
                xy = center + (c0 - center) * (u / s) + (c1 - center) * (v / s)
                return pool.add([xy[0], xy[1], z])

            for u in range(s):
                for v in range(s - u):
                    tris.append((lat(u, v), lat(u + 1, v), lat(u, v + 1)))
                    if u + v + 2 <= s:
                        tris.append((lat(u + 1, v), lat(u + 1, v + 1), lat(u, v + 1)))
    verts = np.array(pool.pts)
    tris = np.array(tris, dtype=np.int32)
    return verts, _orient_outward(verts, tris, np.zeros(3))


def cube(n, side=0.4, corner=(0.0, 0.0, 0.0)):
    """Axis-aligned cube with ``n`` x ``n`` quads (2 triangles each) per face."""
    pool = _VertexPool()
    corner = np.asarray(corner, dtype=np.float64)
    tris = []
    for axis in range(3):
        for side_sel in (0.0, 1.0):
            u_ax, v_ax = [x for x in range(3) if x != axis]
            grid = np.zeros((n + 1, n + 1), dtype=np.int64)
            for i in range(n + 1):
                for j in range(n + 1):
                    p = np.zeros(3)
                    p[axis] = side_sel * side
                    p[u_ax] = side * i / n
                    p[v_ax] = side * j / n
                    grid[i, j] = pool.add(corner + p)
            for i in range(n):
                for j in range(n):
                    tris += [(grid[i, j], grid[i + 1, j], grid[i + 1, j + 1]),
                             (grid[i, j], grid[i + 1, j + 1], grid[i, j + 1])]
    verts = np.array(pool.pts)
    tris = np.array(tris, dtype=np.int32)
    return verts, _orient_outward(verts, tris, corner + side / 2.0)


def three_cubes(k_ext, side=0.4):
    """The three-cube array of Section 4: corners at x = -1, 0, 1, mesh size 2*pi/(10*k_e)."""
    h = 2.0 * np.pi / (10.0 * k_ext)
    n = max(1, int(np.ceil(side / h)))
    return [cube(n, side, (x0, 0.0, 0.0)) for x0 in (-1.0, 0.0, 1.0)]


def _random_rotation(rng):
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def _inside_prism(p, diameter, length):
    """Points p (local prism frame) strictly inside the hexagonal column."""
    R = diameter / 2.0
    apothem = R * np.cos(np.pi / 6)
    inside = np.abs(p[:, 2]) < length / 2.0
    for j in range(6):
        ang = np.pi / 3 * j + np.pi / 6
        nrm = np.array([np.cos(ang), np.sin(ang)])
        inside &= p[:, :2] @ nrm < apothem
    return inside


def aggregate(n_monomers=8, s=7, a=30, seed=4, diameter=1.0, length=2.5, gap=0.1):
    """Disjoint hexagonal prisms with seeded uniform random orientations.

    Each monomer is rotated uniformly on SO(3) and pushed out from the origin
    along a seeded random direction until it neither overlaps any placed
    monomer nor comes within ``gap`` of its vertices.  Returns a list of
    ``(verts, tris)``, one per monomer.
    """
    rng = np.random.default_rng(seed)
    base_v, base_t = hex_prism(s, a, diameter, length)
    placed = []  # (R, c, verts)
    out = []
    for m in range(n_monomers):
        R = _random_rotation(rng)
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        t = 0.0
        while True:
            c = t * u
            v = base_v @ R.T + c
            ok = True
            for (R2, c2, v2) in placed:
                if np.min(np.linalg.norm(v[:, None, :] - v2[None, ::3, :], axis=2)) < gap:
                    ok = False
                    break
                if _inside_prism((v - c2) @ R2, diameter, length).any() or \
                        _inside_prism((v2 - c) @ R, diameter, length).any():
                    ok = False
                    break
            if ok:
                break
            t += 0.05
        placed.append((R, c, v))
        out.append((v, base_t.copy()))
    return out


def union_mesh(meshes):
    """Concatenate disjoint meshes; returns verts, tris and per-mesh triangle offsets."""
    verts, tris, offs = [], [], [0]
    nv = 0
    for (v, t) in meshes:
        verts.append(v)
        tris.append(t + nv)
        nv += len(v)
        offs.append(offs[-1] + len(t))
    return np.concatenate(verts), np.concatenate(tris).astype(np.int32), np.array(offs)


def mean_edge_length(verts, tris):
    e = np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]]])
    e = np.unique(np.sort(e, axis=1), axis=0)
    return float(np.mean(np.linalg.norm(verts[e[:, 0]] - verts[e[:, 1]], axis=1)))
