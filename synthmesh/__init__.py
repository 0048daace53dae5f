"""Seeded synthetic inputs shared by the CPU oracle and the HIP library.

This module produces *inputs only*: node coordinates, simplex connectivity,
boundary faces with their tags, and the refinement parent maps that define
the nested multigrid levels.  It contains none of the solver's arithmetic
(no geometry, no fluxes, no reconstruction); both solver implementations
derive everything else from these arrays independently.

The paper's own meshes (3-D hybrid meshes around cylinders, spheres and
airfoils, Section 6) are not available; these annulus (2-D cylinder) and
spherical-shell (3-D sphere) meshes stand in for them.

Boundary tags (same integer values on both solver sides, as part of the
input format):
    FARFIELD = 1, SLIP = 2, ISOTHERMAL = 3, ADIABATIC = 4
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

FARFIELD = 1
SLIP = 2
ISOTHERMAL = 3
ADIABATIC = 4


@dataclass
class Mesh:
    """A simplex mesh with boundary faces and refinement parent maps.

    coords      float64 [n_nodes, dim]
    cells       int32   [n_cells, dim+1], positively oriented
    bfaces      int32   [n_bfaces, dim]   node ids of boundary faces
    btags       int32   [n_bfaces]
    parents     list of int32 arrays; parents[l][i] is the index, on level
                l+1, of the agglomerate that contains cell i of level l.
                Level 0 is the fine mesh.
    """

    dim: int
    coords: np.ndarray
    cells: np.ndarray
    bfaces: np.ndarray
    btags: np.ndarray
    parents: list = field(default_factory=list)
    info: dict = field(default_factory=dict)

    @property
    def n_cells(self) -> int:
        return int(self.cells.shape[0])

    @property
    def n_nodes(self) -> int:
        return int(self.coords.shape[0])

    def level_sizes(self):
        sizes = [self.n_cells]
        for p in self.parents:
            sizes.append(int(p.max()) + 1 if p.size else 0)
        return sizes


def _radii(n_r, r_in, r_out, q):
    dr0 = (r_out - r_in) * (q - 1.0) / (q ** n_r - 1.0)
    return np.array([r_in + dr0 * (q ** k - 1.0) / (q - 1.0) for k in range(n_r + 1)])


def annulus(n_theta, n_r, r_in=0.5, r_out=10.0, q=1.2, jitter=0.0, seed=0,
            nref=2, wall_tag=SLIP, far_tag=FARFIELD):
    """Triangulated annulus r in [r_in, r_out] around a unit-diameter cylinder.

    Coarsest mesh: n_theta x n_r quads on a geometrically stretched radial
    grid (ratio q), interior rings jittered by +-jitter*h from `seed`
    (numpy default_rng, drawn ring-outer, angle-inner, x then y), each quad
    split into two counter-clockwise triangles along the (i,k)-(i+1,k+1)
    diagonal.  Then `nref` uniform 1->4 refinements by edge midpoints;
    boundary-edge midpoints are moved radially onto their circle.  Child c of
    parent p gets index 4p+c (three corner triangles, then the centre one),
    so each parent map is simply i // 4.
    """
    r = _radii(n_r, r_in, r_out, q)
    th = 2.0 * math.pi * np.arange(n_theta) / n_theta
    xy = np.zeros(((n_r + 1) * n_theta, 2))
    for k in range(n_r + 1):
        xy[k * n_theta:(k + 1) * n_theta, 0] = r[k] * np.cos(th)
        xy[k * n_theta:(k + 1) * n_theta, 1] = r[k] * np.sin(th)
    if jitter > 0.0:
        rng = np.random.default_rng(seed)
        for k in range(1, n_r):
            h = min(r[k + 1] - r[k], r[k] - r[k - 1], 2.0 * math.pi * r[k] / n_theta)
            for i in range(n_theta):
                d = rng.uniform(-1.0, 1.0, size=2)
                xy[k * n_theta + i] += jitter * h * d

    def nid(i, k):
        return k * n_theta + (i % n_theta)

    tris = []
    for k in range(n_r):
        for i in range(n_theta):
            a, b, c, d = nid(i, k), nid(i + 1, k), nid(i + 1, k + 1), nid(i, k + 1)
            tris.append((a, c, b))
            tris.append((a, d, c))
    tris = np.array(tris, dtype=np.int64)
    radius_of_node = np.full(xy.shape[0], np.nan)
    radius_of_node[:n_theta] = r_in
    radius_of_node[n_r * n_theta:] = r_out

    parents = []
    for _ in range(nref):
        xy, tris, radius_of_node = _refine_tri(xy, tris, radius_of_node)
        parents.append(np.arange(tris.shape[0], dtype=np.int64) // 4)
    parents = parents[::-1]  # parents[0] maps the finest level to the next

    bfaces, btags = [], []
    for t in tris:
        for e in ((t[0], t[1]), (t[1], t[2]), (t[2], t[0])):
            ra, rb = radius_of_node[e[0]], radius_of_node[e[1]]
            if not (np.isnan(ra) or np.isnan(rb)) and ra == rb:
                bfaces.append(e)
                btags.append(wall_tag if ra == r_in else far_tag)
    m = Mesh(dim=2, coords=np.ascontiguousarray(xy, dtype=np.float64),
             cells=np.ascontiguousarray(tris, dtype=np.int32),
             bfaces=np.ascontiguousarray(np.array(bfaces), dtype=np.int32),
             btags=np.array(btags, dtype=np.int32),
             parents=[np.ascontiguousarray(p, dtype=np.int32) for p in parents],
             info=dict(kind="annulus", n_theta=n_theta, n_r=n_r, r_in=r_in,
                       r_out=r_out, q=q, jitter=jitter, seed=seed, nref=nref))
    return m


def _refine_tri(xy, tris, radius_of_node):
    mid = {}
    new_xy = [p for p in xy]
    new_rad = list(radius_of_node)

    def midpoint(a, b):
        key = (a, b) if a < b else (b, a)
        if key in mid:
            return mid[key]
        p = 0.5 * (xy[a] + xy[b])
        ra, rb = radius_of_node[a], radius_of_node[b]
        rr = np.nan
        if not (np.isnan(ra) or np.isnan(rb)) and ra == rb:
            p = p * (ra / math.hypot(p[0], p[1]))
            rr = ra
        mid[key] = len(new_xy)
        new_xy.append(p)
        new_rad.append(rr)
        return mid[key]

    out = []
    for t in tris:
        p0, p1, p2 = int(t[0]), int(t[1]), int(t[2])
        m01, m12, m20 = midpoint(p0, p1), midpoint(p1, p2), midpoint(p2, p0)
        out += [(p0, m01, m20), (m01, p1, m12), (m20, m12, p2), (m01, m12, m20)]
    return np.array(new_xy), np.array(out, dtype=np.int64), np.array(new_rad)


def two_triangles():
    """Unit square split into two triangles, all boundaries far field."""
    xy = np.array([[0.0, 0.0], [1.0, 0.0], [1.0, 1.0], [0.0, 1.0]])
    cells = np.array([[0, 1, 2], [0, 2, 3]], dtype=np.int32)
    bf = np.array([[0, 1], [1, 2], [2, 3], [3, 0]], dtype=np.int32)
    return Mesh(2, xy, cells, bf, np.full(4, FARFIELD, dtype=np.int32), [],
                dict(kind="two_triangles"))


def structured_square(n, jitter=0.0, seed=0, tag=FARFIELD):
    """n x n unit-square grid of quads split into triangles (for small tests)."""
    rng = np.random.default_rng(seed)
    xs = np.linspace(0.0, 1.0, n + 1)
    xy = np.array([[x, y] for y in xs for x in xs])
    h = 1.0 / n
    if jitter > 0.0:
        for j in range(1, n):
            for i in range(1, n):
                xy[j * (n + 1) + i] += jitter * h * rng.uniform(-1.0, 1.0, size=2)
    cells = []
    for j in range(n):
        for i in range(n):
            a = j * (n + 1) + i
            b, c, d = a + 1, a + n + 2, a + n + 1
            cells += [(a, b, c), (a, c, d)]
    bf = []
    for i in range(n):
        bf.append((i, i + 1))
        bf.append((n * (n + 1) + i + 1, n * (n + 1) + i))
        bf.append((i * (n + 1), (i + 1) * (n + 1)))
        bf.append(((i + 1) * (n + 1) + n, i * (n + 1) + n))
    return Mesh(2, xy, np.array(cells, dtype=np.int32), np.array(bf, dtype=np.int32),
                np.full(len(bf), tag, dtype=np.int32), [], dict(kind="square", n=n))


def quad_grid_graph(nx, ny):
    """Face-adjacency graph (CSR) of an nx x ny structured quad grid."""
    xadj, adj = [0], []
    for j in range(ny):
        for i in range(nx):
            for di, dj in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                ii, jj = i + di, j + dj
                if 0 <= ii < nx and 0 <= jj < ny:
                    adj.append(jj * nx + ii)
            xadj.append(len(adj))
    return np.array(xadj, dtype=np.int32), np.array(adj, dtype=np.int32)


def draw_flow_params(seed, n, mach=(0.3, 8.0), log10_re=(3.0, 5.0)):
    """Parameter-sweep draws: Mach ~ U[mach], log10(Re) ~ U[log10_re]."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        m = rng.uniform(*mach)
        lr = rng.uniform(*log10_re)
        out.append((float(m), float(10.0 ** lr)))
    return out


_KUHN = ((0, 1, 3, 7), (0, 1, 5, 7), (0, 2, 3, 7), (0, 2, 6, 7), (0, 4, 5, 7), (0, 4, 6, 7))


def _orient_tets(xyz, tets):
    """Swap two nodes of every negatively oriented tetrahedron."""
    a, b, c, d = (xyz[tets[:, k]] for k in range(4))
    vol = np.einsum("ij,ij->i", np.cross(b - a, c - a), d - a)
    neg = vol < 0
    tets[neg, 2], tets[neg, 3] = tets[neg, 3].copy(), tets[neg, 2].copy()
    return tets


def _refine_tet(xyz, tets, surf=None, surf_r=None):
    """1 -> 8 refinement: four corner tetrahedra and the inner octahedron cut
    along the diagonal joining the midpoints of edges 02 and 13.  Child c of
    parent p is 8 p + c.  surf (optional) gives each node's sphere index (-1:
    none); the midpoint of an edge with both ends on sphere s is projected
    onto radius surf_r[s] and inherits s."""
    mid = {}
    pts = [p for p in xyz]
    sf = list(surf) if surf is not None else None

    def midpoint(a, b):
        key = (a, b) if a < b else (b, a)
        if key not in mid:
            mid[key] = len(pts)
            p = 0.5 * (xyz[a] + xyz[b])
            s_new = -1
            if sf is not None and sf[a] >= 0 and sf[a] == sf[b]:
                s_new = sf[a]
                p = p * (surf_r[s_new] / np.linalg.norm(p))
            pts.append(p)
            if sf is not None:
                sf.append(s_new)
        return mid[key]

    out = []
    for t in tets:
        p0, p1, p2, p3 = (int(x) for x in t)
        m01, m02, m03 = midpoint(p0, p1), midpoint(p0, p2), midpoint(p0, p3)
        m12, m13, m23 = midpoint(p1, p2), midpoint(p1, p3), midpoint(p2, p3)
        out += [(p0, m01, m02, m03), (m01, p1, m12, m13), (m02, m12, p2, m23), (m03, m13, m23, p3),
                (m02, m13, m01, m03), (m02, m13, m03, m23), (m02, m13, m23, m12), (m02, m13, m12, m01)]
    xyz = np.array(pts)
    tets = _orient_tets(xyz, np.array(out, dtype=np.int64))
    if sf is None:
        return xyz, tets
    return xyz, tets, np.array(sf)


def _boundary_faces(tets):
    faces = np.concatenate([tets[:, [1, 2, 3]], tets[:, [0, 2, 3]], tets[:, [0, 1, 3]], tets[:, [0, 1, 2]]])
    key = np.sort(faces, axis=1)
    _, first, count = np.unique(key, axis=0, return_index=True, return_counts=True)
    return faces[first[count == 1]]


def box_tets(n, nref=2, jitter=0.0, seed=0, tags=None, size=1.0):
    """Cube [0, size]^3 of n^3 hexahedra, each split into 6 tetrahedra along its
    main diagonal (a conforming split), interior nodes jittered by +-jitter*h,
    then refined 1 -> 8 nref times.  tags maps a side ('x0', 'x1', 'y0', 'y1',
    'z0', 'z1') to its boundary tag (default far field)."""
    rng = np.random.default_rng(seed)
    side_tag = {k: FARFIELD for k in ("x0", "x1", "y0", "y1", "z0", "z1")}
    side_tag.update(tags or {})
    h = size / n
    g = np.linspace(0.0, size, n + 1)
    xyz = np.array([[x, y, z] for z in g for y in g for x in g], dtype=np.float64)
    if jitter > 0.0:
        for k in range(1, n):
            for j in range(1, n):
                for i in range(1, n):
                    xyz[(k * (n + 1) + j) * (n + 1) + i] += jitter * h * rng.uniform(-1.0, 1.0, size=3)

    def nid(i, j, k):
        return (k * (n + 1) + j) * (n + 1) + i

    tets = []
    for k in range(n):
        for j in range(n):
            for i in range(n):
                v = [nid(i + (c & 1), j + ((c >> 1) & 1), k + ((c >> 2) & 1)) for c in range(8)]
                tets += [tuple(v[a] for a in t) for t in _KUHN]
    tets = _orient_tets(xyz, np.array(tets, dtype=np.int64))
    parents = []
    for _ in range(nref):
        xyz, tets = _refine_tet(xyz, tets)
        parents.insert(0, np.arange(len(tets), dtype=np.int32) // 8)
    bf = _boundary_faces(tets)   # faces used by exactly one tetrahedron
    btags = []
    tol = 1e-12 * size
    for f in bf:
        c = xyz[f]
        for d, ax in enumerate("xyz"):
            if np.all(np.abs(c[:, d]) < tol):
                btags.append(side_tag[ax + "0"])
                break
            if np.all(np.abs(c[:, d] - size) < tol):
                btags.append(side_tag[ax + "1"])
                break
        else:
            raise ValueError("boundary face off the box")
    return Mesh(3, np.ascontiguousarray(xyz), np.ascontiguousarray(tets, dtype=np.int32),
                np.ascontiguousarray(bf, dtype=np.int32), np.array(btags, dtype=np.int32), parents,
                dict(kind="box_tets", n=n, nref=nref, jitter=jitter, seed=seed))


def sphere_shell(n_az, n_pol, n_rad, r_in=0.5, r_out=6.0, q=1.2, nref=2, jitter=0.0, seed=0,
                 wall_tag=SLIP, far_tag=FARFIELD):
    """Spherical shell r in [r_in, r_out] around a unit-diameter sphere: an
    (azimuth x polar x radial) grid of hexahedra, each split into 6
    tetrahedra along its index-space diagonal; the polar grid lines collapse
    into one node per radius and the tetrahedra that degenerate there are
    dropped; refined 1 -> 8 nref times with the midpoints of edges on the
    inner or outer sphere projected onto it.  Child c of parent p is 8 p + c."""
    rng = np.random.default_rng(seed)
    radii = _radii(n_rad, r_in, r_out, q)
    nid = {}
    pts = []
    for k in range(n_rad + 1):
        for j in range(n_pol + 1):
            for i in range(n_az):
                key = (0 if j in (0, n_pol) else i, j, k)
                if key in nid:
                    continue
                th = math.pi * j / n_pol
                ph = 2.0 * math.pi * i / n_az
                r = radii[k]
                if jitter > 0.0 and 0 < k < n_rad and 0 < j < n_pol:
                    h = r * math.pi / n_pol
                    r += jitter * h * rng.uniform(-1.0, 1.0)
                    th += jitter * (math.pi / n_pol) * rng.uniform(-1.0, 1.0) * 0.5
                    ph += jitter * (2.0 * math.pi / n_az) * rng.uniform(-1.0, 1.0) * 0.5
                nid[key] = len(pts)
                pts.append([r * math.sin(th) * math.cos(ph), r * math.sin(th) * math.sin(ph), r * math.cos(th)])
    xyz = np.array(pts, dtype=np.float64)

    def node(i, j, k):
        return nid[(0 if j in (0, n_pol) else i % n_az, j, k)]

    tets = []
    for k in range(n_rad):
        for j in range(n_pol):
            for i in range(n_az):
                v = [node(i + (c & 1), j + ((c >> 1) & 1), k + ((c >> 2) & 1)) for c in range(8)]
                for t in _KUHN:
                    tt = tuple(v[a] for a in t)
                    if len(set(tt)) == 4:
                        tets.append(tt)
    tets = _orient_tets(xyz, np.array(tets, dtype=np.int64))
    rad = np.linalg.norm(xyz, axis=1)
    surf = np.where(np.isclose(rad, r_in), 0, np.where(np.isclose(rad, r_out), 1, -1))
    parents = []
    for _ in range(nref):
        xyz, tets, surf = _refine_tet(xyz, tets, surf, (r_in, r_out))
        parents.insert(0, np.arange(len(tets), dtype=np.int32) // 8)
    bf = _boundary_faces(tets)
    on = surf[bf]
    if not np.all((on == on[:, :1]) & (on >= 0)):
        raise ValueError("boundary face off the bounding spheres")
    btags = np.where(on[:, 0] == 0, wall_tag, far_tag).astype(np.int32)
    return Mesh(3, np.ascontiguousarray(xyz), np.ascontiguousarray(tets, dtype=np.int32),
                np.ascontiguousarray(bf, dtype=np.int32), btags, parents,
                dict(kind="sphere_shell", n_az=n_az, n_pol=n_pol, n_rad=n_rad, r_in=r_in, r_out=r_out,
                     q=q, nref=nref, jitter=jitter, seed=seed))


# Named workloads ----------------------------------------------------------

def cylinder_euler_small(seed=0):
    """Inviscid Mach 0.38 cylinder: 32x8 coarsest quads, 2 refinements -> 8,192 triangles."""
    return annulus(32, 8, jitter=0.15, seed=seed, nref=2, wall_tag=SLIP)


def cylinder_ns_large(seed=1):
    """Viscous Mach 8 cylinder: 128x32 coarsest quads, 2 refinements -> 131,072 triangles."""
    return annulus(128, 32, jitter=0.10, seed=seed, nref=2, wall_tag=ISOTHERMAL)
