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
    """A mesh with boundary faces and refinement parent maps.

    coords      float64 [n_nodes, dim]
    cells       int32   [n_cells, dim+1], positively oriented simplices; or,
                when cell_offsets is given (3-D mixed elements), the flat node
                list of every cell, cell i being cells[cell_offsets[i]:
                cell_offsets[i+1]] (4, 5, 6 or 8 nodes: tetrahedron, pyramid,
                prism, hexahedron in the node orders of ELEMENT_ORDER)
    bfaces      int32   [n_bfaces, dim]   node ids of boundary faces; or flat
                (3 or 4 nodes each) when bface_offsets is given
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
    cell_offsets: np.ndarray = None
    bface_offsets: np.ndarray = None

    @property
    def n_cells(self) -> int:
        if self.cell_offsets is not None:
            return int(len(self.cell_offsets) - 1)
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


C4_SHAPES = ((32, 8), (64, 8), (64, 16), (128, 16), (128, 32))


def parameter_sweep(n=64, seed=4, mesh_seed0=4000):
    """The batched parameter sweep: n cylinder annuli whose coarsest (N_theta,
    N_r) is drawn uniformly from C4_SHAPES (8,192 to 131,072 fine triangles
    after two refinements; jitter 0.1, mesh seed mesh_seed0 + b, isothermal
    wall), each with its own Mach ~ U[0.3, 8] and log10 Re ~ U[3, 5] (one
    generator, seeded with `seed`, draws the shapes, then the flows).
    Returns [(mesh, flow parameters)]."""
    rng = np.random.default_rng(seed)
    shapes = [C4_SHAPES[int(k)] for k in rng.integers(0, len(C4_SHAPES), size=n)]
    flows = draw_flow_params(seed, n)
    out = []
    for b, ((nt, nr), (mach, re)) in enumerate(zip(shapes, flows)):
        mesh = annulus(nt, nr, jitter=0.1, seed=mesh_seed0 + b, nref=2, wall_tag=ISOTHERMAL)
        out.append((mesh, dict(mach=mach, reynolds=re, prandtl=0.72, wall_T_ratio=1.0)))
    return out


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


def _kuhn_tets(na, npol, nrad):
    """Kuhn triangulation of the index grid [0, na) x [0, npol) x [0, nrad)
    (azimuth periodic): cube (i, j, k) is cut into 6 tetrahedra along its
    (0,0,0)-(1,1,1) diagonal, one per order in which the path from corner
    (0,0,0) steps along the three axes (_KUHN).  Returns the cube origins
    [n, 3] and the order ids [n] of all tetrahedra, order fastest."""
    i, j, k = np.meshgrid(np.arange(na), np.arange(npol), np.arange(nrad), indexing="ij")
    org = np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1)
    org = np.repeat(org, 6, axis=0)
    perm = np.tile(np.arange(6), len(org) // 6)
    return org, perm


# Axis stepping order of each _KUHN tetrahedron (0 = azimuth, 1 = polar, 2 = radial).
_KUHN_ORDER = np.array([(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)])


def _kuhn_parent(org, perm):
    """The Kuhn tetrahedron of the grid with half the resolution that contains
    each given tetrahedron (Freudenthal refinement nests the two): the cube
    and stepping order of the centroid, computed exactly in index units."""
    c4 = 4 * org.astype(np.int64)                   # centroid x 4, integer
    step = np.array([3, 2, 1])
    for t in range(3):
        c4[np.arange(len(org)), _KUHN_ORDER[perm, t]] += step[t]
    cube = c4 // 8                                  # parent cube (coarse units: c / 2)
    frac = c4 - 8 * cube                            # 8 x fractional part, distinct per axis
    order = np.argsort(-frac, axis=1, kind="stable")
    key = order[:, 0] * 3 + order[:, 1]
    table = np.full(9, -1)
    for n, (a, b, _) in enumerate(_KUHN_ORDER):
        table[a * 3 + b] = n
    return cube, table[key]


def sphere_shell_kuhn(n_az, n_pol, n_rad, r_in=0.5, r_out=6.0, q=1.2, nref=2,
                      wall_tag=SLIP, far_tag=FARFIELD):
    """Spherical shell r in [r_in, r_out] around a unit-diameter sphere, as
    the Kuhn triangulation of an (azimuth x polar x radial) index grid refined
    2^nref times: the finest level is the Kuhn triangulation of the
    (2^nref n_az) x (2^nref n_pol) x (2^nref n_rad) grid mapped by
    phi = 2 pi i / N_az, theta = pi j / N_pol and the geometric radial map
    r(s) = r_in + dr0 (q^s - 1) / (q - 1) (s in coarse index units,
    dr0 = (r_out - r_in)(q - 1) / (q^n_rad - 1)).  The nodes of each polar
    grid line collapse into one per radius; the tetrahedra with repeated
    nodes there (three of the six in every cube of a polar row) are dropped.
    The parent of a tetrahedron is the Kuhn tetrahedron of the grid of half
    the resolution that contains it (Freudenthal refinement nests them), so
    each coarse cell is the agglomerate of its surviving fine descendants.
    Cells are numbered parent-major on every level."""
    f = 2 ** nref
    NA, NP, NR = n_az * f, n_pol * f, n_rad * f
    dr0 = (r_out - r_in) * (q - 1.0) / (q ** n_rad - 1.0)
    # nodes: (i mod NA, j, k) with the two polar lines merged per radius
    ii, jj, kk = np.meshgrid(np.arange(NA), np.arange(NP + 1), np.arange(NR + 1), indexing="ij")
    pole = (jj == 0) | (jj == NP)
    keep = ~pole | (ii == 0)
    nid = -np.ones((NA, NP + 1, NR + 1), dtype=np.int64)
    nid[keep] = np.arange(int(keep.sum()))
    nid[:, 0, :] = nid[0, 0, :]
    nid[:, NP, :] = nid[0, NP, :]
    s = kk[keep] / float(f)
    r = r_in + dr0 * (q ** s - 1.0) / (q - 1.0)
    r[kk[keep] == NR] = r_out
    th = np.pi * jj[keep] / NP
    ph = 2.0 * np.pi * ii[keep] / NA
    xyz = np.stack([r * np.sin(th) * np.cos(ph), r * np.sin(th) * np.sin(ph), r * np.cos(th)], axis=1)
    # finest Kuhn tetrahedra
    org, perm = _kuhn_tets(NA, NP, NR)
    verts = np.empty((len(org), 4, 3), dtype=np.int64)
    verts[:, 0] = org
    for t in range(3):
        verts[:, t + 1] = verts[:, t]
        verts[np.arange(len(org)), t + 1, _KUHN_ORDER[perm, t]] += 1
    ids = nid[verts[..., 0] % NA, verts[..., 1], verts[..., 2]]
    srt = np.sort(ids, axis=1)
    good = np.all(srt[:, 1:] != srt[:, :-1], axis=1)
    org, perm, ids = org[good], perm[good], ids[good]
    # hierarchy: parent Kuhn tetrahedra level by level, as flat ids
    lev_org, lev_perm = [org], [perm]
    dims = [(NA, NP, NR)]
    for l in range(nref):
        o, p_ = _kuhn_parent(lev_org[-1], lev_perm[-1])
        lev_org.append(o)
        lev_perm.append(p_)
        na, npl, nr = dims[-1]
        dims.append((na // 2, npl // 2, nr // 2))

    def flat(o, p_, d):
        return ((o[:, 0] * d[1] + o[:, 1]) * d[2] + o[:, 2]) * 6 + p_

    keys = [flat(lev_org[l], lev_perm[l], dims[l]) for l in range(nref + 1)]
    # parent-major numbering from the coarsest level down
    order = np.lexsort(tuple(keys[l] for l in range(nref + 1)))   # last key is primary
    ids = ids[order]
    keys = [k_[order] for k_ in keys]
    def by_first_appearance(k_):
        _, first, inv = np.unique(k_, return_index=True, return_inverse=True)
        return np.argsort(np.argsort(first))[inv]

    lid = [by_first_appearance(k_) for k_ in keys]      # per fine row: its cell's index on level l
    parents = []
    for l in range(nref):
        par = np.empty(lid[l].max() + 1, dtype=np.int64)
        par[lid[l]] = lid[l + 1]
        parents.append(par.astype(np.int32))
    tets = _orient_tets(xyz, ids.copy())
    bf = _boundary_faces(tets)
    rad = np.linalg.norm(xyz[bf], axis=2)
    on_in = np.all(np.isclose(rad, r_in), axis=1)
    on_out = np.all(np.isclose(rad, r_out), axis=1)
    if not np.all(on_in | on_out):
        raise ValueError("boundary face off the bounding spheres")
    btags = np.where(on_in, wall_tag, far_tag).astype(np.int32)
    return Mesh(3, np.ascontiguousarray(xyz), np.ascontiguousarray(tets, dtype=np.int32),
                np.ascontiguousarray(bf, dtype=np.int32), btags, parents,
                dict(kind="sphere_shell_kuhn", n_az=n_az, n_pol=n_pol, n_rad=n_rad, r_in=r_in, r_out=r_out,
                     q=q, nref=nref))


# Mixed-element meshes -----------------------------------------------------

ELEMENT_ORDER = """Node orders of the mixed-element input format:
tetrahedron (4 nodes) any order; pyramid (5): the base quadrilateral in
cyclic order, then the apex; prism (6): one triangle, then the other with
node 3+k joined to node k by an edge; hexahedron (8): one quadrilateral in
cyclic order, then the opposite one with node 4+k joined to node k."""


def hybrid_box(n, seed=0, grade=0.3, taper=0.3, p_prism=0.3, p_pyramid=0.25, tags=None):
    """Box of n^3 cubes (n even) filled with all four 3-D element types.

    The grid lines of each axis are spaced by seeded factors in
    [1 - grade, 1 + grade] on [0, 1]; then the frustum map scales x and y
    about 0.5 by (1 + taper z), which keeps every face planar (the faces of
    constant x or y become trapezoids, the hexahedra non-affine).  Columns
    (i, j) drawn with probability p_prism are cut into two prisms per cube
    along the diagonal from corner (i, j) to (i+1, j+1); in the other columns
    vertical pairs of cubes (k, k+1), k even, drawn with probability
    p_pyramid, become six pyramids each (apex at a new node at the cube's
    centre), and the two pyramids on the quadrilateral the pair shares are
    cut into two tetrahedra each along the same diagonal; every other cube is
    a hexahedron.  Cells are numbered cube by cube and cubes in Morton order,
    so that the 8 cubes of each 2 x 2 x 2 block are consecutive: parents[0]
    maps a cell to its cube and parents[1] a cube to its block.  tags maps
    a side ('x0', 'x1', 'y0', 'y1', 'z0', 'z1') to its boundary tag
    (default far field).  Node orders: ELEMENT_ORDER."""
    if n % 2:
        raise ValueError("n must be even")
    rng = np.random.default_rng(seed)
    side_tag = {k: FARFIELD for k in ("x0", "x1", "y0", "y1", "z0", "z1")}
    side_tag.update(tags or {})

    def axis():
        w = rng.uniform(1.0 - grade, 1.0 + grade, size=n)
        g = np.concatenate([[0.0], np.cumsum(w)]) / w.sum()
        g[-1] = 1.0
        return g

    gx, gy, gz = axis(), axis(), axis()
    prism_col = rng.random((n, n)) < p_prism
    pyr_pair = rng.random((n, n, n // 2)) < p_pyramid
    # nodes: grid nodes (i, j, k) with k fastest, then one centre node per pyramid cube
    X, Y, Z = np.meshgrid(gx, gy, gz, indexing="ij")
    unit = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    n1 = n + 1
    # cubes in Morton (bit-interleaved) order of (i, j, k): the 8 cubes of a
    # 2 x 2 x 2 block stay consecutive, and so do larger blocks, which keeps
    # most face neighbours close in the numbering; corners a = (a&1, a>>1&1, a>>2&1)
    I, J, K = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    I, J, K = I.ravel(), J.ravel(), K.ravel()
    code = np.zeros(n ** 3, dtype=np.int64)
    for b in range(int(np.ceil(np.log2(n))) + 1):
        code |= ((I >> b) & 1) << (3 * b) | ((J >> b) & 1) << (3 * b + 1) | ((K >> b) & 1) << (3 * b + 2)
    morton = np.argsort(code, kind="stable")
    ci, cj, ck = I[morton], J[morton], K[morton]
    a = np.arange(8)
    v = ((ci[:, None] + (a & 1)) * n1 + cj[:, None] + ((a >> 1) & 1)) * n1 + ck[:, None] + ((a >> 2) & 1)
    is_prism = prism_col[ci, cj]
    is_pyr = ~is_prism & pyr_pair[ci, cj, ck // 2]
    ncube = len(ci)
    cube_ids = np.arange(ncube)
    groups = []    # (cube index, local index, node array [m, nn])
    hexc = ~is_prism & ~is_pyr
    groups.append((cube_ids[hexc], 0, v[hexc][:, [0, 1, 3, 2, 4, 5, 7, 6]]))
    groups.append((cube_ids[is_prism], 0, v[is_prism][:, [0, 1, 3, 4, 5, 7]]))
    groups.append((cube_ids[is_prism], 1, v[is_prism][:, [0, 3, 2, 4, 7, 6]]))
    pc = cube_ids[is_pyr]
    cn = len(unit) + np.arange(len(pc))
    centres = np.stack([0.5 * (gx[ci[pc]] + gx[ci[pc] + 1]), 0.5 * (gy[cj[pc]] + gy[cj[pc] + 1]),
                        0.5 * (gz[ck[pc]] + gz[ck[pc] + 1])], axis=1)
    unit = np.concatenate([unit, centres])
    quads = [[0, 1, 3, 2], [4, 5, 7, 6], [0, 1, 5, 4], [1, 3, 7, 5], [3, 2, 6, 7], [2, 0, 4, 6]]
    vp = v[pc]
    shared = np.where(ck[pc] % 2 == 0, 1, 0)       # the face towards the pair's other cube
    for f, q in enumerate(quads):
        qn = vp[:, q]
        keep = shared != f
        groups.append((pc[keep], 2 * f, np.concatenate([qn[keep], cn[keep, None]], axis=1)))
        cut = ~keep
        groups.append((pc[cut], 2 * f, np.concatenate([qn[cut][:, [0, 1, 2]], cn[cut, None]], axis=1)))
        groups.append((pc[cut], 2 * f + 1, np.concatenate([qn[cut][:, [0, 2, 3]], cn[cut, None]], axis=1)))
    cube_all = np.concatenate([g[0] for g in groups])
    local_all = np.concatenate([np.full(len(g[0]), g[1]) for g in groups])
    order = np.lexsort((local_all, cube_all))
    lens = np.concatenate([np.full(len(g[0]), g[2].shape[1]) for g in groups])
    flat = np.concatenate([g[2].ravel() for g in groups])
    starts = np.concatenate([[0], np.cumsum(lens)[:-1]])
    coff = np.concatenate([[0], np.cumsum(lens[order])]).astype(np.int32)
    cells_flat = flat[np.repeat(starts[order] - coff[:-1], lens[order]) + np.arange(coff[-1])]
    cube_of = cube_all[order]
    s = 1.0 + taper * unit[:, 2]
    xyz = np.stack([(unit[:, 0] - 0.5) * s + 0.5, (unit[:, 1] - 0.5) * s + 0.5, unit[:, 2]], axis=1)
    # boundary faces: cell faces that occur once (local face tables of the node orders)
    ftab = {4: [(1, 2, 3), (0, 2, 3), (0, 1, 3), (0, 1, 2)],
            5: [(0, 1, 2, 3), (0, 1, 4), (1, 2, 4), (2, 3, 4), (3, 0, 4)],
            6: [(0, 1, 2), (3, 4, 5), (0, 1, 4, 3), (1, 2, 5, 4), (2, 0, 3, 5)],
            8: [(0, 1, 2, 3), (4, 5, 6, 7), (0, 1, 5, 4), (1, 2, 6, 5), (2, 3, 7, 6), (3, 0, 4, 7)]}
    faces = []
    for g in groups:
        for f in ftab[g[2].shape[1]]:
            fa = np.full((len(g[0]), 4), -1, dtype=np.int64)
            fa[:, :len(f)] = g[2][:, list(f)]
            faces.append(fa)
    faces = np.concatenate(faces)
    key = np.sort(faces, axis=1) + 1                 # node ids + 1 (0 pads a triangle)
    hi, lo = key[:, 0] << 32 | key[:, 1], key[:, 2] << 32 | key[:, 3]
    srt = np.lexsort((lo, hi))
    hs, ls = hi[srt], lo[srt]
    new_key = np.concatenate([[True], (hs[1:] != hs[:-1]) | (ls[1:] != ls[:-1])])
    grp = np.cumsum(new_key) - 1
    count = np.bincount(grp)
    once = srt[new_key][count == 1]                  # faces used by one cell, in key order
    bfaces, btags = [], []
    tol = 1e-12
    for row in faces[once]:
        nodes = [int(v) for v in row if v >= 0]
        u = unit[nodes]
        for d, ax in enumerate("xyz"):
            if np.all(np.abs(u[:, d]) < tol):
                btags.append(side_tag[ax + "0"])
                break
            if np.all(np.abs(u[:, d] - 1.0) < tol):
                btags.append(side_tag[ax + "1"])
                break
        else:
            raise ValueError("boundary face off the box")
        bfaces.append(nodes)
    boff = np.concatenate([[0], np.cumsum([len(f) for f in bfaces])]).astype(np.int32)
    parents = [cube_of.astype(np.int32), (np.arange(n ** 3, dtype=np.int32) // 8)]
    kinds = np.bincount(np.diff(coff), minlength=9)
    return Mesh(3, np.ascontiguousarray(xyz), cells_flat.astype(np.int32),
                np.array([v for f in bfaces for v in f], dtype=np.int32), np.array(btags, dtype=np.int32),
                parents, dict(kind="hybrid_box", n=n, seed=seed, grade=grade, taper=taper,
                              tets=int(kinds[4]), pyramids=int(kinds[5]), prisms=int(kinds[6]),
                              hexahedra=int(kinds[8])),
                cell_offsets=coff, bface_offsets=boff)


# Named workloads ----------------------------------------------------------

def cylinder_euler_small(seed=0):
    """Inviscid Mach 0.38 cylinder: 32x8 coarsest quads, 2 refinements -> 8,192 triangles."""
    return annulus(32, 8, jitter=0.15, seed=seed, nref=2, wall_tag=SLIP)


def cylinder_ns_large(seed=1):
    """Viscous Mach 8 cylinder: 128x32 coarsest quads, 2 refinements -> 131,072 triangles."""
    return annulus(128, 32, jitter=0.10, seed=seed, nref=2, wall_tag=ISOTHERMAL)
