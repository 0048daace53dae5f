"""Pins of the oracle's mesh set-up, colouring (Alg. 1) and agglomeration (Alg. 3).

Geometry is checked against independent formulas (numpy cross products,
the boundary polygon's shoelace area, closure of every cell); colouring by
brute force over all face-adjacent pairs and by a separate Python BFS on
tiny meshes; agglomeration by its structural invariants and by a separate
Python implementation of the same reading on a tiny mesh.
"""
import math
from collections import deque

import numpy as np
import pytest

import synthmesh as sm


def tri_areas(m):
    x = m.coords
    c = m.cells
    return 0.5 * ((x[c[:, 1], 0] - x[c[:, 0], 0]) * (x[c[:, 2], 1] - x[c[:, 0], 1])
                  - (x[c[:, 2], 0] - x[c[:, 0], 0]) * (x[c[:, 1], 1] - x[c[:, 0], 1]))


@pytest.fixture(scope="module")
def small_annulus():
    return sm.annulus(16, 4, jitter=0.15, seed=7, nref=2)


def test_geometry_closure_and_volumes(orc, small_annulus):
    m = small_annulus
    o = orc.Oracle(m, n_levels=3)
    V, C = o.cell_geometry(0)
    np.testing.assert_allclose(V, tri_areas(m), rtol=1e-14)
    np.testing.assert_allclose(C, m.coords[m.cells].mean(axis=1), rtol=1e-13, atol=1e-14)
    # boundary polygon area by the shoelace formula over the tagged boundary edges
    b = m.bfaces
    x = m.coords
    # orient each boundary edge counter-clockwise around the domain (its cell is on the left)
    area = 0.0
    for l in range(3):
        fg = o.face_geometry(l)
        nc = o.sizes[l][0]
        Vl, Cl = o.cell_geometry(l)
        clos = np.zeros((nc, 2))
        for f in range(len(fg["S"])):
            L, R = fg["LR"][f]
            clos[L] += fg["S"][f] * fg["n"][f]
            if R >= 0:
                clos[R] -= fg["S"][f] * fg["n"][f]
        assert np.abs(clos).max() <= 1e-13 * fg["S"].max()
        np.testing.assert_allclose(Vl.sum(), V.sum(), rtol=1e-13)
        # faces: interior faces shared by two cells, boundary faces once
        nb = (fg["LR"][:, 1] < 0).sum()
        if l == 0:
            assert nb == len(m.btags)
            assert 2 * (len(fg["S"]) - nb) + nb == 3 * nc
    shoelace = 0.0
    fg = o.face_geometry(0)
    for f in np.where(fg["LR"][:, 1] < 0)[0]:
        # outward normal n; the edge direction keeping the domain on the left is (-n_y, n_x)
        t = np.array([-fg["n"][f][1], fg["n"][f][0]])
        mid = fg["xc"][f]
        a, c = mid - 0.5 * fg["S"][f] * t, mid + 0.5 * fg["S"][f] * t
        shoelace += 0.5 * (a[0] * c[1] - c[0] * a[1])
    assert V.sum() == pytest.approx(shoelace, rel=1e-12)


def test_coarse_volumes_are_sums_of_children(orc, small_annulus):
    o = orc.Oracle(small_annulus, n_levels=3)
    V0, C0 = o.cell_geometry(0)
    V1, C1 = o.cell_geometry(1)
    V2, _ = o.cell_geometry(2)
    p0, p1 = small_annulus.parents
    np.testing.assert_allclose(np.bincount(p0, weights=V0), V1, rtol=1e-14)
    np.testing.assert_allclose(np.bincount(p1, weights=V1), V2, rtol=1e-14)
    for d in range(2):
        np.testing.assert_allclose(np.bincount(p0, weights=V0 * C0[:, d]) / V1, C1[:, d], rtol=1e-13, atol=1e-13)


def _python_bfs_colouring(n, nbrs):
    """Independent implementation of the colouring reading (BFS from cell 0)."""
    col = [0] * n
    for s in range(n):
        if col[s]:
            continue
        used = {col[j] for j in nbrs[s] if col[j]}
        k = 1
        while k in used:
            k += 1
        col[s] = k
        q = deque([s])
        while q:
            v = q.popleft()
            for w in nbrs[v]:
                if col[w] == 0:
                    used = {col[j] for j in nbrs[w] if col[j]}
                    k = 1
                    while k in used:
                        k += 1
                    col[w] = k
                    q.append(w)
    return np.array(col)


def _neighbours_local_order(o, level):
    fg = o.face_geometry(level)
    n = o.sizes[level][0]
    nb = [[] for _ in range(n)]
    if level == 0:
        # fine local order = face opposite local node k; rebuild it from node sets
        return None
    for f, (L, R) in enumerate(fg["LR"]):
        if R >= 0:
            nb[L].append(R)
            nb[R].append(L)
    return [sorted(x) for x in nb]


def test_colouring_is_valid_and_matches_python_bfs(orc, small_annulus):
    o = orc.Oracle(small_annulus, n_levels=3)
    for l in (1, 2):
        col, nc = o.coloring(l)
        fg = o.face_geometry(l)
        LR = fg["LR"][fg["LR"][:, 1] >= 0]
        assert (col[LR[:, 0]] != col[LR[:, 1]]).all()
        assert col.min() == 1 and col.max() == nc
        nbrs = _neighbours_local_order(o, l)
        assert nc <= max(len(x) for x in nbrs) + 1
        assert (col == _python_bfs_colouring(len(nbrs), nbrs)).all()


def test_colouring_brute_force_all_pairs_tiny(orc):
    m = sm.structured_square(3, jitter=0.2, seed=2)
    o = orc.Oracle(m, n_levels=1)
    col, nc = o.coloring(0)
    cells = [set(c) for c in m.cells]
    for i in range(len(cells)):
        for j in range(i + 1, len(cells)):
            if len(cells[i] & cells[j]) == 2:   # share an edge
                assert col[i] != col[j]


def test_structured_quad_grid_paints_with_two_colours(orc):
    """A regular structured mesh is painted with exactly two colours (Sec. 4.1)."""
    for nx, ny in ((4, 4), (7, 5)):
        xadj, adj = sm.quad_grid_graph(nx, ny)
        col, nc = orc.coloring_graph(xadj, adj)
        assert nc == 2
        ij = np.array([(i + j) % 2 for j in range(ny) for i in range(nx)])
        assert (col == 1 + ij).all()


def _python_agglomerate(o, skew_limit=0.2):
    """Independent implementation of the Alg. 3 reading on the fine level."""
    fg = o.face_geometry(0)
    V, C = o.cell_geometry(0)
    n = o.sizes[0][0]
    LR = fg["LR"]
    interior = [f for f in range(len(LR)) if LR[f, 1] >= 0]
    Nf = len(interior)
    seen, chosen = set(), []
    for f in interior:
        a, b = int(LR[f, 0]), int(LR[f, 1])
        h = (23 * (a + b) + a * b) % Nf
        if h not in seen:
            seen.add(h)
            chosen.append(f)
    cell_faces = [[] for _ in range(n)]
    for f, (a, b) in enumerate(LR):
        cell_faces[a].append(f)
        if b >= 0:
            cell_faces[b].append(f)
    group = [-1] * n
    for f in chosen:
        a, b = int(LR[f, 0]), int(LR[f, 1])
        if group[a] >= 0 or group[b] >= 0:
            continue
        Cc = (V[a] * C[a] + V[b] * C[b]) / (V[a] + V[b])
        mins = 2.0
        for X in (a, b):
            for g in cell_faces[X]:
                if g == f:
                    continue
                nv = fg["n"][g] * (1.0 if LR[g, 0] == X else -1.0)
                d = fg["xc"][g] - Cc
                mins = min(mins, float(d @ nv) / math.sqrt(float(d @ d)))
        if mins >= skew_limit:
            group[a] = group[b] = f
    agg, gid, nxt = [], {}, 0
    for i in range(n):
        if group[i] < 0:
            agg.append(nxt)
            nxt += 1
        elif group[i] in gid:
            agg.append(gid[group[i]])
        else:
            gid[group[i]] = nxt
            agg.append(nxt)
            nxt += 1
    return np.array(agg), nxt


def test_agglomeration_invariants_and_python_reading(orc):
    m = sm.annulus(8, 3, jitter=0.2, seed=5, nref=1)
    o = orc.Oracle(m, n_levels=1)
    agg, nc = o.agglomerate(0)
    ref, nref = _python_agglomerate(o)
    assert nc == nref and (agg == ref).all()
    counts = np.bincount(agg)
    assert counts.min() >= 1 and counts.max() <= 2 and counts.sum() == m.n_cells
    # first-appearance numbering
    firsts = [np.where(agg == k)[0][0] for k in range(nc)]
    assert firsts == sorted(firsts)
    # merged pairs are face neighbours whose separating face hashes are distinct
    fg = o.face_geometry(0)
    pair_face = {}
    for f, (a, b) in enumerate(fg["LR"]):
        if b >= 0 and agg[a] == agg[b]:
            pair_face[agg[a]] = f
    assert len(pair_face) == (counts == 2).sum()
    Nf = int((fg["LR"][:, 1] >= 0).sum())
    hashes = [(23 * (int(fg["LR"][f, 0]) + int(fg["LR"][f, 1])) + int(fg["LR"][f, 0]) * int(fg["LR"][f, 1])) % Nf
              for f in pair_face.values()]
    assert len(set(hashes)) == len(hashes)


def test_agglomerated_hierarchy_conserves_volume(orc):
    m = sm.annulus(8, 3, jitter=0.1, seed=5, nref=2)
    o = orc.Oracle(m, n_levels=3, use_parents=False)
    V0, _ = o.cell_geometry(0)
    for l in (1, 2):
        Vl, _ = o.cell_geometry(l)
        assert Vl.sum() == pytest.approx(V0.sum(), rel=1e-13)
        assert o.sizes[l][0] < o.sizes[l - 1][0]


def test_invalid_mesh_is_rejected(orc):
    m = sm.two_triangles()
    bad = sm.Mesh(2, m.coords, m.cells[:, ::-1].copy(), m.bfaces, m.btags, [])
    with pytest.raises(orc.OracleError):
        orc.Oracle(bad, n_levels=1)
    missing = sm.Mesh(2, m.coords, m.cells, m.bfaces[:3], m.btags[:3], [])
    with pytest.raises(orc.OracleError):
        orc.Oracle(missing, n_levels=1)
