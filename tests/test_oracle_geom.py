"""Pins of the oracle's geometry against things other than itself: exact
rational arithmetic, the brute-force definition of point location, the
convex hull (scipy Qhull), affine reproduction by linear elements (the
piece-wise linear case of Sec. III) and a hand-derived worked example."""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import meshgen as G
import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def exact_bary(verts, y):
    """Barycentric coordinates in exact rational arithmetic (Cramer's rule)."""
    V = [[Fraction(float(c)) for c in row] for row in verts]
    Y = [Fraction(float(c)) for c in y]
    dim = len(Y)
    E = [[V[k + 1][d] - V[0][d] for d in range(dim)] for k in range(dim)]
    Q = [Y[d] - V[0][d] for d in range(dim)]
    if dim == 2:
        det = E[0][0] * E[1][1] - E[1][0] * E[0][1]
        if det == 0:
            return None
        lb = (Q[0] * E[1][1] - E[1][0] * Q[1]) / det
        lc = (E[0][0] * Q[1] - Q[0] * E[0][1]) / det
        return [1 - lb - lc, lb, lc]

    def det3(a, b, c):
        return (a[0] * (b[1] * c[2] - b[2] * c[1]) - a[1] * (b[0] * c[2] - b[2] * c[0])
                + a[2] * (b[0] * c[1] - b[1] * c[0]))
    d = det3(E[0], E[1], E[2])
    if d == 0:
        return None
    lb = det3(Q, E[1], E[2]) / d
    lc = det3(E[0], Q, E[2]) / d
    ld = det3(E[0], E[1], Q) / d
    return [1 - lb - lc - ld, lb, lc, ld]


def test_golden_two_triangles():
    fx = json.load(open(os.path.join(GOLDEN, "two_triangles.json")))
    coords = np.array(fx["coords"], np.float32)
    cells = np.array(fx["cells"], np.int32)
    x = np.array(fx["field"], np.float64)
    e = fx["expect"]
    g = O.grid_from_dims(coords, fx["dims"])
    assert list(g.o)[:2] == e["origin"] and list(g.h)[:2] == e["spacing"]
    for method in ("brute", "raster"):
        m = O.locate(coords, cells, g, method)
        assert m.cell.tolist() == e["cell_of_node"]
        assert m.vid.tolist() == e["vid"]
        assert m.w.tolist() == e["w"]
    b = O.bound(x, fx["eb_abs"], False, fx["split"])
    assert (b.tau, b.tau1, b.tau2, b.c) == (e["tau"], e["tau1"], e["tau2"], e["c"])
    cz = O.compress(coords, m, g, x, fx["eb_abs"], False, fx["split"])
    assert cz.v.tolist() == e["resampled"]
    assert cz.grid.p.tolist() == e["p"]
    assert O.lorenzo(cz.grid.p, g).tolist() == e["lorenzo"]
    assert cz.grid.codes.tolist() == e["grid_codes"]
    assert cz.xhat.tolist() == e["xhat"]
    assert cz.gv.tolist() == e["back_interp"]
    assert cz.vert.codes.tolist() == e["vertex_codes"]
    xr = O.decompress(coords, g, cz.bound, cz.grid, cz.vert, np.float64)
    assert xr.tolist() == fx["field"]


@pytest.mark.parametrize("dim", [2, 3])
def test_bary_vertices_are_one_hot(dim):
    rng = np.random.default_rng(10 + dim)
    for _ in range(200):
        verts = rng.random((dim + 1, dim)).astype(np.float32)
        for k in range(dim + 1):
            inside, lam, nd = O.bary(verts, verts[k])
            if exact_bary(verts, verts[k]) is None:
                continue
            # exact at vertex a (q = 0); at the others FP32 rounding of the
            # zero numerators may leave a tiny negative coordinate
            assert inside or (dim == 3 and k > 0)
            expect = np.zeros(dim + 1, np.float32)
            expect[k] = 1.0
            if not nd and (dim == 2 or k == 0):
                # q = 0 (vertex a), or in 2-D every numerator is the
                # determinant's own expression or an exact cancellation
                assert lam.tolist() == expect.tolist(), (verts, k, lam)
            else:
                np.testing.assert_allclose(lam, expect, atol=2e-5)


@pytest.mark.parametrize("dim", [2, 3])
def test_bary_against_exact_rationals(dim):
    rng = np.random.default_rng(20 + dim)
    n_nd = 0
    for it in range(400):
        verts = rng.random((dim + 1, dim)).astype(np.float32)
        if it % 4 == 0:
            # a sliver: the last vertex nearly on the face of the others
            w = rng.random(dim)
            w /= w.sum()
            verts[dim] = (w[:, None] * verts[:dim]).sum(0) + rng.normal(0, 1e-5, dim)
            verts = verts.astype(np.float32)
        y = (rng.random(dim) * 1.2 - 0.1).astype(np.float32)
        ex = exact_bary(verts, y)
        inside, lam, nd = O.bary(verts, y)
        if ex is None:
            assert not inside
            continue
        exf = np.array([float(v) for v in ex])
        n_nd += nd
        if nd:
            # FP64 recompute, then rounded: within a few FP32 ulps
            ulp = np.spacing(np.abs(exf).astype(np.float32)).astype(np.float64)
            assert np.all(np.abs(lam - exf) <= 2 * ulp + 1e-12 * np.abs(exf).max()), (lam, exf)
            m = min(ex)
            if abs(float(m) + 2 ** -20) > 1e-9 * max(1.0, float(max(map(abs, ex)))):
                assert inside == (m >= Fraction(-1, 2 ** 20))
        else:
            # FP32 path: |det| > 2^-10 L^dim bounds the conditioning
            assert np.all(np.abs(lam - exf) <= 1e-3 * max(1.0, np.abs(exf).max())), (lam, exf)
            m = float(min(ex))
            if abs(m + 2 ** -20) > 1e-3:
                assert inside == (m >= -2 ** -20)
    assert n_nd > 20


def test_bary_zero_area_never_contains():
    verts = np.array([[0, 0], [1, 1], [2, 2]], np.float32)   # collinear
    for y in ([1, 1], [0.5, 0.5], [0, 0], [3, 3], [1, 0]):
        inside, _, nd = O.bary(verts, np.array(y, np.float32))
        assert nd and not inside
    tet = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 1, 0]], np.float32)   # flat
    inside, _, nd = O.bary(tet, np.array([0.5, 0.5, 0], np.float32))
    assert nd and not inside


def _meshes_2d():
    rng = np.random.default_rng(7)
    out = []
    m = G.delaunay_2d(G.stratified_points_2d(24, rng, drop=10))
    out.append(("delaunay", m, (29, 23)))
    out.append(("aligned", G.structured_tri_mesh(5, 5), (9, 9)))
    # hole: drop the cells whose centroid is within 0.25 of the centre
    s = G.structured_tri_mesh(12, 12, rng, 0.2)
    cen = s.coords[:, s.cells].mean(axis=1)
    keep = np.hypot(cen[0] - 0.5, cen[1] - 0.5) > 0.25
    out.append(("hole", G.Mesh(s.coords, np.ascontiguousarray(s.cells[:, keep])), (17, 15)))
    # degenerate cells prepended (low ids): a repeated vertex, a collinear
    # triple and a sliver over real nodes
    a = G.structured_tri_mesh(6, 6, rng, 0.15)
    coords = np.concatenate([a.coords, np.array([[0.1, 0.5, 0.9, 0.2, 0.6, 0.6],
                                                 [0.1, 0.5, 0.9, 0.5, 0.5, 0.5 + 1e-6]],
                                                np.float32)], axis=1)
    nv = a.n_vertices
    bad = np.array([[nv, nv, nv + 1], [nv, nv + 1, nv + 2], [nv + 3, nv + 4, nv + 5]], np.int32).T
    cells = np.ascontiguousarray(np.concatenate([bad, a.cells], axis=1))
    out.append(("degenerate", G.Mesh(coords, cells), (11, 11)))
    return out


@pytest.mark.parametrize("case", range(4))
def test_locate_raster_equals_brute_2d(case):
    name, mesh, dims = _meshes_2d()[case]
    g = O.grid_from_dims(mesh.coords, dims)
    mb = O.locate(mesh.coords, mesh.cells, g, "brute", fill=None)
    mr = O.locate(mesh.coords, mesh.cells, g, "raster", fill=None)
    assert np.array_equal(mb.cell, mr.cell), name
    assert np.array_equal(mb.vid, mr.vid), name
    assert np.array_equal(mb.w.view(np.uint32), mr.w.view(np.uint32)), name


@pytest.mark.parametrize("jitter,dims", [(0.2, (9, 8, 7)), (0.0, (7, 7, 7))])
def test_locate_raster_equals_brute_3d(jitter, dims):
    mesh = G.kuhn_tet_mesh(5, 11, jitter=jitter)
    g = O.grid_from_dims(mesh.coords, dims)
    mb = O.locate(mesh.coords, mesh.cells, g, "brute", fill=None)
    mr = O.locate(mesh.coords, mesh.cells, g, "raster", fill=None)
    assert np.array_equal(mb.cell, mr.cell)
    assert np.array_equal(mb.w.view(np.uint32), mr.w.view(np.uint32))
    if jitter == 0.0:
        assert mb.n_unresolved == 0      # the unjittered lattice covers its bbox


def test_locate_chosen_cell_contains_node_exactly():
    name, mesh, dims = _meshes_2d()[0]
    g = O.grid_from_dims(mesh.coords, dims)
    m = O.locate(mesh.coords, mesh.cells, g, "brute", fill=None)
    ys = O.grid_nodes(g)
    for j in range(g.count):
        c = m.cell[j]
        if c < 0:
            continue
        verts = mesh.coords[:, mesh.cells[:, c]].T
        ex = exact_bary(verts, ys[:2, j])
        assert float(min(ex)) >= -2 ** -20 - 1e-5
        # every lower-id cell misses the node by exact arithmetic (up to the
        # tolerance band)
        for c2 in range(c):
            ex2 = exact_bary(mesh.coords[:, mesh.cells[:, c2]].T, ys[:2, j])
            assert ex2 is None or float(min(ex2)) < -2 ** -20 + 1e-5


def test_locate_matches_convex_hull():
    """On a Delaunay mesh the located nodes are the nodes inside the convex
    hull of the points (independent Qhull computation)."""
    from scipy.spatial import ConvexHull
    rng = np.random.default_rng(3)
    mesh = G.delaunay_2d(G.stratified_points_2d(40, rng))
    g = O.grid_from_dims(mesh.coords, (37, 41))
    m = O.locate(mesh.coords, mesh.cells, g, "raster", fill=None)
    hull = ConvexHull(mesh.coords.T.astype(np.float64))
    ys = O.grid_nodes(g)[:2].T.astype(np.float64)
    sd = (hull.equations[:, :2] @ ys.T + hull.equations[:, 2:3]).max(axis=0)
    assert np.all(m.cell[sd < -1e-6] >= 0)
    assert np.all(m.cell[sd > 1e-6] < 0)


def test_fill_nearest_bruteforce():
    rng = np.random.default_rng(5)
    mesh = G.delaunay_2d(G.stratified_points_2d(15, rng))
    g = O.grid_from_dims(mesh.coords, (21, 21))
    m = O.locate(mesh.coords, mesh.cells, g, "raster", fill="nearest")
    ys = O.grid_nodes(g)
    cnt = 0
    for j in np.nonzero(m.cell < 0)[0]:
        d = ((mesh.coords[0].astype(np.float64) - ys[0, j]) ** 2
             + (mesh.coords[1].astype(np.float64) - ys[1, j]) ** 2)
        k = m.vid[0, j]
        assert d[k] <= d.min() * (1 + 1e-5) + 1e-12
        assert m.w[:, j].tolist() == [1.0, 0.0, 0.0]
        cnt += 1
    assert cnt > 0
    mm = O.locate(mesh.coords, mesh.cells, g, "raster", fill="midrange")
    assert np.all(mm.vid[:, mm.cell < 0] == -1)


@pytest.mark.parametrize("dim", [2, 3])
def test_affine_field_reproduced(dim):
    """Linear elements reproduce affine fields: |v - f(y)| within a few FP32
    roundings of the magnitudes involved."""
    rng = np.random.default_rng(30 + dim)
    if dim == 2:
        mesh = G.delaunay_2d(G.stratified_points_2d(30, rng))
        dims = (25, 27)
    else:
        mesh = G.kuhn_tet_mesh(6, 4)
        dims = (9, 10, 11)
    alpha = 0.7
    beta = rng.normal(size=dim)
    x = alpha + beta @ mesh.coords.astype(np.float64)
    g = O.grid_from_dims(mesh.coords, dims)
    m = O.locate(mesh.coords, mesh.cells, g, "raster", fill=None)
    v = O.resample(m, x.astype(np.float32), 0.0)
    ys = O.grid_nodes(g)[:dim].astype(np.float64)
    f = alpha + beta @ ys
    sel = m.cell >= 0
    scale = abs(alpha) + (np.abs(beta)[:, None] * np.abs(ys)).sum(0) + np.abs(x).max()
    assert np.all(np.abs(v[sel] - f[sel]) <= 16 * 2.0 ** -24 * scale[sel])
    # weights: sum to one, none below the inside tolerance
    s = m.w[:, sel].astype(np.float64).sum(0)
    assert np.all(np.abs(s - 1) <= 4e-7)
    assert np.all(m.w[:, sel] >= -2 ** -20)


def test_grid_from_dims():
    coords = np.array([[0.25, 2.25, 1.0], [-1.0, 3.0, 0.0]], np.float32)
    g = O.grid_from_dims(coords, (9, 5))
    assert list(g.o)[:2] == [0.25, -1.0]
    assert list(g.h)[:2] == [0.25, 1.0]
    assert g.dims() == (9, 5, 1)


def test_locate_nodes_equals_brute_with_all_cells():
    """The restricted locator with every cell as candidate is the brute-force
    definition (2-D Delaunay with a ragged hull, nearest fill)."""
    rng = np.random.default_rng(21)
    mesh = G.delaunay_2d(G.stratified_points_2d(24, rng, drop=10))
    g = O.grid_from_dims(mesh.coords, (17, 15))
    ref = O.locate(mesh.coords, mesh.cells, g, "brute")
    nodes = np.arange(g.count)
    cand = np.tile(np.arange(mesh.n_cells, dtype=np.int32), (nodes.size, 1))
    got = O.locate_nodes(mesh.coords, mesh.cells, g, nodes, cand)
    assert np.array_equal(got.cell, ref.cell)
    assert np.array_equal(got.vid, ref.vid)
    assert np.array_equal(got.w.view(np.uint32), ref.w.view(np.uint32))


def test_kuhn_candidates_are_complete():
    """For a jittered Kuhn lattice the 27-cube candidate sets give exactly the
    brute-force location of every node (so they may stand in for a full scan
    on meshes too large to scan)."""
    from kuhn_cells import kuhn_candidates
    n = 9
    mesh = G.kuhn_tet_mesh(n, 4)
    g = O.grid_from_dims(mesh.coords, (11, 10, 12))
    ref = O.locate(mesh.coords, mesh.cells, g, "brute")
    nodes = np.arange(g.count)
    pts = np.stack([O.grid_node(g, j) for j in nodes], axis=1)
    got = O.locate_nodes(mesh.coords, mesh.cells, g, nodes, kuhn_candidates(pts, n))
    assert np.array_equal(got.cell, ref.cell)
    assert np.array_equal(got.vid, ref.vid)
    assert np.array_equal(got.w.view(np.uint32), ref.w.view(np.uint32))
    assert ref.n_unresolved > 0          # the ragged hull leaves nodes to the fill


@pytest.mark.parametrize("dim", [2, 3])
def test_near_degenerate_cells_located_with_fp64_weights(dim):
    """Slivers with the lowest cell ids lie across grid rows / planes: the
    nodes inside them are located there (brute force = bin raster), each
    chosen sliver meets the near-degenerate trigger, and the stored weights
    are the exact rational barycentric coordinates rounded once to FP32
    (within one FP32 ulp plus 2^-40), which the FP64 recompute delivers."""
    mesh, dims, _ = G.sliver_mesh(dim)
    ns = mesh.info["n_slivers"]
    g = O.grid_from_dims(mesh.coords, dims)
    mb = O.locate(mesh.coords, mesh.cells, g, "brute", fill=None)
    mr = O.locate(mesh.coords, mesh.cells, g, "raster", fill=None)
    assert np.array_equal(mb.cell, mr.cell)
    assert np.array_equal(mb.w.view(np.uint32), mr.w.view(np.uint32))
    sel = np.nonzero((mb.cell >= 0) & (mb.cell < ns))[0]
    assert sel.size >= 40
    assert set(mb.cell[sel].tolist()) == set(range(ns))
    for j in sel:
        c = mb.cell[j]
        verts = mesh.coords[:, mesh.cells[:, c]].T
        y = O.grid_node(g, j)[:dim]
        inside, lam, nd = O.bary(verts, y)
        assert nd and inside
        ex = exact_bary(verts, y)
        for k in range(dim + 1):
            e = float(ex[k])
            ulp = np.spacing(np.float32(abs(e))).astype(np.float64)
            assert abs(float(mb.w[k, j]) - e) <= ulp + 2.0 ** -40, (j, k)


@pytest.mark.parametrize("dim", [2, 3])
def test_fill_kdtree_equals_brute(dim):
    """The k-d tree candidate fill gives the brute-force nearest-vertex fill
    (FP32 metric, lowest id on ties) on meshes with ragged hulls, including
    a lattice where many vertices tie (unjittered, grid nodes equidistant
    from several vertices)."""
    rng = np.random.default_rng(40 + dim)
    cases = []
    if dim == 2:
        cases.append((G.delaunay_2d(G.stratified_points_2d(30, rng, drop=40)), (37, 33)))
        s = G.structured_tri_mesh(9, 9)
        cen = s.coords[:, s.cells].mean(axis=1)
        keep = np.hypot(cen[0] - 0.5, cen[1] - 0.5) > 0.3
        cases.append((G.Mesh(s.coords, np.ascontiguousarray(s.cells[:, keep])), (17, 17)))
    else:
        cases.append((G.kuhn_tet_mesh(7, 3), (13, 12, 11)))
        s = G.kuhn_tet_mesh(6, 4, jitter=0.0)        # a hole: drop the central cubes' tets
        cen = s.coords[:, s.cells].mean(axis=1)
        keep = np.abs(cen - 0.5).max(axis=0) > 0.25
        cases.append((G.Mesh(s.coords, np.ascontiguousarray(s.cells[:, keep])), (11, 11, 11)))
    for mesh, dims in cases:
        g = O.grid_from_dims(mesh.coords, dims)
        a = O.locate(mesh.coords, mesh.cells, g, "raster", fill="nearest")
        b = O.locate(mesh.coords, mesh.cells, g, "raster", fill="nearest", fill_method="kdtree")
        assert a.n_unresolved > 0
        assert np.array_equal(a.cell, b.cell)
        assert np.array_equal(a.vid, b.vid)
        assert np.array_equal(a.w.view(np.uint32), b.w.view(np.uint32))
