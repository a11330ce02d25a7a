"""Pins of the oracle's nearest-node g and cluster-mean f (Sec. IV-C/IV-D)
with the open-loop residual of Alg. 3: the nearest node equals brute force
over all nodes (points inside and outside the grid box); cluster sums are
exact for integer-valued fields and within a few ulps of the correctly
rounded sum (math.fsum) otherwise; the mean minimises the squared residual
of its cluster; a field constant on every cluster leaves only zero
residuals; every vertex stays within tau (open loop) or tau2 (closed loop);
codes equal the definition evaluated independently; and decoding inverts
coding."""
import math

import numpy as np
import pytest

import meshgen as G
import oracle as O

R = O.RADIUS


def brute_nearest(pts, g):
    nodes = O.grid_nodes(g).astype(np.float64)[: pts.shape[0]]   # [dim, ng]
    d = ((pts.astype(np.float64)[:, :, None] - nodes[:, None, :]) ** 2).sum(axis=0)
    return np.argmin(d, axis=1)


@pytest.mark.parametrize("dims", [(7, 5, 1), (5, 6, 4)])
def test_nearest_nodes_equal_brute_force(dims):
    dim = 2 if dims[2] == 1 else 3
    rng = np.random.default_rng(3)
    g = O.make_grid(dim, dims, (0.1, -0.2, 0.3), (0.25, 0.5, 0.125))
    ext = np.array([(dims[d] - 1) * g.h[d] for d in range(dim)])
    lo = np.array([g.o[d] for d in range(dim)])
    pts = (lo[:, None] - 0.2 * ext[:, None] + 1.4 * ext[:, None] * rng.random((dim, 600))).astype(np.float32)
    m = O.nearest_nodes(pts, g)
    assert np.array_equal(m, brute_nearest(pts, g))


def test_cluster_mean_exact_for_integer_field():
    rng = np.random.default_rng(4)
    ng, nv = 50, 4000
    m = rng.integers(0, ng - 5, nv).astype(np.int32)       # the last nodes stay unvisited
    x = rng.integers(-1000, 1000, nv).astype(np.float64)
    x1, cnt = O.cluster_mean(x, m, ng, 7.5)
    assert np.array_equal(cnt, np.bincount(m, minlength=ng))
    s = np.bincount(m, weights=x, minlength=ng)
    vis = cnt > 0
    assert np.array_equal(x1[vis], s[vis] / cnt[vis])
    assert np.all(x1[~vis] == 7.5)


def test_cluster_mean_near_correctly_rounded_and_least_squares():
    rng = np.random.default_rng(5)
    ng, nv = 40, 3000
    m = rng.integers(0, ng, nv).astype(np.int32)
    x = (rng.normal(size=nv) * 10.0 ** rng.integers(-6, 6, nv)).astype(np.float32)
    x1, cnt = O.cluster_mean(x, m, ng, 0.0)
    for j in range(ng):
        xs = x[m == j].astype(np.float64)
        exact = math.fsum(xs) / xs.size
        assert abs(x1[j] - exact) <= 1e-13 * max(np.abs(xs).sum() / xs.size, 1e-300)
        # the mean minimises the squared residual: the residuals sum to zero
        assert abs(math.fsum(xs - x1[j])) <= 1e-12 * float(np.abs(xs).sum())


def _mesh_field():
    mesh = G.kuhn_tet_mesh(9, 2)
    return mesh, G.field_octaves(mesh.coords, np.random.default_rng(6))


def test_constant_clusters_leave_zero_residuals():
    mesh, _ = _mesh_field()
    g = O.grid_from_dims(mesh.coords, (5, 4, 6))
    m = O.nearest_nodes(mesh.coords, g)
    rng = np.random.default_rng(8)
    phi = rng.normal(size=g.count).astype(np.float32)
    x = phi[m]                                             # the same value on every vertex of a cluster
    cz = O.compress_cluster(mesh.coords, g, x, 1e-3, True, 0.5)
    vis = cz.count > 0
    assert np.array_equal(cz.x1[vis], phi[vis].astype(np.float64))
    assert cz.vert.out_idx.size == 0 and np.all(cz.vert.codes == R)


@pytest.mark.parametrize("eb,split,open_loop,mode", [(1e-2, 0.5, True, O.SPLIT_SUM), (1e-4, 0.3, True, O.SPLIT_SUM),
                                                      (1e-6, 0.9, True, O.SPLIT_SUM),
                                                      (1e-4, 0.5, False, O.SPLIT_SUM),
                                                      (1e-4, 2.0, False, O.SPLIT_FULL)])
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_bound_codes_and_roundtrip(eb, split, open_loop, mode, dtype):
    mesh, f = _mesh_field()
    x = f.astype(dtype)
    g = O.grid_from_dims(mesh.coords, (5, 6, 4))
    cz = O.compress_cluster(mesh.coords, g, x, eb, True, split, open_loop, mode)
    b = cz.bound
    xr = O.decompress_cluster(mesh.coords, g, b, cz.grid, cz.vert, dtype)
    xd = x.astype(np.float64)
    assert np.all(np.abs(xd - xr) <= (b.tau if open_loop else b.tau2))
    # the definition, evaluated here independently
    xh = (b.c + cz.grid.p.astype(np.float64) * b.step1).astype(np.float32).astype(np.float64)
    ref = cz.x1 if open_loop else xh
    q = np.rint((xd - ref[cz.m]) * b.inv2)
    s = xh[cz.m] + q * b.step2
    xq = s if dtype == np.float64 else s.astype(np.float32).astype(np.float64)
    ok = (np.abs(q) <= R - 1) & (np.abs(xd - xq) <= (b.tau if open_loop else b.tau2))
    assert np.array_equal(cz.vert.codes, np.where(ok, q + R, 0).astype(np.uint16))
    assert np.array_equal(cz.vert.out_idx, np.nonzero(~ok)[0])
    assert np.array_equal(xr[ok], xq[ok].astype(dtype))
    assert np.array_equal(xr[~ok], x[~ok])
    # grid part: prequantised cluster means, Lorenzo-coded
    assert np.array_equal(cz.grid.p, np.rint((cz.x1 - b.c) * b.inv1).astype(np.int32))
    if eb == 1e-6:
        assert cz.vert.out_idx.size > 0 or cz.grid.out_idx.size > 0


@pytest.mark.parametrize("dims", [(40, 37, 33), (60, 58, 50), (12, 11, 10)])
def test_grid_coarsen_planes(dims):
    """Grid_Coarsen (Alg. 2): the kept planes of each axis are exactly those
    holding a vertex's nearest node (numpy's unique over the node
    coordinates, an independent count), in their original order; every
    vertex keeps its node's original coordinates."""
    mesh = G.kuhn_tet_mesh(22, 5)
    g = O.grid_from_dims(mesh.coords, dims)
    m = O.nearest_nodes(mesh.coords, g)
    keep, gc, mc = O.grid_coarsen(m, g)
    n = g.dims()
    coords = [m % n[0], (m // n[0]) % n[1], m // (n[0] * n[1])]
    off = [0, n[0], n[0] + n[1]]
    back = []
    for d in range(3):
        visited = np.unique(coords[d])
        k = keep[off[d]:off[d] + n[d]]
        expect = visited if visited.size >= 2 or n[d] < 2 else np.arange(n[d])
        assert np.array_equal(np.nonzero(k >= 0)[0], expect)
        assert np.array_equal(k[k >= 0], np.arange(expect.size))
        assert gc.dims()[d] == expect.size
        back.append(np.nonzero(k >= 0)[0])
    nc = gc.dims()
    cc = [mc % nc[0], (mc // nc[0]) % nc[1], mc // (nc[0] * nc[1])]
    for d in range(3):
        assert np.array_equal(back[d][cc[d]], coords[d])
    print(f"coarsened {dims} -> {nc}")


def test_grid_coarsen_keeps_every_value():
    """The dropped planes hold no vertex, so on the coarsened grid every
    cluster mean, vertex code and decoded value is the same as on the full
    grid (open and closed loop); only the grid codes shrink."""
    mesh = G.kuhn_tet_mesh(22, 5)
    x = G.field_octaves(mesh.coords, np.random.default_rng(3))
    g = O.grid_from_dims(mesh.coords, (60, 58, 50))     # finer than the vertex lattice: empty planes
    for open_loop in (True, False):
        full = O.compress_cluster(mesh.coords, g, x, 1e-4, True, 0.5, open_loop)
        co = O.compress_cluster(mesh.coords, g, x, 1e-4, True, 0.5, open_loop, coarsen=True)
        assert co.grid.codes.size < full.grid.codes.size
        assert np.array_equal(co.x1[co.m], full.x1[full.m])
        assert np.array_equal(co.vert.codes, full.vert.codes)
        a = O.decompress_cluster(mesh.coords, g, full.bound, full.grid, full.vert, x.dtype)
        b = O.decompress_cluster(mesh.coords, g, co.bound, co.grid, co.vert, x.dtype, coarsen=True)
        assert np.array_equal(a.view(np.uint8), b.view(np.uint8))
