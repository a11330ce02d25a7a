"""Pins of the oracle's grid initialisation (Alg. 1): the per-axis spacing is
the nearest-rank percentile of the cells' edge extents (checked against
numpy's inverted-CDF percentile, the textbook nearest-rank definition); on
an aligned triangle mesh a third of the x extents are zero, so k <= 33
selects zero and the G_max loop stops at k = 34 with the mesh spacing
(closed form); the result satisfies (max - min) / spacing < G_max and the
previous k does not; dims follow the spacing form of the grid."""
import math

import numpy as np
import pytest

import meshgen as G
import oracle as O


def edge_extents(coords, cells, d):
    dim = coords.shape[0]
    pairs = [(0, 1), (0, 2), (1, 2)] if dim == 2 else [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]
    c = coords[d].astype(np.float32)
    return np.concatenate([np.abs(c[cells[a]] - c[cells[b]]) for a, b in pairs]).astype(np.float32)


def test_aligned_mesh_closed_form():
    nx, ny = 41, 31
    mesh = G.aligned_tri_mesh(nx, ny)
    g, ku = O.grid_init(mesh.coords, mesh.cells, 10.0, 10_000)
    h = np.float32(mesh.coords[0].max() - mesh.coords[0].min()) / np.float32(nx - 1)
    assert ku[0] == 34.0 and ku[1] == 34.0                  # ranks up to a third are zero extents
    s = edge_extents(mesh.coords, mesh.cells, 0)
    assert np.isclose(g.h[0], float(np.median(s[s > 0])), rtol=1e-6)
    assert g.n[0] == math.ceil((float(mesh.coords[0].max()) - float(mesh.coords[0].min())) / g.h[0]) + 1
    assert abs(g.h[0] - float(h)) <= 1e-6 * float(h)


@pytest.mark.parametrize("k", [0.0, 5.0, 30.0, 50.0, 97.5, 100.0])
def test_percentile_is_nearest_rank(k):
    mesh = G.kuhn_tet_mesh(8, 3)
    g, ku = O.grid_init(mesh.coords, mesh.cells, k, 1 << 40)
    for d in range(3):
        s = edge_extents(mesh.coords, mesh.cells, d)
        assert ku[d] == k
        want = np.percentile(s, k, method="inverted_cdf") if k > 0 else s.min()
        assert g.h[d] == float(want)
        lo, hi = float(mesh.coords[d].min()), float(mesh.coords[d].max())
        assert g.o[d] == lo and g.n[d] == max(2, math.ceil((hi - lo) / g.h[d]) + 1)


@pytest.mark.parametrize("g_max", [8, 20, 40])
def test_g_max_loop(g_max):
    rng = np.random.default_rng(4)
    mesh = G.delaunay_2d(G.stratified_points_2d(30, rng))
    g, ku = O.grid_init(mesh.coords, mesh.cells, 1.0, g_max)
    for d in range(2):
        ext = float(mesh.coords[d].max()) - float(mesh.coords[d].min())
        assert ext / g.h[d] < g_max
        if ku[d] > 1.0:
            s = np.sort(edge_extents(mesh.coords, mesh.cells, d))
            prev = s[max(1, math.ceil((ku[d] - 1) * s.size / 100)) - 1]
            assert not ext / float(prev) < g_max


def test_rejects_degenerate():
    mesh = G.aligned_tri_mesh(5, 5)
    flat = mesh.coords.copy()
    flat[1] = 0.5                                           # every vertex on one line: no y extent
    with pytest.raises(O.OracleError):
        O.grid_init(flat, mesh.cells, 50.0, 100)
    with pytest.raises(O.OracleError):
        O.grid_init(mesh.coords, mesh.cells, 50.0, 1)
