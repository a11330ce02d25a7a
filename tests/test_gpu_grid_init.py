"""GPU parity of the grid initialisation (Alg. 1): the radix-selected
percentile spacing, the dims, the origin and the final k per axis equal the
oracle's (sort-based) exactly, for 2-D and 3-D meshes, percentiles from 0 to
100 and G_max values that make the loop raise k; invalid cells are rejected."""
import numpy as np
import pytest

import meshgen as G
import oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2501_06910_amd import mc as M  # noqa: E402


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _meshes():
    rng = np.random.default_rng(4)
    return {
        "aligned2d": G.aligned_tri_mesh(41, 31),
        "delaunay2d": G.delaunay_2d(G.stratified_points_2d(60, rng)),
        "kuhn3d": G.kuhn_tet_mesh(24, 3),
        "small2d": G.config_small_2d()[0],
    }


MESHES = _meshes()
CASES = [("aligned2d", 10.0, 10_000), ("aligned2d", 50.0, 10_000), ("delaunay2d", 1.0, 20), ("delaunay2d", 30.0, 1 << 40),
         ("kuhn3d", 0.0, 1 << 40), ("kuhn3d", 5.0, 30), ("kuhn3d", 37.5, 1 << 40), ("kuhn3d", 100.0, 1 << 40),
         ("small2d", 10.0, 128)]


@pytest.mark.parametrize("name,k,g_max", CASES)
def test_grid_init_matches_oracle(name, k, g_max):
    mesh = MESHES[name]
    print(f"[grid_init] {name} nv={mesh.n_vertices} nc={mesh.n_cells} k={k} g_max={g_max}", flush=True)
    og, oku = O.grid_init(mesh.coords, mesh.cells, k, g_max)
    g, ku = M.grid_from_percentile(dev(mesh.coords), dev(mesh.cells), k, g_max)
    for d in range(3):
        assert g.dims[d] == og.n[d], d
        assert g.origin[d] == og.o[d], d
        assert g.spacing[d] == og.h[d], d
        assert ku[d] == oku[d], d
    print(f"[grid_init] dims {[g.dims[d] for d in range(3)]} k {ku}")


def test_grid_init_rejects_bad_cells():
    mesh = MESHES["kuhn3d"]
    cells = mesh.cells.copy()
    cells[2, 5] = mesh.n_vertices
    with pytest.raises(M.McError) as e:
        M.grid_from_percentile(dev(mesh.coords), dev(cells), 50.0, 100)
    assert e.value.status == M.ERR_ARG
