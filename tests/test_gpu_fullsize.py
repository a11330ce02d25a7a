"""Parity at the benchmark's full size: the 16M-vertex tetrahedral workload
(252^3 jittered Kuhn lattice, 94.9M tets, 256^3 grid, float32, relative eb
1e-4, split 0.5) in the launch order bench.py times.

Properties checked everywhere: the error split equals the oracle's closed
form, every vertex is within tau2.

Whole arrays: the oracle locates every grid node (bin-raster location,
pinned against brute force by CPU tests; the nodes outside the mesh filled
through k-d tree candidate lists, pinned against the brute-force fill) and
compresses and decompresses the whole field; the plan's mapping, every
grid and vertex code, both outlier lists and every decoded value must
match bit for bit.

Sampled, independently of the raster: on a seeded sample of grid nodes and
of vertices (every vertex outlier included) the oracle computes the results
one by one: the nodes involved are located against the 27-cube candidate
sets of the lattice (pinned against brute-force location by a CPU test),
resampled, prequantised and Lorenzo coded; the vertices are
back-interpolated from those nodes, quantised and decoded."""
import numpy as np
import pytest

import meshgen as G
import oracle as O
from kuhn_cells import kuhn_candidates

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2501_06910_amd import mc as M  # noqa: E402

N_LATTICE = 252


@pytest.fixture(scope="module")
def run():
    mesh, f, cfg = G.config_tet_3d()
    print(f"[fullsize] nv={mesh.n_vertices} nc={mesh.n_cells} dims={cfg['dims']}", flush=True)
    x = torch.from_numpy(f).cuda()
    plan = M.Plan(torch.from_numpy(mesh.coords).cuda(), torch.from_numpy(mesh.cells).cuda(), dims=cfg["dims"])
    plan.tune(x, cfg["eb"], "rel", cfg["split"], cache=True)
    codes = M.compress(plan, x, cfg["eb"], "rel", cfg["split"])
    out = M.decompress(plan, codes)
    torch.cuda.synchronize()
    return mesh, f, cfg, plan, codes.host(), out.cpu().numpy()


def test_bound_everywhere(run):
    mesh, f, cfg, plan, h, xr = run
    r = h["result"]
    assert r["status"] == 0
    b = O.bound(f, cfg["eb"], True, cfg["split"])
    for k in ("tau", "tau1", "tau2", "c", "xmin", "xmax"):
        assert r[k] == getattr(b, k), k
    err = np.abs(f.astype(np.float64) - xr.astype(np.float64))
    print(f"[fullsize] max |x - x'| / tau2 = {err.max() / b.tau2:.6f}; outliers grid {r['n_grid_outliers']} "
          f"vertex {r['n_vertex_outliers']}")
    assert np.all(err <= b.tau2)


def test_full_parity(run):
    mesh, f, cfg, plan, h, xr = run
    g = O.grid_from_dims(mesh.coords, cfg["dims"])
    m = O.locate(mesh.coords, mesh.cells, g, "raster", fill="nearest", fill_method="kdtree")
    print(f"[fullsize] oracle located {g.count} nodes ({m.n_unresolved} filled)", flush=True)
    vid_g, w_g, cell_g = plan.mapping()
    assert np.array_equal(cell_g.cpu().numpy(), m.cell)
    assert np.array_equal(vid_g.cpu().numpy(), m.vid)
    assert np.array_equal(w_g.cpu().numpy().view(np.uint32), m.w.view(np.uint32))
    del vid_g, w_g, cell_g
    assert plan.info()["n_unresolved"] == m.n_unresolved
    oc = O.compress(mesh.coords, m, g, f, cfg["eb"], True, cfg["split"])
    assert np.array_equal(h["grid_codes"], oc.grid.codes)
    assert np.array_equal(h["g_out_idx"], oc.grid.out_idx)
    assert np.array_equal(h["g_out_delta"], oc.grid.out_delta)
    assert np.array_equal(h["vert_codes"], oc.vert.codes)
    assert np.array_equal(h["v_out_idx"], oc.vert.out_idx)
    assert np.array_equal(h["v_out_val"].view(np.uint32), oc.vert.out_val.view(np.uint32))
    xo = O.decompress(mesh.coords, g, oc.bound, oc.grid, oc.vert, f.dtype)
    assert np.array_equal(xr.view(np.uint32), xo.view(np.uint32))
    print(f"[fullsize] whole arrays equal: {g.count} grid codes ({oc.grid.out_idx.size} outliers), "
          f"{mesh.n_vertices} vertex codes ({oc.vert.out_idx.size} outliers), decoded values", flush=True)


def test_sampled_parity(run):
    mesh, f, cfg, plan, h, xr = run
    g = O.grid_from_dims(mesh.coords, cfg["dims"])
    n0, n1, n2 = g.dims()
    b = O.bound(f, cfg["eb"], True, cfg["split"])
    rng = np.random.default_rng(2024)
    gs = np.sort(rng.choice(g.count, 256, replace=False))
    vs = np.union1d(rng.choice(mesh.n_vertices, 256, replace=False), h["v_out_idx"])

    # nodes the samples depend on: Lorenzo neighbours of gs, cell corners of vs
    need = set()
    for j in gs:
        i0, i1, i2 = j % n0, (j // n0) % n1, j // (n0 * n1)
        for a in (0, 1):
            for bb in (0, 1):
                for c in (0, 1):
                    if i0 - a >= 0 and i1 - bb >= 0 and i2 - c >= 0:
                        need.add(int((i0 - a) + n0 * ((i1 - bb) + n1 * (i2 - c))))
    cv = np.ascontiguousarray(mesh.coords[:, vs])
    idx, _ = O.vertex_cells(cv, g)
    for i0, i1, i2 in idx:
        for a in (0, 1):
            for bb in (0, 1):
                for c in (0, 1):
                    need.add(int((i0 + a) + n0 * ((i1 + bb) + n1 * (i2 + c))))
    nodes = np.array(sorted(need), np.int64)
    pts = np.stack([O.grid_node(g, j) for j in nodes], axis=1)
    m = O.locate_nodes(mesh.coords, mesh.cells, g, nodes, kuhn_candidates(pts, N_LATTICE))
    print(f"[fullsize] {nodes.size} nodes located, {m.n_unresolved} filled from the nearest vertex", flush=True)

    # mapping of the sampled nodes
    vid_g, w_g, cell_g = plan.mapping()
    sel = torch.from_numpy(nodes).cuda()
    assert np.array_equal(cell_g[sel].cpu().numpy(), m.cell)
    assert np.array_equal(vid_g[:, sel].cpu().numpy(), m.vid)
    assert np.array_equal(w_g[:, sel].cpu().numpy().view(np.uint32), m.w.view(np.uint32))
    del vid_g, w_g, cell_g

    # resample + prequantise: the other nodes sit at the centre (p = 0)
    v_full = np.full(g.count, np.float32(b.c), np.float32)
    v_full[nodes] = O.resample(m, f, b.c)
    gc = O.grid_quantize(v_full, g, b)
    assert np.array_equal(h["grid_codes"][gs], gc.codes[gs])
    d = O.lorenzo(gc.p, g)
    for j in gs:
        if gc.codes[j] == 0:
            k = np.searchsorted(h["g_out_idx"], j)
            assert h["g_out_idx"][k] == j and h["g_out_delta"][k] == d[j]
    print(f"[fullsize] grid codes of {gs.size} nodes equal", flush=True)

    # back-interpolation, residual codes and decoded values of the sampled vertices
    xhat = O.grid_recon(gc.p, b)
    gv = O.back_interp(cv, g, xhat)
    vc = O.residual_quantize(np.ascontiguousarray(f[vs]), gv, b)
    assert np.array_equal(h["vert_codes"][vs], vc.codes)
    for k, i in enumerate(vc.out_idx):
        pos = np.searchsorted(h["v_out_idx"], vs[i])
        assert h["v_out_idx"][pos] == vs[i]
        assert h["v_out_val"][pos].view(np.uint32) == vc.out_val[k].view(np.uint32)
    xo = O.vertex_decode(vc, gv, b, f.dtype)
    assert np.array_equal(xr[vs].view(np.uint32), xo.view(np.uint32))
    print(f"[fullsize] codes and decoded values of {vs.size} vertices equal", flush=True)
