"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs, element by element.  Mapping ids and weights, grid and
vertex codes, outlier lists and decoded values must be bit-exact; every
vertex must be within tau2 <= tau (Sec. III of the paper)."""
import numpy as np
import pytest

import meshgen as G
import oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2501_06910_amd import mc as M  # noqa: E402

R = O.RADIUS


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


class Case:
    def __init__(self, name, mesh, x, dims, eb, rel, split, fill="nearest", mode="sum"):
        self.name, self.mesh, self.x, self.dims = name, mesh, x, dims
        self.eb, self.rel, self.split, self.fill, self.mode = eb, rel, split, fill, mode
        print(f"[case] {name}: nv={mesh.n_vertices} nc={mesh.n_cells} dims={dims} eb={eb} "
              f"rel={rel} split={split} ({mode}) dtype={x.dtype} fill={fill}", flush=True)
        self.og = O.grid_from_dims(mesh.coords, dims)
        self.om = O.locate(mesh.coords, mesh.cells, self.og, "raster", fill=fill)
        self.dc = dev(mesh.coords)
        self.dcells = dev(mesh.cells)
        self.dx = dev(x)
        self.plan = M.Plan(self.dc, self.dcells, dims=dims, fill=fill)

    def oracle_compress(self):
        return O.compress(self.mesh.coords, self.om, self.og, self.x, self.eb, self.rel, self.split,
                          mode=O.SPLIT_FULL if self.mode == "full" else O.SPLIT_SUM)

    def gpu_compress(self, **kw):
        codes = M.compress(self.plan, self.dx, self.eb, "rel" if self.rel else "abs", self.split, debug=True,
                           split_mode=self.mode, **kw)
        torch.cuda.synchronize()
        return codes


def _cases():
    out = []
    mesh, f, cfg = G.config_small_2d()
    out.append(("small2d", mesh, f, (128, 128), cfg["eb"], False, 0.5, "nearest"))
    rng = np.random.default_rng(12)
    m2 = G.structured_tri_mesh(301, 257, rng, 0.2)
    out.append(("struct2d_f32_ragged", m2, G.field_octaves(m2.coords, rng), (190, 171), 1e-5, True, 0.3, "midrange"))
    # 2-D rows of 12 and 16 segments of 256 columns (one workgroup per chunk
    # of rows, the last segment ragged in the first) and of 17 (the
    # row-segment decoder with its separate pass of segment sums)
    f2 = G.field_octaves(m2.coords, np.random.default_rng(13))
    out.append(("struct2d_f32_3000cols", m2, f2, (3000, 11), 1e-5, True, 0.5, "nearest"))
    out.append(("struct2d_f32_4096cols", m2, f2, (4096, 9), 1e-6, True, 0.5, "nearest"))
    out.append(("struct2d_f32_4300cols", m2, f2, (4300, 10), 1e-5, True, 0.5, "nearest"))
    m3 = G.kuhn_tet_mesh(22, 5)
    out.append(("kuhn3d_f32", m3, G.field_octaves(m3.coords, np.random.default_rng(1)), (25, 23, 21), 1e-4, True,
                0.5, "nearest"))
    m4 = G.kuhn_tet_mesh(17, 6)
    x4 = G.field_octaves(m4.coords, np.random.default_rng(2), dtype=np.float64)
    out.append(("kuhn3d_f64_tiny_eb", m4, x4, (20, 19, 18), 1e-7, True, 0.9, "midrange"))
    # x extent a multiple of 4 above 256 (two 256-column segments in the 3-D
    # decode), ragged y and z chunks, grid outliers at eb 1e-6
    m6 = G.kuhn_tet_mesh(30, 8)
    out.append(("kuhn3d_wide_f32", m6, G.field_octaves(m6.coords, np.random.default_rng(3)), (264, 21, 13), 1e-6,
                True, 0.5, "nearest"))
    # rows that end in a partial quad (two segments, grid outliers), and an
    # x extent above the quad decoder's 1024 (the generic decoder)
    out.append(("kuhn3d_ragged_quads_f32", m6, G.field_octaves(m6.coords, np.random.default_rng(5)), (263, 21, 13),
                1e-6, True, 0.5, "nearest"))
    out.append(("kuhn3d_long_x_f32", m6, G.field_octaves(m6.coords, np.random.default_rng(6)), (1030, 6, 5), 1e-5,
                True, 0.5, "nearest"))
    # three 256-column segments (the decode's four-segment instance, one idle)
    out.append(("kuhn3d_wider_f32", m6, G.field_octaves(m6.coords, np.random.default_rng(4)), (516, 11, 10), 1e-5,
                True, 0.5, "nearest"))
    mesh5, f5, _ = G.config_large_2d(h0=0.004, dims=200)
    out.append(("refined2d_f64", mesh5, f5, (200, 200), 1e-6, True, 0.5, "nearest"))
    # the full split: tau2 = tau, grid step from tau1 = split * tau (up to 16 tau)
    out.append(("small2d_full", mesh, f, (64, 64), cfg["eb"], False, 2.0, "nearest", "full"))
    out.append(("kuhn3d_f32_full", m3, G.field_octaves(m3.coords, np.random.default_rng(1)), (12, 12, 11), 1e-4,
                True, 16.0, "midrange", "full"))
    out.append(("kuhn3d_f64_full_tiny", m4, x4, (20, 19, 18), 1e-7, True, 0.25, "nearest", "full"))
    # slivers with the lowest ids over grid rows / planes: nodes whose
    # weights come from the FP64 recompute of near-degenerate cells
    for dim in (2, 3):
        ms, ds, fs = G.sliver_mesh(dim, 11)
        out.append((f"sliver{dim}d_f32", ms, fs, ds, 1e-5, True, 0.5, "nearest"))
        out.append((f"sliver{dim}d_f64", ms, fs.astype(np.float64), ds, 1e-6, True, 0.5, "midrange"))
    return out


CASES = _cases()


@pytest.fixture(scope="module", params=range(len(CASES)), ids=[c[0] for c in CASES])
def case(request):
    return Case(*CASES[request.param])


def test_grid_matches(case):
    g = case.plan.grid
    for d in range(3):
        assert g.dims[d] == case.og.n[d]
        assert g.origin[d] == case.og.o[d]
        assert g.spacing[d] == case.og.h[d]


def test_plan_mapping_bitexact(case):
    vid, w, cell = case.plan.mapping()
    info = case.plan.info()
    assert info["n_unresolved"] == case.om.n_unresolved
    assert np.array_equal(cell.cpu().numpy(), case.om.cell)
    assert np.array_equal(vid.cpu().numpy(), case.om.vid)
    assert np.array_equal(w.cpu().numpy().view(np.uint32), case.om.w.view(np.uint32))


def test_near_degenerate_count(case):
    """The plan's count of nodes whose weights came from the FP64 recompute
    equals the number of nodes whose chosen cell meets the near-degenerate
    trigger (each checked with the oracle's barycentric routine); the sliver
    meshes have such nodes."""
    info = case.plan.info()
    cells = case.mesh.cells
    coords = case.mesh.coords
    dim = case.mesh.dim
    nd_cells = {}
    expect = 0
    for c in case.om.cell[case.om.cell >= 0].tolist():
        if c not in nd_cells:
            verts = coords[:, cells[:, c]].T
            nd_cells[c] = O.bary(verts, verts[0])[2]
        expect += int(nd_cells[c])
    assert info["n_near_degenerate"] == expect
    if case.name.startswith("sliver"):
        assert expect >= 40


def test_compress_bitexact(case):
    oc = case.oracle_compress()
    codes = case.gpu_compress()
    h = codes.host()
    r = h["result"]
    assert r["status"] == 0
    for k in ("tau", "tau1", "tau2", "c", "xmin", "xmax"):
        assert r[k] == getattr(oc.bound, k), k
    assert np.array_equal(codes.dbg_resampled.cpu().numpy().view(np.uint32), oc.v.view(np.uint32))
    assert np.array_equal(codes.dbg_grid_p.cpu().numpy(), oc.grid.p)
    assert np.array_equal(h["grid_codes"], oc.grid.codes)
    assert np.array_equal(h["g_out_idx"], oc.grid.out_idx)
    assert np.array_equal(h["g_out_delta"], oc.grid.out_delta)
    assert np.array_equal(codes.dbg_vertex_g.cpu().numpy().view(np.uint32), oc.gv.view(np.uint32))
    assert np.array_equal(h["vert_codes"], oc.vert.codes)
    assert np.array_equal(h["v_out_idx"], oc.vert.out_idx)
    assert np.array_equal(h["v_out_val"], oc.vert.out_val)
    print(f"[case] {case.name}: grid outliers {oc.grid.out_idx.size}, vertex outliers {oc.vert.out_idx.size}")


def test_roundtrip_bound_and_parity(case):
    oc = case.oracle_compress()
    codes = case.gpu_compress()
    xr = M.decompress(case.plan, codes)
    torch.cuda.synchronize()
    xg = xr.cpu().numpy()
    xo = O.decompress(case.mesh.coords, case.og, oc.bound, oc.grid, oc.vert, case.x.dtype)
    assert np.array_equal(xg.view(np.uint8), xo.view(np.uint8))
    assert np.all(np.abs(case.x.astype(np.float64) - xg.astype(np.float64)) <= oc.bound.tau2)


def test_deterministic(case):
    a = case.gpu_compress().host()
    b = case.gpu_compress().host()
    for k in ("grid_codes", "g_out_idx", "vert_codes", "v_out_idx"):
        assert np.array_equal(a[k], b[k])


def test_error_statuses():
    mesh, f, cfg = G.config_small_2d()
    dc, dcells = dev(mesh.coords), dev(mesh.cells)
    plan = M.Plan(dc, dcells, dims=(64, 64))
    # non-finite field
    bad = f.copy()
    bad[17] = np.nan
    c = M.compress(plan, dev(bad), 1e-3, "rel", 0.5)
    assert c.result_host()["status"] == M.ERR_ARG
    # relative bound of a constant field: tau = 0
    c = M.compress(plan, dev(np.full_like(f, 2.0)), 1e-3, "rel", 0.5)
    assert c.result_host()["status"] == M.ERR_ARG
    # bound too small for the data range
    c = M.compress(plan, dev(f), 1e-10, "rel", 0.5)
    assert c.result_host()["status"] == M.ERR_RANGE
    # capacity: counts stay exact
    full = M.compress(plan, dev(f), 1e-7, "rel", 0.5).result_host()
    assert full["status"] == 0 and full["n_vertex_outliers"] > 4
    small = M.Codes(plan, torch.float64, g_cap=1, v_cap=2)
    M.compress(plan, dev(f), 1e-7, "rel", 0.5, codes=small)
    r = small.result_host()
    assert r["status"] == M.ERR_CAPACITY
    assert r["n_vertex_outliers"] == full["n_vertex_outliers"]
    assert r["n_grid_outliers"] == full["n_grid_outliers"]


def test_host_validation_errors():
    mesh, f, cfg = G.config_small_2d()
    dc, dcells = dev(mesh.coords), dev(mesh.cells)
    bad_cells = mesh.cells.copy()
    bad_cells[1, 5] = mesh.n_vertices + 3
    with pytest.raises(M.McError) as e:
        M.Plan(dc, dev(bad_cells), dims=(32, 32))
    assert e.value.status == M.ERR_ARG
    plan = M.Plan(dc, dcells, dims=(32, 32))
    for kw in (dict(eb=0.0), dict(eb=-1.0), dict(grid_share=0.0), dict(grid_share=1.0)):
        args = dict(eb=1e-3, grid_share=0.5)
        args.update(kw)
        with pytest.raises(M.McError) as e:
            M.compress(plan, dev(f), args["eb"], "rel", args["grid_share"])
        assert e.value.status == M.ERR_ARG


def test_golden_two_triangles_gpu():
    import json, os
    fx = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "two_triangles.json")))
    coords = np.array(fx["coords"], np.float32)
    cells = np.array(fx["cells"], np.int32)
    x = np.array(fx["field"], np.float64)
    plan = M.Plan(dev(coords), dev(cells), dims=fx["dims"])
    vid, w, cell = plan.mapping()
    e = fx["expect"]
    assert cell.cpu().tolist() == e["cell_of_node"]
    assert vid.cpu().tolist() == e["vid"]
    assert w.cpu().tolist() == e["w"]
    codes = M.compress(plan, dev(x), fx["eb_abs"], "abs", fx["split"], debug=True)
    h = codes.host()
    assert h["grid_codes"].tolist() == e["grid_codes"]
    assert h["vert_codes"].tolist() == e["vertex_codes"]
    assert codes.dbg_resampled.cpu().tolist() == e["resampled"]
    assert M.decompress(plan, codes).cpu().tolist() == fx["field"]
