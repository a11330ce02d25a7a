"""GPU parity of the multilevel interpolation grid predictor (linear and
cubic rules on the prequantised grid; an alternative grid compressor C(x1),
Sec. II and Sec. IV-D): grid codes, grid outlier lists, vertex codes and
decoded values bit for bit against the oracle, for both operator pairs and
both residual coders, on grids decoded wholly in the coarse workgroup and
grids with fine class launches, ragged extents, and tiny error bounds that
force grid outliers (looked up by the decoder).  At the benchmark's full
size (256^3 grid): the codes against the oracle's coding of the same
prequantised grid, and the reconstruction equal to the Lorenzo path's."""
import numpy as np
import pytest

import meshgen as G
import oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2501_06910_amd import mc as M  # noqa: E402

GP = {"linear": O.GPRED_LINEAR, "cubic": O.GPRED_CUBIC}


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _cases():
    out = []
    mesh, f, cfg = G.config_small_2d()
    out.append(("small2d_f64_coarse_only", mesh, f, (64, 64), cfg["eb"], False, 0.5))      # 4096 nodes: one workgroup
    m3 = G.kuhn_tet_mesh(22, 5)
    out.append(("kuhn3d_f32", m3, G.field_octaves(m3.coords, np.random.default_rng(1)), (40, 37, 33), 1e-4, True, 0.5))
    rng = np.random.default_rng(12)
    m2 = G.structured_tri_mesh(601, 499, rng, 0.2)
    out.append(("struct2d_f32", m2, G.field_octaves(m2.coords, rng), (150, 120), 1e-5, True, 0.5))
    out.append(("struct2d_f32_thin", m2, G.field_octaves(m2.coords, rng), (3000, 3), 1e-4, True, 0.5))
    m4 = G.kuhn_tet_mesh(17, 6)
    x4 = G.field_octaves(m4.coords, np.random.default_rng(2), dtype=np.float64)
    out.append(("kuhn3d_f64_tiny_eb", m4, x4, (20, 19, 18), 1e-7, True, 0.9))              # grid outliers
    out.append(("kuhn3d_f64_tiny_eb_fine", m4, x4, (65, 33, 17), 1e-7, True, 0.9))
    return out


CASES = _cases()


def check_grid(h, oc):
    assert h["result"]["status"] == 0
    assert np.array_equal(h["grid_codes"], oc.grid.codes)
    assert np.array_equal(h["g_out_idx"], oc.grid.out_idx)
    assert np.array_equal(h["g_out_delta"], oc.grid.out_delta)
    assert np.array_equal(h["vert_codes"], oc.vert.codes)
    assert np.array_equal(h["v_out_idx"], oc.vert.out_idx)
    assert np.array_equal(h["v_out_val"].view(np.uint8), oc.vert.out_val.view(np.uint8))


@pytest.mark.parametrize("gpred", ["linear", "cubic"])
@pytest.mark.parametrize("name,mesh,x,dims,eb,rel,split", CASES, ids=[c[0] for c in CASES])
def test_interp_linear_pair(name, mesh, x, dims, eb, rel, split, gpred):
    print(f"[interp] {name} {gpred}: nv={mesh.n_vertices} dims={dims} eb={eb} dtype={x.dtype}", flush=True)
    og = O.grid_from_dims(mesh.coords, dims)
    om = O.locate(mesh.coords, mesh.cells, og)
    oc = O.compress(mesh.coords, om, og, x, eb, rel, split, gpred=GP[gpred])
    plan = M.Plan(dev(mesh.coords), dev(mesh.cells), dims=dims)
    xt = dev(x)
    codes = M.Codes(plan, xt.dtype, grid_predictor=gpred)
    M.compress(plan, xt, eb, "rel" if rel else "abs", split, codes=codes)
    out = M.decompress(plan, codes)
    torch.cuda.synchronize()
    h = codes.host()
    check_grid(h, oc)
    xo = O.decompress(mesh.coords, og, oc.bound, oc.grid, oc.vert, x.dtype, gpred=GP[gpred])
    xg = out.cpu().numpy()
    assert np.array_equal(xg.view(np.uint8), xo.view(np.uint8))
    assert np.all(np.abs(x.astype(np.float64) - xg.astype(np.float64)) <= oc.bound.tau2)
    print(f"[interp] {name} {gpred}: grid outliers {oc.grid.out_idx.size}")


@pytest.mark.parametrize("gpred", ["linear", "cubic"])
@pytest.mark.parametrize("name,mesh,x,dims,eb,rel,split", CASES[1:4], ids=[c[0] for c in CASES[1:4]])
def test_interp_cluster_pair_open(name, mesh, x, dims, eb, rel, split, gpred):
    """The paper's pair (nearest-node g, cluster-mean f), open loop."""
    print(f"[interp] cluster {name} {gpred}", flush=True)
    og = O.grid_from_dims(mesh.coords, dims)
    oc = O.compress_cluster(mesh.coords, og, x, eb, rel, split, True, gpred=GP[gpred])
    plan = M.Plan(dev(mesh.coords), None, dims=dims, operators="cluster")
    xt = dev(x)
    codes = M.Codes(plan, xt.dtype, grid_predictor=gpred)
    M.compress(plan, xt, eb, "rel" if rel else "abs", split, codes=codes, residual="open")
    out = M.decompress(plan, codes)
    torch.cuda.synchronize()
    check_grid(codes.host(), oc)
    xo = O.decompress_cluster(mesh.coords, og, oc.bound, oc.grid, oc.vert, x.dtype, gpred=GP[gpred])
    assert np.array_equal(out.cpu().numpy().view(np.uint8), xo.view(np.uint8))


def test_interp_with_delta_residual():
    """Cubic grid codes together with the delta residual coder, full split."""
    m3 = G.kuhn_tet_mesh(22, 5)
    x = G.field_octaves(m3.coords, np.random.default_rng(3))
    dims = (30, 29, 27)
    og = O.grid_from_dims(m3.coords, dims)
    om = O.locate(m3.coords, m3.cells, og)
    oc = O.compress(m3.coords, om, og, x, 1e-4, True, 4.0, mode=O.SPLIT_FULL, delta=True, gpred=O.GPRED_CUBIC)
    plan = M.Plan(dev(m3.coords), dev(m3.cells), dims=dims)
    xt = dev(x)
    codes = M.Codes(plan, xt.dtype, residual_predictor="delta", grid_predictor="cubic")
    M.compress(plan, xt, 1e-4, "rel", 4.0, codes=codes, split_mode="full")
    out = M.decompress(plan, codes)
    torch.cuda.synchronize()
    check_grid(codes.host(), oc)
    xo = O.decompress(m3.coords, og, oc.bound, oc.grid, oc.vert, x.dtype, delta=True, gpred=O.GPRED_CUBIC)
    assert np.array_equal(out.cpu().numpy().view(np.uint8), xo.view(np.uint8))


def test_interp_repeat_and_switch():
    """One plan, calls in a row with the predictors alternating: every call
    decodes to the same field (the predictor only changes the grid codes)."""
    m3 = G.kuhn_tet_mesh(22, 5)
    x = dev(G.field_octaves(m3.coords, np.random.default_rng(5)))
    plan = M.Plan(dev(m3.coords), dev(m3.cells), dims=(33, 31, 29))
    ref = None
    for gp in ("lorenzo", "cubic", "linear", "cubic", "lorenzo"):
        codes = M.Codes(plan, x.dtype, grid_predictor=gp)
        M.compress(plan, x, 1e-4, codes=codes)
        out = M.decompress(plan, codes).cpu().numpy()
        if ref is None:
            ref = out
        assert np.array_equal(out.view(np.uint8), ref.view(np.uint8)), gp


def test_interp_full_size():
    """256^3 grid of the 16M-vertex workload, cubic: the GPU's grid codes
    and outliers equal the oracle's coding of the GPU's prequantised grid
    (p itself is pinned against the oracle on sampled nodes by the
    full-size parity test), and the reconstruction equals the Lorenzo
    path's bit for bit."""
    mesh, f, cfg = G.config_tet_3d()
    print(f"[interp] full size nv={mesh.n_vertices} dims={cfg['dims']}", flush=True)
    x = torch.from_numpy(f).cuda()
    plan = M.Plan(torch.from_numpy(mesh.coords).cuda(), torch.from_numpy(mesh.cells).cuda(), dims=cfg["dims"])
    lz = M.compress(plan, x, cfg["eb"], "rel", cfg["split"])
    ref = M.decompress(plan, lz).cpu().numpy()
    codes = M.Codes(plan, x.dtype, debug=True, grid_predictor="cubic")
    M.compress(plan, x, cfg["eb"], "rel", cfg["split"], codes=codes)
    out = M.decompress(plan, codes).cpu().numpy()
    torch.cuda.synchronize()
    h = codes.host()
    assert h["result"]["status"] == 0
    p = codes.dbg_grid_p.cpu().numpy()
    g = O.grid_from_dims(mesh.coords, cfg["dims"])
    oc = O.grid_codes(p, g, O.GPRED_CUBIC)
    assert np.array_equal(h["grid_codes"], oc.codes)
    assert np.array_equal(h["g_out_idx"], oc.out_idx)
    assert np.array_equal(h["g_out_delta"], oc.out_delta)
    assert np.array_equal(out.view(np.uint8), ref.view(np.uint8))
    print(f"[interp] full size: grid outliers {oc.out_idx.size}")


@pytest.mark.parametrize("dims", [(2, 2, 2), (3, 2, 2), (2, 2, 65), (8192, 2, 2), (2, 3, 1000)])
@pytest.mark.parametrize("gpred", ["linear", "cubic", "temporal"])
def test_extreme_grid_shapes(dims, gpred):
    """Smallest grids (only the coarse workgroup), the widest x extent and
    long thin grids along y and z (many fine launches of few nodes)."""
    mesh = G.kuhn_tet_mesh(9, 4)
    x = G.field_octaves(mesh.coords, np.random.default_rng(8))
    print(f"[interp] extreme {dims} {gpred}", flush=True)
    og = O.grid_from_dims(mesh.coords, dims)
    om = O.locate(mesh.coords, mesh.cells, og)
    ref = None
    if gpred == "temporal":
        ref = O.compress(mesh.coords, om, og, (x * np.float32(0.99)).astype(np.float32), 1e-4, True, 0.5).xhat
    gp = {"linear": O.GPRED_LINEAR, "cubic": O.GPRED_CUBIC, "temporal": O.GPRED_TEMPORAL}[gpred]
    oc = O.compress(mesh.coords, om, og, x, 1e-4, True, 0.5, gpred=gp, gref=ref)
    plan = M.Plan(dev(mesh.coords), dev(mesh.cells), dims=dims)
    xt = dev(x)
    kw = {} if ref is None else dict(grid_ref=dev(ref))
    codes = M.Codes(plan, xt.dtype, grid_predictor=gpred, **kw)
    M.compress(plan, xt, 1e-4, "rel", 0.5, codes=codes)
    out = M.decompress(plan, codes)
    torch.cuda.synchronize()
    check_grid(codes.host(), oc)
    xo = O.decompress(mesh.coords, og, oc.bound, oc.grid, oc.vert, x.dtype, gpred=gp, gref=ref)
    assert np.array_equal(out.cpu().numpy().view(np.uint8), xo.view(np.uint8))


def test_unknown_grid_predictor_rejected():
    mesh = G.kuhn_tet_mesh(9, 2)
    x = dev(G.field_octaves(mesh.coords, np.random.default_rng(6)))
    plan = M.Plan(dev(mesh.coords), dev(mesh.cells), dims=(8, 8, 8))
    codes = M.Codes(plan, x.dtype)
    codes.struct.grid_predictor = 7
    with pytest.raises(M.McError) as e:
        M.compress(plan, x, 1e-3, codes=codes)
    assert e.value.status == M.ERR_ARG
