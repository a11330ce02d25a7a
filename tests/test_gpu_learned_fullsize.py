"""Learned-predictor parity at the benchmark's full size: the refined 2-D
mesh (about 4.0M vertices, Delaunay, float64 rotating tanh front), grid
2048^2, relative eb 1e-4, split 0.5, the network trained on the GPU on
t = 0 (2000 Adam steps of 8192 samples, as the benchmark trains it) and
applied to t = 1.

The oracle locates every grid node (bin raster, the nodes outside the mesh
filled through k-d tree candidate lists) and compresses t = 1.  Checked:
back-interpolated values and grid codes over every element; the network
inputs and the integer shifts on a seeded sample of 65,536 vertices
(inputs bit-exact, shifts equal to the oracle network's on >= 99.9 % of
them: the MFMA summation order differs from the oracle's); and, given the
GPU's shifts, every vertex code, every block flag, the outlier list and
every decoded value, bit for bit.  On the same mesh and grid, the large 2-D
configuration's own field on the plain path at eb 1e-4 and 1e-6: every
array bit for bit."""
import numpy as np
import pytest

import meshgen as G
import oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2501_06910_amd import mc as M  # noqa: E402


@pytest.fixture(scope="module")
def run():
    mesh, series, cfg = G.config_learned_series(steps=2)
    dims = cfg["dims"][:2]
    print(f"[learned-full] nv={mesh.n_vertices} nc={mesh.n_cells} dims={dims}", flush=True)
    plan = M.Plan(torch.from_numpy(mesh.coords).cuda(), torch.from_numpy(mesh.cells).cuda(), dims=dims)
    model = M.Model.train(plan, torch.from_numpy(series[0]).cuda(), eb=cfg["eb"], steps=2000, batch=8192, seed=4)
    x = series[1]
    codes = M.compress(plan, torch.from_numpy(x).cuda(), cfg["eb"], "rel", 0.5, model=model, debug=True)
    torch.cuda.synchronize()
    h = codes.host()
    plain = M.compress(plan, torch.from_numpy(x).cuda(), cfg["eb"], "rel", 0.5).host()
    xr = M.decompress(plan, codes, model=model).cpu().numpy()
    z = model.features(plan, codes)
    print("[learned-full] GPU compress, decompress and features done", flush=True)
    og = O.grid_from_dims(mesh.coords, dims)
    om = O.locate(mesh.coords, mesh.cells, og, "raster", fill="nearest", fill_method="kdtree")
    pc = O.compress(mesh.coords, om, og, x, cfg["eb"], True, 0.5)
    print(f"[learned-full] oracle compress done ({om.n_unresolved} nodes filled)", flush=True)
    return mesh, x, plan, model, codes, h, plain, xr, z, og, pc, om


def test_grid_and_back_interpolation(run):
    mesh, x, plan, model, codes, h, plain, xr, z, og, pc, om = run
    assert h["result"]["status"] == 0
    assert np.array_equal(h["grid_codes"], pc.grid.codes)
    assert np.array_equal(h["g_out_idx"], pc.grid.out_idx)
    assert np.array_equal(codes.dbg_vertex_g.cpu().numpy().view(np.uint32), pc.gv.view(np.uint32))
    # the plain codes of the same field equal the oracle's everywhere
    assert np.array_equal(plain["vert_codes"], pc.vert.codes)
    assert np.array_equal(plain["v_out_idx"], pc.vert.out_idx)


def test_inputs_and_shifts_sampled(run):
    mesh, x, plan, model, codes, h, plain, xr, z, og, pc, om = run
    params, kappa = model.params()
    vs = np.sort(np.random.default_rng(77).choice(mesh.n_vertices, 65536, replace=False))
    zo = O.mlp_features(np.ascontiguousarray(mesh.coords[:, vs]), og, pc.xhat, np.ascontiguousarray(pc.gv[vs]),
                        kappa)
    zg = z[torch.from_numpy(vs).cuda()].cpu().numpy()
    assert np.array_equal(zg.view(np.uint32), zo.view(np.uint32))
    rho_o, _ = O.mlp_forward(2, params, zo)
    rho_q = codes.rho_q.cpu().numpy()[vs]
    same = float(np.mean(O.rho_quantize(rho_o) == rho_q))
    print(f"[learned-full] shifts equal to the oracle network's on {100 * same:.3f} % of {vs.size} vertices")
    assert same >= 0.999


def test_codes_given_shifts_everywhere(run):
    mesh, x, plan, model, codes, h, plain, xr, z, og, pc, om = run
    rho_q = codes.rho_q.cpu().numpy()
    lc = O.learned_codes(x, pc.gv, pc.bound, rho_q)
    assert np.array_equal(h["vert_codes"], lc.codes)
    assert np.array_equal(h["block_flags"][: lc.block_flags.size], lc.block_flags)
    assert np.array_equal(h["v_out_idx"], lc.out_idx)
    assert np.array_equal(h["v_out_val"].view(np.uint64), lc.out_val.view(np.uint64))
    nl = int(sum(bin(int(w)).count("1") for w in lc.block_flags))
    assert h["result"]["n_learned_blocks"] == nl
    xo = O.vertex_decode(lc, pc.gv, pc.bound, x.dtype, rho_q)
    assert np.array_equal(xr.view(np.uint64), xo.view(np.uint64))
    assert np.all(np.abs(x - xr) <= pc.bound.tau2)
    print(f"[learned-full] {x.size} vertex codes, {lc.out_idx.size} outliers, {nl} of "
          f"{(x.size + 4095) // 4096} blocks learned: equal", flush=True)


def test_trained_network_gains(run):
    """What the trained network gains at this size: some blocks take the
    learned codes, and the vertex stream and its code entropy shrink."""
    mesh, x, plan, model, codes, h, plain, xr, z, og, pc, om = run
    hl = dict(h)
    hl["learned"] = True
    sp = M.stream_bytes(plain, 8)
    sl = M.stream_bytes(hl, 8)
    ep, el = M.entropy_bits(plain["vert_codes"]), M.entropy_bits(h["vert_codes"])
    print(f"[learned-full] vertex stream plain {sp['vert']} B ({ep:.4f} b/value), learned {sl['vert']} B "
          f"({el:.4f} b/value), {h['result']['n_learned_blocks']} blocks learned")
    assert h["result"]["n_learned_blocks"] > 0
    assert sl["vert"] + sl["vert_outliers"] < sp["vert"] + sp["vert_outliers"]
    assert el < ep


@pytest.mark.parametrize("eb", [1e-4, 1e-6])
def test_plain_large2d_field_everywhere(run, eb):
    """The large 2-D configuration's own field (tanh front plus Fourier
    noise, float64) on the same mesh and grid, plain path, relative eb 1e-4
    and 1e-6: every grid and vertex code, both outlier lists and every
    decoded value equal to the oracle's; every vertex within tau2."""
    mesh, x, plan, model, codes, h, plain, xr, z, og, pc, om = run
    f = G.field_large_2d(mesh.coords)
    xg = torch.from_numpy(f).cuda()
    c = M.compress(plan, xg, eb, "rel", 0.5)
    xd = M.decompress(plan, c).cpu().numpy()
    torch.cuda.synchronize()
    hg = c.host()
    assert hg["result"]["status"] == 0
    oc = O.compress(mesh.coords, om, og, f, eb, True, 0.5)
    for k in ("tau", "tau1", "tau2", "c"):
        assert hg["result"][k] == getattr(oc.bound, k), k
    assert np.array_equal(hg["grid_codes"], oc.grid.codes)
    assert np.array_equal(hg["g_out_idx"], oc.grid.out_idx)
    assert np.array_equal(hg["g_out_delta"], oc.grid.out_delta)
    assert np.array_equal(hg["vert_codes"], oc.vert.codes)
    assert np.array_equal(hg["v_out_idx"], oc.vert.out_idx)
    assert np.array_equal(hg["v_out_val"].view(np.uint64), oc.vert.out_val.view(np.uint64))
    xo = O.decompress(mesh.coords, og, oc.bound, oc.grid, oc.vert, f.dtype)
    assert np.array_equal(xd.view(np.uint64), xo.view(np.uint64))
    assert np.all(np.abs(f - xd) <= oc.bound.tau2)
    print(f"[large2d eb={eb:g}] whole arrays equal: grid outliers {oc.grid.out_idx.size}, vertex outliers "
          f"{oc.vert.out_idx.size}", flush=True)
