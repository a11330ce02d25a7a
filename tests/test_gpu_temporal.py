"""GPU parity of the time-axis grid predictor (each node of the prequantised
grid predicted from a reference grid, normally the previous timestep's x1'):
grid codes, grid outlier lists, vertex codes, decoded values and the x1'
output bit for bit against the oracle, with the reference computed by the
oracle; both operator pairs; references that force outliers (a tiny bound,
non-finite values); a chained series whose x1' output feeds the next step's
reference through one buffer; and the argument check."""
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


def step_pair(mesh, x0, amp, rng):
    """The field at the next timestep: x0 plus a smooth change."""
    d = np.sin(mesh.coords[0].astype(np.float64) * 5.0 + rng.uniform(0, 6)) * amp
    return (x0.astype(np.float64) + d).astype(x0.dtype)


def _cases():
    out = []
    m3 = G.kuhn_tet_mesh(22, 5)
    x3 = G.field_octaves(m3.coords, np.random.default_rng(1))
    out.append(("kuhn3d_f32", m3, x3, (40, 37, 33), 1e-4, True, 0.5, 0.01, False))
    mesh, f, cfg = G.config_small_2d()
    out.append(("small2d_f64", mesh, f, (64, 64), cfg["eb"], False, 0.5, 0.02, False))
    m4 = G.kuhn_tet_mesh(17, 6)
    x4 = G.field_octaves(m4.coords, np.random.default_rng(2), dtype=np.float64)
    out.append(("kuhn3d_f64_tiny_eb", m4, x4, (20, 19, 18), 1e-7, True, 0.9, 0.05, False))     # grid outliers
    out.append(("kuhn3d_f32_nan_ref", m3, x3, (30, 29, 27), 1e-4, True, 0.5, 0.01, True))     # prediction 0
    return out


CASES = _cases()


@pytest.mark.parametrize("name,mesh,x0,dims,eb,rel,split,amp,nan_ref", CASES, ids=[c[0] for c in CASES])
def test_temporal_linear_pair(name, mesh, x0, dims, eb, rel, split, amp, nan_ref):
    print(f"[temporal] {name}: nv={mesh.n_vertices} dims={dims} eb={eb} dtype={x0.dtype}", flush=True)
    x1 = step_pair(mesh, x0, amp, np.random.default_rng(7))
    og = O.grid_from_dims(mesh.coords, dims)
    om = O.locate(mesh.coords, mesh.cells, og)
    ref = O.compress(mesh.coords, om, og, x0, eb, rel, split).xhat            # the oracle's x1' of step 0
    if nan_ref:
        ref = np.full_like(ref, np.nan)
    oc = O.compress(mesh.coords, om, og, x1, eb, rel, split, gpred=O.GPRED_TEMPORAL, gref=ref)
    plan = M.Plan(dev(mesh.coords), dev(mesh.cells), dims=dims)
    xt = dev(x1)
    xh = torch.empty(plan.n_grid, dtype=torch.float32, device="cuda")
    codes = M.Codes(plan, xt.dtype, grid_predictor="temporal", grid_ref=dev(ref), xhat_out=xh)
    M.compress(plan, xt, eb, "rel" if rel else "abs", split, codes=codes)
    torch.cuda.synchronize()
    assert np.array_equal(xh.cpu().numpy().view(np.uint32), oc.xhat.view(np.uint32))
    xh.zero_()
    out = M.decompress(plan, codes)
    torch.cuda.synchronize()
    assert np.array_equal(xh.cpu().numpy().view(np.uint32), oc.xhat.view(np.uint32))
    h = codes.host()
    assert h["result"]["status"] == 0
    assert np.array_equal(h["grid_codes"], oc.grid.codes)
    assert np.array_equal(h["g_out_idx"], oc.grid.out_idx)
    assert np.array_equal(h["g_out_delta"], oc.grid.out_delta)
    assert np.array_equal(h["vert_codes"], oc.vert.codes)
    xo = O.decompress(mesh.coords, og, oc.bound, oc.grid, oc.vert, x1.dtype, gpred=O.GPRED_TEMPORAL, gref=ref)
    assert np.array_equal(out.cpu().numpy().view(np.uint8), xo.view(np.uint8))
    print(f"[temporal] {name}: grid outliers {oc.grid.out_idx.size} of {og.count}")


def test_temporal_cluster_pair_open():
    m3 = G.kuhn_tet_mesh(22, 5)
    x0 = G.field_octaves(m3.coords, np.random.default_rng(3))
    x1 = step_pair(m3, x0, 0.01, np.random.default_rng(8))
    dims = (33, 31, 29)
    og = O.grid_from_dims(m3.coords, dims)
    ref = O.grid_recon(O.compress_cluster(m3.coords, og, x0, 1e-4, True, 0.5, True).grid.p,
                       O.bound(x0, 1e-4, True, 0.5))
    oc = O.compress_cluster(m3.coords, og, x1, 1e-4, True, 0.5, True, gpred=O.GPRED_TEMPORAL, gref=ref)
    plan = M.Plan(dev(m3.coords), None, dims=dims, operators="cluster")
    xt = dev(x1)
    codes = M.Codes(plan, xt.dtype, grid_predictor="temporal", grid_ref=dev(ref))
    M.compress(plan, xt, 1e-4, "rel", 0.5, codes=codes, residual="open")
    out = M.decompress(plan, codes)
    torch.cuda.synchronize()
    h = codes.host()
    assert h["result"]["status"] == 0
    assert np.array_equal(h["grid_codes"], oc.grid.codes)
    assert np.array_equal(h["vert_codes"], oc.vert.codes)
    xo = O.decompress_cluster(m3.coords, og, oc.bound, oc.grid, oc.vert, x1.dtype, gpred=O.GPRED_TEMPORAL, gref=ref)
    assert np.array_equal(out.cpu().numpy().view(np.uint8), xo.view(np.uint8))


def test_chained_series_one_buffer():
    """Four steps; each step's x1' output is the next step's reference, in
    the same buffer (written after its last read).  Every step decodes to
    the Lorenzo path's values."""
    m3 = G.kuhn_tet_mesh(22, 5)
    rng = np.random.default_rng(11)
    xs = [G.field_octaves(m3.coords, np.random.default_rng(12))]
    for _ in range(3):
        xs.append(step_pair(m3, xs[-1], 0.005, rng))
    plan = M.Plan(dev(m3.coords), dev(m3.cells), dims=(33, 31, 29))
    buf = torch.empty(plan.n_grid, dtype=torch.float32, device="cuda")
    lz = M.Codes(plan, torch.float32, xhat_out=buf)
    M.compress(plan, dev(xs[0]), 1e-4, codes=lz)                      # step 0: Lorenzo, x1' into buf
    tp = M.Codes(plan, torch.float32, grid_predictor="temporal", grid_ref=buf, xhat_out=buf)
    ref_codes = M.Codes(plan, torch.float32)
    for t in range(1, 4):
        x = dev(xs[t])
        prev = buf.clone()
        M.compress(plan, x, 1e-4, codes=tp)
        # buf now holds x1' of step t: decode with a copy of the codes against
        # the reference the step was coded with
        dec = M.Codes(plan, torch.float32, grid_predictor="temporal", grid_ref=prev)
        for k in ("grid_codes", "g_out_idx", "g_out_delta", "vert_codes", "v_out_idx", "v_out_val", "result"):
            getattr(dec, k).copy_(getattr(tp, k))
        y = M.decompress(plan, dec)
        M.compress(plan, x, 1e-4, codes=ref_codes)
        yr = M.decompress(plan, ref_codes)
        torch.cuda.synchronize()
        assert np.array_equal(y.cpu().numpy().view(np.uint8), yr.cpu().numpy().view(np.uint8)), t


def test_temporal_needs_reference():
    mesh = G.kuhn_tet_mesh(9, 2)
    x = dev(G.field_octaves(mesh.coords, np.random.default_rng(6)))
    plan = M.Plan(dev(mesh.coords), dev(mesh.cells), dims=(8, 8, 8))
    codes = M.Codes(plan, x.dtype, grid_predictor="temporal")
    with pytest.raises(M.McError) as e:
        M.compress(plan, x, 1e-3, codes=codes)
    assert e.value.status == M.ERR_ARG
    with pytest.raises(ValueError):
        M.Codes(plan, x.dtype, grid_predictor="temporal", grid_ref=torch.zeros(5, device="cuda"))
