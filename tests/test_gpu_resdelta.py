"""GPU parity of the residual codes with the 1-D Lorenzo predictor along the
vertex order: codes, outlier lists and decoded values bit for bit against
the oracle, every vertex within tau2, on meshes of one to several hundred
tiles (carries across tiles), ragged tails, both dtypes, both splits, and
spikes that force raw restarts."""
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


def _cases():
    out = []
    mesh, f, cfg = G.config_small_2d()
    out.append(("small2d_f64", mesh, f, (64, 64), cfg["eb"], False, 0.5, "sum"))
    m3 = G.kuhn_tet_mesh(22, 5)
    out.append(("kuhn3d_f32_full", m3, G.field_octaves(m3.coords, np.random.default_rng(1)), (12, 11, 10), 1e-4, True,
                4.0, "full"))
    rng = np.random.default_rng(12)
    m2 = G.structured_tri_mesh(601, 499, rng, 0.2)
    x2 = G.field_octaves(m2.coords, rng)
    x2[::1013] += np.float32(3.0)                             # spikes: raw restarts
    out.append(("struct2d_f32_spikes", m2, x2, (150, 120), 1e-5, True, 0.5, "sum"))
    m4 = G.kuhn_tet_mesh(17, 6)
    x4 = G.field_octaves(m4.coords, np.random.default_rng(2), dtype=np.float64)
    out.append(("kuhn3d_f64_tiny_eb", m4, x4, (20, 19, 18), 1e-7, True, 0.9, "sum"))
    return out


CASES = _cases()


@pytest.mark.parametrize("name,mesh,x,dims,eb,rel,split,mode", CASES, ids=[c[0] for c in CASES])
def test_delta_codes_and_roundtrip(name, mesh, x, dims, eb, rel, split, mode):
    print(f"[resdelta] {name}: nv={mesh.n_vertices} dims={dims} eb={eb} split={split} ({mode}) dtype={x.dtype}",
          flush=True)
    og = O.grid_from_dims(mesh.coords, dims)
    om = O.locate(mesh.coords, mesh.cells, og)
    oc = O.compress(mesh.coords, om, og, x, eb, rel, split, mode=O.SPLIT_FULL if mode == "full" else O.SPLIT_SUM,
                    delta=True)
    plan = M.Plan(dev(mesh.coords), dev(mesh.cells), dims=dims)
    xt = dev(x)
    codes = M.Codes(plan, xt.dtype, residual_predictor="delta")
    M.compress(plan, xt, eb, "rel" if rel else "abs", split, codes=codes, split_mode=mode)
    out = M.decompress(plan, codes)
    torch.cuda.synchronize()
    h = codes.host()
    assert h["result"]["status"] == 0
    assert np.array_equal(h["grid_codes"], oc.grid.codes)
    assert np.array_equal(h["vert_codes"], oc.vert.codes)
    assert np.array_equal(h["v_out_idx"], oc.vert.out_idx)
    assert np.array_equal(h["v_out_val"].view(np.uint8), oc.vert.out_val.view(np.uint8))
    xo = O.decompress(mesh.coords, og, oc.bound, oc.grid, oc.vert, x.dtype, delta=True)
    xg = out.cpu().numpy()
    assert np.array_equal(xg.view(np.uint8), xo.view(np.uint8))
    assert np.all(np.abs(x.astype(np.float64) - xg.astype(np.float64)) <= oc.bound.tau2)
    print(f"[resdelta] {name}: {oc.vert.out_idx.size} raw vertices, {(plan.n_vertices + 1023) // 1024} tiles")


@pytest.mark.parametrize("name,mesh,x,dims,eb,rel,split,mode", CASES, ids=[c[0] for c in CASES])
def test_delta_codes_cluster_pair(name, mesh, x, dims, eb, rel, split, mode):
    """The paper's pair (nearest-node g, cluster-mean f), closed loop."""
    print(f"[resdelta] cluster {name}", flush=True)
    og = O.grid_from_dims(mesh.coords, dims)
    oc = O.compress_cluster(mesh.coords, og, x, eb, rel, split, False,
                            O.SPLIT_FULL if mode == "full" else O.SPLIT_SUM, delta=True)
    plan = M.Plan(dev(mesh.coords), None, dims=dims, operators="cluster")
    xt = dev(x)
    codes = M.Codes(plan, xt.dtype, residual_predictor="delta")
    M.compress(plan, xt, eb, "rel" if rel else "abs", split, codes=codes, split_mode=mode)
    out = M.decompress(plan, codes)
    torch.cuda.synchronize()
    h = codes.host()
    assert h["result"]["status"] == 0
    assert np.array_equal(h["grid_codes"], oc.grid.codes)
    assert np.array_equal(h["vert_codes"], oc.vert.codes)
    assert np.array_equal(h["v_out_idx"], oc.vert.out_idx)
    assert np.array_equal(h["v_out_val"].view(np.uint8), oc.vert.out_val.view(np.uint8))
    xo = O.decompress_cluster(mesh.coords, og, oc.bound, oc.grid, oc.vert, x.dtype, delta=True)
    xg = out.cpu().numpy()
    assert np.array_equal(xg.view(np.uint8), xo.view(np.uint8))
    assert np.all(np.abs(x.astype(np.float64) - xg.astype(np.float64)) <= oc.bound.tau2)


def test_delta_rejected_with_open_loop():
    mesh = G.kuhn_tet_mesh(9, 2)
    x = dev(G.field_octaves(mesh.coords, np.random.default_rng(6)))
    cl = M.Plan(dev(mesh.coords), None, dims=(8, 8, 8), operators="cluster")
    with pytest.raises(M.McError) as e:
        M.compress(cl, x, 1e-3, codes=M.Codes(cl, x.dtype, residual_predictor="delta"), residual="open")
    assert e.value.status == M.ERR_UNSUPPORTED
