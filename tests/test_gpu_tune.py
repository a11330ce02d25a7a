"""GPU tests of the launch autotuner: every knob setting gives the same
codes, outliers and decoded values (the knobs reorder tiles, pick cache
policies and launch shapes), and
mc_plan_tune picks a valid mask, restores the profiler state, and leaves
the results unchanged."""
import numpy as np
import pytest

import meshgen as G

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2501_06910_amd import mc as M  # noqa: E402


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _run(plan, x, eb):
    codes = M.compress(plan, x, eb, "rel", 0.5)
    out = M.decompress(plan, codes)
    torch.cuda.synchronize()
    h = codes.host()
    return h, out.cpu().numpy()


@pytest.mark.parametrize("dim", [2, 3])
def test_knobs_do_not_change_results(dim):
    if dim == 2:
        mesh = G.structured_tri_mesh(200, 180, np.random.default_rng(1), 0.2)
        dims = (150, 140)
    else:
        mesh = G.kuhn_tet_mesh(30, 2)
        dims = (32, 28, 36)          # x a multiple of 4: the quad decode kernels
    x = dev(G.field_octaves(mesh.coords, np.random.default_rng(4)))
    plan = M.Plan(dev(mesh.coords), dev(mesh.cells), dims=dims)
    assert plan.remap_mask == 0x1EC
    ref_h, ref_x = _run(plan, x, 1e-5)
    rng = np.random.default_rng(0)
    # bits 9-10: vertex decode 2 / 8 / 4 vertices per thread; 11-12: 1024 / 512 / 2048 range blocks
    for mask in ([0, 0x7F, 0x1FF, 0x55, 0x12A, 0x180, 0x3EC, 0x5EC, 0x7EC, 0x9EC, 0x11EC, 0x1FFF, 0xA00]
                 + [int(m) for m in rng.integers(0, 0x2000, 4)]):
        plan.remap_mask = mask
        h, xo = _run(plan, x, 1e-5)
        assert h["result"] == ref_h["result"], mask
        for k in ("grid_codes", "vert_codes", "g_out_idx", "g_out_delta", "v_out_idx"):
            assert np.array_equal(h[k], ref_h[k]), (mask, k)
        assert np.array_equal(xo.view(np.uint8), ref_x.view(np.uint8)), mask
    with pytest.raises(RuntimeError):
        plan.remap_mask = 0x2000


def test_tune_picks_a_mask_and_keeps_results():
    mesh = G.kuhn_tet_mesh(40, 3)
    x = dev(G.field_octaves(mesh.coords, np.random.default_rng(5)))
    plan = M.Plan(dev(mesh.coords), dev(mesh.cells), dims=(44, 40, 40))
    ref_h, ref_x = _run(plan, x, 1e-4)
    M.profile_enable(True)
    mask = plan.tune(x, 1e-4, reps=3)
    M.profile_reset()
    M.compress(plan, x, 1e-4, "rel", 0.5)
    torch.cuda.synchronize()
    assert "k_resample" in M.profile_read()      # profiling was left on
    M.profile_enable(False)
    assert 0 <= mask <= 0x1FFF and plan.remap_mask == mask
    print(f"[tune] chosen remap mask 0x{mask:02x}")
    h, xo = _run(plan, x, 1e-4)
    assert np.array_equal(h["vert_codes"], ref_h["vert_codes"])
    assert np.array_equal(h["grid_codes"], ref_h["grid_codes"])
    assert np.array_equal(xo.view(np.uint8), ref_x.view(np.uint8))


@pytest.mark.parametrize("dim", [2, 3])
def test_bin_tuning_keeps_the_mapping(dim):
    """The bin edge only speeds up point location: a plan built with the
    tuned edge, and plans built with each candidate edge, hold the same
    mapping bit for bit; the tuner reports a time for every candidate."""
    if dim == 2:
        mesh = G.delaunay_2d(G.stratified_points_2d(120, np.random.default_rng(3), drop=50))
        dims = (130, 117)
    else:
        mesh = G.kuhn_tet_mesh(24, 5)
        dims = (27, 25, 26)
    coords, cells = dev(mesh.coords), dev(mesh.cells)
    grid = M.grid_from_dims(coords, dims)
    best, rec = M.tune_bins(coords, cells, grid)
    assert best in M.BIN_CANDIDATES
    print(f"[bins D={dim}] chosen {best}: {rec}")
    maps = []
    for b in (best,) + M.BIN_CANDIDATES:
        plan = M.Plan(coords, cells, grid=grid, bin_nodes=b)
        assert plan.info()["bin_nodes"] == b
        vid, w, cell = plan.mapping()
        maps.append((vid.cpu().numpy(), w.cpu().numpy().view(np.uint32), cell.cpu().numpy()))
    for m in maps[1:]:
        for a, b in zip(maps[0], m):
            assert np.array_equal(a, b)
    auto = M.Plan(coords, cells, grid=grid, bin_nodes="auto")      # from the tuning cache now
    assert auto.info()["bin_nodes"] == best
