"""Parity of the HIP 1-D serialisation baseline (the Sec. V-C comparison)
with the oracle: codes, outlier lists, result header and decoded values
bit for bit, on mesh fields in vertex order, random walks with spikes that
force raw outliers, ragged lengths around the tile size, both dtypes and
bound modes, the degenerate constant field, outlier capacity overflow, and
reuse of one context with a shorter second field."""
import numpy as np
import pytest

import meshgen as G
import oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2501_06910_amd import mc as M  # noqa: E402


def walk(n, seed, dtype, spikes=997):
    rng = np.random.default_rng(seed)
    x = np.cumsum(rng.normal(size=n)).astype(dtype)
    if spikes:
        x[::spikes] += dtype(500.0)
    return x


def check_parity(ctx, x, eb, relative, cap=None, misalign=False):
    if misalign:                                  # field pointer one element past a 256-byte boundary
        xt = torch.from_numpy(np.concatenate([x[:1], x])).cuda()[1:]
        assert xt.data_ptr() % 16 != 0
    else:
        xt = torch.from_numpy(x).cuda()
    print(f"[serial] n={x.size} dtype={x.dtype} eb={eb} rel={relative} cap={cap} misalign={misalign}", flush=True)
    codes = M.serial_compress(ctx, xt, eb, "rel" if relative else "abs", cap=cap)
    xr = M.serial_decompress(ctx, codes)
    torch.cuda.synchronize()
    h = codes.host()
    r = h["result"]
    oc, oi, ov, b = O.serial_compress(x, eb, relative)
    for k in ("tau", "c", "xmin", "xmax"):
        assert r[k] == getattr(b, k), k
    assert r["tau1"] == b.tau and r["tau2"] == 0.0
    assert r["n_vertex_outliers"] == oi.size and r["n_grid_outliers"] == 0
    assert np.array_equal(h["codes"], oc)
    if cap is not None and oi.size > cap:
        assert r["status"] == M.ERR_CAPACITY
        return r, oi.size
    assert r["status"] == 0
    assert np.array_equal(h["out_idx"], oi)
    assert np.array_equal(h["out_val"].view(np.uint8), ov.view(np.uint8))
    xo = O.serial_decompress(oc, oi, ov, b, x.dtype)
    got = xr.cpu().numpy()
    assert np.array_equal(got.view(np.uint8), xo.view(np.uint8))
    assert np.all(np.abs(got.astype(np.float64) - x.astype(np.float64)) <= b.tau)
    return r, oi.size


@pytest.fixture(scope="module")
def ctx():
    c = M.Serial(1 << 20)
    yield c
    c.destroy()


def test_mesh_field_vertex_order(ctx):
    mesh, f, cfg = G.config_small_2d()
    r, k = check_parity(ctx, f, cfg["eb"], False)
    print(f"[serial] small 2-D mesh field: {k} raw values")


def test_tet_field_vertex_order(ctx):
    mesh = G.kuhn_tet_mesh(30, 8)
    f = G.field_octaves(mesh.coords, np.random.default_rng(11))
    check_parity(ctx, f, 1e-4, True)


@pytest.mark.parametrize("dtype,eb,relative", [(np.float32, 1e-3, True), (np.float32, 1e-6, True),
                                               (np.float64, 1e-6, True), (np.float64, 0.05, False)])
def test_walk_with_spikes(ctx, dtype, eb, relative):
    r, k = check_parity(ctx, walk(300001, 5, dtype), eb, relative)
    if eb <= 1e-6:
        assert k >= 300001 // 997                 # spikes jump by more than R steps: raw


@pytest.mark.parametrize("n", [1, 2, 255, 1023, 1024, 1025, 4097, 16 * 1024 + 3])
def test_ragged_lengths(ctx, n):
    # one value has no range: an absolute bound then
    check_parity(ctx, walk(n, n, np.float32, spikes=7), 1e-3, n > 1)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_unaligned_field_pointer(ctx, dtype):
    check_parity(ctx, walk(70001, 31, dtype), 1e-6, True, misalign=True)


def test_constant_field_is_degenerate(ctx):
    x = np.full(5000, 2.5, np.float32)
    with pytest.raises(O.OracleError):
        O.serial_compress(x, 1e-3, True)          # tau = 0
    codes = M.serial_compress(ctx, torch.from_numpy(x).cuda(), 1e-3, "rel")
    torch.cuda.synchronize()
    assert codes.result_host()["status"] == M.ERR_ARG
    # with an absolute bound it is exact: one code per value, no outliers
    check_parity(ctx, x, 1e-3, False)


def test_capacity_overflow_counts_exact(ctx):
    r, k = check_parity(ctx, walk(100000, 9, np.float32), 1e-6, True, cap=5)
    assert k > 5 and r["n_vertex_outliers"] == k


def test_context_reuse_shorter_field(ctx):
    check_parity(ctx, walk(200000, 21, np.float64), 1e-5, True)
    check_parity(ctx, walk(3001, 22, np.float64), 1e-5, True)


def test_rejects_oversized_field():
    small = M.Serial(1000)
    x = torch.zeros(1001, dtype=torch.float32, device="cuda")
    with pytest.raises(M.McError):
        M.serial_compress(small, x, 1e-3, "rel")
    small.destroy()


def test_range_error_when_bound_too_small(ctx):
    x = walk(4096, 3, np.float64, spikes=0)
    with pytest.raises(O.OracleError):
        O.serial_compress(x, 1e-12, False)        # |x - c| / (2 tau) >= 2^27
    codes = M.serial_compress(ctx, torch.from_numpy(x).cuda(), 1e-12, "abs")
    torch.cuda.synchronize()
    assert codes.result_host()["status"] == M.ERR_RANGE
