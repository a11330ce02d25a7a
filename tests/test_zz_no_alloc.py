"""The allocation-free compress entry point (mc_serial_compress_noalloc)
against the context-based one (mc_serial_compress) it mirrors: codes,
outlier lists and result headers equal, on two calls in a row (the second
on a smaller input, so stale scratch contents from the first call would
show), for both value types, then the limit check."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2501_06910_amd import mc as M  # noqa: E402


def _field(n, dtype, seed):
    rng = np.random.default_rng(seed)
    t = np.linspace(0.0, 40.0, n)
    x = np.sin(t) + 0.01 * rng.normal(size=n)
    spikes = rng.choice(n, max(1, n // 5000), replace=False)
    x[spikes] += rng.choice([-3.0, 3.0], spikes.size)         # raw outliers of the 1-D predictor
    return torch.from_numpy(x.astype(dtype)).cuda()


def _equal(a, b):
    ha, hb = a.host(), b.host()
    for k in ("status", "n_vertex_outliers", "tau", "tau1", "c", "xmin", "xmax"):
        assert ha["result"][k] == hb["result"][k], k
    assert ha["result"]["status"] == 0
    assert np.array_equal(ha["codes"], hb["codes"])
    assert np.array_equal(ha["out_idx"], hb["out_idx"])
    assert np.array_equal(ha["out_val"].view(np.uint8), hb["out_val"].view(np.uint8))
    return ha["result"]["n_vertex_outliers"]


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_noalloc_matches_context_two_calls(dtype):
    sizes = (3_000_017, 123_457)          # second call smaller; both ragged against the 1024-value tiles
    ctx = M.Serial(max(sizes))
    for i, n in enumerate(sizes):
        x = _field(n, dtype, 10 + i)
        print(f"[noalloc] {np.dtype(dtype).name} call {i}: n={n}", flush=True)
        # eb 1e-6 of the range: a jump of half the range is 2.5e5 steps, beyond R,
        # so the spikes become raw outliers
        ref = M.serial_compress(ctx, x, 1e-6, "rel")
        got = M.serial_compress_noalloc(x, 1e-6, "rel")
        torch.cuda.synchronize()
        k = _equal(got, ref)
        assert k > 0
        # decoding the allocation-free codes gives the context's values
        xo = M.serial_decompress(ctx, got)
        xr = M.serial_decompress(ctx, ref)
        torch.cuda.synchronize()
        assert torch.equal(xo, xr)
    ctx.destroy()


def test_noalloc_limit():
    """Above the limit the call fails on the host with MC_ERR_CAPACITY and
    enqueues nothing; the limit is the header's."""
    assert M.serial_noalloc_max() == 1 << 28
    x = torch.zeros(16, dtype=torch.float32, device="cuda")
    codes = M.SerialCodes(16, torch.float32)
    st = M.lib().mc_serial_compress_noalloc(M._ptr(x), 0, (1 << 28) + 1, 1e-3, 0, M.C.byref(codes.struct),
                                            M._stream())
    assert st == 3
    assert "no-allocation limit" in M.lib().mc_last_error().decode()
