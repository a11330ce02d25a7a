"""Streams written from GPU-compressed fields decode to the same bits: the
field is compressed on the GPU, its codes written to a stream on the host,
read back, uploaded and decompressed; the result must equal the
decompression of the original device codes, byte for byte (linear and
cluster operator pairs, both residual coders, the interpolation grid
predictor, plain and learned codes, FP32 and FP64)."""
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


def _roundtrip(plan, x, codes, model=None):
    torch.cuda.synchronize()
    ref = M.decompress(plan, codes, model=model)
    h = codes.host()
    h["learned"] = model is not None
    blob, sec = M.write_stream(h, model.export() if model is not None else None)
    c2, mblob = M.Codes.from_stream(plan, blob)
    m2 = M.Model.load(mblob) if mblob is not None else None
    out = M.decompress(plan, c2, model=m2)
    torch.cuda.synchronize()
    assert torch.equal(out.view(torch.uint8), ref.view(torch.uint8))
    tau2 = h["result"]["tau2"]
    assert (x.double() - out.double()).abs().max().item() <= tau2
    print(f"[stream] {x.numel()} values, {len(blob)} B ({x.numel() * x.element_size() / len(blob):.2f}x): "
          f"{ {k: v for k, v in sec.items() if v} }")
    return blob


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("variant", ["plain", "delta", "cubic", "cluster"])
def test_stream_decodes_to_the_same_bits(dtype, variant):
    mesh = G.kuhn_tet_mesh(20, 4)
    f = G.field_octaves(mesh.coords, np.random.default_rng(6), dtype=dtype)
    x = dev(f)
    ops = "cluster" if variant == "cluster" else "linear"
    plan = M.Plan(dev(mesh.coords), dev(mesh.cells), dims=(23, 22, 21), operators=ops)
    kw = {}
    if variant == "delta":
        kw["residual_predictor"] = "delta"
    if variant == "cubic":
        kw["grid_predictor"] = "cubic"
    codes = M.Codes(plan, x.dtype, **kw)
    eb = 1e-6 if variant == "plain" else 1e-4          # grid and vertex outliers at the tight bound
    M.compress(plan, x, eb, "rel", 0.5, codes=codes)
    blob = _roundtrip(plan, x, codes)
    h = codes.host()
    if variant == "plain":
        assert h["result"]["n_grid_outliers"] > 0 or h["result"]["n_vertex_outliers"] > 0


def test_stream_with_learned_codes_and_model():
    mesh, series, cfg = G.config_learned_series(h0=0.004, dims=200, steps=2)
    plan = M.Plan(dev(mesh.coords), dev(mesh.cells), dims=(200, 200))
    model = M.Model.train(plan, dev(series[0]), eb=1e-4, steps=100, batch=2048, seed=3)
    x = dev(series[1])
    codes = M.Codes(plan, x.dtype, learned=True)
    M.compress(plan, x, 1e-4, "rel", 0.5, model=model, codes=codes)
    _roundtrip(plan, x, codes, model)
