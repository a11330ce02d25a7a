"""Pins of the oracle's time-axis grid predictor (each node of the
prequantised grid predicted from a reference grid both sides hold, normally
the previous timestep's reconstructed grid): a reference equal to the
field's own reconstructed grid leaves every error 0; a reference shifted by
k quantisation steps leaves the errors -k; a non-finite or far reference
predicts 0, so the errors are p itself; decode inverts code; and the
pipeline's p, x1', vertex codes and reconstruction do not depend on the
grid predictor."""
import numpy as np
import pytest

import meshgen as G
import oracle as O


def setup_grid(seed=3, dims=(37, 29, 11), eb=1e-4):
    g = O.make_grid(3, dims, (0.0, 0.0, 0.0), (1.0, 1.0, 1.0))
    rng = np.random.default_rng(seed)
    v = (rng.standard_normal(g.count) * 3.0 + 40.0).astype(np.float32)
    b = O.bound(v, eb, True, 0.5)
    gc = O.grid_quantize(v, g, b)
    return g, b, gc.p


def recon_margin_ok(p, b):
    """x1' = (float)(c + p step1) is within a quarter step of c + p step1,
    so rint((x1' - c) / step1) = p exactly."""
    exact = b.c + p.astype(np.float64) * b.step1
    return np.all(np.abs(exact.astype(np.float32).astype(np.float64) - exact) < 0.25 * b.step1)


def test_own_reconstruction_gives_zero_errors():
    g, b, p = setup_grid()
    assert recon_margin_ok(p, b)
    ref = O.grid_recon(p, b)
    gc = O.grid_codes(p, g, O.GPRED_TEMPORAL, ref, b)
    assert np.all(gc.codes == O.RADIUS) and gc.out_idx.size == 0


def test_shifted_reference_gives_minus_k():
    g, b, p = setup_grid(5)
    k = np.random.default_rng(9).integers(-7, 8, g.count)
    shifted = (p + k).astype(np.int32)
    assert recon_margin_ok(shifted, b)
    ref = (b.c + shifted.astype(np.float64) * b.step1).astype(np.float32)
    gc = O.grid_codes(p, g, O.GPRED_TEMPORAL, ref, b)
    assert np.array_equal(gc.codes.astype(np.int64) - O.RADIUS, -k)


def test_nonfinite_or_far_reference_predicts_zero():
    g, b, p = setup_grid(6, eb=1e-6)          # |p| up to ~5e5: outliers
    ref = np.full(g.count, np.nan, np.float32)
    ref[::3] = np.float32(1e30)
    ref[1::3] = np.float32(-np.inf)
    gc = O.grid_codes(p, g, O.GPRED_TEMPORAL, ref, b)
    d = gc.codes.astype(np.int64) - O.RADIUS
    d[gc.out_idx] = gc.out_delta
    assert np.array_equal(d, p.astype(np.int64))
    assert gc.out_idx.size == int((np.abs(p) > O.RADIUS - 1).sum()) > 0
    q = O.grid_decode(gc.codes, gc.out_idx, gc.out_delta, g, O.GPRED_TEMPORAL, ref, b)
    assert np.array_equal(q, p)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_roundtrip_random_reference(seed):
    g, b, p = setup_grid(seed)
    rng = np.random.default_rng(seed + 10)
    ref = (b.c + (p + rng.integers(-50000, 50000, g.count)) * b.step1).astype(np.float32)
    gc = O.grid_codes(p, g, O.GPRED_TEMPORAL, ref, b)
    assert gc.out_idx.size > 0
    q = O.grid_decode(gc.codes, gc.out_idx, gc.out_delta, g, O.GPRED_TEMPORAL, ref, b)
    assert np.array_equal(q, p)


def test_pipeline_over_two_timesteps():
    """Step 1 coded against step 0's reconstructed grid: the same p, x1',
    vertex codes and reconstruction as with the Lorenzo predictor."""
    mesh = G.kuhn_tet_mesh(10, 3)
    rng = np.random.default_rng(4)
    x0 = G.field_octaves(mesh.coords, rng)
    x1 = (x0 + np.float32(0.01) * np.sin(mesh.coords[0] * 7.0).astype(np.float32)).astype(np.float32)
    g = O.grid_from_dims(mesh.coords, (12, 11, 9))
    m = O.locate(mesh.coords, mesh.cells, g)
    c0 = O.compress(mesh.coords, m, g, x0, 1e-4, True, 0.5)
    ref = c0.xhat
    lz = O.compress(mesh.coords, m, g, x1, 1e-4, True, 0.5)
    tp = O.compress(mesh.coords, m, g, x1, 1e-4, True, 0.5, gpred=O.GPRED_TEMPORAL, gref=ref)
    assert np.array_equal(tp.grid.p, lz.grid.p) and np.array_equal(tp.xhat, lz.xhat)
    assert np.array_equal(tp.vert.codes, lz.vert.codes)
    ya = O.decompress(mesh.coords, g, lz.bound, lz.grid, lz.vert, x1.dtype)
    yb = O.decompress(mesh.coords, g, tp.bound, tp.grid, tp.vert, x1.dtype, gpred=O.GPRED_TEMPORAL, gref=ref)
    assert np.array_equal(ya.view(np.uint8), yb.view(np.uint8))
