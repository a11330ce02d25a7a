"""Pins of the oracle's residual codes with the 1-D Lorenzo predictor along
the vertex order: a residual that is a ramp in quantisation steps codes to a
constant difference (closed form); without outliers the running sum of the
differences equals the plain quantiser's codes (two coders written apart);
spikes beyond R steps are stored raw and decoding restarts there; every
vertex ends within tau2, also through the full pipeline."""
import numpy as np
import pytest

import meshgen as G
import oracle as O

R = O.RADIUS


def _bound(tau):
    x = np.array([0.0, 1.0])
    return O.bound(x, tau, False, 0.5)                       # tau1 = tau2 = tau / 2


def test_ramp_codes_to_constant_difference():
    b = _bound(0.25)                                          # step2 = 0.25, exact in binary
    rng = np.random.default_rng(1)
    gv = rng.integers(-100, 100, 500).astype(np.float32)       # integers: x - g exact
    i = np.arange(500)
    x = gv.astype(np.float64) + (7 + 3 * i) * 0.25
    vc = O.residual_delta(x, gv, b)
    assert vc.out_idx.size == 0
    assert vc.codes[0] == R + 7
    assert np.all(vc.codes[1:] == R + 3)
    assert np.array_equal(O.vertex_decode_delta(vc, gv, b, np.float64), x)


def test_running_sum_equals_plain_codes():
    rng = np.random.default_rng(2)
    n = 5000
    gv = rng.normal(size=n).astype(np.float32)
    x = gv.astype(np.float64) + rng.normal(scale=0.01, size=n)
    b = _bound(1e-3)
    plain = O.residual_quantize(x, gv, b)
    delta = O.residual_delta(x, gv, b)
    assert plain.out_idx.size == 0 and delta.out_idx.size == 0
    q = np.cumsum(delta.codes.astype(np.int64) - R)
    assert np.array_equal(q, plain.codes.astype(np.int64) - R)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_spikes_stored_raw_and_restart(dtype):
    rng = np.random.default_rng(3)
    n = 4000
    gv = rng.normal(size=n).astype(np.float32)
    x = (gv.astype(np.float64) + rng.normal(scale=0.01, size=n)).astype(dtype)
    x[::97] += dtype(100.0)                                   # jumps of 5e4 steps (> R) up and down
    b = _bound(2e-3)
    vc = O.residual_delta(x, gv, b)
    assert vc.out_idx.size >= 2 * (n // 97) - 2
    xr = O.vertex_decode_delta(vc, gv, b, dtype)
    assert np.all(np.abs(x.astype(np.float64) - xr.astype(np.float64)) <= b.tau2)
    # the definition, evaluated here independently
    xd = x.astype(np.float64)
    q = np.rint((xd - gv.astype(np.float64)) * b.inv2).astype(np.int64)
    d = np.diff(np.concatenate([[0], q]))
    s = gv.astype(np.float64) + q * b.step2
    xq = s if dtype == np.float64 else s.astype(np.float32).astype(np.float64)
    ok = (np.abs(xd - xq) <= b.tau2) & (np.abs(d) <= R - 1)
    assert np.array_equal(vc.codes, np.where(ok, d + R, 0).astype(np.uint16))
    assert np.array_equal(vc.out_idx, np.nonzero(~ok)[0])
    assert np.array_equal(xr[ok].astype(np.float64), xq[ok]) and np.array_equal(xr[~ok], x[~ok])


@pytest.mark.parametrize("eb,split,mode", [(1e-3, 0.5, O.SPLIT_SUM), (1e-5, 2.0, O.SPLIT_FULL)])
def test_pipeline_bound(eb, split, mode):
    mesh = G.kuhn_tet_mesh(9, 2)
    x = G.field_octaves(mesh.coords, np.random.default_rng(6))
    g = O.grid_from_dims(mesh.coords, (6, 5, 7))
    m = O.locate(mesh.coords, mesh.cells, g)
    cz = O.compress(mesh.coords, m, g, x, eb, True, split, mode=mode, delta=True)
    xr = O.decompress(mesh.coords, g, cz.bound, cz.grid, cz.vert, x.dtype, delta=True)
    assert np.all(np.abs(x.astype(np.float64) - xr.astype(np.float64)) <= cz.bound.tau2)


def test_cluster_pair_closed_loop_bound():
    mesh = G.kuhn_tet_mesh(9, 2)
    x = G.field_octaves(mesh.coords, np.random.default_rng(7))
    g = O.grid_from_dims(mesh.coords, (5, 6, 4))
    cz = O.compress_cluster(mesh.coords, g, x, 1e-4, True, 2.0, False, O.SPLIT_FULL, delta=True)
    xr = O.decompress_cluster(mesh.coords, g, cz.bound, cz.grid, cz.vert, x.dtype, delta=True)
    assert np.all(np.abs(x.astype(np.float64) - xr.astype(np.float64)) <= cz.bound.tau)
    with pytest.raises(ValueError):
        O.compress_cluster(mesh.coords, g, x, 1e-4, True, 0.5, True, delta=True)
