"""Pins of the oracle's 1-D serialisation baseline: closed forms (a
constant field codes to R everywhere, a ramp of k steps per sample to the
constant difference k), the error bound on every value for both dtypes and
both bound modes, raw storage of spikes, and a lossless round trip of the
codes through the decoder."""
import numpy as np
import pytest

import oracle as O

R = O.RADIUS


def test_constant_field_codes_to_zero_difference():
    x = np.full(1000, 3.25, np.float64)
    codes, oi, ov, b = O.serial_compress(x, 1e-3, False)
    assert b.c == 3.25 and oi.size == 0
    assert np.all(codes == R)


def test_ramp_gives_constant_difference():
    """x_i = c0 + k * 2 tau * i: p_i = k i + p_0, so every difference after
    the first is k (absolute bound, tau exact in binary)."""
    tau, k = 0.125, 3
    i = np.arange(513, dtype=np.float64)
    x = 10.0 + k * 2 * tau * (i - 256)          # centred: c = 10, p_i = k (i - 256)
    codes, oi, ov, b = O.serial_compress(x, tau, False)
    assert b.c == 10.0 and b.tau == tau
    assert codes[0] == R + k * (-256)
    assert np.all(codes[1:] == R + k)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("relative,eb", [(True, 1e-3), (True, 1e-6), (False, 0.01)])
def test_bound_on_every_value(dtype, relative, eb):
    rng = np.random.default_rng(7)
    x = np.cumsum(rng.normal(size=20000)).astype(dtype)
    x[::997] += dtype(500.0)                     # spikes: differences out of range
    codes, oi, ov, b = O.serial_compress(x, eb, relative)
    xr = O.serial_decompress(codes, oi, ov, b, dtype)
    err = np.abs(x.astype(np.float64) - xr.astype(np.float64))
    assert np.all(err <= b.tau)
    assert np.array_equal(x[oi], ov)             # raw values stored exactly
    assert np.array_equal(xr[oi].view(np.uint8), ov.view(np.uint8))
    if relative and eb == 1e-6:
        assert oi.size >= 20                     # the spikes' differences exceed the code range


def test_differences_match_definition_on_small_input():
    x = np.array([0.0, 0.3, 0.31, -0.2, 5.0, 5.05], np.float64)
    codes, oi, ov, b = O.serial_compress(x, 0.05, False)
    c = 0.5 * (5.05 + -0.2)
    p = np.rint((x - c) / 0.1).astype(np.int64)
    d = np.diff(np.concatenate([[0], p]))
    for i in range(x.size):
        if codes[i]:
            assert int(codes[i]) - R == d[i]
