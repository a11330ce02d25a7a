"""Pins of the oracle's multilevel interpolation grid predictor (an
alternative grid compressor: the SZ family's interpolation predictor,
Sec. II; any compressor may serve as C(x1), Sec. IV-D), checked against
properties fixed by the mathematics rather than by its own formulas:

* polynomial exactness: the two-point rule reproduces affine fields and the
  four-point rule (-1, 9, 9, -1)/16 cubic ones, so the errors vanish except
  where a rule cannot apply, and there they equal closed forms;
* floor rounding of a non-exact prediction, on a worked example computed by
  hand;
* decode(encode(p)) == p on random grids of many shapes (the decoder checks
  that every prediction reads an already decoded node);
* the predictor leaves p, x1' and the vertex codes of the pipeline unchanged.
"""
import numpy as np
import pytest

import meshgen as G
import oracle as O


def grid(dims):
    dim = len(dims)
    return O.make_grid(dim, tuple(dims) + (1,) * (3 - dim), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0))


def coords_of(g):
    n = g.dims()
    j = np.arange(g.count)
    return j % n[0], (j // n[0]) % n[1], j // (n[0] * n[1])


@pytest.mark.parametrize("dims", [(9, 9), (17, 17, 17), (33, 33), (5, 5, 5)])
@pytest.mark.parametrize("cubic", [False, True])
def test_affine_field(dims, cubic):
    """p = p0 + sum_d alpha_d i_d on a grid of equal extents n = 2^k + 1:
    both rules reproduce affine data wherever both neighbours exist.  A node
    of stride s along axis a lacks its +s neighbour only when s = 2^k and
    i_a = 2^k = n - 1; the coordinates below a are then multiples of 2^k
    (0 or n - 1) and those above a multiples of 2^(k+1) (only 0).  So the
    non-zero errors are the origin's (p0) and the other corners', each
    predicted by the node n - 1 below along its highest axis at n - 1:
    error alpha_a (n - 1)."""
    g = grid(dims)
    alpha = [3, -7, 11][: len(dims)]
    p0 = 5
    i = coords_of(g)
    p = p0 + sum(alpha[d] * i[d] for d in range(len(dims)))
    d = O.interp_delta(p.astype(np.int32), g, cubic)
    n = dims[0]
    expect = np.zeros(g.count, np.int64)
    expect[0] = p0
    corner = np.ones(g.count, bool)
    for a in range(len(dims)):
        corner &= (i[a] == 0) | (i[a] == n - 1)
    for j in np.nonzero(corner)[0]:
        if j == 0:
            continue
        a = max(x for x in range(len(dims)) if i[x][j] == n - 1)
        expect[j] = alpha[a] * (n - 1)
    assert np.array_equal(d, expect)


@pytest.mark.parametrize("n0", [33, 65])
def test_cubic_polynomial_along_axis0(n0):
    """p = i^3 - 2 i^2 + 5 along axis 0, constant along axis 1.  Nodes
    predicted along axis 1 see a constant: error 0.  Along axis 0 at stride
    s and position i (odd multiple of s): the four-point rule is exact for
    cubics (error 0 where i - 3s >= 0 and i + 3s <= n - 1); the two-point
    rule's error is -(3 i s^2 - 2 s^2) (mean of i +- s minus the value);
    with no +s neighbour the error is p(i) - p(i - s)."""
    g = grid((n0, 6))
    i0, i1, _ = coords_of(g)
    f = lambda x: x ** 3 - 2 * x ** 2 + 5
    p = f(i0).astype(np.int64)
    d = O.interp_delta(p.astype(np.int32), g, True)
    dl = O.interp_delta(p.astype(np.int32), g, False)
    for j in range(g.count):
        x, y = int(i0[j]), int(i1[j])
        if x == 0 and y == 0:
            assert d[j] == 5 and dl[j] == 5
            continue
        # axis 0 is the class axis iff x has strictly fewer trailing zeros
        # than y (y = 0 counts as infinitely many)
        tz = lambda v: 99 if v == 0 else (v & -v).bit_length() - 1
        if not (x != 0 and tz(x) < tz(y)):
            assert d[j] == 0 and dl[j] == 0, (x, y)
            continue
        s = 1 << tz(x)
        if x + s > n0 - 1:
            assert d[j] == f(x) - f(x - s) and dl[j] == f(x) - f(x - s)
            continue
        two_point = -(3 * x * s * s - 2 * s * s)
        assert dl[j] == two_point, (x, s)
        if x - 3 * s >= 0 and x + 3 * s <= n0 - 1:
            assert d[j] == 0, (x, s)
        else:
            assert d[j] == two_point, (x, s)


def test_worked_example_rounding():
    """Grid 9 x 2, row 0 = (0, 7, -1, 4, -2, 3, 0, 1, 6), row 1 = row 0 + 1,
    by hand.  L = 4 (2^4 >= 9); on row 0 the classes are
      x = 8 (s = 8): no +8 neighbour -> p(0) = 0, error 6
      x = 4 (s = 4): two-point floor((0 + 6) / 2) = 3, error -5
      x = 2, 6 (s = 2): two-point floor((0 - 2) / 2) = -1 -> error 0;
                        floor((-2 + 6) / 2) = 2 -> error -2
      x = 1 (s = 1): two-point floor((0 - 1) / 2) = -1 -> error 8
      x = 3: four-point (0, -1, -2, 0): floor((0 - 9 - 18 - 0 + 8) / 16)
             = floor(-19 / 16) = -2 -> error 6 (the two-point rule:
             floor(-3 / 2) = -2 -> error 6)
      x = 5: four-point (-1, -2, 0, 6): floor((1 - 18 + 0 - 6 + 8) / 16)
             = floor(-15 / 16) = -1 -> error 4 (two-point: floor(-2 / 2)
             = -1 -> error 4)
      x = 7: no x + 3 inside -> two-point floor((0 + 6) / 2) = 3 -> error -2
    Row 1 (y = 1, class axis 1, no +1 neighbour): prediction = the node
    below, error 1 everywhere."""
    g = grid((9, 2))
    row = np.array([0, 7, -1, 4, -2, 3, 0, 1, 6], np.int32)
    p = np.concatenate([row, row + 1])
    cub = O.interp_delta(p, g, True)
    lin = O.interp_delta(p, g, False)
    exp_row = [0, 8, 0, 6, -5, 4, -2, -2, 6]
    assert list(cub[:9]) == exp_row
    assert list(lin[:9]) == exp_row
    assert list(cub[9:]) == [1] * 9 and list(lin[9:]) == [1] * 9
    # a case where the two rules differ: x = 3 with p(6) = 30
    row2 = row.copy()
    row2[6] = 30
    p2 = np.concatenate([row2, row2])
    c2 = O.interp_delta(p2, g, True)
    l2 = O.interp_delta(p2, g, False)
    # four-point: floor((0 - 9 - 18 - 30 + 8) / 16) = floor(-49 / 16) = -4 -> error 8
    # two-point:  floor((-1 - 2) / 2) = -2 -> error 6
    assert c2[3] == 8 and l2[3] == 6


@pytest.mark.parametrize("dims", [(2, 2), (3, 2), (2, 7), (64, 64), (100, 37), (2, 2, 2), (17, 16, 15),
                                  (33, 5, 9), (40, 41, 3)])
@pytest.mark.parametrize("gpred", [O.GPRED_LINEAR, O.GPRED_CUBIC])
def test_roundtrip_random(dims, gpred):
    g = grid(dims)
    rng = np.random.default_rng(hash(dims) % 1000)
    # smooth part plus spikes beyond the code radius (outliers)
    i = coords_of(g)
    p = (np.sin(i[0] * 0.3) * 4000 + np.cos(i[1] * 0.2) * 3000 + i[2] * 7).astype(np.int64)
    p += rng.integers(-50, 51, g.count)
    spikes = rng.choice(g.count, size=max(1, g.count // 50), replace=False)
    p[spikes] += rng.choice([-1, 1], spikes.size) * 100000
    p = p.astype(np.int32)
    gc = O.grid_codes(p, g, gpred)
    assert gc.out_idx.size > 0
    assert np.all(np.diff(gc.out_idx) > 0)
    assert np.all(gc.codes[gc.out_idx] == 0)
    q = O.grid_decode(gc.codes, gc.out_idx, gc.out_delta, g, gpred)
    assert np.array_equal(q, p)


def test_pipeline_unchanged_but_grid_codes():
    """Alg. 3 / Alg. 4 with either grid predictor: the same p, x1', vertex
    codes and reconstruction as with the Lorenzo predictor; only the grid
    codes differ."""
    mesh = G.kuhn_tet_mesh(10, 3)
    x = G.field_octaves(mesh.coords, np.random.default_rng(4))
    g = O.grid_from_dims(mesh.coords, (12, 11, 9))
    m = O.locate(mesh.coords, mesh.cells, g)
    ref = O.compress(mesh.coords, m, g, x, 1e-4, True, 0.5)
    xr = O.decompress(mesh.coords, g, ref.bound, ref.grid, ref.vert, x.dtype)
    for gp in (O.GPRED_LINEAR, O.GPRED_CUBIC):
        c = O.compress(mesh.coords, m, g, x, 1e-4, True, 0.5, gpred=gp)
        assert np.array_equal(c.grid.p, ref.grid.p)
        assert np.array_equal(c.xhat, ref.xhat)
        assert np.array_equal(c.vert.codes, ref.vert.codes)
        assert not np.array_equal(c.grid.codes, ref.grid.codes)
        y = O.decompress(mesh.coords, g, c.bound, c.grid, c.vert, x.dtype, gpred=gp)
        assert np.array_equal(y.view(np.uint8), xr.view(np.uint8))
