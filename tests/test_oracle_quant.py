"""Pins of the oracle's error split, grid compressor, back-interpolation,
residual compressor and decoders: closed forms, invariants (the bound of
Sec. III on every vertex), special cases that reduce to textbook linear
quantisation, and brute-force outlier sets."""
import numpy as np
import pytest

import meshgen as G
import oracle as O

R = O.RADIUS


def test_bound_closed_form():
    x = np.array([2.0, 6.0, 3.0])
    b = O.bound(x, 0.25, True, 0.5)
    assert (b.tau, b.tau1, b.tau2, b.c, b.xmin, b.xmax) == (1.0, 0.5, 0.5, 4.0, 2.0, 6.0)
    assert (b.step1, b.inv1, b.step2, b.inv2) == (1.0, 1.0, 1.0, 1.0)
    b = O.bound(x.astype(np.float32), 0.5, False, 0.25)
    assert (b.tau, b.tau1, b.tau2) == (0.5, 0.125, 0.375)
    for bad in [dict(eb=0.0), dict(eb=-1.0), dict(split=0.0), dict(split=1.0),
                dict(eb=float("nan"))]:
        kw = dict(eb=0.1, split=0.5)
        kw.update(bad)
        with pytest.raises(O.OracleError):
            O.bound(x, kw["eb"], True, kw["split"])
    with pytest.raises(O.OracleError):
        O.bound(np.array([1.0, np.nan]), 0.1, True, 0.5)
    with pytest.raises(O.OracleError):
        O.bound(np.array([1.0, np.inf]), 0.1, False, 0.5)
    with pytest.raises(O.OracleError):     # relative eb of a constant field
        O.bound(np.array([3.0, 3.0]), 0.1, True, 0.5)


def test_bound_closed_form_full_split():
    """SPLIT_FULL: tau1 = split * tau only sets the grid step; the residual
    keeps the whole tau (its check alone bounds the vertex error)."""
    x = np.array([2.0, 6.0, 3.0])
    b = O.bound(x, 0.25, True, 2.0, O.SPLIT_FULL)
    assert (b.tau, b.tau1, b.tau2, b.c) == (1.0, 2.0, 1.0, 4.0)
    assert (b.step1, b.inv1, b.step2, b.inv2) == (4.0, 0.25, 2.0, 0.5)
    b = O.bound(x, 0.25, True, 0.5, O.SPLIT_FULL)
    assert (b.tau1, b.tau2) == (0.5, 1.0)
    for split, mode in [(0.0, O.SPLIT_FULL), (16.5, O.SPLIT_FULL), (0.5, 2), (1.0, O.SPLIT_SUM)]:
        with pytest.raises(O.OracleError):
            O.bound(x, 0.25, True, split, mode)


@pytest.mark.parametrize("dims", [(7, 5, 1), (4, 6, 5)])
def test_lorenzo_roundtrip_and_annihilation(dims):
    dim = 2 if dims[2] == 1 else 3
    g = O.make_grid(dim, dims, (0, 0, 0), (1, 1, 1))
    rng = np.random.default_rng(1)
    n = g.count
    p = rng.integers(-2 ** 26, 2 ** 26, n).astype(np.int32)
    d = O.lorenzo(p, g)
    assert np.abs(d).max() < 2 ** 30
    codes = np.zeros(n, np.uint16)          # every node an outlier
    p2 = O.grid_decode(codes, np.arange(n, dtype=np.int32), d.astype(np.int32), g)
    assert np.array_equal(p, p2)
    # separable p(i,j,k) = a(i) + b(j) + c(k): zero error wherever every
    # index is >= 1
    a = rng.integers(-1000, 1000, dims[0])
    bb = rng.integers(-1000, 1000, dims[1])
    cc = rng.integers(-1000, 1000, dims[2]) if dim == 3 else np.zeros(1, int)
    P = (a[None, None, :] + bb[None, :, None] + cc[:, None, None]).astype(np.int32)
    d = O.lorenzo(P.ravel(), g).reshape(dims[2], dims[1], dims[0])
    if dim == 2:
        assert np.all(d[0, 1:, 1:] == 0)
    else:
        assert np.all(d[1:, 1:, 1:] == 0)
    # constant: a single non-zero error at the origin
    d = O.lorenzo(np.full(n, 17, np.int32), g)
    assert d[0] == 17 and np.all(d[1:] == 0)


def test_grid_quantize_bound_and_codes():
    rng = np.random.default_rng(2)
    g = O.make_grid(3, (9, 8, 7), (0, 0, 0), (1, 1, 1))
    v = rng.normal(size=g.count).astype(np.float32)
    b = O.bound(v.astype(np.float64), 1e-5, True, 0.3)
    gc = O.grid_quantize(v, g, b)
    xhat = O.grid_recon(gc.p, b)
    ulp = np.spacing(np.abs(xhat)).astype(np.float64)
    assert np.all(np.abs(v.astype(np.float64) - xhat) <= b.tau1 * (1 + 2 ** -40) + ulp)
    d = O.lorenzo(gc.p, g)
    inside = np.abs(d) <= R - 1
    assert np.array_equal(gc.codes[inside], (d[inside] + R).astype(np.uint16))
    assert np.all(gc.codes[~inside] == 0)
    assert np.array_equal(gc.out_idx, np.nonzero(~inside)[0])
    assert np.array_equal(gc.out_delta, d[~inside])
    assert gc.out_idx.size > 0
    p2 = O.grid_decode(gc.codes, gc.out_idx, gc.out_delta, g)
    assert np.array_equal(p2, gc.p)


def test_grid_quantize_range_error():
    g = O.make_grid(2, (3, 3, 1), (0, 0, 0), (1, 1, 1))
    v = np.zeros(9, np.float32)
    v[4] = 1.0
    b = O.bound(np.array([0.0, 1.0]), 1e-9, False, 0.5)   # |p| would reach 1e9
    with pytest.raises(O.OracleError) as e:
        O.grid_quantize(v, g, b)
    assert e.value.status == O.ERR_RANGE


@pytest.mark.parametrize("dim", [2, 3])
def test_back_interp_multilinear(dim):
    """g reproduces a multilinear grid function; a vertex on a node gets the
    node's value exactly; g stays within the corner range."""
    rng = np.random.default_rng(40 + dim)
    dims = (6, 5, 4) if dim == 3 else (6, 5, 1)
    g = O.make_grid(dim, dims, (0, 0, 0), (1, 1, 1))
    I = np.indices(dims[::-1])[::-1].reshape(3, -1).astype(np.float64)
    c = rng.integers(-8, 8, 5) / 4.0
    f = lambda X: c[0] + c[1] * X[0] + c[2] * X[1] + c[3] * X[0] * X[1] + (
        c[4] * X[2] if dim == 3 else 0)
    xhat = f(I).astype(np.float32)
    nv = 400
    pts = (rng.random((dim, nv)) * (np.array(dims[:dim])[:, None] - 1)).astype(np.float32)
    gv = O.back_interp(pts, g, xhat)
    exact = f(np.vstack([pts.astype(np.float64), np.zeros((3 - dim, nv))]))
    assert np.all(np.abs(gv - exact) <= 1e-5 * (1 + np.abs(exact)))
    nodes = I[:dim, rng.choice(g.count, 50)].astype(np.float32)
    gn = O.back_interp(np.ascontiguousarray(nodes), g, xhat)
    jj = (nodes[0] + dims[0] * nodes[1]
          + (dims[0] * dims[1] * nodes[2] if dim == 3 else 0)).astype(int)
    assert np.array_equal(gn, xhat[jj])
    xr = rng.normal(size=g.count).astype(np.float32)
    gv = O.back_interp(pts, g, xr)
    idx, _ = O.vertex_cells(pts, g)
    for v in range(nv):
        i = idx[v]
        corner = [xr[(i[0] + a) + dims[0] * ((i[1] + b) + dims[1] * (i[2] + cz))]
                  for a in (0, 1) for b in (0, 1) for cz in ((0, 1) if dim == 3 else (0,))]
        lo, hi = min(corner), max(corner)
        slack = 4 * np.spacing(np.float32(max(abs(lo), abs(hi))))
        assert lo - slack <= gv[v] <= hi + slack


def test_aligned_mesh_codes_all_zero():
    """Vertices on grid nodes, FP32 field, equal split: |r| <= tau1 = tau2 so
    |r / (2 tau2)| <= 1/2 and every residual code is R (zero)."""
    mesh = G.aligned_tri_mesh(17, 13)
    g = O.make_grid(2, (17, 13, 1), (0, 0, 0), (1, 1, 1))
    rng = np.random.default_rng(3)
    x = rng.normal(size=mesh.n_vertices).astype(np.float32)
    m = O.locate(mesh.coords, mesh.cells, g)
    assert m.n_unresolved == 0
    cz = O.compress(mesh.coords, m, g, x, 1e-2, True, 0.5)
    assert np.array_equal(cz.v, x)          # each node reproduces its vertex
    assert np.all(cz.vert.codes == R)
    assert cz.vert.out_idx.size == 0


def test_residual_textbook_quantizer():
    """With g = 0 and a power-of-two step the residual codes are textbook
    linear quantisation rint(x / (2 tau2))."""
    rng = np.random.default_rng(4)
    x = rng.normal(size=5000) * 3
    b = O.bound(x, 2.0 ** -6, False, 0.5)        # tau2 = 2^-7, step 2^-6
    gv = np.zeros(x.size, np.float32)
    vc = O.residual_quantize(x, gv, b)
    q = np.rint(x / 2.0 ** -6)
    ok = (np.abs(q) <= R - 1) & (np.abs(x - q * 2.0 ** -6) <= 2.0 ** -7)
    assert np.array_equal(vc.codes[ok], (q[ok] + R).astype(np.uint16))
    assert np.array_equal(vc.out_idx, np.nonzero(~ok)[0])
    assert ok.sum() == x.size


def _roundtrip(coords, cells, dims, x, eb, rel, split, fill="nearest", mode=O.SPLIT_SUM):
    g = O.grid_from_dims(coords, dims)
    m = O.locate(coords, cells, g, "raster", fill=fill)
    cz = O.compress(coords, m, g, x, eb, rel, split, mode=mode)
    xr = O.decompress(coords, g, cz.bound, cz.grid, cz.vert, x.dtype)
    return cz, xr


@pytest.mark.parametrize("eb", [1e-2, 1e-4, 1e-6, 1e-7])
@pytest.mark.parametrize("split", [0.1, 0.5, 0.9])
def test_bound_on_every_vertex_2d(eb, split):
    rng = np.random.default_rng(5)
    mesh = G.delaunay_2d(G.stratified_points_2d(40, rng))
    x = G.field_bumps_2d(mesh.coords, rng)
    cz, xr = _roundtrip(mesh.coords, mesh.cells, (33, 30), x, eb, True, split)
    assert np.all(np.abs(x - xr) <= cz.bound.tau2)
    assert cz.bound.tau1 + cz.bound.tau2 <= cz.bound.tau * (1 + 1e-15)
    # outlier list = brute-force set of non-coded vertices, ascending
    assert np.array_equal(cz.vert.out_idx, np.nonzero(cz.vert.codes == 0)[0])
    assert np.array_equal(cz.vert.out_val, x[cz.vert.out_idx])
    if eb == 1e-7:
        assert cz.grid.out_idx.size > 0
        if split == 0.9:
            assert cz.vert.out_idx.size > 0


@pytest.mark.parametrize("eb,split", [(1e-2, 0.5), (1e-4, 1.0), (1e-4, 4.0), (1e-6, 0.25)])
def test_bound_on_every_vertex_full_split(eb, split):
    """Every vertex within tau2 = tau; the grid part equals the one of the
    sum split with the same tau1 (it depends on tau1 only), and the residual
    codes equal the plain quantiser of x - g(x1') with step 2 tau."""
    rng = np.random.default_rng(9)
    mesh = G.delaunay_2d(G.stratified_points_2d(40, rng))
    x = G.field_bumps_2d(mesh.coords, rng)
    cz, xr = _roundtrip(mesh.coords, mesh.cells, (33, 30), x, eb, True, split, mode=O.SPLIT_FULL)
    assert cz.bound.tau2 == cz.bound.tau and cz.bound.tau1 == split * cz.bound.tau
    assert np.all(np.abs(x - xr) <= cz.bound.tau)
    q = np.rint((x - cz.gv.astype(np.float64)) * cz.bound.inv2)
    ok = cz.vert.codes != 0
    assert np.array_equal(cz.vert.codes[ok].astype(np.int64) - R, q[ok].astype(np.int64))
    if split < 1.0:
        cs, _ = _roundtrip(mesh.coords, mesh.cells, (33, 30), x, eb, True, split)
        assert np.array_equal(cs.grid.codes, cz.grid.codes) and np.array_equal(cs.grid.p, cz.grid.p)


def test_tiny_eb_is_a_range_error():
    """|p| < 2^27 is required; eb = 1e-9 of the range needs |p| ~ 1e9."""
    rng = np.random.default_rng(5)
    mesh = G.delaunay_2d(G.stratified_points_2d(20, rng))
    x = G.field_bumps_2d(mesh.coords, rng)
    with pytest.raises(O.OracleError) as e:
        _roundtrip(mesh.coords, mesh.cells, (16, 16), x, 1e-9, True, 0.5)
    assert e.value.status == O.ERR_RANGE


@pytest.mark.parametrize("eb,split,fill", [(1e-2, 0.3, "nearest"), (1e-5, 0.7, "midrange")])
def test_bound_on_every_vertex_3d(eb, split, fill):
    mesh = G.kuhn_tet_mesh(9, 2)
    x = G.field_octaves(mesh.coords, np.random.default_rng(6))
    cz, xr = _roundtrip(mesh.coords, mesh.cells, (10, 11, 9), x, eb, True, split, fill)
    assert xr.dtype == np.float32
    assert np.all(np.abs(x.astype(np.float64) - xr) <= cz.bound.tau2)


def test_learned_codes_zero_shift_equals_plain():
    rng = np.random.default_rng(7)
    mesh = G.structured_tri_mesh(90, 100, rng, 0.2)
    x = G.field_octaves(mesh.coords, rng, dtype=np.float64)
    g = O.grid_from_dims(mesh.coords, (40, 50))
    m = O.locate(mesh.coords, mesh.cells, g)
    plain = O.compress(mesh.coords, m, g, x, 1e-4, True, 0.5)
    z = np.zeros(mesh.n_vertices, np.int32)
    lc = O.learned_codes(x, plain.gv, plain.bound, z)
    assert np.array_equal(lc.codes, plain.vert.codes)
    assert np.all(lc.block_flags == 0)


def _zz_bits(k):
    z = (np.asarray(k, np.int64) << 1) ^ (np.asarray(k, np.int64) >> 63)
    return np.array([int(v).bit_length() for v in z])


def test_learned_codes_block_choice_and_roundtrip():
    rng = np.random.default_rng(8)
    mesh = G.structured_tri_mesh(120, 110, rng, 0.2)
    x = G.field_octaves(mesh.coords, rng, dtype=np.float32)
    g = O.grid_from_dims(mesh.coords, (40, 40))
    m = O.locate(mesh.coords, mesh.cells, g)
    plain = O.compress(mesh.coords, m, g, x, 1e-5, True, 0.5)
    q = plain.vert.codes.astype(np.int64) - R
    nv = x.size
    # a shift that is good in even blocks and bad in odd blocks
    blk = np.arange(nv) // O.BLOCK
    rho = np.where(blk % 2 == 0, q, q + rng.integers(-50, 50, nv)).astype(np.int32)
    rho[plain.vert.codes == 0] = 7
    lc = O.learned_codes(x, plain.gv, plain.bound, rho)
    nb = (nv + O.BLOCK - 1) // O.BLOCK
    coded = plain.vert.codes != 0
    for bi in range(nb):
        s = slice(bi * O.BLOCK, min(nv, (bi + 1) * O.BLOCK))
        cp = _zz_bits(q[s][coded[s]]).sum() + (~coded[s]).sum() * 64
        cl_raw = q[s] - rho[s]
        okl = coded[s] & (np.abs(cl_raw) <= R - 1)
        cl = _zz_bits(cl_raw[okl]).sum() + (~okl).sum() * 64
        flag = (lc.block_flags[bi // 32] >> (bi % 32)) & 1
        assert flag == int(cl < cp)
    xr = O.vertex_decode(lc, plain.gv, plain.bound, np.float32, rho)
    assert np.all(np.abs(x.astype(np.float64) - xr) <= plain.bound.tau2)
    assert np.array_equal(lc.out_idx, np.nonzero(lc.codes == 0)[0])
