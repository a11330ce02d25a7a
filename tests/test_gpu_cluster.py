"""GPU parity of the paper's own operator pair (nearest-node g, cluster-mean
f; Sec. IV-C/IV-D) with the open-loop residual of Alg. 3 and the closed-loop
option: node map, cluster means (through the prequantised grid), grid and
vertex codes, outlier lists and decoded values bit for bit against the
oracle; every vertex within tau (open) or tau2 (closed)."""
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
    m3 = G.kuhn_tet_mesh(22, 5)
    f3 = G.field_octaves(m3.coords, np.random.default_rng(1))
    out.append(("kuhn3d_f32_open", m3, f3, (12, 11, 10), 1e-4, True, 0.5, "open", "sum"))
    out.append(("kuhn3d_f32_closed_full", m3, f3, (12, 11, 10), 1e-4, True, 2.0, "closed", "full"))
    out.append(("kuhn3d_f32_fine_grid", m3, f3, (40, 37, 33), 1e-3, True, 0.3, "open", "sum"))   # many empty nodes
    mesh, f, cfg = G.config_small_2d()
    out.append(("small2d_f64_open", mesh, f, (40, 40), cfg["eb"], False, 0.5, "open", "sum"))
    out.append(("small2d_f64_closed", mesh, f, (40, 40), cfg["eb"], False, 0.5, "closed", "sum"))
    m4 = G.kuhn_tet_mesh(17, 6)
    x4 = G.field_octaves(m4.coords, np.random.default_rng(2), dtype=np.float64)
    out.append(("kuhn3d_f64_tiny_eb", m4, x4, (9, 10, 8), 1e-7, True, 0.9, "open", "sum"))
    return out


CASES = _cases()


class Case:
    def __init__(self, name, mesh, x, dims, eb, rel, split, residual, mode):
        self.name, self.mesh, self.x, self.dims = name, mesh, x, dims
        self.eb, self.rel, self.split, self.residual, self.mode = eb, rel, split, residual, mode
        print(f"[cluster] {name}: nv={mesh.n_vertices} dims={dims} eb={eb} rel={rel} split={split} ({mode}) "
              f"residual={residual} dtype={x.dtype}", flush=True)
        self.og = O.grid_from_dims(mesh.coords, dims)
        self.dx = dev(x)
        self.plan = M.Plan(dev(mesh.coords), None, dims=dims, operators="cluster")

    def oracle(self):
        return O.compress_cluster(self.mesh.coords, self.og, self.x, self.eb, self.rel, self.split,
                                  self.residual == "open", O.SPLIT_FULL if self.mode == "full" else O.SPLIT_SUM)

    def gpu(self):
        codes = M.compress(self.plan, self.dx, self.eb, "rel" if self.rel else "abs", self.split, debug=True,
                           split_mode=self.mode, residual=self.residual)
        torch.cuda.synchronize()
        return codes


@pytest.fixture(scope="module", params=range(len(CASES)), ids=[c[0] for c in CASES])
def case(request):
    return Case(*CASES[request.param])


def test_node_map_and_cluster_means(case):
    oc = case.oracle()
    assert np.array_equal(case.plan.nodes().cpu().numpy(), oc.m)
    assert case.plan.info()["n_unresolved"] == int((oc.count == 0).sum())
    codes = case.gpu()
    assert np.array_equal(codes.dbg_resampled.cpu().numpy().view(np.uint32),
                          oc.x1.astype(np.float32).view(np.uint32))
    assert np.array_equal(codes.dbg_grid_p.cpu().numpy(), oc.grid.p)
    print(f"[cluster] {case.name}: {int((oc.count == 0).sum())} empty nodes of {oc.count.size}")


def test_node_lists_are_a_stable_sort(case):
    """The plan's per-node vertex lists (its own LSD radix sort) against the
    definition: vertices ordered by node, equal nodes by id, and node j's
    run starting at the number of vertices on nodes before j."""
    m = case.plan.nodes().cpu().numpy()
    noff, vlist = case.plan.node_lists()
    noff, vlist = noff.cpu().numpy(), vlist.cpu().numpy()
    assert np.array_equal(vlist, np.argsort(m, kind="stable").astype(np.int32))
    counts = np.bincount(m, minlength=noff.size - 1)
    assert np.array_equal(noff, np.concatenate([[0], np.cumsum(counts)]).astype(np.int64))


@pytest.mark.parametrize("dims", [(6, 5, 4), (300, 262)])
def test_node_lists_one_and_three_sort_passes(dims):
    """Node lists where the radix sort takes one 8-bit pass (120 nodes) and
    three (78,600 nodes, 17 bits), on a vertex count that is no multiple of
    the sort's 4,096-key tile."""
    if len(dims) == 3:
        mesh = G.kuhn_tet_mesh(19, 3)
    else:
        mesh = G.structured_tri_mesh(211, 173, np.random.default_rng(3), 0.2)
    assert mesh.n_vertices % 4096 != 0
    plan = M.Plan(dev(mesh.coords), None, dims=dims, operators="cluster")
    m = plan.nodes().cpu().numpy()
    noff, vlist = plan.node_lists()
    assert np.array_equal(vlist.cpu().numpy(), np.argsort(m, kind="stable").astype(np.int32))
    counts = np.bincount(m, minlength=plan.n_grid)
    assert np.array_equal(noff.cpu().numpy(), np.concatenate([[0], np.cumsum(counts)]).astype(np.int64))


def test_codes_bitexact(case):
    oc = case.oracle()
    h = case.gpu().host()
    r = h["result"]
    assert r["status"] == 0
    for k in ("tau", "tau1", "tau2", "c", "xmin", "xmax"):
        assert r[k] == getattr(oc.bound, k), k
    assert np.array_equal(h["grid_codes"], oc.grid.codes)
    assert np.array_equal(h["g_out_idx"], oc.grid.out_idx)
    assert np.array_equal(h["g_out_delta"], oc.grid.out_delta)
    assert np.array_equal(h["vert_codes"], oc.vert.codes)
    assert np.array_equal(h["v_out_idx"], oc.vert.out_idx)
    assert np.array_equal(h["v_out_val"].view(np.uint8), oc.vert.out_val.view(np.uint8))
    print(f"[cluster] {case.name}: grid outliers {oc.grid.out_idx.size}, vertex outliers {oc.vert.out_idx.size}")


def test_roundtrip_bitexact_and_bound(case):
    oc = case.oracle()
    codes = case.gpu()
    xr = M.decompress(case.plan, codes)
    torch.cuda.synchronize()
    xg = xr.cpu().numpy()
    xo = O.decompress_cluster(case.mesh.coords, case.og, oc.bound, oc.grid, oc.vert, case.x.dtype)
    assert np.array_equal(xg.view(np.uint8), xo.view(np.uint8))
    bound = oc.bound.tau if case.residual == "open" else oc.bound.tau2
    assert np.all(np.abs(case.x.astype(np.float64) - xg.astype(np.float64)) <= bound)


def test_rejected_combinations():
    mesh = G.kuhn_tet_mesh(9, 2)
    x = dev(G.field_octaves(mesh.coords, np.random.default_rng(6)))
    lin = M.Plan(dev(mesh.coords), dev(mesh.cells), dims=(8, 8, 8))
    with pytest.raises(M.McError) as e:
        M.compress(lin, x, 1e-3, residual="open")          # open loop needs the cluster pair
    assert e.value.status == M.ERR_UNSUPPORTED
    with pytest.raises(M.McError):
        lin.nodes()
    cl = M.Plan(dev(mesh.coords), None, dims=(8, 8, 8), operators="cluster")
    with pytest.raises(M.McError) as e:
        M.compress(cl, x, 1e-3, 2.0, split_mode="full", residual="open")
    assert e.value.status == M.ERR_UNSUPPORTED
    with pytest.raises(M.McError):
        cl.mapping()


@pytest.mark.parametrize("which,dims,open_loop,gpred", [
    ("kuhn3d", (60, 58, 50), True, "lorenzo"),
    ("kuhn3d", (60, 58, 50), False, "cubic"),
    ("kuhn3d", (13, 12, 11), True, "lorenzo"),          # coarser than the lattice: nothing to drop
    ("struct2d", (700, 520), True, "lorenzo"),
    ("struct2d", (700, 520), False, "temporal"),
])
def test_grid_coarsen(which, dims, open_loop, gpred):
    """Grid_Coarsen (Alg. 2) on the GPU: kept planes, node map, codes and
    decoded values bit for bit against the oracle, and the decoded values
    equal to those of the plan without coarsening."""
    if which == "kuhn3d":
        mesh = G.kuhn_tet_mesh(22, 5)
        x = G.field_octaves(mesh.coords, np.random.default_rng(1))
        eb, rel = 1e-4, True
    else:
        rng = np.random.default_rng(21)
        mesh = G.structured_tri_mesh(201, 151, rng, 0.2)             # jittered lattice: empty grid lines
        x = G.field_octaves(mesh.coords, rng, dtype=np.float64)
        eb, rel = 1e-6, True
    print(f"[cluster] coarsen {which} {dims} open={open_loop} {gpred}", flush=True)
    og = O.grid_from_dims(mesh.coords, dims)
    keep, ogc, om = O.grid_coarsen(O.nearest_nodes(mesh.coords, og), og)
    gp = {"lorenzo": O.GPRED_LORENZO, "cubic": O.GPRED_CUBIC, "temporal": O.GPRED_TEMPORAL}[gpred]
    ref = None
    if gpred == "temporal":
        ref = np.linspace(-1.0, 1.0, ogc.count).astype(np.float32)      # any reference both sides hold
    oc = O.compress_cluster(mesh.coords, og, x, eb, rel, 0.5, open_loop, gpred=gp, gref=ref, coarsen=True)
    plan = M.Plan(dev(mesh.coords), None, dims=dims, operators="cluster", coarsen=True)
    assert np.array_equal(plan.kept_planes(), keep)
    assert tuple(plan.grid.dims) == ogc.dims() and plan.n_grid == ogc.count
    assert np.array_equal(plan.nodes().cpu().numpy(), om)
    noff, vlist = plan.node_lists()                  # the lists on the coarsened grid
    assert np.array_equal(vlist.cpu().numpy(), np.argsort(om, kind="stable").astype(np.int32))
    assert int(noff[-1]) == mesh.n_vertices and noff.numel() == ogc.count + 1
    xt = dev(x)
    kw = {} if ref is None else dict(grid_ref=dev(ref))
    codes = M.Codes(plan, xt.dtype, grid_predictor=gpred, **kw)
    M.compress(plan, xt, eb, "rel" if rel else "abs", 0.5, codes=codes, residual="open" if open_loop else "closed")
    out = M.decompress(plan, codes)
    torch.cuda.synchronize()
    h = codes.host()
    assert h["result"]["status"] == 0
    assert np.array_equal(h["grid_codes"], oc.grid.codes)
    assert np.array_equal(h["g_out_idx"], oc.grid.out_idx)
    assert np.array_equal(h["vert_codes"], oc.vert.codes)
    xo = O.decompress_cluster(mesh.coords, og, oc.bound, oc.grid, oc.vert, x.dtype, gpred=gp, gref=ref, coarsen=True)
    assert np.array_equal(out.cpu().numpy().view(np.uint8), xo.view(np.uint8))
    full = M.Plan(dev(mesh.coords), None, dims=dims, operators="cluster")
    fc = M.compress(full, xt, eb, "rel" if rel else "abs", 0.5, residual="open" if open_loop else "closed")
    fo = M.decompress(full, fc)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy().view(np.uint8), fo.cpu().numpy().view(np.uint8))
    print(f"[cluster] coarsened {dims} -> {ogc.dims()}")


def test_grid_coarsen_rejected():
    mesh = G.kuhn_tet_mesh(9, 2)
    with pytest.raises(M.McError) as e:
        M.Plan(dev(mesh.coords), dev(mesh.cells), dims=(8, 8, 8), coarsen=True)
    assert e.value.status == M.ERR_UNSUPPORTED
    plan = M.Plan(dev(mesh.coords), None, dims=(8, 8, 8), operators="cluster")
    with pytest.raises(M.McError) as e:
        plan.kept_planes()
    assert e.value.status == M.ERR_UNSUPPORTED
