"""GPU tests of batched compression: a batch of fields on several meshes of
both dimensions and dtypes, captured once into a HIP graph and replayed,
gives for every item exactly what a separate mc_compress call gives (codes,
outlier lists, result), which the oracle checks in turn on a sample of
items; replays read the fields' current contents; destroying a plan drops
the graphs that used it."""
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


def same(a, b):
    ra, rb = dict(a["result"]), dict(b["result"])
    assert ra == rb
    for k in ("grid_codes", "vert_codes", "g_out_idx", "g_out_delta", "v_out_idx", "block_flags"):
        assert np.array_equal(a[k], b[k]), k
    assert np.array_equal(a["v_out_val"].view(np.uint8), b["v_out_val"].view(np.uint8))


@pytest.fixture(scope="module")
def workload():
    meshes, grids, fields = G.config_batch(seed=5, scale=0.002, n_meshes=4, n_fields=10)
    plans = [M.Plan(dev(m.coords), dev(m.cells), dims=g[:2] if g[2] == 1 else g) for m, g in zip(meshes, grids)]
    xs = [dev(f["data"]) for f in fields]
    return meshes, grids, fields, plans, xs


def _items(fields, plans, xs, codes, models=None):
    items = []
    for i, f in enumerate(fields):
        model = None if models is None else models.get(f["mesh"])
        items.append((plans[f["mesh"]], xs[i], f["eb"], f["eb_mode"], f["split"], model, codes[i]))
    return items


def test_batch_equals_single_calls_and_oracle(workload):
    meshes, grids, fields, plans, xs = workload
    print(f"[batch] {len(meshes)} meshes (nv {[m.n_vertices for m in meshes]}), {len(fields)} fields")
    codes = [M.Codes(plans[f["mesh"]], xs[i].dtype) for i, f in enumerate(fields)]
    M.batch_compress(_items(fields, plans, xs, codes))
    torch.cuda.synchronize()
    got = [c.host() for c in codes]
    for i, f in enumerate(fields):
        ref = M.compress(plans[f["mesh"]], xs[i], f["eb"], f["eb_mode"], f["split"]).host()
        same(got[i], ref)
        assert got[i]["result"]["status"] == 0
    # the oracle on one field per mesh
    for m in range(len(meshes)):
        i = m
        g = grids[m][:2] if grids[m][2] == 1 else grids[m]
        og = O.grid_from_dims(meshes[m].coords, g)
        om = O.locate(meshes[m].coords, meshes[m].cells, og)
        oc = O.compress(meshes[m].coords, om, og, fields[i]["data"], fields[i]["eb"], True, fields[i]["split"])
        assert np.array_equal(got[i]["grid_codes"], oc.grid.codes)
        assert np.array_equal(got[i]["vert_codes"], oc.vert.codes)
        assert np.array_equal(got[i]["g_out_idx"], oc.grid.out_idx)
        assert np.array_equal(got[i]["v_out_idx"], oc.vert.out_idx)


def test_replay_reads_current_fields(workload):
    meshes, grids, fields, plans, xs = workload
    codes = [M.Codes(plans[f["mesh"]], xs[i].dtype) for i, f in enumerate(fields)]
    items = _items(fields, plans, xs, codes)
    M.batch_compress(items)                     # capture (or replay of an identical list)
    torch.cuda.synchronize()
    saved = [x.clone() for x in xs]
    for rep in range(3):
        for i, x in enumerate(xs):              # new contents, same addresses
            x.copy_(saved[i] * (1.0 + 0.25 * (rep + 1)) + 0.1 * rep)
        M.batch_compress(items)                 # replay
        torch.cuda.synchronize()
        for i, f in enumerate(fields):
            ref = M.compress(plans[f["mesh"]], xs[i], f["eb"], f["eb_mode"], f["split"]).host()
            same(codes[i].host(), ref)
    for i, x in enumerate(xs):
        x.copy_(saved[i])
    torch.cuda.synchronize()


def test_batch_with_models_and_errors(workload):
    meshes, grids, fields, plans, xs = workload
    # a model for the first 2-D and the first 3-D mesh, trained on that mesh's first field
    models = {}
    for m in (0, 1):
        models[m] = M.Model.train(plans[m], xs[m], eb=1e-4, steps=20, batch=512, seed=m)
    codes = [M.Codes(plans[f["mesh"]], xs[i].dtype, learned=f["mesh"] in models) for i, f in enumerate(fields)]
    items = _items(fields, plans, xs, codes, models)
    # one item asks for a bound too fine for the grid quantizer's range
    bad = list(items[2])
    bad[2] = 1e-12
    items[2] = tuple(bad)
    M.batch_compress(items)
    torch.cuda.synchronize()
    for i, it in enumerate(items):
        if i == 2:
            continue
        plan, x, eb, mode, share, model, _ = it
        ref = M.compress(plan, x, eb, mode, share, model=model).host()
        same(codes[i].host(), ref)
        assert codes[i].result_host()["status"] == 0
    assert codes[2].result_host()["status"] == M.ERR_RANGE


def test_batch_decompress_equals_single_calls(workload):
    meshes, grids, fields, plans, xs = workload
    models = {0: M.Model.train(plans[0], xs[0], eb=1e-4, steps=10, batch=256, seed=9)}
    codes = [M.Codes(plans[f["mesh"]], xs[i].dtype, learned=f["mesh"] in models) for i, f in enumerate(fields)]
    M.batch_compress(_items(fields, plans, xs, codes, models))
    outs = [torch.empty_like(x) for x in xs]
    ditems = [(plans[f["mesh"]], codes[i], models.get(f["mesh"]), outs[i]) for i, f in enumerate(fields)]
    for rep in range(2):                       # capture, then replay
        for o in outs:
            o.fill_(7.0)
        M.batch_decompress(ditems)
        torch.cuda.synchronize()
        for i, f in enumerate(fields):
            ref = M.decompress(plans[f["mesh"]], codes[i], model=models.get(f["mesh"]))
            assert torch.equal(outs[i].view(torch.uint8), ref.view(torch.uint8)), (rep, i)
            tau2 = codes[i].result_host()["tau2"]
            assert (outs[i].double() - xs[i].double()).abs().max().item() <= tau2


def test_destroyed_plan_drops_its_graph():
    mesh = G.structured_tri_mesh(60, 60, np.random.default_rng(1), 0.2)
    x = dev(G.field_octaves(mesh.coords, np.random.default_rng(2)))
    for dims in ((20, 20), (33, 17)):
        plan = M.Plan(dev(mesh.coords), dev(mesh.cells), dims=dims)
        codes = M.Codes(plan, x.dtype)
        M.batch_compress([(plan, x, 1e-3, "rel", 0.5, None, codes)])
        torch.cuda.synchronize()
        same(codes.host(), M.compress(plan, x, 1e-3, "rel", 0.5).host())
        plan.destroy()
    M.batch_release()


def test_batch_rejects_bad_items(workload):
    meshes, grids, fields, plans, xs = workload
    codes = M.Codes(plans[0], xs[0].dtype)
    with pytest.raises(RuntimeError, match="item 1"):
        M.batch_compress([(plans[0], xs[0], 1e-3, "rel", 0.5, None, codes),
                          (plans[0], xs[0], -1.0, "rel", 0.5, None, codes)])


def test_batch_mixes_operator_pairs_and_residual_coders(workload):
    """One graph over linear plans with plain and delta residual codes and
    cluster plans (open loop): every item equals its single call, replays
    included, and decompresses to the single call's values."""
    meshes, grids, fields, plans, xs = workload
    cplans = [M.Plan(dev(m.coords), None, dims=g[:2] if g[2] == 1 else g, operators="cluster")
              for m, g in zip(meshes, grids)]
    items, singles, codes = [], [], []
    for i, f in enumerate(fields):
        kind = i % 3
        if kind == 0:
            c = M.Codes(plans[f["mesh"]], xs[i].dtype, residual_predictor="delta")
            items.append((plans[f["mesh"]], xs[i], f["eb"], f["eb_mode"], f["split"], None, c))
            singles.append(lambda i=i, f=f: M.compress(
                plans[f["mesh"]], xs[i], f["eb"], f["eb_mode"], f["split"],
                codes=M.Codes(plans[f["mesh"]], xs[i].dtype, residual_predictor="delta")))
        elif kind == 1:
            c = M.Codes(cplans[f["mesh"]], xs[i].dtype)
            items.append((cplans[f["mesh"]], xs[i], f["eb"], f["eb_mode"], f["split"], None, c, "sum", "open"))
            singles.append(lambda i=i, f=f: M.compress(cplans[f["mesh"]], xs[i], f["eb"], f["eb_mode"], f["split"],
                                                       residual="open"))
        else:
            c = M.Codes(plans[f["mesh"]], xs[i].dtype)
            items.append((plans[f["mesh"]], xs[i], f["eb"], f["eb_mode"], f["split"], None, c))
            singles.append(lambda i=i, f=f: M.compress(plans[f["mesh"]], xs[i], f["eb"], f["eb_mode"], f["split"]))
        codes.append(c)
    for rep in range(3):                                   # capture, then replays
        for c in codes:
            c.vert_codes.zero_()
        M.batch_compress(items)
        torch.cuda.synchronize()
        for i, c in enumerate(codes):
            ref = singles[i]()
            same(c.host(), ref.host())
            assert c.result_host()["status"] == 0
            plan = items[i][0]
            a, b = M.decompress(plan, c), M.decompress(plan, ref)
            torch.cuda.synchronize()
            assert torch.equal(a, b)
    for p in cplans:
        p.destroy()


def test_batch_grid_predictors(workload):
    """One graph over items whose grid codes use the interpolation (linear,
    cubic) and time-axis predictors, and the inverse graph: every item
    equals its single call over replays, and the batch decompress equals
    the single decompress."""
    meshes, grids, fields, plans, xs = workload
    refs = {}
    items, ditems, singles, codes, outs = [], [], [], [], []
    kinds = ("cubic", "linear", "temporal")
    for i, f in enumerate(fields):
        plan = plans[f["mesh"]]
        gp = kinds[i % 3]
        kw = {}
        if gp == "temporal":
            if f["mesh"] not in refs:              # the reference grid: x1' of another field on the mesh
                r = torch.empty(plan.n_grid, dtype=torch.float32, device="cuda")
                M.compress(plan, xs[i], f["eb"], f["eb_mode"], f["split"], codes=M.Codes(plan, xs[i].dtype,
                                                                                            xhat_out=r))
                refs[f["mesh"]] = r
            kw = dict(grid_ref=refs[f["mesh"]])
        c = M.Codes(plan, xs[i].dtype, grid_predictor=gp, **kw)
        items.append((plan, xs[i], f["eb"], f["eb_mode"], f["split"], None, c))
        outs.append(torch.empty_like(xs[i]))
        ditems.append((plan, c, None, outs[-1]))
        singles.append(lambda i=i, f=f, gp=gp, kw=kw: M.compress(
            plans[f["mesh"]], xs[i], f["eb"], f["eb_mode"], f["split"],
            codes=M.Codes(plans[f["mesh"]], xs[i].dtype, grid_predictor=gp, **kw)))
        codes.append(c)
    print(f"[batch] grid predictors over {len(items)} items", flush=True)
    for rep in range(3):                                   # capture, then replays
        for c, o in zip(codes, outs):
            c.grid_codes.zero_()
            o.zero_()
        M.batch_compress(items)
        M.batch_decompress(ditems)
        torch.cuda.synchronize()
        for i, c in enumerate(codes):
            ref = singles[i]()
            same(c.host(), ref.host())
            assert c.result_host()["status"] == 0
            b = M.decompress(items[i][0], ref)
            torch.cuda.synchronize()
            assert torch.equal(outs[i], b), (rep, i)


def test_plain_items_take_the_work_list(workload):
    """Plain Lorenzo items of both dimensions and value types, several per
    mesh, go through the work-list stage launches (one launch per stage for
    all of them: a handful of graph nodes instead of a chain per item), and
    every item still equals its single call, over replays, both ways."""
    meshes, grids, fields, plans, xs = workload
    codes = [M.Codes(plans[f["mesh"]], xs[i].dtype) for i, f in enumerate(fields)]
    items = _items(fields, plans, xs, codes)
    outs = [torch.empty_like(x) for x in xs]
    ditems = [(plans[f["mesh"]], codes[i], None, outs[i]) for i, f in enumerate(fields)]
    for rep in range(3):
        for c, o in zip(codes, outs):
            c.vert_codes.zero_()
            o.fill_(3.0)
        M.batch_compress(items)
        M.batch_decompress(ditems)
        torch.cuda.synchronize()
        for i, f in enumerate(fields):
            ref = M.compress(plans[f["mesh"]], xs[i], f["eb"], f["eb_mode"], f["split"])
            same(codes[i].host(), ref.host())
            b = M.decompress(plans[f["mesh"]], ref)
            torch.cuda.synchronize()
            assert torch.equal(outs[i].view(torch.uint8), b.view(torch.uint8)), (rep, i)
    ic = M.batch_graph_info(items)
    idc = M.batch_graph_info(ditems, decompress=True)
    print(f"[batch] work list: compress {ic}, decompress {idc}")
    assert ic["n_batched"] == len(items) and idc["n_batched"] == len(items)
    assert ic["n_nodes"] <= 8            # five stage launches (plus capture bookkeeping)
    kinds = {(m.dim, np.dtype(f["data"].dtype).itemsize) for f, m in ((f, meshes[f["mesh"]]) for f in fields)}
    assert len(kinds) >= 2


def test_batch_scale_005_every_field_against_the_oracle():
    """The 12-mesh, 64-field batch at 5 % of its size (25K-1M vertices per
    mesh, 2-D and 3-D, FP32 and FP64, eb 1e-3..1e-5): one batch compress and
    one batch decompress, then every field's grid and vertex codes, outlier
    lists and decoded values against the oracle, element by element."""
    meshes, grids, fields = G.config_batch(seed=5, scale=0.05)
    print(f"[batch] scale 0.05: {len(meshes)} meshes, nv {[m.n_vertices for m in meshes]}, {len(fields)} fields",
          flush=True)
    plans = [M.Plan(dev(m.coords), dev(m.cells), dims=g[:2] if g[2] == 1 else g) for m, g in zip(meshes, grids)]
    xs = [dev(f["data"]) for f in fields]
    codes = [M.Codes(plans[f["mesh"]], xs[i].dtype) for i, f in enumerate(fields)]
    outs = [torch.empty_like(x) for x in xs]
    items = _items(fields, plans, xs, codes)
    M.batch_compress(items)
    M.batch_decompress([(plans[f["mesh"]], codes[i], None, outs[i]) for i, f in enumerate(fields)])
    torch.cuda.synchronize()
    assert M.batch_graph_info(items)["n_batched"] == len(fields)
    maps = {}
    for i, f in enumerate(fields):
        m = f["mesh"]
        mesh = meshes[m]
        g = grids[m][:2] if grids[m][2] == 1 else grids[m]
        if m not in maps:
            og = O.grid_from_dims(mesh.coords, g)
            maps[m] = (og, O.locate(mesh.coords, mesh.cells, og, "raster", fill="nearest", fill_method="kdtree"))
        og, om = maps[m]
        oc = O.compress(mesh.coords, om, og, f["data"], f["eb"], True, f["split"])
        h = codes[i].host()
        assert h["result"]["status"] == 0
        assert np.array_equal(h["grid_codes"], oc.grid.codes), i
        assert np.array_equal(h["g_out_idx"], oc.grid.out_idx), i
        assert np.array_equal(h["g_out_delta"], oc.grid.out_delta), i
        assert np.array_equal(h["vert_codes"], oc.vert.codes), i
        assert np.array_equal(h["v_out_idx"], oc.vert.out_idx), i
        assert np.array_equal(h["v_out_val"].view(np.uint8), oc.vert.out_val.view(np.uint8)), i
        xo = O.decompress(mesh.coords, og, oc.bound, oc.grid, oc.vert, f["data"].dtype)
        assert np.array_equal(outs[i].cpu().numpy().view(np.uint8), xo.view(np.uint8)), i
    print(f"[batch] scale 0.05: all {len(fields)} fields equal to the oracle", flush=True)
    for p in plans:
        p.destroy()
