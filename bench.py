#!/usr/bin/env python3
"""Throughput benchmark of the multi-component mesh compressor on one MI355X.

A step is one pass of the whole hot path over one field: compress (range,
resample + prequantise, Lorenzo codes, back-interpolation + residual codes)
then decompress (grid decode, vertex decode).  The default workload is the
16M-vertex tetrahedral mesh: a 252^3 jittered lattice with 6 Kuhn tets per
cube, a float32 three-octave field, a 256^3 grid, relative eb 1e-4 and a
50/50 split.  ``value`` is GB/s of mesh values (n_v * 4 bytes) per step.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBPS = 8000.0


def alg_bytes(kernel: str, nv: int, ng: int, D: int, sT: int) -> int:
    """Compulsory HBM bytes of one launch of each kernel (outliers ignored):
    each array the kernel must read or write, once."""
    table = {
        "k_range": nv * sT,                                        # field
        "k_resample": ng * (D + 1) * 8 + nv * sT + ng * 4,         # mapping, field gather, one grid array out
        "k_lorenzo": ng * 4 + ng * 2,                              # p in, codes out
        "k_codes": ng * 4 + ng * 2 + nv * (4 * D + sT + 2) + ng * 4,   # k_lorenzo + k_residual in one launch
        "k_residual": nv * (4 * D + sT + 2) + ng * 4,              # coords, field, codes out, grid (p or x1')
        "k_mlp_residual": nv * (4 * D + sT + 2) + ng * 4,           # as k_residual; shifts stay on chip
        "k_dec_xy_tot": ng * 2,                                    # 2-D: codes
        "k_dec_z_tot": ng * 2,                                     # 3-D: codes
        "k_dec_z_apply": ng * 2 + ng * 4,                          # codes in, z-prefixed errors out
        "k_dec3_tot": ng * 2,                                      # 3-D quads: codes
        "k_dec3_apply": ng * 2 + ng * 4,                           # 3-D quads: codes in, x1' out
        "k_dec_xy_apply": (ng * 4 if D == 3 else ng * 2) + ng * 4,  # errors in, x1' out
        "k_vdecode": nv * (4 * D + 2 + sT) + ng * 4,               # coords, codes, field out, x1'
        "k_mlp_vdecode": nv * (4 * D + 2 + sT) + ng * 4,            # as k_vdecode; shifts stay on chip
    }
    return table.get(kernel, 0)


COMPRESS_PREFIXES = ("k_range", "k_resample", "k_lorenzo", "k_residual", "k_codes",
                     "k_scatter", "k_mlp_residual")
DECOMPRESS_PREFIXES = ("k_dec_", "k_dec3_", "k_vdecode", "k_mlp_vdecode")


def _kernel_source(here: str, kernel: str):
    """The csrc file that defines `kernel` (its __global__ declaration)."""
    import glob
    import re
    pat = re.compile(r"__global__[^;{]*?\b" + re.escape(kernel) + r"\s*\(")
    for p in sorted(glob.glob(os.path.join(here, "paper_2501_06910_amd", "csrc", "*.hip"))):
        if pat.search(open(p).read()):
            return p
    return None


def pmc_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter runs, or
    None when the file defining the kernel (or the shared device header)
    changed since they were taken."""
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(here, "profiles", "tet3d_16M_pmc_traffic.json")
    src = _kernel_source(here, kernel)
    if not os.path.exists(path) or src is None:
        return None
    rec = json.load(open(path))
    shas = rec.get("source_sha256", {})
    for p in (src, os.path.join(here, "paper_2501_06910_amd", "csrc", "mc_dev.h")):
        name = os.path.basename(p)
        if hashlib.sha256(open(p, "rb").read()).hexdigest() != shas.get(name):
            return None
    for name, v in rec["kernels"].items():
        if name.split("<")[0] == kernel:
            return v["traffic_bytes"]
    return None


def method_bytes(nv: int, ng: int, D: int, sT: int):
    """Algorithmic bytes of compress and decompress with the plan cached."""
    bc = nv * sT + ng * 8 * (D + 1) + nv * sT + ng * 6 + nv * 4 * D + nv * sT + ng * 4 + nv * 2
    bd = ng * 2 + ng * 8 + nv * (4 * D + 2 + sT)
    return bc, bd


def workload(name: str):
    import meshgen as G
    if name == "tet3d":
        mesh, f, cfg = G.config_tet_3d()
        desc = ("tet3d: 252^3 jittered lattice (+-20% of the spacing), 6 Kuhn tetrahedra per cube "
                "(16,003,008 vertices, 94,879,506 tets); float32 three-octave sinusoid field; "
                "256^3 grid; relative eb 1e-4; grid share 0.5")
    elif name == "tet3d_small":
        mesh, f, cfg = G.config_tet_3d(n=64, dims=65)
        desc = "tet3d_small: 64^3 jittered Kuhn lattice, float32 field, 65^3 grid, relative eb 1e-4"
    else:
        raise SystemExit(f"unknown workload {name}")
    return mesh, f, cfg, desc


def host_description() -> dict:
    """nproc and the CPU model of the host the oracle runs on."""
    model = None
    try:
        import subprocess
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for ln in out.splitlines():
            if ln.startswith("Model name:"):
                model = ln.split(":", 1)[1].strip()
                break
    except Exception:
        pass
    return {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)), "cpu_model": model}


def cpu_baseline(mesh, f, cfg, eb: float, split: float, h_gpu=None, x_gpu=None, reps: int = 5):
    """The oracle as it stands (plain C, one thread) on the same inputs as
    the timed step: the mapping is computed first and not timed (the paper
    excludes the mapping from its cost), then compress + decompress are
    timed, median of `reps`.  When the GPU's codes and decoded values are
    given they must equal the oracle's, element by element."""
    import oracle as O
    t0 = time.perf_counter()
    g = O.grid_from_dims(mesh.coords, cfg["dims"][:mesh.dim])
    m = O.locate(mesh.coords, mesh.cells, g, "raster", fill="nearest", fill_method="kdtree")
    plan_s = time.perf_counter() - t0
    tc, td = [], []
    for _ in range(reps):
        t0 = time.perf_counter()
        cz = O.compress(mesh.coords, m, g, f, eb, True, split)
        t1 = time.perf_counter()
        xo = O.decompress(mesh.coords, g, cz.bound, cz.grid, cz.vert, f.dtype)
        t2 = time.perf_counter()
        tc.append(t1 - t0)
        td.append(t2 - t1)
    same = None
    if h_gpu is not None:
        same = bool(np.array_equal(h_gpu["grid_codes"], cz.grid.codes)
                    and np.array_equal(h_gpu["g_out_idx"], cz.grid.out_idx)
                    and np.array_equal(h_gpu["vert_codes"], cz.vert.codes)
                    and np.array_equal(h_gpu["v_out_idx"], cz.vert.out_idx)
                    and (x_gpu is None or np.array_equal(x_gpu.view(np.uint8), xo.view(np.uint8))))
    c, d = float(np.median(tc)), float(np.median(td))
    nb = mesh.n_vertices * f.dtype.itemsize
    return {"value": round(nb / (c + d) / 1e9, 4), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": f"the timed workload itself ({mesh.n_vertices} vertices, {mesh.n_cells} cells, grid "
                      f"{'x'.join(str(int(v)) for v in cfg['dims'][:mesh.dim])}), mapping untimed "
                      f"({plan_s:.1f} s); compress + decompress, median of {reps}, one thread",
            "compress_s": round(c, 4), "decompress_s": round(d, 4),
            "compress_GBps": round(nb / c / 1e9, 4), "decompress_GBps": round(nb / d / 1e9, 4),
            "codes_equal_gpu": same, "host": host_description()}


def cold_step_ms(step, reps: int = 20, flush_bytes: int = 1 << 30):
    """Median milliseconds of one step after writing a flush_bytes scratch
    buffer (evicts the 4 MB L2 of every XCD and the 256 MB Infinity
    Cache), HIP events on the current stream around the step only."""
    import torch
    scratch = torch.empty(flush_bytes // 4, dtype=torch.float32, device="cuda")
    ts = []
    for i in range(reps):
        scratch.fill_(float(i))
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        step()
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    del scratch
    return float(np.median(ts))


def copy_ceiling_gbps(nbytes: int = 1 << 30, reps: int = 10) -> float:
    """HBM rate of a plain device-to-device copy (read + write bytes per
    second), the practical ceiling the kernels are also compared with."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    return 2 * nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9


def _timed(fn, reps=5):
    """Mean device milliseconds of fn() over reps back-to-back calls after
    one untimed call, HIP events on the current stream around the reps (an
    event pair around each single call would also count the launch latency
    of the call's first kernel)."""
    import torch
    fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def serial_compare(M, x, eb, h_mc, ms_mc, log, label, shuffle_seed=None):
    """The Sec. V-C comparison on one field: the 1-D serialisation baseline
    (vertex order as generated, or a seeded random order) against the
    multi-component result h_mc (host codes of the same field).  Improvement
    ratio = CR_mc / CR_serial; overhead = (T_mc - T_serial) / T_serial per
    direction, device times.  Renumbering the vertices permutes the
    multi-component vertex codes (same Huffman size) and renumbers its
    outliers, so its CR under the permutation is recomputed exactly from
    h_mc."""
    import torch
    nv, sT = x.numel(), x.element_size()
    h_mc = dict(h_mc)
    if shuffle_seed is not None:
        g = torch.Generator(device="cpu").manual_seed(shuffle_seed)
        perm = torch.randperm(nv, generator=g)
        inv = torch.empty_like(perm)
        inv[perm] = torch.arange(nv)
        x = x[perm.cuda()].contiguous()
        h_mc["v_out_idx"] = np.sort(inv.numpy()[h_mc["v_out_idx"]])
    cr_mc = nv * sT / M.stream_bytes(h_mc, sT)["total"]
    ctx = M.Serial(nv)
    codes = M.SerialCodes(nv, x.dtype)
    out = torch.empty_like(x)
    tc = _timed(lambda: M.serial_compress(ctx, x, eb, "rel", codes=codes))
    td = _timed(lambda: M.serial_decompress(ctx, codes, out=out))
    h = codes.host()
    r = h["result"]
    if r["status"]:
        raise SystemExit(f"serial baseline ({label}): status {r['status']}")
    err = (x.double() - out.double()).abs().max().item()
    if not err <= r["tau"]:
        raise SystemExit(f"serial baseline ({label}): bound violated")
    sb = M.serial_stream_bytes(h, sT)
    cr = nv * sT / sb["total"]
    M.profile_reset()
    M.profile_enable(True)
    for _ in range(5):
        M.serial_compress(ctx, x, eb, "rel", codes=codes)
        M.serial_decompress(ctx, codes, out=out)
    torch.cuda.synchronize()
    M.profile_enable(False)
    kern = {k: round(t / c, 5) for k, (c, t) in M.profile_read().items()}
    row = {"order": "seeded random permutation" if shuffle_seed is not None else "as generated",
           "cr_serial": round(cr, 3), "cr_mc": round(cr_mc, 3), "improvement_ratio": round(cr_mc / cr, 3),
           "raw_values": r["n_vertex_outliers"],
           "serial_GBps": {"compress": round(nv * sT / (tc * 1e-3) / 1e9, 2),
                           "decompress": round(nv * sT / (td * 1e-3) / 1e9, 2)},
           "overhead": {"compress": round((ms_mc[0] - tc) / tc, 3), "decompress": round((ms_mc[1] - td) / td, 3)},
           "kernels_avg_ms": kern}
    log(f"serial baseline {label}: {row}")
    ctx.destroy()
    return row


def design_point(M, mesh, coords, x, eb, log, dims=128, split=4.0, split_mode="full", operators="linear",
                 residual="closed", predictor="none", grid_predictor="lorenzo", coarsen=False):
    """The same field at another setting of the CR sweep (default: the
    best one, a 128^3 grid, one node per ~8 vertices, with the full split
    tau2 = tau and the grid step from tau1 = 4 tau): CR, both directions'
    GB/s, the improvement over the 1-D baseline and the kernel times."""
    import torch
    nv, sT = x.numel(), x.element_size()
    cells = torch.from_numpy(mesh.cells).cuda() if operators == "linear" else None
    plan = M.Plan(coords, cells, dims=(dims, dims, dims), operators=operators, coarsen=coarsen)
    del cells
    codes = M.Codes(plan, x.dtype, residual_predictor=predictor, grid_predictor=grid_predictor)
    out = torch.empty_like(x)
    kw = dict(split_mode=split_mode, residual=residual)
    M.compress(plan, x, eb, "rel", split, codes=codes, **kw)
    M.decompress(plan, codes, out=out)
    h = codes.host()
    r = h["result"]
    err = (x.double() - out.double()).abs().max().item()
    bound = r["tau"] if residual == "open" else r["tau2"]
    if r["status"] or not err <= bound:
        raise SystemExit(f"design point: status {r['status']}, max error {err} vs {bound}")
    tc = _timed(lambda: M.compress(plan, x, eb, "rel", split, codes=codes, **kw))
    td = _timed(lambda: M.decompress(plan, codes, out=out))
    M.profile_reset()
    M.profile_enable(True)
    for _ in range(5):
        M.compress(plan, x, eb, "rel", split, codes=codes, **kw)
        M.decompress(plan, codes, out=out)
    torch.cuda.synchronize()
    M.profile_enable(False)
    kern = {k: round(t / c, 5) for k, (c, t) in M.profile_read().items()}
    sb = M.stream_bytes(h, sT)
    ser = serial_compare(M, x, eb, h, (tc, td), log, f"{operators} {dims}^3, generated order")
    row = {"operators": operators, "grid": [dims] * 3, "coarsened_grid": list(plan.grid.dims) if coarsen else None,
           "split_mode": split_mode, "grid_share": split,
           "residual": residual, "residual_predictor": predictor, "grid_predictor": grid_predictor,
           "cr": round(nv * sT / sb["total"], 3),
           "max_abs_err_over_tau": round(err / r["tau"], 4),
           "compress_GBps": round(nv * sT / (tc * 1e-3) / 1e9, 2),
           "decompress_GBps": round(nv * sT / (td * 1e-3) / 1e9, 2),
           "ms_per_step": round(tc + td, 4), "stream_bytes": sb,
           "improvement_vs_serial": ser["improvement_ratio"], "cr_serial": ser["cr_serial"],
           "kernels_avg_ms": kern}
    log(f"design point: {row}")
    plan.destroy()
    return row


def mlp_flops_per_vertex(D: int) -> int:
    """Multiply-adds of one inference (x2): K_in -> 64 -> 64 -> 64 -> 1 with
    K_in = 4^D + D, the zero padding not counted."""
    kin = 4 ** D + D
    return 2 * (kin * 64 + 64 * 64 * 2 + 64)


def learned_design_point(M, mesh, series, cfg, serial_bytes, log, dims=512, split=1.0, split_mode="full",
                         train_steps=2000, batch=8192):
    """The rotating series at a coarser grid (512^2: one node per ~16
    vertices) with the full split: plain and learned CR over t = 1..8 (the
    model charged once), both forms' GB/s and the gain over the 1-D
    baseline (serial_bytes: its total stream bytes over the same steps)."""
    import torch
    nv, sT = mesh.n_vertices, series[0].dtype.itemsize
    plan = M.Plan(torch.from_numpy(mesh.coords).cuda(), torch.from_numpy(mesh.cells).cuda(), dims=(dims, dims))
    xs = [torch.from_numpy(a).cuda() for a in series]
    model = M.Model.train(plan, xs[0], eb=cfg["eb"], grid_share=split, split_mode=split_mode, steps=train_steps,
                          batch=batch, seed=4)
    model_bytes = len(model.export())                 # the model file as embedded in the stream
    cp, cl = M.Codes(plan, xs[0].dtype), M.Codes(plan, xs[0].dtype, learned=True)
    out = torch.empty_like(xs[0])
    tot = {"plain": 0, "learned": 0}
    times = {"plain_c": [], "plain_d": [], "learned_c": [], "learned_d": []}
    kw = dict(split_mode=split_mode)
    for t in range(1, len(series)):
        x = xs[t]
        times["plain_c"].append(_timed(lambda: M.compress(plan, x, cfg["eb"], "rel", split, codes=cp, **kw)))
        times["plain_d"].append(_timed(lambda: M.decompress(plan, cp, out=out)))
        ep = (x.double() - out.double()).abs().max().item()
        times["learned_c"].append(_timed(lambda: M.compress(plan, x, cfg["eb"], "rel", split, model=model, codes=cl,
                                                            **kw)))
        times["learned_d"].append(_timed(lambda: M.decompress(plan, cl, model=model, out=out)))
        el = (x.double() - out.double()).abs().max().item()
        hp, hl = cp.host(), cl.host()
        hl["learned"] = True
        tau2 = hp["result"]["tau2"]
        if hp["result"]["status"] or hl["result"]["status"] or not (ep <= tau2 and el <= tau2):
            raise SystemExit(f"learned design point: status or bound failure at t={t}")
        tot["plain"] += M.stream_bytes(hp, sT)["total"]
        tot["learned"] += M.stream_bytes(hl, sT)["total"]
    raw = nv * sT * (len(series) - 1)
    med = {k: float(np.median(v)) for k, v in times.items()}
    row = {"grid": [dims, dims], "split_mode": split_mode, "grid_share": split,
           "cr_plain": round(raw / tot["plain"], 3), "cr_learned": round(raw / (tot["learned"] + model_bytes), 3),
           "improvement_vs_serial": {"plain": round(serial_bytes / tot["plain"], 3),
                                     "learned": round(serial_bytes / (tot["learned"] + model_bytes), 3)},
           "plain_GBps": {"compress": round(nv * sT / (med["plain_c"] * 1e-3) / 1e9, 2),
                          "decompress": round(nv * sT / (med["plain_d"] * 1e-3) / 1e9, 2)},
           "learned_GBps": {"compress": round(nv * sT / (med["learned_c"] * 1e-3) / 1e9, 2),
                            "decompress": round(nv * sT / (med["learned_d"] * 1e-3) / 1e9, 2)}}
    log(f"learned design point: {row}")
    model.destroy()
    plan.destroy()
    return row


def large2d_plain(M, plan, mesh, log) -> dict:
    """The large 2-D configuration (the refined annulus mesh, its own
    float64 tanh front plus Fourier noise field, 2048^2 grid, split 0.5),
    plain path at relative eb 1e-4 and 1e-6: CR from the written stream and
    both directions' GB/s (back-to-back means)."""
    import torch
    import meshgen as G
    x = torch.from_numpy(G.field_large_2d(mesh.coords)).cuda()
    nv, sT = mesh.n_vertices, x.element_size()
    rows = []
    for eb in (1e-4, 1e-6):
        codes = M.Codes(plan, x.dtype)
        out = torch.empty_like(x)
        M.compress(plan, x, eb, "rel", 0.5, codes=codes)
        M.decompress(plan, codes, out=out)
        torch.cuda.synchronize()
        h = codes.host()
        r = h["result"]
        if r["status"]:
            raise SystemExit(f"large2d eb={eb}: status {r['status']}")
        err = (x - out).abs().max().item()
        if not err <= r["tau2"]:
            raise SystemExit(f"large2d eb={eb}: bound violated")
        sb = M.stream_bytes(h, sT)
        tc = _timed(lambda: M.compress(plan, x, eb, "rel", 0.5, codes=codes))
        td = _timed(lambda: M.decompress(plan, codes, out=out))
        rows.append({"eb": eb, "cr": round(nv * sT / sb["total"], 3),
                     "compress_GBps": round(nv * sT / (tc * 1e-3) / 1e9, 2),
                     "decompress_GBps": round(nv * sT / (td * 1e-3) / 1e9, 2),
                     "ms_per_step": round(tc + td, 4),
                     "outliers": {"grid": r["n_grid_outliers"], "vertex": r["n_vertex_outliers"]},
                     "max_abs_err_over_tau": round(err / r["tau"], 4)})
        log(f"large2d: {rows[-1]}")
    return {"workload": f"refined-annulus Delaunay mesh ({nv} vertices), float64 tanh front + Fourier noise, "
                        f"grid 2048^2, relative eb 1e-4 and 1e-6, split 0.5, plain path",
            "results": rows}


def learned_section(log, train_steps=2000, batch=8192):
    """Learned vs plain on the rotating-front time series over the refined
    2-D mesh: train on t=0, compress t=1..8 both ways at eb 1e-4; CR with the
    BF16 model charged once to the sequence; both forms' GB/s.  The plain
    codes are also coded with the time-axis grid predictor against the
    previous step's x1' (the same vertex stream, other grid codes)."""
    import torch
    import meshgen as G
    from paper_2501_06910_amd import mc as M
    t0 = time.time()
    mesh, series, cfg = G.config_learned_series()
    log(f"learned: series generated in {time.time() - t0:.1f} s (nv={mesh.n_vertices}, {len(series)} steps)")
    D, nv = mesh.dim, mesh.n_vertices
    sT = series[0].dtype.itemsize
    plan = M.Plan(torch.from_numpy(mesh.coords).cuda(), torch.from_numpy(mesh.cells).cuda(), dims=cfg["dims"][:2])
    ng = plan.n_grid
    x0 = torch.from_numpy(series[0]).cuda()
    torch.cuda.synchronize()
    M.profile_reset()
    M.profile_enable(True)
    t0 = time.time()
    model, loss = M.Model.train(plan, x0, eb=cfg["eb"], steps=train_steps, batch=batch, seed=4, return_loss=True)
    torch.cuda.synchronize()
    train_s = time.time() - t0
    M.profile_enable(False)
    tprof = M.profile_read()
    log(f"learned: trained {train_steps} steps x {batch} in {train_s:.2f} s, loss {loss[0]:.4f} -> "
        f"{float(np.mean(loss[-50:])):.4f}")
    model_bytes = len(model.export())                # the model file as embedded once in the sequence's stream
    nT = len(series) - 1
    per_t = []
    # x1' of the previous and the current step for the time-axis grid predictor
    prev = torch.empty(ng, dtype=torch.float32, device="cuda")
    cur = torch.empty(ng, dtype=torch.float32, device="cuda")
    M.compress(plan, x0, cfg["eb"], "rel", 0.5, codes=M.Codes(plan, x0.dtype, xhat_out=prev))
    cp, cl = M.Codes(plan, x0.dtype, xhat_out=cur), M.Codes(plan, x0.dtype, learned=True)
    ct = M.Codes(plan, x0.dtype, grid_predictor="temporal", grid_ref=prev)
    out = torch.empty_like(x0)
    tot = {"plain": 0, "learned": 0, "raw": 0, "serial": 0, "temporal": 0}
    times = {"plain_c": [], "plain_d": [], "learned_c": [], "learned_d": [], "temporal_c": [], "temporal_d": []}
    sctx, scodes = M.Serial(nv), M.SerialCodes(nv, x0.dtype)
    for t in range(1, len(series)):
        x = torch.from_numpy(series[t]).cuda()
        times["plain_c"].append(_timed(lambda: M.compress(plan, x, cfg["eb"], "rel", 0.5, codes=cp)))
        times["plain_d"].append(_timed(lambda: M.decompress(plan, cp, out=out)))
        ep = (x.double() - out.double()).abs().max().item()
        # the time-axis grid predictor against step t - 1's x1' (same vertex stream)
        times["temporal_c"].append(_timed(lambda: M.compress(plan, x, cfg["eb"], "rel", 0.5, codes=ct)))
        times["temporal_d"].append(_timed(lambda: M.decompress(plan, ct, out=out)))
        et = (x.double() - out.double()).abs().max().item()
        hg = ct.host_grid()
        gb_t = M.grid_stream_bytes(hg["grid_codes"], hg["g_out_idx"], hg["g_out_delta"])
        times["learned_c"].append(_timed(lambda: M.compress(plan, x, cfg["eb"], "rel", 0.5, model=model, codes=cl)))
        times["learned_d"].append(_timed(lambda: M.decompress(plan, cl, model=model, out=out)))
        el = (x.double() - out.double()).abs().max().item()
        hp, hl = cp.host(), cl.host()
        hl["learned"] = True
        if hp["result"]["status"] or hl["result"]["status"]:
            raise SystemExit(f"learned section: status {hp['result']['status']} / {hl['result']['status']}")
        tau2 = hp["result"]["tau2"]
        if not (ep <= tau2 and el <= tau2 and et <= tau2) or hg["result"]["status"]:
            raise SystemExit(f"learned section: bound violated or status at t={t}")
        sbp = M.stream_bytes(hp, sT)
        sp = sbp["total"]
        gb_p = sbp["grid"] + sbp["grid_outliers"]
        tot["temporal"] += sp - gb_p + gb_t
        prev.copy_(cur)                                   # x1' of step t: the next step's reference
        sl = M.stream_bytes(hl)["total"]                  # the model is charged once, below
        tot["plain"] += sp
        tot["learned"] += sl
        tot["raw"] += nv * sT
        M.serial_compress(sctx, x, cfg["eb"], "rel", codes=scodes)
        hs = scodes.host()
        if hs["result"]["status"]:
            raise SystemExit(f"learned section: serial baseline status {hs['result']['status']}")
        ss = M.serial_stream_bytes(hs, sT)["total"]
        tot["serial"] += ss
        per_t.append({"t": t, "cr_plain": round(nv * sT / sp, 3), "cr_learned": round(nv * sT / (sl + model_bytes / nT), 3),
                      "cr_serial": round(nv * sT / ss, 3),
                      "cr_temporal_grid": round(nv * sT / (sp - gb_p + gb_t), 3),
                      "grid_bytes": {"lorenzo": gb_p, "temporal": gb_t},
                      "vert_bits_plain": round(M.entropy_bits(hp["vert_codes"]), 3),
                      "vert_bits_learned": round(M.entropy_bits(hl["vert_codes"]), 3),
                      "learned_blocks": hl["result"]["n_learned_blocks"],
                      "blocks": (nv + 4095) // 4096})
        log(f"learned: t={t} {per_t[-1]}")
    med = {k: float(np.median(v)) for k, v in times.items()}
    # the learned vertex-code kernel (the network on every block whose plain
    # codes are not all zero, then the codes): MFMA rate over its whole
    # duration, counting the vertices of the blocks the network runs on
    vc0 = M.compress(plan, x0, cfg["eb"], "rel", 0.5).host()["vert_codes"]
    nblk = (nv + 4095) // 4096
    run_b = [b for b in range(nblk) if not np.all(vc0[b * 4096:(b + 1) * 4096] == 32768)]
    run_v = sum(min(4096, nv - b * 4096) for b in run_b)
    M.profile_reset()
    M.profile_enable(True)
    for _ in range(5):
        M.compress(plan, x0, cfg["eb"], "rel", 0.5, model=model, codes=cl)
    torch.cuda.synchronize()
    M.profile_enable(False)
    iprof = M.profile_read()
    inf = iprof.get("k_mlp_residual")
    inf_ms = inf[1] / inf[0] if inf else None
    fl = mlp_flops_per_vertex(D) * run_v
    tr = tprof.get("k_mlp_train")
    tr_ms = tr[1] / tr[0] if tr else None
    train_fl = 3 * mlp_flops_per_vertex(D) * batch      # forward + two backward products per layer
    return {
        "series": f"refined-annulus Delaunay mesh ({nv} vertices), float64 tanh front + noise rotated about a "
                  f"seeded centre, {len(series)} timesteps, grid {cfg['dims'][0]}^2, relative eb 1e-4, split 0.5",
        "model": f"MLP {4 ** D + D} -> 64 -> 64 -> 64 -> 1 (ReLU), BF16 weights, {M.param_count(D)} parameters, "
                 f"{model_bytes} B in the stream (charged once to the {nT} coded timesteps)",
        "train": {"steps": train_steps, "batch": batch, "seconds": round(train_s, 3),
                  "loss_first": round(float(loss[0]), 5), "loss_last50": round(float(np.mean(loss[-50:])), 5),
                  "k_mlp_train_avg_ms": round(tr_ms, 5) if tr_ms else None,
                  "k_mlp_train_TFLOPs": round(train_fl / (tr_ms * 1e-3) / 1e12, 2) if tr_ms else None},
        "cr_plain": round(tot["raw"] / tot["plain"], 3),
        "cr_learned": round(tot["raw"] / (tot["learned"] + model_bytes), 3),
        "cr_serial": round(tot["raw"] / tot["serial"], 3),
        "cr_temporal_grid": round(tot["raw"] / tot["temporal"], 3),
        "temporal_GBps": {"compress": round(nv * sT / (med["temporal_c"] * 1e-3) / 1e9, 2),
                          "decompress": round(nv * sT / (med["temporal_d"] * 1e-3) / 1e9, 2)},
        "improvement_ratio": {"plain": round(tot["serial"] / tot["plain"], 3),
                              "learned": round(tot["serial"] / (tot["learned"] + model_bytes), 3)},
        "plain_GBps": {"compress": round(nv * sT / (med["plain_c"] * 1e-3) / 1e9, 2),
                       "decompress": round(nv * sT / (med["plain_d"] * 1e-3) / 1e9, 2)},
        "learned_GBps": {"compress": round(nv * sT / (med["learned_c"] * 1e-3) / 1e9, 2),
                         "decompress": round(nv * sT / (med["learned_d"] * 1e-3) / 1e9, 2)},
        "inference": {"kernel": "k_mlp_residual", "avg_ms": round(inf_ms, 5) if inf_ms else None,
                      "flops_per_vertex": mlp_flops_per_vertex(D),
                      "vertices_run": int(run_v), "blocks_skipped": nblk - len(run_b),
                      "TFLOPs": round(fl / (inf_ms * 1e-3) / 1e12, 2) if inf_ms else None,
                      "mfma_peak_bf16_TFLOPs": 2500.0},
        "per_timestep": per_t,
        "n_vertices": nv, "n_grid": ng,
        "design_point": learned_design_point(M, mesh, series, cfg, tot["serial"], log, train_steps=train_steps,
                                             batch=batch),
        "large2d": large2d_plain(M, plan, mesh, log),
    }


SWEEP_SPLITS = (("sum", 0.1), ("sum", 0.3), ("sum", 0.5), ("sum", 0.7), ("sum", 0.9),
                ("full", 0.5), ("full", 1.0), ("full", 2.0), ("full", 4.0))
# the paper's operator pair: open-loop residual with the sum split, or the
# closed loop with the full split
SWEEP_CLUSTER = (("sum", 0.1, "open"), ("sum", 0.5, "open"), ("sum", 0.9, "open"),
                 ("full", 1.0, "closed"), ("full", 4.0, "closed"))


def cr_sweep(log, ebs=(1e-2, 1e-3, 1e-4, 1e-5, 1e-6), grids=(256, 128, 64), splits=SWEEP_SPLITS):
    """CR of the tet3d workload over relative error bounds, grid resolutions
    (the grid spacing hyperparameter of Sec. V-B) and error splits (sum:
    tau1 + tau2 = tau; full: tau2 = tau), next to the 1-D serialisation
    baseline in the generated and in a seeded random vertex order (CPU
    entropy stage).  Improvement ratio = CR_mc / CR_serial.  Every row also
    carries the CR with the interpolation grid predictors (linear, cubic) in
    place of the Lorenzo predictor: the same vertex stream, other grid codes."""
    import torch
    import meshgen as G
    from paper_2501_06910_amd import mc as M
    mesh, f, cfg = G.config_tet_3d()
    nv, sT = mesh.n_vertices, 4
    x = torch.from_numpy(f).cuda()
    xd = x.double()
    norm = torch.linalg.vector_norm(xd).item()
    out = torch.empty_like(x)
    gen = torch.Generator(device="cpu").manual_seed(7)
    perm = torch.randperm(nv, generator=gen)
    inv = torch.empty_like(perm)
    inv[perm] = torch.arange(nv)
    inv = inv.numpy()
    xs = x[perm.cuda()].contiguous()
    sctx, scodes = M.Serial(nv), M.SerialCodes(nv, x.dtype)
    serial = {}
    for eb in ebs:
        row = {}
        for name, xx in (("generated", x), ("random", xs)):
            M.serial_compress(sctx, xx, eb, "rel", codes=scodes)
            hs = scodes.host()
            row[name] = round(nv * sT / M.serial_stream_bytes(hs, sT)["total"], 3) if not hs["result"]["status"] \
                else None
        serial[eb] = row
        log(f"cr sweep: serial eb={eb} {row}")
    sctx.destroy()
    del xs
    rows = []
    coords = torch.from_numpy(mesh.coords).cuda()
    cells = torch.from_numpy(mesh.cells).cuda()
    for ops in ("linear", "cluster"):
        for gd in grids:
            plan = M.Plan(coords, cells if ops == "linear" else None, dims=(gd, gd, gd), operators=ops)
            codes = M.Codes(plan, x.dtype)
            deltas = [("full", 1.0, "closed", "delta"), ("full", 4.0, "closed", "delta")]
            settings = ([(m_, sp, "closed", "none") for m_, sp in splits] if ops == "linear"
                        else [st + ("none",) for st in SWEEP_CLUSTER]) + deltas
            codes_d = M.Codes(plan, x.dtype, residual_predictor="delta")
            codes_g = {gp: M.Codes(plan, x.dtype, grid_predictor=gp) for gp in ("linear", "cubic")}
            for eb in ebs:
                gcache = {}        # grid bytes per (tau1, grid predictor): the grid codes depend on nothing else
                for mode, sp, resid, pred in settings:
                    cc = codes_d if pred == "delta" else codes
                    M.compress(plan, x, eb, "rel", sp, codes=cc, split_mode=mode, residual=resid)
                    M.decompress(plan, cc, out=out)
                    h = cc.host()
                    r = h["result"]
                    base = {"operators": ops, "grid": gd, "eb": eb, "split_mode": mode, "split": sp,
                            "residual": resid, "residual_predictor": pred}
                    if r["status"]:
                        rows.append(dict(base, status=r["status"]))
                        continue
                    d = (xd - out.double()).abs()
                    sb = M.stream_bytes(h, sT)
                    hr = dict(h)
                    hr["v_out_idx"] = np.sort(inv[h["v_out_idx"]])
                    cr, crr = nv * sT / sb["total"], nv * sT / M.stream_bytes(hr, sT)["total"]
                    s_gen, s_rnd = serial[eb]["generated"], serial[eb]["random"]
                    # the other grid predictors: same p, x1' and vertex codes, other grid codes
                    other = {}
                    for gp, cg in codes_g.items():
                        key = (r["tau1"], gp)
                        if key not in gcache:
                            M.compress(plan, x, eb, "rel", sp, codes=cg, split_mode=mode, residual=resid)
                            hg = cg.host_grid()
                            if hg["result"]["status"]:
                                gcache[key] = None
                            else:
                                gcache[key] = (M.grid_stream_bytes(hg["grid_codes"], hg["g_out_idx"],
                                                                   hg["g_out_delta"]),
                                               hg["result"]["n_grid_outliers"])
                        if gcache[key] is not None:
                            gb, gout = gcache[key]
                            tot = sb["total"] - sb["grid"] - sb["grid_outliers"] + gb
                            other[gp] = {"cr": round(nv * sT / tot, 3), "grid_bytes": gb,
                                         "grid_outlier_rate": gout / plan.n_grid}
                    rows.append(dict(base, cr=round(cr, 3), bits_per_value=round(8 * sb["total"] / nv, 4),
                                     grid_bytes=sb["grid"] + sb["grid_outliers"], vert_bytes=sb["vert"],
                                     grid_predictors=other,
                                     improvement_vs_serial=round(cr / s_gen, 3) if s_gen else None,
                                     # renumbering changes delta codes: no exact figure from these codes
                                     improvement_vs_serial_random_order=(round(crr / s_rnd, 3)
                                                                         if s_rnd and pred == "none" else None),
                                     grid_outlier_rate=r["n_grid_outliers"] / plan.n_grid,
                                     vertex_outlier_rate=r["n_vertex_outliers"] / nv,
                                     linf_over_tau=round(d.max().item() / r["tau"], 4),
                                     rel_l2=float(torch.linalg.vector_norm(d).item() / norm)))
                    log(f"cr sweep: {rows[-1]}")
            plan.destroy()
            del codes, codes_d, codes_g
    return {"serial": {str(k): v for k, v in serial.items()}, "rows": rows}


def grid_sweep(log, ks=(2.0, 5.0, 10.0, 20.0, 30.0, 40.0, 50.0, 60.0, 70.0, 80.0, 90.0), g_max=512, eb=1e-4):
    """CR of the tet3d field over the grid spacing of the paper's grid
    initialisation (Alg. 1: the k-th percentile of the cells' edge extents,
    G_max nodes per axis at most), the analogue of the spacing study of
    Sec. V-B: per k, the grid, its build time, and the CR of the linear pair
    (sum split 0.5 and full split 4.0) and of the paper's pair (open loop,
    tau1 = 0.1 tau), next to the 1-D baseline."""
    import torch
    import meshgen as G
    from paper_2501_06910_amd import mc as M
    mesh, f, cfg = G.config_tet_3d()
    nv, sT = mesh.n_vertices, 4
    x = torch.from_numpy(f).cuda()
    coords = torch.from_numpy(mesh.coords).cuda()
    cells = torch.from_numpy(mesh.cells).cuda()
    sctx, sc = M.Serial(nv), M.SerialCodes(nv, x.dtype)
    M.serial_compress(sctx, x, eb, "rel", codes=sc)
    cr_serial = nv * sT / M.serial_stream_bytes(sc.host(), sT)["total"]
    sctx.destroy()
    out = torch.empty_like(x)
    rows = []
    for k in ks:
        torch.cuda.synchronize()
        t0 = time.time()
        g, ku = M.grid_from_percentile(coords, cells, k, g_max)
        torch.cuda.synchronize()
        t_init = time.time() - t0
        dims = [int(g.dims[d]) for d in range(3)]
        row = {"k": k, "k_used": ku, "dims": dims, "spacing": [g.spacing[d] for d in range(3)],
               "grid_init_seconds": round(t_init, 4), "cr_serial": round(cr_serial, 3)}
        for ops, mode, share, resid in (("linear", "sum", 0.5, "closed"), ("linear", "full", 4.0, "closed"),
                                        ("cluster", "sum", 0.1, "open")):
            plan = M.Plan(coords, cells if ops == "linear" else None, grid=g, operators=ops)
            codes = M.Codes(plan, x.dtype)
            M.compress(plan, x, eb, "rel", share, codes=codes, split_mode=mode, residual=resid)
            M.decompress(plan, codes, out=out)
            h = codes.host()
            r = h["result"]
            bound = r["tau"] if resid == "open" else r["tau2"]
            if r["status"] or not (x.double() - out.double()).abs().max().item() <= bound:
                raise SystemExit(f"grid sweep: failure at k={k} {ops} {mode}")
            cr = nv * sT / M.stream_bytes(h, sT)["total"]
            row[f"cr_{ops}_{mode}_{share}"] = round(cr, 3)
            row[f"improvement_{ops}_{mode}_{share}"] = round(cr / cr_serial, 3)
            plan.destroy()
            del codes
        log(f"grid sweep: {row}")
        rows.append(row)
    return {"g_max": g_max, "eb": eb, "rows": rows}


def batch_section(args, log) -> dict:
    """Many fields on many meshes: 12 meshes of 0.5M..20M vertices (2-D and
    3-D, float32 and float64), 64 fields; a step is one batch compress and
    one batch decompress, each a single HIP graph launch.  Measured plain and
    with the learned predictor per block (one model per mesh, trained on its
    first field)."""
    import torch
    import meshgen as G
    from paper_2501_06910_amd import mc as M
    t0 = time.time()
    meshes, grids, fields = G.config_batch(scale=args.batch_scale, log=lambda m: log(f"batch: {m}"))
    log(f"batch: generated {len(meshes)} meshes / {len(fields)} fields in {time.time() - t0:.1f} s")
    plans = []
    t0 = time.time()
    for m, g in zip(meshes, grids):
        c, k = torch.from_numpy(m.coords).cuda(), torch.from_numpy(m.cells).cuda()
        plans.append(M.Plan(c, k, dims=g[:m.dim]))
        del c, k
    torch.cuda.synchronize()
    plan_s = time.time() - t0
    xs = [torch.from_numpy(f["data"]).cuda() for f in fields]
    outs = [torch.empty_like(x) for x in xs]
    raw = sum(x.numel() * x.element_size() for x in xs)

    def measure(models, tag):
        """One batch compress + one batch decompress per step, each a single
        graph launch; models: per mesh, or None for the plain path."""
        learned = models is not None
        codes = [M.Codes(plans[f["mesh"]], xs[i].dtype, learned=learned) for i, f in enumerate(fields)]
        mod = [models[f["mesh"]] if learned else None for f in fields]
        items = [(plans[f["mesh"]], xs[i], f["eb"], f["eb_mode"], f["split"], mod[i], codes[i])
                 for i, f in enumerate(fields)]
        ditems = [(plans[f["mesh"]], codes[i], mod[i], outs[i]) for i, f in enumerate(fields)]

        def step():
            M.batch_compress(items)
            M.batch_decompress(ditems)

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        worst, total = 0.0, 0
        for i, x in enumerate(xs):
            h = codes[i].host()
            r = h["result"]
            if r["status"]:
                raise SystemExit(f"batch {tag} field {i}: status {r['status']}")
            e = (x.double() - outs[i].double()).abs().max().item()
            if not e <= r["tau2"]:
                raise SystemExit(f"batch {tag} field {i}: bound violated")
            worst = max(worst, e / r["tau"])
            h["learned"] = learned
            total += M.stream_bytes(h, x.element_size())["total"]
        if learned:
            total += sum(len(m.export()) for m in models.values())   # every model file charged once
        for _ in range(args.warmup):        # untimed again after the check's fresh allocations
            step()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record()
        for _ in range(args.steps):
            step()
        ev1.record()
        torch.cuda.synchronize()
        ms_step = ev0.elapsed_time(ev1) / args.steps
        tc = _timed(lambda: M.batch_compress(items))
        td = _timed(lambda: M.batch_decompress(ditems))

        def serial():                      # the same work as separate calls on one stream
            for i, f in enumerate(fields):
                M.compress(plans[f["mesh"]], xs[i], f["eb"], f["eb_mode"], f["split"], model=mod[i], codes=codes[i])
            for i, f in enumerate(fields):
                M.decompress(plans[f["mesh"]], codes[i], model=mod[i], out=outs[i])
        ts = _timed(serial)
        res = {"GBps": round(raw / (ms_step * 1e-3) / 1e9, 2), "ms_per_step": round(ms_step, 4),
               "cr": round(raw / total, 3),
               "compress_GBps": round(raw / (tc * 1e-3) / 1e9, 2),
               "decompress_GBps": round(raw / (td * 1e-3) / 1e9, 2),
               "separate_calls_ms": round(ts, 4), "graph_ms": round(tc + td, 4),
               "max_abs_err_over_tau": round(worst, 4)}
        log(f"batch {tag}: {res}")
        return res

    plain = measure(None, "plain")
    # the learned predictor per block: one model per mesh, trained on its first field
    t0 = time.time()
    models = {}
    for i, f in enumerate(fields):
        if f["mesh"] not in models:
            models[f["mesh"]] = M.Model.train(plans[f["mesh"]], xs[i], eb=f["eb"], eb_mode=f["eb_mode"],
                                              grid_share=f["split"], steps=args.train_steps, seed=4)
    torch.cuda.synchronize()
    train_s = time.time() - t0
    learned = measure(models, "learned")
    learned["train_seconds"] = round(train_s, 3)
    nv_all = [m.n_vertices for m in meshes]
    res = {"workload": f"batch: {len(meshes)} meshes ({min(nv_all)}..{max(nv_all)} vertices, "
                       f"even 2-D jittered triangulations, odd 3-D Kuhn tetrahedra), {len(fields)} fields "
                       f"(float32 on 2-D, float64 on 3-D meshes), relative eb 1e-3/1e-4/1e-5, grids of "
                       f"about n_v/4 nodes, split 0.5, learned predictor per block (one model per mesh)",
           "scale": args.batch_scale, "n_vertices_total": int(sum(x.numel() for x in xs)), "raw_bytes": raw,
           "steps": args.steps, "warmup": args.warmup,
           "learned": learned, "plain": plain, "plan_seconds": round(plan_s, 3)}
    del plans, xs, outs, models
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return res


def batch_main(args, log):
    """The batch workload as the line's workload: ``value`` is the learned
    form's GB/s of mesh values over all fields."""
    b = batch_section(args, log)
    line = {
        "metric": "compress/decompress GB/s of mesh values + CR, learned vs plain, eb=1e-4",
        "value": b["learned"]["GBps"], "unit": "GB/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": b["learned"]["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": b["workload"], "scale": b["scale"], "n_vertices_total": b["n_vertices_total"],
                   "raw_bytes": b["raw_bytes"]},
        "learned": b["learned"],
        "plain": b["plain"],
        "plan_seconds": b["plan_seconds"],
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="tet3d")
    ap.add_argument("--eb", type=float, default=1e-4)
    ap.add_argument("--split", type=float, default=0.5)
    ap.add_argument("--settle", type=float, default=0.5,
                    help="seconds of untimed steps before the warm-up steps (clock ramp under load)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-vs-plain time series section")
    ap.add_argument("--no-batch", action="store_true", help="skip the many-fields batch section")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the 1-D baseline and the design points (profiled runs: only the timed step's kernels)")
    ap.add_argument("--no-tune", action="store_true", help="keep the default launch order (no autotuning)")
    ap.add_argument("--train-steps", type=int, default=2000)
    ap.add_argument("--cr-sweep", action="store_true", help="print the CR sweep over eb and split instead")
    ap.add_argument("--grid-sweep", action="store_true",
                    help="print the CR over the percentile grid spacing of the grid initialisation instead")
    ap.add_argument("--batch-scale", type=float, default=1.0, help="mesh size scale of the batch workload")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (for HBM counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU only; --gpus must be 1 "
                                   "(no multi-GPU decomposition is built)"}))
        sys.exit(2)

    import torch
    from paper_2501_06910_amd import mc as M

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    if args.workload == "batch":
        batch_main(args, log)
        return
    if args.cr_sweep:
        print(json.dumps({"cr_sweep": cr_sweep(log), "workload": "tet3d"}), flush=True)
        return
    if args.grid_sweep:
        print(json.dumps({"grid_sweep": grid_sweep(log), "workload": "tet3d"}), flush=True)
        return

    t0 = time.time()
    mesh, f, cfg, desc = workload(args.workload)
    log(f"workload generated in {time.time() - t0:.1f} s: nv={mesh.n_vertices} nc={mesh.n_cells}")
    D, nv = mesh.dim, mesh.n_vertices
    sT = f.dtype.itemsize
    coords = torch.from_numpy(mesh.coords).cuda()
    cells = torch.from_numpy(mesh.cells).cuda()
    x = torch.from_numpy(f).cuda()
    torch.cuda.synchronize()
    t0 = time.time()
    grid = M.grid_from_dims(coords, cfg["dims"][:D])
    bins = None
    if not args.no_tune:
        b, rec = M.tune_bins(coords, cells, grid)
        bins = {"bin_nodes": b, "timed": rec, "seconds": round(time.time() - t0, 3)}
        log(f"bin edge: {bins}")
        t0 = time.time()
    plan = M.Plan(coords, cells, grid=grid, bin_nodes=bins["bin_nodes"] if bins else 0)
    torch.cuda.synchronize()
    plan_s = time.time() - t0
    del cells
    info = plan.info()
    ng = plan.n_grid
    log(f"plan built in {plan_s:.2f} s: {info}")

    tune = {"remap_mask": plan.remap_mask, "seconds": 0.0, "key": M.tuning_key(plan, x.dtype)}
    if not args.no_tune:
        t0 = time.time()
        tune["cached"] = tune["key"] in M.tuning_cache()
        tune["remap_mask"] = plan.tune(x, args.eb, "rel", args.split, reps=10, cache=True)
        tune["seconds"] = round(time.time() - t0, 3)
        log(f"launch order: remap mask 0x{tune['remap_mask']:02x} "
            f"({'from the tuning cache' if tune['cached'] else 'tuned'}) in {tune['seconds']} s")
    codes = M.Codes(plan, x.dtype)
    out = torch.empty_like(x)

    def step():
        M.compress(plan, x, args.eb, "rel", args.split, codes=codes)
        M.decompress(plan, codes, out=out)

    # the GPU raises its clocks under sustained load over some milliseconds:
    # untimed steps for args.settle seconds first, so that the W warm-up
    # and the K timed steps run at the steady-state clock a continuous
    # compression service sees (the first 20 steps after idle run ~6 % slower)
    t_settle, n_settle = time.time(), 0
    while time.time() - t_settle < args.settle:
        for _ in range(10):
            step()
        torch.cuda.synchronize()
        n_settle += 10
    for _ in range(args.warmup):
        step()

    # timed region: K steps, no per-kernel events, right after the warm-up
    # (the bound check allocates three field-sized FP64 temporaries; the
    # steps that follow such allocations run slower for about a millisecond,
    # so it checks the last timed step instead, after the region)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(args.steps):
        step()
    ev1.record()
    torch.cuda.synchronize()
    ms_step = ev0.elapsed_time(ev1) / args.steps
    log(f"timed {args.steps} steps: {ms_step:.4f} ms/step")
    res = codes.result_host()
    if res["status"] != 0:
        raise SystemExit(f"compress status {res['status']}")
    err = (x.double() - out.double()).abs().max().item()
    if not err <= res["tau2"]:
        raise SystemExit(f"bound violated: {err} > {res['tau2']}")
    log(f"timed steps ok: max |x - x'| = {err:.3e} <= tau2 = {res['tau2']:.3e}")

    # per-kernel durations: HIP events around each launch on its stream
    M.profile_reset()
    M.profile_enable(True)
    ev2, ev3 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev2.record()
    for _ in range(args.steps):
        step()
    ev3.record()
    torch.cuda.synchronize()
    M.profile_enable(False)
    ms_step_ev = ev2.elapsed_time(ev3) / args.steps
    log(f"profiled pass: {ms_step_ev:.4f} ms/step with per-launch events")
    prof = M.profile_read()
    # then each kernel in a pass of its own, events around its launches only
    # (events around every launch lengthen some kernels by up to 15 %)
    iso = {}
    for name in prof:
        M.profile_only(name)
        M.profile_reset()
        M.profile_enable(True)
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        M.profile_enable(False)
        iso[name] = M.profile_read()[name]
    M.profile_only(None)
    kernels = {}
    comp_ms = dec_ms = 0.0
    for name, (cnt, tot) in iso.items():
        avg = tot / cnt
        b = alg_bytes(name, nv, ng, D, sT)
        kernels[name] = {"avg_ms": round(avg, 5), "launches": cnt, "alg_bytes": b,
                         "GBps": round(b / (avg * 1e-3) / 1e9, 1) if b else None,
                         "avg_ms_events_on_all": round(prof[name][1] / prof[name][0], 5)}
        if name.startswith(COMPRESS_PREFIXES):
            comp_ms += avg
        elif name.startswith(DECOMPRESS_PREFIXES):
            dec_ms += avg
    dom = max((k for k in kernels if kernels[k]["alg_bytes"]), key=lambda k: kernels[k]["avg_ms"])
    dk = kernels[dom]
    achieved = dk["alg_bytes"] / (dk["avg_ms"] * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                "traffic": pmc_traffic(dom) if args.workload == "tet3d" else None,
                "alg_bytes_per_launch": dk["alg_bytes"], "avg_ms": dk["avg_ms"]}

    bc, bd = method_bytes(nv, ng, D, sT)
    h = codes.host()
    xr_host = out.cpu().numpy()                     # decoded values of the last timed step
    sb = M.stream_bytes(h, sT)
    cr = nv * sT / sb["total"]
    if args.copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        bb = torch.empty_like(a)
        for _ in range(3):
            bb.copy_(a)
        torch.cuda.synchronize()

    cold_ms = cold_step_ms(step)
    log(f"cold-cache step (1 GiB flush before each): {cold_ms:.4f} ms")
    copy_gbps = copy_ceiling_gbps()
    log(f"copy ceiling: {copy_gbps:.0f} GB/s")
    roofline["frac_of_copy"] = round(achieved / copy_gbps, 4)
    value = nv * sT / (ms_step * 1e-3) / 1e9
    line = {
        "metric": "compress/decompress GB/s of mesh values + CR, learned vs plain, eb=1e-4",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": desc, "n_vertices": nv, "n_cells": mesh.n_cells, "n_grid": ng,
                   "eb": args.eb, "eb_mode": "rel", "grid_share": args.split},
        "roofline": roofline,
        "compress_GBps": round(nv * sT / (comp_ms * 1e-3) / 1e9, 2),
        "decompress_GBps": round(nv * sT / (dec_ms * 1e-3) / 1e9, 2),
        "compress_ms": round(comp_ms, 4),
        "decompress_ms": round(dec_ms, 4),
        "alg_bytes_compress": bc,
        "alg_bytes_decompress": bd,
        "hbm_frac_alg": round((bc + bd) / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
        "cold_cache": {"ms_per_step": round(cold_ms, 4), "GBps": round(nv * sT / (cold_ms * 1e-3) / 1e9, 2),
                       "hbm_frac_alg": round((bc + bd) / (cold_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
                       "flush": "1 GiB written before each of 20 steps; median"},
        "copy_ceiling_GBps": round(copy_gbps, 1),
        "copy_frac_alg": round((bc + bd) / (ms_step * 1e-3) / 1e9 / copy_gbps, 4),
        "cr": round(cr, 3),
        "stream_bytes": sb,
        "outliers": {"grid": h["result"]["n_grid_outliers"], "vertex": h["result"]["n_vertex_outliers"]},
        "max_abs_err_over_tau": round(err / res["tau"], 4),
        "ms_per_step_with_kernel_events": round(ms_step_ev, 4),
        "settle": {"seconds": args.settle, "untimed_steps": n_settle},
        "plan_seconds": round(plan_s, 3),
        "tuning": tune,
        "bin_tuning": bins,
        "plan": {k: info[k] for k in ("n_unresolved", "n_near_degenerate", "n_pairs", "bin_nodes")},
        "kernels": kernels,
    }
    if not args.no_compare:
        mc_c = _timed(lambda: M.compress(plan, x, args.eb, "rel", args.split, codes=codes))
        mc_d = _timed(lambda: M.decompress(plan, codes, out=out))
        line["serial_baseline"] = [serial_compare(M, x, args.eb, h, (mc_c, mc_d), log, "generated order"),
                                   serial_compare(M, x, args.eb, h, (mc_c, mc_d), log, "random order",
                                                  shuffle_seed=7)]
    if args.workload == "tet3d" and not args.no_compare:
        line["design_points"] = [design_point(M, mesh, coords, x, args.eb, log),
                                 design_point(M, mesh, coords, x, args.eb, log, predictor="delta"),
                                 design_point(M, mesh, coords, x, args.eb, log, predictor="delta",
                                              grid_predictor="cubic"),
                                 design_point(M, mesh, coords, x, args.eb, log, dims=cfg["dims"][0],
                                              split=args.split, split_mode="sum", grid_predictor="cubic"),
                                 design_point(M, mesh, coords, x, args.eb, log, split=0.1, split_mode="sum",
                                              operators="cluster", residual="open"),
                                 # the paper's pair on a grid twice as fine as the vertex lattice (about
                                 # every other plane holds no vertex's node), without and with
                                 # Grid_Coarsen (Alg. 2)
                                 design_point(M, mesh, coords, x, args.eb, log, dims=503, split=0.1,
                                              split_mode="sum", operators="cluster", residual="open"),
                                 design_point(M, mesh, coords, x, args.eb, log, dims=503, split=0.1,
                                              split_mode="sum", operators="cluster", residual="open", coarsen=True)]
    if not args.no_learned:
        line["learned"] = learned_section(log, train_steps=args.train_steps)
        line["large2d"] = line["learned"].pop("large2d")
    if not args.no_batch and args.workload == "tet3d":
        # the many-fields workload (12 meshes, 64 fields) with its own steps
        line["batch"] = batch_section(args, log)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle, one thread, the same inputs) ...")
        line["cpu_baseline"] = cpu_baseline(mesh, f, cfg, args.eb, args.split, h_gpu=h, x_gpu=xr_host)
        log(f"cpu baseline: {line['cpu_baseline']}")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
