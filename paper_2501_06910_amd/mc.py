"""Python binding of libmc (include/mc.h): argument marshalling only.

Every step of the compressor runs in the HIP library; torch provides device
memory (tensor storage) and the stream (``torch.cuda.current_stream()``).
Loading fails loudly if the library has not been built -- there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes as C
import json
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmc.so")

OK, ERR_ARG, ERR_RANGE, ERR_CAPACITY, ERR_NOMEM, ERR_DEVICE, ERR_FORMAT, ERR_UNSUPPORTED = range(8)
F32, F64 = 0, 1
EB_ABS, EB_REL = 0, 1
FILL_NEAREST, FILL_MIDRANGE = 0, 1
RADIUS = 32768
BLOCK = 4096


class McGrid(C.Structure):
    _fields_ = [("dim", C.c_int32), ("dims", C.c_int64 * 3), ("origin", C.c_double * 3),
                ("spacing", C.c_double * 3)]


class McPlanOpts(C.Structure):
    _fields_ = [("fill", C.c_int), ("bin_nodes", C.c_int32), ("operators", C.c_int32), ("coarsen", C.c_int32)]


OPS_LINEAR, OPS_CLUSTER = 0, 1
RESIDUAL_CLOSED, RESIDUAL_OPEN = 0, 1


class McPlanInfo(C.Structure):
    _fields_ = [("n_grid", C.c_int64), ("n_vertices", C.c_int64), ("n_cells", C.c_int64),
                ("n_unresolved", C.c_int64), ("n_near_degenerate", C.c_int64), ("n_pairs", C.c_int64),
                ("bin_nodes", C.c_int64), ("device_bytes", C.c_int64), ("invalid_cells", C.c_int32)]


class McParams(C.Structure):
    _fields_ = [("eb", C.c_double), ("eb_mode", C.c_int32), ("grid_share", C.c_double),
                ("model", C.c_void_p), ("split_mode", C.c_int32), ("residual", C.c_int32)]


SPLIT_SUM, SPLIT_FULL = 0, 1


def _split_code(split_mode) -> int:
    if split_mode in ("sum", SPLIT_SUM):
        return SPLIT_SUM
    if split_mode in ("full", SPLIT_FULL):
        return SPLIT_FULL
    raise ValueError("split_mode must be 'sum' or 'full'")


class McResult(C.Structure):
    _fields_ = [("status", C.c_int32), ("dtype", C.c_int32), ("n_grid_outliers", C.c_int64),
                ("n_vertex_outliers", C.c_int64), ("n_learned_blocks", C.c_int64),
                ("tau", C.c_double), ("tau1", C.c_double), ("tau2", C.c_double), ("c", C.c_double),
                ("xmin", C.c_double), ("xmax", C.c_double), ("kappa_unused", C.c_double)]


class McCodes(C.Structure):
    _fields_ = [("grid_codes", C.c_void_p), ("g_out_idx", C.c_void_p), ("g_out_delta", C.c_void_p),
                ("g_out_cap", C.c_int64), ("vert_codes", C.c_void_p), ("v_out_idx", C.c_void_p),
                ("v_out_val", C.c_void_p), ("v_out_cap", C.c_int64), ("block_flags", C.c_void_p),
                ("result", C.c_void_p), ("dbg_resampled", C.c_void_p), ("dbg_grid_p", C.c_void_p),
                ("dbg_vertex_g", C.c_void_p), ("rho_q", C.c_void_p), ("residual_predictor", C.c_int32),
                ("grid_predictor", C.c_int32), ("grid_ref", C.c_void_p), ("xhat_out", C.c_void_p)]


class McTrainOpts(C.Structure):
    _fields_ = [("steps", C.c_int32), ("batch", C.c_int32), ("lr", C.c_float), ("seed", C.c_uint64),
                ("h_loss_out", C.c_void_p), ("sample_steps", C.c_int32)]


class McBatchItem(C.Structure):
    _fields_ = [("plan", C.c_void_p), ("d_field", C.c_void_p), ("dtype", C.c_int), ("params", McParams),
                ("codes", McCodes)]


class McTuning(C.Structure):
    _fields_ = [("remap_mask", C.c_uint32), ("reserved", C.c_uint32 * 3)]


class McStreamHeader(C.Structure):
    _fields_ = [("dim", C.c_int32), ("dtype", C.c_int32), ("dims", C.c_int64 * 3), ("n_vertices", C.c_int64),
                ("grid_predictor", C.c_int32), ("residual_predictor", C.c_int32), ("learned", C.c_int32),
                ("reserved", C.c_int32), ("tau", C.c_double), ("tau1", C.c_double), ("tau2", C.c_double),
                ("c", C.c_double), ("n_grid_outliers", C.c_int64), ("n_vertex_outliers", C.c_int64)]


class McStreamArrays(C.Structure):
    _fields_ = [("grid_codes", C.c_void_p), ("g_out_idx", C.c_void_p), ("g_out_delta", C.c_void_p),
                ("vert_codes", C.c_void_p), ("v_out_idx", C.c_void_p), ("v_out_val", C.c_void_p),
                ("block_flags", C.c_void_p)]


class McBatchDItem(C.Structure):
    _fields_ = [("plan", C.c_void_p), ("codes", McCodes), ("model", C.c_void_p), ("d_out", C.c_void_p),
                ("dtype", C.c_int)]


# every symbol include/mc.h declares, with its ctypes signature
_P = C.c_void_p
_SIGS = {
    "mc_status_string": (C.c_char_p, [C.c_int]),
    "mc_last_error": (C.c_char_p, []),
    "mc_abi_version": (C.c_int32, []),
    "mc_grid_from_dims": (C.c_int, [_P, C.c_int32, C.c_int64, _P, _P, _P]),
    "mc_grid_from_spacing": (C.c_int, [_P, C.c_int32, C.c_int64, _P, _P, _P]),
    "mc_grid_from_percentile": (C.c_int, [_P, _P, C.c_int32, C.c_int64, C.c_int64, C.c_double, C.c_int64, _P, _P,
                                          _P]),
    "mc_plan_create": (C.c_int, [_P, _P, C.c_int32, C.c_int64, C.c_int64, _P, _P, _P, _P]),
    "mc_plan_tune_bins": (C.c_int, [_P, _P, C.c_int32, C.c_int64, C.c_int64, _P, _P, C.c_int32, _P, _P, _P]),
    "mc_plan_get_info": (C.c_int, [_P, _P]),
    "mc_plan_mapping": (C.c_int, [_P, _P, _P, _P, _P]),
    "mc_plan_get_grid": (C.c_int, [_P, _P]),
    "mc_plan_destroy": (C.c_int, [_P]),
    "mc_plan_nodes": (C.c_int, [_P, _P, _P]),
    "mc_plan_node_lists": (C.c_int, [_P, _P, _P, _P]),
    "mc_plan_kept_planes": (C.c_int, [_P, _P, C.c_int64]),
    "mc_compress": (C.c_int, [_P, _P, C.c_int, _P, _P, _P]),
    "mc_decompress": (C.c_int, [_P, _P, _P, _P, C.c_int, _P]),
    "mc_compress_mesh": (C.c_int, [_P, _P, C.c_int32, C.c_int64, C.c_int64, _P, C.c_int, _P, C.c_double,
                                   C.c_int32, C.c_double, _P, _P, _P]),
    "mc_model_param_count": (C.c_int64, [C.c_int32]),
    "mc_model_create": (C.c_int, [C.c_int32, _P, C.c_float, _P]),
    "mc_model_train": (C.c_int, [_P, _P, C.c_int, _P, _P, _P, _P]),
    "mc_model_get_params": (C.c_int, [_P, _P, _P]),
    "mc_model_export": (C.c_int, [_P, _P, C.c_size_t, _P]),
    "mc_model_import": (C.c_int, [_P, C.c_size_t, _P]),
    "mc_model_destroy": (C.c_int, [_P]),
    "mc_model_forward": (C.c_int, [_P, _P, C.c_int64, _P, _P]),
    "mc_model_loss_grad": (C.c_int, [_P, _P, _P, C.c_int64, _P, _P, _P]),
    "mc_model_features": (C.c_int, [_P, _P, _P, C.c_int64, C.c_int64, _P, _P]),
    "mc_batch_compress": (C.c_int, [_P, C.c_int32, _P]),
    "mc_batch_graph_info": (C.c_int, [C.c_int32, _P, C.c_int32, _P, _P]),
    "mc_batch_release": (C.c_int, []),
    "mc_plan_get_tuning": (C.c_int, [_P, _P]),
    "mc_plan_set_tuning": (C.c_int, [_P, _P]),
    "mc_plan_tune": (C.c_int, [_P, _P, C.c_int, _P, _P, _P, C.c_int32, _P, _P]),
    "mc_batch_decompress": (C.c_int, [_P, C.c_int32, _P]),
    "mc_serial_create": (C.c_int, [C.c_int64, _P]),
    "mc_serial_destroy": (C.c_int, [_P]),
    "mc_serial_compress": (C.c_int, [_P, _P, C.c_int, C.c_int64, C.c_double, C.c_int32, _P, _P]),
    "mc_serial_decompress": (C.c_int, [_P, _P, C.c_int64, _P, C.c_int, _P]),
    "mc_serial_noalloc_max": (C.c_int64, []),
    "mc_serial_compress_noalloc": (C.c_int, [_P, C.c_int, C.c_int64, C.c_double, C.c_int32, _P, _P]),
    "mc_profile_enable": (C.c_int, [C.c_int32]),
    "mc_profile_reset": (C.c_int, []),
    "mc_profile_only": (C.c_int, [C.c_char_p]),
    "mc_profile_read": (C.c_int32, [_P, _P, _P, C.c_int32]),
    "mc_huffman_size": (C.c_int64, [_P, C.c_int64]),
    "mc_huffman_encode": (C.c_int64, [_P, C.c_int64, _P, C.c_int64]),
    "mc_huffman_decode": (C.c_int64, [_P, C.c_int64, _P, C.c_int64]),
    "mc_entropy_bits": (C.c_double, [_P, C.c_int64]),
    "mc_stream_size": (C.c_int64, [_P, _P, _P, C.c_int64, _P]),
    "mc_stream_write": (C.c_int64, [_P, _P, _P, C.c_int64, _P, C.c_int64, _P]),
    "mc_stream_read_header": (C.c_int, [_P, C.c_int64, _P, _P]),
    "mc_stream_read": (C.c_int, [_P, C.c_int64, _P, _P, C.c_int64]),
}

_lib = None


def lib():
    """The loaded libmc.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2501_06910_amd.build` (no CPU fallback exists)")
        # torch first: the library's HIP runtime dependency then resolves to
        # the one torch has loaded, so both share one runtime and device
        # state (opened the other way round, two runtimes are loaded and the
        # library's sees no device)
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class McError(RuntimeError):
    def __init__(self, status, where=""):
        msg = lib().mc_last_error().decode()
        super().__init__(f"{where}: {lib().mc_status_string(status).decode()} ({status}): {msg}")
        self.status = status


def _check(st, where):
    if st != OK:
        raise McError(st, where)


def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _dtype_code(t) -> int:
    torch = _torch()
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.float64:
        return F64
    raise TypeError("field must be float32 or float64")


def _require_cuda(t, name, dtype=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")


# ---------------------------------------------------------------------------
# grids and plans
# ---------------------------------------------------------------------------

def grid_from_dims(coords, dims) -> McGrid:
    torch = _torch()
    _require_cuda(coords, "coords", torch.float32)
    g = McGrid()
    d = (C.c_int64 * 3)(*(list(dims) + [1] * (3 - len(dims))))
    _check(lib().mc_grid_from_dims(_ptr(coords), coords.shape[0], coords.shape[1], d, _stream(),
                                   C.byref(g)), "mc_grid_from_dims")
    return g


def grid_from_spacing(coords, spacing) -> McGrid:
    torch = _torch()
    _require_cuda(coords, "coords", torch.float32)
    g = McGrid()
    h = (C.c_double * 3)(*(list(spacing) + [1.0] * (3 - len(spacing))))
    _check(lib().mc_grid_from_spacing(_ptr(coords), coords.shape[0], coords.shape[1], h, _stream(),
                                      C.byref(g)), "mc_grid_from_spacing")
    return g


def grid_from_percentile(coords, cells, k: float, g_max: int):
    """The paper's grid initialisation (Alg. 1): (grid, k used per axis)."""
    torch = _torch()
    _require_cuda(coords, "coords", torch.float32)
    _require_cuda(cells, "cells", torch.int32)
    g = McGrid()
    ku = (C.c_double * 3)()
    _check(lib().mc_grid_from_percentile(_ptr(coords), _ptr(cells), coords.shape[0], coords.shape[1],
                                         cells.shape[1], float(k), int(g_max), _stream(), C.byref(g), ku),
           "mc_grid_from_percentile")
    return g, [ku[0], ku[1], ku[2]]


def make_grid(dim, dims, origin, spacing) -> McGrid:
    g = McGrid()
    g.dim = dim
    for d in range(3):
        g.dims[d] = dims[d] if d < dim else 1
        g.origin[d] = origin[d] if d < dim else 0.0
        g.spacing[d] = spacing[d] if d < dim else 1.0
    return g


class Plan:
    """Field-independent mesh-grid mapping (owns device memory)."""

    def __init__(self, coords, cells, grid: McGrid | None = None, dims=None, fill: str = "nearest",
                 bin_nodes=0, operators: str = "linear", coarsen: bool = False):
        """operators: "linear" (barycentric f, multilinear g) or "cluster"
        (the paper's cluster-mean f and nearest-node g; cells may be None);
        coarsen: Grid_Coarsen (cluster plans), after which `grid` and
        `n_grid` describe the coarsened grid and `kept_planes()` lists it;
        bin_nodes: the point-location bin edge in grid nodes (0: the
        library's default, "auto": the fastest of BIN_CANDIDATES timed by
        mc_plan_tune_bins, kept in the tuning cache per mesh signature)."""
        torch = _torch()
        _require_cuda(coords, "coords", torch.float32)
        if operators not in ("linear", "cluster"):
            raise ValueError("operators must be 'linear' or 'cluster'")
        if cells is not None or operators == "linear":
            _require_cuda(cells, "cells", torch.int32)
        self.dim = int(coords.shape[0])
        self.operators = operators
        if grid is None:
            grid = grid_from_dims(coords, dims)
        self.grid = grid
        self.bin_tuning = None
        if bin_nodes == "auto":
            bin_nodes = 0
            if operators == "linear":
                bin_nodes, self.bin_tuning = tune_bins(coords, cells, grid)
        opts = McPlanOpts(FILL_NEAREST if fill == "nearest" else FILL_MIDRANGE, int(bin_nodes),
                          OPS_CLUSTER if operators == "cluster" else OPS_LINEAR, 1 if coarsen else 0)
        h = C.c_void_p()
        _check(lib().mc_plan_create(_ptr(coords), _ptr(cells), self.dim, coords.shape[1],
                                    0 if cells is None else cells.shape[1], C.byref(grid), C.byref(opts), _stream(),
                                    C.byref(h)), "mc_plan_create")
        self.handle = h
        self.n_vertices = int(coords.shape[1])
        self.grid_given = grid
        self.coarsen = bool(coarsen)
        actual = McGrid()
        _check(lib().mc_plan_get_grid(self.handle, C.byref(actual)), "mc_plan_get_grid")
        self.grid = actual
        self.n_grid = int(actual.dims[0] * actual.dims[1] * actual.dims[2])

    def kept_planes(self) -> np.ndarray:
        """Grid_Coarsen: each given plane's index on the coarsened axis, or -1
        (axis 0, then 1, then 2)."""
        n = int(sum(self.grid_given.dims[d] for d in range(3)))
        out = np.empty(n, np.int32)
        _check(lib().mc_plan_kept_planes(self.handle, out.ctypes.data_as(C.c_void_p), n), "mc_plan_kept_planes")
        return out

    def info(self) -> dict:
        i = McPlanInfo()
        _check(lib().mc_plan_get_info(self.handle, C.byref(i)), "mc_plan_get_info")
        return {k: getattr(i, k) for k, _ in McPlanInfo._fields_}

    def mapping(self):
        torch = _torch()
        vid = torch.empty((self.dim + 1, self.n_grid), dtype=torch.int32, device="cuda")
        w = torch.empty((self.dim + 1, self.n_grid), dtype=torch.float32, device="cuda")
        cell = torch.empty(self.n_grid, dtype=torch.int32, device="cuda")
        _check(lib().mc_plan_mapping(self.handle, _ptr(vid), _ptr(w), _ptr(cell), _stream()), "mc_plan_mapping")
        return vid, w, cell

    def nodes(self):
        """Nearest grid node of every vertex (cluster plans)."""
        torch = _torch()
        m = torch.empty(self.n_vertices, dtype=torch.int32, device="cuda")
        _check(lib().mc_plan_nodes(self.handle, _ptr(m), _stream()), "mc_plan_nodes")
        return m

    def node_lists(self):
        """(noff int64[n_grid + 1], vlist int32[n_vertices]): node j's
        vertices in ascending id order are vlist[noff[j]:noff[j+1]]
        (cluster plans)."""
        torch = _torch()
        noff = torch.empty(self.n_grid + 1, dtype=torch.int64, device="cuda")
        vlist = torch.empty(self.n_vertices, dtype=torch.int32, device="cuda")
        _check(lib().mc_plan_node_lists(self.handle, _ptr(noff), _ptr(vlist), _stream()), "mc_plan_node_lists")
        return noff, vlist

    @property
    def remap_mask(self) -> int:
        t = McTuning()
        _check(lib().mc_plan_get_tuning(self.handle, C.byref(t)), "mc_plan_get_tuning")
        return int(t.remap_mask)

    @remap_mask.setter
    def remap_mask(self, mask: int):
        t = McTuning(mask)
        _check(lib().mc_plan_set_tuning(self.handle, C.byref(t)), "mc_plan_set_tuning")

    def tune(self, field, eb: float, eb_mode: str = "rel", grid_share: float = 0.5, model=None, reps: int = 5,
             cache: bool = False, split_mode="sum") -> int:
        """Chooses the launch-order knobs by timing this field; returns the
        mask.  With cache=True, a mask stored for this device, grid and mesh
        size (tuning_cache.json beside this module) is applied without
        timing, and a new choice is stored there."""
        torch = _torch()
        key = None
        if cache:
            key = tuning_key(self, field.dtype)
            hit = tuning_cache().get(key)
            if hit is not None:
                self.remap_mask = int(hit["remap_mask"])
                return int(hit["remap_mask"])
        codes = Codes(self, field.dtype, learned=model is not None)
        out = torch.empty_like(field)
        prm = McParams(eb, EB_REL if eb_mode == "rel" else EB_ABS, grid_share,
                       None if model is None else model.handle, _split_code(split_mode))
        t = McTuning()
        _check(lib().mc_plan_tune(self.handle, _ptr(field), _dtype_code(field), C.byref(prm), C.byref(codes.struct),
                                  _ptr(out), reps, _stream(), C.byref(t)), "mc_plan_tune")
        if key is not None:
            store_tuning(key, int(t.remap_mask))
        return int(t.remap_mask)

    def destroy(self):
        if getattr(self, "handle", None):
            lib().mc_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# compressed buffers
# ---------------------------------------------------------------------------

TUNING_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_cache.json")


def tuning_key(plan: "Plan", dtype) -> str:
    """Cache key of a tuning: device architecture, grid dims, vertex count, dtype."""
    torch = _torch()
    arch = torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName.split(":")[0]
    g = plan.grid
    dims = "x".join(str(int(g.dims[d])) for d in range(plan.dim))
    # "k13": masks over the thirteen knob bits of this library version
    return f"{arch}|k13|dim{plan.dim}|{dims}|nv{plan.n_vertices}|{str(dtype).replace('torch.', '')}"


BIN_CANDIDATES = (1, 2, 3, 4)


def tune_bins(coords, cells, grid: McGrid, candidates=BIN_CANDIDATES):
    """The fastest point-location bin edge for this mesh and grid
    (mc_plan_tune_bins), from the tuning cache when this device, grid and
    mesh size were timed before.  Returns (bin_nodes, {edge: ms} or the
    cache entry)."""
    torch = _torch()
    arch = torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName.split(":")[0]
    dim = int(coords.shape[0])
    dims = "x".join(str(int(grid.dims[d])) for d in range(dim))
    key = f"{arch}|bins|dim{dim}|{dims}|nv{int(coords.shape[1])}|nc{int(cells.shape[1])}"
    hit = tuning_cache().get(key)
    if hit is not None:
        return int(hit["bin_nodes"]), hit
    cand = np.ascontiguousarray(candidates, np.int32)
    ms = np.zeros(cand.size, np.float64)
    best = C.c_int32()
    _check(lib().mc_plan_tune_bins(_ptr(coords), _ptr(cells), dim, coords.shape[1], cells.shape[1], C.byref(grid),
                                   cand.ctypes.data, cand.size, _stream(), C.byref(best), ms.ctypes.data),
           "mc_plan_tune_bins")
    rec = {"bin_nodes": int(best.value), "ms": {str(int(c)): round(float(t), 4) for c, t in zip(cand, ms)}}
    store_tuning(key, rec)
    return int(best.value), rec


def tuning_cache() -> dict:
    if not os.path.exists(TUNING_CACHE):
        return {}
    with open(TUNING_CACHE) as f:
        return json.load(f)


def store_tuning(key: str, mask):
    c = tuning_cache()
    c[key] = mask if isinstance(mask, dict) else {"remap_mask": mask}
    try:
        tmp = TUNING_CACHE + f".tmp{os.getpid()}"
        with open(tmp, "w") as f:
            json.dump(c, f, indent=1, sort_keys=True)
        os.replace(tmp, TUNING_CACHE)
    except OSError:
        pass            # a read-only install keeps tuning per process


GRID_PREDICTORS = {"lorenzo": 0, "linear": 1, "cubic": 2, "temporal": 3}


class Codes:
    """Device buffers of one compressed field (allocated with torch)."""

    def __init__(self, plan: Plan, dtype, g_cap=None, v_cap=None, learned=False, debug=False,
                 residual_predictor: str = "none", grid_predictor: str = "lorenzo", grid_ref=None,
                 xhat_out=None):
        """residual_predictor: "none" or "delta" (1-D Lorenzo along the vertex
        order); grid_predictor: "lorenzo", "linear" or "cubic" (multilevel
        interpolation) or "temporal" (from the reference grid grid_ref, a
        float32 device tensor of n_grid values, normally the previous
        timestep's x1'); both fixed for the buffers' lifetime, compress and
        decompress.  xhat_out: optional float32 device tensor of n_grid
        values that receives x1' at every compress and decompress."""
        torch = _torch()
        ng, nv = plan.n_grid, plan.n_vertices
        g_cap = ng if g_cap is None else g_cap
        v_cap = nv if v_cap is None else v_cap
        dev = "cuda"
        self.dtype = dtype
        self.grid_codes = torch.empty(ng, dtype=torch.uint16, device=dev)
        self.g_out_idx = torch.empty(max(g_cap, 1), dtype=torch.int32, device=dev)
        self.g_out_delta = torch.empty(max(g_cap, 1), dtype=torch.int32, device=dev)
        self.vert_codes = torch.empty(nv, dtype=torch.uint16, device=dev)
        self.v_out_idx = torch.empty(max(v_cap, 1), dtype=torch.int32, device=dev)
        self.v_out_val = torch.empty(max(v_cap, 1), dtype=dtype, device=dev)
        nblocks = (nv + BLOCK - 1) // BLOCK
        self.block_flags = torch.zeros((nblocks + 31) // 32, dtype=torch.int32, device=dev)
        self.result = torch.zeros(C.sizeof(McResult), dtype=torch.uint8, device=dev)
        self.dbg = debug
        self.dbg_resampled = torch.empty(ng, dtype=torch.float32, device=dev) if debug else None
        self.dbg_grid_p = torch.empty(ng, dtype=torch.int32, device=dev) if debug else None
        self.dbg_vertex_g = torch.empty(nv, dtype=torch.float32, device=dev) if debug else None
        self.rho_q = torch.empty(nv, dtype=torch.int32, device=dev) if (debug and learned) else None
        self.struct = McCodes(
            _ptr(self.grid_codes), _ptr(self.g_out_idx), _ptr(self.g_out_delta), g_cap, _ptr(self.vert_codes),
            _ptr(self.v_out_idx), _ptr(self.v_out_val), v_cap, _ptr(self.block_flags), _ptr(self.result),
            _ptr(self.dbg_resampled), _ptr(self.dbg_grid_p), _ptr(self.dbg_vertex_g), _ptr(self.rho_q),
            {"none": 0, "delta": 1}[residual_predictor], GRID_PREDICTORS[grid_predictor],
            _ptr(self._grid_tensor(grid_ref, ng, "grid_ref")), _ptr(self._grid_tensor(xhat_out, ng, "xhat_out")))
        self.grid_predictor = grid_predictor
        self.grid_ref, self.xhat_out = grid_ref, xhat_out      # kept alive with the buffers
        g = plan.grid
        self.meta = dict(dim=plan.dim, dims=tuple(int(g.dims[d]) for d in range(3)),
                         dtype=F64 if dtype == torch.float64 else F32,
                         grid_predictor=GRID_PREDICTORS[grid_predictor],
                         residual_predictor={"none": 0, "delta": 1}[residual_predictor])

    def set_grid_ref(self, grid_ref):
        """Point the time-axis predictor at another reference grid (the next
        timestep's compress and decompress)."""
        self.struct.grid_ref = _ptr(self._grid_tensor(grid_ref, self.grid_codes.numel(), "grid_ref"))
        self.grid_ref = grid_ref

    @staticmethod
    def _grid_tensor(t, ng, what):
        if t is None:
            return None
        _require_cuda(t, what)
        torch = _torch()
        if t.dtype != torch.float32 or t.numel() != ng or not t.is_contiguous():
            raise ValueError(f"{what} must be a contiguous float32 tensor of n_grid values")
        return t

    @classmethod
    def from_stream(cls, plan: Plan, blob: bytes):
        """Device codes of a stream written by write_stream (mc_stream_read,
        then uploaded), ready for decompress with this plan.  Returns
        (codes, model file bytes or None)."""
        torch = _torch()
        h = read_stream(blob)
        if "meta" not in h:
            raise ValueError("a 1-D baseline stream has no grid: decode it with serial_decompress")
        m = h["meta"]
        g = plan.grid
        if m["dim"] != plan.dim or any(int(g.dims[d]) != m["dims"][d] for d in range(plan.dim)) or \
                h["vert_codes"].size != plan.n_vertices:
            raise ValueError("stream and plan disagree on the grid or the vertex count")
        dtype = torch.float64 if m["dtype"] == F64 else torch.float32
        inv = {v: k for k, v in GRID_PREDICTORS.items()}
        c = cls(plan, dtype, g_cap=max(int(h["g_out_idx"].size), 1), v_cap=max(int(h["v_out_idx"].size), 1),
                learned=h["learned"], grid_predictor=inv[m["grid_predictor"]],
                residual_predictor={0: "none", 1: "delta"}[m["residual_predictor"]])
        c.grid_codes.view(torch.int16).copy_(torch.from_numpy(h["grid_codes"].view(np.int16)))
        c.vert_codes.view(torch.int16).copy_(torch.from_numpy(h["vert_codes"].view(np.int16)))
        for dst, src in ((c.g_out_idx, h["g_out_idx"]), (c.g_out_delta, h["g_out_delta"]),
                         (c.v_out_idx, h["v_out_idx"]), (c.v_out_val, h["v_out_val"])):
            if src.size:
                dst[:src.size].copy_(torch.from_numpy(np.ascontiguousarray(src)))
        c.block_flags.copy_(torch.from_numpy(h["block_flags"].view(np.int32)))
        r = h["result"]
        nl = int(sum(bin(int(w)).count("1") for w in h["block_flags"])) if h["learned"] else 0
        res = McResult(0, m["dtype"], int(r["n_grid_outliers"]), int(r["n_vertex_outliers"]), nl,
                       r["tau"], r["tau1"], r["tau2"], r["c"], 0.0, 0.0, 0.0)
        c.result.copy_(torch.frombuffer(bytearray(bytes(res)), dtype=torch.uint8))
        return c, h["model"]

    def result_host(self) -> dict:
        b = self.result.cpu().numpy().tobytes()
        r = McResult.from_buffer_copy(b)
        return {k: getattr(r, k) for k, _ in McResult._fields_}

    def host_grid(self) -> dict:
        """Host copies of the grid part only (synchronises)."""
        r = self.result_host()
        n = r["n_grid_outliers"]
        return dict(result=r, grid_codes=self.grid_codes.cpu().numpy().view(np.uint16),
                    g_out_idx=self.g_out_idx[:n].cpu().numpy(), g_out_delta=self.g_out_delta[:n].cpu().numpy())

    def host(self) -> dict:
        """Host copies of the compressed representation (synchronises)."""
        r = self.result_host()
        ng_out, nv_out = r["n_grid_outliers"], r["n_vertex_outliers"]
        return dict(
            result=r,
            grid_codes=self.grid_codes.cpu().numpy().view(np.uint16),
            g_out_idx=self.g_out_idx[:ng_out].cpu().numpy(),
            g_out_delta=self.g_out_delta[:ng_out].cpu().numpy(),
            vert_codes=self.vert_codes.cpu().numpy().view(np.uint16),
            v_out_idx=self.v_out_idx[:nv_out].cpu().numpy(),
            v_out_val=self.v_out_val[:nv_out].cpu().numpy(),
            block_flags=self.block_flags.cpu().numpy().view(np.uint32),
            meta=dict(self.meta),
        )


def compress(plan: Plan, field, eb: float, eb_mode: str = "rel", grid_share: float = 0.5, model=None,
             codes: Codes | None = None, debug: bool = False, split_mode="sum", residual: str = "closed") -> Codes:
    """residual: "closed" (against the reconstructed grid) or "open" (against
    the grid before compression, Alg. 3; cluster plans, sum split)."""
    _require_cuda(field, "field")
    if codes is None:
        codes = Codes(plan, field.dtype, learned=model is not None, debug=debug)
    if residual not in ("closed", "open"):
        raise ValueError("residual must be 'closed' or 'open'")
    prm = McParams(eb, EB_REL if eb_mode == "rel" else EB_ABS, grid_share,
                   None if model is None else model.handle, _split_code(split_mode),
                   RESIDUAL_OPEN if residual == "open" else RESIDUAL_CLOSED)
    _check(lib().mc_compress(plan.handle, _ptr(field), _dtype_code(field), C.byref(prm), C.byref(codes.struct),
                             _stream()), "mc_compress")
    return codes


def decompress(plan: Plan, codes: Codes, model=None, out=None):
    torch = _torch()
    if out is None:
        out = torch.empty(plan.n_vertices, dtype=codes.dtype, device="cuda")
    _check(lib().mc_decompress(plan.handle, C.byref(codes.struct), None if model is None else model.handle,
                               _ptr(out), _dtype_code(out), _stream()), "mc_decompress")
    return out


def compress_mesh(coords, cells, field, spacing, eb, eb_mode="rel", grid_share=0.5):
    """One-shot form: plan built and released inside the call."""
    torch = _torch()
    g = McGrid()
    h = (C.c_double * 3)(*(list(spacing) + [1.0] * (3 - len(spacing))))
    # grid first, to size the buffers
    grid = grid_from_spacing(coords, spacing)
    ng = int(grid.dims[0] * grid.dims[1] * grid.dims[2])

    class _Shape:
        n_grid = ng
        n_vertices = int(coords.shape[1])
    codes = Codes(_Shape, field.dtype)
    _check(lib().mc_compress_mesh(_ptr(coords), _ptr(cells), coords.shape[0], coords.shape[1], cells.shape[1],
                                  _ptr(field), _dtype_code(field), h, eb, EB_REL if eb_mode == "rel" else EB_ABS,
                                  grid_share, C.byref(codes.struct), C.byref(g), _stream()), "mc_compress_mesh")
    return codes, g


# ---------------------------------------------------------------------------
# learned predictor
# ---------------------------------------------------------------------------

def param_count(dim: int) -> int:
    return int(lib().mc_model_param_count(dim))


class Model:
    def __init__(self, handle, dim):
        self.handle = handle
        self.dim = dim

    @classmethod
    def create(cls, dim: int, params: np.ndarray, kappa: float):
        p = np.ascontiguousarray(params, np.float32)
        h = C.c_void_p()
        _check(lib().mc_model_create(dim, p.ctypes.data, kappa, C.byref(h)), "mc_model_create")
        return cls(h, dim)

    @classmethod
    def train(cls, plan: Plan, field, eb=1e-4, eb_mode="rel", grid_share=0.5, steps=2000, batch=8192,
              lr=1e-3, seed=0, return_loss=False, split_mode="sum", sample_steps=0):
        prm = McParams(eb, EB_REL if eb_mode == "rel" else EB_ABS, grid_share, None, _split_code(split_mode))
        loss = np.zeros(steps, np.float32)
        opts = McTrainOpts(steps, batch, lr, seed, loss.ctypes.data, sample_steps)
        h = C.c_void_p()
        _check(lib().mc_model_train(plan.handle, _ptr(field), _dtype_code(field), C.byref(prm), C.byref(opts),
                                    _stream(), C.byref(h)), "mc_model_train")
        m = cls(h, plan.dim)
        return (m, loss) if return_loss else m

    def params(self):
        n = param_count(self.dim)
        p = np.empty(n, np.float32)
        k = C.c_float()
        _check(lib().mc_model_get_params(self.handle, p.ctypes.data, C.byref(k)), "mc_model_get_params")
        return p, float(k.value)

    def export(self) -> bytes:
        n = C.c_size_t()
        _check(lib().mc_model_export(self.handle, None, 0, C.byref(n)), "mc_model_export")
        buf = (C.c_char * n.value)()
        _check(lib().mc_model_export(self.handle, buf, n.value, C.byref(n)), "mc_model_export")
        return bytes(buf)

    @classmethod
    def load(cls, blob: bytes):
        h = C.c_void_p()
        _check(lib().mc_model_import(blob, len(blob), C.byref(h)), "mc_model_import")
        return cls(h, int.from_bytes(blob[8:12], "little"))

    def forward(self, z):
        torch = _torch()
        _require_cuda(z, "z", torch.float32)
        rho = torch.empty(z.shape[0], dtype=torch.float32, device="cuda")
        _check(lib().mc_model_forward(self.handle, _ptr(z), z.shape[0], _ptr(rho), _stream()), "mc_model_forward")
        return rho

    def loss_grad(self, z, y):
        torch = _torch()
        g = torch.empty(param_count(self.dim), dtype=torch.float32, device="cuda")
        loss = torch.empty(1, dtype=torch.float32, device="cuda")
        _check(lib().mc_model_loss_grad(self.handle, _ptr(z), _ptr(y), z.shape[0], _ptr(g), _ptr(loss), _stream()),
               "mc_model_loss_grad")
        return float(loss.item()), g

    def features(self, plan: Plan, codes: Codes, v0=0, count=None):
        torch = _torch()
        count = plan.n_vertices - v0 if count is None else count
        kpad = 32 if self.dim == 2 else 96
        z = torch.empty((count, kpad), dtype=torch.float32, device="cuda")
        _check(lib().mc_model_features(self.handle, plan.handle, C.byref(codes.struct), v0, count, _ptr(z),
                                       _stream()), "mc_model_features")
        return z

    def destroy(self):
        if getattr(self, "handle", None):
            lib().mc_model_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# batching, profiling, entropy stage
# ---------------------------------------------------------------------------

def _batch_items(items):
    arr = (McBatchItem * len(items))()
    for i, it in enumerate(items):
        plan, field, eb, mode, share, model, codes = it[:7]
        split = it[7] if len(it) > 7 else "sum"
        resid = it[8] if len(it) > 8 else "closed"
        arr[i].plan = plan.handle
        arr[i].d_field = field.data_ptr()
        arr[i].dtype = _dtype_code(field)
        arr[i].params = McParams(eb, EB_REL if mode == "rel" else EB_ABS, share,
                                 None if model is None else model.handle, _split_code(split),
                                 RESIDUAL_OPEN if resid == "open" else RESIDUAL_CLOSED)
        arr[i].codes = codes.struct
    return arr


def batch_compress(items):
    """items: list of (plan, field, eb, eb_mode, grid_share, model, codes[,
    split_mode[, residual]]).  The first call with a given list captures a HIP graph;
    later calls with the same plans, tensors and parameters replay it."""
    arr = _batch_items(items)
    _check(lib().mc_batch_compress(arr, len(items), _stream()), "mc_batch_compress")


def _batch_ditems(items):
    arr = (McBatchDItem * len(items))()
    for i, (plan, codes, model, out) in enumerate(items):
        _require_cuda(out, "out")
        arr[i].plan = plan.handle
        arr[i].codes = codes.struct
        arr[i].model = None if model is None else model.handle
        arr[i].d_out = out.data_ptr()
        arr[i].dtype = _dtype_code(out)
    return arr


def batch_decompress(items):
    """items: list of (plan, codes, model, out); graph captured and replayed
    like batch_compress."""
    arr = _batch_ditems(items)
    _check(lib().mc_batch_decompress(arr, len(items), _stream()), "mc_batch_decompress")


def batch_graph_info(items, decompress: bool = False) -> dict:
    """The cached graph of this item list: fields on the work-list stage
    launches and the graph's node count."""
    arr = _batch_ditems(items) if decompress else _batch_items(items)
    nb, nn = C.c_int32(), C.c_int64()
    _check(lib().mc_batch_graph_info(1 if decompress else 0, arr, len(items), C.byref(nb), C.byref(nn)),
           "mc_batch_graph_info")
    return {"n_batched": nb.value, "n_nodes": nn.value}


def batch_release():
    """Synchronises the device and frees every cached batch graph."""
    _check(lib().mc_batch_release(), "mc_batch_release")


# ---------------------------------------------------------------------------
# 1-D serialisation baseline (Sec. V-C comparison)
# ---------------------------------------------------------------------------

class Serial:
    """Device workspace of the 1-D baseline for fields of up to n_max values."""

    def __init__(self, n_max: int):
        h = C.c_void_p()
        _check(lib().mc_serial_create(int(n_max), C.byref(h)), "mc_serial_create")
        self.handle = h
        self.n_max = int(n_max)

    def destroy(self):
        if getattr(self, "handle", None):
            lib().mc_serial_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


class SerialCodes:
    """Vertex codes, outliers and result header of one serially compressed field."""

    def __init__(self, n: int, dtype, cap=None):
        torch = _torch()
        cap = n if cap is None else cap
        self.n, self.dtype = n, dtype
        self.codes = torch.empty(n, dtype=torch.uint16, device="cuda")
        self.out_idx = torch.empty(max(cap, 1), dtype=torch.int32, device="cuda")
        self.out_val = torch.empty(max(cap, 1), dtype=dtype, device="cuda")
        self.result = torch.zeros(C.sizeof(McResult), dtype=torch.uint8, device="cuda")
        self.struct = McCodes(None, None, None, 0, _ptr(self.codes), _ptr(self.out_idx), _ptr(self.out_val), cap,
                              None, _ptr(self.result), None, None, None, None)

    def result_host(self) -> dict:
        r = McResult.from_buffer_copy(self.result.cpu().numpy().tobytes())
        return {k: getattr(r, k) for k, _ in McResult._fields_}

    def host(self) -> dict:
        r = self.result_host()
        k = min(r["n_vertex_outliers"], self.out_idx.numel())
        return dict(result=r, codes=self.codes.cpu().numpy().view(np.uint16),
                    out_idx=self.out_idx[:k].cpu().numpy(), out_val=self.out_val[:k].cpu().numpy())


def serial_compress(ctx: Serial, field, eb: float, eb_mode: str = "rel", codes: SerialCodes | None = None,
                    cap=None) -> SerialCodes:
    _require_cuda(field, "field")
    n = field.numel()
    if codes is None:
        codes = SerialCodes(n, field.dtype, cap)
    _check(lib().mc_serial_compress(ctx.handle, _ptr(field), _dtype_code(field), n, eb,
                                    EB_REL if eb_mode == "rel" else EB_ABS, C.byref(codes.struct), _stream()),
           "mc_serial_compress")
    return codes


def serial_compress_noalloc(field, eb: float, eb_mode: str = "rel", codes: SerialCodes | None = None,
                            cap=None) -> SerialCodes:
    """mc_serial_compress_noalloc: the 1-D baseline's compress on the
    library's fixed per-GPU scratch (no context, no device allocation by
    the library; fields of up to serial_noalloc_max() values)."""
    _require_cuda(field, "field")
    n = field.numel()
    if codes is None:
        codes = SerialCodes(n, field.dtype, cap)
    _check(lib().mc_serial_compress_noalloc(_ptr(field), _dtype_code(field), n, eb,
                                            EB_REL if eb_mode == "rel" else EB_ABS, C.byref(codes.struct),
                                            _stream()), "mc_serial_compress_noalloc")
    return codes


def serial_noalloc_max() -> int:
    return int(lib().mc_serial_noalloc_max())


def serial_decompress(ctx: Serial, codes: SerialCodes, out=None):
    torch = _torch()
    if out is None:
        out = torch.empty(codes.n, dtype=codes.dtype, device="cuda")
    _check(lib().mc_serial_decompress(ctx.handle, C.byref(codes.struct), codes.n, _ptr(out), _dtype_code(out),
                                      _stream()), "mc_serial_decompress")
    return out


def serial_stream_bytes(host: dict, value_bytes: int | None = None) -> dict:
    """Section sizes of the baseline's stream (a dim-1 stream: header,
    Huffman-coded codes, outlier index gaps and raw values, checksum), from
    the bytes mc_stream_write produces."""
    return write_stream(host)[1]


def profile_enable(on=True):
    lib().mc_profile_enable(1 if on else 0)


def profile_only(name=None):
    """Bracket only the launches of kernel `name` (None: every kernel)."""
    lib().mc_profile_only(name.encode() if name else None)


def profile_reset():
    lib().mc_profile_reset()


def profile_read() -> dict:
    cap = 64
    names = (C.c_char_p * cap)()
    counts = (C.c_int64 * cap)()
    ms = (C.c_double * cap)()
    n = lib().mc_profile_read(names, counts, ms, cap)
    return {names[i].decode(): (int(counts[i]), float(ms[i])) for i in range(n)}


def huffman_size(sym: np.ndarray) -> int:
    s = np.ascontiguousarray(sym, np.uint16)
    return int(lib().mc_huffman_size(s.ctypes.data, s.size))


def huffman_encode(sym: np.ndarray) -> bytes:
    s = np.ascontiguousarray(sym, np.uint16)
    cap = huffman_size(s)
    out = np.empty(cap, np.uint8)
    n = lib().mc_huffman_encode(s.ctypes.data, s.size, out.ctypes.data, cap)
    if n < 0:
        raise RuntimeError("huffman encode failed")
    return out[:n].tobytes()


def huffman_decode(blob: bytes, n: int) -> np.ndarray:
    out = np.empty(n, np.uint16)
    buf = np.frombuffer(blob, np.uint8)
    used = lib().mc_huffman_decode(buf.ctypes.data, buf.size, out.ctypes.data, n)
    if used < 0:
        raise ValueError("malformed Huffman stream")
    return out


def entropy_bits(sym: np.ndarray) -> float:
    s = np.ascontiguousarray(sym, np.uint16)
    return float(lib().mc_entropy_bits(s.ctypes.data, s.size))


STREAM_SECTIONS = ("header", "grid", "vert", "grid_outliers", "vert_outliers", "block_flags", "model", "checksum")


def _stream_args(host: dict):
    """Header and array structs of a host dict (Codes.host() or
    SerialCodes.host()); the arrays stay referenced by the returned list."""
    keep = []

    def ptr(a, dt):
        if a is None:
            return None
        a = np.ascontiguousarray(a, dt)
        keep.append(a)
        return a.ctypes.data
    r = host["result"]
    h = McStreamHeader()
    if "meta" in host:                               # multi-component codes
        m = host["meta"]
        h.dim, h.dtype = m["dim"], m["dtype"]
        for d in range(3):
            h.dims[d] = m["dims"][d] if d < m["dim"] else 1
        h.n_vertices = host["vert_codes"].size
        h.grid_predictor, h.residual_predictor = m["grid_predictor"], m["residual_predictor"]
        h.learned = 1 if host.get("learned") else 0
        vv = host["v_out_val"]
        arr = McStreamArrays(ptr(host["grid_codes"], np.uint16), ptr(host["g_out_idx"], np.int32),
                             ptr(host["g_out_delta"], np.int32), ptr(host["vert_codes"], np.uint16),
                             ptr(host["v_out_idx"], np.int32), ptr(vv, vv.dtype),
                             ptr(host["block_flags"], np.uint32) if h.learned else None)
        h.n_grid_outliers, h.n_vertex_outliers = host["g_out_idx"].size, host["v_out_idx"].size
    else:                                            # the 1-D baseline
        vv = host["out_val"]
        h.dim, h.dtype = 1, F64 if vv.dtype == np.float64 else F32
        h.dims[0] = h.dims[1] = h.dims[2] = 1
        h.n_vertices = host["codes"].size
        arr = McStreamArrays(None, None, None, ptr(host["codes"], np.uint16), ptr(host["out_idx"], np.int32),
                             ptr(vv, vv.dtype), None)
        h.n_grid_outliers, h.n_vertex_outliers = 0, host["out_idx"].size
    h.tau, h.tau1, h.tau2, h.c = r["tau"], r["tau1"], r["tau2"], r["c"]
    return h, arr, keep


def write_stream(host: dict, model: bytes | None = None) -> tuple:
    """The self-describing stream of one compressed field (mc_stream_write)
    and its section sizes (plus "total").  model: the model file to embed
    (Model.export()), normally once per timestep sequence."""
    h, arr, keep = _stream_args(host)
    mb = 0 if model is None else len(model)
    sec = (C.c_int64 * 8)()
    n = lib().mc_stream_size(C.byref(h), C.byref(arr), model, mb, sec)
    if n < 0:
        raise McError(ERR_ARG, "mc_stream_size")
    buf = (C.c_uint8 * n)()
    got = lib().mc_stream_write(C.byref(h), C.byref(arr), model, mb, buf, n, None)
    if got != n:
        raise McError(ERR_ARG, "mc_stream_write")
    parts = {k: int(sec[i]) for i, k in enumerate(STREAM_SECTIONS)}
    parts["total"] = int(n)
    return bytes(buf), parts


def read_stream(blob: bytes) -> dict:
    """Arrays of a stream (mc_stream_read): a dict shaped like Codes.host()
    (or SerialCodes.host() for a baseline stream) plus "model" (bytes or
    None)."""
    h = McStreamHeader()
    mb = C.c_int64()
    _check(lib().mc_stream_read_header(blob, len(blob), C.byref(h), C.byref(mb)), "mc_stream_read_header")
    vdt = np.float64 if h.dtype == F64 else np.float32
    nv = int(h.n_vertices)
    ng = 0 if h.dim == 1 else int(h.dims[0] * h.dims[1] * h.dims[2])
    gc = np.empty(max(ng, 1), np.uint16)
    gi = np.empty(max(int(h.n_grid_outliers), 1), np.int32)
    gd = np.empty_like(gi)
    vc = np.empty(nv, np.uint16)
    vi = np.empty(max(int(h.n_vertex_outliers), 1), np.int32)
    vv = np.empty(max(int(h.n_vertex_outliers), 1), vdt)
    nb = (nv + BLOCK - 1) // BLOCK
    bf = np.zeros((nb + 31) // 32, np.uint32)
    arr = McStreamArrays(gc.ctypes.data, gi.ctypes.data, gd.ctypes.data, vc.ctypes.data, vi.ctypes.data,
                         vv.ctypes.data, bf.ctypes.data)
    model = (C.c_uint8 * max(mb.value, 1))()
    _check(lib().mc_stream_read(blob, len(blob), C.byref(arr), model, mb.value), "mc_stream_read")
    r = {k: getattr(h, k) for k in ("tau", "tau1", "tau2", "c", "n_grid_outliers", "n_vertex_outliers")}
    ko, kv = int(h.n_grid_outliers), int(h.n_vertex_outliers)
    if h.dim == 1:
        out = dict(result=r, codes=vc, out_idx=vi[:kv], out_val=vv[:kv])
    else:
        out = dict(result=r, grid_codes=gc[:ng], g_out_idx=gi[:ko], g_out_delta=gd[:ko], vert_codes=vc,
                   v_out_idx=vi[:kv], v_out_val=vv[:kv], block_flags=bf, learned=bool(h.learned),
                   meta=dict(dim=int(h.dim), dims=tuple(int(h.dims[d]) for d in range(3)), dtype=int(h.dtype),
                             grid_predictor=int(h.grid_predictor), residual_predictor=int(h.residual_predictor)))
    out["model"] = bytes(model)[:mb.value] if mb.value > 0 else None
    return out


def grid_stream_bytes(grid_codes: np.ndarray, g_out_idx: np.ndarray, g_out_delta: np.ndarray) -> int:
    """Bytes of the grid sections of a stream (the Huffman-coded grid codes
    with their length prefix, and the grid outlier list): what the sections
    "grid" and "grid_outliers" of write_stream count, for other grid codes
    of the same field."""
    def leb(values):
        v = np.asarray(values, np.uint64)
        n = np.ones(v.size, np.int64)
        t = v >> np.uint64(7)
        while np.any(t):
            n += (t > 0)
            t = t >> np.uint64(7)
        return int(n.sum())
    gi = g_out_idx.astype(np.int64)
    g_gap = np.diff(np.concatenate([[-1], gi])) - 1 if gi.size else gi
    zz = ((g_out_delta.astype(np.int64) << 1) ^ (g_out_delta.astype(np.int64) >> 63)).astype(np.uint64)
    hs = huffman_size(grid_codes)
    return leb([hs]) + hs + leb(g_gap) + leb(zz)


def stream_bytes(host: dict, value_bytes: int | None = None, model: bytes | None = None) -> dict:
    """Section sizes (and "total") of the stream mc_stream_write produces for
    this compressed field, with the model file embedded when given.
    value_bytes is implied by the stored values and ignored."""
    return write_stream(host, model)[1]
