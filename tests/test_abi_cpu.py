"""CPU tests of the C ABI: libmc.so loads without a GPU, exports every
function include/mc.h declares, rejects bad arguments before any HIP call,
and its CPU entropy stage round-trips within the textbook Huffman bounds."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2501_06910_amd import mc as M

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "mc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mc_[a-z0-9_]+)\s*\(", src)))


def test_exports_every_declared_symbol():
    lib = M.lib()
    names = declared_functions()
    assert len(names) >= 30
    for n in names:
        assert hasattr(lib, n), n
        assert n in M._SIGS, f"binding lacks {n}"


def test_status_strings_and_version():
    lib = M.lib()
    assert lib.mc_abi_version() == 1
    for s in range(8):
        assert lib.mc_status_string(s)
    assert lib.mc_status_string(99) == b"unknown status"


def test_host_validation_before_device_work():
    lib = M.lib()
    out = C.c_void_p()
    g = M.make_grid(2, (8, 8, 1), (0, 0, 0), (1, 1, 1))
    fake = C.c_void_p(0x1000)   # never dereferenced: validation fails first
    # bad dimension / counts / pointers
    assert lib.mc_plan_create(fake, fake, 4, 10, 10, C.byref(g), None, None, C.byref(out)) == M.ERR_ARG
    assert lib.mc_plan_create(None, fake, 2, 10, 10, C.byref(g), None, None, C.byref(out)) == M.ERR_ARG
    assert lib.mc_plan_create(fake, None, 2, 10, 10, C.byref(g), None, None, C.byref(out)) == M.ERR_ARG
    assert lib.mc_plan_create(fake, fake, 2, 0, 10, C.byref(g), None, None, C.byref(out)) == M.ERR_ARG
    assert lib.mc_plan_create(fake, fake, 2, 10, -1, C.byref(g), None, None, C.byref(out)) == M.ERR_ARG
    bad = M.make_grid(2, (1, 8, 1), (0, 0, 0), (1, 1, 1))
    assert lib.mc_plan_create(fake, fake, 2, 10, 10, C.byref(bad), None, None, C.byref(out)) == M.ERR_ARG
    bad = M.make_grid(2, (8, 8, 1), (0, 0, 0), (0, 1, 1))
    assert lib.mc_plan_create(fake, fake, 2, 10, 10, C.byref(bad), None, None, C.byref(out)) == M.ERR_ARG
    wide = M.make_grid(2, (9000, 8, 1), (0, 0, 0), (1, 1, 1))
    assert lib.mc_plan_create(fake, fake, 2, 10, 10, C.byref(wide), None, None,
                              C.byref(out)) == M.ERR_UNSUPPORTED
    assert b"8192" in lib.mc_last_error()
    # compress / decompress on a NULL plan
    prm = M.McParams(1e-3, M.EB_REL, 0.5, None)
    codes = M.McCodes()
    assert lib.mc_compress(None, fake, M.F32, C.byref(prm), C.byref(codes), None) == M.ERR_ARG
    assert lib.mc_decompress(None, C.byref(codes), None, fake, M.F32, None) == M.ERR_ARG
    assert lib.mc_batch_compress(None, 1, None) == M.ERR_ARG
    # models
    assert lib.mc_model_param_count(2) == 9601
    assert lib.mc_model_param_count(3) == 12737
    assert lib.mc_model_param_count(4) == -1
    p = np.zeros(9601, np.float32)
    assert lib.mc_model_create(5, p.ctypes.data, 1.0, C.byref(out)) == M.ERR_ARG
    assert lib.mc_model_create(2, p.ctypes.data, 0.0, C.byref(out)) == M.ERR_ARG
    p[3] = np.nan
    assert lib.mc_model_create(2, p.ctypes.data, 1.0, C.byref(out)) == M.ERR_ARG
    junk = b"not a model file at all"
    assert lib.mc_model_import(junk, len(junk), C.byref(out)) == M.ERR_FORMAT
    # grids
    assert lib.mc_grid_from_dims(None, 2, 10, None, None, C.byref(g)) == M.ERR_ARG
    # tuning
    t = M.McTuning(0x7F)
    assert lib.mc_plan_get_tuning(None, C.byref(t)) == M.ERR_ARG
    assert lib.mc_plan_set_tuning(None, C.byref(t)) == M.ERR_ARG
    assert lib.mc_plan_tune(None, fake, M.F32, C.byref(prm), C.byref(codes), fake, 3, None, None) == M.ERR_ARG
    # batches
    assert lib.mc_batch_decompress(None, 1, None) == M.ERR_ARG
    assert lib.mc_batch_compress(fake, 0, None) == M.ERR_ARG
    # grid initialisation
    assert lib.mc_grid_from_percentile(None, fake, 2, 10, 10, 50.0, 100, None, C.byref(g), None) == M.ERR_ARG
    assert lib.mc_grid_from_percentile(fake, fake, 2, 10, 10, 150.0, 100, None, C.byref(g), None) == M.ERR_ARG
    assert lib.mc_grid_from_percentile(fake, fake, 2, 10, 10, 50.0, 1, None, C.byref(g), None) == M.ERR_ARG
    # operator pairs
    bad_ops = M.McPlanOpts(M.FILL_NEAREST, 0, 7)
    assert lib.mc_plan_create(fake, None, 2, 10, 0, C.byref(g), C.byref(bad_ops), None, C.byref(out)) == M.ERR_ARG
    lin = M.McPlanOpts(M.FILL_NEAREST, 0, M.OPS_LINEAR)
    assert lib.mc_plan_create(fake, None, 2, 10, 0, C.byref(g), C.byref(lin), None, C.byref(out)) == M.ERR_ARG
    assert lib.mc_plan_nodes(None, fake, None) == M.ERR_ARG
    # 1-D serialisation baseline
    assert lib.mc_serial_create(0, C.byref(out)) == M.ERR_ARG
    assert lib.mc_serial_create(1 << 31, C.byref(out)) == M.ERR_ARG
    assert lib.mc_serial_create(16, None) == M.ERR_ARG
    assert lib.mc_serial_destroy(None) == M.OK
    assert lib.mc_serial_compress(None, fake, M.F32, 16, 1e-3, M.EB_REL, C.byref(codes), None) == M.ERR_ARG
    assert lib.mc_serial_decompress(None, C.byref(codes), 16, fake, M.F32, None) == M.ERR_ARG
    # bin tuning: arguments checked on the host
    cand = (C.c_int32 * 2)(1, 2)
    best = C.c_int32()
    assert lib.mc_plan_tune_bins(fake, None, 2, 10, 10, C.byref(g), cand, 2, None, C.byref(best), None) == M.ERR_ARG
    assert lib.mc_plan_tune_bins(fake, fake, 2, 10, 10, C.byref(g), cand, 0, None, C.byref(best), None) == M.ERR_ARG
    bad_c = (C.c_int32 * 1)(65)
    assert lib.mc_plan_tune_bins(fake, fake, 2, 10, 10, C.byref(g), bad_c, 1, None, C.byref(best), None) == M.ERR_ARG
    # the allocation-free compress: limits and pointers checked on the host
    assert lib.mc_serial_noalloc_max() == 1 << 28
    assert lib.mc_serial_compress_noalloc(None, M.F32, 16, 1e-3, M.EB_REL, C.byref(codes), None) == M.ERR_ARG
    assert lib.mc_serial_compress_noalloc(fake, M.F32, 0, 1e-3, M.EB_REL, C.byref(codes), None) == M.ERR_ARG
    assert lib.mc_serial_compress_noalloc(fake, M.F32, (1 << 28) + 1, 1e-3, M.EB_REL, C.byref(codes),
                                          None) == M.ERR_CAPACITY
    assert b"no-allocation limit" in lib.mc_last_error()
    assert lib.mc_serial_compress_noalloc(fake, M.F32, 16, 0.0, M.EB_REL, C.byref(codes), None) == M.ERR_ARG


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_huffman_roundtrip_and_bounds(seed):
    rng = np.random.default_rng(seed)
    n = 100000
    if seed == 0:
        sym = (32768 + np.round(rng.laplace(0, 3, n))).astype(np.uint16)
    elif seed == 1:
        sym = rng.integers(0, 65536, n).astype(np.uint16)
    else:
        sym = np.full(n, 32768, np.uint16)
        sym[::97] = 32769
    blob = M.huffman_encode(sym)
    assert len(blob) == M.huffman_size(sym)
    back = M.huffman_decode(blob, n)
    assert np.array_equal(back, sym)
    H = M.entropy_bits(sym)
    used = len(np.unique(sym))
    payload_bits = (len(blob) - 4 - 3 * used) * 8
    assert n * H <= payload_bits + 8
    assert payload_bits < n * (H + 1) + 8


def test_huffman_decode_rejects_garbage():
    with pytest.raises(ValueError):
        M.huffman_decode(b"\x05\x00\x00\x00\x01", 10)


def test_entropy_of_uniform_and_constant():
    assert M.entropy_bits(np.full(1000, 7, np.uint16)) == 0.0
    sym = np.repeat(np.arange(256, dtype=np.uint16), 64)
    assert abs(M.entropy_bits(sym) - 8.0) < 1e-12
