"""The self-describing stream (host code, no GPU): every section written is
read back bit for bit, section sizes add up to the stream, the Huffman
sections respect the textbook bound, and damaged or truncated streams are
rejected with MC_ERR_FORMAT instead of being decoded."""
import ctypes as C

import numpy as np
import pytest

from paper_2501_06910_amd import mc as M


def fake_codes(rng, dim, dims, nv, dtype, n_gout, n_vout, learned):
    ng = int(np.prod(dims[:dim]))
    gc = (M.RADIUS + np.round(rng.normal(0, 3, ng))).astype(np.uint16)
    gi = np.sort(rng.choice(ng, n_gout, replace=False)).astype(np.int32)
    gc[gi] = 0
    gd = rng.integers(-(1 << 29), 1 << 29, n_gout).astype(np.int32)
    vc = (M.RADIUS + np.round(rng.laplace(0, 2, nv))).astype(np.uint16)
    vi = np.sort(rng.choice(nv, n_vout, replace=False)).astype(np.int32)
    vc[vi] = 0
    vv = rng.normal(size=n_vout).astype(dtype)
    nb = (nv + M.BLOCK - 1) // M.BLOCK
    bf = np.zeros((nb + 31) // 32, np.uint32)
    if learned:
        for b in rng.choice(nb, nb // 2, replace=False):
            bf[b >> 5] |= np.uint32(1 << (b & 31))
    r = dict(tau=1e-3, tau1=5e-4, tau2=5e-4, c=0.25, n_grid_outliers=n_gout, n_vertex_outliers=n_vout)
    return dict(result=r, grid_codes=gc, g_out_idx=gi, g_out_delta=gd, vert_codes=vc, v_out_idx=vi, v_out_val=vv,
                block_flags=bf, learned=learned,
                meta=dict(dim=dim, dims=tuple(dims) + (1,) * (3 - len(dims)),
                          dtype=M.F64 if dtype == np.float64 else M.F32, grid_predictor=2, residual_predictor=0))


CASES = [(2, (37, 41), 5000, np.float64, 0, 3, False),
         (3, (9, 10, 11), 9000, np.float32, 17, 40, True),
         (3, (4, 4, 4), 1, np.float32, 64, 1, False),          # every grid node an outlier, one vertex
         (2, (128, 128), 20000, np.float32, 5, 0, True)]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_roundtrip_every_section(case):
    rng = np.random.default_rng(case)
    h = fake_codes(rng, *CASES[case])
    model = bytes(rng.integers(0, 256, 333, dtype=np.uint8)) if case % 2 else None
    blob, sec = M.write_stream(h, model)
    assert len(blob) == sec["total"] == sum(v for k, v in sec.items() if k != "total")
    back = M.read_stream(blob)
    for k in ("grid_codes", "g_out_idx", "g_out_delta", "vert_codes", "v_out_idx"):
        assert np.array_equal(back[k], h[k]), k
    assert np.array_equal(back["v_out_val"].view(np.uint8), h["v_out_val"].view(np.uint8))
    if h["learned"]:
        assert np.array_equal(back["block_flags"], h["block_flags"])
    for k in ("tau", "tau1", "tau2", "c"):
        assert back["result"][k] == h["result"][k]
    assert back["meta"] == h["meta"]
    assert back["model"] == model
    # the stored sections are the documented encodings
    assert sec["grid"] >= M.huffman_size(h["grid_codes"]) + 1
    assert sec["vert_outliers"] >= h["v_out_idx"].size * h["v_out_val"].itemsize
    nb = (h["vert_codes"].size + 4095) // 4096
    assert sec["block_flags"] == ((nb + 7) // 8 if h["learned"] else 0)
    assert M.grid_stream_bytes(h["grid_codes"], h["g_out_idx"], h["g_out_delta"]) == \
        sec["grid"] + sec["grid_outliers"]


def test_huffman_sections_within_entropy_bound():
    """Coded bits of a Huffman section lie in [n H, n (H + 1)) (the textbook
    bound); the rest of the section is its code table and length prefix."""
    rng = np.random.default_rng(9)
    h = fake_codes(rng, 3, (40, 40, 40), 200000, np.float32, 0, 0, False)
    _, sec = M.write_stream(h)
    for name, sym in (("grid", h["grid_codes"]), ("vert", h["vert_codes"])):
        H = M.entropy_bits(sym)
        used = len(np.unique(sym))
        table = 4 + 3 * used
        bits = 8 * (sec[name] - table) - 8 * 4          # minus the table and a length prefix of <= 4 bytes
        assert bits <= sym.size * (H + 1) + 8
        assert 8 * (sec[name] - table) >= sym.size * H - 8


def test_serial_stream_roundtrip():
    rng = np.random.default_rng(3)
    n = 7777
    codes = (M.RADIUS + np.round(rng.normal(0, 5, n))).astype(np.uint16)
    oi = np.sort(rng.choice(n, 9, replace=False)).astype(np.int32)
    codes[oi] = 0
    host = dict(result=dict(tau=1e-2, tau1=1e-2, tau2=0.0, c=0.5), codes=codes, out_idx=oi,
                out_val=rng.normal(size=9).astype(np.float64))
    blob, sec = M.write_stream(host)
    assert sec["grid"] == 0 and sec["grid_outliers"] == 0
    back = M.read_stream(blob)
    assert np.array_equal(back["codes"], codes)
    assert np.array_equal(back["out_idx"], oi)
    assert np.array_equal(back["out_val"], host["out_val"])
    assert M.serial_stream_bytes(host)["total"] == len(blob)


def test_damaged_streams_are_rejected():
    rng = np.random.default_rng(5)
    h = fake_codes(rng, 3, (9, 10, 11), 9000, np.float32, 17, 40, True)
    blob, _ = M.write_stream(h, b"model-bytes")
    lib = M.lib()
    hdr = M.McStreamHeader()
    mb = C.c_int64()
    assert lib.mc_stream_read_header(blob, len(blob), C.byref(hdr), C.byref(mb)) == M.OK
    assert mb.value == len(b"model-bytes")
    for cut in (0, 3, 10, len(blob) // 2, len(blob) - 1):
        with pytest.raises(M.McError):
            M.read_stream(blob[:cut])
    for pos in (0, 5, 40, len(blob) // 3, len(blob) - 6):
        bad = bytearray(blob)
        bad[pos] ^= 0x20
        with pytest.raises(M.McError) as e:
            M.read_stream(bytes(bad))
        assert e.value.status == M.ERR_FORMAT
    # writer-side checks: descending outlier indices, out-of-range counts
    h2 = dict(h)
    h2["v_out_idx"] = h["v_out_idx"][::-1].copy()
    with pytest.raises(M.McError):
        M.write_stream(h2)
