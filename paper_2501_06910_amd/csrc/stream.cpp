// stream.cpp -- the self-describing compressed stream (host, outside the hot
// path).  The compression ratio of the method is the original size over the
// compressed size (Sec. IV-A, with the mesh, grid and mapping excluded as
// reusable state); this file assembles the compressed size from real bytes
// and reads them back.
//
// Layout (all integers little-endian; varint = unsigned LEB128):
//   "MCS1"  u16 version  u8 dim (1: the 1-D serialisation baseline, whose
//           stream has no grid sections)  u8 dtype  u8 grid_predictor
//           u8 residual_predictor  u8 flags (bit 0 learned, bit 1 model)  u8 0
//   varint dims[0..dim-1], varint n_vertices
//   f64 tau, tau1, tau2, c
//   varint n_grid_outliers, varint n_vertex_outliers
//   varint bytes, canonical Huffman of the grid codes (mc_huffman_encode)
//   varint bytes, canonical Huffman of the vertex codes
//   grid outliers:   varint index gap (i_k - i_{k-1} - 1, i_{-1} = -1) each,
//                    then varint zigzag(delta) each
//   vertex outliers: varint index gap each, then the raw values (4 or 8 B)
//   learned only: the block flags, ceil(n_blocks / 8) bytes, bit b of byte
//                 b / 8 = block b
//   model only:   varint bytes, the model file (mc_model_export)
//   u32 FNV-1a of every byte before it
#include <stdint.h>
#include <string.h>

#include <vector>

#include "../../include/mc.h"

mc_status mc_fail(mc_status s, const char* fmt, ...);

namespace {

constexpr uint16_t kVersion = 1;
constexpr int kSections = 8;

struct Writer {
    std::vector<uint8_t> b;
    void u8(uint8_t v) { b.push_back(v); }
    void raw(const void* p, size_t n)
    {
        const uint8_t* q = (const uint8_t*)p;
        b.insert(b.end(), q, q + n);
    }
    void var(uint64_t v)
    {
        do {
            uint8_t c = v & 0x7f;
            v >>= 7;
            if (v) c |= 0x80;
            b.push_back(c);
        } while (v);
    }
};

struct Reader {
    const uint8_t* p;
    int64_t n, at = 0;
    bool ok = true;
    bool need(int64_t k)
    {
        if (!ok || k < 0 || at + k > n) ok = false;
        return ok;
    }
    uint8_t u8() { return need(1) ? p[at++] : 0; }
    void raw(void* dst, int64_t k)
    {
        if (!need(k)) return;
        memcpy(dst, p + at, (size_t)k);
        at += k;
    }
    uint64_t var()
    {
        uint64_t v = 0;
        for (int s = 0; s < 64; s += 7) {
            if (!need(1)) return 0;
            const uint8_t c = p[at++];
            v |= (uint64_t)(c & 0x7f) << s;
            if (!(c & 0x80)) return v;
        }
        ok = false;
        return 0;
    }
};

uint32_t fnv1a(const uint8_t* p, size_t n)
{
    uint32_t h = 2166136261u;
    for (size_t i = 0; i < n; ++i) {
        h ^= p[i];
        h *= 16777619u;
    }
    return h;
}

int64_t n_grid_of(const mc_stream_header* h)
{
    if (h->dim == 1) return 0;
    return h->dims[0] * h->dims[1] * (h->dim == 3 ? h->dims[2] : 1);
}

mc_status check_header(const mc_stream_header* h)
{
    if (!h) return mc_fail(MC_ERR_ARG, "header is NULL");
    if (h->dim < 1 || h->dim > 3) return mc_fail(MC_ERR_ARG, "dim must be 1 (serial), 2 or 3");
    if (h->dtype != MC_F32 && h->dtype != MC_F64) return mc_fail(MC_ERR_ARG, "dtype must be MC_F32 or MC_F64");
    if (h->dim > 1)
        for (int d = 0; d < h->dim; ++d)
            if (h->dims[d] < 2 || h->dims[d] > (1LL << 31)) return mc_fail(MC_ERR_ARG, "grid dims out of range");
    if (h->dim == 2 && h->dims[2] != 1) return mc_fail(MC_ERR_ARG, "2-D grids have dims[2] = 1");
    if (h->n_vertices < 1 || h->n_vertices > (1LL << 31)) return mc_fail(MC_ERR_ARG, "n_vertices out of range");
    if (h->n_grid_outliers < 0 || h->n_grid_outliers > n_grid_of(h) || h->n_vertex_outliers < 0 ||
        h->n_vertex_outliers > h->n_vertices)
        return mc_fail(MC_ERR_ARG, "outlier counts out of range");
    if (h->grid_predictor < 0 || h->grid_predictor > 3 || h->residual_predictor < 0 || h->residual_predictor > 1)
        return mc_fail(MC_ERR_ARG, "unknown predictor");
    return MC_OK;
}

// Encodes into w; section_bytes (may be NULL) receives the size of each part.
mc_status encode(const mc_stream_header* h, const mc_stream_arrays* a, const void* model, int64_t model_bytes,
                 Writer& w, int64_t* section_bytes)
{
    mc_status st = check_header(h);
    if (st != MC_OK) return st;
    if (!a || (!a->grid_codes && h->dim > 1) || !a->vert_codes) return mc_fail(MC_ERR_ARG, "code arrays are NULL");
    if (h->n_grid_outliers > 0 && (!a->g_out_idx || !a->g_out_delta)) return mc_fail(MC_ERR_ARG, "grid outliers NULL");
    if (h->n_vertex_outliers > 0 && (!a->v_out_idx || !a->v_out_val)) return mc_fail(MC_ERR_ARG, "vertex outliers NULL");
    if (h->learned && !a->block_flags) return mc_fail(MC_ERR_ARG, "block flags are NULL in learned mode");
    if (model_bytes < 0 || (model_bytes > 0 && !model)) return mc_fail(MC_ERR_ARG, "model bytes without a model");
    const int64_t ng = n_grid_of(h), nv = h->n_vertices;
    int64_t sec[kSections] = {0};
    size_t mark = w.b.size();
    // header
    w.raw("MCS1", 4);
    w.u8(kVersion & 0xff);
    w.u8(kVersion >> 8);
    w.u8((uint8_t)h->dim);
    w.u8((uint8_t)h->dtype);
    w.u8((uint8_t)h->grid_predictor);
    w.u8((uint8_t)h->residual_predictor);
    w.u8((uint8_t)((h->learned ? 1 : 0) | (model_bytes > 0 ? 2 : 0)));
    w.u8(0);
    if (h->dim > 1)
        for (int d = 0; d < h->dim; ++d) w.var((uint64_t)h->dims[d]);
    w.var((uint64_t)nv);
    const double f[4] = {h->tau, h->tau1, h->tau2, h->c};
    w.raw(f, sizeof f);
    w.var((uint64_t)h->n_grid_outliers);
    w.var((uint64_t)h->n_vertex_outliers);
    sec[0] = (int64_t)(w.b.size() - mark);
    // Huffman sections
    for (int s = 0; s < 2; ++s) {
        mark = w.b.size();
        if (s == 0 && h->dim == 1) continue;            // no grid in the serial stream
        const uint16_t* sym = s == 0 ? a->grid_codes : a->vert_codes;
        const int64_t n = s == 0 ? ng : nv;
        const int64_t sz = mc_huffman_size(sym, n);
        if (sz < 0) return mc_fail(MC_ERR_ARG, "Huffman size failed");
        std::vector<uint8_t> buf((size_t)sz);
        const int64_t got = mc_huffman_encode(sym, n, buf.data(), sz);
        if (got != sz) return mc_fail(MC_ERR_DEVICE, "Huffman encoder wrote %lld of %lld bytes", (long long)got,
                                      (long long)sz);
        w.var((uint64_t)sz);
        w.raw(buf.data(), (size_t)sz);
        sec[1 + s] = (int64_t)(w.b.size() - mark);
    }
    // grid outliers
    mark = w.b.size();
    long long prev = -1;
    for (int64_t k = 0; k < h->n_grid_outliers; ++k) {
        const long long i = a->g_out_idx[k];
        if (i <= prev || i >= ng) return mc_fail(MC_ERR_ARG, "grid outlier indices not ascending in the grid");
        w.var((uint64_t)(i - prev - 1));
        prev = i;
    }
    for (int64_t k = 0; k < h->n_grid_outliers; ++k) {
        const int64_t d = a->g_out_delta[k];
        w.var(((uint64_t)d << 1) ^ (uint64_t)(d >> 63));
    }
    sec[3] = (int64_t)(w.b.size() - mark);
    // vertex outliers
    mark = w.b.size();
    prev = -1;
    for (int64_t k = 0; k < h->n_vertex_outliers; ++k) {
        const long long i = a->v_out_idx[k];
        if (i <= prev || i >= nv) return mc_fail(MC_ERR_ARG, "vertex outlier indices not ascending in the mesh");
        w.var((uint64_t)(i - prev - 1));
        prev = i;
    }
    const size_t ts = h->dtype == MC_F64 ? 8 : 4;
    if (h->n_vertex_outliers > 0) w.raw(a->v_out_val, (size_t)h->n_vertex_outliers * ts);
    sec[4] = (int64_t)(w.b.size() - mark);
    // block flags
    mark = w.b.size();
    if (h->learned) {
        const int64_t nb = (nv + MC_BLOCK - 1) / MC_BLOCK;
        for (int64_t i = 0; i < (nb + 7) / 8; ++i) {
            uint8_t c = 0;
            for (int k = 0; k < 8; ++k) {
                const int64_t b = 8 * i + k;
                if (b < nb && ((a->block_flags[b >> 5] >> (b & 31)) & 1u)) c |= (uint8_t)(1u << k);
            }
            w.u8(c);
        }
    }
    sec[5] = (int64_t)(w.b.size() - mark);
    // model
    mark = w.b.size();
    if (model_bytes > 0) {
        w.var((uint64_t)model_bytes);
        w.raw(model, (size_t)model_bytes);
    }
    sec[6] = (int64_t)(w.b.size() - mark);
    const uint32_t crc = fnv1a(w.b.data(), w.b.size());
    w.raw(&crc, 4);
    sec[7] = 4;
    if (section_bytes)
        for (int k = 0; k < kSections; ++k) section_bytes[k] = sec[k];
    return MC_OK;
}

// Parses the header; on success r is positioned at the first section.
mc_status parse_header(Reader& r, mc_stream_header* h, int64_t* model_bytes)
{
    if (r.n < 4 + 4) return mc_fail(MC_ERR_FORMAT, "stream shorter than its header");
    const uint32_t crc = (uint32_t)r.p[r.n - 4] | ((uint32_t)r.p[r.n - 3] << 8) | ((uint32_t)r.p[r.n - 2] << 16) |
                         ((uint32_t)r.p[r.n - 1] << 24);
    if (fnv1a(r.p, (size_t)(r.n - 4)) != crc) return mc_fail(MC_ERR_FORMAT, "stream checksum mismatch");
    r.n -= 4;
    char magic[4];
    r.raw(magic, 4);
    if (!r.ok || memcmp(magic, "MCS1", 4) != 0) return mc_fail(MC_ERR_FORMAT, "not a stream (magic)");
    const uint16_t ver = (uint16_t)(r.u8() | (r.u8() << 8));
    if (ver != kVersion) return mc_fail(MC_ERR_FORMAT, "stream version %u unsupported", (unsigned)ver);
    memset(h, 0, sizeof *h);
    h->dim = r.u8();
    h->dtype = r.u8();
    h->grid_predictor = r.u8();
    h->residual_predictor = r.u8();
    const uint8_t flags = r.u8();
    (void)r.u8();
    h->learned = flags & 1;
    if (h->dim < 1 || h->dim > 3) return mc_fail(MC_ERR_FORMAT, "bad dim in stream");
    h->dims[0] = h->dims[1] = h->dims[2] = 1;
    if (h->dim > 1)
        for (int d = 0; d < h->dim; ++d) h->dims[d] = (int64_t)r.var();
    h->n_vertices = (int64_t)r.var();
    double f[4];
    r.raw(f, sizeof f);
    h->tau = f[0];
    h->tau1 = f[1];
    h->tau2 = f[2];
    h->c = f[3];
    h->n_grid_outliers = (int64_t)r.var();
    h->n_vertex_outliers = (int64_t)r.var();
    if (!r.ok) return mc_fail(MC_ERR_FORMAT, "truncated stream header");
    if (check_header(h) != MC_OK) return mc_fail(MC_ERR_FORMAT, "stream header out of range");
    *model_bytes = (flags & 2) ? -1 : 0;        // size known once the sections before it are walked
    return MC_OK;
}

}  // namespace

extern "C" int64_t mc_stream_size(const mc_stream_header* hdr, const mc_stream_arrays* a, const void* model,
                                  int64_t model_bytes, int64_t* section_bytes)
{
    Writer w;
    if (encode(hdr, a, model, model_bytes, w, section_bytes) != MC_OK) return -1;
    return (int64_t)w.b.size();
}

extern "C" int64_t mc_stream_write(const mc_stream_header* hdr, const mc_stream_arrays* a, const void* model,
                                   int64_t model_bytes, uint8_t* h_out, int64_t cap, int64_t* section_bytes)
{
    if (!h_out || cap < 0) {
        mc_fail(MC_ERR_ARG, "output buffer is NULL");
        return -1;
    }
    Writer w;
    if (encode(hdr, a, model, model_bytes, w, section_bytes) != MC_OK) return -1;
    if ((int64_t)w.b.size() > cap) {
        mc_fail(MC_ERR_CAPACITY, "stream needs %lld bytes, capacity %lld", (long long)w.b.size(), (long long)cap);
        return -1;
    }
    memcpy(h_out, w.b.data(), w.b.size());
    return (int64_t)w.b.size();
}

extern "C" mc_status mc_stream_read_header(const uint8_t* h_in, int64_t n, mc_stream_header* hdr,
                                           int64_t* model_bytes)
{
    if (!h_in || n < 0 || !hdr) return mc_fail(MC_ERR_ARG, "invalid stream arguments");
    Reader r{h_in, n};
    int64_t mb = 0;
    mc_status st = parse_header(r, hdr, &mb);
    if (st != MC_OK) return st;
    if (model_bytes) {
        *model_bytes = 0;
        if (mb < 0) {
            // walk the sections to the model's length prefix
            for (int s = hdr->dim == 1 ? 1 : 0; s < 2; ++s) {
                const uint64_t sz = r.var();
                if (!r.need((int64_t)sz)) break;
                r.at += (int64_t)sz;
            }
            for (int64_t k = 0; k < 2 * hdr->n_grid_outliers + hdr->n_vertex_outliers; ++k) (void)r.var();
            r.at += hdr->n_vertex_outliers * (hdr->dtype == MC_F64 ? 8 : 4);
            if (hdr->learned) r.at += ((hdr->n_vertices + MC_BLOCK - 1) / MC_BLOCK + 7) / 8;
            const int64_t m = (int64_t)r.var();
            if (!r.ok || m < 0 || r.at + m != r.n) return mc_fail(MC_ERR_FORMAT, "malformed model section");
            *model_bytes = m;
        }
    }
    return MC_OK;
}

extern "C" mc_status mc_stream_read(const uint8_t* h_in, int64_t n, const mc_stream_arrays* a, void* model,
                                    int64_t model_cap)
{
    if (!h_in || n < 0 || !a || !a->vert_codes) return mc_fail(MC_ERR_ARG, "invalid stream arguments");
    Reader r{h_in, n};
    mc_stream_header h;
    int64_t mb = 0;
    mc_status st = parse_header(r, &h, &mb);
    if (st != MC_OK) return st;
    if (h.n_grid_outliers > 0 && (!a->g_out_idx || !a->g_out_delta)) return mc_fail(MC_ERR_ARG, "grid outliers NULL");
    if (h.n_vertex_outliers > 0 && (!a->v_out_idx || !a->v_out_val)) return mc_fail(MC_ERR_ARG, "vertex outliers NULL");
    if (h.learned && !a->block_flags) return mc_fail(MC_ERR_ARG, "block flags are NULL in learned mode");
    if (h.dim > 1 && !a->grid_codes) return mc_fail(MC_ERR_ARG, "grid codes buffer is NULL");
    const int64_t ng = n_grid_of(&h), nv = h.n_vertices;
    for (int s = h.dim == 1 ? 1 : 0; s < 2; ++s) {
        const int64_t sz = (int64_t)r.var();
        if (!r.need(sz)) return mc_fail(MC_ERR_FORMAT, "truncated Huffman section");
        uint16_t* sym = s == 0 ? a->grid_codes : a->vert_codes;
        const int64_t cnt = s == 0 ? ng : nv;
        const int64_t used = mc_huffman_decode(r.p + r.at, sz, sym, cnt);
        if (used != sz) return mc_fail(MC_ERR_FORMAT, "Huffman section malformed");
        r.at += sz;
    }
    long long prev = -1;
    for (int64_t k = 0; k < h.n_grid_outliers; ++k) {
        const long long i = prev + 1 + (long long)r.var();
        if (!r.ok || i >= ng) return mc_fail(MC_ERR_FORMAT, "grid outlier index out of range");
        a->g_out_idx[k] = (int32_t)i;
        prev = i;
    }
    for (int64_t k = 0; k < h.n_grid_outliers; ++k) {
        const uint64_t z = r.var();
        const int64_t d = (int64_t)(z >> 1) ^ -(int64_t)(z & 1);
        if (!r.ok || d < INT32_MIN || d > INT32_MAX) return mc_fail(MC_ERR_FORMAT, "grid outlier value out of range");
        a->g_out_delta[k] = (int32_t)d;
    }
    prev = -1;
    for (int64_t k = 0; k < h.n_vertex_outliers; ++k) {
        const long long i = prev + 1 + (long long)r.var();
        if (!r.ok || i >= nv) return mc_fail(MC_ERR_FORMAT, "vertex outlier index out of range");
        a->v_out_idx[k] = (int32_t)i;
        prev = i;
    }
    r.raw(a->v_out_val, h.n_vertex_outliers * (h.dtype == MC_F64 ? 8 : 4));
    if (h.learned) {
        const int64_t nb = (nv + MC_BLOCK - 1) / MC_BLOCK;
        const int64_t nw = (nb + 31) / 32;
        for (int64_t i = 0; i < nw; ++i) a->block_flags[i] = 0u;
        for (int64_t i = 0; i < (nb + 7) / 8; ++i) {
            const uint8_t c = r.u8();
            for (int k = 0; k < 8; ++k) {
                const int64_t b = 8 * i + k;
                if (b < nb && ((c >> k) & 1)) a->block_flags[b >> 5] |= 1u << (b & 31);
            }
        }
    }
    if (mb < 0) {
        const int64_t m = (int64_t)r.var();
        if (!r.need(m)) return mc_fail(MC_ERR_FORMAT, "truncated model section");
        if (model) {
            if (model_cap < m) return mc_fail(MC_ERR_CAPACITY, "model needs %lld bytes", (long long)m);
            memcpy(model, r.p + r.at, (size_t)m);
        }
        r.at += m;
    }
    if (!r.ok || r.at != r.n) return mc_fail(MC_ERR_FORMAT, "stream has %lld trailing or missing bytes",
                                             (long long)(r.n - r.at));
    return MC_OK;
}
