// entropy.cpp -- CPU entropy stage (outside the hot path): canonical
// Huffman coding of uint16 quantisation codes with code lengths limited to
// 24 bits, used to report the compression ratio S / (stream bytes) (the
// paper's ratio of original to compressed size, Sec. IV-A).
//
// Stream layout: u32 n_used, then n_used records (u16 symbol, u8 length) in
// canonical order (length, symbol), then the code bits MSB-first.
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <queue>
#include <vector>

#include "../../include/mc.h"

namespace {

constexpr int kMaxLen = 24;

// Huffman code lengths of the symbols with non-zero frequency; lengths over
// kMaxLen are avoided by flattening the frequencies and rebuilding.
std::vector<uint8_t> code_lengths(std::vector<uint64_t> freq)
{
    const size_t n = freq.size();
    std::vector<uint8_t> len(n, 0);
    for (int attempt = 0; attempt < 64; ++attempt) {
        std::vector<int> used;
        for (size_t i = 0; i < n; ++i)
            if (freq[i]) used.push_back((int)i);
        if (used.empty()) return len;
        if (used.size() == 1) {
            len[used[0]] = 1;
            return len;
        }
        // nodes: leaves 0..m-1, internal m..; parent links
        const size_t m = used.size();
        std::vector<uint64_t> w(2 * m);
        std::vector<int> parent(2 * m, -1);
        typedef std::pair<uint64_t, int> E;
        std::priority_queue<E, std::vector<E>, std::greater<E>> pq;
        for (size_t i = 0; i < m; ++i) {
            w[i] = freq[used[i]];
            pq.push(E(w[i], (int)i));
        }
        int next = (int)m;
        while (pq.size() > 1) {
            E a = pq.top(); pq.pop();
            E b = pq.top(); pq.pop();
            w[next] = a.first + b.first;
            parent[a.second] = next;
            parent[b.second] = next;
            pq.push(E(w[next], next));
            ++next;
        }
        int maxl = 0;
        std::vector<int> depth(next, 0);
        for (int k = next - 2; k >= 0; --k) depth[k] = depth[parent[k]] + 1;
        for (size_t i = 0; i < m; ++i) maxl = std::max(maxl, depth[i]);
        if (maxl <= kMaxLen) {
            for (size_t i = 0; i < m; ++i) len[used[i]] = (uint8_t)depth[i];
            return len;
        }
        for (size_t i = 0; i < n; ++i)
            if (freq[i]) freq[i] = (freq[i] >> 1) | 1u;
    }
    return len;
}

struct Canon {
    std::vector<uint16_t> order;    // symbols sorted by (length, symbol)
    std::vector<uint8_t> len;       // per order entry
    std::vector<uint32_t> code;     // per order entry
};

Canon canonical(const std::vector<uint8_t>& lens)
{
    Canon c;
    for (size_t s = 0; s < lens.size(); ++s)
        if (lens[s]) c.order.push_back((uint16_t)s);
    std::stable_sort(c.order.begin(), c.order.end(),
                     [&](uint16_t a, uint16_t b) { return lens[a] < lens[b]; });
    uint32_t code = 0;
    int prev = 0;
    for (uint16_t s : c.order) {
        const int l = lens[s];
        code <<= (l - prev);
        prev = l;
        c.len.push_back((uint8_t)l);
        c.code.push_back(code);
        ++code;
    }
    return c;
}

std::vector<uint64_t> histogram(const uint16_t* sym, int64_t n)
{
    std::vector<uint64_t> f(65536, 0);
    for (int64_t i = 0; i < n; ++i) f[sym[i]]++;
    return f;
}

}  // namespace

extern "C" int64_t mc_huffman_size(const uint16_t* sym, int64_t n)
{
    if (n < 0 || (n > 0 && !sym)) return -1;
    std::vector<uint64_t> f = histogram(sym, n);
    std::vector<uint8_t> lens = code_lengths(f);
    int64_t used = 0;
    uint64_t bits = 0;
    for (size_t s = 0; s < lens.size(); ++s)
        if (lens[s]) { ++used; bits += (uint64_t)lens[s] * f[s]; }
    return 4 + 3 * used + (int64_t)((bits + 7) / 8);
}

extern "C" int64_t mc_huffman_encode(const uint16_t* sym, int64_t n, uint8_t* out, int64_t cap)
{
    if (n < 0 || (n > 0 && !sym) || !out) return -1;
    std::vector<uint64_t> f = histogram(sym, n);
    std::vector<uint8_t> lens = code_lengths(f);
    Canon c = canonical(lens);
    std::vector<uint32_t> code_of(65536, 0);
    for (size_t k = 0; k < c.order.size(); ++k) code_of[c.order[k]] = c.code[k];
    const int64_t need = mc_huffman_size(sym, n);
    if (need > cap) return -1;
    const uint32_t used = (uint32_t)c.order.size();
    memcpy(out, &used, 4);
    int64_t pos = 4;
    for (size_t k = 0; k < c.order.size(); ++k) {
        out[pos++] = (uint8_t)(c.order[k] & 0xff);
        out[pos++] = (uint8_t)(c.order[k] >> 8);
        out[pos++] = c.len[k];
    }
    uint64_t acc = 0;
    int nacc = 0;
    for (int64_t i = 0; i < n; ++i) {
        const int l = lens[sym[i]];
        acc = (acc << l) | code_of[sym[i]];
        nacc += l;
        while (nacc >= 8) {
            out[pos++] = (uint8_t)(acc >> (nacc - 8));
            nacc -= 8;
        }
    }
    if (nacc > 0) out[pos++] = (uint8_t)(acc << (8 - nacc));
    return pos;
}

extern "C" int64_t mc_huffman_decode(const uint8_t* in, int64_t n_in, uint16_t* sym, int64_t n)
{
    if (!in || n_in < 4 || (n > 0 && !sym)) return -1;
    uint32_t used;
    memcpy(&used, in, 4);
    if ((int64_t)4 + 3ll * used > n_in || used > 65536) return -1;
    std::vector<uint16_t> order(used);
    std::vector<uint8_t> len(used);
    int64_t pos = 4;
    for (uint32_t k = 0; k < used; ++k) {
        order[k] = (uint16_t)(in[pos] | (in[pos + 1] << 8));
        len[k] = in[pos + 2];
        if (len[k] == 0 || len[k] > kMaxLen || (k > 0 && len[k] < len[k - 1])) return -1;
        pos += 3;
    }
    if (used == 0) return n == 0 ? pos : -1;
    // canonical tables: first code and first index per length
    int64_t first_code[kMaxLen + 2], first_idx[kMaxLen + 2], count[kMaxLen + 2];
    memset(count, 0, sizeof count);
    for (uint32_t k = 0; k < used; ++k) count[len[k]]++;
    int64_t code = 0, idx = 0;
    for (int l = 1; l <= kMaxLen; ++l) {
        code <<= 1;
        first_code[l] = code;
        first_idx[l] = idx;
        code += count[l];
        idx += count[l];
    }
    uint64_t acc = 0;
    int nacc = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t c = 0;
        int l = 0;
        for (;;) {
            if (nacc == 0) {
                if (pos >= n_in) return -1;
                acc = in[pos++];
                nacc = 8;
            }
            c = (c << 1) | (int64_t)((acc >> (nacc - 1)) & 1u);
            --nacc;
            ++l;
            if (l > kMaxLen) return -1;
            if (count[l] && c - first_code[l] < count[l] && c >= first_code[l]) {
                sym[i] = order[first_idx[l] + (c - first_code[l])];
                break;
            }
        }
    }
    return pos;
}

extern "C" double mc_entropy_bits(const uint16_t* sym, int64_t n)
{
    if (n <= 0 || !sym) return 0.0;
    std::vector<uint64_t> f = histogram(sym, n);
    double h = 0.0;
    for (uint64_t c : f)
        if (c) {
            const double p = (double)c / (double)n;
            h -= p * std::log2(p);
        }
    return h;
}
