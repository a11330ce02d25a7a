// mc_serial.hip -- host side of the 1-D serialisation baseline (the
// comparison of Sec. V-C): workspace, argument checks and the compress /
// decompress sequences.
//   compress:   k_range -> k_range_final -> k_ser_codes -> k_scatter
//   decompress: k_ser_tot -> k_ser_carry -> k_ser_apply
// mc_serial_compress_noalloc runs the same compress sequence on a
// fixed-size scratch array in device memory (one copy per GPU, resolved
// with hipGetSymbolAddress) instead of a context's allocations.
#include <cmath>
#include <mutex>
#include <vector>

#include "mc_internal.h"

struct mc_serial_s {
    long long n_max = 0, ntiles = 0;
    std::vector<void*> allocs;
    unsigned long long* ctl = nullptr;    // RangeOut at word 0, DevBound at word 16
    unsigned long long* partial = nullptr;
    unsigned int* small = nullptr;        // err at word 2, vsum from word 16
    long long nsmall = 0;
    unsigned int* count = nullptr;        // per tile
    int2* agg = nullptr;
    int* carry = nullptr;
};

template <typename T> static hipError_t ser_alloc(mc_serial s, T** out, size_t n)
{
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, n * sizeof(T) > 0 ? n * sizeof(T) : 16);
    if (e != hipSuccess) return e;
    s->allocs.push_back(q);
    *out = (T*)q;
    return hipSuccess;
}

extern "C" mc_status mc_serial_destroy(mc_serial s)
{
    if (!s) return MC_OK;
    for (void* q : s->allocs) (void)hipFree(q);
    delete s;
    return MC_OK;
}

extern "C" mc_status mc_serial_create(int64_t n_max, mc_serial* out)
{
    if (!out) return mc_fail(MC_ERR_ARG, "out pointer is NULL");
    *out = nullptr;
    if (n_max < 1 || n_max > 0x7fffffffLL) return mc_fail(MC_ERR_ARG, "n_max must be in [1, 2^31 - 1]");
    mc_serial s = new mc_serial_s;
    s->n_max = n_max;
    s->ntiles = (n_max + MC_TILE - 1) / MC_TILE;
    const long long ngv = (s->ntiles + MC_SC_TILES - 1) / MC_SC_TILES;
    s->nsmall = 16 + ngv;
    hipError_t e;
#define SCHK(x) do { if ((e = (x)) != hipSuccess) { mc_serial_destroy(s); return mc_fail(MC_ERR_NOMEM, "%s: %s", #x, hipGetErrorString(e)); } } while (0)
    SCHK(ser_alloc(s, &s->ctl, 64));
    SCHK(ser_alloc(s, &s->partial, (size_t)3 * MC_RANGE_BLOCKS));
    SCHK(ser_alloc(s, &s->small, (size_t)s->nsmall));
    SCHK(ser_alloc(s, &s->count, (size_t)s->ntiles));
    SCHK(ser_alloc(s, &s->agg, (size_t)s->ntiles));
    SCHK(ser_alloc(s, &s->carry, (size_t)s->ntiles));
    SCHK(hipMemset(s->ctl, 0, 64 * sizeof(unsigned long long)));
    SCHK(hipMemset(s->small, 0, (size_t)s->nsmall * 4));
    SCHK(hipDeviceSynchronize());
#undef SCHK
    *out = s;
    return MC_OK;
}

static mc_status ser_check_codes(const mc_codes* c)
{
    if (!c) return mc_fail(MC_ERR_ARG, "codes pointer is NULL");
    if (!c->vert_codes || !c->result) return mc_fail(MC_ERR_ARG, "vert_codes or result is NULL");
    if (c->v_out_cap < 0) return mc_fail(MC_ERR_ARG, "negative outlier capacity");
    if (c->v_out_cap > 0 && (!c->v_out_idx || !c->v_out_val)) return mc_fail(MC_ERR_ARG, "outlier buffers are NULL");
    return MC_OK;
}

extern "C" mc_status mc_serial_compress(mc_serial s, const void* d_field, mc_dtype dtype, int64_t n, double eb,
                                        int32_t eb_mode, const mc_codes* codes, hipStream_t stream)
{
    if (!s) return mc_fail(MC_ERR_ARG, "context is NULL");
    if (!d_field) return mc_fail(MC_ERR_ARG, "field pointer is NULL");
    if (dtype != MC_F32 && dtype != MC_F64) return mc_fail(MC_ERR_ARG, "dtype must be MC_F32 or MC_F64");
    if (n < 1 || n > s->n_max) return mc_fail(MC_ERR_ARG, "n = %lld outside [1, n_max = %lld]", (long long)n, s->n_max);
    if (!(eb > 0.0) || !std::isfinite(eb)) return mc_fail(MC_ERR_ARG, "eb must be finite and > 0");
    if (eb_mode != MC_EB_ABS && eb_mode != MC_EB_REL) return mc_fail(MC_ERR_ARG, "unknown eb_mode");
    mc_status st = ser_check_codes(codes);
    if (st != MC_OK) return st;
    BoundParams bp;
    bp.eb = eb;
    bp.split = 0.5;                       // tau1 / tau2 unused: the codes take the whole tau
    bp.relative = eb_mode == MC_EB_REL;
    bp.mode = MC_SPLIT_SUM;
    RangeOut* cur = (RangeOut*)s->ctl;
    DevBound* bound = (DevBound*)(s->ctl + 16);
    unsigned int* err = s->small + 2;
    unsigned int* vsum = s->small + 16;
    hipError_t e;
#define ECHK(x) do { if ((e = (x)) != hipSuccess) return mc_fail(MC_ERR_DEVICE, "%s: %s", #x, hipGetErrorString(e)); } while (0)
    ECHK(mck::range(d_field, dtype, n, s->partial, cur, bp, bound, s->small, s->nsmall, 0u, stream));
    ECHK(mck::serial_codes(d_field, dtype, n, bound, codes->vert_codes, s->count, vsum, err, codes->result, stream));
    ECHK(mck::compact(nullptr, 1, 1, 1, 0, 0, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 0, d_field, dtype, n,
                      codes->vert_codes, s->count, vsum, codes->v_out_idx, codes->v_out_val, codes->v_out_cap, err,
                      codes->result, stream));
#undef ECHK
    return MC_OK;
}

// ---- compress without allocation --------------------------------------------
// Scratch words of the compress sequence for n values (the layout of a
// context's allocations, packed): RangeOut/DevBound control block, range
// partials, the per-call counters that k_range clears (err at word 2,
// per-group outlier sums from word 16) and the per-tile outlier counts.
namespace {
constexpr long long kNoallocTiles = (MC_SERIAL_NOALLOC_MAX + MC_TILE - 1) / MC_TILE;
constexpr long long kNoallocGroups = (kNoallocTiles + MC_SC_TILES - 1) / MC_SC_TILES;
constexpr size_t kCtlBytes = 64 * 8;
constexpr size_t kPartialBytes = (size_t)3 * MC_RANGE_BLOCKS * 8;
constexpr size_t kSmallBytes = ((size_t)(16 + kNoallocGroups) * 4 + 255) / 256 * 256;
constexpr size_t kCountBytes = ((size_t)kNoallocTiles * 4 + 255) / 256 * 256;
constexpr size_t kScratchBytes = kCtlBytes + kPartialBytes + kSmallBytes + kCountBytes;
}  // namespace

// The scratch array itself.  Its name is only a host-side handle: device
// code gets the per-GPU address from hipGetSymbolAddress below.
static __device__ __align__(256) unsigned char scratch[(kScratchBytes + 255) / 256 * 256];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[64];           // per device, resolved once with that device current

static mc_status scratch_address(void** out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return mc_fail(MC_ERR_DEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= 64) return mc_fail(MC_ERR_UNSUPPORTED, "device index %d above 63", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return mc_fail(MC_ERR_DEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return MC_OK;
}

extern "C" int64_t mc_serial_noalloc_max(void) { return MC_SERIAL_NOALLOC_MAX; }

extern "C" mc_status mc_serial_compress_noalloc(const void* d_field, mc_dtype dtype, int64_t n, double eb,
                                                int32_t eb_mode, const mc_codes* codes, hipStream_t stream)
{
    if (!d_field) return mc_fail(MC_ERR_ARG, "field pointer is NULL");
    if (dtype != MC_F32 && dtype != MC_F64) return mc_fail(MC_ERR_ARG, "dtype must be MC_F32 or MC_F64");
    if (n < 1) return mc_fail(MC_ERR_ARG, "n = %lld must be at least 1", (long long)n);
    if (n > MC_SERIAL_NOALLOC_MAX)
        return mc_fail(MC_ERR_CAPACITY, "n = %lld above the no-allocation limit of %lld values", (long long)n,
                       (long long)MC_SERIAL_NOALLOC_MAX);
    if (!(eb > 0.0) || !std::isfinite(eb)) return mc_fail(MC_ERR_ARG, "eb must be finite and > 0");
    if (eb_mode != MC_EB_ABS && eb_mode != MC_EB_REL) return mc_fail(MC_ERR_ARG, "unknown eb_mode");
    mc_status st = ser_check_codes(codes);
    if (st != MC_OK) return st;
    void* base = nullptr;
    st = scratch_address(&base);
    if (st != MC_OK) return st;
    unsigned char* b = (unsigned char*)base;
    unsigned long long* ctl = (unsigned long long*)b;
    unsigned long long* partial = (unsigned long long*)(b + kCtlBytes);
    unsigned int* small = (unsigned int*)(b + kCtlBytes + kPartialBytes);
    unsigned int* count = (unsigned int*)(b + kCtlBytes + kPartialBytes + kSmallBytes);
    const long long ntiles = (n + MC_TILE - 1) / MC_TILE;
    const long long nsmall = 16 + (ntiles + MC_SC_TILES - 1) / MC_SC_TILES;
    BoundParams bp;
    bp.eb = eb;
    bp.split = 0.5;
    bp.relative = eb_mode == MC_EB_REL;
    bp.mode = MC_SPLIT_SUM;
    RangeOut* cur = (RangeOut*)ctl;
    DevBound* bound = (DevBound*)(ctl + 16);
    unsigned int* err = small + 2;
    unsigned int* vsum = small + 16;
    hipError_t e;
#define ECHK(x) do { if ((e = (x)) != hipSuccess) return mc_fail(MC_ERR_DEVICE, "%s: %s", #x, hipGetErrorString(e)); } while (0)
    // k_range clears small[0 .. nsmall) (err, the outlier sums) before anything reads it
    ECHK(mck::range(d_field, dtype, n, partial, cur, bp, bound, small, nsmall, 0u, stream));
    ECHK(mck::serial_codes(d_field, dtype, n, bound, codes->vert_codes, count, vsum, err, codes->result, stream));
    ECHK(mck::compact(nullptr, 1, 1, 1, 0, 0, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 0, d_field, dtype, n,
                      codes->vert_codes, count, vsum, codes->v_out_idx, codes->v_out_val, codes->v_out_cap, err,
                      codes->result, stream));
#undef ECHK
    return MC_OK;
}

extern "C" mc_status mc_serial_decompress(mc_serial s, const mc_codes* codes, int64_t n, void* d_out, mc_dtype dtype,
                                          hipStream_t stream)
{
    if (!s) return mc_fail(MC_ERR_ARG, "context is NULL");
    if (!d_out) return mc_fail(MC_ERR_ARG, "output pointer is NULL");
    if (dtype != MC_F32 && dtype != MC_F64) return mc_fail(MC_ERR_ARG, "dtype must be MC_F32 or MC_F64");
    if (n < 1 || n > s->n_max) return mc_fail(MC_ERR_ARG, "n = %lld outside [1, n_max = %lld]", (long long)n, s->n_max);
    mc_status st = ser_check_codes(codes);
    if (st != MC_OK) return st;
    hipError_t e = mck::serial_decode(codes->vert_codes, codes->v_out_idx, codes->v_out_val, codes->v_out_cap,
                                      codes->result, n, dtype, s->agg, s->carry, d_out, stream);
    if (e != hipSuccess) return mc_fail(MC_ERR_DEVICE, "serial_decode: %s", hipGetErrorString(e));
    return MC_OK;
}
