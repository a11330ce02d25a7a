// mc_batch.hip -- batched compression (under construction).
#include "mc_internal.h"

extern "C" mc_status mc_batch_compress(const mc_batch_item* items, int32_t n, hipStream_t s)
{
    if (!items || n < 0) return mc_fail(MC_ERR_ARG, "invalid batch");
    for (int32_t i = 0; i < n; ++i) {
        mc_status st = mc_compress(items[i].plan, items[i].d_field, items[i].dtype, &items[i].params, &items[i].codes, s);
        if (st != MC_OK) return st;
    }
    return MC_OK;
}
