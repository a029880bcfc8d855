// Ragged batches: placeholder until the persistent kernel lands.
#include "internal.hpp"

extern "C" {
int dct2d_ragged_plan_create(const dct2d_block*, int64_t, int, int, dct2d_ragged_plan** out)
{
    if (out) *out = nullptr;
    return DCT2D_ERR_ARG;
}
int dct2d_ragged_execute(dct2d_ragged_plan*, float*, void*) { return DCT2D_ERR_ARG; }
void dct2d_ragged_plan_destroy(dct2d_ragged_plan*) {}
int dct2d_ragged_plan_info(const dct2d_ragged_plan*, int64_t*, int32_t*, int32_t*) { return DCT2D_ERR_ARG; }
}
