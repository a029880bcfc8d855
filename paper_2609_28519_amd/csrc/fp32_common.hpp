// Helpers shared by the float32 kernel translation units (kern_fp32.hip, kern_rect256.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "dct1d.hpp"
#include "internal.hpp"

namespace dct {
namespace {

// Returns p unchanged but opaque to the optimiser.  Used once per tile iteration so the
// twiddle loads (scalar, cache-resident) are re-issued inside the loop instead of being
// hoisted out of it, which would pin ~L twiddles in scalar registers for the whole
// kernel and spill them.
__device__ __forceinline__ twptr per_iteration(const float2* p)
{
    asm volatile("" : "+s"(p));
    return (twptr)p;
}

template <int L, int DIR>
__device__ __forceinline__ void apply1d(float (&v)[L], twptr tw)
{
    if (DIR == DCT2D_FORWARD) {
        dct2_ortho<L>(v, tw);
    } else if (DIR == DCT2D_INVERSE) {
        dct3_ortho<L>(v, tw);
    } else {
        dct2_ortho<L>(v, tw);
        // re-read the (identical) twiddles for the inverse instead of keeping the
        // forward's values live in scalar registers across both transforms
        asm volatile("" : "+s"(tw));
        dct3_ortho<L>(v, tw);
    }
}

// Spectral filter of one column in registers: forward transform, coefficient k times
// lam[k * pitch], inverse transform (Prop. 1, eq. 4, with the orthonormal Q).
template <int L>
__device__ __forceinline__ void filter1d(float (&v)[L], const gfloat* lam, int pitch, twptr tw)
{
    dct2_ortho<L>(v, tw);
#pragma unroll
    for (int k = 0; k < L; ++k) v[k] *= lam[k * pitch];
    asm volatile("" : "+s"(tw));
    dct3_ortho<L>(v, tw);
}

} // namespace
} // namespace dct
