// Reference kernels for the roofline figures (measurement helpers, not part of the
// transforms).
//
// The library's reference copy: the practical HBM ceiling of a kernel that reads each
// float32 element once and writes it once, as every transform here does.  Measured on
// MI355X over 512 MiB (sweep of tile size, workgroup size and resident workgroups per
// CU): 256-thread workgroups that each move one 4 KiB tile (one 16-byte chunk per
// lane, consecutive lanes on consecutive chunks), one tile per workgroup, reach
// 6.2 TB/s out of place; larger tiles per workgroup or fewer resident workgroups are
// slower.  The transforms are compared against this kernel timed in the same run.
#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace {

constexpr int kCopyThreads = 256;

__global__ void __launch_bounds__(kCopyThreads) k_copy(const float4* in, float4* out, int64_t n4)
{
    const int64_t k = (int64_t)blockIdx.x * kCopyThreads + threadIdx.x;
    if (k < n4) ((dct::gfloat4*)out)[k] = ((const dct::gfloat4*)in)[k];
}

__global__ void __launch_bounds__(64) k_copy_tail(const float* in, float* out, int64_t from, int64_t n)
{
    const int64_t k = from + threadIdx.x;
    if (k < n) ((dct::gfloat*)out)[k] = ((const dct::gfloat*)in)[k];
}

// The vector-ALU issue reference: each lane runs `iters` rounds of 16 independent float32
// FMAs (no dependency stalls past the first round), so the wall time of a grid with w
// wavefronts per SIMD gives the wave64 FMA instructions a SIMD issues per cycle at that
// occupancy.  The result only feeds a never-true comparison (nothing is stored).
__global__ void __launch_bounds__(256) k_fma_issue(float* sink, int iters)
{
    float a[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) a[i] = threadIdx.x * 1e-3f + i;
    const float b = 1.0000001f, c = 1e-7f;
    for (int k = 0; k < iters; ++k) {
#pragma unroll
        for (int i = 0; i < 16; ++i) a[i] = __builtin_fmaf(a[i], b, c);
    }
    float t = 0.f;
#pragma unroll
    for (int i = 0; i < 16; ++i) t += a[i];
    if (t == 1234.5f) ((dct::gfloat*)sink)[0] = t;
}

} // namespace

extern "C" int dct2d_fma_issue(float* sink, int32_t blocks, int32_t iters, void* stream)
{
    if (!sink || blocks < 1 || iters < 1) return DCT2D_ERR_ARG;
    if (reinterpret_cast<uintptr_t>(sink) & 3u) return DCT2D_ERR_ALIGN;
    k_fma_issue<<<(unsigned)blocks, 256, 0, static_cast<hipStream_t>(stream)>>>(sink, iters);
    return hipGetLastError() == hipSuccess ? DCT2D_OK : DCT2D_ERR_HIP;
}

extern "C" int dct2d_copy(const float* in, float* out, int64_t n, void* stream)
{
    if (n < 0) return DCT2D_ERR_ARG;
    if (n == 0) return DCT2D_OK;
    if (!in || !out) return DCT2D_ERR_ARG;
    if ((reinterpret_cast<uintptr_t>(in) & 15u) || (reinterpret_cast<uintptr_t>(out) & 15u)) return DCT2D_ERR_ALIGN;
    if (in != out) {
        const char* a0 = reinterpret_cast<const char*>(in);
        const char* b0 = reinterpret_cast<const char*>(out);
        if (a0 < b0 + n * 4 && b0 < a0 + n * 4) return DCT2D_ERR_ARG;
    }
    int rc = DCT2D_OK;
    if (!dct::tables_current(&rc)) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t n4 = n / 4;
    if (n4 > 0) {
        const int64_t grid = (n4 + kCopyThreads - 1) / kCopyThreads;
        if (grid > 0x7fffffff) return DCT2D_ERR_ARG;
        k_copy<<<(unsigned)grid, kCopyThreads, 0, s>>>(reinterpret_cast<const float4*>(in),
                                                       reinterpret_cast<float4*>(out), n4);
    }
    if (n4 * 4 < n)
        k_copy_tail<<<1, 64, 0, s>>>(in, out, n4 * 4, n);
    return hipGetLastError() == hipSuccess ? DCT2D_OK : DCT2D_ERR_HIP;
}
