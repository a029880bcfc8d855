// Internal (non-exported) declarations shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/dct2d.h"

namespace dct {

// Lengths with FFT twiddle sets: 8 .. 1024 (index = log2 L - 3).
constexpr int kMinLog = 3, kMaxLog = 10, kNumLens = kMaxLog - kMinLog + 1;
// Sizes with dense Q tables for the matrix (MFMA) paths: 8, 16, 32, 64.
constexpr int kNumDense = 4;

// Plan-owned device tables (Section 3.2: tables built once, reused by every call).
struct DeviceTables {
    int device = -1;
    int num_cu = 0;
    float2* tw = nullptr;               // twiddle bank (complex entries)
    int tw_off[kNumLens] = {};          // offset of TwLayout<L> per length
    // Dense Q_n for the matrix paths, row-major n x n, for n = 8 << i:
    float* q_f32[kNumDense] = {};       // rounded to float32
    uint16_t* q_bf16[kNumDense] = {};   // 3 planes: hi, mid, lo (bf16 bit patterns)
    uint16_t* q_f16[kNumDense] = {};    // 2 planes: hi, lo (fp16 bit patterns)
    uint8_t* q_f8[kNumDense] = {};      // 1 plane: fp8 e4m3 of Q * 2^kF8QShift
    // the same three split tables of Q^T (row-major), so that products with Q read their
    // operand columns as contiguous runs too
    uint16_t* q_bf16_t[kNumDense] = {};
    uint16_t* q_f16_t[kNumDense] = {};
    uint8_t* q_f8_t[kNumDense] = {};
    // Dense Q_n for arbitrary image axes (n <= 1024), generated on demand at plan time.
    void* pool = nullptr;               // single allocation holding everything above
    size_t pool_bytes = 0;
};

constexpr int kF8QShift = 8; // fp8 copy of Q is stored scaled by 2^8 (entries in the normal range)

// Returns the tables of the current device, initialising them on first use.
// Thread-safe.  nullptr on failure (status in *err).
const DeviceTables* tables_current(int* err);
int tables_init_device(int device);
void tables_release_all();
// The current device's tables if dct2d_init (or an earlier call) built them, else nullptr
// with DCT2D_ERR_NOINIT; never allocates.
const DeviceTables* tables_ready(int* err);

// Whole-image transforms (image.hip): per-device set-up of the no-allocation scratch
// (resolves its device address; allocates nothing) and release of the dense Q cache.
int image_scratch_init(int device);
void image_release_all();

// Generates dense float32 Q_n (eq. 1) for an arbitrary n into a device buffer.
int tables_dense_q(int n, float* dst, hipStream_t s);

inline const float2* tw_for(const DeviceTables* t, int L)
{
    int lg = 0;
    while ((1 << lg) < L) ++lg;
    return t->tw + t->tw_off[lg - kMinLog];
}

inline bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// Global-address-space views of float data: kernels access arrays through these so
// the loads and stores compile to global (not flat) memory instructions.
#if defined(__HIP_DEVICE_COMPILE__)
#define DCT_GLOBAL __attribute__((address_space(1)))
#else
#define DCT_GLOBAL
#endif
typedef DCT_GLOBAL float gfloat;
typedef DCT_GLOBAL float4 gfloat4;

// Marks a pointer that is the same in every lane of a wavefront as uniform, so its
// arithmetic stays in scalar registers and memory instructions use a scalar base with
// a 32-bit per-lane offset.  Only for values that really are wave-uniform.
template <typename T>
__device__ __forceinline__ T* uniform_ptr(T* p)
{
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (T*)(((uint64_t)hi << 32) | lo);
}

// ---- array addressing ---------------------------------------------------------------
// Array b of a batch starts at in + in_idx[b] (indexed: ragged batches) or at
// in + b * in_stride (strided batches); likewise for the output.  When a slot is
// given, the base pointer is read from device memory at run time instead (ragged
// plans recorded once as a graph and replayed on any base).
struct Addr {
    const float* in;
    float* out;
    int64_t in_stride, out_stride;
    const int64_t* in_idx;  // nullptr: strided
    const int64_t* out_idx; // nullptr: strided
    float* const* in_slot;  // nullptr: base = in
    float* const* out_slot; // nullptr: base = out
    // spectral filter only: multipliers of array b at lam + b * lam_stride (0: shared)
    const float* lam = nullptr;
    int64_t lam_stride = 0;
    __device__ __forceinline__ const gfloat* lam_for(int64_t b) const { return (const gfloat*)lam + b * lam_stride; }
    __device__ __forceinline__ const gfloat* src(int64_t b) const
    {
        const float* base = in_slot ? *(const gfloat* const DCT_GLOBAL*)in_slot : in;
        return (const gfloat*)base + (in_idx ? ((const DCT_GLOBAL int64_t*)in_idx)[b] : b * in_stride);
    }
    __device__ __forceinline__ gfloat* dst(int64_t b) const
    {
        float* base = out_slot ? *(gfloat* const DCT_GLOBAL*)out_slot : out;
        return (gfloat*)base + (out_idx ? ((const DCT_GLOBAL int64_t*)out_idx)[b] : b * out_stride);
    }
    // the two parts of src / dst, for callers that resolve several arrays at once
    __device__ __forceinline__ const gfloat* src_base() const
    {
        return (const gfloat*)(in_slot ? *(const gfloat* const DCT_GLOBAL*)in_slot : in);
    }
    __device__ __forceinline__ int64_t src_off(int64_t b) const
    {
        return in_idx ? ((const DCT_GLOBAL int64_t*)in_idx)[b] : b * in_stride;
    }
    __device__ __forceinline__ gfloat* dst_base() const
    {
        return (gfloat*)(out_slot ? *(gfloat* const DCT_GLOBAL*)out_slot : out);
    }
    __device__ __forceinline__ int64_t dst_off(int64_t b) const
    {
        return out_idx ? ((const DCT_GLOBAL int64_t*)out_idx)[b] : b * out_stride;
    }
};

// Internal direction of the fused spectral filter (Prop. 1, eq. 4): the round trip
// with the coefficients multiplied by Addr::lam between the forward and inverse
// column transforms.  Float32 path only.
constexpr int DIR_FILTER = DCT2D_FILTER;

// ---- kernel launchers (each returns a DCT2D_* status) ------------------------------
struct Job {
    int dir;           // DCT2D_FORWARD / INVERSE / ROUNDTRIP, or DIR_FILTER
    const float* in;
    float* out;
    int64_t batch;
    int32_t rows, cols;
    int64_t in_stride, out_stride;
    hipStream_t stream;
    int variant;
    const int64_t* in_idx = nullptr;  // optional offset lists (ragged batches)
    const int64_t* out_idx = nullptr;
    float* const* in_slot = nullptr;  // optional device-resident base pointers
    float* const* out_slot = nullptr;
    bool shared = false;              // launched beside other kernels (a ragged plan's branch)
    const float* lam = nullptr;       // DIR_FILTER: multipliers (device), per-array stride
    int64_t lam_stride = 0;
    Addr addr() const { return Addr{in, out, in_stride, out_stride, in_idx, out_idx, in_slot, out_slot, lam, lam_stride}; }
};

// Resolves the precision (DCT2D_AUTO -> the frozen per-size choice) and the frozen
// kernel variant, then launches.  Shared by the basic calls and ragged plans.
int dispatch(const DeviceTables* t, Job j, int precision);

// Dense axis pass (kern_dense.hip): one length-L transform along the columns
// (column_pass) or rows of `count` row-major images, through a dense float32 Q_L.
int launch_dense_axis(const Addr& a, int64_t count, int rows, int cols, bool column_pass, bool inverse,
                      const float* q, hipStream_t s);

int launch_fp32(const DeviceTables* t, const Job& j);
// One pass of direction `dir` along the rows (or, column_pass, the columns) of length
// len <= 256 of `batch` arrays with lines_per_array lines each, one thread per line.
int launch_short_line_pass(const DeviceTables* t, const Addr& a, int64_t batch, int len, int lines_per_array,
                           bool column_pass, int dir, hipStream_t s);
// Power-of-two shapes with an axis of 512 or 1024, the other 8 .. 1024 (kern_long.hip): a row
// pass and a column pass, the second in place on the output.
int launch_long(const DeviceTables* t, const Job& j);
// Rectangles with one axis of 256 and the other at most 128, fused (kern_rect256.hip).
int launch_rect256(const DeviceTables* t, const Job& j);
int fp32_variant_count(int rows, int cols, int dir);
int fp32_default_variant(int rows, int cols, int dir);
int fp32_unshared_variant(int rows, int cols, int variant);

int launch_mfma(const DeviceTables* t, const Job& j, int precision);
int mfma_supported(int rows, int cols, int precision);
int mfma_variant_count(int rows, int cols, int dir, int precision);

} // namespace dct
