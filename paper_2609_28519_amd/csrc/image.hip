// Batched transforms of whole images of any shape with both axes in [8, 1024] (columns a
// multiple of 4): the strided-batch counterpart of the ragged planner's image classes.
//
// Shapes whose axes are both powers of two go to the kernels of the basic calls: up to 256
// the frozen float32-accurate path, with an axis of 512 or 1024 the two-pass long-axis
// kernels (kern_long.hip, no workspace).  Every other shape (axes that are not powers of
// two, such as 384 or 600) is computed exactly from the dense Q_n of eq. 1 (FP64-generated,
// rounded to float32; no zero-padding), one dense product per axis (kern_dense.hip).  A dense pass writes its output tile from whole input rows or
// columns, so the two (round trip: four) passes ping-pong through a workspace of one
// float32 image per image of the batch:
//   forward / inverse   in -> ws (row pass, Q_cols)       ws -> out (column pass, Q_rows)
//   round trip          in -> ws -> out (forward)          out -> ws -> out (inverse)
//
// dct2d_image_transform takes its workspace from the stream-ordered allocator
// (hipMallocAsync / hipFreeAsync on the caller's stream, so concurrent calls on different
// streams never share it) and keeps one dense Q_n per device and length, built on first
// use.  dct2d_image_transform_noalloc is the same computation for callers that cannot
// allocate: its Q tables and workspace live in `scratch`, a fixed device array of this
// file, and the batch is processed in chunks that fit.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <utility>

#include "internal.hpp"

using namespace dct;

namespace {

// ---- the no-allocation scratch ---------------------------------------------------------
// 64 MiB per device, held from the library's load until the process ends.  Layout per
// call: dense Q_rows, then Q_cols (when cols != rows), then the workspace, each region
// 256-byte aligned.  The largest dense shape (1024 x 1020) needs 2 x 4 MiB of tables and
// 4 MiB per image of workspace, so every accepted shape fits at least one image per chunk
// (power-of-two shapes, 1024 x 1024 included, do not use the scratch).
constexpr size_t kScratchBytes = size_t(64) << 20;
__device__ __align__(256) float scratch[kScratchBytes / sizeof(float)];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
// device address of `scratch` per device (the host-side name is only a stand-in)
float* g_scratch[kMaxDevices] = {};
// dense Q_n cache of the allocating entry point: (device, n) -> device table
std::map<std::pair<int, int>, float*> g_q;

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

bool fast_shape(int r, int c) { return is_pow2(r) && is_pow2(c) && r >= 8 && r <= 256 && c >= 8 && c <= 256; }
// power-of-two shapes with an axis of 512 or 1024: the two-pass long-axis kernels (no workspace)
bool long_shape(int r, int c) { return is_pow2(r) && is_pow2(c) && r >= 8 && c >= 8 && r <= 1024 && c <= 1024 && (r > 256 || c > 256); }

int validate(int dir, const float* in, const float* out, int64_t batch, int rows, int cols, int64_t in_stride,
             int64_t out_stride)
{
    if (dir < DCT2D_FORWARD || dir > DCT2D_ROUNDTRIP || batch < 0) return DCT2D_ERR_ARG;
    if (rows < 8 || cols < 8 || rows > 1024 || cols > 1024 || (cols & 3)) return DCT2D_ERR_SIZE;
    const int64_t n = (int64_t)rows * cols;
    if (in_stride < n || out_stride < n) return DCT2D_ERR_STRIDE;
    if (batch == 0) return DCT2D_OK;
    if (!in || !out) return DCT2D_ERR_ARG;
    if ((reinterpret_cast<uintptr_t>(in) & 15u) || (reinterpret_cast<uintptr_t>(out) & 15u) || (in_stride & 3) ||
        (out_stride & 3))
        return DCT2D_ERR_ALIGN;
    if (in == out) {
        if (batch > 1 && in_stride != out_stride) return DCT2D_ERR_ARG;
    } else {
        const char* a0 = reinterpret_cast<const char*>(in);
        const char* a1 = a0 + ((batch - 1) * in_stride + n) * 4;
        const char* b0 = reinterpret_cast<const char*>(out);
        const char* b1 = b0 + ((batch - 1) * out_stride + n) * 4;
        if (a0 < b1 && b0 < a1) return DCT2D_ERR_ARG;
    }
    return DCT2D_OK;
}

// The dense passes of `count` images (count <= 65535, the grid's z extent): in and out
// strided, the workspace packed (rows * cols floats per image).
int dense_passes(int dir, const float* in, float* out, int64_t count, int rows, int cols, int64_t in_stride,
                 int64_t out_stride, const float* q_rows, const float* q_cols, float* ws, hipStream_t s)
{
    const int64_t n = (int64_t)rows * cols;
    const Addr in_ws{in, ws, in_stride, n, nullptr, nullptr, nullptr, nullptr};
    const Addr ws_out{ws, out, n, out_stride, nullptr, nullptr, nullptr, nullptr};
    const Addr out_ws{out, ws, out_stride, n, nullptr, nullptr, nullptr, nullptr};
    const bool inv = dir == DCT2D_INVERSE;
    int rc = launch_dense_axis(in_ws, count, rows, cols, false, inv, q_cols, s);
    if (rc == DCT2D_OK) rc = launch_dense_axis(ws_out, count, rows, cols, true, inv, q_rows, s);
    if (dir == DCT2D_ROUNDTRIP) {
        if (rc == DCT2D_OK) rc = launch_dense_axis(out_ws, count, rows, cols, true, true, q_rows, s);
        if (rc == DCT2D_OK) rc = launch_dense_axis(ws_out, count, rows, cols, false, true, q_cols, s);
    }
    return rc;
}

// Cached dense Q_n of the current device (allocating entry point only).
const float* cached_q(int device, int n, int* err)
{
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_q.find({device, n});
    if (it != g_q.end()) return it->second;
    float* q = nullptr;
    if (hipMalloc(&q, (size_t)n * n * sizeof(float)) != hipSuccess) {
        *err = DCT2D_ERR_NOMEM;
        return nullptr;
    }
    // built on the null stream and completed before first use on any stream
    if (tables_dense_q(n, q, nullptr) != DCT2D_OK || hipDeviceSynchronize() != hipSuccess) {
        hipFree(q);
        *err = DCT2D_ERR_HIP;
        return nullptr;
    }
    g_q[{device, n}] = q;
    return q;
}

// Device address of `scratch` on the current device, resolved once per device.
float* scratch_ptr(int* err)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        *err = DCT2D_ERR_NOINIT;
        return nullptr;
    }
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (g_scratch[dev]) return g_scratch[dev];
    }
    const int rc = image_scratch_init(dev);
    if (rc != DCT2D_OK) {
        *err = rc;
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    return g_scratch[dev];
}

} // namespace

int dct::image_scratch_init(int device)
{
    if (device < 0 || device >= kMaxDevices) return DCT2D_ERR_NOINIT;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_scratch[device]) return DCT2D_OK;
    int prev = 0;
    if (hipGetDevice(&prev) != hipSuccess) return DCT2D_ERR_HIP;
    if (prev != device && hipSetDevice(device) != hipSuccess) return DCT2D_ERR_HIP;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (prev != device) hipSetDevice(prev);
    if (e != hipSuccess || !p) return DCT2D_ERR_HIP;
    g_scratch[device] = static_cast<float*>(p);
    return DCT2D_OK;
}

void dct::image_release_all()
{
    std::lock_guard<std::mutex> lk(g_mu);
    int prev = 0;
    hipGetDevice(&prev);
    for (auto& kv : g_q) {
        hipSetDevice(kv.first.first);
        hipDeviceSynchronize();
        hipFree(kv.second);
    }
    g_q.clear();
    hipSetDevice(prev);
}

extern "C" {

int dct2d_image_transform(int dir, const float* in, float* out, int64_t batch, int32_t rows, int32_t cols,
                          int64_t in_stride, int64_t out_stride, void* stream)
{
    int rc = validate(dir, in, out, batch, rows, cols, in_stride, out_stride);
    if (rc != DCT2D_OK || batch == 0) return rc;
    const DeviceTables* t = tables_current(&rc);
    if (!t) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (fast_shape(rows, cols)) {
        Job j{dir, in, out, batch, rows, cols, in_stride, out_stride, s, 0};
        return dispatch(t, j, DCT2D_AUTO);
    }
    if (long_shape(rows, cols)) {
        Job j{dir, in, out, batch, rows, cols, in_stride, out_stride, s, 0};
        return launch_long(t, j);
    }
    const float* q_rows = cached_q(t->device, rows, &rc);
    const float* q_cols = q_rows ? cached_q(t->device, cols, &rc) : nullptr;
    if (!q_rows || !q_cols) return rc;
    const int64_t n = (int64_t)rows * cols;
    const int64_t per = batch < 65535 ? batch : 65535;
    float* ws = nullptr;
    if (hipMallocAsync(reinterpret_cast<void**>(&ws), (size_t)(per * n) * sizeof(float), s) != hipSuccess)
        return DCT2D_ERR_NOMEM;
    for (int64_t b0 = 0; b0 < batch && rc == DCT2D_OK; b0 += per) {
        const int64_t c = batch - b0 < per ? batch - b0 : per;
        rc = dense_passes(dir, in + b0 * in_stride, out + b0 * out_stride, c, rows, cols, in_stride, out_stride,
                          q_rows, q_cols, ws, s);
    }
    if (hipFreeAsync(ws, s) != hipSuccess && rc == DCT2D_OK) rc = DCT2D_ERR_HIP;
    return rc;
}

int dct2d_image_transform_noalloc(int dir, const float* in, float* out, int64_t batch, int32_t rows, int32_t cols,
                                  int64_t in_stride, int64_t out_stride, void* stream)
{
    int rc = validate(dir, in, out, batch, rows, cols, in_stride, out_stride);
    if (rc != DCT2D_OK || batch == 0) return rc;
    // the tables of dct2d_init; this entry point never builds them itself
    const DeviceTables* t = tables_ready(&rc);
    if (!t) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (fast_shape(rows, cols)) {
        Job j{dir, in, out, batch, rows, cols, in_stride, out_stride, s, 0};
        return dispatch(t, j, DCT2D_AUTO);
    }
    if (long_shape(rows, cols)) {
        Job j{dir, in, out, batch, rows, cols, in_stride, out_stride, s, 0};
        return launch_long(t, j);
    }
    float* base = scratch_ptr(&rc);
    if (!base) return rc;
    const size_t n = (size_t)rows * cols;
    const size_t q_rows_off = 0;
    const size_t q_cols_off = rows == cols ? 0 : align256((size_t)rows * rows * sizeof(float));
    const size_t ws_off = align256(q_cols_off + (size_t)cols * cols * sizeof(float));
    if (ws_off + n * sizeof(float) > kScratchBytes) return DCT2D_ERR_SIZE; // not reached for accepted shapes
    const int64_t fit = (int64_t)((kScratchBytes - ws_off) / (n * sizeof(float)));
    const int64_t per = fit < 65535 ? fit : 65535;
    char* b = reinterpret_cast<char*>(base);
    float* q_rows = reinterpret_cast<float*>(b + q_rows_off);
    float* q_cols = reinterpret_cast<float*>(b + q_cols_off);
    float* ws = reinterpret_cast<float*>(b + ws_off);
    // the tables are rebuilt on the caller's stream every call: the scratch keeps whatever
    // the previous call on this device left in it
    rc = tables_dense_q(rows, q_rows, s);
    if (rc == DCT2D_OK && cols != rows) rc = tables_dense_q(cols, q_cols, s);
    for (int64_t b0 = 0; b0 < batch && rc == DCT2D_OK; b0 += per) {
        const int64_t c = batch - b0 < per ? batch - b0 : per;
        rc = dense_passes(dir, in + b0 * in_stride, out + b0 * out_stride, c, rows, cols, in_stride, out_stride,
                          q_rows, q_cols, ws, s);
    }
    return rc;
}

} // extern "C"
