// C ABI of the library (include/dct2d.h): argument validation, the frozen per-size
// policy, dispatch to the kernel families, and the autotuner.
//
// Validation happens once per call on the host, never per block (the paper's
// argument-check-free control, Section 5.1, shows checks must stay off the hot path).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <vector>

#include "internal.hpp"

using namespace dct;

namespace {

constexpr int kNumPrec = 8;

// Frozen variant table: index [log2 rows - 3][log2 cols - 3][dir][precision] (dir 3: the
// spectral filter, float32 only); starts from the per-size defaults (the variants measured
// fastest on MI355X; the filter starts from the round trip's), overridable by the tuner.
constexpr int kNumDir = 4;
std::mutex g_policy_mu;
int g_variant[6][6][kNumDir][kNumPrec];
bool g_policy_ready = false;

void policy_init_locked()
{
    if (g_policy_ready) return;
    for (int r = 0; r < 6; ++r)
        for (int c = 0; c < 6; ++c)
            for (int d = 0; d < kNumDir; ++d)
                for (int p = 0; p < kNumPrec; ++p)
                    g_variant[r][c][d][p] =
                        p == DCT2D_FP32 ? fp32_default_variant(8 << r, 8 << c, d == DIR_FILTER ? DCT2D_ROUNDTRIP : d) : 0;
    g_policy_ready = true;
}

int lg2(int v)
{
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

bool basic_size_ok(int rows, int cols)
{
    return is_pow2(rows) && is_pow2(cols) && rows >= 8 && rows <= 256 && cols >= 8 && cols <= 256;
}

// Power-of-two shapes with an axis of 512 or 1024 (the other 8 .. 1024): accepted by the
// transform calls and computed by two passes over HBM whose long-axis lines are shared by two
// or four wavefronts (kern_long.hip); no kernel variants, float32 path only.
bool long_axis_size_ok(int rows, int cols)
{
    return is_pow2(rows) && is_pow2(cols) && rows >= 8 && rows <= 1024 && cols >= 8 && cols <= 1024 &&
           (rows > 256 || cols > 256);
}

int variant_for(int rows, int cols, int dir, int prec)
{
    std::lock_guard<std::mutex> lk(g_policy_mu);
    policy_init_locked();
    return g_variant[lg2(rows) - 3][lg2(cols) - 3][dir][prec];
}

// DCT2D_AUTO: the float32-accurate path chosen per size.  Frozen before measurement
// (Section 3.2); the plain float32 path unless a split matrix path is registered faster.
std::atomic<int> g_auto_path[6][6][3];
std::once_flag g_auto_once;

void auto_init()
{
    for (auto& a : g_auto_path)
        for (auto& b : a)
            for (auto& c : b) c.store(DCT2D_FP32);
}

int resolve_precision(int rows, int cols, int dir, int prec)
{
    if (prec != DCT2D_AUTO) return prec;
    std::call_once(g_auto_once, auto_init);
    return g_auto_path[lg2(rows) - 3][lg2(cols) - 3][dir].load();
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

int validate(int dir, const float* in, const float* out, int64_t batch, int32_t rows, int32_t cols,
             int64_t in_stride, int64_t out_stride, int prec)
{
    if (dir < DCT2D_FORWARD || dir > DCT2D_ROUNDTRIP) return DCT2D_ERR_ARG;
    if (prec < 0 || prec >= kNumPrec) return DCT2D_ERR_ARG;
    if (batch < 0) return DCT2D_ERR_ARG;
    if (!basic_size_ok(rows, cols) && !long_axis_size_ok(rows, cols)) return DCT2D_ERR_SIZE;
    const int64_t n = (int64_t)rows * cols;
    if (in_stride < n || out_stride < n) return DCT2D_ERR_STRIDE;
    if (batch == 0) return DCT2D_OK;
    if (!in || !out) return DCT2D_ERR_ARG;
    if (!aligned16(in) || !aligned16(out) || (in_stride & 3) || (out_stride & 3)) return DCT2D_ERR_ALIGN;
    if (in == out) {
        // in place means array b is read and written at the same place; with different
        // strides array b's output would land on another array's input
        if (batch > 1 && in_stride != out_stride) return DCT2D_ERR_ARG;
    } else {
        // partially overlapping buffers are not supported
        const char* a0 = reinterpret_cast<const char*>(in);
        const char* a1 = a0 + ((batch - 1) * in_stride + n) * 4;
        const char* b0 = reinterpret_cast<const char*>(out);
        const char* b1 = b0 + ((batch - 1) * out_stride + n) * 4;
        if (a0 < b1 && b0 < a1) return DCT2D_ERR_ARG;
    }
    return DCT2D_OK;
}

int run(int dir, const float* in, float* out, int64_t batch, int32_t rows, int32_t cols, int64_t in_stride,
        int64_t out_stride, int prec, void* stream)
{
    int rc = validate(dir, in, out, batch, rows, cols, in_stride, out_stride, prec);
    if (rc != DCT2D_OK) return rc;
    if (long_axis_size_ok(rows, cols) && prec != DCT2D_FP32 && prec != DCT2D_AUTO) return DCT2D_ERR_PRECISION;
    if (batch == 0) return rc;
    const DeviceTables* t = tables_current(&rc);
    if (!t) return rc;
    Job j{dir, in, out, batch, rows, cols, in_stride, out_stride, static_cast<hipStream_t>(stream), 0};
    if (long_axis_size_ok(rows, cols)) return launch_long(t, j);
    return dispatch(t, j, prec);
}

int variant_count(int rows, int cols, int dir, int prec)
{
    if (prec == DCT2D_FP32) return fp32_variant_count(rows, cols, dir);
    if (dir == DIR_FILTER) return 0; // the filter exists on the float32 path only
    if (!mfma_supported(rows, cols, prec)) return 0;
    return mfma_variant_count(rows, cols, dir, prec);
}

// Arrays per candidate that the tuner's correctness guard reads back.
constexpr int64_t kTuneSamples = 48;

// Largest sampled relative error the guard accepts per path: the round-trip gate for the
// float32-accurate paths, a bound well above the measured error band for the others.
double tune_tolerance(int prec)
{
    switch (prec) {
    case DCT2D_SPLIT_BF16X3: return 1e-4;
    case DCT2D_BF16: return 5e-2;
    case DCT2D_FP16: return 1e-2;
    case DCT2D_FP8_E4M3: return 0.5;
    default: return 4e-6;
    }
}

__global__ void k_const(float* p, int64_t n, float v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Deterministic scratch fill for tuning: a counter hash mapped to [-1, 1).
__global__ void k_fill(float* p, int64_t n, uint32_t seed)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t x = (uint32_t)i * 2654435761u ^ seed;
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    p[i] = (float)(x >> 8) * (2.0f / 16777216.0f) - 1.0f;
}

} // namespace

int dct::dispatch(const DeviceTables* t, Job j, int prec)
{
    const int p = resolve_precision(j.rows, j.cols, j.dir, prec);
    j.variant = variant_for(j.rows, j.cols, j.dir, p);
    if (p == DCT2D_FP32) {
        if (j.shared) j.variant = fp32_unshared_variant(j.rows, j.cols, j.variant);
        return launch_fp32(t, j);
    }
    if (!mfma_supported(j.rows, j.cols, p)) return DCT2D_ERR_PRECISION;
    return launch_mfma(t, j, p);
}

extern "C" {

int dct2d_init(int device)
{
    int rc = tables_init_device(device);
    if (rc != DCT2D_OK) return rc;
    // resolves the device address of the no-allocation entry point's scratch (no allocation)
    rc = image_scratch_init(device);
    if (rc != DCT2D_OK) return rc;
    std::lock_guard<std::mutex> lk(g_policy_mu);
    policy_init_locked();
    return DCT2D_OK;
}

void dct2d_finalize(void)
{
    image_release_all();
    tables_release_all();
}

int dct2d_forward(float* data, int64_t batch, int32_t rows, int32_t cols, int64_t stride, void* stream)
{
    return run(DCT2D_FORWARD, data, data, batch, rows, cols, stride, stride, DCT2D_AUTO, stream);
}

int dct2d_inverse(float* data, int64_t batch, int32_t rows, int32_t cols, int64_t stride, void* stream)
{
    return run(DCT2D_INVERSE, data, data, batch, rows, cols, stride, stride, DCT2D_AUTO, stream);
}

int dct2d_roundtrip(float* data, int64_t batch, int32_t rows, int32_t cols, int64_t stride, void* stream)
{
    return run(DCT2D_ROUNDTRIP, data, data, batch, rows, cols, stride, stride, DCT2D_AUTO, stream);
}

int dct2d_transform_ex(int dir, const float* in, float* out, int64_t batch, int32_t rows, int32_t cols,
                       int64_t in_stride, int64_t out_stride, int precision, void* stream)
{
    return run(dir, in, out, batch, rows, cols, in_stride, out_stride, precision, stream);
}

int dct2d_filter(const float* in, float* out, int64_t batch, int32_t rows, int32_t cols, int64_t in_stride,
                 int64_t out_stride, const float* lambda, int64_t lambda_stride, void* stream)
{
    if (!basic_size_ok(rows, cols)) return DCT2D_ERR_SIZE; // the fused kernels cover axes <= 256
    int rc = validate(DCT2D_ROUNDTRIP, in, out, batch, rows, cols, in_stride, out_stride, DCT2D_FP32);
    if (rc != DCT2D_OK) return rc;
    const int64_t n = (int64_t)rows * cols;
    if (lambda_stride < 0 || (lambda_stride > 0 && lambda_stride < n)) return DCT2D_ERR_STRIDE;
    if (batch == 0) return DCT2D_OK;
    if (!lambda) return DCT2D_ERR_ARG;
    if (reinterpret_cast<uintptr_t>(lambda) & 3u) return DCT2D_ERR_ALIGN;
    {
        // the multipliers are read while the outputs are written: no overlap
        const char* l0 = reinterpret_cast<const char*>(lambda);
        const char* l1 = l0 + ((batch - 1) * lambda_stride + n) * 4;
        const char* o0 = reinterpret_cast<const char*>(out);
        const char* o1 = o0 + ((batch - 1) * out_stride + n) * 4;
        if (l0 < o1 && o0 < l1) return DCT2D_ERR_ARG;
    }
    const DeviceTables* t = tables_current(&rc);
    if (!t) return rc;
    // a fused round-trip kernel with the multiply between the passes, in the filter's own
    // frozen variant
    Job j{DIR_FILTER, in, out, batch, rows, cols, in_stride, out_stride, static_cast<hipStream_t>(stream),
          variant_for(rows, cols, DIR_FILTER, DCT2D_FP32)};
    j.lam = lambda;
    j.lam_stride = lambda_stride;
    return launch_fp32(t, j);
}

int dct2d_variant_count(int32_t rows, int32_t cols, int dir, int precision)
{
    if (!basic_size_ok(rows, cols) || dir < 0 || dir > DCT2D_FILTER || precision < 0 || precision >= DCT2D_AUTO)
        return 0;
    return variant_count(rows, cols, dir, precision);
}

int dct2d_get_variant(int32_t rows, int32_t cols, int dir, int precision)
{
    if (!basic_size_ok(rows, cols)) return DCT2D_ERR_SIZE;
    if (dir < 0 || dir > DCT2D_FILTER || precision < 0 || precision > DCT2D_AUTO) return DCT2D_ERR_ARG;
    if (dir == DCT2D_FILTER && precision != DCT2D_FP32 && precision != DCT2D_AUTO) return DCT2D_ERR_PRECISION;
    // for DCT2D_AUTO the "variant" is the frozen path (a dct2d_precision value)
    if (precision == DCT2D_AUTO) return dir == DCT2D_FILTER ? DCT2D_FP32 : resolve_precision(rows, cols, dir, DCT2D_AUTO);
    return variant_for(rows, cols, dir, precision);
}

int dct2d_set_variant(int32_t rows, int32_t cols, int dir, int precision, int variant)
{
    if (!basic_size_ok(rows, cols)) return DCT2D_ERR_SIZE;
    if (dir < 0 || dir > DCT2D_FILTER || precision < 0 || precision > DCT2D_AUTO) return DCT2D_ERR_ARG;
    if (dir == DCT2D_FILTER && precision != DCT2D_FP32) {
        if (precision != DCT2D_AUTO) return DCT2D_ERR_PRECISION;
        return variant == DCT2D_FP32 ? DCT2D_OK : DCT2D_ERR_PRECISION; // the filter's only path
    }
    if (precision == DCT2D_AUTO) {
        // freeze the float32-accurate path used by DCT2D_AUTO
        if (variant != DCT2D_FP32 && variant != DCT2D_SPLIT_BF16X6 && variant != DCT2D_SPLIT_FP16X3)
            return DCT2D_ERR_ARG;
        if (variant != DCT2D_FP32 && !mfma_supported(rows, cols, variant)) return DCT2D_ERR_PRECISION;
        std::call_once(g_auto_once, auto_init);
        g_auto_path[lg2(rows) - 3][lg2(cols) - 3][dir].store(variant);
        return DCT2D_OK;
    }
    if (variant < 0 || variant >= variant_count(rows, cols, dir, precision)) return DCT2D_ERR_ARG;
    std::lock_guard<std::mutex> lk(g_policy_mu);
    policy_init_locked();
    g_variant[lg2(rows) - 3][lg2(cols) - 3][dir][precision] = variant;
    return DCT2D_OK;
}

int dct2d_tune(int32_t rows, int32_t cols, int dir, int precision, int64_t batch, void* stream, float* best_ms)
{
    if (!basic_size_ok(rows, cols)) return DCT2D_ERR_SIZE;
    if (dir < 0 || dir > DCT2D_FILTER || precision < 0 || precision > DCT2D_AUTO || batch <= 0) return DCT2D_ERR_ARG;
    if (dir == DCT2D_FILTER) {
        if (precision != DCT2D_FP32 && precision != DCT2D_AUTO) return DCT2D_ERR_PRECISION;
        precision = DCT2D_FP32; // the filter's only path
    }
    if (precision == DCT2D_AUTO) {
        // tune every float32-accurate path, then freeze the fastest one for DCT2D_AUTO
        int best_p = -1;
        float best = 0.f;
        for (int p : {DCT2D_FP32, DCT2D_SPLIT_BF16X6, DCT2D_SPLIT_FP16X3}) {
            if (variant_count(rows, cols, dir, p) <= 0) continue;
            float ms = 0.f;
            const int rc = dct2d_tune(rows, cols, dir, p, batch, stream, &ms);
            if (rc != DCT2D_OK) return rc;
            if (best_p < 0 || ms < best) {
                best_p = p;
                best = ms;
            }
        }
        if (best_p < 0) return DCT2D_ERR_PRECISION;
        std::call_once(g_auto_once, auto_init);
        g_auto_path[lg2(rows) - 3][lg2(cols) - 3][dir].store(best_p);
        if (best_ms) *best_ms = best;
        return DCT2D_OK;
    }
    const int nv = variant_count(rows, cols, dir, precision);
    if (nv <= 0) return DCT2D_ERR_PRECISION;
    int rc = DCT2D_OK;
    const DeviceTables* t = tables_current(&rc);
    if (!t) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t per = (int64_t)rows * cols;
    const int64_t n = batch * per;
    // scratch: input, candidate output, and the back-transform that checks it; for the
    // filter the last rows*cols floats of `chk` hold a constant multiplier array
    float *src = nullptr, *dst = nullptr, *chk = nullptr;
    if (hipMalloc(&src, n * 4) != hipSuccess) return DCT2D_ERR_NOMEM;
    if (hipMalloc(&dst, n * 4) != hipSuccess) { hipFree(src); return DCT2D_ERR_NOMEM; }
    if (hipMalloc(&chk, (n + per) * 4) != hipSuccess) { hipFree(src); hipFree(dst); return DCT2D_ERR_NOMEM; }
    float* lam = chk + n;
    k_fill<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(src, n, 0x5eedu);
    hipEvent_t e0, e1;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    // arrays checked per candidate: spread evenly over the whole batch, first and last
    // included, so every pass of a grid-stride or persistent schedule is seen
    const int64_t ns = batch < kTuneSamples ? batch : kTuneSamples;
    std::vector<int64_t> sample((size_t)ns);
    for (int64_t i = 0; i < ns; ++i) sample[(size_t)i] = ns == 1 ? 0 : i * (batch - 1) / (ns - 1);
    std::vector<float> h_in((size_t)(ns * per)), h_out((size_t)(ns * per));
    auto fetch = [&](const float* dev, std::vector<float>& host) {
        for (int64_t i = 0; i < ns; ++i)
            if (hipMemcpy(host.data() + i * per, dev + sample[(size_t)i] * per, per * 4, hipMemcpyDeviceToHost) !=
                hipSuccess)
                return false;
        return true;
    };
    // max over the sampled arrays of ||out_b - c in_b|| / ||in_b||
    auto worst = [&](float c) {
        double w = 0.0;
        for (int64_t i = 0; i < ns; ++i) {
            double num = 0, den = 0;
            for (int64_t k = 0; k < per; ++k) {
                const double a = h_in[(size_t)(i * per + k)], b = h_out[(size_t)(i * per + k)];
                num += (b - c * a) * (b - c * a);
                den += a * a;
            }
            const double e = den > 0 ? std::sqrt(num / den) : std::sqrt(num);
            if (!(e <= w)) w = e; // NaN propagates as a failure
        }
        return w;
    };
    const double tol = tune_tolerance(precision);
    if (!fetch(src, h_in)) rc = DCT2D_ERR_HIP;
    // 1. correctness guard for every candidate; 2. the candidates that pass are timed in four
    // interleaved rounds (the order rotated each round) and scored by the median of their rounds,
    // so that neither drift over the sweep (clocks, memory state) nor one lucky round decides
    // between close variants
    std::vector<int> passed;
    for (int v = 0; v < nv && rc == DCT2D_OK; ++v) {
        Job j{dir, src, dst, batch, rows, cols, per, per, s, v};
        j.lam = dir == DCT2D_FILTER ? lam : nullptr;
        auto launch = [&]() { return precision == DCT2D_FP32 ? launch_fp32(t, j) : launch_mfma(t, j, precision); };
        // Correctness guard, independent of every other candidate: the candidate's
        // composition with the opposite transform must return the input.  Round trip:
        // its own output.  Filter: multipliers 1 (identity) and -1/2 (-X/2).  Forward and
        // inverse: followed by the frozen float32 inverse / forward; a wrong candidate
        // cannot be cancelled by a correct partner.
        bool ok = true;
        const int checks = dir == DCT2D_FILTER ? 2 : 1;
        for (int c = 0; c < checks && ok && rc == DCT2D_OK; ++c) {
            const float lam_c = c == 0 ? 1.0f : -0.5f;
            if (dir == DCT2D_FILTER) {
                k_const<<<(unsigned)((per + 255) / 256), 256, 0, s>>>(lam, per, lam_c);
                if (hipGetLastError() != hipSuccess) { rc = DCT2D_ERR_HIP; break; }
            }
            if ((rc = launch()) != DCT2D_OK) break;
            const float* res = dst;
            if (dir == DCT2D_FORWARD || dir == DCT2D_INVERSE) {
                Job back{dir == DCT2D_FORWARD ? DCT2D_INVERSE : DCT2D_FORWARD, dst, chk, batch, rows, cols, per, per,
                         s, variant_for(rows, cols, dir == DCT2D_FORWARD ? DCT2D_INVERSE : DCT2D_FORWARD,
                                        DCT2D_FP32)};
                if ((rc = launch_fp32(t, back)) != DCT2D_OK) break;
                res = chk;
            }
            if (hipStreamSynchronize(s) != hipSuccess || !fetch(res, h_out)) { rc = DCT2D_ERR_HIP; break; }
            ok = worst(dir == DCT2D_FILTER ? lam_c : 1.0f) <= tol;
        }
        if (rc != DCT2D_OK) break;
        if (ok) passed.push_back(v); // a candidate that fails the identity is never selected
    }
    if (rc == DCT2D_OK && dir == DCT2D_FILTER && !passed.empty()) {
        k_fill<<<(unsigned)((per + 255) / 256), 256, 0, s>>>(lam, per, 0x1a3bu); // timing multipliers
        if (hipGetLastError() != hipSuccess) rc = DCT2D_ERR_HIP;
    }
    const size_t np = passed.size();
    constexpr int kRounds = 4, kReps = 10;
    std::vector<float> rounds(np * kRounds, 0.f);
    for (int round = 0; round < kRounds && rc == DCT2D_OK; ++round) {
        for (size_t q = 0; q < np && rc == DCT2D_OK; ++q) {
            const size_t idx = (q + (size_t)round) % np;
            // timed in place, as the basic calls run (repeating an orthonormal transform keeps the
            // data bounded); the filter out of place, since repeated filtering would shrink it
            const float* tin = dir == DCT2D_FILTER ? src : dst;
            Job j{dir, tin, dst, batch, rows, cols, per, per, s, passed[idx]};
            j.lam = dir == DCT2D_FILTER ? lam : nullptr;
            auto launch = [&]() { return precision == DCT2D_FP32 ? launch_fp32(t, j) : launch_mfma(t, j, precision); };
            if ((rc = launch()) != DCT2D_OK) break; // warm
            float ms = 0.f;
            hipEventRecord(e0, s);
            for (int r = 0; r < kReps && rc == DCT2D_OK; ++r) rc = launch();
            hipEventRecord(e1, s);
            hipEventSynchronize(e1);
            hipEventElapsedTime(&ms, e0, e1);
            ms /= kReps;
            rounds[idx * kRounds + (size_t)round] = ms;
        }
    }
    std::vector<float> score(np, 0.f);
    for (size_t q = 0; q < np; ++q) {
        float* r = rounds.data() + q * kRounds;
        std::sort(r, r + kRounds);
        score[q] = 0.5f * (r[kRounds / 2 - 1] + r[kRounds / 2]);
    }
    int best = -1;
    float best_t = 0.f;
    for (size_t q = 0; q < np; ++q)
        if (best < 0 || score[q] < best_t) {
            best = passed[q];
            best_t = score[q];
        }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    hipStreamSynchronize(s);
    hipFree(src);
    hipFree(dst);
    hipFree(chk);
    if (rc != DCT2D_OK) return rc;
    if (best < 0) return DCT2D_ERR_HIP;
    if (best_ms) *best_ms = best_t;
    return dct2d_set_variant(rows, cols, dir, precision, best);
}

const char* dct2d_status_string(int status)
{
    switch (status) {
    case DCT2D_OK: return "ok";
    case DCT2D_ERR_ARG: return "invalid argument";
    case DCT2D_ERR_SIZE: return "unsupported array shape";
    case DCT2D_ERR_STRIDE: return "stride smaller than rows*cols";
    case DCT2D_ERR_ALIGN: return "pointer or stride not 16-byte aligned";
    case DCT2D_ERR_PRECISION: return "precision not available for this shape";
    case DCT2D_ERR_HIP: return "HIP runtime error";
    case DCT2D_ERR_NOINIT: return "no usable device";
    case DCT2D_ERR_NOMEM: return "out of memory";
    default: return "unknown status";
    }
}

const char* dct2d_version(void) { return "dct2d-mi355x 0.1.0 (gfx950)"; }

} // extern "C"
