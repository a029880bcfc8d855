// Plan-owned device tables, generated on the GPU in FP64 (the only FP64 work on the
// device) and rounded once to the formats the kernels read.
//
//  * FFT / DCT-IV twiddles for every power-of-two length 8..1024, laid out as
//    TwLayout<L> (dct1d.hpp), with the normalisation factors a_k of eq. 1
//    (Section 2.1) folded into the DCT-IV post-twiddles and the length-2 base case
//    (Section 2.2, Prop. 1: scales folded into the stores).
//  * Dense Q_n of eq. 1 for n = 8, 16, 32, 64 (the matrix paths) in float32, split
//    into three bf16 planes (hi, mid, lo), two fp16 planes (hi, lo), and one fp8
//    e4m3 plane of Q * 2^8.  Each split plane is the round-to-nearest-even of what
//    the previous planes leave of the FP64 value, so hi + mid + lo carries 24
//    significant bits of Q.
//  * Dense float32 Q_n for any n (image axes such as 384), on request.
//
// Cosine arguments are reduced in integers, m = (2j+1)k mod 4n, and evaluated with
// cospi/sincospi so that the zeros and symmetries of eq. 1 are exact.
#include <math.h>

#include <mutex>

#include "dct1d.hpp"
#include "internal.hpp"

namespace dct {
namespace {

// cos(pi m / (2n)) with exact quadrant symmetry.
__device__ double cos_half_turn(long long m, long long n)
{
    const long long period = 4 * n;
    m %= period;
    if (m < 0) m += period;
    if (m > 2 * n) m = period - m;
    double sign = 1.0;
    if (m > n) {
        m = 2 * n - m;
        sign = -1.0;
    }
    if (m == n) return 0.0;
    return sign * cospi((double)m / (double)(2 * n));
}

// Round v to p significant bits (round-to-nearest-even), with quantum no finer than
// 2^qmin (gradual underflow of the target format).
__device__ double round_sig(double v, int p, int qmin)
{
    if (v == 0.0) return 0.0;
    int e;
    frexp(v, &e); // |v| in [2^(e-1), 2^e)
    int q = e - p;
    if (q < qmin) q = qmin;
    return ldexp(rint(ldexp(v, -q)), q);
}

__device__ uint16_t bf16_bits(double r) // r exactly representable in bf16
{
    const float f = (float)r;
    return (uint16_t)(__float_as_uint(f) >> 16);
}

__device__ uint16_t f16_bits(double r) // r exactly representable in fp16
{
    const _Float16 h = (_Float16)(float)r;
    return __builtin_bit_cast(uint16_t, h);
}

// OCP fp8 e4m3 (bias 7, 3 mantissa bits, max 448, subnormal quantum 2^-9); r exact.
__device__ uint8_t f8e4m3_bits(double r)
{
    uint8_t s = r < 0 ? 0x80 : 0;
    double a = fabs(r);
    if (a == 0.0) return s;
    int e;
    frexp(a, &e);
    const int ex = e - 1; // a in [2^ex, 2^(ex+1))
    if (ex < -6) return (uint8_t)(s | (uint8_t)rint(ldexp(a, 9)));
    const int mant = (int)rint((ldexp(a, -ex) - 1.0) * 8.0);
    return (uint8_t)(s | ((ex + 7) << 3) | mant);
}

// Twiddle table of one top length L, layout TwLayout<L> (dct1d.hpp).
__global__ void k_twiddles(float2* out, int L)
{
    const int F = L / 8 > 1 ? L / 8 : 1, TOP = L / 4, SIZE = F + L - 1;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= SIZE) return;
    double s, c;
    if (i < F) { // W_{L/4}^e
        sincospi(2.0 * i / TOP, &s, &c);
        out[i] = make_float2((float)c, (float)-s);
        return;
    }
    if (i == F + L - 2) { // base: length-2 DCT-II scales sqrt(1/L) (= sqrt(2/L) cos(pi/4))
        const double b = sqrt(1.0 / L);
        out[i] = make_float2((float)b, (float)b);
        return;
    }
    // level with DCT-IV length M: entries [F + L - 2M, F + L - M)
    int M = L / 2;
    while (i >= F + L - M) M /= 2;
    const int j = i - (F + L - 2 * M);
    if (j < M / 2) { // pre: exp(-i pi (4n+1)/(4M))
        sincospi((4.0 * j + 1.0) / (4.0 * M), &s, &c);
        out[i] = make_float2((float)c, (float)-s);
    } else { // post, stored conjugated: sqrt(2/L) exp(+i pi k/M)
        const int k = j - M / 2;
        const double a = sqrt(2.0 / L);
        sincospi((double)k / M, &s, &c);
        out[i] = make_float2((float)(a * c), (float)(a * s));
    }
}

__device__ double q_entry(int n, int k, int j)
{
    const double a = k == 0 ? sqrt(1.0 / n) : sqrt(2.0 / n);
    return a * cos_half_turn((long long)(2 * j + 1) * k, n);
}

// Entry i of Q_n (transposed: of Q_n^T) and its splits; qf may be null.
__global__ void k_dense(int n, bool transposed, float* qf, uint16_t* qb, uint16_t* qh, uint8_t* q8)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int nn = n * n;
    if (i >= nn) return;
    const double q = transposed ? q_entry(n, i % n, i / n) : q_entry(n, i / n, i % n);
    if (qf) qf[i] = (float)q;
    // bf16: 8 significant bits, min quantum 2^-133
    const double b0 = round_sig(q, 8, -133);
    const double b1 = round_sig(q - b0, 8, -133);
    const double b2 = round_sig(q - b0 - b1, 8, -133);
    qb[i] = bf16_bits(b0);
    qb[nn + i] = bf16_bits(b1);
    qb[2 * nn + i] = bf16_bits(b2);
    // fp16: 11 significant bits, min quantum 2^-24
    const double h0 = round_sig(q, 11, -24);
    const double h1 = round_sig(q - h0, 11, -24);
    qh[i] = f16_bits(h0);
    qh[nn + i] = f16_bits(h1);
    // fp8 e4m3 of Q * 2^kF8QShift: 4 significant bits, min quantum 2^-9
    q8[i] = f8e4m3_bits(round_sig(ldexp(q, kF8QShift), 4, -9));
}

__global__ void k_dense_f32(int n, float* qf)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)n * n) return;
    qf[i] = (float)q_entry(n, (int)(i / n), (int)(i % n));
}

std::mutex g_mu;
DeviceTables* g_tables[64] = {};

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

} // namespace

int tables_init_device(int device)
{
    std::lock_guard<std::mutex> lk(g_mu);
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev || device >= 64)
        return DCT2D_ERR_NOINIT;
    if (g_tables[device]) return DCT2D_OK;
    int prev = 0;
    if (hipGetDevice(&prev) != hipSuccess) return DCT2D_ERR_HIP;
    if (hipSetDevice(device) != hipSuccess) return DCT2D_ERR_HIP;
    DeviceTables* t = new DeviceTables();
    t->device = device;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
        delete t;
        hipSetDevice(prev);
        return DCT2D_ERR_HIP;
    }
    t->num_cu = prop.multiProcessorCount;
    // layout of the pool
    size_t off = 0;
    size_t tw_entries = 0;
    for (int i = 0; i < kNumLens; ++i) {
        const int L = 1 << (i + kMinLog);
        t->tw_off[i] = (int)tw_entries;
        tw_entries += (size_t)((L / 8 > 1 ? L / 8 : 1) + L - 1);
    }
    const size_t tw_bytes = align_up(tw_entries * sizeof(float2), 256);
    off += tw_bytes;
    size_t dense_off[kNumDense][7];
    for (int i = 0; i < kNumDense; ++i) {
        const size_t nn = (size_t)(8 << i) * (8 << i);
        dense_off[i][0] = off; off = align_up(off + nn * 4, 256);
        for (int tr = 0; tr < 2; ++tr) { // Q, then Q^T
            dense_off[i][1 + 3 * tr] = off; off = align_up(off + 3 * nn * 2, 256);
            dense_off[i][2 + 3 * tr] = off; off = align_up(off + 2 * nn * 2, 256);
            dense_off[i][3 + 3 * tr] = off; off = align_up(off + nn, 256);
        }
    }
    void* pool = nullptr;
    if (hipMalloc(&pool, off) != hipSuccess) {
        delete t;
        hipSetDevice(prev);
        return DCT2D_ERR_NOMEM;
    }
    t->pool = pool;
    t->pool_bytes = off;
    char* base = static_cast<char*>(pool);
    t->tw = reinterpret_cast<float2*>(base);
    for (int i = 0; i < kNumLens; ++i) {
        const int L = 1 << (i + kMinLog);
        const int size = (L / 8 > 1 ? L / 8 : 1) + L - 1;
        k_twiddles<<<(size + 255) / 256, 256>>>(t->tw + t->tw_off[i], L);
    }
    for (int i = 0; i < kNumDense; ++i) {
        const int n = 8 << i;
        t->q_f32[i] = reinterpret_cast<float*>(base + dense_off[i][0]);
        t->q_bf16[i] = reinterpret_cast<uint16_t*>(base + dense_off[i][1]);
        t->q_f16[i] = reinterpret_cast<uint16_t*>(base + dense_off[i][2]);
        t->q_f8[i] = reinterpret_cast<uint8_t*>(base + dense_off[i][3]);
        t->q_bf16_t[i] = reinterpret_cast<uint16_t*>(base + dense_off[i][4]);
        t->q_f16_t[i] = reinterpret_cast<uint16_t*>(base + dense_off[i][5]);
        t->q_f8_t[i] = reinterpret_cast<uint8_t*>(base + dense_off[i][6]);
        k_dense<<<(n * n + 255) / 256, 256>>>(n, false, t->q_f32[i], t->q_bf16[i], t->q_f16[i], t->q_f8[i]);
        k_dense<<<(n * n + 255) / 256, 256>>>(n, true, nullptr, t->q_bf16_t[i], t->q_f16_t[i], t->q_f8_t[i]);
    }
    const hipError_t e1 = hipGetLastError();
    const hipError_t e2 = hipDeviceSynchronize();
    hipSetDevice(prev);
    if (e1 != hipSuccess || e2 != hipSuccess) {
        hipFree(pool);
        delete t;
        return DCT2D_ERR_HIP;
    }
    g_tables[device] = t;
    return DCT2D_OK;
}

const DeviceTables* tables_current(int* err)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        if (err) *err = DCT2D_ERR_NOINIT;
        return nullptr;
    }
    if (dev < 0 || dev >= 64) {
        if (err) *err = DCT2D_ERR_NOINIT;
        return nullptr;
    }
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (g_tables[dev]) return g_tables[dev];
    }
    const int rc = tables_init_device(dev);
    if (rc != DCT2D_OK) {
        if (err) *err = rc;
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    return g_tables[dev];
}

const DeviceTables* tables_ready(int* err)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
        if (err) *err = DCT2D_ERR_NOINIT;
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_tables[dev] && err) *err = DCT2D_ERR_NOINIT;
    return g_tables[dev];
}

void tables_release_all()
{
    std::lock_guard<std::mutex> lk(g_mu);
    int prev = 0;
    hipGetDevice(&prev);
    for (int d = 0; d < 64; ++d) {
        if (!g_tables[d]) continue;
        hipSetDevice(d);
        hipDeviceSynchronize();
        hipFree(g_tables[d]->pool);
        delete g_tables[d];
        g_tables[d] = nullptr;
    }
    hipSetDevice(prev);
}

int tables_dense_q(int n, float* dst, hipStream_t s)
{
    const long long nn = (long long)n * n;
    k_dense_f32<<<(unsigned)((nn + 255) / 256), 256, 0, s>>>(n, dst);
    return hipGetLastError() == hipSuccess ? DCT2D_OK : DCT2D_ERR_HIP;
}

} // namespace dct
