// Dense matrix paths on MFMA for N = 8, 16, 32 and 64 (64 as 2 x 2 tiles of the 32 x 32 form):
// Y = Q X Q^T (eq. 2) as two small matrix products per block, with float32 accuracy
// recovered from low-precision operands by splitting (split-precision products) and
// a power-of-two scale per block.
//
// Lane layouts (v_mfma_f32_16x16x{16,32}, wave64): lane l = 16 g + c holds
//   accumulator  D[4g + i][c], i = 0..3
//   A operand    A[c][k-slots of group g]      B operand  B[k-slots of group g][c]
// A tile S is loaded so that lane (g, c) holds row c, columns 4g..4g+3 of the block
// (one contiguous 16-byte load per lane, the whole 16x16 block per instruction); in
// accumulator terms that is S = X^T.  Then, with B = Q^T:
//   pass 1:  D1 = (S^T) Q^T = X Q^T          (the lane's registers used as A = S^T)
//   pass 2:  D2 = (D1^T) Q^T = (Q X Q^T)^T   (D1's registers used directly as A)
// so lane (g, c) ends with row c, columns 4g..4g+3 of Y and stores them with one
// 16-byte store.  No data moves between the passes; the inverse uses B = Q.  The
// 32x32 instructions (v_mfma_f32_32x32x16, 16 accumulators per lane) follow the same
// scheme with K split over two instructions.  N = 8 packs four 8x8 blocks in a
// 16x16 tile with the block-diagonal diag(Q_8, Q_8).
//
// Precision modes (dct2d_precision): split products use X = X0 + X1 (+ X2) and
// Q = C0 + C1 (+ C2), rounded to nearest even part by part, and keep the products
// C_i X_j with i + j < number of parts, smallest first.  A K=32 instruction carries two
// products at once (k-slots 0-3 of a lane hold part a, slots 4-7 part b, with the
// matching C parts in B).  The per-block scale 2^-e (e from the block maximum, exact
// power of two, zero block -> scale 1) keeps fp16/fp8 parts in range; fp16 and fp8
// rescale again after pass 1.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "internal.hpp"

namespace dct {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

enum Mode { M_BF16X3 = DCT2D_SPLIT_BF16X3, M_BF16X6 = DCT2D_SPLIT_BF16X6, M_FP16X3 = DCT2D_SPLIT_FP16X3,
            M_BF16 = DCT2D_BF16, M_FP16 = DCT2D_FP16, M_FP8 = DCT2D_FP8_E4M3 };

template <int MODE>
struct ModeInfo {
    static constexpr bool f16 = MODE == M_FP16X3 || MODE == M_FP16;
    static constexpr bool f8 = MODE == M_FP8;
    static constexpr int parts = MODE == M_BF16X6 ? 3 : (MODE == M_BF16X3 || MODE == M_FP16X3) ? 2 : 1;
    // block maximum is scaled into [2^T, 2^(T+1)): bf16/fp16 [1,2), fp8 [128,256)
    static constexpr int target = f8 ? 7 : 0;
    static constexpr bool rescale = f16 || f8; // rescale after every pass
};

// ---- conversions (round to nearest even) -----------------------------------------
__device__ __forceinline__ __bf16 to_bf16(float x) { return (__bf16)x; }
__device__ __forceinline__ _Float16 to_f16(float x) { return (_Float16)x; }

// Splits x into `parts` terms of the mode's format; returns them through p[].
template <int MODE>
__device__ __forceinline__ void split(float x, float (&p)[3])
{
    if constexpr (ModeInfo<MODE>::f16) {
        const _Float16 h0 = to_f16(x);
        p[0] = (float)h0;
        if constexpr (ModeInfo<MODE>::parts > 1) p[1] = (float)to_f16(x - p[0]);
    } else {
        const __bf16 b0 = to_bf16(x);
        p[0] = (float)b0;
        if constexpr (ModeInfo<MODE>::parts > 1) {
            const float r1 = x - p[0];
            p[1] = (float)to_bf16(r1);
            if constexpr (ModeInfo<MODE>::parts > 2) p[2] = (float)to_bf16(r1 - p[1]);
        }
    }
}

// ---- per-block power-of-two scale ----------------------------------------------------
// Exponent e with max * 2^-e in [2^T, 2^(T+1)); 0 for a zero (or non-finite) maximum.
template <int T>
__device__ __forceinline__ int scale_exponent(float m)
{
    if (!(m > 0.f) || !(m < __builtin_inff())) return 0;
    int e;
    frexpf(m, &e); // m in [2^(e-1), 2^e)
    return e - 1 - T;
}

// max over the lanes of one block: xor-shuffle over the given lane masks
template <int... MASKS>
__device__ __forceinline__ float lane_max(float v)
{
    ((v = fmaxf(v, __shfl_xor(v, MASKS, 64))), ...);
    return v;
}

// ---- B operands (constant per lane) ---------------------------------------------------
// Q part p (0..parts-1) as float from the split tables.
struct QTab {
    const uint16_t* bf; // 3 planes
    const uint16_t* hf; // 2 planes
    const uint8_t* f8;  // 1 plane (Q * 2^kF8QShift)
    int n;
    const uint16_t* bft; // the same planes of Q^T
    const uint16_t* hft;
    const uint8_t* f8t;
};

__device__ __forceinline__ float bf16_bits_to_f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
__device__ __forceinline__ float f16_bits_to_f(uint16_t b) { return (float)__builtin_bit_cast(_Float16, b); }

// 16x16 tile entry of Q' (Q_16, or diag(Q_8, Q_8) for N = 8), part p, as the mode's
// float value: element [r][c] of the tile matrix.
template <int N, int MODE>
__device__ __forceinline__ float qprime(const QTab& q, int p, int r, int c)
{
    int n = N, rr = r, cc = c;
    if (N == 8) {
        if ((r >> 3) != (c >> 3)) return 0.f;
        rr = r & 7;
        cc = c & 7;
    }
    const int i = rr * n + cc;
    if constexpr (ModeInfo<MODE>::f8) return 0.f; // fp8 operands are built separately
    else if constexpr (ModeInfo<MODE>::f16) return f16_bits_to_f(q.hf[p * n * n + i]);
    else return bf16_bits_to_f(q.bf[p * n * n + i]);
}

template <class V, class E>
__device__ __forceinline__ V make8(const float (&a)[4], const float (&b)[4])
{
    V v;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        v[j] = (E)a[j];
        v[j + 4] = (E)b[j];
    }
    return v;
}

// ---- 16x16 tiles (N = 8, 16) ----------------------------------------------------------
// Lane (g, c): slot j of group g <-> k = 4g + j.  For direction INV = false the pass
// multiplies by B = Q'^T (B[k][c] = Q'[c][k]); for INV = true by B = Q' (B[k][c] = Q'[k][c]).
template <int N, int MODE>
struct B16 {
    float c[3][4]; // part p, slot j
};

template <int N, int MODE>
__device__ __forceinline__ B16<N, MODE> load_b16(const QTab& q, bool inv, int g, int c)
{
    B16<N, MODE> b;
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int k = 4 * g + j;
            b.c[p][j] = p < ModeInfo<MODE>::parts ? (inv ? qprime<N, MODE>(q, p, k, c) : qprime<N, MODE>(q, p, c, k))
                                                  : 0.f;
        }
    return b;
}

// fp8 e4m3 B operand for the K=32 fp8 instruction: slots 0-3 = Q' (scaled by 2^kF8QShift),
// slots 4-7 = 0.  Packed as 8 bytes.
template <int N>
__device__ __forceinline__ long load_b16_f8(const QTab& q, bool inv, int g, int c)
{
    uint64_t v = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int k = 4 * g + j;
        int r = inv ? k : c, cc = inv ? c : k;
        uint8_t byte = 0;
        if (N == 16 || (r >> 3) == (cc >> 3)) {
            if (N == 8) { r &= 7; cc &= 7; }
            byte = q.f8[r * N + cc];
        }
        v |= (uint64_t)byte << (8 * j);
    }
    return (long)v;
}

__device__ __forceinline__ long pack_f8x4(const float (&a)[4])
{
    // v_cvt_pk_fp8_f32: two floats -> two fp8 (e4m3) bytes, round to nearest even
    int lo = __builtin_amdgcn_cvt_pk_fp8_f32(a[0], a[1], 0, false);
    lo = __builtin_amdgcn_cvt_pk_fp8_f32(a[2], a[3], lo, true);
    return (long)(uint32_t)lo;
}

// One pass on a 16x16 tile: returns sum over kept products of A_j * B_i, A = the lane's
// four values d (as the A operand), B = bq.
template <int N, int MODE>
__device__ __forceinline__ f32x4 pass16(const float (&d)[4], const B16<N, MODE>& bq, long bq8)
{
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    if constexpr (MODE == M_FP8) {
        acc = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(pack_f8x4(d), bq8, acc, 0, 0, 0);
    } else {
        float x[3][4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            float p[3];
            split<MODE>(d[j], p);
#pragma unroll
            for (int i = 0; i < ModeInfo<MODE>::parts; ++i) x[i][j] = p[i];
        }
        // Two split products share one K=32 instruction (k slots 0-3 carry one product's
        // four k values, slots 4-7 the other's, over the same four k values of the
        // lane), so two-part modes issue (X1 C0 + X0 C1) and then (X0 C0 + 0), smallest
        // terms first.  The 16x16x16 and 16x16x32 shapes share the accumulator layout,
        // so a chain may mix them; keeping one shape only makes the issue pattern uniform.
        constexpr float z4[4] = {0.f, 0.f, 0.f, 0.f};
        if constexpr (ModeInfo<MODE>::f16 && ModeInfo<MODE>::parts == 2) {
            acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(make8<f16x8, _Float16>(x[1], x[0]),
                                                         make8<f16x8, _Float16>(bq.c[0], bq.c[1]), acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(make8<f16x8, _Float16>(x[0], z4),
                                                         make8<f16x8, _Float16>(bq.c[0], z4), acc, 0, 0, 0);
        } else if constexpr (ModeInfo<MODE>::f16) {
            f16x4 a4, b4;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                a4[j] = (_Float16)x[0][j];
                b4[j] = (_Float16)bq.c[0][j];
            }
            acc = __builtin_amdgcn_mfma_f32_16x16x16f16(a4, b4, acc, 0, 0, 0);
        } else {
            if constexpr (ModeInfo<MODE>::parts == 3) {
                // (X2 C0 + X1 C1), (X0 C2 + X1 C0), (X0 C1 + X0 C0): smallest terms first
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(make8<bf16x8, __bf16>(x[2], x[1]),
                                                              make8<bf16x8, __bf16>(bq.c[0], bq.c[1]), acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(make8<bf16x8, __bf16>(x[0], x[1]),
                                                              make8<bf16x8, __bf16>(bq.c[2], bq.c[0]), acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(make8<bf16x8, __bf16>(x[0], x[0]),
                                                              make8<bf16x8, __bf16>(bq.c[1], bq.c[0]), acc, 0, 0, 0);
            } else if constexpr (ModeInfo<MODE>::parts == 2) {
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(make8<bf16x8, __bf16>(x[1], x[0]),
                                                              make8<bf16x8, __bf16>(bq.c[0], bq.c[1]), acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(make8<bf16x8, __bf16>(x[0], z4),
                                                              make8<bf16x8, __bf16>(bq.c[0], z4), acc, 0, 0, 0);
            } else {
                s16x4 a4, b4;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    a4[j] = __builtin_bit_cast(short, (__bf16)x[0][j]);
                    b4[j] = __builtin_bit_cast(short, (__bf16)bq.c[0][j]);
                }
                acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a4, b4, acc, 0, 0, 0);
            }
        }
    }
    return acc;
}

// Kernel over 16x16 tiles (N = 16: one block per tile; N = 8: four blocks per tile).
// Each wavefront processes UNROLL tiles per iteration of its grid-stride loop.
template <int N, int MODE, int DIR, int UNROLL>
__global__ void __launch_bounds__(256)
k_mfma16(Addr a, int64_t batch, QTab q)
{
    constexpr int BPT = N == 8 ? 4 : 1; // blocks per tile
    constexpr int T0 = ModeInfo<MODE>::target;
    const int lane = threadIdx.x & 63;
    const int g = lane >> 4, c = lane & 15;
    const int64_t wave = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / 64);
    const int64_t ntiles = (batch + BPT - 1) / BPT;

    // The tile (1 KB: one 16 x 16 block, or four 8 x 8 blocks) moves between HBM and the
    // registers as 64 lane-consecutive 16-byte chunks (lane l loads and stores chunk l, so
    // every group of four lanes covers one 64-byte segment); a lane permutation
    // (ds_bpermute) maps the chunks to and from the operand layout, in which lane (g, c) holds
    // chunk `need`: block blk, 16 bytes at float offset off of the block.
    int blk, off;
    if (N == 8) {
        blk = (c >> 3) * 2 + (g >> 1);
        off = (c & 7) * 8 + 4 * (g & 1);
    } else {
        blk = 0;
        off = c * 16 + 4 * g;
    }
    const int need = (blk * N * N + off) / 4;
    // the lane whose operand-layout values form chunk `lane` (inverse of need)
    int holder;
    if (N == 8) {
        const int b8 = lane >> 4, rem = lane & 15;
        holder = 16 * ((b8 & 1) * 2 + (rem & 1)) + (b8 >> 1) * 8 + (rem >> 1);
    } else {
        holder = 16 * (lane & 3) + (lane >> 2);
    }
    const int my_blk = N == 8 ? lane >> 4 : 0; // block of the chunk this lane moves
    // the forward multiplies by Q^T, the inverse by Q; the round trip needs both
    const B16<N, MODE> bf = load_b16<N, MODE>(q, false, g, c);
    const B16<N, MODE> bi = load_b16<N, MODE>(q, true, g, c);
    long bf8 = 0, bi8 = 0;
    if constexpr (MODE == M_FP8) {
        bf8 = load_b16_f8<N>(q, false, g, c);
        bi8 = load_b16_f8<N>(q, true, g, c);
    }
    const float qscale = MODE == M_FP8 ? 1.0f / (float)(1 << kF8QShift) : 1.0f;

    for (int64_t t0 = wave * UNROLL; t0 < ntiles; t0 += nwaves * UNROLL) {
        float d[UNROLL][4];
        bool valid[UNROLL];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            const int64_t b = (t0 + u) * BPT + my_blk;
            valid[u] = (t0 + u) < ntiles && b < batch;
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (valid[u]) v = *reinterpret_cast<const gfloat4*>(a.src(b) + 4 * (lane & (N == 8 ? 15 : 63)));
            d[u][0] = __shfl(v.x, need, 64);
            d[u][1] = __shfl(v.y, need, 64);
            d[u][2] = __shfl(v.z, need, 64);
            d[u][3] = __shfl(v.w, need, 64);
        }
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            // per-block power-of-two scale
            float m = fmaxf(fmaxf(fabsf(d[u][0]), fabsf(d[u][1])), fmaxf(fabsf(d[u][2]), fabsf(d[u][3])));
            m = N == 8 ? lane_max<1, 2, 4, 16>(m) : lane_max<1, 2, 4, 8, 16, 32>(m);
            const int e0 = scale_exponent<T0>(m);
            int etot = e0;
#pragma unroll
            for (int j = 0; j < 4; ++j) d[u][j] = ldexpf(d[u][j], -e0);
            constexpr int npass = DIR == DCT2D_ROUNDTRIP ? 4 : 2;
#pragma unroll
            for (int ps = 0; ps < npass; ++ps) {
                const bool inv = DIR == DCT2D_INVERSE || (DIR == DCT2D_ROUNDTRIP && ps >= 2);
                f32x4 acc = pass16<N, MODE>(d[u], inv ? bi : bf, inv ? bi8 : bf8);
#pragma unroll
                for (int j = 0; j < 4; ++j) d[u][j] = acc[j] * qscale;
                if (ModeInfo<MODE>::rescale && ps + 1 < npass) {
                    // re-normalise the intermediate block (its lanes' grouping is the same
                    // lane set for N = 16; for N = 8 the block moved to the transposed
                    // position, handled by exchanging exponents at the end)
                    float m2 = fmaxf(fmaxf(fabsf(d[u][0]), fabsf(d[u][1])), fmaxf(fabsf(d[u][2]), fabsf(d[u][3])));
                    m2 = N == 8 ? lane_max<1, 2, 4, 16>(m2) : lane_max<1, 2, 4, 8, 16, 32>(m2);
                    int e1 = scale_exponent<T0>(m2);
                    if (N == 8 && (ps & 1) == 0) {
                        // after an odd number of passes lane (g, c) holds tile block (g/2, c/8);
                        // after an even number block (c/8, g/2).  Keep the exponent with the
                        // lanes that will hold this block at the end: they are the lanes of
                        // the transposed group.
                        const int src = ((c >> 3) * 2) * 16 + (g >> 1) * 8; // lane in group (c/8, g/2) ^T
                        const int e1t = __shfl(e1, src, 64);
                        etot += e1t;
                    } else {
                        etot += e1;
                    }
#pragma unroll
                    for (int j = 0; j < 4; ++j) d[u][j] = ldexpf(d[u][j], -e1);
                }
            }
            const float4 o = make_float4(__shfl(ldexpf(d[u][0], etot), holder, 64),
                                         __shfl(ldexpf(d[u][1], etot), holder, 64),
                                         __shfl(ldexpf(d[u][2], etot), holder, 64),
                                         __shfl(ldexpf(d[u][3], etot), holder, 64));
            if (valid[u]) {
                const int64_t b = (t0 + u) * BPT + my_blk;
                *reinterpret_cast<gfloat4*>(a.dst(b) + 4 * (lane & (N == 8 ? 15 : 63))) = o;
            }
        }
    }
}

// ---- 32x32 tiles (N = 32) -------------------------------------------------------------
// Lane l = 32 h + c holds accumulator D[8 (r/4) + 4h + r%4][c], r = 0..15.  As an A
// operand, accumulator values r = 8s .. 8s+7 form the 8 k-slots of instruction half s:
// slot j <-> k = 8 (2s + j/4) + 4h + j%4.
template <int MODE>
struct B32 {
    float c[3][2][8]; // part, instruction half, slot
};

template <int MODE>
__device__ __forceinline__ B32<MODE> load_b32(const QTab& q, bool inv, int h, int c)
{
    B32<MODE> b;
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int k = 8 * (2 * s + j / 4) + 4 * h + (j & 3);
                b.c[p][s][j] =
                    p < ModeInfo<MODE>::parts ? (inv ? qprime<32, MODE>(q, p, k, c) : qprime<32, MODE>(q, p, c, k)) : 0.f;
            }
    return b;
}

template <int MODE>
__device__ __forceinline__ long load_b32_f8(const QTab& q, bool inv, int h, int c, int s)
{
    uint64_t v = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int k = 8 * (2 * s + j / 4) + 4 * h + (j & 3);
        const uint8_t byte = inv ? q.f8[k * 32 + c] : q.f8[c * 32 + k];
        v |= (uint64_t)byte << (8 * j);
    }
    return (long)v;
}

template <class V, class E>
__device__ __forceinline__ V vec8(const float* a)
{
    V v;
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = (E)a[j];
    return v;
}

template <int MODE>
__device__ __forceinline__ f32x16 pass32(const float (&d)[16], const B32<MODE>& bq, const long (&b8)[2])
{
    f32x16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.f;
    if constexpr (MODE == M_FP8) {
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            int lo = __builtin_amdgcn_cvt_pk_fp8_f32(d[8 * s + 0], d[8 * s + 1], 0, false);
            lo = __builtin_amdgcn_cvt_pk_fp8_f32(d[8 * s + 2], d[8 * s + 3], lo, true);
            int hi = __builtin_amdgcn_cvt_pk_fp8_f32(d[8 * s + 4], d[8 * s + 5], 0, false);
            hi = __builtin_amdgcn_cvt_pk_fp8_f32(d[8 * s + 6], d[8 * s + 7], hi, true);
            const long a = (long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_fp8_fp8(a, b8[s], acc, 0, 0, 0);
        }
    } else {
        float x[3][16];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            float p[3];
            split<MODE>(d[r], p);
#pragma unroll
            for (int i = 0; i < ModeInfo<MODE>::parts; ++i) x[i][r] = p[i];
        }
        // products (i = X part, p = Q part) with i + p < parts, smallest first
        constexpr int P = ModeInfo<MODE>::parts;
#pragma unroll
        for (int sum = P - 1; sum >= 0; --sum)
#pragma unroll
            for (int i = sum; i >= 0; --i) {
                const int p = sum - i;
#pragma unroll
                for (int s = 0; s < 2; ++s) {
                    if constexpr (ModeInfo<MODE>::f16)
                        acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(vec8<f16x8, _Float16>(&x[i][8 * s]),
                                                                     vec8<f16x8, _Float16>(bq.c[p][s]), acc, 0, 0, 0);
                    else
                        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(vec8<bf16x8, __bf16>(&x[i][8 * s]),
                                                                      vec8<bf16x8, __bf16>(bq.c[p][s]), acc, 0, 0, 0);
                }
            }
    }
    return acc;
}

// B operands packed once per wavefront in the instruction's element type.
template <int MODE>
struct B32P {
    typedef typename std::conditional<ModeInfo<MODE>::f16, f16x8, bf16x8>::type V;
    V v[3][2];
};

template <int MODE>
__device__ __forceinline__ B32P<MODE> pack_b32(const B32<MODE>& b)
{
    B32P<MODE> r;
    typedef typename B32P<MODE>::V V;
    typedef typename std::conditional<ModeInfo<MODE>::f16, _Float16, __bf16>::type E;
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int s = 0; s < 2; ++s) r.v[p][s] = vec8<V, E>(b.c[p][s]);
    return r;
}

template <int MODE>
__device__ __forceinline__ f32x16 pass32p(const float (&d)[16], const B32P<MODE>& bq, const long (&b8)[2])
{
    f32x16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.f;
    if constexpr (MODE == M_FP8) {
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            int lo = __builtin_amdgcn_cvt_pk_fp8_f32(d[8 * s + 0], d[8 * s + 1], 0, false);
            lo = __builtin_amdgcn_cvt_pk_fp8_f32(d[8 * s + 2], d[8 * s + 3], lo, true);
            int hi = __builtin_amdgcn_cvt_pk_fp8_f32(d[8 * s + 4], d[8 * s + 5], 0, false);
            hi = __builtin_amdgcn_cvt_pk_fp8_f32(d[8 * s + 6], d[8 * s + 7], hi, true);
            const long a = (long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_fp8_fp8(a, b8[s], acc, 0, 0, 0);
        }
    } else {
        typedef typename B32P<MODE>::V V;
        typedef typename std::conditional<ModeInfo<MODE>::f16, _Float16, __bf16>::type E;
        float x[3][16];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            float pp[3];
            split<MODE>(d[r], pp);
#pragma unroll
            for (int i = 0; i < ModeInfo<MODE>::parts; ++i) x[i][r] = pp[i];
        }
        constexpr int P = ModeInfo<MODE>::parts;
#pragma unroll
        for (int sum = P - 1; sum >= 0; --sum)
#pragma unroll
            for (int i = sum; i >= 0; --i) {
                const int p = sum - i;
#pragma unroll
                for (int s = 0; s < 2; ++s) {
                    if constexpr (ModeInfo<MODE>::f16)
                        acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(vec8<V, E>(&x[i][8 * s]), bq.v[p][s], acc, 0, 0,
                                                                     0);
                    else
                        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(vec8<V, E>(&x[i][8 * s]), bq.v[p][s], acc, 0,
                                                                      0, 0);
                }
            }
    }
    return acc;
}

// Each 4 KB block moves between HBM and registers through a per-wavefront LDS tile
// (row pitch 36 floats): the global side is contiguous (lane l carries the l-th
// 16-byte chunk of each 1 KB quarter), the register side is the MFMA layout (lane
// (h, c): row c, columns 8 qq + 4 h .. +3), and the 36-float pitch keeps the 16-byte
// LDS reads and writes of consecutive rows on distinct banks.
constexpr int M32_P = 36;

__device__ __forceinline__ void wave_lds_fence()
{
    // LDS traffic of one wavefront is processed in order; this only orders the compiler
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

template <int MODE, int DIR, int UNROLL>
__global__ void __launch_bounds__(256)
k_mfma32(Addr a, int64_t batch, QTab q)
{
    constexpr int T0 = ModeInfo<MODE>::target;
    __shared__ float4 lds4[4 * UNROLL * 32 * M32_P / 4];
    const int lane = threadIdx.x & 63;
    const int h = lane >> 5, c = lane & 31;
    float* wl = reinterpret_cast<float*>(lds4) + (threadIdx.x >> 6) * UNROLL * 32 * M32_P;
    const int64_t wave = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / 64);
    const B32P<MODE> bf = pack_b32<MODE>(load_b32<MODE>(q, false, h, c));
    const B32P<MODE> bi = pack_b32<MODE>(load_b32<MODE>(q, true, h, c));
    long bf8[2] = {0, 0}, bi8[2] = {0, 0};
    if constexpr (MODE == M_FP8) {
        bf8[0] = load_b32_f8<MODE>(q, false, h, c, 0);
        bf8[1] = load_b32_f8<MODE>(q, false, h, c, 1);
        bi8[0] = load_b32_f8<MODE>(q, true, h, c, 0);
        bi8[1] = load_b32_f8<MODE>(q, true, h, c, 1);
    }
    const float qscale = MODE == M_FP8 ? 1.0f / (float)(1 << kF8QShift) : 1.0f;
    for (int64_t b0 = wave * UNROLL; b0 < batch; b0 += nwaves * UNROLL) {
        // coalesced loads: chunk ch = 64 qq + lane of block u -> row ch / 8, columns 4 (ch % 8)
        float4 g[UNROLL][4];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u)
#pragma unroll
            for (int qq = 0; qq < 4; ++qq) {
                g[u][qq] = make_float4(0.f, 0.f, 0.f, 0.f);
                if (b0 + u < batch) g[u][qq] = *reinterpret_cast<const gfloat4*>(a.src(b0 + u) + 4 * (64 * qq + lane));
            }
        wave_lds_fence();
#pragma unroll
        for (int u = 0; u < UNROLL; ++u)
#pragma unroll
            for (int qq = 0; qq < 4; ++qq) {
                const int ch = 64 * qq + lane;
                *reinterpret_cast<float4*>(wl + u * 32 * M32_P + (ch >> 3) * M32_P + 4 * (ch & 7)) = g[u][qq];
            }
        wave_lds_fence();
        float d[UNROLL][16];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u)
#pragma unroll
            for (int qq = 0; qq < 4; ++qq) {
                const float4 v = *reinterpret_cast<const float4*>(wl + u * 32 * M32_P + c * M32_P + 8 * qq + 4 * h);
                d[u][4 * qq] = v.x; d[u][4 * qq + 1] = v.y; d[u][4 * qq + 2] = v.z; d[u][4 * qq + 3] = v.w;
            }
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            float m = 0.f;
#pragma unroll
            for (int r = 0; r < 16; ++r) m = fmaxf(m, fabsf(d[u][r]));
            m = lane_max<1, 2, 4, 8, 16, 32>(m);
            int etot = scale_exponent<T0>(m);
#pragma unroll
            for (int r = 0; r < 16; ++r) d[u][r] = ldexpf(d[u][r], -etot);
            constexpr int npass = DIR == DCT2D_ROUNDTRIP ? 4 : 2;
#pragma unroll
            for (int ps = 0; ps < npass; ++ps) {
                const bool inv = DIR == DCT2D_INVERSE || (DIR == DCT2D_ROUNDTRIP && ps >= 2);
                const f32x16 acc = pass32p<MODE>(d[u], inv ? bi : bf, inv ? bi8 : bf8);
#pragma unroll
                for (int r = 0; r < 16; ++r) d[u][r] = acc[r] * qscale;
                if (ModeInfo<MODE>::rescale && ps + 1 < npass) {
                    float m2 = 0.f;
#pragma unroll
                    for (int r = 0; r < 16; ++r) m2 = fmaxf(m2, fabsf(d[u][r]));
                    m2 = lane_max<1, 2, 4, 8, 16, 32>(m2);
                    const int e1 = scale_exponent<T0>(m2);
                    etot += e1;
#pragma unroll
                    for (int r = 0; r < 16; ++r) d[u][r] = ldexpf(d[u][r], -e1);
                }
            }
#pragma unroll
            for (int qq = 0; qq < 4; ++qq)
                *reinterpret_cast<float4*>(wl + u * 32 * M32_P + c * M32_P + 8 * qq + 4 * h) =
                    make_float4(ldexpf(d[u][4 * qq], etot), ldexpf(d[u][4 * qq + 1], etot),
                                ldexpf(d[u][4 * qq + 2], etot), ldexpf(d[u][4 * qq + 3], etot));
        }
        wave_lds_fence();
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            if (b0 + u >= batch) continue;
            gfloat* dst = a.dst(b0 + u);
#pragma unroll
            for (int qq = 0; qq < 4; ++qq) {
                const int ch = 64 * qq + lane;
                *reinterpret_cast<gfloat4*>(dst + 4 * ch) =
                    *reinterpret_cast<const float4*>(wl + u * 32 * M32_P + (ch >> 3) * M32_P + 4 * (ch & 7));
            }
        }
        wave_lds_fence();
    }
}

// ---- 64 x 64 blocks as 2 x 2 tiles of the 32 x 32 form ---------------------------------
// The exact 64-point product Q_64 X Q_64^T with Q_64 cut into four 32 x 32 tiles: output
// tile (I, J) of a pass is sum_K A(I, K) B(K, J), eight tile products per pass.  The
// accumulator of tile (K, I) after pass 1 serves as the A operand of tile (I, K) in pass 2
// (the same transpose-by-reuse as the 32 x 32 kernel, applied tile-wise).
//
// B operands live in LDS, built once per workgroup: operand (K, J, part p, instruction half s)
// of a direction holds, for lane (h, c), the eight 16-bit (fp8: 8-bit) values
// B[32 K + k(s, j)][32 J + c], k(s, j) = 8 (2 s + j / 4) + 4 h + j % 4, where B[k][n] is entry
// (n, k) of Q (forward) or of Q^T (inverse); a lane reads one operand with one 16-byte (fp8:
// 8-byte) access, consecutive lanes on consecutive addresses.  24 operands per direction
// (24 KB; the round trip keeps both directions).  The A tile is split into packed parts once
// per (I, K) and stays in registers as 16-bit vectors.
constexpr int kB64Ops = 24; // (K, J, p, s)

__host__ __device__ constexpr int b64_op(int K, int J, int p, int s) { return ((K * 2 + J) * 3 + p) * 2 + s; }

// Builds the B operands of `ndir` directions (d = 0: the first pass's, d = 1: the inverse's
// for the round trip) in LDS; every thread of the workgroup takes part.
template <int MODE>
__device__ __forceinline__ void fill_b64(uint4* lds, const QTab& q, int ndir, bool first_inv)
{
    constexpr bool F8 = ModeInfo<MODE>::f8;
    const int nent = ndir * kB64Ops * 64; // (direction, operand, lane)
    for (int e = threadIdx.x; e < nent; e += blockDim.x) {
        const int lane = e & 63, op = (e >> 6) % kB64Ops, d = e / (64 * kB64Ops);
        const bool inv = d == 0 ? first_inv : true;
        const int s = op & 1, p = (op >> 1) % 3, J = (op / 6) & 1, K = op / 12;
        const int h = lane >> 5, c = lane & 31;
        const int n = 32 * J + c;
        uint32_t w[4] = {0u, 0u, 0u, 0u};
        if (F8 ? p == 0 : p < ModeInfo<MODE>::parts) {
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int k = 32 * K + 8 * (2 * s + j / 4) + 4 * h + (j & 3);
                const int i = n * 64 + k;
                if constexpr (F8) {
                    const uint32_t byte = (inv ? q.f8t : q.f8)[i];
                    w[j / 4] |= byte << (8 * (j & 3));
                } else {
                    const uint32_t bits = ModeInfo<MODE>::f16 ? (inv ? q.hft : q.hf)[p * 4096 + i]
                                                              : (inv ? q.bft : q.bf)[p * 4096 + i];
                    w[j / 2] |= bits << (16 * (j & 1));
                }
            }
        }
        lds[e] = make_uint4(w[0], w[1], w[2], w[3]);
    }
}

template <class V>
__device__ __forceinline__ V lds_b8(const uint4* lds, int d, int op, int lane)
{
    return __builtin_bit_cast(V, lds[(d * kB64Ops + op) * 64 + lane]);
}

// acc(I, J) += A(I, K) * B(K, J) over the kept split products (smallest terms first);
// av[i][s]: part i of the A tile's k-slots of instruction half s.
template <int MODE, class V>
__device__ __forceinline__ void tile_products(f32x16& acc, const V (&av)[3][2], const uint4* lds, int d, int K, int J,
                                              int lane)
{
    constexpr int P = ModeInfo<MODE>::parts;
#pragma unroll
    for (int sum = P - 1; sum >= 0; --sum)
#pragma unroll
        for (int i = sum; i >= 0; --i) {
            const int p = sum - i;
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const V bv = lds_b8<V>(lds, d, b64_op(K, J, p, s), lane);
                if constexpr (ModeInfo<MODE>::f16)
                    acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(av[i][s], bv, acc, 0, 0, 0);
                else
                    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[i][s], bv, acc, 0, 0, 0);
            }
        }
}

// Two workgroups per CU (at most 256 registers per lane, the accumulators included) where
// the kernel fits them without spilling; the three-part round trip keeps one.
template <int MODE, int DIR>
__global__ void __launch_bounds__(256, (MODE == M_BF16X6 && DIR == DCT2D_ROUNDTRIP) ? 1 : 2)
k_mfma64(Addr a, int64_t batch, QTab q)
{
    constexpr int T0 = ModeInfo<MODE>::target;
    constexpr int NDIR = DIR == DCT2D_ROUNDTRIP ? 2 : 1;
    __shared__ uint4 bl[NDIR * kB64Ops * 64];
    fill_b64<MODE>(bl, q, NDIR, DIR == DCT2D_INVERSE);
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int h = lane >> 5, c = lane & 31;
    const int64_t wave = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / 64);
    const float qscale = MODE == M_FP8 ? 1.0f / (float)(1 << kF8QShift) : 1.0f;
    using V = typename std::conditional<ModeInfo<MODE>::f16, f16x8, bf16x8>::type;
    using E = typename std::conditional<ModeInfo<MODE>::f16, _Float16, __bf16>::type;
    for (int64_t b = wave; b < batch; b += nwaves) {
        // d[I][K][16]: lane (h, c) holds row 32 I + c, columns 32 K + 8 qq + 4 h .. +3
        float d[2][2][16];
        const gfloat* src = a.src(b);
#pragma unroll
        for (int I = 0; I < 2; ++I)
#pragma unroll
            for (int K = 0; K < 2; ++K)
#pragma unroll
                for (int qq = 0; qq < 4; ++qq) {
                    const float4 v =
                        *reinterpret_cast<const gfloat4*>(src + (32 * I + c) * 64 + 32 * K + 8 * qq + 4 * h);
                    d[I][K][4 * qq] = v.x; d[I][K][4 * qq + 1] = v.y;
                    d[I][K][4 * qq + 2] = v.z; d[I][K][4 * qq + 3] = v.w;
                }
        float m = 0.f;
#pragma unroll
        for (int I = 0; I < 2; ++I)
#pragma unroll
            for (int K = 0; K < 2; ++K)
#pragma unroll
                for (int r = 0; r < 16; ++r) m = fmaxf(m, fabsf(d[I][K][r]));
        m = lane_max<1, 2, 4, 8, 16, 32>(m);
        int etot = scale_exponent<T0>(m);
#pragma unroll
        for (int I = 0; I < 2; ++I)
#pragma unroll
            for (int K = 0; K < 2; ++K)
#pragma unroll
                for (int r = 0; r < 16; ++r) d[I][K][r] = ldexpf(d[I][K][r], -etot);
        constexpr int npass = DIR == DCT2D_ROUNDTRIP ? 4 : 2;
#pragma unroll
        for (int ps = 0; ps < npass; ++ps) {
            const int dsel = DIR == DCT2D_ROUNDTRIP && ps >= 2 ? 1 : 0;
            f32x16 acc[2][2];
#pragma unroll
            for (int I = 0; I < 2; ++I)
#pragma unroll
                for (int J = 0; J < 2; ++J)
#pragma unroll
                    for (int r = 0; r < 16; ++r) acc[I][J][r] = 0.f;
#pragma unroll
            for (int I = 0; I < 2; ++I)
#pragma unroll
                for (int K = 0; K < 2; ++K) {
                    // A tile (I, K): pass 1 holds X(I, K) at d[I][K]; later passes hold the
                    // previous accumulator tile (K, I), whose registers represent its transpose
                    const float* at = ps == 0 ? d[I][K] : d[K][I];
                    if constexpr (MODE == M_FP8) {
#pragma unroll
                        for (int J = 0; J < 2; ++J)
#pragma unroll
                            for (int s = 0; s < 2; ++s) {
                                int lo = __builtin_amdgcn_cvt_pk_fp8_f32(at[8 * s + 0], at[8 * s + 1], 0, false);
                                lo = __builtin_amdgcn_cvt_pk_fp8_f32(at[8 * s + 2], at[8 * s + 3], lo, true);
                                int hi = __builtin_amdgcn_cvt_pk_fp8_f32(at[8 * s + 4], at[8 * s + 5], 0, false);
                                hi = __builtin_amdgcn_cvt_pk_fp8_f32(at[8 * s + 6], at[8 * s + 7], hi, true);
                                const long av = (long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
                                const uint4 bw = bl[(dsel * kB64Ops + b64_op(K, J, 0, s)) * 64 + lane];
                                const long bv = (long)(((uint64_t)bw.y << 32) | bw.x);
                                acc[I][J] = __builtin_amdgcn_mfma_f32_32x32x16_fp8_fp8(av, bv, acc[I][J], 0, 0, 0);
                            }
                    } else {
                        V av[3][2];
#pragma unroll
                        for (int s = 0; s < 2; ++s)
#pragma unroll
                            for (int r = 0; r < 8; ++r) {
                                float pp[3];
                                split<MODE>(at[8 * s + r], pp);
#pragma unroll
                                for (int i = 0; i < ModeInfo<MODE>::parts; ++i) av[i][s][r] = (E)pp[i];
                            }
#pragma unroll
                        for (int J = 0; J < 2; ++J) tile_products<MODE, V>(acc[I][J], av, bl, dsel, K, J, lane);
                    }
                }
#pragma unroll
            for (int I = 0; I < 2; ++I)
#pragma unroll
                for (int J = 0; J < 2; ++J)
#pragma unroll
                    for (int r = 0; r < 16; ++r) d[I][J][r] = acc[I][J][r] * qscale;
            if (ModeInfo<MODE>::rescale && ps + 1 < npass) {
                float m2 = 0.f;
#pragma unroll
                for (int I = 0; I < 2; ++I)
#pragma unroll
                    for (int J = 0; J < 2; ++J)
#pragma unroll
                        for (int r = 0; r < 16; ++r) m2 = fmaxf(m2, fabsf(d[I][J][r]));
                m2 = lane_max<1, 2, 4, 8, 16, 32>(m2);
                const int e1 = scale_exponent<T0>(m2);
                etot += e1;
#pragma unroll
                for (int I = 0; I < 2; ++I)
#pragma unroll
                    for (int J = 0; J < 2; ++J)
#pragma unroll
                        for (int r = 0; r < 16; ++r) d[I][J][r] = ldexpf(d[I][J][r], -e1);
            }
        }
        // after an even number of passes the lane holds tile (I, J) of Y^T:
        // row 32 J + c, columns 32 I + 8 qq + 4 h .. +3 of Y
        gfloat* dst = a.dst(b);
#pragma unroll
        for (int I = 0; I < 2; ++I)
#pragma unroll
            for (int J = 0; J < 2; ++J)
#pragma unroll
                for (int qq = 0; qq < 4; ++qq)
                    *reinterpret_cast<gfloat4*>(dst + (32 * J + c) * 64 + 32 * I + 8 * qq + 4 * h) =
                        make_float4(ldexpf(d[I][J][4 * qq], etot), ldexpf(d[I][J][4 * qq + 1], etot),
                                    ldexpf(d[I][J][4 * qq + 2], etot), ldexpf(d[I][J][4 * qq + 3], etot));
    }
}

// ---- launchers ---------------------------------------------------------------------------
QTab qtab(const DeviceTables* t, int n)
{
    int i = 0;
    while ((8 << i) < n) ++i;
    return QTab{t->q_bf16[i], t->q_f16[i], t->q_f8[i], n, t->q_bf16_t[i], t->q_f16_t[i], t->q_f8_t[i]};
}

// Resident wavefronts per CU of the grid-stride variants: all 32 the kernels' registers allow,
// or fewer (variants 4 and up) when fewer bytes in flight per CU keep HBM closer to its
// streaming rate.
int waves_per_cu(int variant)
{
    return variant == 4 || variant == 6 ? 16 : variant == 5 || variant == 7 ? 8 : 32;
}

template <int N, int MODE, int DIR, int UNROLL>
int go16(const DeviceTables* t, const Job& j)
{
    constexpr int BPT = N == 8 ? 4 : 1;
    const int64_t ntiles = (j.batch + BPT - 1) / BPT;
    const int64_t waves_needed = (ntiles + UNROLL - 1) / UNROLL;
    // variant 3: one iteration per wavefront (no grid-stride reuse); otherwise grid-stride
    const int64_t cap = j.variant == 3 ? ((int64_t)1 << 32) : (int64_t)t->num_cu * waves_per_cu(j.variant);
    const int64_t waves = waves_needed < cap ? waves_needed : cap;
    const unsigned grid = (unsigned)((waves + 3) / 4);
    k_mfma16<N, MODE, DIR, UNROLL><<<grid, 256, 0, j.stream>>>(j.addr(), j.batch, qtab(t, N));
    return hipGetLastError() == hipSuccess ? DCT2D_OK : DCT2D_ERR_HIP;
}

template <int MODE, int DIR, int UNROLL>
int go32(const DeviceTables* t, const Job& j)
{
    const int64_t waves_needed = (j.batch + UNROLL - 1) / UNROLL;
    const int64_t cap = (int64_t)t->num_cu * waves_per_cu(j.variant);
    const int64_t waves = waves_needed < cap ? waves_needed : cap;
    const unsigned grid = (unsigned)((waves + 3) / 4);
    k_mfma32<MODE, DIR, UNROLL><<<grid, 256, 0, j.stream>>>(j.addr(), j.batch, qtab(t, 32));
    return hipGetLastError() == hipSuccess ? DCT2D_OK : DCT2D_ERR_HIP;
}

template <int MODE, int DIR>
int go64(const DeviceTables* t, const Job& j)
{
    // grid-stride over blocks with only resident workgroups (registers and the LDS operand
    // table bound the residency): a workgroup that waits for a slot would run its share of
    // the blocks after the others have finished
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_mfma64<MODE, DIR>, 256, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    // variants 1 and 2: at most two / one workgroup per CU (fewer blocks in flight per CU)
    if (j.variant == 1 && per_cu > 2) per_cu = 2;
    if (j.variant == 2) per_cu = 1;
    const int64_t cap = (int64_t)t->num_cu * per_cu * 4;
    const int64_t waves = j.batch < cap ? j.batch : cap;
    const unsigned grid = (unsigned)((waves + 3) / 4);
    k_mfma64<MODE, DIR><<<grid, 256, 0, j.stream>>>(j.addr(), j.batch, qtab(t, 64));
    return hipGetLastError() == hipSuccess ? DCT2D_OK : DCT2D_ERR_HIP;
}

template <int MODE, int DIR>
int go_unroll(const DeviceTables* t, const Job& j)
{
    // variant = unroll choice: 0 -> 2 tiles per iteration, 1 -> 1, 2 -> 4; 3: unroll 1, one
    // iteration per wavefront (16 x 16 tiles only); 4, 5: unroll 1 with 16 / 8 wavefronts per
    // CU; 6, 7: unroll 2 with 16 / 8 wavefronts per CU
    const int v = j.variant;
    const bool u1 = v == 1 || v == 3 || v == 4 || v == 5, u4 = v == 2;
    switch (j.rows) {
    case 8:
        return u1 ? go16<8, MODE, DIR, 1>(t, j) : u4 ? go16<8, MODE, DIR, 4>(t, j) : go16<8, MODE, DIR, 2>(t, j);
    case 16:
        return u1 ? go16<16, MODE, DIR, 1>(t, j) : u4 ? go16<16, MODE, DIR, 4>(t, j) : go16<16, MODE, DIR, 2>(t, j);
    case 32:
        return u1 ? go32<MODE, DIR, 1>(t, j) : u4 ? go32<MODE, DIR, 4>(t, j) : go32<MODE, DIR, 2>(t, j);
    case 64:
        return go64<MODE, DIR>(t, j);
    default:
        return DCT2D_ERR_PRECISION;
    }
}

template <int MODE>
int go_dir(const DeviceTables* t, const Job& j)
{
    switch (j.dir) {
    case DCT2D_FORWARD: return go_unroll<MODE, DCT2D_FORWARD>(t, j);
    case DCT2D_INVERSE: return go_unroll<MODE, DCT2D_INVERSE>(t, j);
    default: return go_unroll<MODE, DCT2D_ROUNDTRIP>(t, j);
    }
}

} // namespace

int mfma_supported(int rows, int cols, int precision)
{
    if (precision < DCT2D_SPLIT_BF16X3 || precision > DCT2D_FP8_E4M3) return 0;
    return rows == cols && (rows == 8 || rows == 16 || rows == 32 || rows == 64);
}

int mfma_variant_count(int rows, int cols, int, int precision)
{
    if (!mfma_supported(rows, cols, precision)) return 0;
    // N < 64: unroll 2 / 1 / 4, one-shot grid, capped residency (N = 32: 3 = 1); N = 64:
    // resident workgroups per CU as many as fit / two / one
    return rows == 64 ? 3 : 8;
}

int launch_mfma(const DeviceTables* t, const Job& j, int precision)
{
    if (!mfma_supported(j.rows, j.cols, precision)) return DCT2D_ERR_PRECISION;
    switch (precision) {
    case DCT2D_SPLIT_BF16X3: return go_dir<M_BF16X3>(t, j);
    case DCT2D_SPLIT_BF16X6: return go_dir<M_BF16X6>(t, j);
    case DCT2D_SPLIT_FP16X3: return go_dir<M_FP16X3>(t, j);
    case DCT2D_BF16: return go_dir<M_BF16>(t, j);
    case DCT2D_FP16: return go_dir<M_FP16>(t, j);
    case DCT2D_FP8_E4M3: return go_dir<M_FP8>(t, j);
    default: return DCT2D_ERR_PRECISION;
    }
}

} // namespace dct
