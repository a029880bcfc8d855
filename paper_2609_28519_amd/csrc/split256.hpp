// A length-256 orthonormal DCT-II / DCT-III shared by four threads ("roles"), each holding
// 64 values, through the top two levels of the even/odd recursion of dct1d.hpp:
//
//   u[n] = x[n] + x[255-n], w[n] = x[n] - x[255-n]                       (n < 128)
//   X[2k]   = DCT-II_128(u)[k]:  uu[n] = u[n] + u[127-n] -> DCT-II_64  -> X[4k]      (role 0)
//                                uw[n] = u[n] - u[127-n] -> DCT-IV_64  -> X[4k + 2]  (role 1)
//   X[2k+1] = DCT-IV_128(w)[k]:  one 64-point complex FFT between two twiddle products,
//            split by one radix-2 step over roles 2 and 3: role 2 transforms the even-indexed
//            inputs t[2i], role 3 the odd-indexed t[2i+1] (each a 32-point FFT); role 3
//            multiplies by W_64^k; after an exchange, role 2 forms c[k] = E[k] + W^k O[k]
//            and role 3 c[k + 32] = E[k] - W^k O[k]; each applies the post-twiddles of its
//            half: role 2 yields X[4k + 1] and X[255 - 4k] for k < 32, role 3 the same
//            for 32 <= k < 64.
//
// The inverse (DCT-III_256, Q^T) is the transposed graph (Section 2.2, Prop. 2): role 0
// DCT-III_64 of X[4k], role 1 DCT-IV_64 of X[4k + 2], roles 2 and 3 DCT-IV_128 of the odd
// coefficients (the same split FFT), recombined as u'[n] = aa[n] + ab[n],
// u'[127-n] = aa[n] - ab[n], x[n] = u'[n] + w'[n], x[255-n] = u'[n] - w'[n].
//
// The functions work on one "line" of 256 floats in shared memory through an accessor
// (element i: a.at(i); lines stored as 64 contiguous 16-byte groups also offer a.g4(g) and
// a.s4(g, v), and every access then goes through whole groups), and are split into phases:
// the caller runs every role's phase k before any role's phase k + 1 (a workgroup barrier
// on the GPU), so the host can replay them in order.
//
// Layout of the forward outputs in the line ("blocked"): role 0's 64 values X[4k] at
// [0, 64), role 1's X[4k + 2] at [64, 128), role 3's at [128, 192), role 2's at [192, 256)
// (roles 2 and 3 write where their partner's exchange data was, which they have read).
// Within the two odd blocks, value k of a role is its c index: role 2 holds X[4k + 1]
// (k < 32) at 192 + k and X[255 - 4k] at 255 - k; role 3 holds X[4k + 1] (32 <= k < 64) at
// 128 + (k - 32) and X[255 - 4k] at 191 - (k - 32).  blocked_pos() gives the position of X[m].
#pragma once
#include <hip/hip_runtime.h>

#include "dct1d.hpp"

namespace dct {
namespace s4 {

using T256 = TwLayout<256>;

// Position of coefficient X[m] in the blocked layout.
__host__ __device__ constexpr int blocked_pos(int m)
{
    return (m & 3) == 0   ? m >> 2
           : (m & 3) == 2 ? 64 + (m >> 2)
           : (m & 3) == 1 ? ((m >> 2) < 32 ? 192 + (m >> 2) : 128 + (m >> 2) - 32)
                          // m = 255 - 4k, k = (255 - m) / 4
                          : (((255 - m) >> 2) < 32 ? 255 - ((255 - m) >> 2) : 191 - (((255 - m) >> 2) - 32));
}

// Coefficient index m held at position p of the blocked layout (the inverse of blocked_pos).
__host__ __device__ constexpr int blocked_logical(int p)
{
    return p < 64    ? 4 * p
           : p < 128 ? 4 * (p - 64) + 2
           : p < 160 ? 4 * (p - 128 + 32) + 1      // role 3: X[4k + 1], 32 <= k < 64
           : p < 192 ? 255 - 4 * (191 - p + 32)    // role 3: X[255 - 4k], 32 <= k < 64
           : p < 224 ? 4 * (p - 192) + 1           // role 2: X[4k + 1], k < 32
                     : 255 - 4 * (255 - p);        // role 2: X[255 - 4k], k < 32
}

// ---- accessors ---------------------------------------------------------------------------

// Element i at p[i * STEP]; with STEP 1 the line is 64 contiguous 16-byte groups.
template <int STEP>
struct Strided {
    float* p;
    static constexpr bool VEC = STEP == 1;
    __host__ __device__ float& at(int i) const { return p[i * STEP]; }
    __host__ __device__ float4 g4(int g) const { return reinterpret_cast<const float4*>(p)[g]; }
    __host__ __device__ void s4(int g, float4 v) const { reinterpret_cast<float4*>(p)[g] = v; }
};

// A contiguous line whose 16-byte groups are XOR-permuted by a per-line key < 8: logical
// group g sits at group g ^ key.
struct Swizzled {
    float* p;
    int key;
    static constexpr bool VEC = true;
    __host__ __device__ float& at(int i) const { return p[4 * ((i >> 2) ^ key) + (i & 3)]; }
    __host__ __device__ float4 g4(int g) const { return reinterpret_cast<const float4*>(p)[g ^ key]; }
    __host__ __device__ void s4(int g, float4 v) const { reinterpret_cast<float4*>(p)[g ^ key] = v; }
};

__host__ __device__ __forceinline__ float el(const float4& q, int i) { return i == 0 ? q.x : i == 1 ? q.y : i == 2 ? q.z : q.w; }

// ---- forward -----------------------------------------------------------------------------

// Phase 1: the role's inputs from the natural-order line.  Roles 0, 1: uu / uw (64 reals);
// roles 2, 3: the complex pairs (w[2j], w[127 - 2j]) of their FFT half, j = 2i + (role - 2),
// as v[2i], v[2i + 1].  Vector lines are read as 16-byte groups only.
template <int R, class A>
__host__ __device__ __forceinline__ void fwd_in(const A& a, float (&v)[64])
{
    if constexpr (A::VEC && R < 2) {
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const float4 lo = a.g4(j), hi = a.g4(63 - j), a2 = a.g4(31 - j), b2 = a.g4(32 + j);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float s = el(lo, q) + el(hi, 3 - q), t = el(a2, 3 - q) + el(b2, q);
                v[4 * j + q] = R == 0 ? s + t : s - t;
            }
        }
    } else if constexpr (A::VEC) {
        constexpr int e = 2 * (R - 2); // element of the 16-byte group that holds x[2j]
#pragma unroll
        for (int i = 0; i < 32; ++i) {
            v[2 * i] = el(a.g4(i), e) - el(a.g4(63 - i), 3 - e);          // x[2j] - x[255 - 2j]
            v[2 * i + 1] = el(a.g4(31 - i), 3 - e) - el(a.g4(32 + i), e); // x[127 - 2j] - x[128 + 2j]
        }
    } else if constexpr (R < 2) {
#pragma unroll
        for (int n = 0; n < 64; ++n) {
            const float s = a.at(n) + a.at(255 - n);
            const float t = a.at(127 - n) + a.at(128 + n);
            v[n] = R == 0 ? s + t : s - t;
        }
    } else {
#pragma unroll
        for (int i = 0; i < 32; ++i) {
            const int j = 2 * i + (R - 2);
            v[2 * i] = a.at(2 * j) - a.at(255 - 2 * j);           // w[2j]
            v[2 * i + 1] = a.at(127 - 2 * j) - a.at(128 + 2 * j); // w[127 - 2j]
        }
    }
}

// Roles 2, 3 (forward and inverse alike): pre-twiddles and the 32-point FFT of their half of
// the DCT-IV_128 input pairs; role 3 also applies W_64^k.  f holds 32 complex values.
template <int R>
__host__ __device__ __forceinline__ void fft_half(const float (&v)[64], float (&f)[64], twptr tw)
{
    cf t[32], c[32];
#pragma unroll
    for (int i = 0; i < 32; ++i) t[i] = cmul(cf{v[2 * i], v[2 * i + 1]}, tw[T256::pre(128) + 2 * i + (R - 2)]);
    tw_fence(tw);
    fft_rec<32, 1, false, T256::FFT_TOP>(t, c, tw);
    tw_fence(tw);
#pragma unroll
    for (int k = 0; k < 32; ++k) {
        const cf e = R == 3 ? twiddle_dyn<T256::FFT_TOP, false>(c[k], k, tw) : c[k];
        f[2 * k] = e.x;
        f[2 * k + 1] = e.y;
    }
}

// Roles 2, 3: the exchange half they publish (written where the partner's outputs will go).
template <int R, class A>
__host__ __device__ __forceinline__ void put_half(const A& a, const float (&f)[64])
{
    constexpr int base = R == 2 ? 128 : 192;
    if constexpr (A::VEC) {
#pragma unroll
        for (int g = 0; g < 16; ++g) a.s4(base / 4 + g, make_float4(f[4 * g], f[4 * g + 1], f[4 * g + 2], f[4 * g + 3]));
    } else {
#pragma unroll
        for (int k = 0; k < 64; ++k) a.at(base + k) = f[k];
    }
}

// Roles 2, 3: combine with the partner's half and post-twiddle: o[2k], o[2k + 1] are y[2kk],
// y[127 - 2kk] of the DCT-IV_128 with kk = k + 32 (role - 2).
template <int R, class A>
__host__ __device__ __forceinline__ void combine_half(const A& a, const float (&f)[64], float (&o)[64], twptr tw)
{
    constexpr int pbase = R == 2 ? 192 : 128; // the partner's published half
#pragma unroll
    for (int k = 0; k < 32; ++k) {
        float px, py;
        if constexpr (A::VEC) {
            const float4 g = a.g4(pbase / 4 + k / 2);
            px = k % 2 ? g.z : g.x;
            py = k % 2 ? g.w : g.y;
        } else {
            px = a.at(pbase + 2 * k);
            py = a.at(pbase + 2 * k + 1);
        }
        // role 2: E = f, W^k O = partner;  role 3: W^k O = f, E = partner
        const cf c = R == 2 ? cf{f[2 * k] + px, f[2 * k + 1] + py} : cf{px - f[2 * k], py - f[2 * k + 1]};
        const float2 q = tw[T256::post(128) + k + 32 * (R - 2)];
        o[2 * k] = c.x * q.x + c.y * q.y;
        o[2 * k + 1] = c.x * q.y - c.y * q.x;
    }
}

// Roles 0, 1: the 64-point transforms of the forward.
template <int R>
__host__ __device__ __forceinline__ void fwd_tf01(const float (&v)[64], float (&o)[64], twptr tw)
{
    if constexpr (R == 0) dct2_rec<256, 64>(v, o, tw); else dct4_scaled<256, 64>(v, o, tw);
}

// The role's 64 outputs into the blocked layout (roles 2 and 3 after their exchange).
template <int R, class A>
__host__ __device__ __forceinline__ void fwd_out(const A& a, const float (&o)[64])
{
    if constexpr (A::VEC && R < 2) {
#pragma unroll
        for (int g = 0; g < 16; ++g) a.s4(16 * R + g, make_float4(o[4 * g], o[4 * g + 1], o[4 * g + 2], o[4 * g + 3]));
    } else if constexpr (A::VEC) {
        constexpr int base = R == 2 ? 192 : 128;
#pragma unroll
        for (int g = 0; g < 8; ++g) {
            // positions base + 4g .. +3 hold o[8g], o[8g + 2], o[8g + 4], o[8g + 6]; positions
            // base + 60 - 4g .. +3 hold o[8g + 7], o[8g + 5], o[8g + 3], o[8g + 1]
            a.s4(base / 4 + g, make_float4(o[8 * g], o[8 * g + 2], o[8 * g + 4], o[8 * g + 6]));
            a.s4(base / 4 + 15 - g, make_float4(o[8 * g + 7], o[8 * g + 5], o[8 * g + 3], o[8 * g + 1]));
        }
    } else if constexpr (R < 2) {
#pragma unroll
        for (int k = 0; k < 64; ++k) a.at(64 * R + k) = o[k];
    } else {
        constexpr int base = R == 2 ? 192 : 128;
#pragma unroll
        for (int k = 0; k < 32; ++k) {
            a.at(base + k) = o[2 * k];
            a.at(base + 63 - k) = o[2 * k + 1];
        }
    }
}

// ---- inverse -------------------------------------------------------------------------------

// Phase 1: the role's inputs.  Roles 0, 1: X[4k] / X[4k + 2]; roles 2, 3: the pairs
// (X[4j + 1], X[255 - 4j]) (the odd coefficients yo[2j], yo[127 - 2j]) of their FFT half,
// j = 2i + (role - 2).  NATURAL: the line holds the coefficients in natural order (else in
// the blocked layout).  MUL: coefficient X[m] is first multiplied by lam[m * LSTEP] (the
// spectral filter's multipliers along the line; lam may point to any address space).
template <int R, class A, bool NATURAL = false, bool MUL = false, int LSTEP = 0, typename LP = const float*>
__host__ __device__ __forceinline__ void inv_in(const A& a, float (&v)[64], LP lam = nullptr)
{
    // the value of X[m]
    auto get = [&](int m) -> float {
        const int p = NATURAL ? m : blocked_pos(m);
        if constexpr (A::VEC) return el(a.g4(p >> 2), p & 3);
        else return a.at(p);
    };
    if constexpr (R < 2) {
#pragma unroll
        for (int k = 0; k < 64; ++k) {
            v[k] = get(4 * k + 2 * R);
            if constexpr (MUL) v[k] *= lam[(4 * k + 2 * R) * LSTEP];
        }
    } else {
#pragma unroll
        for (int i = 0; i < 32; ++i) {
            const int j = 2 * i + (R - 2);
            v[2 * i] = get(4 * j + 1);
            v[2 * i + 1] = get(255 - 4 * j);
            if constexpr (MUL) {
                v[2 * i] *= lam[(4 * j + 1) * LSTEP];
                v[2 * i + 1] *= lam[(255 - 4 * j) * LSTEP];
            }
        }
    }
}

template <int R>
__host__ __device__ __forceinline__ void inv_tf01(const float (&v)[64], float (&o)[64], twptr tw)
{
    if constexpr (R == 0) dct3_rec<256, 64>(v, o, tw); else dct4_scaled<256, 64>(v, o, tw);
}

// The recombination into natural order.  With u'[n] = aa[n] + ab[n], u'[127-n] = aa[n] - ab[n]
// (n < 64) and w' the DCT-IV_128 outputs, the four outputs of each n < 64 are
//   x[n] = u'[n] + w'[n],          x[255-n] = u'[n] - w'[n],
//   x[127-n] = u'[127-n] + w'[127-n], x[128+n] = u'[127-n] - w'[127-n],
// so every role can produce 64 of them once it holds aa, ab, w'[n], w'[127-n] for its 16
// values of n (n in [16 role, 16 role + 16)).  Three phases, a barrier after each:
//   inv_part:   each role writes its 64 partial results into the line: aa at [0, 64), ab at
//               [64, 128); role 2's o at [192, 256) and role 3's at [128, 192), i.e. where the
//               partner's exchange half was (which the role itself has read; roles 0 and 1 may
//               run this phase before the exchange, which only uses [128, 256)).  Role 2 holds
//               w'[2kk] = o[2k], w'[127 - 2kk] = o[2k + 1] with kk = k (k < 32), role 3 the
//               same with kk = k + 32, so w'[m] sits at 192 + m (even m < 64), 64 + m (even
//               m >= 64), 192 - m (odd m < 64) and 320 - m (odd m >= 64).
//   inv_gather: each role reads the 64 partials of its n: for n = 4q .. 4q + 3, aa and ab in
//               groups q and 16 + q, and [w'[4q], w'[127-4q], w'[4q+2], w'[125-4q]] in group
//               48 + q, [w'[124-4q], w'[4q+3], w'[126-4q], w'[4q+1]] in group 47 - q.
//   inv_emit:   each role writes its 64 outputs: groups q, 63 - q, 31 - q and 32 + q.
template <int R, class A>
__host__ __device__ __forceinline__ void inv_part(const A& a, const float (&o)[64])
{
    constexpr int base = R == 0 ? 0 : R == 1 ? 64 : R == 2 ? 192 : 128;
    if constexpr (A::VEC) {
#pragma unroll
        for (int g = 0; g < 16; ++g) a.s4(base / 4 + g, make_float4(o[4 * g], o[4 * g + 1], o[4 * g + 2], o[4 * g + 3]));
    } else {
#pragma unroll
        for (int k = 0; k < 64; ++k) a.at(base + k) = o[k];
    }
}

// g[16 qq + i]: i 0..3 aa[n], 4..7 ab[n], 8..15 the two w' groups, n = 4q + (i & 3), q = 4R + qq.
template <int R, class A>
__host__ __device__ __forceinline__ void inv_gather(const A& a, float (&g)[64])
{
#pragma unroll
    for (int qq = 0; qq < 4; ++qq) {
        const int q = 4 * R + qq;
        const int grp[4] = {q, 16 + q, 48 + q, 47 - q};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if constexpr (A::VEC) {
                const float4 v = a.g4(grp[j]);
                g[16 * qq + 4 * j] = v.x;
                g[16 * qq + 4 * j + 1] = v.y;
                g[16 * qq + 4 * j + 2] = v.z;
                g[16 * qq + 4 * j + 3] = v.w;
            } else {
#pragma unroll
                for (int i = 0; i < 4; ++i) g[16 * qq + 4 * j + i] = a.at(4 * grp[j] + i);
            }
        }
    }
}

template <int R, class A>
__host__ __device__ __forceinline__ void inv_emit(const A& a, const float (&g)[64])
{
#pragma unroll
    for (int qq = 0; qq < 4; ++qq) {
        const int q = 4 * R + qq;
        const float* aa = &g[16 * qq];
        const float* ab = aa + 4;
        const float* wa = aa + 8;  // w'[4q], w'[127-4q], w'[4q+2], w'[125-4q]
        const float* wb = aa + 12; // w'[124-4q], w'[4q+3], w'[126-4q], w'[4q+1]
        // w'[n] and w'[127 - n] for n = 4q + i
        const float w1[4] = {wa[0], wb[3], wa[2], wb[1]};
        const float w2[4] = {wa[1], wb[2], wa[3], wb[0]};
        float xa[4], xb[4], xc[4], xd[4]; // x[n], x[255-n], x[127-n], x[128+n]
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float u1 = aa[i] + ab[i], u2 = aa[i] - ab[i];
            xa[i] = u1 + w1[i];
            xb[i] = u1 - w1[i];
            xc[i] = u2 + w2[i];
            xd[i] = u2 - w2[i];
        }
        // group q: x[4q..4q+3]; group 63-q: x[252-4q..255-4q] = xb reversed; group 31-q:
        // x[124-4q..127-4q] = xc reversed; group 32+q: x[128+4q..131+4q] = xd
        if constexpr (A::VEC) {
            a.s4(q, make_float4(xa[0], xa[1], xa[2], xa[3]));
            a.s4(63 - q, make_float4(xb[3], xb[2], xb[1], xb[0]));
            a.s4(31 - q, make_float4(xc[3], xc[2], xc[1], xc[0]));
            a.s4(32 + q, make_float4(xd[0], xd[1], xd[2], xd[3]));
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                a.at(4 * q + i) = xa[i];
                a.at(255 - 4 * q - i) = xb[i];
                a.at(127 - 4 * q - i) = xc[i];
                a.at(128 + 4 * q + i) = xd[i];
            }
        }
    }
}

} // namespace s4
} // namespace dct
