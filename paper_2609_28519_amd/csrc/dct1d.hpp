// One-dimensional orthonormal DCT-II (Q_L x) and its transpose (Q_L^T y) in registers.
//
// Q_L is the matrix of the paper's Section 2.1 eq. 1.  Each routine transforms one
// length-L vector held in a thread's registers; the 2D transforms apply them along
// rows and columns (separable form, Section 1.2 and Section 3.1).  The paper's own
// factorisation (Shao-Johnson scaled split radix on 4-lane NEON bands) was designed
// for a CPU; here every length goes through a half-length complex FFT:
//
//   forward (DCT-II), for L = 2M:
//     v[n] = x[2n], v[L-1-n] = x[2n+1]            even/odd reordering (Makhoul)
//     z[m] = v[2m] + i v[2m+1]                     real length-L data as M complex
//     Z    = DFT_M(z)                              radix-2 FFT in registers
//     V[k] = (Z[k] + Z*[M-k])/2 + W_L^k (Z[k] - Z*[M-k])/(2i)   = DFT_L(v)[k]
//     y[k] = Re(a_k W_4L^k V[k]),  y[L-k] = -Im(a_k W_4L^k V[k])
//   inverse (Q^T = Q^-1): the same steps undone in reverse order, with the factor
//     1/(a_k L) folded into the first twiddle (Section 2.2: scales folded into the
//     transforms, the round trip needs no separate correction).
//
// All twiddles come from the plan-owned table generated on the device in FP64
// (tables.hip); its layout for one length L (M = L/2), in complex entries, is
// TwLayout<L>.  Indices into the table are compile-time constants after unrolling,
// so the loads are wave-uniform and land in scalar registers.
#pragma once
#include <hip/hip_runtime.h>

namespace dct {

struct cf {
    float x, y;
};

__host__ __device__ __forceinline__ cf cadd(cf a, cf b) { return {a.x + b.x, a.y + b.y}; }
__host__ __device__ __forceinline__ cf csub(cf a, cf b) { return {a.x - b.x, a.y - b.y}; }
__host__ __device__ __forceinline__ cf cconj(cf a) { return {a.x, -a.y}; }
__host__ __device__ __forceinline__ cf cmul(cf a, float2 w)
{
    return {a.x * w.x - a.y * w.y, a.x * w.y + a.y * w.x};
}
// a * conj(w)
__host__ __device__ __forceinline__ cf cmulc(cf a, float2 w)
{
    return {a.x * w.x + a.y * w.y, a.y * w.x - a.x * w.y};
}

template <int L>
struct TwLayout {
    static_assert(L >= 4 && (L & (L - 1)) == 0, "power-of-two length");
    static constexpr int M = L / 2;
    static constexpr int FFT = 0;                 // W_M^j,            j = 0..M/2-1
    static constexpr int COMB = M / 2;            // W_L^k,            k = 0..M/2
    static constexpr int POST = COMB + M / 2 + 1; // a_k W_4L^k,        k = 0..M
    static constexpr int PRE = POST + M + 1;      // W_4L^-k/(a_k L),   k = 0..M
    static constexpr int SIZE = PRE + M + 1;
};

__host__ __device__ constexpr int bitrev(int i, int bits)
{
    int r = 0;
    for (int b = 0; b < bits; ++b) r |= ((i >> b) & 1) << (bits - 1 - b);
    return r;
}

__host__ __device__ constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }

// In-place radix-2 decimation-in-time FFT of M complex values in registers.
// INV = false: DFT with W_M = exp(-2 pi i / M); INV = true: unnormalised inverse.
template <int M, bool INV>
__host__ __device__ __forceinline__ void fft_reg(cf (&z)[M], const float2* __restrict__ tw)
{
    constexpr int BITS = ilog2(M);
#pragma unroll
    for (int i = 0; i < M; ++i) {
        const int j = bitrev(i, BITS);
        if (i < j) {
            cf t = z[i];
            z[i] = z[j];
            z[j] = t;
        }
    }
#pragma unroll
    for (int half = 1; half < M; half *= 2) {
        const int step = M / (2 * half); // twiddle exponent stride
#pragma unroll
        for (int i = 0; i < M; i += 2 * half) {
#pragma unroll
            for (int j = 0; j < half; ++j) {
                const int e = j * step;
                cf b = z[i + j + half];
                if (e == 0) {
                } else if (4 * e == M) {
                    // W_M^{M/4} = -i (forward), +i (inverse)
                    b = INV ? cf{-b.y, b.x} : cf{b.y, -b.x};
                } else {
                    b = INV ? cmulc(b, tw[e]) : cmul(b, tw[e]);
                }
                const cf a = z[i + j];
                z[i + j] = cadd(a, b);
                z[i + j + half] = csub(a, b);
            }
        }
    }
}

// x <- Q_L x  (orthonormal DCT-II, eq. 1), L >= 8.
template <int L>
__host__ __device__ __forceinline__ void dct2_ortho(float (&x)[L], const float2* __restrict__ tw)
{
    using T = TwLayout<L>;
    constexpr int M = L / 2;
    cf z[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        // v[n] = x[2n] for n < M, v[n] = x[2(L-1-n)+1] otherwise
        const int n0 = 2 * m, n1 = 2 * m + 1;
        z[m].x = n0 < M ? x[2 * n0] : x[2 * (L - 1 - n0) + 1];
        z[m].y = n1 < M ? x[2 * n1] : x[2 * (L - 1 - n1) + 1];
    }
    fft_reg<M, false>(z, tw + T::FFT);
    const float2* comb = tw + T::COMB;
    const float2* post = tw + T::POST;
    {
        // k = 0 and k = M: V[0] = Re Z0 + Im Z0, V[M] = Re Z0 - Im Z0 (both real)
        const float v0 = z[0].x + z[0].y, vm = z[0].x - z[0].y;
        x[0] = v0 * post[0].x;
        x[M] = vm * post[M].x;
    }
#pragma unroll
    for (int k = 1; k <= M / 2; ++k) {
        const cf zk = z[k], zc = cconj(z[M - k]);
        const cf e = {0.5f * (zk.x + zc.x), 0.5f * (zk.y + zc.y)};
        const cf d = csub(zk, zc);
        const cf o = {0.5f * d.y, -0.5f * d.x}; // d / (2i)
        const cf t = cmul(o, comb[k]);
        const cf p = cmul(cadd(e, t), post[k]);
        x[k] = p.x;
        x[L - k] = -p.y;
        if (k != M - k) {
            const cf q = cmul(cconj(csub(e, t)), post[M - k]);
            x[M - k] = q.x;
            x[M + k] = -q.y;
        }
    }
}

// y <- Q_L^T y  (orthonormal DCT-III, the inverse of dct2_ortho), L >= 8.
template <int L>
__host__ __device__ __forceinline__ void dct3_ortho(float (&y)[L], const float2* __restrict__ tw)
{
    using T = TwLayout<L>;
    constexpr int M = L / 2;
    const float2* comb = tw + T::COMB;
    const float2* pre = tw + T::PRE;
    cf z[M];
    {
        // V'[0] = y0/(a_0 L), V'[M] real; Z'[0] = (V'0 + V'M) + i (V'0 - V'M)
        const float v0 = y[0] * pre[0].x;
        const cf vmc = cmul(cf{y[M], -y[M]}, pre[M]);
        const float vm = vmc.x;
        z[0] = cf{v0 + vm, v0 - vm};
    }
#pragma unroll
    for (int k = 1; k <= M / 2; ++k) {
        const cf vk = cmul(cf{y[k], -y[L - k]}, pre[k]);
        const cf vmk = cmul(cf{y[M - k], -y[M + k]}, pre[M - k]);
        const cf e = cadd(vk, cconj(vmk));
        const cf o = cmulc(csub(vk, cconj(vmk)), comb[k]);
        // Z'[k] = e + i o;  Z'[M-k] = conj(e) + i conj(o)
        z[k] = cf{e.x - o.y, e.y + o.x};
        if (k != M - k) z[M - k] = cf{e.x + o.y, -e.y + o.x};
    }
    fft_reg<M, true>(z, tw + T::FFT);
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int n0 = 2 * m, n1 = 2 * m + 1;
        // x[2n] = v[n] (n < M), x[2(L-1-n)+1] = v[n] (n >= M)
        if (n0 < M) y[2 * n0] = z[m].x; else y[2 * (L - 1 - n0) + 1] = z[m].x;
        if (n1 < M) y[2 * n1] = z[m].y; else y[2 * (L - 1 - n1) + 1] = z[m].y;
    }
}

} // namespace dct
