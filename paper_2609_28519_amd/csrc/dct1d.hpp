// One-dimensional orthonormal DCT-II (Q_L x) and its transpose (Q_L^T y) in registers.
//
// Q_L is the matrix of the paper's Section 2.1 eq. 1.  Each routine transforms one
// length-L vector held in a thread's registers; the 2D transforms apply them along
// rows and columns (separable form, Section 1.2 and Section 3.1).  The paper's own
// factorisation (Shao-Johnson scaled split radix on 4-lane NEON bands) was designed
// for a CPU; here the length-N DCT-II is split by the classical even/odd recursion
//
//   u[n] = x[n] + x[N-1-n],  w[n] = x[n] - x[N-1-n]            (n < N/2)
//   X[2k]   = DCT-II_{N/2}(u)[k]                                  (recursion)
//   X[2k+1] = DCT-IV_{N/2}(w)[k]
//
// and every DCT-IV of length M is one complex FFT of length M/2 between two
// twiddle multiplications:
//   t[n] = (w[2n] + i w[M-1-2n]) exp(-i pi (4n+1)/(4M)),  T = DFT_{M/2}(t),
//   c[k] = T[k] exp(-i pi k/M),  Y[2k] = Re c[k],  Y[M-1-2k] = -Im c[k].
// The inverse (DCT-III, Q^T = Q^-1) is the transposed graph (Section 2.2, Prop. 2):
// even and odd coefficients go through DCT-III_{N/2} and DCT-IV_{N/2} (a symmetric
// matrix, computed by the same routine), then x[n] = u'[n] + w'[n],
// x[N-1-n] = u'[n] - w'[n].  The orthonormal factors a_k (eq. 1) are folded into
// the DCT-IV post-twiddles and the length-2 base case (Section 2.2: scales folded
// into the transforms; the round trip needs no separate correction).
//
// All twiddles come from the plan-owned table generated on the device in FP64
// (tables.hip), laid out as TwLayout<L>.  Indices into the table are compile-time
// constants after unrolling, so the loads are wave-uniform scalar loads.
#pragma once
#include <hip/hip_runtime.h>

namespace dct {

// Pointer to the twiddle table.  On the device it points into the constant address
// space, so wave-uniform reads of it compile to scalar loads.
#if defined(__HIP_DEVICE_COMPILE__)
typedef const __attribute__((address_space(4))) float2* twptr;
#else
typedef const float2* twptr;
#endif

struct cf {
    float x, y;
};

// Re-reads of the twiddle pointer: an optimisation barrier that stops the compiler from
// hoisting every twiddle load of a long transform to its start (which would pin them all
// in scalar registers and spill).  A no-op on the host.
__host__ __device__ __forceinline__ void tw_fence(twptr& tw)
{
#if defined(__HIP_DEVICE_COMPILE__)
    asm volatile("" : "+s"(tw));
#else
    (void)tw;
#endif
}

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

// Twiddle table of top length L (complex entries):
//   [0, F)            W_{L/4}^e, e < F = max(1, L/8)    (FFT twiddles of every level)
//   PRE(M) .. +M/2    exp(-i pi (4n+1)/(4M))            DCT-IV pre-twiddles, M = L/2..2
//   POST(M) .. +M/2   sqrt(2/L) exp(+i pi k/M)          DCT-IV post-twiddles (conjugated)
//   BASE              (sqrt(1/L), sqrt(1/L))            length-2 DCT-II scales
template <int L>
struct TwLayout {
    static_assert(L >= 8 && (L & (L - 1)) == 0, "power-of-two length >= 8");
    static constexpr int F = L / 8 > 1 ? L / 8 : 1;
    static constexpr int FFT_TOP = L / 4;
    static constexpr int pre(int M) { return F + L - 2 * M; }
    static constexpr int post(int M) { return F + L - 2 * M + M / 2; }
    static constexpr int BASE = F + L - 2;
    static constexpr int SIZE = F + L - 1;
};

__host__ __device__ constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }

// Multiply by the twiddle W_TOP^e (forward) or its conjugate (inverse).  e is a loop
// index of a fully unrolled loop, hence a constant after unrolling: trivial exponents
// (0, TOP/4, TOP/2, 3TOP/4) cost no multiplication, the others read W_TOP^e
// (e < TOP/2) from the table (a wave-uniform, scalar load).
template <int TOP, bool INV>
__host__ __device__ __forceinline__ cf twiddle_dyn(cf a, int e0, twptr tw)
{
    e0 %= TOP;
    const bool neg = e0 >= TOP / 2; // W^(e + TOP/2) = -W^e
    const int e = neg ? e0 - TOP / 2 : e0;
    cf r;
    if (e == 0) {
        r = a;
    } else if (4 * e == TOP) { // W^{TOP/4} = -i (forward), +i (inverse)
        r = INV ? cf{-a.y, a.x} : cf{a.y, -a.x};
    } else {
        r = INV ? cmulc(a, tw[e]) : cmul(a, tw[e]);
    }
    if (neg) r = cf{-r.x, -r.y};
    return r;
}

// DFT (INV = false, kernel exp(-2 pi i jk/M)) or unnormalised inverse DFT of the M
// values in[j*S], j < M, written to out[0..M) in natural order.  Recursive
// decimation in time, radix 4 (one radix-2 step when log2 M is odd); all indices
// are compile-time constants, so everything stays in registers.  Twiddles are
// W_TOP^e from the length-TOP table.
template <int M, int S, bool INV, int TOP>
__host__ __device__ __forceinline__ void fft_rec(const cf* in, cf* out, twptr tw)
{
    if constexpr (M == 1) {
        out[0] = in[0];
    } else if constexpr (M == 2) {
        out[0] = cadd(in[0], in[S]);
        out[1] = csub(in[0], in[S]);
    } else if constexpr ((ilog2(M) & 1) == 0) {
        constexpr int Q = M / 4, U = TOP / M;
        cf f0[Q], f1[Q], f2[Q], f3[Q];
        fft_rec<Q, 4 * S, INV, TOP>(in, f0, tw);
        fft_rec<Q, 4 * S, INV, TOP>(in + S, f1, tw);
        fft_rec<Q, 4 * S, INV, TOP>(in + 2 * S, f2, tw);
        fft_rec<Q, 4 * S, INV, TOP>(in + 3 * S, f3, tw);
#pragma unroll
        for (int k = 0; k < Q; ++k) {
            const cf a = f0[k];
            const cf b = twiddle_dyn<TOP, INV>(f1[k], k * U, tw);
            const cf c = twiddle_dyn<TOP, INV>(f2[k], 2 * k * U, tw);
            const cf d = twiddle_dyn<TOP, INV>(f3[k], 3 * k * U, tw);
            const cf t0 = cadd(a, c), t1 = csub(a, c), t2 = cadd(b, d), t3 = csub(b, d);
            // -i*t3 (forward) / +i*t3 (inverse)
            const cf it3 = INV ? cf{-t3.y, t3.x} : cf{t3.y, -t3.x};
            out[k] = cadd(t0, t2);
            out[k + 2 * Q] = csub(t0, t2);
            out[k + Q] = cadd(t1, it3);
            out[k + 3 * Q] = csub(t1, it3);
        }
    } else {
        constexpr int H = M / 2, U = TOP / M;
        cf e[H], o[H];
        fft_rec<H, 2 * S, INV, TOP>(in, e, tw);
        fft_rec<H, 2 * S, INV, TOP>(in + S, o, tw);
#pragma unroll
        for (int k = 0; k < H; ++k) {
            const cf b = twiddle_dyn<TOP, INV>(o[k], k * U, tw);
            out[k] = cadd(e[k], b);
            out[k + H] = csub(e[k], b);
        }
    }
}

// y <- sqrt(2/L) DCT-IV_M(w): one length-M/2 complex FFT between two twiddle products.
template <int L, int M>
__host__ __device__ __forceinline__ void dct4_scaled(const float* w, float* y, twptr tw_in)
{
    using T = TwLayout<L>;
    constexpr int H = M / 2;
    twptr tw = tw_in;
    cf t[H], c[H];
#pragma unroll
    for (int n = 0; n < H; ++n) t[n] = cmul(cf{w[2 * n], w[M - 1 - 2 * n]}, tw[T::pre(M) + n]);
    if (M >= 32) tw_fence(tw);
    fft_rec<H, 1, false, T::FFT_TOP>(t, c, tw);
    if (M >= 32) tw_fence(tw);
#pragma unroll
    for (int k = 0; k < H; ++k) {
        // q = conj(post twiddle):  Re(c p) = c.x q.x + c.y q.y,  -Im(c p) = c.x q.y - c.y q.x
        const float2 q = tw[T::post(M) + k];
        y[2 * k] = c[k].x * q.x + c[k].y * q.y;
        y[M - 1 - 2 * k] = c[k].x * q.y - c[k].y * q.x;
    }
}

// X = (scaled) DCT-II of the length-N vector x, as part of a top-level length-L transform.
template <int L, int N>
__host__ __device__ __forceinline__ void dct2_rec(const float* x, float* X, twptr tw)
{
    if constexpr (N == 2) {
        const float2 b = tw[TwLayout<L>::BASE];
        X[0] = (x[0] + x[1]) * b.x;
        X[1] = (x[0] - x[1]) * b.y;
    } else {
        constexpr int H = N / 2;
        float u[H], w[H], ue[H], wo[H];
#pragma unroll
        for (int n = 0; n < H; ++n) {
            u[n] = x[n] + x[N - 1 - n];
            w[n] = x[n] - x[N - 1 - n];
        }
        twptr tw2 = tw;
        if (N >= 64) tw_fence(tw2);
        dct2_rec<L, H>(u, ue, tw2);
        if (N >= 64) tw_fence(tw2);
        dct4_scaled<L, H>(w, wo, tw2);
#pragma unroll
        for (int k = 0; k < H; ++k) {
            X[2 * k] = ue[k];
            X[2 * k + 1] = wo[k];
        }
    }
}

// x = (scaled) DCT-III of the length-N coefficient vector Y (transpose of dct2_rec).
template <int L, int N>
__host__ __device__ __forceinline__ void dct3_rec(const float* Y, float* x, twptr tw)
{
    if constexpr (N == 2) {
        const float2 b = tw[TwLayout<L>::BASE];
        const float a = Y[0] * b.x, c = Y[1] * b.y;
        x[0] = a + c;
        x[1] = a - c;
    } else {
        constexpr int H = N / 2;
        float ye[H], yo[H], u[H], w[H];
#pragma unroll
        for (int k = 0; k < H; ++k) {
            ye[k] = Y[2 * k];
            yo[k] = Y[2 * k + 1];
        }
        twptr tw2 = tw;
        if (N >= 64) tw_fence(tw2);
        dct3_rec<L, H>(ye, u, tw2);
        if (N >= 64) tw_fence(tw2);
        dct4_scaled<L, H>(yo, w, tw2);
#pragma unroll
        for (int n = 0; n < H; ++n) {
            x[n] = u[n] + w[n];
            x[N - 1 - n] = u[n] - w[n];
        }
    }
}

// x <- Q_L x  (orthonormal DCT-II, eq. 1), L >= 8.
template <int L>
__host__ __device__ __forceinline__ void dct2_ortho(float (&x)[L], twptr tw)
{
    float y[L];
    dct2_rec<L, L>(x, y, tw);
#pragma unroll
    for (int i = 0; i < L; ++i) x[i] = y[i];
}

// y <- Q_L^T y  (orthonormal DCT-III, the inverse of dct2_ortho), L >= 8.
template <int L>
__host__ __device__ __forceinline__ void dct3_ortho(float (&y)[L], twptr tw)
{
    float x[L];
    dct3_rec<L, L>(y, x, tw);
#pragma unroll
    for (int i = 0; i < L; ++i) y[i] = x[i];
}

} // namespace dct
