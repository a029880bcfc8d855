// Length-512 and length-1024 orthonormal DCT-II / DCT-III of one line shared by P = L / 256
// threads ("parts"), each holding at most 256 values, through the top levels of the even/odd
// recursion of dct1d.hpp (the twiddles of the top length L scale every level, as there):
//
//   L = 512:   part 0  X[2k]     = DCT-II_256(u)[k],  u[n] = x[n] + x[511-n]
//              part 1  X[2k+1]   = DCT-IV_256(w)[k],  w[n] = x[n] - x[511-n]
//   L = 1024:  u, w as above over 1024 (n < 512)
//              part 0  X[4k]     = DCT-II_256(uu)[k], uu[n] = u[n] + u[511-n]
//              part 1  X[4k+2]   = DCT-IV_256(uw)[k], uw[n] = u[n] - u[511-n]
//              parts 2, 3  X[2j+1] = DCT-IV_512(w)[j]: one 256-point complex FFT between the
//              two twiddle products of dct1d.hpp, split by one radix-2 step (decimation in
//              time): part 2 transforms t[2i], part 3 t[2i+1] (128 points each) and applies
//              W_256^k; after an exchange, part 2 forms T[k] = E[k] + W^k O[k] and part 3
//              T[k+128] = E[k] - W^k O[k] (k < 128), and each post-twiddles its half.  Part 2
//              then holds Y[2k], Y[511-2k] of the DCT-IV_512 (k < 128) as y[2k], y[2k+1];
//              part 3 holds Y[256+2k], Y[255-2k] the same way.
//
// The inverse (DCT-III_L = Q_L^T) is the transposed graph: the parts invert their blocks of
// coefficients (DCT-III_256 for the even block, DCT-IV for the odd ones, which is its own
// inverse in this scaling) and the results recombine as x[n] = u[n] + w[n],
// x[L-1-n] = u[n] - w[n] (and u[n] = uu[n] + uw[n], u[511-n] = uu[n] - uw[n] for 1024).
//
// The functions here are the per-part steps between which the caller exchanges data (a
// workgroup barrier on the GPU); the host replays them in the same order.  Lines are read
// through an accessor: at(n) (element n), for contiguous lines g4(g) (elements 4g..4g+3), and
// refresh() (re-reads its base pointer at a chunk boundary; nothing on the host).
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "dct1d.hpp"

namespace dct {
namespace lng {

__host__ __device__ __forceinline__ float e4(const float4& q, int i) { return i == 0 ? q.x : i == 1 ? q.y : i == 2 ? q.z : q.w; }

// A compiler-only barrier for memory operations, placed every few input chunks: without it
// the compiler issues all of a line's loads up front and keeps every loaded value live at
// once, which overflows the registers.  A no-op on the host.
__host__ __device__ __forceinline__ void chunk_fence()
{
#if defined(__HIP_DEVICE_COMPILE__)
    asm volatile("" ::: "memory");
#endif
}
// Pins a computed value at this point of the program (an empty assembly statement that reads
// and "rewrites" it): the loads it came from cannot be consumed after a later chunk fence, so
// they are not kept live across chunks.  Used by the L = 512 forward inputs only: elsewhere
// (the inverse inputs, the four-group L = 1024 inputs) they cost more than they save.  A no-op
// on the host.
__host__ __device__ __forceinline__ void pin(float& v)
{
#if defined(__HIP_DEVICE_COMPILE__)
    asm volatile("" : "+v"(v));
#else
    (void)v;
#endif
}
__host__ __device__ __forceinline__ void pin(cf& c)
{
    pin(c.x);
    pin(c.y);
}

// The same, also re-reading the accessor's base pointer (refresh()), so that the addresses of
// later chunks are not computed ahead and held live (arithmetic is not held back by a memory
// barrier).
template <class A>
__host__ __device__ __forceinline__ void chunk_fence(const A& a)
{
    a.refresh();
    chunk_fence();
}

// Reads a line in K chunks with the loads one chunk ahead of the arithmetic: load(c, buf)
// issues the loads of chunk c into buf, use(c, buf) forms that chunk's values and pins them.
// Chunk c + 1 is issued before chunk c is used, so the wait for chunk c leaves chunk c + 1 in
// flight; a pin orders memory operations around it, so without the look-ahead every chunk
// would be a full memory round trip, and without the pins the compiler would keep every
// loaded value of the line live at once.  The accessor's base pointer is re-read before each
// chunk (refresh), so the addresses of later chunks are not computed ahead and held live.
// The chunk sequence is unrolled at compile time (c is an integral_constant): a runtime loop
// over chunks would index the line's value array dynamically and put it in scratch memory.
template <int C0, int K, class Buf, class A, class Load, class Use>
__host__ __device__ __forceinline__ void pipelined_from(const A& x, Buf (&buf)[2], Load& load, Use& use)
{
    if constexpr (C0 < K) {
        if constexpr (C0 + 1 < K) {
            x.refresh();
            load(std::integral_constant<int, C0 + 1>{}, buf[(C0 + 1) & 1]);
        }
        use(std::integral_constant<int, C0>{}, buf[C0 & 1]);
        pipelined_from<C0 + 1, K>(x, buf, load, use);
    }
}

template <int K, class Buf, class A, class Load, class Use>
__host__ __device__ __forceinline__ void pipelined(const A& x, Load&& load, Use&& use)
{
    Buf buf[2];
    load(std::integral_constant<int, 0>{}, buf[0]);
    pipelined_from<0, K>(x, buf, load, use);
}

template <int N>
struct F4s {
    float4 q[N];
};
template <int N>
struct Fs {
    float f[N];
};

// ---- forward inputs ----------------------------------------------------------------------

// L = 512: part 0 u, part 1 w (256 values).
template <int P, class A>
__host__ __device__ __forceinline__ void fwd512_in(const A& x, float (&v)[256])
{
    if constexpr (A::VEC) {
        // chunk: 8 groups g, each x[4g .. 4g+3] and x[508-4g .. 511-4g] = r[3-i]
        constexpr int C = 8;
        pipelined<64 / C, F4s<2 * C>>(
            x,
            [&](auto cc, F4s<2 * C>& b) {
                constexpr int c = decltype(cc)::value;
#pragma unroll
                for (int i = 0; i < C; ++i) {
                    b.q[2 * i] = x.g4(c * C + i);
                    b.q[2 * i + 1] = x.g4(127 - c * C - i);
                }
            },
            [&](auto cc, const F4s<2 * C>& b) {
                constexpr int c = decltype(cc)::value;
#pragma unroll
                for (int i = 0; i < C; ++i) {
                    const int g = c * C + i;
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const float lo = e4(b.q[2 * i], j), hi = e4(b.q[2 * i + 1], 3 - j);
                        v[4 * g + j] = P == 0 ? lo + hi : lo - hi;
                        pin(v[4 * g + j]);
                    }
                }
            });
    } else {
        constexpr int C = 16; // values: x[n], x[511-n]
        pipelined<256 / C, Fs<2 * C>>(
            x,
            [&](auto cc, Fs<2 * C>& b) {
                constexpr int c = decltype(cc)::value;
#pragma unroll
                for (int i = 0; i < C; ++i) {
                    b.f[2 * i] = x.at(c * C + i);
                    b.f[2 * i + 1] = x.at(511 - c * C - i);
                }
            },
            [&](auto cc, const Fs<2 * C>& b) {
                constexpr int c = decltype(cc)::value;
#pragma unroll
                for (int i = 0; i < C; ++i) {
                    const int n = c * C + i;
                    v[n] = P == 0 ? b.f[2 * i] + b.f[2 * i + 1] : b.f[2 * i] - b.f[2 * i + 1];
                    pin(v[n]);
                }
            });
    }
}

// L = 1024, parts 0 and 1: uu / uw (256 values).
template <int P, class A>
__host__ __device__ __forceinline__ void fwd1024_in01(const A& x, float (&v)[256])
{
    if constexpr (A::VEC) {
        // chunk: 4 groups g, each x[4g+i], x[1023-4g-i], x[511-4g-i], x[512+4g+i]
        constexpr int C = 4;
        pipelined<64 / C, F4s<4 * C>>(
            x,
            [&](auto cc, F4s<4 * C>& b) {
                constexpr int c = decltype(cc)::value;
#pragma unroll
                for (int i = 0; i < C; ++i) {
                    const int g = c * C + i;
                    b.q[4 * i] = x.g4(g);
                    b.q[4 * i + 1] = x.g4(255 - g);
                    b.q[4 * i + 2] = x.g4(127 - g);
                    b.q[4 * i + 3] = x.g4(128 + g);
                }
            },
            [&](auto cc, const F4s<4 * C>& b) {
                constexpr int c = decltype(cc)::value;
#pragma unroll
                for (int i = 0; i < C; ++i) {
                    const int g = c * C + i;
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const float s = e4(b.q[4 * i], j) + e4(b.q[4 * i + 1], 3 - j),
                                    d = e4(b.q[4 * i + 2], 3 - j) + e4(b.q[4 * i + 3], j);
                        v[4 * g + j] = P == 0 ? s + d : s - d;
                        pin(v[4 * g + j]);
                    }
                }
            });
    } else {
        constexpr int C = 8; // values: x[n], x[1023-n], x[511-n], x[512+n]
        pipelined<256 / C, Fs<4 * C>>(
            x,
            [&](auto cc, Fs<4 * C>& b) {
                constexpr int c = decltype(cc)::value;
#pragma unroll
                for (int i = 0; i < C; ++i) {
                    const int n = c * C + i;
                    b.f[4 * i] = x.at(n);
                    b.f[4 * i + 1] = x.at(1023 - n);
                    b.f[4 * i + 2] = x.at(511 - n);
                    b.f[4 * i + 3] = x.at(512 + n);
                }
            },
            [&](auto cc, const Fs<4 * C>& b) {
                constexpr int c = decltype(cc)::value;
#pragma unroll
                for (int i = 0; i < C; ++i) {
                    const int n = c * C + i;
                    const float s = b.f[4 * i] + b.f[4 * i + 1], d = b.f[4 * i + 2] + b.f[4 * i + 3];
                    v[n] = P == 0 ? s + d : s - d;
                    pin(v[n]);
                }
            });
    }
}

// The DCT-IV_512 input pair of FFT point n' = 2i + (P - 2): (w[2n'], w[511-2n']) with
// w[n] = x[n] - x[1023-n], times the pre-twiddle.
template <int P>
__host__ __device__ __forceinline__ cf pre512(float wa, float wb, int i, twptr tw)
{
    return cmul(cf{wa, wb}, tw[TwLayout<1024>::pre(512) + 2 * i + (P - 2)]);
}

// L = 1024, parts 2 and 3: the part's 128 pre-twiddled FFT inputs t[i] = t_full[2i + P - 2].
template <int P, class A>
__host__ __device__ __forceinline__ void fwd1024_in23(const A& x, cf (&t)[128], twptr tw)
{
    constexpr int e = 2 * (P - 2); // 2n' = 4i + e
    if constexpr (A::VEC) {
        // points i and 127 - i use the same four groups i, 255 - i, 127 - i, 128 + i
        constexpr int C = 4;
        pipelined<64 / C, F4s<4 * C>>(
            x,
            [&](auto cc, F4s<4 * C>& b) {
                constexpr int c = decltype(cc)::value;
#pragma unroll
                for (int k = 0; k < C; ++k) {
                    const int i = c * C + k;
                    b.q[4 * k] = x.g4(i);
                    b.q[4 * k + 1] = x.g4(255 - i);
                    b.q[4 * k + 2] = x.g4(127 - i);
                    b.q[4 * k + 3] = x.g4(128 + i);
                }
            },
            [&](auto cc, const F4s<4 * C>& b) {
                constexpr int c = decltype(cc)::value;
#pragma unroll
                for (int k = 0; k < C; ++k) {
                    const int i = c * C + k;
                    const float4 &ga = b.q[4 * k], &gb = b.q[4 * k + 1], &gc = b.q[4 * k + 2], &gd = b.q[4 * k + 3];
                    // point i:       x[4i+e] - x[1023-4i-e],       x[511-4i-e] - x[512+4i+e]
                    t[i] = pre512<P>(e4(ga, e) - e4(gb, 3 - e), e4(gc, 3 - e) - e4(gd, e), i, tw);
                    // point 127 - i (2n' = 508 - 4i + e): x[2n'] in group 127 - i, x[1023-2n'] in
                    // group 128 + i, x[511-2n'] in group i, x[512+2n'] in group 255 - i
                    t[127 - i] = pre512<P>(e4(gc, e) - e4(gd, 3 - e), e4(ga, 3 - e) - e4(gb, e), 127 - i, tw);
                    pin(t[i]);
                    pin(t[127 - i]);
                }
            });
    } else {
        // steps j: points j and 127 - j, whose rows are the four quadruples {n, 1023-n, 511-n,
        // 512+n} with n = 4j + e and n = 4j + 3 - e, the rows that parts 0 and 1 read for their
        // values 4j .. 4j+3: two steps per chunk keep the four parts on the same rows (cache
        // lines shared through L2) chunk by chunk.
        constexpr int C = 2;
        pipelined<64 / C, Fs<8 * C>>(
            x,
            [&](auto cc, Fs<8 * C>& b) {
                constexpr int c = decltype(cc)::value;
#pragma unroll
                for (int k = 0; k < C; ++k) {
                    const int j = c * C + k;
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const int m = 4 * (h ? 127 - j : j) + e;
                        b.f[8 * k + 4 * h] = x.at(m);
                        b.f[8 * k + 4 * h + 1] = x.at(1023 - m);
                        b.f[8 * k + 4 * h + 2] = x.at(511 - m);
                        b.f[8 * k + 4 * h + 3] = x.at(512 + m);
                    }
                }
            },
            [&](auto cc, const Fs<8 * C>& b) {
                constexpr int c = decltype(cc)::value;
#pragma unroll
                for (int k = 0; k < C; ++k) {
                    const int j = c * C + k;
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const int i = h ? 127 - j : j;
                        const float* f = b.f + 8 * k + 4 * h;
                        t[i] = pre512<P>(f[0] - f[1], f[2] - f[3], i, tw);
                        pin(t[i]);
                    }
                }
            });
    }
}

// ---- inverse inputs (natural-order coefficients) ---------------------------------------------

// L = 512: part 0 X[2k], part 1 X[2k+1].
template <int P, class A>
__host__ __device__ __forceinline__ void inv512_in(const A& X, float (&v)[256])
{
    if constexpr (A::VEC) {
        constexpr int C = 16; // groups X[4g .. 4g+3]: X[4g+P] = v[2g], X[4g+2+P] = v[2g+1]
        pipelined<128 / C, F4s<C>>(
            X,
            [&](auto cc, F4s<C>& b) {
                constexpr int c = decltype(cc)::value;
#pragma unroll
                for (int i = 0; i < C; ++i) b.q[i] = X.g4(c * C + i);
            },
            [&](auto cc, const F4s<C>& b) {
                constexpr int c = decltype(cc)::value;
#pragma unroll
                for (int i = 0; i < C; ++i) {
                    const int g = c * C + i;
                    v[2 * g] = e4(b.q[i], P);
                    v[2 * g + 1] = e4(b.q[i], 2 + P);
                    pin(v[2 * g]);
                    pin(v[2 * g + 1]);
                }
            });
    } else {
        constexpr int C = 32;
        pipelined<256 / C, Fs<C>>(
            X,
            [&](auto cc, Fs<C>& b) {
                constexpr int c = decltype(cc)::value;
#pragma unroll
                for (int i = 0; i < C; ++i) b.f[i] = X.at(2 * (c * C + i) + P);
            },
            [&](auto cc, const Fs<C>& b) {
                constexpr int c = decltype(cc)::value;
#pragma unroll
                for (int i = 0; i < C; ++i) {
                    v[c * C + i] = b.f[i];
                    pin(v[c * C + i]);
                }
            });
    }
}

// L = 1024, parts 0 and 1: X[4k] / X[4k+2].
template <int P, class A>
__host__ __device__ __forceinline__ void inv1024_in01(const A& X, float (&v)[256])
{
    // chunk c: k in [16c, 16c + 16) and [240 - 16c, 256 - 16c), the float4 groups that parts 2
    // and 3 read in their chunk c, so that a row's cache lines serve all four parts close
    // together in time (otherwise the back half of the row is fetched again from HBM)
    constexpr int C = 16;
    auto kk = [](int c, int i) { return i < C ? c * C + i : 256 - (c + 1) * C + (i - C); };
    pipelined<256 / (2 * C), Fs<2 * C>>(
        X,
        [&](auto cc, Fs<2 * C>& b) {
                constexpr int c = decltype(cc)::value;
#pragma unroll
            for (int i = 0; i < 2 * C; ++i) {
                const int k = kk(c, i);
                if constexpr (A::VEC) b.f[i] = e4(X.g4(k), 2 * P);
                else b.f[i] = X.at(4 * k + 2 * P);
            }
        },
        [&](auto cc, const Fs<2 * C>& b) {
                constexpr int c = decltype(cc)::value;
#pragma unroll
            for (int i = 0; i < 2 * C; ++i) {
                v[kk(c, i)] = b.f[i];
                pin(v[kk(c, i)]);
            }
        });
}

// L = 1024, parts 2 and 3: DCT-IV_512 input points from the odd coefficients yo[j] = X[2j+1]:
// point n' = 2i + (P - 2) pairs yo[2n'] and yo[511-2n'].
template <int P, class A>
__host__ __device__ __forceinline__ void inv1024_in23(const A& X, cf (&t)[128], twptr tw)
{
    // chunk c: points i in [8c, 8c + 8), reading float4 groups [16c, 16c + 16) (yo[2n']) and
    // [240 - 16c, 256 - 16c) (yo[511-2n']), the groups of parts 0 and 1's chunk c
    constexpr int C = 8;
    pipelined<128 / C, Fs<2 * C>>(
        X,
        [&](auto cc, Fs<2 * C>& b) {
                constexpr int c = decltype(cc)::value;
#pragma unroll
            for (int k = 0; k < C; ++k) {
                const int j = 4 * (c * C + k) + 2 * (P - 2);       // 2n'
                const int ma = 2 * j + 1, mb = 2 * (511 - j) + 1; // X indices of yo[2n'], yo[511-2n']
                if constexpr (A::VEC) {
                    b.f[2 * k] = e4(X.g4(ma >> 2), ma & 3);
                    b.f[2 * k + 1] = e4(X.g4(mb >> 2), mb & 3);
                } else {
                    b.f[2 * k] = X.at(ma);
                    b.f[2 * k + 1] = X.at(mb);
                }
            }
        },
        [&](auto cc, const Fs<2 * C>& b) {
                constexpr int c = decltype(cc)::value;
#pragma unroll
            for (int k = 0; k < C; ++k) {
                const int i = c * C + k;
                t[i] = pre512<P>(b.f[2 * k], b.f[2 * k + 1], i, tw);
                pin(t[i]);
            }
        });
}

// ---- the DCT-IV_512 halves (parts 2, 3) -------------------------------------------------

// 128-point FFT of the part's points; part 3 also applies W_256^k.  f: 128 complex values.
template <int P>
__host__ __device__ __forceinline__ void dct4_512_fft(const cf (&t)[128], cf (&f)[128], twptr tw_in)
{
    twptr tw = tw_in;
    tw_fence(tw);
    fft_rec<128, 1, false, TwLayout<1024>::FFT_TOP>(t, f, tw);
    tw_fence(tw);
    if constexpr (P == 3) {
#pragma unroll
        for (int k = 0; k < 128; ++k) f[k] = twiddle_dyn<TwLayout<1024>::FFT_TOP, false>(f[k], k, tw);
    }
}

// After the exchange (own f, partner's pf): part 2 T[k] = f + pf, part 3 T[k+128] = pf - f;
// post-twiddle into y (part 2: y[2k] = Y[2k], y[2k+1] = Y[511-2k]; part 3: Y[256+2k],
// Y[255-2k]).
template <int P>
__host__ __device__ __forceinline__ void dct4_512_post_k(const cf& f, const cf& pf, int k, float (&y)[256], twptr tw)
{
    const cf c = P == 2 ? cadd(f, pf) : csub(pf, f);
    const float2 q = tw[TwLayout<1024>::post(512) + k + 128 * (P - 2)];
    y[2 * k] = c.x * q.x + c.y * q.y;
    y[2 * k + 1] = c.x * q.y - c.y * q.x;
}
template <int P>
__host__ __device__ __forceinline__ void dct4_512_post(const cf (&f)[128], const cf (&pf)[128], float (&y)[256],
                                                       twptr tw)
{
#pragma unroll
    for (int k = 0; k < 128; ++k) dct4_512_post_k<P>(f[k], pf[k], k, y, tw);
}

// X index of value s (< 256) of part P's forward output (L = 1024).
__host__ __device__ constexpr int out1024_index(int P, int s)
{
    return P == 0   ? 4 * s
           : P == 1 ? 4 * s + 2
           : P == 2 ? ((s & 1) ? 2 * (511 - (s & ~1)) + 1 : 2 * s + 1)          // Y[2k] / Y[511-2k], k = s/2
                    : ((s & 1) ? 2 * (255 - (s & ~1)) + 1 : 2 * (256 + s) + 1); // Y[256+2k] / Y[255-2k]
}

// The inverse recombination of L = 1024 needs, for each n < 256, w[n] and w[511-n] of the
// DCT-IV_512 result: part 2 holds them for even n (n = 2k) at y[n] and y[n+1]; part 3 for odd n
// (n = 255 - 2k) at y[256-n] (w[n]) and y[255-n] (w[511-n] = w[256+2k]).
__host__ __device__ constexpr int w_pos_p2(int n, bool mirror) { return mirror ? n + 1 : n; }
__host__ __device__ constexpr int w_pos_p3(int n, bool mirror) { return mirror ? 255 - n : 256 - n; }

} // namespace lng
} // namespace dct
