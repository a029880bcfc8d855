// Arrays with an axis of 512 or 1024 (power-of-two shapes beyond the fused kernels, Section
// 7.1): a row pass and a column pass over HBM, each in place after the first, each line read
// whole before any of it is written.  A pass along an axis of length L in {512, 1024} shares
// every line among P = L / 256 wavefronts of one workgroup ("parts", long1d.hpp), one line
// per lane and 64 lines per workgroup; shorter axes take the one-thread-per-line kernels.
//
// Data between the parts goes through LDS, laid out [value][lane] (consecutive lanes on
// consecutive words, free of bank conflicts):
//   * L = 512: each part hands half of its values to the other (32 KB each) and writes half of
//     the line, forward, half of the interleaved coefficients (a row's first or second half of
//     float4 groups; a column's first or second 256 rows); inverse and round trip columns, the
//     pairs x[n] = u[n] + w[n], x[511-n] = u[n] - w[n] of its half of n.  Inverse and round trip
//     rows: part 1 hands its 256 values to part 0 (64 KB), which writes the whole row.
//   * L = 1024: parts 2 and 3 exchange their FFT halves (128 KB); natural-order outputs then
//     go through LDS in two rounds of 128 KB (a row's forward coefficients by halves of the
//     row; the inverse recombination by halves of n < 256, four output runs per round, one
//     run per part).  The inverse row pass also stages its input through LDS by half-rows.
// The round trip runs along rows and then along columns (Q_h^T Q_h X Q_w^T Q_w, the same
// product as inverse(forward(X))), fused per line: each part inverts its own coefficients in
// registers (for 1024, parts 2 and 3 first regroup their DCT-IV_512 coefficients through LDS).
#include <hip/hip_runtime.h>

#include "dct1d.hpp"
#include "internal.hpp"
#include "long1d.hpp"

namespace dct {
namespace {

constexpr int kLanes = 64;

// refresh(): an empty assembly statement that "rewrites" the base pointer, so that the
// compiler computes the addresses of each chunk of a line after the previous chunk instead of
// all of them up front (held live, they would overflow the registers).
struct GRow { // a contiguous line
    mutable const gfloat* p;
    static constexpr bool VEC = true;
    __device__ float at(int i) const { return p[i]; }
    __device__ float4 g4(int g) const { return *reinterpret_cast<const gfloat4*>(p + 4 * g); }
    __device__ void refresh() const { asm volatile("" : "+v"(p)); }
};
struct GCol { // a strided line (a column)
    mutable const gfloat* p;
    int es;
    static constexpr bool VEC = false;
    __device__ float at(int i) const { return p[(int64_t)i * es]; }
    __device__ float4 g4(int) const { return float4{}; }
    __device__ void refresh() const { asm volatile("" : "+v"(p)); }
};

// Output of a line: element n at dst[n * es] (es = 1 for rows, which use st4 on groups).
struct Out {
    mutable gfloat* dst;
    int es;
    bool ok; // the lane's line exists (lanes past the last line compute a copy and store nothing)
    __device__ void refresh() const { asm volatile("" : "+v"(dst)); }
    __device__ void st(int n, float v) const
    {
        if (ok) dst[(int64_t)n * es] = v;
    }
    __device__ void st4(int g, float a, float b, float c, float d) const
    {
        if (ok) *reinterpret_cast<gfloat4*>(dst + 4 * g) = make_float4(a, b, c, d);
    }
};

__device__ __forceinline__ float& ld(float* lds, int k, int lane) { return lds[k * kLanes + lane]; }

// ---- L = 512 -------------------------------------------------------------------------------

// The first instruction of every part differs between the parts, so the compiler cannot
// hoist the parts' identical loads (both L = 512 parts read the same elements) above the
// branch on the part, where all of them would be live at once.
template <int P>
__device__ __forceinline__ void part_entry()
{
    asm volatile("; long-line part %0" ::"n"(P) : "memory");
}

template <int DIR, bool COLS, int P, class A>
__device__ __forceinline__ void part512(const A& in, const Out& o, float* lds, int lane, twptr tw)
{
    part_entry<P>();
    float v[256], y[256];
    if constexpr (DIR == DCT2D_INVERSE) {
        lng::inv512_in<P>(in, v);
        if constexpr (P == 0) dct3_rec<512, 256>(v, y, tw); else dct4_scaled<512, 256>(v, y, tw);
    } else {
        lng::fwd512_in<P>(in, v);
        if constexpr (P == 0) dct2_rec<512, 256>(v, y, tw); else dct4_scaled<512, 256>(v, y, tw);
        if constexpr (DIR == DCT2D_ROUNDTRIP) {
            twptr tw2 = tw;
            tw_fence(tw2);
            if constexpr (P == 0) dct3_rec<512, 256>(y, v, tw2); else dct4_scaled<512, 256>(y, v, tw2);
#pragma unroll
            for (int n = 0; n < 256; ++n) y[n] = v[n];
        }
    }
    if constexpr (DIR == DCT2D_FORWARD && COLS) {
        // part 0 writes output rows 0 .. 255, part 1 rows 256 .. 511 (X[2k] = y0[k], X[2k+1] =
        // y1[k]), each taking the partner's half of the values through LDS, so only 128 values
        // per part are held across the barrier (which also waits until every part has read the
        // line: the pass is in place)
#pragma unroll
        for (int k = 0; k < 128; ++k) {
            if constexpr (P == 0) ld(lds, k, lane) = y[128 + k];
            else ld(lds, 128 + k, lane) = y[k];
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 128; ++i) {
            const int k = 128 * P + i;
            if constexpr (P == 0) {
                o.st(2 * k, y[k]);
                o.st(2 * k + 1, ld(lds, 128 + k, lane));
            } else {
                o.st(2 * k, ld(lds, k - 128, lane));
                o.st(2 * k + 1, y[k]);
            }
            if ((i & 15) == 15) o.refresh();
        }
        return;
    }
    if constexpr (DIR == DCT2D_FORWARD) {
        // rows: each part writes half of the row's float4 groups (part 0 groups 0..63, part 1
        // groups 64..127), each group X[4g .. 4g+3] = y0[2g], y1[2g], y0[2g+1], y1[2g+1]; each
        // part hands the partner the half of its values the partner's groups need, so only 128
        // values per part are held across the barrier
#pragma unroll
        for (int k = 0; k < 128; ++k) {
            if constexpr (P == 0) ld(lds, k, lane) = y[128 + k]; // y0[128 + k] for part 1
            else ld(lds, 128 + k, lane) = y[k];                  // y1[k] for part 0
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 64; ++i) {
            const int g = 64 * P + i;
            if constexpr (P == 0)
                o.st4(g, y[2 * g], ld(lds, 128 + 2 * g, lane), y[2 * g + 1], ld(lds, 128 + 2 * g + 1, lane));
            else
                o.st4(g, ld(lds, 2 * g - 128, lane), y[2 * g], ld(lds, 2 * g + 1 - 128, lane), y[2 * g + 1]);
        }
        return;
    }
    // inverse and round trip: x[n] = u[n] + w[n], x[511-n] = u[n] - w[n] with u from part 0, w from
    // part 1
    if constexpr (COLS) {
        // part P writes the pairs n in [128 P, 128 P + 128) and hands the partner the half of its
        // values the partner needs (part 0 u[128 .. 255], part 1 w[0 .. 127]), so only 128
        // values per part are held across the barrier
#pragma unroll
        for (int k = 0; k < 128; ++k) {
            if constexpr (P == 0) ld(lds, k, lane) = y[128 + k];
            else ld(lds, 128 + k, lane) = y[k];
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 128; ++i) {
            const int n = 128 * P + i;
            const float u = P == 0 ? y[n] : ld(lds, n - 128, lane);
            const float w = P == 0 ? ld(lds, 128 + n, lane) : y[n];
            o.st(n, u + w);
            o.st(511 - n, u - w);
            if ((i & 15) == 15) o.refresh();
        }
    } else {
        // rows: part 1 hands w to part 0, which writes the whole row in float4 groups (measured
        // faster here than splitting the row between the parts)
        if constexpr (P == 1) {
#pragma unroll
            for (int k = 0; k < 256; ++k) ld(lds, k, lane) = y[k];
        }
        __syncthreads();
        if constexpr (P == 0) {
#pragma unroll
            for (int g = 0; g < 64; ++g) {
                float s4[4], d4[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float w = ld(lds, 4 * g + i, lane);
                    s4[i] = y[4 * g + i] + w;
                    d4[i] = y[4 * g + i] - w;
                }
                o.st4(g, s4[0], s4[1], s4[2], s4[3]);
                o.st4(127 - g, d4[3], d4[2], d4[1], d4[0]);
            }
        }
    }
}

// ---- L = 1024 ------------------------------------------------------------------------------

// The DCT-IV_512 halves of parts 2 and 3 with their exchange (one barrier); LDS floats
// [0, 256) x 64 hold part 2's FFT half, [256, 512) x 64 part 3's.
template <int P>
__device__ __forceinline__ void dct4_512_exchange(const cf (&t)[128], float (&y)[256], float* lds, int lane, twptr tw)
{
    cf f[128];
    lng::dct4_512_fft<P>(t, f, tw);
    constexpr int own = P == 2 ? 0 : 256, other = P == 2 ? 256 : 0;
#pragma unroll
    for (int k = 0; k < 128; ++k) {
        ld(lds, own + 2 * k, lane) = f[k].x;
        ld(lds, own + 2 * k + 1, lane) = f[k].y;
    }
    __syncthreads();
    // the partner's half is read chunk by chunk as the post-twiddle consumes it, and the twiddle
    // pointer is fenced here, so neither the 256 partner values nor the post twiddles are loaded
    // early and held beside f (they would be spilled)
    twptr twp = tw;
    tw_fence(twp);
#pragma unroll
    for (int k = 0; k < 128; ++k) {
        const cf pf{ld(lds, other + 2 * k, lane), ld(lds, other + 2 * k + 1, lane)};
        lng::dct4_512_post_k<P>(f[k], pf, k, y, twp);
        if ((k & 15) == 15) lng::chunk_fence();
    }
}

// Inverse rows (L = 1024): the coefficients of a row pass through LDS in two halves of 512,
// element e of the half at ld(lds, e, lane).  Each part loads a quarter of every half as float4
// groups (groups 32 P .. 32 P + 31 of the half), so every byte of the row is read once; read
// directly, each part would load one float of every float4 group of the row (its quarter of the
// coefficients), and the four parts together fetched the row 2.5 times over.  Then each part
// gathers its own values: parts 0 and 1 X[4k + 2P]; parts 2 and 3 the pair (X[ma], X[mb]) of
// FFT point i, with ma = 8i + 4(P - 2) + 1 and mb = 1023 - 8i - 4(P - 2), which lie in
// different halves (ma in the first half for i < 64, mb for i >= 64), so the first half's value
// is held until the second.  Four workgroup barriers.
template <int P>
__device__ __forceinline__ void inv1024_rows_staged(const GRow& X, float* lds, int lane, float (&v)[256],
                                                    cf (&t)[128], twptr tw)
{
    float held[128];
    auto half = [&](auto hc) {
        constexpr int h = decltype(hc)::value;
        constexpr int C = 16;
        lng::pipelined<32 / C, lng::F4s<C>>(
            X,
            [&](auto cc, lng::F4s<C>& b) {
                constexpr int c = decltype(cc)::value;
#pragma unroll
                for (int i = 0; i < C; ++i) b.q[i] = X.g4(128 * h + 32 * P + c * C + i);
            },
            [&](auto cc, const lng::F4s<C>& b) {
                constexpr int c = decltype(cc)::value;
#pragma unroll
                for (int i = 0; i < C; ++i) {
                    const int g = 32 * P + c * C + i;
                    ld(lds, 4 * g, lane) = b.q[i].x;
                    ld(lds, 4 * g + 1, lane) = b.q[i].y;
                    ld(lds, 4 * g + 2, lane) = b.q[i].z;
                    ld(lds, 4 * g + 3, lane) = b.q[i].w;
                }
            });
        __syncthreads();
        if constexpr (P < 2) {
#pragma unroll
            for (int k = 128 * h; k < 128 * h + 128; ++k) v[k] = ld(lds, 4 * k + 2 * P - 512 * h, lane);
        } else {
#pragma unroll
            for (int i = 0; i < 128; ++i) {
                const int ma = 8 * i + 4 * (P - 2) + 1, mb = 1023 - 8 * i - 4 * (P - 2);
                const bool a_first = i < 64;
                if constexpr (h == 0) held[i] = ld(lds, a_first ? ma : mb, lane);
                else {
                    const float late = ld(lds, (a_first ? mb : ma) - 512, lane);
                    t[i] = lng::pre512<P>(a_first ? held[i] : late, a_first ? late : held[i], i, tw);
                }
            }
        }
        __syncthreads();
    };
    half(std::integral_constant<int, 0>{});
    half(std::integral_constant<int, 1>{});
}

template <int DIR, bool COLS, int P, class A>
__device__ __forceinline__ void part1024(const A& in, const Out& o, float* lds, int lane, twptr tw)
{
    part_entry<P>();
    float y[256];
    if constexpr (P < 2) {
        float v[256];
        if constexpr (DIR != DCT2D_INVERSE) {
            lng::fwd1024_in01<P>(in, v);
            if constexpr (P == 0) dct2_rec<1024, 256>(v, y, tw); else dct4_scaled<1024, 256>(v, y, tw);
        } else {
            if constexpr (COLS) lng::inv1024_in01<P>(in, v);
            else {
                cf unused[128];
                inv1024_rows_staged<P>(in, lds, lane, v, unused, tw);
            }
            if constexpr (P == 0) dct3_rec<1024, 256>(v, y, tw); else dct4_scaled<1024, 256>(v, y, tw);
        }
        __syncthreads(); // the exchange of parts 2 and 3
        if constexpr (DIR == DCT2D_ROUNDTRIP) {
            // the inverse of the part's own coefficients, in registers (uu for part 0, uw for
            // part 1), done here, while parts 2 and 3 regroup their coefficients and run their
            // second exchange, instead of before the first barrier
            twptr tw2 = tw;
            tw_fence(tw2);
            if constexpr (P == 0) dct3_rec<1024, 256>(y, v, tw2); else dct4_scaled<1024, 256>(y, v, tw2);
#pragma unroll
            for (int n = 0; n < 256; ++n) y[n] = v[n];
            // parts 2 and 3 redistribute their coefficients and run the inverse exchange
            __syncthreads();
            __syncthreads();
            __syncthreads();
            __syncthreads();
        }
    } else {
        cf t[128];
        if constexpr (DIR != DCT2D_INVERSE) lng::fwd1024_in23<P>(in, t, tw);
        else if constexpr (COLS) lng::inv1024_in23<P>(in, t, tw);
        else {
            float unused[256];
            inv1024_rows_staged<P>(in, lds, lane, unused, t, tw);
        }
        dct4_512_exchange<P>(t, y, lds, lane, tw);
        if constexpr (DIR == DCT2D_ROUNDTRIP) {
            // round trip: the DCT-IV_512 coefficients Y[j] (= X[2j + 1]) go to LDS slot j (part 2
            // holds Y[2k] and Y[511-2k] as y[2k], y[2k+1]; part 3 Y[256+2k] and Y[255-2k]), then
            // each part gathers the inverse's points, Y[j] and Y[511-j] with j = 4i + 2(P - 2),
            // and the same DCT-IV_512 runs again (its own inverse at this scaling)
            __syncthreads(); // the partner's FFT half has been read
#pragma unroll
            for (int k = 0; k < 128; ++k) {
                ld(lds, P == 2 ? 2 * k : 256 + 2 * k, lane) = y[2 * k];
                ld(lds, P == 2 ? 511 - 2 * k : 255 - 2 * k, lane) = y[2 * k + 1];
            }
            __syncthreads();
#pragma unroll
            for (int i = 0; i < 128; ++i) {
                const int j = 4 * i + 2 * (P - 2);
                t[i] = lng::pre512<P>(ld(lds, j, lane), ld(lds, 511 - j, lane), i, tw);
            }
            __syncthreads(); // read before the inverse exchange writes the area
            dct4_512_exchange<P>(t, y, lds, lane, tw);
        }
    }
    // every part has read the line (before the exchange barrier)
    if constexpr (DIR == DCT2D_FORWARD && COLS) {
#pragma unroll
        for (int s = 0; s < 256; ++s) {
            o.st(lng::out1024_index(P, s), y[s]);
            if ((s & 31) == 31) o.refresh();
        }
        return;
    }
    __syncthreads(); // the exchange area may be reused
    if constexpr (DIR == DCT2D_FORWARD) {
        // rows: coefficients by halves of the row, each part storing a quarter of the half
#pragma unroll
        for (int h = 0; h < 2; ++h) {
#pragma unroll
            for (int s = 0; s < 256; ++s) {
                const int m = lng::out1024_index(P, s);
                if ((m >> 9) == h) ld(lds, m - 512 * h, lane) = y[s];
            }
            __syncthreads();
#pragma unroll
            for (int g = 0; g < 32; ++g) {
                const int q = 128 * P + 4 * g; // position within the half
                o.st4((512 * h + q) / 4, ld(lds, q, lane), ld(lds, q + 1, lane), ld(lds, q + 2, lane),
                      ld(lds, q + 3, lane));
                if ((g & 7) == 7) lng::chunk_fence(o);
            }
            if (h == 0) __syncthreads();
        }
    } else {
        // x[n] = u + w[n], x[1023-n] = u - w[n], x[511-n] = u' + w[511-n], x[512+n] = u' - w[511-n]
        // with u = uu + uw, u' = uu - uw, over n in [128 r, 128 r + 128): LDS rows [0, 128) uu,
        // [128, 256) uw, [256, 384) w[n], [384, 512) w[511-n]
        // the two rounds are separate instantiations (r a compile-time constant): as a loop the
        // compiler would keep it rolled and index y at run time, which puts y in scratch
        auto round = [&](auto rc) {
            constexpr int r = decltype(rc)::value;
#pragma unroll
            for (int i = 0; i < 128; ++i) {
                const int n = 128 * r + i;
                if constexpr (P == 0) ld(lds, i, lane) = y[n];
                if constexpr (P == 1) ld(lds, 128 + i, lane) = y[n];
                if constexpr (P == 2) {
                    if ((n & 1) == 0) {
                        ld(lds, 256 + i, lane) = y[lng::w_pos_p2(n, false)];
                        ld(lds, 384 + i, lane) = y[lng::w_pos_p2(n, true)];
                    }
                }
                if constexpr (P == 3) {
                    if (n & 1) {
                        ld(lds, 256 + i, lane) = y[lng::w_pos_p3(n, false)];
                        ld(lds, 384 + i, lane) = y[lng::w_pos_p3(n, true)];
                    }
                }
            }
            __syncthreads();
            // part P writes run P: 0 x[n] (ascending from 128 r), 1 x[1023-n], 2 x[511-n], 3 x[512+n]
            auto val = [&](int i) {
                const float uu = ld(lds, i, lane), uw = ld(lds, 128 + i, lane);
                if constexpr (P == 0) return uu + uw + ld(lds, 256 + i, lane);
                else if constexpr (P == 1) return uu + uw - ld(lds, 256 + i, lane);
                else if constexpr (P == 2) return uu - uw + ld(lds, 384 + i, lane);
                else return uu - uw - ld(lds, 384 + i, lane);
            };
            // position of value i of the run
            auto pos = [&](int i) {
                const int n = 128 * r + i;
                return P == 0 ? n : P == 1 ? 1023 - n : P == 2 ? 511 - n : 512 + n;
            };
            if constexpr (COLS) {
#pragma unroll
                for (int i = 0; i < 128; ++i) {
                    o.st(pos(i), val(i));
                    if ((i & 31) == 31) o.refresh();
                }
            } else {
                // a run covers 128 consecutive positions: ascending for parts 0 and 3, descending
                // for parts 1 and 2
#pragma unroll
                for (int g = 0; g < 32; ++g) {
                    if constexpr (P == 0 || P == 3) {
                        o.st4(pos(4 * g) / 4, val(4 * g), val(4 * g + 1), val(4 * g + 2), val(4 * g + 3));
                    } else {
                        // positions pos(4g+3) .. pos(4g) ascending
                        o.st4(pos(4 * g + 3) / 4, val(4 * g + 3), val(4 * g + 2), val(4 * g + 1), val(4 * g));
                    }
                    // keeps the LDS reads of later groups from being issued early (each value
                    // reads three), which would hold the next round's values in scratch
                    if ((g & 7) == 7) lng::chunk_fence(o);
                }
            }
            if constexpr (r == 0) __syncthreads();
        };
        round(std::integral_constant<int, 0>{});
        round(std::integral_constant<int, 1>{});
    }
}

// The part of a 1024-point line that this wavefront runs (part is wave-uniform), for the
// round trip: a plain function, force-inlined; as a lambda the compiler kept this, the largest
// instantiation, out of line as a call.
template <int DIR, bool COLS, class A>
__device__ __forceinline__ void parts1024(const A& in, int part, const Out& o, float* lds, int lane, twptr tw)
{
    switch (part) {
    case 0: part1024<DIR, COLS, 0>(in, o, lds, lane, tw); break;
    case 1: part1024<DIR, COLS, 1>(in, o, lds, lane, tw); break;
    case 2: part1024<DIR, COLS, 2>(in, o, lds, lane, tw); break;
    default: part1024<DIR, COLS, 3>(in, o, lds, lane, tw); break;
    }
}

template <int L, int DIR, bool COLS>
__global__ void __launch_bounds__(kLanes * (L / 256), 1)
k_long(Addr a, int64_t total, int32_t lpa, int32_t es, int32_t ls, const float2* __restrict__ tw_in)
{
    constexpr int P = L / 256;
    __shared__ float lds[(L == 512 ? 256 : 512) * kLanes];
    const int part = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int64_t line0 = (int64_t)blockIdx.x * kLanes + lane;
    const bool ok = line0 < total;
    const int64_t line = ok ? line0 : total - 1;
    const int64_t b = line / lpa;
    const int64_t jl = line % lpa;
    const gfloat* src = a.src(b) + jl * ls;
    const Out o{a.dst(b) + jl * ls, es, ok};
    const twptr tw = (twptr)tw_in;
    if constexpr (L == 512) {
        if constexpr (COLS) {
            const GCol in{src, es};
            if (part == 0) part512<DIR, true, 0>(in, o, lds, lane, tw); else part512<DIR, true, 1>(in, o, lds, lane, tw);
        } else {
            const GRow in{src};
            if (part == 0) part512<DIR, false, 0>(in, o, lds, lane, tw); else part512<DIR, false, 1>(in, o, lds, lane, tw);
        }
    } else {
        if constexpr (DIR == DCT2D_ROUNDTRIP) {
            if constexpr (COLS) parts1024<DIR, COLS>(GCol{src, es}, part, o, lds, lane, tw);
            else parts1024<DIR, COLS>(GRow{src}, part, o, lds, lane, tw);
        } else {
            // forward and inverse keep the lambda form (inlined there), whose register
            // allocation measured better (forward rows: 108 B of scratch against 312)
            auto go = [&](const auto& in) {
                switch (part) {
                case 0: part1024<DIR, COLS, 0>(in, o, lds, lane, tw); break;
                case 1: part1024<DIR, COLS, 1>(in, o, lds, lane, tw); break;
                case 2: part1024<DIR, COLS, 2>(in, o, lds, lane, tw); break;
                default: part1024<DIR, COLS, 3>(in, o, lds, lane, tw); break;
                }
            };
            if constexpr (COLS) go(GCol{src, es}); else go(GRow{src});
        }
    }
}

// One pass along an axis of length L of `batch` arrays, lpa lines per array: element n of
// line j at j * ls + n * es from the array's start.
template <int L, int DIR>
int long_pass(const DeviceTables* t, const Addr& a, int64_t batch, int lpa, int es, int ls, bool cols, hipStream_t s)
{
    const int64_t total = batch * lpa;
    if (total == 0) return DCT2D_OK;
    const int64_t grid = (total + kLanes - 1) / kLanes;
    if (grid > 0x7fffffff) return DCT2D_ERR_ARG;
    const float2* tw = tw_for(t, L);
    if (cols) k_long<L, DIR, true><<<(unsigned)grid, kLanes * (L / 256), 0, s>>>(a, total, lpa, es, ls, tw);
    else k_long<L, DIR, false><<<(unsigned)grid, kLanes * (L / 256), 0, s>>>(a, total, lpa, es, ls, tw);
    return hipGetLastError() == hipSuccess ? DCT2D_OK : DCT2D_ERR_HIP;
}

// A pass of direction `dir` along the rows (cols = false) or the columns of rows x cols arrays.
int axis_pass(const DeviceTables* t, const Addr& a, int64_t batch, int rows, int cols, bool column_pass, int dir,
              hipStream_t s)
{
    const int len = column_pass ? rows : cols;
    const int lpa = column_pass ? cols : rows;
    const int es = column_pass ? cols : 1, ls = column_pass ? 1 : cols;
    if (len <= 256) return launch_short_line_pass(t, a, batch, len, lpa, column_pass, dir, s);
    if (len == 512) {
        switch (dir) {
        case DCT2D_FORWARD: return long_pass<512, DCT2D_FORWARD>(t, a, batch, lpa, es, ls, column_pass, s);
        case DCT2D_INVERSE: return long_pass<512, DCT2D_INVERSE>(t, a, batch, lpa, es, ls, column_pass, s);
        default: return long_pass<512, DCT2D_ROUNDTRIP>(t, a, batch, lpa, es, ls, column_pass, s);
        }
    }
    if (len == 1024) {
        if (dir == DCT2D_FORWARD) return long_pass<1024, DCT2D_FORWARD>(t, a, batch, lpa, es, ls, column_pass, s);
        if (dir == DCT2D_INVERSE) return long_pass<1024, DCT2D_INVERSE>(t, a, batch, lpa, es, ls, column_pass, s);
        return long_pass<1024, DCT2D_ROUNDTRIP>(t, a, batch, lpa, es, ls, column_pass, s);
    }
    return DCT2D_ERR_SIZE;
}

} // namespace

int launch_long(const DeviceTables* t, const Job& j)
{
    if (j.dir != DCT2D_FORWARD && j.dir != DCT2D_INVERSE && j.dir != DCT2D_ROUNDTRIP) return DCT2D_ERR_ARG;
    const Addr first = j.addr();
    const Addr in_place{j.out, j.out, j.out_stride, j.out_stride, j.out_idx, j.out_idx, j.out_slot, j.out_slot};
    // rows first (input -> output), then columns in place on the output
    int rc = axis_pass(t, first, j.batch, j.rows, j.cols, false, j.dir, j.stream);
    if (rc == DCT2D_OK) rc = axis_pass(t, in_place, j.batch, j.rows, j.cols, true, j.dir, j.stream);
    return rc;
}

} // namespace dct
