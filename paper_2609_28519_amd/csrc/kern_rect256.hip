// Fused kernels for rectangles with one axis of 256 and the other at most 128 (Section 7.1:
// h x w arrays, Q_h X Q_w^T): the rows of a wide h x 256 array or the columns of a tall
// 256 x w one are the "long lines".
//
// A tile of whole arrays (64 long lines, 128 for a short axis of 128) sits in LDS and
// crosses HBM once each way.  Every long-line transform is shared by four threads, one per
// wavefront role (split256.hpp: the top two levels of the even/odd recursion; 64 values per
// thread); the short-axis transforms take one thread per line (dct1d.hpp).
//
// A long line's forward outputs stay in the blocked layout of split256.hpp: the column pass
// of a wide array works on its positions in that layout (each holds one logical column) and
// the store puts the coefficients back in natural order; a tall array's coefficient row m
// sits in row blocked_pos(m), which the store (forward) and load (inverse) remap.  The
// double-buffered wide inverse runs its column pass first and writes every column to its
// blocked position, so that its row pass also reads blocked lines (whole 16-byte groups).
//
// Two schedules:
//   * k_rect256 (variants 0 and 2): one tile at a time per workgroup, rows of pitch
//     row length + 4 floats (lanes on consecutive rows start 4 banks apart).  Two
//     workgroups per CU at most (a tile is 64 KB), each waiting out its own loads.
//   * k_rect256_db (variant 3, short axis <= 64): one persistent workgroup per CU with two
//     tile buffers.  While a tile is transformed, the next one is copied from HBM straight
//     into the other buffer by LDS DMA loads (global_load_lds_dwordx4: each lane's 16 bytes
//     go to LDS at the instruction's base + 16 x lane), so the loads need no registers and
//     overlap the compute; the stores leave through registers as usual.  Rows are unpadded
//     so that one DMA instruction fills a whole 1 KB run of the tile; their 16-byte groups
//     are XOR-permuted by a row key instead (16-byte row accesses of 8 consecutive rows and
//     4-byte column accesses of 32 consecutive columns stay conflict-free).
#include <hip/hip_runtime.h>

#include "dct1d.hpp"
#include "fp32_common.hpp"
#include "internal.hpp"
#include "split256.hpp"

namespace dct {
namespace {

// ---- barriers ----------------------------------------------------------------------------
// The workgroup barrier of the one-tile schedule.
struct BarSync {
    __device__ static void sync() { __syncthreads(); }
};
// The double-buffered schedule's barrier inside a tile's compute: it orders the LDS accesses
// of the waves (each wave's LDS operations complete before it arrives) but, unlike the
// workgroup-scope fence of __syncthreads, does not wait for the LDS DMA copy of the next tile
// that is in flight into the other buffer.  The memory clobber keeps the compiler from moving
// LDS accesses across it.
struct BarLds {
    __device__ static void sync() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }
};

// ---- the long-line passes (shared by both schedules) ------------------------------------

// Forward of the thread's long line (natural order in, blocked layout out).  Three barriers.
template <int R, class B, class A>
__device__ __forceinline__ void long_fwd(const A& ln, twptr tw)
{
    float v[64], o[64];
    s4::fwd_in<R>(ln, v);
    B::sync(); // every role has read the line
    if constexpr (R < 2) {
        s4::fwd_tf01<R>(v, o, tw);
        s4::fwd_out<R>(ln, o);
        B::sync();
    } else {
        s4::fft_half<R>(v, o, tw);
        s4::put_half<R>(ln, o);
        B::sync(); // both halves published
        s4::combine_half<R>(ln, o, v, tw);
        s4::fwd_out<R>(ln, v);
    }
    B::sync();
}

// Inverse of the thread's long line (natural order out; in: blocked layout, or natural order
// when NATURAL), with the multipliers lam[m * LSTEP] applied to coefficient m first when
// MUL.  Five barriers; every role works in every phase of the recombination.
template <int R, bool NATURAL, bool MUL, int LSTEP, class B, class A>
__device__ __forceinline__ void long_inv(const A& ln, twptr tw, const gfloat* lam)
{
    float v[64], o[64];
    s4::inv_in<R, A, NATURAL, MUL, LSTEP>(ln, v, lam);
    B::sync(); // every role has read the line
    if constexpr (R < 2) {
        s4::inv_tf01<R>(v, o, tw);
        s4::inv_part<R>(ln, o); // [0, 128): not used by the exchange
        B::sync();
    } else {
        s4::fft_half<R>(v, o, tw);
        s4::put_half<R>(ln, o);
        B::sync(); // both halves published
        s4::combine_half<R>(ln, o, v, tw);
        s4::inv_part<R>(ln, v); // over the partner's half, which this role has read
    }
    B::sync(); // every partial published
    s4::inv_gather<R>(ln, o);
    B::sync(); // every partial read: the line may be overwritten
    s4::inv_emit<R>(ln, o);
    B::sync();
}

// One long pass for the thread's (role r, line) with the line accessor `ln`.  KIND: 0
// forward, 1 inverse from the blocked layout, 2 the same with the filter's multipliers
// lam[m * LSTEP], 3 inverse from natural order.
template <int KIND, int LSTEP, class B, class A>
__device__ __forceinline__ void long_role(int r, const A& ln, twptr tw, const gfloat* lam)
{
    constexpr bool NAT = KIND == 3, MUL = KIND == 2;
    if constexpr (KIND == 0) {
        switch (r) {
        case 0: long_fwd<0, B>(ln, tw); break;
        case 1: long_fwd<1, B>(ln, tw); break;
        case 2: long_fwd<2, B>(ln, tw); break;
        default: long_fwd<3, B>(ln, tw); break;
        }
    } else {
        switch (r) {
        case 0: long_inv<0, NAT, MUL, LSTEP, B>(ln, tw, lam); break;
        case 1: long_inv<1, NAT, MUL, LSTEP, B>(ln, tw, lam); break;
        case 2: long_inv<2, NAT, MUL, LSTEP, B>(ln, tw, lam); break;
        default: long_inv<3, NAT, MUL, LSTEP, B>(ln, tw, lam); break;
        }
    }
}

// ---- schedule 1: one tile at a time, padded rows ---------------------------------------

template <int H, int W>
struct R256 {
    static_assert((H == 256) != (W == 256), "one axis of 256");
    static constexpr bool WIDE = W == 256;
    static constexpr int S = WIDE ? H : W;                // short axis
    static_assert(S >= 8 && S <= 128, "short axis 8..128");
    // arrays per tile: 64 long lines (128 for a short axis of 128), so that a wavefront's
    // 64 lanes share one role
    static constexpr int BPW = S >= 64 ? 1 : 64 / S;
    static constexpr int LPT = S * BPW;                    // long lines per tile
    static constexpr int NT = 4 * LPT;                     // one thread per (long line, role)
    static constexpr int P = W + 4;                        // LDS row pitch
    // LDS array pitch: tall tiles hold several arrays side by side in a wavefront's column
    // accesses (lanes = (array, column)); a pitch of S mod 32 banks keeps them apart
    static constexpr int AP = H * P + (!WIDE && S < 32 ? S : 0);
    static constexpr int LDS_FLOATS = BPW * AP;
    static constexpr int CPA = H * W / 4;                  // 16-byte chunks per array
    static constexpr int CPT = BPW * CPA / NT;             // chunks per thread
    static constexpr int SL = BPW * 256;                   // short lines per tile
    static constexpr int STEP = WIDE ? 1 : P;              // element stride along a long line
    static_assert((BPW * CPA) % NT == 0, "whole chunk rounds");
    static_assert(LPT % 64 == 0, "roles uniform per wavefront");
};

template <int H, int W, int KIND>
__device__ __forceinline__ void long_pass(float* lds, int t, twptr tw, const Addr& a, int64_t b0, int64_t batch)
{
    using C = R256<H, W>;
    const int r = t / C::LPT, li = t % C::LPT; // role uniform per wavefront
    const int bb = li / C::S, s = li % C::S;
    const s4::Strided<C::STEP> ln{C::WIDE ? lds + bb * C::AP + s * C::P : lds + bb * C::AP + s};
    const gfloat* lam = nullptr;
    if constexpr (KIND == 2) lam = a.lam_for(b0 + bb < batch ? b0 + bb : b0) + s; // column s, rows m * W
    long_role<KIND, W, BarSync>(r, ln, tw, lam);
}

// The short-axis pass: SL lines of length S per tile (wide arrays: the blocked positions of the
// rows, position c holding logical column blocked_logical(c); tall arrays: natural rows).
template <int H, int W, int PASS>
__device__ __forceinline__ void short_pass(float* lds, int t, twptr tw, const Addr& a, int64_t b0, int64_t batch)
{
    using C = R256<H, W>;
    constexpr int S = C::S;
#pragma unroll 1
    for (int ln = t; ln < C::SL; ln += C::NT) {
        const int bb = ln / 256, c = ln % 256;
        float v[S];
        if constexpr (C::WIDE) {
            float* col = lds + bb * C::AP + c;
#pragma unroll
            for (int r = 0; r < S; ++r) v[r] = col[r * C::P];
            if constexpr (PASS == DIR_FILTER)
                filter1d<S>(v, a.lam_for(b0 + bb < batch ? b0 + bb : b0) + s4::blocked_logical(c), 256, tw);
            else
                apply1d<S, PASS>(v, tw);
#pragma unroll
            for (int r = 0; r < S; ++r) col[r * C::P] = v[r];
        } else {
            float* row = lds + bb * C::AP + c * C::P;
#pragma unroll
            for (int j = 0; j < S / 4; ++j) {
                const float4 q = *reinterpret_cast<const float4*>(row + 4 * j);
                v[4 * j] = q.x; v[4 * j + 1] = q.y; v[4 * j + 2] = q.z; v[4 * j + 3] = q.w;
            }
            apply1d<S, PASS>(v, tw);
#pragma unroll
            for (int j = 0; j < S / 4; ++j)
                *reinterpret_cast<float4*>(row + 4 * j) = make_float4(v[4 * j], v[4 * j + 1], v[4 * j + 2], v[4 * j + 3]);
        }
    }
}

template <int H, int W, int DIR>
__global__ void __launch_bounds__((R256<H, W>::NT))
k_rect256(Addr a, int64_t batch, const float2* __restrict__ tw256_in, const float2* __restrict__ tws_in)
{
    using C = R256<H, W>;
    __shared__ float4 lds4[(C::LDS_FLOATS + 3) / 4];
    float* lds = reinterpret_cast<float*>(lds4);
    const int t = threadIdx.x;
    const int64_t ntiles = (batch + C::BPW - 1) / C::BPW;
    // tall arrays: coefficient rows in the blocked order (inverse in, forward out)
    constexpr bool BLOCKED_IN = DIR == DCT2D_INVERSE && !C::WIDE, BLOCKED_OUT = DIR == DCT2D_FORWARD;
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t b0 = tile * C::BPW;
        // load: chunk f = t + NT i of the tile, array f / CPA; arrays past the batch read a
        // copy of array b0 and are never stored
#pragma unroll
        for (int i = 0; i < C::CPT; ++i) {
            const int f = t + C::NT * i;
            const int bb = f / C::CPA, q = f % C::CPA;
            const int r = q / (W / 4), c4 = q % (W / 4);
            const int64_t b = b0 + bb < batch ? b0 + bb : b0;
            const float4 v = *reinterpret_cast<const gfloat4*>(a.src(b) + 4 * q);
            const int pr = BLOCKED_IN ? s4::blocked_pos(r) : r;
            *reinterpret_cast<float4*>(lds + bb * C::AP + pr * C::P + 4 * c4) = v;
        }
        __syncthreads();
        const twptr tw256 = per_iteration(tw256_in);
        if constexpr (C::WIDE) {
            if constexpr (DIR == DCT2D_INVERSE) {
                long_pass<H, W, 3>(lds, t, tw256, a, b0, batch); // rows from natural order
                short_pass<H, W, DCT2D_INVERSE>(lds, t, per_iteration(tws_in), a, b0, batch);
            } else {
                long_pass<H, W, 0>(lds, t, tw256, a, b0, batch);
                short_pass<H, W, DIR>(lds, t, per_iteration(tws_in), a, b0, batch);
                __syncthreads();
                if constexpr (DIR != DCT2D_FORWARD) long_pass<H, W, 1>(lds, t, per_iteration(tw256_in), a, b0, batch);
            }
        } else {
            if constexpr (DIR == DCT2D_INVERSE) {
                long_pass<H, W, 1>(lds, t, tw256, a, b0, batch);
                short_pass<H, W, DCT2D_INVERSE>(lds, t, per_iteration(tws_in), a, b0, batch);
            } else {
                short_pass<H, W, DCT2D_FORWARD>(lds, t, per_iteration(tws_in), a, b0, batch);
                __syncthreads();
                long_pass<H, W, 0>(lds, t, tw256, a, b0, batch);
                if constexpr (DIR != DCT2D_FORWARD) {
                    long_pass<H, W, DIR == DIR_FILTER ? 2 : 1>(lds, t, per_iteration(tw256_in), a, b0, batch);
                    short_pass<H, W, DCT2D_INVERSE>(lds, t, per_iteration(tws_in), a, b0, batch);
                }
            }
        }
        __syncthreads();
        // store (forward: the long lines' coefficients back from the blocked layout)
#pragma unroll
        for (int i = 0; i < C::CPT; ++i) {
            const int f = t + C::NT * i;
            const int bb = f / C::CPA, q = f % C::CPA;
            const int r = q / (W / 4), c4 = q % (W / 4);
            const float* arr = lds + bb * C::AP;
            float4 v;
            if (BLOCKED_OUT && C::WIDE) {
                const float* s = arr + r * C::P;
                v = make_float4(s[s4::blocked_pos(4 * c4)], s[s4::blocked_pos(4 * c4 + 1)],
                                s[s4::blocked_pos(4 * c4 + 2)], s[s4::blocked_pos(4 * c4 + 3)]);
            } else {
                const int pr = BLOCKED_OUT ? s4::blocked_pos(r) : r;
                v = *reinterpret_cast<const float4*>(arr + pr * C::P + 4 * c4);
            }
            if (b0 + bb < batch) *reinterpret_cast<gfloat4*>(a.dst(b0 + bb) + 4 * q) = v;
        }
        __syncthreads();
    }
}

// ---- schedule 2: persistent, double-buffered, LDS DMA loads ---------------------------

// Strided batches only (array b at in + b * in_stride, out + b * out_stride): the offsets are
// plain arithmetic, so no memory read sits between the copies of a tile (a read would wait
// for every copy issued before it).  Ragged batches take k_rect256.
struct FlatAddr {
    const float* in;
    float* out;
    int64_t in_stride, out_stride;
    const float* lam;
    int64_t lam_stride;
    __device__ __forceinline__ const gfloat* lam_for(int64_t b) const { return (const gfloat*)lam + b * lam_stride; }
    __device__ __forceinline__ const gfloat* src_base() const { return (const gfloat*)in; }
    __device__ __forceinline__ int64_t src_off(int64_t b) const { return b * in_stride; }
    __device__ __forceinline__ gfloat* dst_base() const { return (gfloat*)out; }
    __device__ __forceinline__ int64_t dst_off(int64_t b) const { return b * out_stride; }
};

template <int H, int W>
struct RDB {
    static_assert((H == 256) != (W == 256), "one axis of 256");
    static constexpr bool WIDE = W == 256;
    static constexpr int S = WIDE ? H : W;
    static_assert(S >= 8 && S <= 64, "short axis 8..64");
    static constexpr int BPW = 64 / S;                     // arrays per tile (64 long lines)
    static constexpr int NT = 256;                         // 4 roles x 64 lines
    static constexpr int G = W / 4;                        // 16-byte groups per row
    static constexpr int RPL = G >= 8 ? 1 : 8 / G;         // rows per 32 banks
    static constexpr int KG = G >= 8 ? 8 : G;              // key range
    // LDS array pitch (floats): tall tiles shift consecutive arrays by S banks (lanes of a
    // column access span several arrays when S < 32)
    static constexpr int AP = H * W + (!WIDE && S < 32 ? S : 0);
    static constexpr int TILE = BPW * AP;                  // floats per buffer
    static constexpr int CPT = 64 * 256 / 4 / NT;          // 16-byte chunks per thread (16)
    static constexpr int DMA_PER_WAVE = 64 / (NT / 64);    // 1 KB DMA runs per wavefront (16)
    static_assert(CPT == 16, "the loop's wait counts 16 stores per thread");
    __host__ __device__ static constexpr int key(int r) { return (r / RPL) & (KG - 1); }
    // float offset of group j of row r of array bb (group of the row after the XOR key)
    __host__ __device__ static int at4(int bb, int r, int j) { return bb * AP + r * W + 4 * (j ^ key(r)); }
};

// Column s of a tall array in the swizzled layout (element i = row i).
template <int S>
struct SwzCol {
    float* base; // array base
    int s;
    static constexpr bool VEC = false;
    __device__ float& at(int i) const
    {
        using C = RDB<256, S>;
        return base[i * S + 4 * ((s >> 2) ^ C::key(i)) + (s & 3)];
    }
    __device__ float4 g4(int) const { return float4{}; }
    __device__ void s4(int, float4) const {}
};

// One LDS DMA copy (global_load_lds_dwordx4): lane l's 16 bytes at `g` go to LDS at
// lds_base + 16 l (lds_base wave-uniform).  Written out rather than through the compiler's
// builtin: the compiler cannot tell which LDS object the builtin writes, so it would make the
// first LDS read after it (of the other buffer) wait for the copy, removing the overlap.  The
// instruction has no register results (nothing in flight can overwrite a register); its
// address registers are read at issue.  One wait state separates the M0 write from the copy
// that reads it.  Completion is awaited explicitly (vmcnt and a barrier) before the tile is
// read; the compiler's own counted waits for its loads stay valid because the counter
// completes in issue order (a copy issued before one of its loads only adds to the wait).
__device__ __forceinline__ void lds_copy16(const gfloat* g, float* lds_base)
{
    const uint32_t m0 =
        __builtin_amdgcn_readfirstlane((uint32_t)(uintptr_t)(__attribute__((address_space(3))) float*)lds_base);
    asm volatile("s_mov_b32 m0, %1\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, off" ::"v"((uint64_t)g), "s"(m0)
                 : "memory", "m0");
}

// Issues the LDS DMA copy of tile `tile` into buffer `buf`: the tile's 64 KB as 64 runs of
// 1 KB (16 per wavefront).  Wide: run = one row; tall: run = 256 / S rows of one array.  Lane l
// of a run fills LDS group l of the run, which holds logical group l ^ key of its row.  BLOCKED:
// tall LDS row r receives natural row blocked_logical(r).  Arrays past the batch read a copy of
// the tile's first array (never stored).
template <int H, int W, bool BLOCKED>
__device__ __forceinline__ void dma_tile(float* buf, const FlatAddr& a, int64_t tile, int64_t batch, int wid, int lane)
{
    using C = RDB<H, W>;
    const int64_t b0 = tile * C::BPW;
    const gfloat* src = a.src_base();
    // the wavefront's 16 runs lie in NB arrays (S runs per array): their offsets are resolved
    // before the first copy is issued (an offset-list read between copies would make every
    // copy wait for the ones before it)
    constexpr int NB = C::S < C::DMA_PER_WAVE ? C::DMA_PER_WAVE / C::S : 1;
    const int bb0 = wid * C::DMA_PER_WAVE / C::S;
    int64_t off[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const int64_t b = b0 + bb0 + i < batch ? b0 + bb0 + i : b0;
        off[i] = a.src_off(b);
    }
#pragma unroll
    for (int k = 0; k < C::DMA_PER_WAVE; ++k) {
        const int run = wid * C::DMA_PER_WAVE + k; // 0 .. 63, wave-uniform
        const int i = NB > 1 ? k / C::S : 0;       // array of the run among the wavefront's
        int r, j;
        float* dst;
        if constexpr (C::WIDE) {
            r = run % C::S;
            j = lane ^ C::key(run); // key by tile row
            dst = buf + run * 256;
        } else {
            const int r0 = (run % C::S) * (256 / C::S);
            r = r0 + lane / C::G;
            j = (lane % C::G) ^ C::key(r);
            dst = buf + (bb0 + i) * C::AP + r0 * C::S;
        }
        const int gr = BLOCKED ? s4::blocked_logical(r) : r;
        const gfloat* g = src + off[i] + (int64_t)gr * W + 4 * j;
        lds_copy16(g, dst);
    }
}

template <int H, int W, int KIND>
__device__ __forceinline__ void db_long(float* buf, int t, twptr tw, const FlatAddr& a, int64_t b0, int64_t batch)
{
    using C = RDB<H, W>;
    const int r = t >> 6, li = t & 63; // role = wavefront
    const gfloat* lam = nullptr;
    if constexpr (C::WIDE) {
        // line = tile row li; its groups carry key(li)
        const s4::Swizzled ln{buf + li * 256, C::key(li)};
        long_role<KIND, W, BarLds>(r, ln, tw, lam);
    } else {
        const int bb = li / C::S, s = li % C::S;
        if constexpr (KIND == 2) lam = a.lam_for(b0 + bb < batch ? b0 + bb : b0) + s;
        const SwzCol<C::S> ln{buf + bb * C::AP, s};
        long_role<KIND, W, BarLds>(r, ln, tw, lam);
    }
}

template <int H, int W, int PASS>
__device__ __forceinline__ void db_short(float* buf, int t, twptr tw, const FlatAddr& a, int64_t b0, int64_t batch)
{
    using C = RDB<H, W>;
    constexpr int S = C::S;
#pragma unroll 1
    for (int ln = t; ln < C::BPW * 256; ln += C::NT) {
        const int bb = ln / 256, c = ln % 256;
        float v[S];
        if constexpr (C::WIDE) {
            // column c (a position of the blocked layout) over rows R = bb S + r of the tile
#pragma unroll
            for (int r = 0; r < S; ++r) {
                const int R = bb * S + r;
                v[r] = buf[R * 256 + 4 * ((c >> 2) ^ C::key(R)) + (c & 3)];
            }
            if constexpr (PASS == DIR_FILTER)
                filter1d<S>(v, a.lam_for(b0 + bb < batch ? b0 + bb : b0) + s4::blocked_logical(c), 256, tw);
            else
                apply1d<S, PASS>(v, tw);
#pragma unroll
            for (int r = 0; r < S; ++r) {
                const int R = bb * S + r;
                buf[R * 256 + 4 * ((c >> 2) ^ C::key(R)) + (c & 3)] = v[r];
            }
        } else {
            // row c of array bb
#pragma unroll
            for (int j = 0; j < S / 4; ++j) {
                const float4 q = *reinterpret_cast<const float4*>(buf + C::at4(bb, c, j));
                v[4 * j] = q.x; v[4 * j + 1] = q.y; v[4 * j + 2] = q.z; v[4 * j + 3] = q.w;
            }
            apply1d<S, PASS>(v, tw);
#pragma unroll
            for (int j = 0; j < S / 4; ++j)
                *reinterpret_cast<float4*>(buf + C::at4(bb, c, j)) = make_float4(v[4 * j], v[4 * j + 1], v[4 * j + 2], v[4 * j + 3]);
        }
    }
}

// Wide inverse, column pass first: every column of every array of the tile is inverted and
// written back at its position in the blocked layout, so that the row pass then reads its
// inputs as whole 16-byte groups.  Thread (wavefront w, lane l) takes column c = 4 k + e with
// k = (l & 31) + 32 (l >> 5) and e = ((l & 31) / 8 + w) & 3 in each array: within each half
// wavefront the columns are distinct modulo 32 and so are their blocked positions (which are
// congruent to k), so both the reads and the permuted writes are free of bank conflicts.  All
// columns are read before any is written (the permutation is in place).
template <int H, int W>
__device__ __forceinline__ void db_short_inv_to_blocked(float* buf, int t, twptr tw)
{
    using C = RDB<H, W>;
    static_assert(C::WIDE, "wide tiles");
    constexpr int S = C::S;
    const int w = t >> 6, l = t & 63, kl = l & 31;
    const int k = kl + 32 * (l >> 5);
    const int c = 4 * k + (((kl >> 3) + w) & 3);
    const int p = s4::blocked_pos(c);
    float v[C::BPW][S];
#pragma unroll
    for (int bb = 0; bb < C::BPW; ++bb) {
#pragma unroll
        for (int r = 0; r < S; ++r) {
            const int R = bb * S + r;
            v[bb][r] = buf[R * 256 + 4 * ((c >> 2) ^ C::key(R)) + (c & 3)];
        }
        apply1d<S, DCT2D_INVERSE>(v[bb], tw);
    }
    BarLds::sync();
#pragma unroll
    for (int bb = 0; bb < C::BPW; ++bb) {
#pragma unroll
        for (int r = 0; r < S; ++r) {
            const int R = bb * S + r;
            buf[R * 256 + 4 * ((p >> 2) ^ C::key(R)) + (p & 3)] = v[bb][r];
        }
    }
    BarLds::sync();
}

// Transform and store of the tile in `buf` (its DMA has completed and is visible).
template <int H, int W, int DIR>
__device__ __forceinline__ void db_compute_store(float* buf, int t, const FlatAddr& a, int64_t tile, int64_t batch,
                                                 const float2* tw256_in, const float2* tws_in)
{
    using C = RDB<H, W>;
    const int64_t b0 = tile * C::BPW;
    const twptr tw256 = per_iteration(tw256_in);
    if constexpr (C::WIDE) {
        if constexpr (DIR == DCT2D_INVERSE) {
            db_short_inv_to_blocked<H, W>(buf, t, per_iteration(tws_in));
            db_long<H, W, 1>(buf, t, tw256, a, b0, batch);
        } else {
            db_long<H, W, 0>(buf, t, tw256, a, b0, batch);
            db_short<H, W, DIR>(buf, t, per_iteration(tws_in), a, b0, batch);
            BarLds::sync();
            if constexpr (DIR != DCT2D_FORWARD) db_long<H, W, 1>(buf, t, per_iteration(tw256_in), a, b0, batch);
        }
    } else {
        if constexpr (DIR == DCT2D_INVERSE) {
            db_long<H, W, 1>(buf, t, tw256, a, b0, batch);
            db_short<H, W, DCT2D_INVERSE>(buf, t, per_iteration(tws_in), a, b0, batch);
        } else {
            db_short<H, W, DCT2D_FORWARD>(buf, t, per_iteration(tws_in), a, b0, batch);
            BarLds::sync();
            db_long<H, W, 0>(buf, t, tw256, a, b0, batch);
            if constexpr (DIR != DCT2D_FORWARD) {
                db_long<H, W, DIR == DIR_FILTER ? 2 : 1>(buf, t, per_iteration(tw256_in), a, b0, batch);
                db_short<H, W, DCT2D_INVERSE>(buf, t, per_iteration(tws_in), a, b0, batch);
            }
        }
    }
    BarLds::sync();
    // store: chunk f = 256 i + t (consecutive lanes on consecutive logical groups of a row);
    // an array holds 64 S chunks, a multiple of 256, so chunk round i lies in array
    // 256 i / (64 S) whatever t is; the array offsets are resolved before the first store
    constexpr bool BLOCKED_OUT = DIR == DCT2D_FORWARD;
    gfloat* dbase = a.dst_base();
    int64_t doff[C::BPW];
    bool dok[C::BPW];
#pragma unroll
    for (int bb = 0; bb < C::BPW; ++bb) {
        dok[bb] = b0 + bb < batch;
        doff[bb] = a.dst_off(dok[bb] ? b0 + bb : b0);
    }
#pragma unroll
    for (int i = 0; i < C::CPT; ++i) {
        const int f = t + C::NT * i;
        constexpr int CA = 64 * C::S; // chunks per array
        const int bb = (C::NT * i) / CA;
        int r, j;
        if constexpr (C::WIDE) {
            const int R = f / 64;
            r = R % C::S;
            j = f % 64;
        } else {
            const int q = f % CA;
            r = q / C::G;
            j = q % C::G;
        }
        float4 v;
        if constexpr (C::WIDE && BLOCKED_OUT) {
            const int R = bb * C::S + r;
            const float* row = buf + R * 256;
            auto e = [&](int m) { const int p = s4::blocked_pos(m); return row[4 * ((p >> 2) ^ C::key(R)) + (p & 3)]; };
            v = make_float4(e(4 * j), e(4 * j + 1), e(4 * j + 2), e(4 * j + 3));
        } else if constexpr (C::WIDE) {
            const int R = bb * C::S + r;
            v = *reinterpret_cast<const float4*>(buf + R * 256 + 4 * (j ^ C::key(R)));
        } else {
            const int pr = BLOCKED_OUT ? s4::blocked_pos(r) : r;
            v = *reinterpret_cast<const float4*>(buf + C::at4(bb, pr, j));
        }
        if (dok[bb]) *reinterpret_cast<gfloat4*>(dbase + doff[bb] + (int64_t)r * W + 4 * j) = v;
    }
}

// One stage of the persistent loop: the copy of tile `next` (if any) into `nxt`, then the
// transform and store of tile `tile` from `cur`.  The buffers are distinct __shared__ arrays;
// declaring the pointers __restrict__ gives the copy and the transform disjoint alias scopes
// once inlined, so the compiler's wait-count insertion lets the transform's LDS reads of
// `cur` run while the copy into `nxt` is in flight (without the scopes it makes the first
// LDS read wait for every copy issued before it).
template <int H, int W, int DIR>
__device__ __forceinline__ void db_stage(float* __restrict__ cur, float* __restrict__ nxt, int t, int wid, int lane,
                                         const FlatAddr& a, int64_t tile, int64_t next, int64_t ntiles,
                                         int64_t batch, const float2* tw256_in, const float2* tws_in)
{
    constexpr bool BLOCKED_IN = DIR == DCT2D_INVERSE && !RDB<H, W>::WIDE;
    if (next < ntiles) dma_tile<H, W, BLOCKED_IN>(nxt, a, next, batch, wid, lane);
    db_compute_store<H, W, DIR>(cur, t, a, tile, batch, tw256_in, tws_in);
}

template <int H, int W, int DIR>
__global__ void __launch_bounds__(256, 1)
k_rect256_db(FlatAddr a, int64_t batch, const float2* __restrict__ tw256_in, const float2* __restrict__ tws_in)
{
    using C = RDB<H, W>;
    __shared__ float4 buf0[C::TILE / 4];
    __shared__ float4 buf1[C::TILE / 4];
    float* b0 = reinterpret_cast<float*>(buf0);
    float* b1 = reinterpret_cast<float*>(buf1);
    constexpr bool BLOCKED_IN = DIR == DCT2D_INVERSE && !C::WIDE;
    const int t = threadIdx.x;
    const int wid = __builtin_amdgcn_readfirstlane(t >> 6), lane = t & 63;
    const int64_t ntiles = (batch + C::BPW - 1) / C::BPW;
    int64_t tile = blockIdx.x;
    if (tile >= ntiles) return;
    dma_tile<H, W, BLOCKED_IN>(b0, a, tile, batch, wid, lane);
    // first tile: only its copies are outstanding
    asm volatile("s_waitcnt vmcnt(0)\n\ts_barrier" ::: "memory");
    for (;;) {
        // tile in buffer 0; the next one goes to buffer 1 (released by the previous tile's store)
        int64_t next = tile + gridDim.x;
        db_stage<H, W, DIR>(b0, b1, t, wid, lane, a, tile, next, ntiles, batch, tw256_in, tws_in);
        if (next >= ntiles) break;
        tile = next;
        // Vector memory operations complete in issue order as far as the counter goes: the
        // next tile's copies are done once at most the 16 stores of the tile just finished
        // remain (that tile was not the last, so it was whole and issued all 16).  The
        // barrier then makes every wavefront's copies visible.
        asm volatile("s_waitcnt vmcnt(16)\n\ts_barrier" ::: "memory");
        next = tile + gridDim.x;
        db_stage<H, W, DIR>(b1, b0, t, wid, lane, a, tile, next, ntiles, batch, tw256_in, tws_in);
        if (next >= ntiles) break;
        tile = next;
        asm volatile("s_waitcnt vmcnt(16)\n\ts_barrier" ::: "memory");
    }
}

} // namespace

template <int H, int W>
int launch_rect256_hw(const DeviceTables* t, const Job& j)
{
    using C = R256<H, W>;
    const float2* tw256 = tw_for(t, 256);
    const float2* tws = tw_for(t, C::S);
    if constexpr (C::S <= 64) {
        if (j.variant == 3 && !j.in_idx && !j.out_idx && !j.in_slot && !j.out_slot) {
            using D = RDB<H, W>;
            const FlatAddr fa{j.in, j.out, j.in_stride, j.out_stride, j.lam, j.lam_stride};
            const int64_t ntiles = (j.batch + D::BPW - 1) / D::BPW;
            const int64_t cap = t->num_cu; // one persistent workgroup per CU (two tile buffers)
            const unsigned grid = (unsigned)(ntiles < cap ? ntiles : cap);
            switch (j.dir) {
            case DCT2D_FORWARD: k_rect256_db<H, W, DCT2D_FORWARD><<<grid, 256, 0, j.stream>>>(fa, j.batch, tw256, tws); break;
            case DCT2D_INVERSE: k_rect256_db<H, W, DCT2D_INVERSE><<<grid, 256, 0, j.stream>>>(fa, j.batch, tw256, tws); break;
            case DIR_FILTER: k_rect256_db<H, W, DIR_FILTER><<<grid, 256, 0, j.stream>>>(fa, j.batch, tw256, tws); break;
            default: k_rect256_db<H, W, DCT2D_ROUNDTRIP><<<grid, 256, 0, j.stream>>>(fa, j.batch, tw256, tws); break;
            }
            return hipGetLastError() == hipSuccess ? DCT2D_OK : DCT2D_ERR_HIP;
        }
    }
    const int64_t ntiles = (j.batch + C::BPW - 1) / C::BPW;
    int64_t cap = 0x7fffffff; // variant 0: one tile per workgroup
    if (j.variant >= 2) {
        // resident workgroups only, each looping over tiles
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_rect256<H, W, DCT2D_FORWARD>, C::NT, 0) !=
                hipSuccess ||
            per_cu < 1)
            per_cu = 1;
        cap = (int64_t)t->num_cu * per_cu;
    }
    if (ntiles > 0x7fffffff) return DCT2D_ERR_ARG;
    const unsigned grid = (unsigned)(ntiles < cap ? ntiles : cap);
    switch (j.dir) {
    case DCT2D_FORWARD: k_rect256<H, W, DCT2D_FORWARD><<<grid, C::NT, 0, j.stream>>>(j.addr(), j.batch, tw256, tws); break;
    case DCT2D_INVERSE: k_rect256<H, W, DCT2D_INVERSE><<<grid, C::NT, 0, j.stream>>>(j.addr(), j.batch, tw256, tws); break;
    case DIR_FILTER: k_rect256<H, W, DIR_FILTER><<<grid, C::NT, 0, j.stream>>>(j.addr(), j.batch, tw256, tws); break;
    default: k_rect256<H, W, DCT2D_ROUNDTRIP><<<grid, C::NT, 0, j.stream>>>(j.addr(), j.batch, tw256, tws); break;
    }
    return hipGetLastError() == hipSuccess ? DCT2D_OK : DCT2D_ERR_HIP;
}

template <int S>
int launch_rect256_s(const DeviceTables* t, const Job& j)
{
    return j.cols == 256 ? launch_rect256_hw<S, 256>(t, j) : launch_rect256_hw<256, S>(t, j);
}

int launch_rect256(const DeviceTables* t, const Job& j)
{
    switch (j.cols == 256 ? j.rows : j.cols) {
    case 8: return launch_rect256_s<8>(t, j);
    case 16: return launch_rect256_s<16>(t, j);
    case 32: return launch_rect256_s<32>(t, j);
    case 64: return launch_rect256_s<64>(t, j);
    case 128: return launch_rect256_s<128>(t, j);
    default: return DCT2D_ERR_SIZE;
    }
}

} // namespace dct
