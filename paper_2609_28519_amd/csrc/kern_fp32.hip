// Float32 2D DCT kernels on the vector ALU (all sizes, the "plain FP32" path).
//
// Separable evaluation of eq. 2 (Section 2.1): a length-W transform along every row,
// then a length-H transform along every column, each done on a vector held in registers
// (dct1d.hpp).  The paper's CPU organisation (Section 3.1, Algorithm 1) copies rows into
// padded scratch of stride n+4, runs one pass per lane, re-packs into bands and runs the
// other pass.  The GPU analogues here keep each array on chip between the two passes, so
// every element is read from HBM once and written once (the fused round trip runs the
// forward and inverse column transforms back to back in registers; Prop. 1: no
// intermediate correction):
//
//   k_wave (rows, cols <= 64): one wavefront per tile of 64 / max(rows, cols) arrays;
//     a lane transforms a row, the rows meet in an LDS tile, a lane transforms a
//     column.  Variants stage the tile through LDS with coalesced 16-byte moves and
//     cap the resident workgroups per CU (fewer bytes in flight per CU).
//   k_fused (rows, cols <= 128): a workgroup stages a tile of whole arrays in LDS with
//     a padded row pitch of cols + 4 and runs a row pass and a column pass there.
//   k_split64 / k_split128 / k_split256: one workgroup per array, each transform shared
//     by two halves of the workgroup through the top level of the even/odd recursion.
//   k_rows / k_cols (an axis of 256 in a rectangle): the row pass and the column pass
//     are separate launches over HBM (a thread owns a whole row or column; column
//     accesses are coalesced across the wavefront's consecutive columns).
// The spectral filter (Prop. 1, eq. 4; internal direction DIR_FILTER) is the fused round
// trip of every kernel with one extra step where a thread holds a column's forward
// coefficients: each is multiplied by its entry of the multiplier array before the
// inverse column transform.  The data still crosses HBM once each way.
#include "dct1d.hpp"
#include "fp32_common.hpp"
#include "internal.hpp"

namespace dct {
namespace {

constexpr int cmax(int a, int b) { return a > b ? a : b; }

template <int H, int W>
struct B2D {
    static constexpr int TB = cmax(H, W);            // threads per array
    static constexpr int NT = TB >= 128 ? TB : 256;  // threads per workgroup
    static constexpr int BPW = NT / TB;              // arrays per tile
    static constexpr int P = W + 4;                  // LDS row pitch in floats
    static constexpr int HP = H * P;
    // array pitch in LDS: congruent to TB mod 64 so the arrays of one wavefront start
    // in different banks during column reads
    static constexpr int BS = TB >= 64 ? HP : HP + ((TB - HP % 64) + 64) % 64;
    static constexpr int CPB = H * W / 4;            // float4 chunks per array
    static constexpr int CHUNKS = CPB * BPW;
    static constexpr int CPT = (CHUNKS + NT - 1) / NT;
    static constexpr int LDS_FLOATS = BPW * BS;
};

// Filter step of the split kernels: o[k] *= lam[k * PITCH + off] for k < N, lam wave-uniform.
// Every o[k] is final before the first multiplier load (the loads' offsets depend on a value
// the empty asm statements order after the transform), and at most C loads are in flight:
// loads scheduled into the tail of the transform find its temporaries live and, at the
// register limit, go out one at a time with a wait after each.  32-bit byte offsets from the
// uniform base keep each address in one register.
template <int N, int PITCH, int C>
__device__ __forceinline__ void scale_coefs(float (&o)[N], const gfloat* lam, int off)
{
#pragma unroll
    for (int k = 0; k < N; ++k) asm volatile("" : "+v"(o[k]));
    asm volatile("" : "+v"(off));
    const DCT_GLOBAL char* lb = reinterpret_cast<const DCT_GLOBAL char*>(lam);
#pragma unroll
    for (int k = 0; k < N; ++k) {
        o[k] *= *reinterpret_cast<const gfloat*>(lb + (uint32_t)((k * PITCH + off) * 4));
        if (k % C == C - 1) asm volatile("" : "+v"(off) : "v"(o[k]));
    }
}

// Row pass on an LDS tile: thread (array tb, row r) transforms its row in place.
template <int H, int W, bool INV>
__device__ __forceinline__ void lds_row_pass(float* lds, int tb, int r, twptr tw)
{
    using C = B2D<H, W>;
    if (r < H) {
        float v[W];
        float* row = lds + tb * C::BS + r * C::P;
#pragma unroll
        for (int j = 0; j < W / 4; ++j) {
            const float4 q = *reinterpret_cast<const float4*>(row + 4 * j);
            v[4 * j] = q.x; v[4 * j + 1] = q.y; v[4 * j + 2] = q.z; v[4 * j + 3] = q.w;
        }
        if (INV) dct3_ortho<W>(v, tw); else dct2_ortho<W>(v, tw);
#pragma unroll
        for (int j = 0; j < W / 4; ++j)
            *reinterpret_cast<float4*>(row + 4 * j) = make_float4(v[4 * j], v[4 * j + 1], v[4 * j + 2], v[4 * j + 3]);
    }
}

template <int H, int W, int DIR>
__global__ void __launch_bounds__((B2D<H, W>::NT))
k_fused(Addr a, int64_t batch, const float2* __restrict__ twh_in, const float2* __restrict__ tww_in)
{
    using C = B2D<H, W>;
    __shared__ float4 lds4[(C::LDS_FLOATS + 3) / 4];
    float* lds = reinterpret_cast<float*>(lds4);
    const int t = threadIdx.x;
    const int tb = t / C::TB, tl = t % C::TB;
    const int64_t ntiles = (batch + C::BPW - 1) / C::BPW;
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const twptr twh = per_iteration(twh_in);
        const twptr tww = per_iteration(tww_in);
        const int64_t b0 = tile * C::BPW;
#pragma unroll
        for (int i = 0; i < C::CPT; ++i) {
            const int c = t + C::NT * i;
            if (C::CHUNKS % C::NT == 0 || c < C::CHUNKS) {
                const int b = c / C::CPB, q = c % C::CPB;
                const int r = q / (W / 4), c4 = q % (W / 4);
                float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
                if (b0 + b < batch) v = *reinterpret_cast<const gfloat4*>(a.src(b0 + b) + 4 * q);
                *reinterpret_cast<float4*>(lds + b * C::BS + r * C::P + 4 * c4) = v;
            }
        }
        __syncthreads();
        lds_row_pass<H, W, DIR == DCT2D_INVERSE>(lds, tb, tl, tww);
        __syncthreads();
        if (tl < W) {
            float v[H];
            float* col = lds + tb * C::BS + tl;
#pragma unroll
            for (int r = 0; r < H; ++r) v[r] = col[r * C::P];
            if constexpr (DIR == DIR_FILTER)
                filter1d<H>(v, a.lam_for(b0 + tb < batch ? b0 + tb : b0) + tl, W, twh);
            else
                apply1d<H, DIR>(v, twh);
#pragma unroll
            for (int r = 0; r < H; ++r) col[r * C::P] = v[r];
        }
        __syncthreads();
        if (DIR >= DCT2D_ROUNDTRIP) {
            lds_row_pass<H, W, true>(lds, tb, tl, tww);
            __syncthreads();
        }
#pragma unroll
        for (int i = 0; i < C::CPT; ++i) {
            const int c = t + C::NT * i;
            if (C::CHUNKS % C::NT == 0 || c < C::CHUNKS) {
                const int b = c / C::CPB, q = c % C::CPB;
                const int r = q / (W / 4), c4 = q % (W / 4);
                const float4 v = *reinterpret_cast<const float4*>(lds + b * C::BS + r * C::P + 4 * c4);
                if (b0 + b < batch) *reinterpret_cast<gfloat4*>(a.dst(b0 + b) + 4 * q) = v;
            }
        }
        __syncthreads();
    }
}

// Wave-local fused kernel (one wavefront per workgroup, rows and cols <= 64; a tile is
// the 64/TB consecutive arrays that the lanes of the wavefront cover): each lane
// transforms one row and writes it into the LDS tile; after a wavefront-local barrier
// each lane reads one column, transforms it and stores it (consecutive lanes hold
// consecutive columns).  The round trip goes back through LDS for the inverse row pass.
// Plain variant: the rows come straight from HBM into registers and the results leave
// from registers.  Staged variant: the tile enters and leaves the LDS tile by whole-tile
// coalesced 16-byte moves.  No barrier couples different wavefronts.
template <int H, int W>
struct WaveCfg {
    static constexpr int TB = cmax(H, W);
    static_assert(TB <= 64, "one wavefront per tile");
    static constexpr int BPW = 64 / TB;
    // Rows of 16 or more floats are stored unpadded, with the 16-byte groups of row r
    // XOR-permuted by a row key: the 8 rows that one 8-lane phase of a lane-per-row
    // 16-byte access touches land on 8 different group positions of the 32 banks, a
    // lane-per-column 4-byte access reads a permutation of one row, and an array takes
    // exactly H*W floats (which raises the number of resident workgroups where LDS is the
    // limit).  Rows of 8 use the padded pitch 12.
    static constexpr bool SWZ = W >= 16;
    static constexpr int G = W / 4;                  // 16-byte groups per row
    static constexpr int RPL = W >= 32 ? 1 : 32 / W; // rows per 32-bank line
    static constexpr int P = SWZ ? W : W + 4;
    static constexpr int HP = H * P;
    // array pitch: the arrays of one wavefront start in different banks
    static constexpr int BS = TB >= 64 ? HP : HP + ((TB - HP % 64) + 64) % 64;
    static constexpr int LDS_FLOATS = BPW * BS;
    // float offset of group j of row r, and of element (r, c)
    __device__ static int at4(int r, int j)
    {
        return SWZ ? r * P + 4 * (j ^ ((r / RPL) & (G - 1))) : r * P + 4 * j;
    }
    __device__ static int at(int r, int c) { return at4(r, c >> 2) + (c & 3); }
};

// Row tl of array b from HBM into registers (zeros for a tail slot past the batch).
template <int H, int W>
__device__ __forceinline__ void wave_rows_in(float (&v)[W], const Addr& a, int64_t b, bool valid, int tl)
{
    if (valid) {
        const gfloat* src = a.src(b) + (int64_t)tl * W;
#pragma unroll
        for (int j = 0; j < W / 4; ++j) {
            const float4 q = *reinterpret_cast<const gfloat4*>(src + 4 * j);
            v[4 * j] = q.x; v[4 * j + 1] = q.y; v[4 * j + 2] = q.z; v[4 * j + 3] = q.w;
        }
    } else {
#pragma unroll
        for (int j = 0; j < W; ++j) v[j] = 0.f;
    }
}

template <int H, int W>
__device__ __forceinline__ void lds_row_in(float (&v)[W], const float* tile, int r)
{
    using C = WaveCfg<H, W>;
#pragma unroll
    for (int j = 0; j < W / 4; ++j) {
        const float4 q = *reinterpret_cast<const float4*>(tile + C::at4(r, j));
        v[4 * j] = q.x; v[4 * j + 1] = q.y; v[4 * j + 2] = q.z; v[4 * j + 3] = q.w;
    }
}

template <int H, int W>
__device__ __forceinline__ void lds_row_out(float* tile, int r, const float (&v)[W])
{
    using C = WaveCfg<H, W>;
#pragma unroll
    for (int j = 0; j < W / 4; ++j)
        *reinterpret_cast<float4*>(tile + C::at4(r, j)) = make_float4(v[4 * j], v[4 * j + 1], v[4 * j + 2], v[4 * j + 3]);
}

// Chunk 64 i + t of a wavefront's tile: array bb of the tile, 16-byte chunk q of that array.
// Arrays of 64 chunks or more: one array per instruction (bb known at compile time);
// smaller arrays: 64 / CPB whole arrays per instruction.
template <int H, int W>
struct WaveChunks {
    using C = WaveCfg<H, W>;
    static constexpr int CPB = H * W / 4, CH = CPB * C::BPW, NI = CH / 64;
    static constexpr bool WIDE = CPB >= 64;
    static constexpr int NA = WIDE ? C::BPW : NI; // distinct arrays a lane touches
    static_assert(CH % 64 == 0 && (CPB % 64 == 0 || 64 % CPB == 0), "whole wavefront instructions");
    __device__ static int array(int i, int t) { return WIDE ? (64 * i) / CPB : (64 * i) / CPB + t / CPB; }
    __device__ static int chunk(int i, int t) { return WIDE ? (64 * i) % CPB + t : t % CPB; }
    __device__ static int slot(int i) { return WIDE ? (64 * i) / CPB : i; } // index into the NA arrays
    __device__ static int lds_off(int i, int t)
    {
        const int q = chunk(i, t);
        return array(i, t) * C::BS + C::at4(q / (W / 4), q % (W / 4));
    }
};

// Whole-tile moves between HBM and the wavefront's LDS tile (consecutive lanes on
// consecutive 16-byte chunks).  Array addresses are resolved once, before the first
// access: an offset-list or base-slot read issued after a store would wait for it.
template <int H, int W>
__device__ __forceinline__ void wave_tile_in(float* lds, const Addr& a, int64_t b0, int64_t batch, int t)
{
    using K = WaveChunks<H, W>;
    const gfloat* base = a.src_base();
    const gfloat* p[K::NA];
#pragma unroll
    for (int k = 0; k < K::NA; ++k) {
        const int64_t b = b0 + (K::WIDE ? k : K::array(k, t));
        // a tail slot past the batch transforms a copy of array b0 (always in the batch)
        // and is never stored, so every load is unconditional and all are in flight at once
        p[k] = base + a.src_off(b < batch ? b : b0);
    }
#pragma unroll
    for (int i = 0; i < K::NI; ++i) {
        const float4 v = *reinterpret_cast<const gfloat4*>(p[K::slot(i)] + 4 * K::chunk(i, t));
        *reinterpret_cast<float4*>(lds + K::lds_off(i, t)) = v;
    }
}

template <int H, int W>
__device__ __forceinline__ void wave_tile_out(const float* lds, const Addr& a, int64_t b0, int64_t batch, int t)
{
    using K = WaveChunks<H, W>;
    gfloat* base = a.dst_base();
    gfloat* p[K::NA];
    bool ok[K::NA]; // wave-uniform when WIDE
#pragma unroll
    for (int k = 0; k < K::NA; ++k) {
        const int64_t b = b0 + (K::WIDE ? k : K::array(k, t));
        ok[k] = b < batch;
        p[k] = base + a.dst_off(ok[k] ? b : b0);
        asm volatile("" : "+v"(p[k])); // materialised here, not sunk between the stores
    }
#pragma unroll
    for (int i = 0; i < K::NI; ++i) {
        const float4 v = *reinterpret_cast<const float4*>(lds + K::lds_off(i, t));
        if (ok[K::slot(i)]) *reinterpret_cast<gfloat4*>(p[K::slot(i)] + 4 * K::chunk(i, t)) = v;
    }
}

// Wave-local kernel.  Plain: each lane loads its row from HBM and the results leave from
// registers (columns as 4-byte stores across the lanes, round-trip rows as 16-byte row
// stores).  STAGE: the tile enters and leaves through the LDS tile with whole-tile
// coalesced 16-byte moves, and the lanes read and write their rows and columns there.
template <int H, int W, int DIR, bool STAGE>
__global__ void __launch_bounds__(64)
k_wave(Addr a, int64_t batch, const float2* __restrict__ twh_in, const float2* __restrict__ tww_in)
{
    using C = WaveCfg<H, W>;
    __shared__ float4 lds4[(C::LDS_FLOATS + 3) / 4];
    float* lds = reinterpret_cast<float*>(lds4);
    const int t = threadIdx.x;
    const int tb = t / C::TB, tl = t % C::TB;
    const int64_t ntiles = (batch + C::BPW - 1) / C::BPW;
    float* tile_lds = lds + tb * C::BS;
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t b0 = tile * C::BPW;
        const int64_t b = b0 + tb;
        const bool valid = b < batch;
        if (STAGE) {
            wave_tile_in<H, W>(lds, a, b0, batch, t);
            __syncthreads();
        }
        twptr tww = per_iteration(tww_in);
        if (tl < H) {
            float v[W];
            if (STAGE) lds_row_in<H, W>(v, tile_lds, tl); else wave_rows_in<H, W>(v, a, b, valid, tl);
            if (DIR == DCT2D_INVERSE) dct3_ortho<W>(v, tww); else dct2_ortho<W>(v, tww);
            lds_row_out<H, W>(tile_lds, tl, v);
        }
        // filter: the multipliers of column tl are requested here, so they arrive during the
        // column reads and the forward transform instead of stalling the multiply
        float lq[H];
        if (DIR == DIR_FILTER && tl < W) {
            const gfloat* lp = a.lam_for(valid ? b : b0) + tl;
#pragma unroll
            for (int r = 0; r < H; ++r) lq[r] = lp[r * W];
        }
        __syncthreads();
        twptr twh = per_iteration(twh_in); // the column pass re-reads its twiddles (see per_iteration)
        if (tl < W) {
            float c[H];
#pragma unroll
            for (int r = 0; r < H; ++r) c[r] = tile_lds[C::at(r, tl)];
            if constexpr (DIR == DIR_FILTER) {
                dct2_ortho<H>(c, twh);
#pragma unroll
                for (int r = 0; r < H; ++r) c[r] *= lq[r];
                asm volatile("" : "+s"(twh));
                dct3_ortho<H>(c, twh);
            } else {
                apply1d<H, DIR>(c, twh);
            }
            if (STAGE || DIR >= DCT2D_ROUNDTRIP) {
#pragma unroll
                for (int r = 0; r < H; ++r) tile_lds[C::at(r, tl)] = c[r];
            } else if (valid) {
                gfloat* dst = a.dst(b) + tl;
#pragma unroll
                for (int r = 0; r < H; ++r) dst[(int64_t)r * W] = c[r];
            }
        }
        if (DIR >= DCT2D_ROUNDTRIP) {
            __syncthreads();
            tww = per_iteration(tww_in);
            if (tl < H) {
                float r[W];
                lds_row_in<H, W>(r, tile_lds, tl);
                dct3_ortho<W>(r, tww);
                if (STAGE) {
                    lds_row_out<H, W>(tile_lds, tl, r);
                } else if (valid) {
                    gfloat* dst = a.dst(b) + (int64_t)tl * W;
#pragma unroll
                    for (int j = 0; j < W / 4; ++j)
                        *reinterpret_cast<gfloat4*>(dst + 4 * j) =
                            make_float4(r[4 * j], r[4 * j + 1], r[4 * j + 2], r[4 * j + 3]);
                }
            }
        }
        if (STAGE) {
            __syncthreads();
            wave_tile_out<H, W>(lds, a, b0, batch, t);
        }
        __syncthreads();
    }
}

// Split fused kernel for 128 x 128 arrays: one 256-thread workgroup per array.  Every
// length-128 transform is shared by two wavefronts through the top level of the
// even/odd recursion (dct1d.hpp): the "even" wavefronts (0, 1) work on
// u[n] = x[n] + x[127-n] -> DCT-II_64 (even outputs), the "odd" wavefronts (2, 3) on
// w[n] = x[n] - x[127-n] -> DCT-IV_64 (odd outputs); for the inverse, DCT-III_64 of the
// even and DCT-IV_64 of the odd coefficients, recombined as a + b and a - b.  The role
// is uniform per wavefront (no divergence), each thread holds 64 values, and the
// array's intermediate lives in one LDS tile of odd pitch 129 (conflict-free for the
// stride-2 row writes and the column reads).
//   forward:    rows (HBM -> regs -> LDS)  | columns (LDS -> regs -> HBM, lanes = columns)
//   inverse:    columns (HBM -> regs -> LDS, a|b halves) | rows (LDS, recombined on read)
//               -> a|b halves in LDS | coalesced recombining store
//   round trip: forward rows | forward + inverse columns in registers | inverse rows
constexpr int S128_P = 129;

// STAGE: the forward rows (inverse columns) come from an LDS copy of the array (row pitch
// 132) filled with coalesced 16-byte loads (each wavefront instruction covers two whole
// rows) instead of each thread reading its own row (column) from HBM.
// One array, as seen by the wavefronts of one role (each role runs its own straight-line
// code; both pass the same barriers).
template <int DIR, bool STAGE, int ROLE>
__device__ __forceinline__ void s128_array(const Addr& a, int64_t blk, float* T, const float2* tw_in, int t)
{
    constexpr int L = 128, H = 64, P = S128_P, SP = 132;
    constexpr int role = ROLE; // 0: even half, 1: odd half
    const int idx = t & 127;   // row or column handled by this thread
    twptr tw = per_iteration(tw_in);
    const gfloat* src = a.src(blk);
    gfloat* dst = a.dst(blk);
    float v[H], o[H];
    if (DIR != DCT2D_INVERSE) {
        // ---- forward rows: row idx ------------------------------------------------
        if (STAGE) {
            // (the previous array's last LDS reads precede its final barrier)
            const DCT_GLOBAL char* sb = reinterpret_cast<const DCT_GLOBAL char*>(uniform_ptr(src));
            float q[64];
#pragma unroll
            for (int it = 0; it < 16; ++it) {
                const float4 w = *reinterpret_cast<const gfloat4*>(sb + (uint32_t)((it * 256 + t) * 16));
                q[4 * it] = w.x; q[4 * it + 1] = w.y; q[4 * it + 2] = w.z; q[4 * it + 3] = w.w;
            }
#pragma unroll
            for (int it = 0; it < 16; ++it) {
                const int f = it * 256 + t; // row f / 32, columns 4 (f % 32) .. +3
                *reinterpret_cast<float4*>(&T[(f >> 5) * SP + 4 * (f & 31)]) =
                    make_float4(q[4 * it], q[4 * it + 1], q[4 * it + 2], q[4 * it + 3]);
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < H / 4; ++j) {
                const float4 lo = *reinterpret_cast<const float4*>(&T[idx * SP + 4 * j]);
                const float4 hi = *reinterpret_cast<const float4*>(&T[idx * SP + L - 4 - 4 * j]);
                const float xl[4] = {lo.x, lo.y, lo.z, lo.w};
                const float xh[4] = {hi.w, hi.z, hi.y, hi.x}; // x[127 - (4j + i)]
#pragma unroll
                for (int i = 0; i < 4; ++i) v[4 * j + i] = role == 0 ? xl[i] + xh[i] : xl[i] - xh[i];
            }
            __syncthreads(); // the staged copy is read before the tile overwrites it
        } else {
            const gfloat* row = src + (int64_t)idx * L;
#pragma unroll
            for (int j = 0; j < H / 4; ++j) {
                const float4 lo = *reinterpret_cast<const gfloat4*>(row + 4 * j);
                const float4 hi = *reinterpret_cast<const gfloat4*>(row + L - 4 - 4 * j);
                const float xl[4] = {lo.x, lo.y, lo.z, lo.w};
                const float xh[4] = {hi.w, hi.z, hi.y, hi.x}; // x[127 - (4j + i)]
#pragma unroll
                for (int i = 0; i < 4; ++i) v[4 * j + i] = role == 0 ? xl[i] + xh[i] : xl[i] - xh[i];
            }
        }
        if (role == 0) dct2_rec<L, H>(v, o, tw); else dct4_scaled<L, H>(v, o, tw);
#pragma unroll
        for (int k = 0; k < H; ++k) T[idx * P + 2 * k + role] = o[k];
        __syncthreads();
        // ---- forward columns: column idx from LDS ---------------------------------
#pragma unroll
        for (int n = 0; n < H; ++n) {
            const float xl = T[n * P + idx], xh = T[(L - 1 - n) * P + idx];
            v[n] = role == 0 ? xl + xh : xl - xh;
        }
        if (role == 0) dct2_rec<L, H>(v, o, tw); else dct4_scaled<L, H>(v, o, tw);
        if (DIR == DCT2D_FORWARD) {
#pragma unroll
            for (int k = 0; k < H; ++k) dst[(int64_t)(2 * k + role) * L + idx] = o[k];
            __syncthreads(); // LDS reuse by the next array
            return;
        }
        if (DIR == DIR_FILTER) {
            // The coefficients pass through the tile (coefficient row 2k + role of column idx
            // at T[(2k + role) P + idx]), where lane t scales element t % 128 of rows 2i + t / 128
            // with all of its 64 multiplier loads in flight at once: loaded beside the live
            // coefficients, the same loads would go out one or two at a time.
            // the loads go out once the transform is done (their offsets depend on a value
            // the empty asm statements order after it) and fly during the barrier wait
#pragma unroll
            for (int k = 0; k < H; ++k) asm volatile("" : "+v"(o[k]));
            int lt = t;
            asm volatile("" : "+v"(lt));
            const DCT_GLOBAL char* lb = reinterpret_cast<const DCT_GLOBAL char*>(uniform_ptr(a.lam_for(blk)));
            float lq[H];
#pragma unroll
            for (int i = 0; i < H; ++i) lq[i] = *reinterpret_cast<const gfloat*>(lb + (uint32_t)((i * 256 + lt) * 4));
            __syncthreads(); // every column read before the coefficients overwrite the tile
#pragma unroll
            for (int k = 0; k < H; ++k) T[(2 * k + role) * P + idx] = o[k];
            __syncthreads();
#pragma unroll
            for (int i = 0; i < H; ++i) T[(2 * i + (t >> 7)) * P + idx] *= lq[i];
            __syncthreads();
#pragma unroll
            for (int k = 0; k < H; ++k) o[k] = T[(2 * k + role) * P + idx];
        }
        // round trip: inverse columns on the same data (even -> DCT-III_64, odd -> DCT-IV_64)
        asm volatile("" : "+s"(tw));
        if (role == 0) dct3_rec<L, H>(o, v, tw); else dct4_scaled<L, H>(o, v, tw);
        __syncthreads(); // every column read before the halves overwrite it
#pragma unroll
        for (int n = 0; n < H; ++n) T[(role * H + n) * P + idx] = v[n];
    } else {
        // ---- inverse columns: even (role 0) or odd (role 1) coefficient rows
        if (STAGE) {
            // coalesced 16-byte loads into an LDS copy (pitch 132), then column idx from it
            const DCT_GLOBAL char* sb = reinterpret_cast<const DCT_GLOBAL char*>(uniform_ptr(src));
            float q[64];
#pragma unroll
            for (int it = 0; it < 16; ++it) {
                const float4 w = *reinterpret_cast<const gfloat4*>(sb + (uint32_t)((it * 256 + t) * 16));
                q[4 * it] = w.x; q[4 * it + 1] = w.y; q[4 * it + 2] = w.z; q[4 * it + 3] = w.w;
            }
#pragma unroll
            for (int it = 0; it < 16; ++it) {
                const int f = it * 256 + t;
                *reinterpret_cast<float4*>(&T[(f >> 5) * SP + 4 * (f & 31)]) =
                    make_float4(q[4 * it], q[4 * it + 1], q[4 * it + 2], q[4 * it + 3]);
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < H; ++k) o[k] = T[(2 * k + role) * SP + idx];
            __syncthreads(); // the staged copy is read before the halves overwrite it
        } else {
#pragma unroll
            for (int k = 0; k < H; ++k) o[k] = src[(int64_t)(2 * k + role) * L + idx];
        }
        if (role == 0) dct3_rec<L, H>(o, v, tw); else dct4_scaled<L, H>(o, v, tw);
#pragma unroll
        for (int n = 0; n < H; ++n) T[(role * H + n) * P + idx] = v[n];
    }
    __syncthreads();
    // ---- inverse rows.  LDS holds the column results as halves: rows 0..63 = a,
    // rows 64..127 = b, with Z[n] = a[n] + b[n], Z[127-n] = a[n] - b[n].
    {
        const bool top = idx < H;
        const int rr = top ? idx : L - 1 - idx;
        const float sg = top ? 1.f : -1.f;
#pragma unroll
        for (int k = 0; k < H; ++k) {
            const int c = 2 * k + role;
            o[k] = T[rr * P + c] + sg * T[(H + rr) * P + c];
        }
    }
    if (role == 0) dct3_rec<L, H>(o, v, tw); else dct4_scaled<L, H>(o, v, tw);
    __syncthreads(); // all reads of the column halves done
#pragma unroll
    for (int n = 0; n < H; ++n) T[idx * P + role * H + n] = v[n];
    __syncthreads();
    // ---- store: x[r][n] = a[n] + b[n], x[r][127-n] = a[n] - b[n].  Lane t covers column
    // t % 128 of rows 2i + t / 128: consecutive lanes read consecutive LDS words (no bank
    // conflicts) and write 256-byte segments.
    {
        int c = t & (L - 1);
        asm volatile("" : "+v"(c)); // per array: keeps the 128 offsets below out of the loop preheader
        const int cs = c < H ? c : L - 1 - c;
        const float sg = c < H ? 1.f : -1.f; // exact: one rounding, as a +- b
        DCT_GLOBAL char* db = reinterpret_cast<DCT_GLOBAL char*>(uniform_ptr(dst));
#pragma unroll
        for (int i = 0; i < L / 2; ++i) {
            const int r = 2 * i + (t >> 7);
            *reinterpret_cast<gfloat*>(db + (uint32_t)((r * L + c) * 4)) =
                __builtin_fmaf(sg, T[r * P + H + cs], T[r * P + cs]);
        }
    }
    __syncthreads();
}

template <int DIR, bool STAGE>
__global__ void __launch_bounds__(256, 2) // two workgroups per CU: the LDS tile allows exactly two
k_split128(Addr a, int64_t batch, const float2* __restrict__ tw_in)
{
    constexpr int L = 128, P = S128_P, SP = 132;
    __shared__ float4 T4[(STAGE ? L * SP : L * P) / 4];
    float* const T = reinterpret_cast<float*>(T4);
    const int t = threadIdx.x;
    const bool odd = t >= 128; // the role (uniform per wavefront)
    for (int64_t blk = blockIdx.x; blk < batch; blk += gridDim.x) {
        if (odd) s128_array<DIR, STAGE, 1>(a, blk, T, tw_in, t); else s128_array<DIR, STAGE, 0>(a, blk, T, tw_in, t);
    }
}

// Split fused kernel for 64 x 64 arrays: one 128-thread workgroup (two wavefronts) per
// array; every length-64 transform is shared by the two wavefronts through the top level
// of the even/odd recursion (wavefront 0: the DCT-II_32 / DCT-III_32 half, wavefront 1:
// the DCT-IV_32 half), so a lane holds 32 values and a CU holds twice the wavefronts of
// the wave-local kernel in the same LDS.  The array lives in one unpadded, XOR-swizzled
// 64 x 64 LDS tile (the layout of WaveCfg<64, 64>) and enters and leaves by whole-array
// coalesced 16-byte moves.  Between the passes each row (column) is kept as two halves,
// wavefront 0's results in physical columns (rows) 0..31 and wavefront 1's in 32..63.
//   forward:    rows -> [even | odd coefficient] halves | columns -> [even ; odd]
//               halves | out, each 16-byte chunk gathered from the permuted tile
//   round trip: forward rows | forward and inverse columns in registers -> [p ; q]
//               (z = p + q, z[63-n] = p - q) | inverse rows of the recombined columns
//               -> [p | q] | out, recombining each chunk
//   inverse:    inverse columns -> [p ; q], stored in the column order the forward rows
//               leave | then as the round trip
// One array, as seen by the wavefront of one role (each role runs its own straight-line
// code; both pass the same barriers).
template <int DIR, int ROLE>
__device__ __forceinline__ void split64_array(const Addr& a, int64_t b, float* T, const float2* tw_in)
{
    using C = WaveCfg<64, 64>;
    constexpr int N = 64, H = 32;
    {
        // lane indices are made opaque per array, so the LDS offsets derived from them are
        // computed where they are used instead of being hoisted out of the loop and held
        int t = threadIdx.x;
        asm volatile("" : "+v"(t));
        const int l = t & 63; // row or column of this lane
        {
            // in: chunk c = i * 128 + t is row c / 16, 16-byte group c % 16
            const gfloat* src = a.src(b);
            float4 q[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) q[i] = *reinterpret_cast<const gfloat4*>(src + 4 * (i * 128 + t));
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int c = i * 128 + t;
                *reinterpret_cast<float4*>(T + C::at4(c >> 4, c & 15)) = q[i];
            }
        }
        __syncthreads();
        float v[H], y[H];
        if (DIR != DCT2D_INVERSE) {
            // ---- forward rows: row l; u[n] = x[n] + x[63-n] (role 0), w[n] = x[n] - x[63-n]
            twptr tw = per_iteration(tw_in);
            {
                float x[N];
                lds_row_in<N, N>(x, T, l);
#pragma unroll
                for (int n = 0; n < H; ++n) v[n] = ROLE == 0 ? x[n] + x[N - 1 - n] : x[n] - x[N - 1 - n];
            }
            if constexpr (ROLE == 0) dct2_rec<N, H>(v, y, tw); else dct4_scaled<N, H>(v, y, tw);
            __syncthreads(); // every row is read before the halves overwrite it
#pragma unroll
            for (int g = 0; g < 8; ++g)
                *reinterpret_cast<float4*>(T + C::at4(l, 8 * ROLE + g)) =
                    make_float4(y[4 * g], y[4 * g + 1], y[4 * g + 2], y[4 * g + 3]);
            __syncthreads();
            // ---- columns: physical column l (logical column 2 l, or 2 (l - 32) + 1)
            tw = per_iteration(tw_in);
            {
                float x[N];
#pragma unroll
                for (int r = 0; r < N; ++r) x[r] = T[C::at(r, l)];
#pragma unroll
                for (int n = 0; n < H; ++n) v[n] = ROLE == 0 ? x[n] + x[N - 1 - n] : x[n] - x[N - 1 - n];
            }
            if constexpr (ROLE == 0) dct2_rec<N, H>(v, y, tw); else dct4_scaled<N, H>(v, y, tw);
            if (DIR >= DCT2D_ROUNDTRIP) {
                if (DIR == DIR_FILTER) // coefficient row 2k + ROLE of logical column lc
                    scale_coefs<H, 2 * N, 32>(y, uniform_ptr(a.lam_for(b)), ROLE * N + (l < H ? 2 * l : 2 * (l - H) + 1));
                tw_fence(tw);
                // p (role 0: DCT-III_32 of the even coefficients) or q (role 1: DCT-IV_32 of the odd)
                if constexpr (ROLE == 0) dct3_rec<N, H>(y, v, tw); else dct4_scaled<N, H>(y, v, tw);
            }
            __syncthreads(); // every column is read before the halves overwrite it
#pragma unroll
            for (int n = 0; n < H; ++n) T[C::at(H * ROLE + n, l)] = DIR >= DCT2D_ROUNDTRIP ? v[n] : y[n];
            __syncthreads();
        } else {
            // ---- inverse columns: logical column l; role 0 inverts the even coefficient
            // rows (DCT-III_32 -> p), role 1 the odd ones (DCT-IV_32 -> q).  The halves go
            // to physical column l / 2 (l even) or 32 + l / 2, the column order that the
            // forward rows leave, so the inverse rows below serve both directions.
            twptr tw = per_iteration(tw_in);
#pragma unroll
            for (int k = 0; k < H; ++k) v[k] = T[C::at(2 * k + ROLE, l)];
            if constexpr (ROLE == 0) dct3_rec<N, H>(v, y, tw); else dct4_scaled<N, H>(v, y, tw);
            __syncthreads(); // every column is read before the halves overwrite it
            const int pc = (l & 1) * H + (l >> 1);
#pragma unroll
            for (int n = 0; n < H; ++n) T[C::at(H * ROLE + n, pc)] = y[n];
            __syncthreads();
        }
        if (DIR != DCT2D_FORWARD) {
            // ---- inverse rows: row l.  The tile holds the columns as [p ; q] halves,
            // logical column 2 k + s at physical column 32 s + k, Z[r][.] = p[r] + q[r] for
            // r < 32 and p[63-r] - q[63-r] above.  Role 0 inverts the even coefficients
            // (DCT-III_32 -> p), role 1 the odd ones (DCT-IV_32 -> q).
            twptr tw = per_iteration(tw_in);
            {
                const int rr = l < H ? l : N - 1 - l;
                const float sg = l < H ? 1.f : -1.f; // exact: one rounding, as p +- q
#pragma unroll
                for (int g = 0; g < 8; ++g) {
                    const float4 p4 = *reinterpret_cast<const float4*>(T + C::at4(rr, 8 * ROLE + g));
                    const float4 q4 = *reinterpret_cast<const float4*>(T + C::at4(H + rr, 8 * ROLE + g));
                    v[4 * g] = __builtin_fmaf(sg, q4.x, p4.x);
                    v[4 * g + 1] = __builtin_fmaf(sg, q4.y, p4.y);
                    v[4 * g + 2] = __builtin_fmaf(sg, q4.z, p4.z);
                    v[4 * g + 3] = __builtin_fmaf(sg, q4.w, p4.w);
                }
            }
            if constexpr (ROLE == 0) dct3_rec<N, H>(v, y, tw); else dct4_scaled<N, H>(v, y, tw);
            __syncthreads(); // every row is read before the halves overwrite it
#pragma unroll
            for (int g = 0; g < 8; ++g)
                *reinterpret_cast<float4*>(T + C::at4(l, 8 * ROLE + g)) =
                    make_float4(y[4 * g], y[4 * g + 1], y[4 * g + 2], y[4 * g + 3]);
            __syncthreads();
        }
        {
            // out: chunk c = i * 128 + t is output row R = c / 16, columns 4 g .. 4 g + 3
            gfloat* dst = a.dst(b);
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int c = i * 128 + t, R = c >> 4, g = c & 15;
                float4 o;
                if (DIR == DCT2D_FORWARD) {
                    // logical (R, 4 g + j) sits at physical row (R odd) 32 + R / 2, column
                    // (j odd) 32 + 2 g + j / 2
                    const int pr = (R & 1) * H + (R >> 1);
                    o = make_float4(T[C::at(pr, 2 * g)], T[C::at(pr, H + 2 * g)], T[C::at(pr, 2 * g + 1)],
                                    T[C::at(pr, H + 2 * g + 1)]);
                } else {
                    // row R as [p | q]: x[m] = p[m] + q[m], x[63-m] = p[m] - q[m]
                    const int gg = g < 8 ? g : 15 - g;
                    const float4 p4 = *reinterpret_cast<const float4*>(T + C::at4(R, gg));
                    const float4 q4 = *reinterpret_cast<const float4*>(T + C::at4(R, 8 + gg));
                    o = g < 8 ? make_float4(p4.x + q4.x, p4.y + q4.y, p4.z + q4.z, p4.w + q4.w)
                              : make_float4(p4.w - q4.w, p4.z - q4.z, p4.y - q4.y, p4.x - q4.x);
                }
                *reinterpret_cast<gfloat4*>(dst + 4 * c) = o;
            }
        }
        __syncthreads(); // the tile is read out before the next array is staged in
    }
}

template <int DIR>
__global__ void __launch_bounds__(128, 4) // four wavefronts per SIMD: at most 128 VGPRs
k_split64(Addr a, int64_t batch, const float2* __restrict__ tw_in)
{
    __shared__ float4 T4[64 * 64 / 4];
    float* const T = reinterpret_cast<float*>(T4);
    const bool odd = threadIdx.x >= 64; // the role (uniform per wavefront)
    for (int64_t b = blockIdx.x; b < batch; b += gridDim.x) {
        if (odd) split64_array<DIR, 1>(a, b, T, tw_in); else split64_array<DIR, 0>(a, b, T, tw_in);
    }
}

// Fused kernel for 256 x 256 arrays: one 512-thread workgroup per array, one workgroup
// per CU.  Every length-256 transform is shared by two halves of the workgroup through
// the top level of the even/odd recursion (dct1d.hpp), so each thread holds 128 values:
// group E (wavefronts 0-3) takes the DCT-II_128 / DCT-III_128 half of every row
// transform, group O (wavefronts 4-7) the DCT-IV_128 half.  The array (256 KB) is
// larger than the LDS, which is used in three layouts, each holding half of it:
//   column-half stage: rows 0..255, 128 columns, pitch 132;
//   row-half stage:    128 rows, 256 columns, pitch 260;
//   tile:              rows 0..255, 128 columns, pitch 129 (odd: conflict-free row
//                      writes and column reads).
// The stages move the array between HBM and LDS with coalesced 16-byte accesses (each
// wavefront instruction covers whole 512-byte half-rows or 1 KB rows), in two windows
// each way.  The second pass runs in two rounds through the tile, one per group;
// inside a round, wavefronts with cr = 0 take the even half of each column transform
// and cr = 1 the odd half.
//   forward:    column halves in, rows (E: even outputs, O: odd outputs) | round E:
//               E's outputs (the even columns) through the tile, column transforms |
//               round O: the odd columns | coefficients out by row halves
//   inverse:    row halves in, columns (E: even columns, O: odd columns; per column the
//               halves a, b with Z[n] = a[n] + b[n], Z[255-n] = a[n] - b[n]) | round E:
//               E's halves through the tile, each E thread inverts the even entries of
//               one row (p) | round O: the odd entries (q) | out by column halves: E
//               writes p, O adds q (left half, x[m] = p[m] + q[m]) or subtracts it
//               (right half, x[255-m] = p[m] - q[m])
//   round trip: in as the forward, rows | per round: forward + inverse column
//               transforms in registers, then the inverse rows | out as the inverse.
// Group E reads its round's last tile entries (forward: columns; inverse and round trip:
// rows) during round E but transforms them during round O, beside group O's transforms,
// instead of leaving group O waiting at the barriers; in the round trip, group O's row
// transform likewise runs during round E's column phase.
// Every (group, column half) pair runs its own straight-line path; the four paths
// pass the same sequence of workgroup barriers (forward 12, inverse 14, round trip 18
// per array).  The array is read whole before its first barrier and written after,
// so in-place operation is safe.
namespace s256 {
constexpr int L = 256, H = 128, P = 129, CP = 132, RP = 260;
constexpr int LDS_FLOATS = L * CP; // the largest layout (256 x 132 > 128 x 260 > 256 x 129)

// The thread index, recomputed from the lane count (two ALU instructions) in every
// phase that needs it rather than held in a register for the whole kernel: under the
// register pressure of the 128-value transforms a long-lived index would be spilled,
// and every spill reload waits for all outstanding HBM stores of the wavefront.  The
// asm keeps each recomputation (and the offsets derived from it) inside its phase.
// `wid` is the wavefront index (wave-uniform, a scalar register).
__device__ __forceinline__ int lane_t(int wid)
{
    int l;
    asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(l));
    return wid * 64 + l;
}

// Makes the lane index depend on an already read value, so the reads of the next
// chunk of a phase cannot be issued before that value has arrived: bounds the number
// of LDS reads in flight (and the registers they hold) to one chunk.
__device__ __forceinline__ void after(int& idx, float dep)
{
    asm volatile("" : "+v"(idx) : "v"(dep));
}

// Pins a transform's results before the next workgroup barrier.  The compiler may
// otherwise move pure arithmetic across a barrier (it only orders memory operations),
// which pushes the tail of a group's transform into the phase after the barrier and
// defeats the overlap of the two groups' work.  Empty asm statements that "modify"
// every value are ordered with the barrier and so must follow the arithmetic.
template <int N>
__device__ __forceinline__ void settle(float (&v)[N])
{
#pragma unroll
    for (int k = 0; k < N; ++k) asm volatile("" : "+v"(v[k]));
}

__device__ __forceinline__ void syncs(int n)
{
    for (int k = 0; k < n; ++k) __syncthreads();
}

__device__ __forceinline__ const gfloat4* at4(const gfloat* base, uint32_t byte_off)
{
    return reinterpret_cast<const gfloat4*>(reinterpret_cast<const DCT_GLOBAL char*>(base) + byte_off);
}
__device__ __forceinline__ gfloat4* at4(gfloat* base, uint32_t byte_off)
{
    return reinterpret_cast<gfloat4*>(reinterpret_cast<DCT_GLOBAL char*>(base) + byte_off);
}

// ---- column-half stage: the outer half (array columns 0..63 and 192..255, at stage
// columns 0..63 and 64..127) or the inner half (array columns 64..191).  Either way stage
// row r holds, at columns c and 127 - c (c < 64), the mirrored pair of array columns
// (k, 255 - k) with k = c (outer) or 64 + c (inner), so each half feeds 64 even/odd
// butterflies per row.  Quadruple f = it * 512 + t (it < 16) is row f / 32, stage
// columns 4 (f % 32) .. +3.  Byte offsets are 32-bit from the wave-uniform base.
template <int HF>
__device__ __forceinline__ uint32_t colhalf_off(int f)
{
    const int c4 = f & 31;
    return (uint32_t)((f >> 5) * 1024 + (HF == 0 ? (c4 < 16 ? 16 * c4 : 16 * c4 + 512) : 256 + 16 * c4));
}
template <int HF>
__device__ __forceinline__ void load_colhalf(const gfloat* src, int wid, float (&q)[64])
{
    const int t = lane_t(wid);
#pragma unroll
    for (int it = 0; it < 16; ++it) {
        const float4 v = *at4(src, colhalf_off<HF>(it * 512 + t));
        q[4 * it] = v.x; q[4 * it + 1] = v.y; q[4 * it + 2] = v.z; q[4 * it + 3] = v.w;
    }
}
__device__ __forceinline__ void put_colhalf(float* T, int wid, const float (&q)[64])
{
    const int t = lane_t(wid);
#pragma unroll
    for (int it = 0; it < 16; ++it) {
        const int f = it * 512 + t;
        *reinterpret_cast<float4*>(&T[(f >> 5) * CP + 4 * (f & 31)]) =
            make_float4(q[4 * it], q[4 * it + 1], q[4 * it + 2], q[4 * it + 3]);
    }
}
template <int HF>
__device__ __forceinline__ void out_colhalf(gfloat* dst, const float* T, int wid)
{
    const int t = lane_t(wid);
#pragma unroll
    for (int it = 0; it < 16; ++it) {
        const int f = it * 512 + t;
        *at4(dst, colhalf_off<HF>(f)) = *reinterpret_cast<const float4*>(&T[(f >> 5) * CP + 4 * (f & 31)]);
    }
}

// ---- row-half stage: quadruple f = it * 512 + t (it < 16) is row HF * 128 + f / 64,
// columns 4 (f % 64) .. +3.
template <int HF>
__device__ __forceinline__ void load_rowhalf(const gfloat* src, int wid, float (&q)[64])
{
    const int t = lane_t(wid);
#pragma unroll
    for (int it = 0; it < 16; ++it) {
        const int f = it * 512 + t;
        const float4 v = *at4(src, (uint32_t)((HF * 128 + (f >> 6)) * 1024 + (f & 63) * 16));
        q[4 * it] = v.x; q[4 * it + 1] = v.y; q[4 * it + 2] = v.z; q[4 * it + 3] = v.w;
    }
}
__device__ __forceinline__ void put_rowhalf(float* T, int wid, const float (&q)[64])
{
    const int t = lane_t(wid);
#pragma unroll
    for (int it = 0; it < 16; ++it) {
        const int f = it * 512 + t;
        *reinterpret_cast<float4*>(&T[(f >> 6) * RP + 4 * (f & 63)]) =
            make_float4(q[4 * it], q[4 * it + 1], q[4 * it + 2], q[4 * it + 3]);
    }
}
template <int HF>
__device__ __forceinline__ void out_rowhalf(gfloat* dst, const float* T, int wid)
{
    const int t = lane_t(wid);
#pragma unroll
    for (int it = 0; it < 16; ++it) {
        const int f = it * 512 + t;
        *at4(dst, (uint32_t)((HF * 128 + (f >> 6)) * 1024 + (f & 63) * 16)) =
            *reinterpret_cast<const float4*>(&T[(f >> 6) * RP + 4 * (f & 63)]);
    }
}

// ---- forward rows through the column-half stage: row i; group 0: u[n] = x[n] +
// x[255-n] -> DCT-II_128 (even outputs), group 1: w[n] = x[n] - x[255-n] -> DCT-IV_128
// (odd outputs); n < 64 from the outer half, 64 <= n < 128 from the inner half.  Four
// barriers: outer half in, read, inner half in, read.
template <int G>
__device__ __forceinline__ void rows_from_stage(const float* T, int wid, float (&v)[H], int base)
{
    int r = lane_t(wid) & 255;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const float4 lo = *reinterpret_cast<const float4*>(&T[r * CP + 4 * j]);       // x[k .. k+3]
        const float4 hi = *reinterpret_cast<const float4*>(&T[r * CP + H - 4 - 4 * j]); // x[252-k .. 255-k]
        const float xl[4] = {lo.x, lo.y, lo.z, lo.w};
        const float xh[4] = {hi.w, hi.z, hi.y, hi.x}; // x[255 - (k + q)]
#pragma unroll
        for (int q = 0; q < 4; ++q) v[base + 4 * j + q] = G == 0 ? xl[q] + xh[q] : xl[q] - xh[q];
        if (j % 8 == 7) after(r, v[base + 4 * j + 3]);
    }
}
template <int G>
__device__ __forceinline__ void rows_fwd(const gfloat* src, float* T, int wid, float (&R)[H], twptr tw)
{
    float v[H];
    {
        float qb[64];
        {
            float qa[64];
            load_colhalf<0>(src, wid, qa);
            __syncthreads(); // earlier readers of the LDS are done
            put_colhalf(T, wid, qa);
        }
        // the inner half is requested once the outer half has arrived: half an array in
        // flight per CU at a time, its latency covered by the first row-read window
        load_colhalf<1>(src, wid, qb);
        __syncthreads();
        rows_from_stage<G>(T, wid, v, 0);
        __syncthreads();
        put_colhalf(T, wid, qb);
    }
    __syncthreads();
    rows_from_stage<G>(T, wid, v, H / 2);
    if constexpr (G == 0) dct2_rec<L, H>(v, R, tw); else dct4_scaled<L, H>(v, R, tw);
    settle(R);
}

// The staging part of rows_fwd alone (same four barriers): v receives the row entries and
// the caller transforms them later.
template <int G>
__device__ __forceinline__ void rows_fwd_stage(const gfloat* src, float* T, int wid, float (&v)[H])
{
    {
        float qb[64];
        {
            float qa[64];
            load_colhalf<0>(src, wid, qa);
            __syncthreads(); // earlier readers of the LDS are done
            put_colhalf(T, wid, qa);
        }
        load_colhalf<1>(src, wid, qb);
        __syncthreads();
        rows_from_stage<G>(T, wid, v, 0);
        __syncthreads();
        put_colhalf(T, wid, qb);
    }
    __syncthreads();
    rows_from_stage<G>(T, wid, v, H / 2);
}

// ---- inverse columns through the row-half stage: column 2 cc + G; CR 0: even
// coefficient rows -> DCT-III_128 (a), CR 1: odd coefficient rows -> DCT-IV_128 (b).
// Four barriers, as rows_fwd.
template <int G, int CR>
__device__ __forceinline__ void cols_inv(const gfloat* src, float* T, int wid, float (&R)[H], twptr tw)
{
    float v[H];
    {
        float qa[64], qb[64];
        load_rowhalf<0>(src, wid, qa);
        __syncthreads();
        put_rowhalf(T, wid, qa);
        load_rowhalf<1>(src, wid, qb); // as in rows_fwd: half an array in flight at a time
        __syncthreads();
        int c = lane_t(wid) & 127;
#pragma unroll
        for (int k = 0; k < H / 2; ++k) {
            v[k] = T[(2 * k + CR) * RP + 2 * c + G];
            if (k % 32 == 31) after(c, v[k]);
        }
        __syncthreads();
        put_rowhalf(T, wid, qb);
        __syncthreads();
    }
    int c = lane_t(wid) & 127;
#pragma unroll
    for (int k = H / 2; k < H; ++k) {
        v[k] = T[(2 * k + CR - H) * RP + 2 * c + G];
        if (k % 32 == 31) after(c, v[k]);
    }
    if constexpr (CR == 0) dct3_rec<L, H>(v, R, tw); else dct4_scaled<L, H>(v, R, tw);
    settle(R);
}

// Row i of the tile <- the thread's 128 values.
__device__ __forceinline__ void put_row(float* T, int wid, const float (&R)[H])
{
    const int i = lane_t(wid) & 255;
#pragma unroll
    for (int k = 0; k < H; ++k) T[i * P + k] = R[k];
}

// Forward transform of tile column cc (256 values down the tile rows): CR 0 -> even
// coefficients (DCT-II_128 of u), CR 1 -> odd coefficients (DCT-IV_128 of w).  In two
// parts, so that a group can read its column from the tile before a barrier and transform
// it after later ones (the transform's input is pinned after the barriers it must follow).
template <int CR>
__device__ __forceinline__ void col_fwd_read(const float* T, int wid, float (&v)[H])
{
    int cc = lane_t(wid) & 127;
#pragma unroll
    for (int n = 0; n < H; ++n) {
        const float xl = T[n * P + cc], xh = T[(L - 1 - n) * P + cc];
        v[n] = CR == 0 ? xl + xh : xl - xh;
        if (n % 32 == 31) after(cc, v[n]);
    }
}
template <int CR>
__device__ __forceinline__ void col_fwd_tf(float (&v)[H], float (&o)[H], twptr tw)
{
    settle(v);
    if constexpr (CR == 0) dct2_rec<L, H>(v, o, tw); else dct4_scaled<L, H>(v, o, tw);
    settle(o);
}
// Both parts in one phase (the transform may start while the last reads are in flight).
template <int CR>
__device__ __forceinline__ void col_fwd(const float* T, int wid, float (&o)[H], twptr tw)
{
    int cc = lane_t(wid) & 127;
    float v[H];
#pragma unroll
    for (int n = 0; n < H; ++n) {
        const float xl = T[n * P + cc], xh = T[(L - 1 - n) * P + cc];
        v[n] = CR == 0 ? xl + xh : xl - xh;
        if (n % 32 == 31) after(cc, v[n]);
    }
    if constexpr (CR == 0) dct2_rec<L, H>(v, o, tw); else dct4_scaled<L, H>(v, o, tw);
    settle(o);
}

// Inverse of the same column half: CR 0: DCT-III_128 of the even coefficients (a),
// CR 1: DCT-IV_128 of the odd coefficients (b).
template <int CR>
__device__ __forceinline__ void col_inv(const float (&o)[H], float (&R)[H], twptr tw)
{
    if constexpr (CR == 0) dct3_rec<L, H>(o, R, tw); else dct4_scaled<L, H>(o, R, tw);
    settle(R);
}

// Filter: coefficient row 2k + CR of array column 2 cc + G times its multiplier.
template <int G, int CR>
__device__ __forceinline__ void scale_col(float (&o)[H], const gfloat* lam, int wid)
{
    scale_coefs<H, 2 * L, 32>(o, lam, CR * L + 2 * (lane_t(wid) & 127) + G);
    settle(o);
}

// Column halves into the tile: rows 0..127 hold a, rows 128..255 hold b (column cc).
template <int CR>
__device__ __forceinline__ void put_halves(float* T, int wid, const float (&R)[H])
{
    const int cc = lane_t(wid) & 127;
#pragma unroll
    for (int n = 0; n < H; ++n) T[(CR * H + n) * P + cc] = R[n];
}

// Inverse transform of the entries of row i held in the tile as column halves:
// Z[i][.] = a[r] + b[r] (i < 128, r = i) or a[r] - b[r] (r = 255 - i).  Group 0 has
// the even entries (DCT-III_128), group 1 the odd entries (DCT-IV_128).
// (In two parts, like col_fwd.)
template <int G>
__device__ __forceinline__ void row_inv_read(const float* T, int wid, float (&o)[H])
{
    const int i = lane_t(wid) & 255;
    const bool top = i < H;
    int r = top ? i : L - 1 - i;
    const float sg = top ? 1.f : -1.f; // exact: one rounding, as a +- b
#pragma unroll
    for (int c = 0; c < H; ++c) {
        o[c] = __builtin_fmaf(sg, T[(H + r) * P + c], T[r * P + c]);
        if (c % 32 == 31) after(r, o[c]);
    }
}
template <int G>
__device__ __forceinline__ void row_inv_tf(float (&o)[H], float (&R)[H], twptr tw)
{
    settle(o);
    if constexpr (G == 0) dct3_rec<L, H>(o, R, tw); else dct4_scaled<L, H>(o, R, tw);
    settle(R);
}
template <int G>
__device__ __forceinline__ void row_inv(const float* T, int wid, float (&R)[H], twptr tw)
{
    const int i = lane_t(wid) & 255;
    const bool top = i < H;
    int r = top ? i : L - 1 - i;
    const float sg = top ? 1.f : -1.f; // exact: one rounding, as a +- b
    float o[H];
#pragma unroll
    for (int c = 0; c < H; ++c) {
        o[c] = __builtin_fmaf(sg, T[(H + r) * P + c], T[r * P + c]);
        if (c % 32 == 31) after(r, o[c]);
    }
    if constexpr (G == 0) dct3_rec<L, H>(o, R, tw); else dct4_scaled<L, H>(o, R, tw);
    settle(R);
}

// ---- forward output: coefficient rows 2k + CR (k in half HF of 0..127) of column
// 2 cc + G into the row-half stage, then out.  Four barriers with the stage windows.
template <int G, int CR>
__device__ __forceinline__ void coefs_out(gfloat* dst, float* T, int wid, const float (&o)[H])
{
    {
        const int c = lane_t(wid) & 127;
#pragma unroll
        for (int k = 0; k < H / 2; ++k) T[(2 * k + CR) * RP + 2 * c + G] = o[k];
    }
    __syncthreads();
    out_rowhalf<0>(dst, T, wid);
    __syncthreads();
    {
        const int c = lane_t(wid) & 127;
#pragma unroll
        for (int k = H / 2; k < H; ++k) T[(2 * k + CR - H) * RP + 2 * c + G] = o[k];
    }
    __syncthreads();
    out_rowhalf<1>(dst, T, wid);
}

// ---- inverse output by column halves: x[i][m] = p[m] + q[m], x[i][255-m] = p[m] -
// q[m], m < 64 through the outer half, 64 <= m < 128 through the inner half (stage
// columns m mod 64 and 127 - m mod 64); group 0 writes p into both places, then group 1
// adds and subtracts q.  Five barriers.
template <int G>
__device__ __forceinline__ void rows_out(gfloat* dst, float* T, int wid, const float (&R)[H])
{
#pragma unroll
    for (int hf = 0; hf < 2; ++hf) {
        const int r = lane_t(wid) & 255;
        const int m0 = hf * (H / 2);
        if (G == 0) {
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const float* p = &R[m0 + 4 * j];
                *reinterpret_cast<float4*>(&T[r * CP + 4 * j]) = make_float4(p[0], p[1], p[2], p[3]);
                *reinterpret_cast<float4*>(&T[r * CP + H - 4 - 4 * j]) = make_float4(p[3], p[2], p[1], p[0]);
            }
        }
        __syncthreads();
        if (G == 1) {
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const float* q = &R[m0 + 4 * j];
                float4* lo = reinterpret_cast<float4*>(&T[r * CP + 4 * j]);
                float4* hi = reinterpret_cast<float4*>(&T[r * CP + H - 4 - 4 * j]);
                float4 a = *lo, b = *hi;
                a.x += q[0]; a.y += q[1]; a.z += q[2]; a.w += q[3];
                b.w -= q[0]; b.z -= q[1]; b.y -= q[2]; b.x -= q[3];
                *lo = a;
                *hi = b;
            }
        }
        __syncthreads();
        if (hf == 0) out_colhalf<0>(dst, T, wid); else out_colhalf<1>(dst, T, wid);
        if (hf == 0) __syncthreads();
    }
}

// One (group, column half) path of one array.
template <int DIR, int G, int CR>
__device__ __forceinline__ void path(const gfloat* src, gfloat* dst, float* T, int wid, twptr tw, const gfloat* lam)
{
    float R[H];
    if constexpr (DIR == DCT2D_FORWARD) {
        rows_fwd<G>(src, T, wid, R, tw);
        float o[H];
        tw_fence(tw);
        if constexpr (G == 0) {
            __syncthreads(); // stage reads done
            put_row(T, wid, R);
            __syncthreads();
            {
                // the columns are read now and transformed beside round O's column
                // transforms (after its rows are in the tile), where this group would
                // otherwise wait
                float v[H];
                col_fwd_read<CR>(T, wid, v);
                syncs(2); // round O: its rows into the tile
                col_fwd_tf<CR>(v, o, tw);
            }
            __syncthreads(); // round O
        } else {
            syncs(3); // round E
            put_row(T, wid, R);
            __syncthreads();
            col_fwd<CR>(T, wid, o, tw);
            __syncthreads();
        }
        coefs_out<G, CR>(dst, T, wid, o);
    } else {
        if constexpr (DIR == DCT2D_INVERSE) {
            cols_inv<G, CR>(src, T, wid, R, tw);
            tw_fence(tw);
            if constexpr (G == 0) {
                __syncthreads();
                put_halves<CR>(T, wid, R);
                __syncthreads();
                {
                    // p: the entries are read now and transformed beside round O's rows
                    float o[H];
                    row_inv_read<0>(T, wid, o);
                    syncs(2); // round O: its halves into the tile
                    row_inv_tf<0>(o, R, tw);
                }
                __syncthreads(); // round O
            } else {
                syncs(3); // round E
                put_halves<CR>(T, wid, R);
                __syncthreads();
                row_inv<1>(T, wid, R, tw); // q
                __syncthreads();
            }
        } else {
            if constexpr (G == 0) {
                rows_fwd<G>(src, T, wid, R, tw);
                tw_fence(tw);
                __syncthreads();
                put_row(T, wid, R);
                __syncthreads();
                {
                    float o[H];
                    col_fwd<CR>(T, wid, o, tw);
                    if constexpr (DIR == DIR_FILTER) scale_col<G, CR>(o, lam, wid);
                    tw_fence(tw);
                    col_inv<CR>(o, R, tw);
                }
                __syncthreads();
                put_halves<CR>(T, wid, R);
                __syncthreads();
                {
                    // p: the entries are read now and transformed beside round O's column
                    // transforms, where this group would otherwise wait
                    float o[H];
                    row_inv_read<0>(T, wid, o);
                    syncs(2); // round O: its rows into the tile
                    row_inv_tf<0>(o, R, tw);
                }
                syncs(3); // round O
            } else {
                {
                    // the row transform runs during round E's column phase, where this group
                    // would otherwise wait, instead of beside group E's row transform
                    float v[H];
                    rows_fwd_stage<G>(src, T, wid, v);
                    syncs(2); // round E: stage reads done, its rows into the tile
                    settle(v);
                    dct4_scaled<L, H>(v, R, tw);
                    settle(R);
                }
                tw_fence(tw);
                syncs(3); // round E
                put_row(T, wid, R);
                __syncthreads();
                {
                    float o[H];
                    col_fwd<CR>(T, wid, o, tw);
                    if constexpr (DIR == DIR_FILTER) scale_col<G, CR>(o, lam, wid);
                    tw_fence(tw);
                    col_inv<CR>(o, R, tw);
                }
                __syncthreads();
                put_halves<CR>(T, wid, R);
                __syncthreads();
                row_inv<1>(T, wid, R, tw); // q
                __syncthreads();
            }
        }
        rows_out<G>(dst, T, wid, R);
    }
}
} // namespace s256

// `stagger`: workgroups of the second cohort (every other one on each XCD) first idle for
// about stagger x 8k cycles, so that the two cohorts' HBM phases (the array in, the
// array out) fall into each other's compute phases instead of coinciding on every CU.
template <int DIR>
__global__ void __launch_bounds__(512, 1)
k_split256(Addr a, int64_t batch, const float2* __restrict__ tw_in, int stagger)
{
    using namespace s256;
    __shared__ float4 T4[LDS_FLOATS / 4];
    float* const T = reinterpret_cast<float*>(T4);
    if ((blockIdx.x >> 3) & 1)
        for (int k = 0; k < stagger; ++k) __builtin_amdgcn_s_sleep(127);
    // wavefront index w: group w / 4 (E, O), column half (w / 2) % 2; thread t = 64 w + lane,
    // row of the row phases t % 256, column slot of the column phases t % 128 (column
    // 2 (t % 128) + group)
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int g = wid >> 2, cr = (wid >> 1) & 1;
    for (int64_t blk = blockIdx.x; blk < batch; blk += gridDim.x) {
        const twptr tw = per_iteration(tw_in);
        const gfloat* src = uniform_ptr(a.src(blk));
        gfloat* dst = uniform_ptr(a.dst(blk));
        const gfloat* lam = DIR == DIR_FILTER ? uniform_ptr(a.lam_for(blk)) : nullptr;
        if (g == 0) {
            if (cr == 0) path<DIR, 0, 0>(src, dst, T, wid, tw, lam);
            else path<DIR, 0, 1>(src, dst, T, wid, tw, lam);
        } else {
            if (cr == 0) path<DIR, 1, 0>(src, dst, T, wid, tw, lam);
            else path<DIR, 1, 1>(src, dst, T, wid, tw, lam);
        }
    }
}

// Row pass over HBM: one thread per row of length L (rows of `rows` per array).
template <int L, int DIR>
__global__ void __launch_bounds__(64)
k_rows(Addr a, int64_t batch, int32_t rows, const float2* __restrict__ tw_in)
{
    const twptr tw = (twptr)tw_in;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= batch * rows) return;
    const int64_t b = g / rows;
    const int r = (int)(g % rows);
    const gfloat* src = a.src(b) + (int64_t)r * L;
    gfloat* dst = a.dst(b) + (int64_t)r * L;
    float v[L];
#pragma unroll
    for (int j = 0; j < L / 4; ++j) {
        const float4 q = *reinterpret_cast<const gfloat4*>(src + 4 * j);
        v[4 * j] = q.x; v[4 * j + 1] = q.y; v[4 * j + 2] = q.z; v[4 * j + 3] = q.w;
    }
    apply1d<L, DIR>(v, tw);
#pragma unroll
    for (int j = 0; j < L / 4; ++j)
        *reinterpret_cast<gfloat4*>(dst + 4 * j) = make_float4(v[4 * j], v[4 * j + 1], v[4 * j + 2], v[4 * j + 3]);
}

// Column pass over HBM: one thread per column of length L; consecutive lanes take
// consecutive columns, so every load/store instruction is contiguous across the wave.
template <int L, int DIR>
__global__ void __launch_bounds__(64)
k_cols(Addr a, int64_t batch, int32_t cols, const float2* __restrict__ tw_in)
{
    const twptr tw = (twptr)tw_in;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= batch * cols) return;
    const int64_t b = g / cols;
    const int c = (int)(g % cols);
    const gfloat* src = a.src(b) + c;
    gfloat* dst = a.dst(b) + c;
    float v[L];
#pragma unroll
    for (int r = 0; r < L; ++r) v[r] = src[(int64_t)r * cols];
    if constexpr (DIR == DIR_FILTER)
        filter1d<L>(v, a.lam_for(b) + c, cols, tw);
    else
        apply1d<L, DIR>(v, tw);
#pragma unroll
    for (int r = 0; r < L; ++r) dst[(int64_t)r * cols] = v[r];
}

template <int H, int W>
int launch_fused_hw(const DeviceTables* t, const Job& j)
{
    using C = B2D<H, W>;
    const int64_t ntiles = (j.batch + C::BPW - 1) / C::BPW;
    int per_cu = 0;
    const float2* twh = tw_for(t, H);
    const float2* tww = tw_for(t, W);
    hipError_t e = hipSuccess;
    switch (j.dir) {
    case DCT2D_FORWARD:
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_fused<H, W, DCT2D_FORWARD>, C::NT, 0);
        break;
    case DCT2D_INVERSE:
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_fused<H, W, DCT2D_INVERSE>, C::NT, 0);
        break;
    case DIR_FILTER:
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_fused<H, W, DIR_FILTER>, C::NT, 0);
        break;
    default:
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_fused<H, W, DCT2D_ROUNDTRIP>, C::NT, 0);
        break;
    }
    if (e != hipSuccess || per_cu < 1) per_cu = 1;
    const int64_t cap = (int64_t)t->num_cu * per_cu * 4;
    const unsigned grid = (unsigned)(ntiles < cap ? ntiles : cap);
    switch (j.dir) {
    case DCT2D_FORWARD:
        k_fused<H, W, DCT2D_FORWARD><<<grid, C::NT, 0, j.stream>>>(j.addr(), j.batch, twh, tww);
        break;
    case DCT2D_INVERSE:
        k_fused<H, W, DCT2D_INVERSE><<<grid, C::NT, 0, j.stream>>>(j.addr(), j.batch, twh, tww);
        break;
    case DIR_FILTER:
        k_fused<H, W, DIR_FILTER><<<grid, C::NT, 0, j.stream>>>(j.addr(), j.batch, twh, tww);
        break;
    default:
        k_fused<H, W, DCT2D_ROUNDTRIP><<<grid, C::NT, 0, j.stream>>>(j.addr(), j.batch, twh, tww);
        break;
    }
    return hipGetLastError() == hipSuccess ? DCT2D_OK : DCT2D_ERR_HIP;
}

// Workgroups per CU that the occupancy-capped wave variants allow (5 + 2 k and 6 + 2 k use
// cap k).  Fewer resident tiles keep fewer bytes in flight per CU; on MI355X a plain
// in-place tile copy through LDS moves 6.1 TB/s with about 40 KB in flight per CU and
// 5.4 TB/s with 160 KB, so the cap is a tuning dimension of its own.
constexpr int kWaveCaps[4] = {16, 10, 6, 4};

template <int H, int W, int DIR, bool STAGE>
int launch_wave_dir(const DeviceTables* t, const Job& j)
{
    using C = WaveCfg<H, W>;
    const int64_t ntiles = (j.batch + C::BPW - 1) / C::BPW;
    int64_t cap;
    size_t reserve = 0; // dynamic LDS that only limits residency
    if (j.variant >= 3) {
        cap = (int64_t)1 << 30; // one tile per workgroup (no grid-stride reuse)
        if (j.variant >= 5) {
            const size_t per_wg = (size_t)(160 * 1024 / kWaveCaps[(j.variant - 5) >> 1]) & ~(size_t)255;
            const size_t have = sizeof(float) * ((C::LDS_FLOATS + 3) / 4 * 4);
            reserve = per_wg > have ? per_wg - have : 0;
        }
    } else {
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_wave<H, W, DIR, STAGE>, 64, 0) != hipSuccess ||
            per_cu < 1)
            per_cu = 1;
        cap = (int64_t)t->num_cu * per_cu * 4;
    }
    const unsigned grid = (unsigned)(ntiles < cap ? ntiles : cap);
    k_wave<H, W, DIR, STAGE><<<grid, 64, reserve, j.stream>>>(j.addr(), j.batch, tw_for(t, H), tw_for(t, W));
    return hipGetLastError() == hipSuccess ? DCT2D_OK : DCT2D_ERR_HIP;
}

template <int H, int W, bool STAGE>
int launch_wave_stage(const DeviceTables* t, const Job& j)
{
    switch (j.dir) {
    case DCT2D_FORWARD: return launch_wave_dir<H, W, DCT2D_FORWARD, STAGE>(t, j);
    case DCT2D_INVERSE: return launch_wave_dir<H, W, DCT2D_INVERSE, STAGE>(t, j);
    case DIR_FILTER: return launch_wave_dir<H, W, DIR_FILTER, STAGE>(t, j);
    default: return launch_wave_dir<H, W, DCT2D_ROUNDTRIP, STAGE>(t, j);
    }
}

template <int H, int W>
int launch_wave_hw(const DeviceTables* t, const Job& j)
{
    const bool stage = j.variant == 4 || (j.variant >= 5 && ((j.variant - 5) & 1));
    return stage ? launch_wave_stage<H, W, true>(t, j) : launch_wave_stage<H, W, false>(t, j);
}

template <int H>
int wave_w(const DeviceTables* t, const Job& j)
{
    switch (j.cols) {
    case 8: return launch_wave_hw<H, 8>(t, j);
    case 16: return launch_wave_hw<H, 16>(t, j);
    case 32: return launch_wave_hw<H, 32>(t, j);
    case 64: return launch_wave_hw<H, 64>(t, j);
    default: return DCT2D_ERR_SIZE;
    }
}

int launch_wave(const DeviceTables* t, const Job& j)
{
    switch (j.rows) {
    case 8: return wave_w<8>(t, j);
    case 16: return wave_w<16>(t, j);
    case 32: return wave_w<32>(t, j);
    case 64: return wave_w<64>(t, j);
    default: return DCT2D_ERR_SIZE;
    }
}

template <int DIR, bool STAGE>
int launch_split128_dir(const DeviceTables* t, const Job& j)
{
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_split128<DIR, STAGE>, 256, 0) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    // variants 4, 5: one array per workgroup; 0, 3: a grid-stride loop over 4 x the
    // resident workgroups
    const int64_t cap = j.variant >= 4 ? ((int64_t)1 << 31) - 1 : (int64_t)t->num_cu * per_cu * 4;
    const unsigned grid = (unsigned)(j.batch < cap ? j.batch : cap);
    k_split128<DIR, STAGE><<<grid, 256, 0, j.stream>>>(j.addr(), j.batch, tw_for(t, 128));
    return hipGetLastError() == hipSuccess ? DCT2D_OK : DCT2D_ERR_HIP;
}

int launch_split128(const DeviceTables* t, const Job& j, bool stage)
{
    switch (j.dir) {
    case DCT2D_FORWARD:
        return stage ? launch_split128_dir<DCT2D_FORWARD, true>(t, j) : launch_split128_dir<DCT2D_FORWARD, false>(t, j);
    case DCT2D_INVERSE:
        return stage ? launch_split128_dir<DCT2D_INVERSE, true>(t, j) : launch_split128_dir<DCT2D_INVERSE, false>(t, j);
    case DIR_FILTER:
        return stage ? launch_split128_dir<DIR_FILTER, true>(t, j) : launch_split128_dir<DIR_FILTER, false>(t, j);
    default:
        return stage ? launch_split128_dir<DCT2D_ROUNDTRIP, true>(t, j)
                     : launch_split128_dir<DCT2D_ROUNDTRIP, false>(t, j);
    }
}

template <int DIR>
int launch_split64_dir(const DeviceTables* t, const Job& j)
{
    // one array per workgroup; variants 14, 15 cap the resident workgroups per CU at 6, 4
    // (an LDS reservation, as for the wave-local kernels)
    const unsigned grid = (unsigned)(j.batch < (((int64_t)1 << 31) - 1) ? j.batch : (((int64_t)1 << 31) - 1));
    const size_t tile = 64 * 64 * sizeof(float);
    const size_t per_wg = j.variant >= 14 ? (size_t)(160 * 1024 / (j.variant == 14 ? 6 : 4)) & ~(size_t)255 : tile;
    const size_t reserve = per_wg > tile ? per_wg - tile : 0;
    k_split64<DIR><<<grid, 128, reserve, j.stream>>>(j.addr(), j.batch, tw_for(t, 64));
    return hipGetLastError() == hipSuccess ? DCT2D_OK : DCT2D_ERR_HIP;
}

int launch_split64(const DeviceTables* t, const Job& j)
{
    switch (j.dir) {
    case DCT2D_FORWARD: return launch_split64_dir<DCT2D_FORWARD>(t, j);
    case DCT2D_INVERSE: return launch_split64_dir<DCT2D_INVERSE>(t, j);
    case DIR_FILTER: return launch_split64_dir<DIR_FILTER>(t, j);
    default: return launch_split64_dir<DCT2D_ROUNDTRIP>(t, j);
    }
}

template <int DIR>
int launch_split256_dir(const DeviceTables* t, const Job& j)
{
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_split256<DIR>, 512, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    // variant 0: one resident workgroup per CU looping over arrays; 2: one array per
    // workgroup; 3, 4: as 0 with the second cohort started about 3 x 8k / 6 x 8k cycles late
    const int64_t cap = j.variant == 2 ? ((int64_t)1 << 31) - 1 : (int64_t)t->num_cu * per_cu;
    const unsigned grid = (unsigned)(j.batch < cap ? j.batch : cap);
    const int stagger = j.variant == 3 ? 3 : j.variant == 4 ? 6 : 0;
    k_split256<DIR><<<grid, 512, 0, j.stream>>>(j.addr(), j.batch, tw_for(t, 256), stagger);
    return hipGetLastError() == hipSuccess ? DCT2D_OK : DCT2D_ERR_HIP;
}

int launch_split256(const DeviceTables* t, const Job& j)
{
    switch (j.dir) {
    case DCT2D_FORWARD: return launch_split256_dir<DCT2D_FORWARD>(t, j);
    case DCT2D_INVERSE: return launch_split256_dir<DCT2D_INVERSE>(t, j);
    case DIR_FILTER: return launch_split256_dir<DIR_FILTER>(t, j);
    default: return launch_split256_dir<DCT2D_ROUNDTRIP>(t, j);
    }
}

template <int L, int DIR>
void launch_rows(const DeviceTables* t, const Addr& a, int64_t batch, int rows, hipStream_t s)
{
    const int64_t n = batch * rows;
    k_rows<L, DIR><<<(unsigned)((n + 63) / 64), 64, 0, s>>>(a, batch, rows, tw_for(t, L));
}

template <int L, int DIR>
void launch_cols(const DeviceTables* t, const Addr& a, int64_t batch, int cols, hipStream_t s)
{
    const int64_t n = batch * cols;
    k_cols<L, DIR><<<(unsigned)((n + 63) / 64), 64, 0, s>>>(a, batch, cols, tw_for(t, L));
}

// Row pass with length `len` (runtime) -> template dispatch.
template <int DIR>
int rows_any(const DeviceTables* t, int len, const Addr& a, int64_t batch, int rows, hipStream_t s)
{
    switch (len) {
    case 8: launch_rows<8, DIR>(t, a, batch, rows, s); break;
    case 16: launch_rows<16, DIR>(t, a, batch, rows, s); break;
    case 32: launch_rows<32, DIR>(t, a, batch, rows, s); break;
    case 64: launch_rows<64, DIR>(t, a, batch, rows, s); break;
    case 128: launch_rows<128, DIR>(t, a, batch, rows, s); break;
    case 256: launch_rows<256, DIR>(t, a, batch, rows, s); break;
    default: return DCT2D_ERR_SIZE;
    }
    return hipGetLastError() == hipSuccess ? DCT2D_OK : DCT2D_ERR_HIP;
}

template <int DIR>
int cols_any(const DeviceTables* t, int len, const Addr& a, int64_t batch, int cols, hipStream_t s)
{
    switch (len) {
    case 8: launch_cols<8, DIR>(t, a, batch, cols, s); break;
    case 16: launch_cols<16, DIR>(t, a, batch, cols, s); break;
    case 32: launch_cols<32, DIR>(t, a, batch, cols, s); break;
    case 64: launch_cols<64, DIR>(t, a, batch, cols, s); break;
    case 128: launch_cols<128, DIR>(t, a, batch, cols, s); break;
    case 256: launch_cols<256, DIR>(t, a, batch, cols, s); break;
    default: return DCT2D_ERR_SIZE;
    }
    return hipGetLastError() == hipSuccess ? DCT2D_OK : DCT2D_ERR_HIP;
}

} // namespace

int launch_short_line_pass(const DeviceTables* t, const Addr& a, int64_t batch, int len, int lines_per_array,
                           bool column_pass, int dir, hipStream_t s)
{
    switch (dir) {
    case DCT2D_FORWARD:
        return column_pass ? cols_any<DCT2D_FORWARD>(t, len, a, batch, lines_per_array, s)
                           : rows_any<DCT2D_FORWARD>(t, len, a, batch, lines_per_array, s);
    case DCT2D_INVERSE:
        return column_pass ? cols_any<DCT2D_INVERSE>(t, len, a, batch, lines_per_array, s)
                           : rows_any<DCT2D_INVERSE>(t, len, a, batch, lines_per_array, s);
    case DCT2D_ROUNDTRIP:
        return column_pass ? cols_any<DCT2D_ROUNDTRIP>(t, len, a, batch, lines_per_array, s)
                           : rows_any<DCT2D_ROUNDTRIP>(t, len, a, batch, lines_per_array, s);
    default:
        return DCT2D_ERR_ARG;
    }
}

namespace {

// Two-pass schedule over HBM (rows, then columns; the round trip needs a third pass).
// The first pass reads the input arrays and writes the output arrays; the later
// passes work in place on the output arrays.
int launch_two_pass(const DeviceTables* t, const Job& j)
{
    const Addr first = j.addr();
    const Addr inplace{j.out, j.out, j.out_stride, j.out_stride, j.out_idx, j.out_idx, j.out_slot, j.out_slot,
                       j.lam, j.lam_stride};
    int rc;
    switch (j.dir) {
    case DCT2D_FORWARD:
        rc = rows_any<DCT2D_FORWARD>(t, j.cols, first, j.batch, j.rows, j.stream);
        if (rc) return rc;
        return cols_any<DCT2D_FORWARD>(t, j.rows, inplace, j.batch, j.cols, j.stream);
    case DCT2D_INVERSE:
        rc = rows_any<DCT2D_INVERSE>(t, j.cols, first, j.batch, j.rows, j.stream);
        if (rc) return rc;
        return cols_any<DCT2D_INVERSE>(t, j.rows, inplace, j.batch, j.cols, j.stream);
    default:
        rc = rows_any<DCT2D_FORWARD>(t, j.cols, first, j.batch, j.rows, j.stream);
        if (rc) return rc;
        rc = j.dir == DIR_FILTER ? cols_any<DIR_FILTER>(t, j.rows, inplace, j.batch, j.cols, j.stream)
                                 : cols_any<DCT2D_ROUNDTRIP>(t, j.rows, inplace, j.batch, j.cols, j.stream);
        if (rc) return rc;
        return rows_any<DCT2D_INVERSE>(t, j.cols, inplace, j.batch, j.rows, j.stream);
    }
}

template <int H>
int fused_w(const DeviceTables* t, const Job& j)
{
    switch (j.cols) {
    case 8: return launch_fused_hw<H, 8>(t, j);
    case 16: return launch_fused_hw<H, 16>(t, j);
    case 32: return launch_fused_hw<H, 32>(t, j);
    case 64: return launch_fused_hw<H, 64>(t, j);
    case 128: return launch_fused_hw<H, 128>(t, j);
    default: return DCT2D_ERR_SIZE;
    }
}

int launch_fused(const DeviceTables* t, const Job& j)
{
    switch (j.rows) {
    case 8: return fused_w<8>(t, j);
    case 16: return fused_w<16>(t, j);
    case 32: return fused_w<32>(t, j);
    case 64: return fused_w<64>(t, j);
    case 128: return fused_w<128>(t, j);
    default: return DCT2D_ERR_SIZE;
    }
}

} // namespace

// Variants (frozen per size by the policy table / autotuner):
//   both axes <= 64:  0 wave-local fused, 1 LDS-staged fused, 2 two-pass,
//                     3 wave-local fused with one tile per workgroup, 4 as 3 with the
//                     tile staged through LDS by coalesced 16-byte loads and stores,
//                     5..12 as 3 (odd) or 4 (even) with at most 16, 10, 6, 4 resident
//                     workgroups per CU; 64 x 64 only: 13 split fused (two wavefronts per
//                     transform, one array per workgroup), 14, 15 as 13 with at most 6, 4
//                     resident workgroups per CU
//   128 x 128:        0 split fused (two wavefronts per transform), 1 LDS-staged fused, 2 two-pass,
//                     3 split fused with the rows (inverse: columns) read through an LDS copy
//                     of the array, 4 and 5 as 3 and 0 with one array per workgroup
//   other axes <=128: 0 LDS-staged fused, 1 two-pass
//   256 x 256:        0 split fused (two groups of wavefronts, two LDS rounds), one
//                     resident workgroup per CU; 1 two-pass; 2 split fused, one array
//                     per workgroup; 3, 4 as 0 with the two cohorts of CUs staggered
//   one axis of 256, the other <= 128: 0 fused (k_rect256: the tile in LDS, the length-256
//                     transforms shared by four wavefront roles), one tile per workgroup;
//                     1 two-pass; 2 as 0 with resident workgroups looping over the tiles;
//                     3 (short axis <= 64) k_rect256_db: one persistent workgroup per CU, two
//                     tile buffers filled by LDS DMA while the other is transformed
int fp32_variant_count(int rows, int cols, int)
{
    if (rows == 64 && cols == 64) return 16;
    if (rows <= 64 && cols <= 64) return 13;
    if (rows == 128 && cols == 128) return 6;
    if (rows <= 128 && cols <= 128) return 2;
    if (rows == 256 && cols == 256) return 5;
    return (rows == 256 ? cols : rows) <= 64 ? 4 : 3; // variant 3: short axis <= 64 only
}

// Variant used until the tuner measures otherwise (fastest in measurements on MI355X
// with 512 MiB batches), by the longer axis of arrays up to 64 x 64: 8 staged; 16 staged
// with at most 16 workgroups per CU; 32 at most 10 per CU, staged for the round trip;
// 64 x 64 the two-wavefront split kernel, with at most 4 workgroups per CU for forward and
// inverse.  Rectangles with a longer axis of 32: staged, at most 16 per CU; of 64: staged,
// uncapped (a short axis leaves most lanes of one pass idle, so more resident tiles pay).  The staged split kernel for 128 x 128 with one array per workgroup, the split
// kernel for 256 x 256 with its two cohorts of CUs staggered by about 6 x 8k cycles.
int fp32_default_variant(int rows, int cols, int dir)
{
    if (rows <= 64 && cols <= 64) {
        const int m = rows > cols ? rows : cols;
        const bool rt = dir == DCT2D_ROUNDTRIP;
        if (rows == 64 && cols == 64) return rt ? 13 : 15;
        if (rows != cols && m >= 32) return m == 32 ? 6 : 4;
        return m <= 8 ? 4 : m <= 16 ? 6 : m <= 32 ? (rt ? 8 : 7) : (rt ? 4 : 12);
    }
    if (rows == 128 && cols == 128) return 4;
    if (rows == 256 && cols == 256) return 4;
    if ((rows == 256) != (cols == 256)) {
        // measured on 512 MiB batches: the double-buffered kernel wherever it leads
        const bool wide = cols == 256;
        const int s = wide ? rows : cols;
        if (s == 128) return dir == DCT2D_FORWARD ? 1 : wide ? 0 : 2;
        if (dir != DCT2D_ROUNDTRIP) return 3;
        return wide || s >= 32 ? 0 : 3; // the round trip's arithmetic wants two workgroups per CU
    }
    return 0;
}

// The same kernel family with one tile (array) per workgroup in place of a grid-stride
// loop, for launches that share the GPU with other kernels (the classes of a ragged plan
// run as concurrent graph branches): a grid-stride schedule fixes each workgroup's share
// of the batch, so such a launch ends only when its last-started workgroup does.  On the
// ragged configuration (200k blocks and 8 images) the 256 x 256 class took the batch from
// 0.96 to 0.89 ms.
int fp32_unshared_variant(int rows, int cols, int v)
{
    if (rows <= 64 && cols <= 64) return v == 0 ? 3 : v;
    if (rows == 128 && cols == 128) return v == 0 ? 5 : v == 3 ? 4 : v;
    if (rows == 256 && cols == 256) return v == 0 || v == 3 || v == 4 ? 2 : v;
    if ((rows == 256) != (cols == 256)) return v == 2 || v == 3 ? 0 : v;
    return v;
}

int launch_fp32(const DeviceTables* t, const Job& j)
{
    if (j.rows <= 64 && j.cols <= 64) {
        if (j.variant >= 13) return launch_split64(t, j);
        if (j.variant == 0 || j.variant >= 3) return launch_wave(t, j);
        if (j.variant == 1) return launch_fused(t, j);
        return launch_two_pass(t, j);
    }
    if (j.rows == 128 && j.cols == 128) {
        if (j.variant == 0 || j.variant >= 3) return launch_split128(t, j, j.variant == 3 || j.variant == 4);
        if (j.variant == 1) return launch_fused(t, j);
        return launch_two_pass(t, j);
    }
    if (j.rows <= 128 && j.cols <= 128 && j.variant == 0) return launch_fused(t, j);
    if (j.rows == 256 && j.cols == 256 && j.variant != 1) return launch_split256(t, j);
    if ((j.rows == 256) != (j.cols == 256) && j.variant != 1) return launch_rect256(t, j);
    return launch_two_pass(t, j);
}

} // namespace dct
