// Dense axis passes for whole images: one 1D transform of length L applied along the
// rows or the columns of a batch of h x w images by a float32 matrix product with the
// dense Q_L of eq. 1 (Section 2.1; rectangles and arbitrary axes, Section 7.1).  Used
// for the image axes of ragged batches (1024, 512 and the non-power-of-two 384, which
// the fast transforms do not cover; zero-padding would change the transform).
//
//   column pass   Y = Q_h X      (forward)    Y = Q_h^T X   (inverse)
//   row pass      Y = X Q_w^T    (forward)    Y = X Q_w     (inverse)
//
// Tiled product: a 256-thread workgroup computes a 64 x 64 output tile over K in chunks
// of 16 staged in LDS.  The 16 products of a chunk are summed in a fresh partial that is
// then added to the running sum (blocked summation), which keeps the float32
// accumulation error near 4 unit roundoffs per pass at L = 1024 instead of growing like
// sqrt(L/6).  The even/odd form (axes divisible by 8: every image axis of the workloads)
// runs the products on the matrix cores in float32; the plain form, for other axes,
// gives each thread a 4 x 4 micro-tile on the vector ALU.
#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace dct {
namespace {

constexpr int BM = 64, BN = 64, BK = 16;
typedef float f32x16 __attribute__((ext_vector_type(16)));

// Generic strided operand: element (i, k) at p[i * si + k * sk].
struct Mat {
    const gfloat* p;
    int64_t si, sk;
};

// C[i][j] = sum_k A(i,k) B(k,j) for one batch item per blockIdx.z.  Exactly one of A and B
// is the image (indexed through `a`, item z); the other is the shared Q.  `img_is_a`
// selects which.  The output goes to a.dst(z) with row pitch ldc.
__global__ void __launch_bounds__(256)
k_dense_pass(Addr a, bool img_is_a, Mat qm, int64_t img_si, int64_t img_sk, int M, int N, int K, int64_t ldc)
{
    __shared__ __attribute__((aligned(16))) float As[BK][BM + 4];
    __shared__ __attribute__((aligned(16))) float Bs[BK][BN + 4];
    const int t = threadIdx.x;
    const int z = blockIdx.z;
    const gfloat* img = a.src(z);
    gfloat* dst = a.dst(z);
    const Mat A = img_is_a ? Mat{img, img_si, img_sk} : qm;
    const Mat B = img_is_a ? qm : Mat{img, img_si, img_sk}; // B(k, j) = B.p[k * B.si + j * B.sk]
    const int i0 = blockIdx.y * BM, j0 = blockIdx.x * BN;
    const int ti = (t / 16) * 4, tj = (t % 16) * 4;
    float acc[4][4] = {};
    // load mapping: the index with unit stride varies fastest across threads
    const bool a_k_fast = A.sk == 1;
    const bool b_j_fast = B.sk == 1;
    for (int k0 = 0; k0 < K; k0 += BK) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = t + 256 * q;
            int i, k;
            if (a_k_fast) { k = e % BK; i = e / BK; } else { i = e % BM; k = e / BM; }
            const int gi = i0 + i, gk = k0 + k;
            As[k][i] = (gi < M && gk < K) ? A.p[(int64_t)gi * A.si + (int64_t)gk * A.sk] : 0.f;
            int j, kk;
            if (b_j_fast) { j = e % BN; kk = e / BN; } else { kk = e % BK; j = e / BK; }
            const int gj = j0 + j, gkk = k0 + kk;
            Bs[kk][j] = (gj < N && gkk < K) ? B.p[(int64_t)gkk * B.si + (int64_t)gj * B.sk] : 0.f;
        }
        __syncthreads();
        float part[4][4] = {};
#pragma unroll
        for (int k = 0; k < BK; ++k) {
            const float4 av = *reinterpret_cast<const float4*>(&As[k][ti]);
            const float4 bv = *reinterpret_cast<const float4*>(&Bs[k][tj]);
            const float ar[4] = {av.x, av.y, av.z, av.w};
            const float br[4] = {bv.x, bv.y, bv.z, bv.w};
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
                for (int y = 0; y < 4; ++y) part[x][y] = fmaf(ar[x], br[y], part[x][y]);
        }
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int y = 0; y < 4; ++y) acc[x][y] += part[x][y];
        __syncthreads();
    }
#pragma unroll
    for (int x = 0; x < 4; ++x) {
        const int gi = i0 + ti + x;
        if (gi >= M) continue;
#pragma unroll
        for (int y = 0; y < 4; ++y) {
            const int gj = j0 + tj + y;
            if (gj < N) dst[(int64_t)gi * ldc + gj] = acc[x][y];
        }
    }
}

// Even/odd form of the same pass for an even length L: Q_L's even rows are symmetric and
// its odd rows antisymmetric about the middle column (eq. 1), so
//   forward  Y[2k]   = sum_{n < L/2} Q_L[2k][n]   (x[n] + x[L-1-n])
//            Y[2k+1] = sum_{n < L/2} Q_L[2k+1][n] (x[n] - x[L-1-n])
//   inverse  a[n] = sum_{k < L/2} Q_L[2k][n] Y[2k],  b[n] = sum_{k < L/2} Q_L[2k+1][n] Y[2k+1],
//            x[n] = a[n] + b[n],  x[L-1-n] = a[n] - b[n]
// i.e. two products of half the depth (half the flops of the dense pass), with the
// butterflies fused into the operand loads (forward) or the stores (inverse).  A
// workgroup computes the 64 x 64 tiles of both products for the same output positions
// on the matrix cores in float32 (each wavefront a 32 x 32 sub-tile of each), over K in
// chunks of 16 with blocked summation.
// ROW: transform along the rows (length L = cols); else along the columns (L = rows).
// The source and destination never overlap (the ragged planner ping-pongs through its
// workspace).
// One chunk's operands as loaded from HBM, before the butterflies: u, v from the image,
// b1, b2 from Q_L (zeros outside the matrices).
struct EoRegs {
    float4 u, v, b1, b2;
};

template <bool ROW, bool INV>
__device__ __forceinline__ EoRegs eo_fetch(const gfloat* x, const gfloat* q, int rows, int cols, int L, int i0,
                                           int j0, int k0, int t)
{
    const int HL = L / 2;
    const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
    EoRegs r{z, z, z, z};
    if (ROW) {
        // image rows i0 + t / 4, depth k0 + 4 (t % 4) .. +3
        const int gi = i0 + t / 4, gk = k0 + 4 * (t % 4);
        if (gi < rows && gk < HL) {
            const gfloat* xr = x + (int64_t)gi * cols;
            if (!INV) {
                r.u = *reinterpret_cast<const gfloat4*>(xr + gk);          // x[gk .. gk+3]
                r.v = *reinterpret_cast<const gfloat4*>(xr + L - 4 - gk);  // x[L-1-gk-3 .. L-1-gk]
            } else {
                r.u = *reinterpret_cast<const gfloat4*>(xr + 2 * gk);      // Y[2gk .. 2gk+3]
                r.v = *reinterpret_cast<const gfloat4*>(xr + 2 * gk + 4);  // Y[2gk+4 .. 2gk+7]
            }
        }
        if (!INV) {
            const int gh = j0 + t / 4, gk2 = k0 + 4 * (t % 4);
            if (gh < HL && gk2 < HL) {
                r.b1 = *reinterpret_cast<const gfloat4*>(q + (int64_t)(2 * gh) * L + gk2);
                r.b2 = *reinterpret_cast<const gfloat4*>(q + (int64_t)(2 * gh + 1) * L + gk2);
            }
        } else {
            const int gk2 = k0 + t / 16, gh = j0 + 4 * (t % 16);
            if (gk2 < HL && gh < HL) {
                r.b1 = *reinterpret_cast<const gfloat4*>(q + (int64_t)(2 * gk2) * L + gh);
                r.b2 = *reinterpret_cast<const gfloat4*>(q + (int64_t)(2 * gk2 + 1) * L + gh);
            }
        }
    } else {
        if (!INV) {
            const int gh = i0 + t / 4, gk = k0 + 4 * (t % 4);
            if (gh < HL && gk < HL) {
                r.b1 = *reinterpret_cast<const gfloat4*>(q + (int64_t)(2 * gh) * L + gk);
                r.b2 = *reinterpret_cast<const gfloat4*>(q + (int64_t)(2 * gh + 1) * L + gk);
            }
        } else {
            const int gk = k0 + t / 16, gh = i0 + 4 * (t % 16);
            if (gk < HL && gh < HL) {
                r.b1 = *reinterpret_cast<const gfloat4*>(q + (int64_t)(2 * gk) * L + gh);
                r.b2 = *reinterpret_cast<const gfloat4*>(q + (int64_t)(2 * gk + 1) * L + gh);
            }
        }
        // image depth rows k0 + t / 16, columns j0 + 4 (t % 16) .. +3
        const int gk = k0 + t / 16, gj = j0 + 4 * (t % 16);
        if (gk < HL && gj < cols) {
            if (!INV) {
                r.u = *reinterpret_cast<const gfloat4*>(x + (int64_t)gk * cols + gj);
                r.v = *reinterpret_cast<const gfloat4*>(x + (int64_t)(L - 1 - gk) * cols + gj);
            } else {
                r.u = *reinterpret_cast<const gfloat4*>(x + (int64_t)(2 * gk) * cols + gj);
                r.v = *reinterpret_cast<const gfloat4*>(x + (int64_t)(2 * gk + 1) * cols + gj);
            }
        }
    }
    return r;
}

// The butterflies (forward) or the even/odd split (inverse) of the fetched chunk, into the
// LDS operand tiles: A (BM x BK, k-major), B (BK x BN).
template <bool ROW, bool INV>
__device__ __forceinline__ void eo_stage(const EoRegs& r, float (*A1)[BM + 4], float (*A2)[BM + 4],
                                         float (*B1)[BN + 4], float (*B2)[BN + 4], int t)
{
    float4 p1, p2;
    if (ROW) {
        if (!INV) {
            p1 = make_float4(r.u.x + r.v.w, r.u.y + r.v.z, r.u.z + r.v.y, r.u.w + r.v.x);
            p2 = make_float4(r.u.x - r.v.w, r.u.y - r.v.z, r.u.z - r.v.y, r.u.w - r.v.x);
        } else {
            p1 = make_float4(r.u.x, r.u.z, r.v.x, r.v.z);
            p2 = make_float4(r.u.y, r.u.w, r.v.y, r.v.w);
        }
        const int row = t / 4, c = 4 * (t % 4);
        A1[c][row] = p1.x; A1[c + 1][row] = p1.y; A1[c + 2][row] = p1.z; A1[c + 3][row] = p1.w;
        A2[c][row] = p2.x; A2[c + 1][row] = p2.y; A2[c + 2][row] = p2.z; A2[c + 3][row] = p2.w;
        if (!INV) {
            const int h = t / 4;
            B1[c][h] = r.b1.x; B1[c + 1][h] = r.b1.y; B1[c + 2][h] = r.b1.z; B1[c + 3][h] = r.b1.w;
            B2[c][h] = r.b2.x; B2[c + 1][h] = r.b2.y; B2[c + 2][h] = r.b2.z; B2[c + 3][h] = r.b2.w;
        } else {
            const int k = t / 16, cc = 4 * (t % 16);
            *reinterpret_cast<float4*>(&B1[k][cc]) = r.b1;
            *reinterpret_cast<float4*>(&B2[k][cc]) = r.b2;
        }
    } else {
        if (!INV) {
            const int h = t / 4, c = 4 * (t % 4);
            A1[c][h] = r.b1.x; A1[c + 1][h] = r.b1.y; A1[c + 2][h] = r.b1.z; A1[c + 3][h] = r.b1.w;
            A2[c][h] = r.b2.x; A2[c + 1][h] = r.b2.y; A2[c + 2][h] = r.b2.z; A2[c + 3][h] = r.b2.w;
            p1 = make_float4(r.u.x + r.v.x, r.u.y + r.v.y, r.u.z + r.v.z, r.u.w + r.v.w);
            p2 = make_float4(r.u.x - r.v.x, r.u.y - r.v.y, r.u.z - r.v.z, r.u.w - r.v.w);
        } else {
            const int k = t / 16, c = 4 * (t % 16);
            *reinterpret_cast<float4*>(&A1[k][c]) = r.b1;
            *reinterpret_cast<float4*>(&A2[k][c]) = r.b2;
            p1 = r.u;
            p2 = r.v;
        }
        const int k = t / 16, c = 4 * (t % 16);
        *reinterpret_cast<float4*>(&B1[k][c]) = p1;
        *reinterpret_cast<float4*>(&B2[k][c]) = p2;
    }
}

template <bool ROW, bool INV>
__global__ void __launch_bounds__(256)
k_dense_eo(Addr a, const float* __restrict__ q_in, int rows, int cols)
{
    __shared__ __attribute__((aligned(16))) float A1[BK][BM + 4];
    __shared__ __attribute__((aligned(16))) float A2[BK][BM + 4];
    __shared__ __attribute__((aligned(16))) float B1[BK][BN + 4];
    __shared__ __attribute__((aligned(16))) float B2[BK][BN + 4];
    const int t = threadIdx.x;
    const int z = blockIdx.z;
    const gfloat* x = a.src(z);
    gfloat* dst = a.dst(z);
    const gfloat* q = (const gfloat*)q_in;
    const int L = ROW ? cols : rows, HL = L / 2;
    // output tile of the half-size products: ROW: (image row i, half index h); column
    // pass: (half index h, image column j)
    const int i0 = blockIdx.y * BM, j0 = blockIdx.x * BN;
    const int M = ROW ? rows : HL, N = ROW ? HL : cols;
    const int lane = t & 63, wi = (t >> 6) >> 1, wj = (t >> 6) & 1;
    f32x16 acc1, acc2;
#pragma unroll
    for (int r = 0; r < 16; ++r) { acc1[r] = 0.f; acc2[r] = 0.f; }
    // software pipeline: the next chunk is fetched into registers while this one is
    // multiplied
    EoRegs nx = eo_fetch<ROW, INV>(x, q, rows, cols, L, i0, j0, 0, t);
    for (int k0 = 0; k0 < HL; k0 += BK) {
        eo_stage<ROW, INV>(nx, A1, A2, B1, B2, t);
        if (k0 + BK < HL) nx = eo_fetch<ROW, INV>(x, q, rows, cols, L, i0, j0, k0 + BK, t);
        __syncthreads();
        // ---- the chunk's 16 products of both halves on the matrix cores: wavefront w takes
        // the 32 x 32 sub-tile (w / 2, w % 2); v_mfma_f32_32x32x2f32 takes A[i][k] from lane
        // i + 32 k and B[k][j] from lane j + 32 k (float32 operands and accumulation).  The
        // chunk sums in a fresh accumulator that is then added to the running sum.
        {
            f32x16 p1, p2;
#pragma unroll
            for (int r = 0; r < 16; ++r) { p1[r] = 0.f; p2[r] = 0.f; }
#pragma unroll
            for (int kk = 0; kk < BK / 2; ++kk) {
                const int k = 2 * kk + (lane >> 5);
                p1 = __builtin_amdgcn_mfma_f32_32x32x2f32(A1[k][32 * wi + (lane & 31)], B1[k][32 * wj + (lane & 31)],
                                                          p1, 0, 0, 0);
                p2 = __builtin_amdgcn_mfma_f32_32x32x2f32(A2[k][32 * wi + (lane & 31)], B2[k][32 * wj + (lane & 31)],
                                                          p2, 0, 0, 0);
            }
#pragma unroll
            for (int r = 0; r < 16; ++r) { acc1[r] += p1[r]; acc2[r] += p2[r]; }
        }
        __syncthreads();
    }
    // ---- stores: interleave (forward) or recombine (inverse).  Register r of the lane
    // holds sub-tile row 8 (r / 4) + 4 (lane / 32) + r % 4, column lane % 32.
    const int gj = j0 + 32 * wj + (lane & 31);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int gi = i0 + 32 * wi + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        if (gi >= M || gj >= N) continue;
        if (ROW) {
            gfloat* dr = dst + (int64_t)gi * cols;
            if (!INV) { dr[2 * gj] = acc1[r]; dr[2 * gj + 1] = acc2[r]; }
            else { dr[gj] = acc1[r] + acc2[r]; dr[L - 1 - gj] = acc1[r] - acc2[r]; }
        } else {
            if (!INV) {
                dst[(int64_t)(2 * gi) * cols + gj] = acc1[r];
                dst[(int64_t)(2 * gi + 1) * cols + gj] = acc2[r];
            } else {
                dst[(int64_t)gi * cols + gj] = acc1[r] + acc2[r];
                dst[(int64_t)(L - 1 - gi) * cols + gj] = acc1[r] - acc2[r];
            }
        }
    }
}

} // namespace

// One axis pass over `count` images of rows x cols.  q: dense Q_L (L = rows for a column
// pass, cols for a row pass), row-major, float32.  The images are read through a.src and
// written through a.dst (row pitch = cols in both).
int launch_dense_axis(const Addr& a, int64_t count, int rows, int cols, bool column_pass, bool inverse,
                      const float* q, hipStream_t s)
{
    if (count <= 0) return DCT2D_OK;
    if (count > 65535) return DCT2D_ERR_ARG;
    const int L = column_pass ? rows : cols;
    if (L % 8 == 0) {
        // even/odd form (half the flops); needs L / 2 divisible by 4 for the 16-byte loads
        const int HL = L / 2;
        const dim3 grid = column_pass ? dim3((cols + BN - 1) / BN, (HL + BM - 1) / BM, (unsigned)count)
                                      : dim3((HL + BN - 1) / BN, (rows + BM - 1) / BM, (unsigned)count);
        if (column_pass) {
            if (inverse) k_dense_eo<false, true><<<grid, 256, 0, s>>>(a, q, rows, cols);
            else k_dense_eo<false, false><<<grid, 256, 0, s>>>(a, q, rows, cols);
        } else {
            if (inverse) k_dense_eo<true, true><<<grid, 256, 0, s>>>(a, q, rows, cols);
            else k_dense_eo<true, false><<<grid, 256, 0, s>>>(a, q, rows, cols);
        }
        return hipGetLastError() == hipSuccess ? DCT2D_OK : DCT2D_ERR_HIP;
    }
    int M, N, K;
    Mat qm;
    bool img_is_a;
    int64_t img_si, img_sk;
    if (column_pass) {
        // Y (rows x cols) = Qop (rows x rows) X (rows x cols); Qop = Q or Q^T
        M = rows; N = cols; K = rows;
        qm = inverse ? Mat{(const gfloat*)q, 1, rows} : Mat{(const gfloat*)q, rows, 1};
        img_is_a = false;
        img_si = cols; img_sk = 1; // B(k, j) = X[k][j]
    } else {
        // Y (rows x cols) = X (rows x cols) Qop (cols x cols); Qop = Q^T (fwd) or Q (inv)
        M = rows; N = cols; K = cols;
        // B(k, j): forward Q^T -> Q[j][k] = q[j*cols + k]: B.si (k stride) = 1, B.sk (j stride) = cols
        qm = inverse ? Mat{(const gfloat*)q, cols, 1} : Mat{(const gfloat*)q, 1, cols};
        img_is_a = true;
        img_si = cols; img_sk = 1; // A(i, k) = X[i][k]
    }
    dim3 grid((N + BN - 1) / BN, (M + BM - 1) / BM, (unsigned)count);
    k_dense_pass<<<grid, 256, 0, s>>>(a, img_is_a, qm, img_si, img_sk, M, N, K, cols);
    return hipGetLastError() == hipSuccess ? DCT2D_OK : DCT2D_ERR_HIP;
}

} // namespace dct
