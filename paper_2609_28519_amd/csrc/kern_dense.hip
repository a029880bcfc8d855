// Dense axis passes for whole images: one 1D transform of length L applied along the
// rows or the columns of a batch of h x w images by a float32 matrix product with the
// dense Q_L of eq. 1 (Section 2.1; rectangles and arbitrary axes, Section 7.1).  Used
// for the image axes of ragged batches (1024, 512 and the non-power-of-two 384, which
// the fast transforms do not cover; zero-padding would change the transform).
//
//   column pass   Y = Q_h X      (forward)    Y = Q_h^T X   (inverse)
//   row pass      Y = X Q_w^T    (forward)    Y = X Q_w     (inverse)
//
// Tiled product: a 256-thread workgroup computes a 64 x 64 output tile, each thread a
// 4 x 4 micro-tile, over K in chunks of 16 staged in LDS.  The 16 products of a chunk
// are summed in a fresh partial that is then added to the running sum (blocked
// summation), which keeps the float32 accumulation error near 4 unit roundoffs per
// pass at L = 1024 instead of growing like sqrt(L/6).
#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace dct {
namespace {

constexpr int BM = 64, BN = 64, BK = 16;

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

} // namespace

// One axis pass over `count` images of rows x cols.  q: dense Q_L (L = rows for a column
// pass, cols for a row pass), row-major, float32.  The images are read through a.src and
// written through a.dst (row pitch = cols in both).
int launch_dense_axis(const Addr& a, int64_t count, int rows, int cols, bool column_pass, bool inverse,
                      const float* q, hipStream_t s)
{
    if (count <= 0) return DCT2D_OK;
    if (count > 65535) return DCT2D_ERR_ARG;
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
