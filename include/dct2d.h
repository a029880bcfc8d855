/*
 * dct2d.h -- C ABI of the MI355X (gfx950) batched orthonormal 2D DCT library.
 *
 * The operation (paper, Section 2.1, eq. 1 and eq. 2; rectangles Section 7.1):
 *   (Q_n)_{kj} = a_k cos(pi/n (j + 1/2) k),   a_0 = n^{-1/2},  a_k = (2/n)^{1/2}
 *   forward   Y = Q_h X Q_w^T      (2D DCT-II, orthonormal)
 *   inverse   X = Q_h^T Y Q_w      (2D DCT-III, the Frobenius adjoint of the forward)
 *   roundtrip X' = Q_h^T (Q_h X Q_w^T) Q_w, fused in one pass over memory (Section 3.1,
 *             Prop. 1); its exact result is X.
 * "Exact" in the paper's sense (Section 1.1): no truncated coefficients and no
 * approximate matrix; floating-point results differ from real arithmetic only by
 * rounding and are not bit-identical across algorithms.
 *
 * Data layout (all entry points): an array of `batch` row-major float32 arrays of
 * rows x cols elements.  Array b starts at element b*stride of the buffer; inside an
 * array, element (r, c) is at r*cols + c (rows contiguous, pitch = cols).  This is the
 * paper's "ordinary row-major" natural layout (Section 1.1, Section 3.1).  `stride` is
 * counted in floats and must be >= rows*cols, so arrays never overlap.
 *
 * Pointers: `data`, `in`, `out` and ragged `base` are DEVICE pointers (memory the
 * caller allocated on the current HIP device, e.g. through PyTorch).  The caller
 * owns them; the library never frees them and keeps none of them past the call.  A
 * ragged plan receives its base pointer on every execute call and keeps only a device
 * copy of the last one (to skip the 8-byte update when it repeats); it never
 * dereferences it outside an execute.  Host pointers are accepted only where stated
 * (descriptor arrays of the ragged planner).
 *
 * Streams: `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 * transform calls only enqueue work and return; results are visible after the
 * caller synchronises that stream.  Return codes cover argument validation and
 * launch errors; a fault during execution surfaces at the caller's synchronisation.
 *
 * Sizes accepted by the three basic calls and dct2d_transform_ex: rows and cols each
 * a power of two in [8, 1024] (squares and rectangles).  Axes up to 256 run the fused
 * kernels; a shape with an axis of 512 or 1024 runs two line passes, rows then columns,
 * the second in place on `out` (no workspace, no allocation): a 512- or 1024-point line is
 * split into its even/odd halves (Section 2.2) down to length-256 DCT-II/III and DCT-IV
 * transforms (the DCT-IV of a 512-point half through a 128-point complex FFT), each half
 * held by one wavefront and the halves combined through LDS.  Each pass reads and writes
 * the array once; the round trip is fused per line (forward, then inverse, in one pass).  Float32
 * path only (any other precision: DCT2D_ERR_PRECISION).  The variant, autotuner and
 * filter calls cover axes up to 256.  Any other length returns DCT2D_ERR_SIZE: like the
 * paper (Section 7.1) the basic API rejects non-power-of-two axes instead of
 * zero-padding, which would change the transform.  dct2d_image_transform and ragged
 * plans accept whole images with any axes in [8, 1024], including non-power-of-two
 * lengths (computed exactly from the dense Q_n of eq. 1).
 *
 * Alignment: `data`/`in`/`out` must be 16-byte aligned and strides multiples of 4
 * floats (DCT2D_ERR_ALIGN otherwise).
 *
 * Errors are returned, never thrown, and the library never aborts the process.
 * Thread safety: after dct2d_init, the transform calls may be issued from several
 * host threads; a ragged plan must not be executed concurrently with itself.
 * No call allocates device memory or plans anything after dct2d_init (Section 3.2:
 * plan-owned tables and workspace, no allocation inside a transform), except that
 * the first call on a device initialises it if dct2d_init was not called.
 */
#ifndef DCT2D_H
#define DCT2D_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------------ */
#define DCT2D_OK             0
#define DCT2D_ERR_ARG       -1  /* null pointer with batch > 0, batch < 0, bad enum */
#define DCT2D_ERR_SIZE      -2  /* unsupported rows/cols                           */
#define DCT2D_ERR_STRIDE    -3  /* stride < rows*cols                               */
#define DCT2D_ERR_ALIGN     -4  /* pointer not 16-byte aligned / stride % 4 != 0     */
#define DCT2D_ERR_PRECISION -5  /* precision not available for this size            */
#define DCT2D_ERR_HIP       -6  /* a HIP runtime call or kernel launch failed        */
#define DCT2D_ERR_NOINIT    -7  /* no usable device / library not initialised        */
#define DCT2D_ERR_NOMEM     -8  /* device or host allocation failed (init, plans)    */

/* ---- directions ---------------------------------------------------------------- */
#define DCT2D_FORWARD   0   /* Y = Q_h X Q_w^T            (eq. 2)                  */
#define DCT2D_INVERSE   1   /* X = Q_h^T Y Q_w            (eq. 2)                  */
#define DCT2D_ROUNDTRIP 2   /* inverse(forward(X)), fused (Section 3.1, Prop. 1)   */
#define DCT2D_FILTER    3   /* spectral filter (dct2d_filter, Prop. 1, eq. 4): accepted
                               by the policy / autotuner calls only, float32 path    */

/* ---- arithmetic paths ------------------------------------------------------------
 * DCT2D_FP32        float32 fast transforms on the vector ALU (all sizes).
 * DCT2D_SPLIT_BF16X3  dense Q X Q^T on MFMA, bf16 two-way split of Q and X, three
 *                   products (hi*hi + hi*lo + lo*hi), fp32 accumulation, per-block
 *                   power-of-two scaling.  rows = cols <= 64.  Not float32-accurate
 *                   (~16 significant bits); reported, not gated.
 * DCT2D_SPLIT_BF16X6  as above with a three-way bf16 split and the six products
 *                   whose split indices sum to <= 2; float32-accurate.
 * DCT2D_SPLIT_FP16X3  fp16 two-way split, three products, per-block power-of-two
 *                   scaling before each pass; float32-accurate for finite inputs.
 * DCT2D_BF16 / DCT2D_FP16 / DCT2D_FP8_E4M3  single-pass low precision on MFMA with
 *                   per-block power-of-two scaling (error reported, never gated).
 * DCT2D_AUTO        the library's frozen per-size choice among the float32-accurate
 *                   paths (FP32, SPLIT_BF16X6, SPLIT_FP16X3). */
typedef enum {
    DCT2D_FP32 = 0,
    DCT2D_SPLIT_BF16X3 = 1,
    DCT2D_SPLIT_BF16X6 = 2,
    DCT2D_SPLIT_FP16X3 = 3,
    DCT2D_BF16 = 4,
    DCT2D_FP16 = 5,
    DCT2D_FP8_E4M3 = 6,
    DCT2D_AUTO = 7
} dct2d_precision;

/* Initialise the library on HIP device `device` (0-based): generates the cosine,
 * twiddle and split tables on that device in FP64 (the only FP64 work on the GPU)
 * and rounds them to the formats the kernels read.  Idempotent; safe to call again.
 * Returns DCT2D_OK, DCT2D_ERR_NOINIT (no such device) or DCT2D_ERR_HIP/NOMEM. */
int dct2d_init(int device);

/* Release every device's tables.  Plans must be destroyed first. */
void dct2d_finalize(void);

/* In-place forward transform of `batch` arrays at `data` (device pointer), using the
 * library's default float32-accurate path (DCT2D_AUTO).  batch == 0 is a no-op. */
int dct2d_forward(float* data, int64_t batch, int32_t rows, int32_t cols, int64_t stride,
                  void* stream);

/* In-place inverse transform (eq. 2, DCT-III).  Same arguments and rules. */
int dct2d_inverse(float* data, int64_t batch, int32_t rows, int32_t cols, int64_t stride,
                  void* stream);

/* In-place fused round trip inverse(forward(X)): one read and one write of each array. */
int dct2d_roundtrip(float* data, int64_t batch, int32_t rows, int32_t cols, int64_t stride,
                    void* stream);

/* General entry: direction `dir` (DCT2D_FORWARD/INVERSE/ROUNDTRIP), out-of-place or
 * in-place (in == out allowed, with in_stride == out_stride when batch > 1; partially
 * overlapping buffers are not: DCT2D_ERR_ARG), explicit arithmetic path `precision`
 * (dct2d_precision).  in_stride / out_stride as above.
 * Returns DCT2D_ERR_PRECISION when the path does not exist for the size. */
int dct2d_transform_ex(int dir, const float* in, float* out, int64_t batch, int32_t rows,
                       int32_t cols, int64_t in_stride, int64_t out_stride, int precision,
                       void* stream);

/* Spectral filter (paper, Section 2.1, Prop. 1 and eq. 4, in the orthonormal form
 * where the scale tables are folded into Q):
 *   X' = Q_h^T (L o (Q_h X Q_w^T)) Q_w
 * for a diagonal spectral operator given as an array L of rows x cols float32
 * multipliers: L[k][l] scales 2D coefficient (k, l) (row k of the column transform,
 * column l of the row transform).  L = 1 gives the round trip; the multipliers of a
 * Neumann Poisson solve give the least-squares solver step of phase unwrapping.
 * Fused like dct2d_roundtrip: each array is read once and written once, the multiply
 * happens on chip between the forward and inverse transforms, float32 arithmetic on
 * the vector ALU (the DCT2D_FP32 path; its kernel variant is the policy entry of
 * direction DCT2D_FILTER, which starts as the round trip's and can be tuned).
 *   in, out, batch, rows, cols, in_stride, out_stride: as dct2d_transform_ex (in ==
 *     out allowed; sizes as the basic calls).
 *   lambda: device pointer to the multipliers, row-major with pitch cols, 4-byte
 *     aligned; read only; must not overlap the output arrays.
 *   lambda_stride: 0 = one operator shared by every array; otherwise >= rows*cols and
 *     array b uses lambda + b*lambda_stride (one extra read of rows*cols floats per
 *     array).
 * Errors: as dct2d_transform_ex; DCT2D_ERR_STRIDE for a negative or too small
 * lambda_stride, DCT2D_ERR_ARG for a null lambda (batch > 0) or lambda overlapping
 * the output, DCT2D_ERR_ALIGN for a misaligned lambda. */
int dct2d_filter(const float* in, float* out, int64_t batch, int32_t rows, int32_t cols,
                 int64_t in_stride, int64_t out_stride, const float* lambda, int64_t lambda_stride,
                 void* stream);

/* ---- whole images of any shape ----------------------------------------------------------
 * Batched transform (direction as dct2d_transform_ex) of `batch` images of rows x cols with
 * both axes in [8, 1024] and cols a multiple of 4, including lengths that are not powers of
 * two (384, 600, 1000, ...): the strided-batch form of the ragged planner's image classes.
 * Pointers, strides, alignment and in-place rules as dct2d_transform_ex.  Shapes with both
 * axes powers of two run the basic calls' kernels (DCT2D_AUTO; with an axis of 512 or 1024
 * the two line passes, which use no workspace).  Every other shape
 * is computed exactly from the dense Q_n of eq. 1 (Section 2.1; the paper's own library
 * rejects non-power-of-two axes, Section 7.1, rather than zero-padding them, which would
 * change the transform): one dense float32 product per axis (two for the round trip), with
 * the top even/odd level of Q_n's symmetry taken out where n is a multiple of 8.  The passes
 * go through a workspace of rows*cols floats per image (batch images, at most 65535 at a
 * time), taken from the stream-ordered allocator on `stream` and released on it; the dense
 * Q_n of each length is built once per device on first use (so the first call of a shape
 * synchronises the device) and kept until dct2d_finalize.
 * Errors: DCT2D_ERR_SIZE (shape), DCT2D_ERR_NOMEM (workspace), as dct2d_transform_ex
 * otherwise. */
int dct2d_image_transform(int dir, const float* in, float* out, int64_t batch, int32_t rows,
                          int32_t cols, int64_t in_stride, int64_t out_stride, void* stream);

/* The same transform for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): allocates nothing and
 * never builds tables itself.  dct2d_init must have been called for the current device
 * (DCT2D_ERR_NOINIT otherwise).  The dense Q tables and the workspace live in a fixed
 * 64 MiB device array that the library holds on every device it runs on until the process
 * ends; the tables are rebuilt in it on `stream` by every call and the batch is processed in
 * chunks that fit (every accepted shape fits: the largest, 1024 x 1020, needs 12 MiB for one
 * image), so results equal dct2d_image_transform's.  Shapes whose axes are both powers of
 * two use none of the array (the basic calls' kernels, no tables, no workspace).  Calls on one device share that array: calls that
 * overlap in time on one device (different streams, or threads without ordering) race and
 * give wrong results.  Same arguments and errors as dct2d_image_transform, except that
 * DCT2D_ERR_SIZE also marks a shape needing more than the 64 MiB (none of the accepted
 * shapes does). */
int dct2d_image_transform_noalloc(int dir, const float* in, float* out, int64_t batch,
                                  int32_t rows, int32_t cols, int64_t in_stride,
                                  int64_t out_stride, void* stream);

/* ---- ragged batches: many arrays of different shapes in one launch ------------------
 * A descriptor names one array inside a caller buffer: its first element is at
 * base + offset (floats), its shape rows x cols (pitch = cols).  Arrays must not
 * overlap.  Accepted shapes: both axes in [8, 1024] with cols a multiple of 4; shapes
 * with both axes powers of two <= 256 use the fast kernels of the basic calls, shapes
 * with both axes powers of two and one of 512 or 1024 (1024 x 1024, 64 x 1024) the two
 * float32 line passes of the basic calls, in place (whatever the plan's precision), and
 * any other shape (512 x 384) is computed with dense float32 Q_n tables (exact for
 * non-power-of-two axes; no zero-padding).
 *
 * dct2d_ragged_plan_create copies the (host) descriptor array, groups the items into
 * shape classes, uploads the per-class offset lists to the device, picks each class's
 * kernel configuration from the frozen per-size policy (the autotuner's table), and
 * records the whole batch as one HIP graph with one concurrent branch per class.  It
 * allocates device memory (once, here: offset lists, dense tables, the image
 * workspace).  `dir` is a DCT2D_* direction; `precision` DCT2D_FP32, DCT2D_AUTO or a
 * float32-accurate split path (DCT2D_SPLIT_BF16X6 / DCT2D_SPLIT_FP16X3, used for the
 * classes that have it).  Errors: DCT2D_ERR_SIZE (shape), DCT2D_ERR_ALIGN (offset not a
 * multiple of 4), DCT2D_ERR_ARG (overlap, empty, more than 65535 images of one shape).
 *
 * dct2d_ragged_execute runs the plan in place on the arrays at `base` (device pointer,
 * 16-byte aligned) with one hipGraphLaunch on `stream`.  The graph reads the base from
 * a plan-owned device slot; when `base` differs from the previous call an 8-byte copy
 * on `stream` updates the slot first.  It allocates nothing.  Executions of one plan on
 * different streams must not overlap.
 */
typedef struct {
    int64_t offset;  /* element offset from base (multiple of 4) */
    int32_t rows;    /* array height */
    int32_t cols;    /* array width (= pitch) */
} dct2d_block;

typedef struct dct2d_ragged_plan dct2d_ragged_plan;

int dct2d_ragged_plan_create(const dct2d_block* blocks, int64_t count, int dir, int precision,
                             dct2d_ragged_plan** out_plan);
int dct2d_ragged_execute(dct2d_ragged_plan* plan, float* base, void* stream);
void dct2d_ragged_plan_destroy(dct2d_ragged_plan* plan);

/* Items, shape classes and nodes of the plan's recorded graph (diagnostics). */
int dct2d_ragged_plan_info(const dct2d_ragged_plan* plan, int64_t* items, int32_t* classes,
                           int32_t* graph_nodes);

/* ---- policy / autotuner ----------------------------------------------------------------
 * The per-(rows, cols, dir, precision) kernel configuration is a small integer
 * "variant" chosen by the autotuner ahead of time and frozen (Section 3.2: variants
 * fixed per size and direction before measurement).  dct2d_tune measures the
 * candidate variants for one case on scratch data it allocates itself (call it
 * outside timed regions) and freezes the fastest one that passes a correctness
 * guard which trusts no other candidate: on 48 arrays spread over the whole batch
 * (first and last included) the candidate composed with the opposite transform must
 * return its input (round trip: its own output; forward / inverse: followed by the
 * frozen float32 inverse / forward; filter: multipliers 1 and -1/2 must give X and
 * -X/2) within the round-trip gate 4e-6 (float32-accurate paths) or a bound above
 * the path's error band (single-pass and BF16X3).  A candidate that fails is never
 * frozen; if every candidate fails, dct2d_tune returns DCT2D_ERR_HIP and leaves the
 * table unchanged.  dct2d_get_variant / dct2d_set_variant read and override the
 * frozen table; dct2d_variant_count gives the number of candidates (0 = none).
 * `dir` may also be DCT2D_FILTER, with precision DCT2D_FP32 (or DCT2D_AUTO, which for the
 * filter always means DCT2D_FP32): the filter's own frozen variant, which starts as the
 * round trip's and is tuned on scratch data with one shared multiplier array. */
int dct2d_variant_count(int32_t rows, int32_t cols, int dir, int precision);
int dct2d_get_variant(int32_t rows, int32_t cols, int dir, int precision);
int dct2d_set_variant(int32_t rows, int32_t cols, int dir, int precision, int variant);
int dct2d_tune(int32_t rows, int32_t cols, int dir, int precision, int64_t batch, void* stream,
               float* best_ms);

/* ---- measurement reference -------------------------------------------------------
 * Copies n float32 values from `in` to `out` (device pointers, 16-byte aligned; in ==
 * out allowed, partial overlap is not) with a plain streaming kernel: one read and one
 * write per element, the same algorithmic traffic as a transform.  Not a transform:
 * it is the practical HBM ceiling the benchmark times in the same run (the transforms'
 * achieved GB/s is reported against it as well as against the 8 TB/s peak).
 * Errors: DCT2D_ERR_ARG (n < 0, null pointer with n > 0, overlap), DCT2D_ERR_ALIGN. */
int dct2d_copy(const float* in, float* out, int64_t n, void* stream);

/* Vector-ALU issue reference (measurement helper, no transform): launches `blocks`
 * workgroups of 256 threads, each lane issuing iters x 16 independent float32 FMAs
 * (wave64, no packed math).  With blocks = CUs x w the grid holds w wavefronts per SIMD;
 * 16 x iters x 4 x blocks wavefront instructions over the elapsed time and the SIMD count
 * give the FMA issue rate per SIMD and cycle at that occupancy, the reference for the VALU
 * share of the transform kernels.  `sink`: a device float the kernel never writes in
 * practice (the FMA results only feed a comparison that never holds).  Errors: DCT2D_ERR_ARG (null sink,
 * blocks < 1, iters < 1), DCT2D_ERR_ALIGN. */
int dct2d_fma_issue(float* sink, int32_t blocks, int32_t iters, void* stream);

/* Human-readable text for a status code (static storage). */
const char* dct2d_status_string(int status);

/* Library version string (static storage). */
const char* dct2d_version(void);

#ifdef __cplusplus
}
#endif

#endif /* DCT2D_H */
