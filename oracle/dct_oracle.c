/*
 * FP64 reference ("oracle") for the orthonormal two-dimensional DCT.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant with
 * the HIP implementation.
 *
 * What it computes (paper, Section 2.1, eq. 1 and eq. 2; rectangles Section 7.1):
 *   (Q_n)_{kj} = a_k cos(pi/n (j + 1/2) k),  a_0 = n^{-1/2},  a_k = (2/n)^{1/2}
 *   forward  C(X)    = Q_h X Q_w^T
 *   inverse  C^-1(Y) = Q_h^T Y Q_w
 *   filter   C^-1(L o C(X)) for a diagonal spectral operator given as an array L of
 *            multipliers, L[k][l] scaling coefficient (k, l) (Section 2.1, Prop. 1,
 *            eq. 4, with the orthonormal Q in place of the scaled core and E = I)
 * evaluated exactly as written: the two matrix products one after the other,
 * plain loops, double precision throughout, output kept in double (never
 * rounded to float).  No fast algorithm, no blocking, no fusion.
 *
 * The cosine argument is reduced in integers first: m = (2j+1)k mod 4n and
 * cos(pi m / (2n)) is evaluated on [0, pi/2] through quadrant symmetry, so the
 * exact zeros (m = n, 3n) and the sign symmetries of eq. 1 hold exactly.
 *
 * Threads: blocks are distributed over POSIX threads; every block is computed
 * by one thread with the same serial loops, so the result does not depend on
 * the thread count.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_ERR_ARG -1
#define ORACLE_ERR_NOMEM -2

/* cos(pi * m / (2n)) for an integer m, exact symmetries (eq. 1). */
static double cos_half_turn_fraction(int64_t m, int64_t n)
{
    const double pi = 3.14159265358979323846264338327950288;
    int64_t period = 4 * n; /* cos(pi m/(2n)) has period 4n in m */
    m %= period;
    if (m < 0) m += period;
    if (m > 2 * n) m = period - m;           /* cos(2pi - t) = cos(t)      */
    double sign = 1.0;
    if (m > n) { m = 2 * n - m; sign = -1.0; } /* cos(pi - t) = -cos(t)    */
    if (m == n) return 0.0;                     /* cos(pi/2) = 0 exactly     */
    return sign * cos(pi * (double)m / (double)(2 * n));
}

/* Q_n of eq. 1, row-major, q[k*n + j]. */
int oracle_qmatrix(int32_t n, double* q)
{
    if (n <= 0 || q == NULL) return ORACLE_ERR_ARG;
    const double a0 = sqrt(1.0 / (double)n);
    const double ak = sqrt(2.0 / (double)n);
    for (int32_t k = 0; k < n; ++k)
        for (int32_t j = 0; j < n; ++j)
            q[(int64_t)k * n + j] =
                (k == 0 ? a0 : ak) * cos_half_turn_fraction((int64_t)(2 * j + 1) * k, n);
    return ORACLE_OK;
}

typedef struct {
    int dir;                 /* 0 forward, 1 inverse, 2 inverse(forward(.)), 3 filter */
    const float* xf;         /* float input (or NULL) */
    const double* xd;        /* double input (or NULL) */
    double* y;               /* output, packed rows*cols per array */
    int64_t batch, stride;   /* stride: elements between consecutive input arrays */
    int32_t rows, cols;
    const double* qh;        /* Q_rows */
    const double* qw;        /* Q_cols */
    const double* lam;       /* filter multipliers: array b uses lam + b*lam_stride */
    int64_t lam_stride;
    int64_t next;            /* shared work counter (protected by lock) */
    pthread_mutex_t lock;
    int failed;
} job_t;

/* Y = Q_h X Q_w^T for one array, two products in order (eq. 2). */
static void forward_one(const double* x, double* y, double* t, int32_t h, int32_t w,
                        const double* qh, const double* qw)
{
    /* T = X Q_w^T : T[r][l] = sum_c X[r][c] Q_w[l][c] */
    for (int32_t r = 0; r < h; ++r)
        for (int32_t l = 0; l < w; ++l) {
            double s = 0.0;
            for (int32_t c = 0; c < w; ++c) s += x[(int64_t)r * w + c] * qw[(int64_t)l * w + c];
            t[(int64_t)r * w + l] = s;
        }
    /* Y = Q_h T : Y[k][l] = sum_r Q_h[k][r] T[r][l] */
    for (int32_t k = 0; k < h; ++k)
        for (int32_t l = 0; l < w; ++l) {
            double s = 0.0;
            for (int32_t r = 0; r < h; ++r) s += qh[(int64_t)k * h + r] * t[(int64_t)r * w + l];
            y[(int64_t)k * w + l] = s;
        }
}

/* X = Q_h^T Y Q_w for one array (eq. 2, inverse). */
static void inverse_one(const double* y, double* x, double* t, int32_t h, int32_t w,
                        const double* qh, const double* qw)
{
    /* T = Y Q_w : T[k][c] = sum_l Y[k][l] Q_w[l][c] */
    for (int32_t k = 0; k < h; ++k)
        for (int32_t c = 0; c < w; ++c) {
            double s = 0.0;
            for (int32_t l = 0; l < w; ++l) s += y[(int64_t)k * w + l] * qw[(int64_t)l * w + c];
            t[(int64_t)k * w + c] = s;
        }
    /* X = Q_h^T T : X[r][c] = sum_k Q_h[k][r] T[k][c] */
    for (int32_t r = 0; r < h; ++r)
        for (int32_t c = 0; c < w; ++c) {
            double s = 0.0;
            for (int32_t k = 0; k < h; ++k) s += qh[(int64_t)k * h + r] * t[(int64_t)k * w + c];
            x[(int64_t)r * w + c] = s;
        }
}

static void* worker(void* arg)
{
    job_t* job = (job_t*)arg;
    const int64_t n = (int64_t)job->rows * job->cols;
    double* in = (double*)malloc(sizeof(double) * n);
    double* t = (double*)malloc(sizeof(double) * n);
    double* t2 = (double*)malloc(sizeof(double) * n);
    if (!in || !t || !t2) {
        pthread_mutex_lock(&job->lock);
        job->failed = 1;
        pthread_mutex_unlock(&job->lock);
        free(in); free(t); free(t2);
        return NULL;
    }
    for (;;) {
        pthread_mutex_lock(&job->lock);
        int64_t b = job->next++;
        pthread_mutex_unlock(&job->lock);
        if (b >= job->batch) break;
        const int64_t off = b * job->stride;
        if (job->xf) for (int64_t i = 0; i < n; ++i) in[i] = (double)job->xf[off + i];
        else memcpy(in, job->xd + off, sizeof(double) * n);
        double* out = job->y + b * n;
        if (job->dir == 0) {
            forward_one(in, out, t, job->rows, job->cols, job->qh, job->qw);
        } else if (job->dir == 1) {
            inverse_one(in, out, t, job->rows, job->cols, job->qh, job->qw);
        } else if (job->dir == 2) {
            forward_one(in, t2, t, job->rows, job->cols, job->qh, job->qw);
            inverse_one(t2, out, t, job->rows, job->cols, job->qh, job->qw);
        } else {
            /* Prop. 1: forward, the diagonal operator (one multiplier per
             * coefficient), then the adjoint; all in double */
            const double* lam = job->lam + b * job->lam_stride;
            forward_one(in, t2, t, job->rows, job->cols, job->qh, job->qw);
            for (int64_t i = 0; i < n; ++i) t2[i] *= lam[i];
            inverse_one(t2, out, t, job->rows, job->cols, job->qh, job->qw);
        }
    }
    free(in); free(t); free(t2);
    return NULL;
}

static int run(int dir, const float* xf, const double* xd, double* y, int64_t batch,
               int32_t rows, int32_t cols, int64_t stride, int32_t nthreads,
               const double* lam, int64_t lam_stride)
{
    if (batch < 0 || rows <= 0 || cols <= 0 || (batch > 0 && (y == NULL || (!xf && !xd))))
        return ORACLE_ERR_ARG;
    if (dir == 3 && (lam == NULL || lam_stride < 0 || (lam_stride > 0 && lam_stride < (int64_t)rows * cols)))
        return ORACLE_ERR_ARG;
    if (stride < (int64_t)rows * cols) return ORACLE_ERR_ARG;
    if (batch == 0) return ORACLE_OK;
    double* qh = (double*)malloc(sizeof(double) * rows * rows);
    double* qw = (double*)malloc(sizeof(double) * cols * cols);
    if (!qh || !qw) { free(qh); free(qw); return ORACLE_ERR_NOMEM; }
    oracle_qmatrix(rows, qh);
    oracle_qmatrix(cols, qw);
    job_t job;
    job.dir = dir; job.xf = xf; job.xd = xd; job.y = y;
    job.batch = batch; job.stride = stride; job.rows = rows; job.cols = cols;
    job.qh = qh; job.qw = qw; job.next = 0; job.failed = 0;
    job.lam = lam; job.lam_stride = lam_stride;
    pthread_mutex_init(&job.lock, NULL);
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    if ((int64_t)nthreads > batch) nthreads = (int32_t)batch;
    pthread_t tid[256];
    int started = 0;
    for (int i = 1; i < nthreads; ++i)
        if (pthread_create(&tid[started], NULL, worker, &job) == 0) ++started;
    worker(&job); /* the calling thread works too */
    for (int i = 0; i < started; ++i) pthread_join(tid[i], NULL);
    pthread_mutex_destroy(&job.lock);
    free(qh); free(qw);
    return job.failed ? ORACLE_ERR_NOMEM : ORACLE_OK;
}

/* Forward 2D DCT-II (eq. 2) of `batch` float32 arrays rows x cols; array b starts
 * at x + b*stride (rows contiguous, pitch cols).  y receives batch*rows*cols
 * doubles, packed.  Returns 0, or a negative code on bad arguments. */
int oracle_forward(const float* x, double* y, int64_t batch, int32_t rows, int32_t cols,
                   int64_t stride, int32_t nthreads)
{
    return run(0, x, NULL, y, batch, rows, cols, stride, nthreads, NULL, 0);
}

/* Inverse 2D DCT-III (eq. 2): X = Q_h^T Y Q_w.  Same layout rules as above. */
int oracle_inverse(const float* x, double* y, int64_t batch, int32_t rows, int32_t cols,
                   int64_t stride, int32_t nthreads)
{
    return run(1, x, NULL, y, batch, rows, cols, stride, nthreads, NULL, 0);
}

/* inverse(forward(X)) in double, both products of each kept in double. */
int oracle_roundtrip(const float* x, double* y, int64_t batch, int32_t rows, int32_t cols,
                     int64_t stride, int32_t nthreads)
{
    return run(2, x, NULL, y, batch, rows, cols, stride, nthreads, NULL, 0);
}

/* Double-input variants (for exact test inputs). */
int oracle_forward_d(const double* x, double* y, int64_t batch, int32_t rows, int32_t cols,
                     int64_t stride, int32_t nthreads)
{
    return run(0, NULL, x, y, batch, rows, cols, stride, nthreads, NULL, 0);
}

int oracle_inverse_d(const double* x, double* y, int64_t batch, int32_t rows, int32_t cols,
                     int64_t stride, int32_t nthreads)
{
    return run(1, NULL, x, y, batch, rows, cols, stride, nthreads, NULL, 0);
}

/* Spectral filter of `batch` float32 arrays (layout as oracle_forward):
 * y = Q_h^T (L o (Q_h X Q_w^T)) Q_w with L the rows x cols multipliers at
 * lam + b*lam_stride (lam_stride 0: one operator for every array, else
 * >= rows*cols).  Section 2.1, Prop. 1, eq. 4 (orthonormal form). */
int oracle_filter(const float* x, double* y, int64_t batch, int32_t rows, int32_t cols,
                  int64_t stride, const double* lam, int64_t lam_stride, int32_t nthreads)
{
    return run(3, x, NULL, y, batch, rows, cols, stride, nthreads, lam, lam_stride);
}
