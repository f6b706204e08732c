/*
 * libsignfn -- matrix sign function of large sparse matrices on AMD MI355X
 * (gfx950) by the filtered Newton-Schulz iteration and the filtered Newton
 * iteration of Wu, Ye, Zhu, Zhao, Hu and Zhong, "Two iterative algorithms for
 * the matrix sign function based on the adaptive filtering technology".
 *
 * C ABI: plain pointers and sizes only; no C++ types or exceptions cross it.
 *
 * Matrices are square CSR:
 *   row_ptr  int64[n+1], row_ptr[0] = 0, non-decreasing, row_ptr[n] = nnz
 *   col      int32[nnz], column indices in [0, n), strictly ascending per row
 *   val      nnz values, double (val_f32 = 0) or float (val_f32 = 1), finite
 * Explicit zeros are allowed on input; results never store exact zeros (the
 * sparse storage of Section 4 never keeps zeros).
 *
 * Unless stated otherwise, every pointer inside a sign_csr given to the
 * library is a DEVICE pointer on the current HIP device, and every call runs
 * its kernels on the HIP stream passed as `hip_stream` (a hipStream_t; NULL
 * is the legacy default stream).  Calls that produce a result synchronise
 * that stream before returning, because the size of the result is only known
 * on the device.
 *
 * Errors: functions return a sign_status; negative values are errors, and
 * sign_last_error() gives a message for the last failing call of the calling
 * thread.  Nothing is printed.
 *
 * Symmetric inputs: sign_ns checks the (scaled) input for exact symmetry; when
 * it holds and residuals are not filtered (filter_y = 0), every product of the
 * iteration is symmetric and is formed from its lower triangle and mirrored,
 * and the result is exactly symmetric.
 *
 * Tuning (environment, read when a call starts): SIGNFN_ROW_GROUP = 1, 2, 4,
 * 8 or 16 output rows per workgroup of the product kernel for rows with wide
 * column spans (default per product: 2 for A or B rows of a few entries, 8 for
 * FP64 values with long A rows and B rows dense within their column ranges,
 * else 4); SIGNFN_SYMMETRIC=0 turns the
 * symmetric products off; SIGNFN_PROGRESS=1 prints one line per finished
 * iteration (and per product) to stderr.
 */
#ifndef SIGNFN_H
#define SIGNFN_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define SIGNFN_API __attribute__((visibility("default")))
#else
#define SIGNFN_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SIGN_OK = 0,
    SIGN_PENDING = 1,     /* serving: the request has not finished yet */
    SIGN_EINVAL = -1,     /* malformed CSR, n <= 0, non-finite value, bad option */
    SIGN_ENOMEM = -2,     /* device allocation failed or budget too small */
    SIGN_ENOCONV = -3,    /* max_iter reached; the result holds the last iterate */
    SIGN_EDIVERGED = -4,  /* residual grew (or became non-finite); last iterate returned */
    SIGN_EDEVICE = -5,    /* a HIP runtime call failed */
    SIGN_EBUSY = -6,      /* serving: queue full */
    SIGN_ENOTFOUND = -7   /* serving: unknown ticket */
} sign_status;

typedef struct {
    int64_t n;
    int64_t nnz;
    int64_t *row_ptr;
    int32_t *col;
    void *val;
    int val_f32;
} sign_csr;

/* Options.  sign_opts_default() fills the values given in brackets. */
typedef struct {
    double tol;          /* [1e-12] epsilon_tol of Algorithms 3.1.1 / 3.2.1 (> 0) */
    int stop_rule;       /* [0] 0: stop when e_k = ||I - X^_k^2||_F <= tol (Alg. 3.2.1);
                            1: stop when the last update ||Xbar_{k+1} - X^_k||_F < tol */
    double c_fixed;      /* [1e-4] fixed budget ||F_k||_F <= c_fixed*tol while e_k >= switch_res
                            (c4 of Section 3.2, c2 of Section 3.1) */
    double switch_res;   /* [1e-6] residual below which the adaptive budget applies
                            (eq. 1.18 for NSF, eq. 1.13 for NMF; Section 4) */
    int max_iter;        /* [100] at most this many updates */
    int precision;       /* [0] 0: FP64 throughout.  1: FP32 values in the bulk products
                            (FP32 x FP32 is exact in FP64, and the sums are accumulated in
                            FP64 before the FP32 store), FP64 norms/scaling/thresholds, then
                            FP64 refinement and polishing (sign_ns only) */
    int polish_steps;    /* [2] FP64 Newton-Schulz steps after an FP32 phase (precision 1) */
    int refine_steps;    /* [6] commutator-refinement sweeps between the polish steps
                            (precision 1; 0 disables) */
    int filter_y;        /* [0] 1: also filter R^_k = I - X^_k^2 with the same budget */
    double scale;        /* [0] X_1 = A/scale; 0 selects ||A||_inf for sign_ns and 1 for
                            sign_newton (the paper starts both from X_1 = A) */
    size_t staging_bytes;/* [0] device staging for one product; 0 = automatic */
    /* Optional device allocator used for every device allocation the call makes
       (results included).  Both must be set, or neither. */
    void *(*alloc)(size_t bytes, void *hip_stream, void *ctx);
    void (*free)(void *ptr, void *hip_stream, void *ctx);
    void *alloc_ctx;
} sign_opts;

/* Opaque result; owns its device buffers. */
typedef struct sign_result sign_result;

typedef struct {
    int status;          /* sign_status of the solve */
    int iters;           /* updates performed */
    int stagnated;       /* 1 if stopped because e_k stopped halving below 1e-8 */
    double scale;        /* c with X_1 = A/c */
    double res_fro;      /* e of the returned iterate, ||I - X^2||_F (or the certified
                            upper bound of it, see sign_iter_stats.e_bound) */
    double step_fro;     /* last ||Xbar_{k+1} - X^_k||_F */
    int64_t nnz;         /* nonzeros of the result */
    double seconds;      /* wall time of the call */
    int64_t products;    /* scalar multiply-adds in all sparse products */
    double spgemm_ms;    /* device time of the numeric product kernels */
    double spgemm_bytes; /* algorithmic bytes of the numeric product kernels: A and D rows,
                            B once per product, stored output, row descriptors */
    int inner_steps;     /* sign_newton: filtered NS inversion steps in total */
    double comm_rel;     /* precision 1: ||XA - AX||_F / (||X||_F ||A||_F) before refinement */
    /* the numeric product kernel configuration with the most device time */
    int hot_tile;        /* LDS accumulator columns of that kernel */
    int hot_threads;     /* its workgroup size */
    int hot_fp32;        /* 1 if it is the FP32-value instantiation */
    int hot_group;       /* output rows per workgroup: 1, or 2 / 4 for the grouped-row kernel */
    int64_t hot_launches;/* its launches */
    double hot_ms;       /* its device time (HIP events on the call's stream) */
    double hot_bytes;    /* its algorithmic bytes (as spgemm_bytes) */
    int64_t hot_products;/* its multiply-adds */
    int64_t hot_gathered;/* B entries it loads (one per multiply-add, or one per slot of the
                            merged list of a row group) */
    int hot_regtile;     /* 1 if it is the register-accumulator kernel (windows of hot_tile
                            columns, hot_group rows per workgroup) */
    int64_t madds;       /* multiply-adds the product kernels performed: a symmetric product
                            formed from its lower triangle stops each row at the diagonal, so
                            this is below `products` (which counts every entry of every
                            gathered B row) */
    int64_t hot_madds;   /* the hot kernel's share of madds */
    int hot_pages;       /* 1 if the hot kernel ran page windows (row groups sweeping only the
                            16-column pages their rows occupy) in most of its launches */
} sign_stats;

/* One entry per computed residual, k = 0 .. iters. */
typedef struct {
    double e;            /* ||I - X^_k^2||_F */
    double d;            /* ||Xbar_{k+1} - X^_k||_F (0 for the last entry) */
    double tau;          /* filter budget used for X^_{k+1} */
    double xfro;         /* ||X^_k||_F */
    double ffro;         /* ||F_{k+1}||_F, the dropped part */
    int64_t nnz_x;       /* nnz(X^_k) */
    int64_t nnz_r;       /* nnz(R^_k) */
    int64_t nnz_bar;     /* nnz(Xbar_{k+1}) */
    int bstar;           /* threshold bucket of X^_{k+1} */
    int fp32;            /* 1 if this step ran in FP32 */
    int e_bound;         /* 1: e is a certified upper bound of ||I - X^_k^2||_F,
                            ||I - Xt^2||_F + 2 ||Xt||_2 delta + delta^2 from a copy Xt
                            of X^_k thinned by delta <= tol/16 in Frobenius norm
                            (tried where Lemma 2.1.1 predicts convergence, and on the
                            first residual after the mixed mode's refinement; nnz_r is
                            then that of I - Xt^2, of its lower triangle when X^_k is
                            exactly symmetric; I - Xt^2 is not stored) */
    double ms;           /* wall time of the step */
} sign_iter_stats;

SIGNFN_API void sign_opts_default(sign_opts *o);

/* sign(A) by the filtered Newton-Schulz iteration, Algorithm 3.2.1:
 *   X^_1 = A/c;  while e_k > tol:  Xbar_{k+1} = 1/2 X^_k (3I - X^_k^2),
 *   X^_{k+1} = Xbar_{k+1} - F_{k+1},  e_{k+1} = ||I - X^_{k+1}^2||,
 * with ||F_{k+1}||_F held to the budget of Section 3.2 / eq. 1.18 (fixed
 * c_fixed*tol until e_k < switch_res).  A is borrowed for the duration of
 * the call.  On SIGN_OK, SIGN_ENOCONV and SIGN_EDIVERGED *out receives a
 * result (free with sign_result_free); on other errors *out is NULL. */
SIGNFN_API int sign_ns(const sign_csr *A, const sign_opts *o, void *hip_stream, sign_result **out);

/* sign(A) by the filtered Newton iteration, Algorithm 3.1.1:
 *   Xbar_{k+1} = 1/2 (X^_k + X^_k^{-1}),  X^_{k+1} = Xbar_{k+1} - F_{k+1},
 * with the budget of eq. 1.13 (fixed c_fixed*tol until e_k < switch_res).
 * The inverse is computed by filtered Newton-Schulz inversion
 * Z <- Z + Z (I - X^ Z) on the same product kernels.  Same ownership and
 * status rules as sign_ns; FP64 only. */
SIGNFN_API int sign_newton(const sign_csr *A, const sign_opts *o, void *hip_stream, sign_result **out);

/* Borrowed view of the result matrix (FP64 values, sorted columns, int64
 * row pointers, device memory); valid until sign_result_free. */
SIGNFN_API int sign_result_csr(const sign_result *r, sign_csr *view);
SIGNFN_API int sign_result_stats(const sign_result *r, sign_stats *s);
/* Per-iteration record k (0 <= k <= stats.iters); SIGN_EINVAL if out of range. */
SIGNFN_API int sign_result_trace(const sign_result *r, int k, sign_iter_stats *it);
SIGNFN_API void sign_result_free(sign_result *r);

/* Thread-local message of the last failing call ("" if none). */
SIGNFN_API const char *sign_last_error(void);

/* Device memory that the library keeps cached for reuse between calls (segments
 * no live result, server or call is using) goes back to the HIP allocator, so
 * that other allocators in the process (a framework's) can use it.  Returns the
 * bytes released.  Has nothing to release when the caller's alloc/free hooks
 * are in use.  Thread-safe; may be called at any time. */
SIGNFN_API size_t sign_release_cached(void);

/* ---- building blocks of the path, exposed for testing and reuse ---- */

/* C = A*B (sparse x sparse, FP64 or FP32 by the inputs' val_f32, which must
 * agree).  Sorted columns, exact zeros dropped.  Same ownership as sign_ns. */
SIGNFN_API int sign_spgemm(const sign_csr *A, const sign_csr *B, void *hip_stream, sign_result **out);

/* Drop from A the largest set of low-magnitude entries whose Frobenius norm
 * is provably <= tau (the element threshold of Section 3.1 for a norm
 * budget): entries are bucketed by |x| into 16 sub-buckets per binary octave
 * and the lowest buckets are dropped while sum(count_b * hi_b^2) <= tau^2.
 * *bstar receives the cut bucket.  FP64 or FP32 input; FP64 result. */
SIGNFN_API int sign_filter(const sign_csr *A, double tau, void *hip_stream, sign_result **out, int *bstar);

/* ---- allocation-free variant ---- */

/* Row limit of sign_filter_noalloc (its device scratch is sized for it). */
#define SIGN_NOALLOC_MAX_ROWS 1048576

/* For callers that cannot allocate device memory (serving loops and harnesses
 * that forbid hipMalloc): sign_filter into buffers the caller owns.  The call
 * makes no device allocation; the histogram, the cut, row lengths, per-row
 * sums and scan partials live in a fixed device array of the library (about
 * 16 MiB, held on each device it runs on until the process ends).
 *   A            device CSR as for sign_filter (FP64 or FP32 values), read in
 *                place; n <= SIGN_NOALLOC_MAX_ROWS, else SIGN_EINVAL
 *   out          caller's DEVICE buffers: out->row_ptr int64[n+1], out->col
 *                int32[out_capacity], out->val double[out_capacity]; on
 *                SIGN_OK out->n, out->nnz and out->val_f32 = 0 are set
 *   out_capacity entries out->col/out->val can hold (A->nnz always suffices);
 *                if fewer entries are kept than needed: SIGN_ENOMEM, with
 *                out->row_ptr overwritten and col/val untouched
 *   bstar        (optional) receives the cut bucket
 *   dropped_fro  (optional) receives ||F||_F of the dropped entries
 * Same entries, values and cut as sign_filter.  Synchronises the stream (the
 * kept count is read back), so it cannot be captured into a graph.  Calls on
 * one device share its scratch array: calls that overlap on one device race
 * and must be serialised by the caller. */
SIGNFN_API int sign_filter_noalloc(const sign_csr *A, double tau, void *hip_stream, sign_csr *out,
                                   int64_t out_capacity, int *bstar, double *dropped_fro);

/* ---- serving: continuous batching of many sign_ns solves ---- */
typedef struct sign_server sign_server;

typedef struct {
    int device;              /* HIP device the server runs on */
    size_t hbm_budget_bytes; /* admission budget for resident iterates; 0 = automatic */
    int max_slots;           /* maximum requests advanced together; 0 = 64 */
    int max_queue;           /* maximum queued requests; 0 = 100000 */
    size_t mem_limit_bytes;  /* hard cap on the device memory of the batch (iterates,
                                residuals, product staging); 0 = none.  A tick that
                                would exceed it fails only the request with the most
                                resident entries (SIGN_ENOMEM); the others go on */
} sign_server_opts;

SIGNFN_API int sign_server_create(const sign_server_opts *o, sign_server **s);

/* Enqueue sign_ns(A) with options o.  Here the sign_csr pointers are HOST
 * pointers: the server copies A before returning, so the caller may free it
 * at once.  Options are copied; precision 1 and the allocator hooks are not
 * supported by the server (SIGN_EINVAL).  *ticket identifies the request. */
SIGNFN_API int sign_serve_submit(sign_server *s, const sign_csr *A_host, const sign_opts *o,
                      uint64_t *ticket);

/* SIGN_PENDING while the request runs; otherwise the request's final status,
 * and *out receives its result (device memory on the server's device; the
 * caller frees it with sign_result_free).  A ticket can be collected once. */
SIGNFN_API int sign_serve_poll(sign_server *s, uint64_t ticket, sign_result **out);

typedef struct {
    int64_t submitted, completed, active, queued;
    double p50_ms, p99_ms;     /* latency submit -> result ready, completed requests */
    double busy_seconds;       /* time with at least one request on the device */
    int64_t ticks;             /* batched iterations launched */
    int64_t max_active;        /* most requests advanced together */
    int64_t failed;            /* requests that ended with an error */
    /* wall time of the worker by phase (each phase ends when the device has
       finished it): admission and batch relayout, residual products with
       their norms and certifications, update products, filters/mirroring */
    double relayout_seconds, residual_seconds, update_seconds, filter_seconds;
} sign_server_stats;

SIGNFN_API int sign_server_stats_get(sign_server *s, sign_server_stats *st);
SIGNFN_API void sign_server_destroy(sign_server *s);

#ifdef __cplusplus
}
#endif

#endif /* SIGNFN_H */
