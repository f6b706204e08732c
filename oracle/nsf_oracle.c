/*
 * FP64 CPU oracle for the filtered Newton-Schulz (NSF, Algorithm 3.2.1) and
 * filtered Newton (NMF, Algorithm 3.1.1) matrix sign iterations.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * HIP library is checked against.  Only the test suite, the smoke check and
 * the benchmark's CPU-baseline leg may load it.  It shares no code, header,
 * table or constant with the HIP library.
 *
 * Everything is scalar FP64 on CSR matrices (int64 row pointers, int32 sorted
 * column indices, no stored zeros -- the sparse storage of Section 4).  The
 * only parallelism is OpenMP over independent output rows of a product; the
 * arithmetic inside a row is the textbook order, so results do not depend on
 * the thread count.  Norm sums run serially in storage order.
 *
 * Readings of the paper taken here (the paper leaves these open):
 *   - every norm is the Frobenius norm;
 *   - the element threshold is obtained from the norm budget tau by bucketing
 *     |x| into 16 sub-buckets per binary octave and dropping the largest set
 *     of low buckets whose bound sum(count_b * hi_b^2) stays <= tau^2 (the
 *     selection algorithm itself is delegated by Section 3.1 to an external
 *     reference);
 *   - X_1 = A / ||A||_inf for NSF (Section 2: NS converges only when
 *     ||I - X_1^2|| < 1);
 *   - the eq. 1.18 budget uses the last known filtered quantities R^_k, X^_k;
 *   - the update is evaluated as X^_k + 1/2 X^_k (I - X^_k^2), algebraically
 *     the same as 1/2 X^_k (3I - X^_k^2) of Algorithm 3.2.1.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -shared -fPIC nsf_oracle.c -lm
 */
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* CSR container                                                             */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t n;
    int64_t *rp;   /* n+1 */
    int32_t *ci;   /* nnz, ascending within a row */
    double  *v;    /* nnz, never exactly zero */
} ocsr;

static void ocsr_free(ocsr *m) {
    free(m->rp); free(m->ci); free(m->v);
    m->rp = NULL; m->ci = NULL; m->v = NULL;
}

static int ocsr_alloc(ocsr *m, int64_t n, int64_t nnz) {
    m->n = n;
    m->rp = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    m->ci = (int32_t *)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int32_t));
    m->v = (double *)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(double));
    if (!m->rp || !m->ci || !m->v) { ocsr_free(m); return -1; }
    return 0;
}

static int64_t ocsr_nnz(const ocsr *m) { return m->rp[m->n]; }

static int ocsr_copy_scaled(const ocsr *a, double s, ocsr *out) {
    int64_t nnz = ocsr_nnz(a);
    if (ocsr_alloc(out, a->n, nnz)) return -1;
    memcpy(out->rp, a->rp, sizeof(int64_t) * (size_t)(a->n + 1));
    memcpy(out->ci, a->ci, sizeof(int32_t) * (size_t)nnz);
    for (int64_t p = 0; p < nnz; ++p) out->v[p] = a->v[p] * s;
    return 0;
}

static int ocsr_identity(int64_t n, ocsr *out) {
    if (ocsr_alloc(out, n, n)) return -1;
    for (int64_t i = 0; i < n; ++i) {
        out->rp[i] = i; out->ci[i] = (int32_t)i; out->v[i] = 1.0;
    }
    out->rp[n] = n;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Plain matrix operations                                                   */
/* ------------------------------------------------------------------------ */

/* ||A||_inf = max_i sum_j |a_ij| */
static double norm_inf(const ocsr *a) {
    double best = 0.0;
    for (int64_t i = 0; i < a->n; ++i) {
        double s = 0.0;
        for (int64_t p = a->rp[i]; p < a->rp[i + 1]; ++p) s += fabs(a->v[p]);
        if (s > best) best = s;
    }
    return best;
}

/* ||A||_1 = max_j sum_i |a_ij| */
static double norm_one(const ocsr *a) {
    double *col = (double *)calloc((size_t)a->n, sizeof(double));
    double best = 0.0;
    for (int64_t p = 0; p < ocsr_nnz(a); ++p) col[a->ci[p]] += fabs(a->v[p]);
    for (int64_t j = 0; j < a->n; ++j) if (col[j] > best) best = col[j];
    free(col);
    return best;
}

/* sum of squares of all stored values, serial in storage order */
static double sumsq(const ocsr *a) {
    double s = 0.0;
    for (int64_t p = 0; p < ocsr_nnz(a); ++p) s += a->v[p] * a->v[p];
    return s;
}

static int cmp_i32(const void *x, const void *y) {
    int32_t a = *(const int32_t *)x, b = *(const int32_t *)y;
    return (a > b) - (a < b);
}

/* C = A * B by Gustavson's row-wise method with a dense accumulator.
 * Row i of C is sum_k a_ik * (row k of B), accumulated in the order the
 * entries of row i of A are stored.  Exact zeros are not stored. */
static int matmul(const ocsr *A, const ocsr *B, ocsr *C) {
    const int64_t n = A->n;
    int64_t *cnt = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    int32_t **rc = (int32_t **)calloc((size_t)n, sizeof(int32_t *));
    double **rv = (double **)calloc((size_t)n, sizeof(double *));
    int failed = 0;
    if (!cnt || !rc || !rv) { free(cnt); free(rc); free(rv); return -1; }
#pragma omp parallel
    {
        double *acc = (double *)calloc((size_t)B->n, sizeof(double));
        unsigned char *mark = (unsigned char *)calloc((size_t)B->n, 1);
        int32_t *list = (int32_t *)malloc(sizeof(int32_t) * (size_t)(B->n > 0 ? B->n : 1));
        if (!acc || !mark || !list) {
#pragma omp atomic write
            failed = 1;
        } else {
#pragma omp for schedule(dynamic, 16)
            for (int64_t i = 0; i < n; ++i) {
                int64_t nl = 0;
                for (int64_t p = A->rp[i]; p < A->rp[i + 1]; ++p) {
                    const int32_t k = A->ci[p];
                    const double a = A->v[p];
                    for (int64_t q = B->rp[k]; q < B->rp[k + 1]; ++q) {
                        const int32_t j = B->ci[q];
                        if (!mark[j]) { mark[j] = 1; acc[j] = 0.0; list[nl++] = j; }
                        acc[j] += a * B->v[q];
                    }
                }
                qsort(list, (size_t)nl, sizeof(int32_t), cmp_i32);
                int64_t keep = 0;
                for (int64_t t = 0; t < nl; ++t) if (acc[list[t]] != 0.0) ++keep;
                rc[i] = (int32_t *)malloc(sizeof(int32_t) * (size_t)(keep > 0 ? keep : 1));
                rv[i] = (double *)malloc(sizeof(double) * (size_t)(keep > 0 ? keep : 1));
                if (!rc[i] || !rv[i]) {
#pragma omp atomic write
                    failed = 1;
                }
                int64_t w = 0;
                for (int64_t t = 0; t < nl; ++t) {
                    const int32_t j = list[t];
                    if (acc[j] != 0.0 && rc[i] && rv[i]) { rc[i][w] = j; rv[i][w] = acc[j]; ++w; }
                    mark[j] = 0;
                }
                cnt[i] = keep;
            }
        }
        free(acc); free(mark); free(list);
    }
    int64_t total = 0;
    for (int64_t i = 0; i < n; ++i) total += cnt[i];
    if (!failed && ocsr_alloc(C, n, total) == 0) {
        int64_t off = 0;
        for (int64_t i = 0; i < n; ++i) {
            C->rp[i] = off;
            if (cnt[i]) {
                memcpy(C->ci + off, rc[i], sizeof(int32_t) * (size_t)cnt[i]);
                memcpy(C->v + off, rv[i], sizeof(double) * (size_t)cnt[i]);
            }
            off += cnt[i];
        }
        C->rp[n] = off;
    } else {
        failed = 1;
    }
    for (int64_t i = 0; i < n; ++i) { free(rc[i]); free(rv[i]); }
    free(cnt); free(rc); free(rv);
    return failed ? -1 : 0;
}

/* C = alpha*A + beta*B, merging sorted rows; exact zeros are not stored. */
static int add(double alpha, const ocsr *A, double beta, const ocsr *B, ocsr *C) {
    const int64_t n = A->n;
    if (ocsr_alloc(C, n, ocsr_nnz(A) + ocsr_nnz(B))) return -1;
    int64_t w = 0;
    for (int64_t i = 0; i < n; ++i) {
        C->rp[i] = w;
        int64_t p = A->rp[i], pe = A->rp[i + 1], q = B->rp[i], qe = B->rp[i + 1];
        while (p < pe || q < qe) {
            int32_t j;
            double v;
            if (q >= qe || (p < pe && A->ci[p] < B->ci[q])) {
                j = A->ci[p]; v = alpha * A->v[p]; ++p;
            } else if (p >= pe || B->ci[q] < A->ci[p]) {
                j = B->ci[q]; v = beta * B->v[q]; ++q;
            } else {
                j = A->ci[p]; v = alpha * A->v[p] + beta * B->v[q]; ++p; ++q;
            }
            if (v != 0.0) { C->ci[w] = j; C->v[w] = v; ++w; }
        }
    }
    C->rp[n] = w;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Element threshold from a Frobenius-norm budget                            */
/* ------------------------------------------------------------------------ */
#define ORB_COUNT 2048   /* histogram size; buckets 0..ORB_TOP are used */
#define ORB_TOP 2033     /* |x| >= 1: never dropped */

/* Bucket of |x|: 0 below 2^-127; ORB_TOP at or above 1; otherwise
 * 1 + 16*(E + 127) + j where |x| = 2^E * (1 + f), 0 <= f < 1, and j = floor(16 f). */
int oracle_bucket(double x) {
    const double a = fabs(x);
    if (a >= 1.0) return ORB_TOP;
    if (a == 0.0) return 0;
    int e2;
    const double fr = frexp(a, &e2);      /* a = fr * 2^e2, fr in [0.5, 1) */
    const int E = e2 - 1;                 /* a = (2 fr) * 2^E, 2 fr in [1, 2) */
    if (E < -127) return 0;
    const int j = (int)floor((2.0 * fr - 1.0) * 16.0);
    return 1 + 16 * (E + 127) + j;
}

/* Upper edge of bucket b: every |x| in bucket b satisfies |x| < hi(b). */
double oracle_bucket_hi(int b) {
    if (b <= 0) return ldexp(1.0, -127);
    if (b >= ORB_TOP) return INFINITY;
    const int E = (b - 1) / 16 - 127;
    const int j = (b - 1) % 16;
    return ldexp(1.0 + (double)(j + 1) / 16.0, E);
}

/* Lower edge of bucket b (the element threshold eps when b is the cut). */
double oracle_bucket_lo(int b) {
    if (b <= 0) return 0.0;
    if (b >= ORB_TOP) return 1.0;
    const int E = (b - 1) / 16 - 127;
    const int j = (b - 1) % 16;
    return ldexp(1.0 + (double)j / 16.0, E);
}

/* Cut bucket b*: the largest b <= ORB_TOP with
 *     sum_{b' < b} count[b'] * hi(b')^2 <= tau^2,
 * accumulated in ascending b.  Entries in buckets below b* are dropped, so the
 * dropped part F satisfies ||F||_F^2 <= sum count*hi^2 <= tau^2. */
int oracle_select(const uint64_t *count, double tau) {
    const double t2 = tau * tau;
    double s = 0.0;
    int b = 0;
    while (b < ORB_TOP) {
        const double h = oracle_bucket_hi(b);
        const double hh = h * h;
        const double add_b = (double)count[b] * hh;
        if (s + add_b > t2) break;
        s = s + add_b;
        ++b;
    }
    return b;
}

static void histogram(const ocsr *a, uint64_t *count) {
    memset(count, 0, sizeof(uint64_t) * ORB_COUNT);
    for (int64_t p = 0; p < ocsr_nnz(a); ++p) count[oracle_bucket(a->v[p])]++;
}

/* Drop every entry whose bucket is below bstar.  Returns the sum of squares of
 * the dropped entries in *dropped_sq. */
static int filter(const ocsr *a, int bstar, ocsr *out, double *dropped_sq) {
    if (ocsr_alloc(out, a->n, ocsr_nnz(a))) return -1;
    int64_t w = 0;
    double dsq = 0.0;
    for (int64_t i = 0; i < a->n; ++i) {
        out->rp[i] = w;
        for (int64_t p = a->rp[i]; p < a->rp[i + 1]; ++p) {
            const double v = a->v[p];
            if (v != 0.0 && oracle_bucket(v) >= bstar) {
                out->ci[w] = a->ci[p]; out->v[w] = v; ++w;
            } else {
                dsq += v * v;
            }
        }
    }
    out->rp[a->n] = w;
    *dropped_sq = dsq;
    return 0;
}

/* Filtering of a whole matrix with budget tau: select the cut, then drop. */
static int filter_budget(const ocsr *a, double tau, ocsr *out, int *bstar, double *dropped_sq) {
    uint64_t count[ORB_COUNT];
    histogram(a, count);
    *bstar = oracle_select(count, tau);
    return filter(a, *bstar, out, dropped_sq);
}

/* ------------------------------------------------------------------------ */
/* Options, results                                                          */
/* ------------------------------------------------------------------------ */
enum { OR_OK = 0, OR_EINVAL = -1, OR_ENOMEM = -2, OR_ENOCONV = -3, OR_EDIVERGED = -4 };

typedef struct {
    double tol;         /* epsilon_tol */
    int stop_rule;      /* 0: stop when e_k <= tol; 1: stop when d_{k-1} < tol */
    double c_fixed;     /* c4 (NSF) or c2 (NMF): fixed budget c*tol while e_k >= switch_res */
    double switch_res;  /* switch to the adaptive budget once e_k < switch_res */
    int max_iter;       /* at most this many updates */
    int filter_y;       /* also filter R^_k = I - X^_k^2 with the same budget (NSF) */
    double scale;       /* X_1 = A/scale; 0 selects ||A||_inf */
    int nthreads;       /* OpenMP threads; 0 keeps the runtime default */
    int trace_cap;      /* length of the per-iteration trace arrays */
} or_opts;

typedef struct {
    int64_t n, nnz;
    int64_t *rp;
    int32_t *ci;
    double *v;
    int status, iters, stagnated;
    double scale;
    double res_fro;    /* e of the returned iterate */
    double step_fro;   /* last d_k */
    /* trace, one entry per computed residual (index k-1) */
    double *e, *d, *tau, *xfro, *ffro;
    int64_t *nnz_x, *nnz_bar, *nnz_r;
    int *bstar;
    int64_t inner_total; /* NMF: filtered NS inverse steps in total */
} or_result;

static void trace_alloc(or_result *r, int cap) {
    r->e = (double *)calloc((size_t)cap, sizeof(double));
    r->d = (double *)calloc((size_t)cap, sizeof(double));
    r->tau = (double *)calloc((size_t)cap, sizeof(double));
    r->xfro = (double *)calloc((size_t)cap, sizeof(double));
    r->ffro = (double *)calloc((size_t)cap, sizeof(double));
    r->nnz_x = (int64_t *)calloc((size_t)cap, sizeof(int64_t));
    r->nnz_bar = (int64_t *)calloc((size_t)cap, sizeof(int64_t));
    r->nnz_r = (int64_t *)calloc((size_t)cap, sizeof(int64_t));
    r->bstar = (int *)calloc((size_t)cap, sizeof(int));
}

void oracle_free_result(or_result *r) {
    free(r->rp); free(r->ci); free(r->v);
    free(r->e); free(r->d); free(r->tau); free(r->xfro); free(r->ffro);
    free(r->nnz_x); free(r->nnz_bar); free(r->nnz_r); free(r->bstar);
    memset(r, 0, sizeof(*r));
}

static void hand_over(ocsr *X, or_result *r) {
    r->n = X->n; r->nnz = ocsr_nnz(X);
    r->rp = X->rp; r->ci = X->ci; r->v = X->v;
    X->rp = NULL; X->ci = NULL; X->v = NULL;
}

static int wrap_input(int64_t n, const int64_t *rp, const int32_t *ci, const double *v, ocsr *A) {
    A->n = n;
    A->rp = (int64_t *)rp; A->ci = (int32_t *)ci; A->v = (double *)v;
    if (n <= 0 || rp[0] != 0) return -1;
    for (int64_t i = 0; i < n; ++i) {
        if (rp[i + 1] < rp[i]) return -1;
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
            if (ci[p] < 0 || ci[p] >= n) return -1;
            if (p > rp[i] && ci[p] <= ci[p - 1]) return -1;
            if (!isfinite(v[p])) return -1;
        }
    }
    return 0;
}

/* Progress lines on stderr when ORACLE_PROGRESS=1 (long full-size runs). */
static int progress_on(void) {
    const char *p = getenv("ORACLE_PROGRESS");
    return p && p[0] == '1';
}

static void progress(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    fputs("[oracle] ", stderr);
    vfprintf(stderr, fmt, ap);
    fputc('\n', stderr);
    fflush(stderr);
    va_end(ap);
}

/* Budget of eq. 1.18 after the switch (A4 reading), fixed budget before it. */
double oracle_nsf_budget(double e, double xfro, double tol, double c_fixed, double switch_res) {
    if (e >= switch_res) return c_fixed * tol;
    return 0.75 * e * e / (3.0 * xfro + xfro * xfro * xfro);
}

/* Budget of eq. 1.13 after the switch, fixed budget before it (NMF). */
double oracle_nmf_budget(double e, double xfro, double zfro, double tol, double c_fixed,
                         double switch_res) {
    if (e >= switch_res) return c_fixed * tol;
    return e * e / (xfro + zfro);
}

/* Guards shared by both iterations.  Returns 1 to stop (status in *st). */
static int guards(int k, const double *e, int stop_rule, double tol, int max_iter,
                  int *n_up, int *n_flat, int *st, int *stagnated) {
    const double ek = e[k - 1];
    if (!isfinite(ek)) { *st = OR_EDIVERGED; return 1; }
    if (k >= 2) {
        const double ep = e[k - 2];
        *n_up = (ek > ep && ek > 1.0) ? *n_up + 1 : 0;
        if (*n_up >= 3) { *st = OR_EDIVERGED; return 1; }
        *n_flat = (ek < 1e-8 && ek > 0.5 * ep) ? *n_flat + 1 : 0;
        if (*n_flat >= 2) { *st = OR_OK; *stagnated = 1; return 1; }
    }
    (void)stop_rule; (void)tol;
    if (k - 1 >= max_iter) { *st = OR_ENOCONV; return 1; }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* NSF: Algorithm 3.2.1                                                      */
/* ------------------------------------------------------------------------ */
int oracle_nsf(int64_t n, const int64_t *rp, const int32_t *ci, const double *v,
               const or_opts *o, or_result *res) {
    memset(res, 0, sizeof(*res));
    ocsr A;
    if (!o || o->tol <= 0.0 || o->max_iter < 0 || wrap_input(n, rp, ci, v, &A)) {
        res->status = OR_EINVAL;
        return OR_EINVAL;
    }
#ifdef _OPENMP
    if (o->nthreads > 0) omp_set_num_threads(o->nthreads);
#endif
    const int cap = o->trace_cap > o->max_iter + 2 ? o->trace_cap : o->max_iter + 2;
    trace_alloc(res, cap);

    /* step 1: X^_1 = A / c with c = ||A||_inf */
    const double c = o->scale > 0.0 ? o->scale : norm_inf(&A);
    res->scale = c;
    if (!(c > 0.0)) { res->status = OR_EINVAL; return OR_EINVAL; }
    ocsr X = {0}, I = {0};
    if (ocsr_copy_scaled(&A, 1.0 / c, &X) || ocsr_identity(n, &I)) goto oom;

    int status = OR_OK, n_up = 0, n_flat = 0;
    double d_prev = INFINITY;
    for (int k = 1;; ++k) {
        ocsr Y = {0}, R = {0}, P = {0}, Xbar = {0}, Xn = {0};
        /* residual of the current iterate: R^_k = I - X^_k^2, e_k = ||R^_k||_F */
        if (matmul(&X, &X, &Y) || add(1.0, &I, -1.0, &Y, &R)) { ocsr_free(&Y); goto oom; }
        ocsr_free(&Y);
        const double e = sqrt(sumsq(&R));
        const double xf = sqrt(sumsq(&X));
        if (k - 1 < cap) {
            res->e[k - 1] = e; res->xfro[k - 1] = xf;
            res->nnz_x[k - 1] = ocsr_nnz(&X); res->nnz_r[k - 1] = ocsr_nnz(&R);
        }
        res->iters = k - 1;
        res->res_fro = e;
        if (progress_on())
            progress("nsf k=%d e=%.3e nnz(X)=%lld nnz(R)=%lld", k, e, (long long)ocsr_nnz(&X),
                     (long long)ocsr_nnz(&R));
        /* convergence test of the while loop */
        const int conv = (o->stop_rule == 1) ? (d_prev < o->tol) : (e <= o->tol);
        if (conv) { ocsr_free(&R); status = OR_OK; break; }
        if (k - 1 < cap && guards(k, res->e, o->stop_rule, o->tol, o->max_iter, &n_up, &n_flat,
                                  &status, &res->stagnated)) {
            ocsr_free(&R); break;
        }
        /* filter budget for X^_{k+1} */
        const double tau = oracle_nsf_budget(e, xf, o->tol, o->c_fixed, o->switch_res);
        if (o->filter_y) {
            ocsr Rf = {0};
            int bs; double dsq;
            if (filter_budget(&R, tau, &Rf, &bs, &dsq)) { ocsr_free(&R); goto oom; }
            ocsr_free(&R);
            R = Rf;
        }
        /* step 3: Xbar_{k+1} = X^_k + 1/2 X^_k R^_k */
        if (matmul(&X, &R, &P)) { ocsr_free(&R); goto oom; }
        ocsr_free(&R);
        if (progress_on()) progress("nsf k=%d product X R: %lld entries", k, (long long)ocsr_nnz(&P));
        if (add(1.0, &X, 0.5, &P, &Xbar)) { ocsr_free(&P); goto oom; }
        const double d = 0.5 * sqrt(sumsq(&P));
        ocsr_free(&P);
        /* step 4: X^_{k+1} = Xbar_{k+1} - F_{k+1} */
        int bstar; double dsq;
        if (filter_budget(&Xbar, tau, &Xn, &bstar, &dsq)) { ocsr_free(&Xbar); goto oom; }
        if (k - 1 < cap) {
            res->d[k - 1] = d; res->tau[k - 1] = tau; res->bstar[k - 1] = bstar;
            res->ffro[k - 1] = sqrt(dsq); res->nnz_bar[k - 1] = ocsr_nnz(&Xbar);
        }
        ocsr_free(&Xbar);
        ocsr_free(&X);
        X = Xn;
        d_prev = d;
        res->step_fro = d;
    }
    ocsr_free(&I);
    hand_over(&X, res);
    res->status = status;
    return status;
oom:
    ocsr_free(&X); ocsr_free(&I);
    res->status = OR_ENOMEM;
    return OR_ENOMEM;
}

/* ------------------------------------------------------------------------ */
/* Single products exposed for product-level checks                          */
/* ------------------------------------------------------------------------ */

/* C = A*B for square n x n CSR inputs; result arrays are malloc'd and owned by
 * the caller (free with oracle_free_csr). */
int oracle_spgemm(int64_t n, const int64_t *arp, const int32_t *aci, const double *av,
                  const int64_t *brp, const int32_t *bci, const double *bv,
                  int64_t **crp, int32_t **cci, double **cv, int64_t *cnnz) {
    ocsr A = {n, (int64_t *)arp, (int32_t *)aci, (double *)av};
    ocsr B = {n, (int64_t *)brp, (int32_t *)bci, (double *)bv};
    ocsr C = {0};
    if (matmul(&A, &B, &C)) return OR_ENOMEM;
    *crp = C.rp; *cci = C.ci; *cv = C.v; *cnnz = ocsr_nnz(&C);
    return OR_OK;
}

void oracle_free_csr(int64_t *rp, int32_t *ci, double *v) { free(rp); free(ci); free(v); }

/* One unfiltered NS update X -> X + 1/2 X (I - X^2) (Section 2). */
int oracle_ns_step(int64_t n, const int64_t *rp, const int32_t *ci, const double *v,
                   int64_t **orp, int32_t **oci, double **ov, int64_t *onnz) {
    ocsr X = {n, (int64_t *)rp, (int32_t *)ci, (double *)v};
    ocsr I = {0}, Y = {0}, R = {0}, P = {0}, Xn = {0};
    if (ocsr_identity(n, &I) || matmul(&X, &X, &Y) || add(1.0, &I, -1.0, &Y, &R) ||
        matmul(&X, &R, &P) || add(1.0, &X, 0.5, &P, &Xn)) {
        ocsr_free(&I); ocsr_free(&Y); ocsr_free(&R); ocsr_free(&P); ocsr_free(&Xn);
        return OR_ENOMEM;
    }
    ocsr_free(&I); ocsr_free(&Y); ocsr_free(&R); ocsr_free(&P);
    *orp = Xn.rp; *oci = Xn.ci; *ov = Xn.v; *onnz = ocsr_nnz(&Xn);
    return OR_OK;
}

/* Histogram + cut + drop on a value array, for selection checks. */
int oracle_filter_values(int64_t m, const double *vals, double tau, unsigned char *keep,
                         double *dropped_sq) {
    uint64_t count[ORB_COUNT];
    memset(count, 0, sizeof(count));
    for (int64_t p = 0; p < m; ++p) count[oracle_bucket(vals[p])]++;
    const int bstar = oracle_select(count, tau);
    double dsq = 0.0;
    for (int64_t p = 0; p < m; ++p) {
        keep[p] = (unsigned char)(vals[p] != 0.0 && oracle_bucket(vals[p]) >= bstar);
        if (!keep[p]) dsq += vals[p] * vals[p];
    }
    *dropped_sq = dsq;
    return bstar;
}

double oracle_norm_inf(int64_t n, const int64_t *rp, const int32_t *ci, const double *v) {
    ocsr A = {n, (int64_t *)rp, (int32_t *)ci, (double *)v};
    return norm_inf(&A);
}
double oracle_norm_one(int64_t n, const int64_t *rp, const int32_t *ci, const double *v) {
    ocsr A = {n, (int64_t *)rp, (int32_t *)ci, (double *)v};
    return norm_one(&A);
}

/* ------------------------------------------------------------------------ */
/* NMF: Algorithm 3.1.1, with the inverse computed by filtered Newton-Schulz  */
/* inversion Z <- Z + Z (I - X Z) (the paper's large-scale runs also use a    */
/* filtered inverse, Section 4.4).                                           */
/* ------------------------------------------------------------------------ */

/* ||I - X Z||_F, also returning T = I - X Z when wanted. */
static int inv_residual(const ocsr *X, const ocsr *Z, const ocsr *I, ocsr *T, double *fro) {
    ocsr XZ = {0};
    if (matmul(X, Z, &XZ) || add(1.0, I, -1.0, &XZ, T)) { ocsr_free(&XZ); return -1; }
    ocsr_free(&XZ);
    *fro = sqrt(sumsq(T));
    return 0;
}

/* Transpose of a CSR matrix (sorted columns in the result). */
static int transpose(const ocsr *a, ocsr *t) {
    const int64_t n = a->n, nnz = ocsr_nnz(a);
    if (ocsr_alloc(t, n, nnz)) return -1;
    for (int64_t p = 0; p < nnz; ++p) t->rp[a->ci[p] + 1]++;
    for (int64_t j = 0; j < n; ++j) t->rp[j + 1] += t->rp[j];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!fill) { ocsr_free(t); return -1; }
    memcpy(fill, t->rp, sizeof(int64_t) * (size_t)n);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t p = a->rp[i]; p < a->rp[i + 1]; ++p) {
            const int64_t w = fill[a->ci[p]]++;
            t->ci[w] = (int32_t)i; t->v[w] = a->v[p];
        }
    free(fill);
    return 0;
}

/* Filtered Newton-Schulz inverse of X.  Z (in/out) holds the warm start on
 * entry when *warm is set; on exit Z approximates X^{-1} with
 * ||I - X Z||_F <= target, or the step cap was reached.  Each iterate is
 * filtered with the fixed budget tau_z.  Returns the number of steps. */
static int ns_inverse(const ocsr *X, const ocsr *I, ocsr *Z, int warm, double target, double tau_z,
                      int max_steps, int *err) {
    *err = 0;
    ocsr T = {0};
    double r;
    if (warm) {
        if (inv_residual(X, Z, I, &T, &r)) { *err = 1; return 0; }
        if (!(r < 0.5)) { warm = 0; ocsr_free(&T); ocsr_free(Z); }
    }
    if (!warm) {
        /* Z_0 = X^T / (||X||_1 ||X||_inf): ||I - X Z_0||_2 < 1 for nonsingular X */
        ocsr Xt = {0};
        const double s = norm_one(X) * norm_inf(X);
        if (transpose(X, &Xt) || ocsr_copy_scaled(&Xt, 1.0 / s, Z)) { ocsr_free(&Xt); *err = 1; return 0; }
        ocsr_free(&Xt);
        if (inv_residual(X, Z, I, &T, &r)) { *err = 1; return 0; }
    }
    int steps = 0;
    double r_prev = INFINITY;
    /* stop at the target, at the step cap, or once rounding stalls the
     * quadratic convergence (no halving below 1e-8) */
    while (r > target && steps < max_steps && !(r < 1e-8 && r > 0.5 * r_prev)) {
        r_prev = r;
        ocsr ZT = {0}, Zbar = {0}, Zn = {0};
        int bs; double dsq;
        if (matmul(Z, &T, &ZT) || add(1.0, Z, 1.0, &ZT, &Zbar) ||
            filter_budget(&Zbar, tau_z, &Zn, &bs, &dsq)) {
            ocsr_free(&ZT); ocsr_free(&Zbar); ocsr_free(&T); *err = 1; return steps;
        }
        ocsr_free(&ZT); ocsr_free(&Zbar); ocsr_free(Z);
        *Z = Zn;
        ocsr_free(&T);
        if (inv_residual(X, Z, I, &T, &r)) { *err = 1; return steps; }
        ++steps;
        if (!isfinite(r)) break;
    }
    ocsr_free(&T);
    return steps;
}

int oracle_nmf(int64_t n, const int64_t *rp, const int32_t *ci, const double *v,
               const or_opts *o, or_result *res) {
    memset(res, 0, sizeof(*res));
    ocsr A;
    if (!o || o->tol <= 0.0 || o->max_iter < 0 || wrap_input(n, rp, ci, v, &A)) {
        res->status = OR_EINVAL;
        return OR_EINVAL;
    }
#ifdef _OPENMP
    if (o->nthreads > 0) omp_set_num_threads(o->nthreads);
#endif
    const int cap = o->trace_cap > o->max_iter + 2 ? o->trace_cap : o->max_iter + 2;
    trace_alloc(res, cap);
    /* step 1: X^_1 = A (optionally scaled) */
    const double c = o->scale > 0.0 ? o->scale : norm_inf(&A);
    res->scale = c;
    ocsr X = {0}, I = {0}, Z = {0};
    if (ocsr_copy_scaled(&A, 1.0 / c, &X) || ocsr_identity(n, &I)) goto oom;
    int status = OR_OK, n_up = 0, n_flat = 0, have_z = 0;
    for (int k = 1;; ++k) {
        ocsr Y = {0}, R = {0}, Xbar = {0}, Xn = {0};
        /* step 5 (and step 1): R^_k = I - X^_k^2, e_k = ||R^_k||_F */
        if (matmul(&X, &X, &Y) || add(1.0, &I, -1.0, &Y, &R)) { ocsr_free(&Y); goto oom; }
        ocsr_free(&Y);
        const double e = sqrt(sumsq(&R));
        ocsr_free(&R);
        const double xf = sqrt(sumsq(&X));
        res->e[k - 1] = e; res->xfro[k - 1] = xf; res->nnz_x[k - 1] = ocsr_nnz(&X);
        res->iters = k - 1;
        res->res_fro = e;
        /* step 2: while e_k > tol */
        if (e <= o->tol) { status = OR_OK; break; }
        if (guards(k, res->e, 0, o->tol, o->max_iter, &n_up, &n_flat, &status, &res->stagnated))
            break;
        /* inverse of X^_k by filtered NS inversion, converged to the tolerance:
         * an inexact inverse that is not a function of X^_k would move the
         * limit of the outer iteration away from sign(A) */
        const double target = 0.1 * o->tol;
        int err = 0;
        res->inner_total += ns_inverse(&X, &I, &Z, have_z, target, o->c_fixed * o->tol, 200, &err);
        if (err) goto oom;
        have_z = 1;
        const double zf = sqrt(sumsq(&Z));
        /* step 3: Xbar_{k+1} = 1/2 (X^_k + X^_k^{-1}) */
        if (add(0.5, &X, 0.5, &Z, &Xbar)) goto oom;
        /* step 4: X^_{k+1} = Xbar_{k+1} - F_{k+1}, budget eq. 1.13 / fixed c2*tol */
        const double tau = oracle_nmf_budget(e, xf, zf, o->tol, o->c_fixed, o->switch_res);
        int bstar; double dsq;
        if (filter_budget(&Xbar, tau, &Xn, &bstar, &dsq)) { ocsr_free(&Xbar); goto oom; }
        res->tau[k - 1] = tau; res->bstar[k - 1] = bstar; res->ffro[k - 1] = sqrt(dsq);
        res->nnz_bar[k - 1] = ocsr_nnz(&Xbar);
        {
            ocsr D = {0};
            if (add(1.0, &Xn, -1.0, &X, &D)) { ocsr_free(&Xbar); ocsr_free(&Xn); goto oom; }
            res->d[k - 1] = sqrt(sumsq(&D));
            res->step_fro = res->d[k - 1];
            ocsr_free(&D);
        }
        ocsr_free(&Xbar);
        ocsr_free(&X);
        X = Xn;
    }
    ocsr_free(&I); ocsr_free(&Z);
    hand_over(&X, res);
    res->status = status;
    return status;
oom:
    ocsr_free(&X); ocsr_free(&I); ocsr_free(&Z);
    res->status = OR_ENOMEM;
    return OR_ENOMEM;
}
