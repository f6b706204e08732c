// C ABI of libsignfn (declared in include/signfn.h).
#include <cmath>
#include <cstring>

#include "driver.hpp"

using namespace sfn;

namespace {

template <typename F>
int guarded(F &&f) {
    try {
        set_last_error("");
        return f();
    } catch (const Error &e) {
        set_last_error(e.what());
        return e.status;
    } catch (const std::bad_alloc &) {
        set_last_error("host allocation failed");
        return SIGN_ENOMEM;
    } catch (const std::exception &e) {
        set_last_error(e.what());
        return SIGN_EDEVICE;
    }
}

void check_opts(const sign_opts *o) {
    if (!o) throw Error(SIGN_EINVAL, "options are NULL");
    if (!(o->tol > 0.0) || !std::isfinite(o->tol)) throw Error(SIGN_EINVAL, "tol must be > 0");
    if (o->stop_rule != 0 && o->stop_rule != 1) throw Error(SIGN_EINVAL, "stop_rule must be 0 or 1");
    if (!(o->c_fixed >= 0.0) || !(o->switch_res >= 0.0))
        throw Error(SIGN_EINVAL, "c_fixed and switch_res must be >= 0");
    if (o->max_iter < 0) throw Error(SIGN_EINVAL, "max_iter must be >= 0");
    if (o->precision != 0 && o->precision != 1) throw Error(SIGN_EINVAL, "precision must be 0 or 1");
    if (o->polish_steps < 0 || o->refine_steps < 0)
        throw Error(SIGN_EINVAL, "polish_steps and refine_steps must be >= 0");
    if (!(o->scale >= 0.0) || !std::isfinite(o->scale)) throw Error(SIGN_EINVAL, "scale must be >= 0");
    if ((o->alloc == nullptr) != (o->free == nullptr))
        throw Error(SIGN_EINVAL, "alloc and free hooks must be set together");
}

void check_csr_header(const sign_csr *A) {
    if (!A) throw Error(SIGN_EINVAL, "matrix is NULL");
    if (A->n <= 0) throw Error(SIGN_EINVAL, "n must be > 0");
    if (A->n >= (int64_t)INT32_MAX) throw Error(SIGN_EINVAL, "n must be < 2^31");
    if (A->nnz < 0) throw Error(SIGN_EINVAL, "nnz must be >= 0");
    if (!A->row_ptr || (A->nnz > 0 && (!A->col || !A->val)))
        throw Error(SIGN_EINVAL, "NULL array in matrix");
    if (A->val_f32 != 0 && A->val_f32 != 1) throw Error(SIGN_EINVAL, "val_f32 must be 0 or 1");
}

// Validate a device CSR (row pointers, column range/order, finite values).
void validate(Workspace &w, const sign_csr *A) {
    check_csr_header(A);
    w.flag.ensure(sizeof(int));
    SFN_HIP(hipMemsetAsync(w.flag.get(), 0, sizeof(int), w.s));
    launch_validate(A->row_ptr, A->col, A->val, A->val_f32, A->n, A->nnz, w.flag.as<int>(), w.s);
    const int f = read_scalar(w.flag.as<int>(), w.s);
    if (f) {
        std::string m = "malformed CSR:";
        if (f & 1) m += " row_ptr";
        if (f & 2) m += " column out of range";
        if (f & 4) m += " columns not strictly ascending";
        if (f & 8) m += " non-finite value";
        throw Error(SIGN_EINVAL, m);
    }
}

// ||A||_inf in FP64 (row sums of |a_ij|, then a max).
double norm_inf(Workspace &w, const sign_csr *A) {
    w.rs1.ensure(sizeof(double) * A->n);
    launch_row_abs_sum(A->row_ptr, A->val, A->val_f32, A->n, w.rs1.as<double>(), w.s);
    return w.max_rows(w.rs1, A->n);
}

// X = A * scale as a device matrix of value type V.
template <typename V>
void load_scaled(Workspace &w, const sign_csr *A, double scale, DMat<V> &X) {
    X.ensure_rows(A->n);
    X.ensure_entries(A->nnz);
    SFN_HIP(hipMemcpyAsync(X.beg.get(), A->row_ptr, sizeof(int64_t) * (A->n + 1),
                           hipMemcpyDeviceToDevice, w.s));
    launch_row_len(A->row_ptr, A->n, X.lenp(), w.s);
    if (A->nnz > 0) {
        SFN_HIP(hipMemcpyAsync(X.col.get(), A->col, sizeof(int32_t) * A->nnz,
                               hipMemcpyDeviceToDevice, w.s));
        if (A->val_f32)
            launch_scale_copy<float, V>((const float *)A->val, X.valp(), A->nnz, scale, w.s);
        else
            launch_scale_copy<double, V>((const double *)A->val, X.valp(), A->nnz, scale,
                                         w.s);
    }
    X.nnz = A->nnz;
}

template <typename Vi, typename Vo>
void convert(Workspace &w, const DMat<Vi> &In, DMat<Vo> &Out) {
    Out.ensure_rows(In.n);
    Out.ensure_entries(In.nnz);
    SFN_HIP(hipMemcpyAsync(Out.beg.get(), In.beg.get(), sizeof(int64_t) * (In.n + 1),
                           hipMemcpyDeviceToDevice, w.s));
    SFN_HIP(hipMemcpyAsync(Out.len.get(), In.len.get(), sizeof(int32_t) * In.n,
                           hipMemcpyDeviceToDevice, w.s));
    if (In.nnz > 0) {
        SFN_HIP(hipMemcpyAsync(Out.col.get(), In.col.get(), sizeof(int32_t) * In.nnz,
                               hipMemcpyDeviceToDevice, w.s));
        launch_scale_copy<Vi, Vo>(In.valp(), Out.valp(), In.nnz, 1.0,
                                  w.s);
    }
    Out.nnz = In.nnz;
}

// Mixed precision (precision 1):
//  1. the NSF loop with FP32 values (each product's sums accumulated in FP64
//     LDS -- a product of two FP32 values is exact in FP64, and LDS atomic adds
//     of FP32 are far slower on this chip -- and rounded once to FP32 on
//     store; FP64 norms, budget and scaling) to its rounding floor,
//     tol32 = max(tol, 32 u32 sqrt(n)), with
//     the budget c_fixed*tol32 that matches FP32 resolution;
//  2. one FP64 Newton-Schulz step (removes the error part that commutes with
//     the sign);
//  3. commutator refinement: the error part E that anticommutes with S is a
//     neutral direction of every Newton-type sign iteration, but [A, X] =
//     S(|A|E + E|A|), so X <- X - w X [A, X] with w = 1/(2 mean|lambda|)
//     contracts it by about (kappa-1)/(kappa+1) per sweep;
//  4. FP64 Newton-Schulz steps until e <= tol.
LoopOut mixed_precision(Workspace &w, const sign_csr *A, double c, const sign_opts &o,
                        DMat<double> &X, std::vector<sign_iter_stats> &trace, double &comm_rel) {
    const int64_t n = A->n;
    DMat<float> X32;
    X32.bind(w.al);
    load_scaled<float>(w, A, 1.0 / c, X32);
    LoopParams p32{o.tol, o.c_fixed, o.switch_res, 0, o.max_iter, o.filter_y, 1};
    p32.sym = w.allow_sym && is_symmetric<float>(w, X32);
    p32.tol = std::max(o.tol, 32.0 * 5.960464477539063e-08 * std::sqrt((double)n));
    // the FP32 phase ends when its next residual is predicted below tol32/4; the
    // FP64 polish forms that residual anyway, so the FP32 one is not formed
    p32.predict_stop = o.polish_steps > 0 ? 1 : 0;
    const LoopOut l32 = nsf_loop<float>(w, X32, p32, trace);
    convert<float, double>(w, X32, X);
    X32 = DMat<float>();
    if (l32.status == SIGN_EDIVERGED) return l32;
    // polishing and refinement keep the fixed FP64 budget c_fixed*tol: the
    // FP32 phase ends below the switch residual, and the eq. 1.18 budget there
    // (proportional to e^2) would stop filtering altogether
    LoopParams p64{o.tol, o.c_fixed, 0.0, 0, 0, o.filter_y, 0};
    p64.sym = p32.sym;
    int iters = l32.iters;
    LoopOut lo;
    if (o.polish_steps > 0) {
        // one update; the refinement below starts from its result, and the
        // remaining polish forms that residual again, so it is not formed here
        p64.max_iter = 1;
        p64.check_last = 0;
        lo = nsf_loop<double>(w, X, p64, trace);
        p64.check_last = 1;
        iters += lo.iters;
    }
    if (o.refine_steps > 0) {
        DMat<double> As;
        As.bind(w.al);
        load_scaled<double>(w, A, 1.0 / c, As);
        row_sumsq(w, As, w.rs3);
        const double af = std::sqrt(w.sum_rows(w.rs3, n));
        for (int sweep = 0; sweep < o.refine_steps; ++sweep) {
            // a sweep's matrices (and the previous X, swapped into Xn) are released
            // at its end: only X and A carry over
            DMat<double> P, Cm, Cf, Xb, Xn;
            for (DMat<double> *m : {&P, &Cm, &Cf, &Xb, &Xn}) m->bind(w.al);
            const double t0 = now_s();
            w.note("refine sweep %d: X %lld entries", sweep, (long long)X.nnz);
            product<double>(w, As, X, nullptr, 1.0, 0.0, 0.0, P, nullptr, nullptr);
            // C = A X - X A
            product<double>(w, X, As, &P, -1.0, 1.0, 0.0, Cm, nullptr, &w.rs1);
            const double cn = std::sqrt(w.sum_rows(w.rs1, n));
            row_sumsq(w, X, w.rs3);
            const double xf = std::sqrt(w.sum_rows(w.rs3, n));
            w.rs2.ensure(sizeof(double) * n);
            launch_diag<double>(P.view(), w.rs2.as<double>(), w.s);
            const double mean_abs = w.sum_rows(w.rs2, n) / (double)n;  // trace(|A|)/n
            if (sweep == 0) comm_rel = cn / (xf * af);
            if (!(mean_abs > 0.0)) break;
            // estimated relative error of X: ||E|| ~ ||C|| / (2 mean|lambda|)
            const double est = cn / (2.0 * mean_abs * xf);
            // (an order below the 1e-8 accuracy the mixed mode is held to; the
            // estimate is within the condition of the spectrum's two halves,
            // max|lambda| / min|lambda|, of the error that NS cannot see)
            if (est < 1e-9) {
                w.note("refine sweep %d: estimated error %.3e, done (%.1f ms)", sweep, est,
                       1e3 * (now_s() - t0));
                break;
            }
            const double omega = 1.0 / (2.0 * mean_abs);
            P = DMat<double>();  // not needed until the next sweep: give its memory back
            P.bind(w.al);
            // C thinned by G with ||G||_F <= tol mean|lambda| / 16: the correction then
            // moves by omega X G, which changes ||I - X^2|| by at most about
            // 2 omega ||G|| = ||G|| / mean|lambda| <= tol/16 (||X||_2 ~ 1), and C's
            // smallest entries (at the edge of its pattern) need not be multiplied
            filter<double, double>(w, Cm, o.tol * mean_abs / 16.0, Cf, nullptr, nullptr);
            // X - omega X C, filtered with the fixed budget; the product forms the
            // filter's histogram and stores only entries some cut could keep
            const double tau = o.c_fixed * o.tol;
            w.hist.ensure(sizeof(uint64_t) * kBuckets);
            w.rs5.ensure(sizeof(double) * n);
            SFN_HIP(hipMemsetAsync(w.hist.get(), 0, sizeof(uint64_t) * kBuckets, w.s));
            SFN_HIP(hipMemsetAsync(w.rs5.get(), 0, sizeof(double) * n, w.s));
            const FusedFilter fuse{tau, w.hist.as<uint64_t>(), w.rs5.as<double>()};
            product<double>(w, X, Cf, &X, -omega, 1.0, 0.0, Xb, nullptr, nullptr, false, false,
                            &fuse);
            filter<double, double>(w, Xb, tau, Xn, nullptr, nullptr, 0, true);
            w.note("refine sweep %d: estimated error %.3e, nnz C %lld -> %lld, X %lld (%.1f ms)",
                   sweep, est, (long long)Cm.nnz, (long long)Cf.nnz, (long long)Xn.nnz,
                   1e3 * (now_s() - t0));
            std::swap(X, Xn);
            p64.sym = 0;  // X - w X [A, X] is not exactly symmetric
        }
    }
    if (p32.sym && !p64.sym && !o.filter_y) {
        // refinement left X slightly unsymmetric; the sign of a symmetric A is
        // symmetric, so continue from (X + X^T)/2 (never farther from it) and
        // keep the remaining steps on symmetric products
        const double t0 = now_s();
        DMat<double> Xt, I, Xs;
        for (DMat<double> *m : {&Xt, &I, &Xs}) m->bind(w.al);
        transpose(w, X, Xt);
        I.ensure_rows(n);
        I.ensure_entries(n);
        launch_identity(n, I.begp(), I.lenp(), I.colp(), I.valp(), w.s);
        I.nnz = n;
        product<double>(w, I, Xt, &X, 0.5, 0.5, 0.0, Xs, nullptr, nullptr);
        std::swap(X, Xs);
        p64.sym = 1;
        w.note("symmetric projection: nnz %lld (%.1f ms)", (long long)X.nnz, 1e3 * (now_s() - t0));
    }
    p64.max_iter = std::max(1, o.polish_steps - 1);
    // after refinement the iterate is usually converged already: its residual
    // is certified from a thinned copy first
    p64.cert_first = o.refine_steps > 0;
    const LoopOut l2 = nsf_loop<double>(w, X, p64, trace);
    LoopOut out = l2;
    out.iters = iters + l2.iters;
    return out;
}

Allocator make_alloc(const sign_opts *o, hipStream_t s) {
    Allocator a;
    if (o && o->alloc) {
        a.alloc = o->alloc;
        a.release = o->free;
        a.ctx = o->alloc_ctx;
    }
    a.stream = s;
    return a;
}

// Hand a compact device matrix to a new result object.
template <typename V>
sign_result *make_result(const Allocator &al, DMat<V> &X) {
    auto *r = new sign_result();
    r->al = al;
    r->n = X.n;
    r->nnz = X.nnz;
    r->val_f32 = sizeof(V) == 4;
    r->rp = std::move(X.beg);
    r->col = std::move(X.col);
    r->val = std::move(X.val);
    r->rp.bind(&r->al);
    r->col.bind(&r->al);
    r->val.bind(&r->al);
    return r;
}

int finish(sign_result *r, sign_result **out, int status) {
    *out = r;
    return status;
}

}  // namespace

extern "C" {

void sign_opts_default(sign_opts *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->tol = 1e-12;
    o->stop_rule = 0;
    o->c_fixed = 1e-4;
    o->switch_res = 1e-6;
    o->max_iter = 100;
    o->precision = 0;
    o->polish_steps = 2;
    o->refine_steps = 6;
    o->filter_y = 0;
    o->scale = 0.0;
    o->staging_bytes = 0;
}

const char *sign_last_error(void) { return last_error(); }

size_t sign_release_cached(void) {
    Pool &p = Pool::instance();
    const size_t before = p.cached_bytes();
    p.trim();
    const size_t after = p.cached_bytes();
    return before > after ? before - after : 0;
}

int sign_ns(const sign_csr *A, const sign_opts *o, void *hip_stream, sign_result **out) {
    if (out) *out = nullptr;
    return guarded([&]() -> int {
        if (!out) throw Error(SIGN_EINVAL, "out is NULL");
        check_opts(o);
        const double t_start = now_s();
        hipStream_t s = (hipStream_t)hip_stream;
        Allocator al = make_alloc(o, s);
        Workspace w(&al, o->staging_bytes);
        validate(w, A);
        const double c = o->scale > 0.0 ? o->scale : norm_inf(w, A);
        if (!(c > 0.0) || !std::isfinite(c)) throw Error(SIGN_EINVAL, "scale is zero (A = 0?)");
        std::vector<sign_iter_stats> trace;
        LoopParams p{o->tol, o->c_fixed, o->switch_res, o->stop_rule, o->max_iter, o->filter_y, 0};
        LoopOut lo;
        double comm_rel = 0.0;
        DMat<double> X;
        X.bind(&al);
        if (o->precision == 0) {
            load_scaled<double>(w, A, 1.0 / c, X);
            p.sym = w.allow_sym && is_symmetric<double>(w, X);
            lo = nsf_loop<double>(w, X, p, trace);
        } else {
            lo = mixed_precision(w, A, c, *o, X, trace, comm_rel);
        }
        SFN_HIP(hipStreamSynchronize(s));
        sign_result *r = make_result<double>(al, X);
        r->trace = std::move(trace);
        sign_stats &st = r->stats;
        st.status = lo.status;
        st.iters = lo.iters;
        st.stagnated = lo.stagnated;
        st.scale = c;
        st.res_fro = lo.e;
        st.step_fro = lo.d;
        st.nnz = r->nnz;
        st.products = w.products;
        st.madds = w.madds;
        st.spgemm_ms = w.spgemm_ms;
        st.spgemm_bytes = w.spgemm_bytes;
        st.comm_rel = comm_rel;
        w.hot_stats(st);
        st.seconds = now_s() - t_start;
        return finish(r, out, lo.status);
    });
}

int sign_newton(const sign_csr *A, const sign_opts *o, void *hip_stream, sign_result **out) {
    if (out) *out = nullptr;
    return guarded([&]() -> int {
        if (!out) throw Error(SIGN_EINVAL, "out is NULL");
        check_opts(o);
        if (o->precision != 0) throw Error(SIGN_EINVAL, "sign_newton supports precision 0 only");
        const double t_start = now_s();
        hipStream_t s = (hipStream_t)hip_stream;
        Allocator al = make_alloc(o, s);
        Workspace w(&al, o->staging_bytes);
        validate(w, A);
        // the paper starts Newton from X_1 = A; scale > 0 overrides
        const double c = o->scale > 0.0 ? o->scale : 1.0;
        std::vector<sign_iter_stats> trace;
        LoopParams p{o->tol, o->c_fixed, o->switch_res, 0, o->max_iter, 0, 0};
        DMat<double> X;
        X.bind(&al);
        load_scaled<double>(w, A, 1.0 / c, X);
        int inner = 0;
        const LoopOut lo = nmf_loop(w, X, p, trace, inner);
        SFN_HIP(hipStreamSynchronize(s));
        sign_result *r = make_result<double>(al, X);
        r->trace = std::move(trace);
        sign_stats &st = r->stats;
        st.status = lo.status;
        st.iters = lo.iters;
        st.stagnated = lo.stagnated;
        st.scale = c;
        st.res_fro = lo.e;
        st.step_fro = lo.d;
        st.nnz = r->nnz;
        st.products = w.products;
        st.madds = w.madds;
        st.spgemm_ms = w.spgemm_ms;
        st.spgemm_bytes = w.spgemm_bytes;
        st.inner_steps = inner;
        w.hot_stats(st);
        st.seconds = now_s() - t_start;
        return finish(r, out, lo.status);
    });
}

int sign_spgemm(const sign_csr *A, const sign_csr *B, void *hip_stream, sign_result **out) {
    if (out) *out = nullptr;
    return guarded([&]() -> int {
        if (!out) throw Error(SIGN_EINVAL, "out is NULL");
        hipStream_t s = (hipStream_t)hip_stream;
        Allocator al = make_alloc(nullptr, s);
        Workspace w(&al, 0);
        validate(w, A);
        validate(w, B);
        if (A->n != B->n) throw Error(SIGN_EINVAL, "A and B differ in order");
        if (A->val_f32 != B->val_f32) throw Error(SIGN_EINVAL, "A and B differ in value type");
        const double t0 = now_s();
        sign_result *r;
        if (A->val_f32) {
            DMat<float> a, b, c;
            a.bind(&al); b.bind(&al); c.bind(&al);
            load_scaled<float>(w, A, 1.0, a);
            load_scaled<float>(w, B, 1.0, b);
            product<float>(w, a, b, nullptr, 1.0, 0.0, 0.0, c, nullptr, nullptr);
            SFN_HIP(hipStreamSynchronize(s));
            r = make_result<float>(al, c);
        } else {
            DMat<double> a, b, c;
            a.bind(&al); b.bind(&al); c.bind(&al);
            load_scaled<double>(w, A, 1.0, a);
            load_scaled<double>(w, B, 1.0, b);
            product<double>(w, a, b, nullptr, 1.0, 0.0, 0.0, c, nullptr, nullptr);
            SFN_HIP(hipStreamSynchronize(s));
            r = make_result<double>(al, c);
        }
        r->stats.nnz = r->nnz;
        r->stats.products = w.products;
        r->stats.madds = w.madds;
        r->stats.spgemm_ms = w.spgemm_ms;
        r->stats.spgemm_bytes = w.spgemm_bytes;
        w.hot_stats(r->stats);
        r->stats.seconds = now_s() - t0;
        return finish(r, out, SIGN_OK);
    });
}

int sign_filter(const sign_csr *A, double tau, void *hip_stream, sign_result **out, int *bstar) {
    if (out) *out = nullptr;
    return guarded([&]() -> int {
        if (!out) throw Error(SIGN_EINVAL, "out is NULL");
        if (!(tau >= 0.0) || !std::isfinite(tau)) throw Error(SIGN_EINVAL, "tau must be >= 0");
        hipStream_t s = (hipStream_t)hip_stream;
        Allocator al = make_alloc(nullptr, s);
        Workspace w(&al, 0);
        validate(w, A);
        DMat<double> o;
        o.bind(&al);
        int b;
        if (A->val_f32) {
            DMat<float> a;
            a.bind(&al);
            load_scaled<float>(w, A, 1.0, a);
            b = filter<float, double>(w, a, tau, o, nullptr, &w.rs4);
        } else {
            DMat<double> a;
            a.bind(&al);
            load_scaled<double>(w, A, 1.0, a);
            b = filter<double, double>(w, a, tau, o, nullptr, &w.rs4);
        }
        const double dropped = std::sqrt(w.sum_rows(w.rs4, A->n));
        SFN_HIP(hipStreamSynchronize(s));
        if (bstar) *bstar = b;
        sign_result *r = make_result<double>(al, o);
        r->stats.nnz = r->nnz;
        r->stats.step_fro = dropped;  // ||F||_F of the dropped part
        return finish(r, out, SIGN_OK);
    });
}

int sign_result_csr(const sign_result *r, sign_csr *view) {
    return guarded([&]() -> int {
        if (!r || !view) throw Error(SIGN_EINVAL, "NULL argument");
        view->n = r->n;
        view->nnz = r->nnz;
        view->row_ptr = r->rp.as<int64_t>();
        view->col = r->col.as<int32_t>();
        view->val = r->val.get();
        view->val_f32 = r->val_f32;
        return SIGN_OK;
    });
}

int sign_result_stats(const sign_result *r, sign_stats *s) {
    return guarded([&]() -> int {
        if (!r || !s) throw Error(SIGN_EINVAL, "NULL argument");
        *s = r->stats;
        return SIGN_OK;
    });
}

int sign_result_trace(const sign_result *r, int k, sign_iter_stats *it) {
    return guarded([&]() -> int {
        if (!r || !it) throw Error(SIGN_EINVAL, "NULL argument");
        if (k < 0 || k >= (int)r->trace.size()) throw Error(SIGN_EINVAL, "trace index out of range");
        *it = r->trace[k];
        return SIGN_OK;
    });
}

void sign_result_free(sign_result *r) { delete r; }

}  // extern "C"
