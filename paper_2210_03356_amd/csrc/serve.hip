// Serving: continuous batching of filtered Newton-Schulz solves.
//
// Every active request is one diagonal block ("segment") of a single
// block-diagonal batch matrix.  One tick advances every active request by one
// iteration of Algorithm 3.2.1 with the same kernels as sign_ns: one product
// launch computes the residuals of all requests, one computes all updates,
// and the filter selects a separate cut per segment from per-segment
// histograms and budgets.  Norms are per-segment fixed-order sums.  Row i of a
// product only reads rows of its own block, so a request's iterates do not
// depend on which other requests share the batch (up to the order of the LDS
// atomic additions).
//
// Requests that finish are copied out and their rows masked (no further
// work); requests waiting in the queue are admitted between ticks while a
// slot is free and the predicted bytes of the resident iterates fit the HBM
// budget; each admission also compacts the rows of finished requests away.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <limits>
#include <thread>
#include <unordered_map>

#include "driver.hpp"

using namespace sfn;

namespace {

struct Req {
    uint64_t id = 0;
    int64_t n = 0;
    std::vector<int64_t> rp;
    std::vector<int32_t> ci;
    std::vector<double> va;
    sign_opts o{};
    double t_submit = 0.0, t_done = 0.0;
    size_t pred = 0;
    // batch state
    int64_t base = 0;
    bool live = false;
    double c = 1.0;
    std::vector<double> es;
    double xf = 0.0, d_prev = std::numeric_limits<double>::infinity();
    double ff_prev = std::numeric_limits<double>::infinity();  // ||F|| of the last cut
    bool no_cert = false;  // a certification of its residual failed: form it in full
    int n_up = 0, n_flat = 0, stagnated = 0, updates = 0;
    int status = SIGN_PENDING;
    std::string err;
    std::vector<sign_iter_stats> trace;
    sign_result *result = nullptr;
    // a request is deleted once it has left the batch and its ticket was
    // collected (both under the server mutex)
    bool in_batch = false, collected = false;
    bool sym = false;  // A equals its transpose exactly
};

double wall() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

// Hard cap on the device memory held by the batch (sign_server_opts
// mem_limit_bytes): the batch allocator refuses a request that would take the
// bytes it holds beyond the cap, which surfaces as SIGN_ENOMEM on the host.
struct MemCap {
    std::mutex mu;
    size_t limit = 0, held = 0;
    std::unordered_map<void *, size_t> sizes;
};

void *cap_alloc(size_t bytes, void *, void *ctx) {
    auto *c = static_cast<MemCap *>(ctx);
    std::lock_guard<std::mutex> lk(c->mu);
    if (c->held + bytes > c->limit) return nullptr;
    void *p = nullptr;
    try {
        p = Pool::instance().get(bytes);
    } catch (const Error &) {
        return nullptr;
    }
    c->held += bytes;
    c->sizes[p] = bytes;
    return p;
}

void cap_free(void *p, void *, void *ctx) {
    auto *c = static_cast<MemCap *>(ctx);
    {
        std::lock_guard<std::mutex> lk(c->mu);
        auto it = c->sizes.find(p);
        if (it != c->sizes.end()) {
            c->held -= it->second;
            c->sizes.erase(it);
        }
    }
    Pool::instance().put(p);
}

// Per-request state a tick changes before its last product: restored when the
// tick is abandoned (a request failed alone) and run again.
struct TickMark {
    Req *r;
    size_t es, trace;
    int n_up, n_flat;
};

}  // namespace

struct sign_server {
    int device = 0;
    size_t budget = 0, used = 0;
    MemCap cap;             // the batch allocator's cap (when mem_limit_bytes > 0)
    Allocator al_out;       // results handed to callers: plain pool, no cap
    int64_t failed = 0;
    double t_relayout = 0.0, t_residual = 0.0, t_update = 0.0, t_filter = 0.0;
    int max_slots = 64, max_queue = 100000;
    hipStream_t stream = nullptr;
    Allocator al;
    std::thread worker;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Req *> queue;
    std::unordered_map<uint64_t, Req *> tickets;
    std::vector<double> latencies_ms;
    bool stop = false;
    uint64_t next_id = 1;
    int64_t submitted = 0, completed = 0, ticks = 0, max_active = 0;
    std::atomic<int64_t> active_count{0};
    double busy = 0.0;
    // batch (worker thread only)
    std::vector<Req *> active;
    DMat<double> X, R, Xb, Xn, Xl, Xt;
    DevBuf seg_d, row_seg, skip, moves;
    DevBuf rowsym;         // rows of requests that take the symmetric products
    bool any_sym = false;

    void run();
    void relayout(std::vector<Req *> &admit, Workspace &w);
    void tick(Workspace &w);
    void finish(Req *r, int status, Workspace &w);
    void fail_all(int status, const std::string &msg);
    // one request ends with an error; its rows stay masked until the next relayout
    void fail_one(Req *r, int status, const std::string &msg);
    // the live request holding the most entries of the batch iterate
    Req *largest_live(Workspace &w);
    void drop_temporaries(Workspace &w);
};

namespace {

// Admission table: entries per row that a request holds on the device at its
// peak -- the iterate, its residual and the update's candidates -- by the average
// row length of A (which tells the served stencils apart), the matrix order and the
// tolerance.  Calibrated on FP64 oracle solves of the served families (1D
// tridiagonal at n = 8192; 2D 5-point and convection-diffusion at 128^2 and 256^2;
// tol 1e-6 / 1e-10 / 1e-12), peak x 1.25 rounded up; the 2D fill grows with the grid
// until the sign's decay radius fits, so 2D has two size classes.  Entries: {largest
// average row length, largest n (0: any), smallest tol, entries per row}; the first
// match applies, and matrices matching none (e.g. 3D stencils) are predicted dense.
struct FillEntry {
    double avg_max;
    int64_t n_max;
    double tol_min;
    double per_row;
};
constexpr FillEntry kFill[] = {
    {3.5, 0, 1e-8, 260},
    {3.5, 0, 1e-11, 360},
    {3.5, 0, 0.0, 410},
    {6.0, 16384, 1e-8, 6810},
    {6.0, 16384, 1e-11, 11740},
    {6.0, 16384, 0.0, 14390},
    {6.0, 0, 1e-8, 8400},
    {6.0, 0, 1e-11, 14340},
    {6.0, 0, 0.0, 17720},
};

// predicted device bytes of one request at its peak: 12 B per FP64 CSR entry plus
// per-row work arrays
size_t predict_bytes(int64_t n, int64_t nnz, double tol) {
    const double avg = (double)nnz / (double)n;
    double per_row = 3.0 * (double)n;
    for (const FillEntry &f : kFill) {
        if (avg <= f.avg_max && (f.n_max == 0 || n <= f.n_max) && tol >= f.tol_min) {
            per_row = f.per_row;
            break;
        }
    }
    per_row = std::min(per_row, 3.0 * (double)n);
    return (size_t)(12.0 * (double)n * per_row) + (size_t)(64 * n);
}

void host_validate(const sign_csr *A) {
    if (!A || A->n <= 0 || A->n >= INT32_MAX || A->nnz < 0 || !A->row_ptr ||
        (A->nnz > 0 && (!A->col || !A->val)))
        throw Error(SIGN_EINVAL, "malformed request matrix header");
    if (A->val_f32) throw Error(SIGN_EINVAL, "serving takes FP64 values");
    const int64_t *rp = A->row_ptr;
    if (rp[0] != 0 || rp[A->n] != A->nnz) throw Error(SIGN_EINVAL, "malformed CSR: row_ptr");
    const double *v = (const double *)A->val;
    for (int64_t i = 0; i < A->n; ++i) {
        if (rp[i + 1] < rp[i]) throw Error(SIGN_EINVAL, "malformed CSR: row_ptr");
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
            if (A->col[p] < 0 || A->col[p] >= A->n)
                throw Error(SIGN_EINVAL, "malformed CSR: column out of range");
            if (p > rp[i] && A->col[p] <= A->col[p - 1])
                throw Error(SIGN_EINVAL, "malformed CSR: columns not strictly ascending");
            if (!std::isfinite(v[p])) throw Error(SIGN_EINVAL, "malformed CSR: non-finite value");
        }
    }
}

// A equals its transpose exactly (pattern and values); A is a validated CSR
bool host_is_symmetric(const sign_csr *A) {
    const int64_t *rp = A->row_ptr;
    const double *v = (const double *)A->val;
    for (int64_t i = 0; i < A->n; ++i)
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
            const int32_t j = A->col[p];
            const int32_t *b = A->col + rp[j], *e = A->col + rp[j + 1];
            const int32_t *f = std::lower_bound(b, e, (int32_t)i);
            if (f == e || *f != i || v[rp[j] + (f - b)] != v[p]) return false;
        }
    return true;
}

sign_result *result_from(const Allocator &al, DMat<double> &X) {
    auto *r = new sign_result();
    r->al = al;
    r->n = X.n;
    r->nnz = X.nnz;
    r->val_f32 = 0;
    r->rp = std::move(X.beg);
    r->col = std::move(X.col);
    r->val = std::move(X.val);
    r->rp.bind(&r->al);
    r->col.bind(&r->al);
    r->val.bind(&r->al);
    return r;
}

// Assemble `dst` from blocks of other matrices (device relayout).
void assemble(Workspace &w, DevBuf &table, const std::vector<SegMove> &moves, int64_t rows,
              DMat<double> &dst) {
    dst.ensure_rows(rows);
    if (moves.empty() || rows == 0) {
        const int64_t z = 0;
        SFN_HIP(hipMemcpyAsync(dst.begp(), &z, sizeof(z), hipMemcpyHostToDevice, w.s));
        SFN_HIP(hipStreamSynchronize(w.s));
        dst.nnz = 0;
        dst.ensure_entries(1);
        return;
    }
    table.ensure(sizeof(SegMove) * moves.size());
    SFN_HIP(hipMemcpyAsync(table.get(), moves.data(), sizeof(SegMove) * moves.size(),
                           hipMemcpyHostToDevice, w.s));
    int64_t maxr = 0;
    for (const SegMove &m : moves) maxr = std::max(maxr, m.nrows);
    launch_move_len(table.as<SegMove>(), (int)moves.size(), maxr, dst.lenp(), w.s);
    w.tmp.ensure(sizeof(int64_t) * scan_tmp_elems(rows));
    launch_exclusive_scan_i32(dst.lenp(), rows, dst.begp(), w.tmp.as<int64_t>(), 0, w.s);
    const int64_t total = read_scalar(dst.begp() + rows, w.s);
    dst.ensure_entries(total);
    launch_move_rows(table.as<SegMove>(), (int)moves.size(), maxr, dst.begp(), dst.colp(),
                     dst.valp(), w.s);
    dst.nnz = total;
}

}  // namespace

void sign_server::fail_all(int status, const std::string &msg) {
    std::lock_guard<std::mutex> lk(mu);
    for (Req *r : active) {
        if (r->status == SIGN_PENDING) {
            r->status = status;
            r->err = msg;
            r->t_done = wall();
            used -= std::min(used, r->pred);
            ++completed;
            ++failed;
        }
        r->in_batch = false;
        r->live = false;
        if (r->collected) delete r;
    }
    active.clear();
    active_count = 0;
    X = DMat<double>();
    X.bind(&al);
}

void sign_server::fail_one(Req *r, int status, const std::string &msg) {
    if (r->in_batch && r->live)
        launch_fill_u8(skip.as<uint8_t>(), r->base, r->base + r->n, 1, stream);
    std::lock_guard<std::mutex> lk(mu);
    r->status = status;
    r->err = msg;
    r->live = false;
    r->t_done = wall();
    used -= std::min(used, r->pred);
    ++completed;
    ++failed;
}

Req *sign_server::largest_live(Workspace &w) {
    (void)w;
    std::vector<int64_t> beg((size_t)X.n + 1, 0);
    if (X.n > 0 && X.begp())
        SFN_HIP(hipMemcpyAsync(beg.data(), X.begp(), sizeof(int64_t) * (X.n + 1),
                               hipMemcpyDeviceToHost, stream));
    SFN_HIP(hipStreamSynchronize(stream));
    Req *best = nullptr;
    int64_t most = -1;
    for (Req *r : active) {
        if (!r->live) continue;
        const int64_t e = (r->base + r->n <= X.n) ? beg[r->base + r->n] - beg[r->base] : 0;
        if (e > most || (e == most && best && r->n > best->n)) { most = e; best = r; }
    }
    return best;
}

void sign_server::drop_temporaries(Workspace &w) {
    (void)hipStreamSynchronize(stream);
    for (DMat<double> *m : {&R, &Xb, &Xn, &Xl, &Xt}) {
        *m = DMat<double>();
        m->bind(&al);
    }
    for (DevBuf *b : {&w.stage_col, &w.stage_val, &w.cursor, &w.cnext, &w.mk, &w.mm, &w.mc,
                      &w.cv, &w.symtcol, &w.symtval})
        b->reset();
    w.row_skip = nullptr;
}

void sign_server::finish(Req *r, int status, Workspace &w) {
    // copy the request's rows out of the batch, columns back to 0-based (into
    // memory the caller owns after the poll: the plain pool, not the batch cap)
    DMat<double> out;
    out.bind(&al_out);
    std::vector<SegMove> mv{{X.view(), r->base, 0, r->n, -r->base}};
    DevBuf tab(&al);
    assemble(w, tab, mv, r->n, out);
    SFN_HIP(hipStreamSynchronize(stream));
    sign_result *res = result_from(al_out, out);
    res->trace = std::move(r->trace);
    sign_stats &st = res->stats;
    st.status = status;
    st.iters = r->updates;
    st.stagnated = r->stagnated;
    st.scale = r->c;
    st.res_fro = r->es.empty() ? 0.0 : r->es.back();
    st.step_fro = std::isfinite(r->d_prev) ? r->d_prev : 0.0;
    st.nnz = res->nnz;
    launch_fill_u8(skip.as<uint8_t>(), r->base, r->base + r->n, 1, stream);
    std::lock_guard<std::mutex> lk(mu);
    r->result = res;
    r->status = status;
    r->live = false;
    r->t_done = wall();
    res->stats.seconds = r->t_done - r->t_submit;
    latencies_ms.push_back(1e3 * (r->t_done - r->t_submit));
    used -= std::min(used, r->pred);
    ++completed;
}

// Admission and compaction: the live requests of the current batch move to
// the front (finished ones leave), the admitted ones are appended as new
// diagonal blocks.  Nothing of the server's state changes until the new batch
// matrix and its tables exist, so a failure (an allocation refused) leaves the
// running batch as it was and concerns only the admitted requests.
void sign_server::relayout(std::vector<Req *> &admit, Workspace &w) {
    std::vector<Req *> keep, gone;
    for (Req *r : active) (r->live ? keep : gone).push_back(r);
    std::vector<SegMove> mv;
    std::vector<int64_t> base_new;
    int64_t rows = 0;
    for (Req *r : keep) {
        mv.push_back({X.view(), r->base, rows, r->n, rows - r->base});
        base_new.push_back(rows);
        rows += r->n;
    }
    // upload and scale the new requests: X_1 = A / ||A||_inf
    std::vector<DMat<double>> fresh(admit.size());
    std::vector<double> scale(admit.size(), 1.0);
    for (size_t q = 0; q < admit.size(); ++q) {
        Req *r = admit[q];
        DMat<double> &F = fresh[q];
        F.bind(&al);
        F.ensure_rows(r->n);
        F.ensure_entries(std::max<int64_t>(1, (int64_t)r->ci.size()));
        SFN_HIP(hipMemcpyAsync(F.begp(), r->rp.data(), sizeof(int64_t) * (r->n + 1),
                               hipMemcpyHostToDevice, stream));
        if (!r->ci.empty()) {
            SFN_HIP(hipMemcpyAsync(F.colp(), r->ci.data(), sizeof(int32_t) * r->ci.size(),
                                   hipMemcpyHostToDevice, stream));
            SFN_HIP(hipMemcpyAsync(F.valp(), r->va.data(), sizeof(double) * r->va.size(),
                                   hipMemcpyHostToDevice, stream));
        }
        launch_row_len(F.begp(), r->n, F.lenp(), stream);
        F.nnz = (int64_t)r->ci.size();
        w.rs1.ensure(sizeof(double) * r->n);
        launch_row_abs_sum(F.begp(), F.valp(), 0, r->n, w.rs1.as<double>(), stream);
        double c = r->o.scale > 0.0 ? r->o.scale : w.max_rows(w.rs1, r->n);
        if (!(c > 0.0)) c = 1.0;
        scale[q] = c;
        launch_scale_copy<double, double>(F.valp(), F.valp(), F.nnz, 1.0 / c, stream);
        mv.push_back({F.view(), 0, rows, r->n, rows});
        base_new.push_back(rows);
        rows += r->n;
    }
    DMat<double> X2;
    X2.bind(&al);
    assemble(w, moves, mv, rows, X2);
    // tables of the new batch, in buffers of their own until the commit (the
    // running batch keeps its tables if an allocation is refused here)
    const int S = (int)(keep.size() + admit.size());
    DevBuf seg2(&al), rseg2(&al), skip2(&al), rsym2(&al);
    seg2.ensure(sizeof(int64_t) * (S + 1));
    rseg2.ensure(sizeof(int32_t) * std::max<int64_t>(rows, 1));
    skip2.ensure(std::max<int64_t>(rows, 1));
    rsym2.ensure(std::max<int64_t>(rows, 1));
    w.rs3.ensure(sizeof(double) * std::max<int64_t>(rows, 1));
    w.red.ensure(sizeof(double) * std::max(S, 1));
    SFN_HIP(hipStreamSynchronize(stream));

    // commit
    std::swap(seg_d, seg2);
    std::swap(row_seg, rseg2);
    std::swap(skip, skip2);
    std::swap(rowsym, rsym2);
    std::swap(X, X2);
    X2 = DMat<double>();
    fresh.clear();
    const size_t nkeep = keep.size();
    for (size_t q = 0; q < nkeep; ++q) keep[q]->base = base_new[q];
    for (size_t q = 0; q < admit.size(); ++q) {
        Req *r = admit[q];
        r->base = base_new[nkeep + q];
        r->c = scale[q];
        r->live = true;
        keep.push_back(r);
    }
    {
        std::lock_guard<std::mutex> lk(mu);
        for (Req *r : gone) {
            r->in_batch = false;
            if (r->collected) delete r;
        }
        for (Req *r : admit) r->in_batch = true;
    }
    active = keep;
    active_count = (int64_t)active.size();
    max_active = std::max<int64_t>(max_active, (int64_t)active.size());
    // segment tables
    std::vector<int64_t> seg_h(S + 1, 0);
    for (int q = 0; q < S; ++q) seg_h[q + 1] = seg_h[q] + active[q]->n;
    SFN_HIP(hipMemcpyAsync(seg_d.get(), seg_h.data(), sizeof(int64_t) * (S + 1),
                           hipMemcpyHostToDevice, stream));
    int64_t maxr = 0;
    for (Req *r : active) maxr = std::max(maxr, r->n);
    launch_row_segments(seg_d.as<int64_t>(), S, maxr, row_seg.as<int32_t>(), stream);
    launch_fill_u8(skip.as<uint8_t>(), 0, rows, 0, stream);
    // symmetric requests with unfiltered residuals take the symmetric products
    any_sym = false;
    for (Req *r : active) {
        const bool sy = r->sym && !r->o.filter_y;
        launch_fill_u8(rowsym.as<uint8_t>(), r->base, r->base + r->n, sy ? 1 : 0, stream);
        any_sym = any_sym || sy;
    }
    // ||X^_1||_F of the new requests
    if (!admit.empty()) {
        row_sumsq(w, X, w.rs3);
        const std::vector<double> sq = seg_sums(w, w.rs3, seg_d.as<int64_t>(), S);
        for (int q = 0; q < S; ++q)
            if (active[q]->es.empty()) active[q]->xf = std::sqrt(sq[q]);
    }
}

void sign_server::tick(Workspace &w) {
    double tp = wall();
    auto phase = [&](double &acc) {
        const double t = wall();
        acc += t - tp;
        tp = t;
    };
    const int S = (int)active.size();
    const int64_t *segd = seg_d.as<int64_t>();
    w.row_skip = skip.as<uint8_t>();
    ++ticks;
    std::vector<int64_t> seg_h(S + 1, 0);
    for (int q = 0; q < S; ++q) seg_h[q + 1] = seg_h[q] + active[q]->n;
    // Requests whose residual Lemma 2.1.1 and their last cut predict far below
    // tol have it certified from a copy thinned by delta (as sign_ns does):
    // e <= ||I - Xt^2|| + 2 ||Xt||_2 delta + delta^2.  The other requests get a
    // zero budget, which keeps their rows whole, so one product serves both.
    std::vector<char> pred(S, 0);
    std::vector<double> s_one_inf(S, 1.0), delta2(S, 0.0);
    bool any_pred = false, any_pred_nonsym = false;
    for (int q = 0; q < S; ++q) {
        Req *r = active[q];
        if (!r->live || r->no_cert || r->o.stop_rule != 0 || r->es.empty()) continue;
        const double ep = r->es.back();
        if (0.75 * ep * ep * (1.0 + ep / 3.0) + 2.5 * r->ff_prev <= 0.25 * r->o.tol) {
            pred[q] = 1;
            any_pred = true;
            if (!(r->sym && !r->o.filter_y)) any_pred_nonsym = true;
        }
    }
    const uint8_t *rs = any_sym ? rowsym.as<uint8_t>() : nullptr;
    if (any_pred) {
        if (any_pred_nonsym) {
            const std::vector<double> p = seg_norm_one_inf(w, X, segd, S);
            for (int q = 0; q < S; ++q) s_one_inf[q] = std::sqrt(p[q]);
        }
        std::vector<double> tc(S, 0.0);
        for (int q = 0; q < S; ++q) {
            if (!pred[q]) continue;
            const bool sy = active[q]->sym && !active[q]->o.filter_y;
            tc[q] = active[q]->o.tol / (16.0 * (sy ? 1.0 : s_one_inf[q]));
        }
        std::vector<int> bs;
        filter_seg(w, X, seg_h, segd, row_seg.as<int32_t>(), tc, Xt, nullptr, &w.rs4, bs);
        delta2 = seg_sums(w, w.rs4, segd, S);
    }
    // residuals of all requests: R^ = I - X^ X^ (thinned rows for the predicted)
    product<double>(w, any_pred ? Xt : X, any_pred ? Xt : X, nullptr, -1.0, 0.0, 1.0, R, nullptr,
                    &w.rs1, false, false, nullptr, rs);
    std::vector<double> e2 = seg_sums(w, w.rs1, segd, S);
    std::vector<char> bound(S, 0);
    if (any_pred) {
        bool failed = false;
        for (int q = 0; q < S; ++q) {
            if (!pred[q]) continue;
            const bool sy = active[q]->sym && !active[q]->o.filter_y;
            const double et = std::sqrt(e2[q]), dl = std::sqrt(delta2[q]);
            const double b = et + 2.0 * (sy ? std::sqrt(1.0 + et) : s_one_inf[q]) * dl + dl * dl;
            if (b <= active[q]->o.tol) {
                e2[q] = b * b;
                bound[q] = 1;
            } else {
                active[q]->no_cert = true;
                failed = true;
            }
        }
        if (failed) {
            // a request that goes on needs its true residual for the update
            product<double>(w, X, X, nullptr, -1.0, 0.0, 1.0, R, nullptr, &w.rs1, false, false,
                            nullptr, rs);
            e2 = seg_sums(w, w.rs1, segd, S);
            std::fill(bound.begin(), bound.end(), 0);
        }
    }
    phase(t_residual);
    std::vector<double> tau(S, 0.0), tau_r(S, 0.0);
    bool any_live = false, any_fy = false;
    for (int q = 0; q < S; ++q) {
        Req *r = active[q];
        if (!r->live) continue;
        const double e = std::sqrt(e2[q]);
        r->es.push_back(e);
        const int k = (int)r->es.size();
        sign_iter_stats it{};
        it.e = e;
        it.e_bound = bound[q];
        it.xfro = r->xf;
        const bool conv = r->o.stop_rule == 1 ? (r->d_prev < r->o.tol) : (e <= r->o.tol);
        int st = SIGN_PENDING;
        if (conv) st = SIGN_OK;
        else if (!std::isfinite(e)) st = SIGN_EDIVERGED;
        else {
            if (k >= 2) {
                const double ep = r->es[k - 2];
                r->n_up = (e > ep && e > 1.0) ? r->n_up + 1 : 0;
                r->n_flat = (e < 1e-8 && e > 0.5 * ep) ? r->n_flat + 1 : 0;
                if (r->n_up >= 3) st = SIGN_EDIVERGED;
                else if (r->n_flat >= 2) { st = SIGN_OK; r->stagnated = 1; }
            }
            if (st == SIGN_PENDING && k - 1 >= r->o.max_iter) st = SIGN_ENOCONV;
        }
        r->trace.push_back(it);
        if (st != SIGN_PENDING) {
            finish(r, st, w);
            continue;
        }
        any_live = true;
        tau[q] = nsf_budget(e, r->xf, r->o.tol, r->o.c_fixed, r->o.switch_res);
        if (r->o.filter_y) { tau_r[q] = tau[q]; any_fy = true; }
    }
    phase(t_relayout);  // copies of the finished requests out of the batch
    if (!any_live) return;
    std::vector<int> bstar;
    if (any_fy) {
        filter_seg(w, R, seg_h, segd, row_seg.as<int32_t>(), tau_r, Xn, nullptr, nullptr, bstar);
        std::swap(R, Xn);
        phase(t_filter);
    }
    // updates of all requests: Xbar = X^ + 1/2 X^ R^
    // (rows of symmetric requests: lower triangles, filtered with the entries
    // below the diagonal counted twice, then mirrored)
    product<double>(w, X, R, &X, 0.5, 1.0, 0.0, Xb, &w.rs2, nullptr, false, rs != nullptr,
                    nullptr, rs);
    const std::vector<double> d2 = seg_sums(w, w.rs2, segd, S);
    phase(t_update);
    LowerRows lower;
    lower.rows = rs;
    if (rs) {
        filter_seg(w, Xb, seg_h, segd, row_seg.as<int32_t>(), tau, Xl, &w.rs3, &w.rs4, bstar,
                   lower);
        symmetrize<double>(w, Xl, Xn, lower);
    } else {
        filter_seg(w, Xb, seg_h, segd, row_seg.as<int32_t>(), tau, Xn, &w.rs3, &w.rs4, bstar);
    }
    const std::vector<double> k2 = seg_sums(w, w.rs3, segd, S);
    const std::vector<double> f2 = seg_sums(w, w.rs4, segd, S);
    phase(t_filter);
    for (int q = 0; q < S; ++q) {
        Req *r = active[q];
        if (!r->live) continue;
        sign_iter_stats &it = r->trace.back();
        it.d = std::sqrt(d2[q]);
        it.tau = tau[q];
        it.ffro = std::sqrt(f2[q]);
        it.bstar = bstar[q];
        r->ff_prev = it.ffro;
        r->xf = std::sqrt(k2[q]);
        r->d_prev = it.d;
        r->updates += 1;
    }
    std::swap(X, Xn);
    w.row_skip = nullptr;
}

void sign_server::run() {
    if (hipSetDevice(device) != hipSuccess) {
        (void)hipGetLastError();
        fail_all(SIGN_EDEVICE, "hipSetDevice failed in the server thread");
        return;
    }
    Workspace w(&al, 0);
    for (;;) {
        std::vector<Req *> admit;
        {
            std::unique_lock<std::mutex> lk(mu);
            bool has_live = false;
            for (Req *r : active) has_live |= r->live;
            if (!has_live) cv.wait(lk, [&] { return stop || !queue.empty(); });
            if (stop) break;
            int live = 0;
            for (Req *r : active) live += r->live ? 1 : 0;
            while (!queue.empty() && live + (int)admit.size() < max_slots) {
                Req *r = queue.front();
                if (used + r->pred > budget && (live + admit.size()) > 0) break;
                queue.pop_front();
                used += r->pred;
                admit.push_back(r);
            }
        }
        const double t0 = wall();
        // Failures are isolated where the cause is a refused allocation
        // (SIGN_ENOMEM, a host-side error): a request that does not fit at
        // admission fails alone (relayout leaves the batch as it was), and a
        // tick that does not fit fails the live request holding the most entries,
        // after which the tick runs again for the others from the state before it.
        // Any other error (a HIP runtime failure) ends every active request.
        try {
            if (!admit.empty()) {
                try {
                    relayout(admit, w);
                } catch (const Error &e) {
                    if (e.status != SIGN_ENOMEM) throw;
                    drop_temporaries(w);
                    // admit them one at a time: only those that do not fit fail
                    for (Req *r : admit) {
                        std::vector<Req *> one{r};
                        try {
                            relayout(one, w);
                        } catch (const Error &e1) {
                            if (e1.status != SIGN_ENOMEM) throw;
                            drop_temporaries(w);
                            fail_one(r, SIGN_ENOMEM,
                                     std::string("admission: ") + e1.what() +
                                         " (the running batch is unaffected)");
                        }
                    }
                }
                t_relayout += wall() - t0;
            }
            for (;;) {
                bool has_live = false;
                for (Req *r : active) has_live |= r->live;
                if (!has_live) break;
                std::vector<TickMark> marks;
                for (Req *r : active)
                    if (r->live)
                        marks.push_back({r, r->es.size(), r->trace.size(), r->n_up, r->n_flat});
                try {
                    tick(w);
                    SFN_HIP(hipStreamSynchronize(stream));
                    break;
                } catch (const Error &e) {
                    if (e.status != SIGN_ENOMEM) throw;
                    drop_temporaries(w);
                    // requests the abandoned tick finished keep their results; the
                    // others return to their state before it
                    for (const TickMark &m : marks) {
                        if (!m.r->live) continue;
                        m.r->es.resize(m.es);
                        m.r->trace.resize(m.trace);
                        m.r->n_up = m.n_up;
                        m.r->n_flat = m.n_flat;
                    }
                    Req *victim = largest_live(w);
                    if (!victim) break;
                    fail_one(victim, SIGN_ENOMEM,
                             std::string(e.what()) +
                                 " (this request holds the most entries of the batch; the "
                                 "other requests continue)");
                }
            }
        } catch (const Error &e) {
            w.row_skip = nullptr;
            fail_all(e.status, e.what());
        } catch (const std::exception &e) {
            w.row_skip = nullptr;
            fail_all(SIGN_EDEVICE, e.what());
        }
        busy += wall() - t0;
    }
}

extern "C" {

int sign_server_create(const sign_server_opts *o, sign_server **s) {
    if (s) *s = nullptr;
    try {
        if (!o || !s) throw Error(SIGN_EINVAL, "NULL argument");
        if (o->max_slots < 0 || o->max_queue < 0) throw Error(SIGN_EINVAL, "negative limits");
        SFN_HIP(hipSetDevice(o->device));
        auto *sv = new sign_server();
        sv->device = o->device;
        sv->max_slots = o->max_slots > 0 ? o->max_slots : 64;
        sv->max_queue = o->max_queue > 0 ? o->max_queue : 100000;
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
            (void)hipGetLastError();
            fr = size_t(16) << 30;
        }
        sv->budget = o->hbm_budget_bytes > 0 ? o->hbm_budget_bytes : fr / 2;
        if (hipStreamCreate(&sv->stream) != hipSuccess) {
            (void)hipGetLastError();
            delete sv;
            throw Error(SIGN_EDEVICE, "hipStreamCreate failed");
        }
        sv->al.stream = sv->stream;
        sv->al_out.stream = sv->stream;
        if (o->mem_limit_bytes > 0) {
            sv->cap.limit = o->mem_limit_bytes;
            sv->al.alloc = cap_alloc;
            sv->al.release = cap_free;
            sv->al.ctx = &sv->cap;
        }
        for (DevBuf *b : {&sv->seg_d, &sv->row_seg, &sv->skip, &sv->moves, &sv->rowsym})
            b->bind(&sv->al);
        for (DMat<double> *m : {&sv->X, &sv->R, &sv->Xb, &sv->Xn, &sv->Xl, &sv->Xt})
            m->bind(&sv->al);
        sv->worker = std::thread([sv] { sv->run(); });
        *s = sv;
        return SIGN_OK;
    } catch (const Error &e) {
        set_last_error(e.what());
        return e.status;
    } catch (const std::exception &e) {
        set_last_error(e.what());
        return SIGN_EDEVICE;
    }
}

int sign_serve_submit(sign_server *s, const sign_csr *A, const sign_opts *o, uint64_t *ticket) {
    try {
        if (!s || !A || !o || !ticket) throw Error(SIGN_EINVAL, "NULL argument");
        if (!(o->tol > 0.0) || o->max_iter < 0 || (o->stop_rule != 0 && o->stop_rule != 1))
            throw Error(SIGN_EINVAL, "invalid options");
        if (o->precision != 0) throw Error(SIGN_EINVAL, "serving supports precision 0 only");
        if (o->alloc || o->free) throw Error(SIGN_EINVAL, "serving does not take allocator hooks");
        host_validate(A);
        auto *r = new Req();
        r->sym = host_is_symmetric(A);
        r->n = A->n;
        r->rp.assign(A->row_ptr, A->row_ptr + A->n + 1);
        r->ci.assign(A->col, A->col + A->nnz);
        r->va.assign((const double *)A->val, (const double *)A->val + A->nnz);
        r->o = *o;
        r->pred = predict_bytes(A->n, A->nnz, o->tol);
        r->t_submit = wall();
        {
            std::lock_guard<std::mutex> lk(s->mu);
            if ((int)s->queue.size() >= s->max_queue) {
                delete r;
                throw Error(SIGN_EBUSY, "queue full");
            }
            r->id = s->next_id++;
            s->tickets[r->id] = r;
            s->queue.push_back(r);
            ++s->submitted;
            *ticket = r->id;
        }
        s->cv.notify_one();
        return SIGN_OK;
    } catch (const Error &e) {
        set_last_error(e.what());
        return e.status;
    } catch (const std::bad_alloc &) {
        set_last_error("host allocation failed");
        return SIGN_ENOMEM;
    }
}

int sign_serve_poll(sign_server *s, uint64_t ticket, sign_result **out) {
    if (out) *out = nullptr;
    if (!s || !out) {
        set_last_error("NULL argument");
        return SIGN_EINVAL;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) {
        set_last_error("unknown or already collected ticket");
        return SIGN_ENOTFOUND;
    }
    Req *r = it->second;
    if (r->status == SIGN_PENDING) return SIGN_PENDING;
    const int st = r->status;
    *out = r->result;
    r->result = nullptr;
    if (!*out) set_last_error(r->err);
    s->tickets.erase(it);
    r->collected = true;
    if (!r->in_batch) delete r;
    return st;
}

int sign_server_stats_get(sign_server *s, sign_server_stats *st) {
    if (!s || !st) {
        set_last_error("NULL argument");
        return SIGN_EINVAL;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    std::memset(st, 0, sizeof(*st));
    st->submitted = s->submitted;
    st->completed = s->completed;
    st->queued = (int64_t)s->queue.size();
    st->active = s->active_count.load();
    st->ticks = s->ticks;
    st->max_active = s->max_active;
    st->busy_seconds = s->busy;
    st->failed = s->failed;
    st->relayout_seconds = s->t_relayout;
    st->residual_seconds = s->t_residual;
    st->update_seconds = s->t_update;
    st->filter_seconds = s->t_filter;
    if (!s->latencies_ms.empty()) {
        std::vector<double> v = s->latencies_ms;
        std::sort(v.begin(), v.end());
        auto pct = [&](double p) {
            const size_t i = (size_t)std::min<double>(v.size() - 1, std::floor(p * (v.size() - 1) + 0.5));
            return v[i];
        };
        st->p50_ms = pct(0.50);
        st->p99_ms = pct(0.99);
    }
    return SIGN_OK;
}

void sign_server_destroy(sign_server *s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv.notify_all();
    if (s->worker.joinable()) s->worker.join();
    (void)hipStreamSynchronize(s->stream);
    for (auto &kv : s->tickets) {
        if (kv.second->result) sign_result_free(kv.second->result);
        kv.second->collected = true;
        if (!kv.second->in_batch) delete kv.second;
    }
    for (Req *r : s->active)
        if (r->collected) delete r;  // every remaining request is collected now
    s->tickets.clear();
    s->queue.clear();
    s->active.clear();
    s->X = DMat<double>();
    s->R = DMat<double>();
    s->Xb = DMat<double>();
    s->Xn = DMat<double>();
    for (DevBuf *b : {&s->seg_d, &s->row_seg, &s->skip, &s->moves}) b->reset();
    (void)hipStreamDestroy(s->stream);
    delete s;
}

}  // extern "C"
