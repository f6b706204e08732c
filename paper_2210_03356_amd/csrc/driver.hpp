// Host drivers of libsignfn: one sparse product, one filtering step, and the
// filtered Newton-Schulz / filtered Newton loops built from them.
#pragma once

#include <chrono>
#include <initializer_list>
#include <vector>

#include "runtime.hpp"

namespace sfn {

// Per-call scratch shared by every product and filter of one solve.
struct Workspace {
    Allocator *al;
    hipStream_t s;
    size_t staging_limit;  // bytes of gapped product output per batch
    bool staging_auto;     // staging_limit follows the free memory (see auto_staging)
    size_t auto_staging() const;
    DevBuf lo, span, cap, work, capoff, workoff, tmp, bins, counts, cursor, stage_col, stage_val;
    DevBuf rs1, rs2, rs3, rs4, icnt, hist, tau, bstar, seg, red, flag, zero_b;
    DevBuf cstat, mk, mm, mc, cv, mlen, cnext;
    DevBuf symcnt, symoff, symfill, symtcol, symtval;  // mirroring of symmetric products
    DevBuf rs5;                                        // per-row sums not stored by a product
    DevBuf pst;                                        // column-range statistics of a plan
    DevBuf plen, pbeg, plist;                          // page lists of a product's B rows
    const uint8_t *row_skip = nullptr;  // optional row mask for products (serving)
    int row_group = 8;                  // wide rows computed in groups of 1, 2, 4, 8 or 16
    bool auto_group = true;             // choose 4 or 8 per product from its column ranges
    bool allow_sym = true;              // symmetric products from their lower triangle
    // register-accumulator product (k_spgemm_regtile): rows per group and
    // windows of 64*rt_nb columns; rt_mode 0 off, 1 by the per-product rule,
    // 2 for every product it supports
    int rt_mode = 0, rt_group = 16, rt_nb = 4;
    // page windows for row groups (kernels.hpp PageLists): 0 off, 1 for products
    // whose B rows occupy few of the pages of their column ranges, 2 always;
    // pages of 2^page_shift columns
    int page_mode = 1, page_shift = 4;
    // filtered residuals (filter_y) formed in two passes -- norm and histogram,
    // then only the kept entries -- so that the unfiltered residual is never
    // stored: from the first step (SIGNFN_RESIDUAL_TWO_PASS=1), else once an
    // unfiltered residual outgrows a quarter of the device's memory
    bool residual_two_pass = false;
    bool low_memory = false;  // set with two passes: product staging capped at 8 GB
    bool progress = false;              // one stderr line per finished iteration
    hipEvent_t ev[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    // accumulated product statistics, in total and per row class (kernel tile)
    struct ClassStat {
        int64_t launches = 0, rows = 0, products = 0, a_nnz = 0, d_nnz = 0, out = 0;
        int64_t gathered = 0;  // B entries loaded (once per slot of a row group)
        int64_t madds = 0;     // multiply-adds performed (fewer than products when rows stop
                               // at the diagonal)
        int64_t page_launches = 0;  // launches with page windows
        double ms = 0.0, bytes = 0.0;
    };
    ClassStat cls[2][kClasses];  // [FP64, FP32][row class 1..3]
    ClassStat grp[2][5];         // [FP64, FP32][log2 of the row group] (class 4)
    ClassStat rt[2];             // [FP64, FP32] register-accumulator groups
    int rt_used_group = 0, rt_used_nb = 0;  // configuration of the last such launch
    double merge_ms = 0.0;
    int64_t products = 0;
    int64_t madds = 0;  // multiply-adds the product kernels performed
    double spgemm_ms = 0.0;
    double spgemm_bytes = 0.0;
    // fill the hot-kernel fields (class with the most device time) of s
    void hot_stats(sign_stats &s) const;
    explicit Workspace(Allocator *a, size_t staging_bytes);
    ~Workspace();
    // ||rows||: deterministic sum of a per-row double array over [0, n)
    double sum_rows(const DevBuf &rows, int64_t n);
    // several row-sum totals with one synchronisation
    std::vector<double> sum_rows_many(std::initializer_list<const DevBuf *> rows, int64_t n);
    DevBuf whole, sums;   // {0, n} segment for whole-matrix sums, their results
    DevBuf rb;            // device record of scalars read back in one copy
    // pinned host memory of the calling thread for read-backs (64 int64 words)
    static int64_t *pinned();
    // gathers the listed device scalars (int64 words) and copies them to
    // pinned host memory in one transfer; synchronises the stream
    const int64_t *read_back(const ScalarGather &g);
    int64_t whole_n = -1;
    double max_rows(const DevBuf &rows, int64_t n);
    // the progress line of an iteration that just ended (when progress is set)
    void report(const char *loop, int k, const sign_iter_stats &it) const;
    // a free-form progress line (when progress is set)
    void note(const char *fmt, ...) const __attribute__((format(printf, 2, 3)));
};

// C = diag*I + coef*A*B + dcoef*D (D may be null); C becomes compact CSR.
// sq_prod[i] receives the sum of squares of row i of coef*A*B and sq_out[i]
// that of the stored row of C (either may be null); only their totals are
// meaningful when sym is set.  sym: the caller knows C is symmetric (A, B, D
// symmetric and AB = BA); only the lower triangle is computed and the upper
// one is its mirror.  keep_lower (with sym): C receives the lower triangle only.
// A product whose output is filtered next with budget tau: the product adds the
// filter's bucket histogram of all its entries to hist (kBuckets, zeroed by the
// caller) and stores only entries that some cut could keep; the sums of squares
// of the others go to sq_pre[row].
struct FusedFilter {
    double tau;
    uint64_t *hist;
    double *sq_pre;
    // >= 0: a cut already chosen -- store only entries of buckets >= keep_from
    // (instead of the safe edge of tau)
    int keep_from = -1;
};
template <typename V>
void product(Workspace &w, const DMat<V> &A, const DMat<V> &B, const DMat<V> *D, double coef,
             double dcoef, double diag, DMat<V> &C, DevBuf *sq_prod, DevBuf *sq_out,
             bool sym = false, bool keep_lower = false, const FusedFilter *ff = nullptr,
             const uint8_t *row_sym = nullptr);
// (row_sym: per-row flags instead of sym, for block-diagonal batches whose
// symmetric blocks -- and only those -- take the symmetric route)

// Per-row sums of squares of C = diag*I + coef*A*B into sq_out without storing C
// (sym as in product: only the lower triangle is formed, the sums weighted so
// that they are the full matrix's).  Returns the entry count of C (of its lower
// triangle when sym).
template <typename V>
int64_t product_sumsq(Workspace &w, const DMat<V> &A, const DMat<V> &B, double coef,
                      double diag, DevBuf *sq_out, bool sym);

// C (full, compact) from the lower triangle L (compact) of a symmetric matrix
// (or of the rows of its symmetric diagonal blocks flagged in lower.rows).
template <typename V>
void symmetrize(Workspace &w, const DMat<V> &L, DMat<V> &C, LowerRows lower = LowerRows{1, nullptr});

// true if X equals its transpose exactly (pattern and values)
template <typename V>
bool is_symmetric(Workspace &w, const DMat<V> &X);

// Out = In without its largest low-magnitude part of Frobenius norm <= tau.
// Returns the cut bucket; sq_keep/sq_drop (optional) receive per-row sums of
// squares of kept / dropped entries.
// lower: In is the lower triangle of a symmetric matrix (Out likewise); the cut
// and the sums of squares count entries below the diagonal twice.
// The filter's cut (bucket index) for budget tau from the histogram in w.hist
// (one segment of n rows), read back to the host.
int select_cut(Workspace &w, int64_t n, double tau);
// hist_ready: the histogram of In is already in w.hist (a fused product);
// candidates (optional): the histogram's total count.
template <typename V, typename Vo>
int filter(Workspace &w, const DMat<V> &In, double tau, DMat<Vo> &Out, DevBuf *sq_keep,
           DevBuf *sq_drop, int lower = 0, bool hist_ready = false,
           int64_t *candidates = nullptr);

// Filtering of a block-diagonal batch: segment s owns rows [seg_h[s], seg_h[s+1])
// (seg_d: the same boundaries on the device, row_seg: segment of every row)
// and is cut with its own budget tau_h[s].  bstar_h receives the cuts.
void filter_seg(Workspace &w, const DMat<double> &In, const std::vector<int64_t> &seg_h,
                const int64_t *seg_d, const int32_t *row_seg, const std::vector<double> &tau_h,
                DMat<double> &Out, DevBuf *sq_keep, DevBuf *sq_drop, std::vector<int> &bstar_h,
                LowerRows lower = LowerRows());

// Per-segment sums of a per-row FP64 array (deterministic).
std::vector<double> seg_sums(Workspace &w, const DevBuf &rows, const int64_t *seg_d, int nseg);
// Per-segment maxima of a per-row FP64 array.
std::vector<double> seg_maxs(Workspace &w, const DevBuf &rows, const int64_t *seg_d, int nseg);
// ||X_s||_1 * ||X_s||_inf of every diagonal block s of a block-diagonal FP64 matrix.
std::vector<double> seg_norm_one_inf(Workspace &w, const DMat<double> &X, const int64_t *seg_d,
                                     int nseg);

// ||X||_F^2 per row into rows (via the survivor pass with an all-keeping cut).
template <typename V>
void row_sumsq(Workspace &w, const DMat<V> &X, DevBuf &rows);

// Budget of the filter: c_fixed*tol before the switch, eq. 1.18 / eq. 1.13 after.
double nsf_budget(double e, double xfro, double tol, double c_fixed, double switch_res);
double nmf_budget(double e, double xfro, double zfro, double tol, double c_fixed,
                  double switch_res);

struct LoopParams {
    double tol, c_fixed, switch_res;
    int stop_rule, max_iter, filter_y;
    int fp32;     // recorded in the trace
    int sym = 0;  // the iterate is symmetric: symmetric products from their lower triangle
    // 0: after max_iter updates, return without forming the last iterate's
    // residual (a caller that continues from it)
    int check_last = 1;
    // 1: certify the first residual from a thinned copy too (FP64; see nsf_loop)
    int cert_first = 0;
    // 1: stop, without forming it, once the next residual is predicted at most
    // tol/4 (a caller that forms it itself, in higher precision; status SIGN_OK)
    int predict_stop = 0;
};

struct LoopOut {
    int status = SIGN_OK;
    int iters = 0;
    int stagnated = 0;
    double e = 0.0, d = 0.0, xfro = 0.0;
};

// Algorithm 3.2.1 on X (compact, modified in place to the final iterate).
template <typename V>
LoopOut nsf_loop(Workspace &w, DMat<V> &X, const LoopParams &p,
                 std::vector<sign_iter_stats> &trace);

// Algorithm 3.1.1 on X (FP64, compact, modified in place to the final iterate);
// the inverse of each iterate by filtered Newton-Schulz inversion.
LoopOut nmf_loop(Workspace &w, DMat<double> &X, const LoopParams &p,
                 std::vector<sign_iter_stats> &trace, int &inner_steps);

// Out = X^T (compact, sorted rows).
void transpose(Workspace &w, const DMat<double> &X, DMat<double> &Out);

inline double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

}  // namespace sfn
