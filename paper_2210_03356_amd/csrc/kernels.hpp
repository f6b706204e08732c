// Device kernels of libsignfn and their host-side launchers (gfx950, wave64).
//
// Matrices on the device are addressed row by row through (beg, len):
// row i occupies col[beg[i] .. beg[i]+len[i]) and val[...].  A compact CSR
// has beg = row_ptr (n+1 entries, beg[n] = nnz); a "gapped" matrix produced
// by a product keeps each row at a reserved offset with room to spare.
// Columns are strictly ascending within every row.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sfn {

constexpr int kBuckets = 2048;   // histogram length (buckets 0 .. kBucketTop used)
constexpr int kClasses = 5;      // row classes of the numeric product (0 = empty)
constexpr int kBucketTop = 2033; // |x| >= 1: never dropped

template <typename V>
struct MatView {
    int64_t n = 0;
    const int64_t *beg = nullptr;
    const int32_t *len = nullptr;
    const int32_t *col = nullptr;
    const V *val = nullptr;
};

// Launch geometry of the numeric product for one row class.
// Rows stored as the lower triangle of a symmetric matrix: all rows (all != 0),
// the rows flagged in `rows` (when non-null), or none.
struct LowerRows {
    int all = 0;
    const uint8_t *rows = nullptr;
#ifdef __HIPCC__
    __host__ __device__ bool of(int64_t i) const { return rows ? rows[i] != 0 : all != 0; }
#endif
    bool any() const { return all != 0 || rows != nullptr; }
};

// Occupied column pages of B's rows: page p holds columns [p << shift, (p+1) << shift);
// row k occupies the ascending pages pg[beg[k] .. beg[k] + len[k]).  Given to a
// product, its row groups run their windows over the pages they occupy instead
// of over every column of their range.
struct PageLists {
    const int64_t *beg = nullptr;
    const int32_t *len = nullptr;
    const int32_t *pg = nullptr;
    int shift = 4;
};

// Output options of the numeric product.
struct ProductEpi {
    PageLists pages;           // page-compressed windows for row groups (pg == nullptr: off)
    LowerRows lower;           // rows that store only columns <= the row (symmetric product)
    int keep_from = 0;         // store only entries whose bucket >= keep_from
    uint64_t *hist = nullptr;  // += bucket histogram of all nonzero entries (weighted
                               //    as launch_histogram with `lower`), kBuckets long
    double *sq_pre = nullptr;  // [row] sum of squares of the entries not stored
                               //    because of keep_from (weighted likewise)
    int short_b = 0;           // B's rows are short: each lane walks its own slot's row
    int no_store = 0;          // form row lengths and sums of squares only, store nothing
    unsigned long long *madds = nullptr;  // += multiply-adds performed (products of an A
                                          //    and a B entry added into a window)
};

struct BinCfg {
    int tile;     // LDS accumulator slots (columns per window)
    int threads;  // workgroup size
};

// ---- validation / setup --------------------------------------------------
// flag bits: 1 row_ptr, 2 column range, 4 column order, 8 non-finite value
void launch_validate(const int64_t *rp, const int32_t *ci, const void *val, int f32, int64_t n,
                     int64_t nnz, int *flag, hipStream_t s);
// per-row sum of |a_ij| into out[n] (FP64)
void launch_row_abs_sum(const int64_t *rp, const void *val, int f32, int64_t n, double *out,
                        hipStream_t s);
// len[i] = rp[i+1]-rp[i]
void launch_row_len(const int64_t *rp, int64_t n, int32_t *len, hipStream_t s);
// dst = src * scale (typed conversion); counts n entries
template <typename Vi, typename Vo>
void launch_scale_copy(const Vi *src, Vo *dst, int64_t n, double scale, hipStream_t s);

// ---- reductions (deterministic: fixed partition and order) -----------------
// out[s] = sum_{r in [seg[s], seg[s+1])} x[r]   (one workgroup per segment)
void launch_seg_sum(const double *x, const int64_t *seg, int nseg, double *out, hipStream_t s);
void launch_seg_max(const double *x, const int64_t *seg, int nseg, double *out, hipStream_t s);

// ---- scans -------------------------------------------------------------------
// out[0..n] = init + exclusive prefix of in[0..n) (int64 or int32 input).
// tmp must hold scan_tmp_elems(n) int64.
int64_t scan_tmp_elems(int64_t n);
void launch_exclusive_scan_i64(const int64_t *in, int64_t n, int64_t *out, int64_t *tmp,
                               int64_t init, hipStream_t s);
void launch_exclusive_scan_i32(const int32_t *in, int64_t n, int64_t *out, int64_t *tmp,
                               int64_t init, hipStream_t s);

// ---- product C = diag*I + coef*A*B + dcoef*D ---------------------------------
// Plan: per row i of A (rows [r0, r1)): column window [lo[i], lo[i]+span[i]),
// reserved output capacity cap[i], product count work[i].
// Rows with skip[i] != 0 (skip may be null) get an empty output and no work.
// out[0] += entries, out[1] += column ranges (last - first + 1) of B's nonempty rows
template <typename V>
void launch_row_density(MatView<V> B, unsigned long long *out, hipStream_t s);
template <typename V>
void launch_plan(MatView<V> A, MatView<V> B, MatView<V> D, int diag, int64_t r0, int64_t r1,
                 int32_t *lo, int32_t *span, int64_t *cap, int64_t *work, const uint8_t *skip,
                 hipStream_t s);
// Page lists of B's rows (PageLists): len[k] = number of distinct pages
// (column >> shift) of row k; then, with beg the exclusive scan of len, the
// pages themselves in ascending order.
template <typename V>
void launch_page_count(MatView<V> B, int shift, int32_t *len, hipStream_t s);
template <typename V>
void launch_page_fill(MatView<V> B, int shift, const int64_t *beg, int32_t *pg, hipStream_t s);
// Largest group column range (pages of 2^shift columns) the LDS page table of
// the group kernels holds; wider groups use dense windows.
constexpr int kPageMaxHost = 8192;

// Row classes: 0 empty, 1..3 tiles.  Writes row lists per class (bins[c] holds
// up to r1-r0 rows), counts into counts[4] (device), and len=0 for empty rows.
// Row classes 1..3 by column span (and work), class 4 = leaders i of aligned
// groups of `group` consecutive wide rows (group 2, 4, 8 or 16; 1 disables grouping;
// the other rows of a group are then listed nowhere).
// cstat (optional): per class c, cstat[8c+1] += products, [8c+2] += nnz of the
// A rows, [8c+3] += nnz of the D rows (d_len may be null).
void launch_bin_rows(const int32_t *span, const int64_t *work, int64_t r0, int64_t r1,
                     int small_tile, int mid_tile, int group, int32_t *bins, int64_t bin_stride,
                     int32_t *counts, int32_t *out_len, double *sq_prod, double *sq_out,
                     const int32_t *a_len, const int32_t *d_len, int64_t *cstat,
                     hipStream_t s);
// Groups: merged list of the group's A rows stored in the group's index range
// of A (A must be compact): slot columns mk, row masks mm, coefficient offsets
// mc (into cv, relative to the group's first index), coefficients cv ordered
// by (slot, row); *gathered += sum of nnz(B_k) over the slots.
template <typename V>
void launch_merge_group(int group, const int32_t *leads, int ngroups, MatView<V> A, MatView<V> B,
                        int32_t *mk, uint32_t *mm, int32_t *mc, V *cv, int32_t *mlen,
                        int64_t *gathered, hipStream_t s);
template <typename V>
void launch_spgemm_group(int group, const int32_t *leads, int ngroups, const int32_t *mk,
                         const uint32_t *mm, const int32_t *mc, const V *cv, const int32_t *mlen,
                         MatView<V> A, MatView<V> B, MatView<V> D, double coef, double dcoef,
                         double diag, const int32_t *lo, const int32_t *span, int64_t base,
                         const int64_t *off, int32_t *out_col, V *out_val, int32_t *out_len,
                         int32_t *cursor, int32_t *cnext, double *sq_prod, double *sq_out,
                         int64_t *out_count, ProductEpi epi, hipStream_t s);
// tile = LDS accumulator columns per row of the group
BinCfg group_config(int group, int value_bytes);
// The same product for groups of `group` rows (merged lists as above) with
// register accumulators: windows of 64*nb columns placed where the group's
// rows still have entries, one LDS write/read/clear per B entry and the
// group's multiply-adds in registers (k_spgemm_regtile).  Supported (group,
// nb): (8, 4), (8, 8), (16, 2), (16, 4), (32, 2).  Not for epi.short_b.
bool regtile_supported(int group, int nb);
constexpr int kRegTileThreadsHost = 512;
template <typename V>
void launch_spgemm_regtile(int group, int nb, const int32_t *leads, int ngroups,
                           const int32_t *mk, const uint32_t *mm, const int32_t *mc, const V *cv,
                           const int32_t *mlen, MatView<V> A, MatView<V> B, MatView<V> D,
                           double coef, double dcoef, double diag, const int32_t *lo,
                           const int32_t *span, int64_t base, const int64_t *off,
                           int32_t *out_col, V *out_val, int32_t *out_len, int32_t *cursor,
                           int32_t *cnext, double *sq_prod, double *sq_out, int64_t *out_count,
                           ProductEpi epi, hipStream_t s);

// Symmetric products (the full matrix C from its lower triangle L, both compact):
// cnt[c] += #{j > c : L(j, c) != 0}; out = a + b (row lengths);
// place: L rows to the front of C rows, strictly-lower entries appended to
// their column's mirror list (tcol/tval at toff[c] + arrival order; fill
// zeroed); rank: each mirror list written ordered after the row's lower part
// (llen null: at the start of the row, as for a transpose).
template <typename V>
void launch_sym_count(MatView<V> L, LowerRows lower, int32_t *cnt, hipStream_t s);
void launch_add_len(const int32_t *a, const int32_t *b, int64_t n, int32_t *out, hipStream_t s);
template <typename V>
void launch_sym_place(MatView<V> L, LowerRows lower, const int64_t *cbeg, int32_t *ccol, V *cval,
                      const int64_t *toff, int32_t *fill, int32_t *tcol, V *tval, hipStream_t s);
template <typename V>
void launch_sym_rank(int64_t n, const int64_t *cbeg, const int32_t *llen, const int64_t *toff,
                     const int32_t *tcnt, const int32_t *tcol, const V *tval, int32_t *ccol,
                     V *cval, hipStream_t s);
// *flag |= 1 unless X equals its transpose exactly (pattern and values)
template <typename V>
void launch_sym_check(MatView<V> X, int *flag, hipStream_t s);

// Numeric product for the rows listed in `rows` (class cfg).  Row i writes
// at out_col/out_val[off[i] - base .. ), out_len[i], sq_prod[i] (sum of squares
// of coef*A*B) and sq_out[i] (sum of squares of the stored output), when the
// latter two pointers are non-null.  cursor, cnext: int32 scratch per nonzero of
// A (sweep position in B_k and the column found there, for multi-window rows).
// out_count (optional) accumulates the number of stored entries.
template <typename V>
void launch_spgemm(int cls, const int32_t *rows, int nrows, MatView<V> A, MatView<V> B,
                   MatView<V> D, double coef, double dcoef, double diag, const int32_t *lo,
                   const int32_t *span, int64_t base, const int64_t *off, int32_t *out_col,
                   V *out_val, int32_t *out_len, int32_t *cursor, int32_t *cnext, double *sq_prod,
                   double *sq_out, int64_t *out_count, ProductEpi epi, hipStream_t s);
BinCfg bin_config(int cls, int value_bytes);

// Copy rows [r0, r1) from a gapped layout (row i at src_off[i] - src_base)
// into a compact one (dst_ptr absolute row starts).
template <typename V>
void launch_copy_rows(const int64_t *src_off, int64_t src_base, const int32_t *len,
                      const int32_t *scol, const V *sval, int64_t r0, int64_t r1,
                      const int64_t *dst_ptr, int32_t *dcol, V *dval, hipStream_t s);

// ---- filtering ---------------------------------------------------------------
// Histogram of bucket(|x|) per segment.  seg_rows[s]..seg_rows[s+1] are the
// rows of segment s; hist is nseg x kBuckets (uint64), zeroed by the caller.
// lower: X is the lower triangle of a symmetric matrix; entries below the
// diagonal count twice (here and in launch_count_keep's sums of squares).
template <typename V>
void launch_histogram(MatView<V> X, const int64_t *seg_rows, int nseg, int64_t max_seg_rows,
                      uint64_t *hist, LowerRows lower, hipStream_t s);
// bstar[s] = cut bucket for budget tau[s] (one thread per segment, ascending
// FP64 accumulation without contraction).
void launch_select(const uint64_t *hist, const double *tau, int nseg, int *bstar, hipStream_t s);
// Survivors per row (bucket >= bstar[seg], value != 0) and their/dropped sums of squares.
template <typename V>
void launch_count_keep(MatView<V> X, const int32_t *row_seg, const int *bstar, int32_t *cnt,
                       double *sq_keep, double *sq_drop, LowerRows lower, hipStream_t s);
template <typename V, typename Vo>
void launch_scatter_keep(MatView<V> X, const int32_t *row_seg, const int *bstar,
                         const int64_t *dst_ptr, int32_t *dcol, Vo *dval, hipStream_t s);

// ---- read-back helpers -----------------------------------------------------------
// Per-workgroup counters of the product kernels (entries written, multiply-adds,
// B entries of merged lists) are added at counter + (block % kSpread) *
// kSpreadStride: spread over 32 cache lines, which thousands of one-wave
// workgroups would otherwise contend on.  Counter j of row class c lives at
// spread + (c * kSpreadCounters + j) * kSpread * kSpreadStride.
constexpr int kSpread = 32;
constexpr int kSpreadStride = 8;  // int64 words: 64 bytes apart
constexpr int kSpreadCounters = 3;
constexpr int64_t kSpreadWords = (int64_t)kClasses * kSpreadCounters * kSpread * kSpreadStride;
// dst[j] = *src[j] for j < n (int64 words), so scattered scalars come back to
// the host in one copy; with fold set, also fold_dst[8c + 4 + j] (j = 0, 1, 2:
// slots 4, 5, 6 of class c) = the sum of spread counter j of class c (order
// of the counters: entries written, B entries of merged lists, multiply-adds).
struct ScalarGather {
    const int64_t *src[8] = {};
    int n = 0;
    const int64_t *fold = nullptr;
    int64_t *fold_dst = nullptr;
    void add(const void *p) { src[n++] = static_cast<const int64_t *>(p); }
};
void launch_gather_scalars(const ScalarGather &g, int64_t *dst, hipStream_t s);
// *dst = sum of the kBuckets counts of hist
void launch_hist_total(const uint64_t *hist, int64_t *dst, hipStream_t s);
// seg = {0, n}, *tau_dev = tau (one launch instead of two host copies)
void launch_set_filter_args(int64_t *seg, int64_t n, double *tau_dev, double tau, hipStream_t s);

// ---- misc -----------------------------------------------------------------------
// row_seg[r] = s for rows of segment s
void launch_row_segments(const int64_t *seg_rows, int nseg, int64_t max_seg_rows, int32_t *row_seg,
                         hipStream_t s);

// ---- batch relayout (serving) -------------------------------------------------
// Row block [src_row, src_row + nrows) of src moves to [dst_row, ...) of the
// destination with every column index shifted by col_shift.
struct SegMove {
    MatView<double> src;
    int64_t src_row, dst_row, nrows, col_shift;
};
void launch_move_len(const SegMove *t, int nseg, int64_t max_rows, int32_t *dst_len,
                     hipStream_t s);
void launch_move_rows(const SegMove *t, int nseg, int64_t max_rows, const int64_t *dst_beg,
                      int32_t *dst_col, double *dst_val, hipStream_t s);
void launch_fill_u8(uint8_t *p, int64_t lo, int64_t hi, uint8_t v, hipStream_t s);

// ---- filtered Newton support ---------------------------------------------------
// beg[0..n] = 0..n, len = 1, col = i, val = 1 (identity of order n, compact)
void launch_identity(int64_t n, int64_t *beg, int32_t *len, int32_t *col, double *val,
                     hipStream_t s);
// colsum[j] += |x_ij| (colsum zeroed by the caller)
template <typename V>
void launch_col_abs_sum(MatView<V> X, double *colsum, hipStream_t s);
// transpose: count per column, then fill rows of X^T at tp[j] + atomic slot;
// rows of the result are unordered until ranked with launch_sym_rank
template <typename V>
void launch_transpose_count(MatView<V> X, int32_t *cnt, hipStream_t s);
template <typename V>
void launch_transpose_fill(MatView<V> X, const int64_t *tp, int32_t *fill, int32_t *tcol, V *tval,
                           hipStream_t s);
// diag[i] = X_ii in FP64 (0 when not stored)
template <typename V>
void launch_diag(MatView<V> X, double *diag, hipStream_t s);

}  // namespace sfn
