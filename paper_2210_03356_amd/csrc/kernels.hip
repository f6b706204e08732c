// Device kernels of libsignfn for gfx950 (CDNA4, wave64).
//
// The numeric product is row-wise Gustavson: row i of C = diag*I + coef*A*B + D
// is accumulated in an LDS-resident dense window of `tile` consecutive columns
// with native LDS atomic adds of FP64 values (for FP32-valued matrices too: the
// product of two FP32 values is exact in FP64, and ds_add_f32 is far slower
// here); k_spgemm_regtile is a register-accumulator variant.  Rows whose column
// range exceeds the tile are swept in several windows; B's rows are sorted,
// so each (row of A entry, window) pair resumes from a per-entry cursor and
// every B entry is read once per output row.  Groups of rows whose outputs fill
// a small part of their column range can instead run their windows over the
// 16-column pages they occupy (page windows, k_spgemm_rows with PG).  The
// finished window is scanned in column order and its nonzeros written out, so
// results come out sorted and without stored zeros.  The path is gather- and
// latency-bound (no dense contraction), so MFMA is not used.
#include "kernels.hpp"

#include <climits>
#include <cmath>
#include <type_traits>

namespace sfn {

namespace {

constexpr int kWave = 64;
constexpr int kUnroll = 4;  // 64-entry chunks of a B row gathered per sweep step
constexpr int kRegTileThreads = 512;  // workgroup of the register-accumulator product

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }
__device__ __forceinline__ int wave_id() { return threadIdx.x / kWave; }

__device__ __forceinline__ int rl_i32(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ __forceinline__ int64_t rl_i64(int64_t v, int l) {
    const int lo = __builtin_amdgcn_readlane((int)(v & 0xffffffff), l);
    const int hi = __builtin_amdgcn_readlane((int)(v >> 32), l);
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
__device__ __forceinline__ double rl_val(double v, int l) {
    return __longlong_as_double(rl_i64(__double_as_longlong(v), l));
}
__device__ __forceinline__ float rl_val(float v, int l) {
    return __int_as_float(rl_i32(__float_as_int(v), l));
}

// Workgroups are dispatched round-robin over the 8 XCDs (id b runs on XCD
// b % 8).  Neighbouring output rows gather nearly the same rows of B, so the
// row list is dealt out in chunks of kXcdChunk consecutive rows, chunk c to
// XCD c % 8: the workgroups resident on one XCD then work on consecutive rows
// (their gathers hit that XCD's L2), and the eight XCDs together work on
// 8*kXcdChunk consecutive rows (their misses share the Infinity Cache).  The
// tail that does not fill a whole round is split into eight contiguous bands.
// A bijection of [0, nb) for every nb.
constexpr int kXcdChunk = 64;
constexpr int kPageMax = kPageMaxHost;  // LDS page table of the group kernels (int16 ranks)
constexpr int kPageMinShift = 4;        // pages hold at least 16 columns

__device__ __forceinline__ int xcd_band(int b, int nb) {
    const int per = (nb + 7) >> 3;
    const int full = 8 - (8 * per - nb);  // XCDs whose band holds `per` rows
    const int x = b & 7, q = b >> 3;
    return x * per - max(0, x - full) + q;
}

__device__ __forceinline__ int xcd_row(int b, int nb) {
    constexpr int round = 8 * kXcdChunk;
    const int full = nb / round;
    if (b < full * round) {
        const int x = b & 7, q = b >> 3;
        return (q / kXcdChunk) * round + x * kXcdChunk + (q % kXcdChunk);
    }
    return full * round + xcd_band(b - full * round, nb - full * round);
}

// number of set bits of m in lanes below the calling lane
__device__ __forceinline__ int lanes_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ __forceinline__ int wave_min(int v) {
    for (int o = kWave / 2; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ int wave_max(int v) {
    for (int o = kWave / 2; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
    return v;
}

// inclusive scan across the wave
__device__ __forceinline__ int64_t wave_incl_scan(int64_t v) {
    const int lane = lane_id();
    for (int o = 1; o < kWave; o <<= 1) {
        const int64_t t = __shfl_up(v, o);
        if (lane >= o) v += t;
    }
    return v;
}

// Bucket of |x| from the IEEE-754 binary64 pattern: 0 below 2^-127, kBucketTop
// at or above 1, else 1 + 16*(E+127) + (top four fraction bits).
__device__ __forceinline__ int bucket_of(double x) {
    const uint64_t b = (uint64_t)__double_as_longlong(x) & 0x7fffffffffffffffull;
    if (b >= 0x3ff0000000000000ull) return kBucketTop;
    const int E = (int)(b >> 52) - 1023;
    if (E < -127) return 0;
    return 1 + 16 * (E + 127) + (int)((b >> 48) & 15u);
}

// Weight of an entry (row, col) in a Frobenius norm taken over the stored part
// of a matrix: 1 when the whole matrix is stored; for a symmetric matrix held
// by its lower triangle, 2 below the diagonal (the entry stands for itself and
// its mirror), 1 on it, 0 above (not stored).
__device__ __forceinline__ double sym_weight(bool lower, int col, int row) {
    if (!lower) return 1.0;
    return col < row ? 2.0 : (col == row ? 1.0 : 0.0);
}

template <typename T>
__device__ __forceinline__ double as_f64(T v) { return (double)v; }

// ---------------------------------------------------------------------------
// validation and setup
// ---------------------------------------------------------------------------
__global__ void k_validate(const int64_t *rp, const int32_t *ci, const void *val, int f32,
                           int64_t n, int64_t nnz, int *flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0 && (rp[0] != 0 || rp[n] != nnz)) atomicOr(flag, 1);
    if (i >= n) return;
    const int64_t b = rp[i], e = rp[i + 1];
    if (b < 0 || e < b || e > nnz) { atomicOr(flag, 1); return; }
    int f = 0;
    int prev = -1;
    for (int64_t p = b; p < e; ++p) {
        const int c = ci[p];
        if (c < 0 || c >= n) f |= 2;
        if (c <= prev) f |= 4;
        prev = c;
        const double v = f32 ? (double)((const float *)val)[p] : ((const double *)val)[p];
        if (!isfinite(v)) f |= 8;
    }
    if (f) atomicOr(flag, f);
}

__global__ void k_row_abs_sum(const int64_t *rp, const void *val, int f32, int64_t n,
                              double *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int64_t p = rp[i]; p < rp[i + 1]; ++p)
        s += fabs(f32 ? (double)((const float *)val)[p] : ((const double *)val)[p]);
    out[i] = s;
}

__global__ void k_row_len(const int64_t *rp, int64_t n, int32_t *len) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) len[i] = (int32_t)(rp[i + 1] - rp[i]);
}

template <typename Vi, typename Vo>
__global__ void k_scale_copy(const Vi *src, Vo *dst, int64_t n, double scale) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = (Vo)((double)src[i] * scale);
}

// ---------------------------------------------------------------------------
// deterministic segmented reductions: one workgroup per segment, each thread
// sums a fixed strided subset, then a fixed tree
// ---------------------------------------------------------------------------
constexpr int kRedThreads = 1024;

template <bool kMax>
__global__ __launch_bounds__(kRedThreads) void k_seg_reduce(const double *x, const int64_t *seg,
                                                            double *out) {
    __shared__ double sh[kRedThreads];
    const int s = blockIdx.x;
    const int64_t lo = seg[s], hi = seg[s + 1];
    double acc = 0.0;
    for (int64_t r = lo + threadIdx.x; r < hi; r += kRedThreads)
        acc = kMax ? fmax(acc, x[r]) : acc + x[r];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kRedThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            sh[threadIdx.x] = kMax ? fmax(sh[threadIdx.x], sh[threadIdx.x + w])
                                   : sh[threadIdx.x] + sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[s] = sh[0];
}

// ---------------------------------------------------------------------------
// exclusive scan (three passes, fixed partition)
// ---------------------------------------------------------------------------
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanChunk = kScanThreads * kScanItems;

template <typename T, int NT = kScanThreads>
__device__ int64_t block_excl_scan(int64_t v, int64_t *sh_w, int64_t *total) {
    const int lane = lane_id(), w = wave_id();
    const int64_t inc = wave_incl_scan(v);
    if (lane == kWave - 1) sh_w[w] = inc;
    __syncthreads();
    int64_t before = 0, tot = 0;
    for (int q = 0; q < NT / kWave; ++q) {
        if (q < w) before += sh_w[q];
        tot += sh_w[q];
    }
    __syncthreads();
    *total = tot;
    return before + inc - v;
}

template <typename T>
__global__ __launch_bounds__(kScanThreads) void k_scan_partial(const T *in, int64_t n,
                                                               int64_t *part) {
    __shared__ int64_t shw[kScanThreads / kWave];
    const int64_t base = (int64_t)blockIdx.x * kScanChunk;
    int64_t s = 0;
    for (int q = 0; q < kScanItems; ++q) {
        const int64_t i = base + (int64_t)q * kScanThreads + threadIdx.x;
        if (i < n) s += (int64_t)in[i];
    }
    int64_t tot;
    block_excl_scan<T>(s, shw, &tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// single workgroup: exclusive scan of the block totals in place
__global__ __launch_bounds__(kScanThreads) void k_scan_top(int64_t *part, int64_t nb) {
    __shared__ int64_t shw[kScanThreads / kWave];
    int64_t carry = 0;
    for (int64_t base = 0; base < nb; base += kScanThreads) {
        const int64_t i = base + threadIdx.x;
        const int64_t v = i < nb ? part[i] : 0;
        int64_t tot;
        const int64_t ex = block_excl_scan<int64_t>(v, shw, &tot);
        if (i < nb) part[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) part[nb] = carry;
}

template <typename T>
__global__ __launch_bounds__(kScanThreads) void k_scan_final(const T *in, int64_t n,
                                                             const int64_t *part, int64_t nb,
                                                             int64_t init, int64_t *out) {
    __shared__ int64_t shw[kScanThreads / kWave];
    const int64_t base = (int64_t)blockIdx.x * kScanChunk;
    // thread-contiguous items for the in-thread serial scan
    int64_t vals[kScanItems];
    int64_t s = 0;
    for (int q = 0; q < kScanItems; ++q) {
        const int64_t i = base + (int64_t)threadIdx.x * kScanItems + q;
        vals[q] = i < n ? (int64_t)in[i] : 0;
        s += vals[q];
    }
    int64_t tot;
    int64_t run = init + part[blockIdx.x] + block_excl_scan<T>(s, shw, &tot);
    for (int q = 0; q < kScanItems; ++q) {
        const int64_t i = base + (int64_t)threadIdx.x * kScanItems + q;
        if (i < n) out[i] = run;
        run += vals[q];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = init + part[nb];
}

// the whole scan in one workgroup, for n <= kScanOneMax: short arrays (small
// matrices, few segments) then cost one launch instead of three
constexpr int kScanOneThreads = 1024;
constexpr int64_t kScanOneMax = (int64_t)kScanOneThreads * kScanItems;

template <typename T>
__global__ __launch_bounds__(kScanOneThreads) void k_scan_one(const T *in, int64_t n,
                                                              int64_t init, int64_t *out) {
    __shared__ int64_t shw[kScanOneThreads / kWave];
    int64_t vals[kScanItems];
    int64_t s = 0;
    for (int q = 0; q < kScanItems; ++q) {
        const int64_t i = (int64_t)threadIdx.x * kScanItems + q;
        vals[q] = i < n ? (int64_t)in[i] : 0;
        s += vals[q];
    }
    int64_t tot;
    int64_t run = init + block_excl_scan<T, kScanOneThreads>(s, shw, &tot);
    for (int q = 0; q < kScanItems; ++q) {
        const int64_t i = (int64_t)threadIdx.x * kScanItems + q;
        if (i < n) out[i] = run;
        run += vals[q];
    }
    if (threadIdx.x == 0) out[n] = init + tot;
}

// ---------------------------------------------------------------------------
// product planning and row classes
// ---------------------------------------------------------------------------
template <typename V>
__global__ void k_plan(MatView<V> A, MatView<V> B, MatView<V> D, int diag, int64_t r0,
                       int64_t r1, int32_t *lo, int32_t *span, int64_t *cap, int64_t *work,
                       const uint8_t *skip) {
    const int64_t i = r0 + (int64_t)blockIdx.x * (blockDim.x / kWave) + wave_id();
    if (i >= r1) return;  // uniform per wave
    const int lane = lane_id();
    if (skip && skip[i]) {  // masked row: empty output, no work
        if (lane == 0) { lo[i] = 0; span[i] = 0; cap[i] = 0; work[i] = 0; }
        return;
    }
    const int64_t ab = A.beg[i];
    const int al = A.len[i];
    int64_t u = 0;
    int mn = INT_MAX, mx = -1;
    for (int t = lane; t < al; t += kWave) {
        const int k = A.col[ab + t];
        const int bl = B.len[k];
        if (bl > 0) {
            const int64_t bb = B.beg[k];
            u += bl;
            mn = min(mn, B.col[bb]);
            mx = max(mx, B.col[bb + bl - 1]);
        }
    }
    u = wave_sum(u);
    mn = wave_min(mn);
    mx = wave_max(mx);
    if (lane == 0) {
        int64_t extra = 0;
        if (D.len) {
            const int dl = D.len[i];
            if (dl > 0) {
                const int64_t db = D.beg[i];
                mn = min(mn, D.col[db]);
                mx = max(mx, D.col[db + dl - 1]);
                extra += dl;
            }
        }
        if (diag) {
            mn = min(mn, (int)i);
            mx = max(mx, (int)i);
            extra += 1;
        }
        if (mx < 0) {
            lo[i] = 0; span[i] = 0; cap[i] = 0; work[i] = 0;
        } else {
            const int sp = mx - mn + 1;
            lo[i] = mn;
            span[i] = sp;
            cap[i] = min((int64_t)sp, u + extra);
            work[i] = u;
        }
    }
}

// Entries and column ranges (last - first + 1) of the nonempty rows of B,
// summed: their ratio is the density of a B row within its range.
constexpr int kSpanThreads = 256;
template <typename V>
__global__ __launch_bounds__(kSpanThreads) void k_row_density(MatView<V> B,
                                                              unsigned long long *out) {
    __shared__ int64_t ws[kSpanThreads / kWave], wc[kSpanThreads / kWave];
    const int64_t i = (int64_t)blockIdx.x * kSpanThreads + threadIdx.x;
    int64_t len = 0, rng = 0;
    if (i < B.n) {
        const int l = B.len[i];
        if (l > 0) {
            const int64_t b = B.beg[i];
            len = l;
            rng = (int64_t)B.col[b + l - 1] - B.col[b] + 1;
        }
    }
    len = wave_sum(len);
    rng = wave_sum(rng);
    if (lane_id() == 0) { ws[wave_id()] = len; wc[wave_id()] = rng; }
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t a = 0, b = 0;
        for (int w = 0; w < kSpanThreads / kWave; ++w) { a += ws[w]; b += wc[w]; }
        if (a) {
            atomicAdd(&out[0], (unsigned long long)a);
            atomicAdd(&out[1], (unsigned long long)b);
        }
    }
}

// Page lists of B's rows, one wave per row: an entry starts a new page when its
// page differs from the previous entry's (the row is sorted), so the pages come
// out distinct and ascending.
template <typename V, bool kFill>
__global__ void k_row_pages(MatView<V> B, int shift, int32_t *len, const int64_t *beg,
                            int32_t *pg) {
    const int64_t k = (int64_t)blockIdx.x * (blockDim.x / kWave) + wave_id();
    if (k >= B.n) return;  // uniform per wave
    const int lane = lane_id();
    const int l = B.len[k];
    const int32_t *col = B.col + B.beg[k];
    int count = 0;
    int64_t at = kFill ? beg[k] : 0;
    for (int t0 = 0; t0 < l; t0 += kWave) {
        const int t = t0 + lane;
        const int p = t < l ? col[t] >> shift : INT_MAX;
        const int prev = t < l && t > 0 ? col[t - 1] >> shift : INT_MIN;
        const bool start = t < l && p != prev;
        const uint64_t m = __ballot(start);
        if (kFill && start) pg[at + lanes_below(m)] = p;
        at += __popcll(m);
        count += __popcll(m);
    }
    if (!kFill && lane == 0) len[k] = count;
}

constexpr int kBinThreads = 256;

// Row classes: 0 empty, 1 small window, 2 mid window, 3 wide rows swept in
// 8192-column (FP64) windows, 4 leaders of groups of consecutive wide rows that
// are computed together (the other rows of a group get no class of their own).
__device__ __forceinline__ int row_class(const int32_t *span, const int64_t *work, int64_t i,
                                         int small_tile, int mid_tile) {
    const int sp = span[i];
    if (sp == 0) return 0;
    if (sp <= small_tile && work[i] <= (int64_t)8 * small_tile) return 1;
    if (sp <= mid_tile) return 2;
    return 3;
}

__global__ __launch_bounds__(kBinThreads) void k_bin_rows(
    const int32_t *span, const int64_t *work, int64_t r0, int64_t r1, int small_tile,
    int mid_tile, int group, int32_t *bins, int64_t bin_stride, int32_t *counts,
    int32_t *out_len, double *sq_prod, double *sq_out, const int32_t *a_len,
    const int32_t *d_len, int64_t *cstat) {
    __shared__ int wc[kBinThreads / kWave][kClasses];
    __shared__ int base[kClasses];
    __shared__ unsigned long long bsum[kClasses][3];
    if (threadIdx.x < 3 * kClasses) bsum[threadIdx.x / 3][threadIdx.x % 3] = 0ull;
    const int64_t i = r0 + (int64_t)blockIdx.x * kBinThreads + threadIdx.x;
    int cls = -1;
    if (i < r1) {
        cls = row_class(span, work, i, small_tile, mid_tile);
        if (cls == 0) {
            out_len[i] = 0;
            if (sq_prod) sq_prod[i] = 0.0;
            if (sq_out) sq_out[i] = 0.0;
        } else if (cls == 3 && group > 1) {
            // aligned groups of `group` consecutive wide rows are computed together
            const int64_t lead = r0 + (i - r0) / group * group;
            bool whole = lead + group <= r1;
            for (int r = 0; whole && r < group; ++r)
                whole = row_class(span, work, lead + r, small_tile, mid_tile) == 3;
            if (whole) cls = (i == lead) ? 4 : -1;  // members are computed by their leader
        }
    }
    const int lane = lane_id(), w = wave_id();
    int rank = 0;
    for (int c = 1; c < kClasses; ++c) {
        const uint64_t m = __ballot(cls == c);
        if (cls == c) rank = lanes_below(m);
        if (lane == 0) wc[w][c] = __popcll(m);
    }
    __syncthreads();
    if (threadIdx.x < kClasses && threadIdx.x > 0) {
        int t = 0;
        for (int q = 0; q < kBinThreads / kWave; ++q) t += wc[q][threadIdx.x];
        base[threadIdx.x] = t ? atomicAdd(&counts[threadIdx.x], t) : 0;
    }
    __syncthreads();
    if (cls >= 1) {
        int off = base[cls] + rank;
        for (int q = 0; q < w; ++q) off += wc[q][cls];
        bins[(int64_t)cls * bin_stride + off] = (int32_t)i;
        const int nr = cls == 4 ? group : 1;
        for (int r = 0; r < nr; ++r) {
            atomicAdd(&bsum[cls][0], (unsigned long long)work[i + r]);
            atomicAdd(&bsum[cls][1], (unsigned long long)a_len[i + r]);
            if (d_len) atomicAdd(&bsum[cls][2], (unsigned long long)d_len[i + r]);
        }
    }
    __syncthreads();
    if (cstat && threadIdx.x >= 3 && threadIdx.x < 3 * kClasses) {
        const int c = threadIdx.x / 3, f = threadIdx.x % 3;
        if (bsum[c][f]) atomicAdd((unsigned long long *)&cstat[c * 8 + 1 + f], bsum[c][f]);
    }
}

// Merged A-row list of a group of R consecutive rows i .. i+R-1 (R <= 32), in
// slot order (ascending column k of the union of the R sorted column lists):
//   mk[s]  the column k,
//   mm[s]  bit r set when row i+r has an entry at k,
//   mc[s]  offset of the slot's first coefficient in cv,
//   cv     the group's entries ordered by (slot, r), so the coefficient of row
//          i+r at slot s is cv[mc[s] + popcount(mm[s] & ((1 << r) - 1))].
// Slots and coefficients are stored from index beg[i] of A's index range: A is
// compact, so the group owns [beg[i], beg[i+R]) and neither the union nor the
// entries overflow it.  mlen[i] = number of slots.  One workgroup per group
// sweeps the columns in chunks: it marks the columns present (LDS bitmasks),
// scans them into slot positions and coefficient offsets, and writes slots and
// coefficients.  *gathered += sum of nnz(B_k) over the slots.
constexpr int kMergeChunk = 4096;
constexpr int kMergeThreads = 256;

template <typename V, int R>
__global__ __launch_bounds__(kMergeThreads) void k_merge_group(
    const int32_t *__restrict__ leads, MatView<V> A, MatView<V> B, int32_t *__restrict__ mk,
    uint32_t *__restrict__ mm, int32_t *__restrict__ mc, V *__restrict__ cv,
    int32_t *__restrict__ mlen, unsigned long long *__restrict__ gathered) {
    static_assert(R >= 2 && R <= 32, "group size");
    constexpr int NW = kMergeThreads / kWave;
    constexpr int PER = kMergeChunk / kMergeThreads;  // consecutive columns per thread
    __shared__ uint32_t mask[kMergeChunk];
    __shared__ int32_t coff[kMergeChunk];
    __shared__ int64_t st[R], en[R];
    __shared__ int fst[R + 1];
    __shared__ int64_t wt[NW];
    __shared__ int lohi[2];

    const int i = leads[blockIdx.x];
    const int lane = lane_id(), wave = wave_id();
    const int64_t gb = A.beg[i];
    if (threadIdx.x == 0) {
        int lo = INT_MAX, hi = INT_MIN;
        for (int r = 0; r < R; ++r) {
            const int l = A.len[i + r];
            if (l > 0) {
                lo = min(lo, A.col[A.beg[i + r]]);
                hi = max(hi, A.col[A.beg[i + r] + l - 1] + 1);
            }
        }
        lohi[0] = lo;
        lohi[1] = hi;
    }
    if (threadIdx.x < R) st[threadIdx.x] = A.beg[i + threadIdx.x];
    __syncthreads();
    const int64_t lo = lohi[0], hi = lohi[1];
    int64_t nslot = 0, ncoef = 0;  // slots and coefficients written so far (uniform)
    unsigned long long g = 0;
    for (int64_t c0 = lo; c0 < hi; c0 += kMergeChunk) {
        const int64_t c1 = min(hi, c0 + kMergeChunk);
        for (int q = threadIdx.x; q < kMergeChunk; q += kMergeThreads) mask[q] = 0u;
        if (threadIdx.x < R) {
            // end of list r's entries below c1 (binary search from its chunk start)
            const int r = threadIdx.x;
            int64_t a = st[r], b = A.beg[i + r] + A.len[i + r];
            while (a < b) {
                const int64_t m = (a + b) >> 1;
                if (A.col[m] < c1) a = m + 1;
                else b = m;
            }
            en[r] = a;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int f = 0;
            for (int r = 0; r < R; ++r) {
                fst[r] = f;
                f += (int)(en[r] - st[r]);
            }
            fst[R] = f;
        }
        __syncthreads();
        const int tot = fst[R];
        for (int f = threadIdx.x; f < tot; f += kMergeThreads) {
            int r = 0;
            while (f >= fst[r + 1]) ++r;
            const int k = A.col[st[r] + (f - fst[r])];
            atomicOr(&mask[k - c0], 1u << r);
        }
        __syncthreads();
        // exclusive scan of (slots, coefficients) over the chunk, packed as
        // (slots << 32 | coefficients): neither field can carry into the other
        const int q0 = threadIdx.x * PER;
        int ns = 0, nc = 0;
        for (int u = 0; u < PER; ++u) {
            const uint32_t m = mask[q0 + u];
            ns += m != 0u;
            nc += __popc(m);
        }
        const int64_t pk = ((int64_t)ns << 32) | (int64_t)nc;
        const int64_t inc = wave_incl_scan(pk);
        if (lane == kWave - 1) wt[wave] = inc;
        __syncthreads();
        int64_t before = inc - pk, total = 0;
        for (int w = 0; w < NW; ++w) {
            if (w < wave) before += wt[w];
            total += wt[w];
        }
        int64_t ps = nslot + (before >> 32), pc = ncoef + (before & 0xffffffffll);
        for (int u = 0; u < PER; ++u) {
            const uint32_t m = mask[q0 + u];
            if (m) {
                const int k = (int)(c0 + q0 + u);
                mk[gb + ps] = k;
                mm[gb + ps] = m;
                mc[gb + ps] = (int32_t)pc;
                coff[q0 + u] = (int32_t)pc;
                g += (unsigned long long)B.len[k];
                ++ps;
                pc += __popc(m);
            }
        }
        __syncthreads();
        for (int f = threadIdx.x; f < tot; f += kMergeThreads) {
            int r = 0;
            while (f >= fst[r + 1]) ++r;
            const int64_t e = st[r] + (f - fst[r]);
            const int q = (int)(A.col[e] - c0);
            cv[gb + coff[q] + __popc(mask[q] & ((1u << r) - 1u))] = A.val[e];
        }
        nslot += total >> 32;
        ncoef += total & 0xffffffffll;
        __syncthreads();
        if (threadIdx.x < R) st[threadIdx.x] = en[threadIdx.x];
        __syncthreads();
    }
    if (threadIdx.x == 0) mlen[i] = (int32_t)nslot;
    g = wave_sum(g);
    if (gathered && lane == 0 && g) atomicAdd(gathered + (blockIdx.x % kSpread) * kSpreadStride, g);
}


// Entries p .. p + U*64 - 1 of a B row (base bb, length bl >= 1), one per lane
// and step u.  The loads are unconditional (positions clamped to the row's
// last entry) and their results are not inspected here, so a chunk issues as
// one straight run of loads whose latency later work can hide; lanes past the
// row end hold a copy of the last entry and are masked by the consumer.
template <typename V, int U>
__device__ __forceinline__ void gather_chunk(const MatView<V> &B, int64_t bb, int p, int bl,
                                             int lane, int (&c)[U], V (&bv)[U]) {
    const int32_t *colp = B.col + bb;
    const V *valp = B.val + bb;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int at = min(p + u * kWave + lane, bl - 1);
        c[u] = colp[at];
        bv[u] = valp[at];
    }
}

// Whether a chunk loaded at position p of a B row of length bl lies wholly
// inside the window (all its entries exist and the last, the largest column,
// is below whi); uniform over the wave.
template <int U>
__device__ __forceinline__ bool chunk_full(const int (&c)[U], int p, int bl, int whi) {
    const int last = __builtin_amdgcn_readlane(c[U - 1], kWave - 1);
    return p + U * kWave <= bl && last < whi;
}

// Accumulator slot of a column inside the current window, and back.  Dense
// windows hold consecutive columns from wlo.  Page windows hold, page after
// page, the pages of the group's column range that hold entries: tab gives a
// page's rank among them in column order (pages numbered from plo), the window
// holds ranks r0 .. r0 + T/2^shift - 1, and wpg lists the window's pages by place.
struct WinMap {
    const int16_t *tab;  // nullptr: dense window
    const int16_t *wpg;
    int wlo, plo, r0, shift;
    __device__ __forceinline__ int slot(int col) const {
        if (!tab) return col - wlo;
        return (((int)tab[(col >> shift) - plo] - r0) << shift) | (col & ((1 << shift) - 1));
    }
    __device__ __forceinline__ int col(int s) const {
        if (!tab) return wlo + s;
        return ((plo + (int)wpg[s >> shift]) << shift) | (s & ((1 << shift) - 1));
    }
};

// Adds one chunk loaded by gather_chunk at position p of a B row of length bl
// (columns c, values bv) times the group's coefficients aq into the LDS windows
// (columns below whi, slots from wm) of the rows present at the slot (bits of
// mq; a uniform test).
// Lanes whose entry lies outside the window or past the row end are masked
// off.  Returns the number of the chunk's entries inside the window (a prefix
// of the chunk) and, in *next, the column of the first entry after them
// (INT_MAX past the row end).
template <typename V, int R, int T, int U>
__device__ __forceinline__ int group_accumulate(double (*acc)[T], const int (&c)[U],
                                                const V (&bv)[U], const V (&aq)[R], uint32_t mq,
                                                int p, int bl, const WinMap &wm, int whi,
                                                int lane, int *next) {
    int got = 0, col[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        col[u] = p + u * kWave + lane < bl ? c[u] : INT_MAX;
        got += __popcll(__ballot(col[u] < whi));
    }
    // a slot present in every row of the group (most of them) adds without
    // testing the row bits
    const bool full = mq == (R >= 32 ? ~0u : (1u << R) - 1u);
#pragma unroll
    for (int u = 0; u < U; ++u) {
        if (col[u] < whi) {
            const int s = wm.slot(col[u]);
            if (full) {
#pragma unroll
                for (int r = 0; r < R; ++r)
                    atomicAdd(&acc[r][s], (double)aq[r] * (double)bv[u]);
            } else {
#pragma unroll
                for (int r = 0; r < R; ++r)
                    if ((mq >> r) & 1u) atomicAdd(&acc[r][s], (double)aq[r] * (double)bv[u]);
            }
        }
    }
    if (got < U * kWave) {
        int cs = INT_MAX;
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (u == (got >> 6)) cs = col[u];
        *next = __shfl(cs, got & (kWave - 1));
    }
    return got;
}


// ---------------------------------------------------------------------------
// numeric product: C = diag*I + coef*A*B + dcoef*D, row-wise (Gustavson)
// ---------------------------------------------------------------------------
// One workgroup computes R consecutive output rows i .. i+R-1 (R = 1: a single
// row, whose own A entries are the slots; R > 1: the merged A list of the
// group from k_merge_group).  The rows' columns are swept in windows of T
// consecutive columns held as dense LDS accumulators (R x T values, native
// ds_add).  Each wave takes 64 slots at a time (fewer when the list is short,
// so that every wave gets some); lane q holds slot q's B-row descriptor and
// coefficients, broadcast with readlane.  A slot's B row
// is streamed in chunks of U x 64 entries (coalesced col/val loads); B rows are
// sorted, so the entries inside the window are a prefix of what is loaded, and
// the sweep of a B row stops at the first chunk that runs past the window.
// The first chunk of the next slot is loaded before the current one is
// accumulated.  A row wider than T sweeps several windows, resuming each B row
// from its per-slot cursor and skipping B rows with nothing left in the window
// (cnext), so each B entry is read once per group.  With R > 1 every gathered
// chunk feeds the windows of all R rows -- neighbouring rows of these matrices
// reference almost the same rows of B, so the group pays its B bytes once.
// When B's rows are short (a few entries, e.g. B = A), each lane instead walks
// its own slot's row, a wave adding 64 slots at once.
// Finished windows get the D row and the diagonal added in LDS and are written
// in column order (per-wave ballot compaction, zeros dropped); per-row sums of
// squares of the product and of the output come out in a fixed order.
// PG (page windows, with epi.pages): the group first marks in an LDS table the
// pages (2^shift columns) of its column range that its B rows, D rows and
// diagonal occupy, ranks them, and runs its windows over the occupied pages
// only: the output rows of a grid operator fill a small part of their column
// range, so a few page windows replace many dense ones.  A group whose range
// fits one dense window, or holds more pages than the table, uses dense windows.
template <typename V, int R, int T, int NT, int U, bool PG>
__global__ __launch_bounds__(NT) void k_spgemm_rows(
    const int32_t *__restrict__ rows, const int32_t *__restrict__ mk,
    const uint32_t *__restrict__ mm, const int32_t *__restrict__ mc, const V *__restrict__ cv,
    const int32_t *__restrict__ mlen, MatView<V> A, MatView<V> B, MatView<V> D, V coef,
    V dcoef, V diag, const int32_t *__restrict__ row_lo, const int32_t *__restrict__ row_span,
    const int64_t *__restrict__ off, int64_t base, int32_t *__restrict__ out_col,
    V *__restrict__ out_val, int32_t *__restrict__ out_len, int32_t *__restrict__ cursor,
    int32_t *__restrict__ cnext, double *__restrict__ sq_prod, double *__restrict__ sq_out,
    int64_t *__restrict__ out_count, ProductEpi epi) {
    constexpr int NW = NT / kWave;
    constexpr int REG = T / NW;
    static_assert(T % (NW * kWave) == 0, "tile must split evenly over the waves");
    // FP64 accumulators for both value types: LDS atomic add of FP32 is far
    // slower than of FP64 on this chip, and a product of two FP32 values is
    // exact in FP64
    __shared__ double acc[R][T];
    __shared__ int wcnt[NW];
    __shared__ double wsum[2 * R][NW];  // per-wave partial sums of squares, per row
    __shared__ int wrt[R];              // entries written so far, per row
    __shared__ uint32_t hst[kBuckets];  // bucket histogram of the candidates
    __shared__ double wpre[R][NW];      // per-wave sums of squares not stored, per row
    __shared__ int16_t ptab[PG ? kPageMax : 1];             // page -> rank (-1: empty)
    __shared__ int16_t wpg[PG ? (T >> kPageMinShift) : 1];  // window place -> page
    __shared__ int64_t scan_w[NW];
    __shared__ int wnext;
    __shared__ unsigned long long madd_sh;

    const int lane = lane_id(), wave = wave_id();
    const int i = rows[xcd_row(blockIdx.x, gridDim.x)];
    int lo = INT_MAX, hi = INT_MIN;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        lo = min(lo, row_lo[i + r]);
        hi = max(hi, row_lo[i + r] + row_span[i + r]);
    }
    // lower: only columns <= the row itself (the product is symmetric and its
    // upper triangle is mirrored afterwards); B rows are then read only up to
    // the diagonal, as the sweep stops at the last window
    bool all_lower = true;
#pragma unroll
    for (int r = 0; r < R; ++r) all_lower = all_lower && epi.lower.of(i + r);
    if (all_lower) hi = min(hi, i + R);
    const int64_t mbeg = A.beg[i];
    const int ml = R == 1 ? A.len[i] : mlen[i];
    const bool has_d = D.len != nullptr;
    // slots per wave and batch: at most 64, sized so that every wave gets the same
    // number of batches and slots (a list of 1,500 slots: two batches of 47 per
    // wave, not two of 64 for half the waves and one for the others -- each
    // window waits for its slowest wave)
    const int rounds = (ml + NW * kWave - 1) / (NW * kWave);
    const int step = max(1, (ml + NW * rounds - 1) / (NW * max(rounds, 1)));

    for (int q = threadIdx.x; q < 2 * R * NW; q += NT) (&wsum[0][0])[q] = 0.0;
    if (threadIdx.x < R) wrt[threadIdx.x] = 0;
    if (threadIdx.x == 0) madd_sh = 0ull;
    unsigned long long madd = 0;  // multiply-adds of this wave (uniform), or lane (short B)
    if (epi.hist)
        for (int q = threadIdx.x; q < kBuckets; q += NT) hst[q] = 0u;
    for (int q = threadIdx.x; q < R * NW; q += NT) (&wpre[0][0])[q] = 0.0;

    int nwin = hi > lo ? (hi - lo + T - 1) / T : 0;
    bool pm = false;
    int S = 0, plo = 0, np = 0, npg = 0;  // npg: occupied pages
    if constexpr (PG) {
        S = epi.pages.shift;
        plo = lo >> S;
        np = hi > lo ? ((hi - 1) >> S) - plo + 1 : 0;
        // (a range that fits one dense window gains nothing from pages)
        pm = np > 0 && np <= kPageMax && hi - lo > T;
    }
    if (pm) {
        // mark the occupied pages: those of every slot's B row, of the D rows
        // and of the diagonal (plain stores of 1: concurrent writers agree)
        for (int q = threadIdx.x; q < np; q += NT) ptab[q] = 0;
        __syncthreads();
        const PageLists &pl = epi.pages;
        // slots spread over the waves as in the accumulation below
        for (int t0 = wave * step; t0 < ml; t0 += NW * step) {
            const int t = t0 + lane;
            int64_t pb = 0;
            int pn = 0;
            if (lane < step && t < ml) {
                const int k = R == 1 ? A.col[mbeg + t] : mk[mbeg + t];
                pb = pl.beg[k];
                pn = pl.len[k];
            }
            uint64_t act = __ballot(pn > 0);
            while (act) {
                const int q = __builtin_ctzll(act);
                act &= act - 1;
                const int64_t b = rl_i64(pb, q);
                const int l = rl_i32(pn, q);
                for (int j0 = 0; j0 < l; j0 += U * kWave) {
                    int pq[U];
#pragma unroll
                    for (int u = 0; u < U; ++u) pq[u] = pl.pg[b + min(j0 + u * kWave + lane, l - 1)];
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const int rel = pq[u] - plo;
                        if (rel >= 0 && rel < np) ptab[rel] = 1;
                    }
                }
            }
        }
        if (has_d) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int dl = D.len[i + r];
                const int64_t db = D.beg[i + r];
                for (int q = threadIdx.x; q < dl; q += NT) {
                    const int rel = (D.col[db + q] >> S) - plo;
                    if (rel >= 0 && rel < np) ptab[rel] = 1;
                }
            }
        }
        if (diag != V(0) && threadIdx.x < R) {
            const int ir = i + threadIdx.x;
            if (ir >= lo && ir < hi) ptab[(ir >> S) - plo] = 1;
        }
        __syncthreads();
        // ranks in column order: each thread scans a run of consecutive pages
        constexpr int PER = (kPageMax + NT - 1) / NT;
        const int q0 = threadIdx.x * PER;
        int cnt = 0;
#pragma unroll
        for (int e = 0; e < PER; ++e)
            if (q0 + e < np) cnt += ptab[q0 + e];
        int64_t total = 0;
        int run = (int)block_excl_scan<int64_t, NT>(cnt, scan_w, &total);
#pragma unroll
        for (int e = 0; e < PER; ++e)
            if (q0 + e < np) {
                const int m = ptab[q0 + e];
                ptab[q0 + e] = (int16_t)(m ? run : -1);
                run += m;
            }
        npg = (int)total;
        nwin = (npg + (T >> S) - 1) / (T >> S);
        __syncthreads();
    }
    const bool multi = nwin > 1;
    for (int w = 0; w < nwin; ++w) {
        int wlo, whi, nsl, r0 = 0;
        if (pm) {
            // this window's pages: ranks r0 .. r1 - 1; the next window starts at
            // the page of rank r1 (or at the end of the range)
            const int tp = T >> S;
            r0 = w * tp;
            const int r1 = min(npg, r0 + tp);
            if (threadIdx.x == 0) wnext = -1;
            __syncthreads();
            for (int q = threadIdx.x; q < np; q += NT) {
                const int rk = ptab[q];
                if (rk >= r0 && rk < r1) wpg[rk - r0] = (int16_t)q;
                else if (rk == r1) wnext = q;
            }
            __syncthreads();
            const int nx = wnext;
            wlo = (plo + wpg[0]) << S;
            whi = nx >= 0 ? (plo + nx) << S : hi;
            nsl = (r1 - r0) << S;
        } else {
            wlo = lo + w * T;
            whi = min(hi, wlo + T);
            nsl = whi - wlo;
        }
        const bool first = (w == 0);
        const WinMap wm{pm ? ptab : nullptr, wpg, wlo, plo, r0, S};
        for (int s = threadIdx.x; s < nsl; s += NT)
#pragma unroll
            for (int r = 0; r < R; ++r) acc[r][s] = 0.0;
        __syncthreads();

        for (int t0 = wave * step; t0 < ml; t0 += NW * step) {
            const int t = t0 + lane;
            const bool own = lane < step && t < ml;
            // after the first window a slot's next column alone says whether it has
            // entries in this one: a batch with none skips its descriptor loads
            // (its cursors stay as they are)
            if (!first && !__ballot(own && cnext[mbeg + t] < whi)) continue;
            int bl = 0, cur = 0, nc = INT_MIN, msk = 0;
            int64_t bb = 0;
            V a[R];  // this lane's slot: coefficient of each row of the group (0 if absent)
#pragma unroll
            for (int r = 0; r < R; ++r) a[r] = V(0);
            if (own) {
                const int64_t pa = mbeg + t;
                int k;
                if constexpr (R == 1) {  // a single row: its own entries are the slots
                    k = A.col[pa];
                    a[0] = coef * A.val[pa];
                    msk = 1;
                } else {
                    k = mk[pa];
                    const uint32_t m = mm[pa];
                    const V *cp = cv + mbeg + mc[pa];
                    int j = 0;
#pragma unroll
                    for (int r = 0; r < R; ++r)
                        if ((m >> r) & 1u) a[r] = coef * cp[j++];
                    msk = (int)m;
                }
                bb = B.beg[k];
                bl = B.len[k];
                if (!first) { cur = cursor[pa]; nc = cnext[pa]; }
            }
            if (epi.short_b) {
                // short B rows: every lane walks the in-window part of its own
                // slot's row, so a wave adds up to 64 slots at once
                if (own && cur < bl && nc < whi) {
                    int p = cur, nx = INT_MAX;
                    for (; p < bl; ++p) {
                        const int col = B.col[bb + p];
                        if (col >= whi) { nx = col; break; }
                        const double bvv = (double)B.val[bb + p];
#pragma unroll
                        for (int r = 0; r < R; ++r)
                            if ((msk >> r) & 1)
                                atomicAdd(&acc[r][wm.slot(col)], (double)a[r] * bvv);
                    }
                    madd += (unsigned long long)(p - cur) * (unsigned)__popc((unsigned)msk);
                    cur = p;
                    nc = nx;
                }
                if (multi && own) { cursor[mbeg + t] = cur; cnext[mbeg + t] = nc; }
                continue;
            }
            // slots with B entries left in this window; the others cost nothing
            uint64_t act = __ballot(own && cur < bl && nc < whi);
            if (act) {
                int c[U], cn[U];
                V bv[U], bn[U];
                int q = __builtin_ctzll(act);
                act &= act - 1;
                int p = rl_i32(cur, q), blq = rl_i32(bl, q);
                int64_t bbq = rl_i64(bb, q);
                gather_chunk<V, U>(B, bbq, p, blq, lane, c, bv);
                while (true) {
                    // issue the first chunk of the next active slot before this
                    // slot's accumulation, so its latency overlaps the atomics.  The
                    // loads are issued on every pass (re-reading this slot's chunk
                    // when no slot is left) so that all paths wait alike.
                    const bool more = act != 0;
                    const int qn = more ? __builtin_ctzll(act) : q;
                    act &= act - 1;
                    const int pn = rl_i32(cur, qn), bln = rl_i32(bl, qn);
                    const int64_t bbn = rl_i64(bb, qn);
                    gather_chunk<V, U>(B, bbn, pn, bln, lane, cn, bn);
                    V aq[R];
#pragma unroll
                    for (int r = 0; r < R; ++r) aq[r] = rl_val(a[r], q);
                    const uint32_t mq = (uint32_t)rl_i32(msk, q);
                    // A chunk lying wholly inside the window (its last entry in the
                    // row and before whi) is followed by a refill from the same row:
                    // that refill is issued before the chunk is accumulated, so its
                    // latency overlaps the atomics (as the next slot's does).
                    int cr[U];
                    V br[U];
                    if (chunk_full<U>(c, p, blq, whi))
                        gather_chunk<V, U>(B, bbq, p + U * kWave, blq, lane, cr, br);
                    int nxt = INT_MAX;
                    int got = group_accumulate<V, R, T, U>(acc, c, bv, aq, mq, p, blq, wm,
                                                           whi, lane, &nxt);
                    const int pstart = p;
                    p += got;
                    while (got == U * kWave) {  // the refill was issued above
#pragma unroll
                        for (int u = 0; u < U; ++u) { c[u] = cr[u]; bv[u] = br[u]; }
                        if (chunk_full<U>(c, p, blq, whi))
                            gather_chunk<V, U>(B, bbq, p + U * kWave, blq, lane, cr, br);
                        got = group_accumulate<V, R, T, U>(acc, c, bv, aq, mq, p, blq, wm,
                                                           whi, lane, &nxt);
                        p += got;
                    }
                    madd += (unsigned long long)(p - pstart) * (unsigned)__popc(mq);
                    // column of the first entry beyond the window, for the next one
                    if (multi && lane == q) nc = nxt;
                    if (multi && lane == q) cur = p;
                    if (!more) break;
                    q = qn;
                    p = pn;
                    blq = bln;
                    bbq = bbn;
#pragma unroll
                    for (int u = 0; u < U; ++u) { c[u] = cn[u]; bv[u] = bn[u]; }
                }
            }
            if (multi && own) { cursor[mbeg + t] = cur; cnext[mbeg + t] = nc; }
        }
        __syncthreads();

        if (sq_prod) {
            for (int r = 0; r < R; ++r) {
                double x = 0.0;
                for (int s = threadIdx.x; s < nsl; s += NT) {
                    const double v = acc[r][s];
                    x += sym_weight(epi.lower.of(i + r), wm.col(s), i + r) * v * v;
                }
                x = wave_sum(x);
                if (lane == 0) wsum[2 * r][wave] += x;
            }
            __syncthreads();
        }
        if (has_d) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int dl = D.len[i + r];
                const int64_t db = D.beg[i + r];
                for (int q = threadIdx.x; q < dl; q += NT) {
                    const int c = D.col[db + q];
                    if (c >= wlo && c < whi)
                        acc[r][wm.slot(c)] += (double)dcoef * (double)D.val[db + q];
                }
            }
            __syncthreads();
        }
        if (diag != V(0) && threadIdx.x < R) {
            const int r = threadIdx.x, ir = i + r;
            if (ir >= wlo && ir < whi) acc[r][wm.slot(ir)] += (double)diag;
        }
        __syncthreads();

        for (int r = 0; r < R; ++r) {
            const int64_t obase = off[i + r] - base;
            const int rbeg = wave * REG;
            // columns written for this row: all, or up to the diagonal
            const bool low = epi.lower.of(i + r);
            int cw = 0;
            double pr = 0.0;
            for (int s0 = rbeg; s0 < rbeg + REG && s0 < nsl; s0 += kWave) {
                const int s = s0 + lane;
                const int cs = s < nsl ? wm.col(s) : INT_MAX;
                const V v = cs != INT_MAX && (!low || cs <= i + r) ? (V)acc[r][s] : V(0);
                bool keep = v != V(0);
                if (keep && (epi.hist || epi.keep_from > 0)) {
                    // the filter's histogram counts every candidate; entries in
                    // buckets below keep_from are dropped by any cut it can choose
                    const int bk = bucket_of(as_f64(v));
                    const double wgt = sym_weight(low, cs, i + r);
                    if (epi.hist) atomicAdd(&hst[bk], (uint32_t)wgt);
                    if (bk < epi.keep_from) {
                        keep = false;
                        pr += wgt * as_f64(v) * as_f64(v);
                    }
                }
                cw += __popcll(__ballot(keep));
            }
            if (epi.sq_pre) {
                pr = wave_sum(pr);
                if (lane == 0) wpre[r][wave] += pr;
            }
            if (lane == 0) wcnt[wave] = cw;
            __syncthreads();
            int o = wrt[r], tot = 0;
            double y = 0.0;
            for (int wv = 0; wv < NW; ++wv) {
                const int c = wcnt[wv];
                if (wv < wave) o += c;
                tot += c;
            }
            for (int s0 = rbeg; s0 < rbeg + REG && s0 < nsl; s0 += kWave) {
                const int s = s0 + lane;
                const int cs = s < nsl ? wm.col(s) : INT_MAX;
                const V v = cs != INT_MAX && (!low || cs <= i + r) ? (V)acc[r][s] : V(0);
                const bool nz = v != V(0) && (epi.keep_from == 0 ||
                                              bucket_of(as_f64(v)) >= epi.keep_from);
                const uint64_t m = __ballot(nz);
                if (nz) {
                    if (!epi.no_store) {
                        const int64_t pos = obase + o + lanes_below(m);
                        out_col[pos] = cs;
                        out_val[pos] = v;
                    }
                    y += sym_weight(low, cs, i + r) * as_f64(v) * as_f64(v);
                }
                o += __popcll(m);
            }
            y = wave_sum(y);
            if (lane == 0) wsum[2 * r + 1][wave] += y;
            __syncthreads();  // every wave has read wrt[r] and wcnt
            if (threadIdx.x == 0) wrt[r] += tot;
        }
    }
    if (epi.madds) {
        // short B rows: per lane; otherwise the same count in every lane of a wave
        if (epi.short_b) madd = wave_sum(madd);
        if (lane == 0 && madd) atomicAdd(&madd_sh, madd);
    }
    __syncthreads();
    if (epi.madds && threadIdx.x == 0 && madd_sh)
        atomicAdd(epi.madds + (blockIdx.x % kSpread) * kSpreadStride, madd_sh);
    if (epi.hist)
        for (int q = threadIdx.x; q < kBuckets; q += NT)
            if (hst[q]) atomicAdd((unsigned long long *)&epi.hist[q], (unsigned long long)hst[q]);
    if (epi.sq_pre && threadIdx.x < R) {
        double x = 0.0;
        for (int w = 0; w < NW; ++w) x += wpre[threadIdx.x][w];
        epi.sq_pre[i + threadIdx.x] = x;
    }
    if (threadIdx.x == 0) {
        unsigned long long tw = 0;
        for (int r = 0; r < R; ++r) {
            double x = 0.0, y = 0.0;
            for (int w = 0; w < NW; ++w) { x += wsum[2 * r][w]; y += wsum[2 * r + 1][w]; }
            out_len[i + r] = wrt[r];
            if (sq_prod) sq_prod[i + r] = x;
            if (sq_out) sq_out[i + r] = y;
            tw += (unsigned long long)wrt[r];
        }
        if (out_count)
            atomicAdd((unsigned long long *)(out_count + (blockIdx.x % kSpread) * kSpreadStride),
                      tw);
    }
}

// ---------------------------------------------------------------------------
// numeric product with register accumulators (row groups, short windows)
// ---------------------------------------------------------------------------
// The same product as k_spgemm_rows for a group of R consecutive output rows
// i .. i+R-1 (merged slot list from k_merge_group), accumulated in registers
// instead of LDS atomics.  The columns are swept in windows of W = 64*NB
// columns; lane l of every wave holds the R x NB partial sums of columns
// wlo + 64j + l.  A window starts at the smallest column that any slot's B row,
// any D row or the diagonal still has to add (per-slot cursors as in
// k_spgemm_rows), so the empty stretches between the column clusters of a
// grid-ordered matrix cost nothing.  Each wave takes a fixed share of the
// slots; a slot's in-window B entries (a prefix of what is left of its row)
// come in 64-entry chunks, are written to the wave's own LDS strip at their
// column offset, read back by the lanes that own those columns, cleared, and
// multiplied by the slot's R coefficients (scalar loads) into the registers:
// one LDS write, read and clear per B entry instead of R atomic adds, and the
// R multiply-adds in registers.  At the window's end every wave adds its
// registers into the shared R x W LDS window (one atomic add per column and
// row), and each row is finished by one wave (R/NW rows per wave): products'
// sum of squares, the D row and the diagonal added through the wave's strip,
// the filter's histogram and pre-drop, compaction in column order.
template <typename V, int R, int NB, int NT>
__global__ __launch_bounds__(NT) void k_spgemm_regtile(
    const int32_t *__restrict__ rows, const int32_t *__restrict__ mk,
    const uint32_t *__restrict__ mm, const int32_t *__restrict__ mc, const V *__restrict__ cv,
    const int32_t *__restrict__ mlen, MatView<V> A, MatView<V> B, MatView<V> D, V coef,
    V dcoef, V diag, const int32_t *__restrict__ row_lo, const int32_t *__restrict__ row_span,
    const int64_t *__restrict__ off, int64_t base, int32_t *__restrict__ out_col,
    V *__restrict__ out_val, int32_t *__restrict__ out_len, int32_t *__restrict__ cursor,
    int32_t *__restrict__ cnext, double *__restrict__ sq_prod, double *__restrict__ sq_out,
    int64_t *__restrict__ out_count, ProductEpi epi) {
    constexpr int NW = NT / kWave;
    constexpr int W = kWave * NB;
    static_assert(R % NW == 0 || NW % R == 0, "rows must split evenly over the waves");
    constexpr int RPW = R >= NW ? R / NW : 1;  // rows finished per wave
    __shared__ double acc[R][W];
    __shared__ double strip[NW][W];
    __shared__ uint32_t hst[kBuckets];
    __shared__ int wmin[NW];

    const int lane = lane_id(), wave = wave_id();
    const int i = rows[xcd_row(blockIdx.x, gridDim.x)];
    int hi = INT_MIN;
#pragma unroll
    for (int r = 0; r < R; ++r) hi = max(hi, row_lo[i + r] + row_span[i + r]);
    bool all_lower = true;
#pragma unroll
    for (int r = 0; r < R; ++r) all_lower = all_lower && epi.lower.of(i + r);
    if (all_lower) hi = min(hi, i + R);
    const int64_t mbeg = A.beg[i];
    const int ml = mlen[i];
    const bool has_d = D.len != nullptr;

    for (int q = threadIdx.x; q < R * W; q += NT) (&acc[0][0])[q] = 0.0;
    for (int q = threadIdx.x; q < NW * W; q += NT) (&strip[0][0])[q] = 0.0;
    if (epi.hist)
        for (int q = threadIdx.x; q < kBuckets; q += NT) hst[q] = 0u;

    // slots: cursor at the start of the B row, next column its first
    int mymin = INT_MAX;
    for (int t0 = wave * kWave; t0 < ml; t0 += NT) {
        const int t = t0 + lane;
        if (t < ml) {
            const int k = mk[mbeg + t];
            const int bl = B.len[k];
            const int c0 = bl > 0 ? B.col[B.beg[k]] : INT_MAX;
            cursor[mbeg + t] = 0;
            cnext[mbeg + t] = c0;
            mymin = min(mymin, c0);
        }
    }
    // rows finished by this wave: D cursor, next D column, next diagonal column
    int dpos[RPW], dnx[RPW];
    double sq_p[RPW], sq_o[RPW], sq_r[RPW];
    int wrt[RPW];
#pragma unroll
    for (int u = 0; u < RPW; ++u) {
        const int r = wave + u * NW;
        dpos[u] = 0;
        dnx[u] = INT_MAX;
        sq_p[u] = 0.0;
        sq_o[u] = 0.0;
        sq_r[u] = 0.0;
        wrt[u] = 0;
        if (r < R) {
            if (has_d && D.len[i + r] > 0) dnx[u] = D.col[D.beg[i + r]];
            if (diag != V(0)) dnx[u] = min(dnx[u], i + r);
            mymin = min(mymin, dnx[u]);
        }
    }
    mymin = wave_min(mymin);
    if (lane == 0) wmin[wave] = mymin;
    __syncthreads();
    int wlo = INT_MAX;
    for (int w = 0; w < NW; ++w) wlo = min(wlo, wmin[w]);
    double *mystrip = strip[wave];

    while (wlo < hi) {
        const int whi = (int)min((int64_t)wlo + W, (int64_t)hi);
        double racc[R][NB];
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int j = 0; j < NB; ++j) racc[r][j] = 0.0;
        uint32_t touched = 0u;  // bit j: block j of some row received products
        mymin = INT_MAX;
        for (int t0 = wave * kWave; t0 < ml; t0 += NT) {
            const int t = t0 + lane;
            const bool own = t < ml;
            int nc = own ? cnext[mbeg + t] : INT_MAX;
            const bool was_active = nc < whi;
            uint64_t act = __ballot(was_active);
            if (!act) {
                mymin = min(mymin, nc);
                continue;
            }
            int cur = 0, bl = 0, msk = 0, cpo = 0;
            int64_t bb = 0;
            if (was_active) {
                const int64_t pa = mbeg + t;
                const int k = mk[pa];
                msk = (int)mm[pa];
                cpo = mc[pa];
                bb = B.beg[k];
                bl = B.len[k];
                cur = cursor[pa];
            }
            // first chunk of the first active slot
            int q = __builtin_ctzll(act);
            act &= act - 1;
            int p = rl_i32(cur, q), blq = rl_i32(bl, q);
            int64_t bbq = rl_i64(bb, q);
            int cc;
            V bv;
            {
                const int at = min(p + lane, blq - 1);
                cc = B.col[bbq + at];
                bv = B.val[bbq + at];
            }
            while (true) {
                // issue the next active slot's first chunk before this one is used
                const bool more = act != 0;
                const int qn = more ? __builtin_ctzll(act) : q;
                act &= act - 1;
                const int pn = rl_i32(cur, qn), bln = rl_i32(bl, qn);
                const int64_t bbn = rl_i64(bb, qn);
                int cn;
                V bn;
                {
                    const int at = min(pn + lane, bln - 1);
                    cn = B.col[bbn + at];
                    bn = B.val[bbn + at];
                }
                // this slot's coefficients (uniform: scalar loads)
                const uint32_t mq = (uint32_t)rl_i32(msk, q);
                const V *cp = cv + mbeg + rl_i32(cpo, q);
                double a[R];
                {
                    int idx = 0;
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        a[r] = 0.0;
                        if ((mq >> r) & 1u) a[r] = (double)(coef * cp[idx++]);
                    }
                }
                int nxt = INT_MAX;
                while (true) {
                    const bool in = p + lane < blq && cc < whi;
                    const uint64_t bal = __ballot(in);
                    const int got = __popcll(bal);
                    if (got > 0) {
                        // columns of the chunk's first and last in-window entries
                        const int c_first = rl_i32(cc, 0) - wlo;
                        const int c_last = __shfl(cc, got - 1) - wlo;
                        const int jlo = c_first >> 6, jhi = c_last >> 6;
                        if (in) mystrip[cc - wlo] = (double)bv;
                        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                        __builtin_amdgcn_wave_barrier();
                        double x[NB];
#pragma unroll
                        for (int j = 0; j < NB; ++j)
                            x[j] = (j >= jlo && j <= jhi) ? mystrip[j * kWave + lane] : 0.0;
                        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
                        __builtin_amdgcn_wave_barrier();
                        if (in) mystrip[cc - wlo] = 0.0;
#pragma unroll
                        for (int j = 0; j < NB; ++j) {
                            if (j >= jlo && j <= jhi) {
                                touched |= 1u << j;
#pragma unroll
                                for (int r = 0; r < R; ++r)
                                    if ((mq >> r) & 1u) racc[r][j] = fma(a[r], x[j], racc[r][j]);
                            }
                        }
                    }
                    p += got;
                    if (got < kWave) {
                        // the entry after the in-window ones (if the row goes on)
                        if (p < blq) nxt = __shfl(cc, got);
                        break;
                    }
                    if (p >= blq) break;
                    const int at = min(p + lane, blq - 1);
                    cc = B.col[bbq + at];
                    bv = B.val[bbq + at];
                }
                if (lane == q) { cur = p; nc = nxt; }
                if (!more) break;
                q = qn;
                p = pn;
                blq = bln;
                bbq = bbn;
                cc = cn;
                bv = bn;
            }
            if (was_active) {  // slots outside the window keep their cursors
                cursor[mbeg + t] = cur;
                cnext[mbeg + t] = nc;
            }
            mymin = min(mymin, nc);
        }
        // add this wave's registers into the shared window
        if (touched) {
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int j = 0; j < NB; ++j)
                    if ((touched >> j) & 1u) atomicAdd(&acc[r][j * kWave + lane], racc[r][j]);
        }
        __syncthreads();

        // finish this wave's rows for the window
        const int nsl = whi - wlo;
#pragma unroll
        for (int u = 0; u < RPW; ++u) {
            const int r = wave + u * NW;
            if (r >= R) break;
            const int ir = i + r;
            const bool low = epi.lower.of(ir);
            const int lim = low ? min(nsl, ir + 1 - wlo) : nsl;
            double v[NB];
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                const int s = j * kWave + lane;
                v[j] = acc[r][s];
                acc[r][s] = 0.0;
                if (sq_prod) sq_p[u] += sym_weight(low, wlo + s, ir) * v[j] * v[j];
            }
            if (has_d && dnx[u] < whi && dpos[u] < D.len[ir]) {
                const int dl = D.len[ir];
                const int64_t db = D.beg[ir];
                while (true) {
                    const int at = dpos[u] + lane;
                    const int c = at < dl ? D.col[db + at] : INT_MAX;
                    const bool in = c < whi;
                    const int got = __popcll(__ballot(in));
                    if (in) mystrip[c - wlo] = (double)dcoef * (double)D.val[db + at];
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
#pragma unroll
                    for (int j = 0; j < NB; ++j) v[j] += mystrip[j * kWave + lane];
                    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    if (in) mystrip[c - wlo] = 0.0;
                    dpos[u] += got;
                    if (got < kWave) break;
                }
            }
            // next column this row needs from D or the diagonal (recomputed every
            // window: a column already passed must never be proposed again)
            dnx[u] = has_d && dpos[u] < D.len[ir] ? D.col[D.beg[ir] + dpos[u]] : INT_MAX;
            if (diag != V(0)) {
                if (ir >= wlo && ir < whi) {
                    const int s = ir - wlo;
                    if (lane == (s & (kWave - 1))) {
#pragma unroll
                        for (int j = 0; j < NB; ++j)
                            if (j == (s >> 6)) v[j] += (double)diag;
                    }
                }
                if (ir >= whi) dnx[u] = min(dnx[u], ir);
            }
            const int64_t obase = off[ir] - base;
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                const int s = j * kWave + lane;
                const V val = s < lim ? (V)v[j] : V(0);
                bool keep = val != V(0);
                const double wgt = sym_weight(low, wlo + s, ir);
                if (keep && (epi.hist || epi.keep_from > 0)) {
                    const int bk = bucket_of(as_f64(val));
                    if (epi.hist) atomicAdd(&hst[bk], (uint32_t)wgt);
                    if (bk < epi.keep_from) {
                        keep = false;
                        sq_r[u] += wgt * as_f64(val) * as_f64(val);
                    }
                }
                const uint64_t m = __ballot(keep);
                if (keep) {
                    if (!epi.no_store) {
                        const int64_t pos = obase + wrt[u] + lanes_below(m);
                        out_col[pos] = wlo + s;
                        out_val[pos] = val;
                    }
                    sq_o[u] += wgt * as_f64(val) * as_f64(val);
                }
                wrt[u] += __popcll(m);
            }
            mymin = min(mymin, dnx[u]);
        }
        mymin = wave_min(mymin);
        if (lane == 0) wmin[wave] = mymin;
        __syncthreads();
        // every candidate lies at or beyond whi (slots stopped at their first
        // entry >= whi, D cursors likewise, passed diagonals are not proposed);
        // the bound keeps the sweep moving forward whatever the inputs
        int nxt_lo = INT_MAX;
        for (int w = 0; w < NW; ++w) nxt_lo = min(nxt_lo, wmin[w]);
        wlo = max(nxt_lo, whi);
    }
    if (epi.hist) {
        __syncthreads();
        for (int q = threadIdx.x; q < kBuckets; q += NT)
            if (hst[q]) atomicAdd((unsigned long long *)&epi.hist[q], (unsigned long long)hst[q]);
    }
    unsigned long long tw = 0;
#pragma unroll
    for (int u = 0; u < RPW; ++u) {
        const int r = wave + u * NW;
        if (r >= R) break;
        const double xp = wave_sum(sq_p[u]), xo = wave_sum(sq_o[u]), xr = wave_sum(sq_r[u]);
        if (lane == 0) {
            out_len[i + r] = wrt[u];
            if (sq_prod) sq_prod[i + r] = xp;
            if (sq_out) sq_out[i + r] = xo;
            if (epi.sq_pre) epi.sq_pre[i + r] = xr;
        }
        tw += (unsigned long long)wrt[u];
    }
    if (out_count && lane == 0 && tw)
        atomicAdd((unsigned long long *)(out_count + (blockIdx.x % kSpread) * kSpreadStride), tw);
}

// ---------------------------------------------------------------------------
// gapped -> compact copy (one wave per row)
// ---------------------------------------------------------------------------
template <typename V>
__global__ void k_copy_rows(const int64_t *src_off, int64_t src_base, const int32_t *len,
                            const int32_t *scol, const V *sval, int64_t r0, int64_t r1,
                            const int64_t *dst_ptr, int32_t *dcol, V *dval) {
    const int64_t i = r0 + (int64_t)blockIdx.x * (blockDim.x / kWave) + wave_id();
    if (i >= r1) return;
    const int l = len[i];
    const int64_t s = src_off[i] - src_base, d = dst_ptr[i];
    for (int p = lane_id(); p < l; p += kWave) {
        dcol[d + p] = scol[s + p];
        dval[d + p] = sval[s + p];
    }
}

// ---------------------------------------------------------------------------
// filtering: histogram, selection, survivor count, scatter
// ---------------------------------------------------------------------------
constexpr int kHistThreads = 512;
constexpr int kHistRowsPerBlock = 128;

template <typename V>
__global__ __launch_bounds__(kHistThreads) void k_histogram(MatView<V> X, const int64_t *seg_rows,
                                                            uint64_t *hist, LowerRows lower) {
    __shared__ uint32_t h[kBuckets];
    const int s = blockIdx.y;
    const int64_t rlo = seg_rows[s], rhi = seg_rows[s + 1];
    const int64_t first = rlo + (int64_t)blockIdx.x * kHistRowsPerBlock;
    if (first >= rhi) return;  // whole block
    for (int b = threadIdx.x; b < kBuckets; b += kHistThreads) h[b] = 0;
    __syncthreads();
    const int64_t last = min(first + kHistRowsPerBlock, rhi);
    for (int64_t r = first + wave_id(); r < last; r += kHistThreads / kWave) {
        const int64_t b0 = X.beg[r];
        const int l = X.len[r];
        for (int p = lane_id(); p < l; p += kWave)
            atomicAdd(&h[bucket_of(as_f64(X.val[b0 + p]))],
                      (uint32_t)sym_weight(lower.of(r), X.col[b0 + p], (int)r));
    }
    __syncthreads();
    for (int b = threadIdx.x; b < kBuckets; b += kHistThreads)
        if (h[b]) atomicAdd((unsigned long long *)&hist[(int64_t)s * kBuckets + b],
                            (unsigned long long)h[b]);
}

__device__ double bucket_hi(int b) {
    if (b <= 0) return ldexp(1.0, -127);
    const int E = (b - 1) / 16 - 127;
    const int j = (b - 1) % 16;
    return ldexp(1.0 + (double)(j + 1) / 16.0, E);
}

// One workgroup per segment: the bucket terms count_b * hi_b^2 are formed in
// parallel into LDS (each the same FP64 operations as a sequential pass), then
// one thread adds them in ascending order, uncontracted, and stops at the cut.
constexpr int kSelectThreads = 256;
__global__ __launch_bounds__(kSelectThreads) void k_select(const uint64_t *hist,
                                                           const double *tau, int nseg,
                                                           int *bstar) {
#pragma clang fp contract(off)
    constexpr int kBatch = 32;
    constexpr int kPadded = (kBucketTop + kBatch - 1) / kBatch * kBatch;
    __shared__ double add[kPadded];
    const int s = blockIdx.x;
    if (s >= nseg) return;
    const uint64_t *c = hist + (int64_t)s * kBuckets;
    // zero terms past the top bucket: adding 0 never crosses the budget
    for (int b = threadIdx.x; b < kPadded; b += kSelectThreads) {
        const double h = b < kBucketTop ? bucket_hi(b) : 0.0;
        const double hh = h * h;
        add[b] = b < kBucketTop ? (double)c[b] * hh : 0.0;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    // Ascending walk: the cut is the first bucket whose term takes the running
    // sum past tau^2.  Terms are read in register batches; within a batch the
    // running sums are formed first and compared afterwards: up to the first
    // crossing they are the plain walk's sums, in its order, and the sums
    // formed past it are discarded.  Only the additions sit on the dependent
    // chain.
    const double t2 = tau[s] * tau[s];
    double acc = 0.0;
    int b = kBucketTop;
    for (int base = 0; base < kPadded; base += kBatch) {
        double t[kBatch], ps[kBatch];
#pragma unroll
        for (int q = 0; q < kBatch; ++q) t[q] = add[base + q];
        double a = acc;
#pragma unroll
        for (int q = 0; q < kBatch; ++q) {
            a = a + t[q];
            ps[q] = a;
        }
        int hit = kBatch;
#pragma unroll
        for (int q = kBatch - 1; q >= 0; --q)
            if (ps[q] > t2) hit = q;
        if (hit < kBatch) {
            b = base + hit;
            break;
        }
        acc = a;
    }
    bstar[s] = b < kBucketTop ? b : kBucketTop;
}

template <typename V>
__global__ void k_count_keep(MatView<V> X, const int32_t *row_seg, const int *bstar,
                             int32_t *cnt, double *sq_keep, double *sq_drop, LowerRows lower) {
    const int64_t i = (int64_t)blockIdx.x * (blockDim.x / kWave) + wave_id();
    if (i >= X.n) return;
    const int b = bstar[row_seg ? row_seg[i] : 0];
    const int64_t b0 = X.beg[i];
    const int l = X.len[i];
    int k = 0;
    double sk = 0.0, sd = 0.0;
    for (int p = lane_id(); p < l; p += kWave) {
        const double v = as_f64(X.val[b0 + p]);
        const double wv = sym_weight(lower.of(i), X.col[b0 + p], (int)i) * v * v;
        if (v != 0.0 && bucket_of(v) >= b) { ++k; sk += wv; }
        else sd += wv;
    }
    k = wave_sum(k);
    sk = wave_sum(sk);
    sd = wave_sum(sd);
    if (lane_id() == 0) {
        cnt[i] = k;
        if (sq_keep) sq_keep[i] = sk;
        if (sq_drop) sq_drop[i] = sd;
    }
}

template <typename V, typename Vo>
__global__ void k_scatter_keep(MatView<V> X, const int32_t *row_seg, const int *bstar,
                               const int64_t *dst_ptr, int32_t *dcol, Vo *dval) {
    const int64_t i = (int64_t)blockIdx.x * (blockDim.x / kWave) + wave_id();
    if (i >= X.n) return;
    const int b = bstar[row_seg ? row_seg[i] : 0];
    const int64_t b0 = X.beg[i];
    const int l = X.len[i];
    int64_t o = dst_ptr[i];
    for (int p0 = 0; p0 < l; p0 += kWave) {
        const int p = p0 + lane_id();
        double v = 0.0;
        int c = 0;
        if (p < l) { v = as_f64(X.val[b0 + p]); c = X.col[b0 + p]; }
        const bool keep = p < l && v != 0.0 && bucket_of(v) >= b;
        const uint64_t m = __ballot(keep);
        if (keep) {
            const int64_t w = o + lanes_below(m);
            dcol[w] = c;
            dval[w] = (Vo)v;
        }
        o += __popcll(m);
    }
}

// ---------------------------------------------------------------------------
// misc
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_fill(T *p, int64_t n, T v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_row_segments(const int64_t *seg_rows, int32_t *row_seg) {
    const int s = blockIdx.y;
    const int64_t r = seg_rows[s] + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r < seg_rows[s + 1]) row_seg[r] = s;
}

// ---------------------------------------------------------------------------
// identity, column norms, transpose (filtered Newton: inverse start)
// ---------------------------------------------------------------------------
__global__ void k_identity(int64_t n, int64_t *beg, int32_t *len, int32_t *col, double *val) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n) return;
    beg[i] = i;
    if (i == n) return;
    len[i] = 1;
    col[i] = (int32_t)i;
    val[i] = 1.0;
}

template <typename V>
__global__ void k_col_abs_sum(MatView<V> X, double *colsum) {
    const int64_t i = (int64_t)blockIdx.x * (blockDim.x / kWave) + wave_id();
    if (i >= X.n) return;
    const int64_t b = X.beg[i];
    for (int p = lane_id(); p < X.len[i]; p += kWave)
        atomicAdd(&colsum[X.col[b + p]], fabs(as_f64(X.val[b + p])));
}

template <typename V>
__global__ void k_transpose_count(MatView<V> X, int32_t *cnt) {
    const int64_t i = (int64_t)blockIdx.x * (blockDim.x / kWave) + wave_id();
    if (i >= X.n) return;
    const int64_t b = X.beg[i];
    for (int p = lane_id(); p < X.len[i]; p += kWave) atomicAdd(&cnt[X.col[b + p]], 1);
}

template <typename V>
__global__ void k_transpose_fill(MatView<V> X, const int64_t *tp, int32_t *fill, int32_t *tcol,
                                 V *tval) {
    const int64_t i = (int64_t)blockIdx.x * (blockDim.x / kWave) + wave_id();
    if (i >= X.n) return;
    const int64_t b = X.beg[i];
    for (int p = lane_id(); p < X.len[i]; p += kWave) {
        const int j = X.col[b + p];
        const int64_t w = tp[j] + atomicAdd(&fill[j], 1);
        tcol[w] = (int32_t)i;
        tval[w] = X.val[b + p];
    }
}

// ---------------------------------------------------------------------------
// symmetric products: the full matrix from its lower triangle L
// ---------------------------------------------------------------------------
// cnt[c] += number of entries L(j, c) with j > c over the lower rows j (wave per row j)
template <typename V>
__global__ void k_sym_count(MatView<V> L, LowerRows lower, int32_t *cnt) {
    const int64_t j = (int64_t)blockIdx.x * (blockDim.x / kWave) + wave_id();
    if (j >= L.n || !lower.of(j)) return;
    const int64_t b = L.beg[j];
    for (int p = lane_id(); p < L.len[j]; p += kWave) {
        const int c = L.col[b + p];
        if (c < j) atomicAdd(&cnt[c], 1);
    }
}

// out[i] = a[i] + b[i]
__global__ void k_add_len(const int32_t *a, const int32_t *b, int64_t n, int32_t *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = a[i] + b[i];
}

// Row j of L goes to the front of row j of C; for a lower row j, every
// strictly-lower entry L(j, c) is also appended, unordered, to row c's mirror
// list in (tcol, tval) at toff[c] + (arrival order).  Wave per row j.
template <typename V>
__global__ void k_sym_place(MatView<V> L, LowerRows lower, const int64_t *cbeg, int32_t *ccol,
                            V *cval, const int64_t *toff, int32_t *fill, int32_t *tcol, V *tval) {
    // consecutive rows on one XCD: the mirror entries they append to a row c
    // are then neighbours in that XCD's L2 and leave it as whole lines
    const int64_t j = (int64_t)xcd_row(blockIdx.x, gridDim.x) * (blockDim.x / kWave) + wave_id();
    if (j >= L.n) return;
    const bool low = lower.of(j);
    const int64_t b = L.beg[j], o = cbeg[j];
    for (int p = lane_id(); p < L.len[j]; p += kWave) {
        const int c = L.col[b + p];
        const V v = L.val[b + p];
        ccol[o + p] = c;
        cval[o + p] = v;
        if (low && c < j) {
            const int64_t w = toff[c] + atomicAdd(&fill[c], 1);
            tcol[w] = (int32_t)j;
            tval[w] = v;
        }
    }
}

// Row c of C gets its list of tcnt[c] unordered (key, value) pairs, ordered by
// key, after its first llen[c] entries (none when llen is null): the keys are
// ranked with an LDS bitmap over chunks of kRankChunk consecutive keys from the
// smallest (rank = set bits below the key), so no comparison sort is needed
// and any list length is handled.  Keys of a row are distinct.  One workgroup
// per row.  (The mirror of a lower triangle: keys j > c; a transpose: any.)
constexpr int kRankChunk = 65536;
constexpr int kRankThreads = 256;

template <typename V>
__global__ __launch_bounds__(kRankThreads) void k_sym_rank(
    const int64_t *cbeg, const int32_t *llen, const int64_t *toff, const int32_t *tcnt,
    const int32_t *tcol, const V *tval, int32_t *ccol, V *cval) {
    constexpr int NWORD = kRankChunk / 32;
    constexpr int PER = NWORD / kRankThreads;
    __shared__ uint32_t bits[NWORD];
    __shared__ int32_t wpre[NWORD];
    __shared__ int red[kRankThreads / kWave];
    __shared__ int wtot[kRankThreads / kWave];
    const int c = blockIdx.x;
    const int m = tcnt[c];
    if (m == 0) return;
    const int64_t tb = toff[c];
    const int64_t ob = cbeg[c] + (llen ? llen[c] : 0);
    const int lane = lane_id(), wave = wave_id();
    // smallest and largest key, to bound the chunks
    int kmin = INT_MAX, kmax = INT_MIN;
    for (int q = threadIdx.x; q < m; q += kRankThreads) {
        const int key = tcol[tb + q];
        kmin = min(kmin, key);
        kmax = max(kmax, key);
    }
    kmin = wave_min(kmin);
    kmax = wave_max(kmax);
    if (lane == 0) { red[wave] = kmin; wtot[wave] = kmax; }
    __syncthreads();
    for (int w = 0; w < kRankThreads / kWave; ++w) {
        kmin = min(kmin, red[w]);
        kmax = max(kmax, wtot[w]);
    }
    __syncthreads();  // red and wtot are reused below
    int done = 0;  // keys ranked in earlier chunks
    for (int64_t k0 = kmin; k0 <= kmax; k0 += kRankChunk) {
        // words that can hold a key of this chunk; the others are neither
        // cleared nor counted
        const int64_t span = ((kmax - k0) >> 5) + 1;
        const int nw = span < NWORD ? (int)span : NWORD;
        for (int q = threadIdx.x; q < nw; q += kRankThreads) bits[q] = 0u;
        __syncthreads();
        for (int q = threadIdx.x; q < m; q += kRankThreads) {
            const int64_t d = (int64_t)tcol[tb + q] - k0;
            if (d >= 0 && d < kRankChunk) atomicOr(&bits[d >> 5], 1u << (d & 31));
        }
        __syncthreads();
        // exclusive prefix of popcounts over the words (PER consecutive words per thread)
        int loc = 0;
        for (int u = 0; u < PER; ++u) {
            const int q = threadIdx.x * PER + u;
            if (q < nw) loc += __popc(bits[q]);
        }
        const int inc = (int)wave_incl_scan((int64_t)loc);
        if (lane == kWave - 1) wtot[wave] = inc;
        __syncthreads();
        int before = inc - loc, total = 0;
        for (int w = 0; w < kRankThreads / kWave; ++w) {
            if (w < wave) before += wtot[w];
            total += wtot[w];
        }
        for (int u = 0; u < PER; ++u) {
            const int q = threadIdx.x * PER + u;
            if (q < nw) {
                wpre[q] = before;
                before += __popc(bits[q]);
            }
        }
        __syncthreads();
        for (int q = threadIdx.x; q < m; q += kRankThreads) {
            const int key = tcol[tb + q];
            const int64_t d = (int64_t)key - k0;
            if (d >= 0 && d < kRankChunk) {
                const int wd = (int)(d >> 5);
                const int r = done + wpre[wd] + __popc(bits[wd] & ((1u << (d & 31)) - 1u));
                ccol[ob + r] = key;
                cval[ob + r] = tval[tb + q];
            }
        }
        done += total;
        __syncthreads();
    }
}

// flag |= 1 if some entry (i, j, v) has no entry (j, i) of the same value
// (wave per row, binary search in the sorted row j)
template <typename V>
__global__ void k_sym_check(MatView<V> X, int *flag) {
    const int64_t i = (int64_t)blockIdx.x * (blockDim.x / kWave) + wave_id();
    if (i >= X.n) return;
    const int64_t b = X.beg[i];
    int bad = 0;
    for (int p = lane_id(); p < X.len[i]; p += kWave) {
        const int j = X.col[b + p];
        const int64_t bj = X.beg[j];
        int lo = 0, hi = X.len[j];
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (X.col[bj + mid] < i) lo = mid + 1;
            else hi = mid;
        }
        if (!(lo < X.len[j] && X.col[bj + lo] == i && X.val[bj + lo] == X.val[b + p])) bad = 1;
    }
    if (__ballot(bad) && lane_id() == 0) atomicOr(flag, 1);
}

// diag[i] = X_ii (0 if absent), wave per row, binary search in the sorted row
template <typename V>
__global__ void k_diag(MatView<V> X, double *diag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= X.n) return;
    const int64_t b = X.beg[i];
    int lo = 0, hi = X.len[i];
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (X.col[b + mid] < i) lo = mid + 1;
        else hi = mid;
    }
    diag[i] = (lo < X.len[i] && X.col[b + lo] == i) ? as_f64(X.val[b + lo]) : 0.0;
}

inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

template <typename V>
void launch_diag(MatView<V> X, double *diag, hipStream_t s) {
    if (X.n > 0) k_diag<V><<<blocks_for(X.n, 256), 256, 0, s>>>(X, diag);
}
template void launch_diag<double>(MatView<double>, double *, hipStream_t);
template void launch_diag<float>(MatView<float>, double *, hipStream_t);

void launch_identity(int64_t n, int64_t *beg, int32_t *len, int32_t *col, double *val,
                     hipStream_t s) {
    k_identity<<<blocks_for(n + 1, 256), 256, 0, s>>>(n, beg, len, col, val);
}

template <typename V>
void launch_col_abs_sum(MatView<V> X, double *colsum, hipStream_t s) {
    if (X.n > 0) k_col_abs_sum<V><<<blocks_for(X.n, 4), 256, 0, s>>>(X, colsum);
}
template void launch_col_abs_sum<double>(MatView<double>, double *, hipStream_t);

template <typename V>
void launch_transpose_count(MatView<V> X, int32_t *cnt, hipStream_t s) {
    if (X.n > 0) k_transpose_count<V><<<blocks_for(X.n, 4), 256, 0, s>>>(X, cnt);
}
template <typename V>
void launch_transpose_fill(MatView<V> X, const int64_t *tp, int32_t *fill, int32_t *tcol, V *tval,
                           hipStream_t s) {
    if (X.n > 0) k_transpose_fill<V><<<blocks_for(X.n, 4), 256, 0, s>>>(X, tp, fill, tcol, tval);
}
template void launch_transpose_count<double>(MatView<double>, int32_t *, hipStream_t);
template void launch_transpose_fill<double>(MatView<double>, const int64_t *, int32_t *, int32_t *,
                                            double *, hipStream_t);
template <typename V>
void launch_sym_count(MatView<V> L, LowerRows lower, int32_t *cnt, hipStream_t s) {
    if (L.n > 0) k_sym_count<V><<<blocks_for(L.n, 4), 256, 0, s>>>(L, lower, cnt);
}
void launch_add_len(const int32_t *a, const int32_t *b, int64_t n, int32_t *out, hipStream_t s) {
    if (n > 0) k_add_len<<<blocks_for(n, 256), 256, 0, s>>>(a, b, n, out);
}
template <typename V>
void launch_sym_place(MatView<V> L, LowerRows lower, const int64_t *cbeg, int32_t *ccol, V *cval,
                      const int64_t *toff, int32_t *fill, int32_t *tcol, V *tval, hipStream_t s) {
    if (L.n > 0)
        k_sym_place<V><<<blocks_for(L.n, 4), 256, 0, s>>>(L, lower, cbeg, ccol, cval, toff, fill,
                                                          tcol, tval);
}
template <typename V>
void launch_sym_rank(int64_t n, const int64_t *cbeg, const int32_t *llen, const int64_t *toff,
                     const int32_t *tcnt, const int32_t *tcol, const V *tval, int32_t *ccol,
                     V *cval, hipStream_t s) {
    if (n > 0)
        k_sym_rank<V><<<(unsigned)n, kRankThreads, 0, s>>>(cbeg, llen, toff, tcnt, tcol, tval,
                                                           ccol, cval);
}
template <typename V>
void launch_sym_check(MatView<V> X, int *flag, hipStream_t s) {
    if (X.n > 0) k_sym_check<V><<<blocks_for(X.n, 4), 256, 0, s>>>(X, flag);
}
#define SFN_SYM_INST(V)                                                                        \
    template void launch_sym_count<V>(MatView<V>, LowerRows, int32_t *, hipStream_t);          \
    template void launch_sym_place<V>(MatView<V>, LowerRows, const int64_t *, int32_t *, V *,  \
                                      const int64_t *, int32_t *, int32_t *, V *, hipStream_t); \
    template void launch_sym_rank<V>(int64_t, const int64_t *, const int32_t *,                \
                                     const int64_t *, const int32_t *, const int32_t *,        \
                                     const V *, int32_t *, V *, hipStream_t);                  \
    template void launch_sym_check<V>(MatView<V>, int *, hipStream_t);
SFN_SYM_INST(double)
SFN_SYM_INST(float)
#undef SFN_SYM_INST

// ===========================================================================
// launchers
// ===========================================================================
void launch_validate(const int64_t *rp, const int32_t *ci, const void *val, int f32, int64_t n,
                     int64_t nnz, int *flag, hipStream_t s) {
    k_validate<<<blocks_for(n, 256), 256, 0, s>>>(rp, ci, val, f32, n, nnz, flag);
}

void launch_row_abs_sum(const int64_t *rp, const void *val, int f32, int64_t n, double *out,
                        hipStream_t s) {
    k_row_abs_sum<<<blocks_for(n, 256), 256, 0, s>>>(rp, val, f32, n, out);
}

void launch_row_len(const int64_t *rp, int64_t n, int32_t *len, hipStream_t s) {
    k_row_len<<<blocks_for(n, 256), 256, 0, s>>>(rp, n, len);
}

template <typename Vi, typename Vo>
void launch_scale_copy(const Vi *src, Vo *dst, int64_t n, double scale, hipStream_t s) {
    if (n <= 0) return;
    k_scale_copy<Vi, Vo><<<blocks_for(n, 256), 256, 0, s>>>(src, dst, n, scale);
}
template void launch_scale_copy<double, double>(const double *, double *, int64_t, double, hipStream_t);
template void launch_scale_copy<double, float>(const double *, float *, int64_t, double, hipStream_t);
template void launch_scale_copy<float, double>(const float *, double *, int64_t, double, hipStream_t);
template void launch_scale_copy<float, float>(const float *, float *, int64_t, double, hipStream_t);

void launch_seg_sum(const double *x, const int64_t *seg, int nseg, double *out, hipStream_t s) {
    if (nseg > 0) k_seg_reduce<false><<<nseg, kRedThreads, 0, s>>>(x, seg, out);
}
void launch_seg_max(const double *x, const int64_t *seg, int nseg, double *out, hipStream_t s) {
    if (nseg > 0) k_seg_reduce<true><<<nseg, kRedThreads, 0, s>>>(x, seg, out);
}

int64_t scan_tmp_elems(int64_t n) { return (n + kScanChunk - 1) / kScanChunk + 2; }

template <typename T>
static void scan_impl(const T *in, int64_t n, int64_t *out, int64_t *tmp, int64_t init,
                      hipStream_t s) {
    const int64_t nb = (n + kScanChunk - 1) / kScanChunk;
    if (nb == 0) {
        k_fill<int64_t><<<1, 1, 0, s>>>(out, 1, init);
        return;
    }
    if (n <= kScanOneMax) {
        k_scan_one<T><<<1, kScanOneThreads, 0, s>>>(in, n, init, out);
        return;
    }
    k_scan_partial<T><<<(unsigned)nb, kScanThreads, 0, s>>>(in, n, tmp);
    k_scan_top<<<1, kScanThreads, 0, s>>>(tmp, nb);
    k_scan_final<T><<<(unsigned)nb, kScanThreads, 0, s>>>(in, n, tmp, nb, init, out);
}
void launch_exclusive_scan_i64(const int64_t *in, int64_t n, int64_t *out, int64_t *tmp,
                               int64_t init, hipStream_t s) {
    scan_impl<int64_t>(in, n, out, tmp, init, s);
}
void launch_exclusive_scan_i32(const int32_t *in, int64_t n, int64_t *out, int64_t *tmp,
                               int64_t init, hipStream_t s) {
    scan_impl<int32_t>(in, n, out, tmp, init, s);
}

template <typename V>
void launch_row_density(MatView<V> B, unsigned long long *out, hipStream_t s) {
    if (B.n <= 0) return;
    const int64_t nb = (B.n + kSpanThreads - 1) / kSpanThreads;
    k_row_density<V><<<(unsigned)nb, kSpanThreads, 0, s>>>(B, out);
}
template void launch_row_density<double>(MatView<double>, unsigned long long *, hipStream_t);
template void launch_row_density<float>(MatView<float>, unsigned long long *, hipStream_t);

template <typename V>
void launch_page_count(MatView<V> B, int shift, int32_t *len, hipStream_t s) {
    if (B.n <= 0) return;
    k_row_pages<V, false><<<blocks_for(B.n, 4), 256, 0, s>>>(B, shift, len, nullptr, nullptr);
}
template <typename V>
void launch_page_fill(MatView<V> B, int shift, const int64_t *beg, int32_t *pg, hipStream_t s) {
    if (B.n <= 0) return;
    k_row_pages<V, true><<<blocks_for(B.n, 4), 256, 0, s>>>(B, shift, nullptr, beg, pg);
}
template void launch_page_count<double>(MatView<double>, int, int32_t *, hipStream_t);
template void launch_page_count<float>(MatView<float>, int, int32_t *, hipStream_t);
template void launch_page_fill<double>(MatView<double>, int, const int64_t *, int32_t *,
                                       hipStream_t);
template void launch_page_fill<float>(MatView<float>, int, const int64_t *, int32_t *,
                                      hipStream_t);

template <typename V>
void launch_plan(MatView<V> A, MatView<V> B, MatView<V> D, int diag, int64_t r0, int64_t r1,
                 int32_t *lo, int32_t *span, int64_t *cap, int64_t *work, const uint8_t *skip,
                 hipStream_t s) {
    if (r1 <= r0) return;
    k_plan<V><<<blocks_for(r1 - r0, 4), 256, 0, s>>>(A, B, D, diag, r0, r1, lo, span, cap, work,
                                                     skip);
}
template void launch_plan<double>(MatView<double>, MatView<double>, MatView<double>, int, int64_t,
                                  int64_t, int32_t *, int32_t *, int64_t *, int64_t *,
                                  const uint8_t *, hipStream_t);
template void launch_plan<float>(MatView<float>, MatView<float>, MatView<float>, int, int64_t,
                                 int64_t, int32_t *, int32_t *, int64_t *, int64_t *,
                                 const uint8_t *, hipStream_t);

// ---- batch relayout for serving -------------------------------------------------
__global__ void k_move_len(const SegMove *t, int32_t *dst_len) {
    const SegMove m = t[blockIdx.y];
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r < m.nrows) dst_len[m.dst_row + r] = m.src.len[m.src_row + r];
}

__global__ void k_move_rows(const SegMove *t, const int64_t *dst_beg, int32_t *dst_col,
                            double *dst_val) {
    const SegMove m = t[blockIdx.y];
    const int64_t r = (int64_t)blockIdx.x * (blockDim.x / kWave) + wave_id();
    if (r >= m.nrows) return;
    const int64_t sb = m.src.beg[m.src_row + r], db = dst_beg[m.dst_row + r];
    const int l = m.src.len[m.src_row + r];
    for (int p = lane_id(); p < l; p += kWave) {
        dst_col[db + p] = (int32_t)(m.src.col[sb + p] + m.col_shift);
        dst_val[db + p] = m.src.val[sb + p];
    }
}

__global__ void k_fill_u8(uint8_t *p, int64_t lo, int64_t hi, uint8_t v) {
    const int64_t i = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < hi) p[i] = v;
}

void launch_move_len(const SegMove *t, int nseg, int64_t max_rows, int32_t *dst_len,
                     hipStream_t s) {
    if (nseg <= 0 || max_rows <= 0) return;
    k_move_len<<<dim3(blocks_for(max_rows, 256), nseg), 256, 0, s>>>(t, dst_len);
}
void launch_move_rows(const SegMove *t, int nseg, int64_t max_rows, const int64_t *dst_beg,
                      int32_t *dst_col, double *dst_val, hipStream_t s) {
    if (nseg <= 0 || max_rows <= 0) return;
    k_move_rows<<<dim3(blocks_for(max_rows, 4), nseg), 256, 0, s>>>(t, dst_beg, dst_col, dst_val);
}
// One thread gathers scalars scattered over device memory into one record
// (read back with a single copy); the bucket total of a histogram is summed by
// one workgroup.
__global__ void k_gather_scalars(ScalarGather g, int64_t *dst) {
    const int t = threadIdx.x;
    if (t == 0)
        for (int j = 0; j < g.n; ++j) dst[j] = *g.src[j];
    if (g.fold && t < kClasses * kSpreadCounters) {
        const int64_t *p = g.fold + (int64_t)t * kSpread * kSpreadStride;
        int64_t a = 0;
        for (int q = 0; q < kSpread; ++q) a += p[q * kSpreadStride];
        g.fold_dst[(t / kSpreadCounters) * 8 + 4 + t % kSpreadCounters] = a;
    }
}

__global__ __launch_bounds__(256) void k_hist_total(const uint64_t *hist, int64_t *dst) {
    __shared__ unsigned long long part[256 / kWave];
    unsigned long long t = 0;
    for (int b = threadIdx.x; b < kBuckets; b += 256) t += hist[b];
    t = wave_sum(t);
    if (lane_id() == 0) part[wave_id()] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long a = 0;
        for (int w = 0; w < 256 / kWave; ++w) a += part[w];
        *dst = (int64_t)a;
    }
}

__global__ void k_set_filter_args(int64_t *seg, int64_t n, double *tau_dev, double tau) {
    seg[0] = 0;
    seg[1] = n;
    *tau_dev = tau;
}

void launch_gather_scalars(const ScalarGather &g, int64_t *dst, hipStream_t s) {
    if (g.n > 0 || g.fold) k_gather_scalars<<<1, kWave, 0, s>>>(g, dst);
}

void launch_hist_total(const uint64_t *hist, int64_t *dst, hipStream_t s) {
    k_hist_total<<<1, 256, 0, s>>>(hist, dst);
}

void launch_set_filter_args(int64_t *seg, int64_t n, double *tau_dev, double tau, hipStream_t s) {
    k_set_filter_args<<<1, 1, 0, s>>>(seg, n, tau_dev, tau);
}

void launch_fill_u8(uint8_t *p, int64_t lo, int64_t hi, uint8_t v, hipStream_t s) {
    if (hi > lo) k_fill_u8<<<blocks_for(hi - lo, 256), 256, 0, s>>>(p, lo, hi, v);
}

void launch_bin_rows(const int32_t *span, const int64_t *work, int64_t r0, int64_t r1,
                     int small_tile, int mid_tile, int group, int32_t *bins, int64_t bin_stride,
                     int32_t *counts, int32_t *out_len, double *sq_prod, double *sq_out,
                     const int32_t *a_len, const int32_t *d_len, int64_t *cstat,
                     hipStream_t s) {
    if (r1 <= r0) return;
    k_bin_rows<<<blocks_for(r1 - r0, kBinThreads), kBinThreads, 0, s>>>(
        span, work, r0, r1, small_tile, mid_tile, group, bins, bin_stride, counts, out_len,
        sq_prod, sq_out, a_len, d_len, cstat);
}

BinCfg bin_config(int cls, int value_bytes) {
    (void)value_bytes;  // FP64 accumulators for both value types
    switch (cls) {
        case 1: return {512, 64};
        case 2: return {4096, 256};
        default: return {8192, 512};
    }
}

template <typename V>
void launch_merge_group(int group, const int32_t *leads, int ngroups, MatView<V> A, MatView<V> B,
                        int32_t *mk, uint32_t *mm, int32_t *mc, V *cv, int32_t *mlen,
                        int64_t *gathered, hipStream_t s) {
    if (ngroups <= 0) return;
    unsigned long long *g = (unsigned long long *)gathered;
    switch (group) {
        case 2:
            k_merge_group<V, 2><<<ngroups, kMergeThreads, 0, s>>>(leads, A, B, mk, mm, mc, cv,
                                                                   mlen, g);
            break;
        case 4:
            k_merge_group<V, 4><<<ngroups, kMergeThreads, 0, s>>>(leads, A, B, mk, mm, mc, cv,
                                                                   mlen, g);
            break;
        case 8:
            k_merge_group<V, 8><<<ngroups, kMergeThreads, 0, s>>>(leads, A, B, mk, mm, mc, cv,
                                                                   mlen, g);
            break;
        case 32:
            k_merge_group<V, 32><<<ngroups, kMergeThreads, 0, s>>>(leads, A, B, mk, mm, mc, cv,
                                                                    mlen, g);
            break;
        default:
            k_merge_group<V, 16><<<ngroups, kMergeThreads, 0, s>>>(leads, A, B, mk, mm, mc, cv,
                                                                    mlen, g);
            break;
    }
}
template void launch_merge_group<double>(int, const int32_t *, int, MatView<double>,
                                         MatView<double>, int32_t *, uint32_t *, int32_t *,
                                         double *, int32_t *, int64_t *, hipStream_t);
template void launch_merge_group<float>(int, const int32_t *, int, MatView<float>, MatView<float>,
                                        int32_t *, uint32_t *, int32_t *, float *, int32_t *,
                                        int64_t *, hipStream_t);

// LDS accumulators of a group kernel: 128 KB for groups of 4 and more (64 KB for
// pairs), split into `group` windows.
BinCfg group_config(int group, int value_bytes) {
    (void)value_bytes;  // FP64 accumulators for both value types
    if (group == 2) return {4096, 512};
    return {16384 / group, 1024};
}

template <typename V, int R>
static void group_launch(const int32_t *leads, int ngroups, const int32_t *mk, const uint32_t *mm,
                         const int32_t *mc, const V *cv, const int32_t *mlen, MatView<V> A,
                         MatView<V> B, MatView<V> D, double coef, double dcoef, double diag,
                         const int32_t *lo, const int32_t *span, int64_t base, const int64_t *off,
                         int32_t *out_col, V *out_val, int32_t *out_len, int32_t *cursor,
                         int32_t *cnext, double *sq_prod, double *sq_out, int64_t *out_count,
                         ProductEpi epi, hipStream_t s) {
    constexpr int T = R == 2 ? 4096 : 16384 / R;
    constexpr int NT = R == 2 ? 512 : 1024;
    if (epi.pages.pg)
        k_spgemm_rows<V, R, T, NT, kUnroll, true><<<ngroups, NT, 0, s>>>(
            leads, mk, mm, mc, cv, mlen, A, B, D, (V)coef, (V)dcoef, (V)diag, lo, span, off, base,
            out_col, out_val, out_len, cursor, cnext, sq_prod, sq_out, out_count, epi);
    else
        k_spgemm_rows<V, R, T, NT, kUnroll, false><<<ngroups, NT, 0, s>>>(
            leads, mk, mm, mc, cv, mlen, A, B, D, (V)coef, (V)dcoef, (V)diag, lo, span, off, base,
            out_col, out_val, out_len, cursor, cnext, sq_prod, sq_out, out_count, epi);
}

template <typename V>
void launch_spgemm_group(int group, const int32_t *leads, int ngroups, const int32_t *mk,
                         const uint32_t *mm, const int32_t *mc, const V *cv, const int32_t *mlen,
                         MatView<V> A, MatView<V> B, MatView<V> D, double coef, double dcoef,
                         double diag, const int32_t *lo, const int32_t *span, int64_t base,
                         const int64_t *off, int32_t *out_col, V *out_val, int32_t *out_len,
                         int32_t *cursor, int32_t *cnext, double *sq_prod, double *sq_out,
                         int64_t *out_count, ProductEpi epi, hipStream_t s) {
    if (ngroups <= 0) return;
#define SFN_GROUP_ARGS                                                                        \
    leads, ngroups, mk, mm, mc, cv, mlen, A, B, D, coef, dcoef, diag, lo, span, base, off,    \
        out_col, out_val, out_len, cursor, cnext, sq_prod, sq_out, out_count, epi, s
    switch (group) {
        case 2: group_launch<V, 2>(SFN_GROUP_ARGS); break;
        case 4: group_launch<V, 4>(SFN_GROUP_ARGS); break;
        case 8: group_launch<V, 8>(SFN_GROUP_ARGS); break;
        default: group_launch<V, 16>(SFN_GROUP_ARGS); break;
    }
#undef SFN_GROUP_ARGS
}
template void launch_spgemm_group<double>(int, const int32_t *, int, const int32_t *,
                                          const uint32_t *, const int32_t *, const double *,
                                          const int32_t *, MatView<double>, MatView<double>,
                                          MatView<double>, double, double, double,
                                          const int32_t *, const int32_t *, int64_t,
                                          const int64_t *, int32_t *, double *, int32_t *,
                                          int32_t *, int32_t *, double *, double *, int64_t *,
                                          ProductEpi, hipStream_t);
template void launch_spgemm_group<float>(int, const int32_t *, int, const int32_t *,
                                         const uint32_t *, const int32_t *, const float *,
                                         const int32_t *, MatView<float>, MatView<float>,
                                         MatView<float>, double, double, double, const int32_t *,
                                         const int32_t *, int64_t, const int64_t *, int32_t *,
                                         float *, int32_t *, int32_t *, int32_t *, double *,
                                         double *, int64_t *, ProductEpi, hipStream_t);

template <typename V, int R, int NB>
static void regtile_launch(const int32_t *leads, int ngroups, const int32_t *mk, const uint32_t *mm,
                           const int32_t *mc, const V *cv, const int32_t *mlen, MatView<V> A,
                           MatView<V> B, MatView<V> D, double coef, double dcoef, double diag,
                           const int32_t *lo, const int32_t *span, int64_t base,
                           const int64_t *off, int32_t *out_col, V *out_val, int32_t *out_len,
                           int32_t *cursor, int32_t *cnext, double *sq_prod, double *sq_out,
                           int64_t *out_count, ProductEpi epi, hipStream_t s) {
    k_spgemm_regtile<V, R, NB, kRegTileThreads><<<ngroups, kRegTileThreads, 0, s>>>(
        leads, mk, mm, mc, cv, mlen, A, B, D, (V)coef, (V)dcoef, (V)diag, lo, span, off, base,
        out_col, out_val, out_len, cursor, cnext, sq_prod, sq_out, out_count, epi);
}

bool regtile_supported(int group, int nb) {
    return (group == 8 && (nb == 4 || nb == 8)) || (group == 16 && (nb == 2 || nb == 4)) ||
           (group == 32 && nb == 2);
}

template <typename V>
void launch_spgemm_regtile(int group, int nb, const int32_t *leads, int ngroups,
                           const int32_t *mk, const uint32_t *mm, const int32_t *mc, const V *cv,
                           const int32_t *mlen, MatView<V> A, MatView<V> B, MatView<V> D,
                           double coef, double dcoef, double diag, const int32_t *lo,
                           const int32_t *span, int64_t base, const int64_t *off,
                           int32_t *out_col, V *out_val, int32_t *out_len, int32_t *cursor,
                           int32_t *cnext, double *sq_prod, double *sq_out, int64_t *out_count,
                           ProductEpi epi, hipStream_t s) {
    if (ngroups <= 0) return;
#define SFN_RT_ARGS                                                                           \
    leads, ngroups, mk, mm, mc, cv, mlen, A, B, D, coef, dcoef, diag, lo, span, base, off,    \
        out_col, out_val, out_len, cursor, cnext, sq_prod, sq_out, out_count, epi, s
    if (group == 8 && nb == 8) regtile_launch<V, 8, 8>(SFN_RT_ARGS);
    else if (group == 8) regtile_launch<V, 8, 4>(SFN_RT_ARGS);
    else if (group == 16 && nb == 2) regtile_launch<V, 16, 2>(SFN_RT_ARGS);
    else if (group == 16) regtile_launch<V, 16, 4>(SFN_RT_ARGS);
    else regtile_launch<V, 32, 2>(SFN_RT_ARGS);
#undef SFN_RT_ARGS
}
template void launch_spgemm_regtile<double>(int, int, const int32_t *, int, const int32_t *,
                                            const uint32_t *, const int32_t *, const double *,
                                            const int32_t *, MatView<double>, MatView<double>,
                                            MatView<double>, double, double, double,
                                            const int32_t *, const int32_t *, int64_t,
                                            const int64_t *, int32_t *, double *, int32_t *,
                                            int32_t *, int32_t *, double *, double *, int64_t *,
                                            ProductEpi, hipStream_t);
template void launch_spgemm_regtile<float>(int, int, const int32_t *, int, const int32_t *,
                                           const uint32_t *, const int32_t *, const float *,
                                           const int32_t *, MatView<float>, MatView<float>,
                                           MatView<float>, double, double, double,
                                           const int32_t *, const int32_t *, int64_t,
                                           const int64_t *, int32_t *, float *, int32_t *,
                                           int32_t *, int32_t *, double *, double *, int64_t *,
                                           ProductEpi, hipStream_t);

template <typename V>
void launch_spgemm(int cls, const int32_t *rows, int nrows, MatView<V> A, MatView<V> B,
                   MatView<V> D, double coef, double dcoef, double diag, const int32_t *lo,
                   const int32_t *span, int64_t base, const int64_t *off, int32_t *out_col,
                   V *out_val, int32_t *out_len, int32_t *cursor, int32_t *cnext, double *sq_prod,
                   double *sq_out, int64_t *out_count, ProductEpi epi, hipStream_t s) {
    if (nrows <= 0) return;
    const V c = (V)coef, d = (V)diag, dc = (V)dcoef;
#define SFN_ROW_ARGS                                                                          \
    rows, nullptr, nullptr, nullptr, nullptr, nullptr, A, B, D, c, dc, d, lo, span, off, base, \
        out_col, out_val, out_len, cursor, cnext, sq_prod, sq_out, out_count, epi
    switch (cls) {
        case 1:
            k_spgemm_rows<V, 1, 512, 64, kUnroll, false><<<nrows, 64, 0, s>>>(SFN_ROW_ARGS);
            break;
        case 2:
            k_spgemm_rows<V, 1, 4096, 256, kUnroll, false><<<nrows, 256, 0, s>>>(SFN_ROW_ARGS);
            break;
        default:
            k_spgemm_rows<V, 1, 8192, 512, kUnroll, false><<<nrows, 512, 0, s>>>(SFN_ROW_ARGS);
            break;
    }
#undef SFN_ROW_ARGS
}
template void launch_spgemm<double>(int, const int32_t *, int, MatView<double>, MatView<double>,
                                    MatView<double>, double, double, double, const int32_t *,
                                    const int32_t *, int64_t, const int64_t *, int32_t *, double *,
                                    int32_t *, int32_t *, int32_t *, double *, double *, int64_t *,
                                    ProductEpi, hipStream_t);
template void launch_spgemm<float>(int, const int32_t *, int, MatView<float>, MatView<float>,
                                   MatView<float>, double, double, double, const int32_t *,
                                   const int32_t *, int64_t, const int64_t *, int32_t *, float *,
                                   int32_t *, int32_t *, int32_t *, double *, double *, int64_t *,
                                   ProductEpi, hipStream_t);

template <typename V>
void launch_copy_rows(const int64_t *src_off, int64_t src_base, const int32_t *len,
                      const int32_t *scol, const V *sval, int64_t r0, int64_t r1,
                      const int64_t *dst_ptr, int32_t *dcol, V *dval, hipStream_t s) {
    if (r1 <= r0) return;
    k_copy_rows<V><<<blocks_for(r1 - r0, 4), 256, 0, s>>>(src_off, src_base, len, scol, sval, r0,
                                                         r1, dst_ptr, dcol, dval);
}
template void launch_copy_rows<double>(const int64_t *, int64_t, const int32_t *, const int32_t *,
                                       const double *, int64_t, int64_t, const int64_t *,
                                       int32_t *, double *, hipStream_t);
template void launch_copy_rows<float>(const int64_t *, int64_t, const int32_t *, const int32_t *,
                                      const float *, int64_t, int64_t, const int64_t *, int32_t *,
                                      float *, hipStream_t);

template <typename V>
void launch_histogram(MatView<V> X, const int64_t *seg_rows, int nseg, int64_t max_seg_rows,
                      uint64_t *hist, LowerRows lower, hipStream_t s) {
    if (nseg <= 0 || max_seg_rows <= 0) return;
    dim3 grid(blocks_for(max_seg_rows, kHistRowsPerBlock), nseg);
    k_histogram<V><<<grid, kHistThreads, 0, s>>>(X, seg_rows, hist, lower);
}
template void launch_histogram<double>(MatView<double>, const int64_t *, int, int64_t, uint64_t *,
                                       LowerRows, hipStream_t);
template void launch_histogram<float>(MatView<float>, const int64_t *, int, int64_t, uint64_t *,
                                      LowerRows, hipStream_t);

void launch_select(const uint64_t *hist, const double *tau, int nseg, int *bstar, hipStream_t s) {
    if (nseg > 0) k_select<<<nseg, kSelectThreads, 0, s>>>(hist, tau, nseg, bstar);
}

template <typename V>
void launch_count_keep(MatView<V> X, const int32_t *row_seg, const int *bstar, int32_t *cnt,
                       double *sq_keep, double *sq_drop, LowerRows lower, hipStream_t s) {
    if (X.n <= 0) return;
    k_count_keep<V><<<blocks_for(X.n, 4), 256, 0, s>>>(X, row_seg, bstar, cnt, sq_keep, sq_drop,
                                                       lower);
}
template void launch_count_keep<double>(MatView<double>, const int32_t *, const int *, int32_t *,
                                        double *, double *, LowerRows, hipStream_t);
template void launch_count_keep<float>(MatView<float>, const int32_t *, const int *, int32_t *,
                                       double *, double *, LowerRows, hipStream_t);

template <typename V, typename Vo>
void launch_scatter_keep(MatView<V> X, const int32_t *row_seg, const int *bstar,
                         const int64_t *dst_ptr, int32_t *dcol, Vo *dval, hipStream_t s) {
    if (X.n <= 0) return;
    k_scatter_keep<V, Vo><<<blocks_for(X.n, 4), 256, 0, s>>>(X, row_seg, bstar, dst_ptr, dcol,
                                                             dval);
}
template void launch_scatter_keep<double, double>(MatView<double>, const int32_t *, const int *,
                                                  const int64_t *, int32_t *, double *,
                                                  hipStream_t);
template void launch_scatter_keep<float, float>(MatView<float>, const int32_t *, const int *,
                                                const int64_t *, int32_t *, float *, hipStream_t);
template void launch_scatter_keep<float, double>(MatView<float>, const int32_t *, const int *,
                                                 const int64_t *, int32_t *, double *,
                                                 hipStream_t);
template void launch_scatter_keep<double, float>(MatView<double>, const int32_t *, const int *,
                                                 const int64_t *, int32_t *, float *, hipStream_t);

void launch_row_segments(const int64_t *seg_rows, int nseg, int64_t max_seg_rows, int32_t *row_seg,
                         hipStream_t s) {
    if (nseg <= 0 || max_seg_rows <= 0) return;
    dim3 grid(blocks_for(max_seg_rows, 256), nseg);
    k_row_segments<<<grid, 256, 0, s>>>(seg_rows, row_seg);
}

}  // namespace sfn
