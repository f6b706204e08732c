// Host drivers: sparse product with batching, filtering, Algorithm 3.2.1 loop.
#include "driver.hpp"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>

namespace sfn {

// Row classes of the numeric product (kernel tiles in kernels.hip).
constexpr int kSmallTile = 512;
constexpr int kMidTile = 4096;

Workspace::Workspace(Allocator *a, size_t staging_bytes) : al(a), s(a->stream) {
    for (DevBuf *b : {&lo, &span, &cap, &work, &capoff, &workoff, &tmp, &bins, &counts, &cursor,
                      &stage_col, &stage_val, &rs1, &rs2, &rs3, &rs4, &icnt, &hist, &tau,
                      &bstar, &seg, &red, &flag, &zero_b, &cstat, &mk, &mm, &mc, &cv, &mlen, &cnext, &symcnt, &symoff, &symfill,
                      &symtcol, &symtval, &rs5, &whole, &sums, &pst, &rb, &plen, &pbeg, &plist})
        b->bind(a);
    // rows per workgroup for wide rows: 1 (off), 2, 4, 8 or 16
    if (const char *ge = std::getenv("SIGNFN_ROW_GROUP")) {
        const int g = std::atoi(ge);
        if (g == 1 || g == 2 || g == 4 || g == 8 || g == 16) {
            row_group = g;
            auto_group = false;
        }
    }
    if (const char *se = std::getenv("SIGNFN_SYMMETRIC")) allow_sym = se[0] != '0';
    // SIGNFN_REGTILE: "off" (default), "auto", or "<rows>x<nb>" to use the
    // register-accumulator product for every product it supports
    if (const char *re = std::getenv("SIGNFN_REGTILE")) {
        int g = 0, b = 0;
        if (std::strcmp(re, "off") == 0 || std::strcmp(re, "0") == 0) {
            rt_mode = 0;
        } else if (std::strcmp(re, "auto") == 0) {
            rt_mode = 1;
        } else if (std::sscanf(re, "%dx%d", &g, &b) == 2 && regtile_supported(g, b)) {
            rt_mode = 2;
            rt_group = g;
            rt_nb = b;
        }
    }
    if (const char *pe = std::getenv("SIGNFN_PROGRESS")) progress = pe[0] == '1';
    // SIGNFN_PAGES: "off" dense windows for every row group, "auto" (default)
    // page windows by the per-product rule, "on" page windows for every group
    if (const char *pg = std::getenv("SIGNFN_PAGES")) {
        if (std::strcmp(pg, "off") == 0 || std::strcmp(pg, "0") == 0) page_mode = 0;
        else if (std::strcmp(pg, "on") == 0) page_mode = 2;
        else page_mode = 1;
    }
    if (const char *rt = std::getenv("SIGNFN_RESIDUAL_TWO_PASS")) residual_two_pass = rt[0] == '1';
    if (const char *ps = std::getenv("SIGNFN_PAGE_SHIFT")) {
        const int v = std::atoi(ps);
        if (v >= 4 && v <= 8) page_shift = v;
    }
    // SIGNFN_STAGING_BYTES: staging budget of every product when the call sets none
    if (staging_bytes == 0)
        if (const char *sb = std::getenv("SIGNFN_STAGING_BYTES"))
            staging_bytes = (size_t)std::strtoull(sb, nullptr, 10);
    staging_auto = staging_bytes == 0;
    staging_limit = staging_auto ? auto_staging() : staging_bytes;
    for (auto &e : ev) SFN_HIP(hipEventCreate(&e));
}

// A quarter of the memory that is free, idle in the caching pool or held by
// the staging buffers themselves, capped so that one reservation stays a
// modest share of HBM.
size_t Workspace::auto_staging() const {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
        (void)hipGetLastError();
        fr = size_t(8) << 30;
    }
    const size_t avail = fr + (al->alloc ? 0 : Pool::instance().cached_bytes()) +
                         stage_col.size() + stage_val.size();
    return std::min<size_t>(size_t(24) << 30, std::max<size_t>(size_t(256) << 20, avail / 4));
}

Workspace::~Workspace() {
    (void)hipStreamSynchronize(s);
    for (auto &e : ev)
        if (e) (void)hipEventDestroy(e);
}

void Workspace::hot_stats(sign_stats &st) const {
    // the launch configuration with the most device time: a row class 1..3,
    // or row groups of 2^g rows
    int hv = 0, h = 1, hg = -1;
    const ClassStat *best = &cls[0][1];
    for (int v = 0; v < 2; ++v) {
        for (int c = 1; c < 4; ++c)
            if (cls[v][c].ms > best->ms) { best = &cls[v][c]; hv = v; h = c; hg = -1; }
        for (int g = 0; g < 5; ++g)
            if (grp[v][g].ms > best->ms) { best = &grp[v][g]; hv = v; h = 4; hg = g; }
    }
    bool hrt = false;
    for (int v = 0; v < 2; ++v)
        if (rt[v].ms > best->ms) { best = &rt[v]; hv = v; hrt = true; }
    const ClassStat &c = *best;
    int group = hg >= 0 ? 1 << hg : 1;
    BinCfg cfg = h == 4 ? group_config(group, hv ? 4 : 8) : bin_config(h, hv ? 4 : 8);
    if (hrt) {
        group = rt_used_group;
        cfg = BinCfg{64 * rt_used_nb, kRegTileThreadsHost};
    }
    st.hot_tile = cfg.tile;
    st.hot_threads = cfg.threads;
    st.hot_fp32 = hv;
    st.hot_group = group;
    st.hot_regtile = hrt ? 1 : 0;
    st.hot_launches = c.launches;
    st.hot_ms = c.ms;
    st.hot_bytes = c.bytes;
    st.hot_products = c.products;
    st.hot_gathered = c.gathered;
    st.hot_madds = c.madds;
    st.hot_pages = 2 * c.page_launches > c.launches ? 1 : 0;
}

int64_t *Workspace::pinned() {
    // one small page-locked block per host thread, kept for the thread's life:
    // read-backs land in it without a staging copy
    thread_local int64_t *p = nullptr;
    thread_local int64_t fallback[64];
    if (!p) {
        void *q = nullptr;
        if (hipHostMalloc(&q, sizeof(int64_t) * 64, hipHostMallocDefault) == hipSuccess && q)
            p = static_cast<int64_t *>(q);
        else {
            (void)hipGetLastError();
            p = fallback;
        }
    }
    return p;
}

const int64_t *Workspace::read_back(const ScalarGather &g) {
    rb.ensure(sizeof(int64_t) * 64);
    int64_t *h = pinned();
    launch_gather_scalars(g, rb.as<int64_t>(), s);
    SFN_HIP(hipMemcpyAsync(h, rb.get(), sizeof(int64_t) * (size_t)g.n, hipMemcpyDeviceToHost, s));
    SFN_HIP(hipStreamSynchronize(s));
    return h;
}

double Workspace::sum_rows(const DevBuf &rows, int64_t n) {
    return sum_rows_many({&rows}, n)[0];
}

std::vector<double> Workspace::sum_rows_many(std::initializer_list<const DevBuf *> rows,
                                             int64_t n) {
    const int k = (int)rows.size();
    whole.ensure(2 * sizeof(int64_t));
    if (whole_n != n) {
        const int64_t h[2] = {0, n};
        SFN_HIP(hipMemcpyAsync(whole.get(), h, sizeof(h), hipMemcpyHostToDevice, s));
        whole_n = n;
    }
    sums.ensure(sizeof(double) * (size_t)k);
    int j = 0;
    for (const DevBuf *r : rows)
        launch_seg_sum(r->as<double>(), whole.as<int64_t>(), 1, sums.as<double>() + j++, s);
    std::vector<double> out((size_t)k);
    SFN_HIP(hipMemcpyAsync(out.data(), sums.get(), sizeof(double) * (size_t)k,
                           hipMemcpyDeviceToHost, s));
    SFN_HIP(hipStreamSynchronize(s));
    return out;
}

double Workspace::max_rows(const DevBuf &rows, int64_t n) {
    seg.ensure(2 * sizeof(int64_t));
    red.ensure(sizeof(double));
    const int64_t h[2] = {0, n};
    SFN_HIP(hipMemcpyAsync(seg.get(), h, sizeof(h), hipMemcpyHostToDevice, s));
    launch_seg_max(rows.as<double>(), seg.as<int64_t>(), 1, red.as<double>(), s);
    return read_scalar(red.as<double>(), s);
}

void Workspace::report(const char *loop, int k, const sign_iter_stats &it) const {
    if (!progress) return;
    std::fprintf(stderr, "[signfn] %s k=%d%s e%s%.3e nnz_x=%lld nnz_r=%lld nnz_bar=%lld ms=%.1f\n",
                 loop, k, it.fp32 ? " fp32" : "", it.e_bound ? "<=" : "=", it.e,
                 (long long)it.nnz_x, (long long)it.nnz_r,
                 (long long)it.nnz_bar, it.ms);
    std::fflush(stderr);
}

void Workspace::note(const char *fmt, ...) const {
    if (!progress) return;
    std::fputs("[signfn] ", stderr);
    va_list ap;
    va_start(ap, fmt);
    std::vfprintf(stderr, fmt, ap);
    va_end(ap);
    std::fputc('\n', stderr);
    std::fflush(stderr);
}

namespace {
// Largest bucket b such that every bucket below b has its upper edge at most
// tau / sqrt(U): with at most U candidates, the entries there have a sum of
// squares <= tau^2, so every cut the selection can take drops them.
int safe_drop_bucket(double tau, double U) {
    if (!(tau > 0.0) || !(U >= 1.0)) return 0;
    const double t = tau / std::sqrt(U);
    int b = 0;
    while (b < kBucketTop) {
        const double hi = b == 0 ? std::ldexp(1.0, -127)
                                 : std::ldexp(1.0 + (double)((b - 1) % 16 + 1) / 16.0,
                                              (b - 1) / 16 - 127);
        if (hi > t) break;
        ++b;
    }
    return b;
}

template <typename V>
// no_store: only the per-row sums of squares and the entry counts of C are
// formed (C gets its row lengths and starts but no entries).
void product_rows(Workspace &w, const DMat<V> &A, const DMat<V> &B, const DMat<V> *D,
                  double coef, double dcoef, double diag, DMat<V> &C, DevBuf *sq_prod,
                  DevBuf *sq_out, LowerRows lower, const FusedFilter *ff,
                  bool no_store = false) {
    const int64_t n = A.n;
    hipStream_t s = w.s;
    if (B.n != n || (D && D->n != n)) throw Error(SIGN_EINVAL, "product: shape mismatch");
    w.lo.ensure(sizeof(int32_t) * n);
    w.span.ensure(sizeof(int32_t) * n);
    w.cap.ensure(sizeof(int64_t) * n);
    w.work.ensure(sizeof(int64_t) * n);
    w.capoff.ensure(sizeof(int64_t) * (n + 1));
    w.workoff.ensure(sizeof(int64_t) * (n + 1));
    w.tmp.ensure(sizeof(int64_t) * scan_tmp_elems(n));
    if (sq_prod) sq_prod->ensure(sizeof(double) * n);
    if (sq_out) sq_out->ensure(sizeof(double) * n);
    C.ensure_rows(n);

    MatView<V> Dv;
    if (D) Dv = D->view();
    launch_plan<V>(A.view(), B.view(), Dv, diag != 0.0, 0, n, w.lo.as<int32_t>(),
                   w.span.as<int32_t>(), w.cap.as<int64_t>(), w.work.as<int64_t>(), w.row_skip,
                   s);
    launch_exclusive_scan_i64(w.cap.as<int64_t>(), n, w.capoff.as<int64_t>(), w.tmp.as<int64_t>(),
                              0, s);
    launch_exclusive_scan_i64(w.work.as<int64_t>(), n, w.workoff.as<int64_t>(),
                              w.tmp.as<int64_t>(), 0, s);
    // totals of the plan (and B's density) come back in one copy
    int64_t tot[2];
    unsigned long long pst[2] = {0, 0};
    // B's density over its rows' column ranges (progress: reported with the product)
    const bool want_pst = w.auto_group || w.progress || w.page_mode == 1;
    ScalarGather pg;
    pg.add(w.capoff.as<int64_t>() + n);
    pg.add(w.workoff.as<int64_t>() + n);
    if (want_pst) {
        w.pst.ensure(2 * sizeof(unsigned long long));
        SFN_HIP(hipMemsetAsync(w.pst.get(), 0, 2 * sizeof(unsigned long long), s));
        launch_row_density<V>(B.view(), w.pst.as<unsigned long long>(), s);
        pg.add(w.pst.as<unsigned long long>());
        pg.add(w.pst.as<unsigned long long>() + 1);
    }
    // B with a few entries per row (e.g. B = A): lane-per-slot accumulation
    const bool short_b = B.nnz <= 16 * std::max<int64_t>(B.n, 1);
    // page lists of B's rows, for page windows of row groups: counted and
    // scanned here, so that their total comes back with the plan's (not for
    // n <= 2048, where column ranges are too short for pages to gain anything,
    // nor for short B rows: X·A with A the stencil runs fastest in pairs with
    // dense windows -- in groups of 4 with page windows the 256x256 Laplacian's
    // takes 4.7 ms against 3.7, the 32^3 Laplacian's 15.9 against 10.9, and the
    // 512x512 convection-diffusion gains 2% of a mixed solve;
    // SIGNFN_PAGES=on still forces them onto products with long A rows).
    const bool pages_wanted =
        w.page_mode != 0 && n > 2048 &&
        (!short_b || (w.page_mode == 2 && A.nnz >= 64 * std::max<int64_t>(n, 1)));
    if (pages_wanted) {
        w.plen.ensure(sizeof(int32_t) * n);
        w.pbeg.ensure(sizeof(int64_t) * (n + 1));
        launch_page_count<V>(B.view(), w.page_shift, w.plen.as<int32_t>(), s);
        launch_exclusive_scan_i32(w.plen.as<int32_t>(), n, w.pbeg.as<int64_t>(),
                                  w.tmp.as<int64_t>(), 0, s);
        pg.add(w.pbeg.as<int64_t>() + n);
    }
    int64_t page_total = 0;
    {
        const int64_t *h = w.read_back(pg);
        tot[0] = h[0];
        tot[1] = h[1];
        int at = 2;
        if (want_pst) {
            pst[0] = (unsigned long long)h[at++];
            pst[1] = (unsigned long long)h[at++];
        }
        if (pages_wanted) page_total = h[at++];
    }
    const int64_t total_cap = tot[0];
    w.products += tot[1];
    ProductEpi epi;
    epi.lower = lower;
    epi.no_store = no_store ? 1 : 0;
    epi.short_b = short_b ? 1 : 0;
    if (ff) {
        // the filter's histogram comes out of the product, and entries that no
        // cut can keep are not stored (the candidates number at most total_cap,
        // counted twice below the diagonal of a symmetric product)
        epi.hist = ff->hist;
        epi.sq_pre = ff->sq_pre;
        epi.keep_from = ff->keep_from >= 0
                            ? ff->keep_from
                            : safe_drop_bucket(ff->tau, (lower.any() ? 2.0 : 1.0) *
                                                            (double)total_cap);
    }

    // batches of rows whose reserved output fits the staging budget
    const size_t entry = sizeof(int32_t) + sizeof(V);
    // memory use changes as iterates grow: the budget follows it for products
    // that need more than a gigabyte of staging (smaller ones keep the last one)
    if (w.staging_auto && (double)total_cap * (double)entry > (double)(size_t(1) << 30))
        w.staging_limit = w.low_memory ? std::min<size_t>(w.auto_staging(), size_t(8) << 30)
                                       : w.auto_staging();
    const int64_t budget = std::max<int64_t>((int64_t)(w.staging_limit / entry), n);
    if (w.progress && total_cap > (int64_t)1 << 30 && !w.al->alloc)
        w.note("product: %lld rows, %lld reserved entries, staging %.1f GB, pool %.1f GB in use, "
               "%.1f GB cached", (long long)n, (long long)total_cap, w.staging_limit / 1e9,
               Pool::instance().used_bytes() / 1e9, Pool::instance().cached_bytes() / 1e9);
    std::vector<int64_t> cuts{0};
    std::vector<int64_t> capoff_h;
    // (a product that stores nothing runs in one batch -- batches cost it ~10% --
    // except under memory pressure, where batches keep its per-A-entry cursors
    // and merged lists to one batch's A entries instead of all of A)
    if (total_cap <= budget || (no_store && !w.low_memory)) {
        cuts.push_back(n);
    } else {
        capoff_h.resize(n + 1);
        SFN_HIP(hipMemcpyAsync(capoff_h.data(), w.capoff.get(), sizeof(int64_t) * (n + 1),
                               hipMemcpyDeviceToHost, s));
        SFN_HIP(hipStreamSynchronize(s));
        int64_t r0 = 0;
        while (r0 < n) {
            // largest r1 with capoff[r1] - capoff[r0] <= budget (at least one row)
            auto it = std::upper_bound(capoff_h.begin() + r0 + 1, capoff_h.end(),
                                       capoff_h[r0] + budget);
            int64_t r1 = (int64_t)(it - capoff_h.begin()) - 1;
            if (r1 <= r0) r1 = r0 + 1;
            cuts.push_back(r1);
            r0 = r1;
        }
    }
    const int64_t a_extent = A.capacity();
    // The per-A-entry arrays (cursors, merged group lists) cover the A entries
    // of one batch when the product runs in several batches and A is compact:
    // batch [r0, r1) then uses A's index range [beg[r0], beg[r1]), and the
    // arrays are addressed through pointers shifted by beg[r0].
    std::vector<int64_t> abeg_h;
    if (cuts.size() > 2) {
        std::vector<int32_t> alen_h(n);
        abeg_h.resize(n + 1);
        SFN_HIP(hipMemcpyAsync(abeg_h.data(), A.begp(), sizeof(int64_t) * (n + 1),
                               hipMemcpyDeviceToHost, s));
        SFN_HIP(hipMemcpyAsync(alen_h.data(), A.lenp(), sizeof(int32_t) * n,
                               hipMemcpyDeviceToHost, s));
        SFN_HIP(hipStreamSynchronize(s));
        for (int64_t i = 0; i < n && !abeg_h.empty(); ++i)
            if (abeg_h[i] + alen_h[i] != abeg_h[i + 1]) abeg_h.clear();  // not compact
    }
    w.bins.ensure(sizeof(int32_t) * kClasses * (size_t)std::max<int64_t>(n, 1));
    w.counts.ensure(sizeof(int32_t) * kClasses);
    // class statistics, then the spread per-workgroup counters (kernels.hpp)
    w.cstat.ensure(sizeof(int64_t) * (8 * kClasses + kSpreadWords));
    int64_t *const spread = w.cstat.as<int64_t>() + 8 * kClasses;
    // spread counter j of class c: 0 entries written, 1 B entries of merged
    // lists, 2 multiply-adds
    auto counter = [&](int c, int j) { return spread + (c * kSpreadCounters + j) * kSpread * kSpreadStride; };
    // row groups need A compact (rows i .. i+g-1 adjacent in storage) -- every
    // matrix built here is; the merged lists reuse A's index range
    // Groups of 8 rows (2048-column windows) halve the B traffic of groups of 4
    // (4096), but every window costs a pass over the group's slots.  Measured
    // per product on the 2D and 3D workloads: groups of 8 pay off only for FP64
    // values with long A rows (hundreds of entries: the rows of a group then
    // share most of their slots) and B rows holding many entries per window
    // (density within their column range times 2048 of ~200 or more);
    // products whose A or B rows hold a few entries (A·X and X·A with A the
    // stencil) run fastest in pairs (two 512-thread workgroups per CU); all
    // others (FP32 values, sparse B rows) in groups of 4.  A served batch (row
    // mask set) mixes requests at different steps, whose rows the averages do
    // not describe: it takes no pairs.
    // Page windows (kernels.hip k_spgemm_rows) pay off when B's rows occupy few
    // of the 16-column pages of their column ranges: measured per product, 2D
    // grid products (pages 0.04 - 0.3 of the range) gain up to 1.5x, 3D ones
    // (0.33 - 0.7) lose 3 - 9% to the marking and the page lookups.
    const double page_range = std::ldexp((double)page_total, w.page_shift);
    const bool pages_ok =
        pages_wanted && (w.page_mode == 2 || (pst[1] > 0 && page_range <= 0.3 * (double)pst[1]));
    // With page windows the fill of the occupied pages decides instead: groups
    // of 8 win for FP64 values with long A rows when B's entries fill 55% or
    // more of its pages (2D grids, 0.59 - 0.7) and lose 5 - 13% below (3D,
    // ~0.5). Squares of an iterate with short rows (X·X, hundreds of entries
    // or fewer) gain 15 - 35% in groups of 8 at any fill and precision: the
    // rows of a group gather the same B rows their own neighbours hold. Pairs
    // lose to groups of 4 (up to 3x on the stencil products).
    int group = w.row_group;
    if (w.auto_group && w.row_skip && sizeof(V) == 8) {
        // a served batch mixes requests whose rows the averages do not describe:
        // groups of 8 measured best for it (2,000 requests at 50/s: 29.2 against 28.4
        // solves/s with the rules; 400 requests: 28.5 against 27.4)
        group = 8;
    } else if (w.auto_group && pst[1] > 0) {
        const bool long_a = A.nnz >= 512 * n;
        if (pages_ok) {
            const bool full_pages = (double)pst[0] >= 0.55 * page_range;
            const bool short_square = &A == &B && !long_a;
            group = ((sizeof(V) == 8 && long_a && full_pages) || short_square) ? 8 : 4;
        } else {
            const bool dense_b = 2048ull * pst[0] >= 200ull * pst[1];
            if (!w.row_skip && (A.nnz < 64 * n || B.nnz <= 16 * n))
                group = 2;
            else
                group = (sizeof(V) == 8 && long_a && dense_b) ? 8 : 4;
        }
    }
    // The register-accumulator kernel (k_spgemm_regtile) trades the LDS atomic
    // per product for one LDS round trip per gathered B entry and register
    // multiply-adds, with groups of rt_group rows sharing every gathered entry.
    bool use_rt = false;
    if (w.rt_mode > 0 && !epi.short_b && (w.rt_mode == 2 || (!w.row_skip && A.nnz >= 64 * n))) {
        use_rt = true;
        group = w.rt_group;
    }
    if (group > 1) w.mlen.ensure(sizeof(int32_t) * (size_t)std::max<int64_t>(n, 1));
    // row groups run their windows over the column pages they occupy
    if (pages_ok && group > 1 && !use_rt) {
        w.plist.ensure(sizeof(int32_t) * (size_t)std::max<int64_t>(page_total, 1));
        launch_page_fill<V>(B.view(), w.page_shift, w.pbeg.as<int64_t>(), w.plist.as<int32_t>(),
                            s);
        epi.pages.beg = w.pbeg.as<int64_t>();
        epi.pages.len = w.plen.as<int32_t>();
        epi.pages.pg = w.plist.as<int32_t>();
        epi.pages.shift = w.page_shift;
    }
    const double ms_before = w.spgemm_ms;

    int64_t running = 0;
    for (size_t b = 0; b + 1 < cuts.size(); ++b) {
        const int64_t r0 = cuts[b], r1 = cuts[b + 1];
        const int64_t base = capoff_h.empty() ? 0 : capoff_h[r0];
        const int64_t bcap = capoff_h.empty() ? total_cap : capoff_h[r1] - base;
        if (!no_store) {
            w.stage_col.ensure(sizeof(int32_t) * (size_t)std::max<int64_t>(bcap, 1));
            w.stage_val.ensure(sizeof(V) * (size_t)std::max<int64_t>(bcap, 1));
        }
        const int64_t abase = abeg_h.empty() ? 0 : abeg_h[r0];
        const size_t aext =
            (size_t)std::max<int64_t>(abeg_h.empty() ? a_extent : abeg_h[r1] - abase, 1);
        w.cursor.ensure(sizeof(int32_t) * aext);
        w.cnext.ensure(sizeof(int32_t) * aext);
        if (group > 1) {
            w.mk.ensure(sizeof(int32_t) * aext);
            w.mm.ensure(sizeof(uint32_t) * aext);
            w.mc.ensure(sizeof(int32_t) * aext);
            w.cv.ensure(sizeof(V) * aext);
        }
        // indexed by A entry: every index a kernel uses lies in [abase, abase + aext)
        int32_t *cursor_a = w.cursor.as<int32_t>() - abase;
        int32_t *cnext_a = w.cnext.as<int32_t>() - abase;
        int32_t *mk_a = group > 1 ? w.mk.as<int32_t>() - abase : nullptr;
        uint32_t *mm_a = group > 1 ? w.mm.as<uint32_t>() - abase : nullptr;
        int32_t *mc_a = group > 1 ? w.mc.as<int32_t>() - abase : nullptr;
        V *cv_a = group > 1 ? w.cv.as<V>() - abase : nullptr;
        SFN_HIP(hipMemsetAsync(w.counts.get(), 0, sizeof(int32_t) * kClasses, s));
        SFN_HIP(hipMemsetAsync(w.cstat.get(), 0, sizeof(int64_t) * (8 * kClasses + kSpreadWords),
                               s));
        launch_bin_rows(w.span.as<int32_t>(), w.work.as<int64_t>(), r0, r1, kSmallTile, kMidTile,
                        group, w.bins.as<int32_t>(), n, w.counts.as<int32_t>(),
                        C.lenp(), sq_prod ? sq_prod->as<double>() : nullptr,
                        sq_out ? sq_out->as<double>() : nullptr, A.lenp(),
                        D ? D->lenp() : nullptr, w.cstat.as<int64_t>(), s);
        int32_t cnt[kClasses];
        SFN_HIP(hipMemcpyAsync(cnt, w.counts.get(), sizeof(cnt), hipMemcpyDeviceToHost, s));
        SFN_HIP(hipStreamSynchronize(s));
        SFN_HIP(hipEventRecord(w.ev[0], s));
        if (cnt[4] > 0) {
            const int32_t *leads = w.bins.as<int32_t>() + (int64_t)4 * n;
            launch_merge_group<V>(group, leads, cnt[4], A.view(), B.view(), mk_a, mm_a, mc_a,
                                  cv_a, w.mlen.as<int32_t>(), counter(4, 1), s);
            SFN_HIP(hipEventRecord(w.ev[1], s));
            if (use_rt) {
                launch_spgemm_regtile<V>(group, w.rt_nb, leads, cnt[4], mk_a, mm_a, mc_a, cv_a,
                                         w.mlen.as<int32_t>(), A.view(), B.view(), Dv, coef,
                                         dcoef, diag, w.lo.as<int32_t>(), w.span.as<int32_t>(),
                                         base, w.capoff.as<int64_t>(),
                                         w.stage_col.as<int32_t>(), w.stage_val.as<V>(),
                                         C.lenp(), cursor_a, cnext_a,
                                         sq_prod ? sq_prod->as<double>() : nullptr,
                                         sq_out ? sq_out->as<double>() : nullptr,
                                         counter(4, 0), epi, s);
            } else {
                epi.madds = (unsigned long long *)counter(4, 2);
                launch_spgemm_group<V>(group, leads, cnt[4], mk_a, mm_a, mc_a, cv_a,
                                       w.mlen.as<int32_t>(), A.view(), B.view(), Dv, coef, dcoef,
                                       diag, w.lo.as<int32_t>(), w.span.as<int32_t>(), base,
                                       w.capoff.as<int64_t>(), w.stage_col.as<int32_t>(),
                                       w.stage_val.as<V>(), C.lenp(), cursor_a, cnext_a,
                                       sq_prod ? sq_prod->as<double>() : nullptr,
                                       sq_out ? sq_out->as<double>() : nullptr,
                                       counter(4, 0), epi, s);
            }
        } else {
            SFN_HIP(hipEventRecord(w.ev[1], s));
        }
        SFN_HIP(hipEventRecord(w.ev[2], s));
        for (int cls = 3; cls >= 1; --cls) {
            epi.madds = (unsigned long long *)counter(cls, 2);
            launch_spgemm<V>(cls, w.bins.as<int32_t>() + (int64_t)cls * n, cnt[cls], A.view(),
                             B.view(), Dv, coef, dcoef, diag, w.lo.as<int32_t>(),
                             w.span.as<int32_t>(), base, w.capoff.as<int64_t>(),
                             w.stage_col.as<int32_t>(), w.stage_val.as<V>(), C.lenp(),
                             cursor_a, cnext_a,
                             sq_prod ? sq_prod->as<double>() : nullptr,
                             sq_out ? sq_out->as<double>() : nullptr,
                             counter(cls, 0), epi, s);
            SFN_HIP(hipEventRecord(w.ev[6 - cls], s));
        }
        // compact row starts of this batch, continuing from the previous batches
        launch_exclusive_scan_i32(C.lenp() + r0, r1 - r0, C.begp() + r0,
                                  w.tmp.as<int64_t>(), running, s);
        // the class statistics and the stored total (gathered into the unused
        // slot 0 of class 0) come back in one copy
        int64_t *cs = Workspace::pinned();
        {
            ScalarGather eg;
            eg.add(C.begp() + r1);
            eg.fold = spread;
            eg.fold_dst = w.cstat.as<int64_t>();
            launch_gather_scalars(eg, w.cstat.as<int64_t>(), s);
            SFN_HIP(hipMemcpyAsync(cs, w.cstat.get(), sizeof(int64_t) * 8 * kClasses,
                                   hipMemcpyDeviceToHost, s));
            SFN_HIP(hipStreamSynchronize(s));
        }
        int64_t cs_h[8 * kClasses];
        std::memcpy(cs_h, cs, sizeof(cs_h));
        const int64_t end = cs_h[0];
        {
            float mm = 0.f;
            SFN_HIP(hipEventElapsedTime(&mm, w.ev[0], w.ev[1]));
            w.merge_ms += mm;
        }
        // event pairs bracketing the numeric launches: class 4 ev[1]..ev[2],
        // class 3 ev[2]..ev[3], class 2 ev[3]..ev[4], class 1 ev[4]..ev[5]
        const int evb[kClasses] = {0, 4, 3, 2, 1};
        for (int cls = 4; cls >= 1; --cls) {
            float ms = 0.f;
            SFN_HIP(hipEventElapsedTime(&ms, w.ev[evb[cls]], w.ev[evb[cls] + 1]));
            w.spgemm_ms += ms;
            if (cnt[cls] <= 0) continue;
            const int lg = group >= 16 ? 4 : group >= 8 ? 3 : group >= 4 ? 2 : group >= 2 ? 1 : 0;
            Workspace::ClassStat &c = cls == 4 ? (use_rt ? w.rt[sizeof(V) == 4 ? 1 : 0]
                                                         : w.grp[sizeof(V) == 4 ? 1 : 0][lg])
                                               : w.cls[sizeof(V) == 4 ? 1 : 0][cls];
            if (cls == 4 && use_rt) {
                w.rt_used_group = group;
                w.rt_used_nb = w.rt_nb;
            }
            const int64_t *q = cs_h + cls * 8;
            c.launches += 1;
            c.rows += cls == 4 ? (int64_t)group * cnt[cls] : cnt[cls];
            c.products += q[1];
            // the register-accumulator kernel does not count: its plan's products
            const int64_t md = cls == 4 && use_rt ? q[1] : q[6];
            c.madds += md;
            w.madds += md;
            if (cls == 4 && epi.pages.pg) c.page_launches += 1;
            c.a_nnz += q[2];
            c.d_nnz += q[3];
            c.out += q[4];
            c.ms += ms;
            // algorithmic (compulsory) bytes: the A and D rows of the launch, its
            // share of B (each entry once per product, cache-perfect), the stored
            // output, row descriptors
            const double eb = (double)(sizeof(int32_t) + sizeof(V));
            const double rows_here = cls == 4 ? (double)group * cnt[cls] : (double)cnt[cls];
            const double b_share = n > 0 ? (double)B.nnz * rows_here / (double)n : 0.0;
            const double bytes = eb * ((double)q[2] + (double)q[3] + (double)q[4] + b_share) +
                                 24.0 * rows_here;
            c.gathered += cls == 4 ? q[5] : q[1];
            c.bytes += bytes;
            w.spgemm_bytes += bytes;
        }
        if (no_store) {
            running = end;
            continue;
        }
        if (b == 0 && cuts.size() > 2 && bcap > 0) {
            // size C once from the first batch's fill ratio, so that later
            // batches rarely grow it (a grow keeps the old block alongside)
            const double est = 1.1 * (double)end * (double)total_cap / (double)bcap;
            C.ensure_entries(std::max<int64_t>(end, (int64_t)std::min(est, (double)total_cap)));
        }
        if (end > C.capacity() && !capoff_h.empty() && capoff_h[r1] > 0) {
            // a grow copies the entries stored so far: grow once to what the fill
            // ratio of the rows done so far predicts for the whole product
            const double fill = (double)end / (double)capoff_h[r1];
            const double est = (double)end + 1.1 * fill * (double)(total_cap - capoff_h[r1]);
            w.note("product: batch %zu of %zu outgrew the output (%lld > %lld entries), "
                   "regrown from the fill ratio %.3f", b + 1, cuts.size() - 1, (long long)end,
                   (long long)C.capacity(), fill);
            C.ensure_entries(std::max<int64_t>(end, (int64_t)std::min(est, (double)total_cap)),
                             running);
        }
        C.ensure_entries(end, running);
        launch_copy_rows<V>(w.capoff.as<int64_t>(), base, C.lenp(),
                            w.stage_col.as<int32_t>(), w.stage_val.as<V>(), r0, r1,
                            C.begp(), C.colp(), C.valp(), s);
        running = end;
    }
    C.nnz = running;
    if (w.progress && pst[1] > 0)
        w.note("product: %lld rows, %s, groups of %d, B entries per 2048 columns %.0f, "
               "B pages %.3f of the range (%s), A %.0f and B %.0f per row, output %lld, "
               "%.2f ms", (long long)n, sizeof(V) == 4 ? "FP32" : "FP64", group,
               2048.0 * (double)pst[0] / (double)pst[1],
               std::ldexp((double)page_total, w.page_shift) / (double)pst[1],
               epi.pages.pg ? "page windows" : "dense windows", (double)A.nnz / (double)n,
               (double)B.nnz / (double)n, (long long)running, w.spgemm_ms - ms_before);
}


}  // namespace

// C (full) from the lower triangle L of a symmetric matrix: rows of L first,
// then each row's mirror list (the strictly-lower entries of its column),
// ordered by column.
template <typename V>
void symmetrize(Workspace &w, const DMat<V> &L, DMat<V> &C, LowerRows lower) {
    const int64_t n = L.n;
    hipStream_t s = w.s;
    C.ensure_rows(n);
    w.symcnt.ensure(sizeof(int32_t) * std::max<int64_t>(n, 1));
    w.symfill.ensure(sizeof(int32_t) * std::max<int64_t>(n, 1));
    w.symoff.ensure(sizeof(int64_t) * (n + 1));
    w.tmp.ensure(sizeof(int64_t) * scan_tmp_elems(n));
    SFN_HIP(hipMemsetAsync(w.symcnt.get(), 0, sizeof(int32_t) * n, s));
    SFN_HIP(hipMemsetAsync(w.symfill.get(), 0, sizeof(int32_t) * n, s));
    launch_sym_count<V>(L.view(), lower, w.symcnt.as<int32_t>(), s);
    launch_exclusive_scan_i32(w.symcnt.as<int32_t>(), n, w.symoff.as<int64_t>(),
                              w.tmp.as<int64_t>(), 0, s);
    launch_add_len(L.lenp(), w.symcnt.as<int32_t>(), n, C.lenp(), s);
    launch_exclusive_scan_i32(C.lenp(), n, C.begp(), w.tmp.as<int64_t>(), 0, s);
    int64_t tot[2];
    {
        ScalarGather g;
        g.add(C.begp() + n);
        g.add(w.symoff.as<int64_t>() + n);
        const int64_t *h = w.read_back(g);
        tot[0] = h[0];
        tot[1] = h[1];
    }
    C.ensure_entries(tot[0]);
    w.symtcol.ensure(sizeof(int32_t) * (size_t)std::max<int64_t>(tot[1], 1));
    w.symtval.ensure(sizeof(V) * (size_t)std::max<int64_t>(tot[1], 1));
    launch_sym_place<V>(L.view(), lower, C.begp(), C.colp(), C.valp(), w.symoff.as<int64_t>(),
                        w.symfill.as<int32_t>(), w.symtcol.as<int32_t>(), w.symtval.as<V>(), s);
    launch_sym_rank<V>(n, C.begp(), L.lenp(), w.symoff.as<int64_t>(), w.symcnt.as<int32_t>(),
                       w.symtcol.as<int32_t>(), w.symtval.as<V>(), C.colp(), C.valp(), s);
    C.nnz = tot[0];
}
template void symmetrize<double>(Workspace &, const DMat<double> &, DMat<double> &, LowerRows);
template void symmetrize<float>(Workspace &, const DMat<float> &, DMat<float> &, LowerRows);

template <typename V>
void product(Workspace &w, const DMat<V> &A, const DMat<V> &B, const DMat<V> *D, double coef,
             double dcoef, double diag, DMat<V> &C, DevBuf *sq_prod, DevBuf *sq_out, bool sym,
             bool keep_lower, const FusedFilter *ff, const uint8_t *row_sym) {
    LowerRows lower;
    lower.all = sym ? 1 : 0;
    lower.rows = row_sym;
    if (!lower.any() || keep_lower) {
        product_rows<V>(w, A, B, D, coef, dcoef, diag, C, sq_prod, sq_out, lower, ff);
        return;
    }
    DMat<V> L;
    L.bind(w.al);
    product_rows<V>(w, A, B, D, coef, dcoef, diag, L, sq_prod, sq_out, lower, ff);
    symmetrize<V>(w, L, C, lower);
}

template <typename V>
int64_t product_sumsq(Workspace &w, const DMat<V> &A, const DMat<V> &B, double coef,
                      double diag, DevBuf *sq_out, bool sym) {
    LowerRows lower;
    lower.all = sym ? 1 : 0;
    DMat<V> C;
    C.bind(w.al);
    product_rows<V>(w, A, B, nullptr, coef, 0.0, diag, C, nullptr, sq_out, lower, nullptr, true);
    return C.nnz;
}
template int64_t product_sumsq<double>(Workspace &, const DMat<double> &, const DMat<double> &,
                                       double, double, DevBuf *, bool);

template <typename V>
bool is_symmetric(Workspace &w, const DMat<V> &X) {
    w.flag.ensure(sizeof(int));
    SFN_HIP(hipMemsetAsync(w.flag.get(), 0, sizeof(int), w.s));
    launch_sym_check<V>(X.view(), w.flag.as<int>(), w.s);
    return read_scalar(w.flag.as<int>(), w.s) == 0;
}
template bool is_symmetric<double>(Workspace &, const DMat<double> &);
template bool is_symmetric<float>(Workspace &, const DMat<float> &);

template <typename V, typename Vo>
int filter(Workspace &w, const DMat<V> &In, double tau, DMat<Vo> &Out, DevBuf *sq_keep,
           DevBuf *sq_drop, int lower, bool hist_ready, int64_t *candidates) {
    const int64_t n = In.n;
    hipStream_t s = w.s;
    Out.ensure_rows(n);
    w.hist.ensure(sizeof(uint64_t) * kBuckets);
    w.seg.ensure(2 * sizeof(int64_t));
    w.tau.ensure(sizeof(double));
    w.bstar.ensure(sizeof(int64_t));  // read back as a 64-bit word
    w.tmp.ensure(sizeof(int64_t) * scan_tmp_elems(n));
    if (sq_keep) sq_keep->ensure(sizeof(double) * n);
    if (sq_drop) sq_drop->ensure(sizeof(double) * n);
    launch_set_filter_args(w.seg.as<int64_t>(), n, w.tau.as<double>(), tau, s);
    if (!hist_ready) {
        SFN_HIP(hipMemsetAsync(w.hist.get(), 0, sizeof(uint64_t) * kBuckets, s));
            LowerRows lr;
        lr.all = lower;
        launch_histogram<V>(In.view(), w.seg.as<int64_t>(), 1, n, w.hist.as<uint64_t>(), lr, s);
    }
    launch_select(w.hist.as<uint64_t>(), w.tau.as<double>(), 1, w.bstar.as<int>(), s);
    LowerRows lrk;
    lrk.all = lower;
    launch_count_keep<V>(In.view(), nullptr, w.bstar.as<int>(), Out.lenp(),
                         sq_keep ? sq_keep->as<double>() : nullptr,
                         sq_drop ? sq_drop->as<double>() : nullptr, lrk, s);
    launch_exclusive_scan_i32(Out.lenp(), n, Out.begp(),
                              w.tmp.as<int64_t>(), 0, s);
    // kept total, cut and (when asked) the candidate count in one copy
    int64_t total;
    int bstar;
    {
        w.rb.ensure(sizeof(int64_t) * 64);
        ScalarGather g;
        g.add(Out.begp() + n);
        g.add(w.bstar.get());
        launch_gather_scalars(g, w.rb.as<int64_t>(), s);
        if (candidates) launch_hist_total(w.hist.as<uint64_t>(), w.rb.as<int64_t>() + 2, s);
        int64_t *h = Workspace::pinned();
        SFN_HIP(hipMemcpyAsync(h, w.rb.get(), sizeof(int64_t) * 3, hipMemcpyDeviceToHost, s));
        SFN_HIP(hipStreamSynchronize(s));
        total = h[0];
        bstar = (int)(uint32_t)(uint64_t)h[1];  // the low word holds the int
        if (candidates) *candidates = h[2];
    }
    Out.ensure_entries(total);
    launch_scatter_keep<V, Vo>(In.view(), nullptr, w.bstar.as<int>(), Out.begp(),
                               Out.colp(), Out.valp(), s);
    Out.nnz = total;
    return bstar;
}

int select_cut(Workspace &w, int64_t n, double tau) {
    hipStream_t s = w.s;
    w.seg.ensure(2 * sizeof(int64_t));
    w.tau.ensure(sizeof(double));
    w.bstar.ensure(sizeof(int64_t));
    launch_set_filter_args(w.seg.as<int64_t>(), n, w.tau.as<double>(), tau, s);
    launch_select(w.hist.as<uint64_t>(), w.tau.as<double>(), 1, w.bstar.as<int>(), s);
    return read_scalar(w.bstar.as<int>(), s);
}

void filter_seg(Workspace &w, const DMat<double> &In, const std::vector<int64_t> &seg_h,
                const int64_t *seg_d, const int32_t *row_seg, const std::vector<double> &tau_h,
                DMat<double> &Out, DevBuf *sq_keep, DevBuf *sq_drop, std::vector<int> &bstar_h,
                LowerRows lower) {
    const int64_t n = In.n;
    const int nseg = (int)tau_h.size();
    hipStream_t s = w.s;
    Out.ensure_rows(n);
    w.hist.ensure(sizeof(uint64_t) * kBuckets * nseg);
    w.tau.ensure(sizeof(double) * nseg);
    w.bstar.ensure(sizeof(int) * nseg);
    w.tmp.ensure(sizeof(int64_t) * scan_tmp_elems(n));
    if (sq_keep) sq_keep->ensure(sizeof(double) * n);
    if (sq_drop) sq_drop->ensure(sizeof(double) * n);
    int64_t maxrows = 0;
    for (int q = 0; q < nseg; ++q) maxrows = std::max(maxrows, seg_h[q + 1] - seg_h[q]);
    SFN_HIP(hipMemcpyAsync(w.tau.get(), tau_h.data(), sizeof(double) * nseg,
                           hipMemcpyHostToDevice, s));
    SFN_HIP(hipMemsetAsync(w.hist.get(), 0, sizeof(uint64_t) * kBuckets * nseg, s));
    launch_histogram<double>(In.view(), seg_d, nseg, maxrows, w.hist.as<uint64_t>(), lower, s);
    launch_select(w.hist.as<uint64_t>(), w.tau.as<double>(), nseg, w.bstar.as<int>(), s);
    launch_count_keep<double>(In.view(), row_seg, w.bstar.as<int>(), Out.lenp(),
                              sq_keep ? sq_keep->as<double>() : nullptr,
                              sq_drop ? sq_drop->as<double>() : nullptr, lower, s);
    launch_exclusive_scan_i32(Out.lenp(), n, Out.begp(), w.tmp.as<int64_t>(), 0, s);
    int64_t total;
    bstar_h.resize(nseg);
    SFN_HIP(hipMemcpyAsync(&total, Out.begp() + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    SFN_HIP(hipMemcpyAsync(bstar_h.data(), w.bstar.get(), sizeof(int) * nseg,
                           hipMemcpyDeviceToHost, s));
    SFN_HIP(hipStreamSynchronize(s));
    Out.ensure_entries(total);
    launch_scatter_keep<double, double>(In.view(), row_seg, w.bstar.as<int>(), Out.begp(),
                                        Out.colp(), Out.valp(), s);
    Out.nnz = total;
}

std::vector<double> seg_sums(Workspace &w, const DevBuf &rows, const int64_t *seg_d, int nseg) {
    std::vector<double> h(nseg);
    if (nseg == 0) return h;
    w.red.ensure(sizeof(double) * nseg);
    launch_seg_sum(rows.as<double>(), seg_d, nseg, w.red.as<double>(), w.s);
    SFN_HIP(hipMemcpyAsync(h.data(), w.red.get(), sizeof(double) * nseg, hipMemcpyDeviceToHost,
                           w.s));
    SFN_HIP(hipStreamSynchronize(w.s));
    return h;
}

std::vector<double> seg_maxs(Workspace &w, const DevBuf &rows, const int64_t *seg_d, int nseg) {
    std::vector<double> h(nseg);
    if (nseg == 0) return h;
    w.red.ensure(sizeof(double) * nseg);
    launch_seg_max(rows.as<double>(), seg_d, nseg, w.red.as<double>(), w.s);
    SFN_HIP(hipMemcpyAsync(h.data(), w.red.get(), sizeof(double) * nseg, hipMemcpyDeviceToHost,
                           w.s));
    SFN_HIP(hipStreamSynchronize(w.s));
    return h;
}

std::vector<double> seg_norm_one_inf(Workspace &w, const DMat<double> &X, const int64_t *seg_d,
                                     int nseg) {
    const int64_t n = X.n;
    w.rs4.ensure(sizeof(double) * std::max<int64_t>(n, 1));
    SFN_HIP(hipMemsetAsync(w.rs4.get(), 0, sizeof(double) * n, w.s));
    launch_col_abs_sum<double>(X.view(), w.rs4.as<double>(), w.s);
    const std::vector<double> one = seg_maxs(w, w.rs4, seg_d, nseg);
    launch_row_abs_sum(X.begp(), X.valp(), 0, n, w.rs4.as<double>(), w.s);
    std::vector<double> inf = seg_maxs(w, w.rs4, seg_d, nseg);
    for (int q = 0; q < nseg; ++q) inf[q] *= one[q];
    return inf;
}

template <typename V>
void row_sumsq(Workspace &w, const DMat<V> &X, DevBuf &rows) {
    const int64_t n = X.n;
    rows.ensure(sizeof(double) * n);
    w.icnt.ensure(sizeof(int32_t) * std::max<int64_t>(n, 1));
    w.zero_b.ensure(sizeof(int));
    SFN_HIP(hipMemsetAsync(w.zero_b.get(), 0, sizeof(int), w.s));
    launch_count_keep<V>(X.view(), nullptr, w.zero_b.as<int>(), w.icnt.as<int32_t>(),
                         rows.as<double>(), nullptr, LowerRows(), w.s);
}

double nsf_budget(double e, double xfro, double tol, double c_fixed, double switch_res) {
    if (e >= switch_res) return c_fixed * tol;
    return 0.75 * e * e / (3.0 * xfro + xfro * xfro * xfro);
}

double nmf_budget(double e, double xfro, double zfro, double tol, double c_fixed,
                  double switch_res) {
    if (e >= switch_res) return c_fixed * tol;
    return e * e / (xfro + zfro);
}

namespace {
// Dst = Src (compact FP64), a device copy
void copy_mat(Workspace &w, const DMat<double> &Src, DMat<double> &Dst) {
    const int64_t n = Src.n;
    Dst.ensure_rows(n);
    Dst.ensure_entries(Src.nnz);
    SFN_HIP(hipMemcpyAsync(Dst.begp(), Src.begp(), sizeof(int64_t) * (n + 1),
                           hipMemcpyDeviceToDevice, w.s));
    SFN_HIP(hipMemcpyAsync(Dst.lenp(), Src.lenp(), sizeof(int32_t) * n, hipMemcpyDeviceToDevice,
                           w.s));
    if (Src.nnz > 0) {
        SFN_HIP(hipMemcpyAsync(Dst.colp(), Src.colp(), sizeof(int32_t) * Src.nnz,
                               hipMemcpyDeviceToDevice, w.s));
        SFN_HIP(hipMemcpyAsync(Dst.valp(), Src.valp(), sizeof(double) * Src.nnz,
                               hipMemcpyDeviceToDevice, w.s));
    }
    Dst.nnz = Src.nnz;
}

// ||M||_inf (largest absolute row sum) of a compact FP64 matrix
double inf_norm(Workspace &w, const DMat<double> &M) {
    w.rs4.ensure(sizeof(double) * std::max<int64_t>(M.n, 1));
    launch_row_abs_sum(M.begp(), M.valp(), 0, M.n, w.rs4.as<double>(), w.s);
    return w.max_rows(w.rs4, M.n);
}

// ||X||_1 * ||X||_inf of a compact FP64 matrix
double norm_one_inf(Workspace &w, const DMat<double> &X) {
    const int64_t n = X.n;
    w.rs4.ensure(sizeof(double) * n);
    SFN_HIP(hipMemsetAsync(w.rs4.get(), 0, sizeof(double) * n, w.s));
    launch_col_abs_sum<double>(X.view(), w.rs4.as<double>(), w.s);
    const double one = w.max_rows(w.rs4, n);
    launch_row_abs_sum(X.begp(), X.valp(), 0, n, w.rs4.as<double>(), w.s);
    const double inf = w.max_rows(w.rs4, n);
    return one * inf;
}

// Upper bound of ||I - X^2||_F from a thinned copy Xt = X - D (||D||_F = delta,
// D the entries of a filter cut with budget tau_c):
//   I - X^2 = (I - Xt^2) - (Xt D + D Xt) - D^2,
//   ||I - X^2||_F <= ||I - Xt^2||_F + 2 ||Xt||_2 delta + delta^2,
// with ||Xt||_2 <= sqrt(||X||_1 ||X||_inf) (dropping entries lowers both), and
// for an exactly symmetric Xt also ||Xt||_2^2 = ||Xt^2||_2 <= 1 + ||I - Xt^2||_F.
// nnz_r receives the entry count of I - Xt^2 (of its lower triangle when sym).
double thinned_residual_bound(Workspace &w, const DMat<double> &X, bool sym, double tol,
                              DMat<double> &Xt, int64_t *nnz_r) {
    const int64_t n = X.n;
    const double s_one_inf = sym ? 1.0 : std::sqrt(norm_one_inf(w, X));
    const double tau_c = tol / (16.0 * s_one_inf);
    filter<double, double>(w, X, tau_c, Xt, nullptr, &w.rs4);
    // only the norm of I - Xt^2 is needed: nothing is stored
    *nnz_r = product_sumsq<double>(w, Xt, Xt, -1.0, 1.0, &w.rs1, sym);
    const std::vector<double> sums = w.sum_rows_many({&w.rs1, &w.rs4}, n);
    const double et = std::sqrt(sums[0]);
    const double delta = std::sqrt(sums[1]);
    const double s2 = sym ? std::sqrt(1.0 + et) : s_one_inf;
    return et + 2.0 * s2 * delta + delta * delta;
}
}  // namespace

template <typename V>
LoopOut nsf_loop(Workspace &w, DMat<V> &X, const LoopParams &p,
                 std::vector<sign_iter_stats> &trace) {
    const int64_t n = X.n;
    DMat<V> R, Xb, Xn, Xl;
    R.bind(w.al); Xb.bind(w.al); Xn.bind(w.al); Xl.bind(w.al);
    LoopOut out;
    row_sumsq(w, X, w.rs3);
    double xf = std::sqrt(w.sum_rows(w.rs3, n));
    double d_prev = std::numeric_limits<double>::infinity();
    double ff_prev = std::numeric_limits<double>::infinity();
    int n_up = 0, n_flat = 0;
    std::vector<double> es;
    // Under memory pressure (filter_y): the residual and the update are formed
    // in two passes, so that neither the unfiltered residual nor the update's
    // candidates are ever stored -- from the first step when asked
    // (SIGNFN_RESIDUAL_TWO_PASS=1), else from the step whose one-pass form runs
    // out of device memory; dead matrices and the product staging then go back
    // to the pool as soon as they are dead, and the staging is capped.
    bool two_pass = w.residual_two_pass;
    if (two_pass) w.low_memory = true;
    auto release_dead = [&]() {
        Xb.release_entries();
        Xn.release_entries();
        w.stage_col.reset();
        w.stage_val.reset();
    };
    for (int k = 1;; ++k) {
        const double t0 = now_s();
        if (!p.check_last && k - 1 >= p.max_iter) {
            // the caller continues from X^_k and does not use its residual
            out.status = SIGN_ENOCONV;
            out.iters = k - 1;
            out.xfro = xf;
            break;
        }
        if (p.predict_stop && p.stop_rule == 0 && k >= 2) {
            // Lemma 2.1.1 and the last cut bound e_k by about 3/4 e_{k-1}^2 + 2||F_k||
            const double ep = es.back();
            const double pred = 0.75 * ep * ep * (1.0 + ep / 3.0) + 2.5 * ff_prev;
            if (pred <= 0.25 * p.tol) {
                out.status = SIGN_OK;
                out.iters = k - 1;
                out.xfro = xf;
                out.e = pred;
                break;
            }
        }
        // residual of the current iterate: R^_k = I - X^_k^2
        // symmetric products keep X^ exactly symmetric only when R^ stays the
        // exact polynomial I - X^2 (R^ not filtered): then X^R^ is symmetric too
        const bool sym = p.sym && !p.filter_y;
        // Where Lemma 2.1.1 (R_{k+1} = 3/4 R_k^2 + 1/4 R_k^3) and the last cut
        // predict e_k far below tol, e_k <= tol is first certified from a thinned
        // copy of X^_k, whose square costs a fraction of X^_k^2; the full residual
        // is formed only if that bound does not reach tol.  (cert_first: the
        // caller expects the first iterate to be converged already.)
        double e = -1.0;
        int e_bound = 0;
        int64_t nnz_cert = 0;
        if constexpr (sizeof(V) == 8) {
            bool try_cert = p.stop_rule == 0 && k == 1 && p.cert_first;
            if (p.stop_rule == 0 && k >= 2) {
                const double ep = es.back();
                const double pred = 0.75 * ep * ep * (1.0 + ep / 3.0) + 2.5 * ff_prev;
                try_cert = pred <= 0.25 * p.tol;
            }
            if (try_cert) {
                try {
                    DMat<double> Xt;
                    Xt.bind(w.al);
                    const double b = thinned_residual_bound(w, X, sym, p.tol, Xt, &nnz_cert);
                    if (b <= p.tol) { e = b; e_bound = 1; }
                } catch (const Error &err) {
                    // no room for the thinned copy and its square: the full
                    // residual below certifies instead
                    if (err.status != SIGN_ENOMEM) throw;
                    w.note("ns k=%d: out of device memory certifying from a thinned copy; "
                           "forming the residual", k);
                    release_dead();
                }
            }
        }
        // two passes (filter_y only): this one forms e_k and the filter's
        // histogram of R_k and stores nothing; the kept entries come after the cut
        auto residual_first_pass = [&]() {
            w.hist.ensure(sizeof(uint64_t) * kBuckets);
            SFN_HIP(hipMemsetAsync(w.hist.get(), 0, sizeof(uint64_t) * kBuckets, w.s));
            const FusedFilter hist_only{0.0, w.hist.as<uint64_t>(), nullptr};
            product_rows<V>(w, X, X, nullptr, -1.0, 0.0, 1.0, R, nullptr, &w.rs1, LowerRows{},
                            &hist_only, true);
            e = std::sqrt(w.sum_rows(w.rs1, n));
        };
        bool residual_two_pass = !e_bound && p.filter_y && two_pass;
        if (residual_two_pass) {
            residual_first_pass();
        } else if (!e_bound) {
            try {
                if (p.filter_y) {
                    // the residual's filter takes its histogram from the product
                    // (every candidate counted; its budget is not known yet, so
                    // nothing is dropped early)
                    w.hist.ensure(sizeof(uint64_t) * kBuckets);
                    SFN_HIP(hipMemsetAsync(w.hist.get(), 0, sizeof(uint64_t) * kBuckets, w.s));
                    const FusedFilter hist_only{0.0, w.hist.as<uint64_t>(), nullptr};
                    product<V>(w, X, X, nullptr, -1.0, 0.0, 1.0, R, nullptr, &w.rs1, sym, false,
                               &hist_only);
                } else {
                    product<V>(w, X, X, nullptr, -1.0, 0.0, 1.0, R, nullptr, &w.rs1, sym);
                }
                e = std::sqrt(w.sum_rows(w.rs1, n));
            } catch (const Error &err) {
                if (err.status != SIGN_ENOMEM || !p.filter_y || sym) throw;
                w.note("ns k=%d: out of device memory forming the residual; this and the "
                       "next steps in two passes", k);
                two_pass = true;
                w.low_memory = true;
                release_dead();
                R.release_entries();
                residual_two_pass = true;
                residual_first_pass();
            }
        }
        es.push_back(e);
        sign_iter_stats it{};
        it.e = e; it.xfro = xf; it.nnz_x = X.nnz; it.nnz_r = e_bound ? nnz_cert : R.nnz;
        it.fp32 = p.fp32;
        it.e_bound = e_bound;
        out.iters = k - 1; out.e = e; out.xfro = xf;
        const bool conv = (p.stop_rule == 1) ? (d_prev < p.tol) : (e <= p.tol);
        bool stop = conv;
        if (conv) out.status = SIGN_OK;
        if (!stop) {
            if (!std::isfinite(e)) { out.status = SIGN_EDIVERGED; stop = true; }
            else if (k >= 2) {
                const double ep = es[k - 2];
                n_up = (e > ep && e > 1.0) ? n_up + 1 : 0;
                n_flat = (e < 1e-8 && e > 0.5 * ep) ? n_flat + 1 : 0;
                if (n_up >= 3) { out.status = SIGN_EDIVERGED; stop = true; }
                else if (n_flat >= 2) { out.status = SIGN_OK; out.stagnated = 1; stop = true; }
            }
            if (!stop && k - 1 >= p.max_iter) { out.status = SIGN_ENOCONV; stop = true; }
        }
        if (stop) {
            it.ms = 1e3 * (now_s() - t0);
            trace.push_back(it);
            w.report("ns", k, it);
            break;
        }
        const double tau = nsf_budget(e, xf, p.tol, p.c_fixed, p.switch_res);
        if (residual_two_pass) {
            // the cut from the first pass's histogram; the second pass stores the
            // entries of the buckets from one below it: its sums may round apart
            // from the first pass's by the order of the LDS additions, and an entry
            // on a bucket edge must not slip below the cut
            const int bstar = select_cut(w, n, tau);
            w.note("ns k=%d: residual in two passes, %lld entries, cut at bucket %d", k,
                   (long long)R.nnz, bstar);
            const FusedFilter keep{tau, nullptr, nullptr, std::max(bstar - 1, 0)};
            product_rows<V>(w, X, X, nullptr, -1.0, 0.0, 1.0, R, nullptr, nullptr, LowerRows{},
                            &keep);
        } else if (p.filter_y) {
            try {
                filter<V, V>(w, R, tau, Xn, nullptr, nullptr, 0, true);
            } catch (const Error &err) {
                if (err.status != SIGN_ENOMEM) throw;
                // the kept residual does not fit beside the unfiltered one: once
                // more with the dead matrices and the staging released, and the
                // next steps in two passes
                w.note("ns k=%d: out of device memory filtering the residual; the next "
                       "steps in two passes", k);
                two_pass = true;
                w.low_memory = true;
                release_dead();
                filter<V, V>(w, R, tau, Xn, nullptr, nullptr, 0, true);
            }
            std::swap(R, Xn);
        }
        // Xbar_{k+1} = X^_k + 1/2 X^_k R^_k  (= 1/2 X^_k (3I - X^_k^2))
        // (symmetric: the lower triangle of Xbar is filtered, with entries below
        // the diagonal counted twice, and the survivors are mirrored)
        // (fused: the filter's histogram comes out of the product, and entries no
        // cut can keep are never stored)
        w.hist.ensure(sizeof(uint64_t) * kBuckets);
        w.rs5.ensure(sizeof(double) * n);
        SFN_HIP(hipMemsetAsync(w.hist.get(), 0, sizeof(uint64_t) * kBuckets, w.s));
        SFN_HIP(hipMemsetAsync(w.rs5.get(), 0, sizeof(double) * n, w.s));  // rows with no output
        const FusedFilter fuse{tau, w.hist.as<uint64_t>(), w.rs5.as<double>()};
        int bstar = 0;
        int64_t nbar = 0;
        // under memory pressure Xbar is never stored either: a first pass forms its
        // histogram and ||Xbar - X^_k||, the cut follows, and a second pass stores
        // X^_{k+1} directly (from one bucket below the cut, as for the residual),
        // with the sums of squares kept and dropped per row
        auto update_two_pass = [&]() {
            release_dead();  // candidates of a one-pass step, a swapped-out residual
            SFN_HIP(hipMemsetAsync(w.hist.get(), 0, sizeof(uint64_t) * kBuckets, w.s));
            const FusedFilter hist_only{0.0, w.hist.as<uint64_t>(), nullptr};
            product_rows<V>(w, X, R, &X, 0.5, 1.0, 0.0, Xn, &w.rs2, nullptr, LowerRows{},
                            &hist_only, true);
            bstar = select_cut(w, n, tau);
            w.rb.ensure(sizeof(int64_t) * 64);
            launch_hist_total(w.hist.as<uint64_t>(), w.rb.as<int64_t>(), w.s);
            nbar = read_scalar(w.rb.as<int64_t>(), w.s);
            w.rs3.ensure(sizeof(double) * n);
            w.rs4.ensure(sizeof(double) * n);
            SFN_HIP(hipMemsetAsync(w.rs4.get(), 0, sizeof(double) * n, w.s));  // rows with no output
            const FusedFilter keep{tau, nullptr, w.rs4.as<double>(), std::max(bstar - 1, 0)};
            product_rows<V>(w, X, R, &X, 0.5, 1.0, 0.0, Xn, nullptr, &w.rs3, LowerRows{}, &keep);
            // the step's inputs and the products' staging go back to the pool
            // (X^_k is not read again)
            R.release_entries();
            X.release_entries();
            w.stage_col.reset();
            w.stage_val.reset();
        };
        if (two_pass && !sym) {
            update_two_pass();
        } else {
            try {
                product<V>(w, X, R, &X, 0.5, 1.0, 0.0, Xb, &w.rs2, nullptr, sym, sym, &fuse);
                // X^_{k+1} = Xbar_{k+1} - F_{k+1}
                // (nbar: entries of the full Xbar -- the histogram counts every
                // candidate, twice below the diagonal of a symmetric product)
                if (sym) {
                    bstar = filter<V, V>(w, Xb, tau, Xl, &w.rs3, &w.rs4, 1, true, &nbar);
                    symmetrize<V>(w, Xl, Xn);
                } else {
                    bstar = filter<V, V>(w, Xb, tau, Xn, &w.rs3, &w.rs4, 0, true, &nbar);
                }
            } catch (const Error &err) {
                if (err.status != SIGN_ENOMEM || !p.filter_y || sym) throw;
                w.note("ns k=%d: out of device memory forming the update; this and the next "
                       "steps in two passes", k);
                two_pass = true;
                w.low_memory = true;
                SFN_HIP(hipMemsetAsync(w.rs5.get(), 0, sizeof(double) * n, w.s));
                update_two_pass();
            }
        }
        const std::vector<double> sums = w.sum_rows_many({&w.rs2, &w.rs5, &w.rs3, &w.rs4}, n);
        const double d = std::sqrt(sums[0]);
        const double xf_new = std::sqrt(sums[2]);
        const double ff = std::sqrt(sums[3] + sums[1]);
        it.d = d; it.tau = tau; it.ffro = ff; it.bstar = bstar; it.nnz_bar = nbar;
        it.ms = 1e3 * (now_s() - t0);
        trace.push_back(it);
        w.report("ns", k, it);
        std::swap(X, Xn);
        if (two_pass) {
            // the previous iterate and any candidates left from one-pass steps
            Xb.release_entries();
            Xn.release_entries();
        }
        xf = xf_new;
        d_prev = d;
        ff_prev = ff;
        out.d = d;
    }
    return out;
}

void transpose(Workspace &w, const DMat<double> &X, DMat<double> &Out) {
    const int64_t n = X.n;
    hipStream_t s = w.s;
    Out.ensure_rows(n);
    Out.ensure_entries(X.nnz);
    w.icnt.ensure(sizeof(int32_t) * std::max<int64_t>(n, 1));
    w.tmp.ensure(sizeof(int64_t) * scan_tmp_elems(n));
    w.symtcol.ensure(sizeof(int32_t) * (size_t)std::max<int64_t>(X.nnz, 1));
    w.symtval.ensure(sizeof(double) * (size_t)std::max<int64_t>(X.nnz, 1));
    SFN_HIP(hipMemsetAsync(w.icnt.get(), 0, sizeof(int32_t) * n, s));
    launch_transpose_count<double>(X.view(), w.icnt.as<int32_t>(), s);
    launch_exclusive_scan_i32(w.icnt.as<int32_t>(), n, Out.begp(), w.tmp.as<int64_t>(), 0, s);
    SFN_HIP(hipMemcpyAsync(Out.lenp(), w.icnt.get(), sizeof(int32_t) * n, hipMemcpyDeviceToDevice,
                           s));
    SFN_HIP(hipMemsetAsync(w.icnt.get(), 0, sizeof(int32_t) * n, s));
    // entries of column j of X, unordered, then ranked by row into row j of Out
    launch_transpose_fill<double>(X.view(), Out.begp(), w.icnt.as<int32_t>(),
                                  w.symtcol.as<int32_t>(), w.symtval.as<double>(), s);
    launch_sym_rank<double>(n, Out.begp(), nullptr, Out.begp(), Out.lenp(),
                            w.symtcol.as<int32_t>(), w.symtval.as<double>(), Out.colp(),
                            Out.valp(), s);
    Out.nnz = X.nnz;
}


LoopOut nmf_loop(Workspace &w, DMat<double> &X, const LoopParams &p,
                 std::vector<sign_iter_stats> &trace, int &inner_steps) {
    const int64_t n = X.n;
    DMat<double> I, R, Z, T, T2, Zb, Xb, Xn, D;
    for (DMat<double> *m : {&I, &R, &Z, &T, &T2, &Zb, &Xb, &Xn, &D}) m->bind(w.al);
    I.ensure_rows(n);
    I.ensure_entries(n);
    launch_identity(n, I.begp(), I.lenp(), I.colp(), I.valp(), w.s);
    I.nnz = n;
    LoopOut out;
    row_sumsq(w, X, w.rs3);
    double xf = std::sqrt(w.sum_rows(w.rs3, n));
    int n_up = 0, n_flat = 0;
    bool have_z = false;
    std::vector<double> es;
    const double target = 0.1 * p.tol;
    const double tau_z = p.c_fixed * p.tol;
    for (int k = 1;; ++k) {
        const double t0 = now_s();
        // residual R^_k = I - X^_k^2 (Alg. 3.1.1 steps 1 and 5)
        product<double>(w, X, X, nullptr, -1.0, 0.0, 1.0, R, nullptr, &w.rs1);
        const double e = std::sqrt(w.sum_rows(w.rs1, n));
        es.push_back(e);
        sign_iter_stats it{};
        it.e = e; it.xfro = xf; it.nnz_x = X.nnz; it.nnz_r = R.nnz;
        out.iters = k - 1; out.e = e; out.xfro = xf;
        bool stop = e <= p.tol;
        if (stop) out.status = SIGN_OK;
        if (!stop) {
            if (!std::isfinite(e)) { out.status = SIGN_EDIVERGED; stop = true; }
            else if (k >= 2) {
                const double ep = es[k - 2];
                n_up = (e > ep && e > 1.0) ? n_up + 1 : 0;
                n_flat = (e < 1e-8 && e > 0.5 * ep) ? n_flat + 1 : 0;
                if (n_up >= 3) { out.status = SIGN_EDIVERGED; stop = true; }
                else if (n_flat >= 2) { out.status = SIGN_OK; out.stagnated = 1; stop = true; }
            }
            if (!stop && k - 1 >= p.max_iter) { out.status = SIGN_ENOCONV; stop = true; }
        }
        if (stop) {
            it.ms = 1e3 * (now_s() - t0);
            trace.push_back(it);
            w.report("newton", k, it);
            break;
        }
        // Z ~ X^_k^{-1} by filtered Newton-Schulz inversion Z <- Z + Z (I - X^_k Z).
        // Its residual T = I - X^_k Z squares every step, so it converges from any
        // start with ||T_0|| < 1 in a submultiplicative norm; a start is taken when
        // ||T_0||_inf < 1/2, in this order of preference:
        //  - X^_k itself (T_0 = R^_k, already formed): near convergence X^-1 ~ X;
        //  - the previous inverse Z or 2Z: for an eigenvalue x of the previous
        //    iterate the new one is (x + 1/x)/2, and I - X^_k Z and I - 2 X^_k Z have
        //    eigenvalues (1 - 1/x^2)/2 and -1/x^2, so 2Z is the better start while
        //    |x| > sqrt(3) (the early steps from an unscaled A), Z after;
        //  - X^T / (||X||_1 ||X||_inf), which always converges.
        double r = std::numeric_limits<double>::infinity();
        bool started = false;
        if (inf_norm(w, R) < 0.5) {
            copy_mat(w, X, Z);
            std::swap(T, R);
            r = e;
            started = true;
        } else if (have_z) {
            product<double>(w, X, Z, nullptr, -1.0, 0.0, 1.0, T, nullptr, &w.rs1);
            const double r1 = std::sqrt(w.sum_rows(w.rs1, n));
            const double n1 = inf_norm(w, T);
            // I - 2 X^_k Z = 2T - I
            product<double>(w, I, T, nullptr, 2.0, 0.0, -1.0, T2, nullptr, &w.rs2);
            const double n2 = inf_norm(w, T2);
            if (n2 < n1 && n2 < 0.5) {
                launch_scale_copy<double, double>(Z.valp(), Z.valp(), Z.nnz, 2.0, w.s);
                std::swap(T, T2);
                r = std::sqrt(w.sum_rows(w.rs2, n));
                started = true;
            } else if (n1 < 0.5) {
                r = r1;
                started = true;
            }
        }
        if (!started) {
            // Z_0 = X^T / (||X||_1 ||X||_inf): ||I - X Z_0||_2 < 1 for nonsingular X
            const double sc = norm_one_inf(w, X);
            transpose(w, X, Z);
            launch_scale_copy<double, double>(Z.valp(), Z.valp(), Z.nnz, 1.0 / sc, w.s);
            product<double>(w, X, Z, nullptr, -1.0, 0.0, 1.0, T, nullptr, &w.rs1);
            r = std::sqrt(w.sum_rows(w.rs1, n));
        }
        have_z = true;
        int steps = 0;
        double r_prev = std::numeric_limits<double>::infinity();
        while (r > target && steps < 200 && !(r < 1e-8 && r > 0.5 * r_prev)) {
            r_prev = r;
            product<double>(w, Z, T, &Z, 1.0, 1.0, 0.0, Zb, nullptr, nullptr);
            filter<double, double>(w, Zb, tau_z, Z, nullptr, nullptr);
            product<double>(w, X, Z, nullptr, -1.0, 0.0, 1.0, T, nullptr, &w.rs1);
            r = std::sqrt(w.sum_rows(w.rs1, n));
            ++steps;
            if (!std::isfinite(r)) break;
        }
        inner_steps += steps;
        have_z = true;
        w.note("newton k=%d: %d inverse steps to %.3e", k, steps, r);
        row_sumsq(w, Z, w.rs2);
        const double zf = std::sqrt(w.sum_rows(w.rs2, n));
        // Xbar_{k+1} = 1/2 (X^_k + X^_k^{-1})  (Alg. 3.1.1 step 3)
        product<double>(w, X, I, &Z, 0.5, 0.5, 0.0, Xb, nullptr, nullptr);
        // X^_{k+1} = Xbar_{k+1} - F_{k+1}, budget eq. 1.13 / fixed (step 4)
        const double tau = nmf_budget(e, xf, zf, p.tol, p.c_fixed, p.switch_res);
        const int bstar = filter<double, double>(w, Xb, tau, Xn, &w.rs3, &w.rs4);
        const double xf_new = std::sqrt(w.sum_rows(w.rs3, n));
        const double ff = std::sqrt(w.sum_rows(w.rs4, n));
        product<double>(w, Xn, I, &X, 1.0, -1.0, 0.0, D, nullptr, &w.rs1);
        const double d = std::sqrt(w.sum_rows(w.rs1, n));
        it.d = d; it.tau = tau; it.ffro = ff; it.nnz_bar = Xb.nnz; it.bstar = bstar;
        it.ms = 1e3 * (now_s() - t0);
        trace.push_back(it);
        w.report("newton", k, it);
        std::swap(X, Xn);
        xf = xf_new;
        out.d = d;
    }
    return out;
}

template void product<double>(Workspace &, const DMat<double> &, const DMat<double> &,
                              const DMat<double> *, double, double, double, DMat<double> &,
                              DevBuf *, DevBuf *, bool, bool, const FusedFilter *,
                              const uint8_t *);
template void product<float>(Workspace &, const DMat<float> &, const DMat<float> &,
                             const DMat<float> *, double, double, double, DMat<float> &, DevBuf *,
                             DevBuf *, bool, bool, const FusedFilter *, const uint8_t *);
template int filter<double, double>(Workspace &, const DMat<double> &, double, DMat<double> &,
                                    DevBuf *, DevBuf *, int, bool, int64_t *);
template int filter<float, float>(Workspace &, const DMat<float> &, double, DMat<float> &,
                                  DevBuf *, DevBuf *, int, bool, int64_t *);
template int filter<float, double>(Workspace &, const DMat<float> &, double, DMat<double> &,
                                   DevBuf *, DevBuf *, int, bool, int64_t *);
template int filter<double, float>(Workspace &, const DMat<double> &, double, DMat<float> &,
                                   DevBuf *, DevBuf *, int, bool, int64_t *);
template void row_sumsq<double>(Workspace &, const DMat<double> &, DevBuf &);
template void row_sumsq<float>(Workspace &, const DMat<float> &, DevBuf &);
template LoopOut nsf_loop<double>(Workspace &, DMat<double> &, const LoopParams &,
                                  std::vector<sign_iter_stats> &);
template LoopOut nsf_loop<float>(Workspace &, DMat<float> &, const LoopParams &,
                                 std::vector<sign_iter_stats> &);

}  // namespace sfn
