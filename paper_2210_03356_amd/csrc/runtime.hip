// Device memory for libsignfn: caching pool, allocator hooks, grow-only buffers.
#include <algorithm>
#include <iterator>

#include "runtime.hpp"

namespace sfn {

namespace {
thread_local std::string g_last_error;

}  // namespace

void set_last_error(const std::string &m) { g_last_error = m; }
const char *last_error() { return g_last_error.c_str(); }

Pool &Pool::instance() {
    static Pool *p = new Pool();  // never destroyed: segments live until process exit
    return *p;
}

namespace {
constexpr size_t kAlign = 512;                     // sub-allocation granularity
constexpr size_t kMinSplit = size_t(1) << 20;      // smallest remainder kept as a block
constexpr size_t kSegment = size_t(2) << 30;       // segment size for small requests
constexpr size_t kHuge = size_t(8) << 30;          // requests that get a segment of their own
size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
}  // namespace

void Pool::insert_free(Block *b) {
    b->free = true;
    free_.emplace(b->size, b);
    cached_ += b->size;
}

void Pool::erase_free(Block *b) {
    auto range = free_.equal_range(b->size);
    for (auto it = range.first; it != range.second; ++it)
        if (it->second == b) {
            free_.erase(it);
            break;
        }
    cached_ -= b->size;
    b->free = false;
}

// Free whole segments with no used block (largest first) until `need` bytes
// have been returned, or none is left.  Caller holds mu_.
bool Pool::release_free_segments(size_t need) {
    size_t got = 0;
    for (;;) {
        int best = -1;
        for (int sgi = 0; sgi < (int)segs_.size(); ++sgi) {
            Block *h = seg_head_[sgi];
            if (!segs_[sgi].first || !h || !h->free || h->next) continue;  // not a single free block
            if (best < 0 || segs_[sgi].second > segs_[best].second) best = sgi;
        }
        if (best < 0) return got > 0;
        Block *h = seg_head_[best];
        erase_free(h);
        (void)hipFree(segs_[best].first);
        got += segs_[best].second;
        segs_[best].first = nullptr;
        seg_head_[best] = nullptr;
        delete h;
        if (got >= need) return true;
    }
}

void *Pool::get(size_t bytes) {
    const size_t b = align_up(bytes ? bytes : 1, kAlign);
    std::lock_guard<std::mutex> lk(mu_);
    auto it = free_.lower_bound(b);
    if (b >= kHuge && it != free_.end() && it->second->size > b + b / 4) {
        // a huge request that would split a much larger cached block: take a
        // segment of its own while HIP has room, so that the block's tail is
        // not stranded next to a live allocation (a segment is returned only
        // when wholly free).  Smaller requests reuse cached blocks: a fresh
        // hipMalloc for each would cost more than the memory it saves.
        char *p = nullptr;
        if (hipMalloc((void **)&p, align_up(b, size_t(2) << 20)) == hipSuccess) {
            const size_t want = align_up(b, size_t(2) << 20);
            Block *blk = new Block{p, want, false, nullptr, nullptr, (int)segs_.size()};
            segs_.push_back({p, want});
            seg_head_.push_back(blk);
            insert_free(blk);
            it = free_.lower_bound(b);
            while (it->second != blk) ++it;
        } else {
            (void)hipGetLastError();
        }
    }
    if (it == free_.end()) {
        // a new segment: exactly the request when large, else a shared segment
        const size_t want = b >= kSegment ? align_up(b, size_t(2) << 20) : kSegment;
        char *p = nullptr;
        hipError_t e = hipMalloc((void **)&p, want);
        while (e != hipSuccess) {
            (void)hipGetLastError();
            if (!release_free_segments(want)) break;
            e = hipMalloc((void **)&p, want);
        }
        if (e != hipSuccess) {
            (void)hipGetLastError();
            size_t fr = 0, tot = 0;
            if (hipMemGetInfo(&fr, &tot) != hipSuccess) (void)hipGetLastError();
            size_t used = 0;
            for (const auto &u : used_) used += u.second->size;
            throw Error(SIGN_ENOMEM, "device allocation of " + std::to_string(want) +
                                         " bytes failed (pool: " + std::to_string(used) +
                                         " bytes in use, " + std::to_string(cached_) +
                                         " cached; device: " + std::to_string(fr) + " of " +
                                         std::to_string(tot) + " free)");
        }
        Block *blk = new Block{p, want, false, nullptr, nullptr, (int)segs_.size()};
        segs_.push_back({p, want});
        seg_head_.push_back(blk);
        insert_free(blk);
        it = free_.lower_bound(b);
    }
    Block *blk = it->second;
    erase_free(blk);
    if (blk->size - b >= kMinSplit) {  // split off the tail as a free block
        Block *rest = new Block{blk->ptr + b, blk->size - b, false, blk, blk->next, blk->seg};
        if (blk->next) blk->next->prev = rest;
        blk->next = rest;
        blk->size = b;
        insert_free(rest);
    }
    used_[blk->ptr] = blk;
    return blk->ptr;
}

void Pool::put(void *p) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(mu_);
    auto u = used_.find(p);
    if (u == used_.end()) return;
    Block *blk = u->second;
    used_.erase(u);
    // coalesce with free neighbours
    if (blk->next && blk->next->free) {
        Block *n = blk->next;
        erase_free(n);
        blk->size += n->size;
        blk->next = n->next;
        if (n->next) n->next->prev = blk;
        delete n;
    }
    if (blk->prev && blk->prev->free) {
        Block *pv = blk->prev;
        erase_free(pv);
        pv->size += blk->size;
        pv->next = blk->next;
        if (blk->next) blk->next->prev = pv;
        delete blk;
        blk = pv;
    }
    insert_free(blk);
}

void Pool::trim() {
    std::lock_guard<std::mutex> lk(mu_);
    release_free_segments(~size_t(0));
}

size_t Pool::used_bytes() {
    std::lock_guard<std::mutex> lk(mu_);
    size_t used = 0;
    for (const auto &u : used_) used += u.second->size;
    return used;
}

size_t Pool::cached_bytes() {
    std::lock_guard<std::mutex> lk(mu_);
    return cached_;
}

void *Allocator::get(size_t bytes) {
    if (alloc) {
        void *p = alloc(bytes, (void *)stream, ctx);
        if (!p) throw Error(SIGN_ENOMEM, "allocator hook returned NULL for " +
                                             std::to_string(bytes) + " bytes");
        return p;
    }
    return Pool::instance().get(bytes);
}

void Allocator::put(void *p) {
    if (!p) return;
    if (release) release(p, (void *)stream, ctx);
    else Pool::instance().put(p);
}

DevBuf &DevBuf::operator=(DevBuf &&o) noexcept {
    if (this != &o) {
        reset();
        al_ = o.al_;
        p_ = o.p_;
        bytes_ = o.bytes_;
        o.p_ = nullptr;
        o.bytes_ = 0;
    }
    return *this;
}

void DevBuf::ensure(size_t bytes, size_t keep_bytes) {
    // a large buffer whose contents are not kept and that would be less than
    // half used is given back and allocated anew at the new size: iterates
    // trade buffers (swaps) and would otherwise each keep the largest size any
    // of them ever had
    constexpr size_t kShrinkFrom = size_t(1) << 30;
    if (p_ && !keep_bytes && bytes_ >= kShrinkFrom && bytes < bytes_ / 2) {
        SFN_HIP(hipStreamSynchronize(al_->stream));
        al_->put(p_);
        p_ = nullptr;
        bytes_ = 0;
    }
    if (bytes <= bytes_ && p_) return;
    // grow geometrically so repeated growth stays cheap, by at most a quarter
    // beyond the request (these buffers reach tens of GB)
    const size_t want = std::max(bytes, std::min(bytes_ + bytes_ / 2, bytes + bytes / 4));
    if (p_ && !keep_bytes) {
        // nothing to keep: release the old block first, so both never coexist
        SFN_HIP(hipStreamSynchronize(al_->stream));
        al_->put(p_);
        p_ = nullptr;
        bytes_ = 0;
    }
    void *np = al_->get(want);
    if (p_) {
        SFN_HIP(hipMemcpyAsync(np, p_, std::min(keep_bytes, bytes_), hipMemcpyDeviceToDevice,
                               al_->stream));
        SFN_HIP(hipStreamSynchronize(al_->stream));
        al_->put(p_);
    }
    p_ = np;
    bytes_ = want;
}

void DevBuf::reset() {
    if (p_ && al_) al_->put(p_);
    p_ = nullptr;
    bytes_ = 0;
}

}  // namespace sfn
