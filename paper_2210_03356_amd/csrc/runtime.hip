// Device memory for libsignfn: caching pool, allocator hooks, grow-only buffers.
#include <algorithm>

#include "runtime.hpp"

namespace sfn {

namespace {
thread_local std::string g_last_error;

size_t round_bytes(size_t b) {
    if (b == 0) b = 1;
    const size_t big = size_t(2) << 20;
    if (b >= big) return (b + big - 1) / big * big;
    return (b + 255) / 256 * 256;
}
}  // namespace

void set_last_error(const std::string &m) { g_last_error = m; }
const char *last_error() { return g_last_error.c_str(); }

Pool &Pool::instance() {
    static Pool *p = new Pool();  // never destroyed: blocks live until process exit
    return *p;
}

void *Pool::get(size_t bytes) {
    const size_t b = round_bytes(bytes);
    {
        std::lock_guard<std::mutex> lk(mu_);
        auto it = free_.lower_bound(b);
        if (it != free_.end() && it->first <= 2 * b) {
            void *p = it->second;
            cached_ -= it->first;
            free_.erase(it);
            return p;
        }
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, b);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        trim();
        e = hipMalloc(&p, b);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            throw Error(SIGN_ENOMEM, "device allocation of " + std::to_string(b) + " bytes failed");
        }
    }
    std::lock_guard<std::mutex> lk(mu_);
    size_[p] = b;
    return p;
}

void Pool::put(void *p) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(mu_);
    auto it = size_.find(p);
    if (it == size_.end()) return;
    free_.emplace(it->second, p);
    cached_ += it->second;
}

void Pool::trim() {
    std::lock_guard<std::mutex> lk(mu_);
    for (auto &kv : free_) {
        (void)hipFree(kv.second);
        size_.erase(kv.second);
    }
    free_.clear();
    cached_ = 0;
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
    if (bytes <= bytes_ && p_) return;
    // grow geometrically so repeated growth stays cheap
    size_t want = std::max(bytes, bytes_ + bytes_ / 2);
    void *np = al_->get(want);
    if (p_ && keep_bytes) {
        SFN_HIP(hipMemcpyAsync(np, p_, std::min(keep_bytes, bytes_), hipMemcpyDeviceToDevice,
                               al_->stream));
        SFN_HIP(hipStreamSynchronize(al_->stream));
    } else if (p_) {
        SFN_HIP(hipStreamSynchronize(al_->stream));
    }
    if (p_) al_->put(p_);
    p_ = np;
    bytes_ = want;
}

void DevBuf::reset() {
    if (p_ && al_) al_->put(p_);
    p_ = nullptr;
    bytes_ = 0;
}

}  // namespace sfn
