// Host runtime of libsignfn: errors, device memory, device matrices.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstring>
#include <map>
#include <mutex>
#include <stdexcept>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/signfn.h"
#include "kernels.hpp"

namespace sfn {

// Errors thrown inside the library and turned into a sign_status at the ABI.
struct Error : std::runtime_error {
    int status;
    Error(int st, const std::string &msg) : std::runtime_error(msg), status(st) {}
};

#define SFN_HIP(call)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess)                                                             \
            throw ::sfn::Error(SIGN_EDEVICE, std::string(#call) + ": " +                  \
                                                 hipGetErrorString(e_));                  \
    } while (0)

// Device memory: either the caller's hooks or a process-wide pool.  The pool
// takes large segments from hipMalloc and sub-allocates them best-fit, with
// block splitting and coalescing of free neighbours, so that the growing and
// shrinking matrices of repeated solves are served without further calls to
// hipMalloc/hipFree (each of which maps or unmaps gigabytes).  Blocks handed
// back are idle: every call synchronises its stream before returning its
// workspace.
class Pool {
  public:
    static Pool &instance();
    void *get(size_t bytes);
    void put(void *p);
    void trim();             // return entirely free segments to the driver
    size_t cached_bytes();   // free bytes held in segments
    size_t used_bytes();     // bytes handed out and not yet returned

  private:
    struct Block {
        char *ptr;
        size_t size;
        bool free;
        Block *prev, *next;  // address neighbours within the segment
        int seg;
    };
    void insert_free(Block *b);
    void erase_free(Block *b);
    bool release_free_segments(size_t need);
    std::mutex mu_;
    std::multimap<size_t, Block *> free_;
    std::unordered_map<void *, Block *> used_;
    std::vector<std::pair<char *, size_t>> segs_;  // base, size (nullptr once released)
    std::vector<Block *> seg_head_;
    size_t cached_ = 0;
};

struct Allocator {
    void *(*alloc)(size_t, void *, void *) = nullptr;
    void (*release)(void *, void *, void *) = nullptr;
    void *ctx = nullptr;
    hipStream_t stream = nullptr;
    void *get(size_t bytes);
    void put(void *p);
};

// Grow-only device buffer.
class DevBuf {
  public:
    DevBuf() = default;
    explicit DevBuf(Allocator *a) : al_(a) {}
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept { *this = std::move(o); }
    DevBuf &operator=(DevBuf &&o) noexcept;
    ~DevBuf() { reset(); }
    void bind(Allocator *a) { al_ = a; }
    // ensure at least `bytes`; contents are kept only if keep_bytes > 0 (prefix copied);
    // without keep_bytes, a buffer of 1 GB or more that would be less than half used
    // is reallocated at the new size
    void ensure(size_t bytes, size_t keep_bytes = 0);
    void reset();
    void *get() const { return p_; }
    size_t size() const { return bytes_; }
    template <typename T> T *as() const { return static_cast<T *>(p_); }
    void *release_ownership() { void *p = p_; p_ = nullptr; bytes_ = 0; return p; }

  private:
    Allocator *al_ = nullptr;
    void *p_ = nullptr;
    size_t bytes_ = 0;
};

// Device matrix addressed by (beg, len); compact when beg[i+1] = beg[i] + len[i].
template <typename V>
struct DMat {
    int64_t n = 0;
    int64_t nnz = 0;      // stored entries (compact) / used extent (gapped)
    DevBuf beg, len, col, val;
    void bind(Allocator *a) { beg.bind(a); len.bind(a); col.bind(a); val.bind(a); }
    void ensure_rows(int64_t rows) {
        n = rows;
        beg.ensure(sizeof(int64_t) * (size_t)(rows + 1));
        len.ensure(sizeof(int32_t) * (size_t)(rows > 0 ? rows : 1));
    }
    void ensure_entries(int64_t m, int64_t keep = 0) {
        const size_t mm = (size_t)(m > 0 ? m : 1);
        col.ensure(sizeof(int32_t) * mm, sizeof(int32_t) * (size_t)keep);
        val.ensure(sizeof(V) * mm, sizeof(V) * (size_t)keep);
    }
    int64_t *begp() const { return static_cast<int64_t *>(beg.get()); }
    int32_t *lenp() const { return static_cast<int32_t *>(len.get()); }
    int32_t *colp() const { return static_cast<int32_t *>(col.get()); }
    V *valp() const { return static_cast<V *>(val.get()); }
    MatView<V> view() const {
        MatView<V> v;
        v.n = n;
        v.beg = beg.as<int64_t>();
        v.len = len.as<int32_t>();
        v.col = col.as<int32_t>();
        v.val = val.as<V>();
        return v;
    }
    int64_t capacity() const { return (int64_t)(col.size() / sizeof(int32_t)); }
    // give the entry arrays back (row arrays kept); later work on the stream that
    // reuses the blocks runs after the work that used them
    void release_entries() {
        col.reset();
        val.reset();
        nnz = 0;
    }
};

// Small host<->device helpers (synchronous on the given stream).
template <typename T>
inline T read_scalar(const T *dev, hipStream_t s) {
    T h;
    SFN_HIP(hipMemcpyAsync(&h, dev, sizeof(T), hipMemcpyDeviceToHost, s));
    SFN_HIP(hipStreamSynchronize(s));
    return h;
}
template <typename T>
inline void write_scalar(T *dev, T v, hipStream_t s) {
    SFN_HIP(hipMemcpyAsync(dev, &v, sizeof(T), hipMemcpyHostToDevice, s));
    SFN_HIP(hipStreamSynchronize(s));
}

// Thread-local message of the last failing ABI call.
void set_last_error(const std::string &m);
const char *last_error();

}  // namespace sfn

// The opaque ABI result.
struct sign_result {
    sfn::Allocator al;
    int64_t n = 0, nnz = 0;
    int val_f32 = 0;
    sfn::DevBuf rp, col, val;
    sign_stats stats{};
    std::vector<sign_iter_stats> trace;
};
