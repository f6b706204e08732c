// sign_filter_noalloc: the norm-budget filter of sign_filter (element threshold
// of Section 3.1 chosen from a bucket histogram, drop, compaction) for callers
// that cannot allocate device memory.  The caller passes the input and the
// output buffers; every other buffer the kernels use (histogram, cut bucket,
// row lengths, per-row dropped sums of squares, scan partials, small scalars)
// lives in `scratch`, a file-scope device array of fixed size.
//
// Each device the library runs on holds its own copy of `scratch` until the
// process ends.  Host code never uses the array's name as an address: the
// device address is looked up once per device with hipGetSymbolAddress and
// kept in scratch_ptr[device].  Calls on one device share that memory, so
// calls that overlap on one device (several host threads, or several streams
// without ordering between them) race and must be serialised by the caller.
#include <cmath>
#include <mutex>

#include "driver.hpp"

using namespace sfn;

namespace {

constexpr int64_t kMaxRows = SIGN_NOALLOC_MAX_ROWS;
constexpr int64_t kScanTmp = (kMaxRows + 2047) / 2048 + 2;  // >= scan_tmp_elems(kMaxRows)

// Layout of the scratch array (byte offsets; every part 256-byte aligned).
constexpr size_t kOffHist = 0;                                       // uint64 [kBuckets]
constexpr size_t kOffSmall = kOffHist + sizeof(uint64_t) * kBuckets; // 256 B of scalars
constexpr size_t kOffLenIn = kOffSmall + 256;                        // int32  [kMaxRows]
constexpr size_t kOffLenOut = kOffLenIn + sizeof(int32_t) * kMaxRows; // int32 [kMaxRows]
constexpr size_t kOffSqDrop = kOffLenOut + sizeof(int32_t) * kMaxRows; // double [kMaxRows]
constexpr size_t kOffScan = kOffSqDrop + sizeof(double) * kMaxRows;   // int64 [kScanTmp]
constexpr size_t kScratchBytes = kOffScan + sizeof(int64_t) * ((kScanTmp + 31) / 32 * 32);
static_assert(kOffLenIn % 256 == 0 && kOffLenOut % 256 == 0 && kOffSqDrop % 256 == 0 &&
                  kOffScan % 256 == 0,
              "scratch parts are 256-byte aligned");

// Scalars inside the 256-byte small part.
struct Small {
    int64_t seg[2];   // one segment: rows [0, n)
    double tau;       // the budget
    double dropped;   // sum of squares of the dropped entries
    int bstar;        // cut bucket
    int flag;         // validation flags
};
static_assert(sizeof(Small) <= 256, "small part");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
unsigned char *scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first
// call on that device, with the device current).
unsigned char *scratch_on_current_device() {
    int dev = 0;
    SFN_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) throw Error(SIGN_EDEVICE, "device index out of range");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            throw Error(SIGN_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                          hipGetErrorString(e));
        scratch_ptr[dev] = (unsigned char *)p;
    }
    return scratch_ptr[dev];
}

// Clears the histogram and writes the scalars (a kernel rather than memset and
// host copies, so that the call records only kernel launches before its first
// read-back).
__global__ void k_noalloc_init(uint64_t *hist, Small *sm, int64_t n, double tau) {
    for (int b = threadIdx.x; b < kBuckets; b += blockDim.x) hist[b] = 0ull;
    if (threadIdx.x == 0) {
        sm->seg[0] = 0;
        sm->seg[1] = n;
        sm->tau = tau;
        sm->dropped = 0.0;
        sm->bstar = 0;
        sm->flag = 0;
    }
}

template <typename V>
int filter_into(const sign_csr *A, double tau, hipStream_t s, sign_csr *out, int64_t out_cap,
                int *bstar_out, double *dropped_out) {
    const int64_t n = A->n;
    unsigned char *base = scratch_on_current_device();
    uint64_t *hist = (uint64_t *)(base + kOffHist);
    Small *sm = (Small *)(base + kOffSmall);
    int32_t *len_in = (int32_t *)(base + kOffLenIn);
    int32_t *len_out = (int32_t *)(base + kOffLenOut);
    double *sq_drop = (double *)(base + kOffSqDrop);
    int64_t *scan_tmp = (int64_t *)(base + kOffScan);
    if (scan_tmp_elems(n) > kScanTmp) throw Error(SIGN_EINVAL, "scan scratch too small");

    k_noalloc_init<<<1, 256, 0, s>>>(hist, sm, n, tau);
    launch_validate(A->row_ptr, A->col, A->val, A->val_f32, n, A->nnz, &sm->flag, s);
    int flag = 0;
    SFN_HIP(hipMemcpyAsync(&flag, &sm->flag, sizeof(int), hipMemcpyDeviceToHost, s));
    SFN_HIP(hipStreamSynchronize(s));
    if (flag) {
        std::string m = "malformed CSR:";
        if (flag & 1) m += " row_ptr";
        if (flag & 2) m += " column out of range";
        if (flag & 4) m += " columns not strictly ascending";
        if (flag & 8) m += " non-finite value";
        throw Error(SIGN_EINVAL, m);
    }

    // the input is read in place: rows start at row_ptr, lengths from its differences
    launch_row_len(A->row_ptr, n, len_in, s);
    MatView<V> X;
    X.n = n;
    X.beg = A->row_ptr;
    X.len = len_in;
    X.col = A->col;
    X.val = (const V *)A->val;
    LowerRows none;
    launch_histogram<V>(X, sm->seg, 1, n, hist, none, s);
    launch_select(hist, &sm->tau, 1, &sm->bstar, s);
    launch_count_keep<V>(X, nullptr, &sm->bstar, len_out, nullptr, sq_drop, none, s);
    launch_exclusive_scan_i32(len_out, n, out->row_ptr, scan_tmp, 0, s);
    launch_seg_sum(sq_drop, sm->seg, 1, &sm->dropped, s);
    int64_t total = 0;
    Small h;
    SFN_HIP(hipMemcpyAsync(&total, out->row_ptr + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    SFN_HIP(hipMemcpyAsync(&h, sm, sizeof(Small), hipMemcpyDeviceToHost, s));
    SFN_HIP(hipStreamSynchronize(s));
    if (total > out_cap)
        throw Error(SIGN_ENOMEM, "output capacity " + std::to_string(out_cap) + " < " +
                                     std::to_string(total) + " kept entries");
    if (total > 0 && (!out->col || !out->val))
        throw Error(SIGN_EINVAL, "NULL output column or value array");
    launch_scatter_keep<V, double>(X, nullptr, &sm->bstar, out->row_ptr, out->col,
                                   (double *)out->val, s);
    SFN_HIP(hipStreamSynchronize(s));
    out->n = n;
    out->nnz = total;
    out->val_f32 = 0;
    if (bstar_out) *bstar_out = h.bstar;
    if (dropped_out) *dropped_out = std::sqrt(h.dropped);
    return SIGN_OK;
}

}  // namespace

extern "C" int sign_filter_noalloc(const sign_csr *A, double tau, void *hip_stream,
                                   sign_csr *out, int64_t out_capacity, int *bstar,
                                   double *dropped_fro) {
    try {
        set_last_error("");
        if (!A || !out) throw Error(SIGN_EINVAL, "NULL argument");
        if (A->n <= 0) throw Error(SIGN_EINVAL, "n must be > 0");
        if (A->n > kMaxRows)
            throw Error(SIGN_EINVAL, "n = " + std::to_string(A->n) +
                                         " exceeds the row limit of sign_filter_noalloc (" +
                                         std::to_string(kMaxRows) + ")");
        if (A->nnz < 0) throw Error(SIGN_EINVAL, "nnz must be >= 0");
        if (!A->row_ptr || (A->nnz > 0 && (!A->col || !A->val)))
            throw Error(SIGN_EINVAL, "NULL array in matrix");
        if (A->val_f32 != 0 && A->val_f32 != 1) throw Error(SIGN_EINVAL, "val_f32 must be 0 or 1");
        if (!out->row_ptr) throw Error(SIGN_EINVAL, "NULL output row_ptr");
        if (out_capacity < 0) throw Error(SIGN_EINVAL, "out_capacity must be >= 0");
        if (!(tau >= 0.0) || !std::isfinite(tau)) throw Error(SIGN_EINVAL, "tau must be >= 0");
        hipStream_t s = (hipStream_t)hip_stream;
        return A->val_f32 ? filter_into<float>(A, tau, s, out, out_capacity, bstar, dropped_fro)
                          : filter_into<double>(A, tau, s, out, out_capacity, bstar, dropped_fro);
    } catch (const Error &e) {
        set_last_error(e.what());
        return e.status;
    } catch (const std::exception &e) {
        set_last_error(e.what());
        return SIGN_EDEVICE;
    }
}
