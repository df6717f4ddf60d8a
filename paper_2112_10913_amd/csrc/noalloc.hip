// The ordering phase (Section IV, Algorithm 3) for callers that cannot
// allocate device memory: citron_order_noalloc validates a device CSR and
// writes the degree-ordered DAG into the caller's buffers, with every piece
// of working memory -- the out-degree array the scan reads, the scan's tile
// sums, the error and maximum words -- in one statically allocated device
// array of this file.  No hipMalloc, hipFree or allocating library call is
// made on this path.
//
// The array is a file-scope __device__ object: each device the library runs
// on holds its own copy at its own address, kept until the process ends.
// Host code never passes the array's name to a kernel or a copy (on the
// host it is only a stand-in symbol); it asks the runtime for the device
// address once per device (hipGetSymbolAddress, with that device current)
// and uses that address everywhere.
#include "api_internal.h"

#include <mutex>

namespace citron {

namespace {

// Largest vertex count the static working memory is sized for (the Chung-Lu
// configuration graph has 2^22 vertices).
constexpr int32_t kNoAllocMaxN = 1 << 22;
// scan workspace ints reserved (scan_workspace_ints(2^22 + 1) is 2,052)
constexpr int64_t kNoAllocScanInts = 8192;
// layout, in int32 words: [0] error bits, [1] largest out-degree, [2..63]
// unused, [64 .. 64 + n] out-degrees, then the scan workspace
constexpr int64_t kOutdegOff = 64;
constexpr int64_t kScanOff = kOutdegOff + (int64_t)kNoAllocMaxN + 64;
constexpr int64_t kScratchInts = kScanOff + kNoAllocScanInts;

__device__ __align__(256) int32_t scratch[kScratchInts];

constexpr int kMaxDevices = 64;
std::mutex g_mu[kMaxDevices];          // one call at a time per device
int32_t* g_ptr[kMaxDevices] = {};      // device address of scratch, per device

// Device address of this device's copy of the array (looked up once, with
// the device current).
citron_status scratch_of(int dev, int32_t** out)
{
    if (!g_ptr[dev]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(CITRON_EDEVICE, "hipGetSymbolAddress(scratch) gave a null address");
        g_ptr[dev] = static_cast<int32_t*>(p);
    }
    *out = g_ptr[dev];
    return CITRON_OK;
}

}  // namespace

}  // namespace citron

using namespace citron;

extern "C" citron_status citron_order_noalloc(int32_t n, int64_t nnz, const int32_t* row_ptr,
                                              const int32_t* col_idx, int32_t* dag_ptr, int32_t* dag_col,
                                              int32_t* max_outdeg, void* stream)
{
    if (n < 0 || n > kNoAllocMaxN)
        return fail(CITRON_EINVAL, "citron_order_noalloc: n must be in 0..2^22 (size of its static memory)");
    if (nnz < 0 || nnz > 0x7fffffffLL || nnz % 2)
        return fail(CITRON_EINVAL, "citron_order_noalloc: nnz must be even and in 0..2^31-1");
    if (!row_ptr || !dag_ptr || !max_outdeg || (nnz > 0 && (!col_idx || !dag_col)))
        return fail(CITRON_EINVAL, "citron_order_noalloc: NULL pointer");
    if ((int64_t)scan_workspace_ints(n) > kNoAllocScanInts)
        return fail(CITRON_EINVAL, "citron_order_noalloc: scan workspace exceeds its static size");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(CITRON_EDEVICE, "device index out of range");
    std::lock_guard<std::mutex> lock(g_mu[dev]);
    int32_t* base = nullptr;
    citron_status st = scratch_of(dev, &base);
    if (st) return st;
    int32_t* err = base;
    int32_t* mx = base + 1;
    int32_t* outdeg = base + kOutdegOff;
    int32_t* ws = base + kScanOff;
    hipStream_t s = (hipStream_t)stream;

    // offsets first: row_ptr[0] = 0 and row_ptr[n] = nnz (host words on the
    // caller's stack; a copy to pageable memory allocates nothing here)
    int32_t ends[2] = {-1, -1};
    e = hipMemcpyAsync(&ends[0], row_ptr, sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&ends[1], row_ptr + n, sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "citron_order_noalloc: reading row_ptr");
    if (ends[0] != 0 || (int64_t)ends[1] != nnz)
        return fail(CITRON_EINVAL, "invalid CSR: row_ptr[0] must be 0 and row_ptr[n] must equal nnz");
    // validation as in citron_load_csr: offsets, then entries
    for (int stage = 0; stage < 2; ++stage) {
        int32_t bits = 0;
        e = launch_fill_i32(err, 0, 1, s);
        if (e == hipSuccess) e = launch_validate(n, nnz, row_ptr, col_idx, err, stage, s);
        if (e == hipSuccess) e = hipMemcpyAsync(&bits, err, sizeof(int32_t), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "citron_order_noalloc: validation");
        if (bits) return fail(CITRON_EINVAL, "invalid CSR (bits " + std::to_string(bits) +
                                                 ": 1 offsets, 2 id range, 4 self-loop, 8 order, 16 symmetry)");
    }
    // Algorithm 3: out-degrees, scan, scatter
    e = launch_fill_i32(mx, 0, 1, s);
    if (e == hipSuccess)
        e = launch_orient(n, row_ptr, col_idx, outdeg, dag_ptr, dag_col, nullptr, mx, ws, s);
    if (e == hipSuccess && n == 0) e = launch_fill_i32(dag_ptr, 0, 1, s);
    int32_t res[2] = {0, -1};
    if (e == hipSuccess) e = hipMemcpyAsync(&res[0], mx, sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&res[1], dag_ptr + n, sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "citron_order_noalloc: ordering kernels");
    if ((int64_t)res[1] != nnz / 2) return fail(CITRON_EDEVICE, "ordering produced a wrong arc count");
    *max_outdeg = res[0];
    return CITRON_OK;
}
