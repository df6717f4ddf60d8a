// Input validation, device-wide exclusive scan and the ordering phase
// (Section IV, Algorithm 3 of Lonkar & Beamer): count the out-degree of
// every vertex under the degree ordering, prefix-sum the counts into the
// DAG row offsets, and place the kept neighbours of each row in their input
// (ascending id) order.
#include "kernels.h"

namespace citron {

// ------------------------------------------------------------ wave helpers

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

__device__ __forceinline__ int wave_inclusive_scan(int v)
{
    const int lane = lane_id();
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        int t = __shfl_up(v, o, kWave);
        if (lane >= o) v += t;
    }
    return v;
}

// ------------------------------------------------------------- validation

// err bits: 1 row_ptr out of range or decreasing, 2 column id out of range,
// 4 self-loop, 8 row not strictly ascending, 16 asymmetric.
__global__ void validate_row_ptr_kernel(int32_t n, int64_t nnz, const int32_t* __restrict__ row_ptr,
                                        int32_t* __restrict__ err)
{
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    int32_t a = row_ptr[u], b = row_ptr[u + 1];
    if (a < 0 || b < a || (int64_t)b > nnz) atomicOr(err, 1);
}

__global__ void validate_entries_kernel(int32_t n, const int32_t* __restrict__ row_ptr,
                                        const int32_t* __restrict__ col, int32_t* __restrict__ err)
{
    const int64_t u = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    if (u >= n) return;
    const int lane = lane_id();
    const int32_t a = row_ptr[u], b = row_ptr[u + 1];
    int bits = 0;
    for (int32_t e = a + lane; e < b; e += kWave) {
        const int32_t v = col[e];
        if (v < 0 || v >= n) { bits |= 2; continue; }
        if (v == (int32_t)u) bits |= 4;
        if (e > a && col[e - 1] >= v) bits |= 8;
        // symmetry: u must appear in row v (row v is checked for order by
        // its own wave; a binary search on an unsorted row may miss u, which
        // is then reported as asymmetric, still an error)
        int32_t lo = row_ptr[v], hi = row_ptr[v + 1];
        while (lo < hi) {
            int32_t mid = lo + ((hi - lo) >> 1);
            if (col[mid] < (int32_t)u) lo = mid + 1;
            else hi = mid;
        }
        if (lo >= row_ptr[v + 1] || col[lo] != (int32_t)u) bits |= 16;
    }
    if (bits) atomicOr(err, bits);
}

// ------------------------------------------------------------------- scan
//
// Exclusive prefix sum of n int32 values into out[0..n], out[n] = total,
// by reduce-then-scan over tiles of kScanTile values (recursive on the tile
// sums).  The totals must fit int32 (they are CSR offsets).

constexpr int kScanBlock = 256;
constexpr int kScanPer = 16;
constexpr int kScanTile = kScanBlock * kScanPer;

__device__ int block_exclusive_scan(int v, int* total)
{
    __shared__ int wsum[kScanBlock / kWave];
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    int inc = wave_inclusive_scan(v);
    if (lane == kWave - 1) wsum[wid] = inc;
    __syncthreads();
    int off = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kScanBlock / kWave; ++w) {
        if (w < wid) off += wsum[w];
        tot += wsum[w];
    }
    __syncthreads();
    *total = tot;
    return off + inc - v;
}

__global__ void scan_tile_sums_kernel(const int32_t* __restrict__ in, int64_t n, int32_t* __restrict__ sums)
{
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
    int s = 0;
#pragma unroll
    for (int i = 0; i < kScanPer; ++i)
        if (base + i < n) s += in[base + i];
    int tot;
    block_exclusive_scan(s, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ void scan_tiles_kernel(const int32_t* __restrict__ in, int64_t n,
                                  const int32_t* __restrict__ tile_off, int32_t* __restrict__ out)
{
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
    int vals[kScanPer];
    int s = 0;
#pragma unroll
    for (int i = 0; i < kScanPer; ++i) {
        vals[i] = (base + i < n) ? in[base + i] : 0;
        s += vals[i];
    }
    int tot;
    int run = block_exclusive_scan(s, &tot) + (tile_off ? tile_off[blockIdx.x] : 0);
#pragma unroll
    for (int i = 0; i < kScanPer; ++i) {
        if (base + i < n) out[base + i] = run;
        run += vals[i];
    }
    // the thread holding element n-1 writes the total into out[n]
    if (n > 0 && base <= n - 1 && n - 1 < base + kScanPer) out[n] = run;
    if (n == 0 && blockIdx.x == 0 && threadIdx.x == 0) out[0] = tile_off ? tile_off[0] : 0;
    (void)tot;
}

size_t scan_workspace_ints(int64_t n)
{
    if (n <= kScanTile) return 1;
    const int64_t tiles = (n + kScanTile - 1) / kScanTile;
    return (size_t)(2 * tiles + 1) + scan_workspace_ints(tiles);
}

// in and out may not alias; out receives n + 1 values.
// ws: scan_workspace_ints(n) ints: [tile sums | scanned tile sums | deeper].
hipError_t scan_exclusive(const int32_t* in, int32_t* out, int64_t n, int32_t* ws, hipStream_t s)
{
    if (n <= kScanTile) {
        scan_tiles_kernel<<<1, kScanBlock, 0, s>>>(in, n, nullptr, out);
        return hipGetLastError();
    }
    const int64_t tiles = (n + kScanTile - 1) / kScanTile;
    int32_t* sums = ws;
    int32_t* offs = ws + tiles;
    scan_tile_sums_kernel<<<(unsigned)tiles, kScanBlock, 0, s>>>(in, n, sums);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = scan_exclusive(sums, offs, tiles, ws + 2 * tiles + 1, s);
    if (e != hipSuccess) return e;
    scan_tiles_kernel<<<(unsigned)tiles, kScanBlock, 0, s>>>(in, n, offs, out);
    return hipGetLastError();
}

// --------------------------------------------------------------- ordering

// omega(u) < omega(v): lower key first, ties by lower id.  The key is the
// undirected degree for the degree ordering (Section IV), or the round in
// which a vertex left the peeling for the core ordering.
__device__ __forceinline__ bool keeps(int32_t du, int32_t u, int32_t dv, int32_t v)
{
    return du < dv || (du == dv && u < v);
}

// key of v: its degree, or key[v] when a key array is given
__device__ __forceinline__ int32_t key_of(const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ key,
                                          int32_t v)
{
    return key ? key[v] : row_ptr[v + 1] - row_ptr[v];
}

// Out-degree of every vertex (first loop of Algorithm 3).  One wavefront per
// vertex; each lane takes four row entries per step so that four neighbour
// degree gathers are in flight.  Also tracks the largest out-degree.
__global__ void orient_count_kernel(int32_t n, const int32_t* __restrict__ row_ptr,
                                    const int32_t* __restrict__ col, const int32_t* __restrict__ key,
                                    int32_t* __restrict__ outdeg, int32_t* __restrict__ max_outdeg)
{
    const int64_t u = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    if (u >= n) return;
    const int lane = lane_id();
    const int32_t a = row_ptr[u], b = row_ptr[u + 1];
    const int32_t du = key_of(row_ptr, key, (int32_t)u);
    int cnt = 0;
    for (int32_t e0 = a; e0 < b; e0 += 4 * kWave) {
        int32_t v[4], dv[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            int32_t e = e0 + j * kWave + lane;
            v[j] = e < b ? col[e] : -1;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j)
            dv[j] = v[j] >= 0 ? key_of(row_ptr, key, v[j]) : 0;
#pragma unroll
        for (int j = 0; j < 4; ++j)
            cnt += (v[j] >= 0 && keeps(du, (int32_t)u, dv[j], v[j])) ? 1 : 0;
    }
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, kWave);
    if (lane == 0) {
        outdeg[u] = cnt;
        atomicMax(max_outdeg, cnt);
    }
}

// Place the kept neighbours (second loop of Algorithm 3).  One wavefront per
// vertex walks its row in 64-entry steps; a ballot marks the kept entries and
// each lane writes at the count of kept entries before it, so the row keeps
// its ascending order.  dag_src (may be null) receives the source vertex of
// every arc.
__global__ void orient_scatter_kernel(int32_t n, const int32_t* __restrict__ row_ptr,
                                      const int32_t* __restrict__ col, const int32_t* __restrict__ key,
                                      const int32_t* __restrict__ dag_ptr,
                                      int32_t* __restrict__ dag_col, int32_t* __restrict__ dag_src)
{
    const int64_t u = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    if (u >= n) return;
    const int lane = lane_id();
    const int32_t a = row_ptr[u], b = row_ptr[u + 1];
    const int32_t du = key_of(row_ptr, key, (int32_t)u);
    int32_t out = dag_ptr[u];
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
    for (int32_t e0 = a; e0 < b; e0 += kWave) {
        const int32_t e = e0 + lane;
        int32_t v = -1;
        bool keep = false;
        if (e < b) {
            v = col[e];
            keep = keeps(du, (int32_t)u, key_of(row_ptr, key, v), v);
        }
        const unsigned long long mask = __ballot(keep);
        if (keep) {
            const int32_t pos = out + __popcll(mask & below);
            dag_col[pos] = v;
            if (dag_src) dag_src[pos] = (int32_t)u;
        }
        out += __popcll(mask);
    }
}

// ------------------------------------------------------------ host wrappers

hipError_t launch_validate(int32_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col,
                           int32_t* err, int stage, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    if (stage == 0) {
        validate_row_ptr_kernel<<<(n + 255) / 256, 256, 0, s>>>(n, nnz, row_ptr, err);
    } else {
        const int64_t threads = (int64_t)n * kWave;
        validate_entries_kernel<<<(unsigned)((threads + 255) / 256), 256, 0, s>>>(n, row_ptr, col, err);
    }
    return hipGetLastError();
}

hipError_t launch_orient(int32_t n, const int32_t* row_ptr, const int32_t* col, int32_t* outdeg,
                         int32_t* dag_ptr, int32_t* dag_col, int32_t* dag_src, int32_t* max_outdeg,
                         int32_t* scan_ws, hipStream_t s, const int32_t* key)
{
    if (n == 0) return hipSuccess;
    const int64_t threads = (int64_t)n * kWave;
    const unsigned blocks = (unsigned)((threads + 255) / 256);
    orient_count_kernel<<<blocks, 256, 0, s>>>(n, row_ptr, col, key, outdeg, max_outdeg);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = scan_exclusive(outdeg, dag_ptr, n, scan_ws, s);
    if (e != hipSuccess) return e;
    orient_scatter_kernel<<<blocks, 256, 0, s>>>(n, row_ptr, col, key, dag_ptr, dag_col, dag_src);
    return hipGetLastError();
}

}  // namespace citron
