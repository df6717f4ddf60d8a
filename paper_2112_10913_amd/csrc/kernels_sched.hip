// Work schedules of the count kernel.
//
// The plan: vertices of out-degree >= 2 by out-degree (descending), the
// heavy ones (out-degree > 64) as items of their own, the light ones packed
// into batches of about light_rows rows, and a header with the item counts.
// The heavy arcs: arcs of heavy vertices by |C_uv| (descending).
//
// Both orders break ties by id, so they are fixed by the graph alone: the
// strided shares of a count (citron_count_part) cover the same items in
// every process, and shares counted by different handles of one graph add
// up to the count.  Each order is a device radix sort of 64-bit keys
// (bucket << 32 | id); entries outside the schedule get the largest key and
// sort to the end.  The bucket sizes (the scans the schedule indexes by
// bucket) are read off the sorted keys, with no histogram atomics.
#include "kernels.h"

#include <hipcub/device/device_radix_sort.hpp>

namespace citron {

typedef unsigned long long u64;

// plan: key of vertex u = (D - d(u)) << 32 | u for out-degree d(u) >= 2
__global__ void plan_keys_kernel(int32_t n, const int32_t* __restrict__ dag_ptr, int32_t D, u64* __restrict__ keys)
{
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    const int d = dag_ptr[u + 1] - dag_ptr[u];
    keys[u] = d >= 2 ? ((u64)(unsigned)(D - d) << 32) | (u64)(unsigned)u : ~0ull;
}

// heavy arcs: key of arc e = (D - 1 - |C_uv|) << 32 | e when the source has
// out-degree > 64
__global__ void harc_keys_kernel(int64_t m, const int32_t* __restrict__ dag_ptr, const int32_t* __restrict__ dag_src,
                                 const int32_t* __restrict__ arc_c, int32_t D, u64* __restrict__ keys)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m) return;
    const int u = dag_src[e];
    const bool heavy = dag_ptr[u + 1] - dag_ptr[u] > kLightMaxDeg;
    keys[e] = heavy ? ((u64)(unsigned)(D - 1 - arc_c[e]) << 32) | (u64)e : ~0ull;
}

// bounds[b] = number of sorted keys with bucket < b, for b = 0..nb, where
// the bucket of a key is its high word (the sentinel ~0 counts as bucket
// nb): thread i fills the bounds between the buckets of keys i - 1 and i.
__global__ void bucket_bounds_kernel(int64_t n, const u64* __restrict__ keys, int32_t nb, int32_t* __restrict__ bounds)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const unsigned hi = (unsigned)(keys[i] >> 32);
    const int b = hi < (unsigned)nb ? (int)hi : nb;
    int prev = -1;
    if (i > 0) {
        const unsigned ph = (unsigned)(keys[i - 1] >> 32);
        prev = ph < (unsigned)nb ? (int)ph : nb;
    }
    for (int x = prev + 1; x <= b; ++x) bounds[x] = (int32_t)i;
    if (i == n - 1)
        for (int x = b + 1; x <= nb; ++x) bounds[x] = (int32_t)n;
}

// out[i] = low word of keys[i] for i < *count (the entries in the schedule)
__global__ void unpack_keys_kernel(int64_t n, const u64* __restrict__ keys, const int32_t* __restrict__ count,
                                   int32_t* __restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && i < *count) out[i] = (int32_t)(unsigned)keys[i];
}

size_t sched_sort_temp_bytes(int64_t n)
{
    size_t bytes = 0;
    if (n <= 0) return 1;
    if (hipcub::DeviceRadixSort::SortKeys(nullptr, bytes, (const u64*)nullptr, (u64*)nullptr, (int)n, 0, 64) !=
        hipSuccess)
        return 0;
    return bytes > 0 ? bytes : 1;
}

// Sorted keys -> bounds of nb buckets -> the ids of the first bounds[nb].
static hipError_t sort_and_split(int64_t n, int32_t nb, int32_t* bounds, int32_t* out, const SortBuffers& sb,
                                 hipStream_t s)
{
    const unsigned blocks = (unsigned)((n + 255) / 256);
    size_t tb = sb.temp_bytes;
    hipError_t e = hipcub::DeviceRadixSort::SortKeys(sb.temp, tb, (const u64*)sb.keys_a, sb.keys_b, (int)n, 0, 64, s);
    if (e != hipSuccess) return e;
    bucket_bounds_kernel<<<blocks, 256, 0, s>>>(n, sb.keys_b, nb, bounds);
    unpack_keys_kernel<<<blocks, 256, 0, s>>>(n, sb.keys_b, bounds + nb, out);
    return hipGetLastError();
}

hipError_t sched_plan_order(int32_t n, const int32_t* dag_ptr, int32_t D, int32_t* bounds, int32_t* order,
                            const SortBuffers& sb, hipStream_t s)
{
    if (n <= 0) return launch_fill_i32(bounds, 0, D, s);
    plan_keys_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, dag_ptr, D, sb.keys_a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // buckets D - d for d = D .. 2: D - 1 of them
    return sort_and_split(n, D - 1, bounds, order, sb, s);
}

hipError_t sched_heavy_arcs(int64_t m, const int32_t* dag_ptr, const int32_t* dag_src, const int32_t* arc_c,
                            int32_t D, int32_t* bounds, int32_t* harcs, const SortBuffers& sb, hipStream_t s)
{
    if (m <= 0) return launch_fill_i32(bounds, 0, D + 1, s);
    harc_keys_kernel<<<(unsigned)((m + 255) / 256), 256, 0, s>>>(m, dag_ptr, dag_src, arc_c, D, sb.keys_a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // buckets D - 1 - c for c = D - 1 .. 0: D of them
    return sort_and_split(m, D, bounds, harcs, sb, s);
}

// ---------------------------------------------------------------- plan

// light_deg[j] = out-degree of order[n_heavy + j]; n_heavy and the light
// count are read from the scanned histogram.
__global__ void plan_light_deg_kernel(const int32_t* __restrict__ dag_ptr, const int32_t* __restrict__ order,
                                      const int32_t* __restrict__ hist_scan, int32_t D,
                                      int32_t* __restrict__ light_deg, int32_t n)
{
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t n_heavy = D > kLightMaxDeg ? hist_scan[D - kLightMaxDeg] : 0;
    const int32_t n_all = hist_scan[D - 1];
    const int32_t n_light = n_all - n_heavy;
    if (j >= n) return;
    if (j < n_light) {
        int u = order[n_heavy + j];
        light_deg[j] = dag_ptr[u + 1] - dag_ptr[u];
    } else {
        light_deg[j] = 0;
    }
}

__global__ void plan_batches_kernel(const int32_t* __restrict__ hist_scan, int32_t D,
                                    const int32_t* __restrict__ light_pre, int32_t light_rows,
                                    int32_t* __restrict__ batch_start)
{
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t n_heavy = D > kLightMaxDeg ? hist_scan[D - kLightMaxDeg] : 0;
    const int32_t n_light = hist_scan[D - 1] - n_heavy;
    if (j >= n_light) return;
    int b = light_pre[j] / light_rows;
    if (j == 0 || light_pre[j - 1] / light_rows != b) batch_start[b] = (int32_t)j;
    if (j == n_light - 1) batch_start[b + 1] = n_light;
}

__global__ void plan_header_kernel(const int32_t* __restrict__ hist_scan, int32_t D,
                                   const int32_t* __restrict__ light_pre, int32_t light_rows,
                                   int32_t split_min_deg, int32_t split_factor,
                                   const int32_t* __restrict__ batch_start, PlanHeader* __restrict__ h)
{
    const int32_t n_heavy = D > kLightMaxDeg ? hist_scan[D - kLightMaxDeg] : 0;
    const int32_t n_light = hist_scan[D - 1] - n_heavy;
    int32_t n_split = 0;
    if (split_factor > 1 && split_min_deg <= D) {
        int32_t thr = split_min_deg > kLightMaxDeg ? split_min_deg : kLightMaxDeg + 1;
        n_split = thr <= D ? hist_scan[D - thr + 1] : 0;
    }
    int32_t n_batches = n_light > 0 ? light_pre[n_light - 1] / light_rows + 1 : 0;
    (void)batch_start;
    h->n_heavy = n_heavy;
    h->n_split = n_split;
    h->split_factor = split_factor > 1 ? split_factor : 1;
    h->n_light = n_light;
    h->n_batches = n_batches;
    h->n_items = n_split * h->split_factor + (n_heavy - n_split) + n_batches;
    h->light_rows = light_rows;
    h->max_rows = light_rows + kLightMaxDeg - 1;
}

hipError_t launch_plan(int32_t n, const int32_t* dag_ptr, int32_t max_outdeg, int32_t light_rows,
                       int32_t split_min_deg, int32_t split_factor, const PlanBuffers& pb,
                       int32_t* scan_ws, const SortBuffers& sb, hipStream_t s)
{
    // D >= 2 keeps the bucket arithmetic valid for graphs without any
    // vertex of out-degree 2 or more (the plan is then empty).
    const int32_t D = max_outdeg > 2 ? max_outdeg : 2;
    const unsigned nb = (unsigned)((n + 255) / 256);
    // order: vertices of out-degree >= 2 by out-degree descending, ties by
    // id (the same order in every process); hist_scan[i] = vertices with
    // out-degree > D - i (buckets 0..i-1), hist_scan[D - 1] = all of them
    hipError_t e = sched_plan_order(n, dag_ptr, D, pb.hist_scan, pb.order, sb, s);
    if (e != hipSuccess) return e;
    if (n > 0)
        plan_light_deg_kernel<<<nb, 256, 0, s>>>(dag_ptr, pb.order, pb.hist_scan, D, pb.light_deg, n);
    e = scan_exclusive(pb.light_deg, pb.light_pre, n, scan_ws, s);
    if (e != hipSuccess) return e;
    if (n > 0)
        plan_batches_kernel<<<nb, 256, 0, s>>>(pb.hist_scan, D, pb.light_pre, light_rows, pb.batch_start);
    plan_header_kernel<<<1, 1, 0, s>>>(pb.hist_scan, D, pb.light_pre, light_rows, split_min_deg,
                                       split_factor, pb.batch_start, pb.header);
    return hipGetLastError();
}

}  // namespace citron
