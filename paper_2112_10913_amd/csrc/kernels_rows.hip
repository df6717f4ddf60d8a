// Subgraph construction of the counting phase (Lonkar & Beamer, Section V-B,
// Algorithm 5) and the schedule of the count kernel.
//
// For every vertex u with out-list N->(u) = (v_0 < ... < v_{d-1}) the rows
// of the subgraph induced on N->(u) are built once per graph: row i is
// N->(v_i) cap N->(u), a bitmap over the positions 0..d-1 of N->(u) with
// W(u) = ceil(d/64) words.  Row i is also the candidate set C_uv of the arc
// u -> v_i, so its popcount |C_uv| is the arc's triangle count and the arc's
// cost estimate.  The rows do not depend on k; every count reuses them.
//
// Work items are vertices sorted by out-degree (descending): one item per
// heavy vertex (out-degree > 64), and batches of light vertices of about
// `light_rows` rows.  A workgroup intersects, for all (row, entry) pairs of
// an item spread over its threads, each entry of N->(v_i) with N->(u) by a
// binary search in LDS; the bitmap is assembled in LDS in chunks of rows and
// written out to device memory with coalesced stores.
#include "kernels.h"

namespace citron {

typedef unsigned long long u64;

namespace {

constexpr int kWave_ = kWave;
constexpr int kBuildBitmapWords = 2048;   // 16 KB of LDS per chunk of rows

__device__ __forceinline__ int lane_of() { return threadIdx.x & (kWave_ - 1); }

__device__ __forceinline__ int wave_incl_scan(int v)
{
    const int lane = lane_of();
#pragma unroll
    for (int o = 1; o < kWave_; o <<= 1) {
        int t = __shfl_up(v, o, kWave_);
        if (lane >= o) v += t;
    }
    return v;
}

__device__ __forceinline__ int upper_bound_i32(const int32_t* a, int n, int32_t x)
{
    int lo = 0, hi = n;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (a[mid] <= x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ int lower_bound_i32(const int32_t* a, int n, int32_t x)
{
    int lo = 0, hi = n;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (a[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

struct BuildCtrl {
    int32_t item;
    int32_t kind;      // 0 light batch, 1 heavy vertex
    int32_t first;
    int32_t nb;
    int32_t R;
    int32_t pad[3];
    int32_t wsum[16];
};

}  // namespace

__host__ __device__ inline int build_rows_cap(int light_rows, int max_deg)
{
    const int rc = light_rows + kLightMaxDeg;
    return max_deg > rc ? max_deg : rc;
}

int32_t build_lds_bytes(int32_t light_rows, int32_t max_deg)
{
    const int Dc = build_rows_cap(light_rows, max_deg);
    const int Vc = (light_rows + kLightMaxDeg) / 2 + 2;
    int b = (int)sizeof(BuildCtrl) + 4 * 4 * (Dc + 4) + 4 * 4 * Vc;
    b = (b + 15) & ~15;
    return b + 8 * kBuildBitmapWords;
}

__global__ void __launch_bounds__(256) build_rows_kernel(BuildParams P)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int T = blockDim.x, tid = threadIdx.x, lane = lane_of(), wid = tid / kWave_;
    const int nwaves = T / kWave_;
    const int Dc = build_rows_cap(P.plan.light_rows, P.max_deg);
    const int Vc = (P.plan.light_rows + kLightMaxDeg) / 2 + 2;
    BuildCtrl* ctrl = reinterpret_cast<BuildCtrl*>(smem);
    int32_t* row_v = reinterpret_cast<int32_t*>(smem + sizeof(BuildCtrl));
    int32_t* row_owner = row_v + (Dc + 4);
    int32_t* row_begin = row_owner + (Dc + 4);
    int32_t* pre = row_begin + (Dc + 4);
    int32_t* vert_u = pre + (Dc + 4);
    int32_t* vert_base = vert_u + Vc;
    int32_t* vert_deg = vert_base + Vc;
    int32_t* vert_arc0 = vert_deg + Vc;
    size_t off = (size_t)((unsigned char*)(vert_arc0 + Vc) - smem);
    off = (off + 15) & ~(size_t)15;
    u64* bm = reinterpret_cast<u64*>(smem + off);
    const int32_t* __restrict__ dag_ptr = P.dag_ptr;
    const int32_t* __restrict__ dag_col = P.dag_col;
    const int n_items = P.plan.n_heavy + P.plan.n_batches;
    u64 tri = 0, st_entries = 0, st_rows = 0, st_verts = 0, st_bytes = 0;

    for (;;) {
        if (tid == 0) {
            int g = atomicAdd(P.item_ctr, 1);
            ctrl->item = g < n_items ? g : -1;
            if (g < n_items) {
                if (g < P.plan.n_heavy) {
                    const int u = P.order[g];
                    const int d = dag_ptr[u + 1] - dag_ptr[u];
                    ctrl->kind = 1;
                    ctrl->nb = 1;
                    ctrl->R = d;
                    vert_u[0] = u;
                    vert_base[0] = 0;
                    vert_deg[0] = d;
                    vert_arc0[0] = dag_ptr[u];
                } else {
                    const int b = g - P.plan.n_heavy;
                    const int s0 = P.batch_start[b], s1 = P.batch_start[b + 1];
                    ctrl->kind = 0;
                    ctrl->first = s0;
                    ctrl->nb = s1 - s0;
                    ctrl->R = P.light_pre[s1] - P.light_pre[s0];
                }
            }
        }
        __syncthreads();
        if (ctrl->item < 0) break;
        const int kind = ctrl->kind, nb = ctrl->nb, R = ctrl->R;
        if (kind == 0) {
            const int s0 = ctrl->first;
            const int base0 = P.light_pre[s0];
            for (int j = tid; j < nb; j += T) {
                const int u = P.order[P.plan.n_heavy + s0 + j];
                vert_u[j] = u;
                vert_base[j] = P.light_pre[s0 + j] - base0;
                vert_deg[j] = P.light_pre[s0 + j + 1] - P.light_pre[s0 + j];
                vert_arc0[j] = dag_ptr[u];
            }
        }
        __syncthreads();
        // rows: v = N->(u)[i] and the length of N->(v)
        for (int r = tid; r < R; r += T) {
            const int b = (kind == 0) ? upper_bound_i32(vert_base, nb, r) - 1 : 0;
            const int v = dag_col[vert_arc0[b] + (r - vert_base[b])];
            row_v[r] = v;
            row_owner[r] = b;
            const int a0 = dag_ptr[v];
            row_begin[r] = a0;
            pre[r] = dag_ptr[v + 1] - a0;
        }
        __syncthreads();
        {   // block-wide exclusive scan of the row lengths, pre[R] = total
            int carry = 0;
            for (int base = 0; base < R; base += T) {
                const int r = base + tid;
                const int v = r < R ? pre[r] : 0;
                const int inc = wave_incl_scan(v);
                if (lane == kWave_ - 1) ctrl->wsum[wid] = inc;
                __syncthreads();
                int o = 0, tot = 0;
                for (int w = 0; w < nwaves; ++w) {
                    const int x = ctrl->wsum[w];
                    if (w < wid) o += x;
                    tot += x;
                }
                if (r < R) pre[r] = carry + o + inc - v;
                __syncthreads();
                carry += tot;
            }
            if (tid == 0) pre[R] = carry;
        }
        __syncthreads();
        const int W = (kind == 0) ? 1 : (R + 63) >> 6;
        const int chunk = kBuildBitmapWords / W;
        if (tid == 0) {
            st_verts += (u64)nb;
            st_rows += (u64)R;
            st_entries += (u64)pre[R];
            st_bytes += 4ull * ((u64)R + 2ull * nb) + 4ull * ((u64)pre[R] + 2ull * R);
        }
        for (int r0 = 0; r0 < R; r0 += chunk) {
            const int r1 = min(R, r0 + chunk);
            for (int i = tid; i < (r1 - r0) * W; i += T) bm[i] = 0ull;
            __syncthreads();
            // Algorithm 5: each entry x of N->(v_r) looked up in N->(u)
            const int t1 = pre[r1];
            for (int t = pre[r0] + tid; t < t1; t += T) {
                const int r = upper_bound_i32(pre, R + 1, t) - 1;
                const int x = dag_col[row_begin[r] + (t - pre[r])];
                const int b = row_owner[r];
                const int32_t* nu = row_v + vert_base[b];
                const int du = vert_deg[b];
                const int p = lower_bound_i32(nu, du, x);
                if (p < du && nu[p] == x)
                    atomicOr(&bm[(r - r0) * W + (p >> 6)], 1ull << (p & 63));
            }
            __syncthreads();
            // write the chunk out; one thread per row also records |C_uv|
            for (int i = tid; i < (r1 - r0) * W; i += T) {
                const int r = r0 + i / W, w = i - (i / W) * W;
                const int b = row_owner[r];
                const int li = r - vert_base[b];
                P.rows[(int64_t)P.rows_off[vert_u[b]] + (int64_t)li * W + w] = bm[i];
            }
            for (int r = r0 + tid; r < r1; r += T) {
                int c = 0;
                for (int w = 0; w < W; ++w) c += __popcll(bm[(r - r0) * W + w]);
                const int b = row_owner[r];
                P.arc_c[vert_arc0[b] + (r - vert_base[b])] = c;
                tri += (u64)c;
            }
            __syncthreads();
        }
    }
    // triangles (k = 3) and build counters
#pragma unroll
    for (int o = kWave_ / 2; o > 0; o >>= 1) {
        unsigned lo = __shfl_xor((unsigned)tri, o, kWave_);
        unsigned hi = __shfl_xor((unsigned)(tri >> 32), o, kWave_);
        tri += ((u64)hi << 32) | lo;
    }
    if (lane == 0 && tri) {
        const u64 old = atomicAdd(P.tri_acc, tri);
        if (old + tri < old) atomicOr(P.tri_ovf, 1);
    }
    if (tid == 0 && st_verts) {
        atomicAdd(P.build_stats + kStatVertices, st_verts);
        atomicAdd(P.build_stats + kStatRows, st_rows);
        atomicAdd(P.build_stats + kStatEntries, st_entries);
        atomicAdd(P.build_stats + kStatBytes, st_bytes);
    }
}

// rows_len[u] = d(u) * W(u), the words of u's rows
__global__ void rows_len_kernel(int32_t n, const int32_t* __restrict__ dag_ptr, int32_t* __restrict__ len)
{
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    const int d = dag_ptr[u + 1] - dag_ptr[u];
    len[u] = d * ((d + 63) >> 6);
}

// per_arc[e] = |C_uv| (the k = 3 per-arc counts)
__global__ void arc_c_to_u64_kernel(int64_t m, const int32_t* __restrict__ arc_c, u64* __restrict__ out)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < m) out[e] = (u64)arc_c[e];
}

hipError_t launch_rows_len(int32_t n, const int32_t* dag_ptr, int32_t* len, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    rows_len_kernel<<<(n + 255) / 256, 256, 0, s>>>(n, dag_ptr, len);
    return hipGetLastError();
}

hipError_t launch_build_rows(const BuildParams& P, int32_t blocks, hipStream_t s)
{
    if (P.plan.n_heavy + P.plan.n_batches <= 0) return hipSuccess;
    const int32_t lds = build_lds_bytes(P.plan.light_rows, P.max_deg);
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)build_rows_kernel,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        if (e != hipSuccess) return e;
    }
    build_rows_kernel<<<blocks, 256, lds, s>>>(P);
    return hipGetLastError();
}

hipError_t launch_arc_c_to_u64(int64_t m, const int32_t* arc_c, u64* out, hipStream_t s)
{
    if (m <= 0) return hipSuccess;
    arc_c_to_u64_kernel<<<(unsigned)((m + 255) / 256), 256, 0, s>>>(m, arc_c, out);
    return hipGetLastError();
}

}  // namespace citron
