// Core ordering on the GPU (Section III, Algorithm 1 and the discussion of
// its cost in Section IV): the paper's Algorithm 1 removes one vertex of
// smallest current degree at a time, a sequential process.  Here all
// vertices whose current degree is at most a threshold t leave in one round
// (level-synchronous peeling): a round marks its frontier, then lowers the
// degree of every neighbour still present by one per edge; a neighbour whose
// degree falls from t + 1 to t joins the next round's frontier (exactly one
// decrement sees that step, so it is appended once).  When a round's
// frontier is empty, t rises to the smallest degree still present.  The
// round numbers are the order key (ties by id): every out-degree of the
// resulting DAG is at most the t of its vertex's round, which never exceeds
// the degeneracy.
#include "kernels.h"

namespace citron {

namespace {

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

// Block-wide minimum, then one atomic per block.
__device__ void block_min_to(int v, int32_t* out)
{
    __shared__ int wmin[1024 / kWave];
    const int lane = lane_id(), wid = threadIdx.x / kWave;
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, kWave));
    if (lane == 0) wmin[wid] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        int m = wmin[0];
        for (int w = 1; w < (int)(blockDim.x / kWave); ++w) m = min(m, wmin[w]);
        if (m != 0x7fffffff) atomicMin(out, m);
    }
}

}  // namespace

__global__ void peel_init_kernel(int32_t n, const int32_t* __restrict__ row_ptr, int32_t* __restrict__ deg,
                                 int32_t* __restrict__ round, int32_t* __restrict__ min_deg)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int d = 0x7fffffff;
    if (v < n) {
        d = row_ptr[v + 1] - row_ptr[v];
        deg[v] = d;
        round[v] = -1;
    }
    block_min_to(d, min_deg);
}

__global__ void peel_min_kernel(int32_t n, const int32_t* __restrict__ deg, const int32_t* __restrict__ round,
                                int32_t* __restrict__ min_deg)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int d = (v < n && round[v] < 0) ? deg[v] : 0x7fffffff;
    block_min_to(d, min_deg);
}

// Ballot compaction per wave, one atomic per wave.
__global__ void peel_collect_kernel(int32_t n, const int32_t* __restrict__ deg, const int32_t* __restrict__ round,
                                    int32_t t, int32_t* __restrict__ frontier, int32_t* __restrict__ cnt)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = lane_id();
    const bool take = v < n && round[v] < 0 && deg[v] <= t;
    const unsigned long long mask = __ballot(take);
    if (!mask) return;
    int base = 0;
    if (lane == 0) base = atomicAdd(cnt, __popcll(mask));
    base = __shfl(base, 0, kWave);
    if (take) {
        const unsigned long long below = lane == 0 ? 0ull : (~0ull >> (kWave - lane));
        frontier[base + __popcll(mask & below)] = (int32_t)v;
    }
}

__global__ void peel_mark_kernel(int32_t nf, const int32_t* __restrict__ frontier, int32_t* __restrict__ round,
                                 int32_t r)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nf) round[frontier[i]] = r;
}

// One wave per frontier vertex, lanes over its neighbours.
__global__ void peel_relax_kernel(int32_t nf, const int32_t* __restrict__ frontier,
                                  const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                                  int32_t* __restrict__ deg, const int32_t* __restrict__ round, int32_t t,
                                  int32_t* __restrict__ next, int32_t* __restrict__ next_cnt)
{
    const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    if (i >= nf) return;
    const int lane = lane_id();
    const int32_t v = frontier[i];
    const int32_t a = row_ptr[v], b = row_ptr[v + 1];
    for (int32_t e = a + lane; e < b; e += kWave) {
        const int32_t w = col[e];
        if (round[w] >= 0) continue;            // gone, or leaving in this round
        const int32_t old = atomicSub(&deg[w], 1);
        if (old == t + 1) next[atomicAdd(next_cnt, 1)] = w;
    }
}

hipError_t launch_peel_init(int32_t n, const int32_t* row_ptr, int32_t* deg, int32_t* round, int32_t* min_deg,
                            hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    peel_init_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, row_ptr, deg, round, min_deg);
    return hipGetLastError();
}

hipError_t launch_peel_min(int32_t n, const int32_t* deg, const int32_t* round, int32_t* min_deg, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    peel_min_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, deg, round, min_deg);
    return hipGetLastError();
}

hipError_t launch_peel_collect(int32_t n, const int32_t* deg, const int32_t* round, int32_t t, int32_t* frontier,
                               int32_t* cnt, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    peel_collect_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, deg, round, t, frontier, cnt);
    return hipGetLastError();
}

hipError_t launch_peel_round(int32_t nf, const int32_t* frontier, const int32_t* row_ptr, const int32_t* col,
                             int32_t* deg, int32_t* round, int32_t t, int32_t r, int32_t* next, int32_t* next_cnt,
                             hipStream_t s)
{
    if (nf <= 0) return hipSuccess;
    peel_mark_kernel<<<(unsigned)((nf + 255) / 256), 256, 0, s>>>(nf, frontier, round, r);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t threads = (int64_t)nf * kWave;
    peel_relax_kernel<<<(unsigned)((threads + 255) / 256), 256, 0, s>>>(nf, frontier, row_ptr, col, deg, round, t,
                                                                       next, next_cnt);
    return hipGetLastError();
}

}  // namespace citron
