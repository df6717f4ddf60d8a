// k-clique listing through the counting recursion (the paper's conclusion
// names listing as a small change of the counting method): for each listed
// arc u -> v, the k-cliques whose two lowest vertices in the ordering are u
// and v are written out as k vertex ids each, in increasing order of the
// ordering -- u, v, then the chosen candidates level by level.  Within an
// arc the cliques come in the order of a depth-first search that takes the
// candidates of every level in ascending position (= ascending id) order.
//
// One wave per arc at a time (a persistent grid pulls arcs from one
// cursor).  The search state is wave-uniform, lane q holding word q of each
// candidate mask over the positions of N->(u), as in the heavy count engine;
// the masks of the open levels live in the wave's LDS, k - 2 levels of one
// word per lane (3 KB per wave at k = 5, 14 KB at k = 16).  At the last level
// every candidate completes a clique: lane j writes the clique of the j-th
// set bit, so the output rows of one node are written in one step.  The
// offsets of the arcs' output come from their exact counts (a scan of the
// per-arc counts of the count kernel), so no atomics order the output;
// every write is checked against the arc's slot and a mismatch raises a
// flag instead of writing outside it.
#include "kernels.h"

#include <numeric>

namespace citron {

namespace {

typedef unsigned long long u64;

constexpr int kListBlock = 256;                 // 4 waves
constexpr int kListWaves = kListBlock / kWave;

__device__ __forceinline__ int lane_of() { return threadIdx.x & (kWave - 1); }

__device__ __forceinline__ u64 readlane64(u64 v, int lane)
{
    unsigned lo = __builtin_amdgcn_readlane((unsigned)v, lane);
    unsigned hi = __builtin_amdgcn_readlane((unsigned)(v >> 32), lane);
    return ((u64)hi << 32) | lo;
}

// Position of the r-th (0-based) set bit of v.
__device__ __forceinline__ int select64(u64 v, int r)
{
    int pos = 0;
#pragma unroll
    for (int s = 32; s > 0; s >>= 1) {
        const u64 low = v & ((1ull << s) - 1);
        const int c = __popcll(low);
        if (r >= c) {
            r -= c;
            v >>= s;
            pos += s;
        } else {
            v = low;
        }
    }
    return pos;
}

// Levels whose masks are kept for the way back: a node at level t is
// pushed only while k - 2 - t >= 2 vertices remain to choose, so levels
// 0 .. k - 4 are stored; k - 2 (at least 1) bounds them.
__host__ __device__ __forceinline__ int list_levels(int k) { return k > 3 ? k - 2 : 1; }

}  // namespace

__global__ void __launch_bounds__(kListBlock) list_arcs_kernel(ListParams P)
{
    // the open levels' masks, k - 2 levels per wave (sized at launch, so
    // that small k leaves LDS for more resident waves)
    extern __shared__ u64 lds_levels[];
    __shared__ int32_t sPre[kListWaves][kListMaxK];
    const int lane = lane_of();
    const int wid = threadIdx.x / kWave;
    const int k = P.k;
    const int levels = list_levels(k);
    u64* const sM = lds_levels + (size_t)wid * levels * kWave;
    u64* const sR = lds_levels + (size_t)(kListWaves + wid) * levels * kWave;
    int i_next = 0, i_end = 0;          // the wave's claimed run of arcs
    for (;;) {
        if (i_next >= i_end) {
            int i0 = 0;
            if (lane == 0) i0 = atomicAdd(P.cursor, P.chunk);
            i0 = __shfl(i0, 0, kWave);
            i_next = i0;
            i_end = i0 + P.chunk;
        }
        const int j = i_next++;
        if (j >= P.n_arcs) break;
        // claim j lists arc j * stride mod n_arcs (stride coprime to
        // n_arcs): a run of claims spreads over the list, so the arcs of one
        // heavy vertex, adjacent in DAG order, do not land in one wave's run
        const int i = (int)(((long long)j * P.stride) % P.n_arcs);
        const int e = P.arcs[i];
        const int u = P.dag_src[e];
        const int a0 = P.dag_ptr[u];
        const int d = P.dag_ptr[u + 1] - a0;
        const int r = e - a0;
        const long long slot0 = P.offsets[i];
        const long long slot_n = P.offsets[i + 1] - slot0;
        long long done = 0;                     // cliques of this arc written so far
        if (lane == 0) {
            sPre[wid][0] = u;
            sPre[wid][1] = P.dag_col[e];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if (k == 2) {
            if (lane == 0) {
                if (slot_n >= 1) {
                    P.out[2 * slot0] = u;
                    P.out[2 * slot0 + 1] = P.dag_col[e];
                } else {
                    atomicOr(P.err, 1);
                }
            }
            done = 1;
        } else {
            const int W = (d + 63) >> 6;
            const u64* __restrict__ rows = P.rows + P.rows_off[u];
            // level 0: the arc's candidate set C_uv, k - 2 vertices to choose
            u64 M = lane < W ? rows[(long long)r * W + lane] : 0ull;
            u64 R = M;
            int t = 0;                          // level; k - 2 - t vertices still to choose
            for (;;) {
                const int need = k - 2 - t;
                if (need == 1) {
                    // every candidate of M completes a clique
                    int before = 0;
                    for (int w = 0; w < W; ++w) {
                        const u64 mw = readlane64(M, w);
                        const int pc = __popcll(mw);
                        for (int j0 = 0; j0 < pc; j0 += kWave) {
                            const int j = j0 + lane;
                            if (j < pc) {
                                const long long idx = done + before + j;
                                const int x = w * 64 + select64(mw, j);
                                if (idx < slot_n) {
                                    int32_t* o = P.out + (slot0 + idx) * k;
                                    for (int c = 0; c < k - 1; ++c) o[c] = sPre[wid][c];
                                    o[k - 1] = P.dag_col[a0 + x];
                                } else {
                                    atomicOr(P.err, 1);
                                }
                            }
                        }
                        before += pc;
                    }
                    done += before;
                    R = 0ull;                   // node finished
                }
                // next candidate of this level, or back up
                const u64 b = __ballot(R != 0ull);
                if (b == 0ull) {
                    if (t == 0) break;
                    --t;
                    M = sM[t * kWave + lane];
                    R = sR[t * kWave + lane];
                    continue;
                }
                const int f = __builtin_ctzll(b);
                const u64 Rf = readlane64(R, f);
                const int x = f * 64 + __builtin_ctzll(Rf);
                if (lane == f) R &= R - 1;
                const u64 ch = M & (lane < W ? rows[(long long)x * W + lane] : 0ull);
                int cc = __popcll(ch);
#pragma unroll
                for (int o = kWave / 2; o > 0; o >>= 1) cc += __shfl_xor(cc, o, kWave);
                if (cc >= need - 1) {
                    // descend: the level's state is kept for the way back
                    sM[t * kWave + lane] = M;
                    sR[t * kWave + lane] = R;
                    if (lane == 0) sPre[wid][2 + t] = P.dag_col[a0 + x];
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    ++t;
                    M = ch;
                    R = ch;
                }
            }
        }
        if (lane == 0 && done != slot_n) atomicOr(P.err, 2);
        __builtin_amdgcn_wave_barrier();
    }
}

hipError_t launch_list_arcs(const ListParams& P, int32_t blocks, hipStream_t s)
{
    if (P.n_arcs <= 0) return hipSuccess;
    if (P.k < 2 || P.k > kListMaxK) return hipErrorInvalidValue;
    const size_t lds = 2 * (size_t)kListWaves * list_levels(P.k) * kWave * sizeof(u64);
    // arcs claimed per atomic on the shared cursor (its atomics are
    // serialised): runs of up to 16 arcs, about eight claims per wave
    ListParams Q = P;
    const int64_t waves = (int64_t)blocks * kListWaves;
    int64_t c = (int64_t)P.n_arcs / (waves * 8);
    c = c < 1 ? 1 : (c > 16 ? 16 : c);
    if ((int64_t)P.n_arcs + waves * c >= (1ll << 31)) c = 1;
    Q.chunk = (int32_t)c;
    // a stride near 0.618 n_arcs (consecutive claims then land far apart,
    // as in Fibonacci hashing) that shares no factor with n_arcs
    int64_t st = 1;
    if (c > 1) {
        for (int64_t t = (int64_t)(0.6180339887 * P.n_arcs); t < P.n_arcs; ++t)
            if (std::gcd(t, (int64_t)P.n_arcs) == 1) {
                st = t;
                break;
            }
    }
    Q.stride = (int32_t)st;
    list_arcs_kernel<<<blocks, kListBlock, lds, s>>>(Q);
    return hipGetLastError();
}

// ------------------------------------------------------- 64-bit exclusive scan

namespace {
constexpr int kScan64Block = 256;
constexpr int kScan64Per = 8;
constexpr int kScan64Tile = kScan64Block * kScan64Per;

__device__ long long block_exclusive_scan64(long long v, long long* total)
{
    __shared__ long long wsum[kScan64Block / kWave];
    const int lane = lane_of(), wid = threadIdx.x / kWave;
    long long inc = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const long long t = __shfl_up(inc, o, kWave);
        if (lane >= o) inc += t;
    }
    if (lane == kWave - 1) wsum[wid] = inc;
    __syncthreads();
    long long off = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kScan64Block / kWave; ++w) {
        if (w < wid) off += wsum[w];
        tot += wsum[w];
    }
    __syncthreads();
    *total = tot;
    return off + inc - v;
}
}  // namespace

__global__ void scan64_tile_sums_kernel(const u64* __restrict__ in, int64_t n, long long* __restrict__ sums)
{
    const int64_t base = (int64_t)blockIdx.x * kScan64Tile + (int64_t)threadIdx.x * kScan64Per;
    long long s = 0;
#pragma unroll
    for (int i = 0; i < kScan64Per; ++i)
        if (base + i < n) s += (long long)in[base + i];
    long long tot;
    block_exclusive_scan64(s, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ void scan64_tiles_kernel(const u64* __restrict__ in, int64_t n, const long long* __restrict__ tile_off,
                                    long long* __restrict__ out)
{
    const int64_t base = (int64_t)blockIdx.x * kScan64Tile + (int64_t)threadIdx.x * kScan64Per;
    long long vals[kScan64Per];
    long long s = 0;
#pragma unroll
    for (int i = 0; i < kScan64Per; ++i) {
        vals[i] = (base + i < n) ? (long long)in[base + i] : 0;
        s += vals[i];
    }
    long long tot;
    long long run = block_exclusive_scan64(s, &tot) + (tile_off ? tile_off[blockIdx.x] : 0);
#pragma unroll
    for (int i = 0; i < kScan64Per; ++i) {
        if (base + i < n) out[base + i] = run;
        run += vals[i];
    }
    if (n > 0 && base <= n - 1 && n - 1 < base + kScan64Per) out[n] = run;
    if (n == 0 && blockIdx.x == 0 && threadIdx.x == 0) out[0] = tile_off ? tile_off[0] : 0;
}

size_t scan64_workspace(int64_t n)
{
    if (n <= kScan64Tile) return 1;
    const int64_t tiles = (n + kScan64Tile - 1) / kScan64Tile;
    return (size_t)(2 * tiles + 1) + scan64_workspace(tiles);
}

// out[0..n] = exclusive prefix sums of in[0..n) (out[n] = total); in holds
// non-negative counts below 2^63 in total.  ws: scan64_workspace(n) words.
hipError_t scan_exclusive64(const u64* in, long long* out, int64_t n, long long* ws, hipStream_t s)
{
    if (n <= kScan64Tile) {
        scan64_tiles_kernel<<<1, kScan64Block, 0, s>>>(in, n, nullptr, out);
        return hipGetLastError();
    }
    const int64_t tiles = (n + kScan64Tile - 1) / kScan64Tile;
    long long* sums = ws;
    long long* offs = ws + tiles;
    scan64_tile_sums_kernel<<<(unsigned)tiles, kScan64Block, 0, s>>>(in, n, sums);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // the tile sums are scanned as unsigned words holding non-negative values
    e = scan_exclusive64(reinterpret_cast<const u64*>(sums), offs, tiles, ws + 2 * tiles + 1, s);
    if (e != hipSuccess) return e;
    scan64_tiles_kernel<<<(unsigned)tiles, kScan64Block, 0, s>>>(in, n, offs, out);
    return hipGetLastError();
}

}  // namespace citron
