// Counting phase of the degree-ordered k-clique counter (Lonkar & Beamer,
// Section III Algorithm 2, Section V-B heuristics), as one persistent HIP
// kernel for gfx950.
//
// Input: the subgraph rows built once per graph (kernels_rows.hip): for an
// arc u -> v_i, row i of u is the candidate mask C_uv over the positions of
// N->(u).  The k-cliques whose two lowest vertices (in the degree ordering)
// are u and v_i are the (k-2)-cliques of the subgraph induced on C_uv; they
// are counted by depth-first recursion over masks M' = M AND row_x, with the
// last level summing popcounts only (degrees-only heuristic) and masks too
// small for the rest of the clique pruned (size heuristic).
//
// Scheduling.  Every wave works on its own and pulls items from one global
// cursor: first the arcs of heavy vertices (out-degree > 64) in order of
// |C_uv|, largest first, then the light vertices (out-degree <= 64).
//
// Engines.  Light work -- subgraphs with at most 64 vertices, one 64-bit
// word per row -- is searched by the light engine: one depth-first search
// per lane over one first-level branch at a time, rows in the wave's LDS
// buffer.  A heavy arc is walked by the whole wave in step (lane q holding
// word q of each mask, rows read from device memory) until a node has at
// most 64 candidates; that node's induced subgraph is then compacted to one
// word per row and queued in the wave's LDS buffer for the light engine.
//
// Exact arithmetic: per-lane uint64 accumulators (a lane adds at most 64 per
// step and cannot run 2^58 steps, so these never wrap); wave sums and the
// global accumulator are carry-checked, and a carry sets the query's
// overflow flag.
#include "kernels.h"

namespace citron {

typedef unsigned long long u64;

constexpr int kMaxBlock = 512;          // threads per count workgroup (8 waves)
constexpr int kWaveBufRows = 256;       // one-word rows queued per wave
constexpr int kLdsStackLevels = 8;      // deeper stacks (k > 12) live in device memory
constexpr int kArcMaxC = 256;           // heavy arcs with |C_uv| <= this are copied to LDS
constexpr int kArcWords = kArcMaxC * (kArcMaxC / 64);   // 8 KB per wave
constexpr int kLaneMaxWords = 4;        // multi-word masks a lane holds in registers
constexpr int kDonateMinIdle = 8;       // idle lanes that trigger work donation
constexpr int kBurstIters = 32;         // last-level steps of one leaf burst at most
constexpr int kBurstMinLanes = 32;      // lanes at a last-level node to keep a burst going

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ int lane_of() { return threadIdx.x & (kWave - 1); }

__device__ __forceinline__ u64 shfl64(u64 v, int src)
{
    unsigned lo = __shfl((unsigned)v, src, kWave);
    unsigned hi = __shfl((unsigned)(v >> 32), src, kWave);
    return ((u64)hi << 32) | lo;
}

__device__ __forceinline__ u64 readlane64(u64 v, int lane)
{
    unsigned lo = __builtin_amdgcn_readlane((unsigned)v, lane);
    unsigned hi = __builtin_amdgcn_readlane((unsigned)(v >> 32), lane);
    return ((u64)hi << 32) | lo;
}

// Sum over the wave of per-lane values in 0..127, from seven ballots (no
// LDS traffic, no cross-lane shuffles).
__device__ __forceinline__ int wave_sum_small(int v)
{
    int s = 0;
#pragma unroll
    for (int b = 0; b < 7; ++b) s += __popcll(__ballot((v >> b) & 1)) << b;
    return s;
}

__device__ __forceinline__ u64 wave_sum_u64(u64 v)
{
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += shfl64(v, lane_of() ^ o);
    return v;
}

// Wave-wide carry-checked reduction; lane 0 adds the total to *dst.
__device__ void wave_flush(u64 acc, int ovf, u64* dst, int32_t* ovf_dst)
{
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        const u64 other = shfl64(acc, lane_of() ^ o);
        ovf |= __shfl_xor(ovf, o, kWave);
        const u64 s = acc + other;
        ovf |= (s < acc) ? 1 : 0;
        acc = s;
    }
    if (lane_of() == 0) {
        if (acc) {
            const u64 old = atomicAdd(dst, acc);
            if (old + acc < old) ovf = 1;
        }
        if (ovf) atomicOr(ovf_dst, 1);
    }
}

__device__ __forceinline__ void wave_flush_stats(const u64* vals, u64* dst)
{
#pragma unroll
    for (int i = 0; i < kNumStats; ++i) {
        if ((i >= kStatWaveBusy && i <= kStatWaves) || i >= kStatWaveBusyMax) continue;   // written once per wave
        const u64 v = wave_sum_u64(vals[i]);
        if (lane_of() == 0 && v) atomicAdd(dst + i, v);
    }
}

// Position of the r-th (0-based) set bit of v; always in 0..63.
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

// A W-word mask held one word per lane (lane w holds word w, lanes >= W
// hold 0).  Returns, in lane j, the position of the j-th set bit (for j
// below the popcount).  Uniform control flow: the whole wave calls it.
__device__ __forceinline__ int wave_select(u64 m, int j, int W)
{
    int before = 0, my_w = 0, my_r = 0;
    u64 my_word = 0;
    for (int w = 0; w < W; ++w) {
        const u64 mw = readlane64(m, w);
        const int pc = __popcll(mw);
        const bool here = j >= before && j < before + pc;
        my_w = here ? w : my_w;
        my_r = here ? j - before : my_r;
        my_word = here ? mw : my_word;
        before += pc;
    }
    return my_w * 64 + select64(my_word, my_r);
}

// ------------------------------------------------------------------ layout

__host__ __device__ inline int stack_levels(int max_k) { return max_k > 4 ? max_k - 4 : 1; }
__host__ __device__ inline bool stack_in_lds(int max_k) { return stack_levels(max_k) <= kLdsStackLevels; }
// per wave: four stacks (light M/R, heavy M/R) of levels x 64 words
__host__ __device__ inline int64_t wave_stack_words(int max_k) { return 4ll * stack_levels(max_k) * kWave; }
__host__ __device__ inline int wave_lds_bytes(int max_k)
{
    int b = 8 * kWaveBufRows + 4 * kWaveBufRows + 4 * kWaveBufRows;   // rows, meta, tags
    b += 8 * kArcWords;                                               // arc subgraph copy
    b += 32 * kWave;                                                  // donation mailbox
    b += 4 * kWaveBufRows;                                            // unit list
    if (stack_in_lds(max_k)) b += 8 * (int)wave_stack_words(max_k);
    return b;
}

int32_t count_lds_bytes(int32_t, int32_t max_k, int32_t wg_waves)
{
    return wg_waves * wave_lds_bytes(max_k);
}

int64_t count_scratch_words(int32_t, int32_t max_k, int32_t wg_waves)
{
    if (stack_in_lds(max_k)) return 0;
    return ((int64_t)wg_waves * wave_stack_words(max_k) + 31) & ~31ll;
}

// ------------------------------------------------------------ light engine
//
// Depth-first search with one 64-bit mask per level and one independent
// search per lane.  A unit is one row of a queued subgraph: choosing the
// row's vertex leaves `need` more vertices to choose from the row's mask.
// A lane that finishes a unit takes the next one at once.

struct Acc {
    u64 acc;
    int ovf;
    u64 st[kNumStats];   // per-lane work counters (instrumented launches only)
};

struct WaveBuf {
    u64* arc;        // LDS copy of one heavy arc's subgraph (multi-word rows)
    u64* mbox;       // donation mailbox: per lane M, R, and (need, base, tag)
    u64* rows;
    int32_t* meta;   // (first row of the subgraph << 8) | need
    int32_t* tags;   // arc of the unit (per-arc output)
    u64* sM;         // light stacks
    u64* sR;
    u64* hM;         // heavy stacks
    u64* hR;
    int32_t* units;  // rows that are search roots (a part of a split arc uses some rows only)
    int n;           // rows in use (wave-uniform)
    int nu;          // units in use (wave-uniform)
};

template <bool kStats, bool kPerArc>
__device__ __forceinline__ void light_engine(const WaveBuf& wb, Acc& A, u64* __restrict__ per_arc)
{
    const int lane = lane_of();
    const u64 lt_mask = lane == 0 ? 0ull : (~0ull >> (kWave - lane));
    const u64* __restrict__ rows = wb.rows;
    u64* __restrict__ sM = wb.sM;
    u64* __restrict__ sR = wb.sR;
    const int nunits = wb.nu;
    int next = 0;                      // wave-uniform unit counter
    bool active = false;
    u64 M = 0, R = 0, uacc = 0;
    int t = 0, need = 0, base = 0, tag = 0;
    for (;;) {
        const u64 want = __ballot(!active);
        if (want && next < nunits) {
            const int u = next + __popcll(want & lt_mask);
            next += __popcll(want);
            if (!active && u < nunits) {
                const int row = wb.units[u];
                const int mt = wb.meta[row];
                const u64 m1 = rows[row];
                base = mt >> 8;
                need = mt & 255;
                const int c = __popcll(m1);
                if (kStats) A.st[kStatLightUnits] += 1;
                if (kPerArc) tag = wb.tags[row];
                if (need == 1) {
                    A.acc += (u64)c;
                    if (kPerArc && c) atomicAdd(per_arc + tag, (u64)c);
                } else if (c >= need) {
                    M = m1;
                    R = m1;
                    t = 1;
                    uacc = 0;
                    active = true;
                }
            }
        }
        const u64 act = __ballot(active);
        if (act == 0ull) {
            if (next >= nunits) break;
            continue;
        }
        if (next >= nunits && __popcll(~act) >= kDonateMinIdle) {
            // work donation: no unit is left and lanes are idle, so every busy
            // lane offers the upper half of the remaining candidates of its
            // shallowest level that still holds real work; idle lanes take
            // them as new search roots (counts only depend on the subtree)
            int lvl = 0;
            u64 Ml = 0ull, Rl = 0ull;
            if (active) {
                for (int l = 1; l <= t; ++l) {
                    const u64 r = (l == t) ? R : sR[(l - 1) * kWave + lane];
                    const int pc = __popcll(r);
                    if (pc >= 2 && (need + (t - l) >= 3 || pc >= 8)) {
                        lvl = l;
                        Rl = r;
                        Ml = (l == t) ? M : sM[(l - 1) * kWave + lane];
                        break;
                    }
                }
            }
            const u64 donors = __ballot(lvl > 0);
            if (donors) {
                const u64 idle = ~act;
                const int np = min(__popcll(donors), __popcll(idle));
                if (lvl > 0) {
                    const int r = __popcll(donors & lt_mask);
                    if (r < np) {
                        const int recv = select64(idle, r);
                        const int p = select64(Rl, __popcll(Rl) / 2);
                        const u64 low = Rl & ((1ull << p) - 1);
                        if (lvl == t) R = low;
                        else sR[(lvl - 1) * kWave + lane] = low;
                        u64* mb = wb.mbox + 4 * recv;
                        mb[0] = Ml;
                        mb[1] = Rl & ~low;
                        mb[2] = ((u64)(unsigned)base << 32) | (unsigned)(need + (t - lvl));
                        mb[3] = (u64)(unsigned)tag;
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                if (!active && __popcll(idle & lt_mask) < np) {
                    const u64* mb = wb.mbox + 4 * lane;
                    M = mb[0];
                    R = mb[1];
                    need = (int)(unsigned)mb[2];
                    base = (int)(mb[2] >> 32);
                    tag = (int)(unsigned)mb[3];
                    t = 1;
                    uacc = 0;
                    active = true;
                    if (kStats) A.st[kStatDonations] += 1;
                }
                __builtin_amdgcn_wave_barrier();
            }
        }
        if (kStats && lane == 0) {
            A.st[kStatLightIters] += 1;
            A.st[kStatLightActive] += (u64)__popcll(act);
        }
        if (active) {
            if (R != 0ull) {
                if (need == 2) {
                    // degrees-only last level, two candidates per step
                    const int x1 = __builtin_ctzll(R);
                    R &= R - 1;
                    const u64 r1 = rows[base + x1];
                    u64 r2 = 0ull;
                    int two = 0;
                    if (R != 0ull) {
                        const int x2 = __builtin_ctzll(R);
                        R &= R - 1;
                        r2 = rows[base + x2];
                        two = 1;
                    }
                    const u64 c = (u64)(__popcll(M & r1) + __popcll(M & r2));
                    A.acc += c;
                    if (kPerArc) uacc += c;
                    if (kStats) A.st[kStatWordOps] += 1 + two;
                } else {
                    const int x = __builtin_ctzll(R);
                    R &= R - 1;
                    const u64 nm = M & rows[base + x];
                    if (__popcll(nm) >= need - 1) {
                        sM[(t - 1) * kWave + lane] = M;
                        sR[(t - 1) * kWave + lane] = R;
                        M = nm;
                        R = nm;
                        ++t;
                        --need;
                        if (kStats) A.st[kStatPushes] += 1;
                    }
                }
            }
            if (need == 2 && R != 0ull) {
                // leaf burst: while most lanes sit at a last-level node, run
                // only last-level steps, two candidates at a time
                for (int it = 0; it < kBurstIters; ++it) {
                    const bool leaf = R != 0ull;
                    if (__popcll(__ballot(leaf)) < kBurstMinLanes) break;
                    if (leaf) {
                        const int x1 = __builtin_ctzll(R);
                        R &= R - 1;
                        const u64 r1 = rows[base + x1];
                        u64 r2 = 0ull;
                        int two = 0;
                        if (R != 0ull) {
                            const int x2 = __builtin_ctzll(R);
                            R &= R - 1;
                            r2 = rows[base + x2];
                            two = 1;
                        }
                        const u64 c = (u64)(__popcll(M & r1) + __popcll(M & r2));
                        A.acc += c;
                        if (kPerArc) uacc += c;
                        if (kStats) A.st[kStatWordOps] += 1 + two;
                    }
                }
            }
            if (R == 0ull) {
                if (t == 1) {
                    active = false;
                    if (kPerArc && uacc) atomicAdd(per_arc + tag, uacc);
                } else {
                    --t;
                    ++need;
                    if (kStats) A.st[kStatLightPops] += 1;
                    M = sM[(t - 1) * kWave + lane];
                    R = sR[(t - 1) * kWave + lane];
                }
            }
        }
    }
}

template <bool kStats, bool kPerArc>
__device__ __forceinline__ void flush_tasks(WaveBuf& wb, Acc& A, u64* per_arc)
{
    if (wb.n == 0) return;
    if (kStats && lane_of() == 0) A.st[kStatFlushes] += 1;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    light_engine<kStats, kPerArc>(wb, A, per_arc);
    __builtin_amdgcn_wave_barrier();
    wb.n = 0;
    wb.nu = 0;
}

// ------------------------------------------------------------ heavy engine

struct HeavyCtx {
    const u64* __restrict__ rows;   // the source vertex's rows in device memory
    int W;                          // words per row
    int L;                          // vertices of the clique inside the subgraph (k - 1)
    int tag;                        // the arc (per-arc output)
};

// Handle a node with mask m (c candidates, `need` more vertices to choose).
// Returns true when the caller must search it depth first (c > 64 and
// need >= 3).
template <bool kStats, bool kPerArc, bool kGlobal>
__device__ __forceinline__ void heavy_dfs(const HeavyCtx& H, u64 M, int need0, int lvl0, int part, int P,
                                          WaveBuf& wb, Acc& A, u64& uacc, u64* per_arc);

// Copy the subgraph induced on the c candidates of m (rows in H, device
// memory) to the wave's LDS buffer, compacted to W2 = ceil(c/64) words per
// row: lane a rebuilds row a by extracting, word by word, the bits at the
// candidates' positions.  c <= kArcMaxC.
__device__ __forceinline__ int copy_to_lds(const HeavyCtx& H, u64 M, int c, u64* __restrict__ dst)
{
    const int q = lane_of();
    const int W2 = (c + 63) >> 6;
    for (int a0 = 0; a0 < c; a0 += kWave) {
        const int a = a0 + q;
        const int xa = wave_select(M, a, H.W);
        const u64* __restrict__ src = H.rows + (int64_t)(a < c ? xa : 0) * H.W;
        unsigned o[8] = {0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};
        int b = 0;
        for (int w = 0; w < H.W; ++w) {
            u64 mw = readlane64(M, w);
            if (mw == 0ull) continue;
            const u64 word = a < c ? src[w] : 0ull;
            const unsigned wlo = (unsigned)word, whi = (unsigned)(word >> 32);
            while (mw) {
                const int p = __builtin_ctzll(mw);
                mw &= mw - 1;
                const unsigned bit = ((p < 32 ? wlo : whi) >> (p & 31)) & 1u;
#pragma unroll
                for (int h = 0; h < 8; ++h)
                    if ((b >> 5) == h) o[h] |= bit << (b & 31);
                ++b;
            }
        }
        if (a < c)
            for (int i = 0; i < W2; ++i) dst[a * W2 + i] = ((u64)o[2 * i + 1] << 32) | o[2 * i];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    return W2;
}

// Handle a node with mask m (c candidates, `need` more vertices to choose;
// rows in device memory when kGlobal, else in the wave's LDS copy).  Returns
// true when the caller must search it depth first.  lvl is the first free
// level of the heavy stacks.  Only first-level branches j = part (mod P)
// of the node are taken (P > 1 at the root of a split arc only).
template <bool kStats, bool kPerArc, bool kGlobal>
__device__ __forceinline__ bool heavy_node(const HeavyCtx& H, u64 m, int c, int need, int lvl, int part, int P,
                                           WaveBuf& wb, Acc& A, u64& uacc, u64* per_arc)
{
    const int lane = lane_of();
    if (c < need) return false;
    if (need == 1) {
        if (lane == 0) {
            A.acc += (u64)c;
            if (kPerArc) uacc += (u64)c;
        }
        return false;
    }
    if (need == 2) {
        // degrees-only last level on multi-word rows: lanes over candidates
        for (int j0 = 0; j0 < c; j0 += kWave) {
            const int j = j0 + lane;
            const int x = wave_select(m, j, H.W);
            u64 s = 0;
            if (j < c) {
                const u64* __restrict__ rx = H.rows + (int64_t)x * H.W;
                for (int w = 0; w < H.W; ++w) s += (u64)__popcll(readlane64(m, w) & rx[w]);
            }
            A.acc += s;
            if (kPerArc) uacc += s;
            if (kStats && j < c) {
                A.st[kStatWordOps] += H.W;
                A.st[kStatHeavyLeafCand] += 1;
            }
        }
        return false;
    }
    if (need == 3 && c > kWave && H.W <= kLaneMaxWords) {
        // two levels left, many candidates: lane j takes the j-th candidate
        // x, forms its child mask m AND row_x (at most 4 words, in
        // registers) and sums the last level of that child itself
        const int nj = (c - part + P - 1) / P;
        for (int j0 = 0; j0 < nj; j0 += kWave) {
            const int jj = j0 + lane;
            const int j = jj < nj ? part + P * jj : c;
            const int x = wave_select(m, j, H.W);
            u64 ch[kLaneMaxWords];
            const u64* __restrict__ rx = H.rows + (int64_t)(j < c ? x : 0) * H.W;
#pragma unroll
            for (int w = 0; w < kLaneMaxWords; ++w) {
                ch[w] = 0ull;
                if (w < H.W) {
                    const u64 mw = readlane64(m, w);
                    if (j < c) ch[w] = mw & rx[w];
                }
            }
            u64 s = 0;
            u64 ops = 0;
#pragma unroll
            for (int w = 0; w < kLaneMaxWords; ++w) {
                if (w >= H.W) break;
                u64 r = ch[w];
                while (r != 0ull) {
                    const int y = w * 64 + __builtin_ctzll(r);
                    r &= r - 1;
                    const u64* __restrict__ ry = H.rows + (int64_t)y * H.W;
                    int cnt = 0;
#pragma unroll
                    for (int i = 0; i < kLaneMaxWords; ++i)
                        if (i < H.W) cnt += __popcll(ch[i] & ry[i]);
                    s += (u64)cnt;
                    if (kStats) ops += H.W;
                }
            }
            A.acc += s;
            if (kPerArc) uacc += s;
            if (kStats) {
                A.st[kStatWordOps] += ops;
                if (j < c) A.st[kStatNeed3Lanes] += 1;
            }
        }
        return false;
    }
    if (kGlobal && need >= 3 && c <= kArcMaxC && c > kWave) {
        // continue from an LDS copy of this node's subgraph
        const int W2 = copy_to_lds(H, m, c, wb.arc);
        const HeavyCtx HL{wb.arc, W2, H.L, H.tag};
        const int rem = c - 64 * lane;
        const u64 all = lane < W2 ? (rem >= 64 ? ~0ull : ((1ull << rem) - 1)) : 0ull;
        if (kStats && lane == 0) A.st[kStatArcLds] += 1;
        if (heavy_node<kStats, kPerArc, false>(HL, all, c, need, lvl, part, P, wb, A, uacc, per_arc))
            heavy_dfs<kStats, kPerArc, false>(HL, all, need, lvl, part, P, wb, A, uacc, per_arc);
        __builtin_amdgcn_wave_barrier();
        return false;
    }
    if (c <= kWave) {
        // compaction: lane a rebuilds row a over the c candidates by
        // extracting, word by word, the bits at the candidates' positions
        if (wb.n + c > kWaveBufRows) flush_tasks<kStats, kPerArc>(wb, A, per_arc);
        const int xa = wave_select(m, lane, H.W);
        const u64* __restrict__ ra = H.rows + (int64_t)(lane < c ? xa : 0) * H.W;
        unsigned nlo = 0, nhi = 0;
        int b = 0;
        for (int w = 0; w < H.W; ++w) {
            u64 mw = readlane64(m, w);
            if (mw == 0ull) continue;
            const u64 word = lane < c ? ra[w] : 0ull;
            const unsigned wlo = (unsigned)word, whi = (unsigned)(word >> 32);
            while (mw) {
                const int p = __builtin_ctzll(mw);
                mw &= mw - 1;
                const unsigned bit = ((p < 32 ? wlo : whi) >> (p & 31)) & 1u;
                if (b < 32) nlo |= bit << b;
                else nhi |= bit << (b - 32);
                ++b;
            }
        }
        if (lane < c) {
            wb.rows[wb.n + lane] = ((u64)nhi << 32) | nlo;
            wb.meta[wb.n + lane] = (wb.n << 8) | (need - 1);
            if (kPerArc) wb.tags[wb.n + lane] = H.tag;
        }
        const bool unit = lane < c && (P == 1 || lane % P == part);
        const u64 um = __ballot(unit);
        if (unit) wb.units[wb.nu + __popcll(um & (lane == 0 ? 0ull : (~0ull >> (kWave - lane))))] = wb.n + lane;
        wb.nu += __popcll(um);
        wb.n += c;
        if (kStats && lane == 0) {
            A.st[kStatCompactions] += 1;
            A.st[kStatCompactRows] += (u64)c;
        }
        return false;
    }
    return true;
}

// Depth-first search, all lanes in step, below a node with mask M (more
// than 64 candidates, need0 more vertices), rows in H; stack levels from lvl0.
template <bool kStats, bool kPerArc, bool kGlobal>
__device__ __forceinline__ void heavy_dfs(const HeavyCtx& H, u64 M, int need0, int lvl0, int part, int P,
                                          WaveBuf& wb, Acc& A, u64& uacc, u64* per_arc)
{
    const int q = lane_of();
    u64 R = M;
    int t = 1;
    int jroot = 0;
    for (;;) {
        const u64 b = __ballot(R != 0ull);
        if (b == 0ull) {
            if (t == 1) break;
            --t;
            M = wb.hM[(lvl0 + t - 1) * kWave + q];
            R = wb.hR[(lvl0 + t - 1) * kWave + q];
            continue;
        }
        const int f = __builtin_ctzll(b);
        const u64 Rf = readlane64(R, f);
        const int x = f * 64 + __builtin_ctzll(Rf);
        if (q == f) R &= R - 1;
        if (t == 1) {
            const int jr = jroot++;
            if (P > 1 && jr % P != part) continue;
        }
        const u64 ch = M & (q < H.W ? H.rows[(int64_t)x * H.W + q] : 0ull);
        const int cc = wave_sum_small(__popcll(ch));
        if (kStats && q == 0) A.st[kStatHeavySteps] += 1;
        if (heavy_node<kStats, kPerArc, kGlobal>(H, ch, cc, need0 - t, lvl0 + t, 0, 1, wb, A, uacc, per_arc)) {
            wb.hM[(lvl0 + t - 1) * kWave + q] = M;
            wb.hR[(lvl0 + t - 1) * kWave + q] = R;
            M = ch;
            R = ch;
            ++t;
            if (kStats && q == 0) A.st[kStatPushes] += 1;
        }
    }
}

template <bool kStats, bool kPerArc>
__device__ __forceinline__ void heavy_arc(const HeavyCtx& H, int r, int part, int P, WaveBuf& wb, Acc& A,
                                          u64* per_arc)
{
    const int q = lane_of();
    u64 uacc = 0;
    const u64 M = q < H.W ? H.rows[(int64_t)r * H.W + q] : 0ull;
    const int c = wave_sum_small(__popcll(M));
    const int need = H.L - 1;
    if (heavy_node<kStats, kPerArc, true>(H, M, c, need, 0, part, P, wb, A, uacc, per_arc))
        heavy_dfs<kStats, kPerArc, true>(H, M, need, 0, part, P, wb, A, uacc, per_arc);
    if (kPerArc) {
        const u64 s = wave_sum_u64(uacc);
        if (q == 0 && s) atomicAdd(per_arc + H.tag, s);
    }
}

// --------------------------------------------------------------- the kernel

struct KParams {
    const QueryDesc* queries;
    int32_t n_queries;
    int32_t total_items;
    int32_t* item_ctr;
    u64* scratch;
    int64_t scratch_words;
    int32_t max_k;
    int32_t flush_rows;     // a wave runs its queue once it holds this many rows
};

template <bool kLdsStack, bool kStats, bool kPerArc>
__global__ void __launch_bounds__(kMaxBlock) count_kernel(KParams P)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = lane_of();
    const int wid = threadIdx.x / kWave;
    const int nwaves = blockDim.x / kWave;
    const int levels = stack_levels(P.max_k);
    unsigned char* wbase = smem + wid * wave_lds_bytes(P.max_k);
    WaveBuf wb;
    wb.rows = reinterpret_cast<u64*>(wbase);
    wb.meta = reinterpret_cast<int32_t*>(wbase + 8 * kWaveBufRows);
    wb.tags = reinterpret_cast<int32_t*>(wbase + 12 * kWaveBufRows);
    wb.arc = reinterpret_cast<u64*>(wbase + 16 * kWaveBufRows);
    wb.mbox = reinterpret_cast<u64*>(wbase + 16 * kWaveBufRows + 8 * kArcWords);
    wb.units = reinterpret_cast<int32_t*>(wbase + 16 * kWaveBufRows + 8 * kArcWords + 32 * kWave);
    u64* stacks;
    if (kLdsStack) {
        stacks = reinterpret_cast<u64*>(wbase + 20 * kWaveBufRows + 8 * kArcWords + 32 * kWave);
    } else {
        stacks = P.scratch + (int64_t)blockIdx.x * P.scratch_words + (int64_t)wid * wave_stack_words(P.max_k);
    }
    (void)nwaves;
    wb.sM = stacks;
    wb.sR = stacks + (int64_t)levels * kWave;
    wb.hM = stacks + 2ll * levels * kWave;
    wb.hR = stacks + 3ll * levels * kWave;
    wb.n = 0;
    wb.nu = 0;

    Acc A;
    A.acc = 0ull;
    A.ovf = 0;
#pragma unroll
    for (int i = 0; i < kNumStats; ++i) A.st[i] = 0ull;
    int cur = -1;                      // query whose work the wave holds
    u64* per_arc = nullptr;
    const u64 t_start = kStats ? wall_clock64() : 0ull;
    u64 item_max = 0ull;

    for (;;) {
        int g = 0;
        if (lane == 0) g = atomicAdd(P.item_ctr, 1);
        g = __shfl(g, 0, kWave);
        if (g >= P.total_items) break;
        int qi = 0;
        {
            int lo = 0, hi = P.n_queries - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (P.queries[mid].item_begin <= g) lo = mid;
                else hi = mid - 1;
            }
            qi = lo;
        }
        const QueryDesc& q = P.queries[qi];
        if (qi != cur) {
            if (cur >= 0) {
                const QueryDesc& oq = P.queries[cur];
                flush_tasks<kStats, kPerArc>(wb, A, per_arc);
                wave_flush(A.acc, A.ovf, oq.acc, oq.overflow);
                if (kStats) wave_flush_stats(A.st, oq.stats);
                A.acc = 0ull;
                A.ovf = 0;
#pragma unroll
                for (int i = 0; i < kNumStats; ++i) A.st[i] = 0ull;
            }
            cur = qi;
            per_arc = q.per_arc;
        }
        const int i = q.item_lo + (g - q.item_begin);
        const int k = q.k;
        const u64 t_item = kStats ? wall_clock64() : 0ull;
        // the item: one part of a heavy arc, or (a part of) a light vertex
        int u, r = -1, part, nparts, tag;
        bool heavy;
        if (q.arc_list) {
            // list mode: one part of one listed arc; counts go to its list slot
            tag = q.arc_items[2 * i];
            const int pw = q.arc_items[2 * i + 1];
            const int e = q.arc_list[tag];
            u = q.dag_src[e];
            r = e - q.dag_ptr[u];
            part = pw & 0xffff;
            nparts = pw >> 16;
            heavy = q.dag_ptr[u + 1] - q.dag_ptr[u] > kLightMaxDeg;
        } else {
            // bucket holding item i, then the arc or vertex and the part (part-major)
            int lo = 0, hi = q.n_buckets - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (q.buckets[4 * mid] <= i) lo = mid;
                else hi = mid - 1;
            }
            const int key = q.buckets[4 * lo + 3] >> 1;
            heavy = (q.buckets[4 * lo + 3] & 1) == 0;
            const int cnt = q.buckets[4 * lo + 2];
            const int local = i - q.buckets[4 * lo];
            part = local / cnt;
            const int which = q.buckets[4 * lo + 1] + (local - part * cnt);
            if (heavy) {
                const int e = q.rows.harcs[which];
                u = q.dag_src[e];
                r = e - q.dag_ptr[u];
                nparts = arc_parts(key, k);
                tag = e;
            } else {
                u = q.order[q.light_first + which];
                nparts = light_parts(key + 1, k);
                tag = -1;
            }
        }
        const int a0 = q.dag_ptr[u];
        const int d = q.dag_ptr[u + 1] - a0;
        if (heavy) {
            HeavyCtx H{q.rows.rows + q.rows.rows_off[u], (d + 63) >> 6, k - 1, tag};
            heavy_arc<kStats, kPerArc>(H, r, part, nparts, wb, A, per_arc);
        } else {
            // rows of the vertex into the wave's buffer; the searched arcs
            // (every nparts-th one, or the one listed) become units
            if (wb.n + d > kWaveBufRows) flush_tasks<kStats, kPerArc>(wb, A, per_arc);
            if (lane < d) {
                wb.rows[wb.n + lane] = q.rows.rows[q.rows.rows_off[u] + lane];
                wb.meta[wb.n + lane] = (wb.n << 8) | (k - 2);
                if (kPerArc) wb.tags[wb.n + lane] = tag < 0 ? a0 + lane : tag;
            }
            const bool unit = lane < d && (r >= 0 ? lane == r : (nparts == 1 || lane % nparts == part));
            const u64 um = __ballot(unit);
            if (unit) wb.units[wb.nu + __popcll(um & (lane == 0 ? 0ull : (~0ull >> (kWave - lane))))] = wb.n + lane;
            wb.nu += __popcll(um);
            wb.n += d;
        }
        if (wb.n >= P.flush_rows) flush_tasks<kStats, kPerArc>(wb, A, per_arc);
        if (kStats && lane == 0) {
            const u64 dt = wall_clock64() - t_item;
            if (dt > (item_max >> 32)) item_max = (dt << 32) | (u64)(unsigned)g;
        }
    }
    if (cur >= 0) {
        const QueryDesc& oq = P.queries[cur];
        flush_tasks<kStats, kPerArc>(wb, A, per_arc);
        wave_flush(A.acc, A.ovf, oq.acc, oq.overflow);
        if (kStats) wave_flush_stats(A.st, oq.stats);
    }
    if (kStats && lane == 0) {
        // wave timing (instrumented single-query launches)
        const u64 t_end = wall_clock64();
        u64* st = P.queries[0].stats;
        atomicAdd(st + kStatWaveBusy, t_end - t_start);
        atomicMin(st + kStatWaveFirst, t_start);
        atomicMax(st + kStatWaveLast, t_end);
        atomicAdd(st + kStatWaves, 1ull);
        atomicMax(st + kStatWaveBusyMax, t_end - t_start);
        atomicMax(st + kStatItemMax, item_max);
    }
}

template <bool kLdsStack, bool kStats, bool kPerArc>
static hipError_t launch_variant(const KParams& P, const CountLaunch& cl, hipStream_t s)
{
    const void* fn = (const void*)count_kernel<kLdsStack, kStats, kPerArc>;
    if (cl.lds_bytes > 65536) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, cl.lds_bytes);
        if (e != hipSuccess) return e;
    }
    count_kernel<kLdsStack, kStats, kPerArc><<<cl.blocks, cl.wg_waves * kWave, cl.lds_bytes, s>>>(P);
    return hipGetLastError();
}

hipError_t launch_count(const CountLaunch& cl, hipStream_t s)
{
    if (cl.total_items <= 0) return hipSuccess;
    if (cl.wg_waves < 1 || cl.wg_waves * kWave > kMaxBlock) return hipErrorInvalidValue;
    KParams P;
    P.queries = cl.queries;
    P.n_queries = cl.n_queries;
    P.total_items = cl.total_items;
    P.item_ctr = cl.item_ctr;
    P.scratch = cl.scratch;
    P.scratch_words = cl.scratch_words;
    P.max_k = cl.max_k;
    P.flush_rows = cl.flush_rows;
    const bool lds = stack_in_lds(cl.max_k);
    const int v = (lds ? 4 : 0) | (cl.stats ? 2 : 0) | (cl.per_arc ? 1 : 0);
    switch (v) {
    case 0: return launch_variant<false, false, false>(P, cl, s);
    case 1: return launch_variant<false, false, true>(P, cl, s);
    case 2: return launch_variant<false, true, false>(P, cl, s);
    case 3: return launch_variant<false, true, true>(P, cl, s);
    case 4: return launch_variant<true, false, false>(P, cl, s);
    case 5: return launch_variant<true, false, true>(P, cl, s);
    case 6: return launch_variant<true, true, false>(P, cl, s);
    default: return launch_variant<true, true, true>(P, cl, s);
    }
}

// ---------------------------------------------------------------- schedule

__global__ void plan_hist_kernel(int32_t n, const int32_t* __restrict__ dag_ptr, int32_t D,
                                 int32_t* __restrict__ hist)
{
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    int d = dag_ptr[u + 1] - dag_ptr[u];
    // bucket 0 holds out-degree D, bucket D-2 holds out-degree 2 (descending)
    if (d >= 2) atomicAdd(&hist[D - d], 1);
}

__global__ void plan_scatter_kernel(int32_t n, const int32_t* __restrict__ dag_ptr, int32_t D,
                                    int32_t* __restrict__ cursor, int32_t* __restrict__ order)
{
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    int d = dag_ptr[u + 1] - dag_ptr[u];
    if (d >= 2) order[atomicAdd(&cursor[D - d], 1)] = (int32_t)u;
}

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

__global__ void check_arcs_kernel(const int32_t* __restrict__ arcs, int32_t n, int64_t m, int32_t* __restrict__ err)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && (arcs[i] < 0 || (int64_t)arcs[i] >= m)) atomicOr(err, 1);
}

__global__ void gather_arc_c_kernel(const int32_t* __restrict__ arcs, int32_t n, const int32_t* __restrict__ arc_c,
                                    u64* __restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (u64)arc_c[arcs[i]];
}

// parts of each listed arc (heavy sources split as in the full schedule)
__global__ void list_parts_kernel(const int32_t* __restrict__ arcs, int32_t n, const int32_t* __restrict__ dag_src,
                                  const int32_t* __restrict__ dag_ptr, const int32_t* __restrict__ arc_c, int32_t k,
                                  int32_t* __restrict__ parts)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int e = arcs[i];
    const int u = dag_src[e];
    const int d = dag_ptr[u + 1] - dag_ptr[u];
    parts[i] = d > kLightMaxDeg ? arc_parts(arc_c[e], k) : 1;
}

__global__ void list_items_kernel(int32_t n, const int32_t* __restrict__ parts, const int32_t* __restrict__ offs,
                                  int32_t* __restrict__ items)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int P = parts[i];
    const int o = offs[i];
    for (int p = 0; p < P; ++p) {
        items[2 * (o + p)] = (int32_t)i;
        items[2 * (o + p) + 1] = p | (P << 16);
    }
}

hipError_t launch_list_parts(const int32_t* arcs, int32_t n, const int32_t* dag_src, const int32_t* dag_ptr,
                             const int32_t* arc_c, int32_t k, int32_t* parts, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    list_parts_kernel<<<(n + 255) / 256, 256, 0, s>>>(arcs, n, dag_src, dag_ptr, arc_c, k, parts);
    return hipGetLastError();
}

hipError_t launch_list_items(int32_t n, const int32_t* parts, const int32_t* offs, int32_t* items, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    list_items_kernel<<<(n + 255) / 256, 256, 0, s>>>(n, parts, offs, items);
    return hipGetLastError();
}

hipError_t launch_check_arcs(const int32_t* arcs, int32_t n, int64_t m, int32_t* err, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    check_arcs_kernel<<<(n + 255) / 256, 256, 0, s>>>(arcs, n, m, err);
    return hipGetLastError();
}

hipError_t launch_gather_arc_c(const int32_t* arcs, int32_t n, const int32_t* arc_c, u64* out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    gather_arc_c_kernel<<<(n + 255) / 256, 256, 0, s>>>(arcs, n, arc_c, out);
    return hipGetLastError();
}

__global__ void fill_i32_kernel(int32_t* p, int32_t v, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

__global__ void fill_u64_kernel(u64* p, u64 v, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    fill_i32_kernel<<<(unsigned)blocks, 256, 0, s>>>(p, v, n);
    return hipGetLastError();
}

hipError_t launch_fill_u64(u64* p, u64 v, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    fill_u64_kernel<<<(unsigned)blocks, 256, 0, s>>>(p, v, n);
    return hipGetLastError();
}

hipError_t launch_plan(int32_t n, const int32_t* dag_ptr, int32_t max_outdeg, int32_t light_rows,
                       int32_t split_min_deg, int32_t split_factor, const PlanBuffers& pb,
                       int32_t* scan_ws, hipStream_t s)
{
    // D >= 2 keeps the bucket arithmetic valid for graphs without any
    // vertex of out-degree 2 or more (the plan is then empty).
    const int32_t D = max_outdeg > 2 ? max_outdeg : 2;
    hipError_t e = launch_fill_i32(pb.hist, 0, D + 1, s);
    if (e != hipSuccess) return e;
    const unsigned nb = (unsigned)((n + 255) / 256);
    if (n > 0) plan_hist_kernel<<<nb, 256, 0, s>>>(n, dag_ptr, D, pb.hist);
    // hist_scan[i] = vertices with out-degree > D - i (buckets 0..i-1)
    e = scan_exclusive(pb.hist, pb.hist_scan, D - 1, scan_ws, s);
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(pb.light_pre, pb.hist_scan, sizeof(int32_t) * (size_t)(D - 1),
                       hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
    if (n > 0) plan_scatter_kernel<<<nb, 256, 0, s>>>(n, dag_ptr, D, pb.light_pre, pb.order);
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
