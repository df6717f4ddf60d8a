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
// buffer, stacks in registers (k <= 8), LDS (k <= 12) or device memory.
// A heavy arc is walked by the whole wave in step (lane q holding word q of
// each mask).  A node with at most 256 candidates is copied to the wave's
// LDS, compacted to ceil(c/64) words per row; a node with at most 64
// candidates is compacted to one word per row and queued for the light
// engine; a node with two levels left and more than 64 candidates is
// finished lane-per-child from the LDS copy (need3_lanes).
//
// Exact arithmetic: per-lane uint64 accumulators (a lane adds at most 64 per
// step and cannot run 2^58 steps, so these never wrap; 32-bit partial sums
// are bounded where they are used); wave sums and the global accumulator
// are carry-checked, and a carry sets the query's overflow flag.
#include "kernels.h"

namespace citron {

typedef unsigned long long u64;

constexpr int kMaxBlock = 512;          // threads per count workgroup (8 waves)
constexpr int kWaveBufRows = 128;       // one-word rows queued per wave
constexpr int kLdsStackLevels = 8;      // deeper stacks (k > 12) live in device memory
constexpr int kArcMaxC = kArcLdsMax;    // LDS subgraph copies hold at most this many rows
constexpr int kLaneMaxWords = 4;        // multi-word masks a lane holds in registers
constexpr int kDonateMinIdle = 8;       // idle lanes that trigger work donation
constexpr int kBurstIters = 32;         // last-level steps of one leaf burst at most
constexpr int kBurstMinLanes = 32;      // lanes at a last-level node to keep a burst going
constexpr int kN3Burst = 8;             // two-level steps between refills of idle lanes
constexpr int kMaxClaim = 16;           // items a wave claims at once, at most
// donation mailbox per lane: M, R, (need, base), and the arc tag of per-arc launches
__host__ __device__ constexpr int mbox_words(bool per_arc) { return per_arc ? 4 : 3; }
constexpr int kPosList = 3 * kWave * 2; // candidate positions the smaller mailbox area holds (1.5 KB)
static_assert(kArcMaxC <= kPosList, "candidate positions of an LDS node fit the mailbox area");

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
        // written once per wave at its end
        if ((i >= kStatWaveBusy && i <= kStatWaves) || (i >= kStatWaveBusyMax && i <= kStatCycTotal)) continue;
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

// Where the search stacks live, by the largest k of a launch: light stacks
// in registers and heavy stacks in device memory (k <= 8: the heavy stacks
// are touched only when a heavy node is pushed or popped, and keeping them
// out of LDS lets more waves share a CU), all in LDS (k <= 12), or all in
// device memory.
constexpr int kRegLevels = 4;
enum StackMode { kStackReg = 0, kStackLds = 1, kStackGlobal = 2 };
__host__ __device__ inline int stack_mode(int max_k)
{
    const int l = stack_levels(max_k);
    return l <= kRegLevels ? kStackReg : (l <= kLdsStackLevels ? kStackLds : kStackGlobal);
}
// per wave: four stacks (light M/R, heavy M/R) of levels x 64 words
__host__ __device__ inline int64_t wave_stack_words(int max_k) { return 4ll * stack_levels(max_k) * kWave; }
// the part of them kept in device memory, per wave
__host__ __device__ inline int64_t wave_global_stack_words(int max_k)
{
    const int mode = stack_mode(max_k);
    return mode == kStackGlobal ? wave_stack_words(max_k) : (mode == kStackReg ? wave_stack_words(max_k) / 2 : 0);
}

// Largest LDS subgraph copy of a launch: nodes with 64 < c <= arc_max
// candidates, ceil(arc_max / 64) words per row.
__host__ __device__ inline int clamp_arc_max(int arc_max)
{
    return arc_max < kWave ? kWave : (arc_max > kArcMaxC ? kArcMaxC : arc_max);
}
__host__ __device__ inline int arc_copy_words(int arc_max)
{
    const int a = clamp_arc_max(arc_max);
    return a * ((a + 63) / 64);
}

// Per-wave LDS, in this order: queued rows (u64), their meta (i32), their
// arc tags (i32, per-arc launches only), the subgraph copy (u64), the
// donation mailbox (u64 per lane), the unit list (i32), the stacks kept in
// LDS.  Every part starts 8-byte aligned; the size is rounded to 16 bytes.
// The LDS per wave bounds the waves per CU (160 KB per CU), and the count
// kernel is latency-bound, so the layout is sized by what a launch uses.
__host__ __device__ inline int wave_lds_bytes(int max_k, int arc_max, bool per_arc)
{
    int b = 8 * kWaveBufRows + 4 * kWaveBufRows + (per_arc ? 4 * kWaveBufRows : 0);
    b += 8 * arc_copy_words(arc_max);
    b += 8 * mbox_words(per_arc) * kWave;
    b += 4 * kWaveBufRows;
    if (stack_mode(max_k) == kStackLds) b += 8 * (int)wave_stack_words(max_k);
    return (b + 15) & ~15;
}

int32_t count_lds_bytes(int32_t arc_max, int32_t max_k, int32_t wg_waves, bool per_arc)
{
    return wg_waves * wave_lds_bytes(max_k, arc_max, per_arc);
}

int64_t count_deep_scratch_words(int32_t max_k, int32_t wg_waves)
{
    if (stack_mode(max_k) != kStackGlobal) return 0;
    return ((int64_t)wg_waves * wave_stack_words(max_k) + 31) & ~31ll;
}

int64_t count_scratch_words(int32_t, int32_t max_k, int32_t wg_waves)
{
    const int64_t w = wave_global_stack_words(max_k);
    if (w == 0) return 0;
    return ((int64_t)wg_waves * w + 31) & ~31ll;
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
    int arc_max;     // nodes with 64 < c <= arc_max are copied to LDS
};

// Per-lane light stack: slot s holds the (M, R) pair of level s + 1.  In
// registers (L > 0 levels, each access a select over the levels, since the
// lanes sit at different depths) or in memory, one word per lane per level.
template <int L>
struct LightStack;

template <>
struct LightStack<4> {
    u64 m0 = 0, m1 = 0, m2 = 0, m3 = 0, r0 = 0, r1 = 0, r2 = 0, r3 = 0;
    __device__ __forceinline__ LightStack(const WaveBuf&) {}
    __device__ __forceinline__ void put(int s, u64 M, u64 R)
    {
        m0 = s == 0 ? M : m0;
        m1 = s == 1 ? M : m1;
        m2 = s == 2 ? M : m2;
        m3 = s == 3 ? M : m3;
        r0 = s == 0 ? R : r0;
        r1 = s == 1 ? R : r1;
        r2 = s == 2 ? R : r2;
        r3 = s == 3 ? R : r3;
    }
    __device__ __forceinline__ void set_r(int s, u64 R)
    {
        r0 = s == 0 ? R : r0;
        r1 = s == 1 ? R : r1;
        r2 = s == 2 ? R : r2;
        r3 = s == 3 ? R : r3;
    }
    __device__ __forceinline__ u64 get_m(int s) const { return s == 0 ? m0 : s == 1 ? m1 : s == 2 ? m2 : m3; }
    __device__ __forceinline__ u64 get_r(int s) const { return s == 0 ? r0 : s == 1 ? r1 : s == 2 ? r2 : r3; }
};
static_assert(kRegLevels == 4, "LightStack<4> holds the register levels");

template <>
struct LightStack<0> {
    u64* __restrict__ sM;
    u64* __restrict__ sR;
    int lane;
    __device__ __forceinline__ LightStack(const WaveBuf& wb) : sM(wb.sM), sR(wb.sR), lane(lane_of()) {}
    __device__ __forceinline__ void put(int s, u64 M, u64 R)
    {
        sM[s * kWave + lane] = M;
        sR[s * kWave + lane] = R;
    }
    __device__ __forceinline__ void set_r(int s, u64 R) { sR[s * kWave + lane] = R; }
    __device__ __forceinline__ u64 get_m(int s) const { return sM[s * kWave + lane]; }
    __device__ __forceinline__ u64 get_r(int s) const { return sR[s * kWave + lane]; }
};

// One degrees-only step on a last-level node: the next two candidates x of
// R (R != 0) leave R, and the result is the sum of popcount(M AND row_x).
// Without a second candidate the first row is read twice and counted once
// (no branch).
__device__ __forceinline__ unsigned leaf_step(const u64* __restrict__ rows, int base, u64 M, u64& R)
{
    const int x1 = __builtin_ctzll(R);
    R &= R - 1;
    const bool two = R != 0ull;
    const int x2 = two ? __builtin_ctzll(R) : x1;
    R &= R - 1;                        // stays 0 when it was 0
    const u64 r1 = rows[base + x1];
    const u64 r2 = rows[base + x2];
    return (unsigned)__popcll(M & r1) + (two ? (unsigned)__popcll(M & r2) : 0u);
}

template <bool kStats, bool kPerArc, int kRegL>
__device__ __forceinline__ void light_engine(const WaveBuf& wb, Acc& A, u64* __restrict__ per_arc)
{
    const int lane = lane_of();
    const u64 lt_mask = lane == 0 ? 0ull : (~0ull >> (kWave - lane));
    const u64* __restrict__ rows = wb.rows;
    LightStack<kRegL> stk(wb);
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
                    const u64 r = (l == t) ? R : stk.get_r(l - 1);
                    const int pc = __popcll(r);
                    if (pc >= 2 && (need + (t - l) >= 3 || pc >= 8)) {
                        lvl = l;
                        Rl = r;
                        Ml = (l == t) ? M : stk.get_m(l - 1);
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
                        else stk.set_r(lvl - 1, low);
                        u64* mb = wb.mbox + mbox_words(kPerArc) * recv;
                        mb[0] = Ml;
                        mb[1] = Rl & ~low;
                        mb[2] = ((u64)(unsigned)base << 32) | (unsigned)(need + (t - lvl));
                        if (kPerArc) mb[3] = (u64)(unsigned)tag;
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                if (!active && __popcll(idle & lt_mask) < np) {
                    const u64* mb = wb.mbox + mbox_words(kPerArc) * lane;
                    M = mb[0];
                    R = mb[1];
                    need = (int)(unsigned)mb[2];
                    base = (int)(mb[2] >> 32);
                    if (kPerArc) tag = (int)(unsigned)mb[3];
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
                    const unsigned c = leaf_step(rows, base, M, R);
                    A.acc += (u64)c;
                    if (kPerArc) uacc += (u64)c;
                    if (kStats) A.st[kStatWordOps] += 2;
                } else {
                    const int x = __builtin_ctzll(R);
                    R &= R - 1;
                    const u64 nm = M & rows[base + x];
                    if (__popcll(nm) >= need - 1) {
                        stk.put(t - 1, M, R);
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
                unsigned bacc = 0;             // <= 2 * 64 * kBurstIters
                for (int it = 0; it < kBurstIters; ++it) {
                    const bool leaf = R != 0ull;
                    if (__popcll(__ballot(leaf)) < kBurstMinLanes) break;
                    if (leaf) {
                        bacc += leaf_step(rows, base, M, R);
                        if (kStats) A.st[kStatWordOps] += 2;
                    }
                }
                A.acc += (u64)bacc;
                if (kPerArc) uacc += (u64)bacc;
            }
            if (R == 0ull) {
                if (t == 1) {
                    active = false;
                    if (kPerArc && uacc) atomicAdd(per_arc + tag, uacc);
                } else {
                    --t;
                    ++need;
                    if (kStats) A.st[kStatLightPops] += 1;
                    M = stk.get_m(t - 1);
                    R = stk.get_r(t - 1);
                }
            }
        }
    }
}

template <bool kStats, bool kPerArc, int kRegL>
__device__ __forceinline__ void flush_tasks(WaveBuf& wb, Acc& A, u64* per_arc)
{
    if (wb.n == 0) return;
    if (kStats && lane_of() == 0) A.st[kStatFlushes] += 1;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const u64 c0 = kStats ? __builtin_readcyclecounter() : 0ull;
    light_engine<kStats, kPerArc, kRegL>(wb, A, per_arc);
    if (kStats && lane_of() == 0) A.st[kStatCycLight] += __builtin_readcyclecounter() - c0;
    __builtin_amdgcn_wave_barrier();
    wb.n = 0;
    wb.nu = 0;
}

// ------------------------------------------------------------ heavy engine

typedef __attribute__((address_space(3))) u64 lds_u64;
typedef __attribute__((address_space(3))) int32_t lds_i32;
typedef __attribute__((address_space(1))) const u64 glb_u64;
typedef __attribute__((address_space(1))) const unsigned char glb_u8;

// Rows of a heavy subgraph: the source vertex's rows in device memory
// (kGlobal), addressed with 32-bit offsets from a wave-uniform base, or a
// compacted copy in the wave's LDS.
template <bool kGlobal>
struct RowRef;
template <>
struct RowRef<true> {
    glb_u64* p;
    __device__ __forceinline__ u64 operator()(unsigned i) const
    {
        return *reinterpret_cast<glb_u64*>(reinterpret_cast<glb_u8*>(p) + (i << 3));
    }
};
template <>
struct RowRef<false> {
    const lds_u64* p;
    __device__ __forceinline__ u64 operator()(unsigned i) const { return p[i]; }
};

template <bool kGlobal>
struct HeavyCtx {
    RowRef<kGlobal> rows;
    int W;     // words per row
    int L;     // vertices of the clique inside the subgraph (k - 1)
    int tag;   // the arc (per-arc output)
};

// Parallel bit extract with a wave-uniform mask (Hacker's Delight, section
// 7-4, "compress"): the masks are prepared once per mask word (scalar
// work), then each lane packs its own word in six shift-and-merge steps.
struct Pext {
    u64 m, v0, v1, v2, v3, v4, v5;
};

__device__ __forceinline__ u64 prefix_xor64(u64 x)
{
    x ^= x << 1;
    x ^= x << 2;
    x ^= x << 4;
    x ^= x << 8;
    x ^= x << 16;
    x ^= x << 32;
    return x;
}

__device__ __forceinline__ Pext pext_prep(u64 m)
{
    Pext p;
    p.m = m;
    u64 mk = ~m << 1;
    u64 v[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        const u64 mp = prefix_xor64(mk);
        v[i] = mp & m;
        m = (m ^ v[i]) | (v[i] >> (1 << i));
        mk &= ~mp;
    }
    p.v0 = v[0];
    p.v1 = v[1];
    p.v2 = v[2];
    p.v3 = v[3];
    p.v4 = v[4];
    p.v5 = v[5];
    return p;
}

__device__ __forceinline__ u64 pext_apply(u64 x, const Pext& p)
{
    u64 t;
    x &= p.m;
    t = x & p.v0; x = (x ^ t) | (t >> 1);
    t = x & p.v1; x = (x ^ t) | (t >> 2);
    t = x & p.v2; x = (x ^ t) | (t >> 4);
    t = x & p.v3; x = (x ^ t) | (t >> 8);
    t = x & p.v4; x = (x ^ t) | (t >> 16);
    t = x & p.v5; x = (x ^ t) | (t >> 32);
    return x;
}

// Row x of H restricted to the candidates of M (lane q holds word q of M)
// and packed: bit i of the result is candidate i.  At most 256 candidates
// (four words o0..o3).  Uniform control flow: the whole wave calls it.
template <bool kGlobal>
__device__ __forceinline__ void pack_row(const HeavyCtx<kGlobal>& H, u64 M, int x, bool valid, u64& o0, u64& o1,
                                         u64& o2, u64& o3)
{
    o0 = o1 = o2 = o3 = 0ull;
    const unsigned base = valid ? (unsigned)(x * H.W) : 0u;
    int off = 0;
    for (int w0 = 0; w0 < H.W; w0 += 4) {
        // four source words in flight at a time
        u64 src[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) src[i] = (valid && w0 + i < H.W) ? H.rows(base + w0 + i) : 0ull;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            if (w0 + i >= H.W) break;
            const u64 mw = readlane64(M, w0 + i);
            if (mw == 0ull) continue;
            const u64 p = pext_apply(src[i], pext_prep(mw));
            const int wi = off >> 6, sh = off & 63;
            const u64 lo = p << sh;
            const u64 hi = sh ? (p >> (64 - sh)) : 0ull;
            // wi is wave-uniform; selects keep o0..o3 in registers
            o0 |= wi == 0 ? lo : 0ull;
            o1 |= (wi == 1 ? lo : 0ull) | (wi == 0 ? hi : 0ull);
            o2 |= (wi == 2 ? lo : 0ull) | (wi == 1 ? hi : 0ull);
            o3 |= (wi == 3 ? lo : 0ull) | (wi == 2 ? hi : 0ull);
            off += __popcll(mw);
        }
    }
}

// Copy the subgraph induced on the c candidates of M to dst in LDS,
// compacted to W2 = ceil(c / 64) words per row; c <= kArcMaxC.
__device__ __forceinline__ int copy_to_lds(const HeavyCtx<true>& H, u64 M, int c, lds_u64* dst)
{
    const int q = lane_of();
    const int W2 = (c + 63) >> 6;
    for (int a0 = 0; a0 < c; a0 += kWave) {
        const int a = a0 + q;
        const int xa = wave_select(M, a, H.W);
        u64 o0, o1, o2, o3;
        pack_row<true>(H, M, xa, a < c, o0, o1, o2, o3);
        if (a < c) {
            lds_u64* d = dst + a * W2;
            d[0] = o0;
            if (W2 > 1) d[1] = o1;
            if (W2 > 2) d[2] = o2;
            if (W2 > 3) d[3] = o3;
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    return W2;
}

// Two levels left on a node of the LDS copy with more than 64 candidates
// (W words per row, W = 2..4): every lane takes a candidate x, forms its
// child mask m AND row_x in registers and sums the last level of that
// child itself, two vertices y of the child per step; a lane that finishes
// takes the next candidate (positions listed in pos), so lanes stay busy
// however uneven the children are.  Returns this lane's sum (< 2^24).
template <int W, bool kStats>
__device__ __forceinline__ unsigned need3_lanes(const HeavyCtx<false>& H, const u64* mw, int nj,
                                                const lds_i32* pos, unsigned& took, unsigned& ops)
{
    const int lane = lane_of();
    const u64 lt = lane == 0 ? 0ull : (~0ull >> (kWave - lane));
    int next = 0;                 // wave-uniform: candidates handed out
    bool act = false;
    u64 ch[W];
#pragma unroll
    for (int i = 0; i < W; ++i) ch[i] = 0ull;
    u64 r = 0ull;
    int w = 0;
    unsigned sum = 0;
    for (;;) {
        const u64 idle = __ballot(!act);
        if (next < nj && (__popcll(idle) >= 8 || idle == ~0ull)) {
            const int jj = next + __popcll(idle & lt);
            next += __popcll(idle);
            if (!act && jj < nj) {
                const unsigned b = (unsigned)(pos[jj] * W);
#pragma unroll
                for (int i = 0; i < W; ++i) ch[i] = mw[i] & H.rows(b + i);
                r = ch[0];
                w = 0;
                act = true;
                if (kStats) ++took;
            }
        } else if (idle == ~0ull) {
            break;
        }
        // a burst of steps between refills: lanes that finish early wait
        // for the next refill (at most kN3Burst - 1 steps)
        for (int it = 0; it < kN3Burst; ++it) {
            if (act) {
                if (r == 0ull) {
#pragma unroll
                    for (int i = 1; i < W; ++i)
                        if (r == 0ull && w < i) {
                            w = i;
                            r = ch[i];
                        }
                    if (r == 0ull) act = false;
                }
            }
            if (act) {
                const int y1 = w * 64 + __builtin_ctzll(r);
                r &= r - 1;
                const bool two = r != 0ull;   // a second vertex of the same word
                const int y2 = two ? w * 64 + __builtin_ctzll(r) : y1;
                if (two) r &= r - 1;
                const unsigned b1 = (unsigned)(y1 * W), b2 = (unsigned)(y2 * W);
                u64 a1[W], a2[W];
#pragma unroll
                for (int i = 0; i < W; ++i) {
                    a1[i] = H.rows(b1 + i);
                    a2[i] = H.rows(b2 + i);
                }
                unsigned c1 = 0, c2 = 0;
#pragma unroll
                for (int i = 0; i < W; ++i) {
                    c1 += __popcll(ch[i] & a1[i]);
                    c2 += __popcll(ch[i] & a2[i]);
                }
                sum += c1 + (two ? c2 : 0u);
                if (kStats) ops += two ? 2 * W : W;
            }
        }
    }
    return sum;
}

template <bool kStats, bool kPerArc, bool kGlobal, int kRegL>
__device__ __forceinline__ void heavy_dfs(const HeavyCtx<kGlobal>& H, u64 M, int need0, int lvl0, int part, int P,
                                          WaveBuf& wb, Acc& A, u64& uacc, u64* per_arc);

// Handle a node with mask m (c candidates, `need` more vertices to choose;
// rows in device memory when kGlobal, else in the wave's LDS copy).  Returns
// true when the caller must search it depth first.  lvl is the first free
// level of the heavy stacks.  Only first-level branches j = part (mod P)
// of the node are taken; P > 1 only at the root of a split arc, which has
// need >= 4 (arc_parts is 1 for k <= 5).
template <bool kStats, bool kPerArc, bool kGlobal, int kRegL>
__device__ __forceinline__ bool heavy_node(const HeavyCtx<kGlobal>& H, u64 m, int c, int need, int lvl, int part,
                                           int P, WaveBuf& wb, Acc& A, u64& uacc, u64* per_arc)
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
            unsigned s = 0;
            const unsigned b = (unsigned)((j < c ? x : 0) * H.W);
            for (int w = 0; w < H.W; ++w) {
                const u64 mw = readlane64(m, w);
                if (j < c && mw) s += __popcll(mw & H.rows(b + w));
            }
            A.acc += (u64)s;
            if (kPerArc) uacc += (u64)s;
            if (kStats && j < c) {
                A.st[kStatWordOps] += H.W;
                A.st[kStatHeavyLeafCand] += 1;
            }
        }
        return false;
    }
    if constexpr (kGlobal) {
    if (c <= wb.arc_max && c > kWave) {
        // continue from an LDS copy of this node's subgraph
        const u64 c0 = kStats ? __builtin_readcyclecounter() : 0ull;
        lds_u64* arc = (lds_u64*)wb.arc;
        const int W2 = copy_to_lds(H, m, c, arc);
        if (kStats && lane == 0) A.st[kStatCycCopy] += __builtin_readcyclecounter() - c0;
        const HeavyCtx<false> HL{RowRef<false>{arc}, W2, H.L, H.tag};
        const int rem = c - 64 * lane;
        const u64 all = lane < W2 ? (rem >= 64 ? ~0ull : ((1ull << rem) - 1)) : 0ull;
        if (kStats && lane == 0) A.st[kStatArcLds] += 1;
        if (heavy_node<kStats, kPerArc, false, kRegL>(HL, all, c, need, lvl, part, P, wb, A, uacc, per_arc))
            heavy_dfs<kStats, kPerArc, false, kRegL>(HL, all, need, lvl, part, P, wb, A, uacc, per_arc);
        __builtin_amdgcn_wave_barrier();
        return false;
    }
    }
    if constexpr (!kGlobal) {
    if (need == 3 && c > kWave) {
        const u64 c0 = kStats ? __builtin_readcyclecounter() : 0ull;
        const int nj = (c - part + P - 1) / P;
        // positions of the candidates taken, in the mailbox area (idle while
        // the light engine is not running); nj <= c <= arc_max <= kArcMaxC <= kPosList
        lds_i32* pos = (lds_i32*)wb.mbox;
        for (int j0 = 0; j0 < nj; j0 += kWave) {
            const int jj = j0 + lane;
            const int x = wave_select(m, jj < nj ? part + P * jj : c, H.W);
            if (jj < nj) pos[jj] = x;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        u64 mw[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) mw[i] = i < H.W ? readlane64(m, i) : 0ull;
        unsigned took = 0, ops = 0, sum;
        if (H.W == 2) sum = need3_lanes<2, kStats>(H, mw, nj, pos, took, ops);
        else if (H.W == 3) sum = need3_lanes<3, kStats>(H, mw, nj, pos, took, ops);
        else sum = need3_lanes<4, kStats>(H, mw, nj, pos, took, ops);
        if (kStats) {
            A.st[kStatNeed3MinOps] += (u64)(ops / H.W) * (u64)((c + 63) >> 6);
            if (lane == 0) A.st[kStatNeed3Nodes] += 1;
        }
        __builtin_amdgcn_wave_barrier();
        A.acc += (u64)sum;
        if (kPerArc) uacc += (u64)sum;
        if (kStats) {
            A.st[kStatWordOps] += ops;
            A.st[kStatNeed3Lanes] += took;
            if (lane == 0) A.st[kStatCycNeed3] += __builtin_readcyclecounter() - c0;
        }
        return false;
    }
    }
    if (c <= kWave) {
        // compaction: lane a packs row a over the c candidates into one
        // word and the node goes to the light engine's queue
        if (wb.n + c > kWaveBufRows) flush_tasks<kStats, kPerArc, kRegL>(wb, A, per_arc);
        const u64 c0 = kStats ? __builtin_readcyclecounter() : 0ull;
        const int xa = wave_select(m, lane, H.W);
        u64 o0, o1, o2, o3;
        pack_row<kGlobal>(H, m, xa, lane < c, o0, o1, o2, o3);
        if (lane < c) {
            wb.rows[wb.n + lane] = o0;
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
            A.st[kStatCycCopy] += __builtin_readcyclecounter() - c0;
        }
        return false;
    }
    return true;
}

// Depth-first search, all lanes in step, below a node with mask M (more
// than 64 candidates, need0 more vertices), rows in H; stack levels from lvl0.
template <bool kStats, bool kPerArc, bool kGlobal, int kRegL>
__device__ __forceinline__ void heavy_dfs(const HeavyCtx<kGlobal>& H, u64 M, int need0, int lvl0, int part, int P,
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
        const u64 ch = M & (q < H.W ? H.rows((unsigned)(x * H.W + q)) : 0ull);
        const int cc = wave_sum_small(__popcll(ch));
        if (kStats && q == 0) A.st[kStatHeavySteps] += 1;
        if (heavy_node<kStats, kPerArc, kGlobal, kRegL>(H, ch, cc, need0 - t, lvl0 + t, 0, 1, wb, A, uacc, per_arc)) {
            wb.hM[(lvl0 + t - 1) * kWave + q] = M;
            wb.hR[(lvl0 + t - 1) * kWave + q] = R;
            M = ch;
            R = ch;
            ++t;
            if (kStats && q == 0) A.st[kStatPushes] += 1;
        }
    }
}

template <bool kStats, bool kPerArc, int kRegL>
__device__ __forceinline__ void heavy_arc(const HeavyCtx<true>& H, int r, int part, int P, WaveBuf& wb, Acc& A,
                                          u64* per_arc)
{
    const int q = lane_of();
    u64 uacc = 0;
    const u64 M = q < H.W ? H.rows((unsigned)(r * H.W + q)) : 0ull;
    const int c = wave_sum_small(__popcll(M));
    const int need = H.L - 1;
    if (heavy_node<kStats, kPerArc, true, kRegL>(H, M, c, need, 0, part, P, wb, A, uacc, per_arc))
        heavy_dfs<kStats, kPerArc, true, kRegL>(H, M, need, 0, part, P, wb, A, uacc, per_arc);
    if (kPerArc) {
        const u64 s = wave_sum_u64(uacc);
        if (q == 0 && s) atomicAdd(per_arc + H.tag, s);
    }
}

// Vertex-rooted unit (Algorithm 2 per vertex): the whole subgraph of u, all
// d positions as candidates and k - 1 vertices still to choose; its first
// level walks the arcs of u in turn within this one work item.
template <bool kStats, bool kPerArc, int kRegL>
__device__ __forceinline__ void heavy_vertex(const HeavyCtx<true>& H, int d, WaveBuf& wb, Acc& A, u64* per_arc)
{
    const int q = lane_of();
    u64 uacc = 0;
    const int rem = d - 64 * q;
    const u64 M = q < H.W ? (rem >= 64 ? ~0ull : ((1ull << rem) - 1ull)) : 0ull;
    if (heavy_node<kStats, kPerArc, true, kRegL>(H, M, d, H.L, 0, 0, 1, wb, A, uacc, per_arc))
        heavy_dfs<kStats, kPerArc, true, kRegL>(H, M, H.L, 0, 0, 1, wb, A, uacc, per_arc);
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
    int32_t arc_lds_max;    // representation switch of heavy nodes (64..kArcMaxC)
    int32_t* progress;      // host-mapped word: items claimed, updated every 512 (nullable)
    int32_t chunk;          // consecutive items a wave claims with one atomic
};

template <int kMode, bool kStats, bool kPerArc>
__global__ void __launch_bounds__(kMaxBlock) __attribute__((amdgpu_waves_per_eu(kMode == kStackReg ? 4 : 2))) count_kernel(KParams P)
{
    constexpr int kRegL = kMode == kStackReg ? kRegLevels : 0;
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = lane_of();
    const int wid = threadIdx.x / kWave;
    const int nwaves = blockDim.x / kWave;
    const int levels = stack_levels(P.max_k);
    unsigned char* wbase = smem + wid * wave_lds_bytes(P.max_k, P.arc_lds_max, kPerArc);
    WaveBuf wb;
    int off = 0;
    wb.rows = reinterpret_cast<u64*>(wbase + off);
    off += 8 * kWaveBufRows;
    wb.meta = reinterpret_cast<int32_t*>(wbase + off);
    off += 4 * kWaveBufRows;
    wb.tags = reinterpret_cast<int32_t*>(wbase + off);     // per-arc launches only
    if (kPerArc) off += 4 * kWaveBufRows;
    wb.arc = reinterpret_cast<u64*>(wbase + off);
    off += 8 * arc_copy_words(P.arc_lds_max);
    wb.mbox = reinterpret_cast<u64*>(wbase + off);
    off += 8 * mbox_words(kPerArc) * kWave;
    wb.units = reinterpret_cast<int32_t*>(wbase + off);
    off += 4 * kWaveBufRows;
    u64* stacks;
    if (kMode == kStackLds)
        stacks = reinterpret_cast<u64*>(wbase + off);
    else
        stacks = P.scratch + (int64_t)blockIdx.x * P.scratch_words + (int64_t)wid * wave_global_stack_words(P.max_k);
    (void)nwaves;
    if (kMode == kStackReg) {
        wb.sM = nullptr;
        wb.sR = nullptr;
        wb.hM = stacks;
        wb.hR = stacks + (int64_t)levels * kWave;
    } else {
        wb.sM = stacks;
        wb.sR = stacks + (int64_t)levels * kWave;
        wb.hM = stacks + 2ll * levels * kWave;
        wb.hR = stacks + 3ll * levels * kWave;
    }
    wb.n = 0;
    wb.nu = 0;
    wb.arc_max = P.arc_lds_max;

    Acc A;
    A.acc = 0ull;
    A.ovf = 0;
#pragma unroll
    for (int i = 0; i < kNumStats; ++i) A.st[i] = 0ull;
    int cur = -1;                      // query whose work the wave holds
    u64* per_arc = nullptr;
    const u64 t_start = kStats ? wall_clock64() : 0ull;
    const u64 cyc_start = kStats ? __builtin_readcyclecounter() : 0ull;
    if (kStats && lane == 0) {
        const u64 now = atomicAdd(P.queries[0].stats + kStatResidentNow, 1ull) + 1;
        atomicMax(P.queries[0].stats + kStatResidentMax, now);
    }
    u64 item_max = 0ull;

    int g_next = 0, g_end = 0;         // the wave's claimed run of items
    for (;;) {
        if (g_next >= g_end) {
            int g0 = 0;
            if (lane == 0) g0 = atomicAdd(P.item_ctr, P.chunk);
            g0 = __shfl(g0, 0, kWave);
            g_next = g0;
            g_end = g0 + P.chunk;
        }
        const int g = g_next++;
        if (g >= P.total_items) break;
        // progress for the host, read without any HIP call while the launch runs
        if (P.progress && lane == 0 && (g & 511) == 0)
            __hip_atomic_store(P.progress, g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
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
                flush_tasks<kStats, kPerArc, kRegL>(wb, A, per_arc);
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
        const int i = q.item_lo + (g - q.item_begin) * q.item_stride;
        const int k = q.k;
        const u64 t_item = kStats ? wall_clock64() : 0ull;
        // the item: one part of a heavy arc, or (a part of) a light vertex
        int u, r = -1, part, nparts, tag;
        int kind = kItemHeavyArc;
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
            const int key = q.buckets[4 * lo + 3] >> 2;
            kind = q.buckets[4 * lo + 3] & 3;
            heavy = kind == kItemHeavyArc || kind == kItemHeavyVertex;
            const int cnt = q.buckets[4 * lo + 2];
            const int local = i - q.buckets[4 * lo];
            part = local / cnt;
            const int which = q.buckets[4 * lo + 1] + (local - part * cnt);
            if (kind == kItemHeavyArc) {
                const int e = q.rows.harcs[which];
                u = q.dag_src[e];
                r = e - q.dag_ptr[u];
                nparts = arc_parts(key, k, q.split_pct);
                tag = e;
            } else if (kind == kItemHeavyVertex) {
                u = q.order[which];
                nparts = 1;
                tag = -1;
            } else {
                u = q.order[q.light_first + which];
                nparts = kind == kItemLightVertex ? light_parts(key + 1, k, q.split_pct) : 1;
                tag = -1;
            }
        }
        const int a0 = q.dag_ptr[u];
        const int d = q.dag_ptr[u + 1] - a0;
        if (heavy) {
            const HeavyCtx<true> H{RowRef<true>{(glb_u64*)(q.rows.rows + q.rows.rows_off[u])},
                                   (d + 63) >> 6, k - 1, tag};
            if (kind == kItemHeavyVertex) heavy_vertex<kStats, kPerArc, kRegL>(H, d, wb, A, per_arc);
            else heavy_arc<kStats, kPerArc, kRegL>(H, r, part, nparts, wb, A, per_arc);
        } else if (kind == kItemLightRoot) {
            // vertex-rooted light vertex: its rows, then one unit rooted at
            // the vertex itself (mask of all d positions, k - 1 to choose)
            if (wb.n + d + 1 > kWaveBufRows) flush_tasks<kStats, kPerArc, kRegL>(wb, A, per_arc);
            if (lane < d) {
                wb.rows[wb.n + lane] = q.rows.rows[q.rows.rows_off[u] + lane];
                wb.meta[wb.n + lane] = (wb.n << 8) | (k - 2);
            }
            if (lane == 0) {
                wb.rows[wb.n + d] = d >= 64 ? ~0ull : ((1ull << d) - 1ull);
                wb.meta[wb.n + d] = (wb.n << 8) | (k - 1);
                wb.units[wb.nu] = wb.n + d;
            }
            wb.nu += 1;
            wb.n += d + 1;
        } else {
            // rows of the vertex into the wave's buffer; the searched arcs
            // (every nparts-th one, or the one listed) become units
            if (wb.n + d > kWaveBufRows) flush_tasks<kStats, kPerArc, kRegL>(wb, A, per_arc);
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
        if (wb.n >= P.flush_rows) flush_tasks<kStats, kPerArc, kRegL>(wb, A, per_arc);
        if (kStats && lane == 0) {
            const u64 dt = wall_clock64() - t_item;
            if (dt > (item_max >> 32)) item_max = (dt << 32) | (u64)(unsigned)g;
        }
    }
    if (cur >= 0) {
        const QueryDesc& oq = P.queries[cur];
        flush_tasks<kStats, kPerArc, kRegL>(wb, A, per_arc);
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
        atomicAdd(st + kStatCycTotal, __builtin_readcyclecounter() - cyc_start);
        atomicAdd(st + kStatResidentNow, ~0ull);   // minus one
    }
}

template <int kMode, bool kStats, bool kPerArc>
static hipError_t launch_variant(const KParams& P, const CountLaunch& cl, hipStream_t s)
{
    const void* fn = (const void*)count_kernel<kMode, kStats, kPerArc>;
    if (cl.lds_bytes > 65536) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, cl.lds_bytes);
        if (e != hipSuccess) return e;
    }
    count_kernel<kMode, kStats, kPerArc><<<cl.blocks, cl.wg_waves * kWave, cl.lds_bytes, s>>>(P);
    return hipGetLastError();
}

template <int kMode>
static hipError_t launch_mode(const KParams& P, const CountLaunch& cl, hipStream_t s)
{
    const int v = (cl.stats ? 2 : 0) | (cl.per_arc ? 1 : 0);
    switch (v) {
    case 0: return launch_variant<kMode, false, false>(P, cl, s);
    case 1: return launch_variant<kMode, false, true>(P, cl, s);
    case 2: return launch_variant<kMode, true, false>(P, cl, s);
    default: return launch_variant<kMode, true, true>(P, cl, s);
    }
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
    // a wave runs its queue once it holds flush_rows rows (at most its buffer)
    P.flush_rows = cl.flush_rows > kWaveBufRows ? kWaveBufRows : cl.flush_rows;
    P.arc_lds_max = clamp_arc_max(cl.arc_lds_max);
    P.progress = cl.progress;
    // Items claimed per atomic.  All waves claim from one device-wide
    // counter, whose atomics are serialised (about 12 ns each on MI355X, so
    // one item per claim caps a launch near 85 M items/s); a wave claims a
    // run of consecutive items instead, short enough that every wave still
    // makes about eight claims.  Items are in descending cost order, so the
    // items of a run cost about the same.
    {
        const int64_t waves = (int64_t)cl.blocks * cl.wg_waves;
        int64_t c = (int64_t)cl.total_items / (waves * 8);
        c = c < 1 ? 1 : (c > kMaxClaim ? kMaxClaim : c);
        // the counter ends at most waves * chunk past total_items
        if ((int64_t)cl.total_items + waves * c >= (1ll << 31)) c = 1;
        P.chunk = (int32_t)c;
    }
    switch (stack_mode(cl.max_k)) {
    case kStackReg: return launch_mode<kStackReg>(P, cl, s);
    case kStackLds: return launch_mode<kStackLds>(P, cl, s);
    default: return launch_mode<kStackGlobal>(P, cl, s);
    }
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
                                  int32_t pct, int32_t* __restrict__ parts)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int e = arcs[i];
    const int u = dag_src[e];
    const int d = dag_ptr[u + 1] - dag_ptr[u];
    parts[i] = d > kLightMaxDeg ? arc_parts(arc_c[e], k, pct) : 1;
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
                             const int32_t* arc_c, int32_t k, int32_t pct, int32_t* parts, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    list_parts_kernel<<<(n + 255) / 256, 256, 0, s>>>(arcs, n, dag_src, dag_ptr, arc_c, k, pct, parts);
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

}  // namespace citron
