// Internal declarations shared by the HIP kernels and the host side of
// libcitron.  Not part of the public ABI (include/citron.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace citron {

constexpr int kWave = 64;            // gfx950 wavefront width
constexpr int kLightMaxDeg = 64;     // out-degree that fits one 64-bit row word
constexpr int kMaxWords = 64;        // row words per subgraph (out-degree <= 4096)
constexpr int kMaxDeg = kMaxWords * 64;
constexpr int kKMax = 32;
constexpr int kArcLdsMax = 256;      // largest candidate set an LDS subgraph copy holds

// Count-kernel statistics slots (citron_work_stats).
enum StatSlot {
    kStatVertices = 0,     // subgraphs built
    kStatRows = 1,         // rows built (arcs)
    kStatEntries = 2,      // out-list entries read by the build
    kStatWordOps = 3,      // last-level AND+popcount row-word operations
    kStatPushes = 4,       // recursion nodes pushed (both engines)
    kStatBytes = 5,        // DAG bytes read by the build
    kStatHeavySteps = 6,   // wave-uniform search steps on multi-word masks
    kStatCompactions = 7,  // nodes compacted to one word per row
    kStatCompactRows = 8,  // rows written by compaction
    kStatLightIters = 9,   // light-engine loop iterations (per wave)
    kStatLightActive = 10, // sum over those iterations of lanes with a unit
    kStatLightUnits = 11,  // units started by the light engine
    kStatFlushes = 12,     // task-buffer flushes
    kStatHeavyLeafCand = 13, // last-level candidates handled on multi-word masks
    kStatLightPops = 14,   // light-engine pops
    kStatWaveBusy = 15,    // sum over waves of (last item done - first item taken), wall-clock ticks
    kStatWaveFirst = 16,   // earliest start of a wave (wall-clock ticks, atomic min)
    kStatWaveLast = 17,    // latest end of a wave (atomic max)
    kStatWaves = 18,       // waves that ran
    kStatArcLds = 19,      // heavy arcs searched from an LDS copy of their subgraph
    kStatNeed3Lanes = 20,  // children handled whole by one lane (two levels left)
    kStatDonations = 21,   // light-engine work donations taken by idle lanes
    kStatWaveBusyMax = 22, // longest busy time of one wave (atomic max)
    kStatItemMax = 23,     // longest item: (ticks << 32) | item index (atomic max)
    kStatResidentNow = 24, // waves resident right now (live counter)
    kStatResidentMax = 25, // most waves resident at once (atomic max)
    kStatCycTotal = 26,    // shader-clock cycles of the waves, start to end
    kStatCycLight = 27,    // ... of which in the light engine
    kStatCycCopy = 28,     // ... of which copying or compacting subgraphs
    kStatCycNeed3 = 29,    // ... of which in lane-per-child two-level searches
    kStatNeed3Nodes = 30,  // nodes finished by lane-per-child two-level searches
    kStatNeed3MinOps = 31, // their row-word operations had rows been ceil(c / 64) words wide
    kNumStats = 32
};

// Schedule of one graph for the count kernel: vertices sorted by out-degree
// (descending), the heavy prefix processed one vertex per workgroup (the
// first n_split of them shared by split_factor workgroups), the light rest
// grouped into batches of about light_rows rows.
struct PlanHeader {
    int32_t n_heavy;      // vertices with out-degree > kLightMaxDeg
    int32_t n_split;      // heavy vertices shared by several workgroups
    int32_t split_factor;
    int32_t n_light;      // vertices with 2 <= out-degree <= kLightMaxDeg
    int32_t n_batches;
    int32_t n_items;      // n_split * split_factor + (n_heavy - n_split) + n_batches
    int32_t light_rows;
    int32_t max_rows;     // largest number of rows of one light batch
};

// Subgraph rows of one graph, built once (they do not depend on k): for
// every vertex u with out-list v_0 < ... < v_{d-1}, row i is the bitmap over
// positions 0..d-1 of N->(u) of N->(v_i) cap N->(u), W(u) = ceil(d/64) words.
struct RowsDev {
    const int32_t* rows_off;        // n + 1: first word of u's rows (< 2^31 words)
    const unsigned long long* rows; // all rows
    const int32_t* arc_c;           // m: popcount of arc e's row = |C_uv|
    const int32_t* harcs;           // arcs of heavy vertices by |C_uv| descending
};

// One query of the count kernel (a (graph, k) pair).
struct QueryDesc {
    const int32_t* dag_ptr;
    const int32_t* dag_src;      // source vertex of every arc
    const int32_t* order;        // vertices by out-degree descending
    RowsDev rows;
    unsigned long long* acc;     // count accumulator
    int32_t* overflow;           // set to 1 when an addition carried
    unsigned long long* per_arc; // optional per-arc counts (nullptr: off)
    unsigned long long* stats;   // optional work counters (nullptr: off)
    // Work items, in buckets of equal cost key, largest key first: heavy-arc
    // buckets (key |C_uv|) and light-vertex buckets (key out-degree - 1),
    // merged.  Bucket b: buckets[4b] = first item, [4b+1] = first arc (index
    // into harcs) or first light vertex (index into the light part of order),
    // [4b+2] = arcs or vertices in the bucket, [4b+3] = key << 2 | kind
    // (BucketKind).  An arc or vertex is split into parts (arc_parts /
    // light_parts); items of a bucket are part-major.  buckets[4 n_buckets]
    // = item count.  The vertex-rooted schedule has only the two vertex
    // kinds, each item one whole vertex (heavy ones indexed in order itself).
    const int32_t* buckets;
    int32_t n_buckets;
    int32_t light_first;         // index in order of the first light vertex
    int32_t k;
    int32_t n_work;              // items of the query (all buckets)
    int32_t item_begin;          // first global item of this query
    int32_t n_items;             // items of this query in the launch
    int32_t item_lo;             // local index of the query's first item in the launch
    int32_t item_stride;         // local item of launch item g: item_lo + (g - item_begin) * item_stride
    int32_t split_pct;           // split scale the buckets were built with (arc_parts, light_parts)
    int32_t pad;
    // list mode (arc_list != nullptr): item j is (slot, part) = (arc_items[2j],
    // arc_items[2j+1] & 0xffff) of arc arc_list[slot], split into
    // arc_items[2j+1] >> 16 parts; its counts go to per-arc slot `slot`
    const int32_t* arc_list;
    const int32_t* arc_items;
};

// Kinds of work item (low two bits of a bucket's key word).
enum BucketKind {
    kItemHeavyArc = 0,     // one part of an arc of a heavy vertex (edge-rooted)
    kItemLightVertex = 1,  // (a part of) a light vertex, its arcs the units (edge-rooted)
    kItemHeavyVertex = 2,  // a whole heavy vertex, searched from its own root (vertex-rooted)
    kItemLightRoot = 3     // a whole light vertex, one unit rooted at the vertex (vertex-rooted)
};

// Parts a heavy arc with |C_uv| = c is split into for a k-clique count; each
// part takes every P-th first-level branch of the arc (speed only).  pct
// scales the default (percent); arcs are split only for k >= 6, where the
// root of an arc has at least four levels left.
__host__ __device__ inline int scale_parts(int base, int pct)
{
    if (base <= 1) return 1;
    const int p = base * pct / 100;
    return p < 1 ? 1 : (p > 64 ? 64 : p);
}

__host__ __device__ inline int arc_parts(int c, int k, int pct)
{
    if (k <= 5) return 1;
    if (k == 6) return scale_parts(c < 64 ? 1 : (c / 32 < 8 ? c / 32 : 8), pct);
    return scale_parts(c < 16 ? 1 : (c / 8 < 32 ? c / 8 : 32), pct);
}

// Parts a light vertex (out-degree d <= 64, its subgraph one word per row)
// is split into; each part takes every P-th arc of the vertex (speed only).
__host__ __device__ inline int light_parts(int d, int k, int pct)
{
    if (k <= 5) return 1;
    if (k == 6) return scale_parts(d >= 32 ? d / 8 : 1, pct);
    return scale_parts(d >= 12 ? d / 2 : 1, pct);
}

}  // namespace citron
