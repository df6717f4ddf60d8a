// Launch wrappers of the HIP kernels of libcitron (host-callable).
#pragma once

#include "internal.h"

namespace citron {

// ---- ordering phase (kernels_order.hip)
size_t scan_workspace_ints(int64_t n);
hipError_t scan_exclusive(const int32_t* in, int32_t* out, int64_t n, int32_t* ws, hipStream_t s);
hipError_t launch_validate(int32_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col,
                           int32_t* err, int stage, hipStream_t s);
// key: nullptr for the degree ordering, else the per-vertex order key (ties by id)
hipError_t launch_orient(int32_t n, const int32_t* row_ptr, const int32_t* col, int32_t* outdeg,
                         int32_t* dag_ptr, int32_t* dag_col, int32_t* dag_src, int32_t* max_outdeg,
                         int32_t* scan_ws, hipStream_t s, const int32_t* key = nullptr);

// ---- core ordering by level-synchronous peeling (kernels_core.hip)
// deg[v] = degree, round[v] = -1; *min_deg = smallest degree (preset to INT_MAX)
hipError_t launch_peel_init(int32_t n, const int32_t* row_ptr, int32_t* deg, int32_t* round, int32_t* min_deg,
                            hipStream_t s);
// *min_deg = smallest deg over vertices with round < 0 (preset to INT_MAX)
hipError_t launch_peel_min(int32_t n, const int32_t* deg, const int32_t* round, int32_t* min_deg, hipStream_t s);
// frontier <- vertices with round < 0 and deg <= t, appended at *cnt
hipError_t launch_peel_collect(int32_t n, const int32_t* deg, const int32_t* round, int32_t t, int32_t* frontier,
                               int32_t* cnt, hipStream_t s);
// round[frontier[i]] = r, then the neighbours still present lose one degree
// per edge; those that fall to t are appended to next at *next_cnt
hipError_t launch_peel_round(int32_t nf, const int32_t* frontier, const int32_t* row_ptr, const int32_t* col,
                             int32_t* deg, int32_t* round, int32_t t, int32_t r, int32_t* next, int32_t* next_cnt,
                             hipStream_t s);

// ---- deterministic schedule order (kernels_sched.hip)
struct SortBuffers {
    unsigned long long* keys_a;   // n keys
    unsigned long long* keys_b;   // n keys
    void* temp;                   // sched_sort_temp_bytes(n)
    size_t temp_bytes;
};
size_t sched_sort_temp_bytes(int64_t n);
// order[0 .. bounds[D-1]) = vertices with out-degree >= 2 by out-degree
// descending, ties by id; bounds[i] (i < D) = vertices of out-degree > D - i
hipError_t sched_plan_order(int32_t n, const int32_t* dag_ptr, int32_t D, int32_t* bounds, int32_t* order,
                            const SortBuffers& sb, hipStream_t s);
// harcs[0 .. bounds[D]) = arcs of vertices with out-degree > 64 by |C_uv|
// descending, ties by arc index; bounds[i] (i <= D) = those with |C_uv| > D - 1 - i
hipError_t sched_heavy_arcs(int64_t m, const int32_t* dag_ptr, const int32_t* dag_src, const int32_t* arc_c,
                            int32_t D, int32_t* bounds, int32_t* harcs, const SortBuffers& sb, hipStream_t s);

// ---- vertex schedule (kernels_sched.hip)
struct PlanBuffers {
    int32_t* hist_scan;    // max_outdeg + 3
    int32_t* order;        // n
    int32_t* light_deg;    // n
    int32_t* light_pre;    // n + 1
    int32_t* batch_start;  // n + 1
    PlanHeader* header;    // device
};
hipError_t launch_plan(int32_t n, const int32_t* dag_ptr, int32_t max_outdeg, int32_t light_rows,
                       int32_t split_min_deg, int32_t split_factor, const PlanBuffers& pb,
                       int32_t* scan_ws, const SortBuffers& sb, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long* p, unsigned long long v, int64_t n, hipStream_t s);

// ---- subgraph rows (kernels_rows.hip)
struct BuildParams {
    const int32_t* dag_ptr;
    const int32_t* dag_col;
    const int32_t* order;
    const int32_t* light_pre;
    const int32_t* batch_start;
    PlanHeader plan;
    int32_t max_deg;
    const int32_t* rows_off;
    unsigned long long* rows;
    int32_t* arc_c;
    unsigned long long* tri_acc;       // triangles (the k = 3 count)
    int32_t* tri_ovf;
    int32_t* item_ctr;
    unsigned long long* build_stats;   // kNumStats slots
};
int32_t build_lds_bytes(int32_t light_rows, int32_t max_deg);
hipError_t launch_rows_len(int32_t n, const int32_t* dag_ptr, int32_t* len, hipStream_t s);
hipError_t launch_build_rows(const BuildParams& P, int32_t blocks, hipStream_t s);
hipError_t launch_arc_c_to_u64(int64_t m, const int32_t* arc_c, unsigned long long* out, hipStream_t s);

// ---- counting phase (kernels_count.hip)
struct CountLaunch {
    const QueryDesc* queries;   // device table
    int32_t n_queries;
    int32_t total_items;
    int32_t* item_ctr;          // device, zeroed by the launch sequence
    unsigned long long* scratch;   // stacks of k > 12, scratch_words per block
    int64_t scratch_words;
    int32_t max_k;
    int32_t blocks;
    int32_t wg_waves;
    int32_t lds_bytes;          // dynamic LDS per block
    int32_t flush_rows;
    int32_t arc_lds_max = 256;  // heavy nodes with 64 < c <= this are copied to LDS
    bool stats;                 // instrumented launch
    bool per_arc;               // some query writes per-arc counts
    int32_t* progress = nullptr;   // host-mapped word for the items claimed (nullable)
};
// device-memory stack words per block of a count launch
int64_t count_scratch_words(int32_t max_deg, int32_t max_k, int32_t wg_waves);
// the part of them that grows with k (all stacks of k > 12)
int64_t count_deep_scratch_words(int32_t max_k, int32_t wg_waves);
// dynamic LDS of a count launch: arc_max is its arc_lds_max tuning value
int32_t count_lds_bytes(int32_t arc_max, int32_t max_k, int32_t wg_waves, bool per_arc);
hipError_t launch_count(const CountLaunch& cl, hipStream_t s);
hipError_t launch_check_arcs(const int32_t* arcs, int32_t n, int64_t m, int32_t* err, hipStream_t s);
hipError_t launch_list_parts(const int32_t* arcs, int32_t n, const int32_t* dag_src, const int32_t* dag_ptr,
                             const int32_t* arc_c, int32_t k, int32_t pct, int32_t* parts, hipStream_t s);
hipError_t launch_list_items(int32_t n, const int32_t* parts, const int32_t* offs, int32_t* items, hipStream_t s);
hipError_t launch_gather_arc_c(const int32_t* arcs, int32_t n, const int32_t* arc_c, unsigned long long* out,
                               hipStream_t s);

// ---- k-clique listing (kernels_list.hip)
constexpr int kListMaxK = 16;                    // largest k listing supports
struct ListParams {
    const int32_t* arcs;         // listed arcs (DAG arc indices)
    int32_t n_arcs;
    int32_t k;
    const int32_t* dag_ptr;
    const int32_t* dag_col;
    const int32_t* dag_src;
    const int32_t* rows_off;
    const unsigned long long* rows;
    const long long* offsets;    // n_arcs + 1: first output clique of each arc
    int32_t* out;                // cliques, k ids each
    int32_t* cursor;             // zeroed before the launch
    int32_t chunk;               // arcs a wave claims per atomic (set by launch_list_arcs)
    int32_t stride;              // claim j lists arc j * stride mod n_arcs (set by launch_list_arcs)
    int32_t* err;                // zeroed before the launch; 1 = slot overrun, 2 = count mismatch
};
hipError_t launch_list_arcs(const ListParams& P, int32_t blocks, hipStream_t s);
size_t scan64_workspace(int64_t n);
hipError_t scan_exclusive64(const unsigned long long* in, long long* out, int64_t n, long long* ws, hipStream_t s);

}  // namespace citron
