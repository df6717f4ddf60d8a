// Host-side state of libcitron shared by api.cpp, batch.cpp and server.cpp.
#pragma once

#include <mutex>
#include <string>
#include <vector>

#include "../../include/citron.h"
#include "kernels.h"

namespace citron {

// Small device-side words of one graph (zeroed by fill kernels, never by
// hipMemsetAsync, so that the sequences stay valid inside captured graphs).
struct SmallDev {
    unsigned long long acc;
    int32_t overflow;
    int32_t item_ctr;
    int32_t err;
    int32_t max_outdeg;
    unsigned long long tri_acc;
    int32_t tri_ovf;
    int32_t build_ctr;
    int32_t peel[4];             // peeling: frontier counts (2), smallest degree, spare
    unsigned long long build_stats[kNumStats];
};

// Pinned host mirror for the copies back.
struct SmallHost {
    uint64_t acc;
    int32_t overflow;
    int32_t item_ctr;
    int32_t err;
    int32_t max_outdeg;
    int32_t ends[2];
    PlanHeader plan;
    QueryDesc query;
    uint64_t stats[kNumStats];
    uint64_t tri_acc;
    int32_t tri_ovf;
    int32_t rows_total;
    int32_t peel[4];
    uint64_t build_stats[kNumStats];
};

}  // namespace citron

struct citron_graph {
    int device = 0;
    hipStream_t stream = nullptr;
    int32_t n = 0;
    int64_t nnz = 0;
    int64_t m = 0;
    int state = 0;                 // 0 LOADED, 1 ORDERED
    int order_kind = 0;            // 0 degree ordering, 1 core ordering (peeling)
    int32_t peel_rounds = 0;       // rounds of the peeling (core ordering)
    int32_t max_outdeg = 0;
    int64_t device_bytes = 0;
    std::mutex mu;

    int32_t* d_row_ptr = nullptr;
    int32_t* d_col = nullptr;
    int32_t* d_outdeg = nullptr;
    int32_t* d_dag_ptr = nullptr;
    int32_t* d_dag_col = nullptr;
    int32_t* d_dag_src = nullptr;
    int32_t* d_scan_ws = nullptr;
    int32_t* d_key = nullptr;              // core ordering: round of each vertex
    size_t scan_ws_ints = 0;
    citron::SmallDev* d_small = nullptr;
    citron::SmallHost* h_small = nullptr;

    citron_tuning tuning;
    citron::PlanBuffers pb = {};
    citron::PlanHeader plan = {};
    citron_tuning plan_tuning = {};
    bool plan_valid = false;
    citron::QueryDesc* d_query = nullptr;
    unsigned long long* d_scratch = nullptr;
    int64_t scratch_bytes = 0;
    unsigned long long* d_stats = nullptr;

    uint64_t seed_base = 0;
    bool seed_pending = false;

    // subgraph rows, built at the first count (they do not depend on k)
    bool rows_valid = false;
    int32_t* d_rows_off = nullptr;          // n + 1
    unsigned long long* d_rows = nullptr;
    int32_t* d_arc_c = nullptr;             // m
    int32_t* d_harcs = nullptr;             // m
    int32_t* d_hscan = nullptr;             // D + 1
    std::vector<int32_t> h_hscan;           // heavy arcs by |C_uv|, scanned
    std::vector<int32_t> h_vscan;           // vertices by out-degree, scanned
    uint64_t tri = 0;
    bool tri_ovf = false;
    // per k: the merged bucket table of the count's work items
    int32_t* d_buckets[CITRON_KMAX + 1] = {};
    // tables superseded by a split change: kept until the graph is freed,
    // since a captured batch or an admitted server request may still read one
    std::vector<int32_t*> retired_buckets;
    int32_t bucket_split[CITRON_KMAX + 1] = {};   // split_pct each table was built with
    int64_t bucket_bytes[CITRON_KMAX + 1] = {};   // device bytes of each table
    int32_t n_buckets[CITRON_KMAX + 1] = {};
    int32_t n_work[CITRON_KMAX + 1] = {};
    // per k: the vertex-rooted schedule (whole vertices, no split)
    int32_t* d_vbuckets[CITRON_KMAX + 1] = {};
    int64_t vbucket_bytes[CITRON_KMAX + 1] = {};
    int32_t n_vbuckets[CITRON_KMAX + 1] = {};
    int32_t n_vwork[CITRON_KMAX + 1] = {};
    uint64_t build_stats[citron::kNumStats] = {};
};

namespace citron {

extern thread_local std::string g_last_error;
citron_status fail(citron_status st, const std::string& msg);
citron_status hip_fail(hipError_t e, const char* what);
citron_tuning default_tuning();
citron_status resolve_tuning(const citron_tuning* in, citron_tuning* out);
int32_t arc_max_for(const citron_tuning& t, int32_t max_k);
int device_cus(int dev);
citron_status ensure_plan(citron_graph* g, const citron_tuning& t);
citron_status ensure_rows(citron_graph* g);
citron_status ensure_buckets(citron_graph* g, int32_t k);
citron_status ensure_vbuckets(citron_graph* g, int32_t k);
citron_status check_count_args(const citron_graph* g, int32_t k, bool* trivial, uint64_t* value);
QueryDesc make_query(const citron_graph* g, int32_t k, unsigned long long* acc, int32_t* ovf,
                     unsigned long long* per_arc, unsigned long long* stats, int32_t item_begin);
void batch_forget_graph(const citron_graph* g);

}  // namespace citron
