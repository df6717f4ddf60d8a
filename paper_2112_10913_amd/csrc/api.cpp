// Host side of the libcitron C ABI (include/citron.h): graph handles,
// validation, the ordering phase, schedules and single / per-arc counts.
// Batched counts live in batch.cpp, the request server in server.cpp.
#include "api_internal.h"

#include <algorithm>
#include <atomic>
#include <cstring>
#include <string>

using namespace citron;

static_assert(kNumStats == CITRON_NSTATS, "work statistics slots of the kernel and of the ABI");

namespace citron {

thread_local std::string g_last_error;

citron_status fail(citron_status st, const std::string& msg)
{
    g_last_error = msg;
    return st;
}

citron_status hip_fail(hipError_t e, const char* what)
{
    return fail(CITRON_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

citron_tuning default_tuning()
{
    citron_tuning t;
    t.size = sizeof(citron_tuning);
    t.wg_waves = 2;
    t.blocks_per_cu = 8;        // 16 waves per CU (the count kernel is latency-bound)
    t.light_rows = 256;
    t.flush_rows = 128;
    t.build_blocks_per_cu = 4;
    t.split_pct = 100;
    t.arc_lds_max = 0;          // by k (arc_max_for)
    return t;
}

// Largest node copied to LDS for a launch whose largest k is max_k, when
// the tuning leaves it to the library: at k <= 5 the copies of up to 256
// candidates pay for the fewer waves their LDS allows (12 per CU); deeper
// counts gain more from 16 waves per CU, which LDS holds with copies of up
// to 192 candidates (224 at k = 6: 14 waves).  Measured on R-MAT 20.
int32_t arc_max_for(const citron_tuning& t, int32_t max_k)
{
    if (t.arc_lds_max) return t.arc_lds_max;
    return max_k <= 5 ? 256 : (max_k == 6 ? 224 : 192);
}

citron_status resolve_tuning(const citron_tuning* in, citron_tuning* out)
{
    citron_tuning d = default_tuning();
    if (!in) { *out = d; return CITRON_OK; }
    if (in->size != (int32_t)sizeof(citron_tuning))
        return fail(CITRON_EINVAL, "citron_tuning.size must be sizeof(citron_tuning)");
    citron_tuning t = *in;
    if (t.wg_waves == 0) t.wg_waves = d.wg_waves;
    if (t.blocks_per_cu == 0) t.blocks_per_cu = d.blocks_per_cu;
    if (t.light_rows == 0) t.light_rows = d.light_rows;
    if (t.flush_rows == 0) t.flush_rows = d.flush_rows;
    if (t.build_blocks_per_cu == 0) t.build_blocks_per_cu = d.build_blocks_per_cu;
    if (t.split_pct == 0) t.split_pct = d.split_pct;
    if (t.arc_lds_max == 0) t.arc_lds_max = d.arc_lds_max;
    if (t.wg_waves < 1 || t.wg_waves > 8) return fail(CITRON_EINVAL, "wg_waves must be in 1..8");
    if (t.blocks_per_cu < 1 || t.blocks_per_cu > 32) return fail(CITRON_EINVAL, "blocks_per_cu must be in 1..32");
    if (t.light_rows < 64 || t.light_rows > 1024 || t.light_rows % 64)
        return fail(CITRON_EINVAL, "light_rows must be a multiple of 64 in 64..1024");
    if (t.flush_rows < 64 || t.flush_rows > 256) return fail(CITRON_EINVAL, "flush_rows must be in 64..256");
    if (t.build_blocks_per_cu < 1 || t.build_blocks_per_cu > 16)
        return fail(CITRON_EINVAL, "build_blocks_per_cu must be in 1..16");
    if (t.split_pct < 25 || t.split_pct > 400) return fail(CITRON_EINVAL, "split_pct must be in 25..400");
    if (t.arc_lds_max != 0 && (t.arc_lds_max < 64 || t.arc_lds_max > kArcLdsMax))
        return fail(CITRON_EINVAL, "arc_lds_max must be 0 (by k) or in 64..256");
    *out = t;
    return CITRON_OK;
}

int device_cus(int dev)
{
    static std::atomic<int> cached[64];   // zero-initialised (static storage)
    if (dev >= 0 && dev < 64) {
        const int c = cached[dev].load(std::memory_order_relaxed);
        if (c) return c;
    }
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 256;
    if (dev >= 0 && dev < 64) cached[dev].store(cus, std::memory_order_relaxed);
    return cus;
}

template <typename T>
static citron_status dalloc(T** p, size_t count, int64_t* acct, const char* what)
{
    *p = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc((void**)p, sizeof(T) * count);
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(CITRON_ENOMEM, std::string("hipMalloc failed for ") + what + ": " + hipGetErrorString(e));
    }
    if (acct) *acct += (int64_t)(sizeof(T) * count);
    return CITRON_OK;
}

template <typename T>
static void dfree(T*& p)
{
    if (p) (void)hipFree((void*)p);
    p = nullptr;
}

static void free_plan(citron_graph* g)
{
    dfree(g->pb.hist_scan);
    dfree(g->pb.order);
    dfree(g->pb.light_deg);
    dfree(g->pb.light_pre);
    dfree(g->pb.batch_start);
    dfree(g->pb.header);
    g->plan_valid = false;
}

static void free_graph_memory(citron_graph* g)
{
    dfree(g->d_row_ptr);
    dfree(g->d_col);
    dfree(g->d_outdeg);
    dfree(g->d_dag_ptr);
    dfree(g->d_dag_col);
    dfree(g->d_dag_src);
    dfree(g->d_small);
    dfree(g->d_scan_ws);
    dfree(g->d_key);
    dfree(g->d_query);
    dfree(g->d_scratch);
    dfree(g->d_stats);
    dfree(g->d_rows_off);
    dfree(g->d_rows);
    dfree(g->d_arc_c);
    dfree(g->d_harcs);
    dfree(g->d_hscan);
    for (int32_t* p : g->retired_buckets) dfree(p);
    g->retired_buckets.clear();
    for (int k = 0; k <= CITRON_KMAX; ++k) {
        dfree(g->d_buckets[k]);
        g->bucket_bytes[k] = 0;
        dfree(g->d_vbuckets[k]);
        g->vbucket_bytes[k] = 0;
    }
    g->rows_valid = false;
    free_plan(g);
    if (g->h_small) (void)hipHostFree(g->h_small);
    g->h_small = nullptr;
}

// Vertex schedule: vertices by out-degree (descending) and light batches of
// about t.light_rows rows for the subgraph build.
citron_status ensure_plan(citron_graph* g, const citron_tuning& t)
{
    if (g->plan_valid && g->plan_tuning.light_rows == t.light_rows) return CITRON_OK;
    hipError_t e = hipSetDevice(g->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    const int32_t D = std::max(g->max_outdeg, 2);
    {
        // each buffer is allocated once; a call that failed part-way keeps
        // what it allocated and a retry allocates only the rest
        int64_t* acct = &g->device_bytes;
        citron_status st;
        if ((!g->pb.hist_scan && (st = dalloc(&g->pb.hist_scan, (size_t)D + 3, acct, "plan"))) ||
            (!g->pb.order && (st = dalloc(&g->pb.order, (size_t)g->n + 1, acct, "plan"))) ||
            (!g->pb.light_deg && (st = dalloc(&g->pb.light_deg, (size_t)g->n + 1, acct, "plan"))) ||
            (!g->pb.light_pre && (st = dalloc(&g->pb.light_pre, (size_t)g->n + 2, acct, "plan"))) ||
            (!g->pb.batch_start && (st = dalloc(&g->pb.batch_start, (size_t)g->n + 2, acct, "plan"))) ||
            (!g->pb.header && (st = dalloc(&g->pb.header, 1, acct, "plan"))))
            return st;
    }
    SortBuffers sb = {};
    {
        citron_status st;
        const size_t tb = sched_sort_temp_bytes(g->n);
        if (tb == 0) return fail(CITRON_EDEVICE, "sort workspace query failed");
        unsigned char* tmp = nullptr;
        if ((st = dalloc(&sb.keys_a, (size_t)g->n + 1, nullptr, "plan order")) ||
            (st = dalloc(&sb.keys_b, (size_t)g->n + 1, nullptr, "plan order")) ||
            (st = dalloc(&tmp, tb, nullptr, "plan order"))) {
            dfree(sb.keys_a);
            dfree(sb.keys_b);
            return st;
        }
        sb.temp = tmp;
        sb.temp_bytes = tb;
    }
    e = launch_plan(g->n, g->d_dag_ptr, g->max_outdeg, t.light_rows, 0, 1, g->pb, g->d_scan_ws, sb, g->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
    dfree(sb.keys_a);
    dfree(sb.keys_b);
    {
        unsigned char* tmp = static_cast<unsigned char*>(sb.temp);
        dfree(tmp);
    }
    if (e != hipSuccess) return hip_fail(e, "plan kernels");
    g->h_vscan.assign((size_t)D, 0);
    e = hipMemcpyAsync(&g->h_small->plan, g->pb.header, sizeof(PlanHeader), hipMemcpyDeviceToHost, g->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(g->h_vscan.data(), g->pb.hist_scan, sizeof(int32_t) * (size_t)D,
                           hipMemcpyDeviceToHost, g->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
    if (e != hipSuccess) return hip_fail(e, "plan");
    g->plan = g->h_small->plan;
    g->plan_tuning = t;
    g->plan_valid = true;
    return CITRON_OK;
}

// Subgraph rows of every vertex (Algorithm 5), per-arc |C_uv|, the triangle
// count and the schedule of heavy arcs; built once per graph.
citron_status ensure_rows(citron_graph* g)
{
    if (g->rows_valid) return CITRON_OK;
    citron_status st = ensure_plan(g, g->tuning);
    if (st) return st;
    hipError_t e = hipSetDevice(g->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    if (g->max_outdeg > kMaxDeg)
        return fail(CITRON_EINVAL, "out-degree above 4096 in the degree-ordered DAG is not supported");
    const int32_t D = std::max(g->max_outdeg, 2);
    hipStream_t s = g->stream;
    int64_t* acct = &g->device_bytes;
    if ((!g->d_rows_off && (st = dalloc(&g->d_rows_off, (size_t)g->n + 1, acct, "row offsets"))) ||
        (!g->d_arc_c && (st = dalloc(&g->d_arc_c, (size_t)g->m, acct, "arc sizes"))) ||
        (!g->d_harcs && (st = dalloc(&g->d_harcs, (size_t)g->m, acct, "heavy arcs"))) ||
        (!g->d_hscan && (st = dalloc(&g->d_hscan, (size_t)D + 1, acct, "arc histogram"))))
        return st;
    // Row offsets are int32, so the rows of all vertices, sum over u of
    // d(u) * ceil(d(u)/64) words, must stay below 2^31.  That sum is at most
    // m * ceil(D/64); only when this bound does not settle it is the exact
    // sum taken, on the host from the DAG offsets.
    if ((int64_t)g->m * ((g->max_outdeg + 63) / 64) >= (1LL << 31)) {
        std::vector<int32_t> ptr((size_t)g->n + 1);
        e = hipMemcpyAsync(ptr.data(), g->d_dag_ptr, sizeof(int32_t) * ptr.size(), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "row sizes");
        int64_t total = 0;
        for (int32_t u = 0; u < g->n; ++u) {
            const int64_t d = ptr[(size_t)u + 1] - ptr[(size_t)u];
            total += d * ((d + 63) / 64);
        }
        if (total >= (1LL << 31)) return fail(CITRON_EINVAL, "subgraph rows exceed 2^31 words");
    }
    // row offsets: exclusive scan of d(u) * W(u) (outdeg buffer as scratch)
    e = launch_rows_len(g->n, g->d_dag_ptr, g->d_outdeg, s);
    if (e == hipSuccess) e = scan_exclusive(g->d_outdeg, g->d_rows_off, g->n, g->d_scan_ws, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(&g->h_small->rows_total, g->d_rows_off + g->n, sizeof(int32_t),
                           hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "row offsets");
    const int64_t words = g->h_small->rows_total;
    if (words < 0) return fail(CITRON_EINVAL, "subgraph rows exceed 2^31 words");
    if (!g->d_rows && (st = dalloc(&g->d_rows, (size_t)std::max<int64_t>(words, 1), acct, "subgraph rows")))
        return st;
    SmallDev* sd = g->d_small;
    // vertices of out-degree < 2 are not built (their arcs close no
    // triangle): their rows and sizes must read as zero
    if ((e = launch_fill_u64(g->d_rows, 0, std::max<int64_t>(words, 1), s)) != hipSuccess ||
        (e = launch_fill_i32(g->d_arc_c, 0, g->m, s)) != hipSuccess ||
        (e = launch_fill_u64(&sd->tri_acc, 0, 1, s)) != hipSuccess ||
        (e = launch_fill_i32(&sd->tri_ovf, 0, 2, s)) != hipSuccess ||
        (e = launch_fill_u64(sd->build_stats, 0, kNumStats, s)) != hipSuccess)
        return hip_fail(e, "fill");
    BuildParams P;
    P.dag_ptr = g->d_dag_ptr;
    P.dag_col = g->d_dag_col;
    P.order = g->pb.order;
    P.light_pre = g->pb.light_pre;
    P.batch_start = g->pb.batch_start;
    P.plan = g->plan;
    P.max_deg = g->max_outdeg;
    P.rows_off = g->d_rows_off;
    P.rows = g->d_rows;
    P.arc_c = g->d_arc_c;
    P.tri_acc = &sd->tri_acc;
    P.tri_ovf = &sd->tri_ovf;
    P.item_ctr = &sd->build_ctr;
    P.build_stats = sd->build_stats;
    e = launch_build_rows(P, device_cus(g->device) * g->tuning.build_blocks_per_cu, s);
    if (e != hipSuccess) return hip_fail(e, "subgraph build");
    SortBuffers sb = {};
    {
        const size_t tb = sched_sort_temp_bytes(g->m);
        if (tb == 0) return fail(CITRON_EDEVICE, "sort workspace query failed");
        unsigned char* tmp = nullptr;
        if ((st = dalloc(&sb.keys_a, (size_t)g->m + 1, nullptr, "arc schedule")) ||
            (st = dalloc(&sb.keys_b, (size_t)g->m + 1, nullptr, "arc schedule")) ||
            (st = dalloc(&tmp, tb, nullptr, "arc schedule"))) {
            dfree(sb.keys_a);
            dfree(sb.keys_b);
            return st;
        }
        sb.temp = tmp;
        sb.temp_bytes = tb;
    }
    e = sched_heavy_arcs(g->m, g->d_dag_ptr, g->d_dag_src, g->d_arc_c, D, g->d_hscan, g->d_harcs, sb, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    dfree(sb.keys_a);
    dfree(sb.keys_b);
    {
        unsigned char* tmp = static_cast<unsigned char*>(sb.temp);
        dfree(tmp);
    }
    if (e != hipSuccess) return hip_fail(e, "arc schedule");
    g->h_hscan.assign((size_t)D + 1, 0);
    e = hipMemcpyAsync(g->h_hscan.data(), g->d_hscan, sizeof(int32_t) * ((size_t)D + 1), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(&g->h_small->tri_acc, &sd->tri_acc, sizeof(uint64_t) + sizeof(int32_t),
                           hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(g->h_small->build_stats, sd->build_stats, sizeof(uint64_t) * kNumStats,
                           hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "subgraph build");
    g->tri = g->h_small->tri_acc;
    g->tri_ovf = g->h_small->tri_ovf != 0;
    memcpy(g->build_stats, g->h_small->build_stats, sizeof(g->build_stats));
    g->rows_valid = true;
    return CITRON_OK;
}

// Device scratch for the count kernel of this graph (grows on demand).
citron_status ensure_scratch(citron_graph* g, int64_t bytes)
{
    if (bytes <= g->scratch_bytes) return CITRON_OK;
    dfree(g->d_scratch);
    g->device_bytes -= g->scratch_bytes;
    g->scratch_bytes = 0;
    citron_status st = dalloc(&g->d_scratch, (size_t)((bytes + 7) / 8), &g->device_bytes, "count scratch");
    if (st) return st;
    g->scratch_bytes = bytes;
    return CITRON_OK;
}

// Work items of a k-clique count (k >= 4): heavy arcs with |C_uv| >= k-2 in
// buckets of equal |C_uv|, light vertices with out-degree >= k-1 in buckets of
// equal out-degree, merged into one table by cost key (|C_uv|, or out-degree
// - 1 for a light vertex), largest first, so that the costliest work starts
// first.  Arcs and vertices are split into parts (arc_parts, light_parts).
citron_status ensure_buckets(citron_graph* g, int32_t k)
{
    const int32_t pct = g->tuning.split_pct;
    if (g->d_buckets[k] && g->bucket_split[k] == pct) return CITRON_OK;
    if (g->d_buckets[k]) {
        // another split: the old table stays valid for readers that hold it
        // (a captured batch, an admitted request) until the graph is freed
        g->retired_buckets.push_back(g->d_buckets[k]);
        g->d_buckets[k] = nullptr;
    }
    const int32_t D = std::max(g->max_outdeg, 2);
    auto v_at_least = [&](int32_t x) -> int64_t {   // vertices with out-degree >= x
        if (x > D) return 0;
        if (x < 2) x = 2;
        return g->h_vscan[(size_t)(D - x + 1)];
    };
    const int64_t n_heavy = v_at_least(kLightMaxDeg + 1);
    struct B { int32_t key, first, cnt, light; };
    std::vector<B> hb, lb;
    // heavy-arc buckets: bucket j of the arc order holds |C_uv| = D-1-j
    for (int32_t j = 0; j < D; ++j) {
        const int32_t c = D - 1 - j;
        if (c < k - 2) break;
        const int32_t cnt = g->h_hscan[(size_t)j + 1] - g->h_hscan[(size_t)j];
        if (cnt > 0) hb.push_back({c, g->h_hscan[(size_t)j], cnt, 0});
    }
    // light-vertex buckets: out-degree d = 64 down to max(k-1, 2)
    for (int32_t d = kLightMaxDeg; d >= std::max(k - 1, 2); --d) {
        const int64_t cnt = v_at_least(d) - v_at_least(d + 1);
        if (cnt > 0) lb.push_back({d - 1, (int32_t)(v_at_least(d + 1) - n_heavy), (int32_t)cnt, 1});
    }
    std::vector<int32_t> tab;
    int64_t items = 0;
    size_t ih = 0, il = 0;
    while (ih < hb.size() || il < lb.size()) {
        const bool take_h = il >= lb.size() || (ih < hb.size() && hb[ih].key >= lb[il].key);
        const B b = take_h ? hb[ih++] : lb[il++];
        const int32_t parts = b.light ? light_parts(b.key + 1, k, pct) : arc_parts(b.key, k, pct);
        tab.push_back((int32_t)items);
        tab.push_back(b.first);
        tab.push_back(b.cnt);
        tab.push_back((b.key << 2) | (b.light ? kItemLightVertex : kItemHeavyArc));
        items += (int64_t)b.cnt * parts;
        if (items > 0x7fffffffLL) return fail(CITRON_EINVAL, "too many work items for one count");
    }
    const int32_t nb = (int32_t)(tab.size() / 4);
    tab.push_back((int32_t)items);
    tab.push_back(0);
    tab.push_back(0);
    tab.push_back(0);
    citron_status st = dalloc(&g->d_buckets[k], tab.size(), &g->device_bytes, "item buckets");
    if (st) return st;
    g->bucket_bytes[k] += (int64_t)(sizeof(int32_t) * tab.size());   // retired tables stay counted
    hipError_t e = hipMemcpy(g->d_buckets[k], tab.data(), sizeof(int32_t) * tab.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "item buckets");
    g->n_buckets[k] = nb;
    g->n_work[k] = (int32_t)items;
    g->bucket_split[k] = pct;
    return CITRON_OK;
}

// Vertex-rooted schedule of a k-clique count (Algorithm 2's unit): every
// vertex with out-degree >= k - 1 is one item, searched from its own root,
// largest out-degree first; heavy vertices (out-degree > 64) by the heavy
// engine, light ones as one light-engine unit each.  No vertex is split.
citron_status ensure_vbuckets(citron_graph* g, int32_t k)
{
    if (g->d_vbuckets[k]) return CITRON_OK;
    const int32_t D = std::max(g->max_outdeg, 2);
    auto v_at_least = [&](int32_t x) -> int64_t {   // vertices with out-degree >= x
        if (x > D) return 0;
        if (x < 2) x = 2;
        return g->h_vscan[(size_t)(D - x + 1)];
    };
    const int64_t n_heavy = v_at_least(kLightMaxDeg + 1);
    std::vector<int32_t> tab;
    int64_t items = 0;
    for (int32_t d = D; d >= std::max(k - 1, 2); --d) {
        const int64_t cnt = v_at_least(d) - v_at_least(d + 1);
        if (cnt <= 0) continue;
        const bool heavy = d > kLightMaxDeg;
        tab.push_back((int32_t)items);
        tab.push_back((int32_t)(heavy ? v_at_least(d + 1) : v_at_least(d + 1) - n_heavy));
        tab.push_back((int32_t)cnt);
        tab.push_back((d << 2) | (heavy ? kItemHeavyVertex : kItemLightRoot));
        items += cnt;
    }
    const int32_t nb = (int32_t)(tab.size() / 4);
    tab.push_back((int32_t)items);
    tab.push_back(0);
    tab.push_back(0);
    tab.push_back(0);
    citron_status st = dalloc(&g->d_vbuckets[k], tab.size(), &g->device_bytes, "vertex buckets");
    if (st) return st;
    g->vbucket_bytes[k] = (int64_t)(sizeof(int32_t) * tab.size());
    hipError_t e = hipMemcpy(g->d_vbuckets[k], tab.data(), sizeof(int32_t) * tab.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "vertex buckets");
    g->n_vbuckets[k] = nb;
    g->n_vwork[k] = (int32_t)items;
    return CITRON_OK;
}

QueryDesc make_query(const citron_graph* g, int32_t k, unsigned long long* acc, int32_t* ovf,
                     unsigned long long* per_arc, unsigned long long* stats, int32_t item_begin)
{
    QueryDesc q;
    memset(&q, 0, sizeof(q));
    q.dag_ptr = g->d_dag_ptr;
    q.dag_src = g->d_dag_src;
    q.order = g->pb.order;
    q.rows.rows_off = g->d_rows_off;
    q.rows.rows = g->d_rows;
    q.rows.arc_c = g->d_arc_c;
    q.rows.harcs = g->d_harcs;
    q.acc = acc;
    q.overflow = ovf;
    q.per_arc = per_arc;
    q.stats = stats;
    q.k = k;
    q.buckets = g->d_buckets[k];
    q.n_buckets = g->n_buckets[k];
    q.light_first = g->plan.n_heavy;
    q.n_work = g->n_work[k];
    q.item_begin = item_begin;
    q.n_items = q.n_work;
    q.item_stride = 1;
    q.split_pct = g->bucket_split[k];
    return q;
}

// Validity of a count request; sets *trivial when the answer is known
// without the kernel.
citron_status check_count_args(const citron_graph* g, int32_t k, bool* trivial, uint64_t* value)
{
    *trivial = false;
    *value = 0;
    if (!g) return fail(CITRON_EINVAL, "graph is NULL");
    if (k < 1 || k > CITRON_KMAX) return fail(CITRON_EINVAL, "k must be in 1..CITRON_KMAX");
    if (g->state != 1) return fail(CITRON_ESTATE, "citron_order must be called before counting");
    if (k == 1) { *trivial = true; *value = (uint64_t)g->n; return CITRON_OK; }
    if (k == 2) { *trivial = true; *value = (uint64_t)g->m; return CITRON_OK; }
    // a rooted k-clique needs a vertex with k-1 out-neighbours
    if (k - 1 > g->max_outdeg) { *trivial = true; *value = 0; return CITRON_OK; }
    if (g->max_outdeg > kMaxDeg)
        return fail(CITRON_EINVAL, "out-degree above 4096 in the degree-ordered DAG is not supported");
    return CITRON_OK;
}

// (slot, part) items of an arc list, in device buffers freed with the object.
struct ListItems {
    int32_t* parts = nullptr;
    int32_t* offs = nullptr;
    int32_t* ws = nullptr;
    int32_t* items = nullptr;
    int32_t total = 0;
    ~ListItems()
    {
        for (int32_t* p : {parts, offs, ws, items})
            if (p) (void)hipFree(p);
    }
    citron_status build(const citron_graph* g, const int32_t* arcs, int32_t n, int32_t k, hipStream_t s)
    {
        if (hipMalloc((void**)&parts, sizeof(int32_t) * (size_t)n) != hipSuccess ||
            hipMalloc((void**)&offs, sizeof(int32_t) * ((size_t)n + 1)) != hipSuccess ||
            hipMalloc((void**)&ws, sizeof(int32_t) * scan_workspace_ints(n)) != hipSuccess)
            return fail(CITRON_ENOMEM, "hipMalloc failed for the arc list");
        hipError_t e = launch_list_parts(arcs, n, g->d_dag_src, g->d_dag_ptr, g->d_arc_c, k, g->tuning.split_pct,
                                         parts, s);
        if (e == hipSuccess) e = scan_exclusive(parts, offs, n, ws, s);
        if (e == hipSuccess) e = hipMemcpyAsync(&g->h_small->ends[0], offs + n, sizeof(int32_t),
                                                hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "arc list parts");
        total = g->h_small->ends[0];
        if (hipMalloc((void**)&items, sizeof(int32_t) * 2 * ((size_t)total + 1)) != hipSuccess)
            return fail(CITRON_ENOMEM, "hipMalloc failed for the arc list");
        e = launch_list_items(n, parts, offs, items, s);
        if (e != hipSuccess) return hip_fail(e, "arc list items");
        return CITRON_OK;
    }
};

// One query through the count kernel; synchronous on the graph's stream.
static citron_status run_single(citron_graph* g, int32_t k, unsigned long long* per_arc, bool stats,
                                uint64_t* out_count, const int32_t* arc_list = nullptr, int32_t n_list = 0,
                                int32_t part = 0, int32_t nparts = 1, uint64_t* stats_out = nullptr,
                                bool vertex_rooted = false)
{
    std::lock_guard<std::mutex> lock(g->mu);
    hipError_t e = hipSetDevice(g->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    citron_status st = ensure_rows(g);
    if (st) return st;
    const uint64_t seed = g->seed_pending ? g->seed_base : 0;
    g->seed_pending = false;
    hipStream_t s = g->stream;
    if (stats) memset(g->h_small->stats, 0, sizeof(g->h_small->stats));
    if (vertex_rooted) {
        // the vertex-rooted unit runs the kernel for every k >= 3 (no
        // triangle shortcut: its k = 3 is the kernel's degrees-only level)
        st = ensure_vbuckets(g, k);
        if (st) return st;
    } else if (k == 3 && arc_list) {
        e = launch_gather_arc_c(arc_list, n_list, g->d_arc_c, per_arc, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "per-arc copy");
        *out_count = 0;   // the caller sums the listed arcs
        return CITRON_OK;
    }
    if (!vertex_rooted && k == 3 && part != 0) {   // a strided part of the triangle sum: all in part 0
        *out_count = 0;
        return CITRON_OK;
    }
    if (!vertex_rooted && k == 3) {
        // triangles: the popcounts of the rows, summed by the build
        if (per_arc) {
            e = launch_arc_c_to_u64(g->m, g->d_arc_c, per_arc, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess) return hip_fail(e, "per-arc copy");
        }
        const uint64_t c = seed + g->tri;
        *out_count = c;
        if (g->tri_ovf || c < seed) return fail(CITRON_EOVERFLOW, "count is >= 2^64; value is mod 2^64");
        return CITRON_OK;
    }
    if (!vertex_rooted) {
        st = ensure_buckets(g, k);
        if (st) return st;
    }
    const citron_tuning& t = g->tuning;
    const int wg = t.wg_waves;
    const int32_t blocks = device_cus(g->device) * t.blocks_per_cu;
    // a unit rooted at a vertex has one more level to choose than one rooted
    // at an arc: its stacks are sized as for k + 1
    const int32_t stack_k = vertex_rooted ? k + 1 : k;
    const int64_t swords = count_scratch_words(g->max_outdeg, stack_k, wg);
    st = ensure_scratch(g, std::max<int64_t>(swords * 8 * blocks, 8));
    if (st) return st;
    if (stats && !g->d_stats) {
        st = dalloc(&g->d_stats, kNumStats, &g->device_bytes, "stats");
        if (st) return st;
    }
    SmallDev* sd = g->d_small;
    if ((e = launch_fill_u64(&sd->acc, seed, 1, s)) != hipSuccess ||
        (e = launch_fill_i32(&sd->overflow, 0, 1, s)) != hipSuccess ||
        (e = launch_fill_i32(&sd->item_ctr, 0, 1, s)) != hipSuccess)
        return hip_fail(e, "fill");
    if (stats && ((e = launch_fill_u64(g->d_stats, 0, kNumStats, s)) != hipSuccess ||
                  (e = launch_fill_u64(g->d_stats + kStatWaveFirst, ~0ull, 1, s)) != hipSuccess))
        return hip_fail(e, "fill");
    if (per_arc && (e = launch_fill_u64(per_arc, 0, arc_list ? n_list : g->m, s)) != hipSuccess)
        return hip_fail(e, "fill");
    g->h_small->query = make_query(g, k, &sd->acc, &sd->overflow, per_arc, stats ? g->d_stats : nullptr, 0);
    if (vertex_rooted) {
        QueryDesc& q = g->h_small->query;
        q.buckets = g->d_vbuckets[k];
        q.n_buckets = g->n_vbuckets[k];
        q.n_work = g->n_vwork[k];
        q.n_items = q.n_work;
    }
    ListItems li;
    if (nparts > 1) {
        // items part, part + nparts, part + 2 nparts, ... of the schedule
        QueryDesc& q = g->h_small->query;
        q.item_lo = part;
        q.item_stride = nparts;
        q.n_items = q.n_work > part ? (q.n_work - part + nparts - 1) / nparts : 0;
    }
    if (arc_list) {
        // items of the listed arcs: heavy ones split into parts like the full schedule
        st = li.build(g, arc_list, n_list, k, s);
        if (st) return st;
        g->h_small->query.arc_list = arc_list;
        g->h_small->query.arc_items = li.items;
        g->h_small->query.n_items = li.total;
    }
    if (!g->d_query) {
        st = dalloc(&g->d_query, 1, &g->device_bytes, "query");
        if (st) return st;
    }
    e = hipMemcpyAsync(g->d_query, &g->h_small->query, sizeof(QueryDesc), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(query)");
    CountLaunch cl;
    cl.queries = g->d_query;
    cl.n_queries = 1;
    cl.total_items = g->h_small->query.n_items;
    cl.item_ctr = &sd->item_ctr;
    cl.scratch = g->d_scratch;
    cl.scratch_words = swords;
    cl.max_k = stack_k;
    cl.blocks = blocks;
    cl.wg_waves = wg;
    cl.lds_bytes = count_lds_bytes(arc_max_for(t, stack_k), stack_k, wg, per_arc != nullptr);
    cl.flush_rows = t.flush_rows;
    cl.arc_lds_max = arc_max_for(t, stack_k);
    cl.stats = stats;
    cl.per_arc = per_arc != nullptr;
    e = launch_count(cl, s);
    if (e != hipSuccess) return hip_fail(e, "count kernel launch");
    e = hipMemcpyAsync(&g->h_small->acc, &sd->acc, sizeof(uint64_t) + sizeof(int32_t) * 2,
                       hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(result)");
    if (stats) {
        e = hipMemcpyAsync(g->h_small->stats, g->d_stats, sizeof(uint64_t) * kNumStats,
                           hipMemcpyDeviceToHost, s);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(stats)");
    }
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "count kernel");
    *out_count = g->h_small->acc;
    if (stats && stats_out) {
        // copied while the graph is still locked: another call may reuse
        // the pinned mirror as soon as the lock is released
        memcpy(stats_out, g->h_small->stats, sizeof(uint64_t) * kNumStats);
        stats_out[kStatVertices] = g->build_stats[kStatVertices];
        stats_out[kStatRows] = g->build_stats[kStatRows];
        stats_out[kStatEntries] = g->build_stats[kStatEntries];
        stats_out[kStatBytes] = g->build_stats[kStatBytes];
    }
    if (g->h_small->overflow) return fail(CITRON_EOVERFLOW, "count is >= 2^64; value is mod 2^64");
    return CITRON_OK;
}

}  // namespace citron

// ====================================================================== ABI

extern "C" {

citron_status citron_load_csr(int32_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col_idx,
                              uint32_t flags, void* stream, citron_graph** out)
{
    if (!out) return fail(CITRON_EINVAL, "out is NULL");
    *out = nullptr;
    // the ordering and validation kernels give each vertex one wave: n * 64
    // work-items must fit a dispatch's 32-bit grid size
    if (n < 0 || n >= (1 << 26)) return fail(CITRON_EINVAL, "n must be in 0..2^26-1");
    if (nnz < 0 || nnz > 0x7fffffffLL) return fail(CITRON_EINVAL, "nnz must be in 0..2^31-1");
    if (nnz % 2) return fail(CITRON_EINVAL, "nnz must be even for a symmetric graph");
    if (!row_ptr) return fail(CITRON_EINVAL, "row_ptr is NULL");
    if (nnz > 0 && !col_idx) return fail(CITRON_EINVAL, "col_idx is NULL");
    if (flags & ~CITRON_DEVICE_PTRS) return fail(CITRON_EINVAL, "unknown flags");
    const bool dev_ptrs = (flags & CITRON_DEVICE_PTRS) != 0;

    citron_graph* g = new (std::nothrow) citron_graph();
    if (!g) return fail(CITRON_ENOMEM, "host allocation failed");
    hipError_t e = hipGetDevice(&g->device);
    if (e != hipSuccess) { delete g; return hip_fail(e, "hipGetDevice"); }
    g->stream = (hipStream_t)stream;
    g->n = n;
    g->nnz = nnz;
    g->m = nnz / 2;
    g->tuning = default_tuning();
    citron_status st;
    int64_t* acct = &g->device_bytes;
    if ((st = dalloc(&g->d_row_ptr, (size_t)n + 1, acct, "row_ptr")) ||
        (st = dalloc(&g->d_col, (size_t)nnz, acct, "col_idx")) ||
        (st = dalloc(&g->d_small, 1, acct, "counters"))) {
        free_graph_memory(g);
        delete g;
        return st;
    }
    e = hipHostMalloc((void**)&g->h_small, sizeof(SmallHost), hipHostMallocDefault);
    if (e != hipSuccess) { free_graph_memory(g); delete g; return fail(CITRON_ENOMEM, "hipHostMalloc"); }
    memset(g->h_small, 0, sizeof(SmallHost));
    const hipMemcpyKind kind = dev_ptrs ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    hipStream_t s = g->stream;
    e = hipMemcpyAsync(g->d_row_ptr, row_ptr, sizeof(int32_t) * ((size_t)n + 1), kind, s);
    if (e == hipSuccess && nnz > 0)
        e = hipMemcpyAsync(g->d_col, col_idx, sizeof(int32_t) * (size_t)nnz, kind, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(g->h_small->ends, g->d_row_ptr, sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(g->h_small->ends + 1, g->d_row_ptr + n, sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) { free_graph_memory(g); delete g; return hip_fail(e, "copying the CSR"); }
    if (g->h_small->ends[0] != 0 || g->h_small->ends[1] != nnz) {
        free_graph_memory(g);
        delete g;
        return fail(CITRON_EINVAL, "row_ptr[0] must be 0 and row_ptr[n] must equal nnz");
    }
    // device-side validation: offsets first (so that rows are in range), then entries
    for (int stage = 0; stage < 2; ++stage) {
        int32_t* err = &g->d_small->err;
        e = launch_fill_i32(err, 0, 1, s);
        if (e == hipSuccess) e = launch_validate(n, nnz, g->d_row_ptr, g->d_col, err, stage, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(&g->h_small->err, err, sizeof(int32_t), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) { free_graph_memory(g); delete g; return hip_fail(e, "validation"); }
        const int32_t bits = g->h_small->err;
        if (bits) {
            std::string why;
            if (bits & 1) why += " row_ptr not non-decreasing within [0, nnz];";
            if (bits & 2) why += " column id out of range;";
            if (bits & 4) why += " self-loop;";
            if (bits & 8) why += " row not strictly ascending (unsorted or duplicate);";
            if (bits & 16) why += " graph not symmetric;";
            free_graph_memory(g);
            delete g;
            return fail(CITRON_EINVAL, "invalid CSR:" + why);
        }
    }
    *out = g;
    return CITRON_OK;
}

// Level-synchronous peeling (kernels_core.hip): g->d_key[v] = the round in
// which v leaves.  Frontier buffers are temporary.
static citron_status peel_key(citron_graph* g)
{
    hipStream_t s = g->stream;
    int64_t* acct = &g->device_bytes;
    citron_status st;
    if (!g->d_key && (st = dalloc(&g->d_key, (size_t)g->n + 1, acct, "order key"))) return st;
    int32_t *deg = nullptr, *fa = nullptr, *fb = nullptr;
    if ((st = dalloc(&deg, (size_t)g->n + 1, nullptr, "peeling")) ||
        (st = dalloc(&fa, (size_t)g->n + 1, nullptr, "peeling")) ||
        (st = dalloc(&fb, (size_t)g->n + 1, nullptr, "peeling"))) {
        dfree(deg); dfree(fa); dfree(fb);
        return st;
    }
    int32_t* cnt = g->d_small->peel;          // [0], [1]: frontier sizes, [2]: smallest degree
    int32_t* hp = g->h_small->peel;
    auto sync_read = [&](int32_t* dst, const int32_t* src, int count) -> hipError_t {
        hipError_t e = hipMemcpyAsync(dst, src, sizeof(int32_t) * (size_t)count, hipMemcpyDeviceToHost, s);
        return e == hipSuccess ? hipStreamSynchronize(s) : e;
    };
    hipError_t e = launch_fill_i32(cnt, 0, 2, s);
    if (e == hipSuccess) e = launch_fill_i32(cnt + 2, 0x7fffffff, 1, s);
    if (e == hipSuccess) e = launch_peel_init(g->n, g->d_row_ptr, deg, g->d_key, cnt + 2, s);
    if (e == hipSuccess) e = sync_read(hp, cnt, 3);
    int32_t t = hp[2], r = 0, remaining = g->n, nf = 0;
    int32_t* cur = fa;
    int32_t* nxt = fb;
    int cur_slot = 0;
    while (e == hipSuccess && remaining > 0) {
        if (nf == 0) {
            // no vertex left at degree <= t: raise t to the smallest degree present
            if (r > 0) {
                e = launch_fill_i32(cnt + 2, 0x7fffffff, 1, s);
                if (e == hipSuccess) e = launch_peel_min(g->n, deg, g->d_key, cnt + 2, s);
                if (e == hipSuccess) e = sync_read(hp + 2, cnt + 2, 1);
                if (e != hipSuccess) break;
                t = hp[2];
            }
            e = launch_fill_i32(cnt + cur_slot, 0, 1, s);
            if (e == hipSuccess) e = launch_peel_collect(g->n, deg, g->d_key, t, cur, cnt + cur_slot, s);
            if (e == hipSuccess) e = sync_read(hp + cur_slot, cnt + cur_slot, 1);
            if (e != hipSuccess) break;
            nf = hp[cur_slot];
            if (nf <= 0) { e = hipErrorUnknown; break; }     // cannot happen while vertices remain
        }
        e = launch_fill_i32(cnt + (1 - cur_slot), 0, 1, s);
        if (e == hipSuccess)
            e = launch_peel_round(nf, cur, g->d_row_ptr, g->d_col, deg, g->d_key, t, r, nxt, cnt + (1 - cur_slot), s);
        if (e == hipSuccess) e = sync_read(hp + (1 - cur_slot), cnt + (1 - cur_slot), 1);
        if (e != hipSuccess) break;
        remaining -= nf;
        ++r;
        nf = hp[1 - cur_slot];
        std::swap(cur, nxt);
        cur_slot = 1 - cur_slot;
    }
    dfree(deg);
    dfree(fa);
    dfree(fb);
    if (e != hipSuccess) return hip_fail(e, "peeling kernels");
    g->peel_rounds = r;
    return CITRON_OK;
}

// Ordering phase: the DAG of the degree ordering (Section IV, Algorithm 3),
// or of the core ordering (key = peeling round) with the same kernels.
static citron_status order_impl(citron_graph* g, int kind)
{
    if (!g) return fail(CITRON_EINVAL, "graph is NULL");
    std::lock_guard<std::mutex> lock(g->mu);
    if (g->state == 1) {
        if (g->order_kind == kind) return CITRON_OK;
        return fail(CITRON_ESTATE, "the graph is already ordered by the other ordering");
    }
    hipError_t e = hipSetDevice(g->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    int64_t* acct = &g->device_bytes;
    citron_status st;
    g->scan_ws_ints = scan_workspace_ints((int64_t)g->n + 1) + 64;
    // a call that failed part-way keeps what it allocated; a retry reuses it
    if ((!g->d_outdeg && (st = dalloc(&g->d_outdeg, (size_t)g->n + 1, acct, "outdeg"))) ||
        (!g->d_dag_ptr && (st = dalloc(&g->d_dag_ptr, (size_t)g->n + 1, acct, "dag_ptr"))) ||
        (!g->d_dag_col && (st = dalloc(&g->d_dag_col, (size_t)g->m, acct, "dag_col"))) ||
        (!g->d_dag_src && (st = dalloc(&g->d_dag_src, (size_t)g->m, acct, "dag_src"))) ||
        (!g->d_scan_ws && (st = dalloc(&g->d_scan_ws, g->scan_ws_ints, acct, "scan workspace"))))
        return st;
    if (kind == 1 && g->n > 0 && (st = peel_key(g))) return st;
    hipStream_t s = g->stream;
    int32_t* mx = &g->d_small->max_outdeg;
    e = launch_fill_i32(mx, 0, 1, s);
    if (e == hipSuccess)
        e = launch_orient(g->n, g->d_row_ptr, g->d_col, g->d_outdeg, g->d_dag_ptr, g->d_dag_col,
                          g->d_dag_src, mx, g->d_scan_ws, s, kind == 1 ? g->d_key : nullptr);
    if (e == hipSuccess && g->n == 0) e = launch_fill_i32(g->d_dag_ptr, 0, 1, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(&g->h_small->max_outdeg, mx, sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(g->h_small->ends, g->d_dag_ptr + g->n, sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "ordering kernels");
    if (g->h_small->ends[0] != g->m) return fail(CITRON_EDEVICE, "ordering produced a wrong arc count");
    g->max_outdeg = g->h_small->max_outdeg;
    g->order_kind = kind;
    g->state = 1;
    // the schedule of the counting phase is part of ordering the graph
    return ensure_plan(g, g->tuning);
}

citron_status citron_order(citron_graph* g) { return order_impl(g, 0); }

citron_status citron_order_core(citron_graph* g) { return order_impl(g, 1); }

citron_status citron_get_order_key(const citron_graph* g, int32_t* key, int32_t* rounds)
{
    if (!g) return fail(CITRON_EINVAL, "graph is NULL");
    if (g->state != 1) return fail(CITRON_ESTATE, "citron_order or citron_order_core must be called first");
    if (!key && g->n > 0) return fail(CITRON_EINVAL, "key is NULL");
    citron_graph* gm = const_cast<citron_graph*>(g);
    std::lock_guard<std::mutex> lock(gm->mu);
    if (rounds) *rounds = g->order_kind == 1 ? g->peel_rounds : 0;
    if (g->n == 0) return CITRON_OK;
    hipError_t e = hipSetDevice(g->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    if (g->order_kind == 1) {
        e = hipMemcpyAsync(key, g->d_key, sizeof(int32_t) * (size_t)g->n, hipMemcpyDeviceToHost, g->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
        if (e != hipSuccess) return hip_fail(e, "copying the order key");
        return CITRON_OK;
    }
    // degree ordering: the key is the degree
    std::vector<int32_t> rp((size_t)g->n + 1);
    e = hipMemcpyAsync(rp.data(), g->d_row_ptr, sizeof(int32_t) * rp.size(), hipMemcpyDeviceToHost, g->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
    if (e != hipSuccess) return hip_fail(e, "copying row_ptr");
    for (int32_t v = 0; v < g->n; ++v) key[v] = rp[(size_t)v + 1] - rp[(size_t)v];
    return CITRON_OK;
}

uint64_t citron_count(citron_graph* g, int32_t k, citron_status* st_out)
{
    citron_status dummy;
    citron_status* st = st_out ? st_out : &dummy;
    bool trivial;
    uint64_t v;
    *st = check_count_args(g, k, &trivial, &v);
    if (*st) return 0;
    if (trivial) return v;
    uint64_t c = 0;
    *st = run_single(g, k, nullptr, false, &c);
    if (*st && *st != CITRON_EOVERFLOW) return 0;
    return c;
}

uint64_t citron_count_vertex_rooted(citron_graph* g, int32_t k, citron_status* st_out)
{
    citron_status dummy;
    citron_status* st = st_out ? st_out : &dummy;
    bool trivial;
    uint64_t v;
    *st = check_count_args(g, k, &trivial, &v);
    if (*st) return 0;
    if (trivial) return v;
    uint64_t c = 0;
    *st = run_single(g, k, nullptr, false, &c, nullptr, 0, 0, 1, nullptr, true);
    if (*st && *st != CITRON_EOVERFLOW) return 0;
    return c;
}

uint64_t citron_count_part(citron_graph* g, int32_t k, int32_t part, int32_t nparts, citron_status* st_out)
{
    citron_status dummy;
    citron_status* st = st_out ? st_out : &dummy;
    if (nparts < 1 || part < 0 || part >= nparts) {
        *st = fail(CITRON_EINVAL, "part must be in 0..nparts-1");
        return 0;
    }
    bool trivial;
    uint64_t v;
    *st = check_count_args(g, k, &trivial, &v);
    if (*st) return 0;
    if (trivial) return part == 0 ? v : 0;
    uint64_t c = 0;
    *st = run_single(g, k, nullptr, false, &c, nullptr, 0, part, nparts);
    if (*st && *st != CITRON_EOVERFLOW) return 0;
    return c;
}

uint64_t citron_count_per_arc(citron_graph* g, int32_t k, uint64_t* per_arc, citron_status* st_out)
{
    citron_status dummy;
    citron_status* st = st_out ? st_out : &dummy;
    if (k < 2) { *st = fail(CITRON_EINVAL, "per-arc counts need k >= 2"); return 0; }
    if (!per_arc && g && g->m > 0) { *st = fail(CITRON_EINVAL, "per_arc is NULL"); return 0; }
    bool trivial;
    uint64_t v;
    *st = check_count_args(g, k, &trivial, &v);
    if (*st) return 0;
    if (trivial) {
        std::lock_guard<std::mutex> lock(g->mu);
        hipError_t e = launch_fill_u64((unsigned long long*)per_arc, k == 2 ? 1ull : 0ull, g->m, g->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
        if (e != hipSuccess) { *st = hip_fail(e, "fill"); return 0; }
        return v;
    }
    uint64_t c = 0;
    *st = run_single(g, k, (unsigned long long*)per_arc, false, &c);
    if (*st && *st != CITRON_EOVERFLOW) return 0;
    return c;
}

uint64_t citron_count_arcs(citron_graph* g, int32_t k, const int32_t* arcs, int32_t n, uint64_t* out,
                           citron_status* st_out)
{
    citron_status dummy;
    citron_status* st = st_out ? st_out : &dummy;
    if (k < 2) { *st = fail(CITRON_EINVAL, "per-arc counts need k >= 2"); return 0; }
    if (n < 0 || n > (1 << 26) || (n > 0 && (!arcs || !out))) {
        *st = fail(CITRON_EINVAL, "arc list: NULL pointer or n outside 0..2^26");
        return 0;
    }
    bool trivial;
    uint64_t v;
    *st = check_count_args(g, k, &trivial, &v);
    if (*st) return 0;
    if (n == 0) return 0;
    {
        std::lock_guard<std::mutex> lock(g->mu);
        hipError_t e = hipSetDevice(g->device);
        int32_t* err = &g->d_small->err;
        if (e == hipSuccess) e = launch_fill_i32(err, 0, 1, g->stream);
        if (e == hipSuccess) e = launch_check_arcs(arcs, n, g->m, err, g->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(&g->h_small->err, err, sizeof(int32_t), hipMemcpyDeviceToHost, g->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
        if (e != hipSuccess) { *st = hip_fail(e, "arc list check"); return 0; }
        if (g->h_small->err) { *st = fail(CITRON_EINVAL, "arc index out of range"); return 0; }
        if (trivial) {
            e = launch_fill_u64((unsigned long long*)out, k == 2 ? 1ull : 0ull, n, g->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
            if (e != hipSuccess) { *st = hip_fail(e, "fill"); return 0; }
            return k == 2 ? (uint64_t)n : 0;
        }
    }
    uint64_t c = 0;
    *st = run_single(g, k, (unsigned long long*)out, false, &c, arcs, n);
    if (*st && *st != CITRON_EOVERFLOW) return 0;
    if (k == 3) {   // sum of the gathered sizes
        std::vector<uint64_t> h((size_t)n);
        if (hipMemcpy(h.data(), out, sizeof(uint64_t) * (size_t)n, hipMemcpyDeviceToHost) != hipSuccess) {
            *st = fail(CITRON_EDEVICE, "copy");
            return 0;
        }
        for (uint64_t x : h) c += x;
    }
    return c;
}

citron_status citron_list_arcs(citron_graph* g, int32_t k, const int32_t* arcs, int32_t n_arcs, int64_t* offsets,
                               int32_t* cliques, int64_t cap, int64_t* total)
{
    if (!total) return fail(CITRON_EINVAL, "total is NULL");
    *total = 0;
    if (!g) return fail(CITRON_EINVAL, "graph is NULL");
    if (k < 2 || k > kListMaxK) return fail(CITRON_EINVAL, "listing needs 2 <= k <= 16");
    if (n_arcs < 0 || n_arcs > (1 << 26) || !offsets || (n_arcs > 0 && !arcs))
        return fail(CITRON_EINVAL, "arc list: NULL pointer or n outside 0..2^26");
    if (cap < 0) return fail(CITRON_EINVAL, "cap must be >= 0");
    if (g->state != 1) return fail(CITRON_ESTATE, "citron_order must be called before listing");
    // exact per-arc counts size the output (checks the arc indices too)
    unsigned long long* per = nullptr;
    long long* ws = nullptr;
    citron_status st = CITRON_OK;
    hipError_t e = hipSetDevice(g->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    const size_t nws = scan64_workspace(n_arcs);
    if (hipMalloc((void**)&per, sizeof(unsigned long long) * (size_t)std::max(n_arcs, 1)) != hipSuccess ||
        hipMalloc((void**)&ws, sizeof(long long) * nws) != hipSuccess) {
        if (per) (void)hipFree(per);
        return fail(CITRON_ENOMEM, "hipMalloc failed for the listing");
    }
    if (n_arcs > 0) {
        citron_status cst;
        (void)citron_count_arcs(g, k, arcs, n_arcs, (uint64_t*)per, &cst);
        if (cst == CITRON_EOVERFLOW) cst = fail(CITRON_EINVAL, "more cliques than a 64-bit count holds");
        st = cst;
    }
    int64_t tot = 0;
    if (!st) {
        std::lock_guard<std::mutex> lock(g->mu);
        hipStream_t s = g->stream;
        e = scan_exclusive64(per, (long long*)offsets, n_arcs, ws, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(&g->h_small->stats[0], offsets + n_arcs, sizeof(int64_t), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) st = hip_fail(e, "listing offsets");
        tot = (int64_t)g->h_small->stats[0];
        *total = tot;
        if (!st && tot > 0 && (tot > cap || !cliques))
            st = fail(CITRON_ENOMEM, "the output holds fewer cliques than the arcs have (see *total)");
        if (!st && tot > 0) {
            if (!g->rows_valid) st = ensure_rows(g);
            ListParams P;
            P.arcs = arcs;
            P.n_arcs = n_arcs;
            P.k = k;
            P.dag_ptr = g->d_dag_ptr;
            P.dag_col = g->d_dag_col;
            P.dag_src = g->d_dag_src;
            P.rows_off = g->d_rows_off;
            P.rows = g->d_rows;
            P.offsets = (const long long*)offsets;
            P.out = cliques;
            P.cursor = &g->d_small->item_ctr;
            P.err = &g->d_small->err;
            if (!st) {
                e = launch_fill_i32(P.cursor, 0, 1, s);
                if (e == hipSuccess) e = launch_fill_i32(P.err, 0, 1, s);
                if (e == hipSuccess) e = launch_list_arcs(P, device_cus(g->device) * 8, s);
                if (e == hipSuccess)
                    e = hipMemcpyAsync(&g->h_small->err, P.err, sizeof(int32_t), hipMemcpyDeviceToHost, s);
                if (e == hipSuccess) e = hipStreamSynchronize(s);
                if (e != hipSuccess) st = hip_fail(e, "listing kernel");
                else if (g->h_small->err)
                    st = fail(CITRON_EDEVICE, "listing found a different number of cliques than the count");
            }
        }
    }
    (void)hipFree(per);
    (void)hipFree(ws);
    return st;
}

citron_status citron_work_stats(citron_graph* g, int32_t k, uint64_t* stats)
{
    if (!stats) return fail(CITRON_EINVAL, "stats is NULL");
    memset(stats, 0, sizeof(uint64_t) * CITRON_NSTATS);
    bool trivial;
    uint64_t v;
    citron_status st = check_count_args(g, k, &trivial, &v);
    if (st) return st;
    if (trivial) return CITRON_OK;
    uint64_t c = 0;
    st = run_single(g, k, nullptr, true, &c, nullptr, 0, 0, 1, stats);
    if (st && st != CITRON_EOVERFLOW) return st;
    return CITRON_OK;
}

citron_status citron_get_dag(const citron_graph* g, int32_t* dag_ptr, int32_t* dag_col)
{
    if (!g) return fail(CITRON_EINVAL, "graph is NULL");
    if (g->state != 1) return fail(CITRON_ESTATE, "citron_order must be called first");
    if (!dag_ptr || (g->m > 0 && !dag_col)) return fail(CITRON_EINVAL, "output pointer is NULL");
    citron_graph* gm = const_cast<citron_graph*>(g);
    std::lock_guard<std::mutex> lock(gm->mu);
    hipError_t e = hipSetDevice(g->device);
    if (e == hipSuccess)
        e = hipMemcpyAsync(dag_ptr, g->d_dag_ptr, sizeof(int32_t) * ((size_t)g->n + 1),
                           hipMemcpyDeviceToHost, g->stream);
    if (e == hipSuccess && g->m > 0)
        e = hipMemcpyAsync(dag_col, g->d_dag_col, sizeof(int32_t) * (size_t)g->m, hipMemcpyDeviceToHost,
                           g->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
    if (e != hipSuccess) return hip_fail(e, "copying the DAG");
    return CITRON_OK;
}

citron_status citron_graph_info(const citron_graph* g, int64_t* n, int64_t* m, int32_t* max_outdeg,
                                int64_t* device_bytes)
{
    if (!g) return fail(CITRON_EINVAL, "graph is NULL");
    if (n) *n = g->n;
    if (m) *m = g->m;
    if (max_outdeg) *max_outdeg = g->state == 1 ? g->max_outdeg : -1;
    if (device_bytes) *device_bytes = g->device_bytes;
    return CITRON_OK;
}

citron_status citron_set_tuning(citron_graph* g, const citron_tuning* t)
{
    if (!g) return fail(CITRON_EINVAL, "graph is NULL");
    citron_tuning r;
    citron_status st = resolve_tuning(t, &r);
    if (st) return st;
    const bool resplit = r.split_pct != g->tuning.split_pct;
    if (resplit) batch_forget_graph(g);   // captured batches hold its schedule
    std::lock_guard<std::mutex> lock(g->mu);
    g->tuning = r;
    return CITRON_OK;
}

citron_status citron_get_tuning(const citron_graph* g, citron_tuning* t)
{
    if (!g || !t) return fail(CITRON_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lock(const_cast<citron_graph*>(g)->mu);
    *t = g->tuning;
    return CITRON_OK;
}

void citron_free(citron_graph* g)
{
    if (!g) return;
    batch_forget_graph(g);
    {
        std::lock_guard<std::mutex> lock(g->mu);
        (void)hipSetDevice(g->device);
        if (g->stream) (void)hipStreamSynchronize(g->stream);
        else (void)hipDeviceSynchronize();
        free_graph_memory(g);
    }
    delete g;
}

const char* citron_last_error(void) { return g_last_error.c_str(); }

citron_status citron_device_info(int32_t* cus, int32_t* lds_bytes, char* name64)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    hipDeviceProp_t p;
    e = hipGetDeviceProperties(&p, dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
    if (cus) *cus = p.multiProcessorCount;
    if (lds_bytes) *lds_bytes = (int32_t)p.sharedMemPerBlock;
    if (name64) {
        strncpy(name64, p.gcnArchName, 63);
        name64[63] = 0;
    }
    return CITRON_OK;
}

citron_status citron_test_seed_accumulator(citron_graph* g, uint64_t base)
{
    if (!g) return fail(CITRON_EINVAL, "graph is NULL");
    std::lock_guard<std::mutex> lock(g->mu);
    g->seed_base = base;
    g->seed_pending = true;
    return CITRON_OK;
}

}  // extern "C"
