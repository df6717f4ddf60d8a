// Batched counts: many (graph, k) queries in one persistent launch of the
// count kernel.  Items of all queries form one global item space; each
// workgroup pulls items from one cursor, so short and long queries share
// the device without a launch (or a host round trip) per query.  The whole
// sequence -- counter resets, descriptor upload, kernel, result download --
// is captured once into a HIP graph per distinct query set and replayed on
// later calls with the same set.
#include "api_internal.h"

#include <algorithm>
#include <cstring>
#include <map>
#include <memory>
#include <vector>

namespace citron {

namespace {

struct BatchKey {
    std::vector<const citron_graph*> graphs;
    std::vector<int32_t> ks;
    int32_t tuning[sizeof(citron_tuning) / sizeof(int32_t)];
    bool operator<(const BatchKey& o) const
    {
        if (graphs != o.graphs) return graphs < o.graphs;
        if (ks != o.ks) return ks < o.ks;
        return memcmp(tuning, o.tuning, sizeof(tuning)) < 0;
    }
};

// Device and pinned host buffers of one captured batch.
struct BatchExec {
    int device = 0;
    int32_t nq = 0;                    // kernel queries
    int32_t total_items = 0;           // work items of the launch
    std::vector<int32_t> qmap;         // kernel query -> caller index
    unsigned long long* d_acc = nullptr;  // nq
    int32_t* d_ovf = nullptr;          // nq
    int32_t* d_item_ctr = nullptr;
    QueryDesc* d_q = nullptr;
    void* d_scratch = nullptr;
    QueryDesc* h_q = nullptr;          // pinned
    unsigned long long* h_acc = nullptr;  // pinned
    int32_t* h_ovf = nullptr;          // pinned
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<const citron_graph*> graphs;

    ~BatchExec()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (d_acc) (void)hipFree(d_acc);
        if (d_ovf) (void)hipFree(d_ovf);
        if (d_item_ctr) (void)hipFree(d_item_ctr);
        if (d_q) (void)hipFree(d_q);
        if (d_scratch) (void)hipFree(d_scratch);
        if (h_q) (void)hipHostFree(h_q);
        if (h_acc) (void)hipHostFree(h_acc);
        if (h_ovf) (void)hipHostFree(h_ovf);
    }
};

std::mutex g_batch_mu;
std::map<BatchKey, std::unique_ptr<BatchExec>> g_cache;

// Progress of the batch launch in flight, for queries from other threads:
// the kernel stores the items claimed (every 512th) into a host-mapped
// pinned word, which the host reads without any HIP call (a copy from the
// device could wait for compute units the launch holds).  Its device
// address is baked into captured launches, so the word lives until the
// process ends.  g_progress_mu guards the published total.
std::mutex g_progress_mu;
int32_t g_run_total = 0;
volatile int32_t* g_progress_word = nullptr;
int32_t* g_progress_dev = nullptr;

// The host-mapped progress word (allocated once, by the first batch).
int32_t* progress_device_word()
{
    if (!g_progress_dev) {
        void* h = nullptr;
        void* d = nullptr;
        if (hipHostMalloc(&h, 64, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) return nullptr;
        if (hipHostGetDevicePointer(&d, h, 0) != hipSuccess) { (void)hipHostFree(h); return nullptr; }
        *static_cast<volatile int32_t*>(h) = 0;
        g_progress_word = static_cast<volatile int32_t*>(h);
        g_progress_dev = static_cast<int32_t*>(d);
    }
    return g_progress_dev;
}
hipStream_t g_stream[64] = {nullptr};
constexpr size_t kMaxCached = 16;

hipStream_t batch_stream(int dev)
{
    if (dev < 0 || dev >= 64) return nullptr;
    if (!g_stream[dev]) {
        if (hipStreamCreateWithFlags(&g_stream[dev], hipStreamNonBlocking) != hipSuccess) g_stream[dev] = nullptr;
    }
    return g_stream[dev];
}

}  // namespace

// Drop cached batches that reference graph g (called when g is freed).
void batch_forget_graph(const citron_graph* g)
{
    std::lock_guard<std::mutex> lock(g_batch_mu);
    for (auto it = g_cache.begin(); it != g_cache.end();) {
        if (std::find(it->first.graphs.begin(), it->first.graphs.end(), g) != it->first.graphs.end())
            it = g_cache.erase(it);
        else
            ++it;
    }
}

citron_status batch_build(const BatchKey& key, const citron_tuning& t, BatchExec* be, hipStream_t s)
{
    const int32_t nq = (int32_t)key.ks.size();
    int32_t total_items = 0, max_k = 4;
    for (int32_t i = 0; i < nq; ++i) max_k = std::max(max_k, key.ks[i]);
    hipError_t e;
    const int wg = t.wg_waves;
    const int32_t blocks = device_cus(be->device) * t.blocks_per_cu;
    const int64_t swords = count_scratch_words(0, max_k, wg);
#define BALLOC(p, bytes)                                                              \
    do {                                                                              \
        e = hipMalloc((void**)&(p), (bytes) > 0 ? (bytes) : 8);                       \
        if (e != hipSuccess) return fail(CITRON_ENOMEM, "hipMalloc failed for batch"); \
    } while (0)
    BALLOC(be->d_acc, sizeof(unsigned long long) * nq);
    BALLOC(be->d_ovf, sizeof(int32_t) * nq);
    BALLOC(be->d_item_ctr, sizeof(int32_t));
    BALLOC(be->d_q, sizeof(QueryDesc) * nq);
    BALLOC(be->d_scratch, (size_t)(swords * 8 * blocks));
#undef BALLOC
    if (hipHostMalloc((void**)&be->h_q, sizeof(QueryDesc) * nq, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&be->h_acc, sizeof(unsigned long long) * nq, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&be->h_ovf, sizeof(int32_t) * nq, hipHostMallocDefault) != hipSuccess)
        return fail(CITRON_ENOMEM, "hipHostMalloc failed for batch");
    for (int32_t i = 0; i < nq; ++i) {
        be->h_q[i] = make_query(key.graphs[i], key.ks[i], be->d_acc + i, be->d_ovf + i, nullptr, nullptr,
                                total_items);
        total_items += be->h_q[i].n_items;
    }
    be->nq = nq;
    be->total_items = total_items;

    CountLaunch cl;
    cl.queries = be->d_q;
    cl.n_queries = nq;
    cl.total_items = total_items;
    cl.item_ctr = be->d_item_ctr;
    cl.scratch = reinterpret_cast<unsigned long long*>(be->d_scratch);
    cl.scratch_words = swords;
    cl.max_k = max_k;
    cl.blocks = blocks;
    cl.wg_waves = wg;
    cl.lds_bytes = count_lds_bytes(arc_max_for(t, max_k), max_k, wg, false);
    cl.flush_rows = t.flush_rows;
    cl.arc_lds_max = arc_max_for(t, max_k);
    cl.stats = false;
    cl.per_arc = false;
    cl.progress = progress_device_word();   // null: no progress reports

    // capture: resets, descriptor upload, kernel, download
    e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    hipError_t ce = launch_fill_u64(be->d_acc, 0, nq, s);
    if (ce == hipSuccess) ce = launch_fill_i32(be->d_ovf, 0, nq, s);
    if (ce == hipSuccess) ce = launch_fill_i32(be->d_item_ctr, 0, 1, s);
    if (ce == hipSuccess)
        ce = hipMemcpyAsync(be->d_q, be->h_q, sizeof(QueryDesc) * nq, hipMemcpyHostToDevice, s);
    if (ce == hipSuccess) ce = launch_count(cl, s);
    if (ce == hipSuccess)
        ce = hipMemcpyAsync(be->h_acc, be->d_acc, sizeof(unsigned long long) * nq, hipMemcpyDeviceToHost, s);
    if (ce == hipSuccess)
        ce = hipMemcpyAsync(be->h_ovf, be->d_ovf, sizeof(int32_t) * nq, hipMemcpyDeviceToHost, s);
    e = hipStreamEndCapture(s, &be->graph);
    if (ce != hipSuccess) return hip_fail(ce, "batch capture");
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&be->exec, be->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    return CITRON_OK;
}

}  // namespace citron

using namespace citron;

extern "C" citron_status citron_count_batch(citron_graph* const* gs, const int32_t* ks, int32_t nq,
                                            uint64_t* counts, citron_status* sts, const citron_tuning* tin)
{
    if (nq < 0) return fail(CITRON_EINVAL, "nq must be >= 0");
    if (nq == 0) return CITRON_OK;
    if (!gs || !ks || !counts) return fail(CITRON_EINVAL, "NULL argument");
    citron_tuning t;
    citron_status st = resolve_tuning(tin, &t);
    if (st) return st;

    std::vector<citron_status> qst(nq, CITRON_OK);
    BatchKey key;
    std::vector<int32_t> qmap;
    int dev = -1;
    for (int32_t i = 0; i < nq; ++i) {
        counts[i] = 0;
        bool trivial;
        uint64_t v;
        qst[i] = check_count_args(gs[i], ks[i], &trivial, &v);
        if (qst[i] == CITRON_OK && !trivial) {
            if (dev < 0) dev = gs[i]->device;
            if (gs[i]->device != dev) {
                qst[i] = fail(CITRON_EINVAL, "all graphs of a batch must live on one device");
                continue;
            }
            key.graphs.push_back(gs[i]);
            key.ks.push_back(ks[i]);
            qmap.push_back(i);
        } else if (qst[i] == CITRON_OK) {
            counts[i] = v;
        }
    }
    if (!key.ks.empty()) {
        memcpy(key.tuning, &t, sizeof(key.tuning));
        std::lock_guard<std::mutex> lock(g_batch_mu);
        hipError_t e = hipSetDevice(dev);
        if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
        // subgraph rows of every graph (built once per graph)
        std::vector<const citron_graph*> uniq(key.graphs.begin(), key.graphs.end());
        std::sort(uniq.begin(), uniq.end());
        uniq.erase(std::unique(uniq.begin(), uniq.end()), uniq.end());
        for (const citron_graph* cg : uniq) {
            citron_graph* g = const_cast<citron_graph*>(cg);
            std::lock_guard<std::mutex> gl(g->mu);
            st = ensure_rows(g);
            if (st) return st;
        }
        for (size_t j = 0; j < key.ks.size(); ++j) {
            citron_graph* g = const_cast<citron_graph*>(key.graphs[j]);
            if (key.ks[j] < 4) continue;
            std::lock_guard<std::mutex> gl(g->mu);
            st = ensure_buckets(g, key.ks[j]);
            if (st) return st;
        }
        // k = 3 is the build's triangle count; the rest go to the kernel
        BatchKey kkey;
        std::vector<int32_t> kmap;
        memcpy(kkey.tuning, key.tuning, sizeof(key.tuning));
        for (size_t j = 0; j < key.ks.size(); ++j) {
            if (key.ks[j] == 3) {
                counts[qmap[j]] = key.graphs[j]->tri;
                if (key.graphs[j]->tri_ovf) qst[qmap[j]] = CITRON_EOVERFLOW;
            } else {
                kkey.graphs.push_back(key.graphs[j]);
                kkey.ks.push_back(key.ks[j]);
                kmap.push_back(qmap[j]);
            }
        }
        if (!kkey.ks.empty()) {
            hipStream_t s = batch_stream(dev);
            if (!s) return fail(CITRON_EDEVICE, "could not create the batch stream");
            auto it = g_cache.find(kkey);
            if (it == g_cache.end()) {
                if (g_cache.size() >= kMaxCached) g_cache.clear();
                std::unique_ptr<BatchExec> be(new BatchExec());
                be->device = dev;
                be->qmap = kmap;
                st = batch_build(kkey, t, be.get(), s);
                if (st) return st;
                it = g_cache.emplace(kkey, std::move(be)).first;
            }
            BatchExec* be = it->second.get();
            {
                std::lock_guard<std::mutex> pl(g_progress_mu);
                if (g_progress_word) *g_progress_word = 0;
                g_run_total = be->total_items;
            }
            e = hipGraphLaunch(be->exec, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            {
                std::lock_guard<std::mutex> pl(g_progress_mu);
                g_run_total = 0;
            }
            if (e != hipSuccess) return hip_fail(e, "batch launch");
            for (int32_t j = 0; j < be->nq; ++j) {
                const int32_t i = kmap[j];
                counts[i] = be->h_acc[j];
                if (be->h_ovf[j]) qst[i] = CITRON_EOVERFLOW;
            }
        }
    }
    citron_status first = CITRON_OK;
    for (int32_t i = 0; i < nq; ++i) {
        if (sts) sts[i] = qst[i];
        if (qst[i] && !first) first = qst[i];
    }
    if (first == CITRON_EOVERFLOW) fail(CITRON_EOVERFLOW, "a batch count is >= 2^64");
    return first;
}

extern "C" citron_status citron_batch_progress(int32_t* items_taken, int32_t* items_total)
{
    if (!items_taken || !items_total) return fail(CITRON_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> pl(g_progress_mu);
    *items_total = g_run_total;
    const int32_t v = (g_run_total && g_progress_word) ? *g_progress_word : 0;
    *items_taken = v < g_run_total ? v : g_run_total;
    return CITRON_OK;
}
