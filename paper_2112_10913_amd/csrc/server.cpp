// Request server over resident graphs with continuous batching.
//
// A server owns one worker thread and one stream on the device that was
// current when it was created.  Requests (graph, k) are queued by
// citron_server_submit and admitted in arrival order as soon as an
// in-flight slot is free and their device footprint fits the memory
// budget.  The worker runs steps back to back: each step is one launch of
// the persistent count kernel over a bounded slice of every admitted
// request's remaining work items, so requests that arrive while others run
// join at the next step and share the device with them, and a request that
// finishes frees its slot for the next one.  Counts are exact integers, so
// a request's count does not depend on which requests it shares steps with.
#include "api_internal.h"

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <thread>

using namespace citron;

namespace {

int64_t now_ns()
{
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct Req {
    uint64_t tag = 0;
    int32_t gid = 0;
    int32_t k = 0;
    int64_t t_submit = 0;
    int64_t t_admit = 0;
    int32_t slot = -1;
    int32_t n_items = 0;
    int32_t cursor = 0;
    int64_t footprint = 0;
    bool fresh = true;        // accumulator not yet zeroed
    QueryDesc q;
};

// Items of one request per step, and of one step in total: small enough that
// a step ends in milliseconds, large enough to fill the device.
constexpr int32_t kItemsPerReq = 8192;
constexpr int32_t kItemsPerStep = 65536;

}  // namespace

struct citron_server {
    int device = 0;
    hipStream_t stream = nullptr;
    int64_t budget = 0;
    int32_t max_slots = 0;
    citron_tuning tuning;
    std::vector<citron_graph*> graphs;

    std::mutex mu;
    std::condition_variable cv;
    std::deque<Req> pending;
    std::vector<Req> active;           // admitted requests
    std::vector<int32_t> free_slots;
    std::deque<citron_result> done;
    int64_t used = 0;
    int64_t submitted = 0;
    int64_t returned = 0;
    bool stop = false;
    std::thread worker;

    // device: per slot accumulator and flag, the step's query table, the cursor
    unsigned long long* d_acc = nullptr;
    int32_t* d_ovf = nullptr;
    int32_t* d_item_ctr = nullptr;
    QueryDesc* d_q = nullptr;
    unsigned long long* d_scratch = nullptr;
    int64_t scratch_words = 0;
    // pinned host mirrors
    QueryDesc* h_q = nullptr;
    unsigned long long* h_acc = nullptr;
    int32_t* h_ovf = nullptr;
    std::string worker_error;
};

namespace {

// Device memory a request needs beyond its resident graph: its slot's
// accumulator and descriptor, and for k > 12 its share of the search stacks
// that live in device memory.
int64_t footprint_of(const citron_server* s, int32_t k)
{
    int64_t b = (int64_t)sizeof(QueryDesc) + 16;
    const int64_t blocks = (int64_t)device_cus(s->device) * s->tuning.blocks_per_cu;
    b += count_scratch_words(0, k, s->tuning.wg_waves) * 8 * blocks;
    return b;
}

void complete(citron_server* s, Req& r, uint64_t count, citron_status st)
{
    citron_result res;
    memset(&res, 0, sizeof(res));
    res.tag = r.tag;
    res.graph_id = r.gid;
    res.k = r.k;
    res.count = count;
    res.status = st;
    res.t_submit_ns = r.t_submit;
    res.t_admit_ns = r.t_admit ? r.t_admit : now_ns();
    res.t_done_ns = now_ns();
    s->done.push_back(res);
}

void worker_main(citron_server* s)
{
    (void)hipSetDevice(s->device);
    const int wg = s->tuning.wg_waves;
    const int32_t blocks = device_cus(s->device) * s->tuning.blocks_per_cu;
    for (;;) {
        std::vector<int32_t> fresh_slots;
        {
            std::unique_lock<std::mutex> lock(s->mu);
            s->cv.wait(lock, [&] { return s->stop || !s->pending.empty() || !s->active.empty(); });
            if (s->stop) return;
            // admission, in arrival order
            while (!s->pending.empty()) {
                Req& r = s->pending.front();
                citron_graph* g = s->graphs[(size_t)r.gid];
                bool trivial = false;
                uint64_t v = 0;
                citron_status st = check_count_args(g, r.k, &trivial, &v);
                if (st == CITRON_OK && (trivial || r.k == 3)) {
                    r.t_admit = now_ns();
                    if (!trivial) v = g->tri;
                    complete(s, r, v, (!trivial && g->tri_ovf) ? CITRON_EOVERFLOW : CITRON_OK);
                    s->pending.pop_front();
                    continue;
                }
                if (st) {
                    r.t_admit = now_ns();
                    complete(s, r, 0, st);
                    s->pending.pop_front();
                    continue;
                }
                r.footprint = footprint_of(s, r.k);
                if (r.footprint > s->budget) {
                    r.t_admit = now_ns();
                    complete(s, r, 0, CITRON_ENOMEM);
                    s->pending.pop_front();
                    continue;
                }
                if (s->free_slots.empty() || s->used + r.footprint > s->budget) break;
                {
                    std::lock_guard<std::mutex> gl(g->mu);
                    st = ensure_buckets(g, r.k);
                }
                if (st) {
                    r.t_admit = now_ns();
                    complete(s, r, 0, st);
                    s->pending.pop_front();
                    continue;
                }
                r.slot = s->free_slots.back();
                s->free_slots.pop_back();
                s->used += r.footprint;
                r.t_admit = now_ns();
                r.q = make_query(g, r.k, s->d_acc + r.slot, s->d_ovf + r.slot, nullptr, nullptr, 0);
                r.n_items = r.q.n_items;
                r.cursor = 0;
                fresh_slots.push_back(r.slot);
                s->active.push_back(r);
                s->pending.pop_front();
            }
            if (s->active.empty()) continue;
        }
        // one step over a slice of every active request (the worker owns
        // `active` outside the lock; submit only touches `pending`)
        int32_t total = 0, maxk = 4, nq = 0;
        const int32_t per_req =
            std::max<int32_t>(64, std::min<int32_t>(kItemsPerReq, kItemsPerStep / (int32_t)s->active.size()));
        std::vector<int32_t> take(s->active.size(), 0);
        for (size_t i = 0; i < s->active.size(); ++i) {
            Req& r = s->active[i];
            take[i] = std::min(per_req, r.n_items - r.cursor);
            QueryDesc q = r.q;
            q.item_begin = total;
            q.item_lo = r.cursor;
            q.n_items = take[i];
            s->h_q[nq++] = q;
            total += take[i];
            maxk = std::max(maxk, r.k);
        }
        hipError_t e = hipSuccess;
        for (int32_t slot : fresh_slots) {
            if (e == hipSuccess) e = launch_fill_u64(s->d_acc + slot, 0, 1, s->stream);
            if (e == hipSuccess) e = launch_fill_i32(s->d_ovf + slot, 0, 1, s->stream);
        }
        if (e == hipSuccess) e = launch_fill_i32(s->d_item_ctr, 0, 1, s->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(s->d_q, s->h_q, sizeof(QueryDesc) * (size_t)nq, hipMemcpyHostToDevice, s->stream);
        if (e == hipSuccess && total > 0) {
            CountLaunch cl;
            cl.queries = s->d_q;
            cl.n_queries = nq;
            cl.total_items = total;
            cl.item_ctr = s->d_item_ctr;
            cl.scratch = s->d_scratch;
            cl.scratch_words = s->scratch_words;
            cl.max_k = maxk;
            cl.blocks = blocks;
            cl.wg_waves = wg;
            cl.lds_bytes = count_lds_bytes(0, maxk, wg);
            cl.flush_rows = s->tuning.flush_rows;
            cl.stats = false;
            cl.per_arc = false;
            e = launch_count(cl, s->stream);
        }
        if (e == hipSuccess)
            e = hipMemcpyAsync(s->h_acc, s->d_acc, sizeof(unsigned long long) * (size_t)s->max_slots,
                               hipMemcpyDeviceToHost, s->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(s->h_ovf, s->d_ovf, sizeof(int32_t) * (size_t)s->max_slots, hipMemcpyDeviceToHost,
                               s->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
        std::lock_guard<std::mutex> lock(s->mu);
        std::vector<Req> still;
        for (size_t i = 0; i < s->active.size(); ++i) {
            Req& r = s->active[i];
            if (e != hipSuccess) {
                s->worker_error = hipGetErrorString(e);
                complete(s, r, 0, CITRON_EDEVICE);
            } else {
                r.cursor += take[i];
                if (r.cursor < r.n_items) {
                    still.push_back(r);
                    continue;
                }
                complete(s, r, s->h_acc[r.slot], s->h_ovf[r.slot] ? CITRON_EOVERFLOW : CITRON_OK);
            }
            s->free_slots.push_back(r.slot);
            s->used -= r.footprint;
        }
        s->active.swap(still);
        s->cv.notify_all();
    }
}

void server_free(citron_server* s)
{
    if (s->d_acc) (void)hipFree(s->d_acc);
    if (s->d_ovf) (void)hipFree(s->d_ovf);
    if (s->d_item_ctr) (void)hipFree(s->d_item_ctr);
    if (s->d_q) (void)hipFree(s->d_q);
    if (s->d_scratch) (void)hipFree(s->d_scratch);
    if (s->h_q) (void)hipHostFree(s->h_q);
    if (s->h_acc) (void)hipHostFree(s->h_acc);
    if (s->h_ovf) (void)hipHostFree(s->h_ovf);
    if (s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
}

}  // namespace

extern "C" {

citron_server* citron_server_create(int64_t hbm_budget_bytes, int32_t max_slots, const citron_tuning* t)
{
    if (hbm_budget_bytes <= 0) { fail(CITRON_EINVAL, "hbm_budget_bytes must be > 0"); return nullptr; }
    if (max_slots < 1 || max_slots > 1024) { fail(CITRON_EINVAL, "max_slots must be in 1..1024"); return nullptr; }
    citron_server* s = new (std::nothrow) citron_server();
    if (!s) { fail(CITRON_ENOMEM, "host allocation failed"); return nullptr; }
    if (resolve_tuning(t, &s->tuning)) { delete s; return nullptr; }
    s->budget = hbm_budget_bytes;
    s->max_slots = max_slots;
    hipError_t e = hipGetDevice(&s->device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
    // deepest supported k sizes the shared stack scratch
    const int32_t blocks = device_cus(s->device) * s->tuning.blocks_per_cu;
    s->scratch_words = count_scratch_words(0, CITRON_KMAX, s->tuning.wg_waves);
    if (e == hipSuccess) e = hipMalloc((void**)&s->d_acc, sizeof(unsigned long long) * (size_t)max_slots);
    if (e == hipSuccess) e = hipMalloc((void**)&s->d_ovf, sizeof(int32_t) * (size_t)max_slots);
    if (e == hipSuccess) e = hipMalloc((void**)&s->d_item_ctr, sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc((void**)&s->d_q, sizeof(QueryDesc) * (size_t)max_slots);
    if (e == hipSuccess)
        e = hipMalloc((void**)&s->d_scratch, (size_t)(s->scratch_words * 8 * blocks));
    if (e == hipSuccess) e = hipHostMalloc((void**)&s->h_q, sizeof(QueryDesc) * (size_t)max_slots, hipHostMallocDefault);
    if (e == hipSuccess)
        e = hipHostMalloc((void**)&s->h_acc, sizeof(unsigned long long) * (size_t)max_slots, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&s->h_ovf, sizeof(int32_t) * (size_t)max_slots, hipHostMallocDefault);
    if (e != hipSuccess) {
        hip_fail(e, "server set-up");
        server_free(s);
        return nullptr;
    }
    for (int32_t i = max_slots - 1; i >= 0; --i) s->free_slots.push_back(i);
    s->worker = std::thread(worker_main, s);
    return s;
}

citron_status citron_server_add_graph(citron_server* s, citron_graph* g, int32_t* graph_id)
{
    if (!s || !g || !graph_id) return fail(CITRON_EINVAL, "NULL argument");
    if (g->state != 1) return fail(CITRON_ESTATE, "graphs must be ordered before they are served");
    if (g->device != s->device) return fail(CITRON_EINVAL, "graph and server live on different devices");
    {
        std::lock_guard<std::mutex> gl(g->mu);
        if (g->max_outdeg >= 3) {   // rows are needed only when some k >= 4 can be nonzero
            citron_status st = ensure_rows(g);
            if (st) return st;
        }
    }
    std::lock_guard<std::mutex> lock(s->mu);
    s->graphs.push_back(g);
    *graph_id = (int32_t)s->graphs.size() - 1;
    return CITRON_OK;
}

citron_status citron_server_submit(citron_server* s, int32_t graph_id, int32_t k, uint64_t tag)
{
    if (!s) return fail(CITRON_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lock(s->mu);
    if (graph_id < 0 || graph_id >= (int32_t)s->graphs.size()) return fail(CITRON_EINVAL, "unknown graph_id");
    Req r;
    r.tag = tag;
    r.gid = graph_id;
    r.k = k;
    r.t_submit = now_ns();
    s->pending.push_back(r);
    ++s->submitted;
    s->cv.notify_all();
    return CITRON_OK;
}

int32_t citron_server_poll(citron_server* s, citron_result* results, int32_t max)
{
    if (!s || !results || max <= 0) return 0;
    std::lock_guard<std::mutex> lock(s->mu);
    int32_t n = 0;
    while (n < max && !s->done.empty()) {
        results[n++] = s->done.front();
        s->done.pop_front();
    }
    s->returned += n;
    return n;
}

int32_t citron_server_pending(citron_server* s)
{
    if (!s) return 0;
    std::lock_guard<std::mutex> lock(s->mu);
    return (int32_t)(s->submitted - s->returned);
}

void citron_server_destroy(citron_server* s)
{
    if (!s) return;
    {
        std::lock_guard<std::mutex> lock(s->mu);
        s->stop = true;
        s->cv.notify_all();
    }
    if (s->worker.joinable()) s->worker.join();
    (void)hipStreamSynchronize(s->stream);
    server_free(s);
}

}  // extern "C"
