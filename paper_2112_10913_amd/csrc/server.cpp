// Request server over resident graphs with continuous batching.
//
// A server owns one worker thread on the device that was current when it
// was created.  Requests (graph, k) are queued by citron_server_submit and
// admitted in arrival order as soon as an in-flight slot is free and their
// device footprint fits the memory budget.  The worker issues steps: each
// step is one launch of the persistent count kernel over work items of
// several admitted requests, so requests that arrive while others run join
// the next step and share the device with them.  Two lanes keep small
// requests from waiting behind large ones:
//   - fast lane (one stream): requests with at most kFastItems items, whole;
//   - heavy lane (two streams): one larger request per step, the requests
//     taken in turn, a slice of its items sized to run about kHeavyStepTargetMs
//     (each request's slice is rescaled from the measured time of its last
//     step), so that a step works on one graph (its rows stay in cache) and
//     a step's persistent grid frees the compute units again within tens
//     of milliseconds for requests that arrive meanwhile; two such steps run
//     at once, and while one drains its last items the other takes the
//     freed compute units.
// Steps of a lane retire in issue order; a request whose items have all
// retired returns its count and frees its slot.  Counts are exact integers,
// so a request's count does not depend on which requests it shares steps
// with.
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
    int64_t id = 0;
    bool fast = false;        // fast lane: issued whole in one step
    int32_t gid = 0;
    int32_t k = 0;
    int64_t t_submit = 0;
    int64_t t_admit = 0;
    int32_t slot = -1;
    int32_t n_items = 0;
    int32_t issued = 0;       // items handed to steps
    int32_t slice = 0;        // heavy lane: items of its next step
    int32_t retired = 0;      // items of retired steps
    bool failed = false;      // a step with its items failed: issue no more
    int64_t footprint = 0;
    QueryDesc q;
};

// Lanes: a request with at most kFastItems items goes whole into one fast
// step (at most kFastStepItems items); larger ones are sliced into heavy
// steps, each step one request's slice: kHeavyFirstSlice items first, then
// rescaled toward kHeavyStepTargetMs per step within [kHeavyMinSlice,
// kHeavyMaxSlice] (its items come largest first, so later slices grow).
constexpr int32_t kFastItems = 4096;
constexpr int32_t kFastStepItems = 65536;
constexpr int32_t kHeavyFirstSlice = 4096;
constexpr int32_t kHeavyMinSlice = 1024;
constexpr int32_t kHeavyMaxSlice = 1 << 22;
constexpr float kHeavyStepTargetMs = 25.0f;
constexpr int kInflight = 3;              // step 0: fast lane; 1, 2: heavy lane

// One step's launch resources (reused once the step has retired).
struct Step {
    hipStream_t stream = nullptr;
    hipEvent_t start = nullptr;          // timing of heavy steps
    hipEvent_t done = nullptr;
    QueryDesc* d_q = nullptr;            // max_slots descriptors
    QueryDesc* h_q = nullptr;            // pinned staging of the same
    int32_t* d_item_ctr = nullptr;
    unsigned long long* d_scratch = nullptr;
    std::vector<std::pair<int64_t, int32_t>> parts;   // (request id, items)
    hipError_t err = hipSuccess;
};

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

    // device: per slot accumulator and flag; the steps' launch resources
    unsigned long long* d_acc = nullptr;
    int32_t* d_ovf = nullptr;
    int64_t scratch_words = 0;
    Step steps[kInflight];
    hipStream_t ctl = nullptr;            // slot resets and result reads
    // pinned host mirrors of the slot results
    unsigned long long* h_acc = nullptr;
    int32_t* h_ovf = nullptr;
    int64_t next_id = 0;
    int64_t rr_last = -1;                 // heavy lane: request of the last heavy step
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
    b += count_deep_scratch_words(k, s->tuning.wg_waves) * 8 * blocks;
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

// Launch one step of a lane.  Fast: every fast request not yet issued,
// whole, up to kFastStepItems items.  Heavy: the next slice of the first
// heavy request (admission order) with items left.  Returns false when the
// lane has nothing to issue.
bool issue_step(citron_server* s, Step& st, bool fast, int wg, int32_t blocks)
{
    int32_t with_work = 0;
    for (const Req& r : s->active)
        if (r.fast == fast && !r.failed && r.issued < r.n_items) ++with_work;
    if (with_work == 0) return false;
    const int32_t cap = fast ? kFastStepItems : kHeavyMaxSlice;
    int32_t total = 0, maxk = 4, nq = 0;
    st.parts.clear();
    // fast lane: admission order; heavy lane: round robin over the heavy
    // requests with items left, from the one after the last served, so that
    // a request needing a few steps is not held behind a long one
    const size_t na = s->active.size();
    size_t first = 0;
    if (!fast && na > 0) {
        size_t best = na;
        for (size_t j = 0; j < na; ++j) {
            const Req& r = s->active[j];
            if (r.fast || r.failed || r.issued >= r.n_items) continue;
            if (best == na) best = j;                         // wrap-around choice
            if (r.id > s->rr_last) { best = j; break; }       // next after the last served
        }
        first = best == na ? 0 : best;
    }
    for (size_t jj = first; jj < na; ++jj) {
        Req& r = s->active[jj];
        if (r.fast != fast || r.failed || r.issued >= r.n_items) continue;
        if (total >= cap) break;
        int32_t take = r.n_items - r.issued;
        if (fast && total + take > cap && total > 0) break;
        if (!fast) {
            if (r.slice <= 0) r.slice = kHeavyFirstSlice;
            take = std::min(take, r.slice);
        }
        QueryDesc q = r.q;
        q.item_begin = total;
        q.item_lo = r.issued;
        q.n_items = take;
        st.h_q[nq++] = q;
        st.parts.emplace_back(r.id, take);
        r.issued += take;
        total += take;
        maxk = std::max(maxk, r.k);
        if (!fast) {                 // one request per heavy step
            s->rr_last = r.id;
            break;
        }
    }
    hipError_t e = hipEventRecord(st.start, st.stream);
    if (e == hipSuccess) e = launch_fill_i32(st.d_item_ctr, 0, 1, st.stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(st.d_q, st.h_q, sizeof(QueryDesc) * (size_t)nq, hipMemcpyHostToDevice, st.stream);
    if (e == hipSuccess) {
        CountLaunch cl;
        cl.queries = st.d_q;
        cl.n_queries = nq;
        cl.total_items = total;
        cl.item_ctr = st.d_item_ctr;
        cl.scratch = st.d_scratch;
        cl.scratch_words = s->scratch_words;
        cl.max_k = maxk;
        cl.blocks = blocks;
        cl.wg_waves = wg;
        cl.lds_bytes = count_lds_bytes(arc_max_for(s->tuning, maxk), maxk, wg, false);
        cl.flush_rows = s->tuning.flush_rows;
        cl.arc_lds_max = arc_max_for(s->tuning, maxk);
        cl.stats = false;
        cl.per_arc = false;
        e = launch_count(cl, st.stream);
    }
    if (e == hipSuccess) e = hipEventRecord(st.done, st.stream);
    st.err = e;
    return true;
}

// Retire a step: credit its items to their requests.  A failed step marks
// its requests failed; they finish once every step holding their items has
// retired, so that no step still adds into a slot that is handed on.
void retire_step(citron_server* s, Step& st, bool fast)
{
    hipError_t e = st.err;
    if (e == hipSuccess) e = hipEventSynchronize(st.done);
    float ms = 0.0f;
    if (e == hipSuccess && !fast && hipEventElapsedTime(&ms, st.start, st.done) != hipSuccess) ms = 0.0f;
    for (const auto& pr : st.parts)
        for (Req& r : s->active)
            if (r.id == pr.first) {
                r.retired += pr.second;
                if (e != hipSuccess) r.failed = true;
                if (!fast && ms > 0.0f && pr.second >= r.slice) {
                    // next slice of this request toward the step target
                    const double scaled = (double)r.slice * kHeavyStepTargetMs / ms;
                    r.slice = (int32_t)std::min<double>(kHeavyMaxSlice,
                                                        std::max<double>(kHeavyMinSlice, scaled));
                }
            }
    if (e != hipSuccess) s->worker_error = hipGetErrorString(e);
    st.parts.clear();
}

void worker_main(citron_server* s)
{
    (void)hipSetDevice(s->device);
    const int wg = s->tuning.wg_waves;
    const int32_t blocks = device_cus(s->device) * s->tuning.blocks_per_cu;
    bool fast_busy = false;                   // step 0
    std::deque<int> heavy_inflight;           // steps 1, 2 in issue order
    std::vector<int> heavy_free = {2, 1};
    for (;;) {
        std::vector<int32_t> fresh_slots;
        {
            std::unique_lock<std::mutex> lock(s->mu);
            s->cv.wait(lock, [&] {
                return s->stop || !s->pending.empty() || !s->active.empty() || fast_busy ||
                       !heavy_inflight.empty();
            });
            if (s->stop) break;
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
                r.id = s->next_id++;
                r.q = make_query(g, r.k, s->d_acc + r.slot, s->d_ovf + r.slot, nullptr, nullptr, 0);
                r.n_items = r.q.n_items;
                r.fast = r.n_items <= kFastItems;
                r.issued = 0;
                r.retired = 0;
                fresh_slots.push_back(r.slot);
                s->active.push_back(r);
                s->pending.pop_front();
            }
            s->cv.notify_all();
        }
        // the worker owns `active` and the steps outside the lock; submit
        // only touches `pending`
        if (!fresh_slots.empty()) {
            // zero the new slots before any step can touch them
            hipError_t e = hipSuccess;
            for (int32_t slot : fresh_slots) {
                if (e == hipSuccess) e = launch_fill_u64(s->d_acc + slot, 0, 1, s->ctl);
                if (e == hipSuccess) e = launch_fill_i32(s->d_ovf + slot, 0, 1, s->ctl);
            }
            if (e == hipSuccess) e = hipStreamSynchronize(s->ctl);
            if (e != hipSuccess) s->worker_error = hipGetErrorString(e);
        }
        // issue what the lanes can take
        if (!fast_busy && issue_step(s, s->steps[0], true, wg, blocks)) fast_busy = true;
        while (!heavy_free.empty() && issue_step(s, s->steps[heavy_free.back()], false, wg, blocks)) {
            heavy_inflight.push_back(heavy_free.back());
            heavy_free.pop_back();
        }
        // retire finished steps; wait (polling, so that arrivals are admitted
        // meanwhile) only when nothing finished and nothing else can be done
        bool retired = false;
        for (;;) {
            if (fast_busy && (s->steps[0].err != hipSuccess || hipEventQuery(s->steps[0].done) != hipErrorNotReady)) {
                retire_step(s, s->steps[0], true);
                fast_busy = false;
                retired = true;
            }
            while (!heavy_inflight.empty()) {
                Step& st = s->steps[heavy_inflight.front()];
                if (st.err == hipSuccess && hipEventQuery(st.done) == hipErrorNotReady) break;
                retire_step(s, st, false);
                heavy_free.push_back(heavy_inflight.front());
                heavy_inflight.pop_front();
                retired = true;
            }
            if (retired || (!fast_busy && heavy_inflight.empty())) break;
            {
                std::lock_guard<std::mutex> lock(s->mu);
                if (s->stop) break;
                if (!s->pending.empty() && !s->free_slots.empty() &&
                    s->used + footprint_of(s, s->pending.front().k) <= s->budget)
                    break;   // admit, then issue
            }
            std::this_thread::sleep_for(std::chrono::microseconds(50));
        }
        // requests whose items have all retired
        std::vector<Req> still;
        std::vector<Req> fin;
        for (Req& r : s->active) {
            if (r.retired == r.n_items || (r.failed && r.retired == r.issued)) fin.push_back(r);
            else still.push_back(r);
        }
        hipError_t e = hipSuccess;
        for (const Req& r : fin) {
            if (r.failed) continue;
            if (e == hipSuccess)
                e = hipMemcpyAsync(s->h_acc + r.slot, s->d_acc + r.slot, sizeof(unsigned long long),
                                   hipMemcpyDeviceToHost, s->ctl);
            if (e == hipSuccess)
                e = hipMemcpyAsync(s->h_ovf + r.slot, s->d_ovf + r.slot, sizeof(int32_t), hipMemcpyDeviceToHost,
                                   s->ctl);
        }
        if (!fin.empty() && e == hipSuccess) e = hipStreamSynchronize(s->ctl);
        if (e != hipSuccess) s->worker_error = hipGetErrorString(e);
        std::lock_guard<std::mutex> lock(s->mu);
        for (Req& r : fin) {
            if (r.failed || e != hipSuccess) complete(s, r, 0, CITRON_EDEVICE);
            else complete(s, r, s->h_acc[r.slot], s->h_ovf[r.slot] ? CITRON_EOVERFLOW : CITRON_OK);
            s->free_slots.push_back(r.slot);
            s->used -= r.footprint;
        }
        s->active.swap(still);
        s->cv.notify_all();
    }
    // stop: let the steps in flight finish before their buffers are freed
    if (fast_busy) (void)hipEventSynchronize(s->steps[0].done);
    for (int si : heavy_inflight) (void)hipEventSynchronize(s->steps[si].done);
}

void server_free(citron_server* s)
{
    for (Step& st : s->steps) {
        if (st.stream) (void)hipStreamSynchronize(st.stream);
        if (st.d_q) (void)hipFree(st.d_q);
        if (st.h_q) (void)hipHostFree(st.h_q);
        if (st.d_item_ctr) (void)hipFree(st.d_item_ctr);
        if (st.d_scratch) (void)hipFree(st.d_scratch);
        if (st.done) (void)hipEventDestroy(st.done);
        if (st.start) (void)hipEventDestroy(st.start);
        if (st.stream) (void)hipStreamDestroy(st.stream);
    }
    if (s->d_acc) (void)hipFree(s->d_acc);
    if (s->d_ovf) (void)hipFree(s->d_ovf);
    if (s->h_acc) (void)hipHostFree(s->h_acc);
    if (s->h_ovf) (void)hipHostFree(s->h_ovf);
    if (s->ctl) (void)hipStreamDestroy(s->ctl);
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
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->ctl, hipStreamNonBlocking);
    // deepest supported k sizes the stack scratch of each step
    const int32_t blocks = device_cus(s->device) * s->tuning.blocks_per_cu;
    s->scratch_words = count_scratch_words(0, CITRON_KMAX, s->tuning.wg_waves);
    if (e == hipSuccess) e = hipMalloc((void**)&s->d_acc, sizeof(unsigned long long) * (size_t)max_slots);
    if (e == hipSuccess) e = hipMalloc((void**)&s->d_ovf, sizeof(int32_t) * (size_t)max_slots);
    if (e == hipSuccess)
        e = hipHostMalloc((void**)&s->h_acc, sizeof(unsigned long long) * (size_t)max_slots, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&s->h_ovf, sizeof(int32_t) * (size_t)max_slots, hipHostMallocDefault);
    for (Step& st : s->steps) {
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&st.stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreate(&st.start);
        if (e == hipSuccess) e = hipEventCreate(&st.done);
        if (e == hipSuccess) e = hipMalloc((void**)&st.d_q, sizeof(QueryDesc) * (size_t)max_slots);
        if (e == hipSuccess)
            e = hipHostMalloc((void**)&st.h_q, sizeof(QueryDesc) * (size_t)max_slots, hipHostMallocDefault);
        if (e == hipSuccess) e = hipMalloc((void**)&st.d_item_ctr, sizeof(int32_t));
        if (e == hipSuccess) e = hipMalloc((void**)&st.d_scratch, (size_t)(s->scratch_words * 8 * blocks));
    }
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
        // the rows (and with them the triangle count that answers k = 3) are
        // needed whenever some k >= 3 can be nonzero: a vertex with two
        // out-neighbours roots a possible triangle
        if (g->max_outdeg >= 2) {
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
    server_free(s);
}

}  // extern "C"
