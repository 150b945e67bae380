// wrs_serve.hip -- a request loop on one device (the wrs_serve_* C ABI).
//
// Build requests create resident alias tables; sample requests draw from them.
// A scheduler thread admits requests in arrival order while they fit an HBM
// budget (one device pool carved by a first-fit allocator, so no hipMalloc on
// the request path; each slot's descriptor buffers, device and pinned host, are
// reserved at creation), packs admitted requests into batched launches (all builds
// of a tick share one launch per phase, all samples share one sampler launch),
// and keeps up to `inflight` such batches running on separate streams while it
// forms the next (continuous batching).  With one_at_a_time = 1 the same loop
// issues one request per launch, strictly in arrival order, as the baseline.
//
// Ordering with the caller: a request submitted with the caller's stream
// records an event on that stream at submission, and its batch waits for the
// event on the device before it reads the request's inputs or writes its
// outputs.  Host weights are copied at submission into a pinned staging arena
// (the caller's buffer is free again when the call returns) and from there
// into pool memory on the batch's stream.
#include <stdio.h>
#include <stddef.h>
#include <string.h>
#include <sys/prctl.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "wrs_internal.h"
#include "wrs_pool.h"

namespace wrs {

static double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// The HBM budget: one device allocation carved by the first-fit allocator.
class Pool {
   public:
    bool init(size_t bytes) {
        bytes = (bytes + 255) & ~(size_t)255;
        void* base = nullptr;
        if (hipMalloc(&base, bytes) != hipSuccess) return false;
        ff_.reset(base, bytes);
        return true;
    }
    ~Pool() {
        if (ff_.base()) (void)hipFree(ff_.base());
    }
    void* alloc(size_t bytes) { return ff_.alloc(bytes); }
    void release(void* p, size_t bytes) { ff_.release(p, bytes); }
    size_t used() const { return ff_.used(); }
    size_t peak() const { return ff_.peak(); }
    size_t size() const { return ff_.size(); }

   private:
    FirstFit ff_;
};

enum { OP_BUILD = 1, OP_SAMPLE = 2 };
enum TableState { T_QUEUED, T_BUILDING, T_READY, T_FAILED };

struct Table {
    uint64_t id;
    int64_t n;
    const float* d_w;
    wrs_entry* d_table = nullptr;
    size_t table_bytes = 0;
    TableState state = T_QUEUED;
    hipEvent_t ready = nullptr;  // while it builds: the event of its batch (not owned)
    int refs = 0;                // queued or running requests using the table
    int status = WRS_OK;
    BuildScalars* sc = nullptr;  // status word of the build (pool memory)
    bool idle = false;           // in the server's idle list
    std::list<Table*>::iterator idle_at;
};

struct Request {
    uint64_t id;
    int op;
    uint64_t table_id;
    int64_t k = 0;
    uint64_t seed = 0;
    int32_t* d_out = nullptr;
    hipEvent_t after = nullptr;  // recorded on the caller's stream at submission
    float* h_stage = nullptr;    // build from host weights: their copy in the staging arena
    size_t stage_bytes = 0;
    double t_submit = 0, t_done = 0;
    int status = WRS_OK;
    bool done = false;
    int build_index = -1;  // position among the builds of its batch
};

struct Batch {
    int slot;
    bool ok = true;  // false: a launch or copy of the batch failed (all its requests fail)
    hipEvent_t ev = nullptr;
    std::vector<Request*> reqs;
    std::vector<std::pair<void*, size_t>> scratch;  // pool memory to give back
    const int32_t* h_status = nullptr;  // build statuses, copied to the slot's pinned buffer by the batch
};

struct Server {
    wrs_serve_config cfg;
    int device = 0;
    Pool pool;
    char* h_arena = nullptr;     // pinned staging for host weights (cfg.host_stage_bytes)
    FirstFit stage;
    std::vector<hipEvent_t> free_events;  // recycled events (submissions, batches, tables)
    std::mutex mu;
    std::condition_variable cv, cv_done;
    std::deque<Request*> queue;
    std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
    std::unordered_map<uint64_t, std::unique_ptr<Table>> tables;
    // Tables that may be evicted (built or failed, no request pending), least
    // recently used first: an eviction takes the front, with no scan.
    std::list<Table*> idle;
    std::vector<hipStream_t> streams;
    std::vector<char*> staging;   // pinned host buffers for descriptors, one per slot
    std::vector<char*> dev_desc;  // device descriptor buffers (pool memory), one per slot
    std::vector<bool> slot_busy;
    int maxb = 1;         // requests per batch
    size_t reserved = 0;  // pool bytes of the slots' descriptor buffers
    std::deque<Batch> running;
    std::thread worker;
    bool stop = false;
    std::atomic<uint64_t> arrivals{0};  // submissions, readable without the lock
    uint64_t next_id = 1;
    // statistics
    uint64_t submitted = 0, completed = 0, failed = 0, builds = 0, samples = 0, items = 0, drawn = 0, launches = 0;
    double t_first = -1, t_last = 0;
    std::vector<double> lat_us;
};

static size_t descriptor_bytes(int njobs) {
    size_t o = 0;
    o = (o + sizeof(JobDesc) * njobs + 255) & ~(size_t)255;
    o = (o + sizeof(int64_t) * PH_COUNT * (njobs + 1) + 255) & ~(size_t)255;
    return o;
}

static size_t status_bytes(int njobs) { return ((size_t)sizeof(int32_t) * njobs + 255) & ~(size_t)255; }

// Descriptor bytes one slot needs for a batch of up to `maxb` requests: the
// build and sample job tables (nb + ns <= maxb) and the build statuses.
static size_t slot_bytes(int maxb) { return 2 * descriptor_bytes(maxb) + status_bytes(maxb); }

// Idle-list membership follows the table's state (lock held): in the list
// exactly when its build is over and no request uses it.
static void idle_update(Server& S, Table* t) {
    const bool want = t->refs == 0 && (t->state == T_READY || t->state == T_FAILED);
    if (want && !t->idle) {
        t->idle_at = S.idle.insert(S.idle.end(), t);
        t->idle = true;
    } else if (!want && t->idle) {
        S.idle.erase(t->idle_at);
        t->idle = false;
    }
}

// An event from the recycled ones, or a new one (lock held).
static hipError_t take_event(Server& S, hipEvent_t* e) {
    if (!S.free_events.empty()) {
        *e = S.free_events.back();
        S.free_events.pop_back();
        return hipSuccess;
    }
    return hipEventCreateWithFlags(e, hipEventDisableTiming);
}

// A request is finished once its batch has run, or when it fails before it
// is issued: the event it waited for, and the host copy of its weights, are
// free again.
static void finish_request(Server& S, Request* r, int status, double t) {
    if (r->after) S.free_events.push_back(r->after);
    r->after = nullptr;
    S.stage.release(r->h_stage, r->stage_bytes);
    r->h_stage = nullptr;
    r->status = status;
    r->done = true;
    r->t_done = t;
    S.completed++;
    if (status != WRS_OK) S.failed++;
    S.lat_us.push_back((t - r->t_submit) * 1e6);
    S.t_last = std::max(S.t_last, t);
    auto it = S.tables.find(r->table_id);
    if (it != S.tables.end()) {
        it->second->refs--;
        idle_update(S, it->second.get());
    }
    S.cv_done.notify_all();
}

// Retire finished batches (called with the lock held).
static void retire(Server& S, bool block) {
    while (!S.running.empty()) {
        Batch& b = S.running.front();
        // no event: it could not be created and the stream was synchronised
        hipError_t q = !b.ev ? hipSuccess : block ? hipEventSynchronize(b.ev) : hipEventQuery(b.ev);
        if (q == hipErrorNotReady) break;
        const double t = now_s();
        // read build statuses from the device for the tables built in this batch
        for (Request* r : b.reqs) {
            auto it = S.tables.find(r->table_id);
            Table* tb = (it != S.tables.end()) ? it->second.get() : nullptr;
            int st = (q == hipSuccess && b.ok) ? WRS_OK : WRS_EDEVICE;
            if (r->op == OP_BUILD && tb) {
                if (st == WRS_OK) st = b.h_status ? b.h_status[r->build_index] : WRS_EDEVICE;
                tb->state = (st == WRS_OK) ? T_READY : T_FAILED;
                tb->status = st;
                tb->ready = nullptr;  // the batch's event is recycled below
            }
            if (r->op == OP_SAMPLE && tb && tb->status != WRS_OK) st = tb->status;
            finish_request(S, r, st, t);
        }
        for (auto& p : b.scratch) S.pool.release(p.first, p.second);
        if (b.ev) S.free_events.push_back(b.ev);  // complete: reused by a later batch
        S.slot_busy[b.slot] = false;
        S.running.pop_front();
        S.cv_done.notify_all();
    }
}

// Drop the least recently used idle table (lock held); false if none is idle.
static bool evict_lru(Server& S) {
    if (S.idle.empty()) return false;
    Table* victim = S.idle.front();
    S.idle.pop_front();
    victim->idle = false;
    S.pool.release(victim->d_table, victim->table_bytes);
    S.pool.release(victim->sc, 256);
    S.tables.erase(victim->id);
    return true;
}

// Drop least recently used idle tables until `need` bytes fit (lock held).
static bool make_room(Server& S, size_t need) {
    while (S.pool.used() + need > S.cfg.hbm_budget_bytes)
        if (!evict_lru(S)) return false;
    return true;
}

// Form and launch one batch on a free slot (lock held).  Returns false if
// nothing could be issued.
static bool issue(Server& S) {
    int slot = -1;
    for (int i = 0; i < (int)S.slot_busy.size(); ++i)
        if (!S.slot_busy[i]) { slot = i; break; }
    if (slot < 0 || S.queue.empty()) return false;
    const int maxb = S.maxb;
    std::vector<Request*> take;
    std::vector<Request*> bld, smp;
    std::vector<std::pair<void*, size_t>> scratch;
    while (!S.queue.empty() && (int)take.size() < maxb) {
        Request* r = S.queue.front();
        Table* tb = S.tables[r->table_id].get();
        if (r->op == OP_BUILD) {
            // a build from host weights also holds their device copy until it retires
            const size_t wsb = build_ws_bytes(tb->n) + 256 + (r->h_stage ? r->stage_bytes : 0);
            const size_t need = tb->table_bytes + wsb + 256;
            void* ws = nullptr;
            bool placed = make_room(S, need);
            if (placed) {
                tb->d_table = (wrs_entry*)S.pool.alloc(tb->table_bytes);
                ws = S.pool.alloc(wsb);
                tb->sc = (BuildScalars*)S.pool.alloc(256);
                if (!tb->d_table || !ws || !tb->sc) {  // fragmentation: undo
                    S.pool.release(tb->d_table, tb->table_bytes);
                    S.pool.release(ws, wsb);
                    S.pool.release(tb->sc, 256);
                    tb->d_table = nullptr;
                    tb->sc = nullptr;
                    placed = false;
                }
            }
            if (!placed) {
                if (evict_lru(S)) continue;  // fragmented: free one more idle table, try again
                if (take.empty() && S.running.empty()) {
                    // Nothing runs and nothing idle can go: the budget is held by
                    // tables that requests queued behind this one still need, so
                    // waiting would never end.
                    set_error("wrs_serve: build of %lld items does not fit beside the tables pending requests hold",
                              (long long)tb->n);
                    tb->state = T_FAILED;
                    tb->status = WRS_ENOMEM;
                    S.queue.pop_front();
                    finish_request(S, r, WRS_ENOMEM, now_s());
                    continue;
                }
                break;  // wait for running batches to retire (FIFO: no overtaking)
            }
            scratch.push_back({ws, wsb});
            tb->state = T_BUILDING;
            bld.push_back(r);
        } else {
            if (tb->state == T_FAILED) {
                S.queue.pop_front();
                finish_request(S, r, tb->status, now_s());
                continue;
            }
            smp.push_back(r);
        }
        take.push_back(r);
        S.queue.pop_front();
    }
    if (take.empty()) return false;
    hipStream_t st = S.streams[slot];
    // nothing of the batch touches a request's inputs or outputs before the
    // work the caller queued on its stream ahead of the submission has run
    for (Request* r : take)
        if (r->after) (void)hipStreamWaitEvent(st, r->after, 0);
    // descriptors: builds first, then samples, each its own job table
    const int nb = (int)bld.size(), ns = (int)smp.size();
    // bb + sb + status_bytes(nb) <= slot_bytes(max batch): the slot's buffers hold it
    const size_t bb = nb ? descriptor_bytes(nb) : 0, sb = ns ? descriptor_bytes(ns) : 0;
    char* dev_desc = S.dev_desc[slot];
    bool ok = true;
    // samples wait for tables built by batches still running on other streams
    for (Request* r : smp) {
        Table* tb = S.tables[r->table_id].get();
        bool same = false;
        for (Request* q : bld) same |= (q->table_id == r->table_id);
        if (!same && tb->ready && tb->state == T_BUILDING) (void)hipStreamWaitEvent(st, tb->ready, 0);
    }
    if (ok && nb) {
        std::vector<JobDesc> d(nb);
        std::vector<int64_t> off((size_t)PH_COUNT * (nb + 1), 0);
        size_t wsi = 0;
        for (int j = 0; j < nb; ++j) {
            Table* tb = S.tables[bld[j]->table_id].get();
            memset(&d[j], 0, sizeof(JobDesc));
            char* wsp = (char*)scratch[wsi++].first;
            d[j].w = tb->d_w;
            if (bld[j]->h_stage) {
                // host weights: copied behind the workspace, then built from there
                float* dw = (float*)(wsp + ((build_ws_bytes(tb->n) + 255) & ~(size_t)255));
                ok = ok && hipMemcpyAsync(dw, bld[j]->h_stage, bld[j]->stage_bytes, hipMemcpyHostToDevice, st) ==
                               hipSuccess;
                d[j].w = dw;
            }
            d[j].table = tb->d_table;
            set_sample_job(d[j], 0, 1);
            build_ws_layout(d[j], wsp, tb->n);
            d[j].sc = tb->sc;
            int64_t b[PH_COUNT];
            phase_blocks(d[j], b);
            for (int p = 0; p < PH_COUNT; ++p) off[(size_t)p * (nb + 1) + j + 1] = off[(size_t)p * (nb + 1) + j] + b[p];
        }
        JobTable jt;
        memset(&jt, 0, sizeof jt);
        if (nb == 1) {
            // one build: its descriptor travels as the launches' argument, with
            // no copy ahead of them
            jt.one = d[0];
        } else {
            char* h = S.staging[slot];
            const size_t o_off = (sizeof(JobDesc) * nb + 255) & ~(size_t)255;
            memcpy(h, d.data(), sizeof(JobDesc) * nb);
            memcpy(h + o_off, off.data(), sizeof(int64_t) * off.size());
            ok = ok && hipMemcpyAsync(dev_desc, h, bb, hipMemcpyHostToDevice, st) == hipSuccess;
            jt.jobs = (const JobDesc*)dev_desc;
            jt.off = (const int64_t*)(dev_desc + o_off);
            jt.njobs = nb;
        }
        int64_t totals[PH_COUNT];
        for (int p = 0; p < PH_COUNT; ++p) totals[p] = off[(size_t)p * (nb + 1) + nb];
        ok = ok && launch_build(jt, totals, st) == hipSuccess;
        S.launches++;
        for (int j = 0; j < nb; ++j) bld[j]->build_index = j;
        // statuses for retire(): gathered on the device, one copy to the pinned buffer
        int32_t* d_st = (int32_t*)(dev_desc + bb + sb);
        int32_t* h_st = (int32_t*)(S.staging[slot] + bb + sb);
        if (nb == 1) {  // the status word is the first field of the job's scalars
            const char* d_sc = (const char*)d[0].sc + offsetof(BuildScalars, status);
            ok = ok && hipMemcpyAsync(h_st, d_sc, sizeof(int32_t), hipMemcpyDeviceToHost, st) == hipSuccess;
        } else {
            ok = ok && launch_collect_status(jt, d_st, st) == hipSuccess;
            ok = ok && hipMemcpyAsync(h_st, d_st, sizeof(int32_t) * nb, hipMemcpyDeviceToHost, st) == hipSuccess;
        }
    }
    if (ok && ns) {
        std::vector<JobDesc> d(ns);
        std::vector<int64_t> off((size_t)PH_COUNT * (ns + 1), 0);
        for (int j = 0; j < ns; ++j) {
            Table* tb = S.tables[smp[j]->table_id].get();
            memset(&d[j], 0, sizeof(JobDesc));
            d[j].table = tb->d_table;
            d[j].n = tb->n;
            set_sample_job(d[j], smp[j]->k);
            d[j].seed = smp[j]->seed;
            d[j].stream_id = 0;
            d[j].out = smp[j]->d_out;
            d[j].sc = tb->sc;  // skips the draws if the build failed
            off[(size_t)PH_SAMPLE * (ns + 1) + j + 1] = off[(size_t)PH_SAMPLE * (ns + 1) + j] + sample_blocks(d[j]);
        }
        JobTable jt;
        memset(&jt, 0, sizeof jt);
        if (ns == 1) {
            jt.one = d[0];  // one sample request: the descriptor is the launch's argument
        } else {
            char* h = S.staging[slot] + bb;
            const size_t o_off = (sizeof(JobDesc) * ns + 255) & ~(size_t)255;
            memcpy(h, d.data(), sizeof(JobDesc) * ns);
            memcpy(h + o_off, off.data(), sizeof(int64_t) * off.size());
            ok = ok && hipMemcpyAsync(dev_desc + bb, h, sb, hipMemcpyHostToDevice, st) == hipSuccess;
            jt.jobs = (const JobDesc*)(dev_desc + bb);
            jt.off = (const int64_t*)(dev_desc + bb + o_off);
            jt.njobs = ns;
        }
        ok = ok && launch_sample(jt, off[(size_t)PH_SAMPLE * (ns + 1) + ns], st) == hipSuccess;
        S.launches++;
    }
    Batch b;
    b.slot = slot;
    b.reqs = take;
    b.scratch = scratch;
    b.h_status = (ok && nb) ? (const int32_t*)(S.staging[slot] + bb + sb) : nullptr;
    if (take_event(S, &b.ev) != hipSuccess) {
        b.ev = nullptr;
        ok = false;
    } else if (hipEventRecord(b.ev, st) != hipSuccess) {
        ok = false;
    }
    // A sample issued later, in another batch, of a table this batch builds
    // waits for this event (recorded after all of the batch's launches, one
    // event per batch instead of one per build).
    for (Request* r : bld) S.tables[r->table_id]->ready = b.ev;
    b.ok = ok;
    if (!ok) {
        // retire() fails every request of the batch; wait so that its slot
        // buffers are free again when the slot is
        set_error("wrs_serve: batch launch failed");
        (void)hipStreamSynchronize(st);
    }
    S.slot_busy[slot] = true;
    S.running.push_back(b);
    return true;
}

static void worker_main(Server* S) {
    (void)hipSetDevice(S->device);
    // The completion poll below sleeps 5 us at a time; with the default 50 us
    // timer slack of a thread each of those sleeps would last about 55 us.
    (void)prctl(PR_SET_TIMERSLACK, 1UL, 0UL, 0UL, 0UL);
    std::unique_lock<std::mutex> lk(S->mu);
    while (true) {
        retire(*S, false);
        bool issued = false;
        while (issue(*S)) issued = true;
        if (S->stop && S->queue.empty() && S->running.empty()) break;
        if (!issued) {
            if (S->running.empty()) {
                // Idle: watch for a submission for up to 200 us before sleeping
                // on the condition variable, so that a request arriving soon is
                // issued without the wake-up of a sleeping thread.
                const uint64_t seen = S->arrivals.load(std::memory_order_acquire);
                lk.unlock();
                bool arrived = false;
                for (const double t0 = now_s(); !arrived && now_s() - t0 < 200e-6;)
                    arrived = S->arrivals.load(std::memory_order_acquire) != seen;
                lk.lock();
                if (!arrived && S->queue.empty() && !S->stop) S->cv.wait_for(lk, std::chrono::milliseconds(50));
            } else {
                // poll the oldest batch; short sleeps keep the completion times sharp
                lk.unlock();
                std::this_thread::sleep_for(std::chrono::microseconds(5));
                lk.lock();
            }
        }
    }
}

}  // namespace wrs

using namespace wrs;

// Streams and pinned buffers of a server (its pool frees itself).
static void release_slots(Server* S) {
    for (auto st : S->streams) (void)hipStreamDestroy(st);
    for (auto p : S->staging)
        if (p) (void)hipHostFree(p);
    S->streams.clear();
    S->staging.clear();
    for (auto e : S->free_events) (void)hipEventDestroy(e);
    S->free_events.clear();
    if (S->h_arena) (void)hipHostFree(S->h_arena);
    S->h_arena = nullptr;
}

// An event recorded on the caller's stream now (lock held); nullptr and
// WRS_OK for WRS_SERVE_UNORDERED.  NULL is the legacy default stream: the
// stream of a framework that has not set one, so it gets an event like any
// other.
static int submission_event(Server& S, void* stream, hipEvent_t* out) {
    *out = nullptr;
    if (stream == WRS_SERVE_UNORDERED) return WRS_OK;
    hipEvent_t e = nullptr;
    if (!S.free_events.empty()) {
        e = S.free_events.back();
        S.free_events.pop_back();
    } else if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
        set_error("wrs_serve_submit: event creation failed");
        return WRS_EDEVICE;
    }
    if (hipEventRecord(e, (hipStream_t)stream) != hipSuccess) {
        S.free_events.push_back(e);
        set_error("wrs_serve_submit: cannot record on the caller's stream");
        return WRS_EDEVICE;
    }
    *out = e;
    return WRS_OK;
}

extern "C" int wrs_serve_create(const wrs_serve_config* cfg, void** srv) {
    if (!cfg || !srv || cfg->hbm_budget_bytes < (1u << 20) || cfg->max_batch < 1 ||
        cfg->max_batch > WRS_SERVE_MAX_BATCH || cfg->inflight < 1 || cfg->inflight > WRS_SERVE_MAX_INFLIGHT) {
        set_error("wrs_serve_create: bad config");
        return WRS_EINVAL;
    }
    auto* S = new Server();
    S->cfg = *cfg;
    if (S->cfg.one_at_a_time) S->cfg.inflight = 1;
    S->maxb = S->cfg.one_at_a_time ? 1 : S->cfg.max_batch;
    (void)hipGetDevice(&S->device);
    if (!S->pool.init(cfg->hbm_budget_bytes)) {
        delete S;
        set_error("wrs_serve_create: cannot reserve %zu bytes", cfg->hbm_budget_bytes);
        return WRS_ENOMEM;
    }
    if (cfg->host_stage_bytes > 0) {
        if (hipHostMalloc((void**)&S->h_arena, cfg->host_stage_bytes) != hipSuccess) {
            delete S;
            set_error("wrs_serve_create: cannot reserve %zu bytes of pinned staging", cfg->host_stage_bytes);
            return WRS_ENOMEM;
        }
        S->stage.reset(S->h_arena, cfg->host_stage_bytes);
    }
    const size_t sbytes = slot_bytes(S->maxb);
    for (int i = 0; i < S->cfg.inflight; ++i) {
        hipStream_t st;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            release_slots(S);
            delete S;
            set_error("wrs_serve_create: stream creation failed");
            return WRS_EDEVICE;
        }
        S->streams.push_back(st);
        char* h = nullptr;
        if (hipHostMalloc((void**)&h, sbytes) != hipSuccess) h = nullptr;
        S->staging.push_back(h);
        char* d = (char*)S->pool.alloc(sbytes);
        S->dev_desc.push_back(d);
        S->slot_busy.push_back(false);
        if (!h || !d) {
            release_slots(S);
            delete S;
            set_error("wrs_serve_create: cannot reserve %zu bytes of descriptors per slot", sbytes);
            return WRS_ENOMEM;
        }
    }
    S->reserved = S->pool.used();
    S->worker = std::thread(worker_main, S);
    *srv = S;
    return WRS_OK;
}

extern "C" int wrs_serve_submit_build(void* srv, const float* w, int64_t n, int32_t w_on_host, void* stream,
                                      uint64_t* table_id, uint64_t* req) {
    auto* S = (Server*)srv;
    if (!S || !w || !table_id || !req || n < 1 || n > 2147483647LL || (w_on_host != 0 && w_on_host != 1)) {
        set_error("wrs_serve_submit_build: bad arguments");
        return WRS_EINVAL;
    }
    const size_t wbytes = (size_t)n * sizeof(float);
    if (w_on_host && wbytes > S->stage.size()) {
        set_error("wrs_serve_submit_build: %zu bytes of host weights exceed the staging arena", wbytes);
        return WRS_ENOMEM;
    }
    const size_t need = (size_t)n * sizeof(wrs_entry) + build_ws_bytes(n) + 1024 + (w_on_host ? wbytes : 0);
    const size_t avail = S->cfg.hbm_budget_bytes > S->reserved ? S->cfg.hbm_budget_bytes - S->reserved : 0;
    if (need > avail) { set_error("wrs_serve_submit_build: request exceeds the HBM budget"); return WRS_ENOMEM; }
    float* stage = nullptr;
    if (w_on_host) {
        // room in the staging arena, waiting for running requests to retire
        std::unique_lock<std::mutex> lk(S->mu);
        S->cv_done.wait(lk, [&] { return (stage = (float*)S->stage.alloc(wbytes)) != nullptr || S->stop; });
        if (!stage) { set_error("wrs_serve_submit_build: server stopping"); return WRS_EINVAL; }
        lk.unlock();
        memcpy(stage, w, wbytes);  // the caller's buffer is free when the call returns
    }
    std::lock_guard<std::mutex> g(S->mu);
    auto r = std::make_unique<Request>();
    const int er = submission_event(*S, stream, &r->after);
    if (er != WRS_OK) {
        S->stage.release(stage, wbytes);
        S->cv_done.notify_all();
        return er;
    }
    auto t = std::make_unique<Table>();
    t->id = S->next_id++;
    t->n = n;
    t->d_w = w_on_host ? nullptr : w;
    t->table_bytes = (size_t)n * sizeof(wrs_entry);
    t->refs = 1;
    r->id = S->next_id++;
    r->op = OP_BUILD;
    r->table_id = t->id;
    r->h_stage = stage;
    r->stage_bytes = stage ? wbytes : 0;
    r->t_submit = now_s();
    if (S->t_first < 0) S->t_first = r->t_submit;
    *table_id = t->id;
    *req = r->id;
    S->queue.push_back(r.get());
    S->tables[t->id] = std::move(t);
    S->reqs[r->id] = std::move(r);
    S->submitted++;
    S->arrivals.fetch_add(1, std::memory_order_release);
    S->builds++;
    S->items += (uint64_t)n;
    S->cv.notify_one();
    return WRS_OK;
}

extern "C" int wrs_serve_submit_sample(void* srv, uint64_t table_id, int64_t k, uint64_t seed, int32_t* d_out,
                                       void* stream, uint64_t* req) {
    auto* S = (Server*)srv;
    if (!S || !req || k < 1 || !d_out) { set_error("wrs_serve_submit_sample: bad arguments"); return WRS_EINVAL; }
    std::lock_guard<std::mutex> g(S->mu);
    auto it = S->tables.find(table_id);
    if (it == S->tables.end()) { set_error("wrs_serve_submit_sample: unknown table %llu", (unsigned long long)table_id); return WRS_ENOTFOUND; }
    auto r = std::make_unique<Request>();
    const int er = submission_event(*S, stream, &r->after);
    if (er != WRS_OK) return er;
    it->second->refs++;
    idle_update(*S, it->second.get());
    r->id = S->next_id++;
    r->op = OP_SAMPLE;
    r->table_id = table_id;
    r->k = k;
    r->seed = seed;
    r->d_out = d_out;
    r->t_submit = now_s();
    if (S->t_first < 0) S->t_first = r->t_submit;
    *req = r->id;
    S->queue.push_back(r.get());
    S->reqs[r->id] = std::move(r);
    S->submitted++;
    S->arrivals.fetch_add(1, std::memory_order_release);
    S->samples++;
    S->drawn += (uint64_t)k;
    S->cv.notify_one();
    return WRS_OK;
}

extern "C" int wrs_serve_poll(void* srv, uint64_t req, int* done, int* status) {
    auto* S = (Server*)srv;
    if (!S || !done || !status) return WRS_EINVAL;
    std::lock_guard<std::mutex> g(S->mu);
    auto it = S->reqs.find(req);
    if (it == S->reqs.end()) return WRS_ENOTFOUND;
    *done = it->second->done;
    *status = it->second->status;
    return WRS_OK;
}

extern "C" int wrs_serve_request_times(void* srv, uint64_t req, double* submit_s, double* done_s) {
    auto* S = (Server*)srv;
    if (!S || !submit_s || !done_s) return WRS_EINVAL;
    std::lock_guard<std::mutex> g(S->mu);
    auto it = S->reqs.find(req);
    if (it == S->reqs.end()) return WRS_ENOTFOUND;
    if (!it->second->done) return WRS_EBUSY;
    *submit_s = it->second->t_submit;
    *done_s = it->second->t_done;
    return WRS_OK;
}

extern "C" int wrs_serve_wait(void* srv, uint64_t req, int* status) {
    auto* S = (Server*)srv;
    if (!S || !status) return WRS_EINVAL;
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->reqs.find(req);
    if (it == S->reqs.end()) return WRS_ENOTFOUND;
    Request* r = it->second.get();
    S->cv_done.wait(lk, [&] { return r->done; });
    *status = r->status;
    return WRS_OK;
}

extern "C" int wrs_serve_release_table(void* srv, uint64_t table_id) {
    auto* S = (Server*)srv;
    if (!S) return WRS_EINVAL;
    std::lock_guard<std::mutex> g(S->mu);
    auto it = S->tables.find(table_id);
    if (it == S->tables.end()) return WRS_ENOTFOUND;
    Table* t = it->second.get();
    if (t->refs > 0 || t->state == T_QUEUED || t->state == T_BUILDING) return WRS_EBUSY;
    if (t->idle) {
        S->idle.erase(t->idle_at);
        t->idle = false;
    }
    S->pool.release(t->d_table, t->table_bytes);
    S->pool.release(t->sc, 256);
    S->tables.erase(it);
    return WRS_OK;
}

extern "C" int wrs_serve_read_table(void* srv, uint64_t table_id, wrs_entry* h_table, int64_t n) {
    auto* S = (Server*)srv;
    if (!S || !h_table) return WRS_EINVAL;
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->tables.find(table_id);
    if (it == S->tables.end()) return WRS_ENOTFOUND;
    Table* t = it->second.get();
    if (n != t->n) return WRS_EINVAL;
    S->cv_done.wait(lk, [&] { return t->state == T_READY || t->state == T_FAILED; });
    if (t->state == T_FAILED) return t->status;
    if (hipMemcpy(h_table, t->d_table, t->table_bytes, hipMemcpyDeviceToHost) != hipSuccess) return WRS_EDEVICE;
    return WRS_OK;
}

extern "C" int wrs_serve_stats(void* srv, wrs_serve_stats_t* out) {
    auto* S = (Server*)srv;
    if (!S || !out) return WRS_EINVAL;
    std::lock_guard<std::mutex> g(S->mu);
    memset(out, 0, sizeof *out);
    out->submitted = S->submitted;
    out->completed = S->completed;
    out->failed = S->failed;
    out->builds = S->builds;
    out->samples = S->samples;
    out->items_built = S->items;
    out->samples_drawn = S->drawn;
    out->launches = S->launches;
    if (!S->lat_us.empty()) {
        std::vector<double> v = S->lat_us;
        auto q = [&](double p) {
            size_t i = (size_t)(p * (v.size() - 1) + 0.5);
            std::nth_element(v.begin(), v.begin() + i, v.end());
            return v[i];
        };
        out->p50_us = q(0.50);
        out->p99_us = q(0.99);
        out->max_us = *std::max_element(v.begin(), v.end());
    }
    out->busy_s = (S->t_first >= 0) ? S->t_last - S->t_first : 0.0;
    out->bytes_in_use = S->pool.used();
    out->bytes_peak = S->pool.peak();
    out->tables_resident = S->tables.size();
    return WRS_OK;
}

extern "C" int wrs_serve_destroy(void* srv) {
    auto* S = (Server*)srv;
    if (!S) return WRS_EINVAL;
    {
        std::lock_guard<std::mutex> g(S->mu);
        S->stop = true;
        S->cv.notify_all();
        S->cv_done.notify_all();
    }
    if (S->worker.joinable()) S->worker.join();
    release_slots(S);
    delete S;
    return WRS_OK;
}
