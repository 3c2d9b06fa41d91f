// Request server: continuous batching of stereo pairs on one device.
//
// Callers submit pairs of any supported shape from any host thread.  One
// scheduler thread owns the device side:
//   * a workspace arena of a fixed byte budget, allocated once and kept
//     resident; each admitted request takes a block of it (first fit) sized by
//     its own footprint and gives it back when its results are complete;
//   * `slots` launch slots spread round-robin over `streams` streams (default
//     priority).  A slot holds one group of requests at a time.  Slots on the
//     same stream run their groups back to back in admission order (the
//     device never waits for the host between them); slots on different
//     streams run concurrently.
// Whenever a slot is free, the scheduler takes requests in arrival order from
// the head of the queue for as long as their workspaces fit and the group
// stays within its limits (a request count, and a total of W * H * D * paths
// cells: a request that fills the device on its own gains nothing from
// sharing a launch, and would only delay the others), and launches them as
// one group: a group of one
// runs through the single-pair kernels, a larger group through the batched
// kernels (one launch per stage for the group).  Requests that arrive while
// groups run are admitted into the next free slot.  Latency is measured from
// submission to the moment the scheduler sees the group's completion event.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/sgm.h"
#include "sgm_batch.h"
#include "sgm_plan.h"

namespace {

using Clock = std::chrono::steady_clock;

// First-fit allocator over [0, size) with coalescing of freed blocks.
class ArenaAllocator {
public:
    void reset(size_t size) {
        free_.clear();
        if (size) free_[0] = size;
        used_ = 0;
    }
    bool alloc(size_t bytes, size_t* off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes, at = it->first + bytes;
            free_.erase(it);
            if (rest) free_[at] = rest;
            used_ += bytes;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t used() const { return used_; }

private:
    std::map<size_t, size_t> free_;
    size_t used_ = 0;
};

struct Request {
    uint64_t ticket = 0;
    sgm_item item{};
    sgm::Plan plan;
    size_t bytes = 0, offset = 0;
    uint64_t cells = 0;  // W * H * D * paths
    Clock::time_point t_submit;
    int status = SGM_REQ_QUEUED;
    double latency_s = 0.0;
};

struct Slot {
    hipStream_t stream = nullptr;  // shared with the other slots of its stream
    hipEvent_t done = nullptr;
    sgm::BatchStaging* st = nullptr;
    std::vector<Request*> group;  // empty and not draining = free
    Clock::time_point t_launch;
    // a group the watchdog declared stuck: its requests have failed and left
    // the slot, whose workspace blocks (offset, bytes) stay reserved until
    // the device completes the group
    bool draining = false;
    std::vector<std::pair<size_t, size_t>> held;
    bool busy() const { return !group.empty() || draining; }
};

}  // namespace

struct sgm_server {
    int device = 0;
    sgm::BatchParams bp{};
    size_t budget = 0;
    void* arena = nullptr;
    ArenaAllocator alloc;  // scheduler thread only
    std::vector<Slot> slots;
    std::vector<hipStream_t> streams;

    std::mutex mu;
    std::condition_variable cv_work;  // new requests or shutdown
    std::condition_variable cv_done;  // a request reached a final state
    std::deque<Request*> pending;
    std::unordered_map<uint64_t, Request*> live;  // every ticket not yet retired
    uint64_t next_ticket = 1;
    int max_group = 32;
    size_t max_pending = 4096;
    uint64_t max_group_cells = uint64_t(1) << 28;
    // while a group runs, another one starts beside it only if at least this
    // many requests are queued: at light load a request then waits for the
    // running one instead of sharing the device with it
    int overlap_queue = 3;
    // a group still running this long after its launch is declared stuck
    // (0: never)
    int watchdog_ms = 0;
    bool stop = false;
    std::atomic<uint64_t> wake{0};  // bumped by every submission and by shutdown
    sgm_server_stats stats{};
    std::thread worker;
};

namespace {

int serr(int code, const std::string& m) {
    sgm::set_last_error(m);
    return code;
}

bool final_status(int s) { return s == SGM_REQ_DONE || s == SGM_REQ_CANCELED || s == SGM_REQ_FAILED; }

// Marks the group of a slot finished (DONE, or FAILED if ok is false), frees
// its workspace blocks and frees the slot.  Called with the lock held.
void retire_group(sgm_server* s, Slot& slot, bool ok, Clock::time_point now) {
    for (Request* r : slot.group) {
        s->alloc.release(r->offset, r->bytes);
        r->status = ok ? SGM_REQ_DONE : SGM_REQ_FAILED;
        r->latency_s = std::chrono::duration<double>(now - r->t_submit).count();
        if (ok)
            s->stats.completed++;
        else
            s->stats.failed++;
        s->stats.running--;
    }
    s->stats.bytes_in_use = s->alloc.used();
    slot.group.clear();
}

// The watchdog: fails the requests of a group that has run longer than the
// limit (their callers stop waiting), keeps its workspace blocks and its
// slot until the device completes it.  Called with the lock held.
void declare_stuck(sgm_server* s, Slot& slot, Clock::time_point now) {
    for (Request* r : slot.group) {
        slot.held.emplace_back(r->offset, r->bytes);
        r->status = SGM_REQ_FAILED;
        r->latency_s = std::chrono::duration<double>(now - r->t_submit).count();
        s->stats.failed++;
        s->stats.timed_out++;
        s->stats.running--;
    }
    slot.group.clear();
    slot.draining = true;
    s->stats.draining_groups++;
}

// A stuck group has completed: its workspace blocks and slot are free again.
void drained(sgm_server* s, Slot& slot) {
    for (const auto& b : slot.held) s->alloc.release(b.first, b.second);
    slot.held.clear();
    slot.draining = false;
    s->stats.draining_groups--;
    s->stats.bytes_in_use = s->alloc.used();
}

bool overdue(const sgm_server* s, const Slot& slot, Clock::time_point now) {
    return s->watchdog_ms > 0 && !slot.group.empty() &&
           now - slot.t_launch > std::chrono::milliseconds(s->watchdog_ms);
}

void scheduler(sgm_server* s) {
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    std::vector<sgm_item> items;
    std::vector<sgm::Plan> plans;
    std::vector<uint8_t*> bases;
    for (;;) {
        // 1. completions
        bool any_busy = false, finished = false;
        for (Slot& slot : s->slots) {
            if (!slot.busy()) continue;
            const hipError_t q = hipEventQuery(slot.done);
            if (q == hipErrorNotReady) {
                any_busy = true;
                const Clock::time_point now = Clock::now();
                if (overdue(s, slot, now)) {
                    declare_stuck(s, slot, now);
                    finished = true;
                }
                continue;
            }
            if (slot.draining)
                drained(s, slot);
            else
                retire_group(s, slot, q == hipSuccess, Clock::now());
            finished = true;
        }
        if (finished) s->cv_done.notify_all();

        // 2. admission: fill free slots from the head of the queue
        for (Slot& slot : s->slots) {
            if (s->pending.empty()) break;
            if (slot.busy()) continue;
            if (any_busy && (int)s->pending.size() < s->overlap_queue) break;
            uint64_t cells = 0;
            while (!s->pending.empty() && (int)slot.group.size() < s->max_group) {
                Request* r = s->pending.front();
                if (!slot.group.empty() && cells + r->cells > s->max_group_cells) break;
                if (!s->alloc.alloc(r->bytes, &r->offset)) break;
                cells += r->cells;
                s->pending.pop_front();
                r->status = SGM_REQ_RUNNING;
                slot.group.push_back(r);
            }
            if (slot.group.empty()) break;  // the head does not fit until memory is freed
            items.clear();
            plans.clear();
            bases.clear();
            for (Request* r : slot.group) {
                items.push_back(r->item);
                plans.push_back(r->plan);
                bases.push_back(static_cast<uint8_t*>(s->arena) + r->offset);
            }
            s->stats.running += slot.group.size();
            s->stats.pending = s->pending.size();
            s->stats.bytes_in_use = s->alloc.used();
            s->stats.peak_bytes = std::max(s->stats.peak_bytes, s->stats.bytes_in_use);
            s->stats.groups++;
            s->stats.grouped_requests += slot.group.size();
            // enqueueing takes tens of microseconds: let submitters in meanwhile
            // (the slot and the allocator belong to this thread only)
            lk.unlock();
            int rc = SGM_OK;
            if (items.size() == 1) {
                const sgm::Workspace ws = sgm::workspace_carve(plans[0], bases[0]);
                if (sgm::launch_pipeline(plans[0], ws, items[0].left, items[0].right, items[0].out, slot.stream) !=
                    hipSuccess)
                    rc = SGM_EHIP;
            } else {
                rc = sgm::batch_enqueue(s->bp, plans.data(), bases.data(), items.data(), (int)items.size(), slot.st,
                                        slot.stream);
            }
            if (rc == SGM_OK && hipEventRecord(slot.done, slot.stream) != hipSuccess) rc = SGM_EHIP;
            slot.t_launch = Clock::now();
            lk.lock();
            if (rc != SGM_OK) {
                retire_group(s, slot, false, Clock::now());
                s->cv_done.notify_all();
            } else {
                any_busy = true;
            }
        }
        s->stats.pending = s->pending.size();

        // 3. wait
        if (s->stop && s->pending.empty() && !any_busy) break;
        if (!any_busy) {
            s->cv_work.wait(lk, [s] { return s->stop || !s->pending.empty(); });
        } else {
            // groups in flight: poll their completion events without the lock
            // (slots belong to this thread) until one completes or a request
            // arrives; a timed sleep here would add its timer slack to every
            // latency
            const uint64_t seen = s->wake.load();
            lk.unlock();
            for (bool ready = false; !ready && s->wake.load() == seen;) {
                const Clock::time_point now = Clock::now();
                for (Slot& slot : s->slots)
                    if (slot.busy() && (hipEventQuery(slot.done) != hipErrorNotReady || overdue(s, slot, now)))
                        ready = true;
                if (!ready) std::this_thread::yield();
            }
            lk.lock();
        }
    }
}

bool check_item(const sgm_server* s, const sgm_item* it, sgm::Plan* plan, size_t* bytes, std::string* why) {
    sgm::BatchLayout L;
    const char* w = "invalid request";
    if (!sgm::batch_plan(s->bp, it, 1, L, &w)) {
        *why = w;
        return false;
    }
    if (!it->left || !it->right || !it->out) {
        *why = "null buffer pointer";
        return false;
    }
    if ((const void*)it->out == (const void*)it->left || (const void*)it->out == (const void*)it->right) {
        *why = "output aliases an input";
        return false;
    }
    *plan = L.plans[0];
    *bytes = L.total;
    return true;
}

}  // namespace

extern "C" {

sgm_server* sgm_server_create(size_t hbm_budget_bytes, int max_slots, int P1, int P2, int census_w, int census_h) {
    return sgm_server_create_ex(hbm_budget_bytes, max_slots, max_slots, P1, P2, census_w, census_h);
}

sgm_server* sgm_server_create_ex(size_t hbm_budget_bytes, int max_slots, int n_streams, int P1, int P2,
                                 int census_w, int census_h) {
    sgm::Plan probe;  // batch-wide parameters, checked on a 1x1 pair
    probe.W = probe.H = probe.D = 1;
    probe.P1 = P1;
    probe.P2 = P2;
    probe.n_paths = 2;
    probe.cw = census_w;
    probe.ch = census_h;
    const char* why = "invalid parameters";
    if (!sgm::plan_finish(probe, &why)) {
        serr(SGM_EINVAL, why);
        return nullptr;
    }
    if (max_slots < 1 || max_slots > 16 || n_streams < 1 || n_streams > max_slots) {
        serr(SGM_EINVAL, "need 1 <= n_streams <= max_slots <= 16");
        return nullptr;
    }
    if (hbm_budget_bytes < 256) {
        serr(SGM_EINVAL, "hbm_budget_bytes too small");
        return nullptr;
    }
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        serr(SGM_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
        return nullptr;
    }
    sgm_server* s = new (std::nothrow) sgm_server;
    if (!s) {
        serr(SGM_ENOMEM, "host allocation failed");
        return nullptr;
    }
    s->device = dev;
    s->bp = sgm::BatchParams{P1, P2, census_w, census_h, false};
    s->budget = hbm_budget_bytes & ~(size_t)255;
    e = sgm::dev_malloc(&s->arena, s->budget);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        serr(SGM_ENOMEM, std::string("server workspace allocation failed: ") + hipGetErrorString(e));
        delete s;
        return nullptr;
    }
    s->alloc.reset(s->budget);
    s->streams.assign(n_streams, nullptr);
    s->slots.resize(max_slots);
    bool ok = true;
    for (hipStream_t& st : s->streams) ok = ok && hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
    for (size_t k = 0; k < s->slots.size(); ++k) {
        Slot& slot = s->slots[k];
        slot.stream = s->streams[k % s->streams.size()];
        slot.st = ok ? sgm::staging_create() : nullptr;
        ok = ok && slot.st && hipEventCreateWithFlags(&slot.done, hipEventDisableTiming) == hipSuccess;
    }
    if (!ok) {
        (void)hipGetLastError();
        serr(SGM_EHIP, "server stream setup failed");
        for (Slot& t : s->slots) {
            if (t.st) sgm::staging_destroy(t.st);
            if (t.done) (void)hipEventDestroy(t.done);
        }
        for (hipStream_t st : s->streams)
            if (st) (void)hipStreamDestroy(st);
        (void)hipFree(s->arena);
        delete s;
        return nullptr;
    }
    s->worker = std::thread(scheduler, s);
    return s;
}

int sgm_server_set_policy(sgm_server* s, int max_group, int max_pending, uint64_t max_group_cells,
                          int overlap_queue) {
    if (!s) return serr(SGM_EINVAL, "null server");
    if (max_group < 1 || max_group > 256 || max_pending < 1 || overlap_queue < 1) return serr(SGM_EINVAL, "bad policy");
    std::lock_guard<std::mutex> lk(s->mu);
    s->max_group = max_group;
    s->max_pending = (size_t)max_pending;
    s->max_group_cells = max_group_cells;
    s->overlap_queue = overlap_queue;
    return SGM_OK;
}

size_t sgm_server_request_bytes(sgm_server* s, const sgm_item* req) {
    if (!s || !req) return 0;
    sgm::BatchLayout L;
    const char* why = "";
    if (!sgm::batch_plan(s->bp, req, 1, L, &why)) return 0;
    return L.total;
}

int sgm_server_submit(sgm_server* s, const sgm_item* req, uint64_t* ticket) {
    if (!s || !req || !ticket) return serr(SGM_EINVAL, "null argument");
    Request* r = new (std::nothrow) Request;
    if (!r) return serr(SGM_ENOMEM, "host allocation failed");
    std::string why;
    if (!check_item(s, req, &r->plan, &r->bytes, &why)) {
        delete r;
        return serr(SGM_EINVAL, why);
    }
    if (r->bytes > s->budget) {
        delete r;
        return serr(SGM_ENOMEM, "request workspace exceeds the server's memory budget");
    }
    r->item = *req;
    r->cells = (uint64_t)req->w * req->h * req->max_disp * req->n_paths;
    r->t_submit = Clock::now();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) {
            delete r;
            return serr(SGM_ECANCELED, "server is shutting down");
        }
        if (s->pending.size() >= s->max_pending) {
            s->stats.rejected++;
            delete r;
            return serr(SGM_EBUSY, "request queue is full");
        }
        r->ticket = s->next_ticket++;
        s->live[r->ticket] = r;
        s->pending.push_back(r);
        s->stats.submitted++;
        s->stats.pending = s->pending.size();
        *ticket = r->ticket;
    }
    s->wake.fetch_add(1);
    s->cv_work.notify_one();
    return SGM_OK;
}

// Reports a ticket's state; a ticket in a final state is retired (a later
// call with it returns SGM_EINVAL).  Called with the lock held.
static int report(sgm_server* s, uint64_t ticket, int* status, double* latency_s) {
    auto it = s->live.find(ticket);
    if (it == s->live.end()) return serr(SGM_EINVAL, "unknown or retired ticket");
    Request* r = it->second;
    if (status) *status = r->status;
    if (latency_s) *latency_s = r->latency_s;
    if (final_status(r->status)) {
        s->live.erase(it);
        delete r;
    }
    return SGM_OK;
}

int sgm_server_poll(sgm_server* s, uint64_t ticket, int* status, double* latency_s) {
    if (!s) return serr(SGM_EINVAL, "null server");
    std::lock_guard<std::mutex> lk(s->mu);
    return report(s, ticket, status, latency_s);
}

int sgm_server_wait(sgm_server* s, uint64_t ticket, int timeout_ms, int* status, double* latency_s) {
    if (!s) return serr(SGM_EINVAL, "null server");
    std::unique_lock<std::mutex> lk(s->mu);
    auto done = [&] {
        auto it = s->live.find(ticket);
        return it == s->live.end() || final_status(it->second->status);
    };
    if (timeout_ms < 0)
        s->cv_done.wait(lk, done);
    else
        s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), done);
    return report(s, ticket, status, latency_s);
}

int sgm_server_cancel(sgm_server* s, uint64_t ticket) {
    if (!s) return serr(SGM_EINVAL, "null server");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->live.find(ticket);
    if (it == s->live.end()) return serr(SGM_EINVAL, "unknown or retired ticket");
    Request* r = it->second;
    if (r->status != SGM_REQ_QUEUED) return serr(SGM_EBUSY, "request already started or finished");
    s->pending.erase(std::find(s->pending.begin(), s->pending.end(), r));
    r->status = SGM_REQ_CANCELED;
    r->latency_s = std::chrono::duration<double>(Clock::now() - r->t_submit).count();
    s->stats.canceled++;
    s->stats.pending = s->pending.size();
    s->cv_done.notify_all();
    return SGM_OK;
}

int sgm_server_set_watchdog(sgm_server* s, int timeout_ms) {
    if (!s) return serr(SGM_EINVAL, "null server");
    if (timeout_ms < 0) return serr(SGM_EINVAL, "timeout_ms must be >= 0");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->watchdog_ms = timeout_ms;
    }
    s->wake.fetch_add(1);  // the scheduler re-reads the limit
    return SGM_OK;
}

int sgm_server_get_stats(sgm_server* s, sgm_server_stats* out) {
    if (!s || !out) return serr(SGM_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->stats;
    out->budget_bytes = s->budget;
    return SGM_OK;
}

void sgm_server_destroy(sgm_server* s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        for (Request* r : s->pending) {  // queued requests never start
            r->status = SGM_REQ_CANCELED;
            s->stats.canceled++;
        }
        s->pending.clear();
    }
    s->wake.fetch_add(1);
    s->cv_work.notify_all();
    s->worker.join();  // running groups finish first
    s->cv_done.notify_all();
    for (Slot& t : s->slots) {
        sgm::staging_destroy(t.st);
        (void)hipEventDestroy(t.done);
    }
    for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
    (void)hipFree(s->arena);
    for (auto& kv : s->live) delete kv.second;
    delete s;
}

}  // extern "C"
