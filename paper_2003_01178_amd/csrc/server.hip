// Serving loop: continuous batching of star queries over shared-scan passes.
//
// The fact table is cut into S segments of segment_rows rows.  A server
// thread runs a clock: each step scans the next segment once per template,
// for every query that occupies one of that template's slots, through
// crystal_run_shared_scan (outputs accumulate per slot).  A query admitted at
// step p is complete after S steps, at which point its slot output is copied
// to pinned host memory and the slot is free again.  Requests that arrive
// while others are on the GPU wait in a FIFO queue per template and are
// admitted into free slots at the next step, so queries at different clock
// phases share every pass.  Slot i of a template is bit i of the batch's
// query masks; the masks are rebuilt when a slot's occupant changes.
//
// A query may carry a deadline: one that has not completed by then is
// dropped (from its queue, or from its slot before its last segment is
// issued) and reported as timed out.  A client may also cancel a ticket.
// Both are applied by the server thread between clock steps.
//
// With fake_executor set, no HIP call is made: a step completes
// fake_step_ns after it is issued and results are zero.  This drives the
// scheduling logic (admission, slot reuse, queue limits, latency accounting)
// on a machine without a GPU.
#include <stdint.h>
#include <string.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "internal.hpp"

namespace crystal {

using Clock = std::chrono::steady_clock;

static int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(Clock::now().time_since_epoch()).count();
}

struct Request {
    int64_t ticket;
    int32_t tmpl;
    crystal_range preds[CRYSTAL_MAX_PREDS];
    crystal_range filters[CRYSTAL_MAX_JOINS];
    int64_t t_submit;
    int64_t deadline;         // absolute steady-clock ns; 0: none
};

struct Result {
    int32_t tmpl = 0;
    std::vector<int64_t> value;
    int32_t done = 0;
    crystal_status status = CRYSTAL_OK;  // CRYSTAL_ETIMEDOUT: dropped at its deadline
    int64_t t_submit = 0;
    int64_t t_done = 0;
};

struct Slot {
    bool busy = false;        // occupied (issuing or draining)
    int64_t ticket = -1;
    int64_t deadline = 0;
    int32_t steps_left = 0;   // segments still to issue
    crystal_range preds[CRYSTAL_MAX_PREDS];
    crystal_range filters[CRYSTAL_MAX_JOINS];
    bool zero_pending = false;
};

struct Completion {
    int t, q;                 // template, slot
    int64_t ticket;           // the slot's occupant when its last segment was issued
};

struct Step {
    hipEvent_t ev = nullptr;
    int64_t t_issue = 0;
    std::vector<Completion> completing;  // slots whose last segment is in this step
};

struct Server {
    crystal_server_config cfg;
    int64_t n_rows = 0;
    int64_t n_segments = 0;
    int64_t clock = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int64_t *pinned = nullptr;        // host copies of slot outputs, then of the status word
    int32_t *status = nullptr;        // device status word (inside the workspace)
    int32_t *pinned_status = nullptr; // its host copy, taken in every step that completes a query
    std::vector<std::vector<Slot>> slots;
    std::vector<std::vector<bool>> masks_dirty;  // [template][0]: slot set changed since the last build
    std::vector<std::deque<Request>> queue;
    std::map<int64_t, Result> results;
    std::deque<Step> inflight;
    std::mutex mu;
    std::condition_variable cv;
    std::thread worker;
    std::atomic<bool> stop{false};
    int64_t next_ticket = 1;
    std::vector<int64_t> cancel_req;  // tickets cancelled by clients, applied by the server thread
    crystal_status error = CRYSTAL_OK;
    // statistics (written by the server thread, read by crystal_server_stats)
    std::atomic<int64_t> admitted{0}, completed{0}, rejected{0}, steps{0}, busy_slot_steps{0}, cancelled{0},
        timed_out{0};

    int64_t n_groups(int t) const { return cfg.templates[t].plan.n_groups; }
    int64_t *slot_out(int t, int s) const {
        int64_t off = 0;
        for (int u = 0; u < t; ++u) off += n_groups(u) * cfg.slots_per_template;
        off += n_groups(t) * s;
        return (int64_t *)cfg.workspace + 2 + off;  // first 16 bytes: status word
    }
    int64_t *pinned_out(int t, int s) const {
        int64_t off = 0;
        for (int u = 0; u < t; ++u) off += n_groups(u) * cfg.slots_per_template;
        return pinned + off + n_groups(t) * s;
    }

    void fail(crystal_status st) {
        std::lock_guard<std::mutex> lk(mu);
        if (error == CRYSTAL_OK) error = st;
    }

    // Issue one clock step; returns false when nothing was active.
    bool issue_step() {
        Step step;
        bool any = false;
        const int64_t seg_lo = clock * cfg.segment_rows;
        const int64_t seg_hi = seg_lo + cfg.segment_rows < n_rows ? seg_lo + cfg.segment_rows : n_rows;
        for (int t = 0; t < cfg.n_templates; ++t) {
            auto &ss = slots[t];
            bool active = false;
            for (auto &sl : ss) active |= sl.busy && sl.steps_left > 0;
            if (!active) continue;
            any = true;
            const crystal_server_template &tp = cfg.templates[t];
            if (!cfg.fake_executor) {
                // rebuild the query masks of joins whose slot set changed
                if (masks_dirty[t][0]) {
                    // every join's table in one batched build (two launches)
                    crystal_range r[CRYSTAL_MAX_JOINS][CRYSTAL_MAX_BATCH];
                    crystal_qmask_build_item items[CRYSTAL_MAX_JOINS];
                    for (int j = 0; j < tp.plan.n_joins; ++j) {
                        for (int q = 0; q < cfg.slots_per_template; ++q) {
                            const bool on = ss[q].busy && ss[q].steps_left > 0;
                            r[j][q] = on ? ss[q].filters[j] : crystal_range{1, 0};
                        }
                        items[j] = crystal_qmask_build_item{&tp.masks[j], tp.dim_keys[j], tp.dim_filter[j],
                                                            tp.dim_rows[j], r[j], cfg.slots_per_template, 0};
                    }
                    if (crystal_qmask_build_batch(items, tp.plan.n_joins, status, stream) != CRYSTAL_OK) {
                        fail(CRYSTAL_EHIP);
                        return false;
                    }
                    masks_dirty[t][0] = false;
                }
                crystal_batch b;
                memset(&b, 0, sizeof(b));
                b.plan = tp.plan;
                for (int j = 0; j < tp.plan.n_joins; ++j) b.masks[j] = tp.masks[j];
                b.n_queries = cfg.slots_per_template;
                int32_t zero[CRYSTAL_MAX_BATCH];
                int n_zero = 0;
                for (int q = 0; q < cfg.slots_per_template; ++q) {
                    Slot &sl = ss[q];
                    const bool on = sl.busy && sl.steps_left > 0;
                    if (sl.zero_pending) {
                        zero[n_zero++] = q;
                        sl.zero_pending = false;
                    }
                    for (int i = 0; i < tp.plan.n_preds; ++i) b.queries[q].preds[i] = on ? sl.preds[i] : crystal_range{1, 0};
                    b.queries[q].out = slot_out(t, q);
                }
                // the outputs of newly admitted queries, cleared in one launch
                if (zero_slots((uint64_t *)slot_out(t, 0), n_groups(t), zero, n_zero, stream) != hipSuccess) {
                    fail(CRYSTAL_EHIP);
                    return false;
                }
                b.row_begin = seg_lo;
                b.row_end = seg_hi;
                if (crystal_run_shared_scan(&b, status, stream) != CRYSTAL_OK) {
                    fail(CRYSTAL_EHIP);
                    return false;
                }
            }
            for (int q = 0; q < cfg.slots_per_template; ++q) {
                Slot &sl = ss[q];
                if (!(sl.busy && sl.steps_left > 0)) continue;
                ++busy_slot_steps;
                if (--sl.steps_left == 0) {
                    step.completing.push_back({t, q, sl.ticket});
                    masks_dirty[t][0] = true;  // its bit must stop matching
                    if (!cfg.fake_executor &&
                        hipMemcpyAsync(pinned_out(t, q), slot_out(t, q), n_groups(t) * 8, hipMemcpyDeviceToHost,
                                       stream) != hipSuccess) {
                        fail(CRYSTAL_EHIP);
                        return false;
                    }
                }
            }
        }
        if (!any) return false;
        // The status word is sticky (the first device error stays), so its
        // copy after a step's kernels covers every step up to this one; it is
        // taken only where results are released.
        if (!cfg.fake_executor && !step.completing.empty() &&
            hipMemcpyAsync(pinned_status, status, 4, hipMemcpyDeviceToHost, stream) != hipSuccess) {
            fail(CRYSTAL_EHIP);
            return false;
        }
        clock = (clock + 1) % n_segments;
        ++steps;
        step.t_issue = now_ns();
        if (!cfg.fake_executor) {
            if (hipEventCreateWithFlags(&step.ev, hipEventDisableTiming) != hipSuccess ||
                hipEventRecord(step.ev, stream) != hipSuccess) {
                fail(CRYSTAL_EHIP);
                return false;
            }
        }
        inflight.push_back(std::move(step));
        return true;
    }

    bool step_done(const Step &s) {
        if (cfg.fake_executor) return now_ns() - s.t_issue >= cfg.fake_step_ns;
        const hipError_t e = hipEventQuery(s.ev);
        if (e == hipErrorNotReady) return false;
        // a failed query retires the step too (so that shutdown never waits on
        // it); the server's error is set, and every later call reports it
        if (e != hipSuccess) fail(CRYSTAL_EHIP);
        return true;
    }

    // Retire completed steps in order: finished queries get their results.
    void retire() {
        while (!inflight.empty() && step_done(inflight.front())) {
            Step s = std::move(inflight.front());
            inflight.pop_front();
            if (s.ev) (void)hipEventDestroy(s.ev);  // the step is complete; nothing to do on failure
            const int64_t t_done = now_ns();
            // a device error (key outside a mask table, full ranked table,
            // group index out of range) means rows were skipped: the results
            // released by this step, and every later one, would be wrong
            if (!cfg.fake_executor && !s.completing.empty()) {
                const int32_t dev_st = __atomic_load_n(pinned_status, __ATOMIC_ACQUIRE);
                if (dev_st != CRYSTAL_OK) fail((crystal_status)dev_st);
            }
            std::lock_guard<std::mutex> lk(mu);
            for (const Completion &c : s.completing) {
                Slot &sl = slots[c.t][c.q];
                // a cancelled query's result entry is gone; its slot is
                // still reserved for it (nothing is admitted into a slot
                // whose last segment is in flight) and is freed here
                auto it = results.find(c.ticket);
                if (it != results.end()) {
                    it->second.value.assign(n_groups(c.t), 0);
                    if (!cfg.fake_executor)
                        memcpy(it->second.value.data(), pinned_out(c.t, c.q), n_groups(c.t) * 8);
                    it->second.done = 1;
                    it->second.t_done = t_done;
                    ++completed;
                }
                if (sl.ticket == c.ticket) sl = Slot();
            }
        }
    }

    // Move queued requests into free slots (FIFO per template).
    void admit() {
        std::lock_guard<std::mutex> lk(mu);
        for (int t = 0; t < cfg.n_templates; ++t) {
            for (int q = 0; q < cfg.slots_per_template && !queue[t].empty(); ++q) {
                Slot &sl = slots[t][q];
                if (sl.busy) continue;
                const Request r = queue[t].front();
                queue[t].pop_front();
                sl.busy = true;
                sl.ticket = r.ticket;
                sl.deadline = r.deadline;
                sl.steps_left = (int32_t)n_segments;
                memcpy(sl.preds, r.preds, sizeof(sl.preds));
                memcpy(sl.filters, r.filters, sizeof(sl.filters));
                sl.zero_pending = true;
                masks_dirty[t][0] = true;
                ++admitted;
            }
        }
    }

    // Drop a query that still has segments to issue: its slot is free for
    // the next admission (in-flight passes may still add into its output,
    // which the next occupant's clear, later on the same stream, resets).
    // Called with mu held.
    bool drop_running(int64_t ticket) {
        for (int t = 0; t < cfg.n_templates; ++t)
            for (auto &sl : slots[t])
                if (sl.busy && sl.ticket == ticket) {
                    if (sl.steps_left == 0) return false;  // its last segment is in flight
                    sl = Slot();
                    masks_dirty[t][0] = true;
                    return true;
                }
        return false;
    }

    bool drop_queued(int64_t ticket) {
        for (auto &dq : queue)
            for (auto it = dq.begin(); it != dq.end(); ++it)
                if (it->ticket == ticket) {
                    dq.erase(it);
                    return true;
                }
        return false;
    }

    // Apply client cancellations and expired deadlines.
    void expire() {
        std::lock_guard<std::mutex> lk(mu);
        for (int64_t tk : cancel_req)
            if (!drop_queued(tk)) drop_running(tk);
        cancel_req.clear();
        const int64_t now = now_ns();
        auto time_out = [&](int64_t ticket) {
            auto it = results.find(ticket);
            if (it == results.end()) return;
            it->second.done = 1;
            it->second.status = CRYSTAL_ETIMEDOUT;
            it->second.t_done = now;
            ++timed_out;
        };
        for (auto &dq : queue)
            for (auto it = dq.begin(); it != dq.end();) {
                if (it->deadline && now >= it->deadline) {
                    time_out(it->ticket);
                    it = dq.erase(it);
                } else {
                    ++it;
                }
            }
        for (int t = 0; t < cfg.n_templates; ++t)
            for (auto &sl : slots[t])
                if (sl.busy && sl.steps_left > 0 && sl.deadline && now >= sl.deadline) {
                    time_out(sl.ticket);
                    sl = Slot();
                    masks_dirty[t][0] = true;
                }
    }

    void run() {
        if (!cfg.fake_executor && hipSetDevice(device_id) != hipSuccess) {
            fail(CRYSTAL_EHIP);
            return;
        }
        while (!stop.load()) {
            retire();
            expire();
            admit();
            bool issued = false;
            if ((int32_t)inflight.size() < cfg.inflight_steps) issued = issue_step();
            if (!issued) {
                std::unique_lock<std::mutex> lk(mu);
                cv.wait_for(lk, std::chrono::microseconds(inflight.empty() ? 200 : 20));
            }
        }
        // drain what is on the GPU before the slots and buffers go away
        while (!inflight.empty()) {
            retire();
            if (!inflight.empty()) std::this_thread::sleep_for(std::chrono::microseconds(50));
        }
    }

    int device_id = 0;
};

static size_t workspace_bytes(const crystal_server_config &c) {
    size_t b = 16;
    for (int t = 0; t < c.n_templates; ++t) b += (size_t)c.templates[t].plan.n_groups * 8 * c.slots_per_template;
    return (b + 255) / 256 * 256;
}

static crystal_status validate(const crystal_server_config &c) {
    if (c.n_templates < 1 || c.n_templates > CRYSTAL_SERVER_MAX_TEMPLATES || c.slots_per_template < 1 ||
        c.slots_per_template > CRYSTAL_MAX_BATCH || c.segment_rows <= 0 || (c.segment_rows & 3) ||
        c.max_queue < 1 || c.inflight_steps < 1 || c.inflight_steps > 64)
        return CRYSTAL_EINVAL;
    int64_t n_rows = -1;
    for (int t = 0; t < c.n_templates; ++t) {
        const crystal_server_template &tp = c.templates[t];
        StarPlanDev d;
        if (star_plan_to_dev(tp.plan, d) != CRYSTAL_OK) return CRYSTAL_EINVAL;
        if (n_rows >= 0 && tp.plan.n_rows != n_rows) return CRYSTAL_EINVAL;  // one fact table
        n_rows = tp.plan.n_rows;
        if (!c.fake_executor)
            for (int j = 0; j < tp.plan.n_joins; ++j) {
                if (!tp.masks[j].mem || !tp.dim_keys[j] || tp.dim_rows[j] < 0) return CRYSTAL_EINVAL;
                for (int i = 0; i < j; ++i)  // each join has its own table (built together)
                    if (tp.masks[i].mem == tp.masks[j].mem) return CRYSTAL_EINVAL;
            }
    }
    if (n_rows <= 0) return CRYSTAL_EINVAL;
    if (!c.fake_executor && (!c.workspace || c.workspace_bytes < workspace_bytes(c))) return CRYSTAL_ESCRATCH;
    return CRYSTAL_OK;
}

}  // namespace crystal

using namespace crystal;

struct crystal_server {
    Server s;
};

extern "C" {

size_t crystal_server_workspace_bytes(const crystal_server_config *cfg) {
    if (!cfg || cfg->n_templates < 1 || cfg->n_templates > CRYSTAL_SERVER_MAX_TEMPLATES) return 0;
    return workspace_bytes(*cfg);
}

crystal_status crystal_server_create(const crystal_server_config *cfg, crystal_server **out) {
    if (!cfg || !out) return CRYSTAL_EINVAL;
    *out = nullptr;
    crystal_status st = validate(*cfg);
    if (st != CRYSTAL_OK) return st;
    crystal_server *h = new crystal_server();
    Server &s = h->s;
    s.cfg = *cfg;
    s.n_rows = cfg->templates[0].plan.n_rows;
    s.n_segments = (s.n_rows + cfg->segment_rows - 1) / cfg->segment_rows;
    s.slots.assign(cfg->n_templates, std::vector<Slot>(cfg->slots_per_template));
    s.masks_dirty.assign(cfg->n_templates, std::vector<bool>(1, true));
    s.queue.resize(cfg->n_templates);
    if (!cfg->fake_executor) {
        if (hipGetDevice(&s.device_id) != hipSuccess) {
            delete h;
            return CRYSTAL_EHIP;
        }
        if (cfg->stream) {
            s.stream = (hipStream_t)cfg->stream;
        } else if (hipStreamCreate(&s.stream) != hipSuccess) {
            delete h;
            return CRYSTAL_EHIP;
        } else {
            s.own_stream = true;
        }
        size_t host_bytes = 0;
        for (int t = 0; t < cfg->n_templates; ++t) host_bytes += (size_t)s.n_groups(t) * 8 * cfg->slots_per_template;
        if (hipHostMalloc((void **)&s.pinned, host_bytes + 8, hipHostMallocDefault) != hipSuccess) {
            if (s.own_stream) (void)hipStreamDestroy(s.stream);
            delete h;
            return CRYSTAL_EHIP;
        }
        s.pinned_status = (int32_t *)((char *)s.pinned + host_bytes);
        *s.pinned_status = CRYSTAL_OK;
        s.status = (int32_t *)cfg->workspace;
        if (fill_u32((uint32_t *)s.status, 4, 0u, s.stream) != hipSuccess) {
            (void)hipHostFree(s.pinned);
            if (s.own_stream) (void)hipStreamDestroy(s.stream);
            delete h;
            return CRYSTAL_EHIP;
        }
    }
    s.worker = std::thread([&s] { s.run(); });
    *out = h;
    return CRYSTAL_OK;
}

crystal_status crystal_server_submit(crystal_server *h, int32_t template_id, const crystal_range *preds,
                                     const crystal_range *dim_filters, int64_t deadline_ns, int64_t *ticket) {
    if (!h || !ticket || deadline_ns < 0) return CRYSTAL_EINVAL;
    Server &s = h->s;
    if (template_id < 0 || template_id >= s.cfg.n_templates) return CRYSTAL_EINVAL;
    const crystal_star_query &p = s.cfg.templates[template_id].plan;
    if ((p.n_preds > 0 && !preds) || (p.n_joins > 0 && !dim_filters)) return CRYSTAL_EINVAL;
    Request r;
    memset(&r, 0, sizeof(r));
    r.tmpl = template_id;
    for (int i = 0; i < p.n_preds; ++i) r.preds[i] = preds[i];
    for (int j = 0; j < p.n_joins; ++j) r.filters[j] = dim_filters[j];
    r.t_submit = now_ns();
    r.deadline = deadline_ns > 0 ? r.t_submit + deadline_ns : 0;
    {
        std::lock_guard<std::mutex> lk(s.mu);
        if (s.error != CRYSTAL_OK) return s.error;
        if ((int64_t)s.queue[template_id].size() >= s.cfg.max_queue) {
            ++s.rejected;
            return CRYSTAL_EBUSY;
        }
        r.ticket = s.next_ticket++;
        Result res;
        res.tmpl = template_id;
        res.t_submit = r.t_submit;
        s.results.emplace(r.ticket, std::move(res));
        s.queue[template_id].push_back(r);
        *ticket = r.ticket;
    }
    s.cv.notify_one();
    return CRYSTAL_OK;
}

crystal_status crystal_server_poll(crystal_server *h, int64_t ticket, int64_t *result, int64_t result_capacity,
                                   int32_t *done, int64_t *latency_ns) {
    if (!h || !done) return CRYSTAL_EINVAL;
    Server &s = h->s;
    std::lock_guard<std::mutex> lk(s.mu);
    if (s.error != CRYSTAL_OK) return s.error;
    auto it = s.results.find(ticket);
    if (it == s.results.end()) return CRYSTAL_EINVAL;
    // the ticket's own template fixes the result size, whatever is done
    if (result && result_capacity < s.n_groups(it->second.tmpl)) return CRYSTAL_EINVAL;
    *done = it->second.done;
    if (!it->second.done) return CRYSTAL_OK;
    if (it->second.status != CRYSTAL_OK) {  // timed out: no result
        const crystal_status st = it->second.status;
        if (latency_ns) *latency_ns = it->second.t_done - it->second.t_submit;
        s.results.erase(it);
        return st;
    }
    if (latency_ns) *latency_ns = it->second.t_done - it->second.t_submit;
    if (result) memcpy(result, it->second.value.data(), it->second.value.size() * 8);
    s.results.erase(it);
    return CRYSTAL_OK;
}

crystal_status crystal_server_cancel(crystal_server *h, int64_t ticket) {
    if (!h) return CRYSTAL_EINVAL;
    Server &s = h->s;
    {
        std::lock_guard<std::mutex> lk(s.mu);
        if (s.error != CRYSTAL_OK) return s.error;
        auto it = s.results.find(ticket);
        if (it == s.results.end()) return CRYSTAL_EINVAL;
        const bool was_done = it->second.done;
        s.results.erase(it);
        ++s.cancelled;
        if (!was_done) s.cancel_req.push_back(ticket);
    }
    s.cv.notify_one();
    return CRYSTAL_OK;
}

crystal_status crystal_server_get_stats(crystal_server *h, crystal_server_stats *out) {
    if (!h || !out) return CRYSTAL_EINVAL;
    Server &s = h->s;
    std::lock_guard<std::mutex> lk(s.mu);
    out->admitted = s.admitted;
    out->completed = s.completed;
    out->rejected = s.rejected;
    out->steps = s.steps;
    out->busy_slot_steps = s.busy_slot_steps;
    out->cancelled = s.cancelled;
    out->timed_out = s.timed_out;
    int64_t q = 0;
    for (auto &d : s.queue) q += (int64_t)d.size();
    out->queued = q;
    out->n_segments = s.n_segments;
    return s.error;
}

crystal_status crystal_server_destroy(crystal_server *h) {
    if (!h) return CRYSTAL_EINVAL;
    Server &s = h->s;
    s.stop.store(true);
    s.cv.notify_all();
    if (s.worker.joinable()) s.worker.join();
    crystal_status st = s.error;
    if (!s.cfg.fake_executor) {
        // teardown: a failure here leaves nothing to undo; the server's own
        // error (if any) is what is reported
        if (hipStreamSynchronize(s.stream) != hipSuccess && st == CRYSTAL_OK) st = CRYSTAL_EHIP;
        if (s.pinned) (void)hipHostFree(s.pinned);
        if (s.own_stream) (void)hipStreamDestroy(s.stream);
    }
    delete h;
    return st;
}

}  // extern "C"
