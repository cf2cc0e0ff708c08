// Serving loop: resident DFAs, admission by device-memory budget, continuous
// batching.
//
// Clients submit (DFA id, device string) requests at any time.  A dispatcher
// thread admits requests in arrival order while the in-flight byte budget and
// the in-flight request cap allow, packs the admitted ones into a batch (one
// persistent matcher launch, see dfa_batch.hip) and runs it on a free slot:
// each slot owns a stream, a device arena, pinned staging for the batch
// descriptors and pinned result records, so dispatching allocates nothing.
// Several slots run at once, so requests that arrive while earlier batches
// are on the GPU join the next batch and overlap with them.  A batch's
// results are copied to pinned memory on its stream; when its event
// completes, the dispatcher publishes the records and releases the budget.
// Every record equals what the request gives alone (same kernels, same
// chunking rule, exact integer results).
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <thread>
#include <unordered_map>

#include <sys/prctl.h>
#include <time.h>

#include "dfa_internal.h"

using namespace dfaspec;

namespace {

uint64_t now_ns() {
    timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (uint64_t)ts.tv_sec * 1000000000ull + (uint64_t)ts.tv_nsec;
}

struct Request {
    uint64_t ticket;
    uint64_t submit_ns;
    uint32_t id;
    const uint8_t *in;
    size_t len;
    uint64_t cost;   // admitted bytes: input + arena estimate
    hipEvent_t ready = nullptr;   // recorded on the producer's stream at submit, or none
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    void *arena = nullptr;
    size_t arena_bytes = 0;
    void *staging = nullptr;        // pinned, descriptors
    size_t staging_bytes = 0;
    uint32_t *d_results = nullptr;
    uint32_t *h_results = nullptr;  // pinned
    bool busy = false;
    std::vector<Request> reqs;
    uint64_t cost = 0;
};

struct Done {
    dfa_result_t r;
    uint64_t submit_ns, done_ns;
};

}  // namespace

struct dfa_server {
    dfa_server_opts_t opts{};
    int device = 0;
    std::vector<const dfa_t *> dfas;
    std::vector<Slot> slots;
    std::mutex mu;
    std::condition_variable cv_submit;   // dispatcher waits for work
    std::condition_variable cv_done;     // clients wait for results
    std::deque<Request> pending;
    std::unordered_map<uint64_t, Done> done;
    uint64_t next_ticket = 1;
    uint64_t inflight_bytes = 0;
    uint32_t inflight_reqs = 0;
    bool stop = false;
    int error = DFA_OK;
    std::thread worker;
    dfa_server_stats_t stats{};
    std::vector<hipEvent_t> free_events;   // producer-stream events for reuse
};

namespace {

uint64_t request_cost(const dfa_t *d, size_t len) {
    // input bytes + two-byte codes + maps of the batch path at 1 KiB chunks
    // (an upper bound)
    const uint64_t stride = (std::max<uint32_t>(d->setmax_host[1], 1u) + 7u) & ~7u;
    return 3ull * len + 64 + ((uint64_t)len / 1024 + 2) * stride * 2 * 2;
}

// Would the request, alone in a batch, fit a slot's arena and staging?  The
// dispatcher shrinks a batch that does not fit down to its first request, so
// a request that passes this test is always run.
bool fits_a_slot(const dfa_server *srv, const dfa_t *d, const uint8_t *in, size_t len) {
    const dfa_t *ds[1] = {d};
    const uint8_t *ins[1] = {in};
    const size_t lens[1] = {len};
    const size_t staging = std::min<size_t>(srv->opts.slot_bytes, 64u << 20);
    const bool packed = batch2_supported(ds, 1) &&
                        (srv->opts.lookahead >= 2 || len >= (256ull << 20));
    if (packed) {
        Batch2Plan p2;
        if (plan_batch2(ds, ins, lens, 1, 0, std::max<uint32_t>(srv->opts.lookahead, 1u), &p2))
            return false;
        return p2.total_bytes <= srv->opts.slot_bytes && p2.desc_bytes <= staging;
    }
    BatchPlan p;
    if (plan_batch(ds, ins, lens, 1, 0, &p)) return false;
    return p.total_bytes <= srv->opts.slot_bytes && p.desc_bytes <= staging;
}

void publish(dfa_server *srv, Slot &sl) {
    const uint64_t t = now_ns();
    std::lock_guard<std::mutex> lk(srv->mu);
    for (size_t k = 0; k < sl.reqs.size(); ++k) {
        Done dn;
        std::memcpy(&dn.r, sl.h_results + 4 * k, sizeof(dfa_result_t));
        dn.submit_ns = sl.reqs[k].submit_ns;
        dn.done_ns = t;
        srv->done.emplace(sl.reqs[k].ticket, dn);
        srv->stats.completed++;
    }
    srv->inflight_bytes -= sl.cost;
    srv->inflight_reqs -= (uint32_t)sl.reqs.size();
    sl.reqs.clear();
    sl.cost = 0;
    sl.busy = false;
    srv->cv_done.notify_all();
}

// Plans and launches the given requests on a slot.  Returns false (and
// leaves the slot idle) if the batch does not fit the slot's arena.
int launch_on_slot(dfa_server *srv, Slot &sl, std::vector<Request> &reqs, bool *fits) {
    *fits = true;
    if (reqs.size() == 1) {
        // a batch of one: the single-string path on the slot's stream, with
        // the slot's arena as its scratch (no descriptors to plan or upload,
        // the same kernels as dfa_match_ex)
        const Request &r = reqs[0];
        if (r.ready) {
            hipError_t we = hipStreamWaitEvent(sl.stream, r.ready, 0);
            if (we != hipSuccess) return hip_fail(we, "server: wait for the producer stream");
        }
        dfa_match_opts_t o{};
        o.lookahead = std::max<uint32_t>(srv->opts.lookahead, 1u);
        int rc = match_in_region(srv->dfas[r.id], r.in, r.len, DFA_Q0, &o, sl.stream,
                                 sl.d_results, static_cast<uint8_t *>(sl.arena), sl.arena_bytes);
        if (rc == DFA_OK) {
            hipError_t e = hipMemcpyAsync(sl.h_results, sl.d_results, sizeof(dfa_result_t),
                                          hipMemcpyDeviceToHost, sl.stream);
            if (e == hipSuccess) e = hipEventRecord(sl.done, sl.stream);
            if (e != hipSuccess) return hip_fail(e, "server: result readback");
            sl.reqs = std::move(reqs);
            sl.busy = true;
            std::lock_guard<std::mutex> lk(srv->mu);
            for (Request &q : sl.reqs)
                if (q.ready) {
                    srv->free_events.push_back(q.ready);
                    q.ready = nullptr;
                }
            return DFA_OK;
        }
        if (rc != DFA_E_TOOBIG) return rc;
        // larger than the arena on this path: the batch path decides
    }
    std::vector<const dfa_t *> ds(reqs.size());
    std::vector<const uint8_t *> ins(reqs.size());
    std::vector<size_t> lens(reqs.size());
    for (size_t k = 0; k < reqs.size(); ++k) {
        ds[k] = srv->dfas[reqs[k].id];
        ins[k] = reqs[k].in;
        lens[k] = reqs[k].len;
    }
    // the packed-pair batch when every DFA has a packed layout and either
    // multi-symbol lookahead is asked for or the batch is large; small
    // batches take the one-chunk-per-wavefront batch, which needs fewer
    // launches (lower latency)
    uint64_t batch_bytes = 0;
    for (size_t k = 0; k < reqs.size(); ++k) batch_bytes += reqs[k].len;
    const bool packed = batch2_supported(ds.data(), ds.size()) &&
                        (srv->opts.lookahead >= 2 || batch_bytes >= (256ull << 20));
    BatchPlan plan;
    Batch2Plan plan2;
    int rc = packed ? plan_batch2(ds.data(), ins.data(), lens.data(), reqs.size(), 0,
                                  std::max<uint32_t>(srv->opts.lookahead, 1u), &plan2)
                    : plan_batch(ds.data(), ins.data(), lens.data(), reqs.size(), 0, &plan);
    if (rc) return rc;
    const size_t total = packed ? plan2.total_bytes : plan.total_bytes;
    const size_t desc_bytes = packed ? plan2.desc_bytes : plan.desc_bytes;
    if (total > sl.arena_bytes || desc_bytes > sl.staging_bytes ||
        reqs.size() > srv->opts.max_batch) {
        *fits = false;
        return DFA_OK;
    }
    // inputs produced on the clients' streams: wait for them on this stream
    for (const Request &r : reqs)
        if (r.ready) {
            hipError_t we = hipStreamWaitEvent(sl.stream, r.ready, 0);
            if (we != hipSuccess) return hip_fail(we, "server: wait for the producer stream");
        }
    std::memcpy(sl.staging, packed ? plan2.desc.data() : plan.desc.data(), desc_bytes);
    hipError_t e = hipMemcpyAsync(sl.arena, sl.staging, desc_bytes, hipMemcpyHostToDevice,
                                  sl.stream);
    if (e != hipSuccess) return hip_fail(e, "server: descriptor upload");
    rc = packed ? launch_batch2(plan2, sl.arena, sl.stream, sl.d_results)
                : launch_batch(plan, sl.arena, sl.stream, sl.d_results);
    if (rc) return rc;
    e = hipMemcpyAsync(sl.h_results, sl.d_results, reqs.size() * sizeof(dfa_result_t),
                       hipMemcpyDeviceToHost, sl.stream);
    if (e == hipSuccess) e = hipEventRecord(sl.done, sl.stream);
    if (e != hipSuccess) return hip_fail(e, "server: result readback");
    sl.reqs = std::move(reqs);
    sl.busy = true;
    // the waits are enqueued: the producer events can be recorded again
    std::lock_guard<std::mutex> lk(srv->mu);
    for (Request &r : sl.reqs)
        if (r.ready) {
            srv->free_events.push_back(r.ready);
            r.ready = nullptr;
        }
    return DFA_OK;
}

void dispatcher(dfa_server *srv) {
    (void)hipSetDevice(srv->device);
    // the dispatcher sleeps in short waits between polls of its slots'
    // events; the default timer slack (50 us) would stretch every wait
    (void)prctl(PR_SET_TIMERSLACK, 1000UL, 0, 0, 0);
    while (true) {
        // 1. completions
        bool any_busy = false;
        for (auto &sl : srv->slots) {
            if (!sl.busy) continue;
            hipError_t q = hipEventQuery(sl.done);
            if (q == hipSuccess) {
                publish(srv, sl);
            } else if (q != hipErrorNotReady) {
                std::lock_guard<std::mutex> lk(srv->mu);
                srv->error = hip_fail(q, "server: batch failed");
                srv->stop = true;
            } else {
                any_busy = true;
            }
        }
        // 2. admission + dispatch into free slots
        std::unique_lock<std::mutex> lk(srv->mu);
        if (srv->stop && srv->pending.empty() && !any_busy) break;
        if (srv->stop && srv->error) break;
        bool admitted = false;
        for (auto &sl : srv->slots) {
            if (sl.busy || srv->pending.empty()) continue;
            std::vector<Request> take;
            uint64_t cost = 0;
            while (!srv->pending.empty() && take.size() < srv->opts.max_batch) {
                const Request &r = srv->pending.front();
                if (srv->inflight_reqs + take.size() + 1 > srv->opts.max_inflight) break;
                if (srv->inflight_bytes + cost + r.cost > srv->opts.budget_bytes && !take.empty())
                    break;
                if (srv->inflight_bytes + cost + r.cost > srv->opts.budget_bytes &&
                    srv->inflight_bytes > 0)
                    break;   // wait for memory to free up
                cost += r.cost;
                take.push_back(r);
                srv->pending.pop_front();
            }
            if (take.empty()) break;
            srv->inflight_bytes += cost;
            srv->inflight_reqs += (uint32_t)take.size();
            srv->stats.batches++;
            lk.unlock();
            // shrink the batch until it fits the slot's arena
            bool fits = false;
            int rc = DFA_OK;
            std::vector<Request> put_back;
            while (!take.empty()) {
                std::vector<Request> attempt = take;
                rc = launch_on_slot(srv, sl, attempt, &fits);
                if (rc || fits) break;
                put_back.insert(put_back.begin(), take.back());
                take.pop_back();
            }
            lk.lock();
            if (rc || take.empty()) {
                if (!rc) rc = fail(DFA_E_TOOBIG, "server: a request exceeds the slot arena");
                srv->error = rc;
                srv->stop = true;
                break;
            }
            admitted = true;
            sl.cost = 0;
            for (auto &r : take) sl.cost += r.cost;
            uint64_t back_cost = 0;
            for (auto it = put_back.rbegin(); it != put_back.rend(); ++it) {
                back_cost += it->cost;
                srv->pending.push_front(*it);
            }
            srv->inflight_bytes -= back_cost;
            srv->inflight_reqs -= (uint32_t)put_back.size();
        }
        if (!admitted) {
            // nothing to launch (no request, no free slot, or the budget or
            // in-flight cap holds the next request back until a batch
            // completes): wait briefly for submissions or completions
            srv->cv_submit.wait_for(lk, std::chrono::microseconds(any_busy ? 5 : 200));
        }
    }
}

}  // namespace

extern "C" int dfa_server_create(const dfa_server_opts_t *opts, dfa_server_t **out) {
    if (!out) return fail(DFA_E_INVAL, "dfa_server_create: out is NULL");
    *out = nullptr;
    std::unique_ptr<dfa_server> srv(new dfa_server());
    dfa_server_opts_t o{};
    if (opts) o = *opts;
    if (!o.budget_bytes) o.budget_bytes = 16ull << 30;
    if (!o.max_inflight) o.max_inflight = 4096;
    if (!o.streams) o.streams = 4;
    if (!o.max_batch) o.max_batch = 256;
    if (!o.slot_bytes) o.slot_bytes = 1ull << 30;
    if (o.lookahead > 64) return fail(DFA_E_INVAL, "dfa_server_create: lookahead above 64");
    srv->opts = o;
    hipError_t e = hipGetDevice(&srv->device);
    if (e != hipSuccess) return hip_fail(e, "dfa_server_create: hipGetDevice");
    srv->slots.resize(o.streams);
    for (auto &sl : srv->slots) {
        // non-blocking streams at the default priority
        e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
        if (e == hipSuccess) e = hipMalloc(&sl.arena, o.slot_bytes);
        sl.arena_bytes = o.slot_bytes;
        sl.staging_bytes = std::min<size_t>(o.slot_bytes, 64u << 20);
        if (e == hipSuccess) e = hipHostMalloc(&sl.staging, sl.staging_bytes, hipHostMallocDefault);
        if (e == hipSuccess) e = hipMalloc(&sl.d_results, (size_t)o.max_batch * sizeof(dfa_result_t));
        if (e == hipSuccess)
            e = hipHostMalloc((void **)&sl.h_results, (size_t)o.max_batch * sizeof(dfa_result_t),
                              hipHostMallocDefault);
        if (e != hipSuccess) {
            dfa_server_destroy(srv.release());
            return fail(DFA_E_NOMEM, "dfa_server_create: slot allocation failed");
        }
    }
    srv->worker = std::thread(dispatcher, srv.get());
    *out = srv.release();
    return DFA_OK;
}

extern "C" int dfa_server_register(dfa_server_t *srv, const dfa_t *d, uint32_t *id) {
    if (!srv || !d || !id) return fail(DFA_E_INVAL, "dfa_server_register: NULL argument");
    std::lock_guard<std::mutex> lk(srv->mu);
    *id = (uint32_t)srv->dfas.size();
    srv->dfas.push_back(d);
    return DFA_OK;
}

namespace {
int submit(dfa_server_t *srv, uint32_t id, const uint8_t *d_input, size_t len,
           hipStream_t producer, bool after, uint64_t *ticket) {
    if (!srv || !ticket || (len && !d_input)) return fail(DFA_E_INVAL, "dfa_server_submit: NULL argument");
    const dfa_t *d = nullptr;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        if (srv->error) return srv->error;
        if (srv->stop) return fail(DFA_E_INVAL, "dfa_server_submit: server is stopping");
        if (id >= srv->dfas.size()) return fail(DFA_E_INVAL, "dfa_server_submit: unknown DFA id");
        d = srv->dfas[id];
    }
    Request r;
    r.id = id;
    r.in = d_input;
    r.len = len;
    r.cost = request_cost(d, len);
    if (r.cost > srv->opts.budget_bytes)
        return fail(DFA_E_TOOBIG, "dfa_server_submit: request exceeds the memory budget");
    if (!fits_a_slot(srv, d, d_input, len))
        return fail(DFA_E_TOOBIG, "dfa_server_submit: request exceeds a slot's arena (slot_bytes)");
    if (after) {
        {
            std::lock_guard<std::mutex> lk(srv->mu);
            if (!srv->free_events.empty()) {
                r.ready = srv->free_events.back();
                srv->free_events.pop_back();
            }
        }
        hipError_t e = r.ready ? hipSuccess
                               : hipEventCreateWithFlags(&r.ready, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventRecord(r.ready, producer);
        if (e != hipSuccess) {
            if (r.ready) {
                std::lock_guard<std::mutex> lk(srv->mu);
                srv->free_events.push_back(r.ready);
            }
            return hip_fail(e, "dfa_server_submit_after: hipEventRecord");
        }
    }
    std::lock_guard<std::mutex> lk(srv->mu);
    r.submit_ns = now_ns();
    r.ticket = srv->next_ticket++;
    srv->pending.push_back(r);
    srv->stats.submitted++;
    srv->stats.bytes += len;
    *ticket = r.ticket;
    srv->cv_submit.notify_one();
    return DFA_OK;
}
}  // namespace

extern "C" int dfa_server_submit(dfa_server_t *srv, uint32_t id, const uint8_t *d_input, size_t len,
                                 uint64_t *ticket) {
    return submit(srv, id, d_input, len, nullptr, false, ticket);
}

extern "C" int dfa_server_submit_after(dfa_server_t *srv, uint32_t id, const uint8_t *d_input,
                                       size_t len, void *producer_stream, uint64_t *ticket) {
    return submit(srv, id, d_input, len, (hipStream_t)producer_stream, true, ticket);
}

extern "C" int dfa_server_poll(dfa_server_t *srv, uint64_t ticket, dfa_result_t *out) {
    if (!srv || !out) return fail(DFA_E_INVAL, "dfa_server_poll: NULL argument");
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->done.find(ticket);
    if (it == srv->done.end()) return srv->error ? srv->error : DFA_E_NOTREADY;
    *out = it->second.r;
    srv->done.erase(it);
    return DFA_OK;
}

extern "C" int dfa_server_wait(dfa_server_t *srv, uint64_t ticket, dfa_result_t *out) {
    if (!srv || !out) return fail(DFA_E_INVAL, "dfa_server_wait: NULL argument");
    std::unique_lock<std::mutex> lk(srv->mu);
    while (true) {
        auto it = srv->done.find(ticket);
        if (it != srv->done.end()) {
            *out = it->second.r;
            srv->done.erase(it);
            return DFA_OK;
        }
        if (srv->error) return srv->error;
        srv->cv_done.wait_for(lk, std::chrono::milliseconds(10));
    }
}

extern "C" int dfa_server_drain(dfa_server_t *srv, dfa_server_done_t *out, size_t cap,
                                size_t *count) {
    if (!srv || !count || (cap && !out)) return fail(DFA_E_INVAL, "dfa_server_drain: NULL argument");
    std::lock_guard<std::mutex> lk(srv->mu);
    size_t k = 0;
    for (auto it = srv->done.begin(); it != srv->done.end() && k < cap;) {
        out[k].ticket = it->first;
        out[k].result = it->second.r;
        out[k].submit_ns = it->second.submit_ns;
        out[k].done_ns = it->second.done_ns;
        ++k;
        it = srv->done.erase(it);
    }
    *count = k;
    return srv->error;
}

extern "C" int dfa_server_stats(dfa_server_t *srv, dfa_server_stats_t *out) {
    if (!srv || !out) return fail(DFA_E_INVAL, "dfa_server_stats: NULL argument");
    std::lock_guard<std::mutex> lk(srv->mu);
    *out = srv->stats;
    out->inflight = srv->inflight_reqs;
    out->pending = srv->pending.size();
    return DFA_OK;
}

extern "C" void dfa_server_destroy(dfa_server_t *srv) {
    if (!srv) return;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
        srv->cv_submit.notify_all();
    }
    if (srv->worker.joinable()) srv->worker.join();
    for (auto &r : srv->pending)
        if (r.ready) (void)hipEventDestroy(r.ready);
    for (hipEvent_t ev : srv->free_events) (void)hipEventDestroy(ev);
    for (auto &sl : srv->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
        if (sl.arena) (void)hipFree(sl.arena);
        if (sl.d_results) (void)hipFree(sl.d_results);
        if (sl.staging) (void)hipHostFree(sl.staging);
        if (sl.h_results) (void)hipHostFree(sl.h_results);
    }
    delete srv;
}
