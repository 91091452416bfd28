// pcg_server.hip -- continuously batching solve server (pcg_server_* ABI).
//
// Requests enter a FIFO queue.  A scheduler thread owned by the server
// admits the head of the queue whenever a batch slot and enough of the HBM
// arena are free (first-fit sub-allocation of the caller's arena), so new
// systems join the running batch at the next launch boundary; after every
// launch of K passes it retires finished systems, frees their memory and
// completes their tickets.  Admission never skips the queue head, so a large
// request cannot starve.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "pcg.h"
#include "pcg_batch_engine.h"

using namespace pcg;

namespace {

using Clock = std::chrono::steady_clock;

// First-fit allocator of 256-byte aligned ranges of [0, size).
class Arena {
public:
    void init(size_t size)
    {
        free_.clear();
        if (size) free_[0] = size;
    }
    bool alloc(size_t bytes, size_t *off)
    {
        bytes = (bytes + 255) & ~size_t(255);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes, at = it->first + bytes;
                free_.erase(it);
                if (rest) free_[at] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = (bytes + 255) & ~size_t(255);
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);  // merge with the following range
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {  // and the preceding one
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t largest() const
    {
        size_t m = 0;
        for (auto &f : free_) m = std::max(m, f.second);
        return m;
    }
    size_t total_free() const
    {
        size_t t = 0;
        for (auto &f : free_) t += f.second;
        return t;
    }

private:
    std::map<size_t, size_t> free_;  // offset -> length
};

enum ReqState { Q_QUEUED, Q_RUNNING, Q_DONE, Q_FAILED };

struct Request {
    uint64_t ticket;
    pcg_operator op;
    pcg_options opt;
    const double *b;
    double *x;
    Clock::time_point t_submit;
    ReqState state = Q_QUEUED;
    int slot = -1;
    int admitted_at = 0;  // server launches issued before the request joined the batch
    size_t off = 0, bytes = 0;
    pcg_result res{};
    pcg_status err = PCG_OK;
};

}  // namespace

struct pcg_server_ {
    char *arena = nullptr;
    size_t arena_bytes = 0;
    int max_slots = 0;
    hipStream_t stream = nullptr;
    size_t tables_bytes = 0;
    int prec = -1;  // fixed by the first request
    std::unique_ptr<BatchEngine> eng;
    Arena heap;
    std::mutex mu;
    std::condition_variable cv_done, cv_work;
    std::deque<Request *> queue;
    std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
    std::unordered_map<int, Request *> running;  // slot -> request
    uint64_t next_ticket = 1;
    bool stop = false;
    std::string error;
    std::thread sched;
    int64_t n_submitted = 0, n_completed = 0, n_failed = 0;
    int max_running = 0;       // most systems resident in one launch
    int launches = 0;          // launches issued by the scheduler
    int fail_at_launch = -1;   // fault injection (PCG_SERVER_FAIL_AT_LAUNCH): that launch fails

    void loop();
    bool admit_head();
    void fail_running(pcg_status st);
};

// A launch failed: every running request fails with `st`.  The stream is
// drained first, so no pass of the failed launch still touches their memory,
// then their batch slots and arena ranges are returned, so the server keeps
// serving the requests that follow.  Called with mu held.
void pcg_server_::fail_running(pcg_status st)
{
    error = g_last_error;
    (void)hipStreamSynchronize(stream);
    for (auto &kv : running) {
        Request *r = kv.second;
        eng->release(kv.first);
        heap.release(r->off, r->bytes);
        r->state = Q_FAILED;
        r->err = st;
        ++n_failed;
    }
    running.clear();
    cv_done.notify_all();
}

bool pcg_server_::admit_head()
{
    // called with mu held
    if (queue.empty() || (int)running.size() >= max_slots) return false;
    Request *r = queue.front();
    size_t off;
    if (!heap.alloc(r->bytes, &off)) return false;
    int slot = -1;
    const pcg_status st = eng->admit(&r->op, &r->opt, r->b, r->x, arena + tables_bytes + off, &slot);
    queue.pop_front();
    if (st != PCG_OK) {
        heap.release(off, r->bytes);
        r->state = Q_FAILED;
        r->err = st;
        ++n_failed;
        cv_done.notify_all();
        return true;
    }
    r->off = off;
    r->slot = slot;
    r->admitted_at = launches;
    r->state = Q_RUNNING;
    running[slot] = r;
    return true;
}

void pcg_server_::loop()
{
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        while (admit_head()) {
        }
        if (stop && running.empty()) return;
        if (running.empty()) {
            cv_work.wait(lk, [&] { return stop || !queue.empty(); });
            continue;
        }
        max_running = std::max(max_running, (int)running.size());
        const bool inject = launches == fail_at_launch;
        lk.unlock();
        pcg_status st;
        if (inject) {
            g_last_error = "injected failure of server launch " + std::to_string(fail_at_launch);
            st = PCG_ERR_HIP;
        } else {
            st = eng->step(nullptr);
        }
        lk.lock();
        ++launches;
        if (st != PCG_OK) {
            // a device error ends every running request
            fail_running(st);
            continue;
        }
        for (auto it = running.begin(); it != running.end();) {
            const int slot = it->first;
            Request *r = it->second;
            if (!eng->done(slot)) {
                ++it;
                continue;
            }
            eng->result(slot, &r->res);
            if (r->opt.history_cap > 0) eng->copy_history(slot, r->opt.history, r->opt.history_cap);
            r->res.seconds = std::chrono::duration<double>(Clock::now() - r->t_submit).count();
            r->res.admitted_at = r->admitted_at;
            r->res.launches = launches - r->admitted_at;
            eng->release(slot);
            heap.release(r->off, r->bytes);
            r->state = Q_DONE;
            ++n_completed;
            it = running.erase(it);
        }
        cv_done.notify_all();
    }
}

extern "C" pcg_status pcg_server_create(pcg_server *out, void *arena, size_t arena_bytes, int32_t max_slots,
                                        void *hip_stream)
{
    if (!out) return invalid("server out-pointer is null");
    *out = nullptr;
    if (!arena || ((uintptr_t)arena % 256)) return invalid("arena must be non-null and 256-byte aligned");
    if (max_slots < 1 || max_slots > 65535) return invalid("max_slots must be in [1, 65535]");
    // every tile of an admitted system needs at least a 512-unknown tile of
    // its vectors (>= 16 KiB), which bounds the item table
    const int64_t max_items = (int64_t)(arena_bytes / (16 * 1024)) + max_slots;
    const size_t tb = (BatchEngine::table_bytes(max_slots, max_items) + 255) & ~size_t(255);
    if (arena_bytes <= tb) return invalid("arena too small for the server tables");
    auto *s = new pcg_server_();
    s->arena = (char *)arena;
    s->arena_bytes = arena_bytes;
    s->max_slots = max_slots;
    s->stream = (hipStream_t)hip_stream;
    s->tables_bytes = tb;
    s->heap.init(arena_bytes - tb);
    s->prec = -1;  // the engine is set up for the first request's precision
    if (const char *f = std::getenv("PCG_SERVER_FAIL_AT_LAUNCH")) s->fail_at_launch = std::atoi(f);
    s->sched = std::thread([s] { s->loop(); });
    *out = s;
    return PCG_OK;
}

extern "C" pcg_status pcg_submit(pcg_server s, const pcg_operator *op, const pcg_options *opt, const double *b,
                                 double *x, uint64_t *ticket)
{
    if (!s) return PCG_ERR_STATE;
    if (!ticket) return invalid("ticket is null");
    pcg_status st = validate_options(opt);
    if (st) return st;
    if ((st = validate_operator(op, opt->prec))) return st;
    if (opt->method == PCG_CG || opt->method == PCG_PIPE_VAR_SHIFT || opt->method == PCG_PIPE_RR)
        return invalid("the server runs the constant-shift pipelined methods (PCG_PIPE, PCG_PIPE_SHIFT)");
    if (opt->flags) return invalid("the server takes no option flags");
    if (!b || !x || b == x) return invalid("b and x must be non-null and distinct");
    BatchEngine::SysLayout L;
    BatchEngine::system_layout(op, opt, &L);
    std::unique_ptr<Request> r(new Request());
    r->op = *op;
    r->opt = *opt;
    r->b = b;
    r->x = x;
    r->bytes = L.bytes;
    r->t_submit = Clock::now();
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return PCG_ERR_STATE;
    if (s->prec < 0) {
        // bind the engine's precision to the first request (nothing runs yet)
        s->eng.reset(new BatchEngine());
        const int64_t max_items = (int64_t)(s->arena_bytes / (16 * 1024)) + s->max_slots;
        // the launch shape of the whole run comes from the first request
        // (0: the engine's defaults), e.g. from pcg_batch_tune on a sample
        if ((st = s->eng->init(s->arena, s->max_slots, max_items, opt->prec, s->stream, opt->iters_per_launch)))
            return st;
        if (opt->grid_blocks) s->eng->set_pass_grid(opt->grid_blocks);
        s->prec = opt->prec;
    } else if (opt->prec != s->prec) {
        return invalid("every request of a server must use the precision of its first request");
    }
    if (((L.bytes + 255) & ~size_t(255)) > s->arena_bytes - s->tables_bytes) return PCG_ERR_BUDGET;
    r->ticket = s->next_ticket++;
    ++s->n_submitted;
    *ticket = r->ticket;
    s->queue.push_back(r.get());
    s->reqs[r->ticket] = std::move(r);
    s->cv_work.notify_one();
    return PCG_OK;
}

static pcg_status take_result(pcg_server s, uint64_t ticket, pcg_result *res, bool block)
{
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return PCG_ERR_STATE;
    Request *r = it->second.get();
    if (block) s->cv_done.wait(lk, [&] { return r->state == Q_DONE || r->state == Q_FAILED; });
    if (r->state == Q_QUEUED || r->state == Q_RUNNING) return PCG_PENDING;
    const pcg_status err = r->state == Q_FAILED ? r->err : PCG_OK;
    if (res) *res = r->res;
    s->reqs.erase(it);
    return err;
}

extern "C" pcg_status pcg_poll(pcg_server s, uint64_t ticket, pcg_result *res)
{
    if (!s) return PCG_ERR_STATE;
    return take_result(s, ticket, res, false);
}

extern "C" pcg_status pcg_wait(pcg_server s, uint64_t ticket, pcg_result *res)
{
    if (!s) return PCG_ERR_STATE;
    return take_result(s, ticket, res, true);
}

extern "C" pcg_status pcg_server_info(pcg_server s, pcg_server_stats *out)
{
    if (!s) return PCG_ERR_STATE;
    if (!out) return invalid("stats is null");
    std::lock_guard<std::mutex> lk(s->mu);
    std::memset(out, 0, sizeof(*out));
    out->submitted = s->n_submitted;
    out->completed = s->n_completed;
    out->failed = s->n_failed;
    out->queued = (int32_t)s->queue.size();
    out->running = (int32_t)s->running.size();
    out->max_running = s->max_running;
    out->launches = s->launches;
    out->arena_bytes = s->arena_bytes - s->tables_bytes;
    out->arena_free = s->heap.total_free();
    out->arena_largest_free = s->heap.largest();
    return PCG_OK;
}

extern "C" pcg_status pcg_server_destroy(pcg_server s)
{
    if (!s) return PCG_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        // queued requests that never started are failed; running ones finish
        for (Request *r : s->queue) {
            r->state = Q_FAILED;
            r->err = PCG_ERR_STATE;
        }
        s->queue.clear();
        s->cv_work.notify_all();
        s->cv_done.notify_all();
    }
    if (s->sched.joinable()) s->sched.join();
    delete s;
    return PCG_OK;
}
