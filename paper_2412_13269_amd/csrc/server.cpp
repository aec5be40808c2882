// Served form of the private query: a continuous-batching request server.
//
// One scheduler thread per server.  Requests wait in a FIFO; the head is
// admitted as soon as a slot (a stream with its own key-switching scratch) is
// free and its work registers fit in the arena.  Admission carves the
// registers out of the arena, launches the whole op list on the slot's stream
// and enqueues a host function behind it; that function stamps the completion
// time and hands the slot back to the scheduler, which returns the memory to
// the arena and admits whatever now fits.  The scheduler never holds its lock
// across a HIP call, and the host function makes none.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <string>
#include <thread>
#include <vector>

#include "internal.h"

using namespace pfx;

namespace {

using Clock = std::chrono::steady_clock;

constexpr size_t kAlign = 256;
constexpr uint32_t kMaxSlots = 16;

// First-fit allocator over one device block; free ranges coalesce on release.
struct Arena {
    char *base = nullptr;
    size_t size = 0;
    std::map<size_t, size_t> free_;   // offset -> length

    void init(char *b, size_t n) {
        base = b;
        size = n;
        free_.clear();
        if (n) free_[0] = n;
    }
    static size_t round(size_t n) { return (n + kAlign - 1) / kAlign * kAlign; }
    bool fits(size_t n) const {
        n = round(n);
        for (auto &kv : free_)
            if (kv.second >= n) return true;
        return false;
    }
    bool alloc(size_t n, size_t &off) {
        n = round(n);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            off = it->first;
            const size_t rest = it->second - n;
            free_.erase(it);
            if (rest) free_[off + n] = rest;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t n) {
        n = round(n);
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + n == next->first) {
            n += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += n;
                return;
            }
        }
        free_[off] = n;
    }
};

enum class State { Queued, Running, Done };

struct Request {
    uint64_t ticket = 0;
    std::vector<pfx_op> ops;
    size_t n_regs = 0, n_inputs = 0;
    std::vector<pfx_ct *> regs;          // inputs (borrowed), then views into the arena
    std::vector<const pfx_pt *> pts;
    int32_t out_reg = -1;
    pfx_ct *out = nullptr;
    uint32_t reg_limbs = 0;
    std::vector<uint8_t> reg_degree;     // capacity degree of each work register
    size_t footprint = 0;
    size_t arena_off = 0;
    int slot = -1;
    State state = State::Queued;
    pfx_status status = PFX_OK;
    std::string error;
    Clock::time_point t_submit, t_admit, t_done;
};

struct Callback {
    pfx_server *srv;
    int slot;
};

}  // namespace

struct pfx_server {
    pfx_ctx *ctx = nullptr;
    const pfx_swk *rlk = nullptr;
    std::vector<const pfx_swk *> gks;
    size_t budget = 0, scratch = 0;
    int max_batch = 1;                   // largest batched launch inside a request
    void *arena_mem = nullptr;
    Arena arena;
    std::vector<void *> streams;
    std::vector<Request *> running;      // per slot; nullptr = free
    std::vector<Callback> callbacks;     // per slot, argument of the completion host function
    std::deque<Request *> queue;
    std::map<uint64_t, Request *> tickets;
    std::vector<std::pair<int, Clock::time_point>> finished;
    uint64_t next_ticket = 1, submitted = 0, completed = 0;
    size_t in_use = 0, peak = 0;
    uint32_t n_running = 0, peak_running = 0;
    bool stop = false;
    std::mutex mu;
    std::condition_variable wake;        // scheduler
    std::condition_variable done;        // pollers
    std::thread worker;
};

namespace {

void on_complete(void *arg) {
    Callback *cb = static_cast<Callback *>(arg);
    pfx_server *s = cb->srv;
    const Clock::time_point now = Clock::now();
    std::lock_guard<std::mutex> g(s->mu);
    s->finished.emplace_back(cb->slot, now);
    s->wake.notify_one();
}

int free_slot(const pfx_server *s) {
    for (size_t i = 0; i < s->running.size(); ++i)
        if (!s->running[i]) return (int)i;
    return -1;
}

bool can_admit(const pfx_server *s) {
    return !s->stop && !s->queue.empty() && free_slot(s) >= 0 && s->arena.fits(s->queue.front()->footprint);
}

// Called with the lock held: carve the registers, mark the slot.
void admit(pfx_server *s, Request *r, int slot) {
    pfx_ctx *c = s->ctx;
    s->arena.alloc(r->footprint, r->arena_off);
    r->slot = slot;
    r->state = State::Running;
    r->t_admit = Clock::now();
    const size_t poly_doubles = (size_t)r->reg_limbs * c->N;
    double *next = reinterpret_cast<double *>(s->arena.base + r->arena_off);
    for (size_t i = r->n_inputs; i < r->n_regs; ++i) {
        pfx_ct *v = new pfx_ct;
        v->ctx = c;
        v->uid = next_uid();
        v->cap_limbs = r->reg_limbs;
        v->cap_degree = r->reg_degree[i];
        v->d = next;
        v->owns = false;
        next += (v->cap_degree + 1) * poly_doubles;
        r->regs[i] = v;
    }
    s->running[slot] = r;
    s->in_use += Arena::round(r->footprint);
    s->peak = std::max(s->peak, s->in_use);
    s->peak_running = std::max(s->peak_running, ++s->n_running);
}

// Called without the lock: every launch of the request, then the completion hook.
void launch(pfx_server *s, Request *r) {
    pfx_ctx *c = s->ctx;
    void *st = s->streams[r->slot];
    pfx_status st_run = run_ops(c, r->ops.data(), r->ops.size(), r->regs.data(), r->n_regs, r->n_inputs,
                                r->pts.data(), r->pts.size(), s->rlk, s->gks.data(), s->gks.size(), st,
                                s->max_batch);   // the slot's batch region was reserved for this size
    std::string err = st_run ? pfx_last_error() : "";
    if (!st_run) {
        st_run = pfx_ct_copy(c, r->regs[r->out_reg], r->out, st);
        if (st_run) err = std::string("output: ") + pfx_last_error();
    }
    {
        std::lock_guard<std::mutex> g(s->mu);
        r->status = st_run;
        r->error = err;
    }
    Callback *cb = &s->callbacks[r->slot];
    if (hipLaunchHostFunc((hipStream_t)st, on_complete, cb) != hipSuccess) {
        (void)hipStreamSynchronize((hipStream_t)st);   // no hook: retire after the stream has drained
        on_complete(cb);
    }
}

// Called with the lock held, after the slot's stream has passed the request.
void retire(pfx_server *s, int slot, Clock::time_point t) {
    Request *r = s->running[slot];
    if (!r) return;
    for (size_t i = r->n_inputs; i < r->n_regs; ++i) delete r->regs[i];
    s->arena.release(r->arena_off, r->footprint);
    s->in_use -= Arena::round(r->footprint);
    s->running[slot] = nullptr;
    --s->n_running;
    r->t_done = t;
    r->state = State::Done;
    ++s->completed;
}

void scheduler(pfx_server *s) {
    (void)hipSetDevice(s->ctx->device);   // launches below report their own errors
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        for (auto &f : s->finished) retire(s, f.first, f.second);
        if (!s->finished.empty()) {
            s->finished.clear();
            s->done.notify_all();
        }
        if (s->stop && s->n_running == 0) break;
        if (can_admit(s)) {
            Request *r = s->queue.front();
            s->queue.pop_front();
            admit(s, r, free_slot(s));
            lk.unlock();
            launch(s, r);
            lk.lock();
            continue;
        }
        s->wake.wait(lk, [s] { return !s->finished.empty() || can_admit(s) || (s->stop && s->n_running == 0); });
    }
}

double seconds(Clock::time_point a, Clock::time_point b) { return std::chrono::duration<double>(b - a).count(); }

}  // namespace

#define REQUIRE(cond, code, msg) \
    do {                         \
        if (!(cond)) return fail(code, msg); \
    } while (0)

extern "C" {

pfx_status pfx_server_create(pfx_ctx *c, size_t hbm_budget, uint32_t slots, uint32_t max_batch,
                             const pfx_swk *rlk, const pfx_swk *const *gks, size_t n_gks, pfx_server **out) {
    REQUIRE(c && out, PFX_EINVAL, "null argument");
    REQUIRE(slots >= 1 && slots <= kMaxSlots, PFX_EINVAL, "slots must be in [1, 16]");
    REQUIRE(max_batch >= 1 && max_batch <= (uint32_t)kMaxBatch, PFX_EINVAL, "max_batch must be in [1, 8]");
    REQUIRE(!rlk || rlk->ctx == c, PFX_EINVAL, "relinearisation key of another context");
    for (size_t i = 0; i < n_gks; ++i) REQUIRE(gks[i] && gks[i]->ctx == c, PFX_EINVAL, "bad Galois key");
    const size_t per_slot = Arena::round(ws_bytes(c)) + (max_batch > 1 ? Arena::round(batch_ws_bytes(c, max_batch)) : 0);
    const size_t scratch = (size_t)slots * per_slot;
    REQUIRE(hbm_budget > scratch, PFX_ENOMEM,
            "budget of " + std::to_string(hbm_budget) + " bytes does not cover the slots' scratch (" +
                std::to_string(scratch) + " bytes)");
    if (hipSetDevice(c->device) != hipSuccess) return fail(PFX_EDEVICE, "hipSetDevice failed");
    std::unique_ptr<pfx_server> s(new pfx_server);
    s->ctx = c;
    s->rlk = rlk;
    s->gks.assign(gks, gks + n_gks);
    s->budget = hbm_budget;
    s->scratch = scratch;
    s->max_batch = (int)max_batch;
    const size_t arena_bytes = (hbm_budget - scratch) / kAlign * kAlign;
    if (arena_bytes) {
        pfx_status r = dmalloc(c, &s->arena_mem, arena_bytes);
        if (r) return r;
    }
    s->arena.init(static_cast<char *>(s->arena_mem), arena_bytes);
    s->running.assign(slots, nullptr);
    s->callbacks.resize(slots);
    for (uint32_t i = 0; i < slots; ++i) {
        void *st = nullptr;
        pfx_status r = pfx_stream_create(c, &st);
        if (!r) {
            s->streams.push_back(st);
            r = ws_reserve(c, (hipStream_t)st);
            if (!r && max_batch > 1) r = batch_ws_reserve(c, (hipStream_t)st, (int)max_batch);
        }
        if (r) {
            for (void *x : s->streams) pfx_stream_destroy(c, x);
            dfree(s->arena_mem);
            return r;
        }
        s->callbacks[i] = Callback{s.get(), (int)i};
    }
    s->worker = std::thread(scheduler, s.get());
    *out = s.release();
    return PFX_OK;
}

pfx_status pfx_server_submit(pfx_server *s, const pfx_request *rq, uint64_t *ticket) {
    REQUIRE(s && rq && ticket, PFX_EINVAL, "null argument");
    REQUIRE(rq->ops || rq->n_ops == 0, PFX_EINVAL, "null op list");
    REQUIRE(rq->n_inputs >= 1 && rq->n_inputs <= rq->n_regs, PFX_EINVAL, "need 1 <= n_inputs <= n_regs");
    REQUIRE(rq->inputs && rq->out, PFX_EINVAL, "null inputs or output");
    REQUIRE(rq->out_reg >= (int32_t)rq->n_inputs && (size_t)rq->out_reg < rq->n_regs, PFX_EINVAL,
            "out_reg must be a work register");
    REQUIRE(rq->out->ctx == s->ctx, PFX_EINVAL, "output of another context");
    REQUIRE(rq->n_pts == 0 || rq->pts, PFX_EINVAL, "null plaintext array");
    std::unique_ptr<Request> r(new Request);
    r->ops.assign(rq->ops, rq->ops + rq->n_ops);
    for (size_t i = 0; i < rq->n_ops; ++i) {
        const pfx_op &o = rq->ops[i];
        if (o.code == PFX_OP_LANE) continue;     // run on the slot's stream, markers ignored
        REQUIRE(o.dst >= (int32_t)rq->n_inputs && (size_t)o.dst < rq->n_regs, PFX_EINVAL,
                "op " + std::to_string(i) + ": destination is not a work register");
        REQUIRE(o.a >= 0 && (size_t)o.a < rq->n_regs, PFX_EINVAL,
                "op " + std::to_string(i) + ": register index out of range");
    }
    r->n_regs = rq->n_regs;
    r->n_inputs = rq->n_inputs;
    r->regs.assign(rq->n_regs, nullptr);
    for (size_t i = 0; i < rq->n_inputs; ++i) {
        const pfx_ct *x = rq->inputs[i];
        REQUIRE(x && x->ctx == s->ctx && x->n_limbs >= 1, PFX_EINVAL,
                "input " + std::to_string(i) + " is null, empty or of another context");
        r->regs[i] = const_cast<pfx_ct *>(x);
        r->reg_limbs = std::max(r->reg_limbs, x->n_limbs);
    }
    for (size_t i = 0; i < rq->n_pts; ++i) REQUIRE(rq->pts[i], PFX_EINVAL, "null plaintext");
    r->pts.assign(rq->pts, rq->pts + rq->n_pts);
    r->out_reg = rq->out_reg;
    r->out = rq->out;
    r->reg_degree.assign(rq->n_regs, 1);
    size_t polys = 0;
    for (size_t i = rq->n_inputs; i < rq->n_regs; ++i) {
        if (rq->reg_degree) {
            REQUIRE(rq->reg_degree[i] == 1 || rq->reg_degree[i] == 2, PFX_EINVAL,
                    "register " + std::to_string(i) + ": degree must be 1 or 2");
            r->reg_degree[i] = rq->reg_degree[i];
        }
        polys += r->reg_degree[i] + 1;
    }
    r->footprint = polys * (size_t)r->reg_limbs * s->ctx->N * sizeof(double);
    REQUIRE(Arena::round(r->footprint) <= s->arena.size, PFX_ENOMEM,
            "footprint of " + std::to_string(r->footprint) + " bytes exceeds the arena (" +
                std::to_string(s->arena.size) + " bytes)");
    std::lock_guard<std::mutex> g(s->mu);
    REQUIRE(!s->stop, PFX_EINVAL, "server is stopping");
    r->t_submit = Clock::now();
    r->ticket = s->next_ticket++;
    *ticket = r->ticket;
    s->tickets[r->ticket] = r.get();
    s->queue.push_back(r.release());
    ++s->submitted;
    s->wake.notify_one();
    return PFX_OK;
}

pfx_status pfx_server_poll(pfx_server *s, uint64_t ticket, int wait, pfx_request_info *info) {
    REQUIRE(s && info, PFX_EINVAL, "null argument");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->tickets.find(ticket);
    REQUIRE(it != s->tickets.end(), PFX_EINVAL, "unknown ticket " + std::to_string(ticket));
    Request *r = it->second;
    if (r->state != State::Done) {
        if (!wait) return PFX_EBUSY;
        s->done.wait(lk, [r] { return r->state == State::Done; });
    }
    std::memset(info, 0, sizeof(*info));
    info->status = r->status;
    info->slot = r->slot;
    info->footprint = r->footprint;
    info->queued_s = seconds(r->t_submit, r->t_admit);
    info->latency_s = seconds(r->t_submit, r->t_done);
    std::strncpy(info->error, r->error.c_str(), sizeof(info->error) - 1);
    s->tickets.erase(it);
    delete r;
    return PFX_OK;
}

pfx_status pfx_server_stats_get(pfx_server *s, pfx_server_stats *st) {
    REQUIRE(s && st, PFX_EINVAL, "null argument");
    std::lock_guard<std::mutex> g(s->mu);
    st->submitted = s->submitted;
    st->completed = s->completed;
    st->queued = s->queue.size();
    st->running = s->n_running;
    st->budget = s->budget;
    st->scratch_bytes = s->scratch;
    st->arena_bytes = s->arena.size;
    st->bytes_in_use = s->in_use;
    st->peak_bytes = s->peak;
    st->slots = (uint32_t)s->running.size();
    st->peak_running = s->peak_running;
    return PFX_OK;
}

void pfx_server_destroy(pfx_server *s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
        s->wake.notify_one();
    }
    s->worker.join();
    for (void *st : s->streams) pfx_stream_destroy(s->ctx, st);   // also waits for the host functions
    for (auto &kv : s->tickets) delete kv.second;                 // queued, finished and unpolled
    dfree(s->arena_mem);
    delete s;
}

}  // extern "C"
