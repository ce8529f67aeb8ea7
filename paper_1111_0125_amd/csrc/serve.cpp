// Serving loop: continuous batching of solve requests.
//
// stag_solver_submit copies a request (gauge, mass, tolerance, inner
// precision, 1..16 right-hand sides) into a queue and returns a ticket. One
// scheduler thread per context:
//   * admits queued requests in arrival order into a batch for their
//     (gauge, inner precision): a slot engine with its own stream, created
//     when HBM allows (the context budget covers batches and result buffers;
//     a request that does not fit waits, and idle batches are released to
//     make room);
//   * starts admitted right-hand sides in free slots at the next block
//     boundary while the other slots are mid-solve;
//   * keeps up to two K-iteration blocks in flight per batch, processes each
//     poll, harvests finished slots into the request's device result buffer
//     and frees the slots.
// Batches of different gauges run on different streams and overlap on the
// device. stag_solver_poll returns PENDING until every right-hand side of a
// ticket has finished, then copies x and the per-RHS stats out.
//
// A right-hand side's arithmetic does not depend on the other slots, the
// kernel block size or when it started, so its result is the same bits alone
// and in any mix.
//
// fp16-storage requests on a gauge that also holds fp32 links: a right-hand
// side whose fp16 inner iteration stalls at its precision floor (ESTALL after
// a few stall updates without progress) is handed over, as stag_cg_solve
// does: it re-enters the queue ahead of new requests as a continuation that
// starts from its current x in the gauge's fp32 batch (no stall restarts);
// its statistics add up both passes and report inner_final = F32.
#include <chrono>
#include <cmath>
#include <cstring>
#include <algorithm>
#include <deque>
#include <limits>
#include <unordered_map>

#include "internal.h"

namespace stag {

using Clock = std::chrono::steady_clock;

struct Ticket {
    stag_ticket id = 0;
    const stag_gauge* g = nullptr;
    double mass = 0, tol = 0;
    int nrhs = 0, prec = 0;
    std::vector<double> b;          // host copy, complex128 [nrhs][Vh][3]
    void* x_dev = nullptr;          // device result, canonical fp64 field layout
    size_t x_bytes = 0;
    std::vector<stag_cg_stats> stats;
    std::vector<stag_cg_stats> first;  // per RHS: the fp16 pass of an escalated RHS
    std::vector<char> escalated;       // per RHS: continued in fp32 from its x
    Clock::time_point t_submit, t_done;
    int remaining = 0;
    // one event per harvested right-hand side, recorded on its batch's stream
    // after its result copy (an escalated right-hand side finishes in another
    // batch than the others, on another stream)
    std::vector<hipEvent_t> copy_evs;
    bool finishing = false;         // all slots harvested, waiting for copy_evs
    bool done = false;
    bool cancelled = false;
};

// A unit of admission: right-hand sides `rhs` of ticket t to start in the
// batch of (t->g, prec); a continuation starts them from the x held in the
// ticket's result buffer.
struct Work {
    Ticket* t = nullptr;
    int prec = 0;
    std::vector<int> rhs;
    bool cont = false;
    hipEvent_t ready = nullptr;  // continuation: recorded after x was exported
};

struct Batch {
    stag_engine* e = nullptr;
    hipStream_t stream = nullptr;
    EngineRun R;
    const stag_gauge* g = nullptr;
    int prec = 0;
    std::vector<Ticket*> slot_ticket;  // per slot, null when free
    std::vector<int> slot_rhs;
    Clock::time_point idle_since;
    int busy = 0;
};

struct Serve {
    stag_ctx* ctx = nullptr;
    std::thread th;
    std::mutex mu;
    std::condition_variable cv;
    bool stop = false;
    bool started = false;
    std::deque<Work> queue;
    std::unordered_map<stag_ticket, Ticket*> tickets;
    // uncollected tickets per gauge (stag_gauge_destroy refuses a gauge with any)
    std::unordered_map<const stag_gauge*, int> gauge_refs;
    // gauges whose batches the scheduler is asked to release (stag_gauge_destroy)
    std::vector<const stag_gauge*> drop;
    std::condition_variable drop_cv;
    stag_ticket next_id = 1;
    std::vector<Batch*> batches;  // scheduler thread only
    int slots = 16;
    int graph_k = 0;
    size_t queue_cap = 4096;
    int use_graph = 1;
};

static int batch_create(Serve* S, const stag_gauge* g, int prec, Batch** out) {
    stag_ctx* ctx = S->ctx;
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        return set_error(ctx, STAG_EDEVICE, "serve: stream creation failed");
    }
    stag_engine* e = nullptr;
    // cleared on the batch's own stream: other batches keep running meanwhile
    int rc = engine_create(ctx, g, prec, S->slots, true, s, &e);
    if (rc) {
        (void)hipStreamDestroy(s);
        return rc;
    }
    Batch* b = new Batch();
    b->e = e;
    b->stream = s;
    b->g = g;
    b->prec = prec;
    b->slot_ticket.assign(S->slots, nullptr);
    b->slot_rhs.assign(S->slots, 0);
    const int K = S->graph_k > 0 ? S->graph_k : default_graph_k(e->Vh);
    run_init(b->R, e, s, e->b64, e->rs64, K, S->use_graph != 0);
    b->idle_since = Clock::now();
    *out = b;
    return STAG_OK;
}

static void batch_destroy(Batch* b) {
    (void)hipStreamSynchronize(b->stream);
    engine_destroy(b->e);
    (void)hipStreamDestroy(b->stream);
    delete b;
}

static void ticket_free(stag_ctx* ctx, Ticket* t) {
    if (t->x_dev) dev_free(ctx, t->x_dev, t->x_bytes);
    for (hipEvent_t e : t->copy_evs) (void)hipEventDestroy(e);
    delete t;
}

// Whether every result copy of ticket t has completed.
static bool copies_done(Ticket* t) {
    for (hipEvent_t e : t->copy_evs) {
        hipError_t q = hipEventQuery(e);
        if (q != hipSuccess) {
            (void)hipGetLastError();
            return false;
        }
    }
    return true;
}

// Try to place work item w into a batch. Returns STAG_OK when started,
// STAG_ENOMEM when it must wait, or another error that fails the ticket.
// Runs on the scheduler thread without S->mu: it touches only the batches
// (scheduler-owned) and fields of a queued ticket that no other thread reads.
static int admit(Serve* S, Work& w) {
    stag_ctx* ctx = S->ctx;
    Ticket* t = w.t;
    const int n = (int)w.rhs.size();
    Batch* bt = nullptr;
    for (Batch* b : S->batches) {
        if (b->g != t->g || b->prec != w.prec) continue;
        if ((int)b->slot_ticket.size() - b->busy >= n) {
            bt = b;
            break;
        }
    }
    const size_t Vh = t->g->g.Vh;
    const size_t xb = (size_t)t->nrhs * Vh * 48;
    if (!t->x_dev) {
        int rc = dev_alloc(ctx, xb, &t->x_dev);
        if (rc) return rc;
        t->x_bytes = xb;
    }
    if (!bt) {
        int rc = batch_create(S, t->g, w.prec, &bt);
        if (rc == STAG_ENOMEM) {
            // release idle batches and retry once
            bool freed = false;
            for (size_t i = 0; i < S->batches.size();) {
                if (S->batches[i]->busy == 0) {
                    batch_destroy(S->batches[i]);
                    S->batches.erase(S->batches.begin() + i);
                    freed = true;
                } else {
                    ++i;
                }
            }
            rc = freed ? batch_create(S, t->g, w.prec, &bt) : STAG_ENOMEM;
        }
        if (rc) return rc;
        S->batches.push_back(bt);
    }
    // free slots, lowest first (keeps the kernel block size small)
    std::vector<SlotInit> inits;
    stag_cg_params p;
    stag_cg_params_default(&p);
    p.tol = t->tol;
    p.inner_prec = w.prec;
    if (w.prec == P16S && (t->g->mask & STAG_MASK_F32))
        p.max_stall = kEscalateStalls;  // somewhere to go: give up early
    if (w.cont) {
        // the fp32 continuation of a stalled fp16 pass: no stall restarts
        p.use_x0 = 1;
        p.stall_iters = std::numeric_limits<int>::max();
    }
    std::vector<int> taken;
    auto release = [&]() {
        for (int s : taken) bt->slot_ticket[s] = nullptr;
    };
    int k = 0;
    for (int s = 0; s < (int)bt->slot_ticket.size() && k < n; ++s) {
        if (bt->slot_ticket[s]) continue;
        const int r = w.rhs[k];
        bt->slot_ticket[s] = t;
        bt->slot_rhs[s] = r;
        taken.push_back(s);
        // upload the canonical complex128 [Vh][3] vector into the slot's x64
        // block and convert it into the engine's colour-major fp64 layout in
        // b64; x64 then starts from zero, or (continuation) from the ticket's
        // current x, converted the same way
        const size_t off = (size_t)s * bt->e->rs64;
        char* x64 = (char*)bt->e->x64 + off;
        hipError_t err = hipMemcpyAsync(x64, t->b.data() + (size_t)r * Vh * 6, Vh * 48,
                                        hipMemcpyHostToDevice, bt->stream);
        if (err == hipSuccess)
            err = launch_import(P64, x64, (char*)bt->e->b64 + off, bt->e->rs64, (uint32_t)Vh, 1,
                                bt->stream);
        if (err == hipSuccess && w.cont && w.ready) err = hipStreamWaitEvent(bt->stream, w.ready, 0);
        if (err == hipSuccess && w.cont)
            err = launch_import(P64, (const char*)t->x_dev + (size_t)r * Vh * 48, x64, bt->e->rs64,
                                (uint32_t)Vh, 1, bt->stream);
        if (err != hipSuccess) {
            (void)hipGetLastError();
            release();
            return set_error(ctx, STAG_EDEVICE, "serve: right-hand side upload: %s",
                             hipGetErrorString(err));
        }
        SlotInit si{s, t->mass, p};
        si.x0_in_place = w.cont;
        si.escalating = w.prec == P16S && (t->g->mask & STAG_MASK_F32);
        inits.push_back(si);
        ++k;
    }
    int hi = 0;
    for (int s = 0; s < (int)bt->slot_ticket.size(); ++s)
        if (bt->slot_ticket[s]) hi = s + 1;
    const int hi_prev = bt->R.busy_hi;
    bt->R.busy_hi = std::max(bt->R.busy_hi, hi);
    int rc = run_start_slots(bt->R, inits);
    if (rc) {
        release();
        bt->R.busy_hi = hi_prev;
        return rc;
    }
    bt->busy += n;
    if (!w.cont) t->remaining = t->nrhs;
    return STAG_OK;
}

// Harvest finished slots of a processed poll.
static void harvest(Serve* S, Batch* b, const RhsState* h) {
    const size_t Vh = b->e->Vh;
    for (int s = 0; s < (int)b->slot_ticket.size(); ++s) {
        Ticket* t = b->slot_ticket[s];
        if (!t) continue;
        if (b->R.last_poll <= b->R.start_after[s]) continue;  // poll predates the start
        if (!flags_terminal(h[s].flags)) continue;
        const int r = b->slot_rhs[s];
        const double secs = std::chrono::duration<double>(Clock::now() - t->t_submit).count();
        fill_stats(h[s], secs, b->prec, &t->stats[r]);
        // x64 (colour-major fp64) -> canonical complex128 [Vh][3] of the result
        hipError_t err = launch_export(P64, (char*)b->e->x64 + (size_t)s * b->e->rs64, b->e->rs64,
                                       (char*)t->x_dev + (size_t)r * Vh * 48, (uint32_t)Vh, 1,
                                       b->stream);
        hipEvent_t ev = nullptr;
        if (err == hipSuccess) err = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (err == hipSuccess) err = hipEventRecord(ev, b->stream);
        if (ev) t->copy_evs.push_back(ev);
        if (err != hipSuccess) {
            (void)hipGetLastError();
            t->stats[r].status = STAG_EDEVICE;
            (void)hipStreamSynchronize(b->stream);  // the copy is then waited for here
        }
        b->slot_ticket[s] = nullptr;
        b->busy -= 1;
        if (t->escalated[r]) {
            // the fp32 continuation ended: report both passes together
            stag_cg_stats& a = t->stats[r];
            const stag_cg_stats& f = t->first[r];
            a.iters += f.iters;
            a.reliable_updates += f.reliable_updates;
            a.restarts += f.restarts;
        } else if (b->prec == P16S && t->stats[r].status == STAG_ESTALL &&
                   (t->g->mask & STAG_MASK_F32)) {
            // fp16 storage hit its precision floor: continue in fp32 from x,
            // which the export above has put into the result buffer; the
            // continuation's upload runs on the fp32 batch's stream, so wait
            // for the export before it is admitted
            t->first[r] = t->stats[r];
            t->escalated[r] = 1;
            Work w;
            w.t = t;
            w.prec = P32;
            w.rhs.push_back(r);
            w.cont = true;
            if (hipEventCreateWithFlags(&w.ready, hipEventDisableTiming) != hipSuccess ||
                hipEventRecord(w.ready, b->stream) != hipSuccess) {
                (void)hipGetLastError();
                (void)hipStreamSynchronize(b->stream);
            }
            S->queue.push_front(w);
            continue;
        }
        t->remaining -= 1;
        if (t->remaining == 0) t->finishing = true;
    }
    int hi = 0;
    for (int s = 0; s < (int)b->slot_ticket.size(); ++s)
        if (b->slot_ticket[s]) hi = s + 1;
    b->R.busy_hi = hi;
    if (b->busy == 0) b->idle_since = Clock::now();
}

// Release the batches of the gauges stag_gauge_destroy asked for (under
// S->mu; the gauge has no uncollected ticket, so its batches are idle apart
// from blocks still in flight, which batch_destroy waits for).
static void drop_batches(Serve* S) {
    if (S->drop.empty()) return;
    for (const stag_gauge* g : S->drop) {
        for (size_t i = 0; i < S->batches.size();) {
            if (S->batches[i]->g == g) {
                batch_destroy(S->batches[i]);
                S->batches.erase(S->batches.begin() + i);
            } else {
                ++i;
            }
        }
    }
    S->drop.clear();
    S->drop_cv.notify_all();
}

static void scheduler(Serve* S) {
    stag_ctx* ctx = S->ctx;
    DeviceGuard dg(ctx->device);
    for (;;) {
        bool progress = false;
        // ---- admission: take the queue's current entries under the lock,
        // admit them without it (batch creation clears device buffers and
        // waits for that), then drop the admitted and failed ones. Only this
        // thread removes entries or adds them at the front; submit appends.
        std::vector<Work> cand;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            if (S->stop) break;
            drop_batches(S);
            bool any_busy = false;
            for (Batch* b : S->batches) any_busy |= b->busy > 0;
            if (S->queue.empty() && !any_busy) {
                S->cv.wait_for(lk, std::chrono::milliseconds(50));
                if (S->stop) break;
                drop_batches(S);
            }
            cand.assign(S->queue.begin(), S->queue.end());
        }
        if (!cand.empty()) {
            std::vector<int> rcs(cand.size());
            for (size_t i = 0; i < cand.size(); ++i) rcs[i] = admit(S, cand[i]);
            std::lock_guard<std::mutex> lk(S->mu);
            std::deque<Work> keep;
            for (size_t i = 0; i < cand.size(); ++i) {
                Work& w = cand[i];
                if (rcs[i] == STAG_ENOMEM) {
                    keep.push_back(w);  // waits for memory
                    continue;
                }
                if (w.ready) (void)hipEventDestroy(w.ready);
                if (rcs[i] == STAG_OK) {
                    progress = true;
                } else {
                    Ticket* t = w.t;
                    for (int r : w.rhs) t->stats[r].status = rcs[i];
                    if (w.cont) {
                        // the other right-hand sides finish where they run; the
                        // ticket completes when their result copies have
                        t->remaining -= 1;
                        if (t->remaining == 0) t->finishing = true;
                    } else {
                        t->done = true;
                        t->t_done = Clock::now();
                    }
                }
            }
            // entries appended by submit meanwhile stay behind the kept ones
            for (size_t i = cand.size(); i < S->queue.size(); ++i) keep.push_back(S->queue[i]);
            S->queue.swap(keep);
        }
        // ---- device progress
        for (Batch* b : S->batches) {
            if (b->busy == 0 && b->R.launched == b->R.polled) continue;
            if (b->R.launched - b->R.polled < 2 && b->busy > 0) {
                if (run_enqueue_block(b->R) == STAG_OK) progress = true;
            }
            if (b->R.polled < b->R.launched) {
                const RhsState* h = nullptr;
                int rc = run_process_poll(b->R, false, &h);
                if (rc == STAG_OK) {
                    std::lock_guard<std::mutex> lk(S->mu);
                    harvest(S, b, h);
                    progress = true;
                }
            }
        }
        // ---- tickets whose result copies completed
        {
            std::lock_guard<std::mutex> lk(S->mu);
            for (auto& kv : S->tickets) {
                Ticket* t = kv.second;
                if (t->finishing && !t->done && copies_done(t)) {
                    t->done = true;
                    t->t_done = Clock::now();
                    progress = true;
                }
            }
            // release batches idle for a while
            const auto now = Clock::now();
            for (size_t i = 0; i < S->batches.size();) {
                Batch* b = S->batches[i];
                if (b->busy == 0 && b->R.launched == b->R.polled &&
                    now - b->idle_since > std::chrono::milliseconds(2000)) {
                    batch_destroy(b);
                    S->batches.erase(S->batches.begin() + i);
                } else {
                    ++i;
                }
            }
        }
        if (!progress) std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
}

static Serve* serve_get(stag_ctx* ctx) {
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (!ctx->serve) {
        ctx->serve = new Serve();
        ctx->serve->ctx = ctx;
    }
    return ctx->serve;
}

}  // namespace stag

using namespace stag;

extern "C" {

int stag_serve_shutdown_internal(stag_ctx* ctx) {
    Serve* S = nullptr;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        S = ctx->serve;
        ctx->serve = nullptr;
    }
    if (!S) return STAG_OK;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv.notify_all();
    if (S->th.joinable()) S->th.join();
    for (Batch* b : S->batches) batch_destroy(b);
    for (auto& kv : S->tickets) ticket_free(ctx, kv.second);
    for (Work& w : S->queue)
        if (w.ready) (void)hipEventDestroy(w.ready);
    delete S;
    return STAG_OK;
}

// stag_gauge_destroy: STAG_EBUSY while a serving ticket on g is uncollected;
// otherwise the scheduler releases g's batches before this returns.
int stag_serve_release_gauge_internal(stag_ctx* ctx, const stag_gauge* g) {
    Serve* S = nullptr;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        S = ctx->serve;
    }
    if (!S) return STAG_OK;
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->gauge_refs.find(g);
    if (it != S->gauge_refs.end() && it->second > 0)
        return set_error(ctx, STAG_EBUSY,
                         "stag_gauge_destroy: %d serving request(s) on this gauge not yet collected",
                         it->second);
    if (!S->started) return STAG_OK;
    S->drop.push_back(g);
    S->cv.notify_all();
    S->drop_cv.wait(lk, [&]() {
        return S->stop || std::find(S->drop.begin(), S->drop.end(), g) == S->drop.end();
    });
    return STAG_OK;
}

int stag_solver_config(stag_ctx* ctx, int slots_per_batch, int graph_k, int queue_cap) {
    if (!ctx) return STAG_EINVAL;
    if (slots_per_batch < 1 || slots_per_batch > STAG_MAX_RHS || queue_cap < 1)
        return set_error(ctx, STAG_EINVAL, "stag_solver_config: bad argument");
    Serve* S = serve_get(ctx);
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->started)
        return set_error(ctx, STAG_EBUSY, "stag_solver_config: serving already started");
    S->slots = pick_n(slots_per_batch);
    S->graph_k = graph_k;
    S->queue_cap = (size_t)queue_cap;
    return STAG_OK;
}

int stag_solver_submit(stag_ctx* ctx, const stag_gauge* g, double mass, int nrhs,
                       const double* b_host, double tol, int inner_prec, stag_ticket* out) {
    if (!ctx) return STAG_EINVAL;
    if (!g || !b_host || !out) return set_error(ctx, STAG_EINVAL, "stag_solver_submit: NULL argument");
    if (g->ctx != ctx) return set_error(ctx, STAG_EINVAL, "stag_solver_submit: gauge of another context");
    if (nrhs < 1 || nrhs > STAG_MAX_RHS)
        return set_error(ctx, STAG_EINVAL, "stag_solver_submit: nrhs %d out of [1, %d]", nrhs, STAG_MAX_RHS);
    if (!(mass > 0.0) || !std::isfinite(mass))
        return set_error(ctx, STAG_EINVAL, "stag_solver_submit: mass must be finite and > 0");
    if (!(tol > 0.0 && tol < 1.0))
        return set_error(ctx, STAG_EINVAL, "stag_solver_submit: tol must be in (0, 1)");
    if (inner_prec < 0 || inner_prec > 2 || !(g->mask & STAG_MASK_F64) || !(g->mask & (1 << inner_prec)))
        return set_error(ctx, STAG_EINVAL,
                         "stag_solver_submit: gauge needs the F64 copy and the inner-precision copy");
    Serve* S = serve_get(ctx);
    Ticket* t = new Ticket();
    t->g = g;
    t->mass = mass;
    t->tol = tol;
    t->nrhs = nrhs;
    t->prec = inner_prec;
    const size_t n = (size_t)nrhs * g->g.Vh * 6;
    t->b.assign(b_host, b_host + n);
    t->stats.resize(nrhs);
    for (auto& s : t->stats) {
        std::memset(&s, 0, sizeof(s));
        s.status = STAG_PENDING;
    }
    t->first.resize(nrhs);
    t->escalated.assign(nrhs, 0);
    t->t_submit = Clock::now();
    Work w;
    w.t = t;
    w.prec = inner_prec;
    for (int r = 0; r < nrhs; ++r) w.rhs.push_back(r);
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->queue.size() >= S->queue_cap) {
            delete t;
            return set_error(ctx, STAG_EBUSY, "stag_solver_submit: queue full");
        }
        t->id = S->next_id++;
        S->tickets[t->id] = t;
        S->gauge_refs[g] += 1;
        S->queue.push_back(w);
        if (!S->started) {
            S->started = true;
            S->th = std::thread(scheduler, S);
        }
    }
    S->cv.notify_all();
    *out = t->id;
    return STAG_OK;
}

int stag_solver_poll(stag_ctx* ctx, stag_ticket ticket, double* x_host, stag_cg_stats* stats,
                     double* latency_s) {
    if (!ctx) return STAG_EINVAL;
    Serve* S = nullptr;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        S = ctx->serve;
    }
    if (!S) return set_error(ctx, STAG_ENOTFOUND, "stag_solver_poll: unknown ticket");
    Ticket* t = nullptr;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        auto it = S->tickets.find(ticket);
        if (it == S->tickets.end())
            return set_error(ctx, STAG_ENOTFOUND, "stag_solver_poll: unknown ticket %lld",
                             (long long)ticket);
        t = it->second;
        if (!t->done) return STAG_PENDING;
        S->tickets.erase(it);
        S->gauge_refs[t->g] -= 1;
    }
    DeviceGuard dg(ctx->device);
    int rc = STAG_OK;
    for (auto& s : t->stats)
        if (rc == STAG_OK && s.status != STAG_OK) rc = s.status;
    if (x_host && t->x_dev) {
        hipError_t err = hipMemcpy(x_host, t->x_dev, t->x_bytes, hipMemcpyDeviceToHost);
        if (err != hipSuccess) {
            (void)hipGetLastError();
            rc = set_error(ctx, STAG_EDEVICE, "stag_solver_poll: copy: %s", hipGetErrorString(err));
        }
    }
    if (stats)
        for (int r = 0; r < t->nrhs; ++r) stats[r] = t->stats[r];
    if (latency_s) *latency_s = std::chrono::duration<double>(t->t_done - t->t_submit).count();
    ticket_free(ctx, t);
    return rc;
}

}  // extern "C"
