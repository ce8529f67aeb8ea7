// CG solver engine: plain fp64 CG (Fig.1) and the corrected mixed-precision
// CG of Sec.3.2 (low-precision inner iterations, fp64 reliable + group-wise
// updates, direction carried over as in Eq.6), for a block of right-hand
// sides ("slots") that share every link load.
//
// All CG scalars live on the device (RhsState) and are produced by the last
// block of each reduction, so an iteration is three kernels with no host
// round trip. The host enqueues blocks of K iterations (one HIP graph
// replay), polls the per-slot flags one block behind the device, and
// enqueues the fp64 true-residual work only when a flag asks for it; those
// kernels are predicated on the flags, so a redundant enqueue is a no-op.
//
// Slots are independent: a slot can start (from x = 0) at any block
// boundary while others are mid-solve, and its arithmetic does not depend on
// the other slots or on the kernel's block size N, so a solve gives the same
// bits alone and in a mix. stag_cg_solve runs one batch of slots to the
// end; the serving loop (serve.cpp) keeps slots busy continuously.
#include <chrono>
#include <cmath>
#include <cstring>

#include "internal.h"

namespace stag {

static size_t state_bytes(int N) { return sizeof(RhsState) * (size_t)N; }

void engine_drop_graphs(stag_engine* e) {
    for (auto& kv : e->graphs) {
        GraphSet& gs = kv.second;
        for (int i = 0; i < 2; ++i) {
            if (gs.g[i]) (void)hipGraphExecDestroy(gs.g[i]);
            for (auto& r : gs.ev[i]) {
                if (r.a) (void)hipEventDestroy(r.a);
                if (r.b) (void)hipEventDestroy(r.b);
            }
        }
    }
    e->graphs.clear();
}

void engine_destroy(stag_engine* e) {
    if (!e) return;
    stag_ctx* ctx = e->ctx;
    engine_drop_graphs(e);
    void* bufs[] = {e->x64, e->r64, e->t64, e->d64, e->Ad64, e->y32, e->rs, e->d, e->t, e->Ad,
                    e->b64, e->st, e->partials};
    for (void* p : bufs)
        if (p) (void)hipFree(p);
    for (int i = 0; i < 2; ++i) {
        if (e->host[i]) (void)hipHostFree(e->host[i]);
        if (e->ev[i]) (void)hipEventDestroy(e->ev[i]);
    }
    if (e->hstage) (void)hipHostFree(e->hstage);
    if (e->cap_stream) (void)hipStreamDestroy(e->cap_stream);
    ctx->used.fetch_sub(e->bytes);
    delete e;
}

int engine_create(stag_ctx* ctx, const stag_gauge* g, int prec, int N, bool own_b,
                  stag_engine** out) {
    stag_engine* e = new stag_engine();
    e->ctx = ctx;
    e->gauge = g;
    e->prec = prec;
    e->N = N;
    e->Vh = g->g.Vh;
    const size_t Vh = e->Vh;
    e->rs64 = spinor_rhs_bytes(P64, Vh);
    e->rsP = spinor_rhs_bytes(prec, Vh);
    e->rs32 = spinor_rhs_bytes(P32, Vh);
    const size_t nparts = (size_t)num_chunks(e->Vh);
    struct Req {
        void** p;
        size_t bytes;
    };
    std::vector<Req> reqs = {
        {&e->x64, N * e->rs64}, {&e->r64, N * e->rs64}, {&e->t64, N * e->rs64},
        {(void**)&e->st, state_bytes(N)}, {(void**)&e->partials, N * nparts * sizeof(double)},
    };
    if (own_b) reqs.push_back({&e->b64, N * e->rs64});
    if (prec == P64) {
        reqs.push_back({&e->d64, N * e->rs64});
        reqs.push_back({&e->Ad64, N * e->rs64});
    } else {
        reqs.push_back({&e->y32, N * e->rs32});
        reqs.push_back({&e->rs, N * e->rsP});
        reqs.push_back({&e->d, N * e->rsP});
        reqs.push_back({&e->t, N * e->rsP});
        reqs.push_back({&e->Ad, N * e->rsP});
    }
    size_t total = 0;
    for (auto& r : reqs) total += r.bytes;
    size_t prev = ctx->used.fetch_add(total);
    if (ctx->budget && prev + total > ctx->budget) {
        ctx->used.fetch_sub(total);
        delete e;
        return set_error(ctx, STAG_ENOMEM, "solver workspace: HBM budget exceeded (%zu + %zu > %zu)",
                         prev, total, ctx->budget);
    }
    e->bytes = total;
    for (auto& r : reqs) {
        if (hipMalloc(r.p, r.bytes) != hipSuccess) {
            (void)hipGetLastError();
            engine_destroy(e);
            return set_error(ctx, STAG_ENOMEM, "solver workspace: hipMalloc(%zu) failed", r.bytes);
        }
    }
    for (int i = 0; i < 2; ++i) {
        if (hipHostMalloc((void**)&e->host[i], state_bytes(N), hipHostMallocDefault) != hipSuccess ||
            hipEventCreateWithFlags(&e->ev[i], hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            engine_destroy(e);
            return set_error(ctx, STAG_EDEVICE, "solver workspace: pinned buffer / event");
        }
    }
    if (hipHostMalloc((void**)&e->hstage, state_bytes(N), hipHostMallocDefault) != hipSuccess ||
        hipStreamCreateWithFlags(&e->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        engine_destroy(e);
        return set_error(ctx, STAG_EDEVICE, "solver workspace: pinned staging / capture stream");
    }
    // Every slot starts free, and the direction / y buffers must hold finite
    // values (beta = 0 multiplies them). hipMemset runs on the null stream,
    // which does not order against the non-blocking streams the solves use:
    // wait for it here.
    hipError_t err = hipMemset(e->st, 0, state_bytes(N));
    if (err == hipSuccess && e->d64) err = hipMemset(e->d64, 0, N * e->rs64);
    if (err == hipSuccess && e->d) err = hipMemset(e->d, 0, N * e->rsP);
    if (err == hipSuccess && e->y32) err = hipMemset(e->y32, 0, N * e->rs32);
    if (err == hipSuccess) err = hipDeviceSynchronize();
    if (err != hipSuccess) {
        (void)hipGetLastError();
        engine_destroy(e);
        return set_error(ctx, STAG_EDEVICE, "solver workspace: init");
    }
    e->tune_lo = get_tune(ctx, prec, pick_n(N), e->Vh);
    e->tune_64 = get_tune(ctx, P64, pick_n(N), e->Vh);
    *out = e;
    return STAG_OK;
}

int engine_acquire(stag_ctx* ctx, const stag_gauge* g, int prec, int N, stag_engine** out) {
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        for (auto* e : ctx->engines)
            if (!e->in_use && e->gauge == g && e->prec == prec && e->N == N && !e->b64) {
                e->in_use = true;
                *out = e;
                return STAG_OK;
            }
    }
    stag_engine* e = nullptr;
    int rc = engine_create(ctx, g, prec, N, false, &e);
    if (rc) return rc;
    e->in_use = true;
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->engines.push_back(e);
    *out = e;
    return STAG_OK;
}

void engine_release(stag_engine* e) {
    std::lock_guard<std::mutex> lk(e->ctx->mu);
    e->in_use = false;
}

// ------------------------------------------------------------------ enqueue helpers

namespace {

struct Ctx {
    stag_engine* e;
    hipStream_t s;
    const void* b;
    size_t b_rs;
    int nk;                          // kernel block size (>= highest busy slot + 1)
    bool timed;
    std::vector<Timing::Rec>* cap;  // non-null while capturing a timed graph
    mutable size_t cap_next;        // next unused record of *cap
};

// Launch `fn` bracketed by timing events when the run is timed. Inside a
// graph capture the events become external event-record nodes of the graph.
template <typename F>
hipError_t timed_launch(const Ctx& c, int kind, F&& fn) {
    if (!c.timed) return fn();
    if (c.cap) {
        if (c.cap_next >= c.cap->size()) return hipErrorInvalidValue;
        Timing::Rec& rec = (*c.cap)[c.cap_next];
        c.cap_next += 1;
        rec.kind = kind;
        hipError_t err = hipEventRecordWithFlags(rec.a, c.s, hipEventRecordExternal);
        if (err == hipSuccess) err = fn();
        if (err == hipSuccess) err = hipEventRecordWithFlags(rec.b, c.s, hipEventRecordExternal);
        return err;
    }
    hipEvent_t a = nullptr;
    hipError_t err = timing_begin(c.e->ctx, c.s, &a);
    if (err != hipSuccess) return err;
    err = fn();
    if (err != hipSuccess) return err;
    return timing_end(c.e->ctx, c.s, kind, a);
}

Reduce make_red(stag_engine* e, int kind) {
    Reduce r{};
    r.partials = e->partials;
    r.st = e->st;
    r.out = nullptr;
    r.kind = kind;
    r.nparts = (int)num_chunks(e->Vh);
    return r;
}

hipError_t hop(const Ctx& c, int prec, int stage, int epi, const void* in, void* out,
               const void* x, int kind, unsigned run, const void* lazy_r = nullptr) {
    stag_engine* e = c.e;
    const HopTune& t = prec == P64 && e->prec != P64 ? e->tune_64 : e->tune_lo;
    int S = stage == 1 ? t.S1 : t.S2;
    if (c.nk > 1) S = 1;
    const size_t rs = spinor_rhs_bytes(prec, e->Vh);
    Reduce red = make_red(e, kind);
    const int p_out = stage == 1 ? 1 : 0;
    const int kk = prec == e->prec && run == F_ACTIVE ? (stage == 1 ? KK_HOP1 : KK_HOP2)
                                                       : (stage == 1 ? KK_HOP1_64 : KK_HOP2_64);
    hipError_t err = timed_launch(c, kk, [&]() {
        return enqueue_hop(e->gauge, prec, S, c.nk, epi, t, in, rs, out, rs, p_out, x, rs, c.b,
                           c.b_rs, nullptr, e->st, run, &red, c.s, lazy_r, rs);
    });
    if (err != hipSuccess || !(epi == EPI_XPAY_DOT || epi == EPI_RESID)) return err;
    return timed_launch(c, KK_OTHER, [&]() { return launch_finalize(c.nk, red, run, c.s); });
}

hipError_t vec(const Ctx& c, int prec, int op, std::initializer_list<std::pair<void*, size_t>> f,
               int kind, unsigned run) {
    stag_engine* e = c.e;
    VecArgs a{};
    int k = 0;
    for (auto& p : f) {
        a.f[k] = p.first;
        a.rs[k] = p.second;
        ++k;
    }
    a.Vh = e->Vh;
    a.st = e->st;
    a.run_mask = run;
    a.swizzle = e->tune_lo.swizzle;
    a.red = make_red(e, kind);
    const int kk = op == OP_UPD_CG || op == OP_UPD_MIXED ? KK_UPDATE : KK_OTHER;
    hipError_t err = timed_launch(c, kk, [&]() { return launch_vec(prec, c.nk, op, a, c.s); });
    if (err != hipSuccess || !(op == OP_INIT_B || op == OP_UPD_CG || op == OP_UPD_MIXED)) return err;
    return timed_launch(c, KK_OTHER, [&]() { return launch_finalize(c.nk, a.red, run, c.s); });
}

// One CG iteration (Fig.1): three work kernels and two one-block reduction
// finalisations (alpha after stage 2, beta and the decisions after the
// update). The direction update
// d = r + beta d of the previous iteration is deferred into the two hop
// stages (stage 1 forms it at the neighbours it gathers, stage 2 at its own
// site, storing it), so no separate pass over d is needed.
hipError_t enqueue_iteration(const Ctx& c) {
    stag_engine* e = c.e;
    hipError_t err;
    if (e->prec == P64) {
        if ((err = hop(c, P64, 1, EPI_PLAIN, e->d64, e->t64, nullptr, FIN_STORE, F_ACTIVE, e->r64)))
            return err;
        if ((err = hop(c, P64, 2, EPI_XPAY_DOT, e->t64, e->Ad64, e->d64, FIN_ALPHA, F_ACTIVE, e->r64)))
            return err;
        return vec(c, P64, OP_UPD_CG,
                   {{e->x64, e->rs64}, {e->r64, e->rs64}, {e->d64, e->rs64}, {e->Ad64, e->rs64}},
                   FIN_CG, F_ACTIVE);
    }
    const int P = e->prec;
    if ((err = hop(c, P, 1, EPI_PLAIN, e->d, e->t, nullptr, FIN_STORE, F_ACTIVE, e->rs))) return err;
    if ((err = hop(c, P, 2, EPI_XPAY_DOT, e->t, e->Ad, e->d, FIN_ALPHA, F_ACTIVE, e->rs))) return err;
    return vec(c, P, OP_UPD_MIXED,
               {{e->y32, e->rs32}, {e->rs, e->rsP}, {e->d, e->rsP}, {e->Ad, e->rsP}}, FIN_MIXED,
               F_ACTIVE);
}

hipError_t state_step(const Ctx& c, int kind, unsigned run) {
    return timed_launch(c, KK_OTHER, [&]() { return launch_state(c.nk, kind, c.e->st, run, c.s); });
}

// fp64 true residual r64 = b - A x64 for the slots whose flags match `run`.
hipError_t enqueue_true_residual(const Ctx& c, unsigned run) {
    stag_engine* e = c.e;
    hipError_t err;
    if ((err = hop(c, P64, 1, EPI_PLAIN, e->x64, e->t64, nullptr, FIN_STORE, run))) return err;
    return hop(c, P64, 2, EPI_RESID, e->t64, e->r64, e->x64, FIN_TRUE, run);
}

// Plain CG: the iterated residual met the tolerance; check the true one and
// either finish or restart from it (r = b - A x, direction d = r).
hipError_t enqueue_check(const Ctx& c) {
    hipError_t err;
    if ((err = enqueue_true_residual(c, F_CONV))) return err;
    return state_step(c, FIN_CG_CHECK, F_CONV);
}

// Mixed CG (Sec.3.2): reliable + group-wise update. x += y in fp64, y = 0,
// r = b - A x in fp64, the low-precision residual restarts from it, and the
// direction carries over (Eq.6) or restarts after a stall.
hipError_t enqueue_update(const Ctx& c) {
    stag_engine* e = c.e;
    const unsigned run = F_RU | F_STALL;
    hipError_t err;
    if ((err = vec(c, e->prec, OP_RU_BEGIN, {{e->x64, e->rs64}, {e->y32, e->rs32}}, FIN_STORE, run)))
        return err;
    if ((err = enqueue_true_residual(c, run))) return err;
    if ((err = vec(c, e->prec, OP_RU_END, {{e->r64, e->rs64}, {e->rs, e->rsP}}, FIN_STORE, run)))
        return err;
    return state_step(c, FIN_RU_END, run);
}

}  // namespace

int status_of_flags(unsigned f) {
    if (f & F_DONE) return STAG_OK;
    if (f & F_BADINPUT) return STAG_EINVAL;
    if (f & F_BREAKDOWN) return STAG_EBREAKDOWN;
    if (f & F_ESTALL) return STAG_ESTALL;
    return STAG_ENOCONV;
}

bool flags_terminal(unsigned f) {
    return (f & (F_DONE | F_BADINPUT | F_BREAKDOWN | F_ESTALL)) ||
           ((f & F_MAXIT) && !(f & (F_CONV | F_RU)));
}

#define RCK(call)                                                                              \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess) {                                                                \
            (void)hipGetLastError();                                                           \
            return set_error(e->ctx, STAG_EDEVICE, "solver: %s: %s", #call, hipGetErrorString(e_)); \
        }                                                                                      \
    } while (0)

// ------------------------------------------------------------------ runs

void run_init(EngineRun& R, stag_engine* e, hipStream_t s, const void* b, size_t b_rs, int K,
              bool use_graph) {
    R.e = e;
    R.s = s;
    R.b = b;
    R.b_rs = b_rs;
    R.K = K;
    R.use_graph = use_graph;
    R.timed = e->ctx->timing.on;
    if (R.timed && e->ctx->timing.no_graph_events) R.use_graph = false;
    R.launched = R.polled = 0;
    R.fix_after.assign(e->N, -1);
    R.start_after.assign(e->N, -1);
    R.last_poll = -1;
    R.busy_hi = 0;
    R.block_graph[0] = R.block_graph[1] = nullptr;
    R.block_inst[0] = R.block_inst[1] = 0;
}

int default_graph_k(uint32_t Vh) { return Vh >= 262144 ? 16 : (Vh >= 32768 ? 32 : 64); }

// Start the given slots from x = 0: per-slot initial state, then the first
// direction d = r = b and |b|^2 (the finalisation turns F_NEW into
// F_ACTIVE, F_DONE for b = 0, or F_BADINPUT).
int run_start_slots(EngineRun& R, const std::vector<SlotInit>& slots) {
    stag_engine* e = R.e;
    if (slots.empty()) return STAG_OK;
    const uint64_t n_unknowns = 3ull * e->Vh;
    for (const SlotInit& si : slots) {
        RhsState& s = e->hstage[si.slot];
        std::memset(&s, 0, sizeof(s));
        const stag_cg_params& p = si.params;
        s.tol2 = p.tol * p.tol;
        s.m2 = si.mass * si.mass;
        s.delta = p.delta > 0 ? p.delta : 0.1;
        s.stall_iters = p.stall_iters > 0 ? p.stall_iters : 100;
        s.max_stall = p.max_stall > 0 ? p.max_stall : 20;
        s.max_iter = p.max_iter > 0 ? p.max_iter : (int)std::min<uint64_t>(10 * n_unknowns, 1000000);
        s.flags = F_NEW;
        RCK(hipMemcpyAsync(e->st + si.slot, &s, sizeof(RhsState), hipMemcpyHostToDevice, R.s));
        if (si.slot + 1 > R.busy_hi) R.busy_hi = si.slot + 1;
        // polls of blocks launched before this start show the slot's previous state
        R.fix_after[si.slot] = R.start_after[si.slot] = R.launched - 1;
    }
    Ctx c{e, R.s, R.b, R.b_rs, pick_n(R.busy_hi), R.timed, nullptr, 0};
    void* b = const_cast<void*>(R.b);
    if (e->prec != P64) {
        RCK(vec(c, e->prec, OP_START, {{b, R.b_rs}, {e->d, e->rsP}, {e->rs, e->rsP}, {e->y32, e->rs32}},
                FIN_STORE, F_NEW));
    } else {
        RCK(vec(c, P64, OP_START, {{b, R.b_rs}, {e->d64, e->rs64}, {nullptr, 0}, {nullptr, 0}},
                FIN_STORE, F_NEW));
    }
    RCK(vec(c, P64, OP_INIT_B, {{b, R.b_rs}, {e->r64, e->rs64}, {e->x64, e->rs64}}, FIN_INIT, F_NEW));
    return STAG_OK;
}

static int get_graphs(EngineRun& R, int nk, GraphSet** out) {
    stag_engine* e = R.e;
    const int ninst = R.timed ? 2 : 1;
    const long long key = ((long long)R.K << 16) | ((long long)nk << 1) | (R.timed ? 1 : 0);
    // the iteration kernels never read b, so one graph serves every b buffer
    auto it = e->graphs.find(key);
    if (it != e->graphs.end()) {
        *out = &it->second;
        return STAG_OK;
    }
    GraphSet gs;
    gs.n = ninst;
    bool ok = true;
    hipError_t bad = hipSuccess;
    // capture on the engine's idle stream (a graph does not depend on the
    // stream it was captured on); replays go to the run's stream
    hipStream_t cs = e->cap_stream;
    for (int inst = 0; inst < ninst && ok; ++inst) {
        Ctx cc{e, cs, R.b, R.b_rs, nk, R.timed, nullptr, 0};
        if (R.timed) {
            gs.ev[inst].resize((size_t)R.K * 5);  // five kernels per iteration
            for (auto& r : gs.ev[inst]) {
                r.a = r.b = nullptr;
                if (hipEventCreate(&r.a) != hipSuccess || hipEventCreate(&r.b) != hipSuccess) ok = false;
            }
            cc.cap = &gs.ev[inst];
        }
        if (!ok) break;
        hipGraph_t graph = nullptr;
        hipError_t berr = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed);
        if (berr != hipSuccess) {
            (void)hipGetLastError();
            bad = berr;
            ok = false;
            break;
        }
        hipError_t cerr = hipSuccess;
        for (int k = 0; k < R.K && cerr == hipSuccess; ++k) cerr = enqueue_iteration(cc);
        hipError_t eerr = hipStreamEndCapture(cs, &graph);
        hipError_t ierr = hipErrorInvalidValue;
        if (cerr == hipSuccess && eerr == hipSuccess && graph)
            ierr = hipGraphInstantiate(&gs.g[inst], graph, nullptr, nullptr, 0);
        if (graph) (void)hipGraphDestroy(graph);
        if (ierr != hipSuccess) {
            (void)hipGetLastError();
            gs.g[inst] = nullptr;
            bad = cerr != hipSuccess ? cerr : eerr != hipSuccess ? eerr : ierr;
            ok = false;
        }
    }
    if (!ok) {
        for (int i = 0; i < 2; ++i) {
            if (gs.g[i]) (void)hipGraphExecDestroy(gs.g[i]);
            for (auto& r : gs.ev[i]) {
                if (r.a) (void)hipEventDestroy(r.a);
                if (r.b) (void)hipEventDestroy(r.b);
            }
        }
        if (R.timed) {
            // the runtime refused event nodes in a capture: time eagerly
            e->ctx->timing.no_graph_events = true;
            R.use_graph = false;
            *out = nullptr;
            return STAG_OK;
        }
        return set_error(e->ctx, STAG_EDEVICE, "solver: graph capture failed: %s",
                         hipGetErrorString(bad));
    }
    auto res = e->graphs.emplace(key, std::move(gs));
    *out = &res.first->second;
    return STAG_OK;
}

// Enqueue K iterations for the busy slots, then the poll of the state.
int run_enqueue_block(EngineRun& R) {
    stag_engine* e = R.e;
    const int nk = pick_n(R.busy_hi > 0 ? R.busy_hi : 1);
    const long long j = R.launched;
    GraphSet* gs = nullptr;
    if (R.use_graph) {
        int rc = get_graphs(R, nk, &gs);
        if (rc) return rc;
    }
    const int buf = (int)(j % 2);
    if (gs) {
        const int inst = (int)(j % gs->n);
        RCK(hipGraphLaunch(gs->g[inst], R.s));
        R.block_graph[buf] = gs;
        R.block_inst[buf] = inst;
    } else {
        Ctx c{e, R.s, R.b, R.b_rs, nk, R.timed, nullptr, 0};
        for (int k = 0; k < R.K; ++k) RCK(enqueue_iteration(c));
        R.block_graph[buf] = nullptr;
    }
    RCK(hipMemcpyAsync(e->host[buf], e->st, state_bytes(e->N), hipMemcpyDeviceToHost, R.s));
    RCK(hipEventRecord(e->ev[buf], R.s));
    R.launched = j + 1;
    return STAG_OK;
}

// Wait for (or, with blocking = false, test) the oldest outstanding poll.
// On success *h points at the polled states (valid until the next block is
// enqueued); fix-up work (true-residual checks, reliable updates) for
// flagged slots is enqueued. Returns STAG_PENDING when not blocking and the
// poll is not complete yet.
int run_process_poll(EngineRun& R, bool blocking, const RhsState** h) {
    stag_engine* e = R.e;
    if (R.polled >= R.launched) return set_error(e->ctx, STAG_EINVAL, "solver: no poll outstanding");
    const long long j = R.polled;
    const int buf = (int)(j % 2);
    if (blocking) {
        RCK(hipEventSynchronize(e->ev[buf]));
    } else {
        hipError_t q = hipEventQuery(e->ev[buf]);
        if (q == hipErrorNotReady) {
            (void)hipGetLastError();
            return STAG_PENDING;
        }
        RCK(q);
    }
    if (R.timed) {
        timing_collect(e->ctx);
        GraphSet* gs = R.block_graph[buf];
        if (gs) {
            Timing& T = e->ctx->timing;
            std::lock_guard<std::mutex> lk(T.mu);
            for (auto& r : gs->ev[R.block_inst[buf]]) {
                float ms = 0.f;
                if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
                    T.count[r.kind] += 1;
                    T.ms[r.kind] += ms;
                }
                (void)hipGetLastError();
            }
        }
    }
    R.polled = j + 1;
    R.last_poll = j;
    const RhsState* st = e->host[buf];
    const bool mixed = e->prec != P64;
    bool need = false;
    for (int r = 0; r < R.busy_hi; ++r) {
        const unsigned f = st[r].flags;
        if (flags_terminal(f) || j <= R.fix_after[r]) continue;
        if ((!mixed && (f & F_CONV)) || (mixed && (f & (F_RU | F_STALL)))) {
            need = true;
            // the fix is enqueued after every block launched so far; the
            // first poll that sees its effect is the next one enqueued
            R.fix_after[r] = R.launched - 1;
        }
    }
    if (need) {
        Ctx c{e, R.s, R.b, R.b_rs, pick_n(R.busy_hi), R.timed, nullptr, 0};
        RCK(mixed ? enqueue_update(c) : enqueue_check(c));
    }
    *h = st;
    return STAG_OK;
}

void fill_stats(const RhsState& s, double secs, stag_cg_stats* out) {
    out->iters = s.iters;
    out->reliable_updates = s.updates;
    out->restarts = s.restarts;
    out->status = flags_terminal(s.flags) ? status_of_flags(s.flags) : STAG_ENOCONV;
    out->true_rel_res = s.bb > 0 ? std::sqrt(s.rr_true / s.bb) : 0.0;
    out->iter_rel_res = s.bb > 0 ? std::sqrt(s.rr / s.bb) : 0.0;
    out->seconds = secs;
}

// ------------------------------------------------------------------ one-shot solve

int engine_solve(stag_engine* e, int n, const double* mass, const void* b64, size_t b_rs,
                 void* x_out, size_t x_rs, const stag_cg_params& p, stag_cg_stats* stats,
                 hipStream_t stream) {
    const auto t0 = std::chrono::steady_clock::now();
    const int K = p.graph_k > 0 ? p.graph_k : default_graph_k(e->Vh);
    EngineRun R;
    run_init(R, e, stream, b64, b_rs, K, p.use_graph != 0);
    std::vector<SlotInit> slots(n);
    for (int r = 0; r < n; ++r) slots[r] = SlotInit{r, mass[r], p};
    int rc = run_start_slots(R, slots);
    if (rc) return rc;
    const long long max_blocks = (2ll * (p.max_iter > 0 ? p.max_iter : 1000000)) / K + 4096;
    rc = run_enqueue_block(R);
    if (rc) return rc;
    std::vector<RhsState> fin(n);
    for (;;) {
        rc = run_enqueue_block(R);
        if (rc) return rc;
        const RhsState* h = nullptr;
        rc = run_process_poll(R, true, &h);
        if (rc) return rc;
        bool all_terminal = true;
        for (int r = 0; r < n; ++r)
            if (!flags_terminal(h[r].flags)) all_terminal = false;
        if (all_terminal || R.launched > max_blocks) {
            // the device enforces max_iter; the block cap only guards the host loop
            std::copy(h, h + n, fin.begin());
            break;
        }
    }
    RCK(hipStreamSynchronize(stream));
    RCK(hipMemcpy2DAsync(x_out, x_rs, e->x64, e->rs64, e->rs64, n, hipMemcpyDeviceToDevice, stream));
    RCK(hipStreamSynchronize(stream));
    if (R.timed) timing_collect(e->ctx);
    const double secs =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    rc = STAG_OK;
    for (int r = 0; r < n; ++r) {
        stag_cg_stats s;
        fill_stats(fin[r], secs, &s);
        if (stats) stats[r] = s;
        if (rc == STAG_OK && s.status != STAG_OK) rc = s.status;
    }
    if (rc == STAG_EINVAL) set_error(e->ctx, rc, "stag_cg_solve: right-hand side is not finite");
    return rc;
}

}  // namespace stag

// ------------------------------------------------------------------ kernel timing

using namespace stag;

extern "C" int stag_time_kernels(stag_ctx* ctx, const stag_gauge* g, int prec, int nrhs, int reps,
                                 double* us_out) {
    if (!ctx) return STAG_EINVAL;
    if (!g || !us_out || prec < 0 || prec > 2 || nrhs < 1 || nrhs > STAG_MAX_RHS || reps < 1)
        return set_error(ctx, STAG_EINVAL, "stag_time_kernels: bad argument");
    if (!(g->mask & (1 << prec)) || !(g->mask & STAG_MASK_F64))
        return set_error(ctx, STAG_EINVAL, "stag_time_kernels: gauge lacks a needed copy");
    DeviceGuard dg(ctx->device);
    const int N = pick_n(nrhs);
    stag_engine* e = nullptr;
    int rc = engine_acquire(ctx, g, prec, N, &e);
    if (rc) return rc;
    hipStream_t s = ctx->stream;
    // every slot active with alpha = beta = 0 (so d = r and the vectors stay
    // put); reductions store their sums instead of changing the state
    for (int r = 0; r < N; ++r) {
        RhsState& st = e->hstage[r];
        std::memset(&st, 0, sizeof(st));
        st.flags = r < nrhs ? F_ACTIVE : 0u;
        st.m2 = 0.01;
        st.rr = 1.0;
    }
    double* sink = nullptr;
    hipError_t err = hipMemcpyAsync(e->st, e->hstage, sizeof(RhsState) * N, hipMemcpyHostToDevice, s);
    if (err == hipSuccess) err = hipMallocAsync((void**)&sink, sizeof(double) * N, s);
    const size_t bytes[] = {N * e->rs64, N * e->rsP, N * e->rs32};
    void* zero64[] = {e->x64, e->r64, e->t64, e->d64, e->Ad64};
    void* zeroP[] = {e->rs, e->d, e->t, e->Ad};
    for (void* p : zero64)
        if (err == hipSuccess && p) err = hipMemsetAsync(p, 0, bytes[0], s);
    for (void* p : zeroP)
        if (err == hipSuccess && p) err = hipMemsetAsync(p, 0, bytes[1], s);
    if (err == hipSuccess && e->y32) err = hipMemsetAsync(e->y32, 0, bytes[2], s);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (err == hipSuccess) err = hipEventCreate(&e0);
    if (err == hipSuccess) err = hipEventCreate(&e1);
    Ctx c{e, s, nullptr, 0, N, false, nullptr, 0};
    const bool mixed = prec != P64;
    auto one = [&](int which) -> hipError_t {
        Reduce red = make_red(e, FIN_STORE);
        red.out = sink;
        const HopTune& t = e->tune_lo;
        const size_t rs = mixed ? e->rsP : e->rs64;
        void* dd = mixed ? e->d : e->d64;
        void* rr = mixed ? e->rs : e->r64;
        void* tt = mixed ? e->t : e->t64;
        void* ad = mixed ? e->Ad : e->Ad64;
        if (which == 0)
            return enqueue_hop(g, prec, N > 1 ? 1 : t.S1, N, EPI_PLAIN, t, dd, rs, tt, rs, 1, nullptr,
                               0, nullptr, 0, nullptr, e->st, F_ACTIVE, nullptr, s, rr, rs);
        if (which == 1)
            return enqueue_hop(g, prec, N > 1 ? 1 : t.S2, N, EPI_XPAY_DOT, t, tt, rs, ad, rs, 0, dd,
                               rs, nullptr, 0, nullptr, e->st, F_ACTIVE, &red, s, rr, rs);
        VecArgs a{};
        if (mixed) {
            void* f[] = {e->y32, e->rs, e->d, e->Ad};
            size_t r4[] = {e->rs32, e->rsP, e->rsP, e->rsP};
            for (int k = 0; k < 4; ++k) {
                a.f[k] = f[k];
                a.rs[k] = r4[k];
            }
        } else {
            void* f[] = {e->x64, e->r64, e->d64, e->Ad64};
            for (int k = 0; k < 4; ++k) {
                a.f[k] = f[k];
                a.rs[k] = e->rs64;
            }
        }
        a.Vh = e->Vh;
        a.st = e->st;
        a.run_mask = F_ACTIVE;
        a.swizzle = e->tune_lo.swizzle;
        a.red = red;
        return launch_vec(prec, N, mixed ? OP_UPD_MIXED : OP_UPD_CG, a, s);
    };
    for (int which = 0; which < 3 && err == hipSuccess; ++which) {
        for (int i = 0; i < 3 && err == hipSuccess; ++i) err = one(which);  // warm-up
        if (err == hipSuccess) err = hipEventRecord(e0, s);
        for (int i = 0; i < reps && err == hipSuccess; ++i) err = one(which);
        if (err == hipSuccess) err = hipEventRecord(e1, s);
        if (err == hipSuccess) err = hipEventSynchronize(e1);
        float ms = 0.f;
        if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
        us_out[which] = ms * 1e3 / reps;
    }
    if (sink) (void)hipFreeAsync(sink, s);
    (void)hipStreamSynchronize(s);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    // the state was overwritten: mark every slot free for the next solve
    (void)hipMemsetAsync(e->st, 0, sizeof(RhsState) * N, s);
    (void)hipStreamSynchronize(s);
    engine_release(e);
    if (err != hipSuccess) {
        (void)hipGetLastError();
        return set_error(ctx, STAG_EDEVICE, "stag_time_kernels: %s", hipGetErrorString(err));
    }
    return STAG_OK;
}
