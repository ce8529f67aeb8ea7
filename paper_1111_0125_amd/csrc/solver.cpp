// CG solver engine: plain fp64 CG (Fig.1) and the corrected mixed-precision
// CG of Sec.3.2 (low-precision inner iterations, fp64 reliable + group-wise
// updates, direction carried over as in Eq.6), for a block of right-hand
// sides that share every link load.
//
// All CG scalars live on the device (RhsState) and are produced by the last
// block of each reduction, so an iteration is four kernels with no host
// round trip. The host enqueues blocks of K iterations (optionally one HIP
// graph replay), polls the per-RHS flags one block behind the device, and
// enqueues the fp64 true-residual work only when a flag asks for it; those
// kernels are predicated on the flags, so a redundant enqueue is a no-op.
#include <chrono>
#include <cmath>
#include <cstring>

#include "internal.h"

namespace stag {

static size_t state_bytes(int N) { return sizeof(RhsState) * (size_t)N; }

void engine_drop_graphs(stag_engine* e) {
    for (int i = 0; i < 2; ++i) {
        if (e->graph[i]) (void)hipGraphExecDestroy(e->graph[i]);
        e->graph[i] = nullptr;
        for (auto& r : e->gev[i]) {
            (void)hipEventDestroy(r.a);
            (void)hipEventDestroy(r.b);
        }
        e->gev[i].clear();
    }
    e->graph_k = 0;
    e->graph_n = 0;
}

void engine_destroy(stag_engine* e) {
    if (!e) return;
    stag_ctx* ctx = e->ctx;
    engine_drop_graphs(e);
    void* bufs[] = {e->x64, e->r64, e->t64, e->d64, e->Ad64, e->y32, e->rs, e->d, e->t, e->Ad,
                    e->st, e->partials, e->counter};
    for (void* p : bufs)
        if (p) (void)hipFree(p);
    for (int i = 0; i < 2; ++i) {
        if (e->host[i]) (void)hipHostFree(e->host[i]);
        if (e->ev[i]) (void)hipEventDestroy(e->ev[i]);
    }
    ctx->used.fetch_sub(e->bytes);
    delete e;
}

static int engine_create(stag_ctx* ctx, const stag_gauge* g, int prec, int N, stag_engine** out) {
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
        {(void**)&e->counter, 256},
    };
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
    // The reduction counter must start at zero; every reduction kernel's last
    // block resets it, so this is the only clear it needs.
    // hipMemset runs on the null stream, which does not order against the
    // non-blocking streams the solves use: wait for it here.
    if (hipMemset(e->counter, 0, 256) != hipSuccess ||
        hipMemset(e->st, 0, state_bytes(N)) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
        (void)hipGetLastError();
        engine_destroy(e);
        return set_error(ctx, STAG_EDEVICE, "solver workspace: init");
    }
    e->tune_lo = get_tune(ctx, prec, N, e->Vh);
    e->tune_64 = get_tune(ctx, P64, N, e->Vh);
    *out = e;
    return STAG_OK;
}

int engine_acquire(stag_ctx* ctx, const stag_gauge* g, int prec, int N, stag_engine** out) {
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        for (auto* e : ctx->engines)
            if (!e->in_use && e->gauge == g && e->prec == prec && e->N == N) {
                e->in_use = true;
                *out = e;
                return STAG_OK;
            }
    }
    stag_engine* e = nullptr;
    int rc = engine_create(ctx, g, prec, N, &e);
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
    bool timed;
    std::vector<Timing::Rec>* cap;  // non-null while capturing a timed graph
    mutable size_t cap_next;        // next unused record of *cap
};

// Launch `fn` bracketed by timing events when the solve is timed. Inside a
// graph capture the events become external event-record nodes of the graph.
template <typename F>
hipError_t timed_launch(const Ctx& c, int kind, F&& fn) {
    if (!c.timed) return fn();
    if (c.cap) {
        // events were created before the capture began; record them as
        // external event nodes of the graph
        if (c.cap_next + 2 > c.cap->size()) return hipErrorInvalidValue;
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

Reduce make_red(stag_engine* e, int kind, uint32_t nparts) {
    Reduce r{};
    r.partials = e->partials;
    r.counter = e->counter;
    r.st = e->st;
    r.out = nullptr;
    r.kind = kind;
    r.nparts = (int)nparts;
    return r;
}

hipError_t hop(const Ctx& c, int prec, int stage, int epi, const void* in, void* out,
               const void* x, int kind, unsigned run) {
    stag_engine* e = c.e;
    const HopTune& t = prec == P64 && e->prec != P64 ? e->tune_64 : e->tune_lo;
    int S = stage == 1 ? t.S1 : t.S2;
    if (e->N > 1) S = 1;
    const size_t rs = spinor_rhs_bytes(prec, e->Vh);
    Reduce red = make_red(e, kind, num_chunks(e->Vh));
    const int p_out = stage == 1 ? 1 : 0;
    const int kk = prec == e->prec && run == F_ACTIVE ? (stage == 1 ? KK_HOP1 : KK_HOP2)
                                                       : (stage == 1 ? KK_HOP1_64 : KK_HOP2_64);
    return timed_launch(c, kk, [&]() {
        return enqueue_hop(e->gauge, prec, S, e->N, epi, t, in, rs, out, rs, p_out, x, rs, c.b,
                           c.b_rs, nullptr, e->st, run, &red, c.s);
    });
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
    a.red = make_red(e, kind, num_chunks(e->Vh));
    const int kk = op == OP_UPD_CG || op == OP_UPD_MIXED ? KK_UPDATE : op == OP_XPAY ? KK_XPAY : KK_OTHER;
    return timed_launch(c, kk, [&]() { return launch_vec(prec, e->N, op, a, c.s); });
}

hipError_t enqueue_iteration(const Ctx& c) {
    stag_engine* e = c.e;
    hipError_t err;
    if (e->prec == P64) {
        if ((err = hop(c, P64, 1, EPI_PLAIN, e->d64, e->t64, nullptr, FIN_STORE, F_ACTIVE))) return err;
        if ((err = hop(c, P64, 2, EPI_XPAY_DOT, e->t64, e->Ad64, e->d64, FIN_ALPHA, F_ACTIVE))) return err;
        if ((err = vec(c, P64, OP_UPD_CG,
                       {{e->x64, e->rs64}, {e->r64, e->rs64}, {e->d64, e->rs64}, {e->Ad64, e->rs64}},
                       FIN_CG, F_ACTIVE)))
            return err;
        return vec(c, P64, OP_XPAY, {{e->r64, e->rs64}, {e->d64, e->rs64}}, FIN_STORE, F_ACTIVE);
    }
    const int P = e->prec;
    if ((err = hop(c, P, 1, EPI_PLAIN, e->d, e->t, nullptr, FIN_STORE, F_ACTIVE))) return err;
    if ((err = hop(c, P, 2, EPI_XPAY_DOT, e->t, e->Ad, e->d, FIN_ALPHA, F_ACTIVE))) return err;
    if ((err = vec(c, P, OP_UPD_MIXED,
                   {{e->y32, e->rs32}, {e->rs, e->rsP}, {e->d, e->rsP}, {e->Ad, e->rsP}}, FIN_MIXED,
                   F_ACTIVE)))
        return err;
    return vec(c, P, OP_XPAY, {{e->rs, e->rsP}, {e->d, e->rsP}}, FIN_STORE, F_ACTIVE);
}

// fp64 true residual r64 = b - A x64 for the RHS whose flags match `run`.
hipError_t enqueue_true_residual(const Ctx& c, unsigned run) {
    stag_engine* e = c.e;
    hipError_t err;
    if ((err = hop(c, P64, 1, EPI_PLAIN, e->x64, e->t64, nullptr, FIN_STORE, run))) return err;
    return hop(c, P64, 2, EPI_RESID, e->t64, e->r64, e->x64, FIN_TRUE, run);
}

hipError_t enqueue_check(const Ctx& c) {
    stag_engine* e = c.e;
    hipError_t err;
    if ((err = enqueue_true_residual(c, F_CONV))) return err;
    return vec(c, P64, OP_CG_CHECK, {{e->r64, e->rs64}, {e->d64, e->rs64}}, FIN_CG_CHECK, F_CONV);
}

hipError_t enqueue_update(const Ctx& c) {
    stag_engine* e = c.e;
    const unsigned run = F_RU | F_STALL;
    hipError_t err;
    if ((err = vec(c, e->prec, OP_RU_BEGIN, {{e->x64, e->rs64}, {e->y32, e->rs32}}, FIN_STORE, run)))
        return err;
    if ((err = enqueue_true_residual(c, run))) return err;
    return vec(c, e->prec, OP_RU_END, {{e->r64, e->rs64}, {e->rs, e->rsP}, {e->d, e->rsP}},
               FIN_RU_END, run);
}

int status_of(unsigned f) {
    if (f & F_DONE) return STAG_OK;
    if (f & F_BADINPUT) return STAG_EINVAL;
    if (f & F_BREAKDOWN) return STAG_EBREAKDOWN;
    if (f & F_ESTALL) return STAG_ESTALL;
    if (f & F_MAXIT) return STAG_ENOCONV;
    return STAG_ENOCONV;
}

bool terminal(unsigned f) {
    return (f & (F_DONE | F_BADINPUT | F_BREAKDOWN | F_ESTALL)) ||
           ((f & F_MAXIT) && !(f & (F_CONV | F_RU)));
}

}  // namespace

#define ECK(call)                                                                              \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess) {                                                                \
            (void)hipGetLastError();                                                           \
            return set_error(e->ctx, STAG_EDEVICE, "solver: %s: %s", #call, hipGetErrorString(e_)); \
        }                                                                                      \
    } while (0)

int engine_solve(stag_engine* e, int n, const double* mass, const void* b64, size_t b_rs,
                 void* x_out, size_t x_rs, const stag_cg_params& p, stag_cg_stats* stats,
                 hipStream_t stream) {
    const auto t0 = std::chrono::steady_clock::now();
    const int N = e->N;
    const bool mixed = e->prec != P64;
    const bool timed = e->ctx->timing.on;
    Ctx c{e, stream, b64, b_rs, timed, nullptr, 0};
    const uint64_t n_unknowns = 3ull * e->Vh;
    const int max_iter = p.max_iter > 0 ? p.max_iter : (int)std::min<uint64_t>(10 * n_unknowns, 1000000);

    RhsState* h0 = e->host[0];
    std::memset(h0, 0, state_bytes(N));
    for (int r = 0; r < n; ++r) {
        RhsState& s = h0[r];
        s.tol2 = p.tol * p.tol;
        s.m2 = mass[r] * mass[r];
        s.delta = p.delta > 0 ? p.delta : 0.1;
        s.stall_iters = p.stall_iters > 0 ? p.stall_iters : 100;
        s.max_stall = p.max_stall > 0 ? p.max_stall : 20;
        s.max_iter = max_iter;
        s.flags = F_ACTIVE;
    }
    ECK(hipMemcpyAsync(e->st, h0, state_bytes(N), hipMemcpyHostToDevice, stream));
    ECK(vec(c, P64, OP_INIT_B, {{(void*)b64, b_rs}, {e->r64, e->rs64}, {e->x64, e->rs64}}, FIN_INIT,
            F_ACTIVE));
    if (mixed) {
        ECK(vec(c, e->prec, OP_START,
                {{e->r64, e->rs64}, {e->d, e->rsP}, {e->rs, e->rsP}, {e->y32, e->rs32}}, FIN_STORE,
                F_ACTIVE));
    } else {
        ECK(vec(c, P64, OP_START, {{e->r64, e->rs64}, {e->d64, e->rs64}, {nullptr, 0}, {nullptr, 0}},
                FIN_STORE, F_ACTIVE));
    }

    int K = p.graph_k > 0 ? p.graph_k : (e->Vh >= 262144 ? 16 : (e->Vh >= 32768 ? 32 : 64));
    bool use_graph = p.use_graph != 0;
    // A timed solve records event nodes inside its graphs; if the runtime
    // refuses them the solve falls back to eager launches with events.
    if (timed && e->ctx->timing.no_graph_events) use_graph = false;
    int ninst = use_graph ? (timed ? 2 : 1) : 0;
    if (use_graph && (e->graph_k != K || e->graph_n != ninst)) {
        engine_drop_graphs(e);
        bool ok = true;
        for (int inst = 0; inst < ninst && ok; ++inst) {
            Ctx cc = c;
            cc.cap = nullptr;
            if (timed) {
                // 4 kernels per iteration, two events each, created up front
                e->gev[inst].resize((size_t)K * 4);
                for (auto& r : e->gev[inst]) {
                    r.a = r.b = nullptr;
                    if (hipEventCreate(&r.a) != hipSuccess || hipEventCreate(&r.b) != hipSuccess) ok = false;
                }
                cc.cap = &e->gev[inst];
                cc.cap_next = 0;
            }
            if (!ok) break;
            hipGraph_t graph = nullptr;
            ECK(hipStreamBeginCapture(stream, hipStreamCaptureModeRelaxed));
            hipError_t cerr = hipSuccess;
            for (int k = 0; k < K && cerr == hipSuccess; ++k) cerr = enqueue_iteration(cc);
            hipError_t eerr = hipStreamEndCapture(stream, &graph);
            hipError_t ierr = hipErrorInvalidValue;
            if (cerr == hipSuccess && eerr == hipSuccess && graph)
                ierr = hipGraphInstantiate(&e->graph[inst], graph, nullptr, nullptr, 0);
            if (graph) (void)hipGraphDestroy(graph);
            if (ierr != hipSuccess) {
                (void)hipGetLastError();
                e->graph[inst] = nullptr;
                if (!timed)
                    return set_error(e->ctx, STAG_EDEVICE, "solver: graph capture failed: %s",
                                     hipGetErrorString(cerr != hipSuccess ? cerr : eerr != hipSuccess ? eerr : ierr));
                ok = false;
            }
        }
        if (!ok) {
            engine_drop_graphs(e);
            e->ctx->timing.no_graph_events = true;
            use_graph = false;
            ninst = 0;
        } else {
            e->graph_k = K;
            e->graph_n = ninst;
        }
    }
    // timings of the graph instance whose replay has completed
    auto collect_graph = [&](int inst) {
        if (!timed || !use_graph) return;
        Timing& T = e->ctx->timing;
        std::lock_guard<std::mutex> lk(T.mu);
        for (auto& r : e->gev[inst]) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
                T.count[r.kind] += 1;
                T.ms[r.kind] += ms;
            }
            (void)hipGetLastError();
        }
    };

    long long launched = 0;  // blocks launched; block j used instance j % ninst
    auto enqueue_block = [&]() -> hipError_t {
        const long long j = launched++;
        if (use_graph) return hipGraphLaunch(e->graph[j % ninst], stream);
        for (int k = 0; k < K; ++k) {
            hipError_t err = enqueue_iteration(c);
            if (err != hipSuccess) return err;
        }
        return hipSuccess;
    };
    int poll_seq = 0;
    auto enqueue_poll = [&](int buf) -> hipError_t {
        hipError_t err = hipMemcpyAsync(e->host[buf], e->st, state_bytes(N), hipMemcpyDeviceToHost, stream);
        if (err == hipSuccess) err = hipEventRecord(e->ev[buf], stream);
        ++poll_seq;
        return err;
    };

    std::vector<int> fix_after(N, -1);  // poll index from which a fix is visible
    ECK(enqueue_block());
    ECK(enqueue_poll(0));
    int bufA = 0, pollA = 0;
    long long blocks = 1;
    const long long max_blocks = (2ll * max_iter) / K + 4096;
    int final_buf = 0;
    for (;;) {
        ECK(enqueue_block());
        ++blocks;
        const int pollB = poll_seq;
        ECK(enqueue_poll(1 - bufA));
        ECK(hipEventSynchronize(e->ev[bufA]));
        if (timed) {
            timing_collect(e->ctx);
            collect_graph((int)(pollA % (ninst ? ninst : 1)));
        }
        const RhsState* h = e->host[bufA];
        bool all_terminal = true, need = false;
        for (int r = 0; r < n; ++r) {
            const unsigned f = h[r].flags;
            if (terminal(f)) continue;
            all_terminal = false;
            if (pollA <= fix_after[r]) continue;
            if ((!mixed && (f & F_CONV)) || (mixed && (f & (F_RU | F_STALL)))) {
                need = true;
                fix_after[r] = pollB;
            }
        }
        if (all_terminal) {
            final_buf = bufA;
            break;
        }
        if (need) ECK(mixed ? enqueue_update(c) : enqueue_check(c));
        if (blocks > max_blocks) {
            // the device enforces max_iter; this only guards the host loop
            ECK(hipStreamSynchronize(stream));
            ECK(hipMemcpy(e->host[bufA], e->st, state_bytes(N), hipMemcpyDeviceToHost));
            final_buf = bufA;
            break;
        }
        bufA = 1 - bufA;
        pollA = pollB;
    }
    ECK(hipStreamSynchronize(stream));
    if (timed) {
        timing_collect(e->ctx);
        // the last launched block (one past the final poll) has completed too
        if (use_graph && launched > pollA + 1) collect_graph((int)((pollA + 1) % ninst));
    }
    ECK(hipMemcpy2DAsync(x_out, x_rs, e->x64, e->rs64, e->rs64, n, hipMemcpyDeviceToDevice, stream));
    ECK(hipStreamSynchronize(stream));
    const double secs =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    int rc = STAG_OK;
    const RhsState* h = e->host[final_buf];
    for (int r = 0; r < n; ++r) {
        const RhsState& s = h[r];
        const int st = terminal(s.flags) ? status_of(s.flags) : STAG_ENOCONV;
        if (stats) {
            stats[r].iters = s.iters;
            stats[r].reliable_updates = s.updates;
            stats[r].restarts = s.restarts;
            stats[r].status = st;
            stats[r].true_rel_res = s.bb > 0 ? std::sqrt(s.rr_true / s.bb) : 0.0;
            stats[r].iter_rel_res = s.bb > 0 ? std::sqrt(s.rr / s.bb) : 0.0;
            stats[r].seconds = secs;
        }
        if (rc == STAG_OK && st != STAG_OK) rc = st;
    }
    if (rc == STAG_EINVAL) set_error(e->ctx, rc, "stag_cg_solve: right-hand side is not finite");
    return rc;
}

}  // namespace stag
