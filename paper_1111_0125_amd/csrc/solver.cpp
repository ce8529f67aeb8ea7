// CG solver engine: plain fp64 CG (Fig.1) and the corrected mixed-precision
// CG of Sec.3.2 (low-precision inner iterations, fp64 reliable + group-wise
// updates, direction carried over as in Eq.6), for a block of right-hand
// sides ("slots") that share every link load.
//
// All CG scalars live on the device (RhsState); each reduction is finalised
// at the start of the kernel that consumes it, so an iteration is three
// kernels with no host round trip. The host enqueues blocks of K iterations
// (one HIP graph replay) and polls the per-slot flags one block behind the
// device. Every few iterations a block runs the fp64 fix-up (true-residual
// check of plain CG, reliable + group-wise update of mixed CG), predicated
// on the flags: it works only on the slots that asked for it.
//
// Slots are independent: a slot can start (from x = 0) at any block
// boundary while others are mid-solve, and its arithmetic does not depend on
// the other slots or on the kernel's block size N, so a solve gives the same
// bits alone and in a mix. stag_cg_solve runs one batch of slots to the
// end; the serving loop (serve.cpp) keeps slots busy continuously.
#include <chrono>
#include <cmath>
#include <cstring>
#include <limits>

#include "internal.h"

namespace stag {

static size_t state_bytes(int N) { return sizeof(RhsState) * (size_t)N; }

void engine_drop_graphs(stag_engine* e) {
    for (auto& kv : e->graphs)
        if (kv.second) (void)hipGraphExecDestroy(kv.second);
    e->graphs.clear();
}

void engine_destroy(stag_engine* e) {
    if (!e) return;
    stag_ctx* ctx = e->ctx;
    engine_drop_graphs(e);
    void* bufs[] = {e->x64, e->r64, e->t64, e->d64, e->Ad64, e->y32, e->rs, e->d, e->t, e->Ad,
                    e->b64, e->st, e->st1, e->partials, e->partials1};
    for (void* p : bufs)
        if (p) (void)hipFree(p);
    for (int i = 0; i < 2; ++i) {
        if (e->host[i]) (void)hipHostFree(e->host[i]);
        if (e->ev[i]) (void)hipEventDestroy(e->ev[i]);
    }
    if (e->hstage) (void)hipHostFree(e->hstage);
    ctx->used.fetch_sub(e->bytes);
    delete e;
}

int engine_create(stag_ctx* ctx, const stag_gauge* g, int prec, int N, bool serving,
                  hipStream_t init_stream, stag_engine** out) {
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
        {(void**)&e->st, state_bytes(N)}, {(void**)&e->st1, state_bytes(N)},
        {(void**)&e->partials, N * nparts * sizeof(double)},
        {(void**)&e->partials1, N * nparts * sizeof(double)},
    };
    // the right-hand sides live in the engine: the fix-up kernels captured in
    // the iteration graphs read them, so their address must not change
    reqs.push_back({&e->b64, N * e->rs64});
    e->serving = serving;
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
    if (hipHostMalloc((void**)&e->hstage, state_bytes(N), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        engine_destroy(e);
        return set_error(ctx, STAG_EDEVICE, "solver workspace: pinned staging");
    }
    // Every slot starts free, and the direction / y buffers must hold finite
    // values (beta = 0 multiplies them). Cleared on the given stream, which
    // is then waited for (only it: other streams' work is not held up), so
    // whatever stream the engine is used on later sees the cleared buffers.
    hipStream_t s = init_stream;
    hipError_t err = hipMemsetAsync(e->st, 0, state_bytes(N), s);
    if (err == hipSuccess) err = hipMemsetAsync(e->st1, 0, state_bytes(N), s);
    if (err == hipSuccess && e->d64) err = hipMemsetAsync(e->d64, 0, N * e->rs64, s);
    if (err == hipSuccess && e->d) err = hipMemsetAsync(e->d, 0, N * e->rsP, s);
    if (err == hipSuccess && e->y32) err = hipMemsetAsync(e->y32, 0, N * e->rs32, s);
    if (err == hipSuccess) err = hipStreamSynchronize(s);
    if (err != hipSuccess) {
        (void)hipGetLastError();
        engine_destroy(e);
        return set_error(ctx, STAG_EDEVICE, "solver workspace: init");
    }
    e->tune_lo = get_tune(ctx, prec, pick_n(N), e->Vh, g->npairs);
    e->tune_64 = get_tune(ctx, P64, pick_n(N), e->Vh, g->npairs);
    *out = e;
    return STAG_OK;
}

int engine_acquire(stag_ctx* ctx, const stag_gauge* g, int prec, int N, stag_engine** out) {
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        for (auto* e : ctx->engines)
            if (!e->in_use && e->gauge == g && e->prec == prec && e->N == N && !e->serving) {
                e->in_use = true;
                *out = e;
                return STAG_OK;
            }
    }
    stag_engine* e = nullptr;
    int rc = engine_create(ctx, g, prec, N, false, ctx->stream, &e);
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

// Finalising a reduction at the start of its consumer costs every wave (one
// RHS) or every block (several) one pass over all the chunk partials of the
// RHS it serves. That pays on small lattices, where a separate one-block
// kernel and its launch would be a large part of an iteration, and not on
// large ones, where the passes would add up to a sizeable fraction of the
// kernel's own traffic. Above this many partials per consumer the reduction
// is finalised by a one-block kernel and consumers read the state.
constexpr size_t kFuseMaxPartials = 2048;

// Kernels of any number of right-hand sides run the direction update as
// its own pass from this many sites per parity on, and blocks of 8 on any
// lattice (measured: at 16^3x32 with 8 RHS the hop stages gain 13 us for a
// ~7 us pass, with 2 or 4 RHS the pass costs what it saves; at 32^3x64 with
// one RHS an fp16+scale iteration takes 17 % less and an fp32 one 1 % less).
constexpr uint32_t kXpayMinSites = 131072;
constexpr int kXpayMinRhs = 8;

bool fuse_finalize(const stag_engine* e, int nk) {
    return (size_t)num_chunks(e->Vh) * (size_t)nk <= kFuseMaxPartials;
}

namespace {

struct Ctx {
    stag_engine* e;
    Issue is;     // a stream, or a graph under construction
    int nk;       // kernel block size (>= highest busy slot + 1)
    bool timed;   // eager only: bracket each kernel with timing events
    int variant;  // mixed CG variant of the run (MixedVariant)
};

// Launch `fn` (one kernel) with timing events recorded at the kernel's
// start and end (hipExtLaunchKernel) when the run is timed.
template <typename F>
hipError_t timed_launch(const Ctx& c, int kind, F&& fn) {
    if (!c.timed) return fn();
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t err = timing_events(c.e->ctx, &a, &b);
    if (err != hipSuccess) return err;
    Issue& is = const_cast<Issue&>(c.is);  // eager launches only: no graph is being built
    is.ev_start = a;
    is.ev_stop = b;
    err = fn();
    is.ev_start = is.ev_stop = nullptr;
    if (err != hipSuccess) return err;
    timing_push(c.e->ctx, kind, a, b);
    return hipSuccess;
}

Reduce make_red(stag_engine* e, int kind, double* partials = nullptr) {
    Reduce r{};
    r.partials = partials ? partials : e->partials;
    r.st = e->st;
    r.out = nullptr;
    r.st_out = nullptr;
    r.kind = kind;
    r.nparts = (int)num_chunks(e->Vh);
    return r;
}

// A reduction produced by a vector kernel: one partial per block of kBlock
// sites (block_partials) instead of one per 64-site chunk.
Reduce make_red_vec(stag_engine* e, int kind, double* partials = nullptr) {
    Reduce r = make_red(e, kind, partials);
    r.nparts = (int)vec_blocks(e->Vh);
    return r;
}

// Optional pieces of a kernel launch inside the solver.
struct Opt {
    RhsState* st = nullptr;          // state read (null: e->st)
    const Reduce* fin = nullptr;     // reduction finalised at kernel start
    bool finalize = true;            // finalise this kernel's reduction right after it
    double* partials = nullptr;      // where this kernel's partials go (null: e->partials)
    const HopExtra* ex = nullptr;    // fp64 stages of a reliable update
};

// A hop stage. With Opt::finalize, a reduction it produces (XPAY_DOT,
// RESID) is finalised in place on e->st by a one-block kernel right after.
hipError_t hop(const Ctx& c, int prec, int stage, int epi, const void* in, void* out,
               const void* x, int kind, unsigned run, const void* lazy_r = nullptr,
               const Opt& o = Opt()) {
    stag_engine* e = c.e;
    const HopTune& t = prec == P64 && e->prec != P64 ? e->tune_64 : e->tune_lo;
    const int S = stage == 1 ? t.S1 : t.S2;
    const size_t rs = spinor_rhs_bytes(prec, e->Vh);
    Reduce red = make_red(e, kind, o.partials);
    RhsState* st = o.st ? o.st : e->st;
    const int p_out = stage == 1 ? 1 : 0;
    const int kk = prec == e->prec && run == F_ACTIVE ? (stage == 1 ? KK_HOP1 : KK_HOP2)
                                                       : (stage == 1 ? KK_HOP1_64 : KK_HOP2_64);
    hipError_t err = timed_launch(c, kk, [&]() {
        return enqueue_hop(e->gauge, prec, S, c.nk, epi, t, in, rs, out, rs, p_out, x, rs, e->b64,
                           e->rs64, nullptr, st, run, &red, c.is, lazy_r, rs, o.fin, o.ex);
    });
    if (err != hipSuccess || !o.finalize || !(epi == EPI_XPAY_DOT || epi == EPI_RESID)) return err;
    return timed_launch(c, KK_OTHER, [&]() { return launch_finalize(c.nk, red, run, c.is); });
}

hipError_t vec(const Ctx& c, int prec, int op, std::initializer_list<std::pair<void*, size_t>> f,
               int kind, unsigned run, const Opt& o = Opt()) {
    stag_engine* e = c.e;
    VecArgs a{};
    int k = 0;
    for (auto& p : f) {
        a.f[k] = p.first;
        a.rs[k] = p.second;
        ++k;
    }
    a.Vh = e->Vh;
    a.st = o.st ? o.st : e->st;
    a.run_mask = run;
    a.swizzle = e->tune_lo.swizzle;
    a.red = make_red_vec(e, kind, o.partials);
    if (o.fin) a.fin = *o.fin;
    const int kk = op == OP_UPD_CG || op == OP_UPD_MIXED ? KK_UPDATE : KK_OTHER;
    hipError_t err = timed_launch(c, kk, [&]() { return launch_vec(prec, c.nk, op, a, c.is); });
    if (err != hipSuccess || !o.finalize || !(op == OP_INIT_B || op == OP_UPD_CG || op == OP_UPD_MIXED))
        return err;
    return timed_launch(c, KK_OTHER, [&]() { return launch_finalize(c.nk, a.red, run, c.is); });
}

// Large lattices, and blocks of 8 or more right-hand sides: the direction
// update d = q(r + beta d) as a pass of its own before stage 1, which then
// gathers one field per neighbour and right-hand side instead of two (the
// gathers, not the compulsory traffic, bound the block hop kernels there)
// and forms no direction (with fp16+scale storage every neighbour's d must
// be re-encoded to the bits stage 2 stores: eight encodes per site, each
// with six divisions, kept stage 1 far below its bandwidth bound); stage 2
// reads d as stored. Four kernels per iteration, bitwise the same results.
bool separate_xpay(const stag_engine* e, int nk) {
    return nk >= kXpayMinRhs || e->Vh >= kXpayMinSites;
}

hipError_t enqueue_iterations_xpay(const Ctx& c, int K) {
    stag_engine* e = c.e;
    const bool mixed = e->prec != P64;
    const int P = e->prec;
    const int kind_r = mixed ? FIN_MIXED : FIN_CG;
    void* d = mixed ? e->d : e->d64;
    void* t = mixed ? e->t : e->t64;
    void* ad = mixed ? e->Ad : e->Ad64;
    void* r = mixed ? e->rs : e->r64;
    const size_t rs = mixed ? e->rsP : e->rs64;
    const bool fuse = fuse_finalize(e, c.nk);
    Reduce pend_r = make_red_vec(e, kind_r, e->partials1);
    pend_r.st = e->st1;
    pend_r.st_out = e->st;
    Reduce pend_a = make_red(e, FIN_ALPHA, e->partials);
    pend_a.st = e->st;
    pend_a.st_out = e->st1;
    hipError_t err;
    for (int k = 0; k < K; ++k) {
        Opt ox;
        if (fuse && k > 0) {
            ox.st = e->st1;
            ox.fin = &pend_r;
        }
        if ((err = timed_launch(c, KK_XPAY, [&]() {
                 VecArgs a{};
                 a.f[0] = r;
                 a.rs[0] = rs;
                 a.f[1] = d;
                 a.rs[1] = rs;
                 a.Vh = e->Vh;
                 a.st = ox.st ? ox.st : e->st;
                 a.run_mask = F_ACTIVE;
                 a.swizzle = e->tune_lo.swizzle;
                 if (ox.fin) a.fin = *ox.fin;
                 return launch_vec(P, c.nk, OP_XPAY, a, c.is);
             })))
            return err;
        if ((err = hop(c, P, 1, EPI_PLAIN, d, t, nullptr, FIN_STORE, F_ACTIVE))) return err;
        Opt o2;
        o2.finalize = !fuse;
        if ((err = hop(c, P, 2, EPI_XPAY_DOT, t, ad, d, FIN_ALPHA, F_ACTIVE, nullptr, o2))) return err;
        Opt ou;
        if (fuse) {
            ou.fin = &pend_a;
            ou.finalize = false;
            ou.partials = e->partials1;
        }
        if (mixed) {
            err = vec(c, P, OP_UPD_MIXED,
                      {{e->y32, e->rs32}, {e->rs, e->rsP}, {e->d, e->rsP}, {e->Ad, e->rsP}},
                      kind_r, F_ACTIVE, ou);
        } else {
            err = vec(c, P64, OP_UPD_CG,
                      {{e->x64, e->rs64}, {e->r64, e->rs64}, {e->d64, e->rs64}, {e->Ad64, e->rs64}},
                      kind_r, F_ACTIVE, ou);
        }
        if (err) return err;
    }
    if (!fuse) return hipSuccess;
    return timed_launch(c, KK_OTHER, [&]() { return launch_finalize(c.nk, pend_r, F_ACTIVE, c.is); });
}

// K CG iterations (Fig.1; Sec.3.2 for a low-precision inner solve), three
// kernels each:
//   stage 1  t = D_oe d, where d = r + beta d (the previous iteration's
//            direction update, deferred) is formed at every neighbour;
//   stage 2  d stored, Ad = m^2 d - D_eo t, chunk partials of <d, Ad>;
//   update   alpha = |r|^2 / <d, Ad>, x (or y) += alpha d, r -= alpha Ad,
//            chunk partials of |r|^2.
// Fused (small lattices): alpha is finalised at the start of the update, the
// |r|^2 of one update (beta, convergence and update triggers) at the start
// of the next iteration's stage 1, and by a one-block kernel after the last
// iteration, which leaves the state in e->st. A many-block kernel that
// finalises reads one state buffer and its block 0 writes the other (update:
// st -> st1, stage 1: st1 -> st), and the two reductions use separate
// partial buffers, so no kernel reads what it writes. Not fused (large
// lattices): a one-block kernel finalises each reduction in place right
// after the kernel that produced it.
hipError_t enqueue_iterations(const Ctx& c, int K) {
    stag_engine* e = c.e;
    const bool mixed = e->prec != P64;
    const int P = e->prec;
    const int kind_r = mixed ? FIN_MIXED : FIN_CG;
    void* d = mixed ? e->d : e->d64;
    void* t = mixed ? e->t : e->t64;
    void* ad = mixed ? e->Ad : e->Ad64;
    void* r = mixed ? e->rs : e->r64;
    const bool fuse = fuse_finalize(e, c.nk);
    if (separate_xpay(e, c.nk)) return enqueue_iterations_xpay(c, K);
    Reduce pend_r = make_red_vec(e, kind_r, e->partials1);
    pend_r.st = e->st1;
    pend_r.st_out = e->st;
    Reduce pend_a = make_red(e, FIN_ALPHA, e->partials);
    pend_a.st = e->st;
    pend_a.st_out = e->st1;
    hipError_t err;
    for (int k = 0; k < K; ++k) {
        Opt o1;
        if (fuse && k > 0) {
            o1.st = e->st1;
            o1.fin = &pend_r;
        }
        if ((err = hop(c, P, 1, EPI_PLAIN, d, t, nullptr, FIN_STORE, F_ACTIVE, r, o1))) return err;
        Opt o2;
        o2.finalize = !fuse;
        if ((err = hop(c, P, 2, EPI_XPAY_DOT, t, ad, d, FIN_ALPHA, F_ACTIVE, r, o2))) return err;
        Opt ou;
        if (fuse) {
            ou.fin = &pend_a;
            ou.finalize = false;
            ou.partials = e->partials1;
        }
        if (mixed) {
            err = vec(c, P, OP_UPD_MIXED,
                      {{e->y32, e->rs32}, {e->rs, e->rsP}, {e->d, e->rsP}, {e->Ad, e->rsP}},
                      kind_r, F_ACTIVE, ou);
        } else {
            err = vec(c, P64, OP_UPD_CG,
                      {{e->x64, e->rs64}, {e->r64, e->rs64}, {e->d64, e->rs64}, {e->Ad64, e->rs64}},
                      kind_r, F_ACTIVE, ou);
        }
        if (err) return err;
    }
    if (!fuse) return hipSuccess;
    return timed_launch(c, KK_OTHER, [&]() { return launch_finalize(c.nk, pend_r, F_ACTIVE, c.is); });
}

// Plain CG (Fig.1): the iterated residual of the slots flagged F_CONV met
// the tolerance; r = b - A x in fp64 and |r|^2, then (finalisation) finish,
// or restart from the true residual with d = r.
hipError_t enqueue_check(const Ctx& c) {
    stag_engine* e = c.e;
    const unsigned run = F_CONV;
    hipError_t err;
    if ((err = hop(c, P64, 1, EPI_PLAIN, e->x64, e->t64, nullptr, FIN_STORE, run))) return err;
    return hop(c, P64, 2, EPI_RESID, e->t64, e->r64, e->x64, FIN_CG_CHECK, run);
}

// Mixed CG (Sec.3.2): reliable + group-wise update of the slots flagged
// F_RU or F_STALL, three kernels: the fp64 stage 1 gathers x + y; stage 2
// stores x += y and y = 0 at its own site, forms r = b - A x with |r|^2 and
// stores the inner residual q(r); the finalisation then finishes the slot
// or carries the direction over (Eq.6), restarting it after a stall.
// Ablations splitting the update into its two ingredients: residual
// replacement alone keeps y (r = b - A (x + y), the solution stays fp32);
// folding alone (x += y, y = 0) leaves r as iterated and checks the true
// residual only once the iterated one has met the tolerance.
hipError_t enqueue_update(const Ctx& c) {
    stag_engine* e = c.e;
    const unsigned run = F_RU | F_STALL;
    hipError_t err;
    if (c.variant == MIXED_FOLD_ONLY) {
        if ((err = vec(c, e->prec, OP_FOLD, {{e->x64, e->rs64}, {e->y32, e->rs32}}, FIN_STORE, run)))
            return err;
        Reduce gw = make_red(e, FIN_FOLD);
        gw.nparts = 0;  // a state transition: nothing to sum
        if ((err = timed_launch(c, KK_OTHER, [&]() { return launch_finalize(c.nk, gw, run, c.is); })))
            return err;
        if ((err = hop(c, P64, 1, EPI_PLAIN, e->x64, e->t64, nullptr, FIN_STORE, F_CHECK))) return err;
        return hop(c, P64, 2, EPI_RESID, e->t64, e->r64, e->x64, FIN_FOLD_CHECK, F_CHECK);
    }
    HopExtra x1;
    x1.lazy_y = e->y32;
    x1.lazy_y_rs = e->rs32;
    HopExtra x2 = x1;
    x2.aux = e->rs;
    x2.aux_rs = e->rsP;
    x2.aux_prec = e->prec;
    x2.keep_y = c.variant == MIXED_RELIABLE ? 1 : 0;
    Opt o1, o2;
    o1.ex = &x1;
    o2.ex = &x2;
    if ((err = hop(c, P64, 1, EPI_PLAIN, e->x64, e->t64, nullptr, FIN_STORE, run, nullptr, o1)))
        return err;
    return hop(c, P64, 2, EPI_RESID, e->t64, e->r64, e->x64, FIN_RU_END, run, nullptr, o2);
}

// One block: K iterations in segments of at most F, each segment followed by
// the fix-up of the slots it flagged (predicated on the flags: a no-op for
// the others), so a flagged slot waits at most F iterations.
hipError_t enqueue_block_group(const Ctx& c, int K, int F) {
    const bool mixed = c.e->prec != P64;
    hipError_t err;
    for (int done = 0; done < K; done += F) {
        if ((err = enqueue_iterations(c, std::min(F, K - done)))) return err;
        if ((err = mixed ? enqueue_update(c) : enqueue_check(c))) return err;
    }
    return hipSuccess;
}

// The engine as the kernels of slots [g0, ...) see it: every slot-strided
// buffer, state and partial array starts at slot g0 (launch shapes for
// kernels of nk right-hand sides).
void slot_view(const stag_engine* e, int g0, int nk, stag_engine* v) {
    v->ctx = e->ctx;
    v->gauge = e->gauge;
    v->prec = e->prec;
    v->N = e->N - g0;
    v->Vh = e->Vh;
    v->rs64 = e->rs64;
    v->rsP = e->rsP;
    v->rs32 = e->rs32;
    auto off = [g0](void* p, size_t rs) -> void* {
        return p ? (void*)((char*)p + (size_t)g0 * rs) : nullptr;
    };
    v->x64 = off(e->x64, e->rs64);
    v->r64 = off(e->r64, e->rs64);
    v->t64 = off(e->t64, e->rs64);
    v->d64 = off(e->d64, e->rs64);
    v->Ad64 = off(e->Ad64, e->rs64);
    v->b64 = off(e->b64, e->rs64);
    v->y32 = off(e->y32, e->rs32);
    v->rs = off(e->rs, e->rsP);
    v->d = off(e->d, e->rsP);
    v->t = off(e->t, e->rsP);
    v->Ad = off(e->Ad, e->rsP);
    v->st = e->st + g0;
    v->st1 = e->st1 + g0;
    const size_t np = num_chunks(e->Vh);
    v->partials = e->partials + (size_t)g0 * np;
    v->partials1 = e->partials1 + (size_t)g0 * np;
    v->tune_lo = get_tune(e->ctx, e->prec, nk, e->Vh, e->gauge->npairs);
    v->tune_64 = get_tune(e->ctx, P64, nk, e->Vh, e->gauge->npairs);
}

// Block kernels serve at most this many right-hand sides: per right-hand
// side an iteration costs less with 8 per kernel than with 12 or 16 (whose
// neighbour gathers miss the caches more), so larger batches run as groups
// of 8 (and the rest), each its own chain of kernels.
constexpr int kMaxGroup = 8;
// The groups' chains overlap on the device. Below kSmallGroupSites sites per
// parity a kernel leaves room for another chain's, and blocks of up to
// kSmallGroupRhs right-hand sides run as groups of kSmallGroup: 8 and 12 RHS
// 10-14 % faster per solve on 16^3 x 32 and 7-10 % on 24^3 x 48 than as 8 and
// 8 + 4; on 32^3 x 64 and for 16 RHS groups of 8 measured as fast or faster.
constexpr int kSmallGroup = 4;
constexpr int kSmallGroupRhs = 12;
constexpr uint32_t kSmallGroupSites = 524288;

int group_size(const stag_engine* e, int nk) {
    return nk <= kSmallGroupRhs && e->Vh < kSmallGroupSites ? kSmallGroup : kMaxGroup;
}

// One block (K iterations with their fix-ups) for the slots below nk. In a
// graph the groups are independent branches.
hipError_t enqueue_block(const Ctx& c, int K, int F) {
    const int gs = group_size(c.e, c.nk);
    if (c.nk <= gs) return enqueue_block_group(c, K, F);
    hipError_t err = hipSuccess;
    for (int g0 = 0; g0 < c.nk && err == hipSuccess; g0 += gs) {
        const int nk = pick_n(std::min(gs, c.nk - g0));
        stag_engine v;
        slot_view(c.e, g0, nk, &v);
        Ctx cg = c;
        cg.e = &v;
        cg.nk = nk;
        if (c.is.gb) c.is.gb->last = nullptr;  // a new branch from the graph's start
        err = enqueue_block_group(cg, K, F);
    }
    return err;
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
    return (f & (F_DONE | F_BADINPUT | F_BREAKDOWN | F_ESTALL | F_INACC)) ||
           ((f & F_MAXIT) && !(f & (F_CONV | F_RU | F_CHECK)));
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
    // plain CG checks its true residual once per block (it converges once);
    // mixed CG updates every ~tens of iterations, so a flagged slot should
    // not idle for a whole block
    R.F = e->prec == P64 ? K : std::min(K, 8);
    R.use_graph = use_graph;
    R.timed = e->ctx->timing.on;
    if (R.timed) R.use_graph = false;  // timing events bracket eager launches
    R.launched = R.polled = 0;
    R.start_after.assign(e->N, -1);
    R.last_poll = -1;
    R.busy_hi = 0;
}

int default_graph_k(uint32_t Vh) { return Vh >= 262144 ? 16 : (Vh >= 32768 ? 32 : 64); }

// Start the given slots, from x = 0 or from an initial guess x0: per-slot
// initial state, r = b and |b|^2 (FIN_INIT), for x0 slots r = b - A x0 in
// fp64 and its norm (FIN_X0), then the first direction d = r (rounded to the
// inner precision, y = 0) and the switch to F_ACTIVE. b = 0 finishes a slot
// at once (FIN_INIT: F_DONE), a non-finite b with F_BADINPUT.
// The state of a slot about to start (before FIN_INIT).
static void start_state(const stag_engine* e, double mass, const stag_cg_params& p, bool x0,
                        bool escalating, RhsState& s) {
    const uint64_t n_unknowns = 3ull * e->Vh;
    std::memset(&s, 0, sizeof(s));
    s.tol2 = p.tol * p.tol;
    s.m2 = mass * mass;
    s.delta = p.delta > 0 ? p.delta : 0.1;
    // the stall safeguard is for fp16 storage; fp32 runs without it
    s.stall_iters = p.stall_iters > 0 ? p.stall_iters
                                      : (e->prec == P16S ? 100 : std::numeric_limits<int>::max());
    s.max_stall = p.max_stall > 0 ? p.max_stall : 20;
    s.max_iter = p.max_iter > 0 ? p.max_iter : (int)std::min<uint64_t>(10 * n_unknowns, 1000000);
    s.flags = F_NEW | (x0 ? F_X0 : 0u);
    s.variant = p.mixed_variant;
    // an fp16-storage pass with somewhere to go hands over as soon as a
    // refinement cycle fails to halve the true residual, or the pass falls
    // far behind the iterations CG needs on the system
    s.slow_ratio = escalating && e->prec == P16S ? kSlowCycleRatio : 0.0;
    s.cg_budget = escalating && e->prec == P16S ? kCgBudget : 0.0;
}

int run_start_slots(EngineRun& R, const std::vector<SlotInit>& slots) {
    stag_engine* e = R.e;
    if (slots.empty()) return STAG_OK;
    bool any_x0 = false;
    for (const SlotInit& si : slots) {
        RhsState& s = e->hstage[si.slot];
        const bool x0 = si.x0 != nullptr || si.x0_in_place;
        start_state(e, si.mass, si.params, x0, si.escalating, s);
        RCK(hipMemcpyAsync(e->st + si.slot, &s, sizeof(RhsState), hipMemcpyHostToDevice, R.s));
        if (si.x0 && !si.x0_in_place)
            RCK(hipMemcpyAsync((char*)e->x64 + (size_t)si.slot * e->rs64, si.x0, e->rs64,
                               hipMemcpyDeviceToDevice, R.s));
        any_x0 |= x0;
        if (si.slot + 1 > R.busy_hi) R.busy_hi = si.slot + 1;
        // polls of blocks launched before this start show the slot's previous state
        R.start_after[si.slot] = R.launched - 1;
    }
    Ctx c{e, Issue{R.s}, pick_n(R.busy_hi), R.timed, R.variant};
    void* b = const_cast<void*>(R.b);
    RCK(vec(c, P64, OP_INIT_B, {{b, R.b_rs}, {e->r64, e->rs64}, {e->x64, e->rs64}}, FIN_INIT, F_NEW));
    if (any_x0) {
        RCK(hop(c, P64, 1, EPI_PLAIN, e->x64, e->t64, nullptr, FIN_STORE, F_X0));
        RCK(hop(c, P64, 2, EPI_RESID, e->t64, e->r64, e->x64, FIN_X0, F_X0));
    }
    if (e->prec != P64) {
        RCK(vec(c, e->prec, OP_START,
                {{e->r64, e->rs64}, {e->d, e->rsP}, {e->rs, e->rsP}, {e->y32, e->rs32}}, FIN_STORE,
                F_NEW));
    } else {
        RCK(vec(c, P64, OP_START, {{e->r64, e->rs64}, {e->d64, e->rs64}, {nullptr, 0}, {nullptr, 0}},
                FIN_STORE, F_NEW));
    }
    Reduce act = make_red(e, FIN_ACTIVATE);
    act.nparts = 0;  // a state transition: nothing to sum
    RCK(timed_launch(c, KK_OTHER, [&]() { return launch_finalize(c.nk, act, F_NEW, c.is); }));
    return STAG_OK;
}

// The graph of one block of work (K iterations with their fix-ups) for
// kernel block size nk, built node by node on first use and kept. Every
// buffer it uses belongs to the engine, so it serves every later block.
static int get_graph(EngineRun& R, int nk, int K, hipGraphExec_t* out) {
    stag_engine* e = R.e;
    const long long key = ((long long)K << 16) | ((long long)R.variant << 8) | (long long)nk;
    auto it = e->graphs.find(key);
    if (it != e->graphs.end()) {
        *out = it->second;
        return STAG_OK;
    }
    GraphBuild gb;
    hipError_t err = hipGraphCreate(&gb.graph, 0);
    if (err == hipSuccess) {
        Issue is;
        is.gb = &gb;
        Ctx c{e, is, nk, false, R.variant};
        err = enqueue_block(c, K, R.F);
    }
    hipGraphExec_t exec = nullptr;
    if (err == hipSuccess) err = hipGraphInstantiate(&exec, gb.graph, nullptr, nullptr, 0);
    if (gb.graph) (void)hipGraphDestroy(gb.graph);
    if (err != hipSuccess) {
        (void)hipGetLastError();
        return set_error(e->ctx, STAG_EDEVICE, "solver: graph construction failed: %s",
                         hipGetErrorString(err));
    }
    e->graphs.emplace(key, exec);
    *out = exec;
    return STAG_OK;
}

// Enqueue one block (K iterations with fix-ups, R.K when K is 0) for the
// busy slots, then the poll of the state.
int run_enqueue_block(EngineRun& R, int K) {
    stag_engine* e = R.e;
    const int nk = pick_n(R.busy_hi > 0 ? R.busy_hi : 1);
    const int k = K > 0 ? K : R.K;
    const long long j = R.launched;
    const int buf = (int)(j % 2);
    if (R.use_graph) {
        hipGraphExec_t exec = nullptr;
        int rc = get_graph(R, nk, k, &exec);
        if (rc) return rc;
        RCK(hipGraphLaunch(exec, R.s));
    } else {
        Ctx c{e, Issue{R.s}, nk, R.timed, R.variant};
        RCK(enqueue_block(c, k, R.F));
    }
    RCK(hipMemcpyAsync(e->host[buf], e->st, state_bytes(e->N), hipMemcpyDeviceToHost, R.s));
    RCK(hipEventRecord(e->ev[buf], R.s));
    R.launched = j + 1;
    return STAG_OK;
}

// Wait for (or, with blocking = false, test) the oldest outstanding poll.
// On success *h points at the polled states (valid until the next block is
// enqueued). Flagged slots need nothing from the host: every block ends its
// segments with the predicated fix-ups. Returns STAG_PENDING when not
// blocking and the poll is not complete yet.
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
    if (R.timed) timing_collect(e->ctx);
    R.polled = j + 1;
    R.last_poll = j;
    const RhsState* st = e->host[buf];
    *h = st;
    return STAG_OK;
}

void fill_stats(const RhsState& s, double secs, int inner_prec, stag_cg_stats* out) {
    out->iters = s.iters;
    out->reliable_updates = s.updates;
    out->restarts = s.restarts;
    out->status = flags_terminal(s.flags) ? status_of_flags(s.flags) : STAG_ENOCONV;
    out->true_rel_res = s.bb > 0 ? std::sqrt(s.rr_true / s.bb) : 0.0;
    out->iter_rel_res = s.bb > 0 ? std::sqrt(s.rr / s.bb) : 0.0;
    out->seconds = secs;
    out->inner_final = inner_prec;
}

// ------------------------------------------------------------------ one-shot solve

// Where one workgroup per right-hand side (tiny.hip) beats the kernel-per-
// stage solver (measured, 1 and 8 RHS): one pass of four lanes per site
// covers the lattice (128 sites per parity, 4^4: 7.3 against 7.8 ms for a
// 1e-10 fp64 solve, 5.2 against 7.4 ms fp32, and 3.5-5x with 8 RHS), or a
// batch of several right-hand sides on up to 648 sites (6^4: 8 RHS in 51
// against 104 ms fp32, 87 against 104 ms fp64). An iteration costs a few
// microseconds of barriers and memory round trips whatever the size, so
// single solves of 6^4 and anything on 8^4 are faster with a kernel per
// stage.
constexpr uint32_t kTinySitesOnePass = 128;
constexpr uint32_t kTinySitesBatch = 648;

static bool tiny_solve_eligible(const stag_engine* e, int n, const stag_cg_params& p) {
    const bool variant_ok = e->prec == P64 || p.mixed_variant == MIXED_CARRY ||
                            p.mixed_variant == MIXED_RESTART;
    const bool size_ok = e->Vh <= kTinySitesOnePass || (n >= 2 && e->Vh <= kTinySitesBatch);
    return p.small_lattice != 0 && size_ok && e->gauge->npairs == 4 && !p.use_x0 && variant_ok &&
           !e->ctx->timing.on;
}

// One-workgroup solves of the n right-hand sides already in e->b64; the final
// states are copied to fin.
static int tiny_solve(stag_engine* e, int n, const double* mass, const stag_cg_params& p,
                      bool escalating, hipStream_t stream, std::vector<RhsState>& fin) {
    const stag_gauge* g = e->gauge;
    const int P = e->prec;
    int max_iter = 0;
    for (int r = 0; r < n; ++r) {
        start_state(e, mass[r], p, false, escalating, e->hstage[r]);
        max_iter = std::max(max_iter, e->hstage[r].max_iter);
    }
    RCK(hipMemcpyAsync(e->st, e->hstage, sizeof(RhsState) * n, hipMemcpyHostToDevice, stream));
    TinyArgs a{};
    for (int q = 0; q < 2; ++q) {
        a.G[q] = g->G[P][q];
        a.gscale[q] = P == P16S ? g->gscale[q] : nullptr;
        a.G64[q] = g->G[P64][q];
    }
    a.r12 = g->r12;
    a.r12_64 = g->r12;
    a.g = g->g;
    a.b64 = e->b64;
    a.x64 = e->x64;
    a.r64 = e->r64;
    a.t64 = e->t64;
    a.rs64 = e->rs64;
    if (P == P64) {
        a.d = e->d64;
        a.t = e->t64;
        a.Ad = e->Ad64;
        a.rs = e->r64;
        a.y = e->x64;
        a.rsP = a.rsY = e->rs64;
    } else {
        a.d = e->d;
        a.t = e->t;
        a.Ad = e->Ad;
        a.rs = e->rs;
        a.y = e->y32;
        a.rsP = e->rsP;
        a.rsY = e->rs32;
    }
    a.st = e->st;
    // every iteration and every fix-up is one loop turn; the state stops at max_iter
    a.cap = (int)std::min<long long>(2ll * max_iter + 64, 1ll << 30);
    RCK(launch_tiny(P, n, a, stream));
    fin.resize(n);
    RCK(hipMemcpyAsync(fin.data(), e->st, sizeof(RhsState) * n, hipMemcpyDeviceToHost, stream));
    RCK(hipStreamSynchronize(stream));
    return STAG_OK;
}

// Copy the solutions out (b = 0 gives x = 0 whatever x0 was) and fill the
// statistics from the final states.
static int engine_solve_finish(stag_engine* e, int n, void* x_out, size_t x_rs,
                               stag_cg_stats* stats, hipStream_t stream,
                               const std::vector<RhsState>& fin,
                               std::chrono::steady_clock::time_point t0) {
    RCK(hipMemcpy2DAsync(x_out, x_rs, e->x64, e->rs64, e->rs64, n, hipMemcpyDeviceToDevice, stream));
    for (int r = 0; r < n; ++r)
        if (fin[r].bb == 0.0 && fin[r].flags == F_DONE)
            RCK(hipMemsetAsync((char*)x_out + (size_t)r * x_rs, 0, e->rs64, stream));
    RCK(hipStreamSynchronize(stream));
    const double secs =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    int rc = STAG_OK;
    for (int r = 0; r < n; ++r) {
        stag_cg_stats s;
        fill_stats(fin[r], secs, e->prec, &s);
        if (stats) stats[r] = s;
        if (rc == STAG_OK && s.status != STAG_OK) rc = s.status;
    }
    if (rc == STAG_EINVAL) set_error(e->ctx, rc, "stag_cg_solve: right-hand side is not finite");
    return rc;
}

// Whether every slot, from its iterated residual at two polls, is predicted
// to meet its tolerance within `budget` more iterations (at the rate between
// the polls). No estimate (no progress, a reliable update in between, a
// finished slot) counts as finished only for terminal slots.
static bool finishes_within(const std::vector<RhsState>& a, const std::vector<RhsState>& b,
                            int budget) {
    if (budget <= 0 || a.size() != b.size()) return false;
    for (size_t r = 0; r < b.size(); ++r) {
        const RhsState& x = a[r];
        const RhsState& y = b[r];
        if (flags_terminal(y.flags)) continue;
        const int kd = y.iters - x.iters;
        if (kd <= 0 || !(y.rr > 0.0) || !(x.rr > y.rr) || !(y.rr_stop > 0.0)) return false;
        if (y.rr <= y.rr_stop) continue;
        if ((double)kd * std::log(y.rr / y.rr_stop) / std::log(x.rr / y.rr) > (double)budget)
            return false;
    }
    return true;
}

int engine_solve(stag_engine* e, int n, const double* mass, const void* b64, size_t b_rs,
                 void* x_out, size_t x_rs, const stag_cg_params& p, stag_cg_stats* stats,
                 hipStream_t stream, bool escalating) {
    const auto t0 = std::chrono::steady_clock::now();
    const int K = p.graph_k > 0 ? p.graph_k : default_graph_k(e->Vh);
    RCK(hipMemcpy2DAsync(e->b64, e->rs64, b64, b_rs, e->rs64, n, hipMemcpyDeviceToDevice, stream));
    std::vector<RhsState> fin(n);
    if (tiny_solve_eligible(e, n, p)) {
        int rc = tiny_solve(e, n, mass, p, escalating, stream, fin);
        if (rc) return rc;
        return engine_solve_finish(e, n, x_out, x_rs, stats, stream, fin, t0);
    }
    EngineRun R;
    run_init(R, e, stream, e->b64, e->rs64, K, p.use_graph != 0);
    R.variant = e->prec != P64 ? p.mixed_variant : MIXED_CARRY;
    std::vector<SlotInit> slots(n);
    for (int r = 0; r < n; ++r) {
        slots[r] = SlotInit{r, mass[r], p};
        if (p.use_x0) slots[r].x0 = (const char*)x_out + (size_t)r * x_rs;
        slots[r].escalating = escalating;
    }
    int rc = run_start_slots(R, slots);
    if (rc) return rc;
    const long long max_blocks = (2ll * (p.max_iter > 0 ? p.max_iter : 1000000)) / R.F + 4096;
    // Blocks are enqueued one ahead of the poll being waited for, so the block
    // after the one that converges runs idle. When the last two polls predict
    // that the block in flight finishes every slot, the next one is short (one
    // segment; results do not depend on how iterations are grouped in blocks).
    std::vector<RhsState> older, newer;
    int k_flight = K;
    rc = run_enqueue_block(R, K);
    if (rc) return rc;
    for (;;) {
        const int k_next = !older.empty() && finishes_within(older, newer, k_flight - R.F) ? R.F : K;
        rc = run_enqueue_block(R, k_next);
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
        older.swap(newer);
        newer.assign(h, h + n);
        k_flight = k_next;
    }
    if (R.variant == MIXED_RELIABLE) {
        // the reliable-update-only ablation never folds y into x: the
        // solution is x + y; report its true residual
        Ctx c{e, Issue{stream}, pick_n(n), R.timed, R.variant};
        const unsigned any = ~0u;
        RCK(vec(c, e->prec, OP_FOLD, {{e->x64, e->rs64}, {e->y32, e->rs32}}, FIN_STORE, any));
        RCK(hop(c, P64, 1, EPI_PLAIN, e->x64, e->t64, nullptr, FIN_STORE, any));
        RCK(hop(c, P64, 2, EPI_RESID, e->t64, e->r64, e->x64, FIN_TRUE, any));
        RCK(hipMemcpyAsync(fin.data(), e->st, sizeof(RhsState) * n, hipMemcpyDeviceToHost, stream));
    }
    RCK(hipStreamSynchronize(stream));
    if (R.timed) timing_collect(e->ctx);
    return engine_solve_finish(e, n, x_out, x_rs, stats, stream, fin, t0);
}

}  // namespace stag

// ------------------------------------------------------------------ kernel timing

namespace stag {

// Average execution time (microseconds, from events recorded at the start
// and the end of each kernel) of the three iteration kernels of engine e
// with tuning t, over `reps` iterations run in order: stage 1 (finalising the
// previous |r|^2 where the solver fuses finalisations), stage 2, update
// (finalising alpha where fused). All of the first
// nrhs slots are active with alpha = beta = 0, so d = r and every vector
// stays put, and the finalisations are FIN_STORE, so the state, and with it
// the work, is the same on every launch. The state is cleared afterwards.
int time_iteration_kernels(stag_engine* e, const HopTune& t, int nrhs, int reps, double* us) {
    stag_ctx* ctx = e->ctx;
    const stag_gauge* g = e->gauge;
    const int N = e->N, prec = e->prec;
    hipStream_t s = ctx->stream;
    for (int r = 0; r < N; ++r) {
        RhsState& st = e->hstage[r];
        std::memset(&st, 0, sizeof(st));
        st.flags = r < nrhs ? F_ACTIVE : 0u;
        st.m2 = 0.01;
        st.rr = 1.0;
    }
    double* sink = nullptr;
    hipError_t err = hipMemcpyAsync(e->st, e->hstage, sizeof(RhsState) * N, hipMemcpyHostToDevice, s);
    if (err == hipSuccess)
        err = hipMemcpyAsync(e->st1, e->hstage, sizeof(RhsState) * N, hipMemcpyHostToDevice, s);
    if (err == hipSuccess) err = hipMallocAsync((void**)&sink, sizeof(double) * N, s);
    const size_t bytes[] = {N * e->rs64, N * e->rsP, N * e->rs32};
    const size_t pbytes = sizeof(double) * N * num_chunks(e->Vh);
    void* zero64[] = {e->x64, e->r64, e->t64, e->d64, e->Ad64};
    void* zeroP[] = {e->rs, e->d, e->t, e->Ad};
    for (void* p : zero64)
        if (err == hipSuccess && p) err = hipMemsetAsync(p, 0, bytes[0], s);
    for (void* p : zeroP)
        if (err == hipSuccess && p) err = hipMemsetAsync(p, 0, bytes[1], s);
    if (err == hipSuccess && e->y32) err = hipMemsetAsync(e->y32, 0, bytes[2], s);
    if (err == hipSuccess) err = hipMemsetAsync(e->partials, 0, pbytes, s);
    if (err == hipSuccess) err = hipMemsetAsync(e->partials1, 0, pbytes, s);
    std::vector<Issue> ev((size_t)(3 * reps), Issue{s});
    for (auto& v : ev) {
        if (err == hipSuccess) err = hipEventCreate(&v.ev_start);
        if (err == hipSuccess) err = hipEventCreate(&v.ev_stop);
    }
    const bool mixed = prec != P64;
    const bool fuse = fuse_finalize(e, N);
    Reduce pend_r = make_red_vec(e, FIN_STORE, e->partials1);
    pend_r.st = e->st1;
    pend_r.st_out = e->st;
    pend_r.out = sink;
    Reduce pend_a = make_red(e, FIN_STORE, e->partials);
    pend_a.st = e->st;
    pend_a.st_out = e->st1;
    pend_a.out = sink;
    auto one = [&](int which, const Issue& is) -> hipError_t {
        Reduce red = make_red(e, FIN_STORE);
        const size_t rs = mixed ? e->rsP : e->rs64;
        void* dd = mixed ? e->d : e->d64;
        void* rr = mixed ? e->rs : e->r64;
        void* tt = mixed ? e->t : e->t64;
        void* ad = mixed ? e->Ad : e->Ad64;
        // blocks on large lattices run the direction update as its own pass
        // (not timed here): their hop stages read d as stored
        const bool xp = separate_xpay(e, N);
        if (which == 0 && xp)
            return enqueue_hop(g, prec, t.S1, N, EPI_PLAIN, t, dd, rs, tt, rs, 1, nullptr, 0,
                               nullptr, 0, nullptr, e->st, F_ACTIVE, nullptr, is);
        if (which == 0)
            return enqueue_hop(g, prec, t.S1, N, EPI_PLAIN, t, dd, rs, tt, rs, 1, nullptr,
                               0, nullptr, 0, nullptr, fuse ? e->st1 : e->st, F_ACTIVE, nullptr, is,
                               rr, rs, fuse ? &pend_r : nullptr);
        if (which == 1)
            return enqueue_hop(g, prec, t.S2, N, EPI_XPAY_DOT, t, tt, rs, ad, rs, 0, dd,
                               rs, nullptr, 0, nullptr, e->st, F_ACTIVE, &red, is,
                               xp ? nullptr : rr, rs);
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
        a.swizzle = t.swizzle;
        a.red = make_red_vec(e, FIN_STORE, e->partials1);
        if (fuse) a.fin = pend_a;
        return launch_vec(prec, N, mixed ? OP_UPD_MIXED : OP_UPD_CG, a, is);
    };
    // in iteration order, each kernel reading what the one before it wrote, as
    // inside a solve (which XCD's L2 holds a vector depends on the block order)
    for (int i = 0; i < 3 && err == hipSuccess; ++i)  // warm-up
        for (int which = 0; which < 3 && err == hipSuccess; ++which) err = one(which, Issue{s});
    for (int i = 0; i < reps && err == hipSuccess; ++i)
        for (int which = 0; which < 3 && err == hipSuccess; ++which)
            err = one(which, ev[(size_t)(3 * i + which)]);
    if (err == hipSuccess) err = hipStreamSynchronize(s);
    for (int which = 0; which < 3 && err == hipSuccess; ++which) {
        double tot = 0.0;
        for (int i = 0; i < reps && err == hipSuccess; ++i) {
            float ms = 0.f;
            const Issue& v = ev[(size_t)(3 * i + which)];
            err = hipEventElapsedTime(&ms, v.ev_start, v.ev_stop);
            tot += ms;
        }
        us[which] = tot * 1e3 / reps;
    }
    if (sink) (void)hipFreeAsync(sink, s);
    (void)hipStreamSynchronize(s);
    for (auto& v : ev) {
        if (v.ev_start) (void)hipEventDestroy(v.ev_start);
        if (v.ev_stop) (void)hipEventDestroy(v.ev_stop);
    }
    // the state was overwritten: mark every slot free for the next solve
    (void)hipMemsetAsync(e->st, 0, sizeof(RhsState) * N, s);
    (void)hipMemsetAsync(e->st1, 0, sizeof(RhsState) * N, s);
    (void)hipStreamSynchronize(s);
    if (err != hipSuccess) {
        (void)hipGetLastError();
        return set_error(ctx, STAG_EDEVICE, "kernel timing: %s", hipGetErrorString(err));
    }
    return STAG_OK;
}

}  // namespace stag

using namespace stag;

extern "C" int stag_time_kernels(stag_ctx* ctx, const stag_gauge* g, int prec, int nrhs, int reps,
                                 double* us_out) {
    if (!ctx) return STAG_EINVAL;
    if (!g || !us_out || prec < 0 || prec > 2 || nrhs < 1 || nrhs > STAG_MAX_RHS || reps < 1 ||
        reps > 100000)
        return set_error(ctx, STAG_EINVAL, "stag_time_kernels: bad argument");
    if (!(g->mask & (1 << prec)) || !(g->mask & STAG_MASK_F64))
        return set_error(ctx, STAG_EINVAL, "stag_time_kernels: gauge lacks a needed copy");
    DeviceGuard dg(ctx->device);
    stag_engine* e = nullptr;
    int rc = engine_acquire(ctx, g, prec, pick_n(nrhs), &e);
    if (rc) return rc;
    rc = time_iteration_kernels(e, e->tune_lo, nrhs, reps, us_out);
    engine_release(e);
    return rc;
}
