// Launch-shape autotuner and kernel event timing.
//
// The autotuner times the two hop stages of A on the actual gauge field for
// every launch shape (lanes per site S, non-temporal link loads, XCD-aware
// block order) and keeps the fastest per stage for (precision, RHS block,
// lattice size). All shapes compute bit-identical results (the hop sum and
// the reduction order do not depend on the shape), so tuning never changes
// a solve's iterates.
#include <algorithm>
#include <cstring>

#include "internal.h"

namespace stag {

hipError_t timing_begin(stag_ctx* ctx, hipStream_t s, hipEvent_t* ev) {
    Timing& T = ctx->timing;
    hipEvent_t a = nullptr;
    {
        std::lock_guard<std::mutex> lk(T.mu);
        if (!T.pool.empty()) {
            a = T.pool.back();
            T.pool.pop_back();
        }
    }
    if (!a) {
        hipError_t e = hipEventCreate(&a);
        if (e != hipSuccess) return e;
    }
    *ev = a;
    return hipEventRecord(a, s);
}

hipError_t timing_end(stag_ctx* ctx, hipStream_t s, int kind, hipEvent_t start) {
    Timing& T = ctx->timing;
    hipEvent_t b = nullptr;
    {
        std::lock_guard<std::mutex> lk(T.mu);
        if (!T.pool.empty()) {
            b = T.pool.back();
            T.pool.pop_back();
        }
    }
    if (!b) {
        hipError_t e = hipEventCreate(&b);
        if (e != hipSuccess) return e;
    }
    hipError_t e = hipEventRecord(b, s);
    std::lock_guard<std::mutex> lk(T.mu);
    T.pending.push_back({kind, start, b});
    return e;
}

void timing_collect(stag_ctx* ctx) {
    Timing& T = ctx->timing;
    std::lock_guard<std::mutex> lk(T.mu);
    size_t keep = 0;
    for (size_t i = 0; i < T.pending.size(); ++i) {
        Timing::Rec r = T.pending[i];
        if (hipEventQuery(r.b) == hipSuccess) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess && r.kind >= 0 && r.kind < KK_COUNT) {
                T.count[r.kind] += 1;
                T.ms[r.kind] += ms;
            }
            (void)hipGetLastError();
            T.pool.push_back(r.a);
            T.pool.push_back(r.b);
        } else {
            (void)hipGetLastError();
            T.pending[keep++] = r;
        }
    }
    T.pending.resize(keep);
}

}  // namespace stag

using namespace stag;

extern "C" {

int stag_timing_enable(stag_ctx* ctx, int on) {
    if (!ctx) return STAG_EINVAL;
    DeviceGuard dg(ctx->device);
    (void)hipDeviceSynchronize();
    timing_collect(ctx);
    std::lock_guard<std::mutex> lk(ctx->timing.mu);
    ctx->timing.on = on != 0;
    for (int k = 0; k < KK_COUNT; ++k) {
        ctx->timing.count[k] = 0;
        ctx->timing.ms[k] = 0.0;
    }
    return STAG_OK;
}

int stag_timing_read(stag_ctx* ctx, int kind, int64_t* count, double* total_ms) {
    if (!ctx || !count || !total_ms || kind < 0 || kind >= KK_COUNT) return STAG_EINVAL;
    timing_collect(ctx);
    std::lock_guard<std::mutex> lk(ctx->timing.mu);
    *count = ctx->timing.count[kind];
    *total_ms = ctx->timing.ms[kind];
    return STAG_OK;
}

int stag_tune_get(stag_ctx* ctx, int prec, int nrhs, int64_t vh, stag_tune_cfg* out) {
    if (!ctx || !out || prec < 0 || prec > 2 || nrhs < 1 || nrhs > STAG_MAX_RHS || vh <= 0)
        return STAG_EINVAL;
    HopTune t = get_tune(ctx, prec, pick_n(nrhs), (uint32_t)vh);
    out->S1 = t.S1;
    out->S2 = t.S2;
    out->nt = t.nt;
    out->swizzle = t.swizzle;
    return STAG_OK;
}

static bool valid_S(int S) { return S == 1 || S == 2 || S == 4; }

static void apply_tune_to_engines(stag_ctx* ctx) {
    std::lock_guard<std::mutex> lk(ctx->mu);
    for (auto* e : ctx->engines) {
        if (e->in_use) continue;
        e->tune_lo = get_tune(ctx, e->prec, e->N, e->Vh);
        e->tune_64 = get_tune(ctx, P64, e->N, e->Vh);
        engine_drop_graphs(e);
    }
}

int stag_tune_set(stag_ctx* ctx, int prec, int nrhs, int64_t vh, const stag_tune_cfg* cfg) {
    if (!ctx || !cfg || prec < 0 || prec > 2 || nrhs < 1 || nrhs > STAG_MAX_RHS || vh <= 0)
        return STAG_EINVAL;
    if (!valid_S(cfg->S1) || !valid_S(cfg->S2))
        return set_error(ctx, STAG_EINVAL, "stag_tune_set: S must be 1, 2 or 4");
    HopTune t;
    t.S1 = cfg->S1;
    t.S2 = cfg->S2;
    t.nt = cfg->nt ? 1 : 0;
    t.swizzle = cfg->swizzle ? 1 : 0;
    set_tune(ctx, prec, pick_n(nrhs), (uint32_t)vh, t);
    apply_tune_to_engines(ctx);
    return STAG_OK;
}

int stag_tune(stag_ctx* ctx, const stag_gauge* g, int prec, int nrhs, stag_tune_cfg* best,
              double* best_ms) {
    if (!ctx || !g || prec < 0 || prec > 2 || nrhs < 1 || nrhs > STAG_MAX_RHS)
        return ctx ? set_error(ctx, STAG_EINVAL, "stag_tune: bad argument") : STAG_EINVAL;
    if (!(g->mask & (1 << prec)))
        return set_error(ctx, STAG_EINVAL, "stag_tune: gauge has no copy in precision %d", prec);
    DeviceGuard dg(ctx->device);
    const int N = pick_n(nrhs);
    const uint32_t Vh = g->g.Vh;
    const size_t rs = spinor_rhs_bytes(prec, Vh);
    void *in = nullptr, *t = nullptr, *out = nullptr;
    double* partials = nullptr;
    RhsState* st = nullptr;
    hipStream_t s = ctx->stream;
    auto cleanup = [&]() {
        void* ps[] = {in, t, out, partials, st};
        for (void* p : ps)
            if (p) (void)hipFree(p);
    };
    if (hipMalloc(&in, rs * N) != hipSuccess || hipMalloc(&t, rs * N) != hipSuccess ||
        hipMalloc(&out, rs * N) != hipSuccess ||
        hipMalloc((void**)&partials, sizeof(double) * N * num_chunks(Vh)) != hipSuccess ||
        hipMalloc((void**)&st, sizeof(RhsState) * N) != hipSuccess) {
        (void)hipGetLastError();
        cleanup();
        return set_error(ctx, STAG_ENOMEM, "stag_tune: workspace allocation failed");
    }
    std::vector<RhsState> hst(N);
    std::memset(hst.data(), 0, sizeof(RhsState) * N);
    for (int r = 0; r < N; ++r) {
        hst[r].m2 = 0.01;
        hst[r].flags = F_ACTIVE;
        hst[r].rr = 1.0;
    }
    (void)hipMemset(in, 0, rs * N);
    (void)hipMemcpy(st, hst.data(), sizeof(RhsState) * N, hipMemcpyHostToDevice);
    (void)hipDeviceSynchronize();  // the null-stream writes above must land before s runs
    Reduce red{};
    red.partials = partials;
    red.st = st;
    red.kind = FIN_STORE;
    red.nparts = (int)num_chunks(Vh);
    double* outv = nullptr;
    (void)hipMalloc((void**)&outv, sizeof(double) * N);
    red.out = outv;

    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    const int reps = Vh >= 262144 ? 10 : 30;
    auto time_stage = [&](int stage, const HopTune& tu, int S) -> double {
        auto launch = [&]() -> hipError_t {
            if (stage == 1)
                return enqueue_hop(g, prec, S, N, EPI_PLAIN, tu, in, rs, t, rs, 1, nullptr, 0,
                                   nullptr, 0, nullptr, nullptr, 0, nullptr, s);
            return enqueue_hop(g, prec, S, N, EPI_XPAY_DOT, tu, t, rs, out, rs, 0, in, rs, nullptr,
                               0, nullptr, st, F_ACTIVE, &red, s);
        };
        if (launch() != hipSuccess) return 1e30;
        (void)hipEventRecord(e0, s);
        for (int i = 0; i < reps; ++i) (void)launch();
        (void)hipEventRecord(e1, s);
        (void)hipEventSynchronize(e1);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        (void)hipGetLastError();
        return ms / reps;
    };
    HopTune bestT;
    double best1 = 1e30, best2 = 1e30;
    const int Ss[] = {1, 2, 4};
    for (int nt = 0; nt <= 1; ++nt)
        for (int sw = 0; sw <= 1; ++sw)
            for (int S : Ss) {
                if (N > 1 && S != 1) continue;
                HopTune tu;
                tu.nt = nt;
                tu.swizzle = sw;
                tu.S1 = tu.S2 = S;
                const double t1 = time_stage(1, tu, S);
                const double t2 = time_stage(2, tu, S);
                // one (nt, swizzle) pair serves both stages; S is per stage
                if (t1 + t2 < best1 + best2) {
                    best1 = t1;
                    best2 = t2;
                    bestT = tu;
                }
            }
    // refine S per stage with the chosen (nt, swizzle)
    for (int S : Ss) {
        if (N > 1 && S != 1) continue;
        HopTune tu = bestT;
        const double t1 = time_stage(1, tu, S);
        if (t1 < best1) {
            best1 = t1;
            bestT.S1 = S;
        }
        const double t2 = time_stage(2, tu, S);
        if (t2 < best2) {
            best2 = t2;
            bestT.S2 = S;
        }
    }
    (void)hipStreamSynchronize(s);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (outv) (void)hipFree(outv);
    cleanup();
    set_tune(ctx, prec, N, Vh, bestT);
    apply_tune_to_engines(ctx);
    if (best) {
        best->S1 = bestT.S1;
        best->S2 = bestT.S2;
        best->nt = bestT.nt;
        best->swizzle = bestT.swizzle;
    }
    if (best_ms) *best_ms = best1 + best2;
    return STAG_OK;
}

}  // extern "C"
