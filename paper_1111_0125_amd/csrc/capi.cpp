// C ABI entry points of libstag: contexts, gauges, fields, the Dirac
// operator, A, and the CG solve. Argument validation happens here, before
// any device work; the solver engine is in solver.cpp.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <limits>
#include <cstdio>
#include <cstring>

#include "internal.h"

using namespace stag;

namespace stag {

static thread_local std::string g_create_err;

int set_error(stag_ctx* ctx, int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (ctx) {
        std::lock_guard<std::mutex> lk(ctx->err_mu);
        ctx->err = buf;
    } else {
        g_create_err = buf;
    }
    return code;
}

int dev_alloc(stag_ctx* ctx, size_t bytes, void** p) {
    *p = nullptr;
    if (bytes == 0) return STAG_OK;
    size_t prev = ctx->used.fetch_add(bytes);
    if (ctx->budget && prev + bytes > ctx->budget) {
        ctx->used.fetch_sub(bytes);
        return set_error(ctx, STAG_ENOMEM, "HBM budget exceeded: %zu + %zu > %zu bytes", prev,
                         bytes, ctx->budget);
    }
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        ctx->used.fetch_sub(bytes);
        *p = nullptr;
        (void)hipGetLastError();
        return set_error(ctx, STAG_ENOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
    }
    return STAG_OK;
}

void dev_free(stag_ctx* ctx, void* p, size_t bytes) {
    if (!p) return;
    (void)hipFree(p);
    ctx->used.fetch_sub(bytes);
}

Geom make_geom(const int L[4]) {
    Geom g{};
    for (int i = 0; i < 4; ++i) g.L[i] = L[i];
    const uint64_t V = (uint64_t)L[0] * L[1] * L[2] * L[3];
    g.Vh = (uint32_t)(V / 2);
    g.hx = (uint32_t)(L[0] / 2);
    g.sy = g.hx;
    g.sz = g.hx * (uint32_t)L[1];
    g.st = g.sz * (uint32_t)L[2];
    g.div_hx = make_fastdiv(g.hx);
    g.div_Ly = make_fastdiv((uint32_t)L[1]);
    g.div_Lz = make_fastdiv((uint32_t)L[2]);
    return g;
}

static long long tune_key(int prec, int N, uint32_t Vh, int npairs) {
    int bucket = 0;
    while ((1u << bucket) < Vh && bucket < 31) ++bucket;
    return ((long long)npairs << 48) | ((long long)prec << 40) | ((long long)N << 32) | bucket;
}

HopTune get_tune(stag_ctx* ctx, int prec, int N, uint32_t Vh, int npairs) {
    {
        std::lock_guard<std::mutex> lk(ctx->tune_mu);
        auto it = ctx->tune.find(tune_key(prec, N, Vh, npairs));
        if (it != ctx->tune.end()) return it->second;
    }
    // Default (what the autotuner finds best on most lattices measured, from
    // 16^3x32 to 32^3x64): one lane per site (two for the improved
    // operator's eight hop pairs: the same four pairs per lane, which keeps
    // the link registers of one lane within the register file), non-temporal
    // link loads, XCD-aware block order.
    (void)Vh;
    HopTune t;
    t.S1 = t.S2 = npairs == 8 ? 2 : 1;
    t.nt = 1;
    t.swizzle = 1;
    return t;
}

void set_tune(stag_ctx* ctx, int prec, int N, uint32_t Vh, int npairs, const HopTune& t) {
    std::lock_guard<std::mutex> lk(ctx->tune_mu);
    ctx->tune[tune_key(prec, N, Vh, npairs)] = t;
}

hipError_t enqueue_hop(const stag_gauge* g, int prec, int S, int N, int epi, const HopTune& t,
                       const void* in, size_t in_rs, void* out, size_t out_rs, int p_out,
                       const void* x, size_t x_rs, const void* b, size_t b_rs, const double* m2,
                       RhsState* st, unsigned run_mask, const Reduce* red, const Issue& is,
                       const void* lazy_r, size_t lazy_r_rs, const Reduce* fin,
                       const HopExtra* ex) {
    // the deferred direction update reads beta from the RHS state, and a
    // finalisation at kernel start needs the state and the partials
    if (lazy_r && !st) return hipErrorInvalidValue;
    if (fin && (!st || !fin->partials || fin->nparts < 1)) return hipErrorInvalidValue;
    // reductions and the m^2 update need their buffers
    if ((epi == EPI_XPAY_DOT || epi == EPI_RESID) && (!red || !red->partials)) return hipErrorInvalidValue;
    if (epi != EPI_PLAIN && !x) return hipErrorInvalidValue;
    if (epi == EPI_RESID && !b) return hipErrorInvalidValue;
    HopArgs a{};
    a.lazy_r = lazy_r;
    a.lazy_r_rs = lazy_r_rs;
    a.gauge = g->G[prec][p_out];
    a.gscale = prec == P16S ? g->gscale[p_out] : nullptr;
    a.r12 = g->r12;
    a.npairs = g->npairs;
    a.in = in;
    a.in_rs = in_rs;
    a.out = out;
    a.out_rs = out_rs;
    a.x = x;
    a.x_rs = x_rs;
    a.b = b;
    a.b_rs = b_rs;
    for (int r = 0; r < kMaxN; ++r) a.m2[r] = m2 ? m2[r] : 0.0;
    a.st = st;
    a.run_mask = run_mask;
    // a predicated fp64 launch of one right-hand side (fix-ups and checks,
    // their slot flagged only now and then) looks at the flags before
    // requesting operands; the iteration's own launches request them first,
    // the state's latency overlapping theirs
    a.gate = prec == P64 && N == 1 && st && !fin && run_mask != F_ACTIVE;
    a.p_out = p_out;
    a.swizzle = t.swizzle;
    a.tile_bps = 0;
    if (t.swizzle >= 2) {
        // t-grouped block order: needs whole blocks per t-slice and groups
        // that divide Lt; otherwise the XCD order alone
        const uint64_t slice = (uint64_t)g->g.st * (uint64_t)S;  // lanes per t-slice
        const uint32_t tb = 1u << (t.swizzle - 1);
        if (slice % kBlock == 0 && g->g.L[3] % (int)tb == 0) a.tile_bps = (uint32_t)(slice / kBlock);
    }
    a.g = g->g;
    if (red) a.red = *red;
    if (fin) a.fin = *fin;
    if (ex) {
        // x + y and q(r) belong to the fp64 stages of a reliable update
        if (prec != P64 || (ex->aux && (epi != EPI_RESID || (ex->aux_prec != P32 && ex->aux_prec != P16S))))
            return hipErrorInvalidValue;
        if (ex->lazy_y && epi != EPI_PLAIN && epi != EPI_RESID) return hipErrorInvalidValue;
        a.lazy_y = ex->lazy_y;
        a.lazy_y_rs = ex->lazy_y_rs;
        a.aux = ex->aux;
        a.aux_rs = ex->aux_rs;
        a.aux_prec = ex->aux_prec;
        a.keep_y = ex->keep_y;
    }
    return launch_hop(prec, S, N, epi, t.nt != 0, a, is);
}

}  // namespace stag

// ============================================================================
// C ABI
// ============================================================================

#define STAG_VERSION 10000

#define HIPCK(ctx, call)                                                              \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess) {                                                       \
            (void)hipGetLastError();                                                  \
            return set_error((ctx), STAG_EDEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
        }                                                                             \
    } while (0)

extern "C" {

int stag_version(void) { return STAG_VERSION; }

const char* stag_last_error(const stag_ctx* ctx) {
    if (!ctx) return g_create_err.c_str();
    return ctx->err.c_str();
}

int stag_create(int device, size_t hbm_budget_bytes, stag_ctx** out) {
    if (!out) return set_error(nullptr, STAG_EINVAL, "stag_create: out is NULL");
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n <= 0) {
        (void)hipGetLastError();
        return set_error(nullptr, STAG_EDEVICE, "stag_create: no HIP device (%s)",
                         hipGetErrorString(e));
    }
    if (device < 0 || device >= n)
        return set_error(nullptr, STAG_EINVAL, "stag_create: device %d out of range [0, %d)",
                         device, n);
    DeviceGuard dg(device);
    hipStream_t s = nullptr;
    e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return set_error(nullptr, STAG_EDEVICE, "hipStreamCreate: %s", hipGetErrorString(e));
    }
    void* scr = nullptr;
    e = scratch_init(device, &scr);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        (void)hipStreamDestroy(s);
        return set_error(nullptr, STAG_EDEVICE, "stag_create: scratch address: %s",
                         hipGetErrorString(e));
    }
    // Temporaries of the asynchronous calls (A's odd intermediate, host
    // import / export staging) come from a pool of the context that keeps
    // freed memory for reuse: the device's default pool returns it at every
    // synchronisation, and a fresh physical allocation in a loop of A
    // applications can take longer than the kernels.
    hipMemPoolProps props{};
    props.allocType = hipMemAllocationTypePinned;
    props.location.type = hipMemLocationTypeDevice;
    props.location.id = device;
    hipMemPool_t pool = nullptr;
    e = hipMemPoolCreate(&pool, &props);
    if (e == hipSuccess) {
        uint64_t keep = UINT64_MAX;
        e = hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        if (pool) (void)hipMemPoolDestroy(pool);
        (void)hipStreamDestroy(s);
        return set_error(nullptr, STAG_EDEVICE, "stag_create: memory pool: %s", hipGetErrorString(e));
    }
    stag_ctx* c = new stag_ctx();
    c->device = device;
    c->stream = s;
    c->scratch = scr;
    c->pool = pool;
    if (hbm_budget_bytes == 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) == hipSuccess) c->budget = fr;
        (void)hipGetLastError();
    } else {
        c->budget = hbm_budget_bytes;
    }
    *out = c;
    return STAG_OK;
}

int stag_serve_shutdown_internal(stag_ctx* ctx);  // serve.cpp
int stag_serve_release_gauge_internal(stag_ctx* ctx, const stag_gauge* g);  // serve.cpp

int stag_destroy(stag_ctx* ctx) {
    if (!ctx) return STAG_OK;
    DeviceGuard dg(ctx->device);
    stag_serve_shutdown_internal(ctx);
    (void)hipStreamSynchronize(ctx->stream);
    std::vector<stag_engine*> engines;
    std::vector<stag_field*> fields;
    std::vector<stag_gauge*> gauges;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        engines.swap(ctx->engines);
        fields.swap(ctx->fields);
        gauges.swap(ctx->gauges);
    }
    for (auto* e : engines) engine_destroy(e);
    for (auto* f : fields) {
        dev_free(ctx, f->data, f->rs * f->nrhs);
        delete f;
    }
    for (auto* g : gauges) {
        for (int p = 0; p < 3; ++p)
            for (int q = 0; q < 2; ++q) (void)hipFree(g->G[p][q]);
        for (int q = 0; q < 2; ++q) (void)hipFree(g->gscale[q]);
        delete g;
    }
    (void)hipStreamDestroy(ctx->stream);
    if (ctx->pool) (void)hipMemPoolDestroy(ctx->pool);
    delete ctx;
    return STAG_OK;
}

int stag_memory_used(const stag_ctx* ctx, size_t* bytes) {
    if (!ctx || !bytes) return STAG_EINVAL;
    *bytes = ctx->used.load();
    return STAG_OK;
}

static hipStream_t pick_stream(stag_ctx* ctx, void* s) {
    return s ? (hipStream_t)s : ctx->stream;
}

namespace {

// Shared body of stag_gauge_create (Ulong null) and
// stag_gauge_create_improved (U = fat links, Ulong = long links).
int gauge_create(stag_ctx* ctx, const int L[4], const double* U, const double* Ulong,
                 int U_on_device, int prec_mask, stag_gauge** out) {
    if (!ctx) return STAG_EINVAL;
    if (!out || !L || !U)
        return set_error(ctx, STAG_EINVAL, "stag_gauge_create: NULL argument");
    *out = nullptr;
    if (Ulong && (prec_mask & STAG_GAUGE_R12))
        return set_error(ctx, STAG_EINVAL,
                         "stag_gauge_create_improved: fat and long links are stored in full "
                         "(STAG_GAUGE_R12 needs SU(3) links)");
    const int npairs = Ulong ? 8 : 4;
    uint64_t V = 1;
    for (int i = 0; i < 4; ++i) {
        if (L[i] < 2 || (L[i] & 1))
            return set_error(ctx, STAG_EINVAL,
                             "stag_gauge_create: extent L[%d] = %d must be even and >= 2", i, L[i]);
        V *= (uint64_t)L[i];
    }
    if (V / 2 >= (1ull << 31))
        return set_error(ctx, STAG_EINVAL, "stag_gauge_create: lattice too large");
    const bool r12 = (prec_mask & STAG_GAUGE_R12) != 0;
    prec_mask &= ~STAG_GAUGE_R12;
    if (prec_mask <= 0 || prec_mask > 7)
        return set_error(ctx, STAG_EINVAL, "stag_gauge_create: bad precision mask %d", prec_mask);
    DeviceGuard dg(ctx->device);
    stag_gauge* g = new stag_gauge();
    g->ctx = ctx;
    for (int i = 0; i < 4; ++i) g->L[i] = L[i];
    g->g = make_geom(L);
    g->mask = prec_mask;
    g->r12 = r12;
    g->npairs = npairs;
    const size_t Vh = g->g.Vh;
    const size_t ubytes = (size_t)V * 4 * 9 * 16;
    void* Ud = nullptr;  // staging of U (and Ulong behind it) for host links
    int rc = STAG_OK;
    auto cleanup = [&]() {
        for (int p = 0; p < 3; ++p)
            for (int q = 0; q < 2; ++q)
                if (g->G[p][q]) dev_free(ctx, g->G[p][q], link_bytes(p, Vh, r12, npairs));
        for (int q = 0; q < 2; ++q)
            if (g->gscale[q]) dev_free(ctx, g->gscale[q], Vh * 4);
        delete g;
    };
    if (!U_on_device) {
        const size_t sbytes = Ulong ? 2 * ubytes : ubytes;
        hipError_t e = hipMalloc(&Ud, sbytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            cleanup();
            return set_error(ctx, STAG_ENOMEM, "stag_gauge_create: staging hipMalloc(%zu): %s",
                             sbytes, hipGetErrorString(e));
        }
        e = hipMemcpy(Ud, U, ubytes, hipMemcpyHostToDevice);
        if (e == hipSuccess && Ulong)
            e = hipMemcpy((char*)Ud + ubytes, Ulong, ubytes, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            (void)hipFree(Ud);
            cleanup();
            return set_error(ctx, STAG_EDEVICE, "stag_gauge_create: copy: %s", hipGetErrorString(e));
        }
    }
    const void* Usrc = U_on_device ? (const void*)U : Ud;
    const void* Nsrc = !Ulong ? nullptr : U_on_device ? (const void*)Ulong : (const char*)Ud + ubytes;
    if (r12) {
        // the third row is rebuilt from the first two: only valid for SU(3)
        int* bad = nullptr;
        int hbad = 0;
        hipError_t e = hipMalloc((void**)&bad, sizeof(int));
        if (e == hipSuccess) e = hipMemsetAsync(bad, 0, sizeof(int), ctx->stream);
        if (e == hipSuccess) e = launch_su3_check(Usrc, (uint64_t)V * 4, 1e-10, bad, ctx->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, ctx->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
        if (bad) (void)hipFree(bad);
        if (e != hipSuccess || hbad) {
            (void)hipGetLastError();
            if (Ud) (void)hipFree(Ud);
            cleanup();
            return e != hipSuccess
                       ? set_error(ctx, STAG_EDEVICE, "stag_gauge_create: SU(3) check: %s",
                                   hipGetErrorString(e))
                       : set_error(ctx, STAG_EINVAL,
                                   "stag_gauge_create: STAG_GAUGE_R12 needs SU(3) links "
                                   "(|U U^+ - 1| or |det U - 1| above 1e-10)");
        }
    }
    for (int p = 0; p < 3 && rc == STAG_OK; ++p) {
        if (!(prec_mask & (1 << p))) continue;
        const size_t gb = link_bytes(p, Vh, r12, npairs);
        for (int q = 0; q < 2 && rc == STAG_OK; ++q) {
            rc = dev_alloc(ctx, gb, &g->G[p][q]);
            if (rc == STAG_OK && p == P16S) rc = dev_alloc(ctx, Vh * 4, (void**)&g->gscale[q]);
            if (rc == STAG_OK) {
                hipError_t e = launch_gauge_pack(p, Usrc, Nsrc, g->G[p][q], g->gscale[q], g->g, q,
                                                 r12, ctx->stream);
                if (e != hipSuccess) {
                    (void)hipGetLastError();
                    rc = set_error(ctx, STAG_EDEVICE, "gauge pack: %s", hipGetErrorString(e));
                }
            }
            g->bytes += gb + (p == P16S ? Vh * 4 : 0);
        }
    }
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (Ud) (void)hipFree(Ud);
    if (rc == STAG_OK && e != hipSuccess) {
        (void)hipGetLastError();
        rc = set_error(ctx, STAG_EDEVICE, "gauge pack sync: %s", hipGetErrorString(e));
    }
    if (rc != STAG_OK) {
        cleanup();
        return rc;
    }
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        ctx->gauges.push_back(g);
    }
    *out = g;
    return STAG_OK;
}

}  // namespace

int stag_gauge_create(stag_ctx* ctx, const int L[4], const double* U, int U_on_device,
                      int prec_mask, stag_gauge** out) {
    return gauge_create(ctx, L, U, nullptr, U_on_device, prec_mask, out);
}

int stag_gauge_create_improved(stag_ctx* ctx, const int L[4], const double* F, const double* N,
                               int links_on_device, int prec_mask, stag_gauge** out) {
    if (ctx && !N) return set_error(ctx, STAG_EINVAL, "stag_gauge_create_improved: NULL argument");
    return gauge_create(ctx, L, F, N, links_on_device, prec_mask, out);
}

int stag_gauge_destroy(stag_gauge* g) {
    if (!g) return STAG_OK;
    stag_ctx* ctx = g->ctx;
    DeviceGuard dg(ctx->device);
    // serving requests still reference the gauge: refuse; else the serving
    // batches on it are released (their in-flight blocks waited for)
    int rc = stag_serve_release_gauge_internal(ctx, g);
    if (rc) return rc;
    (void)hipStreamSynchronize(ctx->stream);
    std::vector<stag_engine*> drop;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        auto& v = ctx->gauges;
        for (size_t i = 0; i < v.size(); ++i)
            if (v[i] == g) {
                v.erase(v.begin() + i);
                break;
            }
        auto& es = ctx->engines;
        for (size_t i = 0; i < es.size();) {
            if (es[i]->gauge == g && !es[i]->in_use) {
                drop.push_back(es[i]);
                es.erase(es.begin() + i);
            } else {
                ++i;
            }
        }
    }
    for (auto* e : drop) engine_destroy(e);
    const size_t Vh = g->g.Vh;
    for (int p = 0; p < 3; ++p)
        for (int q = 0; q < 2; ++q)
            if (g->G[p][q]) dev_free(ctx, g->G[p][q], link_bytes(p, Vh, g->r12, g->npairs));
    for (int q = 0; q < 2; ++q)
        if (g->gscale[q]) dev_free(ctx, g->gscale[q], Vh * 4);
    delete g;
    return STAG_OK;
}

int stag_gauge_sites(const stag_gauge* g, int64_t* vh) {
    if (!g || !vh) return STAG_EINVAL;
    *vh = g->g.Vh;
    return STAG_OK;
}

int stag_field_create(stag_ctx* ctx, const stag_gauge* g, int parity, int prec, int nrhs,
                      stag_field** out) {
    if (!ctx) return STAG_EINVAL;
    if (!g || !out) return set_error(ctx, STAG_EINVAL, "stag_field_create: NULL argument");
    *out = nullptr;
    if (g->ctx != ctx) return set_error(ctx, STAG_EINVAL, "stag_field_create: gauge of another context");
    if (parity != 0 && parity != 1)
        return set_error(ctx, STAG_EINVAL, "stag_field_create: parity %d not 0 or 1", parity);
    if (prec < 0 || prec > 2) return set_error(ctx, STAG_EINVAL, "stag_field_create: precision %d", prec);
    if (nrhs < 1 || nrhs > STAG_MAX_RHS)
        return set_error(ctx, STAG_EINVAL, "stag_field_create: nrhs %d out of [1, %d]", nrhs, STAG_MAX_RHS);
    DeviceGuard dg(ctx->device);
    stag_field* f = new stag_field();
    f->ctx = ctx;
    f->gauge = g;
    f->parity = parity;
    f->prec = prec;
    f->nrhs = nrhs;
    f->rs = spinor_rhs_bytes(prec, g->g.Vh);
    int rc = dev_alloc(ctx, f->rs * nrhs, &f->data);
    if (rc != STAG_OK) {
        delete f;
        return rc;
    }
    // zero-initialise so an export before any import is well defined
    hipError_t e = hipMemsetAsync(f->data, 0, f->rs * nrhs, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        dev_free(ctx, f->data, f->rs * nrhs);
        delete f;
        return set_error(ctx, STAG_EDEVICE, "field init: %s", hipGetErrorString(e));
    }
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        ctx->fields.push_back(f);
    }
    *out = f;
    return STAG_OK;
}

int stag_field_destroy(stag_field* f) {
    if (!f) return STAG_OK;
    stag_ctx* ctx = f->ctx;
    DeviceGuard dg(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        auto& v = ctx->fields;
        for (size_t i = 0; i < v.size(); ++i)
            if (v[i] == f) {
                v.erase(v.begin() + i);
                break;
            }
    }
    dev_free(ctx, f->data, f->rs * f->nrhs);
    delete f;
    return STAG_OK;
}

int stag_field_import(stag_field* f, const double* src, int src_on_device, void* stream) {
    if (!f) return STAG_EINVAL;
    stag_ctx* ctx = f->ctx;
    if (!src) return set_error(ctx, STAG_EINVAL, "stag_field_import: src is NULL");
    DeviceGuard dg(ctx->device);
    hipStream_t s = pick_stream(ctx, stream);
    const size_t Vh = f->gauge->g.Vh;
    const size_t bytes = (size_t)f->nrhs * Vh * 48;
    const void* dsrc = src;
    void* tmp = nullptr;
    if (!src_on_device) {
        HIPCK(ctx, hipMallocFromPoolAsync(&tmp, bytes, ctx->pool, s));
        HIPCK(ctx, hipMemcpyAsync(tmp, src, bytes, hipMemcpyHostToDevice, s));
        dsrc = tmp;
    }
    HIPCK(ctx, launch_import(f->prec, dsrc, f->data, f->rs, (uint32_t)Vh, f->nrhs, s));
    if (tmp) {
        HIPCK(ctx, hipFreeAsync(tmp, s));
        HIPCK(ctx, hipStreamSynchronize(s));
    }
    return STAG_OK;
}

int stag_field_export(const stag_field* f, double* dst, int dst_on_device, void* stream) {
    if (!f) return STAG_EINVAL;
    stag_ctx* ctx = f->ctx;
    if (!dst) return set_error(ctx, STAG_EINVAL, "stag_field_export: dst is NULL");
    DeviceGuard dg(ctx->device);
    hipStream_t s = pick_stream(ctx, stream);
    const size_t Vh = f->gauge->g.Vh;
    const size_t bytes = (size_t)f->nrhs * Vh * 48;
    void* ddst = dst;
    void* tmp = nullptr;
    if (!dst_on_device) {
        HIPCK(ctx, hipMallocFromPoolAsync(&tmp, bytes, ctx->pool, s));
        ddst = tmp;
    }
    HIPCK(ctx, launch_export(f->prec, f->data, f->rs, ddst, (uint32_t)Vh, f->nrhs, s));
    if (tmp) {
        HIPCK(ctx, hipMemcpyAsync(dst, tmp, bytes, hipMemcpyDeviceToHost, s));
        HIPCK(ctx, hipFreeAsync(tmp, s));
        HIPCK(ctx, hipStreamSynchronize(s));
    }
    return STAG_OK;
}

static int check_pair(stag_ctx* ctx, const stag_gauge* g, const stag_field* in,
                      const stag_field* out, const char* fn) {
    if (!g || !in || !out) return set_error(ctx, STAG_EINVAL, "%s: NULL argument", fn);
    if (g->ctx != ctx || in->ctx != ctx || out->ctx != ctx)
        return set_error(ctx, STAG_EINVAL, "%s: objects from another context", fn);
    if (in->gauge != g || out->gauge != g)
        return set_error(ctx, STAG_EINVAL, "%s: field of another gauge", fn);
    if (in == out) return set_error(ctx, STAG_EINVAL, "%s: in and out must differ", fn);
    if (in->prec != out->prec || in->nrhs != out->nrhs)
        return set_error(ctx, STAG_EINVAL, "%s: precision / nrhs mismatch", fn);
    if (!(g->mask & (1 << in->prec)))
        return set_error(ctx, STAG_EINVAL, "%s: gauge has no copy in precision %d", fn, in->prec);
    return STAG_OK;
}

int stag_dslash(stag_ctx* ctx, const stag_gauge* g, const stag_field* in, stag_field* out,
                void* stream) {
    if (!ctx) return STAG_EINVAL;
    int rc = check_pair(ctx, g, in, out, "stag_dslash");
    if (rc) return rc;
    if (out->parity != 1 - in->parity)
        return set_error(ctx, STAG_EINVAL, "stag_dslash: out parity must be 1 - in parity");
    DeviceGuard dg(ctx->device);
    hipStream_t s = pick_stream(ctx, stream);
    const int N = pick_n(in->nrhs);
    // process exactly nrhs blocks: spare slots of the N-kernel get no state
    // and would be processed, so run in chunks of instantiated sizes
    int done = 0;
    while (done < in->nrhs) {
        int n = in->nrhs - done;
        int Nk = pick_n(n);
        if (Nk > n) {
            // largest instantiated size <= n
            static const int ns[] = {16, 12, 8, 4, 2, 1};
            for (int v : ns)
                if (v <= n) {
                    Nk = v;
                    break;
                }
        }
        HopTune t = get_tune(ctx, in->prec, Nk, g->g.Vh, g->npairs);
        const char* ip = (const char*)in->data + (size_t)done * in->rs;
        char* op = (char*)out->data + (size_t)done * out->rs;
        HIPCK(ctx, enqueue_hop(g, in->prec, t.S1, Nk, EPI_PLAIN, t, ip, in->rs, op, out->rs,
                               out->parity, nullptr, 0, nullptr, 0, nullptr, nullptr, 0, nullptr, Issue{s}));
        done += Nk;
    }
    (void)N;
    return STAG_OK;
}

// The two hop stages of A for every right-hand side of `in`, with the odd
// intermediate D_oe in at t (in->nrhs right-hand sides of in->rs bytes).
static int apply_A_stages(stag_ctx* ctx, const stag_gauge* g, const double* mass,
                          const stag_field* in, stag_field* out, void* t, hipStream_t s) {
    int done = 0;
    while (done < in->nrhs) {
        int n = in->nrhs - done;
        int Nk = 1;
        static const int ns[] = {16, 12, 8, 4, 2, 1};
        for (int v : ns)
            if (v <= n) {
                Nk = v;
                break;
            }
        double m2[kMaxN] = {0};
        for (int r = 0; r < Nk; ++r) m2[r] = mass[done + r] * mass[done + r];
        HopTune tu = get_tune(ctx, in->prec, Nk, g->g.Vh, g->npairs);
        const char* ip = (const char*)in->data + (size_t)done * in->rs;
        char* tp = (char*)t + (size_t)done * in->rs;
        char* op = (char*)out->data + (size_t)done * out->rs;
        HIPCK(ctx, enqueue_hop(g, in->prec, tu.S1, Nk, EPI_PLAIN, tu, ip, in->rs, tp, in->rs, 1,
                               nullptr, 0, nullptr, 0, nullptr, nullptr, 0, nullptr, Issue{s}));
        HIPCK(ctx, enqueue_hop(g, in->prec, tu.S2, Nk, EPI_XPAY, tu, tp, in->rs, op, out->rs, 0, ip,
                               in->rs, nullptr, 0, m2, nullptr, 0, nullptr, Issue{s}));
        done += Nk;
    }
    return STAG_OK;
}

static int check_apply_A(stag_ctx* ctx, const stag_gauge* g, const double* mass,
                         const stag_field* in, const stag_field* out, const char* fn) {
    int rc = check_pair(ctx, g, in, out, fn);
    if (rc) return rc;
    if (!mass) return set_error(ctx, STAG_EINVAL, "%s: mass is NULL", fn);
    if (in->parity != 0 || out->parity != 0)
        return set_error(ctx, STAG_EINVAL, "%s: fields must be even (parity 0)", fn);
    for (int r = 0; r < in->nrhs; ++r)
        if (!(mass[r] > 0.0) || !std::isfinite(mass[r]))
            return set_error(ctx, STAG_EINVAL, "%s: mass[%d] must be finite and > 0", fn, r);
    return STAG_OK;
}

int stag_apply_A(stag_ctx* ctx, const stag_gauge* g, const double* mass, const stag_field* in,
                 stag_field* out, void* stream) {
    if (!ctx) return STAG_EINVAL;
    int rc = check_apply_A(ctx, g, mass, in, out, "stag_apply_A");
    if (rc) return rc;
    DeviceGuard dg(ctx->device);
    hipStream_t s = pick_stream(ctx, stream);
    void* t = nullptr;
    HIPCK(ctx, hipMallocFromPoolAsync(&t, in->rs * in->nrhs, ctx->pool, s));
    rc = apply_A_stages(ctx, g, mass, in, out, t, s);
    HIPCK(ctx, hipFreeAsync(t, s));
    return rc;
}

int stag_apply_A_noalloc(stag_ctx* ctx, const stag_gauge* g, const double* mass,
                         const stag_field* in, stag_field* out, void* stream) {
    if (!ctx) return STAG_EINVAL;
    int rc = check_apply_A(ctx, g, mass, in, out, "stag_apply_A_noalloc");
    if (rc) return rc;
    const size_t need = in->rs * (size_t)in->nrhs;
    if (need > kScratchBytes)
        return set_error(ctx, STAG_EINVAL,
                         "stag_apply_A_noalloc: the odd intermediate needs %zu bytes, more than "
                         "the %zu-byte device scratch",
                         need, kScratchBytes);
    if (!ctx->scratch) return set_error(ctx, STAG_EDEVICE, "stag_apply_A_noalloc: no scratch");
    DeviceGuard dg(ctx->device);
    // every hop-stage-1 output site is written before stage 2 reads it, so
    // nothing in the scratch needs clearing
    return apply_A_stages(ctx, g, mass, in, out, ctx->scratch, pick_stream(ctx, stream));
}

void stag_cg_params_default(stag_cg_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->tol = 1e-8;
    p->max_iter = 0;
    p->inner_prec = STAG_F64;
    p->delta = 0.1;
    p->stall_iters = 0;
    p->max_stall = 20;
    p->graph_k = 0;
    p->use_graph = 1;
    p->use_x0 = 0;
    p->escalate = 1;
    p->mixed_variant = STAG_MIXED_CARRY;
    p->small_lattice = 1;
}

int stag_cg_solve(stag_ctx* ctx, const stag_gauge* g, const double* mass, const stag_field* b,
                  stag_field* x, const stag_cg_params* params, stag_cg_stats* stats,
                  void* stream) {
    if (!ctx) return STAG_EINVAL;
    if (!g || !mass || !b || !x || !params)
        return set_error(ctx, STAG_EINVAL, "stag_cg_solve: NULL argument");
    if (g->ctx != ctx || b->ctx != ctx || x->ctx != ctx || b->gauge != g || x->gauge != g)
        return set_error(ctx, STAG_EINVAL, "stag_cg_solve: objects of another context / gauge");
    if (b == x) return set_error(ctx, STAG_EINVAL, "stag_cg_solve: b and x must differ");
    if (b->prec != STAG_F64 || x->prec != STAG_F64 || b->parity != 0 || x->parity != 0)
        return set_error(ctx, STAG_EINVAL, "stag_cg_solve: b and x must be even F64 fields");
    if (b->nrhs != x->nrhs) return set_error(ctx, STAG_EINVAL, "stag_cg_solve: nrhs mismatch");
    const stag_cg_params& p = *params;
    if (!(p.tol > 0.0 && p.tol < 1.0))
        return set_error(ctx, STAG_EINVAL, "stag_cg_solve: tol must be in (0, 1)");
    if (p.inner_prec < 0 || p.inner_prec > 2)
        return set_error(ctx, STAG_EINVAL, "stag_cg_solve: inner precision %d", p.inner_prec);
    if (p.mixed_variant < STAG_MIXED_CARRY || p.mixed_variant > STAG_MIXED_FOLD_ONLY)
        return set_error(ctx, STAG_EINVAL, "stag_cg_solve: mixed_variant %d", p.mixed_variant);
    if (!(g->mask & STAG_MASK_F64) || !(g->mask & (1 << p.inner_prec)))
        return set_error(ctx, STAG_EINVAL,
                         "stag_cg_solve: gauge needs the F64 copy and the inner-precision copy");
    for (int r = 0; r < b->nrhs; ++r)
        if (!(mass[r] > 0.0) || !std::isfinite(mass[r]))
            return set_error(ctx, STAG_EINVAL, "stag_cg_solve: mass[%d] must be finite and > 0", r);
    DeviceGuard dg(ctx->device);
    const int n = b->nrhs;
    hipStream_t s = pick_stream(ctx, stream);
    const auto t0 = std::chrono::steady_clock::now();
    const bool can_escalate = p.inner_prec == STAG_F16S && p.escalate && (g->mask & STAG_MASK_F32);
    // with somewhere to go, an fp16 pass gives up after a few stall restarts
    // without progress instead of the full max_stall
    stag_cg_params p1 = p;
    if (can_escalate) p1.max_stall = std::min(p.max_stall > 0 ? p.max_stall : 20, kEscalateStalls);
    std::vector<stag_cg_stats> st1(n);
    stag_engine* e = nullptr;
    int rc = engine_acquire(ctx, g, p.inner_prec, pick_n(n), &e);
    if (rc) return rc;
    rc = engine_solve(e, n, mass, b->data, b->rs, x->data, x->rs, p1, st1.data(), s, can_escalate);
    engine_release(e);
    bool stalled = false;
    for (const auto& t : st1) stalled |= t.status == STAG_ESTALL;
    if (stalled && can_escalate) {
        // fp16 storage has hit its precision floor: continue from the current
        // x with fp32 inner iterations (converged RHS stop at their start).
        // fp32 needs no stall restarts (they would throw away the Krylov
        // space while the slow modes left over by the fp16 pass converge).
        stag_cg_params p2 = p;
        p2.inner_prec = STAG_F32;
        p2.use_x0 = 1;
        p2.stall_iters = std::numeric_limits<int>::max();
        std::vector<stag_cg_stats> st2(n);
        rc = engine_acquire(ctx, g, STAG_F32, pick_n(n), &e);
        if (rc) return rc;
        rc = engine_solve(e, n, mass, b->data, b->rs, x->data, x->rs, p2, st2.data(), s);
        engine_release(e);
        if (rc == STAG_EINVAL || rc == STAG_ENOMEM || rc == STAG_EDEVICE) return rc;
        const double secs =
            std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        for (int r = 0; r < n; ++r) {
            stag_cg_stats& a = st1[r];
            const stag_cg_stats& c = st2[r];
            a.iters += c.iters;
            a.reliable_updates += c.reliable_updates;
            a.restarts += c.restarts;
            a.status = c.status;
            a.true_rel_res = c.true_rel_res;
            a.iter_rel_res = c.iter_rel_res;
            a.seconds = secs;
            a.inner_final = STAG_F32;
        }
    }
    if (stats)
        for (int r = 0; r < n; ++r) stats[r] = st1[r];
    return rc;
}

}  // extern "C"
