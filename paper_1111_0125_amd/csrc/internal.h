// Host-side objects of libstag (context, gauge, field, solver engine).
#pragma once

#include <atomic>
#include <condition_variable>
#include <cstdarg>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/stag.h"
#include "launch.h"

namespace stag {

struct Serve;  // serving loop (serve.cpp)

// Launch shape of the two hop stages for one (precision, block size) pair.
struct HopTune {
    int S1 = 1, S2 = 1;  // lanes per site of stage 1 (D_oe) and stage 2 (D_eo + xpay)
    int nt = 1;          // non-temporal link loads
    int swizzle = 1;     // block order: 0 plain, 1 XCD-aware, 2-4 XCD-aware in groups of
                         // 2, 4 or 8 t-slices with t fastest (hop kernels; vector kernels
                         // take any value >= 1 as XCD-aware)
};

}  // namespace stag

namespace stag {
// Per-kernel-kind timing collected with HIP events on the launch stream.
enum KernelKind : int {
    KK_HOP1 = 0,      // inner-precision hop, stage 1 (D_oe)
    KK_HOP2 = 1,      // inner-precision hop, stage 2 (D_eo + xpay + dot)
    KK_HOP1_64 = 2,   // fp64 hop stage 1 of a true-residual recompute
    KK_HOP2_64 = 3,   // fp64 hop stage 2 of a true-residual recompute
    KK_UPDATE = 4,    // fused axpy + norm
    KK_XPAY = 5,      // direction update pass (blocks of several RHS on large lattices)
    KK_OTHER = 6,
    KK_COUNT = 7,
};
struct Timing {
    bool on = false;
    long long count[KK_COUNT] = {0};
    double ms[KK_COUNT] = {0};
    std::vector<hipEvent_t> pool;
    struct Rec {
        int kind;
        hipEvent_t a, b;
    };
    std::vector<Rec> pending;
    std::mutex mu;
};
}  // namespace stag

struct stag_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    void* scratch = nullptr;       // this device's copy of the scratch array (scratch.hip)
    hipMemPool_t pool = nullptr;   // stream-ordered temporaries; keeps freed memory for reuse
    size_t budget = 0;
    std::atomic<size_t> used{0};
    std::mutex mu;                 // guards the object lists and the workspace pool
    std::string err;
    std::mutex err_mu;
    std::vector<stag_gauge*> gauges;
    std::vector<stag_field*> fields;
    std::vector<struct stag_engine*> engines;
    std::map<long long, stag::HopTune> tune;  // key: (prec, N, Vh bucket)
    std::mutex tune_mu;
    std::atomic<int> tune_loaded{0};    // stag_tune calls answered from STAG_TUNE_CACHE
    std::atomic<int> tune_measured{0};  // stag_tune calls that timed the shapes
    stag::Serve* serve = nullptr;
    stag::Timing timing;
};

struct stag_gauge {
    stag_ctx* ctx = nullptr;
    int L[4] = {0, 0, 0, 0};
    stag::Geom g{};
    int mask = 0;
    void* G[3][2] = {{nullptr, nullptr}, {nullptr, nullptr}, {nullptr, nullptr}};
    float* gscale[2] = {nullptr, nullptr};  // P16S
    bool r12 = false;                       // every copy in 12-parameter form
    int npairs = 4;                         // hop pairs per site: 8 for the improved operator
    size_t bytes = 0;
};

struct stag_field {
    stag_ctx* ctx = nullptr;
    const stag_gauge* gauge = nullptr;
    int parity = 0, prec = 0, nrhs = 0;
    void* data = nullptr;
    size_t rs = 0;  // bytes per right-hand side
};

// Solver workspace + device state for N right-hand-side slots of one
// (gauge, inner precision).
struct stag_engine {
    stag_ctx* ctx = nullptr;
    const stag_gauge* gauge = nullptr;
    int prec = 0;  // inner precision (P64 = plain CG)
    int N = 1;     // slots
    bool in_use = false;
    uint32_t Vh = 0;
    // fp64 vectors [N]
    void *x64 = nullptr, *r64 = nullptr, *t64 = nullptr, *d64 = nullptr, *Ad64 = nullptr;
    void* b64 = nullptr;  // the right-hand sides being solved [N]
    bool serving = false; // owned by a serving batch (never lent to stag_cg_solve)
    // low-precision vectors [N]
    void *y32 = nullptr, *rs = nullptr, *d = nullptr, *t = nullptr, *Ad = nullptr;
    size_t rs64 = 0, rsP = 0, rs32 = 0;
    // Device state [N]. st is the state between K-iteration blocks (what the
    // host polls and what the fix-up kernels work on); inside a block the
    // state moves st -> st1 -> st as each reduction is finalised by the
    // kernel that consumes it.
    stag::RhsState* st = nullptr;
    stag::RhsState* st1 = nullptr;
    stag::RhsState* host[2] = {nullptr, nullptr};  // pinned poll buffers [N]
    stag::RhsState* hstage = nullptr;              // pinned slot-start staging [N]
    hipEvent_t ev[2] = {nullptr, nullptr};
    // Chunk partials [N][nparts]: partials holds <d, A d> (and every
    // reduction outside the iteration), partials1 the |r|^2 of the update,
    // so a consumer reads one while writing the other.
    double* partials = nullptr;
    double* partials1 = nullptr;
    size_t bytes = 0;
    std::map<long long, hipGraphExec_t> graphs;    // one block of work; key: (K, kernel N)
    stag::HopTune tune_lo, tune_64;
};

namespace stag {

// Host-side state of a sequence of K-iteration blocks on one engine.
struct EngineRun {
    stag_engine* e = nullptr;
    hipStream_t s = nullptr;
    const void* b = nullptr;  // right-hand sides, slot-strided
    size_t b_rs = 0;
    int K = 16;
    int F = 8;                // iterations between the predicated fix-ups
    int variant = 0;          // mixed CG variant (MixedVariant), the same for every slot
    bool use_graph = true;
    bool timed = false;
    long long launched = 0;   // blocks enqueued (block j polls into buffer j % 2)
    long long polled = 0;     // polls processed
    long long last_poll = -1; // index of the last processed poll
    std::vector<long long> start_after;  // polls <= this predate the slot's start
    int busy_hi = 0;          // slots [0, busy_hi) may be busy
};

struct SlotInit {
    int slot;
    double mass;
    stag_cg_params params;
    const void* x0 = nullptr;  // initial guess (fp64 internal layout, one RHS) or null: x = 0
    bool x0_in_place = false;  // the slot's x64 block already holds the initial guess
    bool escalating = false;   // fp16 storage that can hand over to fp32 (slow-cycle exit)
};

void run_init(EngineRun& R, stag_engine* e, hipStream_t s, const void* b, size_t b_rs, int K,
              bool use_graph);
int run_start_slots(EngineRun& R, const std::vector<SlotInit>& slots);
int run_enqueue_block(EngineRun& R, int K = 0);
int run_process_poll(EngineRun& R, bool blocking, const RhsState** h);
void fill_stats(const RhsState& s, double secs, int inner_prec, stag_cg_stats* out);
bool flags_terminal(unsigned f);
int status_of_flags(unsigned f);
int default_graph_k(uint32_t Vh);
// The buffers are cleared on init_stream, which is synchronised before return.
int engine_create(stag_ctx* ctx, const stag_gauge* g, int prec, int N, bool serving,
                  hipStream_t init_stream, stag_engine** out);
// An fp16-storage solve that can hand over to fp32 gives up after this many
// stall updates without halving the true residual (instead of max_stall).
constexpr int kEscalateStalls = 3;
// ... and ends at the first refinement cycle that does not reduce the true
// residual norm by this factor (a working inner solve reduces it by about the
// update threshold delta = 0.1).
constexpr double kSlowCycleRatio = 0.5;
// ... and at the first update after more than this many times the iterations
// the CG convergence bound allows for the reduction reached (measured on Haar
// links: fp32 stays at or under 1.1 of the bound, fp16 storage under 1.6 where
// it pays, m >= 0.05, and far above 2 where it does not, m = 0.02).
constexpr double kCgBudget = 2.0;

}  // namespace stag

namespace stag {

int set_error(stag_ctx* ctx, int code, const char* fmt, ...);

// The device scratch array of the allocation-free entry points (scratch.hip):
// kScratchBytes per GPU, held until the process ends. scratch_init returns
// its device address on `device`, which must be current (looked up once per
// device and kept).
constexpr size_t kScratchBytes = (size_t)48 << 20;
hipError_t scratch_init(int device, void** out);
int dev_alloc(stag_ctx* ctx, size_t bytes, void** p);
void dev_free(stag_ctx* ctx, void* p, size_t bytes);

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

Geom make_geom(const int L[4]);
// Launch shapes per (precision, kernel N, lattice size, hop pairs per site).
HopTune get_tune(stag_ctx* ctx, int prec, int N, uint32_t Vh, int npairs);
void set_tune(stag_ctx* ctx, int prec, int N, uint32_t Vh, int npairs, const HopTune& t);

// Engines (solver.cpp)
int engine_acquire(stag_ctx* ctx, const stag_gauge* g, int prec, int N, stag_engine** out);
void engine_release(stag_engine* e);
// Whether the iteration kernels of e (nk right-hand sides per kernel)
// finalise reductions at their start (small lattices) or leave it to a
// one-block kernel (large ones).
bool fuse_finalize(const stag_engine* e, int nk);
// Average execution time (us) of the three iteration kernels of e under
// tuning t (stage 1, stage 2, update), with the first nrhs slots active.
int time_iteration_kernels(stag_engine* e, const HopTune& t, int nrhs, int reps, double* us);
void engine_destroy(stag_engine* e);
void engine_drop_graphs(stag_engine* e);

// One whole solve of n <= N right-hand sides held in canonical device
// buffers b_dev / x_dev (complex128 [n][Vh][3]) or fields.
// escalating: an fp16-storage solve whose caller hands stalled right-hand
// sides over to fp32 (the pass also ends at a refinement cycle that fails to
// halve the true residual).
int engine_solve(stag_engine* e, int n, const double* mass, const void* b64, size_t b_rs,
                 void* x64_out, size_t x_rs, const stag_cg_params& p, stag_cg_stats* stats,
                 hipStream_t stream, bool escalating = false);

// Event timing helpers (no-ops when timing is off).
hipError_t timing_events(stag_ctx* ctx, hipEvent_t* a, hipEvent_t* b);  // two pooled events
void timing_push(stag_ctx* ctx, int kind, hipEvent_t a, hipEvent_t b);   // record a bracketed launch
void timing_collect(stag_ctx* ctx);  // accumulate every completed record

// Fields of HopArgs used only by the fp64 stages of a reliable update.
struct HopExtra {
    const void* lazy_y = nullptr;
    size_t lazy_y_rs = 0;
    void* aux = nullptr;
    size_t aux_rs = 0;
    int aux_prec = P32;
    int keep_y = 0;
};

hipError_t enqueue_hop(const stag_gauge* g, int prec, int S, int N, int epi, const HopTune& t,
                       const void* in, size_t in_rs, void* out, size_t out_rs, int p_out,
                       const void* x, size_t x_rs, const void* b, size_t b_rs, const double* m2,
                       RhsState* st, unsigned run_mask, const Reduce* red, const Issue& is,
                       const void* lazy_r = nullptr, size_t lazy_r_rs = 0,
                       const Reduce* fin = nullptr, const HopExtra* ex = nullptr);

}  // namespace stag
