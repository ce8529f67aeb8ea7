/*
 * stag.h -- C ABI of libstag: conjugate-gradient solves of b = A x with the
 * even-odd staggered normal operator on one AMD Instinct MI355X (gfx950).
 *
 * What is computed (Jang, Kim and Lee, "Multi GPU Performance of Conjugate
 * Gradient Solver with Staggered Fermions in Mixed Precision", Lattice 2011):
 *
 *   Sec.2, Eq.1      b = A x with A Hermitian positive definite.
 *   Sec.2, Eq.4-5    (D chi)(x) = sum_mu U_mu(x) chi(x+mu) - U_mu(x-mu)^+ chi(x-mu),
 *                    the staggered phase eta_mu(x) = (-1)^(x_0+...+x_{mu-1})
 *                    multiplied into U_mu (text after Eq.5). No factor 1/2.
 *   Sec.2, Eq.2-3    A = -D^2 + m^2, applied on the even sites:
 *                    A chi = m^2 chi - D_eo D_oe chi.
 *   Sec.2, Fig.1     conjugate gradient.
 *   Sec.3.2, Eq.6    corrected mixed-precision CG: low-precision inner
 *                    iterations, fp64 reliable and group-wise updates, the
 *                    search direction carried over across updates, all inner
 *                    products in fp64.
 *   Improved operator (stag_gauge_create_improved): Eq.5 over fat links plus
 *                    the three-hop terms over long links, the action of the
 *                    MILC ensembles Sec.2 sizes its workload on; every call
 *                    below computes with it when given such a gauge.
 *
 * Conventions (fixed by this library; the paper does not state them):
 *   - Lattice extents L = {Lx, Ly, Lz, Lt}, each even and >= 2, periodic.
 *   - Site lex = x + Lx*(y + Ly*(z + Lz*t)); parity (x+y+z+t) mod 2; "even" = 0.
 *   - A parity-p vector is indexed by s = lex / 2 over the sites of parity p.
 *   - Canonical host layouts are interleaved complex128 (re, im doubles):
 *       gauge links  U[t][z][y][x][mu][a][b], mu = 0..3 for x, y, z, t,
 *                    WITHOUT the staggered phases;
 *       vectors      v[rhs][s][c], c = 0..2.
 *   - Solver tolerance is relative to |b|: success means the fp64 true
 *     residual satisfies |b - A x| <= tol |b| for every right-hand side.
 *
 * General rules:
 *   - Every function returns an int status (STAG_OK = 0, negative = error);
 *     no C++ exception crosses this interface. The text of the last error on
 *     a context is available from stag_last_error().
 *   - Objects are opaque and owned by the library; caller buffers passed in
 *     are only read/written during the call (or, for the asynchronous
 *     calls, until the given stream reaches the enqueued work).
 *   - `stream` arguments are hipStream_t values passed as void*; NULL means
 *     the context's own stream. Work is enqueued without a host sync unless
 *     stated otherwise.
 *   - All functions are thread-safe with respect to different contexts.
 *     Calls on one context may come from several threads; the serving calls
 *     (submit/poll) are designed for that.
 */
#ifndef STAG_H
#define STAG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status */
#define STAG_OK 0
#define STAG_PENDING 1        /* serving: the ticket is not finished yet */
#define STAG_EINVAL (-1)      /* invalid argument (bad pointer, size, parity, precision, mass) */
#define STAG_ENOMEM (-2)      /* device memory or the context's HBM budget is exhausted */
#define STAG_EDEVICE (-3)     /* a HIP runtime error; see stag_last_error */
#define STAG_ENOCONV (-4)     /* iteration cap reached before the tolerance */
#define STAG_EBREAKDOWN (-5)  /* <d, A d> <= 0 or a non-finite scalar in the recurrence */
#define STAG_ESTALL (-6)      /* low-precision iteration stopped making progress */
#define STAG_EBUSY (-7)       /* serving queue full, or a gauge still used by serving requests */
#define STAG_ENOTFOUND (-8)   /* unknown or already collected ticket */

/* ------------------------------------------------------------- precisions */
#define STAG_F64 0   /* fp64 storage and arithmetic */
#define STAG_F32 1   /* fp32 storage and arithmetic */
#define STAG_F16S 2  /* fp16 storage with one fp32 scale per site; fp32 arithmetic */

/* bit masks of precisions for stag_gauge_create */
#define STAG_MASK_F64 (1 << STAG_F64)
#define STAG_MASK_F32 (1 << STAG_F32)
#define STAG_MASK_F16S (1 << STAG_F16S)
/* Gauge option (or-ed into prec_mask): store every copy with 12 real
 * parameters per link (two rows; the kernels rebuild the third as the
 * conjugated cross product of the first two, in the copy's arithmetic
 * precision, and apply the staggered phase from the site's coordinates),
 * cutting link traffic by a third (Sec.3.3). F16S copies keep their per-site
 * scale, taken over the full links. Needs SU(3) links: stag_gauge_create
 * checks |U U^+ - 1| and |det U - 1| <= 1e-10 on every link and fails with
 * EINVAL otherwise. */
#define STAG_GAUGE_R12 (1 << 4)

#define STAG_MAX_RHS 16 /* right-hand sides per field / per solve call */

typedef struct stag_ctx stag_ctx;
typedef struct stag_gauge stag_gauge;
typedef struct stag_field stag_field;
typedef int64_t stag_ticket;

/* Library version, encoded as major * 10000 + minor * 100 + patch. */
int stag_version(void);

/* ---------------------------------------------------------------- context
 * stag_create: bind a context to HIP device `device` (0-based) and create
 * its stream. `hbm_budget_bytes` caps the device memory the context may
 * hold (gauges, fields, solver workspaces); 0 means all currently free
 * memory. Errors: EINVAL (null out, bad device), EDEVICE.
 * stag_destroy: waits for the context's work, cancels pending serving
 * tickets, frees every object created from the context. NULL is a no-op.
 * stag_last_error: text of the last error on the context (or of the last
 * failed stag_create on this thread when ctx is NULL); never NULL.
 */
int stag_create(int device, size_t hbm_budget_bytes, stag_ctx** out);
int stag_destroy(stag_ctx* ctx);
const char* stag_last_error(const stag_ctx* ctx);
/* Bytes of device memory currently held by the context. */
int stag_memory_used(const stag_ctx* ctx, size_t* bytes);

/* ---------------------------------------------------------------- gauge
 * stag_gauge_create: make a gauge field resident on the device (Sec.2:
 * A is given by the links U and the mass m).
 *   L           lattice extents {Lx, Ly, Lz, Lt}, each even and >= 2, with
 *               L[0]*L[1]*L[2]*L[3]/2 < 2^31.
 *   U           canonical links, complex128 [t][z][y][x][mu][3][3] without
 *               phases; host memory if U_on_device == 0, device memory of the
 *               context's device otherwise. Copied; the caller keeps ownership.
 *   prec_mask   which stored copies to build (STAG_MASK_*); solves need
 *               STAG_MASK_F64 plus the mask of their inner precision. May
 *               include STAG_GAUGE_R12 (12-parameter copies).
 * The library folds the phases eta_mu into the links (or, with
 * STAG_GAUGE_R12, applies them from the coordinates), splits them by parity
 * and stores, per output site, its eight hop links in a site-coalesced
 * layout. Synchronous. Errors: EINVAL, ENOMEM, EDEVICE.
 */
int stag_gauge_create(stag_ctx* ctx, const int L[4], const double* U, int U_on_device,
                      int prec_mask, stag_gauge** out);
/* stag_gauge_create_improved: the improved staggered operator, i.e. Eq.5
 * with the fat links F in place of U plus the three-hop terms
 *   + eta_mu(x) N_mu(x) chi(x + 3mu) - eta_mu(x - 3mu) N_mu(x - 3mu)^+ chi(x - 3mu)
 * over the long links N (Sec.2 sizes its workload on a MILC fine lattice,
 * an ensemble generated with such an action). The fields are inputs:
 * smearing and the three-link products with their coefficients are the
 * caller's. F and N are canonical complex128
 * [t][z][y][x][mu][3][3] arrays without phases, both on the host or both on
 * the device (links_on_device), copied. Neither needs to be unitary, so
 * STAG_GAUGE_R12 is rejected (EINVAL); otherwise as stag_gauge_create, with
 * sixteen hop links per output site. Every solver, operator, serving and
 * tuning call takes the resulting gauge like any other. */
int stag_gauge_create_improved(stag_ctx* ctx, const int L[4], const double* F, const double* N,
                               int links_on_device, int prec_mask, stag_gauge** out);
/* stag_gauge_destroy: frees the gauge's device copies (and the solver
 * workspaces and serving batches built on it). Errors: EBUSY while a serving
 * request submitted on this gauge has not been collected by stag_solver_poll
 * (the gauge stays valid; collect the tickets and call again). NULL is a no-op. */
int stag_gauge_destroy(stag_gauge* gauge);
/* Number of sites per parity (Vh = Lx*Ly*Lz*Lt/2) of a gauge's lattice. */
int stag_gauge_sites(const stag_gauge* gauge, int64_t* vh);

/* ---------------------------------------------------------------- fields
 * A field holds nrhs (1..STAG_MAX_RHS) vectors of one parity in one storage
 * precision, in a private site-coalesced layout.
 * stag_field_import / stag_field_export convert from / to the canonical
 * complex128 layout [nrhs][Vh][3]; `src`/`dst` are host memory when the
 * *_on_device flag is 0 (then the call synchronises the stream before it
 * returns) or device memory otherwise (asynchronous on `stream`). Importing
 * into F32 / F16S rounds to nearest even (F16S: the site scale is the
 * largest |Re| or |Im| of the site's six reals after rounding to fp32; the
 * payload is fp16(value / scale); a zero site stores scale 0).
 * Errors: EINVAL (null, nrhs out of range, parity not 0/1, bad precision),
 * ENOMEM, EDEVICE.
 */
int stag_field_create(stag_ctx* ctx, const stag_gauge* gauge, int parity, int prec, int nrhs,
                      stag_field** out);
int stag_field_import(stag_field* f, const double* src, int src_on_device, void* stream);
int stag_field_export(const stag_field* f, double* dst, int dst_on_device, void* stream);
int stag_field_destroy(stag_field* f);

/* ---------------------------------------------------------------- operators
 * stag_dslash (Sec.2, Eq.5): out = D in, from parity p of `in` to parity
 * 1 - p of `out`, for every right-hand side (the improved D for a gauge of
 * stag_gauge_create_improved). `in` and `out` must be distinct
 * fields of the same gauge, precision and nrhs; the gauge must hold that
 * precision. F32 / F16S compute in fp32. Asynchronous on `stream`.
 * Errors: EINVAL, EDEVICE.
 */
int stag_dslash(stag_ctx* ctx, const stag_gauge* gauge, const stag_field* in, stag_field* out,
                void* stream);

/* stag_apply_A (Sec.2, Eq.2-3): out_j = m_j^2 in_j - D_eo D_oe in_j on even
 * fields, right-hand side j using mass[j] (host array of in->nrhs finite
 * masses > 0). Asynchronous on `stream`; uses a temporary odd-parity vector
 * allocated stream-ordered from a memory pool of the context, which keeps
 * freed memory for the next call until stag_destroy. Errors: EINVAL (parity
 * 1, mismatch, mass <= 0 or not finite), ENOMEM, EDEVICE.
 */
int stag_apply_A(stag_ctx* ctx, const stag_gauge* gauge, const double* mass, const stag_field* in,
                 stag_field* out, void* stream);

/* stag_apply_A_noalloc: stag_apply_A for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same kernels and the same bits as stag_apply_A, but
 * the temporary odd-parity vector lives in a device scratch array of
 * STAG_NOALLOC_SCRATCH_BYTES that the library holds on each GPU it runs on
 * until the process ends (its address is looked up by stag_create); the call
 * allocates and frees nothing. The caller passes the fields as for
 * stag_apply_A. Errors: as stag_apply_A, plus EINVAL when the intermediate
 * (nrhs * Vh * 48 bytes for F64, * 24 for F32, * 16 for F16S) exceeds the
 * scratch. Every call on one GPU shares that GPU's scratch: calls whose work
 * overlaps on the device (on different streams, or from several contexts on
 * the same GPU) race; calls on one stream are ordered and safe. */
#define STAG_NOALLOC_SCRATCH_BYTES ((size_t)48 << 20)
int stag_apply_A_noalloc(stag_ctx* ctx, const stag_gauge* gauge, const double* mass,
                         const stag_field* in, stag_field* out, void* stream);

/* ---------------------------------------------------------------- solver */
typedef struct stag_cg_params {
    double tol;        /* relative true-residual target, > 0 and < 1 */
    int max_iter;      /* <= 0: min(10 * 3 * Vh, 10^6) */
    int inner_prec;    /* STAG_F64: plain CG (Fig.1); STAG_F32 / STAG_F16S: mixed (Sec.3.2) */
    double delta;      /* mixed: update when |r| < delta * max|r| since the last update; <= 0: 0.1 */
    int stall_iters;   /* mixed: forced update + direction restart after this many
                          iterations without a new residual minimum; <= 0: 100 with
                          STAG_F16S, never with STAG_F32 (fp32 needs no safeguard) */
    int max_stall;     /* mixed: ESTALL after this many consecutive stall updates
                          without halving the true residual; <= 0: 20 */
    int graph_k;       /* iterations per host poll (replayed as one HIP graph when
                          use_graph); <= 0: automatic */
    int use_graph;     /* 1: replay each K-iteration block as one hipGraph */
    int use_x0;        /* 1: x holds the initial guess on entry; 0: start from x = 0 */
    int escalate;      /* F16S inner, gauge with an F32 copy: when the fp16-storage inner
                          iteration cannot refine the system, continue from the current x
                          with F32 inner iterations (no stall restarts); default 1. The
                          fp16 pass ends (ESTALL) after 3 stall updates without progress,
                          at the first refinement cycle that reduces the true residual
                          norm by less than half (a working inner solve reduces it by
                          about delta), or at the first update after more than twice the
                          iterations the CG convergence bound allows for the reduction
                          reached (sqrt(kappa) from the first cycle's largest Lanczos
                          diagonal and mass^2) */
    int mixed_variant; /* mixed: what an update does with the search direction.
                          STAG_MIXED_CARRY (default): keep it, d = r + beta d with
                          beta = |r_true|^2 / |r_prev|^2 (Sec.3.2, Eq.6); the inner cycle
                          ends when |r| < delta max|r| since the update.
                          STAG_MIXED_RESTART: restart it, d = r, every update (the plain
                          iterative refinement of Fig.2); the cycle ends when
                          |r| < delta |r at the cycle start|.
                          Ablations that split Sec.3.2's update into its two
                          ingredients (the paper's group-wise paragraph, read
                          literally, already includes the residual recompute, i.e. it
                          is the default scheme): STAG_MIXED_RELIABLE replaces the
                          inner residual by r = b - A (x + y) computed in fp64 but never
                          folds y into x (the solution stays in fp32);
                          STAG_MIXED_FOLD_ONLY folds y into x in fp64 (y = 0) but never
                          recomputes r, and checks the true residual once, when the
                          iterated one has met tol (ENOCONV if the true one misses it). */
    int small_lattice; /* 1 (default): tiny lattices solve each right-hand side inside
                          one workgroup, which loops over the iterations itself (no
                          kernel launch per stage): up to 128 sites per parity (4^4),
                          and up to 648 (6^4) for calls with several right-hand sides;
                          plain CG and the CARRY / RESTART mixed variants without use_x0
                          on Eq.5 gauges. 0: always the kernel-per-stage solver */
} stag_cg_params;

#define STAG_MIXED_CARRY 0
#define STAG_MIXED_RESTART 1
#define STAG_MIXED_RELIABLE 2
#define STAG_MIXED_FOLD_ONLY 3

typedef struct stag_cg_stats {
    int iters;             /* CG iterations (inner iterations for mixed) */
    int reliable_updates;  /* fp64 updates (mixed) / true-residual checks (plain) */
    int restarts;          /* direction restarts */
    int status;            /* STAG_OK, STAG_ENOCONV, STAG_EBREAKDOWN, STAG_ESTALL, STAG_EINVAL */
    double true_rel_res;   /* |b - A x| / |b| in fp64 at the end */
    double iter_rel_res;   /* iterated residual norm / |b| at the end */
    double seconds;        /* wall time of the whole call */
    int inner_final;       /* inner precision of the last iterations (STAG_F16S solves
                              that escalated end in STAG_F32) */
} stag_cg_stats;

/* Fill *p with the defaults (tol 1e-8, plain fp64 CG, x from 0, escalation on). */
void stag_cg_params_default(stag_cg_params* p);

/* stag_cg_solve: solve A_j x_j = b_j (Sec.2 Eq.1, Fig.1; mixed: Sec.3.2)
 * for every right-hand side j of the even F64 field `b`, writing the even F64
 * field `x` (same nrhs; x starts from 0, or from its contents with use_x0).
 * mass: host array [b->nrhs]. All
 * right-hand sides of one call are iterated together, each with its own
 * scalars, sharing every link load. Success requires the fp64 true
 * residual |b - A x| <= tol |b| for each; b_j = 0 gives x_j = 0. Returns
 * after all solves ended (the host waits on `stream`); per-RHS outcomes are
 * in stats[j] (array of b->nrhs, may be NULL). The return value is STAG_OK
 * when every right-hand side converged, else the first failing status.
 * With an F16S inner precision whose solve stalls (ESTALL) and `escalate`
 * set, the call continues all right-hand sides from the current x with F32
 * inner iterations (those already converged stop at once); stats add up both
 * passes and report inner_final = STAG_F32.
 * Errors: EINVAL (arguments, non-finite b), ENOMEM, EDEVICE; ENOCONV,
 * EBREAKDOWN, ESTALL as solve outcomes (x holds the last iterate).
 */
int stag_cg_solve(stag_ctx* ctx, const stag_gauge* gauge, const double* mass,
                  const stag_field* b, stag_field* x, const stag_cg_params* params,
                  stag_cg_stats* stats, void* stream);


/* ---------------------------------------------------------------- serving
 * Continuous batching of solve requests (each a CG solve as in
 * stag_cg_solve, Sec.2 Fig.1 / Sec.3.2). A scheduler thread of the context
 * admits requests in arrival order into a batch per (gauge, inner
 * precision) when the context's HBM budget allows (requests that do not fit
 * wait), starts their right-hand sides in free slots between K-iteration
 * blocks while other slots are mid-solve, and frees each slot when its
 * right-hand side has finished. Batches of different gauges run on separate
 * streams and overlap on the device. A right-hand side's result does not
 * depend on what else is being solved. An STAG_F16S request on a gauge that
 * also holds F32 links hands a right-hand side whose fp16 inner iteration
 * cannot refine its system (no halving of the true residual over 3 stall
 * updates, or a refinement cycle that does not halve it) over to the
 * gauge's F32 batch, which continues from its current x without stall
 * restarts, as stag_cg_solve escalates; its stats add up both passes and
 * report inner_final = STAG_F32. Without an F32 copy such a right-hand side
 * ends with STAG_ESTALL after max_stall (20) stall updates.
 *
 * stag_solver_submit: copies b_host (complex128 [nrhs][Vh][3], even sites)
 *   before returning; never waits for the GPU. mass > 0, 0 < tol < 1,
 *   inner_prec STAG_F64 / STAG_F32 / STAG_F16S (the gauge must hold F64 and
 *   that copy), 1 <= nrhs <= STAG_MAX_RHS. Thread-safe. Errors: EINVAL,
 *   EBUSY (queue full).
 * stag_solver_poll: STAG_PENDING until every right-hand side of the ticket
 *   has finished; then writes x_host (complex128 [nrhs][Vh][3], may be NULL),
 *   stats[nrhs] (may be NULL) and the submit-to-finish latency in seconds
 *   (may be NULL), releases the ticket and returns STAG_OK or the first
 *   failing per-RHS status. ENOTFOUND for an unknown or collected ticket.
 *   Thread-safe.
 * stag_solver_config: slots per batch (rounded up to 1, 2, 4, 8, 12 or 16),
 *   iterations per block (<= 0: automatic) and queue capacity; only before
 *   the first submit (EBUSY after).
 * stag_destroy cancels pending tickets.
 */
int stag_solver_submit(stag_ctx* ctx, const stag_gauge* gauge, double mass, int nrhs,
                       const double* b_host, double tol, int inner_prec, stag_ticket* out);
int stag_solver_poll(stag_ctx* ctx, stag_ticket ticket, double* x_host, stag_cg_stats* stats,
                     double* latency_s);
int stag_solver_config(stag_ctx* ctx, int slots_per_batch, int graph_k, int queue_cap);

/* ---------------------------------------------------------------- tuning
 * Launch shape of the two hop stages of A: S1 / S2 = lanes per output site
 * (1, 2 or 4) for stage 1 (D_oe) and stage 2 (D_eo with the m^2 update),
 * nt = non-temporal link loads, swizzle = block order: 0 plain, 1 each XCD
 * on a contiguous eighth of the blocks, 2 / 3 / 4 that and then the blocks
 * in groups of 2 / 4 / 8 consecutive t-slices with t running fastest (keeps a
 * site's t-neighbours close in launch order; used where the lattice has
 * whole blocks per t-slice, else as 1). Every shape computes bit-identical
 * results; only speed differs.
 * stag_tune_get / stag_tune_set: the shape used for (prec, nrhs, vh) by
 * gauges of Eq.5's operator, or with STAG_TUNE_IMPROVED or-ed into prec by
 * gauges of the improved operator. stag_tune: time the solver's own iteration
 * kernels (see stag_time_kernels) in every shape on the gauge's actual
 * links and keep the fastest for gauges of its kind (Eq.5 or improved) (synchronous; uses a solver workspace for nrhs right-hand
 * sides, allocated if none is free). best / best_ms may be NULL; best_ms is
 * the time of the two hop stages in milliseconds. Errors: EINVAL, ENOMEM,
 * EDEVICE.
 */
#define STAG_TUNE_IMPROVED (1 << 8)

typedef struct stag_tune_cfg {
    int S1, S2, nt, swizzle;
} stag_tune_cfg;

int stag_tune_get(stag_ctx* ctx, int prec, int nrhs, int64_t vh, stag_tune_cfg* out);
int stag_tune_set(stag_ctx* ctx, int prec, int nrhs, int64_t vh, const stag_tune_cfg* cfg);
int stag_tune(stag_ctx* ctx, const stag_gauge* gauge, int prec, int nrhs, stag_tune_cfg* best,
              double* best_ms);
/* Persistent tune table: when the environment variable STAG_TUNE_CACHE names
 * a file, stag_tune first looks the shape up there, keyed by (device
 * architecture, operator, link form, sites per parity, precision, kernel
 * right-hand-side count), and times the shapes only on a miss, appending the
 * result (one text line per entry; the last entry of a key wins; an
 * unreadable or unwritable file only means measuring). stag_tune_counts:
 * how many stag_tune calls on ctx were answered from the file (loaded) and
 * how many timed the shapes (measured). Errors: EINVAL (null argument). */
int stag_tune_counts(const stag_ctx* ctx, int* loaded, int* measured);

/* ---------------------------------------------------------------- timing
 * While enabled, stag_cg_solve launches its kernels eagerly (no graph) with
 * HIP events recorded at each kernel's start and end (hipExtLaunchKernel, on
 * the launch stream); stag_timing_read
 * returns the number of launches and their summed duration per kind.
 * stag_timing_enable waits for the device and resets the counters.
 */
#define STAG_K_HOP1 0     /* inner-precision D_oe */
#define STAG_K_HOP2 1     /* inner-precision D_eo + m^2 update + <d, A d> */
#define STAG_K_HOP1_64 2  /* fp64 D_oe of a true-residual recompute */
#define STAG_K_HOP2_64 3  /* fp64 D_eo + residual + norm of a recompute */
#define STAG_K_UPDATE 4   /* fused x/y and r update with |r|^2 */
#define STAG_K_XPAY 5     /* the direction update d = r + beta d as its own pass (blocks
                             of 8 or more right-hand sides, and every solve on lattices
                             of 131072 sites per parity or more; otherwise fused into
                             the hop stages) */
#define STAG_K_OTHER 6
int stag_timing_enable(stag_ctx* ctx, int on);
/* stag_time_kernels: average execution time in microseconds of the three
 * kernels of one CG iteration exactly as stag_cg_solve launches them (same
 * buffers, launch shape and arithmetic) for `prec` (STAG_F64: plain CG, else
 * mixed) and nrhs right-hand sides: us[0] = D_oe stage (with the deferred
 * direction update and the finalisation of the previous |r|^2), us[1] = D_eo
 * stage with m^2 update and <d, A d>, us[2] = fused update with |r|^2 (and
 * the finalisation of alpha). Blocks of 8 or more right-hand sides, and
 * every solve on lattices of 131072 or more sites per parity, run the
 * direction update as a pass of its own (not included): their us[0] and
 * us[1] are the hop stages reading d as stored. The three run `reps`
 * (1..100000) times in the solve's order (stage 1, stage 2, update), so each
 * reads what the one before it wrote; each figure is the mean time between
 * events recorded at the start and the end of the kernel
 * (hipExtLaunchKernel) on the context's stream. Synchronous. */
int stag_time_kernels(stag_ctx* ctx, const stag_gauge* gauge, int prec, int nrhs, int reps,
                      double* us);
int stag_timing_read(stag_ctx* ctx, int kind, int64_t* count, double* total_ms);

#ifdef __cplusplus
}
#endif

#endif /* STAG_H */
