// Kernel argument blocks and host-side launchers of libstag.
#pragma once

#include "common.h"

namespace stag {

constexpr int kMaxN = 16;  // largest block of right-hand sides per kernel

// Epilogue of the hop kernel (what is written at each output site).
enum Epi : int {
    EPI_PLAIN = 0,     // out = sum of the eight hops               (D, Eq.5)
    EPI_XPAY = 1,      // out = m^2 x - hops                         (A, second stage)
    EPI_XPAY_DOT = 2,  // same, plus Re<x, out> reduced in fp64      (d^+ A d for alpha)
    EPI_RESID = 3,     // out = b - (m^2 x - hops), plus |out|^2     (true residual)
};

struct HopArgs {
    const void* gauge;     // hop-ordered links of the output parity
    const float* gscale;   // P16S only: per-site link scale
    const void* in;        // input field, opposite parity to the output
    size_t in_rs;          // bytes per right-hand side
    void* out;
    size_t out_rs;
    const void* x;         // same-parity vector for XPAY / XPAY_DOT / RESID
    size_t x_rs;
    const void* b;         // RESID: right-hand side
    size_t b_rs;
    // Deferred direction update (solver iterations): when lazy_r is set the
    // operand is d_new = r + beta d with d the stored previous direction
    // (beta from the RHS state), rounded to the storage precision. Stage 1
    // forms it at every neighbour it gathers; stage 2 forms it at its own
    // site, uses it as x and stores it over d.
    const void* lazy_r;
    size_t lazy_r_rs;
    // fp64 stages of a reliable / group-wise update (P64 only): with lazy_y
    // set the operand is x + y, y being the fp32 correction of the inner
    // solve; stage 2 also stores x + y over x and zeroes y at its own site.
    // With aux set (RESID) the residual is also stored rounded to aux_prec
    // (P32 or P16S), restarting the inner residual from it.
    const void* lazy_y;
    size_t lazy_y_rs;
    void* aux;
    size_t aux_rs;
    int aux_prec;
    int keep_y;            // with lazy_y: use x + y but store neither (reliable-update-only ablation)
    double m2[16];         // mass^2 per right-hand side (used when st is null)
    RhsState* st;          // null: every RHS is processed
    unsigned run_mask;     // process RHS r iff st[r].flags & run_mask
    int gate;              // P64, one RHS: read the flags before any operand, leave if unflagged
    int p_out;
    int swizzle;           // block order (logical_block)
    uint32_t tile_bps;     // blocks per t-slice for the t-grouped orders (0: off)
    int r12;               // links in 12-parameter form
    int npairs;            // hop pairs per site: 4 (Eq.5) or 8 (improved operator)
    Geom g;
    Reduce red;            // XPAY_DOT / RESID: where the chunk partials go
    // Reduction finalised at kernel start (fin.partials null: none): every
    // block sums fin's partials, applies fin.kind to an LDS copy of st and
    // uses that; block 0 writes it to fin.st_out (fin.st is ignored, st is
    // the input state).
    Reduce fin;
};

// Vector (BLAS-like) kernels of the CG iteration; one thread per site.
enum VecOp : int {
    OP_INIT_B = 0,     // r64 = b, x64 = 0, |b|^2 -> FIN_INIT
    OP_START = 1,      // d = q(r64); if rs: rs = q(r64); if y: y = 0
    OP_UPD_CG = 2,     // x += a d, r -= a Ad, |r|^2 -> FIN_CG           (fp64)
    OP_UPD_MIXED = 3,  // y += a d, rs = q(rs - a Ad), |rs|^2 -> FIN_MIXED
    OP_FOLD = 4,       // x64 += y, y = 0 (f0 = x64, f1 = y)
    OP_XPAY = 5,       // d = q(r + beta d) (f0 = r, f1 = d): the direction update as its
                       // own pass, on large lattices and for blocks of 8 or more
};

struct VecArgs {
    void* f[6];        // field slots, meaning depends on the op
    size_t rs[6];      // bytes per right-hand side of each slot
    uint32_t Vh;
    RhsState* st;
    unsigned run_mask;
    int swizzle;
    Reduce red;        // INIT_B / UPD_*: where the chunk partials go
    Reduce fin;        // finalised at kernel start, as in HopArgs
};

// A graph under construction: kernels are appended as a chain of nodes.
struct GraphBuild {
    hipGraph_t graph = nullptr;
    hipGraphNode_t last = nullptr;  // the node the next one depends on
};

// Where a kernel goes: launched on `stream` (with events recorded at the
// start and the end of its execution when ev_start / ev_stop are set), or,
// with gb set, appended to that graph after its last node. Graphs are
// built node by node rather than captured from a stream, so building one
// does not interact with what other threads do meanwhile.
struct Issue {
    hipStream_t stream = nullptr;
    hipEvent_t ev_start = nullptr;
    hipEvent_t ev_stop = nullptr;
    GraphBuild* gb = nullptr;
};

// Issue kernel `func` (host stub address) with grid x block threads;
// args[i] points at the i-th kernel argument.
hipError_t issue_kernel(const Issue& is, const void* func, uint32_t grid, uint32_t block,
                        void** args);

hipError_t launch_hop(int prec, int S, int N, int epi, bool nt, const HopArgs& a, const Issue& is);
hipError_t launch_vec(int prec, int N, int op, const VecArgs& a, const Issue& is);
// One-block fixed-order sum of a reduction kernel's chunk partials and its
// finalisation (R.kind), for the RHS whose flags match run_mask; issued
// right after the kernel that wrote the partials, with the same run_mask.
hipError_t launch_finalize(int N, const Reduce& R, unsigned run_mask, const Issue& is);

// Layout conversion kernels (canonical complex128 <-> internal storage).
// r12: 12-parameter layout.
// Ulong_dev: long links of the improved operator (U_dev then holds the fat
// links), or null; never together with r12.
hipError_t launch_gauge_pack(int prec, const void* U_dev, const void* Ulong_dev, void* G,
                             float* gscale, const Geom& g, int p_out, bool r12, hipStream_t stream);
// Sets *bad_dev = 1 when a link is not SU(3) within tol (bad_dev zeroed by the caller).
hipError_t launch_su3_check(const void* U_dev, uint64_t nlinks, double tol, int* bad_dev,
                            hipStream_t stream);
hipError_t launch_import(int prec, const void* src_dev, void* dst, size_t dst_rs, uint32_t Vh,
                         int nrhs, hipStream_t stream);
hipError_t launch_export(int prec, const void* src, size_t src_rs, void* dst_dev, uint32_t Vh,
                         int nrhs, hipStream_t stream);

// The right-hand-side counts the kernels are instantiated for; a batch of n
// runs in the smallest of these >= n with the spare slots inactive.
inline int pick_n(int n) {
    static const int ns[] = {1, 2, 4, 8, 12, 16};
    for (int v : ns)
        if (v >= n) return v;
    return -1;
}

constexpr int kBlock = 256;  // threads per block of every kernel

// One-workgroup solves of tiny lattices (tiny.hip): one workgroup of
// kTinyBlock threads per right-hand side runs the whole solve.
constexpr int kTinyBlock = 512;

struct TinyArgs {
    const void* G[2];        // inner-precision hop links by output parity
    const float* gscale[2];  // P16S site scales
    const void* G64[2];      // fp64 hop links (true residuals)
    int r12;                 // inner links in 12-parameter form
    int r12_64;              // fp64 links in 12-parameter form
    Geom g;
    // slot-strided buffers (slot = right-hand side = workgroup)
    const void* b64;
    void* x64;
    void* r64;
    void* t64;
    void* d;                 // direction, D_oe d, A d, iterated residual: inner precision
    void* t;                 // (plain CG: the fp64 buffers, rs = r64)
    void* Ad;
    void* rs;
    void* y;                 // fp32 correction (plain CG: x64)
    size_t rs64, rsP, rsY;
    RhsState* st;            // [nrhs]: start state in (before FIN_INIT), final state out
    int cap;                 // loop turns after which the kernel stops whatever the state says
};

hipError_t launch_tiny(int prec, int nrhs, const TinyArgs& a, hipStream_t stream);

// Reduction partials: one per 64-site chunk, whatever the launch shape.
inline uint32_t num_chunks(uint32_t Vh) { return (Vh + 63) / 64; }

inline uint32_t hop_blocks(uint32_t Vh, int S) {
    return (uint32_t)(((uint64_t)Vh * S + kBlock - 1) / kBlock);
}
inline uint32_t vec_blocks(uint32_t Vh) { return (Vh + kBlock - 1) / kBlock; }

}  // namespace stag
