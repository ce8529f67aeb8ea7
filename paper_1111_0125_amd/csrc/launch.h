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
    double m2[16];         // mass^2 per right-hand side (used when st is null)
    RhsState* st;          // null: every RHS is processed
    unsigned run_mask;     // process RHS r iff st[r].flags & run_mask
    int p_out;
    int swizzle;
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
    OP_RU_BEGIN = 5,   // x64 += y, y = 0
    OP_RU_END = 6,     // rs = q(r64) after a true-residual recompute
    OP_ZERO = 8,       // f0 = 0
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

// Optional events recorded at the start and the end of one kernel's
// execution (hipExtLaunchKernel), for timing single launches.
struct LaunchEvents {
    hipEvent_t start;
    hipEvent_t stop;
};

hipError_t launch_hop(int prec, int S, int N, int epi, bool nt, const HopArgs& a,
                      hipStream_t stream, const LaunchEvents* ev = nullptr);
hipError_t launch_vec(int prec, int N, int op, const VecArgs& a, hipStream_t stream,
                      const LaunchEvents* ev = nullptr);
// One-block fixed-order sum of a reduction kernel's chunk partials and its
// finalisation (R.kind), for the RHS whose flags match run_mask; launched
// right after the kernel that wrote the partials, with the same run_mask.
hipError_t launch_finalize(int N, const Reduce& R, unsigned run_mask, hipStream_t stream);
// One-block state transition (FIN_RU_END, FIN_CG_CHECK) of the RHS whose
// flags match run_mask.
hipError_t launch_state(int N, int kind, RhsState* st, unsigned run_mask, hipStream_t stream);

// Layout conversion kernels (canonical complex128 <-> internal storage).
hipError_t launch_gauge_pack(int prec, const void* U_dev, void* G, float* gscale, const Geom& g,
                             int p_out, hipStream_t stream);
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

// Reduction partials: one per 64-site chunk, whatever the launch shape.
inline uint32_t num_chunks(uint32_t Vh) { return (Vh + 63) / 64; }

inline uint32_t hop_blocks(uint32_t Vh, int S) {
    return (uint32_t)(((uint64_t)Vh * S + kBlock - 1) / kBlock);
}
inline uint32_t vec_blocks(uint32_t Vh) { return (Vh + kBlock - 1) / kBlock; }

}  // namespace stag
