// Internal declarations shared by the HIP kernels and the host engine of
// libstag. Not part of the public C ABI (that is include/stag.h).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <cstddef>
#include <cstdint>

namespace stag {

// Storage precisions of a field or of a copy of the gauge field.
enum Prec : int { P64 = 0, P32 = 1, P16S = 2 };

// ---------------------------------------------------------------------------
// Lattice geometry.
//
// Sites are numbered lex = x + Lx*(y + Ly*(z + Lz*t)); parity (x+y+z+t) & 1.
// A parity-p field is indexed by the checkerboard index s = lex >> 1, which is
// a bijection onto [0, Vh) because Lx is even. Periodic in all directions.
// ---------------------------------------------------------------------------

// Division by a constant through a multiply and a shift (Granlund and
// Montgomery, "Division by invariant integers using multiplication", 1994):
// for n < 2^31 and 1 <= d < 2^31, n / d == (n * M) >> (32 + k) with
// k = ceil(log2 d) and M = ceil(2^(32+k) / d), which fits in 33 bits.
struct FastDiv {
    uint64_t mul;
    uint32_t shift;
    uint32_t d;
    __host__ __device__ __forceinline__ uint32_t div(uint32_t n) const {
        return (uint32_t)(((uint64_t)n * mul) >> shift);
    }
};

inline FastDiv make_fastdiv(uint32_t d) {
    FastDiv f;
    f.d = d;
    uint32_t k = 0;
    while ((1ull << k) < d) ++k;
    unsigned __int128 num = ((unsigned __int128)1) << (32 + k);
    f.mul = (uint64_t)((num + d - 1) / d);
    f.shift = 32 + k;
    return f;
}

struct Geom {
    int L[4];          // Lx, Ly, Lz, Lt
    uint32_t Vh;       // sites per parity
    uint32_t hx;       // Lx / 2
    uint32_t sy, sz, st;  // checkerboard strides of y, z, t: hx, hx*Ly, hx*Ly*Lz
    FastDiv div_hx, div_Ly, div_Lz;
};

// Coordinates of the site with checkerboard index s on parity p.
__device__ __forceinline__ void site_coords(const Geom& g, uint32_t s, int p, int& x, int& y,
                                            int& z, int& t) {
    uint32_t row = g.div_hx.div(s);
    uint32_t xh = s - row * g.hx;
    uint32_t r2 = g.div_Ly.div(row);
    y = (int)(row - r2 * (uint32_t)g.L[1]);
    uint32_t r3 = g.div_Lz.div(r2);
    z = (int)(r2 - r3 * (uint32_t)g.L[2]);
    t = (int)r3;
    x = 2 * (int)xh + ((y + z + t + p) & 1);
}

// Checkerboard indices of the forward and backward neighbours of site
// (x, y, z, t) in direction mu (both lie on the opposite parity).
__device__ __forceinline__ void neighbours(const Geom& g, uint32_t s, int x, int y, int z, int t,
                                           int mu, uint32_t& nf, uint32_t& nb) {
    if (mu == 0) {
        uint32_t base = s - (uint32_t)(x >> 1);
        int xf = (x + 1 == g.L[0]) ? 0 : x + 1;
        int xb = (x == 0) ? g.L[0] - 1 : x - 1;
        nf = base + (uint32_t)(xf >> 1);
        nb = base + (uint32_t)(xb >> 1);
    } else if (mu == 1) {
        nf = (y + 1 == g.L[1]) ? s - (uint32_t)(g.L[1] - 1) * g.sy : s + g.sy;
        nb = (y == 0) ? s + (uint32_t)(g.L[1] - 1) * g.sy : s - g.sy;
    } else if (mu == 2) {
        nf = (z + 1 == g.L[2]) ? s - (uint32_t)(g.L[2] - 1) * g.sz : s + g.sz;
        nb = (z == 0) ? s + (uint32_t)(g.L[2] - 1) * g.sz : s - g.sz;
    } else {
        nf = (t + 1 == g.L[3]) ? s - (uint32_t)(g.L[3] - 1) * g.st : s + g.st;
        nb = (t == 0) ? s + (uint32_t)(g.L[3] - 1) * g.st : s - g.st;
    }
}

// The same for the three-hop neighbours x + 3 mu and x - 3 mu of the
// improved operator (also on the opposite parity: the hop length is odd).
// Extents are even and >= 2, so at most two periods are folded.
__device__ __forceinline__ void neighbours3(const Geom& g, uint32_t s, int x, int y, int z, int t,
                                            int mu, uint32_t& nf, uint32_t& nb) {
    const int c = mu == 0 ? x : mu == 1 ? y : mu == 2 ? z : t;
    const int L = g.L[mu];
    int cf = c + 3, cb = c - 3;
    if (cf >= L) cf -= L;
    if (cf >= L) cf -= L;
    if (cb < 0) cb += L;
    if (cb < 0) cb += L;
    if (mu == 0) {
        const uint32_t base = s - (uint32_t)(x >> 1);
        nf = base + (uint32_t)(cf >> 1);
        nb = base + (uint32_t)(cb >> 1);
    } else {
        const int stride = (int)(mu == 1 ? g.sy : mu == 2 ? g.sz : g.st);
        nf = (uint32_t)((int)s + (cf - c) * stride);
        nb = (uint32_t)((int)s + (cb - c) * stride);
    }
}

// ---------------------------------------------------------------------------
// Field storage (per right-hand side; a field with nrhs > 1 holds nrhs such
// blocks back to back, each `rhs_bytes` long):
//   P64   double2 [3][Vh]   (colour-major planes of complex numbers)
//   P32   float2  [3][Vh]
//   P16S  Rec16   [Vh]      (three half2 colours and one fp32 site scale)
// ---------------------------------------------------------------------------
struct __align__(16) Rec16 {
    __half2 c[3];
    float s;
};

inline size_t spinor_rhs_bytes(int prec, size_t Vh) {
    return prec == P64 ? Vh * 48 : prec == P32 ? Vh * 24 : Vh * 16;
}

// ---------------------------------------------------------------------------
// Gauge storage, one array per output parity p (the parity of the sites the
// hop kernel writes). For output site s the kernel reads eight "hop links":
// hop 2*mu   : L = eta_mu(x) U_mu(x)                     applied to chi(x + mu)
// hop 2*mu+1 : L = -(eta_mu(x - mu) U_mu(x - mu))^dagger applied to chi(x - mu)
// so the Dirac operator is a plain sum of eight matrix-vector products.
// The 72 complex entries (hop-major, then row-major 3x3) are stored word-major
// over the sites so that a wavefront reading word w of 64 consecutive sites
// touches one contiguous span:
//   P64   72 words of double2 (one complex)      at [w][Vh]
//   P32   36 words of float4  (two complex)      at [w][Vh]
//   P16S  36 words of uint2   (two half2 complex)at [w][Vh], plus one fp32
//         scale per site at [Vh] (largest |Re|,|Im| over the 144 reals).
// Hop pair mu (hops 2mu, 2mu+1) is 18 complex = words 18mu.. (P64) or 9mu..
// (P32, P16S).
// ---------------------------------------------------------------------------
// 12-parameter storage (SU(3) links): per output site and hop pair mu, the
// first two rows of U_mu(x) then of U_mu(x - mu)^dagger (12 complex, no
// phases): P64 48 words of double2, P32 24 words of float4, P16S 24 words of
// uint2 at [w][Vh] plus the site scale of the full form; pair mu is words
// 12mu.. (P64) or 6mu.. (P32, P16S). The kernels rebuild
// each third row as the conjugated cross product of the first two and apply
// +eta_mu(x) to the forward and -eta_mu(x) to the backward link
// (eta_mu(x - mu) = eta_mu(x): the phase depends on the coordinates before mu).
// ---------------------------------------------------------------------------
// Improved operator (fat links F in place of U, long links N): eight hop
// pairs per output site, pairs 0..3 as above from F and pairs 4 + mu the
// three-hop pair
// hop 8+2mu  : L = eta_mu(x) N_mu(x)                       applied to chi(x + 3mu)
// hop 9+2mu  : L = -(eta_mu(x - 3mu) N_mu(x - 3mu))^dagger applied to chi(x - 3mu)
// in the same word-major layout (P64 144 words, P32 / P16S 72 words; the
// P16S scale covers all 288 reals). Always the full 18-parameter form:
// fat and long links are not unitary.
inline size_t link_bytes(int prec, size_t Vh, bool r12 = false, int npairs = 4) {
    const size_t k = (size_t)npairs / 4;
    if (prec == P64) return k * Vh * (r12 ? 48 : 72) * 16;
    if (prec == P32) return k * Vh * (r12 ? 24 : 36) * 16;
    return k * Vh * (r12 ? 24 : 36) * 8;
}
inline size_t gauge_parity_bytes(int prec, size_t Vh, bool r12 = false, int npairs = 4) {
    return link_bytes(prec, Vh, r12, npairs) + (prec == P16S ? Vh * 4 : 0);
}

// ---------------------------------------------------------------------------
// Per right-hand-side solver state, resident in device memory. Scalars of
// the CG recurrence are computed on the device by the last block of each
// reduction; the host only reads the flags at poll points.
// ---------------------------------------------------------------------------
enum StateFlag : unsigned {
    F_ACTIVE = 1u,       // iterating
    F_CONV = 2u,         // iterated residual met the tolerance (plain CG)
    F_RU = 4u,           // reliable / group-wise update due (mixed CG)
    F_STALL = 8u,        // no new residual minimum for stall_iters iterations
    F_DONE = 16u,        // true residual met the tolerance
    F_BREAKDOWN = 32u,   // <d, A d> <= 0 or not finite
    F_MAXIT = 64u,       // iteration cap reached
    F_ESTALL = 128u,     // repeated stall restarts without progress
    F_BADINPUT = 256u,   // |b|^2 not finite
    F_NEW = 512u,        // slot being started
    F_X0 = 1024u,        // slot being started from an initial guess x0
    F_CHECK = 2048u,     // fold-only ablation: iterated residual converged, true
                         // residual check pending
    F_INACC = 4096u,     // fold-only ablation: the true residual missed the tolerance
};

struct RhsState {
    double rr;        // |r|^2 of the current (iterated) residual
    double rr_old;    // previous |r|^2
    double pAp;       // <d, A d>
    double alpha, beta;
    double bb;        // |b|^2
    double rr_stop;   // tol^2 |b|^2
    double rr_true;   // last recomputed |b - A x|^2
    double rmax, rmin;
    double best_true; // smallest true |r|^2 seen at a stall update
    double delta;     // update threshold (fraction of the running maximum)
    double tol2;      // tol^2
    double m2;        // mass^2
    double rstart;    // |r| when the current inner cycle started (last update)
    double slow_ratio;  // > 0: a non-stall update whose true |r| fell by less than this
                        // factor since the previous update ends the pass (F_ESTALL): the
                        // inner precision cannot refine this system (fp16 storage that
                        // can hand over to fp32); 0: off
    double cg_budget;   // > 0: a non-stall update after more than this many times the
                        // iterations the CG convergence bound allows for the true
                        // residual reduction reached ends the pass (F_ESTALL); 0: off
    double lam;         // largest Lanczos diagonal 1/alpha + beta/alpha_prev of the
                        // pass's first cycle (a lower bound of the largest eigenvalue)
    double rr_true0;    // true |r|^2 at the start of the pass
    int since;        // iterations since the last new residual minimum
    int stall_iters;
    int stall_count;
    int max_stall;
    int iters;
    int max_iter;
    int updates;
    int restarts;
    unsigned flags;
    int variant;      // mixed CG: MIXED_CARRY (Sec.3.2, Eq.6) or MIXED_RESTART (Fig.2)
};

// Mixed CG variants: what an update does with the search direction.
enum MixedVariant : int {
    MIXED_CARRY = 0,    // keep it, d = r + beta d with beta from Eq.6; the inner
                        // cycle ends when |r| < delta * max|r| since the update
    MIXED_RESTART = 1,  // restart it, d = r (iterative refinement of Fig.2); the
                        // cycle ends when |r| < delta * |r at the cycle start|
    // ablations of the two update methods of Sec.3.2 (both are applied above)
    MIXED_RELIABLE = 2,   // reliable update only: r = b - A (x + y) in fp64, y is never
                          // folded into x (the solution stays in fp32)
    MIXED_FOLD_ONLY = 3,  // solution folding only: x += y in fp64, y = 0, r never recomputed
};

// Finalisation applied to a reduced sum (by the one-block finalize kernel).
enum FinKind : int {
    FIN_STORE = 0,     // out[r] = sum
    FIN_ALPHA = 1,     // pAp -> alpha (or breakdown)
    FIN_CG = 2,        // |r|^2 -> beta, convergence / cap (plain CG)
    FIN_MIXED = 3,     // |r|^2 -> beta, update / stall triggers (mixed CG)
    FIN_INIT = 5,      // bb = sum; start state of a solve (from x = 0, or pending x0)
    FIN_RU_END = 6,    // rr_true = sum, then the state after a reliable / group-wise
                       // update (mixed CG)
    FIN_CG_CHECK = 7,  // rr_true = sum, then accept or restart (plain CG)
    FIN_X0 = 8,        // |b - A x0|^2 = sum: residual state of a start from x0
    FIN_ACTIVATE = 9,  // a started slot begins iterating
    FIN_FOLD = 10,       // fold-only ablation: state after folding y into x
    FIN_FOLD_CHECK = 11, // fold-only ablation: rr_true = sum, accept or report
    FIN_TRUE = 12,     // rr_true = sum
};

// A reduction: the producing kernel writes one fp64 partial per 64-site
// chunk and right-hand side; its consumer sums them in a fixed order and
// applies `kind` to the state. The consumer reads the state from st and
// writes the result to st_out (st_out null: in place, one-block consumers
// only), so a many-block consumer never reads what one of its own blocks
// has already overwritten.
struct Reduce {
    double* partials;   // [nrhs][nparts]: one partial per 64-site chunk
    RhsState* st;       // [nrhs] state read
    double* out;        // FIN_STORE destination [nrhs]
    RhsState* st_out;   // [nrhs] state written (null: st)
    int kind;
    int nparts;
};

}  // namespace stag
