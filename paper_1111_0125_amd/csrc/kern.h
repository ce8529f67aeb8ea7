// Device helpers for the libstag kernels: storage codecs per precision,
// coalesced loads, deterministic reductions whose consumers finalise the
// CG scalars.
#pragma once

#include "common.h"
#include "launch.h"

// Contractions are written out as fma() where wanted; no implicit ones, so
// every instantiation of a kernel rounds identically.
#pragma clang fp contract(off)

namespace stag {

typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f2v __attribute__((ext_vector_type(2)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef unsigned u2v __attribute__((ext_vector_type(2)));
typedef unsigned u4v __attribute__((ext_vector_type(4)));

template <bool NT, typename T>
__device__ __forceinline__ T ldg(const T* p) {
    if constexpr (NT) {
        return __builtin_nontemporal_load(p);
    } else {
        return *p;
    }
}

template <int P>
struct Real {
    using T = float;
};
template <>
struct Real<P64> {
    using T = double;
};

// ------------------------------------------------------------------ fp16 + scale

__device__ __forceinline__ float h2f_lo(unsigned w) {
    return __half2float(__ushort_as_half((unsigned short)(w & 0xffffu)));
}
__device__ __forceinline__ float h2f_hi(unsigned w) {
    return __half2float(__ushort_as_half((unsigned short)(w >> 16)));
}
__device__ __forceinline__ unsigned f2h_pair(float lo, float hi) {
    unsigned a = __half_as_ushort(__float2half_rn(lo));
    unsigned b = __half_as_ushort(__float2half_rn(hi));
    return a | (b << 16);
}

// Encode one site (three complex colours) to the 16-byte record; the values
// are replaced by what the record decodes to (so norms see stored values).
__device__ __forceinline__ u4v f16s_encode(float (&re)[3], float (&im)[3]) {
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < 3; ++c) s = fmaxf(s, fmaxf(fabsf(re[c]), fabsf(im[c])));
    u4v w;
    if (s == 0.f) {
        w.x = w.y = w.z = 0u;
        w.w = 0u;
#pragma unroll
        for (int c = 0; c < 3; ++c) re[c] = im[c] = 0.f;
        return w;
    }
    unsigned q[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        q[c] = f2h_pair(__fdiv_rn(re[c], s), __fdiv_rn(im[c], s));
        re[c] = h2f_lo(q[c]) * s;
        im[c] = h2f_hi(q[c]) * s;
    }
    w.x = q[0];
    w.y = q[1];
    w.z = q[2];
    w.w = __float_as_uint(s);
    return w;
}

__device__ __forceinline__ void f16s_decode(u4v w, float (&re)[3], float (&im)[3]) {
    float s = __uint_as_float(w.w);
    re[0] = h2f_lo(w.x) * s;
    im[0] = h2f_hi(w.x) * s;
    re[1] = h2f_lo(w.y) * s;
    im[1] = h2f_hi(w.y) * s;
    re[2] = h2f_lo(w.z) * s;
    im[2] = h2f_hi(w.z) * s;
}

// ------------------------------------------------------------------ spinor access

// Load the colour vector of site s from one right-hand side block.
template <int P, bool NT = false>
__device__ __forceinline__ void load_site(const void* f, uint32_t Vh, uint32_t s,
                                          typename Real<P>::T (&re)[3],
                                          typename Real<P>::T (&im)[3]) {
    if constexpr (P == P64) {
        const d2v* p = (const d2v*)f;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            d2v v = ldg<NT>(p + (size_t)c * Vh + s);
            re[c] = v.x;
            im[c] = v.y;
        }
    } else if constexpr (P == P32) {
        const f2v* p = (const f2v*)f;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            f2v v = ldg<NT>(p + (size_t)c * Vh + s);
            re[c] = v.x;
            im[c] = v.y;
        }
    } else {
        u4v w = ldg<NT>((const u4v*)f + s);
        f16s_decode(w, re, im);
    }
}

// Store (rounding to the storage precision); re/im are replaced by the
// stored values.
template <int P>
__device__ __forceinline__ void store_site(void* f, uint32_t Vh, uint32_t s,
                                           typename Real<P>::T (&re)[3],
                                           typename Real<P>::T (&im)[3]) {
    if constexpr (P == P64) {
        d2v* p = (d2v*)f;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            d2v v;
            v.x = re[c];
            v.y = im[c];
            p[(size_t)c * Vh + s] = v;
        }
    } else if constexpr (P == P32) {
        f2v* p = (f2v*)f;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            f2v v;
            v.x = re[c];
            v.y = im[c];
            p[(size_t)c * Vh + s] = v;
        }
    } else {
        ((u4v*)f)[s] = f16s_encode(re, im);
    }
}

// Round a colour vector to what the storage precision would hold.
template <int P>
__device__ __forceinline__ void round_site(typename Real<P>::T (&re)[3], typename Real<P>::T (&im)[3]) {
    if constexpr (P == P16S) (void)f16s_encode(re, im);
}

// ------------------------------------------------------------------ gauge access

// Third row of an SU(3) matrix whose first two rows are entries o..o+5 of
// (lr, li): the conjugated cross product of rows 0 and 1, written to o+6..o+8.
template <typename T>
__device__ __forceinline__ void third_row(T (&lr)[18], T (&li)[18], int o) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int k1 = (k + 1) % 3, k2 = (k + 2) % 3;
        // a_k1 b_k2 - a_k2 b_k1
        const T pr = fma(lr[o + k1], lr[o + 3 + k2], -(li[o + k1] * li[o + 3 + k2]));
        const T pi = fma(lr[o + k1], li[o + 3 + k2], li[o + k1] * lr[o + 3 + k2]);
        const T qr = fma(lr[o + k2], lr[o + 3 + k1], -(li[o + k2] * li[o + 3 + k1]));
        const T qi = fma(lr[o + k2], li[o + 3 + k1], li[o + k2] * lr[o + 3 + k1]);
        lr[o + 6 + k] = pr - qr;
        li[o + 6 + k] = qi - pi;
    }
}

// Hop pair mu of output site s as stored (forward link then backward link,
// each row-major): with r12 the links are stored as two rows without phases
// (entries 0-5 and 9-14 of the pair). load_pair_raw only issues the loads,
// so that a caller can request several pairs before using any; the 12- or
// 18-entry form is chosen by address and count, not by separate code paths
// (separate paths writing different array positions make the compiler index
// the arrays dynamically, in scratch memory).
template <int P>
struct PairRaw;
template <>
struct PairRaw<P64> {
    d2v v[18];  // r12: entries 0-5 then 9-14; full: entries 0-17
};
template <>
struct PairRaw<P32> {
    f4v v[9];   // two entries each; r12: rows 0-1 forward in v[0..2], backward in v[3..5]
};
template <>
struct PairRaw<P16S> {
    u2v v[9];   // two entries each, as P32
    float sc;
};

template <int P, bool NT>
__device__ __forceinline__ void load_pair_raw(const void* G, const float* gscale, uint32_t Vh,
                                              uint32_t s, int mu, int r12, PairRaw<P>& w) {
    if constexpr (P == P64) {
        const d2v* g = (const d2v*)G + (size_t)((r12 ? 12 : 18) * mu) * Vh + s;
#pragma unroll
        for (int e = 0; e < 12; ++e) w.v[e] = ldg<NT>(g + (size_t)e * Vh);
        if (!r12) {
#pragma unroll
            for (int e = 12; e < 18; ++e) w.v[e] = ldg<NT>(g + (size_t)e * Vh);
        }
    } else if constexpr (P == P32) {
        const f4v* g = (const f4v*)G + (size_t)((r12 ? 6 : 9) * mu) * Vh + s;
#pragma unroll
        for (int e = 0; e < 6; ++e) w.v[e] = ldg<NT>(g + (size_t)e * Vh);
        if (!r12) {
#pragma unroll
            for (int e = 6; e < 9; ++e) w.v[e] = ldg<NT>(g + (size_t)e * Vh);
        }
    } else {
        const u2v* g = (const u2v*)G + (size_t)((r12 ? 6 : 9) * mu) * Vh + s;
        w.sc = gscale[s];
#pragma unroll
        for (int e = 0; e < 6; ++e) w.v[e] = ldg<NT>(g + (size_t)e * Vh);
        if (!r12) {
#pragma unroll
            for (int e = 6; e < 9; ++e) w.v[e] = ldg<NT>(g + (size_t)e * Vh);
        }
    }
}

// Output factors of a hop pair (finish_pair): the pair sum is
// p = S (F chi(x + h) + sigma B chi(x - h)) over the links F, B as
// finish_pair leaves them, S = diag(s01, s01, s2) on the colour rows.
// Stored full links hold the phases (sigma = +1, S = 1); with r12 the phase
// eta goes to S and sigma = -1 (the backward link is -eta U^dagger). Scaling
// by +-1 is exact, so p has the bits of multiplying the links themselves.
// fp16 links are left divided by the site scale s and S carries it (s, and
// s^2 on a row rebuilt from two divided rows): three multiplies per pair in
// place of one per entry.
template <typename T>
struct PairScale {
    T s01, s2, sigma;
};

// The 18 complex entries of a pair from what load_pair_raw loaded, with the
// factors that complete them (PairScale): with r12 the third rows are
// rebuilt. Both forms are formed and one is selected per entry.
template <int P>
__device__ __forceinline__ void finish_pair(int r12, int eta, const PairRaw<P>& w,
                                            typename Real<P>::T (&lr)[18],
                                            typename Real<P>::T (&li)[18],
                                            PairScale<typename Real<P>::T>& ps) {
    using T = typename Real<P>::T;
    T fr[18], fi[18], cr[18], ci[18];  // full, compressed
    if constexpr (P == P64) {
#pragma unroll
        for (int e = 0; e < 18; ++e) {
            fr[e] = w.v[e].x;
            fi[e] = w.v[e].y;
        }
#pragma unroll
        for (int e = 0; e < 6; ++e) {
            cr[e] = w.v[e].x;
            ci[e] = w.v[e].y;
            cr[9 + e] = w.v[6 + e].x;
            ci[9 + e] = w.v[6 + e].y;
        }
    } else {
        // word e holds entries 2e and 2e + 1 (P32 as floats, P16S as fp16
        // pairs, still divided by the site scale)
        T wr[18], wi[18];
#pragma unroll
        for (int e = 0; e < 9; ++e) {
            if constexpr (P == P32) {
                wr[2 * e] = w.v[e].x;
                wi[2 * e] = w.v[e].y;
                wr[2 * e + 1] = w.v[e].z;
                wi[2 * e + 1] = w.v[e].w;
            } else {
                wr[2 * e] = h2f_lo(w.v[e].x);
                wi[2 * e] = h2f_hi(w.v[e].x);
                wr[2 * e + 1] = h2f_lo(w.v[e].y);
                wi[2 * e + 1] = h2f_hi(w.v[e].y);
            }
        }
#pragma unroll
        for (int e = 0; e < 18; ++e) {
            fr[e] = wr[e];
            fi[e] = wi[e];
        }
#pragma unroll
        for (int e = 0; e < 6; ++e) {
            cr[e] = wr[e];
            ci[e] = wi[e];
            cr[9 + e] = wr[6 + e];
            ci[9 + e] = wi[6 + e];
        }
    }
    third_row(cr, ci, 0);
    third_row(cr, ci, 9);
#pragma unroll
    for (int e = 0; e < 18; ++e) {
        lr[e] = r12 ? cr[e] : fr[e];
        li[e] = r12 ? ci[e] : fi[e];
    }
    const T sg = r12 ? (T)eta : T(1);
    if constexpr (P == P16S) {
        ps.s01 = sg * w.sc;
        ps.s2 = r12 ? sg * (w.sc * w.sc) : sg * w.sc;
    } else {
        ps.s01 = ps.s2 = sg;
    }
    ps.sigma = r12 ? T(-1) : T(1);
}

// Both steps at once: hop pair mu of output site s, ready to apply.
template <int P, bool NT>
__device__ __forceinline__ void load_pair(const void* G, const float* gscale, uint32_t Vh,
                                          uint32_t s, int mu, int r12, int eta,
                                          typename Real<P>::T (&lr)[18],
                                          typename Real<P>::T (&li)[18],
                                          PairScale<typename Real<P>::T>& ps) {
    PairRaw<P> w;
    load_pair_raw<P, NT>(G, gscale, Vh, s, mu, r12, w);
    finish_pair<P>(r12, eta, w, lr, li, ps);
}

// eta_mu(x) = (-1)^(x_0 + ... + x_{mu-1}) of the site with coordinates x, y, z.
__device__ __forceinline__ int eta_sign(int mu, int x, int y, int z) {
    const int s = (mu > 0 ? x : 0) + (mu > 1 ? y : 0) + (mu > 2 ? z : 0);
    return (s & 1) ? -1 : 1;
}

// acc += L v for the 3x3 complex matrix starting at entry `o` of (lr, li).
template <typename T>
__device__ __forceinline__ void matvec_acc(const T (&lr)[18], const T (&li)[18], int o,
                                           const T (&vr)[3], const T (&vi)[3], T (&ar)[3],
                                           T (&ai)[3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const T ur = lr[o + 3 * a + b], ui = li[o + 3 * a + b];
            ar[a] = fma(ur, vr[b], ar[a]);
            ar[a] = fma(-ui, vi[b], ar[a]);
            ai[a] = fma(ur, vi[b], ai[a]);
            ai[a] = fma(ui, vr[b], ai[a]);
        }
    }
}

// p = S (F vf + sigma B vb) for one pair (PairScale), in two steps so that
// vb can be formed after vf has been used: pair_start(F vf), then
// pair_finish(vb) adds sigma B vb and applies S.
template <typename T>
__device__ __forceinline__ void pair_start(const T (&lr)[18], const T (&li)[18], const T (&vfr)[3],
                                           const T (&vfi)[3], T (&pr)[3], T (&pi)[3]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) pr[c] = pi[c] = T(0);
    matvec_acc(lr, li, 0, vfr, vfi, pr, pi);
}

template <typename T>
__device__ __forceinline__ void pair_finish(const T (&lr)[18], const T (&li)[18],
                                            const PairScale<T>& ps, const T (&vbr)[3],
                                            const T (&vbi)[3], T (&pr)[3], T (&pi)[3]) {
    T br[3], bi[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        br[c] = ps.sigma * vbr[c];
        bi[c] = ps.sigma * vbi[c];
    }
    matvec_acc(lr, li, 9, br, bi, pr, pi);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const T f = c < 2 ? ps.s01 : ps.s2;
        pr[c] *= f;
        pi[c] *= f;
    }
}

// ------------------------------------------------------------------ launch geometry

// Map the hardware block index to the block of sites it handles (a block
// always handles one contiguous range of sites, so the work, the rounding and
// the reduction chunks do not depend on the mapping).
// swizzle >= 1: each of the eight XCDs (which receive blocks round-robin)
// works on one contiguous eighth of the blocks; neighbouring blocks then
// share that XCD's L2.
// swizzle >= 2 with bps (blocks per t-slice, i.e. per Lx Ly Lz / 2 sites)
// set: those blocks are then taken in groups of TB = 2^(swizzle - 1)
// consecutive t-slices, and within a group t runs fastest. A site's
// t-neighbours are then TB blocks or fewer away in launch order instead of a
// whole slice, so the direction vectors a hop stage gathers there are still
// in L2 (with several right-hand sides a slice's links, inputs and outputs
// overflow the XCD's 4 MB L2, and every input is otherwise fetched again for
// each of its two t-neighbours). The caller sets bps only when the grid is
// Lt x bps blocks and TB divides Lt.
__device__ __forceinline__ uint32_t logical_block(int swizzle, uint32_t bps = 0) {
    const uint32_t k = blockIdx.x, nb = gridDim.x;
    uint32_t v = k;
    if (swizzle && nb >= 16) {
        const uint32_t q = nb >> 3, rem = nb & 7, x = k & 7, i = k >> 3;
        v = x * q + (x < rem ? x : rem) + i;
    }
    if (swizzle >= 2 && bps) {
        const uint32_t tb = 1u << (swizzle - 1);
        const uint32_t grp = tb * bps;  // blocks per group of tb slices
        const uint32_t tg = v / grp, rem = v - tg * grp;
        const uint32_t j = rem / tb, tt = rem - j * tb;
        v = (tg * tb + tt) * bps + j;
    }
    return v;
}

// ------------------------------------------------------------------ reductions

// Per-RHS finalisation of a reduced sum (run by one thread).
__device__ __forceinline__ void finalize_one(int kind, RhsState* sp, double sum, double* out) {
    if (kind == FIN_STORE) {
        if (out) *out = sum;
        return;
    }
    RhsState& s = *sp;
    switch (kind) {
        case FIN_ALPHA:
            s.pAp = sum;
            if (!(sum > 0.0) || !isfinite(sum)) {
                s.flags = F_BREAKDOWN;
            } else {
                // the Lanczos diagonal of this step, a Rayleigh quotient of the
                // residual; taken from the first cycle only (later cycles of a
                // low-precision recurrence lose that meaning)
                if (s.cg_budget > 0.0 && s.updates == 0)
                    s.lam = fmax(s.lam, sum / s.rr + (s.beta > 0.0 && s.alpha > 0.0 ? s.beta / s.alpha : 0.0));
                s.alpha = s.rr / sum;
            }
            break;
        case FIN_CG: {
            s.rr_old = s.rr;
            s.rr = sum;
            s.iters += 1;
            s.beta = sum / s.rr_old;
            if (!isfinite(sum)) {
                s.flags = F_BREAKDOWN;
            } else if (sum <= s.rr_stop) {
                s.flags = F_CONV;
            } else if (s.iters >= s.max_iter) {
                s.flags = F_CONV | F_MAXIT;
            }
            break;
        }
        case FIN_MIXED: {
            s.rr_old = s.rr;
            s.rr = sum;
            s.iters += 1;
            s.beta = sum / s.rr_old;
            const double rn = sqrt(sum);
            s.rmax = fmax(s.rmax, rn);
            if (rn < s.rmin) {
                s.rmin = rn;
                s.since = 0;
            } else {
                s.since += 1;
            }
            if (!isfinite(sum)) {
                s.flags = F_BREAKDOWN;
            } else if (rn < s.delta * (s.variant == MIXED_RESTART ? s.rstart : s.rmax) ||
                       sum <= s.rr_stop) {
                s.flags = F_RU;
            } else if (s.since >= s.stall_iters) {
                s.flags = F_STALL;
            } else if (s.iters >= s.max_iter) {
                s.flags = F_RU | F_MAXIT;
            }
            break;
        }
        case FIN_INIT: {
            // the slot stays F_NEW (with F_X0 when it starts from x0) until
            // its first direction is set; b = 0 finishes it at once
            const unsigned x0 = s.flags & F_X0;
            s.bb = sum;
            s.rr_stop = s.tol2 * sum;
            s.rr = s.rr_old = s.rr_true = s.best_true = s.rr_true0 = sum;
            s.rmax = s.rmin = s.rstart = sqrt(sum);
            s.since = 0;
            s.beta = 0.0;  // first direction d = r
            if (!isfinite(sum)) {
                s.flags = F_BADINPUT;
            } else if (sum == 0.0 || (!x0 && sum <= s.rr_stop)) {
                s.flags = F_DONE;
            } else {
                s.flags = F_NEW | x0;
            }
            break;
        }
        case FIN_X0:
            // r = b - A x0 replaces r = b
            s.rr = s.rr_old = s.rr_true = s.best_true = s.rr_true0 = sum;
            s.rmax = s.rmin = s.rstart = sqrt(sum);
            if (!isfinite(sum)) {
                s.flags = F_BADINPUT;
            } else if (sum <= s.rr_stop) {
                s.flags = F_DONE;
            } else {
                s.flags = F_NEW;
            }
            break;
        case FIN_ACTIVATE:
            s.flags = F_ACTIVE;
            break;
        case FIN_TRUE:
            s.rr_true = sum;
            break;
        case FIN_FOLD: {
            // y has been folded into x; the iterated residual carries on (its
            // beta stays), after a stall from d = r
            const bool stall = (s.flags & F_STALL) != 0;
            s.updates += 1;
            if (s.rr <= s.rr_stop || (s.flags & F_MAXIT)) {
                s.flags = F_CHECK | (s.flags & F_MAXIT);
                break;
            }
            if (stall) {
                s.beta = 0.0;
                s.restarts += 1;
            }
            s.rmax = s.rmin = s.rstart = sqrt(s.rr);
            s.since = 0;
            s.flags = F_ACTIVE;
            break;
        }
        case FIN_FOLD_CHECK:
            s.rr_true = sum;
            s.flags = sum <= s.rr_stop ? F_DONE : ((s.flags & F_MAXIT) ? F_MAXIT : F_INACC);
            break;
        case FIN_RU_END: {
            const double rt = sum;
            const double rt_prev = s.rr_true;  // true |r|^2 at the previous update (or start)
            s.rr_true = rt;
            const bool stall = (s.flags & F_STALL) != 0;
            s.updates += 1;
            if (!isfinite(rt)) {
                s.flags = F_BREAKDOWN;
                break;
            }
            if (rt <= s.rr_stop) {
                s.rr = rt;
                s.flags = F_DONE;
                break;
            }
            if (s.flags & F_MAXIT) {
                s.rr = rt;
                s.flags = F_MAXIT;
                break;
            }
            // a refinement cycle reduces the true residual by about the inner
            // reduction (delta) when the inner precision suffices; one that
            // does not even reach slow_ratio shows the inner iteration cannot
            // refine this system: end the pass so the caller can hand over
            if (!stall && s.slow_ratio > 0.0 && rt > s.slow_ratio * s.slow_ratio * rt_prev) {
                s.rr = rt;
                s.flags = F_ESTALL;
                break;
            }
            // a pass that needs more than cg_budget times the iterations the
            // CG bound allows for the reduction reached so far (sqrt(kappa) from
            // lam and m^2 <= lambda_min; error bound 2 ((sk-1)/(sk+1))^k, the
            // residual up to sk further off) converges much slower than CG can
            // on this system: end it too
            if (!stall && s.cg_budget > 0.0 && s.lam > 0.0 && rt < s.rr_true0) {
                const double sk = sqrt(s.lam / s.m2);
                const double allow = 0.5 * sk * (log(2.0 / sqrt(rt / s.rr_true0)) + log(sk));
                if ((double)s.iters > s.cg_budget * allow) {
                    s.rr = rt;
                    s.flags = F_ESTALL;
                    break;
                }
            }
            // Eq.6: the next direction is r + beta d with beta = |r_true|^2 / |r_prev|^2;
            // a stall, and every update of the Fig.2 variant, restarts it from r
            const bool restart = stall || s.variant == MIXED_RESTART;
            s.beta = restart ? 0.0 : rt / s.rr_old;
            if (restart && !stall) s.restarts += 1;
            if (stall) {
                s.restarts += 1;
                if (rt < 0.25 * s.best_true) {
                    s.stall_count = 0;
                } else {
                    s.stall_count += 1;
                }
            }
            s.best_true = fmin(s.best_true, rt);
            if (stall && s.stall_count >= s.max_stall) {
                s.rr = rt;
                s.flags = F_ESTALL;
                break;
            }
            s.rr = rt;
            s.rmax = s.rmin = s.rstart = sqrt(rt);
            s.since = 0;
            s.flags = F_ACTIVE;
            break;
        }
        case FIN_CG_CHECK: {
            const double rt = sum;
            s.rr_true = rt;
            s.updates += 1;
            if (!isfinite(rt)) {
                s.flags = F_BREAKDOWN;
            } else if (rt <= s.rr_stop) {
                s.flags = F_DONE;
            } else if (s.flags & F_MAXIT) {
                s.flags = F_MAXIT;
            } else {
                s.rr = rt;
                s.restarts += 1;
                s.beta = 0.0;  // restart the direction from the true residual
                s.flags = F_ACTIVE;
            }
            break;
        }
        default:
            break;
    }
}

// Reduction partials are taken over fixed chunks of 64 consecutive sites,
// whatever the launch shape, and each chunk is summed by the same butterfly
// over the site index (the vector kernels, which have one launch shape, add
// a block's four chunk sums into one partial: block_partials); the consumer
// of a reduction then sums the partials of each right-hand side with one
// wavefront in a fixed order (wave_sum_partials). The result is therefore independent of how many
// lanes serve a site, of how many right-hand sides share the kernel and of
// which kernel forms the sum. No block waits for another and no atomics are
// used: on this chip cross-block atomics serialise (tens of ns per block),
// which made an in-kernel "last block finalises" tail cost several
// microseconds.
constexpr int kChunk = 64;

// v[r] is the value of the site handled by this thread (meaningful on the
// first lane of each site, i.e. threadIdx.x % S == 0); the block covers
// kBlock / S consecutive sites starting at blk * (kBlock / S).
template <int N, int S>
__device__ __forceinline__ void block_chunk_partials(double (&v)[N], const Reduce& R, uint32_t blk) {
    constexpr int SPB = kBlock / S;          // sites per block
    constexpr int CPB = SPB / kChunk;        // chunks per block (>= 1)
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if constexpr (S == 1) {
        // one wave is one chunk: reduce straight from registers
#pragma unroll
        for (int r = 0; r < N; ++r) {
            double x = v[r];
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
            const uint32_t ch = blk * CPB + wave;
            if (lane == 0 && ch < (uint32_t)R.nparts) R.partials[(size_t)r * R.nparts + ch] = x;
        }
    } else {
        __shared__ double sv[N][SPB];
        if (threadIdx.x % S == 0) {
#pragma unroll
            for (int r = 0; r < N; ++r) sv[r][threadIdx.x / S] = v[r];
        }
        __syncthreads();
        if (wave < CPB) {
#pragma unroll
            for (int r = 0; r < N; ++r) {
                double x = sv[r][wave * kChunk + lane];
#pragma unroll
                for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
                const uint32_t ch = blk * CPB + wave;
                if (lane == 0 && ch < (uint32_t)R.nparts) R.partials[(size_t)r * R.nparts + ch] = x;
            }
        }
    }
}

// One thread per site, kBlock sites per block (the vector kernels): the
// partial of each right-hand side is the block's, its four 64-site chunk
// sums (the butterfly of block_chunk_partials) added as (c0 + c1) + (c2 + c3).
// A quarter of the chunk count to sum for the reduction's consumers, and
// still the same whatever the launch (the vector kernels have one shape).
template <int N>
__device__ __forceinline__ void block_partials(double (&v)[N], const Reduce& R, uint32_t blk) {
    static_assert(kBlock == 4 * kChunk, "a block is four chunks");
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __shared__ double sw[N][4];
#pragma unroll
    for (int r = 0; r < N; ++r) {
        double x = v[r];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
        if (lane == 0) sw[r][wave] = x;
    }
    __syncthreads();
    if (threadIdx.x < N && blk < (uint32_t)R.nparts) {
        const int r = threadIdx.x;
        R.partials[(size_t)r * R.nparts + blk] = (sw[r][0] + sw[r][1]) + (sw[r][2] + sw[r][3]);
    }
}

// Fixed-order sum of one right-hand side's chunk partials by one
// wavefront: lane l accumulates partials l, l + 64, l + 128, ... into four
// interleaved running sums, combined as (s0 + s1) + (s2 + s3) and then
// across the wave by a butterfly. Every lane returns the same value (each
// exchange adds the same two numbers on both partners). U only sets how
// many rounds of four loads a lane has in flight before it adds them (the
// sum is bound by memory latency when the partials are many); the order of
// the additions, and so the result, is the same for every U.
template <int U = 4>
__device__ __forceinline__ double wave_sum_partials(const double* pp, int nparts) {
    const int lane = threadIdx.x & 63;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int i = lane;
    if constexpr (U > 4) {
        for (; i + (256 * U - 64) < nparts; i += 256 * U) {
            double v[4 * U];
#pragma unroll
            for (int u = 0; u < 4 * U; ++u) v[u] = pp[i + 64 * u];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                s0 += v[4 * u];
                s1 += v[4 * u + 1];
                s2 += v[4 * u + 2];
                s3 += v[4 * u + 3];
            }
        }
    }
#pragma unroll 4
    for (; i + 192 < nparts; i += 256) {
        s0 += pp[i];
        s1 += pp[i + 64];
        s2 += pp[i + 128];
        s3 += pp[i + 192];
    }
    if (i < nparts) s0 += pp[i];
    if (i + 64 < nparts) s1 += pp[i + 64];
    if (i + 128 < nparts) s2 += pp[i + 128];
    double x = (s0 + s1) + (s2 + s3);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

static_assert(sizeof(RhsState) % 8 == 0, "RhsState is copied as 8-byte words");
constexpr int kStateWords = (int)(sizeof(RhsState) / 8);

// Copy the first N states to LDS (block-wide; ends with a barrier).
template <int N>
__device__ __forceinline__ void load_state(const RhsState* st, RhsState* ls) {
    const unsigned long long* src = (const unsigned long long*)st;
    unsigned long long* dst = (unsigned long long*)ls;
    for (int i = threadIdx.x; i < N * kStateWords; i += blockDim.x) dst[i] = src[i];
    __syncthreads();
}

// Finalise reduction R as a one-block kernel of 64 N threads (the result of
// finalize_block, bit for bit): wave r sums RHS r's partials with many
// loads in flight, before the states are read, so the two latencies
// overlap; the sums of RHS not flagged in run_mask are discarded.
template <int N>
__device__ __forceinline__ void finalize_wide(const Reduce& R, unsigned run_mask, RhsState* ls) {
    constexpr int U = N <= 8 ? 16 : 8;  // loads in flight within the register budget
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const double sum = wave_sum_partials<U>(R.partials + (size_t)wave * R.nparts, R.nparts);
    if (!R.st) {
        if (lane == 0 && R.out) R.out[wave] = sum;
        return;
    }
    load_state<N>(R.st, ls);
    if (lane == 0 && (ls[wave].flags & run_mask)) finalize_one(R.kind, ls + wave, sum, R.out ? R.out + wave : nullptr);
    __syncthreads();
    unsigned long long* dst = (unsigned long long*)(R.st_out ? R.st_out : R.st);
    const unsigned long long* src = (const unsigned long long*)ls;
    for (int i = threadIdx.x; i < N * kStateWords; i += blockDim.x) dst[i] = src[i];
}

// Finalise reduction R for the first N right-hand sides, block-wide: the
// states are read from R.st into LDS (ls), every RHS whose flags match
// run_mask gets its partials summed (wave w takes RHS w, w + 4, ...) and
// R.kind applied to its LDS copy; then block 0 writes all N states to
// R.st_out (or back to R.st). Every block of a many-block consumer computes
// the same states, bit for bit, and uses its LDS copy; R.st is never
// written by such a kernel, so late blocks read the same input. With R.st
// null only FIN_STORE is meaningful: block 0 stores the sums to R.out.
template <int N>
__device__ __forceinline__ void finalize_block(const Reduce& R, unsigned run_mask, RhsState* ls) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nw = blockDim.x >> 6;
    if (!R.st) {
        for (int r = wave; r < N; r += nw) {
            const double sum = wave_sum_partials(R.partials + (size_t)r * R.nparts, R.nparts);
            if (lane == 0 && blockIdx.x == 0 && R.out) R.out[r] = sum;
        }
        return;
    }
    load_state<N>(R.st, ls);
    for (int r = wave; r < N; r += nw) {
        if (!(ls[r].flags & run_mask)) continue;  // uniform over the wave
        const double sum = wave_sum_partials(R.partials + (size_t)r * R.nparts, R.nparts);
        if (lane == 0) finalize_one(R.kind, ls + r, sum, blockIdx.x == 0 && R.out ? R.out + r : nullptr);
    }
    __syncthreads();
    if (blockIdx.x == 0) {
        unsigned long long* dst = (unsigned long long*)(R.st_out ? R.st_out : R.st);
        const unsigned long long* src = (const unsigned long long*)ls;
        for (int i = threadIdx.x; i < N * kStateWords; i += blockDim.x) dst[i] = src[i];
    }
}

// f(std::integral_constant<int, I>()) for I = I0 .. I1 - 1: a loop whose
// index is a compile-time constant in the body.
template <int I0, int I1, class F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (I0 < I1) {
        f(std::integral_constant<int, I0>());
        static_for<I0 + 1, I1>(f);
    }
}

// The state a single-RHS kernel without per-RHS state reads (no flags set,
// never written): the read then needs no branch, whose join would make every
// later load wait for it. In global memory like the states themselves, so
// the read stays a scalar load.
static __device__ RhsState kNoState{};

// Single right-hand side, many-block consumer: every wavefront holds the
// input state s (read by the caller), sums the partials and applies R.kind
// in its own registers, bit-identically in every wave, so no barrier or LDS
// is needed; thread 0 of block 0 writes the result to R.st_out (never to the
// input: other waves may still be reading it).
__device__ __forceinline__ void finalize_wave1(const Reduce& R, unsigned run_mask, RhsState& s) {
    // summed before the flags are read: the partials' loads then need not
    // wait for the state's
    const double sum = wave_sum_partials(R.partials, R.nparts);
    if (s.flags & run_mask) {
        const bool t0 = blockIdx.x == 0 && threadIdx.x == 0;
        finalize_one(R.kind, &s, sum, t0 && R.out ? R.out : nullptr);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *R.st_out = s;
}

}  // namespace stag
