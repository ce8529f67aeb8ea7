// Hop kernel: the staggered Dirac operator of Eq.5 applied from one parity
// to the other, with optional second-stage epilogues that complete
// A = m^2 - D_eo D_oe (Eq.3). The phases of Sec.2 are folded into stored full
// links; with 12-parameter links they multiply each hop pair's outputs (as
// does the fp16 site scale: PairScale).
//
// The operator is a sum over NP hop pairs, each a forward and a backward hop
// whose two 3x3 links are stored contiguously per site: NP = 4 for Eq.5
// (pair mu: x +- mu), NP = 8 for the improved operator (pairs 4 + mu add the
// three-hops x +- 3mu over the long links). One output site is handled by S
// lanes of a wavefront (S = 1, 2 or 4); lane j of a site takes the pairs
// [j*NP/S, (j+1)*NP/S), and the S partial colour vectors are summed with
// cross-lane adds. With N > 1 right-hand sides every link is loaded once and
// applied to all of them (the block operator sharing gauge loads).
//
// This file is compiled once per storage precision (HOP_PREC) and pair
// count (HOP_NP).
#include "kern.h"
#include "launch.h"

#ifndef HOP_PREC
#error "HOP_PREC must be defined"
#endif
#ifndef HOP_NP
#define HOP_NP 4
#endif

namespace stag {

// What an operand is made of at one site: the stored input and, for a
// deferred direction update, the stored residual.
template <int P>
struct Raw {
    typename Real<P>::T vr[3], vi[3], rr[3], ri[3];
};

// Load the raw operand of RHS r at site n (the residual only when `lazy`).
template <int P>
__device__ __forceinline__ void load_raw(const HopArgs& a, const char* in_r, int r, uint32_t n,
                                         bool lazy, Raw<P>& w) {
    load_site<P>(in_r, a.g.Vh, n, w.vr, w.vi);
    if (lazy) load_site<P>((const char*)a.lazy_r + (size_t)r * a.lazy_r_rs, a.g.Vh, n, w.rr, w.ri);
}

// The operand from its raw parts: the stored input, or d_new = q(r + beta d)
// for a deferred direction update; with `add_y` in the fp64 stages of a
// reliable update (x gathered by stage 1, x at stage 2's own site), x + y.
template <int P>
__device__ __forceinline__ void combine(const HopArgs& a, const Raw<P>& w, int r, uint32_t n,
                                        bool lazy, double beta, bool add_y,
                                        typename Real<P>::T (&vr)[3],
                                        typename Real<P>::T (&vi)[3]) {
    using T = typename Real<P>::T;
    if (lazy) {
        const T be = (T)beta;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            vr[c] = fma(be, w.vr[c], w.rr[c]);
            vi[c] = fma(be, w.vi[c], w.ri[c]);
        }
        round_site<P>(vr, vi);
    } else {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            vr[c] = w.vr[c];
            vi[c] = w.vi[c];
        }
    }
    if constexpr (P == P64) {
        if (add_y && a.lazy_y) {
            float yr[3], yi[3];
            load_site<P32>((const char*)a.lazy_y + (size_t)r * a.lazy_y_rs, a.g.Vh, n, yr, yi);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                vr[c] = vr[c] + (T)yr[c];
                vi[c] = vi[c] + (T)yi[c];
            }
        }
    }
}

// The own-site operand of stage 2 (x, formed like a stage-1 operand).
template <int P>
__device__ __forceinline__ void load_operand(const HopArgs& a, const char* in_r, int r, uint32_t n,
                                             bool lazy, double beta, typename Real<P>::T (&vr)[3],
                                             typename Real<P>::T (&vi)[3]) {
    Raw<P> w;
    load_raw<P>(a, in_r, r, n, lazy, w);
    combine<P>(a, w, r, n, lazy, beta, true, vr, vi);
}

// Neighbours of hop pair pr (pairs 4..7 are the three-hops of the improved operator).
template <int NP>
__device__ __forceinline__ void pair_neighbours(const Geom& g, uint32_t s, int x, int y, int z,
                                                int t, int pr, uint32_t& nf, uint32_t& nb) {
    if (NP == 4 || pr < 4) {
        neighbours(g, s, x, y, z, t, pr & 3, nf, nb);
    } else {
        neighbours3(g, s, x, y, z, t, pr & 3, nf, nb);
    }
}

template <int P, int S, int N, int EPI, bool NT, int NP>
__global__ __launch_bounds__(kBlock) void k_hop(HopArgs a) {
    // NP: hop pairs per site
    constexpr int B = NP / S;   // pairs per lane
    constexpr int LOGB = B >= 8 ? 3 : B >= 4 ? 2 : B >= 2 ? 1 : 0;
    static_assert(B >= 1 && (1 << LOGB) == B, "pairs per lane must be a power of two");
    using T = typename Real<P>::T;
    const uint32_t blk = logical_block(a.swizzle, a.tile_bps);
    const uint32_t gt = blk * kBlock + threadIdx.x;
    const uint32_t s = gt / S;
    const int j = (int)(gt % S);
    const uint32_t Vh = a.g.Vh;
    const bool valid = s < Vh;
    // stage 1 forms the deferred direction at the neighbours it gathers
    const bool lazy_nb = EPI == EPI_PLAIN && a.lazy_r != nullptr;
    // the improved operator's fat and long links are always stored full
    const int r12 = NP == 4 ? a.r12 : 0;

    // Per-RHS state, finalised here from the previous reduction's partials
    // when a.fin is set. One RHS: each wavefront keeps it in registers (no
    // barrier); the state, the operands of the lane's hop pairs (all of them
    // when they fit in registers, else the first), the own-site operand of
    // the second stage and the partials are all requested before any of them
    // is used, so their memory latencies overlap (an inactive slot reads the
    // operands and discards them). Neighbours go before links: rebuilding
    // 12-parameter links waits for the link loads, and would hold back loads
    // issued after them. Several RHS: the block shares one copy in LDS.
    constexpr bool PRE = N == 1 && P != P16S && B * sizeof(T) <= 8;
    constexpr int PB = N == 1 ? (PRE ? B : 1) : 1;  // pairs requested up front
    __shared__ RhsState ls[N];
    RhsState s1{};
    unsigned act = (1u << N) - 1u;
    int x = 0, y = 0, z = 0, t = 0;
    if (valid) site_coords(a.g, s, a.p_out, x, y, z, t);
    [[maybe_unused]] uint32_t pnf[PB], pnb[PB];
    [[maybe_unused]] PairRaw<P> pl[PB];
    [[maybe_unused]] Raw<P> pwf[PB], pwb[PB], pown;
    if constexpr (N == 1) {
        if constexpr (P == P64) {
            // gated launches (the fp64 fix-ups and checks): an unflagged slot
            // has nothing to do, no operand read and no partials (the
            // reduction's consumer skips unflagged slots). Its own load and
            // branch, so the others need not wait for the flags before
            // their operand loads; the inner-precision kernels, never gated,
            // carry no branch at all.
            if (a.gate) {
                if (!(a.st->flags & a.run_mask)) return;
            }
        }
        s1 = *(a.st ? a.st : &kNoState);
        if (a.st && !(s1.flags & a.run_mask)) act = 0;
        if (valid) {
            static_for<0, PB>([&](auto kc) {
                constexpr int k = decltype(kc)::value;
                pair_neighbours<NP>(a.g, s, x, y, z, t, j * B + k, pnf[k], pnb[k]);
                load_raw<P>(a, (const char*)a.in, 0, pnf[k], lazy_nb, pwf[k]);
                load_raw<P>(a, (const char*)a.in, 0, pnb[k], lazy_nb, pwb[k]);
            });
            if constexpr (PRE && EPI != EPI_PLAIN) {
                if (j == 0) load_raw<P>(a, (const char*)a.x, 0, s, a.lazy_r != nullptr, pown);
            }
            static_for<0, PB>([&](auto kc) {
                constexpr int k = decltype(kc)::value;
                load_pair_raw<P, NT>(a.gauge, a.gscale, Vh, s, j * B + k, r12, pl[k]);
            });
        }
        if (a.st && a.fin.partials) {
            // always: block 0 must pass the state on even when it is inactive
            Reduce F = a.fin;
            F.st = a.st;
            finalize_wave1(F, a.run_mask, s1);
            if (!(s1.flags & a.run_mask)) act = 0;
        }
    } else if (a.st) {
        if (a.fin.partials) {
            Reduce F = a.fin;
            F.st = a.st;
            finalize_block<N>(F, a.run_mask, ls);
        } else {
            load_state<N>(a.st, ls);
        }
        act = 0;
#pragma unroll
        for (int r = 0; r < N; ++r)
            if (ls[r].flags & a.run_mask) act |= 1u << r;
    }
    auto stv = [&](int r) -> const RhsState& {
        if constexpr (N == 1) {
            return s1;
        } else {
            return ls[r];
        }
    };

    T ar[N][3], ai[N][3];
    // pending sums of the lane's pair tree: pd[l] holds the sum of the
    // 2^l pairs that wait for their right-hand sibling
    [[maybe_unused]] T pdr[LOGB > 0 ? LOGB : 1][N][3], pdi[LOGB > 0 ? LOGB : 1][N][3];
#pragma unroll
    for (int r = 0; r < N; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            ar[r][c] = ai[r][c] = T(0);
#pragma unroll
            for (int l = 0; l < (LOGB > 0 ? LOGB : 1); ++l) pdr[l][r][c] = pdi[l][r][c] = T(0);
        }

    if (valid && act) {
        // Each hop pair contributes p = F chi(x+h) + B chi(x-h), accumulated
        // from zero; the pairs are summed along a balanced binary tree
        // ((p0 + p1) + (p2 + p3)) + ..., lane-locally over the aligned block
        // of pairs this lane owns and across the S lanes of the site below.
        // This fixes the rounding independently of S and of the number of
        // right-hand sides.
        // (a loop over the lane's pairs with a compile-time index, so that
        // the arrays of operands requested up front stay in registers)
        static_for<0, B>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            const int mu = j * B + k;  // hop pair index
            uint32_t nf, nb;
            T lr[18], li[18];
            PairScale<T> ps;
            [[maybe_unused]] Raw<P> wfk, wbk;
            if constexpr (N == 1 && k < PB) {
                nf = pnf[k];
                nb = pnb[k];
                finish_pair<P>(r12, eta_sign(mu & 3, x, y, z), pl[k], lr, li, ps);
            } else {
                pair_neighbours<NP>(a.g, s, x, y, z, t, mu, nf, nb);
                if constexpr (N == 1) {
                    // one RHS: neighbours before links, as for the first pair
                    load_raw<P>(a, (const char*)a.in, 0, nf, lazy_nb, wfk);
                    load_raw<P>(a, (const char*)a.in, 0, nb, lazy_nb, wbk);
                }
                load_pair<P, NT>(a.gauge, a.gscale, Vh, s, mu, r12, eta_sign(mu & 3, x, y, z), lr, li, ps);
            }
#pragma unroll
            for (int r = 0; r < N; ++r) {
                if (!((act >> r) & 1u)) continue;
                const char* in_r = (const char*)a.in + (size_t)r * a.in_rs;
                const double be = lazy_nb ? stv(r).beta : 0.0;
                Raw<P> wf, wb;
                if constexpr (N == 1 && k < PB) {
                    wf = pwf[k];
                    wb = pwb[k];
                } else if constexpr (N == 1) {
                    wf = wfk;
                    wb = wbk;
                } else {
                    load_raw<P>(a, in_r, r, nf, lazy_nb, wf);
                    load_raw<P>(a, in_r, r, nb, lazy_nb, wb);
                }
                T vr[3], vi[3], pr[3], pi[3];
                // stage 2 gathers t as stored
                combine<P>(a, wf, r, nf, lazy_nb, be, EPI == EPI_PLAIN, vr, vi);
                pair_start(lr, li, vr, vi, pr, pi);
                combine<P>(a, wb, r, nb, lazy_nb, be, EPI == EPI_PLAIN, vr, vi);
                pair_finish(lr, li, ps, vr, vi, pr, pi);
                // binary-counter walk of the tree: the new pair sum is
                // the right sibling of every pending sum at the levels
                // where k has a 1 bit, and waits at the first 0 bit
                T cr[3], ci[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    cr[c] = pr[c];
                    ci[c] = pi[c];
                }
                bool done = false;
#pragma unroll
                for (int l = 0; l < LOGB; ++l) {
                    if (done) continue;
                    if ((k >> l) & 1) {
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            cr[c] = pdr[l][r][c] + cr[c];
                            ci[c] = pdi[l][r][c] + ci[c];
                        }
                    } else {
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            pdr[l][r][c] = cr[c];
                            pdi[l][r][c] = ci[c];
                        }
                        done = true;
                    }
                }
                if (k == B - 1) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        ar[r][c] = cr[c];
                        ai[r][c] = ci[c];
                    }
                }
            }
        });
    }
    if constexpr (S > 1) {
        // lanes 2i and 2i + 1 hold the sums of consecutive aligned blocks;
        // xor 1 forms the sums of their parent nodes, xor 2 of the next
        // level. IEEE addition is commutative, so both lanes of each
        // exchange hold the same value.
#pragma unroll
        for (int r = 0; r < N; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int off = 1; off < S; off <<= 1) {
                    ar[r][c] = ar[r][c] + __shfl_xor(ar[r][c], off, 64);
                    ai[r][c] = ai[r][c] + __shfl_xor(ai[r][c], off, 64);
                }
    }

    double dv[N];
#pragma unroll
    for (int r = 0; r < N; ++r) dv[r] = 0.0;

    if (valid && j == 0) {
#pragma unroll
        for (int r = 0; r < N; ++r) {
            if (!((act >> r) & 1u)) continue;
            char* out_r = (char*)a.out + (size_t)r * a.out_rs;
            if constexpr (EPI == EPI_PLAIN) {
                store_site<P>(out_r, Vh, s, ar[r], ai[r]);
            } else {
                T xr[3], xi[3], hr[3], hi[3];
                if constexpr (PRE) {
                    combine<P>(a, pown, r, s, a.lazy_r != nullptr, a.lazy_r ? stv(r).beta : 0.0, true,
                               xr, xi);
                } else {
                    load_operand<P>(a, (const char*)a.x + (size_t)r * a.x_rs, r, s, a.lazy_r != nullptr,
                                    a.lazy_r ? stv(r).beta : 0.0, xr, xi);
                }
                if (a.lazy_r) store_site<P>((char*)a.x + (size_t)r * a.x_rs, Vh, s, xr, xi);
                if constexpr (P == P64) {
                    if (a.lazy_y && !a.keep_y) {
                        // x += y in fp64, y = 0 (the group-wise update of Sec.3.2)
                        store_site<P>((char*)a.x + (size_t)r * a.x_rs, Vh, s, xr, xi);
                        float z[3] = {0.f, 0.f, 0.f}, zi[3] = {0.f, 0.f, 0.f};
                        store_site<P32>((char*)a.lazy_y + (size_t)r * a.lazy_y_rs, Vh, s, z, zi);
                    }
                }
                const T m2 = (T)(a.st ? stv(r).m2 : a.m2[r]);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    hr[c] = fma(m2, xr[c], -ar[r][c]);
                    hi[c] = fma(m2, xi[c], -ai[r][c]);
                }
                if constexpr (EPI == EPI_RESID) {
                    T br[3], bi[3];
                    load_site<P>((const char*)a.b + (size_t)r * a.b_rs, Vh, s, br, bi);
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        hr[c] = br[c] - hr[c];
                        hi[c] = bi[c] - hi[c];
                    }
                    store_site<P>(out_r, Vh, s, hr, hi);
                    double acc = 0.0;
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        acc = fma((double)hr[c], (double)hr[c], acc);
                        acc = fma((double)hi[c], (double)hi[c], acc);
                    }
                    dv[r] = acc;
                    if (a.aux) {
                        // the inner residual restarts from the true one: rs = q(r)
                        float qr[3], qi[3];
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            qr[c] = (float)hr[c];
                            qi[c] = (float)hi[c];
                        }
                        char* aux_r = (char*)a.aux + (size_t)r * a.aux_rs;
                        if (a.aux_prec == P16S) {
                            store_site<P16S>(aux_r, Vh, s, qr, qi);
                        } else {
                            store_site<P32>(aux_r, Vh, s, qr, qi);
                        }
                    }
                } else {
                    store_site<P>(out_r, Vh, s, hr, hi);
                    if constexpr (EPI == EPI_XPAY_DOT) {
                        double acc = 0.0;
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            acc = fma((double)xr[c], (double)hr[c], acc);
                            acc = fma((double)xi[c], (double)hi[c], acc);
                        }
                        dv[r] = acc;
                    }
                }
            }
        }
    }
    if constexpr (EPI == EPI_XPAY_DOT || EPI == EPI_RESID) {
        block_chunk_partials<N, S>(dv, a.red, blk);
    }
}

template <int P, int S, int N, int EPI, bool NT>
static hipError_t run_hop(const HopArgs& a, const Issue& is) {
    HopArgs arg = a;
    void* args[] = {&arg};
    return issue_kernel(is, reinterpret_cast<const void*>(&k_hop<P, S, N, EPI, NT, HOP_NP>),
                        hop_blocks(a.g.Vh, S), kBlock, args);
}

// Several RHS: non-temporal link loads, S in {1, 2, 4}.
template <int P, int EPI, int N>
static hipError_t run_block(int S, const HopArgs& a, const Issue& is) {
    if (S == 1) return run_hop<P, 1, N, EPI, true>(a, is);
    if (S == 2) return run_hop<P, 2, N, EPI, true>(a, is);
    if (S == 4) return run_hop<P, 4, N, EPI, true>(a, is);
    return hipErrorInvalidValue;
}

// Dispatch for this precision: N = 1 with S in {1, 2, 4} and both load
// flavours; N > 1 with S in {1, 2, 4} and non-temporal link loads.
template <int P, int EPI>
static hipError_t dispatch_epi(int S, int N, bool nt, const HopArgs& a, const Issue& is) {
    if (N == 1) {
        if (nt) {
            if (S == 1) return run_hop<P, 1, 1, EPI, true>(a, is);
            if (S == 2) return run_hop<P, 2, 1, EPI, true>(a, is);
            if (S == 4) return run_hop<P, 4, 1, EPI, true>(a, is);
        } else {
            if (S == 1) return run_hop<P, 1, 1, EPI, false>(a, is);
            if (S == 2) return run_hop<P, 2, 1, EPI, false>(a, is);
            if (S == 4) return run_hop<P, 4, 1, EPI, false>(a, is);
        }
        return hipErrorInvalidValue;
    }
    switch (N) {
        case 2: return run_block<P, EPI, 2>(S, a, is);
        case 4: return run_block<P, EPI, 4>(S, a, is);
        case 8: return run_block<P, EPI, 8>(S, a, is);
        case 12: return run_block<P, EPI, 12>(S, a, is);
        case 16: return run_block<P, EPI, 16>(S, a, is);
        default: return hipErrorInvalidValue;
    }
}

#define HOP_FN_NAME_(p, np) launch_hop_p##p##_n##np
#define HOP_FN_NAME(p, np) HOP_FN_NAME_(p, np)

hipError_t HOP_FN_NAME(HOP_PREC, HOP_NP)(int S, int N, int epi, bool nt, const HopArgs& a,
                                          const Issue& is) {
    constexpr int P = HOP_PREC;
    switch (epi) {
        case EPI_PLAIN: return dispatch_epi<P, EPI_PLAIN>(S, N, nt, a, is);
        case EPI_XPAY: return dispatch_epi<P, EPI_XPAY>(S, N, nt, a, is);
        case EPI_XPAY_DOT: return dispatch_epi<P, EPI_XPAY_DOT>(S, N, nt, a, is);
        case EPI_RESID:
            if constexpr (P == P64) return dispatch_epi<P, EPI_RESID>(S, N, nt, a, is);
            return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

}  // namespace stag
