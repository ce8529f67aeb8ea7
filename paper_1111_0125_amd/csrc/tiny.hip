// One-workgroup solves for tiny lattices: a whole CG solve (Fig.1, or the
// Sec.3.2 mixed scheme with its reliable and group-wise updates) of one
// right-hand side runs inside a single workgroup, which loops over the
// iterations with workgroup barriers between the stages and keeps the CG
// scalars in LDS. On lattices of a few thousand sites a kernel per stage
// is mostly launch latency; here an iteration costs a few barriers, and
// the right-hand sides of one call run as independent workgroups on
// different compute units. Every loop ends: the state enforces the
// iteration cap, and the kernel stops after `cap` loop turns whatever the
// state says.
#include "kern.h"
#include "launch.h"

namespace stag {

// Sum of one value per thread over the workgroup, in a fixed order: a
// butterfly within each wavefront, then the wavefront sums in wavefront
// order by thread 0. Every thread gets the result.
__device__ __forceinline__ double tiny_block_sum(double v, double* lds) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) lds[wave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < kTinyBlock / 64; ++w) s += lds[w];
        lds[kTinyBlock / 64] = s;
    }
    __syncthreads();
    const double s = lds[kTinyBlock / 64];
    __syncthreads();  // lds is reused by the next sum
    return s;
}

// Sites per pass of a hop stage: four lanes per site, one hop pair each.
constexpr int kTinySites = kTinyBlock / 4;

// The eight hops of Eq.5 at output site s of parity p_out, by the four
// lanes 4i..4i+3 of a site: lane j forms the pair sum p_j = F chi(x + j) +
// B chi(x - j), and two exchanges give (p0 + p1) + (p2 + p3) on all four
// lanes, the rounding of the hop kernel. Every lane of the workgroup calls
// it (the exchanges need all of them); invalid sites contribute nothing.
template <int P>
__device__ __forceinline__ void tiny_hop(const void* G, const float* gscale, const Geom& g, int r12,
                                         bool valid, uint32_t s, int j, int p_out, const void* in,
                                         typename Real<P>::T (&ar)[3],
                                         typename Real<P>::T (&ai)[3]) {
    using T = typename Real<P>::T;
#pragma unroll
    for (int c = 0; c < 3; ++c) ar[c] = ai[c] = T(0);
    if (valid) {
        int x, y, z, t;
        site_coords(g, s, p_out, x, y, z, t);
        uint32_t nf, nb;
        neighbours(g, s, x, y, z, t, j, nf, nb);
        T lr[18], li[18];
        PairScale<T> ps;
        load_pair<P, false>(G, gscale, g.Vh, s, j, r12, eta_sign(j, x, y, z), lr, li, ps);
        T vr[3], vi[3];
        load_site<P>(in, g.Vh, nf, vr, vi);
        pair_start(lr, li, vr, vi, ar, ai);
        load_site<P>(in, g.Vh, nb, vr, vi);
        pair_finish(lr, li, ps, vr, vi, ar, ai);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int off = 1; off < 4; off <<= 1) {
            ar[c] = ar[c] + __shfl_xor(ar[c], off, 64);
            ai[c] = ai[c] + __shfl_xor(ai[c], off, 64);
        }
}

// P = inner precision; P64: plain CG on x64 / r64 / d / t / Ad (all fp64).
template <int P>
__global__ __launch_bounds__(kTinyBlock) void k_tiny(TinyArgs a) {
    using T = typename Real<P>::T;
    constexpr bool mixed = P != P64;
    const int rhs = blockIdx.x;
    const uint32_t Vh = a.g.Vh;
    const int tid = threadIdx.x;
    __shared__ RhsState S;
    __shared__ double lds[kTinyBlock / 64 + 1];
    auto at = [rhs](const void* p, size_t rs) { return (char*)p + (size_t)rhs * rs; };
    const char* b = at(a.b64, a.rs64);
    char* x64 = at(a.x64, a.rs64);
    char* r64 = at(a.r64, a.rs64);
    char* t64 = at(a.t64, a.rs64);
    char* d = at(a.d, a.rsP);
    char* t = at(a.t, a.rsP);
    char* ad = at(a.Ad, a.rsP);
    char* rs = at(a.rs, a.rsP);     // iterated residual (P64: r64)
    char* y = at(a.y, a.rsY);       // correction y (fp32; P64: x64)
    if (tid == 0) S = a.st[rhs];
    __syncthreads();

    // r = b, x = 0, |b|^2 -> the start state (FIN_INIT)
    double acc = 0.0;
    for (uint32_t s = tid; s < Vh; s += kTinyBlock) {
        double br[3], bi[3], z[3] = {0.0, 0.0, 0.0}, zi[3] = {0.0, 0.0, 0.0};
        load_site<P64>(b, Vh, s, br, bi);
        store_site<P64>(r64, Vh, s, br, bi);
        store_site<P64>(x64, Vh, s, z, zi);
#pragma unroll
        for (int c = 0; c < 3; ++c) acc += br[c] * br[c] + bi[c] * bi[c];
    }
    double sum = tiny_block_sum(acc, lds);
    if (tid == 0) finalize_one(FIN_INIT, &S, sum, nullptr);
    __syncthreads();
    if (S.flags & F_NEW) {
        // first direction d = q(r); the inner residual rs = q(r); y = 0
        for (uint32_t s = tid; s < Vh; s += kTinyBlock) {
            double vr[3], vi[3];
            load_site<P64>(r64, Vh, s, vr, vi);
            T qr[3], qi[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                qr[c] = (T)vr[c];
                qi[c] = (T)vi[c];
            }
            store_site<P>(d, Vh, s, qr, qi);
            if constexpr (mixed) {
                store_site<P>(rs, Vh, s, qr, qi);
                float z[3] = {0.f, 0.f, 0.f}, zi[3] = {0.f, 0.f, 0.f};
                store_site<P32>(y, Vh, s, z, zi);
            }
        }
        __syncthreads();
        if (tid == 0) finalize_one(FIN_ACTIVATE, &S, 0.0, nullptr);
        __syncthreads();
    }

    for (int turn = 0; turn < a.cap; ++turn) {
        const unsigned f = S.flags;
        if (f & F_ACTIVE) {
            // one iteration: d = q(r + beta d), t = D_oe d, Ad = m^2 d - D_eo t,
            // alpha, x (y) += alpha d, r = q(r - alpha Ad), |r|^2
            const T be = (T)S.beta;
            for (uint32_t s = tid; s < Vh; s += kTinyBlock) {
                T rr[3], ri[3], dr[3], di[3];
                load_site<P>(rs, Vh, s, rr, ri);
                load_site<P>(d, Vh, s, dr, di);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    dr[c] = fma(be, dr[c], rr[c]);
                    di[c] = fma(be, di[c], ri[c]);
                }
                round_site<P>(dr, di);
                store_site<P>(d, Vh, s, dr, di);
            }
            __syncthreads();
            for (uint32_t base = 0; base < Vh; base += kTinySites) {
                const uint32_t s = base + tid / 4;
                T hr[3], hi[3];
                tiny_hop<P>(a.G[1], a.gscale[1], a.g, a.r12, s < Vh, s, tid & 3, 1, d, hr, hi);
                if (s < Vh && (tid & 3) == 0) store_site<P>(t, Vh, s, hr, hi);
            }
            __syncthreads();
            const T m2 = (T)S.m2;
            acc = 0.0;
            for (uint32_t base = 0; base < Vh; base += kTinySites) {
                const uint32_t s = base + tid / 4;
                T hr[3], hi[3], xr[3], xi[3];
                tiny_hop<P>(a.G[0], a.gscale[0], a.g, a.r12, s < Vh, s, tid & 3, 0, t, hr, hi);
                if (!(s < Vh && (tid & 3) == 0)) continue;
                load_site<P>(d, Vh, s, xr, xi);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    hr[c] = fma(m2, xr[c], -hr[c]);
                    hi[c] = fma(m2, xi[c], -hi[c]);
                }
                store_site<P>(ad, Vh, s, hr, hi);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    acc = fma((double)xr[c], (double)hr[c], acc);
                    acc = fma((double)xi[c], (double)hi[c], acc);
                }
            }
            sum = tiny_block_sum(acc, lds);
            if (tid == 0) finalize_one(FIN_ALPHA, &S, sum, nullptr);
            __syncthreads();
            if (!(S.flags & F_ACTIVE)) continue;  // breakdown
            acc = 0.0;
            if constexpr (mixed) {
                const float al = (float)S.alpha;
                for (uint32_t s = tid; s < Vh; s += kTinyBlock) {
                    float yr[3], yi[3];
                    T sr[3], si[3], dr[3], di[3], qr[3], qi[3];
                    load_site<P32>(y, Vh, s, yr, yi);
                    load_site<P>(rs, Vh, s, sr, si);
                    load_site<P>(d, Vh, s, dr, di);
                    load_site<P>(ad, Vh, s, qr, qi);
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        yr[c] = fmaf(al, dr[c], yr[c]);
                        yi[c] = fmaf(al, di[c], yi[c]);
                        sr[c] = fmaf(-al, qr[c], sr[c]);
                        si[c] = fmaf(-al, qi[c], si[c]);
                    }
                    store_site<P32>(y, Vh, s, yr, yi);
                    round_site<P>(sr, si);
                    store_site<P>(rs, Vh, s, sr, si);
#pragma unroll
                    for (int c = 0; c < 3; ++c)
                        acc += (double)sr[c] * (double)sr[c] + (double)si[c] * (double)si[c];
                }
            } else {
                const double al = S.alpha;
                for (uint32_t s = tid; s < Vh; s += kTinyBlock) {
                    double xr[3], xi[3], sr[3], si[3], dr[3], di[3], qr[3], qi[3];
                    load_site<P64>(x64, Vh, s, xr, xi);
                    load_site<P64>(r64, Vh, s, sr, si);
                    load_site<P64>(d, Vh, s, dr, di);
                    load_site<P64>(ad, Vh, s, qr, qi);
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        xr[c] = fma(al, dr[c], xr[c]);
                        xi[c] = fma(al, di[c], xi[c]);
                        sr[c] = fma(-al, qr[c], sr[c]);
                        si[c] = fma(-al, qi[c], si[c]);
                        acc += sr[c] * sr[c] + si[c] * si[c];
                    }
                    store_site<P64>(x64, Vh, s, xr, xi);
                    store_site<P64>(r64, Vh, s, sr, si);
                }
            }
            sum = tiny_block_sum(acc, lds);
            if (tid == 0) finalize_one(mixed ? FIN_MIXED : FIN_CG, &S, sum, nullptr);
            __syncthreads();
            continue;
        }
        const bool fixup = mixed ? (f & (F_RU | F_STALL)) != 0 : (f & F_CONV) != 0;
        if (!fixup) break;  // finished (or failed)
        // fp64 true residual: (mixed) x += y, y = 0; t64 = D_oe x;
        // r = b - (m^2 x - D_eo t64), |r|^2, (mixed) rs = q(r)
        if constexpr (mixed) {
            for (uint32_t s = tid; s < Vh; s += kTinyBlock) {
                double xr[3], xi[3];
                float yr[3], yi[3], z[3] = {0.f, 0.f, 0.f}, zi[3] = {0.f, 0.f, 0.f};
                load_site<P64>(x64, Vh, s, xr, xi);
                load_site<P32>(y, Vh, s, yr, yi);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    xr[c] = xr[c] + (double)yr[c];
                    xi[c] = xi[c] + (double)yi[c];
                }
                store_site<P64>(x64, Vh, s, xr, xi);
                store_site<P32>(y, Vh, s, z, zi);
            }
            __syncthreads();
        }
        for (uint32_t base = 0; base < Vh; base += kTinySites) {
            const uint32_t s = base + tid / 4;
            double hr[3], hi[3];
            tiny_hop<P64>(a.G64[1], nullptr, a.g, a.r12_64, s < Vh, s, tid & 3, 1, x64, hr, hi);
            if (s < Vh && (tid & 3) == 0) store_site<P64>(t64, Vh, s, hr, hi);
        }
        __syncthreads();
        const double m2 = S.m2;
        acc = 0.0;
        for (uint32_t base = 0; base < Vh; base += kTinySites) {
            const uint32_t s = base + tid / 4;
            double hr[3], hi[3], xr[3], xi[3], br[3], bi[3];
            tiny_hop<P64>(a.G64[0], nullptr, a.g, a.r12_64, s < Vh, s, tid & 3, 0, t64, hr, hi);
            if (!(s < Vh && (tid & 3) == 0)) continue;
            load_site<P64>(x64, Vh, s, xr, xi);
            load_site<P64>(b, Vh, s, br, bi);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                hr[c] = br[c] - fma(m2, xr[c], -hr[c]);
                hi[c] = bi[c] - fma(m2, xi[c], -hi[c]);
            }
            store_site<P64>(r64, Vh, s, hr, hi);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                acc = fma(hr[c], hr[c], acc);
                acc = fma(hi[c], hi[c], acc);
            }
            if constexpr (mixed) {
                float qr[3], qi[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    qr[c] = (float)hr[c];
                    qi[c] = (float)hi[c];
                }
                store_site<P>(rs, Vh, s, qr, qi);
            }
        }
        sum = tiny_block_sum(acc, lds);
        if (tid == 0) finalize_one(mixed ? FIN_RU_END : FIN_CG_CHECK, &S, sum, nullptr);
        __syncthreads();
    }
    if (tid == 0) a.st[rhs] = S;
}

hipError_t launch_tiny(int prec, int nrhs, const TinyArgs& a, hipStream_t stream) {
    TinyArgs arg = a;
    void* args[] = {&arg};
    const void* fn = prec == P64 ? reinterpret_cast<const void*>(&k_tiny<P64>)
                     : prec == P32 ? reinterpret_cast<const void*>(&k_tiny<P32>)
                     : prec == P16S ? reinterpret_cast<const void*>(&k_tiny<P16S>)
                                    : nullptr;
    if (!fn || nrhs < 1 || a.g.Vh < 1) return hipErrorInvalidValue;
    return hipLaunchKernel(fn, dim3((uint32_t)nrhs), dim3(kTinyBlock), args, 0, stream);
}

}  // namespace stag
