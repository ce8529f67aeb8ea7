// Layout kernels: canonical complex128 host layouts <-> internal storage.
//
// Gauge packing folds the staggered phases into the links (Sec.2: the phase
// eta_mu(x) is multiplied into U_mu in advance), builds the eight hop links
// of every output site (sixteen for the improved operator; backward links
// daggered and negated, so the Dirac operator of Eq.5 becomes a plain sum),
// splits by parity and writes the word-major layout of common.h, rounding
// to the storage precision.
#include "kern.h"
#include "launch.h"

namespace stag {

__device__ __forceinline__ double eta_of(int mu, int x, int y, int z) {
    // eta_mu(x) = (-1)^(x_0 + ... + x_{mu-1})
    int s = 0;
    if (mu > 0) s += x;
    if (mu > 1) s += y;
    if (mu > 2) s += z;
    return (s & 1) ? -1.0 : 1.0;
}

// Hop pair pr of output site c (pairs 0..3: one-hop over U, pairs 4..7 of
// the improved operator: three-hop over Ulong): 18 complex in fp64, the
// forward link eta W(x) then -(eta W(x - h))^dagger.
__device__ __forceinline__ void hop_pair(const d2v* __restrict__ U, const d2v* __restrict__ Ulong,
                                         const Geom& g, const int (&c)[4], int pr, double (&lr)[18],
                                         double (&li)[18]) {
    const int mu = pr & 3;
    const int dist = pr < 4 ? 1 : 3;
    const d2v* W = pr < 4 ? U : Ulong;
    const int Lx = g.L[0], Ly = g.L[1], Lz = g.L[2];
    auto lex_of = [&](const int* q) -> size_t {
        return (size_t)q[0] + (size_t)Lx * ((size_t)q[1] + (size_t)Ly * ((size_t)q[2] + (size_t)Lz * q[3]));
    };
    int b[4] = {c[0], c[1], c[2], c[3]};
    b[mu] -= dist;
    while (b[mu] < 0) b[mu] += g.L[mu];
    const double ef = eta_of(mu, c[0], c[1], c[2]);
    const double eb = eta_of(mu, b[0], b[1], b[2]);
    const d2v* uf = W + (lex_of(c) * 4 + mu) * 9;
    const d2v* ub = W + (lex_of(b) * 4 + mu) * 9;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const d2v f = uf[i * 3 + k];
            lr[3 * i + k] = ef * f.x;
            li[3 * i + k] = ef * f.y;
            // -(eb W)^dagger: entry (i, k) = -eb conj(W[k][i])
            const d2v v = ub[k * 3 + i];
            lr[9 + 3 * i + k] = -eb * v.x;
            li[9 + 3 * i + k] = eb * v.y;
        }
}

// Full (18-parameter) packing of every hop pair; Ulong null: Eq.5's four
// pairs, else the improved operator's eight.
template <int P>
__global__ __launch_bounds__(kBlock) void k_gauge_pack(const d2v* __restrict__ U,
                                                       const d2v* __restrict__ Ulong, void* G,
                                                       float* gscale, Geom g, int p_out) {
    const uint32_t s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= g.Vh) return;
    int c[4];
    site_coords(g, s, p_out, c[0], c[1], c[2], c[3]);
    const int np = Ulong ? 8 : 4;
    const size_t Vh = g.Vh;
    double lr[18], li[18];
    float sc = 0.f;
    if constexpr (P == P16S) {
        // one fp32 scale per output site over all the reals it reads
#pragma unroll 1
        for (int pr = 0; pr < np; ++pr) {
            hop_pair(U, Ulong, g, c, pr, lr, li);
#pragma unroll
            for (int e = 0; e < 18; ++e)
                sc = fmaxf(sc, fmaxf(fabsf((float)lr[e]), fabsf((float)li[e])));
        }
        gscale[s] = sc;
    }
#pragma unroll 1
    for (int pr = 0; pr < np; ++pr) {
        hop_pair(U, Ulong, g, c, pr, lr, li);
        if constexpr (P == P64) {
            d2v* o = (d2v*)G + (size_t)(18 * pr) * Vh;
#pragma unroll
            for (int e = 0; e < 18; ++e) {
                d2v v;
                v.x = lr[e];
                v.y = li[e];
                o[(size_t)e * Vh + s] = v;
            }
        } else if constexpr (P == P32) {
            f4v* o = (f4v*)G + (size_t)(9 * pr) * Vh;
#pragma unroll
            for (int w = 0; w < 9; ++w) {
                f4v v;
                v.x = (float)lr[2 * w];
                v.y = (float)li[2 * w];
                v.z = (float)lr[2 * w + 1];
                v.w = (float)li[2 * w + 1];
                o[(size_t)w * Vh + s] = v;
            }
        } else {
            u2v* o = (u2v*)G + (size_t)(9 * pr) * Vh;
#pragma unroll
            for (int w = 0; w < 9; ++w) {
                u2v v;
                if (sc == 0.f) {
                    v.x = v.y = 0u;
                } else {
                    v.x = f2h_pair(__fdiv_rn((float)lr[2 * w], sc), __fdiv_rn((float)li[2 * w], sc));
                    v.y = f2h_pair(__fdiv_rn((float)lr[2 * w + 1], sc),
                                   __fdiv_rn((float)li[2 * w + 1], sc));
                }
                o[(size_t)w * Vh + s] = v;
            }
        }
    }
}

// 12-parameter packing: the first two rows of U_mu(x) and of
// U_mu(x - mu)^dagger per hop pair, without phases (layout in common.h).
// P16S divides by the site scale of the full packing (the largest |Re| or
// |Im| over all 144 reals of the site's eight links, third rows included).
template <int P>
__global__ __launch_bounds__(kBlock) void k_gauge_pack12(const d2v* __restrict__ U, void* G,
                                                         float* gscale, Geom g, int p_out) {
    const uint32_t s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= g.Vh) return;
    int c[4];
    site_coords(g, s, p_out, c[0], c[1], c[2], c[3]);
    const int Lx = g.L[0], Ly = g.L[1], Lz = g.L[2];
    auto lex_of = [&](const int* q) -> size_t {
        return (size_t)q[0] + (size_t)Lx * ((size_t)q[1] + (size_t)Ly * ((size_t)q[2] + (size_t)Lz * q[3]));
    };
    double lr[48], li[48];
    float sc = 0.f;
    const size_t lex = lex_of(c);
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        int b[4] = {c[0], c[1], c[2], c[3]};
        b[mu] = (b[mu] == 0) ? g.L[mu] - 1 : b[mu] - 1;
        const d2v* uf = U + (lex * 4 + mu) * 9;
        const d2v* ub = U + (lex_of(b) * 4 + mu) * 9;
        if constexpr (P == P16S) {
#pragma unroll
            for (int e = 0; e < 9; ++e) {
                const d2v f = uf[e], v = ub[e];
                sc = fmaxf(sc, fmaxf(fabsf((float)f.x), fabsf((float)f.y)));
                sc = fmaxf(sc, fmaxf(fabsf((float)v.x), fabsf((float)v.y)));
            }
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const d2v f = uf[i * 3 + k];
                lr[12 * mu + 3 * i + k] = f.x;
                li[12 * mu + 3 * i + k] = f.y;
                // U^dagger: entry (i, k) = conj(U[k][i])
                const d2v v = ub[k * 3 + i];
                lr[12 * mu + 6 + 3 * i + k] = v.x;
                li[12 * mu + 6 + 3 * i + k] = -v.y;
            }
    }
    const size_t Vh = g.Vh;
    if constexpr (P == P64) {
        d2v* o = (d2v*)G;
#pragma unroll
        for (int e = 0; e < 48; ++e) {
            d2v v;
            v.x = lr[e];
            v.y = li[e];
            o[(size_t)e * Vh + s] = v;
        }
    } else if constexpr (P == P32) {
        f4v* o = (f4v*)G;
#pragma unroll
        for (int w = 0; w < 24; ++w) {
            f4v v;
            v.x = (float)lr[2 * w];
            v.y = (float)li[2 * w];
            v.z = (float)lr[2 * w + 1];
            v.w = (float)li[2 * w + 1];
            o[(size_t)w * Vh + s] = v;
        }
    } else {
        gscale[s] = sc;
        u2v* o = (u2v*)G;
#pragma unroll
        for (int w = 0; w < 24; ++w) {
            u2v v;
            if (sc == 0.f) {
                v.x = v.y = 0u;
            } else {
                v.x = f2h_pair(__fdiv_rn((float)lr[2 * w], sc), __fdiv_rn((float)li[2 * w], sc));
                v.y = f2h_pair(__fdiv_rn((float)lr[2 * w + 1], sc), __fdiv_rn((float)li[2 * w + 1], sc));
            }
            o[(size_t)w * Vh + s] = v;
        }
    }
}

// Flag (bad = 1) every link with max |U U^+ - 1| or |det U - 1| above tol.
// All writers store the same value, so the race is benign.
__global__ __launch_bounds__(kBlock) void k_su3_check(const d2v* __restrict__ U, uint64_t nlinks,
                                                      double tol, int* bad) {
    const uint64_t l = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (l >= nlinks) return;
    double ur[9], ui[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) {
        const d2v v = U[l * 9 + e];
        ur[e] = v.x;
        ui[e] = v.y;
    }
    double err = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            // (U U^+)_ik = sum_j U_ij conj(U_kj)
            double re = 0.0, im = 0.0;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                re += ur[3 * i + j] * ur[3 * k + j] + ui[3 * i + j] * ui[3 * k + j];
                im += ui[3 * i + j] * ur[3 * k + j] - ur[3 * i + j] * ui[3 * k + j];
            }
            if (i == k) re -= 1.0;
            err = fmax(err, fmax(fabs(re), fabs(im)));
        }
    // det U = row0 . (row1 x row2)
    auto cm = [](double ar, double ai, double br, double bi, double& cr, double& ci) {
        cr = ar * br - ai * bi;
        ci = ar * bi + ai * br;
    };
    double dr = 0.0, di = 0.0;
    for (int k = 0; k < 3; ++k) {
        const int k1 = (k + 1) % 3, k2 = (k + 2) % 3;
        double pr, pi, qr, qi;
        cm(ur[3 + k1], ui[3 + k1], ur[6 + k2], ui[6 + k2], pr, pi);
        cm(ur[3 + k2], ui[3 + k2], ur[6 + k1], ui[6 + k1], qr, qi);
        double tr, ti;
        cm(ur[k], ui[k], pr - qr, pi - qi, tr, ti);
        dr += tr;
        di += ti;
    }
    err = fmax(err, fmax(fabs(dr - 1.0), fabs(di)));
    if (!(err <= tol)) *bad = 1;
}

hipError_t launch_su3_check(const void* U_dev, uint64_t nlinks, double tol, int* bad_dev,
                            hipStream_t st) {
    const uint64_t nb = (nlinks + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_su3_check, dim3((uint32_t)nb), dim3(kBlock), 0, st, (const d2v*)U_dev, nlinks,
                       tol, bad_dev);
    return hipGetLastError();
}

hipError_t launch_gauge_pack(int prec, const void* U_dev, const void* Ulong_dev, void* G,
                             float* gscale, const Geom& g, int p_out, bool r12, hipStream_t st) {
    if (r12 && Ulong_dev) return hipErrorInvalidValue;
    if (r12) {
        const dim3 grid((g.Vh + kBlock - 1) / kBlock), block(kBlock);
        const d2v* U = (const d2v*)U_dev;
        switch (prec) {
            case P64: hipLaunchKernelGGL((k_gauge_pack12<P64>), grid, block, 0, st, U, G, gscale, g, p_out); break;
            case P32: hipLaunchKernelGGL((k_gauge_pack12<P32>), grid, block, 0, st, U, G, gscale, g, p_out); break;
            case P16S: hipLaunchKernelGGL((k_gauge_pack12<P16S>), grid, block, 0, st, U, G, gscale, g, p_out); break;
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    const dim3 grid((g.Vh + kBlock - 1) / kBlock), block(kBlock);
    const d2v* U = (const d2v*)U_dev;
    const d2v* N = (const d2v*)Ulong_dev;
    switch (prec) {
        case P64: hipLaunchKernelGGL((k_gauge_pack<P64>), grid, block, 0, st, U, N, G, gscale, g, p_out); break;
        case P32: hipLaunchKernelGGL((k_gauge_pack<P32>), grid, block, 0, st, U, N, G, gscale, g, p_out); break;
        case P16S: hipLaunchKernelGGL((k_gauge_pack<P16S>), grid, block, 0, st, U, N, G, gscale, g, p_out); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Canonical spinors: complex128 [nrhs][Vh][3].
template <int P>
__global__ __launch_bounds__(kBlock) void k_import(const d2v* __restrict__ src, void* dst,
                                                   size_t dst_rs, uint32_t Vh) {
    using T = typename Real<P>::T;
    const uint32_t s = blockIdx.x * kBlock + threadIdx.x;
    const int r = blockIdx.y;
    if (s >= Vh) return;
    const d2v* p = src + ((size_t)r * Vh + s) * 3;
    T re[3], im[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const d2v v = p[c];
        re[c] = (T)v.x;
        im[c] = (T)v.y;
    }
    store_site<P>((char*)dst + (size_t)r * dst_rs, Vh, s, re, im);
}

template <int P>
__global__ __launch_bounds__(kBlock) void k_export(const void* src, size_t src_rs, d2v* dst,
                                                   uint32_t Vh) {
    using T = typename Real<P>::T;
    const uint32_t s = blockIdx.x * kBlock + threadIdx.x;
    const int r = blockIdx.y;
    if (s >= Vh) return;
    T re[3], im[3];
    load_site<P>((const char*)src + (size_t)r * src_rs, Vh, s, re, im);
    d2v* p = dst + ((size_t)r * Vh + s) * 3;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        d2v v;
        v.x = (double)re[c];
        v.y = (double)im[c];
        p[c] = v;
    }
}

hipError_t launch_import(int prec, const void* src_dev, void* dst, size_t dst_rs, uint32_t Vh,
                         int nrhs, hipStream_t st) {
    const dim3 grid((Vh + kBlock - 1) / kBlock, nrhs), block(kBlock);
    const d2v* src = (const d2v*)src_dev;
    switch (prec) {
        case P64: hipLaunchKernelGGL((k_import<P64>), grid, block, 0, st, src, dst, dst_rs, Vh); break;
        case P32: hipLaunchKernelGGL((k_import<P32>), grid, block, 0, st, src, dst, dst_rs, Vh); break;
        case P16S: hipLaunchKernelGGL((k_import<P16S>), grid, block, 0, st, src, dst, dst_rs, Vh); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_export(int prec, const void* src, size_t src_rs, void* dst_dev, uint32_t Vh,
                         int nrhs, hipStream_t st) {
    const dim3 grid((Vh + kBlock - 1) / kBlock, nrhs), block(kBlock);
    d2v* dst = (d2v*)dst_dev;
    switch (prec) {
        case P64: hipLaunchKernelGGL((k_export<P64>), grid, block, 0, st, src, src_rs, dst, Vh); break;
        case P32: hipLaunchKernelGGL((k_export<P32>), grid, block, 0, st, src, src_rs, dst, Vh); break;
        case P16S: hipLaunchKernelGGL((k_export<P16S>), grid, block, 0, st, src, src_rs, dst, Vh); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace stag
