// Vector kernels of the CG iteration (Fig.1 and Sec.3.2): fused axpy + norm
// updates with fp64 reductions, the direction update, and the pieces of the
// reliable / group-wise update. One thread per site handles every active
// right-hand side of the block; the CG scalars come from the device-resident
// per-RHS state, optionally finalised at kernel start from the partials of
// the reduction that precedes the kernel.
#include <hip/hip_ext.h>

#include "kern.h"
#include "launch.h"

namespace stag {

__device__ __forceinline__ char* slot(const VecArgs& a, int k, int r) {
    return (char*)a.f[k] + (size_t)r * a.rs[k];
}

template <int P, int N, int OP>
__global__ __launch_bounds__(kBlock) void k_vec(VecArgs a) {
    using T = typename Real<P>::T;
    const uint32_t blk = logical_block(a.swizzle);
    const uint32_t s = blk * kBlock + threadIdx.x;
    const uint32_t Vh = a.Vh;
    const bool valid = s < Vh;
    // the state of every RHS, in LDS: finalised here from the previous
    // reduction's partials when a.fin is set, else copied as it is
    __shared__ RhsState ls[N];
    unsigned act = (1u << N) - 1u;
    if (a.st) {
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
    double dv[N];
#pragma unroll
    for (int r = 0; r < N; ++r) dv[r] = 0.0;

    if (valid) {
#pragma unroll
        for (int r = 0; r < N; ++r) {
            if (!((act >> r) & 1u)) continue;
            if constexpr (OP == OP_INIT_B) {
                // r64 = b, x64 = 0, |b|^2
                double br[3], bi[3], z[3] = {0.0, 0.0, 0.0}, zi[3] = {0.0, 0.0, 0.0};
                load_site<P64>(slot(a, 0, r), Vh, s, br, bi);
                store_site<P64>(slot(a, 1, r), Vh, s, br, bi);
                store_site<P64>(slot(a, 2, r), Vh, s, z, zi);
                double acc = 0.0;
#pragma unroll
                for (int c = 0; c < 3; ++c) acc += br[c] * br[c] + bi[c] * bi[c];
                dv[r] = acc;
            } else if constexpr (OP == OP_START) {
                // d = q(r64); rs = q(r64); y = 0
                double vr[3], vi[3];
                load_site<P64>(slot(a, 0, r), Vh, s, vr, vi);
                T qr[3], qi[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    qr[c] = (T)vr[c];
                    qi[c] = (T)vi[c];
                }
                store_site<P>(slot(a, 1, r), Vh, s, qr, qi);
                if (a.f[2]) store_site<P>(slot(a, 2, r), Vh, s, qr, qi);
                if (a.f[3]) {
                    float z[3] = {0.f, 0.f, 0.f}, zi[3] = {0.f, 0.f, 0.f};
                    store_site<P32>(slot(a, 3, r), Vh, s, z, zi);
                }
            } else if constexpr (OP == OP_UPD_CG) {
                // x += alpha d; r -= alpha Ad; |r|^2   (all fp64)
                const double al = ls[r].alpha;
                double xr[3], xi[3], rr[3], ri[3], dr[3], di[3], qr[3], qi[3];
                load_site<P64>(slot(a, 0, r), Vh, s, xr, xi);
                load_site<P64>(slot(a, 1, r), Vh, s, rr, ri);
                load_site<P64>(slot(a, 2, r), Vh, s, dr, di);
                load_site<P64>(slot(a, 3, r), Vh, s, qr, qi);
                double acc = 0.0;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    xr[c] = fma(al, dr[c], xr[c]);
                    xi[c] = fma(al, di[c], xi[c]);
                    rr[c] = fma(-al, qr[c], rr[c]);
                    ri[c] = fma(-al, qi[c], ri[c]);
                    acc += rr[c] * rr[c] + ri[c] * ri[c];
                }
                store_site<P64>(slot(a, 0, r), Vh, s, xr, xi);
                store_site<P64>(slot(a, 1, r), Vh, s, rr, ri);
                dv[r] = acc;
            } else if constexpr (OP == OP_UPD_MIXED) {
                // y += alpha d (fp32); rs = q(rs - alpha Ad); |rs|^2 of the stored rs
                const float al = (float)ls[r].alpha;
                float yr[3], yi[3];
                T sr[3], si[3], dr[3], di[3], qr[3], qi[3];
                load_site<P32>(slot(a, 0, r), Vh, s, yr, yi);
                load_site<P>(slot(a, 1, r), Vh, s, sr, si);
                load_site<P>(slot(a, 2, r), Vh, s, dr, di);
                load_site<P>(slot(a, 3, r), Vh, s, qr, qi);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    yr[c] = fmaf(al, dr[c], yr[c]);
                    yi[c] = fmaf(al, di[c], yi[c]);
                    sr[c] = fmaf(-al, qr[c], sr[c]);
                    si[c] = fmaf(-al, qi[c], si[c]);
                }
                store_site<P32>(slot(a, 0, r), Vh, s, yr, yi);
                store_site<P>(slot(a, 1, r), Vh, s, sr, si);
                double acc = 0.0;
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    acc += (double)sr[c] * (double)sr[c] + (double)si[c] * (double)si[c];
                dv[r] = acc;
            } else if constexpr (OP == OP_RU_BEGIN) {
                // x64 += y; y = 0
                double xr[3], xi[3];
                float yr[3], yi[3], z[3] = {0.f, 0.f, 0.f}, zi[3] = {0.f, 0.f, 0.f};
                load_site<P64>(slot(a, 0, r), Vh, s, xr, xi);
                load_site<P32>(slot(a, 1, r), Vh, s, yr, yi);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    xr[c] += (double)yr[c];
                    xi[c] += (double)yi[c];
                }
                store_site<P64>(slot(a, 0, r), Vh, s, xr, xi);
                store_site<P32>(slot(a, 1, r), Vh, s, z, zi);
            } else if constexpr (OP == OP_RU_END) {
                // rs = q(r64): the low-precision residual restarts from the true one
                double vr[3], vi[3];
                load_site<P64>(slot(a, 0, r), Vh, s, vr, vi);
                T sr[3], si[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    sr[c] = (T)vr[c];
                    si[c] = (T)vi[c];
                }
                store_site<P>(slot(a, 1, r), Vh, s, sr, si);
            } else if constexpr (OP == OP_ZERO) {
                T z[3] = {T(0), T(0), T(0)}, zi[3] = {T(0), T(0), T(0)};
                store_site<P>(slot(a, 0, r), Vh, s, z, zi);
            }
        }
    }
    if constexpr (OP == OP_INIT_B || OP == OP_UPD_CG || OP == OP_UPD_MIXED) {
        block_chunk_partials<N, 1>(dv, a.red, blk);
    }
}

template <int P, int N>
static hipError_t run_vec_n(int op, const VecArgs& a, hipStream_t st, const LaunchEvents* ev) {
    const dim3 grid(vec_blocks(a.Vh)), block(kBlock);
#define STAG_VEC_CASE(OPV)                                                                 \
    case OPV:                                                                              \
        if (ev)                                                                            \
            hipExtLaunchKernelGGL((k_vec<P, N, OPV>), grid, block, 0, st, ev->start,        \
                                  ev->stop, 0, a);                                          \
        else                                                                               \
            hipLaunchKernelGGL((k_vec<P, N, OPV>), grid, block, 0, st, a);                 \
        return hipGetLastError();
    switch (op) {
        STAG_VEC_CASE(OP_START)
        STAG_VEC_CASE(OP_ZERO)
        default:
            break;
    }
    if constexpr (P == P64) {
        switch (op) {
            STAG_VEC_CASE(OP_INIT_B)
            STAG_VEC_CASE(OP_UPD_CG)
            default:
                break;
        }
    } else {
        switch (op) {
            STAG_VEC_CASE(OP_UPD_MIXED)
            STAG_VEC_CASE(OP_RU_BEGIN)
            STAG_VEC_CASE(OP_RU_END)
            default:
                break;
        }
    }
#undef STAG_VEC_CASE
    return hipErrorInvalidValue;
}

template <int P>
static hipError_t run_vec(int N, int op, const VecArgs& a, hipStream_t st, const LaunchEvents* ev) {
    switch (N) {
        case 1: return run_vec_n<P, 1>(op, a, st, ev);
        case 2: return run_vec_n<P, 2>(op, a, st, ev);
        case 4: return run_vec_n<P, 4>(op, a, st, ev);
        case 8: return run_vec_n<P, 8>(op, a, st, ev);
        case 12: return run_vec_n<P, 12>(op, a, st, ev);
        case 16: return run_vec_n<P, 16>(op, a, st, ev);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_vec(int prec, int N, int op, const VecArgs& a, hipStream_t st,
                      const LaunchEvents* ev) {
    switch (prec) {
        case P64: return run_vec<P64>(N, op, a, st, ev);
        case P32: return run_vec<P32>(N, op, a, st, ev);
        case P16S: return run_vec<P16S>(N, op, a, st, ev);
        default: return hipErrorInvalidValue;
    }
}

// ------------------------------------------------------------------ reduction finalisation

template <int N>
__global__ __launch_bounds__(kBlock) void k_finalize(Reduce R, unsigned run_mask) {
    __shared__ RhsState ls[N];
    finalize_block<N>(R, run_mask, ls);
}

hipError_t launch_finalize(int N, const Reduce& R, unsigned run_mask, hipStream_t stream) {
    switch (N) {
#define STAG_FIN_CASE(n) \
    case n: hipLaunchKernelGGL((k_finalize<n>), dim3(1), dim3(kBlock), 0, stream, R, run_mask); break;
        STAG_FIN_CASE(1)
        STAG_FIN_CASE(2)
        STAG_FIN_CASE(4)
        STAG_FIN_CASE(8)
        STAG_FIN_CASE(12)
        STAG_FIN_CASE(16)
#undef STAG_FIN_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------ state transitions

template <int N>
__global__ void k_state(RhsState* st, unsigned run_mask, int kind) {
    const int r = threadIdx.x;
    if (r < N && (st[r].flags & run_mask)) finalize_one(kind, st + r, 0.0, nullptr);
}

hipError_t launch_state(int N, int kind, RhsState* st, unsigned run_mask, hipStream_t stream) {
    switch (N) {
#define STAG_STATE_CASE(n) \
    case n: hipLaunchKernelGGL((k_state<n>), dim3(1), dim3(64), 0, stream, st, run_mask, kind); break;
        STAG_STATE_CASE(1)
        STAG_STATE_CASE(2)
        STAG_STATE_CASE(4)
        STAG_STATE_CASE(8)
        STAG_STATE_CASE(12)
        STAG_STATE_CASE(16)
#undef STAG_STATE_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------ hop dispatch

hipError_t launch_hop_p0(int S, int N, int epi, bool nt, const HopArgs& a, hipStream_t st,
                         const LaunchEvents* ev);
hipError_t launch_hop_p1(int S, int N, int epi, bool nt, const HopArgs& a, hipStream_t st,
                         const LaunchEvents* ev);
hipError_t launch_hop_p2(int S, int N, int epi, bool nt, const HopArgs& a, hipStream_t st,
                         const LaunchEvents* ev);

hipError_t launch_hop(int prec, int S, int N, int epi, bool nt, const HopArgs& a,
                      hipStream_t st, const LaunchEvents* ev) {
    switch (prec) {
        case P64: return launch_hop_p0(S, N, epi, nt, a, st, ev);
        case P32: return launch_hop_p1(S, N, epi, nt, a, st, ev);
        case P16S: return launch_hop_p2(S, N, epi, nt, a, st, ev);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace stag
