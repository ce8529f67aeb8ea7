// Vector kernels of the CG iteration (Fig.1 and Sec.3.2): the start of a
// solve and the fused axpy + norm updates with fp64 reductions. One thread
// per site handles every active right-hand side of the block; the CG
// scalars come from the device-resident per-RHS state, optionally finalised
// at kernel start from the partials of the reduction that precedes the
// kernel. Also the reduction finalisation kernel and the issue helper that
// launches a kernel or appends it to a graph.
#include <hip/hip_ext.h>

#include <type_traits>

#include "kern.h"
#include "launch.h"

namespace stag {

__device__ __forceinline__ char* slot(const VecArgs& a, int k, int r) {
    return (char*)a.f[k] + (size_t)r * a.rs[k];
}

// Own-site operands of a fused update: x (fp64 CG) or y (fp32, mixed CG),
// then r (or rs), d and Ad in the iteration's precision.
template <int P, int OP>
struct UpdOps {
    using T = typename Real<P>::T;
    using A = typename std::conditional<OP == OP_UPD_CG, double, float>::type;
    A ar[3], ai[3];
    T sr[3], si[3], dr[3], di[3], qr[3], qi[3];
};

template <int P, int OP>
__device__ __forceinline__ void load_upd(const VecArgs& a, int r, uint32_t s, UpdOps<P, OP>& u) {
    if constexpr (OP == OP_UPD_CG) {
        load_site<P64>(slot(a, 0, r), a.Vh, s, u.ar, u.ai);
    } else {
        load_site<P32>(slot(a, 0, r), a.Vh, s, u.ar, u.ai);
    }
    load_site<P>(slot(a, 1, r), a.Vh, s, u.sr, u.si);
    load_site<P>(slot(a, 2, r), a.Vh, s, u.dr, u.di);
    load_site<P>(slot(a, 3, r), a.Vh, s, u.qr, u.qi);
}

template <int P, int N, int OP>
__global__ __launch_bounds__(kBlock) void k_vec(VecArgs a) {
    using T = typename Real<P>::T;
    const uint32_t blk = logical_block(a.swizzle);
    const uint32_t s = blk * kBlock + threadIdx.x;
    const uint32_t Vh = a.Vh;
    const bool valid = s < Vh;
    // Per-RHS state, finalised here from the previous reduction's partials
    // when a.fin is set. One RHS: each wavefront keeps it in registers (no
    // barrier) and an update requests its operands and the partials before
    // the state is known (an inactive slot discards them). Several RHS: the
    // block shares one copy in LDS.
    constexpr bool UPD = OP == OP_UPD_CG || OP == OP_UPD_MIXED;
    __shared__ RhsState ls[N];
    RhsState s1{};
    unsigned act = (1u << N) - 1u;
    [[maybe_unused]] UpdOps<P, OP> u0;
    if constexpr (N == 1) {
        s1 = *(a.st ? a.st : &kNoState);
        if (a.st && !(s1.flags & a.run_mask)) act = 0;
        if constexpr (UPD) {
            if (valid) load_upd<P, OP>(a, 0, s, u0);
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
    double dv[N];
#pragma unroll
    for (int r = 0; r < N; ++r) dv[r] = 0.0;

    if (valid) {
#pragma unroll
        for (int r = 0; r < N; ++r) {
            if (!((act >> r) & 1u)) continue;
            if constexpr (OP == OP_INIT_B) {
                // r64 = b, x64 = 0 (kept when the slot starts from x0), |b|^2
                double br[3], bi[3], z[3] = {0.0, 0.0, 0.0}, zi[3] = {0.0, 0.0, 0.0};
                load_site<P64>(slot(a, 0, r), Vh, s, br, bi);
                store_site<P64>(slot(a, 1, r), Vh, s, br, bi);
                if (!a.st || !(stv(r).flags & F_X0)) store_site<P64>(slot(a, 2, r), Vh, s, z, zi);
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
                const double al = stv(r).alpha;
                UpdOps<P, OP> u;
                if constexpr (N == 1) {
                    u = u0;
                } else {
                    load_upd<P, OP>(a, r, s, u);
                }
                double acc = 0.0;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    u.ar[c] = fma(al, u.dr[c], u.ar[c]);
                    u.ai[c] = fma(al, u.di[c], u.ai[c]);
                    u.sr[c] = fma(-al, u.qr[c], u.sr[c]);
                    u.si[c] = fma(-al, u.qi[c], u.si[c]);
                    acc += u.sr[c] * u.sr[c] + u.si[c] * u.si[c];
                }
                store_site<P64>(slot(a, 0, r), Vh, s, u.ar, u.ai);
                store_site<P64>(slot(a, 1, r), Vh, s, u.sr, u.si);
                dv[r] = acc;
            } else if constexpr (OP == OP_UPD_MIXED) {
                // y += alpha d (fp32); rs = q(rs - alpha Ad); |rs|^2 of the stored rs
                const float al = (float)stv(r).alpha;
                UpdOps<P, OP> u;
                if constexpr (N == 1) {
                    u = u0;
                } else {
                    load_upd<P, OP>(a, r, s, u);
                }
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    u.ar[c] = fmaf(al, u.dr[c], u.ar[c]);
                    u.ai[c] = fmaf(al, u.di[c], u.ai[c]);
                    u.sr[c] = fmaf(-al, u.qr[c], u.sr[c]);
                    u.si[c] = fmaf(-al, u.qi[c], u.si[c]);
                }
                store_site<P32>(slot(a, 0, r), Vh, s, u.ar, u.ai);
                store_site<P>(slot(a, 1, r), Vh, s, u.sr, u.si);
                double acc = 0.0;
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    acc += (double)u.sr[c] * (double)u.sr[c] + (double)u.si[c] * (double)u.si[c];
                dv[r] = acc;
            } else if constexpr (OP == OP_XPAY) {
                // d = q(r + beta d): the arithmetic of the hop stages' deferred form
                T rr[3], ri[3], dr[3], di[3];
                load_site<P>(slot(a, 0, r), Vh, s, rr, ri);
                load_site<P>(slot(a, 1, r), Vh, s, dr, di);
                const T be = (T)stv(r).beta;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    dr[c] = fma(be, dr[c], rr[c]);
                    di[c] = fma(be, di[c], ri[c]);
                }
                round_site<P>(dr, di);
                store_site<P>(slot(a, 1, r), Vh, s, dr, di);
            } else if constexpr (OP == OP_FOLD) {
                // x64 += y, y = 0
                double xr[3], xi[3];
                float yr[3], yi[3], z[3] = {0.f, 0.f, 0.f}, zi[3] = {0.f, 0.f, 0.f};
                load_site<P64>(slot(a, 0, r), Vh, s, xr, xi);
                load_site<P32>(slot(a, 1, r), Vh, s, yr, yi);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    xr[c] = xr[c] + (double)yr[c];
                    xi[c] = xi[c] + (double)yi[c];
                }
                store_site<P64>(slot(a, 0, r), Vh, s, xr, xi);
                store_site<P32>(slot(a, 1, r), Vh, s, z, zi);
            }
        }
    }
    if constexpr (OP == OP_INIT_B || OP == OP_UPD_CG || OP == OP_UPD_MIXED) {
        block_partials<N>(dv, a.red, blk);
    }
}

template <int P, int N, int OP>
static hipError_t issue_vec(const VecArgs& a, const Issue& is) {
    VecArgs arg = a;
    void* args[] = {&arg};
    return issue_kernel(is, reinterpret_cast<const void*>(&k_vec<P, N, OP>), vec_blocks(a.Vh), kBlock,
                        args);
}

template <int P, int N>
static hipError_t run_vec_n(int op, const VecArgs& a, const Issue& is) {
    switch (op) {
        case OP_START: return issue_vec<P, N, OP_START>(a, is);
        case OP_XPAY: return issue_vec<P, N, OP_XPAY>(a, is);
        default: break;
    }
    if constexpr (P == P64) {
        switch (op) {
            case OP_INIT_B: return issue_vec<P, N, OP_INIT_B>(a, is);
            case OP_UPD_CG: return issue_vec<P, N, OP_UPD_CG>(a, is);
            default: break;
        }
    } else {
        if (op == OP_UPD_MIXED) return issue_vec<P, N, OP_UPD_MIXED>(a, is);
        if (op == OP_FOLD) return issue_vec<P, N, OP_FOLD>(a, is);
    }
    return hipErrorInvalidValue;
}

template <int P>
static hipError_t run_vec(int N, int op, const VecArgs& a, const Issue& is) {
    switch (N) {
        case 1: return run_vec_n<P, 1>(op, a, is);
        case 2: return run_vec_n<P, 2>(op, a, is);
        case 4: return run_vec_n<P, 4>(op, a, is);
        case 8: return run_vec_n<P, 8>(op, a, is);
        case 12: return run_vec_n<P, 12>(op, a, is);
        case 16: return run_vec_n<P, 16>(op, a, is);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_vec(int prec, int N, int op, const VecArgs& a, const Issue& is) {
    switch (prec) {
        case P64: return run_vec<P64>(N, op, a, is);
        case P32: return run_vec<P32>(N, op, a, is);
        case P16S: return run_vec<P16S>(N, op, a, is);
        default: return hipErrorInvalidValue;
    }
}

// ------------------------------------------------------------------ reduction finalisation

template <int N>
__global__ __launch_bounds__(64 * N) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_finalize(Reduce R, unsigned run_mask) {
    __shared__ RhsState ls[N];
    finalize_wide<N>(R, run_mask, ls);
}

template <int N>
static hipError_t issue_finalize(const Reduce& R, unsigned run_mask, const Issue& is) {
    Reduce r = R;
    unsigned m = run_mask;
    void* args[] = {&r, &m};
    return issue_kernel(is, reinterpret_cast<const void*>(&k_finalize<N>), 1, 64 * N, args);
}

hipError_t launch_finalize(int N, const Reduce& R, unsigned run_mask, const Issue& is) {
    switch (N) {
        case 1: return issue_finalize<1>(R, run_mask, is);
        case 2: return issue_finalize<2>(R, run_mask, is);
        case 4: return issue_finalize<4>(R, run_mask, is);
        case 8: return issue_finalize<8>(R, run_mask, is);
        case 12: return issue_finalize<12>(R, run_mask, is);
        case 16: return issue_finalize<16>(R, run_mask, is);
        default: return hipErrorInvalidValue;
    }
}

// ------------------------------------------------------------------ issue

hipError_t issue_kernel(const Issue& is, const void* func, uint32_t grid, uint32_t block,
                        void** args) {
    if (is.gb) {
        hipKernelNodeParams p{};
        p.func = const_cast<void*>(func);
        p.gridDim = dim3(grid);
        p.blockDim = dim3(block);
        p.sharedMemBytes = 0;
        p.kernelParams = args;  // copied into the node
        p.extra = nullptr;
        hipGraphNode_t node = nullptr;
        const hipGraphNode_t dep = is.gb->last;
        hipError_t err = hipGraphAddKernelNode(&node, is.gb->graph, dep ? &dep : nullptr, dep ? 1 : 0, &p);
        if (err == hipSuccess) is.gb->last = node;
        return err;
    }
    if (is.ev_start || is.ev_stop)
        return hipExtLaunchKernel(func, dim3(grid), dim3(block), args, 0, is.stream, is.ev_start,
                                  is.ev_stop, 0);
    return hipLaunchKernel(func, dim3(grid), dim3(block), args, 0, is.stream);
}

// ------------------------------------------------------------------ hop dispatch

hipError_t launch_hop_p0_n4(int S, int N, int epi, bool nt, const HopArgs& a, const Issue& is);
hipError_t launch_hop_p1_n4(int S, int N, int epi, bool nt, const HopArgs& a, const Issue& is);
hipError_t launch_hop_p2_n4(int S, int N, int epi, bool nt, const HopArgs& a, const Issue& is);
hipError_t launch_hop_p0_n8(int S, int N, int epi, bool nt, const HopArgs& a, const Issue& is);
hipError_t launch_hop_p1_n8(int S, int N, int epi, bool nt, const HopArgs& a, const Issue& is);
hipError_t launch_hop_p2_n8(int S, int N, int epi, bool nt, const HopArgs& a, const Issue& is);

hipError_t launch_hop(int prec, int S, int N, int epi, bool nt, const HopArgs& a, const Issue& is) {
    if (a.npairs == 8) {
        if (a.r12) return hipErrorInvalidValue;  // long and fat links are stored in full
        switch (prec) {
            case P64: return launch_hop_p0_n8(S, N, epi, nt, a, is);
            case P32: return launch_hop_p1_n8(S, N, epi, nt, a, is);
            case P16S: return launch_hop_p2_n8(S, N, epi, nt, a, is);
            default: return hipErrorInvalidValue;
        }
    }
    if (a.npairs != 4) return hipErrorInvalidValue;
    switch (prec) {
        case P64: return launch_hop_p0_n4(S, N, epi, nt, a, is);
        case P32: return launch_hop_p1_n4(S, N, epi, nt, a, is);
        case P16S: return launch_hop_p2_n4(S, N, epi, nt, a, is);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace stag
