// Wilson hopping matrix between checkerboards on gfx950, with the fused
// epilogues of the even-odd twisted-mass operator.
//
// One lane owns one output site.  For each of the 8 directions it gathers the
// neighbour's full spinor (12 coalesced complex words of the
// structure-of-arrays layout), projects it onto the two-spin half-spinor
// h = psi_up -/+ e_mu psi_dn that (1 -/+ gamma_mu) leaves independent,
// multiplies h by U or U^dagger (the only dense part: two 3x3 complex
// mat-vecs), and rebuilds the lower two spins from h with a sign, a factor i
// and a spin swap.  Neighbour indices and the boundary phase are computed from
// the site's coordinates, so no index table is read.
//
// Epilogues (all with kappa folded into the coefficients):
//   MODE 0  out_s = c_{s/2} acc_s                      plain H, or A^-1 H
//   MODE 1  out_s = c_{s/2} acc_s + d_{s/2} aux_s       gamma_5 [A aux - H (.)]
//   MODE 2  as MODE 1, plus the per-workgroup partial of |out|^2 (FP64)
#include "common.h"
#include "kernels.h"

namespace tmh {

// e_mu applied to the lower spin pair (p2, p3) of the chiral basis:
// e_0 = -1, e_1 = -i sigma_1, e_2 = -i sigma_2, e_3 = -i sigma_3.
template <typename R, int MU>
__device__ __forceinline__ void e_lower(cx<R> p2, cx<R> p3, cx<R>& r0, cx<R>& r1) {
    if constexpr (MU == 0) {
        r0 = mk<R>(-p2.re, -p2.im);
        r1 = mk<R>(-p3.re, -p3.im);
    } else if constexpr (MU == 1) {
        r0 = mk<R>(p3.im, -p3.re);  // -i p3
        r1 = mk<R>(p2.im, -p2.re);  // -i p2
    } else if constexpr (MU == 2) {
        r0 = mk<R>(-p3.re, -p3.im);
        r1 = p2;
    } else {
        r0 = mk<R>(p2.im, -p2.re);  // -i p2
        r1 = mul_i(p3);             //  i p3
    }
}

// e_mu^dagger applied to (g0, g1).
template <typename R, int MU>
__device__ __forceinline__ void edag(cx<R> g0, cx<R> g1, cx<R>& r0, cx<R>& r1) {
    if constexpr (MU == 0) {
        r0 = mk<R>(-g0.re, -g0.im);
        r1 = mk<R>(-g1.re, -g1.im);
    } else if constexpr (MU == 1) {
        r0 = mul_i(g1);
        r1 = mul_i(g0);
    } else if constexpr (MU == 2) {
        r0 = g1;
        r1 = mk<R>(-g0.re, -g0.im);
    } else {
        r0 = mul_i(g0);
        r1 = mk<R>(g1.im, -g1.re);  // -i g1
    }
}

// One of the 8 terms: DIR = +1 adds (1 - gamma_mu) U_mu(x) psi(x+mu),
// DIR = -1 adds (1 + gamma_mu) U_mu(x-mu)^dagger psi(x-mu).
// jn: even-odd index of the neighbour; link: base of the 9 link words of
// direction MU, taken at index jl.
template <typename R, int MU, int DIR>
__device__ __forceinline__ void hop_term(cx<R> (&acc)[4][3], const typename Word<R>::T* __restrict__ in,
                                         const typename Word<R>::T* __restrict__ link, int S, int jn,
                                         int jl, bool wrap, cx<R> ph) {
    cx<R> psi[4][3];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int a = 0; a < 3; ++a) psi[s][a] = ld<R>(in, (int64_t)(3 * s + a) * S + jn);
    cx<R> u[3][3];
#pragma unroll
    for (int k = 0; k < 9; ++k) u[k / 3][k % 3] = ld<R>(link, (int64_t)k * S + jl);

    // half-spinor h = psi_up - DIR e_mu psi_dn
    cx<R> h[2][3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        cx<R> e0, e1;
        e_lower<R, MU>(psi[2][a], psi[3][a], e0, e1);
        if constexpr (DIR > 0) {
            h[0][a] = psi[0][a] - e0;
            h[1][a] = psi[1][a] - e1;
        } else {
            h[0][a] = psi[0][a] + e0;
            h[1][a] = psi[1][a] + e1;
        }
    }
    if (wrap) {
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int a = 0; a < 3; ++a) h[s][a] = h[s][a] * ph;
    }
    // g = U h (forward) or U^dagger h (backward)
    cx<R> g[2][3];
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            if constexpr (DIR > 0)
                g[s][a] = u[a][0] * h[s][0] + u[a][1] * h[s][1] + u[a][2] * h[s][2];
            else
                g[s][a] = cmul(u[0][a], h[s][0]) + cmul(u[1][a], h[s][1]) + cmul(u[2][a], h[s][2]);
        }
    // upper spins take g, lower spins take -DIR e_mu^dagger g
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        acc[0][a] += g[0][a];
        acc[1][a] += g[1][a];
        cx<R> f0, f1;
        edag<R, MU>(g[0][a], g[1][a], f0, f1);
        if constexpr (DIR > 0) {
            acc[2][a] -= f0;
            acc[3][a] -= f1;
        } else {
            acc[2][a] += f0;
            acc[3][a] += f1;
        }
    }
}

template <typename R, int MU>
__device__ __forceinline__ void hop_mu(cx<R> (&acc)[4][3], const HopArgs<R>& a, const int c[4], int lex,
                                       int i) {
    const int stride = MU == 3 ? 1 : (MU == 2 ? a.g.L[3] : (MU == 1 ? a.g.L[2] * a.g.L[3]
                                                                     : a.g.L[1] * a.g.L[2] * a.g.L[3]));
    const int Lm = a.g.L[MU];
    const cx<R> ph = mk<R>(a.ph_re[MU], a.ph_im[MU]);
    // forward: x + mu, link U_mu(x) on the output parity at index i
    {
        const bool wrap = c[MU] == Lm - 1;
        const int nb = wrap ? lex - (Lm - 1) * stride : lex + stride;
        hop_term<R, MU, +1>(acc, a.in, a.gout + (int64_t)MU * 9 * a.g.S, a.g.S, nb >> 1, i, wrap, ph);
    }
    // backward: x - mu, link U_mu(x - mu) on the input parity at the neighbour
    {
        const bool wrap = c[MU] == 0;
        const int nb = wrap ? lex + (Lm - 1) * stride : lex - stride;
        const int j = nb >> 1;
        hop_term<R, MU, -1>(acc, a.in, a.gin + (int64_t)MU * 9 * a.g.S, a.g.S, j, j, wrap,
                            mk<R>(ph.re, -ph.im));
    }
}

template <typename R, int MODE>
__global__ void __launch_bounds__(kBlock) hop_kernel(HopArgs<R> a) {
    if (a.done && *a.done) return;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int i = blk * kBlock + threadIdx.x;
    double nrm = 0.0;
    if (i < a.g.Vh) {
        int c[4], lex;
        site_coords(a.g, i, a.pout, c, lex);
        cx<R> acc[4][3];
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int k = 0; k < 3; ++k) acc[s][k] = mk<R>(0, 0);
        hop_mu<R, 0>(acc, a, c, lex, i);
        hop_mu<R, 1>(acc, a, c, lex, i);
        hop_mu<R, 2>(acc, a, c, lex, i);
        hop_mu<R, 3>(acc, a, c, lex, i);
        const int S = a.g.S;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const cx<R> cc = mk<R>(a.c_re[s >> 1], a.c_im[s >> 1]);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const int64_t off = (int64_t)(3 * s + k) * S + i;
                cx<R> o = cc * acc[s][k];
                if constexpr (MODE >= 1) o += mk<R>(a.d_re[s >> 1], a.d_im[s >> 1]) * ld<R>(a.aux, off);
                if constexpr (MODE == 2) nrm += (double)o.re * (double)o.re + (double)o.im * (double)o.im;
                st<R>(a.out, off, o);
            }
        }
    }
    if constexpr (MODE == 2) {
        const double s = block_sum(nrm);
        if (threadIdx.x == 0) a.partial[blockIdx.x] = s;
    }
}

int hop_blocks(const Geo& g) { return (g.Vh + kBlock - 1) / kBlock; }

template <typename R>
hipError_t launch_hop(const HopArgs<R>& a, int mode, hipStream_t stream) {
    const int nb = hop_blocks(a.g);
    if (nb == 0) return hipSuccess;
    switch (mode) {
        case 0: hipLaunchKernelGGL((hop_kernel<R, 0>), dim3(nb), dim3(kBlock), 0, stream, a); break;
        case 1: hipLaunchKernelGGL((hop_kernel<R, 1>), dim3(nb), dim3(kBlock), 0, stream, a); break;
        default: hipLaunchKernelGGL((hop_kernel<R, 2>), dim3(nb), dim3(kBlock), 0, stream, a); break;
    }
    return hipGetLastError();
}

template hipError_t launch_hop<double>(const HopArgs<double>&, int, hipStream_t);
template hipError_t launch_hop<float>(const HopArgs<float>&, int, hipStream_t);

}  // namespace tmh
