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
//   MODE 3  CG residual update fused into the last hop of an iteration:
//           with q = MODE 1 result (kept in registers), r -= alpha q and the
//           per-workgroup partial of |r|^2; q is not stored (x is updated
//           with the search direction at the end of the iteration)
//   MODE 4  as MODE 3, plus x += alpha p
#include "common.h"
#include "kernels.h"

#include "hop_body.h"

namespace tmh {

// Traversal order.  Blocks are dealt round-robin to the 8 XCDs; the kernel
// gives each XCD one contiguous range of the lattice instead (whole
// time-slices when T is a multiple of 8), so that neighbouring sites share
// that XCD's L2.  With xgroup > 0 the XCD's range is further visited in
// 64-site units (one wave each) x-group by x-group: all the XCD's
// time-slices for xgroup consecutive x values, then the next group.  The
// sites resident at one time, and their neighbours, then form a more compact
// region than in slice-by-slice order.  With xgroup = kXSlab the XCDs split
// x instead: XCD k owns x in [k LX/8, (k+1) LX/8) over all time-slices and
// sweeps t, so that all XCDs reach their shared x boundaries at the same
// time.  nyb units fill one (t, x) plane.  Returns the first site of the
// unit handled by wave w of hardware block b.
__device__ __forceinline__ int unit_site(int b, int w, int nb, int xgroup, int nyb, int nt, int LX) {
#if TMH_XCD_REMAP
    const int q = nb / kXcds, r = nb % kXcds;
    const int xc = b % kXcds, k = b / kXcds;
    if (xgroup == kXSlab) {
        constexpr int W = kHopBlock / 64;
        const int u = k * W + w;
        const int xw = LX / kXcds, per_t = xw * nyb;
        const int tl = u / per_t, rem = u - tl * per_t;
        const int xi = rem / nyb, yb = rem - xi * nyb;
        return ((tl * LX + xc * xw + xi) * nyb + yb) * 64;
    }
    if (xgroup > 0) {
        constexpr int W = kHopBlock / 64;
        const int u = k * W + w;  // unit rank inside the XCD's range
        const int per_group = nt * xgroup * nyb;
        const int xg = u / per_group, rem = u - xg * per_group;
        const int tl = rem / (xgroup * nyb), rem2 = rem - tl * (xgroup * nyb);
        const int xi = rem2 / nyb, yb = rem2 - xi * nyb;
        return (((xc * nt + tl) * LX + xg * xgroup + xi) * nyb + yb) * 64;
    }
    return (xc * q + (xc < r ? xc : r) + k) * kHopBlock + w * 64;
#else
    return b * kHopBlock + w * 64;
#endif
}

#ifndef TMH_HOP_PIPE_F16
#define TMH_HOP_PIPE_F16 0
#endif
// Software pipelining per storage precision.  FP16 runs without it: the
// single register set (72 VGPRs, 7 waves per SIMD) was measured 4 % faster
// at 32^3x64 than the pipelined one (117 VGPRs, 4 waves).
template <typename P>
constexpr bool kHopPipe = (sizeof(typename Word<P>::T) == 4 ? TMH_HOP_PIPE_F16 : TMH_HOP_PIPE) != 0;

template <typename P, int MODE, int LF>
__global__ void __launch_bounds__(kHopBlock) TMH_HOP_ATTR hop_kernel(HopArgs<P> a) {
    using R = real_t<P>;
    if (a.done && *a.done) return;
    if constexpr (MODE == 0) {
        // The CG step length from the partials of the preceding twist + norm
        // hop, summed in a fixed order (thread t takes t, t + 256, ...); it
        // is read only by the kernels launched after this one.
        if (a.apart && blockIdx.x == 0) {
            double s = 0.0;
            for (int k = threadIdx.x; k < a.napart; k += kHopBlock) s += a.apart[k];
            s = block_sum<kHopBlock>(s);
            if (threadIdx.x == 0) {
                a.ascal[kPQ] = s;
                a.ascal[kAlpha] = a.ascal[kRR] / s;
            }
        }
    }
    const int i = unit_site(blockIdx.x, threadIdx.x >> 6, gridDim.x, a.xgroup, a.nyb, a.nt, a.g.L[1]) +
                  (threadIdx.x & 63);
    double nrm = 0.0;
    if (i < a.g.Vh) {
        int c[4], lex;
        site_coords(a.g, i, a.pout, c, lex);
        cx<R> acc[4][3];
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int k = 0; k < 3; ++k) acc[s][k] = mk<R>(0, 0);
        const SiteNb n = site_neighbours(a.g, c, lex);
        hop_site<P, kHopPipe<P>, kLinkAux, LF>(acc, a, n, i);
        const int S = a.g.S;
        const R alpha = MODE >= 3 ? (R)a.scal[kAlpha] : (R)0;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const cx<R> cc = mk<R>(a.c_re[s >> 1], a.c_im[s >> 1]);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const int64_t comp = (int64_t)(3 * s + k) * S;
                cx<R> o = cc * acc[s][k];
                if constexpr (MODE >= 1)
                    o += mk<R>(a.d_re[s >> 1], a.d_im[s >> 1]) * bload<P, out_aux<P>()>(a.aux + comp, S, i);
                if constexpr (MODE == 2) nrm += (double)o.re * (double)o.re + (double)o.im * (double)o.im;
                if constexpr (MODE >= 3) {
                    cx<R> r = bload<P>(a.rio + comp, S, i);
                    r -= alpha * o;
                    bstore<P>(a.rio + comp, S, i, r);
                    nrm += (double)r.re * (double)r.re + (double)r.im * (double)r.im;
                    if constexpr (MODE == 4) {
                        cx<R> x = bload<P>(a.xio + comp, S, i);
                        x += alpha * bload<P>(a.pin + comp, S, i);
                        bstore<P>(a.xio + comp, S, i, x);
                    }
                } else {
                    bstore<P, out_aux<P>()>(a.out + comp, S, i, o);
                }
            }
        }
    }
    if constexpr (MODE >= 2) {
        const double s = block_sum<kHopBlock>(nrm);
        if (threadIdx.x == 0) a.partial[blockIdx.x] = s;
    }
}

int hop_blocks(const Geo& g) { return (g.Vh + kHopBlock - 1) / kHopBlock; }

#ifndef TMH_HOP_LDS_PAD
#define TMH_HOP_LDS_PAD 0
#endif
template <typename P, int LF>
static hipError_t launch_hop_lf(const HopArgs<P>& a, int mode, int nb, hipStream_t stream) {
    constexpr unsigned lds = TMH_HOP_LDS_PAD;
    switch (mode) {
        case 0: hipLaunchKernelGGL((hop_kernel<P, 0, LF>), dim3(nb), dim3(kHopBlock), lds, stream, a); break;
        case 1: hipLaunchKernelGGL((hop_kernel<P, 1, LF>), dim3(nb), dim3(kHopBlock), lds, stream, a); break;
        case 2: hipLaunchKernelGGL((hop_kernel<P, 2, LF>), dim3(nb), dim3(kHopBlock), lds, stream, a); break;
        case 3: hipLaunchKernelGGL((hop_kernel<P, 3, LF>), dim3(nb), dim3(kHopBlock), lds, stream, a); break;
        default: hipLaunchKernelGGL((hop_kernel<P, 4, LF>), dim3(nb), dim3(kHopBlock), lds, stream, a); break;
    }
    return hipGetLastError();
}

template <typename P>
hipError_t launch_hop(const HopArgs<P>& a, int mode, hipStream_t stream) {
    const int nb = hop_blocks(a.g);
    if (nb == 0) return hipSuccess;
    return a.lf ? launch_hop_lf<P, 1>(a, mode, nb, stream) : launch_hop_lf<P, 0>(a, mode, nb, stream);
}

template hipError_t launch_hop<double>(const HopArgs<double>&, int, hipStream_t);
template hipError_t launch_hop<float>(const HopArgs<float>&, int, hipStream_t);
template hipError_t launch_hop<half_t>(const HopArgs<half_t>&, int, hipStream_t);

}  // namespace tmh
