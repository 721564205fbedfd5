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
#define TMH_HOP_PIPE_F16 2
#endif
// Software pipelining per storage precision.  FP16 (2) pipelines on the
// storage words (hop_site_raw: 89-95 VGPRs, 5 waves per SIMD), 2.5-3.5 %
// faster at 32^3x64 than one term at a time (66-76 VGPRs, 6-7 waves); the
// pipelined form on widened values (1: 117 VGPRs, 4 waves) was 4 % slower
// than one term at a time.
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
        if constexpr (sizeof(typename Word<P>::T) == 4 && TMH_HOP_PIPE_F16 == 2)
            hop_site_raw<kLinkAux, LF>(acc, a, n, i);
        else
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

// ------------------------------------------------------------ t-marching
//
// A site x = (t, x, y, z) and its neighbour x + z^ or x - z^ with z even/odd
// share the even-odd index of their time-slice: the two sites (x, y, 2zp)
// and (x, y, 2zp + 1) form a pair, and at every t one of them is on the
// output parity and the other on the input parity.  The two time neighbours
// of the output site of pair j at t are the input sites of the same pair at
// t - 1 and t + 1.  A thread owns one pair of a tile of kHopBlock pairs and
// walks tm_steps consecutive time-slices; it loads the input site of its pair
// at t + 1 (the forward time neighbour) once, and keeps it in registers for
// the next two steps, where it is the pair's own input site and then the
// backward time neighbour.  Neither time neighbour is read from memory twice;
// the six spatial neighbours of the slice in progress are read from the
// caches, where the tiles of the same XCD working on the same slice have
// just brought them.  XCD k runs one contiguous range of (t-range, tile)
// workgroups, i.e. a contiguous part of one range of time-slices.

template <typename P>
__device__ __forceinline__ void load_psi(cx<real_t<P>> (&psi)[4][3], const typename Word<P>::T* __restrict__ in,
                                         int S, int j) {
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) psi[s][c] = bload<P>(in + (int64_t)(3 * s + c) * S, S, j);
}

// The link of term T only (its spinor comes from the registers).
template <typename P, int T, int LAUX, int LF>
__device__ __forceinline__ void load_link_t(TermData<real_t<P>>& d, const HopArgs<P>& a, const SiteNb& n, int i) {
    constexpr int MU = T / 2;
    constexpr int NC = link_comps<LF>();
    const int S = a.g.S;
    const typename Word<P>::T* link = (T % 2 == 0 ? a.gout : a.gin) + (int64_t)MU * NC * S;
    const int jl = T % 2 == 0 ? i : n.jn[T];
#pragma unroll
    for (int k = 0; k < NC; ++k) d.u[k / 3][k % 3] = bload<P, LAUX>(link + (int64_t)k * S, S, jl);
}

// The 8 terms of one output site in the t-march.  Term 0 (forward t) loads
// psi(t + 1) from memory; term 1 (backward t) takes the projection
// hprev = (1 + gamma_0) psi(t - 1) from the registers.  Afterwards the ring
// advances: hprev <- hcur <- (1 + gamma_0) psi(t + 1).  PIPE issues the
// loads of each term before the previous term is computed.
#ifndef TMH_TM_PIPE
#define TMH_TM_PIPE 1
#endif
template <typename P, int LAUX, int LF>
__device__ __forceinline__ void tm_time_terms(cx<real_t<P>> (&acc)[4][3], TermData<real_t<P>>& d0,
                                              TermData<real_t<P>>& d1, const HopArgs<P>& a, const SiteNb& n,
                                              cx<real_t<P>> (&hprev)[2][3], cx<real_t<P>> (&hcur)[2][3]) {
    using R = real_t<P>;
    add_t<P, 0, LF>(acc, d0, a, n);
    cx<R> hn[2][3];
    project<R, 0, -1>(hn, d0.psi);
    if constexpr (LF == 1) third_row<R>(d1.u);
    add_term_h<R, 0, -1>(acc, hprev, d1.u, (n.wrap >> 1) & 1u, mk<R>(a.ph_re[0], -a.ph_im[0]));
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            hprev[s][c] = hcur[s][c];
            hcur[s][c] = hn[s][c];
        }
}

template <typename P, int LAUX, int LF>
__device__ __forceinline__ void hop_site_tm(cx<real_t<P>> (&acc)[4][3], const HopArgs<P>& a, const SiteNb& n, int i,
                                            cx<real_t<P>> (&hprev)[2][3], cx<real_t<P>> (&hcur)[2][3]) {
    using R = real_t<P>;
    if constexpr (TMH_TM_PIPE) {
        TermData<R> d0, d1;
        load_t<P, 0, LAUX, LF>(d0, a, n, i);
        TMH_SCHED_FENCE();
        load_link_t<P, 1, LAUX, LF>(d1, a, n, i);
        TMH_SCHED_FENCE();
        tm_time_terms<P, LAUX, LF>(acc, d0, d1, a, n, hprev, hcur);
        TMH_SCHED_FENCE();
        load_t<P, 2, LAUX, LF>(d0, a, n, i);
        TMH_SCHED_FENCE();
        load_t<P, 3, LAUX, LF>(d1, a, n, i);
        TMH_SCHED_FENCE();
        add_t<P, 2, LF>(acc, d0, a, n);
        TMH_SCHED_FENCE();
        load_t<P, 4, LAUX, LF>(d0, a, n, i);
        TMH_SCHED_FENCE();
        add_t<P, 3, LF>(acc, d1, a, n);
        TMH_SCHED_FENCE();
        load_t<P, 5, LAUX, LF>(d1, a, n, i);
        TMH_SCHED_FENCE();
        add_t<P, 4, LF>(acc, d0, a, n);
        TMH_SCHED_FENCE();
        load_t<P, 6, LAUX, LF>(d0, a, n, i);
        TMH_SCHED_FENCE();
        add_t<P, 5, LF>(acc, d1, a, n);
        TMH_SCHED_FENCE();
        load_t<P, 7, LAUX, LF>(d1, a, n, i);
        TMH_SCHED_FENCE();
        add_t<P, 6, LF>(acc, d0, a, n);
        TMH_SCHED_FENCE();
        add_t<P, 7, LF>(acc, d1, a, n);
    } else {
        TermData<R> d0, d1;
        load_t<P, 0, LAUX, LF>(d0, a, n, i);
        load_link_t<P, 1, LAUX, LF>(d1, a, n, i);
        tm_time_terms<P, LAUX, LF>(acc, d0, d1, a, n, hprev, hcur);
        TMH_SCHED_FENCE();
#define TMH_TM1_TERM(T)                   \
    load_t<P, T, LAUX, LF>(d0, a, n, i);  \
    add_t<P, T, LF>(acc, d0, a, n);       \
    TMH_SCHED_FENCE();
        TMH_TM1_TERM(2) TMH_TM1_TERM(3) TMH_TM1_TERM(4) TMH_TM1_TERM(5) TMH_TM1_TERM(6) TMH_TM1_TERM(7)
#undef TMH_TM1_TERM
    }
}

template <typename P, int MODE, int LF>
__global__ void __launch_bounds__(kHopBlock) hop_tmarch_kernel(HopArgs<P> a) {
    using R = real_t<P>;
    if (a.done && *a.done) return;
    if constexpr (MODE == 0) {
        // CG step length from the preceding twist + norm hop (as hop_kernel)
        if (a.apart && blockIdx.x == 0) {
            double s = 0.0;
            for (int k = threadIdx.x; k < a.napart; k += kHopBlock) s += a.apart[k];
            s = block_sum<kHopBlock>(s);
            if (threadIdx.x == 0) {
                a.ascal[kPQ] = s;
                a.ascal[kAlpha] = a.ascal[kRR] / s;
            }
            __syncthreads();
        }
    }
    const int L = xcd_remap(blockIdx.x, gridDim.x);
    const int range = L / a.tm_nw, w = L - range * a.tm_nw;
    const int slice = a.tm_slice, T = a.g.L[0], S = a.g.S;
    const int jp = w * kHopBlock + threadIdx.x;  // pair index inside a slice (slice % kHopBlock == 0)
    const int hz = a.g.L[3] >> 1;
    const int row = jp / hz, zp = jp - row * hz;
    const int y = row % a.g.L[2], x = row / a.g.L[2];
    const int t0 = range * a.tm_steps;
    cx<R> hprev[2][3], hcur[2][3];
    {
        cx<R> psi[4][3];
        load_psi<P>(psi, a.in, S, (t0 == 0 ? T - 1 : t0 - 1) * slice + jp);
        project<R, 0, -1>(hprev, psi);
        load_psi<P>(psi, a.in, S, t0 * slice + jp);
        project<R, 0, -1>(hcur, psi);
    }
    __shared__ double wsum[kHopBlock / 64];
    for (int st = 0; st < a.tm_steps; ++st) {
        // The field addresses pass through an empty asm every step, so that
        // the compiler rebuilds the ~170 buffer descriptors inside the step
        // (a few scalar instructions each) instead of hoisting them out of
        // the loop, where they would not fit in the scalar registers.
        HopArgs<P> b = a;
        __asm__ volatile("" : "+s"(b.in), "+s"(b.gout), "+s"(b.gin), "+s"(b.out), "+s"(b.aux));
        if constexpr (MODE >= 3) __asm__ volatile("" : "+s"(b.rio), "+s"(b.xio), "+s"(b.pin));
        const int t = t0 + st;
        const int i = t * slice + jp;
        int c[4];
        c[0] = t;
        c[1] = x;
        c[2] = y;
        c[3] = 2 * zp + ((t + x + y + a.pout) & 1);
        const int lex = ((t * a.g.L[1] + x) * a.g.L[2] + y) * a.g.L[3] + c[3];
        cx<R> acc[4][3];
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int k = 0; k < 3; ++k) acc[s][k] = mk<R>(0, 0);
        const SiteNb n = site_neighbours(a.g, c, lex);
        hop_site_tm<P, kLinkAux, LF>(acc, b, n, i, hprev, hcur);
        const R alpha = MODE >= 3 ? (R)a.scal[kAlpha] : (R)0;
        double nrm = 0.0;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const cx<R> cc = mk<R>(a.c_re[s >> 1], a.c_im[s >> 1]);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const int64_t comp = (int64_t)(3 * s + k) * S;
                cx<R> o = cc * acc[s][k];
                if constexpr (MODE >= 1)
                    o += mk<R>(a.d_re[s >> 1], a.d_im[s >> 1]) * bload<P, out_aux<P>()>(b.aux + comp, S, i);
                if constexpr (MODE == 2) nrm += (double)o.re * (double)o.re + (double)o.im * (double)o.im;
                if constexpr (MODE >= 3) {
                    cx<R> r = bload<P>(b.rio + comp, S, i);
                    r -= alpha * o;
                    bstore<P>(b.rio + comp, S, i, r);
                    nrm += (double)r.re * (double)r.re + (double)r.im * (double)r.im;
                    if constexpr (MODE == 4) {
                        cx<R> xv = bload<P>(b.xio + comp, S, i);
                        xv += alpha * bload<P>(b.pin + comp, S, i);
                        bstore<P>(b.xio + comp, S, i, xv);
                    }
                } else {
                    bstore<P, out_aux<P>()>(b.out + comp, S, i, o);
                }
            }
        }
        if constexpr (MODE >= 2) {
            // one partial per slice tile, at the index the one-site-per-lane
            // kernel's blocks use: the sums keep their count and order
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) nrm += __shfl_xor(nrm, off, 64);
            if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = nrm;
            __syncthreads();
            if (threadIdx.x == 0) {
                double sum = 0.0;
#pragma unroll
                for (int k = 0; k < kHopBlock / 64; ++k) sum += wsum[k];
                a.partial[t * a.tm_nw + w] = sum;
            }
            __syncthreads();
        }
    }
}

int hop_tmarch_blocks(const Geo& g, int steps) { return g.Vh / kHopBlock / steps; }

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

template <typename P, int LF>
static hipError_t launch_tmarch_lf(const HopArgs<P>& a, int mode, int nb, hipStream_t stream) {
    switch (mode) {
        case 0: hipLaunchKernelGGL((hop_tmarch_kernel<P, 0, LF>), dim3(nb), dim3(kHopBlock), 0, stream, a); break;
        case 1: hipLaunchKernelGGL((hop_tmarch_kernel<P, 1, LF>), dim3(nb), dim3(kHopBlock), 0, stream, a); break;
        case 2: hipLaunchKernelGGL((hop_tmarch_kernel<P, 2, LF>), dim3(nb), dim3(kHopBlock), 0, stream, a); break;
        case 3: hipLaunchKernelGGL((hop_tmarch_kernel<P, 3, LF>), dim3(nb), dim3(kHopBlock), 0, stream, a); break;
        default: hipLaunchKernelGGL((hop_tmarch_kernel<P, 4, LF>), dim3(nb), dim3(kHopBlock), 0, stream, a); break;
    }
    return hipGetLastError();
}

template <typename P>
hipError_t launch_hop(const HopArgs<P>& a, int mode, hipStream_t stream) {
    if (a.tm_steps > 0) {
        // the host checked: tm_slice % kHopBlock == 0, tm_steps divides T,
        // tm_nw * kHopBlock == tm_slice, T * tm_slice == Vh
        const int nb = hop_tmarch_blocks(a.g, a.tm_steps);
        if (nb == 0) return hipSuccess;
        return a.lf ? launch_tmarch_lf<P, 1>(a, mode, nb, stream) : launch_tmarch_lf<P, 0>(a, mode, nb, stream);
    }
    const int nb = hop_blocks(a.g);
    if (nb == 0) return hipSuccess;
    return a.lf ? launch_hop_lf<P, 1>(a, mode, nb, stream) : launch_hop_lf<P, 0>(a, mode, nb, stream);
}

template hipError_t launch_hop<double>(const HopArgs<double>&, int, hipStream_t);
template hipError_t launch_hop<float>(const HopArgs<float>&, int, hipStream_t);
template hipError_t launch_hop<half_t>(const HopArgs<half_t>&, int, hipStream_t);

}  // namespace tmh
