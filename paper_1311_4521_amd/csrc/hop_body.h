// Per-site body of the Wilson hopping matrix (shared by the single- and
// multi-right-hand-side kernels): neighbours from coordinates, the 8 terms
// with spin projection to half-spinors, SU(3) x half-spinor and the
// reconstruction of the lower spins.
#pragma once

#include "common.h"
#include "kernels.h"

// Compile-time tuning of the hopping kernel:
//   TMH_HOP_WAVES     minimum waves per SIMD the register allocation must
//                     allow (0: compiler's choice)
//   TMH_HOP_NT_LINKS  load links with non-temporal hints (each link is read
//                     once per application, so it need not displace the
//                     neighbour spinors in the caches)
//   TMH_XCD_REMAP     give every XCD one contiguous range of sites
//   TMH_HOP_SCHED     keep the instruction scheduler from moving work across
//                     the boundaries between the 8 terms
//   TMH_HOP_PIPE      software-pipeline the terms: load term t+1, then
//                     compute term t
//   TMH_HOP_NT_STORE  FP64 only: store the output (and read the fused
//                     epilogue's input at the output site) with non-temporal
//                     hints (measured: a gain in FP64, a small loss in FP32)
//   TMH_HOP_BLOCK     threads per workgroup
#ifndef TMH_HOP_WAVES
#define TMH_HOP_WAVES 0
#endif
#ifndef TMH_HOP_NT_LINKS
#define TMH_HOP_NT_LINKS 1
#endif
#ifndef TMH_XCD_REMAP
#define TMH_XCD_REMAP 1
#endif
#ifndef TMH_HOP_SCHED
#define TMH_HOP_SCHED 1
#endif
#ifndef TMH_HOP_PIPE
#define TMH_HOP_PIPE 1
#endif
#ifndef TMH_HOP_NT_STORE
#define TMH_HOP_NT_STORE 1
#endif
#ifndef TMH_HOP_BLOCK
#define TMH_HOP_BLOCK 256
#endif
#if TMH_HOP_WAVES > 0
#define TMH_HOP_ATTR __attribute__((amdgpu_waves_per_eu(TMH_HOP_WAVES, 8)))
#else
#define TMH_HOP_ATTR
#endif

namespace tmh {

// Cache policy of the link loads: each link is read once per application,
// so a non-temporal hint keeps it from displacing neighbour spinors.
#ifndef TMH_LINK_POLICY
#define TMH_LINK_POLICY 2
#endif
#ifndef TMH_OUT_POLICY
#define TMH_OUT_POLICY 2
#endif
constexpr int kLinkAux = TMH_HOP_NT_LINKS ? TMH_LINK_POLICY : 0;
template <typename P> constexpr int out_aux() { return (TMH_HOP_NT_STORE && sizeof(P) == 8) ? TMH_OUT_POLICY : 0; }
constexpr int kHopBlock = TMH_HOP_BLOCK;
static_assert(kHopBlock == kHopThreads, "the host sizes hop launches with kHopThreads");

// Data one of the 8 terms needs: the neighbour's spinor and the link.
template <typename R> struct TermData {
    cx<R> psi[4][3];
    cx<R> u[3][3];
};

// Link storage: LF = 0 keeps all 9 entries; LF = 1 keeps the first two rows
// (12 reals) and rebuilds the third as the complex conjugate of their cross
// product, exact for special unitary links (det U = 1: U = conj(cofactors)).
template <int LF> constexpr int link_comps() { return LF ? 6 : 9; }

template <typename R>
__device__ __forceinline__ void third_row(cx<R> (&u)[3][3]) {
    const cx<R> c0 = u[0][1] * u[1][2] - u[0][2] * u[1][1];
    const cx<R> c1 = u[0][2] * u[1][0] - u[0][0] * u[1][2];
    const cx<R> c2 = u[0][0] * u[1][1] - u[0][1] * u[1][0];
    u[2][0] = mk<R>(c0.re, -c0.im);
    u[2][1] = mk<R>(c1.re, -c1.im);
    u[2][2] = mk<R>(c2.re, -c2.im);
}

template <typename P, int LAUX, int LF>
__device__ __forceinline__ void load_term(TermData<real_t<P>>& d, const typename Word<P>::T* __restrict__ in,
                                          const typename Word<P>::T* __restrict__ link, int S, int jn, int jl) {
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int a = 0; a < 3; ++a) d.psi[s][a] = bload<P>(in + (int64_t)(3 * s + a) * S, S, jn);
#pragma unroll
    for (int k = 0; k < link_comps<LF>(); ++k) d.u[k / 3][k % 3] = bload<P, LAUX>(link + (int64_t)k * S, S, jl);
    // two-row links: the third row is rebuilt where the term is computed
    // (add_t), so that the loads of a term can be issued ahead of it
}

// FP32 arithmetic (FP32 and FP16 storage): the colour products as chains of
// one multiply and five fused multiply-adds (9-11 % fewer VALU instructions
// than products and sums of complex numbers; measured ~1 % faster)
#ifndef TMH_FMA_CHAINS
#define TMH_FMA_CHAINS 1
#endif
// u0 h0 + u1 h1 + u2 h2 as chains of fused multiply-adds.
template <typename R>
__device__ __forceinline__ cx<R> dot3(cx<R> u0, cx<R> u1, cx<R> u2, cx<R> h0, cx<R> h1, cx<R> h2) {
    R re = u2.im * h2.im;
    re = __builtin_fmaf(u2.re, h2.re, -re);
    re = __builtin_fmaf(-u1.im, h1.im, re);
    re = __builtin_fmaf(u1.re, h1.re, re);
    re = __builtin_fmaf(-u0.im, h0.im, re);
    re = __builtin_fmaf(u0.re, h0.re, re);
    R im = u2.im * h2.re;
    im = __builtin_fmaf(u2.re, h2.im, im);
    im = __builtin_fmaf(u1.im, h1.re, im);
    im = __builtin_fmaf(u1.re, h1.im, im);
    im = __builtin_fmaf(u0.im, h0.re, im);
    im = __builtin_fmaf(u0.re, h0.im, im);
    return {re, im};
}
// conj(u0) h0 + conj(u1) h1 + conj(u2) h2 as chains of fused multiply-adds.
template <typename R>
__device__ __forceinline__ cx<R> dot3c(cx<R> u0, cx<R> u1, cx<R> u2, cx<R> h0, cx<R> h1, cx<R> h2) {
    R re = u2.im * h2.im;
    re = __builtin_fmaf(u2.re, h2.re, re);
    re = __builtin_fmaf(u1.im, h1.im, re);
    re = __builtin_fmaf(u1.re, h1.re, re);
    re = __builtin_fmaf(u0.im, h0.im, re);
    re = __builtin_fmaf(u0.re, h0.re, re);
    R im = u2.im * h2.re;
    im = __builtin_fmaf(u2.re, h2.im, -im);
    im = __builtin_fmaf(-u1.im, h1.re, im);
    im = __builtin_fmaf(u1.re, h1.im, im);
    im = __builtin_fmaf(-u0.im, h0.re, im);
    im = __builtin_fmaf(u0.re, h0.im, im);
    return {re, im};
}

// Spin projection of one term: the half-spinor h = psi_up - DIR e_mu psi_dn
// that (1 - DIR gamma_mu) leaves independent.
template <typename R, int MU, int DIR>
__device__ __forceinline__ void project(cx<R> (&h)[2][3], const cx<R> (&psi)[4][3]) {
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
}

// A term from its projected half-spinor h (taken by value: the boundary
// phase is applied to it here) and its link.
template <typename R, int MU, int DIR>
__device__ __forceinline__ void add_term_h(cx<R> (&acc)[4][3], cx<R> h[2][3], const cx<R> (&u)[3][3], bool wrap,
                                           cx<R> ph);

// One of the 8 terms: DIR = +1 adds (1 - gamma_mu) U_mu(x) psi(x+mu),
// DIR = -1 adds (1 + gamma_mu) U_mu(x-mu)^dagger psi(x-mu).
template <typename R, int MU, int DIR>
__device__ __forceinline__ void add_term(cx<R> (&acc)[4][3], const TermData<R>& d, bool wrap, cx<R> ph) {
    cx<R> h[2][3];
    project<R, MU, DIR>(h, d.psi);
    add_term_h<R, MU, DIR>(acc, h, d.u, wrap, ph);
}

template <typename R, int MU, int DIR>
__device__ __forceinline__ void add_term_h(cx<R> (&acc)[4][3], cx<R> h[2][3], const cx<R> (&u)[3][3], bool wrap,
                                           cx<R> ph) {
    // boundary phase, branch-free so that each term stays one basic block
    const cx<R> eta = wrap ? ph : mk<R>(1, 0);
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int a = 0; a < 3; ++a) h[s][a] = h[s][a] * eta;
    // g = U h (forward) or U^dagger h (backward)
    cx<R> g[2][3];
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            if constexpr (TMH_FMA_CHAINS && sizeof(R) == 4) {
                // one multiply and five fused multiply-adds per real part
                if constexpr (DIR > 0)
                    g[s][a] = dot3(u[a][0], u[a][1], u[a][2], h[s][0], h[s][1], h[s][2]);
                else
                    g[s][a] = dot3c(u[0][a], u[1][a], u[2][a], h[s][0], h[s][1], h[s][2]);
            } else if constexpr (DIR > 0) {
                g[s][a] = u[a][0] * h[s][0] + u[a][1] * h[s][1] + u[a][2] * h[s][2];
            } else {
                g[s][a] = cmul(u[0][a], h[s][0]) + cmul(u[1][a], h[s][1]) + cmul(u[2][a], h[s][2]);
            }
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

// Site geometry shared by the 8 terms.
struct SiteNb {
    int jn[8];     // neighbour even-odd index, term t = 2*mu + (backward ? 1 : 0)
    unsigned wrap; // bit t set when term t crosses the boundary
};

__device__ __forceinline__ SiteNb site_neighbours(const Geo& g, const int c[4], int lex) {
    SiteNb n;
    n.wrap = 0;
    int stride = 1;
#pragma unroll
    for (int mu = 3; mu >= 0; --mu) {
        const int Lm = g.L[mu];
        const bool wf = c[mu] == Lm - 1, wb = c[mu] == 0;
        n.jn[2 * mu] = (wf ? lex - (Lm - 1) * stride : lex + stride) >> 1;
        n.jn[2 * mu + 1] = (wb ? lex + (Lm - 1) * stride : lex - stride) >> 1;
        n.wrap |= (wf ? 1u : 0u) << (2 * mu);
        n.wrap |= (wb ? 1u : 0u) << (2 * mu + 1);
        stride *= Lm;
    }
    return n;
}

// Term t = 2*mu + b: forward (b = 0) uses U_mu(x) from the output parity at
// the site's own index i; backward (b = 1) uses U_mu(x - mu) from the input
// parity at the neighbour's index.
template <typename P, int T, int LAUX, int LF>
__device__ __forceinline__ void load_t(TermData<real_t<P>>& d, const HopArgs<P>& a, const SiteNb& n, int i) {
    constexpr int MU = T / 2;
    constexpr int NC = link_comps<LF>();
    if constexpr (T % 2 == 0)
        load_term<P, LAUX, LF>(d, a.in, a.gout + (int64_t)MU * NC * a.g.S, a.g.S, n.jn[T], i);
    else
        load_term<P, LAUX, LF>(d, a.in, a.gin + (int64_t)MU * NC * a.g.S, a.g.S, n.jn[T], n.jn[T]);
}

template <typename P, int T, int LF = 0>
__device__ __forceinline__ void add_t(cx<real_t<P>> (&acc)[4][3], TermData<real_t<P>>& d, const HopArgs<P>& a,
                                      const SiteNb& n) {
    using R = real_t<P>;
    constexpr int MU = T / 2;
    if constexpr (LF == 1) third_row<R>(d.u);
    const bool wrap = (n.wrap >> T) & 1u;
    if constexpr (T % 2 == 0)
        add_term<R, MU, +1>(acc, d, wrap, mk<R>(a.ph_re[MU], a.ph_im[MU]));
    else
        add_term<R, MU, -1>(acc, d, wrap, mk<R>(a.ph_re[MU], -a.ph_im[MU]));
}

#if TMH_HOP_SCHED
#define TMH_SCHED_FENCE() __builtin_amdgcn_sched_barrier(0)
#else
#define TMH_SCHED_FENCE() ((void)0)
#endif

// Sum of the 8 terms.  PIPE loads term t+1 before computing term t (two
// register sets); otherwise each term is loaded and consumed in turn.  LAUX
// is the cache policy of the link loads.
template <typename P, bool PIPE, int LAUX = kLinkAux, int LF = 0>
__device__ __forceinline__ void hop_site(cx<real_t<P>> (&acc)[4][3], const HopArgs<P>& a, const SiteNb& n,
                                         int i) {
    using R = real_t<P>;
    if constexpr (PIPE) {
    TermData<R> d0, d1;
    load_t<P, 0, LAUX, LF>(d0, a, n, i);
    TMH_SCHED_FENCE();
    load_t<P, 1, LAUX, LF>(d1, a, n, i);
    TMH_SCHED_FENCE();
    add_t<P, 0, LF>(acc, d0, a, n);
    TMH_SCHED_FENCE();
    load_t<P, 2, LAUX, LF>(d0, a, n, i);
    TMH_SCHED_FENCE();
    add_t<P, 1, LF>(acc, d1, a, n);
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
    TermData<R> d;
#define TMH_TERM(T)              \
    load_t<P, T, LAUX, LF>(d, a, n, i);    \
    add_t<P, T, LF>(acc, d, a, n);   \
    TMH_SCHED_FENCE();
    TMH_TERM(0) TMH_TERM(1) TMH_TERM(2) TMH_TERM(3) TMH_TERM(4) TMH_TERM(5) TMH_TERM(6) TMH_TERM(7)
#undef TMH_TERM
    }
}

// FP16 storage, pipelined on the storage words: the loads of term t+1 stay in
// flight while term t is computed, held as binary16 pairs (one register per
// complex number, against two once widened), and each term is widened to
// FP32 just before it is used.  The widening is exact, so the sum is the
// same as the one-term-at-a-time form's.
template <int LF> struct TermRaw {
    h2 psi[12];
    h2 u[link_comps<LF>()];
};

template <int T, int LAUX, int LF>
__device__ __forceinline__ void load_t_raw(TermRaw<LF>& d, const HopArgs<half_t>& a, const SiteNb& n, int i) {
    constexpr int MU = T / 2;
    constexpr int NC = link_comps<LF>();
    const int S = a.g.S;
    const unsigned nb = (unsigned)S * sizeof(h2);
    const h2* link = (T % 2 == 0 ? a.gout : a.gin) + (int64_t)MU * NC * S;
    const unsigned jl = (unsigned)(T % 2 == 0 ? i : n.jn[T]) * sizeof(h2);
    const unsigned jn = (unsigned)n.jn[T] * sizeof(h2);
#pragma unroll
    for (int k = 0; k < 12; ++k) d.psi[k] = BufIO<half_t>::load<0>(buf_rsrc(a.in + (int64_t)k * S, nb), jn);
#pragma unroll
    for (int k = 0; k < NC; ++k) d.u[k] = BufIO<half_t>::load<LAUX>(buf_rsrc(link + (int64_t)k * S, nb), jl);
}

template <int LF>
__device__ __forceinline__ void widen_term(TermData<float>& d, const TermRaw<LF>& r) {
#pragma unroll
    for (int k = 0; k < 12; ++k) d.psi[k / 3][k % 3] = mk<float>((float)r.psi[k].x, (float)r.psi[k].y);
#pragma unroll
    for (int k = 0; k < link_comps<LF>(); ++k) d.u[k / 3][k % 3] = mk<float>((float)r.u[k].x, (float)r.u[k].y);
}

template <int LAUX, int LF>
__device__ __forceinline__ void hop_site_raw(cx<float> (&acc)[4][3], const HopArgs<half_t>& a, const SiteNb& n,
                                             int i) {
    TermRaw<LF> r0, r1;
    TermData<float> d;
    load_t_raw<0, LAUX, LF>(r0, a, n, i);
    TMH_SCHED_FENCE();
    load_t_raw<1, LAUX, LF>(r1, a, n, i);
    TMH_SCHED_FENCE();
#define TMH_RAW_STEP(T, RT, RN)                       \
    widen_term<LF>(d, RT);                            \
    add_t<half_t, T, LF>(acc, d, a, n);               \
    TMH_SCHED_FENCE();                                \
    load_t_raw<T + 2, LAUX, LF>(RT, a, n, i);         \
    TMH_SCHED_FENCE();
    TMH_RAW_STEP(0, r0, r1) TMH_RAW_STEP(1, r1, r0) TMH_RAW_STEP(2, r0, r1) TMH_RAW_STEP(3, r1, r0)
    TMH_RAW_STEP(4, r0, r1) TMH_RAW_STEP(5, r1, r0)
#undef TMH_RAW_STEP
    widen_term<LF>(d, r0);
    add_t<half_t, 6, LF>(acc, d, a, n);
    TMH_SCHED_FENCE();
    widen_term<LF>(d, r1);
    add_t<half_t, 7, LF>(acc, d, a, n);
}

// Multi-right-hand-side form: NR fields `fstride` words apart share every
// link load.  Per term the link goes to registers once and is applied to the
// NR neighbour spinors in turn; right-hand sides r >= nv are skipped.
template <typename P, int T, int LAUX>
__device__ __forceinline__ void load_t_link(TermData<real_t<P>>& d, const HopArgs<P>& a, const SiteNb& n, int i) {
    constexpr int MU = T / 2;
    const int S = a.g.S;
    const typename Word<P>::T* link = (T % 2 == 0 ? a.gout : a.gin) + (int64_t)MU * 9 * S;
    const int jl = T % 2 == 0 ? i : n.jn[T];
#pragma unroll
    for (int k = 0; k < 9; ++k) d.u[k / 3][k % 3] = bload<P, LAUX>(link + (int64_t)k * S, S, jl);
}

template <typename P, int T>
__device__ __forceinline__ void load_t_psi(TermData<real_t<P>>& d, const typename Word<P>::T* in, int S,
                                           const SiteNb& n) {
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) d.psi[s][c] = bload<P>(in + (int64_t)(3 * s + c) * S, S, n.jn[T]);
}

template <typename P, int NR, int LAUX>
__device__ __forceinline__ void hop_site_nr(cx<real_t<P>> (&acc)[NR][4][3], const HopArgs<P>& a, int64_t fstride,
                                            int nv, const SiteNb& n, int i) {
    using R = real_t<P>;
    TermData<R> d;
#define TMH_TERM_NR(T)                                              \
    load_t_link<P, T, LAUX>(d, a, n, i);                            \
    _Pragma("unroll") for (int r = 0; r < NR; ++r) {                \
        if (r < nv) {                                               \
            load_t_psi<P, T>(d, a.in + r * fstride, a.g.S, n);      \
            add_t<P, T>(acc[r], d, a, n);                           \
        }                                                           \
        TMH_SCHED_FENCE();                                          \
    }
    TMH_TERM_NR(0) TMH_TERM_NR(1) TMH_TERM_NR(2) TMH_TERM_NR(3)
    TMH_TERM_NR(4) TMH_TERM_NR(5) TMH_TERM_NR(6) TMH_TERM_NR(7)
#undef TMH_TERM_NR
}

}  // namespace tmh
