// Gauge-link derivative ("fermionic derivative") of L = Re <X, H Y> for the
// hopping matrix H between checkerboards, accumulated per link in FP64.
//
// Every link of the lattice sits in exactly one term of H: a link leaving a
// site of the output parity in the forward term of that site, a link leaving
// a site of the input parity in the backward term of its forward neighbour.
// One thread owns one link, so every link has one writer and no atomics are
// needed.  For the term of link U = U_mu(l):
//   forward   W = kappa eta+ sum_s phi_s X_s^+,  phi = (1 - gamma_mu) Y(l+mu),
//             X = X(l);  M = U W;   Euclidean gradient W^+
//   backward  W = kappa eta- sum_s phi_s X_s^+,  phi = (1 + gamma_mu) Y(l),
//             X = X(l+mu);  M = -W U^+;  Euclidean gradient W
// and the su(3) force is TA(M) = (M - M^+)/2 - tr(M - M^+)/6.  X enters
// through per-chirality coefficients (X_eff = c_{s/2} X_s), which fold the
// gamma_5 and (A^+)^-1 factors of the twisted-mass chain into the kernel.
#include "common.h"
#include "kernels.h"

namespace tmh {

namespace {

// Links and force entries are each touched by one thread once: their loads
// and stores carry the non-temporal hint, which keeps them from displacing
// the spinors, which several threads read.
constexpr int kOnce = 2;

// The sum over the four spins of a term is done on two: phi = (1 + s gamma_mu) y
// has lower spins s E^+ h, where h = y_up + s E y_dn (s = -1 forward, +1
// backward, E the 2x2 spin block of gamma_mu), so
//   W = kappa eta sum_s phi_s (c x)_s^+ = sum_{t=0,1} h_t xt_t^+,
//   xt = f (c_up x_up + s c_dn E x_dn),  f = conj(kappa eta) coeff,
// with f negated for backward su(3) terms.  The link's contribution M is
//   su(3), forward:   U W        = sum_t (U h_t) xt_t^+
//   su(3), backward:  -W U^+     = sum_t h_t (U xt_t)^+   (sign in f)
//   Euclidean, forward:  W^+     = sum_t xt_t h_t^+
//   Euclidean, backward: W       = sum_t h_t xt_t^+
// and the force grows by TA(M) = (M - M^+)/2 - tr(M - M^+)/6 (su(3)) or by M.
template <int MU, bool FWD, int KIND>
__device__ __forceinline__ void term_proj(cx<double> (&h)[2][3], cx<double> (&xt)[2][3], const cx<double> (&x)[4][3],
                                          const cx<double> (&y)[4][3], cx<double> eta, const ForceArgs& t) {
    const cx<double> cu = mk<double>(t.cx_re[0], t.cx_im[0]);
    const cx<double> cd = mk<double>(t.cx_re[1], t.cx_im[1]);
    const double sg = (FWD || KIND != 0) ? t.coeff : -t.coeff;
    const cx<double> f = mk<double>(sg * eta.re, -sg * eta.im);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        cx<double> e0, e1, g0, g1;
        e_lower<double, MU>(y[2][k], y[3][k], e0, e1);
        e_lower<double, MU>(x[2][k], x[3][k], g0, g1);
        g0 = cd * g0;
        g1 = cd * g1;
        cx<double> a0 = cu * x[0][k], a1 = cu * x[1][k];
        if constexpr (FWD) {
            h[0][k] = y[0][k] - e0;
            h[1][k] = y[1][k] - e1;
            a0 -= g0;
            a1 -= g1;
        } else {
            h[0][k] = y[0][k] + e0;
            h[1][k] = y[1][k] + e1;
            a0 += g0;
            a1 += g1;
        }
        xt[0][k] = f * a0;
        xt[1][k] = f * a1;
    }
}

// W[r][q] = sum_t h_t[r] conj(xt_t[q])
__device__ __forceinline__ void term_w(cx<double> (&W)[3][3], const cx<double> (&h)[2][3],
                                       const cx<double> (&xt)[2][3]) {
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int q = 0; q < 3; ++q) W[r][q] = cmul(xt[0][q], h[0][r]) + cmul(xt[1][q], h[1][r]);
}

// force += TA(M) (su(3)) or M (Euclidean) for the link (p, mu) of site i,
// with M[r][q] = m(r, q).
template <int KIND, typename MF>
__device__ __forceinline__ void force_rmw(const ForceArgs& a, int p, int mu, int i, MF m) {
    const int S = a.g.S;
    double2* fo = a.force + ((int64_t)(p * 4 + mu) * 9) * S;
    double tr_im = 0.0;
    if constexpr (KIND == 0) tr_im = (m(0, 0).im + m(1, 1).im + m(2, 2).im) / 3.0;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const int r = k / 3, q = k % 3;
        cx<double> o;
        if constexpr (KIND == 0) {
            const cx<double> mrq = m(r, q), mqr = m(q, r);
            o = mk<double>(0.5 * (mrq.re - mqr.re), 0.5 * (mrq.im + mqr.im));
            if (r == q) o.im -= tr_im;
        } else {
            o = m(r, q);
        }
        const cx<double> fv = bload<double, kOnce>(fo + (int64_t)k * S, S, i);
        bstore<double, kOnce>(fo + (int64_t)k * S, S, i, mk<double>(fv.re + o.re, fv.im + o.im));
    }
}

__device__ __forceinline__ void load_link(cx<double> (&u)[3][3], const ForceArgs& a, int p, int mu, int i) {
    const int S = a.g.S;
    const double2* lk = a.gauge + ((int64_t)(p * 4 + mu) * 9) * S;
#pragma unroll
    for (int k = 0; k < 9; ++k) u[k / 3][k % 3] = bload<double, kOnce>(lk + (int64_t)k * S, S, i);
}

__device__ __forceinline__ void load_spinor(cx<double> (&v)[4][3], const double2* f, int S, int i) {
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int k = 0; k < 3; ++k) v[s][k] = bload<double>(f + (int64_t)(3 * s + k) * S, S, i);
}

// Forward neighbours of the site with coordinates c and lex index lex: eo
// index jn[mu] and whether the step wraps.
__device__ __forceinline__ void forward_nbs(const Geo& g, const int (&c)[4], int lex, int (&jn)[4], bool (&wr)[4]) {
    int stride = 1;
#pragma unroll
    for (int mu = 3; mu >= 0; --mu) {
        const int Lm = g.L[mu];
        wr[mu] = c[mu] == Lm - 1;
        jn[mu] = (wr[mu] ? lex - (Lm - 1) * stride : lex + stride) >> 1;
        stride *= Lm;
    }
}

__device__ __forceinline__ cx<double> term_eta(const ForceArgs& a, int mu, bool wrap, bool forward) {
    if (!wrap) return mk<double>(a.kappa, 0.0);
    return mk<double>(a.kappa * a.ph_re[mu], (forward ? a.kappa : -a.kappa) * a.ph_im[mu]);
}

// One link of one bilinear; own is the field at the link's site.  M is
// formed entry by entry from the two-spin factors, so the kernel holds no
// 3x3 accumulator.
template <int MU, bool FWD, int KIND>
__device__ __forceinline__ void force_link(const ForceArgs& a, int p, int i, int j, bool wrap,
                                           const cx<double> (&own)[4][3]) {
    cx<double> h[2][3], xt[2][3];
    {
        cx<double> nb[4][3];
        load_spinor(nb, FWD ? a.Y : a.X, a.g.S, j);
        if constexpr (FWD)
            term_proj<MU, true, KIND>(h, xt, own, nb, term_eta(a, MU, wrap, true), a);
        else
            term_proj<MU, false, KIND>(h, xt, nb, own, term_eta(a, MU, wrap, false), a);
    }
    // M[r][q] = sum_t av_t[r] conj(bv_t[q])
    cx<double> av[2][3], bv[2][3];
    if constexpr (KIND == 0) {
        cx<double> u[3][3];
        load_link(u, a, p, MU, i);
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                if constexpr (FWD) {
                    av[t][r] = u[r][0] * h[t][0] + u[r][1] * h[t][1] + u[r][2] * h[t][2];
                    bv[t][r] = xt[t][r];
                } else {
                    av[t][r] = h[t][r];
                    bv[t][r] = u[r][0] * xt[t][0] + u[r][1] * xt[t][1] + u[r][2] * xt[t][2];
                }
            }
    } else {
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                av[t][r] = FWD ? xt[t][r] : h[t][r];
                bv[t][r] = FWD ? h[t][r] : xt[t][r];
            }
    }
    force_rmw<KIND>(a, p, MU, i, [&](int r, int q) { return cmul(bv[0][q], av[0][r]) + cmul(bv[1][q], av[1][r]); });
}

// ----------------------------------------------------- two bilinears at once
//
// The force of Re <chi, Qhat psi> is the sum of the derivatives of two
// bilinears, one through H_oe and one through H_eo.  Every link sits in one
// term of each, forward (F) in one and backward (B) in the other; the kernel
// below forms M = U W_F + W_B U^+ (su(3); W_F^+ + W_B for the Euclidean
// gradient) per link and adds it to the force in one read-modify-write,
// where two single-bilinear launches would read and write every force entry
// twice.
template <int MU, int KIND>
__device__ __forceinline__ void force2_link(const ForceArgs& f, const ForceArgs& b, int p, int i, int j, bool wrap) {
    // one bilinear after the other, each with its own site's field, so that
    // only one pair of fields is held at a time
    cx<double> WF[3][3], WB[3][3];
    {
        cx<double> h[2][3], xt[2][3];
        {
            cx<double> x[4][3], y[4][3];
            load_spinor(x, f.X, f.g.S, i);
            load_spinor(y, f.Y, f.g.S, j);
            term_proj<MU, true, KIND>(h, xt, x, y, term_eta(f, MU, wrap, true), f);
        }
        term_w(WF, h, xt);
    }
    {
        cx<double> h[2][3], xt[2][3];
        {
            cx<double> x[4][3], y[4][3];
            load_spinor(x, b.X, f.g.S, j);
            load_spinor(y, b.Y, f.g.S, i);
            term_proj<MU, false, KIND>(h, xt, x, y, term_eta(f, MU, wrap, false), b);
        }
        term_w(WB, h, xt);
    }
    if constexpr (KIND == 0) {
        cx<double> u[3][3];
        load_link(u, f, p, MU, i);
        force_rmw<0>(f, p, MU, i, [&](int r, int q) {
            cx<double> s = u[r][0] * WF[0][q] + u[r][1] * WF[1][q] + u[r][2] * WF[2][q];
#pragma unroll
            for (int k = 0; k < 3; ++k) s += WB[r][k] * mk<double>(u[q][k].re, -u[q][k].im);
            return s;
        });
    } else {
        force_rmw<1>(f, p, MU, i, [&](int r, int q) {
            return mk<double>(WF[q][r].re + WB[r][q].re, -WF[q][r].im + WB[r][q].im);
        });
    }
}

// ------------------------------------------------------- one link per thread
//
// Wave w of a workgroup takes the links of direction mu = w of 64 sites of
// one time-slice, so the four waves load the same own fields at the same
// time and every spinor a workgroup needs is requested when it starts.
// Consecutive logical blocks take kLinkTG consecutive time-slices of the
// same 64 spatial sites (both parities each), so most forward time
// neighbours are requested by a workgroup that runs at about the same time.
#ifndef TMH_FORCE_LINK_TG
#define TMH_FORCE_LINK_TG 2
#endif
constexpr int kLinkTG = TMH_FORCE_LINK_TG;
constexpr int kLinkBlock = 256;

__host__ __device__ inline int link_units(const Geo& g) { return (g.Vh / g.L[0] + 63) / 64; }

__host__ inline int link_blocks(const Geo& g) { return 2 * kLinkTG * ((g.L[0] + kLinkTG - 1) / kLinkTG) * link_units(g); }

__device__ __forceinline__ bool link_site(const Geo& g, int& p, int& i, int& mu) {
    const int v3h = g.Vh / g.L[0];
    const int nsu = link_units(g);
    const int vb = xcd_remap(blockIdx.x, gridDim.x);
    const int r = vb >> 1, tw = r % kLinkTG, r2 = r / kLinkTG;
    const int su = r2 % nsu, tg = r2 / nsu;
    mu = threadIdx.x >> 6;
    const int t = tg * kLinkTG + tw, s = su * 64 + (threadIdx.x & 63);
    p = (vb & 1) ^ (tw & 1);
    i = t * v3h + s;
    return t < g.L[0] && s < v3h;
}

template <bool FWD, int KIND>
__device__ __forceinline__ void force_one_link(const ForceArgs& a, int p, int i, int mu, const int (&jn)[4],
                                               const bool (&wr)[4]) {
    cx<double> own[4][3];
    load_spinor(own, FWD ? a.X : a.Y, a.g.S, i);
    switch (mu) {
        case 0: force_link<0, FWD, KIND>(a, p, i, jn[0], wr[0], own); break;
        case 1: force_link<1, FWD, KIND>(a, p, i, jn[1], wr[1], own); break;
        case 2: force_link<2, FWD, KIND>(a, p, i, jn[2], wr[2], own); break;
        default: force_link<3, FWD, KIND>(a, p, i, jn[3], wr[3], own); break;
    }
}

template <int KIND>
__global__ void __launch_bounds__(kLinkBlock) __attribute__((amdgpu_waves_per_eu(4, 8)))
force_lk_kernel(ForceArgs a) {
    int p, i, mu;
    if (!link_site(a.g, p, i, mu)) return;
    int c[4], lex;
    site_coords(a.g, i, p, c, lex);
    int jn[4];
    bool wr[4];
    forward_nbs(a.g, c, lex, jn, wr);
    if (p == a.pout)
        force_one_link<true, KIND>(a, p, i, mu, jn, wr);
    else
        force_one_link<false, KIND>(a, p, i, mu, jn, wr);
}

template <int KIND>
__device__ __forceinline__ void force2_one_link(const ForceArgs& f, const ForceArgs& b, int p, int i, int mu,
                                                const int (&jn)[4], const bool (&wr)[4]) {
    switch (mu) {
        case 0: force2_link<0, KIND>(f, b, p, i, jn[0], wr[0]); break;
        case 1: force2_link<1, KIND>(f, b, p, i, jn[1], wr[1]); break;
        case 2: force2_link<2, KIND>(f, b, p, i, jn[2], wr[2]); break;
        default: force2_link<3, KIND>(f, b, p, i, jn[3], wr[3]); break;
    }
}

// 168 VGPRs, three waves per SIMD (two bilinears' 3x3 factors; measured 9 %
// faster than two waves with 175)
template <int KIND>
__global__ void __launch_bounds__(kLinkBlock) __attribute__((amdgpu_waves_per_eu(3, 8)))
force2_lk_kernel(ForceArgs a, ForceArgs b) {
    int p, i, mu;
    if (!link_site(a.g, p, i, mu)) return;
    int c[4], lex;
    site_coords(a.g, i, p, c, lex);
    int jn[4];
    bool wr[4];
    forward_nbs(a.g, c, lex, jn, wr);
    if (p == a.pout)
        force2_one_link<KIND>(a, b, p, i, mu, jn, wr);
    else
        force2_one_link<KIND>(b, a, p, i, mu, jn, wr);
}

}  // namespace

hipError_t launch_force2(const ForceArgs& a, const ForceArgs& b, hipStream_t s) {
    if (a.g.Vh == 0) return hipSuccess;
    if (a.kind == 0)
        hipLaunchKernelGGL(force2_lk_kernel<0>, dim3(link_blocks(a.g)), dim3(kLinkBlock), 0, s, a, b);
    else
        hipLaunchKernelGGL(force2_lk_kernel<1>, dim3(link_blocks(a.g)), dim3(kLinkBlock), 0, s, a, b);
    return hipGetLastError();
}

hipError_t launch_force(const ForceArgs& a, hipStream_t s) {
    if (a.g.Vh == 0) return hipSuccess;
    if (a.kind == 0)
        hipLaunchKernelGGL(force_lk_kernel<0>, dim3(link_blocks(a.g)), dim3(kLinkBlock), 0, s, a);
    else
        hipLaunchKernelGGL(force_lk_kernel<1>, dim3(link_blocks(a.g)), dim3(kLinkBlock), 0, s, a);
    return hipGetLastError();
}

}  // namespace tmh
