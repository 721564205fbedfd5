// Gauge-link derivative ("fermionic derivative") of L = Re <X, H Y> for the
// hopping matrix H between checkerboards, accumulated per link in FP64.
//
// Every link of the lattice sits in exactly one term of H: a link leaving a
// site of the output parity in the forward term of that site, a link leaving
// a site of the input parity in the backward term of its forward neighbour.
// One thread owns one site and its 4 links, so every link has one writer and
// no atomics are needed.  For the term of link U = U_mu(l):
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
// the spinors, which four threads read.
constexpr int kOnce = 2;

// Grid: 2 * nb workgroups, remapped so that each XCD owns one contiguous
// range of (parity, site block) pairs: both parities of a range of sites
// and their neighbours then share that XCD's L2.  Registers are held to
// 168 for three waves per SIMD (measured 4 % faster than two).
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3, 8))) force_kernel(ForceArgs a) {
    const int vb = xcd_remap(blockIdx.x, gridDim.x);
    const int p = vb & 1;       // parity of the link sites of this workgroup
    const int i = (vb >> 1) * kBlock + threadIdx.x;
    if (i >= a.g.Vh) return;
    int c[4], lex;
    site_coords(a.g, i, p, c, lex);
    const bool forward = p == a.pout;
    const int S = a.g.S;
    // the field taken at the link's own site
    cx<double> own[4][3];
    const double2* own_f = forward ? a.X : a.Y;
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int k = 0; k < 3; ++k) own[s][k] = bload<double>(own_f + (int64_t)(3 * s + k) * S, S, i);
    int stride = 1;
#pragma unroll
    for (int mu = 3; mu >= 0; --mu) {
        const int Lm = a.g.L[mu];
        const bool wrap = c[mu] == Lm - 1;
        const int j = (wrap ? lex - (Lm - 1) * stride : lex + stride) >> 1;
        stride *= Lm;
        // the field taken at the forward neighbour l + mu
        cx<double> nb[4][3];
        const double2* nb_f = forward ? a.Y : a.X;
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int k = 0; k < 3; ++k) nb[s][k] = bload<double>(nb_f + (int64_t)(3 * s + k) * S, S, j);
        const cx<double>(&x)[4][3] = forward ? own : nb;
        const cx<double>(&y)[4][3] = forward ? nb : own;
        // phi = (1 -/+ gamma_mu) y through the half-spinor h = y_up -/+ e_mu y_dn
        cx<double> phi[4][3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            cx<double> e0, e1, f0, f1;
            switch (mu) {
                case 0: e_lower<double, 0>(y[2][k], y[3][k], e0, e1); break;
                case 1: e_lower<double, 1>(y[2][k], y[3][k], e0, e1); break;
                case 2: e_lower<double, 2>(y[2][k], y[3][k], e0, e1); break;
                default: e_lower<double, 3>(y[2][k], y[3][k], e0, e1); break;
            }
            if (forward) {
                phi[0][k] = y[0][k] - e0;
                phi[1][k] = y[1][k] - e1;
            } else {
                phi[0][k] = y[0][k] + e0;
                phi[1][k] = y[1][k] + e1;
            }
            switch (mu) {
                case 0: edag<double, 0>(phi[0][k], phi[1][k], f0, f1); break;
                case 1: edag<double, 1>(phi[0][k], phi[1][k], f0, f1); break;
                case 2: edag<double, 2>(phi[0][k], phi[1][k], f0, f1); break;
                default: edag<double, 3>(phi[0][k], phi[1][k], f0, f1); break;
            }
            // lower spins: -e^+ h for (1 - gamma), +e^+ h for (1 + gamma)
            phi[2][k] = forward ? mk<double>(-f0.re, -f0.im) : f0;
            phi[3][k] = forward ? mk<double>(-f1.re, -f1.im) : f1;
        }
        // W = kappa eta sum_s phi_s (c_s x_s)^+
        cx<double> eta = mk<double>(a.kappa, 0.0);
        if (wrap) eta = mk<double>(a.kappa * a.ph_re[mu], (forward ? a.kappa : -a.kappa) * a.ph_im[mu]);
        cx<double> W[3][3];
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int q = 0; q < 3; ++q) W[r][q] = mk<double>(0, 0);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const cx<double> cs = mk<double>(a.cx_re[s >> 1], a.cx_im[s >> 1]);
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const cx<double> xq = cs * x[s][q];  // W_rq += phi_r conj(xq)
#pragma unroll
                for (int r = 0; r < 3; ++r) W[r][q] += cmul(xq, phi[s][r]);
            }
        }
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int q = 0; q < 3; ++q) W[r][q] = eta * W[r][q];
        const double2* lk = a.gauge + ((int64_t)(p * 4 + mu) * 9) * S;
        double2* fo = a.force + ((int64_t)(p * 4 + mu) * 9) * S;
        cx<double> out[3][3];
        if (a.kind == 0) {
            cx<double> u[3][3];
#pragma unroll
            for (int k = 0; k < 9; ++k) u[k / 3][k % 3] = bload<double, kOnce>(lk + (int64_t)k * S, S, i);
            cx<double> M[3][3];
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    if (forward)  // U W
                        M[r][q] = u[r][0] * W[0][q] + u[r][1] * W[1][q] + u[r][2] * W[2][q];
                    else {        // -W U^+
                        const cx<double> t = W[r][0] * mk<double>(u[q][0].re, -u[q][0].im) +
                                             W[r][1] * mk<double>(u[q][1].re, -u[q][1].im) +
                                             W[r][2] * mk<double>(u[q][2].re, -u[q][2].im);
                        M[r][q] = mk<double>(-t.re, -t.im);
                    }
                }
            // TA(M) = (M - M^+)/2 - tr(M - M^+)/6
            const double tr_im = (M[0][0].im + M[1][1].im + M[2][2].im) / 3.0;
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    out[r][q] = mk<double>(0.5 * (M[r][q].re - M[q][r].re), 0.5 * (M[r][q].im + M[q][r].im));
                    if (r == q) out[r][q].im -= tr_im;
                }
        } else {
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
                for (int q = 0; q < 3; ++q)
                    out[r][q] = forward ? mk<double>(W[q][r].re, -W[q][r].im) : W[r][q];
        }
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            const cx<double> f = bload<double, kOnce>(fo + (int64_t)k * S, S, i);
            const cx<double> o = out[k / 3][k % 3];
            bstore<double, kOnce>(fo + (int64_t)k * S, S, i, mk<double>(f.re + a.coeff * o.re, f.im + a.coeff * o.im));
        }
    }
}

// ----------------------------------------------------- two bilinears at once
//
// The force of Re <chi, Qhat psi> is the sum of the derivatives of two
// bilinears, one through H_oe and one through H_eo.  Every link sits in one
// term of each; the kernel below forms both terms of a link and adds their
// sum to the force in one read-modify-write, where two launches of
// force_kernel read and write every force entry twice.

// W = kappa eta sum_s phi_s (c_{s/2} x_s)^+, phi = (1 -/+ gamma_mu) y.
template <int MU>
__device__ __forceinline__ void term_w(cx<double> (&W)[3][3], const cx<double> (&x)[4][3],
                                       const cx<double> (&y)[4][3], bool forward, cx<double> eta,
                                       const ForceArgs& t) {
    cx<double> phi[4][3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        cx<double> e0, e1, f0, f1;
        e_lower<double, MU>(y[2][k], y[3][k], e0, e1);
        if (forward) {
            phi[0][k] = y[0][k] - e0;
            phi[1][k] = y[1][k] - e1;
        } else {
            phi[0][k] = y[0][k] + e0;
            phi[1][k] = y[1][k] + e1;
        }
        edag<double, MU>(phi[0][k], phi[1][k], f0, f1);
        phi[2][k] = forward ? mk<double>(-f0.re, -f0.im) : f0;
        phi[3][k] = forward ? mk<double>(-f1.re, -f1.im) : f1;
    }
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int q = 0; q < 3; ++q) W[r][q] = mk<double>(0, 0);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const cx<double> cs = mk<double>(t.cx_re[s >> 1], t.cx_im[s >> 1]);
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const cx<double> xq = cs * x[s][q];
#pragma unroll
            for (int r = 0; r < 3; ++r) W[r][q] += cmul(xq, phi[s][r]);
        }
    }
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int q = 0; q < 3; ++q) W[r][q] = eta * W[r][q];
}

// out += coeff * (TA(M) | Euclidean gradient) of one term of the link u.
__device__ __forceinline__ void term_out(cx<double> (&out)[3][3], const cx<double> (&W)[3][3],
                                         const cx<double> (&u)[3][3], bool forward, int kind, double coeff) {
    if (kind == 0) {
        cx<double> M[3][3];
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                if (forward)  // U W
                    M[r][q] = u[r][0] * W[0][q] + u[r][1] * W[1][q] + u[r][2] * W[2][q];
                else {        // -W U^+
                    const cx<double> t = W[r][0] * mk<double>(u[q][0].re, -u[q][0].im) +
                                         W[r][1] * mk<double>(u[q][1].re, -u[q][1].im) +
                                         W[r][2] * mk<double>(u[q][2].re, -u[q][2].im);
                    M[r][q] = mk<double>(-t.re, -t.im);
                }
            }
        const double tr_im = (M[0][0].im + M[1][1].im + M[2][2].im) / 3.0;
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                cx<double> o = mk<double>(0.5 * (M[r][q].re - M[q][r].re), 0.5 * (M[r][q].im + M[q][r].im));
                if (r == q) o.im -= tr_im;
                out[r][q] += mk<double>(coeff * o.re, coeff * o.im);
            }
    } else {
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const cx<double> o = forward ? mk<double>(W[q][r].re, -W[q][r].im) : W[r][q];
                out[r][q] += mk<double>(coeff * o.re, coeff * o.im);
            }
    }
}

template <int MU>
__device__ __forceinline__ void force2_link(const ForceArgs& a, const ForceArgs& b, int p, int i, int j, bool wrap) {
    const int S = a.g.S;
    cx<double> u[3][3];
    const double2* lk = a.gauge + ((int64_t)(p * 4 + MU) * 9) * S;
    if (a.kind == 0) {
#pragma unroll
        for (int k = 0; k < 9; ++k) u[k / 3][k % 3] = bload<double, kOnce>(lk + (int64_t)k * S, S, i);
    }
    cx<double> out[3][3];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int q = 0; q < 3; ++q) out[r][q] = mk<double>(0, 0);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const ForceArgs& t = k == 0 ? a : b;
        const bool forward = p == t.pout;
        // x at the output-parity end of the term, y at the input-parity end
        const double2* xf = t.X;
        const double2* yf = t.Y;
        const int ix = forward ? i : j, iy = forward ? j : i;
        cx<double> x[4][3], y[4][3];
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                x[s][c] = bload<double>(xf + (int64_t)(3 * s + c) * S, S, ix);
                y[s][c] = bload<double>(yf + (int64_t)(3 * s + c) * S, S, iy);
            }
        cx<double> eta = mk<double>(a.kappa, 0.0);
        if (wrap) eta = mk<double>(a.kappa * a.ph_re[MU], (forward ? a.kappa : -a.kappa) * a.ph_im[MU]);
        cx<double> W[3][3];
        term_w<MU>(W, x, y, forward, eta, t);
        term_out(out, W, u, forward, a.kind, t.coeff);
    }
    double2* fo = a.force + ((int64_t)(p * 4 + MU) * 9) * S;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const cx<double> f = bload<double, kOnce>(fo + (int64_t)k * S, S, i);
        const cx<double> o = out[k / 3][k % 3];
        bstore<double, kOnce>(fo + (int64_t)k * S, S, i, mk<double>(f.re + o.re, f.im + o.im));
    }
}

__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2, 8)))
force2_kernel(ForceArgs a, ForceArgs b) {
    const int vb = xcd_remap(blockIdx.x, gridDim.x);
    const int p = vb & 1;
    const int i = (vb >> 1) * kBlock + threadIdx.x;
    if (i >= a.g.Vh) return;
    int c[4], lex;
    site_coords(a.g, i, p, c, lex);
    int stride = 1;
    int jn[4];
    bool wr[4];
#pragma unroll
    for (int mu = 3; mu >= 0; --mu) {
        const int Lm = a.g.L[mu];
        wr[mu] = c[mu] == Lm - 1;
        jn[mu] = (wr[mu] ? lex - (Lm - 1) * stride : lex + stride) >> 1;
        stride *= Lm;
    }
    force2_link<3>(a, b, p, i, jn[3], wr[3]);
    force2_link<2>(a, b, p, i, jn[2], wr[2]);
    force2_link<1>(a, b, p, i, jn[1], wr[1]);
    force2_link<0>(a, b, p, i, jn[0], wr[0]);
}

}  // namespace

hipError_t launch_force2(const ForceArgs& a, const ForceArgs& b, hipStream_t s) {
    const int nb = (a.g.Vh + kBlock - 1) / kBlock;
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(force2_kernel, dim3(2 * nb), dim3(kBlock), 0, s, a, b);
    return hipGetLastError();
}

hipError_t launch_force(const ForceArgs& a, hipStream_t s) {
    const int nb = (a.g.Vh + kBlock - 1) / kBlock;
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(force_kernel, dim3(2 * nb), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

}  // namespace tmh
