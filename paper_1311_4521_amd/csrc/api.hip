// C-ABI of libtmhop (declared in include/tmhop.h): lattice handle, argument
// checks, the hopping-matrix and twisted-mass launchers, the CG drivers.
#include <math.h>
#include <stdio.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "../../include/tmhop.h"
#include "api_internal.h"
#include "common.h"
#include "kernels.h"

using tmh::Geo;
using tmh::HopArgs;

struct tmh_lattice {
    int dims[4];
    int device;
    hipStream_t stream;
    Geo g;
    int npartial;           // partial-sum slots (max of hop and BLAS grids)
    double* partial;        // reduction partials
    double* scal;           // CG scalars (tmh::CgScal)
    int* flags;             // {done, iterations}
    double* h_scal;         // pinned host mirror of scal
    int* h_flags;           // pinned host mirror of flags
    void* even[3];          // intermediate even field per base precision (Qtm), prec_slot order
    void* even2;            // second FP64 even field (force chain, full solve)
    void* odd_rhs[2];       // FP64 odd fields of the full-lattice solve
    void* mrhs[5];          // multi-RHS CG fields r, p, v, q (odd) and the even te, FP64
    int mrhs_cap;           // right-hand sides mrhs[] can hold
    int tuned[2][17];       // autotuned batch tile shape per (precision, nrhs <= 16), -1: none
    int xgroup;             // hop traversal: x values per group (0: even-odd order)
    bool xtuned[6];         // traversal tuned for launches of one storage code ...
    int xgroup_code[6];     // ... and its value (tmh_autotune_hop)
    double2* v64[4];        // FP64 CG vectors r, p, v, q
    void* vlow[2][5];       // inner CG vectors r, p, v, q, d of the mixed solve: [0] FP32, [1] FP16
    void* glow[2];          // FP32 / FP16 copy of the links for the mixed-precision inner solve
    double2* gauge64r12;    // FP64 two-row copy of the links for the TMH_F64_R12 solve
    // launch timing (tmh_profile_*): event pairs around hopping-matrix launches
    struct EventPair {
        hipEvent_t start, stop;
        int kind;
    };
    bool prof_on;
    std::vector<EventPair> prof_pending;
    std::vector<EventPair> prof_free;
    double prof_ms[TMH_PROFILE_KINDS];
    long long prof_count[TMH_PROFILE_KINDS];
    long long prof_skipped[TMH_PROFILE_KINDS];  // launches that found the CG done and returned at once
};

namespace {

struct DeviceGuard {
    int old = -1;
    bool ok = false;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&old) != hipSuccess) old = -1;
        ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard() {
        if (old >= 0) (void)hipSetDevice(old);
    }
};

#define TMH_TRY_HIP(expr)                            \
    do {                                             \
        if ((expr) != hipSuccess) return TMH_ERR_HIP; \
    } while (0)

#define TMH_TRY(expr)                   \
    do {                                \
        tmh_status st__ = (expr);       \
        if (st__ != TMH_OK) return st__; \
    } while (0)

// A precision code is a storage word (FP64, FP32, or FP16 with FP32
// arithmetic) and a link storage format (9 entries, or two rows for the _R12
// codes); spinors of an _R12 code are those of its base precision.
bool prec_valid(tmh_prec p) { return p >= TMH_F64 && p <= TMH_F16_R12; }
tmh_prec base_prec(tmh_prec p) {
    if (p == TMH_F64 || p == TMH_F64_R12) return TMH_F64;
    if (p == TMH_F32 || p == TMH_F32_R12) return TMH_F32;
    return TMH_F16;
}
int link_format(tmh_prec p) { return (p == TMH_F64_R12 || p == TMH_F32_R12 || p == TMH_F16_R12) ? 1 : 0; }
int link_comps(tmh_prec p) { return link_format(p) ? 6 : 9; }
size_t word_bytes(tmh_prec p) {
    if (!prec_valid(p)) return 0;
    const tmh_prec b = base_prec(p);
    return b == TMH_F64 ? 16 : (b == TMH_F32 ? 8 : 4);
}
// Slot of a base precision in per-precision scratch arrays.
int prec_slot(tmh_prec p) {
    const tmh_prec b = base_prec(p);
    return b == TMH_F64 ? 0 : (b == TMH_F32 ? 1 : 2);
}
// The precision code of storage P with link format lf.
template <typename P> int prec_code(int lf);
template <> int prec_code<double>(int lf) { return lf ? TMH_F64_R12 : TMH_F64; }
template <> int prec_code<float>(int lf) { return lf ? TMH_F32_R12 : TMH_F32; }
template <> int prec_code<tmh::half_t>(int lf) { return lf ? TMH_F16_R12 : TMH_F16; }
// Calls f with a value of the storage type of p's base precision.
template <typename F> tmh_status dispatch(tmh_prec p, F&& f) {
    const tmh_prec b = base_prec(p);
    if (b == TMH_F64) return f(double{});
    if (b == TMH_F32) return f(float{});
    return f(tmh::half_t{});
}

bool overlap(const void* a, size_t na, const void* b, size_t nb) {
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + nb && y < x + na;
}

tmh_status ensure(void** p, size_t bytes) {
    if (*p) return TMH_OK;
    if (hipMalloc(p, bytes) != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return TMH_ERR_NOMEM;
    }
    return TMH_OK;
}

// The x-group traversal of the hop kernel applies when the geometry tiles
// exactly: 64-site units fill whole (t, x) planes, every XCD owns whole
// time-slices and a whole number of workgroups, and the group divides LX.
// The x-slab traversal needs whole planes, LX a multiple of 8 and a whole
// number of workgroups per XCD.
static_assert(tmh::kXSlab == TMH_TRAVERSAL_XSLAB, "the kernels and the ABI name the x-slab order alike");
static_assert(tmh::kTMarch0 - 4 == TMH_TRAVERSAL_TMARCH(4), "the kernels and the ABI name the t-march alike");
// Steps per workgroup of a t-march traversal code, 0 for other codes.
int tmarch_steps(int code) { return code < tmh::kTMarch0 ? tmh::kTMarch0 - code : 0; }
// The t-march needs whole tiles of kHopThreads pairs per time-slice and a
// whole number of ranges of `steps` time-slices.
bool tmarch_ok(const tmh_lattice* l, int steps) {
    const int64_t slice = (int64_t)l->dims[1] * l->dims[2] * l->dims[3] / 2;
    return steps >= 1 && steps <= l->dims[0] && l->dims[0] % steps == 0 && slice % tmh::kHopThreads == 0;
}
bool xgroup_ok(const tmh_lattice* l, int xg) {
    if (tmarch_steps(xg) > 0) return tmarch_ok(l, tmarch_steps(xg));
    const int plane = l->dims[2] * l->dims[3] / 2;
    const bool tiles = plane % 64 == 0 && l->g.Vh % (64 * 8) == 0 &&
                       (l->g.Vh / 64 / 8) % (tmh::kHopThreads / 64) == 0;
    if (xg == tmh::kXSlab) return tiles && l->dims[1] % 8 == 0;
    return xg > 0 && tiles && l->dims[0] % 8 == 0 && l->dims[1] % xg == 0;
}

// Default: the largest group of x values whose sites (xg LY LZ / 2 per
// time-slice) stay within 8192, i.e. about half the sites one XCD holds in
// flight; 0 (even-odd order) when the geometry does not tile.
int default_xgroup(const tmh_lattice* l) {
    const int plane = l->dims[2] * l->dims[3] / 2;
    int best = 0;
    for (int xg = 1; xg <= l->dims[1]; ++xg)
        if (xgroup_ok(l, xg) && (int64_t)xg * plane <= 8192) best = xg;
    return best;
}

#ifndef TMH_SITE_PAD
#define TMH_SITE_PAD 0
#endif
// Site stride of the component arrays: Vh rounded up to 64 sites, plus a pad.
int64_t site_stride(int64_t vh) { return (vh + 63) / 64 * 64 + TMH_SITE_PAD; }

size_t spinor_bytes(const tmh_lattice* l, tmh_prec p) { return (size_t)12 * l->g.S * word_bytes(p); }
size_t gauge_bytes(const tmh_lattice* l, tmh_prec p) {
    return (size_t)8 * link_comps(p) * l->g.S * word_bytes(p);
}

tmh_status even_scratch(tmh_lattice* l, tmh_prec p, void** out) {
    const int k = prec_slot(p);
    TMH_TRY(ensure(&l->even[k], spinor_bytes(l, p)));
    *out = l->even[k];
    return TMH_OK;
}

template <typename R>
HopArgs<R> hop_args(const tmh_lattice* l, int pout, void* out, const void* gauge, const void* in,
                    const double theta[4], int lf = 0) {
    using W = typename tmh::Word<R>::T;
    HopArgs<R> a;
    memset(&a, 0, sizeof a);
    a.out = (W*)out;
    a.in = (const W*)in;
    const W* g = (const W*)gauge;
    const int64_t per_parity = (int64_t)4 * (lf ? 6 : 9) * l->g.S;
    a.gout = g + pout * per_parity;
    a.gin = g + (1 - pout) * per_parity;
    a.g = l->g;
    a.pout = pout;
    a.lf = lf;
    const int code = prec_code<R>(lf);
    const int xg = l->xtuned[code] ? l->xgroup_code[code] : l->xgroup;
    if (tmarch_steps(xg) > 0) {
        if (tmarch_ok(l, tmarch_steps(xg))) {
            a.tm_steps = tmarch_steps(xg);
            a.tm_slice = l->dims[1] * l->dims[2] * l->dims[3] / 2;
            a.tm_nw = a.tm_slice / tmh::kHopThreads;
        }
    } else if (xgroup_ok(l, xg)) {
        a.xgroup = xg;
        a.nyb = l->dims[2] * l->dims[3] / 2 / 64;
        a.nt = l->dims[0] / 8;
    }
    for (int m = 0; m < 4; ++m) {
        a.ph_re[m] = (tmh::real_t<R>)cos(M_PI * theta[m]);
        a.ph_im[m] = (tmh::real_t<R>)sin(M_PI * theta[m]);
    }
    return a;
}

// Folds the durations of all recorded event pairs into the totals (waits).
tmh_status prof_flush(tmh_lattice* l) {
    for (auto& e : l->prof_pending) {
        if (hipEventSynchronize(e.stop) != hipSuccess) return TMH_ERR_HIP;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, e.start, e.stop) != hipSuccess) return TMH_ERR_HIP;
        l->prof_ms[e.kind] += ms;
        l->prof_count[e.kind] += 1;
        l->prof_free.push_back(e);
    }
    l->prof_pending.clear();
    return TMH_OK;
}

constexpr size_t kMaxPendingEvents = 1024;

// Launches one hopping-matrix kernel; with timing on, brackets it with a pair
// of events on the handle's stream.
template <typename R>
hipError_t hop_launch(tmh_lattice* l, const HopArgs<R>& a, int mode) {
    if (!l->prof_on) return tmh::launch_hop<R>(a, mode, l->stream);
    if (l->prof_pending.size() >= kMaxPendingEvents && prof_flush(l) != TMH_OK) return hipErrorUnknown;
    tmh_lattice::EventPair e;
    if (!l->prof_free.empty()) {
        e = l->prof_free.back();
        l->prof_free.pop_back();
    } else {
        if (hipEventCreate(&e.start) != hipSuccess) return hipErrorUnknown;
        if (hipEventCreate(&e.stop) != hipSuccess) {
            (void)hipEventDestroy(e.start);
            return hipErrorUnknown;
        }
    }
    e.kind = 4 * prec_code<R>(a.lf) + (mode < 3 ? mode : 3);
    hipError_t err = hipEventRecord(e.start, l->stream);
    if (err == hipSuccess) err = tmh::launch_hop<R>(a, mode, l->stream);
    if (err == hipSuccess) err = hipEventRecord(e.stop, l->stream);
    if (err != hipSuccess) {
        l->prof_free.push_back(e);
        return err;
    }
    l->prof_pending.push_back(e);
    return hipSuccess;
}

// Qhat(sign) in -> out through the even scratch `te`; with `partial` the
// second launch also writes the |out|^2 partials.
template <typename R>
tmh_status qtm_launch(tmh_lattice* l, void* out, const void* gauge, const void* in, void* te, double kappa,
                      double mu, const double theta[4], int sign, double* partial, const int* done, int lf = 0,
                      bool timed = true) {
    const double mt = 2.0 * kappa * mu * sign;
    const double D = 1.0 + mt * mt;
    HopArgs<R> a = hop_args<R>(l, 0, te, gauge, in, theta, lf);
    a.done = done;
    // A^-1 = (1 - i mt gamma_5)/D: upper spins (1 - i mt)/D, lower (1 + i mt)/D
    a.c_re[0] = (tmh::real_t<R>)(kappa / D);
    a.c_im[0] = (tmh::real_t<R>)(-kappa * mt / D);
    a.c_re[1] = (tmh::real_t<R>)(kappa / D);
    a.c_im[1] = (tmh::real_t<R>)(kappa * mt / D);
    TMH_TRY_HIP(timed ? hop_launch<R>(l, a, 0) : tmh::launch_hop<R>(a, 0, l->stream));
    HopArgs<R> b = hop_args<R>(l, 1, out, gauge, te, theta, lf);
    b.done = done;
    b.aux = (const typename tmh::Word<R>::T*)in;
    b.partial = partial;
    // gamma_5 [A in - kappa H te]: upper (1 + i mt) in - kappa H te,
    // lower kappa H te - (1 - i mt) in
    b.c_re[0] = (tmh::real_t<R>)(-kappa);
    b.c_re[1] = (tmh::real_t<R>)kappa;
    b.d_re[0] = (tmh::real_t<R>)1;
    b.d_im[0] = (tmh::real_t<R>)mt;
    b.d_re[1] = (tmh::real_t<R>)-1;
    b.d_im[1] = (tmh::real_t<R>)mt;
    const int mode = partial ? 2 : 1;
    TMH_TRY_HIP(timed ? hop_launch<R>(l, b, mode) : tmh::launch_hop<R>(b, mode, l->stream));
    return TMH_OK;
}

// force += coeff * P(dRe<X, H Y>/dU), X on parity pout taken as c_{s/2} X_s.
tmh::ForceArgs force_args(tmh_lattice* l, int pout, void* force, const void* gauge, const void* X, const void* Y,
                          double kappa, const double theta[4], double coeff, int kind, double cu_re, double cu_im,
                          double cd_re, double cd_im) {
    tmh::ForceArgs f;
    memset(&f, 0, sizeof f);
    f.force = (double2*)force;
    f.gauge = (const double2*)gauge;
    f.X = (const double2*)X;
    f.Y = (const double2*)Y;
    f.g = l->g;
    f.pout = pout;
    f.kind = kind;
    f.kappa = kappa;
    f.coeff = coeff;
    for (int m = 0; m < 4; ++m) {
        f.ph_re[m] = cos(M_PI * theta[m]);
        f.ph_im[m] = sin(M_PI * theta[m]);
    }
    f.cx_re[0] = cu_re;
    f.cx_im[0] = cu_im;
    f.cx_re[1] = cd_re;
    f.cx_im[1] = cd_im;
    return f;
}

hipError_t force_launch(tmh_lattice* l, int pout, void* force, const void* gauge, const void* X, const void* Y,
                        double kappa, const double theta[4], double coeff, int kind, double cu_re, double cu_im,
                        double cd_re, double cd_im) {
    return tmh::launch_force(
        force_args(l, pout, force, gauge, X, Y, kappa, theta, coeff, kind, cu_re, cu_im, cd_re, cd_im), l->stream);
}

// The second operator of a CG iteration: q = Qhat(-) v, never stored; the
// last launch applies r -= alpha q (alpha from the device scalars), with x
// non-null also x += alpha p, and writes the |r|^2 partials.
template <typename R>
tmh_status qtm_update(tmh_lattice* l, void* x, void* r, const void* p, const void* gauge, const void* v, void* te,
                      double kappa, double mu, const double theta[4], double* partial, const int* done,
                      int lf) {
    using W = typename tmh::Word<R>::T;
    const double mt = -2.0 * kappa * mu;
    const double D = 1.0 + mt * mt;
    HopArgs<R> a = hop_args<R>(l, 0, te, gauge, v, theta, lf);
    a.done = done;
    a.c_re[0] = (tmh::real_t<R>)(kappa / D);
    a.c_im[0] = (tmh::real_t<R>)(-kappa * mt / D);
    a.c_re[1] = (tmh::real_t<R>)(kappa / D);
    a.c_im[1] = (tmh::real_t<R>)(kappa * mt / D);
    // alpha = |r|^2 / (p, A p) from the norm partials of the hop before
    a.apart = partial;
    a.napart = tmh::hop_blocks(l->g);
    a.ascal = l->scal;
    TMH_TRY_HIP(hop_launch<R>(l, a, 0));
    HopArgs<R> b = hop_args<R>(l, 1, nullptr, gauge, te, theta, lf);
    b.done = done;
    b.aux = (const W*)v;
    b.partial = partial;
    b.rio = (W*)r;
    b.xio = (W*)x;
    b.pin = (const W*)p;
    b.scal = l->scal;
    b.c_re[0] = (tmh::real_t<R>)(-kappa);
    b.c_re[1] = (tmh::real_t<R>)kappa;
    b.d_re[0] = (tmh::real_t<R>)1;
    b.d_im[0] = (tmh::real_t<R>)mt;
    b.d_re[1] = (tmh::real_t<R>)-1;
    b.d_im[1] = (tmh::real_t<R>)mt;
    TMH_TRY_HIP(hop_launch<R>(l, b, x ? 4 : 3));
    return TMH_OK;
}

tmh_status check_lat(const tmh_lattice* l) { return l ? TMH_OK : TMH_ERR_ARG; }

tmh_status check_prec(tmh_prec p) { return prec_valid(p) ? TMH_OK : TMH_ERR_UNSUPPORTED; }
// Entry points that take full 9-entry links only.
tmh_status check_prec_full(tmh_prec p) { return (p == TMH_F64 || p == TMH_F32) ? TMH_OK : TMH_ERR_UNSUPPORTED; }

tmh_status check_theta(const double* theta) {
    if (!theta) return TMH_ERR_ARG;
    for (int m = 0; m < 4; ++m)
        if (!isfinite(theta[m])) return TMH_ERR_ARG;
    return TMH_OK;
}

// Host copy of n device doubles / ints from the scalar area (waits).
tmh_status read_scalars(tmh_lattice* l) {
    TMH_TRY_HIP(hipMemcpyAsync(l->h_scal, l->scal, sizeof(double) * tmh::kNScal, hipMemcpyDeviceToHost,
                               l->stream));
    TMH_TRY_HIP(hipMemcpyAsync(l->h_flags, l->flags, sizeof(int) * 2, hipMemcpyDeviceToHost, l->stream));
    TMH_TRY_HIP(hipStreamSynchronize(l->stream));
    return TMH_OK;
}

template <typename R>
tmh_status reduce_dot(tmh_lattice* l, double* result, const void* a, const void* b) {
    using W = typename tmh::Word<R>::T;
    TMH_TRY_HIP(tmh::launch_dot_partial<R>(l->partial, (const W*)a, (const W*)b, l->g, nullptr, l->stream));
    TMH_TRY_HIP(tmh::launch_reduce(l->scal + tmh::kNorm, l->partial, tmh::blas_blocks(l->g), nullptr,
                                   l->stream));
    TMH_TRY(read_scalars(l));
    *result = l->h_scal[tmh::kNorm];
    return TMH_OK;
}

// r = b - Qhat(-) Qhat(+) x in precision R, and |r|^2 (waits).
template <typename R>
tmh_status true_residual(tmh_lattice* l, void* r, const void* b, const void* x, void* v, void* q, void* te,
                         const void* gauge, double kappa, double mu, const double theta[4], double* rr,
                         int lf = 0) {
    using W = typename tmh::Word<R>::T;
    TMH_TRY(qtm_launch<R>(l, v, gauge, x, te, kappa, mu, theta, +1, nullptr, nullptr, lf));
    TMH_TRY(qtm_launch<R>(l, q, gauge, v, te, kappa, mu, theta, -1, nullptr, nullptr, lf));
    TMH_TRY_HIP(tmh::launch_sub_norm<R>((W*)r, (const W*)b, (const W*)q, l->partial, l->g, l->stream));
    TMH_TRY_HIP(tmh::launch_reduce(l->scal + tmh::kNorm, l->partial, tmh::blas_blocks(l->g), nullptr,
                                   l->stream));
    TMH_TRY(read_scalars(l));
    *rr = l->h_scal[tmh::kNorm];
    return TMH_OK;
}

// The first residual of a solve: r = b when the start vector is zero (the
// usual case, which then needs no operator application), else b - A x.
tmh_status initial_residual(tmh_lattice* l, void* r, const void* b, const void* x, void* v, void* q, void* te,
                            const void* gauge, double kappa, double mu, const double theta[4], double bb,
                            double* rr, int lf = 0) {
    double xx;
    TMH_TRY(reduce_dot<double>(l, &xx, x, x));
    if (xx != 0.0) return true_residual<double>(l, r, b, x, v, q, te, gauge, kappa, mu, theta, rr, lf);
    TMH_TRY_HIP(tmh::launch_copy<double>((double2*)r, (const double2*)b, l->g, l->stream));
    *rr = bb;
    return TMH_OK;
}

// CG recursion on A x = r0 where x holds the start vector and r holds
// r0 - A x.  Iterates until |r|^2 <= stop or max_iter; scalars stay on the
// device, the host looks at the flags once every kChunk iterations.
constexpr int kChunk = 8;

template <typename R>
tmh_status cg_recursion(tmh_lattice* l, void* x, void* r, void* p, void* v, void* q, void* te, const void* gauge,
                        double kappa, double mu, const double theta[4], double stop, int max_iter, int* iters,
                        int lf = 0) {
    using W = typename tmh::Word<R>::T;
    const int nb_hop = tmh::hop_blocks(l->g), nb_blas = tmh::blas_blocks(l->g);
    // rr = |r|^2 into scal, flags reset
    TMH_TRY_HIP(tmh::launch_dot_partial<R>(l->partial, (const W*)r, (const W*)r, l->g, nullptr, l->stream));
    TMH_TRY_HIP(tmh::launch_cg_init(l->scal, l->partial, nb_blas, l->flags, stop, l->stream));
    TMH_TRY_HIP(tmh::launch_copy<R>((W*)p, (const W*)r, l->g, l->stream));
    *iters = 0;
    if (max_iter <= 0) return TMH_OK;
    int enqueued = 0;
    for (;;) {
        enqueued += kChunk;
        for (int k = 0; k < kChunk; ++k) {
            // v = Qhat(+) p with |v|^2 = (p, A p)
            TMH_TRY(qtm_launch<R>(l, v, gauge, p, te, kappa, mu, theta, +1, l->partial, l->flags, lf));
            // q = Qhat(-) v = A p, fused with r -= alpha q and |r|^2 (its
            // first hop also sets alpha from the partials of (p, A p)).  The
            // solution update x += alpha p goes with the last hop in FP64,
            // with the direction update p = r + beta p in FP32 and FP16:
            // measured, each is the faster placement for its precision.
            if constexpr (sizeof(W) == 16) {
                TMH_TRY(qtm_update<R>(l, x, r, p, gauge, v, te, kappa, mu, theta, l->partial, l->flags, lf));
                TMH_TRY_HIP(tmh::launch_cg_beta(l->scal, l->partial, nb_hop, l->flags, max_iter, l->stream));
                TMH_TRY_HIP(tmh::launch_cg_p<R>((W*)p, (const W*)r, l->scal, l->g, l->flags, l->stream));
            } else {
                TMH_TRY(qtm_update<R>(l, nullptr, r, nullptr, gauge, v, te, kappa, mu, theta, l->partial, l->flags,
                                      lf));
                TMH_TRY_HIP(tmh::launch_cg_beta(l->scal, l->partial, nb_hop, l->flags, max_iter, l->stream));
                TMH_TRY_HIP(tmh::launch_cg_px<R>((W*)p, (W*)x, (const W*)r, l->scal, l->g, l->flags,
                                                 enqueued - kChunk + k, l->stream));
            }
        }
        TMH_TRY(read_scalars(l));
        if (l->h_flags[0]) break;
    }
    *iters = l->h_flags[1];
    if (l->prof_on) {
        // iterations enqueued after convergence ran as empty launches: two
        // A^-1 stores, one twist + norm and one twist + update each
        const long long skipped = enqueued - *iters;
        const int base = 4 * prec_code<R>(lf);
        l->prof_skipped[base + 0] += 2 * skipped;
        l->prof_skipped[base + 2] += skipped;
        l->prof_skipped[base + 3] += skipped;
    }
    return TMH_OK;
}

tmh_status alloc_cg64(tmh_lattice* l) {
    for (int k = 0; k < 4; ++k) TMH_TRY(ensure((void**)&l->v64[k], spinor_bytes(l, TMH_F64)));
    void* te;
    return even_scratch(l, TMH_F64, &te);
}

// Precision of the inner solve of storage P (FP32 or FP16) and its slot.
template <typename P> constexpr tmh_prec low_prec() { return sizeof(P) == 4 ? TMH_F32 : TMH_F16; }
template <typename P> constexpr int low_slot() { return sizeof(P) == 4 ? 0 : 1; }

template <typename P> tmh_status alloc_low(tmh_lattice* l) {
    constexpr tmh_prec lp = low_prec<P>();
    for (int k = 0; k < 5; ++k) TMH_TRY(ensure(&l->vlow[low_slot<P>()][k], spinor_bytes(l, lp)));
    TMH_TRY(ensure(&l->glow[low_slot<P>()], gauge_bytes(l, lp)));
    void* te;
    return even_scratch(l, lp, &te);
}

// Two-row copies of the links are used where every link's stored third row
// matches the conjugate cross product of its first two to these bounds
// (special unitary links): below the rounding of the entries in the copy's
// precision.  Otherwise all 9 entries are kept.
constexpr double kR12Tol64 = 1e-14;
template <typename P> constexpr double r12_tol() { return sizeof(P) == 4 ? 1e-7 : 1e-4; }

// Largest deviation found by the last compress launch (waits).
tmh_status link_deviation(tmh_lattice* l, double* dev) {
    TMH_TRY_HIP(tmh::launch_reduce_max(l->scal + tmh::kNorm, l->partial, tmh::link_check_blocks(l->g), l->stream));
    TMH_TRY(read_scalars(l));
    *dev = l->h_scal[tmh::kNorm];
    return TMH_OK;
}

// Links for the FP64 recursion: the caller's 9-entry field, or with r12 a
// two-row copy when the links pass the check (*lf = 1).
tmh_status links64(tmh_lattice* l, const void* gauge, bool r12, const void** used, int* lf) {
    *used = gauge;
    *lf = 0;
    if (!r12) return TMH_OK;
    TMH_TRY(ensure((void**)&l->gauge64r12, gauge_bytes(l, TMH_F64_R12)));
    TMH_TRY_HIP(tmh::launch_compress_links<double>(l->gauge64r12, (const double2*)gauge, l->partial, l->g,
                                                   l->stream));
    double dev;
    TMH_TRY(link_deviation(l, &dev));
    if (dev <= kR12Tol64) {
        *used = l->gauge64r12;
        *lf = 1;
    }
    return TMH_OK;
}

// Narrows the FP64 links into the inner solve's copy (storage P): two rows
// with r12 when the links pass the check (*lf = 1), else all 9 entries.
template <typename P> tmh_status links_low(tmh_lattice* l, const void* gauge, bool r12, int* lf) {
    using W = typename tmh::Word<P>::T;
    W* dst = (W*)l->glow[low_slot<P>()];
    *lf = 0;
    if (r12) {
        TMH_TRY_HIP(tmh::launch_compress_links<P>(dst, (const double2*)gauge, l->partial, l->g, l->stream));
        double dev;
        TMH_TRY(link_deviation(l, &dev));
        if (dev <= r12_tol<P>()) return *lf = 1, TMH_OK;
    }
    TMH_TRY_HIP(tmh::launch_narrow<P>(dst, (const double2*)gauge, 72, 1.0, l->g, l->stream));
    return TMH_OK;
}

tmh_status cg_fp64(tmh_lattice* l, void* x, const void* b, const void* gauge, double kappa, double mu,
                   const double theta[4], double tol, int max_iter, int* iters, double* res, bool r12) {
    TMH_TRY(alloc_cg64(l));
    void *r = l->v64[0], *p = l->v64[1], *v = l->v64[2], *q = l->v64[3], *te = l->even[TMH_F64];
    double bb;
    TMH_TRY(reduce_dot<double>(l, &bb, b, b));
    *iters = 0;
    *res = 0.0;
    if (bb == 0.0) {
        TMH_TRY_HIP(tmh::launch_zero<double>((double2*)x, l->g, l->stream));
        TMH_TRY_HIP(hipStreamSynchronize(l->stream));
        return TMH_OK;
    }
    const double stop = tol * tol * bb;
    const void* gr;
    int lf;
    TMH_TRY(links64(l, gauge, r12, &gr, &lf));
    double rr;
    TMH_TRY(initial_residual(l, r, b, x, v, q, te, gr, kappa, mu, theta, bb, &rr, lf));
    int total = 0;
    for (int restart = 0;; ++restart) {
        *res = sqrt(rr / bb);
        if (*res <= tol) return *iters = total, TMH_OK;
        if (restart > 3 || total >= max_iter) break;
        int it = 0;
        TMH_TRY(cg_recursion<double>(l, x, r, p, v, q, te, gr, kappa, mu, theta, stop, max_iter - total, &it, lf));
        total += it;
        TMH_TRY(true_residual<double>(l, r, b, x, v, q, te, gr, kappa, mu, theta, &rr, lf));
    }
    *iters = total;
    return TMH_ERR_NOT_CONVERGED;
}

// Defect correction: FP64 true residual and solution update, inner CG in
// FP32 or in FP16 storage.  The inner target is the remaining factor, but no
// tighter than the inner precision can hold.
#ifndef TMH_INNER_TOL_F16
#define TMH_INNER_TOL_F16 3e-3
#endif
template <typename P> constexpr double inner_tol_min() { return sizeof(P) == 4 ? 1e-5 : TMH_INNER_TOL_F16; }
constexpr int kMaxOuter = 64;
// The inner system is scaled: the residual enters the inner solve scaled to
// unit mean square per real component, so that the recursion's vectors stay
// inside the normal range of FP16 (from 6.1e-5) or FP32 (from 1.2e-38)
// whatever the source's magnitude; the correction is scaled back.
template <typename P>
tmh_status cg_mixed(tmh_lattice* l, void* x, const void* b, const void* gauge, double kappa, double mu,
                    const double theta[4], double tol, int max_iter, int* iters, double* res, bool r12) {
    using W = typename tmh::Word<P>::T;
    TMH_TRY(alloc_cg64(l));
    TMH_TRY(alloc_low<P>(l));
    void *r = l->v64[0], *v = l->v64[2], *q = l->v64[3], *te = l->even[0];
    void** vl = l->vlow[low_slot<P>()];
    W *rl = (W*)vl[0], *pl = (W*)vl[1], *vv = (W*)vl[2], *ql = (W*)vl[3], *dl = (W*)vl[4];
    void* tel = l->even[prec_slot(low_prec<P>())];
    int lf = 0;
    TMH_TRY(links_low<P>(l, gauge, r12, &lf));
    double bb;
    TMH_TRY(reduce_dot<double>(l, &bb, b, b));
    *iters = 0;
    *res = 0.0;
    if (bb == 0.0) {
        TMH_TRY_HIP(tmh::launch_zero<double>((double2*)x, l->g, l->stream));
        TMH_TRY_HIP(hipStreamSynchronize(l->stream));
        return TMH_OK;
    }
    // the FP64 residuals run on the FP64 two-row copy when the links pass
    // its check (the same operator to rounding), else on the caller's links
    const void* g64;
    int lf64;
    TMH_TRY(links64(l, gauge, r12, &g64, &lf64));
    double rr;
    TMH_TRY(initial_residual(l, r, b, x, v, q, te, g64, kappa, mu, theta, bb, &rr, lf64));
    int total = 0;
    for (int outer = 0;; ++outer) {
        *res = sqrt(rr / bb);
        if (*res <= tol) return *iters = total, TMH_OK;
        if (outer >= kMaxOuter || total >= max_iter || !(rr > 0.0)) break;
        double inner = 0.5 * tol / *res;
        if (inner < inner_tol_min<P>()) inner = inner_tol_min<P>();
        const double scale = sqrt(24.0 * l->g.Vh / rr);
        TMH_TRY_HIP(tmh::launch_narrow<P>(rl, (const double2*)r, 12, scale, l->g, l->stream));
        TMH_TRY_HIP(tmh::launch_zero<P>(dl, l->g, l->stream));
        int it = 0;
        // the stop test is relative to the scaled residual, |scale r|^2
        TMH_TRY(cg_recursion<P>(l, dl, rl, pl, vv, ql, tel, l->glow[low_slot<P>()], kappa, mu, theta,
                                inner * inner * scale * scale * rr, max_iter - total, &it, lf));
        total += it;
        TMH_TRY_HIP(tmh::launch_add_widen<P>((double2*)x, dl, 1.0 / scale, l->g, l->stream));
        TMH_TRY(true_residual<double>(l, r, b, x, v, q, te, g64, kappa, mu, theta, &rr, lf64));
    }
    *iters = total;
    return TMH_ERR_NOT_CONVERGED;
}

// Runs the solver that `inner` names.
tmh_status cg_dispatch(tmh_lattice* l, void* x, const void* b, const void* gauge, double kappa, double mu,
                       const double theta[4], double tol, int max_iter, tmh_prec inner, int* iters, double* res) {
    const bool r12 = link_format(inner) == 1;
    switch (base_prec(inner)) {
        case TMH_F64: return cg_fp64(l, x, b, gauge, kappa, mu, theta, tol, max_iter, iters, res, r12);
        case TMH_F32: return cg_mixed<float>(l, x, b, gauge, kappa, mu, theta, tol, max_iter, iters, res, r12);
        default: return cg_mixed<tmh::half_t>(l, x, b, gauge, kappa, mu, theta, tol, max_iter, iters, res, r12);
    }
}

}  // namespace

namespace tmh_api {

tmh_status qtm_check(const tmh_lattice* l, const void* out, const void* gauge, const void* in, double kappa,
                     double mu, const double theta[4], int sign, tmh_prec prec) {
    TMH_TRY(check_lat(l));
    TMH_TRY(check_prec(prec));
    TMH_TRY(check_theta(theta));
    if (sign != 1 && sign != -1) return TMH_ERR_ARG;
    if (!out || !gauge || !in || !isfinite(kappa) || !isfinite(mu)) return TMH_ERR_ARG;
    const size_t sb = spinor_bytes(l, prec);
    if (overlap(out, sb, in, sb) || overlap(out, sb, gauge, gauge_bytes(l, prec))) return TMH_ERR_ALIAS;
    return TMH_OK;
}

tmh_status qtm_run(tmh_lattice* l, void* out, const void* gauge, const void* in, void* te, double kappa,
                   double mu, const double theta[4], int sign, tmh_prec prec, bool timed) {
    const int lf = link_format(prec);
    return dispatch(prec, [&](auto tag) {
        using P = decltype(tag);
        return qtm_launch<P>(l, out, gauge, in, te, kappa, mu, theta, sign, nullptr, nullptr, lf, timed);
    });
}

int lattice_device(const tmh_lattice* l) { return l->device; }

size_t lattice_spinor_bytes(const tmh_lattice* l, tmh_prec prec) { return spinor_bytes(l, prec); }

}  // namespace tmh_api

extern "C" {

tmh_status tmh_lattice_create(tmh_lattice** out, const int dims[4], int device, void* hip_stream) {
    if (!out || !dims) return TMH_ERR_ARG;
    *out = nullptr;
    int64_t V = 1;
    for (int m = 0; m < 4; ++m) {
        if (dims[m] < 2 || (dims[m] & 1)) return TMH_ERR_GEOMETRY;
        V *= dims[m];
        if (V > ((int64_t)1 << 30)) return TMH_ERR_GEOMETRY;
    }
    // every component array (S FP64 complexes) must stay below 4 GiB: the
    // kernels address it through 32-bit buffer offsets
    if (site_stride(V / 2) * 16 >= ((int64_t)1 << 32)) return TMH_ERR_GEOMETRY;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return TMH_ERR_HIP;
    DeviceGuard guard(device);
    if (!guard.ok) return TMH_ERR_HIP;
    tmh_lattice* l = new (std::nothrow) tmh_lattice();
    if (!l) return TMH_ERR_NOMEM;
    memcpy(l->dims, dims, sizeof l->dims);
    l->device = device;
    l->stream = (hipStream_t)hip_stream;
    for (int m = 0; m < 4; ++m) l->g.L[m] = dims[m];
    l->g.Vh = (int)(V / 2);
    l->g.S = (int)site_stride(V / 2);
    for (auto& row : l->tuned)
        for (int& v : row) v = -1;
    l->xgroup = default_xgroup(l);
    // address of this device's fixed scratch (allocation-free entry points);
    // a failure here is reported by those entry points, which query again
    (void)tmh_api::noalloc_setup(device);
    const int nh = tmh::hop_blocks(l->g), nbl = tmh::blas_blocks(l->g);
    l->npartial = nh > nbl ? nh : nbl;
    tmh_status st = ensure((void**)&l->partial, sizeof(double) * l->npartial);
    if (st == TMH_OK) st = ensure((void**)&l->scal, sizeof(double) * tmh::kNScal);
    if (st == TMH_OK) st = ensure((void**)&l->flags, sizeof(int) * 2);
    if (st == TMH_OK && hipHostMalloc((void**)&l->h_scal, sizeof(double) * tmh::kNScal, hipHostMallocDefault) !=
                            hipSuccess)
        st = TMH_ERR_NOMEM;
    if (st == TMH_OK &&
        hipHostMalloc((void**)&l->h_flags, sizeof(int) * 2, hipHostMallocDefault) != hipSuccess)
        st = TMH_ERR_NOMEM;
    if (st != TMH_OK) {
        tmh_lattice_destroy(l);
        return st;
    }
    *out = l;
    return TMH_OK;
}

void tmh_lattice_destroy(tmh_lattice* l) {
    if (!l) return;
    DeviceGuard guard(l->device);
    (void)hipStreamSynchronize(l->stream);
    (void)hipFree(l->partial);
    (void)hipFree(l->scal);
    (void)hipFree(l->flags);
    if (l->h_scal) (void)hipHostFree(l->h_scal);
    if (l->h_flags) (void)hipHostFree(l->h_flags);
    for (void* p : l->even) (void)hipFree(p);
    (void)hipFree(l->even2);
    for (void* p : l->odd_rhs) (void)hipFree(p);
    for (void* p : l->mrhs) (void)hipFree(p);
    for (void* p : l->v64) (void)hipFree(p);
    for (auto& vs : l->vlow)
        for (void* p : vs) (void)hipFree(p);
    for (void* p : l->glow) (void)hipFree(p);
    (void)hipFree(l->gauge64r12);
    (void)prof_flush(l);
    for (auto& e : l->prof_free) {
        (void)hipEventDestroy(e.start);
        (void)hipEventDestroy(e.stop);
    }
    delete l;
}

tmh_status tmh_lattice_set_traversal(tmh_lattice* l, int xgroup) {
    TMH_TRY(check_lat(l));
    if (xgroup < 0 && xgroup != TMH_TRAVERSAL_XSLAB && tmarch_steps(xgroup) == 0) return TMH_ERR_ARG;
    if (xgroup != 0 && !xgroup_ok(l, xgroup)) return TMH_ERR_UNSUPPORTED;
    l->xgroup = xgroup;
    for (bool& t : l->xtuned) t = false;  // an explicit order applies to every code
    return TMH_OK;
}

int tmh_lattice_traversal(const tmh_lattice* l) { return l ? l->xgroup : -1; }

tmh_status tmh_lattice_set_stream(tmh_lattice* l, void* hip_stream) {
    TMH_TRY(check_lat(l));
    l->stream = (hipStream_t)hip_stream;
    return TMH_OK;
}

size_t tmh_half_volume(const tmh_lattice* l) { return l ? (size_t)l->g.Vh : 0; }
size_t tmh_site_stride(const tmh_lattice* l) { return l ? (size_t)l->g.S : 0; }
size_t tmh_spinor_bytes(const tmh_lattice* l, tmh_prec p) { return l ? spinor_bytes(l, p) : 0; }
size_t tmh_gauge_bytes(const tmh_lattice* l, tmh_prec p) { return l ? gauge_bytes(l, p) : 0; }

tmh_status tmh_gauge_import(tmh_lattice* l, void* dst, const double* src, tmh_prec prec) {
    TMH_TRY(check_lat(l));
    TMH_TRY(check_prec(prec));
    if (!dst || !src) return TMH_ERR_ARG;
    if (overlap(dst, gauge_bytes(l, prec), src, (size_t)2 * l->g.Vh * 4 * 9 * 16)) return TMH_ERR_ALIAS;
    DeviceGuard guard(l->device);
    const bool r12 = link_format(prec) == 1;
    return dispatch(prec, [&](auto tag) {
        using P = decltype(tag);
        using W = typename tmh::Word<P>::T;
        TMH_TRY_HIP(r12 ? tmh::launch_gauge_import_r12<P>((W*)dst, src, l->g, l->stream)
                        : tmh::launch_gauge_import<P>((W*)dst, src, l->g, l->stream));
        return TMH_OK;
    });
}

tmh_status tmh_spinor_import(tmh_lattice* l, void* dst, const double* src, tmh_prec prec) {
    TMH_TRY(check_lat(l));
    TMH_TRY(check_prec(prec));
    if (!dst || !src) return TMH_ERR_ARG;
    if (overlap(dst, spinor_bytes(l, prec), src, (size_t)l->g.Vh * 12 * 16)) return TMH_ERR_ALIAS;
    DeviceGuard guard(l->device);
    return dispatch(prec, [&](auto tag) {
        using P = decltype(tag);
        TMH_TRY_HIP(tmh::launch_spinor_import<P>((typename tmh::Word<P>::T*)dst, src, l->g, l->stream));
        return TMH_OK;
    });
}

tmh_status tmh_spinor_export(tmh_lattice* l, double* dst, const void* src, tmh_prec prec) {
    TMH_TRY(check_lat(l));
    TMH_TRY(check_prec(prec));
    if (!dst || !src) return TMH_ERR_ARG;
    if (overlap(dst, (size_t)l->g.Vh * 12 * 16, src, spinor_bytes(l, prec))) return TMH_ERR_ALIAS;
    DeviceGuard guard(l->device);
    return dispatch(prec, [&](auto tag) {
        using P = decltype(tag);
        TMH_TRY_HIP(tmh::launch_spinor_export<P>(dst, (const typename tmh::Word<P>::T*)src, l->g, l->stream));
        return TMH_OK;
    });
}

tmh_status tmh_hop_apply(tmh_lattice* l, tmh_dir dir, void* out, const void* gauge, const void* in, double kappa,
                         const double theta[4], tmh_prec prec) {
    TMH_TRY(check_lat(l));
    TMH_TRY(check_prec(prec));
    TMH_TRY(check_theta(theta));
    if (dir != TMH_EO && dir != TMH_OE) return TMH_ERR_ARG;
    if (!out || !gauge || !in || !isfinite(kappa)) return TMH_ERR_ARG;
    const size_t sb = spinor_bytes(l, prec);
    if (overlap(out, sb, in, sb) || overlap(out, sb, gauge, gauge_bytes(l, prec))) return TMH_ERR_ALIAS;
    DeviceGuard guard(l->device);
    const int pout = dir == TMH_EO ? 0 : 1;
    const int lf = link_format(prec);
    return dispatch(prec, [&](auto tag) {
        using P = decltype(tag);
        HopArgs<P> a = hop_args<P>(l, pout, out, gauge, in, theta, lf);
        a.c_re[0] = a.c_re[1] = (tmh::real_t<P>)kappa;
        TMH_TRY_HIP(hop_launch<P>(l, a, 0));
        return TMH_OK;
    });
}

tmh_status tmh_qtm_apply(tmh_lattice* l, void* out, const void* gauge, const void* in, double kappa, double mu,
                         const double theta[4], int sign, tmh_prec prec) {
    TMH_TRY(tmh_api::qtm_check(l, out, gauge, in, kappa, mu, theta, sign, prec));
    DeviceGuard guard(l->device);
    void* te;
    TMH_TRY(even_scratch(l, prec, &te));
    return tmh_api::qtm_run(l, out, gauge, in, te, kappa, mu, theta, sign, prec, true);
}

tmh_status tmh_cg_solve(tmh_lattice* l, void* x, const void* b, const void* gauge, double kappa, double mu,
                        const double theta[4], double rel_tol, int max_iter, tmh_prec inner, int* iters,
                        double* true_rel_res) {
    TMH_TRY(check_lat(l));
    TMH_TRY(check_prec(inner));
    TMH_TRY(check_theta(theta));
    if (!x || !b || !gauge || !iters || !true_rel_res) return TMH_ERR_ARG;
    if (!isfinite(kappa) || !isfinite(mu) || !(rel_tol > 0.0) || max_iter < 0) return TMH_ERR_ARG;
    const size_t sb = spinor_bytes(l, TMH_F64);
    if (overlap(x, sb, b, sb) || overlap(x, sb, gauge, gauge_bytes(l, TMH_F64))) return TMH_ERR_ALIAS;
    DeviceGuard guard(l->device);
    tmh_status st = cg_dispatch(l, x, b, gauge, kappa, mu, theta, rel_tol, max_iter, inner, iters, true_rel_res);
    if (hipStreamSynchronize(l->stream) != hipSuccess) return TMH_ERR_HIP;
    return st;
}

tmh_status tmh_hop_force(tmh_lattice* l, tmh_dir dir, void* force, const void* gauge, const void* left,
                         const void* right, double kappa, const double theta[4], double coeff,
                         tmh_force_kind kind) {
    TMH_TRY(check_lat(l));
    TMH_TRY(check_theta(theta));
    if (dir != TMH_EO && dir != TMH_OE) return TMH_ERR_ARG;
    if (kind != TMH_FORCE_SU3 && kind != TMH_FORCE_EUCLID) return TMH_ERR_ARG;
    if (!force || !gauge || !left || !right || !isfinite(kappa) || !isfinite(coeff)) return TMH_ERR_ARG;
    const size_t gb = gauge_bytes(l, TMH_F64), sb = spinor_bytes(l, TMH_F64);
    if (overlap(force, gb, gauge, gb) || overlap(force, gb, left, sb) || overlap(force, gb, right, sb))
        return TMH_ERR_ALIAS;
    DeviceGuard guard(l->device);
    TMH_TRY_HIP(force_launch(l, dir == TMH_EO ? 0 : 1, force, gauge, left, right, kappa, theta, coeff, kind,
                             1.0, 0.0, 1.0, 0.0));
    return TMH_OK;
}

tmh_status tmh_qtm_force(tmh_lattice* l, void* force, const void* gauge, const void* chi, const void* psi,
                         double kappa, double mu, const double theta[4], int sign, double coeff,
                         tmh_force_kind kind) {
    TMH_TRY(check_lat(l));
    TMH_TRY(check_theta(theta));
    if (sign != 1 && sign != -1) return TMH_ERR_ARG;
    if (kind != TMH_FORCE_SU3 && kind != TMH_FORCE_EUCLID) return TMH_ERR_ARG;
    if (!force || !gauge || !chi || !psi || !isfinite(kappa) || !isfinite(mu) || !isfinite(coeff))
        return TMH_ERR_ARG;
    const size_t gb = gauge_bytes(l, TMH_F64), sb = spinor_bytes(l, TMH_F64);
    if (overlap(force, gb, gauge, gb) || overlap(force, gb, chi, sb) || overlap(force, gb, psi, sb))
        return TMH_ERR_ALIAS;
    DeviceGuard guard(l->device);
    void* te;
    TMH_TRY(even_scratch(l, TMH_F64, &te));
    TMH_TRY(ensure(&l->even2, spinor_bytes(l, TMH_F64)));
    const double mt = 2.0 * kappa * mu * sign;
    const double D = 1.0 + mt * mt;
    // te = A^-1 H_eo psi; force -= coeff * dRe<gamma_5 chi, H_oe te>
    HopArgs<double> a = hop_args<double>(l, 0, te, gauge, psi, theta);
    a.c_re[0] = kappa / D;
    a.c_im[0] = -kappa * mt / D;
    a.c_re[1] = kappa / D;
    a.c_im[1] = kappa * mt / D;
    TMH_TRY_HIP(hop_launch<double>(l, a, 0));
    // w = H_eo chi; force -= coeff * dRe<(A^+)^-1 gamma_5 w, H_eo psi>,
    // (A^+)^-1 gamma_5 = diag((1 + i mt)/D, -(1 - i mt)/D) on upper/lower spins
    HopArgs<double> b = hop_args<double>(l, 0, l->even2, gauge, chi, theta);
    b.c_re[0] = b.c_re[1] = kappa;
    TMH_TRY_HIP(hop_launch<double>(l, b, 0));
    // both derivatives in one pass over the links and the force
    TMH_TRY_HIP(tmh::launch_force2(
        force_args(l, 1, force, gauge, chi, te, kappa, theta, -coeff, kind, 1.0, 0.0, -1.0, 0.0),
        force_args(l, 0, force, gauge, l->even2, psi, kappa, theta, -coeff, kind, 1.0 / D, mt / D, -1.0 / D, mt / D),
        l->stream));
    return TMH_OK;
}

tmh_status tmh_solve_full(tmh_lattice* l, void* x_even, void* x_odd, const void* b_even, const void* b_odd,
                          const void* gauge, double kappa, double mu, const double theta[4], double rel_tol,
                          int max_iter, tmh_prec inner, int* iters, double* true_rel_res) {
    TMH_TRY(check_lat(l));
    TMH_TRY(check_prec(inner));
    TMH_TRY(check_theta(theta));
    if (!x_even || !x_odd || !b_even || !b_odd || !gauge || !iters || !true_rel_res) return TMH_ERR_ARG;
    if (!isfinite(kappa) || !isfinite(mu) || !(rel_tol > 0.0) || max_iter < 0) return TMH_ERR_ARG;
    const size_t sb = spinor_bytes(l, TMH_F64), gb = gauge_bytes(l, TMH_F64);
    const void* ins[3] = {b_even, b_odd, gauge};
    const size_t insz[3] = {sb, sb, gb};
    for (int k = 0; k < 3; ++k)
        if (overlap(x_even, sb, ins[k], insz[k]) || overlap(x_odd, sb, ins[k], insz[k])) return TMH_ERR_ALIAS;
    if (overlap(x_even, sb, x_odd, sb)) return TMH_ERR_ALIAS;
    DeviceGuard guard(l->device);
    TMH_TRY(ensure(&l->even2, sb));
    for (int k = 0; k < 2; ++k) TMH_TRY(ensure(&l->odd_rhs[k], sb));
    const double mt = 2.0 * kappa * mu;
    const double D = 1.0 + mt * mt;
    // A^-1 = (1 - i mt gamma_5)/D: upper (1 - i mt)/D, lower (1 + i mt)/D
    const double ai_re = 1.0 / D, ai_up = -mt / D, ai_dn = mt / D;
    // even2 = A^-1 b_e
    TMH_TRY_HIP(tmh::launch_chiral_scale((double2*)l->even2, (const double2*)b_even, ai_re, ai_up, ai_re, ai_dn,
                                         l->g, l->stream));
    // odd_rhs[0] = gamma_5 (b_o + H_oe A^-1 b_e)
    HopArgs<double> a = hop_args<double>(l, 1, l->odd_rhs[0], gauge, l->even2, theta);
    a.aux = (const double2*)b_odd;
    a.c_re[0] = kappa;
    a.c_re[1] = -kappa;
    a.d_re[0] = 1.0;
    a.d_re[1] = -1.0;
    TMH_TRY_HIP(hop_launch<double>(l, a, 1));
    // odd_rhs[1] = Qhat(-) gamma_5 bhat_o: the right-hand side of Qhat^+ Qhat x_o
    void* te;
    TMH_TRY(even_scratch(l, TMH_F64, &te));
    TMH_TRY(qtm_launch<double>(l, l->odd_rhs[1], gauge, l->odd_rhs[0], te, kappa, mu, theta, -1, nullptr,
                               nullptr));
    tmh_status st = cg_dispatch(l, x_odd, l->odd_rhs[1], gauge, kappa, mu, theta, rel_tol, max_iter, inner, iters,
                                true_rel_res);
    if (st != TMH_OK && st != TMH_ERR_NOT_CONVERGED) return st;
    // x_e = A^-1 (b_e + H_eo x_o)
    HopArgs<double> b = hop_args<double>(l, 0, x_even, gauge, x_odd, theta);
    b.aux = (const double2*)b_even;
    b.c_re[0] = kappa * ai_re;
    b.c_im[0] = kappa * ai_up;
    b.c_re[1] = kappa * ai_re;
    b.c_im[1] = kappa * ai_dn;
    b.d_re[0] = ai_re;
    b.d_im[0] = ai_up;
    b.d_re[1] = ai_re;
    b.d_im[1] = ai_dn;
    TMH_TRY_HIP(hop_launch<double>(l, b, 1));
    if (hipStreamSynchronize(l->stream) != hipSuccess) return TMH_ERR_HIP;
    return st;
}

}  // extern "C"

// ------------------------------------------------------------------ batches

namespace {

int default_shape(const tmh_lattice* l, int nrhs, tmh_prec prec) {
    if (nrhs >= 1 && nrhs <= 16 && l->tuned[prec][nrhs] >= 0) return l->tuned[prec][nrhs];
    return nrhs >= 4 ? tmh::kShape1x4 : (nrhs >= 2 ? tmh::kShape2x2 : tmh::kShape4x1);
}

int hop_tiles(const Geo& g, int shape) {
    int sw, ry, nr;
    tmh::batch_shape(shape, &sw, &ry, &nr);
    return (g.Vh + 64 * sw - 1) / (64 * sw);
}

int hop_items(const Geo& g, int nrhs, int shape) {
    const int per = tmh::batch_rhs_per_item(shape);
    return hop_tiles(g, shape) * ((nrhs + per - 1) / per);
}

template <typename R>
tmh::BatchHopTask<R> hop_task(const tmh_lattice* l, int pout, void* out, const void* gauge, const void* in,
                              const void* aux, int nrhs, const double theta[4]) {
    using W = typename tmh::Word<R>::T;
    tmh::BatchHopTask<R> t;
    memset(&t, 0, sizeof t);
    t.out = (W*)out;
    t.in = (const W*)in;
    t.aux = (const W*)aux;
    t.gout = (const W*)gauge + (int64_t)pout * 36 * l->g.S;
    t.gin = (const W*)gauge + (int64_t)(1 - pout) * 36 * l->g.S;
    t.fstride = (int64_t)12 * l->g.S;
    t.g = l->g;
    t.pout = pout;
    t.nrhs = nrhs;
    for (int m = 0; m < 4; ++m) {
        t.ph_re[m] = (R)cos(M_PI * theta[m]);
        t.ph_im[m] = (R)sin(M_PI * theta[m]);
    }
    return t;
}

// Tile order of a batched hop task (batch.hip, tile_site): x-group order
// where tiles fill whole (t, x) planes and T splits into 8 chunks, with the
// largest group whose time-slice holds at most TMH_BATCH_XG_SITES
// site-right-hand-side pairs (at least one x value); else even-odd order.
#ifndef TMH_BATCH_XG_SITES
#define TMH_BATCH_XG_SITES 8192
#endif
template <typename R> void batch_traversal(tmh::BatchHopTask<R>& t, const tmh_lattice* l, int shape) {
    int sw, ry, nr;
    tmh::batch_shape(shape, &sw, &ry, &nr);
    const int nsl = 64 * sw, plane = l->dims[2] * l->dims[3] / 2;
    t.xgroup = 0;
    if (TMH_BATCH_XG_SITES <= 0 || plane % nsl != 0 || l->dims[0] % 8 != 0) return;
    int best = 1;
    for (int xg = 1; xg <= l->dims[1]; ++xg)
        if (l->dims[1] % xg == 0 && (int64_t)xg * plane * t.nrhs <= TMH_BATCH_XG_SITES) best = xg;
    t.xgroup = best;
    t.nyt = plane / nsl;
    t.nt = l->dims[0] / 8;
}

// The t-march shapes need whole tiles (256 pairs, or 64 for the shape with
// four right-hand sides per workgroup) per time-slice.
bool batch_tmarch_ok(const tmh_lattice* l, int shape) {
    return ((int64_t)l->dims[1] * l->dims[2] * l->dims[3] / 2) % (256 / tmh::batch_tmarch_rg(shape)) == 0;
}

// t-march layout of a task: the fewest ranges of time-slices (dividing T)
// whose workgroups (tiles x ranges x right-hand-side groups) reach 512, two
// per CU, so that every workgroup walks as many slices as the grid allows.
template <typename R>
void batch_tmarch_setup(tmh::BatchHopTask<R>& t, const tmh_lattice* l, int nrhs, int shape) {
    const int T = l->dims[0];
    t.tm_rg = tmh::batch_tmarch_rg(shape);
    t.tm_slice = l->dims[1] * l->dims[2] * l->dims[3] / 2;
    t.tm_nw = t.tm_slice / (256 / t.tm_rg);
    const int64_t groups = (nrhs + t.tm_rg - 1) / t.tm_rg;
    // FP32: walks of at most 8 slices (measured 6 % faster with 12
    // right-hand sides at 32^3x64; FP64 gains nothing from shorter walks)
    const int max_steps = sizeof(R) == 4 ? 8 : T;
    int ranges = T;
    for (int d = 1; d <= T; ++d)
        if (T % d == 0 && (int64_t)t.tm_nw * groups * d >= 512 && T / d <= max_steps) {
            ranges = d;
            break;
        }
    t.tm_steps = T / ranges;
}

// Coefficients of the four hop steps of Qhat(sign): step 0 stores A^-1 H,
// step 1 forms gamma_5 [A aux - H].
template <typename R>
void qtm_coeffs(tmh::BatchHopTask<R>& t, int step, double kappa, double mu, int sign) {
    const double mt = 2.0 * kappa * mu * sign, D = 1.0 + mt * mt;
    if (step == 0) {
        t.c_re[0] = (R)(kappa / D);
        t.c_im[0] = (R)(-kappa * mt / D);
        t.c_re[1] = (R)(kappa / D);
        t.c_im[1] = (R)(kappa * mt / D);
    } else {
        t.c_re[0] = (R)(-kappa);
        t.c_re[1] = (R)kappa;
        t.d_re[0] = (R)1;
        t.d_im[0] = (R)mt;
        t.d_re[1] = (R)-1;
        t.d_im[1] = (R)mt;
    }
}

tmh_status mrhs_scratch(tmh_lattice* l, int nrhs) {
    if (nrhs <= l->mrhs_cap) return TMH_OK;
    for (void*& p : l->mrhs) {
        (void)hipFree(p);
        p = nullptr;
    }
    l->mrhs_cap = 0;
    for (void*& p : l->mrhs) TMH_TRY(ensure(&p, (size_t)nrhs * spinor_bytes(l, TMH_F64)));
    l->mrhs_cap = nrhs;
    return TMH_OK;
}

struct StreamGuard {  // a private non-null stream for graph capture, ordered after `user`
    hipStream_t user, own = nullptr;
    hipEvent_t ev = nullptr;
    bool ok = false;
    explicit StreamGuard(hipStream_t u) : user(u) {
        ok = hipStreamCreateWithFlags(&own, hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess &&
             hipEventRecord(ev, user) == hipSuccess && hipStreamWaitEvent(own, ev, 0) == hipSuccess;
    }
    ~StreamGuard() {
        if (own) {
            (void)hipStreamSynchronize(own);
            (void)hipStreamDestroy(own);
        }
        if (ev) (void)hipEventDestroy(ev);
    }
};

}  // namespace

extern "C" {

tmh_status tmh_hop_apply_mrhs(tmh_lattice* l, tmh_dir dir, void* out, const void* gauge, const void* in, int nrhs,
                              double kappa, const double theta[4], tmh_prec prec, int shape) {
    TMH_TRY(check_lat(l));
    TMH_TRY(check_prec_full(prec));
    TMH_TRY(check_theta(theta));
    if (dir != TMH_EO && dir != TMH_OE) return TMH_ERR_ARG;
    if (!out || !gauge || !in || nrhs < 1 || !isfinite(kappa) || shape < -1 || shape >= tmh::kNumShapes)
        return TMH_ERR_ARG;
    const size_t sb = (size_t)nrhs * spinor_bytes(l, prec);
    if (overlap(out, sb, in, sb) || overlap(out, sb, gauge, gauge_bytes(l, prec))) return TMH_ERR_ALIAS;
    DeviceGuard guard(l->device);
    if (shape < 0) shape = default_shape(l, nrhs, prec);
    if (tmh::batch_is_tmarch(shape) && !batch_tmarch_ok(l, shape)) return TMH_ERR_UNSUPPORTED;
    const int pout = dir == TMH_EO ? 0 : 1;
    const int items = hop_items(l->g, nrhs, shape);
    if (prec == TMH_F64) {
        tmh::BatchHopTable<double> tab;
        memset(&tab, 0, sizeof tab);
        tab.ntasks = 1;
        tab.t[0] = hop_task<double>(l, pout, out, gauge, in, nullptr, nrhs, theta);
        tab.t[0].c_re[0] = tab.t[0].c_re[1] = kappa;
        batch_traversal(tab.t[0], l, shape);
        if (tmh::batch_is_tmarch(shape)) batch_tmarch_setup(tab.t[0], l, nrhs, shape);
        TMH_TRY_HIP(tmh::launch_batch_hop<double>(tab, items, shape, 0, l->stream));
    } else {
        tmh::BatchHopTable<float> tab;
        memset(&tab, 0, sizeof tab);
        tab.ntasks = 1;
        tab.t[0] = hop_task<float>(l, pout, out, gauge, in, nullptr, nrhs, theta);
        tab.t[0].c_re[0] = tab.t[0].c_re[1] = (float)kappa;
        batch_traversal(tab.t[0], l, shape);
        if (tmh::batch_is_tmarch(shape)) batch_tmarch_setup(tab.t[0], l, nrhs, shape);
        TMH_TRY_HIP(tmh::launch_batch_hop<float>(tab, items, shape, 0, l->stream));
    }
    return TMH_OK;
}

tmh_status tmh_batch_cg_solve(const tmh_batch_member* m, int nmem, double rel_tol, int max_iter, int shape,
                              int use_graph, int* iters, double* true_rel_res) {
    if (!m || nmem < 1 || nmem > tmh::kMaxBatchTasks || !iters || !true_rel_res) return TMH_ERR_ARG;
    if (!(rel_tol > 0.0) || max_iter < 0 || shape < -1 || shape >= tmh::kNumShapes) return TMH_ERR_ARG;
    int nsys = 0;
    for (int k = 0; k < nmem; ++k) {
        TMH_TRY(check_lat(m[k].lat));
        TMH_TRY(check_theta(m[k].theta));
        if (!m[k].x || !m[k].b || !m[k].gauge || m[k].nrhs < 1) return TMH_ERR_ARG;
        if (!isfinite(m[k].kappa) || !isfinite(m[k].mu)) return TMH_ERR_ARG;
        if (m[k].lat->device != m[0].lat->device) return TMH_ERR_ARG;
        const size_t sb = (size_t)m[k].nrhs * spinor_bytes(m[k].lat, TMH_F64);
        if (overlap(m[k].x, sb, m[k].b, sb) || overlap(m[k].x, sb, m[k].gauge, gauge_bytes(m[k].lat, TMH_F64)))
            return TMH_ERR_ALIAS;
        for (int j = 0; j < k; ++j)
            if (m[j].lat == m[k].lat) return TMH_ERR_ARG;  // scratch is per lattice handle
        nsys += m[k].nrhs;
    }
    tmh_lattice* l0 = m[0].lat;
    DeviceGuard guard(l0->device);
    if (shape < 0) shape = default_shape(l0, m[0].nrhs, TMH_F64);
    if (tmh::batch_is_tmarch(shape))
        for (int k = 0; k < nmem; ++k)
            if (!batch_tmarch_ok(m[k].lat, shape)) return TMH_ERR_UNSUPPORTED;
    for (int k = 0; k < nmem; ++k) TMH_TRY(mrhs_scratch(m[k].lat, m[k].nrhs));
    // per-system partial slots, scalars, flags
    int64_t pstride = 1;
    int items_hop = 0, items_vec = 0;
    tmh::BatchSysTable systab;
    memset(&systab, 0, sizeof systab);
    systab.ntasks = nmem;
    for (int k = 0, s0 = 0; k < nmem; ++k) {
        const Geo& g = m[k].lat->g;
        systab.sys0[k] = s0;
        systab.nrhs[k] = m[k].nrhs;
        systab.ntile_hop[k] = hop_tiles(g, shape);
        systab.ntile_vec[k] = tmh::batch_vec_tiles(g.Vh);
        pstride = std::max<int64_t>(pstride, std::max(systab.ntile_hop[k], systab.ntile_vec[k]));
        s0 += m[k].nrhs;
    }
    double* partial = nullptr;
    double* scal = nullptr;
    int* flags = nullptr;
    double* h_scal = nullptr;
    int* h_flags = nullptr;
    tmh_status st = TMH_OK;
    auto cleanup = [&]() {
        (void)hipFree(partial);
        (void)hipFree(scal);
        (void)hipFree(flags);
        if (h_scal) (void)hipHostFree(h_scal);
        if (h_flags) (void)hipHostFree(h_flags);
    };
    if (hipMalloc((void**)&partial, sizeof(double) * pstride * nsys) != hipSuccess ||
        hipMalloc((void**)&scal, sizeof(double) * tmh::kNScal * nsys) != hipSuccess ||
        hipMalloc((void**)&flags, sizeof(int) * 2 * nsys) != hipSuccess ||
        hipHostMalloc((void**)&h_scal, sizeof(double) * tmh::kNScal * nsys, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&h_flags, sizeof(int) * 2 * nsys, hipHostMallocDefault) != hipSuccess) {
        cleanup();
        return TMH_ERR_NOMEM;
    }
    // task tables of every step
    tmh::BatchHopTable<double> H[8];  // 0..3: CG iteration; 4..7: true residual A x
    memset(H, 0, sizeof H);
    tmh::BatchVecTable Vp, Vsub, Vnb, Vcp, Vnx, Vrb;
    memset(&Vp, 0, sizeof Vp);
    memset(&Vsub, 0, sizeof Vsub);
    memset(&Vnb, 0, sizeof Vnb);
    memset(&Vcp, 0, sizeof Vcp);
    memset(&Vnx, 0, sizeof Vnx);
    memset(&Vrb, 0, sizeof Vrb);
    for (int k = 0, s0 = 0; k < nmem; ++k) {
        tmh_lattice* l = m[k].lat;
        const int n = m[k].nrhs;
        void *r = l->mrhs[0], *p = l->mrhs[1], *v = l->mrhs[2], *q = l->mrhs[3], *te = l->mrhs[4];
        void* x = m[k].x;
        const void* b = m[k].b;
        const void* in0[8] = {p, te, v, te, x, te, v, te};
        void* out0[8] = {te, v, te, q, te, v, te, q};
        const void* aux0[8] = {nullptr, p, nullptr, v, nullptr, x, nullptr, v};
        const int signs[8] = {+1, +1, -1, -1, +1, +1, -1, -1};
        for (int h = 0; h < 8; ++h) {
            auto t = hop_task<double>(l, h % 2 == 0 ? 0 : 1, out0[h], m[k].gauge, in0[h], aux0[h], n, m[k].theta);
            qtm_coeffs(t, h % 2, m[k].kappa, m[k].mu, signs[h]);
            batch_traversal(t, l, shape);
            t.partial = partial;
            t.pstride = pstride;
            t.flags = h < 4 ? flags : nullptr;
            if (h == 3) {  // the iteration's last hop carries the CG update (q is not stored)
                t.rio = (double2*)r;
                t.xio = (double2*)x;
                t.pin = (const double2*)p;
                t.scal = scal;
            }
            t.sys0 = s0;
            t.item0 = H[h].ntasks == 0 ? 0 : H[h].t[H[h].ntasks - 1].item0 + hop_items(m[k - 1].lat->g, m[k - 1].nrhs, shape);
            if (tmh::batch_is_tmarch(shape)) batch_tmarch_setup(t, l, n, shape);
            H[h].t[H[h].ntasks++] = t;
        }
        tmh::BatchVecTask vt;
        memset(&vt, 0, sizeof vt);
        vt.partial = partial;
        vt.fstride = (int64_t)12 * l->g.S;
        vt.pstride = pstride;
        vt.Vh = l->g.Vh;
        vt.S = l->g.S;
        vt.nrhs = n;
        vt.ntile = tmh::batch_vec_tiles(l->g.Vh);
        vt.sys0 = s0;
        vt.item0 = items_vec;
        auto push = [&](tmh::BatchVecTable& T, void* a, void* bb, const void* c, const void* d) {
            tmh::BatchVecTask u = vt;
            u.a = (double2*)a;
            u.b = (double2*)bb;
            u.c = (const double2*)c;
            u.d = (const double2*)d;
            T.t[T.ntasks++] = u;
        };
        push(Vp, p, nullptr, r, nullptr);
        push(Vsub, r, nullptr, b, q);
        push(Vnb, nullptr, nullptr, b, nullptr);
        push(Vcp, p, nullptr, r, nullptr);
        push(Vnx, nullptr, nullptr, x, nullptr);
        push(Vrb, r, nullptr, b, nullptr);
        items_vec += n * vt.ntile;
        items_hop += hop_items(l->g, n, shape);
        s0 += n;
    }
    const double tol2 = rel_tol * rel_tol;
    tmh::batch_prepare(shape);
    StreamGuard sg(l0->stream);
    if (!sg.ok) {
        cleanup();
        return TMH_ERR_HIP;
    }
    hipStream_t s = sg.own;
    auto read_back = [&]() -> tmh_status {
        TMH_TRY_HIP(hipMemcpyAsync(h_scal, scal, sizeof(double) * tmh::kNScal * nsys, hipMemcpyDeviceToHost, s));
        TMH_TRY_HIP(hipMemcpyAsync(h_flags, flags, sizeof(int) * 2 * nsys, hipMemcpyDeviceToHost, s));
        TMH_TRY_HIP(hipStreamSynchronize(s));
        return TMH_OK;
    };
    auto true_res = [&]() -> tmh_status {
        for (int h = 4; h < 8; ++h) TMH_TRY_HIP(tmh::launch_batch_hop<double>(H[h], items_hop, shape, h % 2, s));
        TMH_TRY_HIP(tmh::launch_batch_vec(2, Vsub, items_vec, scal, flags, s));
        TMH_TRY_HIP(tmh::launch_batch_scalar(2, nsys, systab, scal, flags, partial, pstride, tol2, max_iter, s));
        return read_back();
    };
    auto iteration = [&](int budget) -> hipError_t {
        hipError_t e;
        if ((e = tmh::launch_batch_hop<double>(H[0], items_hop, shape, 0, s)) != hipSuccess) return e;
        if ((e = tmh::launch_batch_hop<double>(H[1], items_hop, shape, 2, s)) != hipSuccess) return e;
        if ((e = tmh::launch_batch_scalar(0, nsys, systab, scal, flags, partial, pstride, tol2, budget, s)) != hipSuccess)
            return e;
        if ((e = tmh::launch_batch_hop<double>(H[2], items_hop, shape, 0, s)) != hipSuccess) return e;
        if ((e = tmh::launch_batch_hop<double>(H[3], items_hop, shape, 3, s)) != hipSuccess) return e;
        if ((e = tmh::launch_batch_scalar(1, nsys, systab, scal, flags, partial, pstride, tol2, budget, s)) != hipSuccess)
            return e;
        return tmh::launch_batch_vec(1, Vp, items_vec, scal, flags, s);
    };
    std::vector<int> total(nsys, 0);
    std::vector<double> bb(nsys), res(nsys, 0.0);
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int graph_budget = -1;
    do {
        // |x|^2 (into kNorm), then |b|^2 per system; the |b|^2 partials stay
        // in place for the restart step when every start vector is zero
        if (tmh::launch_batch_vec(3, Vnx, items_vec, scal, flags, s) != hipSuccess ||
            tmh::launch_batch_scalar(2, nsys, systab, scal, flags, partial, pstride, tol2, max_iter, s) != hipSuccess ||
            tmh::launch_batch_vec(3, Vnb, items_vec, scal, flags, s) != hipSuccess ||
            tmh::launch_batch_scalar(4, nsys, systab, scal, flags, partial, pstride, tol2, max_iter, s) != hipSuccess) {
            st = TMH_ERR_HIP;
            break;
        }
        if ((st = read_back()) != TMH_OK) break;
        // A system with b = 0 has the solution x = 0, as in tmh_cg_solve:
        // its x is cleared here, so that its residual is 0 and the CG
        // initialisation marks it done before the first iteration.
        for (int k = 0, mk = 0, r = 0; k < nsys && st == TMH_OK; ++k) {
            if (h_scal[k * tmh::kNScal + tmh::kBB] == 0.0 && h_scal[k * tmh::kNScal + tmh::kNorm] != 0.0) {
                const size_t sb = spinor_bytes(m[mk].lat, TMH_F64);
                if (hipMemsetAsync((char*)m[mk].x + r * sb, 0, sb, s) != hipSuccess) st = TMH_ERR_HIP;
                h_scal[k * tmh::kNScal + tmh::kNorm] = 0.0;
            }
            if (++r == m[mk].nrhs) {
                ++mk;
                r = 0;
            }
        }
        if (st != TMH_OK) break;
        bool zero_start = true;
        for (int k = 0; k < nsys; ++k) {
            bb[k] = h_scal[k * tmh::kNScal + tmh::kBB];
            if (h_scal[k * tmh::kNScal + tmh::kNorm] != 0.0) zero_start = false;
        }
        if (zero_start) {
            // r = b needs no operator application
            if (tmh::launch_batch_vec(4, Vrb, items_vec, scal, flags, s) != hipSuccess) {
                st = TMH_ERR_HIP;
                break;
            }
            for (int k = 0; k < nsys; ++k) h_scal[k * tmh::kNScal + tmh::kNorm] = bb[k];
        } else if ((st = true_res()) != TMH_OK) {
            break;
        }
        int it_done = 0;
        for (int restart = 0;; ++restart) {
            bool all = true;
            for (int k = 0; k < nsys; ++k) {
                const double rr = h_scal[k * tmh::kNScal + tmh::kNorm];
                res[k] = bb[k] > 0.0 ? sqrt(rr / bb[k]) : 0.0;
                if (res[k] > rel_tol) all = false;
            }
            if (all || restart > 3 || it_done >= max_iter) break;
            const int budget = max_iter - it_done;
            if (tmh::launch_batch_scalar(3, nsys, systab, scal, flags, partial, pstride, tol2, budget, s) != hipSuccess ||
                tmh::launch_batch_vec(4, Vcp, items_vec, scal, flags, s) != hipSuccess) {
                st = TMH_ERR_HIP;
                break;
            }
            if (use_graph && graph_budget != budget) {
                if (exec) (void)hipGraphExecDestroy(exec);
                if (graph) (void)hipGraphDestroy(graph);
                exec = nullptr;
                graph = nullptr;
                if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
                    st = TMH_ERR_HIP;
                    break;
                }
                const hipError_t e = iteration(budget);
                if (hipStreamEndCapture(s, &graph) != hipSuccess || e != hipSuccess ||
                    hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
                    st = TMH_ERR_HIP;
                    break;
                }
                graph_budget = budget;
            }
            bool running = true;
            while (running) {
                for (int c = 0; c < kChunk; ++c) {
                    const hipError_t e = use_graph ? hipGraphLaunch(exec, s) : iteration(budget);
                    if (e != hipSuccess) {
                        st = TMH_ERR_HIP;
                        break;
                    }
                }
                if (st != TMH_OK || (st = read_back()) != TMH_OK) break;
                running = false;
                for (int k = 0; k < nsys; ++k)
                    if (!h_flags[2 * k]) running = true;
            }
            if (st != TMH_OK) break;
            int mx = 0;
            for (int k = 0; k < nsys; ++k) {
                total[k] += h_flags[2 * k + 1];
                mx = std::max(mx, h_flags[2 * k + 1]);
            }
            it_done += mx;
            if ((st = true_res()) != TMH_OK) break;
        }
    } while (false);
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    bool conv = st == TMH_OK;
    for (int k = 0; k < nsys; ++k) {
        iters[k] = total[k];
        true_rel_res[k] = res[k];
        if (res[k] > rel_tol) conv = false;
    }
    if (hipStreamSynchronize(s) != hipSuccess && st == TMH_OK) st = TMH_ERR_HIP;
    cleanup();
    if (st != TMH_OK) return st;
    return conv ? TMH_OK : TMH_ERR_NOT_CONVERGED;
}

tmh_status tmh_autotune_mrhs(tmh_lattice* l, const void* gauge, int nrhs, tmh_prec prec, const char* cache_path,
                             int* best_shape, double* best_us) {
    TMH_TRY(check_lat(l));
    TMH_TRY(check_prec_full(prec));
    if (!gauge || nrhs < 1 || nrhs > 16 || !best_shape || !best_us) return TMH_ERR_ARG;
    DeviceGuard guard(l->device);
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, l->device) == hipSuccess) arch = prop.gcnArchName;
    const size_t sp = arch.find(':');
    if (sp != std::string::npos) arch = arch.substr(0, sp);
    char key[256];
    snprintf(key, sizeof key, "%s %dx%dx%dx%d %s %d", arch.c_str(), l->dims[0], l->dims[1], l->dims[2], l->dims[3],
             prec == TMH_F64 ? "f64" : "f32", nrhs);
    if (cache_path) {
        if (FILE* f = fopen(cache_path, "r")) {
            // the outputs are written only on a hit (or after timing)
            int hit_shape = -1;
            double hit_us = 0.0;
            char line[512];
            while (fgets(line, sizeof line, f)) {
                int sh = -1;
                double us = 0.0;
                const size_t kl = strlen(key);
                if (strncmp(line, key, kl) == 0 && line[kl] == ' ' && sscanf(line + kl, " %d %lf", &sh, &us) == 2 &&
                    sh >= 0 && sh < tmh::kNumShapes) {
                    hit_shape = sh;
                    hit_us = us;
                }
            }
            fclose(f);
            if (hit_shape >= 0 && hit_us > 0.0) {
                *best_shape = hit_shape;
                *best_us = hit_us;
                l->tuned[prec][nrhs] = hit_shape;
                return TMH_OK;
            }
        }
    }
    // time every shape on scratch fields
    void *in = nullptr, *out = nullptr;
    const size_t sb = (size_t)nrhs * spinor_bytes(l, prec);
    if (hipMalloc(&in, sb) != hipSuccess || hipMalloc(&out, sb) != hipSuccess) {
        (void)hipFree(in);
        return TMH_ERR_NOMEM;
    }
    tmh_status st = TMH_OK;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    double best = 1e300;
    int bs = -1;
    const double theta[4] = {1.0, 0.0, 0.0, 0.0};
    if (hipMemsetAsync(in, 0, sb, l->stream) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
        hipEventCreate(&e1) != hipSuccess)
        st = TMH_ERR_HIP;
    for (int sh = 0; sh < tmh::kNumShapes && st == TMH_OK; ++sh) {
        if (tmh::batch_is_tmarch(sh) && !batch_tmarch_ok(l, sh)) continue;
        for (int w = 0; w < 2 && st == TMH_OK; ++w)
            st = tmh_hop_apply_mrhs(l, TMH_EO, out, gauge, in, nrhs, 0.1, theta, prec, sh);
        if (st != TMH_OK) break;
        const int reps = 5;
        if (hipEventRecord(e0, l->stream) != hipSuccess) st = TMH_ERR_HIP;
        for (int k = 0; k < reps && st == TMH_OK; ++k)
            st = tmh_hop_apply_mrhs(l, k % 2 ? TMH_OE : TMH_EO, out, gauge, in, nrhs, 0.1, theta, prec, sh);
        float ms = 0.f;
        if (st == TMH_OK && (hipEventRecord(e1, l->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                             hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
            st = TMH_ERR_HIP;
        const double us = 1e3 * ms / reps;
        if (st == TMH_OK && us < best) {
            best = us;
            bs = sh;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(l->stream);
    (void)hipFree(in);
    (void)hipFree(out);
    if (st != TMH_OK) return st;
    *best_shape = bs;
    *best_us = best;
    l->tuned[prec][nrhs] = bs;
    if (cache_path) {
        if (FILE* f = fopen(cache_path, "a")) {
            fprintf(f, "%s %d %.3f\n", key, bs, best);
            fclose(f);
        }
    }
    return TMH_OK;
}

tmh_status tmh_autotune_hop(tmh_lattice* l, const void* gauge, tmh_prec prec, const char* cache_path, int* best_xgroup,
                            double* best_us) {
    TMH_TRY(check_lat(l));
    TMH_TRY(check_prec(prec));
    if (!gauge || !best_xgroup || !best_us) return TMH_ERR_ARG;
    DeviceGuard guard(l->device);
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, l->device) == hipSuccess) arch = prop.gcnArchName;
    const size_t sp = arch.find(':');
    if (sp != std::string::npos) arch = arch.substr(0, sp);
    char key[256];
    static const char* const kPrecName[6] = {"f64", "f32", "f64r12", "f32r12", "f16", "f16r12"};
    snprintf(key, sizeof key, "%s %dx%dx%dx%d %s hop", arch.c_str(), l->dims[0], l->dims[1], l->dims[2], l->dims[3],
             kPrecName[prec]);
    if (cache_path) {
        if (FILE* f = fopen(cache_path, "r")) {
            char line[512];
            int xg = -1;
            double us = 0.0;
            const size_t kl = strlen(key);
            while (fgets(line, sizeof line, f)) {
                int a = -1;
                double b = 0.0;
                if (strncmp(line, key, kl) == 0 && line[kl] == ' ' && sscanf(line + kl, " %d %lf", &a, &b) == 2 &&
                    (a == 0 || xgroup_ok(l, a))) {
                    xg = a;
                    us = b;
                }
            }
            fclose(f);
            if (xg != -1) {
                l->xgroup = xg;
                l->xtuned[prec] = true;
                l->xgroup_code[prec] = xg;
                *best_xgroup = xg;
                *best_us = us;
                return TMH_OK;
            }
        }
    }
    void *in = nullptr, *out = nullptr;
    const size_t sb = spinor_bytes(l, prec);
    if (hipMalloc(&in, sb) != hipSuccess || hipMalloc(&out, sb) != hipSuccess) {
        (void)hipFree(in);
        return TMH_ERR_NOMEM;
    }
    tmh_status st = TMH_OK;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const double theta[4] = {1.0, 0.0, 0.0, 0.0};
    double best = 1e300;
    int bx = 0;
    const int saved = l->xgroup, saved_code = l->xgroup_code[prec];
    const bool saved_tuned = l->xtuned[prec];
    l->xtuned[prec] = true;
    if (hipMemsetAsync(in, 0, sb, l->stream) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
        hipEventCreate(&e1) != hipSuccess)
        st = TMH_ERR_HIP;
    std::vector<int> cands = {0};
    if (xgroup_ok(l, tmh::kXSlab)) cands.push_back(tmh::kXSlab);
    for (int xg = 1; xg <= l->dims[1]; ++xg)
        if (xgroup_ok(l, xg)) cands.push_back(xg);
    // t-march step counts whose grids hold between 64 and 4096 workgroups
    for (int st = 1; st <= l->dims[0]; ++st)
        if (tmarch_ok(l, st)) {
            const int nb = tmh::hop_tmarch_blocks(l->g, st);
            if (nb >= 64 && nb <= 4096) cands.push_back(tmh::kTMarch0 - st);
        }
    // two rounds over the candidates, each candidate's time the smaller of
    // its two, so that a drift of the clock or of other load during one
    // round does not decide between orders a few per cent apart
    std::vector<double> cand_us(cands.size(), 1e300);
    for (int round = 0; round < 2 && st == TMH_OK; ++round) {
        for (size_t ci = 0; ci < cands.size() && st == TMH_OK; ++ci) {
            const int xg = cands[ci];
            l->xgroup = xg;
            l->xgroup_code[prec] = xg;
            // a chain of hops, each reading what the previous one wrote, as
            // inside the solvers (a hop repeated on one input finds more of
            // it in the caches)
            for (int w = 0; w < 2 && st == TMH_OK; ++w)
                st = tmh_hop_apply(l, w % 2 ? TMH_OE : TMH_EO, w % 2 ? in : out, gauge, w % 2 ? out : in, 0.1,
                                   theta, prec);
            const int reps = 6;
            if (st == TMH_OK && hipEventRecord(e0, l->stream) != hipSuccess) st = TMH_ERR_HIP;
            for (int k = 0; k < reps && st == TMH_OK; ++k)
                st = tmh_hop_apply(l, k % 2 ? TMH_OE : TMH_EO, k % 2 ? in : out, gauge, k % 2 ? out : in, 0.1,
                                   theta, prec);
            float ms = 0.f;
            if (st == TMH_OK && (hipEventRecord(e1, l->stream) != hipSuccess ||
                                 hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                st = TMH_ERR_HIP;
            if (st == TMH_OK) cand_us[ci] = std::min(cand_us[ci], 1e3 * ms / reps);
        }
    }
    for (size_t ci = 0; ci < cands.size(); ++ci)
        if (cand_us[ci] < best) {
            best = cand_us[ci];
            bx = cands[ci];
        }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(l->stream);
    (void)hipFree(in);
    (void)hipFree(out);
    if (st != TMH_OK) {
        l->xgroup = saved;
        l->xgroup_code[prec] = saved_code;
        l->xtuned[prec] = saved_tuned;
        return st;
    }
    l->xgroup = bx;
    l->xgroup_code[prec] = bx;
    *best_xgroup = bx;
    *best_us = best;
    if (cache_path) {
        if (FILE* f = fopen(cache_path, "a")) {
            fprintf(f, "%s %d %.3f\n", key, bx, best);
            fclose(f);
        }
    }
    return TMH_OK;
}

tmh_status tmh_gauge_export(tmh_lattice* l, double* dst, const void* src, tmh_prec prec) {
    TMH_TRY(check_lat(l));
    TMH_TRY(check_prec(prec));
    if (!dst || !src) return TMH_ERR_ARG;
    if (overlap(dst, (size_t)2 * l->g.Vh * 4 * 9 * 16, src, gauge_bytes(l, prec))) return TMH_ERR_ALIAS;
    DeviceGuard guard(l->device);
    const bool r12 = link_format(prec) == 1;
    return dispatch(prec, [&](auto tag) {
        using P = decltype(tag);
        using W = typename tmh::Word<P>::T;
        TMH_TRY_HIP(r12 ? tmh::launch_gauge_export_r12<P>(dst, (const W*)src, l->g, l->stream)
                        : tmh::launch_gauge_export<P>(dst, (const W*)src, l->g, l->stream));
        return TMH_OK;
    });
}

tmh_status tmh_scalar_prod_r(tmh_lattice* l, double* result, const void* a, const void* b, tmh_prec prec) {
    TMH_TRY(check_lat(l));
    TMH_TRY(check_prec(prec));
    if (!result || !a || !b) return TMH_ERR_ARG;
    DeviceGuard guard(l->device);
    return dispatch(prec, [&](auto tag) { return reduce_dot<decltype(tag)>(l, result, a, b); });
}

tmh_status tmh_norm2(tmh_lattice* l, double* result, const void* a, tmh_prec prec) {
    return tmh_scalar_prod_r(l, result, a, a, prec);
}

tmh_status tmh_stream_copy(tmh_lattice* l, void* dst, const void* src, size_t nbytes) {
    TMH_TRY(check_lat(l));
    if (!dst || !src || nbytes % 16 != 0 || ((uintptr_t)dst | (uintptr_t)src) % 16 != 0) return TMH_ERR_ARG;
    if (overlap(dst, nbytes, src, nbytes)) return TMH_ERR_ALIAS;
    DeviceGuard guard(l->device);
    TMH_TRY_HIP(tmh::launch_stream_copy(dst, src, nbytes, l->stream));
    return TMH_OK;
}

tmh_status tmh_profile_enable(tmh_lattice* l, int on) {
    TMH_TRY(check_lat(l));
    DeviceGuard guard(l->device);
    TMH_TRY(prof_flush(l));
    l->prof_on = on != 0;
    for (int k = 0; k < TMH_PROFILE_KINDS; ++k) {
        l->prof_ms[k] = 0.0;
        l->prof_count[k] = 0;
        l->prof_skipped[k] = 0;
    }
    return TMH_OK;
}

tmh_status tmh_profile_read(tmh_lattice* l, int kind, long long* launches, double* total_ms) {
    TMH_TRY(check_lat(l));
    if (kind < 0 || kind >= TMH_PROFILE_KINDS || !launches || !total_ms) return TMH_ERR_ARG;
    DeviceGuard guard(l->device);
    TMH_TRY(prof_flush(l));
    *launches = l->prof_count[kind] - l->prof_skipped[kind];
    *total_ms = l->prof_ms[kind];
    return TMH_OK;
}

const char* tmh_status_string(tmh_status st) {
    switch (st) {
        case TMH_OK: return "ok";
        case TMH_ERR_ARG: return "invalid argument";
        case TMH_ERR_GEOMETRY: return "invalid lattice geometry (extents must be even and >= 2)";
        case TMH_ERR_ALIAS: return "output buffer overlaps an input buffer";
        case TMH_ERR_HIP: return "HIP runtime error";
        case TMH_ERR_NOMEM: return "device allocation failed";
        case TMH_ERR_NOT_CONVERGED: return "CG did not converge within max_iter";
        case TMH_ERR_UNSUPPORTED: return "unsupported precision or feature";
        case TMH_ERR_SCRATCH: return "field larger than the fixed scratch of the allocation-free call";
    }
    return "unknown status";
}

}  // extern "C"
