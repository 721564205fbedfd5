// Host-side launch interface of the device kernels (internal to libtmhop).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace tmh {

// Traversal code of the hop kernels for one x-slab per XCD (see hop.hip).
constexpr int kXSlab = -8;
// Traversal codes of the t-marching hop kernel: kTMarch0 - steps.
constexpr int kTMarch0 = -1024;

// Arguments of one hopping-matrix launch on fields of storage precision P
// (double, float or half_t), arithmetic in real_t<P>.
template <typename P> struct HopArgs {
    using R = real_t<P>;
    typename Word<P>::T* out;
    const typename Word<P>::T* in;
    const typename Word<P>::T* gout;  // links U_mu(x) of the output parity
    const typename Word<P>::T* gin;   // links U_mu(y) of the input parity
    const typename Word<P>::T* aux;   // MODE >= 1: field added at the output site
    double* partial;                  // MODE 2: per-workgroup |out|^2; MODE 3: |r|^2
    typename Word<P>::T* rio;         // MODE 3, 4: r -= alpha out (out itself is not stored)
    typename Word<P>::T* xio;         // MODE 4: x += alpha p
    const typename Word<P>::T* pin;   // MODE 4: p
    const double* scal;               // MODE 3: alpha = scal[kAlpha]
    const double* apart;              // MODE 0, optional: workgroup 0 also sets the CG step,
    int napart;                       //   ascal[kAlpha] = ascal[kRR] / sum of apart[0..napart)
    double* ascal;
    const int* done;                  // optional device flag: skip when set
    Geo g;
    int pout;                         // parity of the output sites
    int lf;                           // link storage: 0 = 9 entries, 1 = two rows (12 reals)
    int xgroup, nyb, nt;              // traversal order (see hop.hip), xgroup = 0: eo order
    int tm_steps;                     // > 0: t-marching kernel, each workgroup walks tm_steps time-slices
    int tm_nw;                        //   workgroup tiles per time-slice (tm_slice / kHopThreads)
    int tm_slice;                     //   sites per parity in one time-slice, LX LY LZ / 2
    R ph_re[4], ph_im[4];             // exp(i pi theta_mu)
    R c_re[2], c_im[2];               // coefficient of the hopping sum, upper/lower spins
    R d_re[2], d_im[2];               // coefficient of aux, upper/lower spins
};

// Gauge-link derivative of Re <X, H Y> (force.hip): FP64 fields, the force
// in the internal gauge layout, force += coeff * (TA(M) | Euclidean gradient).
struct ForceArgs {
    double2* force;
    const double2* gauge;
    const double2* X;      // on the output parity of H
    const double2* Y;      // on the input parity of H
    Geo g;
    int pout;              // output parity of H
    int kind;              // 0: su(3) force TA(M), 1: Euclidean gradient
    double kappa, coeff;
    double ph_re[4], ph_im[4];
    double cx_re[2], cx_im[2];  // X_eff = c_{s/2} X_s
};
hipError_t launch_force(const ForceArgs& a, hipStream_t s);
// The derivatives of two bilinears Re <X_k, H_k Y_k> (k = 0, 1) whose hopping
// matrices map opposite parities (a.pout = 1 - b.pout), summed per link
// before the one read-modify-write of the force; gauge, force, g, kind and
// phases are taken from a.
hipError_t launch_force2(const ForceArgs& a, const ForceArgs& b, hipStream_t s);

int hop_blocks(const Geo& g);
// Workgroups of a t-marching hop launch (tm_steps > 0).
int hop_tmarch_blocks(const Geo& g, int steps);
constexpr int kHopThreads = 256;  // workgroup size of hop_kernel (TMH_HOP_BLOCK)
template <typename R> hipError_t launch_hop(const HopArgs<R>& a, int mode, hipStream_t s);

// Layout conversion (layout.hip).
template <typename R>
hipError_t launch_gauge_import(typename Word<R>::T* dst, const double* src, const Geo& g, hipStream_t s);
template <typename R>
hipError_t launch_spinor_import(typename Word<R>::T* dst, const double* src, const Geo& g, hipStream_t s);
template <typename R>
hipError_t launch_spinor_export(double* dst, const typename Word<R>::T* src, const Geo& g, hipStream_t s);
template <typename R>
hipError_t launch_gauge_export(double* dst, const typename Word<R>::T* src, const Geo& g, hipStream_t s);
template <typename R>
hipError_t launch_gauge_import_r12(typename Word<R>::T* dst, const double* src, const Geo& g, hipStream_t s);
template <typename R>
hipError_t launch_gauge_export_r12(double* dst, const typename Word<R>::T* src, const Geo& g, hipStream_t s);
// Internal full FP64 links -> two-row links of type R, with the per-block
// maximum of |conj(row0 x row1) - row2| over the links in partial[]
// (link_check_blocks(g) entries, no more than hop_blocks(g)).
template <typename R>
hipError_t launch_compress_links(typename Word<R>::T* dst, const double2* src, double* partial, const Geo& g,
                                 hipStream_t s);
int link_check_blocks(const Geo& g);
// out[0] = max(partial[0..n))
hipError_t launch_reduce_max(double* out, const double* partial, int n, hipStream_t s);
// Internal FP64 -> storage of P (spinor: ncomp = 12, gauge: ncomp = 72),
// every value multiplied by `scale` first.
template <typename P>
hipError_t launch_narrow(typename Word<P>::T* dst, const double2* src, int ncomp, double scale, const Geo& g,
                         hipStream_t s);

// BLAS-1 and reductions (blas.hip).  All reductions write per-workgroup
// partials; reduce_partials sums them in a fixed order into out[0].
int blas_blocks(const Geo& g);
template <typename R>
hipError_t launch_dot_partial(double* partial, const typename Word<R>::T* a, const typename Word<R>::T* b,
                              const Geo& g, const int* done, hipStream_t s);
hipError_t launch_reduce(double* out, const double* partial, int n, const int* done, hipStream_t s);

// CG building blocks on one parity.  scal[] holds the device scalars
// (see CgScal), flags[] = {done, iterations}.
enum CgScal { kRR = 0, kPQ = 1, kAlpha = 2, kBeta = 3, kStop = 4, kRRNew = 5, kNorm = 6, kBB = 7, kNScal = 8 };
template <typename R>
hipError_t launch_cg_xr(typename Word<R>::T* x, typename Word<R>::T* r, const typename Word<R>::T* p,
                        const typename Word<R>::T* q, const double* scal, double* partial, const Geo& g,
                        const int* flags, hipStream_t s);
hipError_t launch_cg_beta(double* scal, const double* partial, int n, int* flags, int max_iter,
                          hipStream_t s);
// p = r + beta p (skipped once the CG is done).
template <typename R>
hipError_t launch_cg_p(typename Word<R>::T* p, const typename Word<R>::T* r, const double* scal,
                       const Geo& g, const int* flags, hipStream_t s);
// x += alpha p, p = r + beta p, if CG iteration `it` (0-based) ran.
template <typename R>
hipError_t launch_cg_px(typename Word<R>::T* p, typename Word<R>::T* x, const typename Word<R>::T* r,
                        const double* scal, const Geo& g, const int* flags, int it, hipStream_t s);
// out = a - b, with |out|^2 partials (true residual).
template <typename R>
hipError_t launch_sub_norm(typename Word<R>::T* out, const typename Word<R>::T* a,
                           const typename Word<R>::T* b, double* partial, const Geo& g, hipStream_t s);
// out_s = c_up in_s (spins 0,1) or c_dn in_s (spins 2,3), FP64.
hipError_t launch_chiral_scale(double2* out, const double2* in, double cu_re, double cu_im, double cd_re,
                               double cd_im, const Geo& g, hipStream_t s);
// x += scale * y (FP64 x, y of storage P): defect-correction update.
template <typename P>
hipError_t launch_add_widen(double2* x, const typename Word<P>::T* y, double scale, const Geo& g, hipStream_t s);
template <typename R>
hipError_t launch_copy(typename Word<R>::T* dst, const typename Word<R>::T* src, const Geo& g, hipStream_t s);
template <typename R>
hipError_t launch_zero(typename Word<R>::T* dst, const Geo& g, hipStream_t s);
// Streaming device copy of nbytes (a multiple of 16): bandwidth reference.
hipError_t launch_stream_copy(void* dst, const void* src, size_t nbytes, hipStream_t s);
// Copies src to dst and resets the CG scalars: scal[kRR] = |src|^2 from the
// given partials, flags = {0, 0}.
hipError_t launch_cg_init(double* scal, const double* partial, int n, int* flags, double stop,
                          hipStream_t s);

// ----------------------------------------------------------------- batches
// (batch.hip) A batch task is one lattice with nrhs fields stored back to
// back; systems are numbered across tasks (sys0 = first system of a task),
// CG scalars live at scal[sys * kNScal], flags at flags[2 * sys].
// A tile shape: SW waves of 64 sites x RY wave groups, each thread applying
// every link it loads to NR right-hand sides (an item holds RY * NR of them).
enum BatchShapeId {
    kShape4x1 = 0,
    kShape2x2 = 1,
    kShape1x4 = 2,
    kShape2x4 = 3,
    kShape1x12 = 4,
    kShape2x1r2 = 5,
    kShape1x2r2 = 6,
    kShape2x2r2 = 7,
    kShape1x4r3 = 8,
    kShape2x2r3 = 9,
    kShape1x3r4 = 10,
    kShape2x1r4 = 11,
    kShapeMfma = 12,  // 64 sites x 8 right-hand sides, link products on the matrix cores
    kShapeTMarch = 13,      // t-march: a workgroup walks time-slices for one tile and one rhs
    kShapeTMarchPipe = 14,  // the same, loads of the next term issued before each term
    kShapeTMarch4 = 15,     // t-march: a workgroup walks time-slices for 64 pairs and 4 rhs
    kShapeTMarchLds = 16,   // the same, each step's links staged once in LDS for the 4 rhs
    kNumShapes = 17
};
void batch_shape(int shape, int* sites_waves, int* wave_groups, int* rhs_per_thread);
inline bool batch_is_tmarch(int shape) {
    return shape == kShapeTMarch || shape == kShapeTMarchPipe || shape == kShapeTMarch4 || shape == kShapeTMarchLds;
}
// Right-hand sides of one t-march workgroup (its 256 threads are 256 / rg
// pairs times rg right-hand sides).
inline int batch_tmarch_rg(int shape) { return (shape == kShapeTMarch4 || shape == kShapeTMarchLds) ? 4 : 1; }
// Workgroups of a t-march launch of one task.
__host__ __device__ inline int batch_tmarch_blocks(int T, int steps, int nw, int nrhs, int rg) {
    return T / steps * nw * ((nrhs + rg - 1) / rg);
}
int batch_rhs_per_item(int shape);

template <typename R> struct BatchHopTask {
    typename Word<R>::T* out;
    const typename Word<R>::T* in;
    const typename Word<R>::T* aux;
    const typename Word<R>::T* gout;
    const typename Word<R>::T* gin;
    double* partial;       // MODE 2, 3: partial[sys * pstride + tile]
    const int* flags;      // optional: skip system when flags[2 * sys] != 0
    typename Word<R>::T* rio;            // MODE 3: r -= alpha q (q not stored)
    typename Word<R>::T* xio;            // MODE 3: x += alpha p
    const typename Word<R>::T* pin;      // MODE 3: p
    const double* scal;                  // MODE 3: alpha = scal[sys * kNScal + kAlpha]
    int64_t fstride;       // words between the fields of consecutive right-hand sides
    int64_t pstride;
    Geo g;
    int pout, nrhs, sys0, item0;
    // tile order: xgroup = 0 visits tiles in even-odd order; xgroup > 0
    // visits each eighth of the time-slices (nt of them) x-group by x-group,
    // nyt tiles filling one (t, x) plane
    int xgroup, nyt, nt;
    // t-march shapes: each workgroup walks tm_steps time-slices of one tile
    // of 256 / tm_rg pairs (tm_nw tiles per slice of tm_slice pairs) for
    // tm_rg right-hand sides
    int tm_steps, tm_nw, tm_slice, tm_rg;
    R ph_re[4], ph_im[4], c_re[2], c_im[2], d_re[2], d_im[2];
};
constexpr int kMaxBatchTasks = 8;  // lattices per batch (task tables travel as kernel arguments)
template <typename R> struct BatchHopTable {
    BatchHopTask<R> t[kMaxBatchTasks];
    int ntasks;
};
template <typename R>
hipError_t launch_batch_hop(const BatchHopTable<R>& tasks, int nitems, int shape, int mode, hipStream_t s);

struct BatchVecTask {
    double2* a;
    double2* b;
    const double2* c;
    const double2* d;
    double* partial;
    int64_t fstride, pstride;
    int Vh, S, nrhs, ntile, sys0, item0;
};
// op 0: x += alpha p, r -= alpha q (+|r|^2); 1: p = r + beta p; 2: r = b - q (+|r|^2);
// 3: |c|^2 partials; 4: a = c
struct BatchVecTable {
    BatchVecTask t[kMaxBatchTasks];
    int ntasks;
};
hipError_t launch_batch_vec(int op, const BatchVecTable& tasks, int nitems, const double* scal, const int* flags,
                            hipStream_t s);
int batch_vec_tiles(int Vh);
// Queries (once) the resident workgroups of every batch kernel of this shape,
// so that later launches, also under graph capture, query nothing.
void batch_prepare(int shape);

// Partial-sum counts per task: systems sys0 .. sys0 + nrhs - 1 of task k sum
// ntile_hop partials after a MODE 2 or 3 hop and ntile_vec after a vector kernel.
struct BatchSysTable {
    int sys0[kMaxBatchTasks], nrhs[kMaxBatchTasks], ntile_hop[kMaxBatchTasks], ntile_vec[kMaxBatchTasks];
    int ntasks;
};
// op 0: alpha; 1: beta + flags; 2: scal[kNorm] = sum; 3: CG init; 4: scal[kBB] = sum
hipError_t launch_batch_scalar(int op, int nsys, const BatchSysTable& sys, double* scal, int* flags,
                               const double* partial, int64_t pstride, double tol2, int max_iter, hipStream_t s);

}  // namespace tmh
