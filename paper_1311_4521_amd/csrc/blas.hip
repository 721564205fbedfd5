// BLAS-1, deterministic reductions and the CG update kernels.
//
// Reductions are two-pass and run in a fixed order: every workgroup reduces
// its lanes (wave64 shuffles, then the 4 waves through LDS) into one FP64
// partial, and one workgroup sums the partials in index order.  The result
// is therefore bitwise reproducible for a given lattice size.  CG scalars
// (alpha, beta, |r|^2) never leave the device inside the iteration; kernels
// given a `done` flag return at once when it is set, so the host can enqueue
// several iterations ahead and stop on convergence.
#include "common.h"
#include "kernels.h"

namespace tmh {

namespace {

constexpr int kMaxBlasBlocks = 1024;

__device__ __forceinline__ bool is_done(const int* flags) { return flags != nullptr && flags[0] != 0; }

// Sum of partial[0..n) by one workgroup, thread t taking t, t+256, ... in
// order.  Valid in thread 0.
__device__ __forceinline__ double sum_partials(const double* __restrict__ partial, int n) {
    double s = 0.0;
    for (int k = threadIdx.x; k < n; k += kBlock) s += partial[k];
    return block_sum(s);
}

template <typename R>
__global__ void __launch_bounds__(kBlock) dot_partial_kernel(double* __restrict__ partial,
                                                             const typename Word<R>::T* __restrict__ a,
                                                             const typename Word<R>::T* __restrict__ b, Geo g,
                                                             const int* flags) {
    if (is_done(flags)) return;
    double s = 0.0;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < g.Vh; i += gridDim.x * kBlock) {
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            const auto x = a[(int64_t)c * g.S + i];
            const auto y = b[(int64_t)c * g.S + i];
            s += (double)x.x * (double)y.x + (double)x.y * (double)y.y;
        }
    }
    s = block_sum(s);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kBlock) reduce_kernel(double* out, const double* __restrict__ partial, int n,
                                                        const int* flags) {
    if (is_done(flags)) return;
    const double s = sum_partials(partial, n);
    if (threadIdx.x == 0) out[0] = s;
}

__global__ void __launch_bounds__(kBlock) cg_init_kernel(double* scal, const double* __restrict__ partial, int n,
                                                         int* flags, double stop) {
    const double s = sum_partials(partial, n);
    if (threadIdx.x == 0) {
        scal[kRR] = s;
        scal[kStop] = stop;
        flags[0] = s <= stop ? 1 : 0;
        flags[1] = 0;
    }
}

__global__ void __launch_bounds__(kBlock) cg_beta_kernel(double* scal, const double* __restrict__ partial, int n,
                                                         int* flags, int max_iter) {
    if (is_done(flags)) return;
    const double rr = sum_partials(partial, n);
    if (threadIdx.x == 0) {
        scal[kBeta] = rr / scal[kRR];
        scal[kRR] = rr;
        const int it = flags[1] + 1;
        flags[1] = it;
        if (rr <= scal[kStop] || it >= max_iter) flags[0] = 1;
    }
}

// x += alpha p, r -= alpha q, partial |r|^2.
template <typename R>
__global__ void __launch_bounds__(kBlock) cg_xr_kernel(typename Word<R>::T* __restrict__ x,
                                                       typename Word<R>::T* __restrict__ r,
                                                       const typename Word<R>::T* __restrict__ p,
                                                       const typename Word<R>::T* __restrict__ q,
                                                       const double* __restrict__ scal, double* __restrict__ partial,
                                                       Geo g, const int* flags) {
    if (is_done(flags)) return;
    const real_t<R> alpha = (real_t<R>)scal[kAlpha];
    double s = 0.0;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < g.Vh; i += gridDim.x * kBlock) {
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            const int64_t k = (int64_t)c * g.S + i;
            auto xv = x[k];
            auto rv = r[k];
            const auto pv = p[k];
            const auto qv = q[k];
            xv.x += alpha * pv.x;
            xv.y += alpha * pv.y;
            rv.x -= alpha * qv.x;
            rv.y -= alpha * qv.y;
            x[k] = xv;
            r[k] = rv;
            s += (double)rv.x * (double)rv.x + (double)rv.y * (double)rv.y;
        }
    }
    s = block_sum(s);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// p = r + beta p.
template <typename R>
__global__ void __launch_bounds__(kBlock) cg_p_kernel(typename Word<R>::T* __restrict__ p,
                                                      const typename Word<R>::T* __restrict__ r,
                                                      const double* __restrict__ scal, Geo g, const int* flags) {
    if (is_done(flags)) return;
    const real_t<R> beta = (real_t<R>)scal[kBeta];
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < g.Vh; i += gridDim.x * kBlock) {
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            const int64_t k = (int64_t)c * g.S + i;
            auto pv = p[k];
            const auto rv = r[k];
            pv.x = rv.x + beta * pv.x;
            pv.y = rv.y + beta * pv.y;
            p[k] = pv;
        }
    }
}

// End of CG iteration `it` (0-based): x += alpha p, then p = r + beta p.
// Runs only if that iteration ran (flags[1] counts the iterations done), so
// the iteration that reaches the stop criterion still updates x, and the
// iterations enqueued after it return at once.
template <typename R>
__global__ void __launch_bounds__(kBlock) cg_px_kernel(typename Word<R>::T* __restrict__ p,
                                                       typename Word<R>::T* __restrict__ x,
                                                       const typename Word<R>::T* __restrict__ r,
                                                       const double* __restrict__ scal, Geo g, const int* flags,
                                                       int it) {
    if (flags[1] != it + 1) return;
    const real_t<R> alpha = (real_t<R>)scal[kAlpha];
    const real_t<R> beta = (real_t<R>)scal[kBeta];
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < g.Vh; i += gridDim.x * kBlock) {
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            const int64_t k = (int64_t)c * g.S + i;
            auto pv = p[k];
            auto xv = x[k];
            const auto rv = r[k];
            xv.x += alpha * pv.x;
            xv.y += alpha * pv.y;
            pv.x = rv.x + beta * pv.x;
            pv.y = rv.y + beta * pv.y;
            x[k] = xv;
            p[k] = pv;
        }
    }
}

template <typename R>
__global__ void __launch_bounds__(kBlock) sub_norm_kernel(typename Word<R>::T* __restrict__ out,
                                                          const typename Word<R>::T* __restrict__ a,
                                                          const typename Word<R>::T* __restrict__ b,
                                                          double* __restrict__ partial, Geo g) {
    double s = 0.0;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < g.Vh; i += gridDim.x * kBlock) {
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            const int64_t k = (int64_t)c * g.S + i;
            auto v = a[k];
            const auto w = b[k];
            v.x -= w.x;
            v.y -= w.y;
            out[k] = v;
            s += (double)v.x * (double)v.x + (double)v.y * (double)v.y;
        }
    }
    s = block_sum(s);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

template <typename P>
__global__ void __launch_bounds__(kBlock) add_widen_kernel(double2* __restrict__ x,
                                                           const typename Word<P>::T* __restrict__ y, double scale,
                                                           Geo g) {
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < g.Vh; i += gridDim.x * kBlock) {
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            const int64_t k = (int64_t)c * g.S + i;
            double2 v = x[k];
            const auto w = y[k];
            v.x += scale * (double)w.x;
            v.y += scale * (double)w.y;
            x[k] = v;
        }
    }
}

// out_s = c_{s/2} in_s: a site-local function of gamma_5 (upper spins take
// c_up, lower spins c_dn), e.g. (1 +- i mt gamma_5)^-1.
__global__ void __launch_bounds__(kBlock) chiral_scale_kernel(double2* __restrict__ out,
                                                              const double2* __restrict__ in, double cu_re,
                                                              double cu_im, double cd_re, double cd_im, Geo g) {
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < g.Vh; i += gridDim.x * kBlock) {
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            const int64_t k = (int64_t)c * g.S + i;
            const double2 v = in[k];
            const double a = c < 6 ? cu_re : cd_re, b = c < 6 ? cu_im : cd_im;
            out[k] = make_double2(a * v.x - b * v.y, a * v.y + b * v.x);
        }
    }
}

template <typename R>
__global__ void __launch_bounds__(kBlock) copy_kernel(typename Word<R>::T* __restrict__ dst,
                                                      const typename Word<R>::T* __restrict__ src, Geo g) {
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < g.Vh; i += gridDim.x * kBlock) {
#pragma unroll
        for (int c = 0; c < 12; ++c) dst[(int64_t)c * g.S + i] = src[(int64_t)c * g.S + i];
    }
}

template <typename R>
__global__ void __launch_bounds__(kBlock) zero_kernel(typename Word<R>::T* __restrict__ dst, Geo g) {
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < g.Vh; i += gridDim.x * kBlock) {
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            typename Word<R>::T z;
            z.x = 0;
            z.y = 0;
            dst[(int64_t)c * g.S + i] = z;
        }
    }
}

// dst = src for n 16-byte words, 4 words per thread per pass, non-temporal.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
__global__ void __launch_bounds__(kBlock) stream_copy_kernel(u32x4* __restrict__ dst, const u32x4* __restrict__ src,
                                                             int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * kBlock * 4;
    for (int64_t base = (int64_t)blockIdx.x * kBlock * 4 + threadIdx.x; base < n; base += stride) {
        u32x4 v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (base + k * kBlock < n) v[k] = __builtin_nontemporal_load(src + base + k * kBlock);
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (base + k * kBlock < n) __builtin_nontemporal_store(v[k], dst + base + k * kBlock);
    }
}

}  // namespace

hipError_t launch_stream_copy(void* dst, const void* src, size_t nbytes, hipStream_t s) {
    const int64_t n = (int64_t)(nbytes / 16);
    if (n == 0) return hipSuccess;
    int64_t nb = (n + kBlock * 4 - 1) / (kBlock * 4);
    if (nb > 65536) nb = 65536;
    hipLaunchKernelGGL(stream_copy_kernel, dim3((unsigned)nb), dim3(kBlock), 0, s, (u32x4*)dst,
                       (const u32x4*)src, n);
    return hipGetLastError();
}

int blas_blocks(const Geo& g) {
    const int nb = (g.Vh + kBlock - 1) / kBlock;
    return nb < kMaxBlasBlocks ? (nb > 0 ? nb : 1) : kMaxBlasBlocks;
}

template <typename R>
hipError_t launch_dot_partial(double* partial, const typename Word<R>::T* a, const typename Word<R>::T* b,
                              const Geo& g, const int* done, hipStream_t s) {
    hipLaunchKernelGGL((dot_partial_kernel<R>), dim3(blas_blocks(g)), dim3(kBlock), 0, s, partial, a, b, g,
                       done);
    return hipGetLastError();
}

hipError_t launch_reduce(double* out, const double* partial, int n, const int* done, hipStream_t s) {
    hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(kBlock), 0, s, out, partial, n, done);
    return hipGetLastError();
}

hipError_t launch_cg_init(double* scal, const double* partial, int n, int* flags, double stop, hipStream_t s) {
    hipLaunchKernelGGL(cg_init_kernel, dim3(1), dim3(kBlock), 0, s, scal, partial, n, flags, stop);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_cg_xr(typename Word<R>::T* x, typename Word<R>::T* r, const typename Word<R>::T* p,
                        const typename Word<R>::T* q, const double* scal, double* partial, const Geo& g,
                        const int* flags, hipStream_t s) {
    hipLaunchKernelGGL((cg_xr_kernel<R>), dim3(blas_blocks(g)), dim3(kBlock), 0, s, x, r, p, q, scal, partial,
                       g, flags);
    return hipGetLastError();
}

hipError_t launch_cg_beta(double* scal, const double* partial, int n, int* flags, int max_iter, hipStream_t s) {
    hipLaunchKernelGGL(cg_beta_kernel, dim3(1), dim3(kBlock), 0, s, scal, partial, n, flags, max_iter);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_cg_p(typename Word<R>::T* p, const typename Word<R>::T* r, const double* scal, const Geo& g,
                       const int* flags, hipStream_t s) {
    hipLaunchKernelGGL((cg_p_kernel<R>), dim3(blas_blocks(g)), dim3(kBlock), 0, s, p, r, scal, g, flags);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_cg_px(typename Word<R>::T* p, typename Word<R>::T* x, const typename Word<R>::T* r,
                        const double* scal, const Geo& g, const int* flags, int it, hipStream_t s) {
    hipLaunchKernelGGL((cg_px_kernel<R>), dim3(blas_blocks(g)), dim3(kBlock), 0, s, p, x, r, scal, g, flags, it);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_sub_norm(typename Word<R>::T* out, const typename Word<R>::T* a, const typename Word<R>::T* b,
                           double* partial, const Geo& g, hipStream_t s) {
    hipLaunchKernelGGL((sub_norm_kernel<R>), dim3(blas_blocks(g)), dim3(kBlock), 0, s, out, a, b, partial, g);
    return hipGetLastError();
}

hipError_t launch_chiral_scale(double2* out, const double2* in, double cu_re, double cu_im, double cd_re,
                               double cd_im, const Geo& g, hipStream_t s) {
    hipLaunchKernelGGL(chiral_scale_kernel, dim3(blas_blocks(g)), dim3(kBlock), 0, s, out, in, cu_re, cu_im, cd_re,
                       cd_im, g);
    return hipGetLastError();
}

template <typename P>
hipError_t launch_add_widen(double2* x, const typename Word<P>::T* y, double scale, const Geo& g, hipStream_t s) {
    hipLaunchKernelGGL((add_widen_kernel<P>), dim3(blas_blocks(g)), dim3(kBlock), 0, s, x, y, scale, g);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_copy(typename Word<R>::T* dst, const typename Word<R>::T* src, const Geo& g, hipStream_t s) {
    hipLaunchKernelGGL((copy_kernel<R>), dim3(blas_blocks(g)), dim3(kBlock), 0, s, dst, src, g);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_zero(typename Word<R>::T* dst, const Geo& g, hipStream_t s) {
    hipLaunchKernelGGL((zero_kernel<R>), dim3(blas_blocks(g)), dim3(kBlock), 0, s, dst, g);
    return hipGetLastError();
}

#define TMH_INST(R)                                                                                          \
    template hipError_t launch_dot_partial<R>(double*, const Word<R>::T*, const Word<R>::T*, const Geo&,     \
                                              const int*, hipStream_t);                                      \
    template hipError_t launch_cg_xr<R>(Word<R>::T*, Word<R>::T*, const Word<R>::T*, const Word<R>::T*,       \
                                        const double*, double*, const Geo&, const int*, hipStream_t);         \
    template hipError_t launch_cg_p<R>(Word<R>::T*, const Word<R>::T*, const double*, const Geo&, const int*, \
                                       hipStream_t);                                                         \
    template hipError_t launch_cg_px<R>(Word<R>::T*, Word<R>::T*, const Word<R>::T*, const double*,           \
                                        const Geo&, const int*, int, hipStream_t);                           \
    template hipError_t launch_sub_norm<R>(Word<R>::T*, const Word<R>::T*, const Word<R>::T*, double*,        \
                                           const Geo&, hipStream_t);                                         \
    template hipError_t launch_copy<R>(Word<R>::T*, const Word<R>::T*, const Geo&, hipStream_t);              \
    template hipError_t launch_zero<R>(Word<R>::T*, const Geo&, hipStream_t);

TMH_INST(double)
TMH_INST(float)
TMH_INST(half_t)
#undef TMH_INST
template hipError_t launch_add_widen<float>(double2*, const float2*, double, const Geo&, hipStream_t);
template hipError_t launch_add_widen<half_t>(double2*, const h2*, double, const Geo&, hipStream_t);

}  // namespace tmh
