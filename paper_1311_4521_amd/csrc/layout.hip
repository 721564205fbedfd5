// Canonical <-> internal layout conversion and precision conversion.
//
// Canonical (FP64, device): gauge [4][V][3][3] by lex site, spinor [Vh][4][3].
// Internal: structure of arrays with site stride S (see tmhop.h): every
// complex component is its own array of S words, so the 64 lanes of a wave
// touching 64 consecutive sites read one contiguous segment.
#include "common.h"
#include "kernels.h"

namespace tmh {

namespace {

// FP64 -> storage word of P, one rounding to nearest even.
template <typename P> __device__ __forceinline__ typename Word<P>::T cvt(double re, double im) {
    typename Word<P>::T w;
    w.x = static_cast<decltype(w.x)>(re);
    w.y = static_cast<decltype(w.y)>(im);
    return w;
}

// One thread per (mu, lex site): the 9 link entries go to the parity block
// and even-odd index of that site.
template <typename R>
__global__ void __launch_bounds__(kBlock) gauge_import_kernel(typename Word<R>::T* __restrict__ dst,
                                                              const double2* __restrict__ src, Geo g,
                                                              int64_t V) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= 4 * V) return;
    const int mu = (int)(t / V);
    const int64_t lex = t - (int64_t)mu * V;
    int64_t r = lex;
    const int z = (int)(r % g.L[3]);
    r /= g.L[3];
    const int y = (int)(r % g.L[2]);
    r /= g.L[2];
    const int x = (int)(r % g.L[1]);
    const int tt = (int)(r / g.L[1]);
    const int p = (tt + x + y + z) & 1;
    const int i = (int)(lex >> 1);
    const double2* s = src + t * 9;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const double2 v = s[k];
        dst[((int64_t)(p * 4 + mu) * 9 + k) * g.S + i] = cvt<R>(v.x, v.y);
    }
}

template <typename R>
__global__ void __launch_bounds__(kBlock) gauge_export_kernel(double2* __restrict__ dst,
                                                              const typename Word<R>::T* __restrict__ src, Geo g,
                                                              int64_t V) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= 4 * V) return;
    const int mu = (int)(t / V);
    const int64_t lex = t - (int64_t)mu * V;
    int64_t r = lex;
    const int z = (int)(r % g.L[3]);
    r /= g.L[3];
    const int y = (int)(r % g.L[2]);
    r /= g.L[2];
    const int x = (int)(r % g.L[1]);
    const int tt = (int)(r / g.L[1]);
    const int p = (tt + x + y + z) & 1;
    const int i = (int)(lex >> 1);
    double2* d = dst + t * 9;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const typename Word<R>::T v = src[((int64_t)(p * 4 + mu) * 9 + k) * g.S + i];
        d[k] = make_double2((double)v.x, (double)v.y);
    }
}

template <typename R>
__global__ void __launch_bounds__(kBlock) spinor_import_kernel(typename Word<R>::T* __restrict__ dst,
                                                               const double2* __restrict__ src, Geo g) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= g.Vh) return;
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        const double2 v = src[(int64_t)i * 12 + c];
        dst[(int64_t)c * g.S + i] = cvt<R>(v.x, v.y);
    }
}

template <typename R>
__global__ void __launch_bounds__(kBlock) spinor_export_kernel(double2* __restrict__ dst,
                                                               const typename Word<R>::T* __restrict__ src,
                                                               Geo g) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= g.Vh) return;
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        const typename Word<R>::T v = src[(int64_t)c * g.S + i];
        dst[(int64_t)i * 12 + c] = make_double2((double)v.x, (double)v.y);
    }
}

// Canonical links -> two-row storage: rows 0 and 1 of U_mu(x) (6 complexes)
// at ((p*4 + mu)*6 + 3a + b)*S + i.
template <typename R>
__global__ void __launch_bounds__(kBlock) gauge_import_r12_kernel(typename Word<R>::T* __restrict__ dst,
                                                                  const double2* __restrict__ src, Geo g, int64_t V) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= 4 * V) return;
    const int mu = (int)(t / V);
    const int64_t lex = t - (int64_t)mu * V;
    int64_t r = lex;
    const int z = (int)(r % g.L[3]);
    r /= g.L[3];
    const int y = (int)(r % g.L[2]);
    r /= g.L[2];
    const int x = (int)(r % g.L[1]);
    const int tt = (int)(r / g.L[1]);
    const int p = (tt + x + y + z) & 1;
    const int i = (int)(lex >> 1);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const double2 v = src[t * 9 + k];
        dst[((int64_t)(p * 4 + mu) * 6 + k) * g.S + i] = cvt<R>(v.x, v.y);
    }
}

// Two-row storage -> canonical links, the third row rebuilt.
template <typename R>
__global__ void __launch_bounds__(kBlock) gauge_export_r12_kernel(double2* __restrict__ dst,
                                                                  const typename Word<R>::T* __restrict__ src, Geo g,
                                                                  int64_t V) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= 4 * V) return;
    const int mu = (int)(t / V);
    const int64_t lex = t - (int64_t)mu * V;
    int64_t r = lex;
    const int z = (int)(r % g.L[3]);
    r /= g.L[3];
    const int y = (int)(r % g.L[2]);
    r /= g.L[2];
    const int x = (int)(r % g.L[1]);
    const int tt = (int)(r / g.L[1]);
    const int p = (tt + x + y + z) & 1;
    const int i = (int)(lex >> 1);
    cx<double> u[3][3];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const typename Word<R>::T v = src[((int64_t)(p * 4 + mu) * 6 + k) * g.S + i];
        u[k / 3][k % 3] = mk<double>((double)v.x, (double)v.y);
    }
    const cx<double> c0 = u[0][1] * u[1][2] - u[0][2] * u[1][1];
    const cx<double> c1 = u[0][2] * u[1][0] - u[0][0] * u[1][2];
    const cx<double> c2 = u[0][0] * u[1][1] - u[0][1] * u[1][0];
    u[2][0] = mk<double>(c0.re, -c0.im);
    u[2][1] = mk<double>(c1.re, -c1.im);
    u[2][2] = mk<double>(c2.re, -c2.im);
#pragma unroll
    for (int k = 0; k < 9; ++k) dst[t * 9 + k] = make_double2(u[k / 3][k % 3].re, u[k / 3][k % 3].im);
}

// Internal full FP64 links -> two-row links, one thread per even-odd index
// (its 8 links: both parities, 4 directions); per-block maximum deviation of
// the stored third row from the rebuilt one into partial[blockIdx.x].
template <typename R>
__global__ void __launch_bounds__(kBlock) compress_links_kernel(typename Word<R>::T* __restrict__ dst,
                                                                const double2* __restrict__ src,
                                                                double* __restrict__ partial, Geo g) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    double dev = 0.0;
    if (i < g.Vh) {
        for (int pm = 0; pm < 8; ++pm) {  // parity * 4 + mu
            cx<double> u[3][3];
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                const double2 v = src[((int64_t)pm * 9 + k) * g.S + i];
                u[k / 3][k % 3] = mk<double>(v.x, v.y);
            }
#pragma unroll
            for (int k = 0; k < 6; ++k)
                dst[((int64_t)pm * 6 + k) * g.S + i] = cvt<R>(u[k / 3][k % 3].re, u[k / 3][k % 3].im);
            const cx<double> c0 = u[0][1] * u[1][2] - u[0][2] * u[1][1];
            const cx<double> c1 = u[0][2] * u[1][0] - u[0][0] * u[1][2];
            const cx<double> c2 = u[0][0] * u[1][1] - u[0][1] * u[1][0];
            const double d = fmax(fmax(fabs(c0.re - u[2][0].re), fabs(-c0.im - u[2][0].im)),
                                  fmax(fmax(fabs(c1.re - u[2][1].re), fabs(-c1.im - u[2][1].im)),
                                       fmax(fabs(c2.re - u[2][2].re), fabs(-c2.im - u[2][2].im))));
            dev = (d == d) ? fmax(dev, d) : INFINITY;  // a NaN entry fails the check
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) dev = fmax(dev, __shfl_xor(dev, off, 64));
    __shared__ double wmax[kBlock / 64];
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = dev;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = 0.0;
#pragma unroll
        for (int w = 0; w < kBlock / 64; ++w) m = fmax(m, wmax[w]);
        partial[blockIdx.x] = m;
    }
}

__global__ void __launch_bounds__(kBlock) reduce_max_kernel(double* out, const double* __restrict__ partial, int n) {
    double m = 0.0;
    for (int k = threadIdx.x; k < n; k += kBlock) m = fmax(m, partial[k]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
    __shared__ double wmax[kBlock / 64];
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = 0.0;
#pragma unroll
        for (int w = 0; w < kBlock / 64; ++w) r = fmax(r, wmax[w]);
        out[0] = r;
    }
}

template <typename P>
__global__ void __launch_bounds__(kBlock) narrow_kernel(typename Word<P>::T* __restrict__ dst,
                                                        const double2* __restrict__ src, int ncomp, double scale,
                                                        Geo g) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= g.Vh) return;
    for (int c = 0; c < ncomp; ++c) {
        const double2 v = src[(int64_t)c * g.S + i];
        dst[(int64_t)c * g.S + i] = cvt<P>(scale * v.x, scale * v.y);
    }
}

inline int nblocks(int64_t n) { return (int)((n + kBlock - 1) / kBlock); }

}  // namespace

template <typename R>
hipError_t launch_gauge_import(typename Word<R>::T* dst, const double* src, const Geo& g, hipStream_t s) {
    const int64_t V = 2 * (int64_t)g.Vh;
    if (V == 0) return hipSuccess;
    hipLaunchKernelGGL((gauge_import_kernel<R>), dim3(nblocks(4 * V)), dim3(kBlock), 0, s, dst,
                       (const double2*)src, g, V);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_gauge_export(double* dst, const typename Word<R>::T* src, const Geo& g, hipStream_t s) {
    const int64_t V = 2 * (int64_t)g.Vh;
    if (V == 0) return hipSuccess;
    hipLaunchKernelGGL((gauge_export_kernel<R>), dim3(nblocks(4 * V)), dim3(kBlock), 0, s, (double2*)dst, src,
                       g, V);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_spinor_import(typename Word<R>::T* dst, const double* src, const Geo& g, hipStream_t s) {
    if (g.Vh == 0) return hipSuccess;
    hipLaunchKernelGGL((spinor_import_kernel<R>), dim3(nblocks(g.Vh)), dim3(kBlock), 0, s, dst,
                       (const double2*)src, g);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_spinor_export(double* dst, const typename Word<R>::T* src, const Geo& g, hipStream_t s) {
    if (g.Vh == 0) return hipSuccess;
    hipLaunchKernelGGL((spinor_export_kernel<R>), dim3(nblocks(g.Vh)), dim3(kBlock), 0, s, (double2*)dst,
                       src, g);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_gauge_import_r12(typename Word<R>::T* dst, const double* src, const Geo& g, hipStream_t s) {
    const int64_t V = 2 * (int64_t)g.Vh;
    if (V == 0) return hipSuccess;
    hipLaunchKernelGGL((gauge_import_r12_kernel<R>), dim3(nblocks(4 * V)), dim3(kBlock), 0, s, dst,
                       (const double2*)src, g, V);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_gauge_export_r12(double* dst, const typename Word<R>::T* src, const Geo& g, hipStream_t s) {
    const int64_t V = 2 * (int64_t)g.Vh;
    if (V == 0) return hipSuccess;
    hipLaunchKernelGGL((gauge_export_r12_kernel<R>), dim3(nblocks(4 * V)), dim3(kBlock), 0, s, (double2*)dst, src,
                       g, V);
    return hipGetLastError();
}

int link_check_blocks(const Geo& g) { return nblocks(g.Vh); }

template <typename R>
hipError_t launch_compress_links(typename Word<R>::T* dst, const double2* src, double* partial, const Geo& g,
                                 hipStream_t s) {
    if (g.Vh == 0) return hipSuccess;
    hipLaunchKernelGGL((compress_links_kernel<R>), dim3(nblocks(g.Vh)), dim3(kBlock), 0, s, dst, src, partial, g);
    return hipGetLastError();
}

hipError_t launch_reduce_max(double* out, const double* partial, int n, hipStream_t s) {
    hipLaunchKernelGGL(reduce_max_kernel, dim3(1), dim3(kBlock), 0, s, out, partial, n);
    return hipGetLastError();
}

template hipError_t launch_gauge_import_r12<double>(double2*, const double*, const Geo&, hipStream_t);
template hipError_t launch_gauge_import_r12<float>(float2*, const double*, const Geo&, hipStream_t);
template hipError_t launch_gauge_export_r12<double>(double*, const double2*, const Geo&, hipStream_t);
template hipError_t launch_gauge_export_r12<float>(double*, const float2*, const Geo&, hipStream_t);
template hipError_t launch_compress_links<double>(double2*, const double2*, double*, const Geo&, hipStream_t);
template hipError_t launch_compress_links<float>(float2*, const double2*, double*, const Geo&, hipStream_t);

template <typename P>
hipError_t launch_narrow(typename Word<P>::T* dst, const double2* src, int ncomp, double scale, const Geo& g,
                         hipStream_t s) {
    if (g.Vh == 0) return hipSuccess;
    hipLaunchKernelGGL((narrow_kernel<P>), dim3(nblocks(g.Vh)), dim3(kBlock), 0, s, dst, src, ncomp, scale, g);
    return hipGetLastError();
}

template hipError_t launch_gauge_import<double>(double2*, const double*, const Geo&, hipStream_t);
template hipError_t launch_gauge_import<float>(float2*, const double*, const Geo&, hipStream_t);
template hipError_t launch_gauge_export<double>(double*, const double2*, const Geo&, hipStream_t);
template hipError_t launch_gauge_export<float>(double*, const float2*, const Geo&, hipStream_t);
template hipError_t launch_spinor_import<double>(double2*, const double*, const Geo&, hipStream_t);
template hipError_t launch_spinor_import<float>(float2*, const double*, const Geo&, hipStream_t);
template hipError_t launch_spinor_export<double>(double*, const double2*, const Geo&, hipStream_t);
template hipError_t launch_spinor_export<float>(double*, const float2*, const Geo&, hipStream_t);
template hipError_t launch_gauge_import<half_t>(h2*, const double*, const Geo&, hipStream_t);
template hipError_t launch_gauge_export<half_t>(double*, const h2*, const Geo&, hipStream_t);
template hipError_t launch_spinor_import<half_t>(h2*, const double*, const Geo&, hipStream_t);
template hipError_t launch_spinor_export<half_t>(double*, const h2*, const Geo&, hipStream_t);
template hipError_t launch_gauge_import_r12<half_t>(h2*, const double*, const Geo&, hipStream_t);
template hipError_t launch_gauge_export_r12<half_t>(double*, const h2*, const Geo&, hipStream_t);
template hipError_t launch_compress_links<half_t>(h2*, const double2*, double*, const Geo&, hipStream_t);
template hipError_t launch_narrow<float>(float2*, const double2*, int, double, const Geo&, hipStream_t);
template hipError_t launch_narrow<half_t>(h2*, const double2*, int, double, const Geo&, hipStream_t);

}  // namespace tmh
