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

template <typename R> __device__ __forceinline__ typename Word<R>::T cvt(double re, double im) {
    typename Word<R>::T w;
    w.x = (R)re;
    w.y = (R)im;
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

__global__ void __launch_bounds__(kBlock) narrow_kernel(float2* __restrict__ dst, const double2* __restrict__ src,
                                                        int ncomp, Geo g) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= g.Vh) return;
    for (int c = 0; c < ncomp; ++c) {
        const double2 v = src[(int64_t)c * g.S + i];
        dst[(int64_t)c * g.S + i] = make_float2((float)v.x, (float)v.y);
    }
}

__global__ void __launch_bounds__(kBlock) widen_kernel(double2* __restrict__ dst, const float2* __restrict__ src,
                                                       int ncomp, Geo g) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= g.Vh) return;
    for (int c = 0; c < ncomp; ++c) {
        const float2 v = src[(int64_t)c * g.S + i];
        dst[(int64_t)c * g.S + i] = make_double2((double)v.x, (double)v.y);
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

hipError_t launch_narrow(float2* dst, const double2* src, int ncomp, const Geo& g, hipStream_t s) {
    if (g.Vh == 0) return hipSuccess;
    hipLaunchKernelGGL(narrow_kernel, dim3(nblocks(g.Vh)), dim3(kBlock), 0, s, dst, src, ncomp, g);
    return hipGetLastError();
}

hipError_t launch_widen(double2* dst, const float2* src, int ncomp, const Geo& g, hipStream_t s) {
    if (g.Vh == 0) return hipSuccess;
    hipLaunchKernelGGL(widen_kernel, dim3(nblocks(g.Vh)), dim3(kBlock), 0, s, dst, src, ncomp, g);
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

}  // namespace tmh
