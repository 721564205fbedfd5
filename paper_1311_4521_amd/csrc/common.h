// Internal device helpers of libtmhop: complex words, lattice geometry,
// deterministic block reductions and the XCD-aware block mapping.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tmh {

constexpr int kBlock = 256;  // threads per workgroup (4 wave64s)
constexpr int kXcds = 8;     // MI355X: 8 XCDs, workgroups dealt round-robin

// Storage precision P of a field: double and float store and compute in
// that type; half_t stores FP16 and computes in FP32.
struct half_t {};
template <typename P> struct Math { using R = P; };
template <> struct Math<half_t> { using R = float; };
template <typename P> using real_t = typename Math<P>::R;

// Storage word of one complex number.
struct alignas(4) h2 {
    _Float16 x, y;
};
template <typename R> struct Word;
template <> struct Word<double> { using T = double2; };
template <> struct Word<float> { using T = float2; };
template <> struct Word<half_t> { using T = h2; };

template <typename R> struct cx {
    R re, im;
};

template <typename R> __device__ __forceinline__ cx<R> mk(R re, R im) { return {re, im}; }
template <typename R> __device__ __forceinline__ cx<R> operator+(cx<R> a, cx<R> b) {
    return {a.re + b.re, a.im + b.im};
}
template <typename R> __device__ __forceinline__ cx<R> operator-(cx<R> a, cx<R> b) {
    return {a.re - b.re, a.im - b.im};
}
template <typename R> __device__ __forceinline__ cx<R> operator*(cx<R> a, cx<R> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R> __device__ __forceinline__ cx<R> operator*(R s, cx<R> a) {
    return {s * a.re, s * a.im};
}
// i * a
template <typename R> __device__ __forceinline__ cx<R> mul_i(cx<R> a) { return {-a.im, a.re}; }
// conj(a) * b
template <typename R> __device__ __forceinline__ cx<R> cmul(cx<R> a, cx<R> b) {
    return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
template <typename R> __device__ __forceinline__ void operator+=(cx<R>& a, cx<R> b) {
    a.re += b.re;
    a.im += b.im;
}
template <typename R> __device__ __forceinline__ void operator-=(cx<R>& a, cx<R> b) {
    a.re -= b.re;
    a.im -= b.im;
}

template <typename R>
__device__ __forceinline__ cx<R> ld(const typename Word<R>::T* __restrict__ p, int64_t k) {
    typename Word<R>::T w = p[k];
    return {w.x, w.y};
}
template <typename R>
__device__ __forceinline__ void st(typename Word<R>::T* __restrict__ p, int64_t k, cx<R> v) {
    typename Word<R>::T w;
    w.x = v.re;
    w.y = v.im;
    p[k] = w;
}

// Spin algebra of the chiral basis.
// e_mu applied to the lower spin pair (p2, p3) of the chiral basis:
// e_0 = -1, e_1 = -i sigma_1, e_2 = -i sigma_2, e_3 = -i sigma_3.
template <typename R, int MU>
__device__ __forceinline__ void e_lower(cx<R> p2, cx<R> p3, cx<R>& r0, cx<R>& r1) {
    if constexpr (MU == 0) {
        r0 = mk<R>(-p2.re, -p2.im);
        r1 = mk<R>(-p3.re, -p3.im);
    } else if constexpr (MU == 1) {
        r0 = mk<R>(p3.im, -p3.re);  // -i p3
        r1 = mk<R>(p2.im, -p2.re);  // -i p2
    } else if constexpr (MU == 2) {
        r0 = mk<R>(-p3.re, -p3.im);
        r1 = p2;
    } else {
        r0 = mk<R>(p2.im, -p2.re);  // -i p2
        r1 = mul_i(p3);             //  i p3
    }
}

// e_mu^dagger applied to (g0, g1).
template <typename R, int MU>
__device__ __forceinline__ void edag(cx<R> g0, cx<R> g1, cx<R>& r0, cx<R>& r1) {
    if constexpr (MU == 0) {
        r0 = mk<R>(-g0.re, -g0.im);
        r1 = mk<R>(-g1.re, -g1.im);
    } else if constexpr (MU == 1) {
        r0 = mul_i(g1);
        r1 = mul_i(g0);
    } else if constexpr (MU == 2) {
        r0 = g1;
        r1 = mk<R>(-g0.re, -g0.im);
    } else {
        r0 = mul_i(g0);
        r1 = mk<R>(g1.im, -g1.re);  // -i g1
    }
}

// Raw buffer access to one component array: the descriptor (base, size) is
// uniform and lives in SGPRs, the per-lane byte offset is one VGPR.  Offsets
// at or beyond `nbytes` read as zero and drop stores (hardware range check).
// Word 3 = 0x00020000 is the raw-buffer format for gfx9-family parts.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* base, unsigned nbytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)nbytes, 0x00020000);
}

template <typename R> struct BufIO;
template <> struct BufIO<double> {
    template <int AUX>
    __device__ static __forceinline__ double2 load(__amdgpu_buffer_rsrc_t r, unsigned off) {
        const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, AUX);
        double2 w;
        __builtin_memcpy(&w, &v, sizeof w);
        return w;
    }
    template <int AUX>
    __device__ static __forceinline__ void store(__amdgpu_buffer_rsrc_t r, unsigned off, double2 w) {
        unsigned int __attribute__((ext_vector_type(4))) v;
        __builtin_memcpy(&v, &w, sizeof w);
        __builtin_amdgcn_raw_buffer_store_b128(v, r, off, 0, AUX);
    }
};
template <> struct BufIO<float> {
    template <int AUX>
    __device__ static __forceinline__ float2 load(__amdgpu_buffer_rsrc_t r, unsigned off) {
        const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, AUX);
        float2 w;
        __builtin_memcpy(&w, &v, sizeof w);
        return w;
    }
    template <int AUX>
    __device__ static __forceinline__ void store(__amdgpu_buffer_rsrc_t r, unsigned off, float2 w) {
        unsigned int __attribute__((ext_vector_type(2))) v;
        __builtin_memcpy(&v, &w, sizeof w);
        __builtin_amdgcn_raw_buffer_store_b64(v, r, off, 0, AUX);
    }
};

template <> struct BufIO<half_t> {
    template <int AUX>
    __device__ static __forceinline__ h2 load(__amdgpu_buffer_rsrc_t r, unsigned off) {
        const auto v = __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, AUX);
        h2 w;
        __builtin_memcpy(&w, &v, sizeof w);
        return w;
    }
    template <int AUX>
    __device__ static __forceinline__ void store(__amdgpu_buffer_rsrc_t r, unsigned off, h2 w) {
        unsigned int v;
        __builtin_memcpy(&v, &w, sizeof w);
        __builtin_amdgcn_raw_buffer_store_b32(v, r, off, 0, AUX);
    }
};

// Element `i` of the component array starting at `base` (S words), widened
// to the arithmetic type of P.
template <typename P, int AUX = 0>
__device__ __forceinline__ cx<real_t<P>> bload(const typename Word<P>::T* base, int S, int i) {
    const unsigned wb = sizeof(typename Word<P>::T);
    const auto w = BufIO<P>::template load<AUX>(buf_rsrc(base, (unsigned)S * wb), (unsigned)i * wb);
    return {(real_t<P>)w.x, (real_t<P>)w.y};
}
// Stores v rounded to the storage type of P (round to nearest even).
template <typename P, int AUX = 0>
__device__ __forceinline__ void bstore(typename Word<P>::T* base, int S, int i, cx<real_t<P>> v) {
    const unsigned wb = sizeof(typename Word<P>::T);
    typename Word<P>::T w;
    w.x = v.re;
    w.y = v.im;
    BufIO<P>::template store<AUX>(buf_rsrc(base, (unsigned)S * wb), (unsigned)i * wb, w);
}

// Lattice extents and strides as seen by the kernels.
struct Geo {
    int L[4];   // T, LX, LY, LZ
    int Vh;     // sites per parity
    int S;      // site stride of the structure-of-arrays layout (>= Vh)
};

// Coordinates and lex index of the site with even-odd index i on parity p:
// lex = 2i + ((t + x + y + p) & 1) because LZ is even.
__device__ __forceinline__ void site_coords(const Geo& g, int i, int p, int c[4], int& lex) {
    const unsigned l2 = 2u * (unsigned)i;
    const unsigned row = l2 / (unsigned)g.L[3];
    const unsigned y = row % (unsigned)g.L[2];
    const unsigned r2 = row / (unsigned)g.L[2];
    const unsigned x = r2 % (unsigned)g.L[1];
    const unsigned t = r2 / (unsigned)g.L[1];
    const unsigned odd = (t + x + y + (unsigned)p) & 1u;
    c[0] = (int)t;
    c[1] = (int)x;
    c[2] = (int)y;
    c[3] = (int)(l2 - row * (unsigned)g.L[3] + odd);
    lex = (int)(l2 + odd);
}

// Deal workgroups so that XCD k (which receives hardware blocks k, k+8, ...)
// owns one contiguous range of logical blocks: neighbouring sites then share
// that XCD's L2.  A bijection of [0, nb).
__device__ __forceinline__ int xcd_remap(int b, int nb) {
    const int q = nb / kXcds, r = nb % kXcds;
    const int x = b % kXcds, k = b / kXcds;
    return x * q + (x < r ? x : r) + k;
}

// Sum over a workgroup of NT threads (a multiple of 64), in a fixed order;
// the result is valid in thread 0.  Call at most once per kernel.
template <int NT = kBlock>
__device__ __forceinline__ double block_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    __shared__ double wsum[NT / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) wsum[wid] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int w = 0; w < NT / 64; ++w) s += wsum[w];
    }
    return s;
}

}  // namespace tmh
