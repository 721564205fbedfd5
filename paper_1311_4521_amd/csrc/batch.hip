// Batched operators: many right-hand sides on several lattices in one
// persistent launch per operator step.
//
// A batch is a list of tasks, one per lattice, each with nrhs fields stored
// one after another (field r of a task at base + r * fstride words).  The
// work of a launch is a list of items, task after task; an item is a tile of
// 64*SW sites of one lattice for a group of RY * NR right-hand sides: the RY
// wave groups of a workgroup read the same links for the same sites (the
// second and later reads come from L1/L2), and each thread applies the links
// it loads to NR right-hand sides from registers.  The groups of a tile are
// consecutive items.  A fixed
// (persistent) grid walks the items: XCD k takes one contiguous range of
// items, its workgroups stride through it.
//
// BLAS-1 and reductions run per system (task, rhs); every system keeps its
// own CG scalars and flags, and a system whose flag is set is skipped, so the
// batch keeps iterating until its last system converges.
#include <mutex>
#include <vector>

#include "common.h"
#include "hop_body.h"
#include "kernels.h"

namespace tmh {

void batch_shape(int shape, int* sw, int* ry, int* nr) {
    static const int SW[kNumShapes] = {4, 2, 1, 2, 1, 2, 1, 2, 1, 2, 1, 2, 1, 4, 4, 1, 1};
    static const int RY[kNumShapes] = {1, 2, 4, 4, 12, 1, 2, 2, 4, 2, 3, 1, 8, 1, 1, 4, 4};
    static const int NR[kNumShapes] = {1, 1, 1, 1, 1, 2, 2, 2, 3, 3, 4, 4, 1, 1, 1, 1, 1};
    *sw = SW[shape];
    *ry = RY[shape];
    *nr = NR[shape];
}

int batch_rhs_per_item(int shape) {
    int sw, ry, nr;
    batch_shape(shape, &sw, &ry, &nr);
    return ry * nr;
}

namespace {

// Range of items of XCD k and the stride of its workgroups.
struct XcdRange {
    int start, count, k, nper;
};
__device__ __forceinline__ XcdRange xcd_range(int nitems) {
    XcdRange r;
    const int x = blockIdx.x % kXcds;
    r.k = blockIdx.x / kXcds;
    r.nper = gridDim.x / kXcds;
    const int q = nitems / kXcds, m = nitems % kXcds;
    r.start = x * q + (x < m ? x : m);
    r.count = q + (x < m ? 1 : 0);
    return r;
}

// First site of tile `tile` (nsl sites) of a task.  In x-group order the
// lattice is cut into 8 chunks of nt time-slices (one per XCD when the batch
// is one lattice); a chunk is visited x-group by x-group, each group over
// all the chunk's slices for xgroup consecutive x values.  All the
// right-hand sides of a tile are consecutive items, so the input one tile
// needs is the tile's neighbourhood in every right-hand side; this order
// brings the t neighbours of the tiles resident at one time closer than
// even-odd order does (measured: 3 % faster at 32^3x64 with 12 right-hand
// sides).
__device__ __forceinline__ int tile_site(int tile, int nsl, int xgroup, int nyt, int nt, int LX) {
    if (xgroup <= 0) return tile * nsl;
    const int per_chunk = nt * LX * nyt;
    const int chunk = tile / per_chunk;
    int rem = tile - chunk * per_chunk;
    const int per_group = nt * xgroup * nyt;
    const int xg = rem / per_group;
    rem -= xg * per_group;
    const int tl = rem / (xgroup * nyt);
    rem -= tl * (xgroup * nyt);
    const int xi = rem / nyt, yb = rem - xi * nyt;
    return (((chunk * nt + tl) * LX + xg * xgroup + xi) * nyt + yb) * nsl;
}

template <typename Table> __device__ __forceinline__ int find_task(const Table& tab, int item) {
    int t = 0;
    while (t + 1 < tab.ntasks && tab.t[t + 1].item0 <= item) ++t;
    return t;
}

template <typename R, int MODE, int SW, int RY, int NR, bool PIPE>
__global__ void __launch_bounds__(64 * SW * RY) batch_hop_kernel(BatchHopTable<R> tasks, int nitems) {
    constexpr int NSL = 64 * SW;
    const int lane_site = threadIdx.x % NSL;
    const int slot = threadIdx.x / NSL;
    __shared__ double red[SW * RY * NR];
    const XcdRange xr = xcd_range(nitems);
    for (int it = xr.k; it < xr.count; it += xr.nper) {
        const int item = xr.start + it;
        const BatchHopTask<R>& T = tasks.t[find_task(tasks, item)];
        const int local = item - T.item0;
        // tile major: the groups of right-hand sides of a tile are neighbours
        // in the item list, so they run close in time and share the links
        const int ngroups = (T.nrhs + RY * NR - 1) / (RY * NR);
        const int tile = local / ngroups;
        const int rhs0 = ((local - tile * ngroups) * RY + slot) * NR;
        const int i = tile_site(tile, NSL, T.xgroup, T.nyt, T.nt, T.g.L[1]) + lane_site;
        const int nv = rhs0 < T.nrhs ? (T.nrhs - rhs0 < NR ? T.nrhs - rhs0 : NR) : 0;
        unsigned live = 0;  // bit r: right-hand side rhs0 + r is computed and stored
#pragma unroll
        for (int r = 0; r < NR; ++r)
            if (r < nv && !(T.flags && T.flags[2 * (T.sys0 + rhs0 + r)])) live |= 1u << r;
        double nrm[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r) nrm[r] = 0.0;
        if (live && i < T.g.Vh) {
            HopArgs<R> a;
            a.in = T.in + rhs0 * T.fstride;
            a.gout = T.gout;
            a.gin = T.gin;
            a.g = T.g;
            a.pout = T.pout;
            a.lf = 0;
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                a.ph_re[m] = T.ph_re[m];
                a.ph_im[m] = T.ph_im[m];
            }
            int c[4], lex;
            site_coords(T.g, i, T.pout, c, lex);
            cx<R> acc[NR][4][3];
#pragma unroll
            for (int r = 0; r < NR; ++r)
#pragma unroll
                for (int s = 0; s < 4; ++s)
#pragma unroll
                    for (int k = 0; k < 3; ++k) acc[r][s][k] = mk<R>(0, 0);
            const SiteNb n = site_neighbours(T.g, c, lex);
            // links shared by several right-hand sides are kept in the caches
            // unless this thread is their only user
            constexpr int LAUX = (RY == 1 && NR == 1) ? kLinkAux : 0;
            if constexpr (NR == 1)
                hop_site<R, PIPE, LAUX>(acc[0], a, n, i);
            else
                hop_site_nr<R, NR, LAUX>(acc, a, T.fstride, nv, n, i);
            const int S = T.g.S;
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                if (!((live >> r) & 1u)) continue;
                const int64_t fo = (rhs0 + r) * T.fstride;
                typename Word<R>::T* out = T.out + fo;
                const typename Word<R>::T* aux = T.aux + fo;
                const R alpha = MODE == 3 ? (R)T.scal[(int64_t)(T.sys0 + rhs0 + r) * kNScal + kAlpha] : (R)0;
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const cx<R> cc = mk<R>(T.c_re[s >> 1], T.c_im[s >> 1]);
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        const int64_t comp = (int64_t)(3 * s + k) * S;
                        cx<R> o = cc * acc[r][s][k];
                        if constexpr (MODE >= 1)
                            o += mk<R>(T.d_re[s >> 1], T.d_im[s >> 1]) *
                                 bload<R, out_aux<R>()>(aux + comp, S, i);
                        if constexpr (MODE == 2) nrm[r] += (double)o.re * (double)o.re + (double)o.im * (double)o.im;
                        if constexpr (MODE == 3) {
                            // the CG update: r -= alpha q, x += alpha p, |r|^2
                            cx<R> rv = bload<R>(T.rio + fo + comp, S, i);
                            rv -= alpha * o;
                            bstore<R>(T.rio + fo + comp, S, i, rv);
                            cx<R> xv = bload<R>(T.xio + fo + comp, S, i);
                            xv += alpha * bload<R>(T.pin + fo + comp, S, i);
                            bstore<R>(T.xio + fo + comp, S, i, xv);
                            nrm[r] += (double)rv.re * (double)rv.re + (double)rv.im * (double)rv.im;
                        } else {
                            bstore<R, out_aux<R>()>(out + comp, S, i, o);
                        }
                    }
                }
            }
        }
        if constexpr (MODE >= 2) {
            // per right-hand side: the SW waves of a slot sum their sites
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                double v = nrm[r];
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
                if ((threadIdx.x & 63) == 0) red[(threadIdx.x >> 6) * NR + r] = v;
            }
            __syncthreads();
            if (lane_site < NR && rhs0 + lane_site < T.nrhs) {
                double v = 0.0;
#pragma unroll
                for (int w = 0; w < SW; ++w) v += red[(slot * SW + w) * NR + lane_site];
                T.partial[(int64_t)(T.sys0 + rhs0 + lane_site) * T.pstride + tile] = v;
            }
            __syncthreads();
        }
    }
}

// ------------------------------------------------------------------ MFMA
//
// The same hop with the link products on the matrix cores (shape
// kShapeMfma, FP64 and FP32).  Per term, the colour product of two sites is
// one real block-diagonal product: rows (sigma, a, re/im) and columns
// (sigma, b, re/im) of two 6x6 blocks [[Re U, -Im U], [Im U, Re U]] (or the
// same for U^dagger), sigma = 0, 1 the site of the pair, against a 12 x 16
// operand whose columns are (spin, rhs) of the half-spinors h of 2 spins x 8
// right-hand sides: three 16x16x4 products (K = 12) per site pair and term.
// Rows 12-15 of the result are zero.  An item is 64 sites x 8 right-hand
// sides; wave w of its 8 waves holds sites 8w..8w+7, lane l the pair
// (site 8w + l/8, rhs l%8), which projects the neighbour spinor to h, writes
// it into the operand in LDS, and after the products reads its part of the
// result back from LDS and rebuilds the lower spins (-DIR e_mu^dagger g).
// Half of each 16x16 block and a quarter of its rows are zeros, so the
// matrix cores do 16/6 times the floating-point work of the vector path;
// both peaks are equal for FP64 on this chip.

template <typename R> struct Mfma;
template <> struct Mfma<double> {
    typedef double V4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ V4 mma(double a, double b, V4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // Row of the result element that lane l holds as value v (the column is l % 16).
    static __device__ __forceinline__ int row(int l, int v) { return (l >> 4) + 4 * v; }
};
template <> struct Mfma<float> {
    typedef float V4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ V4 mma(float a, float b, V4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int l, int v) { return 4 * (l >> 4) + v; }
};

constexpr int kMfmaWaves = 8;  // waves per item: 64 sites, 8 per wave
constexpr int kMfmaRhs = 8;    // right-hand sides per item

// Orders the LDS traffic of one wave (the lanes exchange data through LDS
// within the wave only).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename R, int TT>
__device__ __forceinline__ void mfma_term(cx<R> (&acc)[4][3], const BatchHopTask<R>& T, const SiteNb& n, int i,
                                          bool in_range, bool live, int r, R* sBD, cx<R>* sU, int lane) {
    using W = typename Word<R>::T;
    constexpr int MU = TT / 2, DIR = (TT % 2 == 0) ? +1 : -1;
    const int S = T.g.S;
    const int pair = lane >> 4, sigma = (lane >> 3) & 1, rl = lane & 7, s8 = lane >> 3, e = lane & 7;
    // 1. half-spinor of this lane's (neighbour site, rhs) with the boundary phase
    cx<R> h[2][3];
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int a = 0; a < 3; ++a) h[s][a] = mk<R>(0, 0);
    if (live) {
        const W* in = T.in + (int64_t)r * T.fstride;
        cx<R> psi[4][3];
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int a = 0; a < 3; ++a) psi[s][a] = bload<R>(in + (int64_t)(3 * s + a) * S, S, n.jn[TT]);
        const bool wrap = (n.wrap >> TT) & 1u;
        const cx<R> eta = wrap ? mk<R>(T.ph_re[MU], DIR > 0 ? T.ph_im[MU] : -T.ph_im[MU]) : mk<R>(1, 0);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            cx<R> e0, e1;
            e_lower<R, MU>(psi[2][a], psi[3][a], e0, e1);
            h[0][a] = (DIR > 0 ? psi[0][a] - e0 : psi[0][a] + e0) * eta;
            h[1][a] = (DIR > 0 ? psi[1][a] - e1 : psi[1][a] + e1) * eta;
        }
    }
    R* B = sBD + pair * 192;  // operand of this site pair: B[k][j], k = sigma*6 + b*2 + ri, j = spin*8 + rhs
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            B[(sigma * 6 + b * 2) * 16 + s * 8 + rl] = h[s][b].re;
            B[(sigma * 6 + b * 2 + 1) * 16 + s * 8 + rl] = h[s][b].im;
        }
    // 2. the links of the wave's 8 sites: lane (site s8, entry e) loads entry e, lanes e = 0 also entry 8
    {
        const W* link = (DIR > 0 ? T.gout : T.gin) + (int64_t)MU * 9 * S;
        const int jl = DIR > 0 ? i : n.jn[TT];
        cx<R> u0 = mk<R>(0, 0), u8 = mk<R>(0, 0);
        if (in_range) {
            u0 = bload<R>(link + (int64_t)e * S, S, jl);
            if (e == 0) u8 = bload<R>(link + (int64_t)8 * S, S, jl);
        }
        sU[s8 * 9 + e] = u0;
        if (e == 0) sU[s8 * 9 + 8] = u8;
    }
    wave_lds_sync();
    // 3. three products per site pair
    typename Mfma<R>::V4 d[4];
    const int arow = lane & 15;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        d[p] = typename Mfma<R>::V4{0, 0, 0, 0};
#pragma unroll
        for (int kk = 0; kk < 3; ++kk) {
            const int k = kk * 4 + (lane >> 4);
            R a = 0;
            if (arow < 12 && arow / 6 == k / 6) {
                const int sr = arow / 6, ar = (arow % 6) >> 1, ro = arow & 1, bk = (k % 6) >> 1, ri = k & 1;
                const cx<R> u = DIR > 0 ? sU[(2 * p + sr) * 9 + 3 * ar + bk] : sU[(2 * p + sr) * 9 + 3 * bk + ar];
                // real form of u (forward) or conj(u) (backward, U^dagger entry (ar, bk) = conj U(bk, ar))
                const R ui = DIR > 0 ? u.im : -u.im;
                a = (ro == ri) ? u.re : (ro == 0 ? -ui : ui);
            }
            d[p] = Mfma<R>::mma(a, sBD[p * 192 + k * 16 + (lane & 15)], d[p]);
        }
    }
    wave_lds_sync();
    // 4. results back through LDS (the operand area is free now), then per lane
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int v = 0; v < 4; ++v) sBD[p * 256 + Mfma<R>::row(lane, v) * 16 + (lane & 15)] = d[p][v];
    wave_lds_sync();
    if (live) {
        const R* D = sBD + pair * 256;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            cx<R> g[2];
#pragma unroll
            for (int s = 0; s < 2; ++s)
                g[s] = mk<R>(D[(sigma * 6 + a * 2) * 16 + s * 8 + rl], D[(sigma * 6 + a * 2 + 1) * 16 + s * 8 + rl]);
            acc[0][a] += g[0];
            acc[1][a] += g[1];
            cx<R> f0, f1;
            edag<R, MU>(g[0], g[1], f0, f1);
            if constexpr (DIR > 0) {
                acc[2][a] -= f0;
                acc[3][a] -= f1;
            } else {
                acc[2][a] += f0;
                acc[3][a] += f1;
            }
        }
    }
    wave_lds_sync();
}

template <typename R, int MODE>
__global__ void __launch_bounds__(64 * kMfmaWaves) batch_hop_mfma_kernel(BatchHopTable<R> tasks, int nitems) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int sl = wv * 8 + (lane >> 3);  // site of this lane inside the 64-site tile
    const int rl = lane & 7;
    __shared__ R sBD[kMfmaWaves][4 * 256];
    __shared__ cx<R> sU[kMfmaWaves][8 * 9];
    __shared__ double red[kMfmaWaves][kMfmaRhs];
    const XcdRange xr = xcd_range(nitems);
    for (int it = xr.k; it < xr.count; it += xr.nper) {
        const int item = xr.start + it;
        const BatchHopTask<R>& T = tasks.t[find_task(tasks, item)];
        const int local = item - T.item0;
        const int ngroups = (T.nrhs + kMfmaRhs - 1) / kMfmaRhs;
        const int tile = local / ngroups;
        const int rhs0 = (local - tile * ngroups) * kMfmaRhs;
        const int i = tile_site(tile, 64, T.xgroup, T.nyt, T.nt, T.g.L[1]) + sl;
        const int r = rhs0 + rl;
        const bool in_range = i < T.g.Vh;
        const bool live = in_range && r < T.nrhs && !(T.flags && T.flags[2 * (T.sys0 + r)]);
        SiteNb n;
        n.wrap = 0;
#pragma unroll
        for (int k = 0; k < 8; ++k) n.jn[k] = 0;
        if (in_range) {
            int c[4], lex;
            site_coords(T.g, i, T.pout, c, lex);
            n = site_neighbours(T.g, c, lex);
        }
        cx<R> acc[4][3];
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int k = 0; k < 3; ++k) acc[s][k] = mk<R>(0, 0);
        R* bd = sBD[wv];
        cx<R>* su = sU[wv];
        mfma_term<R, 0>(acc, T, n, i, in_range, live, r, bd, su, lane);
        mfma_term<R, 1>(acc, T, n, i, in_range, live, r, bd, su, lane);
        mfma_term<R, 2>(acc, T, n, i, in_range, live, r, bd, su, lane);
        mfma_term<R, 3>(acc, T, n, i, in_range, live, r, bd, su, lane);
        mfma_term<R, 4>(acc, T, n, i, in_range, live, r, bd, su, lane);
        mfma_term<R, 5>(acc, T, n, i, in_range, live, r, bd, su, lane);
        mfma_term<R, 6>(acc, T, n, i, in_range, live, r, bd, su, lane);
        mfma_term<R, 7>(acc, T, n, i, in_range, live, r, bd, su, lane);
        double nrm = 0.0;
        if (live) {
            const int S = T.g.S;
            const int64_t fo = (int64_t)r * T.fstride;
            typename Word<R>::T* out = T.out + fo;
            const typename Word<R>::T* aux = T.aux + fo;
            const R alpha = MODE == 3 ? (R)T.scal[(int64_t)(T.sys0 + r) * kNScal + kAlpha] : (R)0;
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const cx<R> cc = mk<R>(T.c_re[s >> 1], T.c_im[s >> 1]);
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const int64_t comp = (int64_t)(3 * s + k) * S;
                    cx<R> o = cc * acc[s][k];
                    if constexpr (MODE >= 1)
                        o += mk<R>(T.d_re[s >> 1], T.d_im[s >> 1]) * bload<R, out_aux<R>()>(aux + comp, S, i);
                    if constexpr (MODE == 2) nrm += (double)o.re * (double)o.re + (double)o.im * (double)o.im;
                    if constexpr (MODE == 3) {
                        cx<R> rv = bload<R>(T.rio + fo + comp, S, i);
                        rv -= alpha * o;
                        bstore<R>(T.rio + fo + comp, S, i, rv);
                        cx<R> xv = bload<R>(T.xio + fo + comp, S, i);
                        xv += alpha * bload<R>(T.pin + fo + comp, S, i);
                        bstore<R>(T.xio + fo + comp, S, i, xv);
                        nrm += (double)rv.re * (double)rv.re + (double)rv.im * (double)rv.im;
                    } else {
                        bstore<R, out_aux<R>()>(out + comp, S, i, o);
                    }
                }
            }
        }
        if constexpr (MODE >= 2) {
            // per right-hand side: lanes with the same l % 8, then the 8 waves in order
#pragma unroll
            for (int off = 8; off < 64; off <<= 1) nrm += __shfl_xor(nrm, off, 64);
            if (lane < kMfmaRhs) red[wv][lane] = nrm;
            __syncthreads();
            if (threadIdx.x < kMfmaRhs && rhs0 + (int)threadIdx.x < T.nrhs) {
                double v = 0.0;
#pragma unroll
                for (int w = 0; w < kMfmaWaves; ++w) v += red[w][threadIdx.x];
                T.partial[(int64_t)(T.sys0 + rhs0 + threadIdx.x) * T.pstride + tile] = v;
            }
            __syncthreads();
        }
    }
}

// ------------------------------------------------------------- t-march
//
// The multi-right-hand-side form of the t-marching hop (hop.hip): a
// workgroup owns one tile of 256 site pairs of a time-slice, one right-hand
// side, and a range of tm_steps time-slices, which it walks.  A thread keeps
// the projections (1 + gamma_0) psi of its pair's input sites at t - 1 and t
// (the backward time term two and one steps later) in registers and loads
// each input site once, as the forward time neighbour.  The workgroups of a
// tile for all right-hand sides are consecutive, so an XCD works on a few
// tiles for all right-hand sides at once: the links they share are read
// once, and one step's new data (the next slice of those tiles for every
// right-hand side and their links) stays small against the L2, so the
// spatial neighbours read in the next step are still there.

// Workgroups of the t-march are dealt to XCDs so that each XCD takes one
// contiguous eighth of every task (its tiles for all right-hand sides), task
// after task: the XCDs get equal shares of lattices whose workgroups walk
// different numbers of time-slices.  Hardware workgroup b runs on XCD b % 8
// as its (b / 8)-th; returns the task and its local workgroup index, or
// false past the end of the XCD's list.
template <typename R>
__device__ __forceinline__ bool tmarch_block(const BatchHopTable<R>& tasks, int& ti, int& local) {
    const int x = blockIdx.x % kXcds;
    int j = blockIdx.x / kXcds;
    for (ti = 0; ti < tasks.ntasks; ++ti) {
        const BatchHopTask<R>& T = tasks.t[ti];
        const int nb = batch_tmarch_blocks(T.g.L[0], T.tm_steps, T.tm_nw, T.nrhs, T.tm_rg);
        const int q = nb / kXcds, m = nb % kXcds;
        const int cnt = q + (x < m ? 1 : 0);
        if (j < cnt) {
            local = x * q + (x < m ? x : m) + j;
            return true;
        }
        j -= cnt;
    }
    return false;
}

// RG right-hand sides per workgroup: its 256 threads are RG groups (of
// 256 / RG pairs) that walk the same pairs for consecutive right-hand sides,
// so the links of a step are requested by the RG groups at the same time.
// The t-march link loads keep the default cache policy: the workgroups of a
// tile for all right-hand sides read each link through L2 (with the
// non-temporal hint every right-hand side fetched its links again, 1.7x
// slower at 32^3x64 with 12 right-hand sides).
constexpr int kTmLinkAux = 0;
// Staged links keep the default policy too: the workgroups of a tile for the
// other right-hand-side groups load the same links at about the same time.
#ifndef TMH_TM_LDS_RHS_OUTER
#define TMH_TM_LDS_RHS_OUTER 1
#endif
// (with the groups outermost each group fetches the links once, and they
// pass L2 with the non-temporal hint)
constexpr int kTmStageAux = TMH_TM_LDS_RHS_OUTER ? TMH_LINK_POLICY : 0;

// The link of term TT of one step for this thread's pair, into registers.
template <typename R, int TT>
__device__ __forceinline__ void tm_fetch(cx<R> (&u)[9], const HopArgs<R>& b, const SiteNb& n, int i) {
    constexpr int MU = TT / 2;
    const int S = b.g.S;
    const typename Word<R>::T* link = (TT % 2 == 0 ? b.gout : b.gin) + (int64_t)MU * 9 * S;
    const int jl = TT % 2 == 0 ? i : n.jn[TT];
#pragma unroll
    for (int k = 0; k < 9; ++k) u[k] = bload<R, kTmStageAux>(link + (int64_t)k * S, S, jl);
}

// Wave v's share of one half of a step's links: term 4 * HALF + v.
template <typename R, int HALF>
__device__ __forceinline__ void tm_fetch_wave(cx<R> (&u)[9], int wave, const HopArgs<R>& b, const SiteNb& n,
                                              int i) {
    switch (wave) {
        case 0: tm_fetch<R, 4 * HALF + 0>(u, b, n, i); break;
        case 1: tm_fetch<R, 4 * HALF + 1>(u, b, n, i); break;
        case 2: tm_fetch<R, 4 * HALF + 2>(u, b, n, i); break;
        default: tm_fetch<R, 4 * HALF + 3>(u, b, n, i); break;
    }
}

template <typename R>
__device__ __forceinline__ void tm_put(cx<R>* lk, int term, const cx<R> (&u)[9], int lane) {
#pragma unroll
    for (int k = 0; k < 9; ++k) lk[(term * 9 + k) * 64 + lane] = u[k];
}

// The neighbour spinor of term TT from memory and its link from memory or
// from the staged links.
template <typename R, int TT, bool LDS>
__device__ __forceinline__ void tm_load(TermData<R>& d, const HopArgs<R>& b, const SiteNb& n, int i, const cx<R>* lk) {
    if constexpr (LDS) {
        const int S = b.g.S;
        const int lane = (int)threadIdx.x % 64;
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int a = 0; a < 3; ++a) d.psi[s][a] = bload<R>(b.in + (int64_t)(3 * s + a) * S, S, n.jn[TT]);
#pragma unroll
        for (int k = 0; k < 9; ++k) d.u[k / 3][k % 3] = lk[(TT * 9 + k) * 64 + lane];
    } else {
        load_t<R, TT, kTmLinkAux, 0>(d, b, n, i);
    }
}

template <typename R, int MODE, bool PIPE, int RG, bool LDS>
__device__ __forceinline__ void tmarch_body(const BatchHopTable<R>& tasks) {
    using W = typename Word<R>::T;
    constexpr int kPairs = 256 / RG;  // pairs of one tile
    static_assert(!LDS || (RG == 4 && !PIPE), "links are staged for one wave per right-hand side");
    extern __shared__ unsigned char tm_lds[];
    cx<R>* lk = reinterpret_cast<cx<R>*>(tm_lds);  // LDS: [term][entry][pair] links of one step
    int ti, local;
    if (!tmarch_block(tasks, ti, local)) return;
    const BatchHopTask<R>& T = tasks.t[ti];
    const int ngr = (T.nrhs + RG - 1) / RG;
    int rgi, w, range;
    if constexpr (LDS && TMH_TM_LDS_RHS_OUTER) {
        // right-hand-side groups outermost: an XCD's resident workgroups
        // cover a thicker block of the lattice for one group at a time
        const int nranges = T.g.L[0] / T.tm_steps;
        w = local % T.tm_nw;
        const int tmp = local / T.tm_nw;
        range = tmp % nranges;
        rgi = tmp / nranges;
    } else {
        rgi = local % ngr;
        const int tmp = local / ngr;
        w = tmp % T.tm_nw;
        range = tmp / T.tm_nw;
    }
    // the same for a whole wave (kPairs is a multiple of 64): kept in an SGPR
    const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x / kPairs);
    const int rhs = rgi * RG + wave;
    const bool active = rhs < T.nrhs && !(T.flags && T.flags[2 * (T.sys0 + rhs)]);
    if constexpr (!LDS) {
        if (!active) return;
    } else {
        // the waves stage the links together: the workgroup stays while one
        // of its right-hand sides is still iterating
        bool any = false;
#pragma unroll
        for (int r = 0; r < RG; ++r) {
            const int q = rgi * RG + r;
            any = any || (q < T.nrhs && !(T.flags && T.flags[2 * (T.sys0 + q)]));
        }
        if (!any) return;
    }
    const int slice = T.tm_slice, LT = T.g.L[0], S = T.g.S;
    const int jp = w * kPairs + (int)threadIdx.x % kPairs;
    const int hz = T.g.L[3] >> 1;
    const int row = jp / hz, zp = jp - row * hz;
    const int y = row % T.g.L[2], x = row / T.g.L[2];
    const int t0 = range * T.tm_steps;
    const int64_t fo = (int64_t)(active ? rhs : rgi * RG) * T.fstride;
    HopArgs<R> a;
    a.in = T.in + fo;
    a.gout = T.gout;
    a.gin = T.gin;
    a.g = T.g;
    a.pout = T.pout;
    a.lf = 0;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        a.ph_re[m] = T.ph_re[m];
        a.ph_im[m] = T.ph_im[m];
    }
    cx<R> hprev[2][3], hcur[2][3];
    if (active) {
        cx<R> psi[4][3];
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int c = 0; c < 3; ++c)
                psi[s][c] = bload<R>(a.in + (int64_t)(3 * s + c) * S, S, (t0 == 0 ? LT - 1 : t0 - 1) * slice + jp);
        project<R, 0, -1>(hprev, psi);
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int c = 0; c < 3; ++c) psi[s][c] = bload<R>(a.in + (int64_t)(3 * s + c) * S, S, t0 * slice + jp);
        project<R, 0, -1>(hcur, psi);
    }
    const R alpha = (MODE == 3 && active) ? (R)T.scal[(int64_t)(T.sys0 + rhs) * kNScal + kAlpha] : (R)0;
    __shared__ double wsum[4];
    // LDS: each half of a step's links (terms 0-3, 4-7; wave v holds term
    // 4 h + v) is fetched into registers while the other half is computed,
    // then written to LDS; a barrier after each half.
    const int lane = (int)threadIdx.x % kPairs;
    cx<R> lreg[9];
    auto step_nb = [&](int t) {
        int cc[4];
        cc[0] = t;
        cc[1] = x;
        cc[2] = y;
        cc[3] = 2 * zp + ((t + x + y + T.pout) & 1);
        const int lx = ((t * T.g.L[1] + x) * T.g.L[2] + y) * T.g.L[3] + cc[3];
        return site_neighbours(T.g, cc, lx);
    };
    if constexpr (LDS) {
        tm_fetch_wave<R, 0>(lreg, wave, a, step_nb(t0), t0 * slice + jp);
        tm_put(lk, wave, lreg, lane);
        __syncthreads();
    }
    for (int st = 0; st < T.tm_steps; ++st) {
        HopArgs<R> b = a;
        // rebuilt descriptors every step (see hop_tmarch_kernel)
        __asm__ volatile("" : "+s"(b.in), "+s"(b.gout), "+s"(b.gin));
        const int t = t0 + st;
        const int i = t * slice + jp;
        int c[4];
        c[0] = t;
        c[1] = x;
        c[2] = y;
        c[3] = 2 * zp + ((t + x + y + T.pout) & 1);
        const int lex = ((t * T.g.L[1] + x) * T.g.L[2] + y) * T.g.L[3] + c[3];
        const SiteNb n = site_neighbours(T.g, c, lex);
        // half B of this step's links, fetched while half A is computed
        if constexpr (LDS) tm_fetch_wave<R, 1>(lreg, wave, b, n, i);
        cx<R> acc[4][3];
        if (active) {
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int k = 0; k < 3; ++k) acc[s][k] = mk<R>(0, 0);
        {
            // forward time term from memory; its backward projection joins the ring
            TermData<R> d;
            tm_load<R, 0, LDS>(d, b, n, i, lk);
            cx<R> hf[2][3], hn[2][3];
            project<R, 0, +1>(hf, d.psi);
            project<R, 0, -1>(hn, d.psi);
            add_term_h<R, 0, +1>(acc, hf, d.u, (n.wrap >> 0) & 1u, mk<R>(b.ph_re[0], b.ph_im[0]));
            // backward time term from the ring
            TermData<R> e;
            if constexpr (LDS) {
#pragma unroll
                for (int k = 0; k < 9; ++k) e.u[k / 3][k % 3] = lk[(9 + k) * 64 + lane];
            } else {
                const typename Word<R>::T* link = b.gin;
#pragma unroll
                for (int k = 0; k < 9; ++k) e.u[k / 3][k % 3] = bload<R, kTmLinkAux>(link + (int64_t)k * S, S, n.jn[1]);
            }
            add_term_h<R, 0, -1>(acc, hprev, e.u, (n.wrap >> 1) & 1u, mk<R>(b.ph_re[0], -b.ph_im[0]));
#pragma unroll
            for (int s = 0; s < 2; ++s)
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    hprev[s][k] = hcur[s][k];
                    hcur[s][k] = hn[s][k];
                }
        }
        TMH_SCHED_FENCE();
        if constexpr (PIPE) {
            TermData<R> d0, d1;
            load_t<R, 2, kTmLinkAux, 0>(d0, b, n, i);
            TMH_SCHED_FENCE();
            load_t<R, 3, kTmLinkAux, 0>(d1, b, n, i);
            TMH_SCHED_FENCE();
            add_t<R, 2>(acc, d0, b, n);
            TMH_SCHED_FENCE();
            load_t<R, 4, kTmLinkAux, 0>(d0, b, n, i);
            TMH_SCHED_FENCE();
            add_t<R, 3>(acc, d1, b, n);
            TMH_SCHED_FENCE();
            load_t<R, 5, kTmLinkAux, 0>(d1, b, n, i);
            TMH_SCHED_FENCE();
            add_t<R, 4>(acc, d0, b, n);
            TMH_SCHED_FENCE();
            load_t<R, 6, kTmLinkAux, 0>(d0, b, n, i);
            TMH_SCHED_FENCE();
            add_t<R, 5>(acc, d1, b, n);
            TMH_SCHED_FENCE();
            load_t<R, 7, kTmLinkAux, 0>(d1, b, n, i);
            TMH_SCHED_FENCE();
            add_t<R, 6>(acc, d0, b, n);
            TMH_SCHED_FENCE();
            add_t<R, 7>(acc, d1, b, n);
        } else {
            TermData<R> d;
#define TMH_TM_TERM(TT)                \
    tm_load<R, TT, LDS>(d, b, n, i, lk); \
    add_t<R, TT>(acc, d, b, n);          \
    TMH_SCHED_FENCE();
            TMH_TM_TERM(2) TMH_TM_TERM(3)
        }
        }  // active
        if constexpr (LDS) {
            // half B in place; after the barrier every wave is also done with
            // half A, which takes the next step's links
            tm_put(lk, 4 + wave, lreg, lane);
            __syncthreads();
            if (st + 1 < T.tm_steps) tm_fetch_wave<R, 0>(lreg, wave, b, step_nb(t + 1), (t + 1) * slice + jp);
        }
        if (active) {
        if constexpr (!PIPE) {
            TermData<R> d;
            TMH_TM_TERM(4) TMH_TM_TERM(5) TMH_TM_TERM(6) TMH_TM_TERM(7)
        }
#undef TMH_TM_TERM
        W* out = T.out + fo;
        const W* aux = T.aux + fo;
        W* rio = T.rio + fo;
        W* xio = T.xio + fo;
        const W* pin = T.pin + fo;
        __asm__ volatile("" : "+s"(out), "+s"(aux));
        if constexpr (MODE == 3) __asm__ volatile("" : "+s"(rio), "+s"(xio), "+s"(pin));
        double nrm = 0.0;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const cx<R> cc = mk<R>(T.c_re[s >> 1], T.c_im[s >> 1]);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const int64_t comp = (int64_t)(3 * s + k) * S;
                cx<R> o = cc * acc[s][k];
                if constexpr (MODE >= 1)
                    o += mk<R>(T.d_re[s >> 1], T.d_im[s >> 1]) * bload<R, out_aux<R>()>(aux + comp, S, i);
                if constexpr (MODE == 2) nrm += (double)o.re * (double)o.re + (double)o.im * (double)o.im;
                if constexpr (MODE == 3) {
                    cx<R> rv = bload<R>(rio + comp, S, i);
                    rv -= alpha * o;
                    bstore<R>(rio + comp, S, i, rv);
                    cx<R> xv = bload<R>(xio + comp, S, i);
                    xv += alpha * bload<R>(pin + comp, S, i);
                    bstore<R>(xio + comp, S, i, xv);
                    nrm += (double)rv.re * (double)rv.re + (double)rv.im * (double)rv.im;
                } else {
                    bstore<R, out_aux<R>()>(out + comp, S, i, o);
                }
            }
        }
        if constexpr (MODE >= 2) {
            // one partial per (system, slice tile), as the tiles of 64 * SW
            // sites of the other shapes
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) nrm += __shfl_xor(nrm, off, 64);
            if constexpr (RG == 1) {
                if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = nrm;
                __syncthreads();
                if (threadIdx.x == 0)
                    T.partial[(int64_t)(T.sys0 + rhs) * T.pstride + t * T.tm_nw + w] =
                        wsum[0] + wsum[1] + wsum[2] + wsum[3];
                __syncthreads();
            } else {
                static_assert(kPairs == 64, "one wave per right-hand side and tile");
                if ((threadIdx.x & 63) == 0) T.partial[(int64_t)(T.sys0 + rhs) * T.pstride + t * T.tm_nw + w] = nrm;
            }
        }
        }  // active
        if constexpr (LDS) {
            if (st + 1 < T.tm_steps) tm_put(lk, wave, lreg, lane);
            __syncthreads();  // half A of the next step in place, half B read
        }
    }
}

template <typename R, int MODE, bool PIPE, int RG, bool LDS>
__global__ void __launch_bounds__(256) batch_tmarch_kernel(BatchHopTable<R> tasks) {
    tmarch_body<R, MODE, PIPE, RG, LDS>(tasks);
}

// The LDS-staged form with registers held for two waves per SIMD (its
// twist epilogues would otherwise take a few AGPRs past 256 and drop to one).
template <typename R, int MODE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 8)))
batch_tmarch_lds_kernel(BatchHopTable<R> tasks) {
    tmarch_body<R, MODE, false, 4, true>(tasks);
}

// ---------------------------------------------------------------- BLAS-1

constexpr int kVecTile = kBlock;  // sites per item of the vector kernels

__device__ __forceinline__ bool sys_done(const int* flags, int sys) { return flags && flags[2 * sys] != 0; }

// op 0: a += alpha c, b -= alpha d, partial |b|^2        (x, r, p, q)
// op 1: a = c + beta a                                  (p, r)
// op 2: a = c - d, partial |a|^2                        (r, b, q)
// op 3: partial |c|^2
// op 4: a = c                                           (copy)
template <int OP>
__global__ void __launch_bounds__(kBlock) batch_vec_kernel(BatchVecTable tasks, int nitems,
                                                           const double* __restrict__ scal, const int* flags) {
    const XcdRange xr = xcd_range(nitems);
    for (int it = xr.k; it < xr.count; it += xr.nper) {
        const int item = xr.start + it;
        const BatchVecTask& T = tasks.t[find_task(tasks, item)];
        const int local = item - T.item0;
        const int rhs = local / T.ntile, tile = local - rhs * T.ntile;
        const int sys = T.sys0 + rhs;
        const bool skip = (OP <= 1) && sys_done(flags, sys);
        const int i = tile * kVecTile + threadIdx.x;
        const int64_t base = rhs * T.fstride;
        double nrm = 0.0;
        if (!skip && i < T.Vh) {
            const double alpha = (OP == 0) ? scal[sys * kNScal + kAlpha] : 0.0;
            const double beta = (OP == 1) ? scal[sys * kNScal + kBeta] : 0.0;
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                const int64_t k = base + (int64_t)c * T.S + i;
                if constexpr (OP == 0) {
                    double2 x = T.a[k], r = T.b[k];
                    const double2 p = T.c[k], q = T.d[k];
                    x.x += alpha * p.x;
                    x.y += alpha * p.y;
                    r.x -= alpha * q.x;
                    r.y -= alpha * q.y;
                    T.a[k] = x;
                    T.b[k] = r;
                    nrm += r.x * r.x + r.y * r.y;
                } else if constexpr (OP == 1) {
                    double2 p = T.a[k];
                    const double2 r = T.c[k];
                    p.x = r.x + beta * p.x;
                    p.y = r.y + beta * p.y;
                    T.a[k] = p;
                } else if constexpr (OP == 2) {
                    const double2 b = T.c[k], q = T.d[k];
                    const double2 r = make_double2(b.x - q.x, b.y - q.y);
                    T.a[k] = r;
                    nrm += r.x * r.x + r.y * r.y;
                } else if constexpr (OP == 3) {
                    const double2 v = T.c[k];
                    nrm += v.x * v.x + v.y * v.y;
                } else {
                    T.a[k] = T.c[k];
                }
            }
        }
        if constexpr (OP == 0 || OP == 2 || OP == 3) {
            // skipped systems still write a partial (zero) to keep the sums defined
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) nrm += __shfl_xor(nrm, off, 64);
            __shared__ double red[kBlock / 64];
            if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = nrm;
            __syncthreads();
            if (threadIdx.x == 0 && !skip) {
                double s = 0.0;
#pragma unroll
                for (int w = 0; w < kBlock / 64; ++w) s += red[w];
                T.partial[(int64_t)sys * T.pstride + tile] = s;
            }
            __syncthreads();
        }
    }
}

// -------------------------------------------------------- per-system scalars

// Sum of n partials of system `sys` by one workgroup (fixed order).
__device__ __forceinline__ double sys_sum(const double* __restrict__ partial, int64_t pstride, int sys, int n) {
    double s = 0.0;
    for (int k = threadIdx.x; k < n; k += kBlock) s += partial[(int64_t)sys * pstride + k];
    return block_sum(s);
}

// op 0 (alpha): pq = sum(hop partials), alpha = rr / pq
// op 1 (beta):  rr' = sum(hop partials of the fused update), beta = rr'/rr, rr = rr', iterations, done
// op 2 (norm):  scal[kNorm] = sum(vec partials)
// op 3 (init):  rr = sum(vec partials); stop = tol^2 scal[kBB]; done = rr <= stop; iterations = 0
// op 4 (bb):    scal[kBB] = sum(vec partials)
template <int OP>
__global__ void __launch_bounds__(kBlock) batch_scalar_kernel(BatchSysTable sys, double* scal, int* flags,
                                                              const double* __restrict__ partial, int64_t pstride,
                                                              double tol2, int max_iter) {
    const int s = blockIdx.x;
    if ((OP == 0 || OP == 1) && flags[2 * s]) return;
    int t = 0;
    while (t + 1 < sys.ntasks && sys.sys0[t + 1] <= s) ++t;
    const int n = (OP == 0 || OP == 1) ? sys.ntile_hop[t] : sys.ntile_vec[t];
    const double v = sys_sum(partial, pstride, s, n);
    if (threadIdx.x != 0) return;
    double* sc = scal + (int64_t)s * kNScal;
    if constexpr (OP == 0) {
        sc[kPQ] = v;
        sc[kAlpha] = sc[kRR] / v;
    } else if constexpr (OP == 1) {
        sc[kBeta] = v / sc[kRR];
        sc[kRR] = v;
        const int it = flags[2 * s + 1] + 1;
        flags[2 * s + 1] = it;
        if (v <= sc[kStop] || it >= max_iter) flags[2 * s] = 1;
    } else if constexpr (OP == 2) {
        sc[kNorm] = v;
    } else if constexpr (OP == 4) {
        sc[kBB] = v;
    } else {
        sc[kRR] = v;
        sc[kStop] = tol2 * sc[kBB];
        flags[2 * s] = v <= sc[kStop] ? 1 : 0;
        flags[2 * s + 1] = 0;
    }
}

}  // namespace

// ------------------------------------------------------------------ launchers

template <typename R, int MODE, int SW, int RY, int NR = 1>
static const void* batch_hop_fn() {
    constexpr bool pipe = false;  // the persistent loop leaves no room for two register sets
    return reinterpret_cast<const void*>(&batch_hop_kernel<R, MODE, SW, RY, NR, pipe>);
}

template <typename R, int MODE>
static const void* batch_hop_sel(int shape) {
    switch (shape) {
        case kShapeMfma: return reinterpret_cast<const void*>(&batch_hop_mfma_kernel<R, MODE>);
        case kShape4x1: return batch_hop_fn<R, MODE, 4, 1>();
        case kShape2x2: return batch_hop_fn<R, MODE, 2, 2>();
        case kShape1x4: return batch_hop_fn<R, MODE, 1, 4>();
        case kShape2x4: return batch_hop_fn<R, MODE, 2, 4>();
        case kShape1x12: return batch_hop_fn<R, MODE, 1, 12>();
        case kShape2x1r2: return batch_hop_fn<R, MODE, 2, 1, 2>();
        case kShape1x2r2: return batch_hop_fn<R, MODE, 1, 2, 2>();
        case kShape2x2r2: return batch_hop_fn<R, MODE, 2, 2, 2>();
        case kShape1x4r3: return batch_hop_fn<R, MODE, 1, 4, 3>();
        case kShape2x2r3: return batch_hop_fn<R, MODE, 2, 2, 3>();
        case kShape1x3r4: return batch_hop_fn<R, MODE, 1, 3, 4>();
        default: return batch_hop_fn<R, MODE, 2, 1, 4>();
    }
}

template <typename R>
static const void* batch_hop_kernel_ptr(int shape, int mode) {
    switch (mode) {
        case 0: return batch_hop_sel<R, 0>(shape);
        case 1: return batch_hop_sel<R, 1>(shape);
        case 2: return batch_hop_sel<R, 2>(shape);
        default: return batch_hop_sel<R, 3>(shape);
    }
}

// Workgroups of `fn` the device holds at once (CUs x resident workgroups per
// CU), queried once per kernel and device and remembered, so that launches
// made while a stream is being captured into a graph query nothing.
static int resident_blocks(const void* fn, int threads) {
    struct Entry {
        const void* fn;
        int dev, threads, blocks;
    };
    static std::mutex mu;
    static std::vector<Entry> cache;
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lock(mu);
    for (const Entry& e : cache)
        if (e.fn == fn && e.dev == dev && e.threads == threads) return e.blocks;
    int ncu = 256, per = 1;
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, threads, 0) != hipSuccess || per < 1) per = 1;
    cache.push_back({fn, dev, threads, ncu * per});
    return ncu * per;
}

// Persistent grid: all the workgroups that fit on the device at once, a
// multiple of the XCD count, no more than the items need.
static int persistent_grid(const void* fn, int threads, int nitems) {
    int grid = resident_blocks(fn, threads);
    const int need = (nitems + kXcds - 1) / kXcds * kXcds;
    if (grid > need) grid = need;
    grid = (grid + kXcds - 1) / kXcds * kXcds;
    return grid < kXcds ? kXcds : grid;
}

template <typename R, bool PIPE, int RG, bool LDS>
static hipError_t launch_tmarch(const BatchHopTable<R>& tab, int mode, hipStream_t s) {
    // every XCD's list holds ceil(nb / 8) workgroups of each task at most
    int per_xcd = 0;
    for (int k = 0; k < tab.ntasks; ++k) {
        const BatchHopTask<R>& t = tab.t[k];
        if (t.tm_rg != RG) return hipErrorInvalidValue;
        per_xcd += (batch_tmarch_blocks(t.g.L[0], t.tm_steps, t.tm_nw, t.nrhs, RG) + kXcds - 1) / kXcds;
    }
    const int grid = per_xcd * kXcds;
    if (grid == 0) return hipSuccess;
    const unsigned lds = LDS ? 8 * 9 * 64 * sizeof(cx<R>) : 0;
    if (lds > 65536) {
        // above the default limit of dynamic LDS per workgroup (gfx950 has
        // 160 KB per CU)
        static bool raised[4] = {false, false, false, false};
        if (!raised[mode & 3]) {
            const void* fn = nullptr;
            switch (mode) {
                case 0: fn = reinterpret_cast<const void*>(&batch_tmarch_lds_kernel<R, 0>); break;
                case 1: fn = reinterpret_cast<const void*>(&batch_tmarch_lds_kernel<R, 1>); break;
                case 2: fn = reinterpret_cast<const void*>(&batch_tmarch_lds_kernel<R, 2>); break;
                default: fn = reinterpret_cast<const void*>(&batch_tmarch_lds_kernel<R, 3>); break;
            }
            const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
            raised[mode & 3] = true;
        }
    }
    if constexpr (LDS) {
        switch (mode) {
            case 0: hipLaunchKernelGGL((batch_tmarch_lds_kernel<R, 0>), dim3(grid), dim3(256), lds, s, tab); break;
            case 1: hipLaunchKernelGGL((batch_tmarch_lds_kernel<R, 1>), dim3(grid), dim3(256), lds, s, tab); break;
            case 2: hipLaunchKernelGGL((batch_tmarch_lds_kernel<R, 2>), dim3(grid), dim3(256), lds, s, tab); break;
            default: hipLaunchKernelGGL((batch_tmarch_lds_kernel<R, 3>), dim3(grid), dim3(256), lds, s, tab); break;
        }
    } else {
        switch (mode) {
            case 0: hipLaunchKernelGGL((batch_tmarch_kernel<R, 0, PIPE, RG, false>), dim3(grid), dim3(256), 0, s, tab); break;
            case 1: hipLaunchKernelGGL((batch_tmarch_kernel<R, 1, PIPE, RG, false>), dim3(grid), dim3(256), 0, s, tab); break;
            case 2: hipLaunchKernelGGL((batch_tmarch_kernel<R, 2, PIPE, RG, false>), dim3(grid), dim3(256), 0, s, tab); break;
            default: hipLaunchKernelGGL((batch_tmarch_kernel<R, 3, PIPE, RG, false>), dim3(grid), dim3(256), 0, s, tab); break;
        }
    }
    return hipGetLastError();
}

template <typename R>
hipError_t launch_batch_hop(const BatchHopTable<R>& tasks, int nitems, int shape, int mode, hipStream_t s) {
    // t-march shapes: the host has set tm_steps, tm_nw, tm_slice and tm_rg of
    // every task (slices of whole tiles of 256 / tm_rg pairs, steps dividing T)
    if (shape == kShapeTMarch) return launch_tmarch<R, false, 1, false>(tasks, mode, s);
    if (shape == kShapeTMarchPipe) return launch_tmarch<R, true, 1, false>(tasks, mode, s);
    if (shape == kShapeTMarch4) return launch_tmarch<R, false, 4, false>(tasks, mode, s);
    if (shape == kShapeTMarchLds) return launch_tmarch<R, false, 4, true>(tasks, mode, s);
    if (nitems == 0) return hipSuccess;
    int sw, ry, nr;
    batch_shape(shape, &sw, &ry, &nr);
    const int threads = 64 * sw * ry;
    const void* fn = batch_hop_kernel_ptr<R>(shape, mode);
    const int grid = persistent_grid(fn, threads, nitems);
    BatchHopTable<R> tab = tasks;
    void* args[] = {(void*)&tab, (void*)&nitems};
    return hipLaunchKernel(fn, dim3(grid), dim3(threads), args, 0, s);
}

template <int OP> static const void* vec_fn() { return reinterpret_cast<const void*>(&batch_vec_kernel<OP>); }

hipError_t launch_batch_vec(int op, const BatchVecTable& tasks, int nitems, const double* scal, const int* flags,
                            hipStream_t s) {
    if (nitems == 0) return hipSuccess;
    const void* fn = op == 0 ? vec_fn<0>() : op == 1 ? vec_fn<1>() : op == 2 ? vec_fn<2>() : op == 3 ? vec_fn<3>()
                                                                                                : vec_fn<4>();
    const int grid = persistent_grid(fn, kBlock, nitems);
    BatchVecTable tab = tasks;
    void* args[] = {(void*)&tab, (void*)&nitems, (void*)&scal, (void*)&flags};
    return hipLaunchKernel(fn, dim3(grid), dim3(kBlock), args, 0, s);
}

hipError_t launch_batch_scalar(int op, int nsys, const BatchSysTable& sys, double* scal, int* flags,
                               const double* partial, int64_t pstride, double tol2, int max_iter, hipStream_t s) {
    if (nsys == 0) return hipSuccess;
    switch (op) {
        case 0: hipLaunchKernelGGL(batch_scalar_kernel<0>, dim3(nsys), dim3(kBlock), 0, s, sys, scal, flags, partial,
                                   pstride, tol2, max_iter); break;
        case 1: hipLaunchKernelGGL(batch_scalar_kernel<1>, dim3(nsys), dim3(kBlock), 0, s, sys, scal, flags, partial,
                                   pstride, tol2, max_iter); break;
        case 2: hipLaunchKernelGGL(batch_scalar_kernel<2>, dim3(nsys), dim3(kBlock), 0, s, sys, scal, flags, partial,
                                   pstride, tol2, max_iter); break;
        case 3: hipLaunchKernelGGL(batch_scalar_kernel<3>, dim3(nsys), dim3(kBlock), 0, s, sys, scal, flags, partial,
                                   pstride, tol2, max_iter); break;
        default: hipLaunchKernelGGL(batch_scalar_kernel<4>, dim3(nsys), dim3(kBlock), 0, s, sys, scal, flags,
                                    partial, pstride, tol2, max_iter); break;
    }
    return hipGetLastError();
}

int batch_vec_tiles(int Vh) { return (Vh + kVecTile - 1) / kVecTile; }

void batch_prepare(int shape) {
    if (batch_is_tmarch(shape)) return;  // not persistent: nothing to size
    int sw, ry, nr;
    batch_shape(shape, &sw, &ry, &nr);
    for (int mode = 0; mode < 4; ++mode) {
        (void)resident_blocks(batch_hop_kernel_ptr<double>(shape, mode), 64 * sw * ry);
        (void)resident_blocks(batch_hop_kernel_ptr<float>(shape, mode), 64 * sw * ry);
    }
    const void* v[5] = {vec_fn<0>(), vec_fn<1>(), vec_fn<2>(), vec_fn<3>(), vec_fn<4>()};
    for (const void* f : v) (void)resident_blocks(f, kBlock);
}

template hipError_t launch_batch_hop<double>(const BatchHopTable<double>&, int, int, int, hipStream_t);
template hipError_t launch_batch_hop<float>(const BatchHopTable<float>&, int, int, int, hipStream_t);

}  // namespace tmh
