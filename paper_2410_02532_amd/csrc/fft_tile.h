// fft_tile.h -- LDS-staged Stockham FFT over a batch of short transforms held
// by one workgroup, plus the complex helpers the kernels share.
//
// A tile keeps `count` transforms of length m (a power of two) in LDS; element
// n of transform t sits at lds_index(t*m + n). Each stage of radix R (8, 4 or
// 2) reads R values per butterfly at stride m/R, twiddles them, applies the
// R-point DFT in registers and writes them back at stride p in the
// self-sorting (Stockham) order, so the result comes out in natural order
// without a bit-reversal pass. The stage is done in place: every thread loads
// all of its butterflies into registers, the workgroup synchronizes, then
// every thread writes. Twiddles of the butterflies come from one table
// e^{-2 pi i q/TWL}, q < TWL, built on the host in FP64.
#pragma once
#include <hip/hip_runtime.h>

namespace opo {

constexpr int kThreads = 256;   // threads per workgroup of every tile kernel
constexpr int kTwL = 8192;      // length of the butterfly twiddle table
// Tile points per thread (register budget of a stage): a tile holds at most
// kThreads * max_pts<R>() points.
template <typename R> __host__ __device__ constexpr int max_pts() { return sizeof(R) == 4 ? 16 : 8; }

template <typename R> struct cplx_of;
template <> struct cplx_of<float> { using type = float2; };
template <> struct cplx_of<double> { using type = double2; };
template <typename R> using cplx = typename cplx_of<R>::type;

template <typename V> __device__ __forceinline__ V mk(decltype(V::x) re, decltype(V::x) im)
{
    V v;
    v.x = re;
    v.y = im;
    return v;
}
template <typename V> __device__ __forceinline__ V cadd(V a, V b) { return mk<V>(a.x + b.x, a.y + b.y); }
template <typename V> __device__ __forceinline__ V csub(V a, V b) { return mk<V>(a.x - b.x, a.y - b.y); }
template <typename V> __device__ __forceinline__ V cmul(V a, V b)
{
    return mk<V>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
template <typename V> __device__ __forceinline__ V cmulc(V a, V b)
{
    return mk<V>(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
template <typename V> __device__ __forceinline__ V conjv(V a) { return mk<V>(a.x, -a.y); }
template <typename V, typename S> __device__ __forceinline__ V cscale(V a, S s) { return mk<V>(a.x * s, a.y * s); }
// multiply by -i*dir... : rot(a, dir) = a * (dir * i)
template <int DIR, typename V> __device__ __forceinline__ V rot90(V a)
{
    // DIR = +1: a * i ; DIR = -1: a * (-i)
    return DIR > 0 ? mk<V>(-a.y, a.x) : mk<V>(a.y, -a.x);
}

// LDS padding: one spare element every 2^shift elements spreads strided
// accesses over the banks (8-byte elements: every 16, 16-byte: every 8).
template <typename R> struct lds_pad { static constexpr int shift = sizeof(R) == 4 ? 4 : 3; };
template <typename R> __device__ __forceinline__ int lds_index(int e) { return e + (e >> lds_pad<R>::shift); }
template <typename R> __host__ __device__ constexpr int lds_elems(int n) { return n + (n >> (sizeof(R) == 4 ? 4 : 3)) + 1; }

// R-point DFT in registers, y_k = sum_j x_j e^{DIR 2 pi i jk/R}.
template <int DIR, typename V> __device__ __forceinline__ void dft2(V *x)
{
    V a = x[0], b = x[1];
    x[0] = cadd(a, b);
    x[1] = csub(a, b);
}

template <int DIR, typename V> __device__ __forceinline__ void dft4(V *x)
{
    V a = cadd(x[0], x[2]), b = csub(x[0], x[2]);
    V c = cadd(x[1], x[3]), d = rot90<DIR>(csub(x[1], x[3]));
    x[0] = cadd(a, c);
    x[2] = csub(a, c);
    x[1] = cadd(b, d);
    x[3] = csub(b, d);
}

template <int DIR, typename V> __device__ __forceinline__ void dft8(V *x)
{
    using S = decltype(V::x);
    const S h = S(0.70710678118654752440);
    V e[4] = {x[0], x[2], x[4], x[6]};
    V o[4] = {x[1], x[3], x[5], x[7]};
    dft4<DIR>(e);
    dft4<DIR>(o);
    // w^k = e^{DIR 2 pi i k/8}
    V o1 = mk<V>(h * (o[1].x - DIR * o[1].y), h * (o[1].y + DIR * o[1].x));
    V o2 = rot90<DIR>(o[2]);
    V o3 = mk<V>(h * (-o[3].x - DIR * o[3].y), h * (-o[3].y + DIR * o[3].x));
    x[0] = cadd(e[0], o[0]);
    x[4] = csub(e[0], o[0]);
    x[1] = cadd(e[1], o1);
    x[5] = csub(e[1], o1);
    x[2] = cadd(e[2], o2);
    x[6] = csub(e[2], o2);
    x[3] = cadd(e[3], o3);
    x[7] = csub(e[3], o3);
}

template <int RAD, int DIR, typename V> __device__ __forceinline__ void dft(V *x)
{
    if constexpr (RAD == 8) dft8<DIR>(x);
    else if constexpr (RAD == 4) dft4<DIR>(x);
    else dft2<DIR>(x);
}

// One Stockham stage of radix RAD over `count` transforms of length m whose
// sub-transforms of length p are already done.
template <typename R, int DIR, int RAD>
__device__ __forceinline__ void fft_stage(cplx<R> *s, int count, int log2m, int p,
                                          const cplx<R> *__restrict__ tw)
{
    using V = cplx<R>;
    constexpr int NB = max_pts<R>() / RAD;   // butterflies a thread may own
    const int m = 1 << log2m;
    const int nb = m / RAD;             // butterflies per transform
    const int lognb = log2m - (RAD == 8 ? 3 : RAD == 4 ? 2 : 1);
    const int total = count << lognb;
    const int tw_stride = kTwL / (p * RAD);
    V v[NB][RAD];
#pragma unroll
    for (int u = 0; u < NB; ++u) {
        const int b = threadIdx.x + u * kThreads;
        if (b < total) {
            const int t = b >> lognb, i = b & (nb - 1);
            const int base = t << log2m;
#pragma unroll
            for (int r = 0; r < RAD; ++r)
                v[u][r] = s[lds_index<R>(base + i + r * nb)];
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < NB; ++u) {
        const int b = threadIdx.x + u * kThreads;
        if (b < total) {
            const int t = b >> lognb, i = b & (nb - 1);
            const int base = t << log2m;
            const int k = i & (p - 1);
            if (p > 1) {
#pragma unroll
                for (int r = 1; r < RAD; ++r) {
                    V w = tw[r * k * tw_stride];
                    if (DIR > 0) w = conjv(w);
                    v[u][r] = cmul(v[u][r], w);
                }
            }
            dft<RAD, DIR>(v[u]);
            const int j = (i - k) * RAD + k;
#pragma unroll
            for (int r = 0; r < RAD; ++r)
                s[lds_index<R>(base + j + r * p)] = v[u][r];
        }
    }
    __syncthreads();
}

// Unnormalized DFT of `count` transforms of length 2^log2m in LDS, DIR = -1
// forward (e^{-...}), +1 inverse (e^{+...}). Expects a synchronized tile.
template <typename R, int DIR>
__device__ void tile_fft(cplx<R> *s, int count, int log2m, const cplx<R> *__restrict__ tw)
{
    int p = 1, left = log2m;
    while (left >= 3) {
        fft_stage<R, DIR, 8>(s, count, log2m, p, tw);
        p <<= 3;
        left -= 3;
    }
    if (left == 2) fft_stage<R, DIR, 4>(s, count, log2m, p, tw);
    else if (left == 1) fft_stage<R, DIR, 2>(s, count, log2m, p, tw);
}

} // namespace opo
