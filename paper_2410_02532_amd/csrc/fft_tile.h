// fft_tile.h -- register-resident Stockham FFT over short transforms held by a
// workgroup, plus the complex helpers the kernels share.
//
// A transform of length N is spread over N/PF threads; thread t of the
// transform keeps the PF samples at positions t + m*(N/PF), m < PF, in
// registers. Each Stockham stage of radix RS (8, 4 or 2, dividing PF) runs
// PF/RS butterflies per thread whose inputs are exactly those register
// samples: butterfly u of thread t has index i = t + u*(N/PF) and reads
// positions i + r*(N/RS). The stage twiddles by w^{r k} (k = i mod P, P the
// product of the earlier radices, w = e^{-+2 pi i/(P RS)}), applies the
// RS-point DFT and writes the self-sorting positions j + r*P,
// j = (i - k)*RS + k. Between stages the samples go through LDS (one write,
// one read back of the thread's own positions). In the last stage P = N/RS,
// so j = i and the outputs land on the thread's own positions: the result
// comes back in natural order in registers, with no LDS traffic. Twiddles
// come from a stage-major table built on the host in FP64 (held as
// compensated FP32 pairs in the FP32 path), and are loaded once per stage and
// reused for every transform the thread owns.
#pragma once
#include <hip/hip_runtime.h>
#include <type_traits>

namespace opo {

constexpr int kThreads = 256;   // threads per workgroup of every tile kernel
constexpr int kTwL = 8192;      // longest transform the twiddle table serves

// Stage-major twiddle table: for a stage of radix RS after sub-transforms of
// length P, the factors w^{r k} = e^{-2 pi i r k/(P RS)}, r = 1..RS-1, of
// butterfly class k < P sit at tw_index(RS, P, k) + r - 1. One thread's
// factors are contiguous and consecutive k are adjacent, so a stage reads a
// compact, coalesced block instead of strided entries of one long table.
// Entries of radix rs: P runs over the powers of two with P*rs <= kTwL, and
// sum_{P = 1, 2, ..., M} P = 2M - 1.
__host__ __device__ constexpr int tw_block_size(int rs) { return (2 * (kTwL / rs) - 1) * (rs - 1); }
__host__ __device__ constexpr int tw_block(int rs)
{
    return rs == 2    ? 0
           : rs == 4  ? tw_block_size(2)
           : rs == 8  ? tw_block_size(2) + tw_block_size(4)
                      : tw_block_size(2) + tw_block_size(4) + tw_block_size(8);
}
__host__ __device__ constexpr int tw_index(int rs, int p, int k)
{
    return tw_block(rs) + (p - 1 + k) * (rs - 1);
}
constexpr int kTwEntries = tw_block_size(2) + tw_block_size(4) + tw_block_size(8) + tw_block_size(16);

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
// a * (DIR i): DIR = +1 multiplies by i, DIR = -1 by -i
template <int DIR, typename V> __device__ __forceinline__ V rot90(V a)
{
    return DIR > 0 ? mk<V>(-a.y, a.x) : mk<V>(a.y, -a.x);
}

// A unit-modulus factor (twiddle, propagator, mirror) carried with FP64
// accuracy. In the FP32 path it is the FP32 value hi nearest to the FP64
// factor plus the FP32 remainder lo, and x*(hi + lo) is formed with the small
// product first: the factor's own rounding then no longer biases |x| by the
// same amount at every step (a per-frequency error that a plain FP32 factor
// would compound over 10^5 steps). In the FP64 path it is the factor itself.
template <typename R> struct Phasor;
template <> struct Phasor<float> {
    float2 hi, lo;
};
template <> struct Phasor<double> {
    double2 hi;
};

template <typename R> __host__ __device__ __forceinline__ Phasor<R> make_phasor(double re, double im);
template <> __host__ __device__ __forceinline__ Phasor<float> make_phasor<float>(double re, double im)
{
    Phasor<float> p;
    p.hi.x = static_cast<float>(re);
    p.hi.y = static_cast<float>(im);
    p.lo.x = static_cast<float>(re - static_cast<double>(p.hi.x));
    p.lo.y = static_cast<float>(im - static_cast<double>(p.hi.y));
    return p;
}
template <> __host__ __device__ __forceinline__ Phasor<double> make_phasor<double>(double re, double im)
{
    Phasor<double> p;
    p.hi.x = re;
    p.hi.y = im;
    return p;
}

// x * w (CONJ = false) or x * conj(w) (CONJ = true).
template <bool CONJ = false>
__device__ __forceinline__ float2 pmul(float2 x, const Phasor<float> &w)
{
    const float hy = CONJ ? -w.hi.y : w.hi.y, ly = CONJ ? -w.lo.y : w.lo.y;
    float re = x.x * w.lo.x - x.y * ly;
    float im = x.x * ly + x.y * w.lo.x;
    re = fmaf(x.x, w.hi.x, re);
    re = fmaf(-x.y, hy, re);
    im = fmaf(x.x, hy, im);
    im = fmaf(x.y, w.hi.x, im);
    return make_float2(re, im);
}
template <bool CONJ = false>
__device__ __forceinline__ double2 pmul(double2 x, const Phasor<double> &w)
{
    return CONJ ? cmulc(x, w.hi) : cmul(x, w.hi);
}

// LDS padding: one spare element every 2^shift elements spreads strided
// accesses over the banks (8-byte elements: every 16, 16-byte: every 8).
#ifndef OPO_LDS_SHIFT_F32
#define OPO_LDS_SHIFT_F32 5
#endif
template <typename R> __host__ __device__ constexpr int lds_shift() { return sizeof(R) == 4 ? OPO_LDS_SHIFT_F32 : 3; }
template <typename R> __device__ __forceinline__ int lds_index(int e) { return e + (e >> lds_shift<R>()); }
template <typename R> __host__ __device__ constexpr int lds_elems(int n) { return n + (n >> lds_shift<R>()) + 1; }

// Workgroup barrier that orders LDS accesses only: global loads still in
// flight (a prefetch of the next tile) are not waited for, unlike
// __syncthreads().
__device__ __forceinline__ void lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// The same for an exchange among the lanes of one wavefront (every transform of
// the exchange lies within one wave): LDS accesses of one wave complete in
// order, so only code motion has to be stopped, no barrier is needed.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

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

// s * 1/sqrt(2): in FP32 with the constant split in hi + lo, so that the
// eighth-root twiddles keep unit modulus to FP64 accuracy (a plain FP32
// 1/sqrt(2) has |w|^2 = 1 - 2.7e-8, the same at every step).
__device__ __forceinline__ float mul_rsqrt2(float a)
{
    const float hi = 0.70710677f;                 // nearest FP32 to 1/sqrt(2)
    const float lo = 1.21016175e-08f;             // 1/sqrt(2) - hi
    return fmaf(a, hi, a * lo);
}
__device__ __forceinline__ double mul_rsqrt2(double a) { return a * 0.70710678118654752440; }

template <int DIR, typename V> __device__ __forceinline__ void dft8(V *x)
{
    V e[4] = {x[0], x[2], x[4], x[6]};
    V o[4] = {x[1], x[3], x[5], x[7]};
    dft4<DIR>(e);
    dft4<DIR>(o);
    // w^k = e^{DIR 2 pi i k/8}
    V o1 = mk<V>(mul_rsqrt2(o[1].x - DIR * o[1].y), mul_rsqrt2(o[1].y + DIR * o[1].x));
    V o2 = rot90<DIR>(o[2]);
    V o3 = mk<V>(mul_rsqrt2(-o[3].x - DIR * o[3].y), mul_rsqrt2(-o[3].y + DIR * o[3].x));
    x[0] = cadd(e[0], o[0]);
    x[4] = csub(e[0], o[0]);
    x[1] = cadd(e[1], o1);
    x[5] = csub(e[1], o1);
    x[2] = cadd(e[2], o2);
    x[6] = csub(e[2], o2);
    x[3] = cadd(e[3], o3);
    x[7] = csub(e[3], o3);
}

// 16 points as 4 x 4: DFT4 over the samples j1 + 4 j2 of each j1, the
// internal twiddles w^{j1 k1} (w = e^{DIR 2 pi i/16}), then DFT4 over j1;
// output k1 + 4 k2. w^2, w^4 and w^6 take the eighth-root products of dft8;
// w, w^3 and w^9 = -w are compensated FP32 phasors like every other
// unit-modulus factor.
template <int DIR, typename V> __device__ __forceinline__ void dft16(V *x)
{
    using R = decltype(x[0].x);
    constexpr double c8 = 0.92387953251128675613, s8 = 0.38268343236508977173;   // cos, sin of pi/8
    const Phasor<R> w1 = make_phasor<R>(c8, DIR * s8);
    const Phasor<R> w3 = make_phasor<R>(s8, DIR * c8);
    V a[4][4];
#pragma unroll
    for (int j1 = 0; j1 < 4; ++j1) {
#pragma unroll
        for (int j2 = 0; j2 < 4; ++j2) a[j1][j2] = x[j1 + 4 * j2];
        dft4<DIR>(a[j1]);
    }
    // a[j1][k1] *= w^{j1 k1}
    a[1][1] = pmul(a[1][1], w1);
    a[1][2] = mk<V>(mul_rsqrt2(a[1][2].x - DIR * a[1][2].y), mul_rsqrt2(a[1][2].y + DIR * a[1][2].x));
    a[1][3] = pmul(a[1][3], w3);
    a[2][1] = mk<V>(mul_rsqrt2(a[2][1].x - DIR * a[2][1].y), mul_rsqrt2(a[2][1].y + DIR * a[2][1].x));
    a[2][2] = rot90<DIR>(a[2][2]);
    a[2][3] = mk<V>(mul_rsqrt2(-a[2][3].x - DIR * a[2][3].y), mul_rsqrt2(-a[2][3].y + DIR * a[2][3].x));
    a[3][1] = pmul(a[3][1], w3);
    a[3][2] = mk<V>(mul_rsqrt2(-a[3][2].x - DIR * a[3][2].y), mul_rsqrt2(-a[3][2].y + DIR * a[3][2].x));
    a[3][3] = pmul(a[3][3], w1);
    a[3][3] = mk<V>(-a[3][3].x, -a[3][3].y);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        V b[4] = {a[0][k1], a[1][k1], a[2][k1], a[3][k1]};
        dft4<DIR>(b);
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) x[k1 + 4 * k2] = b[k2];
    }
}

template <int RAD, int DIR, typename V> __device__ __forceinline__ void dft(V *x)
{
    if constexpr (RAD == 16) dft16<DIR>(x);
    else if constexpr (RAD == 8) dft8<DIR>(x);
    else if constexpr (RAD == 4) dft4<DIR>(x);
    else dft2<DIR>(x);
}

// Radix of the stage that follows sub-transforms of length P. Radix 16 serves
// transforms of up to R16 points: 2048 in the row tiles (at 4096 four radix-8
// stages ran faster than three radix-16 ones there); the resident passes, whose
// threads hold 16 samples of a transform anyway, use it at every length.
template <int N, int PF, int P, int R16 = 2048> __host__ __device__ constexpr int stage_radix()
{
    return (N <= R16 && N / P >= 16 && PF % 16 == 0) ? 16
           : (N / P >= 8 && PF % 8 == 0) ? 8
           : (N / P >= 4 && PF % 4 == 0) ? 4
                                          : 2;
}

// One stage over NTR transforms held by this thread. Position n of transform
// tr lives at LDS element base[tr] + n*LS; t is the thread's index in its
// transform.
template <typename R, int N, int PF, int NTR, int DIR, int LS, int RS, int P, bool LIN, bool WAVE>
__device__ __forceinline__ void reg_stage(cplx<R> (&v)[NTR][PF], cplx<R> *lds, const int (&base)[NTR],
                                          int t, const Phasor<R> *__restrict__ tw)
{
    // LDS element of position e: padded by lds_index, or as given when the layout
    // is already padded by the caller (LIN: linear in e, so that the offsets of a
    // thread's positions are compile-time constants)
    auto at = [](int e) { return LIN ? e : lds_index<R>(e); };
    using V = cplx<R>;
    constexpr int NBT = PF / RS;       // butterflies per thread and transform
    constexpr int STRIDE = N / PF;     // distance between a thread's samples
    constexpr bool LAST = P * RS == N;
    Phasor<R> w[NBT][RS];
    if constexpr (P > 1) {
#pragma unroll
        for (int u = 0; u < NBT; ++u) {
            const int k = (t + u * STRIDE) & (P - 1);
            const Phasor<R> *q = tw + tw_index(RS, P, k);
#pragma unroll
            for (int r = 1; r < RS; ++r)
                w[u][r] = q[r - 1];
        }
    }
#pragma unroll
    for (int tr = 0; tr < NTR; ++tr) {
#pragma unroll
        for (int u = 0; u < NBT; ++u) {
            V x[RS];
#pragma unroll
            for (int r = 0; r < RS; ++r)
                x[r] = v[tr][u + r * NBT];
            if constexpr (P > 1) {
#pragma unroll
                for (int r = 1; r < RS; ++r)
                    x[r] = pmul<(DIR > 0)>(x[r], w[u][r]);
            }
            dft<RS, DIR>(x);
            if constexpr (LAST) {
#pragma unroll
                for (int r = 0; r < RS; ++r)
                    v[tr][u + r * NBT] = x[r];
            } else {
                const int i = t + u * STRIDE;
                const int k = i & (P - 1);
                const int j = (i - k) * RS + k;
#pragma unroll
                for (int r = 0; r < RS; ++r)
                    lds[at(base[tr] + (j + r * P) * LS)] = x[r];
            }
        }
    }
    if constexpr (!LAST) {
        if constexpr (WAVE) wave_lds_sync(); else lds_sync();
#pragma unroll
        for (int tr = 0; tr < NTR; ++tr)
#pragma unroll
            for (int m = 0; m < PF; ++m)
                v[tr][m] = lds[at(base[tr] + (t + m * STRIDE) * LS)];
        if constexpr (WAVE) wave_lds_sync(); else lds_sync();
    }
}

template <typename R, int N, int PF, int NTR, int DIR, int LS, int P, int R16, bool LIN, bool WAVE>
__device__ __forceinline__ void reg_fft_from(cplx<R> (&v)[NTR][PF], cplx<R> *lds, const int (&base)[NTR],
                                             int t, const Phasor<R> *__restrict__ tw)
{
    if constexpr (P < N) {
        constexpr int RS = stage_radix<N, PF, P, R16>();
        reg_stage<R, N, PF, NTR, DIR, LS, RS, P, LIN, WAVE>(v, lds, base, t, tw);
        reg_fft_from<R, N, PF, NTR, DIR, LS, P * RS, R16, LIN, WAVE>(v, lds, base, t, tw);
    }
}

// Unnormalized DFT (DIR -1: e^{-...}, +1: e^{+...}) of NTR transforms of
// length N. On entry and on exit v[tr][m] is sample t + m*(N/PF). Every
// thread of the workgroup must call it (it synchronizes the workgroup when
// N > PF). LS is the LDS element stride between consecutive positions; radix-16
// stages serve transforms of up to R16 points. LIN: base and LS already lay the
// positions out without bank conflicts (no lds_index padding). WAVE: the threads
// of every transform exchanging through this thread's LDS positions belong to its
// own wavefront, so the exchanges synchronize the wave only.
template <typename R, int N, int PF, int NTR, int DIR, int LS, int R16 = 2048, bool LIN = false, bool WAVE = false>
__device__ __forceinline__ void reg_fft(cplx<R> (&v)[NTR][PF], cplx<R> *lds, const int (&base)[NTR], int t,
                                        const Phasor<R> *__restrict__ tw)
{
    reg_fft_from<R, N, PF, NTR, DIR, LS, 1, R16, LIN, WAVE>(v, lds, base, t, tw);
}

// The same transforms stage by stage through one transform's worth of LDS:
// each stage loads its twiddles once and then writes, exchanges and reads
// back the NTR transforms in turn (the arithmetic of each transform is that of
// reg_fft). Used where NTR transforms would not fit LDS together.
template <typename R, int N, int PF, int NTR, int DIR, int RS, int P>
__device__ __forceinline__ void reg_stage_seq(cplx<R> (&v)[NTR][PF], cplx<R> *lds, int t,
                                              const Phasor<R> *__restrict__ tw)
{
    using V = cplx<R>;
    constexpr int NBT = PF / RS;
    constexpr int STRIDE = N / PF;
    constexpr bool LAST = P * RS == N;
    Phasor<R> w[NBT][RS];
    if constexpr (P > 1) {
#pragma unroll
        for (int u = 0; u < NBT; ++u) {
            const int k = (t + u * STRIDE) & (P - 1);
            const Phasor<R> *q = tw + tw_index(RS, P, k);
#pragma unroll
            for (int r = 1; r < RS; ++r)
                w[u][r] = q[r - 1];
        }
    }
#pragma unroll
    for (int tr = 0; tr < NTR; ++tr) {
#pragma unroll
        for (int u = 0; u < NBT; ++u) {
            V x[RS];
#pragma unroll
            for (int r = 0; r < RS; ++r)
                x[r] = v[tr][u + r * NBT];
            if constexpr (P > 1) {
#pragma unroll
                for (int r = 1; r < RS; ++r)
                    x[r] = pmul<(DIR > 0)>(x[r], w[u][r]);
            }
            dft<RS, DIR>(x);
            if constexpr (LAST) {
#pragma unroll
                for (int r = 0; r < RS; ++r)
                    v[tr][u + r * NBT] = x[r];
            } else {
                const int i = t + u * STRIDE;
                const int k = i & (P - 1);
                const int j = (i - k) * RS + k;
#pragma unroll
                for (int r = 0; r < RS; ++r)
                    lds[lds_index<R>(j + r * P)] = x[r];
            }
        }
        if constexpr (!LAST) {
            lds_sync();
#pragma unroll
            for (int m = 0; m < PF; ++m)
                v[tr][m] = lds[lds_index<R>(t + m * STRIDE)];
            lds_sync();
        }
    }
}

template <typename R, int N, int PF, int NTR, int DIR, int P, int R16>
__device__ __forceinline__ void reg_fft_seq_from(cplx<R> (&v)[NTR][PF], cplx<R> *lds, int t,
                                                 const Phasor<R> *__restrict__ tw)
{
    if constexpr (P < N) {
        constexpr int RS = stage_radix<N, PF, P, R16>();
        reg_stage_seq<R, N, PF, NTR, DIR, RS, P>(v, lds, t, tw);
        reg_fft_seq_from<R, N, PF, NTR, DIR, P * RS, R16>(v, lds, t, tw);
    }
}

// Unnormalized DFT of NTR transforms of length N, one at a time through LDS
// positions 0..N-1 (stride 1), in the layout of reg_fft.
template <typename R, int N, int PF, int NTR, int DIR, int R16 = 2048>
__device__ __forceinline__ void reg_fft_seq(cplx<R> (&v)[NTR][PF], cplx<R> *lds, int t,
                                            const Phasor<R> *__restrict__ tw)
{
    reg_fft_seq_from<R, N, PF, NTR, DIR, 1, R16>(v, lds, t, tw);
}

} // namespace opo
