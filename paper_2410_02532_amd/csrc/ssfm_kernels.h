// ssfm_kernels.h -- gfx950 kernels of one symmetrized split-step Fourier step
// (arXiv 2410.02532, Sec. 2.2, Eqs. 10-11) and of the cavity round trip
// (Eq. 6, Sec. 2.3, Sec. 4.1), for a batch of OPO instances of uneven size.
//
// Each field of nt = n1*n2 samples is transformed with a four-step FFT: the
// column pass does n2-point transforms down the columns j1 (stride n1) and
// multiplies by W_nt^{j1 k2}; the row pass does n1-point transforms along the
// contiguous rows. A z-step therefore touches HBM twice:
//
//   column pass  [inverse column FFT] -> [RK4 half-step of the previous step]
//                -> [round-trip boundary] -> [RK4 half-step of this step]
//                -> [forward column FFT + twiddle]
//   row pass     forward row FFT -> linear propagator -> inverse row FFT
//                -> conjugate twiddle
//
// The RK4 half-steps (Eqs. 2-4 without the linear operator) are pointwise in
// time and need the three fields of a sample together, so a column tile holds
// `cols` columns of all three fields; the linear propagator (Eq. 5) is
// pointwise in frequency and per field, so a row tile holds `rows` rows of one
// field. Phase arguments (dispersion, dk z, GDD, EOM) are formed and reduced
// modulo one revolution in FP64 and only then turned into FP32 phasors.
#pragma once
#include "fft_tile.h"

namespace opo {

// Per-instance description, built on the host and read by every tile.
struct InstDesc {
    long long off;        // element offset of the pump field; signal +nt, idler +2nt
    long long pump_off;   // element offset of the input-pump samples, -1 = constant pump
    int nt, log2nt;
    int n1, log2n1;       // row length (contiguous)
    int n2, log2n2;       // column length (stride n1)
    int log2cols;         // columns per column tile
    int log2rows;         // rows per row tile
    int tile_a0, tiles_a; // first column tile of the instance, and count
    int tile_b0, tiles_b; // first row tile, and count (3 fields x n2/rows)
    int tw4_off;          // four-step twiddle tables: 2^tw4_bits low entries, then high
    int tw4_bits;
    int res_mask, gdd_mask, eom_mask, pad0;
    double length_mm;
    double kappa[3];      // 1/mm per V/m
    double dk_rev;        // dk / (2 pi)  [rev/mm]
    double disp[3][3];    // dispersion phase [rev/mm] = c0 ks + c1 ks^2 + c2 ks^3 per field
    double alpha_half[3]; // alpha_x / 2
    double mirror[3][2];  // sqrt(R_x) e^{i delta_x}
    double gdd_rev;       // GDD phase [rev] = gdd_rev * ks^2
    double eom_beta;      // EOM phase = beta sin(2 pi rho_j), rho_j = eom_rev0 + eom_rev_step j
    double eom_rev0, eom_rev_step;
    double pump_cw[2];
};

enum : int {
    A_INV = 1,        // start with the inverse column FFT (data left by a row pass)
    A_RK_PREV = 2,    // second half-step of the previous z-step
    A_ENERGY = 4,     // FP64 partial sums of |A_x|^2 after the pass
    A_MIRROR = 8,     // sqrt(R) e^{i delta} on resonant fields (Eq. 6)
    A_EOM = 16,       // EOM phase on the selected fields (Sec. 2.3)
    A_REFRESH = 32,   // input pump into a non-resonant pump, zero non-resonant s/i
    A_RK_THIS = 64,   // first half-step of this z-step
    A_FWD = 128,      // end with the forward column FFT + twiddle (else store samples)
};

enum : int {
    B_DISP = 1,       // multiply by the linear propagator of a step dz (Eq. 5)
    B_GDD = 2,        // multiply the GDD fields by e^{i gamma w^2/2} (Sec. 2.3)
    B_FWD_ONLY = 4,   // forward row FFT only (spectrum read-out)
};

template <typename R> struct StepArgs {
    const InstDesc *inst;
    const int *tile_inst;     // tile -> instance
    cplx<R> *state;
    const cplx<R> *pump;
    const cplx<R> *tw;        // butterfly twiddles e^{-2 pi i q/kTwL}
    const cplx<R> *tw4;       // four-step twiddle tables
    double *partial;          // [column tiles][3] energy partial sums
    int flags;
    int step;                 // z-step j whose first half-step this launch runs
    int nz;                   // steps per pass (dz = L/nz when dz_arg <= 0)
    double dz_arg;            // explicit step, or <= 0
    double zbase;             // z of step 0
};

// e^{2 pi i rho}, rho reduced modulo 1 in FP64 before the cast.
template <typename R> __device__ __forceinline__ cplx<R> phasor_rev(double rho);
template <> __device__ __forceinline__ float2 phasor_rev<float>(double rho)
{
    const double r = rho - rint(rho);
    float sn, cs;
    sincospif(static_cast<float>(2.0 * r), &sn, &cs);
    return make_float2(cs, sn);
}
template <> __device__ __forceinline__ double2 phasor_rev<double>(double rho)
{
    const double r = rho - rint(rho);
    double sn, cs;
    sincospi(2.0 * r, &sn, &cs);
    return make_double2(cs, sn);
}

// e^{i theta} for a small real angle in the working precision.
template <typename R> __device__ __forceinline__ cplx<R> phasor_small(R th);
template <> __device__ __forceinline__ float2 phasor_small<float>(float th)
{
    float sn, cs;
    sincosf(th, &sn, &cs);
    return make_float2(cs, sn);
}
template <> __device__ __forceinline__ double2 phasor_small<double>(double th)
{
    double sn, cs;
    sincos(th, &sn, &cs);
    return make_double2(cs, sn);
}

template <typename R> __device__ __forceinline__ R sin_rev(double rho);
template <> __device__ __forceinline__ float sin_rev<float>(double rho)
{
    return sinpif(static_cast<float>(2.0 * (rho - rint(rho))));
}
template <> __device__ __forceinline__ double sin_rev<double>(double rho)
{
    return sinpi(2.0 * (rho - rint(rho)));
}

// Four-step twiddle W_nt^m = e^{-2 pi i m/nt} from a low and a high table.
template <typename R>
__device__ __forceinline__ cplx<R> twiddle4(const cplx<R> *__restrict__ t, int bits, unsigned m)
{
    const cplx<R> lo = t[m & ((1u << bits) - 1u)];
    const cplx<R> hi = t[(1u << bits) + (m >> bits)];
    return cmul(hi, lo);
}

// Coupling coefficients of one RK4 stage position z, pre-scaled by h/2:
// (i kappa_p e^{-i dk z}, i kappa_s e^{+i dk z}, i kappa_i e^{+i dk z}) * h/2.
template <typename R> struct Coupling {
    cplx<R> c[3];
};

template <typename R>
__device__ __forceinline__ Coupling<R> coupling_at(const InstDesc &d, double z, double half_h)
{
    using V = cplx<R>;
    const double r = d.dk_rev * z;
    const double rr = r - rint(r);
    double sn, cs;
    sincospi(2.0 * rr, &sn, &cs);
    Coupling<R> k;
    // i kappa e^{-i th} = kappa (sin th + i cos th); i kappa e^{+i th} = kappa (-sin th + i cos th)
    const double kp = d.kappa[0] * half_h, ks = d.kappa[1] * half_h, ki = d.kappa[2] * half_h;
    k.c[0] = mk<V>(static_cast<R>(kp * sn), static_cast<R>(kp * cs));
    k.c[1] = mk<V>(static_cast<R>(-ks * sn), static_cast<R>(ks * cs));
    k.c[2] = mk<V>(static_cast<R>(-ki * sn), static_cast<R>(ki * cs));
    return k;
}

// Right-hand side of Eqs. 2-4 (nonlinear part) times h/2.
template <typename V, typename K>
__device__ __forceinline__ void cwe_rhs(const K &k, V ap, V as, V ai, V &fp, V &fs, V &fi)
{
    fp = cmul(k.c[0], cmul(as, ai));
    fs = cmul(k.c[1], cmulc(ap, ai));
    fi = cmul(k.c[2], cmulc(ap, as));
}

// Classical coupled RK4 over one step h with stage coefficients at z0, z0+h/2,
// z0+h (each pre-scaled by h/2, so y + h/2 k_n becomes y + k'_n).
template <typename R>
__device__ __forceinline__ void rk4_point(const Coupling<R> &c0, const Coupling<R> &c1,
                                          const Coupling<R> &c2, cplx<R> &ap, cplx<R> &as,
                                          cplx<R> &ai)
{
    using V = cplx<R>;
    V p1, s1, i1, p2, s2, i2, p3, s3, i3, p4, s4, i4;
    cwe_rhs(c0, ap, as, ai, p1, s1, i1);
    cwe_rhs(c1, cadd(ap, p1), cadd(as, s1), cadd(ai, i1), p2, s2, i2);
    cwe_rhs(c1, cadd(ap, p2), cadd(as, s2), cadd(ai, i2), p3, s3, i3);
    const R two = R(2);
    cwe_rhs(c2, mk<V>(ap.x + two * p3.x, ap.y + two * p3.y), mk<V>(as.x + two * s3.x, as.y + two * s3.y),
            mk<V>(ai.x + two * i3.x, ai.y + two * i3.y), p4, s4, i4);
    const R third = R(1) / R(3);
    ap = mk<V>(ap.x + third * (p1.x + two * (p2.x + p3.x) + p4.x),
               ap.y + third * (p1.y + two * (p2.y + p3.y) + p4.y));
    as = mk<V>(as.x + third * (s1.x + two * (s2.x + s3.x) + s4.x),
               as.y + third * (s1.y + two * (s2.y + s3.y) + s4.y));
    ai = mk<V>(ai.x + third * (i1.x + two * (i2.x + i3.x) + i4.x),
               ai.y + third * (i1.y + two * (i2.y + i3.y) + i4.y));
}

// Fixed-order workgroup sum of three doubles; the result is valid in thread 0.
__device__ __forceinline__ void block_sum3(double v[3], double *scratch /* [3*kThreads/64] */)
{
#pragma unroll
    for (int x = 0; x < 3; ++x) {
        double s = v[x];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1)
            s += __shfl_down(s, o, 64);
        v[x] = s;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0)
        for (int x = 0; x < 3; ++x)
            scratch[x * (kThreads / 64) + wave] = v[x];
    __syncthreads();
    if (threadIdx.x == 0)
        for (int x = 0; x < 3; ++x) {
            double s = 0.0;
            for (int w = 0; w < kThreads / 64; ++w)
                s += scratch[x * (kThreads / 64) + w];
            v[x] = s;
        }
}

// ------------------------------------------------------------------------
// Column pass: time-domain work of a z-step boundary on `cols` columns of the
// three fields of one instance.
template <typename R>
__global__ __launch_bounds__(kThreads) void column_pass(StepArgs<R> a)
{
    using V = cplx<R>;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    V *s = reinterpret_cast<V *>(lds_raw);
    __shared__ double red[3 * kThreads / 64];

    const int tile = blockIdx.x;
    const InstDesc &d = a.inst[a.tile_inst[tile]];
    const int flags = a.flags;
    const int nt = d.nt, n1 = d.n1, log2n2 = d.log2n2, n2 = d.n2;
    const int log2c = d.log2cols, cols = 1 << log2c;
    const int c0 = (tile - d.tile_a0) << log2c;
    const int npts = 3 * cols * n2;   // tile points
    const int nptf = cols * n2;       // points per field
    V *g = a.state + d.off;

    for (int q = threadIdx.x; q < npts; q += kThreads) {
        const int c = q & (cols - 1), rest = q >> log2c;
        const int j2 = rest & (n2 - 1), f = rest >> log2n2;
        s[lds_index<R>(((f << log2c) + c) * n2 + j2)] =
            g[static_cast<long long>(f) * nt + c0 + c + static_cast<long long>(n1) * j2];
    }
    __syncthreads();
    if (flags & A_INV) tile_fft<R, +1>(s, 3 * cols, log2n2, a.tw);

    const double dz = a.dz_arg > 0.0 ? a.dz_arg : d.length_mm / a.nz;
    const double zb = a.dz_arg > 0.0 ? a.zbase : 0.0;
    const double half_h = 0.25 * dz;  // h = dz/2, coefficients carry h/2
    Coupling<R> kp0, kp1, kp2, kt0, kt1, kt2;
    if (flags & A_RK_PREV) {
        const double z0 = zb + (a.step - 1) * dz + 0.5 * dz;
        kp0 = coupling_at<R>(d, z0, half_h);
        kp1 = coupling_at<R>(d, z0 + 0.25 * dz, half_h);
        kp2 = coupling_at<R>(d, z0 + 0.5 * dz, half_h);
    }
    if (flags & A_RK_THIS) {
        const double z0 = zb + a.step * dz;
        kt0 = coupling_at<R>(d, z0, half_h);
        kt1 = coupling_at<R>(d, z0 + 0.25 * dz, half_h);
        kt2 = coupling_at<R>(d, z0 + 0.5 * dz, half_h);
    }
    V mir[3];
#pragma unroll
    for (int x = 0; x < 3; ++x)
        mir[x] = mk<V>(static_cast<R>(d.mirror[x][0]), static_cast<R>(d.mirror[x][1]));
    const V pcw = mk<V>(static_cast<R>(d.pump_cw[0]), static_cast<R>(d.pump_cw[1]));
    const R beta = static_cast<R>(d.eom_beta);
    double en[3] = {0.0, 0.0, 0.0};

    for (int q = threadIdx.x; q < nptf; q += kThreads) {
        const int c = q >> log2n2, j2 = q & (n2 - 1);
        const int e0 = lds_index<R>(c * n2 + j2);
        const int e1 = lds_index<R>((cols + c) * n2 + j2);
        const int e2 = lds_index<R>((2 * cols + c) * n2 + j2);
        V y[3] = {s[e0], s[e1], s[e2]};
        const long long j = static_cast<long long>(c0 + c) + static_cast<long long>(n1) * j2;
        if (flags & A_RK_PREV) rk4_point<R>(kp0, kp1, kp2, y[0], y[1], y[2]);
        if (flags & A_ENERGY) {
#pragma unroll
            for (int x = 0; x < 3; ++x)
                en[x] += static_cast<double>(y[x].x) * y[x].x + static_cast<double>(y[x].y) * y[x].y;
        }
        if (flags & A_MIRROR) {
#pragma unroll
            for (int x = 0; x < 3; ++x)
                if (d.res_mask & (1 << x)) y[x] = cmul(y[x], mir[x]);
        }
        if ((flags & A_EOM) && d.eom_mask) {
            const R th = beta * sin_rev<R>(d.eom_rev0 + d.eom_rev_step * static_cast<double>(j));
            const V e = phasor_small<R>(th);
#pragma unroll
            for (int x = 0; x < 3; ++x)
                if (d.eom_mask & (1 << x)) y[x] = cmul(y[x], e);
        }
        if (flags & A_REFRESH) {
            if (!(d.res_mask & 1)) y[0] = d.pump_off >= 0 ? a.pump[d.pump_off + j] : pcw;
            if (!(d.res_mask & 2)) y[1] = mk<V>(R(0), R(0));
            if (!(d.res_mask & 4)) y[2] = mk<V>(R(0), R(0));
        }
        if (flags & A_RK_THIS) rk4_point<R>(kt0, kt1, kt2, y[0], y[1], y[2]);
        s[e0] = y[0];
        s[e1] = y[1];
        s[e2] = y[2];
    }
    if (flags & A_ENERGY) {
        block_sum3(en, red);
        if (threadIdx.x == 0)
            for (int x = 0; x < 3; ++x)
                a.partial[tile * 3 + x] = en[x];
    }
    __syncthreads();

    if (flags & A_FWD) {
        tile_fft<R, -1>(s, 3 * cols, log2n2, a.tw);
        const V *t4 = a.tw4 + d.tw4_off;
        for (int q = threadIdx.x; q < npts; q += kThreads) {
            const int c = q & (cols - 1), rest = q >> log2c;
            const int k2 = rest & (n2 - 1), f = rest >> log2n2;
            const V v = s[lds_index<R>(((f << log2c) + c) * n2 + k2)];
            const unsigned m = (static_cast<unsigned>(c0 + c) * static_cast<unsigned>(k2)) & (nt - 1);
            g[static_cast<long long>(f) * nt + c0 + c + static_cast<long long>(n1) * k2] =
                cmul(v, twiddle4<R>(t4, d.tw4_bits, m));
        }
    } else {
        for (int q = threadIdx.x; q < npts; q += kThreads) {
            const int c = q & (cols - 1), rest = q >> log2c;
            const int j2 = rest & (n2 - 1), f = rest >> log2n2;
            g[static_cast<long long>(f) * nt + c0 + c + static_cast<long long>(n1) * j2] =
                s[lds_index<R>(((f << log2c) + c) * n2 + j2)];
        }
    }
}

// ------------------------------------------------------------------------
// Row pass: frequency-domain work of a z-step on `rows` rows of one field.
template <typename R>
__global__ __launch_bounds__(kThreads) void row_pass(StepArgs<R> a)
{
    using V = cplx<R>;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    V *s = reinterpret_cast<V *>(lds_raw);

    const int tile = blockIdx.x;
    const InstDesc &d = a.inst[a.tile_inst[tile]];
    const int flags = a.flags;
    const int nt = d.nt, n1 = d.n1, log2n1 = d.log2n1, n2 = d.n2;
    const int log2r = d.log2rows, rows = 1 << log2r;
    const int local = tile - d.tile_b0;
    const int per_field = n2 >> log2r;
    const int f = local / per_field;
    const int r0 = (local - f * per_field) << log2r;
    const int npts = rows * n1;
    V *g = a.state + d.off + static_cast<long long>(f) * nt + static_cast<long long>(n1) * r0;

    for (int q = threadIdx.x; q < npts; q += kThreads)
        s[lds_index<R>(q)] = g[q];
    __syncthreads();
    tile_fft<R, -1>(s, rows, log2n1, a.tw);

    if (flags & B_FWD_ONLY) {
        for (int q = threadIdx.x; q < npts; q += kThreads)
            g[q] = s[lds_index<R>(q)];
        return;
    }

    const double inv_nt = 1.0 / nt;
    if (flags & B_DISP) {
        const double dz = a.dz_arg > 0.0 ? a.dz_arg : d.length_mm / a.nz;
        const R amp = static_cast<R>(exp(-d.alpha_half[f] * dz) * inv_nt);
        const double c1 = d.disp[f][0] * dz, c2 = d.disp[f][1] * dz, c3 = d.disp[f][2] * dz;
        for (int q = threadIdx.x; q < npts; q += kThreads) {
            const int r = q >> log2n1, k1 = q & (n1 - 1);
            const int k = (r0 + r) + n2 * k1;
            const double ks = static_cast<double>(k < (nt >> 1) ? k : k - nt);
            const double rho = ks * (c1 + ks * (c2 + ks * c3));
            const int e = lds_index<R>(q);
            s[e] = cscale(cmul(s[e], phasor_rev<R>(rho)), amp);
        }
    } else if (flags & B_GDD) {
        const bool on = (d.gdd_mask >> f) & 1;
        const R amp = static_cast<R>(inv_nt);
        for (int q = threadIdx.x; q < npts; q += kThreads) {
            const int e = lds_index<R>(q);
            if (on) {
                const int r = q >> log2n1, k1 = q & (n1 - 1);
                const int k = (r0 + r) + n2 * k1;
                const double ks = static_cast<double>(k < (nt >> 1) ? k : k - nt);
                s[e] = cscale(cmul(s[e], phasor_rev<R>(d.gdd_rev * ks * ks)), amp);
            } else {
                s[e] = cscale(s[e], amp);
            }
        }
    }
    __syncthreads();
    tile_fft<R, +1>(s, rows, log2n1, a.tw);

    const V *t4 = a.tw4 + d.tw4_off;
    for (int q = threadIdx.x; q < npts; q += kThreads) {
        const int r = q >> log2n1, j1 = q & (n1 - 1);
        const unsigned m = (static_cast<unsigned>(j1) * static_cast<unsigned>(r0 + r)) & (nt - 1);
        g[q] = cmulc(s[lds_index<R>(q)], twiddle4<R>(t4, d.tw4_bits, m));
    }
}

// ------------------------------------------------------------------------
// Per-instance energies of one round trip from the column-tile partial sums,
// summed in tile order (deterministic), into history row `*counter`.
__global__ __launch_bounds__(kThreads) void energy_reduce(const InstDesc *inst, int n_inst,
                                                          const double *partial, double *hist,
                                                          int *counter, int capacity)
{
    const int slot = *counter;
    for (int ii = threadIdx.x; ii < n_inst; ii += kThreads) {
        const InstDesc &d = inst[ii];
        double e[3] = {0.0, 0.0, 0.0};
        for (int t = 0; t < d.tiles_a; ++t)
            for (int x = 0; x < 3; ++x)
                e[x] += partial[(d.tile_a0 + t) * 3 + x];
        if (slot < capacity)
            for (int x = 0; x < 3; ++x)
                hist[(static_cast<long long>(slot) * n_inst + ii) * 3 + x] = e[x];
    }
    __syncthreads();
    if (threadIdx.x == 0) *counter = slot + 1;
}

__global__ void set_counter(int *counter, int v)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *counter = v;
}

} // namespace opo
