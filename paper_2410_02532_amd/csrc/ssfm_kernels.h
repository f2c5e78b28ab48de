// ssfm_kernels.h -- gfx950 kernels of one symmetrized split-step Fourier step
// (arXiv 2410.02532, Sec. 2.2, Eqs. 10-11) and of the cavity round trip
// (Eq. 6, Sec. 2.3, Sec. 4.1), for a batch of OPO instances of uneven size.
//
// Each field of nt = n1*n2 samples is transformed with a four-step FFT: the
// column pass does n2-point transforms down the columns j1 (stride n1), the
// row pass n1-point transforms along the contiguous rows, and the twiddle
// W_nt^{j1 k2} is applied on both sides of the row pass by the column pass.
// A z-step therefore touches HBM twice:
//
//   column pass  [x conj twiddle, inverse column FFT] -> [RK4 half-step of
//                the previous step] -> [round-trip boundary] -> [RK4
//                half-step of this step] -> [forward column FFT, x twiddle]
//   row pass     forward row FFT -> linear propagator / nt -> inverse row FFT
//
// The RK4 half-steps (Eqs. 2-4 without the linear operator) are pointwise in
// time and need the fields of a sample together, so a column tile holds COLS
// adjacent columns of every field (COLS*8 B = 128 B per row, one cache line);
// the linear propagator (Eq. 5) is pointwise in frequency and per field, so a
// row tile holds whole rows of one field. An instance couples three waves
// (pump, signal, idler) or, at degeneracy, two (pump and signal, with the
// signal equation of the paper's degenerate case and the pump coefficient
// 2 pi d_eff/(n_p lambda_s) that conserves n_p|A_p|^2 + n_s|A_s|^2). Both kernels keep
// every sample in registers from load to store (fft_tile.h) and are
// specialized at compile time for the transform length; the host groups the
// tiles of a batch by that length and launches each group.
//
// Phase arguments (dispersion, dk z, GDD, EOM) are formed and reduced modulo
// one revolution in FP64 and turned into phasors in FP64; in the FP32 path
// every unit-modulus factor (twiddles, propagator, mirror, GDD, EOM) is then
// applied as a compensated hi + lo pair (fft_tile.h, Phasor).
#pragma once
#include "fft_tile.h"

namespace opo {

// Per-instance description, built on the host and read by every tile.
struct InstDesc {
    long long off;        // element offset of the pump field; signal +nt, idler +2nt
    long long pump_off;   // element offset of the input-pump samples, -1 = constant pump
    long long disp_off;   // offset of the instance's linear-propagator table (nf nt entries)
    long long w4_off;     // offset of the four-step twiddle table W_nt^{j1 k2} at k2 * n1 + j1
    int nt, log2nt;
    int n1, log2n1;       // row length (contiguous)
    int n2, log2n2;       // column length (stride n1)
    int cols;             // columns per column tile
    int rows;             // rows per row tile
    int tile_a0, tiles_a; // first column tile of the instance, and count
    int tile_b0, tiles_b; // first row tile, and count (nf fields x row blocks)
    int res_mask, gdd_mask, eom_mask;
    int nf;               // coupled waves: 3 (p, s, i) or 2 (p, s; degenerate)
    int pump_windows;     // > 1: round trip m reads window m of the input pump (zero after)
    int kerr;             // Kerr term on (gamma below)
    int resident;         // fixed-step passes run in resident_pass (one workgroup holds
                          // the instance); its propagator table is then in natural bin order
    double length_mm;
    double kappa[3];      // 1/mm per V/m; two waves: (kappa_p2, kappa_s, 0)
    double dk_rev;        // dk / (2 pi)  [rev/mm]
    double disp[3][3];    // dispersion phase [rev/mm] = c0 ks + c1 ks^2 + c2 ks^3 per field
    double alpha_half[3]; // alpha_x / 2
    double mirror[3][2];  // sqrt(R_x) e^{i delta_x}
    double gdd_rev;       // GDD phase [rev] = gdd_rev * ks^2
    double eom_beta;      // EOM phase = beta sin(2 pi rho_j), rho_j = eom_rev0 + eom_rev_step j
    double eom_rev0, eom_rev_step;
    double pump_cw[2];
    double inject;        // resonant pump: input coupled in per round trip, sqrt(1 - R_p)
    double gamma[3];      // Kerr coefficients [1/mm per (V/m)^2]
};

enum : int {
    A_INV = 1,        // start with the inverse column FFT (data left by a row pass)
    A_RK_PREV = 2,    // second half-step of the previous z-step
    A_ENERGY = 4,     // FP64 partial sums of |A_x|^2 after the pass
    A_MIRROR = 8,     // sqrt(R) e^{i delta} on resonant fields (Eq. 6)
    A_EOM = 16,       // EOM phase on the selected fields (Sec. 2.3)
    A_REFRESH = 32,   // input pump into a non-resonant pump, zero non-resonant s/i
                      // (also: record the fields leaving the crystal with A_ENERGY)
    A_RK_THIS = 64,   // first half-step of this z-step
    A_FWD = 128,      // end with the forward column FFT + twiddle (else store samples)
    A_GDD = 256,      // resident passes: GDD between the energies and the mirror
};

enum : int {
    B_DISP = 1,       // multiply by the linear propagator of a step dz (Eq. 5)
    B_GDD = 2,        // multiply the GDD fields by e^{i gamma w^2/2} (Sec. 2.3)
    B_FWD_ONLY = 4,   // forward row FFT only (spectrum read-out)
};

// Step control of one instance under the adaptive step (local-error method,
// the step-size scheme of the literature the paper points to), FP64.
struct AdaptState {
    double z;            // position reached by the accepted steps
    double end;          // where the propagation ends
    double dz;           // step of the next attempt (already cut at the end)
    double tol;          // error tolerance of the run
    int max_attempts;    // attempt budget of the run (accepted + rejected)
    int status;          // 0 running, 1 reached the end, 2 attempt budget spent
    int last;            // the next attempt ends at `end`
    int pend;            // the last attempt was kept: the coarse and fine
                         // buffers hold a step still to be extrapolated
    int accepted, rejected;
};

template <typename R> struct StepArgs {
    const InstDesc *inst;
    const int *tile_inst;     // tile -> instance
    int inst_only;            // 1 + the instance of every tile of the launch, or 0 (tiles
                              // of several instances: look each up in tile_inst)
    cplx<R> *state;
    const cplx<R> *pump;
    const Phasor<R> *tw;      // butterfly twiddles e^{-2 pi i q/kTwL}
    const Phasor<R> *w4tab;   // four-step twiddles W_nt^{j1 k2} per (nt, n1), from FP64
    const Phasor<R> *disp;    // linear-propagator tables H_x(k)/nt in row-pass order
    double *partial;          // [column tiles][3] energy partial sums
    // [0] energy-history slot, [1] round trips completed, [2] stop: a round
    // trip had non-finite energies (every later tile of the call stores
    // nothing), [3] a boundary launch stored a non-finite value
    int *counter;
    cplx<R> *snap;            // round trips: A_REFRESH tiles first copy the fields
                              // they load here (the state the round trip starts from)
    cplx<R> *record;          // per-round-trip record of the fields leaving the crystal, or null
    long long record_stride;  // elements per record slot (the whole state)
    int record_cap;           // record slots
    int tile0;                // first tile of this launch (tiles are grouped by shape)
    int tile_count;           // tiles of this launch
    const int *block_map;     // mixed launches: workgroup -> tile (see mixed_pass)
    int flags;
    int nz;                   // steps per pass (dz = L/nz when dz_arg <= 0)
    int disp_sel;             // row pass: propagator table of this step size (0 or 1)
    double dz_arg;            // explicit step, or <= 0
    double zbase;             // z of step 0
    // RK4 half-steps of a column launch, in units of the instance's dz: the
    // second half of the previous step starts at zf_prev with size hf_prev,
    // the first half of this step at zf_this with size hf_this (z from zbase)
    double zf_prev, hf_prev, zf_this, hf_this;
    // adaptive step: per-instance z and dz (instances not running skip their
    // tiles), the launch's step is adapt_scale * dz, the propagator table of
    // dz/2 is per instance at off (a row pass of dz applies it twice), and a
    // column launch may load its fields from src instead of state
    const AdaptState *adapt;
    double adapt_scale;
    const cplx<R> *src;
};

// Element q of the array at base, q formed in 32 bits (below 2^28 within one
// instance's arrays): the address is a uniform 64-bit base plus a 32-bit
// per-lane byte offset, which the loads and stores take directly.
template <typename T> __device__ __forceinline__ T &el32(T *base, unsigned q)
{
    using B = typename std::conditional<std::is_const<T>::value, const char, char>::type;
    return *reinterpret_cast<T *>(reinterpret_cast<B *>(base) + q * static_cast<unsigned>(sizeof(T)));
}

// ---------------------------------------------------------------- shapes --
// Column tile for columns of length 2^ln2: PF samples per thread and field,
// COLS columns so that COLS * sizeof(complex) = 128 B (one cache line), and
// at most 8 samples per thread and field (the 256-point FP32 columns then
// take 8 columns, 64 B: 16 samples of three fields held the registers of
// two waves per SIMD and ran at half the speed).
template <typename R> __host__ __device__ constexpr int col_pf(int ln2)
{
    const int n = 1 << ln2;
    const int cmin = 128 / (2 * static_cast<int>(sizeof(R)));
    const int pfmax = 8;
    if (n == 1) return 1;
    int pf = cmin * n / kThreads;
    pf = pf < 2 ? 2 : pf;
    return pf > pfmax ? pfmax : pf;
}
template <typename R> __host__ __device__ constexpr int col_cols(int ln2)
{
    return kThreads * col_pf<R>(ln2) >> ln2;
}
// LDS layout of a column tile: position p of column c of field f at element
// f*ROW*n2 + p*ROW + c with ROW = COLS + OPO_COL_PAD, so that every offset
// between a thread's positions is a compile-time constant.
#ifndef OPO_COL_PAD
#define OPO_COL_PAD 1
#endif
template <typename R> __host__ __device__ constexpr int col_lds_row(int ln2) { return col_cols<R>(ln2) + OPO_COL_PAD; }
// Column tiles whose fields would need more than 32 KB of LDS for one
// exchange pass their fields through it one at a time (a single field's
// worth of LDS), so that several workgroups still fit a CU.
template <typename R> __host__ __device__ constexpr bool col_seq_lds(int ln2)
{
    return 3LL * col_cols<R>(ln2) * (1LL << ln2) * 2 * static_cast<long long>(sizeof(R)) > 32768;
}

// Row tile for rows of length 2^ln1: PF samples per thread, at least 16
// threads (128 B) along a row, ROWS rows per tile. FP32 rows of 4096 points
// take 16 samples (radix-16 stages, one row per workgroup). Rows of 1024 and
// 2048 points take 8: with 16 their radix-16 stages held the mixed kernel at
// 128 VGPRs (four workgroups per CU, one register spilled); with 8 it needs 95
// and five fit, and the batched sweep runs 6 % faster (3.42e10 -> 3.63e10;
// a batch of 2^16 instances alone 4 % slower, 3.24e10 -> 3.10e10). (At 256
// points the tiles of four times the rows halve the workgroups of a single
// instance, whose launches are then too few to fill the chip; in FP64 the
// registers are better spent on occupancy.)
#ifndef OPO_ROW_WAVE_MAX
#define OPO_ROW_WAVE_MAX 64
#endif
#ifndef OPO_ROW_R16_MIN
#define OPO_ROW_R16_MIN 4096
#endif
template <typename R> __host__ __device__ constexpr int row_pf(int ln1)
{
    const int n = 1 << ln1;
    if (n == 1) return 1;
    if (sizeof(R) == 4 && n >= OPO_ROW_R16_MIN) return n / 16 > kThreads ? n / kThreads : 16;
    int pf = n / 16;
    pf = pf < 2 ? 2 : pf;
    pf = pf > 8 ? 8 : pf;
    return n / pf > kThreads ? n / kThreads : pf;  // at most one row per workgroup
}
template <typename R> __host__ __device__ constexpr int row_rows(int ln1)
{
    return kThreads * row_pf<R>(ln1) >> ln1;
}
template <typename R> constexpr int kMaxLog2N1 = sizeof(R) == 4 ? 12 : 11;   // 256 threads per row
constexpr int kMaxLog2N2 = 8;

// e^{2 pi i rho} in FP64, rho reduced modulo one revolution first.
__device__ __forceinline__ double2 unit_rev(double rho)
{
    double sn, cs;
    sincospi(2.0 * (rho - rint(rho)), &sn, &cs);
    return make_double2(cs, sn);
}

// Coupling coefficients of the RK4 stages of the two half-steps a column tile
// runs, pre-scaled by h/2 (h = dz/2): (i kappa_p e^{-i dk z}, i kappa_s
// e^{+i dk z}, i kappa_i e^{+i dk z}) * h/2 at z0, z0 + h/2, z0 + h.
template <typename R> struct Coupling {
    cplx<R> c[2][3][3];   // [previous / this half-step][stage position][field]
    R g[2][3];            // Kerr coefficients gamma_x h/2 [previous / this half-step]
};

// Computed by six threads in FP64 and shared through LDS.
template <typename R>
__device__ __forceinline__ void coupling_tile(const InstDesc &d, double z_prev, double h_prev, double z_this,
                                              double h_this, Coupling<R> *out)
{
    using V = cplx<R>;
    const int q = threadIdx.x;
    if (q < 6) {
        const int which = q / 3, st = q - 3 * which;
        const double h = which ? h_this : h_prev;
        const double z = (which ? z_this : z_prev) + 0.5 * h * st;
        const double r = d.dk_rev * z;
        double sn, cs;
        sincospi(2.0 * (r - rint(r)), &sn, &cs);
        const double hh = 0.5 * h;
        const double kp = d.kappa[0] * hh, ks = d.kappa[1] * hh, ki = d.kappa[2] * hh;
        // i kappa e^{-i th} = kappa (sin th + i cos th); i kappa e^{+i th} = kappa (-sin th + i cos th)
        out->c[which][st][0] = mk<V>(static_cast<R>(kp * sn), static_cast<R>(kp * cs));
        out->c[which][st][1] = mk<V>(static_cast<R>(-ks * sn), static_cast<R>(ks * cs));
        out->c[which][st][2] = mk<V>(static_cast<R>(-ki * sn), static_cast<R>(ki * cs));
        out->g[which][st] = static_cast<R>(d.gamma[st] * hh);   // st doubles as the field index
    }
}

// Right-hand side of Eqs. 2-4 (nonlinear part) times h/2, with the stage's
// coupling coefficients k (i kappa e^{-+i dk z} h/2).
template <typename V>
__device__ __forceinline__ void cwe_rhs(const V (&k)[3], V ap, V as, V ai, V &fp, V &fs, V &fi)
{
    fp = cmul(k[0], cmul(as, ai));
    fs = cmul(k[1], cmulc(ap, ai));
    fi = cmul(k[2], cmulc(ap, as));
}

// y + i c t for a real c (one FMA per component).
template <typename V, typename S> __device__ __forceinline__ V add_ic(V y, S c, V t)
{
    return mk<V>(y.x - c * t.y, y.y + c * t.x);
}

// RK4 with dk = 0: every stage coefficient is the same i c_x (c_x = kappa_x h/2),
// so the stage slopes are i c_x t_n with t_n the bare products, and c_x moves
// into the FMAs that form the stage inputs and the final combination.
template <typename R>
__device__ __forceinline__ void rk4_point_imag(const cplx<R> (&c)[3][3], cplx<R> &ap, cplx<R> &as, cplx<R> &ai)
{
    using V = cplx<R>;
    const R cp = c[0][0].y, cs = c[0][1].y, ci = c[0][2].y;
    const R two = R(2), third = R(1) / R(3);
    const V p1 = cmul(as, ai), s1 = cmulc(ap, ai), i1 = cmulc(ap, as);
    V bp = add_ic(ap, cp, p1), bs = add_ic(as, cs, s1), bi = add_ic(ai, ci, i1);
    const V p2 = cmul(bs, bi), s2 = cmulc(bp, bi), i2 = cmulc(bp, bs);
    bp = add_ic(ap, cp, p2);
    bs = add_ic(as, cs, s2);
    bi = add_ic(ai, ci, i2);
    const V p3 = cmul(bs, bi), s3 = cmulc(bp, bi), i3 = cmulc(bp, bs);
    bp = add_ic(ap, two * cp, p3);
    bs = add_ic(as, two * cs, s3);
    bi = add_ic(ai, two * ci, i3);
    const V p4 = cmul(bs, bi), s4 = cmulc(bp, bi), i4 = cmulc(bp, bs);
    auto comb = [&](V t1, V t2, V t3, V t4) {
        return mk<V>(t1.x + two * (t2.x + t3.x) + t4.x, t1.y + two * (t2.y + t3.y) + t4.y);
    };
    ap = add_ic(ap, third * cp, comb(p1, p2, p3, p4));
    as = add_ic(as, third * cs, comb(s1, s2, s3, s4));
    ai = add_ic(ai, third * ci, comb(i1, i2, i3, i4));
}

// Classical coupled RK4 over one step h with stage coefficients at z0, z0+h/2,
// z0+h (each pre-scaled by h/2, so y + h/2 k_n becomes y + k'_n).
template <typename R>
__device__ __forceinline__ void rk4_point(const cplx<R> (&c)[3][3], cplx<R> &ap, cplx<R> &as,
                                          cplx<R> &ai)
{
    using V = cplx<R>;
    V p1, s1, i1, p2, s2, i2, p3, s3, i3, p4, s4, i4;
    cwe_rhs(c[0], ap, as, ai, p1, s1, i1);
    cwe_rhs(c[1], cadd(ap, p1), cadd(as, s1), cadd(ai, i1), p2, s2, i2);
    cwe_rhs(c[1], cadd(ap, p2), cadd(as, s2), cadd(ai, i2), p3, s3, i3);
    const R two = R(2);
    cwe_rhs(c[2], mk<V>(ap.x + two * p3.x, ap.y + two * p3.y), mk<V>(as.x + two * s3.x, as.y + two * s3.y),
                  mk<V>(ai.x + two * i3.x, ai.y + two * i3.y), p4, s4, i4);
    const R third = R(1) / R(3);
    ap = mk<V>(ap.x + third * (p1.x + two * (p2.x + p3.x) + p4.x),
               ap.y + third * (p1.y + two * (p2.y + p3.y) + p4.y));
    as = mk<V>(as.x + third * (s1.x + two * (s2.x + s3.x) + s4.x),
               as.y + third * (s1.y + two * (s2.y + s3.y) + s4.y));
    ai = mk<V>(ai.x + third * (i1.x + two * (i2.x + i3.x) + i4.x),
               ai.y + third * (i1.y + two * (i2.y + i3.y) + i4.y));
}

// The two-wave right-hand side times h/2: (i kappa_p2 A_s^2 e^{-i dk z},
// i kappa_s A_p A_s^* e^{+i dk z}) with the same stage coefficients.
template <typename V>
__device__ __forceinline__ void cwe2_rhs(const V (&k)[3], V ap, V as, V &fp, V &fs)
{
    fp = cmul(k[0], cmul(as, as));
    fs = cmul(k[1], cmulc(ap, as));
}

// Two-wave RK4 with dk = 0, factored like rk4_point_imag.
template <typename R>
__device__ __forceinline__ void rk4_point2_imag(const cplx<R> (&c)[3][3], cplx<R> &ap, cplx<R> &as)
{
    using V = cplx<R>;
    const R cp = c[0][0].y, cs = c[0][1].y;
    const R two = R(2), third = R(1) / R(3);
    const V p1 = cmul(as, as), s1 = cmulc(ap, as);
    V bp = add_ic(ap, cp, p1), bs = add_ic(as, cs, s1);
    const V p2 = cmul(bs, bs), s2 = cmulc(bp, bs);
    bp = add_ic(ap, cp, p2);
    bs = add_ic(as, cs, s2);
    const V p3 = cmul(bs, bs), s3 = cmulc(bp, bs);
    bp = add_ic(ap, two * cp, p3);
    bs = add_ic(as, two * cs, s3);
    const V p4 = cmul(bs, bs), s4 = cmulc(bp, bs);
    ap = add_ic(ap, third * cp,
                mk<V>(p1.x + two * (p2.x + p3.x) + p4.x, p1.y + two * (p2.y + p3.y) + p4.y));
    as = add_ic(as, third * cs,
                mk<V>(s1.x + two * (s2.x + s3.x) + s4.x, s1.y + two * (s2.y + s3.y) + s4.y));
}

template <typename R>
__device__ __forceinline__ void rk4_point2(const cplx<R> (&c)[3][3], cplx<R> &ap, cplx<R> &as)
{
    using V = cplx<R>;
    V p1, s1, p2, s2, p3, s3, p4, s4;
    cwe2_rhs(c[0], ap, as, p1, s1);
    cwe2_rhs(c[1], cadd(ap, p1), cadd(as, s1), p2, s2);
    cwe2_rhs(c[1], cadd(ap, p2), cadd(as, s2), p3, s3);
    const R two = R(2);
    cwe2_rhs(c[2], mk<V>(ap.x + two * p3.x, ap.y + two * p3.y), mk<V>(as.x + two * s3.x, as.y + two * s3.y),
                   p4, s4);
    const R third = R(1) / R(3);
    ap = mk<V>(ap.x + third * (p1.x + two * (p2.x + p3.x) + p4.x),
               ap.y + third * (p1.y + two * (p2.y + p3.y) + p4.y));
    as = mk<V>(as.x + third * (s1.x + two * (s2.x + s3.x) + s4.x),
               as.y + third * (s1.y + two * (s2.y + s3.y) + s4.y));
}

// Kerr terms times h/2 added to the stage slopes f: i g_x (|A_x|^2 + 2 sum_{y != x}
// |A_y|^2) A_x (self- and cross-phase modulation, the chi(3) extension of the
// nonlinear operator).
template <typename R, int NF>
__device__ __forceinline__ void kerr_add(const R (&g)[3], const cplx<R> (&y)[3], cplx<R> (&f)[3])
{
    R p[NF];
#pragma unroll
    for (int x = 0; x < NF; ++x) p[x] = y[x].x * y[x].x + y[x].y * y[x].y;
    R tot = R(0);
#pragma unroll
    for (int x = 0; x < NF; ++x) tot += p[x];
#pragma unroll
    for (int x = 0; x < NF; ++x) {
        const R w = g[x] * (R(2) * tot - p[x]);
        f[x].x -= w * y[x].y;
        f[x].y += w * y[x].x;
    }
}

// RK4 half-step with the Kerr terms (general coupling coefficients).
template <typename R, int NF>
__device__ __forceinline__ void rk4_kerr(const cplx<R> (&c)[3][3], const R (&g)[3], cplx<R> &y0, cplx<R> &y1,
                                         cplx<R> &y2)
{
    using V = cplx<R>;
    const V y[3] = {y0, y1, y2};
    V k[4][3], t[3];
    auto slope = [&](int st, const V (&in)[3], V (&out)[3]) {
        if constexpr (NF == 3) cwe_rhs(c[st], in[0], in[1], in[2], out[0], out[1], out[2]);
        else {
            cwe2_rhs(c[st], in[0], in[1], out[0], out[1]);
            out[2] = mk<V>(R(0), R(0));
        }
        kerr_add<R, NF>(g, in, out);
    };
    const R two = R(2), third = R(1) / R(3);
    slope(0, y, k[0]);
#pragma unroll
    for (int x = 0; x < 3; ++x) t[x] = cadd(y[x], k[0][x]);
    slope(1, t, k[1]);
#pragma unroll
    for (int x = 0; x < 3; ++x) t[x] = cadd(y[x], k[1][x]);
    slope(1, t, k[2]);
#pragma unroll
    for (int x = 0; x < 3; ++x) t[x] = mk<V>(y[x].x + two * k[2][x].x, y[x].y + two * k[2][x].y);
    slope(2, t, k[3]);
    V r[3];
#pragma unroll
    for (int x = 0; x < 3; ++x)
        r[x] = mk<V>(y[x].x + third * (k[0][x].x + two * (k[1][x].x + k[2][x].x) + k[3][x].x),
                     y[x].y + third * (k[0][x].y + two * (k[1][x].y + k[2][x].y) + k[3][x].y));
    y0 = r[0];
    y1 = r[1];
    if constexpr (NF == 3) y2 = r[2];
}

// RK4 half-step of the NF coupled waves at one time point (y2 unused for two).
template <typename R, int NF>
__device__ __forceinline__ void rk4_fields(const Coupling<R> &cp, int which, bool imag, bool kerr, cplx<R> &y0,
                                           cplx<R> &y1, cplx<R> &y2)
{
    const cplx<R>(&c)[3][3] = cp.c[which];
    if (kerr) {
        rk4_kerr<R, NF>(c, cp.g[which], y0, y1, y2);
        return;
    }
    if constexpr (NF == 3) {
        if (imag) rk4_point_imag<R>(c, y0, y1, y2);
        else rk4_point<R>(c, y0, y1, y2);
    } else {
        if (imag) rk4_point2_imag<R>(c, y0, y1);
        else rk4_point2<R>(c, y0, y1);
    }
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

struct ColumnShared {
    double red[3 * kThreads / 64];
};

// ------------------------------------------------------------------------
// The column FFTs of the NF fields of a tile: all fields through LDS
// together, or one after another for the large columns (col_seq_lds).
template <typename R, int LN2, int PF, int NF, int DIR, int COLS>
__device__ __forceinline__ void column_fft(cplx<R> (&v)[NF][PF], cplx<R> *s, const int (&base)[NF], int t,
                                           const Phasor<R> *__restrict__ tw)
{
    constexpr int N = 1 << LN2;
    constexpr int ROW = col_lds_row<R>(LN2);
    if constexpr (N > 1 && col_seq_lds<R>(LN2)) {
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            cplx<R> w[1][PF];
#pragma unroll
            for (int m = 0; m < PF; ++m) w[0][m] = v[f][m];
            const int b1[1] = {base[0]};
            reg_fft<R, N, PF, 1, DIR, ROW, 2048, true>(w, s, b1, t, tw);
#pragma unroll
            for (int m = 0; m < PF; ++m) v[f][m] = w[0][m];
        }
    } else {
        reg_fft<R, N, PF, NF, DIR, ROW, 2048, true>(v, s, base, t, tw);
    }
}

// Column pass of one tile: COLS columns j1 = c0 + c of the NF fields.
// Thread (c, t) holds samples j2 (or k2) = t + m*T, m < PF, of column c.
template <typename R, int LN2, int NF>
__device__ __forceinline__ void column_tile(const StepArgs<R> &a, const InstDesc &d, int tile,
                                            cplx<R> *s, Coupling<R> *cpl, double *red)
{
    using V = cplx<R>;
    constexpr int N = 1 << LN2;
    constexpr int PF = col_pf<R>(LN2);
    constexpr int COLS = col_cols<R>(LN2);
    constexpr int T = N / PF;
    const int flags = a.flags;
    const int c = threadIdx.x % COLS, t = threadIdx.x / COLS;
    const int nt = d.nt, n1 = d.n1;
    const int j1 = (tile - d.tile_a0) * COLS + c;
    const bool act = j1 < n1;
    // a round trip of this call had non-finite energies: compute, store nothing
    // (the flag is first needed at the stores, so its load hides behind the field loads)
    const bool stopped = a.counter[2] != 0;
    // sample m of field f of this thread's column: q0 + m*cstep + f*nt from the
    // instance's first sample (uniform bases, 32-bit offsets)
    V *g = a.state + d.off;
    const V *gs = (a.src ? a.src : a.state) + d.off;
    const unsigned q0 = static_cast<unsigned>(j1 + n1 * t);
    const unsigned cstep = static_cast<unsigned>(n1 * T);

    double dz = a.dz_arg > 0.0 ? a.dz_arg : d.length_mm / a.nz;
    double zb = a.dz_arg > 0.0 ? a.zbase : 0.0;
    if (a.adapt) {
        const AdaptState &st = a.adapt[a.inst_only > 0 ? a.inst_only - 1 : a.tile_inst[tile]];
        dz = st.dz * a.adapt_scale;
        zb = st.z;
    }
    V v[NF][PF];
    // four-step twiddle W_nt^{j1 k2} of sample m, read from the table of this
    // (nt, n1) where it is used (before the inverse and after the forward
    // column FFT) rather than held in registers; the COLS columns of a row of
    // the table are adjacent, and the tables of a batch stay in L2
    const Phasor<R> *w4t = a.w4tab + d.w4_off;
    auto w4 = [&](int m) { return act ? el32(w4t, q0 + m * cstep) : make_phasor<R>(1.0, 0.0); };
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int m = 0; m < PF; ++m)
            v[f][m] = act ? el32(gs, q0 + m * cstep + f * nt) : mk<V>(R(0), R(0));
    // the state this round trip starts from (time samples: A_REFRESH never
    // follows an inverse transform), kept to restore after a non-finite one
    if ((flags & A_REFRESH) && a.snap != nullptr && act && !stopped) {
        V *sp = a.snap + d.off;
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
            for (int m = 0; m < PF; ++m)
                el32(sp, q0 + m * cstep + f * nt) = v[f][m];
    }

    // the FP64 phasors of the RK4 couplings, formed by six threads once the field
    // loads are in flight (their latency then covers it)
    if (flags & (A_RK_PREV | A_RK_THIS))
        coupling_tile<R>(d, zb + a.zf_prev * dz, a.hf_prev * dz, zb + a.zf_this * dz, a.hf_this * dz, cpl);

    int base[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f)
        base[f] = f * col_lds_row<R>(LN2) * N + c;
    if (flags & A_INV) {
        if constexpr (N > 1) {
#pragma unroll
            for (int m = 0; m < PF; ++m) {
                const Phasor<R> w = w4(m);
#pragma unroll
                for (int f = 0; f < NF; ++f) v[f][m] = pmul<true>(v[f][m], w);
            }
        }
        column_fft<R, LN2, PF, NF, +1, COLS>(v, s, base, t, a.tw);
    }
    if (flags & (A_RK_PREV | A_RK_THIS)) __syncthreads();   // couplings visible

    const V pcw = mk<V>(static_cast<R>(d.pump_cw[0]), static_cast<R>(d.pump_cw[1]));
    const bool imag = d.dk_rev == 0.0;   // couplings i kappa h/2 without a phase
    const bool kerr = d.kerr != 0;
    double en[3] = {0.0, 0.0, 0.0};
    // round trips completed: the window of a long input pump that the refresh
    // reads, and the record slot of the pass that A_ENERGY ends
    const int rt = (flags & (A_REFRESH | A_ENERGY)) ? a.counter[1] : 0;
    const bool rec = (flags & A_ENERGY) && a.record != nullptr && rt < a.record_cap && act && !stopped;
    bool nonfinite = false;              // a boundary value about to be stored is NaN or Inf
    V *rg = rec ? a.record + static_cast<long long>(rt) * a.record_stride + d.off : nullptr;
    long long pwin = 0;                  // offset of the input-pump window, -1 = past the last
    if (d.pump_windows > 1) pwin = rt < d.pump_windows ? static_cast<long long>(rt) * nt : -1;
#pragma unroll
    for (int m = 0; m < PF; ++m) {
        const unsigned j = q0 + m * cstep;   // time index of the sample
        V y0 = v[0][m], y1 = v[1][m], y2 = v[NF - 1][m];
        if (flags & A_RK_PREV) rk4_fields<R, NF>(*cpl, 0, imag, kerr, y0, y1, y2);
        if ((flags & A_ENERGY) && act) {
            en[0] += static_cast<double>(y0.x) * y0.x + static_cast<double>(y0.y) * y0.y;
            en[1] += static_cast<double>(y1.x) * y1.x + static_cast<double>(y1.y) * y1.y;
            if constexpr (NF == 3) en[2] += static_cast<double>(y2.x) * y2.x + static_cast<double>(y2.y) * y2.y;
        }
        if (rec) {
            el32(rg, j) = y0;
            el32(rg, j + nt) = y1;
            if constexpr (NF == 3) el32(rg, j + 2 * nt) = y2;
        }
        if (flags & A_MIRROR) {
            if (d.res_mask & 1) y0 = pmul(y0, make_phasor<R>(d.mirror[0][0], d.mirror[0][1]));
            if (d.res_mask & 2) y1 = pmul(y1, make_phasor<R>(d.mirror[1][0], d.mirror[1][1]));
            if (NF == 3 && (d.res_mask & 4)) y2 = pmul(y2, make_phasor<R>(d.mirror[2][0], d.mirror[2][1]));
        }
        if ((flags & A_EOM) && d.eom_mask) {
            // beta sin(2 pi f t_j), with f t_j reduced modulo one revolution in FP64
            const double th = d.eom_beta * unit_rev(d.eom_rev0 + d.eom_rev_step * static_cast<double>(j)).y;
            double sn, cs;
            sincos(th, &sn, &cs);
            const Phasor<R> e = make_phasor<R>(cs, sn);
            if (d.eom_mask & 1) y0 = pmul(y0, e);
            if (d.eom_mask & 2) y1 = pmul(y1, e);
            if (NF == 3 && (d.eom_mask & 4)) y2 = pmul(y2, e);
        }
        if (flags & A_REFRESH) {
            V pin = pcw;                 // input pump sample of this round trip
            if (d.pump_off >= 0) pin = (act && pwin >= 0) ? el32(a.pump + d.pump_off + pwin, j) : mk<V>(R(0), R(0));
            if (!(d.res_mask & 1)) y0 = pin;
            else if (d.inject != 0.0) y0 = cadd(y0, pmul(pin, make_phasor<R>(d.inject, 0.0)));
            if (!(d.res_mask & 2)) y1 = mk<V>(R(0), R(0));
            if (NF == 3 && !(d.res_mask & 4)) y2 = mk<V>(R(0), R(0));
        }
        if (flags & A_RK_THIS) rk4_fields<R, NF>(*cpl, 1, imag, kerr, y0, y1, y2);
        if (flags & A_MIRROR)
            nonfinite = nonfinite || !(isfinite(y0.x) && isfinite(y0.y) && isfinite(y1.x) && isfinite(y1.y) &&
                                       isfinite(y2.x) && isfinite(y2.y));
        v[0][m] = y0;
        v[1][m] = y1;
        if constexpr (NF == 3) v[2][m] = y2;
    }
    if (flags & A_ENERGY) {
        block_sum3(en, red);
        if (threadIdx.x == 0 && !stopped)
            for (int x = 0; x < 3; ++x)
                a.partial[tile * 3 + x] = en[x];
    }
    // the end of a round trip: energy_reduce treats a non-finite stored field like
    // a non-finite energy (benign race: every writer stores 1)
    if (nonfinite && act && !stopped) a.counter[3] = 1;

    if (flags & A_FWD) {
        column_fft<R, LN2, PF, NF, -1, COLS>(v, s, base, t, a.tw);
        if constexpr (N > 1) {
#pragma unroll
            for (int m = 0; m < PF; ++m) {
                const Phasor<R> w = w4(m);
#pragma unroll
                for (int f = 0; f < NF; ++f) v[f][m] = pmul(v[f][m], w);
            }
        }
    }
    if (act && !stopped) {
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
            for (int m = 0; m < PF; ++m)
                el32(g, q0 + m * cstep + f * nt) = v[f][m];
    }
}

template <typename R, int L, int HI, int NF>
__device__ __forceinline__ void column_dispatch(const StepArgs<R> &a, const InstDesc &d, int tile, cplx<R> *s,
                                                Coupling<R> *cpl, double *red)
{
    if (d.log2n2 == L) column_tile<R, L, NF>(a, d, tile, s, cpl, red);
    else if constexpr (L < HI) column_dispatch<R, L + 1, HI, NF>(a, d, tile, s, cpl, red);
}

// Column pass over the tiles of NF-wave instances whose log2 n2 lies in [LO, HI].
template <typename R, int LO, int HI, int NF>
__global__ __launch_bounds__(kThreads) void column_pass(StepArgs<R> a)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    __shared__ Coupling<R> cpl;
    __shared__ double red[3 * kThreads / 64];
    const int tile = a.tile0 + blockIdx.x;
    // a launch over one instance skips the dependent load of the tile's instance
    const int ii = a.inst_only > 0 ? a.inst_only - 1 : a.tile_inst[tile];
    if (a.adapt && a.adapt[ii].status != 0) return;
    column_dispatch<R, LO, HI, NF>(a, a.inst[ii], tile, reinterpret_cast<cplx<R> *>(lds_raw), &cpl, red);
}

// ------------------------------------------------------------------------
// Row pass of one tile: rows k2 = r0 + w of one field. Thread (w, t) holds
// samples j1 (or k1) = t + m*T, m < PF, of row w.
// PRE: read the propagator into registers before the forward transform, so that
// its load latency hides behind the transform instead of following it. It costs
// 4 PF registers, which the standalone row pass of a launch too small to hide
// latency can spare (one 2^14 instance 5 % faster, a 2^18 one 10 %) and the mixed
// kernel, bound by its occupancy, cannot (the batched sweep 4 % slower).
template <typename R, int LN1, bool PRE>
__device__ __forceinline__ void row_tile(const StepArgs<R> &a, const InstDesc &d, int tile, cplx<R> *s)
{
    using V = cplx<R>;
    constexpr int N = 1 << LN1;
    constexpr int PF = row_pf<R>(LN1);
    constexpr int ROWS = row_rows<R>(LN1);
    constexpr int T = N / PF;
    const int flags = a.flags;
    const int w = threadIdx.x / T, t = threadIdx.x % T;
    const int nt = d.nt, n2 = d.n2;
    const int blocks = (n2 + ROWS - 1) / ROWS;
    const int local = tile - d.tile_b0;
    const int f = local / blocks;
    const int k2 = (local - f * blocks) * ROWS + w;
    const bool act = k2 < n2;
    const bool stopped = a.counter[2] != 0;   // see column_tile
    V *g = a.state + d.off + static_cast<long long>(f) * nt + static_cast<long long>(N) * k2 + t;

    V v[1][PF];
#pragma unroll
    for (int m = 0; m < PF; ++m)
        v[0][m] = act ? g[m * T] : mk<V>(R(0), R(0));
    // H_f(k)/nt from the instance's table, laid out like the rows
    const long long toff = a.adapt ? d.off : d.disp_off;
    const Phasor<R> *h = a.disp + toff + static_cast<long long>(a.disp_sel * d.nf + f) * nt +
                         static_cast<long long>(N) * k2 + t;
    Phasor<R> hr[PRE ? PF : 1];
    const bool pre = PRE && (flags & B_DISP) && !(flags & B_FWD_ONLY) && !a.adapt;
    if constexpr (PRE) {
        if (pre) {
#pragma unroll
            for (int m = 0; m < PF; ++m) hr[m] = act ? h[m * T] : make_phasor<R>(1.0, 0.0);
        }
    }
    const int base[1] = {w * N};
    // a row of at most 64 threads lies within one wavefront (rows start at
    // multiples of T), and rows occupy disjoint LDS
    constexpr bool WAVE = T <= OPO_ROW_WAVE_MAX;
    reg_fft<R, N, PF, 1, -1, 1, 2048, false, WAVE>(v, s, base, t, a.tw);

    if (!(flags & B_FWD_ONLY)) {
        if (pre) {
#pragma unroll
            for (int m = 0; m < PF; ++m)
                if (act) v[0][m] = pmul(v[0][m], hr[PRE ? m : 0]);
        } else if (flags & B_DISP) {
#pragma unroll
            for (int m = 0; m < PF; ++m)
                if (act) v[0][m] = pmul(v[0][m], h[m * T]);
            if (a.adapt && a.adapt_scale == 1.0) {   // adaptive coarse step: H(dz)/nt = (H(dz/2)/nt)^2 nt
                const R scale = static_cast<R>(nt);      // a power of two: exact
#pragma unroll
                for (int m = 0; m < PF; ++m)
                    if (act) v[0][m] = cscale(pmul(v[0][m], h[m * T]), scale);
            }
        } else if (flags & B_GDD) {
            const double inv_nt = 1.0 / nt;
            if ((d.gdd_mask >> f) & 1) {
#pragma unroll
                for (int m = 0; m < PF; ++m) {
                    const int k = k2 + n2 * (t + m * T);
                    const double ks = static_cast<double>(k < (nt >> 1) ? k : k - nt);
                    const double2 e = unit_rev(d.gdd_rev * ks * ks);
                    v[0][m] = pmul(v[0][m], make_phasor<R>(e.x * inv_nt, e.y * inv_nt));
                }
            } else {
#pragma unroll
                for (int m = 0; m < PF; ++m)
                    v[0][m] = cscale(v[0][m], static_cast<R>(inv_nt));
            }
        }
        reg_fft<R, N, PF, 1, +1, 1, 2048, false, WAVE>(v, s, base, t, a.tw);
    }
    if (act && !stopped)
#pragma unroll
        for (int m = 0; m < PF; ++m)
            g[m * T] = v[0][m];
}

template <typename R, int L, int HI, bool PRE>
__device__ __forceinline__ void row_dispatch(const StepArgs<R> &a, const InstDesc &d, int tile, cplx<R> *s)
{
    if (d.log2n1 == L) row_tile<R, L, PRE>(a, d, tile, s);
    else if constexpr (L < HI) row_dispatch<R, L + 1, HI, PRE>(a, d, tile, s);
}

// Row pass over the tiles of instances whose log2 n1 lies in [LO, HI].
template <typename R, int LO, int HI>
__global__ __launch_bounds__(kThreads) void row_pass(StepArgs<R> a)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int tile = a.tile0 + blockIdx.x;
    const int ii = a.inst_only > 0 ? a.inst_only - 1 : a.tile_inst[tile];   // as in column_pass
    if (a.adapt && a.adapt[ii].status != 0) return;
    row_dispatch<R, LO, HI, true>(a, a.inst[ii], tile, reinterpret_cast<cplx<R> *>(lds_raw));
}

// Size ranges served by one launch: shapes of similar register use share a
// kernel (the workgroups of different sizes then overlap on the GPU).
constexpr int kColRanges[][2] = {{0, 6}, {7, 7}, {8, 8}};
constexpr int kRowRanges[][2] = {{0, 5}, {6, 11}, {12, 12}};

// ------------------------------------------------------------------------
// Mixed pass: the column tiles of one half of a batch and the row tiles of
// the other half in one launch. The halves are a launch apart in their z-step
// sequences, so every launch pairs the VALU-bound column work of one half
// with the memory-latency-bound row work of the other. The host orders the
// workgroups so that every CU gets both kinds, and so that row tile t of
// every instance runs on XCD t mod 8 (workgroups are dealt to the eight XCDs
// round robin): each XCD's L2 then holds one eighth of a shared propagator
// table instead of all of it.
// Workgroups per CU the mixed kernel is compiled for: at least four (at most
// 128 VGPRs) for FP32 columns of up to 64 points, else whatever the registers
// allow. (The kernel for columns of up to 64 points and rows of up to 2048
// now needs 95 VGPRs; asking for five changes nothing.)
#ifndef OPO_MIXED_MIN_BLOCKS
#define OPO_MIXED_MIN_BLOCKS 4
#endif
template <typename R, int CR, int RR> constexpr int mixed_min_blocks()
{
    return sizeof(R) == 4 && CR == 0 && RR <= 1 ? OPO_MIXED_MIN_BLOCKS : 1;
}

constexpr int kNoTile = -2147483647 - 1;

template <typename R, int CR, int RR, int NF>
__global__ __launch_bounds__(kThreads, (mixed_min_blocks<R, CR, RR>())) void mixed_pass(StepArgs<R> ac,
                                                                                        StepArgs<R> ar)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    __shared__ Coupling<R> cpl;
    __shared__ double red[3 * kThreads / 64];
    cplx<R> *s = reinterpret_cast<cplx<R> *>(lds_raw);
    // block -> tile map built on the host: >= 0 a column tile, < 0 row tile -1-code
    const int code = ac.block_map[blockIdx.x];
    if (code == kNoTile) return;
    if (code >= 0) {
        column_dispatch<R, kColRanges[CR][0], kColRanges[CR][1], NF>(ac, ac.inst[ac.tile_inst[code]], code, s, &cpl,
                                                                 red);
    } else {
        const int tile = -1 - code;
        row_dispatch<R, kRowRanges[RR][0], kRowRanges[RR][1], false>(ar, ar.inst[ar.tile_inst[tile]], tile, s);
    }
}

// ------------------------------------------------------------------------
// Resident pass: one workgroup holds one instance of nt = 2^LN points for a
// whole crystal pass, and in a round trip also the boundary on both sides, so
// the fields cross HBM once per pass instead of twice per z-step. Thread t
// keeps samples t + m*T (m < PF, T = nt/PF) of every field in registers: the
// RK4 half-steps find the NF fields of a time point in one thread, and the
// full-length transforms of one field at a time (Stockham stages with LDS
// exchanges, fft_tile.h) return the bins in natural order to the same
// positions, where the natural-order propagator table H_x(k)/nt applies.
// Shapes: FP32 nt 2^10..2^12 and FP64 2^10..2^11. Samples per thread and
// field (res_pf): 8 (radix-8 stages; FP64 2^10: 4), so that an instance runs
// on nt/8 threads, two waves per SIMD at 2^12, with the fields, a stage's
// twiddles and the RK4 in registers without spills. With 16 samples (radix
// 16, half the threads, one wave per SIMD) the launches waited on latency: a
// batch of 2^12 instances ran at 3.8e10 field-point-steps/s against 5.6e10
// with 8. With 4, FP32 2^12 (1024 threads, four waves per SIMD) spills and
// 2^10..2^11 gain alone but slow a mix of sizes down (more waves beside the
// 2^12 instances); FP64 2^10 gains 5 %. FP32 2^13 spills with 512 threads of
// 16 samples and with 1024 of 8.
constexpr int kResMinLog2 = 10;
template <typename R> constexpr int kResMaxLog2 = sizeof(R) == 4 ? 12 : 11;
template <typename R, int LN> __host__ __device__ constexpr int res_pf()
{
    return (sizeof(R) == 8 && LN <= 10) ? 4 : 8;
}
template <typename R, int LN> __host__ __device__ constexpr int res_threads() { return (1 << LN) / res_pf<R, LN>(); }

// Fixed-order sum of three doubles over the W waves of a workgroup; the result
// is valid in thread 0.
template <int W> __device__ __forceinline__ void block_sum3_w(double v[3], double *scratch /* [3*W] */)
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
            scratch[x * W + wave] = v[x];
    __syncthreads();
    if (threadIdx.x == 0)
        for (int x = 0; x < 3; ++x) {
            double s = 0.0;
            for (int w = 0; w < W; ++w)
                s += scratch[x * W + w];
            v[x] = s;
        }
}

// The workgroups of a launch run the instances a.tile_inst[a.tile0 + b]. The
// flags select, as in the column tile: A_REFRESH (snapshot, input pump, zero
// non-resonant fields) before the pass; A_ENERGY (FP64 energies into the
// instance's first column-tile partial slot, the others zeroed, and the
// record), A_GDD, A_MIRROR and A_EOM after it. Without them the launch is a
// plain pass of nz steps from zbase (explicit dz_arg) or from 0 (L/nz).
// The table pointer, hidden from the optimizer: loads through it stay in the
// z-step loop instead of being hoisted out of it and held in registers for the
// whole pass (the tables are the same at every step).
template <typename P> __device__ __forceinline__ P *step_local(P *p)
{
    asm volatile("" : "+v"(p));
    return p;
}

template <typename R, int LN, int NF>
__global__ __launch_bounds__((res_threads<R, LN>())) void resident_pass(StepArgs<R> a)
{
    using V = cplx<R>;
    constexpr int N = 1 << LN, PF = res_pf<R, LN>(), T = N / PF, W = T / 64;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    __shared__ Coupling<R> cpl;
    __shared__ double red[3 * W];
    V *s = reinterpret_cast<V *>(lds_raw);
    const int ii = a.tile_inst[a.tile0 + blockIdx.x];
    const InstDesc &d = a.inst[ii];
    const int t = threadIdx.x;
    const int flags = a.flags;
    const bool stopped = a.counter[2] != 0;   // see column_tile
    V *g = a.state + d.off + t;

    V v[NF][PF];
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int m = 0; m < PF; ++m)
            v[f][m] = g[f * N + m * T];

    const int rt = (flags & (A_REFRESH | A_ENERGY)) ? a.counter[1] : 0;
    if (flags & A_REFRESH) {
        if (a.snap != nullptr && !stopped) {
            V *sp = a.snap + d.off + t;
#pragma unroll
            for (int f = 0; f < NF; ++f)
#pragma unroll
                for (int m = 0; m < PF; ++m)
                    sp[f * N + m * T] = v[f][m];
        }
        long long pwin = 0;
        if (d.pump_windows > 1) pwin = rt < d.pump_windows ? static_cast<long long>(rt) * N : -1;
        const V pcw = mk<V>(static_cast<R>(d.pump_cw[0]), static_cast<R>(d.pump_cw[1]));
#pragma unroll
        for (int m = 0; m < PF; ++m) {
            V pin = pcw;
            if (d.pump_off >= 0) pin = pwin >= 0 ? a.pump[d.pump_off + pwin + t + m * T] : mk<V>(R(0), R(0));
            if (!(d.res_mask & 1)) v[0][m] = pin;
            else if (d.inject != 0.0) v[0][m] = cadd(v[0][m], pmul(pin, make_phasor<R>(d.inject, 0.0)));
            if (!(d.res_mask & 2)) v[1][m] = mk<V>(R(0), R(0));
            if (NF == 3 && !(d.res_mask & 4)) v[NF - 1][m] = mk<V>(R(0), R(0));
        }
    }

    const double dz = a.dz_arg > 0.0 ? a.dz_arg : d.length_mm / a.nz;
    const double zb = a.dz_arg > 0.0 ? a.zbase : 0.0;
    const bool imag = d.dk_rev == 0.0;   // couplings without a phase: the same at every step
    const bool kerr = d.kerr != 0;
    const Phasor<R> *H = a.disp + d.disp_off + t;
    for (int j = 0; j < a.nz; ++j) {
        // couplings of step j: [1] its first half from z_j, [0] its second half from z_j + dz/2
        if (j == 0 || !imag) {
            __syncthreads();                 // the previous step's readers are done
            coupling_tile<R>(d, zb + (static_cast<double>(j) + 0.5) * dz, 0.5 * dz,
                             zb + static_cast<double>(j) * dz, 0.5 * dz, &cpl);
            __syncthreads();
        }
#pragma unroll
        for (int m = 0; m < PF; ++m)
            rk4_fields<R, NF>(cpl, 1, imag, kerr, v[0][m], v[1][m], v[NF - 1][m]);
        reg_fft_seq<R, N, PF, NF, -1, N>(v, s, t, step_local(a.tw));
        const Phasor<R> *Hj = step_local(H);
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
            for (int m = 0; m < PF; ++m) v[f][m] = pmul(v[f][m], Hj[f * N + m * T]);
        reg_fft_seq<R, N, PF, NF, +1, N>(v, s, t, step_local(a.tw));
#pragma unroll
        for (int m = 0; m < PF; ++m)
            rk4_fields<R, NF>(cpl, 0, imag, kerr, v[0][m], v[1][m], v[NF - 1][m]);
    }

    if (flags & A_ENERGY) {
        double en[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int m = 0; m < PF; ++m)
#pragma unroll
            for (int f = 0; f < NF; ++f)
                en[f] += static_cast<double>(v[f][m].x) * v[f][m].x + static_cast<double>(v[f][m].y) * v[f][m].y;
        if (a.record != nullptr && rt < a.record_cap && !stopped) {
            V *rg = a.record + static_cast<long long>(rt) * a.record_stride + d.off + t;
#pragma unroll
            for (int f = 0; f < NF; ++f)
#pragma unroll
                for (int m = 0; m < PF; ++m)
                    rg[f * N + m * T] = v[f][m];
        }
        block_sum3_w<W>(en, red);
        // the instance's column-tile slots of the partial sums (energy_reduce adds them)
        if (!stopped)
            for (int q = t; q < d.tiles_a; q += T)
                for (int x = 0; x < 3; ++x)
                    a.partial[(d.tile_a0 + q) * 3 + x] = q == 0 ? en[x] : 0.0;
    }
    if ((flags & A_GDD) && d.gdd_mask) {
        const double inv_nt = 1.0 / N;
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            if (!((d.gdd_mask >> f) & 1)) continue;
            V w[1][PF];
#pragma unroll
            for (int m = 0; m < PF; ++m) w[0][m] = v[f][m];
            reg_fft_seq<R, N, PF, 1, -1, N>(w, s, t, a.tw);
#pragma unroll
            for (int m = 0; m < PF; ++m) {
                const int k = t + m * T;
                const double ks = static_cast<double>(k < (N >> 1) ? k : k - N);
                const double2 e = unit_rev(d.gdd_rev * ks * ks);
                w[0][m] = pmul(w[0][m], make_phasor<R>(e.x * inv_nt, e.y * inv_nt));
            }
            reg_fft_seq<R, N, PF, 1, +1, N>(w, s, t, a.tw);
#pragma unroll
            for (int m = 0; m < PF; ++m) v[f][m] = w[0][m];
        }
    }
    bool nonfinite = false;
    if (flags & (A_MIRROR | A_EOM)) {
#pragma unroll
        for (int m = 0; m < PF; ++m) {
            V y0 = v[0][m], y1 = v[1][m], y2 = v[NF - 1][m];
            if (flags & A_MIRROR) {
                if (d.res_mask & 1) y0 = pmul(y0, make_phasor<R>(d.mirror[0][0], d.mirror[0][1]));
                if (d.res_mask & 2) y1 = pmul(y1, make_phasor<R>(d.mirror[1][0], d.mirror[1][1]));
                if (NF == 3 && (d.res_mask & 4)) y2 = pmul(y2, make_phasor<R>(d.mirror[2][0], d.mirror[2][1]));
            }
            if ((flags & A_EOM) && d.eom_mask) {
                const long long j = t + m * T;
                const double th = d.eom_beta * unit_rev(d.eom_rev0 + d.eom_rev_step * static_cast<double>(j)).y;
                double sn, cs;
                sincos(th, &sn, &cs);
                const Phasor<R> e = make_phasor<R>(cs, sn);
                if (d.eom_mask & 1) y0 = pmul(y0, e);
                if (d.eom_mask & 2) y1 = pmul(y1, e);
                if (NF == 3 && (d.eom_mask & 4)) y2 = pmul(y2, e);
            }
            if (flags & A_MIRROR)
                nonfinite = nonfinite || !(isfinite(y0.x) && isfinite(y0.y) && isfinite(y1.x) && isfinite(y1.y) &&
                                           isfinite(y2.x) && isfinite(y2.y));
            v[0][m] = y0;
            v[1][m] = y1;
            if constexpr (NF == 3) v[2][m] = y2;
        }
    }
    if (nonfinite && !stopped) a.counter[3] = 1;   // see column_tile
    if (!stopped) {
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
            for (int m = 0; m < PF; ++m)
                g[f * N + m * T] = v[f][m];
    }
}

// ------------------------------------------------------------------------
// Linear propagator of one z-step (Eq. 5) for the nf fields of an instance,
// H_x(k)/nt = exp{[-alpha_x/2 + i(-db1 w + b2 w^2/2 - b3 w^3/6)] dz}/nt,
// formed in FP64 (phase reduced modulo one revolution) and stored in the
// row-pass order (position k2*n1 + k1 holds bin k = k2 + n2*k1), or in natural
// bin order for the resident passes.
template <typename R>
__device__ __forceinline__ Phasor<R> propagator(const InstDesc &d, long long q, double dz, bool natural)
{
    const int f = static_cast<int>(q / d.nt);
    const int p = static_cast<int>(q - static_cast<long long>(f) * d.nt);
    const int k2 = p >> d.log2n1, k1 = p & (d.n1 - 1);
    const int k = natural ? p : k2 + d.n2 * k1;
    const double ks = static_cast<double>(k < (d.nt >> 1) ? k : k - d.nt);
    const double rho = dz * ks * (d.disp[f][0] + ks * (d.disp[f][1] + ks * d.disp[f][2]));
    const double amp = exp(-d.alpha_half[f] * dz) / d.nt;
    const double2 e = unit_rev(rho);
    return make_phasor<R>(amp * e.x, amp * e.y);
}

template <typename R>
__global__ __launch_bounds__(kThreads) void disp_table(const InstDesc *inst, int owner, Phasor<R> *out,
                                                       double dz, int sel)
{
    const InstDesc &d = inst[owner];
    out += static_cast<long long>(sel) * d.nf * d.nt;     // table of the sel-th step size
    const long long n = static_cast<long long>(d.nf) * d.nt;
    for (long long q = blockIdx.x * static_cast<long long>(kThreads) + threadIdx.x; q < n;
         q += static_cast<long long>(gridDim.x) * kThreads)
        out[d.disp_off + q] = propagator<R>(d, q, dz, d.resident != 0);
}

// ------------------------------------------------------------------------
// Adaptive step (local-error method). Every attempt of a running instance
// takes one symmetrized step of dz on a copy u_c and two of dz/2 on a copy
// u_f; d = ||u_f - u_c|| / ||u_f|| over all its fields decides: d > 2 tol
// rejects and halves dz; otherwise (4 u_f - u_c)/3 becomes the fields, z
// advances, and dz shrinks by 2^(1/3) when d > tol, grows by 2^(1/3) when
// d < tol/2. The kernels below run once per attempt around the step
// launches: begin, [coarse, fine passes], error, control. Each of begin and
// error covers instance b / chunks with `chunks` workgroups.
constexpr double kAdaptGrow = 1.25992104989487316477;   // 2^(1/3), the nearest double
constexpr double kAdaptSlack = 1.0 + 1e-9;   // a step that stops within 1e-9 dz of the end goes to it

// Fields of the attempt: the extrapolation of the step kept by the previous
// attempt (also for instances that have just stopped), and for a running
// instance its propagator table of dz/2. The first column launch of the
// coarse and of the fine step then loads u and stores into u_c or u_f.
template <typename R>
__global__ __launch_bounds__(kThreads) void adapt_begin(const InstDesc *inst, const AdaptState *ctl, int chunks,
                                                        cplx<R> *u, const cplx<R> *uc, const cplx<R> *uf,
                                                        Phasor<R> *tab)
{
    using V = cplx<R>;
    const int ii = blockIdx.x / chunks, ch = blockIdx.x - ii * chunks;
    const AdaptState st = ctl[ii];
    const bool run = st.status == 0;
    if (!run && !st.pend) return;
    const InstDesc &d = inst[ii];
    const long long n = static_cast<long long>(d.nf) * d.nt;
    for (long long q = ch * static_cast<long long>(kThreads) + threadIdx.x; q < n;
         q += static_cast<long long>(chunks) * kThreads) {
        const long long j = d.off + q;
        if (st.pend) {
            const V f = uf[j], c = uc[j];
            u[j] = mk<V>((R(4) * f.x - c.x) / R(3), (R(4) * f.y - c.y) / R(3));
        }
        if (run) tab[j] = propagator<R>(d, q, 0.5 * st.dz, false);   // the adaptive step runs column/row tiles
    }
}

// FP64 partial sums of |u_f - u_c|^2 and |u_f|^2 of each running instance.
template <typename R>
__global__ __launch_bounds__(kThreads) void adapt_error(const InstDesc *inst, const AdaptState *ctl, int chunks,
                                                        const cplx<R> *uc, const cplx<R> *uf, double *part)
{
    __shared__ double red[3 * kThreads / 64];
    const int ii = blockIdx.x / chunks, ch = blockIdx.x - ii * chunks;
    if (ctl[ii].status != 0) return;
    const InstDesc &d = inst[ii];
    const long long n = static_cast<long long>(d.nf) * d.nt;
    double v[3] = {0.0, 0.0, 0.0};
    for (long long q = ch * static_cast<long long>(kThreads) + threadIdx.x; q < n;
         q += static_cast<long long>(chunks) * kThreads) {
        const double fx = uf[d.off + q].x, fy = uf[d.off + q].y;
        const double ex = fx - static_cast<double>(uc[d.off + q].x), ey = fy - static_cast<double>(uc[d.off + q].y);
        v[0] += ex * ex + ey * ey;
        v[1] += fx * fx + fy * fy;
    }
    block_sum3(v, red);
    if (threadIdx.x == 0) {
        part[2 * static_cast<long long>(blockIdx.x)] = v[0];
        part[2 * static_cast<long long>(blockIdx.x) + 1] = v[1];
    }
}

// One wave per instance (lane 0 decides). mode 0 starts a run from z0 over
// `length` with step dz0; mode 1 takes the decision of the attempt just made.
// Both then prepare the next attempt: stop at the end or when the budget is
// spent, else cut a step that would pass the end.
__global__ __launch_bounds__(kThreads) void adapt_control(AdaptState *ctl, int n_inst, int chunks,
                                                          const double *part, int mode, double z0, double length,
                                                          double dz0, double tol, int max_attempts);

// ------------------------------------------------------------------------
// Per-instance energies of one round trip from the column-tile partial sums,
// summed in tile order (deterministic), into history row counter[0]. A
// non-finite energy, or a non-finite value stored by the boundary launch
// (counter[3]), sets the stop flag counter[2] instead: the row is not written,
// the counters do not advance, and every later launch of the call stores
// nothing, so the state the round trip started from (kept by its refresh
// launch) is the last finite one.
__global__ __launch_bounds__(kThreads) void energy_reduce(const InstDesc *inst, int n_inst,
                                                          const double *partial, double *hist,
                                                          int *counter, int capacity);

// counter[0] = slot; counter[1] = rt unless rt < 0; clear_flags: counter[2] = counter[3] = 0.
__global__ void set_counter(int *counter, int slot, int rt, int clear_flags);

// ------------------------------------------------------------------------
// Spectrum read-out into caller memory without allocating: the column and row
// passes run on a one-instance batch held in a fixed scratch area. spectrum_prep
// writes there the descriptor of instance i as that batch's only instance
// (fields at offset 0, tiles counted from 0), a zeroed tile -> instance map of
// map_len entries and zeroed counters (one workgroup).
__global__ __launch_bounds__(kThreads) void spectrum_prep(const InstDesc *inst, int i, InstDesc *desc,
                                                          int *counter, int *map, int map_len);

// out[f nt + k] = bin k of field f, from the row-pass layout, where bin
// k = k2 + n2 k1 sits at position k2 n1 + k1 of its field.
template <typename R>
__global__ __launch_bounds__(kThreads) void spectrum_order(const InstDesc *desc, const cplx<R> *src, cplx<R> *out)
{
    const InstDesc &d = *desc;
    const long long n = static_cast<long long>(d.nf) * d.nt;
    for (long long q = blockIdx.x * static_cast<long long>(kThreads) + threadIdx.x; q < n;
         q += static_cast<long long>(gridDim.x) * kThreads) {
        const long long f = q >> d.log2nt;
        const int k = static_cast<int>(q & (d.nt - 1));
        const int k2 = k & (d.n2 - 1), k1 = k >> d.log2n2;
        out[q] = src[(f << d.log2nt) + (static_cast<long long>(k2) << d.log2n1) + k1];
    }
}

} // namespace opo
