/*
 * opo_oracle.c -- plain, slow, FP64 CPU reference of the optical parametric
 * oscillator hot path: fixed-step symmetrized split-step Fourier (SSFM)
 * propagation of the three-wave coupled-wave equations through a chi(2)
 * crystal, repeated over cavity round trips.
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the CPU
 * baseline of the benchmark load this file. It shares no code, header, table
 * or constant with the GPU library and must never be linked into it.
 *
 * Sources (arXiv 2410.02532, "CUDA-based optical parametric oscillator
 * simulator"):
 *   Eqs. 2-4   coupled-wave equations                       -> cwe_rhs
 *   Sec. 2.1   kappa_x = 2 pi d_eff / (n_x lambda_x)        -> ora_kappa
 *   Eq. 5      linear operator (loss, GVM, GVD, TOD)        -> ora_dispersion
 *   Sec. 2.2   RK4 for the nonlinear part, Eq. 10/11 split  -> ora_rk4, ora_pass
 *   Eq. 9      unsymmetrized split (negative control only)  -> ora_pass_unsym
 *   Eq. 6      resonant-field boundary condition            -> ora_roundtrips
 *   Sec. 2.3   intracavity GDD and EOM                      -> ora_gdd, ora_eom
 *   Sec. 4.1   main loop: pump read, pass, GDD, phase, EOM  -> ora_roundtrips
 *   Sec. 2.4   degenerate signal equation (two waves)        -> cwe2_rhs
 *   Sec. 1     Kerr term named as an extension                -> kerr_rhs
 *   Sec. 1     adaptive step (local-error method) named as an
 *              extension                                      -> ora_propagate_adaptive
 *   Sec. 1     several crystals per round trip               -> ora_roundtrips_multi
 *   Sec. 4.1   nanosecond regime: long pump read slice by slice,
 *              per-round-trip output record (ReadPump,
 *              SaveRoundTrip)                                -> ora_roundtrips_rec
 *
 * Readings of passages the paper leaves open (each one is also recorded in
 * the design notes):
 *   - Fourier convention: forward X_k = sum_j x_j e^{-2 pi i jk/N} (not
 *     normalized), inverse with e^{+...} and 1/N. Angular frequency of bin k
 *     is 2 pi k/T for k < N/2 and 2 pi (k-N)/T otherwise (Nyquist negative).
 *   - Eq. 5 is taken in the physically derived form (group-velocity term with
 *     the sign that moves a slower field to later times, third-order term
 *     beta3/6 d^3/dtau^3 without the printed i and 1/3):
 *       H_x(w) = exp{ [ -alpha_x/2 + i(-db1_x w + b2_x w^2/2 - b3_x w^3/6) ] dz }
 *     with db1_x = 1/v_x - 1/v_s (signal co-moving frame).
 *   - RK4 advances the three fields together (classical coupled RK4) and
 *     evaluates e^{+-i dk z} at the stage positions z0, z0+h/2, z0+h; the
 *     first half-step of step j covers [z_j, z_j + dz/2], the second
 *     [z_j + dz/2, z_j + dz]. Adjacent half-steps are not merged.
 *   - Round trip: at its start a non-resonant pump is re-read from the input
 *     pump and non-resonant signal/idler start at zero; after the pass the
 *     energies sum_j |A_x(t_j)|^2 are recorded, then GDD, then
 *     sqrt(R_x) e^{i delta_x} on resonant fields, then the EOM phase.
 *   - Fourth-order splitting (crystal order = 4; the paper keeps the
 *     second-order symmetrized step and points to the literature for
 *     higher orders): every step of size dz is the composition of three
 *     symmetrized steps of a dz, b dz, a dz, a = 1/(2 - 2^(1/3)), b = 1 - 2a
 *     (the Yoshida / Suzuki triple jump), each with its own z range.
 *   - Several crystals per round trip (an extension the paper names): the
 *     fields pass them in order, each crystal with its own parameters, step
 *     count and z measured from its own entrance (so its e^{i dk z} starts at
 *     1); nothing acts between them, and the boundary follows the last.
 *   - Kerr term (the chi(3) extension the paper names as a simple addition,
 *     in the coupled nonlinear Schroedinger form): each field gains
 *     i gamma_x (|A_x|^2 + 2 sum_{y != x} |A_y|^2) A_x in the nonlinear
 *     operator, gamma_x = (2 pi / lambda_x) n2 (n_x eps0 c / 2), so that the
 *     self-phase per length is k0 n2 I with I = n eps0 c |A|^2 / 2.
 *   - Resonant pump (pump-resonant and triply resonant cavities): the paper
 *     leaves the pump injection unprinted. At the start of every round trip
 *     the input pump couples in through the pump mirror, A_p += sqrt(1 - R_p)
 *     A_in, while sqrt(R_p) e^{i delta_p} acts on the circulating pump at the
 *     end of the round trip like on any resonant field.
 *   - Nanosecond regime: the input pump is a long record of n_slices
 *     consecutive windows of nt samples; round trip m reads window m into a
 *     non-resonant pump, and a zero pump once the record is exhausted. The
 *     per-round-trip output is each field as it leaves the crystal (after the
 *     pass, before GDD and the mirror), stored as window m of the output.
 *   - Two coupled waves (degenerate operation, signal = idler; nf = 2): the
 *     paper gives the signal equation dA_s/dz = i kappa_s A_p A_s^* (with
 *     e^{+i dk z}) and leaves the pump equation unprinted. We take
 *     dA_p/dz = i kappa_p2 A_s^2 e^{-i dk z} with kappa_p2 = 2 pi d_eff /
 *     (n_p lambda_s), the coefficient for which n_p|A_p|^2 + n_s|A_s|^2 is
 *     conserved (kappa_p/2 at lambda_s = 2 lambda_p). Fields are then stored
 *     as pump, signal; the idler entries of the parameters are unused.
 *   - Adaptive step (the paper keeps a fixed dz and points to the step-size
 *     literature): the local-error method with the relative error of a step
 *     measured over all fields together, the accept band [tol/2, tol] and
 *     rejection above 2 tol, growth and shrink by 2^(1/3), halving on
 *     rejection, and Richardson extrapolation (4 u_f - u_c)/3 of the accepted
 *     step; the last step is cut to end exactly at the end of the crystal
 *     (stretched instead when it would stop within 1e-9 of a step short).
 *
 * Units: t [ps], z [mm], omega [rad/ps], lambda [um], d_eff [pm/V],
 * dk [1/mm], alpha [1/mm], db1 [ps/mm], b2 [fs^2/mm], b3 [fs^3/mm],
 * GDD [fs^2], f_pm [THz], fields A [V/m]. kappa is returned in
 * 1/(mm V/m) so that kappa*A is in 1/mm.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

#define ORA_PI 3.14159265358979323846
#define ORA_CBRT2 1.25992104989487316477   /* 2^(1/3), the nearest double (libm cbrt is not
                                             always correctly rounded) */

typedef struct {
    int nt;                /* time points, a power of two                 */
    int nf;                /* coupled waves: 3 (p, s, i) or 2 (p, s)      */
    double t_window_ps;    /* T: time window = round-trip time slice        */
    double length_mm;      /* crystal length L                              */
    double lambda_um[3];   /* pump, signal, idler wavelengths               */
    double n[3];           /* refractive indices                            */
    double deff_pm_per_v;  /* effective nonlinear coefficient               */
    double dk_per_mm;      /* phase mismatch dk = k_p - k_s - k_i (Eq. 1)   */
    double alpha_per_mm[3];
    double db1_ps_per_mm[3];
    double b2_fs2_per_mm[3];
    double b3_fs3_per_mm[3];
    double n2_m2_per_w;    /* Kerr (chi(3)) nonlinear index, 0 = none       */
    int order;             /* splitting order: 2 (symmetrized) or 4         */
} ora_crystal;

typedef struct {
    int resonant[3];       /* which fields feel Eq. 6                       */
    double refl[3];        /* R_x = 1 - theta_x                             */
    double delta_rad[3];   /* detuning phase per round trip                 */
    double gdd_fs2;        /* chirped-mirror GDD gamma                      */
    int gdd_on[3];
    double eom_beta;       /* EOM modulation depth                          */
    double eom_fpm_thz;    /* EOM frequency                                 */
    int eom_on[3];
} ora_cavity;

/* ---------------------------------------------------------------- FFT -- */

/* Twiddles w_r = e^{-2 pi i r/N}, r < N/2, from cos/sin in double. */
static cplx *twiddles(int n)
{
    int h = n / 2 > 0 ? n / 2 : 1;
    cplx *w = malloc(sizeof(cplx) * (size_t)h);
    for (int r = 0; r < h; r++) {
        double a = 2.0 * ORA_PI * (double)r / (double)n;
        w[r] = cos(a) - I * sin(a);
    }
    return w;
}

/* Iterative radix-2 decimation-in-time FFT with bit-reversal reordering.
 * inverse = 0: X_k = sum_j x_j e^{-2 pi i jk/N};
 * inverse = 1: x_j = (1/N) sum_k X_k e^{+2 pi i jk/N}. In place. */
static void fft_with(cplx *x, int n, int inverse, const cplx *w)
{
    for (int i = 1, j = 0; i < n; i++) {
        int bit = n >> 1;
        for (; j & bit; bit >>= 1)
            j ^= bit;
        j ^= bit;
        if (i < j) {
            cplx t = x[i];
            x[i] = x[j];
            x[j] = t;
        }
    }
    for (int len = 2; len <= n; len <<= 1) {
        int half = len / 2, stride = n / len;
        for (int base = 0; base < n; base += len) {
            for (int k = 0; k < half; k++) {
                cplx wk = inverse ? conj(w[k * stride]) : w[k * stride];
                cplx u = x[base + k];
                cplx v = x[base + k + half] * wk;
                x[base + k] = u + v;
                x[base + k + half] = u - v;
            }
        }
    }
    if (inverse)
        for (int i = 0; i < n; i++)
            x[i] /= (double)n;
}

void ora_fft(cplx *x, int n, int inverse)
{
    cplx *w = twiddles(n);
    fft_with(x, n, inverse, w);
    free(w);
}

/* ------------------------------------------------------ coefficients -- */

/* Angular frequency of DFT bin k on a window of T ps (numpy fftfreq order). */
double ora_omega(int k, int n, double t_window_ps)
{
    int ks = (k < n / 2) ? k : k - n;
    return 2.0 * ORA_PI * (double)ks / t_window_ps;
}

/* Nonlinear coupling, Sec. 2.1: kappa_x = 2 pi d_eff / (n_x lambda_x).
 * pm/V over um gives 1e-6 per metre; 1e-3 more converts to per mm.
 * Two waves: (kappa_p2, kappa_s, 0), kappa_p2 = 2 pi d_eff / (n_p lambda_s). */
void ora_kappa(const ora_crystal *c, double kappa[3])
{
    for (int x = 0; x < 3; x++)
        kappa[x] = 2.0 * ORA_PI * c->deff_pm_per_v / (c->n[x] * c->lambda_um[x]) * 1e-9;
    if (c->nf == 2) {
        kappa[0] = 2.0 * ORA_PI * c->deff_pm_per_v / (c->n[0] * c->lambda_um[1]) * 1e-9;
        kappa[2] = 0.0;
    }
}

/* Frequency-domain propagator of Eq. 5 (reading above) over a step dz. */
void ora_dispersion(const ora_crystal *c, int x, double dz, cplx *h)
{
    double b2 = c->b2_fs2_per_mm[x] * 1e-6; /* ps^2/mm */
    double b3 = c->b3_fs3_per_mm[x] * 1e-9; /* ps^3/mm */
    for (int k = 0; k < c->nt; k++) {
        double w = ora_omega(k, c->nt, c->t_window_ps);
        double phase = -c->db1_ps_per_mm[x] * w + 0.5 * b2 * w * w - b3 * w * w * w / 6.0;
        h[k] = cexp((-0.5 * c->alpha_per_mm[x] + I * phase) * dz);
    }
}

/* ------------------------------------------------------- nonlinear -- */

/* Right-hand side of Eqs. 2-4 without the linear operator, at one time
 * point; ph = e^{+i dk z}. */
static void cwe_rhs(const double kap[3], cplx ph, cplx ap, cplx as, cplx ai, cplx out[3])
{
    out[0] = I * kap[0] * as * ai * conj(ph);
    out[1] = I * kap[1] * ap * conj(ai) * ph;
    out[2] = I * kap[2] * ap * conj(as) * ph;
}

/* The two-wave (degenerate) right-hand side: pump and signal. */
static void cwe2_rhs(const double kap[3], cplx ph, cplx ap, cplx as, cplx out[3])
{
    out[0] = I * kap[0] * as * as * conj(ph);
    out[1] = I * kap[1] * ap * conj(as) * ph;
    out[2] = 0.0;
}

/* Kerr coefficients gamma_x in 1/mm per (V/m)^2 (0 without n2). */
void ora_kerr(const ora_crystal *c, double gamma[3])
{
    const double eps0 = 8.8541878128e-12, c0 = 299792458.0;
    for (int x = 0; x < 3; x++)
        gamma[x] = 2.0 * ORA_PI / (c->lambda_um[x] * 1e-6) * c->n2_m2_per_w *
                   (0.5 * c->n[x] * eps0 * c0) * 1e-3;
}

/* Self- and cross-phase modulation of the nf fields, added to out. */
static void kerr_rhs(int nf, const double gam[3], const cplx y[3], cplx out[3])
{
    double p[3] = {0.0, 0.0, 0.0};
    for (int x = 0; x < nf; x++)
        p[x] = creal(y[x]) * creal(y[x]) + cimag(y[x]) * cimag(y[x]);
    for (int x = 0; x < nf; x++) {
        double phi = p[x];
        for (int o = 0; o < nf; o++)
            if (o != x)
                phi += 2.0 * p[o];
        out[x] += I * gam[x] * phi * y[x];
    }
}

static void rhs(int nf, const double kap[3], const double gam[3], int kerr, cplx ph,
                const cplx y[3], cplx out[3])
{
    if (nf == 2)
        cwe2_rhs(kap, ph, y[0], y[1], out);
    else
        cwe_rhs(kap, ph, y[0], y[1], y[2], out);
    if (kerr)
        kerr_rhs(nf, gam, y, out);
}

/* One classical RK4 step of size h from z0 for all time points of the
 * nf fields stored as A[x*nt + j]. */
void ora_rk4(const ora_crystal *c, cplx *a, double z0, double h)
{
    int n = c->nt, nf = c->nf;
    double kap[3], gam[3];
    ora_kappa(c, kap);
    ora_kerr(c, gam);
    int kerr = c->n2_m2_per_w != 0.0;
    cplx ph0 = cexp(I * c->dk_per_mm * z0);
    cplx ph1 = cexp(I * c->dk_per_mm * (z0 + 0.5 * h));
    cplx ph2 = cexp(I * c->dk_per_mm * (z0 + h));
    for (int j = 0; j < n; j++) {
        cplx y[3] = {0.0, 0.0, 0.0};
        for (int x = 0; x < nf; x++)
            y[x] = a[x * n + j];
        cplx k1[3], k2[3], k3[3], k4[3], t[3];
        rhs(nf, kap, gam, kerr, ph0, y, k1);
        for (int x = 0; x < 3; x++)
            t[x] = y[x] + 0.5 * h * k1[x];
        rhs(nf, kap, gam, kerr, ph1, t, k2);
        for (int x = 0; x < 3; x++)
            t[x] = y[x] + 0.5 * h * k2[x];
        rhs(nf, kap, gam, kerr, ph1, t, k3);
        for (int x = 0; x < 3; x++)
            t[x] = y[x] + h * k3[x];
        rhs(nf, kap, gam, kerr, ph2, t, k4);
        for (int x = 0; x < nf; x++)
            a[x * n + j] = y[x] + h / 6.0 * (k1[x] + 2.0 * k2[x] + 2.0 * k3[x] + k4[x]);
    }
}

/* -------------------------------------------------------- linear -- */

static void linear_with(cplx *field, int n, const cplx *h, const cplx *w)
{
    fft_with(field, n, 0, w);
    for (int k = 0; k < n; k++)
        field[k] *= h[k];
    fft_with(field, n, 1, w);
}

/* e^{L_x dz} for the nf fields: FFT, multiply by H_x, inverse FFT. */
void ora_linear(const ora_crystal *c, cplx *a, double dz)
{
    int n = c->nt;
    cplx *w = twiddles(n);
    cplx *h = malloc(sizeof(cplx) * (size_t)n);
    for (int x = 0; x < c->nf; x++) {
        ora_dispersion(c, x, dz, h);
        linear_with(a + (size_t)x * n, n, h, w);
    }
    free(h);
    free(w);
}

/* ---------------------------------------------------------- SSFM -- */

/* One symmetrized step of size tau from z (Eqs. 10-11): N(tau/2) ->
 * F^-1 e^{L tau} F -> N(tau/2), with the propagators h of that step. */
static void strang_step(const ora_crystal *c, cplx *a, double z, double tau, const cplx *h,
                        const cplx *w)
{
    int n = c->nt;
    ora_rk4(c, a, z, 0.5 * tau);
    for (int x = 0; x < c->nf; x++)
        linear_with(a + (size_t)x * n, n, h + (size_t)x * n, w);
    ora_rk4(c, a, z + 0.5 * tau, 0.5 * tau);
}

/* Fourth-order composition of symmetrized steps (the higher-order splitting
 * the paper points to for users who need it): S(a dz) S(b dz) S(a dz) with
 * a = 1/(2 - 2^(1/3)), b = 1 - 2a; the middle step runs backwards. */
#define ORA_TJ_A 1.35120719195965763405
#define ORA_TJ_B (-1.70241438391931526810)

/* nz steps of size dz, step j starting at z0 + j dz: symmetrized (order 2)
 * or the fourth-order composition (order 4). */
void ora_pass(const ora_crystal *c, cplx *a, int nz, double dz, double z0)
{
    int n = c->nt;
    cplx *w = twiddles(n);
    cplx *h = malloc(sizeof(cplx) * (size_t)n * 3);
    cplx *hb = malloc(sizeof(cplx) * (size_t)n * 3);
    int four = c->order == 4;
    for (int x = 0; x < c->nf; x++) {
        ora_dispersion(c, x, four ? ORA_TJ_A * dz : dz, h + (size_t)x * n);
        if (four)
            ora_dispersion(c, x, ORA_TJ_B * dz, hb + (size_t)x * n);
    }
    for (int j = 0; j < nz; j++) {
        double zj = z0 + (double)j * dz;
        if (!four) {
            strang_step(c, a, zj, dz, h, w);
        } else {
            strang_step(c, a, zj, ORA_TJ_A * dz, h, w);
            strang_step(c, a, zj + ORA_TJ_A * dz, ORA_TJ_B * dz, hb, w);
            strang_step(c, a, zj + (ORA_TJ_A + ORA_TJ_B) * dz, ORA_TJ_A * dz, h, w);
        }
    }
    free(hb);
    free(h);
    free(w);
}

/* Negative control: the unsymmetrized split of Eq. 9, e^{L dz} e^{N dz}
 * (a full RK4 step, then the full linear step). Not part of the method. */
void ora_pass_unsym(const ora_crystal *c, cplx *a, int nz, double dz, double z0)
{
    int n = c->nt;
    cplx *w = twiddles(n);
    cplx *h = malloc(sizeof(cplx) * (size_t)n * 3);
    for (int x = 0; x < c->nf; x++)
        ora_dispersion(c, x, dz, h + (size_t)x * n);
    for (int j = 0; j < nz; j++) {
        ora_rk4(c, a, z0 + (double)j * dz, dz);
        for (int x = 0; x < c->nf; x++)
            linear_with(a + (size_t)x * n, n, h + (size_t)x * n, w);
    }
    free(h);
    free(w);
}

/* ---------------------------------------------- intracavity elements -- */

/* Chirped-mirror GDD (Sec. 2.3): A~(w) -> A~(w) e^{i gamma w^2/2}. */
void ora_gdd(cplx *field, int n, double t_window_ps, double gdd_fs2)
{
    double g = gdd_fs2 * 1e-6; /* ps^2 */
    cplx *w = twiddles(n);
    fft_with(field, n, 0, w);
    for (int k = 0; k < n; k++) {
        double om = ora_omega(k, n, t_window_ps);
        field[k] *= cexp(I * 0.5 * g * om * om);
    }
    fft_with(field, n, 1, w);
    free(w);
}

/* Electro-optic phase modulator (Sec. 2.3): A(t) -> A(t) e^{i beta sin(2 pi f t)},
 * t_j = -T/2 + j T/N. */
void ora_eom(cplx *field, int n, double t_window_ps, double beta, double fpm_thz)
{
    double dt = t_window_ps / (double)n;
    for (int j = 0; j < n; j++) {
        double t = -0.5 * t_window_ps + (double)j * dt;
        field[j] *= cexp(I * beta * sin(2.0 * ORA_PI * fpm_thz * t));
    }
}

/* ----------------------------------------------------- round trips -- */

/* Round trips with a long input pump and an output record (nanosecond
 * regime). pump_in holds n_slices windows of nt samples; round trip m reads
 * window m (m < n_slices) into a non-resonant pump, else a zero pump.
 * record, if not NULL, receives window m of every field as it leaves the
 * crystal: record[(m*nf + x)*nt + j]. energy[m*3+x] as ora_roundtrips. */
static void roundtrips(const ora_crystal *cs, int n_cryst, const int *nzs, const ora_cavity *cav,
                       cplx *a, const cplx *pump_in, int n_slices, int same_pump, int n_rt,
                       double *energy, cplx *record)
{
    const ora_crystal *c = cs;   /* grid and field count: the same in every crystal */
    int n = c->nt;
    for (int m = 0; m < n_rt; m++) {
        int w = same_pump ? 0 : m;
        if (!cav->resonant[0]) {
            if (w < n_slices)
                memcpy(a, pump_in + (size_t)w * n, sizeof(cplx) * (size_t)n);
            else
                memset(a, 0, sizeof(cplx) * (size_t)n);
        } else if (w < n_slices) {
            /* resonant pump: the input couples in through a mirror of
             * transmission 1 - R_p */
            double t = sqrt(1.0 - cav->refl[0]);
            for (int j = 0; j < n; j++)
                a[j] += t * pump_in[(size_t)w * n + j];
        }
        for (int x = 1; x < c->nf; x++)
            if (!cav->resonant[x])
                memset(a + (size_t)x * n, 0, sizeof(cplx) * (size_t)n);

        /* the crystals of the round trip in order, each from its own entrance */
        for (int k = 0; k < n_cryst; k++)
            ora_pass(cs + k, a, nzs[k], cs[k].length_mm / (double)nzs[k], 0.0);

        if (record)
            memcpy(record + (size_t)m * c->nf * n, a, sizeof(cplx) * (size_t)c->nf * n);
        for (int x = 0; x < 3; x++) {
            double e = 0.0;
            if (x >= c->nf) {
                energy[m * 3 + x] = 0.0;
                continue;
            }
            for (int j = 0; j < n; j++) {
                cplx v = a[(size_t)x * n + j];
                e += creal(v) * creal(v) + cimag(v) * cimag(v);
            }
            energy[m * 3 + x] = e;
        }
        for (int x = 0; x < c->nf; x++)
            if (cav->gdd_on[x] && cav->gdd_fs2 != 0.0)
                ora_gdd(a + (size_t)x * n, n, c->t_window_ps, cav->gdd_fs2);
        for (int x = 0; x < c->nf; x++)
            if (cav->resonant[x]) {
                cplx f = sqrt(cav->refl[x]) * cexp(I * cav->delta_rad[x]);
                for (int j = 0; j < n; j++)
                    a[(size_t)x * n + j] *= f;
            }
        for (int x = 0; x < c->nf; x++)
            if (cav->eom_on[x] && cav->eom_beta != 0.0)
                ora_eom(a + (size_t)x * n, n, c->t_window_ps, cav->eom_beta, cav->eom_fpm_thz);
    }
}

void ora_roundtrips_rec(const ora_crystal *c, const ora_cavity *cav, cplx *a,
                        const cplx *pump_in, int n_slices, int nz, int n_rt,
                        double *energy, cplx *record)
{
    roundtrips(c, 1, &nz, cav, a, pump_in, n_slices, 0, n_rt, energy, record);
}

/* Round trips through n_cryst crystals in sequence (crystal k with nzs[k]
 * steps of its own L/nz, z from its own entrance), then the boundary as in
 * ora_roundtrips_rec. Every crystal has the grid and field count of the first. */
void ora_roundtrips_multi(const ora_crystal *cs, int n_cryst, const int *nzs,
                          const ora_cavity *cav, cplx *a, const cplx *pump_in, int n_slices,
                          int n_rt, double *energy, cplx *record)
{
    roundtrips(cs, n_cryst, nzs, cav, a, pump_in, n_slices, 0, n_rt, energy, record);
}

/* n_rt cavity round trips (Sec. 4.1 main loop with Eq. 6) with the same
 * input pump every round trip. energy[m*3+x] receives sum_j |A_x(t_j)|^2
 * after the crystal pass of round trip m (0 for x >= nf). */
void ora_roundtrips(const ora_crystal *c, const ora_cavity *cav, cplx *a,
                    const cplx *pump_in, int nz, int n_rt, double *energy)
{
    roundtrips(c, 1, &nz, cav, a, pump_in, 1, 1, n_rt, energy, NULL);
}

/* ------------------------------------------------------ adaptive step -- */

/* Propagation from z0 over `length` with the step chosen by the local-error
 * method (Sinkin et al., J. Lightwave Technol. 21, 61 (2003): the adaptive
 * scheme of the step-size literature the paper points to for users who need
 * one). From z, a coarse symmetrized step of dz and two fine ones of dz/2 give
 * d = ||u_f - u_c|| / ||u_f||, the norms over every sample of every field.
 * d > 2 tol: the attempt is rejected and dz halved. Otherwise
 * (4 u_f - u_c)/3 is accepted, z advances by dz, and dz is divided by 2^(1/3)
 * if d > tol, multiplied by it if d < tol/2. A step that would pass the end,
 * or stop short of it by less than 1e-9 dz, is cut (or stretched) to end
 * there, and z is then set to the end itself. A d that is not a number
 * rejects the attempt, except for fields that are zero everywhere (0/0),
 * which keep it with dz unchanged. Second-order steps
 * only (the extrapolation weights assume them). Returns 0; -1 when max_steps
 * attempts (accepted and rejected) do not reach the end; -2 for order != 2. */
int ora_propagate_adaptive(const ora_crystal *c, cplx *a, double z0, double length, double tol, double dz0,
                           int max_steps, int *accepted, int *rejected)
{
    *accepted = 0;
    *rejected = 0;
    if (c->order != 2) return -2;
    const size_t n = (size_t)c->nf * (size_t)c->nt;
    cplx *uc = malloc(sizeof(cplx) * n), *uf = malloc(sizeof(cplx) * n);
    const double grow = ORA_CBRT2, end = z0 + length;
    double z = z0, dz = dz0;
    int rc = 0;
    while (z < end) {
        if (*accepted + *rejected >= max_steps) {
            rc = -1;
            break;
        }
        const double rest = end - z;
        const int last = rest <= dz * (1.0 + 1e-9);   /* no sliver of < 1e-9 dz left over */
        if (last) dz = rest;
        memcpy(uc, a, sizeof(cplx) * n);
        memcpy(uf, a, sizeof(cplx) * n);
        ora_pass(c, uc, 1, dz, z);
        ora_pass(c, uf, 2, 0.5 * dz, z);
        double num = 0.0, den = 0.0;
        for (size_t i = 0; i < n; i++) {
            const cplx e = uf[i] - uc[i];
            num += creal(e) * creal(e) + cimag(e) * cimag(e);
            den += creal(uf[i]) * creal(uf[i]) + cimag(uf[i]) * cimag(uf[i]);
        }
        /* d is undefined (0/0) for fields that are zero everywhere: the attempt
         * is kept with dz unchanged. Any other d that is not a number (a step
         * that overflowed, non-finite fields) rejects the attempt like a too
         * large error; the attempt budget ends a run that never recovers. */
        const int zero = num == 0.0 && den == 0.0;
        const double d = sqrt(num / den);
        if (!zero && !(d <= 2.0 * tol)) {
            dz *= 0.5;
            ++*rejected;
            continue;
        }
        for (size_t i = 0; i < n; i++)
            a[i] = (4.0 * uf[i] - uc[i]) / 3.0;
        z = last ? end : z + dz;
        ++*accepted;
        if (d > tol)
            dz /= grow;
        else if (d < 0.5 * tol)
            dz *= grow;
    }
    free(uf);
    free(uc);
    return rc;
}
