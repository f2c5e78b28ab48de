/*
 * opo.h -- C ABI of the MI355X (gfx950) optical parametric oscillator hot path.
 *
 * The library propagates the three-wave coupled-wave equations (Eqs. 2-4 of
 * arXiv 2410.02532) for pump (p, index 0), signal (s, 1) and idler (i, 2), or
 * at degeneracy the two-wave equations for pump and signal (see n_fields),
 * through a chi(2) crystal with the fixed-step symmetrized split-step Fourier
 * method (Sec. 2.2, Eqs. 10-11: nonlinear half-step by RK4, linear step in
 * the frequency domain, nonlinear half-step), and repeats the pass over cavity
 * round trips with the resonant-field boundary condition of Eq. 6 and the
 * intracavity elements of Sec. 2.3 (chirped-mirror GDD, electro-optic phase
 * modulator), in the loop order of Sec. 4.1.
 *
 * Conventions shared by every call:
 *   - Units: time ps, length mm, wavelength um, d_eff pm/V, dk 1/mm,
 *     alpha 1/mm, group-delay mismatch ps/mm, GVD fs^2/mm, TOD fs^3/mm,
 *     GDD fs^2, EOM frequency THz, phases rad, fields V/m.
 *   - Grid (Sec. 2.4): nt samples t_j = -T/2 + j T/nt over a window T; nt is
 *     a power of two. Frequency bin k has angular frequency 2 pi k/T for
 *     k < nt/2 and 2 pi (k - nt)/T otherwise.
 *   - Linear operator (Eq. 5, read in its physically derived form): over a
 *     step dz the spectrum of field x is multiplied by
 *     exp{[-alpha_x/2 + i(-db1_x w + b2_x w^2/2 - b3_x w^3/6)] dz}, db1_x being
 *     the group-delay mismatch to the signal (a positive value is slower and
 *     drifts to later t). The phase is formed and reduced modulo 2 pi in FP64.
 *   - Coupling (Sec. 2.1): kappa_x = 2 pi d_eff/(n_x lambda_x).
 *   - Two waves (degenerate operation, signal = idler): dA_s/dz =
 *     i kappa_s A_p A_s^* e^{+i dk z}, the signal equation of the paper's
 *     degenerate case (Sec. 2.4), and dA_p/dz = i kappa_p2 A_s^2 e^{-i dk z}
 *     with kappa_p2 = 2 pi d_eff/(n_p lambda_s), the pump coefficient that
 *     conserves n_p|A_p|^2 + n_s|A_s|^2 (the paper does not print it). The
 *     idler entries of every per-field array are then unused.
 *   - Host field arrays are interleaved complex128: re, im, re, im, ...
 *   - Every call returns an opo_status; negative values are errors and
 *     opo_last_error() returns a message for the calling thread. No C++
 *     exception crosses the boundary. A handle must not be used from two
 *     threads at once; distinct handles are independent.
 */
#ifndef OPO_H
#define OPO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    OPO_OK = 0,
    OPO_EINVAL = -1,     /* bad argument, size or physical parameter            */
    OPO_ENOMEM = -2,     /* device or host allocation failed                    */
    OPO_EDEVICE = -3,    /* no usable gfx950 device, or a HIP call failed       */
    OPO_ENONFINITE = -4, /* a round-trip energy became NaN or Inf               */
    OPO_ESTATE = -5,     /* NULL or already destroyed handle, bad call order    */
    OPO_ESTEPS = -6      /* adaptive step: attempt budget spent before the end  */
} opo_status;

enum { OPO_F32 = 0, OPO_F64 = 1 };

typedef struct opo_s opo_t;

/* Fields and grid of one instance. */
typedef struct {
    int32_t nt;             /* time samples, power of two, 2 .. 2^20 (FP64: 2^19) */
    double t_window_ps;     /* window T (> 0)                                     */
    double lambda_um[3];    /* wavelengths p, s, i (> 0)                          */
    double n[3];            /* refractive indices (> 0)                           */
    const double *init;     /* n_fields*nt complex128 initial fields p, s(, i)
                               (time domain), host memory, copied; NULL = zero    */
    const double *pump_in;  /* nt complex128 input pump read into a non-resonant
                               pump at the start of every round trip (or
                               pump_windows windows of nt, see below); NULL = the
                               constant pump_cw below                             */
    double pump_cw[2];      /* constant input pump (re, im) when pump_in is NULL  */
    int32_t n_fields;       /* coupled waves: 3 (or 0) = pump, signal, idler;
                               2 = pump and degenerate signal                     */
    int32_t pump_windows;   /* nanosecond regime (Sec. 4.1 pump read): pump_in
                               holds pump_windows consecutive windows of nt
                               samples and round trip m (counted from opo_init)
                               reads window m, then a zero pump once m >=
                               pump_windows; 0 or 1 = the same nt samples every
                               round trip                                         */
} opo_fields_t;

/* Crystal: length, z-grid and the coefficients of Eqs. 2-5. */
typedef struct {
    double length_mm;       /* L (> 0)                                            */
    int32_t nz;             /* steps per pass in cavity_roundtrip (>= 1); every
                               instance of a batch must use the same nz           */
    double deff_pm_per_v;   /* d_eff                                              */
    double dk_per_mm;       /* phase mismatch dk = k_p - k_s - k_i (Eq. 1)        */
    double alpha_per_mm[3]; /* field loss alpha_x (power attenuation)             */
    double db1_ps_per_mm[3];/* 1/v_x - 1/v_s                                      */
    double b2_fs2_per_mm[3];/* GVD k''_x                                          */
    double b3_fs3_per_mm[3];/* TOD k'''_x                                         */
    double n2_m2_per_w;     /* Kerr index n2 [m^2/W], 0 = none: the nonlinear step
                               adds i gamma_x (|A_x|^2 + 2 sum_{y != x} |A_y|^2) A_x
                               with gamma_x = (2 pi/lambda_x) n2 (n_x eps0 c/2),
                               the chi(3) extension the paper names (Sec. 1)      */
} opo_crystal_t;

/* Cavity: Eq. 6 and the Sec. 2.3 elements, applied after every pass. */
typedef struct {
    int32_t resonant[3];    /* 1 = field is fed back (Eq. 6); a non-resonant pump
                               is re-read from the input, a non-resonant signal or
                               idler restarts from zero. A resonant pump (pump-
                               enhanced or triply resonant cavities) receives the
                               input through its mirror at the start of every
                               round trip: A_p += sqrt(1 - R_p) A_in              */
    double refl[3];         /* R_x = 1 - theta_x in [0, 1] (resonant fields)      */
    double delta_rad[3];    /* detuning phase delta_x per round trip              */
    double gdd_fs2;         /* chirped-mirror GDD gamma: spectrum * e^{i gamma w^2/2} */
    int32_t gdd_on[3];      /* fields that receive the GDD                        */
    double eom_beta;        /* EOM depth: A(t) * e^{i beta sin(2 pi f t)}         */
    double eom_fpm_thz;     /* EOM frequency f                                    */
    int32_t eom_on[3];      /* fields that pass the EOM                           */
} opo_cavity_t;

/* Run-time options. A zeroed struct (or NULL) selects the defaults. */
typedef struct {
    int32_t precision;      /* OPO_F32: complex64 fields, FFTs and RK4 with FP64
                               phase arguments and energy sums (default);
                               OPO_F64: complex128 throughout                     */
    int32_t device;         /* HIP device ordinal (default 0)                     */
    void *stream;           /* hipStream_t to run on; NULL = a stream the library
                               creates (default priority)                         */
    void *state;            /* optional device buffer of opo_state_bytes() bytes
                               that holds the fields; owned by the caller and
                               kept alive until opo_destroy; NULL = the library
                               allocates it                                       */
    uint64_t state_bytes;   /* size of *state                                     */
    int32_t col_log2;       /* four-step split nt = n1 * n2 (Sec. 2.2 FFTs): log2 n2
                               for instances of nt > 2^10, 0 = the schedule's
                               split (schedule 0) or the default (n2 = 64 from
                               2^13 up to the longest rows). 5 (n2 = 32) gives a
                               single instance of 2^13..2^17 twice the column
                               workgroups with half the work each: faster alone,
                               slower in a large batch. Clamped to n2 <= n1 and
                               n1 <= 4096 (FP32) or 2048 (FP64). Results differ
                               from another split by rounding only. 0 or 4..8,
                               else OPO_EINVAL                                    */
    int32_t schedule;       /* how fixed-step passes run:
                               0 = automatic: per instance from a built-in table
                               keyed by precision, field count, nt and whether the
                               handle's fields fill the chip (at least 2^20
                               complex samples in all: batch entries) or not
                               (one instance or a few), chosen by timing the
                               candidates on MI355X (one shape in one kind of
                               handle always gets the same schedule; an instance
                               alone and the same instance in a full batch may
                               differ in rounding);
                               1 = two passes per z-step (column and row tiles of
                               a four-step FFT) for every instance;
                               2 = resident where served: one workgroup holds an
                               instance for a whole pass and its boundary
                               (FP32 nt 2^10..2^12, FP64 2^10..2^11; split order
                               2, one crystal), two passes for the others.
                               Resident results differ from two-pass ones by
                               rounding only. Else OPO_EINVAL                     */
    int32_t use_graph;      /* 1 = replay each round trip from a hipGraph
                               (default), -1 = plain launches                     */
    int32_t profile;        /* 1 = bracket every kernel launch with a pair of
                               hipEvents on the handle's stream and accumulate
                               per-kernel device time (plain launches instead of
                               the graph, one stream synchronization per round
                               trip); read with opo_kernel_times                  */
    int32_t record_rt;      /* > 0: keep on the device, for each of the first
                               record_rt round trips (counted from opo_init),
                               every field as it leaves the crystal (after the
                               pass, before GDD and the mirror; Sec. 4.1 round-
                               trip save), read with opo_get_record. Costs
                               record_rt * opo_state_bytes() of device memory     */
    int32_t n_crystals;     /* crystals per round trip, K >= 1 (0 = 1): the crystal
                               array of opo_init_batch then holds n*K entries,
                               instance-major (crystals[i*K + k] is crystal k of
                               instance i); the fields pass them in order, each
                               with its own nz (shared by the instances) and z
                               from its own entrance, and the boundary follows
                               the last; ssfm_propagate uses crystal 0            */
    int32_t split_order;    /* 2 (or 0): the symmetrized step of Eqs. 10-11;
                               4: fourth-order composition of symmetrized steps
                               of a dz, b dz, a dz, a = 1/(2 - 2^(1/3)), b = 1 - 2a
                               (the higher-order splitting the paper leaves to
                               the user; three times the work per step, the step
                               criterion applies to |b| dz)                       */
} opo_options_t;

/* Device bytes of field state for n instances (n_fields * nt complex values
 * each) at a precision. */
uint64_t opo_state_bytes(int32_t n, const opo_fields_t *fields, int32_t precision);

/* Create a handle for one OPO instance: validates every parameter (nt a power
 * of two in range, finite positive physical constants, R in [0, 1], and the
 * step criterion of Sec. 2.4, kappa_x |A|max dz < 0.5 for dz = L/nz), copies the
 * host inputs to the device and builds the FFT and coupling tables. On error
 * *h is NULL. */
int opo_init(opo_t **h, const opo_fields_t *fields, const opo_crystal_t *crystal,
             const opo_cavity_t *cavity, const opo_options_t *options);

/* Same for n independent instances (arrays of n structs; nt may differ) that
 * advance together in every launch. */
int opo_init_batch(opo_t **h, int32_t n, const opo_fields_t *fields,
                   const opo_crystal_t *crystals, const opo_cavity_t *cavities,
                   const opo_options_t *options);

/* One crystal pass of nz symmetrized SSFM steps of size dz [mm] (Eq. 11) for
 * every instance, continuing z from the end of the previous call (so two calls
 * of nz/2 equal one of nz). No cavity operation. Asynchronous on the handle's
 * stream; opo_sync waits. */
int ssfm_propagate(opo_t *h, int32_t nz, double dz);

/* Propagation of every instance over length_mm [mm] from the handle's z with
 * the step chosen per instance by the local-error method (the adaptive step
 * the paper leaves to the user, Sec. 1, for its fixed-step Sec. 2.2): an
 * attempt from z compares one symmetrized step of dz with two of dz/2;
 * d = ||u_f - u_c|| / ||u_f|| over all fields of the instance. d > 2 tol
 * rejects the attempt and halves dz; otherwise the fields become
 * (4 u_f - u_c)/3, z advances by dz, and dz is divided by 2^(1/3) if d > tol,
 * multiplied by it if d < tol/2. The first attempt uses dz0; a step that would
 * pass the end (or stop within 1e-9 dz of it) ends there. max_attempts counts
 * accepted and rejected attempts per instance. Needs split_order 2; uses
 * crystal 0; no cavity operation. accepted, rejected and z_end (n entries
 * each, or NULL) receive each instance's counts and the z it reached. Returns
 * OPO_ESTEPS if an instance spent its budget first (its fields then hold the
 * last accepted step, at z_end); the handle's z advances by length_mm. The
 * first call allocates two state-sized copies and a per-instance propagator
 * table (2x the state in FP32, 1x in FP64) kept until opo_destroy.
 * Synchronizes the stream. */
int ssfm_propagate_adaptive(opo_t *h, double length_mm, double tol, double dz0, int32_t max_attempts,
                            int32_t *accepted, int32_t *rejected, double *z_end);

/* n_rt cavity round trips (Sec. 4.1): read the input pump into a non-resonant
 * pump and zero non-resonant signal/idler, one pass of crystal.nz steps with
 * dz = L/nz from z = 0, record sum_j |A_x(t_j)|^2 in FP64, apply GDD, the
 * mirror factor sqrt(R_x) e^{i delta_x} of Eq. 6, then the EOM. Appends n_rt
 * rows to the energy history. Synchronizes the stream at the end.
 * Non-finite results (the too-large step of Sec. 2.4 ends in NaN): if a round
 * trip m records an energy that is not finite, or ends with a field value that
 * is not finite, the call stops there and returns OPO_ENONFINITE. Round trip m
 * appends no row and no later round trip runs; the fields, z and the count of
 * round trips completed (which selects the next input-pump window and record
 * slot) are those after round trip m - 1, the last finite one (the fields m
 * started from). opo_get_progress and the message name m. The library keeps
 * that starting state in a device buffer of opo_state_bytes() bytes. */
int cavity_roundtrip(opo_t *h, int32_t n_rt);

/* Wait for all work queued on the handle's stream. */
int opo_sync(opo_t *h);

/* Copy field `field` (0 p, 1 s, 2 i; < n_fields) of instance `inst` to/from host memory
 * as nt interleaved complex128 values. domain 0 = time samples A(t_j);
 * domain 1 (get only) = unnormalized DFT sum_j A(t_j) e^{-2 pi i jk/nt} in
 * natural bin order. set also resets the handle's z to 0 (opo_set_progress
 * sets it). Stored at the handle's precision: complex64 values read with get
 * and set back are restored bit for bit. */
int opo_get_fields(opo_t *h, int32_t inst, int32_t field, int32_t domain, double *out);
int opo_set_fields(opo_t *h, int32_t inst, int32_t field, const double *in);

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): the spectrum of every
 * field of instance `inst`, written to caller device memory without any
 * allocation. out: device pointer to n_fields * nt complex values at the
 * handle's precision (complex64 for OPO_F32, complex128 for OPO_F64), field-
 * major, bin k of field x at out[x * nt + k] in natural bin order: the
 * unnormalized DFT sum_j A(t_j) e^{-2 pi i jk/nt}, the same values, bit for
 * bit, as opo_get_fields with domain 1. The caller owns out and keeps it alive
 * until the stream has passed the call. Asynchronous on the handle's stream (no
 * synchronization); the fields are not changed.
 * Scratch: a fixed 16 MiB device array that each GPU the library runs on
 * holds until the process ends; the call takes its device address on the
 * first use on a device. An instance needing more than 16 MiB - 16 KiB
 * (n_fields * nt * 8 bytes in FP32, * 16 in FP64: up to 3 x 2^19 points in
 * FP32, 3 x 2^18 in FP64) is rejected with OPO_EINVAL. Every call on a GPU
 * shares that array and overwrites it: calls that overlap on one GPU (two
 * handles on different streams, or two threads) race, so serialize them.
 * OPO_EINVAL for a bad instance or a NULL out. */
int opo_get_spectrum_noalloc(opo_t *h, int32_t inst, void *out);

/* Checkpoint and resume (the per-round-trip save of Sec. 4.1). A run is
 * resumed bit for bit by a handle created with the same inputs and options:
 * set every field with opo_set_fields, then opo_set_progress with what
 * opo_get_progress and the energy histories gave.
 * get: *rt_done = round trips completed since opo_init (= energy-history
 * rows), *z_mm = the z that the next ssfm_propagate continues from (either
 * pointer may be NULL).
 * set: the handle continues as after rt_done round trips: the next round trip
 * reads input-pump window rt_done (pump_windows > 1) and record slot rt_done,
 * the energy history becomes the rt_done rows of `history` (rt_done x
 * instances x 3 doubles, round-trip major, as the per-instance histories
 * stacked; NULL only for rt_done = 0), and z becomes z_mm (finite, >= 0).
 * The record (record_rt option) is not restored: slots of round trips run
 * before the restore read as zeros. OPO_EINVAL for bad arguments. Waits for
 * the handle's stream. */
int opo_get_progress(opo_t *h, int32_t *rt_done, double *z_mm);
int opo_set_progress(opo_t *h, int32_t rt_done, double z_mm, const double *history);

/* Energy history: out receives min(capacity, rows) rows of 3 doubles
 * sum_j |A_x(t_j)|^2 (p, s, i; the idler entry is 0 for two waves) after each
 * pass of cavity_roundtrip, oldest first; *rows receives the number recorded
 * so far. */
int opo_get_energy_history(opo_t *h, int32_t inst, double *out, int32_t capacity,
                           int32_t *rows);

/* Output power history [W], the same rows as the energy history: each field's
 * mean intensity over the window as it leaves the crystal,
 * I_x = n_x eps0 c E_x / (2 nt) (Sec. 2.1 field units, V/m), times the
 * effective beam area area_m2 [m^2], times 1 - R_x for a resonant field (the
 * part its output coupler passes; Eq. 6) or 1 for a non-resonant field (it
 * leaves the cavity whole). The idler entry is 0 for two waves. For an
 * on-axis Gaussian peak I = 2P / (pi w0^2), area_m2 = pi w0^2 / 2. OPO_EINVAL
 * for area_m2 <= 0 or a bad instance, capacity or pointer. */
int opo_get_power_history(opo_t *h, int32_t inst, double area_m2, double *out, int32_t capacity,
                          int32_t *rows);

/* Field `field` of instance `inst` as it left the crystal in round trip rt
 * (counted from opo_init; rt < record_rt and < the round trips run so far),
 * nt interleaved complex128 time samples, from the record of the record_rt
 * option. OPO_EINVAL for a round trip outside the record. */
int opo_get_record(opo_t *h, int32_t inst, int32_t field, int32_t rt, double *out);

/* Time samples t_j [ps] and angular frequencies w_k [rad/ps] of an instance. */
int opo_get_grid(opo_t *h, int32_t inst, double *t, double *omega);

/* The schedule instance `inst` runs (see opo_options_t.schedule): the four-step
 * split nt = n1 * n2 of its column and row tiles (log2 of each; the adaptive step
 * and the spectrum read-out use them for every instance), and whether its
 * fixed-step passes run resident (1) or as two passes per z-step (0). Any
 * output pointer may be NULL. OPO_EINVAL for a bad instance. */
int opo_get_plan(opo_t *h, int32_t inst, int32_t *log2_n1, int32_t *log2_n2, int32_t *resident);

/* Kernel classes timed by the profile option: column pass, row pass, energy
 * reduction, the mixed pass that runs the column tiles of one half of a batch
 * together with the row tiles of the other half, and the resident pass (under
 * the profile option it runs before the two-pass launches instead of beside
 * them). */
enum { OPO_K_COLUMN = 0, OPO_K_ROW = 1, OPO_K_ENERGY = 2, OPO_K_MIXED = 3, OPO_K_RESIDENT = 4, OPO_K_CLASSES = 5 };

/* Device time [ms] summed over launches, and launch counts, of each kernel
 * class since the handle was created (profile option), OPO_K_CLASSES
 * entries each; zeros without the profile option. */
int opo_kernel_times(opo_t *h, double *ms, int64_t *launches);

/* Number of instances, and the current z [mm] of the handle. */
int opo_info(opo_t *h, int32_t *n_instances, double *z_mm);

/* Release all device memory the library allocated, and the handle. */
int opo_destroy(opo_t *h);

/* Message of the last error on the calling thread ("" if none). */
const char *opo_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* OPO_H */
