"""Seeded synthetic workloads shared by the tests, the benchmark and the smoke check.

This module only *describes* inputs: crystal/cavity parameter dicts, initial
fields and input-pump arrays, built from numpy's PCG64 generator with fixed
seeds. It contains none of the propagation arithmetic; both the GPU library
and the CPU oracle receive the arrays it returns.

Recipe (synthetic stand-ins for the paper's workloads, arXiv 2410.02532):
  * crystal: 5 mm long, lambda_p = 1.064 um, lambda_s = 1.6 um, idler from
    energy conservation (Sec. 2.1, Eq. 1 with dk = 0), n = 2.2 for all fields,
    d_eff = 14 pm/V, group-velocity mismatch (+0.2, 0, -0.1) ps/mm relative to
    the signal, GVD (250, 150, 100) fs^2/mm, TOD 0 (500 fs^3/mm for the
    synchronously pumped case), no loss;
  * grid: T = 100 ps window (round-trip time of the paper's examples, Sec. 2.4),
    Nt a power of two (Sec. 2.4 uses 2^10 .. 2^15);
  * pump: CW of amplitude A_p0 everywhere, or a Gaussian pulse; field from
    power through the on-axis peak intensity of a Gaussian beam,
    I = 2P/(pi w0^2), |A|^2 = 2I/(n eps0 c);
  * signal and idler start as complex Gaussian noise of relative amplitude
    1e-20: A(t_j) = 1e-20 A_p0 (g1 + i g2)/sqrt(2), g ~ N(0, 1) (the paper seeds
    the resonant fields with random amplitude and phase, Sec. 4.2-4.4);
  * pump level in units of the oscillation threshold N = P/P_th, where P_th is
    the plane-wave, dispersionless, undepleted threshold: SRO
    cosh(G L) = 1/sqrt(R_s), DRO cosh(G L) = (1 + sqrt(R_s R_i))/(sqrt(R_s) + sqrt(R_i)),
    with G^2 = k_s k_i |A_p|^2. This only chooses the input amplitude;
  * degenerate (two-wave) workloads: lambda_p = 0.532 um, lambda_s = 1.064 um
    (the paper's degenerate examples), other crystal values as above; the
    in-phase signal quadrature gains e^{G L} per pass with G = k_s |A_p|, so
    the threshold is sqrt(R_s) e^{G L} = 1 (N = P/P_th as above);
  * nanosecond regime: a 10 ns (intensity FWHM) Gaussian pump spread over
    consecutive round-trip windows of T = 100 ps (one window per round trip),
    centred in the record; the paper's peak powers 75, 100 and 250 W keep
    their ratios as peak levels of 3, 4 and 10 times the CW threshold at
    R_s = 0.5 (the beam size that would fix the absolute scale is not printed).
"""
import math

import numpy as np

EPS0 = 8.8541878128e-12
C0 = 299792458.0

LAMBDA_P_UM = 1.064
LAMBDA_S_UM = 1.6
LAMBDA_I_UM = 1.0 / (1.0 / LAMBDA_P_UM - 1.0 / LAMBDA_S_UM)
LAMBDA_P_DEG_UM = 0.532
LAMBDA_S_DEG_UM = 1.064

T_WINDOW_PS = 100.0
LENGTH_MM = 5.0
N_INDEX = 2.2
DEFF_PM_PER_V = 14.0
NOISE_REL = 1e-20


def crystal(nt, b3=0.0, t_window_ps=T_WINDOW_PS, length_mm=LENGTH_MM, dk_per_mm=0.0,
            db1=(0.2, 0.0, -0.1), b2=(250.0, 150.0, 100.0), alpha=(0.0, 0.0, 0.0),
            n=(N_INDEX, N_INDEX, N_INDEX), deff=DEFF_PM_PER_V,
            lambdas=(LAMBDA_P_UM, LAMBDA_S_UM, LAMBDA_I_UM)):
    """Crystal parameter dict in the units the oracle and the library take."""
    return dict(nt=int(nt), t_window_ps=float(t_window_ps), length_mm=float(length_mm),
                lambda_um=tuple(float(v) for v in lambdas), n=tuple(float(v) for v in n),
                deff_pm_per_v=float(deff), dk_per_mm=float(dk_per_mm),
                alpha_per_mm=tuple(float(v) for v in alpha),
                db1_ps_per_mm=tuple(float(v) for v in db1),
                b2_fs2_per_mm=tuple(float(v) for v in b2),
                b3_fs3_per_mm=(float(b3),) * 3 if np.isscalar(b3) else tuple(b3))


def cavity(resonant=(0, 1, 0), refl=(0.0, 0.98, 0.0), delta=(0.0, 0.0, 0.0), gdd_fs2=0.0,
           gdd_on=None, eom_beta=0.0, eom_fpm_thz=0.0, eom_on=None):
    """Cavity dict; GDD and EOM act on the resonant fields unless masks are given."""
    res = tuple(int(bool(r)) for r in resonant)
    return dict(resonant=res, refl=tuple(float(r) for r in refl),
                delta_rad=tuple(float(d) for d in delta), gdd_fs2=float(gdd_fs2),
                gdd_on=res if gdd_on is None else tuple(int(bool(g)) for g in gdd_on),
                eom_beta=float(eom_beta), eom_fpm_thz=float(eom_fpm_thz),
                eom_on=res if eom_on is None else tuple(int(bool(g)) for g in eom_on))


def field_from_power(power_w, waist_um, n=N_INDEX):
    """|A| [V/m] of a Gaussian beam's on-axis peak for power P and waist w0."""
    w0 = waist_um * 1e-6
    intensity = 2.0 * power_w / (math.pi * w0 * w0)
    return math.sqrt(2.0 * intensity / (n * EPS0 * C0))


def coupling_product(cr):
    """k_s k_i in (1/mm per V/m)^2 for the threshold recipe."""
    k = [2.0 * math.pi * cr["deff_pm_per_v"] / (cr["n"][x] * cr["lambda_um"][x]) * 1e-9
         for x in (1, 2)]
    return k[0] * k[1]


def threshold_amplitude(cr, refl_s, refl_i=None):
    """Pump amplitude at the plane-wave SRO (refl_i None) or DRO threshold."""
    if refl_i is None:
        target = 1.0 / math.sqrt(refl_s)
    else:
        target = (1.0 + math.sqrt(refl_s * refl_i)) / (math.sqrt(refl_s) + math.sqrt(refl_i))
    gl = math.acosh(target)
    return gl / (cr["length_mm"] * math.sqrt(coupling_product(cr)))


def crystal2(nt, **kw):
    """Two-wave (degenerate) crystal dict: pump 0.532 um, signal 1.064 um."""
    kw.setdefault("lambdas", (LAMBDA_P_DEG_UM, LAMBDA_S_DEG_UM, LAMBDA_S_DEG_UM))
    cr = crystal(nt, **kw)
    cr["nf"] = 2
    return cr


def threshold_amplitude_degenerate(cr, refl_s):
    """Pump amplitude at the plane-wave threshold of the degenerate oscillator."""
    k_s = 2.0 * math.pi * cr["deff_pm_per_v"] / (cr["n"][1] * cr["lambda_um"][1]) * 1e-9
    return -0.5 * math.log(refl_s) / (cr["length_mm"] * k_s)


def long_pulse(nt, n_windows, peak, fwhm_ps, t_window_ps=T_WINDOW_PS):
    """A Gaussian pump e^{-t^2/(2 T0^2)} (intensity FWHM fwhm_ps) sampled over n_windows
    consecutive windows of nt points, centred in the record; shape (n_windows, nt)."""
    t0 = fwhm_ps / (2.0 * math.sqrt(math.log(2.0)))
    centre = 0.5 * n_windows * t_window_ps
    t = (np.arange(n_windows)[:, None] + 0.5) * t_window_ps + time_grid(nt, t_window_ps)[None, :]
    return peak * np.exp(-(t - centre) ** 2 / (2.0 * t0 * t0)) + 0j


def noise(nt, amplitude, seed):
    """Complex Gaussian noise amplitude*(g1 + i g2)/sqrt(2) from PCG64(seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    g = rng.standard_normal((2, nt))
    return amplitude * (g[0] + 1j * g[1]) / math.sqrt(2.0)


def time_grid(nt, t_window_ps=T_WINDOW_PS):
    return -0.5 * t_window_ps + np.arange(nt) * (t_window_ps / nt)


def gaussian_pulse(nt, peak, fwhm_ps, t_window_ps=T_WINDOW_PS):
    """Field e^{-t^2/(2 T0^2)} with an intensity FWHM of fwhm_ps, centred."""
    t0 = fwhm_ps / (2.0 * math.sqrt(math.log(2.0)))
    t = time_grid(nt, t_window_ps)
    return peak * np.exp(-t * t / (2.0 * t0 * t0)) + 0j


def initial_fields(nt, pump, seed):
    """Stack (pump, signal noise, idler noise) with the 1e-20 relative seed."""
    pump = np.broadcast_to(np.asarray(pump, dtype=np.complex128), (nt,))
    amp = NOISE_REL * float(np.max(np.abs(pump)))
    a = np.empty((3, nt), dtype=np.complex128)
    a[0] = pump
    a[1] = noise(nt, amp, seed)
    a[2] = noise(nt, amp, seed + 7919)
    return a


def config(name, **over):
    """Workload dict for one named configuration.

    Keys: crystal, cavity, nz, n_rt, fields (nf, nt) complex128, pump_in (nt,),
    precision ('f32' or 'f64'), instances (list of such dicts for batches).
    """
    if name == "single_pass":          # one pass, no cavity, Nt = 2^10, complex128
        nt = over.get("nt", 1 << 10)
        cr = crystal(nt)
        ap0 = field_from_power(10.0, 30.0)
        return dict(name=name, crystal=cr, cavity=cavity(resonant=(0, 0, 0), refl=(0, 0, 0)),
                    nz=over.get("nz", 100), n_rt=0, fields=initial_fields(nt, ap0, 1000),
                    pump_in=np.full(nt, ap0 + 0j), precision="f64")
    if name == "sro_cw":               # CW singly resonant OPO, Nt = 2^14, 2000 round trips
        nt = over.get("nt", 1 << 14)
        level = over.get("level", 3.0)
        cr = crystal(nt)
        ap0 = math.sqrt(level) * threshold_amplitude(cr, 0.98)
        return dict(name=name, crystal=cr, cavity=cavity(),
                    nz=over.get("nz", 100), n_rt=over.get("n_rt", 2000),
                    fields=initial_fields(nt, ap0, over.get("seed", 1000)),
                    pump_in=np.full(nt, ap0 + 0j), precision=over.get("precision", "f32"))
    if name == "sync_pumped":          # 2 ps Gaussian pump, TOD, Nt = 2^16..2^18
        nt = over.get("nt", 1 << 16)
        cr = crystal(nt, b3=500.0)
        peak = 2.0 * threshold_amplitude(cr, 0.98)   # peak power 4x the CW threshold
        pump = gaussian_pulse(nt, peak, 2.0)
        return dict(name=name, crystal=cr, cavity=cavity(),
                    nz=over.get("nz", 100), n_rt=over.get("n_rt", 1000),
                    fields=initial_fields(nt, pump, over.get("seed", 1000)),
                    pump_in=pump, precision=over.get("precision", "f32"))
    if name == "batched_sweep":        # 256 uneven-Nt CW SROs
        count = over.get("count", 256)
        rng = np.random.Generator(np.random.PCG64(3))
        sizes = 1 << rng.integers(over.get("min_log2", 12), over.get("max_log2", 16) + 1,
                                  size=count)
        levels = rng.uniform(1.0, 6.0, size=count)
        deltas = rng.uniform(-0.5, 0.5, size=count)
        refls = rng.uniform(0.90, 0.99, size=count)
        inst = []
        for b in range(count):
            nt = int(sizes[b])
            cr = crystal(nt)
            ap0 = math.sqrt(levels[b]) * threshold_amplitude(cr, refls[b])
            inst.append(dict(crystal=cr,
                             cavity=cavity(refl=(0.0, refls[b], 0.0), delta=(0.0, deltas[b], 0.0)),
                             fields=initial_fields(nt, ap0, 1000 + b),
                             pump_in=np.full(nt, ap0 + 0j)))
        return dict(name=name, instances=inst, nz=over.get("nz", 100),
                    n_rt=over.get("n_rt", 500), precision="f32", levels=levels.tolist())
    if name == "small_sweep":          # the batched sweep over the paper's small grids 2^10..2^12
        w = config("batched_sweep", **dict(dict(min_log2=10, max_log2=12), **over))
        w["name"] = name
        return w
    if name == "degenerate_cw":        # two-wave degenerate CW oscillator, Nt = 2^14
        nt = over.get("nt", 1 << 14)
        level = over.get("level", 3.0)
        refl = over.get("refl", 0.98)
        cr = crystal2(nt)
        ap0 = math.sqrt(level) * threshold_amplitude_degenerate(cr, refl)
        f = initial_fields(nt, ap0, over.get("seed", 1000))
        return dict(name=name, crystal=cr, cavity=cavity(refl=(0.0, refl, 0.0)),
                    nz=over.get("nz", 100), n_rt=over.get("n_rt", 2000), fields=f[:2].copy(),
                    pump_in=np.full(nt, ap0 + 0j), precision=over.get("precision", "f32"))
    if name == "degenerate_sweep":     # 256 uneven-Nt two-wave degenerate oscillators
        count = over.get("count", 256)
        rng = np.random.Generator(np.random.PCG64(4))
        sizes = 1 << rng.integers(over.get("min_log2", 12), over.get("max_log2", 16) + 1,
                                  size=count)
        levels = rng.uniform(1.0, 6.0, size=count)
        deltas = rng.uniform(-0.5, 0.5, size=count)
        refls = rng.uniform(0.90, 0.99, size=count)
        inst = []
        for b in range(count):
            nt = int(sizes[b])
            cr = crystal2(nt)
            ap0 = math.sqrt(levels[b]) * threshold_amplitude_degenerate(cr, refls[b])
            f = initial_fields(nt, ap0, 2000 + b)
            inst.append(dict(crystal=cr,
                             cavity=cavity(refl=(0.0, refls[b], 0.0), delta=(0.0, deltas[b], 0.0)),
                             fields=f[:2].copy(), pump_in=np.full(nt, ap0 + 0j)))
        return dict(name=name, instances=inst, nz=over.get("nz", 100),
                    n_rt=over.get("n_rt", 500), precision="f32")
    if name == "ns_pulsed":            # degenerate OPO pumped by 10 ns pulses, window per RT
        nt = over.get("nt", 1 << 12)
        windows = over.get("windows", 400)
        refl = over.get("refl", 0.5)
        levels = over.get("levels", (3.0, 4.0, 10.0))
        inst = []
        for b, level in enumerate(levels):
            cr = crystal2(nt)
            peak = math.sqrt(level) * threshold_amplitude_degenerate(cr, refl)
            pump = long_pulse(nt, windows, peak, over.get("fwhm_ps", 10000.0))
            f = initial_fields(nt, peak, 3000 + b)
            f[0] = pump[0]
            inst.append(dict(crystal=cr, cavity=cavity(refl=(0.0, refl, 0.0)),
                             fields=f[:2].copy(), pump_in=pump))
        return dict(name=name, instances=inst, nz=over.get("nz", 100),
                    n_rt=over.get("n_rt", windows), precision="f32")
    if name == "adaptive_pulsed":      # uneven-Nt single-pass amplifiers under the adaptive step
        count = over.get("count", 128)
        rng = np.random.Generator(np.random.PCG64(5))
        sizes = 1 << rng.integers(over.get("min_log2", 12), over.get("max_log2", 16) + 1,
                                  size=count)
        gains = rng.uniform(3.0, 8.0, size=count)        # small-signal gain-length at the peak
        dks = rng.uniform(-1.0, 1.0, size=count)
        inst = []
        for b in range(count):
            nt = int(sizes[b])
            cr = crystal(nt, b3=500.0, dk_per_mm=float(dks[b]))
            peak = gains[b] / (cr["length_mm"] * math.sqrt(coupling_product(cr)))
            pump = gaussian_pulse(nt, peak, 2.0)
            f = initial_fields(nt, pump, 4000 + b)
            f[1] += gaussian_pulse(nt, 1e-3 * peak, 1.0)
            inst.append(dict(crystal=cr, cavity=cavity(resonant=(0, 0, 0), refl=(0.0, 0.0, 0.0)),
                             fields=f, pump_in=pump))
        return dict(name=name, instances=inst, nz=over.get("nz", 100), n_rt=0,
                    tol=over.get("tol", 1e-5), precision="f32")
    if name == "dro_large":            # DRO, Nt = 2^20, GDD +-2000 fs^2, EOM 1 rad at 1/T
        nt = over.get("nt", 1 << 20)
        count = over.get("count", 16)
        inst = []
        for b in range(count):
            cr = crystal(nt)
            ap0 = math.sqrt(3.0) * threshold_amplitude(cr, 0.98, 0.98)
            cav = cavity(resonant=(0, 1, 1), refl=(0.0, 0.98, 0.98),
                         gdd_fs2=2000.0 if b < count // 2 else -2000.0,
                         eom_beta=1.0, eom_fpm_thz=1.0 / T_WINDOW_PS)
            inst.append(dict(crystal=cr, cavity=cav, fields=initial_fields(nt, ap0, 1000 + b),
                             pump_in=np.full(nt, ap0 + 0j)))
        return dict(name=name, instances=inst, nz=over.get("nz", 200),
                    n_rt=over.get("n_rt", 500), precision="f32")
    raise KeyError(name)
