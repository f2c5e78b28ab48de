"""Pins of the oracle's two-wave (degenerate) model against closed forms and the paper.

At degeneracy (signal = idler) the paper solves two coupled waves. It prints
the signal equation dA_s/dz = i kappa_s A_p A_s^* (Sec. 2.4, step-size
discussion) and leaves the pump equation unprinted; the oracle takes
dA_p/dz = i kappa_p2 A_s^2 e^{-i dk z} with kappa_p2 = 2 pi d_eff/(n_p lambda_s).
Pins: the power invariant that fixes kappa_p2, the undepleted phase-sensitive
gain (with and without phase mismatch), the depleted tanh/sech solution, the
reduction of the three-wave model with A_i = A_s, and two results the paper
reports for the degenerate CW oscillator (Sec. 4, two-CWE example): the signal
phase settles at pi/4 or -3pi/4, and the pump depletion peaks at N = 4.
"""
import numpy as np
import pytest

import oracle
from paper_2410_02532_amd import workloads as W

LP, LS = 0.532, 1.064


def crystal2(nt, **kw):
    kw.setdefault("lambdas", (LP, LS, LS))
    c = W.crystal(nt, **kw)
    c["nf"] = 2
    return c


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _power(c, a):
    return c["n"][0] * np.sum(np.abs(a[0]) ** 2) + c["n"][1] * np.sum(np.abs(a[1]) ** 2)


def test_kappa_two_wave():
    c = crystal2(8, n=(2.2, 2.1, 2.1))
    k = oracle.kappa(c)
    two_pi_d = 2 * np.pi * c["deff_pm_per_v"] * 1e-9
    assert k[0] == pytest.approx(two_pi_d / (2.2 * LS), rel=1e-15)
    assert k[1] == pytest.approx(two_pi_d / (2.1 * LS), rel=1e-15)
    assert k[2] == 0.0
    # at lambda_s = 2 lambda_p the pump coefficient is half the three-wave kappa_p
    assert k[0] == pytest.approx(0.5 * two_pi_d / (2.2 * LP), rel=1e-15)


@pytest.mark.parametrize("dk", [0.0, 3.0])
def test_power_invariant(dk):
    """n_p|A_p|^2 + n_s|A_s|^2 is conserved by the coupled equations for any dk (the
    property that fixes the unprinted pump coefficient); RK4 keeps it to its
    truncation error, and the lossless linear step is unitary."""
    nt = 64
    c = crystal2(nt, dk_per_mm=dk, n=(2.2, 2.1, 2.1))
    g = _rng(5)
    ap = 4e7
    a = np.stack([ap * (1 + 0.3 * g.standard_normal(nt)) + 0j,
                  0.5 * ap * (g.standard_normal(nt) + 1j * g.standard_normal(nt))])
    p0 = _power(c, a)
    b = oracle.rk4(c, a, 0.3, 0.01)                     # kappa A h ~ 0.016
    assert abs(_power(c, b) / p0 - 1) < 1e-10
    assert np.max(np.abs(b - a)) > 1e-3 * ap           # the step did something
    b = oracle.ssfm_pass(c, a, 200, 0.025)      # kappa A h ~ 0.02: RK4 drift ~1e-9
    assert abs(_power(c, b) / p0 - 1) < 1e-8
    # a pump coefficient of kappa_p (instead of kappa_p/2) would break it: halving n_p
    # doubles kappa_p2, and the same invariant then drifts
    c_bad = dict(c, n=(1.1, 2.1, 2.1))
    b = oracle.rk4(c_bad, a, 0.3, 0.01)
    assert abs(_power(c, b) / p0 - 1) > 1e-4


@pytest.mark.parametrize("dk", [0.0, 0.2, 0.8])
def test_undepleted_phase_sensitive_gain(dk):
    """Weak signal, real pump A_p, G = kappa_s A_p, d = dk/2, g = sqrt(G^2 - d^2):
    A_s(z) = e^{i d z} [A0 (cosh gz - i d/g sinh gz) + i G/g A0^* sinh gz]
    (oscillatory for d > G, where g is imaginary)."""
    nt = 8
    c = crystal2(nt, dk_per_mm=dk, db1=(0, 0, 0), b2=(0, 0, 0))
    k = oracle.kappa(c)
    ap = 1.0 / (k[1] * c["length_mm"])                  # G L = 1
    g = _rng(7)
    a0 = 1e-7 * ap * (g.standard_normal(nt) + 1j * g.standard_normal(nt))
    a = np.stack([np.full(nt, ap + 0j), a0])
    L = c["length_mm"]
    out = oracle.ssfm_pass(c, a, 400, L / 400)
    G = k[1] * ap
    d = 0.5 * dk
    gg = np.sqrt(complex(G * G - d * d))
    ref = np.exp(1j * d * L) * (a0 * (np.cosh(gg * L) - 1j * d / gg * np.sinh(gg * L))
                                + 1j * G / gg * np.conj(a0) * np.sinh(gg * L))
    assert np.max(np.abs(out[1] - ref)) / np.max(np.abs(ref)) < 1e-9
    assert np.max(np.abs(out[0] - ap)) / ap < 1e-12     # pump undepleted


def test_depleted_tanh_sech():
    """dk = 0, real pump p0, signal e^{i pi/4} s0: with q = sqrt(kappa_p2/kappa_s) s,
    R^2 = p0^2 + q0^2 and c = atanh(p0/R): p = R tanh(c - kappa_s R z),
    q = R sech(c - kappa_s R z). The run goes through full conversion."""
    nt = 4
    c = crystal2(nt, db1=(0, 0, 0), b2=(0, 0, 0))
    k = oracle.kappa(c)
    L = c["length_mm"]
    p0 = 12.0 / (k[1] * L)
    s0 = 1e-3 * p0
    a = np.stack([np.full(nt, p0 + 0j), np.full(nt, s0 * np.exp(1j * np.pi / 4))])
    nz = 4000
    out = oracle.ssfm_pass(c, a, nz, L / nz)
    r = np.sqrt(k[0] / k[1])
    q0 = r * s0
    R = np.hypot(p0, q0)
    arg = np.arctanh(p0 / R) - k[1] * R * L
    p_ref = R * np.tanh(arg)
    s_ref = R / np.cosh(arg) / r
    assert arg < -1.0                                   # past the conversion point
    assert np.max(np.abs(out[0] - p_ref)) / p0 < 1e-8
    assert np.max(np.abs(out[1] - s_ref * np.exp(1j * np.pi / 4))) / (R / r) < 1e-8


def test_three_wave_with_equal_signal_and_idler_reduces_to_two_wave():
    """With lambda_s = lambda_i = 2 lambda_p and identical signal/idler parameters, the
    three-wave model started from A_s = A_i = A/sqrt(2) keeps A_s = A_i and equals the
    two-wave model started from A: A_s(3) = A(2)/sqrt(2) at every z."""
    nt = 128
    kw = dict(lambdas=(LP, LS, LS), db1=(0.2, 0.0, 0.0), b2=(250.0, 150.0, 150.0),
              dk_per_mm=0.5, n=(2.2, 2.1, 2.1))
    c3 = W.crystal(nt, **kw)
    c2 = crystal2(nt, **kw)
    g = _rng(11)
    ap = 3e7
    pump = ap * np.exp(-((np.arange(nt) - nt / 2) / 20.0) ** 2) + 0j
    sig = 0.2 * ap * (g.standard_normal(nt) + 1j * g.standard_normal(nt))
    o3 = oracle.ssfm_pass(c3, np.stack([pump, sig / np.sqrt(2), sig / np.sqrt(2)]), 100, 0.05)
    o2 = oracle.ssfm_pass(c2, np.stack([pump, sig]), 100, 0.05)
    scale = np.max(np.abs(o2))
    assert np.max(np.abs(o3[0] - o2[0])) / scale < 1e-13
    assert np.max(np.abs(np.sqrt(2) * o3[1] - o2[1])) / scale < 1e-13
    assert np.max(np.abs(o3[1] - o3[2])) / scale < 1e-14


def _threshold_amplitude(c, refl):
    """Degenerate, single resonant field, dk = 0, no dispersion, undepleted: the
    in-phase quadrature gains e^{G L} per pass, so sqrt(R) e^{G_th L} = 1."""
    k = oracle.kappa(c)
    return -0.5 * np.log(refl) / c["length_mm"] / k[1]


def test_pump_depletion_peaks_at_four_times_threshold():
    """The paper's degenerate CW example: pump depletion is largest at N = 4. Plane-wave
    uniform fields at R = 0.98 settle to the mean-field result
    1 - (2 - sqrt(N))^2 / N, which is 1 at N = 4."""
    nt = 4
    refl = 0.98
    c = crystal2(nt, db1=(0, 0, 0), b2=(0, 0, 0))
    cav = W.cavity(resonant=(0, 1, 0), refl=(0.0, refl, 0.0))
    ath = _threshold_amplitude(c, refl)
    dep = {}
    for n_level in (2.0, 3.0, 4.0, 5.0, 6.0):
        ap = np.sqrt(n_level) * ath
        a = np.stack([np.full(nt, ap + 0j), np.full(nt, 1e-3 * ap * np.exp(1j * np.pi / 4))])
        a, e = oracle.roundtrips(c, cav, a, np.full(nt, ap + 0j), 20, 4000)
        assert abs(e[-1, 1] / e[-2, 1] - 1) < 1e-8      # steady state
        dep[n_level] = 1 - e[-1, 0] / (nt * ap * ap)
        mean_field = 1 - (2 - np.sqrt(n_level)) ** 2 / n_level
        assert abs(dep[n_level] - mean_field) < 3e-3, (n_level, dep[n_level], mean_field)
        assert np.allclose(np.angle(a[1]), np.pi / 4, atol=1e-9)
    assert max(dep, key=dep.get) == 4.0
    assert dep[4.0] > 0.9999


def test_signal_phase_states_from_noise():
    """From the seeded noise, with dispersion, the degenerate signal locks to the two
    phase states pi/4 and -3pi/4 of a real pump (paper, two-CWE CW example)."""
    nt = 128
    refl = 0.90
    c = crystal2(nt)
    cav = W.cavity(resonant=(0, 1, 0), refl=(0.0, refl, 0.0))
    ap = np.sqrt(3.0) * _threshold_amplitude(c, refl)
    f = W.initial_fields(nt, ap, 1000)
    a, e = oracle.roundtrips(c, cav, np.stack([f[0], f[1]]), np.full(nt, ap + 0j), 40, 1200)
    assert e[-1, 1] > 1e20 * e[0, 1]                    # oscillating
    mag = np.abs(a[1])
    ph = np.angle(a[1][mag > 0.5 * mag.max()])
    d1 = np.abs(np.angle(np.exp(1j * (ph - np.pi / 4))))
    d2 = np.abs(np.angle(np.exp(1j * (ph + 3 * np.pi / 4))))
    assert np.all(np.minimum(d1, d2) < 0.03)
    assert ph.size >= 8
