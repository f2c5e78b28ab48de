"""Pins of the oracle's nanosecond regime: a long input pump read one round-trip window at
a time, and the per-round-trip record of the fields leaving the crystal (Sec. 4.1, the
pump read and round-trip save steps of the main loop; Sec. 4, nanosecond example)."""
import numpy as np

import oracle
from paper_2410_02532_amd import workloads as W


def _sro(nt, **kw):
    cr = W.crystal(nt, **kw)
    cav = W.cavity(refl=(0.0, 0.9, 0.0))
    return cr, cav


def test_one_repeated_window_equals_plain_round_trips():
    nt, nz, nrt = 256, 10, 12
    w = W.config("sro_cw", nt=nt, nz=nz, level=4.0)
    a, e = oracle.roundtrips(w["crystal"], w["cavity"], w["fields"], w["pump_in"], nz, nrt)
    pump_long = np.tile(w["pump_in"], nrt)
    b, f, rec = oracle.roundtrips_record(w["crystal"], w["cavity"], w["fields"], pump_long, nz, nrt)
    assert np.array_equal(a, b) and np.array_equal(e, f)
    # the record holds the fields leaving the crystal: their energies are the history
    for m in range(nrt):
        for x in range(3):
            assert abs(np.sum(np.abs(rec[m, x]) ** 2) - e[m, x]) <= 1e-13 * e[m, x]


def test_windows_are_read_in_order_and_zero_after_the_last():
    """Without coupling or dispersion the pump leaves the crystal unchanged, so the record
    shows window m of the input at round trip m, then zeros."""
    nt, nz, windows, nrt = 64, 4, 5, 8
    cr, cav = _sro(nt, deff=0.0, db1=(0, 0, 0), b2=(0, 0, 0))
    g = np.random.Generator(np.random.PCG64(1))
    pump_long = (g.standard_normal((windows, nt)) + 1j * g.standard_normal((windows, nt))) * 1e6
    a0 = np.zeros((3, nt), complex)
    _, e, rec = oracle.roundtrips_record(cr, cav, a0, pump_long, nz, nrt)
    for m in range(nrt):
        ref = pump_long[m] if m < windows else np.zeros(nt)
        assert np.max(np.abs(rec[m, 0] - ref)) <= 1e-14 * 1e6 * 4, m
    assert np.all(e[windows:, 0] == 0.0)


def test_record_of_two_wave_instances():
    nt, nz, nrt = 128, 8, 6
    w = W.config("degenerate_cw", nt=nt, nz=nz, level=3.0, refl=0.8)
    pump_long = np.tile(w["pump_in"], nrt)
    a, e, rec = oracle.roundtrips_record(w["crystal"], w["cavity"], w["fields"], pump_long, nz, nrt)
    assert rec.shape == (nrt, 2, nt)
    a2, e2 = oracle.roundtrips(w["crystal"], w["cavity"], w["fields"], w["pump_in"], nz, nrt)
    assert np.array_equal(a, a2) and np.array_equal(e, e2)


def test_stronger_pulses_deplete_more_and_oscillate_earlier():
    """The paper's nanosecond example: the greater the pump power, the greater its depletion
    and the faster the signal rises. Degenerate oscillator at R = 0.5, pulses of 200 windows
    (intensity FWHM) peaking at 3, 4 and 10 times the CW threshold (the paper's 75, 100 and
    250 W ratios), a 1e-3 seed to keep the run short. Rise = first window whose signal energy
    exceeds 1 % of the peak pump window's."""
    nt, windows, refl = 32, 400, 0.5
    rise, depletion = [], []
    for level in (3.0, 4.0, 10.0):
        cr = W.crystal2(nt, db1=(0, 0, 0), b2=(0, 0, 0))
        peak = np.sqrt(level) * W.threshold_amplitude_degenerate(cr, refl)
        pump = W.long_pulse(nt, windows, peak, fwhm_ps=200 * 100.0)
        a0 = np.stack([pump[0], np.full(nt, 1e-3 * peak * np.exp(1j * np.pi / 4))])
        cav = W.cavity(refl=(0.0, refl, 0.0))
        _, e, rec = oracle.roundtrips_record(cr, cav, a0, pump, 10, windows)
        sig = e[:, 1]
        rise.append(int(np.argmax(sig > 0.01 * nt * peak * peak)))
        depletion.append(1.0 - e[:, 0].sum() / np.sum(np.abs(pump) ** 2))
    assert 0 < rise[2] < rise[1] < rise[0]
    assert 0.3 < depletion[0] < depletion[1] < depletion[2]
