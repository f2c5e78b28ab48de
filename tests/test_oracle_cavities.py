"""Pins of the oracle's pump-resonant cavities (pump-enhanced and triply resonant): the input
pump couples in through the pump mirror, A_p += sqrt(1 - R_p) A_in, at the start of every
round trip, and the circulating pump takes sqrt(R_p) e^{i delta_p} at its end."""
import numpy as np
import pytest

import oracle
from paper_2410_02532_amd import workloads as W


@pytest.mark.parametrize("refl, delta", [(0.9, 0.0), (0.6, 0.7)])
def test_empty_ring_fills_as_a_geometric_series(refl, delta):
    """No coupling, dispersion or loss: after the pass of round trip m the pump is
    sqrt(1-R) A_in sum_{k<=m} q^k, q = sqrt(R) e^{i delta}; the steady state is the
    ring-resonator enhancement sqrt(1-R) A_in / (1 - q)."""
    nt, nz, nrt = 16, 3, 60
    cr = W.crystal(nt, deff=0.0, db1=(0, 0, 0), b2=(0, 0, 0))
    cav = W.cavity(resonant=(1, 0, 0), refl=(refl, 0.0, 0.0), delta=(delta, 0.0, 0.0))
    a_in = 3.0e6 * np.exp(0.4j)
    a0 = np.zeros((3, nt), complex)
    a, e = oracle.roundtrips(cr, cav, a0, np.full(nt, a_in), nz, nrt)
    q = np.sqrt(refl) * np.exp(1j * delta)
    m = np.arange(nrt)
    amp = np.sqrt(1 - refl) * a_in * (1 - q ** (m + 1)) / (1 - q)
    assert np.allclose(e[:, 0], nt * np.abs(amp) ** 2, rtol=1e-12, atol=0)
    # the final state has had the mirror applied: q times the last pass output
    assert np.allclose(a[0], q * amp[-1], rtol=1e-12, atol=0)
    ss = np.sqrt(1 - refl) * a_in / (1 - q)
    assert abs(e[-1, 0] / (nt * abs(ss) ** 2) - 1) < 2 * abs(q) ** nrt


def test_pump_enhanced_threshold():
    """A singly resonant oscillator with a resonant pump (R_p = 0.8): the circulating pump
    is enhanced by sqrt(1-R_p)/(1 - sqrt(R_p)), so the input threshold is the plain SRO
    threshold divided by that factor. Uniform plane waves just below it decay, just above
    it grow."""
    nt, nz, refl_p, refl_s = 8, 10, 0.8, 0.95
    cr = W.crystal(nt, db1=(0, 0, 0), b2=(0, 0, 0))
    a_th = W.threshold_amplitude(cr, refl_s)
    enh = np.sqrt(1 - refl_p) / (1 - np.sqrt(refl_p))
    cav = W.cavity(resonant=(1, 1, 0), refl=(refl_p, refl_s, 0.0))
    growth = {}
    for f in (0.97, 1.03):
        a_in = f * a_th / enh
        ss = a_in * enh                       # start at the empty-cavity steady state:
        a0 = np.stack([np.full(nt, ss * np.sqrt(refl_p) + 0j),   # + sqrt(1-R_p) a_in = ss
                       np.full(nt, 1e-12 * a_th + 0j), np.zeros(nt, complex)])
        a, e = oracle.roundtrips(cr, cav, a0, np.full(nt, a_in + 0j), nz, 400)
        assert abs(e[0, 0] / (nt * ss * ss) - 1) < 1e-9     # pump already at steady state
        growth[f] = e[-1, 1] / e[1, 1]
    assert growth[0.97] < 0.5 and growth[1.03] > 2.0


def test_triply_resonant_round_trips_keep_the_input_coupler_in_the_history():
    """Triply resonant cavity from noise (all three fields fed back): a pass at round trip 0
    starts from the injected pump only."""
    nt, nz = 64, 5
    cr = W.crystal(nt)
    cav = W.cavity(resonant=(1, 1, 1), refl=(0.7, 0.9, 0.9))
    f = W.initial_fields(nt, 0.0, 1)
    f[0] = 0.0
    a_in = 2.0 * W.threshold_amplitude(cr, 0.9, 0.9)
    a, e = oracle.roundtrips(cr, cav, f, np.full(nt, a_in + 0j), nz, 3)
    b = oracle.ssfm_pass(cr, np.stack([np.full(nt, np.sqrt(0.3) * a_in + 0j), f[1], f[2]]), nz,
                         cr["length_mm"] / nz)
    assert np.allclose(e[0], np.sum(np.abs(b) ** 2, axis=1), rtol=1e-13)
