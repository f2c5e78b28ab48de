"""Pins of the oracle's round trips through several crystals in sequence (each with its own
parameters, step count and z from its own entrance)."""
import numpy as np

import oracle
from paper_2410_02532_amd import workloads as W


def test_two_halves_equal_one_crystal_without_mismatch():
    """With dk = 0 nothing depends on where z starts, so two identical crystals of L/2 with
    nz/2 steps each give exactly one crystal of L with nz steps."""
    nt, nz, nrt = 256, 20, 6
    w = W.config("sro_cw", nt=nt, nz=nz, level=4.0)
    half = dict(w["crystal"], length_mm=0.5 * w["crystal"]["length_mm"])
    a1, e1 = oracle.roundtrips(w["crystal"], w["cavity"], w["fields"], w["pump_in"], nz, nrt)
    a2, e2, _ = oracle.roundtrips_multi([half, half], [nz // 2, nz // 2], w["cavity"], w["fields"],
                                        w["pump_in"], nrt)
    assert np.array_equal(a1, a2) and np.array_equal(e1, e2)


def test_opposite_dispersion_cancels():
    """Two passive crystals of equal length with opposite group-velocity mismatch, GVD and
    TOD restore the input field (dispersion compensation), up to FFT rounding."""
    nt = 512
    kw = dict(deff=0.0, db1=(0.3, 0.0, -0.2), b2=(400.0, 300.0, 200.0))
    c1 = W.crystal(nt, b3=(900.0, 500.0, 300.0), **kw)
    c2 = W.crystal(nt, deff=0.0, db1=(-0.3, 0.0, 0.2), b2=(-400.0, -300.0, -200.0),
                   b3=(-900.0, -500.0, -300.0))
    t = W.time_grid(nt)
    a = np.stack([np.exp(-t * t / 8.0) * (1 + 0.5j), np.exp(-(t - 3) ** 2 / 2.0) + 0j,
                  W.noise(nt, 0.3, 4)]) * 1e6
    cav = W.cavity(resonant=(1, 1, 1), refl=(1.0, 1.0, 1.0))
    mid = oracle.ssfm_pass(c1, a, 7, c1["length_mm"] / 7)
    assert np.linalg.norm(mid - a) > 0.1 * np.linalg.norm(a)          # the first one disperses
    out, e, _ = oracle.roundtrips_multi([c1, c2], [7, 9], cav, a, np.zeros(nt), 1)
    assert np.max(np.abs(out - a)) < 1e-12 * np.max(np.abs(a))


def test_cascade_is_the_composition_of_passes_each_from_its_entrance():
    """With mismatch the cascade is pass(c2) after pass(c1), each with z from 0, then the
    boundary; the energies after the last crystal are the history."""
    nt = 128
    c1 = W.crystal(nt, dk_per_mm=1.3, deff=30.0)
    c2 = W.crystal(nt, dk_per_mm=-0.7, deff=20.0, length_mm=3.0, b2=(100.0, 50.0, 80.0))
    g = np.random.Generator(np.random.PCG64(2))
    a = (g.standard_normal((3, nt)) + 1j * g.standard_normal((3, nt))) * np.array([[3e6], [1e5], [1e3]])
    cav = W.cavity(resonant=(1, 1, 1), refl=(1.0, 1.0, 1.0))
    out, e, rec = oracle.roundtrips_multi([c1, c2], [10, 6], cav, a, np.zeros(nt), 1, record=True)
    ref = oracle.ssfm_pass(c2, oracle.ssfm_pass(c1, a, 10, c1["length_mm"] / 10), 6, 0.5)
    assert np.array_equal(rec[0], ref)
    assert np.allclose(e[0], np.sum(np.abs(ref) ** 2, axis=1), rtol=1e-13)
