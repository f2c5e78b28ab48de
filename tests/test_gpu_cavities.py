"""Parity of the HIP path's pump-resonant cavities (pump-enhanced and triply resonant) with
the FP64 oracle: the input pump couples in through the pump mirror every round trip."""
import sys

import numpy as np
import pytest

import torch  # noqa: F401  (imported at collection: the first import can take minutes)

import oracle
from paper_2410_02532_amd import opo as B
from paper_2410_02532_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL_E = {"f64": 1e-10, "f32": 1e-3}


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _check_energies(e, e_ref, tol, fields=(0, 1, 2)):
    for x in fields:
        live = e_ref[:, x] > 0.0
        assert np.max(np.abs(e[live, x] - e_ref[live, x]) / e_ref[live, x]) <= tol, x


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_empty_ring_pump_enhancement(precision):
    """No coupling, dispersion or loss, detuned pump resonance: the circulating pump fills as
    the geometric series of the input coupler."""
    nt, nz, nrt = 256, 4, 80
    cr = W.crystal(nt, deff=0.0)
    cav = W.cavity(resonant=(1, 0, 0), refl=(0.85, 0.0, 0.0), delta=(0.3, 0.0, 0.0))
    a0 = np.zeros((3, nt), complex)
    t = W.time_grid(nt)
    pump = 2e6 * np.exp(-t * t / (2 * 20.0 ** 2)) + 0j
    ins = dict(crystal=cr, cavity=cav, fields=a0, pump_in=pump)
    ref, e_ref = oracle.roundtrips(cr, cav, a0, pump, nz, nrt)
    with B.Opo([ins], nz, precision=precision) as h:
        h.cavity_roundtrip(nrt)
        e = h.energy_history()
        got = h.get_fields()
    _check_energies(e, e_ref, TOL_E[precision], fields=(0,))
    assert np.linalg.norm(got[0] - ref[0]) / np.linalg.norm(ref[0]) <= (1e-11 if precision == "f64" else 1e-4)


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_triply_resonant_oscillator(precision):
    """Pump, signal and idler all resonant (R = 0.7, 0.9, 0.9), input at twice the DRO
    threshold, from the noise seed: 200 round trips through build-up and saturation."""
    say("TRO", precision)
    nt, nz, nrt = 1024, 20, 200
    cr = W.crystal(nt)
    cav = W.cavity(resonant=(1, 1, 1), refl=(0.7, 0.9, 0.9))
    a_in = 2.0 * W.threshold_amplitude(cr, 0.9, 0.9)
    f = W.initial_fields(nt, a_in, 7)
    f[0] = 0.0
    ins = dict(crystal=cr, cavity=cav, fields=f, pump_in=np.full(nt, a_in + 0j))
    ref, e_ref = oracle.roundtrips(cr, cav, f, ins["pump_in"], nz, nrt)
    assert e_ref[-1, 1] > 1e30 * e_ref[0, 1]         # oscillates within the run
    with B.Opo([ins], nz, precision=precision) as h:
        h.cavity_roundtrip(nrt)
        e = h.energy_history()
    _check_energies(e, e_ref, TOL_E[precision])


def test_pump_enhanced_batch_equals_singles_and_oracle():
    """Pump-enhanced singly resonant instances of several sizes in one batch (mixed schedule):
    each equals its own single run bit for bit, and the oracle."""
    say("pump-enhanced batch")
    insts = []
    for b, nt in enumerate([4096, 8192, 4096, 16384]):
        w = W.config("sro_cw", nt=nt, level=2.0)
        cav = W.cavity(resonant=(1, 1, 0), refl=(0.6 + 0.05 * b, 0.95, 0.0), delta=(0.1 * b, 0.0, 0.0))
        f = w["fields"].copy()
        f[0] = 0.0
        insts.append(dict(crystal=w["crystal"], cavity=cav, fields=f, pump_in=w["pump_in"]))
    nz, nrt = 6, 4
    with B.Opo(insts, nz, precision="f32", schedule="two_pass") as hb:
        hb.cavity_roundtrip(nrt)
        batch = [(hb.get_fields(i), hb.energy_history(i)) for i in range(len(insts))]
    for i, ins in enumerate(insts):
        with B.Opo([ins], nz, precision="f32", schedule="two_pass") as h:
            h.cavity_roundtrip(nrt)
            assert np.array_equal(batch[i][0], h.get_fields())
            assert np.array_equal(batch[i][1], h.energy_history())
        _, e_ref = oracle.roundtrips(ins["crystal"], ins["cavity"], ins["fields"], ins["pump_in"], nz, nrt)
        _check_energies(batch[i][1], e_ref, TOL_E["f32"])
