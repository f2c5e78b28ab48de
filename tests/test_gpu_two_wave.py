"""Parity of the HIP path's two-wave (degenerate) model with the FP64 oracle.

Same bars as the three-wave path: complex128 to 1e-11 relative L2 per field and
pass or run of round trips, complex64 to 1e-4 and 1e-3 in round-trip energies. Two-wave
instances share launches with three-wave ones; each instance of such a batch
equals its own single-instance run bit for bit.
"""
import sys

import numpy as np
import pytest

import torch  # noqa: F401  (imported at collection: the first import can take minutes)

import oracle
from paper_2410_02532_amd import opo as B
from paper_2410_02532_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-11, "f32": 1e-4}
TOL_E = {"f64": 1e-10, "f32": 1e-3}


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def rel_l2(got, ref):
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))


def _stress2(nt, seed=0, t_window=40.0, dk=0.4):
    """Pulsed pump, seeded signal, mismatch, loss, GVM, GVD and TOD on both waves."""
    cr = W.crystal2(nt, t_window_ps=t_window, deff=60.0, b3=(300.0, -150.0, 0.0), dk_per_mm=dk,
                    alpha=(0.02, 0.01, 0.0), db1=(0.25, 0.0, 0.0), b2=(250.0, 150.0, 0.0),
                    n=(2.25, 2.2, 2.2))
    t = W.time_grid(nt, t_window)
    pump = 2.0e6 * np.exp(-t * t / (2 * (0.2 * t_window) ** 2)) * np.exp(0.3j)
    a = np.empty((2, nt), complex)
    a[0] = pump
    a[1] = 3.0e5 * np.exp(-(t - 1.0) ** 2 / (2 * (0.1 * t_window) ** 2)) + W.noise(nt, 1e3, seed + 1)
    cav = W.cavity(resonant=(0, 1, 0), refl=(0.0, 0.9, 0.0), delta=(0.0, 0.2, 0.0))
    return dict(crystal=cr, cavity=cav, fields=a, pump_in=pump)


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("nt", [2, 8, 512, 1 << 12, 1 << 14, 1 << 16])
def test_two_wave_pass_parity(nt, precision):
    say("two-wave pass parity nt=%d %s" % (nt, precision))
    ins = _stress2(nt, seed=nt)
    nz, dz = 20, 0.25
    ref = oracle.ssfm_pass(ins["crystal"], ins["fields"], nz, dz)
    with B.Opo([ins], nz, precision=precision) as h:
        h.ssfm_propagate(nz, dz)
        got = h.get_fields()
    assert got.shape == (2, nt)
    for x in range(2):
        assert rel_l2(got[x], ref[x]) <= TOL[precision], (x, rel_l2(got[x], ref[x]))


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_degenerate_oscillator_round_trips(precision):
    """The degenerate CW oscillator from noise (Nt = 2^10, 4x threshold, R = 0.7): energies
    of 300 round trips through the exponential build-up into the depleted steady state, and
    the final signal modulus."""
    say("degenerate oscillator round trips", precision)
    w = W.config("degenerate_cw", nt=1024, nz=25, level=4.0, refl=0.7)
    nrt = 300
    ref, e_ref = oracle.roundtrips(w["crystal"], w["cavity"], w["fields"], w["pump_in"], w["nz"], nrt)
    with B.from_workload(w, precision=precision) as h:
        h.cavity_roundtrip(nrt)
        e = h.energy_history()
        got = h.get_fields()
    assert e.shape == (nrt, 3)
    assert np.all(e[:, 2] == 0.0)
    assert e_ref[-1, 1] > 1e35 * e_ref[0, 1] and e_ref[-1, 0] < 0.1 * e_ref[0, 0]   # saturated
    for x in range(2):
        assert np.max(np.abs(e[:, x] - e_ref[:, x]) / e_ref[:, x]) <= TOL_E[precision], x
    assert rel_l2(np.abs(got[1]), np.abs(ref[1])) <= (1e-9 if precision == "f64" else 1e-3)


def test_two_and_three_wave_instances_share_a_batch():
    """Two-wave and three-wave instances of several sizes in one handle (mixed schedule):
    each equals its own single-instance run bit for bit, and the oracle."""
    say("mixed two/three-wave batch")
    insts = []
    for b, nt in enumerate([4096, 8192, 4096, 16384, 8192]):
        if b % 2 == 0:
            ins = _stress2(nt, seed=60 + b)
        else:
            ins = W.config("sro_cw", nt=nt)
            ins = dict(crystal=ins["crystal"], cavity=ins["cavity"], fields=ins["fields"],
                       pump_in=ins["pump_in"])
        ins["cavity"] = W.cavity(resonant=(0, 1, 0), refl=(0.0, 0.85 + 0.02 * b, 0.0),
                                 delta=(0.0, -0.1 * b, 0.0), eom_beta=0.3, eom_fpm_thz=1.0 / 40.0)
        insts.append(ins)
    nz, nrt = 6, 3
    with B.Opo(insts, nz, precision="f32", schedule="two_pass") as hb:
        hb.cavity_roundtrip(nrt)
        batch = [(hb.get_fields(i), hb.energy_history(i)) for i in range(len(insts))]
    for i, ins in enumerate(insts):
        nf = ins["crystal"].get("nf", 3)
        assert batch[i][0].shape == (nf, ins["crystal"]["nt"])
        with B.Opo([ins], nz, precision="f32", schedule="two_pass") as h:
            h.cavity_roundtrip(nrt)
            assert np.array_equal(batch[i][0], h.get_fields())
            assert np.array_equal(batch[i][1], h.energy_history())
        ref, e_ref = oracle.roundtrips(ins["crystal"], ins["cavity"], ins["fields"], ins["pump_in"], nz, nrt)
        for x in range(nf):
            assert rel_l2(batch[i][0][x], ref[x]) <= TOL["f32"], (i, x)
            assert np.max(np.abs(batch[i][1][:, x] - e_ref[:, x]) / e_ref[:, x]) <= TOL_E["f32"]


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_two_wave_gdd_eom_and_spectrum(precision):
    """GDD and EOM on the resonant signal of a two-wave instance, and the spectrum read-out."""
    ins = _stress2(2048, seed=9)
    ins["cavity"] = W.cavity(resonant=(0, 1, 0), refl=(0.0, 0.95, 0.0), delta=(0.0, 0.3, 0.0),
                             gdd_fs2=-900.0, eom_beta=0.8, eom_fpm_thz=2.0 / 40.0)
    nz, nrt = 12, 5
    ref, e_ref = oracle.roundtrips(ins["crystal"], ins["cavity"], ins["fields"], ins["pump_in"], nz, nrt)
    with B.Opo([ins], nz, precision=precision) as h:
        h.cavity_roundtrip(nrt)
        e = h.energy_history()
        got = h.get_fields()
        spec = h.get_fields(domain=1)
    for x in range(2):
        assert np.max(np.abs(e[:, x] - e_ref[:, x]) / e_ref[:, x]) <= TOL_E[precision]
        assert rel_l2(got[x], ref[x]) <= TOL[precision], (x, rel_l2(got[x], ref[x]))
        assert rel_l2(spec[x], np.fft.fft(got[x])) <= (1e-13 if precision == "f64" else 1e-6)


def test_degenerate_sweep_full_size_sampled():
    """The 256-instance degenerate sweep in the benchmark's launch configuration, two round
    trips; one instance of every size is replayed by the oracle."""
    say("degenerate sweep 256, 2 RT")
    w = W.config("degenerate_sweep")
    insts = w["instances"]
    with B.from_workload(w) as h:
        h.cavity_roundtrip(2)
        picks = {}
        for i, ins in enumerate(insts):
            picks.setdefault(ins["crystal"]["nt"], i)
        got = {i: (h.get_fields(i), h.energy_history(i)) for i in picks.values()}
    assert len(picks) == 5
    for i, (a, e) in got.items():
        ins = insts[i]
        ref, e_ref = oracle.roundtrips(ins["crystal"], ins["cavity"], ins["fields"], ins["pump_in"], w["nz"], 2)
        for x in range(2):
            assert rel_l2(a[x], ref[x]) <= 2e-4, (i, x)
            assert np.max(np.abs(e[:, x] - e_ref[:, x]) / e_ref[:, x]) <= 1e-3
