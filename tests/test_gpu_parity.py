"""Parity of the gfx950 HIP path (through the C ABI) with the FP64 CPU oracle.

Both sides receive the same seeded inputs from the workloads module. Bars:
complex128 runs match the oracle to 1e-11 relative L2 per field; complex64 runs
(FP64 phase arguments and energies) to 1e-4 relative L2 per field, and 1e-3 in
round-trip energies, as the target of the method's FP32 path states. The field
bars hold for one pass and for runs of round trips alike: the largest error
measured after 40 round trips of the SRO is 8e-6 (complex64) and 2e-13
(complex128), a twelfth and a fiftieth of the bar. Bit-exact equalities hold where the same kernels run on
the same data (batch vs single, graph vs plain launches, repeated runs, a pass
split in two calls).
"""
import math
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


def rel_max(got, ref):
    return float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))


def _stress(nt, seed=0, t_window=40.0, deff=60.0, b3=300.0, dk=0.4, alpha=(0.02, 0.01, 0.03)):
    """Pulsed pump, seeded signal and idler, every term of Eqs. 2-5 switched on."""
    cr = W.crystal(nt, t_window_ps=t_window, deff=deff, b3=(b3, -0.5 * b3, 0.7 * b3), dk_per_mm=dk,
                   alpha=alpha, db1=(0.25, 0.0, -0.15), b2=(250.0, 150.0, 100.0),
                   n=(2.25, 2.2, 2.15))
    t = W.time_grid(nt, t_window)
    rng = np.random.Generator(np.random.PCG64(seed))
    pump = 2.0e6 * np.exp(-t * t / (2 * (0.2 * t_window) ** 2)) * np.exp(0.3j)
    a = np.empty((3, nt), complex)
    a[0] = pump
    a[1] = 3.0e5 * np.exp(-(t - 1.0) ** 2 / (2 * (0.1 * t_window) ** 2)) + W.noise(nt, 1e3, seed + 1)
    a[2] = W.noise(nt, 2e4, seed + 2) * rng.uniform(0.5, 1.5)
    cav = W.cavity(resonant=(0, 1, 1), refl=(0.0, 0.9, 0.7), delta=(0.0, 0.2, -0.4))
    return dict(crystal=cr, cavity=cav, fields=a, pump_in=pump)


def _handle(inst, nz, precision, **kw):
    return B.Opo([inst], nz, precision=precision, **kw)


@pytest.mark.parametrize("precision, nt", [(p, n) for p in ("f64", "f32")
                                           for n in (2, 4, 8, 64, 512, 1 << 12, 1 << 14, 1 << 16)]
                         + [("f64", 1 << 19), ("f32", 1 << 20)])   # the largest grids
def test_pass_parity(nt, precision):
    say("pass parity nt=%d %s" % (nt, precision))
    ins = _stress(nt, seed=nt)
    nz, dz = 20, 0.25
    ref = oracle.ssfm_pass(ins["crystal"], ins["fields"], nz, dz)
    with _handle(ins, nz, precision) as h:
        h.ssfm_propagate(nz, dz)
        got = h.get_fields()
        assert h.info()[1] == pytest.approx(nz * dz)
    tol = TOL[precision]
    if precision == "f64":
        # The dispersion phase of a bin is formed in FP64 on both sides but not in the same
        # order: at the Nyquist edge of the 2^19 grid on this 40 ps window the third-order
        # term reaches ~9e5 rad per step, whose argument carries ~1e-10 rad of rounding. For
        # broadband (noise-seeded) fields that bounds the relative difference by about
        # phi_max * 2^-53 * sqrt(nz); the bar keeps a factor 4 over it and 1e-11 below it.
        cr = ins["crystal"]
        wn = np.pi * nt / cr["t_window_ps"]
        phi = max(abs(cr["db1_ps_per_mm"][x]) * wn + abs(cr["b2_fs2_per_mm"][x]) * 1e-6 * wn ** 2 / 2
                  + abs(cr["b3_fs3_per_mm"][x]) * 1e-9 * wn ** 3 / 6 for x in range(3)) * dz
        tol = max(tol, 4 * phi * 2.0 ** -53 * np.sqrt(nz))
    for x in range(3):
        assert rel_l2(got[x], ref[x]) <= tol, (x, rel_l2(got[x], ref[x]))
        assert rel_max(got[x], ref[x]) <= 10 * tol


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_single_pass_workload(precision):
    """The single-pass workload at its full size: Nt = 2^10, Nz = 100, CW pump, noise seeds."""
    w = W.config("single_pass")
    say("single pass workload", precision)
    dz = w["crystal"]["length_mm"] / w["nz"]
    ref = oracle.ssfm_pass(w["crystal"], w["fields"], w["nz"], dz)
    with B.from_workload(w, precision=precision) as h:
        h.ssfm_propagate(w["nz"], dz)
        got = h.get_fields()
    for x in range(3):
        assert rel_l2(got[x], ref[x]) <= TOL[precision], (x, rel_l2(got[x], ref[x]))


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_pass_split_in_two_calls_is_identical(precision):
    ins = _stress(4096, seed=3)
    with _handle(ins, 20, precision) as h1, _handle(ins, 20, precision) as h2:
        h1.ssfm_propagate(20, 0.25)
        h2.ssfm_propagate(10, 0.25)
        h2.ssfm_propagate(10, 0.25)
        assert np.array_equal(h1.get_fields(), h2.get_fields())


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_roundtrip_parity_sro(precision):
    """CW singly resonant OPO above threshold, idler and pump non-resonant."""
    say("round trips SRO", precision)
    w = W.config("sro_cw", nt=1024, nz=25, level=4.0)
    nrt = 40
    ref, e_ref = oracle.roundtrips(w["crystal"], w["cavity"], w["fields"], w["pump_in"], w["nz"], nrt)
    with B.from_workload(w, precision=precision) as h:
        h.cavity_roundtrip(nrt)
        e = h.energy_history()
        got = h.get_fields()
    assert e.shape == (nrt, 3)
    for x in range(3):
        assert np.max(np.abs(e[:, x] - e_ref[:, x]) / e_ref[:, x]) <= TOL_E[precision]
        assert rel_l2(got[x], ref[x]) <= TOL[precision]


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_roundtrip_parity_gdd_eom_pulsed(precision):
    """Doubly resonant cavity with GDD on both resonant fields, an EOM, detuning, loss,
    a pulsed pump re-read every round trip and every dispersion order."""
    say("round trips GDD+EOM", precision)
    ins = _stress(2048, seed=5)
    ins["cavity"] = W.cavity(resonant=(0, 1, 1), refl=(0.0, 0.95, 0.9), delta=(0.0, 0.3, -0.2),
                             gdd_fs2=-900.0, eom_beta=0.8, eom_fpm_thz=2.0 / 40.0)
    nz, nrt = 12, 6
    ref, e_ref = oracle.roundtrips(ins["crystal"], ins["cavity"], ins["fields"], ins["pump_in"], nz, nrt)
    with _handle(ins, nz, precision) as h:
        h.cavity_roundtrip(nrt)
        e = h.energy_history()
        got = h.get_fields()
    for x in range(3):
        assert np.max(np.abs(e[:, x] - e_ref[:, x]) / e_ref[:, x]) <= TOL_E[precision]
        assert rel_l2(got[x], ref[x]) <= TOL[precision], (x, rel_l2(got[x], ref[x]))


def test_batch_of_uneven_sizes_equals_singles_and_oracle():
    """Instances of different nt in one handle: each equals its own single-instance run
    bit for bit, and the oracle within the FP32 bar."""
    say("batch uneven")
    sizes = [16, 4096, 256, 8192, 2, 1024]
    insts = []
    for b, nt in enumerate(sizes):
        ins = _stress(nt, seed=10 + b)
        ins["cavity"] = W.cavity(resonant=(0, 1, 0), refl=(0.0, 0.8 + 0.02 * b, 0.0),
                                 delta=(0.0, 0.1 * b, 0.0))
        insts.append(ins)
    nz, nrt = 8, 3
    with B.Opo(insts, nz, precision="f32", schedule="two_pass") as hb:
        hb.cavity_roundtrip(nrt)
        batch = [(hb.get_fields(i), hb.energy_history(i)) for i in range(len(sizes))]
    for i, ins in enumerate(insts):
        with _handle(ins, nz, "f32", schedule="two_pass") as h:
            h.cavity_roundtrip(nrt)
            assert np.array_equal(batch[i][0], h.get_fields())
            assert np.array_equal(batch[i][1], h.energy_history())
        ref, e_ref = oracle.roundtrips(ins["crystal"], ins["cavity"], ins["fields"], ins["pump_in"],
                                       nz, nrt)
        for x in range(3):
            assert rel_l2(batch[i][0][x], ref[x]) <= TOL["f32"], (i, x)


def test_graph_replay_equals_plain_launches_and_is_deterministic():
    w = W.config("sro_cw", nt=2048, nz=10, level=3.0)
    outs = []
    for graph in (True, False, True):
        with B.from_workload(w, use_graph=graph) as h:
            h.cavity_roundtrip(7)
            h.cavity_roundtrip(5)
            outs.append((h.get_fields(), h.energy_history()))
    for o in outs[1:]:
        assert np.array_equal(o[0], outs[0][0])
        assert np.array_equal(o[1], outs[0][1])
    assert outs[0][1].shape == (12, 3)


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_spectrum_readout(precision):
    ins = _stress(1 << 13, seed=7)
    with _handle(ins, 5, precision) as h:
        h.ssfm_propagate(5, 0.2)
        a = h.get_fields()
        spec = h.get_fields(domain=1)
        t, w = h.grid()
    for x in range(3):
        ref = np.fft.fft(a[x])
        assert rel_l2(spec[x], ref) <= (1e-13 if precision == "f64" else 1e-6)
    assert np.allclose(t, W.time_grid(1 << 13, 40.0))
    assert np.allclose(w, 2 * np.pi * np.fft.fftfreq(1 << 13, 40.0 / (1 << 13)))


def test_nonfinite_energy_is_reported():
    w = W.config("sro_cw", nt=256, nz=5)
    with B.from_workload(w) as h:
        a = h.get_fields()
        a[1, 17] = np.nan
        h.set_fields(a)
        with pytest.raises(B.OpoError) as ei:
            h.cavity_roundtrip(3)
        assert ei.value.code == B.OPO_ENONFINITE
        assert "round trip 0" in str(ei.value)


def test_full_size_sro_bench_configuration():
    """The CW SRO workload at its full size (Nt = 2^14, Nz = 100) in the launch
    configuration the benchmark times, over three round trips from the same input."""
    w = W.config("sro_cw")
    nrt = 3
    say("full-size SRO f32")
    ref, e_ref = oracle.roundtrips(w["crystal"], w["cavity"], w["fields"], w["pump_in"], w["nz"], nrt)
    with B.from_workload(w, precision="f32") as h:
        h.cavity_roundtrip(nrt)
        e = h.energy_history()
        got = h.get_fields()
    for x in range(3):
        assert np.max(np.abs(e[:, x] - e_ref[:, x]) / e_ref[:, x]) <= TOL_E["f32"]
        assert rel_l2(got[x], ref[x]) <= TOL["f32"], (x, rel_l2(got[x], ref[x]))


def test_mixed_schedule_batch_equals_singles_and_oracle():
    """A batch whose sizes share one column and one row kernel runs as two halves a launch
    apart, column tiles of one half together with row tiles of the other; every instance
    still equals its own single-instance run bit for bit, and the oracle."""
    say("mixed-schedule batch")
    sizes = [8192, 4096, 16384, 4096, 8192]
    insts = []
    for b, nt in enumerate(sizes):
        ins = _stress(nt, seed=40 + b)
        ins["cavity"] = W.cavity(resonant=(0, 1, 0), refl=(0.0, 0.85 + 0.02 * b, 0.0),
                                 delta=(0.0, -0.1 * b, 0.0), eom_beta=0.3, eom_fpm_thz=1.0 / 40.0)
        insts.append(ins)
    nz, nrt = 6, 3
    with B.Opo(insts, nz, precision="f32", schedule="two_pass") as hb:
        hb.cavity_roundtrip(nrt)
        batch = [(hb.get_fields(i), hb.energy_history(i)) for i in range(len(sizes))]
        hb.ssfm_propagate(5, 0.1)
        prop = [hb.get_fields(i) for i in range(len(sizes))]
    for i, ins in enumerate(insts):
        with _handle(ins, nz, "f32", schedule="two_pass") as h:
            h.cavity_roundtrip(nrt)
            assert np.array_equal(batch[i][0], h.get_fields())
            assert np.array_equal(batch[i][1], h.energy_history())
            h.ssfm_propagate(5, 0.1)
            assert np.array_equal(prop[i], h.get_fields())
        ref, e_ref = oracle.roundtrips(ins["crystal"], ins["cavity"], ins["fields"], ins["pump_in"], nz, nrt)
        for x in range(3):
            assert rel_l2(batch[i][0][x], ref[x]) <= TOL["f32"], (i, x)
            assert np.max(np.abs(batch[i][1][:, x] - e_ref[:, x]) / e_ref[:, x]) <= TOL_E["f32"]


def test_mixed_schedule_with_gdd_and_eom():
    """A batch on the mixed schedule whose cavities carry chirped-mirror GDD (on the signal
    only for one instance) and an EOM: the GDD row pass and the column pass after it cover
    both halves; every instance equals its own single run bit for bit, and the oracle."""
    say("mixed schedule + GDD")
    sizes = [4096, 8192, 4096, 8192]
    insts = []
    for b, nt in enumerate(sizes):
        ins = _stress(nt, seed=70 + b)
        ins["cavity"] = W.cavity(resonant=(0, 1, 1), refl=(0.0, 0.9, 0.85), delta=(0.0, 0.1 * b, -0.2),
                                 gdd_fs2=-800.0 + 500.0 * b, gdd_on=(0, 1, 0) if b == 2 else None,
                                 eom_beta=0.4, eom_fpm_thz=1.0 / 40.0)
        insts.append(ins)
    nz, nrt = 6, 3
    with B.Opo(insts, nz, precision="f32", schedule="two_pass") as hb:
        hb.cavity_roundtrip(nrt)
        batch = [(hb.get_fields(i), hb.energy_history(i)) for i in range(len(sizes))]
    for i, ins in enumerate(insts):
        with _handle(ins, nz, "f32", schedule="two_pass") as h:
            h.cavity_roundtrip(nrt)
            assert np.array_equal(batch[i][0], h.get_fields())
            assert np.array_equal(batch[i][1], h.energy_history())
        ref, e_ref = oracle.roundtrips(ins["crystal"], ins["cavity"], ins["fields"], ins["pump_in"], nz, nrt)
        for x in range(3):
            assert rel_l2(batch[i][0][x], ref[x]) <= TOL["f32"], (i, x)
            assert np.max(np.abs(batch[i][1][:, x] - e_ref[:, x]) / e_ref[:, x]) <= TOL_E["f32"]


def test_fp64_mixed_schedule_batch():
    """The FP64 kernels on the mixed schedule: a batch equals its single runs bit for bit and
    the oracle to the FP64 bar."""
    say("FP64 mixed batch")
    insts = []
    for b, nt in enumerate([2048, 4096, 2048, 4096]):
        ins = _stress(nt, seed=90 + b)
        ins["cavity"] = W.cavity(resonant=(0, 1, 0), refl=(0.0, 0.8 + 0.03 * b, 0.0), delta=(0.0, 0.2 * b, 0.0))
        insts.append(ins)
    nz, nrt = 6, 3
    with B.Opo(insts, nz, precision="f64", schedule="two_pass") as hb:
        hb.cavity_roundtrip(nrt)
        batch = [(hb.get_fields(i), hb.energy_history(i)) for i in range(len(insts))]
    for i, ins in enumerate(insts):
        with _handle(ins, nz, "f64", schedule="two_pass") as h:
            h.cavity_roundtrip(nrt)
            assert np.array_equal(batch[i][0], h.get_fields())
            assert np.array_equal(batch[i][1], h.energy_history())
        ref, e_ref = oracle.roundtrips(ins["crystal"], ins["cavity"], ins["fields"], ins["pump_in"], nz, nrt)
        for x in range(3):
            assert rel_l2(batch[i][0][x], ref[x]) <= TOL["f64"], (i, x)
            assert np.max(np.abs(batch[i][1][:, x] - e_ref[:, x]) / e_ref[:, x]) <= TOL_E["f64"]


def test_zero_round_trips_and_bad_steps():
    w = W.config("sro_cw", nt=256, nz=5)
    with B.from_workload(w) as h:
        a0 = h.get_fields()
        h.cavity_roundtrip(0)
        assert h.energy_history().shape == (0, 3)
        assert np.array_equal(h.get_fields(), a0)
        for nz, dz in ((0, 0.1), (3, 0.0), (3, -1.0), (3, float("nan"))):
            with pytest.raises(B.OpoError) as ei:
                h.ssfm_propagate(nz, dz)
            assert ei.value.code == B.OPO_EINVAL
        with pytest.raises(B.OpoError):
            h.cavity_roundtrip(-1)
