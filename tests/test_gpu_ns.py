"""Parity of the HIP path's nanosecond regime with the FP64 oracle: a long input pump read one
round-trip window at a time, and the on-device record of the fields leaving the crystal."""
import sys

import numpy as np
import pytest

import torch  # noqa: F401  (imported at collection: the first import can take minutes)

import oracle
from paper_2410_02532_amd import opo as B
from paper_2410_02532_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-10, "f32": 1e-3}


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def rel_l2(got, ref):
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))


def _windowed(nt, windows, seed, nf=3):
    cr = W.crystal(nt, deff=40.0) if nf == 3 else W.crystal2(nt, deff=40.0)
    g = np.random.Generator(np.random.PCG64(seed))
    t = W.time_grid(nt)
    env = np.exp(-((np.arange(windows) - windows / 2) / (windows / 3)) ** 2)
    pump = (2.0e6 * env[:, None] * np.exp(-t[None, :] ** 2 / (2 * 30.0 ** 2))
            * np.exp(1j * g.uniform(0, 2 * np.pi, size=(windows, 1))))
    f = W.initial_fields(nt, 2.0e6, seed)[:nf]
    f[1] += W.noise(nt, 1e4, seed + 5)
    f[0] = pump[0]
    return dict(crystal=cr, cavity=W.cavity(refl=(0.0, 0.8, 0.0)), fields=f, pump_in=pump)


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("nf", [3, 2])
def test_windowed_pump_and_record(precision, nf):
    """12 pump windows, 15 round trips (the last three with a zero pump), a record of 20:
    every recorded field and every energy against the oracle; round trips outside the record
    are refused."""
    say("windowed pump + record", precision, nf)
    nt, nz, windows, nrt = 512, 10, 12, 15
    ins = _windowed(nt, windows, seed=21 + nf, nf=nf)
    a_ref, e_ref, rec_ref = oracle.roundtrips_record(ins["crystal"], ins["cavity"], ins["fields"],
                                                     ins["pump_in"], nz, nrt)
    with B.Opo([ins], nz, precision=precision, record_rt=20) as h:
        h.cavity_roundtrip(9)
        h.cavity_roundtrip(nrt - 9)          # the round-trip count carries across calls
        e = h.energy_history()
        rec = [h.record(m) for m in range(nrt)]
        with pytest.raises(B.OpoError) as ei:
            h.record(nrt)
        assert ei.value.code == B.OPO_EINVAL
    for m in range(nrt):
        for x in range(nf):
            if not np.any(rec_ref[m, x]):           # e.g. the pump after the last window
                assert not np.any(rec[m][x]), (m, x)
                continue
            assert rel_l2(rec[m][x], rec_ref[m, x]) <= TOL[precision], (m, x)
    for x in range(nf):
        live = e_ref[:, x] > 0.0
        assert np.max(np.abs(e[live, x] - e_ref[live, x]) / e_ref[live, x]) <= TOL[precision], x
        assert np.all(e[~live, x] == 0.0)
    if nf == 3:   # no input pump after the last window, and nothing regenerates one
        assert np.all(e_ref[windows:, 0] == 0.0) and np.all(e[windows:, 0] == 0.0)


def test_record_capacity_and_batch():
    """A record shorter than the run keeps the first round trips; a batch (mixed schedule)
    records each instance as its own run does."""
    say("record capacity, batch")
    nt, nz, windows = 1024, 8, 6
    insts = [_windowed(nt, windows, seed=s) for s in (31, 32)]
    with B.Opo(insts, nz, precision="f32", record_rt=5, schedule="two_pass") as hb:
        hb.cavity_roundtrip(8)
        recs = [[hb.record(m, i) for m in range(5)] for i in range(2)]
        with pytest.raises(B.OpoError):
            hb.record(5, 0)
    for i, ins in enumerate(insts):
        with B.Opo([ins], nz, precision="f32", record_rt=5, schedule="two_pass") as h:
            h.cavity_roundtrip(8)
            for m in range(5):
                assert np.array_equal(recs[i][m], h.record(m))


def test_ns_pulsed_workload():
    """The nanosecond workload at reduced grid (Nt = 2^10, Nz = 50): two degenerate
    oscillators pumped by 10 ns pulses at 10 and 20 times threshold over 400 round-trip
    windows, from the 1e-20 noise seed; energies of every round trip against the oracle
    (signal energies below 1e-20 of the peak pump window are FP32 underflow territory and
    are left out)."""
    say("ns pulsed workload 2 x 2^10 x 400 RT")
    w = W.config("ns_pulsed", nt=1024, nz=50, levels=(10.0, 20.0))
    with B.from_workload(w, record_rt=w["n_rt"]) as h:
        h.cavity_roundtrip(w["n_rt"])
        got = [(h.energy_history(i), h.record(300, i)) for i in range(2)]
    for i, ins in enumerate(w["instances"]):
        _, e_ref, rec_ref = oracle.roundtrips_record(ins["crystal"], ins["cavity"], ins["fields"],
                                                     ins["pump_in"], w["nz"], w["n_rt"])
        e = got[i][0]
        floor = 1e-20 * e_ref[:, 0].max()
        assert e_ref[:, 1].max() > 1e-3 * e_ref[:, 0].max()          # it oscillates
        assert np.max(np.abs(e[:, 0] - e_ref[:, 0]) / e_ref[:, 0]) <= 1e-3
        ok = e_ref[:, 1] > floor
        assert np.max(np.abs(e[ok, 1] - e_ref[ok, 1]) / e_ref[ok, 1]) <= 1e-3
        assert rel_l2(np.abs(got[i][1][0]), np.abs(rec_ref[300, 0])) <= 1e-3
