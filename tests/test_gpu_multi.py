"""Parity of the HIP path's round trips through several crystals with the FP64 oracle."""
import sys

import numpy as np
import pytest

import torch  # noqa: F401  (imported at collection: the first import can take minutes)

import oracle
from paper_2410_02532_amd import opo as B
from paper_2410_02532_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL_E = {"f64": 1e-10, "f32": 1e-3}
TOL = {"f64": 1e-11, "f32": 1e-4}


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def rel_l2(got, ref):
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))


def _cascade(nt, seed):
    """A chi(2) crystal with mismatch followed by a shorter one with other dispersion, a Kerr
    index and the opposite mismatch; a singly resonant cavity above threshold."""
    c1 = W.crystal(nt, dk_per_mm=0.6)
    c2 = W.crystal(nt, dk_per_mm=-0.4, length_mm=3.0, b2=(-150.0, 100.0, 250.0), b3=200.0,
                   db1=(0.1, 0.0, 0.3))
    c2["n2_m2_per_w"] = 1e-17
    ap0 = 3.0 * W.threshold_amplitude(c1, 0.8)
    return dict(crystal=c1, crystals=[c1, c2], cavity=W.cavity(refl=(0.0, 0.8, 0.0), delta=(0.0, 0.2, 0.0)),
                fields=W.initial_fields(nt, ap0, seed), pump_in=np.full(nt, ap0 + 0j))


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_two_crystals_round_trips(precision):
    say("two crystals", precision)
    nt, nzs, nrt = 2048, [12, 8], 40
    ins = _cascade(nt, 5)
    ref, e_ref, _ = oracle.roundtrips_multi(ins["crystals"], nzs, ins["cavity"], ins["fields"],
                                            ins["pump_in"], nrt)
    assert e_ref[-1, 1] > 1e10 * e_ref[0, 1]
    with B.Opo([ins], nzs, precision=precision) as h:
        h.cavity_roundtrip(nrt)
        e = h.energy_history()
        got = h.get_fields()
    for x in range(3):
        assert np.max(np.abs(e[:, x] - e_ref[:, x]) / e_ref[:, x]) <= TOL_E[precision], x
        assert rel_l2(got[x], ref[x]) <= TOL[precision], x


def test_two_halves_match_one_crystal():
    """Without mismatch two crystals of L/2 (nz/2 steps each) run the same arithmetic as one
    crystal of L."""
    nt, nz, nrt = 1024, 20, 5
    w = W.config("sro_cw", nt=nt, nz=nz, level=4.0)
    half = dict(w["crystal"], length_mm=0.5 * w["crystal"]["length_mm"])
    one = dict(crystal=w["crystal"], cavity=w["cavity"], fields=w["fields"], pump_in=w["pump_in"])
    two = dict(one, crystals=[half, half])
    with B.Opo([one], nz) as h1, B.Opo([two], [nz // 2, nz // 2]) as h2:
        h1.cavity_roundtrip(nrt)
        h2.cavity_roundtrip(nrt)
        a1, a2 = h1.get_fields(), h2.get_fields()
        e1, e2 = h1.energy_history(), h2.energy_history()
    for x in range(3):
        assert rel_l2(a2[x], a1[x]) <= 1e-6
        assert np.max(np.abs(e2[:, x] - e1[:, x]) / e1[:, x]) <= 1e-6


def test_cascade_batch_equals_singles_and_oracle():
    say("cascade batch")
    insts = [_cascade(nt, 20 + b) for b, nt in enumerate([4096, 8192, 4096, 16384])]
    nzs, nrt = [10, 6], 3
    with B.Opo(insts, nzs, precision="f32", record_rt=nrt, schedule="two_pass") as hb:
        hb.cavity_roundtrip(nrt)
        batch = [(hb.get_fields(i), hb.energy_history(i), hb.record(nrt - 1, i)) for i in range(len(insts))]
    for i, ins in enumerate(insts):
        with B.Opo([ins], nzs, precision="f32", schedule="two_pass") as h:
            h.cavity_roundtrip(nrt)
            assert np.array_equal(batch[i][0], h.get_fields())
            assert np.array_equal(batch[i][1], h.energy_history())
        _, e_ref, rec = oracle.roundtrips_multi(ins["crystals"], nzs, ins["cavity"], ins["fields"],
                                                ins["pump_in"], nrt, record=True)
        for x in range(3):
            assert np.max(np.abs(batch[i][1][:, x] - e_ref[:, x]) / e_ref[:, x]) <= 1e-3
            assert rel_l2(batch[i][2][x], rec[-1, x]) <= 1e-4
