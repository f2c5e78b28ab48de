"""The col_log2 option (four-step split nt = n1 * n2 chosen by the caller): every split
the kernels support matches the oracle per pass; bad values are refused."""
import sys

import numpy as np
import pytest

import torch  # noqa: F401  (imported at collection: the first import can take minutes)

import oracle
from paper_2410_02532_amd import opo as B
from paper_2410_02532_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-11, "f32": 1e-4}


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def rel_l2(got, ref):
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))


def _pulsed(nt, seed):
    cr = W.crystal(nt, t_window_ps=40.0, deff=60.0, b3=300.0, dk_per_mm=0.4,
                   db1=(0.25, 0.0, -0.15), b2=(250.0, 150.0, 100.0))
    t = W.time_grid(nt, 40.0)
    a = np.stack([2.0e7 * np.exp(-t * t / 128.0) + 0j,
                  3.0e6 * np.exp(-(t - 1.0) ** 2 / 32.0) + W.noise(nt, 1e4, seed),
                  W.noise(nt, 2e5, seed + 1)])
    return dict(crystal=cr, cavity=W.cavity(), fields=a, pump_in=a[0].copy())


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("nt,col", [(1 << 11, 4), (1 << 14, 4), (1 << 14, 5), (1 << 14, 7), (1 << 16, 5),
                                    (1 << 16, 8), (1 << 17, 5)])
def test_split_parity(nt, col, precision):
    say("split nt=%d col_log2=%d %s" % (nt, col, precision))
    ins = _pulsed(nt, seed=nt + col)
    nz, dz = 40, 0.125
    ref = oracle.ssfm_pass(ins["crystal"], ins["fields"], nz, dz)
    with B.Opo([ins], nz, precision=precision, col_log2=col) as h:
        h.ssfm_propagate(nz, dz)
        got = h.get_fields()
    for x in range(3):
        assert rel_l2(got[x], ref[x]) <= TOL[precision], (x, rel_l2(got[x], ref[x]))


def test_split_round_trips_and_batch():
    """Round trips of an SRO with columns of 32 match the automatic split to FP32
    rounding, and a batch under the option equals its members run alone."""
    say("split round trips")
    w = W.config("sro_cw", nt=1 << 14, nz=20, level=3.0)
    one = dict(crystal=w["crystal"], cavity=w["cavity"], fields=w["fields"], pump_in=w["pump_in"])
    other = dict(one, fields=W.initial_fields(1 << 13, w["pump_in"][0], 7),
                 crystal=W.crystal(1 << 13), pump_in=np.full(1 << 13, w["pump_in"][0]))
    with B.Opo([one], 20, col_log2=5) as h5, B.Opo([one], 20, schedule="two_pass") as h0:
        h5.cavity_roundtrip(30)
        h0.cavity_roundtrip(30)
        e5, e0 = h5.energy_history(), h0.energy_history()
    assert np.max(np.abs(e5 - e0) / e0) < 1e-3
    with B.Opo([one, other], 20, col_log2=5, schedule="two_pass") as hb:
        hb.cavity_roundtrip(5)
        batch = [hb.get_fields(i) for i in range(2)]
    for i, ins in enumerate((one, other)):
        with B.Opo([ins], 20, col_log2=5, schedule="two_pass") as h:
            h.cavity_roundtrip(5)
            assert np.array_equal(h.get_fields(), batch[i])


def test_split_bad_values():
    ins = _pulsed(1 << 12, 3)
    for col in (-1, 1, 3, 9):
        with pytest.raises(B.OpoError) as e:
            B.Opo([ins], 10, col_log2=col)
        assert e.value.code == B.OPO_EINVAL


def test_tuner_split_model_matches_the_library():
    """The schedule tuner labels and deduplicates its candidates with the split it expects
    the library's plan to give for each col_log2 option (and for the default); that model
    must be the library's own (opo_get_plan)."""
    from paper_2410_02532_amd import tune
    for prec in ("f32", "f64"):
        for l in (10, 11, 13, 14, 17, tune.MAX_LOG2[prec]):
            ins = dict(crystal=W.crystal(1 << l), cavity=W.cavity(), fields=W.initial_fields(1 << l, 1e6, 1),
                       pump_in=np.full(1 << l, 1e6 + 0j))
            for cl in (0, 4, 5, 6, 7, 8):
                with B.Opo([ins], 2, precision=prec, col_log2=cl, schedule="two_pass") as h:
                    l1, l2, res = h.plan(0)
                assert (l1 + l2, l2, res) == (l, tune.split_of(l, prec, cl), False), (prec, l, cl)
