"""Parity of the HIP path's fourth-order splitting (split_order = 4: the triple jump of
symmetrized steps) with the FP64 oracle."""
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


def _case(nt, seed, nf=3, kerr=0.0):
    mk = W.crystal if nf == 3 else W.crystal2
    cr = mk(nt, t_window_ps=40.0, deff=40.0, b3=(300.0, -150.0, 100.0), dk_per_mm=0.6,
            alpha=(0.02, 0.01, 0.03), db1=(0.25, 0.0, -0.15), b2=(250.0, 150.0, 100.0))
    cr["n2_m2_per_w"] = kerr
    t = W.time_grid(nt, 40.0)
    a = np.empty((nf, nt), complex)
    a[0] = 2.0e6 * np.exp(-t * t / (2 * 8.0 ** 2)) * np.exp(0.3j)
    a[1] = 3.0e5 * np.exp(-(t - 1.0) ** 2 / (2 * 4.0 ** 2)) + W.noise(nt, 1e3, seed + 1)
    if nf == 3:
        a[2] = W.noise(nt, 2e4, seed + 2)
    return dict(crystal=cr, cavity=W.cavity(refl=(0.0, 0.85, 0.0)), fields=a, pump_in=a[0].copy())


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("nt, nf, kerr", [(512, 3, 0.0), (4096, 2, 0.0), (1 << 16, 3, 2e-17)])
def test_fourth_order_pass_parity(nt, nf, kerr, precision):
    say("order-4 pass nt=%d nf=%d %s" % (nt, nf, precision))
    ins = _case(nt, nt, nf, kerr)
    nz, dz = 12, 0.25
    ref = oracle.ssfm_pass(dict(ins["crystal"], order=4), ins["fields"], nz, dz)
    with B.Opo([ins], nz, precision=precision, split_order=4) as h:
        h.ssfm_propagate(nz, dz)
        got = h.get_fields()
    for x in range(nf):
        assert rel_l2(got[x], ref[x]) <= TOL[precision], (x, rel_l2(got[x], ref[x]))


def test_fourth_order_round_trips_batch():
    """Round trips with the fourth-order step in a batch on the mixed schedule: each
    instance equals its own single run bit for bit, and the oracle's energies."""
    say("order-4 batch")
    insts = [_case(nt, 30 + b) for b, nt in enumerate([4096, 8192, 4096, 8192])]
    nz, nrt = 8, 3
    with B.Opo(insts, nz, precision="f32", split_order=4, schedule="two_pass") as hb:
        hb.cavity_roundtrip(nrt)
        batch = [(hb.get_fields(i), hb.energy_history(i)) for i in range(len(insts))]
    for i, ins in enumerate(insts):
        with B.Opo([ins], nz, precision="f32", split_order=4, schedule="two_pass") as h:
            h.cavity_roundtrip(nrt)
            assert np.array_equal(batch[i][0], h.get_fields())
            assert np.array_equal(batch[i][1], h.energy_history())
        ref, e_ref = oracle.roundtrips(dict(ins["crystal"], order=4), ins["cavity"], ins["fields"],
                                       ins["pump_in"], nz, nrt)
        for x in range(3):
            assert rel_l2(batch[i][0][x], ref[x]) <= 1e-4, (i, x)
            assert np.max(np.abs(batch[i][1][:, x] - e_ref[:, x]) / e_ref[:, x]) <= 1e-3


def test_split_order_is_validated():
    ins = _case(64, 1)
    with pytest.raises(B.OpoError) as ei:
        B.Opo([ins], 8, split_order=3)
    assert ei.value.code == B.OPO_EINVAL
