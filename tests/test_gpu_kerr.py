"""Parity of the HIP path's Kerr (chi(3)) term with the FP64 oracle: self- and cross-phase
modulation added to the RK4 nonlinear step, alone and together with chi(2)."""
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


def _kerr_stress(nt, nf, seed):
    """Pulsed pump, seeded signal (and idler), chi(2) with mismatch, every dispersion
    order, and a Kerr index that turns the fields by about a radian over the pass."""
    mk = W.crystal if nf == 3 else W.crystal2
    cr = mk(nt, t_window_ps=40.0, deff=60.0, b3=(300.0, -150.0, 100.0), dk_per_mm=0.4,
            alpha=(0.02, 0.01, 0.03), db1=(0.25, 0.0, -0.15), b2=(250.0, 150.0, 100.0))
    cr["n2_m2_per_w"] = 2e-17
    t = W.time_grid(nt, 40.0)
    a = np.empty((nf, nt), complex)
    a[0] = 2.0e7 * np.exp(-t * t / (2 * 8.0 ** 2)) * np.exp(0.3j)
    a[1] = 3.0e6 * np.exp(-(t - 1.0) ** 2 / (2 * 4.0 ** 2)) + W.noise(nt, 1e4, seed + 1)
    if nf == 3:
        a[2] = W.noise(nt, 2e5, seed + 2)
    return dict(crystal=cr, cavity=W.cavity(), fields=a, pump_in=a[0].copy())


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("nf", [3, 2])
@pytest.mark.parametrize("nt", [512, 1 << 13, 1 << 16])
def test_kerr_pass_parity(nt, nf, precision):
    say("kerr pass nt=%d nf=%d %s" % (nt, nf, precision))
    ins = _kerr_stress(nt, nf, seed=nt + nf)
    nz, dz = 40, 0.125
    g = oracle.kerr(ins["crystal"])
    assert g[0] * np.max(np.abs(ins["fields"][0])) ** 2 * nz * dz > 0.5     # Kerr phase matters
    ref = oracle.ssfm_pass(ins["crystal"], ins["fields"], nz, dz)
    with B.Opo([ins], nz, precision=precision) as h:
        h.ssfm_propagate(nz, dz)
        got = h.get_fields()
    for x in range(nf):
        assert rel_l2(got[x], ref[x]) <= TOL[precision], (x, rel_l2(got[x], ref[x]))


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_fundamental_soliton(precision):
    """Anomalous GVD with self-phase modulation over one dispersion length: the HIP path
    against the oracle (which keeps the sech shape to its split-step error)."""
    nt, T, t0, b2 = 1024, 5.0, 0.1, -2000.0
    cr = W.crystal(nt, t_window_ps=T, deff=0.0, db1=(0, 0, 0), b2=(b2, 0.0, 0.0))
    cr["n2_m2_per_w"] = 1e-19
    gam = oracle.kerr(cr)[0]
    p0 = abs(b2) * 1e-6 / (gam * t0 * t0)
    a = np.zeros((3, nt), complex)
    a[0] = np.sqrt(p0) / np.cosh(W.time_grid(nt, T) / t0)
    ins = dict(crystal=cr, cavity=W.cavity(resonant=(0, 0, 0), refl=(0, 0, 0)), fields=a, pump_in=a[0])
    nz = 200
    ref = oracle.ssfm_pass(cr, a, nz, cr["length_mm"] / nz)
    with B.Opo([ins], nz, precision=precision) as h:
        h.ssfm_propagate(nz, cr["length_mm"] / nz)
        got = h.get_fields()
    assert rel_l2(got[0], ref[0]) <= TOL[precision]
    assert rel_l2(np.abs(got[0]), np.abs(a[0])) < 1e-4            # the shape is kept


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_kerr_oscillator_round_trips(precision):
    """A singly resonant oscillator (R_s = 0.7, twice threshold) with a Kerr crystal, from
    noise through saturation: energies of 150 round trips against the oracle, and a batch
    with a Kerr-free twin where each instance equals its own single run."""
    nt, nz, nrt = 2048, 20, 150
    cr = W.crystal(nt)
    ap0 = 2.0 * W.threshold_amplitude(cr, 0.7)
    kcr = dict(cr, n2_m2_per_w=3e-17)
    ins = dict(crystal=kcr, cavity=W.cavity(refl=(0.0, 0.7, 0.0)), fields=W.initial_fields(nt, ap0, 11),
               pump_in=np.full(nt, ap0 + 0j))
    _, e_ref = oracle.roundtrips(kcr, ins["cavity"], ins["fields"], ins["pump_in"], nz, nrt)
    assert e_ref[-1, 1] > 1e35 * e_ref[0, 1]
    plain = dict(ins, crystal=cr)
    with B.Opo([ins, plain], nz, precision=precision, schedule="two_pass") as h:
        h.cavity_roundtrip(nrt)
        e = h.energy_history(0)
        pair = [h.get_fields(i) for i in range(2)]
    for x in range(3):
        assert np.max(np.abs(e[:, x] - e_ref[:, x]) / e_ref[:, x]) <= (1e-9 if precision == "f64" else 1e-3)
    for i, one in enumerate((ins, plain)):
        with B.Opo([one], nz, precision=precision, schedule="two_pass") as h:
            h.cavity_roundtrip(nrt)
            assert np.array_equal(h.get_fields(), pair[i])
