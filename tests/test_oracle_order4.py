"""Pins of the oracle's fourth-order splitting (order = 4): each step of dz is the triple
jump S(a dz) S(b dz) S(a dz) of symmetrized steps, a = 1/(2 - 2^(1/3)), b = 1 - 2a."""
import numpy as np

import oracle
from paper_2410_02532_amd import workloads as W

A_TJ = 1.0 / (2.0 - 2.0 ** (1.0 / 3.0))


def _case(nt=256, order=2):
    """Every term on: pulsed pump, seeded signal and idler, mismatch, GVM, GVD and TOD,
    strong enough coupling that the split matters."""
    cr = W.crystal(nt, t_window_ps=20.0, deff=40.0, dk_per_mm=0.8, db1=(0.3, 0.0, -0.2),
                   b2=(800.0, 500.0, 300.0), b3=(2000.0, 1000.0, 500.0), length_mm=2.0)
    cr["order"] = order
    t = W.time_grid(nt, 20.0)
    a = np.stack([2e6 * np.exp(-t * t / 8.0) + 0j,
                  2e5 * np.exp(-(t - 1.0) ** 2 / 2.0) + W.noise(nt, 1e3, 3),
                  W.noise(nt, 1e4, 4)])
    return cr, a


def test_fourth_order_convergence():
    """Halving dz divides the error of the triple jump by ~16 (order 4); the symmetrized
    step by ~4 (order 2) on the same case."""
    cr4, a = _case(order=4)
    L = cr4["length_mm"]
    ref = oracle.ssfm_pass(cr4, a, 512, L / 512)
    errs = []
    for nz in (16, 32, 64):
        out = oracle.ssfm_pass(cr4, a, nz, L / nz)
        errs.append(np.linalg.norm(out - ref) / np.linalg.norm(ref))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 12.0 < r1 < 20.0 and 12.0 < r2 < 20.0, (errs, r1, r2)
    cr2, _ = _case(order=2)
    e2 = [np.linalg.norm(oracle.ssfm_pass(cr2, a, nz, L / nz) - ref) / np.linalg.norm(ref) for nz in (32, 64)]
    assert 3.3 < e2[0] / e2[1] < 4.7
    assert errs[1] < 0.2 * e2[0]                     # more accurate at the same step count


def test_linear_steps_compose_exactly():
    """Without coupling a + b + a = 1 makes the three propagators one step's, so the triple
    jump equals the symmetrized pass up to rounding."""
    cr4, a = _case(order=4)
    cr4 = dict(cr4, deff_pm_per_v=0.0)
    cr2 = dict(cr4, order=2)
    L = cr4["length_mm"]
    o4 = oracle.ssfm_pass(cr4, a, 10, L / 10)
    o2 = oracle.ssfm_pass(cr2, a, 10, L / 10)
    assert np.max(np.abs(o4 - o2)) < 1e-11 * np.max(np.abs(a))


def test_coefficients():
    assert abs(2 * A_TJ + (1 - 2 * A_TJ) - 1.0) < 1e-15
    assert abs(2 * A_TJ ** 3 + (1 - 2 * A_TJ) ** 3) < 1e-14       # the third-order condition
