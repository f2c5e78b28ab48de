"""Pins of the oracle's Kerr (chi(3)) term, the extension the paper names for its nonlinear
operator: i gamma_x (|A_x|^2 + 2 sum_{y != x} |A_y|^2) A_x with
gamma_x = (2 pi/lambda_x) n2 (n_x eps0 c/2)."""
import numpy as np
import pytest

import oracle
from paper_2410_02532_amd import workloads as W

EPS0, C0 = 8.8541878128e-12, 299792458.0


def _kerr_crystal(nt, n2, **kw):
    kw.setdefault("deff", 0.0)
    kw.setdefault("db1", (0, 0, 0))
    kw.setdefault("b2", (0, 0, 0))
    c = W.crystal(nt, **kw)
    c["n2_m2_per_w"] = n2
    return c


def test_gamma_formula():
    c = _kerr_crystal(8, 3e-20, n=(2.2, 2.1, 2.0))
    g = oracle.kerr(c)
    for x in range(3):
        lam = c["lambda_um"][x] * 1e-6
        ref = 2 * np.pi / lam * 3e-20 * 0.5 * c["n"][x] * EPS0 * C0 * 1e-3
        assert g[x] == pytest.approx(ref, rel=1e-14)
    assert np.all(oracle.kerr(W.crystal(8)) == 0.0)


def test_self_and_cross_phase_closed_form():
    """Without chi(2) or dispersion the moduli stay fixed and each field turns by
    gamma_x (|A_x|^2 + 2 sum_{y != x} |A_y|^2) L."""
    nt, nz = 16, 200
    c = _kerr_crystal(nt, 2e-19)
    g = np.random.Generator(np.random.PCG64(3))
    a = (g.uniform(0.5, 1.5, (3, nt)) * np.exp(1j * g.uniform(0, 6.3, (3, nt)))) * 6e7
    L = c["length_mm"]
    out = oracle.ssfm_pass(c, a, nz, L / nz)
    gam = oracle.kerr(c)
    p = np.abs(a) ** 2
    for x in range(3):
        phi = gam[x] * (p[x] + 2 * (p.sum(0) - p[x])) * L
        assert np.max(np.abs(out[x] - a[x] * np.exp(1j * phi))) / np.max(np.abs(a[x])) < 1e-10
    assert np.max(gam[0] * 5 * p.max() * L) > 0.5                 # phases of order one


def test_fundamental_soliton_keeps_its_shape():
    """Anomalous GVD (b2 < 0) with self-phase modulation: A = sqrt(P0) sech(t/T0), with
    gamma P0 T0^2 = |b2|, propagates unchanged in modulus and turns by gamma P0 z / 2. The
    split-step error falls about fourfold when dz halves (second order)."""
    nt, T, t0, b2 = 1024, 5.0, 0.1, -2000.0                     # ps, ps, fs^2/mm
    c = _kerr_crystal(nt, 1e-19, t_window_ps=T, b2=(b2, 0.0, 0.0))
    gam = oracle.kerr(c)[0]
    p0 = abs(b2) * 1e-6 / (gam * t0 * t0)
    t = W.time_grid(nt, T)
    a = np.zeros((3, nt), complex)
    a[0] = np.sqrt(p0) / np.cosh(t / t0)
    L = c["length_mm"]                                           # one dispersion length
    errs = []
    for nz in (50, 100, 200):
        out = oracle.ssfm_pass(c, a, nz, L / nz)
        ref = a[0] * np.exp(0.5j * gam * p0 * L)
        errs.append(np.linalg.norm(out[0] - ref) / np.linalg.norm(ref))
    assert errs[-1] < 1e-4
    assert 3.3 < errs[0] / errs[1] < 4.7 and 3.3 < errs[1] / errs[2] < 4.7


def test_kerr_keeps_the_manley_rowe_power_invariant():
    """Kerr terms change phases only, so with chi(2) on the n-weighted power of the three
    fields stays conserved (dispersion and mismatch included)."""
    nt = 128
    c = _kerr_crystal(nt, 1e-19, deff=14.0, db1=(0.2, 0.0, -0.1), b2=(250.0, 150.0, 100.0),
                      dk_per_mm=0.5)
    g = np.random.Generator(np.random.PCG64(9))
    a = (g.standard_normal((3, nt)) + 1j * g.standard_normal((3, nt))) * 1e7
    out = oracle.ssfm_pass(c, a, 200, 0.025)
    n = np.array(c["n"])[:, None]
    lam = np.array(c["lambda_um"])[:, None]
    # photon-flux weighted: n|A|^2 lambda is conserved per pair exchange; total power n|A|^2 too
    p_in, p_out = np.sum(n * np.abs(a) ** 2), np.sum(n * np.abs(out) ** 2)
    assert abs(p_out / p_in - 1) < 1e-9
    q_in = np.sum((n * lam * np.abs(a) ** 2)[1]) - np.sum((n * lam * np.abs(a) ** 2)[2])
    q_out = np.sum((n * lam * np.abs(out) ** 2)[1]) - np.sum((n * lam * np.abs(out) ** 2)[2])
    assert abs(q_out - q_in) / np.sum(n * lam * np.abs(a) ** 2) < 1e-9
