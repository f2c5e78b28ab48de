"""Parity of the HIP path's adaptive step (local-error method) with the FP64 oracle: the
step sequence of every instance (accepted and rejected attempts, the z it reaches) and
the fields, single instances and uneven batches whose instances take different steps."""
import sys

import numpy as np
import pytest

import torch  # noqa: F401  (imported at collection: the first import can take minutes)

import oracle
from paper_2410_02532_amd import opo as B
from paper_2410_02532_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-10, "f32": 2e-4}


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def rel_l2(got, ref):
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))


def _inst(nt, seed, deff=40.0, dk=0.8, nf=3, n2=0.0, scale=1.0):
    """Pulsed pump with a seeded signal (and idler), mismatch, GVM, GVD and TOD."""
    mk = W.crystal if nf == 3 else W.crystal2
    cr = mk(nt, t_window_ps=20.0, deff=deff, dk_per_mm=dk, db1=(0.3, 0.0, -0.2),
            b2=(800.0, 500.0, 300.0), b3=(2000.0, 1000.0, 500.0), length_mm=2.0)
    cr["n2_m2_per_w"] = n2
    t = W.time_grid(nt, 20.0)
    a = np.empty((nf, nt), complex)
    a[0] = 2e6 * scale * np.exp(-t * t / 8.0)
    a[1] = 2e5 * np.exp(-(t - 1.0) ** 2 / 2.0) + W.noise(nt, 1e3, seed)
    if nf == 3:
        a[2] = W.noise(nt, 1e4, seed + 1)
    return dict(crystal=cr, cavity=W.cavity(), fields=a, pump_in=a[0].copy())


def _oracle(ins, L, tol, dz0, z0=0.0):
    return oracle.propagate_adaptive(ins["crystal"], ins["fields"], L, tol, dz0, z0=z0)


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("nt,tol,dz0", [(1024, 1e-4, 0.05), (4096, 1e-5, 0.05), (2048, 1e-4, 1.0)])
def test_adaptive_single(nt, tol, dz0, precision):
    """FP64: the oracle's accepted / rejected counts and fields (dz0 = 1 forces
    rejections first). FP32: d is formed in FP64 but from FP32 fields, whose rounding
    moves d by up to about 1e-7 / tol of itself, and the controller keeps d near its
    thresholds; a decision may then fall the other way. The counts may differ by a
    step or two and the fields by the adaptive error itself (both runs are within
    about tol of the exact solution), so FP32 is held to 10 tol and to 2 attempts."""
    say("adaptive single nt=%d tol=%g dz0=%g %s" % (nt, tol, dz0, precision))
    ins = _inst(nt, seed=nt)
    L = 2.0
    ref, acc, rej = _oracle(ins, L, tol, dz0)
    if dz0 >= 1.0:
        assert rej > 0
    with B.Opo([ins], 40, precision=precision) as h:
        ga, gr, gz = h.ssfm_propagate_adaptive(L, tol, dz0)
        got = h.get_fields()
    assert gz[0] == L
    if precision == "f64":
        assert (ga[0], gr[0]) == (acc, rej)
        bound = TOL["f64"]
    else:
        assert abs(ga[0] - acc) <= 2 and abs(gr[0] - rej) <= 2, ((ga[0], gr[0]), (acc, rej))
        bound = TOL["f32"] if (ga[0], gr[0]) == (acc, rej) else 10 * tol
    for x in range(3):
        assert rel_l2(got[x], ref[x]) <= bound, (x, rel_l2(got[x], ref[x]))


def test_adaptive_batch_uneven():
    """Instances of different size, coupling, wave count and Kerr index take different
    step sequences in one batch; each equals its own single run and the oracle."""
    say("adaptive batch")
    insts = [_inst(1024, 3), _inst(8192, 5, deff=25.0, dk=-0.5), _inst(2048, 7, nf=2),
             _inst(4096, 9, n2=2e-17, scale=3.0), _inst(512, 11, deff=0.0)]
    L, tol, dz0 = 2.0, 1e-6, 0.1
    with B.Opo(insts, 40, precision="f64", schedule="two_pass") as hb:
        acc_b, rej_b, z_b = hb.ssfm_propagate_adaptive(L, tol, dz0)
        batch = [hb.get_fields(i) for i in range(len(insts))]
    assert len(set(acc_b.tolist())) > 2                 # the sequences differ
    for i, ins in enumerate(insts):
        with B.Opo([ins], 40, precision="f64", schedule="two_pass") as h:
            a1, r1, _ = h.ssfm_propagate_adaptive(L, tol, dz0)
            assert (a1[0], r1[0]) == (acc_b[i], rej_b[i])
            assert np.array_equal(h.get_fields(), batch[i])
        ref, acc, rej = _oracle(ins, L, tol, dz0)
        assert (acc, rej) == (acc_b[i], rej_b[i]), i
        nf = ref.shape[0]
        for x in range(nf):
            assert rel_l2(batch[i][x], ref[x]) <= TOL["f64"], (i, x)


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_adaptive_large(precision):
    """2^16 points per field (several column and row tiles of the largest shapes)."""
    nt = 1 << 16
    say("adaptive large %s" % precision)
    ins = _inst(nt, seed=2)
    L, tol, dz0 = 1.0, 1e-4, 0.1
    ref, acc, rej = _oracle(ins, L, tol, dz0)
    with B.Opo([ins], 40, precision=precision) as h:
        ga, gr, _ = h.ssfm_propagate_adaptive(L, tol, dz0)
        got = h.get_fields()
    same = (ga[0], gr[0]) == (acc, rej)
    assert same or (precision == "f32" and abs(ga[0] - acc) <= 2 and abs(gr[0] - rej) <= 2)
    for x in range(3):
        assert rel_l2(got[x], ref[x]) <= (TOL[precision] if same else 10 * tol)


def test_adaptive_then_fixed_steps_continue_z():
    """The handle's z advances by the length: fixed steps after it see e^{i dk z} from
    there, and a second adaptive call starts from there too."""
    say("adaptive then fixed")
    ins = _inst(1024, 13)
    tol, dz0 = 1e-6, 0.1
    a1, _, _ = _oracle(ins, 0.7, tol, dz0)
    a2 = oracle.ssfm_pass(ins["crystal"], a1, 5, 0.1, 0.7)
    a3, acc, rej = oracle.propagate_adaptive(ins["crystal"], a2, 0.8, tol, dz0, z0=1.2)
    with B.Opo([ins], 40, precision="f64") as h:
        h.ssfm_propagate_adaptive(0.7, tol, dz0)
        h.ssfm_propagate(5, 0.1)
        ga, gr, gz = h.ssfm_propagate_adaptive(0.8, tol, dz0)
        got = h.get_fields()
    assert (ga[0], gr[0]) == (acc, rej) and gz[0] == pytest.approx(2.0, abs=1e-15)
    for x in range(3):
        assert rel_l2(got[x], a3[x]) <= TOL["f64"]


def test_adaptive_edges():
    """Zero length leaves the fields; a spent budget reports OPO_ESTEPS with the z
    reached; bad arguments and a fourth-order handle are refused."""
    say("adaptive edges")
    ins = _inst(256, 17)
    with B.Opo([ins], 40, precision="f64") as h:
        before = h.get_fields()
        acc, rej, z = h.ssfm_propagate_adaptive(0.0, 1e-6, 0.1)
        assert (acc[0], rej[0], z[0]) == (0, 0, 0.0)
        assert np.array_equal(h.get_fields(), before)
        with pytest.raises(B.OpoError) as e:
            h.ssfm_propagate_adaptive(2.0, 1e-300, 0.1, max_attempts=5)
        assert e.value.code == B.OPO_ESTEPS
        assert np.array_equal(h.get_fields(), before)      # every attempt was rejected
        for bad in [(-1.0, 1e-6, 0.1), (1.0, 0.0, 0.1), (1.0, 1e-6, 0.0), (float("nan"), 1e-6, 0.1)]:
            with pytest.raises(B.OpoError) as e:
                h.ssfm_propagate_adaptive(*bad)
            assert e.value.code == B.OPO_EINVAL
        with pytest.raises(B.OpoError) as e:
            h.ssfm_propagate_adaptive(1.0, 1e-6, 0.1, max_attempts=0)
        assert e.value.code == B.OPO_EINVAL
    with B.Opo([ins], 40, precision="f64", split_order=4) as h:
        with pytest.raises(B.OpoError) as e:
            h.ssfm_propagate_adaptive(1.0, 1e-6, 0.1)
        assert e.value.code == B.OPO_EINVAL


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_adaptive_graph_replay_equals_plain_launches(precision):
    """The attempt replayed from a graph (many replays, host read-backs between chunks,
    and a second call on the same handle) equals plain launches bit for bit."""
    say("adaptive graph vs plain %s" % precision)
    insts = [_inst(2048, 21), _inst(4096, 23, dk=-0.3), _inst(1024, 25, nf=2)]
    L, tol, dz0 = 2.0, 1e-5, 0.05
    out = {}
    for g in (True, False):
        with B.Opo(insts, 40, precision=precision, use_graph=g) as h:
            r1 = h.ssfm_propagate_adaptive(1.2, tol, dz0)
            r2 = h.ssfm_propagate_adaptive(L - 1.2, tol, dz0)
            out[g] = (r1, r2, [h.get_fields(i) for i in range(len(insts))])
    for k in range(2):
        for q in range(3):
            assert np.array_equal(out[True][k][q], out[False][k][q])
    for i in range(len(insts)):
        assert np.array_equal(out[True][2][i], out[False][2][i])


def test_adaptive_smallest_grids_and_zero_fields():
    """nt = 2 and 4 (one-point columns and rows) beside a regular instance, and an
    all-zero instance: its d is 0/0, never above a threshold, so every attempt is kept
    at dz0 and the count is ceil(L / dz0), as in the oracle."""
    say("adaptive tiny and zero")

    def cw(nt):
        cr = W.crystal(nt, t_window_ps=20.0, deff=40.0, dk_per_mm=0.8)
        a = np.stack([np.full(nt, 2e6 + 0j), np.full(nt, 2e5 + 1e4j), np.full(nt, 1e4 + 0j)])
        return dict(crystal=cr, cavity=W.cavity(), fields=a, pump_in=a[0].copy())

    zero = dict(crystal=W.crystal(64, t_window_ps=20.0, deff=40.0), cavity=W.cavity(),
                fields=np.zeros((3, 64), complex), pump_in=np.zeros(64, complex))
    insts = [cw(2), cw(4), _inst(1024, 31), zero]
    L, tol, dz0 = 2.0, 1e-7, 0.3
    with B.Opo(insts, 40, precision="f64") as h:
        acc, rej, z = h.ssfm_propagate_adaptive(L, tol, dz0)
        got = [h.get_fields(i) for i in range(len(insts))]
    assert (acc[3], rej[3]) == (int(np.ceil(L / dz0)), 0)
    assert np.all(got[3] == 0) and np.all(z == L)
    for i, ins in enumerate(insts[:3]):
        ref, ra, rr = _oracle(ins, L, tol, dz0)
        assert (acc[i], rej[i]) == (ra, rr), i
        for x in range(3):
            assert rel_l2(got[i][x], ref[x]) <= TOL["f64"], (i, x)


def test_adaptive_largest_fp32_grid():
    """2^20 points per field (256-point columns, 4096-point rows) in FP32 against the
    oracle over a short length."""
    say("adaptive 2^20 f32")
    nt = 1 << 20
    cr = W.crystal(nt, t_window_ps=100.0, deff=40.0, dk_per_mm=0.8, b3=500.0)
    t = W.time_grid(nt, 100.0)
    a = np.stack([3e6 * np.exp(-t * t / 8.0) + 0j,
                  2e5 * np.exp(-(t - 1.0) ** 2 / 2.0) + W.noise(nt, 1e3, 3), W.noise(nt, 1e4, 4)])
    ins = dict(crystal=cr, cavity=W.cavity(), fields=a, pump_in=a[0].copy())
    L, tol, dz0 = 0.5, 1e-4, 0.05
    ref, ra, rr = _oracle(ins, L, tol, dz0)
    with B.Opo([ins], 40, precision="f32") as h:
        acc, rej, _ = h.ssfm_propagate_adaptive(L, tol, dz0)
        got = h.get_fields()
    same = (acc[0], rej[0]) == (ra, rr)
    assert same or (abs(acc[0] - ra) <= 2 and abs(rej[0] - rr) <= 2)
    for x in range(3):
        assert rel_l2(got[x], ref[x]) <= (TOL["f32"] if same else 10 * tol), x


def test_adaptive_pulsed_workload_sampled():
    """The benchmark's adaptive workload as the benchmark runs it (128 uneven instances,
    FP32, tol 1e-5, dz0 = L/100): the three smallest instances and the first of the
    largest against the oracle, and every instance reaches the end."""
    say("adaptive workload, sampled")
    w = W.config("adaptive_pulsed")
    insts = w["instances"]
    L = insts[0]["crystal"]["length_mm"]
    with B.Opo(insts, w["nz"], precision="f32") as h:
        acc, rej, z = h.ssfm_propagate_adaptive(L, w["tol"], L / w["nz"])
        order = sorted(range(len(insts)), key=lambda i: (insts[i]["crystal"]["nt"], i))
        big = max(insts[i]["crystal"]["nt"] for i in order)
        picks = order[:3] + [next(i for i in order if insts[i]["crystal"]["nt"] == big)]
        got = {i: h.get_fields(i) for i in picks}
    assert np.all(z == L)
    for i in picks:
        ref, ra, rr = oracle.propagate_adaptive(insts[i]["crystal"], insts[i]["fields"], L, w["tol"], L / w["nz"])
        same = (acc[i], rej[i]) == (ra, rr)
        assert same or (abs(acc[i] - ra) <= 2 and abs(rej[i] - rr) <= 2), (i, (acc[i], rej[i]), (ra, rr))
        for x in range(3):
            assert rel_l2(got[i][x], ref[x]) <= (TOL["f32"] if same else 10 * w["tol"]), (i, x)
