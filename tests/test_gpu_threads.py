"""Distinct handles are independent: two handles driven from two host threads at the
same time (each on its own stream; the library releases the interpreter lock during
its calls) give exactly the results of running them one after the other."""
import sys
import threading

import numpy as np
import pytest

import torch  # noqa: F401  (imported at collection: the first import can take minutes)

from paper_2410_02532_amd import opo as B
from paper_2410_02532_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _work(w, out, key, precision):
    insts = w["instances"] if "instances" in w else [w]
    with B.Opo(insts, w["nz"], precision=precision) as h:
        h.cavity_roundtrip(20)
        h.ssfm_propagate(7, 0.1)
        out[key] = ([h.get_fields(i) for i in range(len(insts))], h.energy_history(0))


def test_two_handles_in_two_threads_equal_sequential_runs():
    say("two handles, two threads")
    a = W.config("batched_sweep", count=12, nz=20)
    b = W.config("sro_cw", nt=1 << 13, nz=20)
    seq = {}
    _work(a, seq, "a", "f32")
    _work(b, seq, "b", "f64")
    par = {}
    errs = []

    def run(w, key, prec):
        try:
            _work(w, par, key, prec)
        except Exception as e:   # surfaced below, in the test's own thread
            errs.append(e)

    ts = [threading.Thread(target=run, args=(a, "a", "f32")), threading.Thread(target=run, args=(b, "b", "f64"))]
    for t in ts:
        t.start()
    for t in ts:
        t.join(timeout=240)
    assert not errs, errs
    assert not any(t.is_alive() for t in ts)
    for k in ("a", "b"):
        for x, y in zip(seq[k][0], par[k][0]):
            assert np.array_equal(x, y)
        assert np.array_equal(seq[k][1], par[k][1])
