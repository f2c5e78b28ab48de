"""The C-ABI library loads, exports every symbol include/opo.h declares, and
rejects bad arguments on the host side (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2410_02532_amd import opo as B
from paper_2410_02532_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "opo.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("opo_init", "ssfm_propagate", "cavity_roundtrip"):
        assert must in names
    assert sorted(B.EXPORTS) == names


def test_library_exports_every_declared_symbol():
    lib = B.load()
    for name in _declared():
        assert hasattr(lib, name), name
        assert isinstance(getattr(lib, name), ctypes._CFuncPtr)


def _one(nt=64, nz=10, **cav):
    cr = W.crystal(nt)
    ins = dict(crystal=cr, cavity=W.cavity(**cav), fields=W.initial_fields(nt, 1e6, 1),
               pump_in=np.full(nt, 1e6 + 0j))
    return B._structs([ins], nz)


def _init(fields, crystals, cavities, n=1, precision=0):
    lib = B.load()
    h = ctypes.c_void_p()
    opt = B.OptionsT(precision=precision)
    rc = lib.opo_init_batch(ctypes.byref(h), n, fields, crystals, cavities, ctypes.byref(opt))
    return rc, h


def test_state_bytes():
    lib = B.load()
    n, f, c, k, keep = _one(nt=256)
    assert lib.opo_state_bytes(1, f, 0) == 3 * 256 * 8
    assert lib.opo_state_bytes(1, f, 1) == 3 * 256 * 16
    assert lib.opo_state_bytes(0, f, 0) == 0
    f[0].n_fields = 2                       # two waves: pump and degenerate signal
    assert lib.opo_state_bytes(1, f, 0) == 2 * 256 * 8
    assert lib.opo_state_bytes(1, f, 1) == 2 * 256 * 16


def test_two_wave_structs_from_the_binding():
    cr = W.crystal2(128)
    f = W.initial_fields(128, 1e6, 1)[:2]
    ins = dict(crystal=cr, cavity=W.cavity(), fields=f, pump_in=np.full(128, 1e6 + 0j))
    n, fs, c, k, keep = B._structs([ins], 10)
    assert fs[0].n_fields == 2
    assert B.load().opo_state_bytes(1, fs, 0) == 2 * 128 * 8
    with pytest.raises(ValueError):
        B._structs([dict(ins, fields=W.initial_fields(128, 1e6, 1))], 10)   # (3, nt) for nf = 2


@pytest.mark.parametrize("mutate, what", [
    (lambda f, c, k: setattr(f[0], "nt", 96), "power of two"),
    (lambda f, c, k: setattr(f[0], "nt", 1), "power of two"),
    (lambda f, c, k: setattr(f[0], "nt", 1 << 21), "power of two"),
    (lambda f, c, k: setattr(f[0], "t_window_ps", -1.0), "t_window"),
    (lambda f, c, k: setattr(c[0], "nz", 0), "nz"),
    (lambda f, c, k: setattr(c[0], "length_mm", float("nan")), "length"),
    (lambda f, c, k: k[0].refl.__setitem__(1, 1.5), "reflectivit"),
    (lambda f, c, k: c[0].b2_fs2_per_mm.__setitem__(0, float("inf")), "finite"),
    (lambda f, c, k: setattr(c[0], "deff_pm_per_v", 1e6), "step too large"),
    (lambda f, c, k: setattr(f[0], "n_fields", 4), "n_fields"),
    (lambda f, c, k: setattr(f[0], "n_fields", 1), "n_fields"),
])
def test_init_rejects_bad_arguments(mutate, what):
    n, f, c, k, keep = _one()
    mutate(f, c, k)
    rc, h = _init(f, c, k)
    assert rc == B.OPO_EINVAL
    assert h.value is None
    assert what in B.last_error()


def test_batch_must_share_nz_and_bad_precision():
    lib = B.load()
    n, f, c, k, keep = _one()
    f2, c2, k2 = (B.FieldsT * 2)(f[0], f[0]), (B.CrystalT * 2)(c[0], c[0]), (B.CavityT * 2)(k[0], k[0])
    c2[1].nz = c2[0].nz + 1
    rc, _ = _init(f2, c2, k2, n=2)
    assert rc == B.OPO_EINVAL and "share nz" in B.last_error()
    rc, _ = _init(f, c, k, precision=7)
    assert rc == B.OPO_EINVAL
    h = ctypes.c_void_p()
    assert lib.opo_init_batch(ctypes.byref(h), 0, f, c, k, None) == B.OPO_EINVAL
    assert lib.opo_init(None, f, c, k, None) == B.OPO_EINVAL


def test_calls_on_invalid_handles():
    lib = B.load()
    bogus = ctypes.c_void_p(0x1234)
    assert lib.ssfm_propagate(None, 10, 0.1) == B.OPO_ESTATE
    assert lib.cavity_roundtrip(bogus, 1) == B.OPO_ESTATE
    assert lib.opo_sync(None) == B.OPO_ESTATE
    assert lib.opo_destroy(bogus) == B.OPO_ESTATE
    out = np.zeros(8)
    assert lib.opo_get_fields(None, 0, 0, 0, out.ctypes.data) == B.OPO_ESTATE
    assert "handle" in B.last_error()
    rt, z = ctypes.c_int32(), ctypes.c_double()
    assert lib.opo_get_progress(bogus, ctypes.byref(rt), ctypes.byref(z)) == B.OPO_ESTATE
    assert lib.opo_set_progress(None, 0, 0.0, None) == B.OPO_ESTATE


def test_bad_device_ordinal_is_reported():
    """A device ordinal no HIP device has (the library checks the device before it
    allocates anything)."""
    n, f, c, k, keep = _one()
    lib = B.load()
    h = ctypes.c_void_p()
    opt = B.OptionsT(device=97)
    assert lib.opo_init_batch(ctypes.byref(h), 1, f, c, k, ctypes.byref(opt)) == B.OPO_EDEVICE
    assert h.value is None and "ordinal 97" in B.last_error()


def test_no_device_is_reported():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    n, f, c, k, keep = _one()
    rc, h = _init(f, c, k)
    assert rc == B.OPO_EDEVICE
    assert h.value is None


def test_empty_batch_is_rejected():
    n, f, c, k, keep = _one()
    rc, h = _init(f, c, k, n=0)
    assert rc == B.OPO_EINVAL and h.value is None
    assert B.load().opo_state_bytes(0, f, 0) == 0


@pytest.mark.parametrize("schedule", [-1, 3])
def test_bad_schedule_is_rejected(schedule):
    """The schedule option takes 0 (automatic), 1 (two passes) or 2 (resident where served);
    checked before any device call."""
    n, f, c, k, keep = _one()
    h = ctypes.c_void_p()
    opt = B.OptionsT(schedule=schedule)
    assert B.load().opo_init_batch(ctypes.byref(h), 1, f, c, k, ctypes.byref(opt)) == B.OPO_EINVAL
    assert h.value is None and "schedule" in B.last_error()


def test_schedule_table_is_well_formed():
    """Every entry of the automatic schedule's table names a valid split and asks for the
    resident pass only where the kernel serves the shape (FP32 2^10..2^12, FP64 2^10..2^11);
    no key appears twice."""
    path = os.path.join(ROOT, "paper_2410_02532_amd", "csrc", "schedule_table.inc")
    rows = [tuple(int(v) for v in re.findall(r"-?\d+", line))
            for line in open(path) if line.strip().startswith("{")]
    assert rows
    keys = [r[:4] for r in rows]
    assert len(keys) == len(set(keys))
    for f64, nf, l, batched, col, res in rows:
        assert f64 in (0, 1) and nf in (2, 3) and batched in (0, 1)
        assert 1 <= l <= (19 if f64 else 20)
        assert col == 0 or 4 <= col <= 8
        if res:
            assert 10 <= l <= (11 if f64 else 12), (f64, nf, l)
