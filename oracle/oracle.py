"""ctypes front end of the FP64 C oracle (``opo_oracle.c``).

Test infrastructure only. Every function takes and returns numpy complex128
arrays; fields are stacked as ``a[x, j]`` with x = 0 pump, 1 signal, 2 idler
(three coupled waves) or x = 0 pump, 1 signal (two waves, crystal key
``nf`` = 2). Parameters come as plain dicts (keys as in :class:`Crystal` /
:class:`Cavity`; ``nf`` defaults to 3).
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "opo_oracle.c")
_LIB_PLAIN = os.path.join(_HERE, "libopo_oracle.so")
_LIB_SANITIZE = os.path.join(_HERE, "libopo_oracle_sanitize.so")
# ORACLE_LIB=sanitize loads the AddressSanitizer/UBSan build (CPU test runs only)
_LIB = _LIB_SANITIZE if os.environ.get("ORACLE_LIB") == "sanitize" else _LIB_PLAIN

_c3 = ctypes.c_double * 3
_i3 = ctypes.c_int * 3


class Crystal(ctypes.Structure):
    _fields_ = [
        ("nt", ctypes.c_int),
        ("nf", ctypes.c_int),
        ("t_window_ps", ctypes.c_double),
        ("length_mm", ctypes.c_double),
        ("lambda_um", _c3),
        ("n", _c3),
        ("deff_pm_per_v", ctypes.c_double),
        ("dk_per_mm", ctypes.c_double),
        ("alpha_per_mm", _c3),
        ("db1_ps_per_mm", _c3),
        ("b2_fs2_per_mm", _c3),
        ("b3_fs3_per_mm", _c3),
        ("n2_m2_per_w", ctypes.c_double),
        ("order", ctypes.c_int),
    ]

    @classmethod
    def from_dict(cls, d):
        c = cls()
        for name, ctype in cls._fields_:
            defaults = {"nf": 3, "n2_m2_per_w": 0.0, "order": 2}
            v = d.get(name, defaults[name]) if name in defaults else d[name]
            if ctype in (_c3,):
                setattr(c, name, _c3(*[float(x) for x in v]))
            elif ctype is ctypes.c_int:
                setattr(c, name, int(v))
            else:
                setattr(c, name, float(v))
        return c


class Cavity(ctypes.Structure):
    _fields_ = [
        ("resonant", _i3),
        ("refl", _c3),
        ("delta_rad", _c3),
        ("gdd_fs2", ctypes.c_double),
        ("gdd_on", _i3),
        ("eom_beta", ctypes.c_double),
        ("eom_fpm_thz", ctypes.c_double),
        ("eom_on", _i3),
    ]

    @classmethod
    def from_dict(cls, d):
        c = cls()
        for name, ctype in cls._fields_:
            v = d[name]
            if ctype is _i3:
                setattr(c, name, _i3(*[int(x) for x in v]))
            elif ctype is _c3:
                setattr(c, name, _c3(*[float(x) for x in v]))
            else:
                setattr(c, name, float(v))
        return c


def build(force=False, sanitize=False):
    """Compile the oracle with gcc (strict IEEE: no fast-math). sanitize: with
    AddressSanitizer and UndefinedBehaviorSanitizer into libopo_oracle_sanitize.so, which
    ORACLE_LIB selects (the process must preload gcc's libasan)."""
    lib = _LIB_SANITIZE if sanitize else _LIB_PLAIN
    if force or not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(_SRC):
        tmp = lib + ".tmp%d" % os.getpid()
        extra = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                 "-fno-sanitize-recover=all"] if sanitize else []
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fno-fast-math",
                               "-ffp-contract=off"] + extra + [_SRC, "-o", tmp, "-lm"])
        os.replace(tmp, lib)
    return lib


_lib = None


def _load():
    global _lib
    if _lib is None:
        build(sanitize=_LIB == _LIB_SANITIZE)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.ora_fft.argtypes = [P, ctypes.c_int, ctypes.c_int]
        lib.ora_omega.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double]
        lib.ora_omega.restype = ctypes.c_double
        lib.ora_kappa.argtypes = [ctypes.POINTER(Crystal), P]
        lib.ora_kerr.argtypes = [ctypes.POINTER(Crystal), P]
        lib.ora_dispersion.argtypes = [ctypes.POINTER(Crystal), ctypes.c_int, ctypes.c_double, P]
        lib.ora_rk4.argtypes = [ctypes.POINTER(Crystal), P, ctypes.c_double, ctypes.c_double]
        lib.ora_linear.argtypes = [ctypes.POINTER(Crystal), P, ctypes.c_double]
        lib.ora_pass.argtypes = [ctypes.POINTER(Crystal), P, ctypes.c_int, ctypes.c_double,
                                 ctypes.c_double]
        lib.ora_pass_unsym.argtypes = lib.ora_pass.argtypes
        lib.ora_gdd.argtypes = [P, ctypes.c_int, ctypes.c_double, ctypes.c_double]
        lib.ora_eom.argtypes = [P, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double]
        lib.ora_roundtrips.argtypes = [ctypes.POINTER(Crystal), ctypes.POINTER(Cavity), P, P,
                                       ctypes.c_int, ctypes.c_int, P]
        lib.ora_roundtrips_rec.argtypes = [ctypes.POINTER(Crystal), ctypes.POINTER(Cavity), P, P,
                                           ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P]
        lib.ora_propagate_adaptive.argtypes = [ctypes.POINTER(Crystal), P, ctypes.c_double, ctypes.c_double,
                                               ctypes.c_double, ctypes.c_double, ctypes.c_int, P, P]
        lib.ora_propagate_adaptive.restype = ctypes.c_int
        lib.ora_roundtrips_multi.argtypes = [ctypes.POINTER(Crystal), ctypes.c_int, P,
                                             ctypes.POINTER(Cavity), P, P, ctypes.c_int,
                                             ctypes.c_int, P, P]
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _cplx(a):
    return np.ascontiguousarray(a, dtype=np.complex128).copy()


def _nf(crystal):
    nf = int(crystal.get("nf", 3))
    if nf not in (2, 3):
        raise ValueError("nf must be 2 or 3")
    return nf


def _fields(a, crystal):
    a = _cplx(a)
    shape = (_nf(crystal), crystal["nt"])
    if a.shape != shape:
        raise ValueError("fields must have shape %s, got %s" % (shape, a.shape))
    return a


def fft(x):
    """Unnormalized forward DFT, X_k = sum_j x_j e^{-2 pi i jk/N} (radix-2)."""
    x = _cplx(x)
    _load().ora_fft(_ptr(x), x.size, 0)
    return x


def ifft(x):
    """Inverse DFT with the 1/N factor."""
    x = _cplx(x)
    _load().ora_fft(_ptr(x), x.size, 1)
    return x


def omega(n, t_window_ps):
    lib = _load()
    return np.array([lib.ora_omega(k, n, t_window_ps) for k in range(n)])


def kappa(crystal):
    out = np.zeros(3)
    _load().ora_kappa(ctypes.byref(Crystal.from_dict(crystal)), _ptr(out))
    return out


def kerr(crystal):
    """Kerr coefficients gamma_x [1/mm per (V/m)^2]."""
    out = np.zeros(3)
    _load().ora_kerr(ctypes.byref(Crystal.from_dict(crystal)), _ptr(out))
    return out


def dispersion(crystal, field, dz):
    h = np.zeros(crystal["nt"], dtype=np.complex128)
    _load().ora_dispersion(ctypes.byref(Crystal.from_dict(crystal)), field, dz, _ptr(h))
    return h


def rk4(crystal, a, z0, h):
    a = _fields(a, crystal)
    _load().ora_rk4(ctypes.byref(Crystal.from_dict(crystal)), _ptr(a), z0, h)
    return a


def linear(crystal, a, dz):
    a = _fields(a, crystal)
    _load().ora_linear(ctypes.byref(Crystal.from_dict(crystal)), _ptr(a), dz)
    return a


def ssfm_pass(crystal, a, nz, dz, z0=0.0):
    """nz symmetrized SSFM steps of size dz starting at z0; returns new fields."""
    a = _fields(a, crystal)
    _load().ora_pass(ctypes.byref(Crystal.from_dict(crystal)), _ptr(a), int(nz), float(dz),
                     float(z0))
    return a


def ssfm_pass_unsym(crystal, a, nz, dz, z0=0.0):
    a = _fields(a, crystal)
    _load().ora_pass_unsym(ctypes.byref(Crystal.from_dict(crystal)), _ptr(a), int(nz),
                           float(dz), float(z0))
    return a


def gdd(field, t_window_ps, gdd_fs2):
    f = _cplx(field)
    _load().ora_gdd(_ptr(f), f.size, t_window_ps, gdd_fs2)
    return f


def eom(field, t_window_ps, beta, fpm_thz):
    f = _cplx(field)
    _load().ora_eom(_ptr(f), f.size, t_window_ps, beta, fpm_thz)
    return f


def roundtrips(crystal, cavity, a, pump_in, nz, n_rt):
    """n_rt cavity round trips. Returns (fields, energies[n_rt, 3]); the idler column is
    zero for two waves."""
    nt = crystal["nt"]
    a = _fields(a, crystal)
    p = _cplx(np.broadcast_to(np.asarray(pump_in, dtype=np.complex128), (nt,)))
    e = np.zeros((int(n_rt), 3))
    _load().ora_roundtrips(ctypes.byref(Crystal.from_dict(crystal)),
                           ctypes.byref(Cavity.from_dict(cavity)), _ptr(a), _ptr(p),
                           int(nz), int(n_rt), _ptr(e))
    return a, e


def roundtrips_record(crystal, cavity, a, pump_long, nz, n_rt, record=True):
    """Nanosecond regime: round trip m reads window m of pump_long (n_slices x nt samples,
    a zero pump after the last window) into a non-resonant pump. Returns (fields,
    energies[n_rt, 3], record[n_rt, nf, nt] of the fields leaving the crystal, or None)."""
    nt = crystal["nt"]
    nf = _nf(crystal)
    a = _fields(a, crystal)
    p = _cplx(np.asarray(pump_long, dtype=np.complex128).reshape(-1))
    if p.size % nt or p.size == 0:
        raise ValueError("pump_long must hold whole windows of nt samples")
    e = np.zeros((int(n_rt), 3))
    rec = np.zeros((int(n_rt), nf, nt), dtype=np.complex128) if record else None
    _load().ora_roundtrips_rec(ctypes.byref(Crystal.from_dict(crystal)),
                               ctypes.byref(Cavity.from_dict(cavity)), _ptr(a), _ptr(p),
                               p.size // nt, int(nz), int(n_rt), _ptr(e),
                               _ptr(rec) if record else None)
    return a, e, rec


def roundtrips_multi(crystals, nzs, cavity, a, pump_in, n_rt, record=False):
    """Round trips through the crystals in order (crystal k with nzs[k] steps). pump_in is
    (nt,) for the same pump every round trip or (windows, nt). Returns (fields,
    energies[n_rt, 3], record or None)."""
    c0 = crystals[0]
    nt = c0["nt"]
    nf = _nf(c0)
    a = _fields(a, c0)
    p = np.asarray(pump_in, dtype=np.complex128)
    if p.ndim == 1:
        p = np.broadcast_to(p, (int(n_rt), nt))
    p = _cplx(p.reshape(-1))
    arr = (Crystal * len(crystals))(*[Crystal.from_dict(c) for c in crystals])
    nz_arr = np.ascontiguousarray(nzs, dtype=np.intc)
    e = np.zeros((int(n_rt), 3))
    rec = np.zeros((int(n_rt), nf, nt), dtype=np.complex128) if record else None
    _load().ora_roundtrips_multi(arr, len(crystals), _ptr(nz_arr), ctypes.byref(Cavity.from_dict(cavity)),
                                 _ptr(a), _ptr(p), p.size // nt, int(n_rt), _ptr(e),
                                 _ptr(rec) if record else None)
    return a, e, rec


def propagate_adaptive(crystal, a, length, tol, dz0, max_steps=100000, z0=0.0, budget_ok=False):
    """Propagation from z0 over `length` mm with the local-error adaptive step (second-order
    steps only). Returns (fields, accepted steps, rejected steps); raises RuntimeError when
    max_steps attempts do not reach the end, unless budget_ok (the fields then hold the last
    accepted step)."""
    a = _fields(a, crystal)
    acc, rej = ctypes.c_int(), ctypes.c_int()
    rc = _load().ora_propagate_adaptive(ctypes.byref(Crystal.from_dict(crystal)), _ptr(a), float(z0),
                                        float(length), float(tol), float(dz0), int(max_steps),
                                        ctypes.byref(acc), ctypes.byref(rej))
    if rc == -2:
        raise ValueError("the adaptive step needs second-order steps (order 2)")
    if rc != 0 and not budget_ok:
        raise RuntimeError("adaptive propagation did not reach the end in %d attempts" % max_steps)
    return a, acc.value, rej.value
