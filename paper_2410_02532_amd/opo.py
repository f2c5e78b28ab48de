"""Python binding of the gfx950 C-ABI library ``libopo.so`` (include/opo.h).

Argument marshalling only: every step of the propagation runs in the HIP
kernels behind the C ABI. PyTorch supplies the device memory that holds the
fields and the stream the library runs on. The library must be built
(``python -m paper_2410_02532_amd.build``); there is no fallback.
"""
import ctypes
import os

import numpy as np

# OPO_LIB selects another build of the library (the host-sanitizer build of the CPU tests)
LIB_PATH = os.environ.get("OPO_LIB") or os.path.join(os.path.dirname(os.path.abspath(__file__)), "libopo.so")

OPO_OK, OPO_EINVAL, OPO_ENOMEM, OPO_EDEVICE, OPO_ENONFINITE, OPO_ESTATE, OPO_ESTEPS = 0, -1, -2, -3, -4, -5, -6
OPO_F32, OPO_F64 = 0, 1
STATUS = {0: "OPO_OK", -1: "OPO_EINVAL", -2: "OPO_ENOMEM", -3: "OPO_EDEVICE",
          -4: "OPO_ENONFINITE", -5: "OPO_ESTATE", -6: "OPO_ESTEPS"}

EXPORTS = ("opo_state_bytes", "opo_init", "opo_init_batch", "ssfm_propagate", "ssfm_propagate_adaptive",
           "cavity_roundtrip",
           "opo_sync", "opo_get_fields", "opo_set_fields", "opo_get_progress", "opo_set_progress",
           "opo_get_energy_history",
           "opo_get_power_history",
           "opo_get_record", "opo_get_grid", "opo_kernel_times", "opo_info", "opo_destroy",
           "opo_last_error", "opo_get_spectrum_noalloc", "opo_get_plan")
KERNEL_CLASSES = ("column_pass", "row_pass", "energy_reduce", "mixed_pass", "resident_pass")
SCHEDULES = {"auto": 0, "two_pass": 1, "resident": 2}

_d3 = ctypes.c_double * 3
_i3 = ctypes.c_int32 * 3
_d2 = ctypes.c_double * 2


class FieldsT(ctypes.Structure):
    _fields_ = [("nt", ctypes.c_int32), ("t_window_ps", ctypes.c_double), ("lambda_um", _d3),
                ("n", _d3), ("init", ctypes.POINTER(ctypes.c_double)),
                ("pump_in", ctypes.POINTER(ctypes.c_double)), ("pump_cw", _d2),
                ("n_fields", ctypes.c_int32), ("pump_windows", ctypes.c_int32)]


class CrystalT(ctypes.Structure):
    _fields_ = [("length_mm", ctypes.c_double), ("nz", ctypes.c_int32),
                ("deff_pm_per_v", ctypes.c_double), ("dk_per_mm", ctypes.c_double),
                ("alpha_per_mm", _d3), ("db1_ps_per_mm", _d3), ("b2_fs2_per_mm", _d3),
                ("b3_fs3_per_mm", _d3), ("n2_m2_per_w", ctypes.c_double)]


class CavityT(ctypes.Structure):
    _fields_ = [("resonant", _i3), ("refl", _d3), ("delta_rad", _d3), ("gdd_fs2", ctypes.c_double),
                ("gdd_on", _i3), ("eom_beta", ctypes.c_double), ("eom_fpm_thz", ctypes.c_double),
                ("eom_on", _i3)]


class OptionsT(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("device", ctypes.c_int32),
                ("stream", ctypes.c_void_p), ("state", ctypes.c_void_p),
                ("state_bytes", ctypes.c_uint64), ("col_log2", ctypes.c_int32),
                ("schedule", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("profile", ctypes.c_int32), ("record_rt", ctypes.c_int32),
                ("n_crystals", ctypes.c_int32), ("split_order", ctypes.c_int32)]


class OpoError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (STATUS.get(code, code), msg))
        self.code = code


_lib = None


def load():
    """Load libopo.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libopo.so is not built; run `python -m paper_2410_02532_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P, I, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    lib.opo_state_bytes.argtypes = [I, ctypes.POINTER(FieldsT), I]
    lib.opo_state_bytes.restype = ctypes.c_uint64
    lib.opo_init.argtypes = [ctypes.POINTER(P), ctypes.POINTER(FieldsT), ctypes.POINTER(CrystalT),
                             ctypes.POINTER(CavityT), ctypes.POINTER(OptionsT)]
    lib.opo_init_batch.argtypes = [ctypes.POINTER(P), I, ctypes.POINTER(FieldsT),
                                   ctypes.POINTER(CrystalT), ctypes.POINTER(CavityT),
                                   ctypes.POINTER(OptionsT)]
    lib.ssfm_propagate.argtypes = [P, I, D]
    lib.ssfm_propagate_adaptive.argtypes = [P, D, D, D, I, P, P, P]
    lib.cavity_roundtrip.argtypes = [P, I]
    lib.opo_sync.argtypes = [P]
    lib.opo_get_fields.argtypes = [P, I, I, I, P]
    lib.opo_set_fields.argtypes = [P, I, I, P]
    lib.opo_get_spectrum_noalloc.argtypes = [P, I, P]
    lib.opo_get_plan.argtypes = [P, I, ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(I)]
    lib.opo_get_progress.argtypes = [P, ctypes.POINTER(I), ctypes.POINTER(D)]
    lib.opo_set_progress.argtypes = [P, I, D, P]
    lib.opo_get_energy_history.argtypes = [P, I, P, I, ctypes.POINTER(I)]
    lib.opo_get_record.argtypes = [P, I, I, I, P]
    lib.opo_get_power_history.argtypes = [P, I, D, P, I, ctypes.POINTER(I)]
    lib.opo_get_grid.argtypes = [P, I, P, P]
    lib.opo_info.argtypes = [P, ctypes.POINTER(I), ctypes.POINTER(D)]
    lib.opo_kernel_times.argtypes = [P, P, P]
    lib.opo_destroy.argtypes = [P]
    lib.opo_last_error.argtypes = []
    lib.opo_last_error.restype = ctypes.c_char_p
    for name in ("opo_init", "opo_init_batch", "ssfm_propagate", "ssfm_propagate_adaptive",
                 "cavity_roundtrip", "opo_sync",
                 "opo_get_fields", "opo_set_fields", "opo_get_spectrum_noalloc", "opo_get_plan",
                 "opo_get_progress", "opo_set_progress",
                 "opo_get_energy_history", "opo_get_record",
                 "opo_get_power_history",
                 "opo_get_grid",
                 "opo_kernel_times", "opo_info", "opo_destroy"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def last_error():
    return load().opo_last_error().decode()


def _check(code):
    if code != OPO_OK:
        raise OpoError(code, last_error())
    return code


def _crystal_struct(c, cr, nz):
    c.length_mm = cr["length_mm"]
    c.nz = int(nz)
    c.deff_pm_per_v = cr["deff_pm_per_v"]
    c.dk_per_mm = cr["dk_per_mm"]
    c.alpha_per_mm = _d3(*cr["alpha_per_mm"])
    c.db1_ps_per_mm = _d3(*cr["db1_ps_per_mm"])
    c.b2_fs2_per_mm = _d3(*cr["b2_fs2_per_mm"])
    c.b3_fs3_per_mm = _d3(*cr["b3_fs3_per_mm"])
    c.n2_m2_per_w = float(cr.get("n2_m2_per_w", 0.0))


def _structs(instances, nz):
    """ctypes arrays for a list of instance dicts (crystal, cavity, fields, pump_in).

    nz is the step count of the crystal, or a list with one per crystal when the instances
    carry "crystals" (crystals per round trip, in order; "crystal" is then the first)."""
    n = len(instances)
    nzs = [int(v) for v in nz] if np.ndim(nz) else [int(nz)]
    kc = len(nzs)
    fields, crystals, cavities = (FieldsT * n)(), (CrystalT * (n * kc))(), (CavityT * n)()
    keep = []
    for i, ins in enumerate(instances):
        crs = ins.get("crystals", [ins["crystal"]])
        if len(crs) != kc:
            raise ValueError("instance %d has %d crystals for %d step counts" % (i, len(crs), kc))
        cr, cav = crs[0], ins["cavity"]
        f = fields[i]
        f.nt = int(cr["nt"])
        nf = int(cr.get("nf", 3))
        f.n_fields = nf
        f.t_window_ps = cr["t_window_ps"]
        f.lambda_um = _d3(*cr["lambda_um"])
        f.n = _d3(*cr["n"])
        init = np.ascontiguousarray(np.asarray(ins["fields"], dtype=np.complex128).reshape(nf, f.nt))
        keep.append(init)
        f.init = init.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        pump = np.asarray(ins.get("pump_in", 0.0), dtype=np.complex128)
        if pump.ndim == 2:                  # (windows, nt): one window per round trip
            pump = np.ascontiguousarray(pump.reshape(-1, f.nt))
            keep.append(pump)
            f.pump_in = pump.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            f.pump_windows = pump.shape[0]
            f.pump_cw = _d2(0.0, 0.0)
        elif pump.ndim == 0 or np.all(pump == pump.flat[0]):
            v = complex(pump.flat[0]) if pump.size else 0j
            f.pump_in = ctypes.POINTER(ctypes.c_double)()
            f.pump_cw = _d2(v.real, v.imag)
        else:
            pump = np.ascontiguousarray(pump.reshape(f.nt))
            keep.append(pump)
            f.pump_in = pump.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            f.pump_cw = _d2(0.0, 0.0)
        for st in range(kc):
            _crystal_struct(crystals[i * kc + st], crs[st], nzs[st])
        k = cavities[i]
        k.resonant = _i3(*[int(v) for v in cav["resonant"]])
        k.refl = _d3(*cav["refl"])
        k.delta_rad = _d3(*cav["delta_rad"])
        k.gdd_fs2 = cav["gdd_fs2"]
        k.gdd_on = _i3(*[int(v) for v in cav["gdd_on"]])
        k.eom_beta = cav["eom_beta"]
        k.eom_fpm_thz = cav["eom_fpm_thz"]
        k.eom_on = _i3(*[int(v) for v in cav["eom_on"]])
    return n, fields, crystals, cavities, keep


class Opo:
    """A handle over one or several OPO instances on one GPU.

    instances: list of dicts with keys crystal, cavity, fields (nf, nt), pump_in; the
    crystal's ``nf`` (default 3) selects three coupled waves or the two-wave degenerate
    model. pump_in of shape (windows, nt) is a long pump read one window per round trip.
    record_rt > 0 keeps the fields leaving the crystal for the first record_rt round trips
    (read with record()). Several crystals per round trip: each instance carries
    "crystals" (in order) and nz is a list of step counts, one per crystal.
    schedule: "auto" (the library's table by shape), "two_pass" or "resident" (see
    opo_options_t.schedule in include/opo.h).
    The field state lives in a torch uint8 tensor on ``device``; the library
    runs on a torch stream (default priority) created for the handle.
    """

    def __init__(self, instances, nz, precision="f32", device=0, col_log2=0,
                 use_graph=True, profile=False, record_rt=0, split_order=2, schedule="auto"):
        import torch
        lib = load()
        self._lib = lib
        self.n, fields, crystals, cavities, keep = _structs(instances, nz)
        self.nts = [int(ins["crystal"]["nt"]) for ins in instances]
        self.nfs = [int(ins["crystal"].get("nf", 3)) for ins in instances]
        self.precision = OPO_F64 if precision in ("f64", OPO_F64) else OPO_F32
        nbytes = lib.opo_state_bytes(self.n, fields, self.precision)
        self._dev = torch.device("cuda", device)
        self._stream = torch.cuda.Stream(self._dev)   # default priority
        self._state = torch.empty(int(nbytes), dtype=torch.uint8, device=self._dev)
        self._state.record_stream(self._stream)
        torch.cuda.current_stream(self._dev).synchronize()
        opt = OptionsT(precision=self.precision, device=device,
                       stream=ctypes.c_void_p(self._stream.cuda_stream),
                       state=ctypes.c_void_p(self._state.data_ptr()), state_bytes=nbytes,
                       col_log2=int(col_log2), schedule=SCHEDULES[schedule], use_graph=1 if use_graph else -1,
                       profile=1 if profile else 0, record_rt=int(record_rt),
                       n_crystals=len(nz) if np.ndim(nz) else 1, split_order=int(split_order))
        h = ctypes.c_void_p()
        _check(lib.opo_init_batch(ctypes.byref(h), self.n, fields, crystals, cavities,
                                  ctypes.byref(opt)))
        del keep
        self.h = h

    # --- the three calls of the boundary
    def ssfm_propagate(self, nz, dz):
        _check(self._lib.ssfm_propagate(self.h, int(nz), float(dz)))

    def ssfm_propagate_adaptive(self, length, tol, dz0, max_attempts=100000):
        """Adaptive-step propagation of every instance over `length` mm (local-error
        method). Returns (accepted, rejected, z_end) arrays, one entry per instance;
        raises OpoError (OPO_ESTEPS) when an instance spends max_attempts first."""
        n = len(self.nts)
        acc = np.zeros(n, np.int32)
        rej = np.zeros(n, np.int32)
        zend = np.zeros(n, np.float64)
        _check(self._lib.ssfm_propagate_adaptive(self.h, float(length), float(tol), float(dz0),
                                                 int(max_attempts), acc.ctypes.data, rej.ctypes.data,
                                                 zend.ctypes.data))
        return acc, rej, zend

    def cavity_roundtrip(self, n_rt):
        return _check(self._lib.cavity_roundtrip(self.h, int(n_rt)))

    def sync(self):
        _check(self._lib.opo_sync(self.h))

    def get_fields(self, inst=0, domain=0):
        nt, nf = self.nts[inst], self.nfs[inst]
        out = np.empty((nf, nt), dtype=np.complex128)
        for x in range(nf):
            buf = np.empty(nt, dtype=np.complex128)
            _check(self._lib.opo_get_fields(self.h, inst, x, domain, buf.ctypes.data))
            out[x] = buf
        return out

    def set_fields(self, a, inst=0):
        nt, nf = self.nts[inst], self.nfs[inst]
        a = np.ascontiguousarray(np.asarray(a, dtype=np.complex128).reshape(nf, nt))
        for x in range(nf):
            row = np.ascontiguousarray(a[x])
            _check(self._lib.opo_set_fields(self.h, inst, x, row.ctypes.data))

    def spectrum_noalloc(self, out, inst=0):
        """Spectra of every field of instance inst into the device tensor `out` (nf * nt
        complex values at the handle's precision, contiguous) through the entry point that
        allocates nothing; queued on the handle's stream (sync() waits)."""
        import torch
        nt, nf = self.nts[inst], self.nfs[inst]
        want = torch.complex128 if self.precision == OPO_F64 else torch.complex64
        if out.dtype != want or out.numel() != nf * nt or not out.is_contiguous() or out.device != self._dev:
            raise ValueError("out must be a contiguous %s tensor of %d values on %s" % (want, nf * nt, self._dev))
        _check(self._lib.opo_get_spectrum_noalloc(self.h, int(inst), ctypes.c_void_p(out.data_ptr())))

    def plan(self, inst=0):
        """(log2 n1, log2 n2, resident) of an instance: its four-step split and whether its
        fixed-step passes run resident."""
        l1, l2, res = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(self._lib.opo_get_plan(self.h, int(inst), ctypes.byref(l1), ctypes.byref(l2), ctypes.byref(res)))
        return l1.value, l2.value, bool(res.value)

    def progress(self):
        """(round trips completed since opo_init, z of the next ssfm_propagate)."""
        rt, z = ctypes.c_int32(), ctypes.c_double()
        _check(self._lib.opo_get_progress(self.h, ctypes.byref(rt), ctypes.byref(z)))
        return rt.value, z.value

    def set_progress(self, rt_done, z, history):
        """Continue as after rt_done round trips, z (see include/opo.h); history has shape
        (rt_done, instances, 3)."""
        hist = np.ascontiguousarray(np.asarray(history, dtype=np.float64).reshape(int(rt_done), self.n, 3))
        _check(self._lib.opo_set_progress(self.h, int(rt_done), float(z),
                                          hist.ctypes.data if rt_done else None))

    def checkpoint(self):
        """Everything a handle built from the same inputs needs to resume this run bit for
        bit: fields of every instance, the energy histories, round trips completed, z."""
        rt, z = self.progress()
        hist = np.stack([self.energy_history(i) for i in range(self.n)], axis=1) if rt else \
            np.zeros((0, self.n, 3))
        return {"fields": [self.get_fields(i) for i in range(self.n)], "history": hist, "rt_done": rt, "z": z}

    def restore(self, ck):
        for i, a in enumerate(ck["fields"]):
            self.set_fields(a, i)
        self.set_progress(ck["rt_done"], ck["z"], ck["history"])

    def energy_history(self, inst=0):
        rows = ctypes.c_int32()
        _check(self._lib.opo_get_energy_history(self.h, inst, None, 0, ctypes.byref(rows)))
        out = np.zeros((rows.value, 3))
        if rows.value:
            _check(self._lib.opo_get_energy_history(self.h, inst, out.ctypes.data, rows.value,
                                                    ctypes.byref(rows)))
        return out

    def power_history(self, area_m2, inst=0):
        """Output powers [W] per round trip (rows, 3) over an effective beam area [m^2]."""
        rows = ctypes.c_int32()
        _check(self._lib.opo_get_power_history(self.h, inst, float(area_m2), None, 0, ctypes.byref(rows)))
        out = np.zeros((rows.value, 3))
        if rows.value:
            _check(self._lib.opo_get_power_history(self.h, inst, float(area_m2), out.ctypes.data, rows.value,
                                                   ctypes.byref(rows)))
        return out

    def record(self, rt, inst=0):
        """Fields (nf, nt) of instance inst as they left the crystal in round trip rt."""
        nt, nf = self.nts[inst], self.nfs[inst]
        out = np.empty((nf, nt), dtype=np.complex128)
        for x in range(nf):
            buf = np.empty(nt, dtype=np.complex128)
            _check(self._lib.opo_get_record(self.h, inst, x, int(rt), buf.ctypes.data))
            out[x] = buf
        return out

    def grid(self, inst=0):
        nt = self.nts[inst]
        t, w = np.empty(nt), np.empty(nt)
        _check(self._lib.opo_get_grid(self.h, inst, t.ctypes.data, w.ctypes.data))
        return t, w

    def kernel_times(self):
        """{kernel class: (total device ms, launches)} under the profile option."""
        ms = np.zeros(len(KERNEL_CLASSES))
        n = np.zeros(len(KERNEL_CLASSES), dtype=np.int64)
        _check(self._lib.opo_kernel_times(self.h, ms.ctypes.data, n.ctypes.data))
        return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(KERNEL_CLASSES)}

    @property
    def stream(self):
        return self._stream

    def info(self):
        n, z = ctypes.c_int32(), ctypes.c_double()
        _check(self._lib.opo_info(self.h, ctypes.byref(n), ctypes.byref(z)))
        return n.value, z.value

    def close(self):
        if getattr(self, "h", None):
            _check(self._lib.opo_destroy(self.h))
            self.h = None
            self._state = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def from_workload(w, precision=None, **kw):
    """Handle for a workload dict of the workloads module (single or batched)."""
    insts = w["instances"] if "instances" in w else [w]
    return Opo(insts, w["nz"], precision=precision or w.get("precision", "f32"), **kw)
