"""Python binding of the MI355X QED Monte Carlo library (``libqedmi.so``).

Argument marshalling only: every call goes through the C ABI declared in
``include/qedmi.h`` and every step of the computation runs in the library's
HIP kernels.  PyTorch tensors are used only as device memory and for the
current stream.  Importing the package does not require a GPU; calling
into the library does, and fails loudly when ``libqedmi.so`` is missing.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqedmi.so")

QED_OK, QED_ERR_INVALID, QED_ERR_HIP, QED_ERR_ALLOC, QED_ERR_CAPACITY, QED_ERR_IO, QED_ERR_STATE = \
    0, -1, -2, -3, -4, -5, -6
FP64, FP32, BF16 = 0, 1, 2
BW, QS = 0, 1
ELECTRON, POSITRON, PHOTON, ION = 0, 1, 2, 3
CHI_FP64, CHI_COMP32, CHI_FP32 = 0, 1, 2
STAT_UPDATES, STAT_QS_EVENTS, STAT_BW_EVENTS, STAT_PHOTONS_KEPT = 0, 1, 2, 3
STAT_SURR_BATCHES, STAT_SURR_FALLBACK, STAT_NONFINITE, STAT_SCAN_TIMEOUT, STATS_LEN = 4, 5, 6, 7, 8
SURR_NPARAM = 64 * 2 + 64 + 64 * 64 + 64 + 64 + 1

# Every symbol the header declares (checked by the CPU test suite).
EXPORTS = (
    "qed_table_generate", "qed_table_from_host", "qed_table_save", "qed_table_load",
    "qed_table_host_data", "qed_table_to_device", "qed_table_destroy", "qed_table_generate_device",
    "qed_context_create", "qed_context_destroy", "qed_context_set_units",
    "qed_chi_lepton", "qed_chi_photon", "qed_init_optical_depth", "qed_evolve_optical_depth",
    "qed_generate_pairs", "qed_generate_photon_and_update_momentum", "qed_step", "qed_step_noalloc", "qed_read_count",
    "qed_table_rate", "qed_table_sample",
    "qed_surrogate_train", "qed_surrogate_from_host", "qed_surrogate_get_params", "qed_surrogate_bands",
    "qed_surrogate_forward", "qed_surrogate_grad", "qed_surrogate_sample", "qed_surrogate_destroy",
    "qed_schwinger_rate", "qed_schwinger_pairs", "qed_push", "qed_traffic_calibrate",
    "qed_last_error", "qed_version",
)


class QedError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"qedmi error {code}: {msg}")
        self.code = code


class TableParams(C.Structure):
    _fields_ = [("process", C.c_int32), ("n_chi", C.c_int32), ("n_frac", C.c_int32),
                ("n_threads", C.c_int32), ("chi_min", C.c_double), ("chi_max", C.c_double),
                ("frac_min", C.c_double)]


class ParticlesC(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("ux", "uy", "uz", "ex", "ey", "ez", "bx", "by", "bz", "tau", "w")] + \
               [("n", C.c_int64), ("id_base", C.c_int64), ("species", C.c_int32), ("dtype", C.c_int32)]


class AppendC(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("ux", "uy", "uz", "w", "tau")] + \
               [("parent", C.c_void_p), ("count", C.c_void_p), ("capacity", C.c_int64),
                ("dtype", C.c_int32), ("pad_", C.c_int32)]


class StepDescC(C.Structure):
    _fields_ = [("bw", C.c_void_p), ("qs", C.c_void_p), ("bw_surrogate", C.c_void_p),
                ("qs_surrogate", C.c_void_p), ("sets", C.POINTER(ParticlesC)), ("n_sets", C.c_int32),
                ("n_tiles", C.c_int32), ("tiles", C.POINTER(C.c_int64)), ("photons", C.POINTER(AppendC)),
                ("electrons", C.POINTER(AppendC)), ("positrons", C.POINTER(AppendC)),
                ("flags", C.POINTER(C.c_void_p)), ("stats", C.c_void_p), ("dt", C.c_double),
                ("seed", C.c_uint64), ("step", C.c_uint64), ("photon_min_energy", C.c_double),
                ("chi_mode", C.c_int32), ("pad_", C.c_int32), ("chi_qed_min", C.c_double)]


class CellsC(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("ex", "ey", "ez", "bx", "by", "bz")] + \
               [("n", C.c_int64), ("cell_id_base", C.c_int64), ("dtype", C.c_int32), ("pad_", C.c_int32)]


class UnitsC(C.Structure):
    _fields_ = [("system", C.c_int32), ("pad_", C.c_int32), ("ref", C.c_double)]


UNITS_SI, UNITS_NORM_OMEGA, UNITS_NORM_LAMBDA, UNITS_HL_MEV = 0, 1, 2, 3


class FieldC(C.Structure):
    _fields_ = [("kind", C.c_int32), ("direction", C.c_int32), ("e0", C.c_double * 3), ("b0", C.c_double * 3),
                ("amplitude", C.c_double), ("wavelength", C.c_double), ("phase", C.c_double)]


class SurrogateCfg(C.Structure):
    _fields_ = [("process", C.c_int32), ("n_samples", C.c_int32), ("batch", C.c_int32),
                ("steps", C.c_int32), ("lr", C.c_float), ("probe_tol", C.c_float),
                ("chi_lo", C.c_double), ("chi_hi", C.c_double), ("seed", C.c_uint64),
                ("probe_every", C.c_int32), ("tail_permille", C.c_int32),
                ("ks_budget", C.c_float), ("pad_", C.c_int32)]


_lib = None


def lib():
    """Load libqedmi.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2110_00256_amd/build.py")
        L = C.CDLL(LIB_PATH)
        i32, vp, d, u64, i64 = C.c_int32, C.c_void_p, C.c_double, C.c_uint64, C.c_int64
        P = C.POINTER
        sig = {
            "qed_table_generate": [P(TableParams), P(vp)],
            "qed_table_generate_device": [P(TableParams), P(vp), vp],
            "qed_table_from_host": [P(TableParams), vp, vp, P(vp)],
            "qed_table_save": [vp, C.c_char_p],
            "qed_table_load": [C.c_char_p, P(vp)],
            "qed_table_host_data": [vp, P(vp), P(vp), P(TableParams)],
            "qed_table_to_device": [vp, vp],
            "qed_context_create": [i32, P(vp)],
            "qed_context_set_units": [vp, P(UnitsC)],
            "qed_chi_lepton": [vp, P(ParticlesC), i32, vp, vp],
            "qed_chi_photon": [vp, P(ParticlesC), i32, vp, vp],
            "qed_init_optical_depth": [vp, P(ParticlesC), u64, vp],
            "qed_evolve_optical_depth": [vp, vp, P(ParticlesC), d, i32, vp, vp],
            "qed_generate_pairs": [vp, vp, P(ParticlesC), vp, u64, u64, i32, P(AppendC), P(AppendC), vp],
            "qed_generate_photon_and_update_momentum": [vp, vp, P(ParticlesC), vp, u64, u64, i32, d,
                                                        P(AppendC), vp],
            "qed_step": [vp, P(StepDescC), vp],
            "qed_step_noalloc": [vp, P(StepDescC), vp],
            "qed_read_count": [P(AppendC), P(i64), vp],
            "qed_table_rate": [vp, i32, vp, vp, vp, i64, vp],
            "qed_table_sample": [vp, i32, vp, vp, vp, vp, i64, vp],
            "qed_surrogate_train": [vp, vp, P(SurrogateCfg), P(vp), P(C.c_float), vp],
            "qed_surrogate_from_host": [vp, P(SurrogateCfg), vp, P(vp)],
            "qed_surrogate_get_params": [vp, vp],
            "qed_surrogate_bands": [vp, vp, P(u64)],
            "qed_surrogate_forward": [vp, vp, vp, i64, vp],
            "qed_surrogate_grad": [vp, vp, vp, i64, vp, vp, vp],
            "qed_surrogate_sample": [vp, vp, vp, vp, i64, vp],
            "qed_schwinger_rate": [vp, P(CellsC), vp, vp],
            "qed_schwinger_pairs": [vp, P(CellsC), d, d, d, u64, u64, P(AppendC), P(AppendC), vp],
            "qed_push": [vp, P(ParticlesC), vp, vp, vp, P(FieldC), d, d, vp],
            "qed_traffic_calibrate": [vp, vp, i64, i32, vp],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = i32
        for name in ("qed_table_destroy", "qed_context_destroy", "qed_surrogate_destroy"):
            getattr(L, name).argtypes = [vp]
            getattr(L, name).restype = None
        L.qed_last_error.restype = C.c_char_p
        L.qed_version.restype = C.c_char_p
        _lib = L
    return _lib


def check(code):
    if code != QED_OK:
        raise QedError(code, lib().qed_last_error().decode())
    return code


def _stream(stream=None):
    if stream is not None:
        return C.c_void_p(int(stream))
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


# ------------------------------------------------------------------ tables
class Table:
    """Library-owned lookup table (qed_table*)."""

    def __init__(self, handle, keep=None):
        self.h = C.c_void_p(handle)
        self._keep = keep

    @classmethod
    def generate(cls, process, chi_min, chi_max, n_chi, n_frac, frac_min=1e-12, n_threads=0):
        p = TableParams(process, n_chi, n_frac, n_threads, chi_min, chi_max, frac_min)
        h = C.c_void_p()
        check(lib().qed_table_generate(C.byref(p), C.byref(h)))
        return cls(h.value)

    @classmethod
    def generate_device(cls, process, chi_min, chi_max, n_chi, n_frac, frac_min=1e-12, stream=None):
        """Generate on the current GPU (FP64 HIP quadrature); synchronous."""
        p = TableParams(process, n_chi, n_frac, 0, chi_min, chi_max, frac_min)
        h = C.c_void_p()
        check(lib().qed_table_generate_device(C.byref(p), C.byref(h), _stream(stream)))
        return cls(h.value)

    @classmethod
    def from_host(cls, process, chi_min, chi_max, ln_rate, cdf, frac_min=1e-12):
        import numpy as np
        ln_rate = np.ascontiguousarray(ln_rate, dtype=np.float64)
        cdf = np.ascontiguousarray(cdf, dtype=np.float64)
        p = TableParams(process, ln_rate.shape[0], cdf.shape[-1], 0, chi_min, chi_max, frac_min)
        h = C.c_void_p()
        check(lib().qed_table_from_host(C.byref(p), ln_rate.ctypes.data, cdf.ctypes.data, C.byref(h)))
        return cls(h.value)

    @classmethod
    def load(cls, path):
        h = C.c_void_p()
        check(lib().qed_table_load(os.fsencode(path), C.byref(h)))
        return cls(h.value)

    def save(self, path):
        check(lib().qed_table_save(self.h, os.fsencode(path)))

    def host_data(self):
        """(params, ln_rate copy, cdf copy) as numpy arrays."""
        import numpy as np
        a, b = C.c_void_p(), C.c_void_p()
        p = TableParams()
        check(lib().qed_table_host_data(self.h, C.byref(a), C.byref(b), C.byref(p)))
        lr = np.ctypeslib.as_array(C.cast(a, C.POINTER(C.c_double)), (p.n_chi,)).copy()
        cdf = np.ctypeslib.as_array(C.cast(b, C.POINTER(C.c_double)), (p.n_chi, p.n_frac)).copy()
        return p, lr, cdf

    def to_device(self, stream=None):
        check(lib().qed_table_to_device(self.h, _stream(stream)))
        return self

    def __del__(self):
        if getattr(self, "h", None) is not None and self.h.value and _lib is not None:
            _lib.qed_table_destroy(self.h)
            self.h = None


class Context:
    def __init__(self, device=0):
        h = C.c_void_p()
        check(lib().qed_context_create(device, C.byref(h)))
        self.h = h

    def set_units(self, system, ref=0.0):
        """Unit system of the arrays and scalars of every call through this context."""
        check(lib().qed_context_set_units(self.h, C.byref(UnitsC(system, 0, float(ref)))))

    def __del__(self):
        if getattr(self, "h", None) is not None and self.h.value and _lib is not None:
            _lib.qed_context_destroy(self.h)
            self.h = None


def table_rate(table: Table, chi, gamma, out, stream=None, bf16_tables=False):
    dt = BF16 if bf16_tables else dtype_code(chi)
    check(lib().qed_table_rate(table.h, dt, _ptr(chi), _ptr(gamma), _ptr(out), chi.numel(), _stream(stream)))


def table_sample(table: Table, chi, u, out, electron_selected=None, stream=None, bf16_tables=False):
    dt = BF16 if bf16_tables else dtype_code(chi)
    check(lib().qed_table_sample(table.h, dt, _ptr(chi), _ptr(u), _ptr(out), _ptr(electron_selected),
                                 chi.numel(), _stream(stream)))


# --------------------------------------------------------------- particles
KEYS = ("ux", "uy", "uz", "ex", "ey", "ez", "bx", "by", "bz", "tau", "w")


def dtype_code(t):
    import torch
    if t.dtype == torch.float64:
        return FP64
    if t.dtype == torch.float32:
        return FP32
    raise TypeError("particle arrays must be float64 or float32")


def particles(arrs: dict, species: int, id_base: int = 0):
    """qed_particles over a dict of contiguous device tensors (keys KEYS;
    'w' optional).  The caller keeps the tensors alive."""
    ref = arrs["ux"]
    n = ref.numel()
    for k in KEYS:
        t = arrs.get(k)
        if t is not None:
            assert t.is_contiguous() and t.numel() == n and t.dtype == ref.dtype, k
    return ParticlesC(*[_ptr(arrs.get(k)) for k in KEYS], n, id_base, species, dtype_code(ref))


class AppendBuffer:
    """Device product buffer: SoA arrays, parent ids and a device count."""

    def __init__(self, capacity, dtype, device="cuda"):
        import torch
        self.capacity = int(capacity)
        cap = max(self.capacity, 1)
        self.a = {k: torch.zeros(cap, dtype=dtype, device=device) for k in ("ux", "uy", "uz", "w", "tau")}
        self.parent = torch.full((cap,), -1, dtype=torch.int64, device=device)
        self.count = torch.zeros(1, dtype=torch.int64, device=device)
        self.c = AppendC(*[_ptr(self.a[k]) for k in ("ux", "uy", "uz", "w", "tau")], _ptr(self.parent),
                         _ptr(self.count), self.capacity, dtype_code(self.a["ux"]), 0)

    def read_count(self, stream=None):
        v = C.c_int64()
        code = lib().qed_read_count(C.byref(self.c), C.byref(v), _stream(stream))
        if code not in (QED_OK, QED_ERR_CAPACITY):
            check(code)
        return v.value

    def reset(self):
        self.count.zero_()

    def __getitem__(self, k):
        n = min(int(self.count.item()), self.capacity)
        return (self.parent if k == "parent" else self.a[k])[:n]


# ------------------------------------------------------------- entry points
def chi_lepton(ctx, p: ParticlesC, chi_out, chi_mode=CHI_FP64, stream=None):
    check(lib().qed_chi_lepton(ctx.h, C.byref(p), chi_mode, _ptr(chi_out), _stream(stream)))


def chi_photon(ctx, p: ParticlesC, chi_out, chi_mode=CHI_FP64, stream=None):
    check(lib().qed_chi_photon(ctx.h, C.byref(p), chi_mode, _ptr(chi_out), _stream(stream)))


def init_optical_depth(ctx, p: ParticlesC, seed, stream=None):
    check(lib().qed_init_optical_depth(ctx.h, C.byref(p), seed, _stream(stream)))


def evolve_optical_depth(ctx, table: Table, p: ParticlesC, dt, flags=None, chi_mode=CHI_FP64, stream=None):
    check(lib().qed_evolve_optical_depth(ctx.h, table.h, C.byref(p), dt, chi_mode, _ptr(flags), _stream(stream)))


def generate_pairs(ctx, bw: Table, photons: ParticlesC, flags, seed, step, electrons: AppendBuffer,
                   positrons: AppendBuffer, chi_mode=CHI_FP64, stream=None):
    check(lib().qed_generate_pairs(ctx.h, bw.h, C.byref(photons), _ptr(flags), seed, step, chi_mode,
                                   C.byref(electrons.c), C.byref(positrons.c), _stream(stream)))


def generate_photon_and_update_momentum(ctx, qs: Table, leptons: ParticlesC, flags, seed, step,
                                        photons: AppendBuffer, photon_min_energy=0.0, chi_mode=CHI_FP64,
                                        stream=None):
    check(lib().qed_generate_photon_and_update_momentum(ctx.h, qs.h, C.byref(leptons), _ptr(flags), seed, step,
                                                        chi_mode, photon_min_energy, C.byref(photons.c),
                                                        _stream(stream)))


class StepDesc:
    """Holds a qed_step_desc and everything it points to."""

    def __init__(self, sets, bw=None, qs=None, photons=None, electrons=None, positrons=None, tiles=None,
                 flags=None, stats=None, dt=0.0, seed=1, step=0, photon_min_energy=0.0, chi_mode=CHI_FP64,
                 bw_surrogate=None, qs_surrogate=None, chi_qed_min=0.0):
        self._sets = (ParticlesC * len(sets))(*sets)
        self._keep = [bw, qs, photons, electrons, positrons, tiles, flags, stats, bw_surrogate, qs_surrogate]
        fl = None
        if flags is not None:
            fl = (C.c_void_p * len(sets))(*[(f.data_ptr() if f is not None else None) for f in flags])
            self._keep.append(fl)
        tl = None
        if tiles is not None:
            import numpy as np
            self._tiles = np.ascontiguousarray(tiles, dtype=np.int64).reshape(-1)
            tl = self._tiles.ctypes.data_as(C.POINTER(C.c_int64))
        self.c = StepDescC(
            bw.h if bw else None, qs.h if qs else None,
            bw_surrogate.h if bw_surrogate else None, qs_surrogate.h if qs_surrogate else None,
            self._sets, len(sets), 0 if tiles is None else len(self._tiles) // 3, tl,
            C.pointer(photons.c) if photons else None, C.pointer(electrons.c) if electrons else None,
            C.pointer(positrons.c) if positrons else None, fl,
            stats.data_ptr() if stats is not None else None, dt, seed, step, photon_min_energy, chi_mode, 0,
            chi_qed_min)

    def set_step(self, step):
        self.c.step = step


def step(ctx, desc: StepDesc, stream=None):
    check(lib().qed_step(ctx.h, C.byref(desc.c), _stream(stream)))


def step_noalloc(ctx, desc: StepDesc, stream=None):
    """qed_step_noalloc: the same step with the library's fixed per-GPU
    scratch (ctx may be None: SI units, current device)."""
    check(lib().qed_step_noalloc(ctx.h if ctx is not None else None, C.byref(desc.c), _stream(stream)))


def traffic_calibrate(src, dst, n_bytes, mode, stream=None):
    """qed_traffic_calibrate: stream n_bytes with the step's access pattern
    (mode 0 read src, 1 write dst, 2 copy), for counter calibration."""
    check(lib().qed_traffic_calibrate(_ptr(src), _ptr(dst), int(n_bytes), int(mode), _stream(stream)))


def version():
    return lib().qed_version().decode()


# --------------------------------------------------------------- surrogate
class Surrogate:
    """Learned inverse CDF (qed_surrogate*)."""

    def __init__(self, handle, table):
        self.h = C.c_void_p(handle)
        self._table = table

    @staticmethod
    def cfg(process, chi_lo, chi_hi, n_samples=1 << 22, batch=16384, steps=20000, lr=3e-3, probe_tol=0.5,
            seed=7, probe_every=16, tail_permille=0, ks_budget=0.0):
        return SurrogateCfg(process, n_samples, batch, steps, lr, probe_tol, chi_lo, chi_hi, seed, probe_every,
                            tail_permille, ks_budget, 0)

    @classmethod
    def train(cls, ctx, table, cfg, stream=None):
        h = C.c_void_p()
        loss = C.c_float()
        check(lib().qed_surrogate_train(ctx.h, table.h, C.byref(cfg), C.byref(h), C.byref(loss), _stream(stream)))
        return cls(h.value, table), loss.value

    @classmethod
    def from_host(cls, table, cfg, params):
        import numpy as np
        p = np.ascontiguousarray(params, dtype=np.float32)
        assert p.size == SURR_NPARAM
        h = C.c_void_p()
        check(lib().qed_surrogate_from_host(table.h, C.byref(cfg), p.ctypes.data, C.byref(h)))
        return cls(h.value, table)

    def bands(self):
        """(per-band largest CDF-space error, served-band mask)."""
        import numpy as np
        err = np.zeros(64, dtype=np.float32)
        mask = C.c_uint64()
        check(lib().qed_surrogate_bands(self.h, err.ctypes.data, C.byref(mask)))
        return err, mask.value

    def params(self):
        import numpy as np
        p = np.zeros(SURR_NPARAM, dtype=np.float32)
        check(lib().qed_surrogate_get_params(self.h, p.ctypes.data))
        return p

    def forward(self, x, y, stream=None):
        check(lib().qed_surrogate_forward(self.h, _ptr(x), _ptr(y), y.numel(), _stream(stream)))

    def grad(self, x, t, grad, loss, stream=None):
        check(lib().qed_surrogate_grad(self.h, _ptr(x), _ptr(t), t.numel(), _ptr(grad), _ptr(loss),
                                       _stream(stream)))

    def sample(self, chi, u, out, stream=None):
        check(lib().qed_surrogate_sample(self.h, _ptr(chi), _ptr(u), _ptr(out), chi.numel(), _stream(stream)))

    def __del__(self):
        if getattr(self, "h", None) is not None and self.h.value and _lib is not None:
            _lib.qed_surrogate_destroy(self.h)
            self.h = None


# ---------------------------------------------------------------- Schwinger
def cells(d: dict, cell_id_base=0) -> CellsC:
    """Cell view of device field tensors ex, ey, ez, bx, by, bz (one dtype)."""
    t = d["ex"]
    return CellsC(*[_ptr(d[k]) for k in ("ex", "ey", "ez", "bx", "by", "bz")], t.numel(), int(cell_id_base),
                  dtype_code(t), 0)


def schwinger_rate(ctx, c: CellsC, rate_out, stream=None):
    check(lib().qed_schwinger_rate(ctx.h, C.byref(c), _ptr(rate_out), _stream(stream)))


def schwinger_pairs(ctx, c: CellsC, cell_volume, dt, weight, seed, step, electrons: AppendBuffer,
                    positrons: AppendBuffer, stream=None):
    check(lib().qed_schwinger_pairs(ctx.h, C.byref(c), float(cell_volume), float(dt), float(weight), seed, step,
                                    C.byref(electrons.c), C.byref(positrons.c), _stream(stream)))


# -------------------------------------------------------------------- push
FIELD_UNIFORM, FIELD_CP_WAVE = 0, 1


def uniform_field(e0=(0.0, 0.0, 0.0), b0=(0.0, 0.0, 0.0)) -> FieldC:
    return FieldC(FIELD_UNIFORM, 1, (C.c_double * 3)(*e0), (C.c_double * 3)(*b0), 0.0, 0.0, 0.0)


def cp_wave(amplitude, wavelength, direction=1, phase=0.0) -> FieldC:
    return FieldC(FIELD_CP_WAVE, direction, (C.c_double * 3)(), (C.c_double * 3)(), amplitude, wavelength, phase)


def push(ctx, p: ParticlesC, x, y, z, field: FieldC, t, dt, stream=None):
    check(lib().qed_push(ctx.h, C.byref(p), _ptr(x), _ptr(y), _ptr(z), C.byref(field), float(t), float(dt),
                         _stream(stream)))
