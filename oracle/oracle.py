"""ctypes front end of the CPU oracle (``qed_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and
the CPU-baseline leg of the benchmark; never by the library.  It exposes the
oracle's FP64 functions on numpy arrays.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qed_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

BW, QS = 0, 1
ELECTRON, POSITRON, PHOTON, ION = 0, 1, 2, 3
INIT_STEP = (1 << 64) - 1

_dp = C.POINTER(C.c_double)
_u8p = C.POINTER(C.c_uint8)
_i64p = C.POINTER(C.c_int64)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no FP contraction, OpenMP)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-shared", "-fPIC",
               "-o", _LIB + ".tmp", _SRC, "-lquadmath", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Table(C.Structure):
    _fields_ = [("proc", C.c_int), ("n_chi", C.c_int), ("n_frac", C.c_int),
                ("chi_min", C.c_double), ("chi_max", C.c_double), ("frac_min", C.c_double),
                ("ln_rate", _dp), ("cdf", _dp)]


class _Particles(C.Structure):
    _fields_ = [(k, _dp) for k in ("ux", "uy", "uz", "ex", "ey", "ez", "bx", "by", "bz", "tau", "w")] + \
               [("n", C.c_int64), ("id_base", C.c_int64), ("species", C.c_int32)]


class _Field(C.Structure):
    _fields_ = [("kind", C.c_int), ("dir", C.c_int), ("e0", C.c_double * 3), ("b0", C.c_double * 3),
                ("amp", C.c_double), ("lam", C.c_double), ("phase", C.c_double)]


class _Append(C.Structure):
    _fields_ = [(k, _dp) for k in ("ux", "uy", "uz", "w", "tau")] + \
               [("parent", _i64p), ("capacity", C.c_int64), ("count", C.c_int64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        d, i, u64, vp = C.c_double, C.c_int, C.c_uint64, C.c_void_p
        L.orc_schwinger_field.restype = d
        L.orc_rate_prefactor.restype = d
        L.orc_philox4x64_10.argtypes = [C.POINTER(u64), C.POINTER(u64), C.POINTER(u64)]
        L.orc_u01.argtypes = [u64]; L.orc_u01.restype = d
        L.orc_draws.argtypes = [u64, u64, u64, u64, u64, _dp]
        L.orc_bessel_pair_scaled.argtypes = [d, d, d, _dp, _dp]
        for f in ("orc_bessel_k", "orc_bessel_ik"):
            getattr(L, f).argtypes = [d, d]; getattr(L, f).restype = d
        L.orc_table_row.argtypes = [i, d, i, d, _dp, _dp]
        L.orc_grid_chi.argtypes = [d, d, i, i]; L.orc_grid_chi.restype = d
        L.orc_table_generate.argtypes = [i, d, d, i, i, d, _dp, _dp]
        for f in ("orc_bw_T", "orc_qs_G"):
            getattr(L, f).argtypes = [d]; getattr(L, f).restype = d
        for f in ("orc_bw_cdf_at", "orc_qs_cdf_at"):
            getattr(L, f).argtypes = [d, d]; getattr(L, f).restype = d
        for f in ("orc_chi_lepton", "orc_chi_photon"):
            getattr(L, f).argtypes = [d] * 9; getattr(L, f).restype = d
        L.orc_chi_literal_q.argtypes = [d] * 9 + [i]; L.orc_chi_literal_q.restype = d
        L.orc_chi_literal_q_n.argtypes = [C.c_int64] + [_dp] * 9 + [i, _dp]
        L.orc_rate_bw.argtypes = [C.POINTER(_Table), d, d]; L.orc_rate_bw.restype = d
        L.orc_rate_qs.argtypes = [C.POINTER(_Table), d, d]; L.orc_rate_qs.restype = d
        L.orc_sample_bw.argtypes = [C.POINTER(_Table), d, d, C.POINTER(C.c_int)]
        L.orc_sample_bw.restype = d
        L.orc_sample_qs_lnxi.argtypes = [C.POINTER(_Table), d, d]; L.orc_sample_qs_lnxi.restype = d
        L.orc_init_optical_depth.argtypes = [C.POINTER(_Particles), u64]
        L.orc_step.argtypes = [C.POINTER(_Table), C.POINTER(_Table), C.POINTER(_Particles), d, u64, u64,
                               d, d, _u8p, C.POINTER(_Append), C.POINTER(_Append)]
        L.orc_step.restype = C.c_int64
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_set_threads.restype = None
        L.orc_max_threads.argtypes = []
        L.orc_max_threads.restype = C.c_int
        L.orc_generate.argtypes = [C.POINTER(_Table), C.POINTER(_Table), C.POINTER(_Particles), _u8p,
                                   u64, u64, d, C.POINTER(_Append), C.POINTER(_Append)]
        L.orc_generate.restype = C.c_int64
        L.orc_evolve.argtypes = [C.POINTER(_Table), C.POINTER(_Particles), d, _u8p]
        L.orc_chi_n.argtypes = [C.c_int64] + [_dp] * 9 + [i, _dp]
        L.orc_rate_n.argtypes = [C.POINTER(_Table), C.c_int64, _dp, _dp, _dp]
        L.orc_sample_n.argtypes = [C.POINTER(_Table), C.c_int64, _dp, _dp, _dp, _u8p]
        L.orc_mlp_grad.argtypes = [_dp, C.c_int64, _dp, _dp, _dp, _dp, _dp, i]
        L.orc_mlp_grad.restype = d
        L.orc_compact.argtypes = [C.c_int64, _i64p, C.POINTER(C.c_int32), C.POINTER(_u8p), _i64p, C.c_int32,
                                  _i64p, C.c_int64]
        L.orc_compact.restype = C.c_int64
        L.orc_schwinger_rate.argtypes = [d] * 6; L.orc_schwinger_rate.restype = d
        L.orc_schwinger_rate_n.argtypes = [C.c_int64] + [_dp] * 7
        L.orc_schwinger_count.argtypes = [d, C.c_uint64, C.c_uint64, C.c_uint64, _dp]
        L.orc_schwinger_count.restype = C.c_int64
        L.orc_schwinger_pairs.argtypes = [C.c_int64] + [_dp] * 6 + [C.c_int64, d, d, d, C.c_uint64, C.c_uint64,
                                                                 C.POINTER(_Append), C.POINTER(_Append)]
        L.orc_schwinger_pairs.restype = C.c_int64
        L.orc_push.argtypes = [C.POINTER(_Particles), _dp, _dp, _dp, C.POINTER(_Field), d, d]
        _lib = L
    return _lib


def _ptr(a, t=_dp):
    return a.ctypes.data_as(t)


# ---------------------------------------------------------------- scalars
def schwinger_field() -> float:
    return lib().orc_schwinger_field()


def rate_prefactor() -> float:
    return lib().orc_rate_prefactor()


def philox_block(ctr, key):
    c = (C.c_uint64 * 4)(*[int(x) & 0xFFFFFFFFFFFFFFFF for x in ctr])
    k = (C.c_uint64 * 2)(*[int(x) & 0xFFFFFFFFFFFFFFFF for x in key])
    o = (C.c_uint64 * 4)()
    lib().orc_philox4x64_10(c, k, o)
    return [int(x) for x in o]


def u01(w: int) -> float:
    return lib().orc_u01(w)


def draws(seed, pid, step, species, block=0):
    out = np.zeros(4)
    lib().orc_draws(seed, pid, step & 0xFFFFFFFFFFFFFFFF, species, block, _ptr(out))
    return out


def bessel_k(nu, x):
    return lib().orc_bessel_k(nu, x)


def bessel_ik(nu, x):
    return lib().orc_bessel_ik(nu, x)


def bessel_pair_scaled(x, nu_k, nu_ik):
    a, b = C.c_double(), C.c_double()
    lib().orc_bessel_pair_scaled(x, nu_k, nu_ik, C.byref(a), C.byref(b))
    return a.value, b.value


def bw_T(chi):
    return lib().orc_bw_T(chi)


def qs_G(chi):
    return lib().orc_qs_G(chi)


def bw_cdf_at(chi, xi):
    return lib().orc_bw_cdf_at(chi, xi)


def qs_cdf_at(chi, xi):
    return lib().orc_qs_cdf_at(chi, xi)


def chi_lepton(*a):
    return lib().orc_chi_lepton(*[float(x) for x in a])


def chi_photon(*a):
    return lib().orc_chi_photon(*[float(x) for x in a])


def chi_literal_q(*a, photon=False):
    return lib().orc_chi_literal_q(*[float(x) for x in a], int(photon))


def chi_literal_q_array(pop: dict, photon: bool) -> np.ndarray:
    """The printed chi formula in binary128 for every particle of pop."""
    keys = ("ux", "uy", "uz", "ex", "ey", "ez", "bx", "by", "bz")
    cols = [np.ascontiguousarray(pop[k], dtype=np.float64) for k in keys]
    out = np.zeros(len(cols[0]))
    lib().orc_chi_literal_q_n(len(out), *[_ptr(c) for c in cols], int(photon), _ptr(out))
    return out


def chi_array(pop: dict, photon: bool) -> np.ndarray:
    keys = ("ux", "uy", "uz", "ex", "ey", "ez", "bx", "by", "bz")
    cols = [np.ascontiguousarray(pop[k], dtype=np.float64) for k in keys]
    out = np.zeros(len(cols[0]))
    lib().orc_chi_n(len(out), *[_ptr(c) for c in cols], int(photon), _ptr(out))
    return out


# ---------------------------------------------------------------- tables
class Table:
    """Oracle lookup table for one process (BW or QS)."""

    def __init__(self, proc, chi_min, chi_max, n_chi, n_frac, frac_min=1e-12,
                 ln_rate=None, cdf=None):
        self.proc, self.chi_min, self.chi_max = proc, float(chi_min), float(chi_max)
        self.n_chi, self.n_frac, self.frac_min = int(n_chi), int(n_frac), float(frac_min)
        if ln_rate is None:
            ln_rate = np.zeros(n_chi)
            cdf = np.zeros((n_chi, n_frac))
            lib().orc_table_generate(proc, self.chi_min, self.chi_max, self.n_chi, self.n_frac,
                                     self.frac_min, _ptr(ln_rate), _ptr(cdf))
        self.ln_rate = np.ascontiguousarray(ln_rate, dtype=np.float64)
        self.cdf = np.ascontiguousarray(cdf, dtype=np.float64).reshape(n_chi, n_frac)
        self._c = _Table(proc, self.n_chi, self.n_frac, self.chi_min, self.chi_max, self.frac_min,
                         _ptr(self.ln_rate), _ptr(self.cdf))

    @property
    def cstruct(self):
        return C.byref(self._c)

    def chi_grid(self):
        return np.array([lib().orc_grid_chi(self.chi_min, self.chi_max, self.n_chi, n)
                         for n in range(self.n_chi)])

    def frac_grid(self):
        N = self.n_frac
        if self.proc == BW:
            return 0.5 * np.arange(N) / (N - 1)
        lmin = np.log(self.frac_min)
        g = np.exp(lmin * (1.0 - np.arange(N) / (N - 1)))
        g[-1] = 1.0
        return g

    def rate(self, chi, gamma):
        f = lib().orc_rate_bw if self.proc == BW else lib().orc_rate_qs
        return f(self.cstruct, float(chi), float(gamma))

    def sample_bw(self, chi, r):
        e = C.c_int()
        xi = lib().orc_sample_bw(self.cstruct, float(chi), float(r), C.byref(e))
        return xi, bool(e.value)

    def sample_qs_lnxi(self, chi, r):
        return lib().orc_sample_qs_lnxi(self.cstruct, float(chi), float(r))

    def rate_n(self, chi, gamma):
        chi = np.ascontiguousarray(chi, dtype=np.float64)
        gamma = np.ascontiguousarray(np.broadcast_to(gamma, chi.shape), dtype=np.float64)
        out = np.zeros(chi.shape)
        lib().orc_rate_n(self.cstruct, chi.size, _ptr(chi), _ptr(gamma), _ptr(out))
        return out

    def sample_n(self, chi, r):
        """BW: (xi, electron_selected); QS: ln xi."""
        r = np.ascontiguousarray(r, dtype=np.float64)
        chi = np.ascontiguousarray(np.broadcast_to(chi, r.shape), dtype=np.float64)
        out = np.zeros(r.shape)
        sel = np.zeros(r.shape, dtype=np.uint8)
        lib().orc_sample_n(self.cstruct, r.size, _ptr(chi), _ptr(r), _ptr(out), _ptr(sel, _u8p))
        return (out, sel.astype(bool)) if self.proc == BW else out


def table_row(proc, chi, n_frac, frac_min=1e-12):
    row = np.zeros(n_frac)
    lr = C.c_double()
    lib().orc_table_row(proc, float(chi), int(n_frac), float(frac_min), C.byref(lr), _ptr(row))
    return lr.value, row


# ---------------------------------------------------------------- step
class Particles:
    """FP64 SoA copy of a population for the oracle (arrays are owned here)."""

    KEYS = ("ux", "uy", "uz", "ex", "ey", "ez", "bx", "by", "bz", "tau", "w")

    def __init__(self, pop: dict, species: int, id_base: int = 0, tau=None):
        n = len(pop["ux"])
        self.a = {}
        for k in self.KEYS:
            if k == "tau":
                v = np.zeros(n) if tau is None else np.array(tau, dtype=np.float64)
            else:
                v = np.array(pop[k], dtype=np.float64)
            self.a[k] = np.ascontiguousarray(v)
        self.n, self.species, self.id_base = n, species, id_base
        self._c = _Particles(*[_ptr(self.a[k]) for k in self.KEYS], n, id_base, species)

    def __getitem__(self, k):
        return self.a[k]

    @property
    def cstruct(self):
        return C.byref(self._c)


class Append:
    KEYS = ("ux", "uy", "uz", "w", "tau")

    def __init__(self, capacity: int):
        cap = max(int(capacity), 1)
        self.a = {k: np.zeros(cap) for k in self.KEYS}
        self.parent = np.full(cap, -1, dtype=np.int64)
        self._c = _Append(*[_ptr(self.a[k]) for k in self.KEYS], _ptr(self.parent, _i64p),
                          int(capacity), 0)

    @property
    def count(self):
        return self._c.count

    @count.setter
    def count(self, v):
        self._c.count = int(v)

    def __getitem__(self, k):
        if k == "parent":
            return self.parent[:min(self.count, self._c.capacity)]
        return self.a[k][:min(self.count, self._c.capacity)]

    @property
    def cstruct(self):
        return C.byref(self._c)


def init_optical_depth(p: Particles, seed: int):
    lib().orc_init_optical_depth(p.cstruct, seed)


def set_threads(n: int) -> None:
    """Threads of the oracle's OpenMP loops."""
    lib().orc_set_threads(int(n))


def max_threads() -> int:
    return int(lib().orc_max_threads())


def step(bw: Table, qs: Table, p: Particles, dt: float, seed: int, step_idx: int,
         a1: Append, a2: Append | None = None, photon_min_energy: float = 0.0, flags=None,
         chi_qed_min: float = 0.0):
    if a2 is None:
        a2 = Append(0)
    fl = None if flags is None else _ptr(flags, _u8p)
    return lib().orc_step(bw.cstruct, qs.cstruct, p.cstruct, dt, seed, step_idx,
                          photon_min_energy, chi_qed_min, fl, a1.cstruct, a2.cstruct)


def generate(bw: Table, qs: Table, p: Particles, flags: np.ndarray, seed: int, step_idx: int,
             a1: Append, a2: Append | None = None, photon_min_energy: float = 0.0):
    if a2 is None:
        a2 = Append(0)
    flags = np.ascontiguousarray(flags, dtype=np.uint8)
    return lib().orc_generate(bw.cstruct, qs.cstruct, p.cstruct, _ptr(flags, _u8p), seed, step_idx,
                              photon_min_energy, a1.cstruct, a2.cstruct)


def evolve(t: Table, p: Particles, dt: float, flags=None):
    fl = None if flags is None else _ptr(flags, _u8p)
    lib().orc_evolve(t.cstruct, p.cstruct, dt, fl)


# ---------------------------------------------------------------- MLP
MLP_NPARAM = 4417


def mlp_forward(params, x, bf16=False):
    p = np.ascontiguousarray(params, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 2)
    y = np.zeros(len(x))
    lib().orc_mlp_grad(_ptr(p), len(x), _ptr(x), None, None, None, _ptr(y), int(bf16))
    return y


def mlp_grad(params, x, t, w=None, bf16=False):
    """(loss, grad) of 0.5 sum w (y - t)^2 / n."""
    p = np.ascontiguousarray(params, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 2)
    t = np.ascontiguousarray(t, dtype=np.float64)
    g = np.zeros(MLP_NPARAM)
    wp = None if w is None else _ptr(np.ascontiguousarray(w, dtype=np.float64))
    loss = lib().orc_mlp_grad(_ptr(p), len(x), _ptr(x), _ptr(t), wp, _ptr(g), None, int(bf16))
    return loss, g


def compact(tiles, set_stream, flags, id_base, stream):
    """Parent ids of one product stream in (tile, index) order."""
    tiles = np.ascontiguousarray(tiles, dtype=np.int64).reshape(-1)
    ss = np.ascontiguousarray(set_stream, dtype=np.int32)
    fl = [np.ascontiguousarray(f, dtype=np.uint8) for f in flags]
    fp = (_u8p * len(fl))(*[_ptr(f, _u8p) for f in fl])
    ib = np.ascontiguousarray(id_base, dtype=np.int64)
    cap = int(sum(int(f.sum()) for f in fl)) + 1
    out = np.zeros(cap, dtype=np.int64)
    k = lib().orc_compact(len(tiles) // 3, _ptr(tiles, _i64p), ss.ctypes.data_as(C.POINTER(C.c_int32)), fp,
                          _ptr(ib, _i64p), stream, _ptr(out, _i64p), cap)
    return out[:k]


# ---------------------------------------------------------------- Schwinger
FIELD_KEYS = ("ex", "ey", "ez", "bx", "by", "bz")


def schwinger_rate(ex, ey, ez, bx, by, bz):
    """Pair production rate per unit volume (m^-3 s^-1) for one field point."""
    return lib().orc_schwinger_rate(float(ex), float(ey), float(ez), float(bx), float(by), float(bz))


def schwinger_rate_array(cells: dict) -> np.ndarray:
    cols = [np.ascontiguousarray(cells[k], dtype=np.float64) for k in FIELD_KEYS]
    out = np.zeros(len(cols[0]))
    lib().orc_schwinger_rate_n(len(out), *[_ptr(c) for c in cols], _ptr(out))
    return out


def schwinger_count(lam, seed, cell, step):
    """(number of macro-pairs, margin of the deciding comparison)."""
    m = C.c_double()
    k = lib().orc_schwinger_count(float(lam), seed, cell, step, C.byref(m))
    return k, m.value


def schwinger_pairs(cells: dict, cell_id_base, dv, dt, weight, seed, step, capacity):
    cols = [np.ascontiguousarray(cells[k], dtype=np.float64) for k in FIELD_KEYS]
    el, po = Append(capacity), Append(capacity)
    lib().orc_schwinger_pairs(len(cols[0]), *[_ptr(c) for c in cols], cell_id_base, dv, dt, weight, seed, step,
                              el.cstruct, po.cstruct)
    return el, po


# ---------------------------------------------------------------- push
def uniform_field(e0=(0.0, 0.0, 0.0), b0=(0.0, 0.0, 0.0)):
    return _Field(0, 1, (C.c_double * 3)(*e0), (C.c_double * 3)(*b0), 0.0, 0.0, 0.0)


def cp_wave(amplitude, wavelength, direction=1, phase=0.0):
    return _Field(1, direction, (C.c_double * 3)(), (C.c_double * 3)(), amplitude, wavelength, phase)


def push(p: Particles, x, y, z, field, t, dt):
    """Boris push of p (in place) and of the positions x, y, z (float64 arrays)."""
    for a in (x, y, z):
        assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    lib().orc_push(p.cstruct, _ptr(x), _ptr(y), _ptr(z), C.byref(field), float(t), float(dt))
