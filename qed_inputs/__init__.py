"""Seeded synthetic particle populations for the QED Monte Carlo step.

This module only draws inputs (momenta, fields, weights, tile layouts).  It
holds none of the method's arithmetic: no quantum parameter, no rate, no
table, no sampling.  Both the HIP path and the CPU oracle consume exactly the
arrays produced here, so the two sides see bit-identical inputs.

All draws come from numpy's Philox4x64-10 bit generator keyed on
``(seed, 1)``; the runtime Monte Carlo draws of the method use key word
``0`` and are generated separately by each side.

Units: momentum ``u = p / (m_e c)`` (dimensionless); E in V/m; B in T.
Photons carry ``u`` with ``gamma_gamma = |u|``.
"""
from __future__ import annotations

import numpy as np

# CODATA 2018 exact / recommended values (SI).
M_E = 9.1093837015e-31      # kg
C_LIGHT = 299792458.0       # m/s
Q_E = 1.602176634e-19       # C
HBAR = 1.054571817e-34      # J s
E_SCHWINGER = M_E * M_E * C_LIGHT ** 3 / (Q_E * HBAR)   # ~1.3233e18 V/m
MEC2_MEV = 0.51099895000    # electron rest energy in MeV

SPECIES_ELECTRON = 0
SPECIES_POSITRON = 1
SPECIES_PHOTON = 2
SPECIES_ION = 3

FIELDS = ("ux", "uy", "uz", "ex", "ey", "ez", "bx", "by", "bz", "w")


def _rng(seed: int) -> np.random.Generator:
    key = np.array([seed & 0xFFFFFFFFFFFFFFFF, 1], dtype=np.uint64)
    return np.random.Generator(np.random.Philox(key=key))


def laser_e0(a0: float | np.ndarray, wavelength: float = 0.8e-6):
    """Peak field of a laser with normalised amplitude a0: a0 m_e c omega / q_e."""
    omega = 2.0 * np.pi * C_LIGHT / wavelength
    return a0 * M_E * C_LIGHT * omega / Q_E


def _loguniform(rng, lo, hi, n):
    return np.exp(rng.uniform(np.log(lo), np.log(hi), n))


def _cap_directions(rng, n, half_angle, axis_sign):
    """Unit vectors uniform over the spherical cap theta <= half_angle about
    axis_sign * x (uniform in cos(theta) and in azimuth)."""
    cth = rng.uniform(np.cos(half_angle), 1.0, n)
    sth = np.sqrt(np.maximum(0.0, 1.0 - cth * cth))
    az = rng.uniform(0.0, 2.0 * np.pi, n)
    return axis_sign * cth, sth * np.cos(az), sth * np.sin(az)


def _pack(ux, uy, uz, ex, ey, ez, bx, by, bz, w, dtype):
    d = dict(ux=ux, uy=uy, uz=uz, ex=ex, ey=ey, ez=ez, bx=bx, by=by, bz=bz, w=w)
    return {k: np.ascontiguousarray(v, dtype=dtype) for k, v in d.items()}


def _momenta(gamma, nx, ny, nz, photon):
    mag = gamma if photon else np.sqrt(np.maximum(gamma * gamma - 1.0, 0.0))
    return mag * nx, mag * ny, mag * nz


def plane_wave_counter(n: int, seed: int, photon: bool, stream: int = 0,
                       a0: float = 100.0, wavelength: float = 0.8e-6,
                       gamma_range=(1e2, 1e4), dtype=np.float64):
    """Small parity workload: momenta along -x, gamma log-uniform, uniform
    plane-wave field E_y = c B_z = a0 E0 cos(phi), phi ~ U[0, 2 pi)."""
    rng = _rng(seed * 4096 + stream)
    phi = rng.uniform(0.0, 2.0 * np.pi, n)
    gamma = _loguniform(rng, gamma_range[0], gamma_range[1], n)
    w = rng.uniform(0.5, 1.5, n)
    ey = laser_e0(a0, wavelength) * np.cos(phi)
    bz = ey / C_LIGHT
    z = np.zeros(n)
    ux, uy, uz = _momenta(gamma, -np.ones(n), z, z, photon)
    return _pack(ux, uy, uz, z, ey, z, z, z, bz, w, dtype)


def plane_wave_cone(n: int, seed: int, photon: bool, stream: int = 0,
                    a0_range=(10.0, 1000.0), gamma_range=(1e2, 1e5),
                    half_angle: float = 0.1, axis_sign: float = -1.0,
                    wavelength: float = 0.8e-6, dtype=np.float64):
    """Roofline workload: directions uniform in a cap of half-angle 0.1 rad
    about -x (or +x for the co-propagating subset), gamma log-uniform,
    linearly polarised plane wave with a0 log-uniform per particle."""
    rng = _rng(seed * 4096 + stream)
    nx, ny, nz = _cap_directions(rng, n, half_angle, axis_sign)
    gamma = _loguniform(rng, gamma_range[0], gamma_range[1], n)
    a0 = _loguniform(rng, a0_range[0], a0_range[1], n)
    phi = rng.uniform(0.0, 2.0 * np.pi, n)
    w = rng.uniform(0.5, 1.5, n)
    ey = laser_e0(a0, wavelength) * np.cos(phi)
    bz = ey / C_LIGHT
    z = np.zeros(n)
    ux, uy, uz = _momenta(gamma, nx, ny, nz, photon)
    return _pack(ux, uy, uz, z, ey, z, z, z, bz, w, dtype)


def paper_uniform(n: int, seed: int, stream: int = 0, dtype=np.float64):
    """The paper's benchmark population (Sec. 4): each E component uniform in
    [-E_s/100, E_s/100], each B component in [-E_s/(100c), E_s/(100c)], each
    momentum component uniform in [-1, 1] GeV/c."""
    rng = _rng(seed * 4096 + stream)
    umax = 1000.0 / MEC2_MEV          # 1 GeV/c in units of m_e c
    emax = E_SCHWINGER / 100.0
    bmax = emax / C_LIGHT
    ux, uy, uz = (rng.uniform(-umax, umax, n) for _ in range(3))
    ex, ey, ez = (rng.uniform(-emax, emax, n) for _ in range(3))
    bx, by, bz = (rng.uniform(-bmax, bmax, n) for _ in range(3))
    w = rng.uniform(0.5, 1.5, n)
    return _pack(ux, uy, uz, ex, ey, ez, bx, by, bz, w, dtype)


def wide_chi(n: int, seed: int, photon: bool, stream: int = 0,
             a0_range=(3.0, 3000.0), gamma_range=(1e2, 1e5), dtype=np.float64):
    """Event-kernel workload spanning roughly three decades either side of
    chi ~ 1: counter-propagating, phase fixed at the field crest."""
    rng = _rng(seed * 4096 + stream)
    gamma = _loguniform(rng, gamma_range[0], gamma_range[1], n)
    a0 = _loguniform(rng, a0_range[0], a0_range[1], n)
    w = rng.uniform(0.5, 1.5, n)
    ey = laser_e0(a0)
    bz = ey / C_LIGHT
    z = np.zeros(n)
    ux, uy, uz = _momenta(gamma, -np.ones(n), z, z, photon)
    return _pack(ux, uy, uz, z, ey, z, z, z, bz, w, dtype)


def lognormal_tiles(total: int, n_tiles: int, seed: int, sigma: float = 1.0,
                    stream: int = 0) -> np.ndarray:
    """Tile sizes proportional to lognormal(sigma) draws, normalised to
    ``total`` with largest-remainder rounding (sizes sum exactly to total)."""
    rng = _rng(seed * 4096 + 2048 + stream)
    raw = rng.lognormal(0.0, sigma, n_tiles)
    share = raw / raw.sum() * total
    base = np.floor(share).astype(np.int64)
    short = total - int(base.sum())
    order = np.argsort(-(share - base), kind="stable")
    base[order[:short]] += 1
    return base


def gaussian_pulse(n: int, seed: int, photon: bool, stream: int = 0,
                   a0: float = 500.0, waist: float = 2e-6, wavelength: float = 0.8e-6,
                   fwhm_s: float = 30e-15, dtype=np.float32):
    """Full-step workload fields: linearly polarised (E_y, B_z = E_y / c)
    paraxial Gaussian beam at focus, Gaussian temporal envelope of 30 fs
    intensity FWHM, sampled at uniform random positions x in [-10 lambda,
    10 lambda], y, z in [-2 w0, 2 w0].  Momenta as in plane_wave_cone."""
    rng = _rng(seed * 4096 + stream)
    nx, ny, nz = _cap_directions(rng, n, 0.1, -1.0)
    gamma = _loguniform(rng, 1e2, 1e5, n)
    w = rng.uniform(0.5, 1.5, n)
    x = rng.uniform(-10 * wavelength, 10 * wavelength, n)
    y = rng.uniform(-2 * waist, 2 * waist, n)
    zz = rng.uniform(-2 * waist, 2 * waist, n)
    k = 2.0 * np.pi / wavelength
    env_len = C_LIGHT * fwhm_s          # intensity FWHM in length
    env = np.exp(-2.0 * np.log(2.0) * (x / env_len) ** 2)
    trans = np.exp(-(y * y + zz * zz) / (waist * waist))
    ey = laser_e0(a0, wavelength) * env * trans * np.cos(k * x)
    bz = ey / C_LIGHT
    z = np.zeros(n)
    ux, uy, uz = _momenta(gamma, nx, ny, nz, photon)
    return _pack(ux, uy, uz, z, ey, z, z, z, bz, w, dtype)


def parity_population(seed: int = 1, n: int = 1 << 16, dtype=np.float64):
    """Parity workload: n electrons + n photons, a0 = 100 plane wave."""
    return (plane_wave_counter(n, seed, photon=False, stream=0, dtype=dtype),
            plane_wave_counter(n, seed, photon=True, stream=1, dtype=dtype))


def cone_population(seed: int = 1, n: int = 1 << 24, dtype=np.float64):
    """Roofline workload: n leptons + n photons in a 0.1 rad cone."""
    return (plane_wave_cone(n, seed, photon=False, stream=0, dtype=dtype),
            plane_wave_cone(n, seed, photon=True, stream=1, dtype=dtype))


def subsample(pop: dict, idx: np.ndarray) -> dict:
    return {k: np.ascontiguousarray(v[idx]) for k, v in pop.items()}


def fullstep_layout(n_per_species: int, tiles_per_species: int, seed: int = 1, sigma: float = 1.0,
                    n_species: int = 4) -> np.ndarray:
    """Tile list (set, begin, end) for n_species sets of n_per_species
    particles each, every set cut into tiles_per_species lognormal tiles; the
    list interleaves the sets tile by tile, as the species of one spatial
    tile of a PIC grid would be visited."""
    sizes = [lognormal_tiles(n_per_species, tiles_per_species, seed, sigma, stream=s) for s in range(n_species)]
    offs = [np.concatenate([[0], np.cumsum(z)]) for z in sizes]
    rows = []
    for k in range(tiles_per_species):
        for s in range(n_species):
            rows.append((s, int(offs[s][k]), int(offs[s][k + 1])))
    return np.array(rows, dtype=np.int64)


def fullstep_population(n_per_species: int, seed: int = 1):
    """Electrons, positrons, photons (Gaussian pulse fields, FP32) and ions
    (random FP32 values, passed through untouched)."""
    el = gaussian_pulse(n_per_species, seed, photon=False, stream=0)
    po = gaussian_pulse(n_per_species, seed, photon=False, stream=1)
    ph = gaussian_pulse(n_per_species, seed, photon=True, stream=2)
    rng = _rng(seed * 4096 + 3)
    ion = {k: rng.standard_normal(n_per_species).astype(np.float32) for k in FIELDS}
    return el, po, ph, ion


def uniforms(n: int, seed: int, stream: int = 0) -> np.ndarray:
    """n uniforms in the open interval (0, 1) (inverse-CDF sampling inputs)."""
    rng = _rng(seed * 4096 + 3072 + stream)
    u = rng.random(n)
    return np.where(u > 0.0, u, 2.0 ** -54)


def loguniform_chi(n: int, seed: int, lo: float, hi: float, stream: int = 0) -> np.ndarray:
    """n quantum parameters log-uniform in [lo, hi]."""
    return _loguniform(_rng(seed * 4096 + 3584 + stream), lo, hi, n)
