"""Pins of the CPU oracle against what the paper and mathematics fix.

Each test checks the oracle against something other than itself: numpy's
Philox, scipy/mpmath Bessel functions, closed-form asymptotes and limits,
the quantum parameters the paper prints for its literature benchmarks,
binary128 evaluation of the printed chi formula, Lorentz invariance,
conservation laws, and Monte Carlo statistics.
"""
import json
import math
import os

import mpmath as mp
import numpy as np
import pytest
from scipy import integrate, special, stats

from oracle import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


# ----------------------------------------------------------------- Philox
@pytest.mark.parametrize("ctr,key", [
    ([0, 0, 0, 0], [0, 0]),
    ([5, 6, 7, 8], [1, 0]),
    ([123456789, 2**64 - 1, 2, 0], [2**63 + 17, 0]),
    ([2**64 - 1, 3, 1, 0], [1, 0]),            # id wraps the first word
    ([42, (1 << 64) - 1, 2, 0], [1, 0]),        # INIT step
])
def test_philox_matches_numpy(ctr, key):
    # numpy increments the counter before producing a block
    v = sum(int(c) << (64 * k) for k, c in enumerate(ctr))
    v = (v - 1) % (1 << 256)
    prev = [(v >> (64 * k)) & (2**64 - 1) for k in range(4)]
    g = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.array(prev, dtype=np.uint64))
    assert O.philox_block(ctr, key) == [int(x) for x in g.random_raw(4)]


def test_u01_exact_open_interval():
    assert O.u01(0) == 2.0 ** -53
    assert O.u01(2**64 - 1) == 1.0 - 2.0 ** -53
    rng = np.random.default_rng(0)
    for w in rng.integers(0, 2**63, 1000, dtype=np.uint64):
        u = O.u01(int(w) * 2 + 1)
        m = (int(w) * 2 + 1) >> 12
        assert u == (2 * m + 1) / 2.0**53
        assert 0.0 < u < 1.0
        # 1 - u is exact: (1 - u) + u reproduces 1 and 1 - (1 - u) reproduces u
        assert 1.0 - (1.0 - u) == u


# ----------------------------------------------------------------- Bessel
@pytest.mark.parametrize("nu", [1 / 3, 2 / 3, 5 / 3])
def test_bessel_k_vs_scipy(nu):
    for x in np.geomspace(1e-8, 700, 40):
        ref = special.kve(nu, x)
        ek, _ = O.bessel_pair_scaled(x, nu, nu)
        assert abs(ek / ref - 1) < 2e-14, (nu, x)


@pytest.mark.parametrize("nu", [1 / 3, 5 / 3])
def test_bessel_tail_integral_vs_scipy(nu):
    for x in (1e-6, 1e-3, 0.05, 0.7, 3.0, 25.0, 300.0, 3000.0):
        # e^x int_x^inf K_nu: below s = 1 in log variable (K_nu ~ s^-nu), above it directly
        ref = integrate.quad(lambda s: special.kve(nu, s) * np.exp(-(s - x)), max(x, 1.0), np.inf,
                             epsabs=0, epsrel=1e-13, limit=500)[0]
        if x < 1.0:
            ref += integrate.quad(lambda y: special.kv(nu, np.exp(y)) * np.exp(y) * np.exp(x),
                                  np.log(x), 0.0, epsabs=0, epsrel=1e-13, limit=500)[0]
        _, eik = O.bessel_pair_scaled(x, nu, nu)
        assert abs(eik / ref - 1) < 5e-14, (nu, x)


def test_inner_integral_substitution_matches_printed_form():
    """int_X^inf sqrt(s) K_{1/3}((2/3) s^{3/2}) ds as printed (Sec. 2.1) equals
    IK_{1/3}(z) with z = (2/3) X^{3/2}, the form the oracle integrates."""
    mp.mp.dps = 25
    for X in (0.2, 1.0, 3.0):
        lit = mp.quad(lambda s: mp.sqrt(s) * mp.besselk(mp.mpf(1) / 3, mp.mpf(2) / 3 * s**1.5),
                      [X, X + 1, X + 4, mp.inf])
        z = 2.0 / 3.0 * X**1.5
        assert abs(O.bessel_ik(1 / 3, z) / float(lit) - 1) < 1e-13


# ----------------------------------------------------------------- T(chi), G(chi)
def _T_scipy(chi):
    """Independent evaluation of the printed T(chi_gamma) (Sec. 2.1): outer
    integral over u in [0, chi] with scipy, inner tail integral from scipy's
    K_{1/3} and the printed X(chi, u) = (chi/(u (chi - u)))^{2/3}."""
    def bracket(u):
        X = (chi / (u * (chi - u))) ** (2.0 / 3.0)
        z = 2.0 / 3.0 * X**1.5
        ik = integrate.quad(lambda s: special.kv(1 / 3, s), z, np.inf, epsabs=0, epsrel=1e-12, limit=200)[0]
        return ik - (2.0 - chi * X**1.5) * special.kv(2 / 3, z)
    val = integrate.quad(bracket, 0, chi / 2, epsabs=0, epsrel=1e-11, limit=400)[0] * 2
    return val / (math.pi * math.sqrt(3) * chi**2)


def _ik53_scipy(y):
    """int_y^inf K_{5/3} through the recurrence K_{5/3} = -2 K'_{2/3} - K_{1/3}:
    2 K_{2/3}(y) - int_y^inf K_{1/3}(s) ds (scipy Bessel functions)."""
    tail = integrate.quad(lambda s: special.kv(1 / 3, s), max(y, 1.0), np.inf, epsabs=0, epsrel=1e-13)[0]
    if y < 1.0:
        tail += integrate.quad(lambda t: special.kv(1 / 3, np.exp(t)) * np.exp(t), np.log(y), 0.0,
                               epsabs=0, epsrel=1e-13, limit=200)[0]
    return 2 * special.kv(2 / 3, y) - tail


def _qs_bracket_scipy(chi, xi):
    Y = 2.0 / 3.0 * xi / (chi * (1 - xi))
    return _ik53_scipy(Y) + xi * xi / (1 - xi) * special.kv(2 / 3, Y)


def _qs_integral_scipy(chi, a, b):
    """int_a^b of the QS bracket, in s = xi^{1/3} (removes the xi^{-2/3} end point)."""
    sa, sb = a ** (1 / 3), b ** (1 / 3)
    pts = [p ** (1 / 3) for p in (chi * 1e-3, chi * 1e-2, chi * 0.1, chi, 0.5, 0.9) if a < p < b]
    f = lambda s: _qs_bracket_scipy(chi, s**3) * 3 * s * s if s**3 < 1 else 0.0
    return integrate.quad(f, sa, sb, points=pts or None, epsabs=0, epsrel=1e-12, limit=800)[0]


def _G_scipy(chi):
    """Independent evaluation of the printed G(chi) (Sec. 2.2)."""
    return math.sqrt(3) / (2 * math.pi) * _qs_integral_scipy(chi, 0.0, 1.0)


@pytest.mark.parametrize("chi", [0.5, 1.0, 10.0, 100.0])
def test_T_vs_independent_quadrature(chi):
    assert abs(O.bw_T(chi) / _T_scipy(chi) - 1) < 1e-9


@pytest.mark.parametrize("chi", [0.01, 1.0, 30.0])
def test_G_vs_independent_quadrature(chi):
    assert abs(O.qs_G(chi) / _G_scipy(chi) - 1) < 1e-9


def _C_T():
    """Large-chi constant of T ~ C_T chi^{-1/3} from Beta/Gamma functions:
    C_T = (1/(pi sqrt3)) 2^{-1/3} Gamma(2/3) (3/2)^{2/3} [B(2/3,2/3) - 2 B(5/3,5/3)]."""
    B = special.beta
    return (1 / (math.pi * math.sqrt(3))) * 2 ** (-1 / 3) * special.gamma(2 / 3) * 1.5 ** (2 / 3) * \
        (B(2 / 3, 2 / 3) - 2 * B(5 / 3, 5 / 3))


def _C_G():
    """Large-chi constant of G ~ C_G chi^{2/3}."""
    B = special.beta
    return (math.sqrt(3) / (2 * math.pi)) * 1.5 ** (2 / 3) * \
        (1.5 * 2 ** (2 / 3) * special.gamma(5 / 3) * B(1 / 3, 5 / 3) +
         2 ** (-1 / 3) * special.gamma(2 / 3) * B(7 / 3, 2 / 3))


def test_T_asymptotes():
    # small chi: T -> (3/16) sqrt(3/2) exp(-8/(3 chi)) (saddle point at xi = 1/2)
    small = lambda c: 3 / 16 * math.sqrt(1.5) * math.exp(-8 / (3 * c))
    r = [O.bw_T(c) / small(c) for c in (0.1, 0.02, 0.005)]
    assert r[0] < r[1] < r[2] < 1.0
    assert abs(r[2] - 1) < 2e-3
    # T(chi) underflows double precision for chi < ~3.8e-3: compare ln T
    lr, _ = O.table_row(O.BW, 1e-3, 3)
    assert abs(lr - (math.log(3 / 16 * math.sqrt(1.5)) - 8 / (3 * 1e-3))) < 1e-3
    # large chi: T -> C_T chi^{-1/3}
    assert abs(_C_T() - 0.3796123) < 1e-6
    r = [O.bw_T(c) / (_C_T() * c ** (-1 / 3)) for c in (1e3, 1e4, 1e5)]
    assert r[0] < r[1] < r[2] < 1.0
    assert abs(r[2] - 1) < 1.5e-3


def test_G_classical_limit_and_large_chi():
    # chi -> 0: G/chi -> 5 sqrt3 / 4, the classical synchrotron photon number
    # rate, with first correction factor (1 - (8 sqrt3/15) chi)
    lim = 5 * math.sqrt(3) / 4
    for c in (1e-4, 1e-3):
        g = O.qs_G(c) / c
        assert abs(g / (lim * (1 - 8 * math.sqrt(3) / 15 * c)) - 1) < 1e-5
    r = [O.qs_G(c) / (_C_G() * c ** (2 / 3)) for c in (1e3, 1e4, 1e5)]
    assert r[0] < r[1] < r[2] < 1.0
    assert abs(r[2] - 1) < 5e-4


# ----------------------------------------------------------------- CDFs
def test_bw_cdf_endpoints_and_small_chi_gaussian():
    lr, row = O.table_row(O.BW, 1.0, 33)
    assert row[0] == 0.0 and row[-1] == 0.5
    assert np.all(np.diff(row) > 0)
    # denominator of the CDF is the 1D table: ln T agrees with the point value
    assert abs(math.exp(lr) / O.bw_T(1.0) - 1) < 1e-13
    # small chi: the pair spectrum is a Gaussian about xi = 1/2 of width sqrt(3 chi)/8
    chi = 1e-3
    sigma = math.sqrt(3 * chi) / 8
    for k in (1.0, 2.0):
        p = O.bw_cdf_at(chi, 0.5 - k * sigma)
        assert abs(p / stats.norm.cdf(-k) - 1) < 0.03


def test_bw_cdf_vs_independent_quadrature():
    chi = 2.0

    def B(xi):
        z = 2 / (3 * chi * xi * (1 - xi))
        ik = integrate.quad(lambda s: special.kv(1 / 3, s), z, np.inf, epsabs=0, epsrel=1e-12, limit=200)[0]
        return ik + (1 / (xi * (1 - xi)) - 2) * special.kv(2 / 3, z)
    tot = 2 * integrate.quad(B, 0, 0.5, epsabs=0, epsrel=1e-12, limit=400)[0]
    for xi in (0.05, 0.2, 0.4):
        part = integrate.quad(B, 0, xi, epsabs=0, epsrel=1e-12, limit=400)[0]
        assert abs(O.bw_cdf_at(chi, xi) / (part / tot) - 1) < 1e-9


def test_qs_cdf_small_xi_law_and_classical_limit():
    chi = 0.3
    lr, row = O.table_row(O.QS, chi, 65, 1e-12)
    assert row[-1] == 0.0 and np.all(np.diff(row) > 0)
    # small xi: P ~ xi^{1/3}, coefficient from IK_{5/3}(Y) ~ (3/2) 2^{2/3} Gamma(5/3) Y^{-2/3}
    c = 1.5 * 2 ** (2 / 3) * special.gamma(5 / 3) * (1.5 * chi) ** (2 / 3)
    norm = O.qs_G(chi) * 2 * math.pi / math.sqrt(3)
    for xi in (1e-12, 1e-11):
        assert abs(O.qs_cdf_at(chi, xi) / (3 * c * xi ** (1 / 3) / norm) - 1) < 1e-3
    # chi -> 0: spectrum in y = 2 xi/(3 chi) tends to IK_{5/3}(y) normalised by 5 pi / 3
    chi = 1e-4
    for y in (0.1, 1.0, 3.0):
        cl = integrate.quad(lambda s: _ik53_scipy(s**3) * 3 * s * s, 0, y ** (1 / 3),
                            epsabs=0, epsrel=1e-11, limit=200)[0] * 3 / (5 * math.pi)
        assert abs(O.qs_cdf_at(chi, 1.5 * chi * y) / cl - 1) < 5e-4


def test_qs_cdf_vs_independent_quadrature():
    chi = 5.0
    tot = _qs_integral_scipy(chi, 0.0, 1.0)
    for xi in (1e-3, 0.1, 0.6):
        part = _qs_integral_scipy(chi, 0.0, xi)
        assert abs(O.qs_cdf_at(chi, xi) / (part / tot) - 1) < 1e-9


# ----------------------------------------------------------------- chi
ES = O.schwinger_field()
C_LIGHT = 299792458.0


def test_schwinger_field_printed_value():
    g = _gold("schwinger_field.json")
    assert abs(ES / g["E_s_V_per_m"] - 1) < g["rel_tol"]


def test_chi_printed_literature_cases():
    g = _gold("ridgers_cases.json")
    for case in g["cases"]:
        gam = case["gamma0"]
        u = math.sqrt(gam * gam - 1)
        if case["geometry"] == "perpendicular_B":
            chi = O.chi_lepton(u, 0, 0, 0, 0, 0, 0, 0, case["B_over_Es_c"] * ES / C_LIGHT)
        else:
            e0 = case["E0_over_Es"] * ES
            # circular polarisation: rotating (E_y, E_z), wave along +x, particle along -x
            chi = O.chi_lepton(-u, 0, 0, 0, e0 / math.sqrt(2), e0 / math.sqrt(2),
                               0, -e0 / math.sqrt(2) / C_LIGHT, e0 / math.sqrt(2) / C_LIGHT)
        assert abs(chi / case["chi"] - 1) < g["rel_tol"], case["name"]


def test_chi_closed_forms():
    e = 3.7e14
    # at rest: chi = |E|/E_s
    assert O.chi_lepton(0, 0, 0, e, 2 * e, 0, 1, 2, 3) == pytest.approx(math.sqrt(5) * e / ES, rel=1e-15)
    for gam in (1.5, 10.0, 1e3, 1e5):
        u = math.sqrt(gam * gam - 1)
        # counter-propagating a plane wave E_y = c B_z travelling along +x
        c1 = O.chi_lepton(-u, 0, 0, 0, e, 0, 0, 0, e / C_LIGHT)
        assert c1 == pytest.approx((gam + u) * e / ES, rel=1e-14)
        cp = O.chi_photon(-gam, 0, 0, 0, e, 0, 0, 0, e / C_LIGHT)
        assert cp == pytest.approx(2 * gam * e / ES, rel=1e-14)
    # co-propagating (no cancellation at moderate gamma): chi = |E|/((gamma + |u|) E_s)
    gam = 3.0
    u = math.sqrt(gam * gam - 1)
    b = e / C_LIGHT
    exact = e / ((gam + u) * ES)
    assert O.chi_lepton(u, 0, 0, 0, e, 0, 0, 0, b) == pytest.approx(exact, rel=1e-13)
    # photons co-propagating with a plane wave: chi = 0 up to the rounding of B = E/c
    assert O.chi_photon(10.0, 0, 0, 0, e, 0, 0, 0, b) < 1e-15 * 20 * e / ES


def _boost_x(beta, u, E, B, photon):
    """Lorentz boost along x (velocity beta c) of a particle momentum u and
    fields E, B (SI), evaluated in binary floating point with mpmath."""
    mp.mp.dps = 40
    beta = mp.mpf(beta)
    g = 1 / mp.sqrt(1 - beta * beta)
    ux, uy, uz = [mp.mpf(x) for x in u]
    e0 = mp.sqrt(ux * ux + uy * uy + uz * uz) if photon else mp.sqrt(1 + ux * ux + uy * uy + uz * uz)
    ex, ey, ez = [mp.mpf(x) for x in E]
    bx, by, bz = [mp.mpf(x) for x in B]
    c = mp.mpf(C_LIGHT)
    u2 = (g * (ux - beta * e0), uy, uz)
    E2 = (ex, g * (ey - beta * c * bz), g * (ez + beta * c * by))
    B2 = (bx, g * (by + beta * ez / c), g * (bz - beta * ey / c))
    return [float(x) for x in u2], [float(x) for x in E2], [float(x) for x in B2]


def test_chi_lorentz_invariance_and_printed_formula():
    rng = np.random.default_rng(7)
    for _ in range(40):
        photon = bool(rng.integers(2))
        u = rng.normal(size=3) * 10 ** rng.uniform(0, 3)
        E = rng.normal(size=3) * 1e15
        B = rng.normal(size=3) * 1e15 / C_LIGHT
        f = O.chi_photon if photon else O.chi_lepton
        c0 = f(*u, *E, *B)
        lit = O.chi_literal_q(*u, *E, *B, photon=photon)
        assert c0 == pytest.approx(lit, rel=1e-13)
        u2, E2, B2 = _boost_x(rng.uniform(-0.9, 0.9), u, E, B, photon)
        assert f(*u2, *E2, *B2) == pytest.approx(c0, rel=1e-12)


# ----------------------------------------------------------------- table accuracy claims
def test_paper_table_accuracy_claims():
    for claim in _gold("table_accuracy_claims.json")["claims"]:
        proc = O.BW if claim["process"] == "BW" else O.QS
        n = claim["table_points"]
        t = O.Table(proc, claim["chi_min"], claim["chi_max"], n, 3)
        # midpoints between knots are where linear interpolation in ln is worst
        lg = np.log(t.chi_grid())
        mids = np.exp(0.5 * (lg[1:] + lg[:-1]))
        mids = mids[mids > claim["check_above_chi"]][::max(1, len(mids) // 12)]
        exact = np.array([O.bw_T(c) if proc == O.BW else O.qs_G(c) for c in mids])
        interp = t.rate_n(mids, 1.0) / (O.rate_prefactor() * (mids if proc == O.BW else 2.0 / 3.0))
        err = np.max(np.abs(interp / exact - 1))
        assert err < claim["max_rel_error"], (claim["text"], err)
