"""Statistical and physical pins of the oracle at 10^7 samples.

* Photon and pair spectra (Sec. 3.1, Sec. 3.2 sampling): the oracle's
  samples are checked three ways.  First, they invert the interpolated table
  CDF exactly.  Second, their exact one-sample Kolmogorov-Smirnov distance to
  that CDF stays within the critical value.  Third, their distance to the
  exact CDF stays within the critical value plus the table's own
  interpolation error.  The exact CDF is a 4097-knot quadrature row, and its
  accuracy is bounded by leaving out every other knot.
* Total rates (Sec. 2.1 BW rate, Sec. 2.2 QS rate, Sec. 3 optical depth):
  the fraction of particles without an event after k steps is
  exp(-rate k dt), with the rate taken from the integrated cross section.
* The continuations outside the tables (Sec. 3.1, 3.2 leave them open):
  the BW rate's asymptotic rules and the QS CDF below its first knot follow
  the exact integrals with the error the neglected terms predict.
* The classical radiation drag below the minimum quantum parameter (Sec. 6):
  its power equals Larmor's formula in SI (the synchrotron and linear
  cases); iterating it in a fixed magnetic field converges at first order
  to the closed-form cooling trajectory; and it is the chi -> 0 limit of the
  quantum-synchrotron power, which reproduces the known Gaunt-factor
  expansion 1 - (55 sqrt3/16) chi + 48 chi^2.
"""
import math

import numpy as np
import pytest

import qed_inputs as QI
from oracle import oracle as O

N = 10 ** 7
# Kolmogorov distribution: P(sqrt(n) D_n > 1.628) = 0.01
KS_CRIT = 1.628 / math.sqrt(N)
N_REF = 4097          # knots of the reference CDF row (odd: the half grid keeps both ends)
R0 = O.rate_prefactor()

# SI constants (CODATA 2018) for the textbook formulas, independent of the
# oracle's alpha-based prefactor
E_CHARGE = 1.602176634e-19
M_E = 9.1093837015e-31
C = 299792458.0
EPS0 = 8.8541878128e-12


def _ks_exact(F_sorted):
    """sup |ECDF - F| for the sorted samples' CDF values."""
    n = len(F_sorted)
    i = np.arange(1, n + 1, dtype=np.float64)
    return max(float(np.max(i / n - F_sorted)), float(np.max(F_sorted - (i - 1) / n)))


def _qs_lnk(n, frac_min=1e-12):
    return math.log(frac_min) * (1.0 - np.arange(n) / (n - 1))


def _qs_F(lnx, lnk, L):
    """QS CDF of a row of ln P at log-spaced knots, linear in ln xi, and the
    small-xi law P ~ xi^(1/3) below the first knot (Sec. 3.2 sampling)."""
    out = np.interp(lnx, lnk, L)
    lo = lnx < lnk[0]
    out[lo] = L[0] + (lnx[lo] - lnk[0]) / 3.0
    return np.exp(out)


def _bw_full_F(x, k, P):
    """CDF over [0, 1] of the electron's fraction for a half-row P on
    [0, 1/2] (the spectrum is symmetric about 1/2, Sec. 2.1)."""
    lo = np.interp(np.minimum(x, 0.5), k, P)
    hi = 1.0 - np.interp(np.minimum(1.0 - x, 0.5), k, P)
    return np.where(x <= 0.5, lo, hi)


@pytest.mark.parametrize("chi", [1e-3, 0.05, 1.0, 20.0, 1e3])
def test_qs_photon_spectrum_1e7(chi):
    tab = O.Table(O.QS, chi / 1.5, chi * 1.5, 3, 256)   # chi is the middle knot
    r = np.random.default_rng(11).random(N)
    lx = tab.sample_n(chi, r)
    lnk = _qs_lnk(256)
    # exact inversion of the interpolated table CDF
    Ft = _qs_F(lx, lnk, tab.cdf[1])
    assert np.max(np.abs(np.log(Ft) - np.log(r))) < 1e-9
    order = np.argsort(lx)
    d_table = _ks_exact(Ft[order])
    assert d_table <= KS_CRIT, d_table
    # reference: a 4097-knot quadrature row; its interpolation error is about
    # a quarter of what leaving out every other knot gives
    _, Lf = O.table_row(O.QS, chi, N_REF)
    lnkf = _qs_lnk(N_REF)
    ref_err = float(np.max(np.abs(_qs_F(lnkf[1::2], lnkf[0::2], Lf[0::2]) - np.exp(Lf[1::2]))))
    table_err = float(np.max(np.abs(_qs_F(lnkf, lnk, tab.cdf[1]) - np.exp(Lf))))
    d_exact = _ks_exact(_qs_F(lx[order], lnkf, Lf))
    assert d_exact <= KS_CRIT + table_err + ref_err, (d_exact, table_err, ref_err)
    # the 256-knot table resolves the spectrum to the paper's per-cent level
    # (Sec. 3.2: 128 points give a few per cent); at small chi far better
    assert table_err < (1e-3 if chi <= 1.0 else 1e-2), table_err


@pytest.mark.parametrize("chi", [0.05, 1.0, 20.0, 1e3])
def test_bw_pair_spectrum_1e7(chi):
    tab = O.Table(O.BW, chi / 1.5, chi * 1.5, 3, 256)
    r = np.random.default_rng(12).random(N)
    xi, esel = tab.sample_n(chi, r)
    # r <= 1/2 selects the electron, and r -> 1 - r the positron (Sec. 3.1)
    np.testing.assert_array_equal(esel, r <= 0.5)
    k = 0.5 * np.arange(256) / 255
    folded = np.where(esel, r, 1.0 - r)
    assert np.max(np.abs(np.interp(xi, k, tab.cdf[1]) - folded)) < 1e-12
    xe = np.where(esel, xi, 1.0 - xi)      # the electron's fraction
    order = np.argsort(xe)
    xs = xe[order]
    d_table = _ks_exact(_bw_full_F(xs, k, tab.cdf[1]))
    assert d_table <= KS_CRIT, d_table
    _, Pf = O.table_row(O.BW, chi, N_REF)
    kf = 0.5 * np.arange(N_REF) / (N_REF - 1)
    ref_err = float(np.max(np.abs(np.interp(kf[1::2], kf[0::2], Pf[0::2]) - Pf[1::2])))
    table_err = float(np.max(np.abs(np.interp(kf, k, tab.cdf[1]) - Pf)))
    d_exact = _ks_exact(_bw_full_F(xs, kf, Pf))
    assert d_exact <= KS_CRIT + table_err + ref_err, (d_exact, table_err, ref_err)
    assert table_err < (1e-4 if chi <= 20.0 else 2e-3), table_err


def _beam(n, gamma, e_field, photon):
    """n identical particles counter-propagating a plane-wave field."""
    u = gamma if photon else math.sqrt(gamma * gamma - 1)
    z = np.zeros(n)
    return dict(ux=np.full(n, -u), uy=z.copy(), uz=z.copy(), ex=z.copy(), ey=np.full(n, e_field),
                ez=z.copy(), bx=z.copy(), by=z.copy(), bz=np.full(n, e_field / QI.C_LIGHT),
                w=np.ones(n))


@pytest.mark.parametrize("photon", [False, True])
def test_survival_matches_integrated_rate_1e7(photon):
    """With tau ~ Exp(1), the fraction of particles that have had no event
    after k steps is exp(-rate k dt) (Sec. 3: the optical depth is the
    integral of the rate), with the rate from the integrated cross section
    (T(chi_gamma) for BW, G(chi) for QS) evaluated by quadrature."""
    gamma, e = 2000.0, 2e14
    pop1 = _beam(1, gamma, e, photon)
    args = [pop1[k][0] for k in ("ux", "uy", "uz", "ex", "ey", "ez", "bx", "by", "bz")]
    chi = O.chi_photon(*args) if photon else O.chi_lepton(*args)
    if photon:
        rate = R0 * chi / gamma * O.bw_T(chi)
    else:
        rate = 2.0 / 3.0 * R0 * O.qs_G(chi) / gamma
    proc = O.BW if photon else O.QS
    tab = O.Table(proc, chi / 1.5, chi * 1.5, 3, 64)    # chi is a knot: no interpolation error
    bw = tab if photon else O.Table(O.BW, 1e-3, 1e2, 4, 4)
    qs = O.Table(O.QS, 1e-3, 1e2, 4, 4) if photon else tab
    assert tab.rate(chi, gamma) == pytest.approx(rate, rel=1e-9)
    dt = 0.15 / rate
    pop = _beam(N, gamma, e, photon)
    p = O.Particles(pop, O.PHOTON if photon else O.ELECTRON, id_base=1 << 33)
    O.init_optical_depth(p, seed=21)
    alive = np.ones(N, dtype=bool)
    flags = np.zeros(N, dtype=np.uint8)
    a1, a2 = O.Append(N), O.Append(N if photon else 0)
    for k in range(1, 4):
        a1.count = 0
        a2.count = 0
        O.step(bw, qs, p, dt, seed=21, step_idx=k, a1=a1, a2=a2, flags=flags)
        alive &= flags == 0
        pk = math.exp(-rate * k * dt)
        sd = math.sqrt(N * pk * (1 - pk))
        assert abs(int(alive.sum()) - N * pk) < 5 * sd, (k, int(alive.sum()), N * pk, sd)
    del p, pop


# ------------------------------------------------------------ classical drag
_TINY = {}


def _classical_step(pop, dt):
    """One oracle step of electrons with every particle below the minimum
    quantum parameter (classical regime); returns the new gamma."""
    if not _TINY:   # the tables are never read in the classical regime
        _TINY["bw"], _TINY["qs"] = O.Table(O.BW, 1e-3, 1e2, 4, 4), O.Table(O.QS, 1e-3, 1e2, 4, 4)
    bw, qs = _TINY["bw"], _TINY["qs"]
    n = len(pop["ux"])
    p = O.Particles(pop, O.ELECTRON, tau=np.full(n, 0.7))
    flags = np.zeros(n, dtype=np.uint8)
    O.step(bw, qs, p, dt, 1, 0, O.Append(n), flags=flags, chi_qed_min=1e30)
    assert np.all(flags == 0) and np.all(p["tau"] == 0.7)
    u1 = np.stack([p["ux"], p["uy"], p["uz"]], 1)
    return u1, np.sqrt(1.0 + np.sum(u1 * u1, 1))


def test_classical_drag_power_is_larmor():
    """The drag's power equals Larmor's (Lienard's) radiated power in SI:
    synchrotron, v perpendicular to B: P = e^4 B^2 gamma^2 v^2 / (6 pi eps0 m^2 c^3);
    linear acceleration, E parallel to v: P = e^4 E^2 / (6 pi eps0 m^2 c^3)."""
    k4 = E_CHARGE ** 4 / (6.0 * math.pi * EPS0 * M_E ** 2 * C ** 3)
    mc2 = M_E * C * C
    cases = []
    for gamma, b in ((50.0, 1e3), (1e3, 2e4), (3e4, 5e4)):
        cases.append(("sync", gamma, b))
    for gamma, e in ((20.0, 1e13), (5e3, 3e14)):
        cases.append(("lin", gamma, e))
    for kind, gamma, f in cases:
        um = math.sqrt(gamma * gamma - 1.0)
        pop = {k: np.zeros(1) for k in QI.FIELDS}
        pop["w"][0] = 1.0
        if kind == "sync":        # u along y, B along z
            pop["uy"][0] = um
            pop["bz"][0] = f
            expect = k4 * f * f * (C * um) ** 2           # gamma^2 v^2 = c^2 |u|^2
        else:                     # u and E along x
            pop["ux"][0] = um
            pop["ex"][0] = f
            expect = k4 * f * f
        dt = 1e-4 * gamma * mc2 / expect                  # gamma changes by 1e-4 of itself
        u0 = np.stack([pop["ux"], pop["uy"], pop["uz"]], 1)
        u1, g1 = _classical_step(pop, dt)
        power = (gamma - float(g1[0])) * mc2 / dt
        assert power == pytest.approx(expect, rel=2e-8), (kind, gamma, f)
        # the drag acts along u: the direction is unchanged
        cos = float(np.sum(u0 * u1)) / (np.linalg.norm(u0) * np.linalg.norm(u1))
        assert cos == pytest.approx(1.0, abs=1e-15)


def test_classical_drag_cooling_trajectory():
    """In a fixed B perpendicular to u, the drag obeys dgamma/dt = -K (gamma^2 - 1)
    with K = e^4 B^2 / (6 pi eps0 m^3 c^3), whose solution is
    gamma(t) = coth(K t + arcoth gamma0); the oracle's step (explicit in
    gamma) converges to it at first order in dt."""
    b, gamma0 = 1e6, 1e3
    K = E_CHARGE ** 4 * b * b / (6.0 * math.pi * EPS0 * M_E ** 3 * C ** 3)
    t_end = 2.0 / (K * gamma0)
    exact = 1.0 / math.tanh(K * t_end + math.atanh(1.0 / gamma0))
    errs = []
    for nsteps in (250, 500, 1000):
        dt = t_end / nsteps
        pop = {k: np.zeros(1) for k in QI.FIELDS}
        pop["uy"][0] = math.sqrt(gamma0 ** 2 - 1)
        pop["bz"][0] = b
        pop["w"][0] = 1.0
        for _ in range(nsteps):
            u1, g1 = _classical_step(pop, dt)
            pop["ux"][0], pop["uy"][0], pop["uz"][0] = u1[0]
        errs.append(float(g1[0]) - exact)
    assert exact < 0.5 * gamma0              # the particle cools substantially
    # first order: halving dt halves the error
    for e1, e2 in zip(errs, errs[1:]):
        assert 1.9 < e1 / e2 < 2.1, errs
    assert abs(errs[-1]) < 1e-2 * exact, errs


def test_classical_drag_is_small_chi_limit_of_qs_power():
    """The quantum-synchrotron power, rate x mean photon energy =
    (2/3)(alpha m c^2/hbar) G(chi) <xi> m c^2 for gamma >> 1 (Sec. 2.2), over the
    drag's power is the Gaunt factor g(chi) = 1 - (55 sqrt3/16) chi + 48 chi^2 + O(chi^3),
    which tends to 1 as chi -> 0."""
    lnk = _qs_lnk(N_REF)
    xk = np.exp(lnk)
    xk[-1] = 1.0
    for chi in (1e-4, 1e-3):
        _, L = O.table_row(O.QS, chi, N_REF)
        # <xi> = int_0^1 (1 - P) dxi; below the first knot 1 - P = 1 to O(xi_min^(1/3))
        mean_xi = float(np.trapezoid((1.0 - np.exp(L)) * xk, lnk)) + xk[0]
        p_quantum = 2.0 / 3.0 * R0 * O.qs_G(chi) * mean_xi          # in m c^2 per second
        # the drag at this chi: u along y, B along z, gamma large
        gamma = 1e5
        um = math.sqrt(gamma * gamma - 1.0)
        b = chi * 1.3232855e18 / (C * um)                              # chi = c |u| B / E_s
        pop = {k: np.zeros(1) for k in QI.FIELDS}
        pop["uy"][0], pop["bz"][0], pop["w"][0] = um, b, 1.0
        chi_o = float(O.chi_array(pop, False)[0])
        dt = 1e-6 * gamma / (R0 * chi_o ** 2)
        _, g1 = _classical_step(pop, dt)
        p_drag = (gamma - float(g1[0])) / dt * (chi / chi_o) ** 2       # rescaled to chi exactly
        gaunt = 1.0 - 55.0 * math.sqrt(3.0) / 16.0 * chi + 48.0 * chi * chi
        assert p_quantum / p_drag == pytest.approx(gaunt, abs=600.0 * chi ** 3 + 2e-8), (chi, p_quantum / p_drag)


@pytest.mark.parametrize("chi", [1e-3, 1.0, 1e3])
def test_qs_extrapolation_below_first_knot_is_exact_cdf(chi):
    """Below the first CDF knot xi_min the sampler continues the table with
    P = P(xi_min) (xi/xi_min)^(1/3) (Sec. 3.2 leaves this region open).  The
    exact CDF by quadrature follows that law there: its relative deviation
    is O(xi^(2/3)), far below any sampling resolution."""
    xi_min = 1e-12
    _, row = O.table_row(O.QS, chi, 3, xi_min)
    for xi in (1e-13, 1e-15):
        # a row whose first knot is xi: ln P there by quadrature of the
        # spectrum from 0 to xi
        _, low = O.table_row(O.QS, chi, 3, xi)
        assert low[0] == pytest.approx(row[0] + math.log(xi / xi_min) / 3.0, abs=1e-5)


def test_bw_rate_out_of_table_rules_approach_exact_T():
    """The BW rate outside the tabulated chi range (Sec. 3.1 leaves it open;
    the runtime continues ln T with the asymptotes of the integral, matched
    at the table edge).  Against T by quadrature (Sec. 2.1):
    * above chi_max the rule keeps the large-chi law T ~ chi^(-1/3); the
      neglected term of T's expansion is O(chi^(-2/3)), so at a fixed
      multiple of chi_max the relative error falls by about 10^(2/3) per
      decade of chi_max (a wrong exponent would leave it constant);
    * below chi_min the rule keeps the small-chi law
      T ~ exp(-8/(3 chi)); the neglected prefactor term is O(chi), so at a
      fixed fraction of chi_min the error halves with chi_min (a wrong
      coefficient of 1/chi would grow it exponentially)."""
    r0 = O.rate_prefactor()

    def err(table, c):
        return table.rate(c, 1.0) / (r0 * c) / O.bw_T(c) - 1.0

    above = {cm: [err(O.Table(O.BW, 1e-2, cm, 8, 8), f * cm) for f in (2.0, 4.0)] for cm in (1e2, 1e3)}
    for i in range(2):
        assert above[1e3][i] < 0.0 and abs(above[1e3][i]) < 1.2e-2
        ratio = above[1e2][i] / above[1e3][i]
        assert 10 ** (2 / 3) * 0.9 < ratio < 10 ** (2 / 3) * 1.2
    below = {cm: [err(O.Table(O.BW, cm, 1.0, 8, 8), f * cm) for f in (0.75, 0.5)] for cm in (0.04, 0.02)}
    for i in range(2):
        assert below[0.02][i] < 0.0 and abs(below[0.02][i]) < 2e-3
        ratio = below[0.04][i] / below[0.02][i]
        assert 1.9 < ratio < 2.1
