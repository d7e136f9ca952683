"""Pins of the oracle's Schwinger pair production (Sec. 2.3) against what the
physics fixes independently of the printed invariant formulas:

* a pure electric field reduces to Schwinger's leading term
  (q_e E)^2 / (4 pi^3 hbar^2 c) exp(-pi E_s / E);
* parallel E and B: the invariants are E and cB themselves;
* pure magnetic and crossed (plane-wave) fields give no pairs;
* the rate per unit volume and time is Lorentz invariant;
* the per-cell count is Poisson (mean, variance, pmf), Gaussian above 25;
* pairs are at rest, in cell order, with the macro-weight given."""
import math

import numpy as np
import pytest

import qed_inputs as QI
from oracle import oracle as O

C = QI.C_LIGHT
ES = QI.E_SCHWINGER


def _textbook_pure_e(e):
    return (QI.Q_E * e) ** 2 / (4 * math.pi ** 3 * QI.HBAR ** 2 * C) * math.exp(-math.pi * ES / e)


@pytest.mark.parametrize("frac", [0.02, 0.1, 0.5, 1.0, 3.0])
def test_pure_electric_field_is_schwinger_leading_term(frac):
    e = frac * ES
    for comp in range(3):
        f = [0.0] * 6
        f[comp] = e
        assert O.schwinger_rate(*f) == pytest.approx(_textbook_pure_e(e), rel=1e-13)


@pytest.mark.parametrize("ef,bf", [(0.1, 0.05), (0.3, 0.3), (0.05, 2.0), (1.0, 1e-3)])
def test_parallel_fields(ef, bf):
    e, cb = ef * ES, bf * ES
    pref = QI.Q_E ** 2 * ES ** 2 / (4 * math.pi ** 2 * QI.HBAR ** 2 * C)
    x = math.pi * cb / e
    expect = pref * ef * bf / math.tanh(x) * math.exp(-math.pi / ef)
    n = np.array([1.0, -2.0, 0.5]) / np.linalg.norm([1.0, -2.0, 0.5])
    got = O.schwinger_rate(*(e * n), *(cb / C * n))
    assert got == pytest.approx(expect, rel=1e-12)
    # antiparallel: same invariants up to the sign of G
    assert O.schwinger_rate(*(e * n), *(-cb / C * n)) == pytest.approx(expect, rel=1e-12)


def test_no_pairs_without_invariant_electric_part():
    assert O.schwinger_rate(0, 0, 0, 0, 0, 0) == 0.0
    assert O.schwinger_rate(0, 0, 0, 0.0, 0.0, 1e10) == 0.0          # pure B
    e = 0.5 * ES
    assert O.schwinger_rate(0, e, 0, 0, 0, e / C) == 0.0               # crossed, |E| = c|B|
    # weak field: exp(-pi E_s/E) underflows
    assert O.schwinger_rate(1e-3 * ES, 0, 0, 0, 0, 0) == 0.0


def _boost(e, b, beta_vec):
    """Field transformation to a frame moving with velocity beta c."""
    beta = np.asarray(beta_vec, dtype=np.float64)
    b2 = beta @ beta
    g = 1.0 / math.sqrt(1.0 - b2)
    n = beta / math.sqrt(b2)
    v = beta * C
    e_par, b_par = (e @ n) * n, (b @ n) * n
    e_new = e_par + g * (e - e_par + np.cross(v, b))
    b_new = b_par + g * (b - b_par - np.cross(v, e) / C ** 2)
    return e_new, b_new


def test_lorentz_invariance():
    rng = np.random.default_rng(7)
    for _ in range(20):
        e = rng.normal(size=3) * 0.2 * ES
        b = rng.normal(size=3) * 0.2 * ES / C
        r0 = O.schwinger_rate(*e, *b)
        beta = rng.normal(size=3)
        beta *= rng.uniform(0.1, 0.9) / np.linalg.norm(beta)
        e1, b1 = _boost(e, b, beta)
        # invariants first: the boost itself is checked
        assert (e1 @ e1 - C ** 2 * b1 @ b1) == pytest.approx(e @ e - C ** 2 * b @ b, rel=1e-9, abs=1e-9 * (e @ e))
        assert O.schwinger_rate(*e1, *b1) == pytest.approx(r0, rel=1e-8)


def test_count_is_poisson_small_mean():
    lam = 3.7
    n = 200000
    ks = np.array([O.schwinger_count(lam, 11, c, 0)[0] for c in range(n)])
    assert abs(ks.mean() - lam) < 5 * math.sqrt(lam / n)
    assert abs(ks.var() - lam) < 5 * lam * math.sqrt(2.0 / n) * 2
    for k in range(8):
        p = math.exp(-lam) * lam ** k / math.factorial(k)
        assert abs(np.mean(ks == k) - p) < 5 * math.sqrt(p * (1 - p) / n)
    assert O.schwinger_count(0.0, 11, 5, 0)[0] == 0


def test_count_gaussian_large_mean():
    lam = 400.0
    n = 50000
    ks = np.array([O.schwinger_count(lam, 12, c, 3)[0] for c in range(n)])
    assert abs(ks.mean() - lam) < 5 * math.sqrt(lam / n)
    assert abs(ks.std() - math.sqrt(lam)) < 0.05 * math.sqrt(lam)


def test_pairs_at_rest_in_cell_order():
    rng = np.random.default_rng(3)
    n = 4000
    cells = {k: np.zeros(n) for k in O.FIELD_KEYS}
    cells["ex"] = rng.uniform(0.05, 0.2, n) * ES
    dv, dt = 1e-21, 1e-17
    rate = O.schwinger_rate_array(cells)
    lam = rate * dv * dt
    w = float(np.median(lam) / 2)
    el, po = O.schwinger_pairs(cells, 100, dv, dt, w, 5, 2, capacity=n * 64)
    assert el.count == po.count > 0
    k_expect = sum(O.schwinger_count(l / w, 5, 100 + i, 2)[0] for i, l in enumerate(lam))
    assert el.count == k_expect
    for a in (el, po):
        assert np.all(a["ux"] == 0) and np.all(a["uy"] == 0) and np.all(a["uz"] == 0)
        assert np.all(a["w"] == w)
        assert np.all(a["tau"] > 0)
        assert np.all(np.diff(a["parent"]) >= 0)
        assert a["parent"][0] >= 100 and a["parent"][-1] < 100 + n
    assert np.array_equal(el["parent"], po["parent"])
    # electron and positron of one pair draw different optical depths
    assert np.mean(el["tau"] == po["tau"]) < 1e-3
    # mean macro-pairs per cell tracks lambda / w
    assert abs(el.count / np.sum(lam / w) - 1) < 5 / math.sqrt(el.count)


def test_rate_array_matches_scalar():
    rng = np.random.default_rng(9)
    cells = {k: rng.normal(size=50) * 0.1 * (ES if k[0] == "e" else ES / C) for k in O.FIELD_KEYS}
    arr = O.schwinger_rate_array(cells)
    for i in range(50):
        assert arr[i] == O.schwinger_rate(*[cells[k][i] for k in O.FIELD_KEYS])
