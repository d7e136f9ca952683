"""Pins of the oracle's runtime path: table interpolation, inverse-CDF
sampling, the optical-depth step, kinematics and the ordered append.

The statistical pins (event fractions against the integrated cross
sections, spectra against quadrature CDFs, 10^7 samples each) and the
pins of the classical drag are in test_oracle_statistics.py."""
import math

import numpy as np
import pytest

import qed_inputs as QI
from oracle import oracle as O

R0 = O.rate_prefactor()


@pytest.fixture(scope="module")
def tables64():
    return (O.Table(O.BW, 1e-3, 1e2, 64, 64), O.Table(O.QS, 1e-3, 1e2, 64, 64))


def test_rate_exact_at_knots_and_linear_in_log_between(tables64):
    bw, qs = tables64
    chi = bw.chi_grid()
    for n in (0, 1, 17, 62, 63):
        g = 7.0
        assert bw.rate(chi[n], g) == pytest.approx(R0 * chi[n] / g * math.exp(bw.ln_rate[n]), rel=1e-13)
        assert qs.rate(chi[n], g) == pytest.approx(2 / 3 * R0 * math.exp(qs.ln_rate[n]) / g, rel=1e-13)
    # between knots: the paper's formula ln T* = ln T_n + (ln chi* - ln chi_n) slope
    rng = np.random.default_rng(3)
    lc = np.log(chi)
    for x in rng.uniform(lc[0], lc[-1], 200):
        ref_lnT = np.interp(x, lc, bw.ln_rate)
        ref_lnG = np.interp(x, lc, qs.ln_rate)
        c = math.exp(x)
        assert bw.rate(c, 3.0) == pytest.approx(R0 * c / 3.0 * math.exp(ref_lnT), rel=1e-12)
        assert qs.rate(c, 3.0) == pytest.approx(2 / 3 * R0 * math.exp(ref_lnG) / 3.0, rel=1e-12)


def test_rate_out_of_table_rules(tables64):
    bw, qs = tables64
    # QS: first / last stored value (Sec. 3.2), including chi = 0
    assert qs.rate(0.0, 2.0) == pytest.approx(2 / 3 * R0 * math.exp(qs.ln_rate[0]) / 2.0, rel=1e-15)
    assert qs.rate(1e6, 2.0) == pytest.approx(2 / 3 * R0 * math.exp(qs.ln_rate[-1]) / 2.0, rel=1e-15)
    # BW: asymptotic forms matched at the edges; continuous there; zero at chi = 0
    assert bw.rate(0.0, 10.0) == 0.0
    for edge in (bw.chi_min, bw.chi_max):
        lo, hi = bw.rate(edge * (1 - 1e-12), 10.0), bw.rate(edge * (1 + 1e-12), 10.0)
        assert lo == pytest.approx(hi, rel=1e-9)
    assert bw.rate(1e-4, 10.0) < 1e-300 * R0


def test_sampling_inverts_table_at_knots(tables64):
    bw, qs = tables64
    chi = bw.chi_grid()
    xi_bw, xi_qs = bw.frac_grid(), qs.frac_grid()
    for n in (5, 40, 63):
        for m in range(1, 63, 7):
            p = bw.cdf[n, m]
            if 0 < p < 0.5:
                xi, esel = bw.sample_bw(chi[n], p)
                assert esel and xi == pytest.approx(xi_bw[m], rel=1e-9, abs=1e-12)
                if p > 1e-3:   # 1 - (1 - p) reproduces p only to ~1e-16 absolute
                    xi2, esel2 = bw.sample_bw(chi[n], 1 - p)
                    assert not esel2 and xi2 == pytest.approx(xi_bw[m], rel=1e-9, abs=1e-12)
            lnxi = qs.sample_qs_lnxi(chi[n], math.exp(qs.cdf[n, m]))
            assert lnxi == pytest.approx(math.log(xi_qs[m]), rel=1e-9, abs=1e-9)


def test_qs_sampler_below_first_knot_is_cube_law(tables64):
    _, qs = tables64
    chi = 0.5
    L0 = np.interp(np.log(chi), np.log(qs.chi_grid()), qs.cdf[:, 0])
    for k in (1.0, 5.0):
        r = math.exp(L0 - k)
        assert qs.sample_qs_lnxi(chi, r) == pytest.approx(math.log(1e-12) - 3 * k, rel=1e-13)


def _fixed_population(n, gamma, e_field, photon):
    u = gamma if photon else math.sqrt(gamma * gamma - 1)
    z = np.zeros(n)
    return dict(ux=np.full(n, -u), uy=z.copy(), uz=z.copy(), ex=z.copy(), ey=np.full(n, e_field),
                ez=z.copy(), bx=z.copy(), by=z.copy(), bz=np.full(n, e_field / QI.C_LIGHT),
                w=np.linspace(0.5, 1.5, n))


def test_step_kinematics_conservation_and_order(tables64):
    bw, qs = tables64
    el, ph = QI.parity_population(seed=1, n=1 << 12)
    for pop, sp in ((el, O.ELECTRON), (ph, O.PHOTON)):
        p = O.Particles(pop, sp, id_base=77)
        O.init_optical_depth(p, seed=1)
        u0 = np.stack([p["ux"].copy(), p["uy"].copy(), p["uz"].copy()], 1)
        tau0 = p["tau"].copy()
        a1, a2 = O.Append(1 << 12), O.Append(1 << 12)
        flags = np.zeros(p.n, dtype=np.uint8)
        ev = O.step(bw, qs, p, 1e-16, seed=1, step_idx=3, a1=a1, a2=a2, flags=flags)
        idx = np.nonzero(flags)[0]
        assert ev == len(idx) > 0
        np.testing.assert_array_equal(a1["parent"], idx + 77)
        assert np.all(np.diff(a1["parent"]) > 0)
        np.testing.assert_array_equal(a1["w"], pop["w"][idx])
        # non-event particles: tau decreased, momentum untouched
        ne = flags == 0
        assert np.all(p["tau"][ne] <= tau0[ne])
        u1 = np.stack([p["ux"], p["uy"], p["uz"]], 1)
        np.testing.assert_array_equal(u1[ne], u0[ne])
        umag = np.linalg.norm(u0[idx], axis=1, keepdims=True)
        if sp == O.ELECTRON:
            pg = np.stack([a1["ux"], a1["uy"], a1["uz"]], 1)
            np.testing.assert_allclose(u1[idx] + pg, u0[idx], rtol=0, atol=1e-15 * float(umag.max()) * 4)
            # redrawn parent tau is -ln(u1) of the event block
            for j in idx[:50]:
                d = O.draws(1, 77 + j, 3, O.ELECTRON)
                assert p["tau"][j] == -math.log(d[1])
                assert a1["tau"][list(idx).index(j)] == -math.log(d[2])
        else:
            pe = np.stack([a1["ux"], a1["uy"], a1["uz"]], 1)
            pp = np.stack([a2["ux"], a2["uy"], a2["uz"]], 1)
            np.testing.assert_allclose(pe + pp, u0[idx], rtol=0, atol=1e-15 * float(umag.max()) * 4)
            assert np.all(np.isinf(p["tau"][idx]))
            np.testing.assert_array_equal(a2["parent"], a1["parent"])
            # collinear products: both along the photon
            cos = np.sum(pe * u0[idx], 1) / (np.linalg.norm(pe, axis=1) * umag[:, 0])
            np.testing.assert_allclose(cos, 1.0, atol=1e-12)
            # energy defect of collinear massive products <= (1/(2 g))(1/xi + 1/(1 - xi))
            ge = np.sqrt(1 + np.sum(pe * pe, 1))
            gp = np.sqrt(1 + np.sum(pp * pp, 1))
            gg = umag[:, 0]
            xi = np.linalg.norm(pe, axis=1) / gg
            bound = (1 / (2 * gg)) * (1 / xi + 1 / (1 - xi))
            assert np.all(ge + gp - gg <= bound * (1 + 1e-9) + 1e-12)


@pytest.mark.parametrize("emin", [0.0, 30.0])
def test_generate_equals_step_on_its_own_events(tables64, emin):
    """The step of Fig. 1 split into the paper's separate calls: the
    optical-depth evolution gives the step's event flags and, where there is
    no event, its optical depths; the production calls (pair generation,
    photon emission with momentum update; Sec. 3.1, 3.2) on those flags
    create the same products in the same order, give the flagged parents
    the same momenta and optical depths and leave every other particle as
    it was, with and without a photon energy threshold.  The oracle's step
    and its separate calls are different code paths, so this pins each
    against the other."""
    bw, qs = tables64
    el, ph = QI.parity_population(seed=4, n=3000)
    for pop, sp in ((el, O.ELECTRON), (ph, O.PHOTON)):
        ps = O.Particles(pop, sp, id_base=500)
        O.init_optical_depth(ps, seed=4)
        tau0 = ps["tau"].copy()
        pg = O.Particles(pop, sp, id_base=500, tau=tau0)
        s1, s2 = O.Append(3000), O.Append(3000)
        flags = np.zeros(ps.n, dtype=np.uint8)
        O.step(bw, qs, ps, 1e-16, seed=4, step_idx=7, a1=s1, a2=s2, photon_min_energy=emin, flags=flags)
        assert 0 < int(flags.sum()) < ps.n
        g1, g2 = O.Append(3000), O.Append(3000)
        O.generate(bw, qs, pg, flags, 4, 7, g1, g2 if sp == O.PHOTON else None, photon_min_energy=emin)
        assert g1.count == s1.count
        if sp == O.PHOTON or emin == 0.0:
            assert g1.count == int(flags.sum())
        else:   # the photon threshold keeps some photons and drops others
            assert 0 < g1.count < int(flags.sum())
        for k in ("parent", "ux", "uy", "uz", "w", "tau"):
            np.testing.assert_array_equal(g1[k], s1[k])
            if sp == O.PHOTON:
                np.testing.assert_array_equal(g2[k], s2[k])
        ev = flags == 1
        for k in ("ux", "uy", "uz", "tau"):
            np.testing.assert_array_equal(pg[k][ev], ps[k][ev])
        np.testing.assert_array_equal(pg["tau"][~ev], tau0[~ev])
        for k in ("ux", "uy", "uz"):
            np.testing.assert_array_equal(pg[k][~ev], np.asarray(pop[k], dtype=np.float64)[~ev])
        # and the evolution call is its other half: the same flags, and the
        # step's optical depths wherever there was no event
        pe = O.Particles(pop, sp, id_base=500, tau=tau0)
        fe = np.zeros(pe.n, dtype=np.uint8)
        O.evolve(bw if sp == O.PHOTON else qs, pe, 1e-16, fe)
        np.testing.assert_array_equal(fe, flags)
        np.testing.assert_array_equal(pe["tau"][~ev], ps["tau"][~ev])


def test_init_optical_depth_keying():
    pop = _fixed_population(64, 10.0, 1e12, False)
    p = O.Particles(pop, O.POSITRON, id_base=2**40)
    O.init_optical_depth(p, seed=9)
    for i in (0, 13, 63):
        ctr = [2**40 + i, 2**64 - 1, O.POSITRON, 0]
        v = sum(c << (64 * k) for k, c in enumerate(ctr)) - 1
        g = np.random.Philox(key=np.array([9, 0], dtype=np.uint64),
                             counter=np.array([(v >> (64 * k)) & (2**64 - 1) for k in range(4)], dtype=np.uint64))
        w = int(g.random_raw(1)[0])
        assert p["tau"][i] == -math.log((2 * (w >> 12) + 1) / 2.0**53)


def test_capacity_and_threshold(tables64):
    bw, qs = tables64
    el, _ = QI.parity_population(seed=2, n=1 << 12)
    ref = O.Particles(el, O.ELECTRON)
    O.init_optical_depth(ref, seed=2)
    small = O.Particles(el, O.ELECTRON, tau=ref["tau"])
    a_full, a_small = O.Append(1 << 12), O.Append(10)
    n_full = O.step(bw, qs, ref, 1e-16, 2, 0, a_full)
    O.step(bw, qs, small, 1e-16, 2, 0, a_small)
    assert a_small.count == a_full.count == n_full > 10
    np.testing.assert_array_equal(a_small["ux"], a_full["ux"][:10])
    np.testing.assert_array_equal(small["ux"], ref["ux"])
    # threshold: photons below it are dropped but the parent still recoils
    thr = O.Particles(el, O.ELECTRON, tau=small["tau"] * 0 + ref["tau"])
    base = O.Particles(el, O.ELECTRON, tau=ref["tau"])
    O.init_optical_depth(base, 2)
    O.init_optical_depth(thr, 2)
    a_b, a_t = O.Append(1 << 12), O.Append(1 << 12)
    O.step(bw, qs, base, 1e-16, 2, 0, a_b)
    O.step(bw, qs, thr, 1e-16, 2, 0, a_t, photon_min_energy=2.0)
    gg = np.linalg.norm(np.stack([a_b["ux"], a_b["uy"], a_b["uz"]], 1), axis=1)
    keep = gg >= 2.0
    assert a_t.count == int(keep.sum()) < a_b.count
    np.testing.assert_array_equal(a_t["parent"], a_b["parent"][keep])
    np.testing.assert_array_equal(thr["ux"], base["ux"])


def test_qed_threshold_classical_drag():
    """Below chi_qed_min (Sec. 6, WarpX's minimum quantum parameter): no
    optical-depth evolution; photons untouched; leptons lose the classically
    radiated energy (2/3) (alpha m c^2/hbar) chi^2 dt (in m c^2) along u."""
    import math
    import qed_inputs as QI
    qs = O.Table(O.QS, 1e-3, 1e2, 16, 16)
    bw = O.Table(O.BW, 1e-3, 1e2, 16, 16)
    n = 4
    d = {k: np.zeros(n) for k in QI.FIELDS}
    d["ux"][:] = [-100.0, -2000.0, -5000.0, -0.5]
    d["uy"][:] = [3.0, 0.0, 10.0, 0.1]
    d["ey"][:] = 1e13
    d["bz"][:] = 1e13 / QI.C_LIGHT
    d["w"][:] = 1.0
    chi = O.chi_array(d, False)
    thr = float(np.sort(chi)[2] * 1.0001)          # three below, one above
    p = O.Particles(d, O.ELECTRON, tau=np.full(n, 0.5))
    flags = np.zeros(n, dtype=np.uint8)
    dt = 1e-16
    O.step(bw, qs, p, dt, 1, 0, O.Append(n), flags=flags, chi_qed_min=thr)
    for i in range(n):
        u0 = np.array([d["ux"][i], d["uy"][i], 0.0])
        u1 = np.array([p["ux"][i], p["uy"][i], p["uz"][i]])
        if chi[i] < thr:
            assert p["tau"][i] == 0.5 and flags[i] == 0
            assert u1 @ u1 < u0 @ u0            # energy lost (its amount: test_oracle_statistics)
            assert np.allclose(np.cross(u0, u1), 0.0, atol=1e-12 * (u0 @ u0))   # along u
        else:
            assert p["tau"][i] != 0.5                                    # evolved as usual
    # photons below the threshold are left alone
    ph = O.Particles(d, O.PHOTON, tau=np.full(n, 0.5))
    O.step(bw, qs, ph, dt, 1, 0, O.Append(n), O.Append(n), chi_qed_min=1e9)
    assert np.all(ph["tau"] == 0.5) and np.all(ph["ux"] == d["ux"])
