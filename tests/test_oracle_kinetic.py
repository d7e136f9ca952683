"""Pins of the kinetic reference (oracle/kinetic.py) for electrons radiating
in a static perpendicular magnetic field: probability conservation, the
exact one-step law, and agreement with the oracle's own particle loop
(Boris push + Monte Carlo step) within the statistical error."""
import math

import numpy as np
import pytest

import qed_inputs as QI
from oracle import kinetic as K
from oracle import oracle as O

C, ES = QI.C_LIGHT, QI.E_SCHWINGER


@pytest.fixture(scope="module")
def qs():
    return O.Table(O.QS, 1e-3, 1e2, 32, 32)


def _edges(u0, n=600):
    return np.exp(np.linspace(np.log(0.3), np.log(u0 * 1.001), n + 1))


def test_implied_cdf_matches_sampling(qs):
    """The forward CDF inverts the table sampler: P(sample(r)) = r."""
    rng = np.random.default_rng(1)
    for chi in (2e-3, 0.5, 7.0, 80.0):
        r = rng.uniform(1e-6, 1 - 1e-9, 2000)
        lx = qs.sample_n(np.full(2000, chi), r)
        p = K.implied_cdf(qs, chi, np.exp(lx))
        assert np.max(np.abs(p - r) / r) < 1e-9


def test_probability_is_conserved_and_first_step_is_exact(qs):
    b, u0, dt = 1e-3, 999.9995, 1e-17
    ch = K.StaticFieldChain(qs, b, u0, dt, _edges(u0), np.exp(np.linspace(np.log(1e-25), np.log(1e3), 401)))
    w = qs.rate(u0 * b, math.sqrt(1 + u0 * u0))
    ch.step()
    p1 = -math.expm1(-w * dt)
    assert ch.atom == pytest.approx(1 - p1, rel=1e-14)
    assert ch.atom + ch.cells.sum() == pytest.approx(1.0, abs=1e-12)
    assert ch.photons.sum() == pytest.approx(p1, rel=1e-9)
    ch.run(49)
    assert ch.atom + ch.cells.sum() == pytest.approx(1.0, abs=1e-10)


def test_chain_matches_oracle_particle_loop(qs):
    """Case 1 geometry (B = 1e-3 E_s/c, gamma0 = 1000), 60 steps of 1e-17 s:
    the oracle's push + step loop over 2^15 electrons against the chain."""
    n, steps, dt = 1 << 15, 60, 1e-17
    b_si = 1e-3 * ES / C
    g0 = 1000.0
    u0 = math.sqrt(g0 * g0 - 1)
    d = {k: np.zeros(n) for k in QI.FIELDS}
    d["uy"][:] = u0
    d["w"][:] = 1.0
    p = O.Particles(d, O.ELECTRON)
    O.init_optical_depth(p, 5)
    x, y, z = np.zeros(n), np.zeros(n), np.zeros(n)
    f = O.uniform_field(b0=(0.0, 0.0, b_si))
    e_ph = np.exp(np.linspace(np.log(1e-12), np.log(2e3), 401))
    ph_hist = np.zeros(len(e_ph) - 1)
    for s in range(steps):
        O.push(p, x, y, z, f, s * dt, dt)
        a = O.Append(n)
        O.step(qs, qs, p, dt, 5, s, a)
        en = np.sqrt(a["ux"] ** 2 + a["uy"] ** 2 + a["uz"] ** 2)
        ph_hist += np.histogram(en, e_ph)[0]
    um = np.sqrt(p["ux"] ** 2 + p["uy"] ** 2 + p["uz"] ** 2)
    # |u| is kept by the rotation, so the chain in |u| = u0 b is the model
    ch = K.StaticFieldChain(qs, u0 * 0 + b_si * C / ES, u0, dt, _edges(u0), e_ph).run(steps)
    # never-emitted fraction
    atom_mc = np.mean(np.abs(um - u0) < 1e-9 * u0)
    assert abs(atom_mc - ch.atom) < 5 * math.sqrt(ch.atom * (1 - ch.atom) / n) + 1e-12
    # |u| distribution on 12 coarse cells
    coarse = np.exp(np.linspace(np.log(0.3), np.log(u0 * 1.001), 13))
    mc = np.histogram(um[np.abs(um - u0) >= 1e-9 * u0], coarse)[0] / n
    fine_c = np.sqrt(ch.eu[:-1] * ch.eu[1:])
    ref = np.array([ch.cells[(fine_c >= lo) & (fine_c < hi)].sum() for lo, hi in zip(coarse[:-1], coarse[1:])])
    sig = np.sqrt(np.maximum(ref, 1e-6) / n)
    assert np.all(np.abs(mc - ref) < 5 * sig + 2e-3), (mc, ref)
    # photons per electron and mean photon energy
    e_c = np.sqrt(e_ph[:-1] * e_ph[1:])
    assert ph_hist.sum() / n == pytest.approx(ch.photons.sum(), rel=5 / math.sqrt(ph_hist.sum()) + 1e-3)
    assert (ph_hist @ e_c) / ph_hist.sum() == pytest.approx((ch.photons @ e_c) / ch.photons.sum(), rel=0.03)
