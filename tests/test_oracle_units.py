"""Pins of the oracle's unit factors (Sec. 4 unit systems) against values
the unit systems fix independently of the conversion code."""
import math

import pytest

import qed_inputs as QI
from oracle import units as U


def test_schwinger_field_in_heaviside_lorentz_mev():
    """In natural Heaviside-Lorentz units the critical field is m_e^2 / e
    with e = sqrt(4 pi alpha): 0.862 MeV^2."""
    f = U.factors(U.HL_MEV)
    es_hl = QI.E_SCHWINGER / f["e"]
    assert es_hl == pytest.approx(U.ME_MEV ** 2 / math.sqrt(4 * math.pi * U.ALPHA), rel=1e-13)
    # m_e c^2 from m_e, c, e agrees with the tabulated 0.51099895 MeV (rounding ~1e-11)
    assert U.ME_MEV == pytest.approx(QI.MEC2_MEV, rel=1e-10)
    # c B_s = E_s: the magnetic critical field has the same value in HL
    assert (QI.E_SCHWINGER / QI.C_LIGHT) / f["b"] == pytest.approx(es_hl, rel=1e-12)


def test_normalised_units():
    """E_s in units of m_e c w / e is m_e c^2 / (hbar w); the reference field
    of a 0.8 um laser is the a0 = 1 field; 1 / w is the time unit."""
    lam = 0.8e-6
    w = 2 * math.pi * QI.C_LIGHT / lam
    f = U.factors(U.NORM_LAMBDA, lam)
    assert QI.E_SCHWINGER / f["e"] == pytest.approx(QI.M_E * QI.C_LIGHT ** 2 / (QI.HBAR * w), rel=1e-12)
    assert f["e"] == pytest.approx(QI.laser_e0(1.0, lam), rel=1e-14)
    assert f["t"] == pytest.approx(lam / (2 * math.pi * QI.C_LIGHT), rel=1e-14)
    assert U.factors(U.NORM_OMEGA, w) == pytest.approx(f, rel=1e-14)


def test_hl_time_and_momentum_units():
    f = U.factors(U.HL_MEV)
    assert f["t"] == pytest.approx(6.582119569e-22, rel=1e-9)      # hbar / MeV in s
    assert f["u"] * U.ME_MEV == pytest.approx(1.0, rel=1e-15)
