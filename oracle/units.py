"""Unit systems of the interface (paper Sec. 4): the factor that turns a
value in each system into the oracle's SI convention (E in V/m, B in T,
u = p/(m_e c), t in s, energies in m_e c^2).

TEST INFRASTRUCTURE ONLY (part of the oracle).

  SI            all factors 1.
  normalised    c = e = m_e = 1 with a reference angular frequency w:
                E in m_e c w / e, B in m_e w / e, t in 1/w; u and energies as
                in SI.  With a reference wavelength lambda, w = 2 pi c/lambda.
  HL, 1 MeV     hbar = c = eps0 = 1: energies in MeV, momenta in MeV/c,
                time in hbar/MeV, E and B in MeV^2 with the charge
                e = sqrt(4 pi alpha) (Heaviside-Lorentz), so that
                q E = force in MeV^2 = MeV / (hbar c / MeV).
"""
from __future__ import annotations

import math

import qed_inputs as QI

ALPHA = 7.2973525693e-3          # CODATA 2018
ME_MEV = QI.M_E * QI.C_LIGHT ** 2 / (1e6 * QI.Q_E)   # m_e c^2 in MeV from the SI constants

SI, NORM_OMEGA, NORM_LAMBDA, HL_MEV = 0, 1, 2, 3


def factors(system: int, ref: float = 0.0) -> dict:
    f = dict(e=1.0, b=1.0, u=1.0, t=1.0, energy=1.0)
    if system in (NORM_OMEGA, NORM_LAMBDA):
        w = ref if system == NORM_OMEGA else 2.0 * math.pi * QI.C_LIGHT / ref
        f.update(e=QI.M_E * QI.C_LIGHT * w / QI.Q_E, b=QI.M_E * w / QI.Q_E, t=1.0 / w)
    elif system == HL_MEV:
        mev_j = 1e6 * QI.Q_E
        force = mev_j / (QI.HBAR * QI.C_LIGHT / mev_j)       # newtons per MeV^2
        e_hl = math.sqrt(4.0 * math.pi * ALPHA)
        f.update(e=e_hl * force / QI.Q_E, b=e_hl * force / QI.Q_E / QI.C_LIGHT, u=1.0 / ME_MEV,
                 t=QI.HBAR / mev_j, energy=1.0 / ME_MEV)
    return f


def to_system(pop: dict, system: int, ref: float = 0.0) -> dict:
    """SI population (u, E, B, w) -> values in `system`."""
    f = factors(system, ref)
    out = {}
    for k, v in pop.items():
        s = f["u"] if k[0] == "u" else f["e"] if k[0] == "e" else f["b"] if k[0] == "b" else 1.0
        out[k] = v / s
    return out
