"""Pins of the oracle's particle push (Boris scheme in prescribed fields)
against what the mechanics fixes: the exact rotation of the Boris scheme in
a pure magnetic field, exact uniform acceleration in a pure electric field,
the E x B drift, the field structure of a circularly polarised plane wave,
light-speed photon motion, and the quantum parameter of the paper's
counter-propagating benchmark geometry (Sec. 5.1, case 2)."""
import math

import numpy as np
import pytest

import qed_inputs as QI
from oracle import oracle as O

C, QE, ME, ES = QI.C_LIGHT, QI.Q_E, QI.M_E, QI.E_SCHWINGER


def _pop(u, species=O.ELECTRON):
    u = np.atleast_2d(np.asarray(u, dtype=np.float64))
    n = len(u)
    d = {k: np.zeros(n) for k in QI.FIELDS}
    d["ux"], d["uy"], d["uz"] = u[:, 0].copy(), u[:, 1].copy(), u[:, 2].copy()
    d["w"] = np.ones(n)
    p = O.Particles(d, species)
    return p, np.zeros(n), np.zeros(n), np.zeros(n)


def _rotate_z(v, ang):
    c, s = math.cos(ang), math.sin(ang)
    return np.array([c * v[0] - s * v[1], s * v[0] + c * v[1], v[2]])


@pytest.mark.parametrize("species,sign", [(O.ELECTRON, -1.0), (O.POSITRON, 1.0)])
def test_pure_magnetic_field_is_an_exact_rotation(species, sign):
    b = 1e-3 * ES / C                       # case 1 field
    u0 = np.array([0.0, 1000.0, 0.0])
    p, x, y, z = _pop(u0, species)
    f = O.uniform_field(b0=(0.0, 0.0, b))
    dt = 1e-17
    g = math.sqrt(1 + u0 @ u0)
    theta = 2 * math.atan(QE * b * dt / (2 * ME * g))   # rotation angle of one Boris step
    for n in range(1, 201):
        O.push(p, x, y, z, f, (n - 1) * dt, dt)
    u = np.array([p["ux"][0], p["uy"][0], p["uz"][0]])
    # positive charge rotates clockwise about +z (du/dt = (q/m) u x B / gamma)
    expect = _rotate_z(u0, -sign * 200 * theta)
    assert np.linalg.norm(u) == pytest.approx(np.linalg.norm(u0), rel=1e-13)
    assert np.allclose(u, expect, rtol=0, atol=1e-9 * np.linalg.norm(u0))
    # the Boris angle approximates the cyclotron angle omega dt to O(dt^3)
    wdt = QE * b * dt / (ME * g)
    assert abs(theta - wdt) < wdt ** 3


def test_pure_electric_field_is_exact_uniform_acceleration():
    e = np.array([1e12, -2e11, 5e11])
    p, x, y, z = _pop([0.0, 0.0, 0.0], O.POSITRON)
    f = O.uniform_field(e0=tuple(e))
    dt = 1e-16
    for n in range(50):
        O.push(p, x, y, z, f, n * dt, dt)
    u = np.array([p["ux"][0], p["uy"][0], p["uz"][0]])
    assert np.allclose(u, QE * e / (ME * C) * 50 * dt, rtol=1e-13)
    # the stored fields are the prescribed ones
    assert p["ex"][0] == e[0] and p["ey"][0] == e[1] and p["ez"][0] == e[2]


def test_exb_drift():
    b = 1.0
    e = 0.01 * C * b                        # E << cB: drift speed 0.01 c
    p, x, y, z = _pop([0.0, 0.0, 0.0], O.ELECTRON)
    f = O.uniform_field(e0=(0.0, e, 0.0), b0=(0.0, 0.0, b))
    w = QE * b / ME
    dt = 2 * math.pi / w / 200
    n = 200 * 50                            # 50 gyrations
    for k in range(n):
        O.push(p, x, y, z, f, k * dt, dt)
    vd = x[0] / (n * dt)                    # E x B = (E_y B_z) x_hat / B^2
    assert vd == pytest.approx(e / b, rel=0.02)
    assert abs(y[0]) < 0.05 * abs(x[0])


def test_cp_wave_fields_and_photon_motion():
    a, lam = 1.22e-4 * ES, 0.8e-6
    p, x, y, z = _pop([[-5.0, 0.0, 0.0], [0.0, 3.0, 4.0]], O.PHOTON)
    x[:] = [1e-7, -3e-7]
    f = O.cp_wave(a, lam, direction=1, phase=0.3)
    dt = 2e-16
    O.push(p, x, y, z, f, 1e-15, dt)
    assert x[0] == pytest.approx(1e-7 - C * dt, rel=1e-15)
    assert y[1] == pytest.approx(C * dt * 0.6, rel=1e-15) and z[1] == pytest.approx(C * dt * 0.8, rel=1e-15)
    for i in range(2):
        e = np.array([p["ex"][i], p["ey"][i], p["ez"][i]])
        bb = np.array([p["bx"][i], p["by"][i], p["bz"][i]])
        assert np.linalg.norm(e) == pytest.approx(a, rel=1e-14)
        assert np.linalg.norm(bb) * C == pytest.approx(a, rel=1e-14)
        assert abs(e @ bb) < 1e-14 * a * a / C                     # G = 0
        assert np.cross(e, bb) @ np.array([1.0, 0, 0]) > 0        # Poynting along +x
        ph = 2 * math.pi / lam * (x[i] - C * (1e-15 + dt)) + 0.3
        assert e[1] == pytest.approx(a * math.cos(ph), abs=1e-12 * a)


def test_counterpropagating_case2_chi():
    """Sec. 5.1 case 2: gamma0 = 4120 against a CP wave of E0 = 1.22e-4 E_s
    gives chi ~ 1 (exactly (gamma + |u|) E0 / E_s for motion along -x)."""
    g0 = 4120.0
    um = math.sqrt(g0 * g0 - 1)
    p, x, y, z = _pop([-um, 0.0, 0.0], O.ELECTRON)
    f = O.cp_wave(1.22e-4 * ES, 0.8e-6, direction=1)
    O.push(p, x, y, z, f, 0.0, 0.0)        # dt = 0: only stores the fields
    chi = O.chi_array({k: p[k] for k in QI.FIELDS[:9]}, False)[0]
    assert chi == pytest.approx((g0 + um) * 1.22e-4, rel=1e-12)
    assert chi == pytest.approx(1.0, rel=0.01)
