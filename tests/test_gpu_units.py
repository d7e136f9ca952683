"""The fused step and the chi calls with the caller's arrays in each unit
system of the interface (Sec. 4: SI, normalised with a reference frequency
or wavelength, Heaviside-Lorentz with 1 MeV), against the oracle run on the
same population in SI (FP64).  Converting the inputs costs one rounding per
value, so values are compared at 1e-12 (u, tau, products, converted back to
SI) and chi at 1e-13; event flags and product parents are bit-exact."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_2110_00256_amd as Q  # noqa: E402
import qed_inputs as QI  # noqa: E402
from oracle import oracle as O  # noqa: E402
from oracle import units as U  # noqa: E402
from tests.gpu_util import dev_pop, host, rel_close  # noqa: E402

SYSTEMS = [(U.SI, 0.0), (U.NORM_OMEGA, 2.354564459e15), (U.NORM_LAMBDA, 0.8e-6), (U.HL_MEV, 0.0)]
RANGE = (1e-3, 1e2)


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return Q.Context(0)


@pytest.fixture(scope="module")
def tabs():
    return ((Q.Table.generate(Q.BW, *RANGE, 64, 64).to_device(),
             Q.Table.generate(Q.QS, *RANGE, 64, 64, 1e-12).to_device()),
            (O.Table(O.BW, *RANGE, 64, 64), O.Table(O.QS, *RANGE, 64, 64, 1e-12)))


@pytest.mark.parametrize("system,ref", SYSTEMS)
def test_step_in_unit_system(ctx, tabs, system, ref):
    (bw, qs), (obw, oqs) = tabs
    n, seed, dt_si, steps = 20000, 13, 1e-16, 3
    f = U.factors(system, ref)
    el, ph = QI.parity_population(seed=seed, n=n)
    oe, og = O.Particles(el, O.ELECTRON, 0), O.Particles(ph, O.PHOTON, n)
    O.init_optical_depth(oe, seed)
    O.init_optical_depth(og, seed)
    de = dev_pop(U.to_system(el, system, ref), torch.float64, tau=oe["tau"])
    dg = dev_pop(U.to_system(ph, system, ref), torch.float64, tau=og["tau"])
    pe, pg = Q.particles(de, Q.ELECTRON, 0), Q.particles(dg, Q.PHOTON, n)
    ctx.set_units(system, ref)
    try:
        chi = torch.empty(n, dtype=torch.float64, device="cuda")
        Q.chi_lepton(ctx, pe, chi)
        assert rel_close(host(chi), O.chi_array(el, False), 1e-13, floor=1e-300) <= 1.0
        bufs = [Q.AppendBuffer(steps * n, torch.float64) for _ in range(3)]
        flags = [torch.zeros(n, dtype=torch.uint8, device="cuda") for _ in range(2)]
        threshold_si = 2.0                                  # m_e c^2
        desc = Q.StepDesc([pe, pg], bw=bw, qs=qs, photons=bufs[0], electrons=bufs[1], positrons=bufs[2],
                          flags=flags, dt=dt_si / f["t"], seed=seed, photon_min_energy=threshold_si / f["energy"])
        apps = [O.Append(steps * n) for _ in range(3)]
        for s in range(steps):
            desc.set_step(s)
            Q.step(ctx, desc)
            fe, fg = np.zeros(n, np.uint8), np.zeros(n, np.uint8)
            O.step(obw, oqs, oe, dt_si, seed, s, apps[0], photon_min_energy=threshold_si, flags=fe)
            O.step(obw, oqs, og, dt_si, seed, s, apps[1], apps[2], flags=fg)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(flags[0].cpu().numpy(), fe)
            np.testing.assert_array_equal(flags[1].cpu().numpy(), fg)
    finally:
        ctx.set_units(Q.UNITS_SI)
    for d, o in ((de, oe), (dg, og)):
        umag = np.sqrt(o["ux"] ** 2 + o["uy"] ** 2 + o["uz"] ** 2)
        for k in ("ux", "uy", "uz"):
            assert rel_close(host(d[k]) * f["u"], o[k], 1e-12, floor=np.maximum(umag, 1e-300)) <= 1.0, k
        assert rel_close(host(d["tau"]), o["tau"], 1e-12) <= 1.0
    for b, a in zip(bufs, apps):
        cnt = int(b.count.item())
        assert cnt == a.count
        np.testing.assert_array_equal(b.parent[:cnt].cpu().numpy(), a["parent"])
        pm = np.sqrt(a["ux"] ** 2 + a["uy"] ** 2 + a["uz"] ** 2)
        for k in ("ux", "uy", "uz"):
            assert rel_close(host(b.a[k][:cnt]) * f["u"], a[k], 1e-12, floor=np.maximum(pm, 1e-300)) <= 1.0
