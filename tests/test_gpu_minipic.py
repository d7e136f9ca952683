"""Closed loop of particle push + QED step on the GPU against the same loop in
the oracle (FP64), for the three benchmark geometries of Sec. 5.1:
  case 1  gamma0 = 1000 perpendicular to a static B = 1e-3 E_s/c (chi = 1), 1 fs
  case 2  gamma0 = 4120 against a CP plane wave, E0 = 1.22e-4 E_s (chi = 1), 3 fs
  case 3  gamma0 = 1000 perpendicular to B = 9e-3 E_s/c (chi = 9), 0.1 fs
Each step: push (Boris, fields at the new positions stored), then the QED
step (photon emission, parent recoil); photons are collected, not evolved.
Bar as for the fused step: event flags, photon counts and parent ids
bit-exact every step; momenta, positions and optical depths within 1e-12
relative (the two pushes round differently: the oracle is compiled without
contraction, the kernel may fuse multiply-adds).  Then the loop's exact
invariant: in a static magnetic field the Boris rotation keeps |u| and
collinear emission moves |u| into the photon, so sum |u_e| + sum gamma_photon
stays constant."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_2110_00256_amd as Q  # noqa: E402
import qed_inputs as QI  # noqa: E402
from oracle import oracle as O  # noqa: E402
from tests.gpu_util import host, rel_close  # noqa: E402

C, ES = QI.C_LIGHT, QI.E_SCHWINGER
CASES = {
    "case1": dict(gamma0=1000.0, field=("B", 1e-3), t_end=1e-15, steps=100),
    "case2": dict(gamma0=4120.0, field=("CP", 1.22e-4), t_end=3e-15, steps=100),
    "case3": dict(gamma0=1000.0, field=("B", 9e-3), t_end=1e-16, steps=100),
}
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


def _initial(case, n, seed):
    """Mono-energetic electrons: along +y in a B along +z, along -x against
    the wave (which runs along +x); positions spread over one wavelength."""
    c = CASES[case]
    um = math.sqrt(c["gamma0"] ** 2 - 1)
    rng = np.random.default_rng(seed)
    d = {k: np.zeros(n) for k in QI.FIELDS}
    if c["field"][0] == "B":
        d["uy"][:] = um
    else:
        d["ux"][:] = -um
    d["w"] = rng.uniform(0.5, 1.5, n)
    pos = [rng.uniform(0, 0.8e-6, n), np.zeros(n), np.zeros(n)]
    return d, pos


def _fields(case):
    kind, amp = CASES[case]["field"]
    if kind == "B":
        return Q.uniform_field(b0=(0.0, 0.0, amp * ES / C)), O.uniform_field(b0=(0.0, 0.0, amp * ES / C))
    return Q.cp_wave(amp * ES, 0.8e-6, 1), O.cp_wave(amp * ES, 0.8e-6, 1)


@pytest.mark.parametrize("case", list(CASES))
def test_loop_matches_oracle(ctx, tabs, case):
    (bw, qs), (obw, oqs) = tabs
    n, seed = 4096, 11
    cfg = CASES[case]
    dt = cfg["t_end"] / cfg["steps"]
    d, pos = _initial(case, n, seed)
    g = {k: torch.as_tensor(v).cuda() for k, v in d.items()}
    g["tau"] = torch.empty(n, dtype=torch.float64, device="cuda")
    gx = [torch.as_tensor(p.copy()).cuda() for p in pos]
    pe = Q.particles(g, Q.ELECTRON, 0)
    Q.init_optical_depth(ctx, pe, seed)
    op = O.Particles(d, O.ELECTRON, 0)
    O.init_optical_depth(op, seed)
    ox = [p.copy() for p in pos]
    gf, of = _fields(case)
    ph = Q.AppendBuffer(n, torch.float64)
    flags = torch.zeros(n, dtype=torch.uint8, device="cuda")
    desc = Q.StepDesc([pe], bw=bw, qs=qs, photons=ph, electrons=Q.AppendBuffer(0, torch.float64),
                      positrons=Q.AppendBuffer(0, torch.float64), flags=[flags], dt=dt, seed=seed)
    u_abs0 = np.sqrt(d["ux"] ** 2 + d["uy"] ** 2 + d["uz"] ** 2)
    photon_energy = 0.0
    events = 0
    for s in range(cfg["steps"]):
        t = s * dt
        Q.push(ctx, pe, *gx, gf, t, dt)
        O.push(op, *ox, of, t, dt)
        ph.reset()
        desc.set_step(s)
        Q.step(ctx, desc)
        oa = O.Append(n)
        ofl = np.zeros(n, dtype=np.uint8)
        O.step(obw, oqs, op, dt, seed, s, oa, flags=ofl)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(flags.cpu().numpy(), ofl, err_msg=f"{case} step {s}")
        cnt = int(ph.count.item())
        assert cnt == oa.count, f"{case} step {s}"
        np.testing.assert_array_equal(ph.parent[:cnt].cpu().numpy(), oa["parent"])
        pu = np.sqrt(sum(host(ph.a[k][:cnt]) ** 2 for k in ("ux", "uy", "uz")))
        assert rel_close(pu, np.sqrt(oa["ux"] ** 2 + oa["uy"] ** 2 + oa["uz"] ** 2), 1e-12,
                         floor=cfg["gamma0"]) <= 1.0
        photon_energy += float(np.sum(pu * host(ph.a["w"][:cnt])))
        events += cnt
    for k in ("ux", "uy", "uz"):
        assert rel_close(host(g[k]), op[k], 1e-12, floor=cfg["gamma0"]) <= 1.0, k
    assert rel_close(host(g["tau"]), op["tau"], 1e-12) <= 1.0
    for a, b in zip(gx, ox):
        assert rel_close(host(a), b, 1e-12, floor=1e-6) <= 1.0
    assert events > n // 2, "too few emissions to test anything"
    if CASES[case]["field"][0] == "B":
        u_abs = np.sqrt(sum(host(g[k]) ** 2 for k in ("ux", "uy", "uz")))
        before = float(np.sum(u_abs0 * d["w"]))
        after = float(np.sum(u_abs * d["w"])) + photon_energy
        assert after == pytest.approx(before, rel=1e-12)
    print(f"{case}: {events} photons over {cfg['steps']} steps")


@pytest.mark.parametrize("case", ["case1", "case3"])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("n_tab", [32, 256])
def test_static_field_spectra_match_kinetic_reference(ctx, case, dtype, n_tab):
    """2^20 electrons through the GPU loop against the kinetic reference
    (the exact Markov chain of the same tables): never-emitted fraction,
    |u| distribution on 12 cells, photons per electron, mean photon energy."""
    from oracle import kinetic as K
    n = 1 << 20
    cfg = CASES[case]
    steps, dt = cfg["steps"], cfg["t_end"] / cfg["steps"]
    b_norm = cfg["field"][1]
    rng_tab = (1e-3, 1e2)
    bw = Q.Table.generate(Q.BW, *rng_tab, n_tab, n_tab).to_device()
    qs = Q.Table.generate(Q.QS, *rng_tab, n_tab, n_tab, 1e-12).to_device()
    oqs = O.Table(O.QS, *rng_tab, n_tab, n_tab, 1e-12)
    d, pos = _initial(case, n, 3)
    d["w"][:] = 1.0
    g = {k: torch.as_tensor(v).to("cuda", dtype) for k, v in d.items()}
    g["tau"] = torch.empty(n, dtype=dtype, device="cuda")
    gx = [torch.as_tensor(p).to("cuda", dtype) for p in pos]
    pe = Q.particles(g, Q.ELECTRON, 0)
    Q.init_optical_depth(ctx, pe, 3)
    gf, _ = _fields(case)
    ph = Q.AppendBuffer(n, dtype)
    desc = Q.StepDesc([pe], bw=bw, qs=qs, photons=ph, electrons=Q.AppendBuffer(0, dtype),
                      positrons=Q.AppendBuffer(0, dtype), dt=dt, seed=3)
    u0 = math.sqrt(cfg["gamma0"] ** 2 - 1)
    e_ph = np.exp(np.linspace(np.log(1e-25), np.log(2 * cfg["gamma0"]), 401))
    ph_hist = np.zeros(len(e_ph) - 1)
    for s in range(steps):
        Q.push(ctx, pe, *gx, gf, s * dt, dt)
        ph.reset()
        desc.set_step(s)
        Q.step(ctx, desc)
        cnt = int(ph.count.item())
        en = torch.sqrt(ph.a["ux"][:cnt].double() ** 2 + ph.a["uy"][:cnt].double() ** 2 +
                        ph.a["uz"][:cnt].double() ** 2).cpu().numpy()
        ph_hist += np.histogram(en, e_ph)[0]
    um = np.sqrt(sum(host(g[k]) ** 2 for k in ("ux", "uy", "uz")))
    edges = np.exp(np.linspace(np.log(0.3), np.log(u0 * 1.001), 601))
    ch = K.StaticFieldChain(oqs, b_norm, u0, dt, edges, e_ph).run(steps)
    # never-emitted electrons keep |u| to rounding; in FP32 the rounding of
    # 100 rotations (~1e-6 of |u|) hides the softest emissions, so the
    # fraction is checked in FP64 only
    tol_atom = 1e-9 if dtype == torch.float64 else 1e-6
    atom = np.abs(um - u0) < tol_atom * u0
    res = {"atom": (float(atom.mean()), ch.atom)}
    if dtype == torch.float64:
        assert abs(atom.mean() - ch.atom) < 5 * math.sqrt(ch.atom * (1 - ch.atom) / n) + 1e-4
    coarse = np.exp(np.linspace(np.log(0.3), np.log(u0 * 1.001), 13))
    mc = np.histogram(um[~atom], coarse)[0] / n
    fc = np.sqrt(edges[:-1] * edges[1:])
    ref = np.array([ch.cells[(fc >= lo) & (fc < hi)].sum() for lo, hi in zip(coarse[:-1], coarse[1:])])
    res["max_cell_dev"] = float(np.max(np.abs(mc - ref)))
    assert np.all(np.abs(mc - ref) < 5 * np.sqrt(np.maximum(ref, 1e-6) / n) + 2e-3), (mc, ref)
    e_c = np.sqrt(e_ph[:-1] * e_ph[1:])
    res["photons_per_e"] = (float(ph_hist.sum() / n), float(ch.photons.sum()))
    res["mean_photon"] = (float(ph_hist @ e_c / ph_hist.sum()), float(ch.photons @ e_c / ch.photons.sum()))
    assert res["photons_per_e"][0] == pytest.approx(res["photons_per_e"][1], rel=5 / math.sqrt(ph_hist.sum()) + 1e-3)
    assert res["mean_photon"][0] == pytest.approx(res["mean_photon"][1], rel=0.01)
    print(f"{case} {dtype} {n_tab}x{n_tab}: {res}")
