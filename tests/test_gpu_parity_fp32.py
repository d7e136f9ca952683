"""FP32 HIP path against the FP64 oracle, compared step by step: before
each step the oracle takes the GPU's FP32 state (exactly representable in
FP64), so that an allowed event flip does not propagate.

Bar: values within 1e-5 relative (tau: scale max(|tau|, 1); momenta: the
parent's |u|); an event flag may differ only where the oracle's updated
optical depth lies within 1e-6 of zero; products are matched by parent id
and compared for every parent whose flag agrees."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_2110_00256_amd as Q  # noqa: E402
import qed_inputs as QI  # noqa: E402
from oracle import oracle as O  # noqa: E402
from tests.gpu_util import compare_append, host, lib_tables, oracle_tables, rel_close  # noqa: E402

RTOL = 1e-5
TIE = 1e-6
RANGE = (1e-4, 1e3)


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return Q.Context(0)


@pytest.fixture(scope="module")
def tabs():
    return lib_tables(RANGE, RANGE, 256, 256), oracle_tables(RANGE, RANGE, 256, 256)


def _check_products(g_arrays, g_parent, o_app, ok_parents, what, parent_umag):
    o_parent = o_app["parent"]
    gi = {int(p): i for i, p in enumerate(g_parent)}
    oi = {int(p): i for i, p in enumerate(o_parent)}
    common = [p for p in oi if p in ok_parents]
    missing = [p for p in common if p not in gi]
    assert not missing, f"{what}: {len(missing)} products missing on the GPU"
    if not common:
        return 0
    g_idx = np.array([gi[p] for p in common])
    o_idx = np.array([oi[p] for p in common])
    umag = np.array([parent_umag(p) for p in common])
    for k in ("ux", "uy", "uz"):
        r = rel_close(g_arrays[k][g_idx], o_app[k][o_idx], RTOL, floor=np.maximum(umag, 1e-30))
        assert r <= 1.0, f"{what}.{k} {r:.3g} x tol"
    for k in ("w", "tau"):
        r = rel_close(g_arrays[k][g_idx], o_app[k][o_idx], RTOL)
        assert r <= 1.0, f"{what}.{k} {r:.3g} x tol"
    # products in ascending parent order (ordered append)
    assert np.all(np.diff(g_parent) > 0)
    return len(common)


@pytest.mark.parametrize("chi_mode", [Q.CHI_FP64, Q.CHI_COMP32])
def test_fp32_stepwise(ctx, tabs, chi_mode):
    (bw, qs), (obw, oqs) = tabs
    n = 1 << 16
    el, ph = QI.cone_population(seed=21, n=n)
    dt = 1e-16
    d_e = {k: torch.as_tensor(v).to("cuda", torch.float32) for k, v in el.items()}
    d_g = {k: torch.as_tensor(v).to("cuda", torch.float32) for k, v in ph.items()}
    d_e["tau"] = torch.empty(n, dtype=torch.float32, device="cuda")
    d_g["tau"] = torch.empty(n, dtype=torch.float32, device="cuda")
    pe, pg = Q.particles(d_e, Q.ELECTRON, 0), Q.particles(d_g, Q.PHOTON, n)
    Q.init_optical_depth(ctx, pe, 21)
    Q.init_optical_depth(ctx, pg, 21)
    bufs = [Q.AppendBuffer(n, torch.float32) for _ in range(3)]
    fe = torch.zeros(n, dtype=torch.uint8, device="cuda")
    fg = torch.zeros(n, dtype=torch.uint8, device="cuda")
    desc = Q.StepDesc([pe, pg], bw=bw, qs=qs, photons=bufs[0], electrons=bufs[1], positrons=bufs[2],
                      flags=[fe, fg], dt=dt, seed=21, chi_mode=chi_mode)
    total_flips = checked = 0
    for s in range(3):
        before = [{k: host(v) for k, v in d.items()} for d in (d_e, d_g)]
        for b in bufs:
            b.reset()
        desc.set_step(s)
        Q.step(ctx, desc)
        torch.cuda.synchronize()
        after = [{k: host(v) for k, v in d.items()} for d in (d_e, d_g)]
        gflags = [fe.cpu().numpy(), fg.cpu().numpy()]
        o_ph, o_el, o_po = O.Append(n), O.Append(n), O.Append(n)
        for si, (sp, idb) in enumerate(((O.ELECTRON, 0), (O.PHOTON, n))):
            op = O.Particles(before[si], sp, id_base=idb, tau=before[si]["tau"])
            # tau the oracle sees just before its event test, for the tie rule
            probe = O.Particles(before[si], sp, id_base=idb, tau=before[si]["tau"])
            O.evolve(obw if sp == O.PHOTON else oqs, probe, dt)
            of = np.zeros(n, dtype=np.uint8)
            if sp == O.PHOTON:
                O.step(obw, oqs, op, dt, 21, s, o_el, o_po, flags=of)
            else:
                O.step(obw, oqs, op, dt, 21, s, o_ph, flags=of)
            flip = gflags[si] != of
            assert np.all(np.abs(probe["tau"][flip]) < TIE), "event flip away from tau = 0"
            total_flips += int(flip.sum())
            ok = ~flip
            # momenta on the scale of |u| before the step (the parent's |u|)
            umag = np.sqrt(before[si]["ux"] ** 2 + before[si]["uy"] ** 2 + before[si]["uz"] ** 2)
            pmag = (lambda um, base: (lambda pid: um[pid - base]))(umag, idb)
            assert rel_close(after[si]["tau"][ok], op["tau"][ok], RTOL) <= 1.0, f"tau step {s}"
            for k in ("ux", "uy", "uz"):
                assert rel_close(after[si][k][ok], op[k][ok], RTOL, floor=np.maximum(umag[ok], 1e-30)) <= 1.0
            ok_parents = set((np.nonzero(ok)[0] + idb).tolist())
            if sp == O.PHOTON:
                g_el = {k: host(v) for k, v in bufs[1].a.items()}
                g_po = {k: host(v) for k, v in bufs[2].a.items()}
                ne = int(bufs[1].count.item())
                checked += _check_products({k: v[:ne] for k, v in g_el.items()}, bufs[1].parent[:ne].cpu().numpy(),
                                           o_el, ok_parents, f"electrons step {s}", pmag)
                _check_products({k: v[:ne] for k, v in g_po.items()}, bufs[2].parent[:ne].cpu().numpy(),
                                o_po, ok_parents, f"positrons step {s}", pmag)
            else:
                g_ph = {k: host(v) for k, v in bufs[0].a.items()}
                npn = int(bufs[0].count.item())
                checked += _check_products({k: v[:npn] for k, v in g_ph.items()}, bufs[0].parent[:npn].cpu().numpy(),
                                           o_ph, ok_parents, f"photons step {s}", pmag)
    assert checked > 1000
    assert total_flips <= 10


@pytest.mark.parametrize("mode,tol", [(Q.CHI_FP64, 1e-7), (Q.CHI_COMP32, 1e-6), (Q.CHI_FP32, 1e-3)])
def test_fp32_chi_modes(ctx, mode, tol):
    """chi on FP32 data (counter-propagating cone: no catastrophic
    cancellation) against the oracle on the same (exactly widened) inputs."""
    for photon in (False, True):
        pop = QI.plane_wave_cone(20000, 31, photon, stream=int(photon), dtype=np.float32)
        d = {k: torch.as_tensor(v).cuda() for k, v in pop.items()}
        d["tau"] = torch.zeros(20000, dtype=torch.float32, device="cuda")
        p = Q.particles(d, Q.PHOTON if photon else Q.ELECTRON)
        out = torch.empty(20000, dtype=torch.float32, device="cuda")
        (Q.chi_photon if photon else Q.chi_lepton)(ctx, p, out, chi_mode=mode)
        torch.cuda.synchronize()
        ref = O.chi_array({k: v.astype(np.float64) for k, v in pop.items()}, photon)
        assert rel_close(host(out), ref, tol, floor=1e-30) <= 1.0


def test_comp32_beats_fp32_on_copropagating(ctx):
    """Co-propagating particles: sqrt(.) cancels catastrophically; the
    compensated FP32 chi stays close to the binary128 value of the printed
    formula on the same inputs while plain FP32 does not."""
    pop = QI.plane_wave_cone(2000, 41, False, axis_sign=1.0, half_angle=0.0, gamma_range=(1e2, 1e3),
                             dtype=np.float32)
    d = {k: torch.as_tensor(v).cuda() for k, v in pop.items()}
    d["tau"] = torch.zeros(2000, dtype=torch.float32, device="cuda")
    p = Q.particles(d, Q.ELECTRON)
    outs = {}
    for mode in (Q.CHI_FP64, Q.CHI_COMP32, Q.CHI_FP32):
        out = torch.empty(2000, dtype=torch.float32, device="cuda")
        Q.chi_lepton(ctx, p, out, chi_mode=mode)
        outs[mode] = host(out)
    torch.cuda.synchronize()
    keys = ("ux", "uy", "uz", "ex", "ey", "ez", "bx", "by", "bz")
    ref = np.array([O.chi_literal_q(*[float(pop[k][i]) for k in keys]) for i in range(2000)])
    err = {m: np.median(np.abs(outs[m] / ref - 1)) for m in outs}
    assert err[Q.CHI_COMP32] < 1e-4
    assert err[Q.CHI_FP64] < 1e-4
    assert err[Q.CHI_FP32] > 10 * err[Q.CHI_COMP32]


@pytest.mark.parametrize("every", [1, 3, 97])
def test_fp32_standalone_generate(ctx, tabs, every):
    """The FP32 production calls (pair generation; photon emission with the
    parent's momentum update, Sec. 3.1, 3.2) against the oracle on the same
    FP32 inputs, over a count that leaves a partial last chunk: flags on
    every particle, on one in three and on one in 97 (most slices of 64
    then hold no or one flagged particle).  Counts and parent ids exact;
    momenta within 1e-5 of the parent's |u|, optical depths and weights
    within 1e-5 relative."""
    (bw, qs), (obw, oqs) = tabs
    n = 9037
    for photon in (False, True):
        pop = QI.plane_wave_counter(n, 11, photon, stream=int(photon))
        pop = {k: np.asarray(v, dtype=np.float32).astype(np.float64) for k, v in pop.items()}
        sp = O.PHOTON if photon else O.ELECTRON
        flags = (np.arange(n) % every == 0).astype(np.uint8)
        d = {k: torch.as_tensor(v).to("cuda", torch.float32) for k, v in pop.items()}
        d["tau"] = torch.ones(n, dtype=torch.float32, device="cuda")
        p = Q.particles(d, sp, 777)
        op = O.Particles(pop, sp, id_base=777, tau=np.ones(n))
        fl = torch.as_tensor(flags).cuda()
        a1, a2 = Q.AppendBuffer(n, torch.float32), Q.AppendBuffer(n, torch.float32)
        o1, o2 = O.Append(n), O.Append(n)
        if photon:
            Q.generate_pairs(ctx, bw, p, fl, 10, 42, a1, a2)
            O.generate(obw, oqs, op, flags, 10, 42, o1, o2)
        else:
            Q.generate_photon_and_update_momentum(ctx, qs, p, fl, 10, 42, a1)
            O.generate(obw, oqs, op, flags, 10, 42, o1)
        torch.cuda.synchronize()
        assert o1.count == int(flags.sum())
        umag = np.sqrt(pop["ux"] ** 2 + pop["uy"] ** 2 + pop["uz"] ** 2)
        pu = umag[o1["parent"][: o1.count] - 777]
        compare_append(a1, o1, RTOL, "generate a1", parent_umag=pu)
        if photon:
            compare_append(a2, o2, RTOL, "generate a2", parent_umag=pu)
        assert rel_close(host(d["tau"]), op["tau"], RTOL) <= 1.0
        for k in ("ux", "uy", "uz"):
            assert rel_close(host(d[k]), op[k], RTOL, floor=np.maximum(umag, 1e-30)) <= 1.0
