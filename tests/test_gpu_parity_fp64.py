"""FP64 HIP path against the FP64 oracle on the same seeded inputs.

Bar: event flags, product counts and parent indices bit-exact; momenta and
optical depths within 1e-12 relative (scale max(|value|, 1) for tau and the
parent's |u| for momenta).  Each side generates its own tables (independent
quadratures that agree to ~1e-14)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_2110_00256_amd as Q  # noqa: E402
import qed_inputs as QI  # noqa: E402
from oracle import oracle as O  # noqa: E402
from tests.gpu_util import compare_append, dev_pop, host, lib_tables, oracle_tables, rel_close  # noqa: E402

RTOL = 1e-12
C1_BW = (1e-3, 1e2)
C1_QS = (1e-3, 1e2)


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return Q.Context(0)


@pytest.fixture(scope="module")
def tabs():
    return lib_tables(C1_BW, C1_QS, 64, 64), oracle_tables(C1_BW, C1_QS, 64, 64)


def _fields(pop):
    return {k: pop[k] for k in QI.FIELDS}


def test_chi_matches_oracle(ctx):
    for pop, photon in ((QI.plane_wave_counter(3000, 4, False), False),
                        (QI.plane_wave_counter(3000, 4, True, stream=1), True),
                        (QI.plane_wave_cone(3000, 5, False), False),
                        (QI.plane_wave_cone(3000, 5, True, stream=1), True),
                        (QI.paper_uniform(3000, 6), False)):
        d = dev_pop(pop, torch.float64)
        sp = Q.PHOTON if photon else Q.ELECTRON
        p = Q.particles(d, sp)
        out = torch.empty_like(d["ux"])
        (Q.chi_photon if photon else Q.chi_lepton)(ctx, p, out)
        torch.cuda.synchronize()
        ref = O.chi_array(pop, photon)
        assert rel_close(host(out), ref, 1e-14, floor=1e-300) <= 1.0


def test_init_optical_depth_matches_oracle(ctx):
    pop = QI.plane_wave_counter(5000, 7, False)
    d = dev_pop(pop, torch.float64)
    p = Q.particles(d, Q.POSITRON, id_base=123456789)
    Q.init_optical_depth(ctx, p, seed=99)
    op = O.Particles(pop, O.POSITRON, id_base=123456789)
    O.init_optical_depth(op, 99)
    torch.cuda.synchronize()
    assert rel_close(host(d["tau"]), op["tau"], 1e-15) <= 1.0


def test_evolve_matches_oracle(ctx, tabs):
    (bw, qs), (obw, oqs) = tabs
    for photon in (False, True):
        pop = QI.plane_wave_counter(20000, 8, photon, stream=int(photon))
        sp = O.PHOTON if photon else O.ELECTRON
        op = O.Particles(pop, sp)
        O.init_optical_depth(op, 3)
        d = dev_pop(pop, torch.float64, tau=op["tau"])
        p = Q.particles(d, sp)
        fl = torch.zeros(len(pop["ux"]), dtype=torch.uint8, device="cuda")
        Q.evolve_optical_depth(ctx, bw if photon else qs, p, 1e-16, flags=fl)
        ofl = np.zeros(op.n, dtype=np.uint8)
        O.evolve(obw if photon else oqs, op, 1e-16, ofl)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(fl.cpu().numpy(), ofl)
        assert ofl.sum() > 0
        assert rel_close(host(d["tau"]), op["tau"], RTOL) <= 1.0


def _run_steps(ctx, tabs, n_e, n_g, steps, seed=1, dt=1e-16, threshold=0.0, cap=None, tiles=None,
               check_each_step=True, chi_qed_min=0.0):
    """Run the fused step on GPU and the oracle side by side; compare."""
    (bw, qs), (obw, oqs) = tabs
    el, ph = QI.parity_population(seed=seed, n=max(n_e, n_g))
    el = {k: v[:n_e] for k, v in el.items()}
    ph = {k: v[:n_g] for k, v in ph.items()}
    oe, og = O.Particles(el, O.ELECTRON, id_base=0), O.Particles(ph, O.PHOTON, id_base=1 << 40)
    O.init_optical_depth(oe, seed)
    O.init_optical_depth(og, seed)
    de, dg = dev_pop(el, torch.float64), dev_pop(ph, torch.float64)
    pe, pg = Q.particles(de, Q.ELECTRON, 0), Q.particles(dg, Q.PHOTON, 1 << 40)
    Q.init_optical_depth(ctx, pe, seed)
    Q.init_optical_depth(ctx, pg, seed)
    torch.cuda.synchronize()
    assert rel_close(host(de["tau"]), oe["tau"], 1e-15) <= 1.0
    # the GPU path continues from the oracle's initial tau bit for bit
    de["tau"].copy_(torch.as_tensor(oe["tau"]))
    dg["tau"].copy_(torch.as_tensor(og["tau"]))
    capacity = cap if cap is not None else steps * max(n_e, n_g, 1)
    ph_b = Q.AppendBuffer(capacity, torch.float64)
    el_b = Q.AppendBuffer(capacity, torch.float64)
    po_b = Q.AppendBuffer(capacity, torch.float64)
    o_ph, o_el, o_po = O.Append(capacity), O.Append(capacity), O.Append(capacity)
    fe = torch.zeros(max(n_e, 1), dtype=torch.uint8, device="cuda")
    fg = torch.zeros(max(n_g, 1), dtype=torch.uint8, device="cuda")
    stats = torch.zeros(Q.STATS_LEN, dtype=torch.int64, device="cuda")
    desc = Q.StepDesc([pe, pg], bw=bw, qs=qs, photons=ph_b, electrons=el_b, positrons=po_b,
                      flags=[fe, fg], stats=stats, dt=dt, seed=seed, photon_min_energy=threshold, tiles=tiles,
                      chi_qed_min=chi_qed_min)
    total_events = 0
    pu = {"ph": [], "el": [], "po": []}   # parent |u| of every product, in slot order
    # A particle's momentum is compared on the scale of the largest |u| it has
    # had: an emission that leaves |u'| << |u| carries the rounding error of
    # the subtraction u - p_gamma, which is set by |u|, into later steps.
    uscale = [np.sqrt(o["ux"] ** 2 + o["uy"] ** 2 + o["uz"] ** 2) if o.n else None for o in (oe, og)]
    for s in range(steps):
        u_before = [np.sqrt(o["ux"] ** 2 + o["uy"] ** 2 + o["uz"] ** 2) if o.n else None for o in (oe, og)]
        uscale = [None if a is None else np.maximum(a, b) for a, b in zip(uscale, u_before)]
        desc.set_step(s)
        Q.step(ctx, desc)
        ofe = np.zeros(max(n_e, 1), dtype=np.uint8)
        ofg = np.zeros(max(n_g, 1), dtype=np.uint8)
        if tiles is None:
            total_events += O.step(obw, oqs, oe, dt, seed, s, o_ph, photon_min_energy=threshold, flags=ofe[:n_e],
                                   chi_qed_min=chi_qed_min)
            total_events += O.step(obw, oqs, og, dt, seed, s, o_el, o_po, flags=ofg[:n_g], chi_qed_min=chi_qed_min)
        else:
            total_events += _oracle_tiles(obw, oqs, [oe, og], tiles, dt, seed, s, o_ph, o_el, o_po, threshold,
                                          [ofe, ofg])
        torch.cuda.synchronize()
        for key, app, o, ub in (("ph", o_ph, oe, u_before[0]), ("el", o_el, og, u_before[1]),
                                ("po", o_po, og, u_before[1])):
            par = app.parent[len(pu[key]):min(app.count, app._c.capacity)]
            pu[key].extend((ub[par - o.id_base]).tolist() if len(par) else [])
        if check_each_step or s == steps - 1:
            if n_e:
                np.testing.assert_array_equal(fe[:n_e].cpu().numpy(), ofe[:n_e], err_msg=f"electron flags step {s}")
            if n_g:
                np.testing.assert_array_equal(fg[:n_g].cpu().numpy(), ofg[:n_g], err_msg=f"photon flags step {s}")
            for d, o, umag in ((de, oe, uscale[0]), (dg, og, uscale[1])):
                if o.n == 0:
                    continue
                assert rel_close(host(d["tau"]), o["tau"], RTOL) <= 1.0, f"tau step {s}"
                for k in ("ux", "uy", "uz"):
                    assert rel_close(host(d[k]), o[k], RTOL, floor=np.maximum(umag, 1e-300)) <= 1.0
            compare_append(ph_b, o_ph, RTOL, f"photons step {s}", pu["ph"])
            compare_append(el_b, o_el, RTOL, f"electrons step {s}", pu["el"])
            compare_append(po_b, o_po, RTOL, f"positrons step {s}", pu["po"])
    st = stats.cpu().numpy()
    assert st[Q.STAT_SCAN_TIMEOUT] == 0
    assert st[Q.STAT_UPDATES] == steps * (n_e + n_g)
    assert st[Q.STAT_QS_EVENTS] + st[Q.STAT_BW_EVENTS] == total_events
    return total_events, (ph_b, el_b, po_b), (o_ph, o_el, o_po)


def _oracle_tiles(obw, oqs, osets, tiles, dt, seed, s, o_ph, o_el, o_po, threshold, oflags):
    """Oracle over tiles: leptons' tiles first then photons' tiles, each in
    tile order, every tile an index range of its set (ids preserved)."""
    ev = 0
    for stream in (0, 1):
        for (si, b, e) in np.asarray(tiles).reshape(-1, 3):
            o = osets[si]
            if (o.species == O.PHOTON) != (stream == 1) or e <= b:
                continue
            sub = {k: o[k][b:e] for k in O.Particles.KEYS if k != "tau"}
            t = O.Particles(sub, o.species, id_base=o.id_base + b, tau=o["tau"][b:e])
            f = np.zeros(e - b, dtype=np.uint8)
            if stream == 0:
                ev += O.step(obw, oqs, t, dt, seed, s, o_ph, photon_min_energy=threshold, flags=f)
            else:
                ev += O.step(obw, oqs, t, dt, seed, s, o_el, o_po, flags=f)
            for k in O.Particles.KEYS:
                o[k][b:e] = t[k]
            oflags[si][b:e] = f
    return ev


def test_parity_workload_ten_steps(ctx, tabs):
    """The parity workload: 2^16 electrons + 2^16 photons, 10 steps."""
    ev, _, _ = _run_steps(ctx, tabs, 1 << 16, 1 << 16, 10)
    assert ev > 1000


@pytest.mark.parametrize("n_e,n_g", [(1, 0), (0, 1), (4095, 4097), (12289, 300), (0, 0)])
def test_ragged_and_empty(ctx, tabs, n_e, n_g):
    _run_steps(ctx, tabs, n_e, n_g, 3, seed=3)


def test_tiles_follow_tile_order(ctx, tabs):
    n = 20000
    # electrons split into 5 tiles listed out of index order, photons into 3
    tiles = [(0, 12000, 20000), (0, 0, 5000), (1, 9000, 20000), (0, 5000, 7000), (1, 0, 9000),
             (0, 7000, 12000)]
    _run_steps(ctx, tabs, n, n, 2, seed=4, tiles=tiles)


def _random_layout(rng, n_e, n_g, pieces=5):
    """Each set cut at random points into `pieces` tiles, all tiles shuffled."""
    tl = []
    for si, n in ((0, n_e), (1, n_g)):
        cuts = sorted(rng.choice(np.arange(1, n), pieces - 1, replace=False).tolist())
        edges = [0, *cuts, n]
        tl += [(si, int(a), int(b)) for a, b in zip(edges[:-1], edges[1:])]
    order = rng.permutation(len(tl))
    return [tl[i] for i in order]


def test_tile_layout_changes_every_step_without_sync(ctx, tabs):
    """A new tile list every step (cut points and tile order, hence product
    order, change), the steps queued back to back with no host
    synchronisation between them: the tile list reaches the device through
    pinned double-buffered staging and the chunk table is built there.  The
    products of all steps, the final state and the last flags match the
    oracle run over the same tile lists."""
    (bw, qs), (obw, oqs) = tabs
    n, steps, seed, dt = 20000, 6, 21, 1e-16
    rng = np.random.default_rng(5)
    layouts = [_random_layout(rng, n, n) for _ in range(steps)]
    el, ph = QI.parity_population(seed=seed, n=n)
    oe, og = O.Particles(el, O.ELECTRON, id_base=0), O.Particles(ph, O.PHOTON, id_base=1 << 40)
    O.init_optical_depth(oe, seed)
    O.init_optical_depth(og, seed)
    de, dg = dev_pop(el, torch.float64, tau=oe["tau"]), dev_pop(ph, torch.float64, tau=og["tau"])
    pe, pg = Q.particles(de, Q.ELECTRON, 0), Q.particles(dg, Q.PHOTON, 1 << 40)
    cap = steps * n
    bufs = [Q.AppendBuffer(cap, torch.float64) for _ in range(3)]
    orc = [O.Append(cap) for _ in range(3)]
    fe = torch.zeros(n, dtype=torch.uint8, device="cuda")
    fg = torch.zeros(n, dtype=torch.uint8, device="cuda")
    u0 = [np.sqrt(o["ux"] ** 2 + o["uy"] ** 2 + o["uz"] ** 2) for o in (oe, og)]
    for s in range(steps):
        desc = Q.StepDesc([pe, pg], bw=bw, qs=qs, photons=bufs[0], electrons=bufs[1], positrons=bufs[2],
                          flags=[fe, fg], tiles=layouts[s], dt=dt, seed=seed, step=s)
        Q.step(ctx, desc)
    ofe, ofg = np.zeros(n, dtype=np.uint8), np.zeros(n, dtype=np.uint8)
    for s in range(steps):
        _oracle_tiles(obw, oqs, [oe, og], layouts[s], dt, seed, s, orc[0], orc[1], orc[2], 0.0, [ofe, ofg])
    torch.cuda.synchronize()
    np.testing.assert_array_equal(fe.cpu().numpy(), ofe)
    np.testing.assert_array_equal(fg.cpu().numpy(), ofg)
    assert orc[0].count > 1000 and orc[1].count > 10
    for b, o, what, os_ in zip(bufs, orc, ("photons", "electrons", "positrons"), (oe, og, og)):
        par = o.parent[:o.count] - os_.id_base
        compare_append(b, o, RTOL, what, (u0[0] if os_ is oe else u0[1])[par])
    for d, o, um in ((de, oe, u0[0]), (dg, og, u0[1])):
        fin = np.isfinite(o["tau"])
        assert np.array_equal(np.isinf(host(d["tau"])), ~fin)
        assert rel_close(host(d["tau"])[fin], o["tau"][fin], RTOL) <= 1.0
        for k in ("ux", "uy", "uz"):
            assert rel_close(host(d[k]), o[k], RTOL, floor=np.maximum(um, 1e-300)) <= 1.0


def test_nonfinite_inputs_are_counted(ctx, tabs):
    """NaN or infinite momenta and fields give a non-finite chi, and a NaN or
    -inf optical depth a non-finite update: each such particle is counted in
    the NONFINITE statistic.  A decayed photon (tau = +inf) is not."""
    (bw, qs), _ = tabs
    n, seed = 5000, 3
    el, ph = QI.parity_population(seed=seed, n=n)
    el["ux"][5] = np.nan
    el["ey"][7] = np.inf
    el["bz"][8] = -np.inf
    ph["bz"][11] = np.nan
    te = np.full(n, 0.5)
    tg = np.full(n, 0.5)
    te[9] = np.nan
    te[10] = -np.inf
    tg[20] = np.inf            # a photon that decayed earlier
    de, dg = dev_pop(el, torch.float64, tau=te), dev_pop(ph, torch.float64, tau=tg)
    pe, pg = Q.particles(de, Q.ELECTRON, 0), Q.particles(dg, Q.PHOTON, 1 << 40)
    bufs = [Q.AppendBuffer(2 * n, torch.float64) for _ in range(3)]
    stats = torch.zeros(Q.STATS_LEN, dtype=torch.int64, device="cuda")
    desc = Q.StepDesc([pe, pg], bw=bw, qs=qs, photons=bufs[0], electrons=bufs[1], positrons=bufs[2],
                      stats=stats, dt=1e-16, seed=seed)
    Q.step(ctx, desc)
    st = stats.cpu().numpy()
    assert st[Q.STAT_NONFINITE] == 6, st
    assert st[Q.STAT_UPDATES] == 2 * n
    assert st[Q.STAT_SCAN_TIMEOUT] == 0
    assert np.isinf(host(dg["tau"])[20])


def test_tiles_with_odd_boundaries(ctx, tabs):
    """Tiles starting at odd indices (the streaming phase falls back from
    16-byte loads to one element per load) and ragged tile ends."""
    n = 20000
    tiles = [(0, 1, 7001), (1, 3, 20000), (0, 7001, 20000), (0, 0, 1), (1, 0, 3)]
    _run_steps(ctx, tabs, n, n, 2, seed=14, tiles=tiles)


def test_unaligned_arrays(ctx, tabs):
    """Particle arrays that are views one element into their allocation
    (not 16-byte aligned): same results as the oracle."""
    (bw, qs), (obw, oqs) = tabs
    n, seed = 9001, 15
    el, _ = QI.parity_population(seed=seed, n=n)
    oe = O.Particles(el, O.ELECTRON, id_base=0)
    O.init_optical_depth(oe, seed)
    full = {k: torch.zeros(n + 1, dtype=torch.float64, device="cuda") for k in list(el) + ["tau"]}
    d = {k: v[1:] for k, v in full.items()}
    for k in el:
        d[k].copy_(torch.as_tensor(el[k]))
    d["tau"].copy_(torch.as_tensor(oe["tau"]))
    pe = Q.particles(d, Q.ELECTRON, 0)
    ph_b = Q.AppendBuffer(n, torch.float64)
    desc = Q.StepDesc([pe], bw=bw, qs=qs, photons=ph_b, electrons=Q.AppendBuffer(0, torch.float64),
                      positrons=Q.AppendBuffer(0, torch.float64), dt=1e-16, seed=seed)
    o_ph = O.Append(n)
    u0 = np.sqrt(oe["ux"] ** 2 + oe["uy"] ** 2 + oe["uz"] ** 2)
    Q.step(ctx, desc)
    O.step(obw, oqs, oe, 1e-16, seed, 0, o_ph)
    torch.cuda.synchronize()
    assert o_ph.count > 100
    compare_append(ph_b, o_ph, RTOL, "photons", u0[o_ph.parent[:o_ph.count]])
    assert rel_close(host(d["tau"]), oe["tau"], RTOL) <= 1.0
    for k in ("ux", "uy", "uz"):
        assert rel_close(host(d[k]), oe[k], RTOL, floor=np.maximum(u0, 1e-300)) <= 1.0


def test_photon_threshold(ctx, tabs):
    ev, (ph_b, _, _), (o_ph, _, _) = _run_steps(ctx, tabs, 30000, 10, 3, seed=5, threshold=2.0)
    assert 0 < o_ph.count < ev


def test_qed_threshold_classical_regime(ctx, tabs):
    """WarpX's minimum quantum parameter (Sec. 6): below chi_qed_min photons
    keep their optical depth and leptons radiate classically; about half of
    the parity workload's particles are below 0.5."""
    ev_on, _, _ = _run_steps(ctx, tabs, 20000, 20000, 4, seed=12, chi_qed_min=0.5)
    ev_off, _, _ = _run_steps(ctx, tabs, 20000, 20000, 4, seed=12)
    assert 0 < ev_on < ev_off


def test_capacity_overflow_counts_and_prefix(ctx, tabs):
    ev, (ph_b, el_b, po_b), (o_ph, _, _) = _run_steps(ctx, tabs, 20000, 20000, 2, seed=6, cap=50)
    assert ph_b.read_count() == o_ph.count > ph_b.capacity == 50


def test_bit_identical_rerun(ctx, tabs):
    (bw, qs), _ = tabs
    el, ph = QI.parity_population(seed=9, n=30000)
    outs = []
    for _ in range(2):
        de, dg = dev_pop(el, torch.float64), dev_pop(ph, torch.float64)
        pe, pg = Q.particles(de, Q.ELECTRON, 0), Q.particles(dg, Q.PHOTON, 1 << 40)
        Q.init_optical_depth(ctx, pe, 9)
        Q.init_optical_depth(ctx, pg, 9)
        bufs = [Q.AppendBuffer(200000, torch.float64) for _ in range(3)]
        desc = Q.StepDesc([pe, pg], bw=bw, qs=qs, photons=bufs[0], electrons=bufs[1], positrons=bufs[2],
                          dt=1e-16, seed=9)
        for s in range(4):
            desc.set_step(s)
            Q.step(ctx, desc)
        torch.cuda.synchronize()
        outs.append([t.cpu().numpy().copy() for t in list(de.values()) + list(dg.values())] +
                    [b.a[k].cpu().numpy().copy() for b in bufs for k in b.a] + [b.parent.cpu().numpy() for b in bufs])
    for a, b in zip(*outs):
        np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("every", [3, 1, 2])
def test_standalone_generate_matches_oracle(ctx, tabs, every):
    """Flagged particles produce: one in three (a chunk's optical depths all
    fit the free LDS slots but the last), all (none fit: every event draws
    again in the write phase) and one in two (half fit)."""
    (bw, qs), (obw, oqs) = tabs
    n = 9000
    for photon in (False, True):
        pop = QI.plane_wave_counter(n, 10, photon, stream=int(photon))
        sp = O.PHOTON if photon else O.ELECTRON
        flags = (np.arange(n) % every == 0).astype(np.uint8)
        op = O.Particles(pop, sp, id_base=777)
        O.init_optical_depth(op, 10)
        d = dev_pop(pop, torch.float64, tau=op["tau"])
        p = Q.particles(d, sp, 777)
        fl = torch.as_tensor(flags).cuda()
        a1, a2 = Q.AppendBuffer(n, torch.float64), Q.AppendBuffer(n, torch.float64)
        o1, o2 = O.Append(n), O.Append(n)
        if photon:
            Q.generate_pairs(ctx, bw, p, fl, 10, 42, a1, a2)
            O.generate(obw, oqs, op, flags, 10, 42, o1, o2)
        else:
            Q.generate_photon_and_update_momentum(ctx, qs, p, fl, 10, 42, a1)
            O.generate(obw, oqs, op, flags, 10, 42, o1)
        torch.cuda.synchronize()
        compare_append(a1, o1, RTOL, "generate a1")
        if photon:
            compare_append(a2, o2, RTOL, "generate a2")
        assert rel_close(host(d["tau"]), op["tau"], RTOL) <= 1.0
        for k in ("ux", "uy", "uz"):
            assert rel_close(host(d[k]), op[k], RTOL, floor=1.0) <= 1.0


@pytest.mark.parametrize("every", [1, 3])
def test_standalone_photon_emission_with_threshold(ctx, tabs, every):
    """Photon emission with a photon energy threshold (Sec. 3.2): every
    flagged lepton recoils and redraws its optical depth, only photons at or
    above the threshold are appended, in parent order, counts and parents
    exact against the oracle."""
    (bw, qs), (obw, oqs) = tabs
    n = 9000
    pop = QI.plane_wave_counter(n, 12, False, stream=0)
    flags = (np.arange(n) % every == 0).astype(np.uint8)
    op = O.Particles(pop, O.ELECTRON, id_base=91)
    O.init_optical_depth(op, 12)
    d = dev_pop(pop, torch.float64, tau=op["tau"])
    p = Q.particles(d, O.ELECTRON, 91)
    fl = torch.as_tensor(flags).cuda()
    a1, o1 = Q.AppendBuffer(n, torch.float64), O.Append(n)
    emin = 30.0
    Q.generate_photon_and_update_momentum(ctx, qs, p, fl, 12, 5, a1, photon_min_energy=emin)
    O.generate(obw, oqs, op, flags, 12, 5, o1, photon_min_energy=emin)
    torch.cuda.synchronize()
    assert 0 < o1.count < int(flags.sum())
    compare_append(a1, o1, RTOL, "thresholded photons")
    assert rel_close(host(d["tau"]), op["tau"], RTOL) <= 1.0
    for k in ("ux", "uy", "uz"):
        assert rel_close(host(d[k]), op[k], RTOL, floor=1.0) <= 1.0


def test_table_rate_and_sample_match_oracle(ctx, tabs):
    """The runtime rate and inverse-CDF sampling functions in isolation, over
    chi inside and outside the table range and u over (0, 1)."""
    (bw, qs), (obw, oqs) = tabs
    rng = np.random.default_rng(5)
    n = 200000
    chi = np.exp(rng.uniform(np.log(1e-5), np.log(1e4), n))
    gam = np.exp(rng.uniform(0, np.log(1e5), n))
    u = np.array([O.u01(int(w)) for w in rng.integers(0, 2**63, n, dtype=np.uint64) * 2 + 1])
    dchi, dgam, du = (torch.as_tensor(x).cuda() for x in (chi, gam, u))
    for t, ot in ((bw, obw), (qs, oqs)):
        out = torch.empty_like(dchi)
        Q.table_rate(t, dchi, dgam, out)
        torch.cuda.synchronize()
        # rates below 1 /s are zero for any time step; their relative rounding
        # grows with |ln T| near the exp underflow
        assert rel_close(host(out), ot.rate_n(chi, gam), 1e-13, floor=1.0) <= 1.0
        sel = torch.zeros(n, dtype=torch.uint8, device="cuda")
        Q.table_sample(t, dchi, du, out, sel)
        torch.cuda.synchronize()
        ref = ot.sample_n(chi, u)
        if ot.proc == O.BW:
            ref, esel = ref
            np.testing.assert_array_equal(sel.cpu().numpy().astype(bool), esel)
        err = np.abs(host(out) - ref)
        i = int(np.argmax(err))
        print(f"proc {ot.proc}: max |sample - oracle| = {err[i]:.3e} at chi={chi[i]!r} u={u[i]!r} "
              f"gpu={host(out)[i]!r} oracle={ref[i]!r}", flush=True)
        assert err[i] < (1e-13 if ot.proc == O.BW else 1e-12)
