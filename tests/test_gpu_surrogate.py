"""Learned inverse-CDF surrogate: forward and gradients of the BF16-MFMA
kernels against the oracle's FP64 MLP (with the same BF16 operand rounding
emulated), GPU training, KS distance of the sampled spectra against the
table, domain fallback, the per-batch probe, and the surrogate inside the
fused step."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_2110_00256_amd as Q  # noqa: E402
import qed_inputs as QI  # noqa: E402
from oracle import oracle as O  # noqa: E402

RANGE = (1e-4, 1e4)


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return Q.Context(0)


@pytest.fixture(scope="module")
def tables():
    return (Q.Table.generate(Q.BW, RANGE[0], RANGE[1], 97, 256).to_device(),
            Q.Table.generate(Q.QS, RANGE[0], RANGE[1], 97, 256).to_device())


def _random_params(seed):
    rng = np.random.default_rng(seed)
    p = np.zeros(Q.SURR_NPARAM)
    p[:128] = rng.uniform(-1.5, 1.5, 128)
    p[128:192] = rng.uniform(-1.5, 1.5, 64)
    p[192:4288] = rng.uniform(-1, 1, 4096) * np.sqrt(6 / 128)
    p[4288:4352] = rng.uniform(-0.1, 0.1, 64)
    p[4352:4416] = rng.uniform(-1, 1, 64) * np.sqrt(6 / 65)
    p[4416] = 0.3
    return p.astype(np.float32)


def test_forward_matches_oracle(tables):
    bw, qs = tables
    p = _random_params(1)
    s = Q.Surrogate.from_host(qs, Q.Surrogate.cfg(Q.QS, 1e-3, 1e3), p)
    rng = np.random.default_rng(2)
    x = rng.uniform(-1, 1, size=(5000, 2)).astype(np.float32)
    dx = torch.as_tensor(x).cuda().contiguous()
    y = torch.empty(5000, dtype=torch.float32, device="cuda")
    s.forward(dx, y)
    torch.cuda.synchronize()
    g = y.cpu().numpy().astype(np.float64)
    ref_q = O.mlp_forward(p.astype(np.float64), x.astype(np.float64), bf16=True)
    ref = O.mlp_forward(p.astype(np.float64), x.astype(np.float64), bf16=False)
    scale = np.max(np.abs(ref))
    err_q = np.abs(g - ref_q) / scale
    print(f"forward vs oracle(bf16 emulated): median {np.median(err_q):.2e} max {err_q.max():.2e}; "
          f"vs FP64: max {np.max(np.abs(g - ref)) / scale:.2e}")
    assert np.median(err_q) < 1e-5 and err_q.max() < 5e-3
    assert np.max(np.abs(g - ref)) / scale < 5e-2


def test_gradient_matches_oracle(tables):
    _, qs = tables
    p = _random_params(3)
    s = Q.Surrogate.from_host(qs, Q.Surrogate.cfg(Q.QS, 1e-3, 1e3), p)
    rng = np.random.default_rng(4)
    n = 4096
    x = rng.uniform(-1, 1, size=(n, 2)).astype(np.float32)
    t = rng.normal(size=n).astype(np.float32)
    grad = torch.zeros(Q.SURR_NPARAM, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    s.grad(torch.as_tensor(x).cuda(), torch.as_tensor(t).cuda(), grad, loss)
    torch.cuda.synchronize()
    g = grad.cpu().numpy().astype(np.float64)
    lq, gq = O.mlp_grad(p.astype(np.float64), x.astype(np.float64), t.astype(np.float64), bf16=True)
    l0, g0 = O.mlp_grad(p.astype(np.float64), x.astype(np.float64), t.astype(np.float64), bf16=False)
    assert abs(loss.item() - lq) < 1e-4 * abs(lq)
    # Element by element against the oracle with the kernel's BF16 operand
    # rounding emulated.  What remains is FP32 arithmetic: sums of n terms in
    # fixed order (relative error ~ sqrt(n) 2^-24 of the sum of |terms|), the
    # hardware exp and reciprocal of SiLU, and the rare hidden activation
    # whose BF16 rounding the FP32 rounding flips.  Entries that cancel to
    # near zero are measured against 1e-3 of the group's largest entry.
    for name, sl in (("W1", slice(0, 128)), ("b1", slice(128, 192)), ("W2", slice(192, 4288)),
                     ("b2", slice(4288, 4352)), ("W3", slice(4352, 4416)), ("b3", slice(4416, 4417))):
        ref = gq[sl]
        rel = np.abs(g[sl] - ref) / np.maximum(np.abs(ref), 1e-3 * np.max(np.abs(ref)))
        rel_0 = np.linalg.norm(g[sl] - g0[sl]) / np.linalg.norm(g0[sl])
        print(f"grad {name}: per element vs bf16-emulated oracle max {rel.max():.2e} median {np.median(rel):.2e}; "
              f"norm vs FP64 oracle {rel_0:.2e}")
        assert rel.max() < 1e-3, name
        assert np.median(rel) < 1e-5, name
        assert rel_0 < 5e-2, name


def _ks_paired(a, b):
    """Exact two-sample Kolmogorov-Smirnov distance sup_x |ECDF_a - ECDF_b|
    of two samples of equal size (here drawn with the same uniforms), taken
    over every value either sample holds, tails included."""
    sa, sb = np.sort(a), np.sort(b)
    vals = np.union1d(sa, sb)
    d = np.abs(np.searchsorted(sa, vals, "right") - np.searchsorted(sb, vals, "right"))
    return float(d.max() / len(a))


@pytest.fixture(scope="module")
def tables512():
    """The 512 x 512 tables the surrogate is fitted to (chi over [1e-4, 1e4])."""
    return (Q.Table.generate(Q.BW, RANGE[0], RANGE[1], 512, 512).to_device(),
            Q.Table.generate(Q.QS, RANGE[0], RANGE[1], 512, 512).to_device())


KS_GATE = 1e-3      # spectrum KS distance the surrogate path must meet
KS_BUDGET = 8e-4    # per-band validation budget (the gate less a margin for chi between validation points)


@pytest.fixture(scope="module")
def trained(ctx, tables512):
    """Both surrogates trained on 2^24 samples, 40000 Adam steps of 16384,
    then validated band by band against the table."""
    out = {}
    for proc in (Q.BW, Q.QS):
        table = tables512[0] if proc == Q.BW else tables512[1]
        cfg = Q.Surrogate.cfg(proc, 1e-3, 1e3, n_samples=1 << 24, batch=16384, steps=40000, lr=3e-3,
                              probe_tol=1.0, tail_permille=500, ks_budget=KS_BUDGET)
        out[proc] = Q.Surrogate.train(ctx, table, cfg)
    return out


CHI_GRID = (1e-3, 3e-3, 1e-2, 3e-2, 0.1, 0.3, 1.0, 3.0, 10.0, 30.0, 100.0, 300.0, 1e3)


def _ks_by_chi(s, table, proc, rng, chis=CHI_GRID, n=1 << 21):
    """Exact paired KS distance between the surrogate path's and the table's
    sampled spectra (same uniforms, n per chi) at each chi.  QS: the photon's
    fraction.  BW: the electron's fraction over [0, 1] (Sec. 2.1: the pair
    spectrum, symmetric about 1/2), i.e. the folded sample xi if u <= 1/2
    and 1 - xi otherwise; the folded sample alone would count every
    difference twice."""
    kss = []
    for chi in chis:
        u = rng.random(n).astype(np.float32)
        dc = torch.full((n,), chi, dtype=torch.float32, device="cuda")
        du = torch.as_tensor(u).cuda()
        out_s = torch.empty(n, dtype=torch.float32, device="cuda")
        out_t = torch.empty(n, dtype=torch.float32, device="cuda")
        s.sample(dc, du, out_s)
        Q.table_sample(table, dc, du, out_t)
        torch.cuda.synchronize()
        a, b = out_s.cpu().numpy().astype(np.float64), out_t.cpu().numpy().astype(np.float64)
        if proc == Q.BW:
            a, b = np.where(u <= 0.5, a, 1.0 - a), np.where(u <= 0.5, b, 1.0 - b)
        ks = _ks_paired(a, b)
        kss.append(ks)
        print(f"  chi={chi:g}: KS(surrogate, table) = {ks:.2e}")
    return kss


def _served(s):
    err, mask = s.bands()
    served = [(mask >> b) & 1 for b in range(64)]
    return err, float(np.mean(served))


@pytest.mark.parametrize("proc", [Q.QS, Q.BW])
def test_train_ks_fallback(ctx, tables512, trained, proc):
    table = tables512[0] if proc == Q.BW else tables512[1]
    s, loss = trained[proc]
    err, served = _served(s)
    print(f"process {proc}: final weighted loss {loss:.3e}; network serves {served:.2f} of the bands "
          f"(band errors {err.min():.2e} .. {err.max():.2e})")
    assert np.isfinite(loss)
    rng = np.random.default_rng(5)
    # the validated domain meets the KS gate at every chi, wherever the
    # short training left the network (the table serves the rest)
    chis = list(CHI_GRID) + list(np.exp(rng.uniform(np.log(1e-3), np.log(1e3), 24)))
    kss = _ks_by_chi(s, table, proc, rng, chis, n=1 << 20)
    assert max(kss) <= KS_GATE, max(kss)
    # outside the trained range the surrogate is the table, bit for bit
    chi = np.exp(rng.uniform(np.log(2e3), np.log(9e3), 10000)).astype(np.float32)
    u = rng.random(10000).astype(np.float32)
    dc, du = torch.as_tensor(chi).cuda(), torch.as_tensor(u).cuda()
    a, b = torch.empty_like(dc), torch.empty_like(dc)
    s.sample(dc, du, a)
    Q.table_sample(table, dc, du, b)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(a.cpu().numpy(), b.cpu().numpy())


@pytest.fixture(scope="module")
def bench_trained(ctx, tables512):
    """Both surrogates with the training the benchmark uses: 2^24 samples,
    half of them even in the network's second input, 320000 Adam steps of
    16384, band validation at 8e-4."""
    out = {}
    for proc in (Q.BW, Q.QS):
        table = tables512[0] if proc == Q.BW else tables512[1]
        cfg = Q.Surrogate.cfg(proc, 1e-3, 1e3, n_samples=1 << 24, batch=16384, steps=320000, lr=3e-3,
                              probe_tol=1.0, tail_permille=500, ks_budget=KS_BUDGET)
        out[proc] = Q.Surrogate.train(ctx, table, cfg)
    return out


@pytest.mark.parametrize("proc", [Q.QS, Q.BW])
def test_ks_with_benchmark_training(ctx, tables512, bench_trained, proc):
    """With the benchmark's training, the exact KS distance of the surrogate
    path's spectrum to the table's is within 1e-3 at 13 chi over the trained
    range and at 24 random chi, 2^21 samples each, and the network serves
    most of the range."""
    table = tables512[0] if proc == Q.BW else tables512[1]
    s, loss = bench_trained[proc]
    err, served = _served(s)
    print(f"process {proc}: final weighted loss {loss:.3e}; network serves {served:.2f} of the bands")
    rng = np.random.default_rng(6)
    chis = list(CHI_GRID) + list(np.exp(rng.uniform(np.log(1e-3), np.log(1e3), 24)))
    kss = _ks_by_chi(s, table, proc, rng, chis)
    assert max(kss) <= KS_GATE, max(kss)
    assert served >= 0.5


def test_band_validation_refuses_an_untrained_network(ctx, tables512):
    """A network with random weights fails the validation in every band, so
    the surrogate path samples exactly as the table does."""
    table = tables512[1]
    s = Q.Surrogate.from_host(table, Q.Surrogate.cfg(Q.QS, 1e-3, 1e3, ks_budget=KS_BUDGET), _random_params(9))
    err, served = _served(s)
    assert served == 0.0 and err.min() > KS_BUDGET
    rng = np.random.default_rng(10)
    n = 1 << 16
    chi = np.exp(rng.uniform(np.log(1e-3), np.log(1e3), n)).astype(np.float32)
    u = rng.random(n).astype(np.float32)
    dc, du = torch.as_tensor(chi).cuda(), torch.as_tensor(u).cuda()
    a, b = torch.empty_like(dc), torch.empty_like(dc)
    s.sample(dc, du, a)
    Q.table_sample(table, dc, du, b)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(a.cpu().numpy(), b.cpu().numpy())


def test_step_with_surrogate_probe_and_counts(ctx, tables):
    bw, qs = tables
    cfg_q = Q.Surrogate.cfg(Q.QS, 1e-3, 1e3, n_samples=1 << 21, steps=3000, probe_tol=1.0)
    cfg_b = Q.Surrogate.cfg(Q.BW, 1e-3, 1e3, n_samples=1 << 21, steps=3000, probe_tol=1.0)
    sq, _ = Q.Surrogate.train(ctx, qs, cfg_q)
    sb, _ = Q.Surrogate.train(ctx, bw, cfg_b)
    cfg_q0 = Q.Surrogate.cfg(Q.QS, 1e-3, 1e3, probe_tol=0.0, probe_every=1)
    cfg_b0 = Q.Surrogate.cfg(Q.BW, 1e-3, 1e3, probe_tol=0.0, probe_every=1)
    sq0 = Q.Surrogate.from_host(qs, cfg_q0, sq.params())
    sb0 = Q.Surrogate.from_host(bw, cfg_b0, sb.params())
    el, ph = QI.cone_population(seed=8, n=1 << 18)
    results = {}
    for name, surr in (("table", (None, None)), ("probe0", (sb0, sq0)), ("surr", (sb, sq))):
        d = []
        for pop in (el, ph):
            t = {k: torch.as_tensor(v).to("cuda", torch.float32) for k, v in pop.items()}
            t["tau"] = torch.empty_like(t["ux"])
            d.append(t)
        pe, pg = Q.particles(d[0], Q.ELECTRON, 0), Q.particles(d[1], Q.PHOTON, 1 << 18)
        Q.init_optical_depth(ctx, pe, 8)
        Q.init_optical_depth(ctx, pg, 8)
        bufs = [Q.AppendBuffer(1 << 18, torch.float32) for _ in range(3)]
        stats = torch.zeros(Q.STATS_LEN, dtype=torch.int64, device="cuda")
        fe = torch.zeros(1 << 18, dtype=torch.uint8, device="cuda")
        fg = torch.zeros(1 << 18, dtype=torch.uint8, device="cuda")
        desc = Q.StepDesc([pe, pg], bw=bw, qs=qs, photons=bufs[0], electrons=bufs[1], positrons=bufs[2],
                          flags=[fe, fg], stats=stats, dt=1e-16, seed=8, bw_surrogate=surr[0], qs_surrogate=surr[1])
        Q.step(ctx, desc)
        torch.cuda.synchronize()
        results[name] = dict(flags=(fe.cpu().numpy(), fg.cpu().numpy()), stats=stats.cpu().numpy(),
                             ph=bufs[0], el=bufs[1], state=[{k: v.cpu().numpy() for k, v in x.items()} for x in d])
    t0, p0, s1 = results["table"], results["probe0"], results["surr"]
    # with probe_tol = 0 every batch falls back: bit-identical to the table path
    assert p0["stats"][Q.STAT_SURR_BATCHES] > 0
    assert p0["stats"][Q.STAT_SURR_FALLBACK] == p0["stats"][Q.STAT_SURR_BATCHES]
    for k in ("ux", "tau"):
        np.testing.assert_array_equal(p0["state"][0][k], t0["state"][0][k])
    np.testing.assert_array_equal(p0["ph"].a["ux"].cpu().numpy(), t0["ph"].a["ux"].cpu().numpy())
    # with the surrogate: same events, same product counts and parents
    for i in range(2):
        np.testing.assert_array_equal(s1["flags"][i], t0["flags"][i])
    assert int(s1["ph"].count.item()) == int(t0["ph"].count.item())
    n = int(t0["ph"].count.item())
    np.testing.assert_array_equal(s1["ph"].parent[:n].cpu().numpy(), t0["ph"].parent[:n].cpu().numpy())
    assert s1["stats"][Q.STAT_SURR_BATCHES] > 0
    print("surrogate batches", s1["stats"][Q.STAT_SURR_BATCHES], "fallbacks", s1["stats"][Q.STAT_SURR_FALLBACK])
    # photon energies: distributions close
    e_s = np.linalg.norm(np.stack([s1["ph"].a[k][:n].cpu().numpy() for k in ("ux", "uy", "uz")], 1), axis=1)
    e_t = np.linalg.norm(np.stack([t0["ph"].a[k][:n].cpu().numpy() for k in ("ux", "uy", "uz")], 1), axis=1)
    ks = _ks_paired(np.log(e_s), np.log(e_t))
    print(f"photon energy KS (surrogate vs table, same draws) {ks:.2e}")
    assert ks < 0.1


def test_step_with_surrogate_and_photon_threshold(ctx, tables):
    """The surrogate inside the thresholded photon emission (Sec. 4: only
    photons above a minimum energy are created).  With every probe failing
    (tolerance 0) the step must equal the table path bit for bit; with the
    trained network the event flags equal the table path's (they do not
    depend on the sample), every kept photon is above the threshold and the
    parents are the flagged leptons in order."""
    bw, qs = tables
    cfg_q = Q.Surrogate.cfg(Q.QS, 1e-3, 1e3, n_samples=1 << 21, steps=3000, probe_tol=1.0)
    sq, _ = Q.Surrogate.train(ctx, qs, cfg_q)
    sq0 = Q.Surrogate.from_host(qs, Q.Surrogate.cfg(Q.QS, 1e-3, 1e3, probe_tol=0.0, probe_every=1), sq.params())
    el, ph = QI.cone_population(seed=9, n=1 << 18)
    threshold = 50.0   # photon energy floor, m c^2
    results = {}
    for name, surr in (("table", None), ("probe0", sq0), ("surr", sq)):
        d = []
        for pop in (el, ph):
            t = {k: torch.as_tensor(v).to("cuda", torch.float32) for k, v in pop.items()}
            t["tau"] = torch.empty_like(t["ux"])
            d.append(t)
        pe, pg = Q.particles(d[0], Q.ELECTRON, 0), Q.particles(d[1], Q.PHOTON, 1 << 18)
        Q.init_optical_depth(ctx, pe, 9)
        Q.init_optical_depth(ctx, pg, 9)
        bufs = [Q.AppendBuffer(1 << 18, torch.float32) for _ in range(3)]
        stats = torch.zeros(Q.STATS_LEN, dtype=torch.int64, device="cuda")
        fe = torch.zeros(1 << 18, dtype=torch.uint8, device="cuda")
        desc = Q.StepDesc([pe, pg], bw=bw, qs=qs, photons=bufs[0], electrons=bufs[1], positrons=bufs[2],
                          flags=[fe, None], stats=stats, dt=1e-16, seed=9, photon_min_energy=threshold,
                          qs_surrogate=surr)
        Q.step(ctx, desc)
        torch.cuda.synchronize()
        n = int(bufs[0].count.item())
        results[name] = dict(flags=fe.cpu().numpy(), stats=stats.cpu().numpy(), n=n,
                             parent=bufs[0].parent[:n].cpu().numpy(),
                             u=np.stack([bufs[0].a[k][:n].cpu().numpy() for k in ("ux", "uy", "uz")], 1),
                             state={k: d[0][k].cpu().numpy() for k in ("ux", "uy", "uz", "tau")})
    t0, p0, s1 = results["table"], results["probe0"], results["surr"]
    assert t0["n"] > 0 and t0["n"] < int(t0["flags"].sum())   # the threshold drops some photons
    assert p0["stats"][Q.STAT_SURR_BATCHES] > 0
    assert p0["stats"][Q.STAT_SURR_FALLBACK] == p0["stats"][Q.STAT_SURR_BATCHES]
    assert p0["n"] == t0["n"]
    np.testing.assert_array_equal(p0["parent"], t0["parent"])
    np.testing.assert_array_equal(p0["u"], t0["u"])
    for k in ("ux", "uy", "uz", "tau"):
        np.testing.assert_array_equal(p0["state"][k], t0["state"][k])
    np.testing.assert_array_equal(s1["flags"], t0["flags"])
    assert s1["stats"][Q.STAT_SURR_BATCHES] > 0
    assert s1["n"] > 0
    # kept photons: above the threshold (FP32 energy, one rounding of slack),
    # parents strictly increasing and all flagged
    energy = np.linalg.norm(s1["u"].astype(np.float64), axis=1)
    assert energy.min() >= threshold * (1 - 1e-6)
    assert np.all(np.diff(s1["parent"]) > 0)
    assert np.all(s1["flags"][s1["parent"]] == 1)


@pytest.mark.parametrize("proc", [Q.QS, Q.BW])
def test_gain_over_table(ctx, tables512, bench_trained, proc):
    """What the trained network gains over the table it replaces, and where.
    The standalone sampling call over 2^24 events (chi log-uniform over the
    trained range, 2^16 more outside it), timed with HIP events, for the
    table alone and for the network (its validated bands; the table
    elsewhere), with tables of 512^2, 2048^2 and 4096^2 points: 2, 32 and
    128 MiB of FP32 row pairs, the network 26 KB.  With tables resident in
    the L2 of an XCD (4 MiB) the table search is the faster; once they
    outgrow it, the search's scattered probes miss and the network gains.
    Asserted: the network path is faster than the 4096^2 table, and the
    out-of-range events match the table bit for bit."""
    n_in, n_out = 1 << 24, 1 << 16
    params = bench_trained[proc][0].params()
    chi = np.concatenate([QI.loguniform_chi(n_in, 3, 1e-3, 1e3), QI.loguniform_chi(n_out, 4, 2e3, 9e3)])
    u = QI.uniforms(n_in + n_out, 3, stream=proc)
    dc = torch.as_tensor(chi.astype(np.float32)).cuda()
    du = torch.as_tensor(u.astype(np.float32)).cuda()
    a, b = torch.empty_like(dc), torch.empty_like(dc)

    def timed(fn, reps=10):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    gains = {}
    for size in (512, 2048, 4096):
        table = (tables512[0] if proc == Q.BW else tables512[1]) if size == 512 else \
            Q.Table.generate_device(proc, RANGE[0], RANGE[1], size, size).to_device()
        s = Q.Surrogate.from_host(table, Q.Surrogate.cfg(proc, 1e-3, 1e3, ks_budget=KS_BUDGET), params)
        _, served = _served(s)
        t_table = timed(lambda: Q.table_sample(table, dc, du, b))
        t_net = timed(lambda: s.sample(dc, du, a))
        np.testing.assert_array_equal(a[n_in:].cpu().numpy(), b[n_in:].cpu().numpy())
        gains[size] = t_table / t_net
        print(f"process {proc}, {size}^2 tables ({4 * (size - 1) * size * 2 / 2**20:.1f} MiB FP32): table "
              f"{t_table:.3f} ms, network {t_net:.3f} ms (serving {served:.2f} of the bands), gain x{gains[size]:.2f}")
    assert gains[4096] > 1.0, gains
