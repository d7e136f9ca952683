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
    for name, sl in (("W1", slice(0, 128)), ("b1", slice(128, 192)), ("W2", slice(192, 4288)),
                     ("b2", slice(4288, 4352)), ("W3", slice(4352, 4416)), ("b3", slice(4416, 4417))):
        rel_q = np.linalg.norm(g[sl] - gq[sl]) / np.linalg.norm(gq[sl])
        rel_0 = np.linalg.norm(g[sl] - g0[sl]) / np.linalg.norm(g0[sl])
        print(f"grad {name}: vs bf16-emulated oracle {rel_q:.2e}, vs FP64 oracle {rel_0:.2e}")
        assert rel_q < 2e-3, name
        assert rel_0 < 5e-2, name


def _ks_paired(a, b):
    """sup over a quantile grid of |ECDF_a - ECDF_b| for samples drawn with
    the same uniforms."""
    g = np.quantile(b, np.linspace(0.0005, 0.9995, 2000))
    sa, sb = np.sort(a), np.sort(b)
    return float(np.max(np.abs(np.searchsorted(sa, g, "right") - np.searchsorted(sb, g, "right")) / len(a)))


@pytest.fixture(scope="module")
def tables512():
    """The 512 x 512 tables the surrogate is fitted to (chi over [1e-4, 1e4])."""
    return (Q.Table.generate(Q.BW, RANGE[0], RANGE[1], 512, 512).to_device(),
            Q.Table.generate(Q.QS, RANGE[0], RANGE[1], 512, 512).to_device())


@pytest.fixture(scope="module")
def trained(ctx, tables512):
    """Both surrogates trained on 2^24 samples, 40000 Adam steps of 16384."""
    out = {}
    for proc in (Q.BW, Q.QS):
        table = tables512[0] if proc == Q.BW else tables512[1]
        cfg = Q.Surrogate.cfg(proc, 1e-3, 1e3, n_samples=1 << 24, batch=16384, steps=40000, lr=3e-3,
                              probe_tol=1.0)
        out[proc] = Q.Surrogate.train(ctx, table, cfg)
    return out


def _ks_by_chi(s, table, proc, rng):
    """Paired KS distance between the network's and the table's samples
    (same uniforms, 2^20 per chi) at chi = 1e-3 ... 1e3."""
    n = 1 << 20
    kss = []
    for chi in (1e-3, 1e-2, 1e-1, 1.0, 10.0, 100.0, 1e3):
        if proc == Q.BW and chi < 0.05:
            continue  # pairs are not produced there (T(chi) ~ exp(-8/(3 chi)))
        u = rng.random(n).astype(np.float32)
        dc = torch.full((n,), chi, dtype=torch.float32, device="cuda")
        du = torch.as_tensor(u).cuda()
        out_s = torch.empty(n, dtype=torch.float32, device="cuda")
        out_t = torch.empty(n, dtype=torch.float32, device="cuda")
        s.sample(dc, du, out_s)
        Q.table_sample(table, dc, du, out_t)
        torch.cuda.synchronize()
        ks = _ks_paired(out_s.cpu().numpy(), out_t.cpu().numpy())
        kss.append(ks)
        print(f"  chi={chi:g}: KS(surrogate, table) = {ks:.2e}")
    return kss


@pytest.mark.parametrize("proc", [Q.QS, Q.BW])
def test_train_ks_fallback(ctx, tables512, trained, proc):
    table = tables512[0] if proc == Q.BW else tables512[1]
    s, loss = trained[proc]
    print(f"process {proc}: final weighted loss {loss:.3e}")
    assert np.isfinite(loss)
    rng = np.random.default_rng(5)
    kss = _ks_by_chi(s, table, proc, rng)
    # 40000 steps; measured on MI355X: QS <= 1.8e-3, BW <= 3.4e-3 (paired KS
    # noise with 2^20 samples ~ 1e-4); the bar leaves room for training-order
    # effects
    assert max(kss) < 5e-3
    # outside the trained range the surrogate is the table, bit for bit
    chi = np.exp(rng.uniform(np.log(2e3), np.log(9e3), 10000)).astype(np.float32)
    u = rng.random(10000).astype(np.float32)
    dc, du = torch.as_tensor(chi).cuda(), torch.as_tensor(u).cuda()
    a, b = torch.empty_like(dc), torch.empty_like(dc)
    s.sample(dc, du, a)
    Q.table_sample(table, dc, du, b)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(a.cpu().numpy(), b.cpu().numpy())


@pytest.mark.parametrize("proc", [Q.QS, Q.BW])
def test_ks_with_benchmark_training(ctx, tables512, proc):
    """The training the benchmark uses (2^24 samples, 320000 Adam steps of
    16384): measured on MI355X, KS <= 1e-3 up to chi = 1e2 and 1.05e-3 (QS)
    / 1.16e-3 (BW) at the upper end of the trained range."""
    table = tables512[0] if proc == Q.BW else tables512[1]
    cfg = Q.Surrogate.cfg(proc, 1e-3, 1e3, n_samples=1 << 24, batch=16384, steps=320000, lr=3e-3, probe_tol=1.0)
    s, loss = Q.Surrogate.train(ctx, table, cfg)
    print(f"process {proc}: final weighted loss {loss:.3e}")
    kss = _ks_by_chi(s, table, proc, np.random.default_rng(6))
    assert max(kss[:-1]) < 1.2e-3 and kss[-1] < 1.6e-3


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


def test_gain_over_table(ctx, tables512, trained):
    """What the network buys over the table: sampling time for 2^26 events
    with chi log-uniform over the trained range plus 2^16 out-of-range
    events (which fall back to the table), both kernels timed with HIP
    events on the launch stream, and the memory each needs; the fallback
    events match the table bit for bit.  The times are reported, not
    asserted: with 512 x 512 FP32 tables resident in L2 the table search is
    the faster of the two on this hardware."""
    n_in, n_out = 1 << 26, 1 << 16
    for proc in (Q.QS, Q.BW):
        table = tables512[0] if proc == Q.BW else tables512[1]
        s, _ = trained[proc]
        chi = np.concatenate([QI.loguniform_chi(n_in, 3, 1e-3, 1e3), QI.loguniform_chi(n_out, 4, 2e3, 9e3)])
        u = QI.uniforms(n_in + n_out, 3, stream=proc)
        dc = torch.as_tensor(chi.astype(np.float32)).cuda()
        du = torch.as_tensor(u.astype(np.float32)).cuda()
        a, b = torch.empty_like(dc), torch.empty_like(dc)
        times = {}
        for name, fn in (("table", lambda: Q.table_sample(table, dc, du, b)), ("surrogate", lambda: s.sample(dc, du, a))):
            fn()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(10):
                fn()
            e1.record()
            torch.cuda.synchronize()
            times[name] = e0.elapsed_time(e1) / 10
        np.testing.assert_array_equal(a[n_in:].cpu().numpy(), b[n_in:].cpu().numpy())
        tp = table.host_data()[0]
        print(f"process {proc}: table {times['table']:.3f} ms, surrogate {times['surrogate']:.3f} ms "
              f"for {n_in + n_out} events, {n_out / (n_in + n_out):.2e} of them out of range "
              f"(gain x{times['table'] / times['surrogate']:.2f}); "
              f"table {4 * tp.n_chi * (tp.n_frac + 1)} B in FP32, network {4 * 4417 + 2 * 4096} B")
        assert times["surrogate"] > 0 and times["table"] > 0
