"""Full QED sub-step over four species in lognormal tiles (one persistent
launch): the product append is bit-exact against the oracle's sequential
compaction of the GPU's own event flags (parents in tile, then index,
order), ions are never touched, and the event fraction sits near the 1%
the time step was derived for."""
import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_2110_00256_amd as Q  # noqa: E402
import qed_inputs as QI  # noqa: E402
from oracle import oracle as O  # noqa: E402

GOLD = os.path.join(os.path.dirname(__file__), "golden", "fullstep_dt.json")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return Q.Context(0)


def test_tiled_four_species_compaction(ctx):
    dt = json.load(open(GOLD))["dt_s"]
    n, tps = 1 << 17, 64
    pops = QI.fullstep_population(n, seed=3)
    tiles = QI.fullstep_layout(n, tps, seed=3)
    assert tiles.shape == (4 * tps, 3)
    bw = Q.Table.generate(Q.BW, 1e-4, 1e4, 128, 128).to_device()
    qs = Q.Table.generate(Q.QS, 1e-4, 1e4, 128, 128).to_device()
    species = (Q.ELECTRON, Q.POSITRON, Q.PHOTON, Q.ION)
    dev, sets = [], []
    for i, (pop, sp) in enumerate(zip(pops, species)):
        d = {k: torch.as_tensor(v).cuda() for k, v in pop.items()}
        d["tau"] = torch.empty(n, dtype=torch.float32, device="cuda") if sp != Q.ION else \
            torch.as_tensor(np.arange(n, dtype=np.float32)).cuda()
        dev.append(d)
        sets.append(Q.particles(d, sp, id_base=i * n))
    for s in sets[:3]:
        Q.init_optical_depth(ctx, s, 3)
    ion_before = {k: v.clone() for k, v in dev[3].items()}
    bufs = [Q.AppendBuffer(n, torch.float32) for _ in range(3)]
    flags = [torch.zeros(n, dtype=torch.uint8, device="cuda") for _ in range(4)]
    stats = torch.zeros(Q.STATS_LEN, dtype=torch.int64, device="cuda")
    desc = Q.StepDesc(sets, bw=bw, qs=qs, photons=bufs[0], electrons=bufs[1], positrons=bufs[2], tiles=tiles,
                      flags=flags, stats=stats, dt=dt, seed=3)
    set_stream = [0, 0, 1, -1]
    id_base = [0, n, 2 * n, 3 * n]
    total_ev = 0
    for step in range(3):
        for b in bufs:
            b.reset()
        desc.set_step(step)
        Q.step(ctx, desc)
        torch.cuda.synchronize()
        fl = [f.cpu().numpy() for f in flags]
        for stream, b in ((0, bufs[0]), (1, bufs[1]), (1, bufs[2])):
            ref = O.compact(tiles, set_stream, fl, id_base, stream)
            got = b.parent[: int(b.count.item())].cpu().numpy()
            np.testing.assert_array_equal(got, ref)
        total_ev += sum(int(f.sum()) for f in fl[:3])
    for k in ion_before:
        assert torch.equal(dev[3][k], ion_before[k])
    st = stats.cpu().numpy()
    assert st[Q.STAT_UPDATES] == 3 * 3 * n
    assert st[Q.STAT_SCAN_TIMEOUT] == 0
    frac = total_ev / (3 * 3 * n)
    print(f"event fraction per step {frac:.4f}")
    assert 0.005 < frac < 0.02


def test_surrogate_path_at_full_size(ctx):
    """The full sub-step as configured: 2^25 particles in each of the four
    species (2^27 in all), 1024 lognormal tiles per species interleaved
    species by species, FP32 fields of the focused Gaussian pulse, the
    FP32 + learned-surrogate path, one persistent launch per step.  The
    append of every product stream is bit-exact against the oracle's
    sequential compaction of the GPU's flags, the network sampled most event
    batches, ions are untouched and every particle was updated once."""
    dt = json.load(open(GOLD))["dt_s"]
    n, tps = 1 << 25, 1024
    print(f"surrogate full-size step: 4 x {n} particles, {4 * tps} tiles", flush=True)
    pops = QI.fullstep_population(n, seed=5)
    tiles = QI.fullstep_layout(n, tps, seed=5)
    bw = Q.Table.generate(Q.BW, 1e-4, 1e4, 256, 256).to_device()
    qs = Q.Table.generate(Q.QS, 1e-4, 1e4, 256, 256).to_device()
    sq, _ = Q.Surrogate.train(ctx, qs, Q.Surrogate.cfg(Q.QS, 1e-3, 1e3, n_samples=1 << 22, steps=20000))
    sb, _ = Q.Surrogate.train(ctx, bw, Q.Surrogate.cfg(Q.BW, 1e-3, 1e3, n_samples=1 << 22, steps=20000))
    species = (Q.ELECTRON, Q.POSITRON, Q.PHOTON, Q.ION)
    dev, sets = [], []
    for i, (pop, sp) in enumerate(zip(pops, species)):
        d = {k: torch.as_tensor(v).cuda() for k, v in pop.items()}
        d["tau"] = torch.empty(n, dtype=torch.float32, device="cuda") if sp != Q.ION else \
            torch.as_tensor(np.arange(n, dtype=np.float32)).cuda()
        dev.append(d)
        sets.append(Q.particles(d, sp, id_base=i * n))
    del pops
    for s in sets[:3]:
        Q.init_optical_depth(ctx, s, 5)
    ion_before = {k: v.clone() for k, v in dev[3].items()}
    cap = n // 8
    bufs = [Q.AppendBuffer(cap, torch.float32) for _ in range(3)]
    flags = [torch.zeros(n, dtype=torch.uint8, device="cuda") for _ in range(4)]
    stats = torch.zeros(Q.STATS_LEN, dtype=torch.int64, device="cuda")
    desc = Q.StepDesc(sets, bw=bw, qs=qs, photons=bufs[0], electrons=bufs[1], positrons=bufs[2], tiles=tiles,
                      flags=flags, stats=stats, dt=dt, seed=5, bw_surrogate=sb, qs_surrogate=sq)
    set_stream = [0, 0, 1, -1]
    id_base = [0, n, 2 * n, 3 * n]
    total_ev = 0
    for step in range(2):
        for b in bufs:
            b.reset()
        desc.set_step(step)
        Q.step(ctx, desc)
        torch.cuda.synchronize()
        fl = [f.cpu().numpy() for f in flags]
        for stream, b in ((0, bufs[0]), (1, bufs[1]), (1, bufs[2])):
            ref = O.compact(tiles, set_stream, fl, id_base, stream)
            cnt = int(b.count.item())
            assert cnt == len(ref) <= cap
            np.testing.assert_array_equal(b.parent[:cnt].cpu().numpy(), ref)
        total_ev += sum(int(f.sum()) for f in fl[:3])
        print(f"step {step}: {total_ev} events so far", flush=True)
    for k in ion_before:
        assert torch.equal(dev[3][k], ion_before[k])
    st = stats.cpu().numpy()
    assert st[Q.STAT_UPDATES] == 2 * 3 * n
    assert st[Q.STAT_SCAN_TIMEOUT] == 0 and st[Q.STAT_NONFINITE] == 0
    assert st[Q.STAT_SURR_BATCHES] > 0
    assert st[Q.STAT_SURR_FALLBACK] < 0.05 * st[Q.STAT_SURR_BATCHES]
    frac = total_ev / (2 * 3 * n)
    print(f"event fraction per step {frac:.4f}; surrogate batches {st[Q.STAT_SURR_BATCHES]}, "
          f"fallbacks {st[Q.STAT_SURR_FALLBACK]}")
    assert 0.005 < frac < 0.02
