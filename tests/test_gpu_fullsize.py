"""The FP64 fused step at the benchmark's full size and launch configuration
(2^24 leptons + 2^24 photons in the 0.1 rad cone, 256 x 256 tables over chi
in [1e-4, 1e3], dt = 0.1 fs, one qed_step over both sets, persistent grid
sized by occupancy) against the oracle over every particle: the oracle runs
a whole step of this size in about a second on the host's cores.

Bar as for the small parity cases: event flags, product counts and parent
ids bit-exact; optical depths within 1e-12 relative (scale max(|tau|, 1)),
momenta within 1e-12 of the largest |u| the particle has had (products: of
the parent's |u| at creation)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_2110_00256_amd as Q  # noqa: E402
import qed_inputs as QI  # noqa: E402
from oracle import oracle as O  # noqa: E402
from tests.gpu_util import compare_append, dev_pop, host, lib_tables, oracle_tables, rel_close  # noqa: E402

N = 1 << 24
RANGE = (1e-4, 1e3)
DT = 1e-16
SEED = 1
RTOL = 1e-12


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return Q.Context(0)


def test_bench_size_fp64_step_matches_oracle(ctx):
    print("tables 256 x 256 (library and oracle)", flush=True)
    (bw, qs) = lib_tables(RANGE, RANGE, 256, 256)
    (obw, oqs) = oracle_tables(RANGE, RANGE, 256, 256)
    print("population 2^24 + 2^24", flush=True)
    el, ph = QI.cone_population(seed=SEED, n=N)
    oe, og = O.Particles(el, O.ELECTRON, id_base=0), O.Particles(ph, O.PHOTON, id_base=N)
    O.init_optical_depth(oe, SEED)
    O.init_optical_depth(og, SEED)
    de, dg = dev_pop(el, torch.float64, tau=oe["tau"]), dev_pop(ph, torch.float64, tau=og["tau"])
    del el, ph
    pe, pg = Q.particles(de, Q.ELECTRON, 0), Q.particles(dg, Q.PHOTON, N)
    bufs = [Q.AppendBuffer(N, torch.float64) for _ in range(3)]
    flags = [torch.zeros(N, dtype=torch.uint8, device="cuda") for _ in range(2)]
    stats = torch.zeros(Q.STATS_LEN, dtype=torch.int64, device="cuda")
    desc = Q.StepDesc([pe, pg], bw=bw, qs=qs, photons=bufs[0], electrons=bufs[1], positrons=bufs[2],
                      flags=flags, stats=stats, dt=DT, seed=SEED)
    # a particle's momentum is compared on the scale of the largest |u| it
    # has had: an emission that leaves |u'| << |u| carries the rounding of
    # u - p_gamma, which is set by |u|, into later steps
    uscale = [np.zeros(N), np.zeros(N)]
    for s in range(2):
        u_before = [np.sqrt(o["ux"] ** 2 + o["uy"] ** 2 + o["uz"] ** 2) for o in (oe, og)]
        uscale = [np.maximum(a, b) for a, b in zip(uscale, u_before)]
        for b in bufs:
            b.reset()
        desc.set_step(s)
        Q.step(ctx, desc)
        apps = [O.Append(N) for _ in range(3)]
        fe, fg = np.zeros(N, np.uint8), np.zeros(N, np.uint8)
        ev = O.step(obw, oqs, oe, DT, SEED, s, apps[0], flags=fe)
        ev += O.step(obw, oqs, og, DT, SEED, s, apps[1], apps[2], flags=fg)
        torch.cuda.synchronize()
        print(f"step {s}: {apps[0].count} photons, {apps[1].count} pairs", flush=True)
        assert ev > N // 10
        np.testing.assert_array_equal(flags[0].cpu().numpy(), fe, err_msg=f"lepton flags step {s}")
        np.testing.assert_array_equal(flags[1].cpu().numpy(), fg, err_msg=f"photon flags step {s}")
        for d, o, ub in ((de, oe, uscale[0]), (dg, og, uscale[1])):
            assert rel_close(host(d["tau"]), o["tau"], RTOL) <= 1.0, f"tau step {s}"
            for k in ("ux", "uy", "uz"):
                assert rel_close(host(d[k]), o[k], RTOL, floor=np.maximum(ub, 1e-300)) <= 1.0, f"{k} step {s}"
        for b, a, o, ub, what in ((bufs[0], apps[0], oe, u_before[0], "photons"),
                                  (bufs[1], apps[1], og, u_before[1], "electrons"),
                                  (bufs[2], apps[2], og, u_before[1], "positrons")):
            par = a.parent[:a.count]
            compare_append(b, a, RTOL, f"{what} step {s}", ub[par - o.id_base])
    st = stats.cpu().numpy()
    assert st[Q.STAT_SCAN_TIMEOUT] == 0
    assert st[Q.STAT_UPDATES] == 2 * 2 * N
