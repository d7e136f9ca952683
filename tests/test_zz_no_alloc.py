"""qed_step_noalloc (the fused step with the library's fixed per-GPU
scratch, for callers that cannot allocate) against qed_step on the same
inputs.  Both run the same kernels, so every output must be bit-identical:
flags, optical depths, momenta, append counts and products, statistics.
Two calls in a row, the second on a smaller input with a shuffled tile
list, so the second call reuses scratch the first one left behind."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_2110_00256_amd as Q  # noqa: E402
import qed_inputs as QI  # noqa: E402
from tests.gpu_util import lib_tables  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return Q.Context(0)


@pytest.fixture(scope="module")
def tabs():
    return lib_tables((1e-3, 1e2), (1e-3, 1e2), 64, 64)


def _population(n_e, n_g, seed, dtype):
    el, ph = QI.parity_population(seed=seed, n=max(n_e, n_g))
    out = []
    for pop, n in ((el, n_e), (ph, n_g)):
        d = {k: torch.as_tensor(np.ascontiguousarray(v[:n])).to(device="cuda", dtype=dtype) for k, v in pop.items()}
        d["tau"] = torch.zeros(n, dtype=dtype, device="cuda")
        out.append(d)
    return out


def _layout(rng, n_e, n_g, pieces=7):
    tl = []
    for si, n in ((0, n_e), (1, n_g)):
        cuts = sorted(rng.choice(np.arange(1, n), pieces - 1, replace=False).tolist())
        edges = [0, *cuts, n]
        tl += [(si, int(a), int(b)) for a, b in zip(edges[:-1], edges[1:])]
    return [tl[i] for i in rng.permutation(len(tl))]


def _run(ctx, tabs, pops, tiles, seed, dtype, noalloc, noalloc_ctx=None, steps=2):
    """Two steps through qed_step (noalloc False) or qed_step_noalloc with
    `noalloc_ctx` (None: no context, SI units on the current device)."""
    bw, qs = tabs
    de, dg = pops
    pe, pg = Q.particles(de, Q.ELECTRON, 0), Q.particles(dg, Q.PHOTON, 1 << 40)
    Q.init_optical_depth(ctx, pe, seed)
    Q.init_optical_depth(ctx, pg, seed)
    n = max(len(de["ux"]), len(dg["ux"]))
    bufs = [Q.AppendBuffer(steps * n, dtype) for _ in range(3)]
    flags = [torch.zeros(len(d["ux"]), dtype=torch.uint8, device="cuda") for d in (de, dg)]
    stats = torch.zeros(Q.STATS_LEN, dtype=torch.int64, device="cuda")
    desc = Q.StepDesc([pe, pg], bw=bw, qs=qs, photons=bufs[0], electrons=bufs[1], positrons=bufs[2],
                      flags=flags, stats=stats, tiles=tiles, dt=1e-16, seed=seed)
    for s in range(steps):
        desc.set_step(s)
        if noalloc:
            Q.step_noalloc(noalloc_ctx, desc)
        else:
            Q.step(ctx, desc)
    torch.cuda.synchronize()
    return bufs, flags, stats


def _same(a, b, what):
    assert torch.equal(a, b), what


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_noalloc_matches_step_on_two_calls(ctx, tabs, dtype):
    rng = np.random.default_rng(2)
    # first call without a context, second (smaller, tiled) with one
    cases = [(1 << 16, 1 << 16, None, 7, None), (12289, 3001, _layout(rng, 12289, 3001), 8, ctx)]
    for call, (n_e, n_g, tiles, seed, nctx) in enumerate(cases):
        ref_pops = _population(n_e, n_g, seed, dtype)
        new_pops = _population(n_e, n_g, seed, dtype)
        rb, rf, rs = _run(ctx, tabs, ref_pops, tiles, seed, dtype, noalloc=False)
        nb, nf, ns = _run(ctx, tabs, new_pops, tiles, seed, dtype, noalloc=True, noalloc_ctx=nctx)
        assert int(rs[Q.STAT_QS_EVENTS].item()) > 100, call
        _same(rs, ns, f"call {call} stats")
        for i in range(2):
            _same(rf[i], nf[i], f"call {call} flags {i}")
            for k in ("ux", "uy", "uz", "tau"):
                _same(ref_pops[i][k], new_pops[i][k], f"call {call} set {i} {k}")
        for b1, b2, what in zip(rb, nb, ("photons", "electrons", "positrons")):
            c = int(b1.count.item())
            assert c == int(b2.count.item()), (call, what)
            assert c > 0, (call, what)
            _same(b1.parent[:c], b2.parent[:c], f"call {call} {what} parent")
            for k in ("ux", "uy", "uz", "w", "tau"):
                _same(b1.a[k][:c], b2.a[k][:c], f"call {call} {what} {k}")

