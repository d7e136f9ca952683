"""The oracle's MLP reference (used to check the surrogate's kernels) is
pinned by central finite differences of its own loss in FP64."""
import numpy as np

from oracle import oracle as O


def test_mlp_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    p = rng.normal(size=O.MLP_NPARAM) * 0.3
    x = rng.uniform(-1, 1, size=(37, 2))
    t = rng.normal(size=37)
    w = rng.uniform(0.5, 2.0, size=37)
    loss, g = O.mlp_grad(p, x, t, w)
    idx = np.concatenate([rng.choice(128, 6, replace=False), 128 + rng.choice(64, 4, replace=False),
                          192 + rng.choice(4096, 12, replace=False), 4288 + rng.choice(64, 4, replace=False),
                          4352 + rng.choice(64, 4, replace=False), [4416]])
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (O.mlp_grad(pp, x, t, w)[0] - O.mlp_grad(pm, x, t, w)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), i
    # loss is the stated mean, and forward agrees with the loss' y
    y = O.mlp_forward(p, x)
    assert abs(loss - 0.5 * np.mean(w * (y - t) ** 2)) < 1e-12


def test_mlp_bf16_emulation_is_close():
    rng = np.random.default_rng(1)
    p = rng.normal(size=O.MLP_NPARAM) * 0.3
    x = rng.uniform(-1, 1, size=(64, 2))
    y0, y1 = O.mlp_forward(p, x), O.mlp_forward(p, x, bf16=True)
    assert 0 < np.max(np.abs(y1 - y0)) < 0.05 * np.max(np.abs(y0))
