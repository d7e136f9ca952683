"""Tables generated on the GPU (FP64 HIP quadrature) against the oracle's own
quadrature of the same definitions (Sec. 2.1, 2.2 integrals, Sec. 3.1, 3.2
table layout), and against the host generator; the time of both generators
is printed (the paper generates on the CPU only).

Bar: ln T / ln G within 1e-12 of max(|ln|, 1); BW CDF within 1e-12 of
max(P, 1e-10); QS ln P within 1e-12 absolute; end points exact (measured on
MI355X: 1e-15 for the rates, 7e-14 for the CDFs)."""
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_2110_00256_amd as Q  # noqa: E402
from oracle import oracle as O  # noqa: E402

TOL = 1e-12


@pytest.fixture(scope="module")
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.zeros(1, device="cuda")
    return True


@pytest.mark.parametrize("proc,cmin,cmax,nc,nf", [
    (Q.BW, 1e-3, 1e2, 64, 64),
    (Q.QS, 1e-3, 1e2, 64, 64),
    (Q.BW, 1e-4, 1e4, 33, 256),
    (Q.QS, 1e-4, 1e4, 33, 256),
    (Q.QS, 1e-4, 1e3, 7, 1000),
])
def test_device_tables_match_oracle(gpu, proc, cmin, cmax, nc, nf):
    t = Q.Table.generate_device(proc, cmin, cmax, nc, nf)
    p, lr, cdf = t.host_data()
    assert (p.n_chi, p.n_frac) == (nc, nf)
    ot = O.Table(proc, cmin, cmax, nc, nf)
    e_rate = np.max(np.abs(lr - ot.ln_rate) / np.maximum(1, np.abs(ot.ln_rate)))
    if proc == Q.BW:
        assert np.all(cdf[:, 0] == 0) and np.all(cdf[:, -1] == 0.5)
        e_cdf = np.max(np.abs(cdf - ot.cdf) / np.maximum(ot.cdf, 1e-10))
    else:
        assert np.all(cdf[:, -1] == 0)
        e_cdf = np.max(np.abs(cdf - ot.cdf))
    print(f"proc {proc} {nc}x{nf} [{cmin:g}, {cmax:g}]: rate {e_rate:.2e}, cdf {e_cdf:.2e}")
    assert e_rate < TOL and e_cdf < TOL


def test_device_generation_time(gpu):
    for n in (256, 512):
        for proc in (Q.BW, Q.QS):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            td = Q.Table.generate_device(proc, 1e-4, 1e4, n, n)
            t1 = time.perf_counter()
            th = Q.Table.generate(proc, 1e-4, 1e4, n, n)
            t2 = time.perf_counter()
            _, lr_d, cdf_d = td.host_data()
            _, lr_h, cdf_h = th.host_data()
            d_rate = np.max(np.abs(lr_d - lr_h) / np.maximum(1, np.abs(lr_h)))
            print(f"proc {proc} {n}x{n}: device {t1 - t0:.3f} s, host {t2 - t1:.3f} s, max rate diff {d_rate:.2e}")
            assert d_rate < TOL
