"""The traffic-calibration call streams exactly the bytes it is given:
the write pass fills the buffer, the copy reproduces it, the read pass
leaves the destination alone for finite data, and bad arguments are
refused."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_2110_00256_amd as Q  # noqa: E402


def test_calibration_passes():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    n = (1 << 20) + 3
    src = torch.as_tensor(np.arange(n, dtype=np.float64) * 0.5).cuda()
    dst = torch.full((n,), -1.0, dtype=torch.float64, device="cuda")
    Q.traffic_calibrate(src, dst, 8 * n, 0)
    torch.cuda.synchronize()
    assert torch.all(dst == -1.0)
    Q.traffic_calibrate(src, dst, 8 * n, 1)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(dst.cpu().numpy(), np.arange(n, dtype=np.float64))
    Q.traffic_calibrate(src, dst, 8 * n, 2)
    torch.cuda.synchronize()
    assert torch.equal(dst, src)
    Q.traffic_calibrate(src, dst, 8 * n, 3)
    torch.cuda.synchronize()
    assert torch.equal(dst, src)
    dst.fill_(-1.0)
    Q.traffic_calibrate(src, dst, 8 * n, 4)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(dst.cpu().numpy(), np.arange(n, dtype=np.float64))
    for bad in ((8 * n + 4, 0), (8 * n, 5), (8 * n, -1)):
        with pytest.raises(Q.QedError):
            Q.traffic_calibrate(src, dst, *bad)
