"""Library checks that need no GPU: the C ABI loads and exports every
declared symbol, host-side table generation agrees with the oracle's
independent quadrature, table files round-trip and reject corruption, and
invalid arguments are refused before anything is launched."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import paper_2110_00256_amd as Q
from oracle import oracle as O

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "qedmi.h")


def test_every_declared_symbol_is_exported():
    src = open(HEADER).read()
    declared = set(re.findall(r"^\s*(?:int32_t|void|const char\*)\s+(qed_\w+)\s*\(", src, re.M))
    assert declared == set(Q.EXPORTS)
    L = Q.lib()
    for name in declared:
        assert hasattr(L, name), name
    assert "gfx950" in Q.version()


@pytest.mark.parametrize("proc,cmin,cmax,nc,nf", [
    (Q.BW, 1e-3, 1e2, 64, 64),
    (Q.QS, 1e-3, 1e2, 64, 64),
    (Q.BW, 1e-4, 1e3, 12, 256),
    (Q.QS, 1e-4, 1e3, 12, 256),
])
def test_library_tables_match_oracle(proc, cmin, cmax, nc, nf):
    t = Q.Table.generate(proc, cmin, cmax, nc, nf)
    p, lr, cdf = t.host_data()
    assert (p.n_chi, p.n_frac) == (nc, nf)
    ot = O.Table(proc, cmin, cmax, nc, nf)
    assert np.max(np.abs(lr - ot.ln_rate) / np.maximum(1, np.abs(ot.ln_rate))) < 1e-13
    if proc == Q.BW:
        assert np.all(cdf[:, 0] == 0) and np.all(cdf[:, -1] == 0.5)
        assert np.max(np.abs(cdf - ot.cdf) / np.maximum(ot.cdf, 1e-10)) < 1e-12
    else:
        assert np.all(cdf[:, -1] == 0)
        assert np.max(np.abs(cdf - ot.cdf)) < 1e-13


def test_table_file_roundtrip_and_corruption(tmp_path):
    t = Q.Table.generate(Q.QS, 1e-2, 1e1, 8, 16)
    path = str(tmp_path / "qs.tab")
    t.save(path)
    u = Q.Table.load(path)
    p0, lr0, c0 = t.host_data()
    p1, lr1, c1 = u.host_data()
    np.testing.assert_array_equal(lr0, lr1)
    np.testing.assert_array_equal(c0, c1)
    raw = bytearray(open(path, "rb").read())
    raw[200] ^= 0x40
    bad = str(tmp_path / "bad.tab")
    open(bad, "wb").write(bytes(raw))
    with pytest.raises(Q.QedError) as e:
        Q.Table.load(bad)
    assert e.value.code == Q.QED_ERR_IO
    open(bad, "wb").write(bytes(raw[:100]))
    with pytest.raises(Q.QedError) as e:
        Q.Table.load(bad)
    assert e.value.code == Q.QED_ERR_IO
    with pytest.raises(Q.QedError) as e:
        Q.Table.load(str(tmp_path / "missing.tab"))
    assert e.value.code == Q.QED_ERR_IO


def test_from_host_wraps_arrays():
    ot = O.Table(O.BW, 1e-2, 1e1, 6, 9)
    t = Q.Table.from_host(Q.BW, 1e-2, 1e1, ot.ln_rate, ot.cdf)
    _, lr, cdf = t.host_data()
    np.testing.assert_array_equal(lr, ot.ln_rate)
    np.testing.assert_array_equal(cdf, ot.cdf)


@pytest.mark.parametrize("kw", [
    dict(process=7), dict(n_chi=1), dict(n_frac=2), dict(chi_min=0.0), dict(chi_max=1e-5),
    dict(process=Q.QS, frac_min=1.5),
])
def test_invalid_table_params(kw):
    args = dict(process=Q.BW, chi_min=1e-3, chi_max=1e2, n_chi=8, n_frac=8, frac_min=1e-12)
    args.update(kw)
    p = Q.TableParams(args["process"], args["n_chi"], args["n_frac"], 1, args["chi_min"], args["chi_max"],
                      args["frac_min"])
    h = C.c_void_p()
    assert Q.lib().qed_table_generate(C.byref(p), C.byref(h)) == Q.QED_ERR_INVALID
    assert h.value is None
    assert Q.lib().qed_last_error()


def test_null_arguments_are_refused_without_launch():
    L = Q.lib()
    assert L.qed_step(None, None, None) == Q.QED_ERR_INVALID
    assert L.qed_step_noalloc(None, None, None) == Q.QED_ERR_INVALID
    assert L.qed_chi_lepton(None, None, 0, None, None) == Q.QED_ERR_INVALID
    assert L.qed_read_count(None, None, None) == Q.QED_ERR_INVALID
    assert L.qed_table_to_device(None, None) == Q.QED_ERR_INVALID
    assert L.qed_context_create(0, None) == Q.QED_ERR_INVALID
    assert L.qed_schwinger_rate(None, None, None, None) == Q.QED_ERR_INVALID
    assert L.qed_schwinger_pairs(None, None, 1.0, 1.0, 1.0, 0, 0, None, None, None) == Q.QED_ERR_INVALID


def _desc_with_tiles(n, tiles, species=Q.ELECTRON):
    """A step descriptor over one set of n particles whose array pointers are
    dummies: the calls below are refused before anything touches them."""
    dummy = 1 << 20
    p = (Q.ParticlesC * 1)(Q.ParticlesC(*([dummy] * 11), n, 0, species, Q.FP64))
    t = np.ascontiguousarray(np.asarray(tiles, dtype=np.int64).reshape(-1))
    d = Q.StepDescC()
    d.sets = p
    d.n_sets = 1
    d.n_tiles = len(t) // 3
    d.tiles = t.ctypes.data_as(C.POINTER(C.c_int64))
    d.dt = 1e-16
    return d, (p, t)


def _refusal(tiles, n=1000):
    d, keep = _desc_with_tiles(n, tiles)
    rc = Q.lib().qed_step(None, C.byref(d), None)
    del keep
    return rc, Q.lib().qed_last_error().decode()


def test_tile_overlap_is_refused_before_launch():
    """Tiles of one set must be disjoint (an overlapping particle would be
    stepped twice).  The check is on the host, before the first HIP call and
    before the context is looked at, so it runs here without a GPU; tiles
    out of order but disjoint pass it and stop at the next check (the
    missing context)."""
    rc, msg = _refusal([(0, 0, 600), (0, 500, 1000)])
    assert rc == Q.QED_ERR_INVALID and "overlap" in msg
    rc, msg = _refusal([(0, 600, 1000), (0, 0, 300), (0, 250, 600)])     # out of order and overlapping
    assert rc == Q.QED_ERR_INVALID and "overlap" in msg
    rc, msg = _refusal([(0, 0, 1001)])
    assert rc == Q.QED_ERR_INVALID and "out of range" in msg
    rc, msg = _refusal([(0, 600, 1000), (0, 0, 300), (0, 300, 600), (0, 300, 300)])   # disjoint, shuffled, one empty
    assert rc == Q.QED_ERR_INVALID and "context" in msg



def test_noalloc_limits_are_refused_before_launch():
    """qed_step_noalloc's fixed scratch holds 8192 tiles and 65536 chunks of
    4096 particles; beyond either the call is refused with a message, before
    any HIP call (so this runs without a GPU)."""
    for tiles, n, what in (([(0, i, i + 1) for i in range(8193)], 8193, "8192 tiles"),
                           ([(0, 0, (1 << 28) + 1)], (1 << 28) + 1, "65536 chunks")):
        d, keep = _desc_with_tiles(n, tiles)
        assert Q.lib().qed_step_noalloc(None, C.byref(d), None) == Q.QED_ERR_INVALID
        assert what in Q.lib().qed_last_error().decode()
        del keep
    # an overlap is refused the same way as by qed_step
    d, keep = _desc_with_tiles(1000, [(0, 0, 600), (0, 500, 1000)])
    assert Q.lib().qed_step_noalloc(None, C.byref(d), None) == Q.QED_ERR_INVALID
    assert "overlap" in Q.lib().qed_last_error().decode()


def test_traffic_calibration_arguments_are_checked_before_launch():
    """The counter-calibration call refuses a bad mode, a byte count that is
    not a whole number of 8-byte words, and a missing buffer, before any HIP
    call (so this runs without a GPU); zero bytes is a no-op."""
    L = Q.lib()
    L.qed_traffic_calibrate.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_int32, C.c_void_p]
    dummy = C.c_void_p(8)   # never dereferenced: every case below returns before a launch
    for src, dst, nb, mode in ((dummy, dummy, 64, 5), (dummy, dummy, 64, -1), (dummy, dummy, 12, 0),
                               (dummy, dummy, -8, 1), (None, dummy, 64, 0), (dummy, None, 64, 1),
                               (None, dummy, 64, 3)):
        assert L.qed_traffic_calibrate(src, dst, nb, mode, None) == Q.QED_ERR_INVALID, (nb, mode)
        assert L.qed_last_error()
    assert L.qed_traffic_calibrate(None, None, 0, 0, None) == Q.QED_OK
