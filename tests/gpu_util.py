"""Helpers shared by the GPU tests: move seeded populations to the device,
run the oracle on the same inputs, compare with explicit tolerances."""
from __future__ import annotations

import numpy as np

import paper_2110_00256_amd as Q
import qed_inputs as QI
from oracle import oracle as O

SPECIES_STREAM = {O.ELECTRON: 0, O.POSITRON: 0, O.PHOTON: 1}


def dev_pop(pop: dict, dtype, tau=None):
    import torch
    out = {k: torch.as_tensor(np.ascontiguousarray(v)).to(device="cuda", dtype=dtype).contiguous()
           for k, v in pop.items()}
    n = len(pop["ux"])
    out["tau"] = (torch.zeros(n, dtype=dtype, device="cuda") if tau is None
                  else torch.as_tensor(np.asarray(tau)).to(device="cuda", dtype=dtype).contiguous())
    return out


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def rel_close(a, b, rtol, floor=1.0):
    """|a - b| <= rtol * max(|b|, floor), elementwise; returns max ratio."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    both_inf = np.isinf(a) & np.isinf(b) & (np.sign(a) == np.sign(b))
    with np.errstate(invalid="ignore"):
        d = np.where(both_inf, 0.0, np.abs(a - b))
    scale = np.maximum(np.abs(np.where(np.isinf(b), 1.0, b)), floor)
    r = d / (rtol * scale)
    return float(np.max(r)) if r.size else 0.0


def lib_tables(bw_range, qs_range, n_chi, n_frac, frac_min=1e-12):
    bw = Q.Table.generate(Q.BW, bw_range[0], bw_range[1], n_chi, n_frac).to_device()
    qs = Q.Table.generate(Q.QS, qs_range[0], qs_range[1], n_chi, n_frac, frac_min).to_device()
    return bw, qs


def oracle_tables(bw_range, qs_range, n_chi, n_frac, frac_min=1e-12):
    return (O.Table(O.BW, bw_range[0], bw_range[1], n_chi, n_frac),
            O.Table(O.QS, qs_range[0], qs_range[1], n_chi, n_frac, frac_min))


def compare_append(gpu_buf, orc_buf, rtol, what, parent_umag=None):
    """Counts and parent ids bit-exact, values within rtol; momenta on the
    scale of the parent's |u| at creation (parent_umag, one per product;
    default: the product's own |u|)."""
    n_g = int(gpu_buf.count.item())
    assert n_g == orc_buf.count, f"{what}: count {n_g} vs oracle {orc_buf.count}"
    n = min(n_g, gpu_buf.capacity)
    np.testing.assert_array_equal(gpu_buf.parent[:n].cpu().numpy(), orc_buf["parent"][:n], err_msg=what)
    if parent_umag is None:
        umag = np.sqrt(orc_buf["ux"] ** 2 + orc_buf["uy"] ** 2 + orc_buf["uz"] ** 2)
    else:
        umag = np.asarray(parent_umag, dtype=np.float64)
    for k in ("ux", "uy", "uz"):
        r = rel_close(host(gpu_buf.a[k][:n]), orc_buf[k][:n], rtol, floor=np.maximum(umag[:n], 1e-300))
        assert r <= 1.0, f"{what}.{k}: {r:.3g} x tolerance"
    for k in ("w", "tau"):
        r = rel_close(host(gpu_buf.a[k][:n]), orc_buf[k][:n], rtol)
        assert r <= 1.0, f"{what}.{k}: {r:.3g} x tolerance"
