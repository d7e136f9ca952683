"""Derive the time step of the full-step workload (4 species in lognormal
tiles, focused Gaussian pulse) so that the mean per-step event fraction of
the QED-active particles is 1%, using the oracle's rates on a 2^20-particle
subsample.  Writes tests/golden/fullstep_dt.json.  Run: python oracle/derive_fullstep_dt.py"""
import json
import math
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import qed_inputs as QI  # noqa: E402
from oracle import oracle as O  # noqa: E402

TARGET = 0.01
CHI_RANGE = (1e-4, 1e4)


def main():
    n = 1 << 20
    per = n // 3
    bw = O.Table(O.BW, CHI_RANGE[0], CHI_RANGE[1], 256, 3)
    qs = O.Table(O.QS, CHI_RANGE[0], CHI_RANGE[1], 256, 3)
    rates = []
    for sp, stream in ((O.ELECTRON, 0), (O.POSITRON, 1), (O.PHOTON, 2)):
        pop = QI.gaussian_pulse(per, seed=1, photon=(sp == O.PHOTON), stream=stream, dtype=np.float32)
        pop64 = {k: v.astype(np.float64) for k, v in pop.items()}
        chi = O.chi_array(pop64, sp == O.PHOTON)
        u2 = pop64["ux"] ** 2 + pop64["uy"] ** 2 + pop64["uz"] ** 2
        gam = np.sqrt(u2) if sp == O.PHOTON else np.sqrt(1 + u2)
        rates.append((bw if sp == O.PHOTON else qs).rate_n(chi, gam))
    r = np.concatenate(rates)

    def frac(dt):
        return float(np.mean(-np.expm1(-r * dt)))

    lo, hi = 1e-22, 1e-14
    for _ in range(200):
        mid = math.sqrt(lo * hi)
        if frac(mid) < TARGET:
            lo = mid
        else:
            hi = mid
    dt = math.sqrt(lo * hi)
    out = {"dt_s": dt, "event_fraction": frac(dt), "target": TARGET, "subsample": n,
           "recipe": "qed_inputs.gaussian_pulse, seed 1, streams 0/1/2 for e-/e+/photons, FP32 inputs; "
                     "oracle 256-point rate tables over chi [1e-4, 1e4]; mean of 1 - exp(-rate dt)"}
    path = os.path.join(ROOT, "tests", "golden", "fullstep_dt.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
