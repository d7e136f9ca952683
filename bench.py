#!/usr/bin/env python3
"""Throughput of the fused QED step on one MI355X.

Workload (default): 2^24 leptons + 2^24 photons, momenta in a 0.1 rad cone
about -x with gamma log-uniform in [1e2, 1e5], linearly polarised plane-wave
fields with a0 log-uniform in [10, 1000], 256 x 256 tables over chi in
[1e-4, 1e3], dt = 0.1 fs.  One "step" is one qed_step over all 2^25
particles (chi, rate, tau update, events, sampling, product append).

value = FP64 table-path particle updates per second over the timed steps;
the FP32 path is reported beside it.  Inputs are resident in HBM before the
timed region; product buffers are emptied (one 3-element fill) before each
step, as a PIC code does when it merges the products.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
# surrogate bands whose largest CDF-space error against the table exceeds
# this are sampled by the table (KS gate 1e-3 less a margin)
SURR_KS_BUDGET = 8e-4
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "QED particle updates/s at 1 MI355X (FP64 table vs FP32+surrogate), % HBM peak"
HBM_PEAK_GBS = 8000.0

# algorithmic bytes per particle update (u, E, B, tau read; tau written) and extra per
# event (parent u written, w read, product records)
BYTES = {
    "f64": dict(base=88, qs_event=80, bw_event=104),
    "f32": dict(base=44, qs_event=44, bw_event=60),
}
# the same split into bytes read and written: per update u, E, B, tau read and
# tau written; per QS event w read, parent u, photon (u, w, tau) and parent id
# written; per BW event w read, two products and their parent ids written
BYTES_RW = {
    "f64": dict(base=(80, 8), qs_event=(8, 72), bw_event=(8, 96)),
    "f32": dict(base=(40, 4), qs_event=(4, 40), bw_event=(4, 56)),
}


# HBM bytes per launch measured with rocprofv3 (FETCH_SIZE, WRITE_SIZE, each
# calibrated on a stream with the step's own access pattern) live in this summary, tagged with a digest of
# the step kernel's sources; they are reported only while the digest matches.
PROFILE = os.path.join(ROOT, "profiles", "step_kernel_cone_2x2e24.md")
KERNEL_SOURCES = ("step.hip", "device_physics.hpp", "internal.hpp", "surrogate.hpp", "constants.hpp")


def kernel_digest():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2110_00256_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """The profile summary's traffic record ({"bytes_per_launch": {path: HBM
    bytes}, "fetch_bytes_per_launch", "write_bytes_per_launch",
    "calibration"}), or {} if the step kernel's sources have changed since."""
    try:
        with open(PROFILE) as f:
            for line in f:
                if line.startswith("traffic-json: "):
                    d = json.loads(line[len("traffic-json: "):])
                    return d if d.get("source_digest") == kernel_digest() else {}
    except OSError:
        pass
    return {}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_tables(Q, n_chi, n_frac, chi_range):
    bw = Q.Table.generate(Q.BW, chi_range[0], chi_range[1], n_chi, n_frac).to_device()
    qs = Q.Table.generate(Q.QS, chi_range[0], chi_range[1], n_chi, n_frac, 1e-12).to_device()
    return bw, qs


def run_path(Q, torch, ctx, tables, pops, dtype, steps, warmup, dt, chi_mode, seed=1, surrogates=(None, None)):
    tdt = torch.float64 if dtype == "f64" else torch.float32
    el, ph = pops
    dev = []
    for pop in (el, ph):
        d = {k: torch.as_tensor(v).to("cuda", dtype=tdt) for k, v in pop.items()}
        d["tau"] = torch.empty_like(d["ux"])
        dev.append(d)
    n_e, n_g = len(el["ux"]), len(ph["ux"])
    pe = Q.particles(dev[0], Q.ELECTRON, 0)
    pg = Q.particles(dev[1], Q.PHOTON, n_e)
    Q.init_optical_depth(ctx, pe, seed)
    Q.init_optical_depth(ctx, pg, seed)
    counts = torch.zeros(3, dtype=torch.int64, device="cuda")
    cap = (n_e + n_g) // 2
    bufs = []
    for i in range(3):
        b = Q.AppendBuffer(cap, tdt)
        b.c.count = counts.data_ptr() + 8 * i
        b.count = counts[i:i + 1]
        bufs.append(b)
    stats = torch.zeros(Q.STATS_LEN, dtype=torch.int64, device="cuda")
    bw, qs = tables
    desc = Q.StepDesc([pe, pg], bw=bw, qs=qs, photons=bufs[0], electrons=bufs[1], positrons=bufs[2],
                      stats=stats, dt=dt, seed=seed, chi_mode=chi_mode, bw_surrogate=surrogates[0],
                      qs_surrogate=surrogates[1])
    step = 0
    for _ in range(warmup):
        counts.zero_()
        desc.set_step(step)
        Q.step(ctx, desc)
        step += 1
    torch.cuda.synchronize()
    need = int(counts.max().item())
    if need > cap:
        raise RuntimeError(f"product capacity {cap} too small ({need})")
    stats.zero_()
    ev0 = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ev1 = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        counts.zero_()
        desc.set_step(step)
        ev0[i].record()
        Q.step(ctx, desc)
        ev1[i].record()
        step += 1
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = np.array([a.elapsed_time(b) for a, b in zip(ev0, ev1)])
    st = stats.cpu().numpy()
    assert st[Q.STAT_SCAN_TIMEOUT] == 0, "look-back wait abandoned"
    updates = int(st[Q.STAT_UPDATES])
    assert updates == steps * (n_e + n_g)
    qs_ev, bw_ev = int(st[Q.STAT_QS_EVENTS]), int(st[Q.STAT_BW_EVENTS])
    by = BYTES[dtype]
    alg_bytes = by["base"] * updates + by["qs_event"] * qs_ev + by["bw_event"] * bw_ev
    rw = BYTES_RW[dtype]
    alg_rw = [rw["base"][i] * updates + rw["qs_event"][i] * qs_ev + rw["bw_event"][i] * bw_ev for i in (0, 1)]
    kern_s = kern_ms.sum() / 1e3
    res = dict(
        updates_per_s=updates / wall,
        ms_per_step=wall / steps * 1e3,
        kernel_ms_mean=float(kern_ms.mean()),
        kernel_ms_median=float(np.median(kern_ms)),
        achieved_gbs=alg_bytes / kern_s / 1e9,
        alg_bytes_per_launch=alg_bytes / steps,
        alg_read_bytes_per_launch=alg_rw[0] / steps,
        alg_write_bytes_per_launch=alg_rw[1] / steps,
        qs_event_fraction=qs_ev / (steps * n_e),
        bw_event_fraction=bw_ev / (steps * n_g),
        surrogate_batches=int(st[Q.STAT_SURR_BATCHES]),
        surrogate_fallbacks=int(st[Q.STAT_SURR_FALLBACK]),
    )
    del dev, bufs
    return res


_ORACLE_TABLES = {}


def cpu_baseline(pops_small, tables_params, dt, seed=1, min_seconds=10.0, max_steps=400):
    """The oracle, as it stands, on a bounded sample of the same workload."""
    from oracle import oracle as O
    n_chi, n_frac, rng = tables_params
    key = (n_chi, n_frac, rng[0], rng[1])
    if key not in _ORACLE_TABLES:
        log("cpu_baseline: generating oracle tables")
        _ORACLE_TABLES[key] = (O.Table(O.BW, rng[0], rng[1], n_chi, n_frac), O.Table(O.QS, rng[0], rng[1], n_chi, n_frac))
    obw, oqs = _ORACLE_TABLES[key]
    el, ph = pops_small
    oe, og = O.Particles(el, O.ELECTRON, 0), O.Particles(ph, O.PHOTON, 1 << 40)
    O.init_optical_depth(oe, seed)
    O.init_optical_depth(og, seed)
    n = oe.n + og.n
    a1, a2, a3 = O.Append(oe.n), O.Append(og.n), O.Append(og.n)
    log(f"cpu_baseline: timing oracle steps over {n} particles for at least {min_seconds} s")
    steps = 0
    t0 = time.perf_counter()
    while steps < max_steps and (steps == 0 or time.perf_counter() - t0 < min_seconds):
        a1.count = a2.count = a3.count = 0
        O.step(obw, oqs, oe, dt, seed, steps, a1)
        O.step(obw, oqs, og, dt, seed, steps, a2, a3)
        steps += 1
    wall = time.perf_counter() - t0
    cores = O.max_threads()
    return dict(value=steps * n / wall, unit="particle updates/s", cores=cores, kind="oracle",
                cpu=cpu_model(),
                sample=f"{oe.n} leptons + {og.n} photons of the same workload, {steps} steps "
                       f"(FP64 C oracle, OpenMP over particles, sequential append), {wall:.1f} s")


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline_one_thread(pops_small, tables_params, dt, seed=1, min_seconds=5.0):
    """The same oracle on one thread (a smaller sample: per-update cost does
    not depend on the population size)."""
    from oracle import oracle as O
    threads = O.max_threads()
    O.set_threads(1)
    try:
        r = cpu_baseline(pops_small, tables_params, dt, seed, min_seconds=min_seconds)
    finally:
        O.set_threads(threads)
    return r


def fullstep(Q, torch, QI, args):
    """4 species x 2^(log2n + 1) particles (default 2^25 each: 2^27 in all),
    1024 lognormal tiles per species interleaved, FP32 fields of a focused
    Gaussian pulse, dt for 1% events; one persistent launch per step."""
    n = 1 << (args.log2n + 1)
    dt = json.load(open(os.path.join(ROOT, "tests", "golden", "fullstep_dt.json")))["dt_s"]
    log(f"fullstep: generating 4 x {n} particles and 4096 tiles")
    pops = QI.fullstep_population(n, seed=1)
    tiles = QI.fullstep_layout(n, 1024, seed=1)
    ctx = Q.Context(0)
    log("fullstep: 256x256 tables over [1e-4, 1e4]")
    bw = Q.Table.generate(Q.BW, 1e-4, 1e4, 256, 256).to_device()
    qs = Q.Table.generate(Q.QS, 1e-4, 1e4, 256, 256).to_device()
    species = (Q.ELECTRON, Q.POSITRON, Q.PHOTON, Q.ION)
    dev, sets = [], []
    for i, (pop, sp) in enumerate(zip(pops, species)):
        d = {k: torch.as_tensor(v).cuda() for k, v in pop.items()}
        d["tau"] = torch.zeros(n, dtype=torch.float32, device="cuda")
        dev.append(d)
        sets.append(Q.particles(d, sp, id_base=i * n))
    del pops
    log("fullstep: training surrogates")
    t0 = time.perf_counter()
    sq, lq = Q.Surrogate.train(ctx, qs, Q.Surrogate.cfg(Q.QS, 1e-3, 1e3, n_samples=1 << 24, steps=args.surrogate_steps,
                                                        tail_permille=500, ks_budget=SURR_KS_BUDGET))
    sb, lb = Q.Surrogate.train(ctx, bw, Q.Surrogate.cfg(Q.BW, 1e-3, 1e3, n_samples=1 << 24, steps=args.surrogate_steps,
                                                        tail_permille=500, ks_budget=SURR_KS_BUDGET))
    train_s = time.perf_counter() - t0
    out = {"workload": "fullstep: 4 x 2^%d particles (e-, e+, photons, ions passthrough), 4096 lognormal tiles, "
                       "Gaussian pulse a0=500 w0=2um, FP32, dt %.3e s" % (int(np.log2(n)), dt),
           "surrogate_train_s": train_s, "surrogate_final_loss": {"qs": lq, "bw": lb}}
    for name, surr in (("fp32_table", (None, None)), ("fp32_surrogate", (sb, sq))):
        for s in sets[:3]:
            Q.init_optical_depth(ctx, s, 1)
        counts = torch.zeros(3, dtype=torch.int64, device="cuda")
        bufs = []
        for i in range(3):
            b = Q.AppendBuffer(n // 8, torch.float32)
            b.c.count = counts.data_ptr() + 8 * i
            b.count = counts[i:i + 1]
            bufs.append(b)
        stats = torch.zeros(Q.STATS_LEN, dtype=torch.int64, device="cuda")
        desc = Q.StepDesc(sets, bw=bw, qs=qs, photons=bufs[0], electrons=bufs[1], positrons=bufs[2], tiles=tiles,
                          stats=stats, dt=dt, seed=1, bw_surrogate=surr[0], qs_surrogate=surr[1])
        for w in range(args.warmup):
            counts.zero_()
            desc.set_step(w)
            Q.step(ctx, desc)
        torch.cuda.synchronize()
        stats.zero_()
        e0 = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
        e1 = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
        t0 = time.perf_counter()
        for i in range(args.steps):
            counts.zero_()
            desc.set_step(args.warmup + i)
            e0[i].record()
            Q.step(ctx, desc)
            e1[i].record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        km = float(np.mean([a.elapsed_time(b) for a, b in zip(e0, e1)]))
        st = stats.cpu().numpy()
        upd = int(st[Q.STAT_UPDATES])
        qs_ev, bw_ev = int(st[Q.STAT_QS_EVENTS]), int(st[Q.STAT_BW_EVENTS])
        by = BYTES["f32"]
        alg = by["base"] * upd + by["qs_event"] * qs_ev + by["bw_event"] * bw_ev
        out[name] = {"updates_per_s": upd / wall, "kernel_ms_mean": km, "event_fraction": (qs_ev + bw_ev) / upd,
                     "achieved_gbs": alg / (km * 1e-3 * args.steps) / 1e9,
                     "frac": alg / (km * 1e-3 * args.steps) / 1e9 / HBM_PEAK_GBS,
                     "surrogate_batches": int(st[Q.STAT_SURR_BATCHES]),
                     "surrogate_fallbacks": int(st[Q.STAT_SURR_FALLBACK])}
        log(f"fullstep {name}: {out[name]}")
    print(json.dumps(out), flush=True)


# The paper's own kernel timings (Sec. 4, Table comp, NVIDIA Quadro GV100,
# CUDA), ms for 1e8 particles, FP64 / FP32: context for the paper workload.
PAPER_GV100_MS = {
    "bw_evol": (14.52, 7.43), "bw_prod": (29.94, 15.70),
    "qs_evol": (14.62, 7.39), "qs_em": (26.88, 14.15),
}


def paper(Q, torch, QI, args):
    """The paper's benchmark (Sec. 4): 1e8 particles with E, B and p
    components uniform in +-E_s/100, +-E_s/(100c), +-1 GeV/c, optical depth
    Exp(1); 256-point rate tables and 256x256 CDF tables, chi_min 1e-3 (QS)
    and 0.02 (BW), chi_max 1e3; each of the four standalone calls applied to
    every particle (for pair production and photon emission: every particle
    is flagged and produces), timed on the device, FP64 and FP32."""
    n = args.paper_n
    log(f"paper: generating 2 x {n} particles")
    pops = (QI.paper_uniform(n, seed=1, stream=0), QI.paper_uniform(n, seed=1, stream=1))
    ctx = Q.Context(0)
    log("paper: tables")
    bw = Q.Table.generate(Q.BW, 0.02, 1e3, 256, 256).to_device()
    qs = Q.Table.generate(Q.QS, 1e-3, 1e3, 256, 256, 1e-12).to_device()
    out = {"workload": f"paper Sec. 4 benchmark: {n} particles per call, uniform E, B, p; 256 / 256x256 tables; "
                       "every particle produces in bw_prod and qs_em",
           "particles": n, "runs": args.steps}
    for dt_name, tdt, idx in (("f64", torch.float64, 0), ("f32", torch.float32, 1)):
        dev = []
        for pop in pops:
            d = {k: torch.as_tensor(v).to("cuda", dtype=tdt) for k, v in pop.items()}
            d["tau"] = torch.empty_like(d["ux"])
            dev.append(d)
        pl = Q.particles(dev[0], Q.ELECTRON, 0)
        pg = Q.particles(dev[1], Q.PHOTON, n)
        Q.init_optical_depth(ctx, pl, 1)
        Q.init_optical_depth(ctx, pg, 1)
        saved = [{k: d[k].clone() for k in ("ux", "uy", "uz", "tau")} for d in dev]
        flags = torch.ones(n, dtype=torch.uint8, device="cuda")
        ph = Q.AppendBuffer(n, tdt)
        el, po = Q.AppendBuffer(n, tdt), Q.AppendBuffer(n, tdt)
        dt = 1e-16

        def restore():
            for d, s0 in zip(dev, saved):
                for k, v in s0.items():
                    d[k].copy_(v)
            for b in (ph, el, po):
                b.reset()

        calls = {
            "bw_evol": lambda: Q.evolve_optical_depth(ctx, bw, pg, dt),
            "bw_prod": lambda: Q.generate_pairs(ctx, bw, pg, flags, 1, 0, el, po),
            "qs_evol": lambda: Q.evolve_optical_depth(ctx, qs, pl, dt),
            "qs_em": lambda: Q.generate_photon_and_update_momentum(ctx, qs, pl, flags, 1, 0, ph),
        }
        res = {}
        for name, fn in calls.items():
            restore()
            fn()
            ms = []
            for _ in range(args.steps):
                restore()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                fn()
                e1.record()
                torch.cuda.synchronize()
                ms.append(e0.elapsed_time(e1))
            if name == "bw_prod":
                assert int(el.count.item()) == n and int(po.count.item()) == n
            if name == "qs_em":
                assert int(ph.count.item()) == n
            m = float(np.mean(ms))
            gv = PAPER_GV100_MS[name][idx]
            res[name] = {"ms_mean": m, "updates_per_s": n / (m * 1e-3), "gv100_cuda_ms_for_1e8": gv,
                         "speedup_vs_gv100": gv * (n / 1e8) / m}
            log(f"paper {dt_name} {name}: {m:.3f} ms ({res[name]['speedup_vs_gv100']:.1f}x the GV100 time)")
        out[dt_name] = res
        del dev, saved, ph, el, po, flags
        torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


def extras(Q, torch, QI, args):
    """Throughput of the library's other kernels (one JSON line): the
    Schwinger rate and pair count over 2^26 cells (fields uniform in
    +-E_s/10, +-E_s/(10c)), and the Boris push of 2^25 electrons through a
    circularly polarised wave (E0 = 1.22e-4 E_s, 0.8 um), FP64, HIP events on
    the launch stream, mean of 10 calls after one warm-up; and the device
    table generation (256 x 256 and 512 x 512 over chi in [1e-4, 1e3], wall
    time of the synchronous call after one warm-up)."""
    ctx = Q.Context(0)
    out = {"workload": "extras: Schwinger rate/pairs on 2^26 cells, push of 2^25 electrons, FP64"}

    def timed(fn, reps=10):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    n = 1 << 26
    g = torch.Generator(device="cuda")
    g.manual_seed(1)
    es = QI.E_SCHWINGER
    d = {k: (torch.rand(n, generator=g, device="cuda", dtype=torch.float64) * 2 - 1) * es / 10 *
         (1.0 if k[0] == "e" else 1.0 / QI.C_LIGHT) for k in ("ex", "ey", "ez", "bx", "by", "bz")}
    c = Q.cells(d)
    rate = torch.empty(n, dtype=torch.float64, device="cuda")
    ms = timed(lambda: Q.schwinger_rate(ctx, c, rate))
    out["schwinger_rate"] = {"cells": n, "ms": ms, "cells_per_s": n / (ms * 1e-3),
                             "achieved_gbs": 56 * n / (ms * 1e-3) / 1e9}
    # cell volume 1e-28 m^3 and dt 1e-18 s: about 3e5 pairs from these fields
    el, po = Q.AppendBuffer(1 << 21, torch.float64), Q.AppendBuffer(1 << 21, torch.float64)

    def pairs():
        el.reset()
        po.reset()
        Q.schwinger_pairs(ctx, c, 1e-28, 1e-18, 1.0, 1, 0, el, po)
    ms = timed(pairs)
    out["schwinger_pairs"] = {"cells": n, "ms": ms, "cells_per_s": n / (ms * 1e-3), "pairs": int(el.count.item())}
    del d, c, rate
    m = 1 << 25
    um = 4120.0
    pe = {k: torch.zeros(m, dtype=torch.float64, device="cuda") for k in QI.FIELDS}
    pe["ux"].fill_(-um)
    pe["tau"] = torch.ones(m, dtype=torch.float64, device="cuda")
    x = torch.rand(m, generator=g, device="cuda", dtype=torch.float64) * 0.8e-6
    y, z = torch.zeros_like(x), torch.zeros_like(x)
    pp = Q.particles(pe, Q.ELECTRON, 0)
    f = Q.cp_wave(1.22e-4 * es, 0.8e-6, 1)
    ms = timed(lambda: Q.push(ctx, pp, x, y, z, f, 0.0, 3e-17))
    # read u and x, y, z; write u, x, y, z and the six field components
    out["push"] = {"particles": m, "ms": ms, "particles_per_s": m / (ms * 1e-3),
                   "achieved_gbs": 144 * m / (ms * 1e-3) / 1e9}
    # table generation on the device (FP64 quadrature), synchronous calls
    tg = {}
    for nn in (256, 512):
        for name, proc in (("bw", Q.BW), ("qs", Q.QS)):
            Q.Table.generate_device(proc, 1e-4, 1e3, nn, nn)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            Q.Table.generate_device(proc, 1e-4, 1e3, nn, nn)
            tg[f"{name}_{nn}x{nn}_ms"] = (time.perf_counter() - t0) * 1e3
    out["table_generation_device"] = tg
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--log2n", type=int, default=24, help="particles per species = 2^log2n")
    ap.add_argument("--dt", type=float, default=1e-16,
                    help="time step of the cone workload in s (1e-16: 31%% lepton events per step; "
                         "5.5e-18: about 1%% of all particles)")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--surrogate-steps", type=int, default=320000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-log2n", type=int, default=22,
                    help="the oracle is timed on the first 2^k particles of each species, whole steps, >= 10 s")
    ap.add_argument("--calibration-mib", type=int, default=0,
                    help="first stream this many MiB with the step's access patterns: non-temporal read, write "
                         "and copy passes, then temporal read and write passes (qed_traffic_calibrate modes 0-4), "
                         "so that HBM counters can be scaled for each")
    ap.add_argument("--workload", choices=("cone", "fullstep", "paper", "extras"), default="cone",
                    help="cone: the default roofline workload; fullstep: 4 species in lognormal tiles, "
                         "Gaussian pulse, FP32 table and FP32+surrogate paths; paper: the paper's own "
                         "benchmark of the four standalone calls")
    ap.add_argument("--paper-n", type=int, default=100_000_000, help="particles of the paper workload")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: this build has no multi-GPU path (asked for --gpus {args.gpus}).",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2110_00256_amd as Q
    import qed_inputs as QI

    if args.calibration_mib:
        nb = args.calibration_mib << 20
        src = torch.ones(nb // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for mode in (0, 1, 2, 3, 4):
            Q.traffic_calibrate(src, dst, nb, mode)
            torch.cuda.synchronize()
        log(f"bench: calibration passes of {args.calibration_mib} MiB done")
        del src, dst

    if args.workload == "fullstep":
        fullstep(Q, torch, QI, args)
        return
    if args.workload == "paper":
        paper(Q, torch, QI, args)
        return
    if args.workload == "extras":
        extras(Q, torch, QI, args)
        return

    n = 1 << args.log2n
    dt = args.dt
    chi_range = (1e-4, 1e3)
    log(f"bench: generating inputs 2^{args.log2n} leptons + 2^{args.log2n} photons")
    pops = QI.cone_population(seed=1, n=n)
    ctx = Q.Context(0)
    log("bench: generating 256x256 tables")
    tables = make_tables(Q, 256, 256, chi_range)
    log("bench: FP64 table path")
    r64 = run_path(Q, torch, ctx, tables, pops, "f64", args.steps, args.warmup, dt, Q.CHI_FP64)
    log(f"bench: FP64 {r64['updates_per_s']:.3e} upd/s, kernel {r64['kernel_ms_mean']:.3f} ms")
    r32 = None
    if not args.no_fp32:
        log("bench: FP32 table path")
        r32 = run_path(Q, torch, ctx, tables, pops, "f32", args.steps, args.warmup, dt, Q.CHI_FP64)
        log(f"bench: FP32 {r32['updates_per_s']:.3e} upd/s, kernel {r32['kernel_ms_mean']:.3f} ms")
    rs, train = None, None
    if not args.no_fp32 and not args.no_surrogate:
        log("bench: training BW and QS surrogates on the device (chi in [1e-3, 1e3])")
        t0 = time.perf_counter()
        sb, lb = Q.Surrogate.train(ctx, tables[0], Q.Surrogate.cfg(Q.BW, 1e-3, 1e3, n_samples=1 << 24,
                                                                   steps=args.surrogate_steps, tail_permille=500,
                                                                   ks_budget=SURR_KS_BUDGET))
        sq, lq = Q.Surrogate.train(ctx, tables[1], Q.Surrogate.cfg(Q.QS, 1e-3, 1e3, n_samples=1 << 24,
                                                                   steps=args.surrogate_steps, tail_permille=500,
                                                                   ks_budget=SURR_KS_BUDGET))
        served = {k: float(np.mean([(s.bands()[1] >> b) & 1 for b in range(64)])) for k, s in (("bw", sb), ("qs", sq))}
        train = {"seconds": time.perf_counter() - t0, "steps": args.surrogate_steps, "final_loss": {"bw": lb, "qs": lq},
                 "ks_budget": SURR_KS_BUDGET, "served_band_fraction": served}
        log("bench: FP32 + surrogate path")
        rs = run_path(Q, torch, ctx, tables, pops, "f32", args.steps, args.warmup, dt, Q.CHI_FP64,
                      surrogates=(sb, sq))
        log(f"bench: FP32+surrogate {rs['updates_per_s']:.3e} upd/s, kernel {rs['kernel_ms_mean']:.3f} ms")
    cpu = cpu1 = None
    if not args.no_cpu_baseline:
        m = 1 << args.cpu_sample_log2n
        small = tuple({k: v[:m] for k, v in p.items()} for p in pops)
        cpu = cpu_baseline(small, (256, 256, chi_range), dt)
        log(f"bench: oracle {cpu['value']:.3e} upd/s on {cpu['cores']} threads")
        m1 = m >> 4
        cpu1 = cpu_baseline_one_thread(tuple({k: v[:m1] for k, v in p.items()} for p in pops),
                                       (256, 256, chi_range), dt)
        log(f"bench: oracle {cpu1['value']:.3e} upd/s on {cpu1['cores']} thread")

    # the profile was taken on the default workload (2^24 + 2^24, dt 1e-16 s)
    traffic = measured_traffic() if (args.log2n == 24 and args.dt == 1e-16) else {}

    def traffic_gbs(key, r, kind="bytes_per_launch"):
        v = traffic.get(kind, {}).get(key)
        return v / (r["kernel_ms_mean"] * 1e-3) / 1e9 if v is not None else None

    out = {
        "metric": METRIC,
        "value": r64["updates_per_s"],
        "unit": "particle updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r64["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"cone plane wave: 2^{args.log2n} leptons + 2^{args.log2n} photons, 256x256 "
                               f"tables over chi [1e-4, 1e3], dt {dt:g} s, FP64 table path",
                   "particles": 2 * n, "dt_s": dt, "table": "256x256",
                   "qs_event_fraction": r64["qs_event_fraction"], "bw_event_fraction": r64["bw_event_fraction"]},
        "roofline": {"bound": "hbm", "achieved": r64["achieved_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": r64["achieved_gbs"] / HBM_PEAK_GBS, "traffic": traffic_gbs("f64", r64),
                     "kernel": "step_kernel<double>", "kernel_ms_mean": r64["kernel_ms_mean"],
                     "alg_bytes_per_launch": r64["alg_bytes_per_launch"],
                     "hbm_bytes_per_launch": traffic.get("bytes_per_launch", {}).get("f64"),
                     "traffic_fetch": traffic_gbs("f64", r64, "fetch_bytes_per_launch"),
                     "traffic_write": traffic_gbs("f64", r64, "write_bytes_per_launch"),
                     "alg_read_bytes_per_launch": r64["alg_read_bytes_per_launch"],
                     "alg_write_bytes_per_launch": r64["alg_write_bytes_per_launch"],
                     "traffic_calibration": traffic.get("calibration"), "kernel_digest": kernel_digest()},
        "cpu_baseline": cpu,
        "cpu_baseline_one_thread": cpu1,
    }
    if r32 is not None:
        out["fp32_table_path"] = {
            "value": r32["updates_per_s"], "ms_per_step": r32["ms_per_step"],
            "kernel_ms_mean": r32["kernel_ms_mean"], "achieved_gbs": r32["achieved_gbs"],
            "frac": r32["achieved_gbs"] / HBM_PEAK_GBS, "alg_bytes_per_launch": r32["alg_bytes_per_launch"],
            "qs_event_fraction": r32["qs_event_fraction"], "bw_event_fraction": r32["bw_event_fraction"],
            "speedup_vs_fp64": r32["updates_per_s"] / r64["updates_per_s"], "traffic": traffic_gbs("f32", r32)}
    if rs is not None:
        out["fp32_surrogate_path"] = {
            "value": rs["updates_per_s"], "ms_per_step": rs["ms_per_step"],
            "kernel_ms_mean": rs["kernel_ms_mean"], "achieved_gbs": rs["achieved_gbs"],
            "frac": rs["achieved_gbs"] / HBM_PEAK_GBS, "alg_bytes_per_launch": rs["alg_bytes_per_launch"],
            "speedup_vs_fp64": rs["updates_per_s"] / r64["updates_per_s"],
            "speedup_vs_fp32_table": rs["updates_per_s"] / r32["updates_per_s"],
            "surrogate_batches": rs["surrogate_batches"], "surrogate_fallbacks": rs["surrogate_fallbacks"],
            "training": train, "traffic": traffic_gbs("f32s", rs)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
