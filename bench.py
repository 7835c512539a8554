#!/usr/bin/env python3
"""Throughput of the SBS diffusion-reaction engine on one MI355X.

Workload: one 1 Gy pulse of 70 MeV-proton-like spur tracks (780 z-parallel
tracks, ~4e5 molecules of 7 species) in a 10 um periodic cube, evolved from
1 ps to 1 ms (3000 steps, log-spaced step end times), species counts recorded
at 100 log-spaced times.  One benchmark "step" is one whole run of that
workload: injection from device-resident arrays, every SBS step (jump + PBC,
cell binning, scan, scatter, pair search + Brownian bridge, matching,
products), records, and reading the counts and G-values back.

Metric: molecule-steps/s = sum over SBS steps of the live molecules / wall s.

Also printed: the roofline position of the dominant kernel (HIP events on the
engine's stream in a separate profiled run) and the FP64 CPU oracle timed on a
bounded sample of the same workload on this host.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
# Algorithmic HBM bytes per work unit of the streaming kernels (what the kernel
# must move at least once): per live molecule for k_bin / k_scatter, per bin
# for the scan.
ALG_BYTES = {
    "k_bin": 16 + 8 + 8,                          # read position+meta, uid; write (bin, rank)
    "k_scan": 4 + 4 + 4 + 4,                      # per bin: read count twice (reduce, apply); write start; clear count
    "k_scatter": 16 + 8 + 8 + 4 + 16 + 16 + 8,    # read pos, uid, (bin, rank), start; write pos, pos0, uid
    "k_pairs": 16 + 16 + 8,                       # read sorted end/start positions and uid once
}
# Algorithmic FP32 operations per candidate pair of the species-bin search
# (many molecules per cell, the arithmetic dominates): the minimum-image end
# separation (3 subtract, 3 multiply, 2 add).
ALG_FLOP_PER_CANDIDATE = 8


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-steps", type=int, default=40, help="SBS steps of the oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (5 times) to calibrate HBM counters")
    return ap.parse_args()


def kernels_hash():
    h = hashlib.sha256()
    for f in ("kernels.hip", "engine.h"):
        h.update(open(os.path.join(ROOT, "paper_2509_03313_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def cpu_baseline(wl, n_steps):
    """The FP64 oracle on the first n_steps SBS steps of the same workload,
    one host thread."""
    import numpy as np

    import oracle
    chem = oracle.make_chem(wl.D, wl.reactions)
    s = oracle.Instance(wl.L, 1000, 0)
    inj = wl.injections[0]
    s.inject(inj.xyz.astype(np.float64), inj.species.astype(np.int32), inj.edep_ev)
    sched = oracle.schedule(0.0, wl.t_end, [0.0], list(wl.records), wl.dt0, wl.ratio, oracle.dt_max(chem, wl.L))
    ms = 0
    t_prev = 0.0
    t0 = time.perf_counter()
    for k in range(min(n_steps, len(sched))):
        ms += s.n
        s.step(chem, sched[k] - t_prev)
        t_prev = sched[k]
    dt = time.perf_counter() - t0
    return dict(value=ms / dt, unit="molecule-steps/s", cores=1, kind="oracle",
                sample=f"first {min(n_steps, len(sched))} of {len(sched)} SBS steps of the same workload "
                       f"({ms} molecule-steps, {dt:.1f} s, 1 thread)")


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this engine runs on one GPU; --gpus {args.gpus} is not supported "
              "(instances shard across GPUs without communication, see DESIGN.md)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes_read": n * 4, "bytes_written": n * 4, "launches": 5}))
        return

    from paper_2509_03313_amd import gsbs
    from paper_2509_03313_amd import workload as W

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    dev = torch.device("cuda:0")
    wl = W.single_pulse_large(args.seed)
    inj = wl.injections[0]
    xyz_d = torch.from_numpy(np.ascontiguousarray(inj.xyz)).to(dev)
    sp_d = torch.from_numpy(np.ascontiguousarray(inj.species)).to(dev)
    cap = int(len(inj.species) * 1.5) + 4096

    def engine(tune):
        # warmup runs explore the search-grid configurations; timed runs use what they learned
        p = gsbs.gsbs_default_params()
        p.autotune = 1 if tune else 0
        return gsbs.Engine(wl.L, 1000, W.D_CONFIG, W.REACTIONS, params=p, capacity=cap)

    def run(e):
        e.inject(0, 0.0, xyz_d, sp_d, inj.edep_ev)
        e.set_records(0, wl.records)
        e.advance_to(wl.t_end)
        return e.counts(0), e.gvalues(0)

    def note(*a):
        print("[bench]", *a, file=sys.stderr, flush=True)

    for k in range(args.warmup):
        e = engine(True)
        t = time.perf_counter()
        run(e)
        note(f"warmup {k}: {time.perf_counter() - t:.2f} s, stats {e.stats()}")
        e.close()
    engines = [engine(False) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for e in engines:
        run(e)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    note(f"timed {args.steps} runs: {wall:.2f} s")
    stats = [e.stats() for e in engines]
    msteps = sum(s["molecule_steps"] for s in stats)
    sbs_steps = stats[0]["steps"]
    counts, gv = engines[-1].counts(0), engines[-1].gvalues(0)
    for e in engines:
        e.close()
    value = msteps / wall

    roofline = None
    prof = None
    if not args.no_profile:
        e = engine(False)
        gsbs.gsbs_set_profiling(e.ctx, True)
        run(e)
        prof = gsbs.gsbs_get_profile(e.ctx)
        pst = e.stats()
        note(f"profile: {prof}")
        e.close()
        dom = max(prof, key=lambda k: prof[k][0])
        tot_ms, launches, work, cand = prof[dom]
        avg_s = tot_ms / 1e3 / max(launches, 1)
        if dom in ALG_BYTES:
            ach = ALG_BYTES[dom] * work / (tot_ms / 1e3) / 1e9
            roofline = dict(bound="hbm", achieved=round(ach, 2), peak=HBM_PEAK_GBS, unit="GB/s",
                            frac=round(ach / HBM_PEAK_GBS, 5), traffic=None, kernel=dom,
                            avg_launch_us=round(avg_s * 1e6, 3), alg_bytes_per_unit=ALG_BYTES[dom],
                            units_per_launch=round(work / max(launches, 1), 1))
        elif dom == "k_pairs_sp":
            ach = ALG_FLOP_PER_CANDIDATE * cand / (tot_ms / 1e3) / 1e12
            roofline = dict(bound="alu", achieved=round(ach, 4), peak=FP32_PEAK_TFLOPS, unit="TFLOP/s",
                            frac=round(ach / FP32_PEAK_TFLOPS, 6), traffic=None, kernel=dom,
                            avg_launch_us=round(avg_s * 1e6, 3), alg_flop_per_candidate=ALG_FLOP_PER_CANDIDATE,
                            candidates_per_launch=round(cand / max(launches, 1), 1))
        else:
            roofline = dict(bound="latency", achieved=None, peak=None, unit=None, frac=None, traffic=None,
                            kernel=dom, avg_launch_us=round(avg_s * 1e6, 3))
        tr = os.path.join(ROOT, "profiles", "traffic.json")
        if os.path.exists(tr):
            t = json.load(open(tr))
            if t.get("kernels_hash") == kernels_hash() and dom in t.get("per_launch_bytes", {}):
                roofline["traffic"] = t["per_launch_bytes"][dom]

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(wl, args.cpu_steps)
        note(f"cpu baseline: {cpu}")

    line = {
        "metric": "molecule-steps/s of SBS diffusion-reaction",
        "value": round(value, 1),
        "unit": "molecule-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "single pulse, 1 Gy, 10 um periodic cube, ~4e5 molecules, 1 ps -> 1 ms",
                   "molecules": int(len(inj.species)), "sbs_steps": int(sbs_steps), "L_nm": wl.L,
                   "species": 7, "reactions": 9},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "profile_ms": {k: round(v[0], 3) for k, v in prof.items()} if prof else None,
        "profile_work": {k: v[2] for k, v in prof.items()} if prof else None,
        "profile_launches": {k: v[1] for k, v in prof.items()} if prof else None,
        "profile_candidates": {k: v[3] for k, v in prof.items() if v[3]} if prof else None,
        "tuning": gsbs.gsbs_get_tuning(),
        "final_counts": counts[-1].tolist(),
        "G_H2O2_end": float(gv[-1][W.H2O2]),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
