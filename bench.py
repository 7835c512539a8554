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
    "k_bin": 16 + 8 + 8 + 16,                     # read position+meta, uid; write (bin, rank), moved position
    "k_scan": 4 + 4 + 4,                          # per bin: read count; write start; clear count
    "k_scatter": 8 + 16 + 16 + 8 + 4 + 16 + 16 + 8,  # read (bin, rank), moved and start position, uid, start;
                                                  # write pos, pos0, uid
    "k_pairs": 16 + 16 + 8,                       # read sorted end/start positions and uid once
}
# Algorithmic FP32 operations per candidate pair of the species-bin search
# (many molecules per cell, the arithmetic dominates): the minimum-image end
# separation (3 subtract, 3 multiply, 2 add), the same for the start
# separation, and the bridge exponent bound (r0 - R)(r1 - R) / s (2 subtract,
# 2 multiply) that decides whether the pair is evaluated.
ALG_FLOP_PER_CANDIDATE = 20


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20,
                    help="timed benchmark steps (campaign: --chunk SBS steps each; single pulse: whole runs)")
    ap.add_argument("--warmup", type=int, default=5, help="untimed steps before (the autotuner explores in them)")
    ap.add_argument("--chunk", type=int, default=1000, help="campaign: global SBS steps per benchmark step")
    ap.add_argument("--search-split", type=int, default=0,
                    help="species-bin search: partner-stream slices per box (0: chosen by the library)")
    ap.add_argument("--step-graph", type=int, default=-1, help="1/0: HIP step graphs on/off (-1: library default)")
    ap.add_argument("--live", choices=("dominant", "all"), default="all",
                    help="campaign: time the warmup's dominant kernel or every step kernel with HIP events")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--instances", type=int, default=64, help="cubes of the batched campaign")
    ap.add_argument("--budget", type=int, default=20000, help="SBS steps per campaign instance at most")
    ap.add_argument("--single-pulse", action="store_true",
                    help="one 1 Gy pulse in a 10 um cube, 1 ps -> 1 ms, instead of the batched campaign")
    ap.add_argument("--cpu-steps", type=int, default=None,
                    help="SBS steps of the oracle sample (default 80 for the single pulse, 600 for the campaign)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (5 times) to calibrate HBM counters")
    ap.add_argument("--batched", type=int, default=0, metavar="N",
                    help="the batched metric: N independent instances of uneven size stepped together")
    ap.add_argument("--batched-t-end", type=float, default=100.0, help="end time (ns) of the batched runs")
    ap.add_argument("--numodes", type=int, default=0, metavar="N",
                    help="the rate equations: N batched mixtures, then 20-pulse SBS + rate-equation runs")
    ap.add_argument("--volume-scaling", action="store_true",
                    help="SBS + PBCs, Gillespie runs and the rate equations of one homogeneous mixture in "
                         "0.2, 0.5 and 1 um cubes")
    ap.add_argument("--ssa-realisations", type=int, default=4096, help="Gillespie runs per cube edge")
    ap.add_argument("--ssa-throughput", type=int, default=524288, metavar="N",
                    help="Gillespie runs of the 0.5 um volume-scaling cube timed for the event rate")
    ap.add_argument("--dose-rate", action="store_true",
                    help="the paper's dose-rate study: 1 us pulse trains at 2e5 and 1e6 Gy/s to 20 Gy, "
                         "average dose rates 0.01-1e5 Gy/s, 2 um cube, SBS + rate equations")
    ap.add_argument("--dose-rate-seeds", type=int, default=3, help="pulse trains per grid point")
    ap.add_argument("--ph7", action="store_true", help="dose-rate study in pH 7 water (background ions and "
                                                        "R9's reverse in the rate equations)")
    ap.add_argument("--o2", action="store_true", help="dose-rate study in aerated water (O2 scavenging of e_aq "
                                                      "and H, superoxide reactions)")
    ap.add_argument("--surrogate", action="store_true",
                    help="the second metric: 20-pulse wall time with the inter-pulse network vs plain SBS")
    ap.add_argument("--sur-L", type=float, default=10000.0, help="cube edge (nm) of the held-out and 20-pulse runs")
    ap.add_argument("--sur-train-L", type=float, default=5000.0, help="cube edge (nm) of the training runs")
    ap.add_argument("--sur-plans", type=str, default="3456,384", help="training runs, one count per set")
    ap.add_argument("--sur-pulses", type=str, default="4,10", help="pulses per training and held-out run, one per set")
    ap.add_argument("--sur-held", type=str, default="96,32", help="held-out runs for the error table, one per set")
    ap.add_argument("--mlp", action="store_true", help="throughput of the surrogate network's kernels")
    ap.add_argument("--no-extra-configs", action="store_true",
                    help="campaign: skip the single-cube 1-pulse and 20-pulse runs reported beside it")
    ap.add_argument("--mlp-batches", type=str, default="1024,16384,131072", help="--mlp: batch sizes")
    ap.add_argument("--mlp-iters", type=int, default=50, help="--mlp: timed iterations per batch size")
    ap.add_argument("--sur-eval-pulses", type=int, default=10, help="pulses of the plain / hybrid comparison runs")
    ap.add_argument("--sur-rate-range", type=str, default="1,3000", help="average dose rates (Gy/s) of the "
                                                                          "training runs, log-uniform")
    ap.add_argument("--sur-cap", type=float, default=5e7, help="training intervals are simulated at most this long "
                                                              "(ns) after the hand-over")
    ap.add_argument("--sur-rates", type=str, default="1000,100,10,1",
                    help="average dose rates (Gy/s) of the 20-pulse runs")
    ap.add_argument("--sur-save", type=str, default="", help="path prefix to save the model, held-out set and runs")
    ap.add_argument("--sur-lean", action="store_true",
                    help="no warm-up and no budget run; the hybrid run first (for long intervals)")
    ap.add_argument("--sur-load", type=str, default="", help="saved network (Surrogate.save): skip generating and training")
    ap.add_argument("--sur-data", type=str, default="",
                    help="npz of the training and held-out samples: read if it exists, else written after generating")
    ap.add_argument("--sur-generate-only", action="store_true", help="stop after generating (and saving) the samples")
    ap.add_argument("--sur-batch", type=str, default="512",
                    help="training runs stepped together in one context, one per set (the last repeats)")
    return ap.parse_args()


def surrogate_bench(args):
    """Train the inter-pulse network on SBS runs of the engine itself, then run
    --sur-eval-pulses pulses of 1 Gy with and without it on the same pulses and
    seeds."""
    import numpy as np
    import torch

    from paper_2509_03313_amd import surrogate as SU

    def note(*a):
        print("[bench]", *a, file=sys.stderr, flush=True)

    if args.sur_load:
        s = SU.Surrogate(1024)
        s.load(args.sur_load)
        note(f"network, normalisation and table read from {args.sur_load}")
        line_train = {"model": os.path.basename(args.sur_load)}
    else:
        t0 = time.perf_counter()
        rates = tuple(float(r) for r in args.sur_rate_range.split(","))
        doses = (0.7, 1.3)
        ints = lambda v: [int(x) for x in str(v).split(",") if x]  # noqa: E731
        pulses, n_plans, held_runs = ints(args.sur_pulses), ints(args.sur_plans), ints(args.sur_held)
        bsz_list = ints(args.sur_batch)
        bsz_of = lambda k: bsz_list[min(k, len(bsz_list) - 1)]  # noqa: E731
        if not (len(pulses) == len(n_plans) == len(held_runs)):
            raise SystemExit("--sur-pulses, --sur-plans and --sur-held take lists of one length")
        # sets of training runs in the small cube and held-out runs in the large one (its
        # count noise, ~0.5 % of the H2O2 made per pulse, is small enough for the 1 % table
        # to mean something), one per pulse count
        jobs = []
        for k, (npl, nh, npu) in enumerate(zip(n_plans, held_runs, pulses)):
            jobs.append(("train", SU.random_plans(args.seed + 1 + 10 * k, npl, L=args.sur_train_L, n_pulses=npu,
                                                  rates=rates, doses=doses), bsz_of(k), 1000 + 100000 * k, k, npu))
            jobs.append(("held", SU.random_plans(args.seed + 2 + 10 * k, nh, L=args.sur_L, n_pulses=npu, rates=rates,
                                                 doses=doses), 32, 2000 + 100000 * k, k, npu))
        n_train_runs = sum(n_plans)
        sets = {"train": {}, "held": {}}
        for name, pl_all, bsz, seed0, k, npu in jobs:
            dst = sets[name]
            for b0 in range(0, len(pl_all), bsz):
                # with --sur-data every batch is kept in a file of its own, so that a
                # generation split over several runs resumes where it stopped
                tag = f"{name}{b0}_{bsz}" + (f"_s{k}p{npu}" if k else "")
                part = f"{args.sur_data}.{tag}.npz" if args.sur_data else ""
                if part and os.path.exists(part):
                    z = np.load(part)
                    d = {q: z[q] for q in z.files}
                else:
                    d = SU.generate(pl_all[b0:b0 + bsz], seed=seed0 + b0, t_cap=args.sur_cap, log=note)
                    if part:
                        np.savez(part, **d)
                for q, v in d.items():
                    dst[q] = np.concatenate([dst[q], v]) if q in dst else v
                note(f"{name} samples {len(dst['X'])} after {time.perf_counter() - t0:.1f} s")
        train, held = sets["train"], sets["held"]
        t_gen = time.perf_counter() - t0
        if args.sur_data:
            np.savez(args.sur_data, **{"train_" + q: v for q, v in train.items()},
                     **{"held_" + q: v for q, v in held.items()})
        if args.sur_generate_only:
            note(f"generated {len(train['X'])} training and {len(held['X'])} held-out samples in {t_gen:.1f} s")
            return
        n, n_held = len(train["X"]), len(held["X"])
        # two candidates, with and without the pair-correlation inputs; one half of the
        # held-out samples picks the candidate, the other half fills its error table
        hperm = np.random.default_rng(args.seed + 3).permutation(n_held)
        sub = lambda d, k: {key: v[k] for key, v in d.items()}  # noqa: E731
        pick, tab = sub(held, hperm[: n_held // 2]), sub(held, hperm[n_held // 2:])
        t1 = time.perf_counter()
        cands = {}
        for gw in (1.0, 0.0):
            c = SU.Surrogate(1024)
            c.init_weights(args.seed)
            hist = c.fit(train, epochs=60, batch=64, lr=5e-4, log=note, g_weight=gw)
            e = c.build_table(pick, n_dt=3, n_c=2)
            cands[gw] = (float(np.quantile(e, 0.95)), float(np.median(e)), c, hist)
            note(f"pair-correlation weight {gw:g}: held-out relative H2O2 error median {np.median(e):.4f}, "
                 f"p95 {np.quantile(e, 0.95):.4f}")
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t1
        gw_best = min(cands, key=lambda k: cands[k][0])
        s, hist = cands[gw_best][2], cands[gw_best][3]
        # the half that picked the candidate also gives its mean residual; the table half
        # then measures the calibrated network
        bias = s.calibrate(pick)
        note(f"calibration: mean log10 residual per species {np.round(bias, 5).tolist()}")
        err = s.build_table(tab, n_dt=3, n_c=2)
        if args.sur_save:
            s.save(args.sur_save + "_model.npz")
            np.savez(args.sur_save + "_held.npz", **held)
        note(f"chosen weight {gw_best:g}; table half: median {np.median(err):.4f}, p95 {np.quantile(err, 0.95):.4f}; "
             f"table {np.round(s.table, 4).tolist()} over log10 dt edges {np.round(s.dt_edges, 2).tolist()}, "
             f"log10 C_tot edges {np.round(s.c_edges, 2).tolist()}")
        line_train = {
            "config": {"train_runs": n_plans, "train_L_nm": args.sur_train_L, "train_pulses_per_run": pulses,
                       "train_avg_rates_gy_s": list(rates), "train_interval_cap_ns": args.sur_cap, "samples": int(n),
                       "held_out_runs": held_runs, "held_out": int(n_held)},
            "generate_s": round(t_gen, 1), "train_s": round(t_train, 2), "final_loss": round(hist[-1], 6),
            "pair_correlation_weight": gw_best, "calibration_log10_bias": [round(float(b), 6) for b in bias],
            "held_out_h2o2_rel_err_p95_by_weight": {str(k): round(v[0], 5) for k, v in cands.items()},
            "held_out_h2o2_rel_err_median": round(float(np.median(err)), 5),
            "held_out_h2o2_rel_err_p95": round(float(np.quantile(err, 0.95)), 5)}
    note(f"table {np.round(s.table, 4).tolist()}")
    runs = []
    for rate in [float(r) for r in args.sur_rates.split(",") if r]:
        plan = SU.PulsePlan(args.sur_L, args.seed + 77, args.sur_eval_pulses, 1.0, 1e6, rate)
        if args.sur_lean:
            # long intervals: the hybrid run goes first and warms the grid tuner for the
            # plain run (its own time includes the exploration); no budget run
            hyb = SU.run(plan, s, log=note)
            plain = SU.run(plan, None, log=note)
            hyb_b = hyb
        else:
            note(f"rate {rate:g}: warming the grid tuner")
            SU.run(SU.PulsePlan(args.sur_L, 5, 2, 1.0, 1e6, rate), None, log=note)
            plain = SU.run(plan, None, log=note)
            hyb = SU.run(plan, s, log=note)
            # the same with the run's summed error estimate held within the 1 % bar
            hyb_b = SU.run(plan, s, budget=0.01, log=note)
        rel = np.abs(hyb["g_h2o2"] - plain["g_h2o2"]) / plain["g_h2o2"]
        rel_b = np.abs(hyb_b["g_h2o2"] - plain["g_h2o2"]) / plain["g_h2o2"]
        note(f"network intervals {np.nonzero(hyb['used'])[0].tolist()}; H2O2 at pulse starts plain "
             f"{plain['n_h2o2'].tolist()} hybrid {hyb['n_h2o2'].tolist()}")
        if args.sur_save:
            np.savez(args.sur_save + f"_runs_{rate:g}.npz", **{"plain_" + k: v for k, v in plain.items()},
                     **{"hyb_" + k: v for k, v in hyb.items()})
        note(f"rate {rate:g}: plain {plain['wall']:.2f} s, hybrid {hyb['wall']:.2f} s, network intervals "
             f"{hyb['intervals_by_network']}/{args.sur_eval_pulses - 1}, max |dG(H2O2)|/G {rel.max():.4f}, end {rel[-1]:.4f}; "
             f"with the 1 % budget {hyb_b['wall']:.2f} s, {hyb_b['intervals_by_network']}/{args.sur_eval_pulses - 1} intervals, "
             f"max {rel_b.max():.4f}")
        runs.append(dict(avg_rate_gy_s=rate, wall_plain_s=round(plain["wall"], 3), wall_hybrid_s=round(hyb["wall"], 3),
                         speedup=round(plain["wall"] / hyb["wall"], 3), intervals_by_network=hyb["intervals_by_network"],
                         g_h2o2_plain=[round(float(x), 5) for x in plain["g_h2o2"]],
                         g_h2o2_hybrid=[round(float(x), 5) for x in hyb["g_h2o2"]],
                         max_rel_dG_h2o2=round(float(rel.max()), 5), end_rel_dG_h2o2=round(float(rel[-1]), 5),
                         steps_plain=plain["steps"], steps_hybrid=hyb["steps"],
                         budget_1pct=dict(wall_hybrid_s=round(hyb_b["wall"], 3),
                                          speedup=round(plain["wall"] / hyb_b["wall"], 3),
                                          intervals_by_network=hyb_b["intervals_by_network"],
                                          error_estimate_spent=round(hyb_b["error_estimate_spent"], 5),
                                          max_rel_dG_h2o2=round(float(rel_b.max()), 5),
                                          end_rel_dG_h2o2=round(float(rel_b[-1]), 5))))
        if args.sur_save:  # each rate as it ends
            with open(args.sur_save + "_runs.jsonl", "a") as f:
                f.write(json.dumps(runs[-1]) + "\n")
    line = {
        "metric": f"{args.sur_eval_pulses}-pulse wall time, plain SBS / SBS with the inter-pulse network",
        "value": runs[0]["speedup"] if runs else None, "unit": "x", "higher_is_better": True, "n_gpus": 1,
        "dtype": "f32 SBS, bf16 network with f32 accumulation", "data": "synthetic",
        "config": {"workload": f"{args.sur_eval_pulses} pulses x 1 Gy, {args.sur_L:g} nm periodic cube, pulse rate "
                               f"1e6 Gy/s, 2 batches per pulse"},
        "train": line_train,
        "runs": runs,
    }
    print(json.dumps(line), flush=True)


def kernels_hash():
    h = hashlib.sha256()
    for f in ("kernels.hip", "engine.h", "device_common.h"):
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


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def measured_traffic(workload, kernel):
    """HBM bytes per launch of a kernel on a workload, from the scaled
    FETCH_SIZE + WRITE_SIZE counters in profiles/traffic.json; None when the
    file has no such entry or was taken on other kernel sources."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    t = json.load(open(TRAFFIC_FILE))
    if t.get("kernels_hash") != kernels_hash():
        return None
    return t.get("workloads", {}).get(workload, {}).get("per_launch_bytes", {}).get(kernel)


def add_traffic(r, workload):
    """Counter bytes per launch of the roofline's kernel, and the HBM rate they
    give over its measured mean launch time (with its fraction of peak)."""
    t = measured_traffic(workload, r["kernel"])
    r["traffic"] = t
    if t and r.get("avg_launch_us"):
        gbs = t / (r["avg_launch_us"] * 1e-6) / 1e9
        r["traffic_gbs"] = round(gbs, 1)
        r["traffic_frac"] = round(gbs / HBM_PEAK_GBS, 5)
    return r


def roofline_of(prof, kernel=None, workload=None):
    """Roofline object of one kernel of a profile (by default the one with the
    most time): HBM for the streaming kernels, FP32 vector for the species-bin
    search."""
    dom = kernel or max(prof, key=lambda k: prof[k][0])
    tot_ms, launches, work, cand = prof[dom]
    avg_s = tot_ms / 1e3 / max(launches, 1)
    if dom in ALG_BYTES:
        ach = ALG_BYTES[dom] * work / (tot_ms / 1e3) / 1e9
        r = dict(bound="hbm", achieved=round(ach, 2), peak=HBM_PEAK_GBS, unit="GB/s",
                 frac=round(ach / HBM_PEAK_GBS, 5), traffic=None, kernel=dom,
                 avg_launch_us=round(avg_s * 1e6, 3), alg_bytes_per_unit=ALG_BYTES[dom],
                 units_per_launch=round(work / max(launches, 1), 1))
    elif dom == "k_pairs_sp":
        ach = ALG_FLOP_PER_CANDIDATE * cand / (tot_ms / 1e3) / 1e12
        r = dict(bound="alu", achieved=round(ach, 4), peak=FP32_PEAK_TFLOPS, unit="TFLOP/s",
                 frac=round(ach / FP32_PEAK_TFLOPS, 6), traffic=None, kernel=dom,
                 avg_launch_us=round(avg_s * 1e6, 3), alg_flop_per_candidate=ALG_FLOP_PER_CANDIDATE,
                 candidates_per_launch=round(cand / max(launches, 1), 1))
    else:
        r = dict(bound="latency", achieved=None, peak=None, unit=None, frac=None, traffic=None,
                 kernel=dom, avg_launch_us=round(avg_s * 1e6, 3))
    if workload:
        add_traffic(r, workload)
    return r


def batched_bench(args):
    """Batched instances: the first pulse of 64 independent cubes of uneven size
    (edges 2-10 um, 0.1-2 Gy) stepped together from 1 ps to --batched-t-end."""
    import numpy as np
    import torch

    from paper_2509_03313_amd import gsbs
    from paper_2509_03313_amd import workload as W

    def note(*a):
        print("[bench]", *a, file=sys.stderr, flush=True)

    insts = W.batched_first_pulses(args.seed, args.batched)
    Ls = [L for L, _ in insts]
    caps = [int(len(j.species) * 1.5) + 4096 for _, j in insts]
    dev = [(torch.from_numpy(np.ascontiguousarray(j.xyz)).cuda(), torch.from_numpy(np.ascontiguousarray(j.species)).cuda())
           for _, j in insts]
    n_mol = sum(len(j.species) for _, j in insts)
    t_end = args.batched_t_end
    rec = np.concatenate([[0.0], W.log_times(W.DT0_NS, t_end, 20)])
    rec[-1] = t_end
    note(f"{len(insts)} instances, {n_mol} molecules, to {t_end:g} ns")

    def engine(tune):
        p = gsbs.gsbs_default_params()
        p.autotune = 1 if tune else 0
        return gsbs.Engine(Ls, 1000, W.D_CONFIG, W.REACTIONS, params=p, capacity=caps)

    def run(e):
        for i, (_, j) in enumerate(insts):
            e.inject(i, 0.0, dev[i][0], dev[i][1], j.edep_ev)
            e.set_records(i, rec)
        e.advance_to([t_end] * len(insts))

    for k in range(args.warmup):
        e = engine(True)
        t = time.perf_counter()
        run(e)
        torch.cuda.synchronize()
        note(f"warmup {k}: {time.perf_counter() - t:.2f} s, stats {e.stats()}")
        e.close()
    engines = [engine(False) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for e in engines:
        run(e)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stats = [e.stats() for e in engines]
    for e in engines:
        e.close()
    msteps = sum(s_["molecule_steps"] for s_ in stats)
    note(f"timed {args.steps} runs: {wall:.2f} s")
    e = engine(False)
    gsbs.gsbs_set_profiling(e.ctx, True)
    run(e)
    prof = gsbs.gsbs_get_profile(e.ctx)
    e.close()
    note(f"profile: {prof}")
    line = {
        "metric": "molecule-steps/s of SBS diffusion-reaction, batched instances",
        "value": round(msteps / wall, 1), "unit": "molecule-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(wall / args.steps * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{len(insts)} batched instances (edges 2-10 um, first pulse of 0.1-2 Gy), "
                               f"1 ps -> {t_end:g} ns", "instances": len(insts), "molecules": n_mol,
                   "sbs_steps": stats[0]["steps"]},
        "roofline": roofline_of(prof),
        "roofline_streaming": {k: roofline_of(prof, k) for k in ("k_bin", "k_scatter") if k in prof},
        "profile_ms": {k: round(v[0], 3) for k, v in prof.items()},
        "profile_launches": {k: v[1] for k, v in prof.items()},
    }
    print(json.dumps(line), flush=True)


# Algorithmic FP64 operations of one accepted step of the rate-equation integrator
# (four-stage Rosenbrock) for the 7-species, 9-reaction scheme: three right-hand
# sides (~63 each), the Jacobian (~108), the stage matrix (~50), the 7 x 7 LU
# (203), four triangular solve pairs (91 each), stage and error vectors (~126).
ALG_FLOP_PER_ODE_STEP = 1040
FP64_PEAK_TFLOPS = 78.6


def numodes_bench(args):
    """The rate equations of the beam-off stage: batched throughput on the
    device, and 20-pulse runs alternating SBS with them (the paper's scheme)
    against plain SBS on the same pulses and seeds."""
    import numpy as np
    import torch

    from paper_2509_03313_amd import gsbs
    from paper_2509_03313_amd import surrogate as SU
    from paper_2509_03313_amd import workload as W

    def note(*a):
        print("[bench]", *a, file=sys.stderr, flush=True)

    rng = np.random.default_rng(args.seed + 9)
    n = args.numodes
    c0 = torch.as_tensor(10.0 ** rng.uniform(-8, -5, size=(n, 7)), device="cuda")
    dt = torch.full((n,), 1e6, dtype=torch.float64, device="cuda")
    e = gsbs.Engine(1000.0, 1, W.D_CONFIG, W.REACTIONS)
    gsbs.gsbs_numodes(e.ctx, c0[:64], dt[:64])  # warm
    torch.cuda.synchronize()
    # HIP events on the engine's stream (torch's current stream) around the call:
    # the launch plus the copy-back of the step counts
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    c1, steps = gsbs.gsbs_numodes(e.ctx, c0, dt, rtol=1e-6)
    ev1.record()
    ev1.synchronize()
    wall_host = time.perf_counter() - t0
    wall_ode = ev0.elapsed_time(ev1) / 1e3
    note(f"event time {wall_ode * 1e3:.2f} ms, host time {wall_host * 1e3:.2f} ms")
    e.close()
    tot_steps = int(np.sum(steps))
    ach = ALG_FLOP_PER_ODE_STEP * tot_steps / wall_ode / 1e12
    note(f"{n} mixtures over 1 ms: {wall_ode * 1e3:.1f} ms, {tot_steps} steps ({np.mean(steps):.0f} per mixture)")
    runs = []
    for rate in [float(r) for r in args.sur_rates.split(",") if r]:
        plan = SU.PulsePlan(args.sur_L, args.seed + 77, 20, 1.0, 1e6, rate)
        SU.run(SU.PulsePlan(args.sur_L, 5, 2, 1.0, 1e6, rate), None)  # warm the grid tuner
        plain = SU.run(plan, None)
        hyb = SU.run(plan, None, numodes_rtol=1e-6)
        rel = np.abs(hyb["g_h2o2"] - plain["g_h2o2"]) / plain["g_h2o2"]
        note(f"rate {rate:g}: plain {plain['wall']:.2f} s, SBS + rate equations {hyb['wall']:.2f} s, "
             f"max |dG(H2O2)|/G {rel.max():.4f}, end {rel[-1]:.4f}")
        runs.append(dict(avg_rate_gy_s=rate, wall_plain_s=round(plain["wall"], 3), wall_numodes_s=round(hyb["wall"], 3),
                         speedup=round(plain["wall"] / hyb["wall"], 3),
                         g_h2o2_plain=[round(float(x), 5) for x in plain["g_h2o2"]],
                         g_h2o2_numodes=[round(float(x), 5) for x in hyb["g_h2o2"]],
                         max_rel_dG_h2o2=round(float(rel.max()), 5), end_rel_dG_h2o2=round(float(rel[-1]), 5)))
    line = {
        "metric": "20-pulse wall time, plain SBS / SBS with the rate equations between pulses",
        "value": runs[0]["speedup"] if runs else None, "unit": "x", "higher_is_better": True, "n_gpus": 1,
        "dtype": "f32 SBS, f64 rate equations", "data": "synthetic",
        "config": {"workload": f"20 pulses x 1 Gy, {args.sur_L:g} nm periodic cube, pulse rate 1e6 Gy/s, "
                               f"2 batches per pulse; rate equations at rtol 1e-6"},
        "batched_rate_equations": {"mixtures": n, "interval_ns": 1e6, "wall_ms": round(wall_ode * 1e3, 3),
                                   "mixtures_per_s": round(n / wall_ode, 1), "steps": tot_steps,
                                   "roofline": dict(bound="alu", achieved=round(ach, 4), peak=FP64_PEAK_TFLOPS,
                                                    unit="TFLOP/s", frac=round(ach / FP64_PEAK_TFLOPS, 5),
                                                    kernel="k_numodes", alg_flop_per_step=ALG_FLOP_PER_ODE_STEP)},
        "runs": runs,
    }
    print(json.dumps(line), flush=True)


# Algorithmic FP64 operations of one Gillespie event of the 9-reaction scheme:
# nine propensities (pair count and product, ~3 each), their sum (9), the
# running sum of the choice (~5 on average), the waiting time (ln ~20, a
# division and an add) and the uniforms (4).
ALG_FLOP_PER_SSA_EVENT = 70


def volume_scaling_bench(args):
    """The paper's volume-scaling check: one homogeneous mixture in cubes of
    0.2, 0.5 and 1 um; SBS + PBCs (several cubes per edge), Gillespie runs in
    the same volumes and the rate equations, compared species by species."""
    import numpy as np
    import torch

    from paper_2509_03313_amd import gsbs
    from paper_2509_03313_amd import workload as W

    def note(*a):
        print("[bench]", *a, file=sys.stderr, flush=True)

    NA = 6.02214076e23
    t_end = 1e4
    rec = np.concatenate([[0.0], W.log_times(1e-3, t_end, 40)])
    rec[-1] = t_end
    n_sbs = {200.0: 32, 500.0: 8, 1000.0: 2}
    out = []
    for L in W.VOLUME_SCALING_EDGES_NM:
        V = L ** 3 * 1e-24  # nm^3 -> litres
        n0 = W.volume_scaling_counts(L)
        # SBS + PBCs: independent cubes stepped together
        k = n_sbs[L]
        wls = [W.volume_scaling(args.seed * 100 + i, L, t_end=t_end) for i in range(k)]
        e = gsbs.Engine([L] * k, args.seed + 7, W.D_CONFIG, W.REACTIONS)
        for i, wl in enumerate(wls):
            e.inject(i, 0.0, wl.injections[0].xyz, wl.injections[0].species)
            e.set_records(i, rec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e.advance_to(t_end)
        torch.cuda.synchronize()
        wall_sbs = time.perf_counter() - t0
        msteps = e.stats()["molecule_steps"]
        sbs = np.stack([e.counts(i) for i in range(k)]).astype(np.float64)
        e.close()
        # Gillespie runs in the same volume
        e = gsbs.Engine(L, 1, W.D_CONFIG, W.REACTIONS)
        n_r = args.ssa_realisations
        n0d = torch.as_tensor(np.tile(n0.astype(np.int32), (n_r, 1)), device="cuda")
        vol = torch.full((n_r,), V, dtype=torch.float64, device="cuda")
        gsbs.gsbs_ssa(e.ctx, n0d[:64], vol[:64], rec, seed=args.seed)  # warm
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ssa_d, ev = gsbs.gsbs_ssa(e.ctx, n0d, vol, rec, seed=args.seed + 1)
        wall_ssa = time.perf_counter() - t0
        ssa = ssa_d.cpu().numpy().astype(np.float64)
        # the rate equations from the same start, to every record time
        c0 = np.tile(n0 / (NA * V), (len(rec), 1))
        t0 = time.perf_counter()
        ode, _ = gsbs.gsbs_numodes(e.ctx, c0, rec, rtol=1e-8)
        wall_ode = time.perf_counter() - t0
        e.close()
        ode *= NA * V
        m_sbs, m_ssa = sbs.mean(axis=0), ssa.mean(axis=0)
        row = dict(L_nm=L, molecules=int(n0.sum()), sbs_cubes=k, ssa_realisations=n_r,
                   wall_sbs_s=round(wall_sbs, 3), wall_ssa_s=round(wall_ssa, 4), wall_ode_s=round(wall_ode, 4),
                   sbs_molecule_steps=int(msteps), ssa_events=int(ev.sum()), species={})
        for sp in range(7):
            ok = m_ssa[:, sp] >= 20
            if not ok.any():
                continue
            r_ode = ode[ok, sp] / m_ssa[ok, sp]
            r_sbs = m_sbs[ok, sp] / m_ssa[ok, sp]
            row["species"][W.SPECIES[sp]] = dict(
                max_abs_ode_over_ssa_minus_1=round(float(np.max(np.abs(r_ode - 1))), 5),
                sbs_over_ssa_min=round(float(r_sbs.min()), 4), sbs_over_ssa_max=round(float(r_sbs.max()), 4),
                sbs_over_ssa_end=round(float(r_sbs[-1]), 4))
        note(f"L {L:g} nm: {n0.sum()} molecules; SBS {k} cubes {wall_sbs:.2f} s, Gillespie {n_r} runs "
             f"{wall_ssa * 1e3:.1f} ms ({ev.sum()} events), rate equations {wall_ode * 1e3:.1f} ms")
        for name, v in row["species"].items():
            note(f"   {name:5s} |ODE/SSA-1| max {v['max_abs_ode_over_ssa_minus_1']:.4f}   SBS/SSA "
                 f"{v['sbs_over_ssa_min']:.3f}..{v['sbs_over_ssa_max']:.3f} (end {v['sbs_over_ssa_end']:.3f})")
        out.append(row)
    # event rate with the device full: many runs of the 0.5 um cube
    L = 500.0
    V = L ** 3 * 1e-24
    n_r = args.ssa_throughput
    e = gsbs.Engine(L, 1, W.D_CONFIG, W.REACTIONS)
    n0d = torch.as_tensor(np.tile(W.volume_scaling_counts(L).astype(np.int32), (n_r, 1)), device="cuda")
    vol = torch.full((n_r,), V, dtype=torch.float64, device="cuda")
    gsbs.gsbs_ssa(e.ctx, n0d[:64], vol[:64], rec, seed=args.seed)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    _, ev = gsbs.gsbs_ssa(e.ctx, n0d, vol, rec, seed=args.seed + 2)
    e1.record()
    e1.synchronize()
    wall_host = time.perf_counter() - t0
    wall = e0.elapsed_time(e1) / 1e3  # HIP events on the engine's stream: the launch and its copies
    note(f"event time {wall * 1e3:.2f} ms, host time {wall_host * 1e3:.2f} ms")
    e.close()
    ssa_rate = ev.sum() / wall
    ach = ALG_FLOP_PER_SSA_EVENT * ssa_rate / 1e12
    ssa_roof = dict(bound="alu", achieved=round(ach, 5), peak=FP64_PEAK_TFLOPS, unit="TFLOP/s",
                    frac=round(ach / FP64_PEAK_TFLOPS, 6), kernel="k_ssa", alg_flop_per_event=ALG_FLOP_PER_SSA_EVENT)
    note(f"throughput: {n_r} Gillespie runs of the {L:g} nm cube, {ev.sum()} events in {wall * 1e3:.1f} ms "
         f"= {ssa_rate:.3e} events/s")
    # the oracle's direct method on a bounded sample of the same runs, one thread
    from oracle import ssa_oracle as SO
    n_cpu = 4096
    n0h = W.volume_scaling_counts(L)
    t0 = time.perf_counter()
    ev_cpu = sum(SO.ssa(W.REACTIONS, 7, n0h, V, rec, args.seed + 2, m)[1] for m in range(n_cpu))
    dt_cpu = time.perf_counter() - t0
    cpu = dict(value=round(ev_cpu / dt_cpu, 1), unit="events/s", cores=1, kind="oracle",
               sample=f"{n_cpu} of the {n_r} runs ({ev_cpu} events, {dt_cpu:.1f} s, 1 thread)")
    note(f"oracle: {cpu['sample']}")
    line = {
        "metric": "Gillespie events/s, volume-scaling mixture in a 0.5 um cube",
        "value": round(float(ssa_rate), 1), "unit": "events/s", "higher_is_better": True, "n_gpus": 1,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{n_r} runs of the homogeneous mixture at 2.5e5 molecules/um^3 (spur-model "
                               f"fractions) in a 0.5 um cube, 0 to 10 us; comparisons in 0.2, 0.5 and 1 um cubes"},
        "roofline": ssa_roof,
        "cpu_baseline": cpu,
        "volume_scaling": out,
    }
    print(json.dumps(line), flush=True)


def dose_rate_bench(args):
    """The paper's dose-rate grid as one batched run (one instance per pulse
    train): H2O2 yield and radical build-up against the average dose rate for
    the two pulse dose rates."""
    import numpy as np

    from paper_2509_03313_amd import dose_rate as DR

    def note(*a):
        print("[bench]", *a, file=sys.stderr, flush=True)

    trains = DR.paper_trains(seeds=tuple(range(1, args.dose_rate_seeds + 1)))
    note(f"{len(trains)} pulse trains, {sum(t.n_pulses for t in trains)} pulses")
    r = DR.run(trains, seed=args.seed, ph7=args.ph7, o2=args.o2)
    note(f"wall {r['wall']:.1f} s, {r['steps']} steps, {r['molecule_steps']} molecule-steps, "
         f"{r['ode_steps']} rate-equation steps")
    grid = []
    for dp in sorted({t.pulse_rate for t in trains}):
        for rate in sorted({t.avg_rate for t in trains}):
            idx = [k for k, t in enumerate(trains) if t.pulse_rate == dp and t.avg_rate == rate]
            g = np.array([r["g_h2o2"][k] for k in idx])
            gp = np.array([r["g_h2o2_post"][k] for k in idx])
            b = np.array([DR.build_up(trains[k], r["counts"][k]) for k in idx])
            grid.append(dict(pulse_rate_gy_s=dp, avg_rate_gy_s=rate, g_h2o2=round(float(g.mean()), 4),
                             g_h2o2_sem=round(float(g.std(ddof=1) / np.sqrt(len(g))) if len(g) > 1 else 0.0, 4),
                             g_h2o2_post=round(float(gp.mean()), 4), radical_build_up=round(float(b.mean()), 4)))
            note(f"Dp {dp:g} Gy/s  Dav {rate:>8g} Gy/s: G(H2O2) {g.mean():.4f} +- {grid[-1]['g_h2o2_sem']:.4f}"
                 f"  post-irradiation {gp.mean():.4f}  radicals standing / per pulse {b.mean():.3f}")
    line = {
        "metric": "molecule-steps/s of the dose-rate grid (SBS + rate equations, batched pulse trains)",
        "value": round(r["molecule_steps"] / r["wall"], 1), "unit": "molecule-steps/s", "higher_is_better": True,
        "n_gpus": 1, "dtype": "f32 SBS, f64 rate equations", "data": "synthetic",
        "config": {"workload": f"{len(trains)} trains of 1 us pulses at 2e5 / 1e6 Gy/s to 20 Gy, average "
                               f"0.01-1e5 Gy/s, 2 um cube, hand-over 1 us after each pulse"
                               + ("; pH 7 water" if args.ph7 else "") + ("; aerated" if args.o2 else "")},
        "wall_s": round(r["wall"], 2), "grid": grid,
    }
    print(json.dumps(line), flush=True)


# Algorithmic HBM bytes per molecule-step of the whole step: one read and one
# write of the 32-byte molecule record to move and react it, and one read and
# one write to regroup it by cell.  Neighbour reads of the pair search reuse
# LDS and L2 and are not counted.
STEP_BYTES = 128


def cpu_info():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return model, os.cpu_count(), avail


def _oracle_campaign_sample(args_tuple):
    """The FP64 oracle on the first n_steps SBS steps of one campaign instance
    (same batches, drawn by the oracle's copy of the spur model, same Philox
    streams); returns (molecule-steps, seconds)."""
    seed, i, n_steps, budget = args_tuple
    import numpy as np

    import oracle
    from paper_2509_03313_amd import workload as W
    x = W.campaign(seed)[i]
    chem = oracle.make_chem(W.D_CONFIG, W.REACTIONS)
    dm = oracle.dt_max(chem, x.L)
    anchors = np.array([b[0] for b in x.batches])
    events = np.unique(np.concatenate([x.records, anchors]))
    sched = oracle.schedule(0.0, x.t_end, anchors, events, W.DT0_NS, W.RATIO, dm)[:n_steps]
    s = oracle.Instance(x.L, 1000, i)
    k_b = 0
    t_prev = 0.0
    ms = 0
    t0 = time.perf_counter()
    for te in sched:
        while k_b < len(x.batches) and x.batches[k_b][0] <= t_prev:
            t, n_tr, st = x.batches[k_b]
            xyz, sp = oracle.spurs(x.L, 1000, st, n_tr, W.SPUR_SPACING_NM, W.SPUR_MEAN_MOLECULES, W.SPUR_SIGMA_NM,
                                   W.SPUR_FRACTIONS)
            s.inject(xyz, sp, n_tr * x.L * W.LET_KEV_PER_UM)
            k_b += 1
        ms += s.n
        s.step(chem, te - t_prev)
        t_prev = te
    return ms, time.perf_counter() - t0


def campaign_cpu_baseline(args):
    """1-core and all-core FP64 oracle rates on the first --cpu-steps steps of
    campaign instances (one process per instance)."""
    import multiprocessing as mp
    model, ncpu, avail = cpu_info()
    cores = max(1, min(avail or 1, 16))
    ms1, dt1 = _oracle_campaign_sample((args.seed, 0, args.cpu_steps, 0))
    jobs = [(args.seed, i % 64, args.cpu_steps, 0) for i in range(cores)]
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(cores) as pool:
        res = pool.map(_oracle_campaign_sample, jobs)
    wall = time.perf_counter() - t0
    msa = sum(r[0] for r in res)
    return dict(value=round(msa / wall, 1), unit="molecule-steps/s", cores=cores, kind="oracle",
                cpu_model=model, nproc=ncpu, cores_available=avail,
                one_core=dict(value=round(ms1 / dt1, 1), molecule_steps=int(ms1), seconds=round(dt1, 2)),
                all_core=dict(value=round(msa / wall, 1), molecule_steps=int(msa), seconds=round(wall, 2),
                              processes=cores),
                sample=f"first {args.cpu_steps} SBS steps of campaign instances 0..{cores - 1} (one process each; "
                       f"1-core figure: instance 0 alone), FP64 oracle, same batches and Philox streams")


def small_config_us_per_step(runs=5):
    """The 1e4-molecule single pulse in a 1 um cube (2000 steps, 1 ps -> 1 us),
    launch-bound: microseconds per SBS step with the step kernels launched one
    by one and with each chunk of steps replayed as a HIP graph."""
    import ctypes

    import numpy as np
    import torch

    from paper_2509_03313_amd import gsbs
    from paper_2509_03313_amd import workload as W
    wl = W.single_pulse_small(1000)
    stream = torch.cuda.Stream()  # capturable (not the null stream), default priority
    out = {}
    for graph in (0, 1):
        p = gsbs.gsbs_default_params()
        p.step_graph = graph
        p.autotune = 0
        times = []
        for k in range(runs + 1):
            e = gsbs.Engine(wl.L, 1000, wl.D, wl.reactions, params=p, stream=ctypes.c_void_p(stream.cuda_stream))
            e.load_workload(wl)
            stream.synchronize()
            t = time.perf_counter()
            e.advance_to(wl.t_end)
            stream.synchronize()
            dt = time.perf_counter() - t
            n = e.stats()["steps"]
            e.close()
            if k:
                times.append(dt / n * 1e6)
        out["graph" if graph else "eager"] = round(float(np.median(times)), 2)
    out["steps"] = int(n)
    return out


def single_cube_configs(note):
    """The two single-cube workloads beside the campaign, one timed run each
    (wall clock around gsbs_advance_to, inputs already on the device): one
    1 Gy pulse in a 10 um cube (1 ps -> 1 ms), and 20 pulses of 1 Gy at
    1e6 Gy/s, 1000 Gy/s on average, 10 injection batches per pulse and 100
    records per interval in a 10 um cube."""
    import torch

    from paper_2509_03313_amd import gsbs
    from paper_2509_03313_amd import workload as W
    out = {}
    for name, wl, warm in (("single_pulse_10um_1Gy", W.single_pulse_large(0), True),
                           ("multi_pulse_20x1Gy_10um_1000Gys", W.multi_pulse(0), False)):
        res = None
        for tune in ((True, False) if warm else (False,)):
            p = gsbs.gsbs_default_params()
            p.autotune = 1 if tune else 0
            e = gsbs.Engine(wl.L, 1000, W.D_CONFIG, W.REACTIONS, params=p)
            e.load_workload(wl)
            torch.cuda.synchronize()
            t = time.perf_counter()
            e.advance_to(wl.t_end)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t
            st = e.stats()
            g = e.gvalues(0)
            e.close()
            res = dict(molecule_steps_per_s=round(st["molecule_steps"] / wall, 1), wall_s=round(wall, 3),
                       sbs_steps=int(st["steps"]), molecule_steps=int(st["molecule_steps"]),
                       max_live=int(st["max_live"]), injections=len(wl.injections),
                       records=int(len(wl.records)), G_H2O2_end=round(float(g[-1][W.H2O2]), 5))
            note(f"{name}{' (warm)' if tune else ''}: {res}")
        out[name] = res
    return out


def campaign_bench(args):
    """The batched campaign (64 cubes, edges 2-10 um, 0.1-2 Gy per pulse, 1-20
    pulses at 1e6 Gy/s, average 0.01-1e5 Gy/s, 10 batches per pulse), every
    instance to the end of its train or its 20000th SBS step.  One benchmark
    step is --chunk global SBS steps of all instances (by default 1000, so that
    20 steps run the whole campaign); warmup steps run the start of a separate
    copy of the campaign with the grid autotuner exploring."""
    import numpy as np
    import torch

    from paper_2509_03313_amd import campaign as CA
    from paper_2509_03313_amd import gsbs
    from paper_2509_03313_amd import workload as W

    def note(*a):
        print("[bench]", *a, file=sys.stderr, flush=True)

    insts = W.campaign(args.seed, args.instances)
    note(f"{len(insts)} instances, budget {args.budget} SBS steps, {args.chunk} SBS steps per benchmark step")

    def make(tune):
        p = gsbs.gsbs_default_params()
        p.autotune = 1 if tune else 0
        p.search_split = args.search_split
        if args.step_graph >= 0:
            p.step_graph = args.step_graph
        t = time.perf_counter()
        su = CA.setup(insts, budget=args.budget, params=p)
        torch.cuda.synchronize()
        note(f"setup {time.perf_counter() - t:.1f} s: {su.molecules} molecules in {int(su.batches.sum())} batches, "
             f"device bytes {gsbs.gsbs_get_device_bytes(su.engine.ctx) / 2**30:.2f} GiB")
        return su

    prof_w = None
    if args.warmup:
        su = make(True)
        gsbs.gsbs_set_live_timing(su.engine.ctx, gsbs.KERNEL_SLOTS)
        t = time.perf_counter()
        for k in range(args.warmup):
            su.engine.advance_to(su.targets_after((k + 1) * args.chunk))
            note(f"warmup step {k + 1}/{args.warmup}: {time.perf_counter() - t:.2f} s")
        torch.cuda.synchronize()
        prof_w = gsbs.gsbs_get_profile(su.engine.ctx)
        note(f"warmup {args.warmup} steps: {time.perf_counter() - t:.2f} s, stats {su.engine.stats()}, "
             f"profile {prof_w}")
        su.engine.close()
    su = make(False)
    bytes_state = gsbs.gsbs_get_device_bytes(su.engine.ctx)
    live = gsbs.KERNEL_SLOTS if args.live == "all" else (
        (max(prof_w, key=lambda q: prof_w[q][0]),) if prof_w else ("k_pairs",))
    # HIP events around the timed kernels, on the engine's stream, inside the timed region
    gsbs.gsbs_set_live_timing(su.engine.ctx, live)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        su.engine.advance_to(su.targets_after((k + 1) * args.chunk))
        note(f"step {k + 1}/{args.steps}: {time.perf_counter() - t0:.2f} s")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = su.engine.stats()
    prof = gsbs.gsbs_get_profile(su.engine.ctx)
    n_sbs = int(min(args.steps * args.chunk, su.planned_steps.max()))
    done = all(abs(su.engine.time(i) - su.targets[i]) <= 1e-9 * su.targets[i] for i in range(len(insts)))
    g_h2o2 = [float(su.engine.gvalues(i)[-1][W.H2O2]) for i in range(len(insts))] if done else None
    note(f"timed {args.steps} steps: {wall:.2f} s, stats {st}, profile {prof}")
    su.engine.close()
    value = st["molecule_steps"] / wall
    timed = {q: v for q, v in prof.items() if v[1] > 0}
    dom = max(timed, key=lambda q: timed[q][0])
    tot_ms, launches, units = prof[dom][0], prof[dom][1], prof[dom][2]
    ach = STEP_BYTES * units / (tot_ms / 1e3) / 1e9 if tot_ms > 0 else 0.0
    roof = dict(bound="hbm", achieved=round(ach, 1), peak=HBM_PEAK_GBS, unit="GB/s", frac=round(ach / HBM_PEAK_GBS, 5),
                traffic=None, kernel=dom, avg_launch_us=round(tot_ms * 1e3 / max(launches, 1), 3),
                alg_bytes_per_unit=STEP_BYTES, unit_name="molecule-step of the instances the kernel searched",
                units_per_launch=round(units / max(launches, 1), 1))
    add_traffic(roof, "campaign")
    step_ach = value * STEP_BYTES / 1e9
    small = small_config_us_per_step()
    note(f"1 um single pulse, us per SBS step: {small}")
    singles = single_cube_configs(note) if not args.no_extra_configs else None
    cpu = None
    if not args.no_cpu_baseline:
        cpu = campaign_cpu_baseline(args)
        note(f"cpu baseline: {cpu}")
    line = {
        "metric": "molecule-steps/s of SBS diffusion-reaction",
        "value": round(value, 1), "unit": "molecule-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(wall / args.steps * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"batched campaign: {len(insts)} periodic cubes (edges 2-10 um, 0.1-2 Gy per pulse, "
                               f"1-20 pulses of 1e6 Gy/s, average 0.01-1e5 Gy/s, 10 injection batches per pulse), "
                               f"each to the end of its train or its {args.budget}th SBS step; one benchmark step = "
                               f"{args.chunk} SBS steps of all cubes",
                   "instances": len(insts), "step_budget": args.budget, "sbs_steps_per_step": args.chunk,
                   "sbs_steps_timed": n_sbs, "molecules_injected": su.molecules, "max_live": st["max_live"],
                   "device_state_bytes": int(bytes_state), "species": 7, "reactions": 9},
        "ms_per_sbs_step": round(wall / max(n_sbs, 1) * 1e3, 4),
        "roofline": roof,
        "roofline_step": dict(bound="hbm", achieved=round(step_ach, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                              frac=round(step_ach / HBM_PEAK_GBS, 5), alg_bytes_per_molecule_step=STEP_BYTES,
                              target_frac=0.5, gap_to_target=round(0.5 - step_ach / HBM_PEAK_GBS, 5)),
        "cpu_baseline": cpu,
        "small_config_us_per_sbs_step": small,
        "single_cube_configs": singles,
        "live_timed_kernels": list(live),
        "profile_ms": {q: round(v[0], 3) for q, v in timed.items()},
        "profile_launches": {q: int(v[1]) for q, v in timed.items()},
        "profile_candidates": {q: int(v[3]) for q, v in timed.items() if v[3]},
        "profile_launches": {q: v[1] for q, v in timed.items()},
        "profile_work": {q: v[2] for q, v in timed.items()},
        "profile_candidates": {q: v[3] for q, v in timed.items() if v[3]},
        "warmup_profile_ms": {q: round(v[0], 3) for q, v in prof_w.items()} if prof_w else None,
        "reactions": st["reactions"], "pair_candidates": st["pair_candidates"],
        "G_H2O2_end_mean": round(float(np.mean(g_h2o2)), 5) if g_h2o2 else None,
    }
    print(json.dumps(line), flush=True)


# Algorithmic FLOPs of the perceptron per sample (unpadded layer sizes): the
# forward products, and a training step's forward, input-gradient (all but the
# first layer) and weight-gradient products.
MLP_FWD_FLOP = 2 * (296 * 256 + 3 * 256 * 256 + 256 * 7)
MLP_TRAIN_FLOP = 3 * MLP_FWD_FLOP - 2 * 296 * 256
BF16_PEAK_TFLOPS = 2500.0


def mlp_bench(args):
    """Throughput of the surrogate network's kernels (BF16 MFMA, FP32
    accumulation): forward passes and training steps on a batch of random
    inputs, timed with HIP events on the network's stream."""
    import numpy as np
    import torch

    from paper_2509_03313_amd import gsbs

    def note(*a):
        print("[bench]", *a, file=sys.stderr, flush=True)

    out = {}
    for B in [int(b) for b in args.mlp_batches.split(",") if b]:
        net = gsbs.Mlp(B)
        rng = np.random.default_rng(args.seed)
        net.set_weights((rng.standard_normal(net.n) * 0.05).astype(np.float32))
        x = torch.from_numpy(rng.standard_normal((B, gsbs.MLP_IN)).astype(np.float32)).cuda()
        t = torch.from_numpy(rng.standard_normal((B, gsbs.MLP_OUT)).astype(np.float32)).cuda()
        y = torch.empty((B, gsbs.MLP_OUT), dtype=torch.float32, device="cuda")
        res = {}
        for name, fn, flop in (("forward", lambda: net.forward(x, y), MLP_FWD_FLOP),
                               ("train_step", lambda: net.train_step(x, t, 1e-6), MLP_TRAIN_FLOP)):
            for _ in range(3):
                fn()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(args.mlp_iters):
                fn()
            e1.record()
            e1.synchronize()
            sec = e0.elapsed_time(e1) / 1e3 / args.mlp_iters
            tf = flop * B / sec / 1e12
            res[name] = dict(us=round(sec * 1e6, 2), tflops=round(tf, 2), frac_bf16_peak=round(tf / BF16_PEAK_TFLOPS, 5))
            note(f"batch {B} {name}: {sec * 1e6:.1f} us, {tf:.2f} TFLOP/s ({100 * tf / BF16_PEAK_TFLOPS:.2f} % of bf16 peak)")
        out[B] = res
        net.close()
    big = max(out)
    line = {"metric": "surrogate network forward throughput", "value": round(big / (out[big]["forward"]["us"] / 1e6), 1),
            "unit": "samples/s", "higher_is_better": True, "n_gpus": 1, "dtype": "bf16 (fp32 accumulation)",
            "data": "synthetic", "config": {"workload": "296-256-256-256-256-7 perceptron, erf-GELU",
                                             "flop_per_sample_forward": MLP_FWD_FLOP,
                                             "flop_per_sample_train_step": MLP_TRAIN_FLOP},
            "roofline": {"bound": "mfma", "achieved": out[big]["forward"]["tflops"], "peak": BF16_PEAK_TFLOPS,
                         "unit": "TFLOP/s", "frac": out[big]["forward"]["frac_bf16_peak"], "traffic": None},
            "batches": {str(b): r for b, r in out.items()}}
    print(json.dumps(line), flush=True)


def main():
    args = parse()
    if args.cpu_steps is None:
        args.cpu_steps = 80 if args.single_pulse else 600
    if args.gpus != 1:
        print(f"bench.py: this engine runs on one GPU; --gpus {args.gpus} is not supported "
              "(independent instances would shard across GPUs without communication)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    if args.surrogate:
        surrogate_bench(args)
        return
    if args.mlp:
        mlp_bench(args)
        return
    if args.batched:
        batched_bench(args)
        return
    if args.numodes:
        numodes_bench(args)
        return
    if args.volume_scaling:
        volume_scaling_bench(args)
        return
    if args.dose_rate:
        dose_rate_bench(args)
        return
    if not args.single_pulse and not args.calibrate_copy:
        campaign_bench(args)
        return

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
        roofline = roofline_of(prof, workload="single_pulse_10um")

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
        "ms_per_run": round(wall / args.steps * 1e3, 3),  # one benchmark step is one whole run
        "ms_per_sbs_step": round(wall / (args.steps * max(sbs_steps, 1)) * 1e3, 5),
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
