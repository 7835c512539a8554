"""Parity of the HIP engine (through the C ABI) with the FP64 oracle.

Tolerances (each follows from the FP32 arithmetic of the step):
  * cell binning and candidate pair lists on fixed positions: bit-exact
    (both sides decide in FP32 with the same operation order);
  * pair uniforms (24-bit integers): bit-exact;
  * contact probability: |P_gpu - P_oracle| <= 2e-6 + 2e-5 * a * P, a the
    exponent of the planar factor (FP32 rounding amplified by exp);
  * positions after a jump: |x_gpu - x_oracle| <= 2 ulp_f32(L/2) + 1e-5 sigma;
  * species curves over 32 seeds: |mean_gpu - mean_oracle| <=
    max(0.02 mean_oracle, 3 SE) wherever mean_oracle >= 20;
  * integers (species counts per uid, invariants): exact.
"""
import math
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

from paper_2509_03313_amd import workload as W  # noqa: E402


def say(*a):
    print("[gpu-test]", *a, flush=True)


@pytest.fixture(scope="module")
def g():
    import torch
    assert torch.cuda.is_available(), "GPU tests need the device"
    from paper_2509_03313_amd import gsbs
    return gsbs


def make_engine(g, L, seed, D=None, reactions=None, **kw):
    return g.Engine(L, seed, W.D_CONFIG if D is None else D,
                    W.REACTIONS if reactions is None else reactions, **kw)


def minimg(d, L):
    return (d + L / 2) % L - L / 2


def ulp32(x):
    return float(np.spacing(np.float32(x)))


# ------------------------------------------------------------ diffusion ---
@pytest.mark.parametrize("dt", [1e-3, 0.37, 25.0, 2e3])
def test_jump_matches_oracle(g, orc, dt):
    L, seed = 1000.0, 77
    rng = np.random.default_rng(1)
    n = 20000
    x = rng.uniform(-L / 2, L / 2, size=(n, 3)).astype(np.float32)
    x[:4] = [[L / 2 - 1e-3, -L / 2, 0.0], [-L / 2, L / 2 - 1e-4, 1.0], [0.0, 0.0, 0.0], [499.9, -499.9, 3.0]]
    sp = rng.integers(0, 7, size=n).astype(np.uint8)
    uid = rng.permutation(n * 3)[:n].astype(np.uint64)
    say("jump", dt)
    e = make_engine(g, L, seed, reactions=[])
    g.gsbs_debug_set_state(e.ctx, x, sp, uid, step=123)
    g.gsbs_debug_step(e.ctx, dt)
    xg, sg, ug = g.gsbs_debug_get_state(e.ctx, 0)
    o = orc.Instance(L, seed, 0)
    o.set_state(x.astype(np.float64), sp.astype(np.int32), uid, step=123)
    o.step(orc.make_chem(W.D_CONFIG, []), dt)
    xo, _, so, uo = o.state()
    a, b = np.argsort(ug), np.argsort(uo)
    assert np.array_equal(ug[a], uo[b]) and np.array_equal(sg[a], so[b])
    sig = np.sqrt(2 * np.asarray(W.D_CONFIG)[sg[a]] * dt)[:, None]
    err = np.abs(minimg(xg[a].astype(np.float64) - xo[b], L))
    tol = 2 * ulp32(L / 2) + 1e-5 * sig
    assert np.all(err <= tol), (err.max(), np.argmax(err))
    assert np.all(xg >= -L / 2) and np.all(xg < L / 2)
    e.close()


# --------------------------------------------------------- cell binning ---
@pytest.mark.parametrize("nc", [1, 2, 3, 7, 13, 46])
def test_binning_bit_exact(g, orc, nc):
    L = 1000.0
    rng = np.random.default_rng(nc)
    n = 30000
    x = rng.uniform(-L / 2, L / 2, size=(n, 3)).astype(np.float32)
    # positions on and next to cell faces and the cube faces
    faces = (np.arange(nc + 1) * (L / nc) - L / 2).astype(np.float32)
    k = min(len(faces), 200)
    x[:k, 0] = faces[:k]
    x[k:2 * k, 1] = np.nextafter(faces[:k], np.float32(-1e9))
    x[2 * k:3 * k, 2] = np.nextafter(faces[:k], np.float32(1e9))
    x = np.clip(x, np.float32(-L / 2), np.nextafter(np.float32(L / 2), np.float32(0)))
    sp = rng.integers(0, 7, size=n).astype(np.uint8)
    uid = np.arange(n, dtype=np.uint64)
    say("binning nc", nc)
    e = make_engine(g, L, 5)
    g.gsbs_debug_set_state(e.ctx, x, sp, uid)
    g.gsbs_debug_step(e.ctx, 1e-3, g.DEBUG_FIXED | g.DEBUG_SEARCH_ONLY, xyz0=x, nc_force=nc)
    cell, u, ncg = g.gsbs_debug_get_cells(e.ctx)
    assert ncg == nc and len(u) == n
    ref = orc.bin_f32(x, L, nc)
    assert np.array_equal(cell, ref[u.astype(np.int64)])
    # sorted by cell
    assert np.all(np.diff(cell) >= 0)
    e.close()


# ----------------------------------------------------- candidate pairs ---
MODES = {"auto": 0, "species": 8, "whole": 16}


@pytest.mark.parametrize("dt,nc,mode", [(0.05, 0, "auto"), (3.0, 0, "species"), (3.0, 2, "whole"),
                                        (40.0, 1, "whole"), (40.0, 1, "species"), (40.0, 0, "species"),
                                        (3.0, 12, "species"), (0.5, 20, "species"), (3.0, 30, "whole"),
                                        (3.0, 30, "species")])
def test_candidates_bit_exact(g, orc, dt, nc, mode):
    """Candidate pairs on fixed positions equal the oracle's FP32 brute force
    for both search modes, coarse and fine grids (stencil reach 1-4) and grids
    of fewer than 3 cells per axis; P and u24 match the oracle's."""
    L = 400.0
    rng = np.random.default_rng(int(dt * 100) + nc)
    n = 3000
    x0 = rng.uniform(-L / 2, L / 2, size=(n, 3))
    # clustered half: spur-like groups so that many pairs are within R
    x0[: n // 2] = rng.uniform(-L / 2, L / 2, size=(n // 30, 3)).repeat(15, axis=0) + rng.normal(0, 1.5, size=(n // 2, 3))
    x0 = ((x0 + L / 2) % L - L / 2).astype(np.float32)
    x1 = ((x0 + rng.normal(0, math.sqrt(2 * 5 * dt), size=(n, 3)) + L / 2) % L - L / 2).astype(np.float32)
    sp = rng.integers(0, 7, size=n).astype(np.uint8)
    uid = np.arange(n, dtype=np.uint64)
    say("candidates", dt, nc, mode)
    e = make_engine(g, L, 9)
    g.gsbs_debug_set_state(e.ctx, x1, sp, uid, step=4)
    g.gsbs_debug_step(e.ctx, dt, g.DEBUG_FIXED | g.DEBUG_SEARCH_ONLY | g.DEBUG_LOG_ALL | MODES[mode], xyz0=x0,
                      nc_force=nc)
    pr = g.gsbs_debug_get_pairs(e.ctx)
    chem = orc.make_chem(W.D_CONFIG, W.REACTIONS)
    ref = orc.cand_f32(x1, sp, L, chem, dt)
    got = set(map(tuple, pr["uid"].astype(np.int64).tolist()))
    assert got == set(map(tuple, ref.tolist())) and len(got) > 50
    # probabilities and uniforms against the oracle's FP64 formulas on the same inputs
    key = (9, 0)
    worst = 0.0
    for (a, b), P, u24, rx in zip(pr["uid"].astype(np.int64), pr["P"], pr["u24"], pr["rx"]):
        w = orc.philox([a, b, 4, 1], key)
        assert int(w[0]) >> 40 == int(u24)
        r = W.REACTIONS[rx]
        Dab = W.D_CONFIG[r.a] + W.D_CONFIG[r.b]
        R = orc.radius(r.k_in, Dab)
        r1 = np.linalg.norm(minimg(x1[b].astype(np.float64) - x1[a], L))
        r0 = np.linalg.norm(minimg(x0[b].astype(np.float64) - x0[a], L))
        Po = orc.bridge(r0, r1, R, Dab * dt)
        aexp = max((r0 - R) * (r1 - R) / (Dab * dt), 0.0)
        tol = 2e-6 + 2e-5 * (1 + aexp) * Po
        worst = max(worst, abs(P - Po) / tol)
        assert abs(P - Po) <= tol, (a, b, P, Po, r0, r1, R)
    say("worst P error / tol", worst)
    e.close()


@pytest.mark.parametrize("dt,nc", [(3.0, 5), (3.0, 9), (40.0, 4), (40.0, 9)])
def test_candidates_independent_of_search_shape(g, orc, dt, nc):
    """The species-bin search's work split (stream slices per box) and box
    shape change only speed: every setting gives the oracle's FP32 candidate
    set, including cutoffs near L/2 where windows wrap and shifts straddle."""
    L = 400.0
    rng = np.random.default_rng(500 + nc)
    n = 3000
    x0 = rng.uniform(-L / 2, L / 2, size=(n, 3))
    x0[: n // 2] = rng.uniform(-L / 2, L / 2, size=(n // 30, 3)).repeat(15, axis=0) + rng.normal(0, 1.5, size=(n // 2, 3))
    x0 = ((x0 + L / 2) % L - L / 2).astype(np.float32)
    x1 = ((x0 + rng.normal(0, math.sqrt(2 * 5 * dt), size=(n, 3)) + L / 2) % L - L / 2).astype(np.float32)
    sp = rng.integers(0, 7, size=n).astype(np.uint8)
    uid = np.arange(n, dtype=np.uint64)
    chem = orc.make_chem(W.D_CONFIG, W.REACTIONS)
    ref = set(map(tuple, orc.cand_f32(x1, sp, L, chem, dt).tolist()))
    assert len(ref) > 50
    for split in (1, 3, 16):
        for box in (1, 3):
            say("search shape", dt, nc, split, box)
            p = g.gsbs_default_params()
            p.search_split = split
            p.search_box = box
            e = make_engine(g, L, 9, params=p)
            g.gsbs_debug_set_state(e.ctx, x1, sp, uid, step=4)
            g.gsbs_debug_step(e.ctx, dt, g.DEBUG_FIXED | g.DEBUG_SEARCH_ONLY | g.DEBUG_LOG_ALL | MODES["species"],
                              xyz0=x0, nc_force=nc)
            pr = g.gsbs_debug_get_pairs(e.ctx)
            got = [tuple(u) for u in pr["uid"].astype(np.int64).tolist()]
            assert len(got) == len(set(got)), "a pair was tested twice"
            assert set(got) == ref, (split, box, len(got), len(ref))
            e.close()


@pytest.mark.parametrize("dt", [20.0, 500.0])
def test_filtered_search_reacts_like_logged_search(g, dt):
    """Without logging, the species-bin search screens with fused arithmetic and
    skips the evaluation of pairs whose bridge exponent bound exceeds 18
    (P < e^-18 < 2^-25, never accepted), and few accepted pairs are matched in
    LDS; with every candidate logged, every pair is evaluated and matched
    through the global tables.  Both steps must react the same pairs into the
    same state."""
    L = 2000.0
    n = 20000
    rng = np.random.default_rng(int(dt))
    x = rng.uniform(-L / 2, L / 2, size=(n, 3))
    x[: n // 4] = rng.uniform(-L / 2, L / 2, size=(n // 40, 3)).repeat(10, axis=0) + rng.normal(0, 5.0, size=(n // 4, 3))
    x = ((x + L / 2) % L - L / 2).astype(np.float32)
    sp = rng.integers(0, 7, size=n).astype(np.uint8)
    uid = np.arange(n, dtype=np.uint64)
    outs = []
    for flags in (0, g.DEBUG_LOG_ALL):
        say("filtered vs logged", dt, flags)
        e = make_engine(g, L, 11)
        g.gsbs_debug_set_state(e.ctx, x, sp, uid, step=7, next_uid=n)
        g.gsbs_debug_step(e.ctx, dt, flags | MODES["species"])
        outs.append(g.gsbs_debug_get_state(e.ctx, 0))
        e.close()
    (xa, sa, ua), (xb, sb, ub) = outs
    ia, ib = np.argsort(ua), np.argsort(ub)
    assert not np.array_equal(np.sort(ua), uid)  # something reacted
    assert np.array_equal(ua[ia], ub[ib]) and np.array_equal(sa[ia], sb[ib])
    assert np.array_equal(xa[ia], xb[ib])


# ------------------------------------------------ short trajectory parity ---
def test_first_steps_match_oracle(g, orc):
    """Same initial spurs, same Philox streams: the GPU and the oracle follow
    the same trajectory (same reactions, same uids and species, positions
    within tolerance) until FP32 positions and FP32 probabilities flip an
    accept decision.  At a flip each side must have decided correctly from its
    own P, the pair uniform must lie between the two P, and the two P must
    agree to the drift of FP32 positions (2% at steps of femtoseconds)."""
    wl = W.single_pulse_small(3)
    L = wl.L
    inj = wl.injections[0]
    n = len(inj.species)
    uid = np.arange(n, dtype=np.uint64)
    chem = orc.make_chem(wl.D, wl.reactions)
    e = make_engine(g, L, 1000)
    g.gsbs_debug_set_state(e.ctx, inj.xyz, inj.species, uid, step=0, next_uid=n)
    o = orc.Instance(L, 1000, 0)
    o.set_state(inj.xyz.astype(np.float64), inj.species.astype(np.int32), uid, step=0, next_uid=n)
    o.set_log(2)
    sched = orc.schedule(0.0, 50.0, [0.0], [], wl.dt0, wl.ratio, orc.dt_max(chem, L))
    t = 0.0
    n_react = 0
    for k, te in enumerate(sched[:1200]):
        dt = te - t
        t = te
        g.gsbs_debug_step(e.ctx, dt, g.DEBUG_LOG_ALL)
        o.step(chem, dt)
        pg = g.gsbs_debug_get_pairs(e.ctx)
        lo = o.log()
        accg = {tuple(p) for p, f in zip(pg["uid"].tolist(), pg["flag"]) if f & 1}
        acco = {tuple(p) for p, f in zip(lo["uid"].tolist(), lo["flag"]) if f & 1}
        if accg != acco:
            Po = {tuple(p): (P, u) for p, P, u in zip(lo["uid"].tolist(), lo["P"], lo["u24"])}
            Pg = {tuple(p): (P, u) for p, P, u in zip(pg["uid"].tolist(), pg["P"], pg["u24"])}
            for p in accg ^ acco:
                po, uo_ = Po.get(p, (0.0, None))
                pgv, ug_ = Pg.get(p, (0.0, None))
                u24 = uo_ if uo_ is not None else ug_
                uu = (2 * int(u24) + 1) / 2 ** 25
                assert (uu < pgv) == (p in accg) and (uu < po) == (p in acco), (k, p)
                assert min(pgv, po) <= uu <= max(pgv, po), (k, p, uu, pgv, po)
                assert abs(pgv - po) <= 0.02 * max(pgv, po) + 1e-4, (k, p, pgv, po)
            say("accept flip at step", k, "P gpu/oracle straddle u; trajectories diverge from here")
            break
        xg, sg, ug = g.gsbs_debug_get_state(e.ctx, 0)
        xo, _, so, uo = o.state()
        a, b = np.argsort(ug), np.argsort(uo)
        assert np.array_equal(ug[a], uo[b]), k
        assert np.array_equal(sg[a].astype(np.int32), so[b]), k
        err = np.abs(minimg(xg[a].astype(np.float64) - xo[b], L))
        assert err.max() <= 1e-5 * L, (k, err.max())
        n_react += len(accg)
    say("steps compared", k + 1, "accepted pairs", n_react)
    assert n_react > 20
    e.close()


# ------------------------------------------------------ statistical parity ---
def test_species_curves_32_seeds(g):
    """Species counts and G(H2O2) time curves of 32 seeds (one batched launch
    of 32 instances) agree with the oracle's within 2% and 3 SE."""
    gold = np.load(os.path.join(HERE, "golden", "single_pulse_1um_oracle.npz"))
    co = gold["counts"].astype(np.float64)
    seed = int(gold["philox_seed"])
    wls = [W.single_pulse_small(i) for i in range(co.shape[0])]
    say("batched 32 instances")
    e = make_engine(g, [w.L for w in wls], seed)
    for i, w in enumerate(wls):
        e.load_workload(w, inst=i)
    e.advance_to(wls[0].t_end)
    cg = np.stack([e.counts(i) for i in range(len(wls))]).astype(np.float64)
    gg = np.stack([e.gvalues(i) for i in range(len(wls))])
    assert cg.shape == co.shape and np.all(cg >= 0)
    d = cg - co
    mo = co.mean(axis=0)
    mg = cg.mean(axis=0)
    se = d.std(axis=0, ddof=1) / math.sqrt(co.shape[0])
    mask = mo >= 20
    bound = np.maximum(0.02 * mo, 3 * se)
    bad = mask & (np.abs(mg - mo) > bound)
    assert not bad.any(), (np.argwhere(bad)[:5], mg[bad][:5], mo[bad][:5])
    # G(H2O2) curve
    edep = gold["edep"]
    go = co[:, :, W.H2O2] / (edep / 100.0)
    gm = gg[:, :, W.H2O2]
    m = mo[:, W.H2O2] >= 20
    dG = gm - go
    seG = dG.std(axis=0, ddof=1) / math.sqrt(co.shape[0])
    assert np.all(np.abs(gm.mean(0) - go.mean(0))[m] <= np.maximum(0.02 * go.mean(0), 3 * seG)[m])
    st = e.stats()
    say("molecule-steps", st["molecule_steps"], "reactions", st["reactions"])
    assert st["molecule_steps"] > 0
    e.close()


def test_reduced_large_pulse_curves_32_seeds(g):
    """The 10 um single pulse reduced to a 2.5 um cube at the same track
    density (~6e3 molecules, 1 ps -> 1 ms, 3297 steps, the late ones at the
    cube's largest step, so the species-bin search runs): species counts and
    G(H2O2) at 60 log-spaced times of 32 seeds (one batched launch) agree with
    the oracle's within 2 % and 3 SE where the oracle mean is at least 20."""
    gold = np.load(os.path.join(HERE, "golden", "single_pulse_2p5um_oracle.npz"))
    co = gold["counts"].astype(np.float64)
    seed = int(gold["philox_seed"])
    wls = [W.single_pulse_large(i, L=float(gold["L_nm"]), n_records=int(gold["n_records"])) for i in range(co.shape[0])]
    say("batched 32 reduced 10 um pulses")
    e = make_engine(g, [w.L for w in wls], seed)
    for i, w in enumerate(wls):
        e.load_workload(w, inst=i)
    e.advance_to(wls[0].t_end)
    cg = np.stack([e.counts(i) for i in range(len(wls))]).astype(np.float64)
    gg = np.stack([e.gvalues(i) for i in range(len(wls))])
    assert cg.shape == co.shape and np.all(cg >= 0)
    assert np.array_equal(cg[:, 0], co[:, 0])  # the first record is the injected state
    d = cg - co
    mo, mg = co.mean(axis=0), cg.mean(axis=0)
    se = d.std(axis=0, ddof=1) / math.sqrt(co.shape[0])
    bad = (mo >= 20) & (np.abs(mg - mo) > np.maximum(0.02 * mo, 3 * se))
    say("records", co.shape[1], "checked", int((mo >= 20).sum()), "outside", int(bad.sum()))
    assert not bad.any(), (np.argwhere(bad)[:5], mg[bad][:5], mo[bad][:5])
    go = co[:, :, W.H2O2] / (gold["edep"] / 100.0)
    gm = gg[:, :, W.H2O2]
    m = mo[:, W.H2O2] >= 20
    seG = (gm - go).std(axis=0, ddof=1) / math.sqrt(co.shape[0])
    assert np.all(np.abs(gm.mean(0) - go.mean(0))[m] <= np.maximum(0.02 * go.mean(0), 3 * seG)[m])
    st = e.stats()
    assert st["steps"] == int(gold["n_steps"][0])
    say("molecule-steps", st["molecule_steps"], "species-bin candidates", st.get("pair_candidates"))
    e.close()


def test_profiling_mode_times_every_kernel(g):
    """gsbs_set_profiling: every step's kernels get their own pair of HIP
    events (synchronised per step); the profile reports a positive time for
    every kernel that ran, and the run's counts equal an unprofiled run's."""
    wl = W.single_pulse_small(3)
    out = []
    for prof in (False, True):
        e = make_engine(g, wl.L, 1000)
        e.load_workload(wl)
        if prof:
            g.gsbs_set_profiling(e.ctx, True)
        e.advance_to(wl.t_end)
        out.append((e.counts(0), g.gsbs_get_profile(e.ctx) if prof else None, e.stats()["steps"]))
        e.close()
    (c0, _, n0), (c1, pr, n1) = out
    assert np.array_equal(c0, c1) and n0 == n1
    say("profile", {k: (round(v[0], 3), v[1]) for k, v in pr.items()})
    for k in ("k_bin", "k_scan", "k_scatter", "k_react"):
        assert pr[k][1] == n1 and pr[k][0] > 0.0, (k, pr[k])
    assert pr["k_pairs"][1] + pr["k_pairs_sp"][1] >= n1


def test_multi_pulse_curves_32_seeds(g):
    """Four pulses (two injection batches each, the step ramp restarting at
    every batch): species counts at 30 log-spaced times per interval of 32
    seeds agree with the oracle's within 2% and 3 SE."""
    gold = np.load(os.path.join(HERE, "golden", "multi_pulse_1um_oracle.npz"))
    co = gold["counts"].astype(np.float64)
    seed = int(gold["philox_seed"])
    kw = dict(n_pulses=4, dose_per_pulse=1.0, L=1000.0, pulse_rate_gy_s=1e6, avg_rate_gy_s=1e4, n_batches=2,
              n_records=30)
    wls = [W.multi_pulse(i, **kw) for i in range(co.shape[0])]
    say("batched 32 multi-pulse instances")
    e = make_engine(g, [w.L for w in wls], seed)
    for i, w in enumerate(wls):
        e.load_workload(w, inst=i)
    e.advance_to(wls[0].t_end)
    cg = np.stack([e.counts(i) for i in range(len(wls))]).astype(np.float64)
    assert cg.shape == co.shape and np.all(cg >= 0)
    assert np.array_equal(cg[:, 0], co[:, 0])  # the first record is the injected state
    d = cg - co
    mo, mg = co.mean(axis=0), cg.mean(axis=0)
    se = d.std(axis=0, ddof=1) / math.sqrt(co.shape[0])
    bad = (mo >= 20) & (np.abs(mg - mo) > np.maximum(0.02 * mo, 3 * se))
    say("records", co.shape[1], "checked", int((mo >= 20).sum()), "outside", int(bad.sum()))
    assert not bad.any(), (np.argwhere(bad)[:5], mg[bad][:5], mo[bad][:5])
    st = e.stats()
    assert st["steps"] == int(gold["n_steps"][0])  # the same schedule (ramp restarts, records as step ends)
    e.close()


def test_step_graph_equals_eager(g):
    """Capturing each chunk of step launches into a HIP graph changes nothing:
    two instances, one with a second injection mid-run (the capture is cut
    there), give identical counts at every record with and without graphs."""
    wl = W.single_pulse_small(7)
    wl2 = W.single_pulse_small(8, n_tracks=2)
    late = W.single_pulse_small(9, n_tracks=1).injections[0]
    import ctypes
    import torch
    stream = torch.cuda.Stream()  # a capturable stream (not the null stream), default priority
    res = []
    for graph in (0, 1):
        say("step graph", graph)
        p = g.gsbs_default_params()
        p.step_graph = graph
        p.autotune = 0
        e = make_engine(g, [wl.L, wl2.L], 31, params=p, stream=ctypes.c_void_p(stream.cuda_stream))
        e.load_workload(wl, inst=0)
        e.load_workload(wl2, inst=1)
        e.inject(1, 0.37, late.xyz, late.species, late.edep_ev)
        e.advance_to(wl.t_end)
        res.append((e.counts(0), e.counts(1), e.stats()))
        e.close()
    assert np.array_equal(res[0][0], res[1][0]) and np.array_equal(res[0][1], res[1][1])
    assert res[0][2]["steps"] == res[1][2]["steps"] and res[0][2]["reactions"] == res[1][2]["reactions"]


def test_invariants_and_replay(g):
    """Charge and redox balances are exact at every record, and the same seed
    replays to identical counts (outcomes do not depend on atomic order)."""
    wl = W.single_pulse_small(5)
    res = []
    for _ in range(2):
        e = make_engine(g, wl.L, 42)
        e.load_workload(wl)
        e.advance_to(wl.t_end)
        res.append(e.counts())
        e.close()
    c = res[0]
    assert np.array_equal(res[0], res[1])
    Q = c[:, W.H3O] - c[:, W.E_AQ] - c[:, W.OHM]
    Wr = c[:, W.OH] + 2 * c[:, W.H2O2] - c[:, W.E_AQ] - c[:, W.H] - 2 * c[:, W.H2]
    assert np.all(Q == Q[0]) and np.all(Wr == Wr[0])


# ------------------------------------------------------------ edge cases ---
def test_edge_cases(g, orc):
    # an empty instance next to a populated one, an injection mid-run with a
    # record at the same time, and a tiny cube where the search grid has < 3 cells
    wl = W.single_pulse_small(7, n_tracks=1, track_nm=3000.0)
    e = make_engine(g, [wl.L, wl.L, 60.0], 3)
    e.load_workload(wl, inst=0)
    e.set_records(1, [0.0, 10.0])
    rng = np.random.default_rng(0)
    xs = rng.uniform(-30, 30, size=(40, 3)).astype(np.float32)
    ss = rng.integers(0, 7, size=40).astype(np.uint8)
    e.inject(2, 0.0, xs, ss, 100.0)
    e.inject(2, 5.0, xs[:10], ss[:10], 50.0)
    e.set_records(2, [0.0, 5.0, 50.0])
    e.advance_to([20.0, 10.0, 50.0])
    assert e.time(0) == 20.0 and e.time(1) == 10.0 and e.time(2) == 50.0
    c1 = e.counts(1)
    assert np.all(c1 == 0)
    c2 = e.counts(2)
    assert np.all(c2 >= 0) and c2[1].sum() >= c2[0].sum() - 40
    gv = e.gvalues(2)
    assert np.isfinite(gv).all()
    # the tiny cube matches the oracle run of the same input (small enough to be exact)
    w2 = W.Workload("tiny", 60.0, 3, [W.Injection(0.0, xs, ss, 100.0), W.Injection(5.0, xs[:10], ss[:10], 50.0)],
                    np.array([0.0, 5.0, 50.0]), 50.0)
    r = orc.run(w2, inst=2, philox_seed=3)
    say("tiny cube gpu", c2[-1], "oracle", r["counts"][-1])
    assert np.array_equal(c2[0], r["counts"][0]) and np.array_equal(c2[1], r["counts"][1])
    e.close()


def test_full_size_first_steps(g, orc):
    """The ~4e5-molecule 10 um single-pulse workload at full size, in the
    benchmark's launch configuration: the first steps agree with the oracle on
    every accepted pair (or a near-tie), and invariants hold after 300 steps."""
    wl = W.single_pulse_large(0)
    n = wl.n_initial
    say("full size", n)
    inj = wl.injections[0]
    uid = np.arange(n, dtype=np.uint64)
    chem = orc.make_chem(wl.D, wl.reactions)
    e = make_engine(g, wl.L, 2024)
    g.gsbs_debug_set_state(e.ctx, inj.xyz, inj.species, uid, step=0, next_uid=n)
    o = orc.Instance(wl.L, 2024, 0)
    o.set_state(inj.xyz.astype(np.float64), inj.species.astype(np.int32), uid, step=0, next_uid=n)
    o.set_log(1)
    sched = orc.schedule(0.0, 1e6, [0.0], [], wl.dt0, wl.ratio, orc.dt_max(chem, wl.L))
    t = 0.0
    for k in range(3):
        dt = sched[k] - t
        t = sched[k]
        g.gsbs_debug_step(e.ctx, dt)
        o.step(chem, dt)
        pg = g.gsbs_debug_get_pairs(e.ctx)
        lo = o.log()
        accg = {tuple(p) for p, f in zip(pg["uid"].tolist(), pg["flag"]) if f & 1}
        acco = {tuple(p) for p in lo["uid"].tolist()}
        say("step", k, "accepted gpu", len(accg), "oracle", len(acco))
        assert len(accg ^ acco) <= max(2, len(acco) // 1000)
        assert len(acco) > 0
        # every difference is a near-tie: the pair uniform lies within the FP32
        # rounding of P (the bridge exponent of an evaluated pair is at most 18)
        pg_of = {tuple(p): (P, u) for p, P, u in zip(pg["uid"].tolist(), pg["P"], pg["u24"])}
        po_of = {tuple(p): (P, u) for p, P, u in zip(lo["uid"].tolist(), lo["P"], lo["u24"])}
        for pair in accg ^ acco:
            P, u24 = pg_of[pair] if pair in accg else po_of[pair]
            u = (int(u24) + 0.5) * 2.0 ** -24
            assert abs(u - float(P)) <= 2e-6 + 2e-5 * 19 * float(P), (pair, u, P)
    e.close()
    e = make_engine(g, wl.L, 2024)
    e.load_workload(wl)
    e.advance_to(float(sched[299]))
    c = e.current_counts()
    Q = c[W.H3O] - c[W.E_AQ] - c[W.OHM]
    Wr = c[W.OH] + 2 * c[W.H2O2] - c[W.E_AQ] - c[W.H] - 2 * c[W.H2]
    c0 = np.bincount(inj.species, minlength=7)
    assert Q == c0[W.H3O] - c0[W.E_AQ] - c0[W.OHM]
    assert Wr == c0[W.OH] + 2 * c0[W.H2O2] - c0[W.E_AQ] - c0[W.H] - 2 * c0[W.H2]
    e.close()


def test_first_order_channels_match_oracle(g, orc):
    """Aerated water (first-order scavenging of e_aq and H by O2, lumped
    superoxide and its reactions): the GPU and the oracle take the same
    first-order conversions (uid-keyed Philox decisions against the same FP64
    probability) and the same pair reactions, step for step, until an FP32 /
    FP64 accept flip of a pair."""
    wl = W.single_pulse_small(4)
    L = wl.L
    inj = wl.injections[0]
    n = len(inj.species)
    uid = np.arange(n, dtype=np.uint64)
    # scavenging 400x faster than in aerated water, so that many conversions
    # fall within the compared steps (the first ~20 ps)
    fo = [W.FirstOrder(f.name, f.a, 400.0 * f.k, f.products) for f in W.FIRST_ORDER_O2]
    chem = orc.make_chem(W.D_CONFIG_O2, W.REACTIONS_O2, first_order=fo)
    e = make_engine(g, L, 1000, D=W.D_CONFIG_O2, reactions=W.REACTIONS_O2)
    g.gsbs_set_first_order(e.ctx, fo)
    g.gsbs_debug_set_state(e.ctx, inj.xyz, inj.species, uid, step=0, next_uid=n)
    o = orc.Instance(L, 1000, 0)
    o.set_state(inj.xyz.astype(np.float64), inj.species.astype(np.int32), uid, step=0, next_uid=n)
    o.set_log(2)
    sched = orc.schedule(0.0, 200.0, [0.0], [], wl.dt0, wl.ratio, orc.dt_max(chem, L))
    t = 0.0
    for k, te in enumerate(sched[:1500]):
        dt = te - t
        t = te
        g.gsbs_debug_step(e.ctx, dt, g.DEBUG_LOG_ALL)
        o.step(chem, dt)
        pg = g.gsbs_debug_get_pairs(e.ctx)
        lo = o.log()
        accg = {tuple(p) for p, f in zip(pg["uid"].tolist(), pg["flag"]) if f & 1}
        acco = {tuple(p) for p, f in zip(lo["uid"].tolist(), lo["flag"]) if f & 1}
        if accg != acco:
            say("accept flip at step", k)
            break
        xg, sg, ug = g.gsbs_debug_get_state(e.ctx, 0)
        xo, _, so, uo = o.state()
        a, b = np.argsort(ug), np.argsort(uo)
        assert np.array_equal(ug[a], uo[b]), k
        assert np.array_equal(sg[a].astype(np.int32), so[b]), k
        err = np.abs(minimg(xg[a].astype(np.float64) - xo[b], L))
        assert err.max() <= 1e-5 * L, (k, err.max())
    n_sup = int(np.sum(so == W.O2M))
    n_two = int(np.sum(uo >= np.uint64(2 ** 63)))
    say("steps compared", k + 1, "superoxide", n_sup, "second products", n_two)
    assert k > 300 and n_sup > 20 and n_two > 3
    # the device counts follow the conversions
    _, sg, _ = g.gsbs_debug_get_state(e.ctx, 0)
    cg = e.current_counts(0)
    assert np.array_equal(cg, np.bincount(sg.astype(np.int64), minlength=len(cg))[:len(cg)])
    e.close()


def test_first_order_only_batched_matches_oracle_exactly(g, orc):
    """First-order channels alone decide in exact FP64 on both sides, so a
    batched run of two instances with different end times (one idles while
    the other steps) reproduces the oracle's record counts exactly for each
    instance (Philox key (seed, instance))."""
    fo = [W.FirstOrder("e", W.E_AQ, 0.05, (W.OHM,)), W.FirstOrder("H", W.H, 0.02, (W.H2, W.H3O)),
          W.FirstOrder("OH", W.OH, 0.01, ())]
    # one pair reaction whose species never occurs (H2O2 is neither injected nor
    # produced here): the search runs but finds nothing to decide in FP32
    idle = [W.Reaction("idle", W.H2O2, W.H2O2, 0.5, (W.H2,))]
    wls = [W.single_pulse_small(6), W.single_pulse_small(7)]
    ends = [40.0, 120.0]
    seed = 4321
    e = make_engine(g, [w.L for w in wls], seed, reactions=idle)
    g.gsbs_set_first_order(e.ctx, fo)
    for i, w in enumerate(wls):
        e.load_workload(w, inst=i)
    e.advance_to(np.array(ends))
    chem = orc.make_chem(wls[0].D, idle, first_order=fo)
    for i, w in enumerate(wls):
        ref = orc.run(w, chem, inst=i, t_end=ends[i], philox_seed=seed)
        got = e.counts(i)[:len(ref["counts"])]
        say("instance", i, "records", len(ref["counts"]), "final", got[-1].tolist())
        assert np.array_equal(got, ref["counts"]), i
        assert got[-1][W.E_AQ] < ref["counts"][0][W.E_AQ]
    e.close()


def _straddles(orc, x1, x0, sp, uid, L, dt, step, seed, pairs):
    """Pairs (uid, uid) whose uniform lies within the FP32 rounding of the
    oracle's P (the accept decision may go either way between FP32 and FP64)."""
    idx = {int(u): k for k, u in enumerate(uid)}
    ok = []
    for a, b in pairs:
        i, j = idx[a], idx[b]
        r = [q for q in W.REACTIONS if {q.a, q.b} == {int(sp[i]), int(sp[j])}][0]
        Dab = W.D_CONFIG[r.a] + W.D_CONFIG[r.b]
        R = orc.radius(r.k_in, Dab)
        r1 = np.linalg.norm(minimg(x1[j].astype(np.float64) - x1[i], L))
        r0 = np.linalg.norm(minimg(x0[j].astype(np.float64) - x0[i], L))
        P = orc.bridge(r0, r1, R, Dab * dt)
        aexp = max((r0 - R) * (r1 - R) / (Dab * dt), 0.0)
        u = ((int(orc.philox([min(a, b), max(a, b), step, 1], [seed, 0])[0]) >> 40) + 0.5) * 2.0 ** -24
        ok.append(abs(u - P) <= 2e-6 + 2e-5 * (1 + aexp) * P)
    return ok


@pytest.mark.parametrize("dt", [500.0, 2000.0])
def test_full_size_late_regime_species_bin_search(g, orc, dt):
    """A late-regime state of the 10 um cube at full size: 150 000 molecules
    of the spur-model mixture spread through the cube, one step of 0.5 or 2 us
    on fixed positions through the production species-bin search (candidates
    not logged, the library's own box shape and stream split, fused screening
    and the bridge-exponent filter).  The candidate count equals the oracle's
    FP32 count, and the accepted pairs equal the oracle's except pairs whose
    uniform lies within the FP32 rounding of P."""
    L, n, step, seed = 10000.0, 150000, 9, 31
    rng = np.random.default_rng(int(dt))
    x0 = rng.uniform(-L / 2, L / 2, size=(n, 3))
    sp = rng.choice(7, size=n, p=W.SPUR_FRACTIONS).astype(np.uint8)
    sig = np.sqrt(2.0 * np.array(W.D_CONFIG)[sp] * dt)[:, None]
    x1 = ((x0 + rng.normal(size=(n, 3)) * sig + L / 2) % L - L / 2).astype(np.float32)
    x0 = x0.astype(np.float32)
    uid = rng.permutation(np.arange(n, dtype=np.uint64) * 5 + 11)
    say("late regime full size", dt, n)
    e = make_engine(g, L, seed)
    g.gsbs_debug_set_state(e.ctx, x1, sp, uid, step=step)
    c0 = e.stats()["pair_candidates"]
    g.gsbs_debug_step(e.ctx, dt, g.DEBUG_FIXED | g.DEBUG_SEARCH_ONLY | MODES["species"], xyz0=x0)
    ncand = e.stats()["pair_candidates"] - c0
    pr = g.gsbs_debug_get_pairs(e.ctx)
    e.close()
    acc_g = {tuple(p) for p, f in zip(pr["uid"].tolist(), pr["flag"]) if f & 1}
    chem = orc.make_chem(W.D_CONFIG, W.REACTIONS)
    say("oracle decisions")
    pairs, P, u24, ncand_o = orc.accept_f32(x1, x0, sp, uid, L, chem, dt, step, seed, 0)
    acc_o = {(int(min(uid[i], uid[j])), int(max(uid[i], uid[j]))) for i, j in pairs.tolist()}
    diff = acc_g ^ acc_o
    say("candidates gpu", ncand, "oracle", ncand_o, "accepted gpu", len(acc_g), "oracle", len(acc_o),
        "differ", len(diff))
    assert ncand == ncand_o and ncand > 10 ** 6
    assert len(acc_o) > 100
    assert len(diff) <= max(3, len(acc_o) // 1000)
    assert all(_straddles(orc, x1, x0, sp, uid, L, dt, step, seed, sorted(diff)))
