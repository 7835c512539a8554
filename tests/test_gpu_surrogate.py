"""Parity of the surrogate's state kernels (features, re-population) with the
FP64 oracle, through the C ABI.

  * features: the pair-correlation shell counts are integers decided in FP32
    with Eq. 2's operation order on both sides, so the g values (FP64
    normalisation on both sides) agree to 1e-9 relative; log10 concentrations
    and log10 dt to 1e-12; normalisation (f - mu) / sd to FP32 rounding;
  * re-population: counts equal the oracle's stochastic rounding (same Philox
    counter); every new molecule lies in [-L/2, L/2)^3 with consecutive uids;
    the old molecules of the instance are gone and the other instance of the
    context is untouched; positions are uniform (KS test per axis).
"""
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

from oracle import surrogate_oracle as S  # noqa: E402
from paper_2509_03313_amd import workload as W  # noqa: E402


def say(*a):
    print("[gpu-test]", *a, flush=True)


@pytest.fixture(scope="module")
def g():
    import torch
    assert torch.cuda.is_available(), "GPU tests need the device"
    from paper_2509_03313_amd import gsbs
    return gsbs


def state(seed, L, n):
    rng = np.random.default_rng(seed)
    x = rng.uniform(-L / 2, L / 2, size=(n, 3))
    # half in tight clusters so that the short shells are populated
    c = rng.uniform(-L / 2, L / 2, size=(n // 20, 3)).repeat(10, axis=0)
    x[: len(c)] = c + rng.normal(0, 3.0, size=c.shape)
    x = ((x + L / 2) % L - L / 2).astype(np.float32)
    sp = rng.choice(7, size=n, p=[0.2, 0.25, 0.1, 0.2, 0.1, 0.1, 0.05]).astype(np.uint8)
    uid = rng.permutation(np.arange(n, dtype=np.uint64) * 3 + 5)
    return x, sp, uid


@pytest.mark.parametrize("L,n,nref", [(400.0, 3000, 100), (1000.0, 5000, 2000)])
def test_features_match_oracle(g, L, n, nref):
    x, sp, uid = state(int(L) + n, L, n)
    say("features", L, n, nref)
    e = g.Engine(L, 5, W.D_CONFIG, W.REACTIONS)
    g.gsbs_debug_set_state(e.ctx, x, sp, uid, step=2)
    got = g.gsbs_features(e.ctx, 0, 1234.5, r_max=150.0, n_ref_max=nref).astype(np.float64)
    ref = S.features(x, sp.astype(np.int64), uid, L, W.D_CONFIG, W.REACTIONS, 1234.5, r_max=150.0, n_ref_max=nref)
    assert got.shape == (296,)
    assert np.allclose(got[:7], ref[:7], rtol=0, atol=1e-5)
    assert abs(got[-1] - ref[-1]) < 1e-6
    gg, gr = got[7:-1], ref[7:-1]
    bad = np.nonzero(~np.isclose(gg, gr, rtol=2e-7, atol=0))[0]
    say("g features off", len(bad), "max g", gr.max())
    assert len(bad) == 0, (bad[:5], gg[bad[:5]], gr[bad[:5]])
    # normalisation
    mu = np.linspace(-1, 1, 296).astype(np.float32)
    sd = np.linspace(0.5, 2, 296).astype(np.float32)
    gn = g.gsbs_features(e.ctx, 0, 1234.5, r_max=150.0, n_ref_max=nref, mu=mu, sd=sd).astype(np.float64)
    assert np.allclose(gn, np.clip((ref - mu) / sd, -8, 8), rtol=1e-5, atol=1e-5)
    e.close()


def test_repopulate(g):
    L = 500.0
    say("repopulate")
    e = g.Engine([L, L], 77, W.D_CONFIG, W.REACTIONS)
    x, sp, uid = state(3, L, 2000)
    e.inject(0, 0.0, x, sp)
    e.inject(1, 0.0, x[:500], sp[:500])
    e.advance_to([5.0, 5.0])
    before1 = e.current_counts(1)
    mu = np.full(7, -6.0, dtype=np.float32)
    sd = np.full(7, 1.0, dtype=np.float32)
    y = np.array([0.1, 0.5, -0.3, 0.2, 0.0, 0.9, -1.0], dtype=np.float32)
    g.gsbs_repopulate(e.ctx, 0, 1e5, y, mu, sd)
    got = e.current_counts(0)
    assert np.array_equal(e.current_counts(1), before1)
    xs, ss, us = g.gsbs_debug_get_state(e.ctx, 0)
    assert np.all(us >= 2000)  # every old molecule is gone (uids continue the counter)
    assert np.array_equal(np.bincount(ss, minlength=7)[:7], got)
    assert np.all(xs >= -L / 2) and np.all(xs < L / 2)
    assert len(np.unique(us)) == len(us)
    # counts: the oracle's stochastic rounding with the same Philox counter
    t0 = g.gsbs_get_time(e.ctx, 0)
    assert t0 == 1e5
    n_steps = e.stats()["steps"]
    ref = S.repop_counts(y, mu, sd, L, 77, 0, n_steps)
    say("counts", got.tolist(), ref.tolist())
    assert np.array_equal(got, ref)
    from scipy import stats
    for a in range(3):
        assert stats.kstest((xs[:, a] + L / 2) / L, "uniform").pvalue > 1e-4
    # relative: y is the change of the log concentrations from the present counts
    # (same time, so the instance's step counter is still the context's)
    now = e.current_counts(0)
    g.gsbs_repopulate(e.ctx, 0, 1e5, y * 0.1, np.zeros(7, np.float32), sd, relative=True)
    ref = S.repop_counts(y * 0.1, np.zeros(7), sd, L, 77, 0, n_steps, now=now)
    say("relative counts", now.tolist(), e.current_counts(0).tolist(), ref.tolist())
    assert np.array_equal(e.current_counts(0), ref)
    # the instance keeps stepping from its new time
    e.advance_to([1.5e5, 1.5e5])
    assert g.gsbs_get_time(e.ctx, 0) == 1.5e5
    e.close()


def test_surrogate_pipeline(g):
    """Samples from batched plain SBS runs, training on the device kernels, and
    the hybrid schedule: the trained network predicts the next-pulse log
    concentrations better than carrying the switch-time state over unchanged
    (the method without the network would have to simulate the interval) by a
    clear margin on held-out runs of 1 um cubes, where the count noise of ~50
    H2O2 molecules per pulse bounds what any predictor can reach, and
    a hybrid run hands intervals to it and takes fewer SBS steps."""
    from paper_2509_03313_amd import surrogate as SU
    plans = SU.random_plans(1, 48, L=1000.0, n_pulses=4, rates=(500.0, 5000.0), doses=(0.5, 1.5))
    say("surrogate pipeline: generating")
    data = SU.generate(plans, seed=3)
    n = len(data["X"])
    assert n == 48 * 3 and data["X"].shape == (n, 296)
    idx = np.random.default_rng(0).permutation(n)
    tr, he = idx[:112], idx[112:]
    sub = lambda d, k: {key: v[k] for key, v in d.items()}  # noqa: E731
    s = SU.Surrogate(256)
    s.init_weights(0)
    hist = s.fit(sub(data, tr), epochs=40, batch=16, lr=5e-4)
    held = sub(data, he)
    pred = s.predict_log(held["X"], held["Y0"])
    h = SU.H2O2
    true = 10.0 ** held["Y1"][:, h]
    err_net = float(np.mean(np.abs(10.0 ** pred[:, h] - true) / true))
    err_carry = float(np.mean(np.abs(10.0 ** held["Y0"][:, h] - true) / true))
    say("loss", hist[0], "->", hist[-1], "held-out mean relative H2O2 error: network", err_net, "carry", err_carry)
    say("per-species mean |dlog10 C| network", np.mean(np.abs(pred - held["Y1"]), axis=0).round(3).tolist(),
        "carry", np.mean(np.abs(held["Y0"] - held["Y1"]), axis=0).round(3).tolist())
    assert hist[-1] < hist[0] and err_net < 0.75 * err_carry
    s.build_table(sub(data, tr))
    s.table[:] = 0.0  # let the network take every interval in range
    plan = SU.PulsePlan(1000.0, 99, 3, 1.0, 1e6, 1000.0)
    hyb = SU.run(plan, s, tol=1.0)
    plain = SU.run(plan, None)
    say("hybrid", hyb["intervals_by_network"], hyb["steps"], hyb["n_h2o2"].tolist(), "plain", plain["steps"],
        plain["n_h2o2"].tolist())
    assert hyb["intervals_by_network"] >= 1 and hyb["steps"] < plain["steps"]
    # a budget on the summed error estimate: with 0.6 % per interval, 1 % admits one
    s.table[:] = 0.006
    hyb_b = SU.run(plan, s, tol=1.0, budget=0.01)
    say("budgeted hybrid", hyb_b["intervals_by_network"], hyb_b["error_estimate_spent"])
    assert hyb_b["intervals_by_network"] == 1 and abs(hyb_b["error_estimate_spent"] - 0.006) < 1e-12


def _two_cube_engine(g, SU):
    plans = [SU.PulsePlan(1000.0, 40 + i, 3, 1.0, 1e6, 1000.0) for i in range(2)]
    e = g.Engine([p.L for p in plans], 17, W.D_CONFIG, W.REACTIONS)
    for i, p in enumerate(plans):
        for j in p.injections():
            e.inject(i, j.t, j.xyz, j.species, j.edep_ev)
        e.set_records(i, np.unique(np.concatenate([W.log_times(1e-3, 3e6, 40), [p.switch(0), p.start(1)]])))
    return e, plans


def _net(g, SU):
    s = SU.Surrogate(16)
    s.init_weights(5)
    s.mu = np.zeros(296, np.float32)
    s.sd = np.ones(296, np.float32)
    s.mu_y = np.zeros(7, np.float32)
    s.sd_y = np.full(7, 0.01, np.float32)
    s.dt_edges = np.array([3.0, 6.0, 9.0])
    s.c_edges = np.array([-12.0, -6.0, 0.0])
    return s


def test_surrogate_mode_declining_every_interval_is_plain_bit_for_bit(g):
    """gsbs_advance_to(GSBS_SURROGATE) with a table of +inf takes no interval:
    records, final counts and stats equal the GSBS_PLAIN advance (hand-over
    points are step ends in both modes while a surrogate is set)."""
    from paper_2509_03313_amd import surrogate as SU
    s = _net(g, SU)
    s.table = np.full((2, 2), np.inf)
    out = []
    for mode in (g.GSBS_PLAIN, g.GSBS_SURROGATE):
        e, plans = _two_cube_engine(g, SU)
        SU.set_on(e, s)
        e.advance_to(3e6, mode)
        out.append(([e.counts(i) for i in range(2)], [e.current_counts(i) for i in range(2)], e.stats(),
                     [g.gsbs_get_handover_log(e.ctx, i) for i in range(2)]))
        e.close()
    (ca, na, sa, _), (cb, nb, sb, lb) = out
    for i in range(2):
        assert np.array_equal(ca[i], cb[i]) and np.array_equal(na[i], nb[i])
        assert len(lb[i]["taken"]) == 2 and not lb[i]["taken"].any() and np.all(np.isinf(lb[i]["estimate"]))
    # max_live is sampled at synchronisation points, which the hand-over stops add
    keys = ("steps", "molecule_steps", "reactions", "pair_candidates")
    assert {k: sa[k] for k in keys} == {k: sb[k] for k in keys}
    say("declined hand-overs:", lb[0]["t_switch"].tolist(), "steps", sb["steps"])


def test_surrogate_mode_zero_table_hands_every_interval_over(g):
    """A zero table with no input-range guard hands every inter-pulse interval
    to the network: both cubes are re-populated at each next pulse start,
    records inside the handed-over intervals stay empty, and fewer SBS steps
    run; gsbs_pair_corr gives the features' pair-correlation block."""
    from paper_2509_03313_amd import surrogate as SU
    s = _net(g, SU)
    s.table = np.zeros((2, 2))
    s.lo = s.hi = None
    e, plans = _two_cube_engine(g, SU)
    e.advance_to(plans[0].switch(0) - 1.0)
    pc = g.gsbs_pair_corr(e.ctx, 0, 150.0, 512)
    feat = g.gsbs_features(e.ctx, 0, 1.0, r_max=150.0, n_ref_max=512)
    assert pc.shape == (9, 32) and np.array_equal(pc.ravel(), feat[7:7 + 288])
    SU.set_on(e, s)
    e.advance_to(3e6, g.GSBS_SURROGATE)
    for i in range(2):
        lg = g.gsbs_get_handover_log(e.ctx, i)
        assert lg["taken"].all() and len(lg["taken"]) == 2, lg
        assert np.allclose(lg["t_next"], [plans[i].start(1), plans[i].start(2)])
        c = e.counts(i)
        r = e.records[i]
        inside = np.zeros(len(r), dtype=bool)
        for ts, tn in zip(lg["t_switch"], lg["t_next"]):
            inside |= (r > ts) & (r < tn)
        assert inside.any() and np.all(c[inside] == -1)
        assert np.all(c[~inside] >= 0)
    steps_sur = e.stats()["steps"]
    e.close()
    e, _ = _two_cube_engine(g, SU)
    e.advance_to(3e6)
    assert steps_sur < e.stats()["steps"]
    e.close()
    with pytest.raises(g.GsbsError):  # no surrogate set
        e, _ = _two_cube_engine(g, SU)
        try:
            e.advance_to(10.0, g.GSBS_SURROGATE)
        finally:
            e.close()
