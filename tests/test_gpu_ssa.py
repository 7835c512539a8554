"""Parity of the stochastic-kinetics kernel (Gillespie's direct method) with
the oracle, through the C ABI.

Both sides draw the same Philox words and choose every reaction in FP64 from
exact integer pair counts in the same order, so a stream's event sequence is
the same on both: the recorded counts must be identical.  Only the event
times carry the rounding of ln (device and host libraries may differ by an
ulp), so a record time that falls within 1e-9 (relative) of an oracle event
may see the state just before or just after that event.
"""
import math
import os
import sys

import numpy as np
import pytest
from scipy.linalg import expm

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

from oracle import ssa_oracle as S  # noqa: E402
from paper_2509_03313_amd import workload as W  # noqa: E402

NA = 6.02214076e23


def say(*a):
    print("[gpu-test]", *a, flush=True)


@pytest.fixture(scope="module")
def g():
    import torch
    assert torch.cuda.is_available(), "GPU tests need the device"
    from paper_2509_03313_amd import gsbs
    return gsbs


def _same_as_oracle(out, events, reactions, ns, n0, vols, t_rec, seed, stream0, members):
    """Compare the device records of the given volumes with the oracle's."""
    for m in members:
        ref, ne, (ev_t, ev_r) = S.ssa(reactions, ns, n0[m], vols[m], t_rec, seed, stream0 + m,
                                      log_events=1 << 22)
        assert ne >= 0 and len(ev_t) == ne
        for k, tk in enumerate(t_rec):
            if np.array_equal(out[m, k], ref[k]):
                continue
            near = np.abs(ev_t - tk) <= 1e-9 * max(tk, 1e-300)
            assert near.any(), (m, k, out[m, k], ref[k])
            # the device may have put the tied event on the other side
            j = int(np.argmax(near))
            before, _, _ = S.ssa(reactions, ns, n0[m], vols[m], [ev_t[j] * (1 - 1e-12)], seed, stream0 + m)
            after, _, _ = S.ssa(reactions, ns, n0[m], vols[m], [ev_t[j]], seed, stream0 + m)
            assert np.array_equal(out[m, k], before[0]) or np.array_equal(out[m, k], after[0]), (m, k)
        if events is not None:
            assert abs(int(events[m]) - ne) <= 1 and (events[m] == ne or np.any(
                np.abs(ev_t - t_rec[-1]) <= 1e-9 * t_rec[-1])), (m, events[m], ne)


def test_water_scheme_event_for_event(g):
    n = 70  # one full wave and a ragged one
    rng = np.random.default_rng(3)
    vols = 10.0 ** rng.uniform(-19, -17.5, size=n)
    c0 = np.array([2.8e-5, 2.9e-5, 6e-6, 2.9e-5, 5e-6, 1e-6, 1e-6])
    n0 = np.rint(c0[None, :] * NA * vols[:, None] * rng.uniform(0.5, 2.0, size=(n, 7))).astype(np.int32)
    t_rec = np.concatenate([[0.0], np.geomspace(1.0, 1e6, 25)])
    e = g.Engine(1000.0, 1, W.D_CONFIG, W.REACTIONS)
    out, ev = g.gsbs_ssa(e.ctx, n0, vols, t_rec, seed=21, stream0=100)
    e.close()
    say("events", ev.min(), ev.max(), "molecules", n0.sum(axis=1).min(), n0.sum(axis=1).max())
    assert out.shape == (n, len(t_rec), 7) and np.all(ev > 0)
    _same_as_oracle(out, ev, W.REACTIONS, 7, n0, vols, t_rec, 21, 100, range(n))


def test_master_equation_on_device(g):
    # A + A -> B from 9 molecules: the exact distribution of n_A
    r = [W.Reaction("X", 0, 0, 0.95, (1,))]
    V = 1e-18
    c = 9.5 / (NA * V)
    n = 8192
    t = np.array([2e3, 1e4, 6e4])
    e = g.Engine(1000.0, 1, [1.0, 1.0], r)
    out, ev = g.gsbs_ssa(e.ctx, np.tile([9, 0], (n, 1)), np.full(n, V), t, seed=5)
    states = list(range(9, -1, -2))
    Q = np.zeros((5, 5))
    for i, a in enumerate(states[:-1]):
        rate = c * a * (a - 1) / 2
        Q[i + 1, i] += rate
        Q[i, i] -= rate
    for k, tk in enumerate(t):
        p = expm(Q * tk)[:, 0]
        for st, pk in zip(states, p):
            ph = np.mean(out[:, k, 0] == st)
            assert abs(ph - pk) <= 4.5 * math.sqrt(pk * (1 - pk) / n) + 1.5 / n, (tk, st, ph, pk)
    assert np.all(2 * out[:, :, 1] + out[:, :, 0] == 9)
    # a sample of the same run, event for event
    _same_as_oracle(out, ev, r, 2, np.tile([9, 0], (n, 1)), np.full(n, V), t, 5, 0, range(0, n, 997))
    e.close()


def test_edges_and_errors(g):
    r = [W.Reaction("X", 0, 1, 0.5, (2,))]
    e = g.Engine(1000.0, 1, [1.0, 1.0, 1.0], r)
    out, ev = g.gsbs_ssa(e.ctx, np.zeros((0, 3)), np.zeros(0), [1.0], seed=1)
    assert out.shape == (0, 1, 3)
    # a record at 0 sees the start; nothing can react: no events
    out, ev = g.gsbs_ssa(e.ctx, [[5, 5, 0], [5, 0, 2]], [1e-18, 1e-18], [0.0, 1e12], seed=1)
    assert list(out[0, 0]) == [5, 5, 0] and list(out[0, 1]) == [0, 0, 5] and ev[0] == 5
    assert np.all(out[1] == [5, 0, 2]) and ev[1] == 0
    with pytest.raises(g.GsbsError):  # event limit
        g.gsbs_ssa(e.ctx, [[50, 50, 0]], [1e-18], [1e12], seed=1, max_events=10)
    with pytest.raises(g.GsbsError):  # layout
        g.gsbs_ssa(e.ctx, [[5, 5]], [1e-18], [1.0], seed=1)
    with pytest.raises(g.GsbsError):  # descending records
        g.gsbs_ssa(e.ctx, [[5, 5, 0]], [1e-18], [2.0, 1.0], seed=1)
    with pytest.raises(g.GsbsError):  # negative count
        g.gsbs_ssa(e.ctx, [[-1, 5, 0]], [1e-18], [1.0], seed=1)
    with pytest.raises(g.GsbsError):  # volume
        g.gsbs_ssa(e.ctx, [[1, 5, 0]], [0.0], [1.0], seed=1)
    e.close()


def test_device_tensors_match_host_arrays(g):
    import torch
    n = 300
    L = 200.0
    n0 = np.tile(W.volume_scaling_counts(L).astype(np.int32), (n, 1))
    V = L ** 3 * 1e-24  # nm^3 -> litres
    t_rec = np.geomspace(1.0, 1e4, 12)
    e = g.Engine(1000.0, 1, W.D_CONFIG, W.REACTIONS)
    h, evh = g.gsbs_ssa(e.ctx, n0, np.full(n, V), t_rec, seed=9)
    d, evd = g.gsbs_ssa(e.ctx, torch.as_tensor(n0, device="cuda"), torch.full((n,), V, dtype=torch.float64,
                        device="cuda"), t_rec, seed=9)
    e.close()
    assert np.array_equal(h, d.cpu().numpy()) and np.array_equal(evh, evd)
    _same_as_oracle(h, evh, W.REACTIONS, 7, n0, np.full(n, V), t_rec, 9, 0, (0, 151, n - 1))


def test_volume_scaling_cube_sampled(g):
    # the 1 um cube of the volume-scaling mixture (250 000 molecules), a few
    # sampled realisations event for event
    L = 1000.0
    n = 64
    n0 = np.tile(W.volume_scaling_counts(L).astype(np.int32), (n, 1))
    V = L ** 3 * 1e-24
    t_rec = np.concatenate([[0.0], np.geomspace(1e-3, 1e4, 40)])
    e = g.Engine(1000.0, 1, W.D_CONFIG, W.REACTIONS)
    out, ev = g.gsbs_ssa(e.ctx, n0, np.full(n, V), t_rec, seed=17)
    e.close()
    say("events per realisation", ev.min(), ev.max())
    _same_as_oracle(out, ev, W.REACTIONS, 7, n0, np.full(n, V), t_rec, 17, 0, (0, 33, 63))


def test_rate_equations_match_ensemble_mean(g):
    """The paper finds its rate equations and the Gillespie reference within
    1 % of each other for a homogeneous mixture; the device's two solvers on
    the volume-scaling mixture in a 0.5 um cube must agree the same way."""
    L = 500.0
    V = L ** 3 * 1e-24
    n0 = W.volume_scaling_counts(L)
    n = 512
    t_rec = np.concatenate([[0.0], np.geomspace(1e-2, 1e4, 30)])
    e = g.Engine(1000.0, 1, W.D_CONFIG, W.REACTIONS)
    out, ev = g.gsbs_ssa(e.ctx, np.tile(n0.astype(np.int32), (n, 1)), np.full(n, V), t_rec, seed=23)
    ode, _ = g.gsbs_numodes(e.ctx, np.tile(n0 / (NA * V), (len(t_rec), 1)), t_rec, rtol=1e-8)
    e.close()
    ode *= NA * V
    mean = out.mean(axis=0)
    se = out.std(axis=0, ddof=1) / math.sqrt(n)
    say("events per realisation", ev.min(), ev.max())
    ok = mean >= 200
    assert np.all(np.abs(mean - ode)[ok] <= 0.01 * ode[ok] + 3 * se[ok])


def test_sources_event_for_event(g):
    """The water scheme with R9's reverse (a zero-order source) and the pH 7
    background, event for event against the oracle."""
    n = 40
    V = 1e-17
    n0 = S.counts_from_conc([2e-6, 2e-6, 3e-7, 2e-6 + 1e-7, 1e-7, 1e-7, 1e-7], V)
    n0 = np.tile(n0.astype(np.int32), (n, 1))
    t_rec = np.concatenate([[0.0], np.geomspace(1.0, 1e7, 20)])
    e = g.Engine(1000.0, 1, W.D_CONFIG, W.REACTIONS)
    g.gsbs_set_sources(e.ctx, W.SOURCES_PH7)
    out, ev = g.gsbs_ssa(e.ctx, n0, np.full(n, V), t_rec, seed=31)
    e.close()
    say("events", ev.min(), ev.max())
    fired = 0
    for m in range(n):
        ref, ne, (ev_t, ev_r) = S.ssa(W.REACTIONS, 7, n0[m], V, t_rec, 31, m, log_events=1 << 22,
                                      sources=W.SOURCES_PH7)
        assert ne >= 0
        fired += int(np.sum(ev_r == len(W.REACTIONS)))
        for k, tk in enumerate(t_rec):
            if not np.array_equal(out[m, k], ref[k]):
                assert np.any(np.abs(ev_t - tk) <= 1e-9 * tk), (m, k, out[m, k], ref[k])
    # the source took part: its events are in the compared sequences
    say("source events", fired)
    assert fired > 0


def test_first_order_event_for_event(g):
    """Aerated water with the pH 7 source: first-order channels, sources and
    reactions, event for event against the oracle."""
    n = 40
    V = 1e-17
    n0 = S.counts_from_conc([2e-6, 2e-6, 3e-7, 2e-6 + 1e-7, 1e-7, 1e-7, 1e-7, 0.0], V)
    n0 = np.tile(n0.astype(np.int32), (n, 1))
    t_rec = np.concatenate([[0.0], np.geomspace(1.0, 1e7, 20)])
    e = g.Engine(1000.0, 1, W.D_CONFIG_O2, W.REACTIONS_O2)
    g.gsbs_set_first_order(e.ctx, W.FIRST_ORDER_O2)
    g.gsbs_set_sources(e.ctx, W.SOURCES_PH7)
    out, ev = g.gsbs_ssa(e.ctx, n0, np.full(n, V), t_rec, seed=37)
    e.close()
    fo_events = 0
    for m in range(n):
        ref, ne, (ev_t, ev_r) = S.ssa(W.REACTIONS_O2, 8, n0[m], V, t_rec, 37, m, log_events=1 << 22,
                                      sources=W.SOURCES_PH7, first_order=W.FIRST_ORDER_O2)
        assert ne >= 0
        fo_events += int(np.sum((ev_r >= len(W.REACTIONS_O2)) & (ev_r < len(W.REACTIONS_O2) + 2)))
        for k, tk in enumerate(t_rec):
            if not np.array_equal(out[m, k], ref[k]):
                assert np.any(np.abs(ev_t - tk) <= 1e-9 * tk), (m, k, out[m, k], ref[k])
    say("first-order events", fo_events)
    assert fo_events > 0


def test_sbs_pbc_volume_scaling(g):
    """The paper's PBC verification on the device: the volume-scaling mixture
    in 0.2, 0.5 and 1 um cubes, all on the same step times (the 0.2 um cube's
    step cap), gives the same concentrations at every record within 4.5
    standard errors of the cube-to-cube scatter (plus the per-cube rounding of
    the initial counts, and 1e-3 of the value); from 1 us on each edge stays within
    25 % of the mean of Gillespie runs in the same volume (the paper reports
    SBS + PBCs up to 20 % from its Gillespie reference: diffusion-controlled
    rates that homogeneous kinetics leave out)."""
    t_end = 1e4
    rec = np.concatenate([[0.0], W.log_times(1e-3, t_end, 30)])
    rec[-1] = t_end
    e = g.Engine(200.0, 1, W.D_CONFIG, W.REACTIONS)
    cap = e.dt_max()
    e.close()
    cubes = {200.0: 64, 500.0: 8, 1000.0: 4}
    per, ssa = {}, {}
    for L, k in cubes.items():
        say("volume scaling SBS", L, k)
        p = g.gsbs_default_params()
        p.dt_max_ns = cap
        e = g.Engine([L] * k, 7, W.D_CONFIG, W.REACTIONS, params=p)
        for i in range(k):
            wl = W.volume_scaling(5000 + 100 * i + int(L), L, t_end=t_end)
            e.inject(i, 0.0, wl.injections[0].xyz, wl.injections[0].species)
            e.set_records(i, rec)
        e.advance_to(t_end)
        per[L] = np.stack([e.counts(i) for i in range(k)]).astype(np.float64) / (L / 1000.0) ** 3
        e.close()
        V = L ** 3 * 1e-24
        e = g.Engine(L, 1, W.D_CONFIG, W.REACTIONS)
        n_r = 1024
        out, _ = g.gsbs_ssa(e.ctx, np.tile(W.volume_scaling_counts(L).astype(np.int32), (n_r, 1)), np.full(n_r, V),
                            rec, seed=41)
        e.close()
        ssa[L] = out.mean(axis=0) / (L / 1000.0) ** 3
    ref = per[200.0]
    for L in (500.0, 1000.0):
        a, b = ref, per[L]
        d = np.abs(a.mean(axis=0) - b.mean(axis=0))
        se = np.sqrt(a.var(axis=0, ddof=1) / len(a) + b.var(axis=0, ddof=1) / len(b))
        # initial counts are rounded per cube: their difference per um^3 is carried as slack
        init = np.abs(W.volume_scaling_counts(200.0) / 0.2 ** 3 - W.volume_scaling_counts(L) / (L / 1000.0) ** 3)
        lim = 4.5 * se + 1.5 * init[None, :] + 1e-3 * a.mean(axis=0)
        use = b.mean(axis=0) * (L / 1000.0) ** 3 >= 20
        z = (d / np.maximum(se, 1e-9))[use]
        say("edge", L, "vs 0.2 um: largest |diff| / SE", float(z.max()))
        assert np.all(d[use] <= lim[use])
    late = rec >= 1e3
    for L in cubes:
        m = per[L].mean(axis=0)
        ok = late[:, None] & (ssa[L] * (L / 1000.0) ** 3 >= 50)
        r = m[ok] / ssa[L][ok]
        say("edge", L, "SBS / Gillespie after 1 us", float(r.min()), float(r.max()))
        assert np.all((r > 0.75) & (r < 1.33))
