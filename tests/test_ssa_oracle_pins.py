"""Pins of the stochastic-kinetics oracle (Gillespie's direct method; CPU only).

  * A + B -> C and A + A -> B from a handful of molecules: the distribution of
    the counts over 4000 realisations against the exact solution of the
    chemical master equation (the generator's matrix exponential over the few
    reachable states) -- a wrong pair count (n(n-1) instead of n(n-1)/2), a
    wrong constant or a wrong waiting-time law moves it by many sigma;
  * a sink A + S -> S with S kept: survivors binomial with p = exp(-c n_S t);
  * the water scheme in a large volume: ensemble means within 1 % of the rate
    equations (the paper finds its rate equations and the Gillespie reference
    within 1 % of each other for such a mixture);
  * charge and redox balance conserved exactly in every realisation;
  * zero-order sources: Poisson counts alone, and with R9 the pH 7 background
    held at its equilibrium;
  * edge cases: records before the first event, no possible reaction, the
    event limit, and determinism of the counter-based random numbers.
"""
import math
import os
import sys

import numpy as np
from scipy.linalg import expm

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

from oracle import numodes_oracle as N  # noqa: E402
from oracle import ssa_oracle as S  # noqa: E402
from paper_2509_03313_amd import workload as W  # noqa: E402

NA = 6.02214076e23


def _cme(rates, p0, t):
    """Exact distribution at t of a one-way chain of states i -> i+1 with
    rates[i] (the last state absorbing)."""
    m = len(p0)
    Q = np.zeros((m, m))
    for i in range(m - 1):
        Q[i + 1, i] += rates[i]
        Q[i, i] -= rates[i]
    return expm(Q * t) @ p0


def _check_hist(samples, states, p, n):
    for st, pk in zip(states, p):
        ph = np.mean(samples == st)
        assert abs(ph - pk) <= 4.5 * math.sqrt(pk * (1 - pk) / n) + 1.5 / n, (st, ph, pk)


def test_a_plus_b_master_equation():
    r = [W.Reaction("X", 0, 1, 0.5, (2,))]
    V = 1e-18
    c = 5.0 / (NA * V)
    nA0, nB0 = 6, 4
    t = np.array([5e3, 2e4, 8e4])
    ens = S.ensemble(r, 3, [nA0, nB0, 0], V, t, seed=11, n_real=4000)
    states = list(range(nA0, nA0 - nB0 - 1, -1))  # n_A
    rates = [c * a * (a - (nA0 - nB0)) for a in states]
    p0 = np.zeros(len(states))
    p0[0] = 1.0
    for k, tk in enumerate(t):
        _check_hist(ens[:, k, 0], states, _cme(rates, p0, tk), len(ens))
    # stoichiometry: every event turns one A and one B into one C
    assert np.all(ens[:, :, 0] - ens[:, :, 1] == nA0 - nB0)
    assert np.all(ens[:, :, 2] == nA0 - ens[:, :, 0])


def test_self_recombination_master_equation():
    r = [W.Reaction("X", 0, 0, 0.95, (1,))]
    V = 1e-18
    c = 9.5 / (NA * V)
    n0 = 9
    t = np.array([2e3, 1e4, 6e4])
    ens = S.ensemble(r, 2, [n0, 0], V, t, seed=12, n_real=4000)
    states = list(range(n0, -1, -2))
    rates = [c * a * (a - 1) / 2 for a in states]
    p0 = np.zeros(len(states))
    p0[0] = 1.0
    for k, tk in enumerate(t):
        _check_hist(ens[:, k, 0], states, _cme(rates, p0, tk), len(ens))
    assert np.all(2 * ens[:, :, 1] + ens[:, :, 0] == n0)


def test_sink_is_binomial():
    r = [W.Reaction("S", 0, 1, 0.2, (), keep_b=True)]
    V = 1e-17
    c = 2.0 / (NA * V)
    n0, ns = 40, 50
    t = np.array([2e3, 1e4])
    ens = S.ensemble(r, 2, [n0, ns], V, t, seed=13, n_real=3000)
    assert np.all(ens[:, :, 1] == ns)
    for k, tk in enumerate(t):
        p = math.exp(-c * ns * tk)
        states = list(range(n0 + 1))
        pk = [math.comb(n0, s) * p ** s * (1 - p) ** (n0 - s) for s in states]
        _check_hist(ens[:, k, 0], states, pk, len(ens))


def test_water_scheme_large_volume_follows_rate_equations():
    c0 = np.array([2.8e-5, 2.9e-5, 6e-6, 2.9e-5, 5e-6, 1e-6, 1e-6])  # mol/L
    V = 1e-15
    n0 = S.counts_from_conc(c0, V)
    t = np.array([1e2, 1e3, 1e4, 1e5])
    ens = S.ensemble(W.REACTIONS, 7, n0, V, t, seed=14, n_real=8)
    c0x = n0 / (NA * V)
    for k, tk in enumerate(t):
        ref = N.integrate(c0x, tk, W.REACTIONS) * NA * V
        mean = ens[:, k, :].mean(axis=0)
        se = ens[:, k, :].std(axis=0, ddof=1) / math.sqrt(len(ens))
        for s in range(7):
            if ref[s] >= 200:
                assert abs(mean[s] - ref[s]) <= 0.01 * ref[s] + 3 * se[s], (tk, s, mean[s], ref[s])
    Q = ens[..., W.H3O] - ens[..., W.E_AQ] - ens[..., W.OHM]
    R = ens[..., W.OH] + 2 * ens[..., W.H2O2] - ens[..., W.E_AQ] - ens[..., W.H] - 2 * ens[..., W.H2]
    assert np.all(Q == n0[W.H3O] - n0[W.E_AQ] - n0[W.OHM])
    assert np.all(R == n0[W.OH] + 2 * n0[W.H2O2] - n0[W.E_AQ] - n0[W.H] - 2 * n0[W.H2])


def test_edges_and_determinism():
    r = [W.Reaction("X", 0, 1, 0.5, (2,))]
    # a record at t = 0 sees the initial state (waiting times are > 0)
    out, ne, _ = S.ssa(r, 3, [5, 5, 0], 1e-18, [0.0, 1e9], 1, 0)
    assert list(out[0]) == [5, 5, 0] and list(out[1]) == [0, 0, 5] and ne == 5
    # nothing can react: every record is the initial state, no events
    out, ne, _ = S.ssa(r, 3, [5, 0, 2], 1e-18, [0.0, 1.0, 1e12], 1, 0)
    assert ne == 0 and np.all(out == [5, 0, 2])
    # the event limit
    _, ne, _ = S.ssa(r, 3, [50, 50, 0], 1e-18, [1e12], 1, 0, max_events=10)
    assert ne == -1
    # same stream, same trajectory; another stream, another one
    a = S.ssa(r, 3, [50, 50, 0], 1e-18, [1e3, 1e4], 3, 7, log_events=100)
    b = S.ssa(r, 3, [50, 50, 0], 1e-18, [1e3, 1e4], 3, 7, log_events=100)
    c = S.ssa(r, 3, [50, 50, 0], 1e-18, [1e3, 1e4], 3, 8, log_events=100)
    assert np.array_equal(a[2][0], b[2][0]) and not np.array_equal(a[2][0][:5], c[2][0][:5])
    # event times increase; the recorded state is the one after the events up to the record
    ev_t = a[2][0]
    assert np.all(np.diff(ev_t) > 0)
    assert a[0][0][2] == np.sum(ev_t <= 1e3)


def test_source_alone_is_poisson():
    src = [W.Source("S", 1e-12, (0, 1))]
    V = 1e-16
    lam = 1e-12 * NA * V  # per ns
    t = np.array([50.0, 200.0])
    ens = S.ensemble([], 2, [0, 3], V, t, seed=15, n_real=3000, sources=src)
    assert np.all(ens[:, :, 1] - ens[:, :, 0] == 3)
    for k, tk in enumerate(t):
        mu = lam * tk
        states = list(range(0, int(mu + 8 * math.sqrt(mu) + 10)))
        pk = [math.exp(-mu) * mu ** s / math.factorial(s) for s in states]
        _check_hist(ens[:, k, 0], states, pk, len(ens))


def test_autoionisation_holds_the_background():
    # pH 7 background with R9 and its reverse: the mean ion count stays at
    # 1e-7 mol/L (up to the O(1/N) stochastic correction)
    r9 = [W.Reaction("R9", 0, 1, 11.0, ())]
    V = 1e-14  # 602 ions of each kind
    n_eq = 1e-7 * NA * V
    n0 = [int(round(n_eq))] * 2
    t = np.array([1e5, 1e6])
    src = [W.Source("R9 reverse", W.SOURCES_PH7[0].rate, (0, 1))]
    ens = S.ensemble(r9, 2, n0, V, t, seed=16, n_real=64, sources=src)
    assert np.all(ens[:, :, 0] == ens[:, :, 1])
    m = ens[:, :, 0].mean()
    assert abs(m - n_eq) <= 0.02 * n_eq, (m, n_eq)


def test_first_order_channel_is_binomial():
    fo = [W.FirstOrder("A", 0, 2e-3, (1,))]
    t = np.array([100.0, 700.0])
    ens = S.ensemble([], 2, [30, 0], 1e-18, t, seed=17, n_real=3000, first_order=fo)
    assert np.all(ens[:, :, 0] + ens[:, :, 1] == 30)
    for k, tk in enumerate(t):
        p = math.exp(-2e-3 * tk)
        states = list(range(31))
        pk = [math.comb(30, s) * p ** s * (1 - p) ** (30 - s) for s in states]
        _check_hist(ens[:, k, 0], states, pk, len(ens))
