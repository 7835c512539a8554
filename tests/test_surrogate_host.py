"""Host logic of the inter-pulse surrogate (CPU only): pulse plans and the
decision rule that sends an interval to the network or to plain SBS."""
import math
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))


def test_pulse_plan_times_and_energy():
    from paper_2509_03313_amd import surrogate as SU
    from paper_2509_03313_amd import workload as W
    pl = SU.PulsePlan(2000.0, 3, 4, 1.0, 1e6, 1e3, n_batches=2)
    assert pl.width == 1000.0 and pl.period == 1e6
    # hand-over: the settle time after the pulse's last injection (batch 2 at +500 ns)
    assert pl.start(2) == 2e6 and pl.switch(1) == 1e6 + 500.0 + SU.TAU_SETTLE
    inj = pl.injections()
    assert sorted({j.t for j in inj}) == [p * 1e6 + b * 500.0 for p in range(4) for b in range(2)]
    # energy per pulse: tracks x L x LET, tracks from Eq. 5 at 1 Gy
    n_tr = round(W.tracks_per_gray(2000.0))
    e_pulse = sum(j.edep_ev for j in inj if j.t < 1e6)
    assert abs(e_pulse - n_tr * 2000.0 * W.LET_KEV_PER_UM) < 1e-6
    assert pl.edep_until(1e6 - 1e-9, inj) == e_pulse
    # the same plan gives the same molecules
    inj2 = SU.PulsePlan(2000.0, 3, 4, 1.0, 1e6, 1e3, n_batches=2).injections()
    assert all(np.array_equal(a.xyz, b.xyz) and np.array_equal(a.species, b.species) for a, b in zip(inj, inj2))


def test_decision_rule():
    """An interval goes to the network only inside the table's ranges, inside
    the training range of every input (10 % margin) and where the table's
    95th-percentile error is at most the tolerance."""
    from paper_2509_03313_amd import surrogate as SU
    s = object.__new__(SU.Surrogate)
    s.table = np.array([[0.004, 0.02], [0.009, np.inf]])
    s.dt_edges = np.array([5.0, 6.0, 7.0])
    s.c_edges = np.array([-7.0, -6.5, -6.0])
    s.lo, s.hi = -np.ones(4), np.ones(4)
    x = np.zeros(4)
    assert s.usable(5.5, 10 ** -6.8, x)          # bin (0, 0): 0.4 %
    assert not s.usable(5.5, 10 ** -6.2, x)      # bin (0, 1): 2 %
    assert s.usable(6.5, 10 ** -6.8, x)          # bin (1, 0): 0.9 %
    assert not s.usable(6.5, 10 ** -6.2, x)      # empty bin
    assert not s.usable(4.9, 10 ** -6.8, x)      # outside the dt range
    assert not s.usable(5.5, 10 ** -5.9, x)      # outside the C_tot range
    assert not s.usable(5.5, 10 ** -6.8, np.array([0, 0, 1.25, 0]))  # input outside the training range
    assert s.usable(5.5, 10 ** -6.8, np.array([0, 0, 1.15, 0]))      # inside the 10 % margin
    assert not s.usable(6.5, 10 ** -6.8, x, tol=0.005)
    s.table = None
    assert not s.usable(5.5, 10 ** -6.8, x)
