"""Trend pins of the dose-rate study (SBS + rate equations over pulse trains,
2 um cube, 1 us pulses).  The paper's absolute yields depend on its physical
and physico-chemical stages, which are not part of this engine (a synthetic
spur model stands in), so only its qualitative findings are pinned:

  * below a threshold average dose rate the mixture reaches its steady state
    between pulses: almost no radicals (e_aq, OH, H) stand at the next pulse;
    above it they build up;
  * the threshold rises with the pulse dose rate (the paper: ~10 Gy/s at
    2e5 Gy/s, ~100 Gy/s at 1e6 Gy/s): at 10 Gy/s the 0.2 Gy pulses leave more
    radicals standing than the 1 Gy pulses;
  * at 2e5 Gy/s the H2O2 yield rises from the steady-state regime to the
    build-up regime (the paper: +30 %);
  * in the steady-state regime the 1e6 Gy/s pulses give more H2O2 per dose
    than the 2e5 Gy/s pulses (the paper: +26 %);
  * the post-irradiation yield rises with the average dose rate for both
    pulse dose rates, more for the weaker pulses (the paper: +30 %, +20 %).
The engine is deterministic for given seeds, so the values are reproducible;
the margins below are several standard errors of the seed scatter measured
over the full grid.
"""
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))


def say(*a):
    print("[gpu-test]", *a, flush=True)


def test_dose_rate_trends():
    import torch
    assert torch.cuda.is_available(), "GPU tests need the device"
    from paper_2509_03313_amd import dose_rate as DR
    trains = []
    for s in range(3):
        trains.append(DR.Train(2e5, 1.0, 0.2, 50, seed=10 + s))
        trains.append(DR.Train(2e5, 10.0, 0.2, 50, seed=20 + s))
        trains.append(DR.Train(2e5, 1e4, 0.2, 50, seed=30 + s))
        trains.append(DR.Train(1e6, 1.0, 1.0, 10, seed=40 + s))
        trains.append(DR.Train(1e6, 10.0, 1.0, 10, seed=50 + s))
        trains.append(DR.Train(1e6, 1e5, 1.0, 10, seed=60 + s))
    say("running", len(trains), "pulse trains")
    r = DR.run(trains)
    say("wall", round(r["wall"], 1), "s")

    def pick(dp, rate):
        idx = [k for k, t in enumerate(trains) if t.pulse_rate == dp and t.avg_rate == rate]
        g = float(np.mean([r["g_h2o2"][k] for k in idx]))
        b = float(np.mean([DR.build_up(trains[k], r["counts"][k]) for k in idx]))
        gp = float(np.mean([r["g_h2o2_post"][k] for k in idx]))
        say(dp, rate, "G(H2O2)", round(g, 4), "post", round(gp, 4), "build-up", round(b, 4))
        return g, b, gp

    g_lo, b_lo, p_lo = pick(2e5, 1.0)
    _, b_mid, _ = pick(2e5, 10.0)
    g_hi, b_hi, p_hi = pick(2e5, 1e4)
    g6, b6, p6 = pick(1e6, 1.0)
    _, b6_mid, _ = pick(1e6, 10.0)
    _, _, p6_hi = pick(1e6, 1e5)
    assert b_lo < 0.02 and b6 < 0.02          # steady state between pulses
    assert b_hi > 1.0                          # build-up at 1e4 Gy/s
    assert b_mid > 2 * b6_mid                  # the threshold rises with the pulse dose rate
    assert g_hi > 1.1 * g_lo                   # more H2O2 per dose with build-up
    assert g6 > 1.1 * g_lo                     # more H2O2 per dose from the denser pulses
    # post-irradiation (radicals standing at the end recombine): the rise with
    # the average dose rate holds for both pulse dose rates, stronger for the
    # weaker pulses (the paper: +30 % and +20 %)
    assert p_hi > 1.2 * p_lo and p6_hi > 1.1 * p6
    assert p_hi / p_lo > p6_hi / p6
