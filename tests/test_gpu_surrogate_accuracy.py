"""Accuracy of the shipped inter-pulse network (paper_2509_03313_amd/
surrogate_net.npz, trained by bench.py --surrogate on the engine's own SBS
runs: 3456 four-pulse and 384 ten-pulse runs in 5 um cubes, error table from
held-out runs in 10 um cubes) against plain SBS on the same pulses and seeds.

Five 1 Gy pulses at 1e6 Gy/s, 100 Gy/s on average, in a 10 um periodic cube.
gsbs_advance_to(GSBS_SURROGATE) with a 1 % tolerance hands an interval to the
network only when its held-out error estimate (95th percentile of the
relative H2O2 error in its bin of interval length and total concentration)
is within 1 % and every input lies in the training range; the test checks
that some intervals are handed over, that every handed-over interval's
estimate is within the tolerance, that every declined interval ran plain SBS
(the runs agree exactly up to the first interval taken), and that G(H2O2) at
every pulse start stays within 1 % of the plain run's."""
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))


def say(*a):
    print("[gpu-test]", *a, flush=True)


def test_shipped_network_within_one_percent_at_100_gy_per_s():
    import torch
    assert torch.cuda.is_available(), "GPU tests need the device"
    from paper_2509_03313_amd import gsbs
    from paper_2509_03313_amd import surrogate as SU
    path = os.path.join(os.path.dirname(HERE), "paper_2509_03313_amd", "surrogate_net.npz")
    s = SU.Surrogate(64)
    s.load(path)
    plan = SU.PulsePlan(10000.0, 77, 5, 1.0, 1e6, 100.0)
    plain = SU.run(plan, None)
    hyb = SU.run(plan, s, tol=0.01)
    say("plain G(H2O2)", plain["g_h2o2"].round(5).tolist(), "hybrid", hyb["g_h2o2"].round(5).tolist(),
        "network intervals", np.nonzero(hyb["used"])[0].tolist(), "walls", round(plain["wall"], 2),
        round(hyb["wall"], 2))
    assert hyb["intervals_by_network"] >= 1
    # every interval is decided by its held-out estimate: taken within 1 %, else plain SBS
    lg = hyb["handover"]
    assert len(lg["taken"]) == plan.n_pulses - 1
    assert np.array_equal(lg["taken"].astype(bool), lg["estimate"] <= 0.01), lg
    first = int(np.argmax(hyb["used"]))
    # identical trajectories up to the first interval the network takes
    assert np.array_equal(plain["n_h2o2"][:first], hyb["n_h2o2"][:first])
    rel = np.abs(hyb["g_h2o2"] - plain["g_h2o2"]) / plain["g_h2o2"]
    assert rel.max() <= 0.01, rel
    assert hyb["error_estimate_spent"] <= 0.01 * hyb["intervals_by_network"] + 1e-12
