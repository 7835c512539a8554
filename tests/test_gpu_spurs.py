"""Pulses generated on the device (gsbs_inject_pulse) against the oracle's
counter-based spur model: the same tracks, spurs, molecule counts and species
(integer decisions from the same Philox words and the same FP64 running
sums), positions equal up to the FP32 storage and the last bits of the
libraries' log, sin and cos."""
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

import oracle  # noqa: E402
from paper_2509_03313_amd import workload as W  # noqa: E402


def say(*a):
    print("[gpu-test]", *a, flush=True)


@pytest.fixture(scope="module")
def g():
    import torch
    assert torch.cuda.is_available(), "GPU tests need the device"
    from paper_2509_03313_amd import gsbs
    return gsbs


@pytest.mark.parametrize("L,n_tracks,stream,sigma", [(2000.0, 12, 5, 2.0), (10000.0, 780, 0, 2.0),
                                                     (500.0, 3, 9, 40.0)])
def test_pulse_matches_oracle(g, L, n_tracks, stream, sigma):
    seed = 2024
    e = g.Engine(L, seed, W.D_CONFIG, W.REACTIONS)
    n = g.gsbs_inject_pulse(e.ctx, 0, 0.0, n_tracks, W.SPUR_FRACTIONS, stream=stream, sigma_nm=sigma)
    xo, so = oracle.spurs(L, seed, stream, n_tracks, 100.0, 5.13, sigma, W.SPUR_FRACTIONS)
    say("L", L, "tracks", n_tracks, "molecules", n, len(so))
    assert n == len(so)
    e.advance_to(0.0)  # the injection enters at the present step boundary
    xg, sg, ug = g.gsbs_debug_get_state(e.ctx, 0)
    assert len(sg) == n
    order = np.argsort(ug)  # uids follow the emitted order: track, spur, molecule
    assert np.array_equal(sg[order].astype(np.int32), so)
    d = xg[order].astype(np.float64) - xo
    d = (d + L / 2) % L - L / 2
    assert np.abs(d).max() <= 2e-7 * L, np.abs(d).max()
    cnt = e.current_counts(0)
    assert np.array_equal(cnt, np.bincount(so, minlength=7))
    e.close()


def test_pulse_errors_and_energy(g):
    e = g.Engine(1000.0, 1, W.D_CONFIG, W.REACTIONS)
    with pytest.raises(g.GsbsError):  # fractions do not sum to 1
        g.gsbs_inject_pulse(e.ctx, 0, 0.0, 3, [0.5, 0.4, 0, 0, 0, 0, 0])
    with pytest.raises(g.GsbsError):  # spacing
        g.gsbs_inject_pulse(e.ctx, 0, 0.0, 3, W.SPUR_FRACTIONS, spacing_nm=0.0)
    assert g.gsbs_inject_pulse(e.ctx, 0, 0.0, 0, W.SPUR_FRACTIONS) == 0
    n = g.gsbs_inject_pulse(e.ctx, 0, 5.0, 4, W.SPUR_FRACTIONS, stream=1)
    e.set_records(0, [10.0])
    e.advance_to(10.0)
    gv = e.gvalues(0)[0]
    cnt = e.counts(0)[0]
    # G = count / (E / 100 eV) with E = tracks * L * LET (keV/um * nm = eV)
    E = 4 * 1000.0 * 0.8
    assert n > 0 and np.allclose(gv, cnt / (E / 100.0))
    with pytest.raises(g.GsbsError):  # before the present time
        g.gsbs_inject_pulse(e.ctx, 0, 1.0, 2, W.SPUR_FRACTIONS)
    e.close()
