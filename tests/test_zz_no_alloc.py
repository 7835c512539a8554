"""The allocation-free rate-equation entry point (gsbs_numodes_noalloc)
against gsbs_numodes on the same device arrays: identical concentrations and
step counts (the same kernel; only where the step counts are staged
differs), on two calls in a row, the second smaller than the first, so that
the shared device array keeps the first call's larger contents."""
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

from paper_2509_03313_amd import workload as W  # noqa: E402


def test_numodes_noalloc_matches_numodes():
    import torch
    assert torch.cuda.is_available(), "GPU tests need the device"
    from paper_2509_03313_amd import gsbs
    e = gsbs.Engine(1000.0, 1, W.D_CONFIG, W.REACTIONS)
    rng = np.random.default_rng(12)
    for n in (3000, 517):
        c0 = torch.as_tensor(10.0 ** rng.uniform(-8, -5, size=(n, 7)), device="cuda")
        dt = torch.as_tensor(10.0 ** rng.uniform(2, 6, size=n), device="cuda")
        ref, ref_steps = gsbs.gsbs_numodes(e.ctx, c0, dt, rtol=1e-6)
        c1 = torch.full_like(c0, float("nan"))
        steps = gsbs.gsbs_numodes_noalloc(e.ctx, c0, dt, c1, rtol=1e-6)
        torch.cuda.synchronize()
        print("[gpu-test] noalloc", n, "steps", int(steps.min()), int(steps.max()), flush=True)
        assert np.array_equal(steps, ref_steps)
        assert torch.equal(c1, ref)
    # sizes beyond the array are refused before anything runs
    big = torch.zeros(((1 << 20) + 1, 7), dtype=torch.float64, device="cuda")
    with pytest.raises(gsbs.GsbsError):
        gsbs.gsbs_numodes_noalloc(e.ctx, big, torch.zeros((1 << 20) + 1, dtype=torch.float64, device="cuda"),
                                  torch.empty_like(big))
    e.close()
