"""Write tests/golden/multi_pulse_1um_oracle.npz: species counts of the FP64
oracle for 32 seeds of a 4-pulse workload in a 1 um cube (1 Gy per pulse,
pulse rate 1e6 Gy/s, average rate 1e4 Gy/s, 2 injection batches per pulse,
30 log-spaced records per interval): the step ramp restarts at every batch.

Seed i: inputs workload.multi_pulse(i, ...), Philox key (1000, i).  Calls only
oracle/ and the seeded input generator.  Run from the repo root:
    python tests/golden/make_multi_pulse_curves.py
"""
import os
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2509_03313_amd import workload as W  # noqa: E402

PHILOX_SEED = 1000
N_SEEDS = 32
KW = dict(n_pulses=4, dose_per_pulse=1.0, L=1000.0, pulse_rate_gy_s=1e6, avg_rate_gy_s=1e4, n_batches=2,
          n_records=30)


def one(i):
    return oracle.run(W.multi_pulse(i, **KW), inst=i, philox_seed=PHILOX_SEED)


def main():
    oracle.lib()
    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        res = list(ex.map(one, range(N_SEEDS)))
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "multi_pulse_1um_oracle.npz")
    np.savez_compressed(out, times=res[0]["times"], counts=np.stack([r["counts"] for r in res]),
                        edep=np.stack([r["edep"] for r in res]), n_steps=np.array([r["n_steps"] for r in res]),
                        philox_seed=PHILOX_SEED)
    print(out, [r["n_steps"] for r in res][:3], res[0]["counts"][-1])


if __name__ == "__main__":
    main()
