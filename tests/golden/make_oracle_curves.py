"""Write tests/golden/single_pulse_1um_oracle.npz: species counts of the FP64
oracle for 32 seeds of the 1 um, ~1e4-molecule single-pulse workload
(5 isotropic spur tracks, 2000 steps from 1 ps to 1 us).

Seed i: spur input workload.single_pulse_small(i), Philox key (1000, i).
Calls only oracle/ and the seeded input generator.  Run from the repo root:
    python tests/golden/make_oracle_curves.py
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


def one(i):
    wl = W.single_pulse_small(i)
    r = oracle.run(wl, inst=i, philox_seed=PHILOX_SEED)
    return r


def main():
    oracle.lib()
    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        res = list(ex.map(one, range(N_SEEDS)))
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "single_pulse_1um_oracle.npz")
    np.savez_compressed(out,
                        times=res[0]["times"],
                        counts=np.stack([r["counts"] for r in res]),
                        edep=np.stack([r["edep"] for r in res]),
                        n_steps=np.array([r["n_steps"] for r in res]),
                        molecule_steps=np.array([r["molecule_steps"] for r in res]),
                        philox_seed=PHILOX_SEED)
    print(out, [r["n_steps"] for r in res][:3], res[0]["counts"][-1])


if __name__ == "__main__":
    main()
