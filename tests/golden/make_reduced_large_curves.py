"""Write tests/golden/single_pulse_2p5um_oracle.npz: species counts of the FP64
oracle for 32 seeds of a reduced 10 um single pulse: the same 1 Gy of
z-parallel spur tracks at the same density (Eq. 5 track count for the cube),
in a 2.5 um periodic cube (~6e3 molecules), 1 ps -> 1 ms, 60 log-spaced
records (the late steps run at the largest step the cube allows).

Seed i: spur input workload.single_pulse_large(i, L=2500, n_records=60),
Philox key (1000, i).  Calls only oracle/ and the seeded input generator.
Run from the repo root:
    python tests/golden/make_reduced_large_curves.py
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
L_NM = 2500.0
N_RECORDS = 60


def one(i):
    wl = W.single_pulse_large(i, L=L_NM, n_records=N_RECORDS)
    return oracle.run(wl, inst=i, philox_seed=PHILOX_SEED)


def main():
    oracle.lib()
    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        res = list(ex.map(one, range(N_SEEDS)))
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "single_pulse_2p5um_oracle.npz")
    np.savez_compressed(out,
                        times=res[0]["times"],
                        counts=np.stack([r["counts"] for r in res]),
                        edep=np.stack([r["edep"] for r in res]),
                        n_steps=np.array([r["n_steps"] for r in res]),
                        molecule_steps=np.array([r["molecule_steps"] for r in res]),
                        philox_seed=PHILOX_SEED, L_nm=L_NM, n_records=N_RECORDS)
    print(out, [r["n_steps"] for r in res][:3], res[0]["counts"][0], res[0]["counts"][-1],
          sum(r["molecule_steps"] for r in res))


if __name__ == "__main__":
    main()
