"""Write the oracle's values for the full-size parity tests (C2 and C3 workloads).

The direct sums at lmax = 2047 and 4095 over millions of points take tens of core-minutes,
too long for a test on the GPU machine, so they are computed once by this script and stored
beside it.  It calls only the oracle (plain C direct sums of Eq. 2 and Eq. 3) and the seeded
input generators; nothing here comes from the GPU library.

    python tests/golden/make_large_oracle_values.py [--threads N]

Outputs (numpy .npz, plain arrays, no pickles):
  c2_adjoint_columns.npz  m = 0, 1, 2, 64, 511, 1024, 2000, 2047 of the C2 adjoint
                          (deflected 2048 x 4095 grid, lmax 2047): cols [1, 8, 2048] complex
  c3_sample_synthesis.npz synthesis of the 4 C3 coefficient sets on 4096 seeded points:
                          idx [4096], f [4, 4096]
  c3_adjoint_columns.npz  m = 0, 1, 2048, 4000, 4095 of the C3 adjoint of all 4 maps over
                          all 33,550,336 points: cols [4, 5, 4096] complex
  c3_spin2_sample_synthesis.npz
                          spin-2 synthesis (Q, U) of the spin benchmark's two fields (seed 106)
                          on 48 evenly spaced C3 points: idx [48], f [2, 2, 48]
"""
import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2406_14542_amd import inputs  # noqa: E402

C2_MS = [0, 1, 2, 64, 511, 1024, 2000, 2047]
C3_MS = [0, 1, 2048, 4000, 4095]
C3_SAMPLE = 4096
C3_SAMPLE_SEED = 3
SPIN_SEED, SPIN, SPIN_FIELDS, SPIN_SAMPLE = 106, 2, 2, 48


def spin_sample_index(n):
    return np.linspace(0, n - 1, SPIN_SAMPLE).astype(np.int64)


def c3_sample_index(n):
    return np.sort(np.random.default_rng(C3_SAMPLE_SEED).choice(n, C3_SAMPLE, replace=False))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--only", choices=["c2", "c3s", "c3a", "spin"], default=None)
    a = ap.parse_args()
    oracle.build(force=False)
    t = a.threads
    if a.only in (None, "c2"):
        t0 = time.time()
        cfg = inputs.config_c2()
        cols = oracle.adjoint_columns(cfg["lmax"], cfg["theta"], cfg["phi"], cfg["d"], C2_MS,
                                      nthreads=t)
        np.savez_compressed(os.path.join(HERE, "c2_adjoint_columns.npz"), ms=np.array(C2_MS),
                            cols=cols)
        print(f"c2 columns: {time.time() - t0:.0f} s", flush=True)
    if a.only in (None, "spin"):
        t0 = time.time()
        cfg = inputs.config_c3(nmaps=1)
        L = cfg["lmax"]
        alm = inputs.spin_alm(np.random.default_rng(SPIN_SEED), L, L, SPIN, SPIN_FIELDS)
        idx = spin_sample_index(cfg["theta"].size)
        f = oracle.spin_synthesis(L, L, SPIN, cfg["theta"][idx], cfg["phi"][idx], alm, nthreads=t)
        np.savez_compressed(os.path.join(HERE, "c3_spin2_sample_synthesis.npz"), idx=idx, f=f)
        print(f"c3 spin-2 sample synthesis: {time.time() - t0:.0f} s", flush=True)
    if a.only in (None, "c3s", "c3a"):
        cfg = inputs.config_c3()
        L = cfg["lmax"]
        if a.only in (None, "c3s"):
            t0 = time.time()
            idx = c3_sample_index(cfg["theta"].size)
            f = oracle.synthesis(L, L, cfg["theta"][idx], cfg["phi"][idx], cfg["alm"], nthreads=t)
            np.savez_compressed(os.path.join(HERE, "c3_sample_synthesis.npz"), idx=idx, f=f)
            print(f"c3 sample synthesis: {time.time() - t0:.0f} s", flush=True)
        if a.only in (None, "c3a"):
            t0 = time.time()
            cols = oracle.adjoint_columns(L, cfg["theta"], cfg["phi"], cfg["d"], C3_MS,
                                          nthreads=t)
            np.savez_compressed(os.path.join(HERE, "c3_adjoint_columns.npz"),
                                ms=np.array(C3_MS), cols=cols)
            print(f"c3 adjoint columns: {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
