"""Write the oracle's row statistics of the large 128-D workloads (calls only
the oracle and the seeded input generators).

Workload: the 64-component mixture on a random 10-D subspace of R^128 plus
isotropic noise of std 0.05 (the precision configuration's recipe),
perplexity 50, at

* N = 98,304 (the default): above 65,536 points, so a row's distances no
  longer fit the search's register-held form and every row takes the
  streaming search; about 35 minutes of oracle search on eight cores;
* N = 262,144 (--n 262144): the precision configuration itself; about four
  hours on eight cores.

The statistics (beta, m, S, H of Eqs. 1-2 for every row) let a test form
whole rows of P (Eq. 3), hence gradient rows of Eq. 6, without repeating the
search over all rows.

Output: tests/golden/large_rowstats.npz (N = 98,304) or
tests/golden/c3_rowstats.npz (N = 262,144)
Usage: python tests/golden/make_large_reference.py [--n 262144]
"""
import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1812_09869_amd import synth  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
D, PERP = 128, 50.0
OUTPUT = {98304: "large_rowstats.npz", 262144: "c3_rowstats.npz"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=98304, choices=sorted(OUTPUT))
    n = ap.parse_args().n
    x, _ = synth.subspace(n, d=D)
    t0 = time.time()
    st = oracle.calibrate(x, PERP)
    np.savez_compressed(os.path.join(HERE, OUTPUT[n]), beta=st.beta, m=st.m, S=st.S, H=st.H,
                        iters=st.iters)
    print(f"{n} rows calibrated in {time.time() - t0:.0f} s (evaluations "
          f"{st.iters.min()}..{st.iters.max()})", flush=True)


if __name__ == "__main__":
    main()
