"""Write the oracle's row statistics of the 98,304-point, 128-D workload (calls
only the oracle and the seeded input generators).

Workload: the 64-component mixture on a random 10-D subspace of R^128 plus
isotropic noise of std 0.05 (the precision configuration's recipe), 98,304
points, perplexity 50: above 65,536 points, so a row's distances no longer
fit the search's register-held form and every row takes the streaming
search. The statistics (beta, m, S, H of Eqs. 1-2 for every row) let a test
form whole rows of P (Eq. 3), hence gradient rows of Eq. 6, without
repeating the search over all rows.

Output: tests/golden/large_rowstats.npz
Usage: python tests/golden/make_large_reference.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1812_09869_amd import synth  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
N, D, PERP = 98304, 128, 50.0


def main():
    x, _ = synth.subspace(N, d=D)
    t0 = time.time()
    st = oracle.calibrate(x, PERP)
    np.savez_compressed(os.path.join(HERE, "large_rowstats.npz"), beta=st.beta, m=st.m, S=st.S,
                        H=st.H, iters=st.iters)
    print(f"{N} rows calibrated in {time.time() - t0:.0f} s (evaluations "
          f"{st.iters.min()}..{st.iters.max()})", flush=True)


if __name__ == "__main__":
    main()
