"""Write the stored oracle results used by the GPU tests (calls only the oracle).

Output: tests/golden/plain_small_oracle.json — the 2,000-point, 10-D,
8-component workload, perplexity 30, 500 iterations with exaggeration 12 and
momentum 0.5 before iteration 250, then 1 and 0.8, learning rate 200.

Besides the final KL of the run from the stored initial map, it records the
KL reached from sixteen initial maps that differ from it by one FP32 ulp in one
coordinate. Their spread is the chaos floor of the final KL: two exact FP64
runs whose inputs differ by one rounding already disagree by this much, so no
implementation with a different rounding order can be held closer than that.

Usage: python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1812_09869_amd import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "plain_small_oracle.json")


def main():
    x, _ = synth.plain_small()
    st = oracle.calibrate(x, 30.0)
    P = oracle.joint_p(x, st)
    y0 = synth.embedding_init(x.shape[0], synth.SEEDS["init_small"])
    kl0, cn0 = oracle.cost(P, y0)
    checkpoints = {}
    state = None
    t = 0
    for t_end in (1, 10, 250, 500):
        y, u, g = oracle.run(P, y0, t_end - t, start=t, state=state)
        state = (y, u, g)
        t = t_end
        kl, cn = oracle.cost(P, y)
        checkpoints[str(t_end)] = {"kl": kl, "cnorm": cn}
    ens = []
    for r in range(16):
        y0b = y0.copy()
        i, c = (r * 331) % x.shape[0], r % 2
        y0b[i, c] = np.nextafter(y0b[i, c], np.float32(1))
        yb, _, _ = oracle.run(P, y0b, 500)
        ens.append(oracle.cost(P, yb)[0])
    res = {
        "workload": "plain_small: N=2000 D=10 K=8 perplexity=30, 500 iterations",
        "perplexity": 30.0,
        "p_entropy_term": oracle.p_entropy_term(P),
        "beta_min": float(st.beta.min()),
        "beta_max": float(st.beta.max()),
        "bisection_evals_max": int(st.iters.max()),
        "kl_init": kl0,
        "cnorm_init": cn0,
        "checkpoints": checkpoints,
        "final_kl_ulp_ensemble": ens,
    }
    with open(OUT, "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(res, indent=1))


if __name__ == "__main__":
    main()
