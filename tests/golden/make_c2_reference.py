"""Write the oracle's reference run of the 65,536-point benchmark workload
(calls only the oracle and the seeded input generators).

Workload: N=65,536, D=50, the 32-component anisotropic mixture, perplexity 50,
initial map N(0, 1e-4 I) from the benchmark's seed, 1,000 iterations with
exaggeration 12 and momentum 0.5 before iteration 250, then 1 and 0.8,
learning rate 200 (the plain t-SNE schedule of Eq. 10 and the paragraph after
it). Everything is FP64 with the full square P (34 GB in memory): about an
hour per trajectory on eight cores.

Outputs (tests/golden/):
* c2_rowstats.npz: beta, m, S, H of every row (Eqs. 1-2), so that tests can
  form any row of P (Eq. 3) without repeating the search over all rows;
* c2_states.npz: the oracle map after 249 and 999 iterations (the states the
  last exaggerated and the last plain gradient are taken at), rounded to FP32;
* c2_oracle.json: KL and C_norm (Eqs. 5 and 9) after 1, 10, 250, 500, 750 and
  1,000 iterations of the run from the stored initial map, and the same at
  250, 500, 750 and 1,000 for runs whose initial maps differ from it by one
  FP32 ulp in one coordinate (the chaos floor of the final KL: two exact FP64
  runs that differ by one rounding already separate by this much).

The JSON is rewritten after every checkpoint, so an interrupted run keeps what
it reached.

Usage: python tests/golden/make_c2_reference.py [--perturbed K]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1812_09869_amd import synth  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
N, PERP, ITERS = 65536, 50.0, 1000
CHECKS = (1, 10, 250, 500, 750, 1000)


def log(msg):
    print(f"[{time.strftime('%H:%M:%S')}] {msg}", flush=True)


def trajectory(P, y0, res_run, save_states=False, out=None):
    y, u, g = oracle._f64(y0).copy(), None, None
    state = None
    t = 0
    t0 = time.time()
    states = {}
    for t_end in CHECKS:
        stops = [s for s in (249, 999) if save_states and t < s < t_end]
        for s in stops + [t_end]:
            y, u, g = oracle.run(P, y0, s - t, start=t, state=state)
            state = (y, u, g)
            t = s
            if s in (249, 999) and save_states:
                states[f"y{s}"] = y.astype(np.float32)
        kl, cn = oracle.cost(P, y)
        res_run[str(t_end)] = {"kl": kl, "cnorm": cn}
        log(f"  t={t_end}: KL {kl:.10f} C_norm {cn:.10f} ({time.time() - t0:.0f} s)")
        if out is not None:
            out()
    return states


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--perturbed", type=int, default=2)
    args = ap.parse_args()
    x, _ = synth.gmm_aniso(N)
    log(f"calibrating {N} rows")
    st = oracle.calibrate(x, PERP)
    np.savez_compressed(os.path.join(HERE, "c2_rowstats.npz"), beta=st.beta, m=st.m, S=st.S,
                        H=st.H, iters=st.iters)
    log(f"rowstats written (evaluations {st.iters.min()}..{st.iters.max()})")
    P = oracle.joint_p(x, st)
    log("P formed")
    y0 = synth.embedding_init(N, synth.SEEDS["init_aniso"])
    res = {
        "workload": "gmm_aniso: N=65536 D=50 K=32 perplexity=50, 1000 iterations "
                    "(exaggeration 12 and momentum 0.5 for t < 250, then 1 and 0.8; eta 200)",
        "perplexity": PERP,
        "p_entropy_term": oracle.p_entropy_term(P),
        "kl_init": None,
        "checkpoints": {},
        "perturbed": [],
    }
    path = os.path.join(HERE, "c2_oracle.json")

    def write():
        with open(path, "w") as f:
            json.dump(res, f, indent=1)

    res["kl_init"], res["cnorm_init"] = oracle.cost(P, y0)
    write()
    log("base run")
    states = trajectory(P, y0, res["checkpoints"], save_states=True, out=write)
    np.savez_compressed(os.path.join(HERE, "c2_states.npz"), **states)
    for r in range(args.perturbed):
        y0b = y0.copy()
        i, c = (r * 331) % N, r % 2
        y0b[i, c] = np.nextafter(y0b[i, c], np.float32(1))
        entry = {"row": i, "coord": c, "checkpoints": {}}
        res["perturbed"].append(entry)
        log(f"perturbed run {r}: y0[{i}, {c}] one ulp up")
        trajectory(P, y0b, entry["checkpoints"], out=write)
    write()
    log("done")


if __name__ == "__main__":
    main()
