"""Batched iteration: many problems per launch.

* Every problem's state after batched steps is bitwise equal to running
  tsne_step on it alone (same kernels, same reduction order), so the batched
  path inherits the single-problem parity with the oracle; checked on small
  problems and on sampled problems of the full 64-problem workload.
* On the four smallest problems of the 64-problem workload: the gradient at
  oracle states of iterations 0, 249 and 499 (oracle FP64 trajectories cast to
  FP32) matches the oracle to 1e-4, and the batched 500-iteration run passes
  the shared final-KL gate against the stored oracle runs (sixteen starts one
  FP32 ulp apart give the chaos floor: trajectories that differ only in
  rounding separate, so the final KL is only determined up to that spread).
"""
import numpy as np
import pytest
import torch

import oracle
from chaos_gate import final_kl_gate
from paper_1812_09869_amd import _lib, synth
from paper_1812_09869_amd.tsne import BatchedTSNE, ExactTSNE, Schedule, paper_schedule

pytestmark = pytest.mark.gpu


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("rule", ["gains", "range"])
def test_batched_bitwise_equals_single(rule):
    sizes = [(300, 5), (257, 3), (1000, 10), (40, 2), (2048, 7)]
    rng = np.random.Generator(np.random.PCG64(9))
    probs = [((rng.standard_normal((n, d)) * 3).astype(np.float32), 8.0) for n, d in sizes]
    y0s = [synth.embedding_init(n, seed=20 + k) for k, (n, _) in enumerate(sizes)]
    batched = BatchedTSNE([(_t(x), p) for x, p in probs])
    batched.init_states([_t(y) for y in y0s])
    sched = Schedule(switch=2) if rule == "gains" else paper_schedule(0.8)
    batched.run(4, sched=sched)
    for k, ((x, p), y0) in enumerate(zip(probs, y0s)):
        single = ExactTSNE(_t(x), p)
        st = single.init_state(_t(y0))
        single.run(st, 4, sched=sched)
        for a, b in zip(batched.states[k], st):
            assert torch.equal(a, b), k
        assert batched.models[k].status() == 0
    # the batched cost is the single-problem cost, bitwise
    out = torch.empty((len(sizes), 2), dtype=torch.float64, device="cuda")
    _lib.batch_cost(batched._arr, batched._bws, out)
    for k, m in enumerate(batched.models):
        assert torch.equal(out[k], m.cost(batched.states[k][0])), k


def test_more_problems_than_the_lds_table():
    """1,030 small problems: more than the nonzero-tile kernel keeps in its LDS
    table (1,024), so it walks the problem table instead. Every problem's status
    is clean and sampled problems on both sides of the 1,024 boundary are
    bitwise the state of separate runs."""
    count = 1030
    rng = np.random.Generator(np.random.PCG64(31))
    ns = rng.integers(40, 300, count)
    ds = rng.integers(2, 6, count)
    probs = [((rng.standard_normal((int(n), int(d))) * 3).astype(np.float32), 8.0)
             for n, d in zip(ns, ds)]
    y0s = [synth.embedding_init(int(n), seed=500 + k) for k, n in enumerate(ns)]
    print(f"\n[batched] {count} problems, {int(ns.sum())} points", flush=True)
    batched = BatchedTSNE([(_t(x), p) for x, p in probs])
    batched.init_states([_t(y) for y in y0s])
    sched = Schedule(switch=2)
    batched.run(3, sched=sched)
    assert max(m.status() for m in batched.models) == 0
    for k in (0, 511, 1023, 1024, count - 1):
        x, p = probs[k]
        single = ExactTSNE(_t(x), p)
        st = single.init_state(_t(y0s[k]))
        single.run(st, 3, sched=sched)
        for a, b in zip(batched.states[k], st):
            assert torch.equal(a, b), k


def test_full_workload_bitwise_on_sampled_problems():
    """The benchmark's 64-problem workload (636,092 points) in the launch the benchmark
    times: after six batched sweeps of the benchmark schedule (the exaggeration phase),
    the smallest and the largest problem and two others are bitwise the state of a
    separate single-problem run, and every problem's status is clean."""
    data = [synth.batch_problem(p) for p in range(64)]
    print(f"\n[batched] 64 problems, {sum(x.shape[0] for x, _, _ in data)} points", flush=True)
    y0s = [synth.embedding_init(x.shape[0], seed=4100 + p) for p, (x, _, _) in enumerate(data)]
    batched = BatchedTSNE([(_t(x), perp) for x, _, perp in data])
    batched.init_states([_t(y) for y in y0s])
    batched.run(6)
    assert max(m.status() for m in batched.models) == 0
    sizes = [x.shape[0] for x, _, _ in data]
    chosen = sorted({int(np.argmin(sizes)), int(np.argmax(sizes)), 17, 42})
    for k in chosen:
        x, _, perp = data[k]
        single = ExactTSNE(_t(x), perp)
        st = single.init_state(_t(y0s[k]))
        single.run(st, 6)
        for a, b in zip(batched.states[k], st):
            assert torch.equal(a, b), k
        print(f"  problem {k} (n={sizes[k]}): bitwise equal", flush=True)
        del single, st
        torch.cuda.empty_cache()


def test_batched_matches_oracle_on_smallest_problems():
    """The four smallest problems of the 64-problem workload, 500 batched
    iterations: per-step gradients at oracle states, and the KL after 250, 300,
    400 and 500 iterations against the stored oracle runs (the run from the
    stored map and sixteen runs one FP32 ulp apart), gated by the shared
    final-KL rule."""
    import json
    import os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                       "batched_small_oracle.json")))
    ns = []
    for p in range(64):
        x, lab, perp = synth.batch_problem(p)
        ns.append((x.shape[0], p))
    chosen = [p for _, p in sorted(ns)[:4]]
    assert sorted(chosen) == sorted(int(k) for k in gold["problems"])
    data = [synth.batch_problem(p) for p in chosen]
    y0s = [synth.embedding_init(x.shape[0], seed=4100 + p) for (x, _, _), p in zip(data, chosen)]
    batched = BatchedTSNE([(_t(x), perp) for x, _, perp in data])
    batched.init_states([_t(y) for y in y0s])
    kls = {p: {} for p in chosen}
    t = 0
    for t_end in gold["checkpoints"]:
        batched.run(t_end - t, start=t)
        t = t_end
        for k, p in enumerate(chosen):
            kls[p][t_end] = float(batched.models[k].cost(batched.states[k][0]).cpu()[0])
    for k, ((x, lab, perp), p) in enumerate(zip(data, chosen)):
        st = oracle.calibrate(x, perp)
        P = oracle.joint_p(x, st)
        model = batched.models[k]
        state = None
        t = 0
        for t_check in (0, 249, 499):
            y, u, g = oracle.run(P, y0s[k], t_check - t, start=t, state=state)
            state = (y, u, g)
            t = t_check
            alpha = oracle.schedule(t_check).alpha
            y32 = y.astype(np.float32)
            g_ref, _ = oracle.gradient(P, y32.astype(np.float64), alpha)
            g_gpu, _ = model.gradient(_t(y32), alpha)
            rel = np.linalg.norm(g_gpu.cpu().numpy() - g_ref) / np.linalg.norm(g_ref)
            print(f"\n  problem {p} (n={x.shape[0]}, d={x.shape[1]}) t={t_check}: grad rel {rel:.2e}")
            assert rel <= 1e-4
        ref = gold["problems"][str(p)]
        for t_end in gold["checkpoints"]:
            ens = [e[str(t_end)] for e in ref["ensemble"]]
            kr = ref["kl"][str(t_end)]
            print(f"  t={t_end}: KL gpu {kls[p][t_end]:.5f} oracle {kr:.5f} ensemble "
                  f"{min(ens):.5f}..{max(ens):.5f}")
        ens = [e["500"] for e in ref["ensemble"]]
        ok, band, tol = final_kl_gate(kls[p][500], ref["kl"]["500"], ens)
        print(f"  final KL rel diff {abs(kls[p][500] - ref['kl']['500']) / ref['kl']['500']:.2e}"
              f"; oracle band {band / ref['kl']['500']:.2e}, tolerance "
              f"{tol / ref['kl']['500']:.2e}")
        assert ok
        assert model.status() == 0


def test_batch_mismatch_is_ignored_on_device():
    """A step with a problem list other than the planned one changes nothing."""
    rng = np.random.Generator(np.random.PCG64(2))
    xs = [(rng.standard_normal((n, 3))).astype(np.float32) for n in (100, 200)]
    b = BatchedTSNE([(_t(x), 5.0) for x in xs])
    b.init_states([_t(synth.embedding_init(x.shape[0], seed=1)) for x in xs])
    y_before = b.states[0][0].clone()
    arr1 = _lib.batch_problems([(b.models[0].ws, 100, *b.states[0])])
    _lib.batch_step(arr1, b._bws, 1.0, 0.5, 200.0)
    torch.cuda.synchronize()
    assert torch.equal(b.states[0][0], y_before)
