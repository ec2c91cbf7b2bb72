"""GPU parity of the batched form: every instance of a batch must end in the
state the oracle reaches running that instance alone, bit for bit, whatever
the launch plan (persistent grid shape, tag-table policy, graph replay or
plain launches, one launch per instance)."""
import sys

import numpy as np
import pytest

import oracle
import workloads
from statecmp import assert_same_state

pytestmark = pytest.mark.gpu

# (L, q, windows, walkers, sync_attempts, extra options)
MIXED = [
    (6, 3, 3, 2, 360, dict(lnf_init=1.0, lnf_final=1e-3)),
    (8, 10, 4, 2, 640, dict(lnf_init=0.5, lnf_final=1e-6)),
    (12, 4, 5, 3, 1440, dict(lnf_init=1.0, lnf_final=1e-6, schedule=1)),
    (4, 2, 2, 4, 160, dict(lnf_init=1.0, lnf_final=2e-2)),       # converges within the test
    (16, 8, 8, 4, 2560, dict(lnf_init=1e-4, lnf_final=1e-9)),     # table-mode ln f
    (3, 5, 1, 3, 90, dict(lnf_init=0.3, lnf_final=1e-6, exchange=0)),
]


def _pk():
    import paper_1312_3004_amd as pk
    return pk


def make_batch(cases, precision=0, seed=7):
    insts, spins = [], []
    for i, (L, q, h, m, S, extra) in enumerate(cases):
        d = dict(L=L, q=q, windows=h, overlap=0.75, walkers=m, seed=seed, instance=i, sync_attempts=S,
                 precision=precision)
        d.update(extra)
        insts.append(d)
        spins.append(workloads.init_spins(L, q, h * m, 100 + i))
    print(f"[case] batch of {len(cases)} precision={precision}", flush=True)
    sys.stdout.flush()
    return _pk().Batch(insts, spins), insts, spins


def oracle_of(d, spins):
    d = dict(d)
    geo = [d.pop(k) for k in ("L", "q", "windows", "overlap", "walkers")]
    return oracle.Rewl(*geo, spins, threads=8, **d)


def check_against_oracle(b, insts, spins, steps):
    for i, d in enumerate(insts):
        o = oracle_of(d, spins[i])
        o.run(steps * d["sync_attempts"])
        assert_same_state(b.instance(i), o)


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_graph_steps_bitexact(precision):
    b, insts, spins = make_batch(MIXED, precision=precision)
    assert b.plan()["use_graph"] == 1
    b.run(5)
    b.run(4)
    assert b.progress()[0] == 9
    check_against_oracle(b, insts, spins, 9)


def test_plans_give_identical_results():
    ref, insts, spins = make_batch(MIXED)
    ref.run(6)
    plans = [dict(walkers_per_cu=1, tag_policy=1, use_graph=0),
             dict(walkers_per_cu=2, tag_policy=0, use_graph=1),
             # mixed-slot form: one slot per class (plus one more for the largest)
             dict(slot_count=[2, 1, 1, 1, 1, 1], tag_bytes=4096, use_graph=1),
             # only the largest class has slots: they serve every class
             dict(slot_count=[3, 0, 0, 0, 0, 0], tag_bytes=2048, use_graph=0)]
    for p in plans:
        b, _, _ = make_batch(MIXED)
        b.set_plan(**p)
        b.run(6)
        for i in range(len(MIXED)):
            assert_same_state(b.instance(i), ref.instance(i))
    c, _, _ = make_batch(MIXED)
    c.run_per_instance(3)
    c.run(3)
    for i in range(len(MIXED)):
        assert_same_state(c.instance(i), ref.instance(i))
    check_against_oracle(ref, insts, spins, 6)


def test_tuner_steps_are_run_steps():
    b, insts, spins = make_batch(MIXED[:4])
    plan, tried = b.tune(steps_per_plan=1)
    assert len(tried) >= 2 and plan["use_graph"] == 1
    assert all(t["ms_per_step"] > 0 for t in tried)
    assert min(t["ms_per_step"] for t in tried) == pytest.approx(plan["ms_per_step"])
    done = b.progress()[0]
    assert done == len(tried)
    b.run(2)
    check_against_oracle(b, insts, spins, done + 2)


def test_batch_runs_every_instance_to_convergence():
    cases = [(4, 2, 2, 4, 160, dict(lnf_init=1.0, lnf_final=2e-2)),
             (3, 3, 2, 2, 90, dict(lnf_init=1.0, lnf_final=1e-3)),
             (5, 2, 3, 2, 250, dict(lnf_init=1.0, lnf_final=5e-3, schedule=1))]
    b, insts, spins = make_batch(cases)
    st = b.run(100_000)
    assert st == _pk().CONVERGED and b.progress()[1] == len(cases)
    for i, d in enumerate(insts):
        o = oracle_of(d, spins[i])
        assert o.run(10**12) == oracle.CONVERGED
        g = b.instance(i)
        assert_same_state(g, o)
        sg, lg, cg = g.join()
        so, lo, co = o.join()
        assert sg == so == 0 and np.array_equal(cg, co)
        fin = np.isfinite(lo)
        assert np.array_equal(np.isfinite(lg), fin)
        assert np.max(np.abs(lg[fin] - lo[fin])) <= 1e-10


def test_batched_workload_instances_segment():
    # Instances of the 256-instance workload's shapes (its windows, walkers and
    # schedule; the smallest and largest q of each lattice size, q=2 only at
    # L=48 to keep the oracle's walk-in short), one batched step, against the oracle.
    cfg = workloads.BATCHED
    picks = [(L, q) for L in cfg["L_choices"][:-1] for q in (cfg["q_choices"][0], cfg["q_choices"][-1])]
    picks.append((cfg["L_choices"][-1], cfg["q_choices"][0]))
    cases = [(L, q, cfg["windows"], cfg["walkers"], cfg["sweeps_per_sync"] * L * L,
              dict(lnf_init=cfg["lnf_init"], lnf_final=cfg["lnf_final"], flat=cfg["flat"],
                   schedule=cfg["schedule"])) for L, q in picks]
    b, insts, spins = make_batch(cases, seed=cfg["seed"])
    b.run(1)
    check_against_oracle(b, insts, spins, 1)


def test_batched_workload_mixed_slots_match_uniform():
    cfg = workloads.BATCHED
    picks = [(L, cfg["q_choices"][-1]) for L in cfg["L_choices"]] * 2
    cases = [(L, q, cfg["windows"], cfg["walkers"], cfg["sweeps_per_sync"] * L * L,
              dict(lnf_init=cfg["lnf_init"], lnf_final=cfg["lnf_final"], flat=cfg["flat"],
                   schedule=cfg["schedule"])) for L, q in picks]
    a, _, _ = make_batch(cases, seed=cfg["seed"])
    b, _, _ = make_batch(cases, seed=cfg["seed"])
    pa = a.set_plan(walkers_per_cu=5)
    pb = b.set_plan(slot_count=[3, 2, 1, 2], tag_bytes=4096)
    assert pb["nclasses"] == 4 and pb["resident"] == 8 and pb["mixed"] == 1
    a.run(2)
    b.run(2)
    for i in range(len(cases)):
        assert_same_state(b.instance(i), a.instance(i))
