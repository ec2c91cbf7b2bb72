"""State comparison of a GPU run (librewl) and an oracle run, element by element."""
import numpy as np


def assert_same_state(g, o):
    """Every integer and binary64 field of every walker and window must match exactly."""
    assert g.step == o.step and g.round == o.round
    for w in range(g.nw):
        a, b = g.walker(w), o.walker(w)
        assert np.array_equal(a["spins"], b["spins"]), f"spins of walker {w}"
        assert a["E"] == b["E"], f"E of walker {w}"
        assert np.array_equal(a["H"], b["H"]), f"H of walker {w}"
        assert np.array_equal(a["lng"].view(np.uint64), b["lng"].view(np.uint64)), f"ln g of walker {w}"
        assert a["replica"] == b["replica"], f"replica of walker {w}"
        assert a["walkin_attempts"] == b["walkin_attempts"], f"walk-in of walker {w}"
    for k in range(g.h):
        a, b = g.window(k), o.window(k)
        for key in ("lnf", "lnf_last", "regime", "finished", "iterations", "x_att", "x_acc"):
            assert a[key] == b[key], (k, key, a[key], b[key])
        assert np.array_equal(a["visited"], b["visited"]), f"visited of window {k}"
    wa, ta = g.replicas()
    wb, tb = o.replicas()
    assert np.array_equal(wa, wb), "replica windows"
    assert np.array_equal(ta, tb), "replica round trips"
    if g.nw <= 4096:
        for w in range(g.nw):
            assert np.array_equal(g.replica_visits(w), o.replica_visits(w)), f"replica visits of slot {w}"
    if getattr(g, "obs_bins", 0) > 0:
        assert o.obs_bins == g.obs_bins
        for w in range(g.nw):
            for a, b, name in zip(g.obs(w), o.obs(w), ("H(E, O)", "sum of O", "samples")):
                assert np.array_equal(a, b), f"{name} of walker {w}"
