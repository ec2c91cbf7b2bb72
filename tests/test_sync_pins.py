"""Pins of the oracle's sync step (Sec. 2) on planted histograms.

A sync point of window k tests every walker for flatness over the bins the
window has visited, and when all m walkers are flat it averages their ln g,
clears H and halves ln f (f -> sqrt f); with the 1/t schedule of Belardinelli
and Pereyra, ln f becomes W/t once the halved value is not above it (t =
attempts per walker / W), and from then on every sync point sets it to W/t.
The window is finished once ln f drops below ln f_final.

Each rule is checked on histograms planted through the oracle's test hooks,
with no attempts in between, so the expected outcome follows from the rule
alone.  The cases sit on the boundaries a slip would move: the equality
min H = 0.8 <H>, a bin that one walker never reached, a halving by exactly 1/2,
the switch at W/t equal to the halved ln f, and ln f equal to ln f_final.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
import workloads

L, Q = 4, 2   # B = 33 energy bins


def fresh(m=2, h=1, schedule=0, lnf=1.0, lnf_final=1e-6, flat=(4, 5)):
    spins = workloads.init_spins(L, Q, h * m, 3)
    return oracle.Rewl(L, Q, h, 0.75, m, spins, seed=1, flat=flat, lnf_init=lnf, lnf_final=lnf_final,
                       schedule=schedule, sync_attempts=1000)


def plant(o, k, hists):
    """hists[j]: {bin: count} of walker j of window k; the walker has visited exactly those bins."""
    for j, hj in enumerate(hists):
        H = np.zeros(o.W, dtype=np.uint32)
        v = np.zeros(o.W, dtype=np.uint8)
        for b, c in hj.items():
            H[b] = c
            v[b] = 1
        o.plant_walker(k * o.m + j, H, v)


def counts(values, first=3):
    return {first + i: c for i, c in enumerate(values)}


def flat_by_definition(H, frac):
    """min H >= frac * mean H over the visited bins, in exact rationals."""
    H = [Fraction(int(x)) for x in H]
    return len(H) > 0 and min(H) >= frac * (sum(H) / len(H))


# --------------------------------------------------------------------------
# Flatness: min H >= 0.8 <H> over the window's visited bins.

def test_flatness_equality_counts_as_flat():
    # min 4, mean 5: min = 0.8 * mean exactly -> flat, so ln f halves.
    o = fresh()
    plant(o, 0, [counts([4, 5, 5, 5, 6]), counts([4, 5, 5, 5, 6])])
    o.sync_window(0)
    w = o.window(0)
    assert w["lnf"] == 0.5 and w["iterations"] == 1
    assert not o.walker(0)["H"].any() and not o.walker(1)["H"].any()


def test_flatness_one_count_short_is_not_flat():
    # min 4, mean 5.2: 4 < 0.8 * 5.2 -> not flat; nothing changes.
    o = fresh()
    plant(o, 0, [counts([4, 5, 5, 5, 6]), counts([4, 5, 5, 5, 7])])
    o.sync_window(0)
    w = o.window(0)
    assert w["lnf"] == 1.0 and w["iterations"] == 0
    assert o.walker(1)["H"].sum() == 26


def test_flatness_fraction_is_on_the_mean_side():
    # flatness 0.9: min 9, mean 10 is flat (equality); min 9, mean 10.2 is not.
    o = fresh(flat=(9, 10))
    plant(o, 0, [counts([9, 10, 10, 10, 11])] * 2)
    o.sync_window(0)
    assert o.window(0)["lnf"] == 0.5
    o = fresh(flat=(9, 10))
    plant(o, 0, [counts([9, 10, 10, 10, 11]), counts([9, 10, 10, 11, 11])])
    o.sync_window(0)
    assert o.window(0)["lnf"] == 1.0


def test_flatness_matches_the_definition_on_random_histograms():
    # The decision of the integer test 5 min n >= 4 sum against min >= 0.8 mean
    # in exact rationals, for histograms spread around the threshold.
    rng = np.random.default_rng(7)
    for trial in range(300):
        n = int(rng.integers(1, 20))
        base = int(rng.integers(1, 50))
        H = rng.integers(max(base - base // 3, 0), base + base // 3 + 1, size=n)
        H[0] = max(int(np.round(0.8 * H.mean())) + int(rng.integers(-1, 2)), 0)
        o = fresh(m=1)
        plant(o, 0, [counts(list(H), first=0)])
        o.sync_window(0)
        want = flat_by_definition(H, Fraction(4, 5))
        assert (o.window(0)["lnf"] == 0.5) == want, (trial, list(H))


# --------------------------------------------------------------------------
# The visited set is the window's: the union over its walkers, since creation.

def test_bin_missed_by_one_walker_is_not_flat():
    # Walker 1 never reached bin 7, which walker 0 did: over the window's
    # visited bins walker 1's minimum is 0, so the window is not flat (over
    # walker 1's own bins alone it would be).
    o = fresh()
    plant(o, 0, [counts([5, 5, 5, 5, 5]), counts([5, 5, 5, 5])])
    o.sync_window(0)
    w = o.window(0)
    assert w["lnf"] == 1.0 and w["iterations"] == 0
    # control: with that bin counted for walker 1 as well, the window is flat
    o = fresh()
    plant(o, 0, [counts([5, 5, 5, 5, 5]), counts([5, 5, 5, 5, 5])])
    o.sync_window(0)
    assert o.window(0)["lnf"] == 0.5


def test_bins_visited_in_an_earlier_period_still_count():
    # After a halving H restarts; a bin the window reached before still belongs
    # to the visited set, so missing it in the next period is not flat.
    o = fresh(m=1)
    plant(o, 0, [counts([5, 5, 5, 5, 5, 5])])
    o.sync_window(0)
    assert o.window(0)["lnf"] == 0.5
    H = np.zeros(o.W, dtype=np.uint32)
    H[3:8] = 5
    v = np.zeros(o.W, dtype=np.uint8)
    v[3:9] = 1                       # the walker's flags keep bin 8 (reached before)
    o.plant_walker(0, H, v)
    o.sync_window(0)
    assert o.window(0)["lnf"] == 0.5 and o.window(0)["iterations"] == 1


def test_unvisited_bins_do_not_count():
    # Bins no walker has reached (H = 0 there) are outside the test.
    o = fresh()
    plant(o, 0, [counts([6, 6, 6], first=10), counts([6, 6, 6], first=10)])
    o.sync_window(0)
    assert o.window(0)["lnf"] == 0.5


# --------------------------------------------------------------------------
# ln f is halved once per all-flat sync point; ln g is averaged.

def test_lnf_halves_exactly_once_and_ln_g_is_averaged():
    o = fresh(m=3, lnf=0.75)
    rows = [np.arange(o.W, dtype=np.float64) * s for s in (1.0, 2.0, 6.0)]
    for j, r in enumerate(rows):
        o.set_lng(j, r)
    plant(o, 0, [counts([5, 5, 5, 5, 5])] * 3)
    o.sync_window(0)
    w = o.window(0)
    assert w["lnf"] == 0.375 and w["iterations"] == 1 and w["regime"] == 0
    for j in range(3):
        np.testing.assert_array_equal(o.walker(j)["lng"], np.arange(o.W) * 3.0)
    # a second sync point with a histogram that is not flat leaves ln f alone
    plant(o, 0, [counts([1, 5, 5, 5, 5])] * 3)
    o.sync_window(0)
    assert o.window(0)["lnf"] == 0.375 and o.window(0)["iterations"] == 1


# --------------------------------------------------------------------------
# The 1/t schedule.

@pytest.mark.parametrize("dt, switch", [(0, True), (-1, True), (1, False)])
def test_one_over_t_switch_at_the_halved_value(dt, switch):
    # ln f 2^-10 halves to 2^-11.  W/t with t = step / W equals 2^-11 at
    # step = W 2^11: the switch happens when the halved value is <= W/t.
    o = fresh(schedule=1, lnf=2.0**-10)
    step = o.W * (2**11 + dt)
    o.set_step(step)
    plant(o, 0, [counts([5, 5, 5, 5, 5])] * 2)
    o.sync_window(0)
    w = o.window(0)
    if switch:
        assert w["regime"] == 1 and w["lnf"] == o.W / step
    else:
        assert w["regime"] == 0 and w["lnf"] == 2.0**-11


def test_halving_schedule_never_switches():
    o = fresh(schedule=0, lnf=2.0**-10)
    o.set_step(o.W * 2**12)              # W/t far above the halved ln f
    plant(o, 0, [counts([5, 5, 5, 5, 5])] * 2)
    o.sync_window(0)
    assert o.window(0)["regime"] == 0 and o.window(0)["lnf"] == 2.0**-11


def test_one_over_t_regime_needs_no_flatness():
    # In the 1/t regime every sync point averages, clears H and sets ln f = W/t,
    # flat or not.
    o = fresh(schedule=1, lnf=1e-3)
    o.set_window(0, 1e-3, regime=1)
    o.set_lng(0, np.full(o.W, 2.0))
    o.set_lng(1, np.full(o.W, 4.0))
    o.set_step(123_456)
    plant(o, 0, [counts([1, 9, 0, 9]), counts([9, 9, 9, 9])])
    o.sync_window(0)
    w = o.window(0)
    assert w["regime"] == 1 and w["lnf"] == o.W / 123_456 and w["iterations"] == 1
    assert not o.walker(0)["H"].any()
    np.testing.assert_array_equal(o.walker(1)["lng"], np.full(o.W, 3.0))


# --------------------------------------------------------------------------
# Termination of a window: ln f < ln f_final.

@pytest.mark.parametrize("lnf, finished", [(2.0**-2, False), (2.0**-3, True)])
def test_window_finishes_below_lnf_final(lnf, finished):
    o = fresh(lnf=lnf, lnf_final=2.0**-3)
    plant(o, 0, [counts([5, 5, 5, 5, 5])] * 2)
    o.sync_window(0)
    w = o.window(0)
    assert w["finished"] == int(finished)
    if finished:
        assert w["lnf"] == 0.0 and w["lnf_last"] == 2.0**-4
    else:
        assert w["lnf"] == 2.0**-3


def test_windows_are_independent():
    # A flat window halves; its non-flat neighbour keeps its ln f.
    o = fresh(h=2)
    plant(o, 0, [counts([5, 5, 5, 5, 5], first=2)] * 2)
    plant(o, 1, [counts([0, 5, 5, 5, 5], first=2), counts([5, 5, 5, 5, 5], first=2)])
    o.sync_window(0)
    o.sync_window(1)
    assert o.window(0)["lnf"] == 0.5 and o.window(1)["lnf"] == 1.0
