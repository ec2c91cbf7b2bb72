"""Pins of the CPU oracle against facts it does not compute itself.

Each test ties one oracle routine to something independent: rocRAND's
Philox, mpmath's exp, complete enumeration of tiny lattices, closed forms of
the Potts model, the exchange rule of Eq. (1) under exact weights, and the
numbers the paper prints.  A plausible slip anywhere in the oracle (a wrong
sign in the acceptance, a swapped index in Eq. (1), a dropped bond in the
energy, a wrong shift in the join) fails at least one of them.
"""
import json
import math
import os
import subprocess

import mpmath as mp
import numpy as np
import pytest

import oracle
from oracle import bruteforce
import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def exact_lng(L, q):
    g = bruteforce.potts_dos(L, q)
    out = np.full(g.size, -np.inf)
    out[g > 0] = np.log(g[g > 0].astype(np.float64))
    return out


# --------------------------------------------------------------------------
# Philox4x32-10 against rocRAND (black box through its public API).

def test_philox_matches_rocrand(rocrand_ref):
    rng = np.random.default_rng(12345)
    cases = []
    for _ in range(300):
        seed = int(rng.integers(0, 2**63))
        c = [int(x) for x in rng.integers(0, 2**32, size=4, dtype=np.uint64)]
        c[1] &= (1 << 30) - 1          # keep 4 * (low 64 bits) inside the offset range
        cases.append((seed, c))
    # the counters the library actually uses: small steps, walker ids, domains
    for seed in (0, 1, 2**32 + 7):
        for c in ([0, 0, 0, 0], [1, 0, 3, 0], [9999, 0, 63, 2 << 24], [5, 0, 7, (3 << 24) | 17]):
            cases.append((seed, c))
    stdin = "".join(f"{s} {c[2] | (c[3] << 32)} {4 * (c[0] | (c[1] << 32))}\n" for s, c in cases)
    res = subprocess.run([rocrand_ref], input=stdin, capture_output=True, text=True, check=True)
    ref = [list(map(int, line.split())) for line in res.stdout.strip().splitlines()]
    assert len(ref) == len(cases)
    for (seed, c), want in zip(cases, ref):
        got = oracle.philox(c, [seed & 0xFFFFFFFF, seed >> 32])
        assert list(got) == want, (seed, c)


# --------------------------------------------------------------------------
# exp_poly against mpmath.

def test_exp_poly_constants():
    mp.mp.prec = 200
    ln2 = mp.log(2)
    inv, c1, c2 = oracle.constants()
    assert inv == float(1 / ln2)
    # C1 has at most 40 significant bits and C1 + C2 = ln 2 to double-double accuracy
    m, e = math.frexp(c1)
    assert (m * 2**40) == int(m * 2**40)
    assert c2 == float(ln2 - mp.mpf(c1))
    invf, c1f, c2f = oracle.constants32()
    assert np.float32(invf) == np.float32(float(1 / ln2))
    assert float(c2f) == float(np.float32(float(ln2 - mp.mpf(float(c1f)))))


def ulp(x):
    return math.ulp(x)


def test_exp_poly_accuracy():
    mp.mp.prec = 120
    rng = np.random.default_rng(1)
    xs = np.concatenate([-rng.uniform(0, 64, 6000), -rng.uniform(0, 1e-3, 500),
                         -np.array([1e-300, 1e-20, 0.5 * math.log(2), math.log(2), 1.0, 10.0, 63.999999,
                                    64.0, 0.34657359027997264, 0.3465735902799727])])
    worst = 0.0
    for x in xs:
        got = oracle.exp_poly(float(x))
        want = mp.exp(mp.mpf(float(x)))
        err = abs(mp.mpf(got) - want) / mp.mpf(ulp(float(want)))
        worst = max(worst, float(err))
    assert worst <= 2.0, worst
    assert oracle.exp_poly(-64.0000001) == 0.0
    assert oracle.exp_poly(-1000.0) == 0.0


def test_exp_poly32_accuracy():
    mp.mp.prec = 80
    rng = np.random.default_rng(2)
    xs = np.concatenate([-rng.uniform(0, 64, 4000), -rng.uniform(0, 1e-3, 300)]).astype(np.float32)
    worst = 0.0
    for x in xs:
        got = oracle.exp_poly32(float(x))
        want = mp.exp(mp.mpf(float(x)))
        u = float(np.spacing(np.float32(float(want))))
        worst = max(worst, float(abs(mp.mpf(got) - want) / mp.mpf(u)))
    assert worst <= 2.0, worst


def test_twosum_pair_keeps_small_increments():
    # Plain binary32 loses every increment below half an ulp of the running
    # value; the (hi, lo) pair must keep them.  1000 increments is more than a
    # bin receives between two sync points (where the pair is renormalised).
    hi, lo = oracle.twosum_accumulate(16384.0, 0.0, 1e-4, 1000)
    exact = 16384.0 + 1000 * float(np.float32(1e-4))
    assert abs((hi + lo) - exact) < 5e-6
    hi, lo = oracle.twosum_accumulate(1.0, 0.0, 0.3, 1000)      # increments above an ulp
    assert abs((hi + lo) - (1.0 + 1000 * float(np.float32(0.3)))) < 1e-9
    plain = np.float32(16384.0)
    for _ in range(1000):
        plain = np.float32(plain + np.float32(1e-4))
    assert plain == np.float32(16384.0)  # the failure the pair avoids


# --------------------------------------------------------------------------
# Window layout (Sec. 2, Fig. 1) against the paper's L=300 setup.

def test_window_layout_paper_L300():
    paper = json.load(open(os.path.join(GOLDEN, "paper_values.json")))["potts_L300"]
    L, h, o = paper["L"], paper["windows"], paper["overlap"]
    N = L * L
    W, starts = oracle.window_layout(2 * N + 1, h, o, -2 * N)
    assert starts[0] == -2 * N and starts[-1] + W - 1 == 0
    strides = np.diff(starts)
    # 717 equal windows at 75% overlap over 180,001 energies: W = 1001, stride 250
    assert W == 1001 and np.all(strides == 250)
    assert abs((W - 250) / W - o) < 1e-3
    assert h * paper["walkers_per_window"] == 2151  # "approximately 2000 walkers"


@pytest.mark.parametrize("L,h,o", [(8, 4, 0.75), (32, 16, 0.75), (80, 64, 0.75), (16, 8, 0.75),
                                   (48, 8, 0.75), (5, 3, 0.5), (7, 1, 0.75), (10, 9, 0.9)])
def test_window_layout_properties(L, h, o):
    N = L * L
    B = 2 * N + 1
    W, starts = oracle.window_layout(B, h, o, -2 * N)
    assert starts[0] == -2 * N and starts[-1] + W - 1 == 0
    assert np.all(np.diff(starts) >= 0)
    if h > 1:
        # each overlap is within one bin of the requested fraction
        ov = (starts[:-1] + W - starts[1:]) / W
        assert np.all(np.abs(ov - o) <= 1.0 / W + (1 - o) / (h - 1)), ov
        # W is the smallest width for which h windows at overlap o cover B
        assert W - 1 < B / (1 + (h - 1) * (1 - o)) <= W


def test_window_layout_cfg_values():
    W, starts = oracle.window_layout(129, 4, 0.75, -128)
    assert W == 74 and list(starts) == [-128, -110, -91, -73]
    assert oracle.window_layout(2049, 16, 0.75, -2048)[0] == 432
    assert oracle.window_layout(12801, 64, 0.75, -12800)[0] == 765


# --------------------------------------------------------------------------
# Potts energy (Eq. 2) and the brute-force density of states.

def test_potts_energy_matches_enumeration():
    for L, q in [(3, 3), (4, 2)]:
        e = bruteforce.potts_energies(L, q)
        rng = np.random.default_rng(L)
        idx = rng.integers(0, q ** (L * L), 200)
        for i in idx:
            digits = [(int(i) // q**k) % q for k in range(L * L)]
            assert oracle.potts_energy(np.array(digits, dtype=np.int8), L) == e[i]
    for L in (3, 4, 8, 9):
        assert oracle.potts_energy(np.zeros(L * L, np.int8), L) == -2 * L * L
    cb = (np.add.outer(np.arange(8), np.arange(8)) % 2).astype(np.int8)
    assert oracle.potts_energy(cb.reshape(-1), 8) == 0


@pytest.mark.parametrize("L,q", [(3, 3), (4, 2), (3, 2), (3, 4)])
def test_bruteforce_closed_forms(L, q):
    N = L * L
    g = bruteforce.potts_dos(L, q)
    assert g.sum() == q ** N                       # every configuration counted once
    assert g[0] == q                               # ground states: all spins equal
    assert g[1] == g[2] == g[3] == 0               # a domain wall on a torus costs >= 4 bonds
    assert g[4] == N * q * (q - 1)                 # single flipped spin
    if q == 2:
        assert np.all(g[1::2] == 0)                # Ising: broken bonds come in pairs per cycle
        if L % 2 == 0:
            assert np.array_equal(g, g[::-1])      # bipartite lattice: E <-> -2N - E


def test_thermo_matches_direct_sums():
    for L, q in [(4, 2), (3, 3)]:
        lng = exact_lng(L, q)
        T = np.array([0.3, 0.7, 1.0, 2.27, 5.0])
        lnZ, U, C = oracle.thermo(lng, -2 * L * L, T)
        ref = bruteforce.potts_partition(L, q, T)
        np.testing.assert_allclose(lnZ, ref[:, 0], rtol=1e-12)
        np.testing.assert_allclose(U, ref[:, 1], rtol=1e-10, atol=1e-10)
        np.testing.assert_allclose(C, ref[:, 2], rtol=1e-9)
    # infinite temperature: every bond is satisfied with probability 1/q
    lng = exact_lng(3, 3)
    _, U, _ = oracle.thermo(lng, -18, np.array([1e9]))
    assert abs(U[0] - (-18 / 3)) < 1e-6


# --------------------------------------------------------------------------
# The full REWL protocol against the exact density of states.

def converged(L, q, h, m, precision=0, seed=3, threads=4):
    spins = workloads.init_spins(L, q, h * m, seed)
    o = oracle.Rewl(L, q, h, 0.75, m, spins, seed=seed, lnf_final=1e-6, schedule=1,
                    sync_attempts=20000, precision=precision, threads=threads)
    st = o.run(10**10)
    assert st == oracle.CONVERGED
    return o


@pytest.mark.parametrize("L,q,h", [(4, 2, 2), (3, 3, 2)])
def test_converged_dos_matches_enumeration(L, q, h):
    o = converged(L, q, h, 4)
    st, lng, cuts = o.join()
    assert st == oracle.OK
    ex = exact_lng(L, q)
    reach = np.isfinite(ex)
    assert np.array_equal(np.isfinite(lng), reach)   # visited bins = reachable energies
    assert np.max(np.abs(lng[reach] - ex[reach])) <= 0.02
    if q == 2:
        assert np.max(np.abs(lng[reach] - lng[::-1][reach])) <= 0.02
    for k in range(h):
        w = o.window(k)
        assert w["finished"] == 1 and w["regime"] == 1 and w["lnf_last"] < 1e-6
    # every walker's energy still agrees with a full recount of its lattice
    for w in range(o.nw):
        d = o.walker(w)
        assert d["E"] == oracle.potts_energy(d["spins"], L)
        k = w // o.m
        assert o.starts[k] <= d["E"] <= o.starts[k] + o.W - 1


def test_converged_dos_fp32_pair():
    o = converged(4, 2, 2, 4, precision=1)
    st, lng, _ = o.join()
    ex = exact_lng(4, 2)
    reach = np.isfinite(ex)
    assert st == oracle.OK and np.array_equal(np.isfinite(lng), reach)
    assert np.max(np.abs(lng[reach] - ex[reach])) <= 0.02


def test_fixed_exact_weights_give_flat_histogram():
    # With ln g fixed at the exact values (ln f = 0) the walk samples every
    # reachable energy equally often (the WL acceptance of Sec. 2).  A sign
    # or index slip in the acceptance makes H far from flat.
    L, q = 4, 2
    ex = exact_lng(L, q)
    spins = workloads.init_spins(L, q, 1, 5)
    o = oracle.Rewl(L, q, 1, 0.75, 1, spins, seed=9, lnf_init=0.0, fixed_lnf=1, sync_attempts=10**6)
    lng = np.where(np.isfinite(ex), ex, 0.0)
    o.set_lng(0, lng)
    o.run(3_000_000)
    H = o.walker(0)["H"].astype(np.float64)
    reach = np.isfinite(ex)
    assert np.all(H[~reach] == 0)
    rel = H[reach] / H[reach].mean()
    assert np.max(np.abs(rel - 1.0)) < 0.05, rel


def test_exchange_accepts_everything_under_exact_weights():
    # Eq. (1): if every walker's ln g is the exact ln g up to a per-walker
    # constant, the exchange ratio is 1 and every exchange whose energies lie
    # in both windows is accepted; others are rejected.
    L, q, h = 4, 2, 3
    ex = exact_lng(L, q)
    spins = workloads.init_spins(L, q, h, 11)
    o = oracle.Rewl(L, q, h, 0.75, 1, spins, seed=4, lnf_init=0.0, fixed_lnf=1, exchange=0,
                    sync_attempts=500)
    rng = np.random.default_rng(0)
    for w in range(h):
        k = w
        seg = ex[o.starts[k] - o.e_lo: o.starts[k] - o.e_lo + o.W]
        o.set_lng(w, np.where(np.isfinite(seg), seg, 0.0) + rng.normal() * 50)
    o.walkin()
    eligible_total = 0
    for rnd in range(60):
        o.run(97)
        E = [o.walker(w)["E"] for w in range(h)]
        k = rnd % 2
        if k + 1 < h:
            inside = (o.starts[k] <= E[k + 1] <= o.starts[k] + o.W - 1 and
                      o.starts[k + 1] <= E[k] <= o.starts[k + 1] + o.W - 1)
            before = o.window(k)["x_acc"]
            reps = (o.walker(k)["replica"], o.walker(k + 1)["replica"])
            o.exchange()
            after = o.window(k)["x_acc"]
            assert after - before == int(inside)
            eligible_total += int(inside)
            if inside:
                assert (o.walker(k)["replica"], o.walker(k + 1)["replica"]) == reps[::-1]
                assert o.walker(k)["E"] == E[k + 1] and o.walker(k + 1)["E"] == E[k]
        else:
            o.exchange()
    assert eligible_total > 5


def _trips_from_history(windows, h):
    # Round trips of one replica from the sequence of windows it was seen in:
    # keep only the visits to the end windows ('L' lowest, 'H' highest), drop
    # everything before the first 'L', merge repeats; every "HL" that remains
    # closes one lowest -> highest -> lowest path.
    ends = "".join("L" if k == 0 else "H" for k in windows if k in (0, h - 1))
    ends = ends[ends.find("L"):] if "L" in ends else ""
    merged = "".join(c for i, c in enumerate(ends) if i == 0 or c != ends[i - 1])
    return merged.count("HL")


@pytest.mark.parametrize("h,m", [(3, 2), (4, 1), (2, 3), (1, 2)])
def test_replica_round_trips_replayed(h, m):
    # Replica ids move only with accepted exchanges (Eq. (1)); the round-trip
    # counts and the walker-by-replica visit counts (Fig. 7) must equal those
    # replayed from the positions seen at every lookup: creation, each sync
    # point (here every 500 attempts, no exchange there) and each exchange
    # round called on its own.  Exact weights make most exchanges acceptable,
    # so replicas cross the whole range many times.
    L, q = 4, 2
    ex = exact_lng(L, q)
    nw = h * m
    spins = workloads.init_spins(L, q, nw, 13)
    o = oracle.Rewl(L, q, h, 0.75, m, spins, seed=5, lnf_init=0.0, fixed_lnf=1, exchange=0,
                    sync_attempts=500)
    for w in range(nw):
        k = w // m
        seg = ex[o.starts[k] - o.e_lo: o.starts[k] - o.e_lo + o.W]
        o.set_lng(w, np.where(np.isfinite(seg), seg, 0.0))
    o.walkin()
    hist = [[r // m] for r in range(nw)]
    visits = np.eye(nw, dtype=np.int64)
    lookups = 1

    def look():
        reps = [o.walker(w)["replica"] for w in range(nw)]
        for w, r in enumerate(reps):
            visits[w, r] += 1
        return reps

    for rnd in range(300):
        before = o.step // 500
        o.run(31)
        for _ in range(o.step // 500 - before):      # sync points: positions unchanged
            look()
            lookups += 1
        o.exchange()
        for w, r in enumerate(look()):
            hist[r].append(w // m)
        lookups += 1
        if rnd % 50 == 49 or rnd == 299:
            win, trips = o.replicas()
            assert list(win) == [hst[-1] for hst in hist]
            assert list(trips) == [_trips_from_history(hst, h) if h > 1 else 0 for hst in hist]
            got = np.stack([o.replica_visits(w) for w in range(nw)])
            assert np.array_equal(got, visits)
    assert np.all(got.sum(axis=0) == lookups) and np.all(got.sum(axis=1) == lookups)
    assert o.step // 500 >= 18
    if h > 1:
        assert sum(trips) >= 3
        assert sorted(win) == sorted(w // m for w in range(nw))
        assert np.count_nonzero(got[0]) == nw          # every replica reached slot 0
    else:
        assert not trips.any()


@pytest.mark.parametrize("bias,accepted", [(-100.0, 0), (100.0, 1), (-1e-12, 1)])
def test_exchange_planted_weights(bias, accepted):
    # Walker a carries X at E_X = -24 and walker b carries Y at E_Y = -20 (4x4
    # Ising, two windows [-32,-6] and [-26,0], both energies in the overlap).
    # With ln g_b = 0, Eq. (1) gives ln P = ln g_a(E_X) - ln g_a(E_Y) = bias:
    # -100 must be rejected (exp(-100) underflows the 2^-32 grid), +100 accepted,
    # and a ratio a hair below one accepted unless u = 1 - 2^-32.
    L, q = 4, 2
    x = np.zeros(16, np.int8); x[[0, 10]] = 1            # two isolated flips: E = -24
    y = np.zeros(16, np.int8); y[[0, 2, 9]] = 1          # three isolated flips: E = -20
    assert oracle.potts_energy(x, L) == -24 and oracle.potts_energy(y, L) == -20
    o = oracle.Rewl(L, q, 2, 0.75, 1, np.stack([x, y]), seed=4, lnf_init=0.0, fixed_lnf=1, exchange=0)
    assert list(o.starts) == [-32, -26] and o.W == 27
    a = np.zeros(o.W)
    a[-24 - o.starts[0]] = bias
    o.set_lng(0, a)
    assert o.walkin() == oracle.OK
    o.exchange()
    assert o.window(0)["x_att"] == 1 and o.window(0)["x_acc"] == accepted
    assert o.walker(0)["E"] == (-20 if accepted else -24)
    assert o.walker(1)["replica"] == (0 if accepted else 1)


# --------------------------------------------------------------------------
# Joining (Sec. 2, Fig. 2) and determinism.

def test_join_recovers_exact_dos_from_shifted_pieces():
    for L, q, h in [(4, 2, 3), (3, 3, 2), (4, 2, 4)]:
        ex = exact_lng(L, q)
        N = L * L
        B = 2 * N + 1
        W, starts = oracle.window_layout(B, h, 0.75, -2 * N)
        rng = np.random.default_rng(h)
        pieces = np.zeros((h, W))
        vis = np.zeros((h, W), np.uint8)
        for k in range(h):
            seg = ex[starts[k] + 2 * N: starts[k] + 2 * N + W]
            vis[k] = np.isfinite(seg)
            pieces[k] = np.where(np.isfinite(seg), seg, 0.0) + rng.uniform(-100, 100)
        st, out, cuts = oracle.join_pieces(pieces, vis, starts, -2 * N, B, N * math.log(q))
        assert st == oracle.OK
        fin = np.isfinite(ex)
        assert np.array_equal(np.isfinite(out), fin)
        np.testing.assert_allclose(out[fin], ex[fin], atol=1e-9)
        for k in range(h - 1):
            assert starts[k + 1] <= cuts[k] <= starts[k] + W - 1


def test_join_picks_best_matching_slope():
    # Two pieces that agree in slope only at one energy: the join must cut there.
    W = 20
    starts = np.array([0, 10], np.int32)
    e = np.arange(30, dtype=np.float64)
    a = 0.1 * e[:W] ** 2 / 2           # beta_a(E) = 0.1 E
    b = 1.5 * e[10:30] + 7.0           # beta_b(E) = 1.5 -> equal at E = 15
    vis = np.ones((2, W), np.uint8)
    st, out, cuts = oracle.join_pieces(np.stack([a, b]), vis, starts, 0, 30, 0.0)
    assert st == oracle.OK and cuts[0] == 15


def test_split_runs_and_thread_count_are_bitwise_identical():
    L, q, h, m = 4, 3, 3, 2
    spins = workloads.init_spins(L, q, h * m, 21)
    kw = dict(seed=77, sync_attempts=700, lnf_final=1e-3)
    a = oracle.Rewl(L, q, h, 0.75, m, spins, threads=1, **kw)
    b = oracle.Rewl(L, q, h, 0.75, m, spins, threads=4, **kw)
    a.run(12345)
    for n in (1000, 345, 7000, 4000):
        b.run(n)
    assert a.step == b.step and a.round == b.round
    for w in range(h * m):
        da, db = a.walker(w), b.walker(w)
        for key in ("spins", "H", "lng"):
            assert np.array_equal(da[key], db[key]), key
        assert da["E"] == db["E"] and da["replica"] == db["replica"]
    for k in range(h):
        wa, wb = a.window(k), b.window(k)
        assert wa["lnf"] == wb["lnf"] and wa["iterations"] == wb["iterations"]


def test_walkin_places_every_walker_in_its_window():
    L, q, h, m = 8, 10, 4, 2
    spins = workloads.init_spins(L, q, h * m, 1)
    o = oracle.Rewl(L, q, h, 0.75, m, spins, seed=1)
    assert o.walkin() == oracle.OK
    for w in range(h * m):
        d = o.walker(w)
        k = w // m
        assert o.starts[k] <= d["E"] <= o.starts[k] + o.W - 1
        assert d["E"] == oracle.potts_energy(d["spins"], L)


def test_walkin_budget_error():
    L, q = 8, 10
    spins = np.zeros((4, 64), np.int8)                 # all at the ground state
    o = oracle.Rewl(L, q, 4, 0.75, 1, spins, seed=1)
    assert o.walkin(budget=3) == oracle.EBUDGET


def test_invalid_parameters_are_rejected():
    s = np.zeros((1, 4), np.int8)
    with pytest.raises(ValueError):
        oracle.Rewl(2, 2, 1, 0.5, 1, s)
    s = np.zeros((1, 9), np.int8)
    with pytest.raises(ValueError):
        oracle.Rewl(3, 1, 1, 0.5, 1, s)
    with pytest.raises(ValueError):
        oracle.Rewl(3, 2, 1, 1.0, 1, s)
    with pytest.raises(ValueError):
        oracle.Rewl(3, 3, 1, 0.5, 1, np.full((1, 9), 3, np.int8))


# ---------------------------------------------------------------------------
# The ln g shadow (exact reference of the accumulated ln g along a trajectory).
from fractions import Fraction as Fr


def _dd(p):
    return Fr(p[0]) + Fr(p[1])


def test_double_double_steps_against_exact_rationals():
    rng = np.random.default_rng(5)
    for _ in range(2000):
        a = float(rng.uniform(-1e4, 1e4))
        a = oracle.dd_add((a, 0.0), (float(rng.uniform(-1e-12, 1e-12)), 0.0))   # a genuine pair
        b = (float(rng.uniform(-1e4, 1e4)), 0.0)
        b = oracle.dd_add(b, (float(rng.uniform(-1e-12, 1e-12)), 0.0))
        s = oracle.dd_add(a, b)
        exact = _dd(a) + _dd(b)
        if exact != 0:
            assert abs(_dd(s) - exact) <= abs(exact) * Fr(1, 2**100)
        n = int(rng.integers(1, 2**32))
        x = float(rng.uniform(0, 1))
        assert _dd(oracle.dd_mul_count(n, x)) == n * Fr(x)          # exact product
        m = int(rng.integers(1, 1025))
        q = oracle.dd_div_int(a, m)
        assert abs(_dd(q) - _dd(a) / m) <= abs(_dd(a) / m) * Fr(1, 2**100)


def test_shadow_is_exact_for_fixed_increments():
    # Fixed ln f = 0.1 (not a binary fraction): no averaging, so bin b of a
    # walker holds H(b) additions of the same double ln f.
    spins = workloads.init_spins(5, 3, 4, 3)
    o = oracle.Rewl(5, 3, 2, 0.75, 2, spins, seed=4, lnf_init=0.1, fixed_lnf=1, sync_attempts=500,
                    shadow=1)
    o.run(20_000)
    lnf = Fr(0.1)
    worst64 = Fr(0)
    for w in range(4):
        d = o.walker(w)
        hi, lo = o.shadow(w)
        for b in range(o.W):
            exact = int(d["H"][b]) * lnf
            assert abs(Fr(hi[b]) + Fr(lo[b]) - exact) <= exact * Fr(1, 2**100)
            worst64 = max(worst64, abs(Fr(d["lng"][b]) - exact))
    # the binary64 sums of 0.1 do round, by far less than the count times an ulp
    assert 0 < worst64 < Fr(1, 10**9)


@pytest.mark.parametrize("m", [2, 4])
def test_shadow_equals_binary64_where_the_arithmetic_is_exact(m):
    # Halving from ln f = 1 keeps every increment a power of two, and the
    # average over m = 2 or 4 walkers divides by a power of two: binary64 ln g
    # is then exact, and its shadow must equal it bit for bit.
    spins = workloads.init_spins(4, 2, 2 * m, 7)
    o = oracle.Rewl(4, 2, 2, 0.75, m, spins, seed=6, lnf_init=1.0, lnf_final=1e-3, sync_attempts=400,
                    shadow=1, threads=4)
    assert o.run(10**8) == oracle.CONVERGED
    assert min(o.window(k)["iterations"] for k in range(2)) >= 5
    for w in range(2 * m):
        hi, lo = o.shadow(w)
        assert np.array_equal(hi, o.walker(w)["lng"]) and not np.any(lo)


def test_shadow_measures_the_pair_rounding():
    # binary32 (hi, lo) ln g adds ln f rounded to binary32 (TwoSum keeps the
    # rest exact), so along the same trajectory ln g - shadow must be
    # H(b) * (f32(ln f) - ln f) plus the pair's own (tiny) rounding.
    spins = workloads.init_spins(6, 4, 3, 9)
    o = oracle.Rewl(6, 4, 1, 0.75, 3, spins, seed=2, lnf_init=0.1, fixed_lnf=1, sync_attempts=1000,
                    precision=1, shadow=1)
    o.run(50_000)
    step = float(np.float32(0.1)) - 0.1
    for w in range(3):
        hi, lo = o.shadow(w)
        g = o.walker(w)["lng"]
        err = (g - hi) - lo
        expect = o.walker(w)["H"].astype(np.float64) * step
        assert np.max(np.abs(expect)) > 1e-6
        assert np.max(np.abs(err - expect)) < 1e-11


def test_walkin_lid_places_walkers_and_shortens_the_walk():
    # The lid keeps the walk-in's flooded band narrow: every walker still ends
    # inside its window, after far fewer attempts than the unbounded walk.
    spins = workloads.init_spins(32, 10, 16, 4)
    att = {}
    for slack in (0, 16):
        o = oracle.Rewl(32, 10, 16, 0.75, 1, spins, seed=3, walkin_slack=slack, threads=8)
        assert o.walkin() == 0
        for w in range(16):
            E = o.walker(w)["E"]
            assert o.starts[w] <= E <= o.starts[w] + o.W - 1
        att[slack] = max(o.walker(w)["walkin_attempts"] for w in range(16))
    assert att[16] * 10 < att[0]
    with pytest.raises(ValueError):
        oracle.Rewl(16, 10, 8, 0.75, 1, workloads.init_spins(16, 10, 8, 4), walkin_slack=-1)


# ---------------------------------------------------------------------------
# Trimer model (continuous bead displacements).
def _trimer(coords, nmol, box=10.0, e_min=-50.0, bin_w=0.5, bins=400, h=1, m=1, **kw):
    return oracle.Rewl.trimer(nmol, box, e_min, bin_w, bins, h, 0.75, m, coords, **kw)


def test_trimer_pair_energies_closed_forms():
    # one molecule along x with unit bonds: both bonds at rest, head-tail2 at
    # r = 2 beyond the WCA range -> E = 0; a second molecule's tail at the LJ
    # minimum r = 2^(1/6) from the first tail2 -> E = -1 (the binary32
    # coordinates carry r to ~1e-7, so -1 to ~1e-6).
    c = np.array([[1.0, 5.0, 5.0], [2.0, 5.0, 5.0], [3.0, 5.0, 5.0]], dtype=np.float32)
    o = _trimer(c[None], 1)
    assert o.trimer_energy(0) == 0.0
    rmin = 2.0 ** (1.0 / 6.0)
    c2 = np.array([[3.0 + rmin + 2.0, 5.0, 5.0], [3.0 + rmin + 1.0, 5.0, 5.0], [3.0 + rmin, 5.0, 5.0]],
                  dtype=np.float32)
    o2 = _trimer(np.concatenate([c, c2])[None], 2)
    # pairs: tail2(0)-tail2(1) at rmin -> -1; tail2(0)-tail1(1) at rmin+1 -> LJ(2.122);
    # tail1(0)-tail2(1) at rmin+1; tail1(0)-tail1(1) at rmin+2 -> LJ(3.12) = 0 (cut)
    lj = lambda r: 4 * (r ** -12 - r ** -6) if r < 2.5 else 0.0
    expect = -1.0 + 2 * lj(rmin + 1.0)
    assert abs(o2.trimer_energy(0) - expect) < 1e-5
    # bond stretched to r = 1.5: 100 * 0.25 = 25
    c3 = c.copy()
    c3[2, 0] = 3.5
    assert abs(_trimer(c3[None], 1).trimer_energy(0) - 25.0) < 1e-9
    # WCA: head and tail2 at r = 1 (tail2 folded back): 4 (1 - 1) + 1 = 1, bonds 0
    c4 = np.array([[1.0, 5.0, 5.0], [2.0, 5.0, 5.0], [1.5, 5.0 + np.sqrt(0.75), 5.0]], dtype=np.float32)
    assert abs(_trimer(c4[None], 1).trimer_energy(0) - 1.0) < 1e-5


def test_trimer_minimum_image():
    # tails of two molecules across the periodic boundary: x = 0.3 and 9.3 are
    # 1.0 apart through the wall, the LJ energy of r = 1 is 0.
    a = np.array([[0.3, 2.0, 2.0], [0.3, 3.0, 2.0], [0.3, 4.0, 2.0]], dtype=np.float32)
    b = np.array([[9.3, 2.0, 8.0], [9.3, 3.0, 8.0], [9.3, 4.0, 8.0]], dtype=np.float32)   # z 6 apart
    base = _trimer(np.concatenate([a, b])[None], 2).trimer_energy(0)
    b2 = b.copy()
    b2[:, 2] = 2.0
    e = _trimer(np.concatenate([a, b2])[None], 2).trimer_energy(0)
    # heads at r = 1 (WCA: 4 (1 - 1) + 1 = 1), tail1-tail1 and tail2-tail2 at
    # r = 1 (LJ 0), the two tail1-tail2 pairs at sqrt(2); head-tail pairs at
    # sqrt(2) lie beyond the WCA range
    lj = lambda r: 4 * (r ** -12 - r ** -6)
    assert abs((e - base) - (1.0 + 2 * lj(np.sqrt(2.0)))) < 1e-5


def _np_trimer_energy(x, box):
    """Plain binary64 sum of the trimer force field over all pairs (numpy)."""
    n = len(x)
    e = 0.0
    for i in range(n):
        for j in range(i + 1, n):
            d = (x[j] - x[i]).astype(np.float32)
            d = np.where(d > box / 2, d - box, np.where(d < -box / 2, d + box, d)).astype(np.float64)
            r2 = float(np.sum(d * d))
            if i // 3 == j // 3 and abs(i % 3 - j % 3) == 1:
                e += 100.0 * (np.sqrt(r2) - 1.0) ** 2
            elif i % 3 > 0 and j % 3 > 0:
                e += 4 * (r2 ** -6 - r2 ** -3) if r2 < 6.25 else 0.0
            elif r2 < 2 ** (1 / 3):
                e += 4 * (r2 ** -6 - r2 ** -3) + 1.0
    return e


def test_trimer_delta_matches_recomputed_energy_and_drift():
    # Energies are exact sums of the pair terms rounded once to multiples of
    # 2^-32: a move's change equals the difference of the two totals exactly,
    # and the total agrees with the plain binary64 sum within the rounding of
    # the terms (one half unit of 2^-32 per pair, plus the float sum's own).
    x = workloads.init_trimers(8, 5.0, 1, 3)
    o = _trimer(x, 8, box=5.0, e_min=-200.0, bins=1000)
    assert abs(o.trimer_energy(0) - _np_trimer_energy(x[0], 5.0)) <= 300 * 2.0**-33 + 1e-12
    rng = np.random.default_rng(1)
    cur = x[0].copy()
    for _ in range(200):
        b = int(rng.integers(24))
        xn = np.mod(cur[b] + rng.uniform(-0.1, 0.1, 3), 5.0).astype(np.float32)
        d = o.trimer_delta_fx(0, b, xn)
        e0 = _trimer(cur[None], 8, box=5.0, e_min=-200.0, bins=1000).trimer_energy_fx(0)
        cur2 = cur.copy()
        cur2[b] = xn
        e1 = _trimer(cur2[None], 8, box=5.0, e_min=-200.0, bins=1000).trimer_energy_fx(0)
        assert d == e1 - e0
    # the incremental energy of a long run equals a full recompute exactly
    o = _trimer(x, 8, box=5.0, e_min=-200.0, bins=1000, lnf_init=0.0, fixed_lnf=1, sync_attempts=10_000)
    o.run(100_000)
    assert o.energy_fx(0) == o.trimer_energy_fx(0)


def test_trimer_hard_overlap_is_refused_and_rejected():
    # a pair term of 2^18 or more is a hard overlap: a start holding one is
    # refused, and a move creating one is no move at all
    c = np.array([[1.0, 5.0, 5.0], [2.0, 5.0, 5.0], [3.0, 5.0, 5.0],
                  [1.0, 5.0, 5.3], [2.0, 5.0, 6.3], [3.0, 5.0, 7.3]], dtype=np.float32)   # heads 0.3 apart
    with pytest.raises(ValueError):
        _trimer(c[None], 2)
    c[3, 2] = 6.0
    o = _trimer(c[None], 2, e_min=-50.0)
    assert o.trimer_delta_fx(0, 3, np.array([1.0, 5.0, 5.3], dtype=np.float32)) is None
    assert o.trimer_delta_fx(0, 3, np.array([1.0, 5.0, 5.9], dtype=np.float32)) is not None


def test_trimer_fixed_weights_detailed_balance():
    # ln f = 0 and flat ln g: every move inside the range is accepted, so the
    # run is a uniform random walk; with the bead displacement symmetric the
    # energy histogram is the density of states itself, and the walker keeps
    # a consistent energy and bin.
    x = workloads.init_trimers(4, 4.0, 2, 5)
    o = _trimer(x, 4, box=4.0, e_min=-60.0, bins=400, m=2, lnf_init=0.0, fixed_lnf=1, sync_attempts=5000)
    o.run(20_000)
    for w in range(2):
        d = o.walker(w)
        assert d["H"].sum() == 20_000
        assert d["E"] == (o.energy_fx(w) + 60 * 2**32) // 2**31
        assert o.energy_fx(w) == o.trimer_energy_fx(w)


def test_trimer_workload_range_covers_the_anneal_and_the_starts():
    # the trimer workload's bins reach below the lowest energy a seeded
    # Metropolis anneal (the oracle's walk with weights beta E) finds, and
    # above every starting energy of its walkers
    from oracle import trimer_range
    lowest, starts, ok = trimer_range.check()
    assert ok, (lowest, starts.min(), starts.max())
    assert lowest < starts.min() - 300      # the anneal really descends


def test_trimer_rewl_walks_in_and_converges():
    x = workloads.init_trimers(2, 4.0, 4, 8)
    o = _trimer(x, 2, box=4.0, e_min=-6.0, bin_w=0.5, bins=24, h=2, m=2, lnf_init=1.0, lnf_final=1e-3,
                sync_attempts=2000, threads=4)
    assert o.run(10**8) == oracle.CONVERGED
    st, lng, cuts = o.join()
    assert st == 0
    fin = np.isfinite(lng)
    assert fin.sum() > 10
    assert abs(np.log(np.exp(lng[fin]).sum())) < 1e-9          # sum over bins of g = 1
    for w in range(4):
        assert o.starts[w // 2] <= o.walker(w)["E"] <= o.starts[w // 2] + o.W - 1


# --------------------------------------------------------------------------
# Production sampling with fixed weights and observable histograms H(E, O)
# (Sec. 3.2).  O = max_s n_s, the population of the most occupied state.

def enumerate_potts(L, q):
    """Energy and O of every configuration of the L x L lattice (periodic, each bond once)."""
    N = L * L
    idx = np.arange(q ** N, dtype=np.int64)
    s = np.stack([(idx // q ** i) % q for i in range(N)], axis=1).reshape(-1, L, L)
    E = -((s == np.roll(s, 1, axis=1)).sum(axis=(1, 2)) + (s == np.roll(s, 1, axis=2)).sum(axis=(1, 2)))
    O = np.max(np.stack([(s == v).sum(axis=(1, 2)) for v in range(q)]), axis=0)
    return E, O


@pytest.mark.parametrize("h,m,nb", [(1, 2, 7), (2, 1, 26), (3, 2, 1)])
def test_obs_sampled_at_sync_points_from_the_current_lattice(h, m, nb):
    # Each sync point adds the configuration each walker holds then: one count
    # in H(E, O) at O bin floor(O nb / (N + 1)), O added to the bin's sum.
    L, q, S = 5, 4, 50
    N = L * L
    spins = workloads.init_spins(L, q, h * m, 21)
    o = oracle.Rewl(L, q, h, 0.75, m, spins, seed=6, lnf_init=0.05, fixed_lnf=1, exchange=0,
                    sync_attempts=S, obs_bins=nb)
    hist = np.zeros((h * m, o.W, nb), dtype=np.int64)
    tot = np.zeros((h * m, o.W), dtype=np.int64)
    cnt = np.zeros((h * m, o.W), dtype=np.int64)
    for _ in range(6):
        o.run(S)
        for w in range(h * m):
            d = o.walker(w)
            O = int(np.bincount(d["spins"], minlength=q).max())
            b = d["E"] - o.starts[w // m]
            assert 0 <= b < o.W
            hist[w, b, O * nb // (N + 1)] += 1
            tot[w, b] += O
            cnt[w, b] += 1
    for w in range(h * m):
        gh, gs, gc = o.obs(w)
        assert np.array_equal(gh, hist[w]) and np.array_equal(gs, tot[w]) and np.array_equal(gc, cnt[w])


def test_obs_distribution_under_exact_weights_matches_enumeration():
    # With weights 1/g(E) the walk samples, at each energy, configurations
    # uniformly; the pooled H(E, O) must approach the exact conditional
    # distribution of O at E, and the pooled mean of O the exact one.
    L, q = 3, 3
    E, O = enumerate_potts(L, q)
    N = L * L
    ex = exact_lng(L, q)
    e_lo = -2 * N
    spins = workloads.init_spins(L, q, 4, 23)
    o = oracle.Rewl(L, q, 2, 0.75, 2, spins, seed=3, lnf_init=0.0, fixed_lnf=1, exchange=1,
                    sync_attempts=9, obs_bins=N + 1)
    for w in range(4):
        k = w // 2
        seg = ex[o.starts[k] - e_lo: o.starts[k] - e_lo + o.W]
        o.set_lng(w, np.where(np.isfinite(seg), seg, 0.0))
    o.run(9 * 60_000)
    mean, cnt = o.obs_micro()
    reach = np.isfinite(ex)
    assert np.all(cnt[reach] > 0) and np.all(cnt[~reach] == 0)
    pooled = np.zeros((o.B, N + 1))
    for w in range(4):
        off = o.starts[w // 2] - e_lo
        pooled[off: off + o.W] += o.obs(w)[0]
    for b in np.flatnonzero(reach):
        at = E == b + e_lo
        exact_mean = O[at].mean()
        exact_p = np.bincount(O[at], minlength=N + 1) / at.sum()
        assert abs(mean[b] - exact_mean) < 0.08, (b, mean[b], exact_mean)
        assert np.max(np.abs(pooled[b] / pooled[b].sum() - exact_p)) < 0.05, b


def test_obs_thermo_matches_canonical_enumeration():
    L, q = 3, 3
    E, O = enumerate_potts(L, q)
    N = L * L
    B = 2 * N + 1
    n_at = np.bincount(E + 2 * N, minlength=B)
    lng = np.full(B, -np.inf)
    lng[n_at > 0] = np.log(n_at[n_at > 0])
    mu = np.full(B, np.nan)
    for b in np.flatnonzero(n_at):
        mu[b] = O[E + 2 * N == b].mean()
    T = np.array([0.2, 0.5, 0.9, 1.5, 4.0, 50.0])
    got = oracle.obs_thermo(lng, mu, -2 * N, T)
    for t, g in zip(T, got):
        x = -E / t
        p = np.exp(x - x.max())
        assert g == pytest.approx(float((p * O).sum() / p.sum()), rel=1e-12)


def test_production_after_convergence_keeps_weights_and_samples_o():
    L, q = 3, 3
    E, O = enumerate_potts(L, q)
    N = L * L
    spins = workloads.init_spins(L, q, 4, 29)
    o = oracle.Rewl(L, q, 2, 0.75, 2, spins, seed=8, lnf_final=1e-3, sync_attempts=90, obs_bins=5)
    assert o.begin_production() != 0          # not walked in yet
    assert o.run(10**9) == oracle.CONVERGED
    step = o.step
    lng0 = [o.walker(w)["lng"].copy() for w in range(4)]
    assert o.begin_production() == 0
    assert all(o.window(k)["lnf"] == 0.0 and o.window(k)["finished"] == 1 for k in range(2))
    assert all(o.walker(w)["H"].sum() == 0 for w in range(4))
    assert o.run(90 * 10_000) == oracle.OK
    assert o.step == step + 90 * 10_000
    for w in range(4):
        d = o.walker(w)
        assert np.array_equal(d["lng"], lng0[w]) and d["H"].sum() == 90 * 10_000
        assert o.obs(w)[2].sum() == 10_000
    mean, cnt = o.obs_micro()
    for b in np.flatnonzero(cnt > 500):
        assert abs(mean[b] - O[E == b - 2 * N].mean()) < 0.15, b


# --------------------------------------------------------------------------
# Error analysis (Sec. 2): independent runs, bootstrap resampling with the
# joining points found anew for every resample; the error claims of Sec. 2.

def _converged_runs(L, q, h, m, lnf_final, R, seed0=1000):
    runs = []
    for r in range(R):
        spins = workloads.init_spins(L, q, h * m, seed0 + r)
        o = oracle.Rewl(L, q, h, 0.75, m, spins, seed=77, instance=r, lnf_final=lnf_final, sync_attempts=500,
                        threads=4)
        assert o.run(10**12) == oracle.CONVERGED
        runs.append(o)
    return runs


def test_bootstrap_of_identical_runs_has_no_spread():
    o = _converged_runs(4, 2, 3, 2, 1e-3, 1)[0]
    p, v = oracle.run_pieces(o)
    T = np.array([0.5, 1.0, 2.0, 4.0])
    st, out = oracle.bootstrap(np.stack([p] * 5), np.stack([v] * 5), o.starts, o.e_lo, o.B,
                               16 * math.log(2), 50, 9, T)
    assert st == 0
    s, lng, _ = o.join()
    fin = np.isfinite(lng)
    assert np.array_equal(np.isfinite(out["lng_mean"]), fin)
    np.testing.assert_allclose(out["lng_mean"][fin], lng[fin], rtol=0, atol=1e-12)
    # every replicate is the same curve; only the rounding of the means is left
    assert out["lng_std"].max() < 1e-12 and out["U_std"].max() < 1e-12 and out["C_std"].max() < 1e-12
    _, U, C = oracle.thermo(lng, o.e_lo, T)
    np.testing.assert_allclose(out["U_mean"], U, rtol=1e-12)
    np.testing.assert_allclose(out["C_mean"], C, rtol=1e-12)


def test_bootstrap_resamples_runs_with_replacement():
    # Two runs a, b: a replicate joins the mean of the two drawn runs' pieces,
    # i.e. a, (a + b) / 2 or b, with probabilities 1/4, 1/2, 1/4.
    runs = _converged_runs(4, 2, 3, 2, 1e-2, 2)
    (pa, va), (pb, vb) = (oracle.run_pieces(o) for o in runs)
    o = runs[0]
    vis = np.stack([va, vb])
    union = vis.max(axis=0)
    lt = 16 * math.log(2)
    outcomes = []
    for pieces in (pa, (pa + pb) / 2.0, pb):
        st, lng, _ = oracle.join_pieces(pieces, union, o.starts, o.e_lo, o.B, lt)
        assert st == 0
        outcomes.append(lng)
    assert not np.array_equal(outcomes[0], outcomes[2])
    counts = [0, 0, 0]
    for seed in range(400):
        st, out = oracle.bootstrap(np.stack([pa, pb]), vis, o.starts, o.e_lo, o.B, lt, 1, seed, [1.0])
        assert st == 0
        hit = [i for i, x in enumerate(outcomes) if np.array_equal(x, out["lng_mean"])]
        assert len(hit) == 1
        counts[hit[0]] += 1
    freq = np.array(counts) / 400
    assert np.all(np.abs(freq - [0.25, 0.5, 0.25]) < 0.07), freq


def test_error_falls_with_walkers_per_window_and_with_final_lnf():
    # Sec. 2: averaging the m walkers of a window cuts the statistical error as
    # 1/sqrt(m) (squared error / m); the error also falls with ln f_final.
    # 4x4 Ising-like q=2 lattice, exact ln g by enumeration, 32 runs each.
    L, q = 4, 2
    ex = exact_lng(L, q)
    reach = np.isfinite(ex)
    mse = {}
    for m in (1, 4):
        for lf in (1e-3, 1e-4):
            e = []
            for o in _converged_runs(L, q, 2, m, lf, 32):
                st, lng, _ = o.join()
                e.append(np.mean((lng[reach] - ex[reach]) ** 2))
            mse[m, lf] = np.mean(e)
    for lf in (1e-3, 1e-4):
        assert 2.0 < mse[1, lf] / mse[4, lf] < 8.0, mse
    for m in (1, 4):
        assert mse[m, 1e-3] / mse[m, 1e-4] > 2.0, mse


def test_bootstrap_spread_matches_the_spread_of_independent_runs():
    # The bootstrap standard deviation of ln g (mean of R runs) must agree with
    # the sample standard deviation of the runs' joined ln g over sqrt(R).
    L, q, R = 4, 2, 32
    runs = _converged_runs(L, q, 2, 4, 1e-4, R)
    o = runs[0]
    pv = [oracle.run_pieces(r) for r in runs]
    st, out = oracle.bootstrap(np.stack([p for p, _ in pv]), np.stack([v for _, v in pv]), o.starts, o.e_lo,
                               o.B, 16 * math.log(2), 400, 3, [1.0, 2.5])
    assert st == 0
    joined = np.stack([r.join()[1] for r in runs])
    fin = np.all(np.isfinite(joined), axis=0)
    sd = np.full(o.B, np.inf)
    sd[fin] = joined[:, fin].std(axis=0)
    fin[np.argmin(sd)] = False   # the bin the normalisation nearly pins
    direct = joined[:, fin].std(axis=0, ddof=1) / math.sqrt(R)
    ratio = np.median(out["lng_std"][fin] / direct)
    assert 0.8 < ratio < 1.25, ratio
    assert np.all(out["U_std"] > 0) and np.all(out["C_std"] > 0)


# --------------------------------------------------------------------------
# Lipid model with explicit solvent (Sec. 3.2, Eqs. (3)-(5), Fig. 5).

P_, H_, W_ = 0, 1, 2


def _lipid_small(nlip=4, nsol=20, box=4.3, seed=3, walkers=1, **kw):
    x = workloads.init_lipids(nlip, nsol, box, walkers, seed)
    args = dict(lnf_init=0.0, fixed_lnf=1, sync_attempts=10**9)
    args.update(kw)
    return oracle.Rewl.lipid(nlip, nsol, box, -2000.0, 1.0, 6000, 1, 0.0, walkers, x, **args), x


def _np_pair(ti, tj, bonded, r2, eps_ww=1.0):
    """Eqs. (3)-(5) written out with mpmath-grade numpy (independent of the oracle)."""
    if bonded:
        if r2 >= 1.69:
            return np.inf
        v = -0.5 * 30.0 * 1.69 * math.log(1.0 - r2 / 1.69)
        if r2 < 2 ** (1 / 3):
            v += 4.0 * (r2 ** -6 - r2 ** -3) + 1.0
        return v
    if r2 >= 6.25:
        return 0.0
    if (ti == H_) != (tj == H_):
        return 4.0 * (1.05 ** 2 / r2) ** 4.5
    v = 4.0 * (r2 ** -6 - r2 ** -3)
    return eps_ww * v if ti == W_ and tj == W_ else v


def _np_energy(x, types, lipids, box, eps_ww=1.0):
    n = len(types)
    pos = {}
    for k, row in enumerate(lipids):
        for p, i in enumerate(row):
            pos[int(i)] = (k, p)
    e = 0.0
    for i in range(n):
        for j in range(i + 1, n):
            d = (x[j] - x[i]).astype(np.float32)
            d = np.where(d > np.float32(box / 2), d - np.float32(box), np.where(d < -np.float32(box / 2),
                                                                              d + np.float32(box), d))
            r2 = float(np.sum(d.astype(np.float64) ** 2))
            a, b = pos.get(i), pos.get(j)
            bonded = a is not None and b is not None and a[0] == b[0] and abs(a[1] - b[1]) == 1
            e += _np_pair(types[i], types[j], bonded, r2, eps_ww)
    return e


def test_log_poly_accuracy():
    # the logarithm built from basic operations (FENE term of Eq. (5))
    rng = np.random.default_rng(1)
    xs = np.concatenate([rng.uniform(1e-6, 1, 2000), rng.uniform(0.999, 1, 200), 10 ** rng.uniform(-15, 0, 500)])
    for x in xs:
        ref = float(mp.log(mp.mpf(float(x))))
        assert abs(oracle.log_poly(x) - ref) <= 3 * np.spacing(abs(ref)) + 1e-300
    assert oracle.log_poly(1.0) == 0.0 and oracle.log_poly(0.5) == -math.log(2.0)


def test_lipid_potentials_closed_forms():
    o, _ = _lipid_small(eps_ww=0.7)
    assert o.lipid_pair(H_, W_, 0, 1.05 ** 2) == pytest.approx(4.0, rel=1e-14)   # Eq. (3) at r = sigma_rep
    assert o.lipid_pair(H_, P_, 0, 1.05 ** 2) == pytest.approx(4.0, rel=1e-14)
    assert o.lipid_pair(P_, W_, 0, 2 ** (1 / 3)) == pytest.approx(-1.0, rel=1e-14)  # Eq. (4) minimum
    assert o.lipid_pair(H_, H_, 0, 2 ** (1 / 3)) == pytest.approx(-1.0, rel=1e-14)
    assert o.lipid_pair(W_, W_, 0, 2 ** (1 / 3)) == pytest.approx(-0.7, rel=1e-14)  # eps_WW
    assert o.lipid_pair(W_, W_, 0, 6.25) == 0.0 and o.lipid_pair(H_, W_, 0, 6.3) == 0.0
    fene = float(-0.5 * 30 * 1.69 * mp.log(1 - mp.mpf(1) / mp.mpf("1.69")))
    assert o.lipid_pair(P_, H_, 1, 1.0) == pytest.approx(fene + 1.0, rel=1e-14)   # Eq. (5), WCA part 1 at r = 1
    r2 = mp.mpf("1.21")                                                         # r = 1.1 < 2^(1/6)
    ref = -0.5 * 30 * mp.mpf("1.69") * mp.log(1 - r2 / mp.mpf("1.69")) + 4 * (r2 ** -6 - r2 ** -3) + 1
    assert o.lipid_pair(H_, H_, 1, 1.21) == pytest.approx(float(ref), rel=1e-14)
    r2 = mp.mpf("1.44")                                                         # r = 1.2: FENE alone
    assert o.lipid_pair(H_, H_, 1, 1.44) == pytest.approx(float(-0.5 * 30 * mp.mpf("1.69") * mp.log(1 - r2 / mp.mpf("1.69"))), rel=1e-14)
    assert o.lipid_pair(H_, H_, 1, 1.69) == np.inf
    for (ti, tj, b, r2) in [(H_, W_, 0, 1.7), (W_, W_, 0, 1.2), (P_, H_, 1, 0.9), (H_, H_, 0, 2.0)]:
        assert o.lipid_pair(ti, tj, b, r2) == pytest.approx(_np_pair(ti, tj, b, r2, 0.7), rel=1e-12)


def test_lipid_energy_and_displacement_match_direct_sums():
    o, x0 = _lipid_small(eps_ww=0.7)
    x, t, lp = o.lipid_state(0)
    assert list(t[:6]) == [P_, H_, H_, P_, H_, H_] and np.all(t[12:] == W_)
    e = _np_energy(x, t, lp, 4.3, 0.7)
    npair = len(x) * (len(x) - 1) // 2
    assert abs(o.lipid_energy(0) - e) <= npair * 2.0**-33 + 1e-10 * abs(e)
    assert o.energy_fx(0) == o.lipid_energy_fx(0)
    rng = np.random.default_rng(5)
    for b in (0, 1, 2, 7, 13, 23):
        xn = np.mod(x[b] + rng.uniform(-0.1, 0.1, 3), 4.3).astype(np.float32)
        x2 = x.copy()
        x2[b] = xn
        ref = _np_energy(x2, t, lp, 4.3, 0.7) - e
        assert o.lipid_delta_move(0, b, xn) == pytest.approx(ref, rel=1e-9, abs=1e-9)


def _near_solvent(x, t, e, box):
    d = x - x[e]
    d = np.where(d > box / 2, d - box, np.where(d < -box / 2, d + box, d)).astype(np.float64)
    r2 = np.sum(d * d, axis=1)
    return [j for j in range(len(t)) if j != e and t[j] == W_ and r2[j] < 1.69]


def test_lipid_reptation_moves_bonds_types_and_reverses():
    # Fig. 5: a solvent particle near one end becomes the new end bead, the
    # beads shift along the chain, the far end is released as solvent.
    o, _ = _lipid_small(nlip=6, nsol=30, box=4.3, seed=7)
    done = 0
    for lipid in range(6):
        for end in (0, 1):
            x, t, lp = o.lipid_state(0)
            e0 = o.energy_fx(0)
            cand = _near_solvent(x, t, lp[lipid][0 if end == 0 else 2], 4.3)
            if not cand:
                assert o.lipid_reptate(0, lipid, end, 0) is None
                continue
            pick = len(cand) // 2
            cap = cand[pick]
            nc, nr, de = o.lipid_reptate(0, lipid, end, pick)
            x2, t2, lp2 = o.lipid_state(0)
            old = list(lp[lipid])
            new = [cap] + old[:2] if end == 0 else old[1:] + [cap]
            released = old[2] if end == 0 else old[0]
            assert list(lp2[lipid]) == new and [t2[i] for i in new] == [P_, H_, H_] and t2[released] == W_
            assert nc == len(cand) and nr == len(_near_solvent(x2, t2, old[1], 4.3))
            assert released in _near_solvent(x2, t2, old[1], 4.3)
            # within the rounding of the changed pair terms (4 np of them at most)
            assert oracle.fx_to_float(de) == pytest.approx(_np_energy(x2, t2, lp2, 4.3) - _np_energy(x, t, lp, 4.3),
                                                       rel=1e-9, abs=4 * len(x) * 2.0**-33 + 1e-9)
            # exact: the change is the difference of the recomputed totals
            assert o.energy_fx(0) == e0 + de == o.lipid_energy_fx(0)
            # the reverse move: capture the released particle at the other end
            back = _near_solvent(x2, t2, old[1], 4.3).index(released)
            nc2, nr2, de2 = o.lipid_reptate(0, lipid, 1 - end, back)
            x3, t3, lp3 = o.lipid_state(0)
            assert np.array_equal(t3, t) and np.array_equal(lp3, lp) and (nc2, nr2) == (nr, nc)
            assert o.energy_fx(0) == e0 and de2 == -de
            done += 1
    assert done >= 4


def test_lipid_reptation_bias_correction_gives_uniform_states():
    # One lipid and six solvent particles frozen on a 3x3 square lattice
    # (spacing 1: only edge neighbours are within R = 1.3), reptation moves
    # only, flat weights: the acceptance min[1, n_c / n_r] makes every lipid
    # placement (an ordered self-avoiding 3-site path) equally likely,
    # although the number of candidates differs from site to site.
    box = 8.0
    sites = np.array([[i, j, 0.0] for j in range(3) for i in range(3)], dtype=np.float32) + 2.0
    order = [0, 1, 2, 3, 4, 5, 6, 7, 8]
    x = sites[order][None]
    o = oracle.Rewl.lipid(1, 6, box, -1000.0, 1.0, 3000, 1, 0.0, 1, x, rep_prob=1.0, lnf_init=0.0, fixed_lnf=1,
                          sync_attempts=10**9)
    counts = {}
    for _ in range(30000):
        o.run(1)
        key = tuple(o.lipid_state(0)[2][0])
        counts[key] = counts.get(key, 0) + 1
    # reachable placements: ordered paths of 3 edge-adjacent sites
    adj = {s: [t for t in range(9) if abs(s % 3 - t % 3) + abs(s // 3 - t // 3) == 1] for s in range(9)}
    paths = {(a, b, c) for a in range(9) for b in adj[a] for c in adj[b] if c != a}
    assert set(counts) <= paths and len(counts) == len(paths)
    freq = np.array([counts[p] for p in sorted(paths)], dtype=np.float64)
    expected = freq.sum() / len(paths)
    chi2 = float(np.sum((freq - expected) ** 2 / expected))
    # correlated samples: allow a generous bound (dof = 43); a missing n_c/n_r
    # factor drives chi2 into the thousands
    assert chi2 < 400, chi2
