"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Integer state (lattices, energies, histograms, replica ids, counters, joining
energies) must be identical.  ln g must be identical bit for bit: both sides
evaluate the same sequence of separately rounded IEEE operations.  Only the
log-sum-exp normalisation and the thermodynamic sums (different summation
order, library exp/log) carry a tolerance.
"""
import sys

import numpy as np
import pytest

import oracle
from oracle import bruteforce
import workloads
from statecmp import assert_same_state

pytestmark = pytest.mark.gpu


def _pk():
    import paper_1312_3004_amd as pk
    return pk


def make_pair(L, q, h, m, overlap=0.75, spins_seed=1, threads=8, **opts):
    spins = workloads.init_spins(L, q, h * m, spins_seed)
    print(f"[case] L={L} q={q} h={h} m={m} opts={opts}", flush=True)
    sys.stdout.flush()
    g = _pk().Rewl(L, q, h, overlap, m, spins, **opts)
    o = oracle.Rewl(L, q, h, overlap, m, spins, threads=threads, **opts)
    return g, o


FIXED_CASES = [
    # (L, q, h, m, attempts, precision)
    (3, 3, 2, 2, 20011, 0),
    (4, 2, 3, 2, 30000, 0),
    (8, 10, 4, 1, 64123, 0),
    (8, 10, 4, 3, 50000, 1),
    (32, 10, 16, 4, 40000, 0),
    (32, 10, 16, 4, 40000, 1),
    (13, 5, 5, 3, 25000, 0),
]


@pytest.mark.parametrize("L,q,h,m,attempts,precision", FIXED_CASES)
def test_fixed_lnf_trajectories_bitexact(L, q, h, m, attempts, precision):
    g, o = make_pair(L, q, h, m, lnf_init=0.05, fixed_lnf=1, sync_attempts=997, exchange=1,
                     precision=precision, seed=5)
    g.run(attempts)
    o.run(attempts)
    assert_same_state(g, o)


@pytest.mark.parametrize("precision", [0, 1])
def test_fixed_lnf_L80_precision_shape_bitexact(precision):
    # The precision workload's shape: L = 80, 64 windows x 16 walkers (1,024
    # walkers: several per CU, the hashed conflict-tag table of 6,400 sites),
    # walk-in under the lid, then fixed-ln f sync intervals with exchange
    # rounds; ln f is not a binary fraction, so both formats round.
    c = workloads.CONFIGS["potts_q10_L80"]
    g, o = make_pair(c["L"], c["q"], c["windows"], c["walkers"], lnf_init=1.0 / (3 * 2**17), fixed_lnf=1,
                     sync_attempts=c["sync_attempts"], exchange=1, precision=precision, seed=c["seed"],
                     threads=16)
    for n in (12_345, 17_655):
        g.run(n)
        o.run(n)
    assert_same_state(g, o)


@pytest.mark.parametrize("precision", [0, 1])
def test_full_protocol_L8_bitexact_to_convergence(precision):
    c = workloads.CONFIGS["potts_q10_L8"]
    g, o = make_pair(c["L"], c["q"], c["windows"], c["walkers"], seed=c["seed"], flat=c["flat"],
                     lnf_init=c["lnf_init"], lnf_final=c["lnf_final"], schedule=c["schedule"],
                     sync_attempts=c["sync_attempts"], exchange=c["exchange"], precision=precision)
    assert g.run(10**10) == _pk().CONVERGED
    assert o.run(10**10) == oracle.CONVERGED
    assert_same_state(g, o)
    sg, lg, cg = g.join()
    so, lo, co = o.join()
    assert sg == so == 0
    assert np.array_equal(cg, co)
    fin = np.isfinite(lo)
    assert np.array_equal(np.isfinite(lg), fin)
    assert np.max(np.abs(lg[fin] - lo[fin])) <= 1e-10
    T = np.linspace(0.5, 1.0, 201)
    zg, ug, cvg = g.thermo(T)
    zo, uo, cvo = oracle.thermo(lo, -128, T)
    np.testing.assert_allclose(zg, zo, rtol=1e-12, atol=1e-9)
    np.testing.assert_allclose(ug, uo, rtol=1e-9, atol=1e-8)
    np.testing.assert_allclose(cvg, cvo, rtol=1e-8, atol=1e-8)


def test_full_protocol_L32_segment_bitexact():
    # The benchmark workload (L=32, 16 windows x 4 walkers, 1/t schedule),
    # element by element after walk-in and 3 x 10^5 attempts per walker.
    c = workloads.CONFIGS["potts_q10_L32"]
    g, o = make_pair(c["L"], c["q"], c["windows"], c["walkers"], seed=c["seed"], flat=c["flat"],
                     lnf_init=c["lnf_init"], lnf_final=c["lnf_final"], schedule=c["schedule"],
                     sync_attempts=c["sync_attempts"], exchange=c["exchange"])
    for n in (123_457, 76_543, 100_000):
        g.run(n)
        o.run(n)
    assert_same_state(g, o)


def test_split_runs_equal_one_run():
    args = dict(lnf_init=1.0, lnf_final=1e-3, sync_attempts=700, seed=3)
    spins = workloads.init_spins(6, 4, 6, 2)
    a = _pk().Rewl(6, 4, 3, 0.75, 2, spins, **args)
    b = _pk().Rewl(6, 4, 3, 0.75, 2, spins, **args)
    a.run(20_000)
    for n in (1, 63, 64, 65, 699, 700, 701, 17_707):
        b.run(n)
    assert a.step == b.step == 20_000
    for w in range(6):
        da, db = a.walker(w), b.walker(w)
        assert np.array_equal(da["spins"], db["spins"]) and da["E"] == db["E"]
        assert np.array_equal(da["lng"], db["lng"]) and np.array_equal(da["H"], db["H"])


def test_manual_exchange_rounds():
    g, o = make_pair(8, 3, 5, 2, lnf_init=0.02, fixed_lnf=1, exchange=0, sync_attempts=500, seed=8)
    for _ in range(7):
        g.run(333)
        o.run(333)
        g.exchange()
        o.exchange()
    assert_same_state(g, o)


def test_converged_dos_matches_enumeration_on_gpu():
    L, q, h, m = 4, 2, 2, 4
    g, o = make_pair(L, q, h, m, seed=3, lnf_final=1e-6, schedule=1, sync_attempts=20000, spins_seed=3)
    assert g.run(10**10) == _pk().CONVERGED
    st, lng, _ = g.join()
    gex = bruteforce.potts_dos(L, q)
    ex = np.full(gex.size, -np.inf)
    ex[gex > 0] = np.log(gex[gex > 0].astype(float))
    reach = np.isfinite(ex)
    assert st == 0 and np.array_equal(np.isfinite(lng), reach)
    assert np.max(np.abs(lng[reach] - ex[reach])) <= 0.02
    assert o.run(10**10) == oracle.CONVERGED
    assert_same_state(g, o)


# (128, 2, 8, 1): lattice plus ln g and H rows just fit the 160 KiB LDS;
# (128, 2, 4, 1) and (96, 3, 2, 2): they do not, the rows stay in device memory
@pytest.mark.parametrize("L,q,h,m", [(3, 127, 1, 1), (3, 2, 1, 7), (5, 3, 1, 64), (128, 2, 16, 1), (128, 2, 8, 1),
                                     (128, 2, 4, 1), (96, 3, 2, 2)])
def test_edge_shapes(L, q, h, m):
    g, o = make_pair(L, q, h, m, lnf_init=0.5, lnf_final=1e-2, sync_attempts=300, seed=2)
    n = 3000 if L < 100 else 1000
    g.run(n)
    o.run(n)
    assert_same_state(g, o)


@pytest.mark.parametrize("precision", [0, 1])
def test_rows_in_device_memory_small_lnf_bitexact(precision):
    # a run too large for LDS rows (96 x 96, 2 windows of 14,747 bins) on the
    # speculative path (small fixed ln f), several sync intervals
    g, o = make_pair(96, 3, 2, 2, lnf_init=3e-7, fixed_lnf=1, sync_attempts=4001, exchange=1, seed=19,
                     precision=precision)
    g.run(12_003)
    o.run(12_003)
    assert_same_state(g, o)


def test_fixed_exact_weights_and_set_lng():
    L, q = 4, 2
    gex = bruteforce.potts_dos(L, q)
    lng = np.where(gex > 0, np.log(np.maximum(gex, 1).astype(float)), 0.0)
    g, o = make_pair(L, q, 1, 1, lnf_init=0.0, fixed_lnf=1, sync_attempts=10**6, seed=9, spins_seed=5)
    g.set_lng(0, lng)
    o.set_lng(0, lng)
    g.run(500_000)
    o.run(500_000)
    assert_same_state(g, o)
    H = g.walker(0)["H"].astype(float)
    reach = gex > 0
    assert np.max(np.abs(H[reach] / H[reach].mean() - 1)) < 0.1


def test_replica_round_trips_bitexact():
    # Exact weights make most exchanges acceptable (Eq. (1)), so replicas
    # cross the whole range many times; sync points with an exchange round
    # every 31 attempts, then manual rounds.
    L, q, h, m = 4, 2, 3, 2
    gex = bruteforce.potts_dos(L, q)
    ex = np.where(gex > 0, np.log(np.maximum(gex, 1).astype(float)), 0.0)
    g, o = make_pair(L, q, h, m, lnf_init=0.0, fixed_lnf=1, sync_attempts=31, exchange=1, seed=5,
                     spins_seed=13)
    for w in range(h * m):
        k = w // m
        seg = ex[o.starts[k] - o.e_lo: o.starts[k] - o.e_lo + o.W]
        g.set_lng(w, seg)
        o.set_lng(w, seg)
    g.run(31 * 400)
    o.run(31 * 400)
    assert_same_state(g, o)
    for _ in range(9):
        g.exchange()
        o.exchange()
    assert_same_state(g, o)
    win, trips = g.replicas()
    assert trips.sum() >= 10 and sorted(win) == sorted(w // m for w in range(h * m))


def test_replica_visits_kept_up_to_4096_walkers():
    pk = _pk()
    spins = workloads.init_spins(64, 2, 65 * 64, 3)
    print("[case] L=64 q=2 h=65 m=64 replica visits limit", flush=True)
    g = pk.Rewl(64, 2, 65, 0.75, 64, spins, seed=1)
    win, trips = g.replicas()
    assert np.array_equal(win, np.arange(65 * 64) // 64) and not trips.any()
    with pytest.raises(pk.RewlError):
        g.replica_visits(0)
    del g
    g = pk.Rewl(64, 2, 64, 0.75, 64, spins[:4096], seed=1)
    v = g.replica_visits(4095)
    assert v[4095] == 1 and v.sum() == 1


def test_walkin_budget_error_on_gpu():
    spins = np.zeros((4, 64), np.int8)
    g = _pk().Rewl(8, 10, 4, 0.75, 1, spins, seed=1)
    with pytest.raises(_pk().RewlError):
        g.walkin(budget=3)


TABLE_CASES = [
    # (L, q, h, m, attempts, precision, lnf): ln f small enough for the
    # block-table decision path of the attempt kernel
    (8, 10, 4, 2, 40_000, 0, 1e-5),
    (32, 10, 16, 4, 30_000, 0, 1e-7),
    (32, 10, 16, 4, 30_000, 1, 1e-7),
    (4, 2, 2, 3, 30_000, 0, 1e-4),
    (13, 5, 5, 3, 25_000, 1, 2e-4),
    (24, 3, 8, 2, 20_000, 0, 3e-6),
]


@pytest.mark.parametrize("L,q,h,m,attempts,precision,lnf", TABLE_CASES)
def test_small_lnf_trajectories_bitexact(L, q, h, m, attempts, precision, lnf):
    g, o = make_pair(L, q, h, m, lnf_init=lnf, fixed_lnf=1, sync_attempts=1009, exchange=1,
                     precision=precision, seed=11)
    g.run(attempts)
    o.run(attempts)
    assert_same_state(g, o)


@pytest.mark.parametrize("precision", [0, 1])
def test_large_lng_small_lnf_replay_bitexact(precision):
    # ln g values in the thousands with ln f = 3.6e-7 (the 1/t phase of the L=32
    # workload): the speculative commit replays a bin's n visits in closed form,
    # in binary64, and for the (hi, lo) pair whose high word ln f leaves unchanged,
    # in the low word
    L, q, h, m = 32, 10, 4, 2
    g, o = make_pair(L, q, h, m, lnf_init=3.6e-7, fixed_lnf=1, sync_attempts=4001, exchange=1,
                     precision=precision, seed=17)
    for w in range(h * m):
        lng = 1500.0 + 1.4 * np.arange(g.W, dtype=np.float64) + 0.37 * np.sin(0.01 * w * np.arange(g.W))
        g.set_lng(w, lng)
        o.set_lng(w, lng)
    g.run(40_003)
    o.run(40_003)
    assert_same_state(g, o)


@pytest.mark.parametrize("tilt,precision", [(0.7, 0), (-0.7, 0), (0.7, 1), (0.05, 0), (17.0, 0), (-17.0, 1)])
def test_tilted_weights_drive_walker_across_cache(tilt, precision):
    # A steep fixed ln g makes the walker drift through a wide window, so it
    # leaves the 64-energy register cache inside a block.
    L, q = 16, 4
    g, o = make_pair(L, q, 1, 1, lnf_init=1e-6, fixed_lnf=1, sync_attempts=5000, seed=13,
                     precision=precision)
    lng = tilt * np.arange(g.W, dtype=np.float64)
    g.set_lng(0, lng)
    o.set_lng(0, lng)
    g.run(20_011)
    o.run(20_011)
    assert_same_state(g, o)


def assert_same_shadow(g, o):
    for w in range(g.nw):
        gh, gl = g.shadow(w)
        oh, ol = o.shadow(w)
        assert np.array_equal(gh.view(np.uint64), oh.view(np.uint64)), f"shadow hi of walker {w}"
        assert np.array_equal(gl.view(np.uint64), ol.view(np.uint64)), f"shadow lo of walker {w}"


@pytest.mark.parametrize("precision,lnf", [(0, 0.1), (1, 0.1), (1, 3e-6)])
def test_shadow_fixed_lnf_bitexact(precision, lnf):
    g, o = make_pair(12, 4, 4, 3, lnf_init=lnf, fixed_lnf=1, sync_attempts=1000, exchange=1,
                     precision=precision, seed=21, shadow=1)
    g.run(30_000)
    o.run(30_000)
    assert_same_state(g, o)
    assert_same_shadow(g, o)


@pytest.mark.parametrize("precision", [0, 1])
def test_shadow_full_protocol_L8_bitexact(precision):
    c = workloads.CONFIGS["potts_q10_L8"]
    g, o = make_pair(c["L"], c["q"], c["windows"], 2, seed=c["seed"], flat=c["flat"],
                     lnf_init=c["lnf_init"], lnf_final=1e-4, schedule=1, sync_attempts=20_000,
                     exchange=c["exchange"], precision=precision, shadow=1)
    assert g.run(10**10) == _pk().CONVERGED
    assert o.run(10**10) == oracle.CONVERGED
    assert_same_state(g, o)
    assert_same_shadow(g, o)


@pytest.mark.parametrize("slack", [0, 4, 16])
def test_walkin_lid_bitexact(slack):
    g, o = make_pair(20, 10, 6, 2, lnf_init=0.5, sync_attempts=2000, seed=17, walkin_slack=slack)
    g.run(6000)
    o.run(6000)
    assert_same_state(g, o)


def test_checkpoint_resume_bitexact():
    # save after a segment, restore into a fresh run of the same parameters,
    # continue both: identical to the oracle's uninterrupted run
    args = dict(lnf_init=1.0, lnf_final=1e-4, schedule=1, sync_attempts=1500, seed=12, shadow=1)
    g, o = make_pair(10, 6, 4, 2, **args)
    g.run(30_000)
    blob = g.save()
    spins = workloads.init_spins(10, 6, 8, 1)
    g2 = _pk().Rewl(10, 6, 4, 0.75, 2, spins, **args)
    g2.load(blob)
    assert g2.step == 30_000
    g2.run(25_000)
    o.run(55_000)
    assert_same_state(g2, o)
    assert_same_shadow(g2, o)
    bad = _pk().Rewl(10, 6, 4, 0.75, 2, spins, **dict(args, seed=13))
    with pytest.raises(_pk().RewlError):
        bad.load(blob)


def test_get_state_matches_the_oracle():
    # rewl_get_state: spins, E, H, ln g of a walker and its window's ln f in one call
    g, o = make_pair(8, 10, 4, 2, lnf_init=1.0, lnf_final=1e-3, sync_attempts=640, seed=5)
    g.run(640 * 40)
    o.run(640 * 40)
    for w in range(8):
        st, ow = g.state(w), o.walker(w)
        assert np.array_equal(st["spins"], ow["spins"]) and st["E"] == ow["E"]
        assert np.array_equal(st["H"], ow["H"])
        assert np.array_equal(st["lng"].view(np.uint64), ow["lng"].view(np.uint64))
        lnf = o.window(w // 2)["lnf"]
        assert np.float64(st["lnf"]).view(np.uint64) == np.float64(lnf).view(np.uint64)
    with pytest.raises(_pk().RewlError):
        g.state(8)
