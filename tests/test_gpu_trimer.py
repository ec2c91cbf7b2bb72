"""GPU parity of the trimer model (continuous bead displacements): lattices of
bytes (the binary32 coordinates), energy bins, binary64 energies, H, ln g and
exchange decisions identical to the oracle, bit for bit."""
import sys

import numpy as np
import pytest

import oracle
import workloads
from statecmp import assert_same_state

pytestmark = pytest.mark.gpu


def _pk():
    import paper_1312_3004_amd as pk
    return pk


def make_pair(nmol, box, e_min, bin_w, bins, h, m, coords_seed=1, threads=8, **opts):
    x = workloads.init_trimers(nmol, box, h * m, coords_seed)
    print(f"[case] trimer nmol={nmol} box={box} bins={bins} h={h} m={m} opts={opts}", flush=True)
    sys.stdout.flush()
    g = _pk().Rewl.trimer(nmol, box, e_min, bin_w, bins, h, 0.75, m, x, **opts)
    o = oracle.Rewl.trimer(nmol, box, e_min, bin_w, bins, h, 0.75, m, x, threads=threads, **opts)
    return g, o


def assert_same_energies(g, o):
    for w in range(g.nw):
        a, b = g.energy_fx(w), o.energy_fx(w)   # fixed point, units of 2^-32
        assert a == b, (w, a, b)


CASES = [
    # (nmol, box, e_min, bins, h, m, attempts, precision)
    (1, 3.0, -10.0, 60, 1, 2, 3000, 0),
    (8, 5.0, -30.0, 160, 2, 2, 8000, 0),
    (22, 7.0, -40.0, 200, 3, 2, 5000, 0),
    (64, 10.0, -40.0, 160, 4, 2, 4000, 0),
    (8, 5.0, -30.0, 160, 2, 2, 8000, 1),
]


@pytest.mark.parametrize("nmol,box,e_min,bins,h,m,attempts,precision", CASES)
def test_trimer_fixed_lnf_bitexact(nmol, box, e_min, bins, h, m, attempts, precision):
    g, o = make_pair(nmol, box, e_min, 0.5, bins, h, m, lnf_init=0.05, fixed_lnf=1, sync_attempts=997,
                     exchange=1, precision=precision, seed=4)
    g.run(attempts)
    o.run(attempts)
    assert_same_state(g, o)
    assert_same_energies(g, o)


def test_trimer_workload_shape_bitexact():
    # The trimer workload's shape: 64 trimers in the 10-wide box, 16 windows x
    # 4 walkers over its 1,000 bins from e_min = -460: walk-in from the
    # starting energies, then fixed-ln f sync intervals with exchange rounds.
    t = workloads.TRIMER
    g, o = make_pair(t["nmol"], t["box"], t["e_min"], t["bin_w"], t["bins"], t["windows"], t["walkers"],
                     coords_seed=t["seed"], lnf_init=0.01, fixed_lnf=1, sync_attempts=1000, exchange=1,
                     seed=t["seed"], threads=16)
    g.run(2500)
    o.run(2500)
    assert_same_state(g, o)
    assert_same_energies(g, o)
    assert max(g.walker(w)["walkin_attempts"] for w in range(g.nw)) > 0


def test_trimer_start_with_hard_overlap_is_refused():
    # two heads 0.3 apart: a WCA term above 2^18, a hard overlap
    c = np.array([[1.0, 5.0, 5.0], [2.0, 5.0, 5.0], [3.0, 5.0, 5.0],
                  [1.0, 5.0, 5.3], [2.0, 5.0, 6.3], [3.0, 5.0, 7.3]], dtype=np.float32)
    print("[case] trimer start with a hard overlap", flush=True)
    with pytest.raises(_pk().RewlError):
        _pk().Rewl.trimer(2, 10.0, -50.0, 0.5, 400, 1, 0.75, 1, c[None])
    with pytest.raises(ValueError):
        oracle.Rewl.trimer(2, 10.0, -50.0, 0.5, 400, 1, 0.75, 1, c[None])


def test_trimer_full_protocol_bitexact_and_join():
    g, o = make_pair(2, 4.0, -6.0, 0.5, 24, 2, 2, coords_seed=8, lnf_init=1.0, lnf_final=1e-3,
                     sync_attempts=2000, seed=1)
    assert g.run(10**9) == _pk().CONVERGED
    assert o.run(10**9) == oracle.CONVERGED
    assert_same_state(g, o)
    assert_same_energies(g, o)
    sg, lg, cg = g.join()
    so, lo, co = o.join()
    assert sg == so == 0 and np.array_equal(cg, co)
    fin = np.isfinite(lo)
    assert np.array_equal(np.isfinite(lg), fin)
    assert np.max(np.abs(lg[fin] - lo[fin])) <= 1e-10
    T = np.linspace(0.3, 3.0, 28)
    zg, ug, cvg = g.thermo(T)
    zo, uo, cvo = oracle.thermo(lo, -6.0 + 0.25, T, de=0.5)
    np.testing.assert_allclose(zg, zo, rtol=1e-12, atol=1e-9)
    np.testing.assert_allclose(ug, uo, rtol=1e-9, atol=1e-8)
    np.testing.assert_allclose(cvg, cvo, rtol=1e-8, atol=1e-8)


def test_trimer_walkin_from_above_bitexact():
    # windows well below the starting energies: every walker walks in first
    g, o = make_pair(8, 5.0, -30.0, 0.5, 50, 2, 2, coords_seed=3, lnf_init=0.1, fixed_lnf=1,
                     sync_attempts=1000, seed=9)
    g.run(2000)
    o.run(2000)
    assert_same_state(g, o)
    assert_same_energies(g, o)
    assert max(g.walker(w)["walkin_attempts"] for w in range(4)) > 0


def test_trimer_many_molecules_bitexact():
    # 400 molecules (1,200 beads, 19 chunks of 64 partners): one role per wave,
    # 16 waves taking several chunks each
    g, o = make_pair(400, 20.0, -30.0, 0.5, 200, 1, 2, lnf_init=0.05, fixed_lnf=1, sync_attempts=400,
                     seed=6, threads=8)
    g.run(800)
    o.run(800)
    assert_same_state(g, o)
    assert_same_energies(g, o)
