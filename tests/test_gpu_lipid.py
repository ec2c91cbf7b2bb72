"""GPU parity of the lipid model with explicit solvent (Sec. 3.2, Eqs. 3-5,
Fig. 5): coordinates, particle types and lipid rows, energy bins, binary64
energies, H, ln g and exchange decisions identical to the oracle, bit for
bit, under displacement and reptation moves."""
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


def make_pair(nlip, nsol, box, e_min, bin_w, bins, h, m, coords_seed=1, threads=8, **opts):
    x = workloads.init_lipids(nlip, nsol, box, h * m, coords_seed)
    print(f"[case] lipid nlip={nlip} nsol={nsol} box={box:.3f} bins={bins} h={h} m={m} opts={opts}", flush=True)
    sys.stdout.flush()
    g = _pk().Rewl.lipid(nlip, nsol, box, e_min, bin_w, bins, h, 0.75, m, x, **opts)
    o = oracle.Rewl.lipid(nlip, nsol, box, e_min, bin_w, bins, h, 0.75, m, x, threads=threads, **opts)
    return g, o


def assert_same_lipids(g, o):
    for w in range(g.nw):
        a, b = g.energy_fx(w), o.energy_fx(w)   # fixed point, units of 2^-32
        assert a == b, (w, a, b)
        for u, v, name in zip(g.lipid_state(w), o.lipid_state(w), ("coords", "types", "lipids")):
            assert np.array_equal(u, v), f"{name} of walker {w}"


CASES = [
    # (nlip, nsol, box, e_min, bins, h, m, attempts, rep_prob)
    (4, 20, 4.3, 200.0, 160, 2, 2, 3000, 0.3),
    (6, 60, 5.0, 300.0, 320, 3, 2, 2000, None),
    (6, 60, 5.0, 300.0, 320, 2, 3, 2000, 0.9),
]


@pytest.mark.parametrize("nlip,nsol,box,e_min,bins,h,m,attempts,rep_prob", CASES)
def test_lipid_fixed_lnf_bitexact(nlip, nsol, box, e_min, bins, h, m, attempts, rep_prob):
    g, o = make_pair(nlip, nsol, box, e_min, 0.5, bins, h, m, rep_prob=rep_prob, lnf_init=0.05, fixed_lnf=1,
                     sync_attempts=499, exchange=1, seed=4)
    g.run(attempts)
    o.run(attempts)
    assert_same_state(g, o)
    assert_same_lipids(g, o)
    # reptations did happen: some lipid row changed
    moved = any(not np.array_equal(o.lipid_state(w)[2], np.arange(3 * nlip).reshape(nlip, 3)) for w in range(g.nw))
    assert moved


def test_lipid_protocol_segment_bitexact():
    g, o = make_pair(4, 20, 4.3, 200.0, 0.5, 160, 2, 2, coords_seed=3, rep_prob=0.2, lnf_init=1.0,
                     lnf_final=1e-3, sync_attempts=800, seed=2)
    g.run(12_000)
    o.run(12_000)
    assert_same_state(g, o)
    assert_same_lipids(g, o)


def test_lipid_paper_size_segment_bitexact():
    # the paper's system: 125 lipids in 625 solvent particles at density 0.8
    c = workloads.LIPID
    g, o = make_pair(c["nlip"], c["nsol"], c["box"], c["e_min"], c["bin_w"], c["bins"], 4, 2, lnf_init=1.0,
                     sync_attempts=400, seed=c["seed"])
    g.run(1200)
    o.run(1200)
    assert_same_state(g, o)
    assert_same_lipids(g, o)


def test_lipid_argument_errors():
    pk = _pk()
    x = workloads.init_lipids(2, 10, 4.0, 1, 1)
    with pytest.raises(pk.RewlError):
        pk.Rewl.lipid(2, 10, 4.0, 0.0, 0.5, 100, 1, 0.75, 1, x, precision=1)
    with pytest.raises(pk.RewlError):
        pk.Rewl.lipid(2, 10, 4.0, 0.0, 0.5, 100, 1, 0.75, 1, x, rep_prob=1.5)
    bad = x.copy()
    bad[0, 0, 0] = 4.0
    with pytest.raises(pk.RewlError):
        pk.Rewl.lipid(2, 10, 4.0, 0.0, 0.5, 100, 1, 0.75, 1, bad)
