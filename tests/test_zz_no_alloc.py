"""rewl_structure_noalloc against rewl_structure: the entry point that stages
its records in a static device buffer instead of allocating gives the same
records, bit for bit, on two calls in a row (the second on a smaller run), and
refuses runs beyond its buffer."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _pk():
    import paper_1312_3004_amd as pk
    return pk


def lipid_run(nlip, nsol, box, e_min, bins, h, m, attempts, seed):
    x0 = workloads.init_lipids(nlip, nsol, box, h * m, seed)
    print(f"[case] noalloc structure: {nlip} lipids, {nsol} solvent, {h}x{m} walkers", flush=True)
    g = _pk().Rewl.lipid(nlip, nsol, box, e_min, 1.0, bins, h, 0.75, m, x0, lnf_init=1.0, sync_attempts=300,
                         seed=seed)
    if attempts:
        g.run(attempts)
    return g


def test_noalloc_structure_matches_allocating_entry_point():
    c = workloads.LIPID
    big = lipid_run(c["nlip"], c["nsol"], c["box"], c["e_min"], c["bins"], 4, 2, 900, 3)
    small = lipid_run(10, 40, 5.0, 300.0, 400, 2, 2, 600, 5)
    for g in (big, small):
        a = g.structure_noalloc()
        b = g.structure()
        assert a.shape == b.shape == (g.nw, 8)
        assert np.array_equal(a.view(np.uint64), b.view(np.uint64))
        assert np.all(a[:, 3] >= 1)
    # the smaller run's records did not pick up the larger run's rows, and
    # calling again (buffer keeps the previous contents) changes nothing
    a2 = big.structure_noalloc()
    assert np.array_equal(a2.view(np.uint64), big.structure().view(np.uint64))


def test_noalloc_structure_refuses_runs_beyond_its_buffer():
    pk = _pk()
    g = lipid_run(2, 4, 3.0, 0.0, 64, 17, 241, 0, 7)      # 4,097 walkers
    assert g.nw == 4097
    with pytest.raises(pk.RewlError):
        g.structure_noalloc()
    assert g.structure().shape == (4097, 8)
    small = lipid_run(10, 40, 5.0, 300.0, 400, 2, 2, 300, 5)
    assert np.array_equal(small.structure_noalloc().view(np.uint64), small.structure().view(np.uint64))
