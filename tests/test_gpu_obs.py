"""GPU parity of production sampling and observable histograms (Sec. 3.2):
H(E, O) of O = max_s n_s sampled at sync points, the production phase with
frozen weights, pooled microcanonical means and canonical averages, against
the oracle on the same seeded inputs."""
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


def make_pair(L, q, h, m, spins_seed=1, **opts):
    spins = workloads.init_spins(L, q, h * m, spins_seed)
    print(f"[case] L={L} q={q} h={h} m={m} opts={opts}", flush=True)
    sys.stdout.flush()
    g = _pk().Rewl(L, q, h, 0.75, m, spins, **opts)
    o = oracle.Rewl(L, q, h, 0.75, m, spins, threads=8, **opts)
    return g, o


@pytest.mark.parametrize("L,q,h,m,nb,precision", [(8, 10, 4, 2, 65, 0), (8, 10, 4, 2, 13, 1),
                                                  (12, 3, 5, 3, 7, 0), (5, 2, 1, 4, 1, 0)])
def test_obs_sampling_bitexact(L, q, h, m, nb, precision):
    g, o = make_pair(L, q, h, m, lnf_init=0.05, fixed_lnf=1, sync_attempts=333, exchange=1, seed=4,
                     obs_bins=nb, precision=precision)
    g.run(333 * 40)
    o.run(333 * 40)
    assert_same_state(g, o)
    gm, gc = g.obs_micro()
    om, oc = o.obs_micro()
    assert np.array_equal(gc, oc) and gc.sum() == 40 * h * m
    assert np.array_equal(np.isnan(gm), np.isnan(om))
    assert np.array_equal(gm[~np.isnan(gm)], om[~np.isnan(om)])


def test_production_after_convergence_bitexact():
    L, q, h, m = 4, 2, 2, 2
    g, o = make_pair(L, q, h, m, lnf_final=1e-4, schedule=1, sync_attempts=800, seed=6, obs_bins=17,
                     spins_seed=3)
    with pytest.raises(_pk().RewlError):
        g.begin_production()                      # before the walk-in
    assert g.run(10**9) == _pk().CONVERGED
    assert o.run(10**12) == oracle.CONVERGED
    assert_same_state(g, o)
    g.begin_production()
    assert o.begin_production() == 0
    assert_same_state(g, o)
    assert g.run(800 * 300) == _pk().OK
    o.run(800 * 300)
    assert_same_state(g, o)
    assert all(g.window(k)["lnf"] == 0.0 for k in range(h))
    sg, lg, _ = g.join()
    so, lo, _ = o.join()
    assert sg == so == 0
    T = np.array([0.3, 0.8, 1.2, 2.5, 20.0])
    got = g.obs_thermo(T)
    ref = oracle.obs_thermo(lo, o.obs_micro()[0], o.e_lo, T)
    # joined ln g agree to 1e-10 (normalisation order), so the weights to a
    # relative 1e-10; both sums run over at most 33 positive terms
    np.testing.assert_allclose(got, ref, rtol=1e-9)


def test_batch_instances_sample_obs_like_the_oracle():
    cases = [(6, 3, 3, 2, 360, dict(lnf_init=1.0, lnf_final=1e-3, obs_bins=37)),
             (8, 10, 4, 2, 640, dict(lnf_init=0.5, lnf_final=1e-6)),
             (5, 2, 2, 3, 250, dict(lnf_init=1.0, lnf_final=5e-3, schedule=1, obs_bins=4))]
    insts, spins = [], []
    for i, (L, q, h, m, S, extra) in enumerate(cases):
        d = dict(L=L, q=q, windows=h, overlap=0.75, walkers=m, seed=7, instance=i, sync_attempts=S)
        d.update(extra)
        insts.append(d)
        spins.append(workloads.init_spins(L, q, h * m, 100 + i))
    print("[case] batch with observable sampling", flush=True)
    b = _pk().Batch(insts, spins)
    b.run(6)
    c = _pk().Batch(insts, spins)
    c.run_per_instance(6)
    for i, d in enumerate(insts):
        d = dict(d)
        geo = [d.pop(k) for k in ("L", "q", "windows", "overlap", "walkers")]
        o = oracle.Rewl(*geo, spins[i], threads=8, **d)
        o.run(6 * d["sync_attempts"])
        assert_same_state(b.instance(i), o)
        assert_same_state(c.instance(i), o)
    with pytest.raises(_pk().RewlError):
        b.instance(0).begin_production()          # production runs are standalone


def test_obs_argument_errors():
    pk = _pk()
    spins = workloads.init_spins(4, 2, 2, 1)
    with pytest.raises(pk.RewlError):
        pk.Rewl(4, 2, 1, 0.75, 2, spins, obs_bins=18)      # more than N + 1 bins
    g = pk.Rewl(4, 2, 1, 0.75, 2, spins)
    with pytest.raises(pk.RewlError):
        g.obs(0)
    with pytest.raises(pk.RewlError):
        g.obs_micro()
    g = pk.Rewl(4, 2, 1, 0.75, 2, spins, obs_bins=17, lnf_final=1e-2, sync_attempts=500)
    g.run(100)
    with pytest.raises(pk.RewlError):
        g.obs_thermo([1.0])                                # no current join
    with pytest.raises(pk.RewlError):
        g.obs(2)
