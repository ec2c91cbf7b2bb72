"""GPU parity of the bootstrap error analysis (Sec. 2): R independent runs of
one system as the instances of a batch, run to convergence, resampled and
joined anew per resample on the GPU, against the oracle's bootstrap of the
same runs (each run bit-identical to the oracle's run of that instance)."""
import math
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


def runs_of(L, q, h, m, R, lnf_final, S):
    insts, spins = [], []
    for i in range(R):
        insts.append(dict(L=L, q=q, windows=h, overlap=0.75, walkers=m, seed=77, instance=i,
                          lnf_final=lnf_final, sync_attempts=S))
        spins.append(workloads.init_spins(L, q, h * m, 1000 + i))
    print(f"[case] bootstrap over {R} runs of L={L} q={q} h={h} m={m}", flush=True)
    sys.stdout.flush()
    return insts, spins


def oracle_runs(insts, spins):
    out = []
    for d, sp in zip(insts, spins):
        d = dict(d)
        geo = [d.pop(k) for k in ("L", "q", "windows", "overlap", "walkers")]
        o = oracle.Rewl(*geo, sp, threads=8, **d)
        assert o.run(10**12) == oracle.CONVERGED
        out.append(o)
    return out


@pytest.mark.parametrize("L,q,h,m,R,lnf_final,S", [(4, 2, 2, 2, 12, 1e-3, 500), (8, 10, 4, 1, 6, 1e-3, 2000)])
def test_bootstrap_matches_oracle(L, q, h, m, R, lnf_final, S):
    insts, spins = runs_of(L, q, h, m, R, lnf_final, S)
    b = _pk().Batch(insts, spins)
    assert b.run(10**6) == _pk().CONVERGED
    os_ = oracle_runs(insts, spins)
    for i, o in enumerate(os_):
        assert_same_state(b.instance(i), o)
    T = np.array([0.4, 0.7, 1.0, 1.5, 3.0])
    g = b.bootstrap(300, 5, T)
    pv = [oracle.run_pieces(o) for o in os_]
    o = os_[0]
    st, ref = oracle.bootstrap(np.stack([p for p, _ in pv]), np.stack([v for _, v in pv]), o.starts, o.e_lo, o.B,
                               L * L * math.log(q), 300, 5, T)
    assert st == 0
    fin = np.isfinite(ref["lng_mean"])
    assert np.array_equal(np.isfinite(g["lng_mean"]), fin)
    # the two sides differ only in the order of the normalising log-sum-exp
    np.testing.assert_allclose(g["lng_mean"][fin], ref["lng_mean"][fin], rtol=0, atol=1e-9)
    np.testing.assert_allclose(g["lng_std"], ref["lng_std"], rtol=0, atol=1e-9)
    for k in ("U_mean", "U_std", "C_mean", "C_std"):
        np.testing.assert_allclose(g[k], ref[k], rtol=1e-9, atol=1e-12)
    assert g["lng_std"][fin].max() > 0


def test_bootstrap_argument_errors():
    pk = _pk()
    insts, spins = runs_of(4, 2, 2, 2, 3, 1e-2, 500)
    b = pk.Batch(insts, spins)
    with pytest.raises(pk.RewlError):
        b.bootstrap(10, 1, [1.0])                 # not converged yet
    b.run(10**6)
    with pytest.raises(pk.RewlError):
        b.bootstrap(0, 1, [1.0])
    with pytest.raises(pk.RewlError):
        b.bootstrap(10, 1, [-1.0])
    other = insts[:2] + [dict(insts[2], L=5)]
    c = pk.Batch(other, spins[:2] + [workloads.init_spins(5, 2, 4, 9)])
    c.run(10**6)
    with pytest.raises(pk.RewlError):
        c.bootstrap(10, 1, [1.0])                 # instances of different systems
    out = b.bootstrap(50, 2)
    assert np.isfinite(out["lng_mean"]).any()
