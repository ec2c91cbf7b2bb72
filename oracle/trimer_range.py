"""Energy range of the trimer workload from a seeded anneal (test infrastructure).

The trimer model has no exact ground state to take a range from, so the range
of its energy bins is checked against a pre-run: a Metropolis anneal of one
starting configuration of the workload finds a low energy, which the lower end
of the range must not exceed (moves below it are rejected like any move out
of a window, so the density of states is sampled over the range); the upper
end lies above every starting energy of the workload's walkers.

The anneal is the oracle's own walk with fixed weights: with ln g(bin) = beta
* E_bin and ln f = 0 the Wang-Landau acceptance min[1, g(E)/g(E')] is the
Metropolis rule exp(-beta (E' - E)) on binned energies.  beta rises
geometrically from 0.5 to 8 over `stages` stages of `moves` bead moves each,
on 0.5-wide bins over [-1000, 1000).  Only the oracle is called.

    python -m oracle.trimer_range      # prints the lowest energy and the range check
"""
import numpy as np

import oracle
import workloads


def anneal(nmol=64, box=10.0, seed=1, stages=40, moves=50_000, beta0=0.5, beta1=8.0):
    """Lowest energy reached by the anneal of walker 0's starting configuration."""
    x = workloads.init_trimers(nmol, box, 1, seed)
    e_lo, bw, bins = -1000.0, 0.5, 4000
    o = oracle.Rewl.trimer(nmol, box, e_lo, bw, bins, 1, 0.0, 1, x, seed=seed, lnf_init=0.0, fixed_lnf=1,
                           sync_attempts=10**9, exchange=0)
    centres = e_lo + (np.arange(bins) + 0.5) * bw
    lowest = o.energy(0)
    for beta in np.geomspace(beta0, beta1, stages):
        o.set_lng(0, beta * centres)
        for _ in range(10):
            o.run(moves // 10)
            lowest = min(lowest, o.energy(0))
    return lowest


def starting_energies(cfg=workloads.TRIMER):
    """Energies of the workload's starting configurations (one per walker)."""
    n = cfg["windows"] * cfg["walkers"]
    x = workloads.init_trimers(cfg["nmol"], cfg["box"], n, cfg["seed"])
    o = oracle.Rewl.trimer(cfg["nmol"], cfg["box"], cfg["e_min"], cfg["bin_w"], cfg["bins"], 1, 0.0, n, x,
                           seed=cfg["seed"])
    return np.array([o.energy(w) for w in range(n)])


def check(cfg=workloads.TRIMER, margin=0.0, **kw):
    """(lowest, starts, ok): the workload's range reaches at least `margin`
    below the anneal's lowest energy and above every starting energy."""
    lowest = anneal(cfg["nmol"], cfg["box"], cfg["seed"], **kw)
    starts = starting_energies(cfg)
    top = cfg["e_min"] + cfg["bins"] * cfg["bin_w"]
    ok = cfg["e_min"] <= lowest - margin and top > starts.max()
    return lowest, starts, ok


if __name__ == "__main__":
    lowest, starts, ok = check()
    c = workloads.TRIMER
    print(f"anneal lowest energy {lowest:.3f}; starting energies {starts.min():.3f} .. {starts.max():.3f}; "
          f"range [{c['e_min']}, {c['e_min'] + c['bins'] * c['bin_w']}): {'ok' if ok else 'NOT ok'}")
