"""Energies the lipid workload passes through as it relaxes (test infrastructure).

The lipid workload starts from lattice configurations with stretched bonds
(energies 7,230-7,620), far above the energies of a relaxed fluid.  This
script anneals one such start on the oracle's own walk with fixed weights:
ln g(bin) = E_bin / T with ln f = 0 makes the Wang-Landau acceptance
min[1, g(E)/g(E')] the Metropolis rule exp(-(E' - E)/T) on binned energies.
T falls over `temps`, `moves` particle moves (displacements and reptations)
at each, on unit bins over [-4000, 8000).  It prints the mean energy of the
second half of each stage: the band a lower benchmark window can sit in.
Only the oracle is called.

    python -m oracle.lipid_range      # about two minutes on one core
"""
import numpy as np

import oracle
import workloads

TEMPS = (5.0, 4.0, 3.0, 2.5, 2.0, 1.7, 1.5, 1.3, 1.1, 1.0, 0.9, 0.8, 0.7, 0.6, 0.5)


def anneal(cfg=workloads.LIPID, temps=TEMPS, moves=200_000, seed=1):
    """[(T, mean energy over the second half of the stage, lowest energy so far)]."""
    x = workloads.init_lipids(cfg["nlip"], cfg["nsol"], cfg["box"], 1, cfg["seed"])
    e_lo, bw, bins = -4000.0, 1.0, 12000
    o = oracle.Rewl.lipid(cfg["nlip"], cfg["nsol"], cfg["box"], e_lo, bw, bins, 1, 0.0, 1, x,
                          eps_ww=cfg["eps_ww"], seed=seed, lnf_init=0.0, fixed_lnf=1, sync_attempts=10**9,
                          exchange=0)
    centres = e_lo + (np.arange(bins) + 0.5) * bw
    out, lowest = [], o.energy(0)
    for T in temps:
        o.set_lng(0, centres / T)
        es = []
        for _ in range(10):
            o.run(moves // 10)
            es.append(o.energy(0))
            lowest = min(lowest, es[-1])
        out.append((T, float(np.mean(es[5:])), lowest))
    return out


if __name__ == "__main__":
    for T, mean, lowest in anneal():
        print(f"T = {T:4.2f}: mean energy {mean:9.1f}, lowest so far {lowest:9.1f}")
