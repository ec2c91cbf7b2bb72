"""Seeded synthetic inputs shared by the GPU library's tests/benchmark and the
CPU oracle.

This module holds no arithmetic of the method: only the named problem
configurations and the starting lattices (uniform random spins drawn with
numpy's PCG64 from a seed).  Everything the method itself draws during a run
comes from the Philox4x32-10 stream that each side implements on its own.
"""
import numpy as np

# Named workloads.  sync_attempts = attempts per walker between sync points.
CONFIGS = {
    # 2D q=10 Potts, 8x8, h=4 at 75% overlap, m=1, flat 0.8, ln f 1 -> 1e-6 by
    # halving, exchange every 1000 sweeps (64,000 attempts), binary64 ln g.
    "potts_q10_L8": dict(model="potts", L=8, q=10, windows=4, overlap=0.75, walkers=1,
                         flat=(4, 5), lnf_init=1.0, lnf_final=1e-6, schedule=0,
                         sync_attempts=1000 * 64, exchange=1, precision=0, seed=1),
    # 2D q=10 Potts, 32x32, h=16 at 75% overlap, m=4, flat 0.8, ln f 1 -> 1e-8
    # (halving, then 1/t), exchange every 10^4 attempts per walker, binary64.
    "potts_q10_L32": dict(model="potts", L=32, q=10, windows=16, overlap=0.75, walkers=4,
                          flat=(4, 5), lnf_init=1.0, lnf_final=1e-8, schedule=1,
                          sync_attempts=10_000, exchange=1, precision=0, seed=1),
    # 2D q=10 Potts, 80x80, h=64 at 75% overlap, m=16, ln f 1 -> 1e-9 by halving;
    # run in binary64 and in the binary32 (hi, lo) form.
    "potts_q10_L80": dict(model="potts", L=80, q=10, windows=64, overlap=0.75, walkers=16,
                          flat=(4, 5), lnf_init=1.0, lnf_final=1e-9, schedule=0,
                          sync_attempts=10_000, exchange=1, precision=0, seed=1),
}

# Batched workload: 256 independent instances, L from {16,24,32,48} and q from
# {2,4,8,10} drawn per instance, h=8 at 75% overlap, m=4, binary64, the
# schedule of the L=8 workload (halving to 1e-6, flat 0.8, sync every 1000 sweeps).
BATCHED = dict(instances=256, L_choices=(16, 24, 32, 48), q_choices=(2, 4, 8, 10), windows=8,
               overlap=0.75, walkers=4, flat=(4, 5), lnf_init=1.0, lnf_final=1e-6, schedule=0,
               sweeps_per_sync=1000, exchange=1, precision=0, seed=1)


# Amphiphile trimers (head-tail-tail): 64 molecules in a periodic cube of side
# 10, harmonic bonds, tail-tail LJ cut at 2.5, WCA for pairs with a head,
# +-0.1 bead displacements, energy bins of 0.5 over [e_min, e_min + 0.5 bins),
# 16 windows at 75% overlap, 4 walkers each, binary64 ln g.  The energy range
# lies below the lowest energy a seeded Metropolis anneal of a start reaches
# (-457.4) and above the energies of all starting configurations (-52.4 ..
# 30.2); the test suite checks both with the oracle.
TRIMER = dict(model="trimer", nmol=64, box=10.0, e_min=-460.0, bin_w=0.5, bins=1000, windows=16,
              overlap=0.75, walkers=4, flat=(4, 5), lnf_init=1.0, lnf_final=1e-6, schedule=0,
              sync_attempts=20_000, exchange=1, precision=0, seed=1)


# Lipid model with explicit solvent (the paper's system size): 125 P-H-H
# lipids and 625 solvent particles (N = 1000) at number density 0.8 (box
# (1000/0.8)^(1/3)), eps_WW = 1, reptation probability 3M/(10N) = 0.0375,
# 16 windows at 75% overlap with 4 walkers each over 800 one-unit energy bins
# from 7000 (the band just below the lattice starts of init_lipids, 7230 ..
# 7620), binary64 ln g, ln f 1 -> 1e-6 by halving, sync every 2000 attempts.
LIPID = dict(model="lipid", nlip=125, nsol=625, box=(1000 / 0.8) ** (1 / 3), eps_ww=1.0, e_min=7000.0, bin_w=1.0,
             bins=800, windows=16, overlap=0.75, walkers=4, flat=(4, 5), lnf_init=1.0, lnf_final=1e-6, schedule=0,
             sync_attempts=2000, exchange=1, precision=0, seed=1)


def init_lipids(nlip, nsol, box, n_walkers, seed, jitter=0.05):
    """Starting configurations of the lipid model: float32 [n_walkers, np, 3].

    Particles sit on a simple cubic lattice of n = ceil(np^(1/3)) sites per
    side (spacing a = box / n).  Lipid i (particles 3i head, 3i+1, 3i+2 tails)
    takes three consecutive sites of one x-row, in a row slot and orientation
    drawn at random; solvent particles take random free sites; every
    coordinate then moves by a uniform jitter of +-jitter * a.
    """
    np_ = 3 * nlip + nsol
    n = 1
    while n ** 3 < np_:
        n += 1
    a = box / n
    if nlip > n * n * (n // 3):
        raise ValueError("too many lipids for the lattice rows")
    rng = np.random.Generator(np.random.PCG64(seed))
    out = np.zeros((n_walkers, np_, 3), dtype=np.float32)
    for w in range(n_walkers):
        slots = [(row, k) for row in range(n * n) for k in range(n // 3)]
        pick = rng.permutation(len(slots))[:nlip]
        used = set()
        sites = []
        for i in pick:
            row, k = slots[i]
            run = [(row, 3 * k + t) for t in range(3)]
            if rng.integers(2):
                run = run[::-1]
            used.update(run)
            sites.extend(run)
        free = [(row, x) for row in range(n * n) for x in range(n) if (row, x) not in used]
        for i in rng.permutation(len(free))[:nsol]:
            sites.append(free[i])
        pos = np.array([[x, row % n, row // n] for row, x in sites], dtype=np.float64) * a
        pos += rng.uniform(-jitter * a, jitter * a, size=pos.shape)
        pos = np.mod(pos, box).astype(np.float32)
        pos[pos >= np.float32(box)] = np.float32(0.0)
        out[w] = pos
    return out


def init_trimers(nmol, box, n_walkers, seed, min_dist=0.9):
    """Starting configurations: float32 [n_walkers, 3 nmol, 3] in [0, box).

    Per molecule, the head is uniform in the box and each tail sits at unit
    distance from the previous bead along a uniform random direction; a
    molecule is redrawn while any of its beads comes closer than min_dist to
    a bead already placed (minimum image), so the start has no overlaps.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    out = np.zeros((n_walkers, 3 * nmol, 3), dtype=np.float32)
    for w in range(n_walkers):
        placed = np.zeros((0, 3))
        for i in range(nmol):
            for _ in range(100000):
                beads = [rng.uniform(0.0, box, 3)]
                for _t in range(2):
                    v = rng.normal(size=3)
                    beads.append(beads[-1] + v / np.linalg.norm(v))
                beads = np.mod(np.array(beads), box)
                ok = True
                allb = np.concatenate([placed, beads[:0]])
                for b in beads:
                    if len(allb):
                        d = np.abs(allb - b)
                        d = np.minimum(d, box - d)
                        if np.min(np.sum(d * d, axis=1)) < min_dist * min_dist:
                            ok = False
                            break
                    allb = np.concatenate([allb, b[None]])
                if ok:
                    placed = np.concatenate([placed, beads])
                    break
            else:
                raise RuntimeError("could not place a molecule")
        x = placed.astype(np.float32)
        x[x >= np.float32(box)] = np.float32(0.0)
        out[w] = x
    return out


def init_spins(L, q, n_walkers, seed):
    """One uniformly random L x L lattice per walker, values in [0, q), int8."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(0, q, size=(n_walkers, L * L), dtype=np.int8)


def batched_instances(cfg=BATCHED):
    """(L, q) of every instance of the batched workload, drawn from its seed."""
    rng = np.random.Generator(np.random.PCG64(cfg["seed"]))
    Ls = rng.choice(np.array(cfg["L_choices"]), size=cfg["instances"])
    qs = rng.choice(np.array(cfg["q_choices"]), size=cfg["instances"])
    return [(int(a), int(b)) for a, b in zip(Ls, qs)]
