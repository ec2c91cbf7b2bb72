"""Structural observables of the lipid model (test infrastructure).

Only tests/, the smoke check and the CPU-baseline leg of the benchmark may
import this module; the product library never loads it.  Plain numpy in
binary64 (distances from binary32 coordinates), written from Sec. 3.2,
Eqs. (6)-(8), with the readings below where the paper leaves a choice open.

A configuration is x float32[np][3] (coordinates in a periodic cube of side
`box`) and lip int32[M][3] (particle indices of each lipid, polar head first,
then its two hydrophobic tail beads in chain order).

* Minimum image: b - a per axis in binary32, moved once by -+box when it lies
  beyond +-box/2, then widened to binary64 (the same convention as the energy
  of the model).  Squared distances are (dx^2 + dy^2) + dz^2 in binary64.
* S_mol^head (Eq. 6): theta is the angle between a lipid's head-to-first-tail
  bond and a box axis; S_a = (3 <cos^2 theta_a> - 1) / 2 averaged over all
  lipids, reported for the axis a in (x, y, z) that maximises it (the first
  such axis on ties).
* Clusters: two lipids are neighbours when any tail bead of one lies within
  squared distance 1.96 (d < 1.4) of any tail bead of the other; clusters
  are the connected components of that graph (the partition Hoshen-Kopelman
  labelling finds).  The largest cluster is the one with most lipids, the one
  holding the lowest lipid index on ties.
* Unfolding: each cluster is grown breadth first from its lowest-index lipid;
  a lipid found at level k+1 hangs from the lowest-index lipid of level k it
  touches.  The root keeps its stored head position and its chain is made
  whole through its bonds; a child is placed through the first touching tail
  pair (parent centre or end bead, then child centre or end bead, in that
  order) at the parent's unfolded position plus the minimum image, and its
  other beads follow through its bonds.  For a cluster that does not wrap the
  box every contact is then realised in free space and the result does not
  depend on the tree; for one that wraps, this tree fixes the cut.
* Gyration tensor (Eq. 7, read with the square): Q_ii = (1/N) sum_j (r_j^i -
  r_com^i)^2 over the N = 3 x lipids beads of the unfolded largest cluster,
  all beads of equal mass.
* Prolateness (Eq. 8) from the diagonal elements: P = 9 sum_i (Q_ii -
  lambda)^3 / (sum_i Q_ii)^3 with lambda = (sum_i Q_ii) / 3.

structure() returns the record [S, axis, clusters, largest, Q11, Q22, Q33, P].
"""
import numpy as np

TAIL_CONTACT2 = 1.96  # (1.4 sigma)^2, the tail-tail neighbour criterion
RECORD = ("s_mol", "axis", "clusters", "largest", "q11", "q22", "q33", "prolateness")


def min_image(box, a, b):
    """Minimum-image difference b - a (binary32 per axis, wrapped once) as binary64."""
    a = np.asarray(a, dtype=np.float32)
    b = np.asarray(b, dtype=np.float32)
    box = np.float32(box)
    half = np.float32(0.5) * box
    d = b - a
    d = np.where(d > half, d - box, np.where(d < -half, d + box, d))
    return d.astype(np.float64)


def r2_of(d):
    return (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]


def s_mol(x, lip, box):
    """Eq. (6): bond order of the head-to-first-tail bonds, maximised over the box axes."""
    d = min_image(box, x[lip[:, 0]], x[lip[:, 1]])
    cos2 = d * d / r2_of(d)[:, None]
    s = 1.5 * cos2.mean(axis=0) - 0.5
    axis = int(np.argmax(s))
    return float(s[axis]), axis


def contacts(x, lip, box):
    """Neighbour matrix of the lipids: any tail-tail pair closer than 1.4."""
    M = len(lip)
    adj = np.zeros((M, M), dtype=bool)
    for a in (1, 2):
        for b in (1, 2):
            d = min_image(box, x[lip[:, a]][:, None, :], x[lip[:, b]][None, :, :])
            adj |= r2_of(d) < TAIL_CONTACT2
    np.fill_diagonal(adj, False)
    return adj


def clusters(adj):
    """Connected components grown breadth first: (root, level, parent) per lipid."""
    M = len(adj)
    root = np.full(M, -1)
    level = np.full(M, -1)
    parent = np.full(M, -1)
    for r in range(M):
        if root[r] >= 0:
            continue
        root[r], level[r] = r, 0
        frontier, k = [r], 0
        while frontier:
            found = []
            for j in range(M):
                if root[j] >= 0:
                    continue
                touching = [i for i in frontier if adj[i, j]]
                if touching:
                    root[j], level[j], parent[j] = r, k + 1, min(touching)
                    found.append(j)
            frontier, k = found, k + 1
    return root, level, parent


def largest(root):
    """Root of the cluster with most lipids (lowest root on ties) and its size."""
    roots, sizes = np.unique(root, return_counts=True)
    best = int(np.argmax(sizes))  # np.unique sorts the roots, argmax takes the first maximum
    return int(roots[best]), int(sizes[best]), len(roots)


def unfold(x, lip, box, adj, root, level, parent, r):
    """Unfolded bead positions float64[M][3][3] of cluster r (NaN for other lipids)."""
    M = len(lip)
    u = np.full((M, 3, 3), np.nan)

    def chain_from(j, b):
        # Make lipid j whole through its bonds, starting from bead b already placed.
        h, c, t = lip[j]
        if b == 1:
            u[j, 0] = u[j, 1] + min_image(box, x[c], x[h])
            u[j, 2] = u[j, 1] + min_image(box, x[c], x[t])
        elif b == 2:
            u[j, 1] = u[j, 2] + min_image(box, x[t], x[c])
            u[j, 0] = u[j, 1] + min_image(box, x[c], x[h])
        else:
            u[j, 1] = u[j, 0] + min_image(box, x[h], x[c])
            u[j, 2] = u[j, 1] + min_image(box, x[c], x[t])

    u[r, 0] = x[lip[r, 0]].astype(np.float64)
    chain_from(r, 0)
    for k in range(1, int(level[root == r].max()) + 1):
        for j in np.flatnonzero((root == r) & (level == k)):
            i = parent[j]
            for a, b in ((1, 1), (1, 2), (2, 1), (2, 2)):
                d = min_image(box, x[lip[i, a]], x[lip[j, b]])
                if r2_of(d) < TAIL_CONTACT2:
                    u[j, b] = u[i, a] + d
                    chain_from(j, b)
                    break
            else:
                raise AssertionError("tree edge without a touching tail pair")
    return u


def gyration(pos):
    """Eq. (7): diagonal of the gyration tensor of the points pos[n][3]."""
    com = pos.mean(axis=0)
    return ((pos - com) ** 2).mean(axis=0)


def prolateness(q):
    """Eq. (8) from the diagonal elements q[3]."""
    tr = q.sum()
    lam = tr / 3.0
    return 9.0 * ((q - lam) ** 3).sum() / tr ** 3


def structure(x, lip, box):
    """The record [S, axis, clusters, largest, Q11, Q22, Q33, P] of one configuration."""
    x = np.asarray(x, dtype=np.float32).reshape(-1, 3)
    lip = np.asarray(lip, dtype=np.int64).reshape(-1, 3)
    s, axis = s_mol(x, lip, box)
    adj = contacts(x, lip, box)
    root, level, parent = clusters(adj)
    r, size, ncl = largest(root)
    u = unfold(x, lip, box, adj, root, level, parent, r)
    q = gyration(u[root == r].reshape(-1, 3))
    return np.array([s, axis, ncl, size, q[0], q[1], q[2], prolateness(q)])
