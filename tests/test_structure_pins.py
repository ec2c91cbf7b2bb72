"""Pins of the structural observables of the lipid model (Sec. 3.2, Eqs. 6-8).

The oracle in oracle/structure.py is checked here against what the paper and
geometry fix: the limits the paper states for S_mol and the prolateness,
closed forms for collinear and evenly spaced beads, cluster partitions from a
brute-force search over all 27 periodic images handed to scipy's connected
components, invariance of every output under a periodic translation of the
whole box, and free-space contacts after unfolding."""
import numpy as np
import pytest

from oracle import structure as S


def lipid_rows(M, solvent=0):
    return np.arange(3 * M, dtype=np.int32).reshape(M, 3)


def place(beads):
    """beads: float[M][3][3] (head, centre, end) -> (x float32[3M][3], lip)."""
    beads = np.asarray(beads, dtype=np.float64)
    M = len(beads)
    return beads.reshape(3 * M, 3).astype(np.float32), lipid_rows(M)


def straight_lipid(origin, direction, spacing):
    o = np.asarray(origin, dtype=np.float64)
    e = np.asarray(direction, dtype=np.float64)
    e = e / np.linalg.norm(e)
    return np.stack([o, o + spacing * e, o + 2 * spacing * e])


# ---- Eq. 6 ---------------------------------------------------------------

def test_smol_aligned_bonds_reach_one():
    rng = np.random.default_rng(1)
    beads = [straight_lipid(rng.uniform(1, 9, 3), (0, 0, 1), 1.0) for _ in range(20)]
    x, lip = place(beads)
    s, axis = S.s_mol(x, lip, 30.0)
    assert axis == 2 and s == pytest.approx(1.0, abs=1e-12)


def test_smol_diagonal_bonds_give_a_quarter_on_the_first_axis():
    # cos^2 = 1/2 along x and y, 0 along z: S_x = S_y = 1/4, S_z = -1/2.
    beads = [straight_lipid((1.0 + 2 * k, 5.0, 5.0), (1, 1, 0), 1.0) for k in range(8)]
    x, lip = place(beads)
    s, axis = S.s_mol(x, lip, 30.0)
    assert axis == 0 and s == pytest.approx(0.25, abs=1e-6)


def test_smol_in_plane_ring_of_bonds():
    # Bonds at evenly spaced angles in the xy plane: <cos^2> = 1/2 on x and y.
    n = 36
    beads = [straight_lipid((15.0, 15.0, 15.0), (np.cos(2 * np.pi * k / n), np.sin(2 * np.pi * k / n), 0), 0.9)
             for k in range(n)]
    x, lip = place(beads)
    s, axis = S.s_mol(x, lip, 30.0)
    assert s == pytest.approx(0.25, abs=1e-6) and axis in (0, 1)


def test_smol_uses_the_minimum_image():
    # A head at the low face bonded across the boundary: the bond is (-0.7, 0.7, 0).
    box = 10.0
    x = np.array([[0.2, 0.2, 5.0], [box - 0.5, 0.9, 5.0], [box - 1.2, 1.6, 5.0]], dtype=np.float32)
    s, axis = S.s_mol(x, lipid_rows(1), box)
    assert s == pytest.approx(0.25, abs=1e-6)


def test_smol_isotropic_bonds_near_zero():
    # Uniform directions: P2(cos) has mean 0 and variance 1/5 per bond.
    rng = np.random.default_rng(7)
    M = 20000
    v = rng.normal(size=(M, 3))
    v /= np.linalg.norm(v, axis=1)[:, None]
    o = rng.uniform(2, 98, (M, 3))
    beads = np.stack([o, o + v, o + 2 * v], axis=1)
    x, lip = place(beads)
    s, _ = S.s_mol(x, lip, 100.0)
    assert abs(s) < 5 * np.sqrt(0.2 / M)
    assert s >= -0.5


# ---- clusters ------------------------------------------------------------

def brute_contacts(x, lip, box):
    """Tail contacts from explicit distances to all 27 periodic images (binary64)."""
    M = len(lip)
    shifts = np.array([[a, b, c] for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)], dtype=np.float64)
    tails = x.astype(np.float64)[lip[:, 1:]]  # [M][2][3]
    dmin = np.full((M, M), np.inf)
    for ta in range(2):
        for tb in range(2):
            diff = tails[None, :, tb, :] - tails[:, None, ta, :]
            for sh in shifts:
                d = np.sqrt(((diff + sh * box) ** 2).sum(axis=-1))
                dmin = np.minimum(dmin, d)
    np.fill_diagonal(dmin, np.inf)
    return dmin


def random_lipids(M, box, seed, bond=0.97):
    rng = np.random.default_rng(seed)
    o = rng.uniform(0, box, (M, 3))
    v = rng.normal(size=(M, 3))
    v /= np.linalg.norm(v, axis=1)[:, None]
    w = rng.normal(size=(M, 3))
    w /= np.linalg.norm(w, axis=1)[:, None]
    beads = np.stack([o, o + bond * v, o + bond * v + bond * w], axis=1) % box
    return place(beads)


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_clusters_match_connected_components(seed):
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import connected_components

    box, M = 8.0, 60
    x, lip = random_lipids(M, box, seed)
    dmin = brute_contacts(x, lip, box)
    finite = dmin[np.isfinite(dmin)]
    assert np.min(np.abs(finite - 1.4)) > 1e-4  # no pair sits on the threshold
    adj_ref = dmin < 1.4
    adj = S.contacts(x, lip, box)
    assert np.array_equal(adj, adj_ref)
    root, level, parent = S.clusters(adj)
    n, labels = connected_components(csr_matrix(adj_ref), directed=False)
    # same partition: lipids share a root exactly when scipy gives them one label
    assert np.array_equal(root[:, None] == root[None, :], labels[:, None] == labels[None, :])
    r, size, ncl = S.largest(root)
    counts = np.bincount(labels)
    assert ncl == n and size == counts.max()
    assert r == min(np.flatnonzero(labels == labels[i])[0] for i in range(M) if counts[labels[i]] == size)
    # tree: each non-root hangs from a touching lipid one level up
    for j in range(M):
        if root[j] == j:
            assert level[j] == 0 and parent[j] == -1
        else:
            assert adj_ref[parent[j], j] and level[parent[j]] == level[j] - 1 and root[parent[j]] == root[j]


def test_clusters_of_isolated_lipids():
    beads = [straight_lipid((3.0 * k + 1, 1.0, 1.0), (0, 1, 0), 1.0) for k in range(5)]
    x, lip = place(beads)
    rec = S.structure(x, lip, 40.0)
    assert rec[2] == 5 and rec[3] == 1


def test_tree_and_tie_rules_on_a_hand_built_example():
    # Lipids 0..3 are parallel rods along y; rods 1.2 apart touch, rods 1.70
    # or more apart do not, so that 0 - 1, 0 - 2, 1 - 3, 2 - 3 touch and
    # nothing else:
    # root 0; level 1 = {1, 2}; lipid 3 touches both and hangs from 1.
    # Lipids 4, 5 form a second two-lipid cluster far away, and lipids 6..9 a
    # second four-lipid cluster (same size as the first): the largest is the
    # one holding lipid 0.
    up = (0, 1, 0)
    beads = [straight_lipid((5.0, 5.0, 5.0), up, 1.0),     # 0
             straight_lipid((6.2, 5.0, 5.0), up, 1.0),     # 1: 1.2 from 0
             straight_lipid((5.0, 5.0, 6.2), up, 1.0),     # 2: 1.2 from 0
             straight_lipid((6.2, 5.0, 6.2), up, 1.0),     # 3: 1.2 from 1 and 2, 1.70 from 0
             straight_lipid((20.0, 5.0, 5.0), up, 1.0),    # 4
             straight_lipid((21.2, 5.0, 5.0), up, 1.0),    # 5
             straight_lipid((5.0, 20.0, 20.0), up, 1.0),   # 6
             straight_lipid((6.2, 20.0, 20.0), up, 1.0),   # 7
             straight_lipid((7.4, 20.0, 20.0), up, 1.0),   # 8
             straight_lipid((8.6, 20.0, 20.0), up, 1.0)]   # 9
    x, lip = place(beads)
    adj = S.contacts(x, lip, 40.0)
    root, level, parent = S.clusters(adj)
    assert list(root) == [0, 0, 0, 0, 4, 4, 6, 6, 6, 6]
    assert list(level) == [0, 1, 1, 2, 0, 1, 0, 1, 2, 3]
    assert list(parent) == [-1, 0, 0, 1, -1, 4, -1, 6, 7, 8]
    assert S.largest(root) == (0, 4, 3)
    u = S.unfold(x, lip, 40.0, adj, root, level, parent, 0)
    assert np.array_equal(u[0, 0], x[0].astype(np.float64))  # the root keeps its stored head


# ---- Eqs. 7-8 ------------------------------------------------------------

@pytest.mark.parametrize("q,p", [((1.0, 0.0, 0.0), 2.0), ((2.0, 2.0, 0.0), -0.25), ((3.0, 3.0, 3.0), 0.0)])
def test_prolateness_limits(q, p):
    assert S.prolateness(np.array(q)) == pytest.approx(p, abs=1e-15)


def rod(K, s, start, box):
    """K lipids on one line along x, beads every s, the line starting at `start`."""
    xs = (start + s * np.arange(3 * K)) % box
    beads = np.zeros((K, 3, 3))
    beads[:, :, 0] = xs.reshape(K, 3)
    beads[:, :, 1] = 5.0
    beads[:, :, 2] = 5.0
    return place(beads)


@pytest.mark.parametrize("start", [1.0, 25.0])
def test_rod_gyration_closed_form(start):
    # 3K equally spaced collinear beads: Q_xx = s^2 ((3K)^2 - 1) / 12, P = 2.
    K, s, box = 10, 0.6, 30.0
    x, lip = rod(K, s, start, box)
    rec = S.structure(x, lip, box)
    assert rec[2] == 1 and rec[3] == K
    assert rec[4] == pytest.approx(s * s * ((3 * K) ** 2 - 1) / 12, rel=1e-6)
    assert rec[5] == pytest.approx(0.0, abs=1e-10) and rec[6] == pytest.approx(0.0, abs=1e-10)
    assert rec[7] == pytest.approx(2.0, abs=1e-6)
    assert rec[0] == pytest.approx(1.0, abs=1e-9) and rec[1] == 0


def test_rod_wrapping_the_box_unfolds_to_the_same_line():
    # The rod closes on itself through the boundary (30 beads x 0.6 = box);
    # wherever the tree cuts the ring, the beads stay equally spaced.
    K, s = 10, 0.6
    box = 3 * K * s
    x, lip = rod(K, s, 0.0, box)
    adj = S.contacts(x, lip, box)
    assert adj[0, K - 1]  # the ends touch through the boundary
    rec = S.structure(x, lip, box)
    assert rec[3] == K
    assert rec[4] == pytest.approx(s * s * ((3 * K) ** 2 - 1) / 12, rel=1e-5)


def test_single_lipid():
    x, lip = place([straight_lipid((1.0, 2.0, 3.0), (0, 0, 1), 1.0)])
    rec = S.structure(x, lip, 10.0)
    assert list(rec[:4]) == [1.0, 2, 1, 1]
    assert rec[6] == pytest.approx(2.0 / 3.0, abs=1e-9) and rec[7] == pytest.approx(2.0, abs=1e-9)


def compact_cluster(M, centre, seed, box):
    """Lipids random-walked into one touching cluster around `centre`."""
    rng = np.random.default_rng(seed)
    beads = []
    c = np.asarray(centre, dtype=np.float64)
    while len(beads) < M:
        o = c + rng.uniform(-1.6, 1.6, 3)
        v = rng.normal(size=3)
        v /= np.linalg.norm(v)
        beads.append(np.stack([o, o + 0.95 * v, o + 1.9 * v]))
    return np.array(beads) % box


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_periodic_translation_leaves_every_output_unchanged(seed):
    box, M = 20.0, 12
    beads = compact_cluster(M, (10.0, 10.0, 10.0), seed, box)
    x, lip = place(beads)
    ref = S.structure(x, lip, box)
    # Move the whole box so the cluster straddles every face.
    shifted = (beads + np.array([9.3, 10.1, 9.7])) % box
    x2, _ = place(shifted)
    dmin = brute_contacts(x, lip, box)
    assert np.min(np.abs(dmin[np.isfinite(dmin)] - 1.4)) > 1e-4
    got = S.structure(x2, lip, box)
    assert np.array_equal(got[[1, 2, 3]], ref[[1, 2, 3]])
    assert np.allclose(got, ref, rtol=1e-5, atol=1e-5)


@pytest.mark.parametrize("seed", [0, 1])
def test_unfolded_cluster_realises_every_contact_in_free_space(seed):
    box, M = 20.0, 12
    beads = (compact_cluster(M, (10.0, 10.0, 10.0), seed, box) + np.array([9.5, 9.5, 9.5])) % box
    x, lip = place(beads)
    adj = S.contacts(x, lip, box)
    root, level, parent = S.clusters(adj)
    r, size, _ = S.largest(root)
    u = S.unfold(x, lip, box, adj, root, level, parent, r)
    members = np.flatnonzero(root == r)
    for i in members:
        assert np.linalg.norm(u[i, 1] - u[i, 0]) < 1.0 and np.linalg.norm(u[i, 2] - u[i, 1]) < 1.0
        for j in members:
            if adj[i, j]:
                d = min(np.linalg.norm(u[i, a] - u[j, b]) for a in (1, 2) for b in (1, 2))
                assert d < 1.4 + 1e-6


def test_binary32_contact_screen_never_contradicts_binary64():
    # The GPU kernel screens tail contacts with fl32((dx^2 + dy^2) + dz^2) of the
    # binary32 minimum-image differences: below 1.959997 it calls a contact,
    # above 1.960003 none, and leaves the band between to the binary64 test of
    # the definition.  The binary32 sum is within 3 ulp (1.8e-7 relative) of the
    # exact one, the band is 1.5e-6 wide on each side, so the screen can never
    # contradict the binary64 decision; checked here on 2 million differences,
    # most of them within a few ulp of the threshold.
    rng = np.random.default_rng(11)
    n = 2_000_000
    v = rng.normal(size=(n, 3))
    v /= np.linalg.norm(v, axis=1)[:, None]
    r = np.where(rng.random(n) < 0.8, 1.4 + rng.normal(scale=2e-6, size=n), rng.uniform(0.0, 3.0, n))
    d = (v * r[:, None]).astype(np.float32)
    r2f = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
    dd = d.astype(np.float64)
    r2d = (dd[:, 0] * dd[:, 0] + dd[:, 1] * dd[:, 1]) + dd[:, 2] * dd[:, 2]
    lo, hi = np.float32(1.959997), np.float32(1.960003)
    settled = (r2f < lo) | (r2f > hi)
    assert np.array_equal((r2f < lo)[settled], (r2d < S.TAIL_CONTACT2)[settled])
    assert np.max(np.abs(r2f - r2d) / np.maximum(r2d, 1e-30)) < 1.8e-7
    assert (~settled).sum() > 1000   # the band is exercised
