"""Pins of the species-analysis oracle (oracle/species.py) on hand-made bond
graphs whose molecules are known by construction, and against an
independent components routine (scipy's connected_components) with a
minimum-ID relabelling on random graphs."""
import numpy as np
import pytest

from oracle import species as S


def test_hand_made_molecules():
    # atoms 0..7: CO (0-3), H2 (1-5), lone N (2), chain O-C-O (4-6-7), threshold rule
    types = np.array([0, 1, 2, 3, 3, 1, 0, 3])
    bonds = np.array([[0, 3], [1, 5], [4, 6], [6, 7], [2, 4]])
    bo = np.array([1.2, 0.9, 1.5, 1.4, 0.3])        # 0.3 is not "larger than" 0.3
    number, counts, table = S.analyse(8, types, bonds, bo, 0.3)
    # molecules by smallest index: {0,3}=1, {1,5}=2, {2}=3, {4,6,7}=4
    assert list(number) == [1, 2, 3, 1, 4, 2, 4, 4]
    assert counts.tolist() == [[1, 0, 0, 1], [0, 2, 0, 0], [0, 0, 1, 0], [1, 0, 0, 2]]
    assert table.tolist() == [[0, 0, 1, 0, 1], [0, 2, 0, 0, 1], [1, 0, 0, 1, 1], [1, 0, 0, 2, 1]]
    assert S.formula(table[3][:4]) == "C1O2"
    # just above the threshold the N joins the O-C-O chain
    number, counts, table = S.analyse(8, types, bonds, np.array([1.2, 0.9, 1.5, 1.4, 0.3000001]), 0.3)
    assert list(number) == [1, 2, 3, 1, 3, 2, 3, 3]
    assert table.tolist() == [[0, 2, 0, 0, 1], [1, 0, 0, 1, 1], [1, 0, 1, 2, 1]]


def test_isomers_and_repeats_share_a_species():
    # two water-like O-H-H molecules with different bonding (H-O-H vs O-H-H) and a third copy
    types = np.array([3, 1, 1, 3, 1, 1, 1, 3, 1])
    bonds = np.array([[0, 1], [0, 2], [3, 4], [4, 5], [6, 7], [7, 8]])
    number, counts, table = S.analyse(9, types, bonds, np.ones(6))
    assert number.max() == 3
    assert table.tolist() == [[0, 2, 0, 1, 3]]


def test_ring_and_both_directions():
    n = 6
    types = np.zeros(n, dtype=int)
    ring = np.array([[k, (k + 1) % n] for k in range(n)])
    both = np.concatenate([ring, ring[:, ::-1]])
    number, _, table = S.analyse(n, types, both, np.full(both.shape[0], 2.0))
    assert np.all(number == 1) and table.tolist() == [[6, 0, 0, 0, 1]]


def test_against_connected_components():
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components
    rng = np.random.default_rng(2)
    for trial in range(5):
        n = 300
        B = 250
        bonds = rng.integers(0, n, size=(B, 2))
        bo = rng.uniform(0, 1, size=B)
        types = rng.integers(0, 4, size=n)
        number, counts, table = S.analyse(n, types, bonds, bo, 0.3)
        keep = bo > 0.3
        g = coo_matrix((np.ones(keep.sum()), (bonds[keep, 0], bonds[keep, 1])), shape=(n, n))
        nc, lab = connected_components(g, directed=False)
        # minimum atom index per scipy component, ranked
        mins = np.full(nc, n)
        np.minimum.at(mins, lab, np.arange(n))
        order = np.argsort(mins)
        rank = np.empty(nc, dtype=int)
        rank[order] = np.arange(1, nc + 1)
        assert np.array_equal(number, rank[lab])
        assert counts.sum() == n and table[:, 4].sum() == nc
        assert np.array_equal(np.bincount(lab, minlength=nc)[order], counts.sum(1))


def test_empty_and_no_bonds():
    number, counts, table = S.analyse(0, np.zeros(0, int), np.zeros((0, 2), int), np.zeros(0))
    assert number.size == 0 and table.shape == (0, 5)
    number, counts, table = S.analyse(3, np.array([1, 1, 2]), np.zeros((0, 2), int), np.zeros(0))
    assert list(number) == [1, 2, 3]
    assert table.tolist() == [[0, 0, 1, 0, 1], [0, 1, 0, 0, 2]]
