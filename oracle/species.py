"""Molecular species analysis oracle -- test infrastructure only.

Only tests import this module; the GPU library never does.  Plain NumPy and
Python, following the steps of Section 3.4:

  1. two atoms are bonded when the (corrected) bond order between them is
     larger than the threshold (default 0.3); bonded atoms share a molecule,
     whose ID is the smallest global ID (here: the caller's atom index) among
     its atoms -- repeated until every atom has its molecule's ID, i.e. the
     ID is the minimum over the connected component of the bond graph;
  2. the molecule IDs are sorted and renumbered 1..M (M molecules);
  3. a molecule's species is its count of atoms of each element; molecules
     with equal counts are the same species (isomers are not told apart);
  4. the summary lists each distinct species with its number of molecules.

The components are found here by plain breadth-first search.
"""
from __future__ import annotations

from collections import deque

import numpy as np


def molecules(n, bonds, bo, threshold=0.3):
    """Molecule number (1..M, in increasing order of the molecules' smallest atom
    index) of every atom.  bonds: (B, 2) atom index pairs (either or both
    directions), bo: (B,) their bond orders."""
    adj = [[] for _ in range(n)]
    for (i, j), b in zip(np.asarray(bonds).reshape(-1, 2), np.asarray(bo)):
        if b > threshold:
            adj[int(i)].append(int(j))
            adj[int(j)].append(int(i))
    mol_id = np.full(n, -1, dtype=np.int64)      # smallest atom index of the molecule
    for start in range(n):                        # increasing index: start is its component's minimum
        if mol_id[start] >= 0:
            continue
        mol_id[start] = start
        queue = deque([start])
        while queue:
            a = queue.popleft()
            for b in adj[a]:
                if mol_id[b] < 0:
                    mol_id[b] = start
                    queue.append(b)
    ids = np.unique(mol_id)                       # sorted
    number = np.searchsorted(ids, mol_id) + 1     # 1..M
    return number.astype(np.int32), ids


def species(number, types, ntypes=4):
    """(per-molecule element counts (M, ntypes), species table (S, ntypes + 1)):
    each distinct count vector with its number of molecules, in increasing
    lexicographic order of the counts."""
    M = int(number.max()) if number.size else 0
    counts = np.zeros((M, ntypes), dtype=np.int64)
    for m, t in zip(number, types):
        counts[m - 1, t] += 1
    if M == 0:
        return counts, np.zeros((0, ntypes + 1), dtype=np.int64)
    uniq, mult = np.unique(counts, axis=0, return_counts=True)
    return counts, np.concatenate([uniq, mult[:, None]], axis=1)


def analyse(n, types, bonds, bo, threshold=0.3):
    number, ids = molecules(n, bonds, bo, threshold)
    counts, table = species(number, np.asarray(types))
    return number, counts, table


def formula(row, elements=("C", "H", "N", "O")):
    """Chemical formula of a species row, e.g. 'C1H4' (elements with zero count omitted)."""
    return "".join(f"{e}{int(c)}" for e, c in zip(elements, row) if c)
