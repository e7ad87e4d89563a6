"""In-situ species analysis on the GPU (reaxff_species) against the oracle
(oracle/species.py) fed with the oracle's own corrected bond orders: molecule
numbers of every atom, element counts per molecule and the species table,
exactly, at several thresholds (isolated atoms through one percolating
cluster), on clusters and periodic boxes up to 32,480 atoms; bookkeeping
identities at 1,044,000 atoms; call-order and empty cases."""
import numpy as np
import pytest

import reaxff_synth as rs
from oracle import Oracle
from oracle import species as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def params():
    return rs.draw_params(0)


@pytest.fixture(scope="module")
def ff(params):
    from paper_1706_07772_amd import ReaxFF
    f = ReaxFF(params)
    yield f
    f.close()


def gpu_forces(ff, system):
    import torch
    d = torch.device("cuda:0")
    P = torch.tensor(system.pos, dtype=torch.float64, device=d)
    T = torch.tensor(system.type, dtype=torch.int32, device=d)
    Q = torch.tensor(system.q, dtype=torch.float64, device=d)
    box = None if system.box is None else system.box
    ff.build_lists(P, T, box)
    ff.compute_forces(P, T, Q, box)


def clear_threshold(bo, thr):
    """A threshold no bond order lies within 1e-9 (relative) of: both sides then
    decide every bond the same way whatever their last-ulp differences."""
    while np.any(np.abs(bo - thr) <= 1e-9 * thr):
        thr += 1e-7
    return thr


SYSTEMS = {
    "cluster300": lambda: rs.cluster(300, seed=41),
    "periodic870": lambda: rs.small_periodic(30, seed=42),
    "petn_1856": lambda: rs.workload("petn_1856"),
    "petn_32480": lambda: rs.workload("petn_32480"),
}


@pytest.mark.parametrize("name", sorted(SYSTEMS))
def test_species_match_oracle(ff, params, name):
    import torch
    s = SYSTEMS[name]()
    print(f"species {name} n={s.n}", flush=True)
    o = Oracle(s, params)
    _, bonds, _ = o.lists()
    bo = o.bond_terms()[:, 0]
    gpu_forces(ff, s)
    for thr0 in (0.05, 0.3, 1.0):
        thr = clear_threshold(bo, thr0)
        number, counts, table = S.analyse(s.n, s.type, bonds, bo, thr)
        mol, mc, tab = ff.species(s.n, thr)
        torch.cuda.synchronize()
        assert np.array_equal(mol.cpu().numpy(), number), (name, thr)
        assert np.array_equal(mc.cpu().numpy(), counts)
        assert np.array_equal(tab.cpu().numpy(), table)


def test_full_size_bookkeeping(ff, params):
    import torch
    s = rs.workload("petn_1044000")
    gpu_forces(ff, s)
    mol, mc, tab = ff.species(s.n, 0.3)
    torch.cuda.synchronize()
    mol, mc, tab = mol.cpu().numpy(), mc.cpu().numpy(), tab.cpu().numpy()
    M = mc.shape[0]
    print(f"species 1044000: {M} molecules, {tab.shape[0]} species", flush=True)
    assert mol.min() == 1 and mol.max() == M
    # molecule numbers increase with each molecule's smallest atom index
    first = np.full(M, s.n)
    np.minimum.at(first, mol - 1, np.arange(s.n))
    assert np.all(np.diff(first) > 0)
    # per-molecule counts agree with the atoms' numbers and types
    ref = np.zeros((M, 4), dtype=np.int64)
    np.add.at(ref, (mol - 1, s.type), 1)
    assert np.array_equal(mc, ref)
    # the table: distinct rows in increasing order, multiplicities sum to M
    assert tab[:, 4].sum() == M
    keys = [tuple(r) for r in tab[:, :4]]
    assert keys == sorted(keys) and len(set(keys)) == len(keys)
    assert np.array_equal((tab[:, :4] * tab[:, 4:5]).sum(0), np.bincount(s.type, minlength=4))


def test_call_order_and_empty(ff):
    import torch
    from paper_1706_07772_amd import ReaxFFError
    s = rs.cluster(20, seed=43)
    P = torch.tensor(s.pos, dtype=torch.float64, device="cuda:0")
    T = torch.tensor(s.type, dtype=torch.int32, device="cuda:0")
    ff.build_lists(P, T, None)
    with pytest.raises(ReaxFFError) as ei:
        ff.species(s.n)
    assert ei.value.code == -6
    ff.build_lists(torch.zeros((0, 3), dtype=torch.float64, device="cuda:0"),
                   torch.zeros(0, dtype=torch.int32, device="cuda:0"), None)
    ff.compute_forces(torch.zeros((0, 3), dtype=torch.float64, device="cuda:0"),
                      torch.zeros(0, dtype=torch.int32, device="cuda:0"),
                      torch.zeros(0, dtype=torch.float64, device="cuda:0"), None)
    mol, mc, tab = ff.species(0)
    assert mol.numel() == 0 and mc.shape[0] == 0 and tab.shape[0] == 0
