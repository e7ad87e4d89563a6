"""Parity at the benchmark sizes, in the launch configuration bench.py times.

32,480 atoms: the oracle evaluates the whole box (lists as sets, every energy
term, every force).  1,044,000 atoms: list sizes and energies against values
stored by tests/golden/make_golden.py (which calls only the oracle), and the
forces and neighbour sets of sampled atoms against the oracle evaluated on a
35 A sphere around each sampled atom.  The force on an atom depends on
positions at most a few bond lengths plus r_nonb away (the bond-order
correction reaches two bonds, the over/under-coordination and coalition terms
one more, each term's inputs one more), so within 35 A the sphere reproduces
every input of every term that moves the centre atom.
"""
import json
import os

import numpy as np
import pytest

import reaxff_synth as rs
from oracle import TERM_NAMES, Oracle

from _common import (assert_energy_parity, assert_force_parity, assert_lists_equal,
                     extract_subsystem, gpu_eval, pairs_set)

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_energies.json")
SPHERE = 35.0
NSAMPLE = 6


@pytest.fixture(scope="module")
def params():
    return rs.draw_params(0)


@pytest.fixture(scope="module")
def golden():
    with open(GOLDEN) as f:
        return json.load(f)["workloads"]


@pytest.fixture(scope="module")
def ff(params):
    from paper_1706_07772_amd import ReaxFF
    f = ReaxFF(params)
    yield f
    f.close()


def test_petn_32480_full_parity(ff, params, golden):
    s = rs.workload("petn_32480")
    e, f, lists = gpu_eval(ff, s, lists=True)
    o = Oracle(s, params)
    assert_lists_equal(lists, o, o.lists())
    e_ref, e_abs = o.energy_abs()
    _, f_ref = o.forces()
    assert_energy_parity(e, e_ref, e_abs, names=TERM_NAMES)
    assert_force_parity(f, f_ref)
    g = golden["petn_32480"]
    assert ff.list_sizes() == (g["far_pairs"], g["bond_entries"], g["hb_entries"])


@pytest.fixture(scope="module")
def big(ff):
    s = rs.workload("petn_1044000")
    e, f, lists = gpu_eval(ff, s, lists=True)
    print("1.04M counts", ff.interaction_counts(), flush=True)
    return s, e, f, lists, ff.list_sizes()


def test_fullsize_list_sizes(big, golden):
    s, e, f, lists, sizes = big
    g = golden["petn_1044000"]
    assert s.n == g["atoms"]
    assert sizes == (g["far_pairs"], g["bond_entries"], g["hb_entries"])


def test_fullsize_energies(big, golden):
    s, e, f, lists, sizes = big
    g = golden["petn_1044000"]
    e_ref = np.array([g["energies"][t] for t in TERM_NAMES])
    e_abs = np.array([g["abs_sums"][t] for t in TERM_NAMES])
    assert_energy_parity(e, e_ref, e_abs, names=TERM_NAMES)


def test_fullsize_net_force(big):
    s, e, f, lists, sizes = big
    assert np.abs(f.sum(0)).max() <= 1e-11 * np.abs(f).max() * s.n


@pytest.mark.parametrize("k", range(NSAMPLE))
def test_fullsize_sampled_atoms(big, params, k):
    """Force and neighbour sets of a sampled atom against the oracle on a 35 A sphere."""
    s, e, f, lists, sizes = big
    rng = np.random.default_rng(1000 + k)
    c = int(rng.integers(s.n))
    sub, ci, ids = extract_subsystem(s, c, SPHERE)
    o = Oracle(sub, params)
    _, f_sub = o.forces()
    scale = np.linalg.norm(f, axis=1).max()
    err = np.linalg.norm(f[c] - f_sub[ci])
    assert err <= 1e-9 * scale, (c, f[c], f_sub[ci], err / scale)
    # neighbour sets of the centre atom, in caller ids
    of, ob, oh = o.lists()
    gf, gb, gh = lists

    def around(pairs, centre, sym):
        if sym:
            sel = (pairs[:, 0] == centre) | (pairs[:, 1] == centre)
            p = pairs[sel]
            return set(np.where(p[:, 0] == centre, p[:, 1], p[:, 0]).tolist())
        return set(pairs[pairs[:, 0] == centre, 1].tolist())

    ref_far = {int(ids[j]) for j in around(of, ci, True)}
    ref_bond = {int(ids[j]) for j in around(ob, ci, False)}
    ref_hb = {int(ids[j]) for j in around(oh, ci, False)}
    assert around(gf, c, True) == ref_far
    assert around(gb, c, False) == ref_bond
    assert around(gh, c, False) == ref_hb
