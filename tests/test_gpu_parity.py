"""GPU path vs the CPU oracle: lists as exact sets, energies and forces to 1e-9.

Every test calls the HIP library through its C ABI (ctypes binding) and the
oracle through its own library; the two share no code.
"""
import math

import numpy as np
import pytest

import reaxff_synth as rs
from oracle import TERM_NAMES, Oracle

from _common import (assert_energy_parity, assert_force_parity, assert_lists_equal, gpu_eval,
                     to_dev)

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


def _parity(ff, params, system, cutoffs=None):
    if cutoffs is not None:
        from paper_1706_07772_amd import ReaxFF
        ff = ReaxFF(params, cutoffs)
    e, f, lists = gpu_eval(ff, system, lists=True)
    o = Oracle(system, params, cutoffs)
    nborder = assert_lists_equal(lists, o, o.lists())
    e_ref, e_abs = o.energy_abs()
    _, f_ref = o.forces()
    assert_energy_parity(e, e_ref, e_abs, names=TERM_NAMES)
    assert_force_parity(f, f_ref)
    return e, f, nborder


def test_petn_1856_parity(ff, params):
    """The 1,856-atom periodic PETN-stoichiometry box (64 units, 26.7 A)."""
    s = rs.workload("petn_1856")
    e, f, _ = _parity(ff, params, s)
    counts = ff.interaction_counts()
    print("counts", counts, flush=True)
    assert counts["angles"] > 0 and counts["torsions"] > 0 and counts["hbonds"] > 0


@pytest.mark.parametrize("n,seed", [(10, 1), (57, 2), (300, 3), (137, 4)])
def test_cluster_parity(ff, params, n, seed):
    _parity(ff, params, rs.cluster(n, seed=seed))


def test_small_periodic_parity(ff, params):
    """870 atoms in a 20.7 A box: the cell grid has 4 cells per edge, so every cell is
    visited once (the stencil's wrap-around degenerate case)."""
    _parity(ff, params, rs.small_periodic(30, seed=7))


def test_parity_shifted_outside_box(ff, params):
    """Positions given outside [0, L): minimum image and cell wrap must agree."""
    s = rs.small_periodic(40, seed=8)
    s.pos = s.pos + np.array([3.5 * s.box[0], -2.0 * s.box[1], 0.25])
    _parity(ff, params, s)


def test_smooth_threshold_parity(ff, params):
    """Thresholds at zero (every bond pair forms angles and torsions) and a tiny list
    threshold: many more interactions, same parity."""
    cut = dict(rs.DEFAULT_CUTOFFS, bo_cut=1e-6, thb_cut=0.0, thb_cutsq=0.0, hb_bo_cut=0.0)
    _parity(ff, params, rs.cluster(120, seed=9), cut)


def test_net_force_zero(ff, params):
    s = rs.workload("petn_1856")
    e, f = gpu_eval(ff, s)
    assert np.abs(f.sum(0)).max() <= 1e-11 * np.abs(f).max() * s.n


def test_lists_and_forces_deterministic(ff, params):
    s = rs.workload("petn_1856")
    e1, f1, l1 = gpu_eval(ff, s, lists=True)
    e2, f2, l2 = gpu_eval(ff, s, lists=True)
    for a, b in zip(l1, l2):
        assert np.array_equal(a, b)
    assert np.abs(f1 - f2).max() <= 1e-13 * np.abs(f1).max()
    assert np.allclose(e1, e2, rtol=1e-13, atol=0)


# ---------------------------------------------------------------------------
# edge cases
# ---------------------------------------------------------------------------
def test_empty_system(ff, params):
    s = rs.System(pos=np.zeros((0, 3)), type=np.zeros(0, np.int32), q=np.zeros(0), box=None)
    e, f = gpu_eval(ff, s)
    assert f.shape == (0, 3) and np.all(e == 0)
    assert ff.list_sizes() == (0, 0, 0)


def test_single_atom_and_isolated_atoms(ff, params):
    for pos, typ in (([[1.0, 2.0, 3.0]], [2]),
                     ([[0, 0, 0], [12, 0, 0], [0, 12, 0], [0, 0, 12]], [0, 1, 2, 3])):
        s = rs.System(pos=np.array(pos, float), type=np.array(typ, np.int32),
                      q=np.zeros(len(typ)), box=None)
        e, f = gpu_eval(ff, s)
        o = Oracle(s, params)
        e_ref, e_abs = o.energy_abs()
        assert_energy_parity(e, e_ref, e_abs)
        assert np.all(f == 0)


def test_pair_at_exact_cutoff(ff, params):
    """A pair at exactly r = r_nonb is listed (r <= cutoff) and contributes zero."""
    s = rs.System(pos=np.array([[0.0, 0.0, 0.0], [10.0, 0.0, 0.0]]), type=np.array([0, 3], np.int32),
                  q=np.array([0.3, -0.3]), box=None)
    e, f, lists = gpu_eval(ff, s, lists=True)
    assert len(lists[0]) == 1
    assert abs(e[11]) < 1e-15 and np.abs(f).max() < 1e-12


def test_error_paths(ff, params):
    import torch
    from paper_1706_07772_amd import ReaxFFError
    s = rs.cluster(20, seed=3)
    pos, typ, q, box = to_dev(s)
    bad = typ.clone()
    bad[5] = 7
    with pytest.raises(ReaxFFError) as ei:
        ff.build_lists(pos, bad, None)
    assert ei.value.code == -1
    with pytest.raises(ReaxFFError) as ei:
        ff.build_lists(pos, typ, [19.0, 30.0, 30.0])
    assert ei.value.code == -3
    nanpos = pos.clone()
    nanpos[3, 1] = float("nan")
    with pytest.raises(ReaxFFError) as ei:
        ff.build_lists(nanpos, typ, None)
    assert ei.value.code == -5
    # forces for a different n than the lists were built for
    ff.build_lists(pos, typ, None)
    with pytest.raises(ReaxFFError) as ei:
        ff.compute_forces(pos[:10].contiguous(), typ[:10].contiguous(), q[:10].contiguous(), None)
    assert ei.value.code == -6
    # the context still works afterwards
    e, f = gpu_eval(ff, s)
    assert np.isfinite(e).all() and np.isfinite(f).all()
