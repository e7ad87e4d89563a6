"""GPU path vs the CPU oracle: lists as exact sets, energies and forces to 1e-9.

Every test calls the HIP library through its C ABI (ctypes binding) and the
oracle through its own library; the two share no code.
"""
import ctypes
import math

import numpy as np
import pytest

import reaxff_synth as rs
from oracle import TERM_NAMES, Oracle

from _common import (assert_energy_parity, assert_force_parity, assert_lists_equal, gpu_eval,
                     near_straight_chain, to_dev)

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


def _oracle_ref(system, params, cutoffs=None):
    o = Oracle(system, params, cutoffs)
    e_ref, e_abs = o.energy_abs()
    _, f_ref = o.forces()
    return o, o.lists(), e_ref, e_abs, f_ref


def _parity(ff, params, system, cutoffs=None, ff_cut=False, ref=None):
    """ff_cut: ff was made with these cutoffs; otherwise a context is made for
    them.  ref: the oracle's results for this system (_oracle_ref)."""
    if cutoffs is not None and not ff_cut:
        from paper_1706_07772_amd import ReaxFF
        ff = ReaxFF(params, cutoffs)
    e, f, lists = gpu_eval(ff, system, lists=True)
    o, olists, e_ref, e_abs, f_ref = ref if ref is not None else _oracle_ref(system, params, cutoffs)
    nborder = assert_lists_equal(lists, o, olists)
    assert_energy_parity(e, e_ref, e_abs, names=TERM_NAMES)
    assert_force_parity(f, f_ref)
    return e, f, nborder


def _launches(ff):
    """Kernel launch counts since profiling was switched on (name -> launches)."""
    K = 32
    ms = (ctypes.c_double * K)()
    calls = (ctypes.c_int64 * K)()
    names = (ctypes.c_char_p * K)()
    k = ff._lib.reaxff_profile_read(ff._h, K, ms, calls, names)
    return {names[i].decode(): int(calls[i]) for i in range(k)}


def _parity_path(ff, params, system, half, cutoffs=None, ref=None):
    """Parity, and that the nonbonded term took the expected path: the half
    evaluation (pairs once, partial arrays summed per atom) needs at least
    2 reach + 1 cells per edge; smaller grids evaluate every pair from both
    atoms.  cutoffs: those ff was made with."""
    ff._lib.reaxff_profile(ff._h, 1)
    try:
        out = _parity(ff, params, system, cutoffs, ff_cut=True, ref=ref)
        used = _launches(ff)
    finally:
        ff._lib.reaxff_profile(ff._h, 0)
    print("nonbonded launches", used.get("nonbonded", 0), "reduce", used.get("nb_reduce", 0), flush=True)
    assert used.get("nonbonded", 0) > 0
    assert (used.get("nb_reduce", 0) > 0) == half
    return out


def test_half_nonbonded_periodic_shifted(ff, params):
    """6,264 atoms in a 40.05 A periodic box: 8 cells per edge, image shifts per
    stencil column, every pair evaluated once."""
    _parity_path(ff, params, rs.petn_lattice(216, 40.05, seed=11), half=True)


def test_half_nonbonded_open_cluster(ff, params):
    """A 3,000-atom open cluster (about 31 A across, 6 cells per edge): half
    evaluation with stencils clipped at the grid faces."""
    _parity_path(ff, params, rs.cluster(3000, seed=5), half=True)


def test_half_nonbonded_wrapping_both_sides(ff, params):
    """The 1,856-atom box has 5 cells per edge: every stencil column wraps,
    below the cell for some cells and above it for others."""
    _parity_path(ff, params, rs.petn_lattice(64, 26.7, seed=0), half=True)


def test_full_nonbonded_small_grid(ff, params):
    """870 atoms in a 20.7 A box (4 cells per edge): the stencil covers every
    cell, so pairs are evaluated from both atoms."""
    _parity_path(ff, params, rs.petn_lattice(30, 20.7, seed=4), half=False)


@pytest.mark.parametrize("run", [1, 2, 3, 4, 8])
def test_half_nonbonded_run_lengths(params, run):
    """Runs of 1-8 cells per workgroup (the 6,264-atom box has 8 cells per edge,
    so runs of 3 leave a short last run, and the windows of the first and last
    runs wrap below and above; 8 is capped at 4 = 8 - 2 reach) and in the open
    3,000-atom cluster (windows clipped at the grid faces): the same pairs, each
    once, and the same results."""
    from paper_1706_07772_amd import ReaxFF
    ff = ReaxFF(params)
    try:
        ff.set_nb_run(run)
        for s in (rs.petn_lattice(216, 40.05, seed=11), rs.cluster(3000, seed=5)):
            _parity_path(ff, params, s, half=True)
    finally:
        ff.close()


def test_half_nonbonded_runs_minimum_image(params):
    """A 31 A box (2,900 atoms, 6 cells per edge) has too few cells for the
    staged image shifts, so every pair takes the minimum image; runs of 2
    cells (6 - 2 reach) and of 1, with positions inside and outside the box."""
    from paper_1706_07772_amd import ReaxFF
    s = rs.petn_lattice(100, 31.0, seed=14)
    moved = rs.System(pos=s.pos + np.array([31.0, -62.0, 0.5]), type=s.type, q=s.q, box=s.box)
    ref = _oracle_ref(s, params)
    for run in (8, 1):
        ff = ReaxFF(params)
        try:
            ff.set_nb_run(run)
            _parity_path(ff, params, s, half=True, ref=ref)
            _parity_path(ff, params, moved, half=True)
        finally:
            ff.close()


def _slab():
    """A 40 x 40 x 100 A block of 20 A PETN-density cubes in a periodic
    100 x 40 x 100 A box (60 A of vacuum along x): the mean density over the
    box is 40% of the block's."""
    cube = rs.petn_lattice(27, 20.0, seed=21)
    shifts = [np.array([20.0 * a, 20.0 * b, 20.0 * c]) for a in range(2) for b in range(2) for c in range(5)]
    pos = np.concatenate([cube.pos + d for d in shifts])
    typ = np.concatenate([cube.type] * len(shifts)).astype(np.int32)
    q = np.concatenate([cube.q] * len(shifts))
    return rs.System(pos=pos, type=typ, q=q, box=np.array([100.0, 40.0, 100.0]))


def test_half_nonbonded_runs_shortened(params):
    """Runs chosen from the mean density are too long where the atoms are:
    with runs of up to 16 cells allowed, the block's windows (12 upper columns
    of 20 cells and 18 cells of the centre column, about 3,150 atoms) exceed
    the 2,560-atom copy, so the build halves the runs and sweeps again."""
    from paper_1706_07772_amd import ReaxFF
    s = _slab()
    # the library's first choice: the longest run whose upper window at the
    # mean density over the grid's cells fills at most 80% of the copy
    nc = np.floor(s.box / 5.0).astype(int)
    per_cell = s.n / nc.prod()
    k0 = min(16, int(nc[2]) - 4, int(math.floor((0.8 * 2560 / per_cell - 50) / 13)))
    assert k0 == 16
    block = s.n / (40.0 * 40.0 * 100.0) * 125.0   # atoms per cell inside the block
    assert block * (12 * (k0 + 4) + k0 + 2) > 2560 * 1.15
    ff = ReaxFF(params)
    try:
        ff.set_nb_run(16)
        _parity_path(ff, params, s, half=True)
    finally:
        ff.close()


def test_dense_fallbacks_then_normal_density(params):
    """A 15 A nonbonded cutoff (7.5 A cells) at the benchmark density: the
    6,264-atom box has 5 cells per edge and an upper stencil of about 3,150
    atoms, beyond the half evaluation's 2,560-atom LDS copy even for runs of one
    cell, so the build sweeps again with full rows and the nonbonded term
    evaluates every pair from both atoms; the whole-grid stencil (all 6,264
    atoms) exceeds that kernel's LDS copy (2,048) too, so neighbours are read
    from memory through the chunk table.  The same context then builds a box at
    half that density, keeping full far rows (the half evaluation reads the
    rows' upper parts through far_lo)."""
    from paper_1706_07772_amd import ReaxFF
    cut = dict(rs.DEFAULT_CUTOFFS, r_nonb=15.0)
    dense = rs.petn_lattice(216, 40.05, seed=12)
    assert dense.n * 63 / 125 > 2560 and dense.n > 2048
    ff = ReaxFF(params, cut)
    try:
        _parity_path(ff, params, dense, half=False, cutoffs=cut)
        sparse = rs.petn_lattice(108, 40.05, seed=13)
        assert sparse.n * 63 / 125 < 0.8 * 2560
        _parity_path(ff, params, sparse, half=True, cutoffs=cut)
    finally:
        ff.close()


@pytest.mark.parametrize("eps", [1e-2, 1e-4, 1e-6])
def test_near_straight_angle_parity(ff, params, eps):
    """A valence angle and two torsions whose shared angle is straight to within
    eps: both sides take the angle from |a x b| and a . b and the torsion's
    sines from cross products, so no clamp or band exists, and the forces agree
    down to the conditioning of the geometry itself."""
    _parity(ff, params, near_straight_chain(eps))
    # the same chain inside a cluster, so the angle sits among ordinary terms
    c = rs.cluster(120, seed=9)
    chain = near_straight_chain(eps)
    pos = np.concatenate([c.pos, chain.pos + np.array([40.0, 40.0, 40.0])])
    s = rs.System(pos=pos, type=np.concatenate([c.type, chain.type]).astype(np.int32),
                  q=np.concatenate([c.q, chain.q]), box=None)
    _parity(ff, params, s)


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


def test_hydrogen_rich_cluster_parity(ff, params):
    """An H/O-rich cluster (55% H, 35% O) with every bond order above 1e-6
    a bond and every H-acceptor bond a donor bond: hundreds of acceptor rows
    hold more (H, donor bond) pairs than the 128 the acceptor kernel lists in
    LDS, so its direct walk runs beside the listed one; torsions are sparse
    among many bonded atoms, so blocks of torsion tasks span many entries."""
    s = rs.cluster(1500, seed=11, probs=(0.05, 0.55, 0.05, 0.35))
    cut = dict(rs.DEFAULT_CUTOFFS, bo_cut=1e-6, hb_bo_cut=0.0)
    _parity(ff, params, s, cut)
    # (H, donor bond) pairs of each acceptor's row, from the oracle's lists
    _, bonds, hb = Oracle(s, params, cut).lists()
    typ = s.type
    don = np.zeros(len(typ), np.int64)
    m = (typ[bonds[:, 0]] == 1) & np.isin(typ[bonds[:, 1]], (2, 3))
    np.add.at(don, bonds[m, 0], 1)
    per = np.zeros(len(typ), np.int64)
    np.add.at(per, hb[:, 1], don[hb[:, 0]])
    print("acceptor rows over 128 pairs:", int((per > 128).sum()), "max", int(per.max()), flush=True)
    assert (per > 128).sum() > 0


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


@pytest.mark.parametrize("system", ["box", "cluster"])
def test_overlap_matches_in_order(ff, params, system):
    """The nonbonded term on the context's second stream, concurrent with the
    bonded terms, gives the energies and forces of the in-order run (the two
    differ only in the order of floating-point additions)."""
    s = rs.petn_lattice(216, 40.05, seed=11) if system == "box" else rs.cluster(3000, seed=5)
    try:
        ff.set_overlap(False)
        e0, f0 = gpu_eval(ff, s)
        ff.set_overlap(True)
        e1, f1 = gpu_eval(ff, s)
    finally:
        ff.set_overlap(True)
    scale = np.abs(e0).max()
    assert np.abs(e1 - e0).max() <= 1e-12 * scale
    assert np.abs(f1 - f0).max() <= 1e-11 * np.abs(f0).max()


@pytest.mark.parametrize("name", ["petn_1856", "cluster300", "petn_6264"])
def test_caller_owned_lists_capacity_protocol(params, name):
    """reaxff_build_lists_into: undersized caller buffers give REAXFF_ERR_CAPACITY
    with required[] and no lists; buffers grown to required[] (again if the
    rows outgrow the first estimate) give the lists, identical to the context's
    own, and forces through them equal the oracle's.  The 6,264-atom box (8
    cells per edge) numbers its far rows by windows of runs of 4 cells."""
    import torch
    from paper_1706_07772_amd import ListBuffers, ReaxFF, ReaxFFError
    s = {"petn_1856": lambda: rs.workload("petn_1856"), "cluster300": lambda: rs.cluster(300, seed=61),
         "petn_6264": lambda: rs.petn_lattice(216, 40.05, seed=11)}[name]()
    ff = ReaxFF(params)
    try:
        pos, typ, q, box = to_dev(s)
        bufs = ListBuffers(16, 16, 16)
        rc = ff.build_lists_into(pos, typ, box, bufs)
        assert rc == -2 and min(bufs.required) > 16
        with pytest.raises(ReaxFFError) as ei:          # nothing was built
            ff.compute_forces(pos, typ, q, box)
        assert ei.value.code == -6
        tries = 1
        while rc == -2:
            bufs.resize(*bufs.required)
            rc = ff.build_lists_into(pos, typ, box, bufs)
            tries += 1
            assert tries <= 4
        assert rc == 0
        far, bonds, hb = ff.export_lists()
        f, e = ff.compute_forces_from(pos, typ, q, box, bufs)
        torch.cuda.synchronize()
        assert bufs.required[1] == len(bonds)
        o = Oracle(s, params)
        assert_lists_equal((far, bonds, hb), o, o.lists())
        e_ref, e_abs = o.energy_abs()
        _, f_ref = o.forces()
        assert_energy_parity(e.cpu().numpy(), e_ref, e_abs, names=TERM_NAMES)
        assert_force_parity(f.cpu().numpy(), f_ref)
        # the context's own lists: the same sets; the caller's buffers no longer match
        ff.build_lists(pos, typ, box)
        far2, bonds2, hb2 = ff.export_lists()
        assert sorted(map(tuple, far.tolist())) == sorted(map(tuple, far2.tolist()))
        assert sorted(map(tuple, bonds.tolist())) == sorted(map(tuple, bonds2.tolist()))
        with pytest.raises(ReaxFFError) as ei:
            ff.compute_forces_from(pos, typ, q, box, bufs)
        assert ei.value.code == -6
    finally:
        ff.close()


@pytest.mark.parametrize("kind", ["clustered", "sparse", "open_cluster"])
def test_masked_forces_exact_on_marked_atoms(params, kind):
    """reaxff_forces_masked: the forces of the marked atoms from the plain
    evaluation of the atoms within the dependency radius of them equal those of
    the whole system (1e-9), while the evaluated subsystem stays smaller than
    the system when the marked atoms are few or clustered."""
    import torch
    from paper_1706_07772_amd import ReaxFF
    if kind == "open_cluster":
        s = rs.cluster(20000, seed=71)   # about 59 A across
    else:
        s = rs.workload("petn_32480")
    ff = ReaxFF(params)
    try:
        pos, typ, q, box = to_dev(s)
        ff.build_lists(pos, typ, box)
        f_all, _ = ff.compute_forces(pos, typ, q, box)
        f_all = f_all.cpu().numpy()
        R = ff.dependency_radius()
        rng = np.random.default_rng(3)
        if kind == "sparse":
            mask = np.zeros(s.n, dtype=np.uint8)
            mask[rng.choice(s.n, size=3, replace=False)] = 1
        else:
            c = s.pos[rng.integers(s.n)]
            d = s.pos - c
            if s.box is not None:
                d -= s.box * np.rint(d / s.box)
            mask = (np.sqrt((d * d).sum(1)) <= 5.0).astype(np.uint8)
        out = torch.full((s.n, 3), 7.0, dtype=torch.float64, device="cuda:0")
        nsub = ff.forces_masked(pos, typ, q, box, torch.tensor(mask, device="cuda:0"), out)
        torch.cuda.synchronize()
        out = out.cpu().numpy()
        m = mask.astype(bool)
        print(kind, "marked", int(m.sum()), "subsystem", nsub, "of", s.n, "R", R, flush=True)
        assert 0 < m.sum() <= nsub < s.n
        assert np.all(out[~m] == 7.0)                    # unmarked rows untouched
        scale = np.linalg.norm(f_all, axis=1).max()
        err = np.linalg.norm(out[m] - f_all[m], axis=1).max()
        assert err <= 1e-9 * scale, err / scale
        # every atom marked: the whole system
        allm = torch.ones(s.n, dtype=torch.uint8, device="cuda:0")
        out2 = torch.zeros((s.n, 3), dtype=torch.float64, device="cuda:0")
        assert ff.forces_masked(pos, typ, q, box, allm, out2) == s.n
        assert np.abs(out2.cpu().numpy() - f_all).max() <= 1e-12 * scale
    finally:
        ff.close()
