"""Verlet-skin lists (reaxff_set_skin, reaxff_refresh_lists), the paper's
setup of neighbour lists checked every 10 steps.  Lists are supersets, so
list parity is redefined: every pair of the oracle's exact far and H sets is
kept and every kept pair lies within the cutoff plus the skin, while the bond
list (made again at every refresh) equals the oracle's exactly.  Energies and
forces equal the oracle's to 1e-9 after refreshes with moved atoms; a move
beyond half the skin, or `every` refreshes, build the lists again; an MD run
with lists kept over 10 steps follows the oracle's trajectory (lists built
every step) and the GPU's own exact-list trajectory on the 32,480-atom box."""
import numpy as np
import pytest

import reaxff_synth as rs
from oracle import Oracle

from _common import (assert_energy_parity, assert_force_parity, pairs_set, to_dev)

pytestmark = pytest.mark.gpu

SKIN = 0.5


@pytest.fixture(scope="module")
def params():
    return rs.draw_params(0)


def min_image(d, box):
    if box is None:
        return d
    return d - box * np.rint(d / box)


def check_superset(gpu_lists, ora_lists, system, pos_build, r_far, r_hb):
    """Every exact pair at the current positions is kept; every kept pair was
    within the enlarged cutoff at the positions of the build."""
    gf, gb, gh = gpu_lists
    of, ob, oh = ora_lists
    sf, sh = pairs_set(gf, symmetric=True), pairs_set(gh)
    assert pairs_set(of) <= sf and pairs_set(oh) <= sh
    for pairs, r in ((gf, r_far), (gh, r_hb)):
        if len(pairs):
            d = min_image(pos_build[pairs[:, 1]] - pos_build[pairs[:, 0]], system.box)
            assert np.sqrt((d * d).sum(1)).max() <= r * (1 + 1e-12)
    assert pairs_set(gb) == pairs_set(ob)   # bond list exact (no borderline pair in these inputs)


def wrapped(system, pos):
    p = pos if system.box is None else np.mod(pos, system.box)
    return rs.System(pos=p, type=system.type, q=system.q, box=system.box)


@pytest.mark.parametrize("name", ["petn_1856", "cluster300"])
def test_kept_lists_and_forces_over_refreshes(params, name):
    import torch
    from paper_1706_07772_amd import ReaxFF
    s = rs.workload("petn_1856") if name == "petn_1856" else rs.cluster(300, seed=51)
    ff = ReaxFF(params)
    ff.set_skin(SKIN, 10)
    rng = np.random.default_rng(6)
    v = rng.normal(size=s.pos.shape)
    v *= 0.05 / np.linalg.norm(v, axis=1, keepdims=True)   # 0.05 A per refresh, 0.2 A after four
    pos0, typ, q, box = to_dev(s)
    ff.build_lists(pos0, typ, box)
    for k in range(5):
        pos = s.pos + k * v
        P = torch.tensor(pos, dtype=torch.float64, device="cuda:0")
        if k > 0:
            assert ff.refresh_lists(P, typ, box) is False
        f, e = ff.compute_forces(P, typ, q, box)
        torch.cuda.synchronize()
        o = Oracle(wrapped(s, pos), params)
        check_superset(ff.export_lists(), o.lists(), wrapped(s, pos), s.pos, 10.0 + SKIN, 7.5 + SKIN)
        e_ref, e_abs = o.energy_abs()
        _, f_ref = o.forces()
        assert_energy_parity(e.cpu().numpy(), e_ref, e_abs)
        assert_force_parity(f.cpu().numpy(), f_ref)
    assert ff.list_stats() == (1, 4)
    ff.close()


def test_rebuild_rules(params):
    import torch
    from paper_1706_07772_amd import ReaxFF
    s = rs.workload("petn_1856")
    ff = ReaxFF(params)
    ff.set_skin(SKIN, 3)
    pos, typ, q, box = to_dev(s)
    ff.build_lists(pos, typ, box)
    assert ff.refresh_lists(pos, typ, box) is False
    assert ff.refresh_lists(pos, typ, box) is False
    assert ff.refresh_lists(pos, typ, box) is True        # `every` = 3 refreshes
    moved = pos.clone()
    moved[7, 0] += 0.6 * SKIN                              # beyond half the skin
    assert ff.refresh_lists(moved, typ, box) is True
    moved[7, 0] += 0.4 * SKIN                              # within half the skin of the new build
    assert ff.refresh_lists(moved, typ, box) is False
    # a box too small for the enlarged cutoff
    from paper_1706_07772_amd import ReaxFFError
    small = rs.small_periodic(30, seed=52)   # ~20.3 A < 2 (10 + skin)
    p2, t2, q2, b2 = to_dev(small)
    with pytest.raises(ReaxFFError) as ei:
        ff.build_lists(p2, t2, b2)
    assert ei.value.code == -3
    ff.set_skin(0.0, 1)
    ff.build_lists(p2, t2, b2)
    ff.close()


def run_md(params, s, v0, nsteps, skin):
    import torch
    from paper_1706_07772_amd import ReaxFF
    ff = ReaxFF(params)
    if skin:
        ff.set_skin(skin, 10)
    pos, typ, q, box = to_dev(s)
    vel = torch.tensor(v0, dtype=torch.float64, device="cuda:0")
    f, e = ff.step(pos, vel, typ, q, box, 0.1, nsteps)
    torch.cuda.synchronize()
    stats = ff.list_stats()
    out = pos.cpu().numpy(), vel.cpu().numpy(), e.cpu().numpy(), stats
    ff.close()
    return out


def test_md_with_kept_lists_matches_oracle(params):
    s = rs.workload("petn_1856")
    v0 = rs.maxwell_boltzmann(s.type, params.atom["mass"], 300.0, seed=131)
    pos, vel, e, stats = run_md(params, s, v0, 20, SKIN)
    assert stats[0] <= 4 and stats[1] >= 16, stats   # builds at steps 0, 10, 20
    pos_r, vel_r, e_r = Oracle(s, params).md(v0, 0.1, 20)
    assert np.abs(min_image(pos - pos_r, s.box)).max() <= 1e-9
    assert np.abs(vel - vel_r).max() <= 1e-9 * np.abs(vel_r).max()
    assert np.allclose(e, e_r, rtol=1e-8, atol=1e-8 * np.abs(e_r).max())


def test_md_32480_kept_lists_vs_exact_lists(params):
    s = rs.workload("petn_32480")
    v0 = rs.maxwell_boltzmann(s.type, params.atom["mass"], 300.0, seed=132)
    pos_a, vel_a, e_a, st_a = run_md(params, s, v0, 30, 0.0)
    pos_b, vel_b, e_b, st_b = run_md(params, s, v0, 30, SKIN)
    print("builds/refreshes exact", st_a, "kept", st_b, flush=True)
    assert st_b[0] <= 5
    assert np.abs(min_image(pos_a - pos_b, s.box)).max() <= 1e-9
    assert np.allclose(e_a, e_b, rtol=1e-9, atol=1e-9 * np.abs(e_a).max())
