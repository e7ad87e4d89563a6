"""Batched evaluation of many small non-periodic clusters (reaxff_batch_*).

Every cluster's energies and forces against the oracle evaluated on that
cluster alone; far-pair and bond counts against the oracle's lists; every
block size and schedule; the 4,096-cluster batch (sizes 10-300) on sampled
clusters and against the plain path on the same clusters packed far apart in
one system; failure reporting (bad type, scratch capacity) and recovery; the
autotuner.
"""
import numpy as np
import pytest

import reaxff_synth as rs
from oracle import TERM_NAMES, Oracle

from _common import assert_energy_parity, assert_force_parity

pytestmark = pytest.mark.gpu

SCHEDS = (0, 1, 2)
BLOCKS = (64, 128, 256, 512)


@pytest.fixture(scope="module")
def params():
    return rs.draw_params(0)


@pytest.fixture(scope="module")
def ff(params):
    from paper_1706_07772_amd import ReaxFF
    f = ReaxFF(params)
    yield f
    f.close()


def concat(systems):
    off = np.zeros(len(systems) + 1, dtype=np.int64)
    off[1:] = np.cumsum([s.pos.shape[0] for s in systems])
    pos = np.concatenate([s.pos for s in systems]) if off[-1] else np.zeros((0, 3))
    typ = np.concatenate([s.type for s in systems]).astype(np.int32) if off[-1] else np.zeros(0, np.int32)
    q = np.concatenate([s.q for s in systems]) if off[-1] else np.zeros(0)
    return pos, typ, q, off


def split(pos, typ, q, off):
    return [rs.System(pos=pos[off[c]:off[c + 1]], type=typ[off[c]:off[c + 1]], q=q[off[c]:off[c + 1]],
                      box=None) for c in range(off.size - 1)]


def to_dev(pos, typ, q):
    import torch
    d = torch.device("cuda:0")
    return (torch.tensor(pos, dtype=torch.float64, device=d).reshape(-1, 3).contiguous(),
            torch.tensor(typ, dtype=torch.int32, device=d).contiguous(),
            torch.tensor(q, dtype=torch.float64, device=d).contiguous())


def run_batch(ff, pos, typ, q, off, config=None):
    import torch
    from paper_1706_07772_amd import Batch
    b = Batch(ff, off, config)
    P, T, Q = to_dev(pos, typ, q)
    f, e = b.compute(P, T, Q)
    rc, bad = b.status()
    torch.cuda.synchronize()
    out = f.cpu().numpy(), e.cpu().numpy(), b.counts(), rc, bad
    b.close()
    return out


def oracle_ref(system, params):
    """Oracle energies, per-term absolute sums, forces, far-pair and bond counts."""
    n = system.pos.shape[0]
    if n == 0:
        z = np.zeros(12)
        return z, z, np.zeros((0, 3)), 0, 0
    o = Oracle(system, params)
    e, a = o.energy_abs()
    _, f = o.forces()
    far, bonds, _ = o.lists()
    return e, a, f, len(far), len(bonds) // 2


def check_cluster(c, system, params, f_gpu, e_gpu, counts, ref=None):
    e, a, f, nfar, nbond = ref if ref is not None else oracle_ref(system, params)
    assert counts[c, 3] == nfar, (c, counts[c], nfar)
    assert counts[c, 4] == nbond, (c, counts[c], nbond)
    assert_energy_parity(e_gpu[c], e, a, names=TERM_NAMES)
    if f.shape[0]:
        assert_force_parity(f_gpu, f)


@pytest.fixture(scope="module")
def small_batch():
    """24 random clusters of 10-120 atoms plus the edge cases: an empty cluster, one
    atom, one pair, and a maximum-size (384-atom) cluster."""
    rng = np.random.default_rng(7)
    systems = [rs.cluster(int(n), rng=rng) for n in rng.integers(10, 121, size=24)]
    systems.insert(3, rs.System(pos=np.zeros((0, 3)), type=np.zeros(0, np.int32), q=np.zeros(0), box=None))
    systems.insert(7, rs.cluster(1, seed=11))
    pair = rs.System(pos=np.array([[0.0, 0.0, 0.0], [1.2, 0.3, -0.2]]), type=np.array([0, 3], np.int32),
                     q=np.array([0.3, -0.3]), box=None)
    systems.insert(12, pair)
    systems.append(rs.cluster(384, seed=12))
    return systems


@pytest.fixture(scope="module")
def small_refs(small_batch, params):
    return [oracle_ref(s, params) for s in small_batch]


def test_batch_parity_default(ff, params, small_batch, small_refs):
    pos, typ, q, off = concat(small_batch)
    f, e, counts, rc, bad = run_batch(ff, pos, typ, q, off)
    assert rc == 0 and bad == -1
    for c, s in enumerate(small_batch):
        check_cluster(c, s, params, f[off[c]:off[c + 1]], e, counts, small_refs[c])


@pytest.mark.parametrize("block", BLOCKS)
@pytest.mark.parametrize("sched", SCHEDS)
def test_batch_configs(ff, params, small_batch, small_refs, block, sched):
    pos, typ, q, off = concat(small_batch)
    f, e, counts, rc, bad = run_batch(ff, pos, typ, q, off, config=(block, sched, 2))
    assert rc == 0
    for c, s in enumerate(small_batch):
        check_cluster(c, s, params, f[off[c]:off[c + 1]], e, counts, small_refs[c])


def test_batch_counts_match_plain_path(ff, small_batch):
    """Angle, torsion and H-bond counts per cluster equal those of the one-launch-per-
    stage path evaluating the same cluster (same thresholds, other enumeration)."""
    import torch
    pos, typ, q, off = concat(small_batch)
    f, e, counts, rc, bad = run_batch(ff, pos, typ, q, off)
    for c, s in enumerate(small_batch):
        if s.pos.shape[0] < 2:
            assert (counts[c, :3] == 0).all()
            continue
        P, T, Q = to_dev(s.pos, s.type, s.q)
        ff.build_lists(P, T, None)
        ff.compute_forces(P, T, Q, None)
        torch.cuda.synchronize()
        ic = ff.interaction_counts()
        assert (counts[c, 0], counts[c, 1], counts[c, 2]) == (ic["angles"], ic["torsions"], ic["hbonds"]), c


@pytest.fixture(scope="module")
def full_batch(ff):
    """The 4,096-cluster batch (sizes uniform in 10-300, seed 3) with the autotuned
    configuration."""
    import torch
    from paper_1706_07772_amd import Batch
    pos, typ, q, off = rs.cluster_batch(4096, seed=3)
    b = Batch(ff, off)
    P, T, Q = to_dev(pos, typ, q)
    trials = b.tune(P, T, Q, reps=2)
    print("tuner trials", len(trials), "best", b.config, flush=True)
    f, e = b.compute(P, T, Q)
    rc, bad = b.status()
    torch.cuda.synchronize()
    out = dict(pos=pos, typ=typ, q=q, off=off, f=f.cpu().numpy(), e=e.cpu().numpy(), counts=b.counts(),
               rc=rc, bad=bad, trials=trials, config=b.config)
    b.close()
    return out


def test_full_batch_status_and_tuner(full_batch):
    fb = full_batch
    assert fb["rc"] == 0 and fb["bad"] == -1
    assert np.isfinite(fb["e"]).all() and np.isfinite(fb["f"]).all()
    assert len(fb["trials"]) == 48
    best = min(fb["trials"], key=lambda t: t[1])
    assert tuple(fb["config"]) == tuple(best[0])


@pytest.mark.parametrize("k", range(6))
def test_full_batch_sampled_clusters(full_batch, params, k):
    fb = full_batch
    off = fb["off"]
    sizes = np.diff(off)
    rng = np.random.default_rng(300 + k)
    picks = [int(sizes.argmax()), int(sizes.argmin())] + [int(x) for x in rng.integers(0, sizes.size, 4)]
    c = picks[k]
    s = rs.System(pos=fb["pos"][off[c]:off[c + 1]], type=fb["typ"][off[c]:off[c + 1]],
                  q=fb["q"][off[c]:off[c + 1]], box=None)
    check_cluster(c, s, params, fb["f"][off[c]:off[c + 1]], fb["e"], fb["counts"])


def test_full_batch_vs_plain_packed(ff, full_batch):
    """The same 4,096 clusters placed 40 A apart on a grid in one non-periodic system and
    evaluated by the plain path: total energies per term and every force agree."""
    import torch
    fb = full_batch
    off = fb["off"]
    nc = off.size - 1
    side = int(np.ceil(nc ** (1.0 / 3.0)))
    pos = fb["pos"].copy()
    for c in range(nc):
        g = np.array(np.unravel_index(c, (side, side, side)), dtype=np.float64)
        pos[off[c]:off[c + 1]] += 40.0 * g
    P, T, Q = to_dev(pos, fb["typ"], fb["q"])
    ff.build_lists(P, T, None)
    f, e = ff.compute_forces(P, T, Q, None)
    torch.cuda.synchronize()
    e = e.cpu().numpy()
    f = f.cpu().numpy()
    eb = fb["e"].sum(0)
    scale = np.abs(fb["e"]).sum(0)
    assert np.all(np.abs(eb - e) <= 1e-9 * np.maximum(scale, 1e-300)), (eb, e)
    assert_force_parity(fb["f"], f)
    ic = ff.interaction_counts()
    tot = fb["counts"].sum(0)
    assert (tot[0], tot[1], tot[2], tot[3], tot[4]) == (ic["angles"], ic["torsions"], ic["hbonds"],
                                                         ic["far_pairs"], ic["bonds"])


def test_batch_bad_type_reported(ff, params, small_batch, small_refs):
    import torch
    from paper_1706_07772_amd import Batch
    pos, typ, q, off = concat(small_batch)
    typ = typ.copy()
    c_bad = 5
    typ[off[c_bad] + 1] = 7
    b = Batch(ff, off)
    P, T, Q = to_dev(pos, typ, q)
    f, e = b.compute(P, T, Q)
    rc, bad = b.status()
    torch.cuda.synchronize()
    f, e, counts = f.cpu().numpy(), e.cpu().numpy(), b.counts()
    b.close()
    assert rc == -1 and bad == c_bad
    assert np.isnan(e[c_bad]).all() and np.isnan(f[off[c_bad]:off[c_bad + 1]]).all()
    for c, s in enumerate(small_batch):
        if c != c_bad:
            check_cluster(c, s, params, f[off[c]:off[c + 1]], e, counts, small_refs[c])


def test_batch_capacity_grows(ff, params):
    """A tightly packed cluster (every pair bonded) overflows the default scratch slice:
    the status reports it, and the next compute grows the slices and succeeds."""
    import torch
    from paper_1706_07772_amd import Batch
    rng = np.random.default_rng(21)
    dense = rs.System(pos=rng.uniform(0.0, 2.2, size=(24, 3)), type=rng.integers(0, 4, 24).astype(np.int32),
                      q=np.zeros(24), box=None)
    systems = [rs.cluster(30, seed=22), dense, rs.cluster(24, seed=23)]
    pos, typ, q, off = concat(systems)
    b = Batch(ff, off)
    P, T, Q = to_dev(pos, typ, q)
    f, e = b.compute(P, T, Q)
    rc, bad = b.status()
    assert rc == -2 and bad == 1
    f, e = b.compute(P, T, Q)
    rc2, bad2 = b.status()
    torch.cuda.synchronize()
    f, e, counts = f.cpu().numpy(), e.cpu().numpy(), b.counts()
    b.close()
    assert rc2 == 0 and bad2 == -1
    for c, s in enumerate(systems):
        check_cluster(c, s, params, f[off[c]:off[c + 1]], e, counts)


def test_batch_recapture_on_new_buffers(ff, params, small_batch, small_refs):
    """New output buffers (a different graph) give the same results; so does a replay."""
    import torch
    from paper_1706_07772_amd import Batch
    pos, typ, q, off = concat(small_batch)
    b = Batch(ff, off)
    P, T, Q = to_dev(pos, typ, q)
    f1, e1 = b.compute(P, T, Q)
    f1, e1 = f1.clone(), e1.clone()
    f2, e2 = b.compute(P, T, Q)           # replay of the same graph
    f3, e3 = b.compute(P, T, Q, forces=torch.empty_like(f1), energies=torch.empty_like(e1))
    rc, _ = b.status()
    torch.cuda.synchronize()
    b.close()
    assert rc == 0
    for a, c in ((f1, f2), (f1, f3), (e1, e2), (e1, e3)):
        d = (a - c).abs().max().item() if a.numel() else 0.0
        assert d <= 1e-9 * max(a.abs().max().item(), 1.0)


def test_batch_rejects_oversized_cluster(ff):
    from paper_1706_07772_amd import Batch, ReaxFFError
    off = np.array([0, 10, 10 + 385], dtype=np.int64)
    with pytest.raises(ReaxFFError):
        Batch(ff, off)
