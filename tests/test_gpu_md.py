"""reaxff_step (velocity-Verlet NVE, lists rebuilt every step) on the GPU.

Against the oracle's own integrator on a small box for a few steps, then the
32,480-atom box at 300 K for 100 steps of 0.1 fs: bounded energy fluctuation,
momentum conservation, and the dt^2 law of the shadow-energy fluctuation on a
smooth variant of the model (interaction thresholds at zero).
"""
import numpy as np
import pytest

import reaxff_synth as rs
from oracle import Oracle

from _common import to_dev

pytestmark = pytest.mark.gpu

SMOOTH = dict(rs.DEFAULT_CUTOFFS, bo_cut=1e-10, thb_cut=0.0, thb_cutsq=0.0, hb_bo_cut=0.0)


@pytest.fixture(scope="module")
def params():
    return rs.draw_params(0)


def run_gpu(params, s, vel, dt, nsteps, cutoffs=None):
    import torch
    from paper_1706_07772_amd import ReaxFF
    ff = ReaxFF(params, cutoffs)
    pos, typ, q, box = to_dev(s)
    v = torch.tensor(vel, dtype=torch.float64, device=pos.device)
    f, e = ff.step(pos, v, typ, q, box, dt, nsteps)
    torch.cuda.synchronize()
    out = pos.cpu().numpy(), v.cpu().numpy(), f.cpu().numpy(), e.cpu().numpy()
    ff.close()
    return out


def test_trajectory_matches_oracle(params):
    """Ten steps on an 870-atom periodic box: positions, velocities and per-step energies
    agree with the oracle's velocity-Verlet run."""
    s = rs.small_periodic(30, seed=21)
    v0 = rs.maxwell_boltzmann(s.type, params.atom["mass"], 300.0, seed=121)
    pos, vel, f, e = run_gpu(params, s, v0, 0.1, 10)
    o = Oracle(s, params)
    pos_r, vel_r, e_r = o.md(v0, 0.1, 10)
    assert np.abs(pos - pos_r).max() <= 1e-9
    assert np.abs(vel - vel_r).max() <= 1e-9 * np.abs(vel_r).max()
    assert np.allclose(e, e_r, rtol=1e-8, atol=1e-8 * np.abs(e_r).max())


def test_trajectory_32480_matches_oracle(params):
    """Ten steps on the 32,480-atom box at 300 K: positions, velocities and every
    step's energies against the oracle's velocity-Verlet run at 1e-8."""
    s = rs.workload("petn_32480")
    v0 = rs.maxwell_boltzmann(s.type, params.atom["mass"], 300.0, seed=101)
    pos, vel, f, e = run_gpu(params, s, v0, 0.1, 10)
    print("oracle MD, 32,480 atoms, 10 steps", flush=True)
    pos_r, vel_r, e_r = Oracle(s, params).md(v0, 0.1, 10)
    assert np.abs(pos - pos_r).max() <= 1e-8
    assert np.abs(vel - vel_r).max() <= 1e-8 * np.abs(vel_r).max()
    assert np.allclose(e, e_r, rtol=1e-8, atol=1e-8 * np.abs(e_r).max())


def test_nve_32480(params):
    """100 steps of 0.1 fs on the 32,480-atom box at 300 K (lists rebuilt every step)."""
    s = rs.workload("petn_32480")
    m = params.atom["mass"][s.type]
    v0 = rs.maxwell_boltzmann(s.type, params.atom["mass"], 300.0, seed=101)
    pos, vel, f, e = run_gpu(params, s, v0, 0.1, 100)
    tot = e.sum(1)
    ke0 = e[0, -1]
    print("E0", tot[0], "KE0", ke0, "span", tot.max() - tot.min(), flush=True)
    assert np.isfinite(e).all()
    # momentum: zero initially, conserved by the pairwise-balanced forces
    assert np.abs((m[:, None] * vel).sum(0)).max() < 1e-8 * np.abs(m[:, None] * vel).sum()
    # the model's hard interaction thresholds make E jump when an interaction enters or
    # leaves; even so the total energy stays within a small fraction of the kinetic energy
    assert tot.max() - tot.min() < 0.05 * ke0


def test_nve_dt_squared_smooth(params):
    """With the interaction thresholds at zero the energy is nearly smooth and the
    total-energy fluctuation over a fixed time shrinks ~4x when dt is halved.  (A bond
    entering the list still switches on a small coalition term, whose jumps add up over
    large boxes; a 40-atom cluster over 4 fs sees few such events.)"""
    s = rs.cluster(40, seed=8)
    v0 = rs.maxwell_boltzmann(s.type, params.atom["mass"], 300.0, seed=108)
    spans = []
    for dt, steps in ((0.1, 40), (0.05, 80)):
        _, _, _, e = run_gpu(params, s, v0, dt, steps, SMOOTH)
        tot = e.sum(1)
        spans.append(tot.max() - tot.min())
    ratio = spans[0] / spans[1]
    assert 3.0 < ratio < 5.0, (spans, ratio)
