"""Training and evaluation driver of the learned surrogate.

Reference energies and forces come from this library's plain FP64 ReaxFF
evaluation on the GPU; the surrogate's training steps, descriptors and
networks run in its own kernels (reaxff_surrogate_*).  Frames follow the
lattice recipe of the benchmark workloads with the jitter amplitude scaled
by temperature (reaxff_synth.thermal_frame); seeds and temperatures are
drawn from a seeded generator.
"""
from __future__ import annotations

import math
import time

import numpy as np
import torch

import reaxff_synth as rs

from .binding import NDESC, ReaxFF, Surrogate

KCAL_PER_EV = 23.060548


def init_params(members: int, npar: int, seed: int, e_per_atom: float) -> np.ndarray:
    """(members, 4, npar) float32: normal weights scaled by 1/sqrt(fan-in), zero biases,
    output bias e_per_atom."""
    rng = np.random.default_rng(np.random.PCG64(seed))
    th = np.zeros((members, 4, npar), dtype=np.float32)
    nd, h = NDESC, 128
    for m in range(members):
        for e in range(4):
            o = 0
            th[m, e, o:o + nd * h] = rng.normal(size=nd * h) / math.sqrt(nd)
            o += nd * h + h
            th[m, e, o:o + h * h] = rng.normal(size=h * h) / math.sqrt(h)
            o += h * h + h
            th[m, e, o:o + h] = rng.normal(size=h) / math.sqrt(h)
            o += h
            th[m, e, o] = e_per_atom
    return th


class FrameSource:
    """Seeded training / held-out frames: n_units C5H8N4O12 units in a periodic box at
    the crystal density, temperatures uniform in [t_lo, t_hi] K."""

    def __init__(self, n_units: int, seed: int, t_lo: float = 300.0, t_hi: float = 3000.0):
        self.n_units = n_units
        self.box = (n_units * rs.PETN_UNIT_ATOMS / rs.DENSITY) ** (1.0 / 3.0)
        self.rng = np.random.default_rng(np.random.PCG64(seed))
        self.t_lo, self.t_hi = t_lo, t_hi

    def next(self):
        seed = int(self.rng.integers(1 << 30))
        temp = float(self.rng.uniform(self.t_lo, self.t_hi))
        return rs.thermal_frame(self.n_units, self.box, seed, temp), temp


def to_device(system, device="cuda:0"):
    d = torch.device(device)
    return (torch.tensor(system.pos, dtype=torch.float64, device=d).contiguous(),
            torch.tensor(system.type, dtype=torch.int32, device=d).contiguous(),
            torch.tensor(system.q, dtype=torch.float64, device=d).contiguous(),
            None if system.box is None else [float(x) for x in system.box])


def label(ff: ReaxFF, dev_frame):
    """Plain FP64 ReaxFF energy (total) and forces of a device frame."""
    pos, typ, q, box = dev_frame
    ff.build_lists(pos, typ, box)
    f, e = ff.compute_forces(pos, typ, q, box)
    return float(e.sum().item()), f


def fit_normaliser(sur: Surrogate, dev_frames):
    """Per-feature mean and 1/max(std, 1e-3) of the descriptors of the given frames
    (reaxff_surrogate_normaliser over their rows)."""
    G = torch.cat([sur.descriptors(pos, typ, box) for pos, typ, q, box in dev_frames]).contiguous()
    return sur.normaliser(G, 1e-3)


def train(sur: Surrogate, ff: ReaxFF, source: FrameSource, steps: int, nframes: int, lr: float = 1e-3,
          lr_end: float = 1e-4, wE: float = 1.0, wF: float = 1.0, seed: int = 0, log=None):
    """Label nframes frames with the plain path, fit the normaliser, initialise the
    members and take `steps` Adam steps cycling over the frames (cosine-decayed learning
    rate).  Returns a dict of losses and timings."""
    t0 = time.perf_counter()
    frames = []
    for _ in range(nframes):
        sysf, temp = source.next()
        d = to_device(sysf)
        E, F = label(ff, d)
        frames.append((d, E, F.clone(), temp))
    torch.cuda.synchronize()
    t_label = time.perf_counter() - t0
    shift, scale = fit_normaliser(sur, [f[0] for f in frames[:8]])
    e_atom = float(np.mean([f[1] / f[0][0].shape[0] for f in frames]))
    sur.set_params(init_params(sur.members, sur.npar, seed, e_atom), shift, scale)
    losses = []
    t1 = time.perf_counter()
    for it in range(steps):
        (pos, typ, q, box), E, F, temp = frames[it % nframes]
        c = 0.5 * (1.0 + math.cos(math.pi * it / max(steps - 1, 1)))
        rate = lr_end + (lr - lr_end) * c
        loss = sur.train_step(pos, typ, box, E, F, wE, wF, rate)
        if it % 25 == 0 or it == steps - 1:
            lv = loss.cpu().numpy()
            losses.append((it, lv.tolist()))
            if log:
                log(f"train step {it}: loss {np.round(lv, 3).tolist()} lr {rate:.2e}")
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    return dict(losses=losses, label_s=t_label, train_s=t_train, steps=steps, frames=nframes,
                atoms_per_frame=int(frames[0][0][0].shape[0]), ms_per_step=1e3 * t_train / max(steps, 1))


def train_streamed(sur: Surrogate, ff: ReaxFF, source: FrameSource, nframes: int, lr: float = 2e-3,
                   lr_end: float = 1e-4, wE: float = 1.0, wF: float = 1.0, seed: int = 0,
                   norm_frames: int = 8, log=None, log_every: int = 1000):
    """One Adam step per fresh frame: `nframes` frames drawn from `source`, each labelled
    by the plain FP64 path on the GPU as it arrives and used once (nothing stored), with
    a cosine-decayed learning rate.  The normaliser is fitted on the first norm_frames
    frames.  Returns a dict of losses (every log_every steps) and timings."""
    t0 = time.perf_counter()
    first = []
    for _ in range(norm_frames):
        sysf, temp = source.next()
        d = to_device(sysf)
        first.append((d, label(ff, d), temp))
    shift, scale = fit_normaliser(sur, [f[0] for f in first])
    e_atom = float(np.mean([f[1][0] / f[0][0].shape[0] for f in first]))
    sur.set_params(init_params(sur.members, sur.npar, seed, e_atom), shift, scale)
    losses = []
    t_label = 0.0
    t1 = time.perf_counter()
    for it in range(nframes):
        if it < norm_frames:
            (pos, typ, q, box), (E, F), temp = first[it]
        else:
            tl = time.perf_counter()
            sysf, temp = source.next()
            pos, typ, q, box = to_device(sysf)
            E, F = label(ff, (pos, typ, q, box))
            t_label += time.perf_counter() - tl
        c = 0.5 * (1.0 + math.cos(math.pi * it / max(nframes - 1, 1)))
        rate = lr_end + (lr - lr_end) * c
        loss = sur.train_step(pos, typ, box, E, F, wE, wF, rate)
        if it % log_every == 0 or it == nframes - 1:
            lv = loss.cpu().numpy()
            losses.append((it, lv.tolist()))
            if log:
                log(f"streamed step {it}: loss {np.round(lv, 3).tolist()} lr {rate:.2e}")
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    return dict(losses=losses, frames=nframes, atoms_per_frame=int(first[0][0][0].shape[0]),
                seconds=total, label_and_generate_s=t_label, ms_per_frame=1e3 * (time.perf_counter() - t1) / nframes)


def evaluate(sur: Surrogate, ff: ReaxFF, dev_frame, threshold_ev: float = 0.1):
    """Force errors against the plain FP64 forces (eV/A): the ensemble mean, the gated
    forces, and the fallback fraction at the given spread threshold."""
    pos, typ, q, box = dev_frame
    E, Fr = label(ff, dev_frame)
    out = sur.evaluate(pos, typ, box)
    Fg, mask, Es, nf = sur.gated_forces(ff, pos, typ, q, box, threshold_ev * KCAL_PER_EV)
    torch.cuda.synchronize()
    n = pos.shape[0]

    def rmse(a):
        return float(torch.sqrt(((a.double() - Fr) ** 2).sum(1).mean()).item()) / KCAL_PER_EV

    return dict(rmse_mean_ev=rmse(out["fmean"]), rmse_gated_ev=rmse(Fg),
                rmse_zero_ev=float(torch.sqrt((Fr ** 2).sum(1).mean()).item()) / KCAL_PER_EV,
                fallback_fraction=nf / n,
                sigma_median_ev=float(out["sigma"].median().item()) / KCAL_PER_EV,
                energy_err_per_atom_ev=abs(float(out["energies"].mean().item()) - E) / n / KCAL_PER_EV)
