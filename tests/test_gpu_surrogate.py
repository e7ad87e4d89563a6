"""Learned surrogate on the GPU against the FP64 surrogate oracle.

Descriptors (FP32 kernels, factorised moment form) against the oracle's
literal double sums.  Network energies and forces, and the training
gradient, against the oracle run with the same BF16 rounding points as the
kernels (oracle.surrogate's quantiser), on parameters and normalisation
rounded to FP32 once and given to both sides.  Remaining differences: FP32
against FP64 arithmetic, and the rare BF16 rounding that an FP32-level
difference in its input moves across a rounding boundary (about 2^8 x 1e-6
per value); the tolerances below are set from that.  Then: training lowers
the loss; the gate takes the plain FP64 forces exactly where the members
disagree.
"""
import numpy as np
import pytest

import reaxff_synth as rs
from oracle import surrogate as S

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


def dev(system):
    import torch
    d = torch.device("cuda:0")
    return (torch.tensor(system.pos, dtype=torch.float64, device=d).contiguous(),
            torch.tensor(system.type, dtype=torch.int32, device=d).contiguous(),
            torch.tensor(system.q, dtype=torch.float64, device=d).contiguous(),
            None if system.box is None else [float(x) for x in system.box])


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


FRAMES = {
    "periodic_870": lambda: rs.small_periodic(30, seed=21),
    "cluster_150": lambda: rs.cluster(150, seed=31),
}


@pytest.fixture(scope="module", params=sorted(FRAMES))
def frame(request):
    s = FRAMES[request.param]()
    G = S.descriptors(s.pos, s.type, s.box)
    shift, scale = S.normaliser(G)
    return request.param, s, G, f32(shift), f32(scale)


@pytest.fixture(scope="module")
def sur4(ff):
    from paper_1706_07772_amd import Surrogate
    s = Surrogate(ff, 4)
    yield s
    s.close()


def test_descriptors_match_definition(sur4, frame):
    import torch
    name, s, G, shift, scale = frame
    pos, typ, q, box = dev(s)
    Gg = sur4.descriptors(pos, typ, box)
    torch.cuda.synchronize()
    Gg = Gg.cpu().numpy().astype(np.float64)
    colmax = np.abs(G).max(0)
    tol = 3e-5 * (np.abs(G) + 1e-2 * colmax[None, :]) + 1e-7
    bad = np.abs(Gg - G) > tol
    assert not bad.any(), (name, np.argwhere(bad)[:5], np.abs(Gg - G).max())


def _oracle_members(th, shift, scale, s, G, q=S.bf16):
    E, F = [], []
    nb = S.neighbours(s.pos, s.box)
    for m in range(th.shape[0]):
        Ea, Fm, _ = S.model_energy_forces(th[m], shift, scale, s.pos, s.type, s.box, q, nb, G)
        E.append(Ea)
        F.append(Fm)
    return np.array(E), np.array(F)


def test_network_energies_forces(sur4, frame):
    import torch
    name, s, G, shift, scale = frame
    th = f32(S.init_params(4, seed=7, e_per_atom=-0.5))
    sur4.set_params(th, shift, scale)
    pos, typ, q, box = dev(s)
    out = sur4.evaluate(pos, typ, box)
    torch.cuda.synchronize()
    Ea_g = out["eatom"].cpu().numpy().astype(np.float64)
    F_g = out["forces"].cpu().numpy().astype(np.float64)
    E_g = out["energies"].cpu().numpy()
    Ea_r, F_r = _oracle_members(th, shift, scale, s, G)
    eerr = np.abs(Ea_g - Ea_r).max()
    escale = max(np.abs(Ea_r).max(), 1.0)
    ferr = np.linalg.norm(F_g - F_r, axis=2)
    fscale = np.linalg.norm(F_r, axis=2).max()
    frms = np.sqrt((ferr ** 2).mean()) / np.sqrt((np.linalg.norm(F_r, axis=2) ** 2).mean())
    print(name, "energy max err", eerr / escale, "force max err", ferr.max() / fscale, "force rms rel", frms)
    assert eerr <= 2e-3 * escale
    np.testing.assert_allclose(E_g, Ea_r.sum(1), rtol=0, atol=2e-3 * escale * np.sqrt(s.n) + 1e-6)
    assert ferr.max() <= 1e-2 * fscale
    assert frms <= 2e-3
    # ensemble mean and spread from the members
    Fm = out["fmean"].cpu().numpy()
    sig = out["sigma"].cpu().numpy()
    np.testing.assert_allclose(Fm, F_g.mean(0), rtol=1e-5, atol=1e-5 * fscale)
    sig_ref = np.sqrt(((F_g - F_g.mean(0)[None]) ** 2).sum(2).mean(0))
    np.testing.assert_allclose(sig, sig_ref, rtol=1e-4, atol=1e-5 * fscale)


def test_network_net_force_zero(sur4, frame):
    """Any energy of pair displacements has zero net force (FP32 sums)."""
    import torch
    name, s, G, shift, scale = frame
    sur4.set_params(f32(S.init_params(4, seed=8, e_per_atom=-0.5)), shift, scale)
    pos, typ, q, box = dev(s)
    F = sur4.evaluate(pos, typ, box)["forces"]
    torch.cuda.synchronize()
    F = F.cpu().numpy().astype(np.float64)
    for m in range(4):
        assert np.abs(F[m].sum(0)).max() <= 1e-5 * np.abs(F[m]).max() * np.sqrt(s.n)


def test_training_gradient(ff, params):
    """Loss and its forward-over-reverse parameter gradient (lr = 0) against the oracle
    with the kernels' BF16 rounding points, two members, on ReaxFF reference data."""
    import torch
    from paper_1706_07772_amd import Surrogate
    s = rs.cluster(150, seed=31)
    from oracle import Oracle
    o = Oracle(s, params)
    Eref_terms, Fref = o.forces()
    Eref = float(Eref_terms.sum())
    G = S.descriptors(s.pos, s.type, s.box)
    shift, scale = (f32(x) for x in S.normaliser(G))
    th = f32(S.init_params(2, seed=9, e_per_atom=Eref / s.n))
    sur = Surrogate(ff, 2)
    sur.set_params(th, shift, scale)
    pos, typ, q, box = dev(s)
    fref = torch.tensor(Fref, dtype=torch.float64, device=pos.device)
    wE, wF = 1.0, 1.0
    loss = sur.train_step(pos, typ, box, Eref, fref, wE, wF, lr=0.0)
    torch.cuda.synchronize()
    loss = loss.cpu().numpy()
    grad = sur.get_grad().astype(np.float64)
    sur.close()
    for m in range(2):
        L_r, g_r = S.loss_grad(th[m], shift, scale, s.pos, s.type, s.box, Eref, Fref, wE, wF, q=S.bf16)
        print("member", m, "loss", loss[m], L_r)
        assert abs(loss[m] - L_r) <= 2e-3 * abs(L_r)
        sizes = [S.NDESC * S.H, S.H, S.H * S.H, S.H, S.H, 1]
        names = ["W1", "b1", "W2", "b2", "w3", "b3"]
        for e in range(4):
            if not (s.type == e).any():
                assert np.all(grad[m, e] == 0)
                continue
            o0 = 0
            for nm, sz in zip(names, sizes):
                a, b = grad[m, e, o0:o0 + sz], g_r[e, o0:o0 + sz]
                o0 += sz
                rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
                print(m, e, nm, "rel", rel)
                assert rel <= 2e-2, (m, e, nm, rel)


def test_training_lowers_loss(ff, params):
    import torch
    from paper_1706_07772_amd import Surrogate
    from oracle import Oracle
    s = rs.cluster(120, seed=41)
    Et, Fref = Oracle(s, params).forces()
    Eref = float(Et.sum())
    G = S.descriptors(s.pos, s.type, s.box)
    shift, scale = (f32(x) for x in S.normaliser(G))
    sur = Surrogate(ff, 2)
    sur.set_params(f32(S.init_params(2, seed=10, e_per_atom=Eref / s.n)), shift, scale)
    pos, typ, q, box = dev(s)
    fref = torch.tensor(Fref, dtype=torch.float64, device=pos.device)
    losses = []
    for it in range(60):
        losses.append(sur.train_step(pos, typ, box, Eref, fref, 1.0, 1.0, lr=2e-3).cpu().numpy())
    sur.close()
    losses = np.array(losses)
    print("loss", losses[0], losses[-1])
    assert np.all(np.isfinite(losses))
    assert np.all(losses[-1] < 0.5 * losses[0])


def test_gate_and_fallback(ff, sur4, params):
    import torch
    s = rs.small_periodic(30, seed=21)
    G = S.descriptors(s.pos, s.type, s.box)
    shift, scale = (f32(x) for x in S.normaliser(G))
    sur4.set_params(f32(S.init_params(4, seed=12, e_per_atom=-0.5)), shift, scale)
    pos, typ, q, box = dev(s)
    ev = sur4.evaluate(pos, typ, box)
    ff.build_lists(pos, typ, box)
    f_plain, _ = ff.compute_forces(pos, typ, q, box)
    torch.cuda.synchronize()
    f_plain = f_plain.cpu().numpy()
    fmean = ev["fmean"].cpu().numpy()
    sigma = ev["sigma"].cpu().numpy()
    # every atom flagged: the plain forces (a second plain evaluation: its FP64
    # atomic sums may round differently in the last bits)
    fsc = np.abs(f_plain).max()
    F, mask, E, nf = sur4.gated_forces(ff, pos, typ, q, box, threshold=-1.0)
    torch.cuda.synchronize()
    assert nf == s.n and mask.cpu().numpy().all() and sur4.last_nsub == s.n
    np.testing.assert_allclose(F.cpu().numpy(), f_plain, rtol=0, atol=1e-12 * fsc)
    # none flagged: the ensemble mean (FP32 atomic sums: equal to rounding)
    F, mask, E, nf = sur4.gated_forces(ff, pos, typ, q, box, threshold=1e30)
    torch.cuda.synchronize()
    assert nf == 0 and not mask.cpu().numpy().any()
    np.testing.assert_allclose(F.cpu().numpy(), fmean, rtol=1e-4, atol=1e-5 * np.abs(fmean).max())
    # threshold at the median spread: plain forces exactly where flagged
    thr = float(np.median(sigma))
    F, mask, E, nf = sur4.gated_forces(ff, pos, typ, q, box, threshold=thr)
    torch.cuda.synchronize()
    F, mask = F.cpu().numpy(), mask.cpu().numpy().astype(bool)
    assert nf == mask.sum() and 0 < nf < s.n
    clear = np.abs(sigma - thr) > 1e-3 * thr
    assert np.array_equal(mask[clear], (sigma > thr)[clear])
    np.testing.assert_allclose(F[mask], f_plain[mask], rtol=0, atol=1e-12 * fsc)
    np.testing.assert_allclose(F[~mask], fmean[~mask], rtol=1e-4, atol=1e-5 * np.abs(fmean).max())


def test_empty_frame(sur4):
    import torch
    pos = torch.zeros((0, 3), dtype=torch.float64, device="cuda")
    typ = torch.zeros(0, dtype=torch.int32, device="cuda")
    out = sur4.evaluate(pos, typ, None)
    torch.cuda.synchronize()
    assert np.all(out["energies"].cpu().numpy() == 0)


def test_training_gains_over_untrained(ff, params):
    """What training buys: on held-out frames the trained ensemble's mean force is closer
    to the oracle's FP64 ReaxFF forces than the untrained ensemble's and than zero."""
    import torch
    from oracle import Oracle
    from paper_1706_07772_amd import Surrogate
    from paper_1706_07772_amd import training as T
    sur = Surrogate(ff, 2)
    T.train(sur, ff, T.FrameSource(64, seed=1000), steps=150, nframes=24, lr=2e-3, seed=3)
    th_trained = sur.get_params()
    held = T.FrameSource(64, seed=99)
    frames = [held.next()[0] for _ in range(2)]
    refs = [Oracle(f, params).forces()[1] for f in frames]

    def rmse_all():
        out = []
        for f, fr in zip(frames, refs):
            pos, typ, q, box = T.to_device(f)
            fm = sur.evaluate(pos, typ, box)["fmean"]
            torch.cuda.synchronize()
            out.append(np.sqrt(((fm.cpu().numpy() - fr) ** 2).sum(1).mean()))
        return np.array(out)

    trained = rmse_all()
    theta, shift, scale = th_trained
    sur.set_params(T.init_params(2, sur.npar, 3, float(theta[0, 0, -1])), shift, scale)
    untrained = rmse_all()
    sur.close()
    zero = np.array([np.sqrt((fr ** 2).sum(1).mean()) for fr in refs])
    print("rmse kcal/mol/A trained", trained, "untrained", untrained, "zero", zero)
    assert np.all(trained < 0.7 * zero)
    assert np.all(trained < 0.7 * untrained)


def test_fullsize_sampled_atoms(ff):
    """The 1,044,000-atom evaluation at sampled atoms: member forces against the
    oracle on the atoms within 10.5 A of each (a force depends on descriptors
    of atoms within 5 A, which see atoms within 5 A more), non-periodic."""
    import torch
    from _common import extract_subsystem
    from paper_1706_07772_amd import Surrogate
    s = rs.workload("petn_1044000")
    probe = rs.small_periodic(30, seed=21)
    G0 = S.descriptors(probe.pos, probe.type, probe.box)
    shift, scale = (f32(x) for x in S.normaliser(G0))
    th = f32(S.init_params(2, seed=9, e_per_atom=-0.5))
    sur = Surrogate(ff, 2)
    try:
        sur.set_params(th, shift, scale)
        pos, typ, q, box = dev(s)
        out = sur.evaluate(pos, typ, box)
        torch.cuda.synchronize()
        F = out["forces"].cpu().numpy().astype(np.float64)
    finally:
        sur.close()
    fscale = np.linalg.norm(F, axis=2).max()
    rng = np.random.default_rng(77)
    for c in rng.choice(s.n, size=4, replace=False):
        sub, ci, ids = extract_subsystem(s, int(c), 10.5)
        Gs = S.descriptors(sub.pos, sub.type, None)
        _, F_r = _oracle_members(th, shift, scale, sub, Gs)
        err = np.linalg.norm(F[:, c] - F_r[:, ci], axis=1).max()
        print("sampled atom", int(c), "neighbourhood", sub.n, "err", err / fscale, flush=True)
        assert err <= 1e-2 * fscale


def test_normaliser_matches_definition(sur4):
    """reaxff_surrogate_normaliser against the mean and population deviation of
    the same rows in FP64 (the oracle's normaliser)."""
    import torch
    frames = [rs.small_periodic(30, seed=21), rs.cluster(150, seed=31)]
    Gs = [sur4.descriptors(*dev(f)[:2], dev(f)[3]) for f in frames]
    G = torch.cat(Gs).contiguous()
    shift, scale = sur4.normaliser(G, 1e-3)
    ref_shift, ref_scale = S.normaliser(G.cpu().numpy().astype(np.float64))
    np.testing.assert_allclose(shift, ref_shift, rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(scale, ref_scale, rtol=1e-6)


def test_streamed_training_lowers_loss(ff):
    """One Adam step per fresh frame, labelled by the plain path as it arrives: the
    loss over the last frames is below the loss over the first."""
    from paper_1706_07772_amd import Surrogate
    from paper_1706_07772_amd import training as T
    sur = Surrogate(ff, 2)
    try:
        info = T.train_streamed(sur, ff, T.FrameSource(64, seed=2000), nframes=400, lr=2e-3, log_every=50)
    finally:
        sur.close()
    first = np.mean(info["losses"][0][1])
    last = np.mean([np.mean(l) for _, l in info["losses"][-3:]])
    print("streamed loss", first, "->", last, "ms per frame", info["ms_per_frame"], flush=True)
    assert info["frames"] == 400 and last < 0.5 * first
