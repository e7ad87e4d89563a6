"""Pins of the surrogate oracle (CPU).

The descriptor's literal double sum against the factorised moment-tensor form
(an identity, not a retyping), closed forms for one and two neighbours,
invariances and cutoff continuity; the term-by-term descriptor derivative
against the complex-step derivative (adjoint identity) and finite
differences; network input gradients, forces and the forward-over-reverse
loss gradient against finite differences; the bf16 quantiser on exact cases;
Adam's first step in closed form.
"""
import numpy as np
import pytest

import reaxff_synth as rs
from oracle import surrogate as S


def small(n=14, seed=4):
    return rs.cluster(n, seed=seed)


def moment_form(pos, types, box):
    """Angular features from per-element moment vectors and tensors:
    sum_{j,k} w cos = M1_b . M1_c,  sum_{j,k} w cos^2 = M2_b : M2_c."""
    nb = S.neighbours(pos, box)
    n = pos.shape[0]
    out = np.zeros((n, S.NDESC - 4 * S.NR))
    for i in range(n):
        sel, d = nb[i]
        if sel.size == 0:
            continue
        r = np.sqrt((d * d).sum(1))
        u = d / r[:, None]
        A = np.exp(-S.ETA_A * (r[:, None] - S.MU_A[None, :]) ** 2) * S.fcut(r)[:, None]
        M1 = np.zeros((4, S.NA, 3))
        M2 = np.zeros((4, S.NA, 3, 3))
        for j in range(sel.size):
            b = types[sel[j]]
            M1[b] += A[j][:, None] * u[j][None, :]
            M2[b] += A[j][:, None, None] * np.outer(u[j], u[j])[None]
        for p, (b, c) in enumerate(S.PAIRS):
            out[i, 16 * p:16 * p + 8] = (M1[b] * M1[c]).sum(1)
            out[i, 16 * p + 8:16 * p + 16] = (M2[b] * M2[c]).sum((1, 2))
    return out


def test_angular_equals_moment_form():
    s = small(20, 5)
    G = S.descriptors(s.pos, s.type, None)
    np.testing.assert_allclose(G[:, 64:], moment_form(s.pos, s.type, None), rtol=1e-12, atol=1e-12)


def test_angular_equals_moment_form_periodic():
    s = rs.small_periodic(12, seed=3)
    sub = np.arange(60)
    G = S.descriptors(s.pos, s.type, s.box)
    np.testing.assert_allclose(G[sub, 64:], moment_form(s.pos, s.type, s.box)[sub], rtol=1e-12, atol=1e-12)


def test_one_neighbour_closed_form():
    r = 2.3
    pos = np.array([[0.0, 0.0, 0.0], [r, 0.0, 0.0]])
    types = np.array([0, 3], np.int32)
    G = S.descriptors(pos, types, None)
    fc = 0.5 * (np.cos(np.pi * r / 5.0) + 1.0)
    R = np.exp(-S.ETA_R * (r - S.MU_R) ** 2) * fc
    A = np.exp(-S.ETA_A * (r - S.MU_A) ** 2) * fc
    # atom 0 sees one O: radial block of O, angular pair (O, O) with cos = 1
    np.testing.assert_allclose(G[0, 48:64], R, rtol=1e-14)
    assert np.all(G[0, :48] == 0)
    p = S.PAIR_INDEX[(3, 3)]
    np.testing.assert_allclose(G[0, 64 + 16 * p:64 + 16 * p + 8], A * A, rtol=1e-14)
    np.testing.assert_allclose(G[0, 64 + 16 * p + 8:64 + 16 * p + 16], A * A, rtol=1e-14)
    others = np.setdiff1d(np.arange(64, 224), np.arange(64 + 16 * p, 64 + 16 * p + 16))
    assert np.all(G[0, others] == 0)


def test_two_neighbours_closed_form():
    """Centre C with an H at r1 and an N at r2 at angle theta: the (H, N) pair gets
    A(r1) A(r2) cos^l theta once (b < c, one ordered pair)."""
    r1, r2, th = 1.9, 2.6, 1.1
    pos = np.array([[0.0, 0.0, 0.0], [r1, 0.0, 0.0], [r2 * np.cos(th), r2 * np.sin(th), 0.0]])
    types = np.array([0, 1, 2], np.int32)
    G = S.descriptors(pos, types, None)
    A1 = np.exp(-S.ETA_A * (r1 - S.MU_A) ** 2) * S.fcut(r1)
    A2 = np.exp(-S.ETA_A * (r2 - S.MU_A) ** 2) * S.fcut(r2)
    p = S.PAIR_INDEX[(1, 2)]
    np.testing.assert_allclose(G[0, 64 + 16 * p:64 + 16 * p + 8], A1 * A2 * np.cos(th), rtol=1e-13)
    np.testing.assert_allclose(G[0, 64 + 16 * p + 8:64 + 16 * p + 16], A1 * A2 * np.cos(th) ** 2, rtol=1e-13)
    np.testing.assert_allclose(G[0, 64 + 16 * S.PAIR_INDEX[(1, 1)]:][:8], A1 * A1, rtol=1e-13)


def test_invariances():
    s = small(16, 6)
    G = S.descriptors(s.pos, s.type, None)
    rng = np.random.default_rng(1)
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    Gr = S.descriptors(s.pos @ Q.T + np.array([3.0, -1.0, 7.5]), s.type, None)
    np.testing.assert_allclose(Gr, G, rtol=1e-11, atol=1e-12)
    perm = rng.permutation(s.n)
    Gp = S.descriptors(s.pos[perm], s.type[perm], None)
    np.testing.assert_allclose(Gp, G[perm], rtol=1e-12, atol=1e-12)


def test_periodic_image_shift():
    s = rs.small_periodic(12, seed=8)
    G = S.descriptors(s.pos, s.type, s.box)
    shift = np.zeros_like(s.pos)
    shift[::3, 0] = s.box[0]
    shift[1::5, 2] = -2 * s.box[2]
    G2 = S.descriptors(s.pos + shift, s.type, s.box)
    np.testing.assert_allclose(G2, G, rtol=1e-11, atol=1e-11)


def test_cutoff_continuity():
    types = np.array([0, 2], np.int32)
    vals = []
    for r in (5.0 - 1e-6, 5.0 + 1e-6):
        G = S.descriptors(np.array([[0.0, 0, 0], [r, 0, 0]]), types, None)
        vals.append(np.abs(G).max())
    assert vals[0] < 1e-10 and vals[1] == 0.0


def test_vjp_adjoint_of_complex_step():
    """sum_i F_i . v_i = -g . (dG/dx v) for random g, v."""
    s = small(14, 7)
    rng = np.random.default_rng(2)
    g = rng.normal(size=(s.n, S.NDESC))
    v = rng.normal(size=(s.n, 3))
    F = S.descriptor_vjp(s.pos, s.type, None, g)
    J = S.descriptor_jvp(s.pos, s.type, None, v)
    lhs = (F * v).sum()
    rhs = -(g * J).sum()
    assert abs(lhs - rhs) <= 1e-11 * max(abs(rhs), 1.0), (lhs, rhs)


def test_jvp_finite_difference():
    s = small(12, 9)
    rng = np.random.default_rng(3)
    v = rng.normal(size=(s.n, 3))
    h = 1e-5
    fd = (S.descriptors(s.pos + h * v, s.type, None) - S.descriptors(s.pos - h * v, s.type, None)) / (2 * h)
    J = S.descriptor_jvp(s.pos, s.type, None, v)
    np.testing.assert_allclose(J, fd, rtol=1e-6, atol=1e-7)


@pytest.fixture(scope="module")
def model():
    s = small(14, 10)
    G = S.descriptors(s.pos, s.type, None)
    shift, scale = S.normaliser(G)
    th = S.init_params(2, seed=5, e_per_atom=-1.0)
    return s, shift, scale, th


def test_net_input_grad_fd(model):
    s, shift, scale, th = model
    rng = np.random.default_rng(4)
    x = rng.normal(size=(5, S.NDESC))
    E, c = S.net_forward(th[0, 0], x)
    gx = S.net_input_grad(th[0, 0], c)
    d = rng.normal(size=x.shape)
    h = 1e-6
    fd = (S.net_forward(th[0, 0], x + h * d)[0] - S.net_forward(th[0, 0], x - h * d)[0]) / (2 * h)
    np.testing.assert_allclose((gx * d).sum(1), fd, rtol=1e-7, atol=1e-9)


def test_model_forces_fd(model):
    s, shift, scale, th = model
    Ea, F, _ = S.model_energy_forces(th[0], shift, scale, s.pos, s.type, None)
    rng = np.random.default_rng(6)
    v = rng.normal(size=s.pos.shape)
    h = 1e-6
    Ep = S.model_energy_forces(th[0], shift, scale, s.pos + h * v, s.type, None)[0].sum()
    Em = S.model_energy_forces(th[0], shift, scale, s.pos - h * v, s.type, None)[0].sum()
    fd = (Ep - Em) / (2 * h)
    assert abs(-(F * v).sum() - fd) <= 1e-6 * max(abs(fd), 1.0), (-(F * v).sum(), fd)
    # Newton's third law holds for any pair descriptor energy: zero net force
    assert np.abs(F.sum(0)).max() <= 1e-10 * np.abs(F).max()


def test_loss_grad_fd(model):
    """The forward-over-reverse gradient of the energy + force loss against central
    differences along random parameter directions."""
    s, shift, scale, th = model
    Fref = np.random.default_rng(8).normal(size=s.pos.shape) * 5.0
    Eref = -20.0
    L, g = S.loss_grad(th[0], shift, scale, s.pos, s.type, None, Eref, Fref, 1.0, 1.0)
    assert L == pytest.approx(S.loss(th[0], shift, scale, s.pos, s.type, None, Eref, Fref, 1.0, 1.0), rel=1e-13)
    rng = np.random.default_rng(9)
    for trial in range(3):
        d = rng.normal(size=th[0].shape)
        h = 1e-6
        Lp = S.loss(th[0] + h * d, shift, scale, s.pos, s.type, None, Eref, Fref, 1.0, 1.0)
        Lm = S.loss(th[0] - h * d, shift, scale, s.pos, s.type, None, Eref, Fref, 1.0, 1.0)
        fd = (Lp - Lm) / (2 * h)
        an = (g * d).sum()
        assert abs(an - fd) <= 1e-6 * max(abs(fd), 1e-3), (trial, an, fd)


def test_loss_grad_blocks_fd(model):
    """Each parameter block (W1, b1, W2, b2, w3, b3) of one element network separately."""
    s, shift, scale, th = model
    Fref = np.zeros_like(s.pos)
    L, g = S.loss_grad(th[1], shift, scale, s.pos, s.type, None, 3.0, Fref, 0.5, 2.0)
    e = int(s.type[0])
    sizes = [S.NDESC * S.H, S.H, S.H * S.H, S.H, S.H, 1]
    o = 0
    rng = np.random.default_rng(11)
    for sz in sizes:
        d = np.zeros_like(th[1])
        d[e, o:o + sz] = rng.normal(size=sz)
        o += sz
        h = 1e-6
        fd = (S.loss(th[1] + h * d, shift, scale, s.pos, s.type, None, 3.0, Fref, 0.5, 2.0) -
              S.loss(th[1] - h * d, shift, scale, s.pos, s.type, None, 3.0, Fref, 0.5, 2.0)) / (2 * h)
        an = (g * d).sum()
        assert abs(an - fd) <= 1e-6 * max(abs(fd), 1e-4), (sz, an, fd)


def test_bf16_rounding():
    x = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -9, 1.0 + 2.0 ** -7 + 2.0 ** -8, -2.5, 0.0,
                  3.0e-39])
    q = S.bf16(x)
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: ties go to the even mantissa (1.0)
    # 1 + 3 2^-9 is above the tie: rounds up; 1 + 2^-7 + 2^-8 is a tie to even (1 + 2^-6)
    assert list(q[:6]) == [1.0, 1.0, 1.0 + 2.0 ** -7, 1.0 + 2.0 ** -6, -2.5, 0.0]
    # subnormal: bfloat16 spacing there is 2^-133; nearest multiple within half a step
    assert abs(q[6] - 3.0e-39) <= 2.0 ** -134 and (q[6] / 2.0 ** -133) == round(q[6] / 2.0 ** -133)


def test_adam_first_step():
    th = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 0.0])
    t1, m, v = S.adam(th, g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    np.testing.assert_allclose(t1, th - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_ensemble_spread(model):
    s, shift, scale, th = model
    E, Fs, Fbar, sigma = S.ensemble(th, shift, scale, s.pos, s.type, None)
    assert Fs.shape == (2, s.n, 3)
    np.testing.assert_allclose(sigma, 0.5 * np.linalg.norm(Fs[0] - Fs[1], axis=1), rtol=1e-12)
