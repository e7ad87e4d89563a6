"""Plain FP64 oracle of the learned surrogate -- test infrastructure only.

Only tests, the build check and the benchmark's CPU baseline import this
module; the GPU library and its binding never do.

The surrogate is a per-atom energy model E = sum_a E_a(G_a) (Behler and
Parrinello, PRL 98, 146401 (2007)) with atom-centred descriptors G_a built
from neighbours within r_c = 5 A and per-element multilayer perceptrons.
Everything here follows the plain definitions:

Descriptor of atom i (224 features), d_ij = x_j - x_i (minimum image),
f_c(r) = (cos(pi r / r_c) + 1) / 2 for r < r_c:
  radial   G[16 b + k]  = sum_{j of element b} R_k(r_ij),
           R_k(r) = exp(-ETA_R (r - MU_R[k])^2) f_c(r),  k = 0..15
  angular  G[64 + 16 p + 8 (l - 1) + n]
                        = sum_{j of element b} sum_{k of element c}
                          A_n(r_ij) A_n(r_ik) cos^l(theta_jik),  l = 1, 2
           A_n(r) = exp(-ETA_A (r - MU_A[n])^2) f_c(r),  n = 0..7
  for the unordered element pairs p = (b <= c) in the order PAIRS; the double
  sum runs over ordered neighbour pairs (j, k), j = k included.

The oracle evaluates the angular double sum literally (every neighbour pair),
its derivative term by term, and directional derivatives by the complex step.

Network of member m for centre element e (224 -> 128 -> 128 -> 1, SiLU):
  x  = (G - shift) * scale
  Z1 = x W1 + b1,  H1 = silu(Z1),  Z2 = H1 W2 + b2,  H2 = silu(Z2),
  E_a = H2 . w3 + b3.
Matrix products take BF16-rounded operands on the GPU; every function here
takes a quantiser `q` applied at exactly those operands (identity for the
plain FP64 model, bf16 rounding to mirror the kernels).

Training loss of one frame with N atoms (per member):
  L = wE ((sum_a E_a - E_ref) / N)^2 + wF / (3N) sum_i |F_i - F_ref,i|^2
with F = -dE/dx.  Its parameter gradient uses the descriptor-space residual
u_a = sum_i (dG_a/dx_i) (F_i - F_ref,i) (a directional derivative of G) and
the derivative of the network along u_a, differentiated in reverse
(forward-over-reverse).  Adam (Kingma and Ba, 2015) updates the parameters.
"""
from __future__ import annotations

import numpy as np

RC = 5.0
NR = 16
NA = 8
MU_R = 0.5 + 0.3 * np.arange(NR)          # 0.5 .. 5.0 A
ETA_R = 0.5 / 0.3 ** 2
MU_A = 1.0 + 0.5 * np.arange(NA)          # 1.0 .. 4.5 A
ETA_A = 0.5 / 0.5 ** 2
PAIRS = [(b, c) for b in range(4) for c in range(b, 4)]
PAIR_INDEX = {bc: p for p, bc in enumerate(PAIRS)}
# ordered element pair (b, c) -> unordered pair index when b <= c, else -1
PAIR_OF = np.full((4, 4), -1, dtype=np.int64)
for _p, (_b, _c) in enumerate(PAIRS):
    PAIR_OF[_b, _c] = _p
NDESC = 4 * NR + len(PAIRS) * 2 * NA      # 224
H = 128
NPAR = NDESC * H + H + H * H + H + H + 1  # one element network
KCAL_PER_EV = 23.060548


# ---------------------------------------------------------------------------
# precision
# ---------------------------------------------------------------------------
def ident(a):
    return a


def bf16(a):
    """Round to the nearest bfloat16 (ties to even), through float32."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64).reshape(np.shape(a))


# ---------------------------------------------------------------------------
# descriptors
# ---------------------------------------------------------------------------
def neighbours(pos, box):
    """For every atom: neighbour indices and displacements x_j - x_i (minimum image)
    with |d| < RC, by brute force over all pairs; pos may be complex (real part decides)."""
    n = pos.shape[0]
    out = []
    for i in range(n):
        d = pos - pos[i]
        if box is not None:
            L = np.asarray(box, dtype=np.float64)
            d = d - L * np.rint(d.real / L)
        r2 = (d.real ** 2).sum(1)
        sel = np.nonzero((r2 < RC * RC) & (np.arange(n) != i))[0]
        out.append((sel, d[sel]))
    return out


def fcut(r):
    return 0.5 * (np.cos(np.pi * r / RC) + 1.0)


def dfcut(r):
    return -0.5 * np.pi / RC * np.sin(np.pi * r / RC)


def descriptors(pos, types, box, nb=None):
    """G (n, 224) by the plain definition; complex positions give complex G."""
    pos = np.asarray(pos)
    dt = np.complex128 if np.iscomplexobj(pos) else np.float64
    n = pos.shape[0]
    if nb is None:
        nb = neighbours(pos, box)
    G = np.zeros((n, NDESC), dtype=dt)
    for i in range(n):
        sel, d = nb[i]
        if sel.size == 0:
            continue
        r = np.sqrt((d * d).sum(1))
        fc = fcut(r)
        t = types[sel]
        Rk = np.exp(-ETA_R * (r[:, None] - MU_R[None, :]) ** 2) * fc[:, None]      # (m, 16)
        for b in range(4):
            G[i, NR * b:NR * (b + 1)] = Rk[t == b].sum(0)
        An = np.exp(-ETA_A * (r[:, None] - MU_A[None, :]) ** 2) * fc[:, None]      # (m, 8)
        u = d / r[:, None]
        cos = u @ u.T                                                             # (m, m)
        pj = PAIR_OF[t[:, None], t[None, :]]                                      # (m, m)
        for p in range(len(PAIRS)):
            sel_p = (pj == p)                     # ordered pairs (j of b, k of c), b <= c
            if not sel_p.any():
                continue
            base = 4 * NR + 2 * NA * p
            for l in (1, 2):
                wjk = np.where(sel_p, cos ** l, 0.0)
                G[i, base + (l - 1) * NA:base + l * NA] = np.einsum("jk,jn,kn->n", wjk, An, An)
    return G


def descriptor_vjp(pos, types, box, g, nb=None):
    """-sum_a g_a . dG_a/dx_i for every atom i (forces of an energy with dE/dG = g),
    from the term-by-term derivative of the plain definition."""
    n = pos.shape[0]
    if nb is None:
        nb = neighbours(pos, box)
    F = np.zeros((n, 3))
    for i in range(n):
        sel, d = nb[i]
        if sel.size == 0:
            continue
        r = np.sqrt((d * d).sum(1))
        u = d / r[:, None]
        fc, dfc = fcut(r), dfcut(r)
        t = types[sel]
        e = np.exp(-ETA_R * (r[:, None] - MU_R[None, :]) ** 2)
        dRk = (e * (-2.0 * ETA_R * (r[:, None] - MU_R[None, :])) * fc[:, None] + e * dfc[:, None])
        gd = np.zeros((sel.size, 3))                       # dE/dd_j
        for j in range(sel.size):
            gr = g[i, NR * t[j]:NR * (t[j] + 1)]
            gd[j] += (gr * dRk[j]).sum() * u[j]
        ea = np.exp(-ETA_A * (r[:, None] - MU_A[None, :]) ** 2)
        An = ea * fc[:, None]
        dAn = ea * (-2.0 * ETA_A * (r[:, None] - MU_A[None, :])) * fc[:, None] + ea * dfc[:, None]
        cos = u @ u.T
        pj = PAIR_OF[t[:, None], t[None, :]]
        ok = pj >= 0
        pjc = np.where(ok, pj, 0)
        base = 4 * NR + 2 * NA * pjc                                  # (m, m)
        idx = base[:, :, None] + np.arange(NA)[None, None, :]
        g1 = np.where(ok[:, :, None], g[i][idx], 0.0)                 # (m, m, 8)
        g2 = np.where(ok[:, :, None], g[i][idx + NA], 0.0)
        # T_jk = sum_n A_n(r_j) A_n(r_k) (g1 c + g2 c^2)
        s_val = g1 * cos[:, :, None] + g2 * (cos ** 2)[:, :, None]
        dT_drj = np.einsum("jn,kn,jkn->jk", dAn, An, s_val)
        dT_drk = np.einsum("jn,kn,jkn->jk", An, dAn, s_val)
        dT_dc = np.einsum("jn,kn,jkn->jk", An, An, g1 + 2.0 * g2 * cos[:, :, None])
        # dc/dd_j = (u_k - c u_j) / r_j, dc/dd_k = (u_j - c u_k) / r_k
        gd += dT_drj.sum(1)[:, None] * u
        gd += (dT_dc @ u - (dT_dc * cos).sum(1)[:, None] * u) / r[:, None]
        gd += dT_drk.sum(0)[:, None] * u
        gd += (dT_dc.T @ u - (dT_dc * cos).sum(0)[:, None] * u) / r[:, None]
        # d_j = x_j - x_i
        np.add.at(F, sel, -gd)
        F[i] += gd.sum(0)
    return F


def descriptor_jvp(pos, types, box, v, h=1e-20):
    """dG/dx applied to a displacement field v (n,3): the complex-step derivative
    Im G(x + i h v) / h, exact to rounding."""
    G = descriptors(np.asarray(pos, dtype=np.complex128) + 1j * h * np.asarray(v), types, box)
    return G.imag / h


# ---------------------------------------------------------------------------
# network
# ---------------------------------------------------------------------------
def sig(z):
    return 1.0 / (1.0 + np.exp(-z))


def silu(z):
    return z * sig(z)


def dsilu(z):
    s = sig(z)
    return s * (1.0 + z * (1.0 - s))


def d2silu(z):
    s = sig(z)
    return s * (1.0 - s) * (2.0 + z * (1.0 - 2.0 * s))


def unpack(theta):
    """Views of one element network's flat parameter vector."""
    o = 0
    W1 = theta[o:o + NDESC * H].reshape(NDESC, H); o += NDESC * H
    b1 = theta[o:o + H]; o += H
    W2 = theta[o:o + H * H].reshape(H, H); o += H * H
    b2 = theta[o:o + H]; o += H
    w3 = theta[o:o + H]; o += H
    b3 = theta[o:o + 1]
    return W1, b1, W2, b2, w3, b3


def init_params(nmembers, seed, e_per_atom=0.0):
    """(nmembers, 4, NPAR) float64: He-style normal weights, zero biases, b3 = e_per_atom."""
    rng = np.random.default_rng(np.random.PCG64(seed))
    th = np.zeros((nmembers, 4, NPAR))
    for m in range(nmembers):
        for e in range(4):
            W1, b1, W2, b2, w3, b3 = unpack(th[m, e])
            W1[:] = rng.normal(size=W1.shape) * np.sqrt(1.0 / NDESC)
            W2[:] = rng.normal(size=W2.shape) * np.sqrt(1.0 / H)
            w3[:] = rng.normal(size=w3.shape) * np.sqrt(1.0 / H)
            b3[:] = e_per_atom
    return th


def normaliser(G):
    """Per-feature shift and scale of descriptors G (n, 224): mean and 1 / max(std, 1e-3)."""
    shift = G.mean(0)
    scale = 1.0 / np.maximum(G.std(0), 1e-3)
    return shift, scale


def net_forward(theta, x, q=ident):
    """Primal pass of one element network on normalised descriptors x (r, 224)."""
    W1, b1, W2, b2, w3, b3 = unpack(theta)
    xq = q(x)
    Z1 = xq @ q(W1) + b1
    H1 = silu(Z1)
    Z2 = q(H1) @ q(W2) + b2
    H2 = silu(Z2)
    E = H2 @ w3 + b3[0]
    return E, dict(xq=xq, Z1=Z1, H1=H1, Z2=Z2, H2=H2)


def net_input_grad(theta, c, q=ident):
    """dE_a/dx_a (r, 224) from the cached primal pass c."""
    W1, b1, W2, b2, w3, b3 = unpack(theta)
    d2 = w3[None, :] * dsilu(c["Z2"])
    dH1 = q(d2) @ q(W2).T
    d1 = dH1 * dsilu(c["Z1"])
    return q(d1) @ q(W1).T


def model_energy_forces(th_member, shift, scale, pos, types, box, q=ident, nb=None, G=None):
    """One member: per-atom energies (n,), forces (n,3), and the caches."""
    if nb is None:
        nb = neighbours(pos, box)
    if G is None:
        G = descriptors(pos, types, box, nb)
    x = (G - shift) * scale
    n = pos.shape[0]
    Ea = np.zeros(n)
    gG = np.zeros((n, NDESC))
    caches = {}
    for e in range(4):
        rows = np.nonzero(types == e)[0]
        if rows.size == 0:
            continue
        E, c = net_forward(th_member[e], x[rows], q)
        Ea[rows] = E
        gG[rows] = net_input_grad(th_member[e], c, q) * scale
        caches[e] = (rows, c)
    F = descriptor_vjp(pos, types, box, gG, nb)
    return Ea, F, dict(G=G, x=x, gG=gG, caches=caches, nb=nb)


def ensemble(th, shift, scale, pos, types, box, q=ident):
    """All members: energies (M,), forces (M,n,3), mean force and the per-atom spread
    sigma_i = sqrt(mean_m |F_i^m - Fbar_i|^2)."""
    nb = neighbours(pos, box)
    G = descriptors(pos, types, box, nb)
    Es, Fs = [], []
    for m in range(th.shape[0]):
        Ea, F, _ = model_energy_forces(th[m], shift, scale, pos, types, box, q, nb, G)
        Es.append(Ea.sum())
        Fs.append(F)
    Fs = np.array(Fs)
    Fbar = Fs.mean(0)
    sigma = np.sqrt(((Fs - Fbar[None]) ** 2).sum(2).mean(0))
    return np.array(Es), Fs, Fbar, sigma


def loss(th_member, shift, scale, pos, types, box, Eref, Fref, wE, wF, q=ident):
    Ea, F, _ = model_energy_forces(th_member, shift, scale, pos, types, box, q)
    n = pos.shape[0]
    return wE * ((Ea.sum() - Eref) / n) ** 2 + wF / (3 * n) * ((F - Fref) ** 2).sum()


def loss_grad(th_member, shift, scale, pos, types, box, Eref, Fref, wE, wF, q=ident):
    """Loss and its gradient with respect to one member's parameters (4, NPAR)."""
    n = pos.shape[0]
    Ea, F, st = model_energy_forces(th_member, shift, scale, pos, types, box, q)
    res = F - Fref
    L = wE * ((Ea.sum() - Eref) / n) ** 2 + wF / (3 * n) * (res ** 2).sum()
    cE = 2.0 * wE * (Ea.sum() - Eref) / n ** 2
    cF = -2.0 * wF / (3 * n)
    # descriptor-space residual, in normalised coordinates
    u = descriptor_jvp(pos, types, box, res) * scale
    grad = np.zeros_like(th_member)
    for e, (rows, c) in st["caches"].items():
        W1, b1, W2, b2, w3, b3 = unpack(th_member[e])
        gW1, gb1, gW2, gb2, gw3, gb3 = unpack(grad[e])
        s1, s2 = dsilu(c["Z1"]), dsilu(c["Z2"])
        uq = q(u[rows])
        # tangent along u
        dZ1 = uq @ q(W1)
        dH1 = s1 * dZ1
        dZ2 = q(dH1) @ q(W2)
        dH2 = s2 * dZ2
        # reverse of (E, dE) with seeds (cE, cF)
        gw3[:] = (cE * c["H2"] + cF * dH2).sum(0)
        gb3[:] = cE * rows.size
        bZ2 = cE * w3[None, :] * s2 + cF * w3[None, :] * d2silu(c["Z2"]) * dZ2
        bdZ2 = cF * w3[None, :] * s2
        gW2[:] = q(c["H1"]).T @ q(bZ2) + q(dH1).T @ q(bdZ2)
        gb2[:] = bZ2.sum(0)
        bH1 = q(bZ2) @ q(W2).T
        bdH1 = q(bdZ2) @ q(W2).T
        bZ1 = bH1 * s1 + bdH1 * d2silu(c["Z1"]) * dZ1
        bdZ1 = bdH1 * s1
        gW1[:] = c["xq"].T @ q(bZ1) + uq.T @ q(bdZ1)
        gb1[:] = bZ1.sum(0)
    return L, grad


def adam(theta, grad, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (t counts from 1); returns new (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
