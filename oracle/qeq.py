"""Charge equilibration (QEq) oracle -- test infrastructure only.

Only tests and the CPU-baseline timing import this module; the GPU library
never does.  Plain NumPy in FP64.

What is computed (Section 3.3, QEq paragraphs): the charges q that minimise
the electrostatic energy

    E(q) = sum_i (chi_i q_i + 1/2 J_i q_i^2) + sum_{i<j} H_ij q_i q_j

subject to sum_i q_i = Q (here Q = 0), where the off-diagonal coupling is the
force field's tapered, shielded Coulomb interaction over the far-neighbour
pairs (r <= r_nonb),

    H_ij = Tap(r_ij) C_ele / (r_ij^3 + gamma_ij^-3)^(1/3),

and the diagonal is H_ii = J_i.  The paper states the method reduces, by a
Lagrange multiplier, to two linear systems with the common matrix H.  With
H s = -chi and H t = -1 the minimiser is q = s - ((sum s - Q) / sum t) t:
stationarity gives chi + H q = mu 1 and the constraint fixes mu.

Two routes are written here:
  * qeq_exact: the definition, both systems solved directly (dense LU), for
    systems of a few thousand atoms;
  * qeq_cg: the paper's solver -- conjugate gradients with a diagonal
    preconditioner on both systems, iterated together (one product of H with
    both search directions per iteration), stopped when both relative
    residuals |r| / |b| fall to the tolerance (the paper's benchmarks use
    1e-6, Section 4) -- on a dense or a scipy sparse H.
The initial guess of consecutive MD steps is a polynomial extrapolation of
earlier solutions (extrapolate).
"""
from __future__ import annotations

import numpy as np

C_ELE = 332.06371  # kcal A / (mol e^2)


def taper(r, R):
    """Seventh-order taper: 1 at r = 0, zero with three vanishing derivatives at R."""
    u = np.asarray(r, dtype=np.float64) / R
    return 20 * u ** 7 - 70 * u ** 6 + 84 * u ** 5 - 35 * u ** 4 + 1


def pair_coupling(r, gamma, R):
    """Off-diagonal element H_ij for pairs at distance r with mixed shielding gamma."""
    r = np.asarray(r, dtype=np.float64)
    return taper(r, R) * C_ELE / np.cbrt(r ** 3 + np.asarray(gamma, dtype=np.float64) ** -3.0)


def displacements(pos, i, j, box):
    """x_j - x_i per pair, minimum image when box is given."""
    d = pos[j] - pos[i]
    if box is not None:
        L = np.asarray(box, dtype=np.float64)
        d = d - L * np.rint(d / L)
    return d


def qeq_entries(system, params, far, r_nonb=10.0):
    """(i, j, H_ij) over the unordered far pairs (far: (M,2) pairs in caller indices)."""
    far = np.asarray(far, dtype=np.int64).reshape(-1, 2)
    i, j = far[:, 0], far[:, 1]
    d = displacements(system.pos, i, j, system.box)
    r = np.sqrt((d * d).sum(axis=1))
    g = params.pair["gamma"][system.type[i], system.type[j]]
    return i, j, pair_coupling(r, g, r_nonb)


def qeq_diag(system, qp):
    t = np.asarray(system.type)
    return np.asarray(qp["J"], dtype=np.float64)[t], np.asarray(qp["chi"], dtype=np.float64)[t]


def qeq_matrix(system, params, qp, far, r_nonb=10.0):
    """Dense H (n x n): J_i on the diagonal, H_ij on the far pairs, zero elsewhere."""
    n = system.n
    i, j, h = qeq_entries(system, params, far, r_nonb)
    H = np.zeros((n, n))
    H[i, j] = h
    H[j, i] = h
    J, _ = qeq_diag(system, qp)
    H[np.arange(n), np.arange(n)] = J
    return H


def qeq_sparse(system, params, qp, far, r_nonb=10.0):
    """The same H as a scipy CSR matrix (large systems)."""
    import scipy.sparse as sp
    n = system.n
    i, j, h = qeq_entries(system, params, far, r_nonb)
    J, _ = qeq_diag(system, qp)
    rows = np.concatenate([i, j, np.arange(n)])
    cols = np.concatenate([j, i, np.arange(n)])
    vals = np.concatenate([h, h, J])
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


def combine(s, t, Q=0.0):
    """Charges from the two solutions: q = s - ((sum s - Q) / sum t) t."""
    return s - ((s.sum() - Q) / t.sum()) * t


def qeq_exact(H, chi, Q=0.0):
    """(q, s, t): both systems solved directly."""
    n = H.shape[0]
    s = np.linalg.solve(H, -np.asarray(chi, dtype=np.float64))
    t = np.linalg.solve(H, -np.ones(n))
    return combine(s, t, Q), s, t


def qeq_energy(H, chi, q):
    """E(q) = chi . q + 1/2 q^T H q (the diagonal of H holds J)."""
    q = np.asarray(q, dtype=np.float64)
    return float(np.dot(chi, q) + 0.5 * q @ (H @ q))


def qeq_cg(H, chi, J, tol=1e-6, maxit=500, s0=None, t0=None, Q=0.0):
    """The paper's solver on both systems at once.

    Diagonal (Jacobi) preconditioner M = diag(J); each iteration multiplies H
    by both search directions, then updates each system with its own step
    lengths.  Stops when |b - H x| / |b| <= tol for both systems (a system
    whose residual is exactly zero keeps its iterate).  Returns
    (q, s, t, iterations, (relative residual s, relative residual t)).
    """
    n = H.shape[0]
    B = np.stack([-np.asarray(chi, dtype=np.float64), -np.ones(n)], axis=1)
    X = np.zeros((n, 2))
    if s0 is not None:
        X[:, 0] = s0
    if t0 is not None:
        X[:, 1] = t0
    Minv = 1.0 / np.asarray(J, dtype=np.float64)
    R = B - H @ X
    Z = Minv[:, None] * R
    P = Z.copy()
    rz = (R * Z).sum(axis=0)
    bnorm = np.sqrt((B * B).sum(axis=0))

    def rel():
        return np.sqrt((R * R).sum(axis=0)) / bnorm

    it = 0
    res = rel()
    while np.any(res > tol) and it < maxit:
        AP = H @ P
        pap = (P * AP).sum(axis=0)
        alpha = np.where(pap > 0, rz / np.where(pap > 0, pap, 1.0), 0.0)
        X += alpha * P
        R -= alpha * AP
        Z = Minv[:, None] * R
        rz_new = (R * Z).sum(axis=0)
        beta = np.where(rz > 0, rz_new / np.where(rz > 0, rz, 1.0), 0.0)
        P = Z + beta * P
        rz = rz_new
        it += 1
        res = rel()
    s, t = X[:, 0], X[:, 1]
    return combine(s, t, Q), s, t, it, tuple(float(x) for x in res)


def extrapolate(history):
    """Initial guess from earlier solutions, newest first: the value at the next
    step of the polynomial through the last k equally spaced solutions
    (k = 1..4: x1; 2x1 - x2; 3x1 - 3x2 + x3; 4x1 - 6x2 + 4x3 - x4)."""
    coef = {1: (1,), 2: (2, -1), 3: (3, -3, 1), 4: (4, -6, 4, -1)}
    k = min(len(history), 4)
    if k == 0:
        return None
    return sum(c * np.asarray(h, dtype=np.float64) for c, h in zip(coef[k], history[:k]))
