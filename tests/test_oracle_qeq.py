"""Pins of the charge-equilibration oracle (oracle/qeq.py) against what the
mathematics fixes independently of its linear-solve route: closed forms for
two atoms and for isolated atoms, the stationarity (KKT) conditions and the
constraint, the quadratic minimum, the matrix against an all-pairs brute
force, invariances, conjugate gradients against the direct solve, and the
extrapolation's exactness on polynomials."""
import math

import numpy as np
import pytest

import reaxff_synth as rs
from oracle import Oracle
from oracle import qeq as Q

R_NONB = 10.0


@pytest.fixture(scope="module")
def params():
    return rs.draw_params(0)


@pytest.fixture(scope="module")
def qp():
    return rs.draw_qeq_params(0)


def matrix(system, params, qp):
    far, _, _ = Oracle(system, params).lists()
    return Q.qeq_matrix(system, params, qp, far, R_NONB), Q.qeq_diag(system, qp)


def two_atoms(t0, t1, r):
    pos = np.array([[0.0, 0.0, 0.0], [r / math.sqrt(3)] * 3])
    return rs.System(pos=pos, type=np.array([t0, t1], dtype=np.int32), q=np.zeros(2), box=None)


def test_coupling_limits(params):
    g = 0.9
    # r -> 0: the shielding leaves C_ele * gamma (and the taper is 1)
    assert Q.pair_coupling(0.0, g, R_NONB) == pytest.approx(Q.C_ELE * g, rel=1e-15)
    # unshielded limit: tapered Coulomb C_ele Tap(r) / r
    r = 3.7
    u = r / R_NONB
    tap = 1 - 35 * u ** 4 + 84 * u ** 5 - 70 * u ** 6 + 20 * u ** 7
    assert Q.pair_coupling(r, 1e8, R_NONB) == pytest.approx(Q.C_ELE * tap / r, rel=1e-12)
    # zero at the cutoff
    assert abs(Q.pair_coupling(R_NONB, g, R_NONB)) < 1e-12


@pytest.mark.parametrize("t0,t1,r", [(0, 3, 1.4), (1, 2, 3.0), (3, 3, 7.5)])
def test_two_atoms_closed_form(params, qp, t0, t1, r):
    s = two_atoms(t0, t1, r)
    H, (J, chi) = matrix(s, params, qp)
    # by hand: q0 = -q1 = q minimises (chi0 - chi1) q + (J0 + J1 - 2 h) q^2 / 2
    g = math.sqrt(params.pair["gamma"][t0, t0] * params.pair["gamma"][t1, t1])
    u = r / R_NONB
    h = (1 - 35 * u ** 4 + 84 * u ** 5 - 70 * u ** 6 + 20 * u ** 7) * Q.C_ELE / (r ** 3 + g ** -3) ** (1 / 3)
    J0, J1 = qp["J"][t0], qp["J"][t1]
    c0, c1 = qp["chi"][t0], qp["chi"][t1]
    q0 = (c1 - c0) / (J0 + J1 - 2 * h)
    q, _, _ = Q.qeq_exact(H, chi)
    assert q == pytest.approx([q0, -q0], rel=1e-12, abs=1e-15)
    qc, _, _, it, res = Q.qeq_cg(H, chi, J, tol=1e-14)
    assert qc == pytest.approx([q0, -q0], rel=1e-10, abs=1e-14)


def test_isolated_atoms_equalise_electronegativity(params, qp):
    # atoms beyond the cutoff of each other: chi_i + J_i q_i = mu for all i
    rng = np.random.default_rng(5)
    n = 9
    pos = np.array([[12.0 * a, 12.5 * b, 13.0 * c] for a in range(3) for b in range(3) for c in range(1)])
    typ = rng.integers(0, 4, size=n).astype(np.int32)
    s = rs.System(pos=pos, type=typ, q=np.zeros(n), box=None)
    H, (J, chi) = matrix(s, params, qp)
    assert np.count_nonzero(H - np.diag(np.diag(H))) == 0
    mu = (chi / J).sum() / (1.0 / J).sum()
    q, _, _ = Q.qeq_exact(H, chi)
    assert q == pytest.approx((mu - chi) / J, rel=1e-12, abs=1e-15)


@pytest.fixture(scope="module", params=["cluster", "periodic"])
def system(request):
    if request.param == "cluster":
        return rs.cluster(150, seed=21)
    return rs.small_periodic(30, seed=22)


def test_stationarity_and_constraint(params, qp, system):
    H, (J, chi) = matrix(system, params, qp)
    q, s, t = Q.qeq_exact(H, chi)
    assert abs(q.sum()) < 1e-12 * np.abs(q).sum()
    g = chi + H @ q                   # equal to the multiplier mu in every component
    assert np.ptp(g) <= 1e-10 * np.abs(g).max()
    # the two systems themselves
    assert np.abs(H @ s + chi).max() <= 1e-10 * np.abs(chi).max()
    assert np.abs(H @ t + 1.0).max() <= 1e-10


def test_minimum_of_the_energy(params, qp, system):
    H, (J, chi) = matrix(system, params, qp)
    q, _, _ = Q.qeq_exact(H, chi)
    e0 = Q.qeq_energy(H, chi, q)
    rng = np.random.default_rng(3)
    for _ in range(5):
        d = rng.normal(size=q.size) * 0.01
        d -= d.mean()
        e1 = Q.qeq_energy(H, chi, q + d)
        # exact quadratic expansion about a constrained minimum: no linear term
        assert e1 - e0 == pytest.approx(0.5 * d @ (H @ d), rel=1e-6)
        assert e1 > e0
    assert np.linalg.eigvalsh(H).min() > 0


def test_matrix_equals_all_pairs_brute_force(params, qp, system):
    H, _ = matrix(system, params, qp)
    n = system.n
    ref = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            if i == j:
                ref[i, i] = qp["J"][system.type[i]]
                continue
            d = system.pos[j] - system.pos[i]
            if system.box is not None:
                d = d - system.box * np.rint(d / system.box)
            r = math.sqrt(float(d @ d))
            if r <= R_NONB:
                g = params.pair["gamma"][system.type[i], system.type[j]]
                ref[i, j] = Q.pair_coupling(r, g, R_NONB)
    # (the taper rounds to exactly zero just inside the cutoff, so the pattern of
    # nonzeros is not the pair set; the values are compared)
    assert np.abs(H - ref).max() <= 1e-13 * np.abs(ref).max()
    assert np.array_equal(H, H.T)


def test_invariances(params, qp):
    s = rs.cluster(80, seed=23)
    H, (J, chi) = matrix(s, params, qp)
    q, _, _ = Q.qeq_exact(H, chi)
    # permutation
    perm = np.random.default_rng(1).permutation(s.n)
    sp = rs.System(pos=s.pos[perm], type=s.type[perm], q=s.q[perm], box=None)
    Hp, (Jp, chip) = matrix(sp, params, qp)
    qp_, _, _ = Q.qeq_exact(Hp, chip)
    assert qp_ == pytest.approx(q[perm], rel=1e-10, abs=1e-13)
    # rigid rotation and translation
    a = 0.7
    Rz = np.array([[math.cos(a), -math.sin(a), 0], [math.sin(a), math.cos(a), 0], [0, 0, 1]])
    sr = rs.System(pos=s.pos @ Rz.T + np.array([3.0, -2.0, 5.0]), type=s.type, q=s.q, box=None)
    Hr, (Jr, chir) = matrix(sr, params, qp)
    qr, _, _ = Q.qeq_exact(Hr, chir)
    assert qr == pytest.approx(q, rel=1e-9, abs=1e-12)


def test_periodic_shift_invariance(params, qp):
    s = rs.small_periodic(30, seed=24)
    H, (J, chi) = matrix(s, params, qp)
    q, _, _ = Q.qeq_exact(H, chi)
    shifted = np.mod(s.pos + np.array([5.3, -7.1, 11.9]), s.box)
    ss = rs.System(pos=shifted, type=s.type, q=s.q, box=s.box)
    Hs, (Js, chis) = matrix(ss, params, qp)
    qs, _, _ = Q.qeq_exact(Hs, chis)
    assert qs == pytest.approx(q, rel=1e-9, abs=1e-12)


def test_cg_reaches_the_direct_solution(params, qp, system):
    H, (J, chi) = matrix(system, params, qp)
    q, s, t = Q.qeq_exact(H, chi)
    qc, sc, tc, it, res = Q.qeq_cg(H, chi, J, tol=1e-13)
    assert max(res) <= 1e-13 and it > 3
    assert np.abs(qc - q).max() <= 1e-11 * np.abs(q).max()
    # at the paper's tolerance: both relative residuals at or below 1e-6, and
    # the charge error bounded by |r| / lambda_min of each system
    qc6, sc6, tc6, it6, res6 = Q.qeq_cg(H, chi, J, tol=1e-6)
    assert max(res6) <= 1e-6 and it6 < it
    lam = np.linalg.eigvalsh(H).min()
    assert np.linalg.norm(sc6 - s) <= res6[0] * np.linalg.norm(chi) / lam * (1 + 1e-9)
    assert np.linalg.norm(tc6 - t) <= res6[1] * math.sqrt(system.n) / lam * (1 + 1e-9)
    # started at the solution, no iteration is needed
    _, _, _, it0, _ = Q.qeq_cg(H, chi, J, tol=1e-6, s0=s, t0=t)
    assert it0 == 0


def test_cg_on_sparse_matrix_equals_dense(params, qp):
    s = rs.small_periodic(30, seed=25)
    far, _, _ = Oracle(s, params).lists()
    H = Q.qeq_matrix(s, params, qp, far)
    Hs = Q.qeq_sparse(s, params, qp, far)
    assert np.abs(Hs.toarray() - H).max() == 0.0
    J, chi = Q.qeq_diag(s, qp)
    a = Q.qeq_cg(H, chi, J, tol=1e-8)
    b = Q.qeq_cg(Hs, chi, J, tol=1e-8)
    assert a[3] == b[3]
    assert np.abs(a[0] - b[0]).max() <= 1e-9 * np.abs(a[0]).max()   # summation order only


def test_extrapolation_exact_on_polynomials():
    rng = np.random.default_rng(9)
    c = rng.normal(size=(4, 5))

    def x(k):   # a cubic in the step index, per component
        return c[0] + c[1] * k + c[2] * k ** 2 + c[3] * k ** 3

    hist = [x(3), x(2), x(1), x(0)]
    assert Q.extrapolate(hist) == pytest.approx(x(4), rel=1e-12)
    lin = [c[0] + c[1] * 3, c[0] + c[1] * 2]
    assert Q.extrapolate(lin) == pytest.approx(c[0] + c[1] * 4, rel=1e-12)
    assert Q.extrapolate([]) is None


def test_workload_matrix_positive_definite(params, qp):
    s = rs.workload("petn_1856")
    H, _ = matrix(s, params, qp)
    w = np.linalg.eigvalsh(H)
    assert w.min() > 50.0
