"""Charge equilibration on the GPU (reaxff_qeq) against the oracle
(oracle/qeq.py): charges against the direct solve at a tight tolerance; at
the paper's 1e-6 the same iteration count as the oracle's CG, the residual
recomputed with the oracle's own matrix, and the charge error within the
bound that residual gives; extrapolated starts
over a short sequence of configurations; the 32,480-atom box against the
oracle's sparse CG; the 1,044,000-atom box by sampled stationarity; edge
cases (two atoms, no pairs, empty, non-convergence, call order)."""
import numpy as np
import pytest

import reaxff_synth as rs
from oracle import Oracle
from oracle import qeq as Q

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def params():
    return rs.draw_params(0)


@pytest.fixture(scope="module")
def qp():
    return rs.draw_qeq_params(0)


@pytest.fixture(scope="module")
def ff(params):
    from paper_1706_07772_amd import ReaxFF
    f = ReaxFF(params)
    yield f
    f.close()


def gpu_qeq(ff, system, qp, tol, maxit=1000, guess=False, build=True):
    import torch
    d = torch.device("cuda:0")
    P = torch.tensor(system.pos, dtype=torch.float64, device=d)
    T = torch.tensor(system.type, dtype=torch.int32, device=d)
    if build:
        ff.build_lists(P, T, None if system.box is None else system.box)
    q, it, res, s, t = ff.qeq(system.n, qp, tol=tol, maxit=maxit, guess=guess, want_st=True)
    torch.cuda.synchronize()
    return q.cpu().numpy(), it, res, s.cpu().numpy(), t.cpu().numpy()


def launches(ff):
    """Kernel launch counts since profiling was switched on (name -> launches)."""
    import ctypes
    K = 64
    ms = (ctypes.c_double * K)()
    calls = (ctypes.c_int64 * K)()
    names = (ctypes.c_char_p * K)()
    k = ff._lib.reaxff_profile_read(ff._h, K, ms, calls, names)
    return {names[i].decode(): int(calls[i]) for i in range(k)}


def qeq_path(ff, system, qp, tol, mode, **kw):
    """gpu_qeq with the product `mode`, and the product that ran: "half"
    (matrix-free over the half far list) or "stored"."""
    ff.set_qeq_product(mode)
    ff._lib.reaxff_profile(ff._h, 1)
    try:
        out = gpu_qeq(ff, system, qp, tol, **kw)
        k = launches(ff)
    finally:
        ff._lib.reaxff_profile(ff._h, 0)
        ff.set_qeq_product("auto")
    half, rows = k.get("qeq_half", 0), k.get("qeq_rows", 0)
    assert (half > 0) != (rows > 0), k
    return out, "half" if half else "stored"


def dense(system, params, qp):
    far, _, _ = Oracle(system, params).lists()
    H = Q.qeq_matrix(system, params, qp, far)
    J, chi = Q.qeq_diag(system, qp)
    return H, J, chi


def charge_error_bound(s, t, es, et):
    """First-order bound (times 1.1) on max |q - q*| for q = s - (sum s / sum t) t
    when |s - s*| <= es and |t - t*| <= et (2-norms)."""
    lam = abs(s.sum() / t.sum())
    n = s.size
    e = es + lam * et
    return 1.1 * e * (1.0 + np.sqrt(n) * np.abs(t).max() / abs(t.sum()))


SYSTEMS = {
    "cluster150": lambda: rs.cluster(150, seed=31),
    "periodic870": lambda: rs.small_periodic(30, seed=32),
    "petn_1856": lambda: rs.workload("petn_1856"),
}


@pytest.mark.parametrize("name", sorted(SYSTEMS))
def test_charges_match_direct_solve(ff, params, qp, name):
    s = SYSTEMS[name]()
    print(f"qeq parity {name} n={s.n}", flush=True)
    H, J, chi = dense(s, params, qp)
    q_ref, s_ref, t_ref = Q.qeq_exact(H, chi)
    q, it, res, sg, tg = gpu_qeq(ff, s, qp, tol=1e-12)
    assert max(res) <= 1e-12 and it > 3
    assert np.abs(q - q_ref).max() <= 1e-9 * np.abs(q_ref).max()
    assert np.abs(sg - s_ref).max() <= 1e-9 * np.abs(s_ref).max()
    assert np.abs(tg - t_ref).max() <= 1e-9 * np.abs(t_ref).max()
    assert abs(q.sum()) <= 1e-12 * np.abs(q).sum()


@pytest.mark.parametrize("name", sorted(SYSTEMS))
def test_paper_tolerance_same_iterations_as_oracle_cg(ff, params, qp, name):
    s = SYSTEMS[name]()
    H, J, chi = dense(s, params, qp)
    q_cg, s_cg, t_cg, it_cg, res_cg = Q.qeq_cg(H, chi, J, tol=1e-6)
    q, it, res, sg, tg = gpu_qeq(ff, s, qp, tol=1e-6)
    assert abs(it - it_cg) <= 1, (it, it_cg)
    # the residual the GPU stopped at, recomputed with the oracle's matrix
    rs_ = np.linalg.norm(H @ sg + chi) / np.linalg.norm(chi)
    rt_ = np.linalg.norm(H @ tg + 1.0) / np.sqrt(s.n)
    assert rs_ <= 1e-6 * (1 + 1e-6) and rt_ <= 1e-6 * (1 + 1e-6)
    assert abs(rs_ - res[0]) <= 1e-3 * res[0] and abs(rt_ - res[1]) <= 1e-3 * res[1]
    # both stopped iterates are within the bound their residuals give of the
    # exact charges (CG iterates are not reproducible to rounding: differences
    # in summation order grow over the recurrence)
    q_ref, s_ref, t_ref = Q.qeq_exact(H, chi)
    lam_min = np.linalg.eigvalsh(H).min()
    for qq, ss, tt in ((q, sg, tg), (q_cg, s_cg, t_cg)):
        es = np.linalg.norm(H @ ss + chi) / lam_min
        et = np.linalg.norm(H @ tt + 1.0) / lam_min
        assert np.abs(qq - q_ref).max() <= charge_error_bound(ss, tt, es, et)


def test_extrapolated_start(ff, params, qp):
    """Five configurations along a smooth path: with the extrapolated start the
    iterations drop, and every charge vector still meets the tolerance bound."""
    import torch
    base = rs.small_periodic(30, seed=33)
    rng = np.random.default_rng(4)
    vel = rng.normal(size=base.pos.shape) * 0.02
    its = {True: [], False: []}
    for guess in (False, True):
        ff.build_lists(torch.tensor(base.pos, dtype=torch.float64, device="cuda:0"),
                       torch.tensor(base.type, dtype=torch.int32, device="cuda:0"), base.box)
        ff.qeq(base.n, qp, tol=1e-8, guess=False)   # forget earlier solutions
        for k in range(1, 6):
            pos = np.mod(base.pos + k * vel, base.box)
            sk = rs.System(pos=pos, type=base.type, q=base.q, box=base.box)
            q, it, res, sg, tg = gpu_qeq(ff, sk, qp, tol=1e-8, guess=guess)
            its[guess].append(it)
            assert max(res) <= 1e-8
            H, J, chi = dense(sk, params, qp)
            q_ref, _, _ = Q.qeq_exact(H, chi)
            lam = np.linalg.eigvalsh(H).min()
            es = np.linalg.norm(H @ sg + chi) / lam
            et = np.linalg.norm(H @ tg + 1.0) / lam
            assert np.abs(q - q_ref).max() <= charge_error_bound(sg, tg, es, et)
    assert sum(its[True][2:]) < sum(its[False][2:]), its


@pytest.fixture(scope="module")
def box32480(params, qp):
    s = rs.workload("petn_32480")
    print(f"qeq 32480: oracle lists", flush=True)
    far, _, _ = Oracle(s, params).lists()
    return s, Q.qeq_sparse(s, params, qp, far)


@pytest.mark.parametrize("mode", ["auto", "stored"])
def test_box_32480_against_sparse_oracle(ff, params, qp, box32480, mode):
    """Both products: the matrix-free one over the half far list (what "auto"
    takes on this grid) and the stored rows."""
    s, Hs = box32480
    J, chi = Q.qeq_diag(s, qp)
    q_cg, s_cg, t_cg, it_cg, res_cg = Q.qeq_cg(Hs, chi, J, tol=1e-10)
    (q, it, res, sg, tg), path = qeq_path(ff, s, qp, 1e-10, mode)
    assert path == ("half" if mode == "auto" else "stored")
    assert abs(it - it_cg) <= 1, (it, it_cg)
    assert np.abs(q - q_cg).max() <= 1e-8 * np.abs(q_cg).max()
    assert np.linalg.norm(Hs @ sg + chi) / np.linalg.norm(chi) <= 1e-10 * (1 + 1e-6)


@pytest.mark.parametrize("mode", ["auto", "stored"])
def test_full_size_sampled_stationarity(ff, params, qp, mode):
    """1,044,000 atoms, both products: chi_i + (H q)_i equals the common
    multiplier on sampled atoms (their rows of H recomputed on the host from
    the positions), and the charges are neutral."""
    from scipy.spatial import cKDTree
    s = rs.workload("petn_1044000")
    tol = 1e-10
    (q, it, res, sg, tg), path = qeq_path(ff, s, qp, tol, mode)
    assert path == ("half" if mode == "auto" else "stored")
    print(f"qeq 1044000 ({path}): {it} iterations, residuals {res}", flush=True)
    assert max(res) <= tol
    assert abs(q.sum()) <= 1e-9 * np.abs(q).sum()
    box = np.asarray(s.box)
    pos = np.mod(s.pos, box)
    tree = cKDTree(pos, boxsize=box)
    rng = np.random.default_rng(8)
    idx = rng.choice(s.n, size=64, replace=False)
    J, chi = Q.qeq_diag(s, qp)
    g = []
    for i in idx:
        nb = np.array([j for j in tree.query_ball_point(pos[i], 10.0 + 1e-9) if j != i])
        d = Q.displacements(s.pos, np.full(nb.size, i), nb, s.box)
        r = np.sqrt((d * d).sum(1))
        keep = r <= 10.0
        h = Q.pair_coupling(r[keep], params.pair["gamma"][s.type[i], s.type[nb[keep]]], 10.0)
        g.append(chi[i] + J[i] * q[i] + h @ q[nb[keep]])
    g = np.array(g)
    lam = -(sg.sum() / tg.sum())    # q = s + lam t
    bound = tol * (np.linalg.norm(chi) + abs(lam) * np.sqrt(s.n))
    assert np.ptp(g) <= 2 * bound, (np.ptp(g), bound)


@pytest.mark.parametrize("run_max", [1, 3])
def test_matrix_free_run_lengths(params, qp, box32480, run_max):
    """The matrix-free product with runs of 1 and 3 cells per workgroup (other
    window shapes and partial-array layouts than the default 8) against the
    stored rows on the same lists."""
    from paper_1706_07772_amd import ReaxFF
    s, _ = box32480
    ff = ReaxFF(params)
    try:
        ff.set_nb_run(run_max)
        (q, it, res, sg, tg), path = qeq_path(ff, s, qp, 1e-10, "auto")
        assert path == "half"
        (q2, it2, _, _, _), path2 = qeq_path(ff, s, qp, 1e-10, "stored", build=False)
        assert path2 == "stored"
    finally:
        ff.close()
    assert abs(it - it2) <= 1, (it, it2)
    assert max(res) <= 1e-10
    assert np.abs(q - q2).max() <= 1e-9 * np.abs(q2).max()


def test_matrix_free_on_kept_skin_lists(params, qp, box32480):
    """Skin lists kept by a refresh after every atom moved (by less than
    skin / 2): the half far rows then hold pairs out to r_nonb + skin, which
    the matrix-free product must leave out; its charges at the moved positions
    against the oracle's sparse CG there, and against the stored rows."""
    import torch
    from paper_1706_07772_amd import ReaxFF
    s0, _ = box32480
    rng = np.random.default_rng(77)
    moved = rs.System(pos=s0.pos + rng.uniform(-0.25, 0.25, s0.pos.shape), type=s0.type, q=s0.q, box=s0.box)
    ff = ReaxFF(params)
    try:
        ff.set_skin(1.0, 10)
        d = torch.device("cuda:0")
        T = torch.tensor(s0.type, dtype=torch.int32, device=d)
        ff.build_lists(torch.tensor(s0.pos, dtype=torch.float64, device=d), T, s0.box)
        rebuilt = ff.refresh_lists(torch.tensor(moved.pos, dtype=torch.float64, device=d), T, s0.box)
        assert not rebuilt
        (q, it, res, sg, tg), path = qeq_path(ff, moved, qp, 1e-10, "auto", build=False)
        assert path == "half"
        (q2, it2, _, _, _), path2 = qeq_path(ff, moved, qp, 1e-10, "stored", build=False)
        assert path2 == "stored"
    finally:
        ff.close()
    far, _, _ = Oracle(moved, params).lists()
    Hs = Q.qeq_sparse(moved, params, qp, far)
    J, chi = Q.qeq_diag(moved, qp)
    q_cg, s_cg, t_cg, it_cg, _ = Q.qeq_cg(Hs, chi, J, tol=1e-10)
    assert abs(it - it_cg) <= 1 and abs(it2 - it_cg) <= 1, (it, it2, it_cg)
    assert np.abs(q - q_cg).max() <= 1e-8 * np.abs(q_cg).max()
    assert np.abs(q2 - q_cg).max() <= 1e-8 * np.abs(q_cg).max()
    assert np.linalg.norm(Hs @ sg + chi) / np.linalg.norm(chi) <= 1e-10 * (1 + 1e-6)


def test_edge_cases(ff, params, qp):
    import torch
    from paper_1706_07772_amd import ReaxFFError
    # two atoms: closed form
    pos = np.array([[0.0, 0.0, 0.0], [1.0, 1.2, 0.4]])
    s2 = rs.System(pos=pos, type=np.array([0, 3], dtype=np.int32), q=np.zeros(2), box=None)
    H, J, chi = dense(s2, params, qp)
    q0 = (chi[1] - chi[0]) / (J[0] + J[1] - 2 * H[0, 1])
    q, it, res, _, _ = gpu_qeq(ff, s2, qp, tol=1e-13)
    assert q == pytest.approx([q0, -q0], rel=1e-11)
    # atoms farther apart than the cutoff: electronegativity equalisation
    pos = np.array([[0.0, 0, 0], [12.0, 0, 0], [0, 12.5, 0], [0, 0, 13.0]])
    s4 = rs.System(pos=pos, type=np.array([0, 1, 2, 3], dtype=np.int32), q=np.zeros(4), box=None)
    J4, chi4 = Q.qeq_diag(s4, qp)
    mu = (chi4 / J4).sum() / (1 / J4).sum()
    q, it, res, _, _ = gpu_qeq(ff, s4, qp, tol=1e-13)
    assert q == pytest.approx((mu - chi4) / J4, rel=1e-11)
    # empty system
    e = rs.System(pos=np.zeros((0, 3)), type=np.zeros(0, np.int32), q=np.zeros(0), box=None)
    ff.build_lists(torch.zeros((0, 3), dtype=torch.float64, device="cuda:0"),
                   torch.zeros(0, dtype=torch.int32, device="cuda:0"), None)
    q, it, res = ff.qeq(0, qp)
    assert it == 0 and q.numel() == 0
    # not converged within maxit: the error code, with the last iterate
    s = rs.small_periodic(30, seed=34)
    with pytest.raises(ReaxFFError) as ei:
        gpu_qeq(ff, s, qp, tol=1e-14, maxit=2)
    assert ei.value.code == -7
    # lists built for another n
    with pytest.raises(ReaxFFError) as ei:
        ff.qeq(s.n + 1, qp)
    assert ei.value.code == -6
    # bad parameters
    bad = {"chi": qp["chi"], "J": np.array([1.0, 0.0, 1.0, 1.0])}
    with pytest.raises(ReaxFFError) as ei:
        ff.qeq(s.n, bad)
    assert ei.value.code == -1
