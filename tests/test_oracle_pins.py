"""Pins of the CPU oracle against facts fixed outside it.

The paper prints no ReaxFF formula and no worked example, so the oracle is
pinned by: brute-force all-pairs lists, closed forms at special points
(radii ratio 1, exact valence, sigmoid midpoints, cis/trans/linear
geometries), limits of the shielded and tapered forms, the uniqueness of the
7th-order taper, complex-step and finite-difference derivatives of its own
energy, conservation laws (zero net force and torque, invariance under rigid
motions and atom relabelling) and NVE energy conservation with the dt^2 law.
"""
import copy
import math

import numpy as np
import pytest

import reaxff_synth as rs
from oracle import NTERMS, TERM_NAMES, Oracle

T = {name: k for k, name in enumerate(TERM_NAMES)}
C, H, N, O = rs.C, rs.H, rs.N, rs.O


@pytest.fixture(scope="module")
def params():
    return rs.draw_params(0)


def mol(pos, types, q=None):
    pos = np.asarray(pos, dtype=np.float64)
    types = np.asarray(types, dtype=np.int32)
    if q is None:
        q = np.zeros(len(types))
    return rs.System(pos=pos, type=types, q=np.asarray(q, dtype=np.float64), box=None)


def energy_of(params, pos, types, q=None, cut=None):
    return Oracle(mol(pos, types, q), params, cut).energy()


# ---------------------------------------------------------------------------
# lists
# ---------------------------------------------------------------------------
def _numpy_pairs(system):
    """All-pairs squared distances with the minimum image, in plain numpy."""
    x = system.pos
    d = x[None, :, :] - x[:, None, :]
    if system.box is not None:
        L = system.box
        d = d - L * np.rint(d * (1.0 / L))
    r2 = d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1] + d[..., 2] * d[..., 2]
    return r2


@pytest.mark.parametrize("kind", ["periodic", "cluster"])
def test_lists_cells_equal_brute_force(params, kind):
    if kind == "periodic":
        s = rs.small_periodic(30, seed=11)   # 870 atoms, box ~ 20.7 A
    else:
        s = rs.cluster(300, seed=5)
    a = Oracle(s, params).lists()
    b = Oracle(s, params, brute=True).lists()
    for x, y in zip(a, b):
        assert x.shape == y.shape
        assert np.array_equal(x, y)


def test_lists_against_numpy_all_pairs(params):
    s = rs.small_periodic(30, seed=12)
    far, bonds, hb = Oracle(s, params).lists()
    r2 = _numpy_pairs(s)
    n = s.n
    iu = np.triu_indices(n, 1)
    sel = r2[iu] <= 100.0
    ref_far = np.stack([iu[0][sel], iu[1][sel]], 1)
    # allow only pairs within a few ulp of the cutoff to differ (fma vs plain sums)
    got = set(map(tuple, far.tolist()))
    ref = set(map(tuple, ref_far.tolist()))
    for (i, j) in got ^ ref:
        assert abs(r2[i, j] - 100.0) < 1e-12
    # H list: H donors, N/O acceptors within 7.5 A
    t = s.type
    ph = params.atom["p_hbond"][t]
    ref_hb = {(i, j) for i in range(n) for j in np.nonzero(r2[i] <= 56.25)[0]
              if i != j and ph[i] == 1 and ph[j] == 2}
    assert set(map(tuple, hb.tolist())) == ref_hb
    # bond list: full (both directions), every entry within 5 A
    bset = set(map(tuple, bonds.tolist()))
    assert all((j, i) in bset for (i, j) in bset)
    assert all(r2[i, j] <= 25.0 for (i, j) in bset)
    o = Oracle(s, params)
    # every pair within 5 A is a bond iff its raw bond order reaches bo_cut
    cand = np.argwhere(np.triu(r2 <= 25.0, 1))
    for (i, j) in cand[:4000]:
        assert ((i, j) in bset) == (o.bo_raw(i, j) >= 0.01)


def test_far_list_is_half_and_bond_list_full(params):
    s = rs.workload("petn_1856")
    far, bonds, hb = Oracle(s, params).lists()
    assert np.all(far[:, 0] < far[:, 1])
    assert len(np.unique(far, axis=0)) == len(far)
    b = set(map(tuple, bonds.tolist()))
    assert len(b) == len(bonds) and all((j, i) in b for (i, j) in b)


def test_periodic_box_too_small_rejected(params):
    s = rs.small_periodic(30, seed=1, box=19.0)
    with pytest.raises(ValueError):
        Oracle(s, params)


# ---------------------------------------------------------------------------
# bond orders
# ---------------------------------------------------------------------------
def test_bo_raw_closed_form_at_unit_radius_ratio(params):
    """At r equal to every mixed radius, each power is 1: BO'_raw = (1+bo_cut)e^p1 + e^p3 + e^p5."""
    p = copy.deepcopy(params)
    r0 = 1.3
    for name in ("r_s", "r_p", "r_pp"):
        p.pair[name][C, C] = r0
    o = Oracle(mol([[0, 0, 0], [r0, 0, 0]], [C, C]), p)
    pc = p.pair
    ref = (1.01 * math.exp(pc["p_bo1"][C, C]) + math.exp(pc["p_bo3"][C, C])
           + math.exp(pc["p_bo5"][C, C]))
    assert o.bo_raw(0, 1) == pytest.approx(ref, rel=1e-14)
    # H-H has only the sigma component
    rh = params.pair["r_s"][H, H]
    o = Oracle(mol([[0, 0, 0], [0, rh, 0]], [H, H]), params)
    assert o.bo_raw(0, 1) == pytest.approx(1.01 * math.exp(params.pair["p_bo1"][H, H]), rel=1e-14)


def test_correction_exact_valence_and_sigmoid_midpoint(params):
    """H-H at BO' = b with Val_H = Val_boc_H = b: Delta' = 0 on both atoms so f3 = 0 and
    f1 = 1; with p_boc3 = p_boc5 = 1 and p_boc4 = 1/b^2 the f4, f5 exponents vanish,
    f4 = f5 = 1/2, so BO = BO'/4."""
    pos = [[0, 0, 0], [0.8, 0, 0]]
    b = Oracle(mol(pos, [H, H]), params).bond_terms()[0, 3]
    p = copy.deepcopy(params)
    p.atom["val"][H] = b
    p.atom["val_boc"][H] = b
    p.pair["p_boc3"][H, H] = 1.0
    p.pair["p_boc4"][H, H] = 1.0 / (b * b)
    p.pair["p_boc5"][H, H] = 1.0
    o = Oracle(mol(pos, [H, H]), p)
    bt = o.bond_terms()
    at = o.atom_terms()
    assert bt[0, 3] == b
    assert at[0, 0] == pytest.approx(0.0, abs=1e-15)       # Delta'
    assert bt[0, 0] == pytest.approx(0.25 * b, rel=1e-14)
    assert bt[0, 1] == 0.0 and bt[0, 2] == 0.0             # no pi bonds for H


def test_correction_symmetric_diatomic_closed_form(params):
    """C-C diatomic: Delta'_i = Delta'_j = d, so f3 = d exactly and
    f1 = (4 + 2 e^{-p_boc1 d}) / (4 + 2 e^{-p_boc1 d} + d); pi orders get f1^2."""
    p = copy.deepcopy(params)
    o = Oracle(mol([[0, 0, 0], [1.4, 0, 0]], [C, C]), p)
    bt = o.bond_terms()[0]
    bop = bt[3]
    d = bop - 4.0
    # choose p_boc5 to put f4 = f5 = 1/2: p_boc3 (p_boc4 BO'^2 - Delta'boc) = p_boc5
    p.pair["p_boc3"][C, C] = 1.0
    p.pair["p_boc4"][C, C] = 2.0
    p.pair["p_boc5"][C, C] = 2.0 * bop * bop - d
    o = Oracle(mol([[0, 0, 0], [1.4, 0, 0]], [C, C]), p)
    bt = o.bond_terms()[0]
    e = 2.0 * math.exp(-p.general["p_boc1"] * d)
    f1 = (4.0 + e) / (4.0 + e + d)
    assert bt[0] == pytest.approx(bop * f1 * 0.25, rel=1e-12)
    assert bt[1] == pytest.approx(bt[5] * f1 * f1 * 0.25, rel=1e-12)
    assert bt[2] == pytest.approx(bt[6] * f1 * f1 * 0.25, rel=1e-12)


def test_lone_pairs_of_isolated_atoms(params):
    """No bonds: S = 0, Delta_e = -Val_e.  With truncation toward zero,
    nlp = e^{-p_lp1 (2+vlpex)^2} - trunc(-Val_e/2): C (-4): e^{-4p}+2; H (-1): e^{-p};
    N (-5): vlpex = -1, e^{-p}+2; O (-6): e^{-4p}+3."""
    pl = params.general["p_lp1"]
    pos = [[0, 0, 0], [20, 0, 0], [0, 20, 0], [0, 0, 20]]
    at = Oracle(mol(pos, [C, H, N, O]), params).atom_terms()
    ref = [math.exp(-4 * pl) + 2, math.exp(-pl), math.exp(-pl) + 2, math.exp(-4 * pl) + 3]
    assert np.allclose(at[:, 4], ref, rtol=1e-14, atol=0)
    nlp_opt = [0, 0, 1, 2]
    assert np.allclose(at[:, 5], np.array(nlp_opt) - np.array(ref), rtol=1e-14, atol=1e-15)


def test_bond_energy_limits(params):
    """E_bond = -D_s BOsig e^{p_be1 (1 - BOsig^p_be2)} - D_p BOpi - D_pp BOpipi is linear in
    the three well depths: p_be1 = 0 leaves -D_s BOsig; a huge p_be2 (BOsig < 1) sends the
    power to 0 and leaves the factor e^{p_be1}; D_s = 0 isolates the pi parts."""
    pos, ty = [[0, 0, 0], [1.35, 0, 0]], [C, C]
    bt = Oracle(mol(pos, ty), params).bond_terms()[0]
    bo, bopi, bopp = bt[0], bt[1], bt[2]
    sig = bo - bopi - bopp
    assert 0 < sig < 1
    p = copy.deepcopy(params)
    p.pair["p_be1"][C, C] = 0.0
    p.pair["D_p"][C, C] = p.pair["D_pp"][C, C] = 0.0
    assert energy_of(p, pos, ty)[T["bond"]] == pytest.approx(-p.pair["D_s"][C, C] * sig, rel=1e-13)
    p.pair["p_be1"][C, C] = 0.7
    p.pair["p_be2"][C, C] = 5000.0
    assert energy_of(p, pos, ty)[T["bond"]] == pytest.approx(
        -p.pair["D_s"][C, C] * sig * math.exp(0.7), rel=1e-13)
    p = copy.deepcopy(params)
    p.pair["D_s"][C, C] = 0.0
    p.pair["D_pp"][C, C] = 0.0
    assert energy_of(p, pos, ty)[T["bond"]] == pytest.approx(-p.pair["D_p"][C, C] * bopi, rel=1e-13)
    p.pair["D_p"][C, C] = 0.0
    p.pair["D_pp"][C, C] = 10.0
    assert energy_of(p, pos, ty)[T["bond"]] == pytest.approx(-10.0 * bopp, rel=1e-13)


# ---------------------------------------------------------------------------
# nonbonded
# ---------------------------------------------------------------------------
def _dimer(params, r, q=(0.5, -0.5), types=(C, O)):
    return energy_of(params, [[0, 0, 0], [r, 0, 0]], list(types), list(q))


def _far_params(params, vdw_off=False):
    """Bonds switched off (zero sigma radius) so a dimer has nonbonded terms only."""
    p = copy.deepcopy(params)
    for name in ("r_s", "r_p", "r_pp"):
        p.pair[name][:] = 0.0
    if vdw_off:
        p.pair["D_vdw"][:] = 0.0
        p.pair["e_core"][:] = 0.0
    return p


def test_taper_is_the_unique_seventh_order_smoothstep(params):
    """Without shielding (gamma -> infinity) E_coul * r / (C q q) is the taper.  A degree-7
    fit of it must satisfy Tap(0)=1, Tap(R)=0 and vanishing 1st-3rd derivatives at 0 and R."""
    p = _far_params(params, vdw_off=True)
    p.pair["gamma"][:] = 1e8
    qq = 0.5 * -0.5
    rr = np.linspace(0.5, 10.0, 24)
    tap = np.array([_dimer(p, r)[T["coul"]] * r / (332.06371 * qq) for r in rr])
    c = np.polyfit(rr / 10.0, tap, 7)
    res = tap - np.polyval(c, rr / 10.0)
    assert np.abs(res).max() < 1e-12
    poly = np.poly1d(c)
    assert poly(0.0) == pytest.approx(1.0, abs=1e-9)
    assert poly(1.0) == pytest.approx(0.0, abs=1e-9)
    for k in (1, 2, 3):
        assert poly.deriv(k)(0.0) == pytest.approx(0.0, abs=1e-7)
        assert poly.deriv(k)(1.0) == pytest.approx(0.0, abs=1e-7)
    # the pair at exactly r = R is listed and contributes zero
    assert _dimer(p, 10.0)[T["coul"]] == pytest.approx(0.0, abs=1e-15)
    assert _dimer(p, 10.0 + 1e-9)[T["coul"]] == 0.0


def test_coulomb_shielding_limits(params):
    """Shielded Coulomb C q q / (r^3 + gamma^-3)^(1/3): finite C q q gamma as r -> 0."""
    p = _far_params(params, vdw_off=True)
    g = p.pair["gamma"][C, O]
    e = _dimer(p, 1e-4)[T["coul"]]
    assert e == pytest.approx(332.06371 * (0.5 * -0.5) * g, rel=1e-6)


def test_vdw_morse_minimum_without_shielding(params):
    """gamma_w -> infinity and no core term: E_vdW / Tap is a Morse curve with its
    minimum -D at r = r_vdW."""
    p = _far_params(params)
    p.pair["gamma_w"][:] = 1e8
    p.pair["e_core"][:] = 0.0
    rv, D = p.pair["r_vdw"][C, O], p.pair["D_vdw"][C, O]
    pq = _far_params(params, vdw_off=True)
    pq.pair["gamma"][:] = 1e8

    def morse(r):
        tap = _dimer(pq, r)[T["coul"]] * r / (332.06371 * -0.25)
        return _dimer(p, r)[T["vdw"]] / tap

    assert morse(rv) == pytest.approx(-D, rel=1e-10)
    assert morse(rv * 0.99) > -D and morse(rv * 1.01) > -D
    # core term alone: e_core at r = r_core
    pc = _far_params(params)
    pc.pair["D_vdw"][:] = 0.0
    pc.pair["gamma_w"][:] = 1e8
    rc = pc.pair["r_core"][C, O]
    e = _dimer(pc, rc)[T["vdw"]] / (_dimer(pq, rc)[T["coul"]] * rc / (332.06371 * -0.25))
    assert e == pytest.approx(pc.pair["e_core"][C, O], rel=1e-10)


# ---------------------------------------------------------------------------
# angles, torsions, hydrogen bonds
# ---------------------------------------------------------------------------
def _angle_mol(theta, r1=1.35, r2=1.45, types=(C, C, O)):
    pos = [[r1, 0, 0], [0, 0, 0], [r2 * math.cos(theta), r2 * math.sin(theta), 0]]
    return pos, list(types)


def test_valence_minimum_is_zero_at_theta0(params):
    """At fixed bond lengths, E_val(theta) has its minimum 0 exactly at
    theta0 = pi - theta00 (1 - e^{-p_val10 (2 - SBO2_j)}) (radians)."""
    pos, ty = _angle_mol(1.9)
    o = Oracle(mol(pos, ty), params)
    sbo2 = o.atom_terms()[1, 7]
    th00 = math.radians(params.angle["theta00"][C, C, O])
    th0 = math.pi - th00 * (1 - math.exp(-params.general["p_val10"] * (2 - sbo2)))
    e0 = energy_of(params, *_angle_mol(th0))
    assert abs(e0[T["val"]]) < 1e-10 * abs(energy_of(params, *_angle_mol(th0 + 0.3))[T["val"]])
    for d in (-0.05, 0.05):
        assert energy_of(params, *_angle_mol(th0 + d))[T["val"]] > e0[T["val"]]
    # penalty and coalition depend on bond orders only, not on the angle
    e1 = energy_of(params, *_angle_mol(th0 + 0.4))
    assert e1[T["pen"]] == pytest.approx(e0[T["pen"]], rel=1e-12)
    assert e1[T["coa"]] == pytest.approx(e0[T["coa"]], rel=1e-12)


def _chain(omega, theta=1.9, lengths=(1.1, 1.4, 1.3), types=(H, C, N, O)):
    """i-j-k-l with bond angles theta at j and k and dihedral omega (omega=0 is cis).
    Four distinct elements; _chain_params removes the i-k, j-l and i-l bonds, so the
    chain has exactly three bonds and one torsion."""
    r1, r2, r3 = lengths
    j = np.array([0.0, 0.0, 0.0])
    k = np.array([r2, 0.0, 0.0])
    i = j + r1 * np.array([-math.cos(theta), math.sin(theta), 0.0])
    l = k + r3 * np.array([math.cos(theta), math.sin(theta) * math.cos(omega),
                           math.sin(theta) * math.sin(omega)])
    return [i, j, k, l], list(types)


def _chain_params(params, v=None):
    p = copy.deepcopy(params)
    for a, b in ((H, N), (C, O), (H, O)):
        for name in ("r_s", "r_p", "r_pp"):
            p.pair[name][a, b] = p.pair[name][b, a] = 0.0
    if v is not None:
        for name, val in zip(("V1", "V2", "V3"), v):
            p.tors[name][:] = val
    return p


def test_chain_has_one_torsion(params):
    p = _chain_params(params)
    for w in (0.0, 1.0, math.pi):
        bonds = Oracle(mol(*_chain(w)), p).lists()[1]
        assert set(map(tuple, bonds.tolist())) == {(0, 1), (1, 0), (1, 2), (2, 1), (2, 3), (3, 2)}


def test_torsion_dihedral_forms(params):
    """E_tor is even in omega; the V1 form vanishes at trans (pi), the V2 form at cis and
    trans with its maximum at pi/2, the V3 form at pi/3 and pi; V1 enters as V1 (1 + cos w)."""
    p = _chain_params(params)
    for w in (0.4, 1.3, 2.5):
        a = energy_of(p, *_chain(w))[T["tor"]]
        b = energy_of(p, *_chain(-w))[T["tor"]]
        assert a != 0 and a == pytest.approx(b, rel=1e-10)
    p1 = _chain_params(params, (1.0, 0.0, 0.0))
    assert abs(energy_of(p1, *_chain(math.pi))[T["tor"]]) < 1e-12
    a = energy_of(p1, *_chain(0.0))[T["tor"]]
    b = energy_of(p1, *_chain(1.0))[T["tor"]]
    assert a > 0 and a / b == pytest.approx(2.0 / (1.0 + math.cos(1.0)), rel=1e-10)
    p2 = _chain_params(params, (0.0, 10.0, 0.0))
    assert abs(energy_of(p2, *_chain(0.0))[T["tor"]]) < 1e-12
    assert abs(energy_of(p2, *_chain(math.pi))[T["tor"]]) < 1e-12
    e = [energy_of(p2, *_chain(w))[T["tor"]] for w in (1.4, math.pi / 2, 1.75)]
    assert e[1] > e[0] and e[1] > e[2]
    p3 = _chain_params(params, (0.0, 0.0, 1.0))
    assert abs(energy_of(p3, *_chain(math.pi / 3))[T["tor"]]) < 1e-12
    assert abs(energy_of(p3, *_chain(math.pi))[T["tor"]]) < 1e-12
    assert energy_of(p3, *_chain(0.0))[T["tor"]] > 0


def test_conjugation_at_trans_is_angle_independent(params):
    """At omega = 0 or pi the factor 1 + (cos^2 w - 1) sin sin is 1: E_conj does not depend
    on the bond angles (bond lengths fixed); at omega = pi/2 it is 1 - sin(th_ijk) sin(th_jkl)."""
    p = _chain_params(params)
    a = energy_of(p, *_chain(math.pi, theta=1.8))[T["conj"]]
    b = energy_of(p, *_chain(math.pi, theta=2.1))[T["conj"]]
    c = energy_of(p, *_chain(0.0, theta=2.0))[T["conj"]]
    assert a != 0 and a == pytest.approx(b, rel=1e-12) and a == pytest.approx(c, rel=1e-12)
    th = 1.9
    c = energy_of(p, *_chain(math.pi / 2, theta=th))[T["conj"]]
    a = energy_of(p, *_chain(math.pi, theta=th))[T["conj"]]
    assert c == pytest.approx(a * (1 - math.sin(th) ** 2), rel=1e-10)


def _hbond(theta, rz, rx=1.0):
    """X - H ... Z with X-H along -x, the angle X-H-Z equal to theta, |HZ| = rz."""
    h = np.zeros(3)
    x = np.array([-rx, 0.0, 0.0])
    z = rz * np.array([-math.cos(theta), math.sin(theta), 0.0])
    return [x, h, z], [N, H, O]


def test_hydrogen_bond_closed_forms(params):
    """Linear X-H...Z at r_HZ = r0hb: E_hb = p_hb1 (1 - e^{-p_hb2 BO_HX}); at theta = 0: 0."""
    p = copy.deepcopy(params)
    # keep Z out of the bond list so only the H-X bond exists
    p.pair["r_s"][H, O] = p.pair["r_s"][N, O] = 0.0
    r0 = p.hb["r0hb"][N, H, O]
    pos, ty = _hbond(math.pi, r0)
    o = Oracle(mol(pos, ty), p)
    far, bonds, hb = o.lists()
    assert set(map(tuple, bonds.tolist())) == {(0, 1), (1, 0)}
    bo = o.bond_terms()[0, 0]
    ref = p.hb["p_hb1"][N, H, O] * (1 - math.exp(-p.hb["p_hb2"][N, H, O] * bo))
    assert o.energy()[T["hb"]] == pytest.approx(ref, rel=1e-12)
    pos, ty = _hbond(1e-9 * 0.0, 3.0)
    assert abs(energy_of(p, pos, ty)[T["hb"]]) < 1e-20
    # half-angle form: theta = pi/2 gives sin^4(pi/4) = 1/4 of the linear value
    e90 = energy_of(p, *_hbond(math.pi / 2, r0))[T["hb"]]
    assert e90 == pytest.approx(0.25 * ref, rel=1e-12)


# ---------------------------------------------------------------------------
# forces: complex step, finite differences, conservation laws
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def cluster_sys():
    return rs.cluster(60, seed=21)


def test_forces_match_complex_step(params, cluster_sys):
    o = Oracle(cluster_sys, params)
    e, f = o.forces()
    scale = np.abs(f).max()
    rng = np.random.default_rng(0)
    for atom in rng.choice(cluster_sys.n, 8, replace=False):
        for comp in range(3):
            er, de = o.energy_cs(int(atom), comp)
            assert np.allclose(er, e, rtol=1e-13, atol=1e-11)
            assert abs(-de.sum() - f[atom, comp]) <= 1e-11 * scale


def test_forces_match_complex_step_periodic(params):
    s = rs.small_periodic(30, seed=4)
    o = Oracle(s, params)
    e, f = o.forces()
    scale = np.abs(f).max()
    for atom in (0, 17, 401, 869):
        for comp in range(3):
            _, de = o.energy_cs(atom, comp)
            assert abs(-de.sum() - f[atom, comp]) <= 1e-11 * scale


def test_forces_match_finite_differences(params, cluster_sys):
    """Central differences with one Richardson step; the energy is smooth away from the
    list thresholds, which the chosen step does not cross for this system."""
    o = Oracle(cluster_sys, params)
    e, f = o.forces()
    lists0 = o.lists()
    x0 = cluster_sys.pos.copy()
    scale = np.abs(f).max()

    def etot(x):
        o.set_positions(x)
        return o.energy().sum()

    for atom in (0, 13, 42):
        for comp in range(3):
            d = []
            for h in (2e-4, 1e-4):
                xp = x0.copy(); xp[atom, comp] += h
                xm = x0.copy(); xm[atom, comp] -= h
                d.append((etot(xp) - etot(xm)) / (2 * h))
            rich = (4 * d[1] - d[0]) / 3
            assert abs(-rich - f[atom, comp]) <= 1e-6 * scale
    o.set_positions(x0)
    for a, b in zip(o.lists(), lists0):
        assert np.array_equal(a, b)


def test_zero_net_force_and_torque(params, cluster_sys):
    e, f = Oracle(cluster_sys, params).forces()
    scale = np.abs(f).max()
    assert np.abs(f.sum(0)).max() <= 1e-12 * scale * cluster_sys.n
    tq = np.cross(cluster_sys.pos, f).sum(0)
    assert np.abs(tq).max() <= 1e-11 * scale * np.abs(cluster_sys.pos).max() * cluster_sys.n


def test_zero_net_force_periodic(params):
    s = rs.workload("petn_1856")
    e, f = Oracle(s, params).forces()
    assert np.abs(f.sum(0)).max() <= 1e-12 * np.abs(f).max() * s.n


def test_energy_invariant_under_rigid_motion_and_relabelling(params, cluster_sys):
    e0 = Oracle(cluster_sys, params).energy()
    rng = np.random.default_rng(3)
    a = rng.normal(size=(3, 3))
    qm, _ = np.linalg.qr(a)
    s2 = copy.deepcopy(cluster_sys)
    s2.pos = cluster_sys.pos @ qm.T + np.array([3.0, -7.0, 11.0])
    e1 = Oracle(s2, params).energy()
    perm = rng.permutation(cluster_sys.n)
    s3 = rs.System(pos=cluster_sys.pos[perm], type=cluster_sys.type[perm],
                   q=cluster_sys.q[perm], box=None)
    e2 = Oracle(s3, params).energy()
    scale = np.abs(e0).max()
    assert np.allclose(e1, e0, rtol=1e-10, atol=1e-10 * scale)
    assert np.allclose(e2, e0, rtol=1e-12, atol=1e-12 * scale)


def test_periodic_translation_invariance(params):
    s = rs.small_periodic(30, seed=9)
    e0, f0 = Oracle(s, params).forces()
    s2 = copy.deepcopy(s)
    s2.pos = np.mod(s.pos + np.array([4.1, -2.3, 7.7]), s.box)
    e1, f1 = Oracle(s2, params).forces()
    assert np.allclose(e1, e0, rtol=1e-10, atol=1e-9)
    assert np.abs(f1 - f0).max() <= 1e-9 * np.abs(f0).max()


# ---------------------------------------------------------------------------
# dynamics
# ---------------------------------------------------------------------------
def test_nve_energy_fluctuation_scales_with_dt_squared(params):
    """Velocity Verlet conserves a shadow energy: the total-energy fluctuation over a fixed
    time span shrinks by ~4x when dt is halved.  The model's hard bond-order thresholds
    (angle and torsion products, H-bond donor order) make E jump when an interaction
    enters or leaves; with those thresholds at zero and a vanishing list threshold the
    energy is smooth and the dt^2 law must hold."""
    smooth = dict(bo_cut=1e-10, thb_cut=0.0, thb_cutsq=0.0, hb_bo_cut=0.0)
    s = rs.cluster(40, seed=8)
    v = rs.maxwell_boltzmann(s.type, params.atom["mass"], 300.0, seed=108)
    spans = []
    for dt, steps in ((0.1, 40), (0.05, 80)):
        o = Oracle(s, params, smooth)
        _, vend, e = o.md(v, dt, steps)
        tot = e.sum(1)
        spans.append(tot.max() - tot.min())
    ratio = spans[0] / spans[1]
    assert 3.0 < ratio < 5.0, (spans, ratio)
    # momentum is conserved exactly up to rounding (zero net force every step)
    m = params.atom["mass"][s.type]
    assert np.abs((m[:, None] * vend).sum(0)).max() < 1e-10
