"""Closed-form pins of the oracle's coordination, angle and torsion factors.

Each test builds a molecule of two to four atoms whose bond list is fixed by
construction and then chooses parameter values that collapse a factor of the
energy to a value known in closed form: a sigmoid at its midpoint, an
exponential at zero argument, a limit as an exponent grows without bound,
or the zero of a factor.  The only oracle outputs used as inputs are bond
orders, which the bond-order pins of test_oracle_pins.py fix independently.
The functional forms are the ReaxFF terms the paper names in Section 2.1:
lone pair, over- and under-coordination, valence angle with penalty and
coalition, torsion with 4-body conjugation, and the bond-order correction.
"""
import copy
import math

import numpy as np
import pytest

import reaxff_synth as rs
from _common import near_straight_chain  # noqa: E402
from oracle import TERM_NAMES, Oracle

T = {name: k for k, name in enumerate(TERM_NAMES)}
C, H, N, O = rs.C, rs.H, rs.N, rs.O
THB = 0.001   # thb_cut: BOA = BO - thb_cut inside the angle and torsion factors


@pytest.fixture(scope="module")
def params():
    return rs.draw_params(0)


def mol(pos, types, q=None):
    pos = np.asarray(pos, dtype=np.float64)
    types = np.asarray(types, dtype=np.int32)
    q = np.zeros(len(types)) if q is None else np.asarray(q, dtype=np.float64)
    return rs.System(pos=pos, type=types, q=q, box=None)


def no_bond(p, a, b):
    for name in ("r_s", "r_p", "r_pp"):
        p.pair[name][a, b] = p.pair[name][b, a] = 0.0


def bond_table(o):
    """{(i, j): (BO, BOpi, BOpipi, BO')} for every directed bond."""
    bonds = o.lists()[1]
    bt = o.bond_terms()
    return {(int(i), int(j)): bt[k, :4] for k, (i, j) in enumerate(bonds)}


# ---------------------------------------------------------------------------
# lone pair, over- and under-coordination
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("p_lp1", [5.0, 4.0, 7.0])
def test_lone_pair_energy_of_isolated_hydrogen(params, p_lp1):
    """Isolated H: Delta_e = -1, trunc(-1/2) = 0, so nlp = e^{-p_lp1}, nlp_opt = 0 and
    Delta_lp = -e^{-p_lp1}; E_lp = p_lp2 Delta_lp / (1 + e^{-75 Delta_lp})."""
    p = copy.deepcopy(params)
    p.general["p_lp1"] = p_lp1
    p.atom["p_lp2"][H] = 3.0
    e = Oracle(mol([[0, 0, 0]], [H]), p).energy()
    dlp = -math.exp(-p_lp1)
    assert e[T["lp"]] == pytest.approx(3.0 * dlp / (1.0 + math.exp(-75.0 * dlp)), rel=1e-13)
    p.atom["p_lp2"][H] = 0.0
    assert Oracle(mol([[0, 0, 0]], [H]), p).energy()[T["lp"]] == 0.0


def _isolated(params):
    pos = [[0, 0, 0], [20, 0, 0], [0, 20, 0], [0, 0, 20]]
    return mol(pos, [C, H, N, O])


def _isolated_dlp(pl):
    # nlp of isolated atoms (pinned in test_oracle_pins): C, H, N, O; nlp_opt = 0, 0, 1, 2
    nlp = np.array([math.exp(-4 * pl) + 2, math.exp(-pl), math.exp(-pl) + 2,
                    math.exp(-4 * pl) + 3])
    return np.array([0.0, 0.0, 1.0, 2.0]) - nlp


def test_under_coordination_of_isolated_atoms(params):
    """No bonds: the over-coordination sum is empty (E_over = 0) and Sigma_pi = 0, so
    Delta_lpc = -Val - Delta_lp/(1 + p_ovun3).  With p_ovun2 = 0 the sigmoid is 1/2 and
    E_under = -p_ovun5 (1 - e^{p_ovun6 Delta_lpc}) / (2 (1 + p_ovun7))."""
    p = copy.deepcopy(params)
    p.atom["p_ovun2"][:] = 0.0
    p.atom["p_ovun5"][:] = [3.0, 5.0, 7.0, 11.0]
    s = _isolated(p)
    dlp = _isolated_dlp(p.general["p_lp1"])
    val = p.atom["val"]
    g = p.general
    for ov3 in (0.0, g["p_ovun3"]):
        p.general["p_ovun3"] = ov3
        e = Oracle(s, p).energy()
        assert e[T["over"]] == 0.0
        dlpc = -val - dlp / (1.0 + ov3)
        ref = -p.atom["p_ovun5"] * (1 - np.exp(g["p_ovun6"] * dlpc)) / (2 * (1 + g["p_ovun7"]))
        assert e[T["under"]] == pytest.approx(ref.sum(), rel=1e-13)
    # p_ovun5 = 0 switches the term off
    p.atom["p_ovun5"][:] = 0.0
    assert Oracle(s, p).energy()[T["under"]] == 0.0


def test_over_and_under_vanish_where_delta_lpc_is_zero(params):
    """H-H diatomic (no pi orders, so Sigma_pi = 0): Delta = BO - 1, Delta_lp = -nlp with
    nlp = e^{-p_lp1 (1 + BO)^2}.  p_ovun3 does not enter the bond orders; choosing
    1 + p_ovun3 = nlp / (1 - BO) makes Delta_lpc = Delta - Delta_lp/(1 + p_ovun3) zero,
    where both E_over (factor Delta_lpc) and E_under (factor 1 - e^{p_ovun6 Delta_lpc})
    vanish.  Away from it E_over carries sum_j p_ovun1 D_s BO."""
    p = copy.deepcopy(params)
    p.atom["p_ovun5"][H] = 20.0
    p.general["p_lp1"] = 0.3      # an nlp of order 1 keeps 1 + p_ovun3 well conditioned
    s = mol([[0, 0, 0], [0.85, 0, 0]], [H, H])
    bo = bond_table(Oracle(s, p))[(0, 1)][0]
    assert 0.2 < bo < 1.0
    nlp = math.exp(-p.general["p_lp1"] * (1 + bo) ** 2)
    p.general["p_ovun3"] = nlp / (1 - bo) - 1.0
    e = Oracle(s, p).energy()
    sumov = p.pair["p_ovun1"][H, H] * p.pair["D_s"][H, H] * bo
    assert abs(e[T["over"]]) < 1e-13 * sumov
    assert abs(e[T["under"]]) < 1e-13 * 20.0
    # with p_ovun3 = 0 and p_ovun2 = 0: Delta_lpc = BO - 1 + nlp, both terms in closed form
    p.general["p_ovun3"] = 0.0
    p.atom["p_ovun2"][H] = 0.0
    e = Oracle(s, p).energy()
    dlpc = bo - 1 + nlp
    ref_over = 2 * sumov * dlpc / (dlpc + 1.0 + 1e-8) / 2.0
    ref_under = 2 * -20.0 * (1 - math.exp(p.general["p_ovun6"] * dlpc)) / 2.0 / (1 + p.general["p_ovun7"])
    assert e[T["over"]] == pytest.approx(ref_over, rel=1e-12)
    assert e[T["under"]] == pytest.approx(ref_under, rel=1e-12)


def _oco(theta, r=1.25):
    """O - C - O, both C-O bonds of length r, angle theta at C (the O-O bond is removed
    from the parameters by the callers)."""
    return [[r, 0, 0], [0, 0, 0], [r * math.cos(theta), r * math.sin(theta), 0]], [O, C, O]


def test_sigma_pi_uses_the_neighbours_delta_minus_delta_lp(params):
    """Linear O-C-O.  The under-coordination factor 1/(1 + p_ovun7 e^{p_ovun8 Sigma_pi})
    reveals Sigma_pi of C from the ratio of E_under at p_ovun8 = x and 0 (p_ovun3 = 0, so
    Delta_lpc does not depend on Sigma_pi).  For a terminal O with one bond of order b:
    Delta = b - 2, trunc((b - 6)/2) = -2, nlp = e^{-p_lp1 b^2} + 2, Delta_lp = -e^{-p_lp1 b^2};
    Sigma_pi(C) = sum over both O of (b - 2 + e^{-p_lp1 b^2}) (BOpi + BOpipi)."""
    p = copy.deepcopy(params)
    no_bond(p, O, O)
    p.general["p_ovun3"] = 0.0
    p.atom["p_ovun5"][O] = 0.0
    p.atom["p_ovun5"][C] = 25.0
    pos, ty = _oco(math.pi)
    s = mol(pos, ty)
    p.general["p_ovun8"] = 0.0
    o = Oracle(s, p)
    bt = bond_table(o)
    e0 = o.energy()[T["under"]]
    x = 0.3
    p.general["p_ovun8"] = x
    e1 = Oracle(s, p).energy()[T["under"]]
    assert e0 != 0.0
    a7 = p.general["p_ovun7"]
    # e1/e0 = (1 + a7) / (1 + a7 e^{x Sigma_pi})
    sigma_pi = math.log(((1 + a7) * e0 / e1 - 1) / a7) / x
    pl = p.general["p_lp1"]
    ref = 0.0
    for (i, j) in ((1, 0), (1, 2)):
        b, bpi, bpp, _ = bt[(i, j)]
        assert 0 < b < 2
        ref += (b - 2 + math.exp(-pl * b * b)) * (bpi + bpp)
    assert sigma_pi == pytest.approx(ref, rel=1e-9)
    # Delta_lpc(C) = Delta - Delta_lp / (1 + p_ovun3 e^{p_ovun4 Sigma_pi}), read back from
    # E_under(C) with p_ovun2 = p_ovun8 = 0: -p_ovun5 (1 - e^{p_ovun6 Delta_lpc}) / (2 (1 + p_ovun7)).
    # C with 2 < S < 4: Delta_lp = -nlp = -e^{-p_lp1 (S - 2)^2}.
    S = bt[(1, 0)][0] + bt[(1, 2)][0]
    assert 2 < S < 4
    dlp = -math.exp(-pl * (S - 2) ** 2)
    p.general["p_ovun8"] = 0.0
    p.atom["p_ovun2"][C] = 0.0
    g = p.general
    for a3, a4 in ((0.0, 6.0), (40.0, 0.0), (40.0, 6.0), (40.0, -6.0)):
        p.general["p_ovun3"], p.general["p_ovun4"] = a3, a4
        dlpc = (S - 4.0) - dlp / (1.0 + a3 * math.exp(a4 * ref))
        e = Oracle(s, p).energy()[T["under"]]
        assert e == pytest.approx(-25.0 * (1 - math.exp(g["p_ovun6"] * dlpc)) / (2 * (1 + g["p_ovun7"])),
                                  rel=1e-10)


# ---------------------------------------------------------------------------
# SBO and SBO2 of a three-bond centre
# ---------------------------------------------------------------------------
def _co3(r=1.3):
    pos = [[0, 0, 0]] + [[r * math.cos(a), r * math.sin(a), 0.0]
                         for a in (0.0, 2 * math.pi / 3, 4 * math.pi / 3)]
    return mol(pos, [C, O, O, O])


def _co3_params(params):
    p = copy.deepcopy(params)
    no_bond(p, O, O)
    p.general["p_val8"] = 0.0
    return p


def _co3_sums(o):
    bt = bond_table(o)
    b = [bt[(0, j)] for j in (1, 2, 3)]
    S = sum(x[0] for x in b)
    sumpi = sum(x[1] + x[2] for x in b)
    prod = math.prod(math.exp(-x[0] ** 8) for x in b)
    return S, sumpi, prod


def test_sbo_pi_part_at_zero_delta_ang(params):
    """p_val8 = 0 and Val_ang(C) = S_C give Delta_ang = 0 exactly, leaving
    SBO = sum_n (BOpi + BOpipi).  One more unit of Val_ang adds (1 - prod_n e^{-BO^8})."""
    p = _co3_params(params)
    s = _co3()
    S, sumpi, prod = _co3_sums(Oracle(s, p))
    at = Oracle(s, p).atom_terms()
    assert at[0, 2] == pytest.approx(S, rel=1e-15)
    p.atom["val_ang"][C] = at[0, 2]
    sbo0 = Oracle(s, p).atom_terms()[0, 6]
    assert sbo0 == pytest.approx(sumpi, rel=1e-14)
    p.atom["val_ang"][C] = at[0, 2] + 1.0
    sbo1 = Oracle(s, p).atom_terms()[0, 6]
    assert sbo1 - sbo0 == pytest.approx(1.0 - prod, rel=1e-12)
    assert 0.5 < 1.0 - prod <= 1.0


def test_sbo_lone_pair_term_only_when_vlpex_negative(params):
    """SBO depends on p_val8 through -p_val8 (1 - prod) nlp only when vlpex < 0.  C with
    2 < S < 4: Delta_e = S - 4 in (-2, 0), trunc = 0, vlpex = S - 4 < 0 and
    nlp = e^{-p_lp1 (S - 2)^2}.  With Val_e(C) = S - 1 instead, Delta_e = 1, vlpex = 1 >= 0
    and p_val8 drops out."""
    p = _co3_params(params)
    s = _co3()
    S, sumpi, prod = _co3_sums(Oracle(s, p))
    assert 2 < S < 4
    nlp = math.exp(-p.general["p_lp1"] * (S - 2) ** 2)
    sbo = {}
    for v8 in (0.0, 1.7):
        p.general["p_val8"] = v8
        sbo[v8] = Oracle(s, p).atom_terms()[0, 6]
    assert sbo[1.7] - sbo[0.0] == pytest.approx(-1.7 * (1 - prod) * nlp, rel=1e-10)
    p.atom["val_e"][C] = S - 1.0
    sbo = {}
    for v8 in (0.0, 1.7):
        p.general["p_val8"] = v8
        sbo[v8] = Oracle(s, p).atom_terms()[0, 6]
    assert sbo[1.7] == sbo[0.0]


@pytest.mark.parametrize("target", [-0.5, 0.4, 1.0, 1.6, 2.0, 2.7])
def test_sbo2_branches(params, target):
    """Val_ang moves SBO linearly (slope 1 - prod) without touching the bond orders, so
    SBO can be placed in each branch of SBO2.  p_val9 = 1 makes SBO2 = clamp(SBO, 0, 2);
    p_val9 = 2 gives SBO^2 on (0, 1] and 2 - (2 - SBO)^2 on (1, 2)."""
    p = _co3_params(params)
    s = _co3()
    S, sumpi, prod = _co3_sums(Oracle(s, p))
    p.atom["val_ang"][C] = S + (target - sumpi) / (1.0 - prod)
    for pv9 in (1.0, 2.0):
        p.general["p_val9"] = pv9
        at = Oracle(s, p).atom_terms()
        sbo, sbo2 = at[0, 6], at[0, 7]
        assert sbo == pytest.approx(target, abs=1e-12)
        if pv9 == 1.0:
            ref = min(max(sbo, 0.0), 2.0)
        elif sbo <= 0:
            ref = 0.0
        elif sbo <= 1:
            ref = sbo * sbo
        elif sbo < 2:
            ref = 2 - (2 - sbo) ** 2
        else:
            ref = 2.0
        assert sbo2 == pytest.approx(ref, rel=1e-13, abs=1e-15)


# ---------------------------------------------------------------------------
# valence angle amplitude, penalty, coalition
# ---------------------------------------------------------------------------
def _oco_params(params):
    p = copy.deepcopy(params)
    no_bond(p, O, O)
    return p


def test_valence_angle_amplitude_far_from_theta0(params):
    """With p_val2 very large the bracket 1 - e^{-p_val2 (theta0 - theta)^2} is 1 away from
    theta0, leaving E_val = f7(BOA_ij) f7(BOA_jk) f8 p_val1.  Val_ang(C) = 100 makes
    Delta_ang ~ -98: e6 underflows, e7 dominates and f8 = p_val5 (the large SBO puts
    theta0 at pi, far from 100 degrees).  With p_val4 = 1, f7 = 1 - e^{-p_val3 BOA};
    with p_val4 = 2, f7 = 1 - e^{-p_val3 BOA^2}."""
    p = _oco_params(params)
    p.angle["p_val2"][O, C, O] = 1e4
    p.angle["p_val7"][O, C, O] = 3.0
    p.atom["val_ang"][C] = 100.0
    pos, ty = _oco(math.radians(100.0))
    for pv4 in (1.0, 2.0):
        p.angle["p_val4"][O, C, O] = pv4
        o = Oracle(mol(pos, ty), p)
        at = o.atom_terms()
        assert at[1, 7] == 2.0                       # SBO2 = 2: theta0 = pi
        bt = bond_table(o)
        pv3 = p.atom["p_val3"][C]
        f7 = [1 - math.exp(-pv3 * (bt[(1, j)][0] - THB) ** pv4) for j in (0, 2)]
        ref = f7[0] * f7[1] * p.atom["p_val5"][C] * p.angle["p_val1"][O, C, O]
        assert o.energy()[T["val"]] == pytest.approx(ref, rel=1e-13)


@pytest.mark.parametrize("shift,f8", [(0.0, 1.0), (-5.0, 1.0)])
def test_valence_f8_limits(params, shift, f8):
    """f8 = p_val5 - (p_val5 - 1)(2 + e6)/(1 + e6 + e7) equals 1 at Delta_ang = 0
    (e6 = e7 = 1) and tends to 1 for Delta_ang >> 0 (e6 dominates).  theta = 60 degrees is
    at least 40 degrees from any theta0 (>= 100 degrees), so the bracket is 1."""
    p = _oco_params(params)
    p.angle["p_val2"][O, C, O] = 1e4
    p.angle["p_val4"][O, C, O] = 1.0
    pos, ty = _oco(math.radians(60.0))
    S = Oracle(mol(pos, ty), p).atom_terms()[1, 2]
    p.atom["val_ang"][C] = S + shift
    o = Oracle(mol(pos, ty), p)
    bt = bond_table(o)
    pv3 = p.atom["p_val3"][C]
    f7 = [1 - math.exp(-pv3 * (bt[(1, j)][0] - THB)) for j in (0, 2)]
    ref = f7[0] * f7[1] * f8 * p.angle["p_val1"][O, C, O]
    assert o.energy()[T["val"]] == pytest.approx(ref, rel=1e-13)


def test_penalty_closed_forms(params):
    """E_pen = p_pen1 f9 e^{-p_pen2 (BOA_ij - 2)^2} e^{-p_pen2 (BOA_jk - 2)^2} with
    f9 = (2 + e^{-p_pen3 Delta}) / (1 + e^{-p_pen3 Delta} + e^{p_pen4 Delta}).
    p_pen2 = p_pen3 = p_pen4 = 0: E_pen = p_pen1.  p_pen4 = 0 makes f9 = 1 for any p_pen3;
    p_pen3 = 0 gives f9 = 3 / (2 + e^{p_pen4 Delta}), Delta = S_C - Val_C."""
    p = _oco_params(params)
    p.atom["val_ang"][C] = 3.0    # Delta_ang != Delta, so the two cannot be confused
    pos, ty = _oco(math.radians(115.0))
    s = mol(pos, ty)
    p.angle["p_pen1"][O, C, O] = 13.0
    for k in ("p_pen2", "p_pen3", "p_pen4"):
        p.general[k] = 0.0
    o = Oracle(s, p)
    assert o.energy()[T["pen"]] == pytest.approx(13.0, rel=1e-15)
    bt = bond_table(o)
    boa = [bt[(1, j)][0] - THB for j in (0, 2)]
    S = bt[(1, 0)][0] + bt[(1, 2)][0]
    p.general["p_pen2"] = 0.7
    gauss = math.exp(-0.7 * (boa[0] - 2) ** 2) * math.exp(-0.7 * (boa[1] - 2) ** 2)
    assert Oracle(s, p).energy()[T["pen"]] == pytest.approx(13.0 * gauss, rel=1e-13)
    p.general["p_pen3"] = 0.4
    assert Oracle(s, p).energy()[T["pen"]] == pytest.approx(13.0 * gauss, rel=1e-13)
    p.general["p_pen3"] = 0.0
    p.general["p_pen4"] = 4.0
    f9 = 3.0 / (2.0 + math.exp(4.0 * (S - 4.0)))
    assert Oracle(s, p).energy()[T["pen"]] == pytest.approx(13.0 * gauss * f9, rel=1e-12)


def test_coalition_closed_forms(params):
    """E_coa = p_coa1 / (1 + e^{p_coa2 Delta_ang}) e^{-p_coa3 (S_i - BOA_ij)^2}
    e^{-p_coa3 (S_k - BOA_jk)^2} e^{-p_coa4 (BOA_ij - 1.5)^2} e^{-p_coa4 (BOA_jk - 1.5)^2}.
    All of p_coa2,3,4 zero: p_coa1/2.  Terminal O atoms have S = BO, so S_i - BOA_ij =
    thb_cut exactly and p_coa3 = 1e5 gives e^{-0.1} per bond (the centre's S would give a
    vanishing factor).  p_coa2 alone: Delta_ang = S_C - Val_ang."""
    p = _oco_params(params)
    p.atom["val_ang"][C] = 3.3    # Delta_ang != Delta, so the two cannot be confused
    pos, ty = _oco(math.radians(115.0))
    s = mol(pos, ty)
    p.angle["p_coa1"][O, C, O] = -8.0
    for k in ("p_coa2", "p_coa3", "p_coa4"):
        p.general[k] = 0.0
    o = Oracle(s, p)
    assert o.energy()[T["coa"]] == pytest.approx(-4.0, rel=1e-15)
    bt = bond_table(o)
    bo = [bt[(1, j)][0] for j in (0, 2)]
    p.general["p_coa3"] = 1e5
    assert Oracle(s, p).energy()[T["coa"]] == pytest.approx(-4.0 * math.exp(-0.2), rel=1e-6)
    p.general["p_coa3"] = 0.0
    p.general["p_coa4"] = 3.0
    g = math.exp(-3.0 * (bo[0] - THB - 1.5) ** 2) * math.exp(-3.0 * (bo[1] - THB - 1.5) ** 2)
    assert Oracle(s, p).energy()[T["coa"]] == pytest.approx(-4.0 * g, rel=1e-13)
    p.general["p_coa4"] = 0.0
    p.general["p_coa2"] = 2.0
    dang = bo[0] + bo[1] - p.atom["val_ang"][C]
    assert Oracle(s, p).energy()[T["coa"]] == pytest.approx(
        -8.0 / (1.0 + math.exp(2.0 * dang)), rel=1e-13)


# ---------------------------------------------------------------------------
# torsion: f10, f11 and the V2 exponential; conjugation amplitude
# ---------------------------------------------------------------------------
def _chain(omega, theta=1.9, lengths=(1.1, 1.4, 1.3)):
    """H-C-N-O chain, bond angles theta at C and N, dihedral omega (0 = cis)."""
    r1, r2, r3 = lengths
    j = np.array([0.0, 0.0, 0.0])
    k = np.array([r2, 0.0, 0.0])
    i = j + r1 * np.array([-math.cos(theta), math.sin(theta), 0.0])
    l = k + r3 * np.array([math.cos(theta), math.sin(theta) * math.cos(omega),
                           math.sin(theta) * math.sin(omega)])
    return mol([i, j, k, l], [H, C, N, O])


def _chain_params(params, v=(0.0, 0.0, 0.0), p_tor1=0.0):
    p = copy.deepcopy(params)
    for a, b in ((H, N), (C, O), (H, O)):
        no_bond(p, a, b)
    for name, val in zip(("V1", "V2", "V3", "p_tor1"), tuple(v) + (p_tor1,)):
        p.tors[name][:] = val
    p.general["p_tor3"] = 0.0
    p.general["p_tor4"] = 0.0
    return p


def _chain_bonds(o):
    bt = bond_table(o)
    assert set(bt) == {(0, 1), (1, 0), (1, 2), (2, 1), (2, 3), (3, 2)}
    return bt[(0, 1)], bt[(1, 2)], bt[(2, 3)]


def test_torsion_amplitude_at_right_angle(params):
    """omega = pi/2: 1 + cos w = 1, 1 - cos 2w = 2, 1 + cos 3w = 1, so
    E_tor = f10 sin^2(theta) (V1 + 2 V2 e^{p_tor1 (2 - BOpi_jk - f11)^2} + V3) / 2.
    p_tor3 = p_tor4 = 0 gives f11 = 3/3 = 1; p_tor1 = 0 removes the exponential;
    p_tor2 = 1e4 sends each factor of f10 = prod (1 - e^{-p_tor2 BOA}) to 1."""
    th = 1.9
    s = _chain(math.pi / 2, theta=th)
    for v in ((1.0, 0.0, 0.0), (0.0, 1.0, 0.0), (0.0, 0.0, 1.0), (0.7, -1.3, 0.4)):
        p = _chain_params(params, v)
        p.general["p_tor2"] = 1e4
        e = Oracle(s, p).energy()[T["tor"]]
        ref = math.sin(th) ** 2 * (v[0] + 2 * v[1] + v[2]) / 2
        assert e == pytest.approx(ref, rel=1e-12, abs=1e-15)


def test_torsion_f10_and_v2_exponential(params):
    """f10 = prod over the three bonds of (1 - e^{-p_tor2 BOA}); the V2 factor is
    e^{p_tor1 (2 - BOpi_jk - f11)^2} with f11 = 1 (p_tor3 = p_tor4 = 0); BOpi_jk is the
    corrected pi order of the central C-N bond."""
    th = 1.9
    s = _chain(math.pi / 2, theta=th)
    p = _chain_params(params, (0.0, 10.0, 0.0), p_tor1=-3.0)
    pt2 = p.general["p_tor2"] = 5.5
    o = Oracle(s, p)
    b1, b2, b3 = _chain_bonds(o)
    f10 = math.prod(1 - math.exp(-pt2 * (b[0] - THB)) for b in (b1, b2, b3))
    assert b2[1] > 0.05          # the central bond has a pi order
    ref = f10 * math.sin(th) ** 2 * 10.0 * math.exp(-3.0 * (1.0 - b2[1]) ** 2)
    assert o.energy()[T["tor"]] == pytest.approx(ref, rel=1e-12)


def test_torsion_f11(params):
    """f11 = (2 + e^{-p_tor3 D}) / (1 + e^{-p_tor3 D} + e^{p_tor4 D}), D = Delta_ang_j +
    Delta_ang_k.  p_tor4 = 0 makes f11 = 1 whatever p_tor3; p_tor3 = 0 gives
    f11 = 3 / (2 + e^{p_tor4 D}).  Read back through the V2 exponential with p_tor1 = -1."""
    th = 1.9
    s = _chain(math.pi / 2, theta=th)
    p = _chain_params(params, (0.0, 10.0, 0.0), p_tor1=-1.0)
    p.general["p_tor2"] = 1e4
    o = Oracle(s, p)
    b1, b2, b3 = _chain_bonds(o)
    S_c = b1[0] + b2[0]
    S_n = b2[0] + b3[0]
    D = (S_c - p.atom["val_ang"][C]) + (S_n - p.atom["val_ang"][N])
    base = math.sin(th) ** 2 * 10.0

    def e_of(f11):
        return base * math.exp(-1.0 * (2.0 - b2[1] - f11) ** 2)

    p.general["p_tor3"] = 10.0
    assert Oracle(s, p).energy()[T["tor"]] == pytest.approx(e_of(1.0), rel=1e-12)
    p.general["p_tor3"] = 0.0
    p.general["p_tor4"] = 2.0
    f11 = 3.0 / (2.0 + math.exp(2.0 * D))
    assert Oracle(s, p).energy()[T["tor"]] == pytest.approx(e_of(f11), rel=1e-12)


def test_conjugation_amplitude(params):
    """omega = 0: E_conj = p_cot1 prod_b e^{-p_cot2 (BOA_b - 1.5)^2}; p_cot2 = 0 leaves p_cot1."""
    s = _chain(0.0)
    p = _chain_params(params)
    p.tors["p_cot1"][:] = -1.25
    p.general["p_cot2"] = 0.0
    o = Oracle(s, p)
    assert o.energy()[T["conj"]] == pytest.approx(-1.25, rel=1e-14)
    b = _chain_bonds(o)
    p.general["p_cot2"] = 2.5
    ref = -1.25 * math.prod(math.exp(-2.5 * (x[0] - THB - 1.5) ** 2) for x in b)
    assert Oracle(s, p).energy()[T["conj"]] == pytest.approx(ref, rel=1e-13)


# ---------------------------------------------------------------------------
# bond-order correction with Val != Val_boc
# ---------------------------------------------------------------------------
def test_correction_uses_val_in_f1_and_val_boc_in_f4_f5(params):
    """N-O diatomic with uncorrected order b ~ 1.6, Val(N) = 1, Val(O) = 0.5 (both atoms
    over-coordinated in Delta', so f1 depends on the valences), Val_boc(N) = 3.5,
    Val_boc(O) = 4: Delta'_N = b - 1, Delta'_O = b - 0.5, Delta'boc = b - Val_boc.
    With p_boc3 = 1, p_boc4 = 2 and p_boc5 = 2 b^2 - (b - 4), the f5 exponent (O side)
    vanishes: f5 = 1/2, and the N side's is 0.5: f4 = 1 / (1 + e^{0.5}).  f1 takes the
    asymmetric Delta': f2 = e^{-p_boc1 d_N} + e^{-p_boc1 d_O},
    f3 = -ln((e^{-p_boc2 d_N} + e^{-p_boc2 d_O}) / 2) / p_boc2,
    f1 = ((1 + f2)/(1 + f2 + f3) + (0.5 + f2)/(0.5 + f2 + f3)) / 2."""
    p = copy.deepcopy(params)
    p.atom["val"][N] = 1.0
    p.atom["val"][O] = 0.5
    p.atom["val_boc"][N] = 3.5
    s = mol([[0, 0, 0], [1.3, 0, 0]], [N, O])
    o = Oracle(s, p)
    b = o.bond_terms()[0, 3]
    assert b > 1.0
    at = o.atom_terms()
    assert at[0, 0] == pytest.approx(b - 1.0, rel=1e-15)
    assert at[1, 0] == pytest.approx(b - 0.5, rel=1e-15)
    assert at[0, 1] == pytest.approx(b - 3.5, rel=1e-15)
    assert at[1, 1] == pytest.approx(b - 4.0, rel=1e-15)
    p.pair["p_boc3"][N, O] = p.pair["p_boc3"][O, N] = 1.0
    p.pair["p_boc4"][N, O] = p.pair["p_boc4"][O, N] = 2.0
    p.pair["p_boc5"][N, O] = p.pair["p_boc5"][O, N] = 2.0 * b * b - (b - 4.0)
    o = Oracle(s, p)
    bt = o.bond_terms()[0]
    pb1, pb2 = p.general["p_boc1"], p.general["p_boc2"]
    dN, dO = b - 1.0, b - 0.5
    f2 = math.exp(-pb1 * dN) + math.exp(-pb1 * dO)
    f3 = -math.log(0.5 * (math.exp(-pb2 * dN) + math.exp(-pb2 * dO))) / pb2
    f1 = 0.5 * ((1 + f2) / (1 + f2 + f3) + (0.5 + f2) / (0.5 + f2 + f3))
    assert f1 < 0.8             # far from 1: the valences matter
    f45 = 0.5 / (1.0 + math.exp(0.5))
    assert bt[0] == pytest.approx(b * f1 * f45, rel=1e-12)
    assert bt[1] == pytest.approx(bt[5] * f1 * f1 * f45, rel=1e-12)


@pytest.mark.parametrize("eps", [1e-3, 1e-6])
def test_near_straight_angle_forces_match_complex_step(params, eps):
    """Reverse-mode forces equal the complex-step derivatives next to a straight
    angle (the differentiation of the angle from |a x b| and a . b)."""
    s = near_straight_chain(eps)
    o = Oracle(s, params)
    e, f = o.forces()
    assert e[4] != 0.0 and e[7] != 0.0          # a valence angle and a torsion are present
    fcs = np.zeros_like(f)
    for a in range(s.n):
        for k in range(3):
            _, d = o.energy_cs(a, k)
            fcs[a, k] = -d.sum()
    scale = np.abs(fcs).max()
    assert np.abs(f - fcs).max() <= 1e-10 * scale, np.abs(f - fcs).max() / scale


def _rotation(seed):
    q = np.random.default_rng(seed).normal(size=4)
    a, b, c, d = q / np.linalg.norm(q)
    return np.array([[a * a + b * b - c * c - d * d, 2 * (b * c - a * d), 2 * (b * d + a * c)],
                     [2 * (b * c + a * d), a * a - b * b + c * c - d * d, 2 * (c * d - a * b)],
                     [2 * (b * d - a * c), 2 * (c * d + a * b), a * a - b * b - c * c + d * d]])


@pytest.mark.parametrize("eps", [1e-6, 1e-7, 1e-8])
def test_near_straight_angle_forces_rotate_with_the_molecule(params, eps):
    """Forces turn with the molecule up to the conditioning of the geometry
    itself: an offset of eps from a straight line fixes the bend direction only
    to about (rounding of the positions) / eps.  The angle's derivative from
    |a x b| and a . b stays within that (errors ~1e-17/eps of the largest
    force); the arccosine of the cosine, whose derivative divides by
    sqrt(1 - cos^2), misses it by far near a straight angle (~1e-23/eps^2)."""
    s = near_straight_chain(eps)
    _, f = Oracle(s, params).forces()
    worst = 0.0
    for seed in range(5):
        R = _rotation(seed)
        sr = rs.System(pos=s.pos @ R.T + 1.0, type=s.type, q=s.q, box=None)
        _, fr = Oracle(sr, params).forces()
        worst = max(worst, np.abs(fr - f @ R.T).max() / np.abs(f).max())
    assert worst <= max(5e-17 / eps, 1e-12), worst
