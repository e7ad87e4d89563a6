"""Seeded synthetic inputs for the ReaxFF force evaluation.

This module is data only.  It draws force-field parameters from stated
plausibility ranges and builds atom configurations, charges and velocities.
It holds none of the ReaxFF arithmetic: both the CPU oracle and the HIP path
consume the tables it returns and compute everything else themselves.

The paper (Aktulga et al., arXiv:1706.07772) benchmarks on the LAMMPS PETN
crystal (Section 4) with a ReaxFF parameter file that is not available here.
The inputs below stand in for it: PETN stoichiometry C5H8N4O12 (29 atoms per
unit), PETN-like number density, a jittered simple-cubic lattice, and
parameters drawn from seed.  Element order everywhere: C=0, H=1, N=2, O=3.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

ELEMENTS = ("C", "H", "N", "O")
NTYPES = 4
C, H, N, O = 0, 1, 2, 3

#: atoms of each element in one C5H8N4O12 unit (PETN stoichiometry)
PETN_UNIT = (5, 8, 4, 12)
PETN_UNIT_ATOMS = sum(PETN_UNIT)  # 29
#: number density of the synthetic crystal and clusters, atoms / A^3
DENSITY = 0.098

#: names of the general (global) parameters, in a fixed order
GENERAL_NAMES = (
    "p_boc1", "p_boc2", "p_coa2", "p_coa3", "p_coa4", "p_ovun3", "p_ovun4",
    "p_ovun6", "p_ovun7", "p_ovun8", "p_val6", "p_val8", "p_val9", "p_val10",
    "p_pen2", "p_pen3", "p_pen4", "p_tor2", "p_tor3", "p_tor4", "p_cot2",
    "p_vdW1", "p_lp1",
)
ATOM_NAMES = (
    "val", "val_e", "val_boc", "val_ang", "mass", "p_hbond", "p_lp2",
    "p_ovun2", "p_ovun5", "p_val3", "p_val5",
)
PAIR_NAMES = (
    "r_s", "r_p", "r_pp", "D_s", "D_p", "D_pp", "p_be1", "p_be2",
    "p_bo1", "p_bo2", "p_bo3", "p_bo4", "p_bo5", "p_bo6", "p_ovun1",
    "p_boc3", "p_boc4", "p_boc5",
    "D_vdw", "r_vdw", "alpha", "gamma_w", "gamma", "r_core", "e_core", "a_core",
)
ANGLE_NAMES = ("theta00", "p_val1", "p_val2", "p_val4", "p_val7", "p_pen1", "p_coa1")
TORS_NAMES = ("V1", "V2", "V3", "p_tor1", "p_cot1")
HB_NAMES = ("r0hb", "p_hb1", "p_hb2", "p_hb3")

#: default cutoffs (A) and bond-order thresholds
DEFAULT_CUTOFFS = {
    "r_nonb": 10.0,    # nonbonded cutoff, 7th-order taper reaches zero here
    "r_bond": 5.0,     # bond-candidate distance
    "r_hb": 7.5,       # hydrogen-bond acceptor distance
    "bo_cut": 0.01,    # uncorrected bond-order threshold for the bond list
    "thb_cut": 0.001,  # bond-order threshold inside angles and torsions
    "thb_cutsq": 1e-5, # product threshold for angles
    "hb_bo_cut": 0.01, # donor bond-order threshold for hydrogen bonds
}


@dataclass
class Params:
    """Full ReaxFF parameter tables for the four elements.

    general: dict name -> float
    atom:    dict name -> array (4,)
    pair:    dict name -> array (4,4), symmetric
    angle:   dict name -> array (4,4,4) indexed [i, j=centre, k], symmetric in i,k
    tors:    dict name -> array (4,4,4,4) indexed [i,j,k,l], symmetric under reversal
    hb:      dict name -> array (4,4,4) indexed [X, H, Z]; only X,Z in {N,O}, H centre used
    """

    general: dict
    atom: dict
    pair: dict
    angle: dict
    tors: dict
    hb: dict
    seed: int = 0


def _u(rng, lo, hi, size=None):
    return rng.uniform(lo, hi, size=size)


def draw_params(seed: int = 0) -> Params:
    """Draw a C/H/N/O parameter set from seed within fixed plausibility ranges.

    The ranges give each term its physical role (attractive bonds, repulsive
    over-coordination, bent-angle equilibria near 100-125 degrees, and so on);
    they are not values from any published force-field file.
    """
    rng = np.random.default_rng(np.random.PCG64(seed))
    g = {}
    general_ranges = {
        "p_boc1": (40, 60), "p_boc2": (8, 12),
        "p_coa2": (20, 30), "p_coa3": (1, 3), "p_coa4": (2, 4),
        "p_ovun3": (30, 60), "p_ovun4": (5, 8), "p_ovun6": (1, 2),
        "p_ovun7": (8, 12), "p_ovun8": (10, 15),
        "p_val6": (30, 40), "p_val8": (1, 2), "p_val9": (1.0, 1.1), "p_val10": (1.5, 2.5),
        "p_pen2": (5, 8), "p_pen3": (0.3, 0.5), "p_pen4": (3, 5),
        "p_tor2": (5, 6), "p_tor3": (9, 11), "p_tor4": (1.5, 2.5), "p_cot2": (2, 3),
        "p_vdW1": (1.5, 1.6), "p_lp1": (5, 7),
    }
    for name in GENERAL_NAMES:
        lo, hi = general_ranges[name]
        g[name] = float(_u(rng, lo, hi))

    heavy = np.array([True, False, True, True])
    a = {
        "val": np.array([4.0, 1.0, 3.0, 2.0]),
        "val_e": np.array([4.0, 1.0, 5.0, 6.0]),
        "val_boc": np.array([4.0, 1.0, 4.0, 4.0]),
        "val_ang": np.array([4.0, 1.0, 4.0, 4.0]),
        "mass": np.array([12.011, 1.008, 14.007, 15.999]),
        "p_hbond": np.array([0.0, 1.0, 2.0, 2.0]),
    }
    # per-element radii; a non-positive radius means "no such bond component"
    r_s = np.where(heavy, _u(rng, 1.20, 1.45, 4), _u(rng, 0.75, 0.95, 4))
    r_p = np.where(heavy, _u(rng, 1.05, 1.25, 4), -1.0)
    r_pp = np.where(heavy, _u(rng, 0.90, 1.15, 4), -1.0)
    r_vdw = _u(rng, 1.4, 2.1, 4)
    eps = _u(rng, 0.02, 0.20, 4)
    alpha = _u(rng, 9, 11, 4)
    gamma_w = _u(rng, 1.5, 8, 4)
    gamma = _u(rng, 0.7, 1.1, 4)
    p_boc3 = _u(rng, 1, 8, 4)
    p_boc4 = _u(rng, 1, 10, 4)
    p_boc5 = _u(rng, 0, 10, 4)
    a["p_lp2"] = np.where(heavy & (np.arange(4) >= 2), _u(rng, 0.5, 5, 4), 0.0)
    a["p_ovun2"] = _u(rng, -16, -3, 4)
    a["p_ovun5"] = _u(rng, 0, 40, 4)
    a["p_val3"] = _u(rng, 1, 3, 4)
    a["p_val5"] = _u(rng, 2, 3, 4)
    r_core = _u(rng, 1, 2, 4)
    e_core = _u(rng, 0, 0.2, 4)
    a_core = _u(rng, 5, 15, 4)

    p = {name: np.zeros((4, 4)) for name in PAIR_NAMES}
    pair_ranges = {
        "D_s": (70, 160), "D_p": (0, 150), "D_pp": (0, 60),
        "p_be1": (-1, 1), "p_be2": (0.2, 1.5),
        "p_bo1": (-0.2, -0.05), "p_bo2": (5, 9), "p_bo3": (-0.4, -0.1),
        "p_bo4": (5, 12), "p_bo5": (-0.4, -0.1), "p_bo6": (10, 40),
        "p_ovun1": (0.1, 1),
    }
    for i in range(4):
        for j in range(i, 4):
            vals = {}
            for name in ("D_s", "D_p", "D_pp", "p_be1", "p_be2", "p_bo1", "p_bo2",
                         "p_bo3", "p_bo4", "p_bo5", "p_bo6", "p_ovun1"):
                lo, hi = pair_ranges[name]
                vals[name] = float(_u(rng, lo, hi))
            if i == H or j == H:
                vals["D_p"] = 0.0
                vals["D_pp"] = 0.0
            # mixing rules of the synthetic set
            vals["r_s"] = 0.5 * (r_s[i] + r_s[j]) if (r_s[i] > 0 and r_s[j] > 0) else 0.0
            vals["r_p"] = 0.5 * (r_p[i] + r_p[j]) if (r_p[i] > 0 and r_p[j] > 0) else 0.0
            vals["r_pp"] = 0.5 * (r_pp[i] + r_pp[j]) if (r_pp[i] > 0 and r_pp[j] > 0) else 0.0
            vals["p_boc3"] = math.sqrt(p_boc3[i] * p_boc3[j])
            vals["p_boc4"] = math.sqrt(p_boc4[i] * p_boc4[j])
            vals["p_boc5"] = math.sqrt(p_boc5[i] * p_boc5[j])
            vals["D_vdw"] = math.sqrt(eps[i] * eps[j])
            vals["r_vdw"] = 2.0 * math.sqrt(r_vdw[i] * r_vdw[j])
            vals["alpha"] = math.sqrt(alpha[i] * alpha[j])
            vals["gamma_w"] = math.sqrt(gamma_w[i] * gamma_w[j])
            vals["gamma"] = math.sqrt(gamma[i] * gamma[j])
            vals["r_core"] = math.sqrt(r_core[i] * r_core[j])
            vals["e_core"] = math.sqrt(e_core[i] * e_core[j])
            vals["a_core"] = math.sqrt(a_core[i] * a_core[j])
            for name in PAIR_NAMES:
                p[name][i, j] = p[name][j, i] = vals[name]

    ang = {name: np.zeros((4, 4, 4)) for name in ANGLE_NAMES}
    angle_ranges = {
        "theta00": (55, 80), "p_val1": (10, 45), "p_val2": (0.5, 8),
        "p_val4": (1, 3), "p_val7": (0.5, 3), "p_pen1": (0, 60), "p_coa1": (-25, 0),
    }
    for j in range(4):
        for i in range(4):
            for k in range(i, 4):
                for name in ANGLE_NAMES:
                    lo, hi = angle_ranges[name]
                    v = float(_u(rng, lo, hi))
                    ang[name][i, j, k] = ang[name][k, j, i] = v

    tor = {name: np.zeros((4, 4, 4, 4)) for name in TORS_NAMES}
    tors_ranges = {"V1": (-2, 2), "V2": (0, 80), "V3": (0, 1), "p_tor1": (-10, -2), "p_cot1": (-2, 0)}
    for i in range(4):
        for j in range(4):
            for k in range(4):
                for l in range(4):
                    if (i, j, k, l) > (l, k, j, i):
                        continue  # drawn with its reversal
                    for name in TORS_NAMES:
                        lo, hi = tors_ranges[name]
                        v = float(_u(rng, lo, hi))
                        tor[name][i, j, k, l] = tor[name][l, k, j, i] = v

    hb = {name: np.zeros((4, 4, 4)) for name in HB_NAMES}
    hb_ranges = {"r0hb": (1.8, 2.2), "p_hb1": (-5, -1), "p_hb2": (1, 20), "p_hb3": (10, 30)}
    for x in (N, O):
        for z in (N, O):
            for name in HB_NAMES:
                lo, hi = hb_ranges[name]
                hb[name][x, H, z] = float(_u(rng, lo, hi))

    return Params(general=g, atom=a, pair=p, angle=ang, tors=tor, hb=hb, seed=seed)


def draw_qeq_params(seed: int = 0) -> dict:
    """Charge-equilibration parameters per element (C, H, N, O), from their own
    seeded stream (the force-field draw above is unchanged by them).

    chi: electronegativity, kcal/(mol e), in element ranges around 5-9 eV;
    J:   self-Coulomb (twice the hardness), kcal/(mol e^2), 330-420 (14-18 eV),
         which keeps the charge-equilibration matrix of the PETN-density
         lattices positive definite (its off-diagonal part has eigenvalues down
         to about -250 there).
    The shielding gamma of each pair is the force field's Coulomb gamma.
    """
    rng = np.random.default_rng(np.random.SeedSequence([seed, 7]))
    chi_ranges = ((115, 145), (75, 105), (135, 165), (180, 210))
    chi = np.array([float(_u(rng, lo, hi)) for lo, hi in chi_ranges])
    J = np.array([float(_u(rng, 330, 420)) for _ in range(4)])
    return {"chi": chi, "J": J}


@dataclass
class System:
    """One atom configuration.

    pos  (n,3) float64, A;  type (n,) int32 in 0..3;  q (n,) float64, e;
    box  (3,) float64 edge lengths of a periodic orthorhombic box at the origin,
         or None for a non-periodic system.
    """

    pos: np.ndarray
    type: np.ndarray
    q: np.ndarray
    box: np.ndarray | None
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])


def _petn_labels(n_units: int, rng) -> np.ndarray:
    labels = np.repeat(np.arange(4, dtype=np.int32), PETN_UNIT)
    labels = np.tile(labels, n_units)
    rng.shuffle(labels)
    return labels


def _neutral_charges(n: int, rng) -> np.ndarray:
    q = rng.uniform(-0.5, 0.5, size=n)
    return q - q.mean()


def petn_lattice(n_units: int, box_edge: float, seed: int, jitter: float = 0.3) -> System:
    """PETN-stoichiometry atoms on a jittered simple-cubic lattice in a periodic cube.

    n = ceil(N^(1/3)) sites per edge at spacing box_edge/n; N of the n^3 sites
    are chosen by a seeded permutation; each site is (g + 1/2) a plus a uniform
    jitter in [-jitter, jitter]^3, wrapped into the box.  Element labels are
    n_units copies of C5H8N4O12 shuffled by seed; charges are uniform in
    [-0.5, 0.5] e shifted to zero net charge.
    """
    rng = np.random.default_rng(np.random.PCG64(seed))
    natoms = n_units * PETN_UNIT_ATOMS
    nside = int(math.ceil(round(natoms ** (1.0 / 3.0), 12)))
    while nside ** 3 < natoms:
        nside += 1
    a = box_edge / nside
    sites = rng.permutation(nside ** 3)[:natoms]
    g = np.stack(np.unravel_index(sites, (nside, nside, nside)), axis=1).astype(np.float64)
    pos = (g + 0.5) * a + rng.uniform(-jitter, jitter, size=(natoms, 3))
    pos = np.mod(pos, box_edge)
    pos[pos >= box_edge] -= box_edge
    typ = _petn_labels(n_units, rng)
    q = _neutral_charges(natoms, rng)
    return System(pos=pos, type=typ, q=q, box=np.full(3, float(box_edge)),
                  meta={"n_units": n_units, "box": box_edge, "seed": seed,
                        "lattice": nside, "spacing": a})


def cluster(n: int, seed: int | None = None, rng=None, jitter: float = 0.3,
            probs=(0.17, 0.28, 0.14, 0.41)) -> System:
    """One non-periodic cluster of n atoms at the crystal's number density.

    Spacing a = DENSITY^(-1/3); n_side = ceil(n^(1/3)); n random sites of the
    n_side^3 lattice, jittered uniformly by +-jitter; elements i.i.d. with the
    given C/H/N/O probabilities; charges uniform and neutralised per cluster.
    """
    if rng is None:
        rng = np.random.default_rng(np.random.PCG64(seed))
    a = DENSITY ** (-1.0 / 3.0)
    nside = int(math.ceil(round(n ** (1.0 / 3.0), 12)))
    while nside ** 3 < n:
        nside += 1
    sites = rng.permutation(nside ** 3)[:n]
    g = np.stack(np.unravel_index(sites, (nside, nside, nside)), axis=1).astype(np.float64)
    pos = (g + 0.5) * a + rng.uniform(-jitter, jitter, size=(n, 3))
    typ = rng.choice(4, size=n, p=np.asarray(probs)).astype(np.int32)
    q = _neutral_charges(n, rng)
    return System(pos=pos, type=typ, q=q, box=None, meta={"seed": seed, "lattice": nside})


def cluster_batch(nsys: int, seed: int = 3, lo: int = 10, hi: int = 300):
    """nsys independent clusters with sizes uniform in [lo, hi].

    Returns (pos (T,3), type (T,), q (T,), offsets (nsys+1,) int64).
    """
    rng = np.random.default_rng(np.random.PCG64(seed))
    sizes = rng.integers(lo, hi + 1, size=nsys)
    parts = [cluster(int(s), rng=rng) for s in sizes]
    off = np.zeros(nsys + 1, dtype=np.int64)
    off[1:] = np.cumsum(sizes)
    pos = np.concatenate([p.pos for p in parts])
    typ = np.concatenate([p.type for p in parts]).astype(np.int32)
    q = np.concatenate([p.q for p in parts])
    return pos, typ, q, off


def maxwell_boltzmann(types: np.ndarray, mass: np.ndarray, temp: float, seed: int) -> np.ndarray:
    """Velocities (A/fs) drawn at temperature temp (K), centre-of-mass motion removed,
    rescaled to exactly temp with 3N-3 degrees of freedom.

    Units: k_B = 0.0019872043 kcal/(mol K); m v^2 [g/mol A^2/fs^2] = 1/4.184e-4 kcal/mol.
    """
    kb = 0.0019872043
    conv = 4.184e-4
    rng = np.random.default_rng(np.random.PCG64(seed))
    m = mass[types]
    sigma = np.sqrt(kb * temp * conv / m)
    v = rng.normal(size=(types.size, 3)) * sigma[:, None]
    vcom = (m[:, None] * v).sum(0) / m.sum()
    v -= vcom
    ke = 0.5 * (m[:, None] * v * v).sum() / conv
    dof = 3 * types.size - 3
    t_now = 2.0 * ke / (dof * kb)
    v *= math.sqrt(temp / t_now)
    return v


# ---------------------------------------------------------------------------
# The five benchmark workloads (sizes from the PETN benchmark family: 32,480
# atoms is the paper's smallest PETN size; 1,044,000 = 36,000 units).
# ---------------------------------------------------------------------------
WORKLOADS = {
    "petn_1856": dict(n_units=64, box=26.7, seed=0),
    "petn_32480": dict(n_units=1120, box=69.2, seed=1),
    "petn_1044000": dict(n_units=36000, box=220.0, seed=2),
}


def workload(name: str) -> System:
    w = WORKLOADS[name]
    return petn_lattice(w["n_units"], w["box"], w["seed"])


def thermal_frame(n_units: int, box: float, seed: int, temp: float, k_eff: float = 100.0) -> System:
    """A training frame at temperature temp (K): the lattice recipe (its 0.3 A jitter),
    then every atom displaced by an isotropic Gaussian of standard deviation
    sqrt(k_B T / k_eff) per component (a harmonic-well stand-in for thermal motion;
    k_eff in kcal/(mol A^2)), wrapped into the box."""
    s = petn_lattice(n_units, box, seed)
    rng = np.random.default_rng(np.random.PCG64(seed + 7919))
    sigma = math.sqrt(0.0019872043 * temp / k_eff)
    pos = s.pos + rng.normal(scale=sigma, size=s.pos.shape)
    pos -= box * np.floor(pos / box)
    return System(pos=pos, type=s.type, q=s.q, box=s.box, meta=dict(s.meta, temp=temp))


def small_periodic(n_units: int, seed: int, box: float | None = None) -> System:
    """A periodic PETN-stoichiometry box at the crystal density (edge >= 20 A)."""
    natoms = n_units * PETN_UNIT_ATOMS
    if box is None:
        box = (natoms / DENSITY) ** (1.0 / 3.0)
    return petn_lattice(n_units, box, seed)
