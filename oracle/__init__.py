"""ctypes wrapper of the CPU oracle -- test infrastructure only.

The oracle is a plain single-threaded FP64 ReaxFF written from the energy's
definition (see reaxff_oracle.cpp).  Only tests, the build check and the
CPU-baseline timing of the benchmark import this module; the GPU library and
its Python binding never do.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from reaxff_synth import (ANGLE_NAMES, ATOM_NAMES, DEFAULT_CUTOFFS, GENERAL_NAMES,
                          HB_NAMES, PAIR_NAMES, TORS_NAMES, Params, System)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
NTERMS = 12
TERM_NAMES = ("bond", "lp", "over", "under", "val", "pen", "coa", "tor", "conj",
              "hb", "vdw", "coul")
CUTOFF_ORDER = ("r_nonb", "r_bond", "r_hb", "bo_cut", "thb_cut", "thb_cutsq", "hb_bo_cut")

_lib = None

_d = ctypes.POINTER(ctypes.c_double)
_i32 = ctypes.POINTER(ctypes.c_int32)
_i64 = ctypes.POINTER(ctypes.c_int64)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        import importlib
        importlib.import_module(__name__ + ".build").build()
    lib = ctypes.CDLL(LIB_PATH)
    lib.oracle_new.restype = ctypes.c_void_p
    lib.oracle_new.argtypes = [ctypes.c_int32, _d, _i32, _d, _d, _d, _d, _d, _d, _d, _d, _d,
                               ctypes.c_int32]
    lib.oracle_free.argtypes = [ctypes.c_void_p]
    lib.oracle_error.restype = ctypes.c_char_p
    lib.oracle_set_positions.argtypes = [ctypes.c_void_p, _d]
    lib.oracle_list_sizes.argtypes = [ctypes.c_void_p, _i64]
    lib.oracle_get_lists.argtypes = [ctypes.c_void_p, _i32, _i32, _i32]
    lib.oracle_bo_raw.restype = ctypes.c_double
    lib.oracle_bo_raw.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32]
    lib.oracle_energy.argtypes = [ctypes.c_void_p, _d]
    lib.oracle_forces.argtypes = [ctypes.c_void_p, _d, _d]
    lib.oracle_energy_abs.argtypes = [ctypes.c_void_p, _d, _d]
    lib.oracle_energy_cs.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_double, _d, _d]
    lib.oracle_atom_terms.argtypes = [ctypes.c_void_p, _d]
    lib.oracle_bond_terms.argtypes = [ctypes.c_void_p, _d]
    lib.oracle_md.argtypes = [ctypes.c_void_p, _d, _d, ctypes.c_double, ctypes.c_int32, _d]
    lib.oracle_param_counts.argtypes = [_i32]
    counts = np.zeros(6, dtype=np.int32)
    lib.oracle_param_counts(counts.ctypes.data_as(_i32))
    expect = [len(GENERAL_NAMES), len(ATOM_NAMES), len(PAIR_NAMES), len(ANGLE_NAMES),
              len(TORS_NAMES), len(HB_NAMES)]
    if list(counts) != expect:
        raise RuntimeError(f"oracle parameter layout {list(counts)} != {expect}")
    _lib = lib
    return lib


def _ptr(a, t=_d):
    return a.ctypes.data_as(t)


def param_blocks(p: Params):
    """Flatten a parameter set into the oracle's name-major blocks."""
    g = np.array([p.general[k] for k in GENERAL_NAMES], dtype=np.float64)
    a = np.ascontiguousarray(np.stack([p.atom[k] for k in ATOM_NAMES]), dtype=np.float64)
    pr = np.ascontiguousarray(np.stack([p.pair[k] for k in PAIR_NAMES]), dtype=np.float64)
    an = np.ascontiguousarray(np.stack([p.angle[k] for k in ANGLE_NAMES]), dtype=np.float64)
    to = np.ascontiguousarray(np.stack([p.tors[k] for k in TORS_NAMES]), dtype=np.float64)
    hb = np.ascontiguousarray(np.stack([p.hb[k] for k in HB_NAMES]), dtype=np.float64)
    return g, a, pr, an, to, hb


class Oracle:
    """One system held by the oracle, with its lists built at construction."""

    def __init__(self, system: System, params: Params, cutoffs: dict | None = None,
                 brute: bool = False):
        lib = _load()
        self._lib = lib
        cut = dict(DEFAULT_CUTOFFS)
        if cutoffs:
            cut.update(cutoffs)
        self.cutoffs = cut
        self.n = system.n
        self._pos = np.ascontiguousarray(system.pos, dtype=np.float64)
        self._type = np.ascontiguousarray(system.type, dtype=np.int32)
        self._q = np.ascontiguousarray(system.q, dtype=np.float64)
        self._blocks = param_blocks(params)
        self._cut = np.array([cut[k] for k in CUTOFF_ORDER], dtype=np.float64)
        box = None if system.box is None else np.ascontiguousarray(system.box, dtype=np.float64)
        self._box = box
        g, a, pr, an, to, hb = self._blocks
        self._h = lib.oracle_new(self.n, _ptr(self._pos), _ptr(self._type, _i32), _ptr(self._q),
                                 None if box is None else _ptr(box), _ptr(g), _ptr(a), _ptr(pr),
                                 _ptr(an), _ptr(to), _ptr(hb), _ptr(self._cut), int(brute))
        if not self._h:
            raise ValueError("oracle: " + lib.oracle_error().decode())

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.oracle_free(h)
            self._h = None

    def set_positions(self, pos):
        self._pos = np.ascontiguousarray(pos, dtype=np.float64)
        self._lib.oracle_set_positions(self._h, _ptr(self._pos))

    def lists(self):
        """(far (M,2) i<j, bonds (B,2) directed, hb (K,2) (h,z)), each int32, sorted."""
        sz = np.zeros(3, dtype=np.int64)
        self._lib.oracle_list_sizes(self._h, _ptr(sz, _i64))
        far = np.zeros((int(sz[0]), 2), dtype=np.int32)
        bonds = np.zeros((int(sz[1]), 2), dtype=np.int32)
        hb = np.zeros((int(sz[2]), 2), dtype=np.int32)
        self._lib.oracle_get_lists(self._h, _ptr(far, _i32), _ptr(bonds, _i32), _ptr(hb, _i32))
        return far, bonds, hb

    def bo_raw(self, i: int, j: int) -> float:
        return float(self._lib.oracle_bo_raw(self._h, int(i), int(j)))

    def energy(self) -> np.ndarray:
        e = np.zeros(NTERMS)
        self._lib.oracle_energy(self._h, _ptr(e))
        return e

    def energy_abs(self):
        """(energies (12,), sum of |interaction energy| per term (12,))."""
        e = np.zeros(NTERMS)
        a = np.zeros(NTERMS)
        self._lib.oracle_energy_abs(self._h, _ptr(e), _ptr(a))
        return e, a

    def forces(self):
        """(energies (12,), forces (n,3)) with F = -dE/dx."""
        e = np.zeros(NTERMS)
        f = np.zeros((self.n, 3))
        self._lib.oracle_forces(self._h, _ptr(e), _ptr(f))
        return e, f

    def energy_cs(self, atom: int, comp: int, h: float = 1e-30):
        """Complex-step derivative of every energy term w.r.t. x[atom, comp]."""
        er = np.zeros(NTERMS)
        ei = np.zeros(NTERMS)
        rc = self._lib.oracle_energy_cs(self._h, int(atom), int(comp), float(h), _ptr(er), _ptr(ei))
        if rc != 0:
            raise ValueError(self._lib.oracle_error().decode())
        return er, ei / h

    def atom_terms(self) -> np.ndarray:
        """(n,8): Delta', Delta'boc, S, Delta, nlp, Delta_lp, SBO, SBO2."""
        out = np.zeros((self.n, 8))
        self._lib.oracle_atom_terms(self._h, _ptr(out))
        return out

    def bond_terms(self) -> np.ndarray:
        """(B,7) per directed bond: BO, BOpi, BOpipi (corrected), BO' (shifted total),
        BO'sigma (shifted), BO'pi, BO'pipi."""
        sz = np.zeros(3, dtype=np.int64)
        self._lib.oracle_list_sizes(self._h, _ptr(sz, _i64))
        out = np.zeros((int(sz[1]), 7))
        self._lib.oracle_bond_terms(self._h, _ptr(out))
        return out

    def md(self, vel, dt: float, nsteps: int):
        """Velocity-Verlet NVE from the current positions; returns (pos, vel, energies)
        with energies (nsteps+1, 13): 12 potential terms and the kinetic energy."""
        pos = self._pos.copy()
        v = np.ascontiguousarray(vel, dtype=np.float64).copy()
        e = np.zeros((nsteps + 1, NTERMS + 1))
        self._lib.oracle_md(self._h, _ptr(pos), _ptr(v), float(dt), int(nsteps), _ptr(e))
        self._pos = pos
        return pos, v, e

