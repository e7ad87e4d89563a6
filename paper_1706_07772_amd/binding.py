"""Thin ctypes binding of the gfx950 ReaxFF library (include/reaxff.h).

Argument marshalling only: every step of the force evaluation runs in the
HIP kernels of libreaxff_hip.so.  PyTorch supplies device memory and the
current stream.  If the library is missing, loading fails loudly; there is
no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libreaxff_hip.so")
NTERMS = 12
TERM_NAMES = ("bond", "lp", "over", "under", "val", "pen", "coa", "tor", "conj",
              "hb", "vdw", "coul")

ERRORS = {0: "ok", -1: "REAXFF_ERR_ARG", -2: "REAXFF_ERR_CAPACITY", -3: "REAXFF_ERR_BOX",
          -4: "REAXFF_ERR_HIP", -5: "REAXFF_ERR_NONFINITE", -6: "REAXFF_ERR_STATE",
          -7: "REAXFF_ERR_CONVERGENCE"}

_GENERAL = ("p_boc1", "p_boc2", "p_coa2", "p_coa3", "p_coa4", "p_ovun3", "p_ovun4", "p_ovun6",
            "p_ovun7", "p_ovun8", "p_val6", "p_val8", "p_val9", "p_val10", "p_pen2", "p_pen3",
            "p_pen4", "p_tor2", "p_tor3", "p_tor4", "p_cot2", "p_vdW1", "p_lp1")
_ATOM = ("val", "val_e", "val_boc", "val_ang", "mass", "p_hbond", "p_lp2", "p_ovun2", "p_ovun5",
         "p_val3", "p_val5")
_PAIR = ("r_s", "r_p", "r_pp", "D_s", "D_p", "D_pp", "p_be1", "p_be2", "p_bo1", "p_bo2", "p_bo3",
         "p_bo4", "p_bo5", "p_bo6", "p_ovun1", "p_boc3", "p_boc4", "p_boc5", "D_vdw", "r_vdw",
         "alpha", "gamma_w", "gamma", "r_core", "e_core", "a_core")
_ANGLE = ("theta00", "p_val1", "p_val2", "p_val4", "p_val7", "p_pen1", "p_coa1")
_TORS = ("V1", "V2", "V3", "p_tor1", "p_cot1")
_HB = ("r0hb", "p_hb1", "p_hb2", "p_hb3")

_d = ctypes.c_double
_fields = ([(k, _d) for k in _GENERAL] + [(k, _d * 4) for k in _ATOM] +
           [(k, (_d * 4) * 4) for k in _PAIR] + [(k, ((_d * 4) * 4) * 4) for k in _ANGLE] +
           [(k, (((_d * 4) * 4) * 4) * 4) for k in _TORS] + [(k, ((_d * 4) * 4) * 4) for k in _HB])


class CParams(ctypes.Structure):
    _fields_ = _fields


class CCutoffs(ctypes.Structure):
    _fields_ = [(k, _d) for k in ("r_nonb", "r_bond", "r_hb", "bo_cut", "thb_cut", "thb_cutsq",
                                  "hb_bo_cut")]


class CLists(ctypes.Structure):
    """reaxff_lists: caller-owned list buffers and the sizes a build requires."""
    _fields_ = [("far_cap", ctypes.c_int64), ("far_j", ctypes.c_void_p),
                ("bond_cap", ctypes.c_int64), ("bond_j", ctypes.c_void_p), ("bond_mir", ctypes.c_void_p),
                ("hb_cap", ctypes.c_int64), ("hb_j", ctypes.c_void_p),
                ("required", ctypes.c_int64 * 3)]


class ListBuffers:
    """Device buffers (int32 torch tensors) for reaxff_build_lists_into."""

    def __init__(self, far: int = 0, bond: int = 0, hb: int = 0, device="cuda:0"):
        self.device = device
        self.resize(far, bond, hb)

    def resize(self, far: int, bond: int, hb: int):
        mk = lambda k: torch.empty(max(int(k), 1), dtype=torch.int32, device=self.device)
        self.far, self.bond, self.mir, self.hb = mk(far), mk(bond), mk(bond), mk(hb)
        self.c = CLists(int(far), self.far.data_ptr(), int(bond), self.bond.data_ptr(), self.mir.data_ptr(),
                        int(hb), self.hb.data_ptr())

    @property
    def required(self):
        return tuple(int(x) for x in self.c.required)


class QeqParams(ctypes.Structure):
    """reaxff_qeq_params: electronegativity chi and self-Coulomb J per element."""
    _fields_ = [("chi", _d * 4), ("J", _d * 4)]


class BatchConfig(ctypes.Structure):
    """reaxff_batch_config: threads per workgroup, schedule, workgroups per CU."""
    _fields_ = [("block", ctypes.c_int32), ("schedule", ctypes.c_int32),
                ("wg_per_cu", ctypes.c_int32)]

    def as_tuple(self):
        return (int(self.block), int(self.schedule), int(self.wg_per_cu))


SCHEDULES = {0: "static", 1: "lpt", 2: "dynamic"}
BATCH_MAX_ATOMS = 384

_lib = None


def load_library():
    """Load libreaxff_hip.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    lib.reaxff_params_size.restype = i64
    lib.reaxff_create.argtypes = [ctypes.POINTER(CParams), ctypes.POINTER(CCutoffs), ctypes.c_int,
                                  ctypes.POINTER(vp)]
    lib.reaxff_destroy.argtypes = [vp]
    lib.reaxff_build_lists.argtypes = [vp, i64, vp, vp, vp, vp]
    lib.reaxff_compute_forces.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, vp]
    lib.reaxff_step.argtypes = [vp, i64, vp, vp, vp, vp, vp, _d, i32, vp, vp, vp]
    lib.reaxff_list_sizes.argtypes = [vp, ctypes.POINTER(i64)]
    lib.reaxff_build_lists_into.argtypes = [vp, i64, vp, vp, vp, ctypes.POINTER(CLists), vp]
    lib.reaxff_compute_forces_from.argtypes = [vp, i64, vp, vp, vp, vp, ctypes.POINTER(CLists), vp, vp, vp]
    lib.reaxff_set_skin.argtypes = [vp, _d, i32]
    lib.reaxff_refresh_lists.argtypes = [vp, i64, vp, vp, vp, ctypes.POINTER(i32), vp]
    lib.reaxff_list_stats.argtypes = [vp, ctypes.POINTER(i64)]
    lib.reaxff_export_lists.argtypes = [vp, vp, vp, vp]
    lib.reaxff_interaction_counts.argtypes = [vp, ctypes.POINTER(i64)]
    lib.reaxff_batch_create.argtypes = [vp, i32, vp, vp, ctypes.POINTER(vp)]
    lib.reaxff_batch_destroy.argtypes = [vp]
    lib.reaxff_batch_set_config.argtypes = [vp, ctypes.POINTER(BatchConfig)]
    lib.reaxff_batch_get_config.argtypes = [vp, ctypes.POINTER(BatchConfig)]
    lib.reaxff_batch_compute.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    lib.reaxff_batch_status.argtypes = [vp, ctypes.POINTER(i32)]
    lib.reaxff_batch_counts.argtypes = [vp, vp]
    lib.reaxff_batch_tune.argtypes = [vp, vp, vp, vp, vp, vp, vp, i32, i32, vp, vp,
                                      ctypes.POINTER(i32)]
    lib.reaxff_qeq.argtypes = [vp, i64, ctypes.POINTER(QeqParams), _d, i32, i32, vp, vp, vp,
                               ctypes.POINTER(i32), ctypes.POINTER(_d), vp]
    lib.reaxff_species.argtypes = [vp, _d, vp, vp, vp, ctypes.POINTER(i64), ctypes.POINTER(i64), vp]
    lib.reaxff_compute_forces_batched.argtypes = [vp, i32, vp, i32, vp, vp, vp, vp, vp, vp, vp]
    lib.reaxff_surrogate_param_count.restype = i64
    lib.reaxff_surrogate_create.argtypes = [vp, i32, ctypes.POINTER(vp)]
    lib.reaxff_surrogate_destroy.argtypes = [vp]
    lib.reaxff_surrogate_last_error.restype = ctypes.c_char_p
    lib.reaxff_surrogate_last_error.argtypes = [vp]
    lib.reaxff_surrogate_set_params.argtypes = [vp, vp, vp, vp]
    lib.reaxff_surrogate_get_params.argtypes = [vp, vp, vp, vp]
    lib.reaxff_surrogate_descriptors.argtypes = [vp, i64, vp, vp, vp, vp, vp]
    lib.reaxff_surrogate_evaluate.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.reaxff_surrogate_train_step.argtypes = [vp, i64, vp, vp, vp, _d, vp, _d, _d, _d, vp, vp]
    lib.reaxff_surrogate_get_grad.argtypes = [vp, vp]
    lib.reaxff_surrogate_normaliser.argtypes = [vp, i64, vp, _d, vp, vp, vp]
    lib.reaxff_surrogate_context.restype = vp
    lib.reaxff_surrogate_context.argtypes = [vp]
    lib.reaxff_surrogate_gated_forces.argtypes = [vp, vp, i64, vp, vp, vp, vp, _d, vp, vp, vp,
                                                  ctypes.POINTER(i64), ctypes.POINTER(i64), vp]
    lib.reaxff_dependency_radius.restype = _d
    lib.reaxff_dependency_radius.argtypes = [vp]
    lib.reaxff_forces_masked.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, ctypes.POINTER(i64), vp]
    lib.reaxff_profile.argtypes = [vp, i32]
    lib.reaxff_set_overlap.argtypes = [vp, i32]
    lib.reaxff_set_nb_run.argtypes = [vp, i32]
    lib.reaxff_set_qeq_product.argtypes = [vp, i32]
    lib.reaxff_math_eval.argtypes = [i32, i64, vp, vp, vp, vp]
    lib.reaxff_profile_read.argtypes = [vp, i32, vp, vp, vp]
    lib.reaxff_last_error.restype = ctypes.c_char_p
    lib.reaxff_last_error.argtypes = [vp]
    lib.reaxff_strerror.restype = ctypes.c_char_p
    if lib.reaxff_params_size() != ctypes.sizeof(CParams):
        raise RuntimeError("reaxff_params layout mismatch between binding and library")
    _lib = lib
    return lib


def make_cparams(params) -> CParams:
    """Marshal a parameter set (general/atom/pair/angle/tors/hb tables) into reaxff_params."""
    cp = CParams()
    for k in _GENERAL:
        setattr(cp, k, float(params.general[k]))
    for block, names in ((params.atom, _ATOM), (params.pair, _PAIR), (params.angle, _ANGLE),
                         (params.tors, _TORS), (params.hb, _HB)):
        for k in names:
            arr = np.ascontiguousarray(block[k], dtype=np.float64)
            dst = getattr(cp, k)
            ctypes.memmove(ctypes.addressof(dst), arr.ctypes.data, arr.nbytes)
    return cp


def make_ccutoffs(cutoffs: dict | None) -> CCutoffs | None:
    if cutoffs is None:
        return None
    c = CCutoffs()
    for k, _ in CCutoffs._fields_:
        setattr(c, k, float(cutoffs[k]))
    return c


class ReaxFFError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


#: reaxff_math_eval function codes
MATH_FUNCTIONS = {"exp": 0, "exp_r": 1, "exp_c": 2, "log": 3, "log_r": 4, "pow": 5, "rcbrt": 6, "rcp": 7,
                  "rsqrt": 8}


def math_eval(name: str, x, y=None):
    """reaxff_math_eval: the library's FP64 elementary function `name` on the
    float64 device tensor x (and exponents y for "pow"); returns a new tensor."""
    lib = load_library()
    x = x.contiguous()
    out = torch.empty_like(x)
    if y is not None:
        y = y.contiguous()
    code = lib.reaxff_math_eval(MATH_FUNCTIONS[name], x.numel(), _ptr(x), _ptr(y), _ptr(out), _stream())
    if code != 0:
        raise ReaxFFError(code, "reaxff_math_eval failed")
    return out


class ReaxFF:
    """A library context on one GPU (reaxff_create / reaxff_destroy)."""

    def __init__(self, params, cutoffs: dict | None = None, device: int = 0):
        self._lib = load_library()
        self.device = device
        self._cp = make_cparams(params)
        self._cc = make_ccutoffs(cutoffs)
        h = ctypes.c_void_p()
        rc = self._lib.reaxff_create(ctypes.byref(self._cp),
                                     ctypes.byref(self._cc) if self._cc is not None else None,
                                     device, ctypes.byref(h))
        if rc != 0:
            raise ReaxFFError(rc, "reaxff_create failed")
        self._h = h
        self._box = None

    def close(self):
        if getattr(self, "_h", None):
            self._lib.reaxff_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != 0:
            raise ReaxFFError(rc, self._lib.reaxff_last_error(self._h).decode())

    @staticmethod
    def _boxarg(box):
        if box is None:
            return None, None
        b = (ctypes.c_double * 3)(*[float(x) for x in box])
        return b, ctypes.cast(b, ctypes.c_void_p)

    def build_lists(self, pos: torch.Tensor, type_: torch.Tensor, box=None):
        """reaxff_build_lists: pos (n,3) float64 cuda, type (n,) int32 cuda."""
        assert pos.dtype == torch.float64 and pos.is_cuda and pos.is_contiguous()
        assert type_.dtype == torch.int32 and type_.is_cuda and type_.is_contiguous()
        b, bp = self._boxarg(box)
        self._check(self._lib.reaxff_build_lists(self._h, pos.shape[0], _ptr(pos), _ptr(type_), bp,
                                                 _stream()))

    def build_lists_into(self, pos, type_, box, bufs: "ListBuffers", check: bool = True) -> int:
        """reaxff_build_lists_into the caller-owned buffers; returns the code (0, or
        REAXFF_ERR_CAPACITY with bufs.required set) unless check raises on errors."""
        b, bp = self._boxarg(box)
        rc = self._lib.reaxff_build_lists_into(self._h, pos.shape[0], _ptr(pos), _ptr(type_), bp,
                                               ctypes.byref(bufs.c), _stream())
        if check and rc not in (0, -2):
            self._check(rc)
        return int(rc)

    def compute_forces_from(self, pos, type_, q, box, bufs: "ListBuffers", forces=None, energies=None):
        n = pos.shape[0]
        if forces is None:
            forces = torch.empty((n, 3), dtype=torch.float64, device=pos.device)
        if energies is None:
            energies = torch.empty(NTERMS, dtype=torch.float64, device=pos.device)
        b, bp = self._boxarg(box)
        self._check(self._lib.reaxff_compute_forces_from(self._h, n, _ptr(pos), _ptr(type_), _ptr(q), bp,
                                                         ctypes.byref(bufs.c), _ptr(forces), _ptr(energies),
                                                         _stream()))
        return forces, energies

    def set_skin(self, skin: float, every: int = 10):
        """reaxff_set_skin: Verlet-skin lists (skin in A, kept for at most `every` refreshes)."""
        self._check(self._lib.reaxff_set_skin(self._h, float(skin), int(every)))

    def refresh_lists(self, pos: torch.Tensor, type_: torch.Tensor, box=None) -> bool:
        """reaxff_refresh_lists; returns True when the lists were built from scratch."""
        assert pos.dtype == torch.float64 and pos.is_cuda and pos.is_contiguous()
        b, bp = self._boxarg(box)
        rb = ctypes.c_int32(0)
        self._check(self._lib.reaxff_refresh_lists(self._h, pos.shape[0], _ptr(pos), _ptr(type_), bp,
                                                   ctypes.byref(rb), _stream()))
        return bool(rb.value)

    def list_stats(self):
        """(full builds, refreshes that kept the lists) since creation."""
        s = (ctypes.c_int64 * 2)()
        self._check(self._lib.reaxff_list_stats(self._h, s))
        return int(s[0]), int(s[1])

    def compute_forces(self, pos, type_, q, box=None, forces=None, energies=None):
        """reaxff_compute_forces -> (forces (n,3), energies (12,)) float64 cuda tensors."""
        n = pos.shape[0]
        if forces is None:
            forces = torch.empty((n, 3), dtype=torch.float64, device=pos.device)
        if energies is None:
            energies = torch.empty(NTERMS, dtype=torch.float64, device=pos.device)
        assert q.dtype == torch.float64 and q.is_cuda and q.is_contiguous()
        b, bp = self._boxarg(box)
        self._check(self._lib.reaxff_compute_forces(self._h, n, _ptr(pos), _ptr(type_), _ptr(q), bp,
                                                    _ptr(forces), _ptr(energies), _stream()))
        return forces, energies

    def step(self, pos, vel, type_, q, box, dt: float, nsteps: int, forces=None, energies=None):
        """reaxff_step: velocity-Verlet NVE in place on pos, vel.
        Returns (forces (n,3), energies (nsteps+1, 13))."""
        n = pos.shape[0]
        if forces is None:
            forces = torch.empty((n, 3), dtype=torch.float64, device=pos.device)
        if energies is None:
            energies = torch.empty((nsteps + 1, NTERMS + 1), dtype=torch.float64, device=pos.device)
        b, bp = self._boxarg(box)
        self._check(self._lib.reaxff_step(self._h, n, _ptr(pos), _ptr(vel), _ptr(type_), _ptr(q), bp,
                                          float(dt), int(nsteps), _ptr(forces), _ptr(energies),
                                          _stream()))
        return forces, energies

    def list_sizes(self):
        s = (ctypes.c_int64 * 3)()
        self._check(self._lib.reaxff_list_sizes(self._h, s))
        return tuple(int(x) for x in s)

    def export_lists(self):
        """(far (M,2), bonds (B,2), hb (K,2)) int32 numpy arrays in caller indices."""
        nf, nb, nh = self.list_sizes()
        far = np.zeros((nf, 2), dtype=np.int32)
        bonds = np.zeros((nb, 2), dtype=np.int32)
        hb = np.zeros((nh, 2), dtype=np.int32)
        self._check(self._lib.reaxff_export_lists(self._h, far.ctypes.data, bonds.ctypes.data,
                                                  hb.ctypes.data))
        return far, bonds, hb

    def set_overlap(self, enable: bool):
        """Run the nonbonded term concurrently with the bonded terms (default) or in order."""
        self._check(self._lib.reaxff_set_overlap(self._h, 1 if enable else 0))

    def set_nb_run(self, run_max: int):
        """Longest run of cells the half nonbonded evaluation takes per workgroup (1..16)."""
        self._check(self._lib.reaxff_set_nb_run(self._h, int(run_max)))

    #: reaxff_set_qeq_product modes
    QEQ_PRODUCTS = {"auto": 0, "stored": 1}

    def set_qeq_product(self, mode: str):
        """How qeq multiplies by H: "auto" (matrix-free over the half far list when
        the last build left it, the default) or "stored" (rows built once per call)."""
        self._check(self._lib.reaxff_set_qeq_product(self._h, self.QEQ_PRODUCTS[mode]))

    def qeq(self, n: int, qparams, tol: float = 1e-6, maxit: int = 500, guess: bool = True,
            q=None, want_st: bool = False, device=None, check: bool = True):
        """reaxff_qeq over the atoms of the last build_lists: returns
        (q (n,) float64 cuda, iterations, (relative residual s, t)[, s, t])."""
        dev = device if device is not None else torch.device("cuda", self.device)
        if q is None:
            q = torch.empty(n, dtype=torch.float64, device=dev)
        s = t = None
        if want_st:
            s = torch.empty(n, dtype=torch.float64, device=dev)
            t = torch.empty(n, dtype=torch.float64, device=dev)
        qp = QeqParams()
        for k in range(4):
            qp.chi[k] = float(qparams["chi"][k])
            qp.J[k] = float(qparams["J"][k])
        it = ctypes.c_int32(0)
        res = (ctypes.c_double * 2)()
        rc = self._lib.reaxff_qeq(self._h, int(n), ctypes.byref(qp), float(tol), int(maxit), 1 if guess else 0,
                                  _ptr(q), _ptr(s), _ptr(t), ctypes.byref(it), res, _stream())
        if check:
            self._check(rc)
        out = (q, int(it.value), (float(res[0]), float(res[1])))
        if want_st:
            out = out + (s, t)
        return out if check else out + (rc,)

    def species(self, n: int, bo_threshold: float = 0.3, device=None):
        """reaxff_species over the bond orders of the last compute_forces: returns
        (molecule number per atom (n,) int32, element counts per molecule (M,4) int32,
        species table (S,5) int32: C, H, N, O counts and number of molecules) cuda tensors."""
        dev = device if device is not None else torch.device("cuda", self.device)
        mol = torch.empty(n, dtype=torch.int32, device=dev)
        counts = torch.empty((max(n, 1), 4), dtype=torch.int32, device=dev)
        table = torch.empty((max(n, 1), 5), dtype=torch.int32, device=dev)
        nm = ctypes.c_int64(0)
        ns = ctypes.c_int64(0)
        self._check(self._lib.reaxff_species(self._h, float(bo_threshold), _ptr(mol), _ptr(counts), _ptr(table),
                                             ctypes.byref(nm), ctypes.byref(ns), _stream()))
        return mol, counts[:nm.value], table[:ns.value]

    def dependency_radius(self) -> float:
        """reaxff_dependency_radius: the distance within which every input of every
        term that moves an atom lies."""
        return float(self._lib.reaxff_dependency_radius(self._h))

    def forces_masked(self, pos, type_, q, box, mask, forces):
        """reaxff_forces_masked: exact forces written into `forces` at the rows where
        mask (n,) uint8 cuda is nonzero; returns the subsystem's atom count."""
        assert mask.dtype == torch.uint8 and mask.is_cuda and mask.is_contiguous()
        ns = ctypes.c_int64(0)
        b, bp = self._boxarg(box)
        self._check(self._lib.reaxff_forces_masked(self._h, pos.shape[0], _ptr(pos), _ptr(type_), _ptr(q), bp,
                                                   _ptr(mask), _ptr(forces), ctypes.byref(ns), _stream()))
        return int(ns.value)

    def compute_forces_batched(self, sys_off, max_atoms: int, pos, type_, q, forces=None, energies=None,
                               status=None):
        """reaxff_compute_forces_batched (no allocation inside the library): sys_off (nsys+1,)
        int64 cuda offsets, max_atoms an upper bound on any cluster's atoms.  Returns
        (forces (N,3), energies (nsys,12), status (3,) int32) cuda tensors."""
        assert sys_off.dtype == torch.int64 and sys_off.is_cuda and sys_off.is_contiguous()
        nsys = sys_off.shape[0] - 1
        n = pos.shape[0]
        if forces is None:
            forces = torch.empty((n, 3), dtype=torch.float64, device=pos.device)
        if energies is None:
            energies = torch.empty((nsys, NTERMS), dtype=torch.float64, device=pos.device)
        if status is None:
            status = torch.empty(3, dtype=torch.int32, device=pos.device)
        for t, dt in ((pos, torch.float64), (type_, torch.int32), (q, torch.float64), (forces, torch.float64),
                      (energies, torch.float64), (status, torch.int32)):
            assert t.dtype == dt and t.is_cuda and t.is_contiguous()
        assert energies.shape == (nsys, NTERMS) and forces.shape == (n, 3) and status.numel() >= 3
        self._check(self._lib.reaxff_compute_forces_batched(
            self._h, nsys, _ptr(sys_off), int(max_atoms), _ptr(pos), _ptr(type_), _ptr(q), _ptr(forces),
            _ptr(energies), _ptr(status), _stream()))
        return forces, energies, status

    def interaction_counts(self):
        c = (ctypes.c_int64 * 5)()
        self._check(self._lib.reaxff_interaction_counts(self._h, c))
        return dict(zip(("angles", "torsions", "hbonds", "far_pairs", "bonds"), (int(x) for x in c)))


class Batch:
    """A batch plan over many small non-periodic clusters (reaxff_batch_*).

    offsets: int64 (nclusters+1,) host array; cluster c holds atoms
    offsets[c]:offsets[c+1] of the concatenated position/type/charge arrays.
    """

    def __init__(self, ff: ReaxFF, offsets, config=None):
        self._ff = ff
        self._lib = ff._lib
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        self.offsets = off
        self.nclusters = off.size - 1
        self.natoms = int(off[-1])
        h = ctypes.c_void_p()
        cfg = None
        if config is not None:
            cfg = BatchConfig(*config)
        rc = self._lib.reaxff_batch_create(ff._h, self.nclusters, off.ctypes.data,
                                           ctypes.byref(cfg) if cfg is not None else None,
                                           ctypes.byref(h))
        ff._check(rc)
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self._lib.reaxff_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def config(self):
        c = BatchConfig()
        self._ff._check(self._lib.reaxff_batch_get_config(self._h, ctypes.byref(c)))
        return c.as_tuple()

    @config.setter
    def config(self, value):
        c = BatchConfig(*value)
        self._ff._check(self._lib.reaxff_batch_set_config(self._h, ctypes.byref(c)))

    def _bufs(self, pos, forces, energies):
        n = self.natoms
        if forces is None:
            forces = torch.empty((n, 3), dtype=torch.float64, device=pos.device)
        if energies is None:
            energies = torch.empty((self.nclusters, NTERMS), dtype=torch.float64, device=pos.device)
        return forces, energies

    def _check_inputs(self, pos, type_, q, forces, energies):
        n = self.natoms
        assert pos.dtype == torch.float64 and pos.is_cuda and pos.is_contiguous() and pos.shape == (n, 3)
        assert type_.dtype == torch.int32 and type_.is_cuda and type_.is_contiguous() and type_.shape == (n,)
        assert q.dtype == torch.float64 and q.is_cuda and q.is_contiguous() and q.shape == (n,)
        assert forces.dtype == torch.float64 and forces.is_contiguous() and forces.shape == (n, 3)
        assert energies.dtype == torch.float64 and energies.is_contiguous()
        assert energies.shape == (self.nclusters, NTERMS)

    def compute(self, pos, type_, q, forces=None, energies=None):
        """reaxff_batch_compute -> (forces (N,3), energies (nclusters,12)) float64 cuda."""
        forces, energies = self._bufs(pos, forces, energies)
        self._check_inputs(pos, type_, q, forces, energies)
        self._ff._check(self._lib.reaxff_batch_compute(self._h, _ptr(pos), _ptr(type_), _ptr(q),
                                                       _ptr(forces), _ptr(energies), _stream()))
        return forces, energies

    def status(self):
        """(return code, first failing cluster or -1); waits for the last compute."""
        fb = ctypes.c_int32(-1)
        rc = self._lib.reaxff_batch_status(self._h, ctypes.byref(fb))
        return int(rc), int(fb.value)

    def check(self):
        rc, fb = self.status()
        if rc != 0:
            raise ReaxFFError(rc, self._lib.reaxff_last_error(self._ff._h).decode())

    def counts(self):
        """(nclusters, 5) int64: angles, torsions, hbonds, far pairs, bonds per cluster."""
        c = np.zeros((self.nclusters, 5), dtype=np.int64)
        self._ff._check(self._lib.reaxff_batch_counts(self._h, c.ctypes.data))
        return c

    def tune(self, pos, type_, q, forces=None, energies=None, reps: int = 3, max_trials: int = 0):
        """reaxff_batch_tune: returns [(config, ms per launch)] of every trial; the fastest
        becomes the plan's configuration."""
        forces, energies = self._bufs(pos, forces, energies)
        self._check_inputs(pos, type_, q, forces, energies)
        cap = 64
        trials = (BatchConfig * cap)()
        ms = (ctypes.c_double * cap)()
        nt = ctypes.c_int32(0)
        self._ff._check(self._lib.reaxff_batch_tune(self._h, _ptr(pos), _ptr(type_), _ptr(q),
                                                    _ptr(forces), _ptr(energies), _stream(),
                                                    int(reps), int(max_trials), trials, ms,
                                                    ctypes.byref(nt)))
        return [(trials[k].as_tuple(), float(ms[k])) for k in range(nt.value)]


NDESC = 224


class Surrogate:
    """An ensemble of per-element networks on the GPU (reaxff_surrogate_*).

    Parameters are float32 arrays shaped (members, 4, param_count); shift and
    scale (224,) float32.  Energies kcal/mol, forces kcal/(mol A).
    """

    def __init__(self, ff: ReaxFF, members: int = 4):
        self._ff = ff
        self._lib = ff._lib
        self.members = int(members)
        self.npar = int(self._lib.reaxff_surrogate_param_count())
        h = ctypes.c_void_p()
        ff._check(self._lib.reaxff_surrogate_create(ff._h, self.members, ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self._lib.reaxff_surrogate_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != 0:
            raise ReaxFFError(rc, self._lib.reaxff_surrogate_last_error(self._h).decode())

    def set_params(self, theta=None, shift=None, scale=None):
        def arr(x, shape):
            if x is None:
                return None
            a = np.ascontiguousarray(x, dtype=np.float32)
            assert a.size == int(np.prod(shape)), (a.shape, shape)
            return a
        t = arr(theta, (self.members, 4, self.npar))
        sh = arr(shift, (NDESC,))
        sc = arr(scale, (NDESC,))
        self._check(self._lib.reaxff_surrogate_set_params(
            self._h, t.ctypes.data if t is not None else None, sh.ctypes.data if sh is not None else None,
            sc.ctypes.data if sc is not None else None))

    def get_params(self):
        t = np.zeros((self.members, 4, self.npar), dtype=np.float32)
        sh = np.zeros(NDESC, dtype=np.float32)
        sc = np.zeros(NDESC, dtype=np.float32)
        self._check(self._lib.reaxff_surrogate_get_params(self._h, t.ctypes.data, sh.ctypes.data, sc.ctypes.data))
        return t, sh, sc

    def normaliser(self, G, std_floor: float = 1e-3):
        """reaxff_surrogate_normaliser over descriptor rows G (rows, 224) float32 cuda:
        (shift, scale) float32 numpy arrays."""
        assert G.dtype == torch.float32 and G.is_cuda and G.is_contiguous() and G.shape[1] == NDESC
        shift = np.zeros(NDESC, dtype=np.float32)
        scale = np.zeros(NDESC, dtype=np.float32)
        self._check(self._lib.reaxff_surrogate_normaliser(self._h, G.shape[0], _ptr(G), float(std_floor),
                                                          shift.ctypes.data, scale.ctypes.data, _stream()))
        return shift, scale

    def get_grad(self):
        g = np.zeros((self.members, 4, self.npar), dtype=np.float32)
        self._check(self._lib.reaxff_surrogate_get_grad(self._h, g.ctypes.data))
        return g

    @staticmethod
    def _boxarg(box):
        return ReaxFF._boxarg(box)

    def descriptors(self, pos, type_, box=None):
        n = pos.shape[0]
        G = torch.empty((n, NDESC), dtype=torch.float32, device=pos.device)
        b, bp = self._boxarg(box)
        self._check(self._lib.reaxff_surrogate_descriptors(self._h, n, _ptr(pos), _ptr(type_), bp, _ptr(G),
                                                           _stream()))
        return G

    def evaluate(self, pos, type_, box=None):
        """dict: energies (M,) float64, eatom (M,n), forces (M,n,3) float32, fmean (n,3) float64,
        sigma (n,) float32 -- cuda tensors, caller order."""
        n = pos.shape[0]
        M = self.members
        d = pos.device
        out = dict(energies=torch.empty(M, dtype=torch.float64, device=d),
                   eatom=torch.empty((M, n), dtype=torch.float32, device=d),
                   forces=torch.empty((M, n, 3), dtype=torch.float32, device=d),
                   fmean=torch.empty((n, 3), dtype=torch.float64, device=d),
                   sigma=torch.empty(n, dtype=torch.float32, device=d))
        b, bp = self._boxarg(box)
        self._check(self._lib.reaxff_surrogate_evaluate(
            self._h, n, _ptr(pos), _ptr(type_), bp, _ptr(out["energies"]), _ptr(out["eatom"]),
            _ptr(out["forces"]), _ptr(out["fmean"]), _ptr(out["sigma"]), _stream()))
        return out

    def train_step(self, pos, type_, box, eref: float, fref, wE: float = 1.0, wF: float = 1.0,
                   lr: float = 1e-3):
        """Loss of every member before the step (float64 cuda tensor (M,))."""
        loss = torch.empty(self.members, dtype=torch.float64, device=pos.device)
        assert fref.dtype == torch.float64 and fref.is_contiguous() and fref.shape == pos.shape
        b, bp = self._boxarg(box)
        self._check(self._lib.reaxff_surrogate_train_step(
            self._h, pos.shape[0], _ptr(pos), _ptr(type_), bp, float(eref), _ptr(fref), float(wE), float(wF),
            float(lr), _ptr(loss), _stream()))
        return loss

    def gated_forces(self, plain: ReaxFF, pos, type_, q, box, threshold: float):
        """(forces (n,3) float64, mask (n,) uint8, energies (M,), nflagged int)."""
        n = pos.shape[0]
        d = pos.device
        forces = torch.empty((n, 3), dtype=torch.float64, device=d)
        mask = torch.empty(n, dtype=torch.uint8, device=d)
        energies = torch.empty(self.members, dtype=torch.float64, device=d)
        nf = ctypes.c_int64(0)
        ns = ctypes.c_int64(0)
        b, bp = self._boxarg(box)
        self._check(self._lib.reaxff_surrogate_gated_forces(
            self._h, plain._h, n, _ptr(pos), _ptr(type_), _ptr(q), bp, float(threshold), _ptr(forces),
            _ptr(mask), _ptr(energies), ctypes.byref(nf), ctypes.byref(ns), _stream()))
        self.last_nsub = int(ns.value)
        return forces, mask, energies, int(nf.value)
