"""Shared helpers of the parity tests (GPU path vs the CPU oracle)."""
import numpy as np

import reaxff_synth as rs

# tolerance of FP64 parity: energies and forces to 1e-9 relative.  Energies:
# |E_gpu - E_ref| <= 1e-9 * sum over interactions |e| of that term (the sum's
# condition number); forces: max_i |F_gpu,i - F_ref,i| <= 1e-9 * max_i |F_ref,i|.
REL_TOL = 1e-9
# a bond whose raw uncorrected order lies this close (relative) to bo_cut may be
# decided differently by the two sides' pow/exp (last-ulp differences)
BORDER_REL = 1e-12


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def to_dev(system):
    import torch
    dev = torch.device("cuda:0")
    pos = torch.tensor(system.pos, dtype=torch.float64, device=dev).contiguous()
    typ = torch.tensor(system.type, dtype=torch.int32, device=dev).contiguous()
    q = torch.tensor(system.q, dtype=torch.float64, device=dev).contiguous()
    box = None if system.box is None else [float(x) for x in system.box]
    return pos, typ, q, box


def gpu_eval(ff, system, lists=False):
    """Build lists and evaluate forces on the GPU; returns numpy (E, F[, lists])."""
    import torch
    pos, typ, q, box = to_dev(system)
    ff.build_lists(pos, typ, box)
    f, e = ff.compute_forces(pos, typ, q, box)
    torch.cuda.synchronize()
    out = (e.cpu().numpy().copy(), f.cpu().numpy().copy())
    if lists:
        out = out + (ff.export_lists(),)
    return out


def pairs_set(a, symmetric=False):
    if symmetric:
        a = np.sort(a, axis=1)
    return set(map(tuple, a.tolist()))


def assert_lists_equal(gpu_lists, oracle, ora_lists):
    """Far and H lists exactly equal as sets; the bond list equal up to pairs within the
    borderline band of bo_cut (reported and counted)."""
    gf, gb, gh = gpu_lists
    of, ob, oh = ora_lists
    assert len(gf) == len(of), (len(gf), len(of))
    assert pairs_set(gf, symmetric=True) == pairs_set(of)
    assert pairs_set(gh) == pairs_set(oh)
    sb, so = pairs_set(gb), pairs_set(ob)
    diff = sb ^ so
    bo_cut = oracle.cutoffs["bo_cut"]
    for (i, j) in diff:
        raw = oracle.bo_raw(i, j)
        assert abs(raw / bo_cut - 1.0) <= BORDER_REL, ("bond list mismatch", i, j, raw)
    return len(diff)


def assert_energy_parity(e_gpu, e_ref, e_abs, tol=REL_TOL, names=None):
    bad = []
    for t in range(len(e_ref)):
        scale = max(e_abs[t], 1e-300)
        if abs(e_gpu[t] - e_ref[t]) > tol * scale:
            bad.append((t if names is None else names[t], e_gpu[t], e_ref[t], e_abs[t]))
    assert not bad, bad


def assert_force_parity(f_gpu, f_ref, tol=REL_TOL):
    ref = np.linalg.norm(f_ref, axis=1).max()
    err = np.linalg.norm(f_gpu - f_ref, axis=1)
    k = int(err.argmax())
    assert err.max() <= tol * ref, (err.max() / ref, k, f_gpu[k], f_ref[k])


def extract_subsystem(system, center, radius):
    """Atoms within radius of `center` (minimum image), unwrapped around it, as a
    non-periodic system; returns (subsystem, index of the centre atom in it, caller ids)."""
    x = system.pos
    d = x - x[center]
    if system.box is not None:
        L = system.box
        d = d - L * np.rint(d / L)
    r = np.sqrt((d * d).sum(1))
    ids = np.nonzero(r <= radius)[0]
    sub = rs.System(pos=x[center] + d[ids], type=system.type[ids], q=system.q[ids], box=None)
    return sub, int(np.searchsorted(ids, center)), ids


def near_straight_chain(eps):
    """C-C-C-N-O chain: atoms 0-1-2 deviate from a straight line by the angle eps
    (sin of angle 0-1-2 is about eps), 1-2-3-4 is an ordinary bent chain, so the
    straight angle enters a valence angle and two torsions."""
    r = 1.35
    pos = np.array([[0.0, 0.0, 0.0],
                    [r, 0.0, 0.0],
                    [r + r * np.cos(eps), r * np.sin(eps), 0.0],
                    [2 * r + 0.9, 1.1, 0.2],
                    [2 * r + 1.5, 2.3, -0.6]])
    return rs.System(pos=pos, type=np.array([0, 0, 0, 2, 3], dtype=np.int32), q=np.zeros(5), box=None)
