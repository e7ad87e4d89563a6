"""The C ABI boundary without a GPU: the HIP library loads, exports every
function include/reaxff.h declares (and nothing else under the reaxff_
prefix), and its parameter struct has the layout the binding marshals.
No compute call is made here."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "reaxff.h")
LIB = os.path.join(ROOT, "paper_1706_07772_amd", "libreaxff_hip.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(reaxff_\w+)\s*\(", src)))


def exported():
    import subprocess
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], check=True, capture_output=True,
                         text=True).stdout
    return sorted({ln.split()[-1] for ln in out.splitlines() if re.search(r" T reaxff_\w+$", ln)})


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "build the library first (__graft_entry__.build())"
    lib = ctypes.CDLL(LIB)
    names = declared()
    assert len(names) >= 30
    for name in names:
        assert hasattr(lib, name), name
    assert exported() == names


def test_params_layout_matches_binding():
    from paper_1706_07772_amd.binding import CParams, load_library
    lib = load_library()
    assert lib.reaxff_params_size() == ctypes.sizeof(CParams)


def test_create_rejects_asymmetric_tables():
    """reaxff_create refuses parameter tables without the stated symmetries
    (pair [i][j] = [j][i], angle [i][j][k] = [k][j][i], torsion reversal),
    before it touches a device: a bond found from one atom must be found from
    the other, and each interaction has one parameter set."""
    import numpy as np
    import reaxff_synth as rs
    from paper_1706_07772_amd.binding import load_library, make_cparams
    lib = load_library()
    base = rs.draw_params(0)
    for table, name, idx in (("pair", "r_s", (0, 2)), ("angle", "theta00", (0, 1, 3)),
                             ("tors", "V2", (0, 1, 2, 3))):
        p = rs.draw_params(0)
        arr = getattr(p, table)[name].copy()
        arr[idx] += 0.125
        getattr(p, table)[name] = arr
        out = ctypes.c_void_p()
        code = lib.reaxff_create(ctypes.byref(make_cparams(p)), None, 0, ctypes.byref(out))
        assert code == -1 and not out.value, (table, name, code)
    assert np.array_equal(base.pair["r_s"], base.pair["r_s"].T)
