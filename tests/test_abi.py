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
