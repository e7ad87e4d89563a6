"""The FP64 exp and log polynomials of terms.h are the ones their stated
derivation gives (paper_1706_07772_amd/csrc/poly_coeffs.py: Taylor series
economized by Chebyshev polynomials, exact rationals rounded to double)."""
import importlib.util
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_1706_07772_amd", "csrc")


def _gen():
    spec = importlib.util.spec_from_file_location("poly_coeffs", os.path.join(CSRC, "poly_coeffs.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def _literals(body):
    return re.findall(r"0x1\.[0-9a-f]+p-?\d+", body)


def _function(src, name):
    i = src.index(f"__device__ __forceinline__ double {name}(double x) {{")
    return src[i:src.index("\n}\n", i)]


def test_exp_and_log_coefficients_match_their_derivation():
    g = _gen()
    src = open(os.path.join(CSRC, "terms.h")).read()
    exp_c = g.hex_literals(g.exp_coefficients())
    log_c = g.hex_literals(g.log_coefficients())
    assert [float.fromhex(h) for h in exp_c[-2:]] == [1.0, 1.0]
    for name in ("exp_f", "exp_r"):
        lits = [h for h in _literals(_function(src, name)) if h not in ("0x1.8p52",)]
        # the reduction constants (ln 2 split) are named elsewhere; the body
        # holds the ten polynomial coefficients of degree 11 .. 2
        assert lits == exp_c[:10], (name, lits)
    for name in ("log_f", "log_r"):
        lits = [h for h in _literals(_function(src, name)) if h != "0x1.00000800p52"]
        assert lits == log_c, (name, lits)
