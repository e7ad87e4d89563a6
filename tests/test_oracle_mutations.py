"""The oracle's pins must fail on plausible mistakes.

Each case copies the oracle source to a scratch directory, plants one
textual mistake (a swapped valence, a dropped term, a wrong index or sign),
builds it, and runs the CPU pin tests against the mutated build in a child
process.  The case passes when the child's pins FAIL.  Mistakes are planted
only in the CPU oracle; nothing here touches a GPU.
"""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PINS = ["tests/test_oracle_pins.py", "tests/test_oracle_pins_terms.py"]

# (name, text in reaxff_oracle.cpp, replacement)
MUTATIONS = [
    ("boc valence is Val", "B.Dboc[i] = sum - P.a[a_val_boc]", "B.Dboc[i] = sum - P.a[a_val]"),
    ("f1 uses Val_boc", "const double vi = P.a[a_val][ti], vj = P.a[a_val][tj];",
     "const double vi = P.a[a_val_boc][ti], vj = P.a[a_val][tj];"),
    ("f3 drops the j side", "log(0.5 * (exp(-pb2 * B.Dp[i]) + exp(-pb2 * B.Dp[j])))",
     "log(0.5 * (exp(-pb2 * B.Dp[i]) + exp(-pb2 * B.Dp[i])))"),
    ("sigma-pi takes the centre's Delta", "sumpi = sumpi + (B.Delta[j] - B.Dlp[j])",
     "sumpi = sumpi + (B.Delta[i] - B.Dlp[j])"),
    ("sigma-pi sign of Delta_lp", "sumpi = sumpi + (B.Delta[j] - B.Dlp[j])",
     "sumpi = sumpi + (B.Delta[j] + B.Dlp[j])"),
    ("Delta_lpc sign of p_ovun4", "(1.0 + po3 * exp(po4 * sumpi))", "(1.0 + po3 * exp(-po4 * sumpi))"),
    ("under factor sign of p_ovun8", "(1.0 + po7 * exp(po8 * sumpi))", "(1.0 + po7 * exp(-po8 * sumpi))"),
    ("lone-pair switch sign", "exp(-75.0 * B.Dlp[i])", "exp(75.0 * B.Dlp[i])"),
    ("vlpex rule inverted", "re(B.vlpex[i]) < 0.0", "re(B.vlpex[i]) >= 0.0"),
    ("BO^8 becomes BO^4", "const T b4 = b2 * b2;", "const T b4 = b2;"),
    ("SBO2 upper branch", "B.SBO2[i] = 2.0 - pow(2.0 - B.SBO[i], pv9);", "B.SBO2[i] = pow(B.SBO[i], pv9);"),
    ("f8 takes Delta", "const T e6 = exp(pv6 * B.Dang[j])", "const T e6 = exp(pv6 * B.Delta[j])"),
    ("f9 takes Delta_ang", "ep4 = exp(pp4 * B.Delta[j]);", "ep4 = exp(pp4 * B.Dang[j]);"),
    ("coalition takes the centre's S", "exp(-pc3 * sq(B.S[i] - BOA_ij))", "exp(-pc3 * sq(B.S[j] - BOA_ij))"),
    ("coalition repeats a bond", "exp(-pc4 * sq(BOA_jk - 1.5))", "exp(-pc4 * sq(BOA_ij - 1.5))"),
    ("f10 repeats the central bond", "(1.0 - exp(-pt2 * BOA_kl))", "(1.0 - exp(-pt2 * BOA_jk))"),
    ("f11 swaps p_tor3 and p_tor4", "const T et3 = exp(-pt3 * D), et4 = exp(pt4 * D);",
     "const T et3 = exp(-pt4 * D), et4 = exp(pt3 * D);"),
    ("V2 factor takes the total order", "sq(2.0 - B.BOp[b] - f11)", "sq(2.0 - B.BO[b] - f11)"),
    ("conjugation repeats the central bond", "exp(-pcot2 * sq(BOA_kl - 1.5))",
     "exp(-pcot2 * sq(BOA_jk - 1.5))"),
    ("Coulomb shielding power", "std::pow(P.p[gamma_c][ti][tj], -3.0)", "std::pow(P.p[gamma_c][ti][tj], -2.0)"),
    ("H-bond half angle", "const T s4 = sq((1.0 - cth) / 2.0);", "const T s4 = sq((1.0 + cth) / 2.0);"),
]


def _run(case, tmp_root):
    name, old, new = case
    d = os.path.join(tmp_root, "m%02d" % MUTATIONS.index(case))
    os.makedirs(d)
    for sub in ("oracle", "reaxff_synth", "tests"):
        shutil.copytree(os.path.join(ROOT, sub), os.path.join(d, sub),
                        ignore=shutil.ignore_patterns("*.so", "__pycache__", "liboracle*"))
    src = os.path.join(d, "oracle", "reaxff_oracle.cpp")
    text = open(src).read()
    assert text.count(old) >= 1, name
    open(src, "w").write(text.replace(old, new, 1))
    lib = os.path.join(d, "oracle", "liboracle.so")
    subprocess.run(["g++", "-std=c++17", "-O1", "-fno-fast-math", "-ffp-contract=off", "-fPIC",
                    "-shared", "-o", lib, src], check=True)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider"] + PINS,
                       cwd=d, capture_output=True, text=True, timeout=600)
    return name, r.returncode


def test_every_planted_mistake_fails_a_pin(tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        results = list(ex.map(lambda c: _run(c, str(tmp_path)), MUTATIONS))
    survived = [name for name, rc in results if rc == 0]
    assert not survived, f"pins did not catch: {survived}"
