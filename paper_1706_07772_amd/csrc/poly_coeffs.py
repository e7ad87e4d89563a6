"""Derivation of the polynomial coefficients of the FP64 exp and log in terms.h.

exp(r) on |r| <= 0.3466 (ln 2 / 2, the Cody-Waite remainder): the Taylor
series to degree 13, economized to degree 11 by Chebyshev polynomials
(Lanczos): the r^13 term, then the r^12 term, is replaced through
T_13(r/a), T_12(r/a) with a = 0.3466, dropping the T_n part, whose size on
the interval is the error added (at most 3.1e-18 on top of the series'
4.1e-18 truncation).

log(m) = 2 atanh(s) = 2 s + 2 s z p(z), s = (m - 1)/(m + 1), z = s^2 <=
0.02944 for m in [1/sqrt 2, sqrt 2): p(z) = sum_k z^k / (2k + 3) to k = 8,
economized to degree 6 by shifted Chebyshev polynomials T_n(2z/b - 1) on
[0, b], b = 0.02944.

All arithmetic is exact (rationals); each coefficient is then rounded to the
nearest double.  Run as a script to print the C literals in the order of the
Horner evaluation (highest degree first).
"""
from fractions import Fraction as F
import math

EXP_A = F(3466, 10000)
LOG_B = F(2944, 100000)


def chebyshev(n):
    """Coefficients of T_n in powers of its argument (exact)."""
    t = [[F(1)], [F(0), F(1)]]
    for k in range(2, n + 1):
        a = [F(0)] + [2 * c for c in t[k - 1]]
        b = t[k - 2] + [F(0)] * (len(a) - len(t[k - 2]))
        t.append([x - y for x, y in zip(a, b)])
    return t[n]


def _mul(p, q):
    r = [F(0)] * (len(p) + len(q) - 1)
    for i, x in enumerate(p):
        for j, y in enumerate(q):
            r[i + j] += x * y
    return r


def economize(coef, to_degree, basis):
    """Lower a power-series polynomial to `to_degree`: for n from the top, the
    x^n term is replaced by x^n - basis(n)/lead(basis(n)), basis(n) being a
    degree-n polynomial small on the interval (a scaled Chebyshev one)."""
    c = list(coef)
    for n in range(len(c) - 1, to_degree, -1):
        b = basis(n)
        lead = c[n] / b[n]
        for k in range(n + 1):
            c[k] -= lead * b[k]
        c = c[:n]
    return c


def exp_coefficients():
    """exp on |r| <= EXP_A: degree 11, c[0] = c[1] = 1."""
    taylor = [F(1, math.factorial(k)) for k in range(14)]

    def basis(n):   # T_n(r / a)
        return [t / EXP_A ** k for k, t in enumerate(chebyshev(n))]
    return economize(taylor, 11, basis)


def log_coefficients():
    """p(z) on [0, LOG_B]: degree 6."""
    series = [F(1, 2 * k + 3) for k in range(9)]

    def basis(n):   # T_n(2 z / b - 1)
        t, lin, res, pw = chebyshev(n), [F(-1), F(2) / LOG_B], [F(0)] * (n + 1), [F(1)]
        for k in range(n + 1):
            for i, c in enumerate(pw):
                res[i] += t[k] * c
            pw = _mul(pw, lin)
        return res
    return economize(series, 6, basis)


def hex_literals(coef):
    """C hex literals, highest degree first."""
    return [float(c).hex() for c in reversed(coef)]


if __name__ == "__main__":
    print("exp (degree 11 .. 0):", ", ".join(hex_literals(exp_coefficients())))
    print("log p(z) (degree 6 .. 0):", ", ".join(hex_literals(log_coefficients())))
