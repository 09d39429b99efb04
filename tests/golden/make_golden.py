"""Write the closed-form golden fixtures of this folder.

Every value here is one of the paper's printed closed forms evaluated in
exact rational arithmetic (Python ``fractions``) — no oracle, no GPU:

* ``winv_uniform.txt`` — eq:W1inv, the inverse of the eq:modW matrix for
  the uniform weights of eq:W (fidelity 1, commensurability w):
  diagonal (n+w)/(n(n+mw)), off-diagonal w/(n(n+mw)).
* ``zprime_uniform.txt`` — the J_n-coefficient matrix printed after
  eq:W1inv (Section 2.1): diagonal (-m^2 w^2 + m n^2 - m n w - n^2) /
  (w n^2 m^2 (n + w m)), off-diagonal (-m^2 w^2 - m n w - n^2) / (same).
* ``l22inv_uniform.txt`` — Section 3: L22^dagger = I/(n+mw) + w J/(n(n+mw)).
* ``winv_w3.txt`` — Section 2.1.1, eq:W3 weights: diag(w_ii)^-1/(n + sum w_ii)
  + J/(n(n + sum w_ii)).

Run ``python tests/golden/make_golden.py`` to regenerate.
"""
import os
from fractions import Fraction as F

HERE = os.path.dirname(os.path.abspath(__file__))

UNIFORM_CASES = [(2, 200, F(1, 2)), (3, 20000, F(1, 2)), (2, 10000, F(1, 2)),
                 (4, 6, F(10)), (3, 5, F(2))]
W3_CASES = [(7, [F(1), F(2), F(1, 2)]), (10, [F(3, 2), F(1), F(1, 4), F(2)])]


def winv_uniform(m, n, w):
    den = n * (n + m * w)
    return [[(n + w) / den if i == j else w / den for j in range(m)] for i in range(m)]


def zprime_uniform(m, n, w):
    den = w * n * n * m * m * (n + w * m)
    dg = (-m * m * w * w + m * n * n - m * n * w - n * n) / den
    of = (-m * m * w * w - m * n * w - n * n) / den
    return [[dg if i == j else of for j in range(m)] for i in range(m)]


def l22inv_uniform(m, n, w):
    return [[F(1) / (n + m * w) * (1 if i == j else 0) + w / (n * (n + m * w))
             for j in range(m)] for i in range(m)]


def winv_w3(n, ws):
    s = sum(ws)
    m = len(ws)
    return [[(1 / (ws[k] * (n + s)) if k == l else 0) + F(1) / (n * (n + s))
             for l in range(m)] for k in range(m)]


def _fmt(M):
    return ";".join(",".join(f"{x.numerator}/{x.denominator}" for x in row) for row in M)


def main():
    with open(os.path.join(HERE, "winv_uniform.txt"), "w") as f:
        f.write("# eq:W1inv (Section 2.1): inverse of the eq:modW matrix, uniform weights\n")
        f.write("# m n w | rows ';'-separated, entries exact fractions\n")
        for m, n, w in UNIFORM_CASES:
            f.write(f"{m} {n} {w} | {_fmt(winv_uniform(m, n, w))}\n")
    with open(os.path.join(HERE, "zprime_uniform.txt"), "w") as f:
        f.write("# Section 2.1, matrix printed after eq:W1inv: J_n coefficient of L^dagger, uniform weights\n")
        f.write("# m n w | rows\n")
        for m, n, w in UNIFORM_CASES:
            if n <= 200:
                f.write(f"{m} {n} {w} | {_fmt(zprime_uniform(m, n, w))}\n")
    with open(os.path.join(HERE, "l22inv_uniform.txt"), "w") as f:
        f.write("# Section 3: L22^dagger = I_m/(n+mw) + w J_m/(n(n+mw)), uniform weights\n")
        f.write("# m n w | rows\n")
        for m, n, w in UNIFORM_CASES:
            f.write(f"{m} {n} {w} | {_fmt(l22inv_uniform(m, n, w))}\n")
    with open(os.path.join(HERE, "winv_w3.txt"), "w") as f:
        f.write("# Section 2.1.1, eq:W3 weights: W^-1 = diag(w_ii)^-1/(n+sum w_ii) + J_m/(n(n+sum w_ii))\n")
        f.write("# n w_11,..,w_mm | rows\n")
        for n, ws in W3_CASES:
            f.write(f"{n} {','.join(str(x) for x in ws)} | {_fmt(winv_w3(n, ws))}\n")


if __name__ == "__main__":
    main()
