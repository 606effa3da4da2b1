#!/usr/bin/env python3
"""Generate d2q37_tables.h, the compile-time constants of the GPU library.

D2Q37 (arXiv:1703.04594, section 3): 37 populations whose hops reach up to
three lattice points.  The hop set is the 37 integer vectors with |e|^2 in
{0,1,2,4,5,8,9,10}; canonical order is by |e|^2, then by angle in [0, 2 pi).

Weights and the lattice scale c (xi = c e) make the discrete moments equal
to those of the unit-temperature Gaussian up to 8th order:

    sum_l w_l (c e_x)^(2i) (c e_y)^(2j) = (2i-1)!! (2j-1)!!,  2i+2j <= 8, i >= j.

That is 9 equations for 8 shell weights and c.  With t = 1/c^2 they read
S w = b(t), b_k = m_k t^(i_k + j_k), S an integer 9x8 matrix, so a solution
exists exactly when det[S | b(t)] = 0 -- a polynomial in t with integer
coefficients (cofactor expansion along the last column, computed exactly in
rationals).  Its real root that gives positive weights is refined in 80-digit
decimal arithmetic, the weights follow from 8 of the equations, and every
value is rounded once to binary64 / binary32.

Usage:  python gen_d2q37_tables.py [output.h]
"""
from __future__ import annotations

import math
import os
import sys
from decimal import Decimal, getcontext
from fractions import Fraction

getcontext().prec = 80

SHELLS = [0, 1, 2, 4, 5, 8, 9, 10]


def hop_set():
    hops = [(ex, ey) for ex in range(-3, 4) for ey in range(-3, 4) if ex * ex + ey * ey in SHELLS]
    hops.sort(key=lambda h: (h[0] ** 2 + h[1] ** 2, math.atan2(h[1], h[0]) % (2 * math.pi)))
    assert len(hops) == 37
    return hops


def odd_double_factorial(i):
    return math.prod(range(2 * i - 1, 0, -2)) if i > 0 else 1


def det_fraction(M):
    M = [row[:] for row in M]
    n = len(M)
    det = Fraction(1)
    for c in range(n):
        p = next((r for r in range(c, n) if M[r][c] != 0), None)
        if p is None:
            return Fraction(0)
        if p != c:
            M[c], M[p] = M[p], M[c]
            det = -det
        det *= M[c][c]
        for r in range(c + 1, n):
            f = M[r][c] / M[c][c]
            for k in range(c, n):
                M[r][k] -= f * M[c][k]
    return det


def solve_decimal(A, b):
    n = len(A)
    M = [row[:] + [bb] for row, bb in zip(A, b)]
    for c in range(n):
        p = max(range(c, n), key=lambda r: abs(M[r][c]))
        M[c], M[p] = M[p], M[c]
        for r in range(c + 1, n):
            f = M[r][c] / M[c][c]
            for k in range(c, n + 1):
                M[r][k] -= f * M[c][k]
    x = [Decimal(0)] * n
    for r in range(n - 1, -1, -1):
        x[r] = (M[r][n] - sum(M[r][k] * x[k] for k in range(r + 1, n))) / M[r][r]
    return x


def derive():
    hops = hop_set()
    eqs = [(i, j) for i in range(5) for j in range(5) if 2 * i + 2 * j <= 8 and i >= j]
    assert len(eqs) == 9
    S = [[sum(Fraction(ex) ** (2 * i) * Fraction(ey) ** (2 * j)
              for ex, ey in hops if ex * ex + ey * ey == s) for s in SHELLS] for i, j in eqs]
    m = [odd_double_factorial(i) * odd_double_factorial(j) for i, j in eqs]
    deg = [i + j for i, j in eqs]
    # det [S | b(t)] = sum_k (-1)^(k+8) b_k det(S minus row k)
    poly = [Fraction(0)] * 5
    for k in range(9):
        minor = [S[r] for r in range(9) if r != k]
        poly[deg[k]] += (-1) ** (k + 8) * m[k] * det_fraction(minor)

    def p(t):
        return sum(Decimal(c.numerator) / Decimal(c.denominator) * t ** d for d, c in enumerate(poly))

    def dp(t):
        return sum(d * Decimal(c.numerator) / Decimal(c.denominator) * t ** (d - 1)
                   for d, c in enumerate(poly) if d > 0)

    # bracket real roots on t in (0, 5], refine each by Newton, keep the one with w > 0
    grid = [Decimal(k) / 1000 for k in range(1, 5001)]
    candidates = []
    for a, b in zip(grid, grid[1:]):
        if (p(a) < 0) != (p(b) < 0):
            t = (a + b) / 2
            for _ in range(200):
                step = p(t) / dp(t)
                t -= step
                if abs(step) < Decimal(10) ** -75:
                    break
            candidates.append(t)
    solutions = []
    for t in candidates:
        A = [[Decimal(S[r][s].numerator) for s in range(8)] for r in range(8)]
        bvec = [Decimal(m[r]) * t ** deg[r] for r in range(8)]
        w = solve_decimal(A, bvec)
        if all(x > 0 for x in w):
            solutions.append((t, w))
    assert len(solutions) == 1, solutions
    t, w = solutions[0]
    c2 = 1 / t
    c = c2.sqrt()
    # residual check in decimal
    for (i, j), mk, row in zip(eqs, m, S):
        lhs = sum(Decimal(row[s].numerator) * w[s] for s in range(8)) * c2 ** (i + j)
        assert abs(lhs - mk) < Decimal(10) ** -60
    return hops, c, c2, w


def f64(d: Decimal) -> str:
    return float(d).hex()


def f32(d: Decimal) -> str:
    """Nearest binary32 to the exact decimal value (no double rounding)."""
    import numpy as np
    v = np.float32(float(d))
    cands = [v, np.nextafter(v, np.float32(np.inf)), np.nextafter(v, np.float32(-np.inf))]
    best = min(cands, key=lambda x: abs(Decimal(float(x)) - d))
    return repr(float(best)) + "f"


def emit(path):
    hops, c, c2, w = derive()
    shell_of = [SHELLS.index(ex * ex + ey * ey) for ex, ey in hops]
    lines = []
    lines.append("// d2q37_tables.h -- generated by gen_d2q37_tables.py; do not edit.")
    lines.append("// D2Q37 hop set, canonical order, quadrature weights and scale c")
    lines.append("// (exact-rational derivation, rounded once; see the generator).")
    lines.append("#pragma once")
    lines.append("namespace d2q37 {")
    lines.append("constexpr int NPOP = 37;")
    lines.append("constexpr int NSHELL = 8;")
    lines.append("constexpr int EX[NPOP] = {" + ", ".join(str(h[0]) for h in hops) + "};")
    lines.append("constexpr int EY[NPOP] = {" + ", ".join(str(h[1]) for h in hops) + "};")
    lines.append("constexpr int SHELL[NPOP] = {" + ", ".join(map(str, shell_of)) + "};")
    lines.append("constexpr int SHELL_R2[NSHELL] = {" + ", ".join(map(str, SHELLS)) + "};")
    lines.append(f"constexpr double C = {f64(c)};   // {c:.30f}")
    lines.append(f"constexpr double C2 = {f64(c2)};  // {c2:.30f}")
    lines.append(f"constexpr float C_F = {f32(c)};")
    lines.append(f"constexpr float C2_F = {f32(c2)};")
    lines.append("constexpr double W_SHELL[NSHELL] = {" + ", ".join(f64(x) for x in w) + "};")
    lines.append("constexpr float W_SHELL_F[NSHELL] = {" + ", ".join(f32(x) for x in w) + "};")
    lines.append("// shell weights, 30 digits: " + ", ".join(f"{x:.30f}" for x in w))
    lines.append("// |xi|^2 = c^2 |e|^2 of each shell, rounded once")
    lines.append("constexpr double X2_SHELL[NSHELL] = {" + ", ".join(f64(c2 * s) for s in SHELLS) + "};")
    lines.append("constexpr float X2_SHELL_F[NSHELL] = {" + ", ".join(f32(c2 * s) for s in SHELLS) + "};")
    lines.append("}  // namespace d2q37")
    with open(path, "w") as fh:
        fh.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    out = sys.argv[1] if len(sys.argv) > 1 else os.path.join(os.path.dirname(os.path.abspath(__file__)), "d2q37_tables.h")
    emit(out)
    print("wrote", out)
