"""Pins of the oracle's integrator tableau and of its right-hand side against
the trace Einstein equation.  CPU only.

1. The ESDIRK tableau (the implicit part of Kennedy & Carpenter's additive
   scheme ARK4(3)6L[2]SA, Appl. Numer. Math. 44 (2003); the paper names no
   solver, App. A.2 solver options) is read as exact rationals from the
   oracle's C source and checked against the Runge-Kutta order conditions:
   order 4 for the propagating weights, order 3 for the embedded ones, stage
   order 2, stiff accuracy, a constant diagonal gamma = 1/4, L-stability
   (R(z) -> 0 as z -> -inf) and A-stability on the imaginary axis.  The
   perturbation kernel's separately typed rationals are checked to be the same
   numbers.

2. The trace (ii) Einstein equation (Ma & Bertschinger 1995, eq. 21c),
       h_dd + 2 Hc h_d - 2 k^2 eta = -24 pi G a^2 dP,
   is never used by the evolution (App. B.3 evolves eta with the 0i equation
   and takes h' from the 00 equation).  Given energy conservation of each
   species and the Friedmann equations it is an identity, so evaluating it
   algebraically from a state y, the oracle's y' = A y and the closed-form
   background pins the continuity rows, both constraint equations and the
   background at once.
"""
import ast
import math
import os
import re
from fractions import Fraction

import numpy as np
import pytest

import cmb_workloads as W
import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


# ---------------------------------------------------------------- tableau
def _initializer(src: str, name: str) -> str:
    """Text between the braces of `name[...] = { ... };` in C source."""
    m = re.search(re.escape(name) + r"\s*(\[[^\]]*\]\s*)+=\s*\{", src)
    assert m, name
    i = m.end() - 1
    depth = 0
    for j in range(i, len(src)):
        if src[j] == "{":
            depth += 1
        elif src[j] == "}":
            depth -= 1
            if depth == 0:
                return src[i + 1:j]
    raise AssertionError(name)


def _exact(expr: str) -> Fraction:
    """A C constant expression of decimal literals, + - * / and unary minus,
    evaluated exactly (each literal as the decimal number it spells)."""
    tree = ast.parse(expr.strip(), mode="eval")

    def ev(n):
        if isinstance(n, ast.Expression):
            return ev(n.body)
        if isinstance(n, ast.Constant):
            return Fraction(ast.get_source_segment(expr.strip(), n))
        if isinstance(n, ast.UnaryOp) and isinstance(n.op, ast.USub):
            return -ev(n.operand)
        if isinstance(n, ast.BinOp):
            a, b = ev(n.left), ev(n.right)
            if isinstance(n.op, ast.Add):
                return a + b
            if isinstance(n.op, ast.Sub):
                return a - b
            if isinstance(n.op, ast.Mult):
                return a * b
            if isinstance(n.op, ast.Div):
                return a / b
        raise AssertionError(ast.dump(n))

    return ev(tree)


def _elements(body: str) -> list[Fraction]:
    flat = body.replace("{", " ").replace("}", " ")
    return [_exact(e) for e in flat.split(",") if e.strip()]


def _oracle_tableau():
    src = open(os.path.join(ROOT, "oracle", "perturb.c")).read()
    c = _elements(_initializer(src, "RK_c"))
    A = _elements(_initializer(src, "RK_A"))
    bh = _elements(_initializer(src, "RK_bh"))
    s = len(c)
    assert len(A) == s * s and len(bh) == s
    return c, [A[i * s:(i + 1) * s] for i in range(s)], bh


def _order_conditions(b, A, c, order):
    """Residuals of the Runge-Kutta order conditions up to `order` (Butcher
    trees through order 4)."""
    s = len(c)
    Ac = [sum(A[i][j] * c[j] for j in range(s)) for i in range(s)]
    Ac2 = [sum(A[i][j] * c[j] ** 2 for j in range(s)) for i in range(s)]
    AAc = [sum(A[i][j] * Ac[j] for j in range(s)) for i in range(s)]
    dot = lambda u, v: sum(x * y for x, y in zip(u, v))
    conds = [(dot(b, [1] * s), Fraction(1))]
    if order >= 2:
        conds.append((dot(b, c), Fraction(1, 2)))
    if order >= 3:
        conds += [(dot(b, [x * x for x in c]), Fraction(1, 3)), (dot(b, Ac), Fraction(1, 6))]
    if order >= 4:
        conds += [(dot(b, [x ** 3 for x in c]), Fraction(1, 4)),
                  (dot(b, [x * y for x, y in zip(c, Ac)]), Fraction(1, 8)),
                  (dot(b, Ac2), Fraction(1, 12)), (dot(b, AAc), Fraction(1, 24))]
    return [v - t for v, t in conds]


def _stability(A, b, z):
    """R(z) = 1 + z b^T (I - z A)^-1 1, by forward substitution (A is lower
    triangular); exact for Fraction z."""
    s = len(b)
    K = []
    for i in range(s):
        acc = 1 + z * sum(A[i][j] * K[j] for j in range(i))
        K.append(acc / (1 - z * A[i][i]))
    return 1 + z * sum(b[j] * K[j] for j in range(s))


def test_tableau_order_conditions_exact():
    c, A, bh = _oracle_tableau()
    s = len(c)
    b = A[-1]  # stiffly accurate: the propagating weights are the last row
    assert c[0] == 0 and c[-1] == 1
    for i in range(s):
        assert sum(A[i]) == c[i], i                      # row sums
        assert all(A[i][j] == 0 for j in range(i + 1, s))  # lower triangular
    assert A[0][0] == 0                                  # explicit first stage
    assert all(A[i][i] == Fraction(1, 4) for i in range(1, s))
    assert all(r == 0 for r in _order_conditions(b, A, c, 4))
    assert all(r == 0 for r in _order_conditions(bh, A, c, 3))
    # the embedded weights are not order 4, so b - bh estimates the error
    assert any(r != 0 for r in _order_conditions(bh, A, c, 4))
    # stage order 2: sum_j a_ij c_j = c_i^2 / 2 for every implicit stage
    for i in range(1, s):
        assert sum(A[i][j] * c[j] for j in range(s)) == c[i] ** 2 / 2, i


def test_tableau_stability():
    c, A, bh = _oracle_tableau()
    b = A[-1]
    # L-stability: R(z) is a rational function whose numerator degree is
    # below the denominator's, so R(-1e8) must be tiny (exact arithmetic)
    assert abs(_stability(A, b, Fraction(-10 ** 8))) < Fraction(1, 10 ** 6)
    assert abs(_stability(A, b, Fraction(-10 ** 12))) < Fraction(1, 10 ** 10)
    # consistency: R(z) = e^z + O(z^5) near 0
    z = Fraction(1, 1000)
    assert abs(float(_stability(A, b, z)) - math.exp(1e-3)) < 1e-14
    # A-stability: the poles sit at z = 1/gamma = 4 (right half-plane), so
    # |R(iy)| <= 1 on the imaginary axis suffices
    Af = [[float(x) for x in row] for row in A]
    bf = [float(x) for x in b]
    for y in np.concatenate([np.logspace(-3, 6, 4000), -np.logspace(-3, 6, 50)]):
        assert abs(_stability(Af, bf, complex(0.0, y))) <= 1.0 + 1e-12, y


def test_kernel_tableau_is_the_oracle_tableau():
    """The perturbation kernel types the same rationals separately; they must
    be the same numbers (error weights b - bh included)."""
    c, A, bh = _oracle_tableau()
    src = open(os.path.join(ROOT, "paper_2602_15104_amd", "csrc", "k1_common.h")).read()
    kc = _elements(_initializer(src, "Kc"))
    kA = _elements(_initializer(src, "Ka"))
    ke = _elements(_initializer(src, "Ke"))
    s = len(c)
    assert kc == c
    assert [kA[i * s:(i + 1) * s] for i in range(s)] == A
    assert ke == [A[-1][j] - bh[j] for j in range(s)]


def test_tableau_parser_sees_a_planted_typo():
    """The exact checks are sharp: one digit changed in one entry breaks the
    order conditions (a planted mistake in a copy of the tableau)."""
    c, A, bh = _oracle_tableau()
    A2 = [row[:] for row in A]
    A2[3][2] += Fraction(1, 388108)
    A2[3][3] -= Fraction(1, 388108)  # keep the row sum
    assert any(r != 0 for r in _order_conditions(A2[-1], A2, c, 4)) or \
        any(sum(A2[i][j] * c[j] for j in range(len(c))) != c[i] ** 2 / 2 for i in range(1, len(c)))


# ---------------------------------------------------------------- trace equation
def _trace_residual(t, k, lna, y, f):
    """Relative residual of the trace Einstein equation at one state, in
    conformal time, with h' = dh/dln a from the 00 equation and eta', the
    density contrasts' derivatives from f = y' (oracle layout: delta_c,
    delta_b, theta_b, delta_g, ..., delta_nu at the neutrino block, eta last).
    Densities in units where Hc^2 = a^2 sum rho (so 8 pi G/3 -> 1)."""
    bg = t.bg
    prec = t.prec
    lg, lp = int(prec["ell_gamma"]), int(prec["ell_pol"])
    g0 = 3
    n0 = g0 + lg + 1 + (lp + 1 if lp > 0 else 0)
    a = math.exp(lna)
    rg, rur = bg.rt_g0 / a ** 4, bg.rt_ur0 / a ** 4
    rc, rb = bg.rt_c0 / a ** 3, bg.rt_b0 / a ** 3
    rho = rg + rur + rc + rb + bg.rt_L
    drho_dlna = -4.0 * (rg + rur) - 3.0 * (rc + rb)       # Lambda is constant
    Hc = a * math.sqrt(rho)
    Hcp = Hc + a * drho_dlna / (2.0 * math.sqrt(rho))      # dHc/dln a
    eta, etap = y[-1], f[-1]
    dens = [(rc, -3.0 * rc, 0), (rb, -3.0 * rb, 1), (rg, -4.0 * rg, g0), (rur, -4.0 * rur, n0)]
    drho = sum(r * y[i] for r, _, i in dens)
    ddrho = sum(dr * y[i] + r * f[i] for r, dr, i in dens)
    # 00 equation: k^2 eta - Hc h_dot / 2 = -4 pi G a^2 delta rho
    hp = (2.0 * k * k * eta + 3.0 * a * a * drho) / Hc ** 2
    hpp = (2.0 * k * k * (etap - 2.0 * eta * Hcp / Hc) +
           3.0 * (2.0 * a * a * drho + a * a * ddrho - 2.0 * a * a * drho * Hcp / Hc)) / Hc ** 2
    h_d = Hc * hp
    h_dd = Hc * (Hcp * hp + Hc * hpp)
    dP = (rg * y[g0] + rur * y[n0]) / 3.0
    terms = [h_dd, 2.0 * Hc * h_d, -2.0 * k * k * eta, 9.0 * a * a * dP]
    return abs(sum(terms)) / max(abs(x) for x in terms)


@pytest.mark.parametrize("cfg", ["config0", "config1"])
def test_trace_einstein_equation_along_solutions(cfg):
    """P5 (i): along oracle solutions of configs 0 and 1 (several modes, every
    output time) the unused trace equation holds to <= 1e-10 relative."""
    wl = getattr(W, cfg)()
    idx = [0, len(wl.k) // 3, 2 * len(wl.k) // 3, len(wl.k) - 1]
    t = O.build_tables(wl.cosmo, wl.prec, wl.k[idx], 120)
    worst = 0.0
    for i in range(len(idx)):
        k = float(t.k[i])
        r = O.perturb_one(t, k, float(t.lna_i[i]), t.lna_src, want_y=True)
        assert r["status"] == 0
        for j, lna in enumerate(t.lna_src):
            y = r["y"][j]
            if not np.any(y):
                continue
            worst = max(worst, _trace_residual(t, k, float(lna), y, O.rhs(t, k, float(lna), y)))
    assert worst <= 1e-10, worst


def test_trace_einstein_equation_any_state_and_sensitivity():
    """The identity needs no solution: it holds for seeded random states.  A
    planted 0.1 % error in one continuity row (CDM's -h'/2) or in the 0i
    coupling (eta') breaks it by orders of magnitude."""
    wl = W.config1()
    t = O.build_tables(wl.cosmo, wl.prec, wl.k[[10, 200]], 60)
    rng = np.random.Generator(np.random.PCG64(7))
    N = O.state_size(t.prec, 0)
    for k in t.k:
        for lna in (-12.0, -7.0, -3.0, -0.1):
            y = rng.standard_normal(N)
            f = O.rhs(t, float(k), lna, y)
            assert _trace_residual(t, float(k), lna, y, f) <= 1e-11
            f_bad = f.copy()
            f_bad[0] *= 1.001                             # CDM continuity row off by 0.1 %
            f_bad2 = f.copy()
            f_bad2[-1] *= 1.001                           # eta' off by 0.1 %
            assert _trace_residual(t, float(k), lna, y, f_bad) > 1e-7
            assert _trace_residual(t, float(k), lna, y, f_bad2) > 1e-7
