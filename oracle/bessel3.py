"""Oracle for the paper's three-region spherical Bessel scheme and the
line-of-sight projection built on it (arXiv 2602.15104, App. B.4, the
Bessel strategy below the transfer integrals).

TEST INFRASTRUCTURE ONLY: imported by tests/, never by the library.

For each multipole l >= 1 the scheme approximates j_l(x) by
  * 0 for x <= x_start(l), the first x where j_l reaches 1e-10;
  * linear interpolation on 5000 equally spaced samples of j_l over
    [x_start(l), x_5(l)], x_5 being the fifth local maximum of j_l;
  * above x_5 the leading Debye-type asymptotic form
        j_l(x) ~ cos(Q_nu(x) - pi/4) / sqrt(x sqrt(x^2 - nu^2)),
        Q_nu(x) = sqrt(x^2 - nu^2) - nu pi/2 + nu arcsin(nu/x),  nu = l + 1/2.
The samples come from scipy.special.spherical_jn, as in the paper.

Readings (where the paper leaves a choice): "local maximum" is a maximum of
j_l itself (its positive peaks); the first derivative used by the projection
is j_l' = j_{l-1} - (l+1) j_l / x from the same scheme's j_{l-1} and j_l, and
j_l'' follows from Bessel's equation; the x = 0 limits are those of the exact
functions.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import spherical_jn

THRESH = 1e-10
N_PTS = 5000


def x_start(ells: np.ndarray) -> np.ndarray:
    """First x with j_l(x) = 1e-10: j_l rises monotonically from 0 on
    (0, nu], so bisection on [0, nu] (to rounding)."""
    ells = np.asarray(ells)
    lo = np.zeros(len(ells))
    hi = ells + 0.5
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        up = spherical_jn(ells, mid) > THRESH
        hi = np.where(up, mid, hi)
        lo = np.where(up, lo, mid)
        if np.all(hi - lo <= 4e-16 * hi):
            break
    return hi


def x_fifth_max(ells: np.ndarray) -> np.ndarray:
    """Fifth zero of j_l' at which j_l' turns from positive to negative.
    The first maximum lies beyond nu, so all l are scanned together from nu
    in steps of 0.2 (consecutive zeros of j_l' are more than 2 apart) and
    each bracket is then bisected."""
    ells = np.asarray(ells)
    nu = ells + 0.5
    found = np.zeros(len(ells), dtype=np.int64)
    a = np.full(len(ells), np.nan)
    d_prev = spherical_jn(ells, nu, derivative=True)
    i = 0
    while np.any(found < 5):
        i += 1
        assert i < 100000
        x = nu + 0.2 * i
        d = spherical_jn(ells, x, derivative=True)
        hit = (found < 5) & (d_prev > 0) & (d <= 0)
        found += hit
        a = np.where(hit & (found == 5), x - 0.2, a)
        d_prev = d
    b = a + 0.2
    for _ in range(200):
        m = 0.5 * (a + b)
        up = spherical_jn(ells, m, derivative=True) > 0
        a = np.where(up, m, a)
        b = np.where(up, b, m)
        if np.all(b - a <= 4e-16 * b):
            break
    return 0.5 * (a + b)


class Table:
    """x_start, x_5 and the 5000 samples of j_l for 1 <= l <= ell_max
    (index l - 1)."""

    def __init__(self, ell_max: int, n_pts: int = N_PTS):
        ells = np.arange(1, ell_max + 1)
        self.ell_max = ell_max
        self.xs = x_start(ells)
        self.x5 = x_fifth_max(ells)
        self.n = n_pts
        self.dx = (self.x5 - self.xs) / (n_pts - 1)
        self.tab = np.empty((ell_max, n_pts))
        for i, l in enumerate(ells):
            self.tab[i] = spherical_jn(l, self.xs[i] + self.dx[i] * np.arange(n_pts))


def debye(l: int, x):
    """Leading Debye-type form for x above the turning point."""
    nu = l + 0.5
    s = np.sqrt(x * x - nu * nu)
    return np.cos(s - nu * math.pi / 2 + nu * np.arcsin(nu / x) - math.pi / 4) / np.sqrt(x * s)


def j3(T: Table, l: int, x: np.ndarray) -> np.ndarray:
    """The scheme's j_l(x) for an array of x >= 0 (l = 0: sin x / x)."""
    x = np.asarray(x, dtype=np.float64)
    if l == 0:
        return np.where(x > 0, np.sin(x) / np.where(x > 0, x, 1.0), 1.0)
    xs, x5, dx = T.xs[l - 1], T.x5[l - 1], T.dx[l - 1]
    out = np.zeros_like(x)
    mid = (x > xs) & (x <= x5)
    u = (x[mid] - xs) / dx
    i = np.minimum(np.floor(u).astype(np.int64), T.n - 2)
    f = u - i
    out[mid] = (1.0 - f) * T.tab[l - 1, i] + f * T.tab[l - 1, i + 1]
    hi = x > x5
    out[hi] = debye(l, x[hi])
    return out


def los3(t, S: np.ndarray, ell_max: int, pol: bool, T: Table | None = None, k=None, s_pol=None, jfun=None):
    """Delta_T, Delta_E [l-2][k] with the scheme's Bessel functions (or with
    jfun(l, x) in its place, e.g. the exact function, to check the assembly).

      Delta_T = sum_j w_j [S_T0 j + S_T1 j' + s_pol S_T2 (3 j'' + j)/2]
      Delta_E = sqrt(3 (l+2)!/(8 (l-2)!)) sum_j w_j sqrt(6) S_T2 j / x^2
    with j' = j_{l-1} - (l+1) j/x and (3j''+j)/2 = -(3/x) j' + (3 l(l+1)/(2x^2) - 1) j.
    """
    k = np.asarray(t.k if k is None else k, dtype=np.float64)
    chi, w = np.asarray(t.chi_src), np.asarray(t.w_src)
    sp = t.prec["scale_pol"] if s_pol is None else s_pol
    if jfun is None:
        jfun = lambda l, x: j3(T, l, x)  # noqa: E731
    x = k[:, None] * chi[None, :]
    zero = x == 0.0
    xs = np.where(zero, 1.0, x)
    S0, S1, S2 = S[:, 0, :], S[:, 1, :], S[:, 2, :]
    nl = ell_max - 1
    DT = np.zeros((nl, len(k)))
    DE = np.zeros((nl, len(k)))
    jm = jfun(1, x.ravel()).reshape(x.shape)
    for l in range(2, ell_max + 1):
        j = jfun(l, x.ravel()).reshape(x.shape)
        jp = jm - (l + 1) * j / xs
        t2 = -3.0 / xs * jp + (1.5 * l * (l + 1) / (xs * xs) - 1.0) * j
        e2 = j / (xs * xs)
        j_, jp_ = np.where(zero, 0.0, j), np.where(zero, 0.0, jp)
        t2 = np.where(zero, 0.2 if l == 2 else 0.0, t2)
        e2 = np.where(zero, 1.0 / 15.0 if l == 2 else 0.0, e2)
        DT[l - 2] = np.sum(w * (S0 * j_ + S1 * jp_ + sp * S2 * t2), axis=1)
        if pol:
            cl = math.sqrt(3.0 * (l + 2.0) * (l + 1.0) * l * (l - 1.0) / 8.0)
            DE[l - 2] = cl * np.sum(w * math.sqrt(6.0) * S2 * e2, axis=1)
        jm = j
    return DT, DE
