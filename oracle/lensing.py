"""Oracle for the lensing potential (arXiv 2602.15104, App. B.5).

TEST INFRASTRUCTURE ONLY: imported by tests/, never by the library.

Limber's approximation for the lensing-potential spectrum,
  C_l^psipsi = 8 pi^2/(l+1/2)^3 int_0^chi_* dchi/chi P_psi(k = (l+1/2)/chi, tau_0 - chi) ((chi_*-chi)/chi_*)^2,
  P_psi(k, a) = 9 Omega_m(a)^2 H(a)^4 / (8 pi^2 k) P(k, a),
  P(k, a) = 2 pi^2/k^3 P_R(k) delta_m(k, a)^2,                (eq. PK)
with Omega_m = rho_m / rho_tot and H = a H the conformal Hubble rate, so that
9 Omega_m^2 H^4 / 4 = (3/2 a^2 rho_m)^2 in the units where H^2 = sum rho.

Readings: chi_* is tau_0 minus the conformal time of the visibility peak
(the maximum of kappa' e^-kappa over the table knots, refined by the vertex
of the parabola through the three knots around it); the chi integral is the
output-time quadrature (trapezoid in ln a divided by H) over the output
times with 0 < chi < chi_*; delta_m(k, tau_j) at k = (l+1/2)/chi_j is the
natural cubic spline in k of the perturbation grid's values at that output
time, and zero outside the grid's k range; rho_m and delta_m run over CDM,
baryons and massive neutrinos; C_0 = C_1 = 0.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.interpolate import CubicSpline

from . import background as B


def visibility_peak(t):
    """(ln a_*, tau_*, chi_*) of the visibility peak."""
    g = np.exp(np.asarray(t.cols["ln_dk"]) - np.asarray(t.cols["kappa"]))
    n = len(g) - 1
    j = 1 + int(np.argmax(g[1:n]))
    gm, g0, gp = g[j - 1], g[j], g[j + 1]
    den = gm - 2.0 * g0 + gp
    off = 0.5 * (gm - gp) / den if den != 0.0 else 0.0
    lna = t.lna[j] + off * (t.lna[j + 1] - t.lna[j])
    tau = math.exp(B.spline_eval(t.cols["ln_tau"], t.M["ln_tau"], t.L0, t.dl, lna))
    return lna, tau, t.tau0 - tau


def limber_weights(t) -> np.ndarray:
    """Per output time: w_j / chi_j (3/2 a^2 rho_m)^2 ((chi_*-chi_j)/chi_*)^2
    for 0 < chi_j < chi_*, else 0."""
    _, _, cs = visibility_peak(t)
    bg = t.bg
    out = np.zeros(len(t.lna_src))
    for j, (lna, chi, w) in enumerate(zip(t.lna_src, t.chi_src, t.w_src)):
        if not (0.0 < chi < cs):
            continue
        a = math.exp(lna)
        rho_m = bg.rt_m0 / a ** 3 + bg.rho_ncdm(a)[0]
        src = 1.5 * a * a * rho_m
        out[j] = w / chi * src * src * ((cs - chi) / cs) ** 2
    return out


def limber_cl(t, Dm: np.ndarray, ell_max: int, k=None) -> np.ndarray:
    """C_l^psipsi [ell_max + 1] from delta_m[n_k][n_tau] on the k grid."""
    k = np.asarray(t.k if k is None else k, dtype=np.float64)
    W = limber_weights(t)
    sp = CubicSpline(k, np.asarray(Dm), axis=0, bc_type="natural")
    A_s, n_s, kp = t.cosmo["A_s"], t.cosmo["n_s"], t.prec["k_pivot"]
    out = np.zeros(ell_max + 1)
    js = np.nonzero(W)[0]
    chi = np.asarray(t.chi_src)[js]
    for l in range(2, ell_max + 1):
        nu = l + 0.5
        kk = nu / chi
        ok = (kk >= k[0]) & (kk <= k[-1])
        if not np.any(ok):
            continue
        j, kk = js[ok], kk[ok]
        # each output time's own spline at its own k (piecewise cubic form)
        i = np.clip(np.searchsorted(k, kk, side="right") - 1, 0, len(k) - 2)
        dx = kk - k[i]
        c = sp.c
        d = ((c[0, i, j] * dx + c[1, i, j]) * dx + c[2, i, j]) * dx + c[3, i, j]
        out[l] = 8.0 * math.pi ** 2 / nu ** 3 * float(np.sum(W[j] * A_s * (kk / kp) ** (n_s - 1.0) * d * d / kk ** 4))
    return out


# ---------------------------------------------------------------------------
# Lensed spectra from full-sky correlation functions (App. B.5, following the
# correlation-function method of Challinor & Lewis 2005 that the paper
# implements), integrated over the full range of mu = cos(beta) by
# Gauss-Legendre quadrature ("accurate" lensing; no restricted-range variant).
# ---------------------------------------------------------------------------
def _d_explicit(l: int, mp: int, m: int, mu: np.ndarray) -> np.ndarray:
    """Wigner d^l_{m'm}(beta), mu = cos(beta), by Wigner's explicit sum
    (d^l_{m'm} = <l m'| exp(-i J_y beta) |l m>); for small l (start values and
    pins)."""
    f = math.factorial
    c = np.sqrt((1.0 + mu) / 2.0)
    s = np.sqrt(np.maximum((1.0 - mu) / 2.0, 0.0))
    out = np.zeros_like(mu)
    pre = math.sqrt(f(l + m) * f(l - m) * f(l + mp) * f(l - mp))
    for k in range(0, 2 * l + 1):
        a, b, cc, d = l + m - k, k, l - k - mp, k - m + mp
        if min(a, b, cc, d) < 0:
            continue
        coef = (-1) ** (k - m + mp) * pre / (f(a) * f(b) * f(cc) * f(d))
        out = out + coef * c ** (2 * l - 2 * k + m - mp) * s ** (2 * k - m + mp)
    return out


def wigner_d(mp: int, m: int, lmax: int, mu: np.ndarray) -> np.ndarray:
    """d^l_{m'm}(mu) for 0 <= l <= lmax ([lmax+1][n_mu], zero below
    max(|m'|, |m|)) by the three-term recurrence in l:
      l sqrt(((l+1)^2 - m'^2)((l+1)^2 - m^2)) d^{l+1}
        = (2l+1)(l(l+1) mu - m' m) d^l - (l+1) sqrt((l^2 - m'^2)(l^2 - m^2)) d^{l-1}."""
    mu = np.asarray(mu, dtype=np.float64)
    out = np.zeros((lmax + 1, len(mu)))
    l0 = max(abs(mp), abs(m))
    if l0 > lmax:
        return out
    out[l0] = _d_explicit(l0, mp, m, mu)
    prev = np.zeros_like(mu)
    for l in range(l0, lmax):
        if l == 0:
            out[1] = mu * out[0]  # m' = m = 0: P_1
            prev = out[0]
            continue
        a = (2 * l + 1) * (l * (l + 1) * mu - mp * m)
        b = (l + 1) * math.sqrt(max((l * l - mp * mp) * (l * l - m * m), 0))
        c = l * math.sqrt(((l + 1) ** 2 - mp * mp) * ((l + 1) ** 2 - m * m))
        out[l + 1] = (a * out[l] - b * prev) / c
        prev = out[l]
    return out


def x_functions(ells: np.ndarray, sig2: np.ndarray) -> dict:
    """Small-deflection forms of the X_imn(sigma^2) of the method, [l][mu]
    (l >= 2), and the derivatives X'_imn = dX_imn/dsigma^2 that it uses."""
    l = np.asarray(ells, dtype=np.float64)[:, None]
    s = np.asarray(sig2)[None, :]
    ll = l * (l + 1.0)
    X = {}
    X["000"] = np.exp(-ll * s / 4.0)
    X["p000"] = -ll / 4.0 * X["000"]
    X["220"] = 0.25 * np.sqrt(np.maximum((l + 2) * (l - 1) * l * (l + 1), 0)) * np.exp(-(ll - 2.0) * s / 4.0)
    X["022"] = np.exp(-(ll - 4.0) * s / 4.0)
    X["p022"] = -(ll - 4.0) / 4.0 * X["022"]
    X["121"] = -0.5 * np.sqrt(np.maximum((l + 2) * (l - 1), 0)) * np.exp(-(ll - 8.0 / 3.0) * s / 4.0)
    X["112"] = X["121"]
    X["132"] = -0.5 * np.sqrt(np.maximum((l + 3) * (l - 2), 0)) * np.exp(-(ll - 20.0 / 3.0) * s / 4.0)
    X["242"] = 0.25 * np.sqrt(np.maximum((l + 4) * (l + 3) * (l - 2) * (l - 3), 0)) * np.exp(-(ll - 10.0) * s / 4.0)
    return X


class _DRec:
    """d^l_{m'm}(mu) for l = l0, l0+1, ... by the three-term recurrence of
    wigner_d, one multipole at a time (memory O(n_mu))."""

    def __init__(self, mp: int, m: int, mu: np.ndarray):
        self.mp, self.m, self.mu = mp, m, mu
        self.l0 = max(abs(mp), abs(m))
        self.l = -1
        self.cur = np.zeros_like(mu)
        self.prev = np.zeros_like(mu)

    def at(self, l: int) -> np.ndarray:
        """d^l on the nodes; l must not decrease between calls."""
        if l < self.l0:
            return np.zeros_like(self.mu)
        while self.l < l:
            if self.l < self.l0:
                self.cur, self.prev, self.l = _d_explicit(self.l0, self.mp, self.m, self.mu), np.zeros_like(self.mu), \
                    self.l0
                continue
            k, mp, m = self.l, self.mp, self.m
            if k == 0:
                nxt = self.mu * self.cur
            else:
                a = (2 * k + 1) * (k * (k + 1) * self.mu - mp * m)
                b = (k + 1) * math.sqrt(max((k * k - mp * mp) * (k * k - m * m), 0))
                c = k * math.sqrt(((k + 1) ** 2 - mp * mp) * ((k + 1) ** 2 - m * m))
                nxt = (a * self.cur - b * self.prev) / c
            self.prev, self.cur, self.l = self.cur, nxt, k + 1
        return self.cur


def lensed_cl(Cl: np.ndarray, Clpp: np.ndarray, ell_max: int, n_mu: int) -> np.ndarray:
    """Lensed TT, TE, EE, BB [4][ell_max+1] from unlensed Cl[3][L+1] (TT, TE,
    EE; no primordial B) and the lensing-potential spectrum Clpp[L+1]:

      C_gl(b)   = sum_l (2l+1)/(4 pi) l(l+1) C_l^psi d^l_11(b),
      C_gl,2(b) = sum_l (2l+1)/(4 pi) l(l+1) C_l^psi d^l_{1,-1}(b),
      sigma^2   = C_gl(0) - C_gl(b),
      xi_T  = sum_l (2l+1)/(4 pi) C_l^T  [X000^2 d00 + 8/(l(l+1)) C_gl,2 X'000^2 d1-1
                                        + C_gl,2^2 (X'000^2 d00 + X220^2 d2-2)],
      xi_+  = sum_l (2l+1)/(4 pi) (C^E+C^B) [X022^2 d22 + 2 C_gl,2 X132 X121 d31
                                        + C_gl,2^2 (X'022^2 d22 + X242 X220 d40)],
      xi_-  = sum_l (2l+1)/(4 pi) (C^E-C^B) [X022^2 d2-2 + C_gl,2 (X121^2 d1-1 + X132^2 d3-3)
                                        + C_gl,2^2 (2 X'022^2 d2-2 + X220^2 d00 + X242^2 d4-4)/2],
      xi_x  = sum_l (2l+1)/(4 pi) C^X [X022 X000 d02 + C_gl,2 2 X'000/sqrt(l(l+1)) (X112 d11 + X132 d3-1)
                                        + C_gl,2^2 ((2 X'022 X'000 + X220^2) d20 + X220 X242 d-24)/2],
    then  C~^T = 2 pi int xi_T d00,  C~^E +- C~^B = 2 pi int xi_+- d22 (d2-2),
    C~^X = 2 pi int xi_x d20, over mu in [-1, 1] by n_mu-point Gauss-Legendre.
    Only the lensing change of each correlation function is transformed (the
    leading X products enter as X^2 - 1 by expm1) and added to the unlensed
    spectra, which keeps the high-l results free of the low-l rounding."""
    from scipy.special import roots_legendre
    L = len(Clpp) - 1
    mu, w = roots_legendre(n_mu)
    Clpp = np.asarray(Clpp, dtype=np.float64)
    Cgl, Cgl2, Cgl0 = np.zeros(n_mu), np.zeros(n_mu), 0.0
    r11, r1m1 = _DRec(1, 1, mu), _DRec(1, -1, mu)
    for l in range(2, L + 1):
        f = (2 * l + 1) / (4 * math.pi) * l * (l + 1.0) * Clpp[l]
        Cgl += f * r11.at(l)
        Cgl2 += f * r1m1.at(l)
        Cgl0 += f
    sig2 = Cgl0 - Cgl
    pairs = {"00": (0, 0), "1-1": (1, -1), "2-2": (2, -2), "22": (2, 2), "31": (3, 1), "3-3": (3, -3), "40": (4, 0),
             "4-4": (4, -4), "02": (0, 2), "11": (1, 1), "3-1": (3, -1), "20": (2, 0), "-24": (-2, 4)}
    rec = {key: _DRec(a, b, mu) for key, (a, b) in pairs.items()}
    xiT, xiP, xiM, xiX = (np.zeros(n_mu) for _ in range(4))
    c2 = Cgl2
    for l in range(2, L + 1):
        D = {key: r.at(l) for key, r in rec.items()}
        Xl = {key: v[0] for key, v in x_functions(np.array([l]), sig2).items()}
        pre = (2 * l + 1) / (4 * math.pi)
        llp = l * (l + 1.0)
        T, X_, E = Cl[0][l], Cl[1][l], Cl[2][l]
        dT = np.expm1(-llp * sig2 / 2.0)          # X000^2 - 1
        dP = np.expm1(-(llp - 4.0) * sig2 / 2.0)  # X022^2 - 1
        dX = np.expm1(-(2.0 * llp - 4.0) * sig2 / 4.0)  # X022 X000 - 1
        xiT += pre * T * (dT * D["00"] + 8.0 / llp * c2 * Xl["p000"] ** 2 * D["1-1"]
                          + c2 ** 2 * (Xl["p000"] ** 2 * D["00"] + Xl["220"] ** 2 * D["2-2"]))
        xiP += pre * E * (dP * D["22"] + 2.0 * c2 * Xl["132"] * Xl["121"] * D["31"]
                          + c2 ** 2 * (Xl["p022"] ** 2 * D["22"] + Xl["242"] * Xl["220"] * D["40"]))
        xiM += pre * E * (dP * D["2-2"] + c2 * (Xl["121"] ** 2 * D["1-1"] + Xl["132"] ** 2 * D["3-3"])
                          + 0.5 * c2 ** 2 * (2.0 * Xl["p022"] ** 2 * D["2-2"] + Xl["220"] ** 2 * D["00"]
                                             + Xl["242"] ** 2 * D["4-4"]))
        xiX += pre * X_ * (dX * D["02"]
                           + c2 * 2.0 * Xl["p000"] / math.sqrt(llp) * (Xl["112"] * D["11"] + Xl["132"] * D["3-1"])
                           + 0.5 * c2 ** 2 * ((2.0 * Xl["p022"] * Xl["p000"] + Xl["220"] ** 2) * D["20"]
                                              + Xl["220"] * Xl["242"] * D["-24"]))
    out = np.zeros((4, ell_max + 1))
    back = {key: _DRec(a, b, mu) for key, (a, b) in {"00": (0, 0), "22": (2, 2), "2-2": (2, -2), "20": (2, 0)}.items()}
    for l in range(2, ell_max + 1):
        tt = 2 * math.pi * np.sum(w * xiT * back["00"].at(l))
        p = 2 * math.pi * np.sum(w * xiP * back["22"].at(l))
        m = 2 * math.pi * np.sum(w * xiM * back["2-2"].at(l))
        x = 2 * math.pi * np.sum(w * xiX * back["20"].at(l))
        out[0, l] = Cl[0][l] + tt
        out[1, l] = Cl[1][l] + x
        out[2, l] = Cl[2][l] + 0.5 * (p + m)
        out[3, l] = 0.5 * (p - m)
    return out
