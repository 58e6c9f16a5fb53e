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
