"""The CPU oracle for the CMB hot path of arXiv 2602.15104.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, independent
reference against which the HIP library (package ``paper_2602_15104_amd``) is
checked.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg
of ``bench.py`` may import it.  It shares no code with the library: its
tables are built by ``oracle.background`` (Python), its perturbation
integrator, Bessel functions and quadratures are the C files in this folder,
compiled with gcc.

Functions
---------
build_tables(cosmo, prec, k, n_tau)   background/thermo tables, start times,
                                      output grid (App. A.2, B.1, B.2, B.4)
perturb(tab, idx=None, ...)           sources S[k][3][n_tau] (App. B.3, C, B.4)
los(tab, S, ell_max, pol)             transfer functions (App. B.4)
cl(tab, DT, DE, ell_max, pol)         C_ell^{TT,TE,EE} (eq. c_ell_def)
solve(...)                            everything above in order
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
import threading

import numpy as np

from . import background
from .background import OracleError, build_tables  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_BUILD = os.path.join(_HERE, "_build")
_LIB = os.path.join(_BUILD, "liboracle.so")
_SRCS = [os.path.join(_HERE, "perturb.c"), os.path.join(_HERE, "spectra.c")]
_lock = threading.Lock()
_lib = None

STATUS_NAMES = {0: "OK", 1: "MAX_STEPS", 2: "NONFINITE", 3: "STEP_UNDERFLOW", 4: "BAD_INPUT"}


def build_c(force: bool = False) -> str:
    """Compile the oracle's C sources with gcc (-O2, OpenMP, no hand SIMD)."""
    os.makedirs(_BUILD, exist_ok=True)
    newest = max(os.path.getmtime(s) for s in _SRCS)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < newest:
        tmp = _LIB + f".tmp{os.getpid()}"
        cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-o", tmp] + _SRCS + ["-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _OTab(ctypes.Structure):
    _fields_ = [
        ("rt_g0", ctypes.c_double), ("rt_ur0", ctypes.c_double), ("rt_c0", ctypes.c_double),
        ("rt_b0", ctypes.c_double), ("rt_L", ctypes.c_double),
        ("pref_ncdm", ctypes.c_double), ("m_over_T", ctypes.c_double),
        ("n_q", ctypes.c_int), ("q", ctypes.c_void_p), ("W", ctypes.c_void_p),
        ("R_nu", ctypes.c_double),
        ("n", ctypes.c_int), ("L0", ctypes.c_double), ("dl", ctypes.c_double),
        ("f_ldk", ctypes.c_void_p), ("M_ldk", ctypes.c_void_p),
        ("f_kap", ctypes.c_void_p), ("M_kap", ctypes.c_void_p),
        ("f_lcs", ctypes.c_void_p), ("M_lcs", ctypes.c_void_p),
        ("f_ltau", ctypes.c_void_p), ("M_ltau", ctypes.c_void_p),
    ]


class _OPrec(ctypes.Structure):
    _fields_ = [
        ("lg", ctypes.c_int), ("lp", ctypes.c_int), ("ln", ctypes.c_int), ("nq", ctypes.c_int), ("lq", ctypes.c_int),
        ("rtol", ctypes.c_double), ("atol", ctypes.c_double), ("max_steps", ctypes.c_int),
        ("pcoeff", ctypes.c_double), ("icoeff", ctypes.c_double), ("dcoeff", ctypes.c_double),
        ("sw", ctypes.c_double), ("isw", ctypes.c_double), ("dop", ctypes.c_double), ("pol", ctypes.c_double),
        ("grav", ctypes.c_double), ("thom", ctypes.c_double),
    ]


def lib():
    global _lib
    with _lock:
        if _lib is None:
            path = build_c()
            L = ctypes.CDLL(path)
            dp = ctypes.POINTER(ctypes.c_double)
            ip = ctypes.POINTER(ctypes.c_int)
            L.oracle_perturb.restype = ctypes.c_int
            L.oracle_perturb.argtypes = [ctypes.POINTER(_OTab), ctypes.POINTER(_OPrec), ctypes.c_double,
                                         ctypes.c_double, ctypes.c_int, dp, dp, dp, dp, ip, ip, dp, ctypes.c_int, dp,
                                         dp, dp, ctypes.c_int]
            L.oracle_perturb_many_hist.restype = ctypes.c_int
            L.oracle_perturb_many_hist.argtypes = [ctypes.POINTER(_OTab), ctypes.POINTER(_OPrec), ctypes.c_int, dp, dp,
                                                   dp, dp, ctypes.c_int, dp, dp, ip, ip, ip, dp, ip, ctypes.c_int,
                                                   ctypes.c_int]
            L.oracle_perturb_many_tangent.restype = ctypes.c_int
            L.oracle_perturb_many_tangent.argtypes = [ctypes.POINTER(_OTab), ctypes.POINTER(_OTab), dp, ctypes.c_int,
                                                      ctypes.c_int, ctypes.POINTER(_OPrec), ctypes.c_int, dp,
                                                      ctypes.c_int, dp, dp, dp, ip, dp, ip, ctypes.c_int]
            L.oracle_rhs.restype = None
            L.oracle_rhs.argtypes = [ctypes.POINTER(_OTab), ctypes.POINTER(_OPrec), ctypes.c_double, ctypes.c_double,
                                     dp, dp]
            L.oracle_rk4.restype = ctypes.c_int
            L.oracle_rk4.argtypes = [ctypes.POINTER(_OTab), ctypes.POINTER(_OPrec), ctypes.c_double, ctypes.c_double,
                                     ctypes.c_int, dp, dp, dp, ctypes.c_double, ctypes.c_double,
                                     ctypes.POINTER(ctypes.c_long)]
            L.oracle_perturb_many.restype = ctypes.c_int
            L.oracle_perturb_many.argtypes = [ctypes.POINTER(_OTab), ctypes.POINTER(_OPrec), ctypes.c_int, dp, dp,
                                              dp, dp, ctypes.c_int, dp, dp, ip, ip, ip]
            L.oracle_perturb_many_dm.restype = ctypes.c_int
            L.oracle_perturb_many_dm.argtypes = [ctypes.POINTER(_OTab), ctypes.POINTER(_OPrec), ctypes.c_int, dp, dp,
                                                 dp, dp, ctypes.c_int, dp, dp, dp, ip, ip, ip]
            L.oracle_delta_m.restype = ctypes.c_double
            L.oracle_delta_m.argtypes = [ctypes.POINTER(_OTab), ctypes.POINTER(_OPrec), ctypes.c_double, dp]
            L.oracle_sources_state.restype = None
            L.oracle_sources_state.argtypes = [ctypes.POINTER(_OTab), ctypes.POINTER(_OPrec), ctypes.c_double,
                                               ctypes.c_double, dp, dp]
            L.oracle_state_size.restype = ctypes.c_int
            L.oracle_state_size.argtypes = [ctypes.POINTER(_OPrec)]
            L.oracle_matter_pk.argtypes = [ctypes.POINTER(_OTab), ctypes.POINTER(_OPrec), ctypes.c_double, dp,
                                           ctypes.c_double, ctypes.c_double, ctypes.c_double]
            L.oracle_matter_pk.restype = ctypes.c_double
            L.oracle_bessel.restype = None
            L.oracle_bessel.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.POINTER(ctypes.c_longdouble)]
            L.oracle_los_adjoint.restype = None
            L.oracle_los_adjoint.argtypes = [ctypes.c_int, dp, ctypes.c_int, dp, dp, dp, dp, ctypes.c_int,
                                             ctypes.c_double, ctypes.c_int, dp]
            L.oracle_los.restype = None
            L.oracle_los.argtypes = [ctypes.c_int, dp, ctypes.c_int, dp, dp, dp, ctypes.c_int, ctypes.c_double,
                                     ctypes.c_int, dp, dp]
            L.oracle_cl.restype = None
            L.oracle_cl.argtypes = [ctypes.c_int, dp, ctypes.c_int, dp, dp, ctypes.c_int, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_double, dp]
            _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


class _Bound:
    """ctypes views of a Tables object, keeping the arrays alive."""

    def __init__(self, t):
        bg = t.bg
        self.keep = []

        def arr(x):
            a = np.ascontiguousarray(x, dtype=np.float64)
            self.keep.append(a)
            return a.ctypes.data

        self.tab = _OTab(
            bg.rt_g0, bg.rt_ur0, bg.rt_c0, bg.rt_b0, bg.rt_L, bg.pref_ncdm, bg.m_over_T,
            len(bg.q), arr(bg.q if len(bg.q) else np.zeros(1)), arr(bg.W if len(bg.W) else np.zeros(1)), bg.R_nu,
            t.n, t.L0, t.dl,
            arr(t.cols["ln_dk"]), arr(t.M["ln_dk"]), arr(t.cols["kappa"]), arr(t.M["kappa"]),
            arr(t.cols["ln_cs2"]), arr(t.M["ln_cs2"]), arr(t.cols["ln_tau"]), arr(t.M["ln_tau"]))


def make_prec(prec: dict, nq: int, rtol: float = 0.0, atol: float = 0.0) -> _OPrec:
    return _OPrec(int(prec["ell_gamma"]), int(prec["ell_pol"]), int(prec["ell_nu"]), int(nq), int(prec["ell_ncdm"]),
                  rtol, atol, int(prec["max_steps"]), prec["pcoeff"], prec["icoeff"], prec["dcoeff"],
                  prec["scale_sw"], prec["scale_isw"], prec["scale_dop"], prec["scale_pol"],
                  prec.get("gravity_scale", 1.0), prec.get("thomson_scale", 1.0))


def tolerances(prec: dict, k: np.ndarray):
    """(rtol, atol) per mode: small-k values below k_split, large-k values
    at and above it (App. A.2, perturbation solver options)."""
    small = k < prec["k_split"]
    rtol = np.where(small, prec["rtol_small"], prec["rtol_large"]).astype(np.float64)
    atol = np.where(small, prec["atol_small"], prec["atol_large"]).astype(np.float64)
    return rtol, atol


def state_size(prec: dict, nq: int) -> int:
    return lib().oracle_state_size(ctypes.byref(make_prec(prec, nq)))


def perturb(t, idx=None, prec_over: dict | None = None):
    """Sources for the modes t.k[idx] (all modes by default).
    Returns (S[n][3][n_tau], status[n], nsteps[n], naccept[n])."""
    prec = dict(t.prec)
    if prec_over:
        prec.update(prec_over)
    idx = np.arange(len(t.k)) if idx is None else np.asarray(idx, dtype=np.int64)
    k = np.ascontiguousarray(t.k[idx], dtype=np.float64)
    lna0 = np.ascontiguousarray(t.lna_i[idx], dtype=np.float64)
    rtol, atol = tolerances(prec, k)
    if prec_over and "rtol" in prec_over:
        rtol[:] = prec_over["rtol"]
        atol[:] = prec_over["atol"]
    n_out = len(t.lna_src)
    S = np.zeros((len(k), 3, n_out))
    st = np.zeros(len(k), dtype=np.int32)
    ns = np.zeros(len(k), dtype=np.int32)
    na = np.zeros(len(k), dtype=np.int32)
    b = _Bound(t)
    p = make_prec(prec, len(t.bg.q))
    lna_out = np.ascontiguousarray(t.lna_src, dtype=np.float64)
    lib().oracle_perturb_many(ctypes.byref(b.tab), ctypes.byref(p), len(k), _dp(k), _dp(lna0), _dp(rtol), _dp(atol),
                              n_out, _dp(lna_out), _dp(S), _ip(st), _ip(ns), _ip(na))
    return S, st, ns, na


def perturb_dm(t, idx=None):
    """As perturb, plus the matter density contrast delta_m[n][n_tau] at the
    output times (App. B.4 eq. PK's species sum; zero before a mode's start).
    Returns (S, Dm, status, nsteps)."""
    idx = np.arange(len(t.k)) if idx is None else np.asarray(idx, dtype=np.int64)
    k = np.ascontiguousarray(t.k[idx], dtype=np.float64)
    lna0 = np.ascontiguousarray(t.lna_i[idx], dtype=np.float64)
    rtol, atol = tolerances(t.prec, k)
    n_out = len(t.lna_src)
    S = np.zeros((len(k), 3, n_out))
    Dm = np.zeros((len(k), n_out))
    st = np.zeros(len(k), dtype=np.int32)
    ns = np.zeros(len(k), dtype=np.int32)
    na = np.zeros(len(k), dtype=np.int32)
    b = _Bound(t)
    p = make_prec(t.prec, len(t.bg.q))
    lna_out = np.ascontiguousarray(t.lna_src, dtype=np.float64)
    lib().oracle_perturb_many_dm(ctypes.byref(b.tab), ctypes.byref(p), len(k), _dp(k), _dp(lna0), _dp(rtol),
                                 _dp(atol), n_out, _dp(lna_out), _dp(S), _dp(Dm), _ip(st), _ip(ns), _ip(na))
    return S, Dm, st, ns


def delta_m_of_state(t, lna: float, y) -> float:
    """delta_m of one state vector at ln a (tests)."""
    b = _Bound(t)
    p = make_prec(t.prec, len(t.bg.q))
    y = np.ascontiguousarray(y, dtype=np.float64)
    return lib().oracle_delta_m(ctypes.byref(b.tab), ctypes.byref(p), float(lna), _dp(y))


def sources_of_state(t, k: float, lna: float, y) -> np.ndarray:
    """S_T0, S_T1, S_T2 (App. B.4) at ln a from a state in the oracle's layout."""
    b = _Bound(t)
    p = make_prec(t.prec, len(t.bg.q))
    y = np.ascontiguousarray(y, dtype=np.float64)
    out = np.zeros(3)
    lib().oracle_sources_state(ctypes.byref(b.tab), ctypes.byref(p), float(k), float(lna), _dp(y), _dp(out))
    return out


def library_row_order(prec: dict, nq: int) -> np.ndarray:
    """For each state row in the order the library documents (photon T chain
    delta_b, theta_b, theta_g, F_2..; polarisation G_0..; neutrinos delta,
    theta, F_2..; massive Psi_0.. per node; then delta_c, eta, delta_g), the
    index of that variable in the oracle's state layout
    (delta_c, delta_b, theta_b, photon delta_g, theta_g, F_2.., G.., nu.., Psi.., eta)."""
    lg, lp, ln, lq = int(prec["ell_gamma"]), int(prec["ell_pol"]), int(prec["ell_nu"]), int(prec["ell_ncdm"])
    g0 = 3
    p0 = g0 + lg + 1
    n0 = p0 + (lp + 1 if lp > 0 else 0)
    m0 = n0 + ln + 1
    eta = m0 + nq * (lq + 1)
    rows = [1, 2, g0 + 1] + [g0 + l for l in range(2, lg + 1)]
    if lp > 0:
        rows += [p0 + l for l in range(lp + 1)]
    rows += [n0 + l for l in range(ln + 1)]
    for i in range(nq):
        rows += [m0 + i * (lq + 1) + l for l in range(lq + 1)]
    rows += [0, eta, g0]
    return np.array(rows)


def sources_adjoint(t, gS: np.ndarray, points=None) -> np.ndarray:
    """dL/dy [n_k][n_tau][rows] from dL/dS [n_k][3][n_tau], rows in the
    library's documented order, zero before each mode's start.  At a fixed time
    the sources are linear in the state with no constant term, so column i of
    dS/dy is S(e_i) for the unit vector e_i: this is the transpose of that map
    by its definition, from the oracle's own source function.  With points, a
    list of (k index, time index), only those entries are filled."""
    nq = len(t.bg.q)
    N = state_size(t.prec, nq)
    order = library_row_order(t.prec, nq)
    lna_out = np.asarray(t.lna_src)
    out = np.zeros((len(t.k), len(lna_out), N))
    b = _Bound(t)
    p = make_prec(t.prec, nq)
    e = np.zeros(N)
    col = np.zeros(3)
    cols = np.zeros((N, 3))
    pts = points if points is not None else [(ik, j) for ik in range(len(t.k)) for j in range(len(lna_out))]
    for ik, j in pts:
        k, lna = t.k[ik], lna_out[j]
        if lna < t.lna_i[ik]:
            continue
        for i in range(N):
            e[:] = 0.0
            e[i] = 1.0
            lib().oracle_sources_state(ctypes.byref(b.tab), ctypes.byref(p), float(k), float(lna), _dp(e), _dp(col))
            cols[i] = col
        g = cols @ gS[ik, :, j]
        out[ik, j] = g[order]
    return out


def perturb_hist(t, hist=None, hist_n=None):
    """All modes, recording each mode's accepted-step history (hist[n_k][cap]:
    the start, then every accepted step size; counts hist_n), or, given
    hist/hist_n, replaying them without error control.
    Returns (S, status, nsteps, hist, hist_n)."""
    k = np.ascontiguousarray(t.k, dtype=np.float64)
    lna0 = np.ascontiguousarray(t.lna_i, dtype=np.float64)
    rtol, atol = tolerances(t.prec, k)
    n_out = len(t.lna_src)
    cap = int(t.prec["max_steps"]) + 1
    replay = hist is not None
    if not replay:
        hist = np.zeros((len(k), cap))
        hist_n = np.zeros(len(k), dtype=np.int32)
    else:
        hist = np.ascontiguousarray(hist, dtype=np.float64)
        hist_n = np.ascontiguousarray(hist_n, dtype=np.int32)
        cap = hist.shape[1]
    S = np.zeros((len(k), 3, n_out))
    st = np.zeros(len(k), dtype=np.int32)
    ns = np.zeros(len(k), dtype=np.int32)
    na = np.zeros(len(k), dtype=np.int32)
    b = _Bound(t)
    p = make_prec(t.prec, len(t.bg.q))
    lna_out = np.ascontiguousarray(t.lna_src, dtype=np.float64)
    lib().oracle_perturb_many_hist(ctypes.byref(b.tab), ctypes.byref(p), len(k), _dp(k), _dp(lna0), _dp(rtol),
                                   _dp(atol), n_out, _dp(lna_out), _dp(S), _ip(st), _ip(ns), _ip(na), _dp(hist),
                                   _ip(hist_n), cap, 1 if replay else 0)
    return S, st, ns, hist, hist_n


JAC_PARAMS = ("h", "omega_b", "omega_cdm", "tau_reio")


def cl_dns(k, DT, DE, ell_max: int, pol: bool, A_s: float, n_s: float, k_pivot: float = 0.05):
    """dC_l/dn_s: the k quadrature of cl with P(k) ln(k/k_pivot) in place of
    P(k) (C_l depends on n_s only through the primordial spectrum)."""
    k = np.asarray(k, dtype=np.float64)
    kl = np.concatenate(([k[0]], k[:-1]))
    kr = np.concatenate((k[1:], [k[-1]]))
    f = 0.5 * (kr - kl) * A_s * (k / k_pivot) ** (n_s - 1.0) * np.log(k / k_pivot) / k
    out = np.zeros((3, ell_max + 1))
    out[0, 2:] = 4 * math.pi * (DT * DT) @ f
    if pol:
        out[1, 2:] = 4 * math.pi * (DT * DE) @ f
        out[2, 2:] = 4 * math.pi * (DE * DE) @ f
    return out


def jacobian(cosmo: dict, prec: dict, k, n_tau: int, ell_max: int, pol: bool, rel: float = 1e-4, order: int = 4):
    """dC_l/dtheta [6][3][ell_max+1] for theta = (h, omega_b, omega_cdm, ln A_s,
    n_s, tau_reio).  For h, omega_b, omega_cdm and tau_reio: finite
    differences at steps of rel (relative), every perturbed cosmology replaying
    the base cosmology's accepted steps (the derivative of the frozen-step
    discrete map); order 2 is the central difference (f(+e) - f(-e))/(2e),
    order 4 the five-point (8 (f(+e) - f(-e)) - (f(+2e) - f(-2e)))/(12 e).
    For ln A_s C_l itself, for n_s the primordial-weight quadrature cl_dns.
    Returns (C_l, J, status of the base run)."""
    if order not in (2, 4):
        raise ValueError("order must be 2 or 4")
    t = build_tables(cosmo, prec, k, n_tau)
    S, st, ns, hist, hn = perturb_hist(t)
    DT, DE = los(t, S, ell_max, pol)
    C = cl(t.k, DT, DE, ell_max, pol, cosmo["A_s"], cosmo["n_s"], prec["k_pivot"])
    J = np.zeros((6, 3, ell_max + 1))
    slot = {"h": 0, "omega_b": 1, "omega_cdm": 2, "tau_reio": 5}

    def at(name, mult):
        c2 = dict(cosmo)
        c2[name] = cosmo[name] * (1.0 + mult * rel)
        t2 = build_tables(c2, prec, k, n_tau)
        S2 = perturb_hist(t2, hist, hn)[0]
        D2T, D2E = los(t2, S2, ell_max, pol)
        return cl(t2.k, D2T, D2E, ell_max, pol, c2["A_s"], c2["n_s"], prec["k_pivot"])

    for name in JAC_PARAMS:
        e = rel * cosmo[name]
        d1 = at(name, 1.0) - at(name, -1.0)
        if order == 2:
            J[slot[name]] = d1 / (2.0 * e)
        else:
            d2 = at(name, 2.0) - at(name, -2.0)
            J[slot[name]] = (8.0 * d1 - d2) / (12.0 * e)
    J[3] = C
    J[4] = cl_dns(t.k, DT, DE, ell_max, pol, cosmo["A_s"], cosmo["n_s"], prec["k_pivot"])
    return C, J, st


def perturb_tangent(t, tabs, eps, hist, hist_n, order: int = 4):
    """Forward-mode tangents of the sources along the given step histories
    (oracle_perturb_tangent): tabs[d] are the tables at theta_d + eps[d],
    - eps[d] and, for order 4, + 2 eps[d], - 2 eps[d].
    Returns (S[n_k][3][n_tau], Sd[n_k][nd][3][n_tau], status[n_k])."""
    nd = len(tabs)
    k = np.ascontiguousarray(t.k, dtype=np.float64)
    n_out = len(t.lna_src)
    hist = np.ascontiguousarray(hist, dtype=np.float64)
    hist_n = np.ascontiguousarray(hist_n, dtype=np.int32)
    S = np.zeros((len(k), 3, n_out))
    Sd = np.zeros((len(k), nd, 3, n_out))
    st = np.zeros(len(k), dtype=np.int32)
    b = _Bound(t)
    bound = [[_Bound(x) for x in row] + [_Bound(row[0])] * (4 - len(row)) for row in tabs]
    tt = (_OTab * (4 * nd))(*[x.tab for row in bound for x in row])
    e = np.ascontiguousarray(eps, dtype=np.float64)
    p = make_prec(t.prec, len(t.bg.q))
    lna_out = np.ascontiguousarray(t.lna_src, dtype=np.float64)
    lib().oracle_perturb_many_tangent(ctypes.byref(b.tab), tt, _dp(e), nd, order, ctypes.byref(p), len(k), _dp(k),
                                      n_out, _dp(lna_out), _dp(S), _dp(Sd), _ip(st), _dp(hist), _ip(hist_n),
                                      hist.shape[1])
    return S, Sd, st


def cl_tangent(k, DT, DE, dDT, dDE, ell_max: int, pol: bool, A_s: float, n_s: float, k_pivot: float = 0.05):
    """Derivative of cl along (dDT, dDE) [l-2][k] (the quadrature is bilinear
    in the transfer functions): Cdot_XY = sum_k 4 pi w_k P(k)/k
    (dDelta_X Delta_Y + Delta_X dDelta_Y).  Returns [3][ell_max+1]."""
    k = np.asarray(k, dtype=np.float64)
    kl = np.concatenate(([k[0]], k[:-1]))
    kr = np.concatenate((k[1:], [k[-1]]))
    f = 4 * math.pi * 0.5 * (kr - kl) * A_s * (k / k_pivot) ** (n_s - 1.0) / k
    C = np.zeros((3, ell_max + 1))
    C[0, 2:] = np.sum(f * 2.0 * DT * dDT, axis=1)
    if pol:
        C[1, 2:] = np.sum(f * (dDT * DE + DT * dDE), axis=1)
        C[2, 2:] = np.sum(f * 2.0 * DE * dDE, axis=1)
    return C


def jacobian_tangent(cosmo: dict, prec: dict, k, n_tau: int, ell_max: int, pol: bool, rel: float = 1e-4,
                     order: int = 4):
    """dC_l/dtheta [6][3][ell_max+1] by forward mode (section 3; the paper's
    default derivative option): the tangents of the frozen-step discrete map
    (perturb_tangent) with the tables' own dependence on h, omega_b,
    omega_cdm and tau_reio taken as differences (central for order 2,
    five-point for order 4) of table-dependent quantities between the tables
    at theta (1 + m rel), m = +-1 (and +-2); then the projection's tangent,
    los(tables, Sdot) plus the same difference of los at fixed sources, and
    the quadrature's (cl_tangent).  ln A_s and n_s as in jacobian.
    Returns (C_l, J, status of the base run)."""
    if order not in (2, 4):
        raise ValueError("order must be 2 or 4")
    t = build_tables(cosmo, prec, k, n_tau)
    S0, st, ns, hist, hn = perturb_hist(t)
    mults = (1.0, -1.0, 2.0, -2.0)[: 2 if order == 2 else 4]
    tabs, eps = [], []
    for name in JAC_PARAMS:
        row = []
        for mult in mults:
            c2 = dict(cosmo)
            c2[name] = cosmo[name] * (1.0 + mult * rel)
            row.append(build_tables(c2, prec, k, n_tau))
        tabs.append(row)
        eps.append(rel * cosmo[name])
    S, Sd, st2 = perturb_tangent(t, tabs, eps, hist, hn, order)
    DT, DE = los(t, S, ell_max, pol)
    C = cl(t.k, DT, DE, ell_max, pol, cosmo["A_s"], cosmo["n_s"], prec["k_pivot"])
    J = np.zeros((6, 3, ell_max + 1))
    slot = {"h": 0, "omega_b": 1, "omega_cdm": 2, "tau_reio": 5}

    def diff(vals, e):
        if order == 2:
            return (vals[0] - vals[1]) / (2.0 * e)
        return (8.0 * (vals[0] - vals[1]) - (vals[2] - vals[3])) / (12.0 * e)

    for d, name in enumerate(JAC_PARAMS):
        dT, dE = los(t, Sd[:, d], ell_max, pol)
        at = [los(x, S, ell_max, pol) for x in tabs[d]]
        dT = dT + diff([a[0] for a in at], eps[d])
        dE = dE + diff([a[1] for a in at], eps[d])
        J[slot[name]] = cl_tangent(t.k, DT, DE, dT, dE, ell_max, pol, cosmo["A_s"], cosmo["n_s"], prec["k_pivot"])
    J[3] = C
    J[4] = cl_dns(t.k, DT, DE, ell_max, pol, cosmo["A_s"], cosmo["n_s"], prec["k_pivot"])
    st = np.where(st != 0, st, st2)
    return C, J, st


def perturb_one(t, k: float, lna0: float, lna_out, prec_over: dict | None = None, y0=None, want_y: bool = False,
                rtol: float | None = None, atol: float | None = None, acc_cap: int = 0, want_diag: bool = False,
                fixed=None):
    """One mode with full control (tests): custom start, output times,
    initial state, tolerances; optionally the dense-output states and the
    accepted step sequence.  fixed = [start, h_1, h_2, ...] replays those
    steps without error control (the start overrides lna0)."""
    prec = dict(t.prec)
    if prec_over:
        prec.update(prec_over)
    if rtol is None:
        r, a = tolerances(prec, np.array([k]))
        rtol, atol = float(r[0]), float(a[0])
    p = make_prec(prec, len(t.bg.q), rtol, atol)
    N = lib().oracle_state_size(ctypes.byref(p))
    lna_out = np.ascontiguousarray(lna_out, dtype=np.float64)
    n_out = len(lna_out)
    S = np.zeros((3, n_out))
    Y = np.zeros((n_out, N)) if want_y else None
    y0a = None if y0 is None else np.ascontiguousarray(y0, dtype=np.float64)
    acc = np.zeros(max(acc_cap, 1))
    ns = ctypes.c_int(0)
    na = ctypes.c_int(0)
    D = np.zeros((n_out, 4))
    fx = None if fixed is None else np.ascontiguousarray(fixed, dtype=np.float64)
    b = _Bound(t)
    st = lib().oracle_perturb(ctypes.byref(b.tab), ctypes.byref(p), float(k), float(lna0), n_out, _dp(lna_out), _dp(S),
                              _dp(Y) if want_y else None, _dp(y0a) if y0a is not None else None, ctypes.byref(ns),
                              ctypes.byref(na), _dp(acc) if acc_cap else None, acc_cap, _dp(D) if want_diag else None,
                              None, _dp(fx) if fx is not None else None, 0 if fx is None else len(fx) - 1)
    out = {"S": S, "status": st, "nsteps": ns.value, "naccept": na.value, "N": N}
    if want_diag:
        out["diag"] = D  # h', eta', alpha, alpha' per output time
    if want_y:
        out["y"] = Y
    if acc_cap:
        out["accepted_lna"] = acc[: min(na.value, acc_cap)]
    return out


def matter_pk(t, idx=None):
    """Linear matter power spectrum today (App. B.4, eq. PK) [Mpc^3] for the
    modes idx (default all): each mode integrated to a = 1 by the oracle's
    ESDIRK (one output time, ln a = 0), then 2 pi^2/k^3 P_R(k) delta_m^2 with
    delta_m over CDM, baryons and massive neutrinos.  NaN where a mode did not
    finish."""
    idx = np.arange(len(t.k)) if idx is None else np.asarray(idx)
    out = np.full(len(idx), np.nan)
    prec = dict(t.prec)
    c = t.cosmo
    for n, i in enumerate(idx):
        r = perturb_one(t, float(t.k[i]), float(t.lna_i[i]), [0.0], want_y=True)
        if r["status"] != 0:
            continue
        rt, at = tolerances(prec, np.array([t.k[i]]))
        p = make_prec(prec, len(t.bg.q), float(rt[0]), float(at[0]))
        b = _Bound(t)
        y = np.ascontiguousarray(r["y"][-1])
        out[n] = lib().oracle_matter_pk(ctypes.byref(b.tab), ctypes.byref(p), float(t.k[i]), _dp(y), float(c["A_s"]),
                                        float(c["n_s"]), float(prec["k_pivot"]))
    return out


def rk4_one(t, k: float, lna0: float, lna_out, h_max: float = 1e-3, c_stab: float = 0.5, want_y: bool = False,
            prec_over: dict | None = None):
    """Brute-force classical RK4 on the same right-hand side (tests)."""
    prec = dict(t.prec)
    if prec_over:
        prec.update(prec_over)
    p = make_prec(prec, len(t.bg.q), 0.0, 0.0)
    N = lib().oracle_state_size(ctypes.byref(p))
    lna_out = np.ascontiguousarray(lna_out, dtype=np.float64)
    S = np.zeros((3, len(lna_out)))
    Y = np.zeros((len(lna_out), N)) if want_y else None
    ns = ctypes.c_long(0)
    b = _Bound(t)
    lib().oracle_rk4(ctypes.byref(b.tab), ctypes.byref(p), float(k), float(lna0), len(lna_out), _dp(lna_out), _dp(S),
                     _dp(Y) if want_y else None, h_max, c_stab, ctypes.byref(ns))
    out = {"S": S, "nsteps": ns.value}
    if want_y:
        out["y"] = Y
    return out


def rhs(t, k: float, lna: float, y, prec_over: dict | None = None):
    prec = dict(t.prec)
    if prec_over:
        prec.update(prec_over)
    p = make_prec(prec, len(t.bg.q), 0.0, 0.0)
    y = np.ascontiguousarray(y, dtype=np.float64)
    dy = np.zeros_like(y)
    b = _Bound(t)
    lib().oracle_rhs(ctypes.byref(b.tab), ctypes.byref(p), float(k), float(lna), _dp(y), _dp(dy))
    return dy


def bessel(L: int, x: float) -> np.ndarray:
    """j_0..j_L at x, computed in long double, returned as float64."""
    buf = (ctypes.c_longdouble * (L + 1))()
    lib().oracle_bessel(L, float(x), buf)
    return np.array([float(v) for v in buf])


def los(t, S: np.ndarray, ell_max: int, pol: bool, k=None, chi=None, w=None, s_pol: float | None = None):
    """Transfer functions Delta_T, Delta_E [ell-2][k] for 2 <= ell <= ell_max."""
    k = np.ascontiguousarray(t.k if k is None else k, dtype=np.float64)
    chi = np.ascontiguousarray(t.chi_src if chi is None else chi, dtype=np.float64)
    w = np.ascontiguousarray(t.w_src if w is None else w, dtype=np.float64)
    S = np.ascontiguousarray(S, dtype=np.float64)
    nl = ell_max - 1
    DT = np.zeros((nl, len(k)))
    DE = np.zeros((nl, len(k)))
    sp = t.prec["scale_pol"] if s_pol is None else s_pol
    lib().oracle_los(len(k), _dp(k), len(chi), _dp(chi), _dp(w), _dp(S), ell_max, sp, 1 if pol else 0, _dp(DT),
                     _dp(DE))
    return DT, DE


def cl_adjoint(k, DT, DE, gC, ell_max: int, pol: bool, A_s: float, n_s: float, k_pivot: float = 0.05):
    """Transpose of cl: given gC[3][ell_max+1] = dL/dC_l (TT, TE, EE), the
    gradients dL/dDelta_T and dL/dDelta_E [l-2][k]:
      G_T = 4 pi w_k P(k)/k (2 gTT Delta_T + gTE Delta_E),
      G_E = 4 pi w_k P(k)/k (gTE Delta_T + 2 gEE Delta_E)."""
    k = np.asarray(k, dtype=np.float64)
    kl = np.concatenate(([k[0]], k[:-1]))
    kr = np.concatenate((k[1:], [k[-1]]))
    f = 4 * math.pi * 0.5 * (kr - kl) * A_s * (k / k_pivot) ** (n_s - 1.0) / k
    g = np.asarray(gC)[:, 2:ell_max + 1][:, :, None]
    GT = f * (2 * g[0] * DT + (g[1] * DE if pol else 0.0))
    GE = f * (g[1] * DT + 2 * g[2] * DE) if pol else np.zeros_like(DT)
    return GT, GE


def los_adjoint(t, GT, GE, ell_max: int, pol: bool, k=None, s_pol: float | None = None):
    """Transpose of los: dL/dS [k][3][n_tau] from dL/dDelta_T, dL/dDelta_E."""
    k = np.ascontiguousarray(t.k if k is None else k, dtype=np.float64)
    chi = np.ascontiguousarray(t.chi_src, dtype=np.float64)
    w = np.ascontiguousarray(t.w_src, dtype=np.float64)
    gS = np.zeros((len(k), 3, len(chi)))
    sp = t.prec["scale_pol"] if s_pol is None else s_pol
    lib().oracle_los_adjoint(len(k), _dp(k), len(chi), _dp(chi), _dp(w), _dp(np.ascontiguousarray(GT)),
                             _dp(np.ascontiguousarray(GE)), ell_max, sp, 1 if pol else 0, _dp(gS))
    return gS


def cl(k, DT, DE, ell_max: int, pol: bool, A_s: float, n_s: float, k_pivot: float = 0.05):
    """C_ell[3][ell_max+1] (TT, TE, EE), zero for ell < 2."""
    k = np.ascontiguousarray(k, dtype=np.float64)
    Cl = np.zeros((3, ell_max + 1))
    DT = np.ascontiguousarray(DT)
    DE = np.ascontiguousarray(DE)
    lib().oracle_cl(len(k), _dp(k), ell_max, _dp(DT), _dp(DE), 1 if pol else 0, A_s, n_s, k_pivot, _dp(Cl))
    return Cl


def transfer_kgrid(ell_max: int, k_lo: float, k_hi: float) -> np.ndarray:
    """Transfer k-grid (App. A.2, eq. k_transfer_spacing, with eq. defkperiod
    and the k_min / k_max_cmb rules): steps k -> k + k_period linstep k /
    (k + linstep/logstep) from max(k_min_tau0/tau0_fid, k_lo) while below
    min(k_max_tau0_over_l_max ell_max/tau0_fid, k_hi), then that upper end.
    Constants are the App. A.2 defaults."""
    tau0_fid, tau_rec_fid = 1.418668e4, 281.040565
    linstep, logstep = 0.45, 170.0
    kmin = max(0.1 / tau0_fid, k_lo)
    kmax = min(1.8 * ell_max / tau0_fid, k_hi)
    kperiod = 2.0 * math.pi / (tau0_fid - tau_rec_fid)
    out = []
    k = kmin
    while k < kmax:
        out.append(k)
        k = k + kperiod * linstep * k / (k + linstep / logstep)
    out.append(kmax)
    return np.array(out)


def interp_sources(k, S: np.ndarray, kt) -> np.ndarray:
    """Sources S[k][3][n_tau] interpolated onto kt by natural cubic splines in k
    at every (type, output time) (scipy's CubicSpline with natural ends)."""
    from scipy.interpolate import CubicSpline
    sp = CubicSpline(np.asarray(k, dtype=np.float64), S, axis=0, bc_type="natural")
    return sp(np.asarray(kt, dtype=np.float64))


def spectra_on_grid(t, S: np.ndarray, kt, ell_max: int, pol: bool):
    """C_ell on the transfer grid kt: interpolated sources, projection and k
    quadrature there."""
    St = interp_sources(t.k, S, kt)
    DT, DE = los(t, St, ell_max, pol, k=kt)
    C = cl(kt, DT, DE, ell_max, pol, t.cosmo["A_s"], t.cosmo["n_s"], t.prec["k_pivot"])
    return {"St": St, "DT": DT, "DE": DE, "Cl": C}


def solve(cosmo: dict, prec: dict, k, n_tau: int, ell_max: int, pol: bool, tables=None):
    """The whole path for one cosmology: tables, sources, transfers, C_ell."""
    t = build_tables(cosmo, prec, np.asarray(k, dtype=np.float64), n_tau) if tables is None else tables
    S, st, ns, na = perturb(t)
    DT, DE = los(t, S, ell_max, pol)
    C = cl(t.k, DT, DE, ell_max, pol, cosmo["A_s"], cosmo["n_s"], prec["k_pivot"])
    return {"tables": t, "S": S, "status": st, "nsteps": ns, "naccept": na, "DT": DT, "DE": DE, "Cl": C}
