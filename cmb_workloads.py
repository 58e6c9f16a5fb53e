"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module only generates *inputs*: cosmological parameter sets, wavenumber
grids, output-time counts and multipole ranges.  It holds none of the
solver's arithmetic (no background, recombination, perturbation, Bessel or
quadrature code), so both the CPU oracle and the HIP library may consume what
it produces without sharing any of the method.

Workloads follow the sizes of the paper's benchmark (lensing off, unlensed
TT/TE/EE to ell = 2500; Sec. 4 and App. A.2 of arXiv 2602.15104) and the
parameter box of its validation table (Tab. test_params).
"""
from __future__ import annotations

import copy
import math
from dataclasses import dataclass, field

import numpy as np

# Fiducial LambdaCDM point used by every workload (h, omega_b, omega_cdm, A_s,
# n_s, tau_reio), with the paper's defaults for everything else (App. A.2).
FIDUCIAL = {
    "h": 0.674,
    "omega_b": 0.0224,
    "omega_cdm": 0.120,
    "A_s": 2.1e-9,
    "n_s": 0.965,
    "tau_reio": 0.054,
    "z_reio": float("nan"),
    "Delta_z_reio": 0.5,
    "z_reio_He": 3.5,
    "Delta_z_reio_He": 0.5,
    "exp_reio": 1.5,
    "YHe": 0.245,
    "TCMB0": 2.34865418e-4,
    "Neff": float("nan"),
    "N_nu_massless": float("nan"),
    "T_nu_massless": 0.71636856,
    "N_nu_massive": 0.0,
    "m_nu_massive": 0.06,
    "T_nu_massive": 0.71611,
}

# The six parameters that are varied (serving draws, gradients).
VARIED = ("h", "omega_b", "omega_cdm", "A_s", "n_s", "tau_reio")

# Uniform validation box of the paper (Tab. test_params): six parameters.
VALIDATION_BOX = {
    "h": (0.6, 0.8),
    "omega_b": (0.02162, 0.02312),
    "omega_cdm": (0.114, 0.126),
    "A_s": (1.931e-9, 2.256e-9),
    "n_s": (0.9439, 0.9859),
    "tau_reio": (0.0179, 0.0909),
}

# Paper defaults for the precision / static options (App. A.2), with the
# hierarchy cut-offs of each workload filled in below.
PREC_DEFAULT = {
    "ell_gamma": 12,
    "ell_pol": 10,
    "ell_nu": 17,
    "n_q": 0,
    "ell_ncdm": 17,
    "rtol_small": 1e-5,
    "rtol_large": 1e-4,
    "atol_small": 1e-10,
    "atol_large": 1e-6,
    "k_split": 1e-2,
    "max_steps": 2048,
    "R_tc": 1.5e-3,
    "R_large": 7e-2,
    "k_pivot": 0.05,
    "pcoeff": 0.25,
    "icoeff": 0.8,
    "dcoeff": 0.0,
    "scale_sw": 1.0,
    "scale_isw": 1.0,
    "scale_dop": 1.0,
    "scale_pol": 1.0,
    "gravity_scale": 1.0,
    "thomson_scale": 1.0,
    "n_tab": 8192,
}

K_TRANSITION = 0.45 / 170.0  # Mpc^-1, log->linear transition of the step law


def log_grid(k_min: float, k_max: float, n: int) -> np.ndarray:
    """n points spaced uniformly in log k, both ends included (n = 1: k_min
    alone)."""
    if n == 1:
        return np.array([float(k_min)])
    i = np.arange(n, dtype=np.float64)
    return k_min * (k_max / k_min) ** (i / (n - 1))


def step_law_grid(k_min: float, k_max: float, n: int, k_t: float = K_TRANSITION) -> np.ndarray:
    """k_{j+1} = k_j + c k_j/(k_j + k_t), with c chosen by bisection so that
    exactly n points span [k_min, k_max] (logarithmic below k_t, linear above;
    the transfer-grid law of App. A.2, eq. k_transfer_spacing)."""

    def last(c):
        k = k_min
        for _ in range(n - 1):
            k = k + c * k / (k + k_t)
        return k

    lo, hi = 0.0, 1.0
    while last(hi) < k_max:
        hi *= 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if last(mid) < k_max:
            lo = mid
        else:
            hi = mid
    c = 0.5 * (lo + hi)
    ks = np.empty(n)
    ks[0] = k_min
    for j in range(1, n):
        ks[j] = ks[j - 1] + c * ks[j - 1] / (ks[j - 1] + k_t)
    ks[-1] = k_max
    return ks


@dataclass
class Workload:
    name: str
    cosmo: dict
    prec: dict
    k: np.ndarray
    n_tau: int
    ell_max: int
    polarization: bool
    description: str = ""
    extra: dict = field(default_factory=dict)


def fiducial() -> dict:
    return copy.deepcopy(FIDUCIAL)


def prec_for(ell_gamma: int, ell_pol: int, ell_nu: int, n_q: int = 0, ell_ncdm: int = 17, **over) -> dict:
    p = copy.deepcopy(PREC_DEFAULT)
    p.update(ell_gamma=ell_gamma, ell_pol=ell_pol, ell_nu=ell_nu, n_q=n_q, ell_ncdm=ell_ncdm)
    p.update(over)
    return p


def config0() -> Workload:
    """Temperature only, no polarisation hierarchy, massless neutrinos,
    hierarchies cut at ell = 12; 64 log-spaced k in [1e-4, 0.1]; 400 output
    times; C_ell^TT for 2 <= ell <= 500."""
    c = fiducial()
    c["N_nu_massless"] = 3.0
    return Workload("config0_tt_l500", c, prec_for(12, 0, 12), log_grid(1e-4, 0.1, 64), 400, 500, False,
                    "TT, lmax_g=lmax_nu=12, no pol, 64 k log 1e-4..0.1, 400 tau, ell<=500")


def config1() -> Workload:
    """Full TT/TE/EE: photon T+P and massless-neutrino hierarchies cut at
    ell = 24; 400 k on the log/linear step law over [1e-5, 0.5]; 2000 output
    times; 2 <= ell <= 2500."""
    c = fiducial()
    c["N_nu_massless"] = 3.0
    return Workload("config1_ttteee_l2500", c, prec_for(24, 24, 24, max_steps=4096), step_law_grid(1e-5, 0.5, 400), 2000, 2500, True,
                    "TT/TE/EE, lmax_g=lmax_pol=lmax_nu=24, 400 k step-law 1e-5..0.5, 2000 tau, ell<=2500")


def config2() -> Workload:
    """Config 1 plus one massive neutrino (0.06 eV), N_eff = 3.044 in total,
    12 momentum bins x ell <= 17; 600 k up to 0.5."""
    c = fiducial()
    c["Neff"] = 3.044
    c["N_nu_massive"] = 1.0
    c["m_nu_massive"] = 0.06
    return Workload("config2_mnu_l2500", c, prec_for(24, 24, 24, n_q=12, ell_ncdm=17, max_steps=4096), step_law_grid(1e-5, 0.5, 600),
                    2000, 2500, True, "config1 + 1 massive nu 0.06 eV, 12 q x ell<=17, 600 k, 2000 tau")


def tight(wl: Workload, rtol: float = 1e-10, max_steps: int = 400000) -> Workload:
    """The same workload at a much tighter tolerance: rtol for both k ranges,
    each atol scaled by the same factor as its rtol (so atol/rtol keeps the
    paper's ratio), and room for the many more steps."""
    w = copy.deepcopy(wl)
    p = w.prec
    p["atol_small"] = p["atol_small"] * rtol / p["rtol_small"]
    p["atol_large"] = p["atol_large"] * rtol / p["rtol_large"]
    p["rtol_small"] = p["rtol_large"] = rtol
    p["max_steps"] = max_steps
    w.name = wl.name + f"_rtol{rtol:g}"
    return w


# config-1 modes of the tight-tolerance cross-check (spread over the grid,
# both tolerance ranges, the largest k included)
CONFIG1_SUBSET = (0, 50, 100, 150, 200, 250, 300, 399)


def config1_subset(idx=CONFIG1_SUBSET) -> Workload:
    """Config 1 physics on a subset of its k grid."""
    w = config1()
    w.k = np.ascontiguousarray(w.k[list(idx)])
    w.name = w.name + f"_subset{len(idx)}"
    return w


def small_case(n_k: int = 12, n_tau: int = 120, ell_max: int = 60, polarization: bool = True,
               k_min: float = 1e-4, k_max: float = 0.05, ell_g: int = 8) -> Workload:
    """A tiny workload the oracle finishes in seconds, spanning several
    64-wide tiles when batched and a ragged tail."""
    c = fiducial()
    c["N_nu_massless"] = 3.0
    return Workload(f"small_{n_k}k_{n_tau}t_l{ell_max}", c, prec_for(ell_g, ell_g if polarization else 0, ell_g),
                    log_grid(k_min, k_max, n_k), n_tau, ell_max, polarization)


def perturbed_cosmologies(n: int, seed: int, rel_sigma: float = 0.05, base: dict | None = None) -> list[dict]:
    """n cosmologies with each of the six varied parameters drawn independently
    from N(theta0, (rel_sigma*theta0)^2) (PCG64, seeded)."""
    base = fiducial() if base is None else base
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(n):
        c = copy.deepcopy(base)
        for p in VARIED:
            c[p] = float(base[p] * (1.0 + rel_sigma * rng.standard_normal()))
        out.append(c)
    return out


def box_cosmologies(n: int, seed: int) -> list[dict]:
    """n cosmologies uniform over the paper's validation box."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(n):
        c = fiducial()
        c["N_nu_massless"] = 3.0
        for p, (lo, hi) in VALIDATION_BOX.items():
            c[p] = float(lo + (hi - lo) * rng.random())
        out.append(c)
    return out


def serving_requests(n: int = 512, rate_hz: float = 50.0, seed: int = 20260215):
    """Poisson arrivals of cosmologies around the fiducial (5% sigma on each of
    the six parameters) with ell_max uniform in {500, 1000, 2500} and matching
    k counts {100, 250, 400} on [1e-5, 0.5 ell_max/2500]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / rate_hz, size=n)
    t = np.cumsum(gaps)
    choices = [(500, 100), (1000, 250), (2500, 400)]
    reqs = []
    for i in range(n):
        c = fiducial()
        c["N_nu_massless"] = 3.0
        for p in VARIED:
            c[p] = float(FIDUCIAL[p] * (1.0 + 0.05 * rng.standard_normal()))
        lmax, nk = choices[int(rng.integers(0, 3))]
        reqs.append({"arrival_s": float(t[i]), "cosmo": c, "ell_max": lmax, "n_k": nk,
                     "k": step_law_grid(1e-5, 0.5 * lmax / 2500.0, nk)})
    return reqs


def is_nan(x) -> bool:
    return isinstance(x, float) and math.isnan(x)
