"""CPU oracle, part 1: background, recombination and thermodynamics tables.

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain reference against
which the HIP library is checked.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import it; the library never does.

Everything here is plain Python floats (IEEE double) in the order the paper
states the physics, written for a reader to check against arXiv 2602.15104:

* derived parameters and closed-form species densities (App. A.2 derived
  parameters; App. C species background; Sec. 2.4 neutrino parameters and
  eq. Neffdef);
* helium by Saha in its two stages (App. B.1, helium recombination), hydrogen
  by Saha until the ionised fraction drops below 0.99 and then by the Peebles
  three-level atom (App. B.1 names the TLA as the model it uses at late times;
  we use it for all of hydrogen recombination, since the effective-rate tables
  the paper relies on are not available), matter temperature quasi-static
  above z = 700 and by the App. B.1 ODE below;
* tanh reionisation (App. B.2, eqs. h_reion, y_reio, he_reion) and the
  optical depth tau_reion (App. A.2, eq. tau_reion) with the root find for
  z_reion;
* Thomson rate, optical depth kappa, visibility, baryon sound speed
  (App. B.4 below eq. source_functions; App. C baryons);
* start time a_i(k) from R_tc and R_large (App. A.2, eqs. k_start_small and
  k_start_large);
* the output-time grid and line-of-sight trapezoid weights in ln a
  (App. B.6: trapezoid over ln a).

Fixed discretisation (the same on both sides of the parity check, each written
independently): a uniform ln a grid of n_tab intervals from
ln(min_k a_i) - 1/2 to 0; classical RK4 on that grid for the recombination
ODEs; Simpson per interval for conformal time; trapezoid for kappa; natural
cubic splines for ln(1/tau_c), kappa, ln c_s^2 and ln tau.
"""
from __future__ import annotations

import math

import numpy as np

# ---------------------------------------------------------------------------
# Physical constants (CODATA 2018 / AME 2016).  Units: eV, cm, s, Mpc.
# ---------------------------------------------------------------------------
C_M_S = 299792458.0                 # speed of light [m/s]
G_SI = 6.67430e-11                  # Newton's constant [m^3 kg^-1 s^-2]
HBARC_EV_CM = 1.973269804e-5        # hbar*c [eV cm]
EV_J = 1.602176634e-19              # [J]
MPC_M = 3.0856775814913673e22       # [m]
MPC_CM = MPC_M * 100.0
SIGMA_T_CM2 = 6.6524587321e-25      # Thomson cross section [cm^2]
ME_EV = 0.51099895000e6             # electron mass [eV]
AMU_EV = 931.49410242e6             # atomic mass unit [eV]
MH_EV = 1.00782503223 * AMU_EV      # hydrogen atom mass [eV]
MHE_EV = 4.00260325413 * AMU_EV     # helium-4 atom mass [eV]
E_H_EV = 13.598434599702            # hydrogen ionisation energy [eV]
E_HE1_EV = 24.587387                # He I ionisation energy [eV]
E_HE2_EV = 54.417760                # He II ionisation energy [eV]
LAMBDA_2S1S = 8.2245809             # H 2s->1s two-photon rate [1/s]

H100_S = 1.0e5 / MPC_M              # 100 km/s/Mpc in 1/s
H100_MPC = 1.0e5 / C_M_S            # 100 km/s/Mpc in 1/Mpc (c = 1)
# critical density / h^2 in eV/cm^3: 3 H100^2 c^2 / (8 pi G), converted J/m^3 -> eV/cm^3
RHO_CRIT_H2_EV_CM3 = 3.0 * H100_S ** 2 * C_M_S ** 2 / (8.0 * math.pi * G_SI) / EV_J * 1.0e-6


def _inv_hbarc3() -> float:
    """eV^3 -> cm^-3 conversion factor."""
    return 1.0 / HBARC_EV_CM ** 3


def rho_crit_eV4() -> float:
    """critical density / h^2 in eV^4."""
    return RHO_CRIT_H2_EV_CM3 * HBARC_EV_CM ** 3


# ---------------------------------------------------------------------------
# Gauss rule for the massive-neutrino momentum integrals.
# ---------------------------------------------------------------------------
def fermi_dirac_rule(n: int):
    """n-node Gauss rule for integrals  int_0^inf dq q^2/(e^q+1) g(q).

    Built with the Golub-Welsch method from the exact moments
    int_0^inf q^(m+2)/(e^q+1) dq = (1 - 2^-(m+2)) (m+2)! zeta(m+3),
    evaluated in 60-digit arithmetic (the quadrature of App. B.3, eq. mnu_sum,
    with more nodes).  Returns (nodes, weights) as float arrays."""
    import mpmath as mp

    if n == 0:
        return np.zeros(0), np.zeros(0)
    mp.mp.dps = 60
    mom = [(1 - mp.mpf(2) ** (-(m + 2))) * mp.factorial(m + 2) * mp.zeta(m + 3) for m in range(2 * n + 1)]
    # Hankel moment matrix -> Cholesky -> Jacobi matrix (Golub & Welsch 1969)
    H = mp.matrix(n + 1, n + 1)
    for i in range(n + 1):
        for j in range(n + 1):
            H[i, j] = mom[i + j]
    R = mp.cholesky(H)  # lower triangular L, H = L L^T
    L = R
    alpha = []
    beta = []
    for j in range(n):
        a = L[j + 1, j] / L[j, j]
        if j > 0:
            a -= L[j, j - 1] / L[j - 1, j - 1]
        alpha.append(a)
    for j in range(n - 1):
        beta.append(L[j + 1, j + 1] / L[j, j])
    J = mp.matrix(n, n)
    for j in range(n):
        J[j, j] = alpha[j]
    for j in range(n - 1):
        J[j, j + 1] = beta[j]
        J[j + 1, j] = beta[j]
    E, Q = mp.eigsy(J)
    nodes = np.array([float(E[i]) for i in range(n)])
    weights = np.array([float(mom[0] * Q[0, i] ** 2) for i in range(n)])
    order = np.argsort(nodes)
    return nodes[order], weights[order]


# ---------------------------------------------------------------------------
# Cosmology: derived parameters and closed-form background.
# ---------------------------------------------------------------------------
class OracleError(Exception):
    def __init__(self, code: str, msg: str):
        super().__init__(f"{code}: {msg}")
        self.code = code


class Background:
    """Closed-form background (App. C) in units where rt_i(a) = (8 pi G/3) rho_i
    is in Mpc^-2 and the conformal Hubble rate is  Hc = a sqrt(sum_i rt_i)."""

    def __init__(self, cosmo: dict, n_q: int = 12):
        c = dict(cosmo)
        self.c = c
        h = c["h"]
        for key in ("h", "omega_b", "omega_cdm", "A_s", "TCMB0", "YHe"):
            v = c[key]
            if not (v == v) or v <= 0:
                raise OracleError("INVALID", f"{key}={v}")
        self.h = h
        self.H0 = h * H100_MPC                       # Mpc^-1
        rc = rho_crit_eV4()                          # eV^4 per h^2
        # conversion: (8 pi G/3) rho[eV^4] -> Mpc^-2, via rho/rho_crit * H0^2
        self.to_rt = H100_MPC ** 2 / rc              # multiply eV^4 by this -> Mpc^-2
        T0 = c["TCMB0"]
        self.T0 = T0
        self.rt_g0 = (math.pi ** 2 / 15.0) * T0 ** 4 * self.to_rt
        self.rt_c0 = c["omega_cdm"] * H100_MPC ** 2
        self.rt_b0 = c["omega_b"] * H100_MPC ** 2
        # neutrinos (Sec. 2.4): massless  rho = N 7 pi^2/120 T^4 a^-4
        Tml = c["T_nu_massless"] * T0
        Nm = float(c.get("N_nu_massive", 0.0))
        self.N_ncdm = Nm
        self.Tm_ratio = c["T_nu_massive"]
        Tm = self.Tm_ratio * T0
        self.Tncdm0 = Tm
        self.m_over_T = c["m_nu_massive"] / Tm if Nm > 0 else 0.0
        t_inst = (4.0 / 11.0) ** (1.0 / 3.0)
        neff_in = c.get("Neff", float("nan"))
        nml_in = c.get("N_nu_massless", float("nan"))
        if neff_in == neff_in and nml_in == nml_in:
            raise OracleError("CONFLICT", "both Neff and N_nu_massless given")
        per_massless = (c["T_nu_massless"] / t_inst) ** 4
        per_massive = (self.Tm_ratio / t_inst) ** 4
        if neff_in == neff_in:
            nml = (neff_in - Nm * per_massive) / per_massless
            if nml < 0:
                raise OracleError("NEG_NMASSLESS", f"N_nu_massless={nml}")
        else:
            nml = 3.0 if nml_in != nml_in else nml_in
        self.N_massless = nml
        self.Neff = nml * per_massless + Nm * per_massive
        self.rt_ur0 = nml * (7.0 * math.pi ** 2 / 120.0) * Tml ** 4 * self.to_rt
        # massive neutrinos: rho = (N/pi^2) T^4 a^-4 sum_i W_i eps_i (g_s = 2)
        if Nm > 0:
            if n_q <= 0:
                raise OracleError("INVALID", "massive neutrinos need n_q > 0")
            self.q, self.W = fermi_dirac_rule(n_q)
        else:
            self.q, self.W = np.zeros(0), np.zeros(0)
        self.pref_ncdm = Nm / math.pi ** 2 * Tm ** 4 * self.to_rt
        # Lambda closes the budget exactly at a = 1: Hc(1) = H0
        self.rt_L = self.H0 ** 2 - (self.rt_g0 + self.rt_ur0 + self.rt_c0 + self.rt_b0 + self.rho_ncdm(1.0)[0])
        # early-time radiation (massive nu relativistic) and R_nu
        ncdm_rel = self.pref_ncdm * float(np.sum(self.W * self.q)) if Nm > 0 else 0.0
        self.rt_rad_early = self.rt_g0 + self.rt_ur0 + ncdm_rel
        self.R_nu = (self.rt_ur0 + ncdm_rel) / self.rt_rad_early
        # matter
        self.rt_m0 = self.rt_c0 + self.rt_b0
        # recombination inputs
        Y = c["YHe"]
        self.YHe = Y
        self.fHe = Y * MH_EV / ((1.0 - Y) * MHE_EV)
        rho_b_eVcm3 = c["omega_b"] * RHO_CRIT_H2_EV_CM3
        self.nH0 = (1.0 - Y) * rho_b_eVcm3 / MH_EV  # cm^-3
        self.dk_pref = self.nH0 * SIGMA_T_CM2 * MPC_CM  # a n_e sigma_T = x_e * dk_pref * a^-2 [Mpc^-1]

    # -- densities ------------------------------------------------------
    def rho_ncdm(self, a: float):
        """(rho, p) of the massive species, in rt units."""
        if self.N_ncdm <= 0:
            return 0.0, 0.0
        x = a * self.m_over_T
        s_r = 0.0
        s_p = 0.0
        for qi, wi in zip(self.q, self.W):
            e = math.sqrt(qi * qi + x * x)
            s_r += wi * e
            s_p += wi * qi * qi / e
        return self.pref_ncdm * s_r / a ** 4, self.pref_ncdm * s_p / (3.0 * a ** 4)

    def rho_tot(self, a: float):
        """(rho_tot, p_tot) in rt units."""
        rn, pn = self.rho_ncdm(a)
        rr = (self.rt_g0 + self.rt_ur0) / a ** 4
        rho = rr + self.rt_m0 / a ** 3 + self.rt_L + rn
        p = rr / 3.0 - self.rt_L + pn
        return rho, p

    def Hc(self, a: float) -> float:
        """conformal Hubble rate a H [Mpc^-1]."""
        return a * math.sqrt(self.rho_tot(a)[0])

    def Hc_prime(self, a: float) -> float:
        """d Hc / d ln a  =  Hc (1 - 3/2 (rho+p)/rho)."""
        rho, p = self.rho_tot(a)
        return a * math.sqrt(rho) * (1.0 - 1.5 * (rho + p) / rho)

    def H_s(self, a: float) -> float:
        """Hubble rate in 1/s."""
        return self.Hc(a) / a * C_M_S / MPC_M


# ---------------------------------------------------------------------------
# Recombination (App. B.1) and reionisation (App. B.2).
# ---------------------------------------------------------------------------
def _pos_root(B: float, C: float) -> float:
    """positive root of x^2 + B x - C = 0 (C >= 0)."""
    return 2.0 * C / (B + math.sqrt(B * B + 4.0 * C))


def _saha_factor(mu_eV: float, T: float, E: float, nH: float) -> float:
    """(mu T / 2 pi)^{3/2} e^{-E/T} / n_H, dimensionless (n_H in cm^-3)."""
    return (mu_eV * T / (2.0 * math.pi)) ** 1.5 * _inv_hbarc3() * math.exp(-E / T) / nH


MU_E_H = ME_EV * (MH_EV - ME_EV) / MH_EV
MU_E_HE2 = ME_EV * (MHE_EV - 2 * ME_EV) / (MHE_EV - ME_EV)   # e + He++ reduced mass
MU_E_HE1 = ME_EV * (MHE_EV - ME_EV) / MHE_EV                 # e + He+ reduced mass


def helium_electrons(bg: Background, a: float) -> float:
    """Electrons per H nucleus contributed by helium, in Saha equilibrium:
    HeIII <-> HeII while x_HeIII >= 1e-9, then HeII <-> HeI (App. B.1)."""
    T = bg.T0 / a
    nH = bg.nH0 / a ** 3
    f = bg.fHe
    s2 = _saha_factor(MU_E_HE2, T, E_HE2_EV, nH)
    # x(1 + f + x)/(f - x) = s2
    x3 = _pos_root(1.0 + f + s2, s2 * f)
    if x3 >= 1e-9:
        return f + x3
    s1 = 4.0 * _saha_factor(MU_E_HE1, T, E_HE1_EV, nH)
    # x(1 + x)/(f - x) = s1
    return _pos_root(1.0 + s1, s1 * f)


def hydrogen_saha(bg: Background, a: float) -> float:
    """Saha ionised hydrogen fraction, eq. SahaH: x = (sqrt(s^2+4s)-s)/2."""
    T = bg.T0 / a
    s = _saha_factor(MU_E_H, T, E_H_EV, bg.nH0 / a ** 3)
    return 2.0 / (1.0 + math.sqrt(1.0 + 4.0 / s)) if s > 0 else 0.0


def alpha_B(T_eV: float) -> float:
    """Case-B recombination coefficient [cm^3/s]: Pequignot, Petitjean &
    Boisson (1991) fit with the 1.14 fudge factor of Seager, Sasselov & Scott
    (1999)."""
    t = T_eV / 8.617333262e-5 / 1.0e4
    return 1.14 * 1.0e-13 * 4.309 * t ** (-0.6166) / (1.0 + 0.6703 * t ** 0.5300)


def compton_rate(bg: Background, a: float, xe: float) -> float:
    """Gamma_C = 8 sigma_T rho_gamma c / (3 m_e) * x_e/(1+f_He+x_e)  [1/s]."""
    T = bg.T0 / a
    rho_g = (math.pi ** 2 / 15.0) * T ** 4 * _inv_hbarc3()  # eV/cm^3
    return 8.0 * SIGMA_T_CM2 * rho_g * (C_M_S * 100.0) / (3.0 * ME_EV) * xe / (1.0 + bg.fHe + xe)


def tm_quasi_static(bg: Background, a: float, xe: float) -> float:
    """T_m = T_cmb (1 - H/Gamma_C)  (App. B.1)."""
    return bg.T0 / a * (1.0 - bg.H_s(a) / compton_rate(bg, a, xe))


def peebles_rhs(bg: Background, a: float, xp: float, Tm: float):
    """d x_p / d ln a for the three-level atom (Peebles 1968)."""
    Tr = bg.T0 / a
    nH = bg.nH0 / a ** 3
    H = bg.H_s(a)
    xe = xp + helium_electrons(bg, a)
    aB_m = alpha_B(Tm)
    aB_r = alpha_B(Tr)
    beta = aB_r * (ME_EV * Tr / (2.0 * math.pi)) ** 1.5 * _inv_hbarc3() * math.exp(-0.25 * E_H_EV / Tr)
    lam_alpha = 2.0 * math.pi * HBARC_EV_CM / (0.75 * E_H_EV)  # cm
    K = lam_alpha ** 3 / (8.0 * math.pi * H)
    n1s = nH * (1.0 - xp)
    C = (1.0 + K * LAMBDA_2S1S * n1s) / (1.0 + K * (LAMBDA_2S1S + beta) * n1s)
    rate = -C * (aB_m * nH * xe * xp - beta * (1.0 - xp) * math.exp(-0.75 * E_H_EV / Tr))
    return rate / H


def tm_rhs(bg: Background, a: float, xp: float, Tm: float) -> float:
    """d T_m / d ln a = (-2 H T_m + Gamma_C (T_cmb - T_m)) / H (App. B.1)."""
    xe = xp + helium_electrons(bg, a)
    H = bg.H_s(a)
    return (-2.0 * H * Tm + compton_rate(bg, a, xe) * (bg.T0 / a - Tm)) / H


def reion_blend(bg: Background, a: float, xe_rec: float, zre: float) -> float:
    """x_e with the tanh reionisation steps patched on (eqs. h_reion, he_reion)."""
    c = bg.c
    z = 1.0 / a - 1.0
    beta = c["exp_reio"]
    y = (1.0 + z) ** beta
    yre = (1.0 + zre) ** beta
    dy = beta * c["Delta_z_reio"] * (1.0 + zre) ** (beta - 1.0)
    fH = 0.5 * (1.0 + math.tanh((yre - y) / dy))
    fHe = 0.5 * (1.0 + math.tanh((c["z_reio_He"] - z) / c["Delta_z_reio_He"]))
    return xe_rec + ((1.0 + bg.fHe) - xe_rec) * fH + bg.fHe * fHe


def reion_only(bg: Background, z: float, zre: float) -> float:
    """x_e from the tanh terms alone (the quantity in eq. tau_reion)."""
    c = bg.c
    beta = c["exp_reio"]
    y = (1.0 + z) ** beta
    yre = (1.0 + zre) ** beta
    dy = beta * c["Delta_z_reio"] * (1.0 + zre) ** (beta - 1.0)
    return (0.5 * (1.0 + bg.fHe) * (1.0 + math.tanh((yre - y) / dy))
            + 0.5 * bg.fHe * (1.0 + math.tanh((c["z_reio_He"] - z) / c["Delta_z_reio_He"])))


def tau_reion_of(bg: Background, zre: float, n_simpson: int = 2000) -> float:
    """Optical depth from reionisation alone, eq. tau_reion, written in z:
    tau = int_0^zmax dz sigma_T n_H0 (1+z)^2 x_e^reion(z) / H(z), with
    H(z) = (1+z) Hc, by Simpson's rule on n_simpson intervals up to
    zmax = max((y_re + 20 dy)^(1/beta) - 1, z_He + 20 dz_He)."""
    c = bg.c
    beta = c["exp_reio"]
    yre = (1.0 + zre) ** beta
    dy = beta * c["Delta_z_reio"] * (1.0 + zre) ** (beta - 1.0)
    zmax = max((yre + 20.0 * dy) ** (1.0 / beta) - 1.0, c["z_reio_He"] + 20.0 * c["Delta_z_reio_He"])
    hz = zmax / n_simpson
    total = 0.0
    for i in range(n_simpson + 1):
        z = i * hz
        a = 1.0 / (1.0 + z)
        f = bg.dk_pref * (1.0 + z) ** 2 * reion_only(bg, z, zre) / ((1.0 + z) * bg.Hc(a))
        w = 1.0 if (i == 0 or i == n_simpson) else (4.0 if i % 2 == 1 else 2.0)
        total += w * f
    return total * hz / 3.0


def bisect(f, lo: float, hi: float, iters: int = 100) -> float:
    """Plain bisection for an increasing f with f(lo) < 0 < f(hi)."""
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        if f(mid) > 0.0:
            hi = mid
        else:
            lo = mid
    return 0.5 * (lo + hi)


def z_reion_from_tau(bg: Background, tau: float) -> float:
    f = lambda z: tau_reion_of(bg, z) - tau
    lo, hi = 0.0, 50.0
    if not (f(lo) < 0.0 < f(hi)):
        raise OracleError("ROOT", f"tau_reio={tau} not bracketed by z_reion in [0, 50]")
    return bisect(f, lo, hi)


# ---------------------------------------------------------------------------
# Start times a_i(k)  (App. A.2).
# ---------------------------------------------------------------------------
LNA_SEARCH_MIN = math.log(1e-12)


def xe_early(bg: Background, a: float, zre: float) -> float:
    return reion_blend(bg, a, hydrogen_saha(bg, a) + helium_electrons(bg, a), zre)


def lna_tight_coupling(bg: Background, R_tc: float, zre: float) -> float:
    """ln a where Hc tau_c = R_tc, with x_e in its Saha phase."""
    def f(lna):
        a = math.exp(lna)
        dk = xe_early(bg, a, zre) * bg.dk_pref / a ** 2
        return bg.Hc(a) / dk - R_tc
    hi = math.log(1.0 / 1601.0)
    if not (f(LNA_SEARCH_MIN) < 0.0 < f(hi)):
        raise OracleError("ROOT", "R_tc start time not bracketed")
    return bisect(f, LNA_SEARCH_MIN, hi)


def lna_hubble_min(bg: Background) -> float:
    """ln a of the minimum of Hc (end of deceleration), or 0 if not reached."""
    f = lambda lna: bg.Hc_prime(math.exp(lna))
    if f(0.0) <= 0.0:
        return 0.0
    return bisect(f, math.log(0.01), 0.0)


def lna_start(bg: Background, k: float, R_tc: float, R_large: float, zre: float,
              lna_tc: float | None = None, lna_hmin: float | None = None) -> float:
    """min(a_tc, a_large(k)) in ln a; a_large has no root when k/Hc stays
    below R_large until the minimum of Hc, and is then ignored."""
    if lna_tc is None:
        lna_tc = lna_tight_coupling(bg, R_tc, zre)
    if lna_hmin is None:
        lna_hmin = lna_hubble_min(bg)
    f = lambda lna: k / bg.Hc(math.exp(lna)) - R_large
    if f(lna_hmin) <= 0.0:
        return lna_tc
    if f(LNA_SEARCH_MIN) >= 0.0:
        raise OracleError("ROOT", f"k={k} too large for the start-time search")
    return min(lna_tc, bisect(f, LNA_SEARCH_MIN, lna_hmin))


# ---------------------------------------------------------------------------
# Natural cubic spline on a uniform grid (values + second derivatives).
# ---------------------------------------------------------------------------
def natural_spline_M(f: np.ndarray, h: float) -> np.ndarray:
    """Second derivatives M of the natural cubic spline through f on a
    uniform grid of step h:  M_{j-1} + 4 M_j + M_{j+1} = 6 (f_{j+1} - 2 f_j + f_{j-1}) / h^2,
    M_0 = M_n = 0, solved by plain Gaussian elimination on the tridiagonal system."""
    n = len(f) - 1
    M = np.zeros(n + 1)
    if n < 2:
        return M
    m = n - 1
    diag = [4.0] * m
    rhs = [6.0 * (f[j + 1] - 2.0 * f[j] + f[j - 1]) / (h * h) for j in range(1, n)]
    for i in range(1, m):
        w = 1.0 / diag[i - 1]
        diag[i] -= w
        rhs[i] -= w * rhs[i - 1]
    x = [0.0] * m
    x[m - 1] = rhs[m - 1] / diag[m - 1]
    for i in range(m - 2, -1, -1):
        x[i] = (rhs[i] - x[i + 1]) / diag[i]
    M[1:n] = x
    return M


def spline_eval(f: np.ndarray, M: np.ndarray, x0: float, h: float, x: float, deriv: bool = False):
    """Evaluate the spline (and optionally its derivative) at x."""
    n = len(f) - 1
    u = (x - x0) / h
    j = int(math.floor(u))
    j = min(max(j, 0), n - 1)
    B = u - j
    A = 1.0 - B
    val = A * f[j] + B * f[j + 1] + ((A ** 3 - A) * M[j] + (B ** 3 - B) * M[j + 1]) * h * h / 6.0
    if not deriv:
        return val
    d = (f[j + 1] - f[j]) / h - (3.0 * A * A - 1.0) / 6.0 * h * M[j] + (3.0 * B * B - 1.0) / 6.0 * h * M[j + 1]
    return val, d


# ---------------------------------------------------------------------------
# Output-time grid and line-of-sight weights.
# ---------------------------------------------------------------------------
def source_lna_grid(n_tau: int) -> np.ndarray:
    """ceil(0.6 n) points uniform in ln a on [ln a(z=2500), ln a(z=400)], the
    rest uniform in ln a on (ln a(z=400), 0]; the last point is a = 1."""
    n1 = int(math.ceil(0.6 * n_tau))
    n2 = n_tau - n1
    l0 = -math.log(2501.0)
    l1 = -math.log(401.0)
    out = [l0 + (l1 - l0) * i / (n1 - 1) for i in range(n1)]
    out += [l1 + (0.0 - l1) * j / n2 for j in range(1, n2 + 1)]
    out[-1] = 0.0
    return np.array(out)


# ---------------------------------------------------------------------------
# The full table.
# ---------------------------------------------------------------------------
class Tables:
    pass


def build_tables(cosmo: dict, prec: dict, k: np.ndarray, n_tau: int) -> Tables:
    """Background/thermodynamics tables, start times and output grid."""
    k = np.asarray(k, dtype=np.float64)
    if len(k) < 1 or np.any(~np.isfinite(k)) or np.any(k <= 0) or np.any(np.diff(k) <= 0):
        raise OracleError("INVALID", "k must be positive and strictly increasing")
    if n_tau < 3:
        raise OracleError("INVALID", "n_tau < 3")
    bg = Background(cosmo, prec.get("n_q", 12) if cosmo.get("N_nu_massive", 0) > 0 else 0)
    c = bg.c
    if not (c["Delta_z_reio"] > 0 and c["Delta_z_reio_He"] > 0):
        raise OracleError("INVALID", "reionisation widths must be positive")
    tau_in = c.get("tau_reio", float("nan"))
    z_in = c.get("z_reio", float("nan"))
    if tau_in == tau_in and z_in == z_in:
        raise OracleError("CONFLICT", "both tau_reio and z_reio given")
    zre = z_reion_from_tau(bg, tau_in) if tau_in == tau_in else z_in
    if not (zre == zre):
        raise OracleError("INVALID", "neither tau_reio nor z_reio given")

    lna_tc = lna_tight_coupling(bg, prec["R_tc"], zre)
    lna_hmin = lna_hubble_min(bg)
    lna_i = np.array([lna_start(bg, float(kk), prec["R_tc"], prec["R_large"], zre, lna_tc, lna_hmin) for kk in k])
    n = int(prec["n_tab"])
    L0 = float(np.min(lna_i)) - 0.5
    dl = -L0 / n
    lna = np.array([L0 + j * dl for j in range(n)] + [0.0])

    # --- recombination on the grid --------------------------------------
    xe_rec = np.zeros(n + 1)
    Tm = np.zeros(n + 1)
    dlnTm = np.zeros(n + 1)
    j = 0
    # Saha phase: H by Saha while x_p >= 0.99
    while j <= n:
        a = math.exp(lna[j])
        xp = hydrogen_saha(bg, a)
        if xp < 0.99:
            break
        xe = xp + helium_electrons(bg, a)
        xe_rec[j] = xe
        Tm[j] = tm_quasi_static(bg, a, xe)
        dlnTm[j] = -1.0
        j += 1
    if j > n:
        raise OracleError("ROOT", "hydrogen never leaves Saha equilibrium")
    # Peebles phase: RK4 in ln a from knot j
    a = math.exp(lna[j])
    xp = hydrogen_saha(bg, a)
    xe = xp + helium_electrons(bg, a)
    xe_rec[j] = xe
    tm = tm_quasi_static(bg, a, xe)
    Tm[j] = tm
    z_switch = 700.0
    qs = (1.0 / a - 1.0) >= z_switch
    dlnTm[j] = -1.0 if qs else tm_rhs(bg, a, xp, tm) / tm
    while j < n:
        a0 = math.exp(lna[j])
        h = lna[j + 1] - lna[j]
        qs = (1.0 / a0 - 1.0) >= z_switch
        if qs:
            def rhs(lnx, x):
                aa = math.exp(lnx)
                t = tm_quasi_static(bg, aa, x + helium_electrons(bg, aa))
                return peebles_rhs(bg, aa, x, t)
            k1 = rhs(lna[j], xp)
            k2 = rhs(lna[j] + 0.5 * h, xp + 0.5 * h * k1)
            k3 = rhs(lna[j] + 0.5 * h, xp + 0.5 * h * k2)
            k4 = rhs(lna[j] + h, xp + h * k3)
            xp = xp + h / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
            a1 = math.exp(lna[j + 1])
            tm = tm_quasi_static(bg, a1, xp + helium_electrons(bg, a1))
        else:
            def rhs2(lnx, x, t):
                aa = math.exp(lnx)
                return peebles_rhs(bg, aa, x, t), tm_rhs(bg, aa, x, t)
            p1, t1 = rhs2(lna[j], xp, tm)
            p2, t2 = rhs2(lna[j] + 0.5 * h, xp + 0.5 * h * p1, tm + 0.5 * h * t1)
            p3, t3 = rhs2(lna[j] + 0.5 * h, xp + 0.5 * h * p2, tm + 0.5 * h * t2)
            p4, t4 = rhs2(lna[j] + h, xp + h * p3, tm + h * t3)
            xp = xp + h / 6.0 * (p1 + 2.0 * p2 + 2.0 * p3 + p4)
            tm = tm + h / 6.0 * (t1 + 2.0 * t2 + 2.0 * t3 + t4)
        j += 1
        a1 = math.exp(lna[j])
        xe_rec[j] = xp + helium_electrons(bg, a1)
        Tm[j] = tm
        qs1 = (1.0 / a1 - 1.0) >= z_switch
        dlnTm[j] = -1.0 if qs1 else tm_rhs(bg, a1, xp, tm) / tm

    # --- reionisation, Thomson rate, sound speed ------------------------
    xe = np.zeros(n + 1)
    dk = np.zeros(n + 1)
    cs2 = np.zeros(n + 1)
    for j in range(n + 1):
        a = math.exp(lna[j])
        xe[j] = reion_blend(bg, a, xe_rec[j], zre)
        dk[j] = xe[j] * bg.dk_pref / a ** 2
        mu = MH_EV / ((1.0 + xe[j]) * (1.0 - bg.YHe) + (MH_EV / MHE_EV) * bg.YHe)
        cs2[j] = Tm[j] / mu * (1.0 - dlnTm[j] / 3.0)

    # --- conformal time: closed form at L0, Simpson per interval ---------
    a0 = math.exp(L0)
    tau = np.zeros(n + 1)
    rr = bg.rt_rad_early
    tau[0] = 2.0 / bg.rt_m0 * (math.sqrt(rr + bg.rt_m0 * a0) - math.sqrt(rr))
    for j in range(n):
        h = lna[j + 1] - lna[j]
        fa = 1.0 / bg.Hc(math.exp(lna[j]))
        fm = 1.0 / bg.Hc(math.exp(lna[j] + 0.5 * h))
        fb = 1.0 / bg.Hc(math.exp(lna[j + 1]))
        tau[j + 1] = tau[j] + h / 6.0 * (fa + 4.0 * fm + fb)

    # --- optical depth kappa: trapezoid from a = 1 backwards ------------
    kap = np.zeros(n + 1)
    integrand = np.array([dk[j] / bg.Hc(math.exp(lna[j])) for j in range(n + 1)])
    for j in range(n - 1, -1, -1):
        kap[j] = kap[j + 1] + 0.5 * (lna[j + 1] - lna[j]) * (integrand[j] + integrand[j + 1])

    t = Tables()
    t.bg = bg
    t.cosmo = c
    t.prec = dict(prec)
    t.k = k
    t.z_reio = zre
    t.lna_tc = lna_tc
    t.lna_i = lna_i
    t.L0 = L0
    t.dl = dl
    t.n = n
    t.lna = lna
    t.xe = xe
    t.xe_rec = xe_rec
    t.Tm = Tm
    t.cols = {
        "ln_dk": np.log(dk),
        "kappa": kap,
        "ln_cs2": np.log(cs2),
        "ln_tau": np.log(tau),
    }
    t.M = {name: natural_spline_M(v, dl) for name, v in t.cols.items()}
    t.tau0 = tau[n]
    t.tau_knots = tau
    # --- output grid -----------------------------------------------------
    ls = source_lna_grid(n_tau)
    t.lna_src = ls
    tau_src = np.array([math.exp(spline_eval(t.cols["ln_tau"], t.M["ln_tau"], L0, dl, x)) for x in ls])
    chi = t.tau0 - tau_src
    chi[-1] = 0.0
    t.tau_src = tau_src
    t.chi_src = chi
    Hs = np.array([bg.Hc(math.exp(x)) for x in ls])
    w = np.zeros(n_tau)
    for j in range(n_tau):
        lo = ls[j - 1] if j > 0 else ls[j]
        hi = ls[j + 1] if j < n_tau - 1 else ls[j]
        w[j] = 0.5 * (hi - lo) / Hs[j]
    t.w_src = w
    return t


def eval_thermo(t: Tables, lna: float):
    """(dk, kappa, cs2, tau, d dk/d ln a) at ln a from the splines."""
    L0, dl = t.L0, t.dl
    ldk, dldk = spline_eval(t.cols["ln_dk"], t.M["ln_dk"], L0, dl, lna, deriv=True)
    dk = math.exp(ldk)
    kap = spline_eval(t.cols["kappa"], t.M["kappa"], L0, dl, lna)
    cs2 = math.exp(spline_eval(t.cols["ln_cs2"], t.M["ln_cs2"], L0, dl, lna))
    tau = math.exp(spline_eval(t.cols["ln_tau"], t.M["ln_tau"], L0, dl, lna))
    return dk, kap, cs2, tau, dk * dldk
