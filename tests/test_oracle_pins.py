"""Pins for the CPU oracle: checks against closed forms, limits, identities,
library routines and brute force, chosen so that a dropped term, a wrong
sign, index or factor in the oracle fails at least one of them.

All CPU-only (not marked gpu).  Citations refer to arXiv 2602.15104.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy.special import gammaln, spherical_jn

import cmb_workloads as W
import oracle as O
from oracle import background as B

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


@pytest.fixture(scope="module")
def tab12():
    wl = W.small_case(n_k=4, n_tau=50, ell_max=20, ell_g=12)
    return O.build_tables(wl.cosmo, wl.prec, wl.k, wl.n_tau)


def _tau(t, lna):
    return math.exp(B.spline_eval(t.cols["ln_tau"], t.M["ln_tau"], t.L0, t.dl, lna))


# ---------------------------------------------------------------- P1 quadrature
def test_paper_rules_weight_sums():
    """App. B.3: with Psi = 1 the printed rules must reproduce
    int q^4 e^q/(1+e^q)^2 dq = 4 int q^3/(e^q+1) dq = 4 * 7 pi^4/120."""
    target = 7 * math.pi ** 4 / 120
    for key in ("howlett_3pt", "gauss_laguerre_5pt"):
        s = sum(GOLD[key]["K"])
        assert abs(s / target - 1) < 1e-6, (key, s)


@pytest.mark.parametrize("n", [3, 5, 12])
def test_fermi_dirac_rule_moments(n):
    """Gauss rule for q^2/(e^q+1): exact for polynomials of degree < 2n,
    int q^(m+2)/(e^q+1) dq = (1 - 2^-(m+2)) (m+2)! zeta(m+3)."""
    import mpmath as mp
    q, w = B.fermi_dirac_rule(n)
    assert np.all(w > 0) and np.all(np.diff(q) > 0)
    for m in range(0, 2 * n):
        ex = float((1 - mp.mpf(2) ** (-(m + 2))) * mp.factorial(m + 2) * mp.zeta(m + 3))
        assert abs(np.sum(w * q ** m) / ex - 1) < 1e-12, m


def test_massive_nu_massless_limit():
    """rho of a massive species with m -> 0 equals the massless formula
    N 7 pi^2/120 T^4 a^-4 at the massive temperature (Sec. 2.4)."""
    c = W.fiducial()
    c["N_nu_massless"] = 3.0
    c["N_nu_massive"] = 1.0
    c["m_nu_massive"] = 1e-12
    bg = B.Background(c, 12)
    for a in (1e-6, 1e-3, 1.0):
        rho, p = bg.rho_ncdm(a)
        ex = (7 * math.pi ** 2 / 120) * (bg.Tncdm0 ** 4) * bg.to_rt / a ** 4
        assert abs(rho / ex - 1) < 1e-12
        assert abs(p / (rho / 3) - 1) < 1e-12


def test_neff_split():
    """eq. Neffdef: Neff = N_massless (T_ml/T_inst)^4 + N_massive (T_m/T_inst)^4."""
    c = W.fiducial()
    c["Neff"] = 3.044
    c["N_nu_massive"] = 1.0
    bg = B.Background(c, 12)
    ti = (4 / 11) ** (1 / 3)
    assert abs(bg.N_massless * (0.71636856 / ti) ** 4 + (0.71611 / ti) ** 4 - 3.044) < 1e-12
    assert 1.99 < bg.N_massless < 2.01
    c2 = W.fiducial()
    c2["Neff"] = 0.5
    c2["N_nu_massive"] = 1.0
    with pytest.raises(O.OracleError) as e:
        B.Background(c2, 12)
    assert e.value.code == "NEG_NMASSLESS"
    c3 = W.fiducial()
    c3["Neff"] = 3.044
    c3["N_nu_massless"] = 3.0
    with pytest.raises(O.OracleError) as e:
        B.Background(c3, 12)
    assert e.value.code == "CONFLICT"


# ---------------------------------------------------------------- P12/P13 tables
def test_background_closed_forms(tab12):
    bg = tab12.bg
    # Friedmann closure at a = 1 and the scaling of each species
    assert abs(bg.Hc(1.0) / bg.H0 - 1) < 1e-14
    for a in (1e-7, 1e-3, 0.5):
        rho, p = bg.rho_tot(a)
        ex = (bg.rt_g0 + bg.rt_ur0) * a ** -4 + (bg.rt_c0 + bg.rt_b0) * a ** -3 + bg.rt_L
        assert abs(rho / ex - 1) < 1e-14
        # H' from its closed form vs a centred difference in ln a
        h = 1e-5
        fd = (bg.Hc(a * math.exp(h)) - bg.Hc(a * math.exp(-h))) / (2 * h)
        assert abs(bg.Hc_prime(a) - fd) < 1e-7 * abs(bg.Hc(a))
    # photon density: omega_gamma h^2 for T = 2.7255 K is 2.473e-5
    assert abs(bg.rt_g0 / B.H100_MPC ** 2 / 2.4728e-5 - 1) < 2e-3


def test_table_fiducials(tab12):
    """Loose agreement with the fiducial conformal times printed in App. A.2
    (our recombination is a three-level atom, not HyRex, and h differs by 0.3%)."""
    fid = GOLD["fiducials"]
    t = tab12
    assert abs(t.tau0 / fid["tau0_fid_Mpc"] - 1) < 0.01
    g = np.exp(t.cols["ln_dk"] - t.cols["kappa"])
    j = int(np.argmax(g))
    assert abs(t.tau_knots[j] / fid["tau_rec_fid_Mpc"] - 1) < 0.02
    assert 1050 < math.exp(-t.lna[j]) - 1 < 1120
    # sound horizon at the visibility peak, c_s = 1/sqrt(3(1+R)), R = 3 rho_b / 4 rho_g
    bg = t.bg
    rs = 0.0
    for i in range(j):
        for l, wgt in ((t.lna[i], 0.5), (t.lna[i + 1], 0.5)):
            a = math.exp(l)
            R = 0.75 * bg.rt_b0 / bg.rt_g0 * a
            rs += wgt * (t.lna[i + 1] - t.lna[i]) / bg.Hc(a) / math.sqrt(3 * (1 + R))
    assert abs(rs / fid["rs_rec_fid_Mpc"] - 1) < 0.02


def test_thermo_identities(tab12):
    t = tab12
    assert t.cols["kappa"][-1] == 0.0
    # visibility integrates to 1 - e^{-kappa(start)} ~ 1 over the output grid
    g = []
    for l in t.lna_src:
        dk, kap, cs2, tau, dkp = B.eval_thermo(t, l)
        g.append(dk * math.exp(-kap))
    s = float(np.sum(np.array(g) * t.w_src))
    assert abs(s - 1) < 0.05
    # tau_reio re-derived from z_reio equals the input (root find, eq. tau_reion)
    assert abs(B.tau_reion_of(t.bg, t.z_reio) - t.cosmo["tau_reio"]) < 1e-10
    # x_e: fully ionised early (H + both He electrons), reionised late
    assert abs(t.xe[0] - (1 + 2 * t.bg.fHe)) < 1e-6
    assert abs(t.xe[-1] - (1 + 2 * t.bg.fHe)) < 1e-3
    # tight-coupling start: Hc tau_c = R_tc there
    a = math.exp(t.lna_tc)
    dk = B.xe_early(t.bg, a, t.z_reio) * t.bg.dk_pref / a ** 2
    assert abs(t.bg.Hc(a) / dk / t.prec["R_tc"] - 1) < 1e-12


def test_start_times():
    """a_i(k) = min(a_tc, a_large(k)); no root of k/Hc = R_large for tiny k."""
    wl = W.small_case(n_k=6, k_min=1e-5, k_max=0.5)
    t = O.build_tables(wl.cosmo, wl.prec, wl.k, wl.n_tau)
    bg = t.bg
    for k, l in zip(t.k, t.lna_i):
        a = math.exp(l)
        if l < t.lna_tc - 1e-12:
            assert abs(k / bg.Hc(a) / t.prec["R_large"] - 1) < 1e-10
        else:
            assert l == t.lna_tc
    assert t.lna_i[0] == t.lna_tc  # k = 1e-5: superhorizon until today


def test_spline_exact_for_cubic():
    """The natural spline reproduces a linear function exactly and a smooth
    function to O(h^4) in the interior."""
    h = 0.01
    x = np.arange(0, 201) * h
    f = 3.0 - 2.0 * x
    M = B.natural_spline_M(f, h)
    for xx in (0.0033, 0.5, 1.2345, 1.99):
        assert abs(B.spline_eval(f, M, 0.0, h, xx) - (3 - 2 * xx)) < 1e-13
    f = np.sin(x)
    M = B.natural_spline_M(f, h)
    v, d = B.spline_eval(f, M, 0.0, h, 1.0005, deriv=True)
    assert abs(v - math.sin(1.0005)) < 1e-10 and abs(d - math.cos(1.0005)) < 1e-7


def test_invalid_inputs():
    wl = W.small_case()
    with pytest.raises(O.OracleError):
        O.build_tables(wl.cosmo, wl.prec, np.array([0.1, 0.01]), 50)
    c = dict(wl.cosmo)
    c["z_reio"] = 8.0
    with pytest.raises(O.OracleError) as e:
        O.build_tables(c, wl.prec, wl.k, 50)
    assert e.value.code == "CONFLICT"
    c = dict(wl.cosmo)
    c["tau_reio"] = 5.0
    with pytest.raises(O.OracleError) as e:
        O.build_tables(c, wl.prec, wl.k, 50)
    assert e.value.code == "ROOT"


# ---------------------------------------------------------------- P2 free streaming
def test_free_streaming_is_bessel(tab12):
    """Gravity and Thomson scattering off, F_l(0) = delta_l0: the massless
    hierarchies (App. C) solve to F_l(tau) = j_l(k (tau - tau_i)) (plane-wave
    expansion) until the truncation at l_max is felt (k tau ~ l_max)."""
    t = tab12
    N = O.state_size(t.prec, 0)
    lg = t.prec["ell_gamma"]
    g0 = 3
    n0 = g0 + lg + 1 + (t.prec["ell_pol"] + 1 if t.prec["ell_pol"] > 0 else 0)
    k, lna0 = 0.02, -8.0
    lout = np.linspace(-7.9, -1.0, 150)
    y0 = np.zeros(N)
    y0[n0] = 1.0
    y0[g0] = 1.0
    r = O.perturb_one(t, k, lna0, lout, prec_over={"gravity_scale": 0.0, "thomson_scale": 0.0, "max_steps": 100000},
                      y0=y0, want_y=True, rtol=1e-11, atol=1e-14)
    assert r["status"] == 0
    x = k * (np.array([_tau(t, l) for l in lout]) - _tau(t, lna0))
    m = x <= lg / 2
    Y = r["y"]
    for l in range(0, lg // 2 - 1):
        for base in (n0, g0):
            F = {0: Y[:, base], 1: Y[:, base + 1] * 4 / (3 * k), 2: 2 * Y[:, base + 2]}.get(l, Y[:, base + l])
            assert np.max(np.abs(F - spherical_jn(l, x))[m]) < 1e-8, (l, base)


# ---------------------------------------------------------------- P3 superhorizon
def test_superhorizon_adiabatic_mode(tab12):
    """For k tau << 1 the adiabatic growing mode keeps eta constant to
    O((k tau)^2) across equality, with delta_gamma/delta_c = 4/3 and
    delta_b = delta_c (Ma & Bertschinger 1995, eq. 96)."""
    t = tab12
    N = O.state_size(t.prec, 0)
    for k in (1e-6, 5e-7):
        lout = np.linspace(t.lna_tc + 0.01, 0.0, 80)
        r = O.perturb_one(t, k, t.lna_tc, lout, want_y=True, rtol=1e-10, atol=1e-14, prec_over={"max_steps": 100000})
        y = r["y"]
        kt2 = (k * np.array([_tau(t, l) for l in lout])) ** 2
        dev = 1.0 - y[:, N - 1]
        assert np.all(np.abs(dev) <= 0.05 * kt2 + 1e-9)
        # radiation era: eta = 1 - (5 + 4 R_nu)/(12 (15 + 4 R_nu)) (k tau)^2
        Rn = t.bg.R_nu
        c_rd = (5 + 4 * Rn) / (12 * (15 + 4 * Rn))
        assert abs(dev[0] / (c_rd * kt2[0]) - 1) < 0.2
        j = int(np.argmin(np.abs(lout + math.log(1001))))
        assert abs(y[j, 3] / y[j, 0] - 4 / 3) < 1e-7
        assert abs(y[j, 1] / y[j, 0] - 1) < 1e-7


# ---------------------------------------------------------------- P4 tight coupling
def test_tight_coupling_slip(tab12):
    """In tight coupling the photon-baryon slip (theta_b - theta_g)/theta_g is
    proportional to Hc tau_c / R (R = 4 rho_g/3 rho_b), and halves when the
    Thomson rate doubles."""
    t = tab12
    k = 0.05
    lout = np.linspace(-12.5, -9.5, 31)
    slips = []
    for thom in (1.0, 2.0):
        r = O.perturb_one(t, k, -13.0, lout, want_y=True, rtol=1e-10, atol=1e-16,
                          prec_over={"max_steps": 100000, "thomson_scale": thom})
        y = r["y"]
        slips.append((y[:, 2] - y[:, 4]) / y[:, 4])
    a = np.exp(lout)
    R = 4 * t.bg.rt_g0 / (3 * t.bg.rt_b0) / a
    htc = np.array([t.bg.Hc(math.exp(l)) / B.eval_thermo(t, l)[0] for l in lout])
    p = np.polyfit(np.log(htc / R), np.log(np.abs(slips[0])), 1)
    assert abs(p[0] - 1) < 0.05
    ratio = slips[1][:10] / slips[0][:10]
    assert np.all(np.abs(ratio - 0.5) < 0.01)


# ---------------------------------------------------------------- P5 alpha'
def test_alpha_prime_closed_form(tab12):
    """alpha' from the traceless Einstein equation equals the derivative of
    alpha = Hc (h' + 6 eta')/(2k^2) along the solution."""
    t = tab12
    lout = np.linspace(-7.0, -0.5, 3001)
    r = O.perturb_one(t, 0.01, -10.0, lout, want_diag=True, rtol=1e-10, atol=1e-14, prec_over={"max_steps": 100000})
    assert r["status"] == 0
    al, alp = r["diag"][:, 2], r["diag"][:, 3]
    fd = np.gradient(al, lout)
    assert np.max(np.abs(fd[5:-5] - alp[5:-5])) < 1e-4 * np.max(np.abs(alp))


# ---------------------------------------------------------------- P6 brute force
@pytest.mark.parametrize("k", [1e-5, 1e-4, 1e-3])
def test_esdirk_matches_brute_force_rk4(tab12, k):
    """The ESDIRK stepper at rtol 1e-11 against classical RK4 with a step far
    below every time scale (h <= 5e-4 and h |lambda| <= 1/4), compared at the
    ESDIRK's own accepted step points (no interpolation involved)."""
    t = tab12
    e = O.perturb_one(t, k, t.lna_tc, t.lna_src, rtol=1e-11, atol=1e-15, prec_over={"max_steps": 200000},
                      acc_cap=100000)
    acc = e["accepted_lna"][::7]
    e2 = O.perturb_one(t, k, t.lna_tc, acc, rtol=1e-11, atol=1e-15, prec_over={"max_steps": 200000}, want_y=True)
    rb = O.rk4_one(t, k, t.lna_tc, acc, h_max=5e-4, c_stab=0.25, want_y=True)
    sc = np.max(np.abs(rb["y"]), axis=0)
    big = sc > 1e-8 * sc.max()
    err = np.abs(e2["y"] - rb["y"])[:, big] / sc[big]
    assert np.max(err) < 1e-7
    # the sources through the dense output agree to the interpolation level
    rs = O.rk4_one(t, k, t.lna_tc, t.lna_src, h_max=5e-4, c_stab=0.25)
    for i in range(3):
        assert np.max(np.abs(rs["S"][i] - e["S"][i])) < 5e-6 * np.max(np.abs(rs["S"][i]))


def test_esdirk_order_and_step_control(tab12):
    """Global error falls with rtol roughly like rtol (tolerance
    proportionality) and the step count grows like rtol^-1/4 or slower."""
    t = tab12
    k = 0.02
    ref = O.perturb_one(t, k, -10.0, t.lna_src, rtol=1e-11, atol=1e-15, prec_over={"max_steps": 200000})
    errs, steps = [], []
    for rt in (1e-5, 1e-7):
        r = O.perturb_one(t, k, -10.0, t.lna_src, rtol=rt, atol=rt * 1e-4, prec_over={"max_steps": 200000})
        errs.append(np.max(np.abs(r["S"][0] - ref["S"][0])) / np.max(np.abs(ref["S"][0])))
        steps.append(r["nsteps"])
    assert errs[1] < errs[0] / 10
    assert steps[1] < steps[0] * 100 ** 0.3


# ---------------------------------------------------------------- P7 Sachs-Wolfe
def test_sachs_wolfe_plateau():
    """n_s = 1: l(l+1) C_l/(2 pi A_s) approaches 1/25 on large scales
    (Sachs-Wolfe), within the effects of finite recombination, early and late
    ISW (15% with all terms for 10 <= l <= 20; 40% with the SW group alone)."""
    c = W.fiducial()
    c["N_nu_massless"] = 3.0
    c["n_s"] = 1.0
    k = np.concatenate([np.geomspace(1e-6, 1e-4, 40, endpoint=False), np.linspace(1e-4, 4e-3, 300)])
    l = np.arange(21)
    r = O.solve(c, W.prec_for(12, 0, 12), k, 400, 20, False)
    v = 25 * l * (l + 1) * r["Cl"][0] / (2 * math.pi * c["A_s"])
    assert np.all(np.abs(v[10:21] - 1) < 0.15)
    r = O.solve(c, W.prec_for(12, 0, 12, scale_isw=0.0, scale_dop=0.0, scale_pol=0.0), k, 400, 20, False)
    v = 25 * l * (l + 1) * r["Cl"][0] / (2 * math.pi * c["A_s"])
    assert np.all(np.abs(v[2:21] - 1) < 0.4)


# ---------------------------------------------------------------- P8 spike source
@pytest.mark.parametrize("ns", [1.0, 0.965])
def test_spike_source_closed_form(tab12, ns):
    """A unit-weight spike of S_T0 at one output time gives Delta_l(k) =
    j_l(k chi*), and C_l = 4 pi int dk/k P(k) j_l^2(k chi*) has the closed form
    4 pi A_s (k_p chi*)^(1-n_s) 2^(n_s-4) pi Gamma(3-n_s) Gamma(l+(n_s-1)/2)
    / (Gamma((4-n_s)/2)^2 Gamma(l+(5-n_s)/2)); for n_s = 1, 2 pi A_s/(l(l+1))."""
    t = tab12
    j = 30
    chis = t.chi_src[j]
    kk = np.linspace(1e-7, 2000 / chis, 40000)
    S = np.zeros((len(kk), 3, len(t.chi_src)))
    S[:, 0, j] = 1.0 / t.w_src[j]
    DT, DE = O.los(t, S, 20, False, k=kk)
    C = O.cl(kk, DT, DE, 20, False, 2e-9, ns, 0.05)
    L = np.arange(21)
    I = 2 ** (ns - 4) * math.pi * np.exp(gammaln(3 - ns) + gammaln(L + (ns - 1) / 2) - 2 * gammaln((4 - ns) / 2)
                                         - gammaln(L + (5 - ns) / 2))
    ex = 4 * math.pi * 2e-9 * (1 / 0.05) ** (ns - 1) * chis ** (1 - ns) * I
    assert np.max(np.abs(C[0, 2:] / ex[2:] - 1)) < 1e-3
    # Delta itself is the Bessel function (weights applied exactly once)
    jj = 777
    assert np.allclose(DT[:, jj], spherical_jn(np.arange(2, 21), kk[jj] * chis), rtol=1e-12, atol=1e-15)


# ---------------------------------------------------------------- P9/P10 Bessel
@pytest.mark.parametrize("x", [1e-3, 0.7, 3.3, 17.0, 150.0, 999.5, 2400.0, 2520.0, 7000.0])
def test_bessel_vs_mpmath(x):
    import mpmath as mp
    mp.mp.dps = 40
    L = 2501
    j = O.bessel(L, x)
    up = None
    if x > L:
        # all orders below x: 40-digit upward recurrence is exact enough
        X = mp.mpf(x)
        up = [mp.sin(X) / X, mp.sin(X) / X ** 2 - mp.cos(X) / X]
        for l in range(1, L):
            up.append((2 * l + 1) / X * up[l] - up[l - 1])
    for l in sorted(set([0, 1, 2, 3, 10, 100, 1000, 2000, 2400, 2450, 2500, 2501] +
                        [int(x) - 1, int(x), int(x) + 1, int(x) + 40])):
        if l < 0 or l > L:
            continue
        if up is not None:
            ex = float(up[l])
        else:
            ex = float(mp.sqrt(mp.pi / (2 * mp.mpf(x))) * mp.besselj(l + mp.mpf(1) / 2, mp.mpf(x)))
        if abs(ex) > 1e-290:
            assert abs(j[l] - ex) <= 1e-12 * abs(ex), (l, j[l], ex)
        else:
            assert abs(j[l]) < 1e-280


def test_bessel_identities():
    for x in (0.5, 12.0, 480.0, 3000.0):
        j = O.bessel(600, x)
        assert abs(j[0] - math.sin(x) / x) < 1e-15
        assert abs(j[1] - (math.sin(x) / x ** 2 - math.cos(x) / x)) < 1e-14
        assert abs(j[2] - ((3 / x ** 2 - 1) * math.sin(x) / x - 3 * math.cos(x) / x ** 2)) < 1e-14
        if x < 500:
            assert abs(np.sum((2 * np.arange(601) + 1) * j ** 2) - 1) < 1e-12
        assert np.allclose(j[:200], spherical_jn(np.arange(200), x), rtol=1e-10, atol=1e-300)
    j0 = O.bessel(10, 0.0)
    assert j0[0] == 1.0 and np.all(j0[1:] == 0.0)


def test_los_x_zero_limits(tab12):
    """x = 0 (tau = tau_0): j_l = j' = 0, (3j''+j)/2 = delta_l2/5,
    j_l/x^2 = delta_l2/15, and c_2 = sqrt(3 4! / 8 0!) = 3."""
    t = tab12
    n = len(t.chi_src)
    chi = np.zeros(n)
    w = np.zeros(n)
    w[-1] = 1.0
    S = np.zeros((1, 3, n))
    S[0, 2, -1] = 1.0
    DT, DE = O.los(t, S, 6, True, k=np.array([0.1]), chi=chi, w=w, s_pol=1.0)
    assert abs(DT[0, 0] - 0.2) < 1e-15 and np.all(DT[1:, 0] == 0)
    assert abs(DE[0, 0] - 3 * math.sqrt(6) / 15) < 1e-15 and np.all(DE[1:, 0] == 0)


def test_los_matches_direct_sum(tab12):
    """Delta_T and Delta_E against a direct sum with scipy's spherical_jn and
    its derivative (same trapezoid weights)."""
    t = tab12
    rng = np.random.Generator(np.random.PCG64(3))
    n = len(t.chi_src)
    k = np.array([0.003, 0.02, 0.07])
    S = rng.standard_normal((3, 3, n))
    DT, DE = O.los(t, S, 30, True, k=k, s_pol=0.7)
    for ik, kk in enumerate(k):
        x = kk * t.chi_src
        for l in (2, 5, 17, 30):
            xs = np.where(x > 0, x, 1.0)
            j = spherical_jn(l, x)
            jp = spherical_jn(l, x, derivative=True)
            jpp = -2 * jp / xs + (l * (l + 1) / xs ** 2 - 1) * j
            r2 = np.where(x > 0, 0.5 * (3 * jpp + j), 0.2 if l == 2 else 0.0)
            je = np.where(x > 0, j / xs ** 2, 1 / 15 if l == 2 else 0.0)
            T = np.sum(t.w_src * (S[ik, 0] * j + S[ik, 1] * jp + 0.7 * S[ik, 2] * r2))
            cl = math.sqrt(3 * (l + 2) * (l + 1) * l * (l - 1) / 8)
            E = cl * np.sum(t.w_src * math.sqrt(6) * S[ik, 2] * je)
            assert abs(DT[l - 2, ik] - T) < 1e-10 * np.sum(np.abs(t.w_src * S[ik, 0])) + 1e-14
            assert abs(DE[l - 2, ik] - E) < 1e-10 * abs(cl) * np.sum(np.abs(t.w_src * S[ik, 2])) + 1e-14


def test_physical_spectrum_shape():
    """Sanity of the whole oracle on a fine k grid: first acoustic peak of
    D_l^TT near l = 220 at 5000-6500 uK^2; TE positive near l = 300; EE
    reionisation bump at l = 2 (loose, unpinned accuracy)."""
    c = W.fiducial()
    c["N_nu_massless"] = 3.0
    k = np.linspace(2e-5, 0.04, 700)
    r = O.solve(c, W.prec_for(12, 8, 12, max_steps=8000), k, 600, 320, True)
    l = np.arange(321)
    D = l * (l + 1) * r["Cl"] / (2 * math.pi) * 2.7255e6 ** 2
    lp = 150 + int(np.argmax(D[0, 150:320]))
    assert 190 < lp < 250 and 5000 < D[0, lp] < 6500
    assert D[1, 300] > 50
    assert D[2, 2] > D[2, 8]


def test_matter_pk_large_scale_limit():
    """Matter power spectrum today (App. B.4, eq. PK) on scales that entered
    the horizon well after equality: the comoving-gauge Poisson equation with
    Phi = (3/5) R in matter domination and the dust + Lambda growth factor give
    P = 2 pi^2/k^3 P_R(k) [(2/5) (k/H0)^2 D(1) / Omega_m]^2, R = 1 (the eta -> 1
    normalisation).  The oracle must agree to 0.5% at k <= 1e-4 (the radiation
    era and the transfer function move it by ~0.2% there), and fall below it
    as k grows (transfer function < 1)."""
    from scipy.integrate import quad
    wl = W.small_case(n_k=4, k_min=5e-5, k_max=4e-4, n_tau=20)
    k = np.array([5e-5, 1e-4, 2e-4, 4e-4])
    t = O.build_tables(wl.cosmo, wl.prec, k, 20)
    P = O.matter_pk(t)
    c = wl.cosmo
    H0 = c["h"] / 2997.92458
    Om = (c["omega_b"] + c["omega_cdm"]) / c["h"] ** 2

    def E(a):
        return np.sqrt(Om / a ** 3 + 1.0 - Om)

    D1 = 2.5 * Om * E(1.0) * quad(lambda a: 1.0 / (a * E(a)) ** 3, 1e-10, 1.0, epsabs=0, epsrel=1e-12)[0]
    Pa = 2 * np.pi ** 2 / k ** 3 * c["A_s"] * (k / 0.05) ** (c["n_s"] - 1) * (0.4 * (k / H0) ** 2 * D1 / Om) ** 2
    r = P / Pa
    assert np.all(np.abs(r[:2] - 1) < 5e-3), r
    assert np.all(np.diff(r) < 0) and r[-1] < 1.0, r


def test_matter_pk_massive_neutrinos_large_scales():
    """With one massive neutrino, counted in Omega_m today, the large-scale
    P(k) stays within 1.5% of the same limit (the neutrinos were relativistic
    early on and lag the growth slightly)."""
    from scipy.integrate import quad
    wl = W.config2()
    wl.prec.update(ell_gamma=10, ell_pol=10, ell_nu=10, n_q=5, ell_ncdm=8)
    k = np.array([5e-5, 1e-4])
    t = O.build_tables(wl.cosmo, wl.prec, k, 20)
    P = O.matter_pk(t)
    c = wl.cosmo
    H0 = c["h"] / 2997.92458
    Om = (c["omega_b"] + c["omega_cdm"] + t.bg.rho_ncdm(1.0)[0] / (100.0 / 2997.92458) ** 2) / c["h"] ** 2

    def E(a):
        return np.sqrt(Om / a ** 3 + 1.0 - Om)

    D1 = 2.5 * Om * E(1.0) * quad(lambda a: 1.0 / (a * E(a)) ** 3, 1e-10, 1.0, epsabs=0, epsrel=1e-12)[0]
    Pa = 2 * np.pi ** 2 / k ** 3 * c["A_s"] * (k / 0.05) ** (c["n_s"] - 1) * (0.4 * (k / H0) ** 2 * D1 / Om) ** 2
    assert np.all(np.abs(P / Pa - 1) < 1.5e-2), P / Pa


# ---------------------------------------------------------------- P14 transfer k-grid
def test_transfer_kgrid_step_law():
    """App. A.2 eq. k_transfer_spacing with eq. defkperiod: the step is
    logarithmic (d ln k -> k_period logstep) at small k and linear
    (dk -> k_period linstep) at large k; the grid runs from k_min = 0.1/tau0_fid
    to k_max_cmb = 1.8 ell_max/tau0_fid (or the caller's bounds inside them)."""
    fid = GOLD["fiducials"]
    tau0, taur = fid["tau0_fid_Mpc"], fid["tau_rec_fid_Mpc"]
    kper = 2 * math.pi / (tau0 - taur)
    kt = O.transfer_kgrid(20000, 1e-7, 10.0)
    assert kt[0] == 0.1 / tau0 and kt[-1] == 1.8 * 20000 / tau0
    d = np.diff(kt)
    assert np.all(d > 0)
    assert abs(d[0] / kt[0] / (kper * 170.0) - 1) < 3e-3  # k_0 logstep/linstep ~ 3e-3
    assert abs(d[-2] / (kper * 0.45) - 1) < 2e-3  # linstep/(logstep k) ~ 1e-3
    # every step lies between its two limits, and the caller's bounds clip
    assert np.all(d[:-1] < kper * 0.45) and np.all(d[:-1] < kper * 170.0 * kt[:-2])
    kc = O.transfer_kgrid(2500, 1e-3, 0.2)
    assert kc[0] == 1e-3 and kc[-1] == 0.2 and np.all(np.diff(kc) > 0)
    # the last step may be short but never longer than the law
    assert kc[-1] - kc[-2] <= kper * 0.45 * kc[-2] / (kc[-2] + 0.45 / 170.0) * (1 + 1e-14)


def test_interp_sources_spline_properties():
    """Natural cubic splines in k: knots reproduced, linear functions exact,
    zero second derivative at both ends, O(h^4) error on a smooth function."""
    from scipy.interpolate import CubicSpline
    k = np.cumsum(np.linspace(0.01, 0.03, 40))
    kt = np.linspace(k[0], k[-1], 333)
    S = np.empty((len(k), 3, 5))
    for ty in range(3):
        for j in range(5):
            S[:, ty, j] = (ty - 1.5) * k + j
    St = O.interp_sources(k, S, kt)
    for ty in range(3):
        for j in range(5):
            assert np.allclose(St[:, ty, j], (ty - 1.5) * kt + j, rtol=0, atol=1e-13)
    R = np.random.default_rng(3).standard_normal(S.shape)
    assert np.allclose(O.interp_sources(k, R, k), R, rtol=0, atol=1e-14)
    S2 = np.sin(3 * k)[:, None, None] * np.ones((1, 3, 5))
    sp = CubicSpline(k, S2, axis=0, bc_type="natural")
    assert np.max(np.abs(sp(k[[0, -1]], 2))) < 1e-12
    St2 = O.interp_sources(k, S2, kt)
    # interior bound 5/384 h^4 max|f''''| ~ 9e-7; the end error decays ~3.7x a knot
    mid = (kt > k[8]) & (kt < k[-9])
    assert np.max(np.abs(St2[mid, 0, 0] - np.sin(3 * kt[mid]))) < 2e-6


def test_spectra_on_grid_invariants(tab12):
    """On the perturbation grid itself the transfer-grid path is the plain
    path (the spline passes through its knots); a source constant in k gives
    the spike closed form (C_l = 2 pi A_s/(l(l+1)) for n_s = 1) on a dense
    transfer grid."""
    t = tab12
    rng = np.random.default_rng(7)
    S = rng.standard_normal((len(t.k), 3, len(t.chi_src)))
    r = O.spectra_on_grid(t, S, t.k, 20, True)
    DT, DE = O.los(t, S, 20, True)
    C = O.cl(t.k, DT, DE, 20, True, t.cosmo["A_s"], t.cosmo["n_s"], t.prec["k_pivot"])
    assert np.allclose(r["Cl"], C, rtol=1e-12, atol=0)
    j = 30
    chis = t.chi_src[j]
    S = np.zeros((len(t.k), 3, len(t.chi_src)))
    S[:, 0, j] = 1.0 / t.w_src[j]
    kt = np.linspace(t.k[0], t.k[-1], 4000)
    tt = O.build_tables(dict(t.cosmo, n_s=1.0), t.prec, t.k, len(t.chi_src))
    r = O.spectra_on_grid(tt, S, kt, 20, False)
    L = np.arange(21)
    ex = 2 * math.pi * tt.cosmo["A_s"] / (L[2:] * (L[2:] + 1.0))
    xmin, xmax = kt[0] * chis, kt[-1] * chis  # keep l well inside the k range
    ok = (L[2:] > 3 * xmin) & (L[2:] < xmax / 3)
    assert ok.sum() >= 5
    assert np.max(np.abs(r["Cl"][0, 2:][ok] / ex[ok] - 1)) < 1e-3


# ---------------------------------------------------------------- P15 three-region Bessel scheme
@pytest.fixture(scope="module")
def b3tab():
    from oracle import bessel3 as B3
    return B3.Table(80)


def _mp_j(l, x, d=0):
    import mpmath as mp
    f = lambda z: mp.sqrt(mp.pi / (2 * z)) * mp.besselj(l + 0.5, z)  # noqa: E731
    return float(mp.diff(f, mp.mpf(x), d)) if d else float(f(mp.mpf(x)))


@pytest.mark.parametrize("l", [1, 7, 60, 80])
def test_bessel3_edges_vs_mpmath(b3tab, l):
    """x_start: j_l = 1e-10 there; x_5: a zero of j_l' with j_l'' < 0 and
    exactly four positive peaks of j_l before it (mpmath, independent of the
    scipy samples the scheme stores)."""
    import mpmath as mp
    mp.mp.dps = 30
    xs, x5 = b3tab.xs[l - 1], b3tab.x5[l - 1]
    assert abs(_mp_j(l, xs) / 1e-10 - 1) < 1e-9
    amp = abs(_mp_j(l, x5))
    assert abs(_mp_j(l, x5, 1)) < 1e-12 * amp and _mp_j(l, x5, 2) < 0
    grid = np.linspace(xs, x5 - 0.05, 400)
    d = np.array([_mp_j(l, g, 1) for g in grid])
    assert int(np.sum((d[:-1] > 0) & (d[1:] <= 0))) == 4


def test_bessel3_debye_limit():
    """The Debye-type form tends to j_l far above the turning point: its phase
    expands as x - nu pi/2 - pi/4 + nu^2/(2x) + ..., the exact one as
    x - (l+1) pi/2 + l(l+1)/(2x) + ..., and nu^2 - l(l+1) = 1/4, so x |error|
    stays below 1/(8x) (plus higher orders) and reaches it at the zeros."""
    from oracle import bessel3 as B3
    for l in (2, 30):
        for x0 in (400.0, 4000.0):
            xx = x0 + np.linspace(0, 2 * math.pi, 25)
            e = np.array([abs(B3.debye(l, v) - _mp_j(l, v)) * v for v in xx])
            assert np.max(e) <= 1.05 / (8 * x0) and np.max(e) >= 0.8 / (8 * (x0 + 7))


@pytest.mark.parametrize("l", [3, 45, 80])
def test_bessel3_regions(b3tab, l):
    """Zero below x_start; inside [x_start, x_5] linear interpolation within
    its bound dx^2/8 max|j''| (|j''| <= 1) of the exact value; the Debye form
    above x_5."""
    from oracle import bessel3 as B3
    xs, x5, dx = b3tab.xs[l - 1], b3tab.x5[l - 1], b3tab.dx[l - 1]
    rng = np.random.default_rng(l)
    below = rng.uniform(0, xs, 20)
    assert np.all(B3.j3(b3tab, l, below) == 0)
    inside = rng.uniform(xs, x5, 40)
    ex = np.array([_mp_j(l, v) for v in inside])
    assert np.max(np.abs(B3.j3(b3tab, l, inside) - ex)) <= dx * dx / 8 + 1e-14
    above = rng.uniform(x5 * 1.001, 3 * x5, 10)
    assert np.array_equal(B3.j3(b3tab, l, above), B3.debye(l, above))


def test_los3_assembly_with_exact_bessel(tab12):
    """The scheme's projection with the exact j_l in place of the scheme
    equals the oracle's recurrence-based projection (same sources): checks
    j' from j_{l-1}, j'' from Bessel's equation, the weights and the E
    factor."""
    from scipy.special import spherical_jn
    from oracle import bessel3 as B3
    t = tab12
    rng = np.random.default_rng(5)
    S = rng.standard_normal((len(t.k), 3, len(t.chi_src)))
    DT, DE = B3.los3(t, S, 20, True, jfun=lambda l, x: spherical_jn(l, x))
    RT, RE = O.los(t, S, 20, True)
    for a, b in ((DT, RT), (DE, RE)):
        assert np.max(np.abs(a - b)) <= 1e-10 * np.max(np.abs(b))


def test_los3_scheme_error_small(b3tab):
    """The scheme itself against the exact projection on physical sources
    (small hierarchy, l <= 80): the spectra differ at the level of the
    scheme's approximations (measured ~1e-4), far below the spectra."""
    from oracle import bessel3 as B3
    wl = W.small_case(n_k=40, n_tau=150, ell_max=80, k_max=0.05)
    r = O.solve(wl.cosmo, wl.prec, wl.k, wl.n_tau, wl.ell_max, True)
    t = r["tables"]
    DT, DE = B3.los3(t, r["S"], 80, True, T=b3tab)
    C = O.cl(t.k, DT, DE, 80, True, wl.cosmo["A_s"], wl.cosmo["n_s"])
    e = np.max(np.abs(C[0, 2:] / r["Cl"][0, 2:] - 1))
    assert 0 < e < 1e-2


# ---------------------------------------------------------------- P16 lensing potential (Limber)
def test_visibility_peak(tab12):
    """chi_*: the visibility kappa' e^-kappa is stationary there (centred
    difference of the oracle's splines), and tau_* lies within 1% of the
    paper's fiducial tau_rec (App. A.2)."""
    from oracle import lensing as LN
    t = tab12
    lna_s, tau_s, chi_s = LN.visibility_peak(t)

    def g(l):
        dk, kap, cs2, tau, dkp = B.eval_thermo(t, l)
        return dk * math.exp(-kap)

    h = 1e-3
    slope = (g(lna_s + h) - g(lna_s - h)) / (2 * h)
    curv = (g(lna_s + h) - 2 * g(lna_s) + g(lna_s - h)) / h ** 2
    assert abs(slope) < 2e-3 * abs(curv) * t.dl
    assert abs(tau_s / GOLD["fiducials"]["tau_rec_fid_Mpc"] - 1) < 0.01
    assert abs(chi_s - (t.tau0 - tau_s)) < 1e-9


def test_delta_m_growth_late_times():
    """Subhorizon delta_m at late times grows as the matter+Lambda growth
    factor D(a) proportional to H(a) int_0^a da'/(a' H(a'))^3 (radiation and
    neutrino free streaming below 0.5% there), and delta_m today equals the
    one inside P(k) (eq. PK)."""
    from scipy.integrate import quad
    wl = W.small_case(n_k=6, n_tau=200, ell_max=20, k_min=0.02, k_max=0.08)
    wl.prec["max_steps"] = 6000
    t = O.build_tables(wl.cosmo, wl.prec, wl.k, wl.n_tau)
    S, Dm, st, ns = O.perturb_dm(t)
    assert np.all(st == 0)
    bg = t.bg
    Om, OL = bg.rt_m0 / bg.H0 ** 2, bg.rt_L / bg.H0 ** 2

    def D(a):
        E = lambda x: math.sqrt(Om / x ** 3 + OL)  # noqa: E731
        return E(a) * quad(lambda x: 1.0 / (x * E(x)) ** 3, 0, a, limit=200)[0]

    j1 = int(np.argmin(np.abs(t.lna_src - math.log(0.25))))
    for i in range(len(t.k)):
        r = Dm[i, -1] / Dm[i, j1]
        ex = D(1.0) / D(math.exp(t.lna_src[j1]))
        assert abs(r / ex - 1) < 2e-3, (t.k[i], r, ex)  # measured 4.8e-4
    pk = O.matter_pk(t, np.array([2]))
    kk = t.k[2]
    prim = t.cosmo["A_s"] * (kk / t.prec["k_pivot"]) ** (t.cosmo["n_s"] - 1)
    assert abs(2 * math.pi ** 2 / kk ** 3 * prim * Dm[2, -1] ** 2 / pk[0] - 1) < 1e-12


def test_limber_sum_vs_quadrature(tab12):
    """With delta_m = c0 + c1 k (reproduced exactly by the natural spline) and
    n_s = 1, the discrete Limber sum equals the continuous integral over ln a
    (scipy quad of the closed-form integrand on the oracle's background) to
    the output-time quadrature's accuracy."""
    from scipy.integrate import quad
    from oracle import lensing as LN
    t = O.build_tables(dict(tab12.cosmo, n_s=1.0), tab12.prec, np.geomspace(1e-4, 2.0, 30), 400)
    c0, c1 = 0.3, 40.0
    Dm = (c0 + c1 * t.k)[:, None] * np.ones((1, len(t.lna_src)))
    C = LN.limber_cl(t, Dm, 60)
    lna_s, tau_s, chi_s = LN.visibility_peak(t)
    bg = t.bg
    A_s = t.cosmo["A_s"]
    for l in (2, 10, 60):
        nu = l + 0.5

        def f(lna):
            a = math.exp(lna)
            tau = math.exp(B.spline_eval(t.cols["ln_tau"], t.M["ln_tau"], t.L0, t.dl, lna))
            chi = t.tau0 - tau
            kk = nu / chi
            if not (t.k[0] <= kk <= t.k[-1]):
                return 0.0
            src = 1.5 * a * a * (bg.rt_m0 / a ** 3 + bg.rho_ncdm(a)[0])
            return (1.0 / bg.Hc(a)) / chi * src ** 2 * ((chi_s - chi) / chi_s) ** 2 * A_s * (c0 + c1 * kk) ** 2 / kk ** 4

        lo = max(lna_s, t.lna_src[0])
        ref = 8 * math.pi ** 2 / nu ** 3 * quad(f, lo, -1e-9, limit=400, points=[math.log(1 / 401.0)])[0]
        assert abs(C[l] / ref - 1) < 2e-3, (l, C[l], ref)


# ---------------------------------------------------------------- P17 lensed spectra
def _toy_spectra(L, seed=1):
    rng = np.random.default_rng(seed)
    ls = np.arange(2, L + 1)
    Cl = np.zeros((3, L + 1))
    Cl[0, 2:] = rng.uniform(1, 2, L - 1) / ls ** 2
    Cl[2, 2:] = rng.uniform(0.1, 0.2, L - 1) / ls ** 2
    Cl[1, 2:] = rng.uniform(-0.5, 0.5, L - 1) * np.sqrt(Cl[0, 2:] * Cl[2, 2:])
    Cpp = np.zeros(L + 1)
    Cpp[2:] = rng.uniform(0.5, 1.5, L - 1) * 2e-9 / ls ** 4
    return Cl, Cpp


def test_wigner_d_recurrence():
    """The recurrence against Wigner's explicit sum (l <= 12, every pair the
    method uses), d00 = P_l (scipy), and Gauss-Legendre orthogonality
    int d^l_mn d^l'_mn dmu = 2/(2l+1) delta_ll'."""
    from scipy.special import eval_legendre, roots_legendre
    from oracle import lensing as LN
    mu = np.linspace(-0.999, 0.999, 9)
    for a, b in [(0, 0), (1, 1), (1, -1), (2, 2), (2, -2), (3, 1), (3, -1), (3, -3), (4, 0), (4, -4), (0, 2), (2, 0),
                 (-2, 4)]:
        D = LN.wigner_d(a, b, 12, mu)
        for l in range(max(abs(a), abs(b)), 13):
            assert np.max(np.abs(D[l] - LN._d_explicit(l, a, b, mu))) < 1e-13, (a, b, l)
    P = LN.wigner_d(0, 0, 300, mu)
    assert np.max(np.abs(P - np.array([eval_legendre(l, mu) for l in range(301)]))) < 1e-12
    x, w = roots_legendre(120)
    d = LN.wigner_d(2, -2, 100, x)
    G = (d * w) @ d.T
    assert np.max(np.abs(G[2:, 2:] - np.diag(2.0 / (2 * np.arange(2, 101) + 1)))) < 1e-13


@pytest.mark.parametrize("l", [10, 300, 1500])
def test_x_functions_vs_definition(l):
    """Closed small-deflection forms of X_imn against their definition
    X_imn = int_0^inf (2a/s)(a/s)^i exp(-a^2/s) d^l_mn(a) da (s = sigma^2),
    by quadrature, at l^2 s ~ 0.1-2 (magnitudes; the signs of the odd
    ones are fixed by the first-order harmonic pin)."""
    from scipy.special import roots_legendre
    from oracle import lensing as LN
    s = 1.0 / (l * l)
    x, w = roots_legendre(400)
    a = 0.5 * (x + 1) * 8 * math.sqrt(s)
    wa = 0.5 * w * 8 * math.sqrt(s)
    X = LN.x_functions(np.array([l]), np.array([s]))
    for key, (i, m, n) in {"000": (0, 0, 0), "022": (0, 2, 2), "220": (2, 2, 0), "121": (1, 2, 1),
                           "132": (1, 3, 2), "242": (2, 4, 2), "112": (1, 1, 2)}.items():
        d = LN.wigner_d(m, n, l, np.cos(a))[l]
        ref = np.sum(wa * 2 * a / s * (a / s) ** i * np.exp(-a * a / s) * d)
        assert abs(abs(X[key][0, 0]) / abs(ref) - 1) < 2e-3, (key, X[key][0, 0], ref)


def test_lensing_zero_is_identity():
    """No lensing potential: the lensed spectra are the unlensed ones exactly
    and B stays zero."""
    from oracle import lensing as LN
    Cl, _ = _toy_spectra(40)
    out = LN.lensed_cl(Cl, np.zeros(41), 30, 90)
    assert np.array_equal(out[:3, 2:], Cl[:, 2:31]) and np.all(out[3] == 0)


def test_lensing_first_order_tt_vs_harmonic():
    """TT: the part of the lensed spectrum linear in C^psi (Richardson-
    extracted) against the exact first-order harmonic result (Wigner 3j
    sums, sympy),
      dC_l = -l(l+1) R C_l + sum_{l1 l2} C^psi_l1 C_l2 F^2/(2l+1),
      F = (l1(l1+1) + l2(l2+1) - l(l+1))/2 sqrt((2l+1)(2l1+1)(2l2+1)/(4 pi)) (l l1 l2; 0 0 0),
      R = sum l1(l1+1)(2l1+1) C^psi_l1/(8 pi).
    In correlation space the exact first order is
      -C_gl(0)/2 S_00 + C_gl(b)/2 S_11 + C_gl,2(b)/2 S_1-1,  S_mn = sum (2l+1)/(4 pi) l(l+1) C_l d^l_mn,
    while the method carries S_00 in the C_gl(b) term (its known large-angle
    approximation); that difference, C_gl(b)/2 (S_11 - S_00), is added back
    before comparing, so everything else is checked exactly."""
    from scipy.special import roots_legendre
    from sympy.physics.wigner import wigner_3j
    from oracle import lensing as LN
    L, lmax = 18, 12
    Cl, Cpp = _toy_spectra(L, seed=4)
    n_mu = 2 * L + lmax + 4
    base = np.zeros((4, lmax + 1))
    base[:3] = Cl[:, :lmax + 1]
    d1 = LN.lensed_cl(Cl, Cpp, lmax, n_mu)[0] - base[0]
    d2 = LN.lensed_cl(Cl, 2 * Cpp, lmax, n_mu)[0] - base[0]
    A = (4 * d1 - d2) / 2.0
    mu, w = roots_legendre(n_mu)
    ls = np.arange(L + 1)
    Cgl = ((2 * ls + 1) / (4 * math.pi) * ls * (ls + 1.0) * Cpp) @ LN.wigner_d(1, 1, L, mu)
    fT = (2 * ls + 1) / (4 * math.pi) * ls * (ls + 1.0) * Cl[0]
    dxi = 0.5 * Cgl * (fT @ (LN.wigner_d(1, 1, L, mu) - LN.wigner_d(0, 0, L, mu)))
    delta = 2 * math.pi * (LN.wigner_d(0, 0, lmax, mu) @ (w * dxi))
    R = np.sum(ls * (ls + 1) * (2 * ls + 1) * Cpp) / (8 * math.pi)
    H = np.zeros(lmax + 1)
    for l in range(2, lmax + 1):
        H[l] = -l * (l + 1) * R * Cl[0, l]
        for l1 in range(2, L + 1):
            for l2 in range(2, L + 1):
                if not abs(l - l1) <= l2 <= l + l1 or (l + l1 + l2) % 2:
                    continue
                F = 0.5 * (l1 * (l1 + 1) + l2 * (l2 + 1) - l * (l + 1)) * math.sqrt(
                    (2 * l + 1) * (2 * l1 + 1) * (2 * l2 + 1) / (4 * math.pi)) * float(wigner_3j(l, l1, l2, 0, 0, 0))
                H[l] += Cpp[l1] * Cl[0, l2] * F * F / (2 * l + 1)
    assert np.max(np.abs(A[2:] + delta[2:] - H[2:])) < 1e-7 * np.max(np.abs(H[2:]))
    # and the method's own approximation is small against the effect at l >= 8
    assert np.max(np.abs(delta[8:] / H[8:])) < 0.05


def test_lensing_first_order_flat_sky_limit():
    """All four spectra at l ~ 600-1000, where the sphere is flat on the
    lensing scales: the first-order correction (Richardson-extracted) against
    the flat-sky harmonic integrals (psi momentum L, field momentum l1 = l - L,
    phi the angle between l and l1):
      dC^TT = -l^2 R C^TT + int d^2L/(2pi)^2 [L.(l-L)]^2 C^psi_L C^TT_l1,
      dC^EE = -l^2 R C^EE + int ... C^EE_l1 cos^2 2phi,   dC^BB = int ... C^EE_l1 sin^2 2phi,
      dC^TE = -l^2 R C^TE + int ... C^TE_l1 cos 2phi,     R = int L^3 C^psi dL/(4 pi),
    within 3% of each correction (measured 0.8-2%: curvature terms of order
    1/L at the lensing scale L ~ 150, and 1/l)."""
    from oracle import lensing as LN
    L = 1600
    # oscillating field spectra (so that lensing changes them at the percent
    # level) and lensing power localised at L ~ 150 (flat on its own scale)
    cT = lambda x: (1.0 + 0.5 * np.cos(x / 30.0)) / x ** 2  # noqa: E731
    cE = lambda x: 0.05 * (1.0 + 0.8 * np.sin(x / 30.0)) / x ** 2  # noqa: E731
    cX = lambda x: 0.1 / x ** 2 * np.cos(x / 30.0)  # noqa: E731
    cP = lambda x: 1e-6 / x ** 4 * np.exp(-((x - 150.0) / 60.0) ** 2)  # noqa: E731
    ls = np.arange(L + 1, dtype=np.float64)
    Cl = np.zeros((3, L + 1))
    Cl[0, 2:], Cl[1, 2:], Cl[2, 2:] = cT(ls[2:]), cX(ls[2:]), cE(ls[2:])
    Cpp = np.zeros(L + 1)
    Cpp[2:] = cP(ls[2:])
    lmax = 1000
    base = np.zeros((4, lmax + 1))
    base[:3] = Cl[:, :lmax + 1]
    d1 = LN.lensed_cl(Cl, Cpp, lmax, 2800) - base
    d2 = LN.lensed_cl(Cl, 2 * Cpp, lmax, 2800) - base
    A = (4 * d1 - d2) / 2.0
    R = np.sum(ls ** 3 * Cpp) / (4 * math.pi)
    Lg = np.arange(2, L + 1, dtype=np.float64)[:, None]
    th = (np.arange(4096) + 0.5) * 2 * math.pi / 4096
    for l in (600, 1000):
        l1 = np.sqrt(l * l + Lg * Lg - 2 * l * Lg * np.cos(th))
        dot = l * Lg * np.cos(th) - Lg * Lg  # L.(l - L)
        cphi = (l * l - l * Lg * np.cos(th)) / (l * l1)
        c2 = 2 * cphi * cphi - 1
        ok = (l1 >= 2) & (l1 <= L)
        kern = np.where(ok, dot * dot * cP(Lg), 0.0) * Lg / (2 * math.pi) ** 2 * (2 * math.pi / 4096)
        l1s = np.where(ok, l1, 2.0)
        fl = {0: -l * l * R * cT(l) + np.sum(kern * cT(l1s)),
              2: -l * l * R * cE(l) + np.sum(kern * cE(l1s) * c2 * c2),
              3: np.sum(kern * cE(l1s) * (1 - c2 * c2)),
              1: -l * l * R * cX(l) + np.sum(kern * cX(l1s) * c2)}
        for i, ref in fl.items():
            assert abs(A[i, l] / ref - 1) < 0.03, (l, i, A[i, l], ref)


# ---------------------------------------------------------------- P18 parameter derivatives
@pytest.fixture(scope="module")
def jac_case():
    wl = W.small_case(n_k=16, n_tau=150, ell_max=200, k_max=0.1)
    return wl


def test_replay_reproduces_run(jac_case):
    """Replaying a run's own recorded start and step sizes reproduces its
    sources bit for bit (the same sequence of times and stages)."""
    wl = jac_case
    t = O.build_tables(wl.cosmo, wl.prec, wl.k, wl.n_tau)
    S, st, ns, hist, hn = O.perturb_hist(t)
    assert np.array_equal(S, O.perturb(t)[0]) and np.all(st == 0)
    assert np.all(hn == O.perturb(t)[3])  # one history entry per accepted step
    S2, st2, ns2, _, _ = O.perturb_hist(t, hist, hn)
    assert np.array_equal(S2, S) and np.all(ns2 == hn)


def test_restart_from_step_end_continues_run(jac_case):
    """A trajectory checkpoint is the state at the end of an accepted step:
    restarting there (the state as start, the remaining recorded steps
    replayed) continues the run bit for bit after the restart (the oracle
    forms every stage derivative as the right-hand side at the stage value,
    so the derivative it recomputes at the restart is the one it would have
    carried), and writes nothing before it."""
    wl = jac_case
    t = O.build_tables(wl.cosmo, wl.prec, wl.k, wl.n_tau)
    S, st, ns, hist, hn = O.perturb_hist(t)
    lo = np.asarray(t.lna_src)
    for ik in (3, 15):
        k, lna0 = float(t.k[ik]), float(t.lna_i[ik])
        acc = O.perturb_one(t, k, lna0, [], acc_cap=hist.shape[1])["accepted_lna"]
        for j in (max(1, int(hn[ik]) // 3), 2 * int(hn[ik]) // 3):
            tc = float(acc[j - 1])
            yc = O.perturb_one(t, k, lna0, [tc], want_y=True)["y"][0]
            r = O.perturb_one(t, k, tc, lo, y0=yc, fixed=np.concatenate([[tc], hist[ik, 1 + j:1 + hn[ik]]]))
            assert r["status"] == 0 and r["naccept"] == hn[ik] - j
            after = lo > tc
            assert np.all(r["S"][:, ~after] == 0.0)
            assert np.array_equal(r["S"][:, after], S[ik][:, after]), (ik, j)


def test_jacobian_stencils_consistent(jac_case):
    """Frozen steps make the discrete map smooth: the five-point derivative at
    rel 1e-4 and at 2e-4 agree to 1e-6 of each row (measured <= 1.6e-7), and
    the central difference differs from it only by its O(e^2) truncation."""
    wl = jac_case
    C, J4, st = O.jacobian(wl.cosmo, wl.prec, wl.k, wl.n_tau, 120, True, rel=1e-4, order=4)
    _, J4b, _ = O.jacobian(wl.cosmo, wl.prec, wl.k, wl.n_tau, 120, True, rel=2e-4, order=4)
    _, J2, _ = O.jacobian(wl.cosmo, wl.prec, wl.k, wl.n_tau, 120, True, rel=1e-4, order=2)
    assert np.all(st == 0)
    for p in (0, 1, 2, 5):
        m = np.max(np.abs(J4[p][:, 2:]))
        assert np.max(np.abs(J4b[p][:, 2:] - J4[p][:, 2:])) < 1e-6 * m, p
        assert np.max(np.abs(J2[p][:, 2:] - J4[p][:, 2:])) < 1e-4 * m, p
    assert np.array_equal(J4[3], C)


def test_dcl_dns_analytic(tab12):
    """dC/dn_s by the ln(k/k_pivot)-weighted quadrature against a five-point
    difference of the oracle's C_l in n_s on the same transfer functions."""
    t = tab12
    rng = np.random.default_rng(2)
    S = rng.standard_normal((len(t.k), 3, len(t.chi_src)))
    DT, DE = O.los(t, S, 20, True)
    ns, e = 0.965, 1e-3
    f = lambda x: O.cl(t.k, DT, DE, 20, True, 2e-9, x, 0.05)  # noqa: E731
    fd = (8 * (f(ns + e) - f(ns - e)) - (f(ns + 2 * e) - f(ns - 2 * e))) / (12 * e)
    an = O.cl_dns(t.k, DT, DE, 20, True, 2e-9, ns, 0.05)
    assert np.max(np.abs(an[:, 2:] - fd[:, 2:])) < 1e-9 * np.max(np.abs(an[:, 2:]))


def test_dcl_dtau_reio_high_l():
    """Above the reionisation scales the spectra scale as e^{-2 tau_reio}:
    dC/dtau = -2 C (on average over l = 250-300 within 2.5% for EE and over
    l = 200-300 within 10% for TT; late-time sources and the coarse k grid
    scatter single multipoles by ~10%)."""
    wl = W.small_case(n_k=120, n_tau=200, ell_max=300, k_min=1e-4, k_max=0.05)
    wl.prec["max_steps"] = 6000
    C, J, st = O.jacobian(wl.cosmo, wl.prec, wl.k, wl.n_tau, 300, True, rel=1e-4, order=2)
    assert np.all(st == 0)
    ree = J[5, 2, 250:301] / C[2, 250:301]
    rtt = J[5, 0, 200:301] / C[0, 200:301]
    assert abs(np.mean(ree) + 2) < 0.05 and abs(np.mean(rtt) + 2) < 0.2


def test_spectra_adjoint_dot_product(tab12):
    """The oracle's transposed quadrature and projection: <dL/dS, V> equals
    the central difference of L = sum gC C_l(S) along V (exact for this
    quadratic map up to rounding)."""
    t = tab12
    rng = np.random.default_rng(0)
    S = rng.standard_normal((len(t.k), 3, len(t.chi_src)))
    gC = rng.standard_normal((3, 21))

    def L(Sx):
        DT, DE = O.los(t, Sx, 20, True)
        return float(np.sum(gC[:, 2:] * O.cl(t.k, DT, DE, 20, True, 2e-9, 0.96)[:, 2:]))

    DT, DE = O.los(t, S, 20, True)
    GT, GE = O.cl_adjoint(t.k, DT, DE, gC, 20, True, 2e-9, 0.96)
    gS = O.los_adjoint(t, GT, GE, 20, True)
    V = rng.standard_normal(S.shape)
    fd = (L(S + 1e-3 * V) - L(S - 1e-3 * V)) / 2e-3
    assert abs(np.sum(gS * V) / fd - 1) < 1e-11


# ---------------------------------------------------------------- transposed sources
@pytest.fixture(scope="module")
def src_case():
    wl = W.small_case(n_k=3, n_tau=30, ell_max=20, ell_g=8, k_max=0.1)
    return O.build_tables(wl.cosmo, wl.prec, wl.k, wl.n_tau)


def test_sources_adjoint_dot_product(src_case):
    """<dL/dS, S(y)> = <dL/dy, y> at every output time for seeded states y and
    seeded dL/dS: the transposed source map against the forward one (App. B.4)."""
    t = src_case
    rng = np.random.Generator(np.random.PCG64(61))
    gS = rng.standard_normal((len(t.k), 3, len(t.lna_src)))
    gY = O.sources_adjoint(t, gS)
    order = O.library_row_order(t.prec, len(t.bg.q))
    N = len(order)
    assert N == O.state_size(t.prec, len(t.bg.q))
    assert sorted(order) == list(range(N))
    for ik, k in enumerate(t.k):
        for j in range(0, len(t.lna_src), 7):
            y = rng.standard_normal(N)  # oracle layout
            S = O.sources_of_state(t, k, t.lna_src[j], y)
            lhs = float(gS[ik, :, j] @ S) if t.lna_src[j] >= t.lna_i[ik] else 0.0
            rhs = float(gY[ik, j] @ y[order])
            scale = float(np.abs(gS[ik, :, j]) @ np.abs(S)) + 1e-300
            assert abs(lhs - rhs) <= 1e-12 * scale, (ik, j, lhs, rhs)


def test_sources_adjoint_structure(src_case):
    """Only S_T2 = g Pi / 8 with Pi = 2 F_g2 + G_0 + G_2 (App. B.4): dL/dS_T2 = 1
    alone reaches the rows F_g2, G_0 and G_2, in the ratio 2 : 1 : 1; nothing
    reaches any row before a mode's start."""
    t = src_case
    gS = np.zeros((len(t.k), 3, len(t.lna_src)))
    gS[:, 2, :] = 1.0
    gY = O.sources_adjoint(t, gS)
    lg, lp = int(t.prec["ell_gamma"]), int(t.prec["ell_pol"])
    f2, g0 = 3, lg + 2
    for ik in range(len(t.k)):
        for j in range(len(t.lna_src)):
            row = gY[ik, j]
            if t.lna_src[j] < t.lna_i[ik]:
                assert np.all(row == 0.0)
                continue
            nz = set(np.nonzero(row)[0])
            assert nz <= {f2, g0, g0 + 2}, nz
            if row[f2] != 0.0:
                assert lp > 0
                assert abs(row[g0] / row[f2] - 0.5) < 1e-14 and abs(row[g0 + 2] / row[f2] - 0.5) < 1e-14
