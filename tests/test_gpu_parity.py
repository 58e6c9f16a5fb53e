"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Norms (arXiv 2602.15104 has no worked numbers for this path, so the bar is the
oracle):
  sources  per (cosmology, k, type): max_j |S_gpu - S_orc| / max_j |S_orc| <= 1e-8
  C_ell    TT, EE elementwise relative <= 1e-6; TE relative to sqrt(TT EE) <= 1e-6
  Delta    per k: max_l |D_gpu - D_orc| / max_l |D_orc| <= 1e-9 (same sources in)
"""
import math
import os
import sys

import numpy as np
import pytest

import cmb_workloads as W

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def ctx():
    _need_gpu()
    import paper_2602_15104_amd as L
    c = L.Context(0)
    yield c
    c.close()


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def src_err(Sg, So):
    """max over (k, type) of max_j |dS| / max_j |S_orc|."""
    worst = 0.0
    for i in range(So.shape[0]):
        for t in range(3):
            den = np.max(np.abs(So[i, t]))
            if den == 0.0:
                assert np.max(np.abs(Sg[i, t])) == 0.0
                continue
            worst = max(worst, np.max(np.abs(Sg[i, t] - So[i, t])) / den)
    return worst


def lk(D):
    """Transfer functions as the library lays them out, [..., 2, n_k, l - 2],
    in the oracle's order [..., 2, l - 2, n_k]."""
    return np.swapaxes(D, -1, -2)


def cl_err(Cg, Co, lmin=2):
    tt = np.max(np.abs(Cg[0, lmin:] / Co[0, lmin:] - 1))
    if np.any(Co[2, lmin:] != 0):
        ee = np.max(np.abs(Cg[2, lmin:] / Co[2, lmin:] - 1))
        te = np.max(np.abs(Cg[1, lmin:] - Co[1, lmin:]) / np.sqrt(Co[0, lmin:] * Co[2, lmin:]))
    else:
        ee = te = 0.0
    return tt, te, ee


def run_gpu(ctx, tabs, ell_max):
    import torch
    import paper_2602_15104_amd as L
    out = L.solve_batch(ctx, tabs, ell_max)
    torch.cuda.synchronize()
    return {k: (v.cpu().numpy() if v is not None else None) for k, v in out.items()}


@pytest.mark.parametrize("pol", [True, False])
def test_small_case_full_parity(ctx, pol):
    """12 modes (one ragged 64-lane tile), 120 output times, l <= 60."""
    import oracle as O
    import paper_2602_15104_amd as L
    wl = W.small_case(n_k=12, n_tau=120, ell_max=60, polarization=pol)
    _say("case small", wl.name, "pol", pol)
    tab = L.Tables(wl.cosmo, wl.prec, wl.k, wl.n_tau)
    g = run_gpu(ctx, [tab], wl.ell_max)
    r = O.solve(wl.cosmo, wl.prec, wl.k, wl.n_tau, wl.ell_max, pol)
    assert np.all(g["status"] == 0) and np.all(r["status"] == 0)
    assert np.all(np.abs(g["nsteps"][0] - r["nsteps"]) <= 2), (g["nsteps"][0], r["nsteps"])
    e = src_err(g["S"][0], r["S"])
    _say("source err", e)
    assert e <= 1e-8
    tt, te, ee = cl_err(g["Cl"][0], r["Cl"])
    _say("cl err", tt, te, ee)
    assert tt <= 1e-6 and te <= 1e-6 and ee <= 1e-6
    assert np.all(g["Cl"][0, :, :2] == 0)
    if not pol:
        assert np.all(g["Delta"][0, 1] == 0)


def test_config0_full_parity(ctx):
    """Config 0 at full size: TT, 64 modes, 400 output times, l <= 500."""
    import oracle as O
    import paper_2602_15104_amd as L
    wl = W.config0()
    _say("case", wl.name)
    tab = L.Tables(wl.cosmo, wl.prec, wl.k, wl.n_tau)
    g = run_gpu(ctx, [tab], wl.ell_max)
    r = O.solve(wl.cosmo, wl.prec, wl.k, wl.n_tau, wl.ell_max, False)
    assert np.all(g["status"] == 0)
    e = src_err(g["S"][0], r["S"])
    _say("source err", e, "steps gpu/orc", g["nsteps"].sum(), r["nsteps"].sum())
    assert e <= 1e-8
    tt, _, _ = cl_err(g["Cl"][0], r["Cl"])
    _say("cl err TT", tt)
    assert tt <= 1e-6


def test_los_cl_from_same_sources(ctx):
    """K2 + K3 alone: the oracle projects the GPU's own sources (config-0
    grid, l <= 500), so Delta and C_ell compare without integrator effects."""
    import torch
    import oracle as O
    import paper_2602_15104_amd as L
    wl = W.config0()
    wl.prec["ell_pol"] = 6
    tab = L.Tables(wl.cosmo, wl.prec, wl.k, wl.n_tau)
    t_or = O.build_tables(wl.cosmo, wl.prec, wl.k, wl.n_tau)
    rng = np.random.Generator(np.random.PCG64(5))
    S = rng.standard_normal((1, len(wl.k), 3, wl.n_tau))
    dS = torch.tensor(S, device="cuda:0")
    D = torch.empty((1, 2, len(wl.k), wl.ell_max - 1), dtype=torch.float64, device="cuda:0")
    C = torch.empty((1, 3, wl.ell_max + 1), dtype=torch.float64, device="cuda:0")
    ctx.los([tab], wl.ell_max, dS, D)
    ctx.cl([tab], wl.ell_max, D, C)
    torch.cuda.synchronize()
    DT, DE = O.los(t_or, S[0], wl.ell_max, True)
    Dg = lk(D.cpu().numpy()[0])
    for ik in range(len(wl.k)):
        for plane, ref in ((0, DT), (1, DE)):
            den = np.max(np.abs(ref[:, ik]))
            assert np.max(np.abs(Dg[plane][:, ik] - ref[:, ik])) <= 1e-9 * den, (plane, ik)
    Co = O.cl(t_or.k, Dg[0], Dg[1], wl.ell_max, True, wl.cosmo["A_s"], wl.cosmo["n_s"])
    np.testing.assert_allclose(C.cpu().numpy()[0][:, 2:], Co[:, 2:], rtol=1e-12, atol=0)


def test_los_cl_maximum_sizes(ctx):
    """K2 + K3 at the largest sizes the projection accepts: l_max = 10000 and
    4096 output times, on seeded sources, for five k from 1e-4 to 0.8 Mpc^-1
    (k chi up to 11000: the upward-recurrence seeding for x > l_max + 32, and
    Miller's seeding with the cut below it).  Delta against the oracle's
    projection to 1e-9 of each k's largest value, C_l against the oracle's
    quadrature of the same Delta to 1e-12; 4097 output times are refused
    (CMB_E_UNSUPPORTED)."""
    import torch
    import oracle as O
    import paper_2602_15104_amd as L
    wl = W.config0()
    wl.prec["ell_pol"] = 6  # a polarisation hierarchy, so that K2 writes the E plane
    k = np.array([1e-4, 3e-3, 0.05, 0.3, 0.8])
    n_tau, lmax = 4096, 10000
    _say("case los maximum sizes: l_max", lmax, "n_tau", n_tau, "k", k)
    tab = L.Tables(wl.cosmo, wl.prec, k, n_tau)
    t_or = O.build_tables(wl.cosmo, wl.prec, k, n_tau)
    rng = np.random.Generator(np.random.PCG64(9))
    S = rng.standard_normal((1, len(k), 3, n_tau))
    D = torch.empty((1, 2, len(k), lmax - 1), dtype=torch.float64, device="cuda:0")
    C = torch.empty((1, 3, lmax + 1), dtype=torch.float64, device="cuda:0")
    ctx.los([tab], lmax, torch.tensor(S, device="cuda:0"), D)
    ctx.cl([tab], lmax, D, C)
    torch.cuda.synchronize()
    DT, DE = O.los(t_or, S[0], lmax, True)
    Dg = lk(D.cpu().numpy()[0])
    worst = 0.0
    for ik in range(len(k)):
        for plane, ref in ((0, DT), (1, DE)):
            den = np.max(np.abs(ref[:, ik]))
            e = np.max(np.abs(Dg[plane][:, ik] - ref[:, ik])) / den
            worst = max(worst, e)
            assert e <= 1e-9, (plane, ik, e)
    Co = O.cl(k, Dg[0], Dg[1], lmax, True, wl.cosmo["A_s"], wl.cosmo["n_s"])
    np.testing.assert_allclose(C.cpu().numpy()[0][:, 2:], Co[:, 2:], rtol=1e-12, atol=0)
    _say("max-size projection err", worst)
    big = L.Tables(wl.cosmo, wl.prec, k[:2], n_tau + 1)
    Sb = torch.zeros((1, 2, 3, n_tau + 1), dtype=torch.float64, device="cuda:0")
    Db = torch.empty((1, 2, 2, lmax - 1), dtype=torch.float64, device="cuda:0")
    with pytest.raises(L.CmbError) as e:
        ctx.los([big], lmax, Sb, Db)
    assert e.value.name == "CMB_E_UNSUPPORTED"


def test_spike_source_closed_form_gpu(ctx):
    """A unit-weight spike of S_T0 at one output time: Delta_l(k) = j_l(k chi*)
    and, with n_s = 1, l(l+1) C_l/(2 pi A_s) = 1 up to k-quadrature error."""
    import torch
    import paper_2602_15104_amd as L
    c = W.fiducial()
    c["N_nu_massless"] = 3.0
    c["n_s"] = 1.0
    prec = W.prec_for(8, 0, 8)
    n_tau = 60
    k = np.linspace(1e-6, 0.15, 6000)
    tab = L.Tables(c, prec, k, n_tau)
    ex = tab.export()
    j = 30
    chis = ex["chi_src"][j]
    S = np.zeros((1, len(k), 3, n_tau))
    S[0, :, 0, j] = 1.0 / ex["w_src"][j]
    ell_max = 40
    dS = torch.tensor(S, device="cuda:0")
    D = torch.empty((1, 2, len(k), ell_max - 1), dtype=torch.float64, device="cuda:0")
    C = torch.empty((1, 3, ell_max + 1), dtype=torch.float64, device="cuda:0")
    ctx.los([tab], ell_max, dS, D)
    ctx.cl([tab], ell_max, D, C)
    torch.cuda.synchronize()
    from scipy.special import spherical_jn
    Dg = lk(D.cpu().numpy()[0, 0])
    for ik in (10, 777, 3000, 5999):
        np.testing.assert_allclose(Dg[:, ik], spherical_jn(np.arange(2, ell_max + 1), k[ik] * chis), rtol=1e-11,
                                   atol=1e-17)
    l = np.arange(ell_max + 1)
    v = l * (l + 1) * C.cpu().numpy()[0, 0] / (2 * math.pi * c["A_s"])
    assert np.max(np.abs(v[2:] - 1)) < 2e-3


def test_batch_invariance_and_determinism(ctx):
    """A cosmology's result alone equals its result inside a batch of three
    different cosmologies, bit for bit, and repeated runs are bitwise equal."""
    import paper_2602_15104_amd as L
    wl = W.small_case(n_k=70, n_tau=150, ell_max=80, k_max=0.1)
    cosmos = W.perturbed_cosmologies(3, seed=7)
    for cc in cosmos:
        cc["N_nu_massless"] = 3.0
    tabs = [L.Tables(cc, wl.prec, wl.k, wl.n_tau) for cc in cosmos]
    a = run_gpu(ctx, [tabs[1]], wl.ell_max)
    b = run_gpu(ctx, tabs, wl.ell_max)
    c = run_gpu(ctx, tabs, wl.ell_max)
    assert np.array_equal(a["Cl"][0], b["Cl"][1])
    assert np.array_equal(a["S"][0], b["S"][1])
    assert np.array_equal(b["Cl"], c["Cl"])
    assert np.array_equal(b["nsteps"], c["nsteps"])


def test_launch_shape_invariance(ctx):
    """Config-1 hierarchy (79 rows) on 40 modes to k = 0.2, one cosmology in
    four launch shapes: alone (a whole wavefront per mode), among 30
    cosmologies (1200 modes: 32-lane groups), among 60 (2400 modes: 16-lane
    groups) and among 210 (8400 modes: 8-lane groups of ten rows, eight modes
    per wavefront); sources, step counts and C_ell are the same bits in all."""
    import paper_2602_15104_amd as L
    wl = W.config1()
    k = W.log_grid(1e-4, 0.2, 40)
    cosmos = W.perturbed_cosmologies(210, seed=19)
    for cc in cosmos:
        cc["N_nu_massless"] = 3.0
    tabs = [L.Tables(cc, wl.prec, k, 200) for cc in cosmos]
    a = run_gpu(ctx, [tabs[11]], 300)
    b = run_gpu(ctx, tabs[:30], 300)
    c = run_gpu(ctx, tabs[:60], 300)
    d = run_gpu(ctx, tabs, 300)
    for o in (a, b, c, d):
        assert np.all(o["status"] == 0)
    for o in (b, c, d):
        assert np.array_equal(a["nsteps"][0], o["nsteps"][11])
        assert np.array_equal(a["S"][0], o["S"][11])
        assert np.array_equal(a["Cl"][0], o["Cl"][11])
    # a cosmology late in the dense launch too (another wavefront, other slots)
    e = run_gpu(ctx, [tabs[197]], 300)
    assert np.array_equal(e["S"][0], d["S"][197]) and np.array_equal(e["nsteps"][0], d["nsteps"][197])


def test_dense_shape_record_replay(ctx):
    """Step histories in the dense launch shape (8-lane groups, 8400 modes):
    the recorded history and sources of one cosmology equal its solo record
    (a whole wavefront per mode) bit for bit, replaying the dense histories
    reproduces the sources, and the record launch's sources equal the plain
    launch's on every mode."""
    import torch
    import paper_2602_15104_amd as L
    wl = W.config1()
    k = W.log_grid(1e-4, 0.2, 40)
    cosmos = W.perturbed_cosmologies(210, seed=23)
    for cc in cosmos:
        cc["N_nu_massless"] = 3.0
    tabs = [L.Tables(cc, wl.prec, k, 200) for cc in cosmos]
    cap = wl.prec["max_steps"] + 1

    def record(tb):
        n = len(tb)
        S = torch.empty((n, len(k), 3, 200), dtype=torch.float64, device="cuda:0")
        st = torch.empty((n, len(k)), dtype=torch.int32, device="cuda:0")
        H = torch.empty((n, len(k), cap), dtype=torch.float64, device="cuda:0")
        Hn = torch.empty((n, len(k)), dtype=torch.int32, device="cuda:0")
        ctx.perturb_record(tb, S, st, H, Hn)
        torch.cuda.synchronize()
        return S, st, H, Hn

    S, st, H, Hn = record(tabs)
    S1, st1, H1, Hn1 = record([tabs[5]])
    assert torch.all(st == 0) and torch.all(st1 == 0)
    assert torch.equal(Hn[5], Hn1[0])
    for i in range(len(k)):
        n = int(Hn1[0, i].item())
        assert torch.equal(H[5, i, :n + 1], H1[0, i, :n + 1]), i
    assert torch.equal(S[5], S1[0])
    S2 = torch.empty_like(S)
    st2 = torch.empty_like(st)
    ctx.perturb_replay(tabs, H, Hn, S2, st2)
    torch.cuda.synchronize()
    assert torch.all(st2 == 0) and torch.equal(S2, S)
    # the record instance (its own compiled kernel) against the plain one on
    # the same 8400 modes: every source, bit for bit
    S3 = torch.empty_like(S)
    st3 = torch.empty_like(st)
    ns3 = torch.empty_like(st)
    ctx.perturb(tabs, S3, st3, ns3)
    torch.cuda.synchronize()
    assert torch.all(st3 == 0) and torch.equal(S3, S)


def test_batched_parity_box_cosmologies(ctx):
    """Three cosmologies from the paper's validation box in one batch, each
    against its own oracle solve (sources and C_ell)."""
    import oracle as O
    import paper_2602_15104_amd as L
    wl = W.small_case(n_k=20, n_tau=150, ell_max=120, k_max=0.1, ell_g=10)
    cosmos = W.box_cosmologies(3, seed=3)
    tabs = [L.Tables(cc, wl.prec, wl.k, wl.n_tau) for cc in cosmos]
    g = run_gpu(ctx, tabs, wl.ell_max)
    for i, cc in enumerate(cosmos):
        r = O.solve(cc, wl.prec, wl.k, wl.n_tau, wl.ell_max, True)
        e = src_err(g["S"][i], r["S"])
        tt, te, ee = cl_err(g["Cl"][i], r["Cl"])
        _say("box", i, e, tt, te, ee)
        assert e <= 1e-8 and tt <= 1e-6 and te <= 1e-6 and ee <= 1e-6


def test_max_steps_flag(ctx):
    """max_steps = 4: every mode reports CMB_K_MAX_STEPS and its sources are
    zero from the first unreached output time on."""
    import paper_2602_15104_amd as L
    wl = W.small_case(n_k=5, n_tau=40, ell_max=20)
    wl.prec["max_steps"] = 4
    tab = L.Tables(wl.cosmo, wl.prec, wl.k, wl.n_tau)
    g = run_gpu(ctx, [tab], wl.ell_max)
    assert np.all(g["status"] == 1) and np.all(g["nsteps"] == 4)
    assert np.all(g["S"][0][:, :, -1] == 0)
    assert np.all(np.isfinite(g["Cl"]))


def test_single_mode_and_lmax2(ctx):
    """Degenerate sizes: one mode (its trapezoid k-weight is zero, so C_ell is
    exactly zero on both sides) and ell_max = 2 with two modes."""
    import oracle as O
    import paper_2602_15104_amd as L
    wl = W.small_case(n_k=1, n_tau=30, ell_max=2, k_min=0.01, k_max=0.01)
    wl.k = np.array([0.01])
    tab = L.Tables(wl.cosmo, wl.prec, wl.k, wl.n_tau)
    g = run_gpu(ctx, [tab], 2)
    r = O.solve(wl.cosmo, wl.prec, wl.k, wl.n_tau, 2, True)
    assert src_err(g["S"][0], r["S"]) <= 1e-8
    assert np.all(g["Cl"][0] == 0) and np.all(r["Cl"] == 0)
    D = lk(g["Delta"][0])
    den = np.max(np.abs(r["DT"]))
    assert np.max(np.abs(D[0] - r["DT"])) <= 1e-9 * den
    wl.k = np.array([0.005, 0.01])
    tab = L.Tables(wl.cosmo, wl.prec, wl.k, wl.n_tau)
    g = run_gpu(ctx, [tab], 2)
    r = O.solve(wl.cosmo, wl.prec, wl.k, wl.n_tau, 2, True)
    tt, te, ee = cl_err(g["Cl"][0], r["Cl"])
    assert tt <= 1e-6 and ee <= 1e-6 and te <= 1e-6


def test_config1_full_size(ctx):
    """Config 1 at full size, the fiducial cosmology alone (the plain solve's
    launch shape): the sources of all 400 modes against the oracle computed
    live, and the full C_ell against the stored oracle spectrum
    (tests/golden/make_oracle_reference.py)."""
    import oracle as O
    import paper_2602_15104_amd as L
    wl = W.config1()
    _say("case", wl.name)
    ref = os.path.join(GOLD, "oracle_config1_cl.npy")
    assert os.path.exists(ref), "oracle golden missing: run tests/golden/make_oracle_reference.py config1"
    tab = L.Tables(wl.cosmo, wl.prec, wl.k, wl.n_tau)
    g = run_gpu(ctx, [tab], wl.ell_max)
    assert np.all(g["status"] == 0), np.bincount(g["status"].ravel())
    t_or = O.build_tables(wl.cosmo, wl.prec, wl.k, wl.n_tau)
    S, st, ns, na = O.perturb(t_or)
    assert np.all(st == 0)
    e = src_err(g["S"][0], S)
    _say("source err (400 modes)", e, "max step-count difference", np.max(np.abs(g["nsteps"][0] - ns)))
    assert e <= 1e-8
    Co = np.load(ref)
    tt, te, ee = cl_err(g["Cl"][0], Co)
    _say("cl err", tt, te, ee)
    assert tt <= 1e-6 and te <= 1e-6 and ee <= 1e-6


@pytest.mark.parametrize("which", [5, 21])
def test_config1_benchmark_batch_cosmologies(ctx, which):
    """Config 1 in the benchmark's launch configuration: the benchmark's batch
    of 32 seeded cosmologies (5 % Gaussian around the fiducial, seed
    20260215) in one launch; cosmology `which` of it checked in full against
    the oracle computed live on the same inputs: sources of all 400 modes and
    C_ell."""
    import oracle as O
    import paper_2602_15104_amd as L
    wl = W.config1()
    cosmos = W.perturbed_cosmologies(32, seed=20260215)
    for c in cosmos:
        c["N_nu_massless"] = 3.0
    _say("case", wl.name, "benchmark batch of 32, cosmology", which)
    tabs = [L.Tables(c, wl.prec, wl.k, wl.n_tau) for c in cosmos]
    g = run_gpu(ctx, tabs, wl.ell_max)
    assert np.all(g["status"] == 0), np.bincount(g["status"].ravel())
    r = O.solve(cosmos[which], wl.prec, wl.k, wl.n_tau, wl.ell_max, True)
    assert np.all(r["status"] == 0)
    e = src_err(g["S"][which], r["S"])
    tt, te, ee = cl_err(g["Cl"][which], r["Cl"])
    _say("source err (400 modes)", e, "cl err", tt, te, ee, "max step-count difference",
         np.max(np.abs(g["nsteps"][which] - r["nsteps"])))
    assert e <= 1e-8
    assert tt <= 1e-6 and te <= 1e-6 and ee <= 1e-6


def _massive(wl, m_nu, n_q, ell_ncdm):
    c = wl.cosmo
    c["N_nu_massless"] = float("nan")
    c["Neff"] = 3.044
    c["N_nu_massive"] = 1.0
    c["m_nu_massive"] = m_nu
    wl.prec.update(n_q=n_q, ell_ncdm=ell_ncdm)
    return wl


@pytest.mark.parametrize("m_nu", [0.06, 0.6])
def test_massive_nu_small_parity(ctx, m_nu):
    """One massive neutrino species (App. C massive neutrinos, App. B.3 eq.
    mnu_sum) on a small hierarchy: 3 momentum nodes with l <= 6, photon and
    massless cut-offs 8, 10 modes up to k = 0.2 (a ragged set of groups), 100
    output times, l <= 100.  At 0.6 eV the massive terms are large."""
    import oracle as O
    import paper_2602_15104_amd as L
    wl = _massive(W.small_case(n_k=10, n_tau=100, ell_max=100, k_max=0.2), m_nu, 3, 6)
    _say("case massive small m =", m_nu)
    tab = L.Tables(wl.cosmo, wl.prec, wl.k, wl.n_tau)
    g = run_gpu(ctx, [tab], wl.ell_max)
    r = O.solve(wl.cosmo, wl.prec, wl.k, wl.n_tau, wl.ell_max, True)
    assert np.all(g["status"] == 0) and np.all(r["status"] == 0)
    assert np.all(np.abs(g["nsteps"][0] - r["nsteps"]) <= 2), (g["nsteps"][0], r["nsteps"])
    e = src_err(g["S"][0], r["S"])
    tt, te, ee = cl_err(g["Cl"][0], r["Cl"])
    _say("source err", e, "cl err", tt, te, ee)
    assert e <= 1e-8
    assert tt <= 1e-6 and te <= 1e-6 and ee <= 1e-6


def test_massive_nu_batch_invariance(ctx):
    """Two massive-neutrino cosmologies (0.06 and 0.6 eV) in one launch give
    bitwise the results of separate launches."""
    import paper_2602_15104_amd as L
    tabs = []
    for m_nu in (0.06, 0.6):
        wl = _massive(W.small_case(n_k=7, n_tau=60, ell_max=40, k_max=0.1), m_nu, 3, 5)
        tabs.append(L.Tables(wl.cosmo, wl.prec, wl.k, wl.n_tau))
    both = run_gpu(ctx, tabs, 40)
    for i in range(2):
        one = run_gpu(ctx, [tabs[i]], 40)
        assert np.array_equal(both["S"][i], one["S"][0])
        assert np.array_equal(both["Cl"][i], one["Cl"][0])


def test_config2_full_size(ctx):
    """Config 2 (config 1 + one 0.06 eV neutrino, 12 momentum nodes x l <= 17,
    N = 295 rows, 600 modes) at full size: sampled modes' sources against the
    oracle computed live, the full C_ell and the per-mode step counts against
    the stored oracle run (tests/golden/make_oracle_reference.py)."""
    import oracle as O
    import paper_2602_15104_amd as L
    wl = W.config2()
    _say("case", wl.name)
    tab = L.Tables(wl.cosmo, wl.prec, wl.k, wl.n_tau)
    g = run_gpu(ctx, [tab], wl.ell_max)
    assert np.all(g["status"] == 0), np.bincount(g["status"].ravel())
    t_or = O.build_tables(wl.cosmo, wl.prec, wl.k, wl.n_tau)
    idx = np.array([0, 40, 200, 599])
    S, st, ns, na = O.perturb(t_or, idx)
    e = src_err(g["S"][0][idx], S)
    _say("sampled source err", e, "steps", g["nsteps"][0][idx], ns)
    assert e <= 1e-8
    ref = os.path.join(GOLD, "oracle_config2_cl.npy")
    assert os.path.exists(ref), "oracle golden missing: run tests/golden/make_oracle_reference.py config2"
    Co = np.load(ref)
    tt, te, ee = cl_err(g["Cl"][0], Co)
    nso = np.load(os.path.join(GOLD, "oracle_config2_nsteps.npy"))
    _say("cl err", tt, te, ee, "max step-count difference", np.max(np.abs(g["nsteps"][0] - nso)))
    assert tt <= 1e-6 and te <= 1e-6 and ee <= 1e-6
    assert np.max(np.abs(g["nsteps"][0] - nso)) <= 2


def test_hierarchy_size_limits(ctx):
    """Massless hierarchies at the perturbation kernel's edge: l_gamma = l_pol
    = l_nu = 60 gives N = 187 rows, the widest group (64 lanes of five rows,
    one mode per wavefront): four modes up to k = 0.05, sources to 1e-8 and
    C_l to 1e-6 of the oracle's.  l = 110 gives N = 337 rows, more than 64
    lanes of five hold: every entry point that integrates refuses it with
    CMB_E_UNSUPPORTED and leaves the outputs untouched."""
    import torch
    import oracle as O
    import paper_2602_15104_amd as L
    wl = W.small_case(n_k=4, n_tau=60, ell_max=40, k_max=0.05)
    wl.cosmo["N_nu_massless"] = 3.0
    wl.prec.update(ell_gamma=60, ell_pol=60, ell_nu=60)
    _say("case hierarchy l = 60")
    tab = L.Tables(wl.cosmo, wl.prec, wl.k, wl.n_tau)
    assert tab.state_rows() == 187
    g = run_gpu(ctx, [tab], wl.ell_max)
    r = O.solve(wl.cosmo, wl.prec, wl.k, wl.n_tau, wl.ell_max, True)
    assert np.all(g["status"] == 0) and np.all(r["status"] == 0)
    e = src_err(g["S"][0], r["S"])
    tt, te, ee = cl_err(g["Cl"][0], r["Cl"])
    _say("source err", e, "cl err", tt, te, ee, "steps", g["nsteps"][0], r["nsteps"])
    assert e <= 1e-8
    assert tt <= 1e-6 and te <= 1e-6 and ee <= 1e-6
    wl.prec.update(ell_gamma=110, ell_pol=110, ell_nu=110)
    _say("case hierarchy l = 110 (refused)")
    tab = L.Tables(wl.cosmo, wl.prec, wl.k, wl.n_tau)
    assert tab.state_rows() == 337
    n_k = len(wl.k)
    S = torch.full((1, n_k, 3, wl.n_tau), 7.0, dtype=torch.float64, device="cuda:0")
    st = torch.full((1, n_k), 9, dtype=torch.int32, device="cuda:0")
    H = torch.empty((1, n_k, wl.prec["max_steps"] + 1), dtype=torch.float64, device="cuda:0")
    for call in (lambda: ctx.perturb([tab], S, st), lambda: ctx.perturb_record([tab], S, st, H, st),
                 lambda: L.solve_batch(ctx, [tab], wl.ell_max)):
        with pytest.raises(L.CmbError) as ex:
            call()
        assert ex.value.name == "CMB_E_UNSUPPORTED"
    torch.cuda.synchronize()
    assert torch.all(S == 7.0) and torch.all(st == 9)


def test_config1_repeat_bitwise(ctx):
    """Two solves of the full-size TT/TE/EE workload after other kernels have
    used the GPU: every mode finishes and the results repeat bit for bit."""
    import paper_2602_15104_amd as L
    wl = W.config1()
    cosmos = W.perturbed_cosmologies(2, seed=99)
    for cc in cosmos:
        cc["N_nu_massless"] = 3.0
    tabs = [L.Tables(cc, wl.prec, wl.k, wl.n_tau) for cc in cosmos]
    a = run_gpu(ctx, tabs, wl.ell_max)
    b = run_gpu(ctx, tabs, wl.ell_max)
    assert np.all(a["status"] == 0) and np.all(b["status"] == 0)
    assert np.array_equal(a["S"], b["S"]) and np.array_equal(a["Cl"], b["Cl"])


def _gpu_pk(ctx, tab):
    import torch
    n_k, n_tau = len(tab.k), tab.n_tau
    S = torch.empty((1, n_k, 3, n_tau), dtype=torch.float64, device="cuda:0")
    st = torch.empty((1, n_k), dtype=torch.int32, device="cuda:0")
    Pk = torch.empty((1, n_k), dtype=torch.float64, device="cuda:0")
    ctx.perturb_pk([tab], S, st, Pk)
    torch.cuda.synchronize()
    return Pk[0].cpu().numpy(), st[0].cpu().numpy(), S[0].cpu().numpy()


@pytest.mark.parametrize("case", ["small", "small_massive", "config1", "config2"])
def test_matter_pk_parity(ctx, case):
    """Matter power spectrum today (App. B.4, eq. PK) from cmb_perturb_pk
    against the oracle (each mode integrated to a = 1), relative per mode
    <= 1e-8; the sources of the same call equal cmb_perturb's bitwise."""
    import oracle as O
    import paper_2602_15104_amd as L
    if case == "small":
        wl, idx = W.small_case(n_k=12, n_tau=60, ell_max=40, k_max=0.1), None
    elif case == "small_massive":
        wl, idx = _massive(W.small_case(n_k=8, n_tau=60, ell_max=40, k_max=0.1), 0.6, 3, 6), None
    elif case == "config1":
        wl, idx = W.config1(), np.array([0, 150, 399])
    else:
        wl, idx = W.config2(), np.array([0, 200])
    _say("case pk", case)
    tab = L.Tables(wl.cosmo, wl.prec, wl.k, wl.n_tau)
    Pg, st, Sg = _gpu_pk(ctx, tab)
    assert np.all(st == 0) and np.all(Pg > 0)
    ref = run_gpu(ctx, [tab], 2)
    assert np.array_equal(Sg, ref["S"][0])
    t_or = O.build_tables(wl.cosmo, wl.prec, wl.k, wl.n_tau)
    Po = O.matter_pk(t_or, idx)
    Pg_s = Pg if idx is None else Pg[idx]
    e = np.max(np.abs(Pg_s / Po - 1))
    _say("pk err", e)
    assert e <= 1e-8


# ---------------------------------------------------------------- transfer k-grid
def _gpu_on_grid(ctx, tabs, ell_max, S, kt):
    import torch
    B, n_tau = len(tabs), tabs[0].n_tau
    dS = S if isinstance(S, torch.Tensor) else torch.tensor(S, device="cuda:0")
    St = torch.empty((B, len(kt), 3, n_tau), dtype=torch.float64, device="cuda:0")
    D = torch.empty((B, 2, len(kt), ell_max - 1), dtype=torch.float64, device="cuda:0")
    C = torch.empty((B, 3, ell_max + 1), dtype=torch.float64, device="cuda:0")
    ctx.spectra_on_grid(tabs, ell_max, dS, kt, St, D, C)
    torch.cuda.synchronize()
    return St.cpu().numpy(), lk(D.cpu().numpy()), C.cpu().numpy()


def test_transfer_grid_interp_same_sources(ctx):
    """Spline stage alone: seeded random sources on a 50-mode grid, onto a
    transfer grid with ragged spacing, against the oracle's natural splines
    (relative to each (k~, type) row's largest value, <= 1e-12); C_ell of the
    interpolated sources against the oracle's projection of the same."""
    import oracle as O
    import paper_2602_15104_amd as L
    wl = W.small_case(n_k=50, n_tau=90, ell_max=50, k_max=0.1)
    tab = L.Tables(wl.cosmo, wl.prec, wl.k, wl.n_tau)
    t_or = O.build_tables(wl.cosmo, wl.prec, wl.k, wl.n_tau)
    kt = L.transfer_kgrid(1500, wl.k[0], wl.k[-1])
    assert kt[0] == wl.k[0] and kt[-1] == wl.k[-1]
    rng = np.random.Generator(np.random.PCG64(11))
    S = rng.standard_normal((1, len(wl.k), 3, wl.n_tau))
    _say("case interp", len(kt), "points")
    St, D, C = _gpu_on_grid(ctx, [tab], wl.ell_max, S, kt)
    So = O.interp_sources(wl.k, S[0], kt)
    e = src_err(St[0], So)
    _say("interp err", e)
    assert e <= 1e-12
    DT, DE = O.los(t_or, St[0], wl.ell_max, True, k=kt)
    for plane, ref in ((0, DT), (1, DE)):
        assert np.max(np.abs(D[0, plane] - ref)) <= 1e-9 * np.max(np.abs(ref))
    Co = O.cl(kt, D[0, 0], D[0, 1], wl.ell_max, True, wl.cosmo["A_s"], wl.cosmo["n_s"])
    np.testing.assert_allclose(C[0][:, 2:], Co[:, 2:], rtol=1e-12, atol=0)


@pytest.mark.parametrize("pol", [True, False])
def test_transfer_grid_full_parity(ctx, pol):
    """Whole path onto the transfer grid: each side integrates its own modes,
    interpolates its own sources onto k~ and projects there."""
    import oracle as O
    import paper_2602_15104_amd as L
    wl = W.small_case(n_k=24, n_tau=120, ell_max=120, k_max=0.05, polarization=pol)
    tab = L.Tables(wl.cosmo, wl.prec, wl.k, wl.n_tau)
    kt = L.transfer_kgrid(wl.ell_max * 3, wl.k[0], wl.k[-1])
    _say("case transfer small", pol, len(kt))
    g = run_gpu(ctx, [tab], wl.ell_max)
    St, D, C = _gpu_on_grid(ctx, [tab], wl.ell_max, g["S"], kt)
    r = O.solve(wl.cosmo, wl.prec, wl.k, wl.n_tau, wl.ell_max, pol)
    ro = O.spectra_on_grid(r["tables"], r["S"], kt, wl.ell_max, pol)
    e = src_err(St[0], ro["St"])
    tt, te, ee = cl_err(C[0], ro["Cl"])
    _say("source err", e, "cl err", tt, te, ee)
    assert e <= 1e-8 and tt <= 1e-6 and te <= 1e-6 and ee <= 1e-6


def test_transfer_grid_batch_and_errors(ctx):
    """Two cosmologies on one k grid: each result equals its solo call bit for
    bit.  Rejected: k~ outside the mode grid, not increasing, fewer than two
    points, and batches whose k grids differ."""
    import torch
    import paper_2602_15104_amd as L
    wl = W.small_case(n_k=16, n_tau=60, ell_max=30, k_max=0.05)
    cosmos = W.perturbed_cosmologies(2, seed=5)
    for cc in cosmos:
        cc["N_nu_massless"] = 3.0
    tabs = [L.Tables(cc, wl.prec, wl.k, wl.n_tau) for cc in cosmos]
    g = run_gpu(ctx, tabs, wl.ell_max)
    kt = L.transfer_kgrid(2500, wl.k[0], wl.k[-1])
    Sb, Db, Cb = _gpu_on_grid(ctx, tabs, wl.ell_max, g["S"], kt)
    S1, D1, C1 = _gpu_on_grid(ctx, [tabs[1]], wl.ell_max, g["S"][1:], kt)
    assert np.array_equal(Sb[1], S1[0]) and np.array_equal(Cb[1], C1[0])
    dS = torch.tensor(g["S"][:1], device="cuda:0")
    for bad in (np.array([wl.k[0] * 0.5, wl.k[-1]]), kt[::-1].copy(), kt[:1].copy(),
                np.array([wl.k[0], wl.k[-1] * 1.01])):
        with pytest.raises(L.CmbError):
            _gpu_on_grid(ctx, tabs[:1], wl.ell_max, dS, bad)
    other = L.Tables(cosmos[0], wl.prec, wl.k * 1.001, wl.n_tau)
    with pytest.raises(L.CmbError):
        _gpu_on_grid(ctx, [tabs[0], other], wl.ell_max, torch.tensor(g["S"], device="cuda:0"), kt)


def test_config1_transfer_grid(ctx):
    """Config 1 (400 modes, 2000 times, l <= 2500) on the App. A.2 transfer
    grid for l_max = 2500 (1699 points): C_ell against the stored oracle
    spectrum on the same grid (tests/golden/make_oracle_reference.py)."""
    import paper_2602_15104_amd as L
    ref = os.path.join(GOLD, "oracle_config1_transfer_cl.npy")
    assert os.path.exists(ref), "oracle golden missing: run tests/golden/make_oracle_reference.py"
    wl = W.config1()
    tab = L.Tables(wl.cosmo, wl.prec, wl.k, wl.n_tau)
    kt = L.transfer_kgrid(wl.ell_max, wl.k[0], wl.k[-1])
    _say("case config1 transfer", len(kt))
    g = run_gpu(ctx, [tab], wl.ell_max)
    St, D, C = _gpu_on_grid(ctx, [tab], wl.ell_max, g["S"], kt)
    tt, te, ee = cl_err(C[0], np.load(ref))
    _say("cl err", tt, te, ee)
    assert tt <= 1e-6 and te <= 1e-6 and ee <= 1e-6


# ---------------------------------------------------------------- three-region Bessel variant
def test_bessel3_table_parity(ctx):
    """The device-built table (Miller recurrence and root searches on the GPU)
    against the oracle's (scipy samples, its own searches), every l <= 300:
    x_start and x_5 to 1e-12 relative, samples to 1e-12 of each row's peak."""
    from oracle import bessel3 as B3
    xs, x5, tab = ctx.bessel3_table(300)
    T = B3.Table(300)
    e_s, e_5 = np.max(np.abs(xs / T.xs - 1)), np.max(np.abs(x5 / T.x5 - 1))
    err = np.max(np.abs(tab - T.tab), axis=1) / np.max(np.abs(T.tab), axis=1)
    _say("bessel3 table l<=300: x_start", e_s, "x_5", e_5, "samples", np.max(err))
    assert e_s < 1e-12 and e_5 < 1e-12 and np.max(err) < 1e-12


def test_bessel3_table_full_size_sampled(ctx):
    """l_max = 2500: every x_start and x_5, and the samples of a few rows."""
    from scipy.special import spherical_jn
    from oracle import bessel3 as B3
    xs, x5, tab = ctx.bessel3_table(2500)
    ells = np.arange(1, 2501)
    oxs, ox5 = B3.x_start(ells), B3.x_fifth_max(ells)
    assert np.max(np.abs(xs / oxs - 1)) < 1e-12 and np.max(np.abs(x5 / ox5 - 1)) < 1e-12
    for l in (1, 2, 777, 2499, 2500):
        dx = (ox5[l - 1] - oxs[l - 1]) / 4999
        ref = spherical_jn(l, oxs[l - 1] + dx * np.arange(5000))
        assert np.max(np.abs(tab[l - 1] - ref)) < 1e-12 * np.max(np.abs(ref)), l


def test_los_bessel3_same_sources(ctx):
    """The variant projection alone: seeded random sources, 30 modes up to
    k = 0.1 (x up to ~1400, all three regions), 300 output times (two per
    lane, ragged), l <= 150, against the oracle's scheme: Delta per k to 1e-9
    of its largest value, C_ell of the same Delta to 1e-12."""
    import torch
    import oracle as O
    import paper_2602_15104_amd as L
    from oracle import bessel3 as B3
    wl = W.small_case(n_k=30, n_tau=300, ell_max=150, k_max=0.1)
    tab = L.Tables(wl.cosmo, wl.prec, wl.k, wl.n_tau)
    t_or = O.build_tables(wl.cosmo, wl.prec, wl.k, wl.n_tau)
    rng = np.random.Generator(np.random.PCG64(17))
    S = rng.standard_normal((1, len(wl.k), 3, wl.n_tau))
    dS = torch.tensor(S, device="cuda:0")
    D = torch.empty((1, 2, len(wl.k), wl.ell_max - 1), dtype=torch.float64, device="cuda:0")
    C = torch.empty((1, 3, wl.ell_max + 1), dtype=torch.float64, device="cuda:0")
    ctx.los_bessel3([tab], wl.ell_max, dS, D)
    ctx.cl([tab], wl.ell_max, D, C)
    torch.cuda.synchronize()
    DT, DE = B3.los3(t_or, S[0], wl.ell_max, True, T=B3.Table(wl.ell_max))
    Dg = lk(D.cpu().numpy()[0])
    worst = 0.0
    for ik in range(len(wl.k)):
        for plane, ref in ((0, DT), (1, DE)):
            den = np.max(np.abs(ref[:, ik]))
            worst = max(worst, np.max(np.abs(Dg[plane][:, ik] - ref[:, ik])) / den)
    _say("los3 same sources: Delta err", worst)
    assert worst <= 1e-9
    Co = O.cl(t_or.k, Dg[0], Dg[1], wl.ell_max, True, wl.cosmo["A_s"], wl.cosmo["n_s"])
    np.testing.assert_allclose(C.cpu().numpy()[0][:, 2:], Co[:, 2:], rtol=1e-12, atol=0)


def test_los_bessel3_config1_error(ctx):
    """Measured accuracy of the scheme at config 1 (400 modes, 2000 times,
    l <= 2500): its C_ell against the exact recurrence's from the same GPU
    sources.  A measurement, bounded loosely (the scheme's Debye form carries
    a 1/(8x) phase error)."""
    import torch
    import paper_2602_15104_amd as L
    wl = W.config1()
    tab = L.Tables(wl.cosmo, wl.prec, wl.k, wl.n_tau)
    g = run_gpu(ctx, [tab], wl.ell_max)
    dS = torch.tensor(g["S"], device="cuda:0")
    D = torch.empty((1, 2, len(wl.k), wl.ell_max - 1), dtype=torch.float64, device="cuda:0")
    C = torch.empty((1, 3, wl.ell_max + 1), dtype=torch.float64, device="cuda:0")
    ctx.los_bessel3([tab], wl.ell_max, dS, D)
    ctx.cl([tab], wl.ell_max, D, C)
    torch.cuda.synchronize()
    tt, te, ee = cl_err(C.cpu().numpy()[0], g["Cl"][0])
    _say("config1 three-region vs exact: TT", tt, "TE", te, "EE", ee)
    assert tt < 5e-2 and te < 5e-2 and ee < 5e-2


# ---------------------------------------------------------------- lensing potential (Limber)
def _gpu_matter(ctx, tabs, want_pk=True):
    import torch
    B, n_k, n_tau = len(tabs), len(tabs[0].k), tabs[0].n_tau
    S = torch.empty((B, n_k, 3, n_tau), dtype=torch.float64, device="cuda:0")
    st = torch.empty((B, n_k), dtype=torch.int32, device="cuda:0")
    Pk = torch.empty((B, n_k), dtype=torch.float64, device="cuda:0") if want_pk else None
    Dm = torch.empty((B, n_k, n_tau), dtype=torch.float64, device="cuda:0")
    ctx.perturb_matter(tabs, S, st, Pk=Pk, Dm=Dm)
    torch.cuda.synchronize()
    return S, st, Pk, Dm


@pytest.mark.parametrize("case", ["small", "small_massive"])
def test_delta_m_and_limber_parity(ctx, case):
    """delta_m at the output times (cmb_perturb_matter) against the oracle's
    per mode (relative max-norm <= 1e-8), the sources equal cmb_perturb's
    bitwise, and C_l^psipsi (cmb_lensing_potential, l <= 400) against the
    oracle's Limber sum on its own delta_m (<= 1e-6)."""
    import torch
    import oracle as O
    import paper_2602_15104_amd as L
    from oracle import lensing as LN
    wl = W.small_case(n_k=24, n_tau=200, ell_max=40, k_min=1e-4, k_max=0.2)
    wl.prec["max_steps"] = 6000
    if case == "small_massive":
        wl = _massive(wl, 0.3, 4, 6)
    _say("case limber", case)
    tab = L.Tables(wl.cosmo, wl.prec, wl.k, wl.n_tau)
    S, st, Pk, Dm = _gpu_matter(ctx, [tab])
    ref = run_gpu(ctx, [tab], 2)
    assert np.array_equal(S.cpu().numpy()[0], ref["S"][0])
    t_or = O.build_tables(wl.cosmo, wl.prec, wl.k, wl.n_tau)
    So, Dmo, sto, nso = O.perturb_dm(t_or)
    assert np.all(st.cpu().numpy() == 0) and np.all(sto == 0)
    Dg = Dm.cpu().numpy()[0]
    e = max(np.max(np.abs(Dg[i] - Dmo[i])) / np.max(np.abs(Dmo[i])) for i in range(len(wl.k)))
    assert np.array_equal(Dg == 0, Dmo == 0)
    C = torch.empty((1, 401), dtype=torch.float64, device="cuda:0")
    ctx.lensing_potential([tab], 400, Dm, C)
    torch.cuda.synchronize()
    Cg = C.cpu().numpy()[0]
    Co = LN.limber_cl(t_or, Dmo, 400)
    ce = np.max(np.abs(Cg[2:] / Co[2:] - 1))
    _say("delta_m err", e, "Cpp err", ce)
    assert e <= 1e-8 and ce <= 1e-6 and np.all(Cg[:2] == 0)


def test_limber_same_input(ctx):
    """Limber stage alone on seeded random delta_m (two cosmologies on one k
    grid): against the oracle's sum to 1e-12, and each cosmology's result
    equals its solo call bit for bit."""
    import torch
    import paper_2602_15104_amd as L
    import oracle as O
    from oracle import lensing as LN
    wl = W.small_case(n_k=30, n_tau=300, ell_max=40, k_min=1e-4, k_max=0.5)
    cosmos = W.perturbed_cosmologies(2, seed=9)
    for cc in cosmos:
        cc["N_nu_massless"] = 3.0
    tabs = [L.Tables(cc, wl.prec, wl.k, wl.n_tau) for cc in cosmos]
    rng = np.random.Generator(np.random.PCG64(23))
    D = rng.standard_normal((2, len(wl.k), wl.n_tau))
    dD = torch.tensor(D, device="cuda:0")
    C = torch.empty((2, 3001), dtype=torch.float64, device="cuda:0")
    C1 = torch.empty((1, 3001), dtype=torch.float64, device="cuda:0")
    ctx.lensing_potential(tabs, 3000, dD, C)
    ctx.lensing_potential(tabs[1:], 3000, dD[1:], C1)
    torch.cuda.synchronize()
    Cg = C.cpu().numpy()
    assert np.array_equal(Cg[1], C1.cpu().numpy()[0])
    for i, cc in enumerate(cosmos):
        t_or = O.build_tables(cc, wl.prec, wl.k, wl.n_tau)
        Co = LN.limber_cl(t_or, D[i], 3000)
        nz = Co != 0
        assert np.array_equal(Cg[i] != 0, nz)
        assert np.max(np.abs(Cg[i][nz] / Co[nz] - 1)) < 1e-12
    other = L.Tables(cosmos[0], wl.prec, wl.k * 1.001, wl.n_tau)
    with pytest.raises(L.CmbError):
        ctx.lensing_potential([tabs[0], other], 3000, dD, C)


def test_limber_config1(ctx):
    """Config 1 at full size: C_l^psipsi for l <= 3000 from the GPU's delta_m
    against the oracle's Limber sum on the oracle's own delta_m of all 400
    modes (<= 1e-6)."""
    import torch
    import oracle as O
    import paper_2602_15104_amd as L
    from oracle import lensing as LN
    wl = W.config1()
    tab = L.Tables(wl.cosmo, wl.prec, wl.k, wl.n_tau)
    S, st, Pk, Dm = _gpu_matter(ctx, [tab], want_pk=False)
    C = torch.empty((1, 3001), dtype=torch.float64, device="cuda:0")
    ctx.lensing_potential([tab], 3000, Dm, C)
    torch.cuda.synchronize()
    t_or = O.build_tables(wl.cosmo, wl.prec, wl.k, wl.n_tau)
    So, Dmo, sto, nso = O.perturb_dm(t_or)
    Co = LN.limber_cl(t_or, Dmo, 3000)
    Cg = C.cpu().numpy()[0]
    ce = np.max(np.abs(Cg[2:] / Co[2:] - 1))
    l = np.arange(3001)
    _say("config1 Cpp err", ce, "peak [l(l+1)]^2 C/2pi", np.max((l * (l + 1.0)) ** 2 * Cg / (2 * math.pi)))
    assert ce <= 1e-6


# ---------------------------------------------------------------- lensed spectra
def _toy_lensing_inputs(L, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    ls = np.arange(L + 1, dtype=np.float64)
    Cl = np.zeros((3, L + 1))
    ph = rng.uniform(0, 2 * math.pi)
    Cl[0, 2:] = (1.0 + 0.5 * np.cos(ls[2:] / 30.0 + ph)) / ls[2:] ** 2
    Cl[2, 2:] = 0.05 * (1.0 + 0.8 * np.sin(ls[2:] / 30.0 + ph)) / ls[2:] ** 2
    Cl[1, 2:] = 0.1 * np.cos(ls[2:] / 30.0 + ph) / ls[2:] ** 2
    Cpp = np.zeros(L + 1)
    Cpp[2:] = rng.uniform(0.5, 1.5) * 1e-6 / ls[2:] ** 4 * np.exp(-((ls[2:] - 150.0) / 80.0) ** 2)
    return Cl, Cpp


def test_lensed_cl_same_input(ctx):
    """Lensed TT/TE/EE/BB (cmb_lensed_cl) on analytic spectra, two
    cosmologies, L = 600, l <= 450: against the oracle's correlation-function
    lensing, each lensing change to 1e-9 of its largest value, and each
    cosmology's result equals its solo call bit for bit."""
    import torch
    from oracle import lensing as LN
    L, lmax, n_mu = 600, 450, 900
    inp = [_toy_lensing_inputs(L, s) for s in (1, 2)]
    dCl = torch.tensor(np.stack([a for a, _ in inp]), device="cuda:0")
    dP = torch.tensor(np.stack([b for _, b in inp]), device="cuda:0")
    out = torch.empty((2, 4, lmax + 1), dtype=torch.float64, device="cuda:0")
    solo = torch.empty((1, 4, lmax + 1), dtype=torch.float64, device="cuda:0")
    ctx.lensed_cl(dCl, dP, lmax, out, n_mu=n_mu)
    ctx.lensed_cl(dCl[1:], dP[1:], lmax, solo, n_mu=n_mu)
    torch.cuda.synchronize()
    g = out.cpu().numpy()
    assert np.array_equal(g[1], solo.cpu().numpy()[0])
    for c in range(2):
        o = LN.lensed_cl(inp[c][0], inp[c][1], lmax, n_mu)
        base = np.zeros_like(o)
        base[:3] = inp[c][0][:, :lmax + 1]
        for i in range(4):
            dg, do = g[c, i] - base[i], o[i] - base[i]
            e = np.max(np.abs(dg - do)) / np.max(np.abs(do))
            _say("lensed same input c", c, "spectrum", i, "err", e)
            assert e < 1e-9
        assert np.all(g[c][:, :2] == 0)


def test_lensed_cl_config1(ctx):
    """The whole lensed path at config 1: GPU unlensed C_l (l <= 2500),
    delta_m and the Limber C_l^psipsi, then lensed spectra for l <= 2000
    (n_mu = 3700), against the oracle's chain on its own inputs (the stored
    oracle C_l and its own delta_m): lensed TT, EE to 1e-6, TE to 1e-6 of
    sqrt(TT EE), BB to 1e-6 of its peak; the lensing change of TT reaches the
    percent level at high l and BB/EE ~ 1e-2 at l ~ 1000."""
    import torch
    import oracle as O
    import paper_2602_15104_amd as L_
    from oracle import lensing as LN
    ref = os.path.join(GOLD, "oracle_config1_cl.npy")
    assert os.path.exists(ref), "oracle golden missing: run tests/golden/make_oracle_reference.py"
    wl = W.config1()
    Lu, lmax, n_mu = wl.ell_max, 2000, 3700
    tab = L_.Tables(wl.cosmo, wl.prec, wl.k, wl.n_tau)
    S, st, _, Dm = _gpu_matter(ctx, [tab], want_pk=False)
    D = torch.empty((1, 2, len(wl.k), Lu - 1), dtype=torch.float64, device="cuda:0")
    C = torch.empty((1, 3, Lu + 1), dtype=torch.float64, device="cuda:0")
    P = torch.empty((1, Lu + 1), dtype=torch.float64, device="cuda:0")
    ctx.los([tab], Lu, S, D)
    ctx.cl([tab], Lu, D, C)
    ctx.lensing_potential([tab], Lu, Dm, P)
    out = torch.empty((1, 4, lmax + 1), dtype=torch.float64, device="cuda:0")
    ctx.lensed_cl(C, P, lmax, out, n_mu=n_mu)
    torch.cuda.synchronize()
    g = out.cpu().numpy()[0]
    t_or = O.build_tables(wl.cosmo, wl.prec, wl.k, wl.n_tau)
    So, Dmo, sto, nso = O.perturb_dm(t_or)
    Co = np.load(ref)
    Po = LN.limber_cl(t_or, Dmo, Lu)
    o = LN.lensed_cl(Co, Po, lmax, n_mu)
    tt = np.max(np.abs(g[0, 2:] / o[0, 2:] - 1))
    ee = np.max(np.abs(g[2, 2:] / o[2, 2:] - 1))
    te = np.max(np.abs(g[1, 2:] - o[1, 2:]) / np.sqrt(o[0, 2:] * o[2, 2:]))
    bb = np.max(np.abs(g[3, 2:] - o[3, 2:])) / np.max(np.abs(o[3, 2:]))
    lens_tt = np.max(np.abs(o[0, 1500:] / Co[0, 1500:lmax + 1] - 1))
    _say("config1 lensed: TT", tt, "TE", te, "EE", ee, "BB", bb, "| lensing change of TT at l>=1500", lens_tt,
         "BB/EE at 1000", o[3, 1000] / o[2, 1000])
    assert tt < 1e-6 and te < 1e-6 and ee < 1e-6 and bb < 1e-6
    assert 0.01 < lens_tt < 0.5 and 1e-3 < o[3, 1000] / o[2, 1000] < 0.1


# ---------------------------------------------------------------- parameter derivatives
def test_record_replay_bitwise(ctx):
    """cmb_perturb_record equals cmb_perturb bit for bit and records one entry
    per accepted step; cmb_perturb_replay of the same tables reproduces the
    sources bit for bit; replaying another cosmology on these steps runs."""
    import torch
    import paper_2602_15104_amd as L
    wl = W.small_case(n_k=20, n_tau=100, ell_max=40, k_max=0.1)
    cosmos = W.perturbed_cosmologies(2, seed=13)
    for cc in cosmos:
        cc["N_nu_massless"] = 3.0
    tabs = [L.Tables(cc, wl.prec, wl.k, wl.n_tau) for cc in cosmos]
    cap = wl.prec["max_steps"] + 1
    S = torch.empty((2, len(wl.k), 3, wl.n_tau), dtype=torch.float64, device="cuda:0")
    st = torch.empty((2, len(wl.k)), dtype=torch.int32, device="cuda:0")
    ns = torch.empty_like(st)
    H = torch.empty((2, len(wl.k), cap), dtype=torch.float64, device="cuda:0")
    Hn = torch.empty_like(st)
    ctx.perturb_record(tabs, S, st, H, Hn, nsteps=ns)
    S2 = torch.empty_like(S)
    st2 = torch.empty_like(st)
    ns2 = torch.empty_like(st)
    ctx.perturb_replay(tabs, H, Hn, S2, st2, nsteps=ns2)
    S3 = torch.empty_like(S)
    ctx.perturb_replay(tabs[::-1], H, Hn, S3, st2)
    torch.cuda.synchronize()
    ref = run_gpu(ctx, tabs, 2)
    assert np.array_equal(S.cpu().numpy(), ref["S"]) and np.all(st.cpu().numpy() == 0)
    assert np.array_equal(S2.cpu().numpy(), ref["S"])
    assert np.array_equal(ns2.cpu().numpy(), Hn.cpu().numpy())
    assert np.all(Hn.cpu().numpy() <= ns.cpu().numpy())
    assert np.all(np.isfinite(S3.cpu().numpy()))


def _ck_buffers(n, n_k, cap, every, rows):
    import torch
    n_slots = (cap - 1) // every + 1
    return torch.full((n, n_k, n_slots, 1 + 2 * rows), float("nan"), dtype=torch.float64, device="cuda:0")


@pytest.mark.parametrize("massive", [False, True])
def test_checkpoint_segments_bitwise(ctx, massive):
    """Trajectory checkpoints every 16 accepted steps: recording with
    checkpoints equals cmb_perturb bit for bit, a replay writes the same
    checkpoints, and replaying every segment from its checkpoint (in reverse
    order, into one buffer) rebuilds the replay's sources bit for bit, each
    segment writing exactly the outputs its steps reach."""
    import torch
    import paper_2602_15104_amd as L
    wl = W.small_case(n_k=20, n_tau=100, ell_max=40, k_max=0.1)
    if massive:
        wl = _massive(wl, 0.06, 3, 6)
        cosmos = [wl.cosmo]
    else:
        cosmos = W.perturbed_cosmologies(2, seed=17)
        for cc in cosmos:
            cc["N_nu_massless"] = 3.0
    _say("case checkpoint segments, massive =", massive)
    tabs = [L.Tables(cc, wl.prec, wl.k, wl.n_tau) for cc in cosmos]
    n, n_k, E = len(tabs), len(wl.k), 16
    rows = tabs[0].state_rows()
    cap = wl.prec["max_steps"] + 1
    S = torch.empty((n, n_k, 3, wl.n_tau), dtype=torch.float64, device="cuda:0")
    st = torch.empty((n, n_k), dtype=torch.int32, device="cuda:0")
    H = torch.empty((n, n_k, cap), dtype=torch.float64, device="cuda:0")
    Hn = torch.empty_like(st)
    ck = _ck_buffers(n, n_k, cap, E, rows)
    ctx.perturb_checkpoint(tabs, H, Hn, E, ck, S, st)
    S2 = torch.empty_like(S)
    st2 = torch.empty_like(st)
    ck2 = _ck_buffers(n, n_k, cap, E, rows)
    ctx.perturb_checkpoint(tabs, H, Hn, E, ck2, S2, st2, replay=True)
    torch.cuda.synchronize()
    ref = run_gpu(ctx, tabs, 2)
    hn = Hn.cpu().numpy()
    ckh = ck.cpu().numpy()
    assert np.all(st.cpu().numpy() == 0) and np.all(st2.cpu().numpy() == 0)
    assert np.array_equal(S.cpu().numpy(), ref["S"]) and np.array_equal(S2.cpu().numpy(), ref["S"])
    assert np.array_equal(ckh, ck2.cpu().numpy(), equal_nan=True)
    n_seg = int(hn.max()) // E + 1
    ex = [tb.export() for tb in tabs]
    for i in range(n):
        for ik in range(n_k):
            used = hn[i, ik] // E + 1  # slots 0 .. hn // E are written, the rest untouched
            assert np.all(np.isfinite(ckh[i, ik, :used])) and np.all(np.isnan(ckh[i, ik, used:]))
            assert ckh[i, ik, 0, 0] == ex[i]["lna_start"][ik] and np.all(np.diff(ckh[i, ik, :used, 0]) > 0)
    Sseg = torch.full_like(S, float("nan"))
    ns = torch.empty_like(st)
    for seg in reversed(range(n_seg)):
        one = torch.full_like(S, float("nan"))
        ctx.perturb_segment(tabs, H, Hn, E, ck, seg, one, st2, nsteps=ns)
        ctx.perturb_segment(tabs, H, Hn, E, ck, seg, Sseg, st2)
        torch.cuda.synchronize()
        assert np.all(st2.cpu().numpy() == 0)
        want_ns = np.clip(hn - seg * E, 0, E)
        assert np.array_equal(ns.cpu().numpy(), want_ns), seg
        o = one.cpu().numpy()
        for i in range(n):
            for ik in range(n_k):
                if hn[i, ik] <= seg * E:
                    assert np.all(np.isnan(o[i, ik]))
                    continue
                t_a = ckh[i, ik, seg, 0]
                t_b = ckh[i, ik, seg + 1, 0] if (seg + 1) * E < hn[i, ik] else np.inf
                lo = ex[i]["lna_src"]
                inside = (lo <= t_b) & ((lo > t_a) if seg > 0 else True)
                assert np.array_equal(o[i, ik][:, inside], ref["S"][i, ik][:, inside]), (seg, i, ik)
                assert np.all(np.isnan(o[i, ik][:, ~inside])), (seg, i, ik)
    assert np.array_equal(Sseg.cpu().numpy(), ref["S"])


def test_checkpoint_states_parity(ctx):
    """The checkpoints of a replay of the oracle's own recorded steps against
    the oracle: ln a bit for bit (the oracle's accepted step ends), the state
    rows to 1e-8 of each row's largest magnitude, and the carried stage
    derivative against the oracle's right-hand side at its state to 1e-7
    (the last stage's derivative is (Y - R)/(h gamma), whose rounding the
    division by h gamma enlarges)."""
    import torch
    import oracle as O
    import paper_2602_15104_amd as L
    wl = W.small_case(n_k=6, n_tau=60, ell_max=20, k_max=0.1)
    wl.cosmo["N_nu_massless"] = 3.0
    E = 8
    t_or = O.build_tables(wl.cosmo, wl.prec, wl.k, wl.n_tau)
    _, st_o, _, hist, hn = O.perturb_hist(t_or)
    assert np.all(st_o == 0)
    tab = L.Tables(wl.cosmo, wl.prec, wl.k, wl.n_tau)
    rows = tab.state_rows()
    cap = hist.shape[1]
    n_k = len(wl.k)
    H = torch.tensor(hist[None], dtype=torch.float64, device="cuda:0")
    Hn = torch.tensor(hn[None], dtype=torch.int32, device="cuda:0")
    S = torch.empty((1, n_k, 3, wl.n_tau), dtype=torch.float64, device="cuda:0")
    st = torch.empty((1, n_k), dtype=torch.int32, device="cuda:0")
    ck = _ck_buffers(1, n_k, cap, E, rows)
    ctx.perturb_checkpoint([tab], H, Hn, E, ck, S, st, replay=True)
    torch.cuda.synchronize()
    ckh = ck.cpu().numpy()[0]
    assert np.all(st.cpu().numpy() == 0)
    order = O.library_row_order(t_or.prec, 0)
    assert len(order) == rows
    ey = ek = 0.0
    for ik in range(n_k):
        k, lna0 = float(t_or.k[ik]), float(t_or.lna_i[ik])
        acc = O.perturb_one(t_or, k, lna0, [], acc_cap=cap)["accepted_lna"]
        assert len(acc) == hn[ik]
        times = np.concatenate([[lna0], acc[E - 1::E]])
        assert np.array_equal(ckh[ik, :len(times), 0], times), ik
        Y = O.perturb_one(t_or, k, lna0, times, want_y=True)["y"]
        F = np.array([O.rhs(t_or, k, float(tm), y) for tm, y in zip(times, Y)])
        yg, fg = ckh[ik, :len(times), 1:1 + rows], ckh[ik, :len(times), 1 + rows:]
        yo, fo = Y[:, order], F[:, order]
        ey = max(ey, float(np.max(np.abs(yg - yo) / (np.max(np.abs(yo), axis=0) + 1e-300))))
        ek = max(ek, float(np.max(np.abs(fg - fo) / (np.max(np.abs(fo), axis=0) + 1e-300))))
    _say("checkpoint state err", ey, "stage derivative err", ek)
    assert ey <= 1e-8 and ek <= 1e-7


@pytest.mark.parametrize("order", [4, 2])
def test_jacobian_parity(ctx, order):
    """cmb_jacobian against the oracle's frozen-step derivatives for two
    cosmologies (16 modes, l <= 120): every parameter's row to 1e-6 of its
    largest value; the ln A_s row is C_l itself."""
    import torch
    import oracle as O
    import paper_2602_15104_amd as L
    wl = W.small_case(n_k=16, n_tau=150, ell_max=120, k_max=0.1)
    cosmos = W.perturbed_cosmologies(2, seed=21)
    for cc in cosmos:
        cc["N_nu_massless"] = 3.0
    tabs = [L.Tables(cc, wl.prec, wl.k, wl.n_tau) for cc in cosmos]
    lm = wl.ell_max
    C = torch.empty((2, 3, lm + 1), dtype=torch.float64, device="cuda:0")
    J = torch.empty((2, 6, 3, lm + 1), dtype=torch.float64, device="cuda:0")
    st = torch.empty((2, len(wl.k)), dtype=torch.int32, device="cuda:0")
    ctx.jacobian(tabs, lm, C, J, st, rel=1e-4, order=order)
    torch.cuda.synchronize()
    Cg, Jg = C.cpu().numpy(), J.cpu().numpy()
    assert np.all(st.cpu().numpy() == 0)
    for i, cc in enumerate(cosmos):
        Co, Jo, sto = O.jacobian(cc, wl.prec, wl.k, wl.n_tau, lm, True, rel=1e-4, order=order)
        assert np.array_equal(Jg[i, 3], Cg[i])
        for p in range(6):
            m = np.max(np.abs(Jo[p][:, 2:]))
            e = np.max(np.abs(Jg[i, p][:, 2:] - Jo[p][:, 2:])) / m
            _say("jacobian order", order, "cosmology", i, "param", p, "err", e)
            assert e < 1e-6, (i, p, e)


def test_jacobian_config1(ctx):
    """Config 1 (400 modes, 2000 times, l <= 2500), fiducial cosmology:
    cmb_jacobian (five-point, rel 1e-4) against the stored oracle derivatives
    (tests/golden/make_oracle_reference.py), each row to 1e-6 of its largest
    value."""
    import torch
    import paper_2602_15104_amd as L
    ref = os.path.join(GOLD, "oracle_config1_jacobian.npy")
    assert os.path.exists(ref), "oracle golden missing: run tests/golden/make_oracle_reference.py"
    wl = W.config1()
    tab = L.Tables(wl.cosmo, wl.prec, wl.k, wl.n_tau)
    lm = wl.ell_max
    C = torch.empty((1, 3, lm + 1), dtype=torch.float64, device="cuda:0")
    J = torch.empty((1, 6, 3, lm + 1), dtype=torch.float64, device="cuda:0")
    st = torch.empty((1, len(wl.k)), dtype=torch.int32, device="cuda:0")
    ctx.jacobian([tab], lm, C, J, st, rel=1e-4, order=4)
    torch.cuda.synchronize()
    Jg, Jo = J.cpu().numpy()[0], np.load(ref)
    assert np.all(st.cpu().numpy() == 0)
    for p in range(6):
        m = np.max(np.abs(Jo[p][:, 2:]))
        e = np.max(np.abs(Jg[p][:, 2:] - Jo[p][:, 2:])) / m
        _say("config1 jacobian param", p, "err", e)
        assert e < 1e-6


# ---------------------------------------------------------------- spectrum-side adjoint
def test_spectra_adjoint_parity(ctx):
    """cmb_spectra_adjoint on seeded sources and seeded dL/dC_l (40 modes to
    k = 0.1, 300 output times, l <= 150): against the oracle's transposed
    quadrature and projection, per (k, type) to 1e-9 of its largest value."""
    import torch
    import oracle as O
    import paper_2602_15104_amd as L
    wl = W.small_case(n_k=40, n_tau=300, ell_max=150, k_max=0.1)
    tab = L.Tables(wl.cosmo, wl.prec, wl.k, wl.n_tau)
    t_or = O.build_tables(wl.cosmo, wl.prec, wl.k, wl.n_tau)
    rng = np.random.Generator(np.random.PCG64(31))
    S = rng.standard_normal((1, len(wl.k), 3, wl.n_tau))
    gC = rng.standard_normal((1, 3, wl.ell_max + 1))
    dS = torch.tensor(S, device="cuda:0")
    D = torch.empty((1, 2, len(wl.k), wl.ell_max - 1), dtype=torch.float64, device="cuda:0")
    gS = torch.empty_like(dS)
    ctx.los([tab], wl.ell_max, dS, D)
    ctx.spectra_adjoint([tab], wl.ell_max, D, torch.tensor(gC, device="cuda:0"), gS)
    torch.cuda.synchronize()
    DT, DE = O.los(t_or, S[0], wl.ell_max, True)
    GT, GE = O.cl_adjoint(t_or.k, DT, DE, gC[0], wl.ell_max, True, wl.cosmo["A_s"], wl.cosmo["n_s"])
    go = O.los_adjoint(t_or, GT, GE, wl.ell_max, True)
    e = src_err(gS.cpu().numpy()[0], go)
    _say("spectra adjoint err", e)
    assert e <= 1e-9


def test_spectra_adjoint_dot_product_config1(ctx):
    """Config 1 size (400 modes, 2000 times, l <= 2500): for the quadratic
    map S -> L = sum gC C_l(S), <dL/dS, V> equals the central difference of L
    along a seeded direction V (exact for a quadratic up to rounding)."""
    import torch
    import paper_2602_15104_amd as L
    wl = W.config1()
    tab = L.Tables(wl.cosmo, wl.prec, wl.k, wl.n_tau)
    g = run_gpu(ctx, [tab], wl.ell_max)
    S = torch.tensor(g["S"], device="cuda:0")
    rng = np.random.Generator(np.random.PCG64(37))
    V = torch.tensor(rng.standard_normal(g["S"].shape) * np.abs(g["S"]).max(axis=-1, keepdims=True), device="cuda:0")
    gC = torch.tensor(rng.standard_normal((1, 3, wl.ell_max + 1)) / np.maximum(np.abs(g["Cl"]), 1e-30),
                      device="cuda:0")
    D = torch.empty((1, 2, len(wl.k), wl.ell_max - 1), dtype=torch.float64, device="cuda:0")
    C = torch.empty((1, 3, wl.ell_max + 1), dtype=torch.float64, device="cuda:0")

    def loss(Sx):
        ctx.los([tab], wl.ell_max, Sx, D)
        ctx.cl([tab], wl.ell_max, D, C)
        torch.cuda.synchronize()
        return float((gC[:, :, 2:] * C[:, :, 2:]).sum().item())

    e = 1e-3
    fd = (loss(S + e * V) - loss(S - e * V)) / (2 * e)
    ctx.los([tab], wl.ell_max, S, D)
    gS = torch.empty_like(S)
    ctx.spectra_adjoint([tab], wl.ell_max, D, gC, gS)
    torch.cuda.synchronize()
    ad = float((gS * V).sum().item())
    _say("config1 adjoint dot product", ad, fd, ad / fd - 1)
    assert abs(ad / fd - 1) < 1e-8


# ---------------------------------------------------------------- transposed sources
@pytest.mark.parametrize("case", ["pol", "nopol", "massive"])
def test_sources_adjoint_parity(ctx, case):
    """cmb_sources_adjoint on seeded dL/dS (6 modes, 40 output times) against
    the oracle's transpose of its own source map, built from unit vectors:
    every (mode, time) row vector to 1e-10 of its largest entry; zero before
    each mode's start."""
    import torch
    import oracle as O
    import paper_2602_15104_amd as L
    if case == "massive":
        wl = _massive(W.small_case(n_k=6, n_tau=40, ell_max=20, k_max=0.1), 0.06, 3, 5)
    else:
        wl = W.small_case(n_k=6, n_tau=40, ell_max=20, k_max=0.1, polarization=(case == "pol"), ell_g=10)
    tab = L.Tables(wl.cosmo, wl.prec, wl.k, wl.n_tau)
    t_or = O.build_tables(wl.cosmo, wl.prec, wl.k, wl.n_tau)
    rng = np.random.Generator(np.random.PCG64(67))
    gS = rng.standard_normal((1, len(wl.k), 3, wl.n_tau))
    N = tab.state_rows()
    gY = torch.full((1, len(wl.k), wl.n_tau, N), float("nan"), dtype=torch.float64, device="cuda:0")
    ctx.sources_adjoint([tab], torch.tensor(gS, device="cuda:0"), gY)
    torch.cuda.synchronize()
    g = gY.cpu().numpy()[0]
    o = O.sources_adjoint(t_or, gS[0])
    assert g.shape == o.shape
    worst = 0.0
    for ik in range(len(wl.k)):
        for j in range(wl.n_tau):
            m = np.max(np.abs(o[ik, j]))
            if m == 0.0:
                assert np.all(g[ik, j] == 0.0), (ik, j)
                continue
            worst = max(worst, float(np.max(np.abs(g[ik, j] - o[ik, j])) / m))
    _say("sources adjoint", case, "err", worst)
    assert worst <= 1e-10


def test_sources_adjoint_config1_sampled(ctx):
    """Config 1 size (400 modes, 2000 output times, 79 rows; the launch the
    bench times): cmb_sources_adjoint on seeded dL/dS against the oracle at 60
    seeded (mode, time) points, each row vector to 1e-10 of its largest entry;
    every point before its mode's start is zero."""
    import torch
    import oracle as O
    import paper_2602_15104_amd as L
    wl = W.config1()
    tab = L.Tables(wl.cosmo, wl.prec, wl.k, wl.n_tau)
    t_or = O.build_tables(wl.cosmo, wl.prec, wl.k, wl.n_tau)
    rng = np.random.Generator(np.random.PCG64(79))
    gS = rng.standard_normal((1, len(wl.k), 3, wl.n_tau))
    N = tab.state_rows()
    gY = torch.empty((1, len(wl.k), wl.n_tau, N), dtype=torch.float64, device="cuda:0")
    ctx.sources_adjoint([tab], torch.tensor(gS, device="cuda:0"), gY)
    torch.cuda.synchronize()
    pts = [(int(rng.integers(len(wl.k))), int(rng.integers(wl.n_tau))) for _ in range(60)]
    o = O.sources_adjoint(t_or, gS[0], points=pts)
    worst = 0.0
    for ik, j in pts:
        g = gY[0, ik, j].cpu().numpy()
        m = np.max(np.abs(o[ik, j]))
        if m == 0.0:
            assert np.all(g == 0.0)
            continue
        worst = max(worst, float(np.max(np.abs(g - o[ik, j])) / m))
    _say("config1 sources adjoint sampled err", worst)
    assert worst <= 1e-10


def test_sources_adjoint_chain(ctx):
    """The reverse sweep's first three steps chained on seeded sources and
    seeded dL/dC_l: dL/dC_l -> dL/dS (cmb_spectra_adjoint at the projection of
    those sources) -> dL/dy (cmb_sources_adjoint) for two cosmologies, against
    the oracle's own projection and transposes of the same inputs."""
    import torch
    import oracle as O
    import paper_2602_15104_amd as L
    wl = W.small_case(n_k=5, n_tau=40, ell_max=30, k_max=0.05)
    cosmos = W.perturbed_cosmologies(2, seed=71)
    for cc in cosmos:
        cc["N_nu_massless"] = 3.0
    tabs = [L.Tables(cc, wl.prec, wl.k, wl.n_tau) for cc in cosmos]
    rng = np.random.Generator(np.random.PCG64(73))
    S = rng.standard_normal((2, len(wl.k), 3, wl.n_tau))
    gC = rng.standard_normal((2, 3, wl.ell_max + 1))
    D = torch.empty((2, 2, len(wl.k), wl.ell_max - 1), dtype=torch.float64, device="cuda:0")
    ctx.los(tabs, wl.ell_max, torch.tensor(S, device="cuda:0"), D)
    gS = torch.empty((2, len(wl.k), 3, wl.n_tau), dtype=torch.float64, device="cuda:0")
    ctx.spectra_adjoint(tabs, wl.ell_max, D, torch.tensor(gC, device="cuda:0"), gS)
    N = tabs[0].state_rows()
    gY = torch.empty((2, len(wl.k), wl.n_tau, N), dtype=torch.float64, device="cuda:0")
    ctx.sources_adjoint(tabs, gS, gY)
    torch.cuda.synchronize()
    gYg = gY.cpu().numpy()
    for i, cc in enumerate(cosmos):
        t_or = O.build_tables(cc, wl.prec, wl.k, wl.n_tau)
        DT, DE = O.los(t_or, S[i], wl.ell_max, True)
        GT, GE = O.cl_adjoint(t_or.k, DT, DE, gC[i], wl.ell_max, True, cc["A_s"], cc["n_s"])
        go = O.los_adjoint(t_or, GT, GE, wl.ell_max, True)
        yo = O.sources_adjoint(t_or, go)
        e = float(np.max(np.abs(gYg[i] - yo)) / np.max(np.abs(yo)))
        _say("chain cosmology", i, "err", e)
        assert e <= 1e-9


# ---------------------------------------------------------------- torch.autograd exposure
def test_autograd_spectra_from_sources(ctx):
    """spectra_from_sources for two cosmologies (40 modes to k = 0.1, 300
    output times, l <= 150): the forward pass equals cmb_los + cmb_cl and the
    gradient of sum gC C_l equals cmb_spectra_adjoint, bit for bit; the
    gradient matches the oracle's transposed quadrature and projection per
    (k, type) to 1e-9 of its largest value."""
    import torch
    import oracle as O
    import paper_2602_15104_amd as L
    from paper_2602_15104_amd.autograd import spectra_from_sources
    wl = W.small_case(n_k=40, n_tau=300, ell_max=150, k_max=0.1)
    cosmos = W.perturbed_cosmologies(2, seed=41)
    tabs = [L.Tables(c, wl.prec, wl.k, wl.n_tau) for c in cosmos]
    rng = np.random.Generator(np.random.PCG64(43))
    S0 = rng.standard_normal((2, len(wl.k), 3, wl.n_tau))
    gC0 = rng.standard_normal((2, 3, wl.ell_max + 1))
    S = torch.tensor(S0, device="cuda:0", requires_grad=True)
    gC = torch.tensor(gC0, device="cuda:0")
    Cl = spectra_from_sources(ctx, tabs, wl.ell_max, S)
    (Cl * gC).sum().backward()
    D = torch.empty((2, 2, len(wl.k), wl.ell_max - 1), dtype=torch.float64, device="cuda:0")
    C2 = torch.empty((2, 3, wl.ell_max + 1), dtype=torch.float64, device="cuda:0")
    Sd = S.detach().clone()
    ctx.los(tabs, wl.ell_max, Sd, D)
    ctx.cl(tabs, wl.ell_max, D, C2)
    gS = torch.empty_like(Sd)
    ctx.spectra_adjoint(tabs, wl.ell_max, D, gC, gS)
    torch.cuda.synchronize()
    assert torch.equal(Cl.detach(), C2)
    assert torch.equal(S.grad, gS)
    G = S.grad.cpu().numpy()
    for i, c in enumerate(cosmos):
        t_or = O.build_tables(c, wl.prec, wl.k, wl.n_tau)
        DT, DE = O.los(t_or, S0[i], wl.ell_max, True)
        GT, GE = O.cl_adjoint(t_or.k, DT, DE, gC0[i], wl.ell_max, True, c["A_s"], c["n_s"])
        go = O.los_adjoint(t_or, GT, GE, wl.ell_max, True)
        e = src_err(G[i], go)
        _say("autograd spectra adjoint cosmology", i, "err", e)
        assert e <= 1e-9


def test_autograd_cl_of_params(ctx):
    """cl_of_params for two cosmologies (16 modes, l <= 120): C_l equals
    cmb_solve's and the gradient of sum gC C_l with respect to (h, omega_b,
    omega_cdm, ln A_s, n_s, tau_reio) equals cmb_gradient's, bit for bit (the
    backward pass is that call); against the oracle's frozen-step derivatives
    contracted with the same gC, each parameter to 1e-4 of
    sum |gC| |dC/dtheta|."""
    import torch
    import oracle as O
    import paper_2602_15104_amd as L
    from paper_2602_15104_amd import autograd as AG
    wl = W.small_case(n_k=16, n_tau=150, ell_max=120, k_max=0.1)
    cosmos = W.perturbed_cosmologies(2, seed=21)
    for cc in cosmos:
        cc["N_nu_massless"] = 3.0
    th = [[c["h"], c["omega_b"], c["omega_cdm"], math.log(c["A_s"]), c["n_s"], c["tau_reio"]] for c in cosmos]
    theta = torch.tensor(th, dtype=torch.float64, requires_grad=True)
    lm = wl.ell_max
    rng = np.random.Generator(np.random.PCG64(47))
    gC0 = rng.standard_normal((2, 3, lm + 1))
    gC0[:, :, :2] = 0.0
    C = AG.cl_of_params(ctx, theta, cosmos[0], wl.prec, wl.k, wl.n_tau, lm)
    (C * torch.tensor(gC0, device="cuda:0")).sum().backward()
    g = theta.grad.numpy()
    # the same cosmologies through cmb_solve and cmb_gradient directly
    exact = [AG._cosmo_at(cosmos[0], row) for row in th]
    tabs = [L.Tables(c, wl.prec, wl.k, wl.n_tau) for c in exact]
    out = L.solve_batch(ctx, tabs, lm, keep_S=False, keep_Delta=False)
    C2 = torch.empty((2, 3, lm + 1), dtype=torch.float64, device="cuda:0")
    G2 = torch.empty((2, 6), dtype=torch.float64, device="cuda:0")
    st = torch.empty((2, len(wl.k)), dtype=torch.int32, device="cuda:0")
    ctx.gradient(tabs, lm, torch.tensor(gC0, device="cuda:0"), C2, G2, st, rel=1e-4)
    torch.cuda.synchronize()
    assert torch.equal(C.detach(), out["Cl"]) and torch.equal(C2, out["Cl"])
    assert np.array_equal(g, G2.cpu().numpy())
    for i, c in enumerate(exact):
        _, Jo, _ = O.jacobian(c, wl.prec, wl.k, wl.n_tau, lm, True, rel=1e-4, order=4)
        for p in range(6):
            ref = float(np.sum(gC0[i] * Jo[p]))
            scale = float(np.sum(np.abs(gC0[i] * Jo[p])))
            _say("autograd theta cosmology", i, "param", AG.PARAMS[p], g[i, p], ref)
            assert abs(g[i, p] - ref) <= 1e-4 * scale, (i, p)


def test_batch_consistency_errors(ctx):
    """An empty batch, and batches whose cosmologies differ in n_k, n_tau or
    the hierarchy, are CMB_E_INVALID at every batched entry point of the path
    (K1, K2, K3 and the whole solve), and nothing is written: the outputs keep
    their sentinels."""
    import torch
    import paper_2602_15104_amd as L
    wl = W.small_case(n_k=8, n_tau=40, ell_max=20)
    a = L.Tables(wl.cosmo, wl.prec, wl.k, 40)
    other_k = L.Tables(wl.cosmo, wl.prec, wl.k[:7], 40)
    other_tau = L.Tables(wl.cosmo, wl.prec, wl.k, 41)
    pr = dict(wl.prec)
    pr["ell_gamma"] += 1
    other_h = L.Tables(wl.cosmo, pr, wl.k, 40)
    dev = "cuda:0"
    S = torch.full((2, 8, 3, 41), float("nan"), dtype=torch.float64, device=dev)
    st = torch.full((2, 8), -7, dtype=torch.int32, device=dev)
    D = torch.full((2, 2, 8, 19), float("nan"), dtype=torch.float64, device=dev)
    C = torch.full((2, 3, 21), float("nan"), dtype=torch.float64, device=dev)
    for tabs in ([], [a, other_k], [a, other_tau], [a, other_h]):
        calls = (lambda: ctx.perturb(tabs, S, st), lambda: ctx.los(tabs, 20, S, D),
                 lambda: ctx.cl(tabs, 20, D, C), lambda: ctx.solve(tabs, 20, C, st, S=S, Delta=D))
        for call in calls:
            with pytest.raises(L.CmbError) as e:
                call()
            assert e.value.name == "CMB_E_INVALID", (len(tabs), e.value)
    torch.cuda.synchronize()
    assert torch.isnan(S).all() and torch.isnan(D).all() and torch.isnan(C).all()
    assert (st == -7).all()


def test_new_entry_points_reject_bad_arguments(ctx):
    """Argument errors of the lensing, derivative and variant entry points
    come back as CmbError (CMB_E_INVALID) without touching the device."""
    import torch
    import paper_2602_15104_amd as L
    wl = W.small_case(n_k=8, n_tau=40, ell_max=20)
    tab = L.Tables(wl.cosmo, wl.prec, wl.k, wl.n_tau)
    dev = "cuda:0"
    Cl = torch.zeros((1, 3, 101), dtype=torch.float64, device=dev)
    P = torch.zeros((1, 101), dtype=torch.float64, device=dev)
    out = torch.zeros((1, 4, 101), dtype=torch.float64, device=dev)
    with pytest.raises(L.CmbError):
        ctx.lensed_cl(Cl, P, 101, out, n_mu=200)  # ell_max above L
    with pytest.raises(L.CmbError):
        ctx.lensed_cl(Cl, P, 50, out, n_mu=1)  # too few nodes
    J = torch.zeros((1, 6, 3, 21), dtype=torch.float64, device=dev)
    C = torch.zeros((1, 3, 21), dtype=torch.float64, device=dev)
    st = torch.zeros((1, 8), dtype=torch.int32, device=dev)
    for rel, order in ((0.0, 4), (0.5, 4), (1e-4, 3)):
        with pytest.raises(L.CmbError):
            ctx.jacobian([tab], 20, C, J, st, rel=rel, order=order)
    c_z = dict(wl.cosmo)
    c_z["tau_reio"] = float("nan")
    c_z["z_reio"] = 8.0
    tz = L.Tables(c_z, wl.prec, wl.k, wl.n_tau)
    with pytest.raises(L.CmbError):
        ctx.jacobian([tz], 20, C, J, st)  # derivatives need tau_reio
    S = torch.zeros((1, 8, 3, 40), dtype=torch.float64, device=dev)
    H = torch.zeros((1, 8, 10), dtype=torch.float64, device=dev)  # capacity below max_steps + 1
    with pytest.raises(L.CmbError):
        ctx.perturb_record([tab], S, st, H, st)
    with pytest.raises(L.CmbError):
        ctx.lensing_potential([tab], 1, torch.zeros((1, 8, 40), dtype=torch.float64, device=dev), P)
    with pytest.raises(L.CmbError):
        ctx.bessel3_table(0)
    gY = torch.zeros((1, 8, 40, tab.state_rows()), dtype=torch.float64, device=dev)
    with pytest.raises(L.CmbError) as e:
        ctx.sources_adjoint([tab], None, gY)  # dL/dS missing
    assert e.value.name == "CMB_E_INVALID"
    with pytest.raises(L.CmbError):
        ctx.sources_adjoint([tab], S, None)
    cap = wl.prec["max_steps"] + 1
    Hf = torch.zeros((1, 8, cap), dtype=torch.float64, device=dev)
    Hn = torch.zeros((1, 8), dtype=torch.int32, device=dev)
    rows = tab.state_rows()
    few = torch.zeros((1, 8, 2, 1 + 2 * rows), dtype=torch.float64, device=dev)  # too few checkpoint slots
    ck = torch.zeros((1, 8, (cap - 1) // 64 + 1, 1 + 2 * rows), dtype=torch.float64, device=dev)
    for every, buf in ((0, ck), (64, few)):
        with pytest.raises(L.CmbError) as e:
            ctx.perturb_checkpoint([tab], Hf, Hn, every, buf, S, st)
        assert e.value.name == "CMB_E_INVALID"
    for seg in (-1, ck.shape[-2]):
        with pytest.raises(L.CmbError) as e:
            ctx.perturb_segment([tab], Hf, Hn, 64, ck, seg, S, st)
        assert e.value.name == "CMB_E_INVALID"
    roomy = torch.zeros((1, 8, 1000, 1 + 2 * rows), dtype=torch.float64, device=dev)
    for every, seg in ((64, cap // 64 + 1), (1 << 30, 4)):  # past the history; past int range
        with pytest.raises(L.CmbError) as e:
            ctx.perturb_segment([tab], Hf, Hn, every, roomy, seg, S, st)
        assert e.value.name == "CMB_E_INVALID"


@pytest.mark.parametrize("which", ["config0", "config1_subset"])
def test_tight_tolerance_cross_check(ctx, which):
    """Both sides at rtol 1e-10 (each atol scaled alike), each with its own
    adaptive steps (no matched discretisation): config 0 in full, and config
    1's physics on eight of its modes (both tolerance ranges, k up to 0.5).
    Sources to 1e-8 and C_ell to 1e-6 of the oracle's, so the agreement at the
    paper's tolerances is not an artifact of the two sides sharing a step
    sequence.  The oracle side is stored by tests/golden/make_oracle_reference.py."""
    import paper_2602_15104_amd as L
    ref = os.path.join(GOLD, f"oracle_tight_{which}.npz")
    assert os.path.exists(ref), "oracle golden missing: run tests/golden/make_oracle_reference.py tight_config0 tight_config1"
    wl = W.tight(W.config0() if which == "config0" else W.config1_subset())
    z = np.load(ref)
    assert np.array_equal(z["k"], wl.k)
    _say("case tight", wl.name, "oracle steps", int(z["nsteps"].min()), "..", int(z["nsteps"].max()))
    tab = L.Tables(wl.cosmo, wl.prec, wl.k, wl.n_tau)
    g = run_gpu(ctx, [tab], wl.ell_max)
    assert np.all(g["status"] == 0), g["status"]
    e = src_err(g["S"][0], z["S"])
    tt, te, ee = cl_err(g["Cl"][0], z["Cl"])
    # the method's own discretisation error, for scale: the oracle at the
    # paper's tolerances against itself at 1e-10
    e_disc = src_err(z["S_paper"], z["S"])
    _say("source err", e, "cl err", tt, te, ee, "gpu steps", int(g["nsteps"].min()), "..", int(g["nsteps"].max()),
         "| oracle paper-tolerance vs tight", e_disc, cl_err(z["Cl_paper"], z["Cl"]))
    assert e <= 1e-8
    assert tt <= 1e-6 and te <= 1e-6 and ee <= 1e-6


def test_context_budget_failure_and_stream_change():
    """The context after a failed call, and across streams.  A batch whose
    tables exceed the context's budget fails with CMB_E_NOMEM; the previous
    batch then runs again with the same bits (its tables are uploaded again,
    not taken from a stale cache).  Calls on a second stream that change the
    resident tables are ordered after the first stream's work: the results
    equal those of one stream."""
    import torch
    import paper_2602_15104_amd as L
    _need_gpu()
    wl = W.small_case(n_k=6, n_tau=60, ell_max=30)
    cos = W.perturbed_cosmologies(9, seed=3)
    for c in cos:
        c["N_nu_massless"] = 3.0
    tabs = [L.Tables(c, wl.prec, wl.k, wl.n_tau) for c in cos]
    big = L.Context(0)
    ref = run_gpu(big, tabs, wl.ell_max)
    one = run_gpu(big, tabs[:1], wl.ell_max)
    big.close()
    # tables of one cosmology take 8 * 16 * n_tab bytes (1 MiB at 8192 intervals)
    small = L.Context(0, hbm_budget_bytes=3 << 20)
    try:
        a = run_gpu(small, tabs[:1], wl.ell_max)
        with pytest.raises(L.CmbError) as ex:
            run_gpu(small, tabs, wl.ell_max)
        assert ex.value.name == "CMB_E_NOMEM"
        b = run_gpu(small, tabs[:1], wl.ell_max)
        for key in ("S", "Cl", "status", "nsteps"):
            assert np.array_equal(a[key], one[key]) and np.array_equal(b[key], one[key]), key
    finally:
        small.close()
    ctx = L.Context(0)
    try:
        s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
        outs = []
        for i, tb in enumerate(tabs):
            st = s1 if i % 2 == 0 else s2
            with torch.cuda.stream(st):
                outs.append(L.solve_batch(ctx, [tb], wl.ell_max, stream=st.cuda_stream))
        torch.cuda.synchronize()
        for i, o in enumerate(outs):
            assert np.array_equal(o["Cl"][0].cpu().numpy(), ref["Cl"][i]), i
            assert np.array_equal(o["S"][0].cpu().numpy(), ref["S"][i]), i
    finally:
        ctx.close()
