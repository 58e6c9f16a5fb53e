"""GPU: cmb_gradient, the discrete adjoint of the whole path (reverse ESDIRK
sweep over checkpointed segments, transposed dense output and sources, table
tangents by central differences), against the oracle.

  dL/dtheta   against the oracle's frozen-step five-point derivatives (rel
              1e-4) contracted with the same dL/dC_l: per parameter within
              1e-4 of sum |dL/dC_l| |dC_l/dtheta_p|; at config 1 also against
              the oracle's forward-mode tangents;
  dL/dy0      dot products with seeded directions: L is quadratic in the
              sources and the sources are linear in a mode's start state at
              fixed steps, so the oracle's central difference of L along a
              direction of y0 is exact up to rounding.
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


def _case(name):
    """"few": two cosmologies, 16 modes to k = 0.1, 150 output times, l <= 120
    (49..1157 steps a mode: one to nineteen 64-step segments); "many": one
    cosmology, 12 modes to k = 0.03 at rtol 1e-7 (140..2527 steps: three to
    forty segments)."""
    if name == "few":
        wl = W.small_case(n_k=16, n_tau=150, ell_max=120, k_max=0.1)
        cosmos = W.perturbed_cosmologies(2, seed=21)
    else:
        wl = W.tight(W.small_case(n_k=12, n_tau=150, ell_max=120, k_max=0.03), rtol=1e-7, max_steps=4096)
        cosmos = W.perturbed_cosmologies(1, seed=21)
    for cc in cosmos:
        cc["N_nu_massless"] = 3.0
    return wl, cosmos


def _gradient(ctx, tabs, lm, gC, with_y0=False):
    import torch
    import paper_2602_15104_amd as L
    n, n_k = len(tabs), len(tabs[0].k)
    dg = torch.tensor(gC, dtype=torch.float64, device="cuda:0")
    Cl = torch.empty((n, 3, lm + 1), dtype=torch.float64, device="cuda:0")
    grad = torch.full((n, 6), float("nan"), dtype=torch.float64, device="cuda:0")
    st = torch.full((n, n_k), -7, dtype=torch.int32, device="cuda:0")
    y0 = None
    if with_y0:
        N = tabs[0].state_rows()
        y0 = torch.full((n, n_k, N), float("nan"), dtype=torch.float64, device="cuda:0")
    ctx.gradient(tabs, lm, dg, Cl, grad, st, rel=1e-4, dLdy0=y0)
    torch.cuda.synchronize()
    return (Cl.cpu().numpy(), grad.cpu().numpy(), st.cpu().numpy(), None if y0 is None else y0.cpu().numpy())


def _seeded_gC(n, lm, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    g = rng.standard_normal((n, 3, lm + 1))
    g[:, :, :2] = 0.0
    return g


@pytest.mark.parametrize("case", ["few", "many"])
def test_gradient_matches_oracle_differences(ctx, case):
    """C_l equals cmb_solve's; dL/dtheta against the oracle's frozen-step
    derivatives contracted with seeded dL/dC_l, every parameter."""
    import torch
    import oracle as O
    import paper_2602_15104_amd as L
    wl, cosmos = _case(case)
    lm = wl.ell_max
    tabs = [L.Tables(c, wl.prec, wl.k, wl.n_tau) for c in cosmos]
    gC = _seeded_gC(len(cosmos), lm, 47)
    _say("gradient", case, ":", len(cosmos), "cosmologies,", len(wl.k), "modes, l <=", lm)
    Cl, g, st, _ = _gradient(ctx, tabs, lm, gC)
    assert np.all(st == 0), st
    out = L.solve_batch(ctx, tabs, lm, keep_S=False, keep_Delta=False)
    torch.cuda.synchronize()
    assert np.array_equal(Cl, out["Cl"].cpu().numpy())
    for i, c in enumerate(cosmos):
        _, Jo, sto = O.jacobian(c, wl.prec, wl.k, wl.n_tau, lm, True, rel=1e-4, order=4)
        assert np.all(sto == 0)
        for p in range(6):
            ref = float(np.sum(gC[i] * Jo[p]))
            scale = float(np.sum(np.abs(gC[i] * Jo[p])))
            e = abs(g[i, p] - ref) / scale
            _say("gradient cosmology", i, "param", p, "adjoint", g[i, p], "oracle", ref, "err", e)
            assert e <= 1e-4, (i, p, e)


def test_gradient_start_state_dot_products(ctx):
    """dL/dy0 of three modes (low, middle, high k; 3, 16 and 40 segments) of
    one cosmology: against the oracle's central difference of L along a
    seeded direction of each mode's start state, with the oracle's own
    recorded steps."""
    import oracle as O
    import paper_2602_15104_amd as L
    wl, cosmos = _case("many")
    lm = wl.ell_max
    c = cosmos[0]
    tab = L.Tables(c, wl.prec, wl.k, wl.n_tau)
    gC = _seeded_gC(1, lm, 53)
    _say("gradient start-state dot products: 1 cosmology, 12 modes")
    _, _, st, y0g = _gradient(ctx, [tab], lm, gC, with_y0=True)
    assert np.all(st == 0)
    t = O.build_tables(c, wl.prec, wl.k, wl.n_tau)
    S, sto, _, hist, hn = O.perturb_hist(t)
    assert np.all(sto == 0)
    order = O.library_row_order(wl.prec, 0)

    def L_of(Sx):
        DT, DE = O.los(t, Sx, lm, True)
        C = O.cl(t.k, DT, DE, lm, True, c["A_s"], c["n_s"], wl.prec["k_pivot"])
        return float(np.sum(gC[0] * C))

    rng = np.random.Generator(np.random.PCG64(59))
    for ik in (0, 8, 11):
        k, lna0 = float(t.k[ik]), float(t.lna_i[ik])
        fixed = hist[ik, : hn[ik] + 1]
        y_start = O.perturb_one(t, k, lna0, [fixed[0]], want_y=True, fixed=fixed)["y"][0]
        N = len(y_start)
        v = rng.standard_normal(N) * np.max(np.abs(y_start))
        Sp, Sm = S.copy(), S.copy()
        Sp[ik] = O.perturb_one(t, k, lna0, t.lna_src, y0=y_start + v, fixed=fixed)["S"]
        Sm[ik] = O.perturb_one(t, k, lna0, t.lna_src, y0=y_start - v, fixed=fixed)["S"]
        ref = (L_of(Sp) - L_of(Sm)) / 2.0
        got = float(np.dot(y0g[0, ik], v[order]))
        scale = float(np.sum(np.abs(y0g[0, ik] * v[order])))
        e = abs(got - ref) / scale
        _say("dL/dy0 mode", ik, "adjoint", got, "oracle difference", ref, "err", e)
        assert e <= 1e-6, (ik, e)


@pytest.mark.parametrize("case", ["few", "config1"])
def test_gradient_matches_frozen_step_central_differences(ctx, case):
    """Against the library's own frozen-step central differences
    (cmb_jacobian, order 2, rel 1e-4), which replay the very steps the
    adjoint differentiates: the adjoint's table tangents are the same
    central differences, so the two agree far below their O(rel^2)
    truncation, within 1e-6 of sum |dL/dC_l dC_l/dtheta_p| (measured
    2.5e-7 at worst).  Against the five-point stencil they differ by that
    truncation (up to 1.1e-5), which is why the oracle comparison's bar is
    1e-4."""
    import torch
    import paper_2602_15104_amd as L
    if case == "few":
        wl, cosmos = _case("few")
    else:
        wl = W.config1()
        cosmos = [wl.cosmo]
    lm = wl.ell_max
    tabs = [L.Tables(c, wl.prec, wl.k, wl.n_tau) for c in cosmos]
    n = len(tabs)
    gC = _seeded_gC(n, lm, 47 if case == "few" else 61)
    _say("gradient vs central differences:", case)
    _, g, st, _ = _gradient(ctx, tabs, lm, gC)
    assert np.all(st == 0)
    C = torch.empty((n, 3, lm + 1), dtype=torch.float64, device="cuda:0")
    J = torch.empty((n, 6, 3, lm + 1), dtype=torch.float64, device="cuda:0")
    sj = torch.empty((n, len(wl.k)), dtype=torch.int32, device="cuda:0")
    ctx.jacobian(tabs, lm, C, J, sj, rel=1e-4, order=2)
    torch.cuda.synchronize()
    assert np.all(sj.cpu().numpy() == 0)
    Jn = J.cpu().numpy()
    for i in range(n):
        for p in range(6):
            ref = float(np.sum(gC[i] * Jn[i, p]))
            scale = float(np.sum(np.abs(gC[i] * Jn[i, p])))
            e = abs(g[i, p] - ref) / scale
            _say("central", case, "cosmology", i, "param", p, "err", e)
            assert e <= 1e-6, (i, p, e)


def test_gradient_config1(ctx):
    """Config 1 (400 modes, 2000 output times, l <= 2500), fiducial cosmology:
    dL/dtheta for seeded dL/dC_l against the stored oracle derivatives
    (tests/golden/make_oracle_reference.py) contracted with it: the
    frozen-step five-point differences and the forward-mode tangents."""
    import paper_2602_15104_amd as L
    ref = os.path.join(GOLD, "oracle_config1_jacobian.npy")
    assert os.path.exists(ref), "oracle golden missing: run tests/golden/make_oracle_reference.py"
    wl = W.config1()
    lm = wl.ell_max
    tab = L.Tables(wl.cosmo, wl.prec, wl.k, wl.n_tau)
    gC = _seeded_gC(1, lm, 61)
    _say("gradient config1: 400 modes, 2000 times, l <= 2500")
    _, g, st, _ = _gradient(ctx, [tab], lm, gC)
    assert np.all(st == 0)
    ref_fw = os.path.join(GOLD, "oracle_config1_tangent.npy")
    assert os.path.exists(ref_fw), "oracle golden missing: run tests/golden/make_oracle_reference.py config1_tangent"
    for what, path in (("frozen-step differences", ref), ("forward mode", ref_fw)):
        Jo = np.load(path)
        for p in range(6):
            r = float(np.sum(gC[0] * Jo[p]))
            scale = float(np.sum(np.abs(gC[0] * Jo[p])))
            e = abs(g[0, p] - r) / scale
            _say("config1 gradient param", p, "adjoint", g[0, p], "oracle", what, r, "err", e)
            assert e <= 1e-4, (what, p, e)


def test_gradient_refusals(ctx):
    """Massive neutrinos are CMB_E_UNSUPPORTED; a cosmology given by z_reio,
    rel outside (0, 0.01] and ell_max < 2 are CMB_E_INVALID; the outputs keep
    their sentinels."""
    import torch
    import paper_2602_15104_amd as L
    wl = W.small_case(n_k=8, n_tau=60, ell_max=40)
    lm = wl.ell_max
    ok = L.Tables(wl.cosmo, wl.prec, wl.k, wl.n_tau)
    c2 = W.config2()
    heavy = L.Tables(c2.cosmo, c2.prec, wl.k, wl.n_tau)
    cz = dict(wl.cosmo)
    cz["tau_reio"] = float("nan")
    cz["z_reio"] = 8.0
    zre = L.Tables(cz, wl.prec, wl.k, wl.n_tau)
    gC = torch.zeros((1, 3, lm + 1), dtype=torch.float64, device="cuda:0")
    Cl = torch.full((1, 3, lm + 1), 7.0, dtype=torch.float64, device="cuda:0")
    grad = torch.full((1, 6), 7.0, dtype=torch.float64, device="cuda:0")
    st = torch.full((1, 8), 7, dtype=torch.int32, device="cuda:0")
    for tabs, rel, lmx, name in (([heavy], 1e-4, lm, "CMB_E_UNSUPPORTED"), ([zre], 1e-4, lm, "CMB_E_INVALID"),
                                 ([ok], 0.0, lm, "CMB_E_INVALID"), ([ok], 0.02, lm, "CMB_E_INVALID"),
                                 ([ok], 1e-4, 1, "CMB_E_INVALID")):
        with pytest.raises(L.CmbError) as e:
            ctx.gradient(tabs, lmx, gC, Cl, grad, st, rel=rel)
        assert e.value.name == name, (name, e.value.name)
    torch.cuda.synchronize()
    assert torch.all(Cl == 7.0) and torch.all(grad == 7.0) and torch.all(st == 7)
