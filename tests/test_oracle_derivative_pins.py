"""Pin of the oracle's parameter derivatives by two independent
constructions.  CPU only.

The derivatives dC_l/dtheta that the adjoint is checked against come from
the oracle's frozen-step differences (`oracle.jacobian`): whole solves at
theta (1 +- rel) and (1 +- 2 rel) that replay the base solve's accepted steps,
combined by the five-point rule.  Forward mode (section 3 of the paper, whose
default derivative option it is) builds the same derivative another way:
the tangent of the discrete map is carried through every ESDIRK stage
exactly, (I - h gamma A_s) Ydot_s = Rdot_s + h gamma Adot_s Y_s, and only the
tables' own dependence on theta at a fixed state (the right-hand side, the
initial state, the sources, the projection) is differenced
(`oracle.jacobian_tangent`).  Both must give the same numbers up to the
five-point rule's truncation and rounding; a dropped or mis-signed term in
either (the Adot Y term of a stage, the tangent of K_0, the sources' own
table dependence, the projection's) breaks the agreement by orders of
magnitude more than the bar.
"""
import os

import numpy as np

import cmb_workloads as W
import oracle as O


def _case():
    return W.small_case(n_k=6, n_tau=80, ell_max=40)


def test_forward_mode_matches_frozen_step_differences():
    wl = _case()
    a = (wl.cosmo, wl.prec, wl.k, wl.n_tau, wl.ell_max, wl.polarization)
    C_fd, J_fd, st_fd = O.jacobian(*a, rel=1e-4, order=4)
    C_fw, J_fw, st_fw = O.jacobian_tangent(*a, rel=1e-4, order=4)
    assert np.all(st_fd == 0) and np.all(st_fw == 0)
    # the primal is the same solve, bit for bit
    assert np.array_equal(C_fd, C_fw)
    for p in (0, 1, 2, 5):  # h, omega_b, omega_cdm, tau_reio
        for x in range(3):  # TT, TE, EE
            ref = J_fd[p, x, 2:]
            scale = np.max(np.abs(ref))
            assert scale > 0.0
            err = np.max(np.abs(J_fw[p, x, 2:] - ref)) / scale
            # measured <= 2e-9 on this case (central table differences instead
            # of five-point ones give up to 5e-6)
            assert err <= 1e-7, (p, x, err)
    # ln A_s and n_s are the same closed forms in both
    assert np.array_equal(J_fd[3], J_fw[3]) and np.array_equal(J_fd[4], J_fw[4])


def test_forward_mode_sources_are_the_replayed_sources():
    """The tangent integration's primal sources equal the frozen-step replay's
    bit for bit (the same stages in the same order), and a zero parameter
    step of the tables (every table equal to the base) gives zero tangents."""
    wl = _case()
    t = O.build_tables(wl.cosmo, wl.prec, wl.k, wl.n_tau)
    S0, st, ns, hist, hn = O.perturb_hist(t)
    S_rep = O.perturb_hist(t, hist, hn)[0]
    S, Sd, st2 = O.perturb_tangent(t, [[t, t, t, t]], [1e-4], hist, hn, order=4)
    assert np.all(st2 == 0)
    assert np.array_equal(S, S_rep)
    assert np.all(Sd == 0.0)


def test_full_size_derivative_goldens_agree():
    """At config 1 in full (400 modes, 2000 output times, l <= 2500) the two
    stored derivative sets (tests/golden/make_oracle_reference.py
    config1_jacobian, config1_tangent) agree; measured <= 5.5e-8 of the
    largest value per parameter and spectrum."""
    gold = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    fd = np.load(os.path.join(gold, "oracle_config1_jacobian.npy"))
    fw = np.load(os.path.join(gold, "oracle_config1_tangent.npy"))
    assert fd.shape == fw.shape == (6, 3, 2501)
    for p in range(6):
        for x in range(3):
            scale = np.max(np.abs(fd[p, x, 2:]))
            assert scale > 0.0
            err = np.max(np.abs(fw[p, x, 2:] - fd[p, x, 2:])) / scale
            assert err <= 1e-6, (p, x, err)
