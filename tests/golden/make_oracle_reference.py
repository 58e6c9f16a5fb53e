"""Write the oracle spectra used by the GPU parity tests at full size.

    python tests/golden/make_oracle_reference.py [config1] [config2] [config1_transfer] [config1_jacobian]
                                                 [config1_tangent] [tight_config0] [tight_config1]

Calls only the CPU oracle (package ``oracle``) and the seeded workload
generator; re-run it whenever the oracle's arithmetic changes.  Outputs, for
the fiducial cosmology of each workload, C_ell[3][2501] (TT, TE, EE):
  tests/golden/oracle_config1_cl.npy  400 modes, 2000 output times, l <= 2500
  tests/golden/oracle_config2_cl.npy  the same with one massive neutrino
                                      (12 momentum nodes, l_ncdm = 17), 600 modes
plus, for config 2, the per-mode step counts (oracle_config2_nsteps.npy), and
  tests/golden/oracle_config1_transfer_cl.npy  config 1's sources interpolated
                                      onto the App. A.2 transfer grid for
                                      l_max = 2500, projected and integrated there
  tests/golden/oracle_config1_jacobian.npy  dC_l/d(h, omega_b, omega_cdm, ln A_s,
                                      n_s, tau_reio) [6][3][2501] for config 1
                                      (five-point stencil, rel 1e-4, frozen steps)
  tests/golden/oracle_config1_tangent.npy  the same derivatives by forward mode:
                                      tangents carried through the frozen-step
                                      stages, five-point differences of the
                                      table-dependent quantities only
  tests/golden/oracle_tight_config0.npz, oracle_tight_config1_subset.npz
                                      the tight-tolerance cross-check: config 0
                                      in full and config 1 on eight of its modes,
                                      both at rtol 1e-10 (atol scaled alike):
                                      S, Cl, nsteps, and the same at the paper's
                                      tolerances for the discretisation report
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import cmb_workloads as W  # noqa: E402
import oracle as O  # noqa: E402


def tight(name):
    wl = W.config0() if name == "config0" else W.config1_subset()
    wt = W.tight(wl)
    t0 = time.time()
    r = O.solve(wt.cosmo, wt.prec, wt.k, wt.n_tau, wt.ell_max, wt.polarization)
    assert np.all(r["status"] == 0)
    p = O.solve(wl.cosmo, wl.prec, wl.k, wl.n_tau, wl.ell_max, wl.polarization)
    assert np.all(p["status"] == 0)
    out = os.path.join(HERE, f"oracle_tight_{'config1_subset' if name != 'config0' else name}.npz")
    np.savez_compressed(out, k=wt.k, S=r["S"], Cl=r["Cl"], nsteps=np.asarray(r["nsteps"], dtype=np.int32),
                        S_paper=p["S"], Cl_paper=p["Cl"])
    print(f"wrote {os.path.basename(out)} in {time.time() - t0:.1f} s; steps {np.min(r['nsteps'])}.."
          f"{np.max(r['nsteps'])} (paper tolerances {np.max(p['nsteps'])})", flush=True)


def main(which):
    for name in which:
        if name.startswith("tight_"):
            tight(name[len("tight_"):])
            continue
        if name.endswith("_tangent"):
            wl = getattr(W, name.replace("_tangent", ""))()
            t0 = time.time()
            C, J, st = O.jacobian_tangent(wl.cosmo, wl.prec, wl.k, wl.n_tau, wl.ell_max, True, rel=1e-4, order=4)
            assert np.all(st == 0)
            np.save(os.path.join(HERE, f"oracle_{name}.npy"), J)
            print(f"wrote oracle_{name}.npy in {time.time() - t0:.1f} s", flush=True)
            continue
        if name.endswith("_jacobian"):
            wl = getattr(W, name.replace("_jacobian", ""))()
            t0 = time.time()
            C, J, st = O.jacobian(wl.cosmo, wl.prec, wl.k, wl.n_tau, wl.ell_max, True, rel=1e-4, order=4)
            assert np.all(st == 0)
            np.save(os.path.join(HERE, f"oracle_{name}.npy"), J)
            print(f"wrote oracle_{name}.npy in {time.time() - t0:.1f} s", flush=True)
            continue
        transfer = name.endswith("_transfer")
        wl = getattr(W, name.replace("_transfer", ""))()
        t0 = time.time()
        r = O.solve(wl.cosmo, wl.prec, wl.k, wl.n_tau, wl.ell_max, True)
        assert np.all(r["status"] == 0)
        if transfer:
            kt = O.transfer_kgrid(wl.ell_max, wl.k[0], wl.k[-1])
            r = O.spectra_on_grid(r["tables"], r["S"], kt, wl.ell_max, True)
            np.save(os.path.join(HERE, f"oracle_{name}_cl.npy"), r["Cl"])
            print(f"wrote oracle_{name}_cl.npy ({len(kt)} points) in {time.time() - t0:.1f} s", flush=True)
            continue
        np.save(os.path.join(HERE, f"oracle_{name}_cl.npy"), r["Cl"])
        if name == "config2":
            np.save(os.path.join(HERE, f"oracle_{name}_nsteps.npy"), np.asarray(r["nsteps"], dtype=np.int32))
        print(f"wrote oracle_{name}_cl.npy in {time.time() - t0:.1f} s; mean steps {r['nsteps'].mean():.1f}",
              flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["config1", "config2"])
