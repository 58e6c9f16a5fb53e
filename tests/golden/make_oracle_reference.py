"""Write the oracle spectra used by the GPU parity tests at full size.

    python tests/golden/make_oracle_reference.py [config1] [config2] [config1_transfer]

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
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import cmb_workloads as W  # noqa: E402
import oracle as O  # noqa: E402


def main(which):
    for name in which:
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
